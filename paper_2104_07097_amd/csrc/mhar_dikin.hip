// mhar_dikin.hip -- direction covariance fitted to the Dikin ellipsoid (FP64).
//
// Burn-in fit of Sigma = U U^T + diag(exp(2 l)) to the Dikin ellipsoid of
// the polytope at the mean walk state xbar: H = sum_i a_i a_i^T / s_i^2 with
// s = b - A xbar, the Hessian of the log-barrier -sum_i log(b_i - a_i x)
// (its unit ellipsoid at xbar lies inside the polytope).  The objective
//     K(Sigma) = 1/2 tr(H Sigma) - 1/2 log det Sigma
// is the Kullback-Leibler divergence of N(0, Sigma) from N(0, H^{-1}) up to
// a constant.  One training step:
//   1. xbar, s, H = A^T diag(1/s^2) A on the FP64 matrix cores (N x N with
//      N = n rounded up to 64, identity on the padding);
//   2. k power iterations on J = diag(H)^{-1/2} H diag(H)^{-1/2} from the
//      stored unit vector v, lam = v^T J v (lambda_max(J) from below);
//   3. l_i = log(kappa) - 1/2 log(lam H_ii): at kappa = 1, D = diag(exp(2 l))
//      has D^{1/2} H D^{1/2} = J / lam, the largest Gaussian of the Jacobi
//      shape inside the Dikin ellipsoid (up to the estimate of lam); the
//      complement scale kappa in (0, 1] shrinks it;
//   4. dK/dU = H U - Sigma^{-1} U = H U - W C^{-1}, W = D^{-1} U,
//      C = I + U^T W (Woodbury);
//   5. U <- U - eta H^{-1} dK/dU through a blocked Cholesky factor of H.
// The walk states themselves cannot reveal the long axes of an elongated
// body before the walks have explored them; the slacks of all rows at the
// mean state do, through H.
#include <math.h>

#include "mhar_device.hpp"
#include "mhar_internal.hpp"

namespace mhar {

namespace {

constexpr int kNB = 64;   // block size of H and of its Cholesky factor

// s_i = b_i - a_i xbar and w_i = 1 / s_i^2 (0 on padding rows): one wave per row
__global__ __launch_bounds__(256) void dikin_weights_kernel(int n, int m, int m_pad, int lda,
                                                            const double* __restrict__ A64,
                                                            const double* __restrict__ b64,
                                                            const double* __restrict__ xbar,
                                                            double* w, int* status)
{
    const int lane = threadIdx.x & 63;
    const int i = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (i >= m_pad) return;
    const double* ar = A64 + (size_t)i * lda;
    double v = 0.0;
    for (int j = lane; j < n; j += 64) v = fma(ar[j], xbar[j], v);
    v = wave_sum(v);
    if (lane == 0) {
        const double s = b64[i] - v;
        if (i < m) {
            w[i] = 1.0 / (s * s);
            if (!(s > 0.0)) atomicOr(status, 2);
        } else {
            w[i] = 0.0;
        }
    }
}

// H = A^T diag(w) A, one 64 x 64 output tile per workgroup of 8 waves; each
// wave sums a contiguous eighth of the rows of A into all 16 MFMA tiles of
// the output tile, and the eight partial tiles are added in wave order
// through LDS.  f64 16x16x4 MFMA: lane (g, c) supplies a = w_k A[k][p0 + c]
// and b = A[k][q0 + c] for row k = k0 + g; out[r] = C[4 r + g][c].
// Padding columns (index >= n) and the padding diagonal get the identity.
__global__ __launch_bounds__(512) void dikin_hessian_kernel(int n, int N, int m_pad, int lda,
                                                            const double* __restrict__ A64,
                                                            const double* __restrict__ w,
                                                            double* H)
{
    __shared__ double acc_lds[kNB * kNB];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int g = lane >> 4, c = lane & 15;
    const int p0 = blockIdx.y * kNB, q0 = blockIdx.x * kNB;
    const int per = (m_pad / 4 + 7) / 8 * 4;     // rows per wave, a multiple of 4
    const int k_begin = wave * per, k_end = min(m_pad, k_begin + per);
    f64x4 acc[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = f64x4{0, 0, 0, 0};
    bool pok[4], qok[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        pok[t] = p0 + 16 * t + c < lda;
        qok[t] = q0 + 16 * t + c < lda;
    }
    for (int k0 = k_begin; k0 < k_end; k0 += 4) {
        const int k = k0 + g;
        const double* ar = A64 + (size_t)k * lda;
        const double wk = w[k];
        double av[4], bv[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            av[t] = pok[t] ? wk * ar[p0 + 16 * t + c] : 0.0;
            bv[t] = qok[t] ? ar[q0 + 16 * t + c] : 0.0;
        }
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int b = 0; b < 4; ++b) acc[a][b] = mma_f64(av[a], bv[b], acc[a][b]);
    }
    for (int turn = 0; turn < 8; ++turn) {
        if (wave == turn) {
#pragma unroll
            for (int a = 0; a < 4; ++a)
#pragma unroll
                for (int b = 0; b < 4; ++b)
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const int e = (16 * a + out_row<true>(g, r)) * kNB + 16 * b + c;
                        acc_lds[e] = (turn == 0) ? acc[a][b][r] : acc_lds[e] + acc[a][b][r];
                    }
        }
        __syncthreads();
    }
    for (int e = threadIdx.x; e < kNB * kNB; e += 512) {
        const int p = p0 + e / kNB, q = q0 + e % kNB;
        double v = acc_lds[e];
        if (p >= n || q >= n) v = (p == q) ? 1.0 : 0.0;
        H[(size_t)p * N + q] = v;
    }
}

// dsq_i = sqrt(H_ii)
__global__ void dikin_diag_kernel(int N, const double* __restrict__ H, double* dsq)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < N) dsq[i] = sqrt(H[(size_t)i * N + i]);
}

// y_out = J (y_in / |y_in|) over the first n entries (scale = 0: y_in is
// used as it is); one wave per row.  When v is given, v = y_in / |y_in|.
__global__ __launch_bounds__(256) void dikin_power_kernel(int n, int N, const double* __restrict__ H,
                                                          const double* __restrict__ dsq,
                                                          const double* __restrict__ y_in,
                                                          int scale, double* y_out, double* v)
{
    const int lane = threadIdx.x & 63;
    const int i = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (i >= n) return;
    double nrm = 1.0;
    if (scale) {
        double q = 0.0;
        for (int j = lane; j < n; j += 64) q = fma(y_in[j], y_in[j], q);
        nrm = sqrt(wave_sum(q));
    }
    const double* hr = H + (size_t)i * N;
    const double di = dsq[i];
    double t = 0.0;
    for (int j = lane; j < n; j += 64) t = fma(hr[j] / (di * dsq[j]), y_in[j] / nrm, t);
    t = wave_sum(t);
    if (lane == 0) {
        y_out[i] = t;
        if (v) v[i] = y_in[i] / nrm;
    }
}

// lam = v^T y with y = J v (one workgroup); then l_i = -1/2 log(lam H_ii),
// unless a fit step has failed (the covariance then stays as it is)
__global__ __launch_bounds__(1024) void dikin_scales_kernel(int n, int N, const double* __restrict__ H,
                                                            const double* __restrict__ v,
                                                            const double* __restrict__ y,
                                                            const int* status, double log_kappa,
                                                            double* lam_out, double* logsig,
                                                            double* esig)
{
    __shared__ double part[16];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    double s = 0.0;
    for (int i = tid; i < n; i += 1024) s = fma(v[i], y[i], s);
    s = wave_sum(s);
    if (lane == 0) part[wave] = s;
    __syncthreads();
    double lam = 0.0;
    for (int k = 0; k < 16; ++k) lam += part[k];
    if (tid == 0) *lam_out = lam;
    if (*status) return;
    for (int i = tid; i < n; i += 1024) {
        const double l = log_kappa - 0.5 * log(lam * H[(size_t)i * N + i]);
        logsig[i] = l;
        esig[i] = exp(l);
    }
}

// C = I + U^T W (r x r, r <= 64) on the FP64 matrix cores, one workgroup
// of 8 waves: wave w sums a contiguous eighth of the coordinates into all
// 16 output tiles (f64 16x16x4: lane (g, c) supplies a = U[i0 + g][16 ta + c]
// and b = W[i0 + g][16 tb + c]), and the eight partial tiles are added in
// wave order through LDS.
__global__ __launch_bounds__(512) void dikin_cap_kernel(int n, int r, const double* __restrict__ U,
                                                        const double* __restrict__ W, double* C)
{
    __shared__ double acc_lds[64 * 64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int g = lane >> 4, c = lane & 15;
    const int per = ((n + 7) / 8 + 3) / 4 * 4;   // coordinates per wave, a multiple of 4
    const int i_begin = wave * per, i_end = min(n, i_begin + per);
    f64x4 acc[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = f64x4{0, 0, 0, 0};
    for (int i0 = i_begin; i0 < i_end; i0 += 4) {
        const int i = i0 + g;
        double av[4], bv[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const int q = 16 * t + c;
            const bool ok = i < i_end && q < r;
            av[t] = ok ? U[(size_t)i * r + q] : 0.0;
            bv[t] = ok ? W[(size_t)i * r + q] : 0.0;
        }
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int b = 0; b < 4; ++b) acc[a][b] = mma_f64(av[a], bv[b], acc[a][b]);
    }
    for (int turn = 0; turn < 8; ++turn) {
        if (wave == turn) {
#pragma unroll
            for (int a = 0; a < 4; ++a)
#pragma unroll
                for (int b = 0; b < 4; ++b)
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        const int e = (16 * a + out_row<true>(g, q)) * 64 + 16 * b + c;
                        acc_lds[e] = (turn == 0) ? acc[a][b][q] : acc_lds[e] + acc[a][b][q];
                    }
        }
        __syncthreads();
    }
    for (int e = threadIdx.x; e < r * r; e += 512) {
        const int a = e / r, b = e - a * r;
        C[e] = ((a == b) ? 1.0 : 0.0) + acc_lds[a * 64 + b];
    }
}

// HU = H U (n x r) on the FP64 matrix cores: one wave per 16 rows of H,
// the r <= 64 columns as 4 tiles
// of 16 (f64 16x16x4: lane (g, c) supplies a = H[row c][k0 + g] and
// b = U[k0 + g][16 t + c]); out[q] of tile t = row out_row(g, q).
__global__ __launch_bounds__(64) void dikin_hu_kernel(int n, int N, int r, const double* __restrict__ H,
                                                      const double* __restrict__ U, double* HU)
{
    const int lane = threadIdx.x;
    const int g = lane >> 4, c = lane & 15;
    const int row0 = blockIdx.x * 16;   // < N
    const double* hr = H + (size_t)(row0 + c) * N;
    f64x4 acc[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) acc[t] = f64x4{0, 0, 0, 0};
    for (int k0 = 0; k0 < n; k0 += 4) {
        const int k = k0 + g;
        const double av = k < n ? hr[k] : 0.0;
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const int q = 16 * t + c;
            acc[t] = mma_f64(av, (k < n && q < r) ? U[(size_t)k * r + q] : 0.0, acc[t]);
        }
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int row = row0 + out_row<true>(g, q);
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const int col = 16 * t + c;
            if (row < n && col < r) HU[(size_t)row * r + col] = acc[t][q];
        }
    }
}

// Per coordinate row i (one wave, lane = rank column), with HU = H U:
//   gU_i = HU_i - W_i C^{-1},
//   gl_i = exp(2 l_i) (H_ii - (Sigma^{-1})_ii),
//   (Sigma^{-1})_ii = exp(-2 l_i) - W_i C^{-1} W_i^T,
//   rowterm_i = 1/2 (H_ii exp(2 l_i) + U_i . HU_i) - l_i  (K = sum rowterm - 1/2 log det C)
__global__ __launch_bounds__(256) void dikin_grad_kernel(int n, int N, int r,
                                                         const double* __restrict__ H,
                                                         const double* __restrict__ HU,
                                                         const double* __restrict__ U,
                                                         const double* __restrict__ W,
                                                         const double* __restrict__ Cinv,
                                                         const double* __restrict__ logsig,
                                                         double* gU, double* gl, double* rowterm)
{
    const int q = threadIdx.x & 63;
    const int i = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (i >= n) return;
    const double* hr = H + (size_t)i * N;
    double hu = 0.0, wc = 0.0;
    if (q < r) {
        hu = HU[(size_t)i * r + q];
        for (int b = 0; b < r; ++b) wc = fma(W[(size_t)i * r + b], Cinv[b * r + q], wc);
        gU[(size_t)i * r + q] = hu - wc;
    }
    const double wi = (q < r) ? W[(size_t)i * r + q] : 0.0;
    const double uhu = wave_sum((q < r) ? U[(size_t)i * r + q] * hu : 0.0);
    const double wcw = wave_sum(wi * wc);
    if (q == 0) {
        const double l = logsig[i], d = exp(2.0 * l), hii = hr[i];
        const double sinv = exp(-2.0 * l) - wcw;
        gl[i] = d * (hii - sinv);
        rowterm[i] = 0.5 * (hii * d + uhu) - l;
    }
}

// K = sum_i rowterm_i - 1/2 log det C (one workgroup, fixed-shape tree)
__global__ __launch_bounds__(256) void dikin_value_kernel(int n, const double* rowterm,
                                                          const double* logdet, double* K)
{
    __shared__ double ps[256];
    const int tid = threadIdx.x;
    const int per = (n + 255) / 256;
    double s = 0.0;
    for (int i = tid * per; i < min(n, (tid + 1) * per); ++i) s += rowterm[i];
    ps[tid] = s;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (tid < h) ps[tid] += ps[tid + h];
        __syncthreads();
    }
    if (tid == 0) *K = ps[0] - 0.5 * (*logdet);
}

// ---- blocked Cholesky H = L L^T (lower, in place on L, N x N, N % 64 == 0) ----

// copy H into L
__global__ void dikin_copy_kernel(int64_t count, const double* __restrict__ src, double* dst)
{
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < count;
         e += (int64_t)gridDim.x * blockDim.x)
        dst[e] = src[e];
}

// factor the diagonal block kb (right-looking).  256 threads, thread
// (ty, tx) holding the 16 entries (ty + 16 a, tx + 16 b) of the block in
// registers; per column j the owners of column j publish it through LDS,
// every thread scales what it needs by the reciprocal of the pivot's root
// and updates its entries below the diagonal.  A pivot <= 0 sets status bit 1 and is
// replaced by 1 so that the rest stays finite.
__global__ __launch_bounds__(256) void chol_diag_kernel(int N, int kb, double* L, int* status)
{
    __shared__ double col[kNB];
    const int tid = threadIdx.x, ty = tid >> 4, tx = tid & 15;
    const size_t base = (size_t)kb * kNB * N + (size_t)kb * kNB;
    double t[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) t[a][b] = L[base + (size_t)(ty + 16 * a) * N + tx + 16 * b];
    for (int j = 0; j < kNB; ++j) {
        const int bj = j >> 4;
        if (tx == (j & 15)) {
#pragma unroll
            for (int a = 0; a < 4; ++a)
#pragma unroll
                for (int b = 0; b < 4; ++b)
                    if (b == bj) col[ty + 16 * a] = t[a][b];
        }
        __syncthreads();
        double piv = col[j];
        if (!(piv > 0.0)) {
            if (tid == 0) atomicOr(status, 1);
            piv = 1.0;
        }
        const double ljj = sqrt(piv), rj = 1.0 / ljj;
        double li[4], lk[4];
#pragma unroll
        for (int a = 0; a < 4; ++a) {
            const int i = ty + 16 * a;
            li[a] = i > j ? col[i] * rj : 0.0;
        }
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const int k = tx + 16 * b;
            lk[b] = k > j ? col[k] * rj : 0.0;
        }
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                const int i = ty + 16 * a, k = tx + 16 * b;
                if (k == j) {
                    if (i == j) t[a][b] = ljj;
                    else if (i > j) t[a][b] = li[a];
                } else if (k > j && k <= i) {
                    t[a][b] -= li[a] * lk[b];
                }
            }
        __syncthreads();
    }
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const int i = ty + 16 * a, k = tx + 16 * b;
            L[base + (size_t)i * N + k] = (k <= i) ? t[a][b] : 0.0;
        }
}

// panel below the diagonal block: L_ib = A_ib L_kk^{-T} by forward
// substitution, one workgroup per 64-row block ib > kb, four lanes per row:
// lane t of a quad keeps the row's columns k = t (mod 4) in registers, the
// dot product of column c is summed over the quad by shuffles, and the lane
// owning column c divides.
__global__ __launch_bounds__(256) void chol_panel_kernel(int N, int kb, double* L)
{
    __shared__ double D[kNB][kNB + 1];
    const int tid = threadIdx.x, row = tid >> 2, t = tid & 3;
    const int ib = kb + 1 + blockIdx.x;
    const size_t dbase = (size_t)kb * kNB * N + (size_t)kb * kNB;
    const size_t rbase = (size_t)ib * kNB * N + (size_t)kb * kNB + (size_t)row * N;
    for (int e = tid; e < kNB * kNB; e += 256) D[e / kNB][e % kNB] = L[dbase + (size_t)(e / kNB) * N + e % kNB];
    double x[kNB / 4];
#pragma unroll
    for (int m = 0; m < kNB / 4; ++m) x[m] = L[rbase + 4 * m + t];
    __syncthreads();
#pragma unroll
    for (int c = 0; c < kNB; ++c) {
        double v = 0.0;
#pragma unroll
        for (int m = 0; m < kNB / 4; ++m)
            if (4 * m + t < c) v = fma(x[m], D[c][4 * m + t], v);
        v += __shfl_xor(v, 1, 64);
        v += __shfl_xor(v, 2, 64);
        if (t == (c & 3)) x[c >> 2] = (x[c >> 2] - v) / D[c][c];
    }
#pragma unroll
    for (int m = 0; m < kNB / 4; ++m) L[rbase + 4 * m + t] = x[m];
}

// trailing update A_ij -= L_ik L_jk^T for kb < jb <= ib (lower block
// triangle), one 64 x 64 block per workgroup of 4 waves on the FP64 matrix
// cores: wave w owns rows 16 w .. 16 w + 15 of the block
__global__ __launch_bounds__(256) void chol_update_kernel(int N, int kb, double* L)
{
    __shared__ double Li[kNB][kNB + 1];
    __shared__ double Lj[kNB][kNB + 1];
    const int nb = N / kNB - kb - 1;   // blocks after kb
    // blockIdx.x enumerates the lower triangle (ib, jb) of the trailing blocks
    int t = blockIdx.x, ib = 0;
    while (t > ib) {
        t -= ib + 1;
        ++ib;
    }
    const int jb = t;
    if (ib >= nb) return;
    const int I = kb + 1 + ib, Jb = kb + 1 + jb;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int g = lane >> 4, c = lane & 15;
    for (int e = tid; e < kNB * kNB; e += 256) {
        Li[e / kNB][e % kNB] = L[(size_t)(I * kNB + e / kNB) * N + kb * kNB + e % kNB];
        Lj[e / kNB][e % kNB] = L[(size_t)(Jb * kNB + e / kNB) * N + kb * kNB + e % kNB];
    }
    __syncthreads();
    f64x4 acc[4];
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[b] = f64x4{0, 0, 0, 0};
    for (int k0 = 0; k0 < kNB; k0 += 4) {
        const double a = Li[16 * wave + c][k0 + g];
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[b] = mma_f64(a, Lj[16 * b + c][k0 + g], acc[b]);
    }
#pragma unroll
    for (int b = 0; b < 4; ++b)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int row = I * kNB + 16 * wave + out_row<true>(g, r);
            const int col = Jb * kNB + 16 * b + c;
            L[(size_t)row * N + col] -= acc[b][r];
        }
}

// Solve H Y = G for kRhs rank columns per workgroup: L z = g forward, then
// L^T y = z backward; z and y live in LDS (row-major, kRhs per row).  Rows
// are processed in 64-row blocks: the four waves sum the contributions of
// the finished blocks (wave w takes every fourth of them; each loaded entry
// of L serves the kRhs columns), then wave 0 solves the block's triangle
// sequentially, multiplying by the reciprocals of the diagonal.
constexpr int kRhs = 1;
__global__ __launch_bounds__(256) void dikin_solve_kernel(int n, int N, int r,
                                                          const double* __restrict__ L,
                                                          const double* __restrict__ G,
                                                          double* Y)
{
    extern __shared__ double zs[];       // N x kRhs values
    __shared__ double part[4][kNB][kRhs];
    const int a0 = blockIdx.x * kRhs, tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int nblk = N / kNB;
    for (int e = tid; e < N * kRhs; e += 256) {
        const int i = e / kRhs, t = e - i * kRhs;
        zs[e] = (i < n && a0 + t < r) ? G[(size_t)i * r + a0 + t] : 0.0;
    }
    __syncthreads();
    // forward: lane = row of the block, waves split the finished blocks
    for (int kb = 0; kb < nblk; ++kb) {
        const int i = kb * kNB + lane;
        double v[kRhs] = {};
        for (int jb = wave; jb < kb; jb += 4) {
            const double* lr = L + (size_t)i * N + jb * kNB;
            for (int j = 0; j < kNB; ++j) {
                const double l = lr[j];
#pragma unroll
                for (int t = 0; t < kRhs; ++t) v[t] = fma(l, zs[(jb * kNB + j) * kRhs + t], v[t]);
            }
        }
#pragma unroll
        for (int t = 0; t < kRhs; ++t) part[wave][lane][t] = v[t];
        __syncthreads();
        if (wave == 0) {
            double rhs[kRhs];
#pragma unroll
            for (int t = 0; t < kRhs; ++t)
                rhs[t] = zs[i * kRhs + t] - (part[0][lane][t] + part[1][lane][t] + part[2][lane][t] + part[3][lane][t]);
            const double* lr = L + (size_t)i * N + kb * kNB;
            const double rii = 1.0 / lr[lane];   // reciprocal of this row's diagonal
            for (int c = 0; c < kNB; ++c) {
                // row c of the block is final once the earlier rows are
                const double lc = lr[c];
                const double rc = __shfl(rii, c, 64);
#pragma unroll
                for (int t = 0; t < kRhs; ++t) {
                    const double zc = __shfl(rhs[t], c, 64) * rc;
                    if (lane == c) rhs[t] = zc;
                    if (lane > c) rhs[t] -= lc * zc;
                }
            }
#pragma unroll
            for (int t = 0; t < kRhs; ++t) zs[i * kRhs + t] = rhs[t];
        }
        __syncthreads();
    }
    // backward: L^T y = z, blocks from the last; y overwrites z
    for (int kb = nblk - 1; kb >= 0; --kb) {
        const int i = kb * kNB + lane;
        double v[kRhs] = {};
        for (int jb = kb + 1 + wave; jb < nblk; jb += 4)
            for (int j = 0; j < kNB; ++j) {
                const double l = L[(size_t)(jb * kNB + j) * N + i];
#pragma unroll
                for (int t = 0; t < kRhs; ++t) v[t] = fma(l, zs[(jb * kNB + j) * kRhs + t], v[t]);
            }
#pragma unroll
        for (int t = 0; t < kRhs; ++t) part[wave][lane][t] = v[t];
        __syncthreads();
        if (wave == 0) {
            double rhs[kRhs];
#pragma unroll
            for (int t = 0; t < kRhs; ++t)
                rhs[t] = zs[i * kRhs + t] - (part[0][lane][t] + part[1][lane][t] + part[2][lane][t] + part[3][lane][t]);
            const double rii = 1.0 / L[(size_t)i * N + i];
            for (int c = kNB - 1; c >= 0; --c) {
                // column c of the block: L[kb*64 + c][kb*64 + lane] for lane < c
                const double lcl = L[(size_t)(kb * kNB + c) * N + kb * kNB + lane];
                const double rc = __shfl(rii, c, 64);
#pragma unroll
                for (int t = 0; t < kRhs; ++t) {
                    const double yc = __shfl(rhs[t], c, 64) * rc;
                    if (lane == c) rhs[t] = yc;
                    if (lane < c) rhs[t] -= lcl * yc;
                }
            }
#pragma unroll
            for (int t = 0; t < kRhs; ++t) zs[i * kRhs + t] = rhs[t];
        }
        __syncthreads();
    }
    for (int e = tid; e < n * kRhs; e += 256) {
        const int i = e / kRhs, t = e - i * kRhs;
        if (a0 + t < r) Y[(size_t)i * r + a0 + t] = zs[e];
    }
}

// U <- U - eta Y, V = U / exp(l); skipped when a pivot failed (status != 0)
__global__ void dikin_update_kernel(int n, int r, double eta, const double* __restrict__ Y,
                                    const double* __restrict__ esig, const int* status, double* U,
                                    double* V)
{
    if (*status) return;
    const int64_t total = (int64_t)n * r;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int i = (int)(e / r);
        const double u = U[e] - eta * Y[e];
        U[e] = u;
        V[e] = u / esig[i];
    }
}

// power vector init: v_j = first normal of the TRAIN stream (chain j, step 1)
__global__ void dikin_init_kernel(int n, int N, uint64_t seed, double* v)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= N) return;
    double ev = 0.0, od;
    if (j < n) {
        Block4 w = stream_block(seed, 4, (uint32_t)j, 1, 0);
        gauss_pair(w, ev, od);
    }
    v[j] = ev;
}

inline int blocks_for(int64_t total, int threads)
{
    int64_t b = (total + threads - 1) / threads;
    return (int)(b < 1 ? 1 : (b > 65535 ? 65535 : b));
}

}  // namespace

int dikin_order(int n) { return (int)round_up(n, kNB); }

size_t dikin_bytes(int n, int r, int m_pad)
{
    auto al = [](size_t v) { return (v + 255) & ~(size_t)255; };
    const size_t N = (size_t)dikin_order(n);
    size_t b = 0;
    b += 2 * al(N * N * 8);            // H, L
    b += al((size_t)m_pad * 8);        // row weights
    b += 4 * al(N * 8);                // v, y0, y1, dsq
    b += 2 * al((size_t)n * r * 8);    // HU, Y
    b += al(64);                       // lam
    return b;
}

void dikin_carve(PrecondBufs* p, void* ws)
{
    auto al = [](size_t v) { return (v + 255) & ~(size_t)255; };
    char* b = (char*)ws;
    size_t o = 0;
    auto take = [&](size_t bytes) {
        char* q = b + o;
        o += al(bytes);
        return q;
    };
    const size_t N = (size_t)dikin_order(p->n);
    p->N = (int)N;
    p->Hm = (double*)take(N * N * 8);
    p->Lm = (double*)take(N * N * 8);
    p->wrow = (double*)take((size_t)p->m_pad * 8);
    p->pv = (double*)take(N * 8);
    p->py0 = (double*)take(N * 8);
    p->py1 = (double*)take(N * 8);
    p->dsq = (double*)take(N * 8);
    p->HU = (double*)take((size_t)p->n * p->r * 8);
    p->Ysol = (double*)take((size_t)p->n * p->r * 8);
    p->lam = (double*)take(64);
}

hipError_t launch_dikin_init(const PrecondBufs& p, uint64_t seed, hipStream_t stream)
{
    hipLaunchKernelGGL(dikin_init_kernel, dim3((p.N + 255) / 256), dim3(256), 0, stream, p.n, p.N,
                       seed, p.pv);
    return hipGetLastError();
}

// mean state, weights and H
static hipError_t dikin_hessian(const PrecondBufs& p, const double* X, hipStream_t stream)
{
    hipError_t e = launch_precond_mean(p, X, stream);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(dikin_weights_kernel, dim3((p.m_pad + 3) / 4), dim3(256), 0, stream, p.n,
                       p.m, p.m_pad, p.lda, p.A64, p.b64, p.mean, p.wrow, p.status);
    hipLaunchKernelGGL(dikin_hessian_kernel, dim3(p.N / kNB, p.N / kNB), dim3(512), 0, stream,
                       p.n, p.N, p.m_pad, p.lda, p.A64, p.wrow, p.Hm);
    return hipGetLastError();
}

// C, its inverse and log det, the gradient rows and K at the current (U, l)
static hipError_t dikin_gradient(const PrecondBufs& p, hipStream_t stream)
{
    hipLaunchKernelGGL(dikin_cap_kernel, dim3(1), dim3(512), 0, stream, p.n, p.r, p.U, p.W, p.C);
    hipLaunchKernelGGL(dikin_hu_kernel, dim3(p.N / 16), dim3(64), 0, stream, p.n, p.N, p.r, p.Hm,
                       p.U, p.HU);
    hipError_t e = launch_precond_capacitance(p, stream);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(dikin_grad_kernel, dim3((p.n + 3) / 4), dim3(256), 0, stream, p.n, p.N,
                       p.r, p.Hm, p.HU, p.U, p.W, p.Cinv, p.logsig, p.gU, p.gl, p.rowterm);
    hipLaunchKernelGGL(dikin_value_kernel, dim3(1), dim3(256), 0, stream, p.n, p.rowterm,
                       p.nll + 1, p.nll);
    return hipGetLastError();
}

hipError_t launch_dikin_loss(const PrecondBufs& p, const double* X, hipStream_t stream)
{
    hipError_t e = dikin_hessian(p, X, stream);
    if (e == hipSuccess) e = launch_precond_w(p, stream);
    if (e == hipSuccess) e = dikin_gradient(p, stream);
    return e;
}

hipError_t launch_dikin_train(const PrecondBufs& p, const double* X, int k_pow, double eta,
                              hipStream_t stream)
{
    hipError_t e = dikin_hessian(p, X, stream);
    if (e != hipSuccess) return e;
    const int n = p.n, N = p.N;
    hipLaunchKernelGGL(dikin_diag_kernel, dim3((N + 255) / 256), dim3(256), 0, stream, N, p.Hm,
                       p.dsq);
    // k power iterations: y_1 = J v, y_{t+1} = J (y_t / |y_t|); v = y_k / |y_k|;
    // then y = J v for the Rayleigh quotient
    const double* yin = p.pv;
    double* bufs[2] = {p.py0, p.py1};
    for (int it = 0; it < k_pow; ++it) {
        double* yout = bufs[it & 1];
        hipLaunchKernelGGL(dikin_power_kernel, dim3((n + 3) / 4), dim3(256), 0, stream, n, N, p.Hm,
                           p.dsq, yin, it > 0 ? 1 : 0, yout, (double*)nullptr);
        yin = yout;
    }
    double* yfin = bufs[k_pow & 1];
    hipLaunchKernelGGL(dikin_power_kernel, dim3((n + 3) / 4), dim3(256), 0, stream, n, N, p.Hm,
                       p.dsq, yin, 1, yfin, p.pv);
    hipLaunchKernelGGL(dikin_scales_kernel, dim3(1), dim3(1024), 0, stream, n, N, p.Hm, p.pv, yfin,
                       p.status, log(p.kappa), p.lam, p.logsig, p.esig);
    e = launch_precond_w(p, stream);
    if (e == hipSuccess) e = dikin_gradient(p, stream);
    if (e != hipSuccess) return e;
    // Cholesky factor of H
    hipLaunchKernelGGL(dikin_copy_kernel, dim3(blocks_for((int64_t)N * N, 256)), dim3(256), 0,
                       stream, (int64_t)N * N, p.Hm, p.Lm);
    const int nblk = N / kNB;
    for (int kb = 0; kb < nblk; ++kb) {
        hipLaunchKernelGGL(chol_diag_kernel, dim3(1), dim3(256), 0, stream, N, kb, p.Lm, p.status);
        const int rest = nblk - kb - 1;
        if (rest > 0) {
            hipLaunchKernelGGL(chol_panel_kernel, dim3(rest), dim3(256), 0, stream, N, kb, p.Lm);
            hipLaunchKernelGGL(chol_update_kernel, dim3(rest * (rest + 1) / 2), dim3(256), 0, stream,
                               N, kb, p.Lm);
        }
    }
    hipLaunchKernelGGL(dikin_solve_kernel, dim3((p.r + kRhs - 1) / kRhs), dim3(256),
                       (size_t)N * kRhs * 8, stream, n, N, p.r, p.Lm, p.gU, p.Ysol);
    hipLaunchKernelGGL(dikin_update_kernel, dim3(blocks_for((int64_t)n * p.r, 256)), dim3(256), 0,
                       stream, n, p.r, eta, p.Ysol, p.esig, p.status, p.U, p.V);
    return hipGetLastError();
}

}  // namespace mhar
