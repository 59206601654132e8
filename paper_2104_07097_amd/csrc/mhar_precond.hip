// mhar_precond.hip -- learned direction covariance for MHAR (FP64).
//
// The directions of the walks are drawn as d = P (U eps + exp(l) o h) with
// eps ~ N(0, I_r), h ~ N(0, I_n): Gaussian with covariance
// Sigma = U U^T + diag(exp(2 l)), symmetric and independent of the state,
// so every hit-and-run step keeps the uniform law on the polytope.  During
// burn-in (U, l) are fitted to the walk states by Adam on the Gaussian
// negative log-likelihood
//     NLL = 1/2 log det Sigma + 1/2 tr(Sigma^{-1} S),
// S the (1/z) covariance of the z states about their mean, then frozen: a
// fit of Sigma to the covariance of the target brings the body towards the
// near-isotropic position the paper's cost analysis assumes (S3.1).
//
// With D = diag(exp(2 l)), W = D^{-1} U, C = I + U^T W (r x r), Y the
// centred states (z x n), B = Y W (z x r), H = Y^T B / z, G = B^T B / z and
// K = I + C^{-1} G (Woodbury and the determinant lemma):
//     NLL  = sum_i (l_i + S_ii exp(-2 l_i)/2) + log det C / 2 - tr(C^{-1} G) / 2
//     dU   = (W K - D^{-1} H) C^{-1}
//     dl_i = exp(2 l_i) [ (Sigma^{-1})_ii - (Sigma^{-1} S Sigma^{-1})_ii ],
//     (Sigma^{-1})_ii = exp(-2 l_i) - sum_a V_ia W_ia,  V = W C^{-1},
//     (Sigma^{-1} S Sigma^{-1})_ii = exp(-4 l_i) S_ii - 2 exp(-2 l_i) sum_a V_ia H_ia
//                                    + sum_ab V_ia V_ib G_ab.
// Only n x r, z x r and r x r quantities are formed.
#include <math.h>

#include "mhar_device.hpp"
#include "mhar_internal.hpp"

namespace mhar {

namespace {

constexpr uint32_t kTagTrain = 4;

__global__ void precond_init_kernel(int n, int r, uint64_t seed, double* U, double* V,
                                    double* logsig, double* esig, double* m1V, double* m2V,
                                    double* m1l, double* m2l, int* status)
{
    if (blockIdx.x == 0 && threadIdx.x == 0) *status = 0;
    const int64_t total = (int64_t)n * r;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int j = (int)(e / r), q = (int)(e - (int64_t)j * r);
        Block4 w = stream_block(seed, kTagTrain, (uint32_t)j, 0, (uint32_t)(q >> 1));
        double ev, od;
        gauss_pair(w, ev, od);
        U[e] = 0.01 * ((q & 1) ? od : ev);
        V[e] = U[e];   // log scales start at 0
        m1V[e] = 0.0;
        m2V[e] = 0.0;
    }
    for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < n;
         j += (int64_t)gridDim.x * blockDim.x) {
        logsig[j] = 0.0;
        esig[j] = 1.0;
        m1l[j] = 0.0;
        m2l[j] = 0.0;
    }
}

// exp(l) only (restoring a checkpoint brings V with it)
__global__ void esig_kernel(int n, const double* logsig, double* esig)
{
    for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < n; j += gridDim.x * blockDim.x)
        esig[j] = exp(logsig[j]);
}

// scales of a caller-given (U, l): exp(l) and the trained coordinates V = U / exp(l)
__global__ void scales_kernel(int n, int r, const double* U, const double* logsig, double* esig,
                              double* V, int* status)
{
    if (blockIdx.x == 0 && threadIdx.x == 0) *status = 0;
    for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < n; j += gridDim.x * blockDim.x) {
        const double e = exp(logsig[j]);
        esig[j] = e;
        for (int q = 0; q < r; ++q) V[(int64_t)j * r + q] = U[(int64_t)j * r + q] / e;
    }
}

// column means and (1/z) variances of the states, two passes, each split
// over kSplitZ stripes of walks so that the whole device takes part: one
// block of 8 waves per (64 coordinates, stripe), lane = coordinate, partial
// sums in `part` (stripe-major), combined in a fixed order by the reduce
// kernels (mean first, then the squared deviations from it).
constexpr int kSplitZ = 32;
__global__ __launch_bounds__(512) void moment_part_kernel(int n, int z, int lda,
                                                          const double* __restrict__ X,
                                                          const double* __restrict__ mean,
                                                          double* part)
{
    __shared__ double acc[8][64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int i = blockIdx.x * 64 + lane, y = blockIdx.y;
    const int per = (z + kSplitZ - 1) / kSplitZ;
    const int k0 = y * per, k1 = min(z, k0 + per);
    double s = 0.0;
    if (i < n) {
        if (mean) {
            const double mu = mean[i];
            for (int k = k0 + wave; k < k1; k += 8) {
                const double d = X[(size_t)k * lda + i] - mu;
                s = fma(d, d, s);
            }
        } else {
            for (int k = k0 + wave; k < k1; k += 8) s += X[(size_t)k * lda + i];
        }
    }
    acc[wave][lane] = s;
    __syncthreads();
    if (wave == 0 && i < n) {
        double t = 0.0;
        for (int w = 0; w < 8; ++w) t += acc[w][lane];
        part[(size_t)y * n + i] = t;
    }
}

// out_i = (sum of the stripes' partial sums, in stripe order) / z
__global__ void moment_reduce_kernel(int n, int z, const double* __restrict__ part, double* out)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double t = 0.0;
    for (int y = 0; y < kSplitZ; ++y) t += part[(size_t)y * n + i];
    out[i] = t / z;
}

static void launch_moments(const PrecondBufs& p, const double* X, hipStream_t stream)
{
    const dim3 grid((p.n + 63) / 64, kSplitZ);
    hipLaunchKernelGGL(moment_part_kernel, grid, dim3(512), 0, stream, p.n, p.z, p.lda, X,
                       (const double*)nullptr, p.part);
    hipLaunchKernelGGL(moment_reduce_kernel, dim3((p.n + 255) / 256), dim3(256), 0, stream, p.n,
                       p.z, p.part, p.mean);
    hipLaunchKernelGGL(moment_part_kernel, grid, dim3(512), 0, stream, p.n, p.z, p.lda, X,
                       (const double*)p.mean, p.part);
    hipLaunchKernelGGL(moment_reduce_kernel, dim3((p.n + 255) / 256), dim3(256), 0, stream, p.n,
                       p.z, p.part, p.Sd);
}

__global__ void w_kernel(int n, int r, const double* U, const double* logsig, double* W)
{
    const int64_t total = (int64_t)n * r;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int j = (int)(e / r);
        W[e] = U[e] * exp(-2.0 * logsig[j]);
    }
}

// B[k][q] = sum_i (X[k][i] - mean_i) W[i][q]: one wave per state (8 per block),
// one lane per rank column, loads of a block of 8 coordinates issued together
__global__ __launch_bounds__(512) void b_kernel(int n, int r, int z, int lda,
                                                const double* __restrict__ X,
                                                const double* __restrict__ mean,
                                                const double* __restrict__ W, double* B)
{
    const int q = threadIdx.x & 63, k = blockIdx.x * 8 + (threadIdx.x >> 6);
    if (q >= r || k >= z) return;
    const double* xr = X + (size_t)k * lda;
    double v = 0.0;
    int i = 0;
    for (; i + 8 <= n; i += 8) {
        double y[8], w[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            y[u] = xr[i + u] - mean[i + u];
            w[u] = W[(size_t)(i + u) * r + q];
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) v = fma(y[u], w[u], v);
    }
    for (; i < n; ++i) v = fma(xr[i] - mean[i], W[(size_t)i * r + q], v);
    B[(size_t)k * r + q] = v;
}

// H[i][q] = (1/z) sum_k (X[k][i] - mean_i) B[k][q], split over kSplit chunks of
// states: block (i-group of 8, chunk) has one wave per coordinate, lane = q;
// the chunks' partial sums are added in chunk order by h_reduce_kernel.
constexpr int kSplit = 32;
static_assert(kSplitZ <= kSplit, "the partial-sum buffer holds kSplitZ x n values");
__global__ __launch_bounds__(512) void h_part_kernel(int n, int r, int z, int lda,
                                                     const double* __restrict__ X,
                                                     const double* __restrict__ mean,
                                                     const double* __restrict__ B, double* part)
{
    const int q = threadIdx.x & 63, i = blockIdx.x * 8 + (threadIdx.x >> 6), p = blockIdx.y;
    if (q >= r || i >= n) return;
    const int per = (z + kSplit - 1) / kSplit, k0 = p * per, k1 = min(z, k0 + per);
    const double mu = mean[i];
    double v = 0.0;
    int k = k0;
    for (; k + 8 <= k1; k += 8) {
        double y[8], b[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            y[u] = X[(size_t)(k + u) * lda + i] - mu;
            b[u] = B[(size_t)(k + u) * r + q];
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) v = fma(y[u], b[u], v);
    }
    for (; k < k1; ++k) v = fma(X[(size_t)k * lda + i] - mu, B[(size_t)k * r + q], v);
    part[((size_t)p * n + i) * r + q] = v;
}

__global__ void h_reduce_kernel(int n, int r, int z, const double* __restrict__ part, double* H)
{
    const int64_t total = (int64_t)n * r;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        double v = 0.0;
        for (int p = 0; p < kSplit; ++p) v += part[(size_t)p * total + e];
        H[e] = v / z;
    }
}

// Partial sums of G = B^T B over kSplit chunks of states: block p stages its
// rows of B in LDS, 64 at a time; each thread owns 8 of the r x r entries.
__global__ __launch_bounds__(512) void g_part_kernel(int r, int z, const double* __restrict__ B,
                                                     double* part)
{
    __shared__ double Bs[64][kMaxMeq + 1];
    const int tid = threadIdx.x, p = blockIdx.x;
    const int per = (z + kSplit - 1) / kSplit, k0 = p * per, k1 = min(z, k0 + per);
    double acc[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) acc[u] = 0.0;
    for (int kb = k0; kb < k1; kb += 64) {
        const int nb = min(64, k1 - kb);
        __syncthreads();
        for (int e = tid; e < nb * r; e += 512) {
            const int kk = e / r, a = e - kk * r;
            Bs[kk][a] = B[(size_t)(kb + kk) * r + a];
        }
        __syncthreads();
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int e = tid + u * 512;
            if (e < r * r) {
                const int a = e / r, b = e - a * r;
                double g = acc[u];
                for (int kk = 0; kk < nb; ++kk) g = fma(Bs[kk][a], Bs[kk][b], g);
                acc[u] = g;
            }
        }
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
        const int e = tid + u * 512;
        if (e < r * r) part[(size_t)p * r * r + e] = acc[u];
    }
}

// G = (sum of the chunks in chunk order) / z; C = I + U^T W (block per row a,
// thread per column b, sequential over the coordinates)
__global__ void gc_reduce_kernel(int n, int r, int z, const double* __restrict__ part,
                                 const double* __restrict__ U, const double* __restrict__ W,
                                 double* G, double* C)
{
    const int a = blockIdx.x, b = threadIdx.x;
    if (b >= r) return;
    const int e = a * r + b;
    double g = 0.0;
    for (int p = 0; p < kSplit; ++p) g += part[(size_t)p * r * r + e];
    G[e] = g / z;
    double c = (a == b) ? 1.0 : 0.0;
    for (int i = 0; i < n; ++i) c = fma(U[(size_t)i * r + a], W[(size_t)i * r + b], c);
    C[e] = c;
}

// Cholesky of C (r <= 64), log det C, C^{-1} and (K non-null) K = I + C^{-1} G;
// one workgroup of 256 threads.
constexpr int kLd = kMaxMeq + 1;
// Right-looking factorisation with lane i owning row i; C^{-1} column q is
// solved by lane q (forward then backward substitution) in LDS.
__global__ __launch_bounds__(256) void chol_kernel(int r, const double* C, const double* G,
                                                   double* Cinv, double* K, double* logdet,
                                                   int* status)
{
    __shared__ double L[kMaxMeq * kLd];   // rows padded: lanes walk a column
    __shared__ double Y[kMaxMeq * kMaxMeq];
    __shared__ double col[kMaxMeq];
    // right-looking factorisation, thread (ty, tx) holding entries
    // (ty + 16 a, tx + 16 b) in registers; column j published through LDS
    const int tid = threadIdx.x, ty = tid >> 4, tx = tid & 15, lane = tid;
    double t[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const int i = ty + 16 * a, k = tx + 16 * b;
            t[a][b] = (i < r && k < r) ? C[i * r + k] : 0.0;
        }
    int bad = 0;
    double ld = 0.0;
    for (int j = 0; j < r; ++j) {
        if (tx == (j & 15)) {
#pragma unroll
            for (int a = 0; a < 4; ++a)
#pragma unroll
                for (int b = 0; b < 4; ++b)
                    if (b == (j >> 4)) col[ty + 16 * a] = t[a][b];
        }
        __syncthreads();
        const double piv = col[j];
        if (!(piv > 0.0)) {
            bad = 1;
            break;
        }
        const double ljj = sqrt(piv), rj = 1.0 / ljj;
        ld += 2.0 * log(ljj);
        double li[4], lk[4];
#pragma unroll
        for (int a = 0; a < 4; ++a) {
            const int i = ty + 16 * a;
            li[a] = (i > j && i < r) ? col[i] * rj : 0.0;
        }
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const int k = tx + 16 * b;
            lk[b] = (k > j && k < r) ? col[k] * rj : 0.0;
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
    if (tid == 0) {
        *logdet = ld;
        if (bad) atomicOr(status, 4);
    }
    if (bad) return;
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const int i = ty + 16 * a, k = tx + 16 * b;
            if (i < r && k <= i) L[i * kLd + k] = t[a][b];
        }
    __syncthreads();
    if (lane < r) {
        // lane q solves column q of C^{-1}, the column held in registers
        // (loops unrolled over the maximal rank, guarded by r)
        const int q = lane;
        double y[kMaxMeq];
#pragma unroll
        for (int i = 0; i < kMaxMeq; ++i) {
            if (i < r) {
                double v = (i == q) ? 1.0 : 0.0;
#pragma unroll
                for (int k = 0; k < i; ++k) v -= L[i * kLd + k] * y[k];
                y[i] = v / L[i * kLd + i];
            }
        }
#pragma unroll
        for (int i = kMaxMeq - 1; i >= 0; --i) {
            if (i < r) {
                double v = y[i];
#pragma unroll
                for (int k = i + 1; k < kMaxMeq; ++k)
                    if (k < r) v -= L[k * kLd + i] * y[k];
                y[i] = v / L[i * kLd + i];
            }
        }
#pragma unroll
        for (int i = 0; i < kMaxMeq; ++i)
            if (i < r) Y[i * r + q] = y[i];
    }
    __syncthreads();
    for (int e = tid; e < r * r; e += 256) Cinv[e] = Y[e];
    if (!K) return;   // the Dikin fit does not use K
    // G into the rows of L (no longer needed), then K = I + C^{-1} G
    for (int e = tid; e < r * r; e += 256) L[(e / r) * kLd + e % r] = G[e];
    __syncthreads();
    for (int e = tid; e < r * r; e += 256) {
        const int p = e / r, q = e - p * r;
        double v = (p == q) ? 1.0 : 0.0;
        for (int k = 0; k < r; ++k) v = fma(Y[p * r + k], L[k * kLd + q], v);
        K[e] = v;
    }
}

// per coordinate i: dU row, dl_i and the row's NLL term; one block of 64 lanes per row
__global__ void grad_kernel(int n, int r, const double* __restrict__ W, const double* __restrict__ H,
                            const double* __restrict__ K, const double* __restrict__ Cinv,
                            const double* __restrict__ G, const double* __restrict__ logsig,
                            const double* __restrict__ Sd, const int* status, double* gU,
                            double* gl, double* rowterm)
{
    __shared__ double R[kMaxMeq], V[kMaxMeq], Wr[kMaxMeq], Hr[kMaxMeq];
    if (*status) return;   // C was not factorised: Cinv and K are not valid
    const int i = blockIdx.x, q = threadIdx.x;
    const double dinv = exp(-2.0 * logsig[i]);
    if (q < r) {
        Wr[q] = W[(size_t)i * r + q];
        Hr[q] = H[(size_t)i * r + q];
    }
    __syncthreads();
    if (q < r) {
        double v = 0.0, w = 0.0;
        for (int c = 0; c < r; ++c) {
            v = fma(Wr[c], K[c * r + q], v);
            w = fma(Wr[c], Cinv[c * r + q], w);
        }
        R[q] = v - dinv * Hr[q];
        V[q] = w;
    }
    __syncthreads();
    if (q < r) {
        double v = 0.0;
        for (int b = 0; b < r; ++b) v = fma(R[b], Cinv[b * r + q], v);
        gU[(size_t)i * r + q] = v;
    }
    if (q == 0) {
        double vw = 0.0, vh = 0.0, vgv = 0.0;
        for (int a = 0; a < r; ++a) {
            vw = fma(V[a], Wr[a], vw);
            vh = fma(V[a], Hr[a], vh);
            double t = 0.0;
            for (int b = 0; b < r; ++b) t = fma(G[a * r + b], V[b], t);
            vgv = fma(V[a], t, vgv);
        }
        const double sinv = dinv - vw;
        const double sss = dinv * dinv * Sd[i] - 2.0 * dinv * vh + vgv;
        gl[i] = (sinv - sss) / dinv;
        rowterm[i] = logsig[i] + 0.5 * Sd[i] * dinv;
    }
}

// NLL = sum_i rowterm_i + log det C / 2 - tr(C^{-1} G) / 2: one block of 256,
// contiguous partial sums per thread combined by a fixed-shape tree
__global__ __launch_bounds__(256) void nll_kernel(int n, int r, const double* rowterm,
                                                  const double* Cinv, const double* G,
                                                  const double* logdet, double* nll)
{
    __shared__ double ps[256], pt[256];
    const int tid = threadIdx.x;
    const int per = (n + 255) / 256;
    double s = 0.0;
    for (int i = tid * per; i < min(n, (tid + 1) * per); ++i) s += rowterm[i];
    double tr = 0.0;
    for (int e = tid; e < r * r; e += 256) {
        const int p = e / r, q = e - p * r;
        tr = fma(Cinv[p * r + q], G[q * r + p], tr);
    }
    ps[tid] = s;
    pt[tid] = tr;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (tid < h) {
            ps[tid] += ps[tid + h];
            pt[tid] += pt[tid + h];
        }
        __syncthreads();
    }
    if (tid == 0) *nll = ps[0] + 0.5 * (*logdet) - 0.5 * pt[0];
}

// One Adam (Kingma & Ba) update in the scale-free coordinates (V, l), U = diag(exp(l)) V.
// With gU, gl the NLL gradient in (U, l), the chain rule gives dV = exp(l) o gU (row scale)
// and dl = gl + sum_q gU o U (each row).  Gradients in (V, l) are O(1) whatever the axis
// lengths, which keeps Adam's per-entry step from swamping the weak pull on long axes.
// One thread per coordinate row; after the update U = exp(l_new) o V_new.
__global__ void adam_kernel(int n, int r, int64_t t, double lr, double b1, double b2, double eps,
                            double* U, double* V, const double* gU, double* m1V, double* m2V,
                            double* logsig, const double* gl, double* m1l, double* m2l,
                            double* esig, const int* status)
{
    if (*status) return;   // the gradient was not formed
    const double c1 = 1.0 - pow(b1, (double)t), c2 = 1.0 - pow(b2, (double)t);
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const int64_t row = (int64_t)i * r;
        const double e = esig[i];
        double g = gl[i];
        for (int q = 0; q < r; ++q) g = __dadd_rn(g, __dmul_rn(gU[row + q], U[row + q]));
        for (int q = 0; q < r; ++q) {
            const int64_t k = row + q;
            const double gv = __dmul_rn(gU[k], e);
            m1V[k] = b1 * m1V[k] + (1.0 - b1) * gv;
            m2V[k] = b2 * m2V[k] + (1.0 - b2) * gv * gv;
            V[k] -= lr * (m1V[k] / c1) / (sqrt(m2V[k] / c2) + eps);
        }
        m1l[i] = b1 * m1l[i] + (1.0 - b1) * g;
        m2l[i] = b2 * m2l[i] + (1.0 - b2) * g * g;
        logsig[i] -= lr * (m1l[i] / c1) / (sqrt(m2l[i] / c2) + eps);
        const double en = exp(logsig[i]);
        esig[i] = en;
        for (int q = 0; q < r; ++q) U[row + q] = __dmul_rn(en, V[row + q]);
    }
}

inline int blocks_for(int64_t total, int threads)
{
    int64_t b = (total + threads - 1) / threads;
    return (int)(b < 1 ? 1 : (b > 65535 ? 65535 : b));
}

// ---- split screening of the tiled path: A P U and ||U||_F ----

// Y = A_eq U (m_eq x r), one thread per entry, sequential over the coordinates
__global__ void lowrank_aequ_kernel(int n, int lda, int r, int m_eq, const double* __restrict__ Aeq,
                                    const double* __restrict__ U, double* Y)
{
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= m_eq * r) return;
    const int p = e / r, q = e - p * r;
    double v = 0.0;
    for (int j = 0; j < n; ++j) v = fma(Aeq[(size_t)p * lda + j], U[(size_t)j * r + q], v);
    Y[e] = v;
}

// P U = U - W Y (W^T rows = (A_eq A_eq^T)^{-1} A_eq), or a copy of U
__global__ void lowrank_pu_kernel(int n, int lda, int r, int m_eq, const double* __restrict__ WT,
                                  const double* __restrict__ Y, const double* __restrict__ U,
                                  double* PU)
{
    const int64_t total = (int64_t)n * r;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int j = (int)(e / r), q = (int)(e - (int64_t)j * r);
        double v = U[e];
        for (int p = 0; p < m_eq; ++p) v = fma(-WT[(size_t)p * lda + j], Y[p * r + q], v);
        PU[e] = v;
    }
}

// Rows of A P U on the FP64 matrix cores, written as the screening operand
// (the first rk columns of a row of length lda, as A's operand, zero padded)
// with each row's norm rounded up.  One wave per 16 rows, the r <= 64
// columns as 4 tiles of 16; f64 16x16x4: lane (g, c) supplies a = A[row c][k0 + g] and
// b = (P U)[k0 + g][16 t + c]; out[q] of tile t = row out_row(g, q), column
// 16 t + c.
__global__ __launch_bounds__(64) void lowrank_au_kernel(int n, int lda, int r, int rk, int m_pad,
                                                        int bf16, const double* __restrict__ A64,
                                                        const double* __restrict__ PU,
                                                        void* AUop, float* aun)
{
    const int lane = threadIdx.x;
    const int g = lane >> 4, c = lane & 15;
    const int row0 = blockIdx.x * 16;   // m_pad is a multiple of 16
    const double* ar = A64 + (size_t)(row0 + c) * lda;
    f64x4 acc[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) acc[t] = f64x4{0, 0, 0, 0};
    for (int k0 = 0; k0 < n; k0 += 4) {
        const int k = k0 + g;
        const double av = k < n ? ar[k] : 0.0;
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const int q = 16 * t + c;
            const double bv = (k < n && q < r) ? PU[(size_t)k * r + q] : 0.0;
            acc[t] = mma_f64(av, bv, acc[t]);
        }
    }
    // row norms: the 16 lanes of a lane group hold the 16 columns of a tile
    double ss[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        double v = 0.0;
#pragma unroll
        for (int t = 0; t < 4; ++t) v = fma(acc[t][q], acc[t][q], v);
#pragma unroll
        for (int o = 1; o < 16; o <<= 1) v += __shfl_xor(v, o, 64);
        ss[q] = v;
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int row = row0 + out_row<true>(g, q);
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const int col = 16 * t + c;
            if (col >= rk) continue;
            const float v = (float)acc[t][q];   // columns r .. rk - 1 are zero
            const size_t o = (size_t)row * lda + col;
            if (bf16) {
                __bf16 hi, lo;
                split_bf16(v, hi, lo);
                ((__bf16*)AUop)[o] = hi;
                ((__bf16*)AUop)[(size_t)m_pad * lda + o] = lo;
            } else {
                ((float*)AUop)[o] = v;
            }
        }
        if (c == 0) aun[row] = (float)sqrt(ss[q]) * (1.0f + 0x1.0p-20f);
    }
}

// ||U||_F (one workgroup, fixed-shape tree)
__global__ __launch_bounds__(256) void lowrank_frob_kernel(int64_t count, const double* U, double* out)
{
    __shared__ double ps[256];
    const int tid = threadIdx.x;
    double v = 0.0;
    for (int64_t e = tid; e < count; e += 256) v = fma(U[e], U[e], v);
    ps[tid] = v;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (tid < h) ps[tid] += ps[tid + h];
        __syncthreads();
    }
    if (tid == 0) *out = sqrt(ps[0]);
}

}  // namespace

size_t lowrank_bytes(int prec, int n, int r, int m_pad, int lda, int z_pad, int m_eq)
{
    (void)prec;
    auto al = [](size_t v) { return (v + 255) & ~(size_t)255; };
    const size_t rk = (size_t)round_up(r, 32);
    size_t b = 0;
    // the operands keep the row stride lda of A's and the direction's, of
    // which the first rk columns are used
    b += al((size_t)m_pad * lda * 4);      // A P U operand (FP32, or bf16 hi + lo)
    b += al((size_t)m_pad * 4);            // its row norms
    b += al((size_t)z_pad * lda * 4);      // eps operand
    b += al((size_t)n * r * 8);            // P U
    b += al((size_t)(m_eq > 0 ? m_eq : 1) * r * 8);   // A_eq U
    b += al(64);                           // ||U||_F
    b += al((size_t)z_pad * lda * 8);      // isotropic part of the directions
    b += 3 * al((size_t)z_pad * 8);        // hn, en, F
    return b;
}

void lowrank_carve(PrecondBufs* p, void* ws)
{
    auto al = [](size_t v) { return (v + 255) & ~(size_t)255; };
    char* b = (char*)ws;
    size_t o = 0;
    auto take = [&](size_t bytes) {
        char* q = b + o;
        o += al(bytes);
        return q;
    };
    const size_t rk = (size_t)round_up(p->r, 32);
    p->rk = (int)rk;
    p->AUop = take((size_t)p->m_pad * p->lda * 4);
    p->aun = (float*)take((size_t)p->m_pad * 4);
    p->Eop = take((size_t)p->z_pad * p->lda * 4);
    p->PU = (double*)take((size_t)p->n * p->r * 8);
    p->uF = (double*)take(64);
    double* aequ = (double*)take((size_t)(p->m_eq > 0 ? p->m_eq : 1) * p->r * 8);
    p->Hs = (double*)take((size_t)p->z_pad * p->lda * 8);
    p->hn = (double*)take((size_t)p->z_pad * 8);
    p->en = (double*)take((size_t)p->z_pad * 8);
    p->F = (double*)take((size_t)p->z_pad * 8);
    p->AeqU = aequ;
}

hipError_t launch_lowrank_setup(const PrecondBufs& p, hipStream_t stream)
{
    if (p.m_eq > 0)
        hipLaunchKernelGGL(lowrank_aequ_kernel, dim3((p.m_eq * p.r + 255) / 256), dim3(256), 0,
                           stream, p.n, p.lda, p.r, p.m_eq, p.Aeq, p.U, p.AeqU);
    hipLaunchKernelGGL(lowrank_pu_kernel, dim3(blocks_for((int64_t)p.n * p.r, 256)), dim3(256), 0,
                       stream, p.n, p.lda, p.r, p.m_eq, p.WT, p.AeqU, p.U, p.PU);
    hipLaunchKernelGGL(lowrank_au_kernel, dim3(p.m_pad / 16), dim3(64), 0, stream, p.n, p.lda,
                       p.r, p.rk, p.m_pad, p.prec == kBF16X3 ? 1 : 0, p.A64, p.PU, p.AUop, p.aun);
    hipLaunchKernelGGL(lowrank_frob_kernel, dim3(1), dim3(256), 0, stream, (int64_t)p.n * p.r, p.U,
                       p.uF);
    return hipGetLastError();
}


size_t precond_bytes(int n, int r, int z, int lda, int objective, int m_pad)
{
    (void)lda;
    auto al = [](size_t v) { return (v + 255) & ~(size_t)255; };
    const size_t nr = (size_t)n * r, rr = (size_t)r * r;
    size_t b = 0;
    b += 5 * al(nr * 8);              // U, m1V, m2V, W, H
    b += 2 * al(nr * 8);              // gU, V
    b += 8 * al((size_t)n * 8);       // logsig, esig, m1l, m2l, mean, Sd, gl, rowterm
    b += al((size_t)z * r * 8);       // B
    b += 4 * al(rr * 8);              // G, C, Cinv, K
    b += al(64);                      // nll, logdet
    b += al(64);                      // status
    b += al((size_t)kSplit * (nr > rr ? nr : rr) * 8);   // split-K and per-stripe partial sums
    if (objective == 1) b += dikin_bytes(n, r, m_pad);
    return b;
}

void precond_carve(PrecondBufs* p, void* ws)
{
    auto al = [](size_t v) { return (v + 255) & ~(size_t)255; };
    char* b = (char*)ws;
    size_t o = 0;
    const size_t nr = (size_t)p->n * p->r, rr = (size_t)p->r * p->r;
    auto take = [&](size_t bytes) {
        char* q = b + o;
        o += al(bytes);
        return q;
    };
    p->U = (double*)take(nr * 8);
    p->m1V = (double*)take(nr * 8);
    p->m2V = (double*)take(nr * 8);
    p->W = (double*)take(nr * 8);
    p->H = (double*)take(nr * 8);
    p->gU = (double*)take(nr * 8);
    p->V = (double*)take(nr * 8);
    p->logsig = (double*)take((size_t)p->n * 8);
    p->esig = (double*)take((size_t)p->n * 8);
    p->m1l = (double*)take((size_t)p->n * 8);
    p->m2l = (double*)take((size_t)p->n * 8);
    p->mean = (double*)take((size_t)p->n * 8);
    p->Sd = (double*)take((size_t)p->n * 8);
    p->gl = (double*)take((size_t)p->n * 8);
    p->rowterm = (double*)take((size_t)p->n * 8);
    p->B = (double*)take((size_t)p->z * p->r * 8);
    p->GB = (double*)take(rr * 8);
    p->C = (double*)take(rr * 8);
    p->Cinv = (double*)take(rr * 8);
    p->K = (double*)take(rr * 8);
    p->nll = (double*)take(64);
    p->status = (int*)take(64);
    p->part = (double*)take((size_t)kSplit * (nr > rr ? nr : rr) * 8);
    if (p->objective == 1) dikin_carve(p, b + o);
}

hipError_t launch_precond_init(const PrecondBufs& p, uint64_t seed, hipStream_t stream)
{
    hipLaunchKernelGGL(precond_init_kernel, dim3(blocks_for((int64_t)p.n * p.r, 256)), dim3(256), 0,
                       stream, p.n, p.r, seed, p.U, p.V, p.logsig, p.esig, p.m1V, p.m2V, p.m1l, p.m2l,
                       p.status);
    return hipGetLastError();
}

hipError_t launch_precond_set_scales(const PrecondBufs& p, hipStream_t stream)
{
    hipLaunchKernelGGL(scales_kernel, dim3(blocks_for(p.n, 64)), dim3(64), 0, stream, p.n, p.r, p.U,
                       p.logsig, p.esig, p.V, p.status);
    return hipGetLastError();
}

hipError_t launch_precond_grad(const PrecondBufs& p, const double* X, hipStream_t stream)
{
    double* rowterm = p.rowterm;
    launch_moments(p, X, stream);
    hipLaunchKernelGGL(w_kernel, dim3(blocks_for((int64_t)p.n * p.r, 256)), dim3(256), 0, stream,
                       p.n, p.r, p.U, p.logsig, p.W);
    hipLaunchKernelGGL(b_kernel, dim3((p.z + 7) / 8), dim3(512), 0, stream, p.n, p.r, p.z, p.lda,
                       X, p.mean, p.W, p.B);
    hipLaunchKernelGGL(h_part_kernel, dim3((p.n + 7) / 8, kSplit), dim3(512), 0, stream, p.n, p.r,
                       p.z, p.lda, X, p.mean, p.B, p.part);
    hipLaunchKernelGGL(h_reduce_kernel, dim3(blocks_for((int64_t)p.n * p.r, 256)), dim3(256), 0,
                       stream, p.n, p.r, p.z, p.part, p.H);
    hipLaunchKernelGGL(g_part_kernel, dim3(kSplit), dim3(512), 0, stream, p.r, p.z, p.B, p.part);
    hipLaunchKernelGGL(gc_reduce_kernel, dim3(p.r), dim3(64), 0, stream, p.n, p.r, p.z, p.part,
                       p.U, p.W, p.GB, p.C);
    hipLaunchKernelGGL(chol_kernel, dim3(1), dim3(256), 0, stream, p.r, p.C, p.GB, p.Cinv, p.K,
                       p.nll + 1, p.status);
    hipLaunchKernelGGL(grad_kernel, dim3(p.n), dim3(64), 0, stream, p.n, p.r, p.W, p.H, p.K, p.Cinv,
                       p.GB, p.logsig, p.Sd, p.status, p.gU, p.gl, rowterm);
    hipLaunchKernelGGL(nll_kernel, dim3(1), dim3(256), 0, stream, p.n, p.r, rowterm, p.Cinv, p.GB,
                       p.nll + 1, p.nll);
    return hipGetLastError();
}

hipError_t launch_precond_esig(const PrecondBufs& p, hipStream_t stream)
{
    hipLaunchKernelGGL(esig_kernel, dim3(blocks_for(p.n, 256)), dim3(256), 0, stream, p.n, p.logsig,
                       p.esig);
    return hipGetLastError();
}

hipError_t launch_precond_mean(const PrecondBufs& p, const double* X, hipStream_t stream)
{
    launch_moments(p, X, stream);
    return hipGetLastError();
}

hipError_t launch_precond_w(const PrecondBufs& p, hipStream_t stream)
{
    hipLaunchKernelGGL(w_kernel, dim3(blocks_for((int64_t)p.n * p.r, 256)), dim3(256), 0, stream,
                       p.n, p.r, p.U, p.logsig, p.W);
    return hipGetLastError();
}

// C^{-1} and log det C of the capacitance matrix in p.C (K = I + C^{-1} C is
// formed as a by-product and not used)
hipError_t launch_precond_capacitance(const PrecondBufs& p, hipStream_t stream)
{
    hipLaunchKernelGGL(chol_kernel, dim3(1), dim3(256), 0, stream, p.r, p.C, p.C, p.Cinv,
                       (double*)nullptr, p.nll + 1, p.status);
    return hipGetLastError();
}

hipError_t launch_precond_adam(const PrecondBufs& p, int64_t t, double lr, double b1, double b2,
                               double eps, hipStream_t stream)
{
    hipLaunchKernelGGL(adam_kernel, dim3(blocks_for(p.n, 64)), dim3(64), 0, stream, p.n, p.r, t,
                       lr, b1, b2, eps, p.U, p.V, p.gU, p.m1V, p.m2V, p.logsig, p.gl, p.m1l, p.m2l,
                       p.esig, p.status);
    return hipGetLastError();
}

}  // namespace mhar
