// mhar_kernels.hip -- HIP kernels of the Matrix Hit-and-Run step for gfx950.
//
// One workgroup owns a tile of 16 walks and every constraint row, and runs
// many steps per launch.  Per step (paper Alg. 2 with S4.3-S4.5):
//   A. directions: Philox4x32-10 -> Box-Muller normals (S4.3), projection
//      d = h - W (A_eq h) onto null(A_eq) (S3.2, factored form of P);
//      written as FP64 rows and as the matrix-core operand tile in LDS;
//   B. screening: G = A D on the matrix cores (FP64 / FP32 / BF16x3), fused
//      with the deferred slack update s <- s - theta_prev G_prev and with
//      interval bounds of every ratio s_i / g_i (S4.4, Lemma 4.2): a
//      certified upper bound U of each chord end and, per 64-row group, the
//      least lower bound L;
//   D. exact chord: rows whose lower bound does not exceed U are the only
//      rows that can attain the chord end; they are evaluated exactly in
//      FP64 (s_i = b_i - a_i x, g_i = a_i d, sequential sums, no
//      contraction), giving lambda_min / lambda_max; theta is drawn
//      uniformly between them (S4.5) and x <- x + theta d;
//   E. every R steps: exact FP64 recompute of the slack s = b - A X on the
//      matrix cores, which also resets the drift bound.
#include <math.h>

#include "mhar_device.hpp"
#include "mhar_internal.hpp"

namespace mhar {

namespace {

constexpr int kCandCap = 512;   // candidate (row, walk) pairs listed per tile and step
constexpr int kPairCap = 512;   // flagged (walk, row group) pairs listed per tile and step

struct ChainLds {
    double theta[kChainTile];
    double E[kChainTile];
    double dnorm[kChainTile];
    double hnorm[kChainTile];   // split screening: ||isotropic part||, ||eps||, low-rank drift
    double enorm[kChainTile];
    double F[kChainTile];
    double y[kChainTile * kMaxMeq];
    unsigned up[kChainTile];
    unsigned um[kChainTile];
    int flags[kChainTile];
    unsigned long long exact;
    // exact chords: candidate list, and per walk the chord ends as the bits of
    // lambda_max and of -lambda_min (both >= 0, so integer min is float min)
    unsigned long long lmax_bits[kChainTile];
    unsigned long long nlmin_bits[kChainTile];
    int cfl[kChainTile];
    int ncand;
    int2 cand[kCandCap];
    // candidate scan: the flagged (walk, 64-row group) pairs, walk << 16 | group,
    // and each walk's chord-end bounds and screening error terms
    int npairs;
    int pairs[kPairCap];
    float w_up[kChainTile], w_um[kChainTile], w_ed[kChainTile], w_ed2[kChainTile];
    float w_F[kChainTile], w_E[kChainTile];
};

// s_i = b_i - a_i x and g_i = a_i d in FP64 in the order of a sequential sum
// (separate roundings, the device code is built without contraction); the
// loads of a block of 16 are issued before its dependent chain.
__device__ __forceinline__ void exact_row(const double* __restrict__ ar,
                                          const double* __restrict__ xr,
                                          const double* __restrict__ dr, double bi, int n,
                                          double& s_out, double& g_out)
{
    constexpr int B = 16;
    double s = bi, g = 0.0;
    int j = 0;
    for (; j + B <= n; j += B) {
        double av[B], xv[B], dv[B];
#pragma unroll
        for (int u = 0; u < B; ++u) {
            av[u] = ar[j + u];
            xv[u] = xr[j + u];
            dv[u] = dr[j + u];
        }
#pragma unroll
        for (int u = 0; u < B; ++u) {
            s = __dsub_rn(s, __dmul_rn(av[u], xv[u]));
            g = __dadd_rn(g, __dmul_rn(av[u], dv[u]));
        }
    }
    for (; j < n; ++j) {
        s = __dsub_rn(s, __dmul_rn(ar[j], xr[j]));
        g = __dadd_rn(g, __dmul_rn(ar[j], dr[j]));
    }
    s_out = s;
    g_out = g;
}

// Chord-end contribution of one exactly evaluated row (S4.4, Lemma 4.2).
__device__ __forceinline__ void chord_row(ChainLds* cs, int cl, double s, double gg, double bi)
{
    if (s < -1e-12 * fmax(1.0, fabs(bi))) atomicOr(&cs->cfl[cl], kInfeasible);
    if (s < 0.0) s = 0.0;
    if (gg > 0.0) atomicMin(&cs->lmax_bits[cl], (unsigned long long)__double_as_longlong(s / gg));
    else if (gg < 0.0)
        atomicMin(&cs->nlmin_bits[cl], (unsigned long long)__double_as_longlong(-(s / gg)));
}

// Wait until at most N vector-memory operations of this wave are outstanding
// (gfx9 s_waitcnt encoding; expcnt and lgkmcnt left at their maxima).
template <int N>
__device__ __forceinline__ void wait_vm()
{
    static_assert(N >= 0 && N < 64, "vmcnt range");
    __builtin_amdgcn_s_waitcnt((N & 15) | ((N >> 4) << 14) | (7 << 4) | (15 << 8));
}
// Wait for this wave's LDS reads.
__device__ __forceinline__ void wait_lds() { __builtin_amdgcn_s_waitcnt(0xC07F); }

// Exact evaluation of listed candidates through LDS: batches of `nb_max`
// candidates, one per thread; for each chunk of C coordinates the workgroup
// stages the candidates' rows of A and the x and d rows of the 16 walks with
// coalesced 16-byte loads, then every thread continues its sequential sums
// from LDS.  Same arithmetic, in the same order, as exact_row.  A chunk is at
// most kStagePer 16-byte pieces per thread; they are loaded into registers
// all at once, and the next chunk's loads are issued before the current
// chunk's sums, so one load latency per chunk is exposed, not one per piece.
constexpr int kUpd = 16;   // coordinates per lane and block in the state update
static_assert(kThreads == 32 * kChainTile, "32 lanes per walk in the norm pass");
template <int kStagePer>
__device__ void exact_rows_staged(const StepArgs& a, ChainLds* cs, int c0, int nc, double* stage,
                                  int nb_max, int C)
{
    const int tid = threadIdx.x;
    const int n = a.n, lda = a.lda;
    const int ld = C + 2;                     // LDS row stride (doubles), keeps 16-byte alignment
    for (int b0 = 0; b0 < nc; b0 += nb_max) {
        const int nb = min(nb_max, nc - b0);
        const int rows = nb + 2 * kChainTile;
        int2 rc = make_int2(0, 0);
        double s = 0.0, gg = 0.0;
        if (tid < nb) {
            rc = cs->cand[b0 + tid];
            s = a.b64[rc.x];
        }
        // b has landed before the chunk loads are issued (else the first sum
        // would wait for all of them)
        wait_vm<0>();
        // the pieces in flight as plain scalars (an array of vector structs
        // would be placed in LDS by the compiler)
        double vx[kStagePer], vy[kStagePer];
        int off[kStagePer];
        // pass j0 stores the chunk at column j0 (loaded by the previous pass)
        // into the stage, issues the loads of the next chunk, then continues
        // the sums over the staged chunk; the first pass only loads
        for (int j0 = -C; j0 < n; j0 += C) {
            if (j0 >= 0) {
                __syncthreads();                  // the previous chunk is consumed
#pragma unroll
                for (int u = 0; u < kStagePer; ++u)
                    if (off[u] >= 0) *(double2*)(stage + off[u]) = make_double2(vx[u], vy[u]);
                __syncthreads();
            }
            const int jn = j0 + C;
            if (jn < n) {
                // staged width: the whole padded row, even; off[u] is the
                // piece's LDS offset, -1 if the thread has no piece u
                const int halves = min(C, lda - jn) >> 1;
                // nothing is in flight here (the stores above waited for the
                // previous chunk); saying so keeps the compiler from waiting
                // between the pieces below
                wait_vm<0>();
#pragma unroll
                for (int u = 0; u < kStagePer; ++u) {
                    const int e = u * kThreads + tid;
                    off[u] = -1;
                    if (e < rows * halves) {
                        const int r = e / halves, h = e - r * halves;
                        const double* src;
                        if (r < nb) {
                            src = a.A64 + (size_t)cs->cand[b0 + r].x * lda;
                        } else {
                            const int w = r - nb, cl = w & (kChainTile - 1);
                            const int chain = min(c0 + cl, a.z_pad - 1);
                            src = (w < kChainTile ? a.X : a.D) + (size_t)chain * lda;
                        }
                        const double2 t = *(const double2*)(src + jn + 2 * h);
                        vx[u] = t.x;
                        vy[u] = t.y;
                        off[u] = r * ld + 2 * h;
                    }
                }
            }
            if (j0 < 0) continue;
            if (tid < nb) {
                const double* av = stage + tid * ld;
                const double* xv = stage + (nb + rc.y) * ld;
                const double* dv = stage + (nb + kChainTile + rc.y) * ld;
                const int len = min(C, n - j0);
                int j = 0;
                for (; j + 8 <= len; j += 8) {
                    double a8[8], x8[8], d8[8];
#pragma unroll
                    for (int u = 0; u < 8; ++u) {
                        a8[u] = av[j + u];
                        x8[u] = xv[j + u];
                        d8[u] = dv[j + u];
                    }
#pragma unroll
                    for (int u = 0; u < 8; ++u) {
                        s = __dsub_rn(s, __dmul_rn(a8[u], x8[u]));
                        gg = __dadd_rn(gg, __dmul_rn(a8[u], d8[u]));
                    }
                }
                for (; j < len; ++j) {
                    s = __dsub_rn(s, __dmul_rn(av[j], xv[j]));
                    gg = __dadd_rn(gg, __dmul_rn(av[j], dv[j]));
                }
            }
        }
        if (tid < nb) chord_row(cs, rc.y, s, gg, a.b64[rc.x]);
    }
}

__host__ __device__ inline int x_ld(int lda) { return lda + 2; }     // FP64 LDS row stride
__host__ __device__ inline int f32_ld(int lda) { return lda + 4; }   // FP32 LDS row stride
__host__ __device__ inline int bf_ld(int lda) { return lda + 8; }    // bf16 LDS row stride

__host__ __device__ inline size_t big_bytes(int lda)
{
    return (size_t)kChainTile * x_ld(lda) * sizeof(double);
}

template <int P> struct Op;
template <> struct Op<kFP64> {
    typedef double state_t;
    static constexpr bool f64 = true;
};
template <> struct Op<kFP32> {
    typedef float state_t;
    static constexpr bool f64 = false;
};
template <> struct Op<kBF16X3> {
    typedef float state_t;
    static constexpr bool f64 = false;
};

// index of (row, walk c of tile) in a slack / product buffer (Q = m_pad / 16)
template <bool F64>
__device__ __forceinline__ size_t frag_index(int tile, int Q, int row, int c)
{
    return (((size_t)tile * (Q >> 2) + (row >> 6)) * kChainTile + c) * 64 + (row & 63);
}

// ---------------------------------------------------------------------------
// Phase A: directions of the 16 walks of this tile at `step`.
// ---------------------------------------------------------------------------
// sum over j = lane + 64 k of a[j] b[j] as one FMA chain per lane in
// increasing k (before a wave reduction); the loads of 8 coordinates per lane
// are in flight together
__device__ __forceinline__ double lane_dot(const double* a, const double* b, int n, int lane)
{
    double v = 0.0;
    for (int jb = 0; jb < n; jb += 64 * 8) {
        double x[8], y[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const int j = jb + lane + 64 * e;
            x[e] = j < n ? a[j] : 0.0;
            y[e] = j < n ? b[j] : 0.0;
        }
#pragma unroll
        for (int e = 0; e < 8; ++e)
            if (jb + lane + 64 * e < n) v = fma(x[e], y[e], v);
    }
    return v;
}

// Wide (the chords kernel): the low-rank product two coordinates per thread
// with U prefetched, and no norms (the caller computes them with the
// operand); otherwise one coordinate per thread, fewer registers, and the
// norms here.  Both sum each walk over the rank in order.
template <bool Wide>
__device__ void make_directions(const StepArgs& a, ChainLds* cs, int c0, uint64_t step)
{
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int n = a.n, lda = a.lda;
    const int npairs = (n + 1) >> 1;
    for (int item = tid; item < kChainTile * npairs; item += kThreads) {
        int cl = item / npairs, p = item - cl * npairs;
        int chain = c0 + cl;
        if (chain >= a.z) continue;
        Block4 w = stream_block(a.seed, kTagDir, a.chain_offset + (uint32_t)chain, step,
                                (uint32_t)p);
        double ev, od;
        gauss_pair(w, ev, od);
        double* drow = a.D + (size_t)chain * lda;
        drow[2 * p] = ev;
        if (2 * p + 1 < n) drow[2 * p + 1] = od;
    }
    if (a.r > 0) {
        // learned preconditioner: h <- U eps + exp(l) o h, eps ~ N(0, I_r)
        // from the LOWRANK stream (sequential sum over the rank, no contraction)
        __syncthreads();
        double* eps = cs->y;
        const int rpairs = (a.r + 1) >> 1;
        for (int item = tid; item < kChainTile * rpairs; item += kThreads) {
            int cl = item / rpairs, p = item - cl * rpairs;
            int chain = c0 + cl;
            if (chain >= a.z) continue;
            Block4 w = stream_block(a.seed, kTagLowRank, a.chain_offset + (uint32_t)chain, step,
                                    (uint32_t)p);
            double ev, od;
            gauss_pair(w, ev, od);
            eps[cl * kMaxMeq + 2 * p] = ev;
            if (2 * p + 1 < a.r) eps[cl * kMaxMeq + 2 * p + 1] = od;
        }
        __syncthreads();
        if constexpr (Wide) {
            // two coordinates per thread (j and j + kThreads), each walk's sum in
            // rank order.  U is read in blocks of 8 ranks, the next block's loads
            // in flight during the current block's arithmetic; the 16 walks' eps
            // are read two ranks at a time (16-byte LDS reads shared by both
            // coordinates).
            for (int j = tid; j < n; j += 2 * kThreads) {
                const int j2 = j + kThreads;
                const bool two = j2 < n;
                const double* ur = a.U + (size_t)j * a.r;
                const double* ur2 = a.U + (size_t)(two ? j2 : j) * a.r;
                double v[kChainTile], w[kChainTile];
#pragma unroll
                for (int cl = 0; cl < kChainTile; ++cl) {
                    v[cl] = 0.0;
                    w[cl] = 0.0;
                }
                const int r8 = a.r & ~7;
                double un[8], tn[8];
                if (r8 > 0) {
#pragma unroll
                    for (int e = 0; e < 8; ++e) {
                        un[e] = ur[e];
                        tn[e] = ur2[e];
                    }
                }
                int q = 0;
                for (; q < r8; q += 8) {
                    wait_vm<0>();   // this block's U has landed
                    double uc[8], tc[8];
#pragma unroll
                    for (int e = 0; e < 8; ++e) {
                        uc[e] = un[e];
                        tc[e] = tn[e];
                    }
                    if (q + 8 < r8) {
#pragma unroll
                        for (int e = 0; e < 8; ++e) {
                            un[e] = ur[q + 8 + e];
                            tn[e] = ur2[q + 8 + e];
                        }
                    }
#pragma unroll
                    for (int e = 0; e < 8; e += 2) {
#pragma unroll
                        for (int cl = 0; cl < kChainTile; ++cl) {
                            const double2 ep = *(const double2*)(eps + cl * kMaxMeq + q + e);
                            v[cl] = __dadd_rn(v[cl], __dmul_rn(uc[e], ep.x));
                            w[cl] = __dadd_rn(w[cl], __dmul_rn(tc[e], ep.x));
                            v[cl] = __dadd_rn(v[cl], __dmul_rn(uc[e + 1], ep.y));
                            w[cl] = __dadd_rn(w[cl], __dmul_rn(tc[e + 1], ep.y));
                        }
                    }
                }
                for (; q < a.r; ++q) {
                    const double u0 = ur[q], t0 = ur2[q];
#pragma unroll
                    for (int cl = 0; cl < kChainTile; ++cl) {
                        const double e = eps[cl * kMaxMeq + q];
                        v[cl] = __dadd_rn(v[cl], __dmul_rn(u0, e));
                        w[cl] = __dadd_rn(w[cl], __dmul_rn(t0, e));
                    }
                }
                const double es = a.esig[j];
                const double es2 = two ? a.esig[j2] : 0.0;
                // the draws of both coordinates, all loads before the stores
                double h1[kChainTile], h2[kChainTile];
#pragma unroll
                for (int cl = 0; cl < kChainTile; ++cl) {
                    const size_t o = (size_t)(c0 + cl) * lda + j;
                    const bool live = c0 + cl < a.z;
                    h1[cl] = live ? a.D[o] : 0.0;
                    h2[cl] = (live && two) ? a.D[o + kThreads] : 0.0;
                }
#pragma unroll
                for (int cl = 0; cl < kChainTile; ++cl) {
                    if (c0 + cl < a.z) {
                        const size_t o = (size_t)(c0 + cl) * lda + j;
                        const double hs = __dmul_rn(es, h1[cl]);
                        a.D[o] = __dadd_rn(v[cl], hs);
                        if (a.rk > 0) a.Hs[o] = hs;   // the isotropic part, for the split screening
                        if (two) {
                            const size_t o2 = o + kThreads;
                            const double hs2 = __dmul_rn(es2, h2[cl]);
                            a.D[o2] = __dadd_rn(w[cl], hs2);
                            if (a.rk > 0) a.Hs[o2] = hs2;
                        }
                    }
                }
            }
        } else {
            // one coordinate per thread: its row of U is loaded once, in blocks of
            // 8, and applied to the 16 walks
            for (int j = tid; j < n; j += kThreads) {
                const double* ur = a.U + (size_t)j * a.r;
                double v[kChainTile];
#pragma unroll
                for (int cl = 0; cl < kChainTile; ++cl) v[cl] = 0.0;
                int q = 0;
                for (; q + 8 <= a.r; q += 8) {
                    double u8[8];
#pragma unroll
                    for (int e = 0; e < 8; ++e) u8[e] = ur[q + e];
#pragma unroll
                    for (int e = 0; e < 8; ++e)
#pragma unroll
                        for (int cl = 0; cl < kChainTile; ++cl)
                            v[cl] = __dadd_rn(v[cl], __dmul_rn(u8[e], eps[cl * kMaxMeq + q + e]));
                }
                for (; q < a.r; ++q) {
                    const double uq = ur[q];
#pragma unroll
                    for (int cl = 0; cl < kChainTile; ++cl)
                        v[cl] = __dadd_rn(v[cl], __dmul_rn(uq, eps[cl * kMaxMeq + q]));
                }
                const double es = a.esig[j];
#pragma unroll
                for (int cl = 0; cl < kChainTile; ++cl) {
                    if (c0 + cl < a.z) {
                        const size_t o = (size_t)(c0 + cl) * lda + j;
                        const double hs = __dmul_rn(es, a.D[o]);
                        a.D[o] = __dadd_rn(v[cl], hs);
                        if (a.rk > 0) a.Hs[o] = hs;   // the isotropic part, for the split screening
                    }
                }
            }
        }
        if (a.rk > 0) {
            // eps as the second block of the screening operand (its first rk
            // columns, zero padded, in the direction operand's layout) and its
            // norm, before the projection reuses cs->y
            __syncthreads();
            const size_t zr = (size_t)a.z_pad * lda;
            for (int item = tid; item < kChainTile * a.rk; item += kThreads) {
                const int cl = item / a.rk, q = item - cl * a.rk, chain = c0 + cl;
                const float v = (chain < a.z && q < a.r) ? (float)eps[cl * kMaxMeq + q] : 0.0f;
                const size_t o = (size_t)chain * lda + q;
                if (a.prec == kBF16X3) {
                    __bf16 hi, lo;
                    split_bf16(v, hi, lo);
                    ((__bf16*)a.Eop)[o] = hi;
                    ((__bf16*)a.Eop)[zr + o] = lo;
                } else {
                    ((float*)a.Eop)[o] = v;
                }
            }
            for (int cl = wave; cl < kChainTile; cl += kWaves) {
                double v = 0.0;
                if (c0 + cl < a.z && lane < a.r) v = eps[cl * kMaxMeq + lane] * eps[cl * kMaxMeq + lane];
                v = wave_sum(v);
                if (lane == 0) cs->enorm[cl] = sqrt(v);
            }
        }
    }
    // projection onto null(A_eq) of the direction and, for the split
    // screening, of its isotropic part
    for (int part = 0; part < (a.rk > 0 ? 2 : 1) && a.m_eq > 0; ++part) {
        double* base = part ? a.Hs : a.D;
        __syncthreads();
        // y = A_eq h for every walk; one wave per (walk, equality row)
        for (int pr = wave; pr < kChainTile * a.m_eq; pr += kWaves) {
            int cl = pr / a.m_eq, p = pr - cl * a.m_eq;
            int chain = c0 + cl;
            double v = 0.0;
            if (chain < a.z) {
                v = lane_dot(a.Aeq + (size_t)p * lda, base + (size_t)chain * lda, n, lane);
            }
            v = wave_sum(v);
            if (lane == 0) cs->y[cl * kMaxMeq + p] = v;
        }
        __syncthreads();
        // d = h - W y,  W^T rows = (A_eq A_eq^T)^{-1} A_eq
        for (int item = tid; item < kChainTile * n; item += kThreads) {
            int cl = item / n, j = item - cl * n;
            int chain = c0 + cl;
            if (chain >= a.z) continue;
            double* dp = base + (size_t)chain * lda + j;
            double v = *dp;
            for (int p = 0; p < a.m_eq; ++p) v = fma(-a.WT[(size_t)p * lda + j], cs->y[cl * kMaxMeq + p], v);
            *dp = v;
        }
    }
    if (Wide) return;
    __syncthreads();
    // norms of d (wave per walk), and of the isotropic part
    for (int cl = wave; cl < kChainTile; cl += kWaves) {
        int chain = c0 + cl;
        double v = 0.0, w = 0.0;
        if (chain < a.z) {
            const double* dr = a.D + (size_t)chain * lda;
            for (int j = lane; j < n; j += 64) v = fma(dr[j], dr[j], v);
            if (a.rk > 0) {
                const double* hr = a.Hs + (size_t)chain * lda;
                for (int j = lane; j < n; j += 64) w = fma(hr[j], hr[j], w);
            }
        }
        v = wave_sum(v);
        w = wave_sum(w);
        if (lane == 0) {
            cs->dnorm[cl] = sqrt(v);
            cs->hnorm[cl] = sqrt(w);
        }
    }
}

// The directions of the tile as the matrix-core operand in LDS.
template <int P>
__device__ void stage_operand(const StepArgs& a, unsigned char* big, int c0)
{
    const int tid = threadIdx.x;
    const int n = a.n, lda = a.lda;
    if (P == kFP64) {
        double* Dt = (double*)big;
        const int ld = x_ld(lda);
        for (int item = tid; item < kChainTile * lda; item += kThreads) {
            int cl = item / lda, j = item - cl * lda;
            int chain = c0 + cl;
            Dt[cl * ld + j] = (chain < a.z && j < n) ? a.D[(size_t)chain * lda + j] : 0.0;
        }
    } else if (P == kFP32) {
        float* Dt = (float*)big;
        const int ld = f32_ld(lda);
        for (int item = tid; item < kChainTile * lda; item += kThreads) {
            int cl = item / lda, j = item - cl * lda;
            int chain = c0 + cl;
            Dt[cl * ld + j] = (chain < a.z && j < n) ? (float)a.D[(size_t)chain * lda + j] : 0.0f;
        }
    } else {
        __bf16* Dh = (__bf16*)big;
        const int ld = bf_ld(lda);
        __bf16* Dl = Dh + kChainTile * ld;
        for (int item = tid; item < kChainTile * lda; item += kThreads) {
            int cl = item / lda, j = item - cl * lda;
            int chain = c0 + cl;
            float v = (chain < a.z && j < n) ? (float)a.D[(size_t)chain * lda + j] : 0.0f;
            __bf16 hi, lo;
            split_bf16(v, hi, lo);
            Dh[cl * ld + j] = hi;
            Dl[cl * ld + j] = lo;
        }
    }
    __syncthreads();
}

// ---------------------------------------------------------------------------
// Phase B: screening product and fused epilogue over all rows.
// ---------------------------------------------------------------------------
template <int P>
__device__ void screen(const StepArgs& a, ChainLds* cs, unsigned char* big, int tile, int c0,
                       int pending, int T)
{
    typedef typename Op<P>::state_t st_t;
    constexpr bool F64 = Op<P>::f64;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int g = lane >> 4, c = lane & 15;
    const int lda = a.lda, Q = a.m_pad >> 4;
    const int ngroups = a.m_pad / kRowGroup;
    st_t* S = (st_t*)a.S;
    st_t* Gb = (st_t*)a.G;
    float* Lt = a.L + (size_t)tile * ngroups * 2 * kChainTile;

    const bool active = (c0 + c) < a.z;
    const float ed = active ? (float)(cs->dnorm[c] * (double)a.eps_g) * kHighGrow + 1e-30f : 0.0f;
    const float Ek = (float)cs->E[c] * kHighGrow;
    const st_t th = (st_t)cs->theta[c];
    const float bscale = a.u_s * (float)T * kHighGrow;
    float up = kInf, um = kInf;

    for (int row0 = wave * kRowGroup; row0 < a.m_pad; row0 += kWaves * kRowGroup) {
        float acc32[4][4];
        double acc64[4][4];
        if (P == kFP32) {
            const float* Dt = (const float*)big;
            const int ld = f32_ld(lda);
            f32x4 acc[4] = {{0, 0, 0, 0}, {0, 0, 0, 0}, {0, 0, 0, 0}, {0, 0, 0, 0}};
            // A chunks are prefetched one chunk ahead (register double buffer)
            float4 cur[8], nxt[8];
#pragma unroll
            for (int rb = 0; rb < 4; ++rb) {
                const float4* ap = (const float4*)(a.A32 + (size_t)(row0 + 16 * rb + c) * lda + 8 * g);
                cur[2 * rb] = ap[0];
                cur[2 * rb + 1] = ap[1];
            }
            for (int k0 = 0; k0 < lda; k0 += 32) {
                if (k0 + 32 < lda) {
#pragma unroll
                    for (int rb = 0; rb < 4; ++rb) {
                        const float4* ap = (const float4*)(a.A32 + (size_t)(row0 + 16 * rb + c) * lda + k0 + 32 + 8 * g);
                        nxt[2 * rb] = ap[0];
                        nxt[2 * rb + 1] = ap[1];
                    }
                }
                const float4* bp = (const float4*)(Dt + c * ld + k0 + 8 * g);
                const float4 b0 = bp[0], b1 = bp[1];
#pragma unroll
                for (int e = 0; e < 8; ++e) {
                    const float bv = e < 4 ? (&b0.x)[e] : (&b1.x)[e - 4];
#pragma unroll
                    for (int rb = 0; rb < 4; ++rb) {
                        const float av = e < 4 ? (&cur[2 * rb].x)[e] : (&cur[2 * rb + 1].x)[e - 4];
                        acc[rb] = mma_f32(av, bv, acc[rb]);
                    }
                }
#pragma unroll
                for (int q = 0; q < 8; ++q) cur[q] = nxt[q];
            }
#pragma unroll
            for (int rb = 0; rb < 4; ++rb)
#pragma unroll
                for (int r = 0; r < 4; ++r) acc32[rb][r] = acc[rb][r];
        } else if (P == kBF16X3) {
            const __bf16* Dh = (const __bf16*)big;
            const int ld = bf_ld(lda);
            const __bf16* Dl = Dh + kChainTile * ld;
            f32x4 acc[4] = {{0, 0, 0, 0}, {0, 0, 0, 0}, {0, 0, 0, 0}, {0, 0, 0, 0}};
            // A chunks are prefetched one chunk ahead (register double buffer)
            bf16x8 cur[8], nxt[8];
#pragma unroll
            for (int rb = 0; rb < 4; ++rb) {
                const size_t off = (size_t)(row0 + 16 * rb + c) * lda + 8 * g;
                cur[2 * rb] = *(const bf16x8*)(a.Ahi + off);
                cur[2 * rb + 1] = *(const bf16x8*)(a.Alo + off);
            }
            for (int k0 = 0; k0 < lda; k0 += 32) {
                if (k0 + 32 < lda) {
#pragma unroll
                    for (int rb = 0; rb < 4; ++rb) {
                        const size_t off = (size_t)(row0 + 16 * rb + c) * lda + k0 + 32 + 8 * g;
                        nxt[2 * rb] = *(const bf16x8*)(a.Ahi + off);
                        nxt[2 * rb + 1] = *(const bf16x8*)(a.Alo + off);
                    }
                }
                const bf16x8 bh = *(const bf16x8*)(Dh + c * ld + k0 + 8 * g);
                const bf16x8 bl = *(const bf16x8*)(Dl + c * ld + k0 + 8 * g);
#pragma unroll
                for (int rb = 0; rb < 4; ++rb) acc[rb] = mma_bf16(cur[2 * rb + 1], bh, acc[rb]);
#pragma unroll
                for (int rb = 0; rb < 4; ++rb) acc[rb] = mma_bf16(cur[2 * rb], bl, acc[rb]);
#pragma unroll
                for (int rb = 0; rb < 4; ++rb) acc[rb] = mma_bf16(cur[2 * rb], bh, acc[rb]);
#pragma unroll
                for (int q = 0; q < 8; ++q) cur[q] = nxt[q];
            }
#pragma unroll
            for (int rb = 0; rb < 4; ++rb)
#pragma unroll
                for (int r = 0; r < 4; ++r) acc32[rb][r] = acc[rb][r];
        } else {
            const double* Dt = (const double*)big;
            const int ld = x_ld(lda);
            f64x4 acc[4] = {{0, 0, 0, 0}, {0, 0, 0, 0}, {0, 0, 0, 0}, {0, 0, 0, 0}};
            for (int k0 = 0; k0 < lda; k0 += 16) {
                const double2* bp = (const double2*)(Dt + c * ld + k0 + 4 * g);
                double2 b0 = bp[0], b1 = bp[1];
#pragma unroll
                for (int rb = 0; rb < 4; ++rb) {
                    const double2* ap = (const double2*)(a.A64 + (size_t)(row0 + 16 * rb + c) * lda + k0 + 4 * g);
                    double2 a0 = ap[0], a1 = ap[1];
                    acc[rb] = mma_f64(a0.x, b0.x, acc[rb]);
                    acc[rb] = mma_f64(a0.y, b0.y, acc[rb]);
                    acc[rb] = mma_f64(a1.x, b1.x, acc[rb]);
                    acc[rb] = mma_f64(a1.y, b1.y, acc[rb]);
                }
            }
#pragma unroll
            for (int rb = 0; rb < 4; ++rb)
#pragma unroll
                for (int r = 0; r < 4; ++r) acc64[rb][r] = acc[rb][r];
        }

        float lp = kInf, lm = kInf;
#pragma unroll
        for (int rb = 0; rb < 4; ++rb) {
            const int q = (row0 >> 4) + rb;
            // FP32 state: this lane's rows 4g .. 4g + 3 are one 16-byte run
            float4 s4 = make_float4(0, 0, 0, 0), g4 = make_float4(0, 0, 0, 0);
            size_t idx4 = 0;
            if (!F64) {
                idx4 = frag_index<false>(tile, Q, 16 * q + 4 * g, c);
                s4 = *(const float4*)((const float*)S + idx4);
                if (pending) g4 = *(const float4*)((const float*)Gb + idx4);
            }
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = 16 * q + out_row<F64>(g, r);
                const size_t idx = frag_index<F64>(tile, Q, row, c);
                st_t gv = F64 ? (st_t)acc64[rb][r] : (st_t)acc32[rb][r];
                st_t sv;
                if (F64) {
                    sv = S[idx];
                    if (pending) {
                        sv = fma(-th, Gb[idx], sv);
                        S[idx] = sv;
                    }
                    Gb[idx] = gv;
                } else {
                    sv = (&s4.x)[r];
                    if (pending) sv = fma(-th, (st_t)(&g4.x)[r], sv);
                    (&s4.x)[r] = (float)sv;
                }
                const float na = a.rownorm[row];
                float dl = fmaf(na, Ek, fmaf(bscale, a.absb[row], 1e-30f));
                float e = na * ed;
                const float s32 = (float)sv, g32 = (float)gv;
                if (F64) {
                    dl = fmaf(fabsf(s32), 0x1.0p-23f, dl);
                    e = fmaf(fabsf(g32), 0x1.0p-23f, e);
                }
                float lo_p, hi_p, lo_m, hi_m;
                ratio_bounds(s32, g32, dl, e, lo_p, hi_p, lo_m, hi_m);
                up = fminf(up, hi_p);
                um = fminf(um, hi_m);
                lp = fminf(lp, lo_p);
                lm = fminf(lm, lo_m);
            }
            if (!F64) {
                if (pending) *(float4*)((float*)S + idx4) = s4;
                *(float4*)((float*)Gb + idx4) = make_float4(acc32[rb][0], acc32[rb][1], acc32[rb][2],
                                                            acc32[rb][3]);
            }
        }
        // per-group least lower bounds, one value per walk
        lp = fminf(lp, __shfl_xor(lp, 16, 64));
        lp = fminf(lp, __shfl_xor(lp, 32, 64));
        lm = fminf(lm, __shfl_xor(lm, 16, 64));
        lm = fminf(lm, __shfl_xor(lm, 32, 64));
        if (g == 0) {
            const int grp = row0 / kRowGroup;
            Lt[(grp * 2 + 0) * kChainTile + c] = lp;
            Lt[(grp * 2 + 1) * kChainTile + c] = lm;
        }
    }
    up = fminf(up, __shfl_xor(up, 16, 64));
    up = fminf(up, __shfl_xor(up, 32, 64));
    um = fminf(um, __shfl_xor(um, 16, 64));
    um = fminf(um, __shfl_xor(um, 32, 64));
    if (g == 0) {
        atomicMin(&cs->up[c], __float_as_uint(up));
        atomicMin(&cs->um[c], __float_as_uint(um));
    }
}

// ---------------------------------------------------------------------------
// Phase D: exact chords of the candidate rows, theta, state update.
// ---------------------------------------------------------------------------
// `stage` (stage_bytes of LDS free during this phase, may be null) carries the
// candidates' rows through LDS when it holds at least 16 coordinates of them.
// B: flagged groups a wave tests at once (their loads in flight together);
// the register-heavy general kernel takes one at a time.
template <int P, int B>
__device__ void exact_chords(const StepArgs& a, ChainLds* cs, int tile, int c0, uint64_t step,
                             int64_t s_rel, int T, double* stage, size_t stage_bytes)
{
    typedef typename Op<P>::state_t st_t;
    constexpr bool F64 = Op<P>::f64;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int n = a.n, lda = a.lda, Q = a.m_pad >> 4;
    const int ngroups = a.m_pad / kRowGroup;
    const st_t* S = (const st_t*)a.S;
    const st_t* Gb = (const st_t*)a.G;
    const float* Lt = a.L + (size_t)tile * ngroups * 2 * kChainTile;
    const float bscale = a.u_s * (float)T * kHighGrow;
    const double u64 = 0x1.0p-53;
    const unsigned long long kInfBits = 0x7FF0000000000000ull;

    if (tid < kChainTile) {
        cs->lmax_bits[tid] = kInfBits;
        cs->nlmin_bits[tid] = kInfBits;
        cs->cfl[tid] = 0;
    }
    if (tid == 0) cs->ncand = 0;
    __syncthreads();

    // 1. candidate rows of every walk: rows whose lower bound does not exceed
    //    the certified chord-end bound U.  (a) Each walk's 64-row groups whose
    //    least lower bound does not exceed U are listed as (walk, group)
    //    pairs; (b) all waves take the pairs, three at a time with their
    //    loads in flight together, and test the groups' rows.  Candidates are
    //    listed in LDS; past the lists' capacities they are evaluated on the
    //    spot.
    if (tid == 0) cs->npairs = 0;
    __syncthreads();
    // one group's rows for walk cl: the test and the listing of candidates
    auto test_rows = [&](int cl, int qq, float s32, float g32, float na, float nau, float ab,
                         unsigned long long& nex) __attribute__((always_inline)) {
        const int row = qq * kRowGroup + lane;
        float dl = fmaf(nau, cs->w_F[cl], fmaf(na, cs->w_E[cl], fmaf(bscale, ab, 1e-30f)));
        float e = fmaf(nau, cs->w_ed2[cl], na * cs->w_ed[cl]);
        if (F64) {
            dl = fmaf(fabsf(s32), 0x1.0p-23f, dl);
            e = fmaf(fabsf(g32), 0x1.0p-23f, e);
        }
        float lo_p, hi_p, lo_m, hi_m;
        ratio_bounds(s32, g32, dl, e, lo_p, hi_p, lo_m, hi_m);
        const bool cand = (row < a.m) && ((lo_p <= cs->w_up[cl]) || (lo_m <= cs->w_um[cl]));
        nex += __popcll(__ballot(cand));
        if (cand) {
            const int slot = atomicAdd(&cs->ncand, 1);
            if (slot < kCandCap) {
                cs->cand[slot] = make_int2(row, cl);
            } else {
                const int chain = c0 + cl;
                double sx, gg;
                const double bi = a.b64[row];
                exact_row(a.A64 + (size_t)row * lda, a.X + (size_t)chain * lda,
                          a.D + (size_t)chain * lda, bi, n, sx, gg);
                chord_row(cs, cl, sx, gg, bi);
            }
        }
    };
    auto load_rows = [&](int cl, int qq, float& s32, float& g32, float& na, float& nau,
                         float& ab) __attribute__((always_inline)) {
        const int row = qq * kRowGroup + lane;
        const size_t idx = frag_index<F64>(tile, Q, row, cl);
        s32 = (float)S[idx];
        g32 = (float)Gb[idx];
        na = a.rownorm[row];
        nau = a.rk > 0 ? a.aun[row] : 0.0f;
        ab = a.absb[row];
    };
    unsigned long long nex = 0;
    for (int cl = wave; cl < kChainTile; cl += kWaves) {
        const int chain = c0 + cl;
        if (chain >= a.z) continue;
        const float up = __uint_as_float(cs->up[cl]);
        const float um = __uint_as_float(cs->um[cl]);
        if (lane == 0) {
            float ed, ed2 = 0.0f, Fk = 0.0f;
            if (a.rk > 0) {
                const double hn = cs->hnorm[cl], en = cs->enorm[cl];
                const double dx = 0x1.0p-36 * (hn + cs->dnorm[cl] + *a.uF * en);
                ed = (float)(hn * (double)a.eps_g + dx) * kHighGrow + 1e-30f;
                ed2 = (float)(en * (double)a.eps_g) * kHighGrow;
                Fk = (float)cs->F[cl] * kHighGrow;
            } else {
                ed = (float)(cs->dnorm[cl] * (double)a.eps_g) * kHighGrow + 1e-30f;
            }
            cs->w_up[cl] = up;
            cs->w_um[cl] = um;
            cs->w_ed[cl] = ed;
            cs->w_ed2[cl] = ed2;
            cs->w_F[cl] = Fk;
            cs->w_E[cl] = (float)cs->E[cl] * kHighGrow;
        }
        unsigned long long over = 0;   // groups past the pair list's capacity
        for (int qb = 0; qb < ngroups; qb += 64) {
            const int q = qb + lane;
            bool need = false;
            if (q < ngroups)
                need = (Lt[(q * 2 + 0) * kChainTile + cl] <= up) ||
                       (Lt[(q * 2 + 1) * kChainTile + cl] <= um);
            const unsigned long long mask = __ballot(need);
            if (!mask) continue;
            int base = 0;
            if (lane == 0) base = atomicAdd(&cs->npairs, __popcll(mask));
            base = __shfl(base, 0, 64);
            const int slot = base + __popcll(mask & ((1ull << lane) - 1ull));
            if (need && slot < kPairCap) cs->pairs[slot] = (cl << 16) | q;
            over = __ballot(need && slot >= kPairCap);
            while (over) {
                const int qq = qb + __ffsll((long long)over) - 1;
                over &= over - 1;
                float s32, g32, na, nau, ab;
                load_rows(cl, qq, s32, g32, na, nau, ab);
                test_rows(cl, qq, s32, g32, na, nau, ab, nex);
            }
        }
    }
    __syncthreads();
    {
        const int np = min(cs->npairs, kPairCap);
        for (int p0 = wave; p0 < np; p0 += B * kWaves) {
            float s32[B], g32[B], na[B], nau[B], ab[B];
            int cl[B], qq[B];
#pragma unroll
            for (int k = 0; k < B; ++k) {
                const int p = p0 + k * kWaves;
                const int pr = p < np ? cs->pairs[p] : -1;
                cl[k] = pr >> 16;
                qq[k] = pr & 0xffff;
                if (pr >= 0) load_rows(cl[k], qq[k], s32[k], g32[k], na[k], nau[k], ab[k]);
            }
#pragma unroll
            for (int k = 0; k < B; ++k)
                if (p0 + k * kWaves < np) test_rows(cl[k], qq[k], s32[k], g32[k], na[k], nau[k], ab[k], nex);
        }
    }
    if (lane == 0 && nex) atomicAdd(&cs->exact, nex);
    __syncthreads();

    // 2. exact FP64 evaluation of the listed rows, all in parallel
    const int nc = min(cs->ncand, kCandCap);
    const int nb_max = 96;
    // chunk width: what the stage holds, and at most kStagePer pieces per thread
    int C = stage ? (int)(stage_bytes / (sizeof(double) * (nb_max + 2 * kChainTile))) - 2 : 0;
    // (the chords kernel: 16 pieces and 128 columns per chunk, in a stage of
    // its own; the single-kernel path, short of registers: 8 pieces)
    constexpr int kStagePer = B > 1 ? 16 : 8;
    C = min(C, 2 * kStagePer * kThreads / (nb_max + 2 * kChainTile)) & ~15;
    if (C >= 16) {
        exact_rows_staged<kStagePer>(a, cs, c0, nc, stage, nb_max, C);
    } else {
        for (int t = tid; t < nc; t += kThreads) {
            const int2 rc = cs->cand[t];
            const int chain = c0 + rc.y;
            double s, gg;
            const double bi = a.b64[rc.x];
            exact_row(a.A64 + (size_t)rc.x * lda, a.X + (size_t)chain * lda,
                      a.D + (size_t)chain * lda, bi, n, s, gg);
            chord_row(cs, rc.y, s, gg, bi);
        }
    }
    __syncthreads();

    // 3. theta (S4.5), the update and the drift bound of every walk
    for (int cl = wave; cl < kChainTile; cl += kWaves) {
        const int chain = c0 + cl;
        if (chain >= a.z) {
            if (lane == 0) cs->theta[cl] = 0.0;
            continue;
        }
        const double* dr = a.D + (size_t)chain * lda;
        const double lmax = __longlong_as_double((long long)cs->lmax_bits[cl]);
        const double lmin = -__longlong_as_double((long long)cs->nlmin_bits[cl]);
        int fl = cs->cfl[cl];
        double th = 0.0;
        if (lmax == kInfD || lmin == -kInfD) {
            fl |= kUnbounded;
        } else if (!(lmax > lmin)) {
            fl |= kDegenerate;
        } else {
            Block4 w = stream_block(a.seed, kTagTheta, a.chain_offset + (uint32_t)chain, step, 0);
            double u = open_unit(w.w0, w.w1);
            th = __dadd_rn(lmin, __dmul_rn(u, __dsub_rn(lmax, lmin)));
        }
        double xo = 0.0, xn2 = 0.0;
        bool finite = isfinite(th);
        double* xw = a.X + (size_t)chain * lda;
        const bool rec = a.rec_stride > 0 && chain < a.rec_chains &&
                         ((a.rec_s_base + s_rel + 1) % a.rec_stride) == 0;
        double* rp = rec ? a.rec_out + ((size_t)((a.rec_s_base + s_rel + 1) / a.rec_stride - 1) *
                                            a.rec_chains + chain) * n
                         : nullptr;
        // blocks of U coordinates per lane: all loads of a block are issued
        // before its stores (one load latency per block); one per block in
        // the single-kernel path, whose registers are spoken for
        constexpr int U = B > 1 ? kUpd : 1;
        for (int jb = 0; jb < n; jb += 64 * U) {
            double xv[U], dv[U];
#pragma unroll
            for (int e = 0; e < U; ++e) {
                const int j = jb + lane + 64 * e;
                xv[e] = j < n ? xw[j] : 0.0;
                dv[e] = j < n ? dr[j] : 0.0;
            }
#pragma unroll
            for (int e = 0; e < U; ++e) {
                const int j = jb + lane + 64 * e;
                if (j < n) {
                    const double xnew = __dadd_rn(xv[e], __dmul_rn(th, dv[e]));
                    xw[j] = xnew;
                    if (rec) rp[j] = xnew;
                    xo = fma(xv[e], xv[e], xo);
                    xn2 = fma(xnew, xnew, xn2);
                    finite = finite && isfinite(xnew);
                }
            }
        }
        xo = wave_sum(xo);
        xn2 = wave_sum(xn2);
        finite = __all(finite);
        if (!finite) fl |= kNonFinite;
        if (lane == 0) {
            const double dn = cs->dnorm[cl], at = fabs(th);
            const double us = (double)a.u_s;
            double E = cs->E[cl];
            if (a.rk > 0) {
                // the slack update's error, split like the screening bound:
                // |a| part into E, |a P U| part into F
                const double hn = cs->hnorm[cl], en = cs->enorm[cl];
                const double dx = 0x1.0p-36 * (hn + dn + *a.uF * en);
                E += at * (hn * (double)a.eps_g + dx + 2.0 * us * dn);
                cs->F[cl] += at * en * (double)a.eps_g;
            } else {
                E += at * dn * ((double)a.eps_g + 2.0 * us);
            }
            E += 2.0 * u64 * (sqrt(xo) + at * dn);
            E += us * (1.0 + 0x1.0p-20) * sqrt(xn2);
            cs->E[cl] = E;
            cs->theta[cl] = th;
            cs->flags[cl] |= fl;
        }
    }
}

// ---------------------------------------------------------------------------
// Phase E: exact FP64 slack s = b - A X for the 16 walks (matrix cores).
// ---------------------------------------------------------------------------
template <int P>
__device__ void recompute_slack(const StepArgs& a, ChainLds* cs, unsigned char* big, int tile,
                                int c0)
{
    typedef typename Op<P>::state_t st_t;
    constexpr bool F64 = Op<P>::f64;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int g = lane >> 4, c = lane & 15;
    const int n = a.n, lda = a.lda, Q = a.m_pad >> 4;
    st_t* S = (st_t*)a.S;
    double* Xt = (double*)big;
    const int ld = x_ld(lda);
    __syncthreads();
    for (int item = tid; item < kChainTile * lda; item += kThreads) {
        int cl = item / lda, j = item - cl * lda;
        int chain = c0 + cl;
        Xt[cl * ld + j] = (chain < a.z && j < n) ? a.X[(size_t)chain * lda + j] : 0.0;
    }
    __syncthreads();
    // drift coefficient after an exact recompute
    for (int cl = wave; cl < kChainTile; cl += kWaves) {
        double v = 0.0;
        for (int j = lane; j < n; j += 64) v = fma(Xt[cl * ld + j], Xt[cl * ld + j], v);
        v = wave_sum(v);
        if (lane == 0)
            cs->E[cl] = ((double)a.u_s * (1.0 + 0x1.0p-20) + (2.0 * n + 4.0) * 0x1.0p-53) * sqrt(v);
    }
    const bool active = (c0 + c) < a.z;
    int fl = 0;
    for (int row0 = wave * kRowGroup; row0 < a.m_pad; row0 += kWaves * kRowGroup) {
        f64x4 acc[4] = {{0, 0, 0, 0}, {0, 0, 0, 0}, {0, 0, 0, 0}, {0, 0, 0, 0}};
        for (int k0 = 0; k0 < lda; k0 += 16) {
            const double2* bp = (const double2*)(Xt + c * ld + k0 + 4 * g);
            double2 b0 = bp[0], b1 = bp[1];
#pragma unroll
            for (int rb = 0; rb < 4; ++rb) {
                const double2* ap = (const double2*)(a.A64 + (size_t)(row0 + 16 * rb + c) * lda + k0 + 4 * g);
                double2 a0 = ap[0], a1 = ap[1];
                acc[rb] = mma_f64(a0.x, b0.x, acc[rb]);
                acc[rb] = mma_f64(a0.y, b0.y, acc[rb]);
                acc[rb] = mma_f64(a1.x, b1.x, acc[rb]);
                acc[rb] = mma_f64(a1.y, b1.y, acc[rb]);
            }
        }
#pragma unroll
        for (int rb = 0; rb < 4; ++rb) {
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = row0 + 16 * rb + out_row<true>(g, r);
                const double bi = a.b64[row];
                const double s = bi - acc[rb][r];
                if (active && row < a.m) {
                    if (!(s > 0.0)) fl |= kNotInterior;
                    if (s < -1e-12 * fmax(1.0, fabs(bi))) fl |= kInfeasible;
                }
                S[frag_index<F64>(tile, Q, row, c)] = (st_t)s;
            }
        }
    }
    if (fl) atomicOr(&cs->flags[c], fl);
    __syncthreads();
}

// All `a.steps` steps of walk tile `tile` of one problem (the slack, the last
// screening product and the lower bounds stay in HBM between steps).
template <int P>
__device__ void run_tile(const StepArgs& a, unsigned char* smem, int tile)
{
    unsigned char* big = smem;
    ChainLds* cs = (ChainLds*)(smem + big_bytes(a.lda));
    const int tid = threadIdx.x;
    const int c0 = tile * kChainTile;

    if (tid < kChainTile) {
        const int chain = c0 + tid;
        cs->theta[tid] = a.theta[chain];
        cs->E[tid] = a.E[chain];
        cs->flags[tid] = 0;
    }
    if (tid == 0) cs->exact = 0;
    __syncthreads();

    int pending = a.pending0, T = a.T0, since = a.since0;
    if (a.recompute_first) {
        recompute_slack<P>(a, cs, big, tile, c0);
        pending = 0;
        T = 2;
        since = 0;
    }
    for (int s = 0; s < a.steps; ++s) {
        const uint64_t step = a.step0 + (uint64_t)s;
        if (tid < kChainTile) {
            cs->up[tid] = __float_as_uint(kInf);
            cs->um[tid] = __float_as_uint(kInf);
        }
        make_directions<false>(a, cs, c0, step);
        stage_operand<P>(a, big, c0);
        screen<P>(a, cs, big, tile, c0, pending, T);
        __syncthreads();
        exact_chords<P, 1>(a, cs, tile, c0, step, s, T, (double*)big, big_bytes(a.lda));
        __syncthreads();
        pending = 1;
        T += 1;
        since += 1;
        if (since >= a.R) {
            recompute_slack<P>(a, cs, big, tile, c0);
            pending = 0;
            T = 2;
            since = 0;
        }
    }
    __syncthreads();
    if (tid < kChainTile) {
        const int chain = c0 + tid;
        a.theta[chain] = cs->theta[tid];
        a.E[chain] = cs->E[tid];
        if (cs->flags[tid] && chain < a.z) atomicOr(&a.flags[chain], cs->flags[tid]);
    }
    if (tid == 0 && cs->exact) atomicAdd(&a.counters[0], cs->exact);
    __syncthreads();
}

template <int P>
__global__ __launch_bounds__(kThreads) void mhar_steps_kernel(StepArgs a)
{
    extern __shared__ __align__(16) unsigned char smem[];
    run_tile<P>(a, smem, blockIdx.x);
}

// Many problems in one persistent launch: workgroups take (problem, walk
// tile) units from a queue ordered by decreasing cost (longest processing
// time first) through a device counter, and leave when the queue is empty.
template <int P>
__global__ __launch_bounds__(kThreads) void mhar_batch_kernel(const StepArgs* __restrict__ descs,
                                                              const int2* __restrict__ units,
                                                              int nunits, unsigned* next)
{
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ int unit_lds;
    while (true) {
        if (threadIdx.x == 0) unit_lds = (int)atomicAdd(next, 1u);
        __syncthreads();
        const int u = unit_lds;
        __syncthreads();
        if (u >= nunits) break;
        const int2 w = units[u];
        const StepArgs a = descs[w.x];   // a private copy: no aliasing with the stores
        run_tile<P>(a, smem, w.y);
    }
}

// ---------------------------------------------------------------------------
// Tiled path for large problems (FP32 / BF16X3 screening).
//
// With one workgroup per 16 walks, every workgroup streams all of A each
// step, which bounds large problems by the A stream.  The tiled path splits a
// step into three kernels instead:
//   tiled_screen : G = A D as a GEMM over (128-row x 128-walk) tiles, two
//                  workgroups of 4 waves per CU, operands streamed by direct
//                  global-to-LDS loads through two stages, fused with the
//                  deferred slack update and the ratio bounds;
//                  per (64-row group, walk) it writes the least lower bound
//                  and the least upper bound of each chord end;
//   tiled_chords : per 16-walk tile, the chord-end bound as the minimum over
//                  the groups, the exact FP64 chord of the candidate rows,
//                  theta and the update (Phase D), then the next step's
//                  directions (Phase A) written to HBM as FP64 rows and as
//                  the matrix-core operand;
//   tiled_recompute: every R steps the exact slack b - A X as an FP64 GEMM.
// The arithmetic that decides a trajectory (directions, exact chords, theta,
// update) is the same code as the single-kernel path, so trajectories agree.
// ---------------------------------------------------------------------------
// LDS the chords kernel lends to the exact evaluation: 96 candidates and the
// x and d rows of 16 walks, 128 coordinates at a time
constexpr int kChordStageBytes = (96 + 2 * kChainTile) * (128 + 2) * 8;
constexpr int kTR = kScreenRows;   // rows per screening tile
constexpr int kTW = kScreenWalks;  // walks per screening tile
constexpr int kTK = 32;    // K per LDS stage

constexpr int kScreenThreads = 256;   // 4 waves, each a 64-row x 64-walk quarter of a tile
constexpr int kStageBytes = 32768;    // one K-step of both operands, in either format
constexpr int kChunksPerWave = kStageBytes / 1024 / (kScreenThreads / 64);   // 8

// A stage holds one K-step (32 columns) of the tile's 128 rows of A and 128
// walks of the direction operand in four planes of 128 rows x 64 bytes:
//   BF16X3: A hi | A lo | D hi | D lo (32 BF16 columns per row)
//   FP32:   A columns 0-15 | A columns 16-31 | D columns 0-15 | D columns 16-31
// filled by direct global-to-LDS loads: one load instruction writes 1 KB (64
// lanes x 16 bytes) of consecutive LDS, and each lane fetches the global 16
// bytes that belong in its slot.  Rows are not padded; the four 16-byte slots
// of row r are permuted by an XOR with (r >> 1) & 3, which measurements of
// ds_read_b128 on gfx950 show to be free of bank conflicts for the MFMA
// operand reads (16 rows at one slot), unlike row padding or an XOR with r.
constexpr int kPlaneBytes = 8192;
template <int P> struct TileFmt;
template <> struct TileFmt<kBF16X3> {
    static constexpr int per16 = 8;           // elements per 16-byte slot
};
template <> struct TileFmt<kFP32> {
    static constexpr int per16 = 4;
};
__device__ __forceinline__ int slot_swz(int row) { return (row >> 1) & 3; }

// Tile t of the launch for workgroup `bid`: workgroups are dealt round-robin to
// the 8 XCDs, so XCD x gets the contiguous tile range [x*per, (x+1)*per).
__device__ __forceinline__ int xcd_tile(int bid, int total)
{
    const int per = (total + 7) >> 3;
    return (bid & 7) * per + (bid >> 3);
}

// Tile t in groups of kTileGroup row blocks taken column by column, so that
// the tiles an XCD runs at once share a few row blocks of A and a few walk
// blocks of the direction operand in its L2.
constexpr int kTileGroup = 4;
__device__ __forceinline__ void tile_coords(int t, int nrb, int ncb, int& rb, int& cb)
{
    const int span = kTileGroup * ncb, first = t / span * kTileGroup;
    const int gsz = min(nrb - first, kTileGroup), r = t - t / span * span;
    rb = first + r % gsz;
    cb = r / gsz;
}

// Slack schedule of step s of a launch (s = 0 is the launch's first step):
// every step sets pending = 1, T += 1, since += 1, and an exact recompute
// after a step where since reaches R resets pending = 0, T = 2, since = 0.
__device__ __forceinline__ void sched_at(const StepArgs& a, int s, int& pending, int& T,
                                         bool& recompute_after)
{
    const int since = (a.since0 + s) % a.R;
    pending = (s == 0) ? a.pending0 : (since != 0);
    T = (a.since0 + s < a.R) ? a.T0 + s : 2 + since;
    recompute_after = since + 1 == a.R;
}

// Workgroup barrier that the compiler may not move memory accesses across and
// that does not itself wait for the stage loads in flight (wait_vm says which
// loads must have landed).
__device__ __forceinline__ void tile_barrier() { asm volatile("s_barrier" ::: "memory"); }
// 16 bytes from global memory to LDS byte address lds + 16 * lane (the LDS
// base is wave-uniform, in M0).  The instruction returns nothing to
// registers; its completion is counted by vmcnt like any load, and the
// "memory" clobber keeps the compiler from moving memory accesses across it.
__device__ __forceinline__ void load_to_lds(const void* src, unsigned lds)
{
    asm volatile("global_load_lds_dwordx4 %0, off" :: "v"(src), "{m0}"(lds) : "memory");
}

// One (128-row block rb, 128-walk block cb) tile of the screening GEMM and its epilogue.
// SPLIT: the contraction continues over the rk columns of A P U and eps
// (a learned covariance); a separate instantiation keeps the isotropic
// kernel's registers as they were.
template <int P, bool SPLIT>
__device__ void screen_tile(const StepArgs& a, int rb, int cb, int pending, int T)
{
    typedef TileFmt<P> F;
    __shared__ __align__(1024) unsigned char stage0[kStageBytes];
    __shared__ __align__(1024) unsigned char stage1[kStageBytes];
    constexpr int esz = 16 / F::per16;   // bytes per element
    const int R0 = rb * kTR, C0 = cb * kTW;
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);   // uniform: the stage loads' LDS base
    const int g = lane >> 4, c = lane & 15;
    const int wr = wave & 1, wc = wave >> 1;
    const int lda = a.lda;

    // wave w fills plane w: its chunk i (1 KB) holds rows 16 i .. 16 i + 15,
    // lane l the physical slot l % 4 = logical slot ^ slot_swz(row) of row
    // 16 i + l / 4.  Rows past the padded row count (walks past the padded
    // walk count) read the last one: their products are never stored.
    const bool a_side = wave < 2;
    const int half = wave & 1;   // BF16X3: hi / lo part; FP32: columns 0-15 / 16-31
    const unsigned char* src[kChunksPerWave];
    const size_t zl = (size_t)a.z_pad * lda;
#pragma unroll
    for (int i = 0; i < kChunksPerWave; ++i) {
        const int row = 16 * i + (lane >> 2);
        const int logical = (lane & 3) ^ slot_swz(row);
        const unsigned char* base;
        int grow;
        if (a_side) {
            grow = min(R0 + row, a.m_pad - 1);
            base = P == kBF16X3 ? (const unsigned char*)(half ? a.Alo : a.Ahi)
                                : (const unsigned char*)a.A32;
        } else {
            grow = min(C0 + row, a.z_pad - 1);
            base = P == kBF16X3 ? (const unsigned char*)((const __bf16*)a.Dop + (half ? zl : 0))
                                : (const unsigned char*)a.Dop;
        }
        const int col = P == kBF16X3 ? logical * F::per16 : 16 * half + logical * F::per16;
        src[i] = base + ((size_t)grow * lda + col) * esz;
    }
    const int nk = lda / kTK;
    // split screening: after the lda columns of A and the direction operand,
    // rk more columns of A P U and eps, stored with the same row stride, so
    // each source moves by one byte offset per operand and plane
    const int nk_all = SPLIT ? nk + a.rk / kTK : nk;
    auto retarget = [&]() __attribute__((always_inline)) {
        const unsigned char* from;
        const unsigned char* to;
        if (a_side) {
            from = P == kBF16X3 ? (const unsigned char*)(half ? a.Alo : a.Ahi)
                                : (const unsigned char*)a.A32;
            to = (const unsigned char*)a.AUop +
                 (P == kBF16X3 ? (size_t)half * a.m_pad * lda * esz : 0);
        } else {
            // eps and the direction operand share their layout (planes of z_pad x lda)
            from = (const unsigned char*)a.Dop;
            to = (const unsigned char*)a.Eop;
        }
#pragma unroll
        for (int i = 0; i < kChunksPerWave; ++i) src[i] += to - from;
    };
    // K-step k into a stage; K-steps are issued once each, in increasing order
    auto issue = [&](int k, unsigned char* stage) __attribute__((always_inline)) {
        if (SPLIT && k == nk) retarget();
        const size_t koff = (size_t)(k < nk ? k : k - nk) * kTK * esz;
        const unsigned dst = (unsigned)(size_t)stage + wave * kPlaneBytes;
#pragma unroll
        for (int i = 0; i < kChunksPerWave; ++i) load_to_lds(src[i] + koff, dst + i * 1024);
    };

    f32x4 acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = f32x4{0, 0, 0, 0};

    const bool wave_rows = R0 + wr * 64 < a.m_pad;
    const bool wave_live = wave_rows && C0 + wc * 64 < a.z_pad;
    // every operand read takes slot g of 16 consecutive rows; slot_swz(16 t + c) = slot_swz(c)
    const int slot = 16 * (g ^ slot_swz(c));
    auto compute = [&](const unsigned char* base) __attribute__((always_inline)) {
        if (!wave_live) return;
        const unsigned char* A0 = base;
        const unsigned char* A1 = base + kPlaneBytes;
        const unsigned char* D0 = base + 2 * kPlaneBytes;
        const unsigned char* D1 = base + 3 * kPlaneBytes;
        if (P == kBF16X3) {
            bf16x8 ah[4], al[4], bh[4], bl[4];
#pragma unroll
            for (int rt = 0; rt < 4; ++rt) {
                const int row = wr * 64 + rt * 16 + c;
                ah[rt] = *(const bf16x8*)(A0 + row * 64 + slot);
                al[rt] = *(const bf16x8*)(A1 + row * 64 + slot);
            }
#pragma unroll
            for (int ct = 0; ct < 4; ++ct) {
                const int w = wc * 64 + ct * 16 + c;
                bh[ct] = *(const bf16x8*)(D0 + w * 64 + slot);
                bl[ct] = *(const bf16x8*)(D1 + w * 64 + slot);
            }
#pragma unroll
            for (int rt = 0; rt < 4; ++rt)
#pragma unroll
                for (int ct = 0; ct < 4; ++ct) {
                    acc[rt][ct] = mma_bf16(al[rt], bh[ct], acc[rt][ct]);
                    acc[rt][ct] = mma_bf16(ah[rt], bl[ct], acc[rt][ct]);
                    acc[rt][ct] = mma_bf16(ah[rt], bh[ct], acc[rt][ct]);
                }
        } else {
            float4 av[4][2], bv[4][2];
#pragma unroll
            for (int rt = 0; rt < 4; ++rt) {
                const int row = wr * 64 + rt * 16 + c;
                av[rt][0] = *(const float4*)(A0 + row * 64 + slot);
                av[rt][1] = *(const float4*)(A1 + row * 64 + slot);
            }
#pragma unroll
            for (int ct = 0; ct < 4; ++ct) {
                const int w = wc * 64 + ct * 16 + c;
                bv[ct][0] = *(const float4*)(D0 + w * 64 + slot);
                bv[ct][1] = *(const float4*)(D1 + w * 64 + slot);
            }
            // MFMA e takes column 16 (e >> 2) + 4 g + (e & 3) from lane group g,
            // for A and D alike
#pragma unroll
            for (int e = 0; e < 8; ++e)
#pragma unroll
                for (int rt = 0; rt < 4; ++rt)
#pragma unroll
                    for (int ct = 0; ct < 4; ++ct)
                        acc[rt][ct] = mma_f32((&av[rt][e >> 2].x)[e & 3],
                                              (&bv[ct][e >> 2].x)[e & 3], acc[rt][ct]);
        }
    };

    // slack and last product of this wave's entries, two walk tiles (a half)
    // at a time (only this tile writes these entries)
    const float* S = (const float*)a.S;
    const float* Gb = (const float*)a.G;
    const int Q = a.m_pad >> 4;
    auto load_half = [&](int half, float (*sv)[4][4], float (*gp)[4][4]) __attribute__((always_inline)) {
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int cbase = C0 + wc * 64 + (2 * half + h) * 16;
            const int tile = min(cbase, a.z_pad - kChainTile) / kChainTile;
#pragma unroll
            for (int rt = 0; rt < 4; ++rt) {
                // rows 4g .. 4g + 3 of the 16-row block: one 16-byte run
                const size_t idx = frag_index<false>(tile, Q, R0 + wr * 64 + rt * 16 + 4 * g, c);
                const float4 s4 = wave_rows ? *(const float4*)(S + idx) : make_float4(0, 0, 0, 0);
                const float4 g4 = (wave_rows && pending) ? *(const float4*)(Gb + idx)
                                                          : make_float4(0, 0, 0, 0);
                sv[h][rt][0] = s4.x;
                sv[h][rt][1] = s4.y;
                sv[h][rt][2] = s4.z;
                sv[h][rt][3] = s4.w;
                gp[h][rt][0] = g4.x;
                gp[h][rt][1] = g4.y;
                gp[h][rt][2] = g4.z;
                gp[h][rt][3] = g4.w;
            }
        }
    };
    // half 0 of this wave's slack and last product, issued right after the
    // last stage load so that it lands during the last two K-steps: exactly
    // 16 load instructions (rows clamped, G read even without a pending
    // update), which the waits of those K-steps count
    auto load_early = [&](float (*sv)[4][4], float (*gp)[4][4]) __attribute__((always_inline)) {
        const int rbase = min(R0 + wr * 64, a.m_pad - 64);
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int cbase = C0 + wc * 64 + h * 16;
            const int tile = min(cbase, a.z_pad - kChainTile) / kChainTile;
#pragma unroll
            for (int rt = 0; rt < 4; ++rt) {
                const size_t idx = frag_index<false>(tile, Q, rbase + rt * 16 + 4 * g, c);
                const float4 s4 = *(const float4*)(S + idx);
                const float4 g4 = *(const float4*)(Gb + idx);
                sv[h][rt][0] = s4.x;
                sv[h][rt][1] = s4.y;
                sv[h][rt][2] = s4.z;
                sv[h][rt][3] = s4.w;
                gp[h][rt][0] = g4.x;
                gp[h][rt][1] = g4.y;
                gp[h][rt][2] = g4.z;
                gp[h][rt][3] = g4.w;
            }
        }
    };
    // the epilogue's per-row and per-walk terms, once per tile into LDS
    // (read by every wave and lane that needs them): row norms, |b| and the
    // split operand's row norms; per walk the product's error coefficients
    // (ed: |a| part, ed2: |a P U| part), the slack drifts (Ek, Fk) and theta
    __shared__ float row_na[kTR], row_b[kTR], row_nau[kTR];
    __shared__ float walk_ed[kTW], walk_ed2[kTW], walk_E[kTW], walk_F[kTW], walk_th[kTW];
    {
        const int i = tid & (kTR - 1);
        if (tid < kTR) {
            const int row = R0 + i;
            const bool ok = row < a.m_pad;
            row_na[i] = ok ? a.rownorm[row] : 0.0f;
            row_b[i] = ok ? a.absb[row] : 0.0f;
            row_nau[i] = (SPLIT && a.rk > 0 && ok) ? a.aun[row] : 0.0f;
        } else {
            const int chain = C0 + i;
            const bool ok = chain < a.z_pad, active = chain < a.z;
            float ed = 0.0f, ed2 = 0.0f, Fk = 0.0f, Ek = 0.0f, th = 0.0f;
            if (ok) {
                if (SPLIT && a.rk > 0) {
                    // |g_hat - g| <= eps_g (|a| |h| + |a P U| |eps|) + |a| dx
                    const double hn = a.hn[chain], en = a.en[chain];
                    const double dx = 0x1.0p-36 * (hn + a.dn[chain] + *a.uF * en);
                    ed = active ? (float)(hn * (double)a.eps_g + dx) * kHighGrow + 1e-30f : 0.0f;
                    ed2 = active ? (float)(en * (double)a.eps_g) * kHighGrow : 0.0f;
                    Fk = (float)a.F[chain] * kHighGrow;
                } else {
                    ed = active ? (float)(a.dn[chain] * (double)a.eps_g) * kHighGrow + 1e-30f : 0.0f;
                }
                Ek = (float)a.E[chain] * kHighGrow;
                th = (float)a.theta[chain];
            }
            walk_ed[i] = ed;
            walk_ed2[i] = ed2;
            walk_F[i] = Fk;
            walk_E[i] = Ek;
            walk_th[i] = th;
        }
        wait_lds();   // the main loop's barriers publish them
    }
    // two stages: K-step k + 1 lands while K-step k is multiplied; K-step
    // k + 2 is issued into the stage K-step k has left
    float sv0[2][4][4], gp0[2][4][4];
    const int k_sg = nk_all - 3;   // the K-step whose stage issue is the last
    auto kstep = [&](int k, unsigned char* stage) __attribute__((always_inline)) {
        if (k > k_sg) {   // the 16 early loads are younger than this K-step's stage loads
            if (k + 1 < nk_all) wait_vm<kChunksPerWave + 16>();
            else wait_vm<16>();
        } else {
            if (k + 1 < nk_all) wait_vm<kChunksPerWave>();
            else wait_vm<0>();
        }
        tile_barrier();   // every wave's loads of K-step k have landed
        compute(stage);
        wait_lds();
        tile_barrier();   // every wave is done reading the stage
        if (k + 2 < nk_all) issue(k + 2, stage);
        if (k == k_sg) load_early(sv0, gp0);
    };
    issue(0, stage0);
    if (nk_all > 1) issue(1, stage1);
    if (k_sg < 0) load_early(sv0, gp0);
    for (int k = 0; k < nk_all; k += 2) {
        kstep(k, stage0);
        if (k + 1 < nk_all) kstep(k + 1, stage1);
    }
    if (!wave_rows) return;

    // fused epilogue: deferred slack update, new product, interval bounds
    float* Sw = (float*)a.S;
    float* Gw = (float*)a.G;
    const int ngroups = a.m_pad / kRowGroup;
    const int grp = (R0 + wr * 64) / kRowGroup;
    const float bscale = a.u_s * (float)T * kHighGrow;
    // half 0 was loaded during the last K-steps; the isotropic kernel issues
    // half 1's loads before the arithmetic (they land while half 0 is
    // processed), the split kernel, short of registers, after half 0
    float sv1[2][4][4], gp1[2][4][4];
    if (!SPLIT) load_half(1, sv1, gp1);
#pragma unroll
    for (int half = 0; half < 2; ++half) {
        if (SPLIT && half == 1) load_half(1, sv1, gp1);
        float (*sv)[4][4] = half ? sv1 : sv0;
        float (*gp)[4][4] = half ? gp1 : gp0;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int ct = 2 * half + h;
            const int cbase = C0 + wc * 64 + ct * 16;
            if (cbase >= a.z_pad) break;
            const int tile = cbase / kChainTile;
            const int lw = wc * 64 + ct * 16 + c;   // walk within the tile
            const bool split = SPLIT && a.rk > 0;
            const float ed = walk_ed[lw], ed2 = walk_ed2[lw], Fk = walk_F[lw];
            const float Ek = walk_E[lw], th = walk_th[lw];
            float up = kInf, um = kInf, lp = kInf, lm = kInf;
            // the updated slack in place; then the stores of this walk
            // tile's 64 rows back to back, so that each walk's 256-byte run of
            // S and of G reaches the cache whole (no partial lines)
#pragma unroll
            for (int rt = 0; rt < 4; ++rt)
#pragma unroll
                for (int r = 0; r < 4; ++r)
                    if (pending) sv[h][rt][r] = fmaf(-th, gp[h][rt][r], sv[h][rt][r]);
            if (pending) {
#pragma unroll
                for (int rt = 0; rt < 4; ++rt) {
                    const size_t idx = frag_index<false>(tile, Q, R0 + wr * 64 + rt * 16 + 4 * g, c);
                    *(float4*)(Sw + idx) = make_float4(sv[h][rt][0], sv[h][rt][1], sv[h][rt][2],
                                                       sv[h][rt][3]);
                }
            }
#pragma unroll
            for (int rt = 0; rt < 4; ++rt) {
                const size_t idx = frag_index<false>(tile, Q, R0 + wr * 64 + rt * 16 + 4 * g, c);
                *(float4*)(Gw + idx) = make_float4(acc[rt][ct][0], acc[rt][ct][1], acc[rt][ct][2],
                                                   acc[rt][ct][3]);
            }
#pragma unroll
            for (int rt = 0; rt < 4; ++rt) {
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int lr = wr * 64 + rt * 16 + out_row<false>(g, r);   // row within the tile
                    const float gv = acc[rt][ct][r];
                    const float s_ = sv[h][rt][r];
                    const float na = row_na[lr];
                    float dl = fmaf(na, Ek, fmaf(bscale, row_b[lr], 1e-30f));
                    float e = na * ed;
                    if (split) {
                        const float nau = row_nau[lr];
                        dl = fmaf(nau, Fk, dl);
                        e = fmaf(nau, ed2, e);
                    }
                    float lo_p, hi_p, lo_m, hi_m;
                    ratio_bounds(s_, gv, dl, e, lo_p, hi_p, lo_m, hi_m);
                    up = fminf(up, hi_p);
                    um = fminf(um, hi_m);
                    lp = fminf(lp, lo_p);
                    lm = fminf(lm, lo_m);
                }
            }
#pragma unroll
            for (int o = 16; o <= 32; o <<= 1) {
                up = fminf(up, __shfl_xor(up, o, 64));
                um = fminf(um, __shfl_xor(um, o, 64));
                lp = fminf(lp, __shfl_xor(lp, o, 64));
                lm = fminf(lm, __shfl_xor(lm, o, 64));
            }
            if (g == 0) {
                const size_t base = ((size_t)tile * ngroups + grp) * 2 * kChainTile + c;
                a.L[base] = lp;
                a.L[base + kChainTile] = lm;
                a.Ug[base] = up;
                a.Ug[base + kChainTile] = um;
            }
        }
    }
}

template <int P, bool SPLIT>
__global__ __launch_bounds__(kScreenThreads, 2) void tiled_screen_kernel(StepArgs a, int pending, int T)
{
    const int nrb = (a.m_pad + kTR - 1) / kTR, ncb = (a.z_pad + kTW - 1) / kTW;
    const int t = xcd_tile(blockIdx.x, nrb * ncb);
    if (t >= nrb * ncb) return;
    int rb, cb;
    tile_coords(t, nrb, ncb, rb, cb);
    screen_tile<P, SPLIT>(a, rb, cb, pending, T);
}

// Screening tiles of many problems: entry (problem, rb, cb) per workgroup
// (SPLIT when some problem of the batch has a learned covariance).
template <int P, bool SPLIT>
__global__ __launch_bounds__(kScreenThreads, 2) void grouped_screen_kernel(const StepArgs* __restrict__ descs,
                                                                           const int4* __restrict__ tiles,
                                                                           int ntiles, int s)
{
    if ((int)blockIdx.x >= ntiles) return;
    const int4 e = tiles[blockIdx.x];
    const StepArgs a = descs[e.x];   // a private copy: no aliasing with the stores
    int pending, T;
    bool due;
    sched_at(a, s, pending, T, due);
    screen_tile<P, SPLIT>(a, e.y, e.z, pending, T);
}

// Chords of step `step` for one 16-walk tile (do_chords), then the directions
// of step `dir_step` (gen_dirs) as FP64 rows, norms and the screening operand.
template <int P>
__device__ void chords_tile(const StepArgs& a, int tile, uint64_t step, int s_rel, int T,
                            int do_chords, int gen_dirs, uint64_t dir_step)
{
    __shared__ ChainLds cs_lds;
    __shared__ __align__(16) unsigned char stage_lds[kChordStageBytes];
    ChainLds* cs = &cs_lds;
    const int tid = threadIdx.x;
    const int c0 = tile * kChainTile;
    const int lda = a.lda, n = a.n;
    if (do_chords) {
        const int ngroups = a.m_pad / kRowGroup;
        if (tid < kChainTile) {
            const int chain = c0 + tid;
            cs->theta[tid] = a.theta[chain];
            cs->E[tid] = a.E[chain];
            cs->dnorm[tid] = a.dn[chain];
            if (a.rk > 0) {
                cs->hnorm[tid] = a.hn[chain];
                cs->enorm[tid] = a.en[chain];
                cs->F[tid] = a.F[chain];
            }
            cs->flags[tid] = 0;
            cs->up[tid] = __float_as_uint(kInf);
            cs->um[tid] = __float_as_uint(kInf);
        }
        if (tid == 0) cs->exact = 0;
        __syncthreads();
        {
            // chord-end bounds: minimum of the per-group upper bounds
            const int c = tid & 15;
            const float* Ut = a.Ug + (size_t)tile * ngroups * 2 * kChainTile;
            float up = kInf, um = kInf;
            for (int q = tid >> 4; q < ngroups; q += kThreads / kChainTile) {
                up = fminf(up, Ut[(q * 2 + 0) * kChainTile + c]);
                um = fminf(um, Ut[(q * 2 + 1) * kChainTile + c]);
            }
            up = fminf(up, __shfl_xor(up, 16, 64));
            up = fminf(up, __shfl_xor(up, 32, 64));
            um = fminf(um, __shfl_xor(um, 16, 64));
            um = fminf(um, __shfl_xor(um, 32, 64));
            if ((tid & 63) < kChainTile) {
                atomicMin(&cs->up[c], __float_as_uint(up));
                atomicMin(&cs->um[c], __float_as_uint(um));
            }
        }
        __syncthreads();
        exact_chords<P, 3>(a, cs, tile, c0, step, s_rel, T, (double*)stage_lds, kChordStageBytes);
        __syncthreads();
        if (tid < kChainTile) {
            const int chain = c0 + tid;
            a.theta[chain] = cs->theta[tid];
            a.E[chain] = cs->E[tid];
            if (a.rk > 0) a.F[chain] = cs->F[tid];
            if (cs->flags[tid] && chain < a.z) atomicOr(&a.flags[chain], cs->flags[tid]);
        }
        if (tid == 0 && cs->exact) atomicAdd(&a.counters[0], cs->exact);
        __syncthreads();
    }
    if (!gen_dirs) return;
    make_directions<true>(a, cs, c0, dir_step);
    __syncthreads();
    // norms and the screening operand in one pass, 32 lanes per walk: the
    // operand is the direction, or with the split screening its isotropic
    // part (the low-rank part's operand was written with the draws)
    {
        const int cl = tid >> 5, t = tid & 31, chain = c0 + cl;
        const bool live = chain < a.z, split = a.rk > 0;
        const double* dr = a.D + (size_t)chain * lda;
        const double* hr = split ? a.Hs + (size_t)chain * lda : dr;
        double v = 0.0, w = 0.0;
        for (int jb = 0; jb < lda; jb += 32 * kUpd) {
            double dv[kUpd], hv[kUpd];
#pragma unroll
            for (int e = 0; e < kUpd; ++e) {
                const int j = jb + t + 32 * e;
                const bool in = live && j < n;
                dv[e] = in ? dr[j] : 0.0;
                hv[e] = (in && split) ? hr[j] : dv[e];
            }
#pragma unroll
            for (int e = 0; e < kUpd; ++e) {
                v = fma(dv[e], dv[e], v);
                if (split) w = fma(hv[e], hv[e], w);
            }
#pragma unroll
            for (int e = 0; e < kUpd; ++e) {
                const int j = jb + t + 32 * e;
                if (j < lda) {
                    const size_t o = (size_t)chain * lda + j;
                    const float op = (float)hv[e];   // zero past n and for idle walks
                    if (P == kBF16X3) {
                        __bf16 hi, lo;
                        split_bf16(op, hi, lo);
                        ((__bf16*)a.Dop)[o] = hi;
                        ((__bf16*)a.Dop)[(size_t)a.z_pad * lda + o] = lo;
                    } else {
                        ((float*)a.Dop)[o] = op;
                    }
                }
            }
        }
#pragma unroll
        for (int off = 16; off >= 1; off >>= 1) {
            v += __shfl_xor(v, off, 64);
            w += __shfl_xor(w, off, 64);
        }
        if (t == 0) {
            cs->dnorm[cl] = sqrt(v);
            cs->hnorm[cl] = sqrt(w);
        }
    }
    __syncthreads();
    if (tid < kChainTile) {
        a.dn[c0 + tid] = cs->dnorm[tid];
        if (a.rk > 0) {
            a.hn[c0 + tid] = cs->hnorm[tid];
            a.en[c0 + tid] = cs->enorm[tid];
        }
    }
}

// Step counter of graph replays: set before the first replay, advanced by
// the last node of each replay.
__global__ void step_counter_kernel(uint64_t* ctr, uint64_t value, int add)
{
    if (threadIdx.x == 0) *ctr = add ? *ctr + value : value;
}

// Directions of global step `step` for the tiled path, one workgroup of 4
// waves per walk (isotropic directions): draws, projection, norm and the
// operand row.  Draws and projection follow the operation order of
// make_directions (the projection's A_eq h as lane-strided FMA chains and a
// wave reduction), so the directions are bitwise those the chords kernel
// would make (the norm, which only scales certified error terms, may differ
// in its last bits).  With one workgroup per walk instead of per 16 walks,
// small walk counts still fill the device.
constexpr int kDirThreads = 256;
template <int P>
__global__ __launch_bounds__(kDirThreads) void tiled_dirs_kernel(StepArgs a, uint64_t step)
{
    constexpr int kDW = kDirThreads / 64;
    if (a.step_dev) step += *a.step_dev;
    __shared__ double y[kMaxMeq];
    __shared__ double part[kDW];
    const int chain = blockIdx.x;   // < z_pad
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int n = a.n, lda = a.lda;
    const bool live = chain < a.z;
    double* drow = a.D + (size_t)chain * lda;
    const size_t o0 = (size_t)chain * lda;
    // operand element j of this walk
    auto put_op = [&](int j, double v) __attribute__((always_inline)) {
        if (P == kBF16X3) {
            __bf16 hi, lo;
            split_bf16((float)v, hi, lo);
            ((__bf16*)a.Dop)[o0 + j] = hi;
            ((__bf16*)a.Dop)[(size_t)a.z_pad * lda + o0 + j] = lo;
        } else {
            ((float*)a.Dop)[o0 + j] = (float)v;
        }
    };
    // without equalities the draws are the direction: the row, its operand
    // and its squared norm come straight from registers
    const bool direct = a.m_eq == 0;
    double v2 = 0.0;
    if (live) {
        const int npairs = (n + 1) >> 1;
        for (int p = tid; p < npairs; p += kDirThreads) {
            Block4 w = stream_block(a.seed, kTagDir, a.chain_offset + (uint32_t)chain, step, (uint32_t)p);
            double ev, od;
            gauss_pair(w, ev, od);
            const bool has_od = 2 * p + 1 < n;
            drow[2 * p] = ev;
            if (has_od) drow[2 * p + 1] = od;
            if (direct) {
                v2 = fma(ev, ev, v2);
                put_op(2 * p, ev);
                if (has_od) {
                    v2 = fma(od, od, v2);
                    put_op(2 * p + 1, od);
                }
            }
        }
    }
    if (live && !direct) {
        __syncthreads();
        for (int p = wave; p < a.m_eq; p += kDW) {
            double v = lane_dot(a.Aeq + (size_t)p * lda, drow, n, lane);
            v = wave_sum(v);
            if (lane == 0) y[p] = v;
        }
        __syncthreads();
        for (int j = tid; j < n; j += kDirThreads) {
            double v = drow[j];
            for (int p = 0; p < a.m_eq; ++p) v = fma(-a.WT[(size_t)p * lda + j], y[p], v);
            drow[j] = v;
            v2 = fma(v, v, v2);
            put_op(j, v);
        }
    }
    // operand padding past n, and the whole row of an idle walk
    for (int j = (live ? n : 0) + tid; j < lda; j += kDirThreads) put_op(j, 0.0);
    v2 = wave_sum(v2);
    if (lane == 0) part[wave] = v2;
    __syncthreads();
    if (tid == 0) {
        double t = 0.0;
        for (int w = 0; w < kDW; ++w) t += part[w];
        a.dn[chain] = sqrt(t);
    }
}

template <int P>
__global__ __launch_bounds__(kThreads) void tiled_chords_kernel(StepArgs a, uint64_t step,
                                                                int s_rel, int T, int do_chords,
                                                                int gen_dirs, uint64_t dir_step)
{
    if (a.step_dev) {
        const uint64_t base = *a.step_dev;
        step += base;
        dir_step += base;
    }
    chords_tile<P>(a, blockIdx.x, step, s_rel, T, do_chords, gen_dirs, dir_step);
}

// Chords (and next directions) of many problems: entry (problem, 16-walk tile).
template <int P>
__global__ __launch_bounds__(kThreads) void grouped_chords_kernel(const StepArgs* __restrict__ descs,
                                                                  const int2* __restrict__ units,
                                                                  int nunits, int s, int do_chords,
                                                                  int gen_dirs)
{
    if ((int)blockIdx.x >= nunits) return;
    const int2 u = units[blockIdx.x];
    const StepArgs a = descs[u.x];   // a private copy: no aliasing with the stores
    int pending, T;
    bool due;
    sched_at(a, s, pending, T, due);
    const uint64_t step = a.step0 + (uint64_t)s;
    chords_tile<P>(a, u.y, step, s, T, do_chords, gen_dirs, do_chords ? step + 1 : step);
}

// Exact FP64 slack s = b - A X over (128-row x 128-walk) tiles on the FP64
// matrix cores, stored in the screening layout; workgroups of the first row
// block also reset the drift coefficient of their walks.
constexpr int kRR = kRecRows, kRW = kRecWalks, kRK = 16;
constexpr int kRecThreads = 256;   // 4 waves, each 64 rows x 64 walks; two workgroups per CU
constexpr int kRecWaves = kRecThreads / 64;
constexpr int kRRowBytes = kRK * 8 + 16;
constexpr int kRStage = (kRR + kRW) * kRRowBytes;

__device__ void recompute_tile(const StepArgs& a, int rb, int cb, unsigned char* smem)
{
    constexpr int kChunkRow = kRK * 8 / 16;                 // 8
    constexpr int kAChunks = kRR * kChunkRow;               // 2048
    constexpr int kPer = (kRR + kRW) * kChunkRow / kRecThreads;  // 8
    static_assert((kRR + kRW) * kChunkRow % kRecThreads == 0, "chunk split");
    static_assert(kRR == 128 && kRW == 128, "wave layout: 2 x 2 waves of 64 rows x 64 walks");
    const int R0 = rb * kRR, C0 = cb * kRW;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int g = lane >> 4, c = lane & 15;
    const int wr = wave & 1, wc = wave >> 1;   // 64 rows x 64 walks per wave
    const int lda = a.lda, n = a.n;

    if (rb == 0) {
        // drift coefficient after an exact recompute (one wave per walk)
        for (int w = wave; w < kRW; w += kRecWaves) {
            const int chain = C0 + w;
            if (chain >= a.z_pad) break;
            double v = 0.0;
            // blocks of 16 coordinates per lane, all loads of a block in flight
            for (int jb = 0; jb < n; jb += 64 * 16) {
                double x[16];
#pragma unroll
                for (int e = 0; e < 16; ++e) {
                    const int j = jb + lane + 64 * e;
                    x[e] = j < n ? a.X[(size_t)chain * lda + j] : 0.0;
                }
#pragma unroll
                for (int e = 0; e < 16; ++e) v = fma(x[e], x[e], v);
            }
            v = wave_sum(v);
            if (lane == 0) {
                a.E[chain] = ((double)a.u_s * (1.0 + 0x1.0p-20) + (2.0 * n + 4.0) * 0x1.0p-53) * sqrt(v);
                if (a.rk > 0) a.F[chain] = 0.0;
            }
        }
    }

    const double* src[kPer];
    int dst[kPer];
    bool ok[kPer];
#pragma unroll
    for (int i = 0; i < kPer; ++i) {
        const int u = tid + i * kRecThreads;
        if (u < kAChunks) {
            const int row = u / kChunkRow, part = u - row * kChunkRow;
            ok[i] = R0 + row < a.m_pad;
            src[i] = a.A64 + (size_t)(ok[i] ? R0 + row : 0) * lda + part * 2;
            dst[i] = row * kRRowBytes + part * 16;
        } else {
            const int v = u - kAChunks;
            const int row = v / kChunkRow, part = v - row * kChunkRow;
            ok[i] = C0 + row < a.z_pad;
            src[i] = a.X + (size_t)(ok[i] ? C0 + row : 0) * lda + part * 2;
            dst[i] = (kRR + row) * kRRowBytes + part * 16;
        }
    }
    uint4 buf[kPer];
    auto fetch = [&](int k0) __attribute__((always_inline)) {
#pragma unroll
        for (int i = 0; i < kPer; ++i)
            buf[i] = ok[i] ? *(const uint4*)(src[i] + k0) : make_uint4(0, 0, 0, 0);
    };
    auto deposit = [&](int stage) __attribute__((always_inline)) {
        unsigned char* base = smem + stage * kRStage;
#pragma unroll
        for (int i = 0; i < kPer; ++i) *(uint4*)(base + dst[i]) = buf[i];
    };

    f64x4 acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = f64x4{0, 0, 0, 0};
    const bool wave_rows = R0 + wr * 64 < a.m_pad;
    const int nk = lda / kRK;
    fetch(0);
    deposit(0);
    __syncthreads();
    for (int kt = 0; kt < nk; ++kt) {
        if (kt + 1 < nk) fetch((kt + 1) * kRK);
        const unsigned char* base = smem + (kt & 1) * kRStage;
        if (wave_rows) {
            double2 av[4][2], bv[4][2];
#pragma unroll
            for (int rt = 0; rt < 4; ++rt) {
                const unsigned char* p = base + (wr * 64 + rt * 16 + c) * kRRowBytes + 32 * g;
                av[rt][0] = *(const double2*)p;
                av[rt][1] = *(const double2*)(p + 16);
            }
#pragma unroll
            for (int ct = 0; ct < 4; ++ct) {
                const unsigned char* p = base + (kRR + wc * 64 + ct * 16 + c) * kRRowBytes + 32 * g;
                bv[ct][0] = *(const double2*)p;
                bv[ct][1] = *(const double2*)(p + 16);
            }
            // MFMA i takes K index 4g + i from lane group g, for A and X alike
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int rt = 0; rt < 4; ++rt)
#pragma unroll
                    for (int ct = 0; ct < 4; ++ct)
                        acc[rt][ct] = mma_f64((&av[rt][i >> 1].x)[i & 1],
                                              (&bv[ct][i >> 1].x)[i & 1], acc[rt][ct]);
        }
        if (kt + 1 < nk) deposit((kt + 1) & 1);
        __syncthreads();
    }
    if (!wave_rows) return;
    float* S = (float*)a.S;
    const int Q = a.m_pad >> 4;
#pragma unroll
    for (int ct = 0; ct < 4; ++ct) {
        const int cbase = C0 + wc * 64 + ct * 16;
        if (cbase >= a.z_pad) break;
        const int tile = cbase / kChainTile, chain = cbase + c;
        const bool active = chain < a.z;
        int fl = 0;
#pragma unroll
        for (int rt = 0; rt < 4; ++rt) {
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = R0 + wr * 64 + rt * 16 + out_row<true>(g, r);
                const double bi = a.b64[row];
                const double s = bi - acc[rt][ct][r];
                if (active && row < a.m) {
                    if (!(s > 0.0)) fl |= kNotInterior;
                    if (s < -1e-12 * fmax(1.0, fabs(bi))) fl |= kInfeasible;
                }
                S[frag_index<false>(tile, Q, row, c)] = (float)s;
            }
        }
        fl |= __shfl_xor(fl, 16, 64);
        fl |= __shfl_xor(fl, 32, 64);
        if (g == 0 && fl) atomicOr(&a.flags[chain], fl);
    }
}

__global__ __launch_bounds__(kRecThreads, 2) void tiled_recompute_kernel(StepArgs a)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const int nrb = (a.m_pad + kRR - 1) / kRR, ncb = (a.z_pad + kRW - 1) / kRW;
    const int t = xcd_tile(blockIdx.x, nrb * ncb);
    if (t >= nrb * ncb) return;
    recompute_tile(a, t / ncb, t % ncb, smem);
}

// Recompute tiles of many problems: entry (problem, rb, cb).  first != 0: the
// problems flagged recompute_first, before the launch's first step; else the
// problems whose schedule has a recompute after step s.
__global__ __launch_bounds__(kRecThreads, 2) void grouped_recompute_kernel(const StepArgs* __restrict__ descs,
                                                                     const int4* __restrict__ tiles,
                                                                     int ntiles, int s, int first)
{
    extern __shared__ __align__(16) unsigned char smem[];
    if ((int)blockIdx.x >= ntiles) return;
    const int4 e = tiles[blockIdx.x];
    const StepArgs a = descs[e.x];   // a private copy: no aliasing with the stores
    bool run;
    if (first) {
        run = a.recompute_first != 0;
    } else {
        int pending, T;
        sched_at(a, s, pending, T, run);
    }
    if (!run) return;
    recompute_tile(a, e.y, e.z, smem);
}

// ---------------------------------------------------------------------------
// One-time setup kernels
// ---------------------------------------------------------------------------

// FP64 copy with padding, operand form, row norms and |b| (both rounded up).
__global__ void convert_problem_kernel(int prec, int n, int m, int m_pad, int lda,
                                       const double* __restrict__ A, const double* __restrict__ b,
                                       double* A64, float* A32, __bf16* Ahi, __bf16* Alo,
                                       double* b64, float* rownorm, float* absb)
{
    const int lane = threadIdx.x & 63;
    const int row = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    if (row >= m_pad) return;
    const bool real = row < m;
    double ss = 0.0;
    for (int j = lane; j < lda; j += 64) {
        double v = (real && j < n) ? A[(size_t)row * n + j] : 0.0;
        A64[(size_t)row * lda + j] = v;
        if (prec == kFP32) A32[(size_t)row * lda + j] = (float)v;
        if (prec == kBF16X3) {
            __bf16 hi, lo;
            split_bf16((float)v, hi, lo);
            Ahi[(size_t)row * lda + j] = hi;
            Alo[(size_t)row * lda + j] = lo;
        }
        ss = fma(v, v, ss);
    }
    ss = wave_sum(ss);
    if (lane == 0) {
        double bv = real ? b[row] : 1.0;
        b64[row] = bv;
        rownorm[row] = real ? (float)(sqrt(ss) * (1.0 + 0x1.0p-20)) : 0.0f;
        absb[row] = (float)(fabs(bv) * (1.0 + 0x1.0p-20));
    }
}

// Equality setup in one workgroup: G = A_eq A_eq^T, Cholesky G = L L^T
// (pivot <= 1e-12 max diag G: rank deficient), W^T = G^{-1} A_eq.
__global__ void eq_setup_kernel(int n, int lda, int m_eq, const double* __restrict__ Aeq_in,
                                const double* __restrict__ beq_in, double* Aeq, double* beq,
                                double* WT, int* status)
{
    __shared__ double Gs[kMaxMeq * kMaxMeq];
    __shared__ int bad;
    const int tid = threadIdx.x, nt = blockDim.x;
    for (int item = tid; item < m_eq * lda; item += nt) {
        int p = item / lda, j = item - p * lda;
        Aeq[item] = j < n ? Aeq_in[(size_t)p * n + j] : 0.0;
    }
    for (int p = tid; p < m_eq; p += nt) beq[p] = beq_in[p];
    __syncthreads();
    for (int pq = tid; pq < m_eq * m_eq; pq += nt) {
        int p = pq / m_eq, q = pq - p * m_eq;
        double v = 0.0;
        for (int j = 0; j < n; ++j) v = fma(Aeq[(size_t)p * lda + j], Aeq[(size_t)q * lda + j], v);
        Gs[pq] = v;
    }
    __syncthreads();
    if (tid == 0) {
        double md = 0.0;
        for (int i = 0; i < m_eq; ++i) md = fmax(md, Gs[i * m_eq + i]);
        bad = 0;
        for (int j = 0; j < m_eq && !bad; ++j) {
            double piv = Gs[j * m_eq + j];
            for (int k = 0; k < j; ++k) piv -= Gs[j * m_eq + k] * Gs[j * m_eq + k];
            if (!(piv > 1e-12 * md)) {
                bad = 1;
                break;
            }
            double ljj = sqrt(piv);
            Gs[j * m_eq + j] = ljj;
            for (int i = j + 1; i < m_eq; ++i) {
                double v = Gs[i * m_eq + j];
                for (int k = 0; k < j; ++k) v -= Gs[i * m_eq + k] * Gs[j * m_eq + k];
                Gs[i * m_eq + j] = v / ljj;
            }
        }
        *status = bad;
    }
    __syncthreads();
    if (bad) return;
    double y[kMaxMeq];
    for (int j = tid; j < lda; j += nt) {
        for (int p = 0; p < m_eq; ++p) y[p] = Aeq[(size_t)p * lda + j];
        for (int i = 0; i < m_eq; ++i) {
            double v = y[i];
            for (int k = 0; k < i; ++k) v -= Gs[i * m_eq + k] * y[k];
            y[i] = v / Gs[i * m_eq + i];
        }
        for (int i = m_eq - 1; i >= 0; --i) {
            double v = y[i];
            for (int k = i + 1; k < m_eq; ++k) v -= Gs[k * m_eq + i] * y[k];
            y[i] = v / Gs[i * m_eq + i];
        }
        for (int p = 0; p < m_eq; ++p) WT[(size_t)p * lda + j] = y[p];
    }
}

__global__ void dense_projection_kernel(int n, int lda, int m_eq, const double* __restrict__ Aeq,
                                        const double* __restrict__ WT, double* P)
{
    const int64_t total = (int64_t)n * n;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        int i = (int)(e / n), j = (int)(e - (int64_t)i * n);
        double v = 0.0;
        for (int p = 0; p < m_eq; ++p) v = fma(WT[(size_t)p * lda + i], Aeq[(size_t)p * lda + j], v);
        P[e] = (i == j ? 1.0 : 0.0) - v;
    }
}

__global__ void copy_states_kernel(int n, int lda, int z, int z_pad, const double* __restrict__ src,
                                   double* X)
{
    const int64_t total = (int64_t)z_pad * lda;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        int k = (int)(e / lda), j = (int)(e - (int64_t)k * lda);
        X[e] = (k < z && j < n) ? src[(size_t)k * n + j] : 0.0;
    }
}

__global__ void export_states_kernel(int n, int lda, int z, const double* __restrict__ X, double* dst)
{
    const int64_t total = (int64_t)z * n;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        int k = (int)(e / n), j = (int)(e - (int64_t)k * n);
        dst[e] = X[(size_t)k * lda + j];
    }
}

__global__ void eq_residual_kernel(int n, int lda, int z, int m_eq, const double* __restrict__ Aeq,
                                   const double* __restrict__ beq, const double* __restrict__ X,
                                   int* flags)
{
    const int lane = threadIdx.x & 63;
    const int k = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    if (k >= z) return;
    int bad = 0;
    for (int p = 0; p < m_eq; ++p) {
        double v = 0.0;
        for (int j = lane; j < n; j += 64) v = fma(Aeq[(size_t)p * lda + j], X[(size_t)k * lda + j], v);
        v = wave_sum(v);
        if (!(fabs(v - beq[p]) <= 1e-9)) bad = 1;
    }
    if (lane == 0 && bad) atomicOr(&flags[k], kNotInterior);
}

__global__ void fill_i32_kernel(int* p, int64_t count, int value)
{
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < count;
         e += (int64_t)gridDim.x * blockDim.x)
        p[e] = value;
}

__global__ void fill_u64_kernel(unsigned long long* p, int64_t count, unsigned long long value)
{
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < count;
         e += (int64_t)gridDim.x * blockDim.x)
        p[e] = value;
}

__global__ void export_flags_kernel(const int* flags, int z, int32_t* out, int clear_internal)
{
    for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < z; k += gridDim.x * blockDim.x) {
        int v = flags[k];
        out[k] = clear_internal ? (v & 15) : v;
    }
}

inline int grid_for(int64_t total, int threads)
{
    int64_t g = (total + threads - 1) / threads;
    if (g < 1) g = 1;
    if (g > 65535) g = 65535;
    return (int)g;
}

}  // namespace

static_assert((size_t)kChainTile * (kMaxN + 2) * sizeof(double) + sizeof(ChainLds) <= 163840,
              "the general kernel's LDS must fit one CU at the largest n");

size_t step_lds_bytes(int prec, int lda)
{
    (void)prec;
    return big_bytes(lda) + sizeof(ChainLds);
}

template <int P>
static hipError_t launch_steps_t(const StepArgs& a, hipStream_t stream)
{
    const size_t lds = step_lds_bytes(P, a.lda);
    hipError_t e = hipFuncSetAttribute((const void*)mhar_steps_kernel<P>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(mhar_steps_kernel<P>, dim3(a.z_pad / kChainTile), dim3(kThreads), lds,
                       stream, a);
    return hipGetLastError();
}

template <int P>
static hipError_t launch_batch_t(const StepArgs* descs, const int2* units, int nunits,
                                 unsigned* next, int max_lda, int grid, hipStream_t stream)
{
    const size_t lds = step_lds_bytes(P, max_lda);
    // the kernel also has a few bytes of static LDS: request only what is used
    hipError_t e = hipFuncSetAttribute((const void*)mhar_batch_kernel<P>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(mhar_batch_kernel<P>, dim3(grid), dim3(kThreads), lds, stream, descs, units,
                       nunits, next);
    return hipGetLastError();
}

hipError_t launch_batch(int prec, const StepArgs* descs, const int2* units, int nunits,
                        unsigned* next, int max_lda, int grid, hipStream_t stream)
{
    switch (prec) {
    case kFP64: return launch_batch_t<kFP64>(descs, units, nunits, next, max_lda, grid, stream);
    case kFP32: return launch_batch_t<kFP32>(descs, units, nunits, next, max_lda, grid, stream);
    case kBF16X3: return launch_batch_t<kBF16X3>(descs, units, nunits, next, max_lda, grid, stream);
    default: return hipErrorInvalidValue;
    }
}

int batch_blocks_per_cu(int prec, int max_lda)
{
    int nb = 0;
    const size_t lds = step_lds_bytes(prec, max_lda);
    const void* fn = prec == kFP64 ? (const void*)mhar_batch_kernel<kFP64>
                   : prec == kFP32 ? (const void*)mhar_batch_kernel<kFP32>
                                   : (const void*)mhar_batch_kernel<kBF16X3>;
    if (hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, fn, kThreads, lds) != hipSuccess) {
        (void)hipGetLastError();   // do not leave a stale error for the next launch
        return 1;
    }
    return nb < 1 ? 1 : nb;
}

// event pair around one launch when a trace is attached and has room
struct TraceScope {
    KernelTrace* t;
    hipStream_t s;
    int slot;
    TraceScope(KernelTrace* tr, hipStream_t st, int kind) : t(tr), s(st), slot(-1)
    {
        if (t && t->used < t->cap) {
            slot = t->used++;
            t->kind[slot] = kind;
            (void)hipEventRecord(t->ev[2 * slot], s);
        }
    }
    ~TraceScope()
    {
        if (slot >= 0) (void)hipEventRecord(t->ev[2 * slot + 1], s);
    }
};

template <int P>
static hipError_t launch_tiled_t(const StepArgs& a, hipStream_t stream, KernelTrace* trace)
{
    const size_t lds_r = 2 * (size_t)kRStage;
    hipError_t e = hipFuncSetAttribute((const void*)tiled_recompute_kernel,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_r);
    if (e != hipSuccess) return e;
    const int ts = ((a.m_pad + kTR - 1) / kTR) * ((a.z_pad + kTW - 1) / kTW);
    const int tr = ((a.m_pad + kRR - 1) / kRR) * ((a.z_pad + kRW - 1) / kRW);
    const dim3 grid_s((ts + 7) / 8 * 8), grid_r((tr + 7) / 8 * 8), grid_c(a.z_pad / kChainTile);
    int pending = a.pending0, T = a.T0, since = a.since0;
    if (a.recompute_first) {
        TraceScope ts_(trace, stream, kTraceRecompute);
        hipLaunchKernelGGL(tiled_recompute_kernel, grid_r, dim3(kRecThreads), lds_r, stream, a);
        pending = 0;
        T = 2;
        since = 0;
    }
    // isotropic directions come from their own launch, one workgroup per walk;
    // a learned covariance keeps them in the chords kernel
    const bool own_dirs = a.r == 0;
    const dim3 grid_d(a.z_pad);
    if (a.steps > 0) {
        if (own_dirs) {
            TraceScope ts_(trace, stream, kTraceDirs);
            hipLaunchKernelGGL(tiled_dirs_kernel<P>, grid_d, dim3(kDirThreads), 0, stream, a, a.step0);
        } else {
            TraceScope ts_(trace, stream, kTraceChords);
            hipLaunchKernelGGL(tiled_chords_kernel<P>, grid_c, dim3(kThreads), 0, stream, a,
                               (uint64_t)0, 0, T, 0, 1, a.step0);
        }
    }
    for (int s = 0; s < a.steps; ++s) {
        const uint64_t step = a.step0 + (uint64_t)s;
        const bool more = s + 1 < a.steps;
        {
            TraceScope ts_(trace, stream, kTraceScreen);
            if (a.rk > 0)
                hipLaunchKernelGGL((tiled_screen_kernel<P, true>), grid_s, dim3(kScreenThreads), 0,
                                   stream, a, pending, T);
            else
                hipLaunchKernelGGL((tiled_screen_kernel<P, false>), grid_s, dim3(kScreenThreads), 0,
                                   stream, a, pending, T);
        }
        {
            TraceScope ts_(trace, stream, kTraceChords);
            hipLaunchKernelGGL(tiled_chords_kernel<P>, grid_c, dim3(kThreads), 0, stream, a, step, s,
                               T, 1, (int)(more && !own_dirs), step + 1);
        }
        if (more && own_dirs) {
            TraceScope ts_(trace, stream, kTraceDirs);
            hipLaunchKernelGGL(tiled_dirs_kernel<P>, grid_d, dim3(kDirThreads), 0, stream, a, step + 1);
        }
        pending = 1;
        T += 1;
        since += 1;
        if (since >= a.R) {
            TraceScope ts_(trace, stream, kTraceRecompute);
            hipLaunchKernelGGL(tiled_recompute_kernel, grid_r, dim3(kRecThreads), lds_r, stream, a);
            pending = 0;
            T = 2;
            since = 0;
        }
        e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipGetLastError();
}

template <int P>
static hipError_t launch_grouped_t(const StepArgs* descs, const int4* stiles, int nst,
                                   const int2* units, int nunits, const int4* rtiles, int nrt,
                                   int steps, int first, const unsigned char* due,
                                   int any_split, hipStream_t stream)
{
    const size_t lds_r = 2 * (size_t)kRStage;
    hipError_t e = hipFuncSetAttribute((const void*)grouped_recompute_kernel,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_r);
    if (e != hipSuccess) return e;
    if (first)
        hipLaunchKernelGGL(grouped_recompute_kernel, dim3(nrt), dim3(kRecThreads), lds_r, stream, descs,
                           rtiles, nrt, 0, 1);
    if (steps > 0)
        hipLaunchKernelGGL(grouped_chords_kernel<P>, dim3(nunits), dim3(kThreads), 0, stream, descs,
                           units, nunits, 0, 0, 1);
    for (int s = 0; s < steps; ++s) {
        if (any_split)
            hipLaunchKernelGGL((grouped_screen_kernel<P, true>), dim3(nst), dim3(kScreenThreads), 0,
                               stream, descs, stiles, nst, s);
        else
            hipLaunchKernelGGL((grouped_screen_kernel<P, false>), dim3(nst), dim3(kScreenThreads), 0,
                               stream, descs, stiles, nst, s);
        hipLaunchKernelGGL(grouped_chords_kernel<P>, dim3(nunits), dim3(kThreads), 0, stream, descs,
                           units, nunits, s, 1, (int)(s + 1 < steps));
        if (due[s])
            hipLaunchKernelGGL(grouped_recompute_kernel, dim3(nrt), dim3(kRecThreads), lds_r, stream,
                               descs, rtiles, nrt, s, 0);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipGetLastError();
}

hipError_t launch_grouped(int prec, const StepArgs* descs, const int4* stiles, int nst,
                          const int2* units, int nunits, const int4* rtiles, int nrt, int steps,
                          int first, const unsigned char* due, int any_split, hipStream_t stream)
{
    switch (prec) {
    case kFP32: return launch_grouped_t<kFP32>(descs, stiles, nst, units, nunits, rtiles, nrt, steps,
                                               first, due, any_split, stream);
    case kBF16X3: return launch_grouped_t<kBF16X3>(descs, stiles, nst, units, nunits, rtiles, nrt,
                                                   steps, first, due, any_split, stream);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_tiled(int prec, const StepArgs& a, hipStream_t stream, KernelTrace* trace)
{
    switch (prec) {
    case kFP32: return launch_tiled_t<kFP32>(a, stream, trace);
    case kBF16X3: return launch_tiled_t<kBF16X3>(a, stream, trace);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_steps(int prec, const StepArgs& a, hipStream_t stream)
{
    switch (prec) {
    case kFP64: return launch_steps_t<kFP64>(a, stream);
    case kFP32: return launch_steps_t<kFP32>(a, stream);
    case kBF16X3: return launch_steps_t<kBF16X3>(a, stream);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_convert_problem(int prec, int n, int m, int m_pad, int lda, const double* A,
                                  const double* b, double* A64, float* A32, __bf16* Ahi,
                                  __bf16* Alo, double* b64, float* rownorm, float* absb,
                                  hipStream_t stream)
{
    const int rows_per_block = 4;
    hipLaunchKernelGGL(convert_problem_kernel, dim3((m_pad + rows_per_block - 1) / rows_per_block),
                       dim3(64 * rows_per_block), 0, stream, prec, n, m, m_pad, lda, A, b, A64, A32,
                       Ahi, Alo, b64, rownorm, absb);
    return hipGetLastError();
}

// Operand copy in the load order of the register-resident kernel: one
// thread per 16-byte lane unit (layout at StepArgs::Apk).
__global__ void pack_operand_kernel(int prec, int m_pad, int lda, const float* __restrict__ A32,
                                    const __bf16* __restrict__ Ahi, const __bf16* __restrict__ Alo,
                                    uint4* __restrict__ Apk)
{
    const int nk = lda / 32;
    const size_t units = (size_t)(m_pad / 16) * nk * 128;
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= units) return;
    const int l = (int)(i & 63), u = (int)((i >> 6) & 1);
    const size_t blk = i >> 7;   // R * nk + kc
    const int kc = (int)(blk % nk), R = (int)(blk / nk);
    const int g = l >> 4, c = l & 15;
    const size_t row = (size_t)16 * R + c;
    if (prec == kFP32) Apk[i] = *(const uint4*)(A32 + row * lda + 32 * kc + 8 * g + 4 * u);
    else Apk[i] = *(const uint4*)((u ? Alo : Ahi) + row * lda + 32 * kc + 8 * g);
}

hipError_t launch_pack_operand(int prec, int m_pad, int lda, const float* A32, const __bf16* Ahi,
                               const __bf16* Alo, void* Apk, hipStream_t stream)
{
    if ((prec != kFP32 && prec != kBF16X3) || lda % 32 || m_pad % 16) return hipErrorInvalidValue;
    const size_t units = (size_t)(m_pad / 16) * (lda / 32) * 128;
    hipLaunchKernelGGL(pack_operand_kernel, dim3((unsigned)((units + 255) / 256)), dim3(256), 0, stream,
                       prec, m_pad, lda, A32, Ahi, Alo, (uint4*)Apk);
    return hipGetLastError();
}

hipError_t launch_eq_setup(int n, int lda, int m_eq, const double* Aeq_in, const double* beq_in,
                           double* Aeq, double* beq, double* WT, int* status, hipStream_t stream)
{
    hipLaunchKernelGGL(eq_setup_kernel, dim3(1), dim3(256), 0, stream, n, lda, m_eq, Aeq_in,
                       beq_in, Aeq, beq, WT, status);
    return hipGetLastError();
}

hipError_t launch_dense_projection(int n, int lda, int m_eq, const double* Aeq, const double* WT,
                                   double* P, hipStream_t stream)
{
    hipLaunchKernelGGL(dense_projection_kernel, dim3(grid_for((int64_t)n * n, 256)), dim3(256), 0,
                       stream, n, lda, m_eq, Aeq, WT, P);
    return hipGetLastError();
}

hipError_t launch_copy_states(int n, int lda, int z, int z_pad, const double* src, double* X,
                              hipStream_t stream)
{
    hipLaunchKernelGGL(copy_states_kernel, dim3(grid_for((int64_t)z_pad * lda, 256)), dim3(256),
                       0, stream, n, lda, z, z_pad, src, X);
    return hipGetLastError();
}

hipError_t launch_export_states(int n, int lda, int z, const double* X, double* dst,
                                hipStream_t stream)
{
    hipLaunchKernelGGL(export_states_kernel, dim3(grid_for((int64_t)z * n, 256)), dim3(256), 0,
                       stream, n, lda, z, X, dst);
    return hipGetLastError();
}

hipError_t launch_eq_residual(int n, int lda, int z, int m_eq, const double* Aeq,
                              const double* beq, const double* X, int* flags, hipStream_t stream)
{
    hipLaunchKernelGGL(eq_residual_kernel, dim3((z + 3) / 4), dim3(256), 0, stream, n, lda, z,
                       m_eq, Aeq, beq, X, flags);
    return hipGetLastError();
}

hipError_t launch_step_counter(uint64_t* ctr, uint64_t value, int add, hipStream_t stream)
{
    hipLaunchKernelGGL(step_counter_kernel, dim3(1), dim3(64), 0, stream, ctr, value, add);
    return hipGetLastError();
}

hipError_t launch_fill_i32(int* p, int64_t count, int value, hipStream_t stream)
{
    hipLaunchKernelGGL(fill_i32_kernel, dim3(grid_for(count, 256)), dim3(256), 0, stream, p,
                       count, value);
    return hipGetLastError();
}

hipError_t launch_fill_u64(unsigned long long* p, int64_t count, unsigned long long value,
                           hipStream_t stream)
{
    hipLaunchKernelGGL(fill_u64_kernel, dim3(grid_for(count, 256)), dim3(256), 0, stream, p, count,
                       value);
    return hipGetLastError();
}

hipError_t launch_export_flags(const int* flags, int z, int32_t* out, int clear_internal,
                               hipStream_t stream)
{
    hipLaunchKernelGGL(export_flags_kernel, dim3(grid_for(z, 256)), dim3(256), 0, stream, flags,
                       z, out, clear_internal);
    return hipGetLastError();
}

}  // namespace mhar
