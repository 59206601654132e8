// mhar_lane.hip -- a few lanes per walk, every row exact: the MHAR step for
// small problems (n <= 32 in registers, n <= 64 with the walk state in LDS)
// on gfx950.
//
// Same method as the other kernels (paper Alg. 2, S4.3-S4.5), without the
// screening product: a group of G lanes (1 to 8) holds the state x and
// direction d of one walk in registers and evaluates the line-set formula
// of S4.4 for every row in FP64, s_i = b_i - a_i x and g_i = a_i d as
// sequential sums (the order of the other paths' exact rows), then theta
// and the update.  Lane q of a group draws the Box-Muller pairs p = q (mod G)
// and evaluates the rows i = q (mod G); the draws are gathered and the chord
// ends combined (an exact minimum, so in any order) by lane swizzles within
// the group.  For small m n this costs less than the product tile, the
// screening and the workgroup barriers it replaces.  A and b are copied into
// LDS once per launch when they fit (48 KB), since each lane of a group
// reads a different row; the walks are independent, so that copy is the
// only barrier.
//
// The directions are bitwise those of the other paths: the draws come from
// the same counter streams, and A_eq h is summed in the order of their
// wave reduction (one product per lane, then pairwise halving), which a
// single lane can replay because n <= 64 (one product per lane of the wave).
#include <math.h>

#include "mhar_device.hpp"
#include "mhar_internal.hpp"

namespace mhar {

namespace {

constexpr int kLaneThreads = 64;
constexpr int kLaneMaxN = 32;   // x and d of a walk in registers

// Lane moves within 32-lane halves by ds_swizzle in bit mode: lane i reads
// lane ((i & and_mask) | or_mask) ^ xor_mask.
constexpr int swz_pattern(int and_mask, int or_mask, int xor_mask)
{
    return (and_mask & 31) | ((or_mask & 31) << 5) | ((xor_mask & 31) << 10);
}

template <int PAT>
__device__ __forceinline__ double swz(double v)
{
    const int lo = __builtin_amdgcn_ds_swizzle(__double2loint(v), PAT);
    const int hi = __builtin_amdgcn_ds_swizzle(__double2hiint(v), PAT);
    return __hiloint2double(hi, lo);
}

template <int PAT>
__device__ __forceinline__ unsigned long long swz_u64(unsigned long long v)
{
    const int lo = __builtin_amdgcn_ds_swizzle((int)(unsigned)v, PAT);
    const int hi = __builtin_amdgcn_ds_swizzle((int)(unsigned)(v >> 32), PAT);
    return ((unsigned long long)(unsigned)hi << 32) | (unsigned)lo;
}

// value v of lane OWNER of this lane's group of G
template <int G, int OWNER>
__device__ __forceinline__ double group_bcast(double v)
{
    if constexpr (G == 1) return v;
    else return swz<swz_pattern(31 & ~(G - 1), OWNER, 0)>(v);
}

// minimum (as unsigned) and OR over the lanes of a group of G
template <int G>
__device__ __forceinline__ void group_min_or(unsigned long long& a, unsigned long long& b, int& f)
{
    if constexpr (G > 1) {
#pragma unroll
        for (int s = 1; s < G; s <<= 1) {
            // s is a compile-time constant after unrolling; the pattern is
            // selected among the few group sizes
            unsigned long long oa, ob;
            int of;
            if (s == 1) { oa = swz_u64<swz_pattern(31, 0, 1)>(a); ob = swz_u64<swz_pattern(31, 0, 1)>(b); of = __builtin_amdgcn_ds_swizzle(f, swz_pattern(31, 0, 1)); }
            else if (s == 2) { oa = swz_u64<swz_pattern(31, 0, 2)>(a); ob = swz_u64<swz_pattern(31, 0, 2)>(b); of = __builtin_amdgcn_ds_swizzle(f, swz_pattern(31, 0, 2)); }
            else { oa = swz_u64<swz_pattern(31, 0, 4)>(a); ob = swz_u64<swz_pattern(31, 0, 4)>(b); of = __builtin_amdgcn_ds_swizzle(f, swz_pattern(31, 0, 4)); }
            a = oa < a ? oa : a;
            b = ob < b ? ob : b;
            f |= of;
        }
    }
}

// NM: compile-time bound on n (power of two, <= 32).  G: lanes per walk
// (1, 2, 4 or 8); lane q of a walk's group draws the pairs p = q (mod G) and
// evaluates the rows i = q (mod G); the draws are gathered within the group,
// the chord ends combined by an exact minimum, and every lane of the group
// then holds the same theta, direction and state.
template <int NM, int G, bool STAGED>
__global__ __launch_bounds__(kLaneThreads) void lane_kernel(StepArgs a)
{
    static_assert(NM <= 32 && (NM & (NM - 1)) == 0, "NM: power of two up to 32");
    static_assert(G == 1 || G == 2 || G == 4 || G == 8, "G: 1, 2, 4 or 8 lanes per walk");
    constexpr int PK = (NM / 2 + G - 1) / G;   // pairs drawn per lane
    const int q = threadIdx.x & (G - 1);
    const int chain = blockIdx.x * (kLaneThreads / G) + threadIdx.x / G;
    const int n = a.n, m = a.m;
    // A and b staged in LDS when the launch provides room (rows padded by one
    // double, so the lanes of a group, which read different rows, hit
    // different banks); otherwise read from global memory
    extern __shared__ double lane_lds[];
    const int lda = STAGED ? NM + 1 : a.lda;
    const double* __restrict__ A = STAGED ? lane_lds : a.A64;
    const double* __restrict__ b = STAGED ? lane_lds + (size_t)m * (NM + 1) : a.b64;
    if (STAGED) {
        for (int e = threadIdx.x; e < m * (NM + 1); e += kLaneThreads) {
            const int i = e / (NM + 1), j = e - i * (NM + 1);
            lane_lds[e] = j < n ? a.A64[(size_t)i * a.lda + j] : 0.0;
        }
        for (int i = threadIdx.x; i < m; i += kLaneThreads) lane_lds[(size_t)m * (NM + 1) + i] = a.b64[i];
        __syncthreads();
    }
    if (chain >= a.z) return;   // whole groups leave together

    double x[NM];
#pragma unroll
    for (int j = 0; j < NM; ++j) x[j] = j < n ? a.X[(size_t)chain * a.lda + j] : 0.0;
    int fl = 0;
    double theta = a.theta[chain];

    // exact slack of this lane's rows at the launch's start and every R
    // steps (where the other paths recompute it): start point strictly inside?
    auto check_interior = [&]() __attribute__((always_inline)) {
        for (int i = q; i < m; i += G) {
            const double* ar = A + (size_t)i * lda;
            const double bi = b[i];
            double s = bi;
#pragma unroll
            for (int j = 0; j < NM; ++j)
                if (j < n) s = __dsub_rn(s, __dmul_rn(ar[j], x[j]));
            if (!(s > 0.0)) fl |= kNotInterior;
            if (s < -1e-12 * fmax(1.0, fabs(bi))) fl |= kInfeasible;
        }
    };
    if (a.recompute_first || a.steps == 0 || a.since0 == 0) check_interior();

    for (int s = 0; s < a.steps; ++s) {
        const uint64_t step = a.step0 + (uint64_t)s;
        if (s > 0 && (a.since0 + s) % a.R == 0) check_interior();

        // ---- directions: N(0, 1) pairs (this lane's share), gathered ----
        double2 hq[PK];
#pragma unroll
        for (int k = 0; k < PK; ++k) {
            const int p = q + G * k;
            hq[k] = make_double2(0.0, 0.0);
            if (2 * p < n) {
                Block4 w = stream_block(a.seed, kTagDir, a.chain_offset + (uint32_t)chain, step, (uint32_t)p);
                gauss_pair(w, hq[k].x, hq[k].y);
            }
        }
        double d[NM];
#pragma unroll
        for (int j = 0; j < NM; ++j) {
            const int p = j >> 1;
            const double v = (j & 1) ? hq[p / G].y : hq[p / G].x;
            double g;
            switch (p % G) {   // compile-time after unrolling
            case 0: g = group_bcast<G, 0>(v); break;
            case 1: g = group_bcast<G, (G > 1 ? 1 : 0)>(v); break;
            case 2: g = group_bcast<G, (G > 2 ? 2 : 0)>(v); break;
            case 3: g = group_bcast<G, (G > 3 ? 3 : 0)>(v); break;
            case 4: g = group_bcast<G, (G > 4 ? 4 : 0)>(v); break;
            case 5: g = group_bcast<G, (G > 5 ? 5 : 0)>(v); break;
            case 6: g = group_bcast<G, (G > 6 ? 6 : 0)>(v); break;
            default: g = group_bcast<G, (G > 7 ? 7 : 0)>(v); break;
            }
            d[j] = j < n ? g : 0.0;
        }
        if (a.m_eq > 0) {
            // y_p = A_eq h: one product per coordinate (an FMA onto +0, as a
            // lane of the wave reduction forms it), then pairwise halving
            // (coordinates >= NM would only add +0); d_j = h_j - sum_p W_pj y_p
            // in order of p, as each coordinate's FMA chain elsewhere
            double h[NM];
#pragma unroll
            for (int j = 0; j < NM; ++j) h[j] = d[j];
            for (int p = 0; p < a.m_eq; ++p) {
                const double* er = a.Aeq + (size_t)p * a.lda;
                double t[NM];
#pragma unroll
                for (int j = 0; j < NM; ++j) t[j] = j < n ? fma(er[j], h[j], 0.0) : 0.0;
#pragma unroll
                for (int half = NM / 2; half > 0; half >>= 1)
#pragma unroll
                    for (int j = 0; j < half; ++j) t[j] = t[j] + t[j + half];
                const double y = t[0];
                const double* wr = a.WT + (size_t)p * a.lda;
#pragma unroll
                for (int j = 0; j < NM; ++j)
                    if (j < n) d[j] = fma(-wr[j], y, d[j]);
            }
        }

        // ---- chord: every row exactly (S4.4, Lemma 4.2), rows split over the group ----
        unsigned long long lmax_b = (unsigned long long)__double_as_longlong(kInfD);
        unsigned long long nlmin_b = lmax_b;
        for (int i = q; i < m; i += G) {
            const double* ar = A + (size_t)i * lda;
            const double bi = b[i];
            double sx = bi, gx = 0.0;
#pragma unroll
            for (int j = 0; j < NM; ++j) {
                if (j < n) {
                    sx = __dsub_rn(sx, __dmul_rn(ar[j], x[j]));
                    gx = __dadd_rn(gx, __dmul_rn(ar[j], d[j]));
                }
            }
            if (sx < -1e-12 * fmax(1.0, fabs(bi))) fl |= kInfeasible;
            if (sx < 0.0) sx = 0.0;
            // chord ends compared as ordered bits (both >= 0; NaN never wins)
            if (gx > 0.0) {
                const unsigned long long c = (unsigned long long)__double_as_longlong(sx / gx);
                lmax_b = c < lmax_b ? c : lmax_b;
            } else if (gx < 0.0) {
                const unsigned long long c = (unsigned long long)__double_as_longlong(sx / -gx);
                nlmin_b = c < nlmin_b ? c : nlmin_b;
            }
        }
        int fl_any = fl;
        group_min_or<G>(lmax_b, nlmin_b, fl_any);
        fl = fl_any;

        // ---- theta and the update (S4.5, Lemma 4.3), the same in every lane of the group ----
        const double lmax = __longlong_as_double((long long)lmax_b);
        const double lmin = -__longlong_as_double((long long)nlmin_b);
        double th = 0.0;
        if (lmax == kInfD || lmin == -kInfD) {
            fl |= kUnbounded;
        } else if (!(lmax > lmin)) {
            fl |= kDegenerate;
        } else {
            Block4 w = stream_block(a.seed, kTagTheta, a.chain_offset + (uint32_t)chain, step, 0);
            const double u = open_unit(w.w0, w.w1);
            th = __dadd_rn(lmin, __dmul_rn(u, __dsub_rn(lmax, lmin)));
        }
        theta = th;
        bool finite = isfinite(th);
#pragma unroll
        for (int j = 0; j < NM; ++j) {
            if (j < n) {
                x[j] = __dadd_rn(x[j], __dmul_rn(th, d[j]));
                finite = finite && isfinite(x[j]);
            }
        }
        if (!finite) fl |= kNonFinite;
        if (q == 0 && a.rec_stride > 0 && chain < a.rec_chains) {
            const int64_t rs = a.rec_s_base + s + 1;
            if (rs % a.rec_stride == 0) {
                double* rp = a.rec_out + ((size_t)(rs / a.rec_stride - 1) * a.rec_chains + chain) * n;
#pragma unroll
                for (int j = 0; j < NM; ++j)
                    if (j < n) rp[j] = x[j];
            }
        }
    }

    // flags of the interior checks after the last step are combined too
    unsigned long long u0 = 0, u1 = 0;
    group_min_or<G>(u0, u1, fl);
    // exact rows, one atomic per wave (lane 0 is live whenever any lane is)
    const unsigned long long walks = __popcll(__ballot(q == 0));
    if (threadIdx.x == 0 && a.steps > 0)
        atomicAdd(&a.counters[0], walks * (unsigned long long)m * (unsigned long long)a.steps);
    if (q != 0) return;
#pragma unroll
    for (int j = 0; j < NM; ++j)
        if (j < n) a.X[(size_t)chain * a.lda + j] = x[j];
    a.theta[chain] = theta;
    if (fl) atomicOr(&a.flags[chain], fl);
}

// Rows of length 33..64: the same step with x, d and the draws h of each
// walk kept in LDS beside the staged A and b (a workgroup is one wave, so
// LDS hand-offs between the lanes of a group need only a wave-level fence).
// Lane q of a group draws the pairs p = q (mod G), updates the coordinates
// j = q (mod G) and evaluates the rows i = q (mod G); every lane of the group
// forms A_eq h in the order of the other paths' wave reduction (one FMA
// product per coordinate onto +0; pairs of coordinates 32 apart, then
// pairwise halving).
constexpr int kWideN = 64;
constexpr int kWideLd = kWideN + 2;   // LDS row stride (doubles): 16-byte aligned rows, shifted banks

__device__ __forceinline__ void wave_sync_lds()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <int G>
__global__ __launch_bounds__(kLaneThreads) void lane_wide_kernel(StepArgs a)
{
    constexpr int W = kLaneThreads / G;   // walks per workgroup (one wave)
    constexpr int LD = kWideLd;
    const int q = threadIdx.x & (G - 1), wl = threadIdx.x / G;
    const int chain = blockIdx.x * W + wl;
    const int n = a.n, m = a.m;
    extern __shared__ double lane_lds[];
    double* As = lane_lds;                 // m x LD
    double* bs = As + (size_t)m * LD;      // m (padded to even)
    double* xs = bs + ((m + 1) & ~1);      // W x LD
    double* ds = xs + W * LD;              // W x LD
    double* hs = ds + W * LD;              // W x LD
    for (int e = threadIdx.x; e < m * LD; e += kLaneThreads) {
        const int i = e / LD, j = e - i * LD;
        As[e] = j < n ? a.A64[(size_t)i * a.lda + j] : 0.0;
    }
    for (int i = threadIdx.x; i < m; i += kLaneThreads) bs[i] = a.b64[i];
    const bool live = chain < a.z;
    double* xw = xs + wl * LD;
    double* dw = ds + wl * LD;
    double* hw = hs + wl * LD;
    for (int j = q; j < LD; j += G) {
        xw[j] = (live && j < n) ? a.X[(size_t)chain * a.lda + j] : 0.0;
        dw[j] = 0.0;
        hw[j] = 0.0;
    }
    wave_sync_lds();
    if (!live) return;   // whole groups leave together; no wave-wide sync follows for them
    int fl = 0;
    double theta = a.theta[chain];

    auto check_interior = [&]() __attribute__((always_inline)) {
        for (int i = q; i < m; i += G) {
            const double* ar = As + (size_t)i * LD;
            const double bi = bs[i];
            double s = bi;
            for (int j = 0; j < n; ++j) s = __dsub_rn(s, __dmul_rn(ar[j], xw[j]));
            if (!(s > 0.0)) fl |= kNotInterior;
            if (s < -1e-12 * fmax(1.0, fabs(bi))) fl |= kInfeasible;
        }
    };
    if (a.recompute_first || a.steps == 0 || a.since0 == 0) check_interior();

    const int npairs = (n + 1) >> 1;
    for (int s = 0; s < a.steps; ++s) {
        const uint64_t step = a.step0 + (uint64_t)s;
        if (s > 0 && (a.since0 + s) % a.R == 0) check_interior();

        // ---- directions ----
        double* hd = a.m_eq > 0 ? hw : dw;
        for (int p = q; p < npairs; p += G) {
            Block4 w = stream_block(a.seed, kTagDir, a.chain_offset + (uint32_t)chain, step, (uint32_t)p);
            double ev, od;
            gauss_pair(w, ev, od);
            hd[2 * p] = ev;
            if (2 * p + 1 < n) hd[2 * p + 1] = od;
        }
        wave_sync_lds();
        if (a.m_eq > 0) {
            for (int j = q; j < n; j += G) dw[j] = hw[j];
            for (int p = 0; p < a.m_eq; ++p) {
                const double* er = a.Aeq + (size_t)p * a.lda;
                double t[32];
#pragma unroll
                for (int l = 0; l < 32; ++l) {
                    const double lo = l < n ? fma(er[l], hw[l], 0.0) : 0.0;
                    const double hi = l + 32 < n ? fma(er[l + 32], hw[l + 32], 0.0) : 0.0;
                    t[l] = lo + hi;
                }
#pragma unroll
                for (int half = 16; half > 0; half >>= 1)
#pragma unroll
                    for (int l = 0; l < half; ++l) t[l] = t[l] + t[l + half];
                const double y = t[0];
                const double* wr = a.WT + (size_t)p * a.lda;
                for (int j = q; j < n; j += G) dw[j] = fma(-wr[j], y, dw[j]);
            }
            wave_sync_lds();
        }

        // ---- chord: every row exactly, rows split over the group ----
        unsigned long long lmax_b = (unsigned long long)__double_as_longlong(kInfD);
        unsigned long long nlmin_b = lmax_b;
        for (int i = q; i < m; i += G) {
            const double* ar = As + (size_t)i * LD;
            const double bi = bs[i];
            double sx = bi, gx = 0.0;
            for (int j = 0; j < n; ++j) {
                const double aij = ar[j];
                sx = __dsub_rn(sx, __dmul_rn(aij, xw[j]));
                gx = __dadd_rn(gx, __dmul_rn(aij, dw[j]));
            }
            if (sx < -1e-12 * fmax(1.0, fabs(bi))) fl |= kInfeasible;
            if (sx < 0.0) sx = 0.0;
            if (gx > 0.0) {
                const unsigned long long c = (unsigned long long)__double_as_longlong(sx / gx);
                lmax_b = c < lmax_b ? c : lmax_b;
            } else if (gx < 0.0) {
                const unsigned long long c = (unsigned long long)__double_as_longlong(sx / -gx);
                nlmin_b = c < nlmin_b ? c : nlmin_b;
            }
        }
        group_min_or<G>(lmax_b, nlmin_b, fl);

        // ---- theta and the update ----
        const double lmax = __longlong_as_double((long long)lmax_b);
        const double lmin = -__longlong_as_double((long long)nlmin_b);
        double th = 0.0;
        if (lmax == kInfD || lmin == -kInfD) {
            fl |= kUnbounded;
        } else if (!(lmax > lmin)) {
            fl |= kDegenerate;
        } else {
            Block4 w = stream_block(a.seed, kTagTheta, a.chain_offset + (uint32_t)chain, step, 0);
            const double u = open_unit(w.w0, w.w1);
            th = __dadd_rn(lmin, __dmul_rn(u, __dsub_rn(lmax, lmin)));
        }
        theta = th;
        int nf = isfinite(th) ? 0 : kNonFinite;
        const int64_t rs = a.rec_s_base + s + 1;
        const bool rec = a.rec_stride > 0 && chain < a.rec_chains && rs % a.rec_stride == 0;
        double* rp = rec ? a.rec_out + ((size_t)(rs / a.rec_stride - 1) * a.rec_chains + chain) * n : nullptr;
        for (int j = q; j < n; j += G) {
            const double xn = __dadd_rn(xw[j], __dmul_rn(th, dw[j]));
            xw[j] = xn;
            if (!isfinite(xn)) nf = kNonFinite;
            if (rec) rp[j] = xn;
        }
        fl |= nf;
        wave_sync_lds();
    }

    unsigned long long u0 = 0, u1 = 0;
    group_min_or<G>(u0, u1, fl);
    const unsigned long long walks = __popcll(__ballot(q == 0));
    if (threadIdx.x == 0 && a.steps > 0)
        atomicAdd(&a.counters[0], walks * (unsigned long long)m * (unsigned long long)a.steps);
    for (int j = q; j < n; j += G) a.X[(size_t)chain * a.lda + j] = xw[j];
    if (q != 0) return;
    a.theta[chain] = theta;
    if (fl) atomicOr(&a.flags[chain], fl);
}

size_t lane_wide_bytes(int m, int G)
{
    return ((size_t)m * kWideLd + (((size_t)m + 1) & ~(size_t)1) + 3 * (size_t)(kLaneThreads / G) * kWideLd) * sizeof(double);
}

constexpr size_t kLaneWideMax = 96 * 1024;   // LDS bytes of the wide variant
constexpr int kLaneWideG = 8;

}  // namespace

bool lane_fits(int n, int m)
{
    if (n < 1) return false;
    if (n <= kLaneMaxN) return true;
    return n <= kWideN && lane_wide_bytes(m, kLaneWideG) <= kLaneWideMax;
}

constexpr size_t kLaneStageMax = 48 * 1024;   // LDS bytes for the staged A and b

template <int NM, int G>
hipError_t launch_lane_nm(const StepArgs& a, hipStream_t stream)
{
    const dim3 grid((unsigned)(((int64_t)a.z * G + kLaneThreads - 1) / kLaneThreads)), block(kLaneThreads);
    const size_t bytes = ((size_t)a.m * (NM + 1) + a.m) * sizeof(double);
    if (bytes <= kLaneStageMax) hipLaunchKernelGGL((lane_kernel<NM, G, true>), grid, block, bytes, stream, a);
    else hipLaunchKernelGGL((lane_kernel<NM, G, false>), grid, block, 0, stream, a);
    return hipGetLastError();
}

template <int G>
hipError_t launch_lane_g(const StepArgs& a, hipStream_t stream)
{
    if (a.n <= 8) return launch_lane_nm<8, G>(a, stream);
    if (a.n <= 16) return launch_lane_nm<16, G>(a, stream);
    return launch_lane_nm<32, G>(a, stream);
}

// Lanes per walk, from timings on one MI355X (hypercube and simplex, 16 to
// 10^4 walks): 4 for n <= 8; 8 up to n = 16 (the draws dominate); above, 8
// without equalities and 4 with them, whose projection every lane of the
// group repeats.
int lane_group(const StepArgs& a)
{
    if (a.n <= 8) return 4;
    if (a.n <= 16) return 8;
    return a.m_eq > 0 ? 4 : 8;
}

hipError_t launch_lane(const StepArgs& a, hipStream_t stream)
{
    if (!lane_fits(a.n, a.m) || a.r > 0 || a.m_eq > kMaxMeq) return hipErrorInvalidValue;
    if (a.n > kLaneMaxN) {
        const size_t bytes = lane_wide_bytes(a.m, kLaneWideG);
        const void* fn = (const void*)lane_wide_kernel<kLaneWideG>;
        hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
        if (e != hipSuccess) return e;
        const dim3 grid((unsigned)(((int64_t)a.z * kLaneWideG + kLaneThreads - 1) / kLaneThreads)), block(kLaneThreads);
        hipLaunchKernelGGL((lane_wide_kernel<kLaneWideG>), grid, block, bytes, stream, a);
        return hipGetLastError();
    }
    return lane_group(a) == 4 ? launch_lane_g<4>(a, stream) : launch_lane_g<8>(a, stream);
}

}  // namespace mhar
