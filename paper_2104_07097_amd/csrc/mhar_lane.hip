// mhar_lane.hip -- one walk per lane, every row exact: the MHAR step for
// small problems (n <= 32) on gfx950.
//
// Same method as the other kernels (paper Alg. 2, S4.3-S4.5), without the
// screening product: each lane holds the state x and direction d of its own
// walk in registers and evaluates the line-set formula of S4.4 for every
// row in FP64, s_i = b_i - a_i x and g_i = a_i d as sequential sums (the
// order of the other paths' exact rows), then theta and the update.  For
// small m n this costs less than the product tile, the screening and the
// workgroup barriers it replaces.  A and the equality data are read at
// wave-uniform addresses (scalar loads); the walks are independent, so
// there is no barrier and no LDS.
//
// The directions are bitwise those of the other paths: the draws come from
// the same counter streams, and A_eq h is summed in the order of their
// wave reduction (one product per lane, then pairwise halving), which a
// single lane can replay because n <= 32.
#include <math.h>

#include "mhar_device.hpp"
#include "mhar_internal.hpp"

namespace mhar {

namespace {

constexpr int kLaneThreads = 64;
constexpr int kLaneMaxN = 32;   // x and d of a walk in registers

template <int NM>   // compile-time bound on n (power of two, <= 32)
__global__ __launch_bounds__(kLaneThreads) void lane_kernel(StepArgs a)
{
    static_assert(NM <= 32 && (NM & (NM - 1)) == 0, "NM: power of two up to 32");
    const int chain = blockIdx.x * kLaneThreads + threadIdx.x;
    if (chain >= a.z) return;
    const int n = a.n, m = a.m, lda = a.lda;
    const double* __restrict__ A = a.A64;
    const double* __restrict__ b = a.b64;

    double x[NM];
#pragma unroll
    for (int j = 0; j < NM; ++j) x[j] = j < n ? a.X[(size_t)chain * lda + j] : 0.0;
    int fl = 0;
    double theta = a.theta[chain];

    // exact slack of every row at the launch's start and every R steps
    // (where the other paths recompute it): start point strictly inside?
    auto check_interior = [&]() __attribute__((always_inline)) {
        for (int i = 0; i < m; ++i) {
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

        // ---- directions: N(0, 1) pairs, then d = h - W (A_eq h) ----
        double d[NM];
#pragma unroll
        for (int p = 0; p < NM / 2; ++p) {
            d[2 * p] = 0.0;
            d[2 * p + 1] = 0.0;
            if (2 * p < n) {
                Block4 w = stream_block(a.seed, kTagDir, a.chain_offset + (uint32_t)chain, step, (uint32_t)p);
                double ev, od;
                gauss_pair(w, ev, od);
                d[2 * p] = ev;
                if (2 * p + 1 < n) d[2 * p + 1] = od;
            }
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
                const double* er = a.Aeq + (size_t)p * lda;
                double t[NM];
#pragma unroll
                for (int j = 0; j < NM; ++j) t[j] = j < n ? fma(er[j], h[j], 0.0) : 0.0;
#pragma unroll
                for (int half = NM / 2; half > 0; half >>= 1)
#pragma unroll
                    for (int j = 0; j < half; ++j) t[j] = t[j] + t[j + half];
                const double y = t[0];
                const double* wr = a.WT + (size_t)p * lda;
#pragma unroll
                for (int j = 0; j < NM; ++j)
                    if (j < n) d[j] = fma(-wr[j], y, d[j]);
            }
        }

        // ---- chord: every row exactly (S4.4, Lemma 4.2) ----
        unsigned long long lmax_b = (unsigned long long)__double_as_longlong(kInfD);
        unsigned long long nlmin_b = lmax_b;
        // rows are independent: unrolled so that their dependent chains overlap
#pragma unroll 4
        for (int i = 0; i < m; ++i) {
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
                const unsigned long long q = (unsigned long long)__double_as_longlong(sx / gx);
                lmax_b = q < lmax_b ? q : lmax_b;
            } else if (gx < 0.0) {
                const unsigned long long q = (unsigned long long)__double_as_longlong(sx / -gx);
                nlmin_b = q < nlmin_b ? q : nlmin_b;
            }
        }

        // ---- theta and the update (S4.5, Lemma 4.3) ----
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
        if (a.rec_stride > 0 && chain < a.rec_chains) {
            const int64_t rs = a.rec_s_base + s + 1;
            if (rs % a.rec_stride == 0) {
                double* rp = a.rec_out + ((size_t)(rs / a.rec_stride - 1) * a.rec_chains + chain) * n;
#pragma unroll
                for (int j = 0; j < NM; ++j)
                    if (j < n) rp[j] = x[j];
            }
        }
    }

#pragma unroll
    for (int j = 0; j < NM; ++j)
        if (j < n) a.X[(size_t)chain * lda + j] = x[j];
    a.theta[chain] = theta;
    if (fl) atomicOr(&a.flags[chain], fl);
    // exact rows, one atomic per wave (lane 0 is live whenever any lane is)
    const unsigned long long live = __popcll(__ballot(1));
    if (threadIdx.x == 0 && a.steps > 0)
        atomicAdd(&a.counters[0], live * (unsigned long long)m * (unsigned long long)a.steps);
}

}  // namespace

bool lane_fits(int n) { return n >= 1 && n <= kLaneMaxN; }

hipError_t launch_lane(const StepArgs& a, hipStream_t stream)
{
    if (!lane_fits(a.n) || a.r > 0 || a.m_eq > kMaxMeq) return hipErrorInvalidValue;
    const dim3 grid((a.z + kLaneThreads - 1) / kLaneThreads), block(kLaneThreads);
    if (a.n <= 8) hipLaunchKernelGGL(lane_kernel<8>, grid, block, 0, stream, a);
    else if (a.n <= 16) hipLaunchKernelGGL(lane_kernel<16>, grid, block, 0, stream, a);
    else hipLaunchKernelGGL(lane_kernel<32>, grid, block, 0, stream, a);
    return hipGetLastError();
}

}  // namespace mhar
