// mhar_resident.hip -- register-resident MHAR step kernel for small problems
// (n <= 256, m <= 8192) on gfx950.
//
// Same method as mhar_kernels.hip (paper Alg. 2, S4.3-S4.5: directions,
// screening product on the matrix cores, certified bounds, exact FP64 chord
// of the candidate rows, theta, update), laid out so that nothing but A
// leaves the chip between steps:
//   * the slack tile (rows of this workgroup x 16 walks) lives in registers
//     and is updated eagerly (s <- s - theta g) as soon as theta is known;
//   * the states X and directions D of the 16 walks live in LDS as FP64,
//     D double-buffered: the directions of step t+1 (independent of the
//     state) are generated while the workgroup waits at the group barrier
//     of step t;
//   * the screening product G stays in the accumulators of the step; row
//     norms and |b| of the workgroup's rows are cached in LDS;
//   * candidate rows for the exact evaluation are staged into LDS with
//     wide loads, then each lane runs one sequential FP64 dot product;
//   * A is streamed with a register double buffer over a fully unrolled
//     K loop;
//   * the rows of a walk tile are split over `split` workgroups of 512
//     rows each (one per CU); each screens its rows with its own certified
//     bounds, and the group combines the exact chord ends of its walks
//     through device-scope atomics at one barrier per step.  The grid is
//     launched cooperatively, so all workgroups of a group are resident;
//     every wait is bounded in time and raises an error flag.
#include <math.h>

#include "mhar_device.hpp"
#include "mhar_internal.hpp"

namespace mhar {

namespace {

constexpr int kCandBatch = 8;  // most candidate rows staged per wave per batch
constexpr int kRowsPerWg = kWaves * kRowGroup;

struct ResLds {
    double theta[kChainTile];
    double E[kChainTile];
    double dnorm[2][kChainTile];
    double y[kChainTile * kMaxMeq];
    unsigned long long lmax_bits[kChainTile];   // exact lambda_max >= 0 as ordered bits
    unsigned long long nlmin_bits[kChainTile];  // exact -lambda_min >= 0 as ordered bits
    unsigned up[kChainTile];
    unsigned um[kChainTile];
    int flags[kChainTile];
    int cand_row[kWaves][kCandBatch];
    int cand_chain[kWaves][kCandBatch];
    alignas(16) float rownorm[kRowsPerWg];
    alignas(16) float absb[kRowsPerWg];
    unsigned long long exact;
    int ok;
};

struct ResLayout {
    size_t x_off, d_off, op_off, cb_off, st_off, total;
    int cb_rows;  // candidate rows staged per wave
};

__host__ __device__ constexpr size_t al16(size_t v) { return (v + 15) & ~(size_t)15; }

// LDS layout for a padded row length lda; the candidate buffer takes what
// is left of the 160 KB (at most kCandBatch rows per wave).
__host__ __device__ inline ResLayout res_layout(int prec, int lda)
{
    ResLayout L;
    const size_t tile64 = al16((size_t)kChainTile * (lda + 2) * 8);
    L.x_off = 0;
    L.d_off = tile64;                      // two direction buffers
    L.op_off = L.d_off + 2 * tile64;
    const size_t op = prec == kFP32 ? al16((size_t)kChainTile * (lda + 4) * 4)
                                    : al16((size_t)2 * kChainTile * (lda + 8) * 2);
    L.cb_off = L.op_off + op;
    const size_t st = al16(sizeof(ResLds));
    const size_t budget = 163840;
    const size_t used = L.cb_off + st;
    const size_t per_row = (size_t)kWaves * (lda + 2) * 8;   // rows padded by two doubles
    int rows = used < budget ? (int)((budget - used) / per_row) : 0;
    if (rows > kCandBatch) rows = kCandBatch;
    L.cb_rows = rows;
    L.st_off = L.cb_off + al16((size_t)rows * per_row);
    L.total = L.st_off + st;
    return L;
}

// Group barrier of the `split` workgroups that share a walk tile, in two
// halves so that independent work can run between them.  All exchange
// traffic uses relaxed device-scope atomics, which are performed at the
// device coherence point; a thread only arrives after the atomics it issued
// have returned (their results are consumed), so no device-scope fence is
// needed (such fences write back and invalidate the XCD's L2).
__device__ void group_arrive(unsigned* cnt)
{
    __syncthreads();
    if (threadIdx.x == 0) __hip_atomic_fetch_add(cnt, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Wait (bounded by ~1 s of wall clock) until `target` arrivals; returns
// false if the wait timed out or another group failed.
__device__ bool group_wait(unsigned* cnt, unsigned target, int* err, int* ok_lds)
{
    if (threadIdx.x == 0) {
        int ok = 1;
        const uint64_t t0 = wall_clock64();
        while (__hip_atomic_load(cnt, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
            __builtin_amdgcn_s_sleep(1);
            if (__hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
                ok = 0;
                break;
            }
            if (wall_clock64() - t0 > 100000000ull) {
                __hip_atomic_fetch_or(err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                ok = 0;
                break;
            }
        }
        *ok_lds = ok;
    }
    __syncthreads();
    return *ok_lds != 0;
}

// Wave sums of two and four values, exchanged together so that the
// exchange latencies of the values overlap.
// One data-parallel-primitive move of a double (both halves); lanes of rows
// outside row_mask receive 0.
template <int CTRL, int ROWS>
__device__ __forceinline__ double dpp_move(double x)
{
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(x), CTRL, ROWS, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(x), CTRL, ROWS, 0xf, false);
    return __hiloint2double(hi, lo);
}

// Sums of K values over the wave, all lanes get the totals: quad swaps,
// half-row and row mirrors, then the row broadcasts of lanes 15 and 31
// leave the total in lane 63.
template <int K>
__device__ __forceinline__ void wave_sums(double* q)
{
#pragma unroll
    for (int i = 0; i < K; ++i) q[i] += dpp_move<0xB1, 0xf>(q[i]);    // quad_perm 1,0,3,2
#pragma unroll
    for (int i = 0; i < K; ++i) q[i] += dpp_move<0x4E, 0xf>(q[i]);    // quad_perm 2,3,0,1
#pragma unroll
    for (int i = 0; i < K; ++i) q[i] += dpp_move<0x141, 0xf>(q[i]);   // row_half_mirror
#pragma unroll
    for (int i = 0; i < K; ++i) q[i] += dpp_move<0x140, 0xf>(q[i]);   // row_mirror
#pragma unroll
    for (int i = 0; i < K; ++i) q[i] += dpp_move<0x142, 0xa>(q[i]);   // row_bcast15 into rows 1, 3
#pragma unroll
    for (int i = 0; i < K; ++i) q[i] += dpp_move<0x143, 0xc>(q[i]);   // row_bcast31 into rows 2, 3
#pragma unroll
    for (int i = 0; i < K; ++i)
        q[i] = __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(q[i]), 63),
                                __builtin_amdgcn_readlane(__double2loint(q[i]), 63));
}

__device__ __forceinline__ void wave_sum2(double& u, double& v)
{
    double q[2] = {u, v};
    wave_sums<2>(q);
    u = q[0];
    v = q[1];
}

__device__ __forceinline__ void wave_sum4(double* q) { wave_sums<4>(q); }

static_assert(kChainTile == 2 * kWaves, "each wave owns two walks of the tile");

// 16 bytes from global memory to LDS byte address lds + 16 * lane (the LDS
// base is wave-uniform, in M0); counted by vmcnt, returns no registers.
__device__ __forceinline__ void row_to_lds(const void* src, unsigned lds)
{
    asm volatile("global_load_lds_dwordx4 %0, off" :: "v"(src), "{m0}"(lds) : "memory");
}
// Wait until no vector-memory operation of this wave is outstanding.
__device__ __forceinline__ void wait_vm_all() { __builtin_amdgcn_s_waitcnt(0 | (7 << 4) | (15 << 8)); }

template <int P, int NK>
__global__ __launch_bounds__(kThreads) void resident_kernel(StepArgs a)
{
    extern __shared__ __align__(16) unsigned char smem[];
    constexpr int lda = NK * 32;
    const ResLayout LY = res_layout(P, lda);
    double* Xt = (double*)(smem + LY.x_off);
    double* Dbuf = (double*)(smem + LY.d_off);
    unsigned char* op = smem + LY.op_off;
    double* Cb = (double*)(smem + LY.cb_off);
    ResLds* cs = (ResLds*)(smem + LY.st_off);
    const int CB = LY.cb_rows;
    constexpr int xld = lda + 2;
    constexpr int dstride = (int)(al16((size_t)kChainTile * xld * 8) / 8);

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int g = lane >> 4, c = lane & 15;
    // XCD-aware placement: consecutive workgroup ids go to different XCDs,
    // so the `split` workgroups of one tile are taken from the same XCD.
    const int split = a.split;
    int tile, slice;
    if (split > 1 && (gridDim.x % (8 * split)) == 0) {
        const int xcd = blockIdx.x & 7, k = blockIdx.x >> 3;
        tile = (k / split) * 8 + xcd;
        slice = k % split;
    } else {
        tile = blockIdx.x / split;
        slice = blockIdx.x % split;
    }
    const int c0 = tile * kChainTile;
    const int n = a.n, m = a.m, m_pad = a.m_pad;
    const int rbase = slice * kRowsPerWg;
    const int row0 = rbase + wave * kRowGroup;  // this wave's 64 rows
    const bool rows_live = row0 < m_pad;
    const bool active_c = (c0 + c) < a.z;
    unsigned long long* gL = a.gL + (size_t)tile * 3 * 2 * kChainTile;
    unsigned* gbar = a.gbar + tile;
    unsigned nbar = 0;
    const double u64 = 0x1.0p-53;

    // ---- load the tile state and the row constants ----
    for (int item = tid; item < kChainTile * xld; item += kThreads) {
        const int cl = item / xld, j = item - cl * xld;
        const int chain = c0 + cl;
        Xt[item] = (chain < a.z && j < n) ? a.X[(size_t)chain * a.lda + j] : 0.0;
        Dbuf[item] = 0.0;
        Dbuf[dstride + item] = 0.0;
    }
    for (int i = tid; i < kRowsPerWg; i += kThreads) {
        const int row = rbase + i;
        cs->rownorm[i] = row < m_pad ? a.rownorm[row] : 0.0f;
        cs->absb[i] = row < m_pad ? a.absb[row] : 0.0f;
    }
    if (tid < kChainTile) {
        cs->theta[tid] = a.theta[c0 + tid];
        cs->E[tid] = a.E[c0 + tid];
        cs->flags[tid] = 0;
    }
    if (tid == 0) cs->exact = 0;
    __syncthreads();

    // directions of global step `step` into buffer `buf`, plus their norms
    // and the matrix-core operand tile
    auto make_directions = [&](uint64_t step, int buf) __attribute__((always_inline)) {
        double* Dt = Dbuf + buf * dstride;
        const int npairs = (n + 1) >> 1;
        for (int item = tid; item < kChainTile * npairs; item += kThreads) {
            const int cl = item / npairs, p = item - cl * npairs;
            const int chain = c0 + cl;
            if (chain >= a.z) continue;
            Block4 w = stream_block(a.seed, kTagDir, a.chain_offset + (uint32_t)chain, step, (uint32_t)p);
            double ev, od;
            gauss_pair(w, ev, od);
            Dt[cl * xld + 2 * p] = ev;
            if (2 * p + 1 < n) Dt[cl * xld + 2 * p + 1] = od;
        }
        __syncthreads();
        if (a.m_eq > 0) {
            for (int pr = wave; pr < kChainTile * a.m_eq; pr += kWaves) {
                const int cl = pr / a.m_eq, p = pr - cl * a.m_eq;
                double v = 0.0;
                if (c0 + cl < a.z) {
                    const double* er = a.Aeq + (size_t)p * a.lda;
                    for (int j = lane; j < n; j += 64) v = fma(er[j], Dt[cl * xld + j], v);
                }
                v = wave_sum(v);
                if (lane == 0) cs->y[cl * kMaxMeq + p] = v;
            }
            __syncthreads();
            for (int item = tid; item < kChainTile * n; item += kThreads) {
                const int cl = item / n, j = item - cl * n;
                if (c0 + cl >= a.z) continue;
                double v = Dt[cl * xld + j];
                for (int p = 0; p < a.m_eq; ++p) v = fma(-a.WT[(size_t)p * a.lda + j], cs->y[cl * kMaxMeq + p], v);
                Dt[cl * xld + j] = v;
            }
            __syncthreads();
        }
        {
            const int cl0 = wave, cl1 = wave + kWaves;
            double v0 = 0.0, v1 = 0.0;
            for (int j = lane; j < n; j += 64) {
                v0 = fma(Dt[cl0 * xld + j], Dt[cl0 * xld + j], v0);
                v1 = fma(Dt[cl1 * xld + j], Dt[cl1 * xld + j], v1);
            }
            wave_sum2(v0, v1);
            if (lane == 0) {
                cs->dnorm[buf][cl0] = sqrt(v0);
                cs->dnorm[buf][cl1] = sqrt(v1);
            }
        }
        if (P == kFP32) {
            float* Ot = (float*)op;
            constexpr int fld = lda + 4;
            for (int item = tid; item < kChainTile * lda; item += kThreads) {
                const int cl = item / lda, j = item - cl * lda;
                Ot[cl * fld + j] = (float)Dt[cl * xld + j];
            }
        } else {
            __bf16* Oh = (__bf16*)op;
            constexpr int bld = lda + 8;
            __bf16* Ol = Oh + kChainTile * bld;
            for (int item = tid; item < kChainTile * lda; item += kThreads) {
                const int cl = item / lda, j = item - cl * lda;
                __bf16 hi, lo;
                split_bf16((float)Dt[cl * xld + j], hi, lo);
                Oh[cl * bld + j] = hi;
                Ol[cl * bld + j] = lo;
            }
        }
        __syncthreads();
    };

    float S[4][4];   // slack of rows row0 + 16 rb + 4 g + r, walk c
    int T = 2, since = a.since0;
    bool recompute_now = true;   // the slack never crosses a launch boundary
    if (a.steps > 0) make_directions(a.step0, 0);
    for (int s = 0;; ++s) {
        if (recompute_now) {
            // exact FP64 slack b - A x of this wave's rows (FP64 matrix cores)
            {
                const int cl0 = wave, cl1 = wave + kWaves;
                double v0 = 0.0, v1 = 0.0;
                for (int j = lane; j < n; j += 64) {
                    v0 = fma(Xt[cl0 * xld + j], Xt[cl0 * xld + j], v0);
                    v1 = fma(Xt[cl1 * xld + j], Xt[cl1 * xld + j], v1);
                }
                wave_sum2(v0, v1);
                if (lane == 0) {
                    const double f = (double)a.u_s * (1.0 + 0x1.0p-20) + (2.0 * n + 4.0) * u64;
                    cs->E[cl0] = f * sqrt(v0);
                    cs->E[cl1] = f * sqrt(v1);
                }
            }
            int fl = 0;
            if (rows_live) {
                f64x4 acc[4] = {{0, 0, 0, 0}, {0, 0, 0, 0}, {0, 0, 0, 0}, {0, 0, 0, 0}};
                for (int k0 = 0; k0 < lda; k0 += 16) {
                    const double2* bp = (const double2*)(Xt + c * xld + k0 + 4 * g);
                    const double2 b0 = bp[0], b1 = bp[1];
#pragma unroll
                    for (int rb = 0; rb < 4; ++rb) {
                        const double2* ap = (const double2*)(a.A64 + (size_t)(row0 + 16 * rb + c) * a.lda + k0 + 4 * g);
                        const double2 a0 = ap[0], a1 = ap[1];
                        acc[rb] = mma_f64(a0.x, b0.x, acc[rb]);
                        acc[rb] = mma_f64(a0.y, b0.y, acc[rb]);
                        acc[rb] = mma_f64(a1.x, b1.x, acc[rb]);
                        acc[rb] = mma_f64(a1.y, b1.y, acc[rb]);
                    }
                }
#pragma unroll
                for (int rb = 0; rb < 4; ++rb) {
                    float sv[4];
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        // FP64 output: lane (g, c) slot r holds row 4r + g
                        const int row = row0 + 16 * rb + 4 * r + g;
                        const double bi = a.b64[row];
                        const double sx = bi - acc[rb][r];
                        if (active_c && row < m) {
                            if (!(sx > 0.0)) fl |= kNotInterior;
                            if (sx < -1e-12 * fmax(1.0, fabs(bi))) fl |= kInfeasible;
                        }
                        sv[r] = (float)sx;
                    }
                    // operand order: lane (g, c) slot r holds row 4g + r, the
                    // value of lane (r, c) slot g
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const float v0 = __shfl(sv[0], 16 * r + c, 64);
                        const float v1 = __shfl(sv[1], 16 * r + c, 64);
                        const float v2 = __shfl(sv[2], 16 * r + c, 64);
                        const float v3 = __shfl(sv[3], 16 * r + c, 64);
                        S[rb][r] = g == 0 ? v0 : g == 1 ? v1 : g == 2 ? v2 : v3;
                    }
                }
            }
            if (fl) atomicOr(&cs->flags[c], fl);
            T = 2;
            if (s > 0) since = 0;
            recompute_now = false;
            __syncthreads();
        }
        if (s >= a.steps) break;
        const uint64_t step = a.step0 + (uint64_t)s;
        const int buf = s & 1;
        const double* Dt = Dbuf + buf * dstride;
        if (tid < kChainTile) {
            cs->up[tid] = __float_as_uint(kInf);
            cs->um[tid] = __float_as_uint(kInf);
            cs->lmax_bits[tid] = __double_as_longlong(kInfD);
            cs->nlmin_bits[tid] = __double_as_longlong(kInfD);
        }

        // ---------------- B: screening product (this wave's 64 rows) ----------------
        f32x4 acc[4] = {{0, 0, 0, 0}, {0, 0, 0, 0}, {0, 0, 0, 0}, {0, 0, 0, 0}};
        if (rows_live) {
            if (P == kFP32) {
                const float* Ot = (const float*)op;
                constexpr int fld = lda + 4;
                float4 bufa[2][8];
                // packed operand: each load is one contiguous 1 KB unit
                // (wave-uniform base + the lane's 16-byte slot)
                const char* Ab = (const char*)a.Apk + (size_t)(__builtin_amdgcn_readfirstlane(row0) >> 4) * NK * 2048;
                const unsigned loff = 16u * lane;
                auto load = [&](float4* dst, int kc) __attribute__((always_inline)) {
#pragma unroll
                    for (int rb = 0; rb < 4; ++rb) {
                        const char* ap = Ab + (size_t)(rb * NK + kc) * 2048 + loff;
                        dst[2 * rb] = *(const float4*)ap;
                        dst[2 * rb + 1] = *(const float4*)(ap + 1024);
                    }
                };
                load(bufa[0], 0);
#pragma unroll
                for (int kc = 0; kc < NK; ++kc) {
                    if (kc + 1 < NK) load(bufa[(kc + 1) & 1], kc + 1);
                    const float4* bp = (const float4*)(Ot + c * fld + kc * 32 + 8 * g);
                    const float4 b0 = bp[0], b1 = bp[1];
                    const float4* cur = bufa[kc & 1];
#pragma unroll
                    for (int e = 0; e < 8; ++e) {
                        const float bv = e < 4 ? (&b0.x)[e] : (&b1.x)[e - 4];
#pragma unroll
                        for (int rb = 0; rb < 4; ++rb) {
                            const float av = e < 4 ? (&cur[2 * rb].x)[e] : (&cur[2 * rb + 1].x)[e - 4];
                            acc[rb] = mma_f32(av, bv, acc[rb]);
                        }
                    }
                }
            } else {
                const __bf16* Oh = (const __bf16*)op;
                constexpr int bld = lda + 8;
                const __bf16* Ol = Oh + kChainTile * bld;
                bf16x8 bufa[2][8];
                // packed operand: hi and lo parts, each one contiguous 1 KB unit
                const char* Ab = (const char*)a.Apk + (size_t)(__builtin_amdgcn_readfirstlane(row0) >> 4) * NK * 2048;
                const unsigned loff = 16u * lane;
                auto load = [&](bf16x8* dst, int kc) __attribute__((always_inline)) {
#pragma unroll
                    for (int rb = 0; rb < 4; ++rb) {
                        const char* ap = Ab + (size_t)(rb * NK + kc) * 2048 + loff;
                        dst[2 * rb] = *(const bf16x8*)ap;
                        dst[2 * rb + 1] = *(const bf16x8*)(ap + 1024);
                    }
                };
                load(bufa[0], 0);
#pragma unroll
                for (int kc = 0; kc < NK; ++kc) {
                    if (kc + 1 < NK) load(bufa[(kc + 1) & 1], kc + 1);
                    const bf16x8 bh = *(const bf16x8*)(Oh + c * bld + kc * 32 + 8 * g);
                    const bf16x8 bl = *(const bf16x8*)(Ol + c * bld + kc * 32 + 8 * g);
                    const bf16x8* cur = bufa[kc & 1];
#pragma unroll
                    for (int rb = 0; rb < 4; ++rb) acc[rb] = mma_bf16(cur[2 * rb + 1], bh, acc[rb]);
#pragma unroll
                    for (int rb = 0; rb < 4; ++rb) acc[rb] = mma_bf16(cur[2 * rb], bl, acc[rb]);
#pragma unroll
                    for (int rb = 0; rb < 4; ++rb) acc[rb] = mma_bf16(cur[2 * rb], bh, acc[rb]);
                }
            }
        }

        // ---------------- screening: certified bounds, candidate list ----------------
        // Every workgroup screens its rows with its own upper bounds of the
        // chord ends; they can only exceed the bounds over all rows, so the
        // candidate set is a superset of the one the global bound would give.
        // Pass 1 takes the upper bound of each entry's ratio, (s + dl) / (|g| - e)
        // where |g| > e surely, and the minimum per walk and side.  Pass 2
        // keeps the entries whose lower bound max(s - dl, 0) / (|g| + e) can
        // reach that minimum, tested as a product so that no second
        // reciprocal is needed; the same for the other side where |g| < e.
        const float ed = active_c ? (float)(cs->dnorm[buf][c] * (double)a.eps_g) * kHighGrow + 1e-30f : 0.0f;
        const float Ek = (float)cs->E[c] * kHighGrow;
        const float bscale = a.u_s * (float)T * kHighGrow;
        float dls[4][4];
        {
            float up = kInf, um = kInf;
#pragma unroll
            for (int rb = 0; rb < 4; ++rb) {
                const int li0 = wave * kRowGroup + 16 * rb + 4 * g;   // rows li0 .. li0 + 3
                const float4 na4 = *(const float4*)&cs->rownorm[li0];
                const float4 ab4 = *(const float4*)&cs->absb[li0];
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const float na = (&na4.x)[r], ab = (&ab4.x)[r];
                    const float dl = fmaf(na, Ek, fmaf(bscale, ab, 1e-30f));
                    dls[rb][r] = dl;
                    const float gv = acc[rb][r];
                    const float den = fabsf(gv) - na * ed;
                    float h = (S[rb][r] + dl) * __builtin_amdgcn_rcpf(den);
                    h = den > 0.0f ? h : kInf;
                    up = fminf(up, gv > 0.0f ? h : kInf);
                    um = fminf(um, gv < 0.0f ? h : kInf);
                }
            }
            up = fminf(up, __shfl_xor(up, 16, 64));
            up = fminf(up, __shfl_xor(up, 32, 64));
            um = fminf(um, __shfl_xor(um, 16, 64));
            um = fminf(um, __shfl_xor(um, 32, 64));
            __syncthreads();   // the resets above are done
            if (g == 0) {
                atomicMin(&cs->up[c], __float_as_uint(up));
                atomicMin(&cs->um[c], __float_as_uint(um));
            }
        }
        __syncthreads();
        // candidate bits of this lane's 16 entries (slot 4 rb + r)
        unsigned cbits = 0;
        {
            // kScreenSlack covers the roundings of both ratio bounds and of
            // the products below
            const float Up = __uint_as_float(cs->up[c]) * kScreenSlack;
            const float Um = __uint_as_float(cs->um[c]) * kScreenSlack;
#pragma unroll
            for (int rb = 0; rb < 4; ++rb) {
                const int li0 = wave * kRowGroup + 16 * rb + 4 * g;
                const float4 na4 = *(const float4*)&cs->rownorm[li0];
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int row = row0 + 16 * rb + 4 * g + r;
                    const float e = (&na4.x)[r] * ed;
                    const float gv = acc[rb][r], ag = fabsf(gv);
                    const float slo = fmaxf(S[rb][r] - dls[rb][r], 0.0f);
                    const bool pos = gv >= 0.0f;
                    const float us = pos ? Up : Um, uo = pos ? Um : Up;
                    const float go = e - ag;
                    const bool cand = slo <= us * (ag + e) || (go > 0.0f && slo <= uo * go) || slo <= kTinySlack;
                    if (active_c && row < m && cand) cbits |= 1u << (4 * rb + r);
                }
            }
        }

        // ---------------- C: exact chords of the candidate rows ----------------
        {
            constexpr int cld = lda + 2;          // padded: candidate rows on distinct banks
            constexpr int kPer = (lda + 127) / 128;
            double* cb = Cb + (size_t)wave * CB * cld;
            int total = 0;
#pragma unroll
            for (int k = 0; k < 16; ++k) total += __popcll(__ballot((cbits >> k) & 1u));
            for (int base = 0; base < total; base += CB) {
                const int cnt = min(CB, total - base);
                // list: position of an entry = its rank in (slot, lane) order
                int off = 0;
#pragma unroll
                for (int k = 0; k < 16; ++k) {
                    const bool f = (cbits >> k) & 1u;
                    const unsigned long long bk = __ballot(f);
                    const int pos = off - base +
                                    (int)__builtin_amdgcn_mbcnt_hi((unsigned)(bk >> 32),
                                                                   __builtin_amdgcn_mbcnt_lo((unsigned)bk, 0u));
                    if (f && pos >= 0 && pos < cnt) {
                        cs->cand_row[wave][pos] = row0 + 16 * (k >> 2) + 4 * g + (k & 3);
                        cs->cand_chain[wave][pos] = c;
                    }
                    off += __popcll(bk);
                }
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_wave_barrier();
                // each lane < cnt evaluates one candidate
                int rr = 0, cc = 0;
                double bi = 0.0;
                if (lane < cnt) {
                    rr = cs->cand_row[wave][lane];
                    cc = cs->cand_chain[wave][lane];
                    bi = a.b64[rr];
                }
                // stage the rows straight from global memory into LDS, one
                // instruction per 128 coordinates of a row, all in flight at
                // once (no registers held; the wave reads only its own rows)
#pragma unroll
                for (int q = 0; q < kCandBatch; ++q) {
                    if (q < cnt) {
                        const double* ar = a.A64 + (size_t)cs->cand_row[wave][q] * a.lda;
                        const unsigned dst = (unsigned)(size_t)(cb + q * cld);
#pragma unroll
                        for (int t = 0; t < kPer; ++t) {
                            const int j = 2 * lane + 128 * t;
                            if (j < lda) row_to_lds(ar + j, dst + 1024u * t);
                        }
                    }
                }
                wait_vm_all();
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_wave_barrier();
                // the line-set formula of S4.4 in the operation order of a
                // sequential FP64 evaluation: lane q < cnt sums the slack
                // b - a.x of candidate q, lane 32 + q its a.d (a - b is
                // summed as a + (-b), which rounds the same)
                const int qh = lane & 31;
                const int cq = __shfl(cc, qh, 64);   // all lanes take part in the exchange
                double sum = 0.0;
                if (qh < cnt) {
                    const bool slack = lane < 32;
                    const double* av = cb + qh * cld;
                    const double* vv = (slack ? Xt : Dt) + cq * xld;
                    const unsigned flip = slack ? 0x80000000u : 0u;
                    sum = slack ? bi : 0.0;
                    int j = 0;
                    for (; j + 8 <= n; j += 8) {
                        double a8[8], v8[8];
#pragma unroll
                        for (int e = 0; e < 8; ++e) {
                            a8[e] = av[j + e];
                            v8[e] = vv[j + e];
                        }
#pragma unroll
                        for (int e = 0; e < 8; ++e) {
                            double t = __dmul_rn(a8[e], v8[e]);
                            t = __hiloint2double(__double2hiint(t) ^ (int)flip, __double2loint(t));
                            sum = __dadd_rn(sum, t);
                        }
                    }
                    for (; j < n; ++j) {
                        double t = __dmul_rn(av[j], vv[j]);
                        t = __hiloint2double(__double2hiint(t) ^ (int)flip, __double2loint(t));
                        sum = __dadd_rn(sum, t);
                    }
                }
                const double gsum = __shfl(sum, qh + 32, 64);
                if (lane < cnt) {
                    double sx = sum;
                    const double gx = gsum;
                    int fl = 0;
                    if (sx < -1e-12 * fmax(1.0, fabs(bi))) fl |= kInfeasible;
                    if (sx < 0.0) sx = 0.0;
                    if (gx > 0.0)
                        atomicMin(&cs->lmax_bits[cc], (unsigned long long)__double_as_longlong(sx / gx));
                    else if (gx < 0.0)
                        atomicMin(&cs->nlmin_bits[cc], (unsigned long long)__double_as_longlong(sx / -gx));
                    if (fl) atomicOr(&cs->flags[cc], fl);
                }
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_wave_barrier();
            }
            if (lane == 0 && total) atomicAdd(&cs->exact, (unsigned long long)total);
        }
        __syncthreads();

        // ---- combine the exact chord ends of the group; meanwhile the
        //      directions of the next step are generated ----
        const int xslot = (int)(step % 3);
        if (split > 1) {
            if (tid < kChainTile) {
                // results consumed: the atomics are performed before arrival
                const unsigned long long o0 = __hip_atomic_fetch_min(
                    &gL[(xslot * 2 + 0) * kChainTile + tid], cs->lmax_bits[tid], __ATOMIC_RELAXED,
                    __HIP_MEMORY_SCOPE_AGENT);
                const unsigned long long o1 = __hip_atomic_fetch_min(
                    &gL[(xslot * 2 + 1) * kChainTile + tid], cs->nlmin_bits[tid], __ATOMIC_RELAXED,
                    __HIP_MEMORY_SCOPE_AGENT);
                if (o0 == ~0ull || o1 == ~0ull) cs->ok = 3;   // never true: forces the wait
            }
            nbar += 1;
            group_arrive(gbar);
        }
        if (s + 1 < a.steps) make_directions(step + 1, buf ^ 1);
        if (split > 1) {
            if (!group_wait(gbar, nbar * (unsigned)split, a.gerr, &cs->ok)) break;
            if (tid < kChainTile) {
                cs->lmax_bits[tid] = __hip_atomic_load(&gL[(xslot * 2 + 0) * kChainTile + tid],
                                                       __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                cs->nlmin_bits[tid] = __hip_atomic_load(&gL[(xslot * 2 + 1) * kChainTile + tid],
                                                        __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
            // every workgroup has read the slot of the previous step
            if (slice == 0 && tid < 2 * kChainTile) {
                const unsigned long long o = __hip_atomic_exchange(
                    &gL[(int)((step + 2) % 3) * 2 * kChainTile + tid],
                    (unsigned long long)__double_as_longlong(kInfD), __ATOMIC_RELAXED,
                    __HIP_MEMORY_SCOPE_AGENT);
                if (o == ~0ull) cs->ok = 3;   // never true: forces the wait
            }
            __syncthreads();
        }

        // ---------------- D: theta, eager slack update, state update ----------------
        // every wave computes theta of all 16 walks (lanes 0-15), so the
        // slack update needs no further barrier
        double th_l = 0.0;
        int fl_l = 0;
        if (lane < kChainTile) {
            const int chain = c0 + lane;
            if (chain < a.z) {
                const double lmax = __longlong_as_double((long long)cs->lmax_bits[lane]);
                const double lmin = -__longlong_as_double((long long)cs->nlmin_bits[lane]);
                if (lmax == kInfD || lmin == -kInfD) {
                    fl_l = kUnbounded;
                } else if (!(lmax > lmin)) {
                    fl_l = kDegenerate;
                } else {
                    Block4 w = stream_block(a.seed, kTagTheta, a.chain_offset + (uint32_t)chain, step, 0);
                    const double u = open_unit(w.w0, w.w1);
                    th_l = __dadd_rn(lmin, __dmul_rn(u, __dsub_rn(lmax, lmin)));
                }
            }
        }
        const double th_c = __shfl(th_l, c, 64);
        {
            const float th32 = (float)th_c;
#pragma unroll
            for (int rb = 0; rb < 4; ++rb)
#pragma unroll
                for (int r = 0; r < 4; ++r) S[rb][r] = fmaf(-th32, acc[rb][r], S[rb][r]);
        }
        if (wave == 0 && lane < kChainTile) {
            cs->theta[lane] = th_l;
            if (fl_l) cs->flags[lane] |= fl_l;
        }
        {
            // the two walks of this wave, updated together
            const int cl0 = wave, cl1 = wave + kWaves;
            const bool v0 = c0 + cl0 < a.z, v1 = c0 + cl1 < a.z;
            const double th0 = __shfl(th_l, cl0, 64), th1 = __shfl(th_l, cl1, 64);
            const int64_t rs = a.rec_s_base + s + 1;
            const bool recs = slice == 0 && a.rec_stride > 0 && (rs % a.rec_stride) == 0;
            const bool rec0 = recs && v0 && c0 + cl0 < a.rec_chains;
            const bool rec1 = recs && v1 && c0 + cl1 < a.rec_chains;
            double* rp0 = rec0 ? a.rec_out + ((size_t)(rs / a.rec_stride - 1) * a.rec_chains + c0 + cl0) * n : nullptr;
            double* rp1 = rec1 ? a.rec_out + ((size_t)(rs / a.rec_stride - 1) * a.rec_chains + c0 + cl1) * n : nullptr;
            double q[4] = {0.0, 0.0, 0.0, 0.0};   // |x|^2, |x'|^2 of both walks
            bool fin0 = isfinite(th0), fin1 = isfinite(th1);
            for (int j = lane; j < n; j += 64) {
                if (v0) {
                    const double xv = Xt[cl0 * xld + j];
                    const double xnew = __dadd_rn(xv, __dmul_rn(th0, Dt[cl0 * xld + j]));
                    Xt[cl0 * xld + j] = xnew;
                    if (rec0) rp0[j] = xnew;
                    q[0] = fma(xv, xv, q[0]);
                    q[1] = fma(xnew, xnew, q[1]);
                    fin0 = fin0 && isfinite(xnew);
                }
                if (v1) {
                    const double xv = Xt[cl1 * xld + j];
                    const double xnew = __dadd_rn(xv, __dmul_rn(th1, Dt[cl1 * xld + j]));
                    Xt[cl1 * xld + j] = xnew;
                    if (rec1) rp1[j] = xnew;
                    q[2] = fma(xv, xv, q[2]);
                    q[3] = fma(xnew, xnew, q[3]);
                    fin1 = fin1 && isfinite(xnew);
                }
            }
            wave_sum4(q);
            fin0 = __all(fin0);
            fin1 = __all(fin1);
            if (lane < 2) {
                // bound on the slack error carried into the next step
                auto grow_E = [&](int cl, double th, double xo, double xn2, bool finite) {
                    const double dn = cs->dnorm[buf][cl], at = fabs(th);
                    const double us = (double)a.u_s;
                    double E = cs->E[cl];
                    E += at * dn * ((double)a.eps_g + 2.0 * us);
                    E += 2.0 * u64 * (sqrt(xo) + at * dn);
                    E += us * (1.0 + 0x1.0p-20) * sqrt(xn2);
                    cs->E[cl] = E;
                    if (!finite) cs->flags[cl] |= kNonFinite;
                };
                // lanes 0 and 1 grow the bounds of the two walks side by side
                const bool second = lane == 1;
                if (second ? v1 : v0)
                    grow_E(second ? cl1 : cl0, second ? th1 : th0, second ? q[2] : q[0],
                           second ? q[3] : q[1], second ? fin1 : fin0);
            }
        }
        __syncthreads();
        T += 1;
        since += 1;
        recompute_now = since >= a.R;
    }

    // ---- write the tile state back ----
    __syncthreads();
    if (slice == 0) {
        for (int item = tid; item < kChainTile * n; item += kThreads) {
            const int cl = item / n, j = item - cl * n;
            const int chain = c0 + cl;
            if (chain < a.z) a.X[(size_t)chain * a.lda + j] = Xt[cl * xld + j];
        }
        if (tid < kChainTile) {
            a.theta[c0 + tid] = cs->theta[tid];
            a.E[c0 + tid] = cs->E[tid];
        }
    }
    if (tid < kChainTile) {
        const int chain = c0 + tid;
        if (cs->flags[tid] && chain < a.z) atomicOr(&a.flags[chain], cs->flags[tid]);
    }
    if (tid == 0 && cs->exact) atomicAdd(&a.counters[0], cs->exact);
}

template <int P, int NK>
hipError_t launch_res(const StepArgs& a, hipStream_t stream)
{
    const size_t lds = res_layout(P, NK * 32).total;
    const void* fn = (const void*)resident_kernel<P, NK>;
    hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    const dim3 grid((a.z_pad / kChainTile) * a.split), block(kThreads);
    if (a.split > 1) {
        StepArgs copy = a;
        void* args[] = {&copy};
        return hipLaunchCooperativeKernel(fn, grid, block, args, (unsigned)lds, stream);
    }
    hipLaunchKernelGGL((resident_kernel<P, NK>), grid, block, lds, stream, a);
    return hipGetLastError();
}

template <int P, int NK>
int res_blocks_per_cu()
{
    int nb = 0;
    const size_t lds = res_layout(P, NK * 32).total;
    if (hipFuncSetAttribute((const void*)resident_kernel<P, NK>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, (const void*)resident_kernel<P, NK>, kThreads, lds) != hipSuccess) {
        (void)hipGetLastError();   // do not leave a stale error for the next launch
        return 0;
    }
    return nb;
}

template <int P>
hipError_t launch_res_nk(const StepArgs& a, hipStream_t stream)
{
    switch (a.lda / 32) {
    case 1: return launch_res<P, 1>(a, stream);
    case 2: return launch_res<P, 2>(a, stream);
    case 3: return launch_res<P, 3>(a, stream);
    case 4: return launch_res<P, 4>(a, stream);
    case 5: return launch_res<P, 5>(a, stream);
    case 6: return launch_res<P, 6>(a, stream);
    case 7: return launch_res<P, 7>(a, stream);
    case 8: return launch_res<P, 8>(a, stream);
    default: return hipErrorInvalidValue;
    }
}

template <int P>
int res_occupancy(int lda)
{
    switch (lda / 32) {
    case 1: return res_blocks_per_cu<P, 1>();
    case 2: return res_blocks_per_cu<P, 2>();
    case 3: return res_blocks_per_cu<P, 3>();
    case 4: return res_blocks_per_cu<P, 4>();
    case 5: return res_blocks_per_cu<P, 5>();
    case 6: return res_blocks_per_cu<P, 6>();
    case 7: return res_blocks_per_cu<P, 7>();
    case 8: return res_blocks_per_cu<P, 8>();
    default: return 0;
    }
}

}  // namespace

int resident_split(int prec, int lda, int m_pad, int z_pad)
{
    if (prec != kFP32 && prec != kBF16X3) return 0;
    if (lda > kMaxNResident || res_layout(prec, lda).cb_rows < 1) return 0;
    const int rows = kWaves * kRowGroup;
    const int split = (m_pad + rows - 1) / rows;
    if (split > 16) return 0;
    if (split == 1) return 1;
    // a split launch is cooperative: the whole grid must be resident
    int dev = 0, cus = 0, coop = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, dev) != hipSuccess || !coop) return 0;
    const int per_cu = prec == kFP32 ? res_occupancy<kFP32>(lda) : res_occupancy<kBF16X3>(lda);
    const long grid = (long)(z_pad / kChainTile) * split;
    if (per_cu < 1 || grid > (long)per_cu * cus) return 0;
    return split;
}

hipError_t launch_resident(int prec, const StepArgs& a, hipStream_t stream)
{
    if (prec == kFP32) return launch_res_nk<kFP32>(a, stream);
    if (prec == kBF16X3) return launch_res_nk<kBF16X3>(a, stream);
    return hipErrorInvalidValue;
}

}  // namespace mhar
