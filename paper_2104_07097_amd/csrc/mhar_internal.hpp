// mhar_internal.hpp -- data layouts and kernel launchers shared by the host
// runtime (mhar_api.cpp) and the kernels (mhar_kernels.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace mhar {

constexpr int kChainTile = 16;   // walks per workgroup (MFMA N)
constexpr int kWaves = 8;        // waves per workgroup
constexpr int kThreads = 64 * kWaves;
constexpr int kRowGroup = 64;    // rows one wave handles per pass (4 MFMA row blocks)
constexpr int kKAlign = 32;      // padded row length (K) granularity
constexpr int kMaxN = 1152;      // LDS holds 16 padded FP64 rows of length <= kMaxN
constexpr int kMaxNResident = 256;  // longest padded row of the register-resident kernel
constexpr int kMaxNTiled = 8192; // the tiled path keeps no row of length n in LDS
constexpr int kScreenRows = 128; // tiled path: rows x walks of a screening tile
constexpr int kScreenWalks = 128;
constexpr int kRecRows = 128;    // tiled path: rows x walks of a recompute tile
constexpr int kRecWalks = 128;
constexpr int kMaxMeq = 64;
constexpr int kMaxNDikin = 4096; // the Dikin covariance fit keeps two n x n FP64 matrices

enum Prec { kFP64 = 0, kFP32 = 1, kBF16X3 = 2 };

// per-walk status bits (same values as the public header)
constexpr int kUnbounded = 1;
constexpr int kDegenerate = 2;
constexpr int kNonFinite = 4;
constexpr int kInfeasible = 8;
constexpr int kNotInterior = 16;  // internal: start point not strictly inside

inline int64_t round_up(int64_t v, int64_t a) { return (v + a - 1) / a * a; }

// Slack / screening-product buffers: for 16-walk tile t, 64-row group p and
// walk c of the tile, the group's 64 rows are consecutive:
// index ((t*(m_pad/64) + p)*16 + c)*64 + (row mod 64).  A walk's rows of one
// group are one 256-byte run (what the candidate scan reads), and an MFMA
// output lane's four rows (FP32 and BF16 products) are one 16-byte run.

struct StepArgs {
    // problem
    int n, m, m_pad, lda, m_eq;
    int prec;               // Prec of the screening operands
    const double* A64;      // m_pad x lda, zero padded
    const float* A32;       // m_pad x lda (FP32 mode)
    const __bf16* Ahi;      // m_pad x lda (BF16X3 mode)
    const __bf16* Alo;
    // the same operand in the load order of the register-resident kernel
    // (lda <= kMaxNResident): for each 16-row block R and 32-column chunk kc,
    // two 1 KB units of 64 lanes x 16 B; lane 16 g + c of unit u holds row
    // 16 R + c, FP32 columns 32 kc + 8 g + 4 u + (0..3), or the BF16 hi (u = 0)
    // or lo (u = 1) parts of columns 32 kc + 8 g + (0..7)
    const void* Apk;
    const double* b64;      // m_pad (padding rows: 1)
    const float* rownorm;   // m_pad, ||a_i|| rounded up (padding rows: 0)
    const float* absb;      // m_pad, |b_i| rounded up
    const double* Aeq;      // m_eq x lda
    const double* WT;       // m_eq x lda: rows of (A_eq A_eq^T)^{-1} A_eq
    // learned direction covariance U U^T + diag(esig^2) (r = 0: isotropic)
    int r;
    const double* U;        // n x r
    const double* esig;     // n, exp(log_sigma)
    // tiled path with a learned covariance: the screening product is split as
    // A d = A P (exp(l) o h) + (A P U) eps, a contraction over lda + rk columns
    // whose error bound follows each part's norms (rk = 0: not split)
    int rk;                 // r rounded up to 32
    const void* AUop;       // operand of A P U: rows of length lda (first rk used), FP32 or bf16 hi then lo
    const float* aun;       // m_pad, ||(A P U)_i|| rounded up
    void* Eop;              // operand of eps in the layout of Dop (first rk columns used)
    double* Hs;             // z_pad x lda, the isotropic part P (exp(l) o h) in FP64
    double* hn;             // z_pad, ||P (exp(l) o h)||
    double* en;             // z_pad, ||eps||
    double* F;              // z_pad, drift coefficient of the low-rank part of the slack
    const double* uF;       // ||U||_F (one value)
    // chains
    int z, z_pad;
    double* X;              // z_pad x lda
    double* D;              // z_pad x lda
    void* S;                // slack, tile-fragment order, FP64 (FP64 mode) or FP32
    void* G;                // last screening product, same order and type
    float* L;               // per tile: (m_pad/64) x 2 x 16 lower bounds of the chord ratios
    float* Ug;              // tiled path, same layout: upper bounds of the chord ends per group
    void* Dop;              // tiled path: direction operand, z_pad x lda (FP32, or bf16 hi then lo)
    double* dn;             // tiled path: z_pad direction norms
    double* theta;          // z_pad, last theta
    double* E;              // z_pad, slack drift coefficient
    int* flags;             // z_pad
    unsigned long long* counters;  // [0] exact rows evaluated
    uint64_t seed;
    uint32_t chain_offset;
    uint64_t step0;
    int steps;
    int recompute_first;    // run the exact slack recompute before the first step
    int pending0;           // a deferred slack update from the previous step is due
    int T0;                 // rounding count of the slack since the last recompute
    int since0;             // steps since the last recompute
    int R;                  // recompute period
    float eps_g;            // |G_hat - G| <= eps_g ||a|| ||d||
    float u_s;              // unit roundoff of the slack storage
    // row split of the resident kernel (workgroups per walk tile) and the
    // device-scope exchange buffers of a split launch
    int split;
    unsigned long long* gL;        // per tile: 3 slots x 2 x 16 exact chord-end bits
    unsigned* gbar;                // per tile: arrival counter
    int* gerr;                     // set when a group wait timed out
    // recording
    double* rec_out;
    int rec_stride;
    int rec_chains;
    int64_t rec_s_base;
    // graph replays of the tiled path: the step counter at the start of the
    // launch sequence, added to the (then relative) step arguments; else null
    const uint64_t* step_dev;
};

size_t step_lds_bytes(int prec, int lda);
// address and size of this device's static scratch (mhar_noalloc.hip)
hipError_t noalloc_scratch(void** ptr, size_t* bytes);
// one persistent launch over (problem, walk tile) units of many problems
hipError_t launch_batch(int prec, const StepArgs* descs, const int2* units, int nunits,
                        unsigned* next, int max_lda, int grid, hipStream_t stream);
int batch_blocks_per_cu(int prec, int max_lda);
// register-resident kernel for small problems (FP32 / BF16X3, lda <= 256,
// m_pad <= 16 x 512): number of workgroups per walk tile, 0 = not usable
int resident_split(int prec, int lda, int m_pad, int z_pad);
hipError_t launch_resident(int prec, const StepArgs& a, hipStream_t stream);
hipError_t launch_steps(int prec, const StepArgs& a, hipStream_t stream);
// tiled path for large problems (FP32 / BF16X3): per step a screening GEMM and
// a chords + directions kernel, and an FP64 recompute GEMM every R steps
// Optional kernel timing of the tiled path: an event pair around each launch
// (up to cap launches), with the kind of kernel of each pair.
enum TraceKind { kTraceScreen = 0, kTraceChords = 1, kTraceDirs = 2, kTraceRecompute = 3,
                 kTraceKinds = 4 };
struct KernelTrace {
    hipEvent_t* ev;   // 2 * cap events
    int* kind;        // cap
    int cap, used;
};
hipError_t launch_tiled(int prec, const StepArgs& a, hipStream_t stream,
                        KernelTrace* trace = nullptr);
// the tiled path over many problems at once: per step one grouped screening
// launch over the tile table, one grouped chords launch over the 16-walk
// units and, after the steps flagged in `due` (host array of `steps`), one
// grouped recompute launch (each tile checks its own problem's schedule)
hipError_t launch_grouped(int prec, const StepArgs* descs, const int4* stiles, int nst,
                          const int2* units, int nunits, const int4* rtiles, int nrt, int steps,
                          int first, const unsigned char* due, int any_split, hipStream_t stream);

// one-time setup
hipError_t launch_convert_problem(int prec, int n, int m, int m_pad, int lda, const double* A,
                                  const double* b, double* A64, float* A32, __bf16* Ahi,
                                  __bf16* Alo, double* b64, float* rownorm, float* absb,
                                  hipStream_t stream);
hipError_t launch_pack_operand(int prec, int m_pad, int lda, const float* A32, const __bf16* Ahi,
                               const __bf16* Alo, void* Apk, hipStream_t stream);
hipError_t launch_eq_setup(int n, int lda, int m_eq, const double* Aeq_in, const double* beq_in,
                           double* Aeq, double* beq, double* WT, int* status,
                           hipStream_t stream);
hipError_t launch_dense_projection(int n, int lda, int m_eq, const double* Aeq, const double* WT,
                                   double* P, hipStream_t stream);
hipError_t launch_copy_states(int n, int lda, int z, int z_pad, const double* src_zn,
                              double* X, hipStream_t stream);
hipError_t launch_export_states(int n, int lda, int z, const double* X, double* dst_zn,
                                hipStream_t stream);
hipError_t launch_eq_residual(int n, int lda, int z, int m_eq, const double* Aeq,
                              const double* beq, const double* X, int* flags,
                              hipStream_t stream);
// *ctr = value (add = 0) or *ctr += value (add = 1), one thread
hipError_t launch_step_counter(uint64_t* ctr, uint64_t value, int add, hipStream_t stream);
hipError_t launch_fill_i32(int* p, int64_t count, int value, hipStream_t stream);
hipError_t launch_fill_u64(unsigned long long* p, int64_t count, unsigned long long value,
                           hipStream_t stream);
hipError_t launch_export_flags(const int* flags, int z, int32_t* out, int clear_internal,
                               hipStream_t stream);

// ---- learned preconditioner (direction covariance U U^T + diag(exp(2 l))) ----
struct PrecondBufs {
    int n, r, z, lda;
    int objective;                      // 0: Gaussian NLL of the states; 1: Dikin ellipsoid
    double *U, *logsig, *esig;          // covariance factor, log scales, exp(log scales)
    double *V;                          // trained coordinates V = diag(exp(-l)) U (n x r)
    double *m1V, *m2V, *m1l, *m2l;      // Adam moments of V and l
    double *mean, *Sd, *W, *B, *H;      // n, n, n x r, z x r, n x r
    double *GB, *C, *Cinv, *K;          // r x r each
    double *gU, *gl, *rowterm, *nll;    // n x r, n, n, 2 (NLL, log det C)
    double* part;                       // split-K partial sums of H and G
    int* status;                        // sticky: nonzero once a fit step failed (updates skipped)
    // Dikin fit: the problem's rows, the log-barrier Hessian at the mean state
    // (N x N, N = n rounded up to 64) and its Cholesky factor, row weights,
    // power-iteration vectors, sqrt(diag H), H U, the solve result, lambda
    int m, m_pad, N;
    double kappa;                       // complement scale of the diagonal, (0, 1]
    const double *A64, *b64;
    double *Hm, *Lm, *wrow, *pv, *py0, *py1, *dsq, *HU, *Ysol, *lam;
    // split screening of the tiled path (StepArgs::rk): A P U in operand form
    // and its row norms, P U (FP64, m_eq > 0), ||U||_F, and per walk the
    // isotropic part of the direction, its norm, ||eps||, the low-rank drift
    int rk, prec, m_eq, z_pad;
    void *AUop, *Eop;
    float* aun;
    double *PU, *uF, *Hs, *hn, *en, *F, *AeqU;
    const double *Aeq, *WT;
};
size_t precond_bytes(int n, int r, int z, int lda, int objective, int m_pad);
void precond_carve(PrecondBufs* p, void* ws);
hipError_t launch_precond_init(const PrecondBufs& p, uint64_t seed, hipStream_t stream);
hipError_t launch_precond_set_scales(const PrecondBufs& p, hipStream_t stream);
hipError_t launch_precond_grad(const PrecondBufs& p, const double* X, hipStream_t stream);
hipError_t launch_precond_adam(const PrecondBufs& p, int64_t t, double lr, double b1, double b2,
                               double eps, hipStream_t stream);
hipError_t launch_precond_mean(const PrecondBufs& p, const double* X, hipStream_t stream);
hipError_t launch_precond_esig(const PrecondBufs& p, hipStream_t stream);
hipError_t launch_precond_w(const PrecondBufs& p, hipStream_t stream);
hipError_t launch_precond_capacitance(const PrecondBufs& p, hipStream_t stream);
// split screening: workspace bytes, carving, and A P U / ||U||_F after U changed
size_t lowrank_bytes(int prec, int n, int r, int m_pad, int lda, int z_pad, int m_eq);
void lowrank_carve(PrecondBufs* p, void* ws);
hipError_t launch_lowrank_setup(const PrecondBufs& p, hipStream_t stream);
// Dikin fit (mhar_dikin.hip)
constexpr int kDikinPowerIters = 4;   // power iterations per training step
// default complement scale of the Dikin fit: on the rotated box (n = 1000,
// rank 64) the min-marginal ESS of 5000 steps rose from 9.5 k at kappa = 1
// to 17 k at 0.1 and stayed there down to 0.01
constexpr double kDikinKappa = 0.1;
int dikin_order(int n);
size_t dikin_bytes(int n, int r, int m_pad);
void dikin_carve(PrecondBufs* p, void* ws);
hipError_t launch_dikin_init(const PrecondBufs& p, uint64_t seed, hipStream_t stream);
hipError_t launch_dikin_loss(const PrecondBufs& p, const double* X, hipStream_t stream);
hipError_t launch_dikin_train(const PrecondBufs& p, const double* X, int k_pow, double eta,
                              hipStream_t stream);

}  // namespace mhar
