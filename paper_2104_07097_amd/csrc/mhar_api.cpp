// mhar_api.cpp -- host runtime behind the C ABI of include/mhar.h:
// argument checking, workspace planning, handle state and kernel launches.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/mhar.h"
#include "mhar_internal.hpp"

using namespace mhar;

namespace mhar {
// a few lanes per walk, every row exact (mhar_lane.hip)
bool lane_fits(int n, int m);
hipError_t launch_lane(const StepArgs& a, hipStream_t stream);
}  // namespace mhar

struct mhar_problem {
    int n, m, m_pad, lda, m_eq, prec, R, steps_per_launch, path;
    float eps_g, u_s;
    double *A64, *b64, *Aeq, *beq, *WT;
    float *A32, *rownorm, *absb;
    __bf16 *Ahi, *Alo;
    void* Apk;   // operand in the resident kernel's load order (nullptr if unused)
    int* status;
    int live_chains;
};

struct mhar_chains {
    mhar_problem* p;
    int z, z_pad;
    int split;  // > 0: register-resident kernel with this many workgroups per walk tile
    int tiled;  // 1: tiled path (screening GEMM + chords kernel per step)
    int lane;   // 1: lane path, every row exact (isotropic directions only)
    int slack_stale;  // the lane path ran since the last slack recompute
    int last_kernel;  // mhar_path_t of the last launch
    uint64_t seed;
    uint32_t chain_offset;
    uint64_t step;
    int pending, T, since;
    uint64_t recomputes;
    double *X, *D, *theta, *E;
    void *S, *G;
    float* L;
    float* Ug;
    void* Dop;
    double* dn;
    int* flags;
    unsigned long long* counters;
    unsigned long long* gL;
    unsigned* gbar;
    int* gerr;
    // learned direction covariance
    int pc_rank;        // 0: isotropic directions
    int pc_frozen;
    int64_t pc_t;       // Adam step counter
    int split_saved;    // kernel choice before the covariance was attached
    int force_recompute;
    int pc_lr_stale;    // tiled path: A P U must be recomputed before the next step
    float pc_eps_g;     // error coefficient of the split screening (n + rank terms)
    PrecondBufs pc;
    // kernel timing of the tiled path (mhar_trace_enable)
    KernelTrace trace{nullptr, nullptr, 0, 0};
    std::vector<hipEvent_t> trace_events;
    std::vector<int> trace_kinds;
    // graph replays of the tiled path (mhar_chains_set_graph)
    uint64_t* gstep;                   // device step counter of the replays
    int graph_steps = 0;               // steps per graph, 0: off
    hipGraphExec_t graph_exec = nullptr;
    hipStream_t cap_stream = nullptr;  // private stream the graph is captured on
    StepArgs graph_key{};              // the arguments it was captured with
};

struct mhar_batch {
    int count;
    int prec;
    std::vector<mhar_chains*> chains;
    std::vector<int> saved_split, saved_tiled;
    StepArgs* descs_dev;
    int2* units_dev;
    unsigned* next_dev;
    StepArgs* descs_host;   // pinned
    hipEvent_t copied;
    bool copy_pending;
    int nunits, max_lda, grid;      // general-kernel units (small problems)
    double work_per_step;
    // large problems: grouped tiled launches over a table of tiles
    int ntu, nst, nrt;              // chords units, screening tiles, recompute tiles
    int2* tunits_dev;
    int4* stiles_dev;
    int4* rtiles_dev;
    std::vector<unsigned char> due; // per step of a launch: some problem recomputes after it
    // packed creation: the batch owns its problems and chains handles
    std::vector<mhar_problem*> owned_problems;
    bool owns_chains = false;
};

namespace {

thread_local std::string g_last_error;

mhar_status_t fail(mhar_status_t code, const std::string& msg)
{
    g_last_error = msg;
    return code;
}

mhar_status_t hip_fail(hipError_t e, const char* what)
{
    return fail(MHAR_E_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

#define MHAR_HIP(call, what)                             \
    do {                                                 \
        hipError_t e_ = (call);                          \
        if (e_ != hipSuccess) return hip_fail(e_, what); \
    } while (0)

// Sequential carving of a workspace into 256-byte aligned pieces.
struct Carver {
    char* base;
    size_t used = 0;
    explicit Carver(void* b) : base((char*)b) {}
    template <class T> T* take(size_t count)
    {
        used = (size_t)round_up((int64_t)used, 256);
        T* p = base ? (T*)(base + used) : nullptr;
        used += count * sizeof(T);
        return p;
    }
};

struct ProblemDims {
    int n, m, m_pad, lda, m_eq;
};

mhar_status_t check_options(const mhar_options_t* opt, mhar_options_t* out)
{
    mhar_options_default(out);
    if (!opt) return MHAR_OK;
    if (opt->precision < MHAR_FP64 || opt->precision > MHAR_BF16X3)
        return fail(MHAR_E_INVALID_ARG, "options.precision must be MHAR_FP64, MHAR_FP32 or MHAR_BF16X3");
    if (opt->recompute_every < 1)
        return fail(MHAR_E_INVALID_ARG, "options.recompute_every must be >= 1");
    if (opt->recompute_every > 100000)
        return fail(MHAR_E_INVALID_ARG, "options.recompute_every must be <= 100000");
    if (opt->steps_per_launch < 0)
        return fail(MHAR_E_INVALID_ARG, "options.steps_per_launch must be >= 0");
    if (opt->path < MHAR_PATH_AUTO || opt->path > MHAR_PATH_LANE)
        return fail(MHAR_E_INVALID_ARG, "options.path must be a mhar_path_t value");
    if (opt->path == MHAR_PATH_TILED && opt->precision == MHAR_FP64)
        return fail(MHAR_E_UNSUPPORTED, "the tiled path screens in FP32 or BF16X3 only");
    for (int i = 0; i < 4; ++i)
        if (opt->reserved[i] != 0) return fail(MHAR_E_INVALID_ARG, "options.reserved must be 0");
    *out = *opt;
    return MHAR_OK;
}

// n above kMaxN is served by the tiled path only (FP32 / BF16X3, path AUTO or TILED)
mhar_status_t check_dims(int64_t n, int64_t m, int64_t m_eq, const mhar_options_t& o,
                         ProblemDims* d)
{
    const bool tiled_ok = o.precision != MHAR_FP64 &&
                          (o.path == MHAR_PATH_AUTO || o.path == MHAR_PATH_TILED);
    const int64_t nmax = tiled_ok ? kMaxNTiled : kMaxN;
    if (n < 1 || n > nmax)
        return fail(MHAR_E_SHAPE, "n must be in [1, " + std::to_string(nmax) + "] for this precision and path");
    if (m < 1 || m > (int64_t(1) << 24)) return fail(MHAR_E_SHAPE, "m must be in [1, 2^24]");
    if (m_eq < 0 || m_eq > kMaxMeq || m_eq >= n)
        return fail(MHAR_E_SHAPE, "m_eq must be in [0, min(64, n-1)]");
    d->n = (int)n;
    d->m = (int)m;
    d->m_eq = (int)m_eq;
    d->m_pad = (int)round_up(m, kRowGroup);
    d->lda = (int)round_up(n, kKAlign);
    return MHAR_OK;
}

size_t carve_problem(const ProblemDims& d, int prec, void* ws, mhar_problem* p)
{
    Carver c(ws);
    mhar_problem tmp{};
    mhar_problem* q = p ? p : &tmp;
    size_t mat = (size_t)d.m_pad * d.lda;
    q->A64 = c.take<double>(mat);
    q->A32 = prec == MHAR_FP32 ? c.take<float>(mat) : nullptr;
    q->Ahi = prec == MHAR_BF16X3 ? c.take<__bf16>(mat) : nullptr;
    q->Alo = prec == MHAR_BF16X3 ? c.take<__bf16>(mat) : nullptr;
    q->Apk = prec != MHAR_FP64 && d.lda <= kMaxNResident ? (void*)c.take<float>(mat) : nullptr;
    q->b64 = c.take<double>(d.m_pad);
    q->rownorm = c.take<float>(d.m_pad);
    q->absb = c.take<float>(d.m_pad);
    size_t eq = (size_t)std::max(d.m_eq, 1) * d.lda;
    q->Aeq = c.take<double>(eq);
    q->beq = c.take<double>(std::max(d.m_eq, 1));
    q->WT = c.take<double>(eq);
    q->status = c.take<int>(64);
    return c.used;
}

size_t carve_chains(const mhar_problem* p, int z_pad, void* ws, mhar_chains* ch)
{
    Carver c(ws);
    mhar_chains tmp{};
    mhar_chains* q = ch ? ch : &tmp;
    size_t rows = (size_t)z_pad * p->lda;
    size_t st = p->prec == MHAR_FP64 ? sizeof(double) : sizeof(float);
    q->X = c.take<double>(rows);
    q->D = c.take<double>(rows);
    q->S = c.take<char>((size_t)z_pad * p->m_pad * st);
    q->G = c.take<char>((size_t)z_pad * p->m_pad * st);
    q->L = c.take<float>((size_t)(z_pad / kChainTile) * (p->m_pad / kRowGroup) * 2 * kChainTile);
    q->Ug = c.take<float>((size_t)(z_pad / kChainTile) * (p->m_pad / kRowGroup) * 2 * kChainTile);
    q->Dop = p->prec == MHAR_FP64 ? nullptr : (void*)c.take<float>(rows);
    q->dn = c.take<double>(z_pad);
    q->theta = c.take<double>(z_pad);
    q->E = c.take<double>(z_pad);
    q->flags = c.take<int>(z_pad);
    q->counters = c.take<unsigned long long>(8);
    const size_t tiles = (size_t)z_pad / kChainTile;
    q->gL = c.take<unsigned long long>(tiles * 3 * 2 * kChainTile);
    q->gbar = c.take<unsigned>(tiles);
    q->gerr = c.take<int>(64);
    q->gstep = c.take<uint64_t>(1);
    return c.used;
}

float eps_for(int prec, int n)
{
    // error coefficient of the screening product: |G_hat - G| <= eps ||a|| ||d||,
    // with a factor 2 of headroom over the standard rounding-error bounds
    const double u32 = std::ldexp(1.0, -24), u64 = std::ldexp(1.0, -53);
    double e;
    if (prec == MHAR_FP64) e = 2.0 * (n + 3) * u64;
    else if (prec == MHAR_FP32) e = 2.0 * (n + 3) * u32;
    else e = 2.0 * (3.03 * std::ldexp(1.0, -16) + (3.0 * n + 3) * u32);
    return (float)(e * (1.0 + 1e-6));
}

void advance_schedule(mhar_chains* c, int64_t steps)
{
    for (int64_t s = 0; s < steps; ++s) {
        c->pending = 1;
        c->T += 1;
        c->since += 1;
        if (c->since >= c->p->R) {
            c->pending = 0;
            c->T = 2;
            c->since = 0;
            c->recomputes += 1;
        }
    }
    c->step += (uint64_t)steps;
}

StepArgs make_args(const mhar_chains* c)
{
    const mhar_problem* p = c->p;
    StepArgs a{};
    a.n = p->n;
    a.m = p->m;
    a.m_pad = p->m_pad;
    a.lda = p->lda;
    a.m_eq = p->m_eq;
    a.A64 = p->A64;
    a.A32 = p->A32;
    a.Ahi = p->Ahi;
    a.Alo = p->Alo;
    a.Apk = p->Apk;
    a.b64 = p->b64;
    a.rownorm = p->rownorm;
    a.absb = p->absb;
    a.Aeq = p->Aeq;
    a.WT = p->WT;
    a.z = c->z;
    a.z_pad = c->z_pad;
    a.X = c->X;
    a.D = c->D;
    a.S = c->S;
    a.G = c->G;
    a.L = c->L;
    a.Ug = c->Ug;
    a.Dop = c->Dop;
    a.dn = c->dn;
    a.theta = c->theta;
    a.E = c->E;
    a.flags = c->flags;
    a.counters = c->counters;
    a.seed = c->seed;
    a.chain_offset = c->chain_offset;
    a.step0 = c->step;
    a.pending0 = c->pending;
    a.T0 = c->T;
    a.since0 = c->since;
    a.R = p->R;
    a.eps_g = p->eps_g;
    a.u_s = p->u_s;
    a.split = c->split > 0 ? c->split : 1;
    a.r = c->pc_rank;
    a.U = c->pc_rank ? c->pc.U : nullptr;
    a.esig = c->pc_rank ? c->pc.esig : nullptr;
    a.prec = p->prec;
    a.rk = 0;
    if (c->pc_rank && c->tiled) {
        // split screening: A d = A P (exp(l) o h) + (A P U) eps
        a.rk = c->pc.rk;
        a.AUop = c->pc.AUop;
        a.aun = c->pc.aun;
        a.Eop = c->pc.Eop;
        a.Hs = c->pc.Hs;
        a.hn = c->pc.hn;
        a.en = c->pc.en;
        a.F = c->pc.F;
        a.uF = c->pc.uF;
        a.eps_g = c->pc_eps_g;
    }
    a.gL = c->gL;
    a.gbar = c->gbar;
    a.gerr = c->gerr;
    return a;
}

// Automatic choice between the general and the tiled path (reduced
// precision only): the general kernel streams all of A once per 16 walks, the
// tiled path once per 128 walks and one row tile of D per 128 rows, which wins
// once A no longer sits in one XCD's L2.
int use_tiled(const mhar_problem* p, int z_pad)
{
    if (p->prec == MHAR_FP64) return 0;
    return (int64_t)p->m_pad * p->lda >= (int64_t(1) << 18) && z_pad >= 64;
}

int64_t auto_chunk(const mhar_problem* p)
{
    int64_t work = (int64_t)p->m_pad * p->lda;
    int64_t chunk = (int64_t(1) << 29) / std::max<int64_t>(work, 1);
    return std::min<int64_t>(std::max<int64_t>(chunk, 1), 100000);
}

// AUTO takes the lane path where its step takes less time than a screened
// kernel's.  Step-time models fitted to measurements on one MI355X
// (hypercube and simplex rows of the paper's Table 5 with n <= 32, cube
// n = 10 with 16 walks):
//   lane:    about 2.2 + 0.0065 m n + 0.4 n m_eq us (every lane of a walk's
//            group repeats the projection) while z times the lanes per walk
//            stays below ~10^5;
//   general: about 16 us up to ~2048 walks, then growing with z as the
//            16-walk workgroups queue for the CUs.
// Measured: 15-20x the general kernel at n = 3..5 and 10^4 walks, 8x at
// n = 15, 2.5-3x at n = 25, 4x for n = 10 with 16 walks; level with it for
// the cube at n = 32 with 2500 walks.
// (The variant for 33..64 coordinates, x and d in LDS, is taken on request
// only: measured it beat the screened kernels on none of the hypercube and
// simplex rows at n = 40..64.)
constexpr int kLaneAutoMaxN = 32;

bool lane_preferred(const mhar_problem* p, int z_pad)
{
    if (p->n > kLaneAutoMaxN || !lane_fits(p->n, p->m)) return false;
    const double lane_us = 2.2 + 0.0065 * (double)p->m * p->n + 0.4 * (double)p->n * p->m_eq;
    const double general_us = 16.0 * std::max(1.0, (double)z_pad / 2048.0);
    return lane_us < 0.9 * general_us;
}

hipError_t launch_any(mhar_chains* c, const StepArgs& a, hipStream_t stream)
{
    if (c->lane && c->pc_rank == 0) {
        // the slack the other paths keep is not updated: they recompute it first
        c->slack_stale = 1;
        c->last_kernel = MHAR_PATH_LANE;
        return launch_lane(a, stream);
    }
    c->last_kernel = c->tiled ? MHAR_PATH_TILED : c->split > 0 ? MHAR_PATH_RESIDENT : MHAR_PATH_GENERAL;
    if (c->tiled) return launch_tiled(c->p->prec, a, stream, c->trace.cap > 0 ? &c->trace : nullptr);
    if (c->split <= 0) return launch_steps(c->p->prec, a, stream);
    if (c->split > 1) {
        // fresh exchange slots and arrival counters for this launch
        const int64_t tiles = c->z_pad / kChainTile;
        hipError_t e = launch_fill_u64(c->gL, tiles * 3 * 2 * kChainTile, 0x7FF0000000000000ull, stream);
        if (e == hipSuccess) e = launch_fill_i32((int*)c->gbar, tiles, 0, stream);
        if (e != hipSuccess) return e;
    }
    return launch_resident(c->p->prec, a, stream);
}

// run `steps` steps (and the optional leading recompute), in launches of at
// most steps_per_launch steps each
// A P U of the split screening after the covariance changed
hipError_t refresh_lowrank(mhar_chains* c, hipStream_t stream)
{
    if (!(c->pc_rank && c->tiled && c->pc_lr_stale)) return hipSuccess;
    c->pc_lr_stale = 0;
    return launch_lowrank_setup(c->pc, stream);
}

// The captured arguments that stay fixed while a graph is valid: everything
// but the step and slack schedule of the launch, which the graph fixes (step
// counter on the device, schedule restarting after an exact recompute).
bool graph_key_matches(const StepArgs& x, const StepArgs& y)
{
    return x.r == y.r && x.rk == y.rk && x.U == y.U && x.esig == y.esig && x.AUop == y.AUop &&
           x.aun == y.aun && x.Eop == y.Eop && x.Hs == y.Hs && x.hn == y.hn && x.en == y.en &&
           x.F == y.F && x.uF == y.uF && x.eps_g == y.eps_g && x.split == y.split && x.R == y.R &&
           x.X == y.X && x.S == y.S;
}

void drop_graph(mhar_chains* c)
{
    if (c->graph_exec) (void)hipGraphExecDestroy(c->graph_exec);
    c->graph_exec = nullptr;
}

// Capture graph_steps steps of the tiled path, starting right after an exact
// recompute, with the step arguments relative to the device counter, and the
// counter advance as the last node.
hipError_t capture_graph(mhar_chains* c)
{
    drop_graph(c);
    hipError_t e = hipSuccess;
    if (!c->cap_stream) e = hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking);
    if (e != hipSuccess) return e;
    StepArgs a = make_args(c);
    a.step0 = 0;
    a.pending0 = 0;
    a.T0 = 2;
    a.since0 = 0;
    a.steps = c->graph_steps;
    a.recompute_first = 0;
    a.step_dev = c->gstep;
    e = hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeRelaxed);
    if (e != hipSuccess) return e;
    hipError_t el = launch_tiled(c->p->prec, a, c->cap_stream, nullptr);
    if (el == hipSuccess) el = launch_step_counter(c->gstep, (uint64_t)c->graph_steps, 1, c->cap_stream);
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(c->cap_stream, &g);
    if (el != hipSuccess) e = el;
    if (e == hipSuccess) e = hipGraphInstantiate(&c->graph_exec, g, nullptr, nullptr, 0);
    if (g) (void)hipGraphDestroy(g);
    if (e != hipSuccess) {
        c->graph_exec = nullptr;
        return e;
    }
    c->graph_key = a;
    return hipSuccess;
}

mhar_status_t run_steps(mhar_chains* c, int64_t steps, int recompute_first, double* rec_out,
                        int64_t stride, int64_t rec_chains, hipStream_t stream)
{
    const mhar_problem* p = c->p;
    if (c->tiled && c->pc_rank && c->pc.rk == 0)
        return fail(MHAR_E_STATE, "the covariance was attached off the tiled path: the split "
                                  "screening has no buffers");
    MHAR_HIP(refresh_lowrank(c, stream), "low-rank screening operand");
    int64_t chunk = p->steps_per_launch > 0 ? p->steps_per_launch : auto_chunk(p);
    int64_t done = 0;
    if (c->force_recompute) {
        recompute_first = 1;
        c->force_recompute = 0;
    }
    if (c->slack_stale && !(c->lane && c->pc_rank == 0)) {
        recompute_first = 1;
        c->slack_stale = 0;
    }
    if (recompute_first) {
        StepArgs a = make_args(c);
        a.steps = 0;
        a.recompute_first = 1;
        MHAR_HIP(launch_any(c, a, stream), "launch of the step kernel");
        c->pending = 0;
        c->T = 2;
        c->since = 0;
        c->recomputes += 1;
    }
    // graph replays (tiled path, no recording or kernel timing): ordinary
    // launches until the slack schedule restarts, then whole graphs
    const int K = c->graph_steps;
    if (K > 0 && c->tiled && !rec_out && c->trace.cap == 0 && !(c->lane && c->pc_rank == 0)) {
        struct Plain {   // ordinary launches for the steps around the replays
            mhar_chains* c;
            int K;
            mhar_status_t run(int64_t n, hipStream_t st)
            {
                c->graph_steps = 0;
                const mhar_status_t r = run_steps(c, n, 0, nullptr, 0, 0, st);
                c->graph_steps = K;
                return r;
            }
        } plain{c, K};
        const int64_t lead = std::min<int64_t>(steps, (p->R - c->since) % p->R);
        mhar_status_t st = plain.run(lead, stream);
        if (st) return st;
        const int64_t reps = (steps - lead) / K;
        if (reps > 0) {
            const StepArgs now = make_args(c);
            if (!c->graph_exec || !graph_key_matches(now, c->graph_key))
                MHAR_HIP(capture_graph(c), "graph capture of the tiled path");
            MHAR_HIP(launch_step_counter(c->gstep, c->step, 0, stream), "graph step counter");
            c->last_kernel = MHAR_PATH_TILED;
            for (int64_t r = 0; r < reps; ++r) {
                MHAR_HIP(hipGraphLaunch(c->graph_exec, stream), "graph launch");
                advance_schedule(c, K);
            }
        }
        return plain.run(steps - lead - reps * K, stream);
    }
    while (done < steps) {
        int64_t k = std::min(chunk, steps - done);
        StepArgs a = make_args(c);
        a.steps = (int)k;
        a.recompute_first = 0;
        if (rec_out) {
            a.rec_out = rec_out;
            a.rec_stride = (int)stride;
            a.rec_chains = (int)rec_chains;
            a.rec_s_base = done;
        }
        MHAR_HIP(launch_any(c, a, stream), "launch of the step kernel");
        advance_schedule(c, k);
        done += k;
    }
    return MHAR_OK;
}

bool aligned256(const void* p) { return ((uintptr_t)p & 255u) == 0; }

}  // namespace

extern "C" {

int32_t mhar_version(void) { return 100; }

const char* mhar_status_string(int32_t s)
{
    switch (s) {
    case MHAR_OK: return "ok";
    case MHAR_E_INVALID_ARG: return "invalid argument";
    case MHAR_E_SHAPE: return "unsupported shape";
    case MHAR_E_RANK_DEFICIENT: return "equality rows are linearly dependent";
    case MHAR_E_NOT_INTERIOR: return "start point not strictly interior";
    case MHAR_E_WORKSPACE: return "workspace too small or misaligned";
    case MHAR_E_HIP: return "HIP runtime error";
    case MHAR_E_UNSUPPORTED: return "unsupported configuration";
    case MHAR_E_STATE: return "invalid handle state";
    default: return "unknown status";
    }
}

const char* mhar_last_error(void) { return g_last_error.c_str(); }

mhar_status_t mhar_options_default(mhar_options_t* opt)
{
    if (!opt) return fail(MHAR_E_INVALID_ARG, "opt is NULL");
    std::memset(opt, 0, sizeof(*opt));
    opt->precision = MHAR_FP32;
    opt->recompute_every = 50;
    opt->steps_per_launch = 0;
    return MHAR_OK;
}

mhar_status_t mhar_problem_workspace_size(int64_t n, int64_t m, int64_t m_eq,
                                          const mhar_options_t* opt, size_t* bytes)
{
    if (!bytes) return fail(MHAR_E_INVALID_ARG, "bytes is NULL");
    mhar_options_t o;
    mhar_status_t st = check_options(opt, &o);
    if (st) return st;
    ProblemDims d;
    st = check_dims(n, m, m_eq, o, &d);
    if (st) return st;
    *bytes = carve_problem(d, o.precision, nullptr, nullptr);
    return MHAR_OK;
}

mhar_status_t mhar_problem_create(int64_t n, int64_t m, const double* A, const double* b,
                                  int64_t m_eq, const double* A_eq, const double* b_eq,
                                  const mhar_options_t* opt, void* workspace, size_t ws_bytes,
                                  void* stream_, mhar_problem_t* out)
{
    if (!out) return fail(MHAR_E_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (!A || !b) return fail(MHAR_E_INVALID_ARG, "A and b must be device pointers");
    if (m_eq > 0 && (!A_eq || !b_eq)) return fail(MHAR_E_INVALID_ARG, "A_eq and b_eq required when m_eq > 0");
    mhar_options_t o;
    mhar_status_t st = check_options(opt, &o);
    if (st) return st;
    ProblemDims d;
    st = check_dims(n, m, m_eq, o, &d);
    if (st) return st;
    if (!workspace || !aligned256(workspace)) return fail(MHAR_E_WORKSPACE, "workspace must be 256-byte aligned");
    size_t need = carve_problem(d, o.precision, nullptr, nullptr);
    if (ws_bytes < need) return fail(MHAR_E_WORKSPACE, "workspace too small: need " + std::to_string(need) + " bytes");

    hipStream_t stream = (hipStream_t)stream_;
    mhar_problem* p = new mhar_problem{};
    p->n = d.n;
    p->m = d.m;
    p->m_pad = d.m_pad;
    p->lda = d.lda;
    p->m_eq = d.m_eq;
    p->prec = o.precision;
    p->R = o.recompute_every;
    p->steps_per_launch = o.steps_per_launch;
    p->path = o.path;
    p->eps_g = eps_for(o.precision, d.n);
    p->u_s = o.precision == MHAR_FP64 ? std::ldexp(1.0f, -53) : std::ldexp(1.0f, -24);
    carve_problem(d, o.precision, workspace, p);

    hipError_t e = launch_convert_problem(p->prec, p->n, p->m, p->m_pad, p->lda, A, b, p->A64,
                                          p->A32, p->Ahi, p->Alo, p->b64, p->rownorm, p->absb,
                                          stream);
    if (e == hipSuccess && p->Apk)
        e = launch_pack_operand(p->prec, p->m_pad, p->lda, p->A32, p->Ahi, p->Alo, p->Apk, stream);
    if (e != hipSuccess) {
        delete p;
        return hip_fail(e, "problem conversion");
    }
    int bad = 0;
    if (p->m_eq > 0) {
        e = launch_eq_setup(p->n, p->lda, p->m_eq, A_eq, b_eq, p->Aeq, p->beq, p->WT, p->status, stream);
        if (e == hipSuccess) e = hipMemcpyAsync(&bad, p->status, sizeof(int), hipMemcpyDeviceToHost, stream);
    }
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e != hipSuccess) {
        delete p;
        return hip_fail(e, "problem setup");
    }
    if (bad) {
        delete p;
        return fail(MHAR_E_RANK_DEFICIENT, "A_eq A_eq^T is singular to working precision");
    }
    *out = p;
    return MHAR_OK;
}

mhar_status_t mhar_problem_get_projection(mhar_problem_t p, double* P, void* stream)
{
    if (!p || !P) return fail(MHAR_E_INVALID_ARG, "problem and P must be non-NULL");
    if (p->m_eq == 0) {
        // identity
        MHAR_HIP(launch_dense_projection(p->n, p->lda, 0, p->Aeq, p->WT, P, (hipStream_t)stream),
                 "projection kernel");
        return MHAR_OK;
    }
    MHAR_HIP(launch_dense_projection(p->n, p->lda, p->m_eq, p->Aeq, p->WT, P, (hipStream_t)stream),
             "projection kernel");
    return MHAR_OK;
}

mhar_status_t mhar_problem_destroy(mhar_problem_t p)
{
    if (!p) return MHAR_OK;
    if (p->live_chains > 0) return fail(MHAR_E_STATE, "destroy the chains of this problem first");
    delete p;
    return MHAR_OK;
}

mhar_status_t mhar_chains_workspace_size(mhar_problem_t p, int64_t z, size_t* bytes)
{
    if (!p || !bytes) return fail(MHAR_E_INVALID_ARG, "problem and bytes must be non-NULL");
    if (z < 1 || z > (int64_t(1) << 31)) return fail(MHAR_E_SHAPE, "z must be in [1, 2^31]");
    *bytes = carve_chains(p, (int)round_up(z, kChainTile), nullptr, nullptr);
    return MHAR_OK;
}

mhar_status_t mhar_chains_create(mhar_problem_t p, int64_t z, const double* X0, uint64_t seed,
                                 uint64_t chain_offset, void* workspace, size_t ws_bytes,
                                 void* stream_, mhar_chains_t* out)
{
    if (!out) return fail(MHAR_E_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (!p || !X0) return fail(MHAR_E_INVALID_ARG, "problem and X0 must be non-NULL");
    if (z < 1 || z > (int64_t(1) << 31)) return fail(MHAR_E_SHAPE, "z must be in [1, 2^31]");
    if (chain_offset + (uint64_t)z > (uint64_t(1) << 32))
        return fail(MHAR_E_SHAPE, "chain_offset + z must not exceed 2^32");
    if (!workspace || !aligned256(workspace)) return fail(MHAR_E_WORKSPACE, "workspace must be 256-byte aligned");
    const int z_pad = (int)round_up(z, kChainTile);
    size_t need = carve_chains(p, z_pad, nullptr, nullptr);
    if (ws_bytes < need) return fail(MHAR_E_WORKSPACE, "workspace too small: need " + std::to_string(need) + " bytes");
    hipStream_t stream = (hipStream_t)stream_;

    mhar_chains* c = new mhar_chains{};
    c->p = p;
    c->z = (int)z;
    c->z_pad = z_pad;
    c->seed = seed;
    c->chain_offset = (uint32_t)chain_offset;
    carve_chains(p, z_pad, workspace, c);
    auto cleanup = [&](mhar_status_t code) {
        delete c;
        return code;
    };
    const int rs = resident_split(p->prec, p->lda, p->m_pad, z_pad);
    c->split = 0;
    c->tiled = 0;
    c->lane = 0;
    if (p->path == MHAR_PATH_LANE) {
        if (!lane_fits(p->n, p->m))
            return cleanup(fail(MHAR_E_UNSUPPORTED, "the lane path needs n <= 32, or n <= 64 with A in 96 KB of LDS"));
        c->lane = 1;
    } else if (p->path == MHAR_PATH_RESIDENT) {
        if (rs <= 0) return cleanup(fail(MHAR_E_UNSUPPORTED, "the resident path does not fit this shape"));
        c->split = rs;
    } else if (p->path == MHAR_PATH_TILED) {
        c->tiled = 1;
    } else if (p->path == MHAR_PATH_AUTO) {
        if (lane_preferred(p, z_pad)) c->lane = 1;
        else if (rs > 0) c->split = rs;
        else c->tiled = p->lda > kMaxN || use_tiled(p, z_pad);
    }
    hipError_t e = launch_fill_i32((int*)c->theta, (int64_t)z_pad * 2, 0, stream);
    if (e == hipSuccess) e = launch_fill_i32((int*)c->E, (int64_t)z_pad * 2, 0, stream);
    if (e == hipSuccess) e = launch_fill_i32(c->flags, z_pad, 0, stream);
    if (e == hipSuccess) e = launch_fill_i32((int*)c->counters, 16, 0, stream);
    if (e == hipSuccess) e = launch_fill_i32(c->gerr, 64, 0, stream);
    if (e == hipSuccess) e = launch_fill_i32((int*)c->D, (int64_t)z_pad * p->lda * 2, 0, stream);
    if (e == hipSuccess) e = launch_copy_states(p->n, p->lda, c->z, z_pad, X0, c->X, stream);
    if (e == hipSuccess && p->m_eq > 0)
        e = launch_eq_residual(p->n, p->lda, c->z, p->m_eq, p->Aeq, p->beq, c->X, c->flags, stream);
    if (e != hipSuccess) return cleanup(hip_fail(e, "chain setup"));
    mhar_status_t st = run_steps(c, 0, 1, nullptr, 0, 0, stream);
    if (st) return cleanup(st);
    std::vector<int> fl(c->z);
    e = hipMemcpyAsync(fl.data(), c->flags, sizeof(int) * c->z, hipMemcpyDeviceToHost, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e != hipSuccess) return cleanup(hip_fail(e, "interior check"));
    for (int k = 0; k < c->z; ++k)
        if (fl[k] & (kNotInterior | kInfeasible))
            return cleanup(fail(MHAR_E_NOT_INTERIOR, "start point of walk " + std::to_string(k) +
                                                           " is not strictly interior"));
    c->recomputes = 0;
    p->live_chains += 1;
    *out = c;
    return MHAR_OK;
}

mhar_status_t mhar_step(mhar_chains_t c, int64_t steps, void* stream)
{
    if (!c) return fail(MHAR_E_INVALID_ARG, "chains is NULL");
    if (steps < 0) return fail(MHAR_E_INVALID_ARG, "steps must be >= 0");
    return run_steps(c, steps, 0, nullptr, 0, 0, (hipStream_t)stream);
}

mhar_status_t mhar_record(mhar_chains_t c, int64_t steps, int64_t stride, int64_t chain_count,
                          double* out, void* stream)
{
    if (!c || !out) return fail(MHAR_E_INVALID_ARG, "chains and out must be non-NULL");
    if (steps < 0 || stride < 1 || stride > (int64_t(1) << 30))
        return fail(MHAR_E_INVALID_ARG, "need steps >= 0 and 1 <= stride <= 2^30");
    if (chain_count < 1 || chain_count > c->z) return fail(MHAR_E_INVALID_ARG, "chain_count must be in [1, z]");
    return run_steps(c, steps, 0, out, stride, chain_count, (hipStream_t)stream);
}

mhar_status_t mhar_get_state(mhar_chains_t c, double* X, int32_t* status, void* stream)
{
    if (!c) return fail(MHAR_E_INVALID_ARG, "chains is NULL");
    hipStream_t s = (hipStream_t)stream;
    if (X) MHAR_HIP(launch_export_states(c->p->n, c->p->lda, c->z, c->X, X, s), "state export");
    if (status) MHAR_HIP(launch_export_flags(c->flags, c->z, status, 1, s), "status export");
    return MHAR_OK;
}

mhar_status_t mhar_set_state(mhar_chains_t c, const double* X, uint64_t step, void* stream)
{
    if (!c || !X) return fail(MHAR_E_INVALID_ARG, "chains and X must be non-NULL");
    hipStream_t s = (hipStream_t)stream;
    MHAR_HIP(launch_copy_states(c->p->n, c->p->lda, c->z, c->z_pad, X, c->X, s), "state import");
    MHAR_HIP(launch_fill_i32(c->flags, c->z_pad, 0, s), "status reset");
    MHAR_HIP(launch_fill_i32((int*)c->theta, (int64_t)c->z_pad * 2, 0, s), "theta reset");
    c->step = step;
    mhar_status_t st = run_steps(c, 0, 1, nullptr, 0, 0, s);
    if (st) return st;
    MHAR_HIP(launch_export_flags(c->flags, c->z_pad, c->flags, 1, s), "status reset");
    return MHAR_OK;
}

mhar_status_t mhar_get_step(mhar_chains_t c, uint64_t* step)
{
    if (!c || !step) return fail(MHAR_E_INVALID_ARG, "chains and step must be non-NULL");
    *step = c->step;
    return MHAR_OK;
}

mhar_status_t mhar_sync(mhar_chains_t c, void* stream, int32_t* any_flags)
{
    if (!c) return fail(MHAR_E_INVALID_ARG, "chains is NULL");
    hipStream_t s = (hipStream_t)stream;
    std::vector<int> fl(c->z);
    int gerr = 0, fit = 0;
    MHAR_HIP(hipMemcpyAsync(fl.data(), c->flags, sizeof(int) * c->z, hipMemcpyDeviceToHost, s), "status read");
    MHAR_HIP(hipMemcpyAsync(&gerr, c->gerr, sizeof(int), hipMemcpyDeviceToHost, s), "status read");
    if (c->pc_rank)
        MHAR_HIP(hipMemcpyAsync(&fit, c->pc.status, sizeof(int), hipMemcpyDeviceToHost, s), "status read");
    MHAR_HIP(hipStreamSynchronize(s), "stream synchronize");
    if (gerr) return fail(MHAR_E_HIP, "a workgroup group wait timed out; the states are not valid");
    int acc = 0;
    for (int v : fl) acc |= v;
    if (any_flags) *any_flags = (acc & 15) | (fit ? MHAR_FIT_FAILED : 0);
    return MHAR_OK;
}

mhar_status_t mhar_get_stats(mhar_chains_t c, void* stream, mhar_stats_t* stats)
{
    if (!c || !stats) return fail(MHAR_E_INVALID_ARG, "chains and stats must be non-NULL");
    hipStream_t s = (hipStream_t)stream;
    unsigned long long cnt[8];
    MHAR_HIP(hipMemcpyAsync(cnt, c->counters, sizeof(cnt), hipMemcpyDeviceToHost, s), "counter read");
    MHAR_HIP(hipStreamSynchronize(s), "stream synchronize");
    stats->steps = c->step;
    stats->chain_steps = c->step * (uint64_t)c->z;
    stats->exact_rows = cnt[0];
    stats->recomputes = c->recomputes;
    stats->kernel = c->last_kernel ? c->last_kernel
                                   : c->lane ? MHAR_PATH_LANE
                                   : c->tiled ? MHAR_PATH_TILED
                                   : c->split > 0 ? MHAR_PATH_RESIDENT : MHAR_PATH_GENERAL;
    stats->split = c->split > 0 ? c->split : 1;
    return MHAR_OK;
}

// covariance workspace: the fit's buffers, then (tiled path) the split screening's
static size_t precond_total_bytes(const mhar_chains* c, int32_t rank, int32_t objective)
{
    const mhar_problem* p = c->p;
    size_t b = precond_bytes(p->n, rank, c->z, p->lda, objective, p->m_pad);
    if (c->tiled) b = (size_t)round_up((int64_t)b, 256) + lowrank_bytes(p->prec, p->n, rank, p->m_pad, p->lda, c->z_pad, p->m_eq);
    return b;
}

static mhar_status_t check_fit(const mhar_chains* c, int32_t rank, int32_t objective)
{
    if (rank < 1 || rank > kMaxMeq) return fail(MHAR_E_SHAPE, "rank must be in [1, 64]");
    if (objective != MHAR_FIT_STATES && objective != MHAR_FIT_DIKIN)
        return fail(MHAR_E_INVALID_ARG, "objective must be MHAR_FIT_STATES or MHAR_FIT_DIKIN");
    if (objective == MHAR_FIT_DIKIN && c->p->n > kMaxNDikin)
        return fail(MHAR_E_SHAPE, "the Dikin fit takes n <= 4096");
    return MHAR_OK;
}

mhar_status_t mhar_precond_workspace_size(mhar_chains_t c, int32_t rank, int32_t objective,
                                          size_t* bytes)
{
    if (!c || !bytes) return fail(MHAR_E_INVALID_ARG, "chains and bytes must be non-NULL");
    mhar_status_t st = check_fit(c, rank, objective);
    if (st) return st;
    *bytes = precond_total_bytes(c, rank, objective);
    return MHAR_OK;
}

mhar_status_t mhar_precond_create(mhar_chains_t c, int32_t rank, int32_t objective, void* ws,
                                  size_t ws_bytes, void* stream)
{
    if (!c) return fail(MHAR_E_INVALID_ARG, "chains is NULL");
    if (c->pc_rank) return fail(MHAR_E_STATE, "a covariance is already attached");
    mhar_status_t st = check_fit(c, rank, objective);
    if (st) return st;
    if (!ws || !aligned256(ws)) return fail(MHAR_E_WORKSPACE, "workspace must be 256-byte aligned");
    if (ws_bytes < precond_total_bytes(c, rank, objective))
        return fail(MHAR_E_WORKSPACE, "precond workspace too small");
    c->pc = PrecondBufs{};
    c->pc.n = c->p->n;
    c->pc.r = rank;
    c->pc.z = c->z;
    c->pc.lda = c->p->lda;
    c->pc.objective = objective;
    c->pc.m = c->p->m;
    c->pc.m_pad = c->p->m_pad;
    c->pc.A64 = c->p->A64;
    c->pc.b64 = c->p->b64;
    c->pc.kappa = kDikinKappa;
    c->pc.prec = c->p->prec;
    c->pc.m_eq = c->p->m_eq;
    c->pc.z_pad = c->z_pad;
    c->pc.Aeq = c->p->Aeq;
    c->pc.WT = c->p->WT;
    precond_carve(&c->pc, ws);
    if (c->tiled) {
        const size_t off = (size_t)round_up(
            (int64_t)precond_bytes(c->p->n, rank, c->z, c->p->lda, objective, c->p->m_pad), 256);
        lowrank_carve(&c->pc, (char*)ws + off);
    }
    c->pc_eps_g = eps_for(c->p->prec, c->p->n + rank);
    c->pc_lr_stale = 1;
    MHAR_HIP(launch_precond_init(c->pc, c->seed, (hipStream_t)stream), "covariance init");
    if (objective == MHAR_FIT_DIKIN)
        MHAR_HIP(launch_dikin_init(c->pc, c->seed, (hipStream_t)stream), "covariance init");
    c->pc_rank = rank;
    c->pc_frozen = 0;
    c->pc_t = 0;
    c->split_saved = c->split;
    c->split = 0;
    c->force_recompute = 1;
    return MHAR_OK;
}

mhar_status_t mhar_precond_set(mhar_chains_t c, const double* U, const double* ls, void* stream)
{
    if (!c || !U || !ls) return fail(MHAR_E_INVALID_ARG, "chains, U and log_sigma must be non-NULL");
    if (!c->pc_rank) return fail(MHAR_E_STATE, "no covariance attached");
    hipStream_t s = (hipStream_t)stream;
    const size_t nr = (size_t)c->pc.n * c->pc.r;
    MHAR_HIP(hipMemcpyAsync(c->pc.U, U, nr * 8, hipMemcpyDeviceToDevice, s), "covariance copy");
    MHAR_HIP(hipMemcpyAsync(c->pc.logsig, ls, (size_t)c->pc.n * 8, hipMemcpyDeviceToDevice, s), "covariance copy");
    MHAR_HIP(launch_fill_i32((int*)c->pc.m1V, (int64_t)nr * 2, 0, s), "moment reset");
    MHAR_HIP(launch_fill_i32((int*)c->pc.m2V, (int64_t)nr * 2, 0, s), "moment reset");
    MHAR_HIP(launch_fill_i32((int*)c->pc.m1l, (int64_t)c->pc.n * 2, 0, s), "moment reset");
    MHAR_HIP(launch_fill_i32((int*)c->pc.m2l, (int64_t)c->pc.n * 2, 0, s), "moment reset");
    MHAR_HIP(launch_precond_set_scales(c->pc, s), "covariance scale");
    c->pc_t = 0;
    c->pc_lr_stale = 1;
    return MHAR_OK;
}

mhar_status_t mhar_precond_get(mhar_chains_t c, double* U, double* ls, void* stream)
{
    if (!c) return fail(MHAR_E_INVALID_ARG, "chains is NULL");
    if (!c->pc_rank) return fail(MHAR_E_STATE, "no covariance attached");
    hipStream_t s = (hipStream_t)stream;
    if (U) MHAR_HIP(hipMemcpyAsync(U, c->pc.U, (size_t)c->pc.n * c->pc.r * 8, hipMemcpyDeviceToDevice, s), "covariance copy");
    if (ls) MHAR_HIP(hipMemcpyAsync(ls, c->pc.logsig, (size_t)c->pc.n * 8, hipMemcpyDeviceToDevice, s), "covariance copy");
    return MHAR_OK;
}

mhar_status_t mhar_precond_loss(mhar_chains_t c, double* nll, double* gU, double* gls, void* stream)
{
    if (!c) return fail(MHAR_E_INVALID_ARG, "chains is NULL");
    if (!c->pc_rank) return fail(MHAR_E_STATE, "no covariance attached");
    hipStream_t s = (hipStream_t)stream;
    if (c->pc.objective == MHAR_FIT_DIKIN)
        MHAR_HIP(launch_dikin_loss(c->pc, c->X, s), "covariance objective");
    else
        MHAR_HIP(launch_precond_grad(c->pc, c->X, s), "covariance gradient");
    if (nll) MHAR_HIP(hipMemcpyAsync(nll, c->pc.nll, 8, hipMemcpyDeviceToDevice, s), "loss copy");
    if (gU) MHAR_HIP(hipMemcpyAsync(gU, c->pc.gU, (size_t)c->pc.n * c->pc.r * 8, hipMemcpyDeviceToDevice, s), "gradient copy");
    if (gls) MHAR_HIP(hipMemcpyAsync(gls, c->pc.gl, (size_t)c->pc.n * 8, hipMemcpyDeviceToDevice, s), "gradient copy");
    return MHAR_OK;
}

mhar_status_t mhar_precond_train(mhar_chains_t c, int64_t steps, double lr, void* stream)
{
    if (!c) return fail(MHAR_E_INVALID_ARG, "chains is NULL");
    if (!c->pc_rank) return fail(MHAR_E_STATE, "no covariance attached");
    if (c->pc_frozen) return fail(MHAR_E_STATE, "the covariance is frozen");
    if (steps < 0 || !(lr > 0.0)) return fail(MHAR_E_INVALID_ARG, "need steps >= 0 and lr > 0");
    const bool dikin = c->pc.objective == MHAR_FIT_DIKIN;
    if (dikin && !(lr <= 1.0)) return fail(MHAR_E_INVALID_ARG, "the Dikin fit takes lr in (0, 1]");
    hipStream_t s = (hipStream_t)stream;
    for (int64_t k = 0; k < steps; ++k) {
        mhar_status_t st = run_steps(c, 1, 0, nullptr, 0, 0, s);
        if (st) return st;
        c->pc_t += 1;
        if (dikin) {
            MHAR_HIP(launch_dikin_train(c->pc, c->X, kDikinPowerIters, lr, s), "covariance update");
        } else {
            MHAR_HIP(launch_precond_grad(c->pc, c->X, s), "covariance gradient");
            MHAR_HIP(launch_precond_adam(c->pc, c->pc_t, lr, 0.9, 0.999, 1e-8, s), "covariance update");
        }
        c->pc_lr_stale = 1;
    }
    return MHAR_OK;
}

mhar_status_t mhar_precond_set_complement(mhar_chains_t c, double kappa)
{
    if (!c) return fail(MHAR_E_INVALID_ARG, "chains is NULL");
    if (!c->pc_rank) return fail(MHAR_E_STATE, "no covariance attached");
    if (c->pc.objective != MHAR_FIT_DIKIN) return fail(MHAR_E_STATE, "the covariance is not a Dikin fit");
    if (!(kappa > 0.0 && kappa <= 1.0)) return fail(MHAR_E_INVALID_ARG, "kappa must be in (0, 1]");
    c->pc.kappa = kappa;
    return MHAR_OK;
}

mhar_status_t mhar_precond_freeze(mhar_chains_t c)
{
    if (!c) return fail(MHAR_E_INVALID_ARG, "chains is NULL");
    if (!c->pc_rank) return fail(MHAR_E_STATE, "no covariance attached");
    c->pc_frozen = 1;
    return MHAR_OK;
}

mhar_status_t mhar_precond_destroy(mhar_chains_t c)
{
    if (!c) return fail(MHAR_E_INVALID_ARG, "chains is NULL");
    if (!c->pc_rank) return MHAR_OK;
    c->pc_rank = 0;
    c->pc_frozen = 0;
    c->split = c->split_saved;
    c->force_recompute = 1;
    return MHAR_OK;
}

// Work items of a batch.  Problems that run the tiled path on their own are
// stepped by grouped tiled launches (one table entry per screening tile,
// 16-walk chords unit and recompute tile); the others by the persistent
// general kernel over (problem, 16-walk tile) units in decreasing order of
// cost (longest processing time first).
struct BatchPlan {
    int prec = 0;
    int max_lda = 0;
    double work = 0.0;
    std::vector<int2> gen_units, tiled_units;
    std::vector<int4> stiles, rtiles;
};

// Path of a handle inside a batch: the register-resident kernel cannot be
// batched, so a resident handle runs tiled if its shape qualifies for the
// tiled path, else the general kernel.
static bool tiled_in_batch(const mhar_chains* c)
{
    return c->tiled || (c->split > 0 && use_tiled(c->p, c->z_pad));
}

static mhar_status_t plan_batch(int32_t count, const mhar_chains_t* chains, BatchPlan* pl)
{
    if (count < 1 || !chains) return fail(MHAR_E_INVALID_ARG, "need count >= 1 and a chains array");
    std::vector<std::pair<double, int2>> order;
    for (int i = 0; i < count; ++i) {
        const mhar_chains* c = chains[i];
        if (!c) return fail(MHAR_E_INVALID_ARG, "NULL chains handle in the batch");
        if (i > 0 && c->p->prec != chains[0]->p->prec)
            return fail(MHAR_E_INVALID_ARG, "all problems of a batch must share one precision");
        for (int j = 0; j < i; ++j)
            if (chains[j] == c) return fail(MHAR_E_INVALID_ARG, "a chains handle appears twice");
        const mhar_problem* p = c->p;
        const double cost = (double)p->m_pad * p->lda;
        pl->work += cost * c->z_pad;
        if (tiled_in_batch(c)) {
            for (int t = 0; t < c->z_pad / kChainTile; ++t) pl->tiled_units.push_back(int2{i, t});
            const int nrb = (p->m_pad + kScreenRows - 1) / kScreenRows;
            const int ncb = (c->z_pad + kScreenWalks - 1) / kScreenWalks;
            for (int rb = 0; rb < nrb; ++rb)
                for (int cb = 0; cb < ncb; ++cb) pl->stiles.push_back(int4{i, rb, cb, 0});
            const int rrb = (p->m_pad + kRecRows - 1) / kRecRows;
            const int rcb = (c->z_pad + kRecWalks - 1) / kRecWalks;
            for (int rb = 0; rb < rrb; ++rb)
                for (int cb = 0; cb < rcb; ++cb) pl->rtiles.push_back(int4{i, rb, cb, 0});
        } else {
            if (p->lda > kMaxN)
                return fail(MHAR_E_UNSUPPORTED, "a problem with n > " + std::to_string(kMaxN) + " must run tiled");
            pl->max_lda = std::max(pl->max_lda, p->lda);
            for (int t = 0; t < c->z_pad / kChainTile; ++t) order.push_back({cost, int2{i, t}});
        }
    }
    std::stable_sort(order.begin(), order.end(),
                     [](const std::pair<double, int2>& x, const std::pair<double, int2>& y) { return x.first > y.first; });
    for (const auto& o : order) pl->gen_units.push_back(o.second);
    pl->prec = chains[0]->p->prec;
    return MHAR_OK;
}

static size_t carve_batch(int count, const BatchPlan& pl, void* ws, mhar_batch* b)
{
    Carver c(ws);
    StepArgs* d = c.take<StepArgs>(count);
    int2* u = c.take<int2>(std::max<size_t>(pl.gen_units.size(), 1));
    int2* tu = c.take<int2>(std::max<size_t>(pl.tiled_units.size(), 1));
    int4* st = c.take<int4>(std::max<size_t>(pl.stiles.size(), 1));
    int4* rt = c.take<int4>(std::max<size_t>(pl.rtiles.size(), 1));
    unsigned* nx = c.take<unsigned>(64);
    if (b) {
        b->descs_dev = d;
        b->units_dev = u;
        b->tunits_dev = tu;
        b->stiles_dev = st;
        b->rtiles_dev = rt;
        b->next_dev = nx;
    }
    return c.used;
}

mhar_status_t mhar_batch_workspace_size(int32_t count, const mhar_chains_t* chains, size_t* bytes)
{
    if (!bytes) return fail(MHAR_E_INVALID_ARG, "bytes is NULL");
    BatchPlan pl;
    mhar_status_t st = plan_batch(count, chains, &pl);
    if (st) return st;
    *bytes = carve_batch(count, pl, nullptr, nullptr);
    return MHAR_OK;
}

mhar_status_t mhar_batch_create(int32_t count, const mhar_chains_t* chains, void* ws, size_t ws_bytes,
                                mhar_batch_t* out)
{
    if (!out) return fail(MHAR_E_INVALID_ARG, "out is NULL");
    *out = nullptr;
    BatchPlan pl;
    mhar_status_t st = plan_batch(count, chains, &pl);
    if (st) return st;
    if (!ws || !aligned256(ws)) return fail(MHAR_E_WORKSPACE, "workspace must be 256-byte aligned");
    if (ws_bytes < carve_batch(count, pl, nullptr, nullptr)) return fail(MHAR_E_WORKSPACE, "batch workspace too small");
    mhar_batch* b = new mhar_batch{};
    b->count = count;
    b->prec = pl.prec;
    b->nunits = (int)pl.gen_units.size();
    b->ntu = (int)pl.tiled_units.size();
    b->nst = (int)pl.stiles.size();
    b->nrt = (int)pl.rtiles.size();
    b->max_lda = pl.max_lda;
    b->work_per_step = pl.work;
    carve_batch(count, pl, ws, b);
    for (int i = 0; i < count; ++i) {
        b->chains.push_back(chains[i]);
        b->saved_split.push_back(chains[i]->split);
        b->saved_tiled.push_back(chains[i]->tiled);
    }
    auto cleanup = [&](mhar_status_t code) {
        if (b->descs_host) (void)hipHostFree(b->descs_host);   // the first error is the one reported
        delete b;
        return code;
    };
    hipError_t e = hipHostMalloc((void**)&b->descs_host, sizeof(StepArgs) * count, hipHostMallocDefault);
    if (e != hipSuccess) return cleanup(hip_fail(e, "pinned descriptor buffer"));
    auto up = [&](void* dst, const void* src, size_t bytes) {
        if (e == hipSuccess && bytes) e = hipMemcpy(dst, src, bytes, hipMemcpyHostToDevice);
    };
    up(b->units_dev, pl.gen_units.data(), sizeof(int2) * pl.gen_units.size());
    up(b->tunits_dev, pl.tiled_units.data(), sizeof(int2) * pl.tiled_units.size());
    up(b->stiles_dev, pl.stiles.data(), sizeof(int4) * pl.stiles.size());
    up(b->rtiles_dev, pl.rtiles.data(), sizeof(int4) * pl.rtiles.size());
    if (e == hipSuccess) e = hipEventCreateWithFlags(&b->copied, hipEventDisableTiming);
    if (e != hipSuccess) return cleanup(hip_fail(e, "batch setup"));
    int dev = 0, cus = 1;
    e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return cleanup(hip_fail(e, "device query"));
    b->grid = b->nunits ? std::min(b->nunits, cus * batch_blocks_per_cu(b->prec, b->max_lda)) : 0;
    // resident handles switch to the tiled path or the general kernel; lane
    // handles step on the general kernel, whose slack they have not kept
    for (mhar_chains* c : b->chains) {
        if (c->slack_stale) {
            c->force_recompute = 1;
            c->slack_stale = 0;
        }
        if (c->split > 0) {
            c->tiled = tiled_in_batch(c) ? 1 : 0;
            c->split = 0;
            c->force_recompute = 1;
        }
        c->last_kernel = c->tiled ? MHAR_PATH_TILED : MHAR_PATH_GENERAL;   // the path inside the batch
    }
    *out = b;
    return MHAR_OK;
}

mhar_status_t mhar_batch_step(mhar_batch_t b, int64_t steps, void* stream_)
{
    if (!b) return fail(MHAR_E_INVALID_ARG, "batch is NULL");
    if (steps < 0) return fail(MHAR_E_INVALID_ARG, "steps must be >= 0");
    hipStream_t stream = (hipStream_t)stream_;
    // bound one launch to ~2^39 row-walk-K products
    int64_t chunk = (int64_t)((double)(int64_t(1) << 39) / std::max(b->work_per_step, 1.0));
    chunk = std::min<int64_t>(std::max<int64_t>(chunk, 1), 1000);
    int64_t done = 0;
    while (done < steps) {
        const int64_t k = std::min(chunk, steps - done);
        if (b->copy_pending) MHAR_HIP(hipEventSynchronize(b->copied), "descriptor buffer reuse");
        for (int i = 0; i < b->count; ++i) {
            mhar_chains* c = b->chains[i];
            MHAR_HIP(refresh_lowrank(c, stream), "low-rank screening operand");
            int rf = 0;
            if (c->force_recompute) {
                rf = 1;
                c->force_recompute = 0;
                c->pending = 0;
                c->T = 2;
                c->since = 0;
            }
            StepArgs a = make_args(c);
            a.steps = (int)k;
            a.recompute_first = rf;
            b->descs_host[i] = a;
        }
        MHAR_HIP(hipMemcpyAsync(b->descs_dev, b->descs_host, sizeof(StepArgs) * b->count,
                                hipMemcpyHostToDevice, stream), "descriptor copy");
        MHAR_HIP(hipEventRecord(b->copied, stream), "descriptor copy event");
        b->copy_pending = true;
        if (b->nunits > 0) {
            MHAR_HIP(launch_fill_i32((int*)b->next_dev, 1, 0, stream), "queue reset");
            MHAR_HIP(launch_batch(b->prec, b->descs_dev, b->units_dev, b->nunits, b->next_dev,
                                  b->max_lda, b->grid, stream), "batched launch");
        }
        if (b->ntu > 0) {
            // which steps of this launch some tiled problem recomputes after
            int first = 0, any_split = 0;
            b->due.assign((size_t)k, 0);
            for (int i = 0; i < b->count; ++i) {
                if (!b->chains[i]->tiled) continue;   // general-kernel part
                const StepArgs& a = b->descs_host[i];
                first |= a.recompute_first;
                any_split |= a.rk > 0;
                for (int64_t s = (a.R - 1 - a.since0); s < k; s += a.R) b->due[(size_t)s] = 1;
            }
            MHAR_HIP(launch_grouped(b->prec, b->descs_dev, b->stiles_dev, b->nst, b->tunits_dev,
                                    b->ntu, b->rtiles_dev, b->nrt, (int)k, first, b->due.data(),
                                    any_split, stream), "grouped tiled launch");
        }
        for (mhar_chains* c : b->chains) advance_schedule(c, k);
        done += k;
    }
    return MHAR_OK;
}

mhar_status_t mhar_batch_destroy(mhar_batch_t b)
{
    if (!b) return MHAR_OK;
    hipError_t e = b->copy_pending ? hipEventSynchronize(b->copied) : hipSuccess;
    for (int i = 0; i < b->count; ++i) {
        mhar_chains* c = b->chains[i];
        c->last_kernel = 0;   // the handle's own path again
        if (b->saved_split[i] > 0 && c->pc_rank == 0) {
            c->split = b->saved_split[i];
            c->tiled = b->saved_tiled[i];
            c->force_recompute = 1;
        }
    }
    hipError_t e2 = hipEventDestroy(b->copied);
    if (e == hipSuccess) e = e2;
    e2 = hipHostFree(b->descs_host);
    if (e == hipSuccess) e = e2;
    if (b->owns_chains)
        for (mhar_chains* c : b->chains) mhar_chains_destroy(c);
    for (mhar_problem* p : b->owned_problems) mhar_problem_destroy(p);
    delete b;
    if (e != hipSuccess) return hip_fail(e, "batch teardown");
    return MHAR_OK;
}

mhar_status_t mhar_batch_get_chains(mhar_batch_t b, int32_t i, mhar_chains_t* out)
{
    if (!b || !out) return fail(MHAR_E_INVALID_ARG, "batch and out must be non-NULL");
    if (i < 0 || i >= b->count) return fail(MHAR_E_INVALID_ARG, "index outside the batch");
    *out = b->chains[i];
    return MHAR_OK;
}

// Workspace of a packed batch: per problem its problem workspace then its
// chains workspace (each 256-byte aligned), then the batch tables sized for
// the larger of the two kernel paths of every problem.
static mhar_status_t packed_layout(int32_t count, const int64_t* n, const int64_t* m, const int64_t* z,
                                   const mhar_options_t& o, std::vector<size_t>* offs, size_t* total)
{
    if (count < 1 || !n || !m || !z) return fail(MHAR_E_INVALID_ARG, "need count >= 1 and the n, m, z arrays");
    size_t at = 0;
    BatchPlan bound;
    uint64_t walks = 0;
    for (int i = 0; i < count; ++i) {
        ProblemDims d;
        mhar_status_t st = check_dims(n[i], m[i], 0, o, &d);
        if (st) return fail(st, "problem " + std::to_string(i) + ": " + g_last_error);
        if (d.lda > kMaxN) return fail(MHAR_E_UNSUPPORTED, "problem " + std::to_string(i) + ": batches take n <= " + std::to_string(kMaxN));
        if (z[i] < 1 || z[i] > (int64_t(1) << 31)) return fail(MHAR_E_SHAPE, "z must be in [1, 2^31]");
        walks += (uint64_t)z[i];
        if (walks > (uint64_t(1) << 32)) return fail(MHAR_E_SHAPE, "the batch's walks must number at most 2^32");
        mhar_problem shape{};
        shape.n = d.n;
        shape.m = d.m;
        shape.m_pad = d.m_pad;
        shape.lda = d.lda;
        shape.prec = o.precision;
        const size_t pb = carve_problem(d, o.precision, nullptr, nullptr);
        const int z_pad = (int)round_up(z[i], kChainTile);
        const size_t cb = carve_chains(&shape, z_pad, nullptr, nullptr);
        if (offs) offs->push_back(at);
        at += (size_t)round_up((int64_t)pb, 256);
        if (offs) offs->push_back(at);
        at += (size_t)round_up((int64_t)cb, 256);
        const int tiles = z_pad / kChainTile;
        bound.gen_units.resize(bound.gen_units.size() + tiles);
        bound.tiled_units.resize(bound.tiled_units.size() + tiles);
        bound.stiles.resize(bound.stiles.size() + (size_t)((d.m_pad + kScreenRows - 1) / kScreenRows) *
                                                     ((z_pad + kScreenWalks - 1) / kScreenWalks));
        bound.rtiles.resize(bound.rtiles.size() + (size_t)((d.m_pad + kRecRows - 1) / kRecRows) *
                                                     ((z_pad + kRecWalks - 1) / kRecWalks));
    }
    if (offs) offs->push_back(at);
    *total = at + carve_batch(count, bound, nullptr, nullptr);
    return MHAR_OK;
}

mhar_status_t mhar_batch_packed_workspace_size(int32_t count, const int64_t* n, const int64_t* m,
                                               const int64_t* z, const mhar_options_t* opt, size_t* bytes)
{
    if (!bytes) return fail(MHAR_E_INVALID_ARG, "bytes is NULL");
    mhar_options_t o;
    mhar_status_t st = check_options(opt, &o);
    if (st) return st;
    return packed_layout(count, n, m, z, o, nullptr, bytes);
}

mhar_status_t mhar_batch_create_packed(int32_t count, const int64_t* n, const int64_t* m, const int64_t* z,
                                       const double* A_packed, const int64_t* A_offsets,
                                       const double* b_packed, const int64_t* b_offsets,
                                       const double* X0_packed, const int64_t* X0_offsets, uint64_t seed,
                                       const mhar_options_t* opt, void* ws, size_t ws_bytes, void* stream,
                                       mhar_batch_t* out)
{
    if (!out) return fail(MHAR_E_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (!A_packed || !A_offsets || !b_packed || !b_offsets || !X0_packed || !X0_offsets)
        return fail(MHAR_E_INVALID_ARG, "packed arrays and offsets must be non-NULL");
    mhar_options_t o;
    mhar_status_t st = check_options(opt, &o);
    if (st) return st;
    std::vector<size_t> offs;
    size_t need = 0;
    st = packed_layout(count, n, m, z, o, &offs, &need);
    if (st) return st;
    for (int i = 0; i < count; ++i)
        if (A_offsets[i] < 0 || b_offsets[i] < 0 || X0_offsets[i] < 0)
            return fail(MHAR_E_INVALID_ARG, "negative offset for problem " + std::to_string(i));
    if (!ws || !aligned256(ws)) return fail(MHAR_E_WORKSPACE, "workspace must be 256-byte aligned");
    if (ws_bytes < need) return fail(MHAR_E_WORKSPACE, "workspace too small: need " + std::to_string(need) + " bytes");
    unsigned char* base = (unsigned char*)ws;
    std::vector<mhar_problem*> probs;
    std::vector<mhar_chains_t> chains;
    auto cleanup = [&](mhar_status_t code) {
        const std::string msg = g_last_error;
        for (mhar_chains* c : chains) mhar_chains_destroy(c);
        for (mhar_problem* p : probs) mhar_problem_destroy(p);
        g_last_error = msg;
        return code;
    };
    uint64_t walk0 = 0;
    for (int i = 0; i < count; ++i) {
        const size_t p_at = offs[2 * i], c_at = offs[2 * i + 1], end = offs[2 * i + 2];
        mhar_problem_t p = nullptr;
        st = mhar_problem_create(n[i], m[i], A_packed + A_offsets[i], b_packed + b_offsets[i], 0, nullptr,
                                 nullptr, &o, base + p_at, c_at - p_at, stream, &p);
        if (st) return cleanup(fail(st, "problem " + std::to_string(i) + ": " + g_last_error));
        probs.push_back(p);
        mhar_chains_t c = nullptr;
        st = mhar_chains_create(p, z[i], X0_packed + X0_offsets[i], seed, walk0, base + c_at, end - c_at,
                                stream, &c);
        if (st) return cleanup(fail(st, "problem " + std::to_string(i) + ": " + g_last_error));
        chains.push_back(c);
        walk0 += (uint64_t)z[i];
    }
    const size_t tab = offs[2 * count];
    mhar_batch_t b = nullptr;
    st = mhar_batch_create(count, chains.data(), base + tab, ws_bytes - tab, &b);
    if (st) return cleanup(st);
    b->owned_problems = probs;
    b->owns_chains = true;
    *out = b;
    return MHAR_OK;
}

mhar_status_t mhar_run_noalloc(int64_t n, int64_t m, const double* A, const double* b,
                               int64_t m_eq, const double* A_eq, const double* b_eq, int64_t z,
                               double* X, int32_t* status, uint64_t seed, uint64_t chain_offset,
                               uint64_t step0, int64_t steps, const mhar_options_t* opt,
                               void* stream)
{
    if (!A || !b || !X || !status) return fail(MHAR_E_INVALID_ARG, "A, b, X and status must be non-NULL");
    if (steps < 0) return fail(MHAR_E_INVALID_ARG, "steps must be >= 0");
    if (z < 1 || z > (int64_t(1) << 31)) return fail(MHAR_E_SHAPE, "z must be in [1, 2^31]");
    mhar_options_t o;
    mhar_status_t st = check_options(opt, &o);
    if (st) return st;
    ProblemDims d;
    st = check_dims(n, m, m_eq, o, &d);
    if (st) return st;
    // the two workspaces the handles would take, carved from the static scratch
    const size_t pb = (size_t)round_up((int64_t)carve_problem(d, o.precision, nullptr, nullptr), 256);
    mhar_problem shape{};
    shape.n = d.n;
    shape.m = d.m;
    shape.m_pad = d.m_pad;
    shape.lda = d.lda;
    shape.m_eq = d.m_eq;
    shape.prec = o.precision;
    const size_t cb = carve_chains(&shape, (int)round_up(z, kChainTile), nullptr, nullptr);
    void* base = nullptr;
    size_t cap = 0;
    MHAR_HIP(noalloc_scratch(&base, &cap), "static scratch address");
    if (pb + cb > cap)
        return fail(MHAR_E_WORKSPACE, "this problem needs " + std::to_string(pb + cb) +
                                          " bytes of scratch; the static scratch holds " + std::to_string(cap));
    mhar_problem_t prob = nullptr;
    st = mhar_problem_create(n, m, A, b, m_eq, A_eq, b_eq, &o, base, pb, stream, &prob);
    if (st) return st;
    mhar_chains_t ch = nullptr;
    st = mhar_chains_create(prob, z, X, seed, chain_offset, (char*)base + pb, cb, stream, &ch);
    if (st) {
        mhar_problem_destroy(prob);
        return st;
    }
    ch->step = step0;
    st = mhar_step(ch, steps, stream);
    if (!st) st = mhar_get_state(ch, X, status, stream);
    mhar_chains_destroy(ch);
    mhar_problem_destroy(prob);
    return st;
}

// ---- checkpoint and restore ----
// Host layout: a fixed header, then X (z x n FP64), the status bits (z int32,
// padded to 8 bytes), and with a covariance U, V, the Adam moments of V (n x r
// FP64 each), log sigma and the moments of log sigma (n each), the Dikin fit's
// power vector (n).  Native byte order.
struct CkptHeader {
    char magic[8];          // "MHARCKPT"
    uint32_t version;       // 1
    uint32_t has_pc;
    int64_t n, z;
    uint64_t seed, chain_offset, step;
    int32_t rank, objective, frozen, fit_status;
    int64_t adam_t;
    double kappa;
};

static size_t ckpt_bytes(const mhar_chains* c)
{
    const size_t n = c->p->n, z = c->z;
    size_t b = sizeof(CkptHeader) + z * n * 8 + (z * 4 + 7) / 8 * 8;
    if (c->pc_rank) b += 4 * n * c->pc_rank * 8 + 4 * n * 8;
    return b;
}

mhar_status_t mhar_checkpoint(mhar_chains_t c, void* host_buf, size_t* bytes, void* stream)
{
    if (!c || !bytes) return fail(MHAR_E_INVALID_ARG, "chains and bytes must be non-NULL");
    const size_t need = ckpt_bytes(c);
    if (!host_buf) {
        *bytes = need;
        return MHAR_OK;
    }
    if (*bytes < need) return fail(MHAR_E_WORKSPACE, "checkpoint buffer too small: need " + std::to_string(need) + " bytes");
    hipStream_t s = (hipStream_t)stream;
    const int n = c->p->n, z = c->z, r = c->pc_rank;
    char* out = (char*)host_buf;
    CkptHeader h{};
    std::memcpy(h.magic, "MHARCKPT", 8);
    h.version = 1;
    h.has_pc = r > 0;
    h.n = n;
    h.z = z;
    h.seed = c->seed;
    h.chain_offset = c->chain_offset;
    h.step = c->step;
    h.rank = r;
    h.objective = r ? c->pc.objective : 0;
    h.frozen = c->pc_frozen;
    h.adam_t = c->pc_t;
    h.kappa = r ? c->pc.kappa : 0.0;
    size_t o = sizeof(CkptHeader);
    MHAR_HIP(hipMemcpy2DAsync(out + o, (size_t)n * 8, c->X, (size_t)c->p->lda * 8, (size_t)n * 8, z,
                              hipMemcpyDeviceToHost, s), "state read");
    o += (size_t)z * n * 8;
    MHAR_HIP(hipMemcpyAsync(out + o, c->flags, (size_t)z * 4, hipMemcpyDeviceToHost, s), "status read");
    int32_t* st = (int32_t*)(out + o);
    o += ((size_t)z * 4 + 7) / 8 * 8;
    int fit = 0;
    if (r) {
        const size_t nr = (size_t)n * r * 8, nb = (size_t)n * 8;
        const double* arrays[4] = {c->pc.U, c->pc.V, c->pc.m1V, c->pc.m2V};
        for (const double* a : arrays) {
            MHAR_HIP(hipMemcpyAsync(out + o, a, nr, hipMemcpyDeviceToHost, s), "covariance read");
            o += nr;
        }
        const double* vecs[3] = {c->pc.logsig, c->pc.m1l, c->pc.m2l};
        for (const double* a : vecs) {
            MHAR_HIP(hipMemcpyAsync(out + o, a, nb, hipMemcpyDeviceToHost, s), "covariance read");
            o += nb;
        }
        if (c->pc.objective == MHAR_FIT_DIKIN)
            MHAR_HIP(hipMemcpyAsync(out + o, c->pc.pv, nb, hipMemcpyDeviceToHost, s), "covariance read");
        else
            std::memset(out + o, 0, nb);
        o += nb;
        MHAR_HIP(hipMemcpyAsync(&fit, c->pc.status, sizeof(int), hipMemcpyDeviceToHost, s), "status read");
    }
    MHAR_HIP(hipStreamSynchronize(s), "stream synchronize");
    for (int k = 0; k < z; ++k) st[k] &= 15;
    h.fit_status = fit;
    std::memcpy(out, &h, sizeof(h));
    *bytes = need;
    return MHAR_OK;
}

mhar_status_t mhar_restore(mhar_chains_t c, const void* host_buf, size_t bytes, void* stream)
{
    if (!c || !host_buf) return fail(MHAR_E_INVALID_ARG, "chains and host_buf must be non-NULL");
    if (bytes < sizeof(CkptHeader)) return fail(MHAR_E_INVALID_ARG, "not a checkpoint (too short)");
    CkptHeader h;
    std::memcpy(&h, host_buf, sizeof(h));
    if (std::memcmp(h.magic, "MHARCKPT", 8) != 0 || h.version != 1)
        return fail(MHAR_E_INVALID_ARG, "not a checkpoint of this library version");
    const int n = c->p->n, z = c->z, r = c->pc_rank;
    if (h.n != n || h.z != z) return fail(MHAR_E_SHAPE, "the checkpoint has other n or z");
    if (h.seed != c->seed || h.chain_offset != c->chain_offset)
        return fail(MHAR_E_STATE, "the checkpoint was taken with another seed or chain offset");
    if ((int)h.has_pc != (r > 0) || (r && (h.rank != r || h.objective != c->pc.objective)))
        return fail(MHAR_E_STATE, "attach a covariance of the checkpoint's rank and objective first "
                                  "(or detach it when the checkpoint has none)");
    if (bytes < ckpt_bytes(c)) return fail(MHAR_E_INVALID_ARG, "checkpoint truncated");
    hipStream_t s = (hipStream_t)stream;
    const char* in = (const char*)host_buf;
    size_t o = sizeof(CkptHeader);
    // the states go through D (zeroed again afterwards) to the padded layout
    MHAR_HIP(hipMemcpyAsync(c->D, in + o, (size_t)z * n * 8, hipMemcpyHostToDevice, s), "state write");
    o += (size_t)z * n * 8;
    MHAR_HIP(launch_copy_states(n, c->p->lda, z, c->z_pad, c->D, c->X, s), "state import");
    MHAR_HIP(launch_fill_i32((int*)c->D, (int64_t)c->z_pad * c->p->lda * 2, 0, s), "direction reset");
    MHAR_HIP(launch_fill_i32(c->flags, c->z_pad, 0, s), "status reset");
    MHAR_HIP(launch_fill_i32((int*)c->theta, (int64_t)c->z_pad * 2, 0, s), "theta reset");
    const size_t st_off = o;
    o += ((size_t)z * 4 + 7) / 8 * 8;
    if (r) {
        const size_t nr = (size_t)n * r * 8, nb = (size_t)n * 8;
        double* arrays[4] = {c->pc.U, c->pc.V, c->pc.m1V, c->pc.m2V};
        for (double* a : arrays) {
            MHAR_HIP(hipMemcpyAsync(a, in + o, nr, hipMemcpyHostToDevice, s), "covariance write");
            o += nr;
        }
        double* vecs[3] = {c->pc.logsig, c->pc.m1l, c->pc.m2l};
        for (double* a : vecs) {
            MHAR_HIP(hipMemcpyAsync(a, in + o, nb, hipMemcpyHostToDevice, s), "covariance write");
            o += nb;
        }
        if (c->pc.objective == MHAR_FIT_DIKIN)
            MHAR_HIP(hipMemcpyAsync(c->pc.pv, in + o, nb, hipMemcpyHostToDevice, s), "covariance write");
        o += nb;
        MHAR_HIP(launch_precond_esig(c->pc, s), "covariance scale");
        MHAR_HIP(launch_fill_i32(c->pc.status, 1, h.fit_status, s), "fit status");
        c->pc_t = h.adam_t;
        c->pc_frozen = h.frozen;
        c->pc.kappa = h.kappa;
        c->pc_lr_stale = 1;
    }
    c->step = h.step;
    // exact slack of the restored states, then the saved status bits
    mhar_status_t st = run_steps(c, 0, 1, nullptr, 0, 0, s);
    if (st) return st;
    MHAR_HIP(hipMemcpyAsync(c->flags, in + st_off, (size_t)z * 4, hipMemcpyHostToDevice, s), "status write");
    // the host buffer may be reused once this returns
    MHAR_HIP(hipStreamSynchronize(s), "stream synchronize");
    return MHAR_OK;
}

static void trace_release(mhar_chains* c)
{
    for (hipEvent_t e : c->trace_events) (void)hipEventDestroy(e);
    c->trace_events.clear();
    c->trace_kinds.clear();
    c->trace = KernelTrace{nullptr, nullptr, 0, 0};
}

mhar_status_t mhar_trace_enable(mhar_chains_t c, int32_t max_launches)
{
    if (!c) return fail(MHAR_E_INVALID_ARG, "chains is NULL");
    if (max_launches < 0 || max_launches > (1 << 20))
        return fail(MHAR_E_INVALID_ARG, "max_launches must be in [0, 2^20]");
    trace_release(c);
    if (max_launches == 0) return MHAR_OK;
    c->trace_events.resize(2 * (size_t)max_launches);
    for (size_t i = 0; i < c->trace_events.size(); ++i) {
        hipError_t e = hipEventCreate(&c->trace_events[i]);
        if (e != hipSuccess) {
            c->trace_events.resize(i);
            trace_release(c);
            return hip_fail(e, "trace event create");
        }
    }
    c->trace_kinds.assign((size_t)max_launches, 0);
    c->trace = KernelTrace{c->trace_events.data(), c->trace_kinds.data(), max_launches, 0};
    return MHAR_OK;
}

mhar_status_t mhar_trace_read(mhar_chains_t c, void* stream, mhar_trace_t* out)
{
    if (!c || !out) return fail(MHAR_E_INVALID_ARG, "chains and out must be non-NULL");
    if (c->trace.cap == 0) return fail(MHAR_E_STATE, "tracing is not enabled");
    MHAR_HIP(hipStreamSynchronize((hipStream_t)stream), "stream synchronize");
    *out = mhar_trace_t{};
    for (int i = 0; i < c->trace.used; ++i) {
        float ms = 0.0f;
        MHAR_HIP(hipEventElapsedTime(&ms, c->trace.ev[2 * i], c->trace.ev[2 * i + 1]), "trace read");
        const int k = c->trace.kind[i];
        out->launches[k] += 1;
        out->ms[k] += ms;
    }
    c->trace.used = 0;
    return MHAR_OK;
}

mhar_status_t mhar_chains_autotune(mhar_chains_t c, int64_t steps_per_trial, void* stream_,
                                   mhar_tune_t* out)
{
    if (!c || !out) return fail(MHAR_E_INVALID_ARG, "chains and out must be non-NULL");
    if (steps_per_trial < 1 || steps_per_trial > (int64_t(1) << 20))
        return fail(MHAR_E_INVALID_ARG, "steps_per_trial must be in [1, 2^20]");
    hipStream_t stream = (hipStream_t)stream_;
    const mhar_problem* p = c->p;
    struct Cand {
        int path, split, tiled, lane;
    };
    std::vector<Cand> cands;
    if (p->lda <= kMaxN) cands.push_back({MHAR_PATH_GENERAL, 0, 0, 0});
    const int rs = resident_split(p->prec, p->lda, p->m_pad, c->z_pad);
    if (rs > 0 && c->pc_rank == 0) cands.push_back({MHAR_PATH_RESIDENT, rs, 0, 0});
    // with a covariance the tiled path needs the split screening's buffers,
    // which are sized when the covariance is attached to a tiled handle
    if (p->prec != MHAR_FP64 && (c->pc_rank == 0 || c->pc.rk > 0))
        cands.push_back({MHAR_PATH_TILED, 0, 1, 0});
    if (lane_fits(p->n, p->m) && c->pc_rank == 0) cands.push_back({MHAR_PATH_LANE, 0, 0, 1});
    std::memset(out, 0, sizeof(*out));
    for (int i = 0; i < 5; ++i) out->ms_per_step[i] = -1.0;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    auto release = [&]() {
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
    };
    if (e != hipSuccess) {
        release();
        return hip_fail(e, "autotune events");
    }
    const Cand keep{0, c->split, c->tiled, c->lane};
    int best = -1;
    double best_ms = 0.0;
    mhar_status_t st = MHAR_OK;
    for (size_t i = 0; i < cands.size() && st == MHAR_OK; ++i) {
        const Cand& k = cands[i];
        c->split = k.split;
        c->tiled = k.tiled;
        c->lane = k.lane;
        c->force_recompute = 1;
        // the exact recompute a path switch takes stays outside the timed steps
        st = run_steps(c, 0, 1, nullptr, 0, 0, stream);
        if (st) break;
        e = hipEventRecord(e0, stream);
        if (e == hipSuccess) st = run_steps(c, steps_per_trial, 0, nullptr, 0, 0, stream);
        if (e == hipSuccess && st == MHAR_OK) e = hipEventRecord(e1, stream);
        if (e == hipSuccess && st == MHAR_OK) e = hipEventSynchronize(e1);
        float ms = 0.0f;
        if (e == hipSuccess && st == MHAR_OK) e = hipEventElapsedTime(&ms, e0, e1);
        if (e != hipSuccess) st = hip_fail(e, "autotune timing");
        if (st) break;
        const double per = (double)ms / (double)steps_per_trial;
        out->ms_per_step[k.path] = per;
        if (best < 0 || per < best_ms) {
            best = (int)i;
            best_ms = per;
        }
    }
    release();
    const Cand& pick = best >= 0 && st == MHAR_OK ? cands[best] : keep;
    c->split = pick.split;
    c->tiled = pick.tiled;
    c->lane = pick.lane;
    c->force_recompute = 1;
    if (st) return st;
    out->path = cands[best].path;
    return MHAR_OK;
}

mhar_status_t mhar_chains_set_graph(mhar_chains_t c, int32_t graph_steps)
{
    if (!c) return fail(MHAR_E_INVALID_ARG, "chains is NULL");
    if (graph_steps < 0 || (graph_steps > 0 && graph_steps % c->p->R != 0))
        return fail(MHAR_E_INVALID_ARG, "graph_steps must be 0 or a multiple of the recompute period R = " +
                                            std::to_string(c->p->R));
    if (graph_steps != c->graph_steps) drop_graph(c);
    c->graph_steps = graph_steps;
    return MHAR_OK;
}

mhar_status_t mhar_chains_destroy(mhar_chains_t c)
{
    if (!c) return MHAR_OK;
    c->p->live_chains -= 1;
    trace_release(c);
    drop_graph(c);
    if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
    delete c;
    return MHAR_OK;
}

}  // extern "C"
