// C ABI of the HWFV1 library: validation, workspace layout, descriptors,
// per-phase entry points, plans with a captured step graph, and the batched
// ensemble.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cstdarg>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "hw_device.h"
#include "hwfv1.h"

namespace hw {
hipError_t launch_set_desc(const Desc& d, Desc* dst, hipStream_t s);
hipError_t launch_ingest(int prec, const Desc* dd, uint32_t grid,
                         const double* h, const double* qx, const double* qy,
                         const double* z, hipStream_t s);
hipError_t launch_encode_bed(Launch lc, uint32_t nblocks, int pass, int tl,
                             int cpt, hipStream_t s);
hipError_t launch_encode_flow(int prec, Launch lc, uint32_t nblocks, int pass,
                              int tl, int cpt, bool skip, double* details, hipStream_t s,
                              int tiles = 1);
hipError_t launch_flag_only(int prec, Launch lc, uint32_t nblocks, hipStream_t s);
hipError_t launch_regularise(Launch lc, uint32_t nblocks, int fold_pass, int tl,
                             hipStream_t s);
hipError_t launch_traverse(Launch lc, uint32_t nblocks, hipStream_t s);
hipError_t launch_fv1(int prec, const Desc* descs, int n, uint32_t grid,
                      Launch fill, uint32_t fill_blocks, hipStream_t s);
hipError_t launch_export(int prec, const Desc* dd, uint64_t N, double* h,
                         double* qx, double* qy, hipStream_t s);
hipError_t launch_fv1_only(int prec, const Desc* descs, int n, uint32_t grid, hipStream_t s);
hipError_t launch_fv1_heavy(int prec, const Desc* descs, int n, uint32_t grid, hipStream_t s);
hipError_t launch_fill(int prec, Launch fill, uint32_t fill_blocks, uint32_t grid,
                       hipStream_t s);
hipError_t launch_finalize(int prec, const Desc* descs, int n, uint32_t grid, hipStream_t s);
hipError_t launch_forget(const Desc* dd, uint64_t nhist, hipStream_t s);
hipError_t launch_densify(int prec, const Desc* dd, int L, hipStream_t s);
// One thread waits until `ticks` of the constant-rate wall clock have
// passed (at most `ticks` plus one sleep interval; no memory is touched).
// Used by the phase timing only: while it runs, the host queues the step's
// launches and events, so no timed interval contains host launch latency.
__global__ void k_hold(uint64_t ticks)
{
    if (threadIdx.x != 0) return;
    const uint64_t t0 = (uint64_t)wall_clock64();
    while ((uint64_t)wall_clock64() - t0 < ticks) __builtin_amdgcn_s_sleep(16);
}

hipError_t launch_hold(uint64_t ticks, hipStream_t s)
{
    hipLaunchKernelGGL(k_hold, dim3(1), dim3(kWave), 0, s, ticks);
    return hipGetLastError();
}

}  // namespace hw

using hw::Desc;
using hw::Launch;

namespace {

thread_local std::string g_err;

int fail(int code, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
int fail(int code, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

int ok()
{
    g_err.clear();
    return HW_OK;
}

int hip_fail(hipError_t e, const char* what)
{
    return fail(HW_EHIP, "%s: %s", what, hipGetErrorString(e));
}

constexpr size_t kAlign = 256;
size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

int group_level(int L) { return L >= 2 ? L - 2 : 0; }
uint64_t hw_n_fine_(int L) { return 1ull << (2 * L); }
uint64_t n_groups(int L) { return 1ull << (2 * group_level(L)); }
uint32_t n_trav(int L) { return (uint32_t)((n_groups(L) + hw::kBlock - 1) / hw::kBlock); }
uint32_t n_coarse_blocks(int L)
{
    return (uint32_t)((hw::level_off(L) + hw::kBlock - 1) / hw::kBlock);
}
// regularisation threads: one per 2x2 block of levels 1..L-1 (at least one)
uint32_t n_reg_blocks(int L)
{
    const uint64_t t = L >= 2 ? hw::level_off(L - 1) : 1;
    return (uint32_t)((t + hw::kBlock - 1) / hw::kBlock);
}

// Levels per encoding pass for a given number of in-register levels.
int pass_levels(int cp) { return cp + 4; }
int n_passes(int L, int tl) { return (L + tl - 1) / tl; }
uint32_t encode_blocks(int L, int pass, int tl)
{
    const int n_in = L - pass * tl;
    if (n_in <= 0) return 0;
    const int lv = n_in < tl ? n_in : tl;
    return (uint32_t)(1ull << (2 * (n_in - lv)));
}

struct WorkLayout {
    size_t desc, tcount, big_src, gcode, lmap, wet, hist, dryb, bpart, partials, rsig, total;
};

// Entries of the FV1 write history: one per 64-cell Morton block of the
// finest level (at least one).
size_t n_hist(int L) { size_t n = (size_t)hw_n_fine_(L) / 64; return n ? n : 1; }

WorkLayout work_layout(int L)
{
    WorkLayout w;
    size_t o = 0;
    w.desc = o;
    o = align_up(o + sizeof(Desc));
    w.tcount = o;
    // per traversal workgroup: leaf counts, then whole finest block counts
    o = align_up(o + 2 * (n_trav(L) + 1) * sizeof(uint32_t));
    w.big_src = o;
    o = align_up(o + n_groups(L) * sizeof(uint32_t));
    w.gcode = o;
    o = align_up(o + n_groups(L));
    w.lmap = o;
    o = align_up(o + (size_t)hw_n_fine_(L));
    w.wet = o;
    o = align_up(o + 4 * ((size_t)hw_n_fine_(L) / (hw::kLeafBatch * hw::kBlock) + 1));
    w.hist = o;
    o = align_up(o + n_hist(L) * sizeof(uint64_t));
    w.dryb = o;
    o = align_up(o + n_hist(L));
    w.bpart = o;
    o = align_up(o + 2 * n_hist(L) * sizeof(double));
    w.partials = o;
    o = align_up(o + 2 * (size_t)hw::kMaxFv1Grid * hw::kPartial * sizeof(double));
    // one record per regularisation workgroup
    w.rsig = o;
    o = align_up(o + n_reg_blocks(L));
    w.total = o;
    return w;
}

bool aligned(const void* p) { return ((uintptr_t)p % kAlign) == 0; }

int check_problem(const hw_problem* p)
{
    if (!p) return fail(HW_EINVAL, "problem is NULL");
    if (p->L < 1 || p->L > HW_MAX_L)
        return fail(HW_EINVAL, "L = %d outside 1..%d", p->L, HW_MAX_L);
    if (p->precision != HW_FP64 && p->precision != HW_FP32_BULK)
        return fail(HW_EINVAL, "unknown precision %d", p->precision);
    for (int k = 0; k < 4; ++k)
        if (p->bc[k] != HW_BC_WALL && p->bc[k] != HW_BC_OPEN)
            return fail(HW_EINVAL, "bc[%d] = %d is neither wall nor open", k, p->bc[k]);
    if (!(p->eps >= 0.0) || !std::isfinite(p->eps))
        return fail(HW_EINVAL, "eps must be finite and >= 0");
    if (!(p->g > 0.0) || !std::isfinite(p->g)) return fail(HW_EINVAL, "g must be > 0");
    if (!(p->cfl > 0.0) || !(p->cfl <= 1.0)) return fail(HW_EINVAL, "cfl must be in (0, 1]");
    if (!(p->h_tol >= 0.0) || !std::isfinite(p->h_tol))
        return fail(HW_EINVAL, "h_tol must be finite and >= 0");
    if (!(p->dx > 0.0) || !(p->dy > 0.0) || !std::isfinite(p->dx) || !std::isfinite(p->dy))
        return fail(HW_EINVAL, "dx, dy must be finite and > 0");
    if (!(p->dt_max > 0.0) || !std::isfinite(p->dt_max))
        return fail(HW_EINVAL, "dt_max must be finite and > 0");
    if (!(p->manning_n >= 0.0) || !std::isfinite(p->manning_n))
        return fail(HW_EINVAL, "manning_n must be finite and >= 0");
    if (!std::isfinite(p->rain_rate)) return fail(HW_EINVAL, "rain_rate must be finite");
    if (!(p->t_end > 0.0)) return fail(HW_EINVAL, "t_end must be > 0 (or +inf)");
    if (!std::isfinite(p->zsmax) || p->zsmax < 0.0)
        return fail(HW_EINVAL, "zsmax must be finite and >= 0");
    if (!std::isfinite(p->q_peak) || p->q_peak < 0.0)
        return fail(HW_EINVAL, "q_peak must be finite and >= 0");
    if (p->q_peak > 0.0) {
        if (!(p->t_peak > 0.0) || !(p->t_base > p->t_peak))
            return fail(HW_EINVAL, "hydrograph needs 0 < t_peak < t_base");
        if (!(p->inlet_y1 > p->inlet_y0))
            return fail(HW_EINVAL, "inflow segment needs inlet_y1 > inlet_y0");
    }
    return HW_OK;
}

int check_buffers(const hw_problem* p, const hw_buffers* b)
{
    if (!b) return fail(HW_EINVAL, "buffers is NULL");
    const void* ptrs[] = {b->fine[0][0], b->fine[0][1], b->fine[0][2],
                          b->fine[1][0], b->fine[1][1], b->fine[1][2],
                          b->coarse[0], b->coarse[1],   b->coarse[2],
                          b->zhier,      b->zsig,       b->raw,
                          b->sig,        b->leaves,     b->scal,
                          b->work};
    const char* names[] = {"fine[0][0]", "fine[0][1]", "fine[0][2]",
                           "fine[1][0]", "fine[1][1]", "fine[1][2]",
                           "coarse[0]",  "coarse[1]",  "coarse[2]",
                           "zhier",      "zsig",       "raw",
                           "sig",        "leaves",     "scal",
                           "work"};
    for (size_t k = 0; k < sizeof(ptrs) / sizeof(ptrs[0]); ++k) {
        if (!ptrs[k]) return fail(HW_EINVAL, "buffer %s is NULL", names[k]);
        if (!aligned(ptrs[k]))
            return fail(HW_EINVAL, "buffer %s is not 256-byte aligned", names[k]);
    }
    const size_t need = work_layout(p->L).total;
    if (b->work_bytes < need)
        return fail(HW_ECAPACITY, "work buffer has %zu bytes, %zu needed",
                    b->work_bytes, need);
    return HW_OK;
}

Desc make_desc(const hw_problem* p, const hw_buffers* b, double* partials)
{
    Desc d;
    std::memset(&d, 0, sizeof d);
    d.L = p->L;
    d.precision = p->precision;
    for (int k = 0; k < 4; ++k) d.bc[k] = p->bc[k];
    d.group_level = group_level(p->L);
    d.write_skip = 1;
    d.full_outputs = 1;   // the entry points write every output; plans do not
    d.eps = p->eps;
    d.g = p->g;
    d.cfl = p->cfl;
    d.h_tol = p->h_tol;
    d.dx = p->dx;
    d.dy = p->dy;
    d.dt_max = p->dt_max;
    d.manning_n = p->manning_n;
    d.rain_rate = p->rain_rate;
    d.inlet_y0 = p->inlet_y0;
    d.inlet_y1 = p->inlet_y1;
    d.q_peak = p->q_peak;
    d.t_peak = p->t_peak;
    d.t_base = p->t_base;
    d.t_end = p->t_end;
    d.zsmax = p->zsmax;
    for (int s = 0; s < 2; ++s)
        for (int v = 0; v < 3; ++v) d.fine[s][v] = b->fine[s][v];
    for (int v = 0; v < 3; ++v) d.coarse[v] = b->coarse[v];
    d.zhier = b->zhier;
    d.zsig = b->zsig;
    d.raw = b->raw;
    d.sig = b->sig;
    d.leaves = b->leaves;
    d.scal = b->scal;
    const WorkLayout w = work_layout(p->L);
    char* wk = static_cast<char*>(b->work);
    d.tcount = reinterpret_cast<uint32_t*>(wk + w.tcount);
    d.big_src = reinterpret_cast<uint32_t*>(wk + w.big_src);
    d.lmap = reinterpret_cast<uint8_t*>(wk + w.lmap);
    d.gcode = reinterpret_cast<uint8_t*>(wk + w.gcode);
    d.wet = reinterpret_cast<uint8_t*>(wk + w.wet);
    d.hist = reinterpret_cast<uint64_t*>(wk + w.hist);
    d.dryb = reinterpret_cast<uint8_t*>(wk + w.dryb);
    d.bpart = reinterpret_cast<double*>(wk + w.bpart);
    d.nhist = (uint32_t)n_hist(p->L);
    d.partials = partials ? partials : reinterpret_cast<double*>(wk + w.partials);
    d.rsig = reinterpret_cast<uint8_t*>(wk + w.rsig);
    d.nreg = n_reg_blocks(p->L);
    d.ntrav = n_trav(p->L);
    return d;
}

Desc* work_desc(const hw_buffers* b)
{
    return reinterpret_cast<Desc*>(static_cast<char*>(b->work) + work_layout(0).desc);
}

// Default FV1 grid: enough persistent workgroups to fill 256 CUs, capped by
// the leaf count; always a multiple of 8 (one share per XCD).
uint32_t default_fv1_grid(uint64_t max_leaves)
{
    uint64_t chunks = (max_leaves + hw::kBlock - 1) / hw::kBlock;
    uint64_t g = 2048;
    if (chunks < g) g = chunks;
    g = (g + 7) / 8 * 8;
    if (g < 8) g = 8;
    return (uint32_t)g;
}

struct Prep {
    int rc;
    Desc d;
};

// Validate and upload the single-problem descriptor into the workspace.
int prep_single(const hw_problem* p, const hw_buffers* b, hipStream_t s,
                Desc* host_out)
{
    int rc = check_problem(p);
    if (rc) return rc;
    rc = check_buffers(p, b);
    if (rc) return rc;
    *host_out = make_desc(p, b, nullptr);
    hipError_t e = hw::launch_set_desc(*host_out, work_desc(b), s);
    if (e != hipSuccess) return hip_fail(e, "descriptor upload");
    return HW_OK;
}


}  // namespace

// ---------------------------------------------------------------------------
// plans
// ---------------------------------------------------------------------------

struct hw_plan {
    int n = 0;
    int precision = 0;
    int tl = 5, cp = 1;
    uint32_t fv1_grid = 8;
    int write_skip = 1;
    int encode_skip = 1;
    bool uniform = false;                     // uniform FV1 plan (FV1 and finalize only)
    std::vector<hw_problem> problems;
    std::vector<hw_buffers> buffers;
    std::vector<Desc> host_desc;
    // device memory owned by the plan
    void* dmem = nullptr;
    Desc* d_desc = nullptr;
    double* d_partials = nullptr;
    // launch decomposition
    int passes = 0;
    // five levels per pass and at least two passes: the last pass (one
    // workgroup per problem, levels <= 4) runs inside the regularisation
    bool fold_last = false;
    // one FP32 problem, four cells per thread, no span skip: each first-pass
    // workgroup encodes this many tiles (1: the usual form)
    int first_tiles = 1;
    std::vector<uint32_t> enc_blocks;         // per pass
    std::vector<const uint32_t*> enc_prefix;  // per pass (device)
    uint32_t coarse_blocks = 0, trav_blocks = 0, reg_blocks = 0;
    const uint32_t* coarse_prefix = nullptr;
    const uint32_t* reg_prefix = nullptr;
    const uint32_t* trav_prefix = nullptr;
    // captured step
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipStream_t own = nullptr;
};

namespace {

// Launch one phase of a step for all problems of the plan.
hipError_t enqueue_phase(hw_plan* pl, int phase, hipStream_t s)
{
    hipError_t e = hipSuccess;
    const int n = pl->n;
    // a uniform FV1 plan updates every finest cell: no encoding, flags,
    // traversal or copy-down
    if (pl->uniform && phase != HW_PH_FV1 && phase != HW_PH_FINALIZE) return e;
    switch (phase) {
    case HW_PH_ENCODE:
        for (int k = 0; k < pl->passes - (pl->fold_last ? 1 : 0) && e == hipSuccess; ++k) {
            if (!pl->enc_blocks[k]) continue;
            const int tiles = k == 0 ? pl->first_tiles : 1;
            e = hw::launch_encode_flow(pl->precision,
                                       Launch{pl->d_desc, pl->enc_prefix[k], n},
                                       pl->enc_blocks[k] / (uint32_t)tiles, k, pl->tl, pl->cp,
                                       pl->encode_skip != 0, nullptr, s, tiles);
        }
        break;
    case HW_PH_REGULARISE:
        e = hw::launch_regularise(Launch{pl->d_desc, pl->reg_prefix, n}, pl->reg_blocks,
                                  pl->fold_last ? pl->passes - 1 : -1, pl->tl, s);
        break;
    case HW_PH_TRAVERSE:
        e = hw::launch_traverse(Launch{pl->d_desc, pl->trav_prefix, n}, pl->trav_blocks, s);
        break;
    case HW_PH_FV1:
        e = hw::launch_fv1_only(pl->precision, pl->d_desc, n, pl->fv1_grid, s);
        break;
    case HW_PH_FILL:
        // the copy-down and the finalisation share one launch
        e = hw::launch_fill(pl->precision, Launch{pl->d_desc, pl->trav_prefix, n},
                            pl->trav_blocks, pl->fv1_grid, s);
        break;
    case HW_PH_FINALIZE:
        // a uniform FV1 plan has no copy-down: it finalises on its own
        if (pl->uniform) e = hw::launch_finalize(pl->precision, pl->d_desc, n, pl->fv1_grid, s);
        break;
    }
    return e;
}

int enqueue_step(hw_plan* pl, hipStream_t s)
{
    for (int ph = 0; ph < HW_NPHASE; ++ph) {
        hipError_t e = enqueue_phase(pl, ph, s);
        if (e != hipSuccess) return hip_fail(e, "step launch");
    }
    return HW_OK;
}

void plan_release(hw_plan* pl)
{
    if (!pl) return;
    if (pl->exec) (void)hipGraphExecDestroy(pl->exec);
    if (pl->graph) (void)hipGraphDestroy(pl->graph);
    if (pl->own) (void)hipStreamDestroy(pl->own);
    if (pl->dmem) (void)hipFree(pl->dmem);
    delete pl;
}

int plan_capture(hw_plan* pl)
{
    if (pl->exec) return HW_OK;
    hipError_t e;
    if (!pl->own) {
        e = hipStreamCreateWithFlags(&pl->own, hipStreamNonBlocking);
        if (e != hipSuccess) return hip_fail(e, "stream create");
    }
    e = hipStreamBeginCapture(pl->own, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return hip_fail(e, "begin capture");
    int rc = enqueue_step(pl, pl->own);
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(pl->own, &g);
    if (rc) {
        if (g) (void)hipGraphDestroy(g);
        return rc;
    }
    if (e != hipSuccess) return hip_fail(e, "end capture");
    pl->graph = g;
    e = hipGraphInstantiate(&pl->exec, g, nullptr, nullptr, 0);
    if (e != hipSuccess) return hip_fail(e, "graph instantiate");
    return HW_OK;
}

// Replay the step graph on the caller's stream.  The graph runs on the
// caller's stream directly (graph launches are ordinary stream work).
int plan_replay(hw_plan* pl, int64_t steps, hipStream_t s, bool stop_when_done,
                const hw_scalars* watch)
{
    const int64_t chunk = 64;
    int64_t done_steps = 0;
    while (done_steps < steps) {
        int64_t k = steps - done_steps < chunk ? steps - done_steps : chunk;
        for (int64_t q = 0; q < k; ++q) {
            hipError_t e = hipGraphLaunch(pl->exec, s);
            if (e != hipSuccess) return hip_fail(e, "graph launch");
        }
        done_steps += k;
        if (stop_when_done && done_steps < steps) {
            uint32_t all_done = 1;
            for (int i = 0; i < pl->n; ++i) {
                uint32_t dn = 0;
                hipError_t e = hipMemcpyAsync(&dn, &pl->buffers[i].scal->done,
                                              sizeof dn, hipMemcpyDeviceToHost, s);
                if (e == hipSuccess) e = hipStreamSynchronize(s);
                if (e != hipSuccess) return hip_fail(e, "done flag read");
                all_done &= dn;
            }
            if (all_done) break;
        }
    }
    (void)watch;
    return HW_OK;
}

// Complete the spans the last copy-down of each problem left stale (a
// no-op for problems and plans that leave none).
hipError_t plan_densify(hw_plan* pl, hipStream_t s)
{
    for (int i = 0; i < pl->n; ++i) {
        if (!hw::sparse_fine(pl->host_desc[i])) continue;
        hipError_t e = hw::launch_densify(pl->precision, pl->d_desc + i, pl->problems[i].L, s);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

int fill_stats(hw_plan* pl, const std::vector<uint64_t>& step0, hw_stats* stats,
               double wall, hipStream_t s)
{
    hipError_t e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "stream synchronize");
    int rc = HW_OK;
    for (int i = 0; i < pl->n; ++i) {
        hw_scalars sc;
        e = hipMemcpy(&sc, pl->buffers[i].scal, sizeof sc, hipMemcpyDeviceToHost);
        if (e != hipSuccess) return hip_fail(e, "scalar read");
        if (stats) {
            hw_stats& st = stats[i];
            st.steps = (int64_t)(sc.step - step0[i]);
            st.t = sc.t;
            st.dt = sc.dt;
            st.mass0 = sc.mass0;
            st.mass = sc.mass;
            st.n_leaves = sc.n_leaves;
            st.leaf_updates = sc.leaf_updates;
            st.clips = sc.clips;
            st.dry_stored = sc.dry_stored;
            st.dry_skipped = sc.dry_skipped;
            st.wall_s = wall;
        }
        if (sc.nonfinite && rc == HW_OK)
            rc = fail(HW_ENONFINITE, "problem %d: non-finite value (flag %u)", i,
                      sc.nonfinite);
    }
    return rc;
}

}  // namespace

// ---------------------------------------------------------------------------
// Scratch of the traversal variant that allocates nothing
// ---------------------------------------------------------------------------
// mra_traverse_leaves_noalloc keeps what mra_traverse_leaves keeps in the
// caller's workspace (descriptor, per-workgroup leaf counts and offsets,
// walk codes, fill table and leaf-level map) in one array per GPU instead,
// sized for the largest level it accepts.
namespace {

constexpr int kNoAllocMaxL = 11;

constexpr size_t ce_align(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

struct TravScratch {
    size_t desc, tcount, big_src, gcode, lmap, total;
};

constexpr TravScratch trav_scratch_layout(int L)
{
    const size_t N = size_t(1) << (2 * L);
    const size_t groups = size_t(1) << (2 * (L >= 2 ? L - 2 : 0));
    const size_t ntrav = (groups + hw::kBlock - 1) / hw::kBlock;
    TravScratch t{};
    size_t o = 0;
    t.desc = o;
    o = ce_align(o + sizeof(Desc));
    t.tcount = o;
    o = ce_align(o + (ntrav + 1) * sizeof(uint32_t));
    t.big_src = o;
    o = ce_align(o + groups * sizeof(uint32_t));
    t.gcode = o;
    o = ce_align(o + groups);
    t.lmap = o;
    o = ce_align(o + N);
    t.total = o;
    return t;
}

constexpr size_t kScratchBytes = trav_scratch_layout(kNoAllocMaxL).total;

}  // namespace

// One copy per GPU, alive until the process ends.  Host code never uses
// this name as an address: it takes the device address that
// hipGetSymbolAddress returns for the current device (scratch_base).
static __device__ __align__(256) uint8_t scratch[kScratchBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_dev[kMaxDevices] = {};

// Device address of the scratch array on the current device, looked up once
// per device (with that device current) and kept.
int scratch_base(void** out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (dev < 0 || dev >= kMaxDevices)
        return fail(HW_EINVAL, "device %d is beyond the %d devices the library tracks", dev,
                    kMaxDevices);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
        if (!p) return fail(HW_EHIP, "hipGetSymbolAddress(scratch) returned NULL");
        g_scratch_dev[dev] = p;
    }
    *out = g_scratch_dev[dev];
    return HW_OK;
}

}  // namespace

extern "C" {

const char* hw_last_error(void) { return g_err.c_str(); }

int hw_validate(const hw_problem* p)
{
    int rc = check_problem(p);
    return rc ? rc : ok();
}

uint64_t hw_n_fine(int32_t L) { return (L < 0 || L > HW_MAX_L) ? 0 : 1ull << (2 * L); }
uint64_t hw_n_coarse(int32_t L) { return (L < 0 || L > HW_MAX_L) ? 0 : hw::level_off(L); }
uint64_t hw_n_hier(int32_t L) { return (L < 0 || L > HW_MAX_L) ? 0 : hw::level_off(L + 1); }

size_t hw_workspace_bytes(const hw_problem* p)
{
    if (check_problem(p)) return 0;
    return work_layout(p->L).total;
}

void hw_default_tuning(const hw_problem* p, hw_tuning* out)
{
    if (!out) return;
    out->encode_cells_per_thread = 4;
    out->fv1_block = hw::kBlock;
    out->fv1_grid = 0;
    out->fv1_write_skip = 1;
    out->encode_skip = 1;
    out->fill_skip = 1;
    out->block_list = 1;
    // FP32 moves half the bytes per tile, so two tiles per workgroup keep
    // more loads in flight; FP64's paired loads already do
    out->encode_tiles = p && p->precision == HW_FP32_BULK ? 2 : 1;
}

int hw_ingest(const hw_problem* p, const hw_buffers* b, const double* h,
              const double* qx, const double* qy, const double* z,
              hipStream_t stream)
{
    Desc d;
    int rc = prep_single(p, b, stream, &d);
    if (rc) return rc;
    if (!h || !qx || !qy || !z) return fail(HW_EINVAL, "input array is NULL");
    const Desc* dd = work_desc(b);
    const uint64_t N = hw_n_fine(p->L);
    uint64_t grid = (N + hw::kBlock - 1) / hw::kBlock;
    if (grid > 2048) grid = 2048;
    hipError_t e = hw::launch_ingest(p->precision, dd, (uint32_t)grid, h, qx, qy, z, stream);
    if (e != hipSuccess) return hip_fail(e, "ingest launch");
    e = hw::launch_forget(dd, n_hist(p->L), stream);
    if (e != hipSuccess) return hip_fail(e, "history reset launch");
    const int cp = 1, tl = pass_levels(cp);
    for (int k = 0; k < n_passes(p->L, tl); ++k) {
        e = hw::launch_encode_bed(Launch{dd, nullptr, 1}, encode_blocks(p->L, k, tl), k,
                                  tl, cp, stream);
        if (e != hipSuccess) return hip_fail(e, "bed encode launch");
    }
    return ok();
}

int mra_encode(const hw_problem* p, const hw_buffers* b, double* details,
               hipStream_t stream)
{
    Desc d;
    int rc = prep_single(p, b, stream, &d);
    if (rc) return rc;
    if (details && ((uintptr_t)details % 8))
        return fail(HW_EINVAL, "details must be 8-byte aligned");
    const Desc* dd = work_desc(b);
    hw_tuning tu;
    hw_default_tuning(p, &tu);
    const int cp = tu.encode_cells_per_thread == 16 ? 2 : 1, tl = pass_levels(cp);
    for (int k = 0; k < n_passes(p->L, tl); ++k) {
        hipError_t e = hw::launch_encode_flow(p->precision, Launch{dd, nullptr, 1},
                                              encode_blocks(p->L, k, tl), k, tl, cp,
                                              false, details, stream);
        if (e != hipSuccess) return hip_fail(e, "encode launch");
    }
    return ok();
}

int mra_flag(const hw_problem* p, const hw_buffers* b, hipStream_t stream)
{
    Desc d;
    int rc = prep_single(p, b, stream, &d);
    if (rc) return rc;
    const Desc* dd = work_desc(b);
    hipError_t e = hw::launch_flag_only(p->precision, Launch{dd, nullptr, 1},
                                        n_coarse_blocks(p->L), stream);
    if (e == hipSuccess)
        e = hw::launch_regularise(Launch{dd, nullptr, 1}, n_reg_blocks(p->L), -1, 0, stream);
    if (e != hipSuccess) return hip_fail(e, "flag launch");
    return ok();
}

int mra_traverse_leaves(const hw_problem* p, const hw_buffers* b, hipStream_t stream)
{
    Desc d;
    int rc = prep_single(p, b, stream, &d);
    if (rc) return rc;
    const Desc* dd = work_desc(b);
    hipError_t e = hw::launch_traverse(Launch{dd, nullptr, 1}, n_trav(p->L), stream);
    if (e != hipSuccess) return hip_fail(e, "traverse launch");
    return ok();
}

size_t hw_noalloc_scratch_bytes(void) { return kScratchBytes; }

int mra_traverse_leaves_noalloc(const hw_problem* p, const hw_buffers* b,
                                hipStream_t stream)
{
    int rc = check_problem(p);
    if (rc) return rc;
    if (p->L > kNoAllocMaxL)
        return fail(HW_ECAPACITY,
                    "L = %d: mra_traverse_leaves_noalloc holds levels up to %d "
                    "(%zu bytes of scratch per GPU); use mra_traverse_leaves",
                    p->L, kNoAllocMaxL, kScratchBytes);
    if (!b) return fail(HW_EINVAL, "buffers is NULL");
    const void* ptrs[] = {b->sig, b->leaves, b->scal};
    const char* names[] = {"sig", "leaves", "scal"};
    for (int k = 0; k < 3; ++k) {
        if (!ptrs[k]) return fail(HW_EINVAL, "buffer %s is NULL", names[k]);
        if (!aligned(ptrs[k]))
            return fail(HW_EINVAL, "buffer %s is not 256-byte aligned", names[k]);
    }
    void* base = nullptr;
    rc = scratch_base(&base);
    if (rc) return rc;
    // Descriptor with the traversal's scratch arrays in the per-GPU array;
    // nothing else of the workspace is touched by the traversal kernels.
    hw_buffers bb = *b;
    bb.work = base;
    Desc d = make_desc(p, &bb, nullptr);
    const TravScratch t = trav_scratch_layout(p->L);
    char* sb = static_cast<char*>(base);
    d.tcount = reinterpret_cast<uint32_t*>(sb + t.tcount);
    d.big_src = reinterpret_cast<uint32_t*>(sb + t.big_src);
    d.gcode = reinterpret_cast<uint8_t*>(sb + t.gcode);
    d.lmap = reinterpret_cast<uint8_t*>(sb + t.lmap);
    d.wet = nullptr;
    d.hist = nullptr;
    d.dryb = nullptr;
    d.bpart = nullptr;
    d.partials = nullptr;
    d.rsig = nullptr;
    Desc* dd = reinterpret_cast<Desc*>(sb + t.desc);
    hipError_t e = hw::launch_set_desc(d, dd, stream);
    if (e != hipSuccess) return hip_fail(e, "descriptor upload");
    e = hw::launch_traverse(Launch{dd, nullptr, 1}, n_trav(p->L), stream);
    if (e != hipSuccess) return hip_fail(e, "traverse launch");
    return ok();
}

int fv1_step(const hw_problem* p, const hw_buffers* b, hipStream_t stream)
{
    Desc d;
    int rc = prep_single(p, b, stream, &d);
    if (rc) return rc;
    const Desc* dd = work_desc(b);
    const uint32_t grid = default_fv1_grid(hw_n_fine(p->L));
    hipError_t e = hw::launch_fv1(p->precision, dd, 1, grid, Launch{dd, nullptr, 1},
                                  n_trav(p->L), stream);
    if (e != hipSuccess) return hip_fail(e, "fv1 launch");
    return ok();
}

int hw_forget(const hw_problem* p, const hw_buffers* b, hipStream_t stream)
{
    Desc d;
    int rc = prep_single(p, b, stream, &d);
    if (rc) return rc;
    hipError_t e = hw::launch_forget(work_desc(b), n_hist(p->L), stream);
    if (e != hipSuccess) return hip_fail(e, "history reset launch");
    return ok();
}

int hw_export(const hw_problem* p, const hw_buffers* b, double* h, double* qx,
              double* qy, hipStream_t stream)
{
    Desc d;
    int rc = prep_single(p, b, stream, &d);
    if (rc) return rc;
    hipError_t e = hw::launch_export(p->precision, work_desc(b), hw_n_fine(p->L), h, qx,
                                     qy, stream);
    if (e != hipSuccess) return hip_fail(e, "export launch");
    return ok();
}

// Plan of n problems; uniform: every step is the FV1 update of every finest
// cell (no encoding, flags or traversal).
static int plan_create(hw_plan** out, const hw_problem* problems, const hw_buffers* buffers,
                       int32_t n, const hw_tuning* tuning, bool uniform)
{
    if (!out) return fail(HW_EINVAL, "plan output pointer is NULL");
    *out = nullptr;
    if (n < 1 || n > hw::kMaxScen)
        return fail(HW_EINVAL, "plan needs 1..%d problems, got %d", hw::kMaxScen, n);
    if (!problems || !buffers) return fail(HW_EINVAL, "problems/buffers is NULL");
    for (int i = 0; i < n; ++i) {
        int rc = check_problem(&problems[i]);
        if (!rc) rc = check_buffers(&problems[i], &buffers[i]);
        if (rc) {
            std::string m = g_err;
            return fail(rc, "problem %d: %s", i, m.c_str());
        }
        if (problems[i].precision != problems[0].precision)
            return fail(HW_EINVAL, "all problems of a plan need the same precision");
    }
    hw_plan* pl = new (std::nothrow) hw_plan;
    if (!pl) return fail(HW_EINVAL, "out of host memory");
    pl->n = n;
    pl->uniform = uniform;
    pl->precision = problems[0].precision;
    pl->problems.assign(problems, problems + n);
    pl->buffers.assign(buffers, buffers + n);
    hw_tuning tu;
    hw_default_tuning(&problems[0], &tu);
    int maxL = 0;
    uint64_t max_leaves = 0;
    for (int i = 0; i < n; ++i) {
        maxL = problems[i].L > maxL ? problems[i].L : maxL;
        max_leaves += hw_n_fine(problems[i].L);
    }
    {
        hw_problem pm = problems[0];
        pm.L = maxL;
        hw_default_tuning(&pm, &tu);
    }
    if (tuning) {
        if (tuning->encode_cells_per_thread == 4 || tuning->encode_cells_per_thread == 16)
            tu.encode_cells_per_thread = tuning->encode_cells_per_thread;
        else if (tuning->encode_cells_per_thread != 0) {
            delete pl;
            return fail(HW_EINVAL, "encode_cells_per_thread must be 4 or 16");
        }
        if (tuning->fv1_grid < 0 || tuning->fv1_grid > hw::kMaxFv1Grid) {
            delete pl;
            return fail(HW_EINVAL, "fv1_grid must be in 0..%d", hw::kMaxFv1Grid);
        }
        tu.fv1_grid = tuning->fv1_grid;
        if (tuning->fv1_write_skip != 0 && tuning->fv1_write_skip != 1) {
            delete pl;
            return fail(HW_EINVAL, "fv1_write_skip must be 0 or 1");
        }
        tu.fv1_write_skip = tuning->fv1_write_skip;
        if (tuning->encode_skip != 0 && tuning->encode_skip != 1) {
            delete pl;
            return fail(HW_EINVAL, "encode_skip must be 0 or 1");
        }
        tu.encode_skip = tuning->encode_skip;
        if (tuning->fill_skip != 0 && tuning->fill_skip != 1) {
            delete pl;
            return fail(HW_EINVAL, "fill_skip must be 0 or 1");
        }
        tu.fill_skip = tuning->fill_skip;
        if (tuning->encode_tiles != 0 && tuning->encode_tiles != 1 &&
            tuning->encode_tiles != 2 && tuning->encode_tiles != 4) {
            delete pl;
            return fail(HW_EINVAL, "encode_tiles must be 0, 1, 2 or 4");
        }
        if (tuning->encode_tiles != 0) tu.encode_tiles = tuning->encode_tiles;
        if (tuning->block_list < 0 || tuning->block_list > 2) {
            delete pl;
            return fail(HW_EINVAL, "block_list must be 0, 1 or 2");
        }
        tu.block_list = tuning->block_list;
    }
    pl->cp = tu.encode_cells_per_thread == 16 ? 2 : 1;
    pl->write_skip = tu.fv1_write_skip;
    pl->encode_skip = tu.encode_skip;
    pl->tl = pass_levels(pl->cp);
    pl->fv1_grid = tu.fv1_grid > 0 ? (uint32_t)((tu.fv1_grid + 7) / 8 * 8)
                                   : default_fv1_grid(max_leaves);
    if (pl->fv1_grid > (uint32_t)hw::kMaxFv1Grid) pl->fv1_grid = hw::kMaxFv1Grid;

    // decomposition and device memory: descriptors, prefixes, partials
    pl->passes = n_passes(maxL, pl->tl);
    pl->fold_last = !uniform && pl->tl == 5 && pl->passes >= 2;
    std::vector<uint32_t> pre;  // all prefix arrays concatenated
    std::vector<size_t> enc_off(pl->passes);
    for (int k = 0; k < pl->passes; ++k) {
        enc_off[k] = pre.size();
        uint32_t acc = 0;
        for (int i = 0; i < n; ++i) {
            pre.push_back(acc);
            acc += encode_blocks(problems[i].L, k, pl->tl);
        }
        pre.push_back(acc);
        pl->enc_blocks.push_back(acc);
    }
    if (!uniform && n == 1 && pl->cp == 1 && !pl->encode_skip) {
        const int want = tu.encode_tiles;
        if (want > 1 && pl->enc_blocks[0] >= (uint32_t)want && pl->enc_blocks[0] % want == 0)
            pl->first_tiles = want;
    }
    const size_t coarse_off = pre.size();
    {
        uint32_t acc = 0;
        for (int i = 0; i < n; ++i) {
            pre.push_back(acc);
            acc += n_coarse_blocks(problems[i].L);
        }
        pre.push_back(acc);
        pl->coarse_blocks = acc;
    }
    const size_t reg_off = pre.size();
    {
        uint32_t acc = 0;
        for (int i = 0; i < n; ++i) {
            pre.push_back(acc);
            acc += n_reg_blocks(problems[i].L);
        }
        pre.push_back(acc);
        pl->reg_blocks = acc;
    }
    const size_t trav_off = pre.size();
    {
        uint32_t acc = 0;
        for (int i = 0; i < n; ++i) {
            pre.push_back(acc);
            acc += n_trav(problems[i].L);
        }
        pre.push_back(acc);
        pl->trav_blocks = acc;
    }
    const size_t desc_bytes = align_up(n * sizeof(Desc));
    const size_t pre_bytes = align_up(pre.size() * sizeof(uint32_t));
    const size_t part_bytes =
        align_up(2 * (size_t)n * pl->fv1_grid * hw::kPartial * sizeof(double));
    hipError_t e = hipMalloc(&pl->dmem, desc_bytes + pre_bytes + part_bytes);
    if (e != hipSuccess) {
        plan_release(pl);
        return hip_fail(e, "plan allocation");
    }
    char* base = static_cast<char*>(pl->dmem);
    pl->d_desc = reinterpret_cast<Desc*>(base);
    uint32_t* d_pre = reinterpret_cast<uint32_t*>(base + desc_bytes);
    pl->d_partials = reinterpret_cast<double*>(base + desc_bytes + pre_bytes);
    for (int i = 0; i < n; ++i) {
        pl->host_desc.push_back(make_desc(
            &problems[i], &buffers[i],
            pl->d_partials + 2 * (size_t)i * pl->fv1_grid * hw::kPartial));
        pl->host_desc.back().write_skip = pl->write_skip;
        pl->host_desc.back().encode_skip = tu.encode_skip;
        pl->host_desc.back().fill_skip = tu.fill_skip;
        pl->host_desc.back().block_list = tu.block_list;
        pl->host_desc.back().full_outputs = 0;
        pl->host_desc.back().uniform = uniform ? 1 : 0;
    }
    const bool single = n == 1;
    for (int k = 0; k < pl->passes; ++k)
        pl->enc_prefix.push_back(single ? nullptr : d_pre + enc_off[k]);
    pl->coarse_prefix = single ? nullptr : d_pre + coarse_off;
    pl->reg_prefix = single ? nullptr : d_pre + reg_off;
    pl->trav_prefix = single ? nullptr : d_pre + trav_off;
    e = hipMemcpy(pl->d_desc, pl->host_desc.data(), n * sizeof(Desc), hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = hipMemcpy(d_pre, pre.data(), pre.size() * sizeof(uint32_t), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        plan_release(pl);
        return hip_fail(e, "plan upload");
    }
    *out = pl;
    return ok();
}

int hw_plan_create(hw_plan** out, const hw_problem* problems, const hw_buffers* buffers,
                   int32_t n, const hw_tuning* tuning)
{
    return plan_create(out, problems, buffers, n, tuning, false);
}

int hw_plan_create_uniform(hw_plan** out, const hw_problem* problems,
                           const hw_buffers* buffers, int32_t n, const hw_tuning* tuning)
{
    return plan_create(out, problems, buffers, n, tuning, true);
}

int hw_plan_destroy(hw_plan* plan)
{
    plan_release(plan);
    return ok();
}

static int run_plan(hw_plan* pl, int64_t max_steps, hw_stats* stats, hipStream_t stream)
{
    if (max_steps < 0) return fail(HW_EINVAL, "max_steps must be >= 0");
    const auto t0 = std::chrono::steady_clock::now();
    std::vector<uint64_t> step0(pl->n, 0);
    hipError_t e;
    if (stats) {
        for (int i = 0; i < pl->n; ++i) {
            e = hipMemcpyAsync(&step0[i], &pl->buffers[i].scal->step, sizeof(uint64_t),
                               hipMemcpyDeviceToHost, stream);
            if (e != hipSuccess) return hip_fail(e, "step read");
        }
        e = hipStreamSynchronize(stream);
        if (e != hipSuccess) return hip_fail(e, "stream synchronize");
    }
    int rc = plan_capture(pl);
    if (rc) return rc;
    bool finite_end = false;
    for (int i = 0; i < pl->n; ++i) finite_end |= std::isfinite(pl->problems[i].t_end);
    rc = plan_replay(pl, max_steps, stream, finite_end, nullptr);
    if (rc) return rc;
    e = plan_densify(pl, stream);
    if (e != hipSuccess) return hip_fail(e, "densify launch");
    if (stats) {
        e = hipStreamSynchronize(stream);
        if (e != hipSuccess) return hip_fail(e, "stream synchronize");
        const double wall =
            std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        rc = fill_stats(pl, step0, stats, wall, stream);
        if (rc) return rc;
    }
    return ok();
}

int hwfv1_run(const hw_problem* p, const hw_buffers* b, hw_plan* plan,
              int64_t max_steps, hw_stats* stats, hipStream_t stream)
{
    hw_plan* pl = plan;
    if (!pl) {
        int rc = hw_plan_create(&pl, p, b, 1, nullptr);
        if (rc) return rc;
    } else if (pl->n != 1) {
        return fail(HW_EINVAL, "hwfv1_run needs a plan of one problem");
    }
    int rc = run_plan(pl, max_steps, stats, stream);
    if (!plan) {
        if (!rc) {
            hipError_t e = hipStreamSynchronize(stream);
            if (e != hipSuccess) rc = hip_fail(e, "stream synchronize");
        }
        std::string m = g_err;
        plan_release(pl);
        g_err = m;
    }
    return rc;
}

int hwfv1_run_batch(hw_plan* plan, int64_t max_steps, hw_stats* stats,
                    hipStream_t stream)
{
    if (!plan) return fail(HW_EINVAL, "plan is NULL");
    return run_plan(plan, max_steps, stats, stream);
}

int hw_plan_profile(hw_plan* plan, int64_t steps, double* ms_out, hipStream_t stream)
{
    if (!plan) return fail(HW_EINVAL, "plan is NULL");
    if (!ms_out) return fail(HW_EINVAL, "ms_out is NULL");
    if (steps < 0) return fail(HW_EINVAL, "steps must be >= 0");
    for (int ph = 0; ph < HW_NPROF; ++ph) ms_out[ph] = 0.0;
    // Per phase a start and an end event; per single-launch figure a start
    // and an end event around kRepeat more launches of that kernel, made
    // after its phase (before the next phase starts) on the state its first
    // launch saw: the first encoding pass and the heavy FV1 kernel write
    // nothing they read, so the repeats store the same values again.  Their
    // mean leaves out the dispatch gap that an event next to a single
    // launch would add.
    constexpr int kRepeat = 4;
    constexpr int kEv = 2 * HW_NPHASE + 4;
    hipEvent_t ev[kEv];
    for (int k = 0; k < kEv; ++k) {
        hipError_t e = hipEventCreate(&ev[k]);
        if (e != hipSuccess) {
            for (int q = 0; q < k; ++q) (void)hipEventDestroy(ev[q]);
            return hip_fail(e, "event create");
        }
    }
    hipEvent_t* kev = &ev[2 * HW_NPHASE];
    const bool enc_first = !plan->uniform && plan->passes > 0 && plan->enc_blocks[0] > 0;
    // each step is preceded by a 0.5 ms hold on the stream (see launch_hold)
    int dev = 0, khz = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev) != hipSuccess ||
        khz <= 0)
        khz = 100000;
    const uint64_t hold_ticks = (uint64_t)khz / 2;
    int rc = HW_OK;
    for (int64_t st = 0; st < steps && rc == HW_OK; ++st) {
        hipError_t e = hw::launch_hold(hold_ticks, stream);
        for (int ph = 0; ph < HW_NPHASE && e == hipSuccess; ++ph) {
            e = hipEventRecord(ev[2 * ph], stream);
            if (e == hipSuccess) e = enqueue_phase(plan, ph, stream);
            if (e == hipSuccess) e = hipEventRecord(ev[2 * ph + 1], stream);
            if (e == hipSuccess && ph == HW_PH_ENCODE && enc_first) {
                e = hipEventRecord(kev[0], stream);
                for (int r = 0; r < kRepeat && e == hipSuccess; ++r)
                    e = hw::launch_encode_flow(
                        plan->precision, Launch{plan->d_desc, plan->enc_prefix[0], plan->n},
                        plan->enc_blocks[0] / (uint32_t)plan->first_tiles, 0, plan->tl,
                        plan->cp, plan->encode_skip != 0, nullptr, stream, plan->first_tiles);
                if (e == hipSuccess) e = hipEventRecord(kev[1], stream);
            }
            if (e == hipSuccess && ph == HW_PH_FV1) {
                e = hipEventRecord(kev[2], stream);
                for (int r = 0; r < kRepeat && e == hipSuccess; ++r)
                    e = hw::launch_fv1_heavy(plan->precision, plan->d_desc, plan->n,
                                             plan->fv1_grid, stream);
                if (e == hipSuccess) e = hipEventRecord(kev[3], stream);
            }
        }
        if (e == hipSuccess) e = hipEventSynchronize(ev[2 * HW_NPHASE - 1]);
        for (int ph = 0; ph < HW_NPHASE && e == hipSuccess; ++ph) {
            float ms = 0.f;
            e = hipEventElapsedTime(&ms, ev[2 * ph], ev[2 * ph + 1]);
            ms_out[ph] += ms;
        }
        float ms = 0.f;
        if (e == hipSuccess && enc_first) {
            e = hipEventElapsedTime(&ms, kev[0], kev[1]);
            ms_out[HW_PROF_ENCODE_FIRST] += ms / kRepeat;
        }
        ms = 0.f;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, kev[2], kev[3]);
        ms_out[HW_PROF_FV1_HEAVY] += ms / kRepeat;
        if (e != hipSuccess) rc = hip_fail(e, "phase timing");
    }
    if (rc == HW_OK) {
        hipError_t e = plan_densify(plan, stream);
        if (e != hipSuccess) rc = hip_fail(e, "densify launch");
    }
    for (int k = 0; k < kEv; ++k) (void)hipEventDestroy(ev[k]);
    return rc ? rc : ok();
}

}  // extern "C"
