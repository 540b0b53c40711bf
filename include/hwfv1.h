/*
 * hwfv1.h -- C ABI of the MI355X (gfx950) HWFV1 library.
 *
 * HWFV1 is the Haar-wavelet adaptive first-order finite-volume shallow-water
 * model of Chowdhury, Kesserwani, Rouge and Richmond (2022), "GPU-
 * parallelisation of wavelet-based grid adaptation for fast finite volume
 * modelling: application to shallow water flows".  One timestep (Algorithm 3)
 * is:
 *   1. encoding: Haar scaling coefficients of h, qx, qy on every level of the
 *      nested 2^n x 2^n hierarchy (Section 2.1.2, Eq. 3a, Algorithm 1);
 *   2. flagging: normalised details (Eq. 3b-3d) tested against
 *      2^(n-L) eps (Algorithm 1), OR-ed with the static bed flags, then
 *      regularised so that the face neighbours of a significant cell are
 *      refined as well;
 *   3. traversal: one walk per finest cell down the significance tree
 *      (Section 2.2.2, Algorithm 5) and an ordered compaction of the leaf
 *      cells (Section 2.2.3);
 *   4. FV1: per leaf, same-level neighbour lookup (Section 2.1.3, Fig. 3),
 *      HLL fluxes on hydrostatically reconstructed states, forward Euler
 *      (Eq. 2) with the sources of Eq. 1, write-back of the new leaf value to
 *      its finest descendants (decoding with zero details, Algorithm 4), and
 *      the next CFL timestep (minimum reduction, Section 2.2.3).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Array arguments are DEVICE pointers owned by the caller; the library
 *    never frees them.  Apart from hw_plan_create (which allocates a small
 *    descriptor table that hw_plan_destroy releases), no entry point
 *    allocates device memory.
 *  - Every call is asynchronous on the given HIP stream (NULL = the default
 *    stream); outputs are valid once the stream has synchronised.
 *  - Return value: HW_OK (0) or one of the HW_E* codes below;
 *    hw_last_error() then describes the failure (thread-local string).
 *    Argument validation happens on the host before anything is launched,
 *    so an error return means no work was enqueued, except HW_EHIP which
 *    reports a failed HIP launch or runtime call.
 *  - Layouts (N = 4^L finest cells):
 *      finest arrays     N entries in Morton order (bit k of the column
 *                        index i at bit 2k, bit k of the row index j at bit
 *                        2k+1; Section 2.2.1, Fig. 5);
 *      coarse arrays     levels 0..L-1 concatenated, level n at offset
 *                        (4^n - 1)/3, (N - 1)/3 entries: the hierarchy
 *                        Z-order index of Section 2.2.1 (footnote 2);
 *      bed hierarchy     levels 0..L, (4N - 1)/3 FP64 entries, same index;
 *      flags             one byte per coarse cell, (N - 1)/3 entries;
 *      leaves            hierarchy Z-order index (uint32) of every leaf in
 *                        ascending order of its first finest descendant
 *                        (= depth-first order of Algorithm 2), capacity N;
 *                        after a plan step that uses hw_tuning.block_list
 *                        every aligned 8 x 8 block of finest leaves comes
 *                        first, block by block in that order, and the other
 *                        leaves follow in that order.
 *    Row-major host-side fields are [j][i], j the row (y), i the column (x).
 *  - Precision: HW_FP64 keeps h, qx, qy in FP64; HW_FP32_BULK stores and
 *    updates them in FP32 while the significance test, the bed hierarchy,
 *    the bed differences of the reconstruction, t, dt and the mass sum stay
 *    in FP64.  "flow type" below is double for HW_FP64 and float for
 *    HW_FP32_BULK.
 *  - Device pointers must be 256-byte aligned.  1 <= L <= 14.
 */
#ifndef HWFV1_H
#define HWFV1_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status codes */
enum {
    HW_OK = 0,
    HW_EINVAL = 1,      /* invalid argument (problem, pointer, size)       */
    HW_EINPUT = 2,      /* non-finite or negative-depth input data          */
    HW_ECAPACITY = 3,   /* a buffer is smaller than required                */
    HW_EHIP = 4,        /* HIP runtime or launch failure                    */
    HW_ENONFINITE = 5   /* a non-finite value appeared during the run       */
};

enum { HW_FP64 = 0, HW_FP32_BULK = 1 };
enum { HW_BC_WALL = 0, HW_BC_OPEN = 1 };
enum { HW_W = 0, HW_E = 1, HW_S = 2, HW_N = 3 };

#define HW_MAX_L 14

/*
 * Problem: the user inputs L, eps and t_end of Algorithm 3, the physics of
 * Eq. 1 and the forcing.
 *   L           finest level (grid 2^L x 2^L), 1..14
 *   precision   HW_FP64 or HW_FP32_BULK
 *   bc[4]       W, E, S, N boundary: HW_BC_WALL (normal discharge
 *               mirrored) or HW_BC_OPEN (zero-gradient copy)
 *   eps         error threshold, >= 0 (0 reproduces uniform FV1)
 *   g, cfl      gravity (m/s^2) and CFL number (0.5 in the paper)
 *   h_tol       wet/dry depth threshold (m), >= 0
 *   dx, dy      finest cell size (m), > 0
 *   dt_max      largest timestep (s), > 0; also the step when all is dry
 *   manning_n   Manning coefficient (s m^-1/3), >= 0
 *   rain_rate   uniform rainfall (m/s)
 *   inlet_y0/1  west-edge inflow segment (m); q_peak > 0 switches on the
 *               triangular hydrograph Q(t) rising to q_peak (m^3/s) at
 *               t_peak and back to 0 at t_base
 *   t_end       end time (s); +inf for a fixed number of steps
 *   zsmax       s_max of the bed (Section 2.1.2: the largest bed
 *               coefficient of the finest level), >= 0; 0 takes
 *               max(1, max |z|) over the whole grid at ingest.  A domain
 *               padded to the square grid passes the value of its own
 *               cells, so that the padding's high ground does not change
 *               the normalisation of the bed details inside the domain
 */
typedef struct hw_problem {
    int32_t L;
    int32_t precision;
    int32_t bc[4];
    double eps, g, cfl, h_tol;
    double dx, dy, dt_max;
    double manning_n, rain_rate;
    double inlet_y0, inlet_y1, q_peak, t_peak, t_base;
    double t_end;
    double zsmax;
} hw_problem;

/*
 * Device scalars of one run (one hw_scalars record in device memory).  The
 * record is written by hw_ingest and advanced by every fv1_step; read it
 * back with a plain device-to-host copy.
 */
typedef struct hw_scalars {
    double t;            /* simulation time after the last step            */
    double dt;           /* timestep of the next step                      */
    double mass;         /* sum of h * cell area over the leaves           */
    double mass0;        /* the same sum over the initial finest field     */
    double smax[4];      /* guarded s_max of h, qx, qy, z (max(1, max|s|)) */
    double maxspeed;     /* largest wave speed after the last step         */
    double acc[6];       /* internal per-step accumulators                 */
    uint64_t step;       /* steps taken                                    */
    uint64_t n_leaves;   /* leaves of the last traversal                   */
    uint64_t leaf_updates; /* sum of n_leaves over all steps               */
    uint64_t clips;      /* negative depths clipped to zero                */
    uint64_t dry_stored; /* leaf updates done by the dry pass (a group of
                            64 leaves, or a wave of them, all dry with dry
                            neighbours: h kept, discharges zero), with
                            their stores written                           */
    uint64_t dry_skipped;/* the same with the stores skipped (the set being
                            written already held the result); every other
                            leaf update takes the full update              */
    uint32_t cur;        /* finest set (0 or 1) holding the current state  */
    uint32_t done;       /* 1 once t >= t_end                              */
    uint32_t nonfinite;  /* 1 if a non-finite value was produced           */
    uint32_t map_step;   /* equal to step (low 32 bits) when the leaf-level
                            map describes the tree whose copy-down made the
                            current set: written by the FV1 finalisation of
                            a step whose traversal wrote the map; 0 after
                            hw_ingest, hw_forget and a standalone traversal
                            (the next encoding then reads every cell)      */
} hw_scalars;

/*
 * Buffers of one problem (all device memory, caller-owned):
 *   fine[2][3]  two sets of finest h, qx, qy, N entries each, flow type;
 *               hw_scalars.cur names the set holding the current state and
 *               fv1_step writes the other one and flips cur; after a plan
 *               call only fine[cur] is guaranteed complete
 *   coarse[3]   levels 0..L-1 of h, qx, qy, (N-1)/3 entries, flow type;
 *               mra_encode writes every level, the time loop (hwfv1_run,
 *               hwfv1_run_batch, hw_plan_profile) levels 0..L-2 only: the
 *               step reads a level L-1 value from its four finest children
 *               (the same value bit for bit); with hw_tuning.fill_skip it
 *               may also leave levels L-4..L-2 below a coarse leaf of level
 *               <= L-5 unwritten (the step reads no value below a leaf)
 *   zhier       bed on levels 0..L, (4N-1)/3 FP64 (static after ingest)
 *   zsig        static bed significance flags, (N-1)/3 bytes
 *   raw         significance of the current step before regularisation
 *   sig         significance after regularisation, (N-1)/3 bytes
 *   leaves      leaf list, capacity N uint32; the time loop does not write
 *               it in a step where every finest cell is a leaf (n_leaves =
 *               N: the list is then the finest level in Morton order,
 *               (N-1)/3 + m for m = 0..N-1)
 *   scal        one hw_scalars record
 *   work        scratch of hw_workspace_bytes() bytes, private to the
 *               library; between mra_encode and fv1_step it carries the
 *               encoder's per-64-cell block records (dry flags, mass, max
 *               depth) that the FV1 dry pass reads; between
 *               mra_traverse_leaves and fv1_step the traversal's fill table
 *               and the per-finest-cell leaf level map (N bytes) that the
 *               FV1 neighbour lookup reads; across steps it keeps the FV1
 *               write history (hw_forget)
 */
typedef struct hw_buffers {
    void* fine[2][3];
    void* coarse[3];
    double* zhier;
    uint8_t* zsig;
    uint8_t* raw;
    uint8_t* sig;
    uint32_t* leaves;
    hw_scalars* scal;
    void* work;
    size_t work_bytes;
} hw_buffers;

/* Launch-shape choices (all have defaults; see hw_default_tuning). */
typedef struct hw_tuning {
    int32_t encode_cells_per_thread; /* 4 or 16 finest cells per thread in
                                        each encoding pass (5 or 6 levels) */
    int32_t fv1_block;               /* reserved (FV1 workgroups are 256)  */
    int32_t fv1_grid;                /* FV1 persistent workgroups, 8..8192,
                                        0 = automatic                      */
    int32_t fv1_write_skip;          /* 1: skip the stores of 64-cell blocks
                                        the dry case left unchanged at the
                                        two previous steps (see hw_forget);
                                        0: store every leaf every step     */
    int32_t encode_skip;             /* 1: the first encoding pass loads one
                                        cell of a wave's span of finest
                                        cells when the previous step's tree
                                        has one leaf over the whole span
                                        (the copy-down made them equal);
                                        0: load every finest cell          */
    int32_t fill_skip;               /* 1 (with encode_skip): the copy-down
                                        writes, in each span of 1024 finest
                                        cells below one leaf of level
                                        <= L-5, only the cells the next
                                        encoding reads; the span is made
                                        whole when a later tree refines it
                                        and at the end of every run call;
                                        0: write every cell every step     */
    int32_t encode_tiles;            /* plans of one problem without
                                        encode_skip, 4 cells per thread:
                                        first-pass tiles per workgroup, 1,
                                        2 or 4 (more loads in flight per
                                        workgroup, same results bit for
                                        bit); 0 = the default (FP32 2,
                                        FP64 1)                            */
    int32_t block_list;              /* 1: in a step whose whole aligned
                                        8 x 8 blocks of finest leaves hold
                                        at least 2^19 leaves, the traversal
                                        lists those blocks first and FV1
                                        updates each with one wave through
                                        LDS (same results bit for bit;
                                        with fewer, the depth-first order
                                        is faster); 2: whenever there is a
                                        whole block; 0: depth-first list,
                                        every leaf updated on its own      */
} hw_tuning;

typedef struct hw_plan hw_plan;

typedef struct hw_stats {
    int64_t steps;         /* steps taken by this call                     */
    double t, dt;          /* time and next timestep at the end            */
    double mass0, mass;    /* initial and final mass                       */
    uint64_t n_leaves;     /* leaves of the last step                      */
    uint64_t leaf_updates; /* leaf updates over the whole run              */
    uint64_t clips;
    uint64_t dry_stored;   /* leaf updates of the dry pass, stores written */
    uint64_t dry_skipped;  /* ... stores skipped (both over the whole run) */
    double wall_s;         /* host wall time of the call (s)               */
} hw_stats;

/* Thread-local description of the last failure ("" after success). */
const char* hw_last_error(void);

/* Host-side validation of a problem; HW_OK or HW_EINVAL. */
int hw_validate(const hw_problem* p);

/* Element counts for a problem: finest N, coarse (N-1)/3, bed (4N-1)/3. */
uint64_t hw_n_fine(int32_t L);
uint64_t hw_n_coarse(int32_t L);
uint64_t hw_n_hier(int32_t L);

/* Size in bytes of the scratch buffer hw_buffers.work must provide. */
size_t hw_workspace_bytes(const hw_problem* p);

/* Default launch shapes for a problem. */
void hw_default_tuning(const hw_problem* p, hw_tuning* out);

/*
 * Ingest (initial discretisation, Algorithm 3 before the loop).  Inputs are
 * row-major FP64 device arrays of N entries: depth h >= 0, discharges qx,
 * qy, bed z (all finite).  Writes fine[0] (Morton order, flow type), the
 * bed hierarchy zhier (encoded once with Eq. 3a), the static bed flags zsig
 * (bed details tested like Algorithm 1 with s_max of z), and the scalars:
 * t = 0, the first CFL timestep, s_max of every variable, mass0, cur = 0.
 * Errors: HW_EINVAL for a bad problem or pointer, HW_EHIP on launch failure;
 * invalid data (negative or non-finite) is reported asynchronously through
 * hw_scalars.nonfinite = 2.
 */
int hw_ingest(const hw_problem* p, const hw_buffers* b, const double* h,
              const double* qx, const double* qy, const double* z,
              hipStream_t stream);

/*
 * Encoding (Section 2.1.2, Eq. 3a-3d, Algorithm 1): from the current finest
 * set fine[cur] compute the scaling coefficients of levels L-1 .. 0 of h, qx
 * and qy into coarse[].  If details is not NULL it receives the FP64
 * details, laid out [var 0..2][alpha, beta, gamma][(N-1)/3] (9 (N-1)/3
 * doubles); used by tests.
 */
int mra_encode(const hw_problem* p, const hw_buffers* b, double* details,
               hipStream_t stream);

/*
 * Flagging (Algorithm 1 significance test, then regularisation).  For every
 * coarse cell (n, k) and each of h, qx, qy the normalised detail
 * max(|d_alpha|, |d_beta|, |d_gamma|) / s_max is compared with 2^(n-L) eps in
 * FP64 (details formed from the encoded children); raw = any variable
 * significant OR zsig.  sig = raw of the cell OR raw of any of its four
 * in-domain face neighbours on the same level.  Requires mra_encode of the
 * same state.  Writes raw and sig.
 */
int mra_flag(const hw_problem* p, const hw_buffers* b, hipStream_t stream);

/*
 * Traversal (Section 2.2.2, Algorithm 5) and compaction (Section 2.2.3):
 * every finest cell walks from the root towards itself and stops at the
 * first cell that is on the finest level or not significant; that cell is a
 * leaf.  Leaves are written once each, in ascending order of their first
 * finest descendant, to b->leaves; the count goes to hw_scalars.n_leaves.
 * Requires sig.
 */
int mra_traverse_leaves(const hw_problem* p, const hw_buffers* b,
                        hipStream_t stream);

/*
 * Traversal that allocates nothing and takes no workspace: for callers that
 * cannot allocate device memory or pass a workspace (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc).  Same
 * result as mra_traverse_leaves: b->leaves and hw_scalars.n_leaves (and
 * map_step = 0).  Reads b->sig and b->scal, writes b->leaves and b->scal;
 * b->work is ignored and may be NULL, as may every other buffer.
 * The traversal's own scratch (descriptor, per-workgroup leaf counts, walk
 * codes, fill table, leaf-level map) lives in one device array per GPU of
 * hw_noalloc_scratch_bytes() bytes (levels up to 11), which the library
 * holds until the process ends; its address is looked up on the first call
 * on each device.  Every call on a GPU shares that array and every entry a
 * call reads is written by the same call first, so nothing needs clearing;
 * calls that overlap on one GPU (concurrent streams or threads) race.  The
 * fill table and leaf-level map it builds stay in that array, so fv1_step
 * (which reads them from b->work) must follow mra_traverse_leaves, not this
 * variant.  Errors: HW_ECAPACITY for L > 11 (nothing launched), HW_EINVAL
 * for a bad problem or a NULL / misaligned sig, leaves or scal, HW_EHIP on
 * a failed symbol lookup or launch.
 */
int mra_traverse_leaves_noalloc(const hw_problem* p, const hw_buffers* b,
                                hipStream_t stream);

/* Bytes of the per-GPU scratch array used by mra_traverse_leaves_noalloc. */
size_t hw_noalloc_scratch_bytes(void);

/*
 * FV1 update on the leaves (Sections 2.1.1, 2.1.3, 2.2.3): for every leaf
 * (level m, cell c) the neighbour in each direction is the level-m cell on
 * that side, or the coarser leaf that contains it, or a boundary ghost;
 * hydrostatically reconstructed HLL fluxes, forward Euler with timestep
 * hw_scalars.dt, rain, inflow, positivity clip, dry-cell discharge reset and
 * point-implicit Manning friction.  The new value is written to all finest
 * descendants of the leaf in the other finest set (leaves coarser than
 * level L-2 write their first descendant and a fill kernel copies it to the
 * rest); then t += dt, the next
 * CFL timestep, s_max, mass and counters are updated and cur flips.  Does
 * nothing once hw_scalars.done is set.  Requires the leaf list and the
 * encoding of the same state.
 */
int fv1_step(const hw_problem* p, const hw_buffers* b, hipStream_t stream);

/*
 * Full timestep loop (Algorithm 3): encoding, flagging, traversal and FV1
 * for at most max_steps steps or until t_end.  The step's kernels are
 * captured once into a HIP graph held by the plan and replayed; t, dt and
 * the leaf count stay on the device.  plan may be NULL (a temporary plan is
 * made and destroyed).  stats may be NULL; when given, the call
 * synchronises the stream and fills it.  Between the steps of one call the
 * copy-down may leave spans below coarse leaves incomplete
 * (hw_tuning.fill_skip); the call ends by completing them, so afterwards
 * fine[cur] holds the whole state (the other set may not).
 */
int hwfv1_run(const hw_problem* p, const hw_buffers* b, hw_plan* plan,
              int64_t max_steps, hw_stats* stats, hipStream_t stream);

/*
 * Plans.  A plan holds the device descriptors of n problems (n = 1 for
 * hwfv1_run, up to 64 for hwfv1_run_batch), the launch shapes (tuning may
 * be NULL for the defaults) and the captured step graph.  The buffers must
 * stay valid for the life of the plan.
 */
int hw_plan_create(hw_plan** out, const hw_problem* problems,
                   const hw_buffers* buffers, int32_t n,
                   const hw_tuning* tuning);
int hw_plan_destroy(hw_plan* plan);

/*
 * Uniform FV1 plan: the comparison the paper measures its speed-ups against
 * (FV1 on the finest uniform grid, Sections 1 and 3).  Every step updates
 * every finest cell with its four face neighbours (the FV1 step above with
 * all 4^L finest cells as leaves) and then finalises t, dt, s_max and mass;
 * no encoding, flagging or traversal runs, and eps is ignored.  The result
 * equals HWFV1 with eps = 0.  Arguments, ownership and errors as for
 * hw_plan_create; run it with hwfv1_run (one problem) or hwfv1_run_batch.
 * The coarse levels, flags and leaf list are not written; hw_scalars.n_leaves
 * reads 4^L after the first step.
 */
int hw_plan_create_uniform(hw_plan** out, const hw_problem* problems,
                           const hw_buffers* buffers, int32_t n,
                           const hw_tuning* tuning);

/*
 * Batched ensemble: advance the plan's n independent problems (each with
 * its own L, eps, physics, t and dt) by max_steps lockstep steps, one launch
 * per phase covering all problems, captured as one graph per step.  stats
 * may be NULL or point to n records.  Each problem's state evolves exactly
 * as under hwfv1_run.
 */
int hwfv1_run_batch(hw_plan* plan, int64_t max_steps, hw_stats* stats,
                    hipStream_t stream);

/*
 * Phase timing: run `steps` steps of the plan WITHOUT the graph, launching
 * the same kernels as a replay, with HIP events recorded on `stream` around
 * each phase.  ms_out[HW_NPHASE] receives the total milliseconds per phase
 * (HW_PH_*), summed over the steps, and the mean launch time of two single
 * kernels: ms_out[HW_PROF_ENCODE_FIRST], the first encoding pass (the launch
 * that reads the finest level), and ms_out[HW_PROF_FV1_HEAVY], the FV1
 * kernel that performs the full update of wet leaves, each timed over four
 * extra launches made right after its phase (both write nothing they read,
 * so the extra launches store the same values; the phase times exclude
 * them); ms_out must hold HW_NPROF doubles.  Each step is preceded by a
 * 0.5 ms wait kernel on the stream, so that the host has queued the step's
 * launches and events before the GPU reaches them (no timed interval
 * contains host launch latency).  Synchronises the stream.  For tools that need per-kernel averages
 * (roofline reports).  Like hwfv1_run it ends by completing fine[cur] (not
 * timed).
 */
enum {
    HW_PH_ENCODE = 0,     /* all encoding passes (with flags)            */
    HW_PH_REGULARISE = 1,
    HW_PH_TRAVERSE = 2,   /* count, scan and emit                         */
    HW_PH_FV1 = 3,        /* FV1 update and write-back                    */
    HW_PH_FILL = 4,       /* copy-down of coarse leaves                   */
    HW_PH_FINALIZE = 5,   /* reductions, t, dt                            */
    HW_NPHASE = 6,
    HW_PROF_ENCODE_FIRST = 6,   /* first encoding pass alone (in ENCODE) */
    HW_PROF_FV1_HEAVY = 7,      /* full-update FV1 kernel alone (in FV1)  */
    HW_NPROF = 8
};
int hw_plan_profile(hw_plan* plan, int64_t steps, double* ms_out,
                    hipStream_t stream);

/*
 * Forget the FV1 write history kept in the work buffer.  The FV1 step skips
 * the stores of a 64-cell block of finest leaves that the dry case (all
 * depths <= h_tol, no inflow, no rain) has finished at the two previous
 * steps, because the set being written then already holds the result; it
 * learns this from a per-block record of those steps in `work`.  hw_ingest
 * clears the record.  It also sets hw_scalars.map_step to 0, so the next
 * encoding loads every finest cell instead of one per span below a coarser
 * leaf of the previous tree.  Call this after writing fine[][] or scal by
 * any other means (e.g. restoring a saved state) before the next step.
 * Errors:
 * HW_EINVAL for a bad problem or buffers, HW_EHIP on launch failure.
 */
int hw_forget(const hw_problem* p, const hw_buffers* b, hipStream_t stream);

/*
 * Export the current finest set to row-major FP64 device arrays (N each);
 * any output pointer may be NULL to skip that variable.
 */
int hw_export(const hw_problem* p, const hw_buffers* b, double* h,
              double* qx, double* qy, hipStream_t stream);

#ifdef __cplusplus
}
#endif
#endif
