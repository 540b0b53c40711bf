// Device-side definitions shared by the HWFV1 kernels (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "hwfv1.h"

namespace hw {

constexpr int kBlock = 256;             // workgroup size of most kernels
constexpr int kWave = 64;               // CDNA wavefront
constexpr uint32_t kNone = 0xffffffffu; // "no coarse leaf" marker
constexpr int kPartial = 10;            // doubles per FV1 partial record
constexpr int kMaxScen = 64;            // problems per batch
constexpr int kMaxFv1Grid = 8192;
constexpr int kLeafBatch = 2;           // leaves per FV1 thread per iteration
// Slots of hw_scalars.acc holding the step's snapshot of cur and done,
// taken by the light FV1 kernel for the copy-down.
constexpr int STEP_CUR = 4;
constexpr int STEP_DONE = 5;
// Slot of hw_scalars.acc holding the number of whole finest blocks at the
// head of the leaf list (written by every traversal, see block_list).
constexpr int STEP_NBLK = 0;

// Everything a kernel needs to know about one problem.  Lives in device
// memory (the workspace for single-problem calls, the plan for batches).
struct Desc {
    int32_t L, precision, bc[4];
    int32_t group_level;   // level of the traversal groups (max(L-2, 0))
    int32_t write_skip;    // FV1 may skip stores of unchanged dry blocks
    double eps, g, cfl, h_tol, dx, dy, dt_max, manning_n, rain_rate;
    double inlet_y0, inlet_y1, q_peak, t_peak, t_base, t_end;
    double zsmax;          // bed s_max given by the caller (0: from the grid)
    void* fine[2][3];
    void* coarse[3];
    double* zhier;
    uint8_t* zsig;
    uint8_t* raw;
    uint8_t* sig;
    uint32_t* leaves;
    hw_scalars* scal;
    uint32_t* tcount;      // traversal workgroup counts / offsets
    uint32_t* big_src;     // per group: leaf index of a coarser leaf or kNone
    uint8_t* lmap;         // per finest cell: level of the leaf containing it
    uint8_t* gcode;        // per traversal group: walk summary (count pass)
    uint8_t* rsig;         // per regularisation workgroup: every flag it
                           // wrote this step is set
    uint8_t* wet;          // FV1 wet table: 4 bytes per super-chunk
    uint64_t* hist;        // FV1 write history: one entry per 64 finest cells
    uint8_t* dryb;         // per 64 finest cells: the dry case holds for all
                           // of them (written by the first encoding pass)
    double* bpart;         // per 64 finest cells: mass and max |h| (pairs)
    double* partials;      // FV1 / ingest partial records, kPartial each
    uint32_t ntrav;        // traversal workgroups of this problem
    uint32_t nhist;        // entries of hist
    uint32_t nreg;         // regularisation workgroups (records in rsig)
    int32_t full_outputs;  // write every output (the entry points) or only
                           // what the time loop reads (plans): coarse level
                           // L-1, and the leaf list, leaf-level map and fill
                           // table of a step whose leaves are all finest
    int32_t uniform;       // uniform FV1 plan: every finest cell is a leaf,
                           // no encoding, flags or traversal run
    int32_t encode_skip;   // the first encoding pass may load one cell per
                           // wave span below a coarser leaf (plans only)
    int32_t fill_skip;     // the copy-down may leave spans below a coarser
                           // leaf incomplete (plans only, with encode_skip)
    int32_t block_list;    // block-first leaf list (plans only): 0 never,
                           // 1 when whole blocks hold at least 2^19 leaves,
                           // 2 whenever there is one
};

// Tree-sparse finest set (plans, L >= 7).  A span is an aligned run of 1024
// finest cells (one level L-5 cell; 64 traversal groups of 16 cells, one
// wave of the traversal and of the copy-down).  When one leaf at level
// <= L-5 covers a span, the copy-down writes only its groups 0, 16, 32 and
// 48 (the cells the first encoding pass reads there, for either tile); the
// other cells keep older values, and the first encoding pass stores only
// the span's level L-5 value (levels L-4 .. L-2 keep older values too).
// Such a stale span, with those coarse levels, is made whole again from its
// first cell when the next tree no longer covers it (traversal emit pass);
// its finest cells also at the end of every run call (k_densify), so
// outside a run the current set is complete.
__host__ __device__ inline bool sparse_fine(const Desc& d)
{
    return d.fill_skip && d.encode_skip && !d.full_outputs && !d.uniform && d.L >= 7;
}

// Block-first leaf list (plans, L >= 3).  The leaves of every aligned
// 8 x 8 block of finest cells that are all leaves (a level L-3 cell whose
// four traversal groups each hold sixteen finest leaves) come first, block
// by block in ascending Morton order, each block's cells in Morton order;
// the other leaves follow in depth-first order (Algorithm 2).  One wave of
// the FV1 kernels then takes one whole block (the list's waves are aligned
// to 64 entries).  The traversal's scan takes this layout when whole blocks
// hold enough leaves (Desc.block_list), else the depth-first one; the
// entry points keep the depth-first order throughout (their block count is
// 0).
__host__ __device__ inline bool block_list(const Desc& d)
{
    return d.block_list && !d.full_outputs && !d.uniform && d.L >= 3;
}

// Work decomposition of one launch: problem s owns workgroups
// [prefix[s], prefix[s+1]).  prefix == nullptr means one problem that owns
// every workgroup.
struct Launch {
    const Desc* descs;
    const uint32_t* prefix;
    int32_t n;
};

__host__ __device__ inline uint64_t level_off(int n)
{
    return ((uint64_t(1) << (2 * n)) - 1) / 3;
}

__host__ __device__ inline uint32_t part1by1(uint32_t x)
{
    x &= 0x0000ffffu;
    x = (x | (x << 8)) & 0x00ff00ffu;
    x = (x | (x << 4)) & 0x0f0f0f0fu;
    x = (x | (x << 2)) & 0x33333333u;
    x = (x | (x << 1)) & 0x55555555u;
    return x;
}

__host__ __device__ inline uint32_t compact1by1(uint32_t x)
{
    x &= 0x55555555u;
    x = (x | (x >> 1)) & 0x33333333u;
    x = (x | (x >> 2)) & 0x0f0f0f0fu;
    x = (x | (x >> 4)) & 0x00ff00ffu;
    x = (x | (x >> 8)) & 0x0000ffffu;
    return x;
}

__host__ __device__ inline uint32_t morton(uint32_t i, uint32_t j)
{
    return part1by1(i) | (part1by1(j) << 1);
}

// Morton neighbours on a level whose codes use the bits in
// xm (column bits) and ym = xm << 1 (row bits): increment or decrement one
// coordinate and carry through its own bits only.
__host__ __device__ inline uint32_t morton_xp(uint32_t c, uint32_t xm, uint32_t ym)
{
    return (((c | ym) + 1u) & xm) | (c & ym);
}
__host__ __device__ inline uint32_t morton_xm(uint32_t c, uint32_t xm, uint32_t ym)
{
    return (((c & xm) - 1u) & xm) | (c & ym);
}
__host__ __device__ inline uint32_t morton_yp(uint32_t c, uint32_t xm, uint32_t ym)
{
    return (((c | xm) + 1u) & ym) | (c & xm);
}
__host__ __device__ inline uint32_t morton_ym(uint32_t c, uint32_t xm, uint32_t ym)
{
    return (((c & ym) - 1u) & ym) | (c & xm);
}

// True on every lane if the condition holds on at least one lane of the wave.
__device__ inline bool wave_any(bool b) { return __ballot(b) != 0; }

// Level of a hierarchy Z-order index: the n with (4^n-1)/3 <= idx <
// (4^(n+1)-1)/3, i.e. floor(log4(3 idx + 1)).
__device__ inline int level_of(uint32_t idx)
{
    return (31 - __clz(3u * idx + 1u)) >> 1;
}

// Global-address-space view of a pointer: loads and stores through it are
// global (not flat) instructions, with the base in SGPRs when uniform.
template <typename T>
using gp = T __attribute__((address_space(1)))*;

// Load at a 32-bit byte offset from a (uniform) base: lets the compiler use
// the scalar-base + 32-bit vector-offset addressing form instead of a 64-bit
// address per lane.  Every array indexed this way is below 4 GiB.
template <typename T>
__device__ inline T ld_off(gp<const T> base, uint32_t byte_off)
{
    return *reinterpret_cast<gp<const T>>(reinterpret_cast<gp<const char>>(base) + byte_off);
}

// Native vector types (usable through global pointers).
typedef double vd2 __attribute__((ext_vector_type(2)));
typedef float vf4 __attribute__((ext_vector_type(4)));
typedef uint32_t vu4 __attribute__((ext_vector_type(4)));

template <typename T>
__device__ inline gp<T> glob(T* p)
{
    return (gp<T>)p;
}

// Make a value the compiler cannot prove wave-uniform, but that is, live in
// an SGPR (so descriptor reads through it become scalar loads).
__device__ inline int uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ inline uint32_t uniform(uint32_t v)
{
    return (uint32_t)__builtin_amdgcn_readfirstlane((int)v);
}

// Problem of workgroup b and the workgroup's index inside that problem
// (both uniform over the workgroup).
__device__ inline int scen_of(const Launch& l, uint32_t b, uint32_t& local)
{
    if (!l.prefix) {
        local = b;
        return 0;
    }
    int lo = 0, hi = l.n - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (l.prefix[mid] <= b) lo = mid;
        else hi = mid - 1;
    }
    lo = uniform(lo);
    local = uniform(b - l.prefix[lo]);
    return lo;
}

// ---- reductions ---------------------------------------------------------
template <typename V>
__device__ inline V wave_sum(V v)
{
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

template <typename V>
__device__ inline V wave_max(V v)
{
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) {
        V w = __shfl_xor(v, o);
        v = w > v ? w : v;
    }
    return v;
}

// Inclusive prefix sum over a wave.
__device__ inline uint32_t wave_incl_scan(uint32_t v)
{
    const int lane = threadIdx.x & (kWave - 1);
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
        uint32_t w = __shfl_up(v, o);
        if (lane >= o) v += w;
    }
    return v;
}

// Exclusive prefix over a workgroup of blockDim.x threads (multiple of 64,
// at most 1024); returns the exclusive prefix and the workgroup total.
__device__ inline uint32_t block_excl_scan(uint32_t v, uint32_t* lds,
                                           uint32_t& total)
{
    const int lane = threadIdx.x & (kWave - 1);
    const int wid = threadIdx.x / kWave;
    const int nw = blockDim.x / kWave;
    uint32_t inc = wave_incl_scan(v);
    if (lane == kWave - 1) lds[wid] = inc;
    __syncthreads();
    if (wid == 0) {
        uint32_t w = lane < nw ? lds[lane] : 0u;
        uint32_t wi = wave_incl_scan(w);
        if (lane < nw) lds[lane] = wi - w;
        if (lane == nw - 1) lds[16] = wi;
    }
    __syncthreads();
    uint32_t excl = inc - v + lds[wid];
    total = lds[16];
    __syncthreads();
    return excl;
}

// block_excl_scan on 64-bit values (lds: 17 entries).
__device__ inline uint64_t block_excl_scan64(uint64_t v, uint64_t* lds, uint64_t& total)
{
    const int lane = threadIdx.x & (kWave - 1);
    const int wid = threadIdx.x / kWave;
    const int nw = blockDim.x / kWave;
    uint64_t inc = v;
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
        const uint64_t w = __shfl_up(inc, o);
        if (lane >= o) inc += w;
    }
    if (lane == kWave - 1) lds[wid] = inc;
    __syncthreads();
    if (wid == 0) {
        const uint64_t w = lane < nw ? lds[lane] : 0ull;
        uint64_t wi = w;
#pragma unroll
        for (int o = 1; o < kWave; o <<= 1) {
            const uint64_t y = __shfl_up(wi, o);
            if (lane >= o) wi += y;
        }
        if (lane < nw) lds[lane] = wi - w;
        if (lane == nw - 1) lds[16] = wi;
    }
    __syncthreads();
    const uint64_t excl = inc - v + lds[wid];
    total = lds[16];
    __syncthreads();
    return excl;
}

}  // namespace hw
