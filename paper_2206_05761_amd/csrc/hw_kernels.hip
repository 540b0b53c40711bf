// HWFV1 timestep kernels for gfx950 (CDNA4, wave64).
//
// Phases of one timestep (Algorithm 3):
//   k_encode      Haar encoding (Eq. 3a-3d, Algorithm 1) of h, qx, qy over a
//                 Morton tile, several levels per pass, fused with the FP64
//                 significance test; the bed uses the same kernel at ingest.
//   k_regularise  refine the face neighbours of significant cells.
//   k_traverse    per-group walk down the significance tree (Algorithm 5) and
//                 ordered compaction of the leaves (count, scan, emit).
//   k_fv1_light   FV1, every leaf's dry test: groups of 64 leaves that are
//                 dry with dry neighbours are finished there ((h, 0, 0)), the
//                 others marked for the heavy kernel.
//   k_fv1_heavy   FV1 update of the marked leaves with same-level neighbours
//                 (Fig. 3), an 8 x 8 block of finest leaves per wave when all
//                 leaves are finest; both write back to the finest
//                 descendants and leave partial reductions.
//   k_fill_finalize  copy-down of leaves coarser than a traversal group, and
//                 in the same launch t += dt, CFL timestep, s_max, mass
//                 (minimum reduction of Section 2.2.3), flip of the finest
//                 buffer set (k_finalize alone for uniform FV1 plans).
//
// The encoding and the significance test perform, compiled without
// contraction, the same IEEE operations in the same order as the method's
// definition (their FP64 results are bit-identical to it).  The FV1 update
// takes one Newton-refined reciprocal where the definition divides several
// times by the same quantity, a Newton inverse cube root for the friction
// term, and fused multiply-adds at fixed places (written out, so that the
// per-leaf and the block update round alike), so it differs from it by
// rounding only.
#include "hw_device.h"

#include <math.h>
#include <type_traits>

namespace hw {

// ---------------------------------------------------------------------------
// small helpers
// ---------------------------------------------------------------------------

__global__ void k_set_desc(Desc d, Desc* dst)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) *dst = d;
}

struct Haar {
    double s, da, db, dg;
};

// Eq. 3a-3d with orthonormal Haar taps and the averaging factor 1/2: every
// tap product is +-1/2, so each coefficient is a quarter of a sum or a
// difference of the column pairs (s0 + s2), (s1 + s3), (s0 - s2), (s1 - s3).
__device__ inline Haar haar(double c0, double c1, double c2, double c3)
{
    double a = c0 + c2;
    double b = c1 + c3;
    double ad = c0 - c2;
    double bd = c1 - c3;
    Haar h;
    h.s = 0.25 * (a + b);
    h.da = 0.25 * (ad + bd);
    h.db = 0.25 * (a - b);
    h.dg = 0.25 * (ad - bd);
    return h;
}

// Algorithm 1 significance test, in FP64: max |detail| / s_max >= 2^(n-L) eps.
__device__ inline bool significant(const Haar& h, double smax, double thr)
{
    double a = fabs(h.da);
    double b = fabs(h.db);
    double g = fabs(h.dg);
    double m = a > b ? a : b;
    m = m > g ? m : g;
    return (m / smax) >= thr;
}

__device__ inline void load4(gp<const double> p, double o[4])
{
    const vd2 a = *reinterpret_cast<gp<const vd2>>(p);
    const vd2 b = *reinterpret_cast<gp<const vd2>>(p + 2);
    o[0] = a.x;
    o[1] = a.y;
    o[2] = b.x;
    o[3] = b.y;
}

__device__ inline void load4(gp<const float> p, double o[4])
{
    const vf4 a = *reinterpret_cast<gp<const vf4>>(p);
    o[0] = a.x;
    o[1] = a.y;
    o[2] = a.z;
    o[3] = a.w;
}

// The same with a non-temporal load (data read once per step: a wave of
// consecutive lanes covers 1 KB per instruction).
__device__ inline void load4_nt(gp<const float> p, double o[4])
{
    const vf4 a = __builtin_nontemporal_load(reinterpret_cast<gp<const vf4>>(p));
    o[0] = a.x;
    o[1] = a.y;
    o[2] = a.z;
    o[3] = a.w;
}
__device__ inline void load4_nt(gp<const double> p, double o[4]) { load4(p, o); }

// ---------------------------------------------------------------------------
// Encoding with fused significance flags
// ---------------------------------------------------------------------------
//
// A pass covers `tl` levels: the workgroup owns a tile of 4^lv cells of the
// input level n_in (lv = min(tl, n_in)) and produces levels n_in-1 .. n_in-lv.
// Each thread first reduces 4^cp consecutive input cells in registers (cp = 1
// or 2 levels); their values meet in LDS once, and the first wave produces
// the remaining levels (lane shuffles, no further barrier).  Pass 0 reads
// the finest level; pass k reads the coarse level written by pass k-1.
//
// FLOW: h, qx, qy of the current step (flags OR-ed with the static bed
// flags into raw); otherwise the bed (flags into zsig).

// Inflow rate of the west-edge hydrograph at time t (the FV1 kernels'
// inflow_rate, on a descriptor).
__device__ inline double inflow_rate_d(const Desc& d, double t)
{
    if (!(d.q_peak > 0.0)) return 0.0;
    if (t <= d.t_peak) return d.q_peak * t / d.t_peak;
    if (t <= d.t_base) return d.q_peak * (d.t_base - t) / (d.t_base - d.t_peak);
    return 0.0;
}

// Whether the inflow reaches the finest cell c (inflow_on for a finest
// leaf), given whether it flows at all now and the inlet (y0, y1) and cell
// height dy.
__device__ inline bool inflow_fine(bool flowing, double y0, double y1, double dy, int L,
                                   uint32_t c)
{
    const uint32_t lvmask = 0xffffffffu >> (32 - 2 * L);
    if (!flowing || (c & 0x55555555u & lvmask) != 0) return false;
    const double y_lo = (double)compact1by1(c >> 1) * dy;
    const double lo = y_lo > y0 ? y_lo : y0;
    const double yhi = y_lo + dy;
    const double hi = yhi < y1 ? yhi : y1;
    return hi - lo > 0.0;
}

// TILES > 1 (FP32 first pass over the flow variables, four cells per
// thread, single-problem launches): each workgroup encodes TILES adjacent
// tiles TILES b' .. TILES b' + TILES - 1, every thread one parent of each,
// with all child loads issued first, so a workgroup has TILES times the
// bytes in flight for the same serial chain; wave t then runs tile t's
// remaining levels.  Each tile's cells, flags and block records are
// computed exactly as in the one-tile form.
template <typename T, int NV, bool FLOW, bool DET, int CP, bool SKIP = false, int TILES = 1>
__global__ __launch_bounds__(kBlock) void k_encode(Launch lc, int pass,
                                                   int tl, double* details)
{
    uint32_t b;
    const int s = scen_of(lc, blockIdx.x, b);
    const Desc& d = lc.descs[s];
    constexpr bool TWO = TILES > 1;     // the multi-tile form
    constexpr int NT = TILES;           // tiles of this workgroup
    static_assert(NT >= 1 && NT <= 4, "one wave per tile's tail");
    const uint32_t b0 = (uint32_t)NT * b;
    // every scalar this workgroup needs, requested together (one round trip)
    const gp<const hw_scalars> sc = glob(static_cast<const hw_scalars*>(d.scal));
    const uint32_t done = sc->done;
    const int cur = uniform((int)sc->cur);
    double smax_all[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) smax_all[v] = sc->smax[v];
    const double t_now = sc->t;
    const uint64_t step = sc->step;
    const uint32_t map_step = sc->map_step;
    const uint64_t n_leaves = sc->n_leaves;
    // (span-skip form of the first pass) the leaf-level byte of the tile's
    // first cell, requested with the scalars; used only when the map
    // describes the previous tree (tile of 4^min(L, tl) cells, in bounds)
    uint32_t map0 = 255u;
    if (SKIP && FLOW && pass == 0 && d.encode_skip) {
        const int lv0 = d.L < tl ? d.L : tl;
        map0 = glob(static_cast<const uint8_t*>(d.lmap))[(uint64_t)b << (2 * lv0)];
    }
    if (FLOW && done) return;
    const int L = d.L;
    const int n_in = L - pass * tl;
    if (n_in <= 0) return;
    const int lv = n_in < tl ? n_in : tl;
    const int n_lo = n_in - lv;
    const int cp = CP < lv ? CP : lv;   // levels computed in registers
    const int tid = threadIdx.x;
    const uint64_t ncoarse = level_off(L);

    gp<const T> src[NV];
    gp<T> dstb[NV];
    double smax[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        if (FLOW) {
            src[v] = pass == 0
                         ? glob(reinterpret_cast<const T*>(d.fine[cur][v]))
                         : glob(reinterpret_cast<const T*>(d.coarse[v])) +
                               level_off(n_in);
            dstb[v] = glob(reinterpret_cast<T*>(d.coarse[v]));
            smax[v] = smax_all[v];
        } else {
            src[v] = glob(reinterpret_cast<const T*>(d.zhier)) + level_off(n_in);
            dstb[v] = glob(reinterpret_cast<T*>(d.zhier));
            smax[v] = smax_all[3];
        }
    }
    const gp<uint8_t> flags = glob(FLOW ? d.raw : d.zsig);
    const gp<const uint8_t> zsig = glob(static_cast<const uint8_t*>(d.zsig));
    const gp<double> det = glob(details);
    const double eps = d.eps;
    // Level L-1 of the flow variables is stored only when asked for (the
    // time loop reads it from the finest level instead, see parent_value).
    const bool keep_parents = d.full_outputs != 0;

    auto dst_of = [&](int v, int n) -> gp<T> { return dstb[v] + level_off(n); };

    // Encode one cell (n, k) from its four children, store it, flag it
    // (zb: the cell's static bed flag, read ahead of time).
    auto emit = [&](int n, uint64_t k, const double (*ch)[4], double* out, uint8_t zb) {
        const double thr = ldexp(eps, n - L);
        bool f = false;
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            Haar hh = haar(ch[v][0], ch[v][1], ch[v][2], ch[v][3]);
            T sv = (T)hh.s;
            if (!FLOW || n != L - 1 || keep_parents) dst_of(v, n)[k] = sv;
            out[v] = (double)sv;
            if (significant(hh, smax[v], thr)) f = true;
            if (DET) {
                const uint64_t o = level_off(n) + k;
                det[(uint64_t)(v * 3 + 0) * ncoarse + o] = hh.da;
                det[(uint64_t)(v * 3 + 1) * ncoarse + o] = hh.db;
                det[(uint64_t)(v * 3 + 2) * ncoarse + o] = hh.dg;
            }
        }
        const uint64_t o = level_off(n) + k;
        uint8_t fl = f ? 1 : 0;
        if (FLOW) fl |= zb;
        flags[o] = fl ? 1 : 0;
    };

    const int n_mid = n_in - cp;                  // level held per thread
    const uint32_t M = 1u << (2 * (lv - cp));     // active threads

    // Paired form of the first FP64 pass (four cells per thread, full
    // tiles): lane l of wave w loads, per variable, cells (2l, 2l+1) of the
    // wave's first 128 finest cells and of its second 128 with non-temporal
    // 16-byte loads, so that each load instruction of the wave covers 1 KB
    // once; even and odd lanes then swap one pair, and even lane 2j holds
    // the four children of the wave's level-(n_in-1) cell j, odd lane 2j+1
    // those of cell 32 + j.  pidx is the thread's level-(n_in-1) cell in the
    // tile (tid in the other forms).
    const uint32_t lane = (uint32_t)tid & (kWave - 1u);
    const uint32_t wid = (uint32_t)tid / kWave;
    const bool paired = FLOW && sizeof(T) == 8 && pass == 0 && (CP == 1 || cp == 1) &&
                        M == (uint32_t)kBlock;
    const uint32_t pidx = paired ? kWave * wid + ((lane & 1u) ? 32u : 0u) + (lane >> 1)
                                 : (uint32_t)tid;

    // The static bed flags of every cell this thread will emit, requested
    // together with the child values (one round trip instead of one per
    // level).  Tail level i is n_mid - 1 - i, with M >> 2(i+1) threads.
    constexpr int kTail = 6;
    uint8_t zr[4] = {0, 0, 0, 0}, zr2 = 0, zt[kTail];
    if (FLOW) {
        if ((uint32_t)tid < M) {
            const uint64_t o1 = level_off(n_in - 1) + ((uint64_t)b0 << (2 * (lv - 1)));
            if (TWO) {
#pragma unroll
                for (int t = 0; t < NT; ++t)
                    zr[t] = zsig[o1 + ((uint64_t)t << (2 * (lv - 1))) + pidx];
            } else if (CP == 1 || cp == 1) {
                zr[0] = zsig[o1 + pidx];
            } else {
#pragma unroll
                for (int qq = 0; qq < 4; ++qq) zr[qq] = zsig[o1 + 4ull * tid + qq];
                zr2 = zsig[level_off(n_in - 2) + ((uint64_t)b << (2 * (lv - 2))) + tid];
            }
        }
        // the tail of tile t runs on wave t (lane j: cell j of each level)
        const uint32_t tw = TWO ? (uint32_t)tid / kWave : 0u;
        const uint32_t tj = TWO ? (uint32_t)tid & (kWave - 1u) : (uint32_t)tid;
#pragma unroll
        for (int i = 0; i < kTail; ++i) {
            const int n = n_mid - 1 - i;
            const uint32_t c = M >> (2 * (i + 1));
            zt[i] = (n >= n_lo && tj < c && tw < (uint32_t)NT)
                        ? zsig[level_off(n) + (uint64_t)(b0 + tw) * c + tj]
                        : (uint8_t)0;
        }
    }

    // Block flags (first pass over the flow variables, L >= 5): for every
    // 64-cell (8x8) Morton block of the tile, bit 0 = some depth above h_tol
    // (or not a number), bit 1 = the inflow reaches one of its cells, bits
    // 2..5 = some depth above h_tol in its west column, east column, south
    // row, north row; and the block's mass and max |h|.  The FV1 step of a
    // problem whose leaves are all finest treats a block as dry exactly when
    // its bits 0 and 1 are clear and the edge of each neighbour block that
    // touches it is dry (that is every cell's dry test), and takes its mass
    // and max |h| from here instead of re-reading the depths.
    const bool blocks = FLOW && pass == 0 && L >= 5;
    const int cells = (CP == 1 || cp == 1) ? 4 : 16;    // finest cells per thread
    const int tpb = 64 / cells;                         // threads per block
    const T tolT = (T)d.h_tol;
    // everything the block test reads from the descriptor, read once
    const double area = d.dx * d.dy, cell_dy = d.dy;
    const double in_y0 = d.inlet_y0, in_y1 = d.inlet_y1;
    const bool flowing = blocks && d.q_peak > 0.0 && inflow_rate_d(d, t_now) != 0.0;
    const gp<uint8_t> dryb = glob(d.dryb);
    const gp<double> bpart = glob(d.bpart);
    auto block_test = [&](const double* hs) {
        const uint64_t first = ((uint64_t)b << (2 * lv)) + (uint64_t)cells * pidx;
        const uint32_t blk = (uint32_t)(first >> 6);
        const double tolD = (double)tolT;
        // this thread's square inside the block: side sq, corner (ti, tj)
        const int sq = cells == 4 ? 2 : 4;
        const uint32_t r = pidx % (uint32_t)tpb;
        const int ti = (int)compact1by1(r) * sq, tj = (int)compact1by1(r >> 1) * sq;
        bool wet = false, inflow = false, ww = false, we = false, ws = false, wn = false;
        double m = 0.0, hm = 0.0;
        for (int q = 0; q < cells; ++q) {
            const bool w = !(hs[q] <= tolD);
            const int ci = ti + (int)compact1by1((uint32_t)q);
            const int cj = tj + (int)compact1by1((uint32_t)q >> 1);
            wet = wet | w;
            ww = ww | (w & (ci == 0));
            we = we | (w & (ci == 7));
            ws = ws | (w & (cj == 0));
            wn = wn | (w & (cj == 7));
            inflow = inflow | inflow_fine(flowing, in_y0, in_y1, cell_dy, L, (uint32_t)(first + q));
            m += hs[q] * area;
            const double a = fabs(hs[q]);
            hm = a > hm ? a : hm;
        }
        // combine over the block's tpb lanes: an aligned run of consecutive
        // lanes, or in the paired form the lanes of one parity in one half
        // of the wave (stride 2)
        const int ln = tid & (kWave - 1);
        const uint64_t gmask =
            paired ? (((ln & 1) ? 0xAAAAAAAAull : 0x55555555ull) << (ln & 32))
                   : (tpb == 64 ? ~0ull : ((1ull << tpb) - 1ull)) << (ln & ~(tpb - 1));
        const bool bw = (__ballot(wet) & gmask) != 0ull;
        const bool bi = (__ballot(inflow) & gmask) != 0ull;
        const bool bww = (__ballot(ww) & gmask) != 0ull;
        const bool bwe = (__ballot(we) & gmask) != 0ull;
        const bool bws = (__ballot(ws) & gmask) != 0ull;
        const bool bwn = (__ballot(wn) & gmask) != 0ull;
        const int ostep = paired ? 2 : 1;
        for (int o = ostep; o < ostep * tpb; o <<= 1) {
            m += __shfl_xor(m, o);
            const double y = __shfl_xor(hm, o);
            hm = y > hm ? y : hm;
        }
        const bool leader = paired ? (ln & 30) == 0 : (ln & (tpb - 1)) == 0;
        if (leader) {
            dryb[blk] = (uint8_t)((bw ? 1 : 0) | (bi ? 2 : 0) | (bww ? 4 : 0) |
                                          (bwe ? 8 : 0) | (bws ? 16 : 0) | (bwn ? 32 : 0));
            gp<double> bp = bpart + 2ull * blk;
            bp[0] = m;
            bp[1] = hm;
        }
    };

    // Below a leaf of the previous step's tree every finest cell holds the
    // leaf's value (the copy-down of the FV1 update).  When the leaf-level
    // map still describes that tree (it was written in the step that made
    // the current set), a wave whose span of 64 * cells finest cells lies
    // inside one leaf loads the span's first `cells` cells on every lane:
    // the values are the same bits, so everything computed from them is
    // unchanged, and the span costs one or two cache lines per variable
    // instead of all its cells.
    const bool span_skip = SKIP && FLOW && pass == 0 && d.encode_skip && lv - cp >= 3 && step > 0 &&
                           map_step == (uint32_t)step && n_leaves < (1ull << (2 * L));
    // A whole tile inside one leaf (of level <= n_lo): every cell of every
    // level holds the leaf's value and every detail is 0, so each coarse
    // value is that value and each raw flag the static bed flag.  The
    // workgroup stores them (and its block records, from the same test)
    // without the Haar sums, the LDS meet or the first wave's tail.  With
    // the tree-sparse finest set it stores the values of the tile's top
    // level only (the next pass reads it): nothing in the step reads a level
    // below a leaf, and when the step's tree refines the tile, the
    // traversal's emit pass writes them (fill_span_coarse) before FV1 runs.
    if (SKIP && (CP == 1 || cp == 1) && span_skip && M == (uint32_t)kBlock) {
        const uint64_t tile_in = (uint64_t)b << (2 * lv);
        const bool tile_covered = uniform((int)map0) <= n_lo;
        if (tile_covered) {
            const bool top_only = sparse_fine(d);
            T val[NV];
#pragma unroll
            for (int v = 0; v < NV; ++v) val[v] = src[v][tile_in];
            if (blocks) {
                const double hv[4] = {(double)val[0], (double)val[0], (double)val[0],
                                      (double)val[0]};
                block_test(hv);
            }
            flags[level_off(n_in - 1) + ((uint64_t)b << (2 * (lv - 1))) + pidx] = zr[0] ? 1 : 0;
            uint32_t cnt = M;
#pragma unroll
            for (int i = 0; i < kTail; ++i) {
                const int n = n_mid - 1 - i;
                if (n < n_lo) break;
                cnt >>= 2;
                if ((uint32_t)tid < cnt) {
                    const uint64_t k = (uint64_t)b * cnt + tid;
                    if (!top_only || n == n_lo) {
#pragma unroll
                        for (int v = 0; v < NV; ++v) dst_of(v, n)[k] = val[v];
                    }
                    flags[level_off(n) + k] = zt[i] ? 1 : 0;
                }
            }
            return;
        }
    }
    double p[NV];
    __shared__ double lds[NT][NV][kBlock];
    if (TWO) {
        // every tile's children first, then each tile in turn (b names the
        // tile for the block test and the cell indices)
        // (the raw values are held, and widened or paired per tile)
        using RawT = typename std::conditional<sizeof(T) == 4, vf4, vd2>::type;
        constexpr int RW = sizeof(T) == 4 ? 1 : 2;   // raw vectors per variable
        RawT raw[NT][NV][RW];
#pragma unroll
        for (int t = 0; t < NT; ++t)
#pragma unroll
            for (int v = 0; v < NV; ++v) {
                const uint64_t tb = (uint64_t)(b0 + t) << (2 * lv);
                if (sizeof(T) == 4) {
                    raw[t][v][0] = __builtin_nontemporal_load(
                        reinterpret_cast<gp<const RawT>>(src[v] + tb + 4ull * tid));
                } else {
                    // the paired form: cells (2l, 2l+1) of the wave's first and
                    // second 128 finest cells
                    const gp<const RawT> q =
                        reinterpret_cast<gp<const RawT>>(src[v] + tb + 256ull * wid + 2ull * lane);
                    raw[t][v][0] = __builtin_nontemporal_load(q);
                    raw[t][v][RW - 1] = __builtin_nontemporal_load(q + 64);
                }
            }
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            b = b0 + (uint32_t)t;
            double cht[NV][4];
#pragma unroll
            for (int v = 0; v < NV; ++v) {
                if constexpr (sizeof(T) == 4) {
                    cht[v][0] = (double)raw[t][v][0].x;
                    cht[v][1] = (double)raw[t][v][0].y;
                    cht[v][2] = (double)raw[t][v][0].z;
                    cht[v][3] = (double)raw[t][v][0].w;
                } else {
                    const RawT x0 = raw[t][v][0], x1 = raw[t][v][RW - 1];
                    const bool odd = (lane & 1u) != 0u;
                    const RawT give = odd ? x0 : x1;
                    RawT got;
                    got.x = __shfl_xor(give.x, 1);
                    got.y = __shfl_xor(give.y, 1);
                    cht[v][0] = odd ? got.x : x0.x;
                    cht[v][1] = odd ? got.y : x0.y;
                    cht[v][2] = odd ? x1.x : got.x;
                    cht[v][3] = odd ? x1.y : got.y;
                }
            }
            if (blocks) block_test(cht[0]);
            double pt[NV];
            emit(n_in - 1, ((uint64_t)b << (2 * (lv - 1))) + pidx, cht, pt, zr[t]);
#pragma unroll
            for (int v = 0; v < NV; ++v) lds[t][v][pidx] = pt[v];
        }
    } else if ((uint32_t)tid < M) {
        const uint64_t tile_in = (uint64_t)b << (2 * lv);
        // wave-uniform: the span's first cell, and whether the span is covered
        uint64_t wf = 0;
        bool covered = false;
        if (span_skip) {
            wf = tile_in + (uint64_t)cells * uniform((uint32_t)(tid & ~(kWave - 1)));
            const int span_level = L - (cells == 4 ? 4 : 5);
            covered = uniform((int)glob(static_cast<const uint8_t*>(d.lmap))[wf]) <= span_level;
        }
        // All child loads are issued before any store of this thread.  The
        // two load forms sit in separate wave-uniform branches so that the
        // usual one keeps its base-plus-lane-offset addressing.
        if (CP == 1 || cp == 1) {
            double ch[NV][4];
            auto load_children = [&](uint64_t base) {
#pragma unroll
                for (int v = 0; v < NV; ++v) {
                    if (FLOW && pass == 0) load4(src[v] + base, ch[v]);
                    else
#pragma unroll
                        for (int q = 0; q < 4; ++q) ch[v][q] = (double)src[v][base + q];
                }
            };
            if (covered) {
                load_children(wf);   // the same cells on every lane
            } else if (paired) {
                const uint64_t wb = tile_in + 256ull * wid + 2ull * lane;
#pragma unroll
                for (int v = 0; v < NV; ++v) {
                    const gp<const vd2> q = reinterpret_cast<gp<const vd2>>(src[v] + wb);
                    const vd2 x0 = __builtin_nontemporal_load(q);
                    const vd2 x1 = __builtin_nontemporal_load(q + 64);
                    const bool odd = (lane & 1u) != 0u;
                    const vd2 give = odd ? x0 : x1;
                    vd2 got;
                    got.x = __shfl_xor(give.x, 1);
                    got.y = __shfl_xor(give.y, 1);
                    ch[v][0] = odd ? got.x : x0.x;
                    ch[v][1] = odd ? got.y : x0.y;
                    ch[v][2] = odd ? x1.x : got.x;
                    ch[v][3] = odd ? x1.y : got.y;
                }
            } else if (FLOW && pass == 0 && sizeof(T) == 4) {
#pragma unroll
                for (int v = 0; v < NV; ++v) load4_nt(src[v] + tile_in + 4ull * tid, ch[v]);
            } else {
                load_children(tile_in + 4ull * tid);
            }
            if (blocks) block_test(ch[0]);
            emit(n_in - 1, ((uint64_t)b << (2 * (lv - 1))) + pidx, ch, p, zr[0]);
        } else {
            double ch[4][NV][4];
            auto load_children = [&](uint64_t base) {
#pragma unroll
                for (int qq = 0; qq < 4; ++qq)
#pragma unroll
                    for (int v = 0; v < NV; ++v) {
                        if (FLOW && pass == 0) load4(src[v] + base + 4 * qq, ch[qq][v]);
                        else
#pragma unroll
                            for (int q = 0; q < 4; ++q)
                                ch[qq][v][q] = (double)src[v][base + 4 * qq + q];
                    }
            };
            if (covered) load_children(wf);
            else load_children(tile_in + 16ull * tid);
            if (blocks) {
                double hs[16];
#pragma unroll
                for (int qq = 0; qq < 4; ++qq)
#pragma unroll
                    for (int q = 0; q < 4; ++q) hs[4 * qq + q] = ch[qq][0][q];
                block_test(hs);
            }
            double mid[NV][4];
#pragma unroll
            for (int qq = 0; qq < 4; ++qq) {
                double o[NV];
                emit(n_in - 1, ((uint64_t)b << (2 * (lv - 1))) + 4ull * tid + qq,
                     ch[qq], o, zr[qq]);
#pragma unroll
                for (int v = 0; v < NV; ++v) mid[v][qq] = o[v];
            }
            emit(n_in - 2, ((uint64_t)b << (2 * (lv - 2))) + tid, mid, p, zr2);
        }
    }

    // Remaining levels of the tile: every thread's value goes to LDS once,
    // then the first wave alone carries on (the other waves are done): lane
    // j takes the children of cell j of the next level from LDS, and each
    // further level gathers its four children from lanes 4j..4j+3.
    if (!TWO && (uint32_t)tid < M) {
#pragma unroll
        for (int v = 0; v < NV; ++v) lds[0][v][pidx] = p[v];
    }
    __syncthreads();
    // wave t finishes tile t
    const int tw = tid / kWave;
    if (tw >= NT) return;
    const int tj = tid & (kWave - 1);
    b = b0 + (uint32_t)tw;
    uint32_t cnt = M;
#pragma unroll
    for (int i = 0; i < kTail; ++i) {
        const int n = n_mid - 1 - i;
        if (n < n_lo) break;
        cnt >>= 2;
        double ch[NV][4];
#pragma unroll
        for (int v = 0; v < NV; ++v)
#pragma unroll
            for (int q = 0; q < 4; ++q)
                ch[v][q] = i == 0 ? lds[tw][v][(4 * tj + q) & (kBlock - 1)]
                                  : __shfl(p[v], (4 * tj + q) & (kWave - 1));
        if ((uint32_t)tj < cnt) emit(n, (uint64_t)b * cnt + tj, ch, p, zt[i]);
    }
}

// Significance test alone (for the standalone flag entry point): details of
// every coarse cell recomputed from its stored children.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_flag_only(Launch lc)
{
    uint32_t b;
    const int s = scen_of(lc, blockIdx.x, b);
    const Desc& d = lc.descs[s];
    const hw_scalars* sc = d.scal;
    if (sc->done) return;
    const int L = d.L;
    const uint64_t c = (uint64_t)b * kBlock + threadIdx.x;
    if (c >= level_off(L)) return;
    const int n = level_of((uint32_t)c);
    const uint64_t k = c - level_off(n);
    const double thr = ldexp(d.eps, n - L);
    bool f = false;
    for (int v = 0; v < 3; ++v) {
        const T* ch = n + 1 == L
                          ? reinterpret_cast<const T*>(d.fine[sc->cur][v])
                          : reinterpret_cast<const T*>(d.coarse[v]) +
                                level_off(n + 1);
        Haar hh = haar((double)ch[4 * k], (double)ch[4 * k + 1],
                       (double)ch[4 * k + 2], (double)ch[4 * k + 3]);
        if (significant(hh, sc->smax[v], thr)) f = true;
    }
    uint8_t fl = (f ? 1 : 0) | d.zsig[c];
    d.raw[c] = fl ? 1 : 0;
}

// A time-loop step (not the entry points) in which every coarse cell is
// significant after regularisation has every finest cell as a leaf: every
// walk reaches the finest level, so the traversal's count pass has nothing
// to add (the emit pass and the FV1 kernels take the case from n_leaves =
// 4^L).  Each regularisation workgroup records whether every flag it wrote
// is set (rsig, one byte each); a workgroup of the count pass or the scan
// reads all the records (a few KB) and decides.  Not when the current set has spans the previous tree left
// stale: the emit pass then completes them from the count pass's walk
// codes.  Must be reached by the whole workgroup.
__device__ inline bool all_significant_step(const Desc& d, uint32_t* lds)
{
    const hw_scalars* sc = d.scal;
    if (d.full_outputs) return false;
    const bool stale = sparse_fine(d) && sc->step > 0 && sc->map_step == (uint32_t)sc->step;
    if (stale) return false;
    if (!d.rsig) return false;
    // records read as words (the region is 256-byte aligned); the last
    // word's bytes past nreg are masked off
    const gp<const uint32_t> r = reinterpret_cast<gp<const uint32_t>>(glob(d.rsig));
    const uint32_t words = (d.nreg + 3u) / 4u;
    bool zero = false;
    for (uint32_t i = threadIdx.x; i < words; i += blockDim.x) {
        const uint32_t nb = d.nreg - 4u * i;
        const uint32_t m = nb >= 4u ? 0xffffffffu : (1u << (8u * nb)) - 1u;
        zero |= (r[i] & m) != (0x01010101u & m);
    }
    const bool wz = __ballot(zero) != 0ull;
    if ((threadIdx.x & (kWave - 1)) == 0) lds[threadIdx.x / kWave] = wz ? 1u : 0u;
    __syncthreads();
    uint32_t any = 0;
    for (uint32_t w = 0; w < blockDim.x / kWave; ++w) any |= lds[w];
    __syncthreads();
    return any == 0u;
}

// The four cells of regularisation block t (levels 1..L-1); returns whether
// all four are significant.
__device__ inline bool regularise_block(uint32_t t, gp<const uint8_t> raw, gp<uint8_t> sig)
{
    const int n = level_of(t) + 1;
    const uint32_t q = t - (uint32_t)level_off(n - 1);
    // blocks live on level n-1: codes use 2(n-1) bits
    const uint32_t bm = n > 1 ? (0xffffffffu >> (32 - 2 * (n - 1))) : 0u;
    const uint32_t xm = 0x55555555u & bm, ym = 0xaaaaaaaau & bm;
    const uint64_t base = level_off(n);
    const uint64_t o = base + 4ull * q;
    const uint8_t r0 = raw[o], r1 = raw[o + 1], r2 = raw[o + 2], r3 = raw[o + 3];
    uint8_t w1 = 0, w3 = 0, e0 = 0, e2 = 0, s2 = 0, s3 = 0, n0 = 0, n1 = 0;
    if ((q & xm) != 0) {
        const uint64_t ow = base + 4ull * morton_xm(q, xm, ym);
        w1 = raw[ow + 1];
        w3 = raw[ow + 3];
    }
    if ((q & xm) != xm) {
        const uint64_t oe = base + 4ull * morton_xp(q, xm, ym);
        e0 = raw[oe];
        e2 = raw[oe + 2];
    }
    if ((q & ym) != 0) {
        const uint64_t os = base + 4ull * morton_ym(q, xm, ym);
        s2 = raw[os + 2];
        s3 = raw[os + 3];
    }
    if ((q & ym) != ym) {
        const uint64_t on = base + 4ull * morton_yp(q, xm, ym);
        n0 = raw[on];
        n1 = raw[on + 1];
    }
    // children 0 (SW), 1 (SE), 2 (NW), 3 (NE) of the block
    const uint8_t g0 = (r0 | r1 | r2 | w1 | s2) ? 1 : 0;
    const uint8_t g1 = (r1 | r0 | r3 | e0 | s3) ? 1 : 0;
    const uint8_t g2 = (r2 | r3 | r0 | w3 | n0) ? 1 : 0;
    const uint8_t g3 = (r3 | r2 | r1 | e2 | n1) ? 1 : 0;
    sig[o] = g0;
    sig[o + 1] = g1;
    sig[o + 2] = g2;
    sig[o + 3] = g3;
    return (g0 & g1 & g2 & g3) != 0;
}

// The last encoding pass of a flow problem in its simplest form: levels
// n_top - 1 .. 0 from the stored level n_top (0 < n_top < L), one level at
// a time across the workgroup, with the encoder's own cell rule (children
// in Morton order, the stored value rounded to T is the parent's child
// value, the threshold 2^(n-L) eps, the static bed flag or-ed in), so the
// results are the encoding pass's bit for bit.  Must be reached by the
// whole workgroup.
template <typename T>
__device__ inline void encode_top_levels(const Desc& d, int n_top)
{
    const gp<const hw_scalars> sc = glob(static_cast<const hw_scalars*>(d.scal));
    double smax[3];
#pragma unroll
    for (int v = 0; v < 3; ++v) smax[v] = sc->smax[v];
    const int L = d.L;
    const gp<uint8_t> flags = glob(d.raw);
    const gp<const uint8_t> zsig = glob(static_cast<const uint8_t*>(d.zsig));
    for (int n = n_top - 1; n >= 0; --n) {
        const uint32_t cnt = 1u << (2 * n);
        const double thr = ldexp(d.eps, n - L);
        for (uint32_t k = threadIdx.x; k < cnt; k += blockDim.x) {
            bool f = false;
#pragma unroll
            for (int v = 0; v < 3; ++v) {
                const gp<T> lev = glob(reinterpret_cast<T*>(d.coarse[v]));
                const gp<const T> ch = lev + level_off(n + 1) + 4ull * k;
                const Haar hh = haar((double)ch[0], (double)ch[1], (double)ch[2], (double)ch[3]);
                lev[level_off(n) + k] = (T)hh.s;
                if (significant(hh, smax[v], thr)) f = true;
            }
            const uint64_t o = level_off(n) + k;
            flags[o] = (f || zsig[o]) ? 1 : 0;
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// Regularisation: sig = raw of the cell or of any in-domain face neighbour
// on the same level.
// ---------------------------------------------------------------------------
// fold_pass >= 0 (plans, five levels per encoding pass): that last encoding
// pass (one workgroup, levels <= 4) is not launched; the problem's first
// workgroup here runs it first, since only its own blocks (levels 1..4)
// read those flags.
__global__ __launch_bounds__(kBlock) void k_regularise(Launch lc, int fold_pass, int tl)
{
    uint32_t b;
    const int s = scen_of(lc, blockIdx.x, b);
    const Desc& d = lc.descs[s];
    if (d.scal->done) return;
    const int L = d.L;
    if (fold_pass >= 0 && b == 0) {
        const int n_top = L - fold_pass * tl;
        if (n_top > 0) {
            if (d.precision == HW_FP64) encode_top_levels<double>(d, n_top);
            else encode_top_levels<float>(d, n_top);
        }
    }
    const gp<const uint8_t> raw = glob(static_cast<const uint8_t*>(d.raw));
    const gp<uint8_t> sig = glob(d.sig);
    // One thread per 2x2 Morton block of cells on levels 1..L-1; block t
    // of the whole index space [0, (4^(L-1)-1)/3) sits on level
    // n = level_of(t) + 1 with block code q.  Thread 0 also does level 0,
    // which has no neighbours.
    const uint32_t t = b * kBlock + threadIdx.x;
    bool zero = false;
    if (t == 0) {
        sig[0] = raw[0] ? 1 : 0;
        zero = raw[0] == 0;
    }
    if (L >= 2 && t < (uint32_t)level_off(L - 1)) zero |= !regularise_block(t, raw, sig);
    // this workgroup's record: every flag it wrote is set
    const bool wz = __ballot(zero) != 0ull;
    __shared__ uint32_t vote[kBlock / kWave];
    if ((threadIdx.x & (kWave - 1)) == 0) vote[threadIdx.x / kWave] = wz ? 1u : 0u;
    __syncthreads();
    if (threadIdx.x == 0)
        glob(d.rsig)[b] = (vote[0] | vote[1] | vote[2] | vote[3]) ? 0 : 1;
}

// ---------------------------------------------------------------------------
// Traversal and ordered compaction
// ---------------------------------------------------------------------------
//
// A thread owns one group cell g on level Lg = max(L-2, 0), i.e. the 4^(L-Lg)
// finest cells below it.  It walks from the root towards g (Algorithm 5);
// if it stops above Lg at a coarser leaf it emits that leaf only when g holds
// the leaf's first finest descendant (so each leaf is listed once), and
// records the leaf for the copy-down; otherwise it expands the at most two
// levels below g.  Leaves come out in ascending first-descendant order.

// Walk of group g from the root (Algorithm 5 for its 4^(L-Lg) finest
// cells), summarised in one byte: the level (< 15) where the path meets an
// insignificant cell, or 15 when g is significant, with the significance of
// g's four children in the high nibble.
__device__ inline uint32_t walk_code(const Desc& d, uint32_t g)
{
    const int L = d.L;
    const int Lg = d.group_level;
    const gp<const uint8_t> sig = glob(static_cast<const uint8_t*>(d.sig));
    // Flags of every cell on the root-to-g path (levels 0..Lg) and of the
    // four children of g, all loaded before any decision: the walk then
    // costs one memory round trip instead of one per level.
    uint8_t pf[HW_MAX_L];
#pragma unroll
    for (int n = 0; n < HW_MAX_L; ++n) {
        const int nn = n < Lg ? n : Lg;   // levels past Lg repeat Lg (in bounds)
        pf[n] = sig[level_off(nn) + (g >> (2 * (Lg - nn)))];
    }
    const int n1 = Lg + 1;
    const uint64_t kb = n1 < L ? level_off(n1) + 4ull * g : level_off(Lg) + g;
    uint8_t kf[4];
#pragma unroll
    for (int c1 = 0; c1 < 4; ++c1) kf[c1] = sig[n1 < L ? kb + c1 : kb];
    uint32_t path = 0;
#pragma unroll
    for (int n = 0; n < HW_MAX_L; ++n)
        if (n <= Lg && pf[n]) path |= 1u << n;
    const int n = __ffs(~path) - 1;   // first insignificant level on the path
    if (n <= Lg) return (uint32_t)n;
    uint32_t kids = 0;
    if (n1 < L) {
#pragma unroll
        for (int c1 = 0; c1 < 4; ++c1)
            if (kf[c1]) kids |= 1u << c1;
    }
    return 15u | (kids << 4);
}

// Leaves of group g from its walk code, in ascending first-descendant
// order.  A leaf coarser than the group is listed only by the group that
// holds its first finest descendant (so each leaf appears once) and is
// recorded in big for the copy-down; lvl receives the leaf level of each
// quarter of the group.
template <bool WRITE, typename P>
__device__ inline int group_leaves(const Desc& d, uint32_t g, uint32_t code,
                                   P out, uint32_t& big, uint32_t lvl[4])
{
    const int Lg = d.group_level;
    const int n1 = Lg + 1;
    int cnt = 0;
    big = kNone;
    const int n = (int)(code & 15u);
    if (n < Lg) {
        const uint32_t k = g >> (2 * (Lg - n));
        const uint32_t idx = (uint32_t)level_off(n) + k;
        big = idx;
        if ((g & ((1u << (2 * (Lg - n))) - 1u)) == 0) {
            if (WRITE) out[cnt] = idx;
            ++cnt;
        }
        lvl[0] = lvl[1] = lvl[2] = lvl[3] = (uint32_t)n;
        return cnt;
    }
    if (n == Lg) {
        if (WRITE) out[cnt] = (uint32_t)level_off(Lg) + g;
        lvl[0] = lvl[1] = lvl[2] = lvl[3] = (uint32_t)Lg;
        return cnt + 1;
    }
    const uint32_t kids = code >> 4;
    for (uint32_t c1 = 0; c1 < 4; ++c1) {
        const uint32_t k1 = 4 * g + c1;
        if (!((kids >> c1) & 1u)) {
            if (WRITE) out[cnt] = (uint32_t)level_off(n1) + k1;
            ++cnt;
            lvl[c1] = (uint32_t)n1;
        } else {
            for (uint32_t c2 = 0; c2 < 4; ++c2) {
                if (WRITE) out[cnt] = (uint32_t)level_off(n1 + 1) + 4 * k1 + c2;
                ++cnt;
            }
            lvl[c1] = (uint32_t)(n1 + 1);
        }
    }
    return cnt;
}

// Leaf levels of the finest cells of group g: 4^(L-Lg) bytes (16, or 4 when
// L = 1); within each quarter of the group the four values are equal.
__device__ inline void write_level_map(const Desc& d, uint32_t g, const uint32_t lvl[4])
{
    const int per = 1 << (2 * (d.L - d.group_level));
    if (per == 16) {
        const vu4 v = {lvl[0] * 0x01010101u, lvl[1] * 0x01010101u,
                       lvl[2] * 0x01010101u, lvl[3] * 0x01010101u};
        *reinterpret_cast<gp<vu4>>(glob(d.lmap) + 16ull * g) = v;
    } else {
        const uint32_t v = (lvl[0] & 0xffu) | ((lvl[1] & 0xffu) << 8) |
                           ((lvl[2] & 0xffu) << 16) | ((lvl[3] & 0xffu) << 24);
        *reinterpret_cast<gp<uint32_t>>(glob(d.lmap) + 4ull * g) = v;
    }
}

// cnt (1, or a multiple of 4) equal values from p on, with vector stores.
template <typename T>
__device__ inline void store_run(gp<T> p, uint32_t cnt, T v)
{
    if (cnt == 1) {
        p[0] = v;
        return;
    }
    if (sizeof(T) == 8) {
        const vd2 w = {(double)v, (double)v};
        for (uint32_t q = 0; q < cnt; q += 2) *reinterpret_cast<gp<vd2>>(p + q) = w;
    } else {
        const vf4 w = {(float)v, (float)v, (float)v, (float)v};
        for (uint32_t q = 0; q < cnt; q += 4) *reinterpret_cast<gp<vf4>>(p + q) = w;
    }
}

// One wave writes the first cell's value of every variable to all 1024
// cells of the span starting at first, in finest set cur.
template <typename T>
__device__ inline void fill_span(const Desc& d, int cur, uint64_t first)
{
    const uint32_t lane = threadIdx.x & (kWave - 1u);
#pragma unroll
    for (int v = 0; v < 3; ++v) {
        const gp<T> f = glob(reinterpret_cast<T*>(d.fine[cur][v]));
        const T val = f[first];
        store_run<T>(f + first + 16u * lane, 16u, val);
    }
}

// The coarse values of levels L-4 .. L-2 of the span starting at first
// (the first encoding pass wrote only its level L-5 while one leaf covered
// it): every one is the span's first finest value.  One wave.
template <typename T>
__device__ inline void fill_span_coarse(const Desc& d, int cur, uint64_t first)
{
    const uint32_t lane = threadIdx.x & (kWave - 1u);
    const int L = d.L;
#pragma unroll
    for (int v = 0; v < 3; ++v) {
        const T val = glob(reinterpret_cast<const T*>(d.fine[cur][v]))[first];
        const gp<T> c = glob(reinterpret_cast<T*>(d.coarse[v]));
#pragma unroll
        for (int j = 1; j <= 3; ++j) {
            const int n = L - 5 + j;
            if (lane < (1u << (2 * j)))
                c[level_off(n) + (first >> (2 * (L - n))) + lane] = val;
        }
    }
}

// Count pass (EMIT = false): walk, store the walk code of each group and
// the workgroup's leaf count.  Emit pass: rebuild the leaves from the codes,
// place them at the workgroup offset plus the in-workgroup prefix, and write
// the copy-down table and the leaf-level map.
template <bool EMIT>
__global__ __launch_bounds__(kBlock) void k_traverse(Launch lc)
{
    __shared__ uint32_t lds[32];
    uint32_t lb;
    const int s = scen_of(lc, blockIdx.x, lb);
    const Desc& d = lc.descs[s];
    // every scalar the exit tests read, requested together
    const gp<const hw_scalars> sc = glob(static_cast<const hw_scalars*>(d.scal));
    const uint32_t done = sc->done;
    const uint64_t n_leaves = sc->n_leaves, step = sc->step;
    const uint32_t map_step = sc->map_step, cur = sc->cur;
    if (done) return;
    if (!EMIT && all_significant_step(d, lds)) return;
    // Spans of the current set may be stale when the previous step's tree
    // covered them (the map still describes that tree: it was written in
    // the step that made the set).
    const bool stale = EMIT && sparse_fine(d) && step > 0 && map_step == (uint32_t)step;
    // In the time loop a step whose leaves are all finest needs no list,
    // map or fill table: the FV1 kernels take that case from n_leaves.
    if (EMIT && !d.full_outputs && n_leaves == (1ull << (2 * d.L)) && !stale) return;
    const uint32_t ngroups = 1u << (2 * d.group_level);
    const uint32_t g = lb * kBlock + threadIdx.x;
    const bool active = g < ngroups;
    const gp<uint8_t> codes = glob(d.gcode);
    uint32_t code = 0;
    if (active) {
        if (EMIT) {
            code = codes[g];
        } else {
            code = walk_code(d, g);
            codes[g] = (uint8_t)code;
        }
    }
    uint32_t big = kNone;
    uint32_t lvl[4];
    const uint32_t cnt =
        active ? (uint32_t)group_leaves<false>(d, g, code, (uint32_t*)nullptr, big, lvl) : 0u;
    // Block-first list: the four groups of an aligned finest block (lanes
    // 4k .. 4k+3 of one wave) whose codes all say "sixteen finest leaves"
    // are listed in the block region, the other groups' leaves after it.
    const bool blocks = block_list(d);
    const uint32_t lane = threadIdx.x & (kWave - 1u);
    bool full = false;
    if (blocks) {
        const uint64_t fm = __ballot(active && code == 0xFFu);
        full = ((fm >> (lane & ~3u)) & 0xFull) == 0xFull;
    }
    // one scan for both counts: the group's leaves outside whole blocks in
    // the low 16 bits (at most 4096 per workgroup), whole blocks (one per
    // block, at its first lane) above them
    uint32_t ptotal;
    const uint32_t pexcl = block_excl_scan(
        (full ? 0u : cnt) | ((full && (lane & 3u) == 0u) ? 0x10000u : 0u), lds, ptotal);
    const uint32_t excl = pexcl & 0xffffu, total = ptotal & 0xffffu;
    const uint32_t bexcl = pexcl >> 16, btotal = ptotal >> 16;
    if (!EMIT) {
        if (threadIdx.x == 0) {
            glob(d.tcount)[lb] = total;
            if (blocks) glob(d.tcount)[d.ntrav + 1u + lb] = btotal;
        }
        return;
    }
    // The workgroup's leaves are one contiguous run of the list: they are
    // staged in LDS at their in-workgroup offsets and then written with
    // consecutive lanes on consecutive entries.
    __shared__ uint32_t stage[kBlock * 16];
    // The scan chose the layout: block-first (nblk whole blocks head the
    // list) or, with nblk = 0, depth-first, where a group's leaves follow
    // the other leaves and the whole blocks before it in the workgroup
    // (bpos: the whole blocks before its block, from the block's first lane).
    const uint32_t bpos = (uint32_t)__shfl((int)bexcl, (int)(lane & ~3u));
    const uint32_t nblk =
        blocks ? (uint32_t)glob(static_cast<const hw_scalars*>(d.scal))->acc[STEP_NBLK] : 0u;
    const bool bfirst = nblk != 0u;
    if (active) {
        // the map byte of the wave's span as the previous tree left it; the
        // same lane overwrites it below, after this load
        const uint64_t span0 = (uint64_t)(g - (threadIdx.x & (kWave - 1u))) << 4;
        const int old = stale ? (int)glob(static_cast<const uint8_t*>(d.lmap))[span0] : 255;
        if (!(full && bfirst)) {
            const uint32_t at = bfirst ? excl : excl + 64u * bpos + (full ? 16u * (g & 3u) : 0u);
            group_leaves<true>(d, g, code, stage + at, big, lvl);
        }
        glob(d.big_src)[g] = big;
        // a span that lies inside one leaf of level <= L-5 in both trees,
        // at the same level, already holds its map bytes
        const int now = (int)uniform(lvl[0]);
        if (!(old == now && now <= d.L - 5)) write_level_map(d, g, lvl);
        // a stale span this tree refines is made whole before FV1 reads it
        if (old <= d.L - 5 && now > d.L - 5) {
            if (d.precision == HW_FP64) {
                fill_span<double>(d, (int)cur, span0);
                fill_span_coarse<double>(d, (int)cur, span0);
            } else {
                fill_span<float>(d, (int)cur, span0);
                fill_span_coarse<float>(d, (int)cur, span0);
            }
        }
    }
    // a standalone traversal replaces the tree the current set was made with
    if (d.full_outputs && lb == 0 && threadIdx.x == 0) glob(d.scal)->map_step = 0u;
    // block-first: each group of a whole block writes its sixteen finest
    // leaves at the block's place in the block region
    const uint32_t boff = blocks ? glob(d.tcount)[d.ntrav + 1u + lb] : 0u;
    if (bfirst && full) {
        const uint32_t at = 64u * (boff + bpos) + 16u * (g & 3u);
        const uint32_t f = (uint32_t)level_off(d.L) + 16u * g;
        const gp<vu4> o = reinterpret_cast<gp<vu4>>(glob(d.leaves) + at);
#pragma unroll
        for (uint32_t q = 0; q < 4; ++q)
            o[q] = vu4{f + 4u * q, f + 4u * q + 1u, f + 4u * q + 2u, f + 4u * q + 3u};
    }
    __syncthreads();
    const uint32_t n_out = bfirst ? total : total + 64u * btotal;
    const gp<uint32_t> out = glob(d.leaves) + glob(d.tcount)[lb] + 64u * (bfirst ? nblk : boff);
    for (uint32_t i = threadIdx.x; i < n_out; i += kBlock) out[i] = stage[i];
}

// Leaves in whole finest blocks from which a plan step lists them first
// (hw_tuning.block_list = 1; 2 lists any).
constexpr uint64_t kBlockListMin = 1ull << 19;

// Exclusive scan of the per-workgroup leaf counts of one problem (one
// workgroup per problem); the total is the leaf count of the step.
__global__ __launch_bounds__(1024) void k_trav_scan(const Desc* descs)
{
    __shared__ uint32_t lds[32];
    const Desc& d = descs[blockIdx.x];
    const uint32_t done = glob(d.scal)->done;
    if (!done && all_significant_step(d, lds)) {
        if (threadIdx.x == 0) {
            glob(d.scal)->n_leaves = 1ull << (2 * d.L);
            glob(d.scal)->acc[STEP_NBLK] = 0.0;
        }
        return;
    }
    const uint32_t n = d.ntrav;
    // With the block-first list (block_list) the counts of whole finest
    // blocks follow the leaf counts in tcount; both are scanned, and the
    // block total places the other leaves after the block region.
    const bool blocks = block_list(d);
    const gp<uint32_t> cnt = glob(d.tcount);
    const gp<uint32_t> bcnt = cnt + n + 1u;
    // four consecutive counts per thread and round, loaded together; both
    // counts in one 64-bit scan (leaves in the low word, blocks above)
    __shared__ uint64_t lds64[17];
    uint64_t carry = 0;
    for (uint32_t base = 0; base < n; base += 4 * blockDim.x) {
        const uint32_t i0 = base + 4 * threadIdx.x;
        uint64_t v[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            v[k] = i0 + k < n ? cnt[i0 + k] : 0u;
            if (blocks && i0 + k < n) v[k] |= (uint64_t)bcnt[i0 + k] << 32;
        }
        const uint64_t sum = (v[0] + v[1]) + (v[2] + v[3]);
        uint64_t total;
        uint64_t excl = carry + block_excl_scan64(sum, lds64, total);
        if (!done) {
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                if (i0 + k < n) {
                    cnt[i0 + k] = (uint32_t)excl;
                    if (blocks) bcnt[i0 + k] = (uint32_t)(excl >> 32);
                }
                excl += v[k];
            }
        }
        carry += total;
    }
    if (threadIdx.x == 0 && !done) {
        const uint64_t nblk = carry >> 32;
        glob(d.scal)->n_leaves = 64ull * nblk + (carry & 0xffffffffull);
        // the block-first layout only when whole blocks hold enough leaves
        // (with few, the FV1 kernels' chunks are few and each one a
        // workgroup's serial chain; the depth-first order, which spreads the
        // costly leaves over all chunks, is then faster)
        const uint64_t lo = d.block_list == 2 ? 1ull : kBlockListMin;
        glob(d.scal)->acc[STEP_NBLK] = 64ull * nblk >= lo ? (double)nblk : 0.0;
    }
}

// ---------------------------------------------------------------------------
// FV1 update on the leaves
// ---------------------------------------------------------------------------

template <typename T>
struct Cell {
    T h, qx, qy;
    double z;
};

// Everything the FV1 update of one problem reads, as global pointers and
// scalars; built once per problem (wave-uniform, so it lives in SGPRs).
template <typename T>
struct Fv1Ctx {
    gp<const T> fin[3];    // current finest set
    gp<T> fout[3];         // finest set being written
    gp<const T> crs[3];    // coarse levels
    gp<const double> zh;   // bed hierarchy
    gp<const uint8_t> lmap;
    gp<const uint32_t> leaves;
    gp<uint64_t> hist;     // write history (light kernel)
    gp<const uint8_t> dryb;   // dry blocks and their mass / max |h|
    gp<const double> bpart;
    uint64_t step;         // index of the step being taken
    int write_skip;        // stores of unchanged dry blocks may be skipped
    int uniform;           // uniform FV1 plan (no encoder block records)
    int L, Lg;
    int bc[4];
    double dx, dy, g, h_tol, manning_n, rain_rate;
    double inlet_y0, inlet_y1, q_peak, t_peak, t_base;
    double t, dt;
    uint32_t nl;
    uint32_t nb64;         // list entries of whole finest blocks at its head
    const double* rxy;     // LDS: dt/dx_m at [2m], dt/dy_m at [2m+1]
};

// dt / (cell size of level m) for every level, the same divisions the
// update performs, done once per problem by one thread into LDS.
__device__ inline void fill_rxy(double* rxy, const Desc& d, double dt)
{
    if (threadIdx.x == 0)
        for (int m = 0; m <= d.L; ++m) {
            rxy[2 * m] = dt / ldexp(d.dx, d.L - m);
            rxy[2 * m + 1] = dt / ldexp(d.dy, d.L - m);
        }
}

// Leaves of the step: the traversal's count, or every finest cell under a
// uniform FV1 plan.
__device__ inline uint64_t step_leaves(const Desc& d, const hw_scalars* sc)
{
    return d.uniform ? (1ull << (2 * d.L)) : sc->n_leaves;
}

template <typename T>
__device__ inline void make_ctx(Fv1Ctx<T>& x, const Desc& d)
{
    const hw_scalars* sc = d.scal;
    const int cur = uniform((int)sc->cur);
    for (int v = 0; v < 3; ++v) {
        x.fin[v] = glob(reinterpret_cast<const T*>(d.fine[cur][v]));
        x.fout[v] = glob(reinterpret_cast<T*>(d.fine[cur ^ 1][v]));
        x.crs[v] = glob(reinterpret_cast<const T*>(d.coarse[v]));
    }
    x.zh = glob(static_cast<const double*>(d.zhier));
    x.lmap = glob(static_cast<const uint8_t*>(d.lmap));
    x.leaves = glob(static_cast<const uint32_t*>(d.leaves));
    x.hist = glob(d.hist);
    x.dryb = glob(static_cast<const uint8_t*>(d.dryb));
    x.bpart = glob(static_cast<const double*>(d.bpart));
    x.step = sc->step;
    x.write_skip = d.write_skip;
    x.L = d.L;
    x.Lg = d.group_level;
    for (int k = 0; k < 4; ++k) x.bc[k] = d.bc[k];
    x.dx = d.dx;
    x.dy = d.dy;
    x.g = d.g;
    x.h_tol = d.h_tol;
    x.manning_n = d.manning_n;
    x.rain_rate = d.rain_rate;
    x.inlet_y0 = d.inlet_y0;
    x.inlet_y1 = d.inlet_y1;
    x.q_peak = d.q_peak;
    x.t_peak = d.t_peak;
    x.t_base = d.t_base;
    x.t = sc->t;
    x.dt = sc->dt;
    x.nl = uniform((uint32_t)step_leaves(d, sc));
    x.nb64 = block_list(d) ? uniform(64u * (uint32_t)sc->acc[STEP_NBLK]) : 0u;
    x.uniform = d.uniform;
}

// Value of the level-(L-1) cell k of one variable from its four finest
// children, with the encoder's operations in the encoder's order (Eq. 3a
// as in haar), so it equals the encoded value bit for bit.  The time loop
// does not store level L-1; every reader takes it from here.
template <typename T>
__device__ inline T parent_value(gp<const T> f, uint32_t k)
{
    double c[4];
    load4(f + 4ull * k, c);
    const double a = c[0] + c[2];
    const double b = c[1] + c[3];
    return (T)(0.25 * (a + b));
}

// One variable of the hierarchy cell (n, k): finest set, parent rule or
// coarse levels.
template <typename T>
__device__ inline T load_var(const Fv1Ctx<T>& x, int v, int n, uint32_t k)
{
    if (n == x.L) return x.fin[v][k];
    if (n == x.L - 1) return parent_value<T>(x.fin[v], k);
    return x.crs[v][level_off(n) + k];
}

template <typename T>
__device__ inline Cell<T> load_cell(const Fv1Ctx<T>& x, int n, uint32_t k)
{
    Cell<T> c;
    c.h = load_var<T>(x, 0, n, k);
    c.qx = load_var<T>(x, 1, n, k);
    c.qy = load_var<T>(x, 2, n, k);
    c.z = x.zh[level_off(n) + k];
    return c;
}

template <typename T>
__device__ inline T load_h(const Fv1Ctx<T>& x, int n, uint32_t k)
{
    return load_var<T>(x, 0, n, k);
}

// Same-level neighbour (Fig. 3) through the leaf-level map: the leaf that
// contains the first finest descendant of the level-m cell cd is at level lv.
// If lv >= m the level-m cell exists in the tree (it is that leaf or an
// internal node) and its encoded values are used; otherwise the coarser leaf
// at level lv contains it and is used.  Both follow the same root path, so
// this is the first-insignificant-ancestor rule.  The level-m values are
// loaded before lv is known (the slot always exists); only a coarser
// neighbour costs a second load.
template <typename T>
__device__ inline Cell<T> neighbour_fix(const Fv1Ctx<T>& x, int m, uint32_t cd,
                                        int lv, const Cell<T>& spec)
{
    if (lv >= m) return spec;
    return load_cell<T>(x, lv, cd >> (2 * (m - lv)));
}

template <typename T>
__device__ inline Cell<T> ghost_cell(const Fv1Ctx<T>& x, int dir, const Cell<T>& own)
{
    Cell<T> g = own;
    if (x.bc[dir] == HW_BC_WALL) {
        if (dir == HW_W || dir == HW_E) g.qx = -g.qx;
        else g.qy = -g.qy;
    }
    return g;
}

// Reciprocal of a finite x with 2^-1000 < |x| < 2^1000 (the FV1 update's
// wet depths, HLL speed differences and friction denominators): the
// hardware estimate refined by two Newton steps r += r (1 - x r), within
// about an ulp of the correctly rounded quotient, at a third of the
// instructions of the full division.  FP32: the hardware reciprocal (1 ulp).
__device__ inline double rcp_nr(double x)
{
    double r = __builtin_amdgcn_rcp(x);
    double e = fma(-x, r, 1.0);
    r = fma(r, e, r);
    e = fma(-x, r, 1.0);
    return fma(r, e, r);
}
__device__ inline float rcp_nr(float x) { return __builtin_amdgcn_rcpf(x); }

// Square root of a finite x >= 0 (the FV1 update's g h and squared
// speeds): the hardware reciprocal square root estimate y, one coupled
// Goldschmidt step on g = x y, h = y / 2, then two Newton corrections of g
// (Markstein's formulation), within about an ulp of the correctly rounded
// root; x = 0 gives 0 and a NaN stays NaN.  Estimates are taken at
// max(x, 2^-1000), so a root below 2^-500 is off by less than 2^-500.
// FP32: the hardware square root (1 ulp).
__device__ inline double sqrt_nr(double x)
{
    const double y = __builtin_amdgcn_rsq(fmax(x, 0x1p-1000));
    double gq = x * y;
    double hq = 0.5 * y;
    const double r = fma(-gq, hq, 0.5);
    gq = fma(gq, r, gq);
    hq = fma(hq, r, hq);
    double d = fma(-gq, gq, x);
    gq = fma(d, hq, gq);
    d = fma(-gq, gq, x);
    return fma(d, hq, gq);
}
__device__ inline float sqrt_nr(float x) { return __builtin_amdgcn_sqrtf(x); }

// x^(-1/3) for x > 0: a single-precision seed 2^(-log2(x) / 3) from the
// hardware logarithm and exponential, then Newton steps for y^-3 = x,
// y += y (1 - x y^3) / 3, each doubling the correct bits (two steps for
// FP64, one for FP32); outside 1e-30 < x < 1e30, where the seed could
// under- or overflow, 1 / cbrt(x).
__device__ inline double inv_cbrt(double x)
{
    if (!(x > 1e-30 && x < 1e30)) return 1.0 / cbrt(x);
    double y = (double)__builtin_amdgcn_exp2f(__builtin_amdgcn_logf((float)x) *
                                              (-1.0f / 3.0f));
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        const double e = fma(-x, y * y * y, 1.0);
        y = fma(y * e, 1.0 / 3.0, y);
    }
    return y;
}
__device__ inline float inv_cbrt(float x)
{
    if (!(x > 1e-30f && x < 1e30f)) return 1.0f / cbrtf(x);
    float y = __builtin_amdgcn_exp2f(__builtin_amdgcn_logf(x) * (-1.0f / 3.0f));
    const float e = fmaf(-x, y * y * y, 1.0f);
    return fmaf(y * e, 1.0f / 3.0f, y);
}

// 1/h for a wet depth, 0 for a dry one (velocities are then 0).
template <typename T>
__device__ inline T inv_depth(T h, T tol)
{
    return h > tol ? rcp_nr(h) : T(0);
}

// One face between a left and a right state (normal velocity un, tangential
// ut): hydrostatic reconstruction of the depths against the face bed
// max(z_l, z_r), written with bed differences, then the HLL flux with
// two-rarefaction wave-speed estimates and dry-side speeds u -/+ 2c.
template <typename T>
__device__ inline void face_flux(T hl, T unl, T utl, double zl, T hr, T unr,
                                 T utr, double zr, T g, T tol, T F[3],
                                 T& hls_out, T& hrs_out)
{
    // Fused multiply-adds are written out (fma), never left to the
    // compiler: every caller then gets the same roundings, whatever it
    // shares with its neighbours after inlining.
    // (fmax / fmin: maximum and minimum that return the other operand when
    // one is NaN, so a NaN depth clips to 0 as the comparison form does)
    const T dzl = (T)(zr - zl);
    const T dzr = (T)(zl - zr);
    const T hls = fmax(hl - fmax(dzl, T(0)), T(0));
    const T hrs = fmax(hr - fmax(dzr, T(0)), T(0));
    hls_out = hls;
    hrs_out = hrs;
    if (hls <= tol && hrs <= tol) {
        F[0] = T(0);
        F[1] = T(0);
        F[2] = T(0);
        return;
    }
    const T cl = sqrt_nr(g * hls);
    const T cr = sqrt_nr(g * hrs);
    const T ustar = fma(T(0.5), unl + unr, cl) - cr;
    const T cstar = fma(T(0.25), unl - unr, T(0.5) * (cl + cr));
    const T sl = hls <= tol ? fma(T(-2), cr, unr) : fmin(unl - cl, ustar - cstar);
    const T sr = hrs <= tol ? fma(T(2), cl, unl) : fmax(unr + cr, ustar + cstar);
    const T hg = T(0.5) * g;
    const T ql = hls * unl;
    const T qr = hrs * unr;
    const T Ul[3] = {hls, ql, hls * utl};
    const T Ur[2] = {hrs, qr};
    const T Fl[3] = {ql, fma(ql, unl, (hg * hls) * hls), ql * utl};
    const T Fr[3] = {qr, fma(qr, unr, (hg * hrs) * hrs), qr * utr};
    if (sl >= T(0)) {
        F[0] = Fl[0];
        F[1] = Fl[1];
        F[2] = Fl[2];
    } else if (sr <= T(0)) {
        F[0] = Fr[0];
        F[1] = Fr[1];
        F[2] = Fr[2];
    } else {
        // one reciprocal of the speed difference serves the three components
        const T slsr = sl * sr;
        const T inv = rcp_nr(sr - sl);
        // jumps of the conserved variables (the tangential one fused)
        const T dU[3] = {Ur[0] - Ul[0], Ur[1] - Ul[1], fma(hrs, utr, -Ul[2])};
#pragma unroll
        for (int k = 0; k < 3; ++k)
            F[k] = fma(slsr, dU[k], fma(sr, Fl[k], -(sl * Fr[k]))) * inv;
    }
}

template <typename T>
__device__ inline double inflow_rate(const Fv1Ctx<T>& x, double t)
{
    if (!(x.q_peak > 0.0)) return 0.0;
    if (t <= x.t_peak) return x.q_peak * t / x.t_peak;
    if (t <= x.t_base) return x.q_peak * (x.t_base - t) / (x.t_base - x.t_peak);
    return 0.0;
}

// Largest wave speed |u| + c of a cell; ih is 1/h (any value when dry).
template <typename T>
__device__ inline double wave_speed(T h, T qx, T qy, T ih, T g, T tol)
{
    if (!(h > tol)) return 0.0;
    const T c = sqrt_nr(g * h);
    const T u = qx * ih;
    const T v = qy * ih;
    const T su = fabs(u) + c;
    const T sv = fabs(v) + c;
    return (double)(su > sv ? su : sv);
}

// Per-thread accumulators; the same 8 slots form one partial record:
// [0] wave speed, [1] |h|, [2] |qx|, [3] |qy| (maxima), [4] mass, [5] clips
// (sums), [6] non-finite flag, [7] |z| (maxima; |z| only during ingest).
struct Acc {
    double v[kPartial];
};

// Record slots: 0 max wave speed, 1..3 max |h|, |qx|, |qy|, 4 mass, 5 clips,
// 6 non-finite flag, 7 max |z| (ingest), 8 and 9 leaves finished by the dry
// shortcut with their stores written or skipped.
__device__ inline bool slot_is_sum(int q) { return q == 4 || q == 5 || q == 8 || q == 9; }

__device__ inline void acc_reset(Acc& a)
{
#pragma unroll
    for (int q = 0; q < kPartial; ++q) a.v[q] = 0.0;
}

__device__ inline void acc_max(Acc& a, int q, double x)
{
    a.v[q] = x > a.v[q] ? x : a.v[q];
}

// Combine a record into the accumulators (max or sum per slot).
__device__ inline void acc_add_record(Acc& a, const double* r)
{
#pragma unroll
    for (int q = 0; q < kPartial; ++q) {
        if (slot_is_sum(q)) a.v[q] += r[q];
        else acc_max(a, q, r[q]);
    }
}

// Reduce the per-thread accumulators of the workgroup into rec (rec is
// combined, not overwritten).  Must be reached by the whole workgroup.
__device__ inline void acc_flush(Acc& a, double (*red)[kPartial], double* rec)
{
    const int lane = threadIdx.x & (kWave - 1);
    const int wid = threadIdx.x / kWave;
#pragma unroll
    for (int q = 0; q < kPartial; ++q) {
        const double x = slot_is_sum(q) ? wave_sum(a.v[q]) : wave_max(a.v[q]);
        if (lane == 0) red[wid][q] = x;
    }
    __syncthreads();
    // one thread per slot combines the waves in ascending order
    if (threadIdx.x < kPartial) {
        const int q = threadIdx.x;
        const int nw = blockDim.x / kWave;
        const bool sum = slot_is_sum(q);
        double r = red[0][q];
        for (int w = 1; w < nw; ++w) {
            const double y = red[w][q];
            r = sum ? r + y : (y > r ? y : r);
        }
        rec[q] = sum ? rec[q] + r : (r > rec[q] ? r : rec[q]);
    }
    __syncthreads();
    acc_reset(a);
}

// acc_flush into a record of its own in global memory (written once: the
// record takes the workgroup's values, not combined with what it held).
// Must be reached by the whole workgroup.
__device__ inline void acc_flush_store(Acc& a, double (*red)[kPartial], gp<double> out)
{
    const int lane = threadIdx.x & (kWave - 1);
    const int wid = threadIdx.x / kWave;
#pragma unroll
    for (int q = 0; q < kPartial; ++q) {
        const double x = slot_is_sum(q) ? wave_sum(a.v[q]) : wave_max(a.v[q]);
        if (lane == 0) red[wid][q] = x;
    }
    __syncthreads();
    if (threadIdx.x < kPartial) {
        const int q = threadIdx.x;
        const int nw = blockDim.x / kWave;
        const bool sum = slot_is_sum(q);
        double r = red[0][q];
        for (int w = 1; w < nw; ++w) {
            const double y = red[w][q];
            r = sum ? r + y : (y > r ? y : r);
        }
        out[q] = r;
    }
    __syncthreads();
    acc_reset(a);
}

// Finest cell k of the current set (the all-finest form of load_cell).
template <typename T>
__device__ inline Cell<T> load_fine(const Fv1Ctx<T>& x, uint32_t k)
{
    Cell<T> c;
    c.h = ld_off(x.fin[0], k * (uint32_t)sizeof(T));
    c.qx = ld_off(x.fin[1], k * (uint32_t)sizeof(T));
    c.qy = ld_off(x.fin[2], k * (uint32_t)sizeof(T));
    c.z = ld_off(x.zh, (uint32_t)((level_off(x.L) + k) * sizeof(double)));
    return c;
}

// The rest of one leaf's FV1 update once the net fluxes through its four
// faces are known: mass (e, w, n, s: east, west, north, south faces), the
// normal momentum flux of each face with the Audusse bed-slope term of the
// leaf's own side already added (pe, pw, pn, ps), and the tangential
// momentum flux (te, tw, tn, ts).  Forward Euler (Eq. 2) with the level-m
// cell size, the sources, the write-back to the cnt finest cells from f0 on
// in the other set, and the partial record.  inW: the leaf has an
// in-domain west neighbour (no inflow through it).
template <typename T>
__device__ inline void fv1_update(const Fv1Ctx<T>& x, int m, uint32_t c, bool inW,
                                  const Cell<T>& own, T me, T mw, T mn, T ms, T pe, T pw,
                                  T pn, T ps, T te, T tw, T tn, T ts, double dxm, double dym,
                                  uint64_t f0, uint32_t cnt, Acc& acc)
{
    // fused multiply-adds written out, as in face_flux
    const T g = (T)x.g;
    const T tol = (T)x.h_tol;
    const double dt = x.dt;
    const T rx = (T)x.rxy[2 * m];
    const T ry = (T)x.rxy[2 * m + 1];
    T h = fma(-ry, mn - ms, fma(-rx, me - mw, own.h));
    T qx = fma(-ry, tn - ts, fma(-rx, pe - pw, own.qx));
    T qy = fma(-ry, pn - ps, fma(-rx, te - tw, own.qy));

    // sources: rain, west-edge inflow, positivity, dry cells, friction
    if (x.rain_rate != 0.0) h = h + (T)(dt * x.rain_rate);
    if (!inW && x.q_peak > 0.0) {
        const double y_lo = (double)compact1by1(c >> 1) * dym;
        const double lo = y_lo > x.inlet_y0 ? y_lo : x.inlet_y0;
        const double yhi = y_lo + dym;
        const double hi = yhi < x.inlet_y1 ? yhi : x.inlet_y1;
        const double overlap = hi - lo;
        if (overlap > 0.0) {
            const double width = x.inlet_y1 - x.inlet_y0;
            const double q = inflow_rate(x, x.t);
            h = h + (T)(dt * q * overlap / (width * dxm * dym));
        }
    }
    if (h < T(0)) {
        h = T(0);
        acc.v[5] += 1.0;
    }
    const T ih = inv_depth(h, tol);
    if (h <= tol) {
        qx = T(0);
        qy = T(0);
    } else if (x.manning_n > 0.0) {
        const T nm = (T)x.manning_n;
        const T speed = sqrt_nr(fma(qx, qx, qy * qy)) * ih;
        const T cf = g * nm * nm * inv_cbrt(h);
        const T iden = rcp_nr(fma((T)dt * cf * speed, ih, T(1)));
        qx = qx * iden;
        qy = qy * iden;
    }

    // write-back: every finest descendant of the leaf in the other set,
    // except for leaves coarser than a traversal group (the fill copies
    // those from the first descendant)
    store_run<T>(x.fout[0] + f0, cnt, h);
    store_run<T>(x.fout[1] + f0, cnt, qx);
    store_run<T>(x.fout[2] + f0, cnt, qy);

    acc_max(acc, 0, wave_speed<T>(h, qx, qy, ih, g, tol));
    acc_max(acc, 1, fabs((double)h));
    acc_max(acc, 2, fabs((double)qx));
    acc_max(acc, 3, fabs((double)qy));
    acc.v[4] = fma((double)h * dxm, dym, acc.v[4]);
    if (!(isfinite((double)h) && isfinite((double)qx) && isfinite((double)qy)))
        acc.v[6] = 1.0;
}

// Audusse bed-slope term of one side of a face: pressure of the leaf's own
// depth minus that of its reconstructed depth at the face.
template <typename T>
__device__ inline T bed_slope_term(T hg, T h, T hc)
{
    return hg * fma(-hc, hc, h * h);
}

// fv1_update from the four face fluxes (F: the x-flux (mass, normal,
// tangential momentum) of the east and west faces, G: the y-flux of the
// north and south faces) and the leaf's reconstructed depth at each face.
template <typename T>
__device__ inline void fv1_finish(const Fv1Ctx<T>& x, int m, uint32_t c, bool inW,
                                  const Cell<T>& own, const T FE[3], const T FW[3],
                                  const T GN[3], const T GS[3], T hcE, T hcW, T hcN,
                                  T hcS, double dxm, double dym, uint64_t f0,
                                  uint32_t cnt, Acc& acc)
{
    const T hg = T(0.5) * (T)x.g;
    fv1_update<T>(x, m, c, inW, own, FE[0], FW[0], GN[0], GS[0],
                  FE[1] + bed_slope_term(hg, own.h, hcE), FW[1] + bed_slope_term(hg, own.h, hcW),
                  GN[1] + bed_slope_term(hg, own.h, hcN), GS[1] + bed_slope_term(hg, own.h, hcS),
                  FE[2], FW[2], GN[2], GS[2], dxm, dym, f0, cnt, acc);
}

// The full FV1 update of one leaf (the heavy kernel's path; waves whose
// leaves are all dry take fv1_dry_write instead, which gives the same result).
// FIN: the problem's leaves are all finest this step, so the leaf and its
// neighbours are finest cells and no leaf-level byte is needed.
template <typename T, bool FIN>
__device__ inline void fv1_leaf(const Fv1Ctx<T>& x, uint32_t idx, Acc& acc)
{
    const int L = x.L;
    const int m = FIN ? L : level_of(idx);
    const uint32_t c = idx - (uint32_t)level_off(m);
    const T g = (T)x.g;
    const T tol = (T)x.h_tol;
    const double dxm = ldexp(x.dx, L - m);
    const double dym = ldexp(x.dy, L - m);

    const uint32_t lvmask = m > 0 ? (0xffffffffu >> (32 - 2 * m)) : 0u;
    const uint32_t xm = 0x55555555u & lvmask, ym = 0xaaaaaaaau & lvmask;
    const int sh = 2 * (L - m);
    const bool inW = (c & xm) != 0, inE = (c & xm) != xm;
    const bool inS = (c & ym) != 0, inN = (c & ym) != ym;
    const uint32_t cW = inW ? morton_xm(c, xm, ym) : c;
    const uint32_t cE = inE ? morton_xp(c, xm, ym) : c;
    const uint32_t cS = inS ? morton_ym(c, xm, ym) : c;
    const uint32_t cN = inN ? morton_yp(c, xm, ym) : c;
    const int lW = FIN ? L : x.lmap[(uint64_t)cW << sh];
    const int lE = FIN ? L : x.lmap[(uint64_t)cE << sh];
    const int lS = FIN ? L : x.lmap[(uint64_t)cS << sh];
    const int lN = FIN ? L : x.lmap[(uint64_t)cN << sh];
    const Cell<T> own = FIN ? load_fine<T>(x, c) : load_cell<T>(x, m, c);
    const Cell<T> sW = FIN ? load_fine<T>(x, cW) : load_cell<T>(x, m, cW);
    const Cell<T> sE = FIN ? load_fine<T>(x, cE) : load_cell<T>(x, m, cE);
    const Cell<T> sS = FIN ? load_fine<T>(x, cS) : load_cell<T>(x, m, cS);
    const Cell<T> sN = FIN ? load_fine<T>(x, cN) : load_cell<T>(x, m, cN);
    const Cell<T> w = inW ? neighbour_fix<T>(x, m, cW, lW, sW) : ghost_cell<T>(x, HW_W, own);
    const Cell<T> e = inE ? neighbour_fix<T>(x, m, cE, lE, sE) : ghost_cell<T>(x, HW_E, own);
    const Cell<T> so = inS ? neighbour_fix<T>(x, m, cS, lS, sS) : ghost_cell<T>(x, HW_S, own);
    const Cell<T> no = inN ? neighbour_fix<T>(x, m, cN, lN, sN) : ghost_cell<T>(x, HW_N, own);

    // Velocities only matter on faces with a wet side; a wave whose five
    // states are all dry skips the divisions (values stay 0 and unused).
    T uc = T(0), vc = T(0), uw = T(0), vw = T(0), ue = T(0), ve = T(0);
    T us = T(0), vs = T(0), un = T(0), vn = T(0);
    const bool wet = own.h > tol || w.h > tol || e.h > tol || so.h > tol || no.h > tol;
    if (wave_any(wet)) {
        const T rc = inv_depth(own.h, tol), rw = inv_depth(w.h, tol);
        const T re = inv_depth(e.h, tol), rs = inv_depth(so.h, tol);
        const T rn = inv_depth(no.h, tol);
        uc = own.qx * rc;
        vc = own.qy * rc;
        uw = w.qx * rw;
        vw = w.qy * rw;
        ue = e.qx * re;
        ve = e.qy * re;
        us = so.qx * rs;
        vs = so.qy * rs;
        un = no.qx * rn;
        vn = no.qy * rn;
    }

    T FE[3], FW[3], GN[3], GS[3];
    T hcE, hcW, hcN, hcS, unused;
    face_flux<T>(own.h, uc, vc, own.z, e.h, ue, ve, e.z, g, tol, FE, hcE, unused);
    face_flux<T>(w.h, uw, vw, w.z, own.h, uc, vc, own.z, g, tol, FW, unused, hcW);
    face_flux<T>(own.h, vc, uc, own.z, no.h, vn, un, no.z, g, tol, GN, hcN, unused);
    face_flux<T>(so.h, vs, us, so.z, own.h, vc, uc, own.z, g, tol, GS, unused, hcS);
    fv1_finish<T>(x, m, c, inW, own, FE, FW, GN, GS, hcE, hcW, hcN, hcS, dxm, dym,
                  (uint64_t)c << sh, m >= x.Lg ? (1u << sh) : 1u, acc);
}

// LDS of one wave's block update.  Cells: the 8 x 8 cells of the block and
// their 32 face neighbours on a 10 x 10 local grid (local (i + 1, j + 1)
// holds block cell (i, j); corners unused), local (i, j) stored at
// cell_slot(i, j).  Faces, per direction: slot k < 64 holds the west
// (x) or south (y) face of the block cell in Morton position k, slots 64 + r
// the east face of row r (x) or the north face of column r (y); per face the
// mass flux, the normal momentum flux with the bed-slope term of the left
// (lower) side added and with that of the right (upper) side added, and the
// tangential momentum flux.
template <typename T>
struct BlockLds {
    T h[160], u[160], v[160];
    double z[160];
    T F[2][4][72];     // [x, y][mass, normal + left term, normal + right term, tangential][slot]
};

// Slot of local cell (i, j): rows of 16 words, each row rotated by 4 j, so
// that the cells of any aligned 4 x 4 (and 8 x 4) group of lanes fall in
// different LDS banks.
__device__ inline int cell_slot(uint32_t i, uint32_t j)
{
    return (int)(16u * j + ((i + 4u * j) & 15u));
}

// Order LDS writes of the wave before its later LDS reads (the LDS executes
// one wave's operations in order; this keeps the compiler from moving them).
__device__ inline void wave_lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Per-lane constants of the block update (the same for every block): the
// lane's cell in the block, its local slot, the cells on either side of its
// west and south faces, its boundary face in the third pass (lanes 0-15: the
// east face of row lane, or the north face of column lane - 8), the slots of
// its east and north faces, and its halo cell (lanes 0-31: side lane / 8,
// position lane % 8).
struct BlockConst {
    uint32_t bi, bj;       // own cell in the block
    int me;                // own cell's slot
    int wl, sl;            // slots of the cells west and south of it
    int bl, br;            // third pass: slots left and right of the face
    int qe, qn;            // face slots of the own cell's east and north faces
    int hidx;              // halo cell's slot
    uint32_t ei, ej;       // block cell next to the halo cell
    int di, dj;            // offset from that block cell to the halo cell
};

__device__ inline BlockConst block_const()
{
    BlockConst k;
    const uint32_t lane = threadIdx.x & (kWave - 1u);
    k.bi = compact1by1(lane);
    k.bj = compact1by1(lane >> 1);
    k.me = cell_slot(k.bi + 1, k.bj + 1);
    k.wl = cell_slot(k.bi, k.bj + 1);
    k.sl = cell_slot(k.bi + 1, k.bj);
    const uint32_t r = lane & 7u;
    k.bl = lane < 8u ? cell_slot(8, r + 1) : cell_slot(r + 1, 8);
    k.br = lane < 8u ? cell_slot(9, r + 1) : cell_slot(r + 1, 9);
    k.qe = k.bi < 7u ? (int)morton(k.bi + 1, k.bj) : 64 + (int)k.bj;
    k.qn = k.bj < 7u ? (int)morton(k.bi, k.bj + 1) : 64 + (int)k.bi;
    const uint32_t dir = (lane >> 3) & 3u;   // HW_W, HW_E, HW_S, HW_N
    const bool xdir = dir < 2u;
    k.ei = xdir ? (dir == (uint32_t)HW_W ? 0u : 7u) : r;
    k.ej = xdir ? r : (dir == (uint32_t)HW_S ? 0u : 7u);
    k.di = dir == (uint32_t)HW_W ? -1 : dir == (uint32_t)HW_E ? 1 : 0;
    k.dj = dir == (uint32_t)HW_S ? -1 : dir == (uint32_t)HW_N ? 1 : 0;
    k.hidx = xdir ? cell_slot(dir == (uint32_t)HW_W ? 0u : 9u, r + 1)
                  : cell_slot(r + 1, dir == (uint32_t)HW_S ? 0u : 9u);
    return k;
}

// One face of the block update from the staged cells (left / right slots il,
// ir; x: normal velocity u, y: v), stored in face slot q of direction d.
template <typename T>
__device__ inline void block_face(BlockLds<T>& s, int il, int ir, bool isx, int d, int q,
                                  T g, T hg, T tol)
{
    const T hl = s.h[il], hr = s.h[ir];
    const T ul = s.u[il], vl = s.v[il], ur = s.u[ir], vr = s.v[ir];
    T F[3], hls, hrs;
    face_flux<T>(hl, isx ? ul : vl, isx ? vl : ul, s.z[il], hr, isx ? ur : vr, isx ? vr : ur,
                 s.z[ir], g, tol, F, hls, hrs);
    s.F[d][0][q] = F[0];
    s.F[d][1][q] = F[1] + bed_slope_term(hg, hl, hls);
    s.F[d][2][q] = F[1] + bed_slope_term(hg, hr, hrs);
    s.F[d][3][q] = F[2];
}

// The full FV1 update of the 64 finest leaves of one aligned 8 x 8 Morton
// block (cells c0 .. c0 + 63, L >= 3), by one wave.  The result is
// fv1_leaf's for each cell: every face flux is the same call with the same
// arguments, made once per face instead of once from each side (144 faces
// for 64 cells instead of 256: each lane's west face, each lane's south
// face, then the 16 faces on the block's east and north edges), and each
// cell's velocities are formed once instead of once per face that uses
// them.  MIXED: the problem has coarser leaves this step, so a face
// neighbour outside the block may lie inside one; its leaf-level byte then
// names that leaf, whose values replace the finest ones (fv1_leaf's
// neighbour rule).  Otherwise every leaf is finest.
template <typename T, bool MIXED>
__device__ inline void fv1_block(const Fv1Ctx<T>& x, uint32_t c0, Acc& acc, BlockLds<T>& s,
                                 const BlockConst& kc)
{
    const int L = x.L;
    const uint32_t lane = threadIdx.x & (kWave - 1u);
    const T g = (T)x.g;
    const T hg = T(0.5) * g;
    const T tol = (T)x.h_tol;
    const uint32_t side = 1u << L;
    const uint32_t I0 = compact1by1(c0), J0 = compact1by1(c0 >> 1);
    const uint32_t c = c0 + lane;
    // Halo (lanes 0-31): the face neighbour of the block cell (ei, ej), or
    // beyond the domain edge that cell's ghost.  Every load of the block is
    // issued before any is used (lanes 32-63 load their own cell a second
    // time, unused).
    const int nI = (int)(I0 + kc.ei) + kc.di;
    const int nJ = (int)(J0 + kc.ej) + kc.dj;
    const bool in = nI >= 0 && nI < (int)side && nJ >= 0 && nJ < (int)side;
    const uint32_t src = lane >= 32u ? c
                       : in ? morton((uint32_t)nI, (uint32_t)nJ) : c0 + morton(kc.ei, kc.ej);
    const Cell<T> own = load_fine<T>(x, c);
    Cell<T> hc = load_fine<T>(x, src);
    int lv = L;
    if (MIXED && in && lane < 32u) lv = x.lmap[src];
    __builtin_amdgcn_sched_barrier(0);
    if (MIXED && lv < L) hc = load_cell<T>(x, lv, src >> (2 * (L - lv)));
    if (!in && lane < 32u) {
        const int dir = (int)((lane >> 3) & 3u);
        const bool wall = (dir == HW_W && x.bc[HW_W] == HW_BC_WALL) ||
                          (dir == HW_E && x.bc[HW_E] == HW_BC_WALL) ||
                          (dir == HW_S && x.bc[HW_S] == HW_BC_WALL) ||
                          (dir == HW_N && x.bc[HW_N] == HW_BC_WALL);
        if (wall) {
            if (dir < 2) hc.qx = -hc.qx;
            else hc.qy = -hc.qy;
        }
    }
    {
        const T r = inv_depth(own.h, tol);
        s.h[kc.me] = own.h;
        s.u[kc.me] = own.qx * r;
        s.v[kc.me] = own.qy * r;
        s.z[kc.me] = own.z;
    }
    if (lane < 32u) {
        const T r = inv_depth(hc.h, tol);
        s.h[kc.hidx] = hc.h;
        s.u[kc.hidx] = hc.qx * r;
        s.v[kc.hidx] = hc.qy * r;
        s.z[kc.hidx] = hc.z;
    }
    wave_lds_sync();
    block_face<T>(s, kc.wl, kc.me, true, 0, (int)lane, g, hg, tol);
    block_face<T>(s, kc.sl, kc.me, false, 1, (int)lane, g, hg, tol);
    if (lane < 16u) {
        const bool isx = lane < 8u;
        block_face<T>(s, kc.bl, kc.br, isx, isx ? 0 : 1, 64 + (int)(lane & 7u), g, hg, tol);
    }
    wave_lds_sync();
    // own cell: left of its east and north faces, right of its west and
    // south faces
    const int q = (int)lane;
    const T me = s.F[0][0][kc.qe], mw = s.F[0][0][q];
    const T mn = s.F[1][0][kc.qn], ms = s.F[1][0][q];
    const T pe = s.F[0][1][kc.qe], pw = s.F[0][2][q];
    const T pn = s.F[1][1][kc.qn], ps = s.F[1][2][q];
    const T te = s.F[0][3][kc.qe], tw = s.F[0][3][q];
    const T tn = s.F[1][3][kc.qn], ts = s.F[1][3][q];
    const bool inW = (I0 + kc.bi) != 0u;
    fv1_update<T>(x, L, c, inW, own, me, mw, mn, ms, pe, pw, pn, ps, te, tw, tn, ts, x.dx,
                  x.dy, (uint64_t)c, 1u, acc);
    // the next block's LDS writes must not overtake this block's reads
    wave_lds_sync();
}

// True when the west-edge inflow adds water to leaf (m, c) at time t.
template <typename T>
__device__ inline bool inflow_on(const Fv1Ctx<T>& x, int m, uint32_t c)
{
    const uint32_t lvmask = m > 0 ? (0xffffffffu >> (32 - 2 * m)) : 0u;
    if ((c & 0x55555555u & lvmask) != 0 || !(x.q_peak > 0.0)) return false;
    const double dym = ldexp(x.dy, x.L - m);
    const double y_lo = (double)compact1by1(c >> 1) * dym;
    const double lo = y_lo > x.inlet_y0 ? y_lo : x.inlet_y0;
    const double yhi = y_lo + dym;
    const double hi = yhi < x.inlet_y1 ? yhi : x.inlet_y1;
    return hi - lo > 0.0 && inflow_rate(x, x.t) != 0.0;
}

// Dry-shortcut probe of kLeafBatch leaves per thread: each leaf's depth and
// the depths its four faces see (same-level cell, or the coarser leaf that
// contains it; the cell itself beyond the domain edge, as both ghost kinds
// copy the depth).  All leaves' loads are issued before any is consumed:
// first the leaf indices, then every leaf-level byte and depth at once, then,
// only in waves that have a coarser neighbour, the coarser depths.  The
// shortcut holds when all five depths are at most h_tol and no inflow
// reaches the leaf: the full update then leaves h unchanged, sets both
// discharges to 0 and adds no wave speed (fv1_leaf's result in that case).
template <typename T>
struct LightBatch {
    T h[kLeafBatch];
    uint32_t c[kLeafBatch];
    int m[kLeafBatch];
    bool dry[kLeafBatch];
    uint64_t e[kLeafBatch];   // write-history entry of the wave's first cell's block
};

// Leaf indices of one super-chunk (tail lanes repeat the last leaf).
template <typename T>
__device__ inline void light_indices(const Fv1Ctx<T>& x, uint32_t base, uint32_t idx[kLeafBatch])
{
#pragma unroll
    for (int u = 0; u < kLeafBatch; ++u) {
        uint32_t leaf = base + (uint32_t)u * kBlock + threadIdx.x;
        leaf = leaf < x.nl ? leaf : x.nl - 1u;
        idx[u] = ld_off(x.leaves, leaf * 4u);
    }
}

// Sub-chunks of one super-chunk of a mixed problem that are wet by their
// leaves' own depths alone: bit u is set when some leaf of sub-chunk u has
// a depth above h_tol (it fails the dry test whatever its neighbours hold).
// Returns true when that settles every sub-chunk (each has such a leaf or
// no leaf at all), so that neither neighbours nor history need be read; a
// history entry left unrefreshed names an older step and permits no skip.
// Without rain only (rain makes every sub-chunk wet on the general path).
template <typename T>
__device__ inline bool light_wet_by_own_depth(const Fv1Ctx<T>& x, uint32_t base,
                                              const uint32_t idx[kLeafBatch], uint32_t& bits)
{
    const T tol = (T)x.h_tol;
    T h[kLeafBatch];
#pragma unroll
    for (int u = 0; u < kLeafBatch; ++u) {
        const int m = level_of(idx[u]);
        h[u] = load_h<T>(x, m, idx[u] - (uint32_t)level_off(m));
    }
    bool settled = true;
    bits = 0;
#pragma unroll
    for (int u = 0; u < kLeafBatch; ++u) {
        const bool ok = base + (uint32_t)u * kBlock + threadIdx.x < x.nl;
        const bool wet = wave_any(ok && h[u] > tol);
        if (wet) bits |= 1u << u;
        else if (wave_any(ok)) settled = false;
    }
    return settled;
}

// Same-level neighbour codes of cell c on level m (the cell itself beyond
// the domain edge), in the order W, E, S, N.
__device__ inline void neighbour_codes(uint32_t c, int m, uint32_t nb[4])
{
    const uint32_t lvmask = m > 0 ? (0xffffffffu >> (32 - 2 * m)) : 0u;
    const uint32_t xm = 0x55555555u & lvmask, ym = 0xaaaaaaaau & lvmask;
    nb[0] = (c & xm) != 0 ? morton_xm(c, xm, ym) : c;
    nb[1] = (c & xm) != xm ? morton_xp(c, xm, ym) : c;
    nb[2] = (c & ym) != 0 ? morton_ym(c, xm, ym) : c;
    nb[3] = (c & ym) != ym ? morton_yp(c, xm, ym) : c;
}

template <typename T>
__device__ inline void light_probe(const Fv1Ctx<T>& x, const uint32_t idx[kLeafBatch],
                                   LightBatch<T>& b)
{
    constexpr int U = kLeafBatch;
    const int L = x.L;
    const T tol = (T)x.h_tol;
    int lv[U][4];
    T hh[U][5];
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const int m = level_of(idx[u]);
        const uint32_t c = idx[u] - (uint32_t)level_off(m);
        b.m[u] = m;
        b.c[u] = c;
        uint32_t nb[4];
        neighbour_codes(c, m, nb);
        const int sh = 2 * (L - m);
#pragma unroll
        for (int k = 0; k < 4; ++k) lv[u][k] = ld_off(x.lmap, nb[k] << sh);
        hh[u][0] = load_h<T>(x, m, c);
#pragma unroll
        for (int k = 0; k < 4; ++k) hh[u][k + 1] = load_h<T>(x, m, nb[k]);
        // c < 4^m <= 4^L, so c / 64 indexes the table even when unused
        b.e[u] = x.hist[uniform(c) >> 6];
    }
    __builtin_amdgcn_sched_barrier(0);
    bool coarser = false;
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
        for (int k = 0; k < 4; ++k) coarser = coarser || lv[u][k] < b.m[u];
    if (wave_any(coarser)) {
        // rare: some neighbour is a coarser leaf; its codes are recomputed
#pragma unroll
        for (int u = 0; u < U; ++u) {
            uint32_t nb[4];
            neighbour_codes(b.c[u], b.m[u], nb);
#pragma unroll
            for (int k = 0; k < 4; ++k)
                if (lv[u][k] < b.m[u])
                    hh[u][k + 1] = load_h<T>(x, lv[u][k], nb[k] >> (2 * (b.m[u] - lv[u][k])));
        }
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
        b.h[u] = hh[u][0];
        b.dry[u] = hh[u][0] <= tol && hh[u][1] <= tol && hh[u][2] <= tol &&
                   hh[u][3] <= tol && hh[u][4] <= tol && !inflow_on<T>(x, b.m[u], b.c[u]);
    }
}

// light_probe for a problem whose leaves are all finest: leaf i is finest
// cell i and every neighbour is a finest leaf, so no index, no leaf-level
// byte and no coarser depth is needed; all depths come from one base.
template <typename T>
__device__ inline void light_probe_finest(const Fv1Ctx<T>& x, uint32_t base, LightBatch<T>& b)
{
    constexpr int U = kLeafBatch;
    const int L = x.L;
    const T tol = (T)x.h_tol;
    const uint32_t lvmask = L > 0 ? (0xffffffffu >> (32 - 2 * L)) : 0u;
    const uint32_t xm = 0x55555555u & lvmask, ym = 0xaaaaaaaau & lvmask;
    T hh[U][5];
#pragma unroll
    for (int u = 0; u < U; ++u) {
        uint32_t c = base + (uint32_t)u * kBlock + threadIdx.x;
        c = c < x.nl ? c : x.nl - 1u;
        b.m[u] = L;
        b.c[u] = c;
        const uint32_t w = (c & xm) != 0 ? morton_xm(c, xm, ym) : c;
        const uint32_t e = (c & xm) != xm ? morton_xp(c, xm, ym) : c;
        const uint32_t so = (c & ym) != 0 ? morton_ym(c, xm, ym) : c;
        const uint32_t no = (c & ym) != ym ? morton_yp(c, xm, ym) : c;
        hh[u][0] = ld_off(x.fin[0], c * (uint32_t)sizeof(T));
        hh[u][1] = ld_off(x.fin[0], w * (uint32_t)sizeof(T));
        hh[u][2] = ld_off(x.fin[0], e * (uint32_t)sizeof(T));
        hh[u][3] = ld_off(x.fin[0], so * (uint32_t)sizeof(T));
        hh[u][4] = ld_off(x.fin[0], no * (uint32_t)sizeof(T));
        b.e[u] = x.hist[uniform(c) >> 6];
    }
    // Keep every leaf's loads ahead of the first use (one round trip), and
    // consume every loaded value on every path: a load still pending at the
    // loop's back edge would make the next iteration wait for all memory
    // operations, stores included.
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int u = 0; u < U; ++u) {
        asm volatile("" ::"v"(b.e[u]));
        b.h[u] = hh[u][0];
        b.dry[u] = (hh[u][0] <= tol) & (hh[u][1] <= tol) & (hh[u][2] <= tol) &
                   (hh[u][3] <= tol) & (hh[u][4] <= tol) & !inflow_on<T>(x, L, b.c[u]);
    }
}

// The dry shortcut's result (identical to the full update, see fv1_leaf);
// the stores are left out when the set being written already holds it.
template <typename T>
__device__ inline void fv1_dry_write(const Fv1Ctx<T>& x, int m, uint32_t c, T h, Acc& acc,
                                     bool store)
{
    if (store) {
        const int sh = 2 * (x.L - m);
        const uint64_t f0 = (uint64_t)c << sh;
        const uint32_t cnt = m >= x.Lg ? (1u << sh) : 1u;
        store_run<T>(x.fout[0] + f0, cnt, h);
        store_run<T>(x.fout[1] + f0, cnt, T(0));
        store_run<T>(x.fout[2] + f0, cnt, T(0));
    }
    acc_max(acc, 1, fabs((double)h));
    acc.v[4] += ((double)h * ldexp(x.dx, x.L - m)) * ldexp(x.dy, x.L - m);
    acc.v[8] += store ? 1.0 : 0.0;
    acc.v[9] += store ? 0.0 : 1.0;
}

// Write history of one wave's 64 leaves (wave-uniform).  When those leaves
// are the 64 finest cells of one aligned Morton block B, the block's entry
// records (index of the step + 1) << 2 and, in its two low bits, whether the
// dry shortcut finished all 64 at the last two steps that updated it.  If it
// did at steps k-1 and k-2 (entry written at step k-1 with both bits) and
// does again at step k, the set being written at step k holds state k-1 on
// B, which is (h, 0, 0) with the h that steps k-1 and k leave unchanged: the
// result of step k is already in place and its stores are skipped.  Any
// other writer of B's cells (full update, coarser leaves, a misaligned
// wave) does not refresh the entry, so its step no longer matches and the
// next steps store again.  Returns true when the stores may be skipped.
// The entry update and skip decision once the wave is known to be one
// aligned block (c: a lane's cell; the block is c / 64).
template <typename T>
__device__ inline bool light_history_block(const Fv1Ctx<T>& x, bool block, uint32_t c,
                                           bool dry, uint64_t e)
{
    if (!block || !x.write_skip) return false;
    const bool valid = (e >> 2) == x.step;
    const uint64_t bits = ((valid ? (e << 1) : 0ull) | (dry ? 1ull : 0ull)) & 3ull;
    if ((threadIdx.x & (kWave - 1)) == 0) x.hist[c >> 6] = ((x.step + 1) << 2) | bits;
    return dry && valid && (e & 3ull) == 3ull;
}

template <typename T>
__device__ inline bool light_history(const Fv1Ctx<T>& x, bool ok, int m, uint32_t c,
                                     bool dry, uint64_t e)
{
    const uint32_t c0 = uniform(c);
    const uint32_t c63 = (uint32_t)__builtin_amdgcn_readlane((int)c, kWave - 1);
    const bool block = !wave_any(!ok || m != x.L) && (c0 & 63u) == 0u && c63 == c0 + 63u;
    return light_history_block<T>(x, block, c0, dry, e);
}

// Super-chunks of a problem's block region (whole finest blocks at the head
// of a block-first list, which the heavy kernel updates at a fraction of
// the per-leaf cost): 0 when every leaf is finest or the list has none.
__device__ inline uint32_t block_chunks(const Desc& d, const hw_scalars* sc, bool fin)
{
    if (fin || !block_list(d)) return 0u;
    return (64u * (uint32_t)sc->acc[STEP_NBLK]) / (uint32_t)(kLeafBatch * kBlock);
}

// Order in which the schedule visits a problem's nc super-chunks: the nbc
// chunks of the block region and the others interleaved in proportion
// (visit v takes block chunk floor(v nbc / nc) when that count steps up,
// else the next other chunk), so that each XCD's contiguous segment of the
// schedule holds its share of both kinds, each kind in list order.
__device__ inline uint32_t chunk_order(uint32_t v, uint32_t nbc, uint32_t nc)
{
    if (nbc == 0u || nbc >= nc) return v;
    const uint32_t b = (uint32_t)(((uint64_t)v * nbc) / nc);
    const bool blk = (uint32_t)(((uint64_t)(v + 1u) * nbc) / nc) > b;
    return blk ? b : nbc + (v - b);
}

// Chunk bookkeeping shared by the two FV1 kernels: the leaves of every
// problem are cut into super-chunks of kLeafBatch * kBlock leaves; the
// super-chunk sequence of all problems is split into 8 contiguous segments,
// one per XCD (workgroups are dispatched to XCDs round-robin), so that
// neighbouring leaves share an L2.  A workgroup takes every (gridDim.x/8)-th
// super-chunk of its segment.
struct Fv1Sched {
    uint32_t c_begin, c_end, g8;
};

// Whether every finest cell of the problem is a leaf this step (the leaf
// list is then the identity on the finest level).
__device__ inline bool all_finest(const Desc& d, uint64_t n_leaves)
{
    return n_leaves == (1ull << (2 * d.L));
}

// Problems a chunk schedule covers: every stepping problem, only those
// whose leaves are all finest this step, or only the others.
enum { kAllProblems = 0, kFinestOnly = 1, kMixedOnly = 2 };

// Chunk prefix over the stepping problems of the given kind; optionally,
// per problem, whether it steps (mine) and whether its leaves are all
// finest.
__device__ inline Fv1Sched fv1_schedule(const Desc* descs, int n, uint32_t* cpre,
                                        int mode = kAllProblems, uint8_t* mine = nullptr,
                                        uint8_t* finest = nullptr, uint32_t* cblk = nullptr)
{
    constexpr uint32_t SC = kLeafBatch * kBlock;
    if (threadIdx.x == 0) {
        uint32_t a = 0;
        for (int s = 0; s < n; ++s) {
            cpre[s] = a;
            const hw_scalars* sc = descs[s].scal;
            const uint64_t nl = step_leaves(descs[s], sc);
            const bool m = !sc->done;
            const bool fin = all_finest(descs[s], nl);
            if (mine) mine[s] = m ? 1 : 0;
            if (finest) finest[s] = fin ? 1 : 0;
            if (cblk) cblk[s] = block_chunks(descs[s], sc, fin);
            const bool take = m && (mode == kAllProblems || (mode == kFinestOnly) == fin);
            a += take ? ((uint32_t)nl + SC - 1) / SC : 0u;
        }
        cpre[n] = a;
    }
    __syncthreads();
    const uint32_t total = uniform(cpre[n]);
    Fv1Sched f;
    f.g8 = gridDim.x >> 3;
    const uint32_t seg = (total + 7u) / 8u;
    f.c_begin = (blockIdx.x & 7u) * seg + (blockIdx.x >> 3);
    const uint32_t e = (blockIdx.x & 7u) * seg + seg;
    f.c_end = e < total ? e : total;
    return f;
}

// The light kernel's pass over the 64-cell blocks of a problem whose
// leaves are all finest (L >= 5): the first encoding pass has tested every
// block (its own cells and the edge cells of its four neighbour blocks) and
// summed its mass and max |h|, so one lane decides one block from a few
// bytes, with every load in one round trip.  Lane t takes block t % 8 of
// super-chunk sc0 + (t / 8) * stride (cnt super-chunks); a wet block sets
// its bit in the super-chunk's wet word for the heavy kernel; a dry one adds
// its mass and max |h| and, unless the write history allows skipping,
// joins a list whose (h, 0, 0) stores all waves of the workgroup then share.
template <typename T>
__device__ inline void light_blocks(const Fv1Ctx<T>& x, gp<uint8_t> wetb, uint32_t sc0,
                                    uint32_t stride, uint32_t cnt, Acc& acc,
                                    uint32_t* slist, uint32_t& scount)
{
    const int tid = threadIdx.x;
    const int lane = tid & (kWave - 1);
    const int wid = tid / kWave;
    const uint32_t j = (uint32_t)tid >> 3, bi = (uint32_t)tid & 7u;
    const bool act = j < cnt;
    const uint32_t sc = sc0 + (act ? j : 0u) * stride;
    const uint32_t blk = 8u * sc + bi;
    // block codes live on level L-3
    const uint32_t bmask = 0xffffffffu >> (32 - 2 * (x.L - 3));
    const uint32_t bxm = 0x55555555u & bmask, bym = 0xaaaaaaaau & bmask;
    const bool hw = (blk & bxm) != 0, he = (blk & bxm) != bxm;
    const bool hs = (blk & bym) != 0, hn = (blk & bym) != bym;
    const uint32_t st = x.dryb[blk];
    // the edge of each neighbour block that touches this one: the west
    // neighbour's east column, and so on (the block's own byte, masked off,
    // beyond the domain edge)
    const uint32_t w = x.dryb[hw ? morton_xm(blk, bxm, bym) : blk];
    const uint32_t e = x.dryb[he ? morton_xp(blk, bxm, bym) : blk];
    const uint32_t so = x.dryb[hs ? morton_ym(blk, bxm, bym) : blk];
    const uint32_t no = x.dryb[hn ? morton_yp(blk, bxm, bym) : blk];
    const uint64_t eh = x.hist[blk];
    const vd2 mh = *reinterpret_cast<gp<const vd2>>(x.bpart + 2ull * blk);
    if (tid == 0) scount = 0u;
    // bitwise, not short-circuit: a branch per neighbour would wait for each
    // byte before loading the next
    const uint32_t sn = (w & (hw ? 8u : 0u)) | (e & (he ? 4u : 0u)) |
                        (so & (hs ? 32u : 0u)) | (no & (hn ? 16u : 0u));
    const bool dry = x.rain_rate == 0.0 && (st & 3u) == 0u && sn == 0u;
    bool skip = false;
    if (act && x.write_skip) {
        // the same record as for a wave's aligned block of 64 finest leaves
        const bool valid = (eh >> 2) == x.step;
        const uint64_t hb = ((valid ? (eh << 1) : 0ull) | (dry ? 1ull : 0ull)) & 3ull;
        x.hist[blk] = ((x.step + 1) << 2) | hb;
        skip = dry && valid && (eh & 3ull) == 3ull;
    }
    if (act && dry) {
        acc.v[4] += mh.x;
        acc_max(acc, 1, mh.y);
        acc.v[8] += skip ? 0.0 : 64.0;
        acc.v[9] += skip ? 64.0 : 0.0;
    }
    // wet word of the super-chunk: byte (block % 4), bit (block / 4)
    uint32_t word = (act && !dry) ? 1u << (8u * (bi & 3u) + (bi >> 2)) : 0u;
    word |= __shfl_xor(word, 1);
    word |= __shfl_xor(word, 2);
    word |= __shfl_xor(word, 4);
    if (act && bi == 0u) *reinterpret_cast<gp<uint32_t>>(wetb + 4ull * sc) = word;
    __syncthreads();   // scount cleared
    const bool ns = act && dry && !skip;
    const uint64_t m = __ballot(ns);
    if (m) {
        uint32_t at = 0u;
        if (lane == 0) at = atomicAdd(&scount, (uint32_t)__popcll(m));
        at = uniform(at);
        if (ns) slist[at + (uint32_t)__popcll(m & ((1ull << lane) - 1ull))] = blk;
    }
    __syncthreads();
    const uint32_t nst = uniform(scount);
    for (uint32_t k = (uint32_t)wid; k < nst; k += 2u * (kBlock / kWave)) {
        const uint32_t k2 = k + kBlock / kWave;
        const bool two = k2 < nst;
        const uint32_t ca = 64u * uniform(slist[k]) + (uint32_t)lane;
        const uint32_t cb = 64u * uniform(slist[two ? k2 : k]) + (uint32_t)lane;
        const T ha = ld_off(x.fin[0], ca * (uint32_t)sizeof(T));
        const T hb = ld_off(x.fin[0], cb * (uint32_t)sizeof(T));
        x.fout[0][ca] = ha;
        x.fout[1][ca] = T(0);
        x.fout[2][ca] = T(0);
        if (two) {
            x.fout[0][cb] = hb;
            x.fout[1][cb] = T(0);
            x.fout[2][cb] = T(0);
        }
    }
    __syncthreads();   // slist and scount are reused by the next pass
}

// FV1, light kernel: every leaf's dry probe; waves whose leaves are all
// dry (no rain, no inflow on them) are finished here; the others are marked
// in the wet table (one byte per super-chunk and wave, bit u for the wave's
// u-th sub-chunk) for the heavy kernel.  A problem whose leaves are all
// finest this step takes the dry pass over 64-cell blocks (L >= 5) or the
// finest-leaf probe; the others the general probe (leaf list, leaf-level
// map, coarser neighbours).  Records go to slots [0, gridDim.x).
template <typename T>
__global__ __launch_bounds__(kBlock) void k_fv1_light(const Desc* __restrict__ descs, int n)
{
    constexpr int U = kLeafBatch;
    constexpr uint32_t SC = U * kBlock;
    __shared__ uint32_t cpre[kMaxScen + 1];
    __shared__ double rec[kMaxScen][kPartial];
    __shared__ double red[kBlock / kWave][kPartial];
    const int tid = threadIdx.x;
    const int wid = tid / kWave;
    for (int q = tid; q < n * kPartial; q += kBlock) rec[q / kPartial][q % kPartial] = 0.0;
    __shared__ uint8_t mine[kMaxScen];
    __shared__ uint8_t finest[kMaxScen];
    __shared__ uint32_t slist[kBlock];
    __shared__ uint32_t scount;
    Acc acc;
    acc_reset(acc);
    Fv1Ctx<T> x;
    gp<uint8_t> wetb = gp<uint8_t>(nullptr);
    // The step's snapshot of the set and done flag for the copy-down (which
    // runs in the same launch as the finalisation that changes them).
    if (blockIdx.x == 0 && tid < n) {
        const gp<hw_scalars> sc = glob(descs[tid].scal);
        sc->acc[STEP_CUR] = (double)sc->cur;
        sc->acc[STEP_DONE] = (double)sc->done;
    }
    // The problems whose leaves are all finest, then the others, each kind
    // spread over every workgroup (and so over every XCD) on its own: the
    // two kinds cost very differently per chunk.
    for (int kind = 0; kind < 2; ++kind) {
        const bool fin = kind == 0;
        const Fv1Sched f =
            fv1_schedule(descs, n, cpre, fin ? kFinestOnly : kMixedOnly, mine, finest);
        int cs = -1;
        uint32_t c0 = 0, c1 = 0, nbc = 0;
        for (uint32_t ch = f.c_begin; ch < f.c_end; ch += f.g8) {
            if (cs < 0 || ch >= c1) {
                int s = cs < 0 ? 0 : cs;
                while (cpre[s + 1] <= ch) ++s;
                s = uniform(s);
                if (cs >= 0) acc_flush(acc, red, rec[cs]);
                cs = s;
                make_ctx<T>(x, descs[s]);
                wetb = glob(descs[s].wet);
                c0 = uniform(cpre[s]);
                c1 = uniform(cpre[s + 1]);
                nbc = fin ? 0u : uniform(block_chunks(descs[s], descs[s].scal, false));
            }
            if (fin && x.L >= 5 && !x.uniform) {
                // up to 32 of this workgroup's super-chunks at once, all of the
                // current problem
                const uint32_t lim = f.c_end < c1 ? f.c_end : c1;
                uint32_t cnt = (lim - ch + f.g8 - 1u) / f.g8;
                cnt = cnt < 32u ? cnt : 32u;
                light_blocks<T>(x, wetb, ch - c0, f.g8, cnt, acc, slist, scount);
                ch += (cnt - 1u) * f.g8;
                continue;
            }
            // the super-chunk this visit takes (the heavy kernel visits in
            // the same order)
            const uint32_t sc = chunk_order(ch - c0, nbc, c1 - c0);
            const uint32_t base = sc * SC;
            LightBatch<T> b;
            uint32_t bits = 0;
            if (fin) {
                light_probe_finest<T>(x, base, b);
                // every full wave is one aligned 64-cell block of finest leaves
                const double area = x.dx * x.dy;
    #pragma unroll
                for (int u = 0; u < U; ++u) {
                    const bool ok = base + (uint32_t)u * kBlock + tid < x.nl;
                    const bool wet = x.rain_rate != 0.0 || wave_any(ok && !b.dry[u]);
                    const bool skip = light_history_block<T>(x, !wave_any(!ok), b.c[u], !wet, b.e[u]);
                    if (wet) {
                        bits |= 1u << u;
                    } else if (ok) {
                        if (!skip) {
                            x.fout[0][b.c[u]] = b.h[u];
                            x.fout[1][b.c[u]] = T(0);
                            x.fout[2][b.c[u]] = T(0);
                        }
                        acc_max(acc, 1, fabs((double)b.h[u]));
                        acc.v[4] += (double)b.h[u] * area;
                        acc.v[8] += skip ? 0.0 : 1.0;
                        acc.v[9] += skip ? 1.0 : 0.0;
                    }
                }
            } else {
                uint32_t idx[U];
                light_indices<T>(x, base, idx);
                if (x.rain_rate == 0.0 && light_wet_by_own_depth<T>(x, base, idx, bits)) {
                    if ((tid & (kWave - 1)) == 0) wetb[4ull * sc + wid] = (uint8_t)bits;
                    continue;
                }
                light_probe<T>(x, idx, b);
    #pragma unroll
                for (int u = 0; u < U; ++u) {
                    const bool ok = base + (uint32_t)u * kBlock + tid < x.nl;
                    const bool wet = x.rain_rate != 0.0 || wave_any(ok && !b.dry[u]);
                    const bool skip = light_history<T>(x, ok, b.m[u], b.c[u], !wet, b.e[u]);
                    if (wet) bits |= 1u << u;
                    else if (ok) fv1_dry_write<T>(x, b.m[u], b.c[u], b.h[u], acc, !skip);
                }
            }
            if ((tid & (kWave - 1)) == 0) wetb[4ull * sc + wid] = (uint8_t)bits;
        }
        if (cs >= 0) acc_flush(acc, red, rec[cs]);
        __syncthreads();   // cpre is rewritten by the next kind's schedule
    }
    // records of the problems that are stepping
    for (int q = tid; q < n * kPartial; q += kBlock) {
        const int s = q / kPartial;
        if (mine[s])
            descs[s].partials[(uint64_t)blockIdx.x * kPartial + q % kPartial] =
                rec[s][q % kPartial];
    }
}

// FV1, heavy kernel: the full update of the wave-chunks the light kernel
// marked wet.  It runs with its own (smaller, fully resident) grid on the
// same segment scheme; each wave reads the wet words of up to 64 of its
// workgroup's super-chunks at once (one per lane), so that a workgroup with
// no wet super-chunk costs one round trip.  Every wave of a workgroup reads
// the same words and so visits the same super-chunks, in ascending order.
// Records go to slots [rec0, rec0 + gridDim.x).
// FP32 is held to four waves per SIMD (128 VGPRs, none spilled); FP64 stays
// at three (158 VGPRs: held to four it spills 16 to scratch, whose traffic
// takes back most of what the fourth wave gains).
template <typename T>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 ? 4 : 1)))
void k_fv1_heavy(const Desc* __restrict__ descs, int n, uint32_t rec0)
{
    constexpr uint32_t SC = kLeafBatch * kBlock;
    // (no LDS records per problem: a workgroup visits the problems in
    // ascending order, each once, and writes each record when it leaves
    // that problem, so the LDS fits four workgroups per CU)
    __shared__ uint32_t cpre[kMaxScen + 1];
    __shared__ double red[kBlock / kWave][kPartial];
    __shared__ double rxy[2 * (HW_MAX_L + 1)];
    __shared__ const uint8_t* wtab[kMaxScen];
    __shared__ uint32_t cblk[kMaxScen];
    __shared__ BlockLds<T> blds[kBlock / kWave];
    const BlockConst kc = block_const();
    const int tid = threadIdx.x;
    const int wid = tid / kWave;
    const int lane = tid & (kWave - 1);
    const uint64_t slot = ((uint64_t)rec0 + blockIdx.x) * kPartial;
    uint64_t touched = 0;   // problems whose record this workgroup wrote
    if (tid < n) wtab[tid] = descs[tid].wet;
    // ends with a barrier
    const Fv1Sched f = fv1_schedule(descs, n, cpre, kAllProblems, nullptr, nullptr, cblk);
    const uint32_t K = f.c_begin < f.c_end ? (f.c_end - f.c_begin + f.g8 - 1) / f.g8 : 0u;
    Acc acc;
    acc_reset(acc);
    int cs = -1;
    Fv1Ctx<T> x;
    uint32_t c0 = 0, c1 = 0;
    for (uint32_t k0 = 0; k0 < K; k0 += kWave) {
        uint32_t word = 0;
        const uint32_t kl = k0 + (uint32_t)lane;
        if (kl < K) {
            const uint32_t ch = f.c_begin + kl * f.g8;
            int lo = 0, hi = n - 1;
            while (lo < hi) {
                const int mid = (lo + hi + 1) >> 1;
                if (cpre[mid] <= ch) lo = mid;
                else hi = mid - 1;
            }
            const uint32_t sc = chunk_order(ch - cpre[lo], cblk[lo], cpre[lo + 1] - cpre[lo]);
            word = *reinterpret_cast<gp<const uint32_t>>(glob(wtab[lo]) + 4ull * sc);
        }
        uint64_t mask = __ballot(word != 0u);
        while (mask) {
            const int j = __builtin_ctzll(mask);
            mask &= mask - 1;
            const uint32_t wj = (uint32_t)__builtin_amdgcn_readlane((int)word, j);
            const uint32_t ch = f.c_begin + (k0 + (uint32_t)j) * f.g8;
            if (cs < 0 || ch >= c1) {
                int s = cs < 0 ? 0 : cs;
                while (cpre[s + 1] <= ch) ++s;
                s = uniform(s);
                if (cs >= 0) acc_flush_store(acc, red, glob(descs[cs].partials) + slot);
                cs = s;
                touched |= 1ull << s;
                make_ctx<T>(x, descs[s]);
                fill_rxy(rxy, descs[s], x.dt);
                __syncthreads();
                x.rxy = rxy;
                c0 = uniform(cpre[s]);
                c1 = uniform(cpre[s + 1]);
            }
            // The marked sub-chunks of this super-chunk (bit u of byte w: the
            // 64 leaves base + u kBlock + w kWave + lane) are dealt to the
            // workgroup's waves in turn, whichever wave's position they hold.
            const uint32_t base = chunk_order(ch - c0, cblk[cs], c1 - c0) * SC;
            const bool finest = (uint64_t)x.nl == (1ull << (2 * x.L));
            const uint32_t fin_off = (uint32_t)level_off(x.L);
            const uint32_t lane_mask = (1u << kLeafBatch) - 1u;
            uint32_t items = 0;   // bit 4 w + u
#pragma unroll
            for (int w = 0; w < kBlock / kWave; ++w)
                items |= ((wj >> (8 * w)) & lane_mask) << (kLeafBatch * w);
            items = uniform(items);
            // first list entries of the super-chunk's sub-chunks that lie in
            // the block region (lane kLeafBatch w + u: sub-chunk u of wave
            // position w), one load for all of them
            uint32_t lfv = 0u;
            if (!finest && base < x.nb64 && lane < kLeafBatch * (kBlock / kWave)) {
                const uint32_t p = base + (uint32_t)(lane % kLeafBatch) * kBlock +
                                   (uint32_t)(lane / kLeafBatch) * kWave;
                if (p < x.nb64) lfv = ld_off(x.leaves, p * 4u);
            }
            int k = 0;
#pragma unroll 1
            while (items) {
                const int bit = __builtin_ctz(items);
                items &= items - 1u;
                if ((k++ & (kBlock / kWave - 1)) != wid) continue;
                const uint32_t w = (uint32_t)bit / kLeafBatch, u = (uint32_t)bit % kLeafBatch;
                const uint32_t leaf = base + u * kBlock + w * kWave + (uint32_t)lane;
                // the wave's first list entry
                const uint32_t p0 = base + u * kBlock + w * kWave;
                // a whole finest block at the head of a block-first list
                // (its first cell aligned, as the traversal writes it)
                const uint32_t lf = (uint32_t)__builtin_amdgcn_readlane((int)lfv, bit);
                const bool blk = !finest && p0 < x.nb64 && lf >= fin_off &&
                                 ((lf - fin_off) & 63u) == 0u;
                if (finest && x.L >= 3) {
                    // one aligned 8 x 8 block of finest leaves per wave
                    if (p0 < x.nl) fv1_block<T, false>(x, p0, acc, blds[wid], kc);
                } else if (blk) {
                    fv1_block<T, true>(x, lf - fin_off, acc, blds[wid], kc);
                } else if (leaf < x.nl) {
                    if (finest) fv1_leaf<T, true>(x, fin_off + leaf, acc);
                    else fv1_leaf<T, false>(x, x.leaves[leaf], acc);
                }
            }
        }
    }
    if (cs >= 0) acc_flush_store(acc, red, glob(descs[cs].partials) + slot);
    // zero records for the problems this workgroup had no chunk of
    for (int q = tid; q < n * kPartial; q += kBlock) {
        const int s = q / kPartial;
        if (!((touched >> s) & 1ull)) descs[s].partials[slot + q % kPartial] = 0.0;
    }
}

// Copy-down for leaves coarser than the traversal groups: every group below
// such a leaf takes the leaf's new value from its first finest descendant.
// Each lane reads its group's source; the wave then writes the cells of its
// 64 groups with consecutive lanes on consecutive cells (the group data go
// through the wave's slice of LDS).
template <typename T>
__device__ inline void fill_block(const Launch& lc, uint32_t vb)
{
    __shared__ uint32_t s_src[kBlock];
    __shared__ uint64_t s_f0[kBlock];
    __shared__ T s_val[3][kBlock];
    uint32_t lb;
    const int s = scen_of(lc, vb, lb);
    const Desc& d = lc.descs[s];
    const hw_scalars* sc = d.scal;
    if (sc->acc[STEP_DONE] != 0.0) return;
    if (sc->n_leaves == (1ull << (2 * d.L))) return;   // no coarser leaf at all
    const int L = d.L, Lg = d.group_level;
    const uint32_t tid = threadIdx.x;
    const uint32_t lane = tid & (kWave - 1u), w0 = tid & ~(kWave - 1u);
    const uint32_t g = lb * kBlock + tid;
    const int o = uniform((int)sc->acc[STEP_CUR]) ^ 1;
    gp<T> a[3];
#pragma unroll
    for (int v = 0; v < 3; ++v) a[v] = glob(reinterpret_cast<T*>(d.fine[o][v]));
    uint32_t src = kNone;
    if (g < (1u << (2 * Lg))) src = glob(d.big_src)[g];
    uint64_t f0 = 0;
    T val[3] = {T(0), T(0), T(0)};
    if (src != kNone) {
        const int n = level_of(src);
        f0 = (uint64_t)(src - (uint32_t)level_off(n)) << (2 * (L - n));
#pragma unroll
        for (int v = 0; v < 3; ++v) val[v] = a[v][f0];
    }
    if (!wave_any(src != kNone)) return;   // no group of this wave to fill
    s_src[tid] = src;
    s_f0[tid] = f0;
#pragma unroll
    for (int v = 0; v < 3; ++v) s_val[v][tid] = val[v];
    __builtin_amdgcn_wave_barrier();
    const int sh = 2 * (L - Lg);                      // log2 of cells per group
    const uint64_t first = (uint64_t)(g - lane) << sh;  // first cell of the wave's groups
    // The wave's groups are one span; under one leaf at level <= L-5 only
    // groups 0, 16, 32 and 48 are written (what the next encoding reads).
    const uint32_t src0 = uniform(s_src[w0]);
    if (sparse_fine(d) && src0 != kNone && level_of(src0) <= L - 5) {
        const uint32_t q = w0 + 16u * (lane >> 4);
        const uint64_t cell = first + 256u * (lane >> 4) + (lane & 15u);
        if (cell != s_f0[q]) {
#pragma unroll
            for (int v = 0; v < 3; ++v) a[v][cell] = s_val[v][q];
        }
        return;
    }
    for (uint32_t c = lane; c < (kWave << sh); c += kWave) {
        const uint32_t q = w0 + (c >> sh);
        const uint32_t sq = s_src[q];
        const uint64_t cell = first + c;
        if (sq != kNone && cell != s_f0[q]) {
#pragma unroll
            for (int v = 0; v < 3; ++v) a[v][cell] = s_val[v][q];
        }
    }
}

// One workgroup per problem: combine the FV1 partial records, then advance
// t, choose the next CFL timestep (capped at dt_max, shortened to hit
// t_end), update s_max, mass and counters, and flip the finest set.  Four
// waves: with about 1800 records a larger workgroup costs more to start
// than its wider reduction saves (1024 threads: 4.5 us more per step).
constexpr int kFinalBlock = 256;

// (always inlined: called from two kernels, it would otherwise become a
// call, and the call's register convention sets the copy-down's occupancy)
__device__ __attribute__((always_inline)) inline void finalize_problem(
    const Desc& d, int fv1_grid, double (*red)[kPartial], double* tot)
{
    const gp<hw_scalars> sc = glob(d.scal);
    // Every value this kernel reads is requested before any is used: the
    // scalars, and the records (four per thread and round; a record past the
    // end reads as zeros, the identity of every slot).  A finished problem
    // still reads them and writes nothing.
    const uint32_t done = sc->done;
    const double t = sc->t, dt = sc->dt;
    const uint64_t step = sc->step;
    const uint32_t map_step = sc->map_step;
    Acc a;
    acc_reset(a);
    const gp<const vd2> pr = reinterpret_cast<gp<const vd2>>(glob(d.partials));
    for (int b0 = threadIdx.x; b0 < fv1_grid; b0 += 4 * blockDim.x) {
        vd2 r[4][kPartial / 2];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int b = b0 + k * (int)blockDim.x;
            const int bc = b < fv1_grid ? b : fv1_grid - 1;
#pragma unroll
            for (int q = 0; q < kPartial / 2; ++q) r[k][q] = pr[(uint64_t)bc * (kPartial / 2) + q];
        }
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const bool ok = b0 + k * (int)blockDim.x < fv1_grid;
            double v[kPartial];
#pragma unroll
            for (int q = 0; q < kPartial / 2; ++q) {
                v[2 * q] = ok ? r[k][q].x : 0.0;
                v[2 * q + 1] = ok ? r[k][q].y : 0.0;
            }
            acc_add_record(a, v);
        }
    }
    if (threadIdx.x < kPartial) tot[threadIdx.x] = 0.0;
    __syncthreads();
    acc_flush(a, red, tot);
    if (threadIdx.x == 0 && !done) {
        const double tn = t + dt;
        const double ms = tot[0];
        const double dmin = d.dx < d.dy ? d.dx : d.dy;
        double dtn;
        if (ms > 0.0) {
            dtn = d.cfl * dmin / ms;
            dtn = dtn < d.dt_max ? dtn : d.dt_max;
        } else {
            dtn = d.dt_max;
        }
        const double rest = d.t_end - tn;
        dtn = dtn < rest ? dtn : rest;
        sc->t = tn;
        sc->dt = dtn;
        sc->maxspeed = ms;
        sc->mass = tot[4];
        sc->smax[0] = tot[1] > 1.0 ? tot[1] : 1.0;
        sc->smax[1] = tot[2] > 1.0 ? tot[2] : 1.0;
        sc->smax[2] = tot[3] > 1.0 ? tot[3] : 1.0;
        sc->step = step + 1;
        const uint64_t nl = d.uniform ? (1ull << (2 * d.L)) : sc->n_leaves;
        sc->n_leaves = nl;
        // The traversal of this step wrote the leaf-level map (the cases in
        // which its emit pass runs): the map describes the tree whose
        // copy-down made the set the next step reads.
        const bool stale = sparse_fine(d) && step > 0 && map_step == (uint32_t)step;
        if (!d.uniform && (d.full_outputs || nl < (1ull << (2 * d.L)) || stale))
            sc->map_step = (uint32_t)(step + 1);
        sc->leaf_updates += nl;
        sc->clips += (uint64_t)tot[5];
        sc->dry_stored += (uint64_t)tot[8];
        sc->dry_skipped += (uint64_t)tot[9];
        if (tot[6] > 0.0 || !isfinite(ms)) sc->nonfinite |= 1u;
        sc->cur ^= 1u;
        sc->done = (tn < d.t_end) ? 0u : 1u;
    }
}

__global__ __launch_bounds__(kFinalBlock) void k_finalize(const Desc* descs, int fv1_grid)
{
    __shared__ double red[kFinalBlock / kWave][kPartial];
    __shared__ double tot[kPartial];
    finalize_problem(descs[blockIdx.x], fv1_grid, red, tot);
}

// The copy-down and the finalisation in one launch: the first n workgroups
// finalise one problem each (dispatched first: the finalisation is the
// longer chain), the others fill.  The fill reads the finest set and the
// done flag from the step's snapshot (STEP_CUR, STEP_DONE, taken by the
// light FV1 kernel), not from cur and done, which the finalising
// workgroups update in the same launch.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_fill_finalize(Launch lc, uint32_t fill_blocks,
                                                          int fv1_grid)
{
    static_assert(kFinalBlock == kBlock, "one workgroup size for both parts");
    __shared__ double red[kFinalBlock / kWave][kPartial];
    __shared__ double tot[kPartial];
    const uint32_t nf = (uint32_t)lc.n;
    if (blockIdx.x < nf) {
        finalize_problem(lc.descs[blockIdx.x], fv1_grid, red, tot);
        return;
    }
    fill_block<T>(lc, blockIdx.x - nf);
}

// ---------------------------------------------------------------------------
// Ingest: row-major FP64 inputs -> Morton finest set 0 and finest bed level,
// with partial maxima, wave speed and mass for the scalars.
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(kBlock) void k_ingest(const Desc* dd,
                                                   const double* h,
                                                   const double* qx,
                                                   const double* qy,
                                                   const double* z)
{
    __shared__ double red[kBlock / kWave][kPartial];
    __shared__ double rec[kPartial];
    const Desc& d = *dd;
    const int L = d.L;
    const uint64_t N = 1ull << (2 * L);
    const uint32_t S = 1u << L;
    const T g = (T)d.g, tol = (T)d.h_tol;
    T* fh = reinterpret_cast<T*>(d.fine[0][0]);
    T* fqx = reinterpret_cast<T*>(d.fine[0][1]);
    T* fqy = reinterpret_cast<T*>(d.fine[0][2]);
    double* zl = d.zhier + level_off(L);
    Acc a;
    acc_reset(a);
    for (uint64_t f = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; f < N;
         f += (uint64_t)gridDim.x * blockDim.x) {
        const uint32_t i = compact1by1((uint32_t)f), j = compact1by1((uint32_t)f >> 1);
        const uint64_t r = (uint64_t)j * S + i;
        const double hv = h[r], xv = qx[r], yv = qy[r], zv = z[r];
        if (!(hv >= 0.0) || !isfinite(hv) || !isfinite(xv) || !isfinite(yv) ||
            !isfinite(zv))
            a.v[6] = 2.0;
        const T th = (T)hv, tx = (T)xv, ty = (T)yv;
        fh[f] = th;
        fqx[f] = tx;
        fqy[f] = ty;
        zl[f] = zv;
        acc_max(a, 0, wave_speed<T>(th, tx, ty, inv_depth(th, (T)tol), g, tol));
        acc_max(a, 1, fabs((double)th));
        acc_max(a, 2, fabs((double)tx));
        acc_max(a, 3, fabs((double)ty));
        a.v[4] += ((double)th * d.dx) * d.dy;
        acc_max(a, 7, fabs(zv));
    }
    if (threadIdx.x < kPartial) rec[threadIdx.x] = 0.0;
    __syncthreads();
    acc_flush(a, red, rec);
    if (threadIdx.x < kPartial)
        d.partials[(uint64_t)blockIdx.x * kPartial + threadIdx.x] = rec[threadIdx.x];
}

__global__ __launch_bounds__(kBlock) void k_ingest_final(const Desc* dd, int grid)
{
    __shared__ double red[kBlock / kWave][kPartial];
    __shared__ double tot[kPartial];
    const Desc& d = *dd;
    hw_scalars* sc = d.scal;
    Acc a;
    acc_reset(a);
    for (int b = threadIdx.x; b < grid; b += blockDim.x)
        acc_add_record(a, d.partials + (uint64_t)b * kPartial);
    if (threadIdx.x < kPartial) tot[threadIdx.x] = 0.0;
    __syncthreads();
    acc_flush(a, red, tot);
    if (threadIdx.x == 0) {
        const double ms = tot[0];
        const double dmin = d.dx < d.dy ? d.dx : d.dy;
        double dt;
        if (ms > 0.0) {
            dt = d.cfl * dmin / ms;
            dt = dt < d.dt_max ? dt : d.dt_max;
        } else {
            dt = d.dt_max;
        }
        const double rest = d.t_end - 0.0;
        dt = dt < rest ? dt : rest;
        sc->t = 0.0;
        sc->dt = dt;
        sc->mass = tot[4];
        sc->mass0 = tot[4];
        sc->smax[0] = tot[1] > 1.0 ? tot[1] : 1.0;
        sc->smax[1] = tot[2] > 1.0 ? tot[2] : 1.0;
        sc->smax[2] = tot[3] > 1.0 ? tot[3] : 1.0;
        sc->smax[3] = d.zsmax > 0.0 ? d.zsmax : (tot[7] > 1.0 ? tot[7] : 1.0);
        sc->maxspeed = ms;
        for (int q = 0; q < 6; ++q) sc->acc[q] = 0.0;
        sc->step = 0;
        sc->n_leaves = 0;
        sc->leaf_updates = 0;
        sc->clips = 0;
        sc->dry_stored = 0;
        sc->dry_skipped = 0;
        sc->cur = 0;
        sc->done = (0.0 < d.t_end) ? 0u : 1u;
        sc->nonfinite = tot[6] > 0.0 ? 2u : 0u;
        sc->map_step = 0;
    }
}

// Current finest set -> row-major FP64.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_export(const Desc* dd, double* h,
                                                   double* qx, double* qy)
{
    const Desc& d = *dd;
    const int L = d.L;
    const uint64_t N = 1ull << (2 * L);
    const uint32_t S = 1u << L;
    const int cur = (int)d.scal->cur;
    for (uint64_t r = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; r < N;
         r += (uint64_t)gridDim.x * blockDim.x) {
        const uint32_t i = (uint32_t)(r % S), j = (uint32_t)(r / S);
        const uint32_t f = morton(i, j);
        if (h) h[r] = (double)reinterpret_cast<const T*>(d.fine[cur][0])[f];
        if (qx) qx[r] = (double)reinterpret_cast<const T*>(d.fine[cur][1])[f];
        if (qy) qy[r] = (double)reinterpret_cast<const T*>(d.fine[cur][2])[f];
    }
}

// ---------------------------------------------------------------------------
// host-side launchers (used by the C ABI layer)
// ---------------------------------------------------------------------------

hipError_t launch_set_desc(const Desc& d, Desc* dst, hipStream_t s)
{
    hipLaunchKernelGGL(k_set_desc, dim3(1), dim3(64), 0, s, d, dst);
    return hipGetLastError();
}

hipError_t launch_ingest(int prec, const Desc* dd, uint32_t grid,
                         const double* h, const double* qx, const double* qy,
                         const double* z, hipStream_t s)
{
    if (prec == HW_FP64)
        hipLaunchKernelGGL(k_ingest<double>, dim3(grid), dim3(kBlock), 0, s, dd, h, qx, qy, z);
    else
        hipLaunchKernelGGL(k_ingest<float>, dim3(grid), dim3(kBlock), 0, s, dd, h, qx, qy, z);
    hipLaunchKernelGGL(k_ingest_final, dim3(1), dim3(kBlock), 0, s, dd, (int)grid);
    return hipGetLastError();
}

hipError_t launch_encode_bed(Launch lc, uint32_t nblocks, int pass, int tl,
                             int cpt, hipStream_t s)
{
    if (cpt == 2)
        hipLaunchKernelGGL((k_encode<double, 1, false, false, 2>), dim3(nblocks),
                           dim3(kBlock), 0, s, lc, pass, tl, (double*)nullptr);
    else
        hipLaunchKernelGGL((k_encode<double, 1, false, false, 1>), dim3(nblocks),
                           dim3(kBlock), 0, s, lc, pass, tl, (double*)nullptr);
    return hipGetLastError();
}

template <typename T, bool DET>
static void encode_flow_t(Launch lc, uint32_t nblocks, int pass, int tl, int cpt,
                          bool skip, double* details, hipStream_t s)
{
    // the span skip exists in the first pass of plans that allow it only
    if (skip && !DET && pass == 0) {
        if (cpt == 2)
            hipLaunchKernelGGL((k_encode<T, 3, true, false, 2, true>), dim3(nblocks), dim3(kBlock),
                               0, s, lc, pass, tl, details);
        else
            hipLaunchKernelGGL((k_encode<T, 3, true, false, 1, true>), dim3(nblocks), dim3(kBlock),
                               0, s, lc, pass, tl, details);
    } else if (cpt == 2) {
        hipLaunchKernelGGL((k_encode<T, 3, true, DET, 2>), dim3(nblocks), dim3(kBlock), 0, s,
                           lc, pass, tl, details);
    } else {
        hipLaunchKernelGGL((k_encode<T, 3, true, DET, 1>), dim3(nblocks), dim3(kBlock), 0, s,
                           lc, pass, tl, details);
    }
}

// tiles > 1: the multi-tile form of the first pass (nblocks = the tiles /
// tiles; one problem, four cells per thread, no span skip, no detail
// output; tiles 2 or 4).
hipError_t launch_encode_flow(int prec, Launch lc, uint32_t nblocks, int pass,
                              int tl, int cpt, bool skip, double* details, hipStream_t s,
                              int tiles)
{
    if (tiles > 1) {
        if (pass != 0 || cpt != 1 || skip || details || lc.n != 1 || (tiles != 2 && tiles != 4))
            return hipErrorInvalidValue;
        if (prec == HW_FP64) {
            if (tiles == 2)
                hipLaunchKernelGGL((k_encode<double, 3, true, false, 1, false, 2>),
                                   dim3(nblocks), dim3(kBlock), 0, s, lc, pass, tl, details);
            else
                hipLaunchKernelGGL((k_encode<double, 3, true, false, 1, false, 4>),
                                   dim3(nblocks), dim3(kBlock), 0, s, lc, pass, tl, details);
        } else if (tiles == 2) {
            hipLaunchKernelGGL((k_encode<float, 3, true, false, 1, false, 2>), dim3(nblocks),
                               dim3(kBlock), 0, s, lc, pass, tl, details);
        } else {
            hipLaunchKernelGGL((k_encode<float, 3, true, false, 1, false, 4>), dim3(nblocks),
                               dim3(kBlock), 0, s, lc, pass, tl, details);
        }
        return hipGetLastError();
    }
    if (prec == HW_FP64) {
        if (details) encode_flow_t<double, true>(lc, nblocks, pass, tl, cpt, skip, details, s);
        else encode_flow_t<double, false>(lc, nblocks, pass, tl, cpt, skip, details, s);
    } else {
        if (details) encode_flow_t<float, true>(lc, nblocks, pass, tl, cpt, skip, details, s);
        else encode_flow_t<float, false>(lc, nblocks, pass, tl, cpt, skip, details, s);
    }
    return hipGetLastError();
}

hipError_t launch_flag_only(int prec, Launch lc, uint32_t nblocks, hipStream_t s)
{
    if (prec == HW_FP64)
        hipLaunchKernelGGL(k_flag_only<double>, dim3(nblocks), dim3(kBlock), 0, s, lc);
    else
        hipLaunchKernelGGL(k_flag_only<float>, dim3(nblocks), dim3(kBlock), 0, s, lc);
    return hipGetLastError();
}

hipError_t launch_regularise(Launch lc, uint32_t nblocks, int fold_pass, int tl, hipStream_t s)
{
    hipLaunchKernelGGL(k_regularise, dim3(nblocks), dim3(kBlock), 0, s, lc, fold_pass, tl);
    return hipGetLastError();
}

hipError_t launch_traverse(Launch lc, uint32_t nblocks, hipStream_t s)
{
    hipLaunchKernelGGL(k_traverse<false>, dim3(nblocks), dim3(kBlock), 0, s, lc);
    hipLaunchKernelGGL(k_trav_scan, dim3(lc.n), dim3(1024), 0, s, lc.descs);
    hipLaunchKernelGGL(k_traverse<true>, dim3(nblocks), dim3(kBlock), 0, s, lc);
    return hipGetLastError();
}

// Workgroups of the heavy FV1 kernel: about as many as are resident at its
// occupancy, never more than the light kernel's: four waves per SIMD for
// FP32, three for FP64.
uint32_t heavy_grid(int prec, uint32_t grid)
{
    const uint32_t cap = prec == HW_FP64 ? 768u : 1024u;
    return grid < cap ? grid : cap;
}

// The heavy FV1 kernel alone (after the light kernel of the same step: it
// reads the wet table and writes only the other set and its own records).
hipError_t launch_fv1_heavy(int prec, const Desc* descs, int n, uint32_t grid, hipStream_t s)
{
    const uint32_t gh = heavy_grid(prec, grid);
    if (prec == HW_FP64)
        hipLaunchKernelGGL(k_fv1_heavy<double>, dim3(gh), dim3(kBlock), 0, s, descs, n, grid);
    else
        hipLaunchKernelGGL(k_fv1_heavy<float>, dim3(gh), dim3(kBlock), 0, s, descs, n, grid);
    return hipGetLastError();
}

// The light and the heavy FV1 kernels.
hipError_t launch_fv1_only(int prec, const Desc* descs, int n, uint32_t grid, hipStream_t s)
{
    if (prec == HW_FP64)
        hipLaunchKernelGGL(k_fv1_light<double>, dim3(grid), dim3(kBlock), 0, s, descs, n);
    else
        hipLaunchKernelGGL(k_fv1_light<float>, dim3(grid), dim3(kBlock), 0, s, descs, n);
    const hipError_t e = hipGetLastError();
    return e != hipSuccess ? e : launch_fv1_heavy(prec, descs, n, grid, s);
}

// Copy-down and finalisation of the step (fill.n problems, FV1 grid grid).
hipError_t launch_fill(int prec, Launch fill, uint32_t fill_blocks, uint32_t grid,
                       hipStream_t s)
{
    const dim3 blocks(fill_blocks + (uint32_t)fill.n);
    const int records = (int)(grid + heavy_grid(prec, grid));
    if (prec == HW_FP64)
        hipLaunchKernelGGL(k_fill_finalize<double>, blocks, dim3(kBlock), 0, s, fill,
                           fill_blocks, records);
    else
        hipLaunchKernelGGL(k_fill_finalize<float>, blocks, dim3(kBlock), 0, s, fill,
                           fill_blocks, records);
    return hipGetLastError();
}

hipError_t launch_finalize(int prec, const Desc* descs, int n, uint32_t grid, hipStream_t s)
{
    hipLaunchKernelGGL(k_finalize, dim3(n), dim3(kFinalBlock), 0, s, descs,
                       (int)(grid + heavy_grid(prec, grid)));
    return hipGetLastError();
}

hipError_t launch_fv1(int prec, const Desc* descs, int n, uint32_t grid,
                      Launch fill, uint32_t fill_blocks, hipStream_t s)
{
    hipError_t e = launch_fv1_only(prec, descs, n, grid, s);
    if (e == hipSuccess) e = launch_fill(prec, fill, fill_blocks, grid, s);
    return e;
}

// Clears the FV1 write history of one problem (every entry then names no
// step, so the next two steps store everything).
// End of a run: every span of the current set that the last copy-down left
// stale (covered by one leaf of the last tree at level <= L-5) is made
// whole from its first cell.  One wave per span.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_densify(const Desc* dd)
{
    const Desc& d = *dd;
    const hw_scalars* sc = d.scal;
    if (!sparse_fine(d) || sc->step == 0 || sc->map_step != (uint32_t)sc->step) return;
    const uint64_t span = (uint64_t)blockIdx.x * (kBlock / kWave) + threadIdx.x / kWave;
    if (span >= (1ull << (2 * d.L - 10))) return;
    const uint64_t first = span << 10;
    if ((int)glob(static_cast<const uint8_t*>(d.lmap))[first] > d.L - 5) return;
    fill_span<T>(d, uniform((int)sc->cur), first);
}

__global__ __launch_bounds__(kBlock) void k_forget(const Desc* dd)
{
    const gp<uint64_t> hist = glob(dd->hist);
    const uint32_t n = dd->nhist;
    if (blockIdx.x == 0 && threadIdx.x == 0) glob(dd->scal)->map_step = 0u;
    for (uint32_t i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock)
        hist[i] = 0ull;
}

hipError_t launch_forget(const Desc* dd, uint64_t nhist, hipStream_t s)
{
    uint64_t blocks = (nhist + kBlock - 1) / kBlock;
    if (blocks > 1024) blocks = 1024;
    hipLaunchKernelGGL(k_forget, dim3((uint32_t)blocks), dim3(kBlock), 0, s, dd);
    return hipGetLastError();
}

hipError_t launch_densify(int prec, const Desc* dd, int L, hipStream_t s)
{
    if (L < 7) return hipSuccess;
    const uint32_t blocks = (uint32_t)(1ull << (2 * L - 12));   // four spans each
    if (prec == HW_FP64)
        hipLaunchKernelGGL(k_densify<double>, dim3(blocks), dim3(kBlock), 0, s, dd);
    else
        hipLaunchKernelGGL(k_densify<float>, dim3(blocks), dim3(kBlock), 0, s, dd);
    return hipGetLastError();
}

hipError_t launch_export(int prec, const Desc* dd, uint64_t N, double* h,
                         double* qx, double* qy, hipStream_t s)
{
    uint64_t blocks = (N + kBlock - 1) / kBlock;
    if (blocks > 65536) blocks = 65536;
    if (prec == HW_FP64)
        hipLaunchKernelGGL(k_export<double>, dim3((uint32_t)blocks), dim3(kBlock), 0, s, dd, h, qx, qy);
    else
        hipLaunchKernelGGL(k_export<float>, dim3((uint32_t)blocks), dim3(kBlock), 0, s, dd, h, qx, qy);
    return hipGetLastError();
}

}  // namespace hw
