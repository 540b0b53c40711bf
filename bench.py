#!/usr/bin/env python3
"""HWFV1 timestep benchmark on one MI355X.

Headline: timesteps/s of the plain FP64 path on the L = 12 hydrograph
workload (4096^2 finest cells, eps = 1e-3, seeded fractal bed, west-edge
inflow, Manning 0.035), inputs resident in HBM, the whole step (encoding,
flagging, traversal, FV1, fill, finalize) replayed as one HIP graph per step.
Beside it: the FP32-bulk form on the same workload (with its error against
the FP64 run), the batched 64-member ensemble, the roofline of the dominant
kernel (HIP-event phase timing) and the CPU oracle on a bounded sample.

Prints ONE JSON line on stdout; progress goes to stderr.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = ("HWFV1 timesteps/s at L=12, ε=1e-3: FP64 vs FP32-bulk vs batched; "
          "%HBM peak")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def leaf_level_hist(buffers, L):
    import numpy as np
    leaves = buffers.leaf_list().astype(np.int64)
    lvl = np.floor(np.log(3.0 * leaves + 1.0) / np.log(4.0) + 1e-9).astype(np.int64)
    return np.bincount(lvl, minlength=L + 1)


def phase_bytes(L, w, hist, dry=None, uniform=False, sparse=False, fv1_grid=2048, tl=5):
    """Algorithmic HBM bytes of one step per phase (w = bytes per flow word),
    counting only what the step's kernels move.

    encode    read h, qx, qy on the finest level, write the coarse levels
              0..L-2 (the time loop does not store level L-1: its values are
              recomputed from the finest level where needed), read the
              static bed flags, write the raw flags; for L >= 5 also write
              one flag byte and a (mass, max |h|) pair per 64-cell block
    regularise read raw flags (one per cell, neighbours cached), write sig
    traverse  count pass: read the flags of levels 0..L-1 once, write one
              walk code per 16-cell group and one count per workgroup; the
              emit pass runs only when some leaf is coarser than the finest
              level: read the walk codes, write the leaf list, the fill
              table (one word per group) and the leaf-level map (one byte
              per finest cell)
    fv1       general step: per leaf its index, own h, qx, qy and bed (FP64),
              and the finest cells it writes (all descendants for leaves at
              or below the traversal group level, one otherwise).  A step
              whose leaves are all finest, given dry = (stored, skipped) leaf
              updates of the dry pass per step: the full update reads h, qx,
              qy and z and writes h, qx, qy for the other leaves; a stored dry
              leaf reads h and writes h, qx, qy; a skipped one moves nothing;
              for L >= 5 every 64-cell block reads its flag byte, its history
              word and its (mass, max |h|) pair and writes the history word
              (neighbour flag bytes cached), and the wet table is written
    fill      only when some leaf is coarser than a group: read the fill
              table, write the finest cells of coarser leaves (with the
              tree-sparse set, `sparse`, 64 cells of each 1024-cell span
              below a leaf of level <= L-5); and, in the same launch, the
              finalisation: read the partial records of both FV1 kernels
              (80 B each)

    Two single launches are modelled on their own: encode_first_pass (the
    first of the encoding passes, levels L-1 .. L-tl: the finest read, the
    coarse levels it stores, its flags and the 64-cell block records) and
    fv1_heavy (the full updates: per fully updated leaf of an all-finest
    step h, qx, qy and z read and h, qx, qy written; in a general step the
    fv1 figure above less what the light kernel moves, its wet table).

    uniform FV1 plan (FV1 and finalize only): every finest cell reads its
    depth (neighbours cached); the full update reads h, qx, qy and z and
    writes h, qx, qy; a stored dry cell writes h, qx, qy; each 64-cell block
    reads and writes its history word; the wet table is written
    """
    N = 4 ** L
    Nc = (N - 1) // 3
    Lg = max(L - 2, 0)
    nl = int(hist.sum())
    all_finest = int(hist[L]) == N
    fv1_writes = 0
    fill_writes = 0
    for m, cnt in enumerate(hist):
        cnt = int(cnt)
        if m >= Lg:
            fv1_writes += cnt * 4 ** (L - m)
        else:
            fv1_writes += cnt
            if sparse and L >= 7 and m <= L - 5:
                fill_writes += cnt * (4 ** (L - 5 - m) * 64 - 1)
            else:
                fill_writes += cnt * (4 ** (L - m) - 1)
    groups = 4 ** Lg
    ntrav = (groups + 255) // 256
    blocks = N // 64 if L >= 5 else 0
    finalize = 2 * fv1_grid * 80
    if uniform:
        stored, skipped = dry
        full = N - stored - skipped
        fv1 = full * (3 * w + 8 + 3 * w) + stored * 4 * w + skipped * w \
            + (N // 64) * 16 + 4 * (N // 512)
        return {"encode": 0, "regularise": 0, "traverse": 0, "fv1": int(fv1), "fill": 0,
                "finalize": finalize, "n_leaves": N, "encode_first_pass": 0,
                "fv1_heavy": int(full * (3 * w + 8 + 3 * w))}
    fv1 = nl * (4 + 3 * w + 8) + 3 * w * fv1_writes
    heavy = fv1 - 4 * (N // 512)
    if dry is not None and all_finest:
        stored, skipped = dry
        full = N - stored - skipped
        fv1 = full * (3 * w + 8 + 3 * w) + stored * 4 * w + blocks * (1 + 8 + 16 + 8) \
            + 4 * (N // 512)
        heavy = full * (3 * w + 8 + 3 * w)
    lv = min(L, tl)
    first = 3 * w * N + 3 * w * sum(4 ** n for n in range(L - lv, L - 1)) \
        + 2 * sum(4 ** n for n in range(L - lv, L)) + blocks * (1 + 16)
    traverse = Nc + groups + 4 * ntrav
    fill = 0
    if not all_finest:
        traverse += groups + 4 * nl + 4 * groups + N
        fill = 4 * groups + 3 * w * fill_writes
    # the finalisation runs in the copy-down's launch (its phase time too)
    return {
        "encode": 3 * w * N + 3 * w * (Nc - 4 ** (L - 1)) + 2 * Nc + blocks * (1 + 16),
        "regularise": 2 * Nc,
        "traverse": traverse,
        "fv1": int(fv1),
        "fill": fill + finalize,
        "finalize": 0,
        "n_leaves": nl,
        "encode_first_pass": int(first),
        "fv1_heavy": int(heavy),
    }


def time_single(hw, w, precision, steps, warmup, prof_steps, tuning=None, uniform=False):
    import torch
    from paper_2206_05761_amd.autotune import autotune
    log(f"[bench] {w.name} {precision}: ingest")
    sim = hw.Simulation(w.params, w.h, w.qx, w.qy, w.z, precision=precision)
    if tuning is None:
        best, table = autotune([sim.problem], [sim.buffers], use_cache=False)
        log(f"[bench] {precision}: autotuned {best}")
    else:
        best, table = dict(tuning), None
        log(f"[bench] {precision}: fixed tuning {best}")
    plan = hw.Plan([sim.problem], [sim.buffers], tuning=best, uniform=uniform)
    hw.hwfv1_run(sim.problem, sim.buffers, warmup, plan=plan, stats=True)
    s0 = sim.scalars()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record()
    hw.hwfv1_run(sim.problem, sim.buffers, steps, plan=plan, stats=False)
    e1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = e0.elapsed_time(e1)
    s1 = sim.scalars()
    log(f"[bench] {precision}: {steps} steps in {ms:.2f} ms (wall {wall*1e3:.2f} ms), "
        f"t={s1['t']:.3f} s, leaves={s1['n_leaves']}")
    prof = hw.hw_plan_profile(plan, prof_steps)
    hist = leaf_level_hist(sim.buffers, w.L)
    s2 = sim.scalars()
    res = dict(sim=sim, plan=plan, ms=ms, wall=wall, steps=steps,
               leaf_updates=int(s1["leaf_updates"] - s0["leaf_updates"]),
               dry=((s1["dry_stored"] - s0["dry_stored"]) / steps,
                    (s1["dry_skipped"] - s0["dry_skipped"]) / steps),
               prof={k: prof[k] / prof_steps for k in hw.PHASES},
               kernel_ms={k: prof[k] / prof_steps for k in hw.PROF_KERNELS}, hist=hist,
               scalars=s2, tuning=best, tuning_table=table, uniform=uniform)
    return res


KERNEL_SOURCES = ["paper_2206_05761_amd/csrc/hw_kernels.hip",
                  "paper_2206_05761_amd/csrc/hw_device.h"]


def kernel_source_hash():
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def load_traffic(name):
    """Measured HBM bytes from a committed rocprofv3 counter summary
    profiles/<name>.txt: a dict of its key = value lines, or None when there
    is none or the kernel sources have changed since the counters were
    taken."""
    path = os.path.join(ROOT, "profiles", name + ".txt")
    if not os.path.exists(path):
        return None
    kv = {}
    with open(path) as fh:
        text = fh.read()
    for line in text.splitlines():
        if "=" in line and not line.lstrip().startswith("#"):
            k, v = line.split("=", 1)
            kv[k.strip()] = v.strip()
    if kv.get("source_sha256") != kernel_source_hash():
        return None
    return kv


def encode_levels_per_pass(tuning):
    """Levels per encoding pass of a tuning (one or two levels in registers,
    plus four in the workgroup's tile)."""
    return 6 if (tuning or {}).get("encode_cells_per_thread") == 16 else 5


# the single launch each phase's roofline is taken on (others: the phase)
PHASE_KERNEL = {"encode": "encode_first_pass", "fv1": "fv1_heavy"}
KERNEL_NAMES = {"encode_first_pass": "k_encode (first pass, finest level in)",
                "fv1_heavy": "k_fv1_heavy"}


def main_kernel(dom, phase_ms, kernel_ms):
    """The single launch the dominant phase's roofline is taken on: its
    main kernel when that takes at least half of the phase, else the phase
    (e.g. an FV1 phase of dry steps, where the light kernel dominates)."""
    k = PHASE_KERNEL.get(dom)
    if k and kernel_ms.get(k, 0) >= 0.5 * phase_ms[dom]:
        return k
    return dom


def roofline(res, L, w, precision=None, workload=None, sparse=False):
    """The dominant phase's main kernel against the HBM roof: its model bytes
    over its average launch time (HIP events around that launch alone for
    the first encoding pass and the heavy FV1 kernel, around the phase
    otherwise), its measured traffic when a current counter summary exists,
    and the whole step: model bytes of every phase over the sum of the phase
    times, and measured bytes per step over the same time when a current
    whole-step counter summary exists."""
    tuning = res.get("tuning") or {}
    grid = tuning.get("fv1_grid") or 2048
    pb = phase_bytes(L, w, res["hist"], res.get("dry"), res.get("uniform", False),
                     sparse=sparse, fv1_grid=grid, tl=encode_levels_per_pass(tuning))
    prof = {k: v for k, v in res["prof"].items() if v > 0}
    kms = res.get("kernel_ms") or {}
    dom = max((k for k in prof), key=lambda k: prof[k])
    kern = main_kernel(dom, prof, kms)
    if kern != dom:
        k_ms, k_bytes, k_name = kms[kern], pb[kern], KERNEL_NAMES[kern]
    else:
        k_ms, k_bytes, k_name = prof[dom], pb[dom], dom
    achieved = k_bytes / (k_ms * 1e-3) / 1e9
    # the whole step: its graph-replayed time (phase events add a few µs each)
    phases_ms = sum(prof.values())
    step_ms = res["ms"] / res["steps"]
    total_bytes = sum(pb[k] for k in prof)
    per_kernel = {k: {"ms": round(prof[k], 5), "model_bytes": int(pb[k]),
                      "GBs": round(pb[k] / (prof[k] * 1e-3) / 1e9, 1) if prof[k] > 0 else None}
                  for k in prof}
    for k, v in kms.items():
        if v > 0:
            per_kernel[k] = {"ms": round(v, 5), "model_bytes": int(pb[k]),
                             "GBs": round(pb[k] / (v * 1e-3) / 1e9, 1), "within": next(
                                 p for p, q in PHASE_KERNEL.items() if q == k)}
    traffic = None
    step_measured = None
    if precision and workload:
        kv = load_traffic(f"traffic_{kern}_{workload}_{precision}")
        if kv:
            traffic = int(float(kv["fetch_bytes_per_launch"]) + float(kv["write_bytes_per_launch"]))
        kv = load_traffic(f"traffic_step_{workload}_{precision}")
        if kv:
            mb = float(kv["fetch_bytes_per_step"]) + float(kv["write_bytes_per_step"])
            step_measured = {
                "bytes": int(mb),
                "frac": round(mb / (step_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                "model_over_measured": round(total_bytes / mb, 3),
                "source": f"profiles/traffic_step_{workload}_{precision}.txt",
            }
    return {
        "bound": "hbm", "kernel": k_name, "phase": dom, "achieved": round(achieved, 1),
        "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
        "traffic": traffic,
        "algorithmic_bytes": int(k_bytes),
        "avg_ms": round(k_ms, 5),
        "step": {"model_bytes": int(total_bytes), "ms": round(step_ms, 5),
                 "ms_phases": round(phases_ms, 5),
                 "frac": round(total_bytes / (step_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                 "measured": step_measured},
        "phases": per_kernel,
    }


def dry_split(res):
    """Per-step leaf updates of the timed run: full update, and the dry pass
    with stores written or skipped."""
    stored, skipped = res["dry"]
    per_step = res["leaf_updates"] / res["steps"]
    return {"full": round(per_step - stored - skipped, 1), "dry_stored": round(stored, 1),
            "dry_skipped": round(skipped, 1)}


def fp32_error(hw, r64, r32):
    import numpy as np
    a = [t.cpu().numpy() for t in hw.hw_export(r64["sim"].problem, r64["sim"].buffers)]
    b = [t.cpu().numpy() for t in hw.hw_export(r32["sim"].problem, r32["sim"].buffers)]
    la = set(r64["sim"].buffers.leaf_list().tolist())
    lb = set(r32["sim"].buffers.leaf_list().tolist())
    m64 = r64["scalars"]["mass"]
    m32 = r32["scalars"]["mass"]
    return {
        "l1_h": float(np.mean(np.abs(a[0] - b[0]))),
        "linf_h": float(np.max(np.abs(a[0] - b[0]))),
        "linf_qx": float(np.max(np.abs(a[1] - b[1]))),
        "linf_qy": float(np.max(np.abs(a[2] - b[2]))),
        "l1_qx": float(np.mean(np.abs(a[1] - b[1]))),
        "l1_qy": float(np.mean(np.abs(a[2] - b[2]))),
        "leaf_symdiff": len(la ^ lb),
        "mass_rel_err": (m32 - m64) / m64 if m64 else None,
        "vs": "FP64 GPU run of the same steps (equal to the oracle within 1e-10)",
    }


def bench_batch(hw, steps, warmup, n_members):
    import torch
    import workloads as W
    log(f"[bench] batch: generating {n_members} members")
    t0 = time.perf_counter()
    members = W.ensemble_64(n=n_members, n_steps=steps)
    log(f"[bench] batch: inputs in {time.perf_counter() - t0:.1f} s")
    sims = [hw.Simulation(m.params, m.h, m.qx, m.qy, m.z, precision="fp32_bulk")
            for m in members]
    cells = sum(4 ** m.L for m in members)
    from paper_2206_05761_amd.autotune import autotune
    best, table = autotune([s.problem for s in sims], [s.buffers for s in sims],
                           use_cache=False)
    log(f"[bench] batch: autotuned {best}")
    plan = hw.Plan([s.problem for s in sims], [s.buffers for s in sims], tuning=best)
    hw.hwfv1_run_batch(plan, warmup, stats=True)
    lu0 = sum(s.scalars()["leaf_updates"] for s in sims)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    hw.hwfv1_run_batch(plan, steps, stats=False)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    lu1 = sum(s.scalars()["leaf_updates"] for s in sims)
    s_mid = [s.scalars() for s in sims]
    prof = hw.hw_plan_profile(plan, 5)
    s_end = [s.scalars() for s in sims]
    pb = {}
    for m, sim, a, b in zip(members, sims, s_mid, s_end):
        hist = leaf_level_hist(sim.buffers, m.L)
        dry = ((b["dry_stored"] - a["dry_stored"]) / 5.0,
               (b["dry_skipped"] - a["dry_skipped"]) / 5.0)
        for k, v in phase_bytes(m.L, 4, hist, dry,
                                sparse=bool(best.get("encode_skip", 1) and best.get("fill_skip", 1)),
                                fv1_grid=best.get("fv1_grid") or 2048,
                                tl=encode_levels_per_pass(best)).items():
            if k != "n_leaves":
                pb[k] = pb.get(k, 0) + v
    pms = {k: prof[k] / 5 for k in hw.PHASES if prof[k] > 0}
    kms = {k: prof[k] / 5 for k in hw.PROF_KERNELS}
    dom = max(pms, key=lambda k: pms[k])
    kern = main_kernel(dom, pms, kms)
    k_ms = kms[kern] if kern != dom else pms[dom]
    achieved = pb[kern] / (k_ms * 1e-3) / 1e9
    phases_ms = sum(pms.values())
    step_ms = ms / steps
    step_bytes = sum(pb[k] for k in pms)
    levels = sorted(m.L for m in members)
    out = {
        "value": round(steps / (ms * 1e-3), 2), "unit": "ensemble timesteps/s",
        "member_steps_per_s": round(n_members * steps / (ms * 1e-3), 1),
        "leaf_updates_per_s": (lu1 - lu0) / (ms * 1e-3),
        "members": n_members, "finest_cells": cells, "steps": steps,
        "ms_per_step": round(ms / steps, 4), "dtype": "f32 (FP64 significance)",
        "levels": {str(L): levels.count(L) for L in sorted(set(levels))},
        "phase_ms": {k: round(v / 5, 4) for k, v in prof.items()},
        "roofline": {"bound": "hbm", "kernel": KERNEL_NAMES.get(kern, kern), "phase": dom,
                     "achieved": round(achieved, 1),
                     "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                     "algorithmic_bytes": int(pb[kern]), "avg_ms": round(k_ms, 5),
                     "step": {"model_bytes": int(step_bytes), "ms": round(step_ms, 5),
                              "ms_phases": round(phases_ms, 5),
                              "frac": round(step_bytes / (step_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)},
                     "note": "model bytes summed over the members (their leaf levels and "
                             "dry-pass counts after the timed steps), 5 profiled steps"},
        "tuning": best, "autotune_ms_per_step": table,
    }
    plan.close()
    for s in sims:
        s.close()
    return out


def run_to_end_ms(hw, w, uniform, tuning=None):
    """Milliseconds (HIP events) of a FP64 run from the workload's initial
    state to its t_end, on a plan that has already been captured: a first
    run counts the steps, the state is ingested again and exactly that many
    steps are timed."""
    import numpy as np
    import torch
    sim = hw.Simulation(w.params, w.h, w.qx, w.qy, w.z, precision="fp64")
    plan = hw.Plan([sim.problem], [sim.buffers], tuning=tuning, uniform=uniform)
    st = hw.hwfv1_run(sim.problem, sim.buffers, 10 ** 7, plan=plan, stats=True)
    n = st["steps"]
    leaves = st["leaf_updates"] / max(n, 1)
    dev = [torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64).reshape(-1), device="cuda")
           for a in (w.h, w.qx, w.qy, w.z)]
    hw.hw_ingest(sim.problem, sim.buffers, *dev)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    hw.hwfv1_run(sim.problem, sim.buffers, n, plan=plan, stats=False)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    t = sim.scalars()["t"]
    plan.close()
    sim.close()
    return ms, n, leaves, t


def bench_speedup(hw, levels=(8, 9, 10, 11, 12), epss=(1e-4, 1e-3, 1e-2)):
    """Speed-up of HWFV1 over uniform FV1 to reach t = 3.5 s in the circular
    dam break (the paper's Fig. 12 configurations, and L = 12)."""
    import workloads as W
    rows = []
    for L in levels:
        um, un, _, _ = run_to_end_ms(hw, W.circular_dambreak_flat(L), True)
        for eps in epss:
            ms, n, leaves, t = run_to_end_ms(hw, W.circular_dambreak_flat(L, eps), False)
            row = {"L": L, "eps": eps, "steps": n, "hwfv1_ms": round(ms, 3),
                   "uniform_fv1_ms": round(um, 3), "speedup": round(um / ms, 3),
                   "mean_leaf_fraction": round(leaves / 4 ** L, 4)}
            if eps == 1e-3 and L >= 10:
                # the same run with every finest cell read and written each step
                dm, _, _, _ = run_to_end_ms(hw, W.circular_dambreak_flat(L, eps), False,
                                            tuning=dict(encode_skip=0, fill_skip=0))
                row["hwfv1_dense_ms"] = round(dm, 3)
                row["speedup_dense"] = round(um / dm, 3)
            rows.append(row)
            log(f"[bench] speed-up L={L} eps={eps}: {n} steps, HWFV1 {ms:.1f} ms, "
                f"uniform {um:.1f} ms ({un} steps), x{um / ms:.2f}, "
                f"leaves {leaves / 4 ** L:.3f}"
                + (f", dense HWFV1 {row['hwfv1_dense_ms']:.1f} ms" if "hwfv1_dense_ms" in row else ""))
    return {"workload": "circular_dambreak_flat (closed 40 m square, flat, frictionless, "
                        "2.5 m / 0.5 m, dam radius 2.5 m off-centre by (1.3, 0.7) m, to t = 3.5 s)",
            "precision": "fp64", "unit": "ms to t_end (HIP events)",
            "note": "hwfv1_ms with the default plan (tree-sparse finest set: encode_skip, "
                    "fill_skip); hwfv1_dense_ms with both off",
            "rows": rows}


def run_history_ms(hw, w, uniform, chunk):
    """(t, elapsed ms) after every `chunk` steps of a FP64 run from the
    initial state to t_end (HIP events; the plan is captured beforehand)."""
    import numpy as np
    import torch
    sim = hw.Simulation(w.params, w.h, w.qx, w.qy, w.z, precision="fp64")
    plan = hw.Plan([sim.problem], [sim.buffers], uniform=uniform)
    hw.hwfv1_run(sim.problem, sim.buffers, 1, plan=plan, stats=False)
    dev = [torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64).reshape(-1), device="cuda")
           for a in (w.h, w.qx, w.qy, w.z)]
    hw.hw_ingest(sim.problem, sim.buffers, *dev)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e0.record()
    hist = [(0.0, 0.0)]
    while True:
        hw.hwfv1_run(sim.problem, sim.buffers, chunk, plan=plan, stats=False)
        e1 = torch.cuda.Event(enable_timing=True)
        e1.record()
        s = sim.scalars()
        hist.append((s["t"], e0.elapsed_time(e1)))
        if s["done"]:
            break
    steps = sim.scalars()["step"]
    plan.close()
    sim.close()
    return hist, steps


def bench_verification(hw):
    """Section 3.1's cases on the hump shapes of workloads.humps_lake_at_rest
    (FP64, L = 8, eps = 1e-3): the largest discharge over 100 s of still
    water per profile (well-balancedness), and the frictional dam break's
    mean absolute depth difference from uniform FV1 over the basin."""
    import numpy as np
    import workloads as W
    out = {"lake_at_rest_max_discharge": {}, "humps_dambreak_l1_vs_uniform_m": {}}
    for prof in ("smooth", "steeper", "rectangular"):
        w = W.humps_lake_at_rest(prof)
        sim = hw.Simulation(w.params, w.h, w.qx, w.qy, w.z)
        worst = 0.0
        while sim.scalars()["t"] < w.params["t_end"]:
            sim.run(500, stats=False)
            _, qx, qy = sim.export()
            worst = max(worst, float(np.abs(qx).max()), float(np.abs(qy).max()))
        out["lake_at_rest_max_discharge"][prof] = worst
        sim.close()
    for t_end in (6.0, 12.0):
        w = W.humps_dambreak(t_end=t_end)
        rows = w.meta["basin_rows"]
        hs = []
        for uniform in (False, True):
            sim = hw.Simulation(w.params, w.h, w.qx, w.qy, w.z)
            plan = hw.Plan([sim.problem], [sim.buffers], uniform=uniform)
            hw.hwfv1_run(sim.problem, sim.buffers, 100_000, plan=plan, stats=False)
            plan.close()
            hs.append(sim.export()[0][:rows])
            sim.close()
        out["humps_dambreak_l1_vs_uniform_m"][f"{t_end:g} s"] = float(np.abs(hs[0] - hs[1]).mean())
    out["note"] = ("hump shapes chosen to meet Table 3's wetting conditions (the paper only "
                   "draws them); the paper's own L1 differences (4.6e-4 m at 6 s, 9.2e-4 m "
                   "at 12 s) are context, not a target")
    log(f"[bench] verification: {out['lake_at_rest_max_discharge']}, "
        f"{out['humps_dambreak_l1_vs_uniform_m']}")
    return out


def bench_pseudo2d(hw, levels=(8, 9, 10, 11), epss=(1e-4, 1e-3, 1e-2), window=2.5, t_end=40.0):
    """Speed-up of HWFV1 over uniform FV1 through the 40 s pseudo-2D dam
    break, per window of simulated time (the paper's Fig. 14)."""
    import numpy as np
    import workloads as W
    marks = np.arange(0.0, t_end + 1e-9, window)

    def at(hist, t):
        ts, ms = zip(*hist)
        return float(np.interp(t, ts, ms))

    rows = []
    for L in levels:
        chunk = 32 << (L - 8)
        uh, un = run_history_ms(hw, W.pseudo2d_dambreak(L, t_end=t_end), True, chunk)
        u = [at(uh, t) for t in marks]
        for eps in epss:
            hh, hn = run_history_ms(hw, W.pseudo2d_dambreak(L, eps, t_end=t_end), False, chunk)
            h = [at(hh, t) for t in marks]
            win = [round((u[i + 1] - u[i]) / (h[i + 1] - h[i]), 3) for i in range(len(marks) - 1)]
            rows.append({"L": L, "eps": eps, "steps": hn, "hwfv1_ms": round(h[-1], 2),
                         "uniform_fv1_ms": round(u[-1], 2), "speedup": round(u[-1] / h[-1], 3),
                         "window_speedup": win})
            log(f"[bench] pseudo-2D L={L} eps={eps}: {hn} steps, HWFV1 {h[-1]:.0f} ms, "
                f"uniform {u[-1]:.0f} ms, x{u[-1] / h[-1]:.2f}; per {window} s: {win}")
    return {"workload": "pseudo2d_dambreak (flat, frictionless, 6 m | 2 m at x = 10 m, "
                        "50 m square, open ends, to t = 40 s)",
            "precision": "fp64", "window_s": window, "rows": rows}


def host_cpu():
    """Host CPU model and logical CPU count."""
    model = None
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"model": model, "nproc": os.cpu_count()}


def time_oracle(w, n_steps):
    """Oracle steps taken, seconds, leaf updates, and whether the workload's
    run is complete (its step count or its end time reached)."""
    import oracle as O
    o = O.Oracle(w.params, w.h, w.qx, w.qy, w.z)
    t0 = time.perf_counter()
    n = o.run(n_steps)
    dt = time.perf_counter() - t0
    sc = o.scalars()
    done = n >= w.n_steps or sc["t"] >= w.params.get("t_end", math.inf)
    o.close()
    return n, dt, sc["leaf_updates"], done


def cpu_baseline(w, n_steps, c2_steps):
    """The oracle (one thread) on bounded samples: the headline workload's
    first n_steps, the L = 6 dam break over bumps in full, and the first
    c2_steps of the L = 10 circular dam break."""
    import workloads as W
    log(f"[bench] cpu oracle: {n_steps} steps of {w.name}")
    n, dt, lu, _ = time_oracle(w, n_steps)
    out = {"value": round(n / dt, 4), "unit": "timesteps/s", "cores": 1,
           "kind": "oracle",
           "sample": f"first {n} timesteps of {w.name} (L={w.L}, {4 ** w.L} cells), "
                     f"FP64, single thread, {dt:.1f} s",
           "leaf_updates_per_s": lu / dt, "host": host_cpu(), "other": {}}
    for ww, k in ((W.dambreak_bumps_l6(), 10 ** 6), (W.circular_dambreak_l10(), c2_steps)):
        n, dt, lu, done = time_oracle(ww, k)
        log(f"[bench] cpu oracle: {ww.name} {n} steps in {dt:.2f} s")
        out["other"][ww.name] = {"steps": n, "s": round(dt, 3),
                                 "timesteps_per_s": round(n / dt, 3),
                                 "leaf_updates_per_s": lu / dt,
                                 "complete_run": bool(done)}
    return out


def whole_run(hw, w, precision, tuning):
    """Every step of the workload's run from its initial state (HIP events
    around all w.n_steps replays of the captured step), so that the wet
    phase's full FV1 updates count as well as the dry start."""
    import numpy as np
    import torch
    sim = hw.Simulation(w.params, w.h, w.qx, w.qy, w.z, precision=precision)
    plan = hw.Plan([sim.problem], [sim.buffers], tuning=tuning)
    hw.hwfv1_run(sim.problem, sim.buffers, 1, plan=plan, stats=False)
    dev = [torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64).reshape(-1), device="cuda")
           for a in (w.h, w.qx, w.qy, w.z)]
    hw.hw_ingest(sim.problem, sim.buffers, *dev)
    del dev
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    hw.hwfv1_run(sim.problem, sim.buffers, w.n_steps, plan=plan, stats=False)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    s = sim.scalars()
    out = {"steps": int(s["step"]), "t_end_s": s["t"], "ms": round(ms, 3),
           "ms_per_step": round(ms / w.n_steps, 5),
           "value": round(w.n_steps / (ms * 1e-3), 2), "unit": "timesteps/s",
           "leaf_updates": int(s["leaf_updates"]),
           "full_updates": int(s["leaf_updates"] - s["dry_stored"] - s["dry_skipped"]),
           "dry_pass_updates": int(s["dry_stored"] + s["dry_skipped"]),
           "wet_cells_at_end": int((hw.hw_export(sim.problem, sim.buffers)[0]
                                    > w.params["h_tol"]).sum().item())}
    plan.close()
    sim.close()
    return out


def precision_stress(hw, steps, prof_steps):
    """The thin-sheet workload at L = 13 (eps 1e-4, rain, Manning 0.05, 500 m
    relief): FP64 and FP32 bulk over the same steps; timesteps/s, rooflines,
    and the FP32 form's error against FP64 (whose first steps the parity
    tests compare with the oracle)."""
    import numpy as np
    import torch
    import workloads as W
    log("[bench] precision stress: generating the L = 13 sheet-flow inputs")
    w = W.sheetflow_l13(n_steps=steps)
    out = {"workload": w.name, "L": w.L, "eps": w.params["eps"], "steps": steps}
    res = {}
    for prec in ("fp64", "fp32_bulk"):
        r = time_single(hw, w, prec, steps, 2, prof_steps)
        res[prec] = r
        out[prec] = {"value": round(steps / (r["ms"] * 1e-3), 2), "unit": "timesteps/s",
                     "ms_per_step": round(r["ms"] / steps, 5),
                     "n_leaves": int(r["scalars"]["n_leaves"]),
                     "leaf_updates_per_step": dry_split(r),
                     "roofline": roofline(r, w.L, 8 if prec == "fp64" else 4),
                     "mass": r["scalars"]["mass"], "mass0": r["scalars"]["mass0"],
                     "t": r["scalars"]["t"], "tuning": r["tuning"]}
        if prec == "fp64":
            # keep only the exported fields of the FP64 run on the host
            res["f64"] = [t.cpu().numpy() for t in hw.hw_export(r["sim"].problem, r["sim"].buffers)]
            res["leaves64"] = r["sim"].buffers.leaf_list()
            r["plan"].close()
            r["sim"].close()
            del r
            res.pop("fp64")
            torch.cuda.empty_cache()
    r32 = res["fp32_bulk"]
    b = [t.cpu().numpy() for t in hw.hw_export(r32["sim"].problem, r32["sim"].buffers)]
    a = res["f64"]
    l32 = r32["sim"].buffers.leaf_list()
    out["error_fp32_vs_fp64"] = {
        "l1_h": float(np.mean(np.abs(a[0] - b[0]))),
        "linf_h": float(np.max(np.abs(a[0] - b[0]))),
        "l1_qx": float(np.mean(np.abs(a[1] - b[1]))),
        "linf_qx": float(np.max(np.abs(a[1] - b[1]))),
        "l1_qy": float(np.mean(np.abs(a[2] - b[2]))),
        "linf_qy": float(np.max(np.abs(a[2] - b[2]))),
        "leaf_symdiff": int(len(np.setxor1d(res["leaves64"], l32))),
        "n_leaves_fp64": int(len(res["leaves64"])),
        "mass_rel_err": (out["fp32_bulk"]["mass"] - out["fp64"]["mass"]) / out["fp64"]["mass"],
        "vs": "FP64 GPU run of the same steps (its first steps equal the oracle within 1e-10)",
    }
    log(f"[bench] precision stress: FP64 {out['fp64']['value']} steps/s, FP32 bulk "
        f"{out['fp32_bulk']['value']} steps/s, {out['error_fp32_vs_fp64']}")
    r32["plan"].close()
    r32["sim"].close()
    del r32, res
    torch.cuda.empty_cache()
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--prof-steps", type=int, default=20)
    ap.add_argument("--cpu-steps", type=int, default=10)
    ap.add_argument("--cpu-c2-steps", type=int, default=50)
    ap.add_argument("--stress-steps", type=int, default=1000)
    ap.add_argument("--no-stress", action="store_true",
                    help="skip the L = 13 precision-stress runs")
    ap.add_argument("--batch-steps", type=int, default=1000)
    ap.add_argument("--batch-members", type=int, default=64)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-fp32", action="store_true")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--no-speedup", action="store_true",
                    help="skip the uniform-FV1 comparisons")
    ap.add_argument("--no-variants", action="store_true",
                    help="skip the no-write-skip and fully wet FP64 runs")
    ap.add_argument("--tuning", default=None, metavar="CPT,GRID[,SPARSE[,TILES]]",
                    help="fixed launch shape for the single-problem runs "
                         "(encode cells per thread, FV1 workgroups, and optionally "
                         "1/0 for the tree-sparse finest set on/off, and FP32 first-pass "
                         "tiles per workgroup) instead of the autotuner, e.g. 4,2048 or "
                         "4,1024,0")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="also run a plain device copy of this many MiB three "
                         "times (reference kernel for HBM counter scaling)")
    ap.add_argument("--circular", type=int, default=None, metavar="L",
                    help="profiling mode: only run the circular dam break at level L "
                         "(eps 1e-3) from its initial state to t_end, with the "
                         "tree-sparse finest set on or off (--sparse), and print its time")
    ap.add_argument("--sparse", type=int, default=1, choices=(0, 1))
    ap.add_argument("--run", default=None,
                    choices=("hydrograph_l12", "flooded_basin_l12", "sheetflow_l13"),
                    help="profiling mode: only time this workload (--steps after "
                         "--warmup, --precision, default launch shapes or --tuning) "
                         "and print its time and phase split")
    ap.add_argument("--precision", default="fp64", choices=("fp64", "fp32_bulk"))
    ap.add_argument("--circular-steps", type=int, default=0, metavar="K",
                    help="with --circular: run only the first K steps, once "
                         "(for counter collection), instead of to t_end")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path "
              "(Morton-subtree sharding is a design, not an implementation); "
              "run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_2206_05761_amd as hw
    import workloads as W

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(2)
    hw.lib()
    if args.circular is not None:
        w = W.circular_dambreak_flat(args.circular, 1e-3)
        tu = dict(encode_skip=args.sparse, fill_skip=args.sparse)
        if args.circular_steps > 0:
            sim = hw.Simulation(w.params, w.h, w.qx, w.qy, w.z, precision="fp64")
            plan = hw.Plan([sim.problem], [sim.buffers], tuning=tu)
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            st = hw.hwfv1_run(sim.problem, sim.buffers, args.circular_steps, plan=plan)
            e1.record()
            torch.cuda.synchronize()
            ms, n, t = e0.elapsed_time(e1), st["steps"], st["t"]
            leaves = st["leaf_updates"] / max(n, 1)
            plan.close()
            sim.close()
        else:
            ms, n, leaves, t = run_to_end_ms(hw, w, False, tuning=tu)
        print(json.dumps({"workload": w.name, "L": args.circular, "eps": 1e-3,
                          "tree_sparse": bool(args.sparse), "steps": n, "t": t,
                          "ms_to_t_end": round(ms, 3), "ms_per_step": round(ms / n, 5),
                          "mean_leaf_fraction": round(leaves / 4 ** args.circular, 4)}),
              flush=True)
        return
    tuning = None
    if args.tuning:
        vals = [int(v) for v in args.tuning.split(",")]
        tuning = dict(encode_cells_per_thread=vals[0], fv1_grid=vals[1])
        if len(vals) > 2:
            tuning.update(encode_skip=vals[2], fill_skip=vals[2])
        if len(vals) > 3:
            tuning.update(encode_tiles=vals[3])
    if args.run is not None:
        ww = getattr(W, args.run)()
        r = time_single(hw, ww, args.precision, args.steps, args.warmup, args.prof_steps,
                        tuning if tuning is not None else {})
        wb = 8 if args.precision == "fp64" else 4
        if args.copy_calibration_mib > 0:
            n = args.copy_calibration_mib * (1 << 20) // 8
            src = torch.ones(n, dtype=torch.float64, device="cuda")
            dst = torch.empty_like(src)
            for _ in range(3):
                dst.copy_(src)
            torch.cuda.synchronize()
            del src, dst
        print(json.dumps({"workload": ww.name, "precision": args.precision,
                          "steps": args.steps, "warmup": args.warmup,
                          "ms_per_step": round(r["ms"] / args.steps, 5),
                          "leaf_updates_per_step": dry_split(r),
                          "roofline": roofline(r, ww.L, wb, args.precision, ww.name)}),
              flush=True)
        return
    w = W.hydrograph_l12()
    L = w.L
    r64 = time_single(hw, w, "fp64", args.steps, args.warmup, args.prof_steps, tuning)
    value = args.steps / (r64["ms"] * 1e-3)
    line = {
        "metric": METRIC,
        "value": round(value, 2),
        "unit": "timesteps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(r64["ms"] / args.steps, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": w.name, "L": L, "finest_cells": 4 ** L,
                   "eps": w.params["eps"], "domain_m": 10000.0,
                   "bed": "seeded spectral fractal, relief 50 m",
                   "forcing": "west-edge triangular hydrograph 500 m^3/s",
                   "manning_n": w.params["manning_n"], "precision": "fp64"},
        "leaf_updates_per_s": r64["leaf_updates"] / (r64["ms"] * 1e-3),
        "n_leaves": int(r64["scalars"]["n_leaves"]),
        "leaf_updates_per_step": dry_split(r64),
        "roofline": roofline(r64, L, 8, "fp64", w.name),
        "tuning": r64["tuning"], "autotune_ms_per_step": r64["tuning_table"],
    }
    if not args.no_variants:
        # The same FP64 run with every leaf stored every step (no skip of
        # unchanged dry blocks), for comparison with the default.
        tu = dict(r64["tuning"], fv1_write_skip=0)
        rns = time_single(hw, w, "fp64", args.steps, args.warmup, args.prof_steps, tu)
        line["no_write_skip"] = {
            "value": round(args.steps / (rns["ms"] * 1e-3), 2), "unit": "timesteps/s",
            "ms_per_step": round(rns["ms"] / args.steps, 5),
            "fv1_ms": round(rns["prof"]["fv1"], 5),
            "leaf_updates_per_step": dry_split(rns),
            "roofline": roofline(rns, L, 8),
            "note": "FP64, same workload and steps, fv1_write_skip=0",
        }
        rns["plan"].close()
        rns["sim"].close()
        del rns
        # Every cell wet: every leaf takes the full FV1 update.
        ww = W.flooded_basin_l12()
        rw = time_single(hw, ww, "fp64", ww.n_steps, 5, args.prof_steps, tuning)
        h_end = hw.hw_export(rw["sim"].problem, rw["sim"].buffers)[0]
        line["fully_wet"] = {
            "workload": ww.name, "steps": ww.n_steps,
            "value": round(ww.n_steps / (rw["ms"] * 1e-3), 2), "unit": "timesteps/s",
            "ms_per_step": round(rw["ms"] / ww.n_steps, 5),
            "leaf_updates_per_s": rw["leaf_updates"] / (rw["ms"] * 1e-3),
            "n_leaves": int(rw["scalars"]["n_leaves"]),
            "wet_fraction": float((h_end > ww.params["h_tol"]).float().mean().item()),
            "leaf_updates_per_step": dry_split(rw),
            "roofline": roofline(rw, L, 8, "fp64", ww.name),
            "tuning": rw["tuning"],
        }
        rw["plan"].close()
        rw["sim"].close()
        del rw, h_end
        if not args.no_fp32:
            rw = time_single(hw, ww, "fp32_bulk", ww.n_steps, 5, args.prof_steps, tuning)
            line["fully_wet"]["fp32_bulk"] = {
                "value": round(ww.n_steps / (rw["ms"] * 1e-3), 2), "unit": "timesteps/s",
                "ms_per_step": round(rw["ms"] / ww.n_steps, 5),
                "leaf_updates_per_step": dry_split(rw),
                "roofline": roofline(rw, L, 4, "fp32_bulk", ww.name),
                "tuning": rw["tuning"],
            }
            rw["plan"].close()
            rw["sim"].close()
            del rw
        # The whole hydrograph run from t = 0 (dry start, then the wet phase).
        line["whole_run"] = dict(whole_run(hw, w, "fp64", r64["tuning"]), workload=w.name,
                                 precision="fp64")
        log(f"[bench] whole run: {line['whole_run']}")
    if not args.no_speedup:
        # The same workload and steps on the uniform FV1 plan (every finest
        # cell updated, no multiresolution phases).
        ru = time_single(hw, w, "fp64", args.steps, args.warmup, args.prof_steps,
                         r64["tuning"], uniform=True)
        uv = args.steps / (ru["ms"] * 1e-3)
        line["uniform_fv1"] = {
            "workload": w.name, "value": round(uv, 2), "unit": "timesteps/s",
            "ms_per_step": round(ru["ms"] / args.steps, 5),
            "hwfv1_over_uniform": round(value / uv, 3),
            "leaf_updates_per_step": dry_split(ru),
            "roofline": roofline(ru, L, 8),
            "note": "FP64 uniform FV1 plan, same workload, steps and FV1 launch shape",
        }
        ru["plan"].close()
        ru["sim"].close()
        del ru
        line["speedup_series"] = bench_speedup(hw)
        line["speedup_pseudo2d"] = bench_pseudo2d(hw)
        line["verification"] = bench_verification(hw)
    if not args.no_fp32:
        r32 = time_single(hw, w, "fp32_bulk", args.steps, args.warmup, args.prof_steps,
                          tuning)
        line["fp32_bulk"] = {
            "value": round(args.steps / (r32["ms"] * 1e-3), 2), "unit": "timesteps/s",
            "ms_per_step": round(r32["ms"] / args.steps, 5),
            "leaf_updates_per_s": r32["leaf_updates"] / (r32["ms"] * 1e-3),
            "leaf_updates_per_step": dry_split(r32),
            "roofline": roofline(r32, L, 4, "fp32_bulk", w.name),
            "tuning": r32["tuning"],
            "error_vs_fp64": fp32_error(hw, r64, r32),
        }
        r32["plan"].close()
        r32["sim"].close()
        del r32
    r64["plan"].close()
    r64["sim"].close()
    del r64
    torch.cuda.empty_cache()
    if not args.no_stress:
        line["precision_stress"] = precision_stress(hw, args.stress_steps, min(args.prof_steps, 5))
    if not args.no_batch:
        line["batched"] = bench_batch(hw, args.batch_steps, args.warmup,
                                      args.batch_members)
    if args.copy_calibration_mib > 0:
        n = args.copy_calibration_mib * (1 << 20) // 8
        src = torch.ones(n, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        line["copy_calibration_bytes"] = {"read": n * 8, "write": n * 8}
        del src, dst
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline(w, args.cpu_steps, args.cpu_c2_steps)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
