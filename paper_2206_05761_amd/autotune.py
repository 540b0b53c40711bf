"""Autotuner for the HWFV1 launch shapes.

Chooses, for a given set of problems (one, or a batch), the encoding tile
(4 or 16 finest cells per thread, i.e. tiles of 4^5 or 4^6 cells and 5 or 6
levels fused per pass) and the number of persistent FV1 workgroups, by timing
each candidate's captured step graph on the problems themselves, and then
whether the best shape runs with the tree-sparse finest set (the default) or
reads and writes every finest cell (encode_skip = fill_skip = 0), which can
be slightly faster when every leaf is finest.  The state
(both finest sets and the scalars) is saved before and restored after every
candidate (and the FV1 write history forgotten), so tuning leaves the
simulation where it was.  Results are cached
in a JSON file keyed by GPU architecture, precision, batch size and levels.
"""
import json
import os

import torch

from . import Plan, hw_forget, hwfv1_run, hwfv1_run_batch

CANDIDATES = [dict(encode_cells_per_thread=c, fv1_grid=g)
              for c in (4, 16) for g in (1024, 2048, 4096)]
DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "hwfv1_autotune.json")


def _key(problems):
    arch = torch.cuda.get_device_properties(torch.cuda.current_device()).gcnArchName
    prec = int(problems[0].precision)
    levels = sorted(int(p.L) for p in problems)
    return f"{arch}|prec{prec}|n{len(problems)}|L{','.join(map(str, levels))}"


def _load(path):
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _save(path, data):
    try:
        os.makedirs(os.path.dirname(path), exist_ok=True)
        tmp = path + ".tmp"
        with open(tmp, "w") as f:
            json.dump(data, f, indent=1, sort_keys=True)
        os.replace(tmp, path)
    except OSError:
        pass


def _snapshot(buffers):
    return [([t.clone() for t in b.fine[0]], [t.clone() for t in b.fine[1]],
             b.scal.clone()) for b in buffers]


def _restore(problems, buffers, snap):
    for p, b, (f0, f1, sc) in zip(problems, buffers, snap):
        for dst, src in zip(b.fine[0], f0):
            dst.copy_(src)
        for dst, src in zip(b.fine[1], f1):
            dst.copy_(src)
        b.scal.copy_(sc)
        hw_forget(p, b)


def _time(problems, buffers, tuning, steps, warmup):
    plan = Plan(problems, buffers, tuning=tuning)
    try:
        run = (lambda k: hwfv1_run(problems[0], buffers[0], k, plan=plan, stats=False)) \
            if len(problems) == 1 else (lambda k: hwfv1_run_batch(plan, k, stats=False))
        run(warmup)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        run(steps)
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / steps
    finally:
        plan.close()


def autotune(problems, buffers, steps=10, warmup=2, candidates=None,
             cache_path=DEFAULT_CACHE, use_cache=True):
    """Best tuning dict for these problems (and the per-candidate ms/step).

    problems: list of HwProblem; buffers: list of Buffers (same length)."""
    key = _key(problems)
    cache = _load(cache_path) if cache_path else {}
    if use_cache and key in cache:
        return cache[key]["best"], cache[key]["ms_per_step"]
    snap = _snapshot(buffers)
    results = []
    for cand in candidates or CANDIDATES:
        ms = _time(problems, buffers, cand, steps, warmup)
        _restore(problems, buffers, snap)
        results.append((ms, cand))
    torch.cuda.synchronize()
    results.sort(key=lambda r: r[0])
    best = results[0][1]
    if candidates is None:
        # The tree-sparse finest set (on by default) against reading and
        # writing every finest cell, with the best launch shape: each timed
        # twice, alternately; it is kept unless the dense form is clearly
        # faster on this state.
        dense = dict(best, encode_skip=0, fill_skip=0)
        t_on = t_off = float("inf")
        for _ in range(2):
            for cand in (best, dense):
                ms = _time(problems, buffers, cand, 2 * steps, warmup)
                _restore(problems, buffers, snap)
                if cand is best:
                    t_on = min(t_on, ms)
                else:
                    t_off = min(t_off, ms)
        results.append((t_off, dense))
        if t_off < 0.997 * t_on:
            best = dense
    table = {json.dumps(c, sort_keys=True): round(ms, 5) for ms, c in results}
    if cache_path:
        cache[key] = {"best": best, "ms_per_step": table}
        _save(cache_path, cache)
    return best, table
