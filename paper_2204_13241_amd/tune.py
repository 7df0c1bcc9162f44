"""Autotuner for the FP32C tile shapes.

For a given batch layout it builds a plan per candidate shape, times the whole
forward call (binning, pair kernel, combination of the partial sums) and the
whole gradient call (pixel prologue, pair kernel, combination) with HIP events
on the stream, and keeps the fastest: the shape also sets how many partial sums
the combination reads.  Results are cached in a JSON file keyed by the device architecture
and a workload signature (systems, frames, atom and pixel counts bucketed to
powers of two, planar or curved detector), so a later run on the same kind of
workload skips the search.  Cache path: $XS_TUNE_CACHE, else
~/.cache/paper_2204_13241_amd/tune.json.
"""
from __future__ import annotations

import json
import math
import os
from typing import List, Optional

import numpy as np
import torch

from . import api

# (pixels per lane, waves-per-SIMD bound) x atom tiles per item; 32 pixels per run is
# the matrix-core lattice form (the general form then runs 8 pixels per lane)
FWD_CANDIDATES = [(ql, occ, split)
                  for ql, occ in ((1, 0), (2, 0), (2, 4), (4, 0), (4, 4), (8, 0), (8, 3), (8, 4), (32, 0), (32, 3))
                  for split in (16, 32, 64, 128)]
# (atoms per lane, waves-per-SIMD bound) x pixels per item; 32 is the matrix-core
# lattice form, whose third entry is the atom tiles per item (the other systems of such
# a plan run 2 atoms per lane)
GRAD_CANDIDATES = ([(al, occ, pc)
                    for al, occ in ((1, 0), (2, 0), (2, 5), (4, 0), (4, 4), (8, 0))
                    for pc in (2048, 4096, 8192, 16384)]
                   + [(32, 0, split) for split in (32, 64, 128, 256)])


def candidates(cands, lattice: int) -> list:
    """The search space for a lattice setting: with lattice 0 the matrix-core shapes
    (32 per lane, factorized forms) are left out, so only per-pair kernels are timed."""
    return [tuple(c) for c in cands if lattice or c[0] != 32]


def _cache_path() -> str:
    p = os.environ.get("XS_TUNE_CACHE")
    if p:
        return p
    return os.path.join(os.path.expanduser("~"), ".cache", "paper_2204_13241_amd", "tune.json")


def _bucket(n: int) -> int:
    return 0 if n <= 0 else int(round(math.log2(n)))


def signature(systems, planar: bool, lattice: int = 1) -> str:
    arch = torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    na = sum(int(n) * int(t) for n, t, _, _ in systems)
    nq = sum(int(q.shape[0]) * int(t) for _, t, q, _ in systems)
    return "v10|%s|sys=%d|frames=%d|atoms=2^%d|pixels=2^%d|%s|%s" % (
        arch, len(systems), sum(int(t) for _, t, _, _ in systems), _bucket(na), _bucket(nq),
        "planar" if planar else "curved", "lattice" if lattice else "per-pair")


def _load_cache(path):
    try:
        with open(path) as fh:
            return json.load(fh)
    except (OSError, ValueError):
        return {}


def _store_cache(path, data):
    try:
        os.makedirs(os.path.dirname(path), exist_ok=True)
        tmp = path + ".tmp%d" % os.getpid()
        with open(tmp, "w") as fh:
            json.dump(data, fh, indent=1, sort_keys=True)
        os.replace(tmp, path)
    except OSError:
        pass


# A candidate replaces the best shape so far only when it is faster by more than this
# fraction: launch-to-launch noise is about 1%, and a stable pick keeps results (and the
# profiles taken with the default shapes) comparable from run to run.
TIE = 0.03


def _current_first(candidates, current):
    """The candidate list with the currently installed shape (if listed) moved to the front."""
    cands = list(candidates)
    return [c for c in cands if tuple(c) == tuple(current)] + [c for c in cands if tuple(c) != tuple(current)]


def _search(candidates, current, timer) -> dict:
    """Time every candidate (installed shape first); the installed shape is timed again
    at the end, when the clocks have settled, and keeps the better of its two times."""
    times = {}
    for c in _current_first(candidates, current):
        times[tuple(c)] = timer(tuple(c))
    cur = tuple(current)
    if cur in times:
        times[cur] = min(times[cur], timer(cur))
    return times


def _pick(times: dict, current):
    """The installed shape unless another one is faster by more than TIE (the fastest then)."""
    fastest = min(times, key=times.get)
    cur = tuple(current)
    if cur in times and not times[fastest] < times[cur] * (1.0 - TIE):
        return cur
    return fastest


def _time_call(run, reps: int, rounds: int = 2) -> float:
    """Mean time of one call over `reps` calls (HIP events on the current stream), the
    best of `rounds` rounds."""
    run()                                 # warm-up (also builds code objects)
    torch.cuda.synchronize()
    best = float("inf")
    for _ in range(rounds):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            run()
        e1.record()
        torch.cuda.synchronize()
        best = min(best, e0.elapsed_time(e1) / reps)
    return best


def tune(systems, pos: torch.Tensor, f: torch.Tensor, reps: int = 5, use_cache: bool = True,
         fwd_candidates: Optional[List] = None, grad_candidates: Optional[List] = None,
         apply: bool = True, lattice: int = 1) -> dict:
    """Pick the fastest forward and gradient tile shapes for this batch.

    systems: as for api.Plan; pos, f: packed positions and form factors.
    lattice 0 restricts the search to the per-pair form (no lattice factorization, no
    matrix-core shapes); 1 also tries the lattice forms where a plan finds row lattices.
    Returns {"forward": shape, "gradient": shape, "source": "cache"|"search",
    "timings_ms": {...}} and, if apply, installs the shapes (xs_set_tile_shape).
    """
    lattice = 1 if lattice else 0
    qz = torch.cat([q[:, 2] for _, _, q, _ in systems])
    planar = bool((qz == qz[0]).all().item()) if qz.numel() else True
    key = signature(systems, planar, lattice)
    fwd_candidates = candidates(fwd_candidates or FWD_CANDIDATES, lattice)
    grad_candidates = candidates(grad_candidates or GRAD_CANDIDATES, lattice)
    path = _cache_path()
    cache = _load_cache(path) if use_cache else {}
    if use_cache and key in cache:
        best = cache[key]
        if apply:
            api.set_tile_shape(0, **best["forward"])
            api.set_tile_shape(1, **best["gradient"])
        return dict(best, source="cache", key=key)
    old_f, old_g = api.get_tile_shape(0), api.get_tile_shape(1)
    timings = {"forward": {}, "gradient": {}}

    def fwd_shape(c):
        ql, occ, split = c
        return dict(atoms_per_tile=64, q_per_lane=ql, atom_split=split, pixel_split=old_f["pixel_split"],
                    waves_per_simd=occ, lattice=lattice)

    def time_fwd(c):
        api.set_tile_shape(0, **fwd_shape(c))
        plan = api.Plan(systems)
        I = torch.empty(plan.total_out, dtype=torch.float64, device=pos.device)
        amp = torch.empty((plan.total_out, 2), dtype=torch.float64, device=pos.device)
        t = _time_call(lambda: plan.intensity(pos, f, I, amp), reps)
        plan.close()
        return t

    cur_f = (old_f["q_per_lane"], old_f["waves_per_simd"], old_f["atom_split"])
    tf = _search(fwd_candidates, cur_f, time_fwd)
    pick_f = _pick(tf, cur_f)
    timings["forward"] = {"ql%d_occ%d_split%d" % c: t for c, t in tf.items()}
    best_f, best_ft = fwd_shape(pick_f), tf[pick_f]
    api.set_tile_shape(0, **best_f)
    # gradient: amplitudes of the tuned forward, unit-variance weights
    plan = api.Plan(systems)
    I = torch.empty(plan.total_out, dtype=torch.float64, device=pos.device)
    amp = torch.empty((plan.total_out, 2), dtype=torch.float64, device=pos.device)
    plan.intensity(pos, f, I, amp)
    gen = torch.Generator(device=pos.device)
    gen.manual_seed(1234)
    w = torch.randn(plan.total_out, dtype=torch.float64, device=pos.device, generator=gen)
    plan.close()

    def grad_shape(c):
        al, occ, pc = c
        if al == 32:
            return dict(atoms_per_tile=64, q_per_lane=32, atom_split=pc, pixel_split=old_g["pixel_split"],
                        waves_per_simd=0, lattice=lattice)
        return dict(atoms_per_tile=64, q_per_lane=al, atom_split=old_g["atom_split"], pixel_split=pc,
                    waves_per_simd=occ, lattice=lattice)

    def time_grad(c):
        api.set_tile_shape(1, **grad_shape(c))
        plan = api.Plan(systems)
        g = torch.empty((plan.total_pos, 3), dtype=torch.float32, device=pos.device)
        plan.grad(pos, f, amp, w, retile=True, g32=g)  # bins the atoms once
        t = _time_call(lambda: plan.grad(pos, f, amp, w, retile=False, g32=g), reps)
        plan.close()
        return t

    cur_g = (old_g["q_per_lane"], old_g["waves_per_simd"],
             old_g["atom_split"] if old_g["q_per_lane"] == 32 else old_g["pixel_split"])
    tg = _search(grad_candidates, cur_g, time_grad)
    pick_g = _pick(tg, cur_g)
    timings["gradient"] = {("mfma_split%d" % c[2] if c[0] == 32 else "al%d_occ%d_pix%d" % c): t
                           for c, t in tg.items()}
    best_g, best_gt = grad_shape(pick_g), tg[pick_g]
    result = {"forward": best_f, "gradient": best_g, "forward_ms": best_ft, "gradient_ms": best_gt}
    if use_cache:
        cache[key] = result
        _store_cache(path, cache)
    if apply:
        api.set_tile_shape(0, **best_f)
        api.set_tile_shape(1, **best_g)
    else:
        api.set_tile_shape(0, **old_f)
        api.set_tile_shape(1, **old_g)
    return dict(result, source="search", key=key, timings_ms=timings)
