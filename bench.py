"""Benchmark of the direct speckle-intensity path on one MI355X.

Default workload (differentiation): N = 65,536 atoms uniform in a cube at
0.021 atoms per cubic Angstrom, f = 1, 512 x 512 planar pixels with
q_x, q_y in [-3, 3] 1/Angstrom, target intensities from the positions displaced
by Gaussian noise (sigma 0.2 Angstrom).  One step = FP32C forward (amplitude
and intensity of every pixel), speckle-matching loss and dL/dI, FP32C adjoint
dL/dr, and a gradient-descent position update; 2 N Q atom-pixel pair
evaluations per step.  Inputs are resident in GPU memory before timing starts.

Prints one JSON line (metric, value in G atom-q pair evals/s, roofline of the
dominant kernel from HIP-event kernel timings, CPU-oracle baseline, accuracy of
the FP32C results against the exact FP64 form, FP64-form speedup).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = ("G atom-q pair evals/s (fwd+adjoint) vs FP64 form at 1e-5 rel err; % VALU roofline")
UNIT = "G atom-q pair evals/s"
# MI355X: 256 CUs at 2.4 GHz; FP32 vector FMA 128 lanes/clk/CU (157.3 TFLOP/s);
# v_sin_f32 / v_cos_f32 issue at a quarter of that, 32 lanes/clk/CU, and (measured)
# do not overlap with other VALU work of the same CU.
CUS, CLOCK = 256, 2.4e9
VALU_LANES = 128
TRANS_LANES = 32
PEAK_TRANS = CUS * CLOCK * TRANS_LANES          # transcendental lane-ops/s
PEAK_SINCOS_PAIRS = PEAK_TRANS / 2.0           # pairs/s with one sin + one cos each
PEAK_HBM = 8.0e12                              # bytes/s
PEAK_FMA64 = CUS * CLOCK * 64                  # FP64 FMA lane-ops/s (78.6 TFLOP/s)
PEAK_F16_MFMA = 2.5e15                          # dense FP16 matrix flop/s


def alu_peak(n_valu, n_trans, mfma_flops=0.0):
    """Pairs/s when every CU issues only the kernel's per-pair VALU, transcendental and
    FP16 matrix work back to back: transcendental and other VALU instructions do not
    overlap (probes kinds 0 and 1); matrix and VALU instructions overlap about half of the
    VALU time (probes kinds 4 and 5), so for the matrix-core kernels the sum is a
    conservative peak."""
    f16_per_cu_clk = PEAK_F16_MFMA / (CUS * CLOCK)
    return CUS * CLOCK / (n_valu / VALU_LANES + n_trans / TRANS_LANES + mfma_flops / f16_per_cu_clk)


def pair_mix(kernel, lattice, ql, qz_zero, rows=False):
    """Per-pair work (FP32 VALU, transcendental, FP16 matrix flops) of the inner loops.
    forward, general: 2 FMA phase (3 with dq_z), sin + cos, 2 FMA accumulate.
    forward, lattice run of QL pixels: per atom 2 FMA phase (3 with dq_z) + sin + cos
    + 2 FMA for pixel 0 + 4 FMA (complex multiply-add) for each further pixel.
    forward, matrix-core lattice (runs of 32): per (run, atom) add + 2 FMA phase (3 with
    dq_z), sin + cos and the FP16 split of both parts (~10 VALU), shared by the run's 32
    pixels; per (atom, pixel column) of a block the G factor (~20 VALU + sin + cos, shared
    by 128 pixels); per tile and pixel the FP64 fold (3 ops / 64 atoms); 12 matrix
    instructions of 32x32x16 per 16 atoms and 32x32 pixels = 24 flops per pair.
    forward, row form (lane's QL pixels in one detector row): fma(dq_y, d_y, beta) once per
    (lane, atom), then per pair 1 FMA phase (2 with dq_z), sin + cos, 2 FMA accumulate.
    adjoint, general: add + 2 FMA phase (3 with dq_z), sin, 2 FMA (3 with W_z).
    adjoint, row groups (dq_y = 0): add + 1 FMA phase (2 with dq_z), sin, 2 FMA (3 with W_z).
    adjoint, lattice: FMA + add phase, sin, 2 FMA (3 with W_z).
    adjoint, matrix-core lattice (runs of 32): per (run, atom) add + 2 FMA phase (3 with
    dq_z), sin + cos and 2 FMA per component (2 components at q_z = 0, else 3), shared by
    the run's 32 pixels; the G factor per (pixel column, atom) as in the forward (shared by
    128 pixels); 12 matrix instructions of 32x32x16 per component, 16 pixels of a row and
    32 runs x 32 atoms = 24 flops per pair and component."""
    if kernel == "forward_fp32c":
        ph = 2 if qz_zero else 3
        if lattice and ql == 32:
            return (1 + ph + 10) / 32 + 20 / 128 + 3 / 64, 2 / 32 + 2 / 128, 24.0
        if lattice:
            return (ph + 2 + 4 * (ql - 1)) / ql, 2.0 / ql, 0.0
        if rows:
            return (ph - 1) + 1.0 / ql + 2, 2.0, 0.0
        return ph + 2, 2.0, 0.0
    acc = 2 if qz_zero else 3
    if lattice and ql == 32:
        return (1 + (2 if qz_zero else 3) + 2 * acc) / 32 + 20 / 128, 2 / 32 + 2 / 128, 24.0 * acc
    if lattice:
        return 2 + acc, 1.0, 0.0
    if rows:
        return 1 + (1 if qz_zero else 2) + acc, 1.0, 0.0
    return 1 + (2 if qz_zero else 3) + acc, 1.0, 0.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


DEVICE_END = b"// ---------------------------------------------------------------- host side"


def source_hash(path):
    """sha256[:16] of the device-code part of a kernel source (everything before its host
    section), so host-side edits do not invalidate the kernels' counter profiles."""
    with open(path, "rb") as fh:
        src = fh.read()
    cut = src.find(DEVICE_END)
    return hashlib.sha256(src if cut < 0 else src[:cut]).hexdigest()[:16]


def traffic_from_profile(kernel_src, kernel, shape):
    """HBM bytes per launch of a pair kernel from the committed PMC summary, or None
    if the summary is missing or was taken on a different kernel source or tile shape."""
    path = os.path.join(ROOT, "profiles", "pair_kernels_pmc_grad65536.json")
    try:
        d = json.load(open(path))
    except (OSError, ValueError):
        return None
    if d.get("source_sha256_16") != source_hash(kernel_src):
        return None
    rec = d.get("kernels", {}).get(kernel, {})
    if rec.get("tile_shape") != dict(shape):
        return None
    return rec.get("hbm_bytes_per_launch")


def cpu_baseline(pos, f, q, amp, w, budget_s=20.0):
    """The oracle (FP64 form, OpenMP) on a bounded sample of the same workload."""
    import oracle
    threads = min(16, os.cpu_count() or 1)
    N, Q = pos.shape[0], q.shape[0]
    # calibrate on a small forward piece
    t = time.perf_counter()
    oracle.intensity(pos, f, q[:1024], threads=threads)
    per_pair = (time.perf_counter() - t) / (N * 1024)
    n_pix = int(max(64, min(Q, (0.6 * budget_s) / (per_pair * N))))
    n_atoms = int(max(16, min(N, (0.4 * budget_s) / (per_pair * Q))))
    rng = np.random.default_rng(7)
    pix = np.sort(rng.choice(Q, n_pix, replace=False))
    atoms = np.sort(rng.choice(N, n_atoms, replace=False))
    t0 = time.perf_counter()
    oracle.intensity(pos, f, q[pix], threads=threads)
    t1 = time.perf_counter()
    oracle.intensity_grad(pos[atoms], f[atoms], q, amp, w, threads=threads)
    t2 = time.perf_counter()
    pairs = N * n_pix + n_atoms * Q
    return {
        "value": pairs / (t2 - t0) / 1e9,
        "unit": UNIT,
        "cores": threads,
        "kind": "oracle",
        "sample": ("FP64-form forward over all %d atoms x %d random pixels (%.1f s) + FP64-form "
                   "gradient of %d random atoms over all %d pixels (%.1f s)"
                   % (N, n_pix, t1 - t0, n_atoms, Q, t2 - t1)),
    }


def rel_grad_err(g, g_ref):
    g = g.reshape(-1, 3)
    g_ref = g_ref.reshape(-1, 3)
    rms = math.sqrt(float(np.mean(np.sum(g_ref * g_ref, axis=1))))
    return float(np.max(np.linalg.norm(g - g_ref, axis=1)) / rms)


# Tile shapes of the matrix-core lattice leg (the autotuner's pick for this workload
# among the lattice shapes); that leg is reported beside the headline, not as it.
LATTICE_MFMA_SHAPES = (dict(atoms_per_tile=64, q_per_lane=32, atom_split=32, pixel_split=0,
                            waves_per_simd=3, lattice=1),
                       dict(atoms_per_tile=64, q_per_lane=32, atom_split=128, pixel_split=8192,
                            waves_per_simd=0, lattice=1))


def run_grad(args, form="per-pair"):
    """One training step of the differentiation workload, timed.  form "per-pair": the
    direct method as the metric counts it (every atom-pixel pair evaluates its own sine and
    cosine in the forward and its own sine in the adjoint), tile shapes autotuned among the
    per-pair shapes.  form "lattice-mfma": the planar grid factorized into complex matrix
    products on FP16 matrix cores (opt-in form, reported separately)."""
    import torch
    from paper_2204_13241_amd import api, inputs

    dev = "cuda:0"
    w = inputs.workload_grad()
    r0, f_np, q_np, L = w.positions[0][0], w.f[0], w.q[0], w.box[0]
    N, Q = r0.shape[0], q_np.shape[0]
    T = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device=dev)
    pos, f, q = T(r0), T(f_np), T(q_np)
    It = api.intensity(T(w.extra["r_target"]), f, q, "fp64")
    torch.cuda.synchronize()
    log("inputs ready: N=%d Q=%d" % (N, Q))

    tuned = None
    old_shapes = [api.get_tile_shape(0), api.get_tile_shape(1)]
    if form == "lattice-mfma":
        api.set_tile_shape(0, **LATTICE_MFMA_SHAPES[0])
        api.set_tile_shape(1, **LATTICE_MFMA_SHAPES[1])
    elif not args.no_tune:
        from paper_2204_13241_amd import tune
        tuned = tune.tune([(N, 1, q, L)], pos, f, use_cache=not args.retune, lattice=0)
        log("tile shapes (%s): fwd %s  grad %s" % (tuned["source"], tuned["forward"], tuned["gradient"]))
    else:
        for k in (0, 1):
            api.set_tile_shape(k, **dict(old_shapes[k], lattice=0))
    shapes = [api.get_tile_shape(0), api.get_tile_shape(1)]
    # one plan for the whole run: work lists, buffers and pixel order built once
    plan = api.Plan.single(N, 1, q, L)
    I = torch.empty(Q, dtype=torch.float64, device=dev)
    amp = torch.empty((Q, 2), dtype=torch.float64, device=dev)
    g = torch.empty((N, 3), dtype=torch.float32, device=dev)
    state = {"step": None}

    def step():
        plan.intensity(pos, f, I, amp)
        loss, dLdI = api.speckle_loss(I, It)
        plan.grad(pos, f, amp, dLdI, retile=False, g32=g)
        api.position_step(pos, g, state["step"])
        return loss

    # fixed step size from the first gradient: 0.05 Angstrom / max |g|
    plan.intensity(pos, f, I, amp)
    _, dLdI = api.speckle_loss(I, It)
    plan.grad(pos, f, amp, dLdI, retile=False, g32=g)
    state["step"] = 0.05 / float(g.abs().max())
    e_chain_r0 = None
    if not args.no_fp64:
        # FP32C chain (forward -> loss -> adjoint) against the FP64 chain at r0, where
        # I - I_t is not small
        I64, amp64 = api.intensity(pos, f, q, "fp64", return_amp=True)
        _, w64 = api.speckle_loss(I64, It)
        g64 = api.intensity_grad(pos, f, q, amp64, w64, "fp64", out_dtype=torch.float64)
        e_chain_r0 = rel_grad_err(g.double().cpu().numpy(), g64.cpu().numpy())
        del I64, amp64, w64, g64
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    graph = None
    if args.graph:
        s_cap = torch.cuda.Stream()
        s_cap.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s_cap):
            step()
        torch.cuda.current_stream().wait_stream(s_cap)
        torch.cuda.synchronize()
        graph = torch.cuda.CUDAGraph()
        # capture on the warmed-up stream: the library's scratch is cached per stream and
        # cannot grow during capture
        with torch.cuda.graph(graph, stream=s_cap):
            loss_g = step()
        graph.replay()
        torch.cuda.synchronize()
    log("warmup done")
    api.timing_enable(not args.graph)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        if graph is not None:
            graph.replay()
            loss = loss_g
        else:
            loss = step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    if graph is not None:
        # event timers are not recorded inside a replayed graph: the per-kernel figures
        # come from the same number of eager steps right after the timed replays
        api.timing_enable(True)
        for _ in range(args.steps):
            step()
        torch.cuda.synchronize()
    fwd = api.timing_read("fwd32")
    grd = api.timing_read("grad32")
    binr = api.timing_read("bin")
    api.timing_enable(False)
    ms_step = (t1 - t0) * 1e3 / args.steps
    pairs_step = 2.0 * N * Q
    value = pairs_step / (ms_step * 1e-3) / 1e9
    log("timed %d steps: %.3f ms/step, %.1f G pairs/s, loss %.6g" % (args.steps, ms_step, value,
                                                                      float(loss[0])))

    info = plan.describe()
    lattice = info["n_segments"] > 0 and info["n_lattice_segments"] == info["n_segments"]
    rows = info["n_segments"] > 0 and info.get("n_row_segments", 0) == info["n_segments"]
    qz_zero = bool(np.all(q_np[:, 2] == 0.0))
    src = os.path.join(ROOT, "paper_2204_13241_amd", "csrc", "k_fp32c.hip")
    kern = {}
    for name, rec, kind in (("forward_fp32c", fwd, 0), ("adjoint_fp32c", grd, 1)):
        avg_ms = rec["ms"] / max(rec["launches"], 1)
        work = rec["work"] / max(rec["launches"], 1)
        ach = work / (avg_ms * 1e-3) / 1e9
        ql = max(2, shapes[kind]["q_per_lane"]) if lattice else shapes[kind]["q_per_lane"]
        n_valu, n_trans, n_mfma = pair_mix(name, lattice, ql, qz_zero, rows)
        peak = alu_peak(n_valu, n_trans, n_mfma) / 1e9
        # transcendental-issue bound: the unit a per-pair kernel saturates (one v_sin +
        # one v_cos per forward pair, one v_sin per adjoint pair)
        trans_peak = PEAK_TRANS / n_trans / 1e9
        kern[name] = {"avg_ms": avg_ms, "launches": rec["launches"], "pairs_per_launch": work,
                      "form": (("lattice-mfma" if ql == 32 else "lattice") if lattice
                               else ("per-pair rows" if rows else "per-pair general")),
                      "valu_per_pair": n_valu, "trans_per_pair": n_trans, "f16_mfma_flops_per_pair": n_mfma,
                      "achieved_Gpair_s": ach,
                      "trans_peak_Gpair_s": trans_peak, "frac_of_trans_peak": ach / trans_peak,
                      "mix_peak_Gpair_s": peak, "frac_of_mix_peak": ach / peak,
                      "frac_of_sincos_pair_peak": ach / (PEAK_SINCOS_PAIRS / 1e9),
                      "traffic": traffic_from_profile(src, name, shapes[kind])}
    kern["binning"] = {"avg_ms": binr["ms"] / max(binr["launches"], 1), "launches": binr["launches"]}
    dom = max(("forward_fp32c", "adjoint_fp32c"), key=lambda k: kern[k]["avg_ms"])
    if lattice:
        # the factorized form evaluates no sine per pair: its own instruction-mix bound
        roofline = {"bound": "alu", "kernel": dom, "achieved": kern[dom]["achieved_Gpair_s"],
                    "peak": kern[dom]["mix_peak_Gpair_s"], "unit": "Gpair/s",
                    "frac": kern[dom]["frac_of_mix_peak"], "traffic": kern[dom]["traffic"],
                    "peak_kind": "instruction mix incl. FP16 matrix flops"}
    else:
        roofline = {"bound": "alu", "kernel": dom, "achieved": kern[dom]["achieved_Gpair_s"],
                    "peak": kern[dom]["trans_peak_Gpair_s"], "unit": "Gpair/s",
                    "frac": kern[dom]["frac_of_trans_peak"], "traffic": kern[dom]["traffic"],
                    "peak_kind": "v_sin_f32 + v_cos_f32 issue (256 CUs x 2.4 GHz x 32 lanes / transcendentals per pair)"}

    # accuracy against the exact FP64 form at the final positions, and FP64 timing
    extra = {}
    if not args.no_fp64:
        api.timing_enable(True)
        I64, amp64 = api.intensity(pos, f, q, "fp64", return_amp=True)
        _, w64 = api.speckle_loss(I64, It)
        g64 = api.intensity_grad(pos, f, q, amp64, w64, "fp64", out_dtype=torch.float64)
        torch.cuda.synchronize()
        t64f = api.timing_read("fwd64")["ms"]
        t64g = api.timing_read("grad64")["ms"]
        api.timing_enable(False)
        # the timed plan (same form and tile shapes) at the final positions
        I32, amp32 = plan.intensity(pos, f)
        _, w32 = api.speckle_loss(I32, It)
        g32 = plan.grad(pos, f, amp32, w32, retile=False,
                        g64=torch.empty((N, 3), dtype=torch.float64, device=dev))
        g32k = plan.grad(pos, f, amp64, w64, retile=False,
                         g64=torch.empty((N, 3), dtype=torch.float64, device=dev))
        torch.cuda.synchronize()
        I64h, I32h = I64.cpu().numpy(), I32.cpu().numpy()
        inc = float(np.sum(f_np ** 2))
        e_I = float(np.max(np.abs(I32h - I64h) / np.maximum(I64h, inc)))
        g64h = g64.cpu().numpy()
        extra["accuracy_vs_fp64_form"] = {
            "e_I_scaled": e_I,
            "e_I_l2": float(np.linalg.norm(I32h - I64h) / np.linalg.norm(I64h)),
            "e_grad_kernel": rel_grad_err(g32k.cpu().numpy(), g64h),
            "e_grad_chain_r0": e_chain_r0,
            "e_grad_chain_final": rel_grad_err(g32.cpu().numpy(), g64h),
            "tolerance": 1e-5,
            "note": ("e_I and e_grad_kernel are the kernels' errors (the adjoint fed the FP64 amplitude "
                     "and dL/dI); e_grad_chain is forward -> loss -> adjoint in FP32C against the same chain "
                     "in FP64, at r0 and after the timed steps, where I - I_t is small and the loss amplifies "
                     "the forward's relative error"),
        }
        fp64_ms = t64f + t64g
        extra["fp64_form"] = {"fwd_ms": t64f, "grad_ms": t64g,
                              "pairs_per_s": pairs_step / (fp64_ms * 1e-3),
                              "speedup_fp32c_kernels": fp64_ms / (kern["forward_fp32c"]["avg_ms"] + kern["adjoint_fp32c"]["avg_ms"]),
                              "speedup_fp32c_step": fp64_ms / ms_step}
        log("accuracy", extra["accuracy_vs_fp64_form"], "fp64", extra["fp64_form"])
        cpu_amp, cpu_w = amp64.cpu().numpy(), w64.cpu().numpy()
    else:
        cpu_amp = np.zeros((Q, 2))
        cpu_w = np.zeros(Q)
    plan.close()
    for k in (0, 1):
        api.set_tile_shape(k, **old_shapes[k])

    result = {
        "metric": METRIC,
        "value": value,
        "unit": UNIT,
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "fp16-split x2 (matrix), f32 epilogue" if lattice else "f32",
        "data": "synthetic",
        "config": {"workload": "differentiation: N=65536 uniform atoms (rho 0.021/A^3), f=1, 512x512 "
                               "planar q in [-3,3]/A, FP32C forward + loss + FP32C adjoint + GD update",
                   "form": form,
                   "graph": bool(args.graph),
                   "n_atoms": N, "n_q": Q, "pairs_per_step": pairs_step,
                   "precision": ("fp32c: FP32 sine/cosine and tile sums, FP64 phase bases and folds"
                                 if not lattice else "fp32c lattice: FP16 hi/lo split factors on matrix cores"),
                   "tile_shape_fwd": shapes[0], "tile_shape_grad": shapes[1]},
        "roofline": roofline,
        # headline fraction: step pair evaluations per second over the sincos-pair rate
        # R_pair (one v_sin + one v_cos per pair at 32 transcendental lanes/clk/CU, nominal)
        "valu_roofline_frac": value / (PEAK_SINCOS_PAIRS / 1e9),
        "kernels": kern,
    }
    if tuned is not None:
        result["autotune"] = {k: tuned[k] for k in ("source", "key", "forward_ms", "gradient_ms") if k in tuned}
        result["autotune"]["note"] = "forward_ms / gradient_ms: the picked shapes' whole calls when tuned"
    result.update(extra)
    if not args.no_probe and form == "per-pair":
        result["measured_peaks"] = {
            "sincos_lane_ops_per_s": api.roofline_probe(0),
            "fma32_lane_ops_per_s": api.roofline_probe(1),
            "fma64_lane_ops_per_s": api.roofline_probe(2),
            "copy_bytes_per_s": api.roofline_probe(3, 1 << 30),
            "read_bytes_per_s": api.roofline_probe(6, 1 << 31),
            "f16_mfma_flops_per_s": api.roofline_probe(4),
            "f16_mfma_flops_per_s_with_8_fma32_each": api.roofline_probe(5),
        }
        # the same fraction against R_pair from the measured v_sin + v_cos issue rate
        result["valu_roofline_frac_measured"] = value / (result["measured_peaks"]["sincos_lane_ops_per_s"] / 2 / 1e9)
    if not args.no_cpu_baseline and form == "per-pair":
        log("cpu baseline (oracle) ...")
        result["cpu_baseline"] = cpu_baseline(r0, f_np, q_np, cpu_amp, cpu_w, budget_s=args.cpu_budget)
    return result


def run_reductions(args):
    """g2 (trajectory shape: 200 frames x 256^2 pixels, 32 rings, 100 lags) and XSVS
    (XSVS shape: 1024 frames x 1024^2 pixels, 64 rings, W = 1..256) on seeded synthetic
    exponential intensities already in GPU memory, whole calls timed with HIP events.
    g2 is FP64-FMA work (over the pixels inside the rings and lags tau < n_tau, F - tau
    products each) on 105 MB of intensities: its roofline is the FP64 FMA rate; F(q, tau)
    (same shape, complex amplitudes, 4 FMA per product) likewise.  XSVS reads the
    in-ring intensities once (both moments of Eq. (bq_Iq) from one read): its
    roofline is HBM, reported against the nominal 8 TB/s and against the read rate
    of the library's streaming probe measured in the same run."""
    import torch
    from paper_2204_13241_amd import api, inputs
    out = {}
    # streaming rates of the library's probes on this GPU (16-byte loads, four in flight)
    read_rate, copy_rate = api.roofline_probe(6, 1 << 31), api.roofline_probe(3, 1 << 30)
    out["measured_streaming"] = {"read_GB_s": read_rate / 1e9, "copy_GB_s_read_plus_write": copy_rate / 1e9}
    gen = torch.Generator(device="cuda:0")
    for name, F, n_det, q_max, rings, kw in (("g2", 200, 256, 1.5, 32, {"n_tau": 100}),
                                            ("isf", 200, 256, 1.5, 32, {"n_tau": 100}),
                                            ("xsvs", 1024, 1024, 2.0, 64, {"n_levels": 9})):
        gen.manual_seed(2024)
        q = torch.as_tensor(inputs.ewald_detector(n_det, q_max), dtype=torch.float64, device="cuda:0")
        edges = inputs.ring_edges(rings, q_max)
        if name == "isf":
            I = torch.empty((F, q.shape[0], 2), dtype=torch.float64, device="cuda:0").normal_(generator=gen)
            call = lambda: api.isf_rings(I, q, edges, kw["n_tau"], 1.0)
        else:
            I = torch.empty((F, q.shape[0]), dtype=torch.float64, device="cuda:0").exponential_(1.0, generator=gen)
            call = (lambda: api.g2_rings(I, q, edges, kw["n_tau"])) if name == "g2" else \
                   (lambda: api.xsvs_contrast(I, q, edges, kw["n_levels"]))
        call()
        used = int(api.isf_rings(I, q, edges, 1, 1.0)[1].sum()) if name == "isf" else \
            int(api.g2_rings(I[:2], q, edges, 1)[1].sum())   # pixels inside the rings
        torch.cuda.synchronize()
        api.timing_enable(True)
        for _ in range(args.red_reps):
            call()
        torch.cuda.synchronize()
        rec = api.timing_read(name)
        api.timing_enable(False)
        ms = rec["ms"] / max(rec["launches"], 1)
        Qn = int(q.shape[0])
        nbytes = F * used * (16 if name == "isf" else 8)
        rec = {"frames": F, "pixels": Qn, "pixels_in_rings": used, "rings": rings, **kw,
               "avg_ms": ms, "intensity_bytes": nbytes}
        if name in ("g2", "isf"):
            nt = kw["n_tau"]
            fma = used * (nt * F - nt * (nt - 1) // 2) * (4 if name == "isf" else 1)
            ach = fma / (ms * 1e-3)
            rec.update({"bound": "fp64", "fma_per_call": fma, "achieved_TFMA_s": ach / 1e12,
                        "peak_TFMA_s": PEAK_FMA64 / 1e12, "frac": ach / PEAK_FMA64,
                        "input_GB_s": nbytes / (ms * 1e-3) / 1e9})
            log("%s: %.3f ms, %.2f TFMA/s (%.1f%% of FP64 FMA)" % (name, ms, ach / 1e12, 100 * ach / PEAK_FMA64))
        else:
            alg = nbytes
            rec.update({"bound": "hbm", "algorithmic_bytes": alg, "achieved_GB_s": alg / (ms * 1e-3) / 1e9,
                        "peak_GB_s": PEAK_HBM / 1e9, "frac": alg / (ms * 1e-3) / PEAK_HBM,
                        "frac_of_measured_read": alg / (ms * 1e-3) / read_rate})
            log("xsvs: %.3f ms, %.0f GB/s of in-ring intensities read once (%.1f%% of HBM)"
                % (ms, rec["achieved_GB_s"], 100 * rec["frac"]))
        out[name] = rec
        del I
        torch.cuda.empty_cache()
    out.update(run_frames(args, copy_rate))
    return out


def run_frames(args, copy_rate=None):
    """Frame sums and kappa histograms (superposed configurations, exposure integrals,
    Eq. (Erlang)) on seeded exponential intensities in GPU memory: 16-frame exposure sums
    of the 1024-frame, 1M-pixel XSVS shape (HBM-bound: the frames read once, the sums
    written once) and the kappa histogram of the 200-frame, 65,536-pixel g2 shape."""
    import torch
    from paper_2204_13241_amd import api, inputs
    out = {}
    gen = torch.Generator(device="cuda:0")
    gen.manual_seed(2025)

    def timed(fn, reps):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps
    F, Q, W = 1024, 1024 * 1024, 16
    I = torch.empty((F, Q), dtype=torch.float64, device="cuda:0").exponential_(1.0, generator=gen)
    ms = timed(lambda: api.frame_sums(I, F // W, W, W, 1), args.red_reps)
    nbytes = F * Q * 8 + (F // W) * Q * 8
    out["frame_sums"] = {"frames": F, "pixels": Q, "window": W, "avg_ms": ms, "bound": "hbm",
                         "algorithmic_bytes": nbytes, "achieved_GB_s": nbytes / (ms * 1e-3) / 1e9,
                         "peak_GB_s": PEAK_HBM / 1e9, "frac": nbytes / (ms * 1e-3) / PEAK_HBM}
    if copy_rate:
        out["frame_sums"]["frac_of_measured_copy"] = nbytes / (ms * 1e-3) / copy_rate
    log("frame sums: %.3f ms, %.0f GB/s (%.1f%% of HBM)" % (ms, out["frame_sums"]["achieved_GB_s"],
                                                          100 * out["frame_sums"]["frac"]))
    del I
    torch.cuda.empty_cache()
    F, n_det = 200, 256
    q = torch.as_tensor(inputs.ewald_detector(n_det, 1.5), dtype=torch.float64, device="cuda:0")
    I = torch.empty((F, q.shape[0]), dtype=torch.float64, device="cuda:0").exponential_(1.0, generator=gen)
    edges = inputs.ring_edges(32, 1.5)
    ms = timed(lambda: api.ring_histogram(I, q, edges, 100, 8.0), args.red_reps)
    out["ring_histogram"] = {"frames": F, "pixels": int(q.shape[0]), "rings": 32, "bins": 100, "avg_ms": ms,
                             "input_GB_s": F * q.shape[0] * 8 / (ms * 1e-3) / 1e9}
    log("ring histogram: %.3f ms" % ms)
    return out


def run_species(args):
    """q-dependent form factors (two species, Gaussian-sum f_s(|q|)) on the
    differentiation workload's atoms and pixels: one-shot FP32C calls of the species
    path against the same calls with per-atom weights, whole calls timed with HIP
    events (host split of the species and plan building included in both)."""
    import torch
    from paper_2204_13241_amd import api, inputs
    dev = "cuda:0"
    w = inputs.workload_grad()
    r0, q_np, L = w.positions[0][0], w.q[0], w.box[0]
    N, Q = r0.shape[0], q_np.shape[0]
    rng = np.random.default_rng(2204)
    sp_np = (rng.random(N) < 2.0 / 3.0).astype(np.int32)            # 1/3 species 0, 2/3 species 1
    coef = np.array([[3.1, 2.3, 1.5, 0.9, 13.0, 5.5, 0.3, 30.0, 0.2],  # synthetic Gaussian sums
                     [0.49, 0.32, 0.14, 0.04, 10.5, 26.1, 3.1, 57.8, 0.003]])
    pos = torch.as_tensor(r0, dtype=torch.float64, device=dev)
    q = torch.as_tensor(q_np, dtype=torch.float64, device=dev)
    sp = torch.as_tensor(sp_np, dtype=torch.int32, device=dev)
    f_eff = torch.ones(N, dtype=torch.float64, device=dev)

    def timed(fn, reps=5):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps
    # one-shot calls build their plan each time: the better of two rounds of each
    ms_sp = min(timed(lambda: api.intensity_species(pos, sp, coef, q, precision="fp32c", box=L)) for _ in range(2))
    ms_plain = min(timed(lambda: api.intensity(pos, f_eff, q, precision="fp32c", box=L)) for _ in range(2))
    I64 = api.intensity_species(pos, sp, coef, q, precision="fp64")
    I32 = api.intensity_species(pos, sp, coef, q, precision="fp32c", box=L)
    fq = np.zeros((Q, 2))
    qq = np.sum(q_np * q_np, axis=1) / (16 * np.pi ** 2)
    for s_ in range(2):
        a, b, c = coef[s_, :4], coef[s_, 4:8], coef[s_, 8]
        fq[:, s_] = c + np.sum(a[None, :] * np.exp(-b[None, :] * qq[:, None]), axis=1)
    inc = (np.sum(sp_np == 0) * fq[:, 0] ** 2 + np.sum(sp_np == 1) * fq[:, 1] ** 2)
    e = float(np.max(np.abs(I32.cpu().numpy() - I64.cpu().numpy()) / np.maximum(I64.cpu().numpy(), inc)))
    # the plan form: species split and work lists built once, then forward + adjoint per step
    plan = api.SpeciesPlan([(N, 1, q, L)], sp, coef)
    I = torch.empty(Q, dtype=torch.float64, device=dev)
    amp = torch.empty((Q, 2), dtype=torch.float64, device=dev)
    g = torch.empty((N, 3), dtype=torch.float32, device=dev)
    wq = torch.as_tensor(np.random.default_rng(2205).standard_normal(Q), dtype=torch.float64, device=dev)

    def plan_step():
        plan.intensity(pos, I, amp)
        plan.grad(pos, amp, wq, retile=False, g32=g)
    ms_plan = min(timed(plan_step) for _ in range(2))
    e_plan = float(np.max(np.abs(I.cpu().numpy() - I64.cpu().numpy()) / np.maximum(I64.cpu().numpy(), inc)))
    lattice = plan.describe()["n_lattice_segments"]
    plan.close()
    rec = {"workload": "65,536 atoms (two species), 512x512 planar pixels, one frame, synthetic Gaussian-sum "
                       "form factors", "pairs": N * Q, "species_ms": ms_sp, "per_atom_weights_ms": ms_plain,
           "species_Gpair_s": N * Q / (ms_sp * 1e-3) / 1e9, "overhead": ms_sp / ms_plain - 1.0,
           "e_I_scaled_fp32c_vs_fp64": e,
           "plan_step_ms": ms_plan, "plan_step_Gpair_s": 2 * N * Q / (ms_plan * 1e-3) / 1e9,
           "plan_lattice_segments": lattice, "plan_e_I_scaled_vs_fp64": e_plan}
    log("species: %.3f ms per call (per-atom weights %.3f ms), %.0f Gpair/s, e_I %.2e; plan fwd+adjoint "
        "%.3f ms (%.0f Gpair/s, e_I %.2e)" % (ms_sp, ms_plain, rec["species_Gpair_s"], e, ms_plan,
                                             rec["plan_step_Gpair_s"], e_plan))
    return rec


def run_trajectory(args):
    """Trajectory workload (fcc 20^3 + jitter, 32,000 atoms, 200 Brownian frames,
    256x256 Ewald detector: 4.19e11 pairs, the general FP32C form) through one batch
    plan, then g2 on 32 rings: intensities of all frames per call, timed with HIP events;
    frame 0 checked against the FP64 form."""
    import torch
    from paper_2204_13241_amd import api, inputs
    dev = "cuda:0"
    w = inputs.workload_trajectory()
    frames, q_np, L = w.positions[0], w.q[0], w.box[0]
    F, N, Q = frames.shape[0], frames.shape[1], q_np.shape[0]
    pos = torch.as_tensor(frames, dtype=torch.float64, device=dev)
    f = torch.ones(N, dtype=torch.float64, device=dev)
    q = torch.as_tensor(q_np, dtype=torch.float64, device=dev)
    plan = api.Plan.single(N, F, q, L, forward_only=True)
    I = torch.empty((F, Q), dtype=torch.float64, device=dev)
    plan.intensity(pos, f, I, want_amp=False)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    reps = 3
    e0.record()
    for _ in range(reps):
        plan.intensity(pos, f, I, want_amp=False)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    desc = plan.describe()
    plan.close()
    g2, _ = api.g2_rings(I, q, w.edges, w.n_tau)
    # every frame in the exact FP64 form (bit for bit the oracle's), then g2 of both
    api.timing_enable(True)
    I64 = api.intensity(pos, f, q, precision="fp64")
    torch.cuda.synchronize()
    ms64 = api.timing_read("fwd64")["ms"]
    api.timing_enable(False)
    g2_64, _ = api.g2_rings(I64, q, w.edges, w.n_tau)
    inc = float(N)
    e = float(((I - I64).abs() / torch.clamp(I64, min=inc)).max())
    e_g2 = float(((g2 - g2_64).abs() / g2_64.abs()).max())
    rec = {"workload": "fcc 20^3 + 0.3 A jitter (32,000 atoms), 200 Brownian frames, 256x256 Ewald detector "
                       "(q_max 1.5)", "pairs": F * N * Q, "forward_ms": ms,
           "forward_Gpair_s": F * N * Q / (ms * 1e-3) / 1e9,
           "frac_of_sincos_pair_peak": F * N * Q / (ms * 1e-3) / PEAK_SINCOS_PAIRS,
           "form": "per-pair rows" if desc.get("n_row_segments", 0) == desc["n_segments"] else "per-pair general",
           "tile_shape_fwd": api.get_tile_shape(0),
           "plan": desc, "e_I_scaled_all_frames_vs_fp64": e,
           "e_g2_vs_fp64": e_g2, "g2_rings": int(g2.shape[0]), "g2_n_tau": int(g2.shape[1]),
           "fp64_forward_ms": ms64, "speedup_vs_fp64_form": ms64 / ms}
    log("trajectory: %.2f ms per 200-frame forward, %.0f Gpair/s, e_I %.2e, e_g2 %.2e (FP64 form %.1f ms)"
        % (ms, rec["forward_Gpair_s"], e, e_g2, ms64))
    del I64
    return rec


def run_batch(args):
    """Uneven batch (64 systems, N log-uniform in [2000, 64000), uniform positions, f 1.0 /
    2.5 at 80/20, 512x512 Ewald detectors to q_max 1.5): one plan over the whole batch, tile
    shapes autotuned among the per-pair shapes, forward and adjoint of every system in one
    persistent launch each, timed with HIP events; 4 systems checked against the FP64 form."""
    import torch
    from paper_2204_13241_amd import api, inputs, tune
    dev = "cuda:0"
    w = inputs.workload_batch()
    systems, pos_l, f_l = [], [], []
    q = torch.as_tensor(w.q[0], dtype=torch.float64, device=dev)   # one detector for all systems
    for r, f_, L in zip(w.positions, w.f, w.box):
        systems.append((r.shape[1], 1, q, L))
        pos_l.append(r[0])
        f_l.append(f_)
    pos = torch.as_tensor(np.concatenate(pos_l), dtype=torch.float64, device=dev)
    f = torch.as_tensor(np.concatenate(f_l), dtype=torch.float64, device=dev)
    n_atoms = sum(s[0] for s in systems)
    Q = int(q.shape[0])
    pairs = n_atoms * Q
    old = [api.get_tile_shape(0), api.get_tile_shape(1)]
    # a reduced candidate set: each candidate plan runs 3.0e11 pairs per launch
    fc = [(ql, occ, sp) for ql, occ in ((4, 0), (4, 4), (8, 0), (8, 4)) for sp in (32, 64, 128)]
    gc = [(al, occ, pc) for al, occ in ((2, 0), (2, 5), (4, 0)) for pc in (4096, 8192, 16384)]
    tuned = tune.tune(systems, pos, f, reps=3, use_cache=not args.retune, fwd_candidates=fc,
                      grad_candidates=gc, lattice=0)
    plan = api.Plan(systems)
    I = torch.empty(plan.total_out, dtype=torch.float64, device=dev)
    amp = torch.empty((plan.total_out, 2), dtype=torch.float64, device=dev)
    g = torch.empty((plan.total_pos, 3), dtype=torch.float32, device=dev)
    gen = torch.Generator(device=dev)
    gen.manual_seed(77)
    wq = torch.randn(plan.total_out, dtype=torch.float64, device=dev, generator=gen)
    plan.intensity(pos, f, I, amp)
    plan.grad(pos, f, amp, wq, retile=False, g32=g)
    torch.cuda.synchronize()
    api.timing_enable(True)
    reps = 5
    for _ in range(reps):
        plan.intensity(pos, f, I, amp)
        plan.grad(pos, f, amp, wq, retile=False, g32=g)
    torch.cuda.synchronize()
    fwd, grd = api.timing_read("fwd32"), api.timing_read("grad32")
    api.timing_enable(False)
    ms_f = fwd["ms"] / max(fwd["launches"], 1)
    ms_g = grd["ms"] / max(grd["launches"], 1)
    desc = plan.describe()
    # accuracy on 4 systems (smallest, two middle, largest) against the FP64 form
    order = np.argsort([s[0] for s in systems])
    check = [int(order[0]), int(order[len(order) // 3]), int(order[2 * len(order) // 3]), int(order[-1])]
    off = np.concatenate([[0], np.cumsum([s[0] for s in systems])])
    e_I, e_g = 0.0, 0.0
    g32b = plan.grad(pos, f, amp, wq, retile=False)  # FP32C adjoint of the whole batch
    for k in check:
        sl = slice(int(off[k]), int(off[k + 1]))
        I64, amp64 = api.intensity(pos[sl], f[sl], q, "fp64", return_amp=True)
        wk = wq[k * Q:(k + 1) * Q]
        g64 = api.intensity_grad(pos[sl], f[sl], q, amp64, wk, "fp64", out_dtype=torch.float64)
        inc = float((f[sl] ** 2).sum())
        Ik = I[k * Q:(k + 1) * Q]
        e_I = max(e_I, float(((Ik - I64).abs() / torch.clamp(I64, min=inc)).max()))
        e_g = max(e_g, rel_grad_err(g32b[sl].double().cpu().numpy(), g64.cpu().numpy()))
    plan.close()
    for k in (0, 1):
        api.set_tile_shape(k, **old[k])
    rec = {"workload": "64 systems, N log-uniform in [2000, 64000) (sum %d atoms), uniform positions at "
                       "0.021/A^3, f 1.0/2.5 at 80/20, 512x512 Ewald detectors (q_max 1.5)" % n_atoms,
           "pairs_per_pass": pairs, "forward_ms": ms_f, "adjoint_ms": ms_g,
           "forward_Gpair_s": pairs / (ms_f * 1e-3) / 1e9, "adjoint_Gpair_s": pairs / (ms_g * 1e-3) / 1e9,
           "fwd_adjoint_Gpair_s": 2 * pairs / ((ms_f + ms_g) * 1e-3) / 1e9,
           "frac_of_sincos_pair_peak": 2 * pairs / ((ms_f + ms_g) * 1e-3) / PEAK_SINCOS_PAIRS,
           "form": "per-pair", "tile_shapes": tuned.get("forward"), "tile_shapes_grad": tuned.get("gradient"),
           "autotune_source": tuned.get("source"), "plan": desc,
           "e_I_scaled_vs_fp64_4_systems": e_I, "e_grad_vs_fp64_4_systems": e_g,
           "e_grad_note": "FP32C forward amplitude + FP32C adjoint against the FP64 form of both, fixed random dL/dI",
           "checked_systems_atoms": [int(systems[k][0]) for k in check]}
    log("batch: fwd %.2f ms (%.0f Gpair/s), adjoint %.2f ms (%.0f Gpair/s), e_I %.2e, e_g %.2e"
        % (ms_f, rec["forward_Gpair_s"], ms_g, rec["adjoint_Gpair_s"], e_I, e_g))
    return rec


def run_xsvs_pairs(args):
    """XSVS workload (fcc 40^3 + 0.3 A jitter, 256,000 atoms, Brownian D dt = 0.005, 1024x1024
    Ewald detector to q_max 2) on its first `xsvs_frames` frames (all 1024 fit one
    forward-only plan): the pair sums of every frame through one plan (per-pair form), timed
    with HIP events, then the XSVS contrast of those FP32C intensities over 64 rings and
    W = 1 .. frames; the first min(frames, 64) frames in the exact FP64 form give e_I and
    e_beta (the contrast of those frames from both)."""
    import itertools
    import torch
    from paper_2204_13241_amd import api, inputs
    dev = "cuda:0"
    F = args.xsvs_frames
    w = inputs.workload_xsvs(materialize=False)
    frames = np.stack(list(itertools.islice(w.positions[0], F)))
    N, q_np, L = frames.shape[1], w.q[0], w.box[0]
    Q = q_np.shape[0]
    pos = torch.as_tensor(frames, dtype=torch.float64, device=dev)
    del frames
    f = torch.ones(N, dtype=torch.float64, device=dev)
    q = torch.as_tensor(q_np, dtype=torch.float64, device=dev)
    old = api.get_tile_shape(0)
    # one atom chunk per pixel group (4000 tiles): partial sums stay one per pixel and frame
    api.set_tile_shape(0, 64, 4, 4096, 0, 0, 0)
    plan = api.Plan.single(N, F, q, L, forward_only=True)
    I = torch.empty((F, Q), dtype=torch.float64, device=dev)
    plan.intensity(pos, f, I, want_amp=False)
    torch.cuda.synchronize()
    api.timing_enable(True)
    plan.intensity(pos, f, I, want_amp=False)
    torch.cuda.synchronize()
    rec_t = api.timing_read("fwd32")
    api.timing_enable(False)
    ms = rec_t["ms"] / max(rec_t["launches"], 1)
    desc = plan.describe()
    plan.close()
    api.set_tile_shape(0, **old)
    n_levels = min(int(math.log2(F)) + 1, 9)
    api.xsvs_contrast(I, q, w.edges, n_levels)  # first call sizes the working buffers
    api.timing_enable(True)
    api.xsvs_contrast(I, q, w.edges, n_levels)
    torch.cuda.synchronize()
    ms_xsvs = api.timing_read("xsvs")["ms"]
    api.timing_enable(False)
    F64 = min(F, 64)
    n_lv64 = int(math.log2(F64)) + 1
    api.timing_enable(True)
    I64 = api.intensity(pos[:F64], f, q, precision="fp64")
    torch.cuda.synchronize()
    ms64 = api.timing_read("fwd64")["ms"]
    api.timing_enable(False)
    beta32 = api.xsvs_contrast(I[:F64].contiguous(), q, w.edges, n_lv64)
    beta64 = api.xsvs_contrast(I64, q, w.edges, n_lv64)
    e_I = float(((I[:F64] - I64).abs() / torch.clamp(I64, min=float(N))).max())
    b32, b64 = beta32.cpu().numpy(), beta64.cpu().numpy()
    ok = np.isfinite(b64)
    e_b = float(np.max(np.abs(b32[ok] - b64[ok]) / np.abs(b64[ok])))
    pairs = F * N * Q
    rec = {"workload": "fcc 40^3 + 0.3 A jitter (256,000 atoms), Brownian D dt 0.005, 1024x1024 Ewald detector "
                       "(q_max 2), first %d of 1024 frames; XSVS over 64 rings, W = 1..%d" % (F, 2 ** (n_levels - 1)),
           "frames": F, "pairs": pairs, "forward_ms": ms, "forward_Gpair_s": pairs / (ms * 1e-3) / 1e9,
           "frac_of_sincos_pair_peak": pairs / (ms * 1e-3) / PEAK_SINCOS_PAIRS,
           "form": "per-pair", "tile_shape_fwd": {"q_per_lane": 4, "atom_split": 4096}, "plan": desc,
           "plan_kind": "forward only", "xsvs_ms": ms_xsvs, "beta_levels": n_levels,
           "fp64_frames": F64, "e_I_scaled_vs_fp64": e_I, "e_beta_vs_fp64": e_b,
           "fp64_forward_ms": ms64, "speedup_vs_fp64_form": (ms64 / F64) / (ms / F)}
    log("xsvs pairs: %d frames in %.1f ms (%.0f Gpair/s, plan %.1f GB), XSVS %.2f ms; first %d frames: e_I %.2e, "
        "e_beta %.2e (FP64 form %.0f ms)" % (F, ms, rec["forward_Gpair_s"], desc["device_bytes"] / 1e9, ms_xsvs,
                                            F64, e_I, e_b, ms64))
    del I64, I, pos
    torch.cuda.empty_cache()
    return rec


def run_fft(args):
    """FFT-based method (Sec. 3.2, Algorithm 2) beside the direct method, on the shape of
    the paper's Table 1: 4000 atoms (uniform stand-in for the liquid-argon frames) in a
    59.19 A box, N_grid = 400, k = 11, eta = 0.1485 A; the direct method on the same grid's
    81 x 81 slice (l = 0) and 81^3 block of wavevectors (per-pair FP32C plan and FP64 form).
    Accuracy of the FFT method against the exact FP64 form on the 81^3 block, and its
    convergence with N_grid at the wavevector (0, 14, -11) 2 pi / L (Sec. 4.2)."""
    import torch
    from paper_2204_13241_amd import api
    dev = "cuda:0"
    L, N, eta = 59.19, 4000, 0.1485
    rng = np.random.default_rng(2204)
    pos_np = rng.random((N, 3)) * L
    pos = torch.as_tensor(pos_np, dtype=torch.float64, device=dev)
    f = torch.ones(N, dtype=torch.float64, device=dev)

    def timed(fn, reps=5):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps
    n = 400
    k = int(math.floor(10.0 * eta * n / L)) + 1
    ms_fft = timed(lambda: api.fft_intensity(pos, f, L, n, eta, k))
    I_fft = api.fft_intensity(pos, f, L, n, eta, k)
    h = np.arange(-40, 41)
    hx, hy = np.meshgrid(h, h, indexing="ij")
    q_slice = np.stack([hx.ravel(), hy.ravel(), np.zeros(hx.size)], axis=-1) * (2 * math.pi / L)
    hx3, hy3, hz3 = np.meshgrid(h, h, h, indexing="ij")
    hkl3 = np.stack([hx3.ravel(), hy3.ravel(), hz3.ravel()], axis=-1)
    q_block = hkl3 * (2 * math.pi / L)
    out = {"workload": "4000 uniform atoms in a 59.19 A box (Table 1 shape), eta 0.1485 A, k %d" % k,
           "fft_n_grid": n, "fft_ms_per_frame": ms_fft}
    old_shape = api.get_tile_shape(0)
    for name, qn in (("slice_81x81", q_slice), ("block_81x81x81", q_block)):
        qt = torch.as_tensor(qn, dtype=torch.float64, device=dev)
        # a few forward shapes (small pixel sets need small items to fill the GPU); the best
        best = None
        for ql, split in ((1, 2), (1, 8), (2, 8), (4, 16), (8, 16), (8, 64)):
            api.set_tile_shape(0, 64, ql, split, 0, 0, 0)
            plan = api.Plan.single(N, 1, qt, L, forward_only=True)
            ms = timed(lambda: plan.intensity(pos, f, want_amp=False))
            plan.close()
            if best is None or ms < best[0]:
                best = (ms, ql, split)
        api.set_tile_shape(0, **old_shape)
        ms32 = best[0]
        api.timing_enable(True)
        api.intensity(pos, f, qt, "fp64")
        torch.cuda.synchronize()
        ms64 = api.timing_read("fwd64")["ms"]
        api.timing_enable(False)
        out[name] = {"pixels": int(qn.shape[0]), "direct_fp32c_ms": ms32, "direct_fp64_ms": ms64,
                     "direct_fp32c_Gpair_s": N * qn.shape[0] / (ms32 * 1e-3) / 1e9,
                     "direct_fp32c_shape": {"q_per_lane": best[1], "atom_split": best[2]},
                     "note": "plan call: binning, pair sum and combine"}
    # accuracy of the FFT method on the 81^3 block against the exact FP64 form
    qt = torch.as_tensor(q_block, dtype=torch.float64, device=dev)
    I64 = api.intensity(pos, f, qt, "fp64").cpu().numpy()
    idx = np.mod(hkl3, n)
    If = I_fft.cpu().numpy()[idx[:, 0], idx[:, 1], idx[:, 2]]
    out["fft_vs_direct_81cube_max_scaled_err"] = float(np.max(np.abs(If - I64) / np.maximum(I64, N)))
    # convergence with the grid at (0, 14, -11) 2 pi / L (eta fixed, k from 10 eta / delta)
    hq = np.array([[0, 14, -11]])
    I_ref = float(api.intensity(pos, f, torch.as_tensor(hq * (2 * math.pi / L), dtype=torch.float64,
                                                         device=dev), "fp64").cpu()[0])
    conv = []
    for ng in (100, 150, 200, 250, 300, 400):
        kk = int(math.floor(10.0 * eta * ng / L)) + 1
        In = api.fft_intensity(pos, f, L, ng, eta, kk)
        v = float(In[0, 14 % ng, (-11) % ng].cpu())
        conv.append({"n_grid": ng, "k": kk, "rel_err": abs(v - I_ref) / I_ref})
        del In
    out["convergence_at_0_14_m11"] = conv
    out["table1_paper_cpu_s_per_frame"] = {"direct_81x81": 4.1836, "direct_81cube": 416.8243, "fft_400": 0.4527,
                                           "hardware": "32 CPUs (paper, Table 1)"}
    torch.cuda.empty_cache()
    log("fft: %.2f ms per frame at N_grid 400; direct 81x81 %.3f ms, 81^3 %.2f ms (FP32C); err %.1e; conv %s"
        % (ms_fft, out["slice_81x81"]["direct_fp32c_ms"], out["block_81x81x81"]["direct_fp32c_ms"],
           out["fft_vs_direct_81cube_max_scaled_err"], ["%d:%.1e" % (c["n_grid"], c["rel_err"]) for c in conv]))
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-probe", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=20.0)
    ap.add_argument("--graph", action="store_true", help="time HIP-graph replays of the step")
    ap.add_argument("--no-tune", action="store_true", help="keep the default tile shapes")
    ap.add_argument("--retune", action="store_true", help="ignore the tuning cache")
    ap.add_argument("--no-reductions", action="store_true", help="skip the g2 / XSVS timings")
    ap.add_argument("--no-species", action="store_true", help="skip the form-factor (species) timing")
    ap.add_argument("--no-trajectory", action="store_true", help="skip the 200-frame trajectory timing")
    ap.add_argument("--only-reductions", action="store_true", help="time only g2 / XSVS")
    ap.add_argument("--no-step", action="store_true",
                    help="skip the headline step (profiling runs of the other legs only)")
    ap.add_argument("--no-batch", action="store_true", help="skip the 64-system uneven batch")
    ap.add_argument("--no-xsvs-pairs", action="store_true", help="skip the XSVS-workload pair sums")
    ap.add_argument("--no-lattice", action="store_true", help="skip the matrix-core lattice step")
    ap.add_argument("--xsvs-frames", type=int, default=64)
    ap.add_argument("--no-fft", action="store_true", help="skip the FFT-method comparison")
    ap.add_argument("--red-reps", type=int, default=3)
    ap.add_argument("--copy-probe", type=int, default=0, metavar="BYTES",
                    help="only run the library's plain copy kernel on BYTES (HBM counter calibration)")
    args = ap.parse_args()
    if args.copy_probe:
        from paper_2204_13241_amd import api
        rate = api.roofline_probe(3, args.copy_probe)
        print(json.dumps({"copy_bytes": args.copy_probe, "launches": 6, "bytes_per_s": rate}))
        return
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)
    import torch
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(2)
    if args.only_reductions:
        print(json.dumps({"reductions": run_reductions(args)}), flush=True)
        return
    res = {} if args.no_step else run_grad(args, "per-pair")
    if not args.no_lattice:
        lat = run_grad(argparse.Namespace(**dict(vars(args), no_cpu_baseline=True, no_probe=True)),
                       "lattice-mfma")
        res["lattice_mfma_step"] = {k: lat[k] for k in ("value", "unit", "ms_per_step", "dtype", "config",
                                                         "roofline", "valu_roofline_frac", "kernels",
                                                         "accuracy_vs_fp64_form") if k in lat}
        res["lattice_mfma_step"]["note"] = ("planar-grid factorization into complex matrix products on FP16 "
                                            "matrix cores: not a per-pair evaluation, so not the metric")
    if not args.no_batch:
        res["batch"] = run_batch(args)
    if not args.no_xsvs_pairs:
        res["xsvs_pairs"] = run_xsvs_pairs(args)
    if not args.no_fft:
        res["fft_method"] = run_fft(args)
    if not args.no_reductions:
        res["reductions"] = run_reductions(args)
    if not args.no_species:
        res["species_form_factors"] = run_species(args)
    if not args.no_trajectory:
        res["trajectory"] = run_trajectory(args)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
