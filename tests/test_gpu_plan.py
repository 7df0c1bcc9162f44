"""Batch plans: identical to the one-shot calls, uneven batches, HIP-graph replay."""
import numpy as np
import pytest
import torch

import oracle
from paper_2204_13241_amd import inputs as X

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def api():
    from paper_2204_13241_amd import api
    return api


def test_plan_matches_one_shot_bitwise(api):
    """With the general form only (lattice 2: rows and lattices ignored), a plan runs the
    one-shot call's kernels on the same work lists: identical results."""
    from _gpu import dev, host, bitwise_equal
    old = [api.get_tile_shape(k) for k in (0, 1)]
    for k in (0, 1):
        api.set_tile_shape(k, **dict(old[k], lattice=2))
    try:
        _plan_vs_one_shot(api)
    finally:
        for k in (0, 1):
            api.set_tile_shape(k, **old[k])


def _plan_vs_one_shot(api):
    from _gpu import dev, host, bitwise_equal
    w = X.workload_grad(n_atoms=5000, n_det=64)
    r0, f, q, L = dev(w.positions[0][0]), dev(w.f[0]), dev(w.q[0]), w.box[0]
    I1, a1 = api.intensity(r0, f, q, "fp32c", box=L, return_amp=True)
    wgt = dev(np.random.default_rng(3).standard_normal(q.shape[0]))
    g1 = api.intensity_grad(r0, f, q, a1, wgt, "fp32c", box=L)
    plan = api.Plan.single(5000, 1, q, L)
    I2, a2 = plan.intensity(r0, f)
    g2 = plan.grad(r0, f, a2, wgt, retile=False)
    g3 = plan.grad(r0, f, a2, wgt, retile=True)
    torch.cuda.synchronize()
    assert bitwise_equal(host(I1), host(I2)) and bitwise_equal(host(a1).ravel(), host(a2).ravel())
    assert np.array_equal(host(g1), host(g2)) and np.array_equal(host(g2), host(g3))
    plan.close()


def test_plan_uneven_batch_against_oracle(api):
    """Systems of uneven atom count and frames in one plan (reduced uneven batch)."""
    from _gpu import dev, host, scaled_err
    w = X.workload_batch(n_sys=5, n_lo=100, n_hi=4000, n_det=24, seed=11)
    rng = np.random.default_rng(5)
    systems, pos_list, f_list, refs = [], [], [], []
    for k, (p, f, q, L) in enumerate(zip(w.positions, w.f, w.q, w.box)):
        nf = 1 + (k % 3)
        fr = np.concatenate([p, p + 0.3 * rng.standard_normal((nf - 1,) + p.shape[1:])]) if nf > 1 else p
        systems.append((fr.shape[1], nf, dev(q), L))
        pos_list.append(fr.reshape(-1, 3))
        f_list.append(f)
        refs.append(np.stack([oracle.intensity(fr[t], f, q)[0] for t in range(nf)]))
    plan = api.Plan(systems)
    I, _ = plan.intensity(dev(np.concatenate(pos_list)), dev(np.concatenate(f_list)))
    Ih = host(I)
    off = plan.batch.out_off
    for k, r in enumerate(refs):
        got = Ih[off[k]: off[k] + r.size].reshape(r.shape)
        assert scaled_err(got, r, f_list[k]) < 1e-5
    plan.close()


def test_forward_only_plan(api):
    """A forward-only plan (xs_plan_create_forward) over an uneven multi-frame batch gives the
    full plan's intensities and amplitudes bit for bit from less device memory; its grad()
    raises before launching anything."""
    from _gpu import dev, host, bitwise_equal
    from paper_2204_13241_amd import _lib
    rng = np.random.default_rng(17)
    systems, pos_list, f_list = [], [], []
    for k, (n, nf, n_det) in enumerate(((3000, 3, 48), (700, 1, 24), (1500, 2, 32))):
        L = X.box_for(n)
        q = X.ewald_detector(n_det, 1.5) if k != 1 else X.planar_grid(n_det, 2.0)
        systems.append((n, nf, dev(q), L))
        pos_list.append(X.uniform_positions(rng, n * nf, L))
        f_list.append(np.where(rng.random(n) < 0.2, 2.5, 1.0))
    pos, f = dev(np.concatenate(pos_list)), dev(np.concatenate(f_list))
    full = api.Plan(systems)
    fwd = api.Plan(systems, forward_only=True)
    I1, a1 = full.intensity(pos, f)
    I2, a2 = fwd.intensity(pos, f)
    torch.cuda.synchronize()
    d_full, d_fwd = full.describe(), fwd.describe()
    print("forward-only plan: %d bytes (full plan %d)" % (d_fwd["device_bytes"], d_full["device_bytes"]),
          flush=True)
    assert bitwise_equal(host(I1), host(I2)) and bitwise_equal(host(a1).ravel(), host(a2).ravel())
    assert d_fwd["device_bytes"] < d_full["device_bytes"]
    assert d_fwd["n_gradient_items"] == 0 and d_full["n_gradient_items"] > 0
    with pytest.raises(_lib.XsError):
        fwd.grad(pos, f, a2, dev(np.ones(full.total_out)), retile=True)
    full.close()
    fwd.close()


def test_plan_graph_replay(api):
    """Capture forward + adjoint in a HIP graph; every replay equals the eager result."""
    from _gpu import dev, host
    w = X.workload_grad(n_atoms=3000, n_det=48)
    L = w.box[0]
    q = dev(w.q[0])
    pos = dev(w.positions[0][0])
    f = dev(w.f[0])
    wgt = dev(np.random.default_rng(9).standard_normal(q.shape[0]))
    plan = api.Plan.single(3000, 1, q, L)
    I = torch.empty(q.shape[0], dtype=torch.float64, device=pos.device)
    amp = torch.empty((q.shape[0], 2), dtype=torch.float64, device=pos.device)
    g = torch.empty((3000, 3), dtype=torch.float32, device=pos.device)
    # eager reference, and warm-up on the capture stream
    plan.intensity(pos, f, I, amp)
    plan.grad(pos, f, amp, wgt, retile=False, g32=g)
    torch.cuda.synchronize()
    I_ref, g_ref = host(I).copy(), host(g).copy()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        plan.intensity(pos, f, I, amp)
        plan.grad(pos, f, amp, wgt, retile=False, g32=g)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        plan.intensity(pos, f, I, amp)
        plan.grad(pos, f, amp, wgt, retile=False, g32=g)
    for rep in range(4):
        I.zero_()
        g.zero_()
        _ = (pos * 1.0).sum()          # unrelated eager work between replays
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        assert np.array_equal(host(I), I_ref), rep
        assert np.array_equal(host(g), g_ref), rep
    # replay after moving the atoms in place: matches a fresh eager evaluation
    pos.add_(0.05)
    graph.replay()
    torch.cuda.synchronize()
    I_moved = host(I).copy()
    I2, _ = plan.intensity(pos, f)
    torch.cuda.synchronize()
    assert np.array_equal(host(I2), I_moved)
    del graph
    plan.close()


def test_training_step_graph_replay(api):
    """The whole differentiation step (plan forward, speckle loss, plan adjoint, position
    update) captured once: replays, with eager work between them, reproduce eager steps
    bit for bit."""
    from _gpu import dev, host
    w = X.workload_grad(n_atoms=2000, n_det=32)
    L = w.box[0]
    q = dev(w.q[0])
    f = dev(w.f[0])
    It = api.intensity(dev(w.extra["r_target"]), f, q, "fp64")
    plan = api.Plan.single(2000, 1, q, L)
    I = torch.empty(q.shape[0], dtype=torch.float64, device="cuda:0")
    amp = torch.empty((q.shape[0], 2), dtype=torch.float64, device="cuda:0")
    g = torch.empty((2000, 3), dtype=torch.float32, device="cuda:0")

    def step(pos):
        plan.intensity(pos, f, I, amp)
        loss, dLdI = api.speckle_loss(I, It)
        plan.grad(pos, f, amp, dLdI, retile=False, g32=g)
        api.position_step(pos, g, 0.01)
        return loss

    pos_e = dev(w.positions[0][0])
    for _ in range(3):
        step(pos_e)
    torch.cuda.synchronize()
    ref = host(pos_e).copy()
    pos_g = dev(w.positions[0][0])
    start = pos_g.clone()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        step(pos_g)                                   # warm-up on the capture stream
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    pos_g.copy_(start)
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=s):
        step(pos_g)
    pos_g.copy_(start)                                # capture does not run the work
    torch.cuda.synchronize()
    for _ in range(3):
        graph.replay()
        _ = (pos_g * 2.0).sum()                       # unrelated eager work between replays
        torch.cuda.synchronize()
    assert np.array_equal(host(pos_g), ref)
    del graph
    plan.close()
