"""Species plans (q-dependent form factors in the plan form): identical to the one-shot
species calls on the same work lists, uneven batches against the oracle, HIP-graph replay."""
import numpy as np
import pytest
import torch

import oracle
from paper_2204_13241_amd import inputs as X

pytestmark = pytest.mark.gpu

COEF = np.array([[1.2, 2.1, 0.6, 0.3, 11.0, 3.2, 0.9, 0.21, 0.25],
                 [0.5, 0.3, 0.12, 0.08, 6.0, 2.0, 0.7, 0.15, 0.02],
                 [3.0, 2.2, 1.1, 0.4, 9.0, 2.5, 0.6, 0.1, 0.3]])


@pytest.fixture(scope="module")
def api():
    from paper_2204_13241_amd import api
    return api


def _scaled(I, I_ref, sp, q):
    f = oracle.form_factors(q, COEF)[:, sp]
    inc = np.sum(f * f, axis=1)
    return float(np.max(np.abs(I - I_ref) / np.maximum(I_ref, inc)))


def test_species_plan_matches_one_shot_bitwise(api):
    """With the general form only (lattice 2: rows and lattices ignored), the plan runs the
    one-shot call's kernels on the same
    species segments: identical intensities, amplitudes and gradients."""
    from _gpu import dev, host
    old = [api.get_tile_shape(k) for k in (0, 1)]
    for k in (0, 1):
        api.set_tile_shape(k, **dict(old[k], lattice=2))
    try:
        rng = np.random.default_rng(21)
        N, L = 3000, 40.0
        pos = dev(rng.uniform(0, L, (N, 3)))
        sp = dev(rng.integers(0, 3, N), dtype=torch.int32)
        q = dev(X.planar_grid(40, 3.0))
        wgt = dev(rng.standard_normal(q.shape[0]))
        print("species plan vs one-shot", flush=True)
        I1, a1 = api.intensity_species(pos, sp, COEF, q, "fp32c", box=L, return_amp=True)
        g1 = api.intensity_species_grad(pos, sp, COEF, q, a1, wgt, "fp32c", box=L)
        plan = api.SpeciesPlan([(N, 1, q, L)], sp, COEF)
        I2, a2 = plan.intensity(pos)
        g2 = plan.grad(pos, a2, wgt, retile=False)
        g3 = plan.grad(pos, a2, wgt, retile=True)
        torch.cuda.synchronize()
        assert np.array_equal(host(I1), host(I2)) and np.array_equal(host(a1).ravel(), host(a2).ravel())
        assert np.array_equal(host(g1), host(g2)) and np.array_equal(host(g2), host(g3))
        info = plan.describe()
        assert info["n_segments"] == 3 and info["device_bytes"] > 0
        plan.close()
    finally:
        for k in (0, 1):
            api.set_tile_shape(k, **old[k])


# matrix-core lattice shapes (opt-in form for planar grids) and the per-pair defaults
LATTICE_SHAPES = (dict(atoms_per_tile=64, q_per_lane=32, atom_split=64, pixel_split=0, waves_per_simd=0,
                       lattice=1),
                  dict(atoms_per_tile=64, q_per_lane=32, atom_split=128, pixel_split=8192, waves_per_simd=0,
                       lattice=1))


@pytest.mark.parametrize("lattice", [0, 1])
def test_species_plan_uneven_batch_against_oracle(api, lattice):
    """Two systems of uneven size and frame count, one planar (lattice form when asked
    for) and one Ewald detector, one species absent from the second system."""
    old = [api.get_tile_shape(0), api.get_tile_shape(1)]
    try:
        for k in (0, 1):
            api.set_tile_shape(k, **(LATTICE_SHAPES[k] if lattice else dict(old[k], lattice=0)))
        _species_uneven_batch(api, lattice)
    finally:
        for k in (0, 1):
            api.set_tile_shape(k, **old[k])


def _species_uneven_batch(api, lattice):
    from _gpu import dev, host, grad_err
    rng = np.random.default_rng(22)
    N, F, Ls = [700, 350], [2, 1], [32.0, 28.0]
    qs = [X.planar_grid(24, 2.5), X.ewald_detector(16, 1.5)]
    pos = [rng.uniform(0, Ls[i], (F[i], N[i], 3)) for i in range(2)]
    sp = [rng.integers(0, 3, N[0]).astype(np.int32), rng.integers(0, 2, N[1]).astype(np.int32)]
    systems = [(N[i], F[i], dev(qs[i]), Ls[i]) for i in range(2)]
    plan = api.SpeciesPlan(systems, dev(np.concatenate(sp), dtype=torch.int32), COEF)
    pos_d = dev(np.concatenate([p.reshape(-1, 3) for p in pos]))
    print("species plan batch", flush=True)
    I, amp = plan.intensity(pos_d)
    w = [rng.standard_normal((F[i], qs[i].shape[0])) for i in range(2)]
    g = plan.grad(pos_d, amp, dev(np.concatenate([x.ravel() for x in w])), retile=False,
                  g64=torch.empty((plan.total_pos, 3), dtype=torch.float64, device="cuda:0"))
    Ih, gh = host(I), host(g)
    off, poff = plan.batch.out_off, plan.batch.pos_off
    e_I, e_g = 0.0, 0.0
    for i in range(2):
        for t in range(F[i]):
            Ir, ar = oracle.intensity_species(pos[i][t], sp[i], COEF, qs[i])
            o = off[i] + t * qs[i].shape[0]
            e_I = max(e_I, _scaled(Ih[o: o + qs[i].shape[0]], Ir, sp[i], qs[i]))
            gr = oracle.intensity_species_grad(pos[i][t], sp[i], COEF, qs[i], ar, w[i][t])
            po = poff[i] + t * N[i]
            e_g = max(e_g, grad_err(gh[po: po + N[i]], gr))
    print("species plan lattice=%d: e_I %.2e  e_grad %.2e" % (lattice, e_I, e_g), flush=True)
    assert e_I < 1e-5 and e_g < 1e-5, (e_I, e_g)
    assert (plan.describe()["n_lattice_segments"] >= 1) == bool(lattice)
    plan.close()


def test_species_plan_refuses_the_per_atom_calls(api):
    from _gpu import dev
    rng = np.random.default_rng(23)
    q = dev(X.planar_grid(16, 2.0))
    plan = api.SpeciesPlan([(100, 1, q, 20.0)], dev(rng.integers(0, 3, 100), dtype=torch.int32), COEF)
    pos = dev(rng.uniform(0, 20.0, (100, 3)))
    with pytest.raises(RuntimeError, match="species plan"):
        api.Plan.intensity(plan, pos, dev(np.ones(100)))
    plan.close()
    with pytest.raises(RuntimeError, match="species"):
        api.SpeciesPlan([(100, 1, q, 20.0)], dev(np.full(100, 3), dtype=torch.int32), COEF)


def test_species_plan_graph_replay(api):
    """Capture forward + adjoint of a species plan; every replay equals the eager result."""
    from _gpu import dev, host
    rng = np.random.default_rng(24)
    N, L = 2000, 36.0
    q = dev(X.planar_grid(32, 3.0))
    pos = dev(rng.uniform(0, L, (N, 3)))
    plan = api.SpeciesPlan([(N, 1, q, L)], dev(rng.integers(0, 3, N), dtype=torch.int32), COEF)
    wgt = dev(rng.standard_normal(q.shape[0]))
    I = torch.empty(q.shape[0], dtype=torch.float64, device="cuda:0")
    amp = torch.empty((q.shape[0], 2), dtype=torch.float64, device="cuda:0")
    g = torch.empty((N, 3), dtype=torch.float32, device="cuda:0")
    print("species plan graph", flush=True)
    plan.intensity(pos, I, amp)
    plan.grad(pos, amp, wgt, retile=False, g32=g)
    torch.cuda.synchronize()
    I_ref, g_ref = host(I).copy(), host(g).copy()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        plan.intensity(pos, I, amp)
        plan.grad(pos, amp, wgt, retile=False, g32=g)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        plan.intensity(pos, I, amp)
        plan.grad(pos, amp, wgt, retile=False, g32=g)
    for rep in range(3):
        I.zero_()
        g.zero_()
        _ = (pos * 1.0).sum()
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        assert np.array_equal(host(I), I_ref), rep
        assert np.array_equal(host(g), g_ref), rep
    pos.add_(0.05)
    graph.replay()
    torch.cuda.synchronize()
    I_moved = host(I).copy()
    I2, _ = plan.intensity(pos)
    torch.cuda.synchronize()
    assert np.array_equal(host(I2), I_moved)
    del graph
    plan.close()


def test_plans_refuse_reusing_tiles_before_any_forward(api):
    """retile = 0 on a fresh plan has no atom tiles to reuse: a clear error, no launch."""
    from _gpu import dev
    rng = np.random.default_rng(25)
    q = dev(X.planar_grid(16, 2.0))
    pos = dev(rng.uniform(0, 20.0, (100, 3)))
    amp = dev(np.ones((q.shape[0], 2)))
    w = dev(np.ones(q.shape[0]))
    sp_plan = api.SpeciesPlan([(100, 1, q, 20.0)], dev(rng.integers(0, 3, 100), dtype=torch.int32), COEF)
    with pytest.raises(RuntimeError, match="retile = 0"):
        sp_plan.grad(pos, amp, w, retile=False)
    g = sp_plan.grad(pos, amp, w, retile=True)     # re-tiling is always allowed
    torch.cuda.synchronize()
    assert torch.isfinite(g).all()
    sp_plan.close()
    plan = api.Plan.single(100, 1, q, 20.0)
    f = dev(np.ones(100))
    with pytest.raises(RuntimeError, match="retile = 0"):
        plan.grad(pos, f, amp, w, retile=False)
    plan.intensity(pos, f)
    plan.grad(pos, f, amp, w, retile=False)
    torch.cuda.synchronize()
    plan.close()


def test_species_plan_without_atoms_gives_zero_intensity(api):
    from _gpu import dev, host
    q = dev(X.planar_grid(8, 2.0))
    plan = api.SpeciesPlan([(0, 2, q, 20.0)], torch.empty(0, dtype=torch.int32, device="cuda:0"), COEF)
    pos = torch.empty((0, 3), dtype=torch.float64, device="cuda:0")
    I, amp = plan.intensity(pos)
    g = plan.grad(pos, amp, dev(np.ones(2 * q.shape[0])), retile=False)
    torch.cuda.synchronize()
    assert np.array_equal(host(I), np.zeros(2 * q.shape[0])) and g.numel() == 0
    assert plan.describe()["n_segments"] == 0
    plan.close()
