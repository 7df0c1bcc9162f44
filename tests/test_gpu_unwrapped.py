"""FP32C form on positions outside the simulation cell: unwrapped Brownian frames that
drift out of [0, L) and a frame shifted rigidly far outside.  The atoms are binned over
each frame's own bounding box, so tiles stay compact; intensities and gradients against
the oracle (tolerance 1e-5)."""
import numpy as np
import pytest
import torch

import oracle
from paper_2204_13241_amd import inputs as X

from _gpu import dev, grad_err, host

pytestmark = pytest.mark.gpu
TOL = 1e-5


@pytest.fixture(scope="module")
def api():
    from paper_2204_13241_amd import api
    return api


def _frames():
    rng = np.random.default_rng(70)
    n = 1372  # fcc 7^3
    L = X.box_for(n)
    r0 = X.wrap(X.fcc_lattice(7, L / 7) + 0.3 * rng.standard_normal((n, 3)), L)
    # unwrapped Brownian steps with a large step so atoms cross the faces
    frames = np.stack(list(X.brownian_frames(r0, 4, 2.5, None, rng)))
    shifted = r0 + np.array([3.0 * L, -2.0 * L, 0.5 * L])
    return np.concatenate([frames, shifted[None]]), L


def test_fp32c_outside_the_cell_against_oracle(api):
    frames, L = _frames()
    F, N = frames.shape[0], frames.shape[1]
    out_frac = float(np.mean((frames[:4] < 0) | (frames[:4] >= L)))
    print("unwrapped frames: %.1f%% of coordinates outside [0, L)" % (100 * out_frac), flush=True)
    assert out_frac > 0.02
    q = X.ewald_detector(48, 1.5)
    f = np.where(np.random.default_rng(71).random(N) < 0.2, 2.5, 1.0)
    plan = api.Plan.single(N, F, dev(q), L)
    I, amp = plan.intensity(dev(frames), dev(f))
    w = np.random.default_rng(72).standard_normal(F * q.shape[0])
    g = plan.grad(dev(frames), dev(f), amp, dev(w), retile=False,
                  g64=torch.empty((F * N, 3), dtype=torch.float64, device="cuda:0"))
    torch.cuda.synchronize()
    Ih, gh = host(I).reshape(F, -1), host(g).reshape(F, N, 3)
    plan.close()
    inc = float(np.sum(f * f))
    for t in range(F):
        Ir, ar = oracle.intensity(frames[t], f, q)
        e_I = float(np.max(np.abs(Ih[t] - Ir) / np.maximum(Ir, inc)))
        gr = oracle.intensity_grad(frames[t], f, q, ar, w[t * q.shape[0]:(t + 1) * q.shape[0]])
        e_g = grad_err(gh[t], gr)
        print("frame %d: e_I %.2e e_grad %.2e" % (t, e_I, e_g), flush=True)
        assert e_I <= TOL and e_g <= TOL, (t, e_I, e_g)


def test_fp32c_crowded_cells_against_oracle(api):
    """Positions that crowd a few binning cells (a dense cluster with one far atom, and a
    frame with every atom at one point): cells of more than 64 atoms are ordered by the
    bitmap ranking instead of the per-cell insertion sort.  Two frames (two segments),
    intensities and the first frame's gradient against the oracle, and a second call
    bit for bit equal to the first (the scatter into cells is unordered)."""
    rng = np.random.default_rng(73)
    n_cluster = 47 * 64          # the far atom then sits in a tile of its own
    N = n_cluster + 1
    cluster = rng.uniform(0.0, 20.0, (n_cluster, 3))
    f0 = np.concatenate([cluster, [[200.0, 200.0, 200.0]]])
    f1 = np.tile([[1.0, 2.0, 3.0]], (N, 1))
    frames = np.stack([f0, f1])
    q = X.ewald_detector(32, 1.5)
    f = np.where(rng.random(N) < 0.2, 2.5, 1.0)
    L = 20.0
    print("crowded cells: %d atoms, 2 frames, %d pixels" % (N, q.shape[0]), flush=True)
    plan = api.Plan.single(N, 2, dev(q), L)
    I, amp = plan.intensity(dev(frames), dev(f))
    I2, _ = plan.intensity(dev(frames), dev(f))
    w = rng.standard_normal(2 * q.shape[0])
    g = plan.grad(dev(frames), dev(f), amp, dev(w), retile=False,
                  g64=torch.empty((2 * N, 3), dtype=torch.float64, device="cuda:0"))
    torch.cuda.synchronize()
    Ih, gh = host(I).reshape(2, -1), host(g).reshape(2, N, 3)
    assert np.array_equal(host(I).view(np.uint64), host(I2).view(np.uint64))
    plan.close()
    inc = float(np.sum(f * f))
    for t in range(2):
        Ir, ar = oracle.intensity(frames[t], f, q)
        e_I = float(np.max(np.abs(Ih[t] - Ir) / np.maximum(Ir, inc)))
        print("frame %d: e_I %.2e" % (t, e_I), flush=True)
        assert e_I <= TOL, (t, e_I)
    gr = oracle.intensity_grad(frames[0], f, q, oracle.intensity(frames[0], f, q)[1], w[:q.shape[0]])
    e_g = grad_err(gh[0], gr)
    print("frame 0: e_grad %.2e" % e_g, flush=True)
    assert e_g <= TOL
    assert np.allclose(Ih[1], np.sum(f) ** 2, rtol=1e-6, atol=0.0)


def test_fp32c_one_cell_over_several_bitmap_windows(api):
    """140,001 atoms, all but one inside a 1 A cube: one cell of 140,000 atoms, ranked
    over two windows of the atom index range; against the oracle, twice bit for bit."""
    rng = np.random.default_rng(74)
    N = 140001
    pos = np.concatenate([rng.uniform(0.0, 1.0, (N - 1, 3)), [[1000.0, 0.0, 0.0]]])
    f = np.where(rng.random(N) < 0.2, 2.5, 1.0)
    q = X.ewald_detector(16, 1.0)
    print("one crowded cell: %d atoms, %d pixels" % (N, q.shape[0]), flush=True)
    plan = api.Plan.single(N, 1, dev(q), 1.0, forward_only=True)
    I, _ = plan.intensity(dev(pos), dev(f))
    I2, _ = plan.intensity(dev(pos), dev(f))
    torch.cuda.synchronize()
    assert np.array_equal(host(I).view(np.uint64), host(I2).view(np.uint64))
    plan.close()
    Ir, _ = oracle.intensity(pos, f, q)
    e_I = float(np.max(np.abs(host(I) - Ir) / np.maximum(Ir, float(np.sum(f * f)))))
    print("e_I %.2e" % e_I, flush=True)
    assert e_I <= TOL
