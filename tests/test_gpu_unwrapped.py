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
