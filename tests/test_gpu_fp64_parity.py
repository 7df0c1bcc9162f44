"""FP64 form on the GPU against the CPU oracle: bit-for-bit (Sec. 3.1 Algorithm 1)."""
import numpy as np
import pytest

import oracle
from paper_2204_13241_amd import inputs as X

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def api():
    from paper_2204_13241_amd import api
    return api


def _ref_frames(frames, f, q):
    I, A = [], []
    for r in frames:
        i, a = oracle.intensity(r, f, q)
        I.append(i)
        A.append(a)
    return np.stack(I), np.stack(A)


def test_plain_workload_bitwise(api):
    from _gpu import dev, host, bitwise_equal
    w = X.workload_plain()
    pos, f, q = w.positions[0], w.f[0], w.q[0]
    print("plain 1000 atoms x 64x64 planar pixels, FP64 form", flush=True)
    I, amp = api.intensity(dev(pos), dev(f), dev(q), "fp64", return_amp=True)
    Ir, Ar = _ref_frames(pos, f, q)
    assert bitwise_equal(host(I), Ir)
    assert bitwise_equal(host(amp), Ar)


@pytest.mark.parametrize("n_atoms,n_det,n_frames,seed", [
    (0, 16, 1, 1), (1, 16, 2, 2), (257, 23, 3, 3), (1000, 37, 2, 4), (3, 1, 1, 5)])
def test_ragged_and_degenerate_bitwise(api, n_atoms, n_det, n_frames, seed):
    from _gpu import dev, host, bitwise_equal
    rng = np.random.default_rng(seed)
    L = 30.0
    frames = rng.uniform(-5, L + 5, (n_frames, n_atoms, 3))   # positions outside the box too
    f = np.where(rng.random(n_atoms) < 0.2, 2.5, 1.0)
    q = X.ewald_detector(n_det, 2.0) if n_det > 1 else np.array([[0.3, -1.2, 0.7]])
    print("fp64 ragged N=%d Q=%d F=%d" % (n_atoms, q.shape[0], n_frames), flush=True)
    I, amp = api.intensity(dev(frames), dev(f), dev(q), "fp64", return_amp=True)
    Ir, Ar = _ref_frames(frames, f, q)
    assert bitwise_equal(host(I), Ir)
    assert bitwise_equal(host(amp), Ar)


def test_batch_of_systems_bitwise(api):
    from _gpu import dev, host, bitwise_equal
    rng = np.random.default_rng(21)
    systems, refs = [], []
    for n, nd, nf in [(100, 9, 2), (700, 20, 1), (33, 31, 3)]:
        L = X.box_for(n)
        fr = rng.uniform(0, L, (nf, n, 3))
        f = np.where(rng.random(n) < 0.2, 2.5, 1.0)
        q = X.ewald_detector(nd, 1.5)
        systems.append((dev(fr), dev(f), dev(q), L))
        refs.append(_ref_frames(fr, f, q)[0])
    print("fp64 batch of 3 systems", flush=True)
    out = api.intensity_systems(systems, "fp64")
    for o, r in zip(out, refs):
        assert bitwise_equal(host(o), r)


def test_gradient_fp64_bitwise(api):
    from _gpu import dev, host, bitwise_equal
    rng = np.random.default_rng(31)
    n, L = 300, 20.0
    pos = rng.uniform(0, L, (n, 3))
    f = np.where(rng.random(n) < 0.2, 2.5, 1.0)
    q = X.ewald_detector(17, 2.0)
    w = rng.standard_normal(q.shape[0])
    _, amp = oracle.intensity(pos, f, q)
    g_ref = oracle.intensity_grad(pos, f, q, amp, w)
    print("fp64 gradient N=300 Q=289", flush=True)
    g = api.intensity_grad(dev(pos), dev(f), dev(q), dev(amp), dev(w), "fp64",
                           out_dtype=__import__("torch").float64)
    assert bitwise_equal(host(g), g_ref)
