"""g2 and XSVS reductions on the GPU against the oracle: bit-for-bit (Sec. 2.3)."""
import numpy as np
import pytest

import oracle
from paper_2204_13241_amd import inputs as X

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def api():
    from paper_2204_13241_amd import api
    return api


def _speckle_like(rng, F, Q, corr=0.9):
    """Exponentially distributed, time-correlated synthetic intensities [F, Q]."""
    z = rng.standard_normal((Q, 2))
    out = np.empty((F, Q))
    for t in range(F):
        z = corr * z + np.sqrt(1 - corr ** 2) * rng.standard_normal((Q, 2))
        out[t] = 0.5 * (z ** 2).sum(axis=1)
    return out


@pytest.mark.parametrize("F,n_det,n_tau,n_rings,seed", [
    (1, 8, 1, 3, 1), (20, 33, 10, 7, 2), (200, 64, 100, 32, 3), (9000, 5, 3, 2, 4),
    (130, 24, 120, 5, 8), (250, 20, 200, 4, 9), (400, 12, 400, 3, 10)])
def test_g2_bitwise(api, F, n_det, n_tau, n_rings, seed):
    """Lag blocks of 7, 8, 13 and 32 lags over 16 slots (one zero row after each series), the
    staged path for long series (F = 9000), a single frame."""
    from _gpu import dev, host, bitwise_equal
    rng = np.random.default_rng(seed)
    q = X.ewald_detector(n_det, 1.5)
    I = _speckle_like(rng, F, q.shape[0])
    I[:, 3 % q.shape[0]] = 0.0           # a dark pixel is left out
    edges = X.ring_edges(n_rings, 1.5)
    print("g2 F=%d Q=%d tau=%d rings=%d" % (F, q.shape[0], n_tau, n_rings), flush=True)
    g2, cnt = api.g2_rings(dev(I), dev(q), edges, n_tau)
    g2r, cntr = oracle.g2_rings(I, q, edges, n_tau)
    assert np.array_equal(host(cnt), cntr)
    assert bitwise_equal(host(g2), g2r)


@pytest.mark.parametrize("F,n_det,n_levels,n_rings,seed", [
    (1, 8, 1, 2, 1), (7, 21, 3, 5, 2), (64, 48, 7, 16, 3), (1024, 16, 9, 4, 4),
    (1000, 12, 10, 3, 6), (4096, 4, 13, 2, 7)])
def test_xsvs_bitwise(api, F, n_det, n_levels, n_rings, seed):
    from _gpu import dev, host, bitwise_equal
    rng = np.random.default_rng(seed)
    q = X.ewald_detector(n_det, 2.0)
    I = _speckle_like(rng, F, q.shape[0])
    edges = X.ring_edges(n_rings, 2.0)
    print("xsvs F=%d Q=%d levels=%d rings=%d" % (F, q.shape[0], n_levels, n_rings), flush=True)
    beta, win = api.xsvs_contrast(dev(I), dev(q), edges, n_levels, return_windows=True)
    br, wr = oracle.xsvs_contrast(I, q, edges, n_levels, want_windows=True)
    assert bitwise_equal(host(beta), br)
    assert bitwise_equal(host(win), wr)


def test_empty_rings_and_ragged_columns(api):
    """Rings past the detector's largest |q| stay empty (NaN, count 0); column counts
    (150, 75, 37 windows; 70 lags) that are not multiples of the 64-column tile."""
    from _gpu import dev, host, bitwise_equal
    rng = np.random.default_rng(6)
    q = X.ewald_detector(40, 2.0)
    I = _speckle_like(rng, 150, q.shape[0])
    edges = X.ring_edges(12, 4.0)
    beta, win = api.xsvs_contrast(dev(I), dev(q), edges, 3, return_windows=True)
    br, wr = oracle.xsvs_contrast(I, q, edges, 3, want_windows=True)
    assert np.isnan(br[:, -1]).all()
    assert bitwise_equal(host(beta), br)
    assert bitwise_equal(host(win), wr)
    g2, cnt = api.g2_rings(dev(I), dev(q), edges, 70)
    g2r, cntr = oracle.g2_rings(I, q, edges, 70)
    assert cntr[-1] == 0
    assert np.array_equal(host(cnt), cntr)
    assert bitwise_equal(host(g2), g2r)


def test_ring_edges_on_pixel_norms(api):
    """Pixels exactly on a ring edge go to the upper ring on both sides."""
    from _gpu import dev, host, bitwise_equal
    q = np.array([[0.5, 0, 0], [1.0, 0, 0], [0, 0, 1.5], [0.6, 0.8, 0.0], [0, 0, 0.0], [0, 3, 4.0]])
    I = np.arange(1.0, 1.0 + 4 * 6).reshape(4, 6)
    edges = [0.0, 1.0, 1.5]
    g2, cnt = api.g2_rings(dev(I), dev(q), edges, 2)
    g2r, cntr = oracle.g2_rings(I, q, edges, 2)
    assert np.array_equal(host(cnt), cntr)
    assert bitwise_equal(host(g2), g2r)


def test_ring_sizes_around_the_tree_groups(api):
    """Rings of 1, 31, 32, 33, 63, 64, 65, 96, 97, 127, 128, 129, 160, 1023, 1024, 1025 and
    1057 pixels, scattered over the pixel index: every partial chunk, every partial block of
    four chunks and the carries of the levels above, for g2 and for the XSVS moments (two
    launch groups of levels), bit for bit."""
    from _gpu import dev, host, bitwise_equal
    rng = np.random.default_rng(12)
    sizes = [1, 31, 32, 33, 63, 64, 65, 96, 97, 127, 128, 129, 160, 1023, 1024, 1025, 1057]
    edges = np.arange(len(sizes) + 1, dtype=np.float64)
    radius = np.concatenate([np.full(n, r + 0.5) for r, n in enumerate(sizes)])
    radius = radius[rng.permutation(radius.shape[0])]
    phi = rng.uniform(0.0, 2.0 * np.pi, radius.shape[0])
    q = np.stack([radius * np.cos(phi), radius * np.sin(phi), np.zeros_like(phi)], axis=1)
    F = 300
    I = _speckle_like(rng, F, q.shape[0])
    print("ring sizes: %d pixels, %d rings" % (q.shape[0], len(sizes)), flush=True)
    g2, cnt = api.g2_rings(dev(I), dev(q), edges, 20)
    g2r, cntr = oracle.g2_rings(I, q, edges, 20)
    assert np.array_equal(host(cnt), cntr) and list(cntr) == sizes
    assert bitwise_equal(host(g2), g2r)
    beta, win = api.xsvs_contrast(dev(I), dev(q), edges, 8, return_windows=True)
    br, wr = oracle.xsvs_contrast(I, q, edges, 8, want_windows=True)
    assert bitwise_equal(host(beta), br)
    assert bitwise_equal(host(win), wr)
