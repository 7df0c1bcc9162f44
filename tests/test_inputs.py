"""Seeded input generators: the geometry and statistics of the synthetic workloads.

The expected numbers are derived independently of the generator code: the
Ewald-sphere values from k = 2 pi / 1.305 per Angstrom (elastic scattering,
Sec. 2.1) with the half-angle construction worked out by hand, the box edges
from the number density 0.021 per cubic Angstrom.
"""
import math

import numpy as np
import pytest

from paper_2204_13241_amd import inputs


def test_box_edges_at_the_workload_density():
    # (N / 0.021)^(1/3) for the plain, trajectory, differentiation and XSVS sizes
    assert inputs.box_for(32000) == pytest.approx(115.0739, abs=5e-4)
    assert inputs.box_for(65536) == pytest.approx(146.135, abs=5e-4)
    assert inputs.box_for(256000) == pytest.approx(230.148, abs=5e-4)


@pytest.mark.parametrize("q_max,q_perp,corner", [
    (1.5, 1.4816893, 2.1497),
    (2.0, 1.9563863, 2.9016),
])
def test_ewald_detector_geometry(q_max, q_perp, corner):
    n = 8
    q = inputs.ewald_detector(n, q_max)
    k = 2.0 * math.pi / 1.305
    assert q.shape == (n * n, 3)
    # pixel 0 is the (-, -) corner, q_x fastest
    assert q[0, 0] == pytest.approx(-q_perp, abs=1e-7)
    assert q[n - 1, 0] == pytest.approx(q_perp, abs=1e-7)
    assert q[n * (n - 1), 1] == pytest.approx(q_perp, abs=1e-7)
    # elastic: |k_i + q| = |k_i| for every pixel
    kf = q + np.array([0.0, 0.0, k])
    assert np.max(np.abs(np.linalg.norm(kf, axis=1) - k)) < 1e-12
    assert np.linalg.norm(q[0]) == pytest.approx(corner, abs=1e-4)
    # the detector is symmetric under q_x -> -q_x and q_y -> -q_y (same q_z)
    grid = q.reshape(n, n, 3)
    assert np.array_equal(grid[:, ::-1, 0], -grid[:, :, 0])
    assert np.array_equal(grid[::-1, :, 1], -grid[:, :, 1])
    assert np.array_equal(grid[::-1, ::-1, 2], grid[:, :, 2])
    assert np.all(q[:, 2] <= 0.0)


def test_ewald_edge_midpoint_reaches_q_max():
    # an odd grid has a pixel at (Q_perp, 0): its |q| is q_max by construction
    for q_max in (1.5, 2.0):
        n = 9
        q = inputs.ewald_detector(n, q_max).reshape(n, n, 3)
        assert np.linalg.norm(q[n // 2, n - 1]) == pytest.approx(q_max, abs=1e-12)


def test_planar_grid_is_exactly_antisymmetric():
    for n, lim in ((64, 4.0), (512, 3.0), (7, 1.0)):
        q = inputs.planar_grid(n, lim)
        assert np.array_equal(q[::-1], -q)
        assert q[0, 0] == -lim and q[-1, 1] == lim
        assert np.all(q[:, 2] == 0.0)
        step = 2.0 * lim / (n - 1)
        assert np.allclose(np.diff(q[:n, 0]), step, rtol=0, atol=1e-14)


def test_planar_subpixels_average_to_the_pixel_centre():
    n, lim, s = 6, 2.0, 3
    sub = inputs.planar_subpixels(n, lim, s)
    assert sub.shape == (s * s, n * n, 3)
    assert np.allclose(sub.mean(axis=0), inputs.planar_grid(n, lim), rtol=0, atol=1e-14)
    step = 2.0 * lim / (n - 1)
    off = sub - inputs.planar_grid(n, lim)[None]
    assert np.max(np.abs(off[..., :2])) == pytest.approx(step * (0.5 - 0.5 / s), abs=1e-14)


def test_fcc_lattice_and_simple_cubic():
    a = 2.0
    r = inputs.fcc_lattice(3, a)
    assert r.shape == (4 * 27, 3)
    assert len({tuple(x) for x in r}) == r.shape[0]
    # nearest-neighbour distance of fcc is a / sqrt(2), twelve neighbours for an inner site
    d = np.linalg.norm(r - r[13 * 4], axis=1)
    d = d[d > 0]
    assert d.min() == pytest.approx(a / math.sqrt(2.0), abs=1e-12)
    assert np.count_nonzero(np.isclose(d, a / math.sqrt(2.0))) == 12
    sc = inputs.simple_cubic(4, 1.5)
    assert sc.shape == (64, 3) and sc.max() == pytest.approx(4.5)


def test_brownian_frames_wrap_and_step_statistics():
    rng = np.random.default_rng(7)
    L = 10.0
    r0 = inputs.uniform_positions(rng, 4000, L)
    frames = np.stack(list(inputs.brownian_frames(r0, 3, 0.1, L, np.random.default_rng(8))))
    assert np.array_equal(frames[0], r0)
    assert np.all(frames >= 0.0) and np.all(frames < L)
    # minimum-image displacement per component has the step's standard deviation
    dr = frames[1] - frames[0]
    dr -= L * np.round(dr / L)
    assert dr.std() == pytest.approx(0.1, rel=0.03)
    unwrapped = np.stack(list(inputs.brownian_frames(r0, 2, 0.1, None, np.random.default_rng(8))))
    assert np.allclose(inputs.wrap(unwrapped[1], L), frames[1], rtol=0, atol=1e-12)


def test_batch_workload_sizes_and_species_counts():
    w = inputs.workload_batch(n_sys=6, n_det=8)
    sizes = w.extra["sizes"]
    assert len(sizes) == 6 and all(2000 <= n < 64000 for n in sizes)
    for n, f, r, L in zip(sizes, w.f, w.positions, w.box):
        assert np.count_nonzero(f == 2.5) == int(round(0.2 * n))
        assert np.count_nonzero(f == 1.0) == n - int(round(0.2 * n))
        assert r.shape == (1, n, 3) and np.all(r >= 0) and np.all(r < L)
        assert L == pytest.approx((n / 0.021) ** (1.0 / 3.0))


def test_workloads_are_reproducible_from_their_seeds():
    a = inputs.workload_trajectory(n_cells=3, n_frames=4, n_det=8)
    b = inputs.workload_trajectory(n_cells=3, n_frames=4, n_det=8)
    assert np.array_equal(a.positions[0], b.positions[0])
    assert a.positions[0].shape == (4, 108, 3) and a.n_tau == 2
    g = inputs.workload_grad(n_atoms=256, n_det=8, n_fd=16)
    assert np.array_equal(g.extra["fd_atoms"], np.unique(g.extra["fd_atoms"]))
    assert g.extra["fd_atoms"].size == 16
    # the target is unwrapped: displacements are the noise itself
    assert (g.extra["r_target"] - g.positions[0][0]).std() == pytest.approx(0.2, rel=0.1)


def test_ring_edges_are_uniform_and_half_open_on_q_max():
    e = inputs.ring_edges(32, 1.5)
    assert e.shape == (33,) and e[0] == 0.0 and e[-1] == 1.5
    assert np.allclose(np.diff(e), 0.046875, rtol=0, atol=1e-15)
