"""Lattice form of the forward pair sum: detector rows of q-vectors stepping by one
common vector (a planar grid stored row by row), against the oracle and against the
general form; sets that are not such lattices keep the general form bit for bit."""
import numpy as np
import pytest
import torch

import oracle
from paper_2204_13241_amd import inputs as X

pytestmark = pytest.mark.gpu
TOL = 1e-5


@pytest.fixture(scope="module")
def api():
    from paper_2204_13241_amd import api
    return api


@pytest.fixture
def shapes(api):
    old = api.get_tile_shape(0)
    yield
    api.set_tile_shape(0, **old)


def _rows(n1, n2, qlim, tilt=0.0, z0=0.0):
    """n1 rows of n2 pixels: q_x steps along a row, rows at their own q_y (and q_z =
    z0 + tilt * q_x, so tilt != 0 gives rows that step in z as well)."""
    x = np.linspace(-qlim, qlim, n2)
    y = np.linspace(-0.8 * qlim, 0.9 * qlim, n1)
    q = np.zeros((n1 * n2, 3))
    q[:, 0] = np.tile(x, n1)
    q[:, 1] = np.repeat(y, n2)
    q[:, 2] = z0 + tilt * q[:, 0]
    return q


def _system(n_atoms, seed):
    rng = np.random.default_rng(seed)
    L = X.box_for(n_atoms)
    r = X.uniform_positions(rng, n_atoms, L)
    f = np.where(rng.random(n_atoms) < 0.2, 2.5, 1.0)
    return r, f, L


def _plan_I(api, r, f, q, L, ql, lattice, split=8, occ=0):
    from _gpu import dev, host
    api.set_tile_shape(0, 64, ql, split, 0, occ, lattice)
    plan = api.Plan.single(r.shape[0], 1, dev(q), L)
    info = plan.describe()
    I, _ = plan.intensity(dev(r), dev(f), want_amp=False)
    torch.cuda.synchronize()
    out = host(I).copy()
    plan.close()
    return out, info


@pytest.mark.parametrize("ql,occ", [(2, 0), (4, 0), (8, 0), (32, 0), (32, 3)])
def test_lattice_rows_match_oracle(api, shapes, ql, occ):
    """40 rows x 75 pixels (neither a multiple of the 32-row x 8-run item nor of the
    64 x 64 matrix-core item), 3000 atoms, f = 1 or 2.5; the matrix-core form also
    bounded to 3 waves per SIMD."""
    from _gpu import scaled_err
    r, f, L = _system(3000, 21)
    q = _rows(40, 75, 3.0)
    print("lattice ql=%d occ=%d: %d pixels" % (ql, occ, q.shape[0]), flush=True)
    I, info = _plan_I(api, r, f, q, L, ql, 1, occ=occ)
    assert info["n_lattice_segments"] == 1
    ref = oracle.intensity(r, f, q)[0]
    e = scaled_err(I, ref, f)
    print("e_I lattice ql=%d: %.3g" % (ql, e))
    assert e < TOL
    I0, info0 = _plan_I(api, r, f, q, L, ql, 0)
    assert info0["n_lattice_segments"] == 0
    assert scaled_err(I, I0, f) < TOL


@pytest.mark.parametrize("ql", [4, 32])
def test_lattice_rows_stepping_in_z(api, shapes, ql):
    """Rows whose step has a z component (the non-planar lattice branch)."""
    from _gpu import scaled_err
    r, f, L = _system(2000, 22)
    q = _rows(33, 64, 2.5, tilt=0.3, z0=-0.2)
    I, info = _plan_I(api, r, f, q, L, ql, 1)
    assert info["n_lattice_segments"] == 1
    assert scaled_err(I, oracle.intensity(r, f, q)[0], f) < TOL


def test_non_lattice_sets_keep_general_form(api, shapes):
    """An Ewald detector and a grid with one pixel moved by 1e-9 per Angstrom are not
    lattices: the plan's results are bit for bit those of lattice = 0."""
    from _gpu import bitwise_equal
    r, f, L = _system(1500, 23)
    bad = _rows(24, 48, 2.0)
    bad[100, 0] += 1e-9
    for q in (X.ewald_detector(40, 1.5), bad):
        I1, info1 = _plan_I(api, r, f, q, L, 4, 1)
        I0, _ = _plan_I(api, r, f, q, L, 4, 0)
        assert info1["n_lattice_segments"] == 0
        assert bitwise_equal(I1, I0)


@pytest.mark.parametrize("ql", [8, 32])
def test_lattice_in_uneven_batch(api, shapes, ql):
    """A lattice system (2 frames) and an Ewald system (1 frame) in one plan (with the
    matrix-core shape the Ewald system runs the general form at 8 pixels per lane)."""
    from _gpu import dev, host, scaled_err
    ra, fa, La = _system(2500, 24)
    rb, fb, Lb = _system(900, 25)
    rng = np.random.default_rng(26)
    ra2 = np.stack([ra, ra + 0.2 * rng.standard_normal(ra.shape)])
    qa, qb = _rows(35, 70, 3.0), X.ewald_detector(30, 1.5)
    api.set_tile_shape(0, 64, ql, 16, 0, 0, 1)
    plan = api.Plan([(2500, 2, dev(qa), La), (900, 1, dev(qb), Lb)])
    info = plan.describe()
    assert info["n_segments"] == 3 and info["n_lattice_segments"] == 2
    I, _ = plan.intensity(dev(np.concatenate([ra2.reshape(-1, 3), rb])), dev(np.concatenate([fa, fb])),
                          want_amp=False)
    Ih = host(I)
    off = plan.batch.out_off
    for t in range(2):
        got = Ih[off[0] + t * qa.shape[0]: off[0] + (t + 1) * qa.shape[0]]
        assert scaled_err(got, oracle.intensity(ra2[t], fa, qa)[0], fa) < TOL
    assert scaled_err(Ih[off[1]: off[1] + qb.shape[0]], oracle.intensity(rb, fb, qb)[0], fb) < TOL
    plan.close()
