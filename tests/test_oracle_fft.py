"""Pins of the FFT-method oracle (Sec. 3.2, Algorithm 2) to facts outside itself:
the shift theorem of the discrete transform, an explicit DFT on a tiny grid, and the
convergence to the exact direct sum (Sec. 4.2) as the grid is refined."""
import math

import numpy as np

import oracle
from oracle import fft_method as FM


def test_single_atom_on_a_grid_point_gives_f_squared():
    # the atom's Gaussian is the centred one moved by whole grid steps: its transform is
    # the centred transform times a phase, so I = f^2 at every grid wavevector
    L, n, eta = 12.0, 32, 0.5
    k = FM.cutoff_points(L, n, eta)
    delta = L / n
    I = FM.intensity(np.array([[7 * delta, 3 * delta, 30 * delta]]), np.array([2.5]), L, n, eta, k)
    # where the Gaussian's transform is small (near the grid's Nyquist corner) the ratio
    # magnifies rounding; the check covers the wavevectors where it is above 1e-4 of its peak
    G = np.abs(FM.gaussian_transform(L, n, eta, k))
    use = G > 1e-4 * G.max()
    assert use.sum() > 1000
    assert np.max(np.abs(I[use] - 6.25)) <= 1e-10 * 6.25


def test_translation_by_whole_grid_steps_leaves_intensity_unchanged():
    rng = np.random.default_rng(60)
    L, n, eta = 15.0, 40, 0.4
    k = FM.cutoff_points(L, n, eta)
    pos = rng.uniform(0, L, (30, 3))
    f = np.where(rng.random(30) < 0.3, 2.5, 1.0)
    I0 = FM.intensity(pos, f, L, n, eta, k)
    shift = np.array([5, -3, 17]) * (L / n)
    I1 = FM.intensity(np.mod(pos + shift, L), f, L, n, eta, k)
    scale = max(float(np.max(I0)), float(np.sum(f * f)))
    assert np.max(np.abs(I1 - I0)) <= 1e-10 * scale


def test_spreading_and_transform_against_an_explicit_dft():
    # the written-out definition on a tiny grid: every grid point's Gaussian weight summed
    # over atoms and periodic images within the k-point block, then sum_m rho_m e^{-2 pi i h.m/n}
    rng = np.random.default_rng(61)
    L, n, eta, k = 4.0, 6, 0.35, 3
    pos = rng.uniform(0, L, (4, 3))
    f = np.array([1.0, 2.5, 1.0, 0.5])
    delta = L / n
    norm = (1.0 / (math.sqrt(2 * math.pi) * eta)) ** 3
    rho = np.zeros((n, n, n))
    for i in range(4):
        first = [math.ceil(pos[i, c] / delta - k / 2) for c in range(3)]
        for a in range(k):
            for b in range(k):
                for c in range(k):
                    m = (first[0] + a, first[1] + b, first[2] + c)
                    d2 = sum((m[t] * delta - pos[i, t]) ** 2 for t in range(3))
                    rho[m[0] % n, m[1] % n, m[2] % n] += f[i] * norm * math.exp(-d2 / (2 * eta * eta))
    assert np.allclose(FM.spread(pos, f, L, n, eta, k), rho, rtol=0, atol=1e-13 * rho.max())
    h = np.arange(n)
    E = np.exp(-2j * math.pi * np.outer(h, h) / n)
    P = np.einsum("ax,by,cz,xyz->abc", E, E, E, rho)
    Pf = np.fft.fftn(FM.spread(pos, f, L, n, eta, k))
    assert np.allclose(Pf, P, rtol=0, atol=1e-12 * np.abs(P).max())


def test_converges_to_the_direct_method_as_the_grid_is_refined():
    # Sec. 4.2: with eta fixed and k the nearest integer above 10 eta / delta, the relative
    # difference to the exact direct sum (the FP64 form) falls fast with the grid size, down
    # to the level set by cutting each Gaussian at +-5 eta; a wider cut removes that floor
    rng = np.random.default_rng(62)
    L, eta = 14.0, 0.3
    pos = rng.uniform(0, L, (150, 3))
    f = np.ones(150)
    hs = np.array([[0, 3, -2], [1, -4, 2], [2, 2, 2], [-5, 0, 1]])
    q = hs * (2 * math.pi / L)
    I_ref, _ = oracle.intensity(pos, f, q)
    errs = []
    for n in (24, 36, 48, 72):
        k = FM.cutoff_points(L, n, eta)
        I = FM.intensity(pos, f, L, n, eta, k)
        Ih = np.array([I[h[0] % n, h[1] % n, h[2] % n] for h in hs])
        errs.append(float(np.max(np.abs(Ih - I_ref) / np.maximum(I_ref, 150.0))))
    print("FFT method vs direct, n = 24, 36, 48, 72:", ["%.1e" % e for e in errs])
    assert errs[0] > 1e-2 and errs[0] > 10 * errs[1] > 100 * errs[2]
    assert errs[2] < 1e-6 and errs[3] < 1e-6
    n = 72
    k_wide = int(math.floor(14 * eta * n / L)) + 1
    I = FM.intensity(pos, f, L, n, eta, k_wide)
    Ih = np.array([I[h[0] % n, h[1] % n, h[2] % n] for h in hs])
    assert float(np.max(np.abs(Ih - I_ref) / np.maximum(I_ref, 150.0))) < 1e-10
