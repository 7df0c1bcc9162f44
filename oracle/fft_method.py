"""CPU oracle of the FFT-based method (Sec. 3.2, Algorithm 2), plain numpy in FP64.

TEST INFRASTRUCTURE ONLY, like the rest of this package: only the test suite, the
smoke check and the CPU-baseline leg of the benchmark may import it.

The method, in the order of Algorithm 2:
  1. a zero field rho on an n x n x n grid over the periodic box [0, L)^3, spacing
     delta = L / n, grid point m at position m delta;
  2. every atom i adds f_i (1 / (sqrt(2 pi) eta))^3 exp(-|x_m - r_i|^2 / (2 eta^2)) to
     the k grid points nearest to it along each axis (k^3 points, indices taken
     modulo n: periodic images), Eq. (modified_r) with the atom's form factor as weight;
  3. P = FFT(rho) (numpy.fft.fftn: P[h] = sum_m rho[m] exp(-2 pi i h.m / n)); at the
     wavevector q_h = 2 pi h / L the integral of Eq. (pq_rq_app_alt) is delta^3 P[h];
  4. f^eta on the same grid from the FFT of one Gaussian of the same width centred at
     the origin (k^3 points, zero elsewhere), delta^3 G[h];
  5. I(q_h) = |p^eta(q_h)|^2 / f^eta(q_h)^2 = |P[h]|^2 / G[h]^2, Eq. (Iq_pq_new) with
     the form factors already in the weights (q-independent f).
Frequencies follow numpy's FFT order: index h in [0, n) stands for h for h < n/2
and h - n above (numpy.fft.fftfreq(n) * n).
"""
from __future__ import annotations

import math

import numpy as np


def nearest_block(x: float, k: int) -> int:
    """First of the k grid indices nearest to the grid coordinate x: ceil(x - k/2)."""
    return int(math.ceil(x - 0.5 * k))


def spread(pos, f, L: float, n: int, eta: float, k: int) -> np.ndarray:
    """Step 2: the Gaussian-smeared density rho [n, n, n] (float64)."""
    pos = np.asarray(pos, dtype=np.float64).reshape(-1, 3)
    f = np.asarray(f, dtype=np.float64).reshape(-1)
    delta = L / n
    norm = (1.0 / (math.sqrt(2.0 * math.pi) * eta)) ** 3
    rho = np.zeros((n, n, n))
    off = np.arange(k)
    for i in range(pos.shape[0]):
        idx, g = [], []
        for c in range(3):
            m0 = nearest_block(pos[i, c] / delta, k)
            m = m0 + off
            d = m * delta - pos[i, c]
            idx.append(np.mod(m, n))
            g.append(np.exp(-d * d / (2.0 * eta * eta)))
        w = f[i] * norm * g[0][:, None, None] * g[1][None, :, None] * g[2][None, None, :]
        np.add.at(rho, (idx[0][:, None, None], idx[1][None, :, None], idx[2][None, None, :]), w)
    return rho


def gaussian_transform(L: float, n: int, eta: float, k: int) -> np.ndarray:
    """Step 4: FFT of one Gaussian centred at the origin on its k^3 nearest grid points."""
    return np.fft.fftn(spread(np.zeros((1, 3)), np.ones(1), L, n, eta, k))


def intensity(pos, f, L: float, n: int, eta: float, k: int) -> np.ndarray:
    """Steps 1-5: I on every grid wavevector [n, n, n] in FFT order."""
    P = np.fft.fftn(spread(pos, f, L, n, eta, k))
    G = gaussian_transform(L, n, eta, k)
    return (P.real ** 2 + P.imag ** 2) / (G.real ** 2 + G.imag ** 2)


def grid_wavevectors(L: float, n: int) -> np.ndarray:
    """q_h = 2 pi h / L for every grid index [n, n, n, 3], FFT order."""
    h = np.fft.fftfreq(n) * n
    hx, hy, hz = np.meshgrid(h, h, h, indexing="ij")
    return np.stack([hx, hy, hz], axis=-1) * (2.0 * math.pi / L)


def cutoff_points(L: float, n: int, eta: float) -> int:
    """k of the paper: the nearest integer greater than 10 eta / delta."""
    return int(math.floor(10.0 * eta * n / L)) + 1
