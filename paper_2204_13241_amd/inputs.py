"""Seeded synthetic inputs: positions, form factors, wavevectors, rings.

This module holds no arithmetic of the method itself (no phases, sums,
intensities or reductions); it only builds inputs of the shapes used in the
paper's workloads.  Both the HIP path and the CPU oracle are fed from here.

Stand-ins for the paper's data (the molecular-dynamics trajectories of liquid
argon and water are not available): uniform random liquids, fcc crystals with
Gaussian jitter, and Brownian trajectories wrapped into a periodic cube, all at
number density 0.021 per cubic Angstrom.  Detector pixels are either a planar
q-grid (q_z = 0) or a spherical slice of reciprocal space on the Ewald sphere
(Sec. 2.1: elastic scattering, |k_i| = |k_f| = 2 pi / lambda; Sec. 4.3 shows
such a spherical slice).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Optional

import numpy as np

RHO = 0.021            # atoms per cubic Angstrom
WAVELENGTH = 1.305     # Angstrom


def box_for(n_atoms: int, rho: float = RHO) -> float:
    """Edge of the cube holding n_atoms at number density rho."""
    return (n_atoms / rho) ** (1.0 / 3.0)


def uniform_positions(rng: np.random.Generator, n: int, L: float) -> np.ndarray:
    """n positions uniform in [0, L)^3: [n, 3] float64."""
    return rng.random((n, 3)) * L


def fcc_lattice(n_cells: int, a: float) -> np.ndarray:
    """Face-centred cubic lattice of n_cells^3 cubic cells (4 atoms each): [4 n^3, 3]."""
    basis = np.array([[0.0, 0.0, 0.0], [0.0, 0.5, 0.5], [0.5, 0.0, 0.5], [0.5, 0.5, 0.0]])
    g = np.arange(n_cells, dtype=np.float64)
    cells = np.stack(np.meshgrid(g, g, g, indexing="ij"), axis=-1).reshape(-1, 3)
    return ((cells[:, None, :] + basis[None, :, :]) * a).reshape(-1, 3)


def simple_cubic(n: int, a: float) -> np.ndarray:
    """Simple cubic lattice n^3 sites with spacing a: [n^3, 3]."""
    g = np.arange(n, dtype=np.float64) * a
    return np.stack(np.meshgrid(g, g, g, indexing="ij"), axis=-1).reshape(-1, 3)


def wrap(r: np.ndarray, L: float) -> np.ndarray:
    """Fold positions into [0, L) per component: r - L floor(r / L)."""
    return r - L * np.floor(r / L)


def brownian_frames(r0: np.ndarray, n_frames: int, step_sigma: float, L: Optional[float],
                    rng: np.random.Generator):
    """Yield n_frames positions: frame 0 = r0, then r += step_sigma * xi (wrapped if L)."""
    r = np.array(r0, dtype=np.float64, copy=True)
    for t in range(n_frames):
        if t > 0:
            r = r + step_sigma * rng.standard_normal(r.shape)
            if L is not None:
                r = wrap(r, L)
        yield r


def planar_grid(n: int, q_lim: float) -> np.ndarray:
    """n x n pixels in the q_z = 0 plane, q_x, q_y = (2a - (n-1))/(n-1) * q_lim.

    Pixel p = b * n + a (q_x fastest).  The grid is exactly antisymmetric, so
    Friedel partners q and -q are both present bit for bit.
    """
    t = (2.0 * np.arange(n) - (n - 1)) / (n - 1) * q_lim
    qx = np.tile(t, n)
    qy = np.repeat(t, n)
    return np.stack([qx, qy, np.zeros_like(qx)], axis=-1)


def planar_subpixels(n: int, q_lim: float, s: int) -> np.ndarray:
    """Sub-pixel wavevectors of the planar grid planar_grid(n, q_lim): s x s points at the
    centres of an even split of each pixel's cell (cell width = the pixel step), laid
    out as [s*s][n*n][3] (sub-sample major, pixels in planar_grid order)."""
    g = planar_grid(n, q_lim)
    step = 2.0 * q_lim / (n - 1)
    offs = (np.arange(s) + 0.5) / s - 0.5
    out = np.empty((s * s, g.shape[0], 3))
    k = 0
    for oy in offs:
        for ox in offs:
            out[k] = g
            out[k, :, 0] += ox * step
            out[k, :, 1] += oy * step
            k += 1
    return out


def ewald_detector(n: int, q_max: float, wavelength: float = WAVELENGTH) -> np.ndarray:
    """n x n pixels on the Ewald sphere, beam k_i = (0, 0, k), k = 2 pi / lambda.

    Transverse components are uniform, q_x, q_y = (2a - (n-1))/(n-1) * Q_perp,
    and q_z = sqrt(k^2 - q_x^2 - q_y^2) - k keeps |k_f| = |k_i|.  Q_perp =
    q_max cos(theta_max / 2) with sin(theta_max / 2) = q_max / (2k), so the
    edge-midpoint pixels sit at |q| = q_max.
    """
    k = 2.0 * math.pi / wavelength
    half = math.asin(q_max / (2.0 * k))
    q_perp = q_max * math.cos(half)
    t = (2.0 * np.arange(n) - (n - 1)) / (n - 1) * q_perp
    qx = np.tile(t, n)
    qy = np.repeat(t, n)
    qz = np.sqrt(k * k - qx * qx - qy * qy) - k
    return np.stack([qx, qy, qz], axis=-1)


def reciprocal_grid(L: float, hmax: int, plane: Optional[int] = None) -> np.ndarray:
    """Wavevectors 2 pi / L * (h, k, l), |h|,|k|,|l| <= hmax (Sec. 3.1, Algorithm 1 step 1).

    plane=2 keeps l = 0 only (a slice), plane=None the full cube.
    """
    g = np.arange(-hmax, hmax + 1, dtype=np.float64)
    if plane is None:
        hkl = np.stack(np.meshgrid(g, g, g, indexing="ij"), axis=-1).reshape(-1, 3)
    else:
        a, b = np.meshgrid(g, g, indexing="ij")
        hkl = np.zeros((a.size, 3))
        axes = [i for i in range(3) if i != plane]
        hkl[:, axes[0]] = a.reshape(-1)
        hkl[:, axes[1]] = b.reshape(-1)
    return hkl * (2.0 * math.pi / L)


def ring_edges(n_rings: int, q_max: float) -> np.ndarray:
    """Uniform ring edges on [0, q_max): n_rings + 1 values."""
    return np.linspace(0.0, q_max, n_rings + 1)


@dataclass
class Workload:
    """One synthetic workload: systems, frames, pixels and reduction settings."""
    name: str
    positions: list                  # per system: array [F, N, 3] (or generator factory)
    f: list                          # per system: [N]
    q: list                          # per system: [Q, 3]
    box: list                        # per system: edge L
    edges: Optional[np.ndarray] = None
    n_tau: int = 0
    n_levels: int = 0
    extra: dict = field(default_factory=dict)


def workload_plain(seed: int = 101, n_atoms: int = 1000, L: float = 36.2, n_det: int = 64,
                   q_lim: float = 4.0) -> Workload:
    """Plain method, one frame: N=1000, f=1, uniform in L=36.2, 64x64 planar q in [-4, 4]."""
    rng = np.random.default_rng(seed)
    r = uniform_positions(rng, n_atoms, L)
    return Workload("plain-1000-64x64", [r[None]], [np.ones(n_atoms)], [planar_grid(n_det, q_lim)],
                    [L])


def workload_trajectory(seed: int = 102, n_cells: int = 20, n_frames: int = 200,
                        n_det: int = 256, q_max: float = 1.5, n_rings: int = 32,
                        n_tau: Optional[int] = None, jitter: float = 0.3,
                        d_dt: float = 0.01) -> Workload:
    """Liquid-like trajectory: fcc n_cells^3 + jitter, Brownian frames, Ewald detector."""
    rng = np.random.default_rng(seed)
    n = 4 * n_cells ** 3
    L = box_for(n)
    a = L / n_cells
    r0 = wrap(fcc_lattice(n_cells, a) + jitter * rng.standard_normal((n, 3)), L)
    frames = np.stack(list(brownian_frames(r0, n_frames, math.sqrt(2.0 * d_dt), L, rng)))
    return Workload("trajectory-%d-%dframes-%dx%d" % (n, n_frames, n_det, n_det), [frames],
                    [np.ones(n)], [ewald_detector(n_det, q_max)], [L],
                    edges=ring_edges(n_rings, q_max),
                    n_tau=n_tau if n_tau is not None else n_frames // 2)


def batch_sizes(seed: int = 103, n_sys: int = 64, n_lo: int = 2000, n_hi: int = 64000):
    """Atom counts drawn log-uniformly in [n_lo, n_hi)."""
    rng = np.random.default_rng(seed)
    return [int(round(math.exp(rng.uniform(math.log(n_lo), math.log(n_hi))))) for _ in range(n_sys)]


def workload_batch(seed: int = 103, n_sys: int = 64, n_lo: int = 2000, n_hi: int = 64000,
                   n_det: int = 512, q_max: float = 1.5, frac_heavy: float = 0.2,
                   f_light: float = 1.0, f_heavy: float = 2.5) -> Workload:
    """Uneven batch: log-uniform N, uniform positions at rho, 80/20 two-species f."""
    sizes = batch_sizes(seed, n_sys, n_lo, n_hi)
    rng = np.random.default_rng(seed + 1000)
    pos, ff, qs, boxes = [], [], [], []
    q = ewald_detector(n_det, q_max)
    for n in sizes:
        L = box_for(n)
        pos.append(uniform_positions(rng, n, L)[None])
        f = np.full(n, f_light)
        f[rng.permutation(n)[: int(round(frac_heavy * n))]] = f_heavy
        ff.append(f)
        qs.append(q)
        boxes.append(L)
    return Workload("batch-%dsys-%dx%d" % (n_sys, n_det, n_det), pos, ff, qs, boxes,
                    extra={"sizes": sizes})


def workload_xsvs(seed: int = 104, n_cells: int = 40, n_frames: int = 1024, n_det: int = 1024,
                  q_max: float = 2.0, n_rings: int = 64, n_levels: int = 9, jitter: float = 0.3,
                  d_dt: float = 0.005, materialize: bool = True) -> Workload:
    """XSVS: fcc n_cells^3 + jitter, Brownian D dt = 0.005, Ewald detector to q_max = 2."""
    rng = np.random.default_rng(seed)
    n = 4 * n_cells ** 3
    L = box_for(n)
    a = L / n_cells
    r0 = wrap(fcc_lattice(n_cells, a) + jitter * rng.standard_normal((n, 3)), L)
    gen = brownian_frames(r0, n_frames, math.sqrt(2.0 * d_dt), L, rng)
    frames = np.stack(list(gen)) if materialize else gen
    return Workload("xsvs-%d-%dframes-%dx%d" % (n, n_frames, n_det, n_det), [frames], [np.ones(n)],
                    [ewald_detector(n_det, q_max)], [L], edges=ring_edges(n_rings, q_max),
                    n_levels=n_levels)


def workload_grad(seed: int = 105, n_atoms: int = 65536, n_det: int = 512, q_lim: float = 3.0,
                  noise: float = 0.2, target_seed: int = 151, fd_seed: int = 152,
                  n_fd: int = 64) -> Workload:
    """Differentiation: uniform r0, planar q in [-3, 3], target from r0 + 0.2 xi (unwrapped)."""
    rng = np.random.default_rng(seed)
    L = box_for(n_atoms)
    r0 = uniform_positions(rng, n_atoms, L)
    r_target = r0 + noise * np.random.default_rng(target_seed).standard_normal(r0.shape)
    fd_atoms = np.sort(np.random.default_rng(fd_seed).choice(n_atoms, size=min(n_fd, n_atoms),
                                                              replace=False))
    return Workload("grad-%d-%dx%d" % (n_atoms, n_det, n_det), [r0[None]], [np.ones(n_atoms)],
                    [planar_grid(n_det, q_lim)], [L],
                    extra={"r_target": r_target, "fd_atoms": fd_atoms})
