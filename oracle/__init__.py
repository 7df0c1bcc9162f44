"""CPU FP64 oracle for the direct speckle-intensity method (arXiv:2204.13241).

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
CPU-baseline leg of the benchmark may import this package.  The product path
(``paper_2204_13241_amd`` and its HIP library) never imports, links or calls
it, and it shares no code with that path: the arithmetic lives in
``xs_oracle.c`` (plain C, FP64), written from the paper.

Functions (each cites the passage it follows in ``xs_oracle.c``):

- ``intensity``          Sec. 3.1 Algorithm 1, Eqs. (pe_ri), (Iq_pq); FP64 form
- ``intensity_libm``     same sum with long-double libm sin/cos (accuracy reference)
- ``intensity_pairsum``  Sec. 2.1 Eq. (Iq_rij), brute-force pair sum
- ``intensity_grad``     chain rule through Eqs. (pe_ri), (Iq_pq); FP64 form
- ``fd_grad``            central differences of sum_p w_p I_p (rank-one updates)
- ``ring_index``         |q| shells of Sec. 2.3 Eq. (bq_Iq)
- ``g2_rings``           Sec. 2.3 Eq. (g2_def), ring mean of Sec. 4.2
- ``xsvs_contrast``      Sec. 2.3 Eqs. (inte_Iq), (bq_Iq), dyadic exposure windows
- ``isf_rings``          Sec. 2.3 Eq. (Fq_pq), ring mean of Sec. 4.2
- ``siegert``            Sec. 2.3 Eqs. (bq_g2), (norm_Fq), (g2_from_fq), (beta_alt_int)
- ``form_factors``       Sec. 2.1: Gaussian-sum atomic form factors f_s(|q|)
- ``intensity_species``  Eqs. (Iq_rij), (pe_ri) with f_j(q) of each atom's species
- ``intensity_species_grad``  chain rule through the same, FP64 form
- ``frame_sums``         incoherent sums of configurations / exposure integrals (Sec. 4.5, Eq. (inte_Iq))
- ``ring_histogram``     distribution of I / <I>_ring per frame and ring (Sec. 4.5, Eq. (Erlang))
- ``speckle_loss``       loss of the differentiation workload, sum (I - I_t)^2 / sum I_t^2, and dL/dI
- ``position_step``      gradient-descent update r <- r - alpha g (one rounding per value)
- ``fd_loss_grad``       central differences of that loss for selected atoms (rank-one updates)
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "xs_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

_CFLAGS = ["-O2", "-fopenmp", "-ffp-contract=off", "-fno-fast-math", "-Wall",
           "-shared", "-fPIC"]


def build(force: bool = True) -> str:
    """Compile liboracle.so with gcc (contraction off, explicit fma only)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        subprocess.run(["gcc", *_CFLAGS, "-o", tmp, _SRC, "-lm"], check=True)
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        build(force=True)
    lib = ctypes.CDLL(_LIB_PATH)
    P = ctypes.c_void_p
    i64, i32, d = ctypes.c_int64, ctypes.c_int32, ctypes.c_double
    c_int = ctypes.c_int
    sig = {
        "or_max_threads": (i32, []),
        "or_constants": (None, [P]),
        "or_sincos_rev_n": (None, [i64, P, P, P]),
        "or_intensity": (c_int, [i64, P, P, i64, P, P, P, c_int]),
        "or_intensity_libm": (c_int, [i64, P, P, i64, P, P, P, c_int]),
        "or_intensity_pairsum": (c_int, [i64, P, P, i64, P, P]),
        "or_intensity_grad": (c_int, [i64, P, P, i64, P, P, P, P, c_int]),
        "or_fd_grad": (c_int, [i64, P, P, i64, P, P, i64, P, d, P, c_int]),
        "or_ring_index": (c_int, [i64, P, i32, P, P]),
        "or_g2_rings": (c_int, [P, i64, i64, P, P, i32, i32, P, P, c_int]),
        "or_xsvs_contrast": (c_int, [P, i64, i64, P, P, i32, i32, P, P, c_int]),
        "or_isf_rings": (c_int, [P, i64, i64, P, P, i32, i32, d, P, P, c_int]),
        "or_siegert": (c_int, [P, P, i32, i32, i32, P, P, P]),
        "or_form_factors": (c_int, [i64, P, i32, P, P]),
        "or_intensity_species": (c_int, [i64, P, P, i32, P, i64, P, P, P, c_int]),
        "or_intensity_species_grad": (c_int, [i64, P, P, i32, P, i64, P, P, P, P, c_int]),
        "or_frame_sums": (c_int, [P, i64, i64, i64, i64, i64, i64, d, P, c_int]),
        "or_ring_histogram": (c_int, [P, i64, i64, P, P, i32, i32, d, P, P]),
        "or_speckle_loss": (c_int, [i64, P, P, P, P]),
        "or_position_step": (c_int, [i64, P, P, d]),
        "or_fd_loss_grad": (c_int, [i64, P, P, i64, P, P, i64, P, d, P, c_int]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _f64(a, shape_last=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if shape_last is not None and (a.ndim == 0 or a.shape[-1] != shape_last):
        raise ValueError("expected trailing dimension %d, got %s" % (shape_last, a.shape))
    return a


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p) if a is not None else None


def _check(rc, what):
    if rc != 0:
        raise RuntimeError("oracle %s failed with status %d" % (what, rc))


def max_threads() -> int:
    return int(_load().or_max_threads())


def constants():
    """(RN(1/2pi), RN(2pi), RN(2pi - RN(2pi))) as used by the FP64 form."""
    out = np.zeros(3)
    _load().or_constants(_ptr(out))
    return tuple(float(x) for x in out)


def sincos_rev(t):
    """FP64-form (sin(2 pi t), cos(2 pi t)) for t in revolutions."""
    t = _f64(np.atleast_1d(t))
    s = np.empty_like(t)
    c = np.empty_like(t)
    _load().or_sincos_rev_n(t.size, _ptr(t), _ptr(s), _ptr(c))
    return s, c


def _intensity(fn, pos, f, q, threads, want_amp=True):
    pos = _f64(pos, 3).reshape(-1, 3)
    f = _f64(f).reshape(-1)
    q = _f64(q, 3).reshape(-1, 3)
    if f.shape[0] != pos.shape[0]:
        raise ValueError("f and pos disagree on the atom count")
    I = np.empty(q.shape[0])
    amp = np.empty((q.shape[0], 2)) if want_amp else None
    _check(fn(pos.shape[0], _ptr(pos), _ptr(f), q.shape[0], _ptr(q), _ptr(I), _ptr(amp),
              int(threads)), fn.__name__)
    return I, amp


def intensity(pos, f, q, threads: int = 0):
    """FP64 form of the direct method: returns (I [Q], amp [Q, 2]) for one frame."""
    return _intensity(_load().or_intensity, pos, f, q, threads)


def intensity_libm(pos, f, q, threads: int = 0):
    """Long-double libm reference of the same sum: (I, amp)."""
    return _intensity(_load().or_intensity_libm, pos, f, q, threads)


def intensity_pairsum(pos, f, q):
    """Brute-force pair double sum, Eq. (Iq_rij): I [Q]."""
    pos = _f64(pos, 3).reshape(-1, 3)
    f = _f64(f).reshape(-1)
    q = _f64(q, 3).reshape(-1, 3)
    I = np.empty(q.shape[0])
    _check(_load().or_intensity_pairsum(pos.shape[0], _ptr(pos), _ptr(f), q.shape[0],
                                        _ptr(q), _ptr(I)), "pairsum")
    return I


def intensity_grad(pos, f, q, amp, dL_dI, threads: int = 0):
    """FP64-form dL/dr [N, 3] from the amplitude of the same positions and dL/dI [Q]."""
    pos = _f64(pos, 3).reshape(-1, 3)
    f = _f64(f).reshape(-1)
    q = _f64(q, 3).reshape(-1, 3)
    amp = _f64(amp, 2).reshape(-1, 2)
    w = _f64(dL_dI).reshape(-1)
    if amp.shape[0] != q.shape[0] or w.shape[0] != q.shape[0]:
        raise ValueError("amp / dL_dI do not match the pixel count")
    out = np.empty_like(pos)
    _check(_load().or_intensity_grad(pos.shape[0], _ptr(pos), _ptr(f), q.shape[0], _ptr(q),
                                     _ptr(amp), _ptr(w), _ptr(out), int(threads)), "grad")
    return out


def fd_grad(pos, f, q, dL_dI, atoms, h: float = 1e-4, threads: int = 0):
    """Central differences of sum_p w_p I_p for the selected atoms: [n_sel, 3]."""
    pos = _f64(pos, 3).reshape(-1, 3)
    f = _f64(f).reshape(-1)
    q = _f64(q, 3).reshape(-1, 3)
    w = _f64(dL_dI).reshape(-1)
    atoms = np.ascontiguousarray(atoms, dtype=np.int64).reshape(-1)
    out = np.empty((atoms.shape[0], 3))
    _check(_load().or_fd_grad(pos.shape[0], _ptr(pos), _ptr(f), q.shape[0], _ptr(q), _ptr(w),
                              atoms.shape[0], _ptr(atoms), float(h), _ptr(out), int(threads)),
           "fd_grad")
    return out


def ring_index(q, edges):
    """Ring of each pixel (-1 outside [e_0, e_R))."""
    q = _f64(q, 3).reshape(-1, 3)
    edges = _f64(edges).reshape(-1)
    ring = np.empty(q.shape[0], dtype=np.int32)
    _check(_load().or_ring_index(q.shape[0], _ptr(q), edges.shape[0] - 1, _ptr(edges),
                                 _ptr(ring)), "ring_index")
    return ring


def g2_rings(I, q, edges, n_tau: int, threads: int = 0):
    """g2 [n_rings, n_tau] and pixel counts [n_rings] from I [F, Q]."""
    I = _f64(I)
    if I.ndim != 2:
        raise ValueError("I must be [frames, pixels]")
    q = _f64(q, 3).reshape(-1, 3)
    edges = _f64(edges).reshape(-1)
    nr = edges.shape[0] - 1
    g2 = np.empty((nr, n_tau))
    cnt = np.empty(nr, dtype=np.int32)
    _check(_load().or_g2_rings(_ptr(I), I.shape[0], I.shape[1], _ptr(q), _ptr(edges), nr,
                               int(n_tau), _ptr(g2), _ptr(cnt), int(threads)), "g2_rings")
    return g2, cnt


def xsvs_contrast(I, q, edges, n_levels: int, threads: int = 0, want_windows: bool = False):
    """beta [n_levels, n_rings] (and per-window [n_levels, F, n_rings] if asked)."""
    I = _f64(I)
    if I.ndim != 2:
        raise ValueError("I must be [frames, pixels]")
    q = _f64(q, 3).reshape(-1, 3)
    edges = _f64(edges).reshape(-1)
    nr = edges.shape[0] - 1
    beta = np.empty((n_levels, nr))
    win = np.empty((n_levels, I.shape[0], nr)) if want_windows else None
    _check(_load().or_xsvs_contrast(_ptr(I), I.shape[0], I.shape[1], _ptr(q), _ptr(edges), nr,
                                    int(n_levels), _ptr(beta), _ptr(win), int(threads)),
           "xsvs_contrast")
    return (beta, win) if want_windows else beta


def isf_rings(amp, q, edges, n_tau: int, f2_sum: float, threads: int = 0):
    """F(q, tau) per ring [n_rings, n_tau, 2] (re, im) and pixel counts [n_rings]
    from amplitudes amp [F, Q, 2]."""
    amp = _f64(amp, 2)
    if amp.ndim != 3:
        raise ValueError("amp must be [frames, pixels, 2]")
    q = _f64(q, 3).reshape(-1, 3)
    edges = _f64(edges).reshape(-1)
    nr = edges.shape[0] - 1
    F = np.empty((nr, n_tau, 2))
    cnt = np.empty(nr, dtype=np.int32)
    _check(_load().or_isf_rings(_ptr(amp), amp.shape[0], amp.shape[1], _ptr(q), _ptr(edges), nr,
                                int(n_tau), float(f2_sum), _ptr(F), _ptr(cnt), int(threads)),
           "isf_rings")
    return F, cnt


def siegert(g2, F, n_levels: int):
    """(lhs, fhat2, beta_pred): (g2 - 1) / beta0 and |F-hat|^2 [n_rings, n_tau], and the
    contrast predicted from F-hat for W = 1, 2, ..., 2^(n_levels-1) [n_levels, n_rings]."""
    g2 = _f64(g2)
    F = _f64(F, 2)
    nr, nt = g2.shape
    if F.shape != (nr, nt, 2):
        raise ValueError("F must be [n_rings, n_tau, 2] matching g2")
    lhs = np.empty((nr, nt))
    fh = np.empty((nr, nt))
    beta = np.empty((n_levels, nr))
    _check(_load().or_siegert(_ptr(g2), _ptr(F), nr, nt, int(n_levels), _ptr(lhs), _ptr(fh),
                              _ptr(beta)), "siegert")
    return lhs, fh, beta


def _coef(coef):
    c = _f64(coef, 9).reshape(-1, 9)
    return c, c.shape[0]


def form_factors(q, coef):
    """f_s(|q|) [Q, n_species] from Gaussian-sum coefficients coef [n_species, 9]
    (a_1..a_4, b_1..b_4, c; s = |q| / (4 pi))."""
    q = _f64(q, 3).reshape(-1, 3)
    c, ns = _coef(coef)
    out = np.empty((q.shape[0], ns))
    _check(_load().or_form_factors(q.shape[0], _ptr(q), ns, _ptr(c), _ptr(out)), "form_factors")
    return out


def intensity_species(pos, species, coef, q, threads: int = 0):
    """FP64 form with q-dependent form factors: (I [Q], amp [Q, 2]) for one frame."""
    pos = _f64(pos, 3).reshape(-1, 3)
    sp = np.ascontiguousarray(species, dtype=np.int32).reshape(-1)
    if sp.shape[0] != pos.shape[0]:
        raise ValueError("species and pos disagree on the atom count")
    q = _f64(q, 3).reshape(-1, 3)
    c, ns = _coef(coef)
    I = np.empty(q.shape[0])
    amp = np.empty((q.shape[0], 2))
    _check(_load().or_intensity_species(pos.shape[0], _ptr(pos), _ptr(sp), ns, _ptr(c), q.shape[0], _ptr(q),
                                        _ptr(I), _ptr(amp), int(threads)), "intensity_species")
    return I, amp


def intensity_species_grad(pos, species, coef, q, amp, dL_dI, threads: int = 0):
    """FP64-form dL/dr [N, 3] with q-dependent form factors."""
    pos = _f64(pos, 3).reshape(-1, 3)
    sp = np.ascontiguousarray(species, dtype=np.int32).reshape(-1)
    q = _f64(q, 3).reshape(-1, 3)
    c, ns = _coef(coef)
    amp = _f64(amp, 2).reshape(-1, 2)
    w = _f64(dL_dI).reshape(-1)
    g = np.empty((pos.shape[0], 3))
    _check(_load().or_intensity_species_grad(pos.shape[0], _ptr(pos), _ptr(sp), ns, _ptr(c), q.shape[0],
                                             _ptr(q), _ptr(amp), _ptr(w), _ptr(g), int(threads)),
           "intensity_species_grad")
    return g


def frame_sums(I, n_out: int, s_out: int, n_sum: int, s_sum: int, scale: float = 1.0, threads: int = 0):
    """J [n_out, Q]: J[k] = scale * pairwise sum over i < n_sum of I[k s_out + i s_sum] (I [F, Q])."""
    I = _f64(I)
    if I.ndim != 2:
        raise ValueError("I must be [frames, pixels]")
    J = np.empty((n_out, I.shape[1]))
    _check(_load().or_frame_sums(_ptr(I), I.shape[0], I.shape[1], int(n_out), int(s_out), int(n_sum),
                                 int(s_sum), float(scale), _ptr(J), int(threads)), "frame_sums")
    return J


def ring_histogram(I, q, edges, n_bins: int, kappa_max: float):
    """(counts [F, R, n_bins + 1] int64, ring means [F, R]) of kappa = I / <I>_ring."""
    I = _f64(I)
    if I.ndim != 2:
        raise ValueError("I must be [frames, pixels]")
    q = _f64(q, 3).reshape(-1, 3)
    edges = _f64(edges).reshape(-1)
    nr = edges.shape[0] - 1
    counts = np.empty((I.shape[0], nr, n_bins + 1), dtype=np.int64)
    mean = np.empty((I.shape[0], nr))
    _check(_load().or_ring_histogram(_ptr(I), I.shape[0], I.shape[1], _ptr(q), _ptr(edges), nr, int(n_bins),
                                     float(kappa_max), _ptr(counts), _ptr(mean)), "ring_histogram")
    return counts, mean


def speckle_loss(I, It):
    """(L, S, dL/dI [n]) of L = sum (I - It)^2 / S, S = sum It^2 (compensated long-double sums)."""
    I = _f64(I).reshape(-1)
    It = _f64(It).reshape(-1)
    if I.shape != It.shape:
        raise ValueError("I and I_target differ in size")
    out = np.empty(2)
    w = np.empty_like(I)
    _check(_load().or_speckle_loss(I.shape[0], _ptr(I), _ptr(It), _ptr(out), _ptr(w)), "speckle_loss")
    return float(out[0]), float(out[1]), w


def position_step(pos, g, alpha: float):
    """pos - alpha g with one rounding per value (fma), as a new array."""
    pos = np.array(_f64(pos), copy=True)
    g = _f64(g)
    if g.size != pos.size:
        raise ValueError("pos and g differ in size")
    _check(_load().or_position_step(pos.size, _ptr(pos), _ptr(g), float(alpha)), "position_step")
    return pos


def fd_loss_grad(pos, f, q, It, atoms, h: float = 1e-4, threads: int = 0):
    """Central differences of L = sum (I - It)^2 / sum It^2 for the selected atoms: [n_sel, 3]."""
    pos = _f64(pos, 3).reshape(-1, 3)
    f = _f64(f).reshape(-1)
    q = _f64(q, 3).reshape(-1, 3)
    It = _f64(It).reshape(-1)
    if It.shape[0] != q.shape[0]:
        raise ValueError("I_target does not match the pixel count")
    atoms = np.ascontiguousarray(atoms, dtype=np.int64).reshape(-1)
    out = np.empty((atoms.shape[0], 3))
    _check(_load().or_fd_loss_grad(pos.shape[0], _ptr(pos), _ptr(f), q.shape[0], _ptr(q), _ptr(It),
                                   atoms.shape[0], _ptr(atoms), float(h), _ptr(out), int(threads)),
           "fd_loss_grad")
    return out
