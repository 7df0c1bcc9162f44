"""Python API over the HIP library: torch tensors in device memory in, results out.

PyTorch supplies device memory and the current stream; every computation runs
in libxs.so (see include/xs.h).  Tensors must be CUDA (HIP) tensors of the
documented dtype; nothing is moved to or computed on the CPU here.
"""
from __future__ import annotations

import ctypes
import math
from dataclasses import dataclass
from typing import List, Optional, Sequence

import numpy as np
import torch

from . import _lib

PRECISIONS = {"fp64": _lib.XS_FP64, "fp32c": _lib.XS_FP32C}


def _prec(precision) -> int:
    if isinstance(precision, int):
        return precision
    try:
        return PRECISIONS[precision]
    except KeyError:
        raise ValueError("precision must be 'fp64' or 'fp32c', got %r" % (precision,))


def _ptr(t: Optional[torch.Tensor]):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _need(t: torch.Tensor, name: str, dtype=torch.float64):
    if not isinstance(t, torch.Tensor):
        raise TypeError("%s must be a torch.Tensor" % name)
    if not t.is_cuda:
        raise ValueError("%s must live in GPU memory (got device %s)" % (name, t.device))
    if t.dtype != dtype:
        raise ValueError("%s must be %s (got %s)" % (name, dtype, t.dtype))
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)
    return t


@dataclass
class Batch:
    """Host-side batch descriptor (xs_batch) with the arrays it points to."""
    n_atoms: np.ndarray
    n_q: np.ndarray
    n_frames: np.ndarray
    pos_off: np.ndarray
    f_off: np.ndarray
    q_off: np.ndarray
    out_off: np.ndarray
    box: np.ndarray

    def struct(self) -> _lib.XsBatch:
        def p64(a):
            return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))
        b = _lib.XsBatch()
        b.n_sys = int(self.n_atoms.shape[0])
        b.n_atoms = p64(self.n_atoms)
        b.n_q = p64(self.n_q)
        b.n_frames = self.n_frames.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
        b.pos_off = p64(self.pos_off)
        b.f_off = p64(self.f_off)
        b.q_off = p64(self.q_off)
        b.out_off = p64(self.out_off)
        b.box = self.box.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        return b

    @property
    def total_out(self) -> int:
        return int(np.sum(self.n_q * self.n_frames))


def make_batch(n_atoms: Sequence[int], n_q: Sequence[int], n_frames: Sequence[int],
               box: Sequence) -> Batch:
    """Packed layout: systems back to back in pos, f, q and outputs."""
    na = np.ascontiguousarray(n_atoms, dtype=np.int64)
    nq = np.ascontiguousarray(n_q, dtype=np.int64)
    nf = np.ascontiguousarray(n_frames, dtype=np.int32)
    bx = np.asarray(box, dtype=np.float64)
    if bx.size == 1:
        bx = np.full((len(na), 3), float(bx.reshape(-1)[0]))
    bx = np.ascontiguousarray(bx.reshape(len(na), 3))
    pos_off = np.concatenate([[0], np.cumsum(na * nf)[:-1]]).astype(np.int64)
    f_off = np.concatenate([[0], np.cumsum(na)[:-1]]).astype(np.int64)
    q_off = np.concatenate([[0], np.cumsum(nq)[:-1]]).astype(np.int64)
    out_off = np.concatenate([[0], np.cumsum(nq * nf)[:-1]]).astype(np.int64)
    return Batch(na, nq, nf, pos_off, f_off, q_off, out_off, bx.reshape(-1))


def _box3(box, pos: torch.Tensor) -> np.ndarray:
    if box is None:
        raise ValueError("box (edge or 3 edges, Angstrom) is required")
    b = np.asarray(box, dtype=np.float64).reshape(-1)
    return np.full(3, b[0]) if b.size == 1 else b


def intensity(pos: torch.Tensor, f: torch.Tensor, q: torch.Tensor, precision="fp32c",
              box=None, return_amp: bool = False):
    """Direct-method intensity of every frame and pixel.

    pos [F, N, 3] or [N, 3] float64, f [N] float64, q [Q, 3] float64, all on the
    GPU; box: cube edge or 3 edges (Angstrom; required for 'fp32c').
    Returns I [F, Q] (or [Q]) float64, and the amplitude [F, Q, 2] if asked.
    """
    _need(pos, "pos"), _need(f, "f"), _need(q, "q")
    single = pos.dim() == 2
    p3 = pos.unsqueeze(0) if single else pos
    if p3.dim() != 3 or p3.shape[-1] != 3:
        raise ValueError("pos must be [F, N, 3] or [N, 3]")
    F, N = int(p3.shape[0]), int(p3.shape[1])
    if f.shape != (N,):
        raise ValueError("f must be [N]")
    if q.dim() != 2 or q.shape[1] != 3:
        raise ValueError("q must be [Q, 3]")
    Q = int(q.shape[0])
    bx = _box3(box, pos) if _prec(precision) == _lib.XS_FP32C else np.ones(3)
    b = make_batch([N], [Q], [F], bx)
    I = torch.empty((F, Q), dtype=torch.float64, device=pos.device)
    amp = torch.empty((F, Q, 2), dtype=torch.float64, device=pos.device) if return_amp else None
    lib = _lib.load()
    st = b.struct()
    _lib.check(lib.xs_intensity_direct(ctypes.byref(st), _ptr(p3), _ptr(f), _ptr(q), _prec(precision),
                                       _ptr(I), _ptr(amp), _stream()))
    if single:
        I = I[0]
        amp = amp[0] if amp is not None else None
    return (I, amp) if return_amp else I


def intensity_systems(systems: List[tuple], precision="fp32c", return_amp: bool = False):
    """Many independent systems in one call (one persistent launch per phase).

    systems: list of (pos [F_s, N_s, 3], f [N_s], q [Q_s, 3], box) on the GPU.
    Returns a list of I [F_s, Q_s] (and amplitudes).
    """
    if not systems:
        return []
    dev = systems[0][0].device
    for i, (p, f, q, _) in enumerate(systems):
        _need(p, "pos[%d]" % i), _need(f, "f[%d]" % i), _need(q, "q[%d]" % i)
        if p.dim() != 3 or p.shape[-1] != 3 or f.shape != (p.shape[1],) or q.dim() != 2 or q.shape[1] != 3:
            raise ValueError("system %d has inconsistent shapes" % i)
    n_atoms = [int(p.shape[1]) for p, _, _, _ in systems]
    n_frames = [int(p.shape[0]) for p, _, _, _ in systems]
    n_q = [int(q.shape[0]) for _, _, q, _ in systems]
    boxes = np.stack([_box3(bx, None) for _, _, _, bx in systems])
    b = make_batch(n_atoms, n_q, n_frames, boxes)
    pos = torch.cat([p.reshape(-1, 3) for p, _, _, _ in systems]).contiguous()
    ff = torch.cat([f for _, f, _, _ in systems]).contiguous()
    qq = torch.cat([q for _, _, q, _ in systems]).contiguous()
    I = torch.empty(b.total_out, dtype=torch.float64, device=dev)
    amp = torch.empty((b.total_out, 2), dtype=torch.float64, device=dev) if return_amp else None
    st = b.struct()
    _lib.check(_lib.load().xs_intensity_direct(ctypes.byref(st), _ptr(pos), _ptr(ff), _ptr(qq),
                                               _prec(precision), _ptr(I), _ptr(amp), _stream()))
    outs, amps = [], []
    for s in range(len(systems)):
        o = int(b.out_off[s])
        n = n_q[s] * n_frames[s]
        outs.append(I[o:o + n].view(n_frames[s], n_q[s]))
        if return_amp:
            amps.append(amp[o:o + n].view(n_frames[s], n_q[s], 2))
    return (outs, amps) if return_amp else outs


def intensity_grad(pos: torch.Tensor, f: torch.Tensor, q: torch.Tensor, amp: torch.Tensor,
                   dL_dI: torch.Tensor, precision="fp32c", box=None, out_dtype=torch.float32):
    """dL/dpos from the amplitude of the same positions and dL/dI (same shape as I)."""
    _need(pos, "pos"), _need(f, "f"), _need(q, "q"), _need(amp, "amp"), _need(dL_dI, "dL_dI")
    single = pos.dim() == 2
    p3 = pos.unsqueeze(0) if single else pos
    F, N = int(p3.shape[0]), int(p3.shape[1])
    Q = int(q.shape[0])
    if amp.numel() != F * Q * 2 or dL_dI.numel() != F * Q:
        raise ValueError("amp must be [F, Q, 2] and dL_dI [F, Q]")
    bx = _box3(box, pos) if _prec(precision) == _lib.XS_FP32C else np.ones(3)
    b = make_batch([N], [Q], [F], bx)
    g32 = torch.empty(p3.shape, dtype=torch.float32, device=pos.device) if out_dtype == torch.float32 else None
    g64 = torch.empty(p3.shape, dtype=torch.float64, device=pos.device) if out_dtype == torch.float64 else None
    if g32 is None and g64 is None:
        raise ValueError("out_dtype must be torch.float32 or torch.float64")
    st = b.struct()
    _lib.check(_lib.load().xs_intensity_grad(ctypes.byref(st), _ptr(p3), _ptr(f), _ptr(q), _ptr(amp),
                                             _ptr(dL_dI), _prec(precision), _ptr(g32), _ptr(g64),
                                             _stream()))
    g = g32 if g32 is not None else g64
    return g[0] if single else g


def _species_args(species: torch.Tensor, coef, N: int):
    if not isinstance(species, torch.Tensor) or not species.is_cuda or species.dtype != torch.int32:
        raise ValueError("species must be an int32 tensor in GPU memory")
    if species.shape != (N,) or not species.is_contiguous():
        raise ValueError("species must be a contiguous [N] tensor")
    c = np.ascontiguousarray(coef, dtype=np.float64).reshape(-1, 9)
    return c


def intensity_species(pos: torch.Tensor, species: torch.Tensor, coef, q: torch.Tensor, precision="fp32c",
                      box=None, return_amp: bool = False):
    """Intensity with q-dependent form factors f_s(|q|) = c + sum_i a_i exp(-b_i (|q|/4pi)^2).

    pos [F, N, 3] or [N, 3] float64, species [N] int32 (GPU), coef [n_species, 9]
    (a_1..a_4, b_1..b_4, c; host), q [Q, 3] float64.  Returns I [F, Q] (or [Q]) and
    the amplitude [F, Q, 2] if asked."""
    _need(pos, "pos"), _need(q, "q")
    single = pos.dim() == 2
    p3 = pos.unsqueeze(0) if single else pos
    F, N, Q = int(p3.shape[0]), int(p3.shape[1]), int(q.shape[0])
    c = _species_args(species, coef, N)
    bx = _box3(box, pos) if _prec(precision) == _lib.XS_FP32C else np.ones(3)
    b = make_batch([N], [Q], [F], bx)
    I = torch.empty((F, Q), dtype=torch.float64, device=pos.device)
    amp = torch.empty((F, Q, 2), dtype=torch.float64, device=pos.device) if return_amp else None
    st = b.struct()
    _lib.check(_lib.load().xs_intensity_species(ctypes.byref(st), _ptr(p3), _ptr(species), c.shape[0],
                                                c.ctypes.data_as(ctypes.c_void_p), _ptr(q), _prec(precision),
                                                _ptr(I), _ptr(amp), _stream()))
    if single:
        I = I[0]
        amp = amp[0] if amp is not None else None
    return (I, amp) if return_amp else I


def intensity_species_grad(pos: torch.Tensor, species: torch.Tensor, coef, q: torch.Tensor, amp: torch.Tensor,
                           dL_dI: torch.Tensor, precision="fp32c", box=None, out_dtype=torch.float32):
    """dL/dpos with q-dependent form factors, from the amplitude of intensity_species."""
    _need(pos, "pos"), _need(q, "q"), _need(amp, "amp"), _need(dL_dI, "dL_dI")
    single = pos.dim() == 2
    p3 = pos.unsqueeze(0) if single else pos
    F, N, Q = int(p3.shape[0]), int(p3.shape[1]), int(q.shape[0])
    c = _species_args(species, coef, N)
    if amp.numel() != F * Q * 2 or dL_dI.numel() != F * Q:
        raise ValueError("amp must be [F, Q, 2] and dL_dI [F, Q]")
    bx = _box3(box, pos) if _prec(precision) == _lib.XS_FP32C else np.ones(3)
    b = make_batch([N], [Q], [F], bx)
    g32 = torch.empty(p3.shape, dtype=torch.float32, device=pos.device) if out_dtype == torch.float32 else None
    g64 = torch.empty(p3.shape, dtype=torch.float64, device=pos.device) if out_dtype == torch.float64 else None
    if g32 is None and g64 is None:
        raise ValueError("out_dtype must be torch.float32 or torch.float64")
    st = b.struct()
    _lib.check(_lib.load().xs_intensity_species_grad(ctypes.byref(st), _ptr(p3), _ptr(species), c.shape[0],
                                                     c.ctypes.data_as(ctypes.c_void_p), _ptr(q), _ptr(amp),
                                                     _ptr(dL_dI), _prec(precision), _ptr(g32), _ptr(g64),
                                                     _stream()))
    g = g32 if g32 is not None else g64
    return g[0] if single else g


def g2_rings(I: torch.Tensor, q: torch.Tensor, edges, n_tau: int):
    """g2 [n_rings, n_tau] (float64) and the pixel count per ring (int32)."""
    _need(I, "I"), _need(q, "q")
    if I.dim() != 2 or q.shape != (I.shape[1], 3):
        raise ValueError("I must be [F, Q] and q [Q, 3]")
    e = np.ascontiguousarray(edges, dtype=np.float64)
    R = e.shape[0] - 1
    g2 = torch.empty((R, n_tau), dtype=torch.float64, device=I.device)
    cnt = torch.empty(R, dtype=torch.int32, device=I.device)
    _lib.check(_lib.load().xs_g2_rings(_ptr(I), I.shape[0], I.shape[1], _ptr(q),
                                       e.ctypes.data_as(ctypes.c_void_p), R, int(n_tau), _ptr(g2),
                                       _ptr(cnt), _stream()))
    return g2, cnt


def xsvs_contrast(I: torch.Tensor, q: torch.Tensor, edges, n_levels: int,
                  return_windows: bool = False):
    """beta [n_levels, n_rings] (and per-window values [n_levels, F, n_rings])."""
    _need(I, "I"), _need(q, "q")
    if I.dim() != 2 or q.shape != (I.shape[1], 3):
        raise ValueError("I must be [F, Q] and q [Q, 3]")
    e = np.ascontiguousarray(edges, dtype=np.float64)
    R = e.shape[0] - 1
    beta = torch.empty((n_levels, R), dtype=torch.float64, device=I.device)
    win = torch.empty((n_levels, I.shape[0], R), dtype=torch.float64, device=I.device) if return_windows else None
    _lib.check(_lib.load().xs_xsvs_contrast(_ptr(I), I.shape[0], I.shape[1], _ptr(q),
                                            e.ctypes.data_as(ctypes.c_void_p), R, int(n_levels),
                                            _ptr(beta), _ptr(win), _stream()))
    return (beta, win) if return_windows else beta


def isf_rings(amp: torch.Tensor, q: torch.Tensor, edges, n_tau: int, f2_sum: float):
    """F(q, tau) per ring [n_rings, n_tau, 2] (float64: re, im) from amplitudes
    amp [F, Q, 2], and the pixel count per ring (int32)."""
    _need(amp, "amp"), _need(q, "q")
    if amp.dim() != 3 or amp.shape[2] != 2 or q.shape != (amp.shape[1], 3):
        raise ValueError("amp must be [F, Q, 2] and q [Q, 3]")
    e = np.ascontiguousarray(edges, dtype=np.float64)
    R = e.shape[0] - 1
    F = torch.empty((R, n_tau, 2), dtype=torch.float64, device=amp.device)
    cnt = torch.empty(R, dtype=torch.int32, device=amp.device)
    _lib.check(_lib.load().xs_isf_rings(_ptr(amp), amp.shape[0], amp.shape[1], _ptr(q),
                                        e.ctypes.data_as(ctypes.c_void_p), R, int(n_tau), float(f2_sum),
                                        _ptr(F), _ptr(cnt), _stream()))
    return F, cnt


def siegert(g2: torch.Tensor, F: torch.Tensor, n_levels: int):
    """(lhs, fhat2, beta): (g2 - 1) / beta0 and |F-hat|^2 [n_rings, n_tau], and the
    contrast predicted from F-hat for W = 1, 2, ..., 2^(n_levels-1) [n_levels, n_rings]."""
    _need(g2, "g2"), _need(F, "F")
    if g2.dim() != 2 or F.shape != (g2.shape[0], g2.shape[1], 2):
        raise ValueError("g2 must be [R, n_tau] and F [R, n_tau, 2]")
    R, nt = g2.shape
    lhs = torch.empty((R, nt), dtype=torch.float64, device=g2.device)
    fh = torch.empty((R, nt), dtype=torch.float64, device=g2.device)
    beta = torch.empty((n_levels, R), dtype=torch.float64, device=g2.device)
    _lib.check(_lib.load().xs_siegert(_ptr(g2), _ptr(F), R, nt, int(n_levels), _ptr(lhs), _ptr(fh),
                                      _ptr(beta) if n_levels > 0 else None, _stream()))
    return lhs, fh, beta


def frame_sums(I: torch.Tensor, n_out: int, s_out: int, n_sum: int, s_sum: int, scale: float = 1.0):
    """J [n_out, Q]: J[k] = scale * pairwise sum over i < n_sum of I[k s_out + i s_sum] (I [F, Q])."""
    _need(I, "I")
    if I.dim() != 2:
        raise ValueError("I must be [F, Q]")
    J = torch.empty((int(n_out), I.shape[1]), dtype=torch.float64, device=I.device)
    _lib.check(_lib.load().xs_frame_sums(_ptr(I), I.shape[0], I.shape[1], int(n_out), int(s_out), int(n_sum),
                                         int(s_sum), float(scale), _ptr(J), _stream()))
    return J


def intensity_pixel_mean(pos: torch.Tensor, f: torch.Tensor, q_sub: torch.Tensor, precision="fp32c", box=None):
    """Detector-pixel intensity as the mean over S sub-pixel wavevectors (the pixel
    integral of Sec. 3.1).  q_sub [S, Q, 3]: S sub-samples of each of Q pixels.
    Returns [F, Q] (or [Q] for pos [N, 3])."""
    _need(q_sub, "q_sub")
    if q_sub.dim() != 3 or q_sub.shape[2] != 3:
        raise ValueError("q_sub must be [S, Q, 3]")
    S, Q = int(q_sub.shape[0]), int(q_sub.shape[1])
    single = pos.dim() == 2
    I = intensity(pos, f, q_sub.reshape(S * Q, 3), precision=precision, box=box)
    I2 = I.reshape(-1, Q)                   # frames x S rows of Q pixels
    F = I2.shape[0] // S
    J = frame_sums(I2, F, S, S, 1, 1.0 / S)
    return J[0] if single else J


def ring_histogram(I: torch.Tensor, q: torch.Tensor, edges, n_bins: int, kappa_max: float):
    """(counts [F, R, n_bins + 1] int64, ring means [F, R]) of kappa = I / <I>_ring."""
    _need(I, "I"), _need(q, "q")
    if I.dim() != 2 or q.shape != (I.shape[1], 3):
        raise ValueError("I must be [F, Q] and q [Q, 3]")
    e = np.ascontiguousarray(edges, dtype=np.float64)
    R = e.shape[0] - 1
    counts = torch.empty((I.shape[0], R, int(n_bins) + 1), dtype=torch.int64, device=I.device)
    mean = torch.empty((I.shape[0], R), dtype=torch.float64, device=I.device)
    _lib.check(_lib.load().xs_ring_histogram(_ptr(I), I.shape[0], I.shape[1], _ptr(q),
                                             e.ctypes.data_as(ctypes.c_void_p), R, int(n_bins), float(kappa_max),
                                             _ptr(counts), _ptr(mean), _stream()))
    return counts, mean


def fft_intensity(pos: torch.Tensor, f: torch.Tensor, box: float, n_grid: int, eta: float, k: int = None,
                  return_amp: bool = False):
    """FFT-based method (Algorithm 2) for one frame: I [n, n, n] on q_h = 2 pi h / box (FFT
    order), and the amplitude [n, n, n, 2] if asked.  k defaults to the nearest integer
    above 10 eta n / box."""
    _need(pos, "pos"), _need(f, "f")
    if pos.dim() != 2 or pos.shape[1] != 3 or f.shape != (pos.shape[0],):
        raise ValueError("pos must be [N, 3] and f [N]")
    n = int(n_grid)
    if k is None:
        k = int(math.floor(10.0 * eta * n / box)) + 1
    I = torch.empty((n, n, n), dtype=torch.float64, device=pos.device)
    amp = torch.empty((n, n, n, 2), dtype=torch.float64, device=pos.device) if return_amp else None
    _lib.check(_lib.load().xs_fft_intensity(_ptr(pos), _ptr(f), pos.shape[0], float(box), n, float(eta), int(k),
                                            _ptr(I), _ptr(amp), _stream()))
    return (I, amp) if return_amp else I


def get_tile_shape(kind: int) -> dict:
    s = _lib.XsTileShape()
    _lib.check(_lib.load().xs_get_tile_shape(int(kind), ctypes.byref(s)))
    return {"atoms_per_tile": s.atoms_per_tile, "q_per_lane": s.q_per_lane,
            "atom_split": s.atom_split, "pixel_split": s.pixel_split,
            "waves_per_simd": s.waves_per_simd, "lattice": s.lattice}


def set_tile_shape(kind: int, atoms_per_tile=64, q_per_lane=4, atom_split=64, pixel_split=8192,
                   waves_per_simd=0, lattice=None):
    """Set the forward (kind 0) or gradient (kind 1) tile shape (xs_set_tile_shape).
    lattice None means 1 for q_per_lane 32 (the matrix-core lattice form, which needs
    it) and 0 otherwise (the per-pair form everywhere)."""
    if lattice is None:
        lattice = 1 if int(q_per_lane) == 32 else 0
    s = _lib.XsTileShape(int(atoms_per_tile), int(q_per_lane), int(atom_split), int(pixel_split),
                         int(waves_per_simd), int(lattice))
    _lib.check(_lib.load().xs_set_tile_shape(int(kind), ctypes.byref(s)))


class IntensityFn(torch.autograd.Function):
    """I = |sum_j f_j exp(-i q.r_j)|^2 with a hand-written adjoint for dL/dpos.

    forward(pos [F,N,3] or [N,3] float64, f, q, box, precision) -> I;
    backward calls xs_intensity_grad with the saved amplitude.
    """

    @staticmethod
    def forward(ctx, pos, f, q, box, precision="fp32c"):
        I, amp = intensity(pos.detach(), f.detach(), q.detach(), precision, box, return_amp=True)
        ctx.save_for_backward(pos.detach(), f.detach(), q.detach(), amp)
        ctx.box = box
        ctx.precision = precision
        return I

    @staticmethod
    def backward(ctx, grad_I):
        pos, f, q, amp = ctx.saved_tensors
        g = intensity_grad(pos, f, q, amp, grad_I.contiguous().to(torch.float64), ctx.precision,
                           ctx.box, out_dtype=torch.float64)
        return g, None, None, None, None


class IntensitySpeciesFn(torch.autograd.Function):
    """I with q-dependent form factors f_s(|q|) per species, differentiable in pos.

    forward(pos [F,N,3] or [N,3] float64, species [N] int32, coef [n_species, 9] (host),
    q, box, precision) -> I; backward calls xs_intensity_species_grad with the saved
    amplitude.
    """

    @staticmethod
    def forward(ctx, pos, species, coef, q, box, precision="fp32c"):
        I, amp = intensity_species(pos.detach(), species, coef, q.detach(), precision, box, return_amp=True)
        ctx.save_for_backward(pos.detach(), species, q.detach(), amp)
        ctx.coef = coef
        ctx.box = box
        ctx.precision = precision
        return I

    @staticmethod
    def backward(ctx, grad_I):
        pos, species, q, amp = ctx.saved_tensors
        g = intensity_species_grad(pos, species, ctx.coef, q, amp, grad_I.contiguous().to(torch.float64),
                                   ctx.precision, ctx.box, out_dtype=torch.float64)
        return g, None, None, None, None, None


def shutdown():
    _lib.check(_lib.load().xs_shutdown())


def speckle_loss(I: torch.Tensor, I_target: torch.Tensor, want_grad: bool = True):
    """L = sum (I - I_t)^2 / sum I_t^2 and dL/dI (device); returns (loss_buf[2], dL_dI)."""
    _need(I, "I"), _need(I_target, "I_target")
    if I.numel() != I_target.numel():
        raise ValueError("I and I_target differ in size")
    out = torch.empty(2, dtype=torch.float64, device=I.device)
    w = torch.empty_like(I) if want_grad else None
    _lib.check(_lib.load().xs_speckle_loss(_ptr(I), _ptr(I_target), I.numel(), _ptr(out), _ptr(w),
                                           _stream()))
    return out, w


def position_step(pos: torch.Tensor, grad: torch.Tensor, step: float):
    """pos -= step * grad, in place (grad float32 or float64, same shape)."""
    _need(pos, "pos")
    if grad.shape != pos.shape or not grad.is_cuda or not grad.is_contiguous():
        raise ValueError("grad must be a contiguous GPU tensor shaped like pos")
    g32 = grad if grad.dtype == torch.float32 else None
    g64 = grad if grad.dtype == torch.float64 else None
    if g32 is None and g64 is None:
        raise ValueError("grad must be float32 or float64")
    _lib.check(_lib.load().xs_position_step(_ptr(pos), _ptr(g32), _ptr(g64), pos.numel(),
                                            float(step), _stream()))


TIMER_KINDS = {"fwd32": 0, "grad32": 1, "fwd64": 2, "grad64": 3, "bin": 4, "g2": 5, "xsvs": 6, "isf": 7}


def timing_enable(on: bool = True):
    _lib.check(_lib.load().xs_timing_enable(1 if on else 0))


def timing_read(kind) -> dict:
    k = TIMER_KINDS[kind] if isinstance(kind, str) else int(kind)
    ms = ctypes.c_double(0.0)
    n = ctypes.c_int64(0)
    work = ctypes.c_double(0.0)
    _lib.check(_lib.load().xs_timing_read(k, ctypes.byref(ms), ctypes.byref(n), ctypes.byref(work)))
    return {"ms": ms.value, "launches": n.value, "work": work.value}


def roofline_probe(kind: int, nbytes: int = 1 << 30) -> float:
    """0: sin+cos lane-ops/s, 1: FP32 FMA lane-ops/s, 2: FP64 FMA lane-ops/s, 3: copy bytes/s
    (read + write), 4: FP16 matrix flops/s, 5: the same beside FP32 FMAs, 6: read bytes/s."""
    r = ctypes.c_double(0.0)
    _lib.check(_lib.load().xs_roofline_probe(int(kind), int(nbytes), ctypes.byref(r), _stream()))
    return r.value


class Plan:
    """FP32C batch plan over the C ABI (xs_plan_*): fixed batch layout and pixels.

    systems: list of (n_atoms, n_frames, q [Q_s, 3] float64 GPU tensor, box).
    Positions, form factors and outputs use the packed layout of make_batch:
    pos [sum_s F_s N_s, 3], f [sum_s N_s], I [sum_s F_s Q_s], amp [.., 2].
    After construction, intensity() and grad() only launch kernels, so they
    can be captured in a torch.cuda.CUDAGraph and replayed.  forward_only=True
    builds the plan without the adjoint's buffers (xs_plan_create_forward);
    grad() then raises.
    """

    def __init__(self, systems, forward_only: bool = False):
        self._layout(systems)
        h = ctypes.c_void_p()
        create = _lib.load().xs_plan_create_forward if forward_only else _lib.load().xs_plan_create
        _lib.check(create(ctypes.byref(self._st), _ptr(self.q), ctypes.byref(h), _stream()))
        self._h = h

    def _layout(self, systems):
        self._h = ctypes.c_void_p()
        if not systems:
            raise ValueError("a plan needs at least one system")
        for i, (_, _, q, _) in enumerate(systems):
            _need(q, "q[%d]" % i)
        self.n_atoms = [int(n) for n, _, _, _ in systems]
        self.n_frames = [int(t) for _, t, _, _ in systems]
        self.n_q = [int(q.shape[0]) for _, _, q, _ in systems]
        boxes = np.stack([_box3(bx, None) for _, _, _, bx in systems])
        self.batch = make_batch(self.n_atoms, self.n_q, self.n_frames, boxes)
        self.q = torch.cat([q for _, _, q, _ in systems]).contiguous()
        self.total_out = self.batch.total_out
        self.total_pos = int(np.sum(np.asarray(self.n_atoms) * np.asarray(self.n_frames)))
        self.total_f = int(np.sum(self.n_atoms))
        self._st = self.batch.struct()

    @classmethod
    def single(cls, n_atoms: int, n_frames: int, q: torch.Tensor, box, forward_only: bool = False):
        return cls([(n_atoms, n_frames, q, box)], forward_only=forward_only)

    def _check(self, pos, f):
        _need(pos, "pos"), _need(f, "f")
        if pos.numel() != 3 * self.total_pos or f.numel() != self.total_f:
            raise ValueError("pos / f do not match the plan's batch layout")

    def intensity(self, pos, f, I=None, amp=None, want_amp=True):
        self._check(pos, f)
        dev = pos.device
        if I is None:
            I = torch.empty(self.total_out, dtype=torch.float64, device=dev)
        if amp is None and want_amp:
            amp = torch.empty((self.total_out, 2), dtype=torch.float64, device=dev)
        _lib.check(_lib.load().xs_plan_intensity(self._h, _ptr(pos), _ptr(f), _ptr(I), _ptr(amp),
                                                 _stream()))
        return I, amp

    def grad(self, pos, f, amp, dL_dI, retile=True, g32=None, g64=None):
        self._check(pos, f)
        _need(amp, "amp"), _need(dL_dI, "dL_dI")
        if g32 is None and g64 is None:
            g32 = torch.empty((self.total_pos, 3), dtype=torch.float32, device=pos.device)
        _lib.check(_lib.load().xs_plan_grad(self._h, _ptr(pos), _ptr(f), _ptr(amp), _ptr(dL_dI),
                                            1 if retile else 0, _ptr(g32), _ptr(g64), _stream()))
        return g32 if g32 is not None else g64

    def describe(self) -> dict:
        """Segments, segments on the lattice form, work items and device bytes (xs_plan_describe)."""
        info = _lib.XsPlanInfo()
        _lib.check(_lib.load().xs_plan_describe(self._h, ctypes.byref(info)))
        return {k: getattr(info, k) for k, _ in _lib.XsPlanInfo._fields_}

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _lib.check(_lib.load().xs_plan_destroy(self._h))
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class SpeciesPlan(Plan):
    """FP32C batch plan with q-dependent form factors per species (xs_plan_create_species).

    systems as for Plan; species: int32 GPU tensor [sum_s N_s] in the packed layout of f
    (read once here); coef: [n_species, 9] host array (a_1..a_4, b_1..b_4, c).  After
    construction intensity() and grad() only launch kernels (capturable in a graph).
    """

    def __init__(self, systems, species: torch.Tensor, coef):
        self._layout(systems)
        if not isinstance(species, torch.Tensor) or not species.is_cuda or species.dtype != torch.int32:
            raise ValueError("species must be an int32 tensor in GPU memory")
        if species.shape != (self.total_f,) or not species.is_contiguous():
            raise ValueError("species must be a contiguous [sum_s N_s] tensor")
        self.coef = np.ascontiguousarray(coef, dtype=np.float64).reshape(-1, 9)
        self.species = species
        h = ctypes.c_void_p()
        _lib.check(_lib.load().xs_plan_create_species(ctypes.byref(self._st), _ptr(self.q), _ptr(species),
                                                      self.coef.shape[0],
                                                      self.coef.ctypes.data_as(ctypes.c_void_p),
                                                      ctypes.byref(h), _stream()))
        self._h = h

    def _check_pos(self, pos):
        _need(pos, "pos")
        if pos.numel() != 3 * self.total_pos:
            raise ValueError("pos does not match the plan's batch layout")

    def intensity(self, pos, I=None, amp=None, want_amp=True):
        self._check_pos(pos)
        dev = pos.device
        if I is None:
            I = torch.empty(self.total_out, dtype=torch.float64, device=dev)
        if amp is None and want_amp:
            amp = torch.empty((self.total_out, 2), dtype=torch.float64, device=dev)
        _lib.check(_lib.load().xs_plan_intensity_species(self._h, _ptr(pos), _ptr(I), _ptr(amp), _stream()))
        return I, amp

    def grad(self, pos, amp, dL_dI, retile=True, g32=None, g64=None):
        self._check_pos(pos)
        _need(amp, "amp"), _need(dL_dI, "dL_dI")
        if g32 is None and g64 is None:
            g32 = torch.empty((self.total_pos, 3), dtype=torch.float32, device=pos.device)
        _lib.check(_lib.load().xs_plan_grad_species(self._h, _ptr(pos), _ptr(amp), _ptr(dL_dI),
                                                    1 if retile else 0, _ptr(g32), _ptr(g64), _stream()))
        return g32 if g32 is not None else g64
