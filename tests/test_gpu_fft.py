"""FFT-based method (Sec. 3.2, Algorithm 2) on the GPU (xs_fft_intensity) against the
numpy oracle of the same steps, and its agreement with the exact direct sum."""
import math

import numpy as np
import pytest
import torch

import oracle
from oracle import fft_method as FM

from _gpu import dev, host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def api():
    from paper_2204_13241_amd import api
    return api


def _case(n_atoms, L, seed):
    rng = np.random.default_rng(seed)
    pos = rng.uniform(0, L, (n_atoms, 3))
    f = np.where(rng.random(n_atoms) < 0.25, 2.5, 1.0)
    return pos, f


# the density is summed with atomics and transformed by another FFT than numpy's: the two
# differ by rounding, which the division by f^eta magnifies where f^eta is small; compared
# where f^eta is above 1e-4 of its peak, against the incoherent level sum f^2
@pytest.mark.parametrize("n,eta,k", [(48, 0.3, None), (45, 0.35, 12), (64, 0.25, 7)])
def test_fft_method_against_oracle(api, n, eta, k):
    L = 14.0
    pos, f = _case(150, L, n)
    k = k or FM.cutoff_points(L, n, eta)
    print("fft n=%d eta=%g k=%d" % (n, eta, k), flush=True)
    I, amp = api.fft_intensity(dev(pos), dev(f), L, n, eta, k, return_amp=True)
    torch.cuda.synchronize()
    I_ref = FM.intensity(pos, f, L, n, eta, k)
    G = np.abs(FM.gaussian_transform(L, n, eta, k))
    use = G > 1e-4 * G.max()
    inc = float(np.sum(f * f))
    Ih = host(I)
    err = float(np.max(np.abs(Ih[use] - I_ref[use]) / np.maximum(I_ref[use], inc)))
    print("fft n=%d: max scaled error vs oracle %.2e over %d wavevectors" % (n, err, use.sum()), flush=True)
    assert err <= 1e-10
    a = host(amp)
    assert np.allclose((a[..., 0] ** 2 + a[..., 1] ** 2)[use], Ih[use], rtol=1e-12, atol=1e-12 * inc)


def test_fft_amplitude_matches_the_direct_sum_at_low_q(api):
    # with a wide cut (14 eta) the method's error is far below 1e-8 at low |q|: the
    # amplitude p^e = p^eta / f^eta equals the direct method's sum_j f_j e^{-i q.r_j}
    L, n, eta = 14.0, 72, 0.3
    pos, f = _case(150, L, 7)
    k = int(math.floor(14 * eta * n / L)) + 1
    I, amp = api.fft_intensity(dev(pos), dev(f), L, n, eta, k, return_amp=True)
    torch.cuda.synchronize()
    hs = np.array([[0, 3, -2], [1, -4, 2], [2, 2, 2], [-5, 0, 1], [0, 0, 1]])
    q = hs * (2 * math.pi / L)
    I_ref, amp_ref = oracle.intensity(pos, f, q)
    a = host(amp)
    Ih = host(I)
    inc = float(np.sum(f * f))
    for h, ir, ar in zip(hs, I_ref, amp_ref):
        i = tuple(int(x) % n for x in h)
        assert abs(Ih[i] - ir) <= 1e-8 * max(ir, inc)
        assert abs(a[i][0] - ar[0]) <= 1e-8 * math.sqrt(max(ir, inc))
        assert abs(a[i][1] - ar[1]) <= 1e-8 * math.sqrt(max(ir, inc))


def test_fft_single_atom_and_empty_frame(api):
    L, n, eta = 10.0, 40, 0.3
    k = FM.cutoff_points(L, n, eta)
    d = L / n
    I = api.fft_intensity(dev(np.array([[3 * d, 17 * d, 39 * d]])), dev(np.array([2.5])), L, n, eta, k)
    G = np.abs(FM.gaussian_transform(L, n, eta, k))
    use = G > 1e-4 * G.max()
    assert np.max(np.abs(host(I)[use] - 6.25)) <= 1e-10 * 6.25
    I0 = api.fft_intensity(dev(np.zeros((0, 3))), dev(np.zeros(0)), L, n, eta, k)
    torch.cuda.synchronize()
    assert np.all(host(I0) == 0.0)
