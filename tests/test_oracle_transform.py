"""Pins for the oracle's transforms (Sections 2.3, 3.1-3.4).

* sYlm: Eq. (ssh_wigner) against the Goldberg form Eq. (ssh_goldberg) and, at
  s = 0, against scipy's scalar harmonics Eq. (shf); orthonormality by an
  exact quadrature.
* inverse: against the brute-force sum Eq. (ssht_inv) with harmonics built from
  the Wigner sum (no Risbo, no FFT).
* forward: against the least-squares solution on the samples (the unique
  band-limited answer), plus round trips and unit vectors.
* the quadrature weight w(p) against numerical integration.
* planted mistakes: typical slips in the oracle (wrong spin column, transposed
  Delta, dropped phase, wrong weights at odd offsets, wrong extension parity)
  make the brute-force pins fail.
"""

import math

import numpy as np
import pytest
import scipy.integrate as si
import scipy.special as sps

import oracle
from oracle import transform as T
from closed_forms import (forward_lstsq, inverse_direct, sylm_goldberg, sylm_wigner)
import sht_synth


# --------------------------------------------------------------- harmonics ---

def test_goldberg_form_is_wigner_form_times_minus_one_to_m():
    """Eq. (ssh_goldberg) as printed equals (-1)^m Eq. (ssh_wigner) (reading A.R5)."""
    rng = np.random.default_rng(1)
    for _ in range(3):
        th, ph = float(rng.uniform(0.2, 2.9)), float(rng.uniform(0, 2 * math.pi))
        for l in range(0, 4):
            for s in range(-l, l + 1):
                for m in range(-l, l + 1):
                    a = sylm_wigner(l, m, s, th, ph)
                    b = sylm_goldberg(l, m, s, th, ph)
                    assert abs(b - (-1) ** m * a) < 1e-12, (l, m, s)


def test_spin_zero_is_scalar_harmonic():
    """sY_lm at s = 0 equals Y_lm of Eq. (shf) (scipy, Condon-Shortley phase)."""
    rng = np.random.default_rng(2)
    for _ in range(4):
        th, ph = float(rng.uniform(0.1, 3.0)), float(rng.uniform(0, 6.2))
        for l in range(0, 7):
            for m in range(-l, l + 1):
                ref = sps.sph_harm_y(l, m, th, ph)
                assert abs(sylm_wigner(l, m, 0, th, ph) - ref) < 1e-13


@pytest.mark.parametrize("s", [0, 1, -2])
def test_sylm_orthonormal_by_exact_quadrature(s):
    """Orthonormality (Section 2.3) with Gauss-Legendre in cos(theta) x uniform phi."""
    L = 5
    xg, wg = np.polynomial.legendre.leggauss(2 * L + 2)
    thetas = np.arccos(xg)
    nphi = 2 * L + 1
    phis = 2 * math.pi * np.arange(nphi) / nphi
    idx = [(l, m) for l in range(abs(s), L) for m in range(-l, l + 1)]
    Y = np.array([[sylm_wigner(l, m, s, th, ph) for th in thetas for ph in phis] for l, m in idx])
    w = np.repeat(wg, nphi) * (2 * math.pi / nphi)
    G = (Y * w[None, :]) @ Y.conj().T
    assert np.abs(G - np.eye(len(idx))).max() < 1e-12


def test_quadrature_weight_against_numerical_integral():
    for p in range(-9, 10):
        re = si.quad(lambda t: math.sin(t) * math.cos(p * t), 0, math.pi, epsabs=1e-14)[0]
        im = si.quad(lambda t: math.sin(t) * math.sin(p * t), 0, math.pi, epsabs=1e-14)[0]
        w = T.quadrature_weight(np.array([p]))[0]
        assert abs(w - complex(re, im)) < 1e-12, p
    assert T.quadrature_weight(np.array([0]))[0] == 2.0


def test_sampling_nodes():
    L = 5
    th = T.theta_nodes(L)
    assert th.shape == (L,) and abs(th[-1] - math.pi) < 1e-15      # theta_{L-1} = pi kept
    assert abs(th[0] - math.pi / (2 * L - 1)) < 1e-15
    assert T.phi_nodes(L).shape == (2 * L - 1,)


# ----------------------------------------------------------------- inverse ---

@pytest.mark.parametrize("L,s", [(2, 0), (4, 0), (5, 1), (6, -1), (7, 2), (8, -2), (10, 3), (12, 0)])
def test_inverse_equals_brute_force_sum(L, s):
    f = sht_synth.gaussian_flm(L, s, 100 + L + 7 * s)
    a = oracle.inverse(f, L, s)
    b = inverse_direct(f, L, s)
    assert oracle.rel_l2(b, a) < 1e-13


def test_torus_synthesis_fft_route_equals_direct_double_sum():
    """The FFT with bin m mod N and half-sample phases equals Eq. (sht_inv_fast) summed directly."""
    L = 6
    N = 2 * L - 1
    rng = np.random.default_rng(5)
    F = rng.standard_normal((N, N)) + 1j * rng.standard_normal((N, N))
    g = T.torus_synthesis(F, L)
    th, ph = T.theta_nodes(L), T.phi_nodes(L)
    m = np.arange(-(L - 1), L)
    ref = np.zeros((L, N), dtype=complex)
    for t in range(L):
        for p in range(N):
            ref[t, p] = np.sum(F * np.exp(1j * (m[:, None] * ph[p] + m[None, :] * th[t])))
    assert np.abs(g - ref).max() < 1e-11


# ----------------------------------------------------------------- forward ---

@pytest.mark.parametrize("L,s", [(3, 0), (5, 1), (6, -2), (8, 2), (9, 0), (10, -1)])
def test_forward_equals_least_squares_on_samples(L, s):
    f = sht_synth.gaussian_flm(L, s, 300 + L + 11 * s)
    fmap = inverse_direct(f, L, s)
    ref = forward_lstsq(fmap, L, s)
    assert oracle.rel_l2(ref, f) < 1e-12          # lstsq recovers the truth
    got = oracle.forward(fmap, L, s)
    assert oracle.rel_l2(ref, got) < 1e-12


@pytest.mark.parametrize("L,s,l0,m0", [(6, 0, 0, 0), (6, 0, 3, -2), (7, 2, 2, 1), (7, -1, 6, 6)])
def test_forward_of_single_harmonic_is_unit_vector(L, s, l0, m0):
    f = np.zeros(L * L, complex)
    f[l0 * l0 + l0 + m0] = 1.0
    fmap = inverse_direct(f, L, s)
    got = oracle.forward(fmap, L, s)
    assert np.abs(got - f).max() < 1e-13


@pytest.mark.parametrize("L,s", [(8, 0), (32, 1), (64, -2), (128, 2)])
def test_round_trip_exact(L, s):
    f = sht_synth.gaussian_flm(L, s, 900 + L)
    g = oracle.forward(oracle.inverse(f, L, s), L, s)
    assert oracle.rel_l2(f, g) < 1e-13


@pytest.mark.slow
@pytest.mark.parametrize("L,s,spec,bar", [(256, 2, "inv_l_lp1", 1e-13), (1024, -2, "inv_lp1_sq", 1e-12)])
def test_round_trip_at_the_configuration_sizes(L, s, spec, bar):
    """The oracle's own round trip at the band-limits of the spin-2 and the
    batched configurations, with their spectra: the exactness that makes the
    oracle a valid reference there (the GPU bars are 1e-10 and 1e-5)."""
    f = sht_synth.gaussian_flm(L, s, sht_synth.SEED_BASE + 8100 + L, spec)
    g = oracle.forward(oracle.inverse(f, L, s), L, s)
    err = oracle.rel_l2(f, g)
    print(f"oracle round trip L={L} s={s}: {err:.3e}")
    assert err <= bar


def test_round_trip_at_the_largest_configuration_from_golden():
    """L = 2048 (four minutes of oracle time, so stored by
    tests/golden/make_golden.py --round-trip): the oracle's forward of its
    inverse of map 0 equals the input coefficients, regenerated here from
    their seed, at the stored orders, and over all L^2 coefficients."""
    import os
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "L2048_s0_b4.npz")
    wl = {w.name: w for w in sht_synth.WORKLOADS}["L2048_s0_b4"]
    with np.load(path) as d:
        idx, rt, rel_all = d["fwd_index"], d["rt_s0"], float(d["rt_rel_s0"])
    f = wl.flm(0)[0]
    assert oracle.rel_l2(f[idx], rt) <= 1e-12
    assert rel_all <= 1e-12


def test_batch_equals_single_and_forward_rows_subset():
    L, s = 12, 1
    F = np.stack([sht_synth.gaussian_flm(L, s, 40 + b) for b in range(3)])
    maps = oracle.inverse_batch(F, L, s)
    for b in range(3):
        assert np.abs(maps[b] - oracle.inverse(F[b], L, s)).max() < 1e-14
    full = oracle.forward_batch(maps, L, s)
    part = oracle.forward_rows(maps, L, s, ms=[-3, 0, 5])
    for l in range(L):
        for m in (-3, 0, 5):
            if abs(m) <= l:
                k = l * l + l + m
                assert np.abs(full[:, k] - part[:, k]).max() < 1e-13


def test_error_metrics():
    f = np.array([1.0, 2.0, 2.0])
    g = np.array([1.0, 2.0, 0.0])
    e = oracle.error_metrics(f, g)
    assert e["max"] == 2.0 and abs(e["mean"] - 2 / 3) < 1e-15 and e["median"] == 0.0
    assert abs(e["rms"] - math.sqrt(4 / 3)) < 1e-15 and abs(e["rel_rms"] - 2 / 3) < 1e-15


# ------------------------------------------------------- planted mistakes ---

def _inverse_with(monkeypatch, L, s, f, **patch):
    for name, fn in patch.items():
        monkeypatch.setattr(T, name, fn)
    return T.torus_synthesis(T.fourier_coefficients(f, L, s), L)


def test_planted_mistakes_are_caught(monkeypatch):
    L, s = 6, 2
    f = sht_synth.gaussian_flm(L, s, 77)
    truth = inverse_direct(f, L, s)
    assert oracle.rel_l2(truth, oracle.inverse(f, L, s)) < 1e-13

    orig_planes = T.delta_planes

    def transposed(L_, beta=math.pi / 2):
        for l, D in orig_planes(L_, beta):
            yield l, D.T.copy()

    with monkeypatch.context() as mp:
        mp.setattr(T, "delta_planes", transposed)
        bad = T.torus_synthesis(T.fourier_coefficients(f, L, s), L)
    assert oracle.rel_l2(truth, bad) > 1e-3

    with monkeypatch.context() as mp:            # spin column +s instead of -s
        bad = T.torus_synthesis(T.fourier_coefficients(f, L, -s), L)
    assert oracle.rel_l2(truth, bad) > 1e-3

    with monkeypatch.context() as mp:            # phase i^{-(m+s)} dropped
        mp.setattr(T, "_ipow", lambda k: 1.0 + 0j)
        bad = T.torus_synthesis(T.fourier_coefficients(f, L, s), L)
    assert oracle.rel_l2(truth, bad) > 1e-3

    # forward slips
    fl = sht_synth.gaussian_flm(L, 1, 78)
    fmap = inverse_direct(fl, L, 1)
    ref = forward_lstsq(fmap, L, 1)
    assert oracle.rel_l2(ref, oracle.forward(fmap, L, 1)) < 1e-12

    orig_w = T.quadrature_weight

    def w_no_odd_zeros(p):                       # 2/(1-p^2) also at odd |p| > 1
        p = np.asarray(p)
        out = orig_w(p)
        odd = (p % 2 == 1) & (np.abs(p) > 1)
        out[odd] = 2.0 / (1.0 - p[odd].astype(float) ** 2)
        return out

    with monkeypatch.context() as mp:
        mp.setattr(T, "quadrature_weight", w_no_odd_zeros)
        bad = T.forward(fmap, L, 1)
    assert oracle.rel_l2(ref, bad) > 1e-3

    orig_ext = T.theta_extend
    with monkeypatch.context() as mp:            # always the even extension
        mp.setattr(T, "theta_extend", lambda Q, L_, s_, ms: orig_ext(Q, L_, 0, [0] * len(ms)))
        bad = T.forward(fmap, L, 1)
    assert oracle.rel_l2(ref, bad) > 1e-3


@pytest.mark.parametrize("s", [0, 1, -2, 3])
def test_imaginary_weights_cancel_in_the_forward(monkeypatch, s):
    """w(+-1) = +-i pi/2 drops out of f_lm: the sum over +-m' pairs cancels it
    (Delta_{-m',m} Delta_{-m',-s} = (-1)^{m+s} Delta_{m'm} Delta_{m',-s} and the
    extension has parity (-1)^{m+s}), so a real, even-offset kernel suffices."""
    L = 9
    f = sht_synth.gaussian_flm(L, s, 500 + s)
    fmap = oracle.inverse(f, L, s)

    orig_w = T.quadrature_weight

    def w_real(p):
        return orig_w(p).real.astype(complex)

    monkeypatch.setattr(T, "quadrature_weight", w_real)
    assert oracle.rel_l2(f, T.forward(fmap, L, s)) < 1e-13


@pytest.mark.parametrize("L,s", [(6, 1), (8, 2), (9, -3)])
def test_spin_pair_relation(L, s):
    """Section 3.3: for f_{-s} = conj(f_s), {}_{-s}f_{lm} = (-1)^{s+m} conj({}_s f_{l,-m})."""
    f = sht_synth.gaussian_flm(L, s, 31 + L)
    fmap = oracle.inverse(f, L, s)
    g = oracle.forward(np.conj(fmap), L, -s)
    want = np.zeros_like(f)
    for l in range(abs(s), L):
        for m in range(-l, l + 1):
            want[l * l + l + m] = (-1) ** (s + m) * np.conj(f[l * l + l - m])
    assert oracle.rel_l2(want, g) < 1e-12
