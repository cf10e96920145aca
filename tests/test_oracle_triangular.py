"""Pins of the paper's own forward transform (per-order triangular systems,
Section 3.4.2) and of its stability experiment (Section 4.2)."""

import math

import numpy as np
import pytest

import oracle
import sht_synth
from oracle import triangular as T
from oracle.transform import inverse


def test_system_reproduces_the_torus_coefficients_of_a_band_limited_map():
    """D_{m0} f_{., m0} (Eq. (matrix_fwd)) equals the F_{m0 m'}, m' >= 0, that
    the extension and DFT (Sections 3.2, 3.4.1) give for the map of f."""
    for L, s in [(5, 0), (6, 1), (7, -2), (9, 3)]:
        f = sht_synth.gaussian_flm(L, s, 100 + L)
        F = T.torus_rows(inverse(f, L, s), L, s)
        mats = T.system_matrices(L, s, range(-(L - 1), L))
        for m0 in range(-(L - 1), L):
            col = np.zeros(L, dtype=np.complex128)
            for l in range(max(abs(m0), abs(s)), L):
                col[l] = f[l * l + l + m0]
            assert np.allclose(mats[m0] @ col, F[(L - 1) + m0], rtol=0, atol=1e-12), (L, s, m0)


def test_wrong_extension_parity_breaks_the_system():
    """Planted mistake: with the other parity's extension the torus
    coefficients no longer satisfy Eq. (matrix_fwd)."""
    L, s = 6, 0
    f = sht_synth.gaussian_flm(L, s, 3)
    fmap = inverse(f, L, s)
    from oracle.transform import phi_analysis, theta_analysis, theta_extend
    ms = list(range(-(L - 1), L))
    Q = phi_analysis(fmap[None], L)
    wrong = theta_analysis(theta_extend(Q, L, s + 1, ms), L)[0][:, L - 1:]
    mats = T.system_matrices(L, s, ms)
    m0 = 2
    col = np.array([f[l * l + l + m0] if l >= m0 else 0 for l in range(L)], dtype=np.complex128)
    assert not np.allclose(mats[m0] @ col, wrong[(L - 1) + m0], atol=1e-6)


@pytest.mark.parametrize("L,s", [(4, 0), (6, 1), (8, -2), (8, 0)])
def test_triangular_forward_is_exact_at_low_band_limits(L, s):
    """Section 4.2: machine-precision round trips for very low band-limits."""
    f = sht_synth.gaussian_flm(L, s, 7 + L)
    g = T.forward_triangular(inverse(f, L, s), L, s)
    assert oracle.rel_l2(f, g) < 1e-12


def test_spin0_even_odd_split_equals_plain_back_substitution():
    L = 12
    f = sht_synth.gaussian_flm(L, 0, 5)
    fmap = inverse(f, L, 0)
    a = T.forward_triangular(fmap, L, 0, split_spin0=True)
    b = T.forward_triangular(fmap, L, 0, split_spin0=False)
    assert oracle.rel_l2(b, a) < 1e-12
    # the split really separates: D vanishes off the even/odd pattern of l + m'
    D = T.system_matrices(L, 0, [4])[4]
    for mp in range(L):
        for l in range(L):
            if (l + mp) % 2:
                assert abs(D[mp, l]) < 1e-15


def test_conditioning_of_the_printed_example():
    """Section 4.2 prints condition number 6e14 for the s = 0 system with
    band-limit 50 and m0 = 38 (degrees l <= 49 here, the reading of the
    band-limit used throughout).  The all-rows system is well conditioned."""
    c_sq, c_all = T.condition_numbers(50, 0, 38)
    assert 6e14 / 2 < c_sq < 6e14 * 2, c_sq
    assert c_all < 2.0, c_all


def test_instability_grows_with_band_limit_and_least_squares_fixes_it():
    """The Section 4.2 experiment (real s = 0 test functions from U[-1, 1]
    coefficients): machine precision at L = 8, errors exploding by L = 64;
    the least-squares solution of all rows stays exact."""
    rows = T.stability_errors([8, 32, 64], n_maps=2)
    err = {r["L"]: r["rel_rms"] for r in rows}
    assert err[8] < 1e-13
    assert err[32] > 1e3 * err[8]
    assert err[64] > 1e-3
    L = 64
    f = sht_synth.uniform_flm(L, 0, 11)
    g = T.forward_lstsq(inverse(f, L, 0), L, 0)
    assert oracle.rel_l2(f, g) < 1e-12
