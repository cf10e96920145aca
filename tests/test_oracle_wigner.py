"""Pins for the oracle's Delta^l = d^l(pi/2) (Risbo recursion, Section 2.2).

Each check ties the oracle to something other than itself: exact rational
values of the Wigner sum, the paper's Jacobi form Eq. (wignerd_b), Legendre
functions (the s = 0 reduction in Section 2.3), orthogonality, the symmetry
relations Eq. (wignerd_sym1/2/6) and Eq. (wigner_sum_reln).
"""

import math

import numpy as np
import pytest
import scipy.special as sps

from closed_forms import delta_exact, wigner_d_jacobi, wigner_d_sum
from oracle.wigner import DeltaRisbo, delta_plane, delta_planes


def planes(L):
    return {l: D.copy() for l, D in delta_planes(L)}


def test_risbo_matches_exact_rational_wigner_sum():
    """Delta^l_{m'm} vs the exact Wigner sum at pi/2, every entry, l <= 24."""
    P = planes(25)
    worst = 0.0
    for l in list(range(0, 13)) + [17, 24]:
        D = P[l]
        for mp in range(-l, l + 1):
            for m in range(-l, l + 1):
                worst = max(worst, abs(D[l + mp, l + m] - delta_exact(l, mp, m)))
    assert worst < 5e-15


def test_jacobi_form_equals_wigner_sum():
    """Eq. (wignerd_b) (Jacobi form) and the Wigner sum agree: fixes the convention."""
    rng = np.random.default_rng(7)
    for _ in range(6):
        beta = float(rng.uniform(0.1, 3.0))
        for l in range(0, 5):
            for m in range(-l, l + 1):
                for n in range(-l, l + 1):
                    a = wigner_d_jacobi(l, m, n, beta)
                    b = wigner_d_sum(l, m, n, beta)
                    assert abs(a - b) < 1e-13, (l, m, n, beta)
    # standard convention: d^1_{10}(beta) = -sin(beta)/sqrt(2)
    assert abs(wigner_d_sum(1, 1, 0, 0.7) + math.sin(0.7) / math.sqrt(2)) < 1e-15


def test_risbo_vs_jacobi_form_at_pi_over_2():
    D = delta_plane(9)
    l = 9
    for m in range(-l, l + 1):
        for n in range(-l, l + 1):
            assert abs(D[l + m, l + n] - wigner_d_jacobi(l, m, n, math.pi / 2)) < 1e-14


@pytest.mark.parametrize("l", [1, 5, 50, 200])
def test_orthogonality(l):
    D = delta_plane(l)
    assert np.abs(D.T @ D - np.eye(2 * l + 1)).max() < 1e-13 * max(1, l) ** 0.5


@pytest.mark.parametrize("l", [3, 8, 40])
def test_square_is_rotation_by_pi(l):
    """Delta Delta = d(pi/2 + pi/2) = d(pi); d(pi) from the Wigner sum at beta = pi."""
    D = delta_plane(l)
    dpi = np.array([[wigner_d_sum(l, mp, m, math.pi) if l <= 8 else np.nan
                     for m in range(-l, l + 1)] for mp in range(-l, l + 1)])
    sq = D @ D
    if l <= 8:
        assert np.abs(sq - dpi).max() < 1e-13
    # closed form of d(pi): (-1)^{l+m'} delta_{m', -m}
    ref = np.zeros_like(sq)
    for mp in range(-l, l + 1):
        ref[l + mp, l - mp] = (-1) ** (l + mp)
    assert np.abs(sq - ref).max() < 1e-12


def test_symmetries_and_zeros():
    for l in [0, 1, 2, 7, 30, 101]:
        D = delta_plane(l)
        ms = range(-l, l + 1)
        for mp in ms:
            for m in ms:
                v = D[l + mp, l + m]
                # Eq. (wignerd_sym1): d_{m'm} = (-1)^{m'-m} d_{-m',-m}
                assert abs(v - (-1) ** (mp - m) * D[l - mp, l - m]) < 1e-14
                # Eq. (wignerd_sym2) at pi/2: d_{m'm} = (-1)^{l-m} d_{-m',m}
                assert abs(v - (-1) ** (l - m) * D[l - mp, l + m]) < 1e-14
                # Eq. (wignerd_sym6): d_{m',-m} = (-1)^{l+m'} d_{m'm}
                assert abs(D[l + mp, l - m] - (-1) ** (l + mp) * v) < 1e-14
            # zero for m = 0 and odd l + m' (text after Eq. (wignerd_sym6))
            if (l + mp) % 2 == 1:
                assert abs(D[l + mp, l]) < 1e-15


def test_edge_closed_forms():
    """Delta^l_{l,m} = (-1)^{l-m} 2^-l sqrt(C(2l, l+m)); Delta^l_{m,l} = 2^-l sqrt(C(2l, l+m))."""
    for l in [1, 4, 13, 60, 300]:
        D = delta_plane(l)
        for m in range(-l, l + 1):
            lg = 0.5 * (math.lgamma(2 * l + 1) - math.lgamma(l + m + 1) - math.lgamma(l - m + 1)) \
                - l * math.log(2)
            e = math.exp(lg)
            if e < 1e-250:
                continue
            assert abs(D[2 * l, l + m] - (-1) ** (l - m) * e) <= 1e-12 * e + 1e-300
            assert abs(D[l + m, 2 * l] - e) <= 1e-12 * e + 1e-300


def test_column_zero_is_legendre_at_equator():
    """Delta^l_{m0} = sqrt((l-m)!/(l+m)!) P_l^m(0) (s = 0 reduction, Section 2.3)."""
    for l in [0, 1, 2, 5, 10, 20]:
        D = delta_plane(l)
        for m in range(0, l + 1):
            ref = math.sqrt(math.factorial(l - m) / math.factorial(l + m)) * sps.lpmv(m, l, 0.0)
            assert abs(D[l + m, l] - ref) < 1e-13


def test_fourier_series_of_d_eq_wigner_sum_reln():
    """Eq. (wigner_sum_reln): d_{mn}(beta) = i^{n-m} sum_m' Delta_{m'm} Delta_{m'n} e^{i m' beta}."""
    rng = np.random.default_rng(3)
    for l in [1, 3, 6, 10]:
        D = delta_plane(l)
        mps = np.arange(-l, l + 1)
        for _ in range(3):
            beta = float(rng.uniform(0, math.pi))
            e = np.exp(1j * mps * beta)
            for m in range(-l, l + 1):
                for n in range(-l, l + 1):
                    val = (1j) ** ((n - m) % 4) * np.sum(D[:, l + m] * D[:, l + n] * e)
                    assert abs(val.imag) < 1e-13
                    assert abs(val.real - wigner_d_sum(l, m, n, beta)) < 1e-13


def test_recursions_used_by_the_kernels_hold():
    """The two three-term recursions the GPU kernels run (in l at fixed m', m; in m'
    at fixed l, m) are identities of d^l(pi/2); checked on the oracle's planes."""
    P = planes(40)
    for m in range(0, 12):
        for mp in range(0, 12):
            l0 = max(m, mp, 1)
            for l in range(l0, 38):
                lhs = l * math.sqrt(((l + 1) ** 2 - m * m) * ((l + 1) ** 2 - mp * mp)) \
                    * P[l + 1][l + 1 + mp, l + 1 + m]
                prev = P[l - 1][l - 1 + mp, l - 1 + m] if l - 1 >= max(m, mp) else 0.0
                rhs = -(2 * l + 1) * m * mp * P[l][l + mp, l + m] \
                    - (l + 1) * math.sqrt((l * l - m * m) * (l * l - mp * mp)) * prev
                assert abs(lhs - rhs) < 1e-12 * max(1.0, abs(lhs))
    for l in [5, 17, 39]:
        D = P[l]
        for m in range(0, l + 1):
            for mp in range(-l + 1, l):
                lhs = math.sqrt((l + mp) * (l - mp + 1)) * D[l + mp - 1, l + m] \
                    + math.sqrt((l - mp) * (l + mp + 1)) * D[l + mp + 1, l + m]
                assert abs(lhs - 2 * m * D[l + mp, l + m]) < 1e-12 * max(1.0, l)


def test_precompute_count_formula():
    """Section 4.1: sum_{l=0}^{Lp} (l+1)^2 = Lp^3/3 + 3Lp^2/2 + 13Lp/6 + 1 entries with m, n >= 0."""
    for Lp in [0, 1, 7, 50, 1023]:
        count = sum((l + 1) ** 2 for l in range(Lp + 1))
        assert 6 * count == 2 * Lp ** 3 + 9 * Lp ** 2 + 13 * Lp + 6


def test_numpy_and_c_half_steps_agree():
    a, b = DeltaRisbo(use_c=True), DeltaRisbo(use_c=False)
    for _ in range(30):
        a.advance()
        b.advance()
    assert np.array_equal(a.plane, b.plane)
