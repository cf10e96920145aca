"""Closed forms used to pin the oracle.  Independent of oracle/ (no shared code).

* :func:`delta_exact` -- d^l_{m'm}(pi/2) from the standard Wigner sum, in exact
  rational arithmetic: at beta = pi/2 every term carries 2^{-l}, so
  Delta^2 is rational and the sign is that of a rational sum.
* :func:`wigner_d_sum` -- the same sum at any beta (mpmath, 40 digits).
* :func:`wigner_d_jacobi` -- Eq. (wignerd_b) with the Jacobi polynomial written
  as its finite binomial sum (valid for negative integer parameters).
* :func:`sylm_wigner` -- Eq. (ssh_wigner) built on :func:`wigner_d_sum`.
* :func:`sylm_goldberg` -- Eq. (ssh_goldberg) as printed.
* :func:`inverse_direct`, :func:`forward_lstsq` -- brute-force transforms on the
  sampling of Eq. (nodes_theta) / Eq. (nodes_phi), rings t < L.
"""

from __future__ import annotations

import math
from fractions import Fraction
from functools import lru_cache

import mpmath
import numpy as np

mpmath.mp.dps = 40


@lru_cache(maxsize=None)
def _fact(n: int) -> int:
    return math.factorial(n)


def _wigner_terms(l: int, mp: int, m: int):
    """Yield (k, sign, denominator) of the standard Wigner sum."""
    for k in range(0, 2 * l + 1):
        a, b, c = l + m - k, l - k - mp, k - m + mp
        if a < 0 or b < 0 or c < 0:
            continue
        yield k, (-1) ** (k - m + mp), _fact(a) * _fact(k) * _fact(b) * _fact(c)


def delta_exact(l: int, mp: int, m: int) -> float:
    """d^l_{mp,m}(pi/2), exact to double rounding (rational square, exact sign)."""
    if abs(mp) > l or abs(m) > l:
        return 0.0
    S = Fraction(0)
    for k, sg, den in _wigner_terms(l, mp, m):
        S += Fraction(sg, den)
    if S == 0:
        return 0.0
    A = _fact(l + mp) * _fact(l - mp) * _fact(l + m) * _fact(l - m)
    sq = Fraction(A) * S * S / (4 ** l)
    val = mpmath.sqrt(mpmath.mpf(sq.numerator) / mpmath.mpf(sq.denominator))
    return float(val) if S > 0 else -float(val)


def wigner_d_sum(l: int, mp: int, m: int, beta: float) -> float:
    """Standard Wigner sum for d^l_{mp,m}(beta) (convention d^1_{10} = -sin/sqrt2)."""
    if abs(mp) > l or abs(m) > l:
        return 0.0
    b = mpmath.mpf(beta)
    cb, sb = mpmath.cos(b / 2), mpmath.sin(b / 2)
    pref = mpmath.sqrt(_fact(l + mp) * _fact(l - mp) * _fact(l + m) * _fact(l - m))
    tot = mpmath.mpf(0)
    for k, sg, den in _wigner_terms(l, mp, m):
        tot += sg * cb ** (2 * l - 2 * k + m - mp) * sb ** (2 * k - m + mp) / den
    return float(pref * tot)


def _gbinom(x: int, k: int) -> Fraction:
    """Generalised binomial coefficient C(x, k) for integer x (any sign), k >= 0."""
    if k < 0:
        return Fraction(0)
    num = 1
    for j in range(k):
        num *= (x - j)
    return Fraction(num, _fact(k))


def jacobi_poly(n: int, a: int, b: int, x):
    """P_n^{(a,b)}(x) = sum_j C(n+a, n-j) C(n+b, j) ((x-1)/2)^j ((x+1)/2)^{n-j}."""
    x = mpmath.mpf(x)
    tot = mpmath.mpf(0)
    for j in range(n + 1):
        c = _gbinom(n + a, n - j) * _gbinom(n + b, j)
        tot += mpmath.mpf(c.numerator) / c.denominator * ((x - 1) / 2) ** j * ((x + 1) / 2) ** (n - j)
    return tot


def wigner_d_jacobi(l: int, m: int, n: int, beta: float) -> float:
    """Eq. (wignerd_b): d^l_{mn}(beta) via the Jacobi polynomial P_{l-n}^{(n-m, n+m)}.

    Evaluated as printed for n >= |m|; other index pairs are brought there with
    the paper's symmetries Eq. (wignerd_sym1)/(wignerd_sym3) and the transpose
    d_{mn} = (-1)^{m-n} d_{nm}, each of which maps the printed form to itself.
    """
    b = mpmath.mpf(beta)
    if n >= abs(m):
        pref = mpmath.sqrt(mpmath.mpf(_fact(l + n) * _fact(l - n)) / (_fact(l + m) * _fact(l - m)))
        val = pref * mpmath.sin(b / 2) ** (n - m) * mpmath.cos(b / 2) ** (n + m) \
            * jacobi_poly(l - n, n - m, n + m, mpmath.cos(b))
        return float(val)
    if -n >= abs(m):          # sym1: d_{mn} = (-1)^{m-n} d_{-m,-n}
        return (-1) ** (m - n) * wigner_d_jacobi(l, -m, -n, beta)
    # |m| > |n|: transpose
    return (-1) ** (m - n) * wigner_d_jacobi(l, n, m, beta)


def sylm_wigner(l: int, m: int, s: int, theta: float, phi: float) -> complex:
    """Eq. (ssh_wigner): (-1)^s sqrt((2l+1)/4pi) d^l_{m,-s}(theta) e^{i m phi}."""
    if l < abs(s) or abs(m) > l:
        return 0j
    return ((-1) ** s * math.sqrt((2 * l + 1) / (4 * math.pi))
            * wigner_d_sum(l, m, -s, theta) * complex(math.cos(m * phi), math.sin(m * phi)))


def sylm_goldberg(l: int, m: int, s: int, theta: float, phi: float) -> complex:
    """Eq. (ssh_goldberg) exactly as printed (binomial sum in cot(theta/2))."""
    th = mpmath.mpf(theta)
    pref = mpmath.sqrt(mpmath.mpf(2 * l + 1) / (4 * mpmath.pi)
                       * mpmath.mpf(_fact(l + m) * _fact(l - m)) / (_fact(l + s) * _fact(l - s)))
    cot = mpmath.cot(th / 2)
    tot = mpmath.mpf(0)
    for r in range(0, l - s + 1):
        k2 = s - m + r
        if k2 < 0 or k2 > l + s:
            continue
        tot += (math.comb(l - s, r) * math.comb(l + s, k2) * (-1) ** (l - s - r)
                * cot ** (s - m + 2 * r))
    val = pref * mpmath.sin(th / 2) ** (2 * l) * tot
    return complex(float(val)) * complex(math.cos(m * phi), math.sin(m * phi))


def sylm_matrix(L: int, s: int) -> np.ndarray:
    """Y[(t,p), l*l+l+m] = sY_lm(theta_t, phi_p) on rings t < L (brute force)."""
    N = 2 * L - 1
    th = [math.pi * (2 * t + 1) / N for t in range(L)]
    ph = [math.pi * (2 * p + 1) / N for p in range(N)]
    Y = np.zeros((L * N, L * L), dtype=np.complex128)
    for l in range(L):
        for m in range(-l, l + 1):
            if l < abs(s):
                continue
            dcol = np.array([wigner_d_sum(l, m, -s, t) for t in th])
            e = np.exp(1j * m * np.asarray(ph))
            Y[:, l * l + l + m] = ((-1) ** s * math.sqrt((2 * l + 1) / (4 * math.pi))
                                   * np.outer(dcol, e)).ravel()
    return Y


def inverse_direct(flm: np.ndarray, L: int, s: int) -> np.ndarray:
    """Brute force f(theta_t, phi_p) = sum_lm f_lm sY_lm, Eq. (ssht_inv); [L, N]."""
    N = 2 * L - 1
    return (sylm_matrix(L, s) @ np.asarray(flm)).reshape(L, N)


def forward_lstsq(fmap: np.ndarray, L: int, s: int) -> np.ndarray:
    """The f_lm (l >= |s|) whose synthesis reproduces the samples, by least squares.

    Unique for band-limited data: the L(2L-1) samples determine the L^2 - s^2
    coefficients (the synthesis matrix has full column rank on this grid).
    """
    Y = sylm_matrix(L, s)
    keep = [l * l + l + m for l in range(abs(s), L) for m in range(-l, l + 1)]
    sol, *_ = np.linalg.lstsq(Y[:, keep], np.asarray(fmap).ravel(), rcond=None)
    out = np.zeros(L * L, dtype=np.complex128)
    out[keep] = sol
    return out
