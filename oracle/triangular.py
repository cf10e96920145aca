"""The paper's own forward transform: per-order triangular systems (oracle; test use only).

Section 3.4.2 rewrites Eq. (fourier_coeff), for one order m0 and one spin s,
as a matrix equation between the torus coefficients F_{m0 m'} and the
harmonic coefficients f_{l m0}, and keeps only its lower half m' >= 0
(Eq. (matrix_fwd)):

    F_{m0 m'} = sum_{l >= m'} D[m', l] f_{l m0},
    D[m', l]  = i^{-(m0+s)} sqrt((2l+1)/4pi) Delta^l_{m' m0} Delta^l_{m',-s}

(upper triangular in (m', l)).  The torus coefficients come from the
extension of the sampled map chosen by the parity of m0+s (Section 3.2) and
the DFT of Eq. (fourier_series) -- steps O-F1..O-F3 of :mod:`oracle.transform`.
The (-1)^s of Eq. (ssh_wigner) is part of the harmonic convention used by the
rest of this package (F of :func:`oracle.transform.fourier_coefficients`
carries it), so here D carries it too.

Readings where the paper is silent:

* Coefficients with l < l0 = max(|m0|, |s|) do not exist, and the columns of D
  for those l vanish, so the full (L x L) system is singular for m0 != 0.
  The paper's triangular solve is taken on the square block of rows and
  columns l0..L-1 (back substitution from l = L-1 downwards).
* For s = 0 the paper splits each system into the rows and columns of even
  and of odd l + m' (D vanishes elsewhere, Eq. (wignerd_sym6)); that split is
  :func:`solve_split` and is pinned equal to the plain back substitution.
* :func:`forward_lstsq` solves the overdetermined system of all rows
  m' = 0..L-1 by least squares instead -- not the paper's method; it is
  kept as the stable comparison.
"""

from __future__ import annotations

import math
from typing import List, Tuple

import numpy as np

from .transform import phi_analysis, theta_analysis, theta_extend
from .wigner import delta_planes


def _ipow(k: int) -> complex:
    return (1, 1j, -1, -1j)[k % 4]


def system_matrices(L: int, s: int, orders) -> dict:
    """D_{m0} for each m0 in ``orders``: dict m0 -> [L, L] complex array
    D[m', l] (rows m' = 0..L-1, columns l = 0..L-1), zero below the diagonal
    and in the columns l < max(|m0|, |s|)."""
    orders = list(orders)
    out = {m0: np.zeros((L, L), dtype=np.complex128) for m0 in orders}
    for l, D in delta_planes(L):
        if l < abs(s):
            continue
        cl = math.sqrt((2 * l + 1) / (4.0 * math.pi))
        for m0 in orders:
            if abs(m0) > l:
                continue
            ph = (-1.0) ** s * _ipow(-(m0 + s))
            mp = np.arange(0, l + 1)
            out[m0][mp, l] = ph * cl * D[l + mp, l + m0] * D[l + mp, l - s]
    return out


def back_substitute(D: np.ndarray, F: np.ndarray, l0: int) -> np.ndarray:
    """Solve D[l0:, l0:] x = F[l0:] (upper triangular) from the last row up.
    Returns x over l = 0..L-1 (zero below l0)."""
    L = D.shape[0]
    x = np.zeros(L, dtype=np.complex128)
    for l in range(L - 1, l0 - 1, -1):
        acc = F[l] - np.dot(D[l, l + 1:], x[l + 1:])
        x[l] = acc / D[l, l]
    return x


def solve_split(D: np.ndarray, F: np.ndarray, l0: int) -> np.ndarray:
    """s = 0 form: the rows and columns with even l+m' and with odd l+m' form
    two independent triangular systems (Section 3.4.2); solve each."""
    L = D.shape[0]
    x = np.zeros(L, dtype=np.complex128)
    idx = np.arange(l0, L)
    for par in (0, 1):
        # unknown l pairs with row m' = l; keep the rows/columns of one parity of l - l0
        sel = idx[(idx - l0) % 2 == par]
        if sel.size == 0:
            continue
        sub = D[np.ix_(sel, sel)]
        xs = np.zeros(sel.size, dtype=np.complex128)
        for i in range(sel.size - 1, -1, -1):
            xs[i] = (F[sel[i]] - np.dot(sub[i, i + 1:], xs[i + 1:])) / sub[i, i]
        x[sel] = xs
    return x


def torus_rows(fmap: np.ndarray, L: int, s: int) -> np.ndarray:
    """F_{m m'} for m in [-(L-1), L-1] (row (L-1)+m) and m' in [0, L-1],
    from the extension of each order chosen by the parity of m+s (O-F1..O-F3)."""
    ms = list(range(-(L - 1), L))
    Q = phi_analysis(fmap[None], L)
    F = theta_analysis(theta_extend(Q, L, s, ms), L)[0]   # [(L-1)+m, (L-1)+m']
    return F[:, L - 1:]


def forward_triangular(fmap: np.ndarray, L: int, s: int, split_spin0: bool = True) -> np.ndarray:
    """The paper's forward: per order, back substitution on the square block.
    ``fmap`` [L, N]; returns f[l*l + l + m]."""
    F = torus_rows(fmap, L, s)
    mats = system_matrices(L, s, range(-(L - 1), L))
    flm = np.zeros(L * L, dtype=np.complex128)
    for m0 in range(-(L - 1), L):
        l0 = max(abs(m0), abs(s))
        D = mats[m0]
        rhs = F[(L - 1) + m0]
        x = solve_split(D, rhs, l0) if (s == 0 and split_spin0) else back_substitute(D, rhs, l0)
        ls = np.arange(l0, L)
        flm[ls * ls + ls + m0] = x[l0:]
    return flm


def forward_lstsq(fmap: np.ndarray, L: int, s: int) -> np.ndarray:
    """All rows m' = 0..L-1 of each order's system, least squares (stable variant)."""
    F = torus_rows(fmap, L, s)
    mats = system_matrices(L, s, range(-(L - 1), L))
    flm = np.zeros(L * L, dtype=np.complex128)
    for m0 in range(-(L - 1), L):
        l0 = max(abs(m0), abs(s))
        A = mats[m0][:, l0:]
        x, *_ = np.linalg.lstsq(A, F[(L - 1) + m0], rcond=None)
        ls = np.arange(l0, L)
        flm[ls * ls + ls + m0] = x
    return flm


def condition_numbers(L: int, s: int, m0: int) -> Tuple[float, float]:
    """(cond_2 of the paper's square block, cond_2 of the all-rows system)."""
    D = system_matrices(L, s, [m0])[m0]
    l0 = max(abs(m0), abs(s))
    sq = D[l0:, l0:]
    full = D[:, l0:]
    sv_sq = np.linalg.svd(sq, compute_uv=False)
    sv_full = np.linalg.svd(full, compute_uv=False)
    return float(sv_sq[0] / sv_sq[-1]), float(sv_full[0] / sv_full[-1])


def stability_errors(Ls, n_maps: int = 5, seed: int = 0x5EED0000 + 8000) -> List[dict]:
    """The experiment of Section 4.2: real spin-0 test functions defined by
    U[-1, 1] coefficients (made real by f_{l,-m} = (-1)^m conj(f_lm)), inverse
    then the triangular forward; the five error metrics averaged over maps."""
    from .metrics import error_metrics
    from .transform import inverse
    out = []
    rng = np.random.Generator(np.random.PCG64(seed))
    for L in Ls:
        acc = None
        for _ in range(n_maps):
            f = np.zeros(L * L, dtype=np.complex128)
            for l in range(L):
                f[l * l + l] = rng.uniform(-1, 1)
                for m in range(1, l + 1):
                    v = rng.uniform(-1, 1) + 1j * rng.uniform(-1, 1)
                    f[l * l + l + m] = v
                    f[l * l + l - m] = (-1) ** m * np.conj(v)
            g = forward_triangular(inverse(f, L, 0), L, 0)
            e = error_metrics(f, g)
            acc = e if acc is None else {k: acc[k] + e[k] for k in e}
        out.append({"L": L, **{k: v / n_maps for k, v in acc.items()}})
    return out
