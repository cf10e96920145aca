"""Forward and inverse spin SHT, plain FP64 (oracle; test use only).

Conventions (readings of the paper, listed with reasons in the design notes):

* Band-limit: L counts the degrees, 0 <= l < L, and N = 2L - 1 samples per
  torus axis.  (The paper writes the band-limit as the largest degree, with
  N = 2 L_paper + 1; L here is L_paper + 1.)
* Sampling, Eq. (nodes_theta) / Eq. (nodes_phi): theta_t = pi (2t+1)/N,
  phi_p = pi (2p+1)/N.  The sphere keeps the rings t = 0 .. L-1, which
  includes theta_{L-1} = pi (Section 3.4.3: the torus half theta in [0, pi]).
* Maps are stored ``[t, p]`` (theta outer), coefficients ``[l*l + l + m]``.
* Spin harmonics, Eq. (ssh_wigner):
      sY_lm(theta, phi) = (-1)^s sqrt((2l+1)/4pi) d^l_{m,-s}(theta) e^{i m phi},
  and f_lm = 0 for l < |s|.

Inverse (Section 3.1 and 3.4.3):
  O-I1  F_{mm'} = (-1)^s i^{-(m+s)} sum_l sqrt((2l+1)/4pi)
                  Delta^l_{m'm} Delta^l_{m',-s} f_lm          Eq. (fourier_coeff)
  O-I2  f(theta_t, phi_p) = sum_{m,m'} F_{mm'} e^{i(m phi_p + m' theta_t)}
                                                               Eq. (sht_inv_fast)

Forward (exact quadrature on the extended torus; the paper's own forward is a
triangular solve that it shows to be unstable beyond small L, so the forward
is computed from Eq. (ssht_fwd) with the conjugate of Eq. (shf_exp)):
  O-F1  Q_m(t) = N^-1 sum_p f(theta_t, phi_p) e^{-i m phi_p},  t < L
  O-F2  extend in theta: Q~_m(t) = Q_m(t) for t < L and
        (-1)^{m+s} Q_m(2L-2-t) for L <= t < N -- the even extension for
        m+s even and the odd one for m+s odd (Section 3.2)
  O-F3  F_{mm''} = N^-1 sum_t Q~_m(t) e^{-i m'' theta_t}      Eq. (fourier_series),
        exact for the band-limited extension (Section 3.3)
  O-F4  G_{mm'} = int_0^pi sin(theta) dtheta int_0^2pi dphi f e^{-i(m phi + m' theta)}
              = 2pi sum_{m''} F_{mm''} w(m'' - m'),
        w(p) = int_0^pi sin(theta) e^{i p theta} dtheta
  O-F5  f_lm = (-1)^s i^{m+s} sqrt((2l+1)/4pi)
               sum_{m'=-l}^{l} Delta^l_{m'm} Delta^l_{m',-s} G_{mm'}
        (Eq. (ssht_fwd) with the complex conjugate of Eq. (shf_exp)).

The 1-D and 2-D DFTs are numpy FFTs; frequency m maps to bin (m mod N), with
the half-sample phase e^{+-i pi m/N} of Eq. (dft_phase) written out.
"""

from __future__ import annotations

import math
from typing import Iterable, Optional, Sequence

import numpy as np

from .wigner import delta_planes


def _nn(L: int) -> int:
    return 2 * L - 1


def theta_nodes(L: int, torus: bool = False) -> np.ndarray:
    """Eq. (nodes_theta): pi (2t+1)/N for t < L (sphere) or t < N (torus)."""
    N = _nn(L)
    t = np.arange(N if torus else L, dtype=np.float64)
    return math.pi * (2.0 * t + 1.0) / N


def phi_nodes(L: int) -> np.ndarray:
    """Eq. (nodes_phi): pi (2p+1)/N, p < N."""
    N = _nn(L)
    return math.pi * (2.0 * np.arange(N, dtype=np.float64) + 1.0) / N


def _ipow(k: int) -> complex:
    """i^k for any integer k, exact."""
    return (1.0 + 0j, 1j, -1.0 + 0j, -1j)[k % 4]


def _as_batch(x: np.ndarray, ndim: int) -> tuple[np.ndarray, bool]:
    x = np.asarray(x, dtype=np.complex128)
    if x.ndim == ndim:
        return x[None], True
    return x, False


# ---------------------------------------------------------------- inverse ----

def fourier_coefficients(flm: np.ndarray, L: int, s: int) -> np.ndarray:
    """O-I1, Eq. (fourier_coeff).

    ``flm``: [B, L*L] (or [L*L]).  Returns F: [B, N, N] indexed
    ``[b, (L-1) + m, (L-1) + m']``, m, m' in [-(L-1), L-1].  Terms with
    |m| > l or |m'| > l are zero (the paper's convention after
    Eq. (fourier_coeff)); degrees l < |s| do not contribute.
    """
    flm, single = _as_batch(flm, 1)
    B = flm.shape[0]
    N = _nn(L)
    F = np.zeros((B, N, N), dtype=np.complex128)
    for l, D in delta_planes(L):
        if l < abs(s):
            continue
        cl = math.sqrt((2 * l + 1) / (4.0 * math.pi))
        col = D[:, l - s]                    # Delta^l_{m', -s}, m' = -l..l
        A = D * col[:, None]                 # A[m', m] = Delta_{m'm} Delta_{m',-s}
        fl = flm[:, l * l: l * l + 2 * l + 1]  # f_lm, m = -l..l
        lo, hi = L - 1 - l, L + l
        F[:, lo:hi, lo:hi] += cl * (fl[:, :, None] * A.T[None, :, :])
    m = np.arange(-(L - 1), L)
    phase = np.array([(-1.0) ** s * _ipow(-(mm + s)) for mm in m])
    F *= phase[None, :, None]
    return F[0] if single else F


def torus_synthesis(F: np.ndarray, L: int) -> np.ndarray:
    """O-I2, Eq. (sht_inv_fast) on the sampling nodes, kept for t < L.

    ``F``: [B, N, N] as returned by :func:`fourier_coefficients`.
    Returns maps [B, L, N] (theta ring t, phi sample p).
    """
    F, single = _as_batch(F, 2)
    N = _nn(L)
    m = np.arange(-(L - 1), L)
    ph = np.exp(1j * math.pi * m / N)
    X = np.zeros_like(F)
    bins = np.mod(m, N)
    X[:, bins[:, None], bins[None, :]] = F * ph[None, :, None] * ph[None, None, :]
    # numpy's ifft2 divides by N^2; the sum in Eq. (sht_inv_fast) is unnormalised
    g = np.fft.ifft2(X, axes=(1, 2)) * (N * N)   # g[b, p, t]
    out = np.ascontiguousarray(np.transpose(g, (0, 2, 1))[:, :L, :])
    return out[0] if single else out


def inverse(flm: np.ndarray, L: int, s: int) -> np.ndarray:
    """Inverse spin SHT of one map: f_lm [L*L] -> samples [L, N]."""
    return torus_synthesis(fourier_coefficients(flm, L, s), L)


def inverse_batch(flm: np.ndarray, L: int, s: int) -> np.ndarray:
    """Inverse spin SHT of a batch: [B, L*L] -> [B, L, N]."""
    return torus_synthesis(fourier_coefficients(np.asarray(flm)[None] if np.ndim(flm) == 1
                                                else flm, L, s), L)


# ---------------------------------------------------------------- forward ----

def quadrature_weight(p: np.ndarray) -> np.ndarray:
    """w(p) = int_0^pi sin(theta) e^{i p theta} d theta for integer p.

    w(0) = 2; w(+-1) = +- i pi/2; w(p) = 2/(1-p^2) for even p; 0 for odd |p| > 1.
    """
    p = np.asarray(p)
    out = np.zeros(p.shape, dtype=np.complex128)
    even = (p % 2) == 0
    out[even] = 2.0 / (1.0 - p[even].astype(np.float64) ** 2)
    out[p == 1] = 0.5j * math.pi
    out[p == -1] = -0.5j * math.pi
    return out


def phi_analysis(fmap: np.ndarray, L: int, ms: Optional[Sequence[int]] = None) -> np.ndarray:
    """O-F1: Q[b, (L-1)+m, t] = N^-1 sum_p f[b, t, p] e^{-i m phi_p}.

    With ``ms`` given, only those m rows are returned (direct sums), shape [B, len(ms), L].
    """
    fmap, single = _as_batch(fmap, 2)
    N = _nn(L)
    if ms is None:
        m = np.arange(-(L - 1), L)
        Y = np.fft.fft(fmap, axis=2)                     # [B, t, k]
        Q = Y[:, :, np.mod(m, N)] * np.exp(-1j * math.pi * m / N)[None, None, :] / N
        Q = np.transpose(Q, (0, 2, 1))
    else:
        m = np.asarray(ms)
        E = np.exp(-1j * np.outer(m, phi_nodes(L)))     # [len(ms), p]
        Q = np.einsum("mp,btp->bmt", E, fmap) / N
    return Q[0] if single else Q


def theta_extend(Q: np.ndarray, L: int, s: int, ms: Sequence[int]) -> np.ndarray:
    """O-F2: per-m parity extension of Q[b, i, t] (row i has order ms[i]) to N rings."""
    N = _nn(L)
    B, R, _ = Q.shape
    Qt = np.zeros((B, R, N), dtype=np.complex128)
    Qt[:, :, :L] = Q
    sign = np.array([(-1.0) ** (mm + s) for mm in ms])
    t = np.arange(L, N)
    Qt[:, :, L:] = sign[None, :, None] * Q[:, :, 2 * L - 2 - t]
    return Qt


def theta_analysis(Qt: np.ndarray, L: int) -> np.ndarray:
    """O-F3: F[b, i, (L-1)+m''] = N^-1 sum_t Q~[b, i, t] e^{-i m'' theta_t}."""
    N = _nn(L)
    m2 = np.arange(-(L - 1), L)
    Y = np.fft.fft(Qt, axis=2)
    return Y[:, :, np.mod(m2, N)] * np.exp(-1j * math.pi * m2 / N)[None, None, :] / N


def weighted_coefficients(F: np.ndarray, L: int) -> np.ndarray:
    """O-F4: G[b, i, (L-1)+m'] = 2 pi sum_{m''} F[b, i, (L-1)+m''] w(m'' - m')."""
    m = np.arange(-(L - 1), L)
    W = quadrature_weight(m[:, None] - m[None, :])     # W[m'', m'] = w(m'' - m')
    return 2.0 * math.pi * (F @ W)


def harmonic_projection(G: np.ndarray, L: int, s: int, ms: Sequence[int]) -> np.ndarray:
    """O-F5 for the rows ``ms``: returns f[b, l*l + l + m] (zero where not computed)."""
    B = G.shape[0]
    ms = list(ms)
    row_of = {mm: i for i, mm in enumerate(ms)}
    flm = np.zeros((B, L * L), dtype=np.complex128)
    for l, D in delta_planes(L):
        if l < abs(s):
            continue
        cl = math.sqrt((2 * l + 1) / (4.0 * math.pi))
        col = D[:, l - s]
        A = D * col[:, None]                 # [m', m] over -l..l
        lo, hi = L - 1 - l, L + l
        for mm in ms:
            if abs(mm) > l:
                continue
            i = row_of[mm]
            acc = G[:, i, lo:hi] @ A[:, l + mm]  # sum over m' = -l..l
            flm[:, l * l + l + mm] = (-1.0) ** s * _ipow(mm + s) * cl * acc
    return flm


def forward_rows(fmap: np.ndarray, L: int, s: int, ms: Optional[Iterable[int]] = None) -> np.ndarray:
    """Forward transform restricted to orders ``ms`` (all m when None).

    ``fmap``: [B, L, N] (or [L, N]).  Returns [B, L*L] (or [L*L]); entries of
    orders outside ``ms`` are left zero.
    """
    fmap, single = _as_batch(fmap, 2)
    if ms is None:
        ms = list(range(-(L - 1), L))
        Q = phi_analysis(fmap, L)
    else:
        ms = list(ms)
        Q = phi_analysis(fmap, L, ms)
    Qt = theta_extend(Q, L, s, ms)
    F = theta_analysis(Qt, L)
    G = weighted_coefficients(F, L)
    out = harmonic_projection(G, L, s, ms)
    return out[0] if single else out


def forward(fmap: np.ndarray, L: int, s: int) -> np.ndarray:
    """Forward spin SHT of one map: samples [L, N] -> f_lm [L*L]."""
    return forward_rows(fmap, L, s)


def forward_batch(fmap: np.ndarray, L: int, s: int) -> np.ndarray:
    """Forward spin SHT of a batch: [B, L, N] -> [B, L*L]."""
    return forward_rows(np.asarray(fmap), L, s)
