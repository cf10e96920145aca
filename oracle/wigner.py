"""Wigner d-functions at beta = pi/2 by Risbo's recursion (oracle; test use only).

The paper evaluates Delta^l_{m'm} := d^l_{m'm}(pi/2) with the recursion of
Risbo (1996) (Section 2.2, the paragraph after Eq. (wignerd_b)) but does not
print it.  Reading used here: Risbo's recursion is the SU(2) construction in
which the spin-n/2 representation is built from spin-(n-1)/2 and spin-1/2.
With p = sin(beta/2), q = cos(beta/2) and D^n an (n+1) x (n+1) matrix indexed
by c, a in [0, n] (c = n/2 + m', a = n/2 + m), one half step is

    D^{n+1}_{c,a} = ( q sqrt(c a)             D^n_{c-1,a-1}
                    + p sqrt((n+1-c) a)       D^n_{c,a-1}
                    - p sqrt(c (n+1-a))       D^n_{c-1,a}
                    + q sqrt((n+1-c)(n+1-a))  D^n_{c,a} ) / (n+1),

out-of-range entries being zero and D^0 = [1].  Integer spin l is reached at
n = 2l, so Delta^l = D^{2l} and each l costs two half steps.  Convention: the
standard one used by Eq. (wignerd_b) (e.g. d^1_{10}(beta) = -sin(beta)/sqrt(2)).

Values below 1e-300 are flushed to zero after each half step (their
contribution to any sum is below 1e-290 and x86 subnormal arithmetic is slow).
"""

from __future__ import annotations

import ctypes
import math
import os
from typing import Iterator, Optional, Tuple

import numpy as np

_FLUSH = 1e-300
_LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "_risbo.so")
_lib: Optional[ctypes.CDLL] = None


def _c_lib() -> Optional[ctypes.CDLL]:
    """The compiled C half step (oracle/risbo.c), or None if it is not built."""
    global _lib
    if _lib is None and os.path.exists(_LIB_PATH):
        lib = ctypes.CDLL(_LIB_PATH)
        dp = ctypes.POINTER(ctypes.c_double)
        lib.oracle_risbo_half_step.argtypes = [dp, ctypes.c_int, dp, ctypes.c_double,
                                               ctypes.c_double, dp]
        lib.oracle_risbo_half_step.restype = None
        _lib = lib
    return _lib


class DeltaRisbo:
    """Stateful l-outer generator of Delta^l planes for l = 0, 1, 2, ...

    ``plane`` is the current Delta^l as a (2l+1) x (2l+1) array with
    ``plane[l + m', l + m] = Delta^l_{m'm}``.
    """

    def __init__(self, beta: float = math.pi / 2, use_c: bool = True):
        self.p = math.sin(beta / 2.0)
        self.q = math.cos(beta / 2.0)
        if beta == math.pi / 2:  # exact value, avoids sin/cos rounding
            self.p = self.q = math.sqrt(0.5)
        self.n = 0
        self.D = np.ones((1, 1))
        self._lib = _c_lib() if use_c else None

    @property
    def l(self) -> int:
        return self.n // 2

    @property
    def plane(self) -> np.ndarray:
        return self.D

    def _half_step(self) -> None:
        if self._lib is not None:
            self._half_step_c()
            return
        n, D, p, q = self.n, self.D, self.p, self.q
        # sqrt(c a) = sqrt(c) sqrt(a): outer products of sqrt(0..n+1)
        r = np.sqrt(np.arange(n + 2, dtype=np.float64))
        rc = r[1:][:, None]          # sqrt(c),       c = 1 .. n+1
        ra = r[1:][None, :]          # sqrt(a),       a = 1 .. n+1
        rcm = r[::-1][:-1][:, None]  # sqrt(n+1-c),   c = 0 .. n
        ram = r[::-1][:-1][None, :]  # sqrt(n+1-a),   a = 0 .. n
        out = np.zeros((n + 2, n + 2))
        out[1:, 1:] += (q * rc) * ra * D
        out[:-1, 1:] += (p * rcm) * ra * D
        out[1:, :-1] -= (p * rc) * ram * D
        out[:-1, :-1] += (q * rcm) * ram * D
        out *= 1.0 / (n + 1)
        out[np.abs(out) < _FLUSH] = 0.0
        self.D = out
        self.n = n + 1

    def _half_step_c(self) -> None:
        n = self.n
        D = np.ascontiguousarray(self.D)
        out = np.empty((n + 2, n + 2))
        sq = np.sqrt(np.arange(n + 2, dtype=np.float64))
        dp = ctypes.POINTER(ctypes.c_double)
        self._lib.oracle_risbo_half_step(D.ctypes.data_as(dp), n, out.ctypes.data_as(dp),
                                         self.p, self.q, sq.ctypes.data_as(dp))
        self.D = out
        self.n = n + 1

    def advance(self) -> np.ndarray:
        """Move from Delta^l to Delta^{l+1} (two half steps) and return it."""
        self._half_step()
        self._half_step()
        return self.D


def delta_planes(L: int, beta: float = math.pi / 2) -> Iterator[Tuple[int, np.ndarray]]:
    """Yield (l, Delta^l) for l = 0 .. L-1 (the array is reused: copy to keep)."""
    gen = DeltaRisbo(beta)
    yield 0, gen.plane
    for l in range(1, L):
        yield l, gen.advance()


def delta_plane(l: int, beta: float = math.pi / 2) -> np.ndarray:
    """A copy of the single plane Delta^l, ``[l + m', l + m]``."""
    for ll, D in delta_planes(l + 1, beta):
        if ll == l:
            return D.copy()
    raise AssertionError
