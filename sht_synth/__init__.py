"""Seeded synthetic inputs shared by the CPU oracle, the tests and the benchmark.

This module draws random numbers and lays them out; it holds none of the
transform's arithmetic.  Both the oracle and the GPU path receive the very same
host arrays from here.

Layout conventions (shared with the C ABI):

* harmonic coefficients ``flm[b, l*l + l + m]`` for ``0 <= l < L``,
  ``-l <= m <= l`` (complex128);
* coefficients with ``l < |s|`` are zero: spin-``s`` harmonics exist only for
  ``l >= |s|`` (Section 2.3 of the paper).

Workloads follow the paper's test functions (Section 4: random band-limited
functions defined through their harmonic coefficients) with the Gaussian
power spectra of the benchmark configurations.
"""

from __future__ import annotations

import dataclasses
import math
from typing import Callable, List, Sequence

import numpy as np

SEED_BASE = 0x5EED0000


def flm_size(L: int) -> int:
    return L * L


def lm_index(l: int, m: int) -> int:
    return l * l + l + m


def seed_for(config_index: int, map_index: int) -> int:
    """Per-map seed: ``0x5EED0000 + 1000*config_index + map_index``."""
    return SEED_BASE + 1000 * config_index + map_index


def spectrum(name: str) -> Callable[[np.ndarray], np.ndarray]:
    """Power spectra C_l used by the workloads (vectorised over l)."""
    if name == "flat":
        return lambda l: np.ones_like(l, dtype=np.float64)
    if name == "inv_lp1_sq":  # 1/(l+1)^2
        return lambda l: 1.0 / (l.astype(np.float64) + 1.0) ** 2
    if name == "inv_l_lp1":  # 1/(l(l+1)), zero at l = 0
        def f(l):
            lf = l.astype(np.float64)
            out = np.zeros_like(lf)
            nz = lf > 0
            out[nz] = 1.0 / (lf[nz] * (lf[nz] + 1.0))
            return out
        return f
    raise ValueError(f"unknown spectrum {name!r}")


def gaussian_flm(L: int, spin: int, seed: int, spec: str = "flat",
                 lmin: int = 0) -> np.ndarray:
    """One map's coefficients: f_lm = sqrt(C_l) (x + i y)/sqrt(2), x, y ~ N(0,1).

    Drawn with numpy's PCG64 from ``seed``; entries with l < max(|spin|, lmin)
    are zero.  Returns complex128 of length L*L.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    x = rng.standard_normal(L * L)
    y = rng.standard_normal(L * L)
    l_of = np.repeat(np.arange(L), 2 * np.arange(L) + 1)
    cl = spectrum(spec)(l_of)
    f = np.sqrt(cl) * (x + 1j * y) / math.sqrt(2.0)
    f[l_of < max(abs(spin), lmin)] = 0.0
    return f.astype(np.complex128)


def uniform_flm(L: int, spin: int, seed: int) -> np.ndarray:
    """The paper's timing/stability test functions (Section 4): real and
    imaginary parts independent U[-1, 1]; zero for l < |spin|."""
    rng = np.random.Generator(np.random.PCG64(seed))
    f = rng.uniform(-1, 1, L * L) + 1j * rng.uniform(-1, 1, L * L)
    l_of = np.repeat(np.arange(L), 2 * np.arange(L) + 1)
    f[l_of < abs(spin)] = 0.0
    return f.astype(np.complex128)


def batch_flm(L: int, spin: int, batch: int, config_index: int,
              spec: str = "flat", lmin: int = 0, map_offset: int = 0) -> np.ndarray:
    """``batch`` maps stacked as ``[batch, L*L]``; map b uses seed_for(config, map_offset + b)."""
    return np.stack([gaussian_flm(L, spin, seed_for(config_index, map_offset + b), spec, lmin)
                     for b in range(batch)])


def random_complex_map(L: int, seed: int) -> np.ndarray:
    """Unstructured (not band-limited) complex samples, shape [L, 2L-1]."""
    rng = np.random.Generator(np.random.PCG64(seed))
    N = 2 * L - 1
    return (rng.standard_normal((L, N)) + 1j * rng.standard_normal((L, N))).astype(np.complex128)


@dataclasses.dataclass(frozen=True)
class Workload:
    """One benchmark / parity configuration."""
    index: int
    name: str
    L: int
    spins: Sequence[int]
    batch: int
    spec: str
    lmin: int = 0

    def flm(self, spin: int) -> np.ndarray:
        # map_index folds in the spin so each spin class draws distinct maps
        spin_slot = list(self.spins).index(spin)
        return batch_flm(self.L, spin, self.batch, self.index, self.spec, self.lmin,
                         map_offset=100 * spin_slot)


# The five workloads: FP64 s=0 L=32 one map; FP64 s=2 L=256 one map;
# s in {0,+2,-2} L=1024 16 maps per spin (the throughput configuration);
# s=0 L=2048 4 maps flat spectrum; and the mixed serving stream (see trace()).
WORKLOADS: List[Workload] = [
    Workload(0, "L32_s0_b1", 32, (0,), 1, "flat"),
    Workload(1, "L256_s2_b1", 256, (2,), 1, "inv_l_lp1", lmin=2),
    Workload(2, "L1024_s0pm2_b16", 1024, (0, 2, -2), 16, "inv_lp1_sq"),
    Workload(3, "L2048_s0_b4", 2048, (0,), 4, "flat"),
]


@dataclasses.dataclass(frozen=True)
class Request:
    rid: int
    arrival_s: float
    L: int
    spin: int
    batch: int
    seed: int


def trace(n_requests: int = 2000, rate_per_s: float = 1000.0, seed: int = SEED_BASE + 4000,
          L_lo: int = 64, L_hi: int = 2048, spins: Sequence[int] = (0, 1, -1, 2, -2),
          batch_lo: int = 1, batch_hi: int = 32) -> List[Request]:
    """Serving stream: Poisson arrivals at ``rate_per_s``; L log-uniform in
    [L_lo, L_hi] rounded to the nearest multiple of 32 and clamped; spin uniform
    over ``spins``; batch uniform in [batch_lo, batch_hi]."""
    rng = np.random.Generator(np.random.PCG64(seed))
    gaps = rng.exponential(1.0 / rate_per_s, n_requests)
    t = np.cumsum(gaps)
    Ls = np.exp(rng.uniform(math.log(L_lo), math.log(L_hi), n_requests))
    Ls = np.clip(np.rint(Ls / 32.0) * 32, L_lo, L_hi).astype(int)
    sp = rng.choice(np.asarray(spins), n_requests)
    bs = rng.integers(batch_lo, batch_hi + 1, n_requests)
    return [Request(i, float(t[i]), int(Ls[i]), int(sp[i]), int(bs[i]), SEED_BASE + 5000 + i)
            for i in range(n_requests)]


def request_flm(req: Request) -> np.ndarray:
    """Coefficients of a serving request: C_l = 1/(l+1)^2, [batch, L*L]."""
    return np.stack([gaussian_flm(req.L, req.spin, req.seed * 64 + b, "inv_lp1_sq")
                     for b in range(req.batch)])
