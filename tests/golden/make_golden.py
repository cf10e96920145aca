"""Write the sampled full-size expected values used by tests/test_gpu_fullsize.py.

Calls only the CPU oracle (``oracle``) and the seeded input generators
(``sht_synth``); nothing here touches the GPU library.  Run from the
repository root:

    python tests/golden/make_golden.py L1024_s0pm2_b16
    python tests/golden/make_golden.py L2048_s0_b4

With ``--round-trip`` it adds to an existing file, for map 0 of each spin,
the oracle's round trip: the oracle's forward of the oracle's inverse of the
input coefficients, sampled at the coefficients of the orders ``fwd_orders``
(``rt_s<spin>``), and the relative l2 error of the whole round trip over all
L^2 coefficients (``rt_rel_s<spin>``).  A test compares the samples with the
input regenerated from its seed.

For each spin of the workload it stores
  * inverse: the oracle's map of batch members ``INV_MAPS`` at ``NPIX``
    seeded random pixels (t, p);
  * forward: the oracle's coefficients, for every degree, of the orders
    ``fwd_orders`` of an unstructured random map (``fwd_map_seed`` + b), batch
    members ``FWD_MAPS`` -- the forward is a fixed linear operator on any
    map, so this pins it away from band-limited inputs too.
"""

from __future__ import annotations

import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
import sht_synth  # noqa: E402

NPIX = 256
FWD_MAP_SEED = sht_synth.SEED_BASE + 7000


def fwd_orders(L: int) -> list[int]:
    return sorted({0, 1, 3, -(L // 2), L // 2 + 1, L - 1, -(L - 1)})


def members(batch: int) -> list[int]:
    return sorted({0, batch - 1})


def lm_indices(L: int, ms: list[int]) -> np.ndarray:
    return np.asarray([l * l + l + m for m in ms for l in range(abs(m), L)], dtype=np.int64)


def make(name: str) -> str:
    wl = {w.name: w for w in sht_synth.WORKLOADS}[name]
    L, B = wl.L, wl.batch
    rng = np.random.Generator(np.random.PCG64(sht_synth.SEED_BASE + 9000 + wl.index))
    pix_t = rng.integers(0, L, NPIX)
    pix_p = rng.integers(0, 2 * L - 1, NPIX)
    ms = fwd_orders(L)
    idx = lm_indices(L, ms)
    out = {"L": np.int64(L), "batch": np.int64(B), "pix_t": pix_t, "pix_p": pix_p,
           "fwd_orders": np.asarray(ms, dtype=np.int64), "fwd_index": idx,
           "members": np.asarray(members(B), dtype=np.int64),
           "fwd_map_seed": np.int64(FWD_MAP_SEED)}
    for s in wl.spins:
        flm = wl.flm(s)
        inv = []
        fwd = []
        for b in members(B):
            t0 = time.time()
            fmap = oracle.inverse(flm[b], L, s)
            inv.append(fmap[pix_t, pix_p])
            rmap = sht_synth.random_complex_map(L, FWD_MAP_SEED + b)
            g = oracle.forward_rows(rmap, L, s, ms)
            fwd.append(g[idx])
            print(f"{name} s={s} b={b}: {time.time() - t0:.1f} s", flush=True)
        out[f"inv_s{s}"] = np.stack(inv)
        out[f"fwd_s{s}"] = np.stack(fwd)
    out.update(round_trip(wl, idx))
    path = os.path.join(HERE, f"{name}.npz")
    np.savez_compressed(path, **out)
    return path


def round_trip(wl, idx) -> dict:
    """The oracle's inverse then forward of map 0 of each spin: sampled
    coefficients and the whole round trip's relative l2 error."""
    out = {}
    for s in wl.spins:
        f = wl.flm(s)[0]
        t0 = time.time()
        back = oracle.forward(oracle.inverse(f, wl.L, s), wl.L, s)
        out[f"rt_s{s}"] = back[idx]
        out[f"rt_rel_s{s}"] = np.float64(oracle.rel_l2(f, back))
        print(f"{wl.name} s={s} round trip: rel_l2 {out[f'rt_rel_s{s}']:.3e} ({time.time() - t0:.1f} s)",
              flush=True)
    return out


def add_round_trip(name: str) -> str:
    wl = {w.name: w for w in sht_synth.WORKLOADS}[name]
    path = os.path.join(HERE, f"{name}.npz")
    with np.load(path) as d:
        out = {k: d[k] for k in d.files}
    out.update(round_trip(wl, out["fwd_index"]))
    np.savez_compressed(path, **out)
    return path


if __name__ == "__main__":
    args = sys.argv[1:]
    if args and args[0] == "--round-trip":
        for n in args[1:]:
            print(add_round_trip(n))
    else:
        for n in args:
            print(make(n))
