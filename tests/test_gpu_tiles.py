"""Contraction column tiles (sht_tile_set / sht_tune): every tile gives the
transform (against the oracle), the tiles agree bitwise (each output column
is accumulated in the same order whatever its column block), and the
autotuner's pick keeps the results."""

import numpy as np
import pytest
import torch

import oracle
import sht_synth

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-10, "fp32": 1e-5, "bf16x3": 5e-5}
# the 128-column tile is FP32 only
TILES = {"fp64": (16, 32, 64), "fp32": (16, 32, 64, 128), "bf16x3": (16, 32, 64)}


def _sht():
    import paper_0807_4494_amd as sht
    return sht


def rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(a), 1e-300))


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3"])
# L % 4 == 0 takes the 128-column tile's LDS-direct X loads, other L its
# element-wise loads; 4 B = 68 and 132 columns fill both halves of a block.
# Spin 0 runs the parity kernel (complete 16-blocks in parity order, an
# incomplete last block at L = 143; a pinned 128 tile falls back to 64).
@pytest.mark.parametrize("L,s,B", [(48, 0, 2), (64, 1, 6), (100, -2, 7), (70, 2, 17), (132, 3, 33),
                                   (143, 0, 17)])
def test_every_tile_gives_the_transform(L, s, B, prec):
    sht = _sht()
    print(f"[tiles] L={L} s={s} B={B} {prec}", flush=True)
    dev = torch.device("cuda", 0)
    flm = np.stack([sht_synth.gaussian_flm(L, s, 8300 + 17 * L + b) for b in range(B)])
    ref = oracle.inverse_batch(flm, L, s)
    x = torch.from_numpy(flm).to(dev, sht.io_dtype(prec))
    outs = []
    try:
        for tile in TILES[prec]:
            sht.tile_set(L, 4 * B, prec, tile)
            m = sht.inverse(x, L, s, prec)
            f = sht.forward(torch.from_numpy(ref).to(dev, sht.io_dtype(prec)), L, s, prec)
            torch.cuda.synchronize()
            assert rel(ref, m.cpu().numpy()) < TOL[prec], tile
            assert rel(flm, f.cpu().numpy()) < TOL[prec], tile
            outs.append((m, f))
    finally:
        sht.tile_set(L, 4 * B, prec, 0)
    for m, f in outs[1:]:
        assert torch.equal(m, outs[0][0]) and torch.equal(f, outs[0][1])


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_real_path_tiles(prec):
    sht = _sht()
    L, B = 64, 10
    dev = torch.device("cuda", 0)
    rng = np.random.default_rng(5)
    raw = rng.standard_normal((B, L, 2 * L - 1))
    ref = oracle.forward_batch(raw.astype(np.complex128), L, 0)
    got = []
    try:
        for tile in TILES[prec]:
            sht.tile_set(L, 2 * B, prec, tile)
            g = sht.forward_real(torch.from_numpy(raw).to(dev, sht.real_dtype(prec)), L, prec)
            torch.cuda.synchronize()
            assert rel(ref, g.cpu().numpy()) < TOL[prec], tile
            got.append(g)
    finally:
        sht.tile_set(L, 2 * B, prec, 0)
    assert all(torch.equal(g, got[0]) for g in got[1:])


@pytest.mark.parametrize("prec,L,s,B", [("fp32", 128, 2, 6), ("fp32", 96, 0, 16), ("fp64", 64, -1, 5)])
def test_autotuner_pick_keeps_the_results(prec, L, s, B):
    sht = _sht()
    dev = torch.device("cuda", 0)
    try:
        tile = sht.tune(L, s, B, prec)
        print(f"[tune] L={L} s={s} B={B} {prec}: tile {tile}", flush=True)
        assert tile in TILES[prec]
        flm = np.stack([sht_synth.gaussian_flm(L, s, 8700 + b) for b in range(B)])
        ref = oracle.inverse_batch(flm, L, s)
        m = sht.inverse(torch.from_numpy(flm).to(dev, sht.io_dtype(prec)), L, s, prec)
        f = sht.forward(m, L, s, prec)
        assert rel(ref, m.cpu().numpy()) < TOL[prec]
        assert rel(flm, f.cpu().numpy()) < TOL[prec]
    finally:
        sht.tile_set(L, 4 * B, prec, 0)
