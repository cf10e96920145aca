"""Several spins at one band-limit in one call (sht_inverse_multi /
sht_forward_multi): each map's result equals the single-spin call at its
spin and the oracle's transform within the precision's bar.

Bitwise, except for a segment of spin -s that directly follows one of spin
s != 0: it shares that segment's contraction factors through
d^l_{m',s}(pi/2) = (-1)^{l+m'} d^l_{m',-s}(pi/2) (Eq. (wignerd_sym6)), whose
two sides the plan tabulates separately, so it agrees with its own
single-spin call to rounding (relative l2 at most 1e-13 in FP64, 1e-6 in
FP32).  Every other column is accumulated in the same order whatever its
column block or tile."""

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle
import sht_synth

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-10, "fp32": 1e-5, "bf16x3": 2e-5}
ROUNDING = {"fp64": 1e-13, "fp32": 1e-6, "bf16x3": 1e-6}


def _sht():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_0807_4494_amd as sht
    return sht


SEGMENTS = [
    (65, [0, 2, -2, 1], [3, 2, 1, 4]),
    (33, [0, 1, -1, 2, -2, 3, -3, 4], [1, 1, 2, 1, 1, 1, 1, 1]),   # the most segments, tiny batches
    (128, [2, -2], [16, 16]),                                        # two full 64-column blocks
    (200, [-1], [5]),                                                 # one segment = the plain call
    # a pair of 72 columns (FP32: the 128-column tile; L odd, element-wise X loads)
    (257, [2, -2], [9, 9]),
    # L % 4 == 0: the 128-column tile's LDS-direct X loads; unpaired spin 0 after the pair
    (260, [-3, 3, 0], [12, 5, 4]),
    # pairing rule: two (1, -1) pairs in a row; s, s, -s pairs the second s;
    # two spin-0 segments (the parity kernel over both, no pairing)
    (64, [1, -1, 1, -1], [2, 3, 1, 2]),
    (48, [2, 2, -2], [1, 2, 3]),
    (80, [0, 1, 0], [2, 1, 3]),
]


def _flipped(spins):
    """Segments that share the previous segment's contraction (spin -s right
    after a spin s != 0 that is not itself flipped)."""
    out = [False] * len(spins)
    k = 0
    while k + 1 < len(spins):
        if spins[k] != 0 and spins[k + 1] == -spins[k]:
            out[k + 1] = True
            k += 2
        else:
            k += 1
    return out


def _rel(a, b):
    return float(torch.linalg.vector_norm((a - b).to(torch.complex128)) /
                 torch.linalg.vector_norm(b.to(torch.complex128)))


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3"])
@pytest.mark.parametrize("L,spins,batches", SEGMENTS)
def test_multi_spin_call_equals_single_spin_calls(L, spins, batches, prec):
    sht = _sht()
    print(f"[multi] L={L} spins={spins} batches={batches} {prec}", flush=True)
    dev = torch.device("cuda", 0)
    dt = sht.io_dtype(prec)
    flm = np.concatenate([np.stack([sht_synth.gaussian_flm(L, s, 6600 + 37 * k + b) for b in range(n)])
                          for k, (s, n) in enumerate(zip(spins, batches))])
    x = torch.from_numpy(flm).to(dev, dt)
    maps = sht.inverse_multi(x, L, spins, batches, prec)
    back = sht.forward_multi(maps, L, spins, batches, prec)
    torch.cuda.synchronize()
    off = 0
    for s, n, flip in zip(spins, batches, _flipped(spins)):
        sl = slice(off, off + n)
        m1 = sht.inverse(x[sl], L, s, prec)
        f1 = sht.forward(maps[sl], L, s, prec)
        torch.cuda.synchronize()
        if flip:
            assert _rel(maps[sl], m1) <= ROUNDING[prec], (s, "inverse", _rel(maps[sl], m1))
            assert _rel(back[sl], f1) <= ROUNDING[prec], (s, "forward", _rel(back[sl], f1))
        else:
            assert torch.equal(maps[sl], m1), (s, "inverse")
            assert torch.equal(back[sl], f1), (s, "forward")
        ref = oracle.inverse_batch(flm[sl], L, s)
        assert oracle.rel_l2(ref, maps[sl].cpu().numpy()) < TOL[prec]
        assert oracle.rel_l2(flm[sl], back[sl].cpu().numpy()) < TOL[prec]
        off += n


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_every_stage_is_one_traced_step_per_call(prec):
    """A multi-spin call runs each of its eight stages once over all its
    maps (the layout and theta kernels look up each map's segment), however
    many segments it has; the trace counts one entry per stage and call."""
    sht = _sht()
    dev = torch.device("cuda", 0)
    L, spins, batches = 72, [0, 2, -2, 1, 3], [2, 1, 1, 2, 1]
    B = sum(batches)
    x = torch.from_numpy(np.stack([sht_synth.gaussian_flm(L, s, 600 + 17 * k + b)
                                   for k, s in enumerate(spins) for b in range(batches[k])]))
    x = x.to(dev, sht.io_dtype(prec))
    sht.inverse_multi(x, L, spins, batches, prec)   # plans built outside the traced calls
    torch.cuda.synchronize()
    sht.trace_enable(True)
    try:
        sht.trace_read()
        fmap = sht.inverse_multi(x, L, spins, batches, prec)
        back = sht.forward_multi(fmap, L, spins, batches, prec)
        torch.cuda.synchronize()
        counts = {name: n for name, (_, n) in sht.trace_read().items()}
    finally:
        sht.trace_enable(False)
    assert set(counts.values()) == {1}, counts
    err = float(torch.linalg.vector_norm(back - x) / torch.linalg.vector_norm(x))
    assert err <= TOL[prec], err
    assert B == back.shape[0]


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_paired_spins_at_L2048(prec):
    """The spin pair (2, -2) at the largest configured band-limit: the paired
    call (FP32: one 128-column tile for both spins, FFT rows of 8192 points)
    agrees with the single-spin calls to rounding, and its round trip returns
    the coefficients.  The rounding bar is the file's (set for L <= 260)
    scaled by sqrt(L / 256): the contraction sums L terms, whose rounding
    errors add like a random walk."""
    sht = _sht()
    dev = torch.device("cuda", 0)
    L, spins, batches = 2048, [2, -2], [4, 4]
    print(f"[multi] L={L} spins={spins} batches={batches} {prec}", flush=True)
    x = torch.from_numpy(np.stack([sht_synth.gaussian_flm(L, s, 700 + 11 * k + b, "inv_lp1_sq")
                                   for k, s in enumerate(spins) for b in range(batches[k])]))
    x = x.to(dev, sht.io_dtype(prec))
    maps = sht.inverse_multi(x, L, spins, batches, prec)
    back = sht.forward_multi(maps, L, spins, batches, prec)
    bar = ROUNDING[prec] * (L / 256) ** 0.5
    for k, s in enumerate(spins):
        sl = slice(4 * k, 4 * k + 4)
        m1 = sht.inverse(x[sl], L, s, prec)
        f1 = sht.forward(maps[sl], L, s, prec)
        assert _rel(maps[sl], m1) <= bar, (s, "inverse", _rel(maps[sl], m1))
        assert _rel(back[sl], f1) <= bar, (s, "forward", _rel(back[sl], f1))
    err = float(torch.linalg.vector_norm(back - x) / torch.linalg.vector_norm(x))
    assert err <= TOL[prec], err
