"""GPU parity over every output entry at L = 512 and at L = 1024 (and at an
odd L of the same 4096-point FFT range, L = 777).

The sampled full-size tests compare a few hundred pixels and a few orders;
here every entry of chosen maps is compared with the oracle, which takes about
2.5 s per map and direction at L = 512 and 20 s at L = 1024.

* L = 512: one multi-spin call over spins 0, 2, -2, -1, 1 (two pairs whose
  second member shares the first's contraction, with the flipped member
  positive in one pair and negative in the other), every map compared.
* L = 1024: the benchmark's launch configuration (spins 0, 2, -2 with 16 maps
  each in one multi-spin call per direction); one map per spin, at a
  different batch position for each spin, is compared over all its entries.

The forward is fed unstructured random maps: off the band-limited subspace it
is still one fixed linear operator, the quadrature of Section 3.

Bars (relative l2 over all complex entries of a map, Section 4.2's relative
rms): FP64 <= 1e-10, FP32 <= 1e-5, BF16x3 <= 2e-5.
"""

import functools

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle
import sht_synth

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-10, "fp32": 1e-5, "bf16x3": 2e-5}

L_MID, SPINS_MID, B_MID = 512, (0, 2, -2, -1, 1), 2
SEED_MID = sht_synth.SEED_BASE + 9600

BENCH = "L1024_s0pm2_b16"
MEMBER = {0: 0, 2: 7, -2: 15}        # the compared map of each spin's 16
SEED_FWD = sht_synth.SEED_BASE + 9700


def _dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda", 0)


def _sht():
    import paper_0807_4494_amd as sht
    return sht


def _rel(ref, got):
    return float(np.linalg.norm(got - ref) / np.linalg.norm(ref))


# ---- L = 512, every map of a five-segment multi-spin call ----

def _mid_seed(k, b):
    return SEED_MID + 16 * k + b


@functools.lru_cache(maxsize=1)
def _mid_flm():
    return np.stack([sht_synth.gaussian_flm(L_MID, s, _mid_seed(k, b))
                     for k, s in enumerate(SPINS_MID) for b in range(B_MID)])


@functools.lru_cache(maxsize=1)
def _mid_maps():
    return np.stack([sht_synth.random_complex_map(L_MID, _mid_seed(k, b) + 8)
                     for k in range(len(SPINS_MID)) for b in range(B_MID)])


@functools.lru_cache(maxsize=1)
def _mid_inverse_ref():
    flm = _mid_flm()
    return np.stack([oracle.inverse(flm[k * B_MID + b], L_MID, s)
                     for k, s in enumerate(SPINS_MID) for b in range(B_MID)])


@functools.lru_cache(maxsize=1)
def _mid_forward_ref():
    maps = _mid_maps()
    return np.stack([oracle.forward(maps[k * B_MID + b], L_MID, s)
                     for k, s in enumerate(SPINS_MID) for b in range(B_MID)])


@pytest.mark.parametrize("prec", ["fp32", "fp64", "bf16x3"])
def test_inverse_every_entry_L512_multi_spin(prec):
    sht, dev = _sht(), _dev()
    print(f"[full entries] inverse L={L_MID} spins={SPINS_MID} B={B_MID} {prec}", flush=True)
    ref = _mid_inverse_ref()
    x = torch.from_numpy(_mid_flm()).to(dev, sht.io_dtype(prec))
    got = sht.inverse_multi(x, L_MID, list(SPINS_MID), [B_MID] * len(SPINS_MID), prec)
    got = got.cpu().numpy().astype(np.complex128)
    assert got.shape == ref.shape
    for k, s in enumerate(SPINS_MID):
        for b in range(B_MID):
            i = k * B_MID + b
            err = _rel(ref[i], got[i])
            assert err <= TOL[prec], (s, b, prec, err)


@pytest.mark.parametrize("prec", ["fp32", "fp64", "bf16x3"])
def test_forward_every_entry_L512_multi_spin(prec):
    sht, dev = _sht(), _dev()
    print(f"[full entries] forward L={L_MID} spins={SPINS_MID} B={B_MID} {prec}", flush=True)
    ref = _mid_forward_ref()
    x = torch.from_numpy(_mid_maps()).to(dev, sht.io_dtype(prec))
    got = sht.forward_multi(x, L_MID, list(SPINS_MID), [B_MID] * len(SPINS_MID), prec)
    got = got.cpu().numpy().astype(np.complex128)
    assert got.shape == ref.shape
    for k, s in enumerate(SPINS_MID):
        for b in range(B_MID):
            i = k * B_MID + b
            assert np.all(got[i, :s * s] == 0), (s, b, prec)
            err = _rel(ref[i], got[i])
            assert err <= TOL[prec], (s, b, prec, err)


# ---- L = 1024 in the benchmark's launch configuration ----

def _workload():
    return {w.name: w for w in sht_synth.WORKLOADS}[BENCH]


@functools.lru_cache(maxsize=1)
def _bench_flm():
    wl = _workload()
    return {s: wl.flm(s) for s in wl.spins}


@functools.lru_cache(maxsize=None)
def _bench_inverse_ref(s):
    wl = _workload()
    return oracle.inverse(_bench_flm()[s][MEMBER[s]], wl.L, s)


def _fwd_seed(k, b):
    return SEED_FWD + 32 * k + b


@functools.lru_cache(maxsize=None)
def _bench_forward_ref(s):
    wl = _workload()
    k = list(wl.spins).index(s)
    return oracle.forward(sht_synth.random_complex_map(wl.L, _fwd_seed(k, MEMBER[s])), wl.L, s)


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
@pytest.mark.parametrize("s", [0, 2, -2])
def test_inverse_every_entry_benchmark_call(s, prec):
    sht, dev = _sht(), _dev()
    wl = _workload()
    L, B, spins = wl.L, wl.batch, list(wl.spins)
    assert spins == [0, 2, -2] and B == 16
    print(f"[full entries] inverse {BENCH} spin {s} map {MEMBER[s]} {prec}", flush=True)
    ref = _bench_inverse_ref(s)
    flm = _bench_flm()
    x = torch.cat([torch.from_numpy(flm[t]) for t in spins]).to(dev, sht.io_dtype(prec))
    fmap = sht.inverse_multi(x, L, spins, [B] * 3, prec)
    got = fmap[spins.index(s) * B + MEMBER[s]].cpu().numpy().astype(np.complex128)
    err = _rel(ref, got)
    print(f"[full entries] rel l2 {err:.3e}", flush=True)
    assert err <= TOL[prec], (s, prec, err)


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
@pytest.mark.parametrize("s", [0, 2, -2])
def test_forward_every_entry_benchmark_call(s, prec):
    sht, dev = _sht(), _dev()
    wl = _workload()
    L, B, spins = wl.L, wl.batch, list(wl.spins)
    print(f"[full entries] forward {BENCH} spin {s} map {MEMBER[s]} {prec}", flush=True)
    ref = _bench_forward_ref(s)
    k = spins.index(s)
    x = torch.empty((3 * B, L, 2 * L - 1), dtype=sht.io_dtype(prec), device=dev)
    for j in range(3):
        for b in range(B):
            x[j * B + b] = torch.from_numpy(sht_synth.random_complex_map(L, _fwd_seed(j, b))).to(dev, x.dtype)
    out = sht.forward_multi(x, L, spins, [B] * 3, prec)
    got = out[k * B + MEMBER[s]].cpu().numpy().astype(np.complex128)
    assert np.all(got[:s * s] == 0)
    err = _rel(ref, got)
    print(f"[full entries] rel l2 {err:.3e}", flush=True)
    assert err <= TOL[prec], (s, prec, err)


# ---- odd L in the 4096-point FFT range (the last theta block of a map holds one row) ----

L_ODD, S_ODD = 777, -3


@functools.lru_cache(maxsize=1)
def _odd_inputs():
    flm = sht_synth.gaussian_flm(L_ODD, S_ODD, SEED_MID + 500)
    fmap = sht_synth.random_complex_map(L_ODD, SEED_MID + 501)
    return flm, fmap, oracle.inverse(flm, L_ODD, S_ODD), oracle.forward(fmap, L_ODD, S_ODD)


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_every_entry_odd_L(prec):
    sht, dev = _sht(), _dev()
    print(f"[full entries] L={L_ODD} s={S_ODD} {prec}", flush=True)
    flm, fmap, ref_map, ref_flm = _odd_inputs()
    got_map = sht.inverse(torch.from_numpy(flm[None]).to(dev, sht.io_dtype(prec)), L_ODD, S_ODD, prec)
    got_flm = sht.forward(torch.from_numpy(fmap[None]).to(dev, sht.io_dtype(prec)), L_ODD, S_ODD, prec)
    err_i = _rel(ref_map, got_map[0].cpu().numpy().astype(np.complex128))
    err_f = _rel(ref_flm, got_flm[0].cpu().numpy().astype(np.complex128))
    assert err_i <= TOL[prec], err_i
    assert err_f <= TOL[prec], err_f
