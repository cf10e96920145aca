"""GPU tests of the device error metrics (the five measures of Section 4.2)
against the oracle's definitions (oracle.error_metrics, numpy in FP64), on
seeded arrays: sizes that span one and many workgroups with ragged tails,
odd and even counts (median of one or two middle values), ties, exact
reconstructions, a zero reference and the empty array."""

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle

pytestmark = pytest.mark.gpu

SEED = 20260807


def _dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda", 0)


def _pair(n, dtype, seed, kind="noise"):
    rng = np.random.default_rng(seed)
    f = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    if kind == "noise":
        g = f + 1e-3 * (rng.standard_normal(n) + 1j * rng.standard_normal(n)) * rng.uniform(0, 4, n)
    elif kind == "ties":
        # values on a dyadic grid, so the errors are exact: most entries
        # exact, a third off by exactly 1/2 (the median is a tied zero)
        f = rng.integers(-64, 64, n) / 8 + 1j * rng.integers(-64, 64, n) / 8
        g = f.copy()
        idx = rng.choice(n, size=max(1, n // 3), replace=False)
        g[idx] += 0.5
    elif kind == "exact":
        g = f.copy()
    elif kind == "zero_ref":
        f = np.zeros(n, dtype=complex)
        g = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    f = f.astype(dtype)
    g = g.astype(dtype)
    return f, g


def _check(f, g):
    import paper_0807_4494_amd as sht
    dev = _dev()
    got = sht.error_metrics(torch.from_numpy(f).to(dev), torch.from_numpy(g).to(dev))
    # the definitions, in FP64 on the values the device saw
    want = oracle.error_metrics(f.astype(np.complex128), g.astype(np.complex128))
    for k in ("max", "median"):
        # single elements: |f - g| may differ by an ulp (sqrt of a sum of
        # squares against numpy's hypot)
        assert abs(got[k] - want[k]) <= 4e-16 * max(abs(want[k]), 1e-300), (k, got[k], want[k])
    for k in ("mean", "rms", "rel_rms"):
        # sums in a different order
        assert abs(got[k] - want[k]) <= 1e-12 * max(abs(want[k]), 1e-300), (k, got[k], want[k])
    return got


@pytest.mark.parametrize("dtype", [np.complex64, np.complex128])
@pytest.mark.parametrize("n", [1, 2, 3, 255, 256, 257, 4096, 100003, (1 << 20) + 5])
def test_metrics_match_the_definitions(n, dtype):
    print(f"[metrics] n={n} {np.dtype(dtype).name}", flush=True)
    _check(*_pair(n, dtype, SEED + n))


@pytest.mark.parametrize("kind", ["ties", "exact", "zero_ref"])
@pytest.mark.parametrize("n", [6, 1001, 300000])
def test_metrics_special_cases(kind, n):
    print(f"[metrics] {kind} n={n}", flush=True)
    got = _check(*_pair(n, np.complex128, SEED + 7 * n, kind))
    if kind == "exact":
        assert all(v == 0.0 for v in got.values())
    if kind == "ties":
        assert got["median"] == 0.0 and got["max"] == 0.5


def test_metrics_of_an_empty_array():
    import paper_0807_4494_amd as sht
    dev = _dev()
    e = torch.zeros(0, dtype=torch.complex64, device=dev)
    assert sht.error_metrics(e, e) == {k: 0.0 for k in sht.sht.ERROR_METRICS}


def test_round_trip_metrics_of_a_transform():
    """The stability protocol of Section 4.2 on the GPU path: inverse then
    forward, the five metrics against the oracle's on the same arrays."""
    import paper_0807_4494_amd as sht
    import sht_synth
    dev = _dev()
    L, s, B = 96, 2, 2
    flm = np.stack([sht_synth.gaussian_flm(L, s, SEED + b, "inv_lp1_sq") for b in range(B)])
    f = torch.from_numpy(flm).to(dev, torch.complex128)
    back = sht.forward(sht.inverse(f, L, s, "fp64"), L, s, "fp64")
    got = sht.error_metrics(f, back)
    want = oracle.error_metrics(flm, back.cpu().numpy())
    for k in want:
        assert abs(got[k] - want[k]) <= 1e-12 * max(want[k], 1e-300) + 1e-300, (k, got[k], want[k])
    assert got["rel_rms"] <= 1e-10
