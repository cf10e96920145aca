"""GPU parity: the HIP path (through the C ABI) against the CPU oracle.

Inputs are the seeded band-limited coefficients of sht_synth; the forward
transform is fed the oracle's inverse of them (band-limited by construction),
so both directions have a unique exact answer.

Bars (relative l2 over all complex entries, Section 4.2's relative rms):
FP64 path <= 1e-10, FP32 path <= 1e-5.  The BF16x3 contraction (three BF16
products of hi/lo splits, FP32 accumulation) carries ~16 significant bits per
product; its measured error is ~4e-6 per direction, and its bar is 2e-5.
"""

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle
import sht_synth

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-10, "fp32": 1e-5, "bf16x3": 2e-5}


def _dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda", 0)


def _sht():
    import paper_0807_4494_amd as sht
    return sht


def to_dev(a, prec):
    sht = _sht()
    return torch.from_numpy(np.ascontiguousarray(a)).to(device=_dev(), dtype=sht.io_dtype(prec))


def rel(ref, got):
    return oracle.rel_l2(ref, got)


CASES = [(1, 0, 1), (2, 0, 1), (2, 1, 2), (3, -2, 1), (5, 1, 3), (8, 0, 2), (8, -3, 1), (16, 2, 1),
         (32, 0, 1), (33, -1, 2), (64, 2, 1), (100, -2, 3), (101, 3, 2), (129, 0, 1), (256, 2, 1),
         (257, -1, 2),
         # whole column tiles (4B = 16, 64, and 64 + a partial tile): the
         # contraction's full-slab load path
         (96, 1, 4), (160, -2, 16), (200, 0, 20)]


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3"])
@pytest.mark.parametrize("L,s,B", CASES)
def test_inverse_matches_oracle(L, s, B, prec):
    sht = _sht()
    print(f"[parity inverse] L={L} s={s} B={B} {prec}", flush=True)
    flm = np.stack([sht_synth.gaussian_flm(L, s, 7000 + 31 * L + 7 * b + s) for b in range(B)])
    ref = oracle.inverse_batch(flm, L, s)
    got = sht.inverse(to_dev(flm, prec), L, s, prec).cpu().numpy()
    assert got.shape == (B, L, 2 * L - 1)
    assert np.all(np.isfinite(got))
    assert rel(ref, got) < TOL[prec], rel(ref, got)


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3"])
@pytest.mark.parametrize("L,s,B", CASES)
def test_forward_matches_oracle(L, s, B, prec):
    sht = _sht()
    print(f"[parity forward] L={L} s={s} B={B} {prec}", flush=True)
    flm = np.stack([sht_synth.gaussian_flm(L, s, 9000 + 31 * L + 7 * b + s) for b in range(B)])
    fmap = oracle.inverse_batch(flm, L, s)
    ref = oracle.forward_batch(fmap, L, s)
    got = sht.forward(to_dev(fmap, prec), L, s, prec).cpu().numpy()
    assert got.shape == (B, L * L)
    assert np.all(np.isfinite(got))
    # entries with l < |s| are exactly zero
    nzero = s * s
    assert np.all(got[:, :nzero] == 0)
    assert rel(ref, got) < TOL[prec], rel(ref, got)
    assert rel(flm, got) < TOL[prec]


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("L,s,B", [(2, 1, 1), (5, 0, 2), (8, -3, 1), (33, -1, 2), (100, 2, 1), (257, 1, 1)])
def test_forward_of_unstructured_maps_matches_oracle(L, s, B, prec):
    """Off the band-limited subspace the forward is still one fixed linear
    operator (the quadrature of the extended torus); the theta = pi ring of an
    odd-parity row is where a shortcut would differ."""
    sht = _sht()
    print(f"[parity forward, unstructured] L={L} s={s} B={B} {prec}", flush=True)
    fmap = np.stack([sht_synth.random_complex_map(L, 4000 + 13 * L + b) for b in range(B)])
    ref = oracle.forward_batch(fmap, L, s)
    got = sht.forward(to_dev(fmap, prec), L, s, prec).cpu().numpy()
    assert rel(ref, got) < TOL[prec], rel(ref, got)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("name", ["L32_s0_b1", "L256_s2_b1"])
def test_small_workloads_exactly_as_configured(name, prec):
    """The single-map FP64 workloads (L=32 spin 0 flat spectrum; L=256 spin 2
    with C_l = 1/(l(l+1)), l >= 2): inverse and forward against the oracle,
    and the GPU round trip."""
    sht = _sht()
    wl = {w.name: w for w in sht_synth.WORKLOADS}[name]
    L, s = wl.L, wl.spins[0]
    print(f"[workload] {name} {prec}", flush=True)
    flm = wl.flm(s)
    ref_map = oracle.inverse_batch(flm, L, s)
    got_map = sht.inverse(to_dev(flm, prec), L, s, prec)
    assert rel(ref_map, got_map.cpu().numpy()) < TOL[prec]
    ref_f = oracle.forward_batch(ref_map, L, s)
    got_f = sht.forward(to_dev(ref_map, prec), L, s, prec).cpu().numpy()
    assert rel(ref_f, got_f) < TOL[prec]
    back = sht.forward(got_map, L, s, prec).cpu().numpy()
    assert rel(flm, back) < TOL[prec]


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3"])
def test_round_trip_L512(prec):
    sht = _sht()
    L, s, B = 512, 1, 2
    print(f"[round trip] L={L} s={s} B={B} {prec}", flush=True)
    flm = np.stack([sht_synth.gaussian_flm(L, s, 123 + b, "inv_lp1_sq") for b in range(B)])
    f = to_dev(flm, prec)
    back = sht.forward(sht.inverse(f, L, s, prec), L, s, prec).cpu().numpy()
    assert rel(flm, back) < 10 * TOL[prec]


@pytest.mark.parametrize("prec", ["fp32", "bf16x3"])
def test_deterministic_repeat(prec):
    sht = _sht()
    L, s = 96, 2
    flm = to_dev(sht_synth.gaussian_flm(L, s, 5), prec)
    a = sht.inverse(flm, L, s, prec)
    b = sht.inverse(flm, L, s, prec)
    assert torch.equal(a, b)
    fa = sht.forward(a, L, s, prec)
    fb = sht.forward(a, L, s, prec)
    assert torch.equal(fa, fb)


def test_input_rows_below_spin_are_ignored():
    sht = _sht()
    L, s = 20, 2
    flm = sht_synth.gaussian_flm(L, s, 11)
    noisy = flm.copy()
    noisy[: s * s] = 123.0 + 45.0j     # l < |s| entries must be ignored
    a = sht.inverse(to_dev(flm, "fp64"), L, s, "fp64")
    b = sht.inverse(to_dev(noisy, "fp64"), L, s, "fp64")
    assert torch.equal(a, b)


@pytest.mark.parametrize("L,s", [(1, 0), (2, 1), (5, 0), (8, -2), (12, 3), (16, 0), (16, 2)])
def test_triangular_forward_matches_oracle(L, s):
    """The paper's own forward (per-order triangular systems) against the
    oracle's back substitution; both recover the band-limited coefficients at
    these small L, where the systems are still well enough conditioned."""
    sht = _sht()
    print(f"[triangular] L={L} s={s}", flush=True)
    from oracle import triangular as T
    B = 3
    flm = np.stack([sht_synth.gaussian_flm(L, s, 600 + 17 * L + b) for b in range(B)])
    fmap = oracle.inverse_batch(flm, L, s)
    ref = np.stack([T.forward_triangular(fmap[b], L, s, split_spin0=(s == 0)) for b in range(B)])
    got = sht.forward_triangular(to_dev(fmap, "fp64"), L, s).cpu().numpy()
    assert rel(ref, got) < 1e-10, rel(ref, got)
    assert rel(flm, got) < 1e-9


@pytest.mark.parametrize("L,s", [(1, 0), (2, 1), (5, 0), (8, -2), (12, 3), (16, 0), (24, 2), (33, -1)])
def test_least_squares_forward_matches_oracle(L, s):
    """All rows of the per-order systems, least squares on the GPU (conjugate
    gradients on the normal equations) against the oracle's dense solve, on
    band-limited maps (both recover the coefficients) and on unstructured
    maps (a genuine least-squares problem)."""
    sht = _sht()
    print(f"[least squares] L={L} s={s}", flush=True)
    from oracle import triangular as T
    B = 5  # more than one pass of maps
    flm = np.stack([sht_synth.gaussian_flm(L, s, 700 + 13 * L + b) for b in range(B)])
    fmap = oracle.inverse_batch(flm, L, s)
    got = sht.forward_lstsq(to_dev(fmap, "fp64"), L, s).cpu().numpy()
    ref = np.stack([T.forward_lstsq(fmap[b], L, s) for b in range(B)])
    assert rel(ref, got) < 1e-11, rel(ref, got)
    assert rel(flm, got) < 1e-11
    noisy = np.stack([sht_synth.random_complex_map(L, 900 + b) for b in range(2)])
    got = sht.forward_lstsq(to_dev(noisy, "fp64"), L, s).cpu().numpy()
    ref = np.stack([T.forward_lstsq(noisy[b], L, s) for b in range(2)])
    assert rel(ref, got) < 1e-10, rel(ref, got)


@pytest.mark.parametrize("L,s", [(64, 0), (128, 2), (160, -1)])
def test_least_squares_forward_matches_oracle_at_larger_band_limits(L, s):
    """The all-rows systems stay well conditioned as L grows: the GPU solve
    (D in LDS up to L = 128, in global memory beyond) equals the oracle's
    dense least squares, and both return the band-limited coefficients."""
    sht = _sht()
    print(f"[least squares] L={L} s={s}", flush=True)
    from oracle import triangular as T
    flm = sht_synth.gaussian_flm(L, s, 760 + L)[None]
    fmap = oracle.inverse_batch(flm, L, s)
    got = sht.forward_lstsq(to_dev(fmap, "fp64"), L, s).cpu().numpy()
    ref = T.forward_lstsq(fmap[0], L, s)[None]
    assert rel(ref, got) < 1e-11, rel(ref, got)
    assert rel(flm, got) < 1e-11


def test_triangular_forward_far_from_the_diagonal_beyond_lds():
    """L = 160 (D in global memory): the paper's solve has lost the
    coefficients near the diagonal l = |m| (Section 4.2) but still recovers
    those far from it, l - |m| >= 3L/4, as the oracle's solve does."""
    sht = _sht()
    from oracle import triangular as T
    L = 160
    f = _real_test_function(L, 31)
    fmap = sht.inverse(to_dev(f, "fp64"), L, 0, "fp64")
    g = sht.forward_triangular(fmap, L, 0).cpu().numpy()
    l_of = np.repeat(np.arange(L), 2 * np.arange(L) + 1)
    m_of = np.arange(L * L) - l_of * l_of - l_of
    far = (l_of - np.abs(m_of)) >= 3 * L // 4
    ref = T.forward_triangular(oracle.inverse(f, L, 0), L, 0)
    assert np.abs(ref - f)[far].max() < 1e-9
    assert np.abs(g - f)[far].max() < 1e-9, np.abs(g - f)[far].max()
    assert np.abs(g - f).max() > 1e-3          # and near the diagonal it is lost


def _real_test_function(L, seed):
    """A real spin-0 test function of Section 4.2: Re, Im of f_lm (m > 0)
    from U[-1, 1], f_l0 real, f_{l,-m} = (-1)^m conj(f_lm)."""
    f = sht_synth.uniform_flm(L, 0, seed)
    for l in range(L):
        for m in range(1, l + 1):
            f[l * l + l - m] = (-1) ** m * np.conj(f[l * l + l + m])
        f[l * l + l] = f[l * l + l].real
    return f


def residual_structure(f, g, L):
    """Where the errors of a recovered real spin-0 function sit, by distance
    d = l - |m| from the diagonal: the fraction of coefficients off by more
    than 1e-6, the median error near the diagonal (d < 4) and far from it
    (d >= L/2), and the median d of the coefficients off by more than 1e-6."""
    l_of = np.repeat(np.arange(L), 2 * np.arange(L) + 1)
    m_of = np.arange(L * L) - l_of * l_of - l_of
    d = l_of - np.abs(m_of)
    r = np.abs(np.asarray(g) - np.asarray(f))
    bad = r > 1e-6
    return {"max": float(r.max()), "frac_bad": float(bad.mean()),
            "median_near_diagonal": float(np.median(r[d < 4])), "median_far": float(np.median(r[d >= L // 2])),
            "median_d_of_bad": float(np.median(d[bad])) if bad.any() else None}


def test_residual_structure_of_the_paper_forward():
    """Section 4.2's residual experiment on the GPU path: one real spin-0
    U[-1, 1] function through the inverse and the paper's triangular forward.
    At L = 16 and 32 the coefficients are recovered; at L = 64 the first
    large errors sit near the diagonal l = |m| while coefficients far from it
    stay exact; by L = 128 most coefficients are poor."""
    sht = _sht()
    rs = {}
    for L in (16, 32, 64, 128):
        f = _real_test_function(L, 4400 + L)
        fmap = sht.inverse(to_dev(f, "fp64"), L, 0, "fp64")
        g = sht.forward_triangular(fmap, L, 0).cpu().numpy()
        rs[L] = residual_structure(f, g, L)
    print(f"[residual structure] {rs}", flush=True)
    assert rs[16]["max"] < 1e-9
    assert rs[32]["frac_bad"] < 0.05 and rs[32]["median_far"] < 1e-13
    assert rs[64]["median_near_diagonal"] > 1e6 * rs[64]["median_far"]
    assert rs[64]["median_far"] < 1e-12 and rs[64]["median_d_of_bad"] < 64 // 4
    assert rs[128]["frac_bad"] > 0.5


@pytest.mark.parametrize("s", [0, 2, -3])
def test_least_squares_forward_is_exact_at_the_largest_band_limit(s):
    """At L = SHT_TRI_L_MAX, where the square triangular systems are hopeless,
    the all-rows least-squares solve still recovers band-limited
    coefficients to FP64 rounding, for every spin class."""
    sht = _sht()
    from paper_0807_4494_amd import _native as N
    L = N.SHT_TRI_L_MAX
    print(f"[least squares] L={L} s={s}", flush=True)
    flm = np.stack([sht_synth.gaussian_flm(L, s, 750 + b) for b in range(2)])
    fmap = sht.inverse(to_dev(flm, "fp64"), L, s, "fp64")
    got = sht.forward_lstsq(fmap, L, s).cpu().numpy()
    assert rel(flm, got) < 1e-12, rel(flm, got)


def test_triangular_forward_instability_on_the_gpu():
    """Section 4.2 on the GPU: real spin-0 U[-1, 1] test functions; the
    paper's forward is exact at L = 8 and loses accuracy by L = 64, while the
    quadrature forward stays exact."""
    sht = _sht()
    errs = {}
    for L in (8, 32, 64):
        f = sht_synth.uniform_flm(L, 0, 21 + L)
        # real signal: f_{l,-m} = (-1)^m conj(f_lm)
        for l in range(L):
            for m in range(1, l + 1):
                f[l * l + l - m] = (-1) ** m * np.conj(f[l * l + l + m])
            f[l * l + l] = f[l * l + l].real
        fmap = sht.inverse(to_dev(f, "fp64"), L, 0, "fp64")
        g = sht.forward_triangular(fmap, L, 0).cpu().numpy()
        q = sht.forward(fmap, L, 0, "fp64").cpu().numpy()
        ls = sht.forward_lstsq(fmap, L, 0).cpu().numpy()
        errs[L] = rel(f, g)
        assert rel(f, q) < 1e-12
        assert rel(f, ls) < 1e-12, (L, rel(f, ls))   # the least-squares variant stays exact
    print(f"[triangular] rel rms error by L: {errs}", flush=True)
    assert errs[8] < 1e-12
    assert errs[64] > 1e-3


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3"])
@pytest.mark.parametrize("L,s,B", [(33, -1, 2), (100, 2, 3), (257, 0, 1)])
def test_cached_table_mode_matches_oracle(L, s, B, prec):
    """With the plan's cached L^3 contraction table the transforms stream M
    instead of running the recursions; the results keep the same bars."""
    sht = _sht()
    print(f"[table mode] L={L} s={s} B={B} {prec}", flush=True)
    flm = np.stack([sht_synth.gaussian_flm(L, s, 800 + 31 * L + b) for b in range(B)])
    ref_map = oracle.inverse_batch(flm, L, s)
    sht.plan_tables(L, s, prec, True)
    try:
        got_map = sht.inverse(to_dev(flm, prec), L, s, prec).cpu().numpy()
        got_f = sht.forward(to_dev(ref_map, prec), L, s, prec).cpu().numpy()
    finally:
        sht.plan_tables(L, s, prec, False)
    assert rel(ref_map, got_map) < TOL[prec], rel(ref_map, got_map)
    assert rel(flm, got_f) < TOL[prec], rel(flm, got_f)


def _real_signal_flm(L, seed):
    """Coefficients of a real spin-0 signal: f_{l,-m} = (-1)^m conj(f_lm)."""
    f = sht_synth.gaussian_flm(L, 0, seed)
    for l in range(L):
        f[l * l + l] = f[l * l + l].real
        for m in range(1, l + 1):
            f[l * l + l - m] = (-1) ** m * np.conj(f[l * l + l + m])
    return f


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3"])
@pytest.mark.parametrize("L,B", [(1, 1), (2, 2), (7, 3), (33, 1), (96, 8), (100, 20), (257, 2)])
def test_real_signal_path_matches_oracle(L, B, prec):
    """Real spin-0 maps: only m >= 0 is transformed (Section 3.3); the result
    equals the complex transform of the same signal."""
    sht = _sht()
    print(f"[real] L={L} B={B} {prec}", flush=True)
    flm = np.stack([_real_signal_flm(L, 900 + 13 * L + b) for b in range(B)])
    ref_map = oracle.inverse_batch(flm, L, 0)
    assert np.abs(ref_map.imag).max() <= 1e-12 * max(1.0, np.abs(ref_map).max())
    got_map = sht.inverse_real(to_dev(flm, prec), L, prec)
    assert got_map.dtype == sht.real_dtype(prec) and got_map.shape == (B, L, 2 * L - 1)
    assert rel(ref_map.real, got_map.cpu().numpy()) < TOL[prec]
    rmap = torch.from_numpy(np.ascontiguousarray(ref_map.real)).to(_dev())
    back = sht.forward_real(rmap, L, prec).cpu().numpy()
    assert rel(flm, back) < TOL[prec]
    # an unstructured real map: the same linear operator as the complex path
    raw = np.stack([sht_synth.random_complex_map(L, 70 + b).real for b in range(B)])
    ref_f = oracle.forward_batch(raw.astype(np.complex128), L, 0)
    got_f = sht.forward_real(torch.from_numpy(raw).to(_dev()), L, prec).cpu().numpy()
    assert rel(ref_f, got_f) < TOL[prec], rel(ref_f, got_f)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("L,s,B", [(8, 2, 1), (33, -1, 2), (100, 2, 3)])
def test_spin_pair_coefficients(L, s, B, prec):
    """One transform serves a conjugate spin pair (Section 3.3)."""
    sht = _sht()
    flm = np.stack([sht_synth.gaussian_flm(L, s, 1200 + L + b) for b in range(B)])
    fmap = oracle.inverse_batch(flm, L, s)
    ref = oracle.forward_batch(np.conj(fmap), L, -s)
    got = sht.spin_pair(to_dev(flm, prec), L, s, prec).cpu().numpy()
    assert rel(ref, got) < TOL[prec]
    # and through the transforms: the spin -s forward of the conjugate map
    fm = sht.inverse(to_dev(flm, prec), L, s, prec)
    g2 = sht.forward(torch.conj(fm).resolve_conj().contiguous(), L, -s, prec).cpu().numpy()
    assert rel(ref, g2) < TOL[prec]
