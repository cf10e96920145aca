"""CPU checks of the benchmark's synthetic inputs (no GPU): the stability
test functions of Section 4.2 are coefficients of real maps (the oracle's
synthesis of them has no imaginary part) with Re, Im in [-1, 1], and they are
seeded (the same call gives the same functions)."""

import numpy as np
import pytest

import bench
import oracle


@pytest.mark.parametrize("L", [1, 2, 5, 12])
def test_stability_functions_are_real_maps(L):
    fs = bench.real_test_functions(L, 3)
    assert fs.shape == (3, L * L) and fs.dtype == np.complex128
    assert np.all(np.abs(fs.real) <= 1.0) and np.all(np.abs(fs.imag) <= 1.0)
    for f in fs:
        fmap = oracle.inverse(f, L, 0)
        assert np.abs(fmap.imag).max() <= 1e-13 * max(1.0, np.abs(fmap.real).max())
    # m = 0 coefficients are real, and the draws differ between functions
    m0 = np.array([l * l + l for l in range(L)])
    assert np.all(fs[:, m0].imag == 0.0)
    if L > 1:
        assert not np.array_equal(fs[0], fs[1])
    assert np.array_equal(fs, bench.real_test_functions(L, 3))
