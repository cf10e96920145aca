"""CPU tests of the C ABI: the library loads, exports every symbol the header
declares, and rejects bad arguments before touching HIP (no GPU needed)."""

import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "sht.h")


def _lib():
    from paper_0807_4494_amd import _native as N
    try:
        return N, N.load()
    except ImportError as e:
        pytest.fail(f"libsht.so must be built before the tests: {e}")


def header_functions():
    txt = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:const\s+)?[a-z_]+\s*\*?\s*(sht_[a-z_0-9]+)\s*\(", txt, re.M)))


def test_header_declares_the_entry_points():
    names = header_functions()
    for must in ("sht_inverse", "sht_forward", "sht_workspace_bytes", "sht_plan_warmup",
                 "sht_release_all", "sht_status_string", "sht_version"):
        assert must in names


def test_library_exports_every_declared_symbol():
    N, lib = _lib()
    for name in header_functions():
        assert hasattr(lib, name), name
    assert set(header_functions()) == set(N.EXPORTS)


def test_version_and_status_strings():
    N, lib = _lib()
    assert lib.sht_version() == 10000
    for code in (0, -1, -2, -3, -4, -5, -6, -7, -8, -99):
        assert lib.sht_status_string(code)


def test_argument_checks_run_before_any_hip_call():
    N, lib = _lib()
    fake = ctypes.c_void_p(1 << 20)     # never dereferenced: checks fail first
    big = 1 << 40
    call = lambda *a: lib.sht_inverse(*a)
    # sampling / precision
    assert call(8, 0, 1, 1, 0, fake, fake, fake, big, None) == N.SHT_ERR_UNSUPPORTED
    assert call(8, 0, 1, 0, 7, fake, fake, fake, big, None) == N.SHT_ERR_UNSUPPORTED
    # L, spin, batch
    assert call(0, 0, 1, 0, 0, fake, fake, fake, big, None) == N.SHT_ERR_INVALID_ARG
    assert call(4097, 0, 1, 0, 0, fake, fake, fake, big, None) == N.SHT_ERR_INVALID_ARG
    assert call(8, 8, 1, 0, 0, fake, fake, fake, big, None) == N.SHT_ERR_INVALID_ARG
    assert call(8, -8, 1, 0, 0, fake, fake, fake, big, None) == N.SHT_ERR_INVALID_ARG
    assert call(8, 0, 0, 0, 0, fake, fake, fake, big, None) == N.SHT_ERR_INVALID_ARG
    # NULL pointers, alignment, workspace size
    assert call(8, 0, 1, 0, 0, None, fake, fake, big, None) == N.SHT_ERR_INVALID_ARG
    assert call(8, 0, 1, 0, 0, ctypes.c_void_p((1 << 20) + 8), fake, fake, big, None) == N.SHT_ERR_ALIGNMENT
    assert call(8, 0, 1, 0, 0, fake, fake, ctypes.c_void_p((1 << 20) + 16), big, None) == N.SHT_ERR_ALIGNMENT
    need = lib.sht_workspace_bytes(8, 0, 1, 0, 0)
    assert call(8, 0, 1, 0, 0, fake, fake, fake, need - 1, None) == N.SHT_ERR_WORKSPACE
    assert lib.sht_forward(8, 0, 1, 0, 0, fake, fake, fake, need - 1, None) == N.SHT_ERR_WORKSPACE
    # real-signal entry points: map element-aligned, flm complex-aligned
    assert lib.sht_inverse_real(8, 1, 0, 0, ctypes.c_void_p((1 << 20) + 8), fake, fake, big, None) == \
        N.SHT_ERR_ALIGNMENT
    assert lib.sht_forward_real(8, 1, 0, 1, ctypes.c_void_p((1 << 20) + 2), fake, fake, big, None) == \
        N.SHT_ERR_ALIGNMENT
    assert lib.sht_forward_real(0, 1, 0, 0, fake, fake, fake, big, None) == N.SHT_ERR_INVALID_ARG
    assert lib.sht_forward_real(8, 1, 0, 0, fake, fake, fake, need - 1, None) == N.SHT_ERR_WORKSPACE
    # spin pairs: distinct, aligned buffers
    assert lib.sht_spin_pair(8, 2, 1, 0, fake, fake, None) == N.SHT_ERR_INVALID_ARG
    assert lib.sht_spin_pair(8, 2, 1, 0, ctypes.c_void_p((1 << 20) + 8), ctypes.c_void_p(1 << 21), None) == \
        N.SHT_ERR_ALIGNMENT
    assert lib.sht_spin_pair(8, 9, 1, 0, fake, ctypes.c_void_p(1 << 21), None) == N.SHT_ERR_INVALID_ARG
    # the triangular forward: FP64 only, L <= SHT_TRI_L_MAX
    tri = lib.sht_forward_triangular
    assert tri(8, 0, 1, 0, 1, fake, fake, fake, big, None) == N.SHT_ERR_UNSUPPORTED
    assert tri(N.SHT_TRI_L_MAX + 1, 0, 1, 0, 0, fake, fake, fake, big, None) == N.SHT_ERR_UNSUPPORTED
    assert tri(8, 8, 1, 0, 0, fake, fake, fake, big, None) == N.SHT_ERR_INVALID_ARG
    assert tri(8, 0, 1, 0, 0, fake, fake, fake, need - 1, None) == N.SHT_ERR_WORKSPACE
    # the least-squares variant: the same checks
    lsq = lib.sht_forward_lstsq
    assert lsq(8, 0, 1, 0, 1, fake, fake, fake, big, None) == N.SHT_ERR_UNSUPPORTED
    assert lsq(N.SHT_TRI_L_MAX + 1, 0, 1, 0, 0, fake, fake, fake, big, None) == N.SHT_ERR_UNSUPPORTED
    assert lsq(8, 8, 1, 0, 0, fake, fake, fake, big, None) == N.SHT_ERR_INVALID_ARG
    assert lsq(8, 0, 1, 0, 0, None, fake, fake, big, None) == N.SHT_ERR_INVALID_ARG
    assert lsq(8, 0, 1, 0, 0, fake, fake, fake, need - 1, None) == N.SHT_ERR_WORKSPACE


def test_graph_argument_checks_run_before_any_hip_call():
    N, lib = _lib()
    fake = ctypes.c_void_p(1 << 20)     # never dereferenced: checks fail first
    out = ctypes.c_void_p(123)
    big = 1 << 40
    # NULL handle slot, then invalid L / precision (out is cleared first)
    assert lib.sht_graph_create(8, 0, 1, 0, 1, fake, fake, fake, fake, big, None, None) == N.SHT_ERR_INVALID_ARG
    assert lib.sht_graph_create(0, 0, 1, 0, 1, fake, fake, fake, fake, big, None,
                                ctypes.byref(out)) == N.SHT_ERR_INVALID_ARG
    assert out.value is None
    assert lib.sht_graph_create(8, 0, 1, 0, 9, fake, fake, fake, fake, big, None,
                                ctypes.byref(out)) == N.SHT_ERR_UNSUPPORTED
    # unknown handles
    assert lib.sht_graph_launch(None, None) == N.SHT_ERR_INVALID_ARG
    assert lib.sht_graph_launch(fake, None) == N.SHT_ERR_INVALID_ARG
    assert lib.sht_graph_destroy(None) == N.SHT_ERR_INVALID_ARG
    assert lib.sht_graph_destroy(fake) == N.SHT_ERR_INVALID_ARG


def test_tile_and_tune_argument_checks_run_before_any_hip_call():
    N, lib = _lib()
    assert lib.sht_tile_set(0, 4, 1, 32) == N.SHT_ERR_INVALID_ARG
    assert lib.sht_tile_set(64, 0, 1, 32) == N.SHT_ERR_INVALID_ARG
    assert lib.sht_tile_set(64, 4 * 64 + 1, 1, 32) == N.SHT_ERR_INVALID_ARG
    assert lib.sht_tile_set(64, 8, 7, 32) == N.SHT_ERR_UNSUPPORTED
    assert lib.sht_tile_set(64, 8, 1, 48) == N.SHT_ERR_INVALID_ARG
    # the 128-column tile exists for FP32 only
    assert lib.sht_tile_set(64, 8, N.SHT_FP64, 128) == N.SHT_ERR_INVALID_ARG
    assert lib.sht_tile_set(64, 8, N.SHT_BF16X3, 128) == N.SHT_ERR_INVALID_ARG
    assert lib.sht_tile_set(64, 8, N.SHT_FP32, 256) == N.SHT_ERR_INVALID_ARG
    fake = ctypes.c_void_p(1 << 20)
    assert lib.sht_tune(0, 0, 1, 1, fake, 1 << 40, None, None) == N.SHT_ERR_INVALID_ARG
    assert lib.sht_tune(64, 0, 1, 1, None, 1 << 40, None, None) == N.SHT_ERR_INVALID_ARG
    assert lib.sht_tune(64, 0, 1, 1, ctypes.c_void_p((1 << 20) + 8), 1 << 40, None, None) == N.SHT_ERR_ALIGNMENT
    assert lib.sht_tune(64, 0, 1, 1, fake, 16, None, None) == N.SHT_ERR_WORKSPACE


def test_error_metrics_argument_checks_run_before_any_hip_call():
    N, lib = _lib()
    need = lib.sht_error_workspace_bytes()
    assert need >= 32 * 1024 and need % 256 == 0
    fake = ctypes.c_void_p(1 << 20)
    odd = ctypes.c_void_p((1 << 20) + 4)
    call = lib.sht_error_metrics
    assert call(7, 10, fake, fake, fake, fake, need, None) == N.SHT_ERR_UNSUPPORTED
    assert call(1, 10, None, fake, fake, fake, need, None) == N.SHT_ERR_INVALID_ARG
    assert call(1, 10, fake, None, fake, fake, need, None) == N.SHT_ERR_INVALID_ARG
    assert call(1, 10, fake, fake, None, fake, need, None) == N.SHT_ERR_INVALID_ARG
    assert call(1, 10, fake, fake, fake, None, need, None) == N.SHT_ERR_INVALID_ARG
    assert call(0, 1 << 37, fake, fake, fake, fake, need, None) == N.SHT_ERR_INVALID_ARG
    assert call(1, 10, fake, fake, fake, odd, need, None) == N.SHT_ERR_ALIGNMENT
    assert call(0, 10, odd, fake, fake, fake, need, None) == N.SHT_ERR_ALIGNMENT
    assert call(1, 10, fake, fake, ctypes.c_void_p((1 << 20) + 2), fake, need, None) == N.SHT_ERR_ALIGNMENT
    assert call(1, 10, fake, fake, fake, fake, need - 256, None) == N.SHT_ERR_WORKSPACE


def test_workspace_size_formula():
    N, lib = _lib()
    for L, B, p in [(32, 1, 0), (1024, 16, 1), (2048, 4, 1), (255, 3, 0), (2048, 2, 0), (4096, 1, 1),
                    (4096, 2, 0), (2049, 1, 0)]:
        T = 8 if p == 0 else 4
        C, Nn = 4 * B, 2 * L - 1
        al = lambda x: (x + 255) // 256 * 256
        ra = al(max(L * C * L * T, B * L * Nn * 2 * T))
        rb = ra
        # FFT rows whose M-point LDS buffer (M + M/16 complex) exceeds 160 KiB
        # (FP64 beyond L = 2048) add 256 scratch slots of M complex values
        M = 1 << max(3, (4 * L - 4).bit_length())
        rc = al(256 * M * 2 * T) if (M + M // 16) * 2 * T > 160 * 1024 else 0
        assert (rc > 0) == (p == 0 and L > 2048)
        assert lib.sht_workspace_bytes(L, 0, B, 0, p) == ra + rb + rc
    assert lib.sht_workspace_bytes(8, 9, 1, 0, 0) == 0
    assert lib.sht_workspace_bytes(8, 0, 1, 3, 0) == 0


def test_noalloc_argument_checks_run_before_any_hip_call():
    N, lib = _lib()
    fake = ctypes.c_void_p(1 << 20)
    call = lib.sht_inverse_noalloc
    assert call(4097, 0, 1, 0, 0, fake, fake, None) == N.SHT_ERR_INVALID_ARG
    assert call(8, 0, 1, 0, 5, fake, fake, None) == N.SHT_ERR_UNSUPPORTED
    assert call(8, 0, 1, 0, 0, None, fake, None) == N.SHT_ERR_INVALID_ARG
    assert call(8, 0, 1, 0, 0, fake, ctypes.c_void_p((1 << 20) + 8), None) == N.SHT_ERR_ALIGNMENT
    # beyond the static scratch: rejected by size, before any HIP call
    assert lib.sht_workspace_bytes(1024, 0, 16, 0, 1) > N.SHT_NOALLOC_SCRATCH_BYTES
    assert call(1024, 0, 16, 0, 1, fake, fake, None) == N.SHT_ERR_WORKSPACE
    assert lib.sht_workspace_bytes(512, 0, 8, 0, 1) <= N.SHT_NOALLOC_SCRATCH_BYTES
    assert lib.sht_workspace_bytes(512, 0, 9, 0, 1) > N.SHT_NOALLOC_SCRATCH_BYTES


def test_multi_argument_checks_run_before_any_hip_call():
    N, lib = _lib()
    fake = ctypes.c_void_p(1 << 20)
    big = 1 << 40
    arr = lambda *v: (ctypes.c_int * len(v))(*v)
    call = lib.sht_inverse_multi
    assert call(8, 0, arr(0), arr(1), 0, 0, fake, fake, fake, big, None) == N.SHT_ERR_INVALID_ARG
    assert call(8, 9, arr(*[0] * 9), arr(*[1] * 9), 0, 0, fake, fake, fake, big, None) == N.SHT_ERR_INVALID_ARG
    assert call(8, 2, arr(0, 8), arr(1, 1), 0, 0, fake, fake, fake, big, None) == N.SHT_ERR_INVALID_ARG  # |s| >= L
    assert call(8, 2, arr(0, 1), arr(1, 0), 0, 0, fake, fake, fake, big, None) == N.SHT_ERR_INVALID_ARG  # empty segment
    assert call(8, 2, arr(0, 1), arr(40, 25), 0, 0, fake, fake, fake, big, None) == N.SHT_ERR_INVALID_ARG  # > 64 maps
    assert call(8, 1, None, arr(1), 0, 0, fake, fake, fake, big, None) == N.SHT_ERR_INVALID_ARG
    assert call(8, 2, arr(0, 1), arr(1, 1), 0, 7, fake, fake, fake, big, None) == N.SHT_ERR_UNSUPPORTED
    need = lib.sht_workspace_bytes(8, 0, 5, 0, 0)
    assert lib.sht_forward_multi(8, 2, arr(0, 1), arr(2, 3), 0, 0, fake, fake, fake, need - 1, None) == \
        N.SHT_ERR_WORKSPACE
