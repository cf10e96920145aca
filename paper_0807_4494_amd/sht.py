"""Python entry points of the spin SHT (same names as the C ABI).

``inverse(flm, L, spin, precision)`` and ``forward(fmap, L, spin, precision)``
take and return CUDA/HIP torch tensors; torch provides device memory and the
current stream only.

Layouts (see include/sht.h): ``flm`` is complex ``[batch, L*L]`` (index
l*l + l + m) and maps are complex ``[batch, L, 2L-1]`` on the sampling of
Eq. (nodes_theta)/(nodes_phi).  A 1-D ``flm`` / 2-D map is treated as batch 1
and returned unbatched.  complex128 for ``"fp64"``, complex64 otherwise.
"""

from __future__ import annotations

from typing import Optional

import torch

from . import _native as N

PRECISIONS = {"fp64": N.SHT_FP64, "fp32": N.SHT_FP32, "bf16x3": N.SHT_BF16X3}


def _prec(precision) -> int:
    if isinstance(precision, int):
        return precision
    try:
        return PRECISIONS[precision]
    except KeyError:
        raise ValueError(f"precision must be one of {list(PRECISIONS)}") from None


def io_dtype(precision) -> torch.dtype:
    return torch.complex128 if _prec(precision) == N.SHT_FP64 else torch.complex64


def _stream_handle(device: torch.device) -> int:
    return torch.cuda.current_stream(device).cuda_stream


def workspace_bytes(L: int, spin: int, batch: int, precision="fp64") -> int:
    return int(N.load().sht_workspace_bytes(L, spin, batch, N.SHT_SAMPLING_MW, _prec(precision)))


def check_out(name: str, t: torch.Tensor, shape, dtype: torch.dtype, device: torch.device) -> None:
    """A caller's output tensor must be exactly what the library writes: the
    expected shape and dtype, contiguous, on the input's device (the library
    writes through its data pointer, so anything smaller or strided would be
    written past its end)."""
    if not isinstance(t, torch.Tensor):
        raise ValueError(f"{name} must be a torch.Tensor")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")
    if t.dtype != dtype:
        raise ValueError(f"{name} has dtype {t.dtype}, expected {dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if t.device != device:
        raise ValueError(f"{name} is on {t.device}, the input on {device}")


def check_workspace(t: torch.Tensor, device: torch.device) -> None:
    """A caller's workspace: contiguous uint8 on the input's device (its size
    is checked by the library against sht_workspace_bytes)."""
    if not isinstance(t, torch.Tensor) or t.dtype != torch.uint8 or not t.is_contiguous():
        raise ValueError("workspace must be a contiguous torch.uint8 tensor")
    if t.device != device:
        raise ValueError(f"workspace is on {t.device}, the input on {device}")


def _workspace(L, spin, batch, p, device, workspace):
    need = N.load().sht_workspace_bytes(L, spin, batch, N.SHT_SAMPLING_MW, p)
    if need == 0:
        # invalid arguments: let the library report the precise error
        return None, 0
    if workspace is None:
        workspace = torch.empty(need, dtype=torch.uint8, device=device)
    else:
        check_workspace(workspace, device)
    return workspace, workspace.numel() * workspace.element_size()


def _out(out, shape, dtype, device, name="out"):
    """The caller's output tensor after the checks of :func:`check_out`, or a new one."""
    if out is None:
        return torch.empty(shape, dtype=dtype, device=device)
    check_out(name, out, shape, dtype, device)
    return out


def inverse(flm: torch.Tensor, L: int, spin: int = 0, precision="fp64", out: Optional[torch.Tensor] = None,
            workspace: Optional[torch.Tensor] = None) -> torch.Tensor:
    """Inverse spin SHT: f_lm -> samples f(theta_t, phi_p)."""
    p = _prec(precision)
    single = flm.dim() == 1
    f = flm.reshape(1, -1) if single else flm
    if f.shape[-1] != L * L:
        raise ValueError(f"flm has {f.shape[-1]} coefficients per map, expected L*L = {L * L}")
    if not f.is_cuda:
        raise ValueError("flm must be a GPU tensor")
    f = f.to(io_dtype(p)).contiguous()
    B = f.shape[0]
    out = _out(out, (B, L, 2 * L - 1), io_dtype(p), f.device)
    ws, nbytes = _workspace(L, spin, B, p, f.device, workspace)
    rc = N.load().sht_inverse(L, spin, B, N.SHT_SAMPLING_MW, p, f.data_ptr(), out.data_ptr(),
                              ws.data_ptr() if ws is not None else None, nbytes, _stream_handle(f.device))
    N.check(rc, "sht_inverse")
    return out[0] if single else out


def _segments(spins, batches):
    import ctypes
    spins, batches = [int(x) for x in spins], [int(x) for x in batches]
    if len(spins) != len(batches) or not spins:
        raise ValueError("spins and batches must be non-empty and of equal length")
    n = len(spins)
    return n, (ctypes.c_int * n)(*spins), (ctypes.c_int * n)(*batches), sum(batches)


def inverse_multi(flm: torch.Tensor, L: int, spins, batches, precision="fp32", out: Optional[torch.Tensor] = None,
                  workspace: Optional[torch.Tensor] = None) -> torch.Tensor:
    """Inverse transform of maps of several spins at one L in one call
    (``sht_inverse_multi``): ``flm`` [sum(batches), L*L] holds segment k's
    ``batches[k]`` maps of spin ``spins[k]``, segment after segment; the
    result is each map's :func:`inverse` at its spin."""
    p = _prec(precision)
    nseg, sp, bt, B = _segments(spins, batches)
    if not flm.is_cuda or flm.dim() != 2 or tuple(flm.shape) != (B, L * L):
        raise ValueError(f"flm must be a GPU tensor [{B}, {L * L}]")
    f = flm.to(io_dtype(p)).contiguous()
    out = _out(out, (B, L, 2 * L - 1), io_dtype(p), f.device)
    ws, nbytes = _workspace(L, 0, B, p, f.device, workspace)
    rc = N.load().sht_inverse_multi(L, nseg, sp, bt, N.SHT_SAMPLING_MW, p, f.data_ptr(), out.data_ptr(),
                                    ws.data_ptr() if ws is not None else None, nbytes, _stream_handle(f.device))
    N.check(rc, "sht_inverse_multi")
    return out


def forward_multi(fmap: torch.Tensor, L: int, spins, batches, precision="fp32", out: Optional[torch.Tensor] = None,
                  workspace: Optional[torch.Tensor] = None) -> torch.Tensor:
    """Forward transform of maps of several spins at one L in one call
    (``sht_forward_multi``), segment layout as for :func:`inverse_multi`."""
    p = _prec(precision)
    nseg, sp, bt, B = _segments(spins, batches)
    if not fmap.is_cuda or tuple(fmap.shape) != (B, L, 2 * L - 1):
        raise ValueError(f"map must be a GPU tensor [{B}, {L}, {2 * L - 1}]")
    g = fmap.to(io_dtype(p)).contiguous()
    out = _out(out, (B, L * L), io_dtype(p), g.device)
    ws, nbytes = _workspace(L, 0, B, p, g.device, workspace)
    rc = N.load().sht_forward_multi(L, nseg, sp, bt, N.SHT_SAMPLING_MW, p, g.data_ptr(), out.data_ptr(),
                                    ws.data_ptr() if ws is not None else None, nbytes, _stream_handle(g.device))
    N.check(rc, "sht_forward_multi")
    return out


def inverse_noalloc(flm: torch.Tensor, L: int, spin: int, precision, out: torch.Tensor) -> torch.Tensor:
    """Inverse spin SHT through ``sht_inverse_noalloc``: no device memory is
    allocated (the library's static scratch is the workspace), so ``out``
    [batch, L, 2L-1] must be given and ``flm`` must already have the
    precision's dtype and be contiguous; the plan of (L, spin) must be
    resident (:func:`plan_warmup`).  Calls that overlap on one device race."""
    p = _prec(precision)
    if not flm.is_cuda or flm.dim() != 2 or flm.shape[-1] != L * L:
        raise ValueError("flm must be a GPU tensor [batch, L*L]")
    if flm.dtype != io_dtype(p) or not flm.is_contiguous():
        raise ValueError(f"flm must be contiguous {io_dtype(p)}")
    B = flm.shape[0]
    check_out("out", out, (B, L, 2 * L - 1), io_dtype(p), flm.device)
    rc = N.load().sht_inverse_noalloc(L, spin, B, N.SHT_SAMPLING_MW, p, flm.data_ptr(), out.data_ptr(),
                                      _stream_handle(flm.device))
    N.check(rc, "sht_inverse_noalloc")
    return out


def forward(fmap: torch.Tensor, L: int, spin: int = 0, precision="fp64", out: Optional[torch.Tensor] = None,
            workspace: Optional[torch.Tensor] = None) -> torch.Tensor:
    """Forward spin SHT: samples f(theta_t, phi_p) -> f_lm."""
    p = _prec(precision)
    single = fmap.dim() == 2
    g = fmap.reshape(1, *fmap.shape) if single else fmap
    if tuple(g.shape[-2:]) != (L, 2 * L - 1):
        raise ValueError(f"map shape {tuple(g.shape[-2:])}, expected ({L}, {2 * L - 1})")
    if not g.is_cuda:
        raise ValueError("map must be a GPU tensor")
    g = g.to(io_dtype(p)).contiguous()
    B = g.shape[0]
    out = _out(out, (B, L * L), io_dtype(p), g.device)
    ws, nbytes = _workspace(L, spin, B, p, g.device, workspace)
    rc = N.load().sht_forward(L, spin, B, N.SHT_SAMPLING_MW, p, g.data_ptr(), out.data_ptr(),
                              ws.data_ptr() if ws is not None else None, nbytes, _stream_handle(g.device))
    N.check(rc, "sht_forward")
    return out[0] if single else out


def real_dtype(precision) -> torch.dtype:
    return torch.float64 if _prec(precision) == N.SHT_FP64 else torch.float32


def inverse_real(flm: torch.Tensor, L: int, precision="fp64", out: Optional[torch.Tensor] = None,
                 workspace: Optional[torch.Tensor] = None) -> torch.Tensor:
    """Inverse transform of a real spin-0 signal: f_lm (m >= 0 read) -> real samples."""
    p = _prec(precision)
    single = flm.dim() == 1
    f = flm.reshape(1, -1) if single else flm
    if f.shape[-1] != L * L:
        raise ValueError(f"flm has {f.shape[-1]} coefficients per map, expected L*L = {L * L}")
    if not f.is_cuda:
        raise ValueError("flm must be a GPU tensor")
    f = f.to(io_dtype(p)).contiguous()
    B = f.shape[0]
    out = _out(out, (B, L, 2 * L - 1), real_dtype(p), f.device)
    ws, nbytes = _workspace(L, 0, B, p, f.device, workspace)
    rc = N.load().sht_inverse_real(L, B, N.SHT_SAMPLING_MW, p, f.data_ptr(), out.data_ptr(),
                                   ws.data_ptr() if ws is not None else None, nbytes, _stream_handle(f.device))
    N.check(rc, "sht_inverse_real")
    return out[0] if single else out


def forward_real(fmap: torch.Tensor, L: int, precision="fp64", out: Optional[torch.Tensor] = None,
                 workspace: Optional[torch.Tensor] = None) -> torch.Tensor:
    """Forward transform of a real spin-0 map -> f_lm (all m)."""
    p = _prec(precision)
    single = fmap.dim() == 2
    g = fmap.reshape(1, *fmap.shape) if single else fmap
    if tuple(g.shape[-2:]) != (L, 2 * L - 1):
        raise ValueError(f"map shape {tuple(g.shape[-2:])}, expected ({L}, {2 * L - 1})")
    if not g.is_cuda:
        raise ValueError("map must be a GPU tensor")
    if g.is_complex():
        raise ValueError("forward_real takes a real map")
    g = g.to(real_dtype(p)).contiguous()
    B = g.shape[0]
    out = _out(out, (B, L * L), io_dtype(p), g.device)
    ws, nbytes = _workspace(L, 0, B, p, g.device, workspace)
    rc = N.load().sht_forward_real(L, B, N.SHT_SAMPLING_MW, p, g.data_ptr(), out.data_ptr(),
                                   ws.data_ptr() if ws is not None else None, nbytes, _stream_handle(g.device))
    N.check(rc, "sht_forward_real")
    return out[0] if single else out


def spin_pair(flm_s: torch.Tensor, L: int, spin: int, precision="fp64",
              out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """Coefficients of the spin -s field f_{-s} = conj(f_s) from those of f_s."""
    p = _prec(precision)
    single = flm_s.dim() == 1
    f = (flm_s.reshape(1, -1) if single else flm_s).to(io_dtype(p)).contiguous()
    if f.shape[-1] != L * L or not f.is_cuda:
        raise ValueError("flm_s must be a GPU tensor [batch, L*L]")
    out = _out(out, tuple(f.shape), f.dtype, f.device)
    if out.data_ptr() == f.data_ptr():
        raise ValueError("out must not be the input")
    N.check(N.load().sht_spin_pair(L, spin, f.shape[0], p, f.data_ptr(), out.data_ptr(),
                                   _stream_handle(f.device)), "sht_spin_pair")
    return out[0] if single else out


def _forward_tri(fmap, L, spin, out, workspace, entry):
    p = N.SHT_FP64
    single = fmap.dim() == 2
    g = fmap.reshape(1, *fmap.shape) if single else fmap
    if tuple(g.shape[-2:]) != (L, 2 * L - 1):
        raise ValueError(f"map shape {tuple(g.shape[-2:])}, expected ({L}, {2 * L - 1})")
    if not g.is_cuda:
        raise ValueError("map must be a GPU tensor")
    g = g.to(torch.complex128).contiguous()
    B = g.shape[0]
    out = _out(out, (B, L * L), torch.complex128, g.device)
    ws, nbytes = _workspace(L, spin, B, p, g.device, workspace)
    rc = getattr(N.load(), entry)(L, spin, B, N.SHT_SAMPLING_MW, p, g.data_ptr(), out.data_ptr(),
                                  ws.data_ptr() if ws is not None else None, nbytes, _stream_handle(g.device))
    N.check(rc, entry)
    return out[0] if single else out


def forward_triangular(fmap: torch.Tensor, L: int, spin: int = 0, out: Optional[torch.Tensor] = None,
                       workspace: Optional[torch.Tensor] = None) -> torch.Tensor:
    """The paper's own forward transform (per-order triangular systems), FP64,
    L <= 512.  Ill conditioned beyond small L; see :func:`forward`."""
    return _forward_tri(fmap, L, spin, out, workspace, "sht_forward_triangular")


def forward_lstsq(fmap: torch.Tensor, L: int, spin: int = 0, out: Optional[torch.Tensor] = None,
                  workspace: Optional[torch.Tensor] = None) -> torch.Tensor:
    """All rows of the per-order systems, least squares (the stable
    comparison to :func:`forward_triangular`; not the paper's method), FP64,
    L <= 512."""
    return _forward_tri(fmap, L, spin, out, workspace, "sht_forward_lstsq")


def plan_warmup(L: int, spin: int = 0, precision="fp64", device=None) -> None:
    dev = torch.device("cuda", torch.cuda.current_device()) if device is None else torch.device(device)
    N.check(N.load().sht_plan_warmup(L, spin, N.SHT_SAMPLING_MW, _prec(precision), _stream_handle(dev)),
            "sht_plan_warmup")


def plan_tables(L: int, spin: int = 0, precision="fp32", enable: bool = True, device=None) -> None:
    """Build (or, with enable=False, free) the cached L^3 contraction table of
    (L, spin) for this precision class; transforms then stream it."""
    dev = torch.device("cuda", torch.cuda.current_device()) if device is None else torch.device(device)
    N.check(N.load().sht_plan_tables(L, spin, _prec(precision), 1 if enable else 0, _stream_handle(dev)),
            "sht_plan_tables")


def tile_set(L: int, columns: int, precision="fp32", tile: int = 0) -> None:
    """Pin the contraction's column tile (16, 32, 64, and 128 for fp32;
    0 = default) for (L, columns = 4 x batch, precision) on the current
    device."""
    N.check(N.load().sht_tile_set(L, columns, _prec(precision), tile), "sht_tile_set")


def tune(L: int, spin: int, batch: int, precision="fp32", device=None) -> int:
    """Autotuner: time the contraction with each column tile for this shape,
    pin the fastest and return it (synchronises the current stream)."""
    import ctypes
    p = _prec(precision)
    dev = torch.device("cuda", torch.cuda.current_device()) if device is None else torch.device(device)
    ws, nbytes = _workspace(L, spin, batch, p, dev, None)
    out = ctypes.c_int(0)
    N.check(N.load().sht_tune(L, spin, batch, p, ws.data_ptr() if ws is not None else None, nbytes,
                              _stream_handle(dev), ctypes.byref(out)), "sht_tune")
    return int(out.value)


ERROR_METRICS = ("max", "mean", "median", "rms", "rel_rms")


def error_metrics(ref: torch.Tensor, val: torch.Tensor) -> dict:
    """The five error measures of the paper's stability test (Section 4.2)
    of ``val`` against ``ref`` (same shape, complex64 or complex128, on the
    GPU), computed on the device in FP64 (``sht_error_metrics``): max, mean,
    median and rms of |ref - val| and the relative rms
    sqrt(sum |ref - val|^2 / sum |ref|^2).  Synchronises the current stream."""
    if ref.shape != val.shape or ref.dtype != val.dtype:
        raise ValueError("ref and val must have the same shape and dtype")
    if ref.dtype not in (torch.complex64, torch.complex128):
        raise ValueError("ref and val must be complex64 or complex128")
    if not (ref.is_cuda and val.is_cuda) or ref.device != val.device:
        raise ValueError("ref and val must be GPU tensors on one device")
    p = N.SHT_FP64 if ref.dtype == torch.complex128 else N.SHT_FP32
    f, g = ref.contiguous(), val.contiguous()
    lib = N.load()
    need = lib.sht_error_workspace_bytes()
    ws = torch.empty(need, dtype=torch.uint8, device=ref.device)
    out = torch.empty(5, dtype=torch.float64, device=ref.device)
    N.check(lib.sht_error_metrics(p, f.numel(), f.data_ptr() if f.numel() else None,
                                  g.data_ptr() if g.numel() else None, out.data_ptr(), ws.data_ptr(), need,
                                  _stream_handle(ref.device)), "sht_error_metrics")
    vals = out.cpu().tolist()
    return dict(zip(ERROR_METRICS, vals))


class Graph:
    """Captured inverse + forward of one shape (``sht_graph_create``): the
    inverse of ``flm_in`` into ``map`` and the forward of ``map`` into
    ``flm_out``, replayed by ``launch``.  The buffers are allocated here (torch
    device memory) and bound to the graph; write the next input into
    ``flm_in`` before a launch, read the results after it."""

    def __init__(self, L: int, spin: int, batch: int, precision="fp32", device=None):
        import ctypes
        self.L, self.spin, self.batch, self.p = L, spin, batch, _prec(precision)
        dev = torch.device("cuda", torch.cuda.current_device()) if device is None else torch.device(device)
        dt = io_dtype(self.p)
        # every replay's input overwrites all of flm_in, so it needs no clearing
        # (a fill here would also be unordered with the caller's own streams)
        self.flm_in = torch.empty((batch, L * L), dtype=dt, device=dev)
        self.map = torch.empty((batch, L, 2 * L - 1), dtype=dt, device=dev)
        self.flm_out = torch.empty((batch, L * L), dtype=dt, device=dev)
        self.workspace, nbytes = _workspace(L, spin, batch, self.p, dev, None)
        h = ctypes.c_void_p()
        rc = N.load().sht_graph_create(L, spin, batch, N.SHT_SAMPLING_MW, self.p, self.flm_in.data_ptr(),
                                       self.map.data_ptr(), self.flm_out.data_ptr(),
                                       self.workspace.data_ptr() if self.workspace is not None else None,
                                       nbytes, _stream_handle(dev), ctypes.byref(h))
        N.check(rc, "sht_graph_create")
        self._h = h.value
        self.device = dev

    def launch(self, stream: Optional[torch.cuda.Stream] = None) -> None:
        s = stream.cuda_stream if stream is not None else _stream_handle(self.device)
        N.check(N.load().sht_graph_launch(self._h, s), "sht_graph_launch")

    def close(self) -> None:
        if self._h is not None:
            N.check(N.load().sht_graph_destroy(self._h), "sht_graph_destroy")
            self._h = None


def release_all() -> None:
    N.check(N.load().sht_release_all(), "sht_release_all")


def version() -> int:
    return int(N.load().sht_version())


def trace_enable(on: bool = True) -> None:
    """Record HIP events around every stage of subsequent transforms."""
    N.check(N.load().sht_trace_enable(1 if on else 0), "sht_trace_enable")


def trace_read() -> dict:
    """Per-stage {name: (total_ms, launches)} since the last read (waits for the events)."""
    import ctypes
    n = len(N.STAGES)
    ms = (ctypes.c_double * n)()
    cnt = (ctypes.c_int * n)()
    N.check(N.load().sht_trace_read(ms, cnt, n), "sht_trace_read")
    return {name: (ms[i], cnt[i]) for i, name in enumerate(N.STAGES)}
