"""Captured transforms (sht_graph_*): every replay equals the eager inverse +
forward of the same input, with eager work and synchronisations between the
replays, on the creation stream and on another stream."""

import numpy as np
import pytest
import torch

import oracle
import sht_synth

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-10, "fp32": 1e-5, "bf16x3": 5e-5}


def _sht():
    import paper_0807_4494_amd as sht
    return sht


def rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(a), 1e-300))


@pytest.mark.parametrize("prec,L,s,B", [("fp32", 48, 1, 3), ("fp64", 33, -2, 2), ("bf16x3", 64, 0, 4),
                                        ("fp32", 96, 2, 4), ("fp32", 80, 0, 3)])
def test_graph_replays_equal_eager(prec, L, s, B):
    sht = _sht()
    print(f"[graph] L={L} s={s} B={B} {prec}", flush=True)
    dev = torch.device("cuda", 0)
    dt = sht.io_dtype(prec)
    g = sht.Graph(L, s, B, prec, device=dev)
    side = torch.cuda.Stream(device=dev)
    try:
        for rnd in range(4):
            flm = np.stack([sht_synth.gaussian_flm(L, s, 5100 + 97 * rnd + 13 * b + L) for b in range(B)])
            x = torch.from_numpy(flm).to(dev, dt)
            g.flm_in.copy_(x)
            # eager work between the replays
            m_e = sht.inverse(x, L, s, prec)
            f_e = sht.forward(m_e, L, s, prec)
            torch.cuda.synchronize()
            if rnd % 2 == 0:
                g.launch()
            else:
                side.wait_stream(torch.cuda.current_stream(dev))
                g.launch(stream=side)
                torch.cuda.current_stream(dev).wait_stream(side)
            torch.cuda.synchronize()
            assert torch.equal(g.map, m_e), rnd
            assert torch.equal(g.flm_out, f_e), rnd
            if rnd == 3:
                # and the replayed result is the transform (oracle)
                ref = oracle.inverse_batch(flm, L, s)
                assert rel(ref, g.map.cpu().numpy()) < TOL[prec]
                assert rel(flm, g.flm_out.cpu().numpy()) < TOL[prec]
    finally:
        g.close()


def test_graph_handle_is_invalid_after_destroy():
    sht = _sht()
    import ctypes
    from paper_0807_4494_amd import _native as N
    g = sht.Graph(16, 0, 1, "fp32")
    h = g._h
    g.close()
    assert N.load().sht_graph_launch(ctypes.c_void_p(h), None) == N.SHT_ERR_INVALID_ARG


def test_table_stays_while_a_graph_reads_it():
    """A graph captured in cached-table mode keeps reading the table on every
    replay: freeing it is refused (SHT_ERR_BUSY) until the graph is gone, and
    replays meanwhile equal eager launches."""
    sht = _sht()
    from paper_0807_4494_amd import _native as N
    L, s, B, prec = 40, 2, 2, "fp32"
    print(f"[graph+table] L={L} s={s} B={B} {prec}", flush=True)
    dev = torch.device("cuda", 0)
    sht.plan_tables(L, s, prec, True)
    g = sht.Graph(L, s, B, prec, device=dev)
    try:
        with pytest.raises(N.ShtError) as err:
            sht.plan_tables(L, s, prec, False)
        assert err.value.code == N.SHT_ERR_BUSY
        flm = np.stack([sht_synth.gaussian_flm(L, s, 5300 + b) for b in range(B)])
        x = torch.from_numpy(flm).to(dev, sht.io_dtype(prec))
        g.flm_in.copy_(x)
        g.launch()
        m_e = sht.inverse(x, L, s, prec)
        f_e = sht.forward(m_e, L, s, prec)
        torch.cuda.synchronize()
        assert torch.equal(g.map, m_e) and torch.equal(g.flm_out, f_e)
        assert rel(flm, g.flm_out.cpu().numpy()) < TOL[prec]
    finally:
        g.close()
    sht.plan_tables(L, s, prec, False)      # no graph reads it any more


@pytest.mark.parametrize("bad", ["dtype", "batch", "strided"])
def test_bad_output_raises_before_launch(bad):
    sht = _sht()
    dev = torch.device("cuda", 0)
    L, s, B = 16, 1, 2
    x = torch.zeros((B, L * L), dtype=torch.complex128, device=dev)
    if bad == "dtype":
        out = torch.empty((B, L, 2 * L - 1), dtype=torch.complex64, device=dev)
    elif bad == "batch":
        out = torch.empty((B - 1, L, 2 * L - 1), dtype=torch.complex128, device=dev)
    else:
        out = torch.empty((B, 2 * L - 1, L), dtype=torch.complex128, device=dev).transpose(1, 2)
    with pytest.raises(ValueError):
        sht.inverse(x, L, s, "fp64", out=out)
    with pytest.raises(ValueError):
        sht.forward(torch.zeros((B, L, 2 * L - 1), dtype=torch.complex128, device=dev), L, s, "fp64",
                    out=torch.empty((B, L * L + 1), dtype=torch.complex128, device=dev))
