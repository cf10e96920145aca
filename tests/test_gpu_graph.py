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
                                        ("fp32", 96, 2, 4)])
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
