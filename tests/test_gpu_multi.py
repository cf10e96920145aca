"""Several spins at one band-limit in one call (sht_inverse_multi /
sht_forward_multi): each map's result equals the single-spin call at its
spin (bitwise: every output column is accumulated in the same order whatever
its column block) and the oracle's transform within the precision's bar."""

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle
import sht_synth

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-10, "fp32": 1e-5, "bf16x3": 2e-5}


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
]


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
    for s, n in zip(spins, batches):
        sl = slice(off, off + n)
        m1 = sht.inverse(x[sl], L, s, prec)
        f1 = sht.forward(maps[sl], L, s, prec)
        torch.cuda.synchronize()
        assert torch.equal(maps[sl], m1), (s, "inverse")
        assert torch.equal(back[sl], f1), (s, "forward")
        ref = oracle.inverse_batch(flm[sl], L, s)
        assert oracle.rel_l2(ref, maps[sl].cpu().numpy()) < TOL[prec]
        assert oracle.rel_l2(flm[sl], back[sl].cpu().numpy()) < TOL[prec]
        off += n
