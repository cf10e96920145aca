"""The inverse that allocates nothing (sht_inverse_noalloc, static device
scratch) against sht_inverse: the same results on two calls in a row, the
second with a smaller input, within the precision's bar (and bitwise, as both
run the same kernels on the same inputs); refused shapes and missing plans
return their error codes."""

import ctypes

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle
import sht_synth

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-10, "fp32": 1e-5}


def _rel(a, b):
    return float(torch.linalg.vector_norm(a - b) / torch.linalg.vector_norm(a))


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_noalloc_inverse_equals_inverse_on_two_calls(prec):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_0807_4494_amd as sht
    from paper_0807_4494_amd import _native as N
    dev = torch.device("cuda", 0)
    dt = sht.io_dtype(prec)
    # each call smaller than the one before (fewer maps, lower band-limit);
    # the last is spin 0 (parity-ordered panels and the parity kernel in FP32)
    for k, (L, s, B) in enumerate([(160, 2, 5), (96, -1, 2), (64, 0, 1)]):
        print(f"[noalloc] call {k}: L={L} s={s} B={B} {prec}", flush=True)
        flm = np.stack([sht_synth.gaussian_flm(L, s, 7100 + 17 * k + b) for b in range(B)])
        x = torch.from_numpy(flm).to(dev, dt)
        sht.plan_warmup(L, s, prec)
        ref = sht.inverse(x, L, s, prec)
        out = torch.empty((B, L, 2 * L - 1), dtype=dt, device=dev)
        rc = N.load().sht_inverse_noalloc(L, s, B, N.SHT_SAMPLING_MW, sht.PRECISIONS[prec], x.data_ptr(),
                                          out.data_ptr(), torch.cuda.current_stream(dev).cuda_stream)
        assert rc == N.SHT_OK, rc
        torch.cuda.synchronize()
        assert _rel(ref, out) <= TOL[prec]
        assert torch.equal(ref, out)
        # and the transform itself (oracle)
        assert oracle.rel_l2(oracle.inverse_batch(flm, L, s), out.cpu().numpy()) < TOL[prec]


def test_noalloc_refusals():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_0807_4494_amd as sht
    from paper_0807_4494_amd import _native as N
    dev = torch.device("cuda", 0)
    lib = N.load()
    st = torch.cuda.current_stream(dev).cuda_stream
    # a plan that was never built: nothing is built, the call says so
    L, s, B = 77, 3, 1
    x = torch.zeros((B, L * L), dtype=torch.complex128, device=dev)
    out = torch.empty((B, L, 2 * L - 1), dtype=torch.complex128, device=dev)
    assert lib.sht_inverse_noalloc(L, s, B, 0, N.SHT_FP64, x.data_ptr(), out.data_ptr(), st) == \
        N.SHT_ERR_NOT_READY
    # a shape beyond the static scratch
    assert lib.sht_inverse_noalloc(512, 0, 9, 0, N.SHT_FP32, x.data_ptr(), out.data_ptr(), st) == \
        N.SHT_ERR_WORKSPACE
    # the binding wants the output given
    with pytest.raises(TypeError):
        sht.inverse_noalloc(x, L, s, "fp64")
