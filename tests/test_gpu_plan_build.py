"""Plan building: the first call for a new (L, spin) builds its plan on the
library's own stream and waits only for that, not for the work already queued
on the caller's stream; the transform it then enqueues is correct."""

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle
import sht_synth

pytestmark = pytest.mark.gpu


def test_first_use_plan_build_does_not_wait_for_the_callers_stream():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_0807_4494_amd as sht
    dev = torch.device("cuda", 0)
    L, s, B = 203, 3, 2          # a band-limit no other test uses: its plan is new here
    flm = np.stack([sht_synth.gaussian_flm(L, s, 9100 + b) for b in range(B)])
    x = torch.from_numpy(flm).to(dev, torch.complex64)
    st = torch.cuda.Stream(device=dev)
    a = torch.randn(4096, 4096, device=dev)
    torch.cuda.synchronize()
    print("[plan build] queueing about 0.1 s of matrix products, then a first-use transform", flush=True)
    with torch.cuda.stream(st):
        for _ in range(80):
            a = torch.mm(a, a) * (1.0 / 64.0)   # stays finite: ||a|| does not grow
        m = sht.inverse(x, L, s, "fp32")
        pending = not st.query()
    st.synchronize()
    assert pending, "the first-use call waited for the work queued before it on its stream"
    ref = oracle.inverse_batch(flm, L, s)
    assert oracle.rel_l2(ref, m.cpu().numpy()) < 1e-5
