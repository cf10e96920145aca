"""CPU tests of the Python binding's checks on a caller's output and
workspace tensors: the library writes through their data pointers, so a
tensor of the wrong shape, dtype, layout or device must be refused before any
library call."""

import pytest

torch = pytest.importorskip("torch")

from paper_0807_4494_amd import sht

CPU = torch.device("cpu")


def test_matching_output_passes():
    t = torch.empty((2, 5, 9), dtype=torch.complex128)
    sht.check_out("out", t, (2, 5, 9), torch.complex128, CPU)


@pytest.mark.parametrize("bad", ["shape", "batch", "dtype", "strided", "device", "type"])
def test_bad_output_is_refused(bad):
    shape, dt = (2, 5, 9), torch.complex128
    dev = CPU
    if bad == "shape":
        t = torch.empty((2, 5, 8), dtype=dt)
    elif bad == "batch":
        t = torch.empty((1, 5, 9), dtype=dt)
    elif bad == "dtype":
        t = torch.empty(shape, dtype=torch.complex64)        # half the bytes per element
    elif bad == "strided":
        t = torch.empty((2, 9, 5), dtype=dt).transpose(1, 2)  # right shape, not contiguous
    elif bad == "device":
        t = torch.empty(shape, dtype=dt)
        dev = torch.device("cuda", 0)                       # the input's device differs
    else:
        t = [0] * 90
    with pytest.raises(ValueError):
        sht.check_out("out", t, shape, dt, dev)


@pytest.mark.parametrize("bad", ["dtype", "strided", "device"])
def test_bad_workspace_is_refused(bad):
    dev = CPU
    if bad == "dtype":
        w = torch.empty(64, dtype=torch.float32)
    elif bad == "strided":
        w = torch.empty(128, dtype=torch.uint8)[::2]
    else:
        w = torch.empty(64, dtype=torch.uint8)
        dev = torch.device("cuda", 0)
    with pytest.raises(ValueError):
        sht.check_workspace(w, dev)
    sht.check_workspace(torch.empty(64, dtype=torch.uint8), CPU)
