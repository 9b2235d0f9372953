"""GPU: the measurement probes (elm_probe_*) run and report plausible rates.

The probes are not part of the method; they give the device ceilings the
kernels are held against (sustained MFMA rate, streaming read, direct
global->LDS staging).  Checked: each returns a positive time and a rate below
the published peak of its resource, and a buffer too small for the staging
probe is refused with an error.
"""
import pytest
import torch

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def elm():
    from paper_2011_02436_amd import elm as mod
    return mod


def test_probes(elm):
    for dt, peak in (("bf16", 2500.0), ("fp64", 78.6)):
        for rnd in (False, True):
            tf, ms = elm.probe_mfma(dt, rnd)
            print(f"mfma {dt} random={rnd}: {tf:.1f} TFLOP/s ({ms:.3f} ms)")
            assert ms > 0 and 0 < tf <= 1.05 * peak
    tf, ms = elm.probe_mfma("fp64", True, shape=1)
    print(f"mfma fp64 four-block 4x4x4: {tf:.1f} TFLOP/s ({ms:.3f} ms)")
    assert ms > 0 and 0 < tf <= 1.05 * 78.6
    with pytest.raises(elm.ElmError):
        elm.probe_mfma("bf16", True, shape=1)
    buf = torch.empty(1 << 30, dtype=torch.uint8, device="cuda")
    gbs, ms = elm.probe_stream(buf)
    print(f"stream read: {gbs:.0f} GB/s ({ms:.3f} ms)")
    assert ms > 0 and 0 < gbs <= 8000.0
    gbs, ms = elm.probe_dma(buf)
    print(f"dma stream: {gbs:.0f} GB/s ({ms:.3f} ms)")
    assert ms > 0 and 0 < gbs <= 8000.0
    gbs, ms = elm.probe_dma(buf, resident=True)
    print(f"dma resident: {gbs:.0f} GB/s ({ms:.3f} ms)")
    assert ms > 0 and gbs > 0
    with pytest.raises(elm.ElmError):
        elm.probe_dma(buf[: 1 << 20])
