"""The roofline measurement kernels compute what they claim (so that the
bandwidth they report is for real copies), including an odd length."""

import ctypes

import pytest
import torch

from paper_1801_08682_amd import _lib

pytestmark = pytest.mark.gpu


def test_copy_triad_fma():
    P = _lib.load_peaks()
    h = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    vp = lambda t: ctypes.c_void_p(t.data_ptr())
    n = (1 << 20) + 3
    g = torch.Generator(device="cpu").manual_seed(5)
    a = torch.rand(n, generator=g, dtype=torch.float64).cuda()
    b = torch.rand(n, generator=g, dtype=torch.float64).cuda()
    c = torch.zeros_like(a)
    print("case stream copy/triad n", n, flush=True)
    assert P.adg_stream_copy(vp(a), vp(c), n, h) == 0
    torch.cuda.synchronize()
    assert torch.equal(c, a)
    assert P.adg_stream_triad(vp(a), vp(b), vp(c), 0.75, n, h) == 0
    torch.cuda.synchronize()
    ref = (a.cpu() + 0.75 * b.cpu())
    assert float((c.cpu() - ref).abs().max()) <= 1e-15
    sink = torch.zeros(64 * 256, dtype=torch.float64, device="cuda")
    for prec in (0, 1):
        print("case fma precision", prec, flush=True)
        assert P.adg_peak_fma(prec, 64, 1000, vp(sink), h) == 0
        torch.cuda.synchronize()
        vals = sink if prec == 0 else sink.view(torch.float32)[:64 * 256]
        assert bool(torch.isfinite(vals).all()) and float(vals.abs().sum()) > 0
