"""The allocation-free amplitude entry point (dnqs_amplitudes_noalloc, for callers that
cannot allocate device memory) against dnqs_amplitudes, through the C ABI: two calls in a
row on one context, the second on fewer configurations, each equal to the allocating
call bit for bit (same kernels, same arithmetic); a size beyond the scratch region is
refused before any launch."""
import ctypes as C

import numpy as np
import pytest
import torch

from tests import problems as P

pytestmark = pytest.mark.gpu


def _noalloc(dnqs, ctx, widths, theta, dets, precision):
    L = dnqs.lib()
    f = L.dnqs_amplitudes_noalloc
    f.argtypes = [C.c_void_p, C.c_int, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64, C.c_int, C.c_void_p,
                  C.c_void_p]
    f.restype = C.c_int
    n = dets.shape[0]
    la = torch.full((n,), np.nan, dtype=torch.float64, device="cuda")
    sg = torch.full((n,), 7, dtype=torch.int8, device="cuda")
    net = dnqs._native.Net.from_widths(widths)
    st = f(ctx.handle, 0, C.byref(net), C.c_void_p(theta.data_ptr()), C.c_void_p(dets.data_ptr()), n, precision,
           C.c_void_p(la.data_ptr()), C.c_void_p(sg.data_ptr()))
    return st, la, sg


@pytest.mark.parametrize("name,prec", [("m16_5a5b_s16k", "FP32"), ("m28_7a7b_s100k", "MIXED")])
def test_noalloc_equals_allocating_call(name, prec):
    import paper_2601_21310_amd as dnqs
    assert torch.cuda.is_available()
    p = P.problem(name, 5000)
    ctx = dnqs.Context(0)
    ctx.set_integrals(p.h, p.eri, p.e_core, p.wl.n_alpha, p.wl.n_beta)
    theta = torch.from_numpy(p.theta).cuda()
    pr = getattr(dnqs, prec)
    for n in (5000, 1237):   # second call smaller: stale scratch contents must not matter
        dets = dnqs.dets_to_device(p.dets[:n])
        st, la, sg = _noalloc(dnqs, ctx, p.wl.widths, theta, dets, pr)
        assert st == 0, dnqs.lib().dnqs_last_error(ctx.handle)
        la0, sg0 = ctx.amplitudes(p.wl.widths, theta, dets, precision=pr)
        torch.cuda.synchronize()
        assert torch.equal(sg, sg0)
        assert torch.equal(la.view(torch.int64), la0.view(torch.int64))
    # beyond the region: refused on the host, outputs untouched
    big = dnqs.dets_to_device(np.repeat(p.dets[:1], 200000, axis=0))
    st, la, sg = _noalloc(dnqs, ctx, p.wl.widths, theta, big, pr)
    assert dnqs._native.STATUS[st] == "ECAPACITY"
    assert "scratch" in dnqs.lib().dnqs_last_error(ctx.handle).decode()
    torch.cuda.synchronize()
    assert torch.all(sg == 7)
    ctx.close()
