"""Activation recomputation (DNQS_RECOMPUTE; the paper's micro-batched gradient
accumulation, Sec. 3.1): the energy and gradient equal the stored path's bit for bit, on
the benchmark workload (M = 28, |S| = 1e5: two row blocks) and on the large-space network
(M = 56, 112 -> 1024 -> 1024 -> 2688, |S| = 1e5), in FP32 and in the mixed form, while the
context holds less device memory."""
import pytest
import torch

import synth

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("name", ["m28_7a7b_s100k", "m56_12a12b"])
@pytest.mark.parametrize("prec", ["FP32", "MIXED"])
def test_recompute_bit_identical(name, prec):
    import paper_2601_21310_amd as dnqs
    assert torch.cuda.is_available()
    print(f"[recompute] {name} {prec}", flush=True)
    wl = synth.WORKLOADS[name]
    p = synth.make_problem(wl, n_dets=100000, out_scale=1e-2)
    res, held = {}, {}
    for rc in (False, True):
        ctx = dnqs.Context(0)
        ctx.set_integrals(p.h, p.eri, p.e_core, wl.n_alpha, wl.n_beta)
        dets = dnqs.dets_to_device(p.dets)
        theta = torch.from_numpy(p.theta).cuda()
        conn = ctx.build_connections(dets, validate=False)
        r = ctx.energy_and_grad(wl.widths, theta, conn, precision=getattr(dnqs, prec), recompute=rc)
        torch.cuda.synchronize()
        res[rc] = {k: r[k].clone() for k in ("E", "grad", "logabs", "sign", "v")}
        held[rc] = ctx.allocator.live_bytes
        conn.free()
        ctx.close()
    a, b = res[False], res[True]
    print(f"  E {a['E'].item():.12f}; device memory held {held[False] / 2**30:.2f} GiB stored, "
          f"{held[True] / 2**30:.2f} GiB recomputing", flush=True)
    for k in ("E", "grad", "logabs", "v"):
        x, y = a[k], b[k]
        assert torch.equal(x.view(torch.int64) if x.dtype == torch.float64 else x.view(torch.int32),
                           y.view(torch.int64) if y.dtype == torch.float64 else y.view(torch.int32)), k
    assert torch.equal(a["sign"], b["sign"])
    assert held[True] < held[False]
