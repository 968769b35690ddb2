"""Autotuner of the network GEMM tiles (tile height 128/64, weight-gradient split-K).

* a tuned context gives the same energy as the default configuration bit for bit (the
  tile height does not change any element's summation order) and the same gradient up
  to the split-K summation order;
* its table round-trips through export/import, and a context that imports it (tuning
  off) reproduces the tuned results bit for bit;
* malformed tables are rejected and leave the table unchanged;
* the batched path tunes its own shapes and still matches the single-problem results.
"""
import numpy as np
import pytest
import torch

import synth
from tests import problems as P

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dnqs():
    import paper_2601_21310_amd as d
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return d


def _ctx(dnqs, p):
    ctx = dnqs.Context(0)
    ctx.set_integrals(p.h, p.eri, p.e_core, p.wl.n_alpha, p.wl.n_beta)
    return ctx


@pytest.mark.parametrize("prec", ["FP32", "MIXED"])
def test_tuned_matches_default_and_round_trips(dnqs, prec):
    p = P.problem("m16_5a5b_s16k")
    pr = getattr(dnqs, prec)
    theta = torch.from_numpy(p.theta).cuda()
    dets = dnqs.dets_to_device(p.dets)

    base = _ctx(dnqs, p)
    cb = base.build_connections(dets)
    r0 = base.energy_and_grad(p.wl.widths, theta, cb, precision=pr)

    tuned = _ctx(dnqs, p)
    tuned.autotune(True)
    ct = tuned.build_connections(dets)
    r1 = tuned.energy_and_grad(p.wl.widths, theta, ct, precision=pr)   # tunes
    r2 = tuned.energy_and_grad(p.wl.widths, theta, ct, precision=pr)   # uses the table
    torch.cuda.synchronize()
    table = tuned.tune_export()
    lines = [ln.split() for ln in table.strip().splitlines()]
    print(f"  [{prec}] {len(lines)} tuned shapes:\n" + table)
    L = len(p.wl.widths) - 1
    assert len(lines) == 3 * L - 2      # forward for l >= 2, weight gradient per layer, data gradient for l >= 2
    for ln in lines:
        eng, kind, M, N, K, tm, splits = map(int, ln)
        assert tm in (64, 128) and kind in (0, 1, 2)
        assert splits >= 1
    assert r0["E"].item() == r1["E"].item() == r2["E"].item()
    g0, g1, g2 = (r["grad"].double().cpu().numpy() for r in (r0, r1, r2))
    assert np.array_equal(g1, g2)
    assert P.rel_l2(g1, g0) <= (1e-6 if prec == "FP32" else 1e-5)

    imp = _ctx(dnqs, p)
    imp.tune_import(table)
    assert imp.tune_export() == table
    ci = imp.build_connections(dets)
    r3 = imp.energy_and_grad(p.wl.widths, theta, ci, precision=pr)
    torch.cuda.synchronize()
    assert r3["E"].item() == r1["E"].item()
    assert np.array_equal(r3["grad"].double().cpu().numpy(), g1)


def test_tune_import_rejects_bad_tables(dnqs):
    p = P.problem("m8_4a4b_full")
    ctx = _ctx(dnqs, p)
    ctx.tune_import("0 0 4900 64 16 64 1\n")
    good = ctx.tune_export()
    for bad in ["0 0 4900 64 16 96 1\n",          # tile height not 64/128
                "0 1 17 64 4900 128 0\n",         # weight gradient with 0 splits
                "0 2 4900 64 16 128 3\n",         # split-K on a data gradient
                "0 0 4900 64\n",                  # too few fields
                "0 0 4900 64 16 128 1 7\n"]:      # too many fields
        with pytest.raises(dnqs.DnqsError, match="EINVAL"):
            ctx.tune_import(good + bad)
        assert ctx.tune_export() == good


def test_batched_tuned_matches_single(dnqs):
    wl = synth.WORKLOADS["m20_6a6b_curve"]
    curve = synth.make_curve(wl, n_geoms=3, sizes=[700, 300, 1300], out_scale=1.0)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        ctx = dnqs.Context(0)
        ctx.autotune(True)
        conns = []
        for g, p in enumerate(curve):
            ctx.set_integrals(p.h, p.eri, p.e_core, wl.n_alpha, wl.n_beta, slot=g)
            conns.append(ctx.build_connections(dnqs.dets_to_device(p.dets), slot=g))
        thetas = [torch.from_numpy(p.theta).cuda() for p in curve]
        batch = ctx.batch(wl.widths, list(range(len(curve))), conns, thetas)
        out = ctx.energy_and_grad_batched(batch, precision=dnqs.MIXED)
        single = [ctx.energy_and_grad(wl.widths, thetas[g], conns[g], precision=dnqs.MIXED, full_output=True)
                  for g in range(3)]
        stream.synchronize()
    kinds = sorted({int(ln.split()[1]) for ln in ctx.tune_export().strip().splitlines()})
    assert kinds == [0, 1, 2, 3]
    for g in range(3):
        assert abs(out[g]["E"].item() - single[g]["E"].item()) <= 1e-9 * max(1.0, abs(single[g]["E"].item()))
        assert P.rel_l2(out[g]["grad"].double().cpu().numpy(), single[g]["grad"].double().cpu().numpy()) <= 1e-4
