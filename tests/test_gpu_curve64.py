"""Batched geometries at the size of the dissociation-curve workload: 64 geometries with
|S_g| log-uniform in [2^10, 2^16] (about 1e6 determinants), evaluated in one batched call
(one launch per stage over all geometries, rows laid out largest geometry first, the
per-geometry reductions one workgroup per 4096-row item, items largest geometry first).
Every geometry's E and gradient are compared with its single-problem call (full-width
output layer, as the batched call computes it): E to 1e-9 relative, the gradient to 1e-5
relative L2 (the two calls cut the weight-gradient sums over up to 6e4 rows into
different split-K blocks, so FP32 rounding differs by about u sqrt(rows)).  Eight
geometries spread over the size range, the largest and the smallest among them, are
compared with the FP64 oracle (|dE| <= 1e-6 Ha, gradient relative L2 <= 1e-4)."""
import numpy as np
import pytest
import scipy.sparse as sp
import torch

import synth
from tests import problems as P

pytestmark = pytest.mark.gpu

WL = synth.WORKLOADS["m20_6a6b_curve"]


def _step(t0, what):
    import time
    torch.cuda.synchronize()
    print(f"  {time.time() - t0:7.1f}s {what}", flush=True)


def test_curve64_batched_against_single_and_oracle():
    import paper_2601_21310_amd as dnqs
    from oracle import energy
    from oracle import hamiltonian as ham
    assert torch.cuda.is_available()
    curve = synth.make_curve(WL, n_geoms=64, out_scale=1.0)
    sizes = [p.dets.shape[0] for p in curve]
    print(f"[curve64] {len(curve)} geometries, sizes {min(sizes)}..{max(sizes)}, total {sum(sizes)}", flush=True)
    assert max(sizes) > 2 ** 15 and min(sizes) < 2 ** 11
    import time
    t0 = time.time()
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        ctx = dnqs.Context(0)
        conns = []
        for g, p in enumerate(curve):
            ctx.set_integrals(p.h, p.eri, p.e_core, WL.n_alpha, WL.n_beta, slot=g)
            conns.append(ctx.build_connections(dnqs.dets_to_device(p.dets), slot=g, validate=False))
            if g % 16 == 15:
                _step(t0, f"connections of {g + 1} geometries")
        thetas = [torch.from_numpy(p.theta).cuda() for p in curve]
        batch = ctx.batch(WL.widths, list(range(len(curve))), conns, thetas)
        out = ctx.energy_and_grad_batched(batch)
        _step(t0, "batched call")
        single = []
        for g in range(len(curve)):
            single.append(ctx.energy_and_grad(WL.widths, thetas[g], conns[g], full_output=True))
            if g % 16 == 15:
                _step(t0, f"single calls for {g + 1} geometries")
        stream.synchronize()
    for g in range(len(curve)):
        Eb, Es = out[g]["E"].item(), single[g]["E"].item()
        gb, gs = out[g]["grad"].double().cpu().numpy(), single[g]["grad"].double().cpu().numpy()
        assert abs(Eb - Es) <= 1e-9 * max(1.0, abs(Es)), g
        assert P.rel_l2(gb, gs) <= 1e-5, g
    print("  batched = single for all 64 geometries", flush=True)
    order = np.argsort(sizes)
    sample = sorted(set([int(order[0]), int(order[-1])] + [int(order[k]) for k in np.linspace(1, 62, 6).astype(int)]))
    assert len(sample) >= 8
    for g in sample:
        p = curve[g]
        rp, col, val, diag = ham.csr_rows(WL.M, p.h, p.eri, p.e_core, p.dets)
        n = len(diag)
        H = (sp.csr_matrix((val, col, rp), shape=(n, n)) + sp.diags(diag)).tocsr()
        o = energy.energy_and_grad(p.theta, WL.widths, p.dets, WL.M, WL.n_elec, H)
        dE = abs(out[g]["E"].item() - o["E"])
        print(f"  geometry {g} |S| {sizes[g]}: |dE| {dE:.2e}", flush=True)
        P.check_grad(out[g]["grad"].double().cpu().numpy(), o["grad"], WL.widths, 1e-4)
        assert dE <= 1e-6
