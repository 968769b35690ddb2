"""GPU parity at the benchmark's full size: M = 28, 7 alpha + 7 beta, |S| = 1e5, MLP
56 -> 512 -> 512 -> 512 -> 784, in the launch configuration bench.py times.

The oracle computes H_SS, E and grad E at full size (all-pairs H_SS by definition,
torch FP64 autograd); PT2 at full size (3.1e9 pairs) is checked on sampled keys whose
w_a and H_aa the oracle computes one by one.
"""
import functools

import numpy as np
import pytest
import torch

import synth
from tests import problems as P

pytestmark = pytest.mark.gpu

NAME = "m28_7a7b_s100k"


@pytest.fixture(scope="module")
def dnqs():
    import paper_2601_21310_amd as d
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return d


@pytest.fixture(scope="module")
def ctx(dnqs):
    return dnqs.Context(0)


@functools.lru_cache(maxsize=None)
def big(out_scale):
    wl = synth.WORKLOADS[NAME]
    return synth.make_problem(wl, out_scale=out_scale)


@functools.lru_cache(maxsize=None)
def big_hss():
    from oracle import hamiltonian as ham
    p = big(1.0)
    return ham.csr_rows(p.wl.M, p.h, p.eri, p.e_core, p.dets)


@functools.lru_cache(maxsize=None)
def big_energy(out_scale):
    import scipy.sparse as sp

    from oracle import energy
    p = big(out_scale)
    rp, col, val, diag = big_hss()
    n = len(diag)
    H = (sp.csr_matrix((val, col, rp), shape=(n, n)) + sp.diags(diag)).tocsr()
    return energy.energy_and_grad(p.theta, p.wl.widths, p.dets, p.wl.M, p.wl.n_elec, H)


def _gpu(dnqs, ctx, p):
    ctx.set_integrals(p.h, p.eri, p.e_core, p.wl.n_alpha, p.wl.n_beta)
    dets = dnqs.dets_to_device(p.dets)
    theta = torch.from_numpy(p.theta).cuda()
    return dets, theta


def test_fullsize_hss(dnqs, ctx):
    p = big(1.0)
    print("[full] hss", flush=True)
    dets, theta = _gpu(dnqs, ctx, p)
    conn = ctx.build_connections(dets, validate=False)
    rp, col, val, diag = [t.cpu().numpy() for t in conn.export()]
    o_rp, o_col, o_val, o_diag = big_hss()
    assert np.array_equal(rp, o_rp) and np.array_equal(col, o_col)
    assert np.all(np.abs(val - o_val) <= 1e-6 * np.maximum(1.0, np.abs(o_val)))
    big_v = np.abs(o_val) > 1e-5
    assert np.array_equal(np.sign(val[big_v]), np.sign(o_val[big_v]))
    assert np.max(np.abs(diag - o_diag) / np.abs(o_diag)) <= 1e-12
    print(f"  nnz {len(col)}")


def test_fullsize_energy_and_gradient_fp32(dnqs, ctx):
    p = big(1.0)
    print("[full] egrad fp32", flush=True)
    dets, theta = _gpu(dnqs, ctx, p)
    conn = ctx.build_connections(dets, validate=False)
    r = ctx.energy_and_grad(p.wl.widths, theta, conn)
    torch.cuda.synchronize()
    o = big_energy(1.0)
    dE = abs(r["E"].item() - o["E"])
    g = P.rel_l2(r["grad"].double().cpu().numpy(), o["grad"])
    print(f"  E {r['E'].item():.10f} oracle {o['E']:.10f} |dE| {dE:.2e}; grad rel L2 {g:.2e}")
    assert dE <= 1e-6 and g <= 1e-4


@pytest.mark.parametrize("prec", ["MIXED", "SPLIT_BF16"])
@pytest.mark.parametrize("out_scale", [1e-2, 1.0])
def test_fullsize_energy_mixed(dnqs, ctx, prec, out_scale):
    """Split-BF16 network GEMMs: |dE| <= 1e-5 Ha, gradient relative L2 <= 1e-3."""
    p = big(out_scale)
    print(f"[full] egrad {prec} out_scale {out_scale}", flush=True)
    dets, theta = _gpu(dnqs, ctx, p)
    conn = ctx.build_connections(dets, validate=False)
    r = ctx.energy_and_grad(p.wl.widths, theta, conn, precision=getattr(dnqs, prec))
    torch.cuda.synchronize()
    o = big_energy(out_scale)
    dE = abs(r["E"].item() - o["E"])
    g = P.rel_l2(r["grad"].double().cpu().numpy(), o["grad"])
    print(f"  {prec} E {r['E'].item():.10f} oracle {o['E']:.10f} |dE| {dE:.2e}; grad rel L2 {g:.2e}")
    assert dE <= 1e-5 and g <= 1e-3


def test_fullsize_pt2_sampled_keys(dnqs, ctx):
    """w_a and H_aa of sampled external keys against the oracle's one-by-one sums, with
    the GPU's psi passed to both (the reduce-by-key and couplings are what is tested)."""
    from oracle import hamiltonian as ham
    p = big(1.0)
    print("[full] pt2 sampled", flush=True)
    dets, theta = _gpu(dnqs, ctx, p)
    conn = ctx.build_connections(dets, validate=False)
    r = ctx.energy_and_grad(p.wl.widths, theta, conn, want_grad=False)
    mask = (1 << 20) - 1
    out = ctx.pt2(conn, r["logabs"], r["sign"], r["E"], sample_mask=mask, export_cap=300)
    ex = out["export"]
    k = min(int(ex["count"].item()), 300)
    assert k > 50
    keys = dnqs.dets_to_host(ex["keys"][:k])
    la = r["logabs"].cpu().numpy()
    sg = r["sign"].cpu().numpy().astype(np.float64)
    psi = sg * np.exp(la - la.max())          # the scale the export uses
    w_o, haa_o = ham.w_keys(p.wl.M, p.h, p.eri, p.e_core, p.dets, psi, keys)
    w_g = ex["w"][:k].cpu().numpy()
    assert np.max(np.abs(w_g - w_o)) <= 1e-12 * max(1.0, np.max(np.abs(w_o)))
    assert np.max(np.abs(ex["haa"][:k].cpu().numpy() - haa_o)) <= 1e-12 * np.max(np.abs(haa_o))
    for a, b in keys[:50]:
        assert not np.any((p.dets[:, 0] == a) & (p.dets[:, 1] == b)), "exported key lies in S"
    print(f"  {k} sampled keys, max |dw| {np.max(np.abs(w_g - w_o)):.2e}; |P| in sample {out['counts'][1].item()}")
