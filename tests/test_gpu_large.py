"""GPU parity on the large-space shape: M = 56 spatial orbitals (112 spin-orbitals),
12 alpha + 12 beta, MLP 112 -> 1024 -> 1024 -> 2688, on a 1500-determinant slice of S.

This covers the code paths that M <= 32 does not reach: 128-bit keys in the PT2
partition and reduce (diagonal from the global J/K tables), N_e = 24 in the LU (32
lanes per matrix), and the widest network.  PT2 is checked on sampled external keys
whose w_a and H_aa the oracle computes one by one.
"""
import functools

import numpy as np
import pytest
import torch

import synth
from tests import problems as P

pytestmark = pytest.mark.gpu

NAME = "m56_12a12b"
N_DETS = 1500


@pytest.fixture(scope="module")
def dnqs():
    import paper_2601_21310_amd as d
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return d


@pytest.fixture(scope="module")
def ctx(dnqs):
    return dnqs.Context(0)


@functools.lru_cache(maxsize=None)
def prob(out_scale):
    return synth.make_problem(synth.WORKLOADS[NAME], n_dets=N_DETS, out_scale=out_scale)


@functools.lru_cache(maxsize=None)
def oracle_hss():
    from oracle import hamiltonian as ham
    p = prob(1.0)
    return ham.csr_rows(p.wl.M, p.h, p.eri, p.e_core, p.dets)


@functools.lru_cache(maxsize=None)
def oracle_energy(out_scale):
    import scipy.sparse as sp

    from oracle import energy
    p = prob(out_scale)
    rp, col, val, diag = oracle_hss()
    n = len(diag)
    H = (sp.csr_matrix((val, col, rp), shape=(n, n)) + sp.diags(diag)).tocsr()
    return energy.energy_and_grad(p.theta, p.wl.widths, p.dets, p.wl.M, p.wl.n_elec, H)


def _gpu(dnqs, ctx, p):
    ctx.set_integrals(p.h, p.eri, p.e_core, p.wl.n_alpha, p.wl.n_beta)
    return dnqs.dets_to_device(p.dets), torch.from_numpy(p.theta).cuda()


def test_large_hss(dnqs, ctx):
    print("[m56] hss", flush=True)
    p = prob(1.0)
    dets, _ = _gpu(dnqs, ctx, p)
    conn = ctx.build_connections(dets)
    rp, col, val, diag = [t.cpu().numpy() for t in conn.export()]
    o_rp, o_col, o_val, o_diag = oracle_hss()
    assert np.array_equal(rp, o_rp) and np.array_equal(col, o_col)
    assert np.all(np.abs(val - o_val) <= 1e-6 * np.maximum(1.0, np.abs(o_val)))
    assert np.max(np.abs(diag - o_diag) / np.abs(o_diag)) <= 1e-12


def test_large_amplitudes(dnqs, ctx):
    print("[m56] amplitudes", flush=True)
    from oracle import ansatz
    p = prob(1.0)
    dets, theta = _gpu(dnqs, ctx, p)
    la, sg = ctx.amplitudes(p.wl.widths, theta, dets)
    ola, osg = ansatz.amplitudes(p.theta, p.wl.widths, p.dets, p.wl.M, p.wl.n_elec)
    with torch.no_grad():
        A = ansatz.amplitude_matrices(ansatz.params(p.theta, p.wl.widths, p.wl.n_orb, p.wl.n_elec), p.wl.widths,
                                      p.dets, p.wl.M, p.wl.n_elec).numpy()
    bound = 1e-6 + 2.0 * p.wl.n_elec * 2.0 ** -24 * np.linalg.cond(A)
    err = np.abs(la.cpu().numpy() - ola)
    print(f"  |dlog psi| median {np.median(err):.2e} max {err.max():.2e}; max err/bound {np.max(err / bound):.3f}")
    assert np.all(err <= bound)
    assert np.array_equal(sg.cpu().numpy(), osg.astype(np.int8))


@pytest.mark.parametrize("prec,bar_e,bar_g", [("FP32", 1e-6, 1e-4), ("MIXED", 1e-5, 1e-3), ("SPLIT_BF16", 1e-5, 1e-3)])
def test_large_energy_and_gradient(dnqs, ctx, prec, bar_e, bar_g):
    print(f"[m56] egrad {prec}", flush=True)
    p = prob(1e-2)
    dets, theta = _gpu(dnqs, ctx, p)
    conn = ctx.build_connections(dets)
    r = ctx.energy_and_grad(p.wl.widths, theta, conn, precision=getattr(dnqs, prec))
    torch.cuda.synchronize()
    o = oracle_energy(1e-2)
    dE = abs(r["E"].item() - o["E"])
    print(f"  E {r['E'].item():.10f} oracle {o['E']:.10f} |dE| {dE:.2e}")
    P.check_grad(r["grad"].double().cpu().numpy(), o["grad"], p.wl.widths, bar_g)
    assert dE <= bar_e


def test_large_pt2_sampled_keys(dnqs, ctx):
    """128-bit keys: w_a and H_aa of sampled external keys against the oracle."""
    print("[m56] pt2 sampled", flush=True)
    from oracle import hamiltonian as ham
    p = prob(1.0)
    dets, theta = _gpu(dnqs, ctx, p)
    conn = ctx.build_connections(dets)
    r = ctx.energy_and_grad(p.wl.widths, theta, conn, want_grad=False)
    out = ctx.pt2(conn, r["logabs"], r["sign"], r["E"], sample_mask=(1 << 16) - 1, export_cap=300)
    ex = out["export"]
    k = min(int(ex["count"].item()), 300)
    assert k > 50
    keys = dnqs.dets_to_host(ex["keys"][:k])
    la = r["logabs"].cpu().numpy()
    psi = r["sign"].cpu().numpy().astype(np.float64) * np.exp(la - la.max())
    w_o, haa_o = ham.w_keys(p.wl.M, p.h, p.eri, p.e_core, p.dets, psi, keys)
    w_g = ex["w"][:k].cpu().numpy()
    assert np.max(np.abs(w_g - w_o)) <= 1e-12 * max(1.0, np.max(np.abs(w_o)))
    assert np.max(np.abs(ex["haa"][:k].cpu().numpy() - haa_o)) <= 1e-12 * np.max(np.abs(haa_o))
    for a, b in keys[:50]:
        assert not np.any((p.dets[:, 0] == a) & (p.dets[:, 1] == b)), "exported key lies in S"
    print(f"  {k} sampled keys, max |dw| {np.max(np.abs(w_g - w_o)):.2e}; pairs {out['counts'][0].item()}")


def test_large_pt2_slicing_and_reproducibility(dnqs, ctx):
    """128-bit keys (6e8 pairs, 2.4e8 keys of P, 1.3e5 sub-buckets): two calls give the
    same bits, and a run cut into key-space slices (16 MiB descriptor budget) has the
    same pair count, |P| and fingerprint, and the same sums up to FP64 summation order."""
    print("[m56] pt2 slicing / reproducibility", flush=True)
    p = prob(1.0)
    dets, theta = _gpu(dnqs, ctx, p)
    conn = ctx.build_connections(dets)
    r = ctx.energy_and_grad(p.wl.widths, theta, conn, want_grad=False)
    a = ctx.pt2(conn, r["logabs"], r["sign"], r["E"])
    b = ctx.pt2(conn, r["logabs"], r["sign"], r["E"])
    assert torch.equal(a["out"].view(torch.int64), b["out"].view(torch.int64))
    assert torch.equal(a["counts"], b["counts"])
    s = ctx.pt2(conn, r["logabs"], r["sign"], r["E"], max_pair_bytes=1 << 24)
    ca, cs = a["counts"].cpu().numpy(), s["counts"].cpu().numpy()
    assert ca[0] == cs[0] and ca[1] == cs[1] and ca[4] == cs[4] and ca[5] == cs[5]
    oa, os_ = a["out"].cpu().numpy(), s["out"].cpu().numpy()
    assert abs(oa[1] - os_[1]) <= 1e-12 * max(1.0, abs(oa[1]))
    assert abs(oa[2] - os_[2]) <= 1e-12 * max(1.0, abs(oa[2]))
    print(f"  |P| {ca[1]}, sub-buckets {ca[3]} (sliced run {cs[3]}), external {oa[2]:.12e} / {os_[2]:.12e}")


def test_large_candidates_capacity(dnqs, ctx):
    """Every (x, a) candidate of the screened set is held once, so |S| n_exc >= 2^31 is
    refused before any launch (n_exc = 404712 at M = 56, 12 + 12 electrons: 6000
    determinants are past the limit)."""
    print("[m56] candidate capacity", flush=True)
    p = synth.make_problem(synth.WORKLOADS[NAME], n_dets=6000)
    dets, theta = _gpu(dnqs, ctx, p)
    conn = ctx.build_connections(dets)
    r = ctx.energy_and_grad(p.wl.widths, theta, conn, want_grad=False)
    with pytest.raises(dnqs.DnqsError, match="ECAPACITY"):
        ctx.heatbath_candidates(conn, r["logabs"], r["sign"], 1e-3)
    # the context stays usable: PT2 on the same set (which streams its pairs) still runs
    out = ctx.pt2(conn, r["logabs"], r["sign"], r["E"])
    assert out["counts"][0].item() == 6000 * 404712
