"""GPU parity of the outer loop's subspace steps (Algorithm 1, steps 1 and 3) and of the
heat-bath-screened PT2, through the C ABI, against the FP64 oracle; and one small run of
the whole Algorithm 1 on the device.

The heat-bath decisions compare |H_ax psi_x| with eps_HB ||psi|| in FP64 on both sides,
with the same FP64 psi given to both; the Top-K selection is given the same FP64 log|psi|
on both sides, so both selections are compared bit for bit."""
import numpy as np
import pytest
import scipy.sparse as sp
import torch

from tests import problems as P

pytestmark = pytest.mark.gpu

U64 = 2.0 ** -53


@pytest.fixture(scope="module")
def dnqs():
    import paper_2601_21310_amd as d
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return d


@pytest.fixture(scope="module")
def ctx(dnqs):
    return dnqs.Context(0)


def _psi_args(psi):
    with np.errstate(divide="ignore"):
        la = torch.from_numpy(np.log(np.abs(psi))).cuda()
    return la, torch.from_numpy(np.sign(psi).astype(np.int8)).cuda()


@pytest.mark.parametrize("name,n", [("m16_5a5b_s16k", 777), ("m20_6a6b_curve", 1500)])
@pytest.mark.parametrize("eps", [0.0, 1e-5, 1e-3])
def test_heatbath_candidates_equal_oracle(dnqs, ctx, name, n, eps):
    from oracle import hamiltonian as ham
    p = P.problem(name, n)
    ctx.set_integrals(p.h, p.eri, p.e_core, p.wl.n_alpha, p.wl.n_beta)
    conn = ctx.build_connections(dnqs.dets_to_device(p.dets))
    psi = P.oracle_energy(name, n)["psi"]
    la, sg = _psi_args(psi)
    got = dnqs.dets_to_host(ctx.heatbath_candidates(conn, la, sg, eps))
    want, _, _ = ham.pt2_plist(p.wl.M, p.h, p.eri, p.e_core, p.dets, psi, eps_hb=eps)
    print(f"  {name} eps {eps}: |P_eps| {len(got)} (oracle {len(want)})")
    assert np.array_equal(got, want)


@pytest.mark.parametrize("K", [1, 333, 5000, 20000])
def test_select_topk_equals_sort(dnqs, ctx, K):
    p = P.problem("m16_5a5b_s16k", None)
    ctx.set_integrals(p.h, p.eri, p.e_core, p.wl.n_alpha, p.wl.n_beta)
    rng = np.random.default_rng(K)
    dets = p.dets[rng.permutation(len(p.dets))]          # any order
    la = rng.normal(size=len(dets))
    la[rng.choice(len(dets), 300, replace=False)] = 0.25  # ties: broken by the lower determinant
    sg = np.where(rng.uniform(size=len(dets)) < 0.02, 0, 1).astype(np.int8)  # sign 0: smallest
    got = dnqs.dets_to_host(ctx.select_topk(dnqs.dets_to_device(dets), torch.from_numpy(la).cuda(),
                                            torch.from_numpy(sg).cuda(), K))
    key = np.where(sg == 0, -np.inf, la)
    order = np.lexsort((dets[:, 1], dets[:, 0], -key))
    want = dets[order[:min(K, len(dets))]]
    want = want[np.lexsort((want[:, 1], want[:, 0]))]
    assert np.array_equal(got, want)


@pytest.mark.parametrize("eps", [1e-5, 1e-4, 1e-3])
def test_pt2_heatbath_screened(dnqs, ctx, eps):
    """PT2 over the screened P of Eq. 14 (each kept key with its whole w_a) against the
    oracle's screened sum: |P_eps| and the fingerprint exact, the sum within 64 u times its
    first-order sensitivities."""
    from oracle import pt2 as opt2
    name, n = "m16_5a5b_s16k", None
    p = P.problem(name, n)
    ctx.set_integrals(p.h, p.eri, p.e_core, p.wl.n_alpha, p.wl.n_beta)
    conn = ctx.build_connections(dnqs.dets_to_device(p.dets))
    e = P.oracle_energy(name, n)
    psi, E = e["psi"], float(e["E"])
    rp, col, val, diag = P.oracle_hss(name, n)
    H = (sp.csr_matrix((val, col, rp), shape=(len(diag), len(diag))) + sp.diags(diag)).tocsr()
    o = opt2.pt2(p.wl.M, p.h, p.eri, p.e_core, p.dets, psi, H @ psi, diag, E, eps_hb=eps)
    la, sg = _psi_args(psi)
    out = ctx.pt2(conn, la, sg, torch.tensor([E], dtype=torch.float64).cuda(), eps_hb=eps)
    got = out["out"].cpu().numpy()
    cnt = out["counts"].cpu().numpy()
    st = o["stats"]
    bar = 64.0 * U64 * (st["sens_rel_c"] + st["sens_den"] + st["sum_abs"])
    print(f"  eps {eps}: |P_eps| {cnt[1]} (oracle {st['n_p']}); external {got[2]:.12e} oracle {o['external']:.12e}")
    assert cnt[1] == st["n_p"]
    assert (int(cnt[4]) & ((1 << 64) - 1)) == st["fp_sum"] and (int(cnt[5]) & ((1 << 64) - 1)) == st["fp_xor"]
    assert abs(got[2] - o["external"]) <= bar


def test_algorithm1_small(dnqs):
    """Algorithm 1 end to end on the 4900-determinant sector (M = 8, 4+4): three outer
    iterations of 150 inner steps, Top-K with K = 300, eps_HB = 1e-5.  The variational
    energies are bounded by the exact ground state, E_diag by E_var, and the run lowers
    the energy below the reference determinant's."""
    from oracle import fci
    from oracle import hamiltonian as ham
    from paper_2601_21310_amd import algorithm1
    p = P.problem("m8_4a4b_full", None, 1e-2, 0.0)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        ctx = dnqs.Context(0)
        res = algorithm1.run(ctx, p.h, p.eri, p.e_core, p.wl.n_alpha, p.wl.n_beta, p.wl.widths,
                             torch.from_numpy(p.theta).cuda(), K=300, n_outer=3, n_inner=150, eps_hb=1e-5,
                             lr_max=3e-3, decay_steps=400)
        stream.synchronize()
    Hf = ham.dense_sc(p.wl.M, p.h, p.eri, p.e_core, p.dets)
    e_fci, _ = fci.lowest(Hf)
    ref = algorithm1.hf_determinant(p.h, p.wl.n_alpha, p.wl.n_beta)[0]
    e_hf = ham.hdiag(p.wl.M, p.h, p.eri, p.e_core, ref)
    print(f"  E_HF {e_hf:.8f} E_var {res['E_var']:.8f} E_diag {res['E_diag']:.8f} E_total {res['E_total']:.8f} "
          f"E_FCI {e_fci:.8f}; history {res['history']}")
    assert res["V"].shape[0] == 300
    V = dnqs.dets_to_host(res["V"])
    assert np.all((V[1:, 0] > V[:-1, 0]) | ((V[1:, 0] == V[:-1, 0]) & (V[1:, 1] > V[:-1, 1])))
    assert res["E_var"] >= e_fci - 1e-6
    assert res["E_diag"] <= res["E_var"] + 1e-6 and res["E_diag"] >= e_fci - 1e-6
    assert res["E_var"] < e_hf - 1e-3
    assert [h["n_v"] for h in res["history"]][0] == 1
