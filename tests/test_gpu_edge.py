"""GPU parity on degenerate sectors at M = 8: no alpha electrons (0a+3b: the alpha
excitation classes are empty), a full alpha string (8a+2b: no alpha holes), and one
electron of each spin (1a+1b: no same-spin doubles).  Full sectors (P empty) and partial
S (P non-empty) for the H_SS, the energy and gradient, and PT2 on the ground state."""
import functools

import numpy as np
import pytest
import torch

import synth
from tests import problems as P

pytestmark = pytest.mark.gpu

SECTORS = [(0, 3, 0), (8, 2, 0), (1, 1, 0), (0, 3, 30), (8, 2, 20), (1, 1, 40)]


@pytest.fixture(scope="module")
def dnqs():
    import paper_2601_21310_amd as d
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return d


@pytest.fixture(scope="module")
def ctx(dnqs):
    return dnqs.Context(0)


@functools.lru_cache(maxsize=None)
def prob(na, nb, nd):
    wl = synth.Workload(f"edge_{na}a{nb}b", M=8, n_alpha=na, n_beta=nb, rank=8, hidden=(32, 32), n_dets=nd,
                        seed=90 + na + 10 * nb)
    return synth.make_problem(wl)


@functools.lru_cache(maxsize=None)
def oracle(na, nb, nd):
    import scipy.sparse as sp

    from oracle import energy
    from oracle import hamiltonian as ham
    p = prob(na, nb, nd)
    rp, col, val, diag = ham.csr_rows(p.wl.M, p.h, p.eri, p.e_core, p.dets)
    n = len(diag)
    H = (sp.csr_matrix((val, col, rp), shape=(n, n)) + sp.diags(diag)).tocsr()
    return (rp, col, val, diag), H, energy.energy_and_grad(p.theta, p.wl.widths, p.dets, p.wl.M, p.wl.n_elec, H)


@pytest.mark.parametrize("na,nb,nd", SECTORS)
def test_edge_sector(dnqs, ctx, na, nb, nd):
    print(f"[edge] {na}a+{nb}b n_dets={nd or 'full'}", flush=True)
    from oracle import fci
    from oracle import pt2 as opt2
    p = prob(na, nb, nd)
    (o_rp, o_col, o_val, o_diag), H, o = oracle(na, nb, nd)
    ctx.set_integrals(p.h, p.eri, p.e_core, na, nb)
    dets = dnqs.dets_to_device(p.dets)
    conn = ctx.build_connections(dets)
    rp, col, val, diag = [t.cpu().numpy() for t in conn.export()]
    assert np.array_equal(rp, o_rp) and np.array_equal(col, o_col)
    assert np.all(np.abs(val - o_val) <= 1e-6 * np.maximum(1.0, np.abs(o_val)))
    assert np.max(np.abs(diag - o_diag) / np.maximum(1.0, np.abs(o_diag))) <= 1e-12
    theta = torch.from_numpy(p.theta).cuda()
    r = ctx.energy_and_grad(p.wl.widths, theta, conn)
    torch.cuda.synchronize()
    assert abs(r["E"].item() - o["E"]) <= 1e-6
    P.check_grad(r["grad"].double().cpu().numpy(), o["grad"], p.wl.widths, 1e-4)
    E0, psi = fci.lowest_sparse(H) if H.shape[0] > 2 else fci.lowest(H.toarray())
    op = opt2.pt2(p.wl.M, p.h, p.eri, p.e_core, p.dets, psi, H @ psi, o_diag, E0)
    with np.errstate(divide="ignore"):
        la = torch.from_numpy(np.log(np.abs(psi))).cuda()
    sg = torch.from_numpy(np.sign(psi).astype(np.int8)).cuda()
    out = ctx.pt2(conn, la, sg, torch.tensor([E0], dtype=torch.float64).cuda())
    got = out["out"].cpu().numpy()
    cnt = out["counts"].cpu().numpy()
    print(f"  E {r['E'].item():.10f} oracle {o['E']:.10f}; dE_PT2 {got[0]:.3e} oracle {op['dE']:.3e}; |P| {cnt[1]}")
    assert abs(got[0] - op["dE"]) <= 1e-6
    assert cnt[1] == op["stats"]["n_p"] and cnt[0] == op["stats"]["pairs"]
    if nd == 0:
        assert cnt[1] == 0
