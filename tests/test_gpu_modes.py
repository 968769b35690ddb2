"""GPU parity of the target-space objectives of Sec. 2.3 on T = [V; P] (dnqs_build_target),
through the C ABI, against the FP64 oracle (oracle/modes.py): the proxy matrix of Eq. 8
(structure bit-exact, FP32 values within 1e-6 max(1, |H|), FP64 diagonal), the Proxy
objective and its gradient (Eqs. 9-10), the Asymmetric objective (Eq. 6) with its exact
gradient and with the Eq. 7 estimator; bars |dE| <= 1e-6 Ha and gradient relative L2
<= 1e-4 as for the variational objective (FP32 network and LU, FP64 reductions)."""
import functools

import numpy as np
import pytest
import torch

from tests import problems as P

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dnqs():
    import paper_2601_21310_amd as d
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return d


@pytest.fixture(scope="module")
def ctx(dnqs):
    return dnqs.Context(0)


CASES = [("m8_4a4b_full", 150, 0.0), ("m16_5a5b_s16k", 200, 1e-3)]


@functools.lru_cache(maxsize=None)
def _oracle_sets(name, n, eps):
    from oracle import hamiltonian as ham
    from oracle import modes
    p = P.problem(name, n)
    psi = P.oracle_energy(name, n)["psi"]
    Pk, _, _ = ham.pt2_plist(p.wl.M, p.h, p.eri, p.e_core, p.dets, psi, eps_hb=eps)
    print(f"  oracle proxy matrix over |V| {len(p.dets)} + |P| {len(Pk)}", flush=True)
    Hp = modes.proxy_matrix(p.wl.M, p.h, p.eri, p.e_core, p.dets, Pk)
    return p, Pk, Hp


def _target(dnqs, ctx, name, n, eps):
    p, Pk, Hp = _oracle_sets(name, n, eps)
    ctx.set_integrals(p.h, p.eri, p.e_core, p.wl.n_alpha, p.wl.n_beta)
    cv = ctx.build_connections(dnqs.dets_to_device(p.dets))
    ct = ctx.build_target(cv, dnqs.dets_to_device(Pk))
    return p, Pk, Hp, cv, ct


@pytest.mark.parametrize("name,n,eps", CASES)
def test_proxy_matrix(dnqs, ctx, name, n, eps):
    p, Pk, Hp, cv, ct = _target(dnqs, ctx, name, n, eps)
    rp, col, val, diag = [t.cpu().numpy() for t in ct.export()]
    Hoff = Hp.copy()
    Hoff.setdiag(0.0)
    Hoff.eliminate_zeros()
    Hoff.sort_indices()
    print(f"  {name}: |V| {len(p.dets)} |P| {len(Pk)} nnz {len(col)}")
    assert ct.n == len(p.dets) + len(Pk)
    assert np.array_equal(rp, Hoff.indptr) and np.array_equal(col, Hoff.indices)
    assert np.all(np.abs(val - Hoff.data) <= 1e-6 * np.maximum(1.0, np.abs(Hoff.data)))
    assert np.max(np.abs(diag - Hp.diagonal()) / np.maximum(1.0, np.abs(Hp.diagonal()))) <= 1e-12


@pytest.mark.parametrize("name,n,eps", CASES)
def test_proxy_energy_and_gradient(dnqs, ctx, name, n, eps):
    from oracle import modes
    p, Pk, Hp, cv, ct = _target(dnqs, ctx, name, n, eps)
    theta = torch.from_numpy(p.theta).cuda()
    r = ctx.energy_and_grad(p.wl.widths, theta, ct)
    torch.cuda.synchronize()
    o = modes.proxy_energy_and_grad(p.theta, p.wl.widths, p.dets, Pk, p.wl.M, p.wl.n_elec, Hp)
    dE = abs(r["E"].item() - o["E"])
    print(f"  proxy {name}: E {r['E'].item():.10f} oracle {o['E']:.10f} |dE| {dE:.2e}")
    P.check_grad(r["grad"].double().cpu().numpy(), o["grad"], p.wl.widths, 1e-4)
    assert dE <= 1e-6


@pytest.mark.parametrize("name,n,eps", CASES)
@pytest.mark.parametrize("mode", ["asym", "asym_estimator"])
def test_asymmetric_energy_and_gradient(dnqs, ctx, name, n, eps, mode):
    from oracle import modes
    p, Pk, Hp, cv, ct = _target(dnqs, ctx, name, n, eps)
    theta = torch.from_numpy(p.theta).cuda()
    r = ctx.energy_and_grad(p.wl.widths, theta, ct, mode=mode)
    torch.cuda.synchronize()
    # the Asymmetric objective reads only the rows of V of H over T, which the proxy
    # matrix holds exactly
    o = modes.asym_energy_and_grads(p.theta, p.wl.widths, p.dets, Pk, p.wl.M, p.wl.n_elec, Hp)
    want = o["grad"] if mode == "asym" else o["grad_est"]
    dE = abs(r["E"].item() - o["E"])
    other = P.rel_l2(r["grad"].double().cpu().numpy(), o["grad_est"] if mode == "asym" else o["grad"])
    print(f"  {mode} {name}: E {r['E'].item():.10f} oracle {o['E']:.10f} |dE| {dE:.2e} "
          f"(vs the other gradient: rel {other:.2e})")
    g = P.check_grad(r["grad"].double().cpu().numpy(), want, p.wl.widths, 1e-4)
    assert dE <= 1e-6
    if len(Pk):
        assert other > 10 * g   # the two gradients are distinguishable at this bar


def test_target_rejects_overlap(dnqs, ctx):
    p = P.problem("m8_4a4b_full", 150)
    ctx.set_integrals(p.h, p.eri, p.e_core, p.wl.n_alpha, p.wl.n_beta)
    cv = ctx.build_connections(dnqs.dets_to_device(p.dets))
    with pytest.raises(dnqs.DnqsError, match="EINVAL"):
        ctx.build_target(cv, dnqs.dets_to_device(p.dets[10:20]))
