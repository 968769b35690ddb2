"""Occupied-row form of the orbital output layer.

* the plan is used on a set grown around a reference (the reference orbitals dense, the
  others as per-configuration rows) and not on a full space (every orbital occupied in
  half of it);
* energy, log|psi|, sign and gradient equal those of the full-width layer
  (DNQS_FULL_OUTPUT) up to FP32 summation order, in every precision form;
* repeated calls give the same bits (every sum has a fixed order).
The oracle parity of the occupied-row form is that of the energy and gradient tests,
which run on the same connections.
"""
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


def _setup(dnqs, name):
    p = P.problem(name)
    ctx = dnqs.Context(0)
    ctx.set_integrals(p.h, p.eri, p.e_core, p.wl.n_alpha, p.wl.n_beta)
    conn = ctx.build_connections(dnqs.dets_to_device(p.dets))
    return p, ctx, conn


def test_plan_used_around_a_reference_only(dnqs):
    p, _, conn = _setup(dnqs, "m16_5a5b_s16k")
    nd, ne = conn.output_plan()
    occ = np.zeros(2 * p.wl.M)
    for q in range(p.wl.M):
        occ[q] = np.mean((p.dets[:, 0] >> np.uint64(q)) & np.uint64(1))
        occ[p.wl.M + q] = np.mean((p.dets[:, 1] >> np.uint64(q)) & np.uint64(1))
    dense = occ >= 0.35
    print(f"  m16: {nd} dense orbitals, {ne} sparse rows ({ne / len(p.dets):.2f} per configuration)")
    assert nd == int(dense.sum()) and 0 < nd < 2 * p.wl.M
    assert ne == int(round(occ[~dense].sum() * len(p.dets)))
    _, _, full = _setup(dnqs, "m8_4a4b_full")
    assert full.output_plan() == (-1, 0)


@pytest.mark.parametrize("prec", ["FP32", "MIXED", "SPLIT_BF16"])
def test_split_equals_full_width(dnqs, prec):
    p, ctx, conn = _setup(dnqs, "m16_5a5b_s16k")
    pr = getattr(dnqs, prec)
    theta = torch.from_numpy(p.theta).cuda()
    r_full = ctx.energy_and_grad(p.wl.widths, theta, conn, precision=pr, full_output=True)
    r1 = ctx.energy_and_grad(p.wl.widths, theta, conn, precision=pr)
    r2 = ctx.energy_and_grad(p.wl.widths, theta, conn, precision=pr)
    torch.cuda.synchronize()
    g_full, g1, g2 = (r["grad"].double().cpu().numpy() for r in (r_full, r1, r2))
    dE = abs(r1["E"].item() - r_full["E"].item())
    dg = P.rel_l2(g1, g_full)
    # log|psi| per configuration within twice the elimination bound of the amplitude
    # tests (both sides round), kappa from the oracle's A(x); u of the output layer's form
    from oracle import ansatz
    with torch.no_grad():
        A = ansatz.amplitude_matrices(ansatz.params(p.theta, p.wl.widths, p.wl.n_orb, p.wl.n_elec), p.wl.widths,
                                      p.dets, p.wl.M, p.wl.n_elec).numpy()
    u = 2.0 ** -16 if prec == "SPLIT_BF16" else 2.0 ** -24
    bound = 1e-6 + 4.0 * p.wl.n_elec * u * np.linalg.cond(A)
    dl = np.abs(r1["logabs"].cpu().numpy() - r_full["logabs"].cpu().numpy())
    print(f"  [{prec}] |dE| {dE:.2e}, grad rel {dg:.2e}, |dlog psi| median {np.median(dl):.2e} "
          f"max {dl.max():.2e}, max / bound {np.max(dl / bound):.3f}")
    # FP32 output layer on both sides in FP32 and MIXED; in SPLIT_BF16 the full-width
    # layer is split BF16 and the sparse rows FP32, so the mixed-form bars apply
    bar_e, bar_g = (1e-5, 1e-4) if prec == "SPLIT_BF16" else (1e-6, 1e-5)
    assert dE <= bar_e and dg <= bar_g
    assert np.all(dl <= bound)
    well = bound < 0.1
    assert np.array_equal(r1["sign"].cpu().numpy()[well], r_full["sign"].cpu().numpy()[well])
    assert r1["E"].item() == r2["E"].item() and np.array_equal(g1, g2)
