"""GPU parity: the HIP path through the C ABI against the FP64 oracle.

Bars: connection structure and phases bit-exact; FP32 off-diagonal values within
1e-6 max(1, |H|); FP64 diagonal within 1e-12 relative; signs of psi equal and
log|psi| within 1e-6 + 2 N_e eps32 kappa_2(A) (FP32 elimination bound);
|dE| <= 1e-6 Ha; gradient relative L2 <= 1e-4; PT2 on the H_SS ground state within
1e-6 Ha, |P| exact (random-init psi: bar from the oracle's conditioning).
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


@pytest.fixture(scope="module")
def ctx(dnqs):
    return dnqs.Context(0)


def _setup(dnqs, ctx, name, n_dets=None, slot=0):
    p = P.problem(name, n_dets)
    ctx.set_integrals(p.h, p.eri, p.e_core, p.wl.n_alpha, p.wl.n_beta, slot=slot)
    dets = dnqs.dets_to_device(p.dets)
    theta = torch.from_numpy(p.theta).cuda()
    return p, dets, theta


CASES = [("m8_4a4b_full", None), ("m16_5a5b_s16k", None), ("m16_5a5b_s16k", 777), ("m20_6a6b_curve", 1500)]


@pytest.mark.parametrize("name,n", CASES)
def test_hss_structure_and_values(dnqs, ctx, name, n):
    print(f"[hss] {name} n={n}", flush=True)
    p, dets, theta = _setup(dnqs, ctx, name, n)
    conn = ctx.build_connections(dets)
    row_ptr, col, val, diag = [t.cpu().numpy() for t in conn.export()]
    o_rp, o_col, o_val, o_diag = P.oracle_hss(name, n)
    assert np.array_equal(row_ptr, o_rp), "row pointers differ"
    assert np.array_equal(col, o_col), "column indices differ"
    tol = 1e-6 * np.maximum(1.0, np.abs(o_val))
    assert np.all(np.abs(val - o_val) <= tol), f"max |dH| {np.max(np.abs(val - o_val)):.3e}"
    big = np.abs(o_val) > 1e-5
    assert np.array_equal(np.sign(val[big]), np.sign(o_val[big])), "phase mismatch"
    assert np.max(np.abs(diag - o_diag) / np.maximum(1.0, np.abs(o_diag))) <= 1e-12


def test_hss_deterministic(dnqs, ctx):
    p, dets, theta = _setup(dnqs, ctx, "m16_5a5b_s16k")
    a = [t.cpu() for t in ctx.build_connections(dets).export()]
    b = [t.cpu() for t in ctx.build_connections(dets).export()]
    for x, y in zip(a, b):
        assert torch.equal(x, y)


@pytest.mark.parametrize("name,n", CASES)
def test_amplitudes(dnqs, ctx, name, n):
    print(f"[amp] {name} n={n}", flush=True)
    p, dets, theta = _setup(dnqs, ctx, name, n)
    la, sg = ctx.amplitudes(p.wl.widths, theta, dets)
    from oracle import ansatz
    ola, osg = ansatz.amplitudes(p.theta, p.wl.widths, p.dets, p.wl.M, p.wl.n_elec)
    la, sg = la.cpu().numpy(), sg.cpu().numpy()
    assert np.array_equal(sg, osg.astype(np.int8)), "sign mismatch"
    # FP32 elimination: |d log|det A|| <~ N_e eps32 kappa_2(A) (forward error of LU with
    # partial pivoting); kappa from the oracle's own A(x)
    with torch.no_grad():
        A = ansatz.amplitude_matrices(ansatz.params(p.theta, p.wl.widths, p.wl.n_orb, p.wl.n_elec), p.wl.widths,
                                      p.dets, p.wl.M, p.wl.n_elec).numpy()
    kappa = np.linalg.cond(A)
    bound = 1e-6 + 2.0 * p.wl.n_elec * 2.0 ** -24 * kappa
    err = np.abs(la - ola)
    print(f"  |dlog psi| median {np.median(err):.2e} max {err.max():.2e}; max err/bound {np.max(err / bound):.3f}")
    assert np.all(err <= bound), f"worst |dlog psi| {err[np.argmax(err / bound)]:.3e} > bound"


@pytest.mark.parametrize("name,n", CASES)
def test_energy_and_gradient(dnqs, ctx, name, n):
    print(f"[egrad] {name} n={n}", flush=True)
    p, dets, theta = _setup(dnqs, ctx, name, n)
    conn = ctx.build_connections(dets)
    res = ctx.energy_and_grad(p.wl.widths, theta, conn)
    torch.cuda.synchronize()
    o = P.oracle_energy(name, n)
    E = float(res["E"].item())
    assert abs(E - o["E"]) <= 1e-6, f"E {E:.12f} oracle {o['E']:.12f}"
    g = res["grad"].double().cpu().numpy()
    P.check_grad(g, o["grad"], p.wl.widths, 1e-4)
    st = res["stats"].cpu().numpy()
    assert abs(st[1] - np.max(o["logabs"])) <= 1e-5


def test_energy_deterministic(dnqs, ctx):
    p, dets, theta = _setup(dnqs, ctx, "m16_5a5b_s16k")
    conn = ctx.build_connections(dets)
    r1 = ctx.energy_and_grad(p.wl.widths, theta, conn)
    r2 = ctx.energy_and_grad(p.wl.widths, theta, conn)
    torch.cuda.synchronize()
    assert r1["E"].item() == r2["E"].item()
    assert torch.equal(r1["grad"], r2["grad"])


def test_autograd_function(dnqs, ctx):
    p, dets, theta = _setup(dnqs, ctx, "m8_4a4b_full")
    conn = ctx.build_connections(dets)
    th = theta.clone().requires_grad_(True)
    E = dnqs.DetNQSEnergy.apply(th, ctx, p.wl.widths, conn)
    (2.0 * E).backward()
    o = P.oracle_energy("m8_4a4b_full")
    P.check_grad(th.grad.double().cpu().numpy(), 2.0 * o["grad"], p.wl.widths, 1e-4)


PT2_CASES = [("m8_4a4b_full", None), ("m16_5a5b_s16k", 777), ("m16_5a5b_s16k", None), ("m20_6a6b_curve", 1500)]


@pytest.mark.parametrize("name,n", PT2_CASES)
@pytest.mark.parametrize("max_pair_bytes", [0, 1 << 24])
def test_pt2_kernel_on_ground_state(dnqs, ctx, name, n, max_pair_bytes):
    """The paper evaluates PT2 after convergence: psi = lowest eigenvector of H_SS and
    E = its eigenvalue, given to both sides.  Well conditioned (min |E - H_aa| of a few
    Ha here), so the bar is 1e-6 Ha; |P| and the pair count are exact, and sampled
    w_a agree with the oracle's one-by-one sums.  With a 16 MiB descriptor budget the
    key space is processed in 2 to 128 slices (same bars; every key of P exported once)."""
    print(f"[pt2-gs] {name} n={n} max_pair_bytes={max_pair_bytes}", flush=True)
    import scipy.sparse as sp

    from oracle import fci
    from oracle import hamiltonian as ham
    from oracle import pt2 as opt2
    p, dets, theta = _setup(dnqs, ctx, name, n)
    rp, col, val, diag = P.oracle_hss(name, n)
    H = (sp.csr_matrix((val, col, rp), shape=(len(diag), len(diag))) + sp.diags(diag)).tocsr()
    E0, psi = fci.lowest_sparse(H)
    o = opt2.pt2(p.wl.M, p.h, p.eri, p.e_core, p.dets, psi, H @ psi, diag, E0)
    conn = ctx.build_connections(dets)
    with np.errstate(divide="ignore"):
        la = torch.from_numpy(np.log(np.abs(psi))).cuda()
    sg = torch.from_numpy(np.sign(psi).astype(np.int8)).cuda()
    Et = torch.tensor([E0], dtype=torch.float64).cuda()
    out = ctx.pt2(conn, la, sg, Et, sample_mask=0, export_cap=4096, max_pair_bytes=max_pair_bytes)
    got = out["out"].cpu().numpy()
    cnt = out["counts"].cpu().numpy()
    print(f"  dE_PT2 {got[0]:.10f} oracle {o['dE']:.10f} |d| {abs(got[0] - o['dE']):.2e}; |P| {cnt[1]}; "
          f"sub-buckets {cnt[3]}")
    assert abs(got[0] - o["dE"]) <= 1e-6
    assert cnt[1] == o["stats"]["n_p"] and cnt[0] == o["stats"]["pairs"]
    ex = out["export"]
    k = min(int(ex["count"].item()), 4096)
    assert int(ex["count"].item()) == cnt[1]
    if k:
        keys = dnqs.dets_to_host(ex["keys"][:k])
        assert len({(int(a), int(b)) for a, b in keys}) == k, "a key was exported twice"
        w_o, haa_o = ham.w_keys(p.wl.M, p.h, p.eri, p.e_core, p.dets, psi, keys)
        # exported w_a are for psi scaled to max |psi_x| = 1
        w_g = ex["w"][:k].cpu().numpy() * np.max(np.abs(psi))
        assert np.max(np.abs(w_g - w_o)) <= 1e-12 * max(1.0, np.max(np.abs(w_o)))
        assert np.max(np.abs(ex["haa"][:k].cpu().numpy() - haa_o)) <= 1e-12 * np.max(np.abs(haa_o))


@pytest.mark.parametrize("name,n", [("m8_4a4b_full", None), ("m16_5a5b_s16k", 777)])
def test_pt2_end_to_end_random_init(dnqs, ctx, name, n):
    """Whole chain (amplitudes -> E -> PT2) at random-init psi.  E then lies inside the
    spread of H_aa and the sum is ill-conditioned, so the bar is derived from the
    oracle's own response to FP32-level amplitude noise (relative 1e-6, seeded):
    |d| <= 1e-6 + 20 |PT2(psi (1 + 1e-6 xi)) - PT2(psi)|."""
    print(f"[pt2-e2e] {name} n={n}", flush=True)
    import scipy.sparse as sp

    from oracle import pt2 as opt2
    p, dets, theta = _setup(dnqs, ctx, name, n)
    conn = ctx.build_connections(dets)
    res = ctx.energy_and_grad(p.wl.widths, theta, conn, want_grad=False)
    out = ctx.pt2(conn, res["logabs"], res["sign"], res["E"])
    o = P.oracle_pt2(name, n)
    e = P.oracle_energy(name, n)
    rp, col, val, diag = P.oracle_hss(name, n)
    H = (sp.csr_matrix((val, col, rp), shape=(len(diag), len(diag))) + sp.diags(diag)).tocsr()
    rng = np.random.default_rng(12345)
    psi2 = e["psi"] * (1.0 + 1e-6 * rng.normal(size=e["psi"].shape))
    E2 = float(psi2 @ (H @ psi2) / (psi2 @ psi2))
    o2 = opt2.pt2(p.wl.M, p.h, p.eri, p.e_core, p.dets, psi2, H @ psi2, diag, E2)
    bar = 1e-6 + 20.0 * abs(o2["dE"] - o["dE"])
    got = out["out"].cpu().numpy()
    cnt = out["counts"].cpu().numpy()
    print(f"  dE_PT2 {got[0]:.8f} oracle {o['dE']:.8f} |d| {abs(got[0] - o['dE']):.2e} bar {bar:.2e}")
    assert abs(got[0] - o["dE"]) <= bar
    assert cnt[1] == o["stats"]["n_p"] and cnt[0] == o["stats"]["pairs"]


def test_single_determinant_edge(dnqs, ctx):
    """S = {reference}: empty H_SS, E = H_00, PT2 = textbook EN2."""
    p = P.problem("m16_5a5b_s16k")
    ctx.set_integrals(p.h, p.eri, p.e_core, p.wl.n_alpha, p.wl.n_beta)
    ref = np.array([[synth.bits(p.ref_a), synth.bits(p.ref_b)]], dtype=np.uint64)
    dets = dnqs.dets_to_device(ref)
    theta = torch.from_numpy(p.theta).cuda()
    conn = ctx.build_connections(dets)
    assert conn.nnz == 0
    res = ctx.energy_and_grad(p.wl.widths, theta, conn)
    from oracle import hamiltonian as ham
    from oracle import pt2 as opt2
    h00 = ham.hdiag(p.wl.M, p.h, p.eri, p.e_core, ref[0])
    assert abs(res["E"].item() - h00) <= 1e-10
    assert torch.all(res["grad"] == 0)
    out = ctx.pt2(conn, res["logabs"], res["sign"], res["E"])
    o = opt2.pt2(p.wl.M, p.h, p.eri, p.e_core, ref, np.array([1.0]), np.array([h00]), np.array([h00]), h00)
    assert abs(out["out"][0].item() - o["dE"]) <= 1e-6 * max(1.0, abs(o["dE"]))
    assert out["counts"][1].item() == o["stats"]["n_p"]


def test_invalid_inputs_rejected(dnqs, ctx):
    p = P.problem("m8_4a4b_full")
    ctx.set_integrals(p.h, p.eri, p.e_core, p.wl.n_alpha, p.wl.n_beta)
    bad = p.dets[::-1].copy()  # descending
    with pytest.raises(dnqs.DnqsError, match="EINVAL"):
        ctx.build_connections(dnqs.dets_to_device(bad))
    wrong = p.dets.copy()
    wrong[3, 0] = wrong[3, 0] | np.uint64(1 << 7) | np.uint64(1 << 6) | np.uint64(1)
    with pytest.raises(dnqs.DnqsError, match="EINVAL"):
        ctx.build_connections(dnqs.dets_to_device(synth.canonical_sort(wrong)))
    dup = np.concatenate([p.dets[:5], p.dets[4:10]])
    with pytest.raises(dnqs.DnqsError, match="EINVAL"):
        ctx.build_connections(dnqs.dets_to_device(dup))
    with pytest.raises(dnqs.DnqsError, match="ESTATE"):
        ctx.build_connections(dnqs.dets_to_device(p.dets), slot=5)


def test_domain_errors_rejected(dnqs, ctx):
    """psi = 0 (no finite log|psi|) has no normalised PT2, a zero start vector no Krylov
    space: both are refused, outputs untouched, and the context stays usable."""
    p, dets, theta = _setup(dnqs, ctx, "m8_4a4b_full")
    conn = ctx.build_connections(dets)
    res = ctx.energy_and_grad(p.wl.widths, theta, conn, want_grad=False)
    zero = torch.full((conn.n,), float("-inf"), dtype=torch.float64, device="cuda")
    with pytest.raises(dnqs.DnqsError, match="EDOMAIN"):
        ctx.pt2(conn, zero, res["sign"], res["E"])
    with pytest.raises(dnqs.DnqsError, match="EDOMAIN"):
        ctx.lanczos(conn, start=torch.zeros(conn.n, dtype=torch.float64, device="cuda"))
    nan = torch.full((conn.n,), float("nan"), dtype=torch.float64, device="cuda")
    with pytest.raises(dnqs.DnqsError, match="EDOMAIN"):
        ctx.lanczos(conn, start=nan)
    # the context stays usable: the same calls with valid inputs give the oracle's numbers
    rp, col, val, diag = P.oracle_hss("m8_4a4b_full")
    E0 = np.linalg.eigvalsh(np.diag(diag) + _dense(rp, col, val, len(diag)))[0]
    lz = ctx.lanczos(conn, max_iter=400, tol=1e-10, want_vec=False)
    assert abs(lz["E"].item() - E0) <= 2.0 ** -24 * np.linalg.norm(val) + 1e-9 * max(1.0, abs(E0))
    o = P.oracle_pt2("m8_4a4b_full")
    out = ctx.pt2(conn, res["logabs"], res["sign"], res["E"])
    assert out["counts"][1].item() == o["stats"]["n_p"]


def _dense(rp, col, val, m):
    a = np.zeros((m, m))
    for r in range(m):
        a[r, col[rp[r]:rp[r + 1]]] = val[rp[r]:rp[r + 1]]
    return a


# ------------------------------------------------------------------ mixed precision
# Split-BF16 GEMMs carry a relative error near 2^-16 per product (operands split into
# two BF16 parts, the lo*lo term dropped) against 2^-24 for FP32; the bars below are the
# FP32 ones with that unit roundoff, and |dE| <= 1e-5 Ha for the energy.
U_SPLIT = 2.0 ** -16


@pytest.mark.parametrize("prec", ["MIXED", "SPLIT_BF16"])
@pytest.mark.parametrize("name,n", [("m8_4a4b_full", None), ("m16_5a5b_s16k", None), ("m20_6a6b_curve", 1500)])
def test_mixed_energy_small_backflow(dnqs, ctx, name, n, prec):
    """Split-BF16 network GEMMs (output layer FP32 in MIXED, split too in SPLIT_BF16;
    LU FP32, reductions FP64) in the regime of a small output layer (Delta Phi ~ 1e-2):
    |dE| <= 1e-5 Ha against the FP64 oracle, gradient relative L2 <= 1e-3."""
    p = P.problem(name, n, 1e-2, 0.0)
    ctx.set_integrals(p.h, p.eri, p.e_core, p.wl.n_alpha, p.wl.n_beta)
    dets = dnqs.dets_to_device(p.dets)
    theta = torch.from_numpy(p.theta).cuda()
    conn = ctx.build_connections(dets)
    rm = ctx.energy_and_grad(p.wl.widths, theta, conn, precision=getattr(dnqs, prec))
    torch.cuda.synchronize()
    o = P.oracle_energy(name, n, 1e-2, 0.0)
    dEm = abs(rm["E"].item() - o["E"])
    print(f"  {prec} {name} |dE| {dEm:.2e}")
    P.check_grad(rm["grad"].double().cpu().numpy(), o["grad"], p.wl.widths, 1e-3)
    assert dEm <= 1e-5


@pytest.mark.parametrize("prec", ["MIXED", "SPLIT_BF16"])
def test_mixed_energy_full_backflow(dnqs, ctx, prec):
    """A full-scale random output layer (out_scale 1): the same bars."""
    name = "m16_5a5b_s16k"
    p, dets, theta = _setup(dnqs, ctx, name, None)
    conn = ctx.build_connections(dets)
    rm = ctx.energy_and_grad(p.wl.widths, theta, conn, precision=getattr(dnqs, prec))
    torch.cuda.synchronize()
    o = P.oracle_energy(name, None)
    dEm = abs(rm["E"].item() - o["E"])
    print(f"  {prec} at out_scale 1: |dE| {dEm:.2e} Ha")
    P.check_grad(rm["grad"].double().cpu().numpy(), o["grad"], p.wl.widths, 1e-3)
    assert dEm <= 1e-5


@pytest.mark.parametrize("prec", ["MIXED", "SPLIT_BF16"])
@pytest.mark.parametrize("out_scale", [1e-2, 1.0])
def test_mixed_amplitudes(dnqs, ctx, prec, out_scale):
    """Per configuration |d log|psi|| <= 1e-6 + 2 N_e u kappa_2(A) with u = 2^-16, the
    FP32 bound with the split-BF16 unit roundoff; signs agree wherever that bound is
    below log(2) away from a sign change (all but near-singular A)."""
    p = P.problem("m16_5a5b_s16k", None, out_scale, 0.0 if out_scale < 1 else 0.1)
    ctx.set_integrals(p.h, p.eri, p.e_core, p.wl.n_alpha, p.wl.n_beta)
    dets = dnqs.dets_to_device(p.dets)
    theta = torch.from_numpy(p.theta).cuda()
    la, sg = ctx.amplitudes(p.wl.widths, theta, dets, precision=getattr(dnqs, prec))
    from oracle import ansatz
    ola, osg = ansatz.amplitudes(p.theta, p.wl.widths, p.dets, p.wl.M, p.wl.n_elec)
    with torch.no_grad():
        A = ansatz.amplitude_matrices(ansatz.params(p.theta, p.wl.widths, p.wl.n_orb, p.wl.n_elec), p.wl.widths,
                                      p.dets, p.wl.M, p.wl.n_elec).numpy()
    kappa = np.linalg.cond(A)
    bound = 1e-6 + 2.0 * p.wl.n_elec * U_SPLIT * kappa
    la, sg = la.cpu().numpy(), sg.cpu().numpy()
    err = np.abs(la - ola)
    print(f"  {prec} out_scale {out_scale}: |dlog psi| median {np.median(err):.2e} max {err.max():.2e}; "
          f"max err/bound {np.max(err / bound):.3f}")
    assert np.all(err <= bound)
    safe = bound < np.log(2.0)
    assert np.array_equal(sg[safe], osg.astype(np.int8)[safe])
