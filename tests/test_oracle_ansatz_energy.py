"""Pins for the oracle's backflow amplitude, variational energy, gradient and PT2 (CPU).

psi: Leibniz expansion; zero backflow reproduces the CI coefficients of the Slater
determinant prod_k (sum_p Phi0_pk a+_p)|0> built by operator algebra (this fixes the
row order and sign convention against the Fock-state convention of H); a column
swap flips every sign.
E: zero backflow with a spin-block Phi0 on the full sector equals the closed-form
single-determinant energy from density matrices; E >= E_FCI; psi = eigenvector gives
lambda_min.
grad E: central finite differences; invariance of E under Phi -> Phi G.
PT2: exact eigenvector on the full sector gives 0; S = {ref} gives textbook EN2;
dense brute force over the full sector; invariance under psi -> c psi.
"""
import itertools

import numpy as np
import pytest
import torch

import synth
from oracle import ansatz, energy, fci
from oracle import hamiltonian as ham
from oracle import pt2 as opt2


def _small(M=5, na=2, nb=2, hidden=(12, 10), seed=1, out_scale=1.0, bias_scale=0.3):
    h, eri, _ = synth.make_integrals(M, 2 * M, 100 + seed)
    ra, rb = synth.reference_occupation(h, na, nb)
    widths = (2 * M,) + tuple(hidden) + (2 * M * (na + nb),)
    theta = synth.init_theta(widths, M, na, nb, ra, rb, 200 + seed, 300 + seed, out_scale=out_scale,
                             bias_scale=bias_scale)
    return h, eri, ra, rb, widths, theta


def _leibniz(A):
    n = A.shape[0]
    tot = 0.0
    for perm in itertools.permutations(range(n)):
        inv = sum(1 for i in range(n) for j in range(i + 1, n) if perm[i] > perm[j])
        p = 1.0
        for i in range(n):
            p *= A[i, perm[i]]
        tot += (-1) ** inv * p
    return tot


def test_amplitude_equals_leibniz():
    M, na, nb = 4, 2, 2
    h, eri, ra, rb, widths, theta = _small(M, na, nb)
    dets = synth.full_sector(M, na, nb)
    parts = ansatz.params(theta, widths, 2 * M, na + nb)
    with torch.no_grad():
        A = ansatz.amplitude_matrices(parts, widths, dets, M, na + nb).numpy()
    la, s = ansatz.amplitudes(theta, widths, dets, M, na + nb)
    for i in range(len(dets)):
        ref = _leibniz(A[i])
        assert abs(s[i] * np.exp(la[i]) - ref) <= 1e-12 * max(1.0, abs(ref))


def _apply_orbital_creators(phi, M):
    """prod_k c+_k |0>, c+_k = sum_p phi[p,k] a+_p, applied right to left, as {(a,b): coef}."""
    No, Ne = phi.shape
    state = {0: 1.0}                       # 2M-bit integer, spin-orbital k = bit k
    for k in reversed(range(Ne)):
        new = {}
        for z, c in state.items():
            for p in range(No):
                if (z >> p) & 1:
                    continue
                sign = -1.0 if bin(z & ((1 << p) - 1)).count("1") % 2 else 1.0
                z2 = z | (1 << p)
                new[z2] = new.get(z2, 0.0) + sign * phi[p, k] * c
        state = new
    mask = (1 << M) - 1
    return {(z & mask, z >> M): c for z, c in state.items()}


@pytest.mark.parametrize("M,na,nb", [(4, 2, 2), (4, 3, 1), (5, 2, 1)])
def test_zero_backflow_equals_slater_determinant_ci(M, na, nb):
    h, eri, ra, rb, widths, theta = _small(M, na, nb)
    Ne = na + nb
    lay, _ = synth.param_layout(widths, 2 * M, Ne)
    th = theta.copy()
    rng = np.random.default_rng(4)
    for name, off, shape in lay:
        size = int(np.prod(shape))
        if name in (f"W{len(widths) - 1}", f"b{len(widths) - 1}"):
            th[off:off + size] = 0.0
        if name == "Phi0":
            th[off:off + size] = rng.normal(size=size).astype(np.float32)
    phi0 = synth.unpack_theta(th, widths, 2 * M, Ne)["Phi0"].astype(np.float64)
    ci = _apply_orbital_creators(phi0, M)
    dets = synth.full_sector(M, na, nb)
    la, s = ansatz.amplitudes(th, widths, dets, M, Ne)
    for i, (a, b) in enumerate(dets):
        want = ci.get((int(a), int(b)), 0.0)
        assert abs(s[i] * np.exp(la[i]) - want) <= 1e-12 * max(1.0, abs(want))


def test_column_swap_flips_every_sign():
    M, na, nb = 5, 2, 2
    h, eri, ra, rb, widths, theta = _small(M, na, nb)
    Ne = na + nb
    parts = synth.unpack_theta(theta.astype(np.float64), widths, 2 * M, Ne)
    L = len(widths) - 1
    W = parts[f"W{L}"].reshape(widths[-2], 2 * M, Ne)[:, :, [1, 0, 2, 3]].reshape(widths[-2], -1)
    b = parts[f"b{L}"].reshape(2 * M, Ne)[:, [1, 0, 2, 3]].reshape(-1)
    P0 = parts["Phi0"][:, [1, 0, 2, 3]]
    lay, _ = synth.param_layout(widths, 2 * M, Ne)
    th2 = theta.astype(np.float64).copy()
    for name, off, shape in lay:
        size = int(np.prod(shape))
        if name == f"W{L}":
            th2[off:off + size] = W.ravel()
        elif name == f"b{L}":
            th2[off:off + size] = b.ravel()
        elif name == "Phi0":
            th2[off:off + size] = P0.ravel()
    dets = synth.full_sector(M, na, nb)
    la1, s1 = ansatz.amplitudes(theta.astype(np.float64), widths, dets, M, Ne)
    la2, s2 = ansatz.amplitudes(th2, widths, dets, M, Ne)
    assert np.max(np.abs(la1 - la2)) <= 1e-12
    assert np.all(s1 == -s2)


def _closed_form_energy(h, eri, ecore, Ca, Cb):
    """Single-determinant energy from projectors P^s = C (C^T C)^-1 C^T."""
    def proj(Cs):
        if Cs.shape[1] == 0:
            return np.zeros((h.shape[0],) * 2)
        return Cs @ np.linalg.solve(Cs.T @ Cs, Cs.T)
    Pa, Pb = proj(Ca), proj(Cb)
    P = Pa + Pb
    e = ecore + np.sum(h * Pa) + np.sum(h * Pb)
    e += 0.5 * np.einsum("pqrs,pq,rs->", eri, P, P)
    for Ps in (Pa, Pb):
        e -= 0.5 * np.einsum("pqrs,ps,rq->", eri, Ps, Ps)
    return e


@pytest.mark.parametrize("M,na,nb", [(5, 2, 2), (5, 3, 1), (6, 2, 3)])
def test_zero_backflow_energy_equals_closed_form(M, na, nb):
    h, eri, ra, rb, widths, theta = _small(M, na, nb)
    Ne = na + nb
    ecore = 0.8
    rng = np.random.default_rng(M + na)
    lay, _ = synth.param_layout(widths, 2 * M, Ne)
    th = theta.astype(np.float64).copy()
    Ca = rng.normal(size=(M, na))
    Cb = rng.normal(size=(M, nb))
    phi0 = np.zeros((2 * M, Ne))
    phi0[:M, :na] = Ca
    phi0[M:, na:] = Cb
    for name, off, shape in lay:
        size = int(np.prod(shape))
        if name in (f"W{len(widths) - 1}", f"b{len(widths) - 1}"):
            th[off:off + size] = 0.0
        if name == "Phi0":
            th[off:off + size] = phi0.ravel()
    dets = synth.full_sector(M, na, nb)
    H = ham.hss_sparse(M, h, eri, ecore, dets)
    out = energy.energy_and_grad(th, widths, dets, M, Ne, H, want_grad=False)
    assert abs(out["E"] - _closed_form_energy(h, eri, ecore, Ca, Cb)) <= 1e-11


def test_energy_bounds():
    M, na, nb = 5, 2, 2
    h, eri, ra, rb, widths, theta = _small(M, na, nb)
    dets = synth.full_sector(M, na, nb)
    H = ham.hss_sparse(M, h, eri, 0.0, dets)
    e_fci, vec = fci.lowest(H.toarray())
    out = energy.energy_and_grad(theta, widths, dets, M, na + nb, H, want_grad=False)
    assert out["E"] >= e_fci - 1e-12
    assert abs(energy.energy_of_psi(vec, H) - e_fci) <= 1e-12
    # subset S: E >= lambda_min(H_SS)
    rng = np.random.default_rng(0)
    S = synth.canonical_sort(dets[rng.choice(len(dets), 40, replace=False)])
    Hs = ham.hss_sparse(M, h, eri, 0.0, S)
    e_diag, _ = fci.lowest(Hs.toarray())
    out = energy.energy_and_grad(theta, widths, S, M, na + nb, Hs, want_grad=False)
    assert out["E"] >= e_diag - 1e-12 and e_diag >= e_fci - 1e-12


def test_gradient_central_differences():
    M, na, nb = 5, 2, 2
    h, eri, ra, rb, widths, theta = _small(M, na, nb, hidden=(8, 6))
    dets = synth.full_sector(M, na, nb)
    H = ham.hss_sparse(M, h, eri, 0.0, dets)
    th = theta.astype(np.float64)
    g = energy.energy_and_grad(th, widths, dets, M, na + nb, H)["grad"]
    rng = np.random.default_rng(11)
    step = 1e-5
    for _ in range(16):
        d = rng.normal(size=th.shape)
        d /= np.linalg.norm(d)
        ep = energy.energy_and_grad(th + step * d, widths, dets, M, na + nb, H, want_grad=False)["E"]
        em = energy.energy_and_grad(th - step * d, widths, dets, M, na + nb, H, want_grad=False)["E"]
        fd = (ep - em) / (2 * step)
        assert abs(fd - g @ d) <= 1e-7 * max(1.0, abs(fd))


def right_multiplication_residual(grad, theta, widths, n_orb, n_elec):
    """T_lk = sum g_Phi0[p,k] Phi0[p,l] + sum g_W[h,(p,k)] W[h,(p,l)] + sum g_b[(p,k)] b[(p,l)];
    E(Phi G) = E(Phi) for invertible G makes T vanish.  Returns (max|T|, scale)."""
    L = len(widths) - 1
    gp = synth.unpack_theta(np.asarray(grad, dtype=np.float64), widths, n_orb, n_elec)
    tp = synth.unpack_theta(np.asarray(theta, dtype=np.float64), widths, n_orb, n_elec)
    gW = gp[f"W{L}"].reshape(-1, n_orb, n_elec)
    W = tp[f"W{L}"].reshape(-1, n_orb, n_elec)
    gb = gp[f"b{L}"].reshape(n_orb, n_elec)
    b = tp[f"b{L}"].reshape(n_orb, n_elec)
    T = (np.einsum("pk,pl->lk", gp["Phi0"], tp["Phi0"]) + np.einsum("hpk,hpl->lk", gW, W)
         + np.einsum("pk,pl->lk", gb, b))
    scale = (np.abs(np.einsum("pk,pl->lk", np.abs(gp["Phi0"]), np.abs(tp["Phi0"])))
             + np.einsum("hpk,hpl->lk", np.abs(gW), np.abs(W)) + np.einsum("pk,pl->lk", np.abs(gb), np.abs(b)))
    return float(np.max(np.abs(T))), float(np.max(scale))


def test_gradient_right_multiplication_invariance():
    M, na, nb = 5, 2, 2
    h, eri, ra, rb, widths, theta = _small(M, na, nb)
    dets = synth.full_sector(M, na, nb)
    H = ham.hss_sparse(M, h, eri, 0.0, dets)
    g = energy.energy_and_grad(theta, widths, dets, M, na + nb, H)["grad"]
    t, scale = right_multiplication_residual(g, theta, widths, 2 * M, na + nb)
    assert t <= 1e-12 * max(scale, 1.0)
    # and the check is sharp: dropping the Phi0 gradient breaks it
    lay, _ = synth.param_layout(widths, 2 * M, na + nb)
    g2 = g.copy()
    off = lay[-1][1]
    g2[off:] = 0.0
    t2, _ = right_multiplication_residual(g2, theta, widths, 2 * M, na + nb)
    assert t2 > 1e3 * max(t, 1e-15)


# ------------------------------------------------------------------ PT2
def _dense_pt2(Hfull, full, S, psi_S, E):
    """Brute force over the full sector with the dense H."""
    idx = {(int(a), int(b)): i for i, (a, b) in enumerate(full)}
    sidx = np.array([idx[(int(a), int(b))] for a, b in S])
    w = Hfull[:, sidx] @ psi_S
    inS = np.zeros(len(full), bool)
    inS[sidx] = True
    tot = 0.0
    for a in range(len(full)):
        num = (w[a] - E * psi_S[np.where(sidx == a)[0][0]]) if inS[a] else w[a]
        if num == 0.0:
            continue
        tot += num * num / (E - Hfull[a, a])
    return tot / (psi_S @ psi_S)


def test_pt2_vanishes_on_exact_eigenvector():
    M, na, nb = 5, 2, 2
    h, eri, _ = synth.make_integrals(M, 10, 31)
    full = synth.full_sector(M, na, nb)
    H = ham.hss_sparse(M, h, eri, 0.0, full)
    e, vec = fci.lowest(H.toarray())
    v = H @ vec
    res = opt2.pt2(M, h, eri, 0.0, full, vec, v, H.diagonal(), e)
    assert res["stats"]["n_p"] == 0
    assert abs(res["dE"]) <= 1e-20


def test_pt2_single_reference_is_textbook_en2():
    M, na, nb = 5, 2, 2
    h, eri, _ = synth.make_integrals(M, 10, 32)
    ra, rb = synth.reference_occupation(h, na, nb)
    ref = np.array([[synth.bits(ra), synth.bits(rb)]], dtype=np.uint64)
    full = synth.full_sector(M, na, nb)
    Hf = ham.dense_sc(M, h, eri, 0.0, full)
    i0 = [i for i, (a, b) in enumerate(full) if (a, b) == (ref[0, 0], ref[0, 1])][0]
    e0 = Hf[i0, i0]
    en2 = sum(Hf[a, i0] ** 2 / (e0 - Hf[a, a]) for a in range(len(full)) if a != i0 and Hf[a, i0] != 0)
    Hs = ham.hss_sparse(M, h, eri, 0.0, ref)
    psi = np.array([1.0])
    res = opt2.pt2(M, h, eri, 0.0, ref, psi, Hs @ psi, Hs.diagonal(), e0)
    assert abs(res["dE"] - en2) <= 1e-12 * abs(en2)
    assert res["internal"] == 0.0


@pytest.mark.parametrize("M,na,nb,nS", [(5, 2, 2, 30), (6, 3, 2, 60), (6, 2, 2, 1)])
def test_pt2_equals_dense_brute_force(M, na, nb, nS):
    h, eri, _ = synth.make_integrals(M, 2 * M, 40 + M + nS)
    full = synth.full_sector(M, na, nb)
    rng = np.random.default_rng(nS)
    S = synth.canonical_sort(full[rng.choice(len(full), nS, replace=False)])
    Hf = ham.dense_sc(M, h, eri, 0.1, full)
    Hs = ham.hss_sparse(M, h, eri, 0.1, S)
    psi = rng.normal(size=nS)
    E = energy.energy_of_psi(psi, Hs)
    res = opt2.pt2(M, h, eri, 0.1, S, psi, Hs @ psi, Hs.diagonal(), E)
    want = _dense_pt2(Hf, full, S, psi, E)
    assert abs(res["dE"] - want) <= 1e-11 * max(1.0, abs(want))
    # scale invariance
    res2 = opt2.pt2(M, h, eri, 0.1, S, 3.7 * psi, Hs @ (3.7 * psi), Hs.diagonal(), E)
    assert abs(res2["dE"] - res["dE"]) <= 1e-12 * max(1.0, abs(want))


def test_pt2_sampled_subset_and_w_keys():
    M, na, nb = 6, 3, 2
    h, eri, _ = synth.make_integrals(M, 12, 77)
    full = synth.full_sector(M, na, nb)
    rng = np.random.default_rng(3)
    S = synth.canonical_sort(full[rng.choice(len(full), 25, replace=False)])
    Hf = ham.dense_sc(M, h, eri, 0.0, full)
    Hs = ham.hss_sparse(M, h, eri, 0.0, S)
    psi = rng.normal(size=len(S))
    E = energy.energy_of_psi(psi, Hs)
    idx = {(int(a), int(b)): i for i, (a, b) in enumerate(full)}
    sidx = np.array([idx[(int(a), int(b))] for a, b in S])
    w = Hf[:, sidx] @ psi
    inS = np.zeros(len(full), bool)
    inS[sidx] = True
    mask = 3
    want = 0.0
    keys = []
    for a in range(len(full)):
        if inS[a] or w[a] == 0.0:
            continue
        if ham.key_hash(full[a, 0], full[a, 1]) & mask == 0:
            want += w[a] ** 2 / (E - Hf[a, a])
            keys.append(a)
    got, stats = ham.pt2_external(M, h, eri, 0.0, S, psi, E, mask, 0)
    assert abs(got - want) <= 1e-12 * max(1.0, abs(want))
    assert stats["n_p"] == len(keys)
    wk, haa = ham.w_keys(M, h, eri, 0.0, S, psi, full[keys])
    assert np.max(np.abs(wk - w[keys])) <= 1e-12
    assert np.max(np.abs(haa - np.diag(Hf)[keys])) <= 1e-13
