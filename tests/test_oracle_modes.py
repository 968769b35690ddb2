"""Pins for the oracle's Proxy (Eqs. 8-10) and Asymmetric (Eqs. 6-7) objectives (CPU).

The proxy and target matrices are checked against dense operator-algebra Hamiltonians
over the whole sector; the objectives against their reductions (P empty: both equal the
variational objective of Eq. 11 and its gradient, Eq. 12), against an exact eigenvector
(every local energy equals the eigenvalue, the Eq. 7 estimator vanishes), and the exact
gradients against central finite differences in FP64."""
import numpy as np
import pytest
import scipy.sparse as sp

import synth
from oracle import energy, modes
from oracle import hamiltonian as ham


def _setup(M=6, na=2, nb=2, nV=25, seed=3, widths=None):
    h, eri, _ = synth.make_integrals(M, 2 * M, 500 + seed)
    full = synth.full_sector(M, na, nb)
    rng = np.random.default_rng(seed)
    V = synth.canonical_sort(full[rng.choice(len(full), nV, replace=False)])
    P, _, _ = ham.pt2_plist(M, h, eri, 0.1, V)
    widths = widths or [2 * M, 16, 16, 2 * M * (na + nb)]
    ra, rb = synth.reference_occupation(h, na, nb)
    theta = synth.init_theta(widths, M, na, nb, ra, rb, 7 + seed, 8 + seed, out_scale=1.0, bias_scale=0.1)
    return h, eri, full, V, P, widths, theta


def test_proxy_and_target_matrices_equal_operator_algebra():
    M, na, nb = 6, 2, 2
    h, eri, full, V, P, _, _ = _setup(M, na, nb)
    T = np.concatenate([V, P])
    Hd = ham.dense_opalg(M, h, eri, 0.1, full)
    idx = {(int(a), int(b)): i for i, (a, b) in enumerate(full)}
    ti = np.array([idx[(int(a), int(b))] for a, b in T])
    want = Hd[np.ix_(ti, ti)]
    assert np.max(np.abs(modes.target_matrix(M, h, eri, 0.1, V, P).toarray() - want)) <= 1e-12
    nV = len(V)
    wp = want.copy()
    pp = wp[nV:, nV:]
    wp[nV:, nV:] = np.diag(np.diag(pp))
    Hp = modes.proxy_matrix(M, h, eri, 0.1, V, P)
    assert np.max(np.abs(Hp.toarray() - wp)) <= 1e-12
    assert abs(Hp - Hp.T).max() == 0.0


def test_empty_p_reduces_to_variational():
    M, na, nb = 6, 2, 2
    h, eri, full, V, P, widths, theta = _setup(M, na, nb)
    Pn = np.zeros((0, 2), dtype=np.uint64)
    Hv = ham.hss_sparse(M, h, eri, 0.1, V)
    o = energy.energy_and_grad(theta, widths, V, M, na + nb, Hv)
    pr = modes.proxy_energy_and_grad(theta, widths, V, Pn, M, na + nb, modes.proxy_matrix(M, h, eri, 0.1, V, Pn))
    asy = modes.asym_energy_and_grads(theta, widths, V, Pn, M, na + nb, modes.target_matrix(M, h, eri, 0.1, V, Pn))
    for r in (pr, asy):
        assert abs(r["E"] - o["E"]) <= 1e-12
        assert np.max(np.abs(r["grad"] - o["grad"])) <= 1e-10
    assert np.max(np.abs(asy["grad_est"] - o["grad"])) <= 1e-10


def test_asymmetric_eigenvector_local_energies():
    M, na, nb = 6, 2, 2
    h, eri, full, V, P, _, _ = _setup(M, na, nb)
    Ht = modes.target_matrix(M, h, eri, 0.1, V, P)
    w, U = np.linalg.eigh(Ht.toarray())
    psi = U[:, 0]
    nV = len(V)
    assert abs(modes.asym_energy_of_psi(psi, nV, Ht) - w[0]) <= 1e-10
    # every local energy equals the eigenvalue: (E_loc(x) - lambda) psi(x) = (H psi - lambda psi)_x = 0
    eloc = (Ht[:nV] @ psi) / psi[:nV]
    assert np.max(np.abs((eloc - w[0]) * psi[:nV])) <= 1e-10


@pytest.mark.parametrize("mode", ["proxy", "asym"])
def test_exact_gradients_equal_finite_differences(mode):
    M, na, nb = 6, 2, 2
    h, eri, full, V, P, widths, theta = _setup(M, na, nb, nV=20, seed=5)
    theta = theta.astype(np.float64)
    if mode == "proxy":
        H = modes.proxy_matrix(M, h, eri, 0.1, V, P)
        f = lambda th: modes.proxy_energy_and_grad(th, widths, V, P, M, na + nb, H)  # noqa: E731
    else:
        H = modes.target_matrix(M, h, eri, 0.1, V, P)
        f = lambda th: modes.asym_energy_and_grads(th, widths, V, P, M, na + nb, H)  # noqa: E731
    g = f(theta)["grad"]
    rng = np.random.default_rng(11)
    for _ in range(6):
        d = rng.normal(size=theta.shape)
        d /= np.linalg.norm(d)
        eps = 1e-5
        fd = (f(theta + eps * d)["E"] - f(theta - eps * d)["E"]) / (2 * eps)
        assert abs(fd - g @ d) <= 1e-7 * max(1.0, abs(fd))


def test_asymmetric_estimator_is_not_the_gradient():
    """With P non-empty the Eq. 7 estimator misses the terms through psi on P: it differs
    from the exact gradient (the non-conservative field the paper describes)."""
    M, na, nb = 6, 2, 2
    h, eri, full, V, P, widths, theta = _setup(M, na, nb, nV=20, seed=6)
    r = modes.asym_energy_and_grads(theta, widths, V, P, M, na + nb, modes.target_matrix(M, h, eri, 0.1, V, P))
    assert np.linalg.norm(r["grad"] - r["grad_est"]) > 1e-3 * np.linalg.norm(r["grad"])
