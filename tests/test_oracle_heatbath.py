"""Pins for the oracle's heat-bath screen (Eq. 14; Sec. 3.2): a determinant a outside S
enters the screened perturbative set when its largest single coupling
max_x |H_ax psi_x| reaches eps_HB, with psi normalised (||psi||_2 = 1; the paper does
not fix the scale, this build reads it as the normalised amplitude).  A kept key keeps
its whole w_a = sum_x H_ax psi_x in Eq. 13.

Checked against dense operator-algebra matrices over the whole sector, with the set and
the sum formed here by brute force (no excitation generation); eps = 0 reduces to the
unscreened definition; the screened sets shrink monotonically as eps grows (CPU only)."""
import numpy as np
import pytest

import synth
from oracle import energy
from oracle import hamiltonian as ham

CASES = [(6, 3, 2, 40, 1), (5, 2, 2, 20, 2), (6, 2, 3, 55, 3)]


def _brute(M, h, eri, ec, S, psi, eps):
    full = synth.full_sector(M, int(bin(int(S[0][0])).count("1")), int(bin(int(S[0][1])).count("1")))
    H = ham.dense_opalg(M, h, eri, ec, full)
    idx = {(int(a), int(b)): i for i, (a, b) in enumerate(full)}
    sidx = np.array([idx[(int(a), int(b))] for a, b in S])
    inS = np.zeros(len(full), dtype=bool)
    inS[sidx] = True
    C = H[:, sidx] * (psi / np.linalg.norm(psi))[None, :]   # normalised couplings H_ax psi_x
    raw = H[:, sidx] * psi[None, :]
    keep = (~inS) & (np.abs(C).max(axis=1) >= eps) & (np.abs(H[:, sidx]).max(axis=1) > 0)
    if eps == 0.0:
        # structural connection (rank <= 2), not numerical: every det at excitation rank 1-2
        keep = (~inS) & np.array([any(2 <= bin(int(a) ^ int(x[0])).count("1") + bin(int(b) ^ int(x[1])).count("1")
                                      <= 4 for x in S) for a, b in full])
    k = np.nonzero(keep)[0]
    return full[k], raw[k].sum(axis=1), np.diag(H)[k]


@pytest.mark.parametrize("M,na,nb,nS,seed", CASES)
@pytest.mark.parametrize("eps", [0.0, 1e-3, 1e-2, 5e-2])
def test_screened_set_and_sum_equal_brute_force(M, na, nb, nS, seed, eps):
    h, eri, _ = synth.make_integrals(M, 2 * M, 300 + seed)
    full = synth.full_sector(M, na, nb)
    rng = np.random.default_rng(seed)
    S = synth.canonical_sort(full[rng.choice(len(full), nS, replace=False)])
    psi = rng.normal(size=len(S)) * np.exp(-3.0 * rng.uniform(size=len(S)))
    keys_b, w_b, haa_b = _brute(M, h, eri, 0.2, S, psi, eps)
    keys, w, haa = ham.pt2_plist(M, h, eri, 0.2, S, psi, eps_hb=eps)
    assert np.array_equal(keys, keys_b)
    assert np.max(np.abs(w - w_b), initial=0.0) <= 1e-12
    Hs = ham.hss_sparse(M, h, eri, 0.2, S)
    E = energy.energy_of_psi(psi, Hs)
    got, st = ham.pt2_external(M, h, eri, 0.2, S, psi, E, eps_hb=eps)
    t = np.where(w_b != 0, w_b * w_b / (E - haa_b), 0.0)
    assert st["n_p"] == len(keys_b)
    assert abs(got - t.sum()) <= 1e-12 * max(1.0, np.abs(t).sum())


def test_screen_monotone_and_scale_free():
    M, na, nb = 6, 3, 3
    h, eri, _ = synth.make_integrals(M, 12, 333)
    full = synth.full_sector(M, na, nb)
    rng = np.random.default_rng(4)
    S = synth.canonical_sort(full[rng.choice(len(full), 60, replace=False)])
    psi = rng.normal(size=len(S))
    prev = None
    for eps in [0.0, 1e-4, 1e-3, 1e-2, 1e-1, 10.0]:
        keys, _, _ = ham.pt2_plist(M, h, eri, 0.0, S, psi, eps_hb=eps)
        cur = {(int(a), int(b)) for a, b in keys}
        if prev is not None:
            assert cur <= prev
        prev = cur
        # psi -> c psi leaves the screened set unchanged (normalised amplitudes)
        keys2, _, _ = ham.pt2_plist(M, h, eri, 0.0, S, 37.5 * psi, eps_hb=eps)
        assert np.array_equal(keys, keys2)
    assert not prev   # eps far above every coupling: nothing kept
