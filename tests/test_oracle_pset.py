"""Pins for the oracle's listing of P = C(S) minus S (Eq. 1) and for the order-free
fingerprint and error sensitivities its external PT2 sum reports (CPU only).

P is checked against a brute-force filter over the whole sector (excitation rank from
popcounts, not from excitation generation); w_a and H_aa against the dense
Slater-Condon and operator-algebra matrices; the fingerprint against SplitMix64
written out here from its published definition.
"""
import numpy as np
import pytest

import synth
from oracle import energy
from oracle import hamiltonian as ham

MASK64 = (1 << 64) - 1


def _mix64(z):
    """SplitMix64 output function (Steele, Lea and Flood 2014)."""
    z &= MASK64
    z ^= z >> 30
    z = (z * 0xBF58476D1CE4E5B9) & MASK64
    z ^= z >> 27
    z = (z * 0x94D049BB133111EB) & MASK64
    z ^= z >> 31
    return z


def _key_hash(a, b):
    return _mix64(int(a) ^ _mix64(int(b)))


def _brute_p(full, S):
    """Every det of the sector at excitation rank 1 or 2 from some member of S, not in S."""
    sset = {(int(a), int(b)) for a, b in S}
    out = []
    for a, b in full:
        if (int(a), int(b)) in sset:
            continue
        for x in S:
            r = bin(int(a) ^ int(x[0])).count("1") + bin(int(b) ^ int(x[1])).count("1")
            if 2 <= r <= 4:
                out.append((int(a), int(b)))
                break
    return sorted(out)


CASES = [(5, 2, 2, 30, 1), (6, 3, 2, 60, 2), (6, 2, 2, 1, 3), (6, 0, 3, 7, 4), (5, 5, 1, 2, 5),
         (4, 2, 2, 36, 6)]


@pytest.mark.parametrize("M,na,nb,nS,seed", CASES)
def test_plist_equals_brute_force_sector_filter(M, na, nb, nS, seed):
    h, eri, _ = synth.make_integrals(M, 2 * M, 60 + seed)
    full = synth.full_sector(M, na, nb)
    rng = np.random.default_rng(seed)
    S = synth.canonical_sort(full[rng.choice(len(full), min(nS, len(full)), replace=False)])
    keys, w, haa = ham.pt2_plist(M, h, eri, 0.3, S)
    assert w is None and haa is None
    got = [(int(a), int(b)) for a, b in keys]
    assert got == _brute_p(full, S)          # same set, canonical order, no repeats
    if nS >= len(full):
        assert len(got) == 0


@pytest.mark.parametrize("M,na,nb,nS,seed", CASES[:3])
def test_plist_values_equal_dense_matrices(M, na, nb, nS, seed):
    h, eri, _ = synth.make_integrals(M, 2 * M, 70 + seed)
    full = synth.full_sector(M, na, nb)
    rng = np.random.default_rng(seed + 10)
    S = synth.canonical_sort(full[rng.choice(len(full), nS, replace=False)])
    psi = rng.normal(size=len(S))
    keys, w, haa = ham.pt2_plist(M, h, eri, -0.4, S, psi)
    Hop = ham.dense_opalg(M, h, eri, -0.4, full)       # operator algebra, not Slater-Condon
    idx = {(int(a), int(b)): i for i, (a, b) in enumerate(full)}
    sidx = np.array([idx[(int(a), int(b))] for a, b in S])
    kidx = np.array([idx[(int(a), int(b))] for a, b in keys], dtype=np.int64)
    assert np.max(np.abs(w - Hop[kidx][:, sidx] @ psi)) <= 1e-12
    assert np.max(np.abs(haa - np.diag(Hop)[kidx])) <= 1e-12


@pytest.mark.parametrize("mask", [0, 3])
def test_external_fingerprint_and_sensitivities(mask):
    M, na, nb = 6, 3, 2
    h, eri, _ = synth.make_integrals(M, 12, 91)
    full = synth.full_sector(M, na, nb)
    rng = np.random.default_rng(8)
    S = synth.canonical_sort(full[rng.choice(len(full), 40, replace=False)])
    Hs = ham.hss_sparse(M, h, eri, 0.0, S)
    psi = rng.normal(size=len(S))
    E = energy.energy_of_psi(psi, Hs)
    Hf = ham.dense_sc(M, h, eri, 0.0, full)
    idx = {(int(a), int(b)): i for i, (a, b) in enumerate(full)}
    sidx = np.array([idx[(int(a), int(b))] for a, b in S])
    P = _brute_p(full, S)
    kept = [k for k in P if _key_hash(*k) & mask == 0]
    fsum, fxor = 0, 0
    for k in kept:
        hk = _key_hash(*k)
        fsum = (fsum + hk) & MASK64
        fxor ^= hk
    got, st = ham.pt2_external(M, h, eri, 0.0, S, psi, E, mask, 0)
    assert st["n_p"] == len(kept)
    assert st["fp_sum"] == fsum and st["fp_xor"] == fxor
    kidx = np.array([idx[k] for k in kept])
    contrib = Hf[kidx][:, sidx] * psi[None, :]       # H_ax psi_x
    w = contrib.sum(axis=1)
    den = E - np.diag(Hf)[kidx]
    t = w * w / den
    assert abs(got - t.sum()) <= 1e-12 * np.abs(t).sum()
    assert abs(st["sum_abs"] - np.abs(t).sum()) <= 1e-12 * np.abs(t).sum()
    c = np.abs(contrib).sum(axis=1)
    nk = (contrib != 0.0).sum(axis=1)
    assert abs(st["sens_rel_c"] - np.sum(2 * np.abs(w) * c / np.abs(den))) <= 1e-10 * st["sens_rel_c"]
    assert abs(st["sens_abs_c"] - np.sum(2 * np.abs(w) * nk / np.abs(den))) <= 1e-10 * st["sens_abs_c"]
    want_den = np.sum(np.abs(t) * (abs(E) + np.abs(np.diag(Hf)[kidx])) / np.abs(den))
    assert abs(st["sens_den"] - want_den) <= 1e-10 * want_den
