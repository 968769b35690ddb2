"""Pins for the oracle's Hamiltonian, connected set and H_SS (CPU only).

The Slater-Condon rules are checked against brute-force operator algebra (the
dense second-quantised H applied term by term), against closed forms (ERI = 0,
one electron) and against exact excitation counts.
"""
import itertools
import math

import numpy as np
import pytest

import synth
from oracle import fci
from oracle import hamiltonian as ham


def _ints(M, seed, rank=None, ecore=0.0):
    h, eri, _ = synth.make_integrals(M, rank or 2 * M, seed)
    return h, eri, ecore


SECTORS = [(3, 1, 1), (3, 3, 0), (3, 0, 2), (4, 2, 1), (4, 2, 2), (4, 4, 3), (5, 2, 2), (5, 3, 1),
           (4, 0, 0), (6, 3, 3)]


@pytest.mark.parametrize("M,na,nb", SECTORS)
def test_slater_condon_equals_operator_algebra(M, na, nb):
    h, eri, _ = _ints(M, 11 + M + na + 7 * nb)
    ecore = 0.37
    basis = synth.full_sector(M, na, nb)
    H_op = ham.dense_opalg(M, h, eri, ecore, basis)
    H_sc = ham.dense_sc(M, h, eri, ecore, basis)
    assert np.max(np.abs(H_op - H_sc)) <= 1e-12
    assert np.max(np.abs(H_sc - H_sc.T)) <= 1e-12


def test_operator_algebra_general_integrals():
    """Integrals with no low-rank structure (still 8-fold symmetric)."""
    M, na, nb = 4, 2, 2
    rng = np.random.default_rng(5)
    h = rng.normal(size=(M, M))
    h = h + h.T
    eri = synth.symmetrize_eri(rng.normal(size=(M, M, M, M)))
    basis = synth.full_sector(M, na, nb)
    H_op = ham.dense_opalg(M, h, eri, -1.5, basis)
    H_sc = ham.dense_sc(M, h, eri, -1.5, basis)
    assert np.max(np.abs(H_op - H_sc)) <= 1e-12


@pytest.mark.parametrize("M,na,nb", [(5, 2, 2), (6, 3, 2), (6, 1, 4)])
def test_zero_eri_gives_orbital_energy_sum(M, na, nb):
    h, _, _ = _ints(M, 3)
    eri = np.zeros((M,) * 4)
    basis = synth.full_sector(M, na, nb)
    H = ham.dense_sc(M, h, eri, 0.0, basis)
    e_fci, _ = fci.lowest(H)
    eps = np.linalg.eigvalsh(h)
    assert abs(e_fci - (eps[:na].sum() + eps[:nb].sum())) <= 1e-10


def test_one_electron_hamiltonian_is_h():
    M = 6
    h, eri, _ = _ints(M, 4)
    basis = synth.full_sector(M, 1, 0)        # alpha bit p set, p ascending
    H = ham.dense_sc(M, h, eri, 0.0, basis)
    assert np.max(np.abs(H - h)) <= 1e-13
    basis_b = synth.full_sector(M, 0, 1)
    Hb = ham.dense_sc(M, h, eri, 0.0, basis_b)
    assert np.max(np.abs(Hb - h)) <= 1e-13


def _n_exc(M, na, nb):
    s = sum(n * (M - n) for n in (na, nb))
    d = sum(math.comb(n, 2) * math.comb(M - n, 2) for n in (na, nb))
    return s + d + na * (M - na) * nb * (M - nb)


@pytest.mark.parametrize("M,na,nb", [(4, 2, 1), (5, 2, 2), (6, 3, 2), (5, 5, 1), (6, 0, 3)])
def test_excitations_equal_brute_force_rank_filter(M, na, nb):
    basis = synth.full_sector(M, na, nb)
    rng = np.random.default_rng(M * 10 + na)
    for i in rng.choice(len(basis), size=min(6, len(basis)), replace=False):
        x = basis[i]
        ex = ham.excitations(M, x)
        got = {(int(a), int(b)) for a, b in ex}
        assert len(got) == len(ex), "duplicate excitation"
        want = set()
        for y in basis:
            r = (bin(int(x[0]) ^ int(y[0])).count("1") + bin(int(x[1]) ^ int(y[1])).count("1")) // 2
            if r in (1, 2):
                want.add((int(y[0]), int(y[1])))
        assert got == want
        assert len(ex) == _n_exc(M, na, nb)


@pytest.mark.parametrize("M,na,nb,count", [(8, 4, 4, 360), (16, 5, 5, 4235), (28, 7, 7, 30723),
                                           (20, 6, 6, 9954), (56, 12, 12, 404712)])
def test_excitation_counts_closed_form(M, na, nb, count):
    x = (synth.bits(range(na)), synth.bits(range(nb)))
    assert _n_exc(M, na, nb) == count
    L = ham.lib()
    assert L.or_excitations(M, x[0], x[1], None, 0) == count


def test_csr_rows_equal_dense_structure():
    M, na, nb = 6, 3, 2
    h, eri, _ = _ints(M, 9)
    full = synth.full_sector(M, na, nb)
    rng = np.random.default_rng(2)
    S = synth.canonical_sort(full[rng.choice(len(full), size=90, replace=False)])
    H = ham.dense_sc(M, h, eri, 0.2, S)
    row_ptr, col, val, diag = ham.csr_rows(M, h, eri, 0.2, S)
    n = len(S)
    assert np.allclose(diag, np.diag(H), atol=0, rtol=0)
    for i in range(n):
        cols = col[row_ptr[i]:row_ptr[i + 1]]
        assert np.all(np.diff(cols) > 0)
        want = [j for j in range(n) if j != i and
                (bin(int(S[i, 0]) ^ int(S[j, 0])).count("1") + bin(int(S[i, 1]) ^ int(S[j, 1])).count("1")) <= 4]
        assert cols.tolist() == want
        assert np.array_equal(val[row_ptr[i]:row_ptr[i + 1]], H[i, cols])
    # symmetric sparse matrix
    Hs = ham.hss_sparse(M, h, eri, 0.2, S).toarray()
    assert np.max(np.abs(Hs - Hs.T)) <= 1e-14


def test_csr_row_subset_matches_full():
    wl = synth.WORKLOADS["m16_5a5b_s16k"]
    h, eri, _ = synth.make_integrals(wl.M, wl.rank, 1000 + wl.seed)
    ra, rb = synth.reference_occupation(h, wl.n_alpha, wl.n_beta)
    S = synth.sample_dets(wl.M, wl.n_alpha, wl.n_beta, ra, rb, 2000, 7)
    rows = np.array([0, 5, 17, 1999, 1000], dtype=np.int64)
    rp, col, val, diag = ham.csr_rows(wl.M, h, eri, 0.0, S, rows)
    for k, i in enumerate(rows):
        cols = col[rp[k]:rp[k + 1]]
        for c, v in zip(cols, val[rp[k]:rp[k + 1]]):
            assert v == ham.hxy(wl.M, h, eri, 0.0, S[i], S[c])
        assert diag[k] == ham.hdiag(wl.M, h, eri, 0.0, S[i])
