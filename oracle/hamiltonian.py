"""ctypes wrappers around the oracle's C part (sc_oracle.c): Slater-Condon rules,
H_SS by definition, excitation lists, operator-algebra dense H, PT2 external sum.

Test infrastructure only (see the package docstring).
"""
from __future__ import annotations

import ctypes as C

import numpy as np

from . import build_oracle

_lib = None

_dp = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
_u64p = np.ctypeslib.ndpointer(dtype=np.uint64, flags="C_CONTIGUOUS")
_i64p = np.ctypeslib.ndpointer(dtype=np.int64, flags="C_CONTIGUOUS")
_i32p = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")


def _opt(ptr_type):
    """ndpointer that also accepts None."""
    class _P(ptr_type):
        @classmethod
        def from_param(cls, obj):
            if obj is None:
                return None
            return ptr_type.from_param(obj)
    return _P


def lib():
    global _lib
    if _lib is None:
        path = build_oracle.build(force=False)
        L = C.CDLL(path)
        L.or_dense_opalg.argtypes = [C.c_int, _dp, _dp, C.c_double, _u64p, C.c_int64, _dp]
        L.or_dense_opalg.restype = C.c_int
        L.or_dense_sc.argtypes = [C.c_int, _dp, _dp, C.c_double, _u64p, C.c_int64, _dp]
        L.or_dense_sc.restype = C.c_int
        L.or_hdiag.argtypes = [C.c_int, _dp, _dp, C.c_double, C.c_uint64, C.c_uint64]
        L.or_hdiag.restype = C.c_double
        L.or_hxy.argtypes = [C.c_int, _dp, _dp, C.c_double, C.c_uint64, C.c_uint64, C.c_uint64,
                             C.c_uint64]
        L.or_hxy.restype = C.c_double
        L.or_csr_rows.argtypes = [C.c_int, _dp, _dp, C.c_double, _u64p, C.c_int64, _i64p, C.c_int64,
                                  _opt(_i64p), _opt(_i64p), _opt(_i32p), _opt(_dp), _opt(_dp)]
        L.or_csr_rows.restype = C.c_int
        L.or_excitations.argtypes = [C.c_int, C.c_uint64, C.c_uint64, _opt(_u64p), C.c_int64]
        L.or_excitations.restype = C.c_int64
        L.or_pt2_external.argtypes = [C.c_int, _dp, _dp, C.c_double, _u64p, C.c_int64, _dp, C.c_double,
                                      C.c_uint64, C.c_uint64, _i64p, _dp]
        L.or_pt2_external.restype = C.c_double
        L.or_pt2_plist.argtypes = [C.c_int, _dp, _dp, C.c_double, _u64p, C.c_int64, _opt(_dp), _opt(_u64p),
                                   _opt(_dp), _opt(_dp), C.c_int64]
        L.or_pt2_plist.restype = C.c_int64
        L.or_pt2_external_hb.argtypes = [C.c_int, _dp, _dp, C.c_double, _u64p, C.c_int64, _dp, C.c_double,
                                         C.c_uint64, C.c_uint64, C.c_double, _i64p, _dp]
        L.or_pt2_external_hb.restype = C.c_double
        L.or_pt2_plist_hb.argtypes = [C.c_int, _dp, _dp, C.c_double, _u64p, C.c_int64, _opt(_dp), C.c_double,
                                      _opt(_u64p), _opt(_dp), _opt(_dp), C.c_int64]
        L.or_pt2_plist_hb.restype = C.c_int64
        L.or_w_keys.argtypes = [C.c_int, _dp, _dp, C.c_double, _u64p, C.c_int64, _dp, _u64p, C.c_int64,
                                _dp, _opt(_dp)]
        L.or_w_keys.restype = C.c_int
        L.or_key_hash.argtypes = [C.c_uint64, C.c_uint64]
        L.or_key_hash.restype = C.c_uint64
        L.or_num_threads.argtypes = []
        L.or_num_threads.restype = C.c_int
        L.or_set_num_threads.argtypes = [C.c_int]
        L.or_set_num_threads.restype = None
        _lib = L
    return _lib


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _dets(d):
    return np.ascontiguousarray(np.asarray(d, dtype=np.uint64).reshape(-1, 2))


def dense_opalg(M, h, eri, ecore, basis):
    """Dense H over a sorted basis by applying the second-quantised operator."""
    basis = _dets(basis)
    n = basis.shape[0]
    H = np.zeros((n, n))
    rc = lib().or_dense_opalg(M, _f64(h).ravel(), _f64(eri).ravel(), float(ecore), basis.ravel(), n, H)
    if rc != 0:
        raise RuntimeError("operator algebra left the basis (basis is not a full sector)")
    return H


def dense_sc(M, h, eri, ecore, basis):
    """Dense H over a basis by the Slater-Condon rules."""
    basis = _dets(basis)
    n = basis.shape[0]
    H = np.zeros((n, n))
    lib().or_dense_sc(M, _f64(h).ravel(), _f64(eri).ravel(), float(ecore), basis.ravel(), n, H)
    return H


def hdiag(M, h, eri, ecore, det):
    return lib().or_hdiag(M, _f64(h).ravel(), _f64(eri).ravel(), float(ecore), int(det[0]), int(det[1]))


def hxy(M, h, eri, ecore, x, y):
    """<x|H|y>."""
    return lib().or_hxy(M, _f64(h).ravel(), _f64(eri).ravel(), float(ecore), int(x[0]), int(x[1]),
                        int(y[0]), int(y[1]))


def csr_rows(M, h, eri, ecore, dets, rows=None):
    """H_SS rows by definition: returns (row_ptr int64, col int32, val f64, diag f64).

    Columns of each row are every y in S with excitation rank 1 or 2, ascending.
    """
    dets = _dets(dets)
    n = dets.shape[0]
    rows = np.arange(n, dtype=np.int64) if rows is None else np.ascontiguousarray(rows, dtype=np.int64)
    L = lib()
    hf, ef = _f64(h).ravel(), _f64(eri).ravel()
    counts = np.zeros(len(rows), dtype=np.int64)
    L.or_csr_rows(M, hf, ef, float(ecore), dets.ravel(), n, rows, len(rows), counts, None, None, None, None)
    row_ptr = np.zeros(len(rows) + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    nnz = int(row_ptr[-1])
    col = np.zeros(max(nnz, 1), dtype=np.int32)
    val = np.zeros(max(nnz, 1), dtype=np.float64)
    diag = np.zeros(len(rows), dtype=np.float64)
    L.or_csr_rows(M, hf, ef, float(ecore), dets.ravel(), n, rows, len(rows), None, row_ptr[:-1].copy(),
                  col, val, diag)
    return row_ptr, col[:nnz], val[:nnz], diag


def hss_sparse(M, h, eri, ecore, dets):
    """H_SS as a scipy CSR matrix (diagonal included), float64."""
    import scipy.sparse as sp
    row_ptr, col, val, diag = csr_rows(M, h, eri, ecore, dets)
    n = len(diag)
    off = sp.csr_matrix((val, col, row_ptr), shape=(n, n))
    return (off + sp.diags(diag)).tocsr()


def excitations(M, det):
    """All singles and doubles of det as uint64[n, 2] (generation order)."""
    L = lib()
    n = L.or_excitations(M, int(det[0]), int(det[1]), None, 0)
    out = np.zeros(2 * max(n, 1), dtype=np.uint64)
    L.or_excitations(M, int(det[0]), int(det[1]), out, n)
    return out[: 2 * n].reshape(-1, 2)


def key_hash(a, b):
    return int(lib().or_key_hash(int(a), int(b)))


def pt2_external(M, h, eri, ecore, dets, psi, E, sample_mask=0, sample_val=0, eps_hb=0.0):
    """Unnormalised external EN sum over P = C(S) minus S (Eq. 13, second term).

    eps_hb > 0: only the keys a with max_x |H_ax psi_x| >= eps_hb ||psi||_2 (the heat-bath
    screen of Eq. 14 on the normalised psi; each kept key with its whole w_a).
    Returns (sum, stats) with stats: pairs, n_p, n_tiny, min_den; the order-free
    fingerprint of the kept keys fp_sum / fp_xor (sum mod 2^64 and xor of key_hash);
    and first-order sensitivities of the sum (sum_abs = sum |t_a|; sens_rel_c, to a
    relative error in each H_ax psi_x; sens_abs_c, to an absolute error per H_ax psi_x;
    sens_den, to relative errors in E and H_aa).
    """
    dets = _dets(dets)
    psi = _f64(psi)
    si = np.zeros(5, dtype=np.int64)
    sd = np.zeros(5, dtype=np.float64)
    eps_abs = float(eps_hb) * float(np.sqrt(psi @ psi)) if eps_hb > 0 else 0.0
    s = lib().or_pt2_external_hb(M, _f64(h).ravel(), _f64(eri).ravel(), float(ecore), dets.ravel(),
                                 dets.shape[0], psi, float(E), int(sample_mask), int(sample_val), eps_abs, si, sd)
    return s, {"pairs": int(si[0]), "n_p": int(si[1]), "n_tiny": int(si[2]),
               "fp_sum": int(si[3]) & 0xFFFFFFFFFFFFFFFF, "fp_xor": int(si[4]) & 0xFFFFFFFFFFFFFFFF,
               "min_den": float(sd[0]), "sum_abs": float(sd[1]), "sens_rel_c": float(sd[2]),
               "sens_abs_c": float(sd[3]), "sens_den": float(sd[4])}


def pt2_plist(M, h, eri, ecore, dets, psi=None, eps_hb=0.0):
    """P = C(S) minus S written out in canonical order (Eq. 1), with w_a and H_aa when
    psi is given; eps_hb > 0 (psi needed) keeps only the a with max_x |H_ax psi_x| >=
    eps_hb ||psi||_2 (Eq. 14).  Returns (keys uint64[|P|, 2], w, haa) (w, haa None
    without psi)."""
    dets = _dets(dets)
    L = lib()
    hf, ef = _f64(h).ravel(), _f64(eri).ravel()
    p = None if psi is None else _f64(psi)
    eps_abs = float(eps_hb) * float(np.sqrt(p @ p)) if (eps_hb > 0 and p is not None) else 0.0
    n_p = L.or_pt2_plist_hb(M, hf, ef, float(ecore), dets.ravel(), dets.shape[0], p, eps_abs, None, None, None, 0)
    keys = np.zeros(2 * max(n_p, 1), dtype=np.uint64)
    w = np.zeros(max(n_p, 1)) if psi is not None else None
    haa = np.zeros(max(n_p, 1)) if psi is not None else None
    L.or_pt2_plist_hb(M, hf, ef, float(ecore), dets.ravel(), dets.shape[0], p, eps_abs, keys, w, haa, n_p)
    keys = keys[: 2 * n_p].reshape(-1, 2)
    if psi is None:
        return keys, None, None
    return keys, w[:n_p], haa[:n_p]


def w_keys(M, h, eri, ecore, dets, psi, keys):
    """w_a = sum_x H_ax psi_x and H_aa for each key a, computed one by one."""
    dets = _dets(dets)
    keys = _dets(keys)
    k = keys.shape[0]
    w = np.zeros(max(k, 1))
    haa = np.zeros(max(k, 1))
    lib().or_w_keys(M, _f64(h).ravel(), _f64(eri).ravel(), float(ecore), dets.ravel(), dets.shape[0],
                    _f64(psi), keys.ravel(), k, w, haa)
    return w[:k], haa[:k]


def num_threads():
    return int(lib().or_num_threads())


def set_num_threads(k):
    lib().or_set_num_threads(int(k))
