"""Seeded parity problems shared by the GPU tests, with their oracle results cached
per process.  Inputs come from synth; expected values come from oracle/ only."""
from __future__ import annotations

import functools

import numpy as np

import synth


@functools.lru_cache(maxsize=None)
def problem(name: str, n_dets: int | None = None, out_scale: float = 1.0, bias_scale: float = 0.1):
    wl = synth.WORKLOADS[name]
    return synth.make_problem(wl, n_dets=n_dets, out_scale=out_scale, bias_scale=bias_scale)


@functools.lru_cache(maxsize=None)
def oracle_hss(name: str, n_dets: int | None = None, out_scale: float = 1.0, bias_scale: float = 0.1):
    from oracle import hamiltonian as ham
    p = problem(name, n_dets, out_scale, bias_scale)
    return ham.csr_rows(p.wl.M, p.h, p.eri, p.e_core, p.dets)


@functools.lru_cache(maxsize=None)
def oracle_energy(name: str, n_dets: int | None = None, out_scale: float = 1.0, bias_scale: float = 0.1):
    import scipy.sparse as sp

    from oracle import energy
    p = problem(name, n_dets, out_scale, bias_scale)
    row_ptr, col, val, diag = oracle_hss(name, n_dets, out_scale, bias_scale)
    n = len(diag)
    H = (sp.csr_matrix((val, col, row_ptr), shape=(n, n)) + sp.diags(diag)).tocsr()
    out = energy.energy_and_grad(p.theta, p.wl.widths, p.dets, p.wl.M, p.wl.n_elec, H)
    out["diag"] = diag
    return out


@functools.lru_cache(maxsize=None)
def oracle_pt2(name: str, n_dets: int | None = None, out_scale: float = 1.0, bias_scale: float = 0.1):
    from oracle import pt2
    p = problem(name, n_dets, out_scale, bias_scale)
    e = oracle_energy(name, n_dets, out_scale, bias_scale)
    return pt2.pt2(p.wl.M, p.h, p.eri, p.e_core, p.dets, e["psi"], e["v"], e["diag"], e["E"])


def rel_l2(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))
