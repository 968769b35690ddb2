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


def grad_blocks(g, want, widths):
    """Relative L2 error of the whole gradient and of each parameter block (W_l, b_l, Phi0),
    a block's error taken against max(|want_block|, 1e-2 |want|): a block whose own
    gradient is tiny next to the whole is judged on the whole's scale."""
    g = np.asarray(g, dtype=np.float64)
    want = np.asarray(want, dtype=np.float64)
    lay, total = synth.param_layout(widths, widths[0], widths[-1] // widths[0])
    assert g.shape == want.shape == (total,)
    floor = 1e-2 * max(np.linalg.norm(want), 1e-300)
    blocks = {}
    for name, off, shape in lay:
        m = int(np.prod(shape))
        d, w = g[off:off + m] - want[off:off + m], want[off:off + m]
        blocks[name] = float(np.linalg.norm(d) / max(np.linalg.norm(w), floor))
    return rel_l2(g, want), blocks


def check_grad(g, want, widths, tol, label="grad"):
    """Asserts the whole gradient within tol (relative L2) and every block within 10 tol
    (grad_blocks); prints the block errors.  Returns the whole's error."""
    tot, blocks = grad_blocks(g, want, widths)
    print(f"  {label} rel L2 {tot:.2e}; blocks " + " ".join(f"{k} {v:.1e}" for k, v in blocks.items()), flush=True)
    assert tot <= tol, f"{label} rel L2 {tot:.3e} > {tol:.0e}"
    bad = {k: v for k, v in blocks.items() if v > 10.0 * tol}
    assert not bad, f"{label} blocks above {10 * tol:.0e}: {bad}"
    return tot
