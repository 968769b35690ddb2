"""Exact diagonalisation of a dense Hamiltonian (numpy eigh), float64.

Test infrastructure only (see the package docstring).  Gives E_FCI on a full sector
and lambda_min(H_SS) = E_diag on a subset (the diagnostic of Sec. 2.4).
"""
from __future__ import annotations

import numpy as np


def lowest(H) -> tuple:
    """(lowest eigenvalue, its eigenvector) of a dense symmetric matrix."""
    H = np.asarray(H.todense() if hasattr(H, "todense") else H, dtype=np.float64)
    w, V = np.linalg.eigh(H)
    return float(w[0]), V[:, 0].copy()


def lowest_sparse(H, tol: float = 1e-13) -> tuple:
    """(lowest eigenvalue, eigenvector) of a sparse symmetric matrix (scipy eigsh,
    Lanczos); dense eigh below 2000 rows."""
    import scipy.sparse.linalg as sla
    if H.shape[0] < 2000:
        return lowest(H)
    w, V = sla.eigsh(H, k=1, which="SA", tol=tol)
    return float(w[0]), V[:, 0].copy()
