"""Variational energy and gradient (Eqs. 11-12) in float64, plain torch on the CPU.

Test infrastructure only (see the package docstring).

E(theta) = psi^T H_SS psi / psi^T psi over the variational set S (Eq. 11), with
H_SS from the oracle's Slater-Condon rules (diagonal included).  The gradient is
torch autograd of that expression; Eq. 12 is what it equals.  The global scale of
psi is removed with the (detached) maximum of log|psi|, which leaves E and its
gradient unchanged because E is invariant under psi -> c psi.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import torch

from . import ansatz


def _torch_csr(H: sp.csr_matrix) -> torch.Tensor:
    H = H.tocoo()
    idx = torch.from_numpy(np.vstack([H.row, H.col]).astype(np.int64))
    return torch.sparse_coo_tensor(idx, torch.from_numpy(H.data.astype(np.float64)), H.shape).coalesce()


def scaled_psi(logabs: torch.Tensor, sign: torch.Tensor) -> torch.Tensor:
    return sign * torch.exp(logabs - logabs.detach().max())


def energy_and_grad(theta, widths, dets, M: int, n_elec: int, H: sp.csr_matrix, want_grad=True):
    """Returns dict(E, grad (float64 numpy, flat like theta), psi (scaled), v = H psi,
    norm = psi^T psi, logabs, sign)."""
    parts = ansatz.params(theta, widths, 2 * M, n_elec, requires_grad=want_grad)
    logabs, sign = ansatz.log_amplitudes(parts, widths, dets, M, n_elec)
    psi = scaled_psi(logabs, sign)
    Ht = _torch_csr(H)
    v = torch.sparse.mm(Ht, psi.unsqueeze(1)).squeeze(1)
    norm = psi @ psi
    E = (psi @ v) / norm
    out = {"E": float(E.detach()), "psi": psi.detach().numpy(), "v": v.detach().numpy(),
           "norm": float(norm.detach()), "logabs": logabs.detach().numpy(), "sign": sign.detach().numpy()}
    if want_grad:
        E.backward()
        out["grad"] = parts["_flat"].grad.detach().numpy().copy()
    return out


def energy_of_psi(psi: np.ndarray, H: sp.csr_matrix) -> float:
    psi = np.asarray(psi, dtype=np.float64)
    return float(psi @ (H @ psi) / (psi @ psi))
