"""Neural backflow amplitude, written out from Eqs. 2-4 in float64 (plain torch, CPU).

Test infrastructure only (see the package docstring).

psi(x) = det A(x),  A(x)[j,k] = Phi(x)[i_j, k],  Phi(x) = Phi0 + DeltaPhi(x)   (Eqs. 2-4)

DeltaPhi is an MLP of the occupation bits u(x) in {0,1}^{N_o} (spin-orbital order,
alpha block first): h_1 = tanh(W_1^T u + b_1), h_l = tanh(W_l^T h_{l-1} + b_l),
o = W_L^T h_{L-1} + b_L, DeltaPhi[p,k] = o[p*N_e + k].  The residual mapping of
Sec. 2.2 is read as Phi = Phi0 + DeltaPhi only.  i_1 < ... < i_Ne are the occupied
spin-orbitals of x in ascending order.
"""
from __future__ import annotations

import numpy as np
import torch

import synth


def occupation(dets: np.ndarray, M: int) -> np.ndarray:
    """u(x) as float64 [n, 2M]: bit p of alpha -> column p, bit p of beta -> column M+p."""
    dets = np.asarray(dets, dtype=np.uint64).reshape(-1, 2)
    n = dets.shape[0]
    u = np.zeros((n, 2 * M))
    for p in range(M):
        u[:, p] = ((dets[:, 0] >> np.uint64(p)) & np.uint64(1)).astype(np.float64)
        u[:, M + p] = ((dets[:, 1] >> np.uint64(p)) & np.uint64(1)).astype(np.float64)
    return u


def occupied_rows(u: np.ndarray, n_elec: int) -> np.ndarray:
    """Ascending indices of the occupied spin-orbitals, int64 [n, N_e]."""
    idx = np.argsort(-u, axis=1, kind="stable")[:, :n_elec]
    idx.sort(axis=1)
    assert np.all(u[np.arange(u.shape[0])[:, None], idx] == 1.0), "wrong electron count"
    return idx


def params(theta, widths, n_orb, n_elec, requires_grad=False) -> dict:
    """Split the flat theta into float64 torch tensors (a leaf copy of the float32 values)."""
    t = torch.tensor(np.asarray(theta, dtype=np.float64), dtype=torch.float64, requires_grad=requires_grad)
    lay, _ = synth.param_layout(widths, n_orb, n_elec)
    parts = {name: t[off:off + int(np.prod(shape))].view(*shape) for name, off, shape in lay}
    parts["_flat"] = t
    return parts


def log_amplitudes(parts: dict, widths, dets, M: int, n_elec: int):
    """(log|psi|, sign) for each det, as float64 torch tensors with autograd."""
    u_np = occupation(dets, M)
    occ = torch.from_numpy(occupied_rows(u_np, n_elec))
    u = torch.from_numpy(u_np)
    L = len(widths) - 1
    h = u
    for l in range(1, L):
        h = torch.tanh(h @ parts[f"W{l}"] + parts[f"b{l}"])
    o = h @ parts[f"W{L}"] + parts[f"b{L}"]
    n_orb = 2 * M
    phi = parts["Phi0"].unsqueeze(0) + o.view(-1, n_orb, n_elec)
    A = torch.gather(phi, 1, occ.unsqueeze(-1).expand(-1, -1, n_elec))
    sign, logabs = torch.linalg.slogdet(A)
    return logabs, sign


def amplitude_matrices(parts: dict, widths, dets, M: int, n_elec: int):
    """The occupied submatrices A(x) [n, N_e, N_e] (float64)."""
    u_np = occupation(dets, M)
    occ = torch.from_numpy(occupied_rows(u_np, n_elec))
    u = torch.from_numpy(u_np)
    L = len(widths) - 1
    h = u
    for l in range(1, L):
        h = torch.tanh(h @ parts[f"W{l}"] + parts[f"b{l}"])
    o = h @ parts[f"W{L}"] + parts[f"b{L}"]
    phi = parts["Phi0"].unsqueeze(0) + o.view(-1, 2 * M, n_elec)
    return torch.gather(phi, 1, occ.unsqueeze(-1).expand(-1, -1, n_elec))


def amplitudes(theta, widths, dets, M: int, n_elec: int):
    """numpy (log|psi|, sign) without autograd."""
    with torch.no_grad():
        parts = params(theta, widths, 2 * M, n_elec)
        la, s = log_amplitudes(parts, widths, dets, M, n_elec)
    return la.numpy(), s.numpy()
