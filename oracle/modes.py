"""The Proxy and Asymmetric objectives of Sec. 2.3 in float64, plain torch on the CPU.

Test infrastructure only (see the package docstring).

Target set T = V followed by P (P outside V, e.g. the connected set of Eq. 1 or its
heat-bath-screened part of Eq. 14).

Proxy mode (Eqs. 8-10): the proxy Hamiltonian keeps every element with a row or column
in V and only the diagonal of the P-P block; E_proxy = psi_T^T H~ psi_T / psi_T^T psi_T,
and its gradient (Eq. 10) is the autograd derivative of that quotient.

Asymmetric mode (Eqs. 6-7): E_asym = sum_{x in V} p_V(x) E_loc(x) with
E_loc(x) = sum_{x' in T} H_xx' psi(x') / psi(x) and p_V(x) = psi(x)^2 / sum_V psi^2,
which is psi_V^T H_VT psi_T / psi_V^T psi_V.  Two gradients: the exact one (autograd of
that quotient, every amplitude of T differentiated; the paper derives it in its
Supporting Information), and the estimator of Eq. 7,
2 sum_{x in V} p_V(x) (E_loc(x) - E_asym) d ln|psi(x)|, formed here by autograd of a
surrogate whose coefficients are held fixed.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import torch

from . import ansatz
from . import hamiltonian as ham
from .energy import _torch_csr, scaled_psi


def coupling_block(M, h, eri, ecore, rows, cols) -> sp.csr_matrix:
    """<r|H|c> for every r in rows and c in cols at excitation rank 1 or 2 (r != c), by the
    Slater-Condon rules; pairs are found by comparing the bit strings (brute force)."""
    rows = np.asarray(rows, dtype=np.uint64).reshape(-1, 2)
    cols = np.asarray(cols, dtype=np.uint64).reshape(-1, 2)

    def popcount(v):
        return np.unpackbits(np.ascontiguousarray(v).view(np.uint8)).reshape(v.shape[0], 64).sum(axis=1)

    ri, ci, val = [], [], []
    for i, (ra, rb) in enumerate(rows):
        da = popcount(cols[:, 0] ^ ra)
        db = popcount(cols[:, 1] ^ rb)
        for j in np.nonzero((da + db >= 2) & (da + db <= 4))[0]:
            ri.append(i)
            ci.append(int(j))
            val.append(ham.hxy(M, h, eri, ecore, rows[i], cols[j]))
    return sp.csr_matrix((np.array(val, dtype=np.float64), (np.array(ri, dtype=np.int64),
                                                            np.array(ci, dtype=np.int64))),
                         shape=(rows.shape[0], cols.shape[0]))


def proxy_matrix(M, h, eri, ecore, V, P) -> sp.csr_matrix:
    """H~ over T = [V; P] (Eq. 8): H_VV, H_VP, H_PV exact; the P-P block diagonal."""
    Hvv = ham.hss_sparse(M, h, eri, ecore, V)
    Hpv = coupling_block(M, h, eri, ecore, P, V)
    dP = np.array([ham.hdiag(M, h, eri, ecore, a) for a in np.asarray(P, dtype=np.uint64).reshape(-1, 2)])
    return sp.bmat([[Hvv, Hpv.T], [Hpv, sp.diags(dP)]], format="csr")


def target_matrix(M, h, eri, ecore, V, P) -> sp.csr_matrix:
    """The full H over T = [V; P] (the exact Rayleigh quotient of the post-optimisation
    analysis, Sec. 2.4)."""
    T = np.concatenate([np.asarray(V, dtype=np.uint64).reshape(-1, 2), np.asarray(P, dtype=np.uint64).reshape(-1, 2)])
    Hoff = coupling_block(M, h, eri, ecore, T, T)
    dT = np.array([ham.hdiag(M, h, eri, ecore, x) for x in T])
    return (Hoff + sp.diags(dT)).tocsr()


def proxy_energy_and_grad(theta, widths, V, P, M, n_elec, Hp: sp.csr_matrix) -> dict:
    """E_proxy and its gradient (Eqs. 9-10) for T = [V; P]."""
    T = np.concatenate([np.asarray(V, dtype=np.uint64).reshape(-1, 2), np.asarray(P, dtype=np.uint64).reshape(-1, 2)])
    parts = ansatz.params(theta, widths, 2 * M, n_elec, requires_grad=True)
    logabs, sign = ansatz.log_amplitudes(parts, widths, T, M, n_elec)
    psi = scaled_psi(logabs, sign)
    v = torch.sparse.mm(_torch_csr(Hp), psi.unsqueeze(1)).squeeze(1)
    E = (psi @ v) / (psi @ psi)
    E.backward()
    return {"E": float(E.detach()), "grad": parts["_flat"].grad.detach().numpy().copy(),
            "psi": psi.detach().numpy()}


def asym_energy_of_psi(psi_t, n_v: int, Ht: sp.csr_matrix) -> float:
    """Eq. 6 for given amplitudes on T = [V; P] (first n_v are V)."""
    psi_t = np.asarray(psi_t, dtype=np.float64)
    hv = Ht[:n_v] @ psi_t
    pv = psi_t[:n_v]
    return float(pv @ hv / (pv @ pv))


def asym_energy_and_grads(theta, widths, V, P, M, n_elec, Ht: sp.csr_matrix) -> dict:
    """E_asym (Eq. 6) with the exact gradient and the estimator of Eq. 7, for T = [V; P];
    Ht is H over T (only its rows in V are used)."""
    nV = np.asarray(V, dtype=np.uint64).reshape(-1, 2).shape[0]
    T = np.concatenate([np.asarray(V, dtype=np.uint64).reshape(-1, 2), np.asarray(P, dtype=np.uint64).reshape(-1, 2)])
    Hvt = _torch_csr(Ht[:nV])

    def energy(parts):
        logabs, sign = ansatz.log_amplitudes(parts, widths, T, M, n_elec)
        psi = scaled_psi(logabs, sign)
        hv = torch.sparse.mm(Hvt, psi.unsqueeze(1)).squeeze(1)     # (H_VT psi_T)_x, x in V
        pv = psi[:nV]
        return (pv @ hv) / (pv @ pv), psi, hv, logabs

    parts = ansatz.params(theta, widths, 2 * M, n_elec, requires_grad=True)
    E, psi, hv, _ = energy(parts)
    E.backward()
    exact = parts["_flat"].grad.detach().numpy().copy()
    # Eq. 7: 2 sum_V p(x) (E_loc(x) - E) d ln|psi(x)|, coefficients held fixed
    parts2 = ansatz.params(theta, widths, 2 * M, n_elec, requires_grad=True)
    logabs2, _ = ansatz.log_amplitudes(parts2, widths, T, M, n_elec)
    with torch.no_grad():
        pv = psi[:nV]
        p = pv * pv / (pv @ pv)
        eloc = hv / pv
        coef = 2.0 * p * (eloc - E)
    (coef @ logabs2[:nV]).backward()
    est = parts2["_flat"].grad.detach().numpy().copy()
    return {"E": float(E.detach()), "grad": exact, "grad_est": est, "psi": psi.detach().numpy(),
            "hv": hv.detach().numpy()}
