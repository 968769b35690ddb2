"""Epstein-Nesbet PT2 correction of Eq. 13 in float64.

Test infrastructure only (see the package docstring).

dE_PT2 = (1/psi^T psi) [ sum_{a in S} (v_a - E psi_a)^2 / (E - H_aa)
                         + sum_{a in P} w_a^2 / (E - H_aa) ],
v = H_SS psi, w_a = sum_{x in S} H_ax psi_x, P = C(S) minus S.

Readings of the paper used here: psi_V is normalised (division by psi^T psi, which
makes dE invariant under psi -> c psi); the sum over P is unscreened; a term whose
numerator is exactly 0 contributes 0 (this removes 0/0 when S = {reference}).
"""
from __future__ import annotations

import numpy as np

from . import hamiltonian as ham


def internal_sum(psi, v, diag, E):
    psi = np.asarray(psi, dtype=np.float64)
    r = np.asarray(v, dtype=np.float64) - E * psi
    den = E - np.asarray(diag, dtype=np.float64)
    num = r * r
    keep = num != 0.0
    return float(np.sum(num[keep] / den[keep]))


def pt2(M, h, eri, ecore, dets, psi, v, diag, E, sample_mask=0, sample_val=0, eps_hb=0.0):
    """Returns dict(dE, internal, external, norm, stats) (internal/external unnormalised).
    eps_hb > 0: the external sum runs over the heat-bath-screened P of Eq. 14 (keys whose
    largest coupling |H_ax psi_x| reaches eps_hb times ||psi||_2)."""
    psi = np.asarray(psi, dtype=np.float64)
    norm = float(psi @ psi)
    internal = internal_sum(psi, v, diag, E)
    external, stats = ham.pt2_external(M, h, eri, ecore, dets, psi, E, sample_mask, sample_val, eps_hb)
    return {"dE": (internal + external) / norm, "internal": internal, "external": external,
            "norm": norm, "stats": stats}
