"""Algorithm 1 of the paper (variational mode): the outer loop of subspace evolution
around the inner loop of parameter optimisation, composed from library calls only.

Per outer iteration k (Sec. 2.4; Algorithm 1):
  1. subspace expansion: the heat-bath-screened perturbative set P_k of psi on V_{k-1}
     (dnqs_heatbath_candidates, Eq. 14) and H_VV (dnqs_build_connections);
  2. inner loop: n_inner steps of energy + gradient (Eqs. 11-12) and AdamW with the
     cosine learning-rate decay (Sec. 3.3), one captured HIP graph replayed;
  3. subspace pruning: amplitudes on T_k = V_{k-1} u P_k and the Top-K selector
     (dnqs_select_topk) give V_k.
After the last iteration: E_var on V, the diagnostic E_diag = lambda_min(H_VV)
(dnqs_lanczos) and Delta E_PT2 (Eq. 13), E_total = E_var + Delta E_PT2.

This module only orders the calls and moves tensors between them; every step of the
computation runs in the library's kernels.
"""
from __future__ import annotations

import numpy as np
import torch

from . import _native as N


def hf_determinant(h, n_alpha: int, n_beta: int) -> np.ndarray:
    """The reference determinant: the n_alpha and n_beta spatial orbitals of lowest h_pp
    (ties to the lower index), as uint64[1, 2]."""
    order = np.argsort(np.diag(np.asarray(h)), kind="stable")
    a = sum(1 << int(p) for p in order[:n_alpha])
    b = sum(1 << int(p) for p in order[:n_beta])
    return np.array([[a, b]], dtype=np.uint64)


def run(ctx: "N.Context", h, eri, e_core, n_alpha: int, n_beta: int, widths, theta0, K: int, n_outer: int,
        n_inner: int, eps_hb: float = 1e-6, lr_max: float = 1e-3, lr_min: float = 5e-5, decay_steps: int = 800,
        weight_decay: float = 1e-2, precision: int = N.FP32, v0=None, slot: int = 0, eps_pt2: float = 0.0,
        log=None) -> dict:
    """Runs Algorithm 1 and returns the final theta, V, energies and the per-iteration
    history.  theta0: float32 tensor on the context's device (copied); v0: the initial
    variational set as uint64[n, 2] (default: the reference determinant)."""
    dev = f"cuda:{ctx.device}"
    ctx.set_integrals(h, eri, e_core, n_alpha, n_beta, slot=slot)
    V = N.dets_to_device(hf_determinant(h, n_alpha, n_beta) if v0 is None else v0, ctx.device)
    theta = theta0.detach().clone().to(dev).contiguous()
    m = torch.zeros_like(theta)
    v = torch.zeros_like(theta)
    step = torch.zeros(1, dtype=torch.int32, device=dev)
    history = []
    for k in range(n_outer):
        # 1. subspace expansion: P_k from psi on V_{k-1}, and H_VV
        conn = ctx.build_connections(V, slot=slot, validate=False)
        r0 = ctx.energy_and_grad(widths, theta, conn, want_grad=False, precision=precision)
        P = ctx.heatbath_candidates(conn, r0["logabs"], r0["sign"], eps_hb)
        # 2. inner loop on H_VV: energy, gradient and AdamW; captured once and replayed when
        # the context has a stream of its own (a graph cannot be captured on the null stream)
        batch = ctx.batch(widths, [slot], [conn], [theta])
        ctx.energy_and_grad_batched(batch, precision=precision)   # plan built outside the capture

        def inner_step():
            ctx.energy_and_grad_batched(batch, precision=precision)
            ctx.adamw_batched(batch, m, v, step, lr_max=lr_max, lr_min=lr_min, decay_steps=decay_steps,
                              weight_decay=weight_decay)

        if ctx.stream:
            ctx.capture_begin()
            inner_step()
            graph = ctx.capture_end()
            for _ in range(n_inner):
                graph.launch()
            graph.free()
        else:
            for _ in range(n_inner):
                inner_step()
        E_inner = float(batch["buffers"][0]["E"].item())   # energy at the last step's parameters
        # 3. subspace pruning: amplitudes on T_k = V u P_k, Top-K
        T = torch.cat([V, P], dim=0)
        la, sg = ctx.amplitudes(widths, theta, T, slot=slot, precision=precision)
        V = ctx.select_topk(T, la, sg, K, slot=slot)
        history.append({"outer": k, "n_v": int(conn.n), "n_p": int(P.shape[0]), "E_inner": E_inner,
                        "n_next": int(V.shape[0])})
        if log:
            log(history[-1])
        conn.free()
    # 4. post-optimisation: E_var, E_diag and PT2 on the final V
    conn = ctx.build_connections(V, slot=slot, validate=False)
    r = ctx.energy_and_grad(widths, theta, conn, want_grad=False, precision=precision)
    lz = ctx.lanczos(conn, max_iter=300, tol=1e-10, want_vec=False)
    pt = ctx.pt2(conn, r["logabs"], r["sign"], r["E"], eps_hb=eps_pt2)
    E_var = float(r["E"].item())
    dE = float(pt["out"][0].item())
    res = {"theta": theta, "V": V, "E_var": E_var, "E_diag": float(lz["E"].item()), "dE_pt2": dE,
           "E_total": E_var + dE, "n_p": int(pt["counts"][1].item()), "history": history}
    conn.free()
    return res
