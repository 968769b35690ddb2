"""Batched geometries: one launch per stage over several problems, AdamW, and HIP-graph
replay of a whole optimisation step.

* batched E and gradient equal the single-problem results (full-width output layer, as
  the batched call computes it) for every geometry, and every geometry's E and
  per-block gradient are compared with the oracle;
* the AdamW update equals torch.optim.AdamW (CPU, FP32) with the same cosine schedule;
* a captured step (energy_and_grad_batched + adamw_batched), replayed several times
  with eager work in between, reproduces the eager sequence bit for bit.
"""
import math

import numpy as np
import pytest
import torch

import synth
from tests import problems as P

pytestmark = pytest.mark.gpu

WL = synth.WORKLOADS["m20_6a6b_curve"]
SIZES = [300, 900, 1500, 129, 2100]


@pytest.fixture(scope="module")
def dnqs():
    import paper_2601_21310_amd as d
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return d


@pytest.fixture(scope="module")
def curve():
    return synth.make_curve(WL, n_geoms=len(SIZES), sizes=SIZES, out_scale=1.0)


@pytest.fixture(scope="module")
def setup(dnqs, curve):
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        ctx = dnqs.Context(0)
        conns = []
        for g, p in enumerate(curve):
            ctx.set_integrals(p.h, p.eri, p.e_core, WL.n_alpha, WL.n_beta, slot=g)
            conns.append(ctx.build_connections(dnqs.dets_to_device(p.dets), slot=g))
    return ctx, conns, stream


@pytest.mark.parametrize("precision", ["fp32", "mixed"])
def test_batched_equals_single(dnqs, curve, setup, precision):
    ctx, conns, stream = setup
    prec = dnqs.FP32 if precision == "fp32" else dnqs.MIXED
    with torch.cuda.stream(stream):
        thetas = [torch.from_numpy(p.theta).cuda() for p in curve]
        batch = ctx.batch(WL.widths, list(range(len(curve))), conns, thetas)
        out = ctx.energy_and_grad_batched(batch, precision=prec)
        single = [ctx.energy_and_grad(WL.widths, thetas[g], conns[g], precision=prec, full_output=True)
                  for g in range(len(curve))]
        stream.synchronize()
    for g in range(len(curve)):
        Eb, Es = out[g]["E"].item(), single[g]["E"].item()
        gb, gs = out[g]["grad"].double().cpu().numpy(), single[g]["grad"].double().cpu().numpy()
        print(f"  [{precision}] geometry {g} n={SIZES[g]}: |dE| {abs(Eb - Es):.2e}, grad rel {P.rel_l2(gb, gs):.2e}")
        assert abs(Eb - Es) <= 1e-9 * max(1.0, abs(Es))
        assert P.rel_l2(gb, gs) <= (1e-6 if precision == "fp32" else 1e-4)


def test_batched_geometry_against_oracle(dnqs, curve, setup):
    import scipy.sparse as sp

    from oracle import energy
    from oracle import hamiltonian as ham
    ctx, conns, stream = setup
    with torch.cuda.stream(stream):
        thetas = [torch.from_numpy(q.theta).cuda() for q in curve]
        batch = ctx.batch(WL.widths, list(range(len(curve))), conns, thetas)
        out = ctx.energy_and_grad_batched(batch)
        stream.synchronize()
    for g, p in enumerate(curve):
        H = ham.hss_sparse(WL.M, p.h, p.eri, p.e_core, p.dets)
        o = energy.energy_and_grad(p.theta, WL.widths, p.dets, WL.M, WL.n_elec, H)
        dE = abs(out[g]["E"].item() - o["E"])
        print(f"  geometry {g} n={SIZES[g]}: |dE| vs oracle {dE:.2e}", flush=True)
        assert dE <= 1e-6
        P.check_grad(out[g]["grad"].double().cpu().numpy(), o["grad"], WL.widths, 1e-4, label=f"grad[{g}]")


def _lr(t, lr_max, lr_min, T):
    tc = min(t, T)
    return lr_min + 0.5 * (lr_max - lr_min) * (1 + math.cos(math.pi * tc / T))


def test_adamw_matches_torch(dnqs, curve, setup):
    ctx, conns, stream = setup
    cfg = dict(lr_max=1e-2, lr_min=1e-3, decay_steps=5, beta1=0.9, beta2=0.999, eps=1e-8, weight_decay=1e-2)
    with torch.cuda.stream(stream):
        thetas = [torch.from_numpy(p.theta).cuda() for p in curve]
        batch = ctx.batch(WL.widths, list(range(len(curve))), conns, thetas)
        np_ = thetas[0].numel()
        m = torch.zeros(len(curve) * np_, device="cuda")
        v = torch.zeros(len(curve) * np_, device="cuda")
        step = torch.zeros(1, dtype=torch.int32, device="cuda")
        ref = [torch.nn.Parameter(torch.from_numpy(p.theta.copy())) for p in curve]
        opt = torch.optim.AdamW(ref, lr=cfg["lr_max"], betas=(cfg["beta1"], cfg["beta2"]), eps=cfg["eps"],
                                weight_decay=cfg["weight_decay"])
        for t in range(1, 8):
            out = ctx.energy_and_grad_batched(batch)
            grads = [o["grad"].cpu() for o in out]
            ctx.adamw_batched(batch, m, v, step, **cfg)
            for group in opt.param_groups:
                group["lr"] = _lr(t, cfg["lr_max"], cfg["lr_min"], cfg["decay_steps"])
            for r, gr in zip(ref, grads):
                r.grad = gr.clone()
            opt.step()
        stream.synchronize()
    assert step.item() == 7
    for g in range(len(curve)):
        d = (batch["buffers"][g]["theta"].cpu() - ref[g].detach()).abs().max().item()
        assert d <= 2e-6, f"geometry {g}: max |dtheta| {d:.2e}"


def test_graph_replay_matches_eager(dnqs, curve, setup):
    ctx, conns, stream = setup
    kw = dict(lr_max=1e-2, lr_min=1e-3, decay_steps=10)
    with torch.cuda.stream(stream):
        ctx.sync_stream()
        runs = []
        for mode in ("eager", "graph"):
            thetas = [torch.from_numpy(p.theta).cuda() for p in curve]
            batch = ctx.batch(WL.widths, list(range(len(curve))), conns, thetas)
            np_ = thetas[0].numel()
            m = torch.zeros(len(curve) * np_, device="cuda")
            v = torch.zeros(len(curve) * np_, device="cuda")
            step = torch.zeros(1, dtype=torch.int32, device="cuda")
            energies = []
            if mode == "eager":
                for _ in range(4):
                    ctx.energy_and_grad_batched(batch)
                    ctx.adamw_batched(batch, m, v, step, **kw)
                    energies.append([b["E"].item() for b in batch["buffers"]])
            else:
                ctx.energy_and_grad_batched(batch)          # plans the batch outside the capture
                ctx.capture_begin()
                ctx.energy_and_grad_batched(batch)
                ctx.adamw_batched(batch, m, v, step, **kw)
                graph = ctx.capture_end()
                for _ in range(4):
                    graph.launch()
                    stream.synchronize()
                    _ = torch.ones(1024, device="cuda").sum().item()   # eager work between replays
                    energies.append([b["E"].item() for b in batch["buffers"]])
                graph.free()
            stream.synchronize()
            runs.append((energies, [b["theta"].cpu().clone() for b in batch["buffers"]], step.item()))
    (e_e, th_e, s_e), (e_g, th_g, s_g) = runs
    assert s_e == s_g == 4
    assert e_e == e_g
    for a, b in zip(th_e, th_g):
        assert torch.equal(a, b)
