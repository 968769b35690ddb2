"""Benchmark of the deterministic-NQS hot path on one MI355X.

A step is one pass of the whole hot path over the workload's variational set S:
build_connections (H_SS), energy_and_grad (amplitudes, E, gradient), pt2.
Default workload: M = 28 spatial orbitals, 7 alpha + 7 beta electrons, |S| = 1e5,
MLP 56 -> 512 -> 512 -> 512 -> 784, lattice-decaying synthetic integrals.

Prints one JSON line:
  value          amps+grads/s = |S| / mean device time of energy_and_grad
  phases         per-phase device times (HIP events on the library stream) and the
                 H-element and PT2-pair rates
  roofline       the dominant kernel against its roofline
  cpu_baseline   the FP64 oracle on a bounded sample of the same workload
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP32_PEAK_TFLOPS = 157.3
BF16_PEAK_TFLOPS = 2500.0


def n_excitations(M, na, nb):
    c2 = lambda k: k * (k - 1) // 2  # noqa: E731
    sa, sb = na * (M - na), nb * (M - nb)
    return sa + sb + c2(na) * c2(M - na) + c2(nb) * c2(M - nb) + sa * sb


def cpu_baseline(p, sample_n: int):
    """Time the oracle (as it stands) on the first sample_n dets of S: H_SS by its
    definition, amplitudes + energy + gradient in FP64, and the PT2 external sum."""
    import numpy as np
    import scipy.sparse as sp

    from oracle import energy
    from oracle import hamiltonian as ham
    from oracle import pt2 as opt2
    wl = p.wl
    S = p.dets[:sample_n]
    t0 = time.perf_counter()
    row_ptr, col, val, diag = ham.csr_rows(wl.M, p.h, p.eri, p.e_core, S)
    t1 = time.perf_counter()
    H = (sp.csr_matrix((val, col, row_ptr), shape=(len(S), len(S))) + sp.diags(diag)).tocsr()
    o = energy.energy_and_grad(p.theta, wl.widths, S, wl.M, wl.n_elec, H)
    t2 = time.perf_counter()
    npt2 = max(1, sample_n // 20)
    sub = S[:npt2]
    Hs = H[:npt2, :npt2]
    psi = o["psi"][:npt2]
    res = opt2.pt2(wl.M, p.h, p.eri, p.e_core, sub, psi, Hs @ psi, diag[:npt2], o["E"])
    t3 = time.perf_counter()
    nexc = n_excitations(wl.M, wl.n_alpha, wl.n_beta)
    return {
        "value": sample_n / (t2 - t1), "unit": "amps+grads/s", "cores": ham.num_threads(), "kind": "oracle",
        "sample": (f"first {sample_n} dets of S: amplitudes+energy+gradient (torch FP64) {t2 - t1:.2f}s; "
                   f"H_SS by definition {t1 - t0:.2f}s; PT2 external sum on first {npt2} dets "
                   f"({npt2 * nexc} pairs) {t3 - t2:.2f}s"),
        "h_elements_per_s": sample_n * (nexc + 1) / (t1 - t0),
        "pt2_pairs_per_s": res["stats"]["pairs"] / (t3 - t2),
    }


# network GEMM arithmetic: FP32 MFMA; split-BF16 hidden layers with an FP32 orbital
# output layer; split-BF16 everywhere
PRECISIONS = {"fp32": "FP32", "mixed": "MIXED", "split_bf16": "SPLIT_BF16"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="m28_7a7b_s100k")
    ap.add_argument("--n-dets", type=int, default=None)
    ap.add_argument("--precision", choices=list(PRECISIONS), default="mixed")
    ap.add_argument("--out-scale", type=float, default=1e-2,
                    help="scale of the Glorot output layer (small, as the paper initialises it)")
    ap.add_argument("--cpu-sample", type=int, default=3000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-calibration", type=int, default=0,
                    help="only run a device copy of this many MiB (HBM counter calibration) and exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU; --gpus {args.gpus} is not supported (the multi-GPU sharding is a "
              "design only)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    if args.copy_calibration:
        nbytes = args.copy_calibration << 20
        x = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
        y = torch.empty_like(x)
        torch.cuda.synchronize()
        for _ in range(5):
            y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_MiB": args.copy_calibration, "launches": 5}))
        return

    import paper_2601_21310_amd as dnqs
    import synth

    wl = synth.WORKLOADS[args.workload]
    print(f"[bench] building inputs for {wl.name}", file=sys.stderr, flush=True)
    p = synth.make_problem(wl, n_dets=args.n_dets, out_scale=args.out_scale)
    n = p.dets.shape[0]
    prec = getattr(dnqs, PRECISIONS[args.precision])
    ctx = dnqs.Context(0)
    ctx.set_integrals(p.h, p.eri, p.e_core, wl.n_alpha, wl.n_beta)
    dets = dnqs.dets_to_device(p.dets)
    theta = torch.from_numpy(p.theta).cuda()
    nexc = n_excitations(wl.M, wl.n_alpha, wl.n_beta)

    def step():
        conn = ctx.build_connections(dets, validate=False)
        res = ctx.energy_and_grad(wl.widths, theta, conn, want_grad=True, precision=prec)
        out = ctx.pt2(conn, res["logabs"], res["sign"], res["E"])
        nnz = conn.nnz
        conn.free()
        return res, out, nnz

    ctx.autotune(True)   # GEMM tiles are tuned on first use (the warm-up), then fixed
    for i in range(args.warmup):
        print(f"[bench] warmup {i}", file=sys.stderr, flush=True)
        step()
    torch.cuda.synchronize()
    ctx.timing(True)
    ctx.timing_reset()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        res, out, nnz = step()
        print(f"[bench] step {i}", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    fam = {f: ctx.timing_get(f) for f in ("hss", "egrad", "pt2", "pt2_l1", "pt2_l1_fill", "pt2_l2", "pt2_reduce")}
    # energy_and_grad in every precision on the same S, for the speed/accuracy comparison
    conn = ctx.build_connections(dets, validate=False)
    forms = {}
    for name, attr in PRECISIONS.items():
        pr = getattr(dnqs, attr)
        r = ctx.energy_and_grad(wl.widths, theta, conn, want_grad=True, precision=pr)   # tunes new shapes
        r = ctx.energy_and_grad(wl.widths, theta, conn, want_grad=True, precision=pr)
        torch.cuda.synchronize()
        ctx.timing_reset()
        for i in range(max(args.steps, 3)):
            r = ctx.energy_and_grad(wl.widths, theta, conn, want_grad=True, precision=pr)
        torch.cuda.synchronize()
        tg = ctx.timing_get("egrad")
        forms[name] = (tg[0] / max(tg[1], 1), r["E"].item(), r["grad"].double())
    conn.free()
    ctx.timing(False)
    ms_step = (t1 - t0) * 1e3 / args.steps
    t_h = fam["hss"][0] / max(fam["hss"][1], 1)
    t_e = fam["egrad"][0] / max(fam["egrad"][1], 1)
    t_p = fam["pt2"][0] / max(fam["pt2"][1], 1)
    avg = {k: v[0] / max(v[1], 1) for k, v in fam.items()}
    E = res["E"].item()
    t32, E32, g32 = forms["fp32"]
    compare = {}
    for name, (t, Ef, gf) in forms.items():
        compare[name] = {"ms": t, "amps_grads_per_s": n / (t * 1e-3), "speedup_vs_fp32": t32 / t,
                         "abs_E_minus_E_fp32": abs(Ef - E32),
                         "grad_rel_l2_vs_fp32": float(torch.linalg.vector_norm(gf - g32) / torch.linalg.vector_norm(g32))}
    o = out["out"].cpu().numpy()
    c = out["counts"].cpu().numpy()
    pairs = int(c[0])
    # PT2 traffic model: an 8-byte descriptor per (x, a) pair is written by L1, read
    # twice and written once by L2, and read by the reduce: 40 B/pair over the phase.
    pt2_bytes = 40.0 * pairs
    achieved = pt2_bytes / (t_p * 1e-3) / 1e9
    line = {
        "metric": "amps+grads/s and H/PT2 elements/s at |S|=1e5; mixed vs FP32 at 1e-5 Ha",
        "value": n / (t_e * 1e-3),
        "unit": "amps+grads/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32" if prec == dnqs.FP32 else "bf16x3+f32",
        "data": "synthetic",
        "config": {"workload": wl.name, "M": wl.M, "n_alpha": wl.n_alpha, "n_beta": wl.n_beta, "n_dets": n,
                   "widths": list(wl.widths), "precision": args.precision, "out_scale": args.out_scale},
        "phases": {
            "build_connections_ms": t_h, "energy_and_grad_ms": t_e, "pt2_ms": t_p,
            "pt2_l1_ms": avg["pt2_l1"], "pt2_l1_fill_ms": avg["pt2_l1_fill"], "pt2_l2_ms": avg["pt2_l2"],
            "pt2_reduce_ms": avg["pt2_reduce"],
            "h_elements_per_s": n * (nexc + 1) / (t_h * 1e-3), "h_nnz": nnz,
            "pt2_pairs_per_s": pairs / (t_p * 1e-3), "pt2_pairs": pairs, "pt2_unique_P": int(c[1]),
            "pt2_sub_buckets": int(c[3]),
        },
        "results": {"E": E, "dE_pt2": float(o[0]), "E_total": E + float(o[0]), "min_denominator": float(o[3])},
        "precisions": compare,
        "autotune": ctx.tune_export().strip().splitlines(),
        "roofline": {"kernel": "pt2 (L1 + L2 + reduce)", "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "algorithmic_bytes_per_launch": pt2_bytes},
    }
    if not args.no_cpu_baseline:
        print("[bench] cpu baseline", file=sys.stderr, flush=True)
        line["cpu_baseline"] = cpu_baseline(p, args.cpu_sample)
    print(json.dumps(line))


if __name__ == "__main__":
    main()
