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
    """Time the oracle (as it stands) on the first sample_n dets of S: amplitudes + energy +
    gradient in FP64 (the headline unit), H_SS by its definition, and the PT2 external sum
    on the first sample_n / 20 dets.  Protocol: one warm run, then the median of three
    timed runs, with all host cores; the amplitudes + gradient step also on one core."""
    import statistics

    import scipy.sparse as sp
    import torch

    from oracle import energy
    from oracle import hamiltonian as ham
    from oracle import pt2 as opt2
    wl = p.wl
    S = p.dets[:sample_n]
    npt2 = max(1, sample_n // 20)
    nexc = n_excitations(wl.M, wl.n_alpha, wl.n_beta)
    cores = ham.num_threads()
    torch_threads = torch.get_num_threads()

    def hss():
        return ham.csr_rows(wl.M, p.h, p.eri, p.e_core, S)

    row_ptr, col, val, diag = hss()
    H = (sp.csr_matrix((val, col, row_ptr), shape=(len(S), len(S))) + sp.diags(diag)).tocsr()

    def egrad():
        return energy.energy_and_grad(p.theta, wl.widths, S, wl.M, wl.n_elec, H)

    o = egrad()
    psi = o["psi"][:npt2]
    Hs = H[:npt2, :npt2]

    def pt2():
        return opt2.pt2(wl.M, p.h, p.eri, p.e_core, S[:npt2], psi, Hs @ psi, diag[:npt2], o["E"])

    def median3(fn):
        fn()  # warm run
        ts = []
        for _ in range(3):
            t0 = time.perf_counter()
            fn()
            ts.append(time.perf_counter() - t0)
        return statistics.median(ts)

    t_e = median3(egrad)
    t_h = median3(hss)
    t_p = median3(pt2)
    # one core: torch and the oracle's OpenMP part each on one thread
    n1 = max(64, sample_n // 8)
    S1 = S[:n1]
    H1 = H[:n1, :n1]
    torch.set_num_threads(1)
    ham.set_num_threads(1)
    try:
        t_e1 = median3(lambda: energy.energy_and_grad(p.theta, wl.widths, S1, wl.M, wl.n_elec, H1))
    finally:
        torch.set_num_threads(torch_threads)
        ham.set_num_threads(cores)
    return {
        "value": sample_n / t_e, "unit": "amps+grads/s", "cores": cores, "kind": "oracle",
        "sample": (f"first {sample_n} dets of S, median of 3 after a warm run: amplitudes+energy+gradient "
                   f"(torch FP64, {torch_threads} threads) {t_e:.2f}s; H_SS by definition {t_h:.2f}s; PT2 external "
                   f"sum on the first {npt2} dets ({npt2 * nexc} pairs) {t_p:.2f}s; one core: "
                   f"amplitudes+energy+gradient on the first {n1} dets {t_e1:.2f}s"),
        "single_thread_amps_grads_per_s": n1 / t_e1,
        "h_elements_per_s": sample_n * (nexc + 1) / t_h,
        "pt2_pairs_per_s": npt2 * nexc / t_p,
    }


# network GEMM arithmetic: FP32 MFMA; split-BF16 hidden layers with an FP32 orbital
# output layer; split-BF16 everywhere
PRECISIONS = {"fp32": "FP32", "mixed": "MIXED", "split_bf16": "SPLIT_BF16"}


def gemm_flops(widths):
    """FP32-equivalent flops of the network GEMMs per configuration: forward layers 2..L,
    data gradients of layers L..2, weight gradients (bias row included) of layers L..1."""
    L = len(widths) - 1
    fwd = sum(widths[l - 1] * widths[l] for l in range(2, L + 1))
    dgrad = fwd
    wgrad = sum((widths[l - 1] + 1) * widths[l] for l in range(1, L + 1))
    return 2.0 * (fwd + dgrad + wgrad)


def bench_sweep(args, dnqs, synth, torch):
    """|S| sweep on one workload: per size the H_SS build, energy+gradient in FP32 and in
    the mixed form, and PT2 while the pair count is at most --sweep-pt2-max."""
    wl = synth.WORKLOADS[args.workload]
    nexc = n_excitations(wl.M, wl.n_alpha, wl.n_beta)
    fl = gemm_flops(wl.widths)
    rows = []
    for n in [int(float(v)) for v in args.sweep.split(",")]:
        print(f"[bench] sweep |S| = {n}: building inputs", file=sys.stderr, flush=True)
        p = synth.make_problem(wl, n_dets=n, out_scale=args.out_scale)
        ctx = dnqs.Context(0)
        ctx.autotune(True)
        ctx.set_integrals(p.h, p.eri, p.e_core, wl.n_alpha, wl.n_beta)
        dets = dnqs.dets_to_device(p.dets)
        theta = torch.from_numpy(p.theta).cuda()
        ctx.timing(True)
        conn = ctx.build_connections(dets, validate=False)
        nnz = conn.nnz
        ctx.timing_reset()
        conn.free()
        conn = ctx.build_connections(dets, validate=False)
        torch.cuda.synchronize()
        t_h = ctx.timing_get("hss")[0]
        row = {"n_dets": n, "h_nnz": nnz, "build_connections_ms": t_h,
               "h_elements_per_s": n * (nexc + 1) / (t_h * 1e-3)}
        for name in ("fp32", args.precision):
            pr = getattr(dnqs, PRECISIONS[name])
            rc = args.recompute
            r = ctx.energy_and_grad(wl.widths, theta, conn, precision=pr, recompute=rc)   # tunes new shapes
            r = ctx.energy_and_grad(wl.widths, theta, conn, precision=pr, recompute=rc)
            torch.cuda.synchronize()
            ctx.timing_reset()
            for _ in range(max(args.steps, 3)):
                r = ctx.energy_and_grad(wl.widths, theta, conn, precision=pr, recompute=rc)
            torch.cuda.synchronize()
            t = ctx.timing_get("egrad")[0] / max(args.steps, 3)
            peak = FP32_PEAK_TFLOPS if name == "fp32" else BF16_PEAK_TFLOPS / 3.0
            tf = n * fl / (t * 1e-3) / 1e12
            # flops of the full-width network (gemm_flops): with the occupied-row output
            # layer the GEMMs do less work, so this is a dense-equivalent rate
            row[name] = {"energy_and_grad_ms": t, "amps_grads_per_s": n / (t * 1e-3), "E": r["E"].item(),
                         "recompute": bool(rc), "device_bytes_held": ctx.allocator.live_bytes,
                         "dense_equiv_gemm_tflops": tf, "gemm_peak_tflops": peak, "dense_equiv_frac": tf / peak}
        if n * nexc <= args.sweep_pt2_max:
            r = ctx.energy_and_grad(wl.widths, theta, conn, want_grad=False, precision=getattr(dnqs, PRECISIONS[args.precision]))
            ctx.timing_reset()
            out = ctx.pt2(conn, r["logabs"], r["sign"], r["E"])
            torch.cuda.synchronize()
            t_p = ctx.timing_get("pt2")[0]
            c = out["counts"].cpu().numpy()
            row["pt2"] = {"ms": t_p, "pairs": int(c[0]), "pairs_per_s": int(c[0]) / (t_p * 1e-3),
                          "unique_P": int(c[1]), "reduce_launches": ctx.timing_get("pt2_reduce")[1],
                          "dE_pt2": float(out["out"][0].item())}
        conn.free()
        ctx.close()
        rows.append(row)
        print(f"[bench] sweep |S| = {n}: {json.dumps(row)}", file=sys.stderr, flush=True)
    big = rows[-1]
    line = {
        "metric": "amps+grads/s and H/PT2 elements/s over an |S| sweep",
        "value": big[args.precision]["amps_grads_per_s"], "unit": "amps+grads/s", "n_gpus": 1,
        "steps": max(args.steps, 3), "warmup": 2, "ms_per_step": big[args.precision]["energy_and_grad_ms"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "bf16x3+f32", "data": "synthetic",
        "config": {"workload": wl.name, "M": wl.M, "n_alpha": wl.n_alpha, "n_beta": wl.n_beta,
                   "widths": list(wl.widths), "precision": args.precision, "n_exc": nexc,
                   "gemm_flops_per_config": fl},
        "sweep": rows,
    }
    print(json.dumps(line))


def bench_out_scale(args, dnqs, synth, torch):
    """Mixed-precision error and speed against the scale of the output layer (the network
    leaves its near-zero initialisation as it trains): per out_scale, energy+gradient in
    FP32, MIXED and SPLIT_BF16 on the same S, |E - E_FP32|, the gradient's relative L2
    error, and the PT2 correction from each form's psi and E (normalised dE of Eq. 13)."""
    wl = synth.WORKLOADS[args.workload]
    scales = [float(v) for v in args.out_scale_sweep.split(",")]
    p0 = synth.make_problem(wl, n_dets=args.n_dets, out_scale=scales[0])
    ctx = dnqs.Context(0)
    ctx.autotune(True)
    ctx.set_integrals(p0.h, p0.eri, p0.e_core, wl.n_alpha, wl.n_beta)
    dets = dnqs.dets_to_device(p0.dets)
    conn = ctx.build_connections(dets, validate=False)
    n = p0.dets.shape[0]
    rows = []
    ctx.timing(True)
    for sc in scales:
        p = synth.make_problem(wl, n_dets=args.n_dets, out_scale=sc)
        assert (p.dets == p0.dets).all()
        theta = torch.from_numpy(p.theta).cuda()
        row = {"out_scale": sc}
        ref = None
        for name, attr in PRECISIONS.items():
            pr = getattr(dnqs, attr)
            r = ctx.energy_and_grad(wl.widths, theta, conn, precision=pr)   # tunes new shapes
            r = ctx.energy_and_grad(wl.widths, theta, conn, precision=pr)
            torch.cuda.synchronize()
            ctx.timing_reset()
            for _ in range(max(args.steps, 3)):
                r = ctx.energy_and_grad(wl.widths, theta, conn, precision=pr)
            torch.cuda.synchronize()
            t = ctx.timing_get("egrad")[0] / max(args.steps, 3)
            out = ctx.pt2(conn, r["logabs"], r["sign"], r["E"])
            E, g, dE = r["E"].item(), r["grad"].double(), float(out["out"][0].item())
            if ref is None:
                ref = (t, E, g, dE)
            row[name] = {"ms": t, "speedup_vs_fp32": ref[0] / t, "E": E, "abs_E_minus_E_fp32": abs(E - ref[1]),
                         "grad_rel_l2_vs_fp32": float(torch.linalg.vector_norm(g - ref[2]) /
                                                      torch.linalg.vector_norm(ref[2])),
                         "dE_pt2": dE, "abs_dE_pt2_minus_fp32": abs(dE - ref[3])}
        rows.append(row)
        print(f"[bench] out_scale {sc}: {json.dumps(row)}", file=sys.stderr, flush=True)
    ctx.timing(False)
    conn.free()
    line = {
        "metric": "mixed-precision error and speed against the output-layer scale",
        "value": rows[0]["mixed"]["speedup_vs_fp32"], "unit": "x vs FP32", "n_gpus": 1,
        "steps": max(args.steps, 3), "warmup": 2, "ms_per_step": rows[0]["mixed"]["ms"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "bf16x3+f32",
        "data": "synthetic",
        "config": {"workload": wl.name, "n_dets": n, "widths": list(wl.widths)},
        "note": "dE_pt2 at a random-init network's psi: E lies inside the H_aa spread, so the "
                "PT2 values compare the forms, they are not converged corrections",
        "out_scale_sweep": rows,
    }
    print(json.dumps(line))


def bench_curve(args, dnqs, synth, torch):
    """One optimisation step over G geometries: G sequential energy_and_grad calls, one
    batched call, and a replayed HIP graph of the batched step + AdamW (same stream)."""
    wl = synth.WORKLOADS["m20_6a6b_curve"]
    prec = getattr(dnqs, PRECISIONS[args.precision])
    print(f"[bench] building {args.curve} geometries", file=sys.stderr, flush=True)
    curve = synth.make_curve(wl, n_geoms=args.curve, out_scale=args.out_scale)
    sizes = [p.dets.shape[0] for p in curve]
    ntot = sum(sizes)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        ctx = dnqs.Context(0)
        ctx.autotune(True)
        conns = []
        for g, p in enumerate(curve):
            ctx.set_integrals(p.h, p.eri, p.e_core, wl.n_alpha, wl.n_beta, slot=g)
            conns.append(ctx.build_connections(dnqs.dets_to_device(p.dets), slot=g, validate=False))
        thetas = [torch.from_numpy(p.theta).cuda() for p in curve]
        batch = ctx.batch(wl.widths, list(range(len(curve))), conns, thetas)
        np_ = thetas[0].numel()
        m = torch.zeros(len(curve) * np_, device="cuda")
        v = torch.zeros(len(curve) * np_, device="cuda")
        step = torch.zeros(1, dtype=torch.int32, device="cuda")
        reps = max(args.steps, 3)

        def timed(fn):
            for _ in range(max(args.warmup, 1)):
                fn()
            stream.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            for _ in range(reps):
                fn()
            e1.record(stream)
            e1.synchronize()
            return e0.elapsed_time(e1) / reps

        t_seq = timed(lambda: [ctx.energy_and_grad(wl.widths, thetas[g], conns[g], precision=prec, keep=False)
                               for g in range(len(curve))])
        t_bat = timed(lambda: ctx.energy_and_grad_batched(batch, precision=prec))
        ctx.energy_and_grad_batched(batch, precision=prec)
        ctx.capture_begin()
        ctx.energy_and_grad_batched(batch, precision=prec)
        ctx.adamw_batched(batch, m, v, step)
        graph = ctx.capture_end()
        t_graph = timed(graph.launch)
        graph.free()
    line = {
        "metric": "amps+grads/s over a dissociation curve (one optimisation step over all geometries)",
        "value": ntot / (t_graph * 1e-3), "unit": "amps+grads/s", "n_gpus": 1, "steps": reps,
        "warmup": args.warmup, "ms_per_step": t_graph, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32" if prec == dnqs.FP32 else "bf16x3+f32", "data": "synthetic",
        "config": {"workload": wl.name, "geometries": len(curve), "total_dets": ntot, "min_dets": min(sizes),
                   "max_dets": max(sizes), "widths": list(wl.widths), "precision": args.precision},
        "sequential_ms": t_seq, "batched_ms": t_bat, "graph_step_ms": t_graph,
        "speedup_batched_vs_sequential": t_seq / t_bat, "speedup_graph_vs_sequential": t_seq / t_graph,
        "autotune": ctx.tune_export().strip().splitlines(),
    }
    print(json.dumps(line))


# HBM bytes per launch of a kernel from two rocprofv3 --pmc passes (FETCH_SIZE x 2.0,
# WRITE_SIZE x 1.0, the factors a 1 GiB device copy gives), valid only for the kernel
# source they were taken on (profiles/pt2_hss_m28_s1e5_hbm_counters.md).
MEASURED_TRAFFIC = {
    ("k_pt2_reduce", "m28_7a7b_s100k"): ("paper_2601_21310_amd/csrc/k_pt2_reduce.hip",
                                          "d6c838336acef5560292a95e7a7a5fc4e809190c38a5409cfa1df87c5a8aa6bc",
                                          24907113760.0),
}


def measured_traffic(kernel, workload):
    import hashlib
    rec = MEASURED_TRAFFIC.get((kernel, workload))
    if rec is None:
        return None
    path, sha, nbytes = rec
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), path), "rb") as f:
        if hashlib.sha256(f.read()).hexdigest() != sha:
            return None          # the kernel changed since the counters were taken
    return nbytes


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="m28_7a7b_s100k")
    ap.add_argument("--n-dets", type=int, default=None)
    ap.add_argument("--precision", choices=list(PRECISIONS), default="split_bf16",
                    help="form of the timed step (split_bf16: every network GEMM in split BF16, the fastest form "
                         "that meets 1e-5 Ha against the oracle at full size; all three are timed beside it)")
    ap.add_argument("--out-scale", type=float, default=1e-2,
                    help="scale of the Glorot output layer (small, as the paper initialises it)")
    ap.add_argument("--cpu-sample", type=int, default=12000,
                    help="dets of S the oracle is timed on (about 10-30 s of host work in all)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--sweep", default="",
                    help="instead of the headline run: comma-separated |S| values on --workload (e.g. "
                         "m56_12a12b with 1e4,3e4,1e5,3e5,1e6): H_SS, energy+gradient and, up to --sweep-pt2-max "
                         "pairs, PT2 for each")
    ap.add_argument("--sweep-pt2-max", type=float, default=2e10)
    ap.add_argument("--recompute", action="store_true",
                    help="in the sweep: keep only the last hidden layer, recomputing the others by row block")
    ap.add_argument("--curve", type=int, default=0,
                    help="instead of the headline run: energy+gradient over a synthetic dissociation curve of "
                         "this many geometries (M=20, 6a+6b, |S| log-uniform in [2^10, 2^16]), sequential vs "
                         "batched vs a replayed HIP graph of the batched step with AdamW")
    ap.add_argument("--out-scale-sweep", default="",
                    help="instead of the headline run: comma-separated output-layer scales (e.g. "
                         "1e-3,1e-2,1e-1,1): energy+gradient error and speed of each precision form, and the "
                         "PT2 correction from each form's psi")
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

    if args.curve:
        return bench_curve(args, dnqs, synth, torch)
    if args.sweep:
        return bench_sweep(args, dnqs, synth, torch)
    if args.out_scale_sweep:
        return bench_out_scale(args, dnqs, synth, torch)

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
    # Roofline of the dominant kernel, the PT2 reduce, on the group-by model of the PT2
    # step: a pair's key and value (16 + 4 bytes) are written once and read once, and the
    # reduce is the read half, 20 bytes per pair.  The reduce's own HBM stream (one 8-byte
    # descriptor per pair) and its measured traffic are kept beside it.
    t_red = avg["pt2_reduce"]
    # reduce launches per pt2 call (more than one when the key space is sliced)
    red_per_call = fam["pt2_reduce"][1] / max(fam["pt2"][1], 1)
    red_bytes = 20.0 * pairs / max(red_per_call, 1.0)
    achieved = red_bytes / (t_red * 1e-3) / 1e9
    traffic = measured_traffic("k_pt2_reduce", wl.name)
    # the whole PT2 phase against the 40 B/pair group-by model (write + read of a
    # 16-byte key and a 4-byte value per pair)
    pt2_model = 40.0 * pairs
    # PT2 where the method evaluates it, after convergence: the lowest eigenvector of
    # H_SS (GPU Lanczos) stands in for a converged network; the timed step's PT2 runs on
    # the random-init network's psi, where E sits inside the spread of H_aa (intruder
    # terms), so its value is a timing figure only
    conn = ctx.build_connections(dets, validate=False)
    lz = ctx.lanczos(conn, max_iter=400, tol=1e-9)
    vec = lz["vec"]
    la_gs = torch.log(torch.abs(vec))
    sg_gs = torch.sign(vec).to(torch.int8)
    ctx.timing(True)
    ctx.timing_reset()
    gs = ctx.pt2(conn, la_gs, sg_gs, lz["E"])
    torch.cuda.synchronize()
    t_gs = ctx.timing_get("pt2")[0]
    ctx.timing(False)
    gso = gs["out"].cpu().numpy()
    conn.free()
    E_diag = lz["E"].item()
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
        "results": {"E": E, "E_diag": E_diag, "lanczos_iters": lz["iters"], "lanczos_residual": lz["residual"],
                    "dE_pt2_ground_state": float(gso[0]), "E_total_ground_state": E_diag + float(gso[0]),
                    "min_denominator_ground_state": float(gso[3]), "pt2_ground_state_ms": t_gs,
                    "dE_pt2_timed_step": float(o[0]), "min_denominator_timed_step": float(o[3]),
                    "timed_step_note": "random-init network psi: timing only (E inside the H_aa spread)"},
        "precisions": compare,
        "autotune": ctx.tune_export().strip().splitlines(),
        "roofline": {"kernel": "k_pt2_reduce", "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "algorithmic_bytes_per_launch": red_bytes, "model": "20 B/pair (read half of the group-by)",
                     "launch_ms": t_red,
                     "descriptor_stream_GBs": 8.0 * pairs / max(red_per_call, 1.0) / (t_red * 1e-3) / 1e9},
        "pt2_phase_roofline": {"model": "40 B/pair group-by", "bytes": pt2_model, "ms": t_p,
                               "achieved": pt2_model / (t_p * 1e-3) / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                               "frac": pt2_model / (t_p * 1e-3) / 1e9 / HBM_PEAK_GBS},
    }
    if not args.no_cpu_baseline:
        print("[bench] cpu baseline", file=sys.stderr, flush=True)
        line["cpu_baseline"] = cpu_baseline(p, args.cpu_sample)
    print(json.dumps(line))


if __name__ == "__main__":
    main()
