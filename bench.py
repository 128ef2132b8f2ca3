"""Benchmark of the hot path on one MI355X.

Workload (the at-scale float64 configuration): N = 6, product bound B = 4096
(|K| = 4,883,360 rows), chained Henon-Heiles potential lambda = 0.111 plus the laser term
0.05 sin(2t) sum_d x_d (coefficients rebuilt at t + h/2 every step), start vector the
harmonic-oscillator coherent state displaced to x_d = 2 normalised on K, exponential
midpoint steps of h = 0.005 with m = 10 Lanczos vectors and one Gram-Schmidt pass.

One timed "step" is one full time step: coefficient update, 10 applications of H,
the Lanczos recurrences and reductions, the small eigensolve and the combination.
value = H applications per second over the timed region.

Also measured inside this run:
  roofline      -- the H-application kernel timed back to back with HIP events on its
                   own stream; algorithmic bytes 32 |K| per launch (read c, write H c,
                   complex128) against 8 TB/s.
  cpu_baseline  -- the CPU oracle's fast algorithm on the same workload (rank 0 only).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

N_DIM, B_BOUND, M_KRYLOV, H_STEP = 6, 4096, 10, 0.005
HBM_PEAK_GBS = 8000.0


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--graph", type=int, default=1, help="replay the step as a captured HIP graph")
    ap.add_argument("--tile-dim", type=int, default=0)
    ap.add_argument("--matvec-reps", type=int, default=50)
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: this build runs on one GPU only; the multi-GPU path is not built "
              "(see DESIGN.md, 'How the path would shard').", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_1403_3511_amd import hs
    from synth import coherent_state, henon_heiles_chain

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    terms = henon_heiles_chain(N_DIM, 0.111, 0.05)
    lib_terms = [(x[0], x[1], x[2], x[3], x.degrees) for x in terms]
    idx = hs.Index(N_DIM, B_BOUND, args.tile_dim)
    pot = hs.Pot(N_DIM, lib_terms, subtract_harmonic=True)
    k = idx.multi_indices()
    c0 = coherent_state(k, 2.0)
    c0 /= np.linalg.norm(c0)
    c = torch.from_numpy(c0).to(dev)
    ws = hs.workspace(idx, pot, hs.HS_C128, M_KRYLOV)
    t_dev = torch.zeros(1, dtype=torch.float64, device=dev)
    stream = torch.cuda.current_stream()

    def one_step():
        hs.step(idx, pot, c, 0.0, H_STEP, M_KRYLOV, dtype=hs.HS_C128, reorth=True, ws=ws, t_dev=t_dev)

    for _ in range(args.warmup):
        one_step()
    torch.cuda.synchronize()

    graph = None
    if args.graph:
        graph = torch.cuda.CUDAGraph()
        s2 = torch.cuda.Stream()
        s2.wait_stream(stream)
        with torch.cuda.stream(s2):
            with torch.cuda.graph(graph, stream=s2):
                hs.step(idx, pot, c, 0.0, H_STEP, M_KRYLOV, dtype=hs.HS_C128, reorth=True,
                        ws=ws, t_dev=t_dev)
        stream.wait_stream(s2)
        torch.cuda.synchronize()
        graph.replay()  # one more warm step through the graph
        torch.cuda.synchronize()

    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(args.steps):
        if graph is not None:
            graph.replay()
        else:
            one_step()
    e1.record(stream)
    torch.cuda.synchronize()
    ms_total = e0.elapsed_time(e1)
    ms_per_step = ms_total / args.steps
    value = args.steps * M_KRYLOV / (ms_total / 1e3)
    norm_err = abs(float(torch.linalg.norm(c).item()) - 1.0)

    # ---- dominant kernel: H application, back to back on this stream ----
    x = torch.from_numpy(c0).to(dev)
    y = torch.empty_like(x)
    aws = hs.workspace(idx, pot, hs.HS_C128, 0)
    pot.set_time(0.1)
    for _ in range(3):
        hs.apply_h(idx, pot, x, y, hs.HS_C128, aws)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(args.matvec_reps):
        hs.apply_h(idx, pot, x, y, hs.HS_C128, aws)
    e1.record(stream)
    torch.cuda.synchronize()
    us_matvec = e0.elapsed_time(e1) * 1e3 / args.matvec_reps
    alg_bytes = 32.0 * idx.size
    achieved = alg_bytes / (us_matvec * 1e-6) / 1e9
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                "kernel": "k_hh_rows<double>" if pot.fused else "k_pass<double>",
                "us_per_launch": round(us_matvec, 2), "alg_bytes_per_launch": int(alg_bytes)}

    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline(np)

    line = {
        "metric": "Galerkin matvecs/s (H applications per second inside full Magnus-Lanczos steps)",
        "value": round(value, 1),
        "unit": "matvec/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "N=6 B=4096 (|K|=%d) chained Henon-Heiles lambda=0.111 + laser "
                               "0.05 sin(2t); coherent packet x_d=2; m=10, h=0.005, one CGS pass; "
                               "%s" % (idx.size, "HIP graph replay" if graph else "eager"),
                   "rows": idx.size, "m": M_KRYLOV, "h": H_STEP, "tile_dim": idx.tile_dim,
                   "hbm_gbs_matvec": round(achieved, 1), "norm_drift": norm_err},
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


def cpu_baseline(np):
    """The CPU oracle's fast algorithm (NumPy, float64) on the same workload: a bounded
    sample of 3 applications of H on the full set, reported as matvec/s."""
    from oracle.index import IndexSet
    from oracle.operators import Potential, fast_apply_H, subtract_harmonic
    from synth import coherent_state, henon_heiles_chain

    t0 = time.time()
    ix = IndexSet(N_DIM, B_BOUND)
    build_s = time.time() - t0
    terms = henon_heiles_chain(N_DIM, 0.111, 0.05)
    W = subtract_harmonic(Potential(N_DIM, "mono", 1.0, [(x.coef(0.1), x.degrees) for x in terms]))
    v = coherent_state(ix.k, 2.0)
    v /= np.linalg.norm(v)
    reps = 3
    t0 = time.perf_counter()
    for _ in range(reps):
        v = fast_apply_H(ix, W, v)
        v /= np.linalg.norm(v)
    dt = time.perf_counter() - t0
    return {"value": round(reps / dt, 4), "unit": "matvec/s", "cores": 1, "kind": "oracle",
            "sample": "3 applications of H by the NumPy oracle fast algorithm on the full "
                      "N=6 B=4096 set (index build %.1f s not counted), single thread" % build_s}


if __name__ == "__main__":
    main()
