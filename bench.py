"""Benchmark: reconstructed slices/s of batched hybrid AB-GMRES on one MI355X.

Workload (default): 256 independent 512x512 FP32 slices of random-ellipse
phantoms, 720 angles on [0, pi) x 725 unit bins, per-slice noise level drawn
log-uniform in [0.1%, 5%]; hybrid AB-GMRES with the GCV lambda rule and the
discrepancy-principle stop (tau = 1.01, known ||e||), at most 100 iterations,
FP32 projectors and FP64 small solves, all slices in one batched solve whose
per-iteration launch sequence is a replayed hipGraph.  One step = one such
solve of the whole batch, inputs already resident in HBM.

The JSON line also carries: the plain per-slice path (one slice per call,
eager launches, host stop check every iteration) on a subset of the same
slices, with the check that it returns bitwise the same reconstructions; the
projector throughput (compulsory bytes per apply / kernel time); the roofline
of the dominant kernel; and the CPU oracle timed on a bounded sample.

    python bench.py [--steps K] [--warmup W] [--slices S] [--kmax K]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# VALU issue rate: 256 CUs x 4 SIMD x 16 lanes x 2.4 GHz = 3.93e13 lane-ops/s
VALU_LANE_OPS = 256 * 64 * 2.4e9


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=3)
    p.add_argument("--warmup", type=int, default=1)
    p.add_argument("--slices", type=int, default=256)
    p.add_argument("--kmax", type=int, default=100)
    p.add_argument("--n", type=int, default=512)
    p.add_argument("--angles", type=int, default=720)
    p.add_argument("--det", type=int, default=725)
    p.add_argument("--poll", type=int, default=4)
    p.add_argument("--plain-slices", type=int, default=8)
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--quiet", action="store_true")
    return p.parse_args()


def log(args, *a):
    if not args.quiet:
        print(*a, file=sys.stderr, flush=True)


def make_inputs(args, pk, A, torch):
    """Seeded phantoms (synthetic, on the GPU), b = A x + e with ||e|| = eta ||A x||."""
    import numpy as np

    import synth
    S, n = args.slices, args.n
    dev = torch.device("cuda")
    x = torch.empty((S, n, n), dtype=torch.float32, device=dev)
    eta = np.empty(S)
    for s in range(S):
        img, _ = synth.phantom2d(2, s, n, device=dev)
        x[s] = img.to(torch.float32)
        eta[s] = synth.noise_level(2, s, 1e-3, 5e-2)
    bt = pk.project(A, x)
    b = torch.empty_like(bt)
    en = np.empty(S)
    m = bt[0].numel()
    for s in range(S):
        g = torch.as_tensor(synth.noise_direction(2, s, m), device=dev, dtype=torch.float64)
        btd = bt[s].double().reshape(-1)
        nb = float(torch.linalg.vector_norm(btd))
        e = (eta[s] * nb / float(torch.linalg.vector_norm(g))) * g
        b[s] = (btd + e).reshape(bt[s].shape).to(torch.float32)
        en[s] = eta[s] * nb
    torch.cuda.synchronize()
    return x, b, torch.tensor(en, dtype=torch.float64, device=dev), eta


def time_apply(fn, torch, reps=5):
    stream = torch.cuda.current_stream()
    fn()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        fn()
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / 1e3 / reps


def cpu_baseline(args, b_slice, en_slice, k_cap):
    """The FP64 oracle on one slice of the same workload (same rule and stop)."""
    import numpy as np

    import oracle
    from oracle.geometry import Par2D
    from oracle.operators import Par2DOps
    from oracle.solver import hybrid_gmres
    oracle.build_oracle(force=False)
    og = Par2DOps(Par2D(args.n, args.n, args.angles, args.det))
    bb = np.asarray(b_slice, dtype=np.float64).ravel()
    t0 = time.perf_counter()
    o = hybrid_gmres(og.A, og.B, bb, mode="AB", K=k_cap, rule="gcv", stop="dp", tau=1.01,
                     noise_norm=float(en_slice))
    t = time.perf_counter() - t0
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return t, o.iters, threads


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU: the slices of the batched workload are "
                          "independent and shard with no communication, but only the one-GPU path is "
                          "built and measured; rerun with --gpus 1"}))
        sys.exit(2)
    import numpy as np
    import torch

    import paper_2602_17892_amd as pk
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    S, K = args.slices, args.kmax
    g = pk.Geometry(args.n, args.n, args.angles, args.det)
    A = pk.Operator("joseph", g, "f32", "f32")
    B = pk.Operator("pixel", g, "f32", "f32")
    t0 = time.perf_counter()
    x_true, b, en, eta = make_inputs(args, pk, A, torch)
    log(args, f"inputs: {S} slices of {args.n}^2, {args.angles}x{args.det} in {time.perf_counter() - t0:.1f}s")

    ws_bytes = pk.workspace_bytes(A, B, S, "AB", K, stop="dp")
    ws = torch.empty(ws_bytes, dtype=torch.uint8, device="cuda")
    log(args, f"workspace {ws_bytes / 2**30:.1f} GiB")

    def step():
        return pk.solve(A, B, b, mode="AB", k=K, reg="gcv", tau=1.01, noise_norm=en, stop="dp",
                        use_graph=True, poll_every=args.poll, workspace=ws, history=False)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        xb, info = step()
    torch.cuda.synchronize()
    t_batched = (time.perf_counter() - t0) / args.steps
    iters = info["iters"].cpu().numpy()
    status = info["status"].cpu().numpy()
    rre_b = (torch.linalg.vector_norm((xb - x_true).reshape(S, -1).double(), dim=1)
             / torch.linalg.vector_norm(x_true.reshape(S, -1).double(), dim=1)).cpu().numpy()
    log(args, f"batched: {t_batched:.3f}s/step, iters mean {iters.mean():.1f} [{iters.min()}, {iters.max()}], "
              f"median RRE {np.median(rre_b):.4f}")

    # ---- plain per-slice path on a subset (same slices, same rule/stop)
    P = min(args.plain_slices, S)
    idx = np.linspace(0, S - 1, P).round().astype(int)
    ws1 = torch.empty(pk.workspace_bytes(A, B, 1, "AB", K, stop="dp"), dtype=torch.uint8, device="cuda")
    plain = lambda s: pk.solve(A, B, b[s:s + 1], mode="AB", k=K, reg="gcv", tau=1.01, noise_norm=en[s:s + 1],
                               stop="dp", use_graph=False, poll_every=1, workspace=ws1, history=False)
    plain(int(idx[0]))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    same = True
    plain_iters = []
    for s in idx:
        x1, i1 = plain(int(s))
        torch.cuda.synchronize()
        same = same and bool(torch.equal(x1[0], xb[s]))
        plain_iters.append(int(i1["iters"][0]))
    t_plain = (time.perf_counter() - t0) / P
    # the batched run's work on the same subset: scale by the subset's share of iterations
    log(args, f"plain: {t_plain:.3f}s/slice on {P} slices, bitwise equal to batched: {same}")

    # ---- projector throughput over the whole batch (one launch each)
    xin = x_true.contiguous()
    yb = torch.empty_like(b)
    xo = torch.empty_like(xin)
    t_A = time_apply(lambda: pk.project(A, xin, out=yb), torch)
    t_B = time_apply(lambda: pk.backproject(B, b, out=xo), torch)
    n, m = args.n * args.n, args.angles * args.det
    bytes_apply = S * (n + m) * 4
    gbs_A, gbs_B = bytes_apply / t_A / 1e9, bytes_apply / t_B / 1e9
    pairs = S * n * args.angles
    log(args, f"A: {t_A * 1e3:.2f} ms ({gbs_A:.1f} GB/s); B: {t_B * 1e3:.2f} ms ({gbs_B:.1f} GB/s)")

    value = S / t_batched
    out = {
        "metric": "reconstructed slices/sec (hybrid AB-GMRES, GCV lambda, DP stop), batched vs plain; projector GB/s",
        "value": round(value, 3),
        "unit": "slices/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(t_batched * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 projectors+basis, f64 reductions and small solves",
        "data": "synthetic: seeded random-ellipse phantoms, b = A x + relative Gaussian noise",
        "config": {"workload": f"{S} x {args.n}^2 slices, {args.angles} angles x {args.det} bins, "
                               f"eta log-uniform [0.1%,5%], hybrid AB-GMRES GCV + DP stop, kmax {K}",
                   "slices": S, "kmax": K, "poll_every": args.poll},
        "iters": {"mean": float(iters.mean()), "min": int(iters.min()), "max": int(iters.max()),
                  "status_dp": int((status & 2 != 0).sum())},
        "rre_median": float(np.median(rre_b)),
        "plain": {"slices_per_s": round(1.0 / t_plain, 3), "subset": [int(s) for s in idx],
                  "bitwise_equal_to_batched": same, "speedup_batched_vs_plain": round(value * t_plain, 3)},
        "projector": {"A_GBps": round(gbs_A, 2), "A_frac_hbm": round(gbs_A / HBM_PEAK_GBS, 5),
                      "B_GBps": round(gbs_B, 2), "B_frac_hbm": round(gbs_B / HBM_PEAK_GBS, 5),
                      "A_ms_batch": round(t_A * 1e3, 3), "B_ms_batch": round(t_B * 1e3, 3),
                      "B_Gpairs_per_s": round(pairs / t_B / 1e9, 2)},
    }
    if not args.no_cpu_baseline:
        s0 = int(np.argsort(iters)[len(iters) // 2])
        t_cpu, it_cpu, thr = cpu_baseline(args, b[s0].double().cpu().numpy(), float(en[s0]), K)
        out["cpu_baseline"] = {"value": round(1.0 / t_cpu, 5), "unit": "slices/s", "cores": thr, "kind": "oracle",
                               "sample": f"1 slice (index {s0}, median GPU stop iteration {int(iters[s0])}) "
                                         f"solved to its DP stop by the FP64 oracle: {t_cpu:.1f}s, "
                                         f"{it_cpu} iterations"}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
