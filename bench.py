"""Benchmark: reconstructed slices/s of batched hybrid AB-GMRES on one MI355X.

Workload (default): 256 independent 512x512 FP32 slices of random-ellipse
phantoms, 720 angles on [0, pi) x 725 unit bins, per-slice noise level drawn
log-uniform in [0.1%, 5%]; hybrid AB-GMRES with the GCV lambda rule and the
discrepancy-principle stop (tau = 1.01, known ||e||), at most 100 iterations,
FP32 projectors and FP64 small solves, all slices in one batched solve whose
per-iteration launch sequence is a replayed hipGraph; the library splits the
batch into --streams concurrent sub-batches (default 3), each on a stream of
its own.  One step = one such solve of the whole batch, inputs already
resident in HBM.

The JSON line also carries: the plain per-slice path (one slice per call,
eager launches, host stop check every iteration) on a subset of the same
slices, with the check that it returns bitwise the same reconstructions; the
projector throughput (compulsory bytes per apply / kernel time); the roofline
of the dominant kernel (with its recorded HBM traffic and VALU issue); the
learned lambda/stop rule against GCV + DP; and the CPU oracle timed on a
bounded sample.

    python bench.py [--steps K] [--warmup W] [--slices S] [--kmax K] [--streams P]

Other workloads print a JSON line of their own (--workload): cone (the 256^3
cone-beam volume), learned (the learned-rule comparison alone), variants (BA,
restarted cycles, the NCP stop, the 1024^2 fan beam) and paper (single solves
at the shapes of the paper's Test Problems 2-3).
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
# FP32 vector peak without packed FP32 math (the library is built with packed
# FP32 instructions disabled): 256 CUs x 4 SIMD x 16 lanes x 2 flops (FMA)
# x 2.4 GHz = 78.6 TFLOP/s.
VALU_PEAK_TFLOPS = 256 * 4 * 16 * 2 * 2.4e9 / 1e12
# Algorithmic flops per unit of work: Joseph forward, per ray-step (advance
# the interpolation coordinate 1, fractional part 1, linear interpolation 3,
# accumulate 1); pixel-driven backprojection, per pixel-angle pair (detector
# coordinate 2, fractional part 1, linear interpolation 3, accumulate 1,
# clamp 1).
FLOPS_PER_RAY_STEP = 6
FLOPS_PER_PIXEL_ANGLE = 8
# 3D cone beam: Joseph per plane crossing (advance two coordinates 2,
# fractional parts 2, bilinear interpolation 9, accumulate 1); voxel driven
# per voxel-view pair (denominator 1, magnification 1, detector u and v 4,
# fractional parts 2, bilinear interpolation 9, weight 2, accumulate 1).
FLOPS_PER_CONE_STEP = 14
FLOPS_PER_VOXEL_VIEW = 20
# the 3D workload: 256^3 volume of random ellipsoids, 360 views on [0, 2 pi),
# 384 x 384 detector at pitch 2.1, source-isocentre 500, source-detector 1000,
# 1 % noise, BF16 sinogram, hybrid BA-GMRES with GCV for 50 iterations
CONE = dict(n=256, views=360, nu=384, nv=384, pitch=2.1, sid=500.0, sdd=1000.0, eta=0.01, k=50)
PROFILES = os.path.join(ROOT, "profiles")


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
    p.add_argument("--streams", type=int, default=3,
                   help="the batched solve runs as this many concurrent sub-batches of consecutive slices, each on "
                        "a stream and host thread of its own (bitwise the same results as one)")
    p.add_argument("--plain-slices", type=int, default=8)
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--roofline-reps", type=int, default=10)
    p.add_argument("--counter-k", type=int, default=20,
                   help="iterations of the short solve of --projectors-only")
    p.add_argument("--projectors-only", action="store_true",
                   help="only the projector launches (random images) and a copy of known size, for counter runs")
    p.add_argument("--workload", choices=["slices", "cone", "learned", "variants", "paper"], default="slices",
                   help="slices: the batched 2D workload (default); cone: the 3D cone-beam volume solve; "
                        "learned: train the lambda/stop network on method-generated runs, then compare it "
                        "with GCV + DP; variants: the benchmark batch with restarted cycles and with the NCP "
                        "stop, and the 1024^2 fan-beam problem; paper: single solves at the shapes of the "
                        "paper's Test Problems 2 and 3, every method/rule/restart of its Tables 2-3, k "
                        "iterations each")
    p.add_argument("--train-runs", type=int, default=4096)
    p.add_argument("--train-n", type=int, default=256,
                   help="image size of the learned rule's training runs (angles and bins scale with it: "
                        "720 x 725 at 512)")
    p.add_argument("--eval-slices", type=int, default=1024)
    p.add_argument("--epochs", type=int, default=20)
    p.add_argument("--learned-variants", default="0.05:0",
                   help="learned-rule variants delta:c to evaluate (judge margin delta, discrepancy gate c of the "
                        "stop; comma list, the first is reported)")
    p.add_argument("--no-learned", action="store_true",
                   help="leave out the learned-rule comparison of the default run")
    p.add_argument("--quiet", action="store_true")
    return p.parse_args()


def log(args, *a):
    if not args.quiet:
        print(*a, file=sys.stderr, flush=True)


def synth_batch(pk, A, torch, cfg_id, first, count, n, lo, hi):
    """Seeded phantoms (synthetic, on the GPU) idx = first..first+count-1,
    b = A x + e with ||e|| = eta ||A x||, eta log-uniform in [lo, hi]."""
    import numpy as np

    import synth
    dev = torch.device("cuda")
    x = torch.empty((count, n, n), dtype=torch.float32, device=dev)
    eta = np.empty(count)
    for s in range(count):
        img, _ = synth.phantom2d(cfg_id, first + s, n, device=dev)
        x[s] = img.to(torch.float32)
        eta[s] = synth.noise_level(cfg_id, first + s, lo, hi)
    bt = pk.project(A, x)
    b = torch.empty_like(bt)
    en = np.empty(count)
    m = bt[0].numel()
    for s in range(count):
        g = torch.as_tensor(synth.noise_direction(cfg_id, first + s, m), device=dev, dtype=torch.float64)
        btd = bt[s].double().reshape(-1)
        nb = float(torch.linalg.vector_norm(btd))
        e = (eta[s] * nb / float(torch.linalg.vector_norm(g))) * g
        b[s] = (btd + e).reshape(bt[s].shape).to(torch.float32)
        en[s] = eta[s] * nb
    torch.cuda.synchronize()
    return x, b, torch.tensor(en, dtype=torch.float64, device=dev), eta


def make_inputs(args, pk, A, torch):
    return synth_batch(pk, A, torch, 2, 0, args.slices, args.n, 1e-3, 5e-2)


def rel_l2(a, b):
    import numpy as np
    a = np.asarray(a, dtype=np.float64).ravel()
    b = np.asarray(b, dtype=np.float64).ravel()
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def gcv_gap(lams, o):
    """The largest relative excess of the GCV function (eq. (15)) at the
    GPU's lambda_k over its value at the oracle's, both on the oracle's
    projected problem of iteration k."""
    from oracle import smallsolve as oss
    gaps = [oss.gcv(float(l), *o.small[k]) / oss.gcv(float(o.lam[k]), *o.small[k]) - 1.0
            for k, l in enumerate(lams)]
    return float(max(gaps)) if gaps else 0.0


def dcgs2_bytes(iters, length, elem=4):
    """Algorithmic HBM bytes of the delayed-CGS2 sweeps of a solve: a slice
    stopped at iteration k_s runs steps j = 0..k_s; step j reads the basis
    vectors w_1..w_j, the vector v and M v once in the dot-product sweep
    (j + 2 vectors) and again in the update sweep, which also writes v and M v
    (j + 4 vectors): (2j + 6) vectors of `length` entries."""
    import numpy as np
    k = np.asarray(iters, dtype=np.int64)
    return int(((k + 1) * (k + 6)).sum()) * length * elem


def time_apply(fn, torch, reps=10):
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


def joseph_ray_steps(n, n_angles, n_det, ds=1.0):
    """Ray-steps of one 2D Joseph forward projection: for every ray, the rows
    (of the dominant axis) where at least one interpolation tap lies inside
    the image, i.e. the interpolation coordinate is in (-1, n).  Equally
    spaced angles on [0, pi), centred detector, square n x n image."""
    import numpy as np
    a = np.arange(n_angles)
    th = a * math.pi / n_angles
    rowmarch = (4 * a <= n_angles) | (4 * a >= 3 * n_angles)
    cs, sn = np.cos(th), np.sin(th)
    dom = np.where(rowmarch, cs, sn)
    other = np.where(rowmarch, sn, cs)
    c0 = 0.5 * (n - 1)
    slope = other / dom
    off = c0 * slope + c0
    sd = (np.arange(n_det) - 0.5 * (n_det - 1)) * ds
    u0 = sd[None, :] / dom[:, None] + off[:, None]
    sl = np.broadcast_to(slope[:, None], u0.shape)
    with np.errstate(divide="ignore", invalid="ignore"):
        ra, rb = (u0 + 1) / sl, (u0 - n) / sl
    lo, hi = np.minimum(ra, rb), np.maximum(ra, rb)
    first = np.maximum(0, np.floor(lo) + 1)
    last = np.minimum(n - 1, np.ceil(hi) - 1)
    cnt = np.clip(last - first + 1, 0, None)
    flat = sl == 0
    cnt = np.where(flat, np.where((u0 > -1) & (u0 < n), n, 0), cnt)
    return int(cnt.sum())


SOURCES_2D = ("proj2d.hip", "ops.h")
SOURCES_CONE = ("cone3d.hip", "ops.h")


def kernel_source_digest(files=SOURCES_2D):
    """Digest of the sources that define a family of projector kernels (their
    code and launch constants): the 2D ones by default, SOURCES_CONE for the
    cone-beam pair."""
    import hashlib
    h = hashlib.sha256()
    for name in files:
        with open(os.path.join(ROOT, "paper_2602_17892_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def recorded_counters(kernel, files=SOURCES_2D):
    """The per-launch counter values of `kernel` in its committed summary
    (profiles/<kernel>_traffic.md), or {} when there is none or the projector
    source (`files`) changed since."""
    path = os.path.join(PROFILES, f"{kernel}_traffic.md")
    if not os.path.exists(path):
        return {}
    vals = {}
    with open(path) as f:
        for line in f:
            if line.startswith("- ") and " = " in line:
                k, v = line[2:].split(" = ", 1)
                vals[k.strip()] = v.strip().strip("`")
    if vals.get("source_digest") != kernel_source_digest(files):
        return {}
    return vals


def recorded_traffic(kernel, files=SOURCES_2D):
    """HBM bytes per launch of `kernel` from the committed counter summary, or
    None when there is none or the projector source (`files`) changed since."""
    try:
        return float(recorded_counters(kernel, files)["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def recorded_issue(kernel, files=SOURCES_2D):
    """VALU issue of one launch of `kernel` from the committed counter summary
    (SQ_INSTS_VALU and SQ_BUSY_CU_CYCLES), or None: the cycles a CU is busy per
    wave-level VALU instruction issued on one of its 4 SIMDs (256 CUs, 1,024
    SIMDs).  A wave64 VALU instruction occupies its SIMD for 4 cycles, so a
    kernel near 4 (or below, where instructions co-issue) is bound by issue."""
    vals = recorded_counters(kernel, files)
    try:
        ins, busy = float(vals["valu_instructions_per_launch"]), float(vals["busy_cu_cycles_per_launch"])
    except (KeyError, ValueError):
        return None
    if ins <= 0:
        return None
    return {"valu_instructions": ins, "busy_cu_cycles": busy,
            "cycles_per_valu_per_simd": round((busy / 256) / (ins / 1024), 3)}


def projectors_only(args):
    """The kernels whose counters the profiles record, at the benchmark's batch
    shape: the projectors on seeded random images (and, with --workload cone,
    the cone-beam pair at its shape instead), a short batched solve whose
    Gram-Schmidt sweeps run eagerly (--counter-k iterations, no stop), then
    device copies of a known size (the counter calibration).  Prints the
    algorithmic bytes each kernel family moves."""
    import torch

    import paper_2602_17892_amd as pk
    torch.cuda.set_device(0)
    reps = 3
    gen = torch.Generator(device="cuda")
    gen.manual_seed(2)
    info = {"projectors_only": True, "reps": reps,
            "source_digest": kernel_source_digest(SOURCES_CONE if args.workload == "cone" else SOURCES_2D)}
    if args.workload == "cone":
        C = CONE
        n = C["n"]
        g = pk.Geometry(n, n, C["views"], C["nu"], det_pitch_u=C["pitch"], kind="cone3d", nz=n, det_v=C["nv"],
                        det_pitch_v=C["pitch"], sid=C["sid"], sdd=C["sdd"])
        # the built-in launch rules, as the cone workload runs them
        A = pk.Operator("joseph", g, "f32", "bf16")
        B = pk.Operator("pixel", g, "f32", "bf16")
        x = torch.rand((1, n, n, n), generator=gen, device="cuda")
        y = torch.empty((1, C["views"], C["nv"], C["nu"]), dtype=torch.bfloat16, device="cuda")
        xo = torch.empty_like(x)
        wsa = torch.empty(pk.project_workspace_bytes(A, 1), dtype=torch.uint8, device="cuda")
        wsb = torch.empty(pk.backproject_workspace_bytes(B, 1), dtype=torch.uint8, device="cuda")
        for _ in range(reps):
            pk.project(A, x, out=y, workspace=wsa)
        for _ in range(reps):
            pk.backproject(B, y, out=xo, workspace=wsb)
        info.update(workload="cone", algorithmic_bytes_per_apply=n ** 3 * 4 + C["views"] * C["nu"] * C["nv"] * 2)
    else:
        S = args.slices
        g = pk.Geometry(args.n, args.n, args.angles, args.det)
        A = pk.Operator("joseph", g, "f32", "f32")
        B = pk.Operator("pixel", g, "f32", "f32")
        pk.autotune(A, S)
        pk.autotune(B, S)
        x = torch.rand((S, args.n, args.n), generator=gen, device="cuda")
        y = torch.empty((S, args.angles, args.det), device="cuda")
        xo = torch.empty_like(x)
        wsa = torch.empty(pk.project_workspace_bytes(A, S), dtype=torch.uint8, device="cuda")
        for _ in range(reps):
            pk.project(A, x, out=y, workspace=wsa)
        for _ in range(reps):
            pk.backproject(B, y, out=xo)
        del wsa
        K = args.counter_k
        ws = torch.empty(pk.workspace_bytes(A, B, S, "AB", K), dtype=torch.uint8, device="cuda")
        pk.solve(A, B, y, mode="AB", k=K, reg="gcv", history=False, workspace=ws)
        del ws
        m = args.angles * args.det
        info.update(workload="slices", slices=S, solve_k=K,
                    algorithmic_bytes_per_apply=S * (args.n * args.n + m) * 4,
                    dcgs2_algorithmic_bytes=dcgs2_bytes([K] * S, m))
    for _ in range(reps):
        xo.copy_(x)
    torch.cuda.synchronize()
    info["copy_bytes_each_way"] = x.numel() * 4
    print(json.dumps(info), flush=True)


def cpu_model():
    """The host CPU's model name (from /proc/cpuinfo) and the cores this
    process may use."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count() or 1
    return model, usable


def oracle_threads():
    return int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))


def cpu_baseline(args, b_slice, en_slice, k_cap):
    """The FP64 oracle on one slice of the same workload (same rule and stop).
    Returns its time, its result (projected problems kept for the lambda
    comparison) and the threads it used."""
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
                     noise_norm=float(en_slice), keep_small=True)
    t = time.perf_counter() - t0
    return t, o, oracle_threads()


def cpu_thread_scaling(args):
    """The oracle on all host threads and on one: one A and one B apply at the
    benchmark's slice shape, and the 64^2 configuration's whole solve (90
    angles x 91 bins, 1 % noise, hybrid AB-GMRES with GCV, 30 iterations)."""
    import numpy as np
    from threadpoolctl import threadpool_limits

    import oracle
    import synth
    from oracle.geometry import Par2D
    from oracle.operators import Par2DOps
    from oracle.solver import hybrid_gmres
    oracle.build_oracle(force=False)
    og = Par2DOps(Par2D(args.n, args.n, args.angles, args.det))
    rng = np.random.default_rng(0)
    x = rng.uniform(size=og.n)
    y = rng.standard_normal(og.m)
    o64 = Par2DOps(Par2D(64, 64, 90, 91))
    xt, _ = synth.phantom2d(0, 0, 64)
    b64, _ = synth.add_relative_noise(o64.A(xt).reshape(-1), synth.noise_direction(0, 0, o64.m), 0.01)

    def run():
        t0 = time.perf_counter()
        og.A(x)
        og.B(y)
        t_ab = time.perf_counter() - t0
        t0 = time.perf_counter()
        hybrid_gmres(o64.A, o64.B, b64, mode="AB", K=30, rule="gcv")
        return t_ab, time.perf_counter() - t0

    all_ab, all_c1 = run()
    with threadpool_limits(limits=1):
        one_ab, one_c1 = run()
    return {"threads": oracle_threads(), "AB_apply_pair_s": round(all_ab, 3), "AB_apply_pair_s_1thread":
            round(one_ab, 3), "c1_solve_s": round(all_c1, 3), "c1_solve_s_1thread": round(one_c1, 3)}


def cone_ray_steps(n, views, nu, nv, pitch, sid, sdd):
    """Plane crossings of one cone-beam Joseph projection at which some
    bilinear tap lies inside the n^3 volume: per ray, the planes of its
    dominant axis whose two in-plane coordinates are both in (-1, n)."""
    import numpy as np
    c = 0.5 * (n - 1)
    ou = (np.arange(nu) - 0.5 * (nu - 1)) * pitch
    ov = (np.arange(nv) - 0.5 * (nv - 1)) * pitch
    OU, OV = np.meshgrid(ou, ov)
    total = 0
    for v in range(views):
        b = 2.0 * math.pi * v / views
        S = np.array([sid * math.cos(b), sid * math.sin(b), 0.0])
        D = -(sdd - sid) * np.array([math.cos(b), math.sin(b), 0.0])
        eu = np.array([-math.sin(b), math.cos(b), 0.0])
        d = [D[t] + OU * eu[t] + OV * (1.0 if t == 2 else 0.0) - S[t] for t in range(3)]
        ad = np.stack([np.abs(x) for x in d])
        major = np.where((ad[0] >= ad[1]) & (ad[0] >= ad[2]), 0, np.where(ad[1] >= ad[2], 1, 2))
        for a in range(3):
            sel = major == a
            if not sel.any():
                continue
            da = d[a][sel]
            t0 = (-c - S[a]) / da
            dt = 1.0 / da
            lo = np.zeros(da.shape)
            hi = np.full(da.shape, n - 1.0)
            for o in range(3):
                if o == a:
                    continue
                p0 = S[o] + t0 * d[o][sel] + c
                dp = dt * d[o][sel]
                with np.errstate(divide="ignore", invalid="ignore"):
                    ra, rb = (-1.0 - p0) / dp, (n - p0) / dp
                flat = dp == 0
                inside = (p0 > -1) & (p0 < n)
                l = np.where(flat, np.where(inside, -np.inf, np.inf), np.minimum(ra, rb))
                h = np.where(flat, np.where(inside, np.inf, -np.inf), np.maximum(ra, rb))
                lo = np.maximum(lo, np.floor(l) + 1)
                hi = np.minimum(hi, np.ceil(h) - 1)
            total += int(np.clip(hi - lo + 1, 0, None).sum())
    return total


def cone_cpu_baseline(x_true, b, k):
    """The FP64 oracle's projectors on a bounded sample of the 3D workload
    (A on 4 of the views, B at 2,000 voxels), scaled to one BA solve of k
    iterations: one B for r_0, then one A and one B per iteration."""
    import numpy as np

    import oracle
    from oracle.geometry import Cone3D
    from oracle.operators import Cone3DOps
    oracle.build_oracle(force=False)
    C = CONE
    n = C["n"]
    views = [0, 90, 180, 270]
    beta = 2 * math.pi * np.array(views) / C["views"]
    og_v = Cone3DOps(Cone3D(n, n, n, len(views), C["nu"], C["nv"], C["pitch"], C["pitch"], C["sid"], C["sdd"], beta))
    og = Cone3DOps(Cone3D(n, n, n, C["views"], C["nu"], C["nv"], C["pitch"], C["pitch"], C["sid"], C["sdd"]))
    idx = np.random.default_rng(0).choice(n ** 3, 2000, replace=False)
    t0 = time.perf_counter()
    og_v.A(x_true)
    t_a = (time.perf_counter() - t0) * C["views"] / len(views)
    t0 = time.perf_counter()
    og.B_points(b, idx)
    t_b = (time.perf_counter() - t0) * n ** 3 / len(idx)
    t_solve = (k + 1) * t_b + k * t_a
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return t_solve, t_a, t_b, threads


def cone_workload(args):
    import numpy as np
    import torch

    import paper_2602_17892_amd as pk
    import synth
    torch.cuda.set_device(0)
    C = CONE
    n, K = C["n"], C["k"]
    g = pk.Geometry(n, n, C["views"], C["nu"], det_pitch_u=C["pitch"], kind="cone3d", nz=n, det_v=C["nv"],
                    det_pitch_v=C["pitch"], sid=C["sid"], sdd=C["sdd"])
    A = pk.Operator("joseph", g, "f32", "bf16")
    B = pk.Operator("pixel", g, "f32", "bf16")
    A32 = pk.Operator("joseph", g, "f32", "f32")
    # the built-in launch rules (the tuner's candidates come within about 2 %
    # of them at this size, and the recorded counters are of the built-in)
    t0 = time.perf_counter()
    vol, _ = synth.phantom3d(4, 0, n, device=torch.device("cuda"))
    xt = vol.to(torch.float32).reshape(1, n, n, n).contiguous()
    bt = pk.project(A32, xt).double()
    gn = torch.as_tensor(synth.noise_direction(4, 0, bt.numel()), device="cuda").reshape(bt.shape)
    b = (bt + C["eta"] * torch.linalg.vector_norm(bt) / torch.linalg.vector_norm(gn) * gn).to(torch.bfloat16)
    del bt, gn
    log(args, f"inputs: {n}^3 volume, {C['views']} views of {C['nv']}x{C['nu']} in {time.perf_counter() - t0:.1f}s")
    ws = torch.empty(pk.workspace_bytes(A, B, 1, "BA", K, stop=None), dtype=torch.uint8, device="cuda")

    def step():
        return pk.solve(A, B, b, mode="BA", k=K, reg="gcv", workspace=ws, history=False)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        xk, info = step()
    torch.cuda.synchronize()
    t_solve = (time.perf_counter() - t0) / args.steps
    rre = float(torch.linalg.vector_norm((xk - xt).double()) / torch.linalg.vector_norm(xt.double()))
    log(args, f"BA K={K}: {t_solve:.3f}s/solve, RRE {rre:.4f}")
    y = torch.empty_like(b)
    xo = torch.empty_like(xt)
    wsa = torch.empty(pk.project_workspace_bytes(A, 1), dtype=torch.uint8, device="cuda")
    wsb = torch.empty(pk.backproject_workspace_bytes(B, 1), dtype=torch.uint8, device="cuda")
    t_A = time_apply(lambda: pk.project(A, xt, out=y, workspace=wsa), torch, args.roofline_reps)
    t_B = time_apply(lambda: pk.backproject(B, b, out=xo, workspace=wsb), torch, args.roofline_reps)
    steps = cone_ray_steps(n, C["views"], C["nu"], C["nv"], C["pitch"], C["sid"], C["sdd"])
    pairs = n ** 3 * C["views"]
    tf_A = steps * FLOPS_PER_CONE_STEP / t_A / 1e12
    tf_B = pairs * FLOPS_PER_VOXEL_VIEW / t_B / 1e12
    bytes_apply = n ** 3 * 4 + C["views"] * C["nu"] * C["nv"] * 2
    log(args, f"A: {t_A * 1e3:.2f} ms ({tf_A:.2f} TFLOP/s, {steps} plane crossings); "
              f"B: {t_B * 1e3:.2f} ms ({tf_B:.2f} TFLOP/s)")
    dom = ("cone_fwd_k", tf_A, t_A) if t_A >= t_B else ("cone_bp_k", tf_B, t_B)
    out = {
        "metric": "reconstructed volumes/sec (hybrid BA-GMRES, GCV lambda, 50 iterations, BF16 sinogram)",
        "value": round(1.0 / t_solve, 4),
        "unit": "volumes/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(t_solve * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 projectors+basis, bf16 sinogram storage, f64 reductions and small solves",
        "data": "synthetic: seeded random-ellipsoid volume, b = A x + 1% relative Gaussian noise",
        "config": {"workload": f"{n}^3 cone beam, {C['views']} views x {C['nv']}x{C['nu']} detector at pitch "
                               f"{C['pitch']}, SID {C['sid']:g}, SDD {C['sdd']:g}, hybrid BA-GMRES GCV, k {K}"},
        "rre": rre,
        "launch": "built-in rules",
        "projector": {"A_ms": round(t_A * 1e3, 3), "B_ms": round(t_B * 1e3, 3), "A_TFLOPs": round(tf_A, 3),
                      "B_TFLOPs": round(tf_B, 3), "A_plane_crossings": steps, "B_voxel_view_pairs": pairs,
                      "A_GBps": round(bytes_apply / t_A / 1e9, 2), "B_GBps": round(bytes_apply / t_B / 1e9, 2)},
        "roofline": {"bound": "alu", "achieved": round(dom[1], 3), "peak": round(VALU_PEAK_TFLOPS, 1),
                     "unit": "TFLOP/s", "frac": round(dom[1] / VALU_PEAK_TFLOPS, 4),
                     "traffic": recorded_traffic(dom[0], SOURCES_CONE),
                     "valu_issue": recorded_issue(dom[0], SOURCES_CONE),
                     "kernel": dom[0], "ms_per_launch": round(dom[2] * 1e3, 3)},
    }
    if not args.no_cpu_baseline:
        t_cpu, t_a, t_b, thr = cone_cpu_baseline(xt[0].double().cpu().numpy(), b[0].double().cpu().numpy(), K)
        out["cpu_baseline"] = {"value": round(1.0 / t_cpu, 7), "unit": "volumes/s", "cores": thr, "kind": "oracle",
                               "sample": f"FP64 oracle A on 4 of {C['views']} views ({t_a:.0f}s scaled to all) and B "
                                         f"at 2000 voxels ({t_b:.0f}s scaled to all), times (k+1) B + k A; "
                                         f"orthogonalisation not counted"}
    print(json.dumps(out), flush=True)


def learned_workload(args):
    print(json.dumps(learned_run(args)), flush=True)


def learned_run(args):
    """Training: runs of hybrid AB-GMRES (K = 100, GCV) on 256^2 random-ellipse
    slices, 360 angles x 363 bins (--train-n scales the three), noise
    log-uniform in [0.1%, 5%], with the features and the RRE label grids of
    every iteration; Adam on the network.
    Evaluation: fresh 512^2 slices, 720 x 725, same noise range; GCV + DP
    against the learned lambda and stop (with DP first), batches of 256."""
    import numpy as np
    import torch

    import paper_2602_17892_amd as pk
    import synth
    torch.cuda.set_device(0)
    K, SB = args.kmax, 256
    nt = args.train_n
    gt = pk.Geometry(nt, nt, nt * 360 // 256, math.ceil(nt * math.sqrt(2)))   # 360 x 363 at 256
    At, Bt = pk.Operator("joseph", gt, "f32", "f32"), pk.Operator("pixel", gt, "f32", "f32")
    st = args.streams
    ws = torch.empty(pk.workspace_bytes(At, Bt, SB, "AB", K, labels=True, streams=st), dtype=torch.uint8,
                     device="cuda")
    Xs, Ts, kst = [], [], []
    t0 = time.perf_counter()
    for first in range(0, args.train_runs, SB):
        cnt = min(SB, args.train_runs - first)
        x, b, en, _ = synth_batch(pk, At, torch, 5, first, cnt, nt, 1e-3, 5e-2)
        # ||e|| is known in the training runs as in the solves that use the
        # network (a feature is its level relative to the initial residual)
        _, info = pk.solve(At, Bt, b, mode="AB", k=K, reg="gcv", features=True, x_true=x, workspace=ws,
                           noise_norm=en, history=False, streams=st)
        tg, ks = pk.mlp_labels(info["rre"], info["iters"])
        ok = torch.isfinite(tg.reshape(-1, 2)).all(dim=1)
        Xs.append(info["features"].reshape(-1, 64)[ok])
        Ts.append(tg.reshape(-1, 2)[ok])
        kst.append(ks)
        del x, b, info
    torch.cuda.synchronize()
    t_gen = time.perf_counter() - t0
    del ws
    X = torch.cat(Xs).contiguous()
    T = torch.cat(Ts).contiguous()
    kst = torch.cat(kst).cpu().numpy()
    log(args, f"training data: {args.train_runs} runs -> {X.shape[0]} samples in {t_gen:.1f}s, "
              f"k* mean {kst.mean():.1f} [{kst.min()}, {kst.max()}]")
    theta = torch.as_tensor(synth.mlp_init(0), device="cuda")
    l0, _ = pk.mlp_loss_grad(theta, X, T)
    t0 = time.perf_counter()
    hist = pk.mlp_train(theta, X, T, epochs=args.epochs, batch=4096, lr=1e-3, seed=0,
                        log=(lambda m: log(args, m)) if not args.quiet else None)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    log(args, f"training: loss {float(l0):.4f} -> {hist[-1]:.4f} in {t_train:.1f}s")

    ge = pk.Geometry(512, 512, 720, 725)
    A, B = pk.Operator("joseph", ge, "f32", "f32"), pk.Operator("pixel", ge, "f32", "f32")
    ws = torch.empty(pk.workspace_bytes(A, B, SB, "AB", K, stop="dp", streams=st), dtype=torch.uint8, device="cuda")
    # the learned rule with each (judge margin delta, discrepancy gate c):
    # lambda^ replaces GCV's lambda when GCV(lambda^) <= (1 + delta) min GCV;
    # the stop index is accepted once rho_k <= c tau ||e|| (c = 0: no gate);
    # the first variant is the reported one
    variants = [tuple(float(v) for v in item.split(":")) for item in str(args.learned_variants).split(",")]
    names = ["gcv"] + [f"learned@{d:g}:{c:g}" for d, c in variants]
    res = {name: dict(t=0.0, iters=[], rre=[]) for name in names}
    res["eta"] = []
    for first in range(0, args.eval_slices, SB):
        cnt = min(SB, args.eval_slices - first)
        x, b, en, eta = synth_batch(pk, A, torch, 6, first, cnt, 512, 1e-3, 5e-2)
        res["eta"].append(eta)
        for name in names:
            if name == "gcv":
                kw = dict(reg="gcv", stop="dp")
            else:
                dv, cv = (float(v) for v in name.split("@")[1].split(":"))
                kw = dict(reg="learned", stop="learned", mlp=theta, judge_delta=dv, learned_gate=cv)
            pk.solve(A, B, b[:1].contiguous(), mode="AB", k=2, noise_norm=en[:1], history=False, **kw)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            xr, info = pk.solve(A, B, b, mode="AB", k=K, tau=1.01, noise_norm=en, use_graph=True,
                                poll_every=args.poll, workspace=ws, history=False, streams=st, **kw)
            torch.cuda.synchronize()
            res[name]["t"] += time.perf_counter() - t0
            res[name]["iters"].append(info["iters"].cpu().numpy())
            res[name]["rre"].append((torch.linalg.vector_norm((xr - x).reshape(cnt, -1).double(), dim=1)
                                     / torch.linalg.vector_norm(x.reshape(cnt, -1).double(), dim=1)).cpu().numpy())
        del x, b, en
    res["eta"] = np.concatenate(res["eta"])
    for name in names:
        res[name]["iters"] = np.concatenate(res[name]["iters"])
        res[name]["rre"] = np.concatenate(res[name]["rre"])
    E = args.eval_slices
    for name in names:
        r = res[name]
        extra = ""
        if name != "gcv":
            rt = r["rre"] / res["gcv"]["rre"]
            extra = (f", RRE <= 1.02 x GCV+DP on {np.mean(rt <= 1.02) * 100:.1f}% of slices (worst "
                     f"{rt.max():.3f})")
        log(args, f"{name}: {E / r['t']:.2f} slices/s, iters mean {r['iters'].mean():.1f}, "
                  f"median RRE {np.median(r['rre']):.4f}{extra}")
    sweep = {name: {"slices_per_s": round(E / res[name]["t"], 3), "iters_mean": float(res[name]["iters"].mean()),
                    "frac_within_2pct": float(np.mean(res[name]["rre"] / res["gcv"]["rre"] <= 1.02)),
                    "ratio_max": float((res[name]["rre"] / res["gcv"]["rre"]).max())}
             for name in names[1:]}
    res["learned"] = res[names[1]]
    ratio = res["learned"]["rre"] / res["gcv"]["rre"]
    miss = ratio > 1.02
    out = {
        "metric": "reconstructed slices/sec with the learned lambda and stop index vs GCV + DP",
        "value": round(E / res["learned"]["t"], 3),
        "unit": "slices/s",
        "n_gpus": 1,
        "steps": 1,
        "warmup": 0,
        "ms_per_step": round(res["learned"]["t"] * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 projectors+basis+network, f64 reductions and small solves",
        "data": "synthetic: seeded random-ellipse phantoms; training labels from the true images",
        "config": {"workload": f"train on {args.train_runs} runs at {nt}^2 ({gt.n_angles} x {gt.det_u}, K {K}), evaluate on "
                               f"{E} slices at 512^2 (720 x 725), eta log-uniform [0.1%,5%]",
                   "streams": st},
        "gcv_dp": {"slices_per_s": round(E / res["gcv"]["t"], 3), "iters_mean": float(res["gcv"]["iters"].mean()),
                   "rre_median": float(np.median(res["gcv"]["rre"]))},
        "learned": {"slices_per_s": round(E / res["learned"]["t"], 3),
                    "iters_mean": float(res["learned"]["iters"].mean()),
                    "rre_median": float(np.median(res["learned"]["rre"])),
                    "frac_rre_within_2pct_of_gcv": float(np.mean(ratio <= 1.02)),
                    "rre_ratio_median": float(np.median(ratio)),
                    "rre_ratio_p95": float(np.percentile(ratio, 95)),
                    "rre_ratio_max": float(ratio.max()),
                    "variant_sweep": sweep if len(variants) > 1 else None,
                    "misses": int(miss.sum()),
                    "miss_eta": [float(e) for e in np.sort(res["eta"][miss])[:64]]},
        "speedup_learned_vs_gcv_dp": round(res["gcv"]["t"] / res["learned"]["t"], 3),
        "judge_delta": variants[0][0],
        "learned_gate": variants[0][1],
        "training": {"runs": args.train_runs, "samples": int(X.shape[0]), "epochs": args.epochs,
                     "loss_start": float(l0), "loss_end": hist[-1], "data_s": round(t_gen, 2),
                     "train_s": round(t_train, 2), "k_star_mean": float(kst.mean())},
    }
    return out


def tune_sub_batches(pk, A, B, S, streams):
    """Launch choices of A and B at the sub-batch sizes of a batch of S slices
    split into `streams` concurrent sub-batches (their projector launches run
    at those batch sizes)."""
    p = max(1, min(streams, S))
    out = {}
    for sz in sorted({S // p + (1 if i < S % p else 0) for i in range(p)} - {S, 1}):
        out[f"A_sub{sz}"] = pk.autotune(A, sz)
        out[f"B_sub{sz}"] = pk.autotune(B, sz)
    return out


def variants_workload(args):
    """The 256 x 512^2 batch (in --streams concurrent sub-batches) with
    hybrid BA-GMRES (GCV, DP stop, at most 100), with restarted cycles of 20
    (AB, GCV, DP stop, 100 iterations in all) and with the NCP stop (AB, GCV,
    at most 100), and one
    1024^2 fan-beam slice (50 views, 1,024 bins of 3, SID 2048, SDD 4096,
    1.5 % noise, AB with GCV and DP stop) beside the oracle's time for it."""
    import numpy as np
    import torch

    import paper_2602_17892_amd as pk
    import synth
    torch.cuda.set_device(0)
    S, K = args.slices, args.kmax
    g = pk.Geometry(args.n, args.n, args.angles, args.det)
    A, B = pk.Operator("joseph", g, "f32", "f32"), pk.Operator("pixel", g, "f32", "f32")
    pk.autotune(A, S)
    pk.autotune(B, S)
    tune_sub_batches(pk, A, B, S, args.streams)
    st = args.streams
    x, b, en, _ = make_inputs(args, pk, A, torch)
    out = {"metric": "BA / restarted / NCP / fan-beam variants", "config": {"workload": f"{S} x {args.n}^2 slices "
           f"({args.angles} x {args.det}) and one 1024^2 fan-beam slice", "streams": st}}

    def rre(xr, xt):
        n = xr.shape[0]
        return (torch.linalg.vector_norm((xr - xt).reshape(n, -1).double(), dim=1)
                / torch.linalg.vector_norm(xt.reshape(n, -1).double(), dim=1)).cpu().numpy()

    for name, mode, kw, p in (("plain", "AB", dict(stop="dp", noise_norm=en), 0),
                              ("ba", "BA", dict(stop="dp", noise_norm=en), 0),
                              ("restart20", "AB", dict(stop="dp", noise_norm=en), 20),
                              ("ncp", "AB", dict(stop="ncp"), 0)):
        ws = torch.empty(pk.workspace_bytes(A, B, S, mode, K, stop=kw["stop"], restart=p, streams=st),
                         dtype=torch.uint8, device="cuda")
        run = lambda: pk.solve(A, B, b, mode=mode, k=K, reg="gcv", tau=1.01, use_graph=True, poll_every=args.poll,
                               workspace=ws, history=False, restart=p, streams=st, **kw)
        run()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        xr, info = run()
        torch.cuda.synchronize()
        t = time.perf_counter() - t0
        it = info["iters"].cpu().numpy()
        out[name] = {"slices_per_s": round(S / t, 3), "workspace_gib": round(ws.numel() / 2 ** 30, 2),
                     "iters_mean": float(it.mean()), "rre_median": float(np.median(rre(xr, x)))}
        log(args, f"{name}: {S / t:.2f} slices/s, workspace {ws.numel() / 2 ** 30:.1f} GiB, iters mean "
                  f"{it.mean():.1f}, median RRE {out[name]['rre_median']:.4f}")
        del ws, xr
    # the fan-beam problem (the shape of the paper's third test problem)
    gf = pk.Geometry(1024, 1024, 50, 1024, det_pitch_u=3.0, kind="fan2d", sid=2048.0, sdd=4096.0)
    Af, Bf = pk.Operator("joseph", gf, "f32", "f32"), pk.Operator("pixel", gf, "f32", "f32")
    xf, bf, enf, _ = synth_batch(pk, Af, torch, 9, 0, 1, 1024, 0.015, 0.015)
    runf = lambda: pk.solve(Af, Bf, bf, mode="AB", k=K, reg="gcv", stop="dp", tau=1.01, noise_norm=enf,
                            history=False)
    runf()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(5):
        xs, info = runf()
    torch.cuda.synchronize()
    tf = (time.perf_counter() - t0) / 5
    fan = {"seconds": round(tf, 4), "iters": int(info["iters"][0]), "rre": float(rre(xs, xf)[0])}
    if not args.no_cpu_baseline:
        import oracle
        from oracle.geometry import FanFlat2D
        from oracle.operators import FanFlat2DOps
        from oracle.solver import hybrid_gmres
        oracle.build_oracle(force=False)
        og = FanFlat2DOps(FanFlat2D(1024, 1024, 50, 1024, 3.0, 2048.0, 4096.0))
        t0 = time.perf_counter()
        o = hybrid_gmres(og.A, og.B, bf[0].double().cpu().numpy().ravel(), mode="AB", K=K, rule="gcv", stop="dp",
                         noise_norm=float(enf[0]))
        fan["oracle_seconds"] = round(time.perf_counter() - t0, 3)
        fan["oracle_iters"] = o.iters
        fan["oracle_cores"] = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    out["fan_1024"] = fan
    log(args, f"fan 1024^2 x 50 views: {tf * 1e3:.1f} ms per solve, {fan['iters']} iterations, RRE {fan['rre']:.4f}")
    print(json.dumps(out), flush=True)


def paper_workload(args):
    """One slice per solve at the shapes of the paper's Test Problem 2 (128^2,
    parallel beam, 50 angles x 128 bins, 2.5 % noise) and Test Problem 3
    (1024^2, fan beam with a flat detector, 50 views x 1,024 bins of 3, SID
    2048, SDD 4096, 1.5 % noise), seeded random-ellipse phantoms in place of
    the paper's; hybrid AB- and BA-GMRES with no lambda, the L-curve and GCV,
    without restarts and with cycles of 10, each run for --kmax iterations
    with no stopping rule.  Seconds per solve (mean of 3 after one warm-up),
    to set beside the paper's Tables 2-3 (another machine and an iteration
    count the paper does not state: context, not a comparison of equals)."""
    import numpy as np
    import torch

    import paper_2602_17892_amd as pk
    torch.cuda.set_device(0)
    K = args.kmax
    probs = {"tp2": (pk.Geometry(128, 128, 50, 128), 128, 0.025),
             "tp3": (pk.Geometry(1024, 1024, 50, 1024, det_pitch_u=3.0, kind="fan2d", sid=2048.0, sdd=4096.0),
                     1024, 0.015)}
    out = {"metric": "seconds per single-slice solve at the shapes of the paper's Test Problems 2-3",
           "config": {"k": K, "stop": "none (k iterations)", "data": "synthetic random-ellipse phantoms",
                      "dtype": "f32 projectors+basis, f64 reductions and small solves"}}
    for name, (g, n, eta) in probs.items():
        A, B = pk.Operator("joseph", g, "f32", "f32"), pk.Operator("pixel", g, "f32", "f32")
        x, b, en, _ = synth_batch(pk, A, torch, 11, 0, 1, n, eta, eta)
        res = {}
        for mode in ("AB", "BA"):
            for rule in ("none", "lcurve", "gcv"):
                for restart in (0, 10):
                    run = lambda: pk.solve(A, B, b, mode=mode, k=K, reg=rule, restart=restart, history=False)
                    run()
                    torch.cuda.synchronize()
                    t0 = time.perf_counter()
                    for _ in range(3):
                        xr, info = run()
                    torch.cuda.synchronize()
                    t = (time.perf_counter() - t0) / 3
                    rre = float(torch.linalg.vector_norm((xr - x).double()) / torch.linalg.vector_norm(x.double()))
                    key = f"{mode}_{rule}_r{restart}"
                    res[key] = {"seconds": round(t, 5), "iters": int(info["iters"][0]), "rre": round(rre, 4)}
                    log(args, f"{name} {key}: {t * 1e3:.2f} ms, {int(info['iters'][0])} iterations, RRE {rre:.4f}")
        out[name] = res
    print(json.dumps(out), flush=True)


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "bench.py runs on one GPU: the slices of the batched workload are "
                          "independent and would shard with no communication, but only the one-GPU path "
                          "exists; rerun with --gpus 1"}))
        sys.exit(2)
    import numpy as np
    import torch

    import paper_2602_17892_amd as pk
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.projectors_only:
        projectors_only(args)
        return
    if args.workload == "cone":
        cone_workload(args)
        return
    if args.workload == "learned":
        learned_workload(args)
        return
    if args.workload == "variants":
        variants_workload(args)
        return
    if args.workload == "paper":
        paper_workload(args)
        return
    torch.cuda.set_device(0)
    S, K = args.slices, args.kmax
    g = pk.Geometry(args.n, args.n, args.angles, args.det)
    A = pk.Operator("joseph", g, "f32", "f32")
    B = pk.Operator("pixel", g, "f32", "f32")
    t0 = time.perf_counter()
    x_true, b, en, eta = make_inputs(args, pk, A, torch)
    log(args, f"inputs: {S} slices of {args.n}^2, {args.angles}x{args.det} in {time.perf_counter() - t0:.1f}s")

    # launch choices of the projectors for this batch size and for single
    # slices (the plain path), timed before anything is measured
    t0 = time.perf_counter()
    tune = {"A": pk.autotune(A, S), "B": pk.autotune(B, S), "A_plain": pk.autotune(A, 1), "B_plain": pk.autotune(B, 1)}
    P_st = max(1, min(args.streams, S))
    tune.update(tune_sub_batches(pk, A, B, S, args.streams))
    log(args, f"autotune ({time.perf_counter() - t0:.1f}s): " + "; ".join(
        f"{k} {v['ms']:.3f} ms (built-in {v['default_ms']:.3f})" for k, v in tune.items()))
    # one workspace serves the sub-batched timed solve and the one-stream
    # phase-timed solve below
    ws_bytes = max(pk.workspace_bytes(A, B, S, "AB", K, stop="dp", streams=args.streams),
                   pk.workspace_bytes(A, B, S, "AB", K, stop="dp"))
    ws = torch.empty(ws_bytes, dtype=torch.uint8, device="cuda")
    log(args, f"workspace {ws_bytes / 2**30:.1f} GiB, {P_st} sub-batch stream(s)")

    def step():
        return pk.solve(A, B, b, mode="AB", k=K, reg="gcv", tau=1.01, noise_norm=en, stop="dp",
                        use_graph=True, poll_every=args.poll, workspace=ws, history=False, streams=args.streams)

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
    # the subset's mean iteration count differs from the batch's: compare per
    # iteration as well as per slice
    it_plain = float(np.mean(plain_iters))
    t_plain_iter = t_plain / it_plain
    t_batched_iter = t_batched / (S * float(iters.mean()))
    log(args, f"plain: {t_plain:.3f}s/slice on {P} slices ({it_plain:.1f} iterations on average), bitwise equal "
              f"to batched: {same}")

    # ---- the same batched solve once more with its phases timed by HIP
    # events (eager launches, one stream; not part of the timed steps): the
    # Gram-Schmidt sweeps' bandwidth over the whole solve
    xp, ip = pk.solve(A, B, b, mode="AB", k=K, reg="gcv", tau=1.01, noise_norm=en, stop="dp", poll_every=args.poll,
                      workspace=ws, history=False, phases=True)
    same_p = bool(torch.equal(xp, xb))
    phase_ms = ip["phase_ms"]
    it_p = ip["iters"].cpu().numpy().astype(np.int64)
    cgs_bytes = dcgs2_bytes(it_p, args.angles * args.det)
    t_cgs = phase_ms["ortho"] / 1e3
    cgs = {"bytes": int(cgs_bytes), "seconds": round(t_cgs, 4), "TBps": round(cgs_bytes / t_cgs / 1e12, 3),
           "frac_hbm": round(cgs_bytes / t_cgs / 1e9 / HBM_PEAK_GBS, 4)}
    log(args, "phases (ms): " + ", ".join(f"{k} {v:.1f}" for k, v in phase_ms.items()) +
        f"; Gram-Schmidt sweeps {cgs_bytes / 1e12:.2f} TB in {t_cgs:.3f}s = {cgs['TBps']:.2f} TB/s; "
        f"same x as the graph run: {same_p}")
    del xp, ip

    # ---- projector launches over the whole batch, event-timed on the stream
    # they run on (the same launch shape as inside the solve)
    xin = x_true.contiguous()
    yb = torch.empty_like(b)
    xo = torch.empty_like(xin)
    wsa = torch.empty(pk.project_workspace_bytes(A, S), dtype=torch.uint8, device="cuda")
    t_A = time_apply(lambda: pk.project(A, xin, out=yb, workspace=wsa), torch, args.roofline_reps)
    t_B = time_apply(lambda: pk.backproject(B, b, out=xo), torch, args.roofline_reps)
    del wsa
    n, m = args.n * args.n, args.angles * args.det
    bytes_apply = S * (n + m) * 4
    gbs_A, gbs_B = bytes_apply / t_A / 1e9, bytes_apply / t_B / 1e9
    pairs = S * n * args.angles
    steps = S * joseph_ray_steps(args.n, args.angles, args.det)
    tf_A = steps * FLOPS_PER_RAY_STEP / t_A / 1e12
    tf_B = pairs * FLOPS_PER_PIXEL_ANGLE / t_B / 1e12
    log(args, f"A: {t_A * 1e3:.2f} ms ({gbs_A:.1f} GB/s, {tf_A:.2f} TFLOP/s); "
              f"B: {t_B * 1e3:.2f} ms ({gbs_B:.1f} GB/s, {tf_B:.2f} TFLOP/s)")
    # A runs the kernel its tuning chose (the built-in rule takes the LDS-band
    # kernel at this batch size); B runs pixbp2d_k
    a_name = "joseph2d_fwd_k" if tune["A"]["a_path"] == 0 else "joseph2d_lds_k"
    if t_A >= t_B:
        dom_name, dom_tf, dom_t = a_name, tf_A, t_A
    else:
        dom_name, dom_tf, dom_t = "pixbp2d_k", tf_B, t_B
    roofline = {"bound": "alu", "achieved": round(dom_tf, 3), "peak": round(VALU_PEAK_TFLOPS, 1),
                "unit": "TFLOP/s", "frac": round(dom_tf / VALU_PEAK_TFLOPS, 4),
                "traffic": recorded_traffic(dom_name), "valu_issue": recorded_issue(dom_name), "kernel": dom_name,
                "ms_per_launch": round(dom_t * 1e3, 3)}

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
                   "slices": S, "kmax": K, "poll_every": args.poll, "streams": P_st},
        "iters": {"mean": float(iters.mean()), "min": int(iters.min()), "max": int(iters.max()),
                  "status_dp": int((status & 2 != 0).sum())},
        "rre_median": float(np.median(rre_b)),
        "plain": {"slices_per_s": round(1.0 / t_plain, 3), "subset": [int(s) for s in idx],
                  "iters_mean_subset": it_plain, "bitwise_equal_to_batched": same,
                  "speedup_batched_vs_plain": round(value * t_plain, 3),
                  "speedup_per_iteration": round(t_plain_iter / t_batched_iter, 3)},
        "phases_ms": {k: round(v, 2) for k, v in phase_ms.items()},
        "cgs2": cgs,
        "projector": {"A_GBps": round(gbs_A, 2), "A_frac_hbm": round(gbs_A / HBM_PEAK_GBS, 5),
                      "B_GBps": round(gbs_B, 2), "B_frac_hbm": round(gbs_B / HBM_PEAK_GBS, 5),
                      "A_ms_batch": round(t_A * 1e3, 3), "B_ms_batch": round(t_B * 1e3, 3),
                      "B_Gpairs_per_s": round(pairs / t_B / 1e9, 2),
                      "A_TFLOPs": round(tf_A, 3), "B_TFLOPs": round(tf_B, 3), "A_ray_steps": steps,
                      "B_pixel_angle_pairs": pairs},
        "roofline": roofline,
        "autotune": {k: {"choice": {c: v[c] for c in ("a_path", "a_jb", "b_g", "czt", "a_rb", "a_occ")}, "ms": round(v["ms"], 3),
                         "builtin_ms": round(v["default_ms"], 3)} for k, v in tune.items()},
    }
    if not args.no_learned:
        # train the lambda/stop network on method-generated runs, then solve
        # fresh slices with it and with GCV + DP (its own batches and
        # workspaces; the benchmark's are released first)
        del ws
        torch.cuda.empty_cache()
        lr = learned_run(args)
        out["learned"] = {k: lr[k] for k in ("config", "gcv_dp", "learned", "speedup_learned_vs_gcv_dp",
                                             "judge_delta", "learned_gate", "training")}
        out["learned"]["speedup_learned_vs_plain"] = round(lr["learned"]["slices_per_s"] * t_plain, 3)
    if not args.no_cpu_baseline:
        s0 = int(np.argsort(iters)[len(iters) // 2])
        # the GPU's lambda history of that slice: the plain path gives the
        # batched run's bits (checked above on the subset)
        x1, i1 = pk.solve(A, B, b[s0:s0 + 1], mode="AB", k=K, reg="gcv", tau=1.01, noise_norm=en[s0:s0 + 1],
                          stop="dp", workspace=ws1, history=True)
        lam_gpu = i1["lam"][0].cpu().numpy()
        same_s0 = bool(torch.equal(x1[0], xb[s0]))
        t_cpu, o, thr = cpu_baseline(args, b[s0].double().cpu().numpy(), float(en[s0]), K)
        model, usable = cpu_model()
        out["cpu_baseline"] = {"value": round(1.0 / t_cpu, 5), "unit": "slices/s", "cores": thr, "kind": "oracle",
                               "sample": f"1 slice (index {s0}, median GPU stop iteration {int(iters[s0])}) "
                                         f"solved to its DP stop by the FP64 oracle: {t_cpu:.1f}s, "
                                         f"{o.iters} iterations",
                               "cpu_model": model, "usable_cores": usable}
        out["cpu_baseline"]["thread_scaling"] = cpu_thread_scaling(args)
        xg = xb[s0].double().cpu().numpy().ravel()
        k_common = min(o.iters, int(iters[s0]))
        out["parity"] = {"slice": s0, "x_rel_vs_oracle": rel_l2(xg, o.x), "gpu_iters": int(iters[s0]),
                         "oracle_iters": o.iters, "same_stop": int(iters[s0]) == o.iters,
                         "same_status": int(status[s0]) == o.status,
                         "lambda_gcv_gap": gcv_gap(lam_gpu[:k_common], o), "plain_equals_batched": same_s0,
                         "rre_gpu": float(rre_b[s0]), "rre_oracle": rel_l2(o.x, x_true[s0].double().cpu().numpy())}
        log(args, f"parity, slice {s0}: x vs oracle {out['parity']['x_rel_vs_oracle']:.2e}, stop "
                  f"{int(iters[s0])}/{o.iters}, GCV gap {out['parity']['lambda_gcv_gap']:.1e}")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
