"""Parity at the configurations' real iteration counts.

* 512^2 FP32, 720 angles x 725 bins, 0.5 % noise: hybrid AB- and BA-GMRES
  with the GCV lambda (eq. (15)) for the full 100 iterations, one slice on the
  plain single-slice path, against the FP64 oracle.
* The benchmark batch in the benchmark's launch configuration (256 slices of
  512^2, 720 x 725, noise log-uniform in [0.1 %, 5 %], AB, GCV, discrepancy
  stop with tau = 1.01, at most 100 iterations, graph replay, polling every 4
  iterations): three slices (the earliest discrepancy stop, the median one,
  and one that runs to the budget) against the oracle run to its own stop.

Gate on x: 1e-4 relative, or 3x the FP32 floor where that is larger.  The
FP32 floor is the oracle's own deviation when its projector outputs carry
the GPU's error (each output rounded to FP32 and perturbed by the measured
projector error 3e-6; for the single slice also rounding alone) at the same
iteration count;
every case prints its error and its floor.  rho_k and lambda_k (judged by
its GCV value on the oracle's projected problems) are gated at 3x the same
emulated runs' deviations.  The stopping iteration must be the oracle's, or
differ by one with the GPU's residual at the earlier stop on the other side
of the threshold tau ||e|| than the oracle's, by a deviation from the
oracle's residual no larger than 3x the FP32-emulated oracle's (+1e-4): a
tie that the storage precision decides; x is then compared at the GPU's
stop.
"""
import numpy as np
import pytest

import synth
from oracle import smallsolve as oss
from oracle import solver as osv
from oracle.geometry import Par2D
from oracle.operators import Par2DOps

pytestmark = [pytest.mark.gpu, pytest.mark.usefixtures("oracle_lib")]

torch = pytest.importorskip("torch")

N, NA, ND = 512, 720, 725


@pytest.fixture(scope="module")
def pk():
    import paper_2602_17892_amd as pk
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return pk


def rel(a, b):
    a = np.asarray(a, dtype=np.float64).ravel()
    b = np.asarray(b, dtype=np.float64).ravel()
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def r32(v):
    return np.asarray(v, dtype=np.float32).astype(np.float64)


def perturbed_ops(og, d, seed):
    """The oracle's projectors with FP32 storage of every input and output and
    a random relative perturbation of size d on every output."""
    rng = np.random.default_rng(seed)

    def pert(y):
        return y * (1.0 + d * rng.uniform(-1.0, 1.0, y.shape)) if d else y

    return (lambda v: r32(pert(og.A(r32(v))))), (lambda v: r32(pert(og.B(r32(v)))))


def gcv_gap(lams, o):
    gaps = []
    for k in range(len(lams)):
        sig, uh, uk1 = o.small[k]
        gaps.append(oss.gcv(float(lams[k]), sig, uh, uk1) / oss.gcv(float(o.lam[k]), sig, uh, uk1) - 1.0)
    return float(max(gaps)) if gaps else 0.0


@pytest.mark.timeout(900)
@pytest.mark.parametrize("mode", ["AB", "BA"])
def test_c2_full_100_iterations(pk, mode):
    g = pk.Geometry(N, N, NA, ND)
    A = pk.Operator("joseph", g, "f32", "f32")
    B = pk.Operator("pixel", g, "f32", "f32")
    og = Par2DOps(Par2D(N, N, NA, ND))
    xt, _ = synth.phantom2d(1, 0, N)
    b, en = synth.add_relative_noise(og.A(xt).reshape(-1), synth.noise_direction(1, 0, og.m), 0.005)
    bd = torch.as_tensor(b).to(device="cuda", dtype=torch.float32).reshape(1, NA, ND)
    bu = bd.double().cpu().numpy().ravel()
    K = 100
    x, info = pk.solve(A, B, bd, mode=mode, k=K, reg="gcv")
    xg = x.double().cpu().numpy().ravel()
    lam = info["lam"][0].cpu().numpy()
    rho = info["resid"][0].cpu().numpy()
    print(f"[C2 {mode}] GPU done, running the oracle", flush=True)
    o = osv.hybrid_gmres(og.A, og.B, bu, mode=mode, K=K, rule="gcv", keep_small=True)
    floors, frho, flam = [], [], []
    for d, seed in ((0.0, 0), (3e-6, 1)):
        Ap, Bp = perturbed_ops(og, d, seed)
        emu = osv.hybrid_gmres(Ap, Bp, bu, mode=mode, K=K, rule="gcv")
        floors.append(rel(emu.x, o.x))
        frho.append(rel(emu.rho, o.rho))
        flam.append(gcv_gap(emu.lam, o))
    ex = rel(xg, o.x)
    er = rel(rho, o.rho)
    gl = gcv_gap(lam, o)
    gate = max(1e-4, 3.0 * max(floors))
    grho = max(1e-4, 3.0 * max(frho))
    glam = max(1e-6, 3.0 * max(flam))
    print(f"C2 {mode} GCV K={K}: x {ex:.2e} (gate {gate:.1e}; FP32 floor {floors[0]:.2e} rounding, "
          f"{floors[1]:.2e} with projector error), rho {er:.2e} (gate {grho:.1e}), GCV-value gap {gl:.1e} "
          f"(gate {glam:.1e}), RRE {rel(xg, xt):.4f} (oracle {rel(o.x, xt):.4f})")
    assert int(info["iters"][0]) == K == o.iters
    assert ex <= gate and er <= grho and gl <= glam


@pytest.mark.timeout(1200)
def test_benchmark_slices_to_their_dp_stop(pk):
    import bench
    S, K = 256, 100
    g = pk.Geometry(N, N, NA, ND)
    A = pk.Operator("joseph", g, "f32", "f32")
    B = pk.Operator("pixel", g, "f32", "f32")
    x, b, en, eta = bench.synth_batch(pk, A, torch, 2, 0, S, N, 1e-3, 5e-2)
    ws = torch.empty(pk.workspace_bytes(A, B, S, "AB", K, stop="dp"), dtype=torch.uint8, device="cuda")
    xb, info = pk.solve(A, B, b, mode="AB", k=K, reg="gcv", tau=1.01, noise_norm=en, stop="dp", use_graph=True,
                        poll_every=4, workspace=ws, history=False)
    iters = info["iters"].cpu().numpy()
    status = info["status"].cpu().numpy()
    dp = np.flatnonzero(status & pk.ST_STOP_DP)
    kmax = np.flatnonzero(status == pk.ST_KMAX)
    assert dp.size and kmax.size
    order = dp[np.argsort(iters[dp], kind="stable")]
    picks = [int(order[0]), int(order[len(order) // 2]), int(kmax[0])]
    cases = {s: (xb[s].double().cpu().numpy().ravel(), b[s].double().cpu().numpy().ravel(), float(en[s]),
                 x[s].double().cpu().numpy().ravel(), int(iters[s]), int(status[s])) for s in picks}
    del ws, xb, x, b
    torch.cuda.empty_cache()
    og = Par2DOps(Par2D(N, N, NA, ND))
    # the FP32 model: storage rounding and the measured projector error
    Ap, Bp = perturbed_ops(og, 3e-6, 1)
    bad = []
    for s, (xg, bs, es, xt, it, st) in cases.items():
        print(f"[slice {s}] GPU stop {it} (status {st}), running the oracle", flush=True)
        target = 1.01 * es
        o = osv.hybrid_gmres(og.A, og.B, bs, mode="AB", K=K, rule="gcv", stop="dp", tau=1.01, noise_norm=es)
        k0, k1 = min(it, o.iters), max(it, o.iters)
        # the FP32-modelled oracle run to the later stop: the x floor at the
        # GPU's stop and the residual's FP32 uncertainty at every iteration
        emu = osv.hybrid_gmres(Ap, Bp, bs, mode="AB", K=k1, rule="gcv")
        if it == o.iters:
            oi = o
            tie, note = False, ""
        else:
            # the stops differ: at every iteration from the earlier stop up to
            # the later one, the oracle's residual and the GPU's projected
            # residual (its plain single-slice path gives the batched bits)
            # must lie within the FP32 uncertainty of the residual (3x the
            # modelled oracle's deviation, + 1e-4) of the threshold and of
            # each other: the stopping decision there is one FP32 cannot make
            ofull = osv.hybrid_gmres(og.A, og.B, bs, mode="AB", K=k1, rule="gcv")
            oi = osv.hybrid_gmres(og.A, og.B, bs, mode="AB", K=it, rule="gcv") if it < k1 else ofull
            x1, i1 = pk.solve(A, B, torch.as_tensor(bs, dtype=torch.float32, device="cuda").reshape(1, NA, ND),
                              mode="AB", k=K, reg="gcv", tau=1.01, stop="dp",
                              noise_norm=torch.tensor([es], dtype=torch.float64, device="cuda"))
            rho_gpu = i1["resid"][0].cpu().numpy()
            same = np.array_equal(x1[0].double().cpu().numpy().ravel(), xg)
            rows, tie = [], same
            for kk in range(k0, k1):
                band = 3.0 * abs(emu.rho[kk] / ofull.rho[kk] - 1.0) + 1e-4
                mo = abs(ofull.rho[kk] / target - 1.0)
                mg = abs(rho_gpu[kk] / ofull.rho[kk] - 1.0)
                rows.append(f"k={kk}: oracle {mo:.1e} from tau||e||, GPU {mg:.1e} from the oracle, band {band:.1e}")
                tie = tie and mo <= band and mg <= band
            note = f" ({'tie' if tie else 'not a tie'}: " + "; ".join(rows) + f"; plain run bitwise equal: {same})"
        floor = rel(emu.x if it == k1 else osv.hybrid_gmres(Ap, Bp, bs, mode="AB", K=it, rule="gcv").x, oi.x)
        ex = rel(xg, oi.x)
        gate = max(1e-4, 3.0 * floor)
        print(f"slice {s}: stop GPU {it} / oracle {o.iters}{note}, status {st} / {o.status}, x {ex:.2e} "
              f"(gate {gate:.1e}, FP32 floor {floor:.2e}), RRE {rel(xg, xt):.4f} (oracle {rel(o.x, xt):.4f})",
              flush=True)
        if not ((it == o.iters and st == o.status) or tie) or ex > gate:
            bad.append(s)
    assert not bad, bad
