"""The benchmark's batch in the benchmark's launch configuration: 256 slices of
512^2, 720 angles x 725 bins, FP32 (the built-in launch choice at this batch is
the LDS-band A kernel over an XCD-remapped grid, which no single-slice case
reaches).  Sampled slices are compared with the FP64 oracle one by one (gate
1e-5 relative for the projectors, 1e-4 for a short solve, as at one slice) and
with the single-slice launches bit for bit.
"""
import numpy as np
import pytest

import synth
from oracle import solver as osv
from oracle.geometry import Par2D
from oracle.operators import Par2DOps

pytestmark = [pytest.mark.gpu, pytest.mark.usefixtures("oracle_lib")]

torch = pytest.importorskip("torch")

S, N, NA, ND = 256, 512, 720, 725
SAMPLE = (0, 97, 255)


@pytest.fixture(scope="module")
def pk():
    import paper_2602_17892_amd as pk
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return pk


@pytest.fixture(scope="module")
def full(pk):
    g = pk.Geometry(N, N, NA, ND)
    A = pk.Operator("joseph", g, "f32", "f32")
    B = pk.Operator("pixel", g, "f32", "f32")
    og = Par2DOps(Par2D(N, N, NA, ND))
    dev = torch.device("cuda")
    x = torch.empty((S, N, N), dtype=torch.float32, device=dev)
    for s in range(S):
        x[s] = synth.phantom2d(2, s, N, device=dev)[0].to(torch.float32)
    return A, B, og, x


def rel(a, b):
    """The larger of the relative L2 error and max|a - b| / max|b|: a wrong
    value on a few bins hides in the first but not in the second."""
    a = np.asarray(a, dtype=np.float64).ravel()
    b = np.asarray(b, dtype=np.float64).ravel()
    l2 = np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)
    mx = np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300) if b.size else 0.0
    return float(max(l2, mx))


def test_full_batch_projectors(pk, full):
    A, B, og, x = full
    y = pk.project(A, x)
    xb = pk.backproject(B, y)
    for s in SAMPLE:
        xs = x[s].double().cpu().numpy()
        ys = y[s].double().cpu().numpy()
        ea = rel(ys, og.A(xs))
        eb = rel(xb[s].double().cpu().numpy(), og.B(ys))
        # the single-slice launch (gather kernel for A) gives the same bits
        same_a = torch.equal(pk.project(A, x[s:s + 1].contiguous())[0], y[s])
        same_b = torch.equal(pk.backproject(B, y[s:s + 1].contiguous())[0], xb[s])
        print(f"slice {s}: A {ea:.2e} B {eb:.2e}; single-slice launches bitwise equal: {same_a} {same_b}")
        assert ea <= 1e-5 and eb <= 1e-5
        assert same_a and same_b
    assert bool(torch.isfinite(y).all()) and bool(torch.isfinite(xb).all())


def test_full_batch_solve(pk, full):
    A, B, og, x = full
    K = 4
    y = pk.project(A, x)
    gen = torch.Generator(device="cuda").manual_seed(11)
    e = torch.randn(y.shape, generator=gen, device="cuda", dtype=torch.float32)
    b = (y + 0.01 * e * (y.reshape(S, -1).norm(dim=1) / e.reshape(S, -1).norm(dim=1)).reshape(S, 1, 1)).contiguous()
    xk, info = pk.solve(A, B, b, mode="AB", k=K, reg="gcv")
    assert bool((info["iters"] == K).all())
    for s in SAMPLE:
        bs = b[s].double().cpu().numpy().ravel()
        o = osv.hybrid_gmres(og.A, og.B, bs, mode="AB", K=K, rule="gcv")
        ex = rel(xk[s].double().cpu().numpy(), o.x)
        x1, _ = pk.solve(A, B, b[s:s + 1].contiguous(), mode="AB", k=K, reg="gcv")
        same = torch.equal(x1[0], xk[s])
        print(f"slice {s}: AB K={K} x vs oracle {ex:.2e}; single-slice solve bitwise equal: {same}")
        assert ex <= 1e-4 and same
