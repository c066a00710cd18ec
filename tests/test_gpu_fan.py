"""GPU parity of the 2D fan-beam (flat detector) projectors and solves against
the FP64 oracle (oracle.operators.FanFlat2DOps: a separate plain-C 2D
definition; the GPU runs the cone-beam kernels on the image plane).

Gates: relative L2 <= 1e-12 (FP64) and <= 1e-5 (FP32) for A and B; BF16
sinogram storage within one BF16 rounding; FP64 solves <= 1e-8.  The largest
case is the shape of the paper's third test problem (1024^2 image, 50 views,
1,024 bins; the paper gives no source distances, so SID = 2N and SDD = 4N
with bins of 3 units, which cover the magnified image).
"""
import math

import numpy as np
import pytest

import synth
from oracle import solver as osv
from oracle.geometry import FanFlat2D
from oracle.operators import FanFlat2DOps

pytestmark = [pytest.mark.gpu, pytest.mark.usefixtures("oracle_lib")]

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def pk():
    import paper_2602_17892_amd as pk
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return pk


def rel(a, b):
    a = np.asarray(a, dtype=np.float64).ravel()
    b = np.asarray(b, dtype=np.float64).ravel()
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def relp(a, b):
    """Projector error: the larger of the relative L2 error and
    max|a - b| / max|b| (a wrong value on a few bins shows in the second)."""
    a = np.asarray(a, dtype=np.float64).ravel()
    b = np.asarray(b, dtype=np.float64).ravel()
    return float(max(rel(a, b), np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300)))


# nx, ny, views, bins, pitch, sid, sdd
SHAPES = [
    (32, 28, 40, 45, 1.5, 60.0, 120.0),
    (17, 23, 7, 31, 1.2, 30.0, 45.0),       # ragged, wide fan
    (64, 64, 50, 100, 1.0, 100.0, 150.0),
]
TP3 = (1024, 1024, 50, 1024, 3.0, 2048.0, 4096.0)


def make(pk, shape, dt, sino=None, angles=None):
    nx, ny, nv, nu, pu, sid, sdd = shape
    g = pk.Geometry(nx, ny, nv, nu, det_pitch_u=pu, kind="fan2d", sid=sid, sdd=sdd, angles=angles)
    A = pk.Operator("joseph", g, dt, sino or dt)
    B = pk.Operator("pixel", g, dt, sino or dt)
    og = FanFlat2DOps(FanFlat2D(nx, ny, nv, nu, pu, sid, sdd, None if angles is None else np.asarray(angles)))
    return A, B, og


def dev(a, dtype):
    return torch.as_tensor(np.ascontiguousarray(a)).to(device="cuda", dtype=dtype)


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("dt", ["f64", "f32"])
def test_fan_parity(pk, shape, dt):
    nx, ny, nv, nu = shape[:4]
    A, B, og = make(pk, shape, dt)
    r = np.random.default_rng(1)
    tdt = torch.float64 if dt == "f64" else torch.float32
    xd = dev(r.uniform(size=(2, ny, nx)), tdt)
    yd = dev(r.standard_normal((2, nv, nu)), tdt)
    ya, xb = pk.project(A, xd), pk.backproject(B, yd)
    assert tuple(ya.shape) == (2, nv, nu) and tuple(xb.shape) == (2, ny, nx)
    ya, xb = ya.double().cpu().numpy(), xb.double().cpu().numpy()
    xr, yr = xd.double().cpu().numpy(), yd.double().cpu().numpy()
    ea = max(relp(ya[s], og.A(xr[s])) for s in range(2))
    eb = max(relp(xb[s], og.B(yr[s])) for s in range(2))
    tol = 1e-12 if dt == "f64" else 1e-5
    print(f"fan {shape} {dt}: A {ea:.2e} B {eb:.2e}")
    assert ea <= tol and eb <= tol


def test_fan_user_angles_and_bf16(pk):
    shape = SHAPES[0]
    nx, ny, nv, nu = shape[:4]
    angles = np.sort(np.random.default_rng(2).uniform(0, 2 * math.pi, nv))
    angles[3] = math.pi / 4
    A, B, og = make(pk, shape, "f64", angles=angles.tolist())
    x = np.random.default_rng(3).uniform(size=(ny, nx))
    y = np.random.default_rng(4).standard_normal((nv, nu))
    ea = relp(pk.project(A, dev(x, torch.float64)).cpu().numpy(), og.A(x))
    eb = relp(pk.backproject(B, dev(y, torch.float64)).cpu().numpy(), og.B(y))
    A16, B16, og16 = make(pk, shape, "f32", "bf16")
    ya = pk.project(A16, dev(x, torch.float32))
    ref = og16.A(x.astype(np.float32).astype(np.float64))
    step = np.abs(ya.double().cpu().numpy().ravel() - ref) / np.maximum(np.abs(ref), 1e-30)
    print(f"fan user angles: A {ea:.2e} B {eb:.2e}; bf16 A max per entry {step[np.abs(ref) > 1e-3].max():.2e}")
    assert max(ea, eb) <= 1e-12 and step[np.abs(ref) > 1e-3].max() <= 2.0 ** -8


@pytest.mark.parametrize("mode", ["AB", "BA"])
def test_fan_solve_parity(pk, mode):
    shape = SHAPES[2]
    nx, ny, nv, nu = shape[:4]
    A, B, og = make(pk, shape, "f64")
    x, _ = synth.phantom2d(8, 0, nx)
    bt = og.A(x)
    b, _ = synth.add_relative_noise(bt, synth.noise_direction(8, 0, bt.size), 0.01)
    xg, info = pk.solve(A, B, dev(b.reshape(1, nv, nu), torch.float64), mode=mode, k=12, reg="gcv")
    o = osv.hybrid_gmres(og.A, og.B, b, mode=mode, K=12, rule="gcv")
    ex = rel(xg.cpu().numpy(), o.x)
    print(f"fan solve {mode} K=12: x {ex:.2e}")
    assert ex <= 1e-8


def test_fan_tp3_shape(pk):
    nx, ny, nv, nu = TP3[:4]
    A, B, og = make(pk, TP3, "f32")
    x, _ = synth.phantom2d(9, 0, nx)
    xd = dev(x.reshape(1, ny, nx), torch.float32)
    ya = pk.project(A, xd)
    ref = og.A(xd.double().cpu().numpy())
    ea = relp(ya.double().cpu().numpy(), ref)
    y = dev(ref.reshape(1, nv, nu), torch.float32)
    eb = relp(pk.backproject(B, y).double().cpu().numpy(), og.B(y.double().cpu().numpy()))
    # a solve with DP stop at 1.5 % noise against the oracle's stop iteration
    b, en = synth.add_relative_noise(ref, synth.noise_direction(9, 0, ref.size), 0.015)
    bd = dev(b.reshape(1, nv, nu), torch.float32)
    xs, info = pk.solve(A, B, bd, mode="AB", k=60, reg="gcv", stop="dp",
                        noise_norm=torch.tensor([en], dtype=torch.float64, device="cuda"))
    o = osv.hybrid_gmres(og.A, og.B, bd.double().cpu().numpy().ravel(), mode="AB", K=60, rule="gcv", stop="dp",
                         noise_norm=en)
    ex = rel(xs.double().cpu().numpy(), o.x)
    rre = rel(xs.double().cpu().numpy(), x)
    print(f"fan 1024^2 x 50 views: A {ea:.2e} B {eb:.2e}; AB GCV+DP iters {int(info['iters'][0])} / oracle "
          f"{o.iters}, x {ex:.2e}, RRE {rre:.4f}")
    assert ea <= 1e-5 and eb <= 1e-5
    assert int(info["iters"][0]) == o.iters and ex <= 1e-4
