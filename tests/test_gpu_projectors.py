"""GPU parity of the 2D projectors against the FP64 oracle (through the C ABI).

Gates, on both the relative L2 error and the element-wise error
max|gpu - oracle| / max|oracle|: <= 1e-12 for the FP64 instantiation,
<= 1e-5 for FP32; BF16 sinogram storage within 2^-8 (one BF16 rounding) of
the oracle rounded the same way.  Every case prints the larger of the two.
"""
import math

import numpy as np
import pytest

import synth
from oracle.geometry import Par2D
from oracle.operators import Par2DOps

pytestmark = [pytest.mark.gpu, pytest.mark.usefixtures("oracle_lib")]

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def pk():
    import paper_2602_17892_amd as pk
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return pk


def rel(a, b):
    """The larger of the relative L2 error and max|a - b| / max|b|: a wrong
    value on a few bins hides in the first but not in the second."""
    a = np.asarray(a, dtype=np.float64).ravel()
    b = np.asarray(b, dtype=np.float64).ravel()
    l2 = np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)
    mx = np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300) if b.size else 0.0
    return float(max(l2, mx))


SHAPES = [
    (8, 8, 12, 13),        # tiny
    (64, 64, 90, 91),      # 64^2, 90 angles
    (37, 50, 33, 71),      # ragged, nx != ny, odd everything
    (3, 1, 5, 4),          # degenerate strip
]

TOL = {"f64": 1e-12, "f32": 1e-5}


def make_ops(pk, shape, img, sino, angles=None):
    nx, ny, na, nd = shape
    g = pk.Geometry(nx, ny, na, nd, angles=angles)
    A = pk.Operator("joseph", g, img, sino)
    B = pk.Operator("pixel", g, img, sino)
    At = pk.Operator("joseph_t", g, img, sino)
    og = Par2DOps(Par2D(nx, ny, na, nd, angles=None if angles is None else np.asarray(angles)))
    return A, B, At, og


def dev(a, dtype):
    return torch.as_tensor(np.ascontiguousarray(a)).to(device="cuda", dtype=dtype)


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("dt", ["f64", "f32"])
def test_projector_parity(pk, shape, dt):
    nx, ny, na, nd = shape
    A, B, At, og = make_ops(pk, shape, dt, dt)
    tdt = torch.float64 if dt == "f64" else torch.float32
    r = np.random.default_rng(11)
    x = r.uniform(size=(3, ny, nx))
    y = r.standard_normal((3, na, nd))
    # inputs rounded to the storage type first, then promoted for the oracle
    xd, yd = dev(x, tdt), dev(y, tdt)
    xr, yr = xd.double().cpu().numpy(), yd.double().cpu().numpy()
    ya = pk.project(A, xd).double().cpu().numpy()
    xb = pk.backproject(B, yd).double().cpu().numpy()
    xt = pk.backproject(At, yd).double().cpu().numpy()
    ea, eb, et = rel(ya, og.A(xr)), rel(xb, og.B(yr)), rel(xt, og.At(yr))
    print(f"shape={shape} {dt}: A {ea:.2e}  B {eb:.2e}  At {et:.2e}")
    assert ea <= TOL[dt] and eb <= TOL[dt] and et <= TOL[dt]


def test_projector_parity_c2_shape(pk):
    n, na, nd = 512, 720, 725
    A, B, At, og = make_ops(pk, (n, n, na, nd), "f32", "f32")
    x, _ = synth.phantom2d(1, 0, n)
    xd = dev(x, torch.float32)
    xr = xd.double().cpu().numpy()
    y_ref = og.A(xr)
    ya = pk.project(A, xd)
    ea = rel(ya.double().cpu().numpy(), y_ref)
    yd = dev(y_ref, torch.float32)
    yr = yd.double().cpu().numpy()
    eb = rel(pk.backproject(B, yd).double().cpu().numpy(), og.B(yr))
    et = rel(pk.backproject(At, yd).double().cpu().numpy(), og.At(yr))
    print(f"C2 512^2 x 720 x 725 f32: A {ea:.2e}  B {eb:.2e}  At {et:.2e}")
    assert ea <= 1e-5 and eb <= 1e-5 and et <= 1e-5


def test_user_angles_parity(pk):
    angles = np.sort(np.random.default_rng(5).uniform(0, math.pi, 17))
    angles[3] = math.pi / 4
    angles[9] = 3 * math.pi / 4
    A, B, At, og = make_ops(pk, (24, 24, 17, 35), "f64", "f64", angles=angles.tolist())
    x = np.random.default_rng(6).uniform(size=(24, 24))
    y = np.random.default_rng(7).standard_normal((17, 35))
    xd, yd = dev(x, torch.float64), dev(y, torch.float64)
    ea = rel(pk.project(A, xd).cpu().numpy(), og.A(x))
    eb = rel(pk.backproject(B, yd).cpu().numpy(), og.B(y))
    et = rel(pk.backproject(At, yd).cpu().numpy(), og.At(y))
    print(f"user angles f64: A {ea:.2e} B {eb:.2e} At {et:.2e}")
    assert max(ea, eb, et) <= 1e-12


def test_detector_pitch_parity(pk):
    g = pk.Geometry(30, 30, 40, 61, det_pitch_u=0.7)
    A, B, At = (pk.Operator(k, g, "f64", "f64") for k in ("joseph", "pixel", "joseph_t"))
    og = Par2DOps(Par2D(30, 30, 40, 61, det_pitch=0.7))
    x = np.random.default_rng(8).uniform(size=(30, 30))
    y = np.random.default_rng(9).standard_normal((40, 61))
    xd, yd = dev(x, torch.float64), dev(y, torch.float64)
    errs = (rel(pk.project(A, xd).cpu().numpy(), og.A(x)), rel(pk.backproject(B, yd).cpu().numpy(), og.B(y)),
            rel(pk.backproject(At, yd).cpu().numpy(), og.At(y)))
    print("pitch 0.7 f64:", errs)
    assert max(errs) <= 1e-12


def test_bf16_sinogram_storage(pk):
    n, na, nd = 64, 90, 91
    A, B, _, og = make_ops(pk, (n, n, na, nd), "f32", "bf16")
    x, _ = synth.phantom2d(0, 3, n)
    xd = dev(x, torch.float32)
    xr = xd.double().cpu().numpy()
    ref = og.A(xr)
    ya = pk.project(A, xd).double().cpu().numpy()
    ref_bf16 = torch.as_tensor(ref).to(torch.float32).to(torch.bfloat16).double().numpy()
    e64, e16 = rel(ya, ref), rel(ya, ref_bf16)
    yd = dev(ref, torch.bfloat16)
    yr = yd.double().cpu().numpy()
    eb = rel(pk.backproject(B, yd).double().cpu().numpy(), og.B(yr))
    print(f"bf16 sinogram: A vs fp64 oracle {e64:.2e}, vs bf16-rounded oracle {e16:.2e}; B {eb:.2e}")
    assert e64 <= 2 ** -8 and e16 <= 2e-3 and eb <= 1e-5


@pytest.mark.parametrize("shape,dt", [(s, d) for d in ("f64", "f32") for s in SHAPES + [(24, 24, 17, 35)]]
                         + [((512, 512, 720, 725), "f32")])
def test_joseph_gather_and_lds_paths_are_bitwise_equal(pk, shape, dt, monkeypatch):
    """A has two kernels (per-ray gathers from global memory; bands of rows
    staged in LDS, chosen for large batches).  They perform the same
    operations in the same order, so their outputs must be identical bits;
    the parity tests above cover the gather path against the oracle."""
    nx, ny, na, nd = shape
    angles = None
    if shape == (24, 24, 17, 35):
        angles = np.sort(np.random.default_rng(5).uniform(0, math.pi, 17)).tolist()
    g = pk.Geometry(nx, ny, na, nd, angles=angles)
    A = pk.Operator("joseph", g, dt, dt)
    tdt = {"f64": torch.float64, "f32": torch.float32}[dt]
    x = torch.as_tensor(np.random.default_rng(21).uniform(size=(3, ny, nx))).to(device="cuda", dtype=tdt)
    monkeypatch.setenv("ABBA_JOSEPH_PATH", "gather")
    yg = pk.project(A, x)
    monkeypatch.setenv("ABBA_JOSEPH_PATH", "lds")
    yl = pk.project(A, x)
    torch.cuda.synchronize()
    diff = (yg - yl).abs().max().item()
    print(f"{shape} {dt}: max |gather - lds| = {diff:.3e}")
    assert torch.equal(yg, yl)


@pytest.mark.parametrize("shape,dt,batch", [((128, 128, 180, 183), "f32", 128), ((37, 50, 33, 71), "f64", 512),
                                             ((512, 512, 720, 725), "f32", 8)])
def test_backprojector_whole_and_half_tiles_are_bitwise_equal(pk, shape, dt, batch):
    """B takes 32 x 64 pixel tiles, a whole tile per workgroup in batches
    that fill the device and half a tile per workgroup below that (one slice
    of 512^2 is 128 tiles for 256 CUs).  Both stage the tile's window and
    compute positions relative to its start, so a slice backprojected in a
    batch (whole tiles) and alone (halves) must give the same bits."""
    nx, ny, na, nd = shape
    g = pk.Geometry(nx, ny, na, nd)
    B = pk.Operator("pixel", g, dt, dt)
    tdt = {"f64": torch.float64, "f32": torch.float32}[dt]
    assert (-(-nx // 32)) * (-(-ny // 64)) * batch >= 1024 > (-(-nx // 32)) * (-(-ny // 64))
    y = torch.as_tensor(np.random.default_rng(8).standard_normal((batch, na, nd))).to(device="cuda", dtype=tdt)
    xb = pk.backproject(B, y)
    for s in (0, batch // 3, batch - 1):
        x1 = pk.backproject(B, y[s:s + 1].contiguous())
        torch.cuda.synchronize()
        print(f"{shape} {dt} slice {s}: max |batch - alone| = {(xb[s] - x1[0]).abs().max().item():.3e}")
        assert torch.equal(xb[s], x1[0])


def test_adjoint_identity_gpu(pk):
    g = pk.Geometry(64, 64, 90, 91)
    A, At = pk.Operator("joseph", g), pk.Operator("joseph_t", g)
    r = np.random.default_rng(3)
    x = dev(r.standard_normal((64, 64)), torch.float32)
    y = dev(r.standard_normal((90, 91)), torch.float32)
    lhs = float((pk.project(A, x).double() * y.double()).sum())
    rhs = float((x.double() * pk.backproject(At, y).double()).sum())
    scale = float(x.double().norm() * y.double().norm())
    print(f"<Ax,y>={lhs:.9e} <x,A^T y>={rhs:.9e}")
    assert abs(lhs - rhs) <= 1e-6 * scale


def test_run_twice_bitwise(pk):
    g = pk.Geometry(128, 128, 180, 183)
    A, B = pk.Operator("joseph", g), pk.Operator("pixel", g)
    x = dev(synth.phantom2d(2, 0, 128)[0], torch.float32)
    y1, y2 = pk.project(A, x), pk.project(A, x)
    b1, b2 = pk.backproject(B, y1), pk.backproject(B, y1)
    assert torch.equal(y1, y2) and torch.equal(b1, b2)


def test_empty_batch_is_noop(pk):
    g = pk.Geometry(8, 8, 12, 13)
    A = pk.Operator("joseph", g)
    x = torch.zeros((0, 8, 8), device="cuda")
    y = pk.project(A, x)
    assert y.shape == (0, 12, 13)


def test_shape_and_dtype_errors(pk):
    g = pk.Geometry(8, 8, 12, 13)
    A = pk.Operator("joseph", g)
    with pytest.raises(TypeError):
        pk.project(A, torch.zeros((8, 8), device="cuda", dtype=torch.float64))
    with pytest.raises(ValueError):
        pk.project(A, torch.zeros((7, 8), device="cuda"))
    B = pk.Operator("pixel", pk.Geometry(8, 8, 12, 15))
    with pytest.raises(pk.AbbaError) as ei:
        pk.solve(A, B, torch.zeros((12, 13), device="cuda"), k=3)
    assert ei.value.status in (-1, -2)
