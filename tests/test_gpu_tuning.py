"""Launch tuning: every launch choice of a projector computes the same bits
(it changes how work is split over workgroups, never the order of a sum), and
abba_autotune keeps one of them for the batch size it timed."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def pk():
    import paper_2602_17892_amd as pk
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return pk


def ops2d(pk, shape, dt="f32"):
    nx, ny, na, nd = shape
    g = pk.Geometry(nx, ny, na, nd)
    return pk.Operator("joseph", g, dt, dt), pk.Operator("pixel", g, dt, dt)


def images(S, ny, nx, seed, dtype=torch.float32):
    r = np.random.default_rng(seed)
    return torch.as_tensor(r.uniform(size=(S, ny, nx))).to(device="cuda", dtype=dtype)


@pytest.mark.parametrize("shape", [(100, 90, 73, 131), (64, 64, 90, 91), (256, 256, 180, 363)])
@pytest.mark.parametrize("dt", ["f32", "f64"])
def test_2d_launch_choices_bitwise_equal(pk, shape, dt):
    nx, ny, na, nd = shape
    A, B = ops2d(pk, shape, dt)
    S = 3
    tdt = torch.float64 if dt == "f64" else torch.float32
    x = images(S, ny, nx, 1, tdt)
    y = images(S, na, nd, 2, tdt)
    ya0, xb0 = pk.project(A, x), pk.backproject(B, y)
    for path, jb in [(0, 0), (1, 2), (1, 3), (1, 4)]:
        pk.set_tuning(A, S, a_path=path, a_jb=jb)
        assert pk.get_tuning(A, S) == dict(a_path=path, a_jb=jb, b_g=0, czt=0, a_rb=0, a_occ=0, a_tile=0, a_vg=0)
        assert torch.equal(pk.project(A, x), ya0), (path, jb)
    for g in (1, 8, 16, 64, 128):
        pk.set_tuning(B, S, b_g=g)
        assert torch.equal(pk.backproject(B, y), xb0), g
    pk.set_tuning(A, S, clear=True)
    pk.set_tuning(B, S, clear=True)
    assert pk.get_tuning(A, S) is None and pk.get_tuning(B, S) is None


def test_cone_launch_choices_bitwise_equal(pk):
    nx, ny, nz, nvw, nu, nv = 20, 18, 13, 16, 28, 24
    g = pk.Geometry(nx, ny, nvw, nu, det_pitch_u=1.3, kind="cone3d", nz=nz, det_v=nv, det_pitch_v=1.2,
                    sid=40.0, sdd=80.0)
    A = pk.Operator("joseph", g, "f32", "f32")
    B = pk.Operator("pixel", g, "f32", "f32")
    y = images(2, nvw * nv, nu, 3).reshape(2, nvw, nv, nu).contiguous()
    x0 = pk.backproject(B, y)
    for c in (2, 4, 8):
        pk.set_tuning(B, 2, czt=c)
        assert torch.equal(pk.backproject(B, y), x0), c
    x = images(2, nz * ny, nx, 5).reshape(2, nz, ny, nx).contiguous()
    y0 = pk.project(A, x)
    for rb in (1, 3, 5, 8, 64):          # ragged last bands included (24 rows)
        pk.set_tuning(A, 2, a_rb=rb)
        assert torch.equal(pk.project(A, x), y0), rb
    for occ in (5, 4, 3):                # workgroups per CU capped by reserved LDS
        pk.set_tuning(A, 2, a_occ=occ)
        assert pk.get_tuning(A, 2)["a_occ"] == occ
        assert torch.equal(pk.project(A, x), y0), occ
    for tile, occ in ((16, 0), (16, 4), (8, 0), (8, 5), (-1, 0)):   # tiles (ragged: 28 x 24 pixels), rows
        pk.set_tuning(A, 2, a_occ=occ, a_tile=tile)
        assert pk.get_tuning(A, 2)["a_tile"] == tile
        assert torch.equal(pk.project(A, x), y0), ("tile", tile, occ)
    for vg in (1, 3, 5, 16, 100):        # groups of views per tile (ragged last group: 16 views)
        pk.set_tuning(A, 2, a_tile=16, a_vg=vg)
        assert pk.get_tuning(A, 2)["a_vg"] == vg
        assert torch.equal(pk.project(A, x), y0), ("views per group", vg)
    with pytest.raises(pk.AbbaError):
        pk.set_tuning(A, 2, a_tile=4)
    with pytest.raises(pk.AbbaError):
        pk.set_tuning(A, 2, a_vg=-1)


def test_autotune_keeps_a_choice(pk):
    A, B = ops2d(pk, (128, 128, 180, 183))
    S = 16
    x = images(S, 128, 128, 4)
    ya0 = pk.project(A, x)
    ta = pk.autotune(A, S, reps=2)
    tb = pk.autotune(B, S, reps=2)
    print(f"A: {ta}\nB: {tb}")
    assert ta["candidates"] == 4 and tb["candidates"] >= 3
    assert ta["ms"] <= ta["default_ms"] and tb["ms"] <= tb["default_ms"]
    assert pk.get_tuning(A, S) == {k: ta[k] for k in ("a_path", "a_jb", "b_g", "czt", "a_rb", "a_occ", "a_tile",
                                                      "a_vg")}
    assert torch.equal(pk.project(A, x), ya0)
    # the solver uses the stored choice and returns the same bits
    og_b = pk.project(A, x).contiguous()
    x1, _ = pk.solve(A, B, og_b, mode="AB", k=4, reg="gcv")
    pk.set_tuning(A, S, clear=True)
    pk.set_tuning(B, S, clear=True)
    x2, _ = pk.solve(A, B, og_b, mode="AB", k=4, reg="gcv")
    assert torch.equal(x1, x2)


def test_tuning_argument_errors(pk):
    A, _ = ops2d(pk, (16, 16, 20, 23))
    with pytest.raises(pk.AbbaError):
        pk.set_tuning(A, 0, a_path=1)
    with pytest.raises(pk.AbbaError):
        pk.set_tuning(A, 1, a_occ=-1)
    with pytest.raises(pk.AbbaError):
        pk.set_tuning(A, 1, a_occ=1)          # would reserve more than 64 KB of LDS
    with pytest.raises(pk.AbbaError):
        pk.autotune(A, 0)
