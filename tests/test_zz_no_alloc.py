"""abba_project_noalloc (the allocation-free variant of abba_project) through
the C ABI: two calls in a row, the second with a smaller input, each bitwise
equal to abba_project with a caller workspace (the same kernels run); an
input whose scratch exceeds the static buffer is refused."""
import ctypes

import numpy as np
import pytest

pytestmark = [pytest.mark.gpu]

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def pk():
    import paper_2602_17892_amd as pk
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return pk


def call_noalloc(pk, A, x, y):
    rc = pk.lib.abba_project_noalloc(A.handle, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(y.data_ptr()),
                                     x.shape[0], ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    torch.cuda.synchronize()
    return rc


@pytest.mark.parametrize("dt", ["f32", "f64"])
def test_noalloc_matches_project_twice(pk, dt):
    tdt = torch.float32 if dt == "f32" else torch.float64
    rng = np.random.default_rng(9)
    cases = [(pk.Geometry(512, 512, 720, 725), 5), (pk.Geometry(37, 50, 33, 71), 2)]
    for g, batch in cases:      # the second call has the smaller input
        A = pk.Operator("joseph", g, dt, dt)
        x = torch.as_tensor(rng.uniform(size=(batch, g.ny, g.nx)), dtype=tdt, device="cuda")
        ws = torch.empty(pk.project_workspace_bytes(A, batch), dtype=torch.uint8, device="cuda")
        ref = pk.project(A, x, workspace=ws)
        y = torch.full_like(ref, float("nan"))
        assert call_noalloc(pk, A, x, y) == 0, pk.lib.abba_last_error()
        print(f"{dt} {g.ny}x{g.nx}, {g.n_angles}x{g.det_u}, batch {batch}: scratch "
              f"{pk.project_workspace_bytes(A, batch)} bytes, equal to abba_project: {torch.equal(y, ref)}")
        assert torch.equal(y, ref)


def test_noalloc_fan_and_cone(pk):
    rng = np.random.default_rng(10)
    for g in (pk.Geometry(64, 64, 30, 96, det_pitch_u=1.5, kind="fan2d", sid=128.0, sdd=256.0),
              pk.Geometry(24, 20, 16, 40, det_pitch_u=1.5, kind="cone3d", nz=18, det_v=30, det_pitch_v=1.5,
                          sid=60.0, sdd=120.0)):
        A = pk.Operator("joseph", g, "f32", "f32")
        x = torch.as_tensor(rng.uniform(size=(2, *g.image_shape)), dtype=torch.float32, device="cuda")
        ref = pk.project(A, x)
        y = torch.full_like(ref, float("nan"))
        assert call_noalloc(pk, A, x, y) == 0
        assert torch.equal(y, ref)


def test_noalloc_refuses_what_does_not_fit(pk):
    g = pk.Geometry(512, 512, 720, 725)
    A = pk.Operator("joseph", g, "f32", "f32")
    per = pk.project_workspace_bytes(A, 1)
    batch = pk.NOALLOC_SCRATCH_BYTES // per + 1
    x = torch.zeros((batch, 512, 512), device="cuda")
    y = torch.full((batch, 720, 725), float("nan"), device="cuda")
    assert call_noalloc(pk, A, x, y) == -1
    assert b"static buffer" in pk.lib.abba_last_error()
    assert bool(torch.isnan(y).all())
    # the largest batch that fits still runs
    fit = pk.NOALLOC_SCRATCH_BYTES // per
    assert call_noalloc(pk, A, x[:fit], y[:fit]) == 0
    assert bool(torch.isfinite(y[:fit]).all())
