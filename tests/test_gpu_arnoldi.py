"""The GPU's own Arnoldi quantities (Sec. 2.1, eq. (8)) and its breakdown branch.

* The basis W and the Hessenberg matrix H that abba_solve leaves in its
  workspace (located with abba_solve_layout) satisfy the Arnoldi relation
  M W_k = W_{k+1} H_k and W_{k+1}^T W_{k+1} = I: to 1e-12 on the FP64 path
  (64^2, 90 angles x 91 bins, K = 30), for both modes and both Gram-Schmidt
  schedules.  M is applied with the GPU's own projectors.  The FP32 path at
  512^2, 720 x 725 reports its values (gated at 1e-4 only as a sanity bound:
  the basis is stored in FP32).
* In-iteration breakdown (h_{k+1,k} <= 1e-14 ||M w_k|| at k >= 1): on an
  n x n image seen at the two axis angles 0 and pi/2 by n unit bins, A
  takes column and row sums and B = A^T, so M has the eigenvalues n and 2n
  on the range of A^T A (BA) and of A A^T (AB, data in the range of A); the
  Krylov space closes at k = 2, with h_{3,2} at rounding level against
  h_{2,1} ~ 0.05 ||M w||.  With one angle M = n I on its range and the
  space closes at k = 1.  The run must end with ABBA_ST_BREAKDOWN at the
  oracle's iteration and the oracle's x within 1e-8 (FP64), for both
  schedules and modes.
"""
import numpy as np
import pytest

import synth
from oracle import solver as osv
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
    a = np.asarray(a, dtype=np.float64).ravel()
    b = np.asarray(b, dtype=np.float64).ravel()
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def apply_M(pk, A, B, mode, V):
    """M applied to the rows of V (float tensor [k, len]) with the GPU
    projectors: AB: A(B v), BA: B(A v)."""
    g = A.geom
    if mode == "AB":
        y = V.reshape(V.shape[0], g.n_angles, g.det_u).to(B.sino_dtype).contiguous()
        return pk.project(A, pk.backproject(B, y)).reshape(V.shape[0], -1)
    x = V.reshape(V.shape[0], g.ny, g.nx).to(A.img_dtype).contiguous()
    return pk.backproject(B, pk.project(A, x)).reshape(V.shape[0], -1)


def arnoldi_residuals(pk, A, B, mode, ws, lay, s, k, broke=False):
    """(||M W_k - W_{k+1} H_k||_F / ||M W_k||_F, max|W^T W - I|) of slice s
    after k iterations, from the workspace."""
    W, H = pk.basis_views(ws, lay, s + 1)
    nvec = k if broke else k + 1
    Wk1 = W[s, :nvec, :lay["len"]].double()                 # w_1 .. w_{k+1}
    # (k+1) x k, or k x k after a breakdown; entries below the subdiagonal
    # are not defined in the workspace
    Hk = torch.triu(H[s, :k, :nvec].double().T, diagonal=-1)
    MW = apply_M(pk, A, B, mode, W[s, :k, :lay["len"]].contiguous()).double()
    r = torch.linalg.norm(MW.T - Wk1.T @ Hk) / torch.linalg.norm(MW)
    G = Wk1 @ Wk1.T
    o = torch.max(torch.abs(G - torch.eye(nvec, dtype=torch.float64, device=G.device)))
    return float(r), float(o)


def problem(pk, n, na, nd, eta, cfg, idx, dt):
    g = pk.Geometry(n, n, na, nd)
    A = pk.Operator("joseph", g, dt, dt)
    B = pk.Operator("pixel", g, dt, dt)
    og = Par2DOps(Par2D(n, n, na, nd))
    x, _ = synth.phantom2d(cfg, idx, n)
    bt = og.A(x).reshape(-1)
    b, en = synth.add_relative_noise(bt, synth.noise_direction(cfg, idx, og.m), eta)
    tdt = torch.float64 if dt == "f64" else torch.float32
    bd = torch.as_tensor(b).to(device="cuda", dtype=tdt).reshape(1, na, nd)
    return A, B, og, x, bd


@pytest.mark.parametrize("ortho", ["dcgs2", "cgs2"])
@pytest.mark.parametrize("mode", ["AB", "BA"])
def test_arnoldi_relation_f64(pk, mode, ortho):
    A, B, og, xt, bd = problem(pk, 64, 90, 91, 0.01, 0, 1, "f64")
    K = 30
    lay = pk.solve_layout(A, B, 1, mode, K)
    ws = torch.zeros(lay["bytes"], dtype=torch.uint8, device="cuda")
    x, info = pk.solve(A, B, bd, mode=mode, k=K, reg="gcv", ortho=ortho, workspace=ws)
    torch.cuda.synchronize()
    assert int(info["iters"][0]) == K and lay["len"] == (og.m if mode == "AB" else og.n)
    r, o = arnoldi_residuals(pk, A, B, mode, ws, lay, 0, K)
    print(f"f64 {mode} {ortho} K={K}: ||MW - WH||/||MW|| {r:.2e}, max|W^T W - I| {o:.2e}")
    assert r <= 1e-12 and o <= 1e-12


@pytest.mark.parametrize("mode", ["AB", "BA"])
def test_arnoldi_relation_f32_c2_shape(pk, mode):
    A, B, og, xt, bd = problem(pk, 512, 720, 725, 0.005, 1, 0, "f32")
    K = 30
    lay = pk.solve_layout(A, B, 1, mode, K)
    ws = torch.zeros(lay["bytes"], dtype=torch.uint8, device="cuda")
    x, info = pk.solve(A, B, bd, mode=mode, k=K, reg="gcv", workspace=ws)
    torch.cuda.synchronize()
    r, o = arnoldi_residuals(pk, A, B, mode, ws, lay, 0, K)
    print(f"f32 512^2 {mode} K={K}: ||MW - WH||/||MW|| {r:.2e}, max|W^T W - I| {o:.2e} (FP32 basis)")
    assert r <= 1e-4 and o <= 1e-4


def breakdown_problem(pk, n, na, mode, seed):
    """n x n FP64 image, `na` default angles (0, or 0 and pi/2), n bins."""
    g = pk.Geometry(n, n, na, n)
    A = pk.Operator("joseph", g, "f64", "f64")
    B = pk.Operator("pixel", g, "f64", "f64")
    og = Par2DOps(Par2D(n, n, na, n))
    rng = np.random.default_rng(seed)
    x = rng.uniform(0.0, 1.0, n * n)
    if mode == "AB":
        # data in the range of A (noise added to the image), so that r_0 has
        # no component in the null space of A A^T
        b = og.A(x + 0.05 * rng.standard_normal(n * n))
    else:
        b = og.A(x) + 0.05 * rng.standard_normal(og.m)
    bd = torch.as_tensor(b, dtype=torch.float64, device="cuda").reshape(1, na, n)
    return A, B, og, b, bd


@pytest.mark.parametrize("na", [1, 2])
@pytest.mark.parametrize("ortho", ["dcgs2", "cgs2"])
@pytest.mark.parametrize("mode", ["AB", "BA"])
def test_breakdown_inside_the_run(pk, mode, ortho, na):
    n, K = 8, 6
    A, B, og, b, bd = breakdown_problem(pk, n, na, mode, 3)
    lay = pk.solve_layout(A, B, 1, mode, K)
    ws = torch.zeros(lay["bytes"], dtype=torch.uint8, device="cuda")
    x, info = pk.solve(A, B, bd, mode=mode, k=K, reg="gcv", ortho=ortho, workspace=ws)
    torch.cuda.synchronize()
    o = osv.hybrid_gmres(og.A, og.B, b, mode=mode, K=K, rule="gcv", ortho=ortho)
    it, st = int(info["iters"][0]), int(info["status"][0])
    ex = rel(x.cpu().numpy(), o.x)
    r, orth = arnoldi_residuals(pk, A, B, mode, ws, lay, 0, it, broke=True)
    print(f"{mode} {ortho} {na} angle(s): iters {it} (oracle {o.iters}), status {st} (oracle {o.status}), "
          f"x {ex:.2e}, ||MW_k - W_k H_k||/||MW_k|| {r:.2e}, max|W^T W - I| {orth:.2e}")
    assert o.status == osv.STATUS_BREAKDOWN and o.iters == na
    assert st == pk.ST_BREAKDOWN and it == o.iters
    assert ex <= 1e-8 and r <= 1e-12 and orth <= 1e-12
    # the histories stop at the breakdown
    lam = info["lam"][0].cpu().numpy()
    assert np.all(np.isfinite(lam[:it])) and np.all(np.isnan(lam[it:]))


def test_breakdown_in_a_batch(pk):
    """Two slices of one batch break down at different iterations: a constant
    image gives data along an eigenvector of A A^T (breakdown at k = 1), a
    random one at k = 2; each equals its own single-slice run bit for bit and
    the oracle to 1e-8 (FP64, AB)."""
    n, K = 8, 6
    A, B, og, b, bd = breakdown_problem(pk, n, 2, "AB", 5)
    b1 = og.A(np.full(n * n, 0.7))
    bb = torch.stack([torch.as_tensor(b1, dtype=torch.float64, device="cuda").reshape(2, n), bd[0]]).contiguous()
    x, info = pk.solve(A, B, bb, mode="AB", k=K, reg="gcv")
    it = info["iters"].tolist()
    st = info["status"].tolist()
    print(f"batch: iters {it} status {st}")
    assert st == [pk.ST_BREAKDOWN, pk.ST_BREAKDOWN] and it == [1, 2]
    for s, bs in enumerate((b1, b)):
        x1, i1 = pk.solve(A, B, bb[s:s + 1].contiguous(), mode="AB", k=K, reg="gcv")
        assert torch.equal(x1[0], x[s]) and int(i1["iters"][0]) == it[s] and int(i1["status"][0]) == st[s]
        o = osv.hybrid_gmres(og.A, og.B, bs, mode="AB", K=K, rule="gcv")
        assert it[s] == o.iters and o.status == osv.STATUS_BREAKDOWN and rel(x[s].cpu().numpy(), o.x) <= 1e-8


def sigma_check(pk, ws, lay, S, iters):
    """max over slices of max|sigma_GPU - sigma(H_GPU)| / sigma_1 against
    LAPACK on the GPU's own Hessenberg matrix."""
    _, H, sv = pk.basis_views(ws, lay, S, sigma=True)
    worst = 0.0
    for s in range(S):
        k = int(iters[s])
        Hk = np.triu(H[s, :k, :k + 1].double().cpu().numpy().T, -1)
        ref = np.linalg.svd(Hk, compute_uv=False)
        got = sv[s, :k].cpu().numpy()
        worst = max(worst, float(np.max(np.abs(got - ref)) / ref[0]))
    return worst


@pytest.mark.parametrize("mode", ["AB", "BA"])
def test_singular_values_of_h(pk, mode):
    """The small solve's singular values (updated every iteration by the
    secular equation) against LAPACK on the final H_k: FP64 64^2 at K = 30
    and 60, and the 512^2 FP32-basis run at K = 100."""
    for n, na, nd, eta, dt, K in ((64, 90, 91, 0.01, "f64", 30), (64, 90, 91, 0.001, "f64", 60),
                                  (512, 720, 725, 0.005, "f32", 100)):
        A, B, og, xt, bd = problem(pk, n, na, nd, eta, 0, 3, dt)
        lay = pk.solve_layout(A, B, 1, mode, K)
        ws = torch.zeros(lay["bytes"], dtype=torch.uint8, device="cuda")
        x, info = pk.solve(A, B, bd, mode=mode, k=K, reg="gcv", workspace=ws)
        torch.cuda.synchronize()
        e = sigma_check(pk, ws, lay, 1, info["iters"].cpu().numpy())
        print(f"{mode} {n}^2 {dt} K={K}: max |sigma - LAPACK sigma(H)| / sigma_1 = {e:.1e}")
        assert e <= 1e-12


def test_singular_values_in_a_batch(pk):
    """A batch whose slices end at different iterations (breakdowns at k = 2
    and k = 1 on the two-angle geometry): each slice's singular values
    against LAPACK on its own H, and x against the oracle."""
    n, K = 8, 6
    A, B, og, b, bd = breakdown_problem(pk, n, 2, "AB", 5)
    b1 = og.A(np.full(n * n, 0.7))
    bb = torch.stack([bd[0], torch.as_tensor(b1, dtype=torch.float64, device="cuda").reshape(2, n)]).contiguous()
    lay = pk.solve_layout(A, B, 2, "AB", K)
    ws = torch.zeros(lay["bytes"], dtype=torch.uint8, device="cuda")
    x, info = pk.solve(A, B, bb, mode="AB", k=K, reg="gcv", workspace=ws)
    torch.cuda.synchronize()
    it = info["iters"].cpu().numpy()
    e = sigma_check(pk, ws, lay, 2, it)
    print(f"iters {it.tolist()}: max |sigma - LAPACK| / sigma_1 = {e:.1e}")
    assert it.tolist() == [2, 1] and e <= 1e-12
    for s, bs in enumerate((b, b1)):
        o = osv.hybrid_gmres(og.A, og.B, bs, mode="AB", K=K, rule="gcv")
        assert int(it[s]) == o.iters and rel(x[s].cpu().numpy(), o.x) <= 1e-8
