"""Pins for the oracle's projectors against closed forms and invariants.

The paper leaves the projector discretisation open (its experiments call the
ASTRA toolbox, Sec. 4); these tests pin the oracle's Joseph A, exact A^T and
pixel-driven B to results fixed by geometry alone: axis-aligned projections
(plain row / column sums), single-pixel impulse responses (triangles of unit
area), analytic line integrals of ellipses, transposition of the explicit
matrices, and interpolation of constants.
"""
import math

import numpy as np
import pytest

import synth
from oracle.geometry import Cone3D, Par2D
from oracle.operators import Cone3DOps, Par2DOps

pytestmark = pytest.mark.usefixtures("oracle_lib")


def hat(t):
    return np.maximum(0.0, 1.0 - np.abs(t))


def lin_interp_rows(v, u):
    """Linear interpolation of the sequence v (zero outside) at points u."""
    out = np.zeros_like(u, dtype=np.float64)
    for idx in range(len(v)):
        out += v[idx] * hat(u - idx)
    return out


@pytest.mark.parametrize("n,nd", [(8, 13), (64, 91), (9, 12)])
def test_joseph_theta0_is_interpolated_column_sums(n, nd):
    # At t = 0 every ray is vertical: it crosses each row at the same x, so
    # the projection is the column-sum profile sampled at s_d.
    g = Par2D(n, n, 4, nd)
    ops = Par2DOps(g)
    x = np.random.default_rng(1).uniform(size=(n, n))
    y = ops.A(x)
    colsum = x.sum(axis=0)
    u = (np.arange(nd) - (nd - 1) / 2.0) + (n - 1) / 2.0
    np.testing.assert_allclose(y[0], lin_interp_rows(colsum, u), rtol=0, atol=1e-12)


@pytest.mark.parametrize("n,nd", [(8, 13), (64, 91)])
def test_joseph_theta_half_pi_is_row_sums(n, nd):
    # At t = pi/2 rays are horizontal (s = Y): row sums, up to cos(pi/2) ~ 6e-17.
    g = Par2D(n, n, 4, nd)
    ops = Par2DOps(g)
    x = np.random.default_rng(2).uniform(size=(n, n))
    y = ops.A(x)
    rowsum = x.sum(axis=1)
    u = (np.arange(nd) - (nd - 1) / 2.0) + (n - 1) / 2.0
    np.testing.assert_allclose(y[2], lin_interp_rows(rowsum, u), rtol=0, atol=1e-12)


@pytest.mark.parametrize("na", [12, 90])
def test_joseph_impulse_response_is_unit_area_triangle(na):
    # A single pixel at p = X cos t + Y sin t is seen by ray s with weight
    # hat((s - p)/c)/|c|, c the dominant direction cosine (a triangle of
    # half-width |c| and unit area in s).
    n, nd = 10, 17
    g = Par2D(n, n, na, nd)
    ops = Par2DOps(g)
    s = np.arange(nd) - (nd - 1) / 2.0
    for (i, j) in [(0, 0), (3, 7), (9, 4), (5, 5)]:
        x = np.zeros((n, n))
        x[i, j] = 1.0
        y = ops.A(x)
        X, Y = j - (n - 1) / 2.0, i - (n - 1) / 2.0
        for a in range(na):
            th = a * math.pi / na
            c = math.cos(th) if (4 * a <= na or 4 * a >= 3 * na) else math.sin(th)
            p = X * math.cos(th) + Y * math.sin(th)
            np.testing.assert_allclose(y[a], hat((s - p) / c) / abs(c), rtol=0, atol=1e-13)


def ellipse_sinogram(params, thetas, s):
    """Analytic line integrals of a sum of uniform ellipses (textbook result)."""
    out = np.zeros((len(thetas), len(s)))
    for cx, cy, a, b, phi, rho in params:
        for ia, th in enumerate(thetas):
            at2 = (a * math.cos(th - phi)) ** 2 + (b * math.sin(th - phi)) ** 2
            sp = s - (cx * math.cos(th) + cy * math.sin(th))
            inside = sp * sp < at2
            out[ia] += np.where(inside, 2.0 * rho * a * b * np.sqrt(np.maximum(at2 - sp * sp, 0.0)) / at2, 0.0)
    return out


def test_joseph_matches_analytic_ellipse_projections_and_converges():
    errs = []
    for n in (64, 128, 256):
        nd = synth.default_ndet(n)
        na = 45
        g = Par2D(n, n, na, nd)
        ops = Par2DOps(g)
        params = synth.ellipse_params(synth.rng_for(99, 0, 0), n)
        x = synth.rasterize_ellipses(params, n, sub=4)
        y = ops.A(x)
        th = np.arange(na) * math.pi / na
        s = np.arange(nd) - (nd - 1) / 2.0
        ref = ellipse_sinogram(params, th, s)
        errs.append(np.linalg.norm(y - ref) / np.linalg.norm(ref))
    assert errs[0] < 2e-2, errs
    # discretisation error shrinks with the resolution
    assert errs[1] < 0.75 * errs[0] and errs[2] < 0.75 * errs[1], errs


def test_joseph_mass_at_axis_angles():
    n, nd = 32, 47
    g = Par2D(n, n, 8, nd)
    ops = Par2DOps(g)
    x = synth.phantom2d(5, 0, n)[0]
    y = ops.A(x)
    assert abs(y[0].sum() - x.sum()) < 1e-11 * x.sum()
    assert abs(y[4].sum() - x.sum()) < 1e-11 * x.sum()
    # within ~1e-2 at the other angles
    assert np.all(np.abs(y.sum(axis=1) - x.sum()) < 2e-2 * x.sum())


def test_exact_transpose_matches_explicit_matrix():
    g = Par2D(8, 8, 12, 13)
    ops = Par2DOps(g)
    Am = ops.explicit("A")
    Atm = ops.explicit("At")
    assert Am.shape == (g.m, g.n) and Atm.shape == (g.n, g.m)
    np.testing.assert_allclose(Atm, Am.T, rtol=0, atol=1e-14)


@pytest.mark.parametrize("shape", [(8, 8, 12, 13), (64, 64, 90, 91), (12, 7, 10, 19)])
def test_adjoint_identity(shape):
    nx, ny, na, nd = shape
    g = Par2D(nx, ny, na, nd)
    ops = Par2DOps(g)
    r = np.random.default_rng(3)
    x = r.standard_normal((ny, nx))
    y = r.standard_normal((na, nd))
    lhs = float(np.sum(ops.A(x) * y))
    rhs = float(np.sum(x * ops.At(y)))
    assert abs(lhs - rhs) <= 1e-13 * (abs(lhs) + np.linalg.norm(x) * np.linalg.norm(y))


def test_backprojector_interpolates_constants():
    # B applied to an all-ones sinogram returns n_angles / ds at every pixel
    # whose projection stays inside the detector in every view.
    n, nd, na = 16, 31, 20
    for ds in (1.0, 0.75):
        g = Par2D(n, n, na, nd, det_pitch=ds)
        ops = Par2DOps(g)
        xb = ops.B(np.ones((na, nd)))
        X = np.arange(n) - (n - 1) / 2.0
        XX, YY = np.meshgrid(X, X)
        rmax = np.sqrt(XX ** 2 + YY ** 2)
        inside = rmax / ds + 1 < (nd - 1) / 2.0
        assert inside.sum() > 10
        np.testing.assert_allclose(xb[inside], na / ds, rtol=0, atol=1e-12)


def test_backprojector_impulse_response():
    # B of a single sinogram entry (a, d) is hat(t_a(i,j) - d) / ds over the image.
    n, nd, na, ds = 9, 15, 7, 1.25
    g = Par2D(n, n, na, nd, det_pitch=ds)
    ops = Par2DOps(g)
    X = np.arange(n) - (n - 1) / 2.0
    XX, YY = np.meshgrid(X, X)
    for (a, d) in [(0, 7), (3, 2), (6, 11)]:
        y = np.zeros((na, nd))
        y[a, d] = 1.0
        th = a * math.pi / na
        t = (XX * math.cos(th) + YY * math.sin(th)) / ds + (nd - 1) / 2.0
        np.testing.assert_allclose(ops.B(y), hat(t - d) / ds, rtol=0, atol=1e-14)


def test_backprojector_is_unmatched_but_close():
    g = Par2D(8, 8, 12, 13)
    ops = Par2DOps(g)
    Bm = ops.explicit("B")
    Atm = ops.explicit("At")
    rel = np.linalg.norm(Bm - Atm) / np.linalg.norm(Atm)
    assert 1e-3 < rel < 0.6, rel
    # same scale: constant sinogram backprojects to about the same level
    c1 = Bm.sum(axis=1)
    c2 = Atm.sum(axis=1)
    centre = slice(2, 6)
    ratio = c1.reshape(8, 8)[centre, centre] / c2.reshape(8, 8)[centre, centre]
    assert np.all(np.abs(ratio - 1.0) < 0.1)


# ------------------------------------------------------------- cone beam ---

def small_cone(n=12, nu=21, nv=19, views=8, pitch=2.0, sid=40.0, sdd=80.0):
    return Cone3D(n, n, n, views, nu, nv, pitch, pitch, sid, sdd)


def sphere_chords(geom, centre, radius, rho):
    """Analytic chord integral rho * |chord| of a sphere along every ray."""
    out = np.zeros((geom.n_views, geom.nv, geom.nu))
    for w in range(geom.n_views):
        S = geom.src[w]
        for r in range(geom.nv):
            for c in range(geom.nu):
                P = geom.det[w] + (c - (geom.nu - 1) / 2.0) * geom.pu * geom.eu[w] \
                    + (r - (geom.nv - 1) / 2.0) * geom.pv * geom.ev[w]
                d = (P - S) / np.linalg.norm(P - S)
                oc = S - centre
                bq = float(d @ oc)
                disc = bq * bq - (float(oc @ oc) - radius * radius)
                out[w, r, c] = rho * 2.0 * math.sqrt(disc) if disc > 0 else 0.0
    return out


def test_cone_forward_matches_sphere_chords_and_converges():
    errs = []
    for n in (16, 32):
        scale = n / 16.0
        g = small_cone(n=n, nu=int(28 * scale) + 1, nv=int(28 * scale) + 1, views=6,
                       pitch=2.0, sid=4.0 * n, sdd=8.0 * n)
        ops = Cone3DOps(g)
        centre = np.array([1.3, -0.7, 0.4]) * scale
        radius = 5.0 * scale
        X = np.arange(n) - (n - 1) / 2.0
        sub = 4
        offs = (np.arange(sub) + 0.5) / sub - 0.5
        vol = np.zeros((n, n, n))
        for oz in offs:
            for oy in offs:
                for ox in offs:
                    Z, Y, XX = np.meshgrid(X + oz, X + oy, X + ox, indexing="ij")
                    vol += ((XX - centre[0]) ** 2 + (Y - centre[1]) ** 2 + (Z - centre[2]) ** 2
                            <= radius ** 2)
        vol /= sub ** 3
        y = ops.A(vol).reshape(g.n_views, g.nv, g.nu)
        ref = sphere_chords(g, centre, radius, 1.0)
        errs.append(np.linalg.norm(y - ref) / np.linalg.norm(ref))
    # a sphere of radius 5 voxels at n = 16: edge voxels dominate the error,
    # which then halves with the resolution (first-order convergence)
    assert errs[0] < 0.12 and errs[1] < 0.06, errs
    assert errs[1] < 0.6 * errs[0], errs


def test_cone_central_ray_through_constant_cube():
    # odd detector: the central pixel's ray in view 0 runs along -x through
    # the centre of the cube: its integral is n for a constant-1 volume.
    n = 10
    g = small_cone(n=n, nu=21, nv=19, views=4)
    ops = Cone3DOps(g)
    y = ops.A(np.ones(g.n)).reshape(4, g.nv, g.nu)
    for w in range(4):
        assert abs(y[w, (g.nv - 1) // 2, (g.nu - 1) // 2] - n) < 1e-12


def test_cone_backprojector_magnification_weights():
    # B of a constant-1 sinogram = sum over views of (M/pu)(M/pv) with
    # M = sdd / (sid - <x, source direction>) wherever the projection of the
    # voxel lands well inside the detector.
    n = 8
    g = small_cone(n=n, nu=41, nv=41, views=5, pitch=1.0, sid=30.0, sdd=60.0)
    ops = Cone3DOps(g)
    xb = ops.B(np.ones(g.m)).reshape(n, n, n)
    X = np.arange(n) - (n - 1) / 2.0
    beta = 2 * math.pi * np.arange(5) / 5
    for (k, i, j) in [(0, 0, 0), (3, 4, 5), (7, 2, 6), (4, 4, 4)]:
        p = np.array([X[j], X[i], X[k]])
        ref = 0.0
        for b in beta:
            M = g.sdd / (g.sid - (p[0] * math.cos(b) + p[1] * math.sin(b)))
            ref += M * M
        assert abs(xb[k, i, j] - ref) < 1e-11 * ref


def test_cone_backprojector_close_to_transpose_in_scale():
    # <A x, 1> vs <x, B 1>: the backprojector's magnification weight makes B
    # the same scale as A^T (interior, smooth test function).
    n = 12
    g = small_cone(n=n, nu=41, nv=41, views=16, pitch=1.0, sid=30.0, sdd=60.0)
    ops = Cone3DOps(g)
    X = np.arange(n) - (n - 1) / 2.0
    Z, Y, XX = np.meshgrid(X, X, X, indexing="ij")
    x = np.exp(-(XX ** 2 + Y ** 2 + Z ** 2) / 8.0).reshape(-1)
    lhs = float(ops.A(x).sum())
    rhs = float(x @ ops.B(np.ones(g.m)))
    assert abs(lhs - rhs) / abs(lhs) < 3e-2


def test_cone_backprojector_at_points_equals_full():
    g = Cone3D(12, 10, 8, 6, 16, 14, 1.3, 1.2, 30.0, 60.0)
    o = Cone3DOps(g)
    y = np.random.default_rng(1).standard_normal(g.m)
    idx = np.array([0, 5, 77, 123, 500, g.n - 1])
    assert np.array_equal(o.B_points(y, idx), o.B(y)[idx])


def test_fan_flat_approaches_parallel_beam(oracle_lib):
    # a distant source with magnification 2 and detector pitch 2: fan view
    # beta sees (to O(radius / sid)) the parallel projection at
    # theta = beta + pi/2 with unit bins, for both A and B
    from oracle.geometry import FanFlat2D, Par2D
    from oracle.operators import FanFlat2DOps, Par2DOps
    n, nd = 24, 37
    beta = np.array([0.0, 0.3, 1.1, 2.0, 3.9, 5.5])
    fan = FanFlat2DOps(FanFlat2D(n, n, beta.size, nd, 2.0, 1e7, 2e7, beta))
    par = Par2DOps(Par2D(n, n, beta.size, nd, 1.0, beta + np.pi / 2))
    r = np.random.default_rng(2)
    x = r.uniform(size=n * n)
    y = r.standard_normal(beta.size * nd)
    ea = np.linalg.norm(fan.A(x) - par.A(x)) / np.linalg.norm(par.A(x))
    eb = np.linalg.norm(fan.B(y) - par.B(y)) / np.linalg.norm(par.B(y))
    assert ea < 1e-5 and eb < 1e-5


def test_fan_flat_disk_chords(oracle_lib):
    # A of a uniform disk against the chord lengths of the fan rays (the
    # pixelisation error of the disk boundary shrinks at first order)
    from oracle.geometry import FanFlat2D
    from oracle.operators import FanFlat2DOps
    errs = []
    for n in (32, 64, 128):
        R = 0.3 * n
        c = np.arange(n) - 0.5 * (n - 1)
        X, Y = np.meshgrid(c, c)
        sub = 8
        o = (np.arange(sub) + 0.5) / sub - 0.5
        img = np.zeros((n, n))
        for ox in o:
            for oy in o:
                img += ((X + ox) ** 2 + (Y + oy) ** 2 <= R * R)
        img /= sub * sub
        nu, pu, sid, sdd = int(2 * n), 1.0, 2.0 * n, 4.0 * n
        g = FanFlat2D(n, n, 12, nu, pu, sid, sdd)
        y = FanFlat2DOps(g).A(img).reshape(12, nu)
        want = np.zeros_like(y)
        for w in range(12):
            S, D, U = g.src[w], g.det[w], g.eu[w]
            for cc in range(nu):
                P = D + (cc - 0.5 * (nu - 1)) * pu * U
                d = (P - S) / np.linalg.norm(P - S)
                # distance of the line from the centre, chord 2 sqrt(R^2 - h^2)
                h = abs(S[0] * d[1] - S[1] * d[0])
                want[w, cc] = 2 * np.sqrt(max(R * R - h * h, 0.0))
        errs.append(np.abs(y - want).max() / (2 * R))
    assert errs[0] > errs[1] > errs[2] and errs[2] < 0.03


def _bilinear_sino(rng, views, nu, nv, pu, pv):
    """A sinogram whose view w is f_w(u, v) = a + b u + c v + d u v in the
    physical detector coordinates u = (col - (nu-1)/2) pu, v = (row - (nv-1)/2) pv:
    bilinear interpolation reproduces such a function exactly."""
    coef = rng.uniform(0.5, 1.5, size=(views, 4)) * np.array([1.0, 0.3, -0.2, 0.05])
    u = (np.arange(nu) - 0.5 * (nu - 1)) * pu
    v = (np.arange(nv) - 0.5 * (nv - 1)) * pv
    U, V = np.meshgrid(u, v)            # [nv][nu]
    y = np.stack([a + b * U + c * V + d * U * V for a, b, c, d in coef])
    return y, coef


def test_cone_backprojector_of_a_bilinear_sinogram():
    # Voxel-driven B on a sinogram that is bilinear in the detector
    # coordinates, against the textbook projection of a point X from the
    # source: magnification M = sdd / (sid - <X, s>) with s the unit source
    # direction, detector coordinates u = M <X, e_u> and v = M X_z (the
    # detector is perpendicular to s, centred on the central ray).  Then
    # (B y)(X) = sum_w (M/pu)(M/pv) f_w(u, v) exactly wherever the projection
    # stays inside the detector.  A mirrored or swapped detector axis, a
    # half-pixel offset of the detector centre or a wrong weight power all
    # change the result by O(1).
    nx, ny, nz, views, nu, nv, pu, pv, sid, sdd = 9, 7, 6, 5, 45, 37, 0.9, 1.1, 30.0, 62.0
    beta = np.array([0.2, 1.3, 2.5, 3.7, 5.1])
    g = Cone3D(nx, ny, nz, views, nu, nv, pu, pv, sid, sdd, beta)
    ops = Cone3DOps(g)
    y, coef = _bilinear_sino(np.random.default_rng(5), views, nu, nv, pu, pv)
    xb = ops.B(y.reshape(-1)).reshape(nz, ny, nx)
    cx, cy, cz = 0.5 * (nx - 1), 0.5 * (ny - 1), 0.5 * (nz - 1)
    worst = 0.0
    for k in range(nz):
        for i in range(ny):
            for j in range(nx):
                X = np.array([j - cx, i - cy, k - cz])
                ref = 0.0
                for w, b in enumerate(beta):
                    s = np.array([math.cos(b), math.sin(b), 0.0])
                    eu = np.array([-math.sin(b), math.cos(b), 0.0])
                    M = sdd / (sid - X @ s)
                    u, v = M * (X @ eu), M * X[2]
                    # the projection stays at least two bins inside the detector
                    assert abs(u) < (0.5 * (nu - 1) - 2) * pu and abs(v) < (0.5 * (nv - 1) - 2) * pv
                    a, bb, c, d = coef[w]
                    ref += (M / pu) * (M / pv) * (a + bb * u + c * v + d * u * v)
                worst = max(worst, abs(xb[k, i, j] - ref) / abs(ref))
    assert worst < 1e-12, worst


def test_fan_backprojector_finite_source_closed_form(oracle_lib):
    # Pixel-driven fan B at a finite source distance (magnification ~ 2):
    # for a sinogram linear in the detector coordinate u = (col - (nu-1)/2) pu,
    # f_w(u) = a + b u, linear interpolation is exact, and with the textbook
    # projection M = sdd / (sid - <X, s>), u = M <X, e_u> the result is
    # (B y)(X) = sum_w (M/pu) f_w(u).  B 1 = sum_w M/pu is the case b = 0.  A
    # weight (M/pu)^2, a mirrored u axis or a half-bin offset fail.
    from oracle.geometry import FanFlat2D
    from oracle.operators import FanFlat2DOps
    nx, ny, views, nu, pu, sid, sdd = 13, 10, 7, 61, 0.8, 24.0, 50.0
    beta = np.array([0.1, 0.9, 1.7, 2.6, 3.3, 4.4, 5.9])
    g = FanFlat2D(nx, ny, views, nu, pu, sid, sdd, beta)
    ops = FanFlat2DOps(g)
    rng = np.random.default_rng(8)
    coef = rng.uniform(0.5, 1.5, size=(views, 2)) * np.array([1.0, 0.4])
    u = (np.arange(nu) - 0.5 * (nu - 1)) * pu
    for lin in (False, True):
        y = np.stack([a + (b * u if lin else 0.0 * u) for a, b in coef])
        xb = ops.B(y.reshape(-1)).reshape(ny, nx)
        cx, cy = 0.5 * (nx - 1), 0.5 * (ny - 1)
        for i in range(ny):
            for j in range(nx):
                X = np.array([j - cx, i - cy])
                ref = 0.0
                for w, b in enumerate(beta):
                    s = np.array([math.cos(b), math.sin(b)])
                    eu = np.array([-math.sin(b), math.cos(b)])
                    M = sdd / (sid - X @ s)
                    uu = M * (X @ eu)
                    assert abs(uu) < (0.5 * (nu - 1) - 2) * pu
                    a, bb = coef[w]
                    ref += (M / pu) * (a + (bb * uu if lin else 0.0))
                assert abs(xb[i, j] - ref) < 1e-12 * abs(ref), (lin, i, j, xb[i, j], ref)
