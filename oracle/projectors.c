/*
 * ORACLE -- test infrastructure, not part of the product.
 *
 * Plain, slow, FP64 CPU definitions of the CT operators used by hybrid
 * AB-/BA-GMRES (the forward projector A of the linear model Ax ~ b in Sec. 1,
 * eq. (1), and an unmatched backprojector B != A^T, Sec. 2, eqs. (4)-(5)).
 * The paper does not fix a discretisation (its experiments call ASTRA); the
 * readings implemented here are:
 *
 *   A   -- Joseph's ray-driven projector: for each ray, march along the
 *          dominant image axis and linearly interpolate the image along the
 *          other axis at the ray's crossing, weighted by the step length.
 *   A^T -- the exact transpose of A, written as a scatter over the same
 *          ray steps (each step's two interpolation weights are added back
 *          into the two pixels they were read from).
 *   B   -- pixel-driven backprojector: for each pixel and angle, linearly
 *          interpolate the sinogram row at the pixel's projected detector
 *          coordinate.  Weight 1/(detector pitch), so B has the same scale
 *          as A^T.
 *
 * 2D parallel geometry: pixel (i,j) centre (X_j, Y_i) = (j-(nx-1)/2,
 * i-(ny-1)/2); bin d at s_d = (d-(D-1)/2)*ds; ray (a,d) is the line
 * {p : p.(cos t_a, sin t_a) = s_d}.  Row-march rays (|cos| dominant) cross
 * each row i at X = (s - Y_i sin)/cos; column-march rays cross each column j
 * at Y = (s - X_j cos)/sin.  Pixels outside the image read as zero.
 *
 * Each output element is computed by one plain loop in definition order; the
 * OpenMP pragmas only split independent output elements across threads.
 */
#include <math.h>
#include <stddef.h>
#include <string.h>

/* ---------------------------------------------------------------- 2D ---- */

static double pix2(const double *img, int nx, int ny, int i, int j)
{
    if (i < 0 || i >= ny || j < 0 || j >= nx) return 0.0;
    return img[(size_t)i * nx + j];
}

/* y[a][d] = A x for one slice. */
static void joseph2d_one(const double *x, double *y, int nx, int ny,
                         int na, int nd, double ds,
                         const double *cs, const double *sn, const int *rowmarch)
{
    const double cx = 0.5 * (nx - 1), cy = 0.5 * (ny - 1), cd = 0.5 * (nd - 1);
    #pragma omp parallel for schedule(static)
    for (int a = 0; a < na; ++a) {
        for (int d = 0; d < nd; ++d) {
            const double s = (d - cd) * ds;
            double acc = 0.0;
            if (rowmarch[a]) {
                for (int i = 0; i < ny; ++i) {
                    const double Y = i - cy;
                    const double u = (s - Y * sn[a]) / cs[a] + cx;
                    const double j0 = floor(u);
                    const double f = u - j0;
                    const int j = (int)j0;
                    if (j0 < -2.0 || j0 > nx + 1.0) continue;   /* both taps outside */
                    acc += (1.0 - f) * pix2(x, nx, ny, i, j) + f * pix2(x, nx, ny, i, j + 1);
                }
                y[(size_t)a * nd + d] = acc / fabs(cs[a]);
            } else {
                for (int j = 0; j < nx; ++j) {
                    const double X = j - cx;
                    const double v = (s - X * cs[a]) / sn[a] + cy;
                    const double i0 = floor(v);
                    const double g = v - i0;
                    const int i = (int)i0;
                    if (i0 < -2.0 || i0 > ny + 1.0) continue;
                    acc += (1.0 - g) * pix2(x, nx, ny, i, j) + g * pix2(x, nx, ny, i + 1, j);
                }
                y[(size_t)a * nd + d] = acc / fabs(sn[a]);
            }
        }
    }
}

/* x = A^T y for one slice, by scattering every ray step of A (serial). */
static void joseph2d_t_one(const double *y, double *x, int nx, int ny,
                           int na, int nd, double ds,
                           const double *cs, const double *sn, const int *rowmarch)
{
    const double cx = 0.5 * (nx - 1), cy = 0.5 * (ny - 1), cd = 0.5 * (nd - 1);
    memset(x, 0, sizeof(double) * (size_t)nx * ny);
    for (int a = 0; a < na; ++a) {
        for (int d = 0; d < nd; ++d) {
            const double s = (d - cd) * ds;
            if (rowmarch[a]) {
                const double w = y[(size_t)a * nd + d] / fabs(cs[a]);
                for (int i = 0; i < ny; ++i) {
                    const double Y = i - cy;
                    const double u = (s - Y * sn[a]) / cs[a] + cx;
                    const double j0 = floor(u);
                    const double f = u - j0;
                    const int j = (int)j0;
                    if (j0 < -2.0 || j0 > nx + 1.0) continue;
                    if (j >= 0 && j < nx) x[(size_t)i * nx + j] += (1.0 - f) * w;
                    if (j + 1 >= 0 && j + 1 < nx) x[(size_t)i * nx + j + 1] += f * w;
                }
            } else {
                const double w = y[(size_t)a * nd + d] / fabs(sn[a]);
                for (int j = 0; j < nx; ++j) {
                    const double X = j - cx;
                    const double v = (s - X * cs[a]) / sn[a] + cy;
                    const double i0 = floor(v);
                    const double g = v - i0;
                    const int i = (int)i0;
                    if (i0 < -2.0 || i0 > ny + 1.0) continue;
                    if (i >= 0 && i < ny) x[(size_t)i * nx + j] += (1.0 - g) * w;
                    if (i + 1 >= 0 && i + 1 < ny) x[(size_t)(i + 1) * nx + j] += g * w;
                }
            }
        }
    }
}

/* x = B y for one slice: pixel-driven linear interpolation. */
static void pixbp2d_one(const double *y, double *x, int nx, int ny,
                        int na, int nd, double ds,
                        const double *cs, const double *sn)
{
    const double cx = 0.5 * (nx - 1), cy = 0.5 * (ny - 1), cd = 0.5 * (nd - 1);
    #pragma omp parallel for schedule(static)
    for (int i = 0; i < ny; ++i) {
        for (int j = 0; j < nx; ++j) {
            const double X = j - cx, Y = i - cy;
            double acc = 0.0;
            for (int a = 0; a < na; ++a) {
                const double t = (X * cs[a] + Y * sn[a]) / ds + cd;
                const double d0 = floor(t);
                const double f = t - d0;
                const int d = (int)d0;
                double v0 = 0.0, v1 = 0.0;
                if (d >= 0 && d < nd) v0 = y[(size_t)a * nd + d];
                if (d + 1 >= 0 && d + 1 < nd) v1 = y[(size_t)a * nd + d + 1];
                acc += (1.0 - f) * v0 + f * v1;
            }
            x[(size_t)i * nx + j] = acc / ds;
        }
    }
}

void oracle_joseph2d(const double *x, double *y, int batch, int nx, int ny,
                     int na, int nd, double ds,
                     const double *cs, const double *sn, const int *rowmarch)
{
    for (int b = 0; b < batch; ++b)
        joseph2d_one(x + (size_t)b * nx * ny, y + (size_t)b * na * nd,
                     nx, ny, na, nd, ds, cs, sn, rowmarch);
}

void oracle_joseph2d_t(const double *y, double *x, int batch, int nx, int ny,
                       int na, int nd, double ds,
                       const double *cs, const double *sn, const int *rowmarch)
{
    #pragma omp parallel for schedule(dynamic)
    for (int b = 0; b < batch; ++b)
        joseph2d_t_one(y + (size_t)b * na * nd, x + (size_t)b * nx * ny,
                       nx, ny, na, nd, ds, cs, sn, rowmarch);
}

void oracle_pixbp2d(const double *y, double *x, int batch, int nx, int ny,
                    int na, int nd, double ds, const double *cs, const double *sn)
{
    for (int b = 0; b < batch; ++b)
        pixbp2d_one(y + (size_t)b * na * nd, x + (size_t)b * nx * ny,
                    nx, ny, na, nd, ds, cs, sn);
}

/* ---------------------------------------------------------------- 3D ---- */
/*
 * Circular cone beam.  Volume [nz][ny][nx], unit voxels centred at the
 * origin (X_j, Y_i, Z_k as in 2D).  View v has source S_v and a flat
 * detector with centre D_v and in-plane unit axes eu_v (columns, index c)
 * and ev_v (rows, index r); pixel (r,c) sits at
 *   P = D_v + (c-(nu-1)/2)*pu*eu_v + (r-(nv-1)/2)*pv*ev_v.
 * The caller passes, per view, src[3], det[3], eu[3], ev[3] (FP64).
 *
 * A: for the line S->P, march over the planes of its dominant axis and take
 *    the bilinear interpolation of the volume in each plane, weighted by the
 *    ray length between two planes (|dir| / |dir_major|).
 * B: voxel-driven.  Project the voxel centre from S onto the detector plane,
 *    bilinearly interpolate the view there, weight (M/pu)*(M/pv) where
 *    M = |P - S|_along-axis / |x - S|_along-axis is the magnification.
 */

static double vox3(const double *vol, int nx, int ny, int nz, int k, int i, int j)
{
    if (k < 0 || k >= nz || i < 0 || i >= ny || j < 0 || j >= nx) return 0.0;
    return vol[((size_t)k * ny + i) * nx + j];
}

/* bilinear sample of the plane indexed by (p, q) at continuous (fp, fq);
 * fetch(p, q) is the voxel at plane coordinates p (slow) and q (fast). */
#define BILIN(FETCH, up, uq) do {                                            \
        const double p0 = floor(up), q0 = floor(uq);                          \
        const double fp_ = (up) - p0, fq_ = (uq) - q0;                        \
        const int ip = (int)p0, iq = (int)q0;                                 \
        val = (1.0 - fp_) * ((1.0 - fq_) * FETCH(ip, iq) + fq_ * FETCH(ip, iq + 1)) \
            + fp_ * ((1.0 - fq_) * FETCH(ip + 1, iq) + fq_ * FETCH(ip + 1, iq + 1)); \
    } while (0)

static double cone_ray(const double *vol, int nx, int ny, int nz,
                       const double S[3], const double P[3])
{
    const double cx = 0.5 * (nx - 1), cy = 0.5 * (ny - 1), cz = 0.5 * (nz - 1);
    const double d[3] = { P[0] - S[0], P[1] - S[1], P[2] - S[2] };
    const double ad[3] = { fabs(d[0]), fabs(d[1]), fabs(d[2]) };
    const double len = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
    double acc = 0.0, val;
    if (ad[0] >= ad[1] && ad[0] >= ad[2]) {            /* march over x planes */
        for (int j = 0; j < nx; ++j) {
            const double t = ((j - cx) - S[0]) / d[0];
            const double yy = S[1] + t * d[1] + cy;       /* continuous row index  */
            const double zz = S[2] + t * d[2] + cz;       /* continuous slice index */
#define F(p, q) vox3(vol, nx, ny, nz, (p), (q), j)
            BILIN(F, zz, yy);
#undef F
            acc += val;
        }
        return acc * len / ad[0];
    } else if (ad[1] >= ad[2]) {                        /* march over y planes */
        for (int i = 0; i < ny; ++i) {
            const double t = ((i - cy) - S[1]) / d[1];
            const double xx = S[0] + t * d[0] + cx;
            const double zz = S[2] + t * d[2] + cz;
#define F(p, q) vox3(vol, nx, ny, nz, (p), i, (q))
            BILIN(F, zz, xx);
#undef F
            acc += val;
        }
        return acc * len / ad[1];
    } else {                                            /* march over z planes */
        for (int k = 0; k < nz; ++k) {
            const double t = ((k - cz) - S[2]) / d[2];
            const double xx = S[0] + t * d[0] + cx;
            const double yy = S[1] + t * d[1] + cy;
#define F(p, q) vox3(vol, nx, ny, nz, k, (p), (q))
            BILIN(F, yy, xx);
#undef F
            acc += val;
        }
        return acc * len / ad[2];
    }
}

void oracle_cone_fwd(const double *vol, double *sino, int nx, int ny, int nz,
                     int nviews, int nu, int nv, double pu, double pv,
                     const double *src, const double *det,
                     const double *eu, const double *ev)
{
    #pragma omp parallel for schedule(dynamic) collapse(2)
    for (int w = 0; w < nviews; ++w) {
        for (int r = 0; r < nv; ++r) {
            const double *S = src + 3 * w, *D = det + 3 * w;
            const double *U = eu + 3 * w, *V = ev + 3 * w;
            for (int c = 0; c < nu; ++c) {
                const double ou = (c - 0.5 * (nu - 1)) * pu;
                const double ov = (r - 0.5 * (nv - 1)) * pv;
                double P[3];
                for (int t = 0; t < 3; ++t) P[t] = D[t] + ou * U[t] + ov * V[t];
                sino[((size_t)w * nv + r) * nu + c] = cone_ray(vol, nx, ny, nz, S, P);
            }
        }
    }
}

/* B at selected voxels only: out[t] = (B y)[k_t][i_t][j_t] for the flat voxel
 * indices idx[t] = (k_t * ny + i_t) * nx + j_t, t < npts; the same sum as
 * oracle_cone_bp (used to check large volumes on a sample). */
static double cone_bp_voxel(const double *sino, int nx, int ny, int nz,
                            int nviews, int nu, int nv, double pu, double pv,
                            const double *src, const double *det,
                            const double *eu, const double *ev, int k, int i, int j);

void oracle_cone_bp_points(const double *sino, const long long *idx, double *out, int npts,
                           int nx, int ny, int nz, int nviews, int nu, int nv, double pu, double pv,
                           const double *src, const double *det, const double *eu, const double *ev)
{
    #pragma omp parallel for schedule(static)
    for (int t = 0; t < npts; ++t) {
        const long long f = idx[t];
        const int j = (int)(f % nx), i = (int)((f / nx) % ny), k = (int)(f / ((long long)nx * ny));
        out[t] = cone_bp_voxel(sino, nx, ny, nz, nviews, nu, nv, pu, pv, src, det, eu, ev, k, i, j);
    }
}

void oracle_cone_bp(const double *sino, double *vol, int nx, int ny, int nz,
                    int nviews, int nu, int nv, double pu, double pv,
                    const double *src, const double *det,
                    const double *eu, const double *ev)
{
    #pragma omp parallel for schedule(static) collapse(2)
    for (int k = 0; k < nz; ++k)
        for (int i = 0; i < ny; ++i)
            for (int j = 0; j < nx; ++j)
                vol[((size_t)k * ny + i) * nx + j] =
                    cone_bp_voxel(sino, nx, ny, nz, nviews, nu, nv, pu, pv, src, det, eu, ev, k, i, j);
}

static double cone_bp_voxel(const double *sino, int nx, int ny, int nz,
                            int nviews, int nu, int nv, double pu, double pv,
                            const double *src, const double *det,
                            const double *eu, const double *ev, int k, int i, int j)
{
    const double cx = 0.5 * (nx - 1), cy = 0.5 * (ny - 1), cz = 0.5 * (nz - 1);
    const double X[3] = { j - cx, i - cy, k - cz };
    double acc = 0.0;
    for (int w = 0; w < nviews; ++w) {
        const double *S = src + 3 * w, *D = det + 3 * w;
        const double *U = eu + 3 * w, *V = ev + 3 * w;
        /* detector normal n = eu x ev; intersect S + t (X - S) with
         * the plane (P - D).n = 0 */
        const double n[3] = { U[1] * V[2] - U[2] * V[1],
                              U[2] * V[0] - U[0] * V[2],
                              U[0] * V[1] - U[1] * V[0] };
        const double r[3] = { X[0] - S[0], X[1] - S[1], X[2] - S[2] };
        const double num = (D[0] - S[0]) * n[0] + (D[1] - S[1]) * n[1] + (D[2] - S[2]) * n[2];
        const double den = r[0] * n[0] + r[1] * n[1] + r[2] * n[2];
        const double M = num / den;               /* magnification */
        double P[3];
        for (int t = 0; t < 3; ++t) P[t] = S[t] + M * r[t] - D[t];
        const double uu = (P[0] * U[0] + P[1] * U[1] + P[2] * U[2]) / pu + 0.5 * (nu - 1);
        const double vv = (P[0] * V[0] + P[1] * V[1] + P[2] * V[2]) / pv + 0.5 * (nv - 1);
        const double *view = sino + (size_t)w * nv * nu;
        double val;
#define F(p, q) (((p) >= 0 && (p) < nv && (q) >= 0 && (q) < nu) ? view[(size_t)(p) * nu + (q)] : 0.0)
        BILIN(F, vv, uu);
#undef F
        acc += val * (M / pu) * (M / pv);
    }
    return acc;
}

/* ------------------------------------------------------------------------
 * 2D fan beam with a flat detector (the geometry of the paper's third test
 * problem).  View w: source S_w, detector centre D_w, column axis U_w (unit),
 * all in the image plane; bin c at D + (c - (nu-1)/2) pu U.
 *
 * A: for the line S->P, march over the columns (|dx| >= |dy|) or rows of the
 *    image and interpolate linearly along the other axis at the crossing,
 *    zero outside, weighted by |P - S| / |(P - S)_major| (the step length).
 * B: pixel driven.  Project the pixel centre X from S onto the detector line:
 *    M = (D - S).n / (X - S).n with n = the unit normal of the detector
 *    (pointing from the detector to the source), u = (S + M (X - S) - D).U / pu
 *    + (nu-1)/2; interpolate the view linearly at u (zero outside) and weight
 *    by M / pu.
 * ---------------------------------------------------------------------- */
static double fan_ray(const double *img, int nx, int ny, const double S[2], const double P[2])
{
    const double cx = 0.5 * (nx - 1), cy = 0.5 * (ny - 1);
    const double d[2] = { P[0] - S[0], P[1] - S[1] };
    const double len = sqrt(d[0] * d[0] + d[1] * d[1]);
    double acc = 0.0;
    if (fabs(d[0]) >= fabs(d[1])) {
        for (int j = 0; j < nx; ++j) {
            const double t = ((j - cx) - S[0]) / d[0];
            const double yy = S[1] + t * d[1] + cy;
            const double i0 = floor(yy), f = yy - i0;
            acc += (1.0 - f) * pix2(img, nx, ny, (int)i0, j) + f * pix2(img, nx, ny, (int)i0 + 1, j);
        }
        return acc * len / fabs(d[0]);
    }
    for (int i = 0; i < ny; ++i) {
        const double t = ((i - cy) - S[1]) / d[1];
        const double xx = S[0] + t * d[0] + cx;
        const double j0 = floor(xx), f = xx - j0;
        acc += (1.0 - f) * pix2(img, nx, ny, i, (int)j0) + f * pix2(img, nx, ny, i, (int)j0 + 1);
    }
    return acc * len / fabs(d[1]);
}

void oracle_fan_fwd(const double *img, double *sino, int nx, int ny, int nviews, int nu, double pu,
                    const double *src, const double *det, const double *eu)
{
    #pragma omp parallel for schedule(static) collapse(2)
    for (int w = 0; w < nviews; ++w) {
        for (int c = 0; c < nu; ++c) {
            const double *S = src + 2 * w, *D = det + 2 * w, *U = eu + 2 * w;
            const double ou = (c - 0.5 * (nu - 1)) * pu;
            const double P[2] = { D[0] + ou * U[0], D[1] + ou * U[1] };
            sino[(size_t)w * nu + c] = fan_ray(img, nx, ny, S, P);
        }
    }
}

void oracle_fan_bp(const double *sino, double *img, int nx, int ny, int nviews, int nu, double pu,
                   const double *src, const double *det, const double *eu)
{
    const double cx = 0.5 * (nx - 1), cy = 0.5 * (ny - 1);
    #pragma omp parallel for schedule(static) collapse(2)
    for (int i = 0; i < ny; ++i) {
        for (int j = 0; j < nx; ++j) {
            const double X[2] = { j - cx, i - cy };
            double acc = 0.0;
            for (int w = 0; w < nviews; ++w) {
                const double *S = src + 2 * w, *D = det + 2 * w, *U = eu + 2 * w;
                /* unit normal of the detector line, towards the source */
                const double n[2] = { U[1], -U[0] };
                const double num = (D[0] - S[0]) * n[0] + (D[1] - S[1]) * n[1];
                const double den = (X[0] - S[0]) * n[0] + (X[1] - S[1]) * n[1];
                const double M = num / den;
                const double P[2] = { S[0] + M * (X[0] - S[0]) - D[0], S[1] + M * (X[1] - S[1]) - D[1] };
                const double u = (P[0] * U[0] + P[1] * U[1]) / pu + 0.5 * (nu - 1);
                const double u0 = floor(u), f = u - u0;
                const int c = (int)u0;
                const double *row = sino + (size_t)w * nu;
                const double a = (c >= 0 && c < nu) ? row[c] : 0.0;
                const double b = (c + 1 >= 0 && c + 1 < nu) ? row[c + 1] : 0.0;
                acc += ((1.0 - f) * a + f * b) * (M / pu);
            }
            img[(size_t)i * nx + j] = acc;
        }
    }
}
