// 2D parallel-beam operators for gfx950 (wave64).
//
//   A   Joseph's ray-driven projector (the forward model of Sec. 1, eq. (1)).
//   A^T the exact transpose of A, as a per-pixel gather (matched pair, Sec. 3).
//   B   pixel-driven backprojector with linear interpolation (the unmatched
//       B != A^T of eqs. (4)-(5)).
//
// Layout: one thread per ray (A) or per pixel (A^T, B).  Lanes of a wave run
// along detector bins (A) or along a 16-pixel image row (B), so consecutive
// lanes touch neighbouring memory.  Rays that march over image columns read
// a transposed copy of the image, so every ray walks rows of a row-major
// array and its two interpolation taps are adjacent.  All interpolation is
// done in software (FP32, FP64 for double images); nothing uses atomics, so
// results are deterministic.
#include "ops.h"

namespace abba {

// ------------------------------------------------------------ transpose ---
template <typename T>
__global__ __launch_bounds__(256) void transpose_k(VecRef xr, T *__restrict__ xT, int nx, int ny,
                                                   const int *kdev, const int *active) {
    const int s = blockIdx.z;
    if (active && !active[s]) return;
    const int k = kdev ? *kdev : 0;
    const T *x = vec_ptr<T>(xr, s, k);
    T *o = xT + (int64_t)s * nx * ny;
    __shared__ T tile[32][33];
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;   // 32 x 8
    const int j0 = blockIdx.x * 32, i0 = blockIdx.y * 32;
#pragma unroll
    for (int r = ty; r < 32; r += 8) {
        const int i = i0 + r, j = j0 + tx;
        if (i < ny && j < nx) tile[r][tx] = x[(int64_t)i * nx + j];
    }
    __syncthreads();
#pragma unroll
    for (int r = ty; r < 32; r += 8) {
        const int j = j0 + r, i = i0 + tx;
        if (i < ny && j < nx) o[(int64_t)j * ny + i] = tile[tx][r];
    }
}

// v if keep, else +0.0, by masking the bits: the loaded value is always
// consumed, so the compiler cannot move the load under a branch.
__device__ __forceinline__ float keep_if(float v, bool keep) {
    return __uint_as_float(__float_as_uint(v) & (keep ? 0xffffffffu : 0u));
}
__device__ __forceinline__ double keep_if(double v, bool keep) {
    const unsigned long long m = keep ? ~0ull : 0ull;
    return __longlong_as_double((long long)((unsigned long long)__double_as_longlong(v) & m));
}

// ---------------------------------------------------------- Joseph A -------
template <typename TI, typename TO>
__global__ __launch_bounds__(256) void joseph2d_fwd_k(VecRef xr, const TI *__restrict__ xT, VecRef yr,
                                                      const AngleTab<typename acc_of<TI>::type> *__restrict__ tab,
                                                      int nx, int ny, int nd, typename acc_of<TI>::type ds,
                                                      typename acc_of<TI>::type cd, const int *kdev,
                                                      const int *active) {
    typedef typename acc_of<TI>::type T;
    const int s = blockIdx.z;
    if (active && !active[s]) return;
    const int d = blockIdx.x * blockDim.x + threadIdx.x;
    if (d >= nd) return;
    const int k = kdev ? *kdev : 0;
    const int a = blockIdx.y;
    const AngleTab<T> t = tab[a];
    const TI *P;
    int R, C;
    if (t.rowmarch) {
        P = vec_ptr<const TI>(xr, s, k);
        R = ny;
        C = nx;
    } else {
        P = xT + (int64_t)s * nx * ny;
        R = nx;
        C = ny;
    }
    const T sd = ((T)d - cd) * ds;
    const T u0 = fma(sd, t.inv_c, t.off);
    // Rows whose crossing lies in (-1, C), widened by one row on each side.
    // Both ends are clamped to [-2, R+1] before the conversion to int: for a
    // ray that misses the image at a near-zero slope (the column march at
    // exactly 90 degrees has slope cos/sin ~ 6e-17) the quotients are ~1e17
    // and would otherwise saturate the conversion.  So r0 is in [0, R], r1 in
    // [-1, R-1] and the step count below cannot overflow.
    int r0 = 0, r1 = R - 1;
    if (t.slope != (T)0) {
        T ra = (u0 + (T)1) / t.slope, rb = (u0 - (T)C) / t.slope;
        T lo = fmin(ra, rb), hi = fmax(ra, rb);
        lo = fmin(fmax(lo, (T)-2), (T)(R + 1));
        hi = fmin(fmax(hi, (T)-2), (T)(R + 1));
        r0 = max(0, (int)floor(lo) - 1);
        r1 = min(R - 1, (int)ceil(hi) + 1);
    } else if (!(u0 > (T)-1 && u0 < (T)C)) {
        r1 = -1;
    }
    const int nsteps = r1 - r0 + 1;   // <= 0 when the ray misses the image
    // Same clamped loads as one step at a time, four steps per pass: every
    // load is issued before any is consumed, and a tap outside the row is
    // zeroed by masking its bits (no branch, so no per-step memory wait).
    T acc0 = 0, acc1 = 0;
    int r = r0;
    for (int i = 0; i + 4 <= nsteps; i += 4, r += 4) {
        T v[8], f[4];
        bool ok[8];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const T u = fma(-(T)(r + q), t.slope, u0);
            const T jf = floor(u);
            f[q] = u - jf;
            const int j = (int)jf;
            const TI *row = P + (int64_t)(r + q) * C;
            const int ja = min(max(j, 0), C - 1), jb = min(max(j + 1, 0), C - 1);
            v[2 * q] = (T)row[ja];
            v[2 * q + 1] = (T)row[jb];
            ok[2 * q] = j >= 0 && j < C;
            ok[2 * q + 1] = j + 1 >= 0 && j + 1 < C;
        }
#pragma unroll
        for (int e = 0; e < 8; ++e) v[e] = keep_if(v[e], ok[e]);
        acc0 += fma(f[0], v[1] - v[0], v[0]);
        acc1 += fma(f[1], v[3] - v[2], v[2]);
        acc0 += fma(f[2], v[5] - v[4], v[4]);
        acc1 += fma(f[3], v[7] - v[6], v[6]);
    }
    for (; r <= r1; ++r) {   // the last nsteps mod 4 rows
        const T u = fma(-(T)r, t.slope, u0);
        const T jf = floor(u);
        const T f = u - jf;
        const int j = (int)jf;
        const TI *row = P + (int64_t)r * C;
        const int ja = min(max(j, 0), C - 1), jb = min(max(j + 1, 0), C - 1);
        const T v0 = keep_if((T)row[ja], j >= 0 && j < C);
        const T v1 = keep_if((T)row[jb], j + 1 >= 0 && j + 1 < C);
        acc0 += fma(f, v1 - v0, v0);
    }
    const T acc = acc0 + acc1;
    store_as<TO>(vec_ptr<TO>(yr, s, k), (int64_t)a * nd + d, acc * t.w);
}

// ------------------------------------------------ pixel-driven B / A^T -----
template <typename TIN, typename TI, bool EXACT_T>
__global__ __launch_bounds__(256) void back2d_k(VecRef yr, VecRef xr,
                                                const AngleTab<typename acc_of<TI>::type> *__restrict__ tab,
                                                int nx, int ny, int na, int nd,
                                                typename acc_of<TI>::type ds, typename acc_of<TI>::type cd,
                                                typename acc_of<TI>::type wb, int nmax, const int *kdev,
                                                const int *active) {
    typedef typename acc_of<TI>::type T;
    const int s = blockIdx.z;
    if (active && !active[s]) return;
    const int k = kdev ? *kdev : 0;
    const int j = blockIdx.x * 16 + (threadIdx.x & 15);
    const int i = blockIdx.y * 16 + (threadIdx.x >> 4);
    const T X = (T)j - (T)0.5 * (T)(nx - 1);
    const T Y = (T)i - (T)0.5 * (T)(ny - 1);
    const TIN *y = vec_ptr<const TIN>(yr, s, k);
    T acc = 0;
    if (!EXACT_T) {
        // B: linear interpolation of row a at t = (X cos + Y sin)/ds + cd,
        // four angles per pass with masked (branch-free) taps
        T a1 = 0, a2 = 0, a3 = 0;
        int a = 0;
        for (; a + 3 < na; a += 4) {
            T v[8], f[4];
            bool ok[8];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const T t = fma(X, tab[a + q].cb, fma(Y, tab[a + q].sb, cd));
                const T df = floor(t);
                f[q] = t - df;
                const int d = (int)fmax(fmin(df, (T)nd), (T)-2);
                const TIN *row = y + (int64_t)(a + q) * nd;
                const int da = min(max(d, 0), nd - 1), db = min(max(d + 1, 0), nd - 1);
                v[2 * q] = (T)load_as<TIN>(row, da);
                v[2 * q + 1] = (T)load_as<TIN>(row, db);
                ok[2 * q] = d >= 0 && d < nd;
                ok[2 * q + 1] = d + 1 >= 0 && d + 1 < nd;
            }
#pragma unroll
            for (int e = 0; e < 8; ++e) v[e] = keep_if(v[e], ok[e]);
            acc += fma(f[0], v[1] - v[0], v[0]);
            a1 += fma(f[1], v[3] - v[2], v[2]);
            a2 += fma(f[2], v[5] - v[4], v[4]);
            a3 += fma(f[3], v[7] - v[6], v[6]);
        }
        for (; a < na; ++a) {
            const T t = fma(X, tab[a].cb, fma(Y, tab[a].sb, cd));
            const T df = floor(t);
            const T f = t - df;
            const int d = (int)fmax(fmin(df, (T)nd), (T)-2);
            const TIN *row = y + (int64_t)a * nd;
            const int da = min(max(d, 0), nd - 1), db = min(max(d + 1, 0), nd - 1);
            const T v0 = keep_if((T)load_as<TIN>(row, da), d >= 0 && d < nd);
            const T v1 = keep_if((T)load_as<TIN>(row, db), d + 1 >= 0 && d + 1 < nd);
            acc += fma(f, v1 - v0, v0);
        }
        acc = (acc + a1) + (a2 + a3);
        acc *= wb;
    } else {
        // A^T: gather the rays whose Joseph interpolation hat covers this
        // pixel: weight hat((s_d - p)/c)/|c|, p = X cos + Y sin, c the
        // dominant direction cosine of the angle.
        for (int a = 0; a < na; ++a) {
            const AngleTab<T> t = tab[a];
            const T p = fma(X, t.cs, Y * t.sn);
            const T tl = (p - t.absc) / ds + cd;
            const int d0 = (int)fmax(fmin(floor(tl), (T)nd), (T)(-nmax - 1));
            const TIN *row = y + (int64_t)a * nd;
            for (int q = 0; q <= nmax; ++q) {
                const int d = d0 + q;
                const T sdd = ((T)d - cd) * ds;
                const T h = (T)1 - fabs(sdd - p) * t.w;
                const int dc = min(max(d, 0), nd - 1);
                T v = (T)load_as<TIN>(row, dc);
                v = (d >= 0 && d < nd && h > (T)0) ? v : (T)0;
                acc = fma(h * t.w, v, acc);
            }
        }
    }
    if (i < ny && j < nx) vec_ptr<TI>(xr, s, k)[(int64_t)i * nx + j] = (TI)acc;
}

// ------------------------------------------------------------ host side ----
template <typename TI, typename TO>
static int fwd_launch(const abba_op *op, VecRef x, VecRef y, int batch, void *xT, const Launch &L) {
    typedef typename acc_of<TI>::type T;
    const int nx = op->g.nx, ny = op->g.ny, na = op->g.n_angles, nd = op->g.det_u;
    dim3 tg((nx + 31) / 32, (ny + 31) / 32, batch);
    hipLaunchKernelGGL(transpose_k<TI>, tg, dim3(256), 0, L.stream, x, (TI *)xT, nx, ny, L.kdev, L.active);
    ABBA_LAUNCHED("transpose_k");
    dim3 grid((nd + 255) / 256, na, batch);
    hipLaunchKernelGGL((joseph2d_fwd_k<TI, TO>), grid, dim3(256), 0, L.stream, x, (const TI *)xT, y,
                       (const AngleTab<T> *)op->tab, nx, ny, nd, (T)op->g.det_pitch_u,
                       (T)(0.5 * (nd - 1)), L.kdev, L.active);
    ABBA_LAUNCHED("joseph2d_fwd_k");
    return ABBA_OK;
}

int par2d_forward(const abba_op *op, VecRef x, VecRef y, int y_dtype, int batch, void *xT, const Launch &L) {
    if (batch <= 0) return ABBA_OK;
    if (op->img_dtype == ABBA_F64) {
        if (y_dtype != ABBA_F64) return ABBA_ERR_DTYPE;
        return fwd_launch<double, double>(op, x, y, batch, xT, L);
    }
    if (y_dtype == ABBA_F32) return fwd_launch<float, float>(op, x, y, batch, xT, L);
    if (y_dtype == ABBA_BF16) return fwd_launch<float, bf16>(op, x, y, batch, xT, L);
    return ABBA_ERR_DTYPE;
}

template <typename TIN, typename TI>
static int back_launch(const abba_op *op, VecRef y, VecRef x, int batch, const Launch &L) {
    typedef typename acc_of<TI>::type T;
    const int nx = op->g.nx, ny = op->g.ny, na = op->g.n_angles, nd = op->g.det_u;
    const double ds = op->g.det_pitch_u;
    dim3 grid((nx + 15) / 16, (ny + 15) / 16, batch);
    if (op->kind == ABBA_OP_JOSEPH_T) {
        const int nmax = (int)ceil(2.0 / ds) + 2;
        hipLaunchKernelGGL((back2d_k<TIN, TI, true>), grid, dim3(256), 0, L.stream, y, x,
                           (const AngleTab<T> *)op->tab, nx, ny, na, nd, (T)ds, (T)(0.5 * (nd - 1)),
                           (T)(1.0 / ds), nmax, L.kdev, L.active);
    } else {
        hipLaunchKernelGGL((back2d_k<TIN, TI, false>), grid, dim3(256), 0, L.stream, y, x,
                           (const AngleTab<T> *)op->tab, nx, ny, na, nd, (T)ds, (T)(0.5 * (nd - 1)),
                           (T)(1.0 / ds), 0, L.kdev, L.active);
    }
    ABBA_LAUNCHED("back2d_k");
    return ABBA_OK;
}

int par2d_back(const abba_op *op, VecRef y, int y_dtype, VecRef x, int batch, const Launch &L) {
    if (batch <= 0) return ABBA_OK;
    if (op->img_dtype == ABBA_F64) {
        if (y_dtype != ABBA_F64) return ABBA_ERR_DTYPE;
        return back_launch<double, double>(op, y, x, batch, L);
    }
    if (y_dtype == ABBA_F32) return back_launch<float, float>(op, y, x, batch, L);
    if (y_dtype == ABBA_BF16) return back_launch<bf16, float>(op, y, x, batch, L);
    return ABBA_ERR_DTYPE;
}

}  // namespace abba
