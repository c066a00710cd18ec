// 2D parallel-beam operators for gfx950 (wave64).
//
//   A   Joseph's ray-driven projector (the forward model of Sec. 1, eq. (1)).
//   A^T the exact transpose of A, as a per-pixel gather (matched pair, Sec. 3).
//   B   pixel-driven backprojector with linear interpolation (the unmatched
//       B != A^T of eqs. (4)-(5)).
//
// Layout: one thread per ray (A) or per pixel (A^T, B).  Lanes of a wave run
// along detector bins (A) or over a 16 x 4 pixel patch (B), so consecutive
// lanes touch neighbouring memory.
//
// A and B first copy their input into scratch with two zeros on each side of
// every row: the image row-major and transposed (rays that march over image
// columns walk rows of the transposed copy), the sinogram row by row.  An
// interpolation position is then clamped into [-2, len], and its two taps are
// always one 8-byte (FP64: 16-byte) load from the padded row whose values
// are exactly those of the zero-extended row.  There are no per-tap masks and
// no branches in the inner loops, and each step issues a single load.
//
// All launches are 1D; workgroups are renumbered so that each XCD (own L2)
// walks a contiguous range of slices (see xcd_remap).  Nothing uses atomics,
// so results are deterministic.
#include <algorithm>

#include "ops.h"

namespace abba {

constexpr int PAD = 2;   // zeros on each side of a padded row

// Largest number of workgroups per 1D launch (the grid's thread count stays
// below 2^31); larger batches are split into several launches.
constexpr uint32_t MAX_GROUPS = (1u << 31) / 256;
// Largest grid extent used in the y / z dimension.
constexpr int MAX_GRID_YZ = 65535;

// Renumbering of the workgroups of a 1D launch.  The hardware deals
// workgroup L to XCD L mod nxcc; XCD x gets the contiguous range of work
// items starting at x*q + min(x, r) (q, r = total / nxcc, total % nxcc), in
// dispatch order, so each XCD's L2 holds the slices it is working on.  The
// map is a bijection on [0, total) whatever the dispatch order really is.
__device__ __forceinline__ uint32_t xcd_remap(uint32_t L, uint32_t total, uint32_t nxcc) {
    const uint32_t q = total / nxcc, r = total % nxcc;
    const uint32_t x = L % nxcc, slot = L / nxcc;
    return x * q + min(x, r) + slot;
}

// Pointer to the element at 32-bit byte offset `off` from `base`; the two
// taps are read as p[0], p[1] so that they form one wide load.
template <typename T>
__device__ __forceinline__ const T *at_byte(const T *base, uint32_t off) {
    return reinterpret_cast<const T *>(reinterpret_cast<const char *>(base) + off);
}

// Clamp to [lo, hi] in one instruction (FP32); NaN does not occur here.
__device__ __forceinline__ float clampf(float x, float lo, float hi) { return __builtin_amdgcn_fmed3f(x, lo, hi); }
__device__ __forceinline__ double clampf(double x, double lo, double hi) { return fmin(fmax(x, lo), hi); }

// ------------------------------------------------------ padded copies -----
// Image -> xp [ny][nx + 4] (row-major) and xq [nx][ny + 4] (transposed), each
// row with PAD zeros on both sides.  32 x 32 tiles through LDS.
template <typename T>
__global__ __launch_bounds__(256) void pad_image_k(VecRef xr, T *__restrict__ xp, T *__restrict__ xq, int nx,
                                                   int ny, int s0, const int *kdev, const int *active) {
    const int s = s0 + blockIdx.z;
    if (active && !active[s]) return;
    const int k = kdev ? *kdev : 0;
    const T *x = vec_ptr<const T>(xr, s, k);
    const int lp = nx + 2 * PAD, lq = ny + 2 * PAD;
    T *op = xp + (int64_t)s * ny * lp;
    T *oq = xq + (int64_t)s * nx * lq;
    __shared__ T tile[32][33];
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;   // 32 x 8
    const int j0 = blockIdx.x * 32, i0 = blockIdx.y * 32;
#pragma unroll
    for (int r = ty; r < 32; r += 8) {
        const int i = i0 + r, j = j0 + tx;
        T v = (T)0;
        if (i < ny && j < nx) {
            v = x[(int64_t)i * nx + j];
            op[(int64_t)i * lp + j + PAD] = v;
        }
        tile[r][tx] = v;
    }
    // the pads of rows i0..i0+31 of xp: columns 0, 1, nx+2, nx+3
    if (blockIdx.x == 0 && threadIdx.x < 128) {
        const int i = i0 + (threadIdx.x >> 2), c = threadIdx.x & 3;
        if (i < ny) op[(int64_t)i * lp + (c < 2 ? c : nx + c)] = (T)0;
    }
    __syncthreads();
#pragma unroll
    for (int r = ty; r < 32; r += 8) {
        const int j = j0 + r, i = i0 + tx;
        if (i < ny && j < nx) oq[(int64_t)j * lq + i + PAD] = tile[tx][r];
    }
    // the pads of rows j0..j0+31 of xq
    if (blockIdx.y == 0 && threadIdx.x < 128) {
        const int j = j0 + (threadIdx.x >> 2), c = threadIdx.x & 3;
        if (j < nx) oq[(int64_t)j * lq + (c < 2 ? c : ny + c)] = (T)0;
    }
}

// Sinogram -> yp [na][nd + 4] in the accumulation type T, PAD zeros on both
// sides of every row.  One workgroup per (row, slice).
template <typename TIN, typename T>
__global__ __launch_bounds__(256) void pad_sino_k(VecRef yr, T *__restrict__ yp, int na, int nd, int s0,
                                                  const int *kdev, const int *active) {
    const int s = s0 + blockIdx.y;
    if (active && !active[s]) return;
    const int k = kdev ? *kdev : 0;
    const int a = blockIdx.x;
    const TIN *y = vec_ptr<const TIN>(yr, s, k) + (int64_t)a * nd;
    const int ld = nd + 2 * PAD;
    T *o = yp + ((int64_t)s * na + a) * ld;
    for (int c = threadIdx.x; c < ld; c += 256) {
        const int d = c - PAD;
        o[c] = (d >= 0 && d < nd) ? (T)load_as<TIN>(y, d) : (T)0;
    }
}

// ---------------------------------------------------------- Joseph A -------
template <typename TI, typename TO>
__global__ __launch_bounds__(256) void joseph2d_fwd_k(const TI *__restrict__ xp, const TI *__restrict__ xq,
                                                      VecRef yr,
                                                      const AngleTab<typename acc_of<TI>::type> *__restrict__ tab,
                                                      int nx, int ny, int nd, typename acc_of<TI>::type ds,
                                                      typename acc_of<TI>::type cd, int na, int nbx,
                                                      uint32_t nxcc, int s0, const int *kdev,
                                                      const int *active) {
    typedef typename acc_of<TI>::type T;
    // work order: (slice, angle, bin block), bin blocks fastest
    const uint32_t w = xcd_remap(blockIdx.x, gridDim.x, nxcc);
    const uint32_t wa = w / (uint32_t)nbx;
    const int a = (int)(wa % (uint32_t)na);
    const int s = s0 + (int)(wa / (uint32_t)na);
    if (active && !active[s]) return;
    // lanes past the last bin (d >= nd) only take part in the wave's row
    // range below; they store nothing
    const int d = (int)(w % (uint32_t)nbx) * 256 + threadIdx.x;
    const bool live = d < nd;
    const int k = kdev ? *kdev : 0;
    const AngleTab<T> t = tab[a];
    // march over the rows of the padded image (row march) or of its padded
    // transpose (column march); R rows of C pixels, stride C + 4
    const TI *P;
    int R, C;
    if (t.rowmarch) {
        P = xp + (int64_t)s * ny * (nx + 2 * PAD);
        R = ny;
        C = nx;
    } else {
        P = xq + (int64_t)s * nx * (ny + 2 * PAD);
        R = nx;
        C = ny;
    }
    const uint32_t L = (uint32_t)(C + 2 * PAD);
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
    if (!live) {
        r0 = R;
        r1 = -1;
    }
    // The whole wave steps through the union of its lanes' row ranges in
    // lockstep, so that one load instruction reads one image row (a few
    // cache lines) instead of a different row per lane.  In a row outside a
    // lane's own range its taps fall into the zero pads and add exactly 0.
    int rlo = r0, rhi = r1;
    for (int o = 32; o > 0; o >>= 1) {
        rlo = min(rlo, __shfl_xor(rlo, o));
        rhi = max(rhi, __shfl_xor(rhi, o));
    }
    rlo = __builtin_amdgcn_readfirstlane(rlo);
    rhi = __builtin_amdgcn_readfirstlane(rhi);
    const int nsteps = rhi - rlo + 1;   // <= 0 when no ray of the wave meets the image
    // Step in row r: u = u0 - r*slope, taps floor(u) and floor(u)+1, weight
    // u - floor(u).  Clamping floor(u) to [-2, C] keeps the pair inside the
    // padded row (columns jc+2, jc+3) and reads zeros wherever a tap is
    // outside the image.  Four steps per pass, all loads issued first.
    T acc0 = 0, acc1 = 0;
    int r = rlo;
    for (int i = 0; i + 4 <= nsteps; i += 4, r += 4) {
        const TI *Pr = P + (int64_t)r * L;   // row r, the same for the whole wave
        T v0[4], v1[4], f[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const T u = fma(-(T)(r + q), t.slope, u0);
            const T jf = floor(u);
            f[q] = u - jf;
            const TI *p = at_byte(Pr + q * L, (uint32_t)((int)clampf(jf, (T)-2, (T)C) + PAD) * (uint32_t)sizeof(TI));
            v0[q] = (T)p[0];
            v1[q] = (T)p[1];
        }
        acc0 += fma(f[0], v1[0] - v0[0], v0[0]);
        acc1 += fma(f[1], v1[1] - v0[1], v0[1]);
        acc0 += fma(f[2], v1[2] - v0[2], v0[2]);
        acc1 += fma(f[3], v1[3] - v0[3], v0[3]);
    }
    for (; r <= rhi; ++r) {   // the last nsteps mod 4 rows
        const T u = fma(-(T)r, t.slope, u0);
        const T jf = floor(u);
        const T f = u - jf;
        const TI *p = at_byte(P + (int64_t)r * L, (uint32_t)((int)clampf(jf, (T)-2, (T)C) + PAD) * (uint32_t)sizeof(TI));
        const T a0 = (T)p[0];
        const T a1 = (T)p[1];
        acc0 += fma(f, a1 - a0, a0);
    }
    if (!live) return;
    const T acc = acc0 + acc1;
    store_as<TO>(vec_ptr<TO>(yr, s, k), (int64_t)a * nd + d, acc * t.w);
}

// ------------------------------------------------------- pixel-driven B -----
// x[i][j] = wb * sum_a lerp(row a of the sinogram at X cos + Y sin), read from
// the padded sinogram yp (accumulation type T).
template <typename TI>
__global__ __launch_bounds__(256) void pixbp2d_k(const typename acc_of<TI>::type *__restrict__ yp, VecRef xr,
                                                 const AngleTab<typename acc_of<TI>::type> *__restrict__ tab,
                                                 int nx, int ny, int na, int nd, typename acc_of<TI>::type cd,
                                                 typename acc_of<TI>::type wb, int ntx, int nty, uint32_t nxcc,
                                                 int s0, const int *kdev, const int *active) {
    typedef typename acc_of<TI>::type T;
    // work order: (slice, tile row, tile column), 16 x 16 pixel tiles
    const uint32_t w = xcd_remap(blockIdx.x, gridDim.x, nxcc);
    const uint32_t wt = w / (uint32_t)ntx;
    const int ty = (int)(wt % (uint32_t)nty);
    const int s = s0 + (int)(wt / (uint32_t)nty);
    if (active && !active[s]) return;
    const int k = kdev ? *kdev : 0;
    const int j = (int)(w % (uint32_t)ntx) * 16 + (threadIdx.x & 15);
    const int i = ty * 16 + (threadIdx.x >> 4);
    const T X = (T)j - (T)0.5 * (T)(nx - 1);
    const T Y = (T)i - (T)0.5 * (T)(ny - 1);
    const uint32_t ld = (uint32_t)(nd + 2 * PAD);
    const T *Y0 = yp + (int64_t)s * na * ld;
    // bin coordinate t = X cos/ds + Y sin/ds + cd, taps floor(t), floor(t)+1,
    // clamped into the padded row as in A; four angles per pass
    T acc0 = 0, acc1 = 0, acc2 = 0, acc3 = 0;
    int a = 0;
    for (; a + 4 <= na; a += 4) {
        T v0[4], v1[4], f[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const T tt = fma(X, tab[a + q].cb, fma(Y, tab[a + q].sb, cd));
            const T df = floor(tt);
            f[q] = tt - df;
            const uint32_t e = (uint32_t)(a + q) * ld + (uint32_t)((int)clampf(df, (T)-2, (T)nd) + PAD);
            const T *p = at_byte(Y0, e * (uint32_t)sizeof(T));
            v0[q] = p[0];
            v1[q] = p[1];
        }
        acc0 += fma(f[0], v1[0] - v0[0], v0[0]);
        acc1 += fma(f[1], v1[1] - v0[1], v0[1]);
        acc2 += fma(f[2], v1[2] - v0[2], v0[2]);
        acc3 += fma(f[3], v1[3] - v0[3], v0[3]);
    }
    for (; a < na; ++a) {
        const T tt = fma(X, tab[a].cb, fma(Y, tab[a].sb, cd));
        const T df = floor(tt);
        const T f = tt - df;
        const uint32_t e = (uint32_t)a * ld + (uint32_t)((int)clampf(df, (T)-2, (T)nd) + PAD);
        const T *p = at_byte(Y0, e * (uint32_t)sizeof(T));
        const T a0 = p[0];
        const T a1 = p[1];
        acc0 += fma(f, a1 - a0, a0);
    }
    const T acc = ((acc0 + acc1) + (acc2 + acc3)) * wb;
    if (i < ny && j < nx) vec_ptr<TI>(xr, s, k)[(int64_t)i * nx + j] = (TI)acc;
}

// ------------------------------------------------------------ exact A^T ----
// Gather of the rays whose Joseph interpolation hat covers the pixel: weight
// hat((s_d - p)/c)/|c|, p = X cos + Y sin, c the dominant direction cosine.
template <typename TIN, typename TI>
__global__ __launch_bounds__(256) void josephT2d_k(VecRef yr, VecRef xr,
                                                   const AngleTab<typename acc_of<TI>::type> *__restrict__ tab,
                                                   int nx, int ny, int na, int nd, typename acc_of<TI>::type ds,
                                                   typename acc_of<TI>::type cd, int nmax, int ntx, int nty,
                                                   uint32_t nxcc, int s0, const int *kdev, const int *active) {
    typedef typename acc_of<TI>::type T;
    const uint32_t w = xcd_remap(blockIdx.x, gridDim.x, nxcc);
    const uint32_t wt = w / (uint32_t)ntx;
    const int ty = (int)(wt % (uint32_t)nty);
    const int s = s0 + (int)(wt / (uint32_t)nty);
    if (active && !active[s]) return;
    const int k = kdev ? *kdev : 0;
    const int j = (int)(w % (uint32_t)ntx) * 16 + (threadIdx.x & 15);
    const int i = ty * 16 + (threadIdx.x >> 4);
    const T X = (T)j - (T)0.5 * (T)(nx - 1);
    const T Y = (T)i - (T)0.5 * (T)(ny - 1);
    const TIN *y = vec_ptr<const TIN>(yr, s, k);
    T acc = 0;
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
    if (i < ny && j < nx) vec_ptr<TI>(xr, s, k)[(int64_t)i * nx + j] = (TI)acc;
}

// ------------------------------------------------------------ host side ----
static size_t acc_size(const abba_op *op) { return op->img_dtype == ABBA_F64 ? 8 : 4; }

size_t par2d_scratch_bytes(const abba_op *op, int batch) {
    const int64_t nx = op->g.nx, ny = op->g.ny, na = op->g.n_angles, nd = op->g.det_u;
    const int64_t img = ny * (nx + 2 * PAD) + nx * (ny + 2 * PAD);
    const int64_t sino = na * (nd + 2 * PAD);
    return (size_t)batch * (size_t)std::max(img, sino) * acc_size(op);
}

// A padded slice must be addressable with 32-bit byte offsets.
static bool offsets_fit(const abba_op *op) {
    const uint64_t nx = op->g.nx, ny = op->g.ny, na = op->g.n_angles, nd = op->g.det_u;
    const uint64_t lim = 1ull << 31;
    return ny * (nx + 2 * PAD) * acc_size(op) < lim && nx * (ny + 2 * PAD) * acc_size(op) < lim &&
           na * (nd + 2 * PAD) * acc_size(op) < lim;
}

template <typename TI, typename TO>
static int fwd_launch(const abba_op *op, VecRef x, VecRef y, int batch, void *scratch, const Launch &L) {
    typedef typename acc_of<TI>::type T;
    const int nx = op->g.nx, ny = op->g.ny, na = op->g.n_angles, nd = op->g.det_u;
    TI *xp = (TI *)scratch;
    TI *xq = xp + (int64_t)batch * ny * (nx + 2 * PAD);
    for (int s0 = 0; s0 < batch; s0 += MAX_GRID_YZ) {
        const int nb = std::min(MAX_GRID_YZ, batch - s0);
        dim3 tg((nx + 31) / 32, (ny + 31) / 32, nb);
        hipLaunchKernelGGL(pad_image_k<TI>, tg, dim3(256), 0, L.stream, x, xp, xq, nx, ny, s0, L.kdev, L.active);
        ABBA_LAUNCHED("pad_image_k");
    }
    const int nbx = (nd + 255) / 256;
    const uint64_t per_slice = (uint64_t)nbx * na;
    const int chunk = (int)std::min<uint64_t>((uint64_t)batch, MAX_GROUPS / per_slice);
    for (int s0 = 0; s0 < batch; s0 += chunk) {
        const int nb = std::min(chunk, batch - s0);
        hipLaunchKernelGGL((joseph2d_fwd_k<TI, TO>), dim3((uint32_t)(per_slice * nb)), dim3(256), 0, L.stream,
                           (const TI *)xp, (const TI *)xq, y, (const AngleTab<T> *)op->tab, nx, ny, nd,
                           (T)op->g.det_pitch_u, (T)(0.5 * (nd - 1)), na, nbx, (uint32_t)op->nxcc, s0, L.kdev,
                           L.active);
        ABBA_LAUNCHED("joseph2d_fwd_k");
    }
    return ABBA_OK;
}

int par2d_forward(const abba_op *op, VecRef x, VecRef y, int y_dtype, int batch, void *scratch, const Launch &L) {
    if (batch <= 0) return ABBA_OK;
    if (!offsets_fit(op) || (uint64_t)((op->g.det_u + 255) / 256) * op->g.n_angles > MAX_GROUPS)
        return ABBA_ERR_UNSUPPORTED;
    if (op->img_dtype == ABBA_F64) {
        if (y_dtype != ABBA_F64) return ABBA_ERR_DTYPE;
        return fwd_launch<double, double>(op, x, y, batch, scratch, L);
    }
    if (y_dtype == ABBA_F32) return fwd_launch<float, float>(op, x, y, batch, scratch, L);
    if (y_dtype == ABBA_BF16) return fwd_launch<float, bf16>(op, x, y, batch, scratch, L);
    return ABBA_ERR_DTYPE;
}

template <typename TIN, typename TI>
static int back_launch(const abba_op *op, VecRef y, VecRef x, int batch, void *scratch, const Launch &L) {
    typedef typename acc_of<TI>::type T;
    const int nx = op->g.nx, ny = op->g.ny, na = op->g.n_angles, nd = op->g.det_u;
    const double ds = op->g.det_pitch_u;
    const int ntx = (nx + 15) / 16, nty = (ny + 15) / 16;
    const uint64_t per_slice = (uint64_t)ntx * nty;
    const int chunk = (int)std::min<uint64_t>((uint64_t)batch, MAX_GROUPS / per_slice);
    if (op->kind == ABBA_OP_JOSEPH_T) {
        const int nmax = (int)ceil(2.0 / ds) + 2;
        for (int s0 = 0; s0 < batch; s0 += chunk) {
            const int nb = std::min(chunk, batch - s0);
            hipLaunchKernelGGL((josephT2d_k<TIN, TI>), dim3((uint32_t)(per_slice * nb)), dim3(256), 0, L.stream,
                               y, x, (const AngleTab<T> *)op->tab, nx, ny, na, nd, (T)ds, (T)(0.5 * (nd - 1)),
                               nmax, ntx, nty, (uint32_t)op->nxcc, s0, L.kdev, L.active);
            ABBA_LAUNCHED("josephT2d_k");
        }
        return ABBA_OK;
    }
    T *yp = (T *)scratch;
    for (int s0 = 0; s0 < batch; s0 += MAX_GRID_YZ) {
        const int nb = std::min(MAX_GRID_YZ, batch - s0);
        hipLaunchKernelGGL((pad_sino_k<TIN, T>), dim3(na, nb), dim3(256), 0, L.stream, y, yp, na, nd, s0, L.kdev,
                           L.active);
        ABBA_LAUNCHED("pad_sino_k");
    }
    for (int s0 = 0; s0 < batch; s0 += chunk) {
        const int nb = std::min(chunk, batch - s0);
        hipLaunchKernelGGL((pixbp2d_k<TI>), dim3((uint32_t)(per_slice * nb)), dim3(256), 0, L.stream,
                           (const T *)yp, x, (const AngleTab<T> *)op->tab, nx, ny, na, nd, (T)(0.5 * (nd - 1)),
                           (T)(1.0 / ds), ntx, nty, (uint32_t)op->nxcc, s0, L.kdev, L.active);
        ABBA_LAUNCHED("pixbp2d_k");
    }
    return ABBA_OK;
}

int par2d_back(const abba_op *op, VecRef y, int y_dtype, VecRef x, int batch, void *scratch, const Launch &L) {
    if (batch <= 0) return ABBA_OK;
    if (!offsets_fit(op) || (uint64_t)((op->g.nx + 15) / 16) * ((op->g.ny + 15) / 16) > MAX_GROUPS)
        return ABBA_ERR_UNSUPPORTED;
    if (op->img_dtype == ABBA_F64) {
        if (y_dtype != ABBA_F64) return ABBA_ERR_DTYPE;
        return back_launch<double, double>(op, y, x, batch, scratch, L);
    }
    if (y_dtype == ABBA_F32) return back_launch<float, float>(op, y, x, batch, scratch, L);
    if (y_dtype == ABBA_BF16) return back_launch<bf16, float>(op, y, x, batch, scratch, L);
    return ABBA_ERR_DTYPE;
}

}  // namespace abba
