// 2D parallel-beam operators for gfx950 (wave64).
//
//   A   Joseph's ray-driven projector (the forward model of Sec. 1, eq. (1)).
//   A^T the exact transpose of A, as a per-pixel gather (matched pair, Sec. 3).
//   B   pixel-driven backprojector with linear interpolation (the unmatched
//       B != A^T of eqs. (4)-(5)).
//
// Layout: one thread per ray (A) or per pixel (A^T, B).  Lanes of a wave run
// along detector bins (A), over two 32-pixel rows of a tile (B) or four
// 16-pixel rows (A^T), so consecutive lanes touch neighbouring memory.
//
// A first copies the image into scratch with PAD = 16 zeros on each side of
// every row, row-major and transposed (rays that march over image columns
// walk rows of the transposed copy).  Rows are taken in bands of 8; one clamp
// of a ray's position per band keeps all its taps in the band inside the
// padded rows, whose values are exactly those of the zero-extended rows: no
// per-tap masks, clamps or branches in the inner loop.  The batched kernel
// stages each band in LDS as aligned pairs (x[c], x[c+1] - x[c]), so a step
// is one 8-byte (FP64: 16-byte) LDS read.  B
// stages, per angle, the window of sinogram bins a pixel tile projects onto
// in LDS (zeros outside the detector), with every tap inside the window by
// construction, so it needs neither scratch nor a clamp.
//
// All launches are 1D; workgroups are renumbered so that each XCD (own L2)
// walks a contiguous range of slices (see xcd_remap).  Nothing uses atomics,
// so results are deterministic.
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>

#include "ops.h"

namespace abba {

constexpr int PAD = JPAD;   // zeros on each side of a padded row
constexpr int RPAD = 16;  // padded copies have a multiple of RPAD rows (extra rows are zero)

__host__ __device__ constexpr int round_rows(int r) { return (r + RPAD - 1) / RPAD * RPAD; }

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

// t - floor(t) in one instruction.
template <typename T>
__device__ __forceinline__ T fract_of(T t);
template <>
__device__ __forceinline__ float fract_of<float>(float t) { return __builtin_amdgcn_fractf(t); }
template <>
__device__ __forceinline__ double fract_of<double>(double t) { return __builtin_amdgcn_fract(t); }

// ------------------------------------------------------ padded copies -----
// Image -> xp [ny][nx + 2 PAD] (row-major) and xq [nx][ny + 2 PAD]
// (transposed), each row with PAD zeros on both sides.  32 x 32 tiles through
// LDS.
template <typename T>
__global__ __launch_bounds__(256) void pad_image_k(VecRef xr, T *__restrict__ xp, T *__restrict__ xq, int nx,
                                                   int ny, int s0, const int *kdev, const int *active) {
    const int s = s0 + blockIdx.z;
    if (active && !active[s]) return;
    const int k = kdev ? *kdev : 0;
    const T *x = vec_ptr<const T>(xr, s, k);
    const int lp = nx + 2 * PAD, lq = ny + 2 * PAD;
    T *op = xp + (int64_t)s * round_rows(ny) * lp;
    T *oq = xq + (int64_t)s * round_rows(nx) * lq;
    // the zero rows that round both copies up to a multiple of RPAD rows
    if (blockIdx.x == 0 && blockIdx.y == 0) {
        for (int e = threadIdx.x; e < (round_rows(ny) - ny) * lp; e += 256) op[(int64_t)ny * lp + e] = (T)0;
        for (int e = threadIdx.x; e < (round_rows(nx) - nx) * lq; e += 256) oq[(int64_t)nx * lq + e] = (T)0;
    }
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
    // the pads of rows i0..i0+31 of xp: columns [0, PAD) and [nx + PAD, nx + 2 PAD)
    if (blockIdx.x == 0) {
        for (int e = threadIdx.x; e < 32 * 2 * PAD; e += 256) {
            const int i = i0 + e / (2 * PAD), c = e % (2 * PAD);
            if (i < ny) op[(int64_t)i * lp + (c < PAD ? c : nx + c)] = (T)0;
        }
    }
    __syncthreads();
#pragma unroll
    for (int r = ty; r < 32; r += 8) {
        const int j = j0 + r, i = i0 + tx;
        if (i < ny && j < nx) oq[(int64_t)j * lq + i + PAD] = tile[tx][r];
    }
    // the pads of rows j0..j0+31 of xq
    if (blockIdx.y == 0) {
        for (int e = threadIdx.x; e < 32 * 2 * PAD; e += 256) {
            const int j = j0 + e / (2 * PAD), c = e % (2 * PAD);
            if (j < nx) oq[(int64_t)j * lq + (c < PAD ? c : ny + c)] = (T)0;
        }
    }
}

// ---------------------------------------------------------- Joseph A -------
// Ray (a, d) of a march direction with R rows of C pixels (padded rows of
// L = C + 2 PAD entries): u(r) = u0 - r*slope is the interpolation coordinate
// in row r (image column units); |slope| <= 1 (the march runs along the
// dominant direction cosine).  y = w * sum_r lerp(row r at
// u(r)).  The rows are taken in bands of H; a band contributes the sum over
// its rows, accumulated at even and odd rows separately.  Both kernels below
// compute exactly this with the same operations in the same order, so their
// results are bitwise identical; they differ only in where the taps come
// from (global memory or a band staged in LDS).
template <typename T>
struct JBand {
    static constexpr int H = 8;
};
static_assert(RPAD % 16 == 0 && RPAD % 8 == 0, "bands must tile the padded rows");
static_assert(PAD >= 2 * JBand<float>::H && PAD >= 2 * JBand<double>::H, "a band's taps must stay in its pads");

// Rows whose crossing lies in (-1, C), widened by one row on each side.  Both
// ends are clamped to [-2, R+1] before the conversion to int: for a ray that
// misses the image at a near-zero slope (the column march at exactly 90
// degrees has slope cos/sin ~ 6e-17) the quotients are ~1e17 and would
// otherwise saturate the conversion.  r0 ends in [0, R], r1 in [-1, R-1].
template <typename T>
__device__ __forceinline__ void ray_rows(T uc, T slope, int R, int C, int &r0, int &r1) {
    r0 = 0;
    r1 = R - 1;
    if (slope != (T)0) {
        const T ra = (uc + (T)1) / slope, rb = (uc - (T)C) / slope;
        const T lo = fmin(fmax(fmin(ra, rb), (T)-2), (T)(R + 1));
        const T hi = fmin(fmax(fmax(ra, rb), (T)-2), (T)(R + 1));
        r0 = max(0, (int)floor(lo) - 1);
        r1 = min(R - 1, (int)ceil(hi) + 1);
    } else if (!(uc > (T)-1 && uc < (T)C)) {
        r1 = -1;
    }
}

// Union of the row ranges of the 64 rays of a wave (the same in all lanes).
__device__ __forceinline__ void wave_union(int &r0, int &r1) {
    for (int o = 32; o > 0; o >>= 1) {
        r0 = min(r0, __shfl_xor(r0, o));
        r1 = max(r1, __shfl_xor(r1, o));
    }
}

// floor(x) as an int; FP32 has a single instruction for it.
template <typename T>
__device__ __forceinline__ int floor_int(T x);
template <>
__device__ __forceinline__ int floor_int<float>(float x) {
    int r;
    asm("v_cvt_flr_i32_f32 %0, %1" : "=v"(r) : "v"(x));
    return r;
}
template <>
__device__ __forceinline__ int floor_int<double>(double x) { return (int)floor(x); }

// The taps of entry c of padded row q of a band as (x[c], x[c+1] - x[c]):
// read from the padded image (RowTaps) or from pairs staged in LDS with the
// difference already formed by the same subtraction (PairTaps).
template <typename T>
struct pair_of;
template <>
struct pair_of<float> {
    typedef float2 type;
};
template <>
struct pair_of<double> {
    typedef double2 type;
};

template <typename T>
struct RowTaps {
    const T *rows;
    int L;
    __device__ __forceinline__ void get(int q, int c, T &x0, T &dx) const {
        const T *e = at_byte(rows + q * L, (uint32_t)c * (uint32_t)sizeof(T));
        x0 = e[0];
        dx = e[1] - e[0];
    }
};

template <typename T>
struct PairTaps {
    const typename pair_of<T>::type *rows;
    int L;
    __device__ __forceinline__ void get(int q, int c, T &x0, T &dx) const {
        const typename pair_of<T>::type e =
            *at_byte(rows + q * L, (uint32_t)c * (uint32_t)sizeof(typename pair_of<T>::type));
        x0 = e.x;
        dx = e.y;
    }
};

// Contribution of a band (padded rows of L = C + 2 PAD entries) for a ray
// with image coordinate ub = u(b0) in the band's first row; image column c
// is entry c + PAD of a padded row.  ub is clamped
// once to [H-1-PAD, C+PAD-H-1]: with |slope| <= 1 every u(b0+q), q < H, then
// lies in [-PAD, C+PAD-2], so both taps are inside the padded row.  The clamp
// moves ub only when the ray passes the band entirely outside the image
// (ub < H-1-PAD puts every u below 2H-2-PAD <= -2, ub > C+PAD-H-1 every u
// above C+PAD-2H >= C), and then the clamped taps are pad zeros too: the sum
// is exactly that of the zero-extended rows.
template <typename T, int H, typename Taps>
__device__ __forceinline__ T band_sum(const Taps &tp, T ub, T slope) {
    ub = clampf(ub, (T)(H - 1 - PAD), (T)(tp.L - PAD - H - 1));
    T f[H], x0[H], dx[H], a[2];
#pragma unroll
    for (int q = 0; q < H; ++q) {   // all taps of the band first
        const T u = fma(-(T)q, slope, ub);
        f[q] = fract_of(u);
        tp.get(q, floor_int(u) + PAD, x0[q], dx[q]);
    }
    __builtin_amdgcn_sched_barrier(0);   // keep the H loads in flight together
#pragma unroll
    for (int q = 0; q < H; ++q) {
        const T v = fma(f[q], dx[q], x0[q]);
        a[q & 1] = q < 2 ? v : a[q & 1] + v;   // even and odd rows
    }
    return a[0] + a[1];
}

// Gather version: one thread per ray, a wave = 64 consecutive bins of one
// angle, the wave walks the bands that meet the union of its rays' rows.
template <typename TI, typename TO>
__global__ __launch_bounds__(256) void joseph2d_fwd_k(const TI *__restrict__ xp, const TI *__restrict__ xq,
                                                      VecRef yr,
                                                      const AngleTab<typename acc_of<TI>::type> *__restrict__ tab,
                                                      int nx, int ny, int nd, typename acc_of<TI>::type ds,
                                                      typename acc_of<TI>::type cd, int na, int nbx,
                                                      uint32_t nxcc, int s0, const int *kdev,
                                                      const int *active) {
    typedef typename acc_of<TI>::type T;
    static_assert(sizeof(TI) == sizeof(T), "images are stored in the accumulation type");
    constexpr int H = JBand<T>::H;
    // work order: (slice, angle, bin block), bin blocks fastest
    const uint32_t w = xcd_remap(blockIdx.x, gridDim.x, nxcc);
    const uint32_t wa = w / (uint32_t)nbx;
    const int a = (int)(wa % (uint32_t)na);
    const int s = s0 + (int)(wa / (uint32_t)na);
    if (active && !active[s]) return;
    // lanes past the last bin only take part in the wave's row range
    const int d = (int)(w % (uint32_t)nbx) * 256 + threadIdx.x;
    const int k = kdev ? *kdev : 0;
    const AngleTab<T> t = tab[a];
    const T *P;
    int R, C;
    if (t.rowmarch) {
        P = (const T *)xp + (int64_t)s * round_rows(ny) * (nx + 2 * PAD);
        R = ny;
        C = nx;
    } else {
        P = (const T *)xq + (int64_t)s * round_rows(nx) * (ny + 2 * PAD);
        R = nx;
        C = ny;
    }
    const int L = C + 2 * PAD;
    const T sd = ((T)d - cd) * ds;
    const T u0 = fma(sd, t.inv_c, t.off);
    int r0, r1;
    ray_rows(u0, t.slope, R, C, r0, r1);
    if (d >= nd) {
        r0 = R;
        r1 = -1;
    }
    wave_union(r0, r1);
    const int rlo = __builtin_amdgcn_readfirstlane(r0), rhi = __builtin_amdgcn_readfirstlane(r1);
    T acc = 0;
    for (int b0 = rlo / H * H; b0 <= rhi; b0 += H)
        acc += band_sum<T, H>(RowTaps<T>{P + (int64_t)b0 * L, L}, fma(-(T)b0, t.slope, u0), t.slope);
    if (d < nd) store_as<TO>(vec_ptr<TO>(yr, s, k), (int64_t)a * nd + d, acc * t.w);
}

// LDS version: a workgroup takes one slice, JOSEPH_GA angles of one march
// direction and 256*JB bins (JB rays per thread and angle, a launch choice)
// and streams the padded image through LDS band by band; each ray keeps its
// sum in a register.  A wave skips a (ray slot, band) pair exactly when the
// gather version's wave would not visit that band.
constexpr int JB_DEFAULT = 3;

template <typename TI, typename TO, int JB>
__global__ __launch_bounds__(256) void joseph2d_lds_k(const TI *__restrict__ xp, const TI *__restrict__ xq,
                                                      VecRef yr,
                                                      const AngleTab<typename acc_of<TI>::type> *__restrict__ tab,
                                                      const int *__restrict__ agrp, int ngroups, int nbc, int nx,
                                                      int ny, int nd, typename acc_of<TI>::type ds,
                                                      typename acc_of<TI>::type cd, uint32_t nxcc, int s0,
                                                      const int *kdev, const int *active) {
    typedef typename acc_of<TI>::type T;
    static_assert(sizeof(TI) == sizeof(T), "images are stored in the accumulation type");
    constexpr int H = JBand<T>::H;
    constexpr int GA = JOSEPH_GA;
    typedef typename pair_of<T>::type T2;
    extern __shared__ __align__(16) unsigned char smem[];
    T2 *band = reinterpret_cast<T2 *>(smem);   // [H][L] pairs (x[c], x[c+1] - x[c])
    // work order: (slice, angle group, bin chunk of 256*JB)
    const uint32_t w = xcd_remap(blockIdx.x, gridDim.x, nxcc);
    const int bc = (int)(w % (uint32_t)nbc);
    const uint32_t w2 = w / (uint32_t)nbc;
    const int gi = (int)(w2 % (uint32_t)ngroups);
    const int s = s0 + (int)(w2 / (uint32_t)ngroups);
    if (active && !active[s]) return;
    const int k = kdev ? *kdev : 0;
    const int g_first = agrp[4 * gi], g_count = agrp[4 * gi + 1], rowmarch = agrp[4 * gi + 2];
    const int *order = agrp + 4 * ngroups;
    const T *P;
    int R, C;
    if (rowmarch) {
        P = (const T *)xp + (int64_t)s * round_rows(ny) * (nx + 2 * PAD);
        R = ny;
        C = nx;
    } else {
        P = (const T *)xq + (int64_t)s * round_rows(nx) * (ny + 2 * PAD);
        R = nx;
        C = ny;
    }
    const int L = C + 2 * PAD;
    T u0[GA][JB], acc[GA][JB], slope[GA];
    uint32_t rng[GA][JB];   // wave union of rows: first | (last + 1) << 16
#pragma unroll
    for (int ai = 0; ai < GA; ++ai) {
        const int a = order[g_first + min(ai, g_count - 1)];
        const AngleTab<T> t = tab[a];
        slope[ai] = t.slope;
#pragma unroll
        for (int j = 0; j < JB; ++j) {
            const int d = bc * (256 * JB) + j * 256 + (int)threadIdx.x;
            const T sd = ((T)d - cd) * ds;
            u0[ai][j] = fma(sd, t.inv_c, t.off);
            acc[ai][j] = 0;
            int r0, r1;
            ray_rows(u0[ai][j], t.slope, R, C, r0, r1);
            if (ai >= g_count || d >= nd) {
                r0 = R;
                r1 = -1;
            }
            wave_union(r0, r1);
            rng[ai][j] = __builtin_amdgcn_readfirstlane((uint32_t)r0 | ((uint32_t)(r1 + 1) << 16));
        }
    }
    const int Rr = round_rows(R);
    const bool vec4 = (L % 4) == 0;
    for (int b0 = 0; b0 < Rr; b0 += H) {
        __syncthreads();   // the previous band is no longer read
        // the pair of the band's last entry (never read) takes x[c+1] = 0
        const T *src = P + (int64_t)b0 * L;
        const int n = H * L;
        if (vec4 && sizeof(T) == 4) {
            const float *s1 = reinterpret_cast<const float *>(src);
            const float4 *s4 = reinterpret_cast<const float4 *>(src);
            float4 *d4 = reinterpret_cast<float4 *>(band);
            for (int c = threadIdx.x; c < n / 4; c += 256) {
                const float4 v = s4[c];
                const float x4 = 4 * c + 4 < n ? s1[4 * c + 4] : 0.0f;
                d4[2 * c] = make_float4(v.x, v.y - v.x, v.y, v.z - v.y);
                d4[2 * c + 1] = make_float4(v.z, v.w - v.z, v.w, x4 - v.w);
            }
        } else {
            for (int c = threadIdx.x; c < n; c += 256) {
                const T x0 = src[c], x1 = c + 1 < n ? src[c + 1] : (T)0;
                band[c] = T2{x0, x1 - x0};
            }
        }
        __syncthreads();
#pragma unroll
        for (int ai = 0; ai < GA; ++ai) {
#pragma unroll
            for (int j = 0; j < JB; ++j) {
                const int lo = (int)(rng[ai][j] & 0xffffu), hi1 = (int)(rng[ai][j] >> 16);
                if (lo > b0 + H - 1 || hi1 <= b0) continue;   // the same in all lanes of the wave
                acc[ai][j] += band_sum<T, H>(PairTaps<T>{band, L}, fma(-(T)b0, slope[ai], u0[ai][j]), slope[ai]);
            }
        }
    }
#pragma unroll
    for (int ai = 0; ai < GA; ++ai) {
        if (ai >= g_count) break;
        const int a = order[g_first + ai];
        const T wt = tab[a].w;
        TO *yo = vec_ptr<TO>(yr, s, k) + (int64_t)a * nd;
#pragma unroll
        for (int j = 0; j < JB; ++j) {
            const int d = bc * (256 * JB) + j * 256 + (int)threadIdx.x;
            if (d < nd) store_as<TO>(yo, d, acc[ai][j] * wt);
        }
    }
}

// ------------------------------------------------------- pixel-driven B -----
// x[i][j] = wb * sum_a lerp(row a of the sinogram at t = X cos/ds + Y sin/ds + cd).
// The image is cut into tiles of 32 columns x 64 rows.  For a chunk of angles
// a workgroup stages in LDS, per angle, the window of detector bins its tile
// projects onto, as pairs (y[p], y[p+1] - y[p]) with zeros outside the
// detector; a pixel-angle pair is then one LDS read, lerp = v + f*dv.  The
// window of angle a starts at w0 = floor(t_min) - 1 (t_min over the tile's
// corners) and holds W entries, W >= (31 |cos| + 63 |sin|)/ds + 5 over all
// angles, so every tap of the tile lies inside it.  A workgroup takes the
// whole tile (RM = 8 rows per thread) or one half of it (RM = 4, two
// workgroups per tile, for batches too small to fill the device); both stage
// the tile's window and compute t relative to the tile's w0, so a pixel gets
// the same bits either way.
constexpr int BT = 32;    // tile width (columns)
constexpr int BTH = 64;   // tile height (rows)

// Window of B for one (tile, angle), from the operator's table (built once
// when the operator is created): its start w0 and cd - w0 in the
// accumulation type, the addend that makes t relative to the window.
template <typename T>
struct BpWin {
    T par;
    int w0;
};

template <typename TIN, typename TI, int RM>
__global__ __launch_bounds__(256) void pixbp2d_k(VecRef yr, VecRef xr,
                                                 const AngleTab<typename acc_of<TI>::type> *__restrict__ tab,
                                                 const BpWin<typename acc_of<TI>::type> *__restrict__ bpw,
                                                 int nx, int ny, int na, int nd, typename acc_of<TI>::type wb,
                                                 int W, int G, int ntx, int nty, uint32_t nxcc, int s0,
                                                 const int *kdev, const int *active) {
    typedef typename acc_of<TI>::type T;
    extern __shared__ __align__(16) unsigned char smem[];
    T *win = reinterpret_cast<T *>(smem);                                      // [G][W][2]
    int *w0s = reinterpret_cast<int *>(smem + (size_t)G * W * 2 * sizeof(T));   // [G]: w0
    static_assert(RM == 4 || RM == 8, "a workgroup takes a whole tile or one half");
    constexpr int NH = BTH / (8 * RM);   // workgroups per tile
    // work order: (slice, tile row, tile column, half)
    const uint32_t w0i = xcd_remap(blockIdx.x, gridDim.x, nxcc);
    const int half = NH > 1 ? (int)(w0i % (uint32_t)NH) : 0;
    const uint32_t w = w0i / (uint32_t)NH;
    const uint32_t wt = w / (uint32_t)ntx;
    const int ty = (int)(wt % (uint32_t)nty);
    const int tx = (int)(w % (uint32_t)ntx);
    const int s = s0 + (int)(wt / (uint32_t)nty);
    if (active && !active[s]) return;
    const int k = kdev ? *kdev : 0;
    const TIN *y = vec_ptr<const TIN>(yr, s, k);
    const T cx = (T)0.5 * (T)(nx - 1), cy = (T)0.5 * (T)(ny - 1);
    // this thread: column j, rows i0 + 8m (m < RM)
    const int j = tx * BT + (threadIdx.x & 31);
    const int i0 = ty * BTH + half * (8 * RM) + (threadIdx.x >> 5);
    const T X = (T)j - cx;
    T Ym[RM], acc[RM];
#pragma unroll
    for (int m = 0; m < RM; ++m) {
        Ym[m] = (T)(i0 + 8 * m) - cy;
        acc[m] = 0;
    }
    // this tile's windows; the per-angle values of the loop below are
    // wave-uniform loads (scalar memory), not LDS reads
    const BpWin<T> *bw = bpw + ((int64_t)ty * ntx + tx) * na;
    const float winv = 1.0f / (float)W;
    for (int a0 = 0; a0 < na; a0 += G) {
        const int g = min(G, na - a0);
        __syncthreads();   // the previous chunk is no longer read
        for (int al = threadIdx.x; al < g; al += 256) w0s[al] = bw[a0 + al].w0;
        __syncthreads();
        // the windows: entry e = al*W + c of the chunk, all threads over all
        // angles.  al = floor((e + 1/2) / W) in FP32 is exact: (e + 1/2)/W is
        // at least 1/(2W) from an integer and e < G*W <= 8192 (64 KB of LDS)
        // keeps the rounding error far below that.
        for (int e = threadIdx.x; e < g * W; e += 256) {
            const int al = (int)(((float)e + 0.5f) * winv);
            const int p = w0s[al] + (e - al * W);
            const TIN *row = y + (int64_t)(a0 + al) * nd;
            const T v = ((unsigned)p < (unsigned)nd) ? (T)load_as<TIN>(row, p) : (T)0;
            const T vn = ((unsigned)(p + 1) < (unsigned)nd) ? (T)load_as<TIN>(row, p + 1) : (T)0;
            win[2 * e] = v;
            win[2 * e + 1] = vn - v;
        }
        __syncthreads();
        for (int al = 0; al < g; ++al) {
            const T cb = tab[a0 + al].cb, sb = tab[a0 + al].sb;
            // t relative to the window start: t - w0 = fma(Y, sb, X cb + cd - w0)
            const T base = fma(X, cb, bw[a0 + al].par);
            const T *wrow = win + (size_t)al * W * 2;
#pragma unroll
            for (int m = 0; m < RM; ++m) {
                const T t = fma(Ym[m], sb, base);
                const T f = fract_of(t);
                // every pixel of the tile (overhang included) has
                // 1 <= t < 2 + (31 |cos| + 63 |sin|)/ds <= W - 3 up to rounding
                // of a few ulp, so (int) is floor and both taps lie in the
                // window
                const int idx = (int)t;
                const T v = wrow[2 * idx], dv = wrow[2 * idx + 1];
                acc[m] += fma(f, dv, v);
            }
        }
    }
    if (j < nx) {
        TI *xo = vec_ptr<TI>(xr, s, k);
#pragma unroll
        for (int m = 0; m < RM; ++m) {
            const int i = i0 + 8 * m;
            if (i < ny) xo[(int64_t)i * nx + j] = (TI)(acc[m] * wb);
        }
    }
}

// LDS window of the pixel-driven B: entries per angle and angles per chunk.
static void pixbp_window(const abba_op *op, int *W, int *G) {
    double m = 0;
    for (int a = 0; a < op->g.n_angles; ++a) {
        const double th = op->g.angles ? op->g.angles[a] : a * M_PI / op->g.n_angles;
        m = std::max(m, (BT - 1) * std::fabs(std::cos(th)) + (BTH - 1) * std::fabs(std::sin(th)));
    }
    *W = (int)std::ceil(m / op->g.det_pitch_u) + 5;
    const size_t per = (size_t)*W * 2 * (op->img_dtype == ABBA_F64 ? 8 : 4);
    *G = (int)std::max<size_t>(1, std::min<size_t>(32, 32768 / per));
}

// Most angles per chunk whose windows fit in 64 KB of LDS.
static int pixbp_max_g(const abba_op *op, int W) {
    const size_t per = (size_t)W * 2 * (op->img_dtype == ABBA_F64 ? 8 : 4) + 4;
    return (int)std::max<size_t>(1, 65536 / per);
}

// The window of every (tile, angle): w0 = floor(t_min) - 1 with t_min the
// smallest detector coordinate (in bins, centre cd) of the tile's corners,
// computed in FP64 from the FP32 (or FP64) cos/ds and sin/ds the kernel uses.
template <typename T>
static void pixbp_fill_table(const abba_op *op, BpWin<T> *out) {
    const abba_geometry &g = op->g;
    const int btx = (g.nx + BT - 1) / BT, bty = (g.ny + BTH - 1) / BTH, na = g.n_angles;
    const double ds = g.det_pitch_u, cx = 0.5 * (g.nx - 1), cy = 0.5 * (g.ny - 1), cd = 0.5 * (g.det_u - 1);
    for (int a = 0; a < na; ++a) {
        const double th = g.angles ? g.angles[a] : a * M_PI / na;
        const double cb = (double)(T)(std::cos(th) / ds), sb = (double)(T)(std::sin(th) / ds);
        for (int ty = 0; ty < bty; ++ty)
            for (int tx = 0; tx < btx; ++tx) {
                const double X0 = tx * BT - cx, X1 = X0 + (BT - 1), Y0 = ty * BTH - cy, Y1 = Y0 + (BTH - 1);
                const double tmin = cd + std::min(X0 * cb, X1 * cb) + std::min(Y0 * sb, Y1 * sb);
                const int w0 = (int)std::floor(tmin) - 1;
                BpWin<T> &e = out[((int64_t)ty * btx + tx) * na + a];
                e.par = (T)(cd - w0);
                e.w0 = w0;
            }
    }
}

int pixbp_build_table(abba_op *op) {
    if (op->g.kind != ABBA_GEOM_PAR2D) return ABBA_OK;
    const int btx = (op->g.nx + BT - 1) / BT, bty = (op->g.ny + BTH - 1) / BTH;
    const size_t n = (size_t)btx * bty * op->g.n_angles;
    std::vector<unsigned char> host;
    size_t bytes;
    if (op->img_dtype == ABBA_F64) {
        bytes = n * sizeof(BpWin<double>);
        host.resize(bytes);
        pixbp_fill_table(op, reinterpret_cast<BpWin<double> *>(host.data()));
    } else {
        bytes = n * sizeof(BpWin<float>);
        host.resize(bytes);
        pixbp_fill_table(op, reinterpret_cast<BpWin<float> *>(host.data()));
    }
    hipError_t e = hipMalloc(&op->bpw, bytes);
    if (e == hipSuccess) e = hipMemcpy(op->bpw, host.data(), bytes, hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(e, "backprojector window table upload");
    return ABBA_OK;
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
    if (op->kind != ABBA_OP_JOSEPH) return 0;   // only A reads a padded copy
    const int64_t nx = op->g.nx, ny = op->g.ny;
    return (size_t)batch * (size_t)(round_rows(ny) * (nx + 2 * PAD) + round_rows(nx) * (ny + 2 * PAD)) *
           acc_size(op);
}

// A padded slice must be addressable with 32-bit byte offsets.
static bool offsets_fit(const abba_op *op) {
    const uint64_t nx = op->g.nx, ny = op->g.ny;
    const uint64_t lim = 1ull << 31;
    return (uint64_t)round_rows(ny) * (nx + 2 * PAD) * acc_size(op) < lim &&
           (uint64_t)round_rows(nx) * (ny + 2 * PAD) * acc_size(op) < lim;
}

template <typename T>
static bool lds_fits(const abba_op *op) {
    const size_t band_bytes = (size_t)JBand<T>::H * (std::max(op->g.nx, op->g.ny) + 2 * PAD) * 2 * sizeof(T);
    return band_bytes <= 65536 && op->agrp && std::max(op->g.nx, op->g.ny) < 65535;
}

// Workgroups of one slice in the LDS version.
static uint64_t lds_groups(const abba_op *op, int jb) {
    return (uint64_t)op->ngroups * ((op->g.det_u + 256 * jb - 1) / (256 * jb));
}

template <typename TI, typename TO, int JB>
static int lds_launch(const abba_op *op, const TI *xp, const TI *xq, VecRef y, int batch, const Launch &L) {
    typedef typename acc_of<TI>::type T;
    const int nx = op->g.nx, ny = op->g.ny, nd = op->g.det_u;
    const size_t band_bytes = (size_t)JBand<T>::H * (std::max(nx, ny) + 2 * PAD) * 2 * sizeof(T);
    const int nbc = (nd + 256 * JB - 1) / (256 * JB);
    const uint64_t per = lds_groups(op, JB);
    const int ch = (int)std::min<uint64_t>((uint64_t)batch, MAX_GROUPS / per);
    for (int s0 = 0; s0 < batch; s0 += ch) {
        const int nb = std::min(ch, batch - s0);
        hipLaunchKernelGGL((joseph2d_lds_k<TI, TO, JB>), dim3((uint32_t)(per * nb)), dim3(256), band_bytes,
                           L.stream, xp, xq, y, (const AngleTab<T> *)op->tab, (const int *)op->agrp, op->ngroups,
                           nbc, nx, ny, nd, (T)op->g.det_pitch_u, (T)(0.5 * (nd - 1)), (uint32_t)op->nxcc, s0,
                           L.kdev, L.active);
        ABBA_LAUNCHED("joseph2d_lds_k");
    }
    return ABBA_OK;
}

template <typename TI, typename TO>
static int fwd_launch(const abba_op *op, VecRef x, VecRef y, int batch, void *scratch, const Launch &L) {
    typedef typename acc_of<TI>::type T;
    const int nx = op->g.nx, ny = op->g.ny, na = op->g.n_angles, nd = op->g.det_u;
    TI *xp = (TI *)scratch;
    TI *xq = xp + (int64_t)batch * round_rows(ny) * (nx + 2 * PAD);
    for (int s0 = 0; s0 < batch; s0 += MAX_GRID_YZ) {
        const int nb = std::min(MAX_GRID_YZ, batch - s0);
        dim3 tg((nx + 31) / 32, (ny + 31) / 32, nb);
        hipLaunchKernelGGL(pad_image_k<TI>, tg, dim3(256), 0, L.stream, x, xp, xq, nx, ny, s0, L.kdev, L.active);
        ABBA_LAUNCHED("pad_image_k");
    }
    // The LDS version needs a band of rows in 64 KB and enough workgroups to
    // fill the device (it has ~90x fewer than the gather version); both give
    // bitwise identical results, as do its bin-chunk widths.  A tuning entry
    // for this batch size overrides the rule; ABBA_JOSEPH_PATH=gather|lds
    // overrides both.
    const bool lds_ok = lds_fits<T>(op);
    int jb = JB_DEFAULT;
    bool use_lds = lds_ok && lds_groups(op, jb) * (uint64_t)batch >= 8ull * (uint64_t)op->ncu;
    if (const TuneEntry *t = tune_for(op, batch)) {
        if (t->a_path == 0 || t->a_path == 1) use_lds = t->a_path == 1 && lds_ok;
        if (t->a_jb >= 2 && t->a_jb <= 4) jb = t->a_jb;
    }
    const char *force = std::getenv("ABBA_JOSEPH_PATH");
    if (force && std::strcmp(force, "gather") == 0) use_lds = false;
    if (force && std::strcmp(force, "lds") == 0) use_lds = lds_ok;
    if (use_lds) {
        if (jb == 2) return lds_launch<TI, TO, 2>(op, xp, xq, y, batch, L);
        if (jb == 4) return lds_launch<TI, TO, 4>(op, xp, xq, y, batch, L);
        return lds_launch<TI, TO, 3>(op, xp, xq, y, batch, L);
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
static int back_launch(const abba_op *op, VecRef y, VecRef x, int batch, const Launch &L) {
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
    int W, G;
    pixbp_window(op, &W, &G);
    if (const TuneEntry *t = tune_for(op, batch))
        if (t->b_g > 0) G = std::min(t->b_g, pixbp_max_g(op, W));
    const size_t shmem = (size_t)G * (W * 2 * sizeof(T) + 4);
    if ((size_t)W * 2 * sizeof(T) > 32768) return ABBA_ERR_UNSUPPORTED;
    const int btx = (nx + BT - 1) / BT, bty = (ny + BTH - 1) / BTH;
    // half tiles where whole ones would leave CUs idle (fewer than four
    // workgroups per CU); the same bits either way
    const bool halves = (uint64_t)btx * bty * batch < 4ull * (uint64_t)op->ncu;
    const uint64_t tiles = (uint64_t)btx * bty * (halves ? 2 : 1);
    const int bchunk = (int)std::min<uint64_t>((uint64_t)batch, MAX_GROUPS / tiles);
    for (int s0 = 0; s0 < batch; s0 += bchunk) {
        const int nb = std::min(bchunk, batch - s0);
#define PIXBP(RM)                                                                                                  \
    hipLaunchKernelGGL((pixbp2d_k<TIN, TI, RM>), dim3((uint32_t)(tiles * nb)), dim3(256), shmem, L.stream, y, x,     \
                       (const AngleTab<T> *)op->tab, (const BpWin<T> *)op->bpw, nx, ny, na, nd, (T)(1.0 / ds), W, G, \
                       btx, bty, (uint32_t)op->nxcc, s0, L.kdev, L.active)
        if (halves) PIXBP(4);
        else PIXBP(8);
#undef PIXBP
        ABBA_LAUNCHED("pixbp2d_k");
    }
    return ABBA_OK;
}

int par2d_back(const abba_op *op, VecRef y, int y_dtype, VecRef x, int batch, void *scratch, const Launch &L) {
    (void)scratch;
    if (batch <= 0) return ABBA_OK;
    if ((uint64_t)((op->g.nx + 15) / 16) * ((op->g.ny + 15) / 16) > MAX_GROUPS) return ABBA_ERR_UNSUPPORTED;
    if (op->img_dtype == ABBA_F64) {
        if (y_dtype != ABBA_F64) return ABBA_ERR_DTYPE;
        return back_launch<double, double>(op, y, x, batch, L);
    }
    if (y_dtype == ABBA_F32) return back_launch<float, float>(op, y, x, batch, L);
    if (y_dtype == ABBA_BF16) return back_launch<bf16, float>(op, y, x, batch, L);
    return ABBA_ERR_DTYPE;
}

// Launch choices abba_autotune times for this operator (all give the same bits).
int par2d_tune_candidates(const abba_op *op, TuneEntry *out, int cap) {
    int n = 0;
    auto add = [&](TuneEntry e) {
        if (n < cap) out[n++] = e;
    };
    if (op->kind == ABBA_OP_JOSEPH) {
        add(TuneEntry{0, 0, 0, 0, 0, 0});
        const bool fits = op->img_dtype == ABBA_F64 ? lds_fits<double>(op) : lds_fits<float>(op);
        if (fits)
            for (int jb = 2; jb <= 4; ++jb) add(TuneEntry{0, 1, jb, 0, 0, 0});
    } else if (op->kind == ABBA_OP_PIXEL) {
        int W, G;
        pixbp_window(op, &W, &G);
        const int gmax = pixbp_max_g(op, W);
        for (int g : {8, 16, 32, 64, 128})
            if (g <= gmax) add(TuneEntry{0, 0, 0, g, 0, 0});
    }
    return n;
}

}  // namespace abba
