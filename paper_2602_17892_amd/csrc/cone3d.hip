// 3D circular cone-beam operators for gfx950 (the 3D extension of the
// forward model of Sec. 1, eq. (1), and of the unmatched B of eqs. (4)-(5)).
//
// Volume [nz][ny][nx], unit voxels centred at the origin; view v has source
// S_v, a flat detector with centre D_v and unit axes eu_v (columns) and ev_v
// (rows); pixel (r, c) sits at D_v + (c - (nu-1)/2) pu eu_v + (r - (nv-1)/2) pv ev_v.
//
// A  Joseph: the ray S -> pixel marches over the planes of its dominant axis;
//    in each plane the volume is interpolated bilinearly; the sum is weighted
//    by |d| / |d_major| (the ray length between two planes).
// B  voxel driven: the voxel centre is projected from S onto the detector
//    plane (magnification M = (D - S).n / (X - S).n), the view is
//    interpolated bilinearly there and weighted by (M/pu)(M/pv).
//
// The 2D fan beam with a flat detector runs the same kernels as the z = 0
// plane of this geometry (nz = nv = 1, pv = 1): the plane coordinate of every
// tap is exactly 0, so the bilinear interpolation is the linear one, and B
// takes the weight M/pu (one transverse dimension).
//
// Both read zero-padded copies of their input (two zeros on each side of the
// two interpolated axes), so a clamped position reads its taps without masks:
// for A one copy per dominant axis that occurs, permuted so that every plane
// is contiguous with its fast in-plane axis innermost; for B the sinogram.
// Ray set-up is FP64; the per-step arithmetic is in the accumulation type.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <type_traits>
#include <vector>

#include "ops.h"

namespace abba {

constexpr int CPAD = 2;   // zeros on each side of a padded axis

// Per-view constants of B in the accumulation type.
template <typename T>
struct ConeB {
    T n[3];     // detector normal
    T eup[3];   // eu / pu
    T evp[3];   // ev / pv
    T Sn, Su, Sv;
    T cu, cv;   // detector coordinate of the centre, plus the two leading pad entries
    T dist;
};

// ------------------------------------------------------------ host side ----
static void view_of(const abba_geometry &g, int v, ConeView &c) {
    const double b = g.angles ? g.angles[v] : 2.0 * M_PI * v / g.n_angles;
    const double cb = std::cos(b), sb = std::sin(b);
    const double S[3] = {g.sid * cb, g.sid * sb, 0.0};
    const double D[3] = {-(g.sdd - g.sid) * cb, -(g.sdd - g.sid) * sb, 0.0};
    const double eu[3] = {-sb, cb, 0.0}, ev[3] = {0.0, 0.0, 1.0};
    for (int t = 0; t < 3; ++t) {
        c.S[t] = S[t];
        c.D[t] = D[t];
        c.eu[t] = eu[t];
        c.ev[t] = ev[t];
    }
    c.n[0] = eu[1] * ev[2] - eu[2] * ev[1];
    c.n[1] = eu[2] * ev[0] - eu[0] * ev[2];
    c.n[2] = eu[0] * ev[1] - eu[1] * ev[0];
    double dn = 0, sn = 0, su = 0, sv = 0, cu = 0, cv = 0;
    for (int t = 0; t < 3; ++t) {
        dn += (D[t] - S[t]) * c.n[t];
        sn += S[t] * c.n[t];
        su += S[t] * eu[t];
        sv += S[t] * ev[t];
        cu += (S[t] - D[t]) * eu[t];
        cv += (S[t] - D[t]) * ev[t];
    }
    c.dist = dn;
    c.Sn = sn;
    c.Su = su / g.det_pitch_u;
    c.Sv = sv / g.det_pitch_v;
    c.cu = cu / g.det_pitch_u + 0.5 * (g.det_u - 1);
    c.cv = cv / g.det_pitch_v + 0.5 * (g.det_v - 1);
}

// Direction S -> pixel (ou, ov) of view V, evaluated without contraction so
// that host and device classify every ray the same way.
static __host__ __device__ inline void ray_dir(const ConeView &V, double ou, double ov, double *d) {
#pragma clang fp contract(off)
    for (int t = 0; t < 3; ++t) d[t] = V.D[t] + ou * V.eu[t] + ov * V.ev[t] - V.S[t];
}

// Dominant axis of the ray S -> P (ties as in the oracle: x, then y, then z).
static __host__ __device__ inline int major_of(double dx, double dy, double dz) {
    const double ax = fabs(dx), ay = fabs(dy), az = fabs(dz);
    if (ax >= ay && ax >= az) return 0;
    if (ay >= az) return 1;
    return 2;
}

int build_cone_tables(abba_op *op) {
    const abba_geometry &g = op->g;
    const int nv = g.n_angles;
    std::vector<ConeView> tab(nv);
    int axes = 0;
    for (int v = 0; v < nv; ++v) {
        view_of(g, v, tab[v]);
        const ConeView &c = tab[v];
        for (int r = 0; r < g.det_v && axes != 7; ++r)
            for (int col = 0; col < g.det_u; ++col) {
                const double ou = (col - 0.5 * (g.det_u - 1)) * g.det_pitch_u;
                const double ov = (r - 0.5 * (g.det_v - 1)) * g.det_pitch_v;
                double d[3];
                ray_dir(c, ou, ov, d);
                axes |= 1 << major_of(d[0], d[1], d[2]);
            }
    }
    op->cone_axes = axes;
    // B takes a voxel's magnification and detector column once per column of
    // voxels along z: the orbit lies in the plane z = 0 and the detector rows
    // run along z, so the detector normal and the column axis have no z part
    for (int v = 0; v < nv; ++v)
        if (tab[v].n[2] != 0.0 || tab[v].eu[2] != 0.0) {
            set_error("cone view %d: the detector normal or column axis leaves the orbit plane", v);
            return ABBA_ERR_UNSUPPORTED;
        }
    const size_t bytes_d = sizeof(ConeView) * nv;
    const size_t bytes_b = op->img_dtype == ABBA_F64 ? sizeof(ConeB<double>) * nv : sizeof(ConeB<float>) * nv;
    std::vector<unsigned char> host(bytes_d + bytes_b);
    std::memcpy(host.data(), tab.data(), bytes_d);
    for (int v = 0; v < nv; ++v) {
        const ConeView &c = tab[v];
        auto fill = [&](auto *b) {
            typedef typename std::remove_reference<decltype(b->Sn)>::type T;
            for (int t = 0; t < 3; ++t) {
                b->n[t] = (T)c.n[t];
                b->eup[t] = (T)(c.eu[t] / g.det_pitch_u);
                b->evp[t] = (T)(c.ev[t] / g.det_pitch_v);
            }
            b->Sn = (T)c.Sn;
            b->Su = (T)c.Su;
            b->Sv = (T)c.Sv;
            b->cu = (T)(c.cu + CPAD);
            b->cv = (T)(c.cv + CPAD);
            b->dist = (T)c.dist;
        };
        if (op->img_dtype == ABBA_F64) fill(reinterpret_cast<ConeB<double> *>(host.data() + bytes_d) + v);
        else fill(reinterpret_cast<ConeB<float> *>(host.data() + bytes_d) + v);
    }
    hipError_t e = hipMalloc(&op->tab, host.size());
    if (e == hipSuccess) e = hipMemcpy(op->tab, host.data(), host.size(), hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(e, "cone table upload");
    return ABBA_OK;
}

// Padded-copy sizes (elements per slice).
// The padded volume copies hold, at every (plane, p, q), the pair
// (x[plane][p][q], x[plane][p + 1][q]): A's four bilinear taps of a position
// are then the 16 contiguous bytes of two neighbouring pairs, one load.
struct ConeCopies {
    size_t vx, vy, vz;   // pairs over [nx][nz+4][ny+4], [ny][nz+4][nx+4], [nz][ny+4][nx+4] (elements, two
                         // per pair); 0 if the axis never leads
    size_t sino;         // pairs (y[v][u], y[v + 1][u]) over [views][nv+4][nu+4] (elements, two per pair)
};

static ConeCopies cone_copies(const abba_op *op) {
    const size_t nx = op->g.nx, ny = op->g.ny, nz = op->g.nz;
    ConeCopies c;
    c.vx = (op->cone_axes & 1) ? 2 * nx * (nz + 2 * CPAD) * (ny + 2 * CPAD) : 0;
    c.vy = (op->cone_axes & 2) ? 2 * ny * (nz + 2 * CPAD) * (nx + 2 * CPAD) : 0;
    c.vz = (op->cone_axes & 4) ? 2 * nz * (ny + 2 * CPAD) * (nx + 2 * CPAD) : 0;
    c.sino = (size_t)2 * op->g.n_angles * (op->g.det_v + 2 * CPAD) * (op->g.det_u + 2 * CPAD);
    return c;
}

size_t cone_scratch_bytes(const abba_op *op, int batch) {
    const ConeCopies c = cone_copies(op);
    const size_t es = op->img_dtype == ABBA_F64 ? 8 : 4;
    const size_t per = op->kind == ABBA_OP_JOSEPH ? c.vx + c.vy + c.vz : c.sino;
    return (size_t)batch * per * es;
}

// ------------------------------------------------------------- kernels ----
template <typename T>
__global__ __launch_bounds__(256) void cfill_k(T *__restrict__ p, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = (T)0;
}

// Volume -> the padded pair copies of the axes that lead some ray (zeroed
// before): each voxel is the first entry of its own pair and the second
// entry of the pair one row (p) before.  One workgroup per 32 x 32 (y, x)
// tile of one z slice of one volume (blockIdx.z = slice in the batch * nz + z).
template <typename T>
__global__ __launch_bounds__(256) void cone_pad_vol_k(VecRef xr, T *__restrict__ vx, T *__restrict__ vy,
                                                      T *__restrict__ vz, int nx, int ny, int nz, int s0,
                                                      int64_t sx, int64_t sy, int64_t szz, const int *kdev,
                                                      const int *active) {
    const int s = s0 + (int)(blockIdx.z / nz), z = (int)(blockIdx.z % nz);
    if (active && !active[s]) return;
    const int k = kdev ? *kdev : 0;
    const T *x = vec_ptr<const T>(xr, s, k) + (int64_t)z * ny * nx;
    __shared__ T tile[32][33];
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;   // 32 x 8
    const int j0 = blockIdx.x * 32, i0 = blockIdx.y * 32;
    const int Lx = nx + 2 * CPAD, Ly = ny + 2 * CPAD, Lz = nz + 2 * CPAD;
#pragma unroll
    for (int r = ty; r < 32; r += 8) {
        const int i = i0 + r, j = j0 + tx;
        T v = (T)0;
        if (i < ny && j < nx) {
            v = x[(int64_t)i * nx + j];
            if (vz) {
                T *q = vz + (int64_t)s * szz + 2 * (((int64_t)z * Ly + i + CPAD) * Lx + j + CPAD);
                q[0] = v;
                q[1 - 2 * Lx] = v;
            }
            if (vy) {
                T *q = vy + (int64_t)s * sy + 2 * (((int64_t)i * Lz + z + CPAD) * Lx + j + CPAD);
                q[0] = v;
                q[1 - 2 * Lx] = v;
            }
        }
        tile[r][tx] = v;
    }
    if (!vx) return;
    __syncthreads();
#pragma unroll
    for (int r = ty; r < 32; r += 8) {
        const int j = j0 + r, i = i0 + tx;
        if (i < ny && j < nx) {
            T *q = vx + (int64_t)s * sx + 2 * (((int64_t)j * Lz + z + CPAD) * Ly + i + CPAD);
            q[0] = tile[tx][r];
            q[1 - 2 * Ly] = tile[tx][r];
        }
    }
}

// Sinogram -> the padded pair view [views][nv+4][nu+4] in the accumulation
// type: pair (v, u) = (y[v][u], y[v + 1][u]), zeros outside the detector.
// One workgroup per padded row of pairs (view, v) of one slice; every pair,
// pads included, is written, so the buffer needs no clearing before.
template <typename TIN, typename T>
__global__ __launch_bounds__(256) void cone_pad_sino_k(VecRef yr, T *__restrict__ yp, int nviews, int nu, int nv,
                                                       int s0, int64_t ss, const int *kdev, const int *active) {
    const int s = s0 + blockIdx.y;
    if (active && !active[s]) return;
    const int k = kdev ? *kdev : 0;
    const int Lv = nv + 2 * CPAD, Lu = nu + 2 * CPAD;
    const int w = blockIdx.x / Lv, pr = blockIdx.x % Lv;
    const int r0 = pr - CPAD, r1 = r0 + 1;   // the detector rows of the pair
    const bool ok0 = r0 >= 0 && r0 < nv, ok1 = r1 >= 0 && r1 < nv;
    const TIN *y = vec_ptr<const TIN>(yr, s, k) + (int64_t)w * nv * nu;
    T *o = yp + (int64_t)s * ss + 2 * ((int64_t)w * Lv + pr) * Lu;
    for (int pc = threadIdx.x; pc < Lu; pc += 256) {
        const int c = pc - CPAD;
        const bool okc = c >= 0 && c < nu;
        const T v0 = ok0 && okc ? (T)load_as<TIN>(y, (int64_t)r0 * nu + c) : (T)0;
        const T v1 = ok1 && okc ? (T)load_as<TIN>(y, (int64_t)r1 * nu + c) : (T)0;
        o[2 * pc] = v0;
        o[2 * pc + 1] = v1;
    }
}

__device__ __forceinline__ uint32_t cremap(uint32_t L, uint32_t total, uint32_t nxcc) {
    const uint32_t q = total / nxcc, r = total % nxcc;
    const uint32_t x = L % nxcc, slot = L / nxcc;
    return x * q + min(x, r) + slot;
}

// A pointer that is the same in every lane of the wave, made scalar.
template <typename T>
__device__ __forceinline__ const T *uniform_ptr(const T *p) {
    const uint64_t v = reinterpret_cast<uint64_t>(p);
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v), hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
    return reinterpret_cast<const T *>(((uint64_t)hi << 32) | lo);
}

__device__ __forceinline__ float cfract(float t) { return __builtin_amdgcn_fractf(t); }

// a / b: in FP32 through the hardware reciprocal (1 ulp), in FP64 exactly.
__device__ __forceinline__ float cdiv(float a, float b) { return a * __builtin_amdgcn_rcpf(b); }
__device__ __forceinline__ double cdiv(double a, double b) { return a / b; }
__device__ __forceinline__ double cfract(double t) { return __builtin_amdgcn_fract(t); }

// Planes j (of np) whose crossing lies in (-1, n) for a coordinate
// c(j) = c0 + j*dc (unpadded), widened by one; clamped before conversion.
__device__ __forceinline__ void plane_range(double c0, double dc, int n, int np, int &lo, int &hi) {
    if (dc == 0.0) {
        if (!(c0 > -1.0 && c0 < (double)n)) {
            lo = np;
            hi = -1;
        }
        return;
    }
    double a = (-1.0 - c0) / dc, b = ((double)n - c0) / dc;
    double l = fmin(fmax(fmin(a, b), -2.0), (double)(np + 1));
    double h = fmin(fmax(fmax(a, b), -2.0), (double)(np + 1));
    lo = max(lo, (int)floor(l) - 1);
    hi = min(hi, (int)ceil(h) + 1);
}

// A: one thread per ray.  When all the rays of a wave share the dominant
// axis, the wave walks the union of their plane ranges in lockstep.  Two
// launch shapes, dealt to the XCDs in contiguous ranges of workgroups:
// TILE = 0: a workgroup is 256 consecutive detector columns of one row of one
// view; work order (slice, band of rb detector rows, view, row in the band,
// column block), one band of all rows by default (the views outermost).
// TILE = 16: the workgroup is a 16 x 16 tile of detector pixels of one view
// and a wave 16 columns x 4 rows of it; with TILE = 8 a wave is an 8 x 8
// quarter of the tile; nbu and rb are then the tiles per detector row and
// column.  Tile work order: (slice, group of vg views, tile row, tile column,
// view in the group), ngv groups (the last may be ragged); vg = 1 puts the
// views outermost, larger groups run neighbouring views of one tile next to
// each other, whose rays cross nearly the same voxels.  The even and odd
// steps are summed by the parity of the plane index, and steps outside a
// ray's own range read pad zeros, so every decomposition gives the same bits.
// clamp to [lo, hi] (one median-of-three instruction in FP32; equal to
// fmin(fmax(x, lo), hi) for every finite x)
__device__ __forceinline__ float cclamp(float x, float lo, float hi) { return __builtin_amdgcn_fmed3f(x, lo, hi); }
__device__ __forceinline__ double cclamp(double x, double lo, double hi) { return fmin(fmax(x, lo), hi); }

template <typename TI, typename TO, int TILE>
__global__ __launch_bounds__(256) void cone_fwd_k(const TI *__restrict__ vx, const TI *__restrict__ vy,
                                                  const TI *__restrict__ vz, int64_t sx, int64_t sy, int64_t szz,
                                                  VecRef yr, const ConeView *__restrict__ views, int nx, int ny,
                                                  int nz, int nviews, int nu, int nv, double pu, double pv,
                                                  int nbu, int rb, int nrb, int vg, int ngv, int off32, uint32_t nxcc,
                                                  int s0, const int *kdev, const int *active) {
    typedef typename acc_of<TI>::type T;
    const uint32_t w = cremap(blockIdx.x, gridDim.x, nxcc);
    int c, r, vw, s;
    bool live;
    if (TILE) {
        const int vi = (int)(w % (uint32_t)vg);
        const uint32_t w1 = w / (uint32_t)vg;
        const int tu = (int)(w1 % (uint32_t)nbu);
        const uint32_t w2 = w1 / (uint32_t)nbu;
        const int tv = (int)(w2 % (uint32_t)rb);
        const uint32_t w3 = w2 / (uint32_t)rb;
        vw = (int)(w3 % (uint32_t)ngv) * vg + vi;
        s = s0 + (int)(w3 / (uint32_t)ngv);
        if (vw >= nviews) return;   // the ragged last group of views (the whole workgroup)
        const int l = (int)(threadIdx.x & 63), wv = (int)(threadIdx.x >> 6);
        if (TILE == 16) {
            c = tu * 16 + (l & 15);
            r = tv * 16 + wv * 4 + (l >> 4);
        } else {
            c = tu * 16 + (wv & 1) * 8 + (l & 7);
            r = tv * 16 + (wv >> 1) * 8 + (l >> 3);
        }
        live = c < nu && r < nv;
        if (r >= nv) r = nv - 1;   // a dead lane of a ragged tile still computes a valid ray
    } else {
        const int cb = (int)(w % (uint32_t)nbu);
        const uint32_t w2 = w / (uint32_t)nbu;
        const int ri = (int)(w2 % (uint32_t)rb);
        const uint32_t w3 = w2 / (uint32_t)rb;
        vw = (int)(w3 % (uint32_t)nviews);
        const uint32_t w4 = w3 / (uint32_t)nviews;
        r = (int)(w4 % (uint32_t)nrb) * rb + ri;
        s = s0 + (int)(w4 / (uint32_t)nrb);
        if (r >= nv) return;   // the ragged last band (the whole workgroup)
        c = cb * 256 + (int)threadIdx.x;
        live = c < nu;
    }
    if (active && !active[s]) return;
    const int k = kdev ? *kdev : 0;
    const ConeView &V = views[vw];
    // ---- ray set-up (FP64)
    const double ou = (c - 0.5 * (nu - 1)) * pu, ov = (r - 0.5 * (nv - 1)) * pv;
    double d[3];
    ray_dir(V, ou, ov, d);
    const int ax = major_of(d[0], d[1], d[2]);
    const double len = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
    const double cx = 0.5 * (nx - 1), cy = 0.5 * (ny - 1), cz = 0.5 * (nz - 1);
    // plane coordinate a (leading axis), slow in-plane p, fast in-plane q:
    //   x-major: planes x, (p, q) = (z, y);  y-major: planes y, (z, x);  z-major: planes z, (y, x)
    int ia, ip, iq, na, np_, nq;
    double ca, cp, cq;
    const TI *P;
    if (ax == 0) { ia = 0; ip = 2; iq = 1; na = nx; np_ = nz; nq = ny; ca = cx; cp = cz; cq = cy; P = vx + (int64_t)s * sx; }
    else if (ax == 1) { ia = 1; ip = 2; iq = 0; na = ny; np_ = nz; nq = nx; ca = cy; cp = cz; cq = cx; P = vy + (int64_t)s * sy; }
    else { ia = 2; ip = 1; iq = 0; na = nz; np_ = ny; nq = nx; ca = cz; cp = cy; cq = cx; P = vz + (int64_t)s * szz; }
    // crossing of plane j: t = ((j - ca) - S_a) / d_a; coordinate = S + t d + c
    const double t0 = (-ca - V.S[ia]) / d[ia], dt = 1.0 / d[ia];
    const double p0 = V.S[ip] + t0 * d[ip] + cp, dp = dt * d[ip];
    const double q0 = V.S[iq] + t0 * d[iq] + cq, dq = dt * d[iq];
    int jlo = 0, jhi = na - 1;
    plane_range(p0, dp, np_, na, jlo, jhi);
    plane_range(q0, dq, nq, na, jlo, jhi);
    // the host made a copy for every axis that leads some ray (same FP64
    // arithmetic, no contraction); should one be missing, the ray reads nothing
    const bool missing = P == nullptr;
    if (!live || missing) {
        jlo = na;
        jhi = -1;
    }
    // lockstep over the union when the whole wave shares the axis
    const int a0 = __shfl(ax, 0);
    const bool same = __all(ax == a0) && !__any(missing);
    int ulo = jlo, uhi = jhi;
    if (same) {
        for (int o = 32; o > 0; o >>= 1) {
            ulo = min(ulo, __shfl_xor(ulo, o));
            uhi = max(uhi, __shfl_xor(uhi, o));
        }
        jlo = ulo;
        jhi = uhi;
    }
    const int Lq = nq + 2 * CPAD, Lp = np_ + 2 * CPAD;
    const T P0 = (T)(p0 + CPAD), DP = (T)dp, Q0 = (T)(q0 + CPAD), DQ = (T)dq;
    const T pmax = (T)(np_ + CPAD), qmax = (T)(nq + CPAD);
    // The march over planes jlo..jhi in two sums (even and odd planes), the
    // loads of four steps issued before any is combined.  In lockstep the copy
    // is the same for the whole wave: a scalar base and 32-bit byte offsets
    // (off32: a padded pair copy of one slice has < 2^32 bytes and its row
    // indices fit 24 bits), else per-lane 64-bit addresses; both read the same
    // entries.
    T acc0 = 0, acc1 = 0;
    auto march = [&](auto uni_tag) {
        constexpr bool UNI = decltype(uni_tag)::value;
        const TI *Pu = UNI ? uniform_ptr(P) : P;
        // in lockstep the plane range and the copy's row lengths are the
        // wave's (scalar registers): the plane counter and the plane's offset
        // are scalar work
        const int jl = UNI ? __builtin_amdgcn_readfirstlane(jlo) : jlo;
        const int jh = UNI ? __builtin_amdgcn_readfirstlane(jhi) : jhi;
        const uint32_t Lqw = UNI ? (uint32_t)__builtin_amdgcn_readfirstlane(Lq) : (uint32_t)Lq;
        const uint32_t Lpq = UNI ? (uint32_t)__builtin_amdgcn_readfirstlane(Lp * Lq) : (uint32_t)(Lp * Lq);
        // the four taps of plane jj and the two fractions
        auto load = [&](int jj, T &fp, T &fq, T &a00, T &a01, T &a10, T &a11) {
            const T pp = fma((T)jj, DP, P0), qq = fma((T)jj, DQ, Q0);
            fp = cfract(pp);
            fq = cfract(qq);
            const uint32_t ipp = (uint32_t)cclamp(pp, (T)0, pmax), iqq = (uint32_t)cclamp(qq, (T)0, qmax);
            // pairs (p, q) and (p, q + 1): x[p][q], x[p+1][q], x[p][q+1], x[p+1][q+1]
            if constexpr (UNI) {   // global loads: a scalar base plus a 32-bit byte offset
                // (the copy of one slice has < 2^32 bytes, and its rows and row
                // lengths fit a 24-bit multiply: checked by the host)
                const uint32_t ei = (uint32_t)jj * Lpq + __umul24(ipp, Lqw) + iqq;
                typedef const __attribute__((address_space(1))) char gchar;
                typedef const __attribute__((address_space(1))) TI gTI;
                gchar *b = (gchar *)Pu;
                const gTI *e = (const gTI *)(b + ei * (uint32_t)(2 * sizeof(TI)));
                a00 = (T)e[0];
                a10 = (T)e[1];
                a01 = (T)e[2];
                a11 = (T)e[3];
            } else {
                const uint32_t ei = ((uint32_t)jj * (uint32_t)Lp + ipp) * (uint32_t)Lq + iqq;
                const TI *e = Pu + 2 * (int64_t)ei;
                a00 = (T)e[0];
                a10 = (T)e[1];
                a01 = (T)e[2];
                a11 = (T)e[3];
            }
        };
        auto combine = [](T fp, T fq, T a00, T a01, T a10, T a11) -> T {
            const T lo = fma(fq, a01 - a00, a00), hi = fma(fq, a11 - a10, a10);
            return fma(fp, hi - lo, lo);
        };
        auto tap = [&](int jj) -> T {
            T fp, fq, a00, a01, a10, a11;
            load(jj, fp, fq, a00, a01, a10, a11);
            return combine(fp, fq, a00, a01, a10, a11);
        };
        int j = jl;
        if (j <= jh && (j & 1)) {
            acc1 += tap(j);
            ++j;
        }
        for (; j + 3 <= jh; j += 4) {
            T fp[4], fq[4], a00[4], a01[4], a10[4], a11[4], v[4];
#pragma unroll
            for (int h = 0; h < 4; ++h) load(j + h, fp[h], fq[h], a00[h], a01[h], a10[h], a11[h]);
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int h = 0; h < 4; ++h) v[h] = combine(fp[h], fq[h], a00[h], a01[h], a10[h], a11[h]);
            acc0 += v[0];
            acc1 += v[1];
            acc0 += v[2];
            acc1 += v[3];
        }
        if (j + 1 <= jh) {
            const T v0 = tap(j), v1 = tap(j + 1);
            acc0 += v0;
            acc1 += v1;
            j += 2;
        }
        if (j <= jh) acc0 += tap(j);
    };
    if (same && off32)
        march(std::true_type{});
    else
        march(std::false_type{});
    if (!live) return;
    const T wgt = (T)(len / fabs(d[ia]));
    store_as<TO>(vec_ptr<TO>(yr, s, k), ((int64_t)vw * nv + r) * nu + c, (acc0 + acc1) * wgt);
}

// B: one thread per CZT voxels along z (a 16 x 16 (y, x) tile per workgroup;
// CZT is a launch choice that leaves every sum unchanged); loop over the views.
// MP is the power of the magnification in the weight: 2 for the cone beam
// (two transverse detector axes), 1 for the fan beam.
constexpr int CZT_DEFAULT = 4;


template <typename TI, int CZT, int MP>
__global__ __launch_bounds__(256) void cone_bp_k(const typename acc_of<TI>::type *__restrict__ yp, int64_t ss,
                                                 VecRef xr, const ConeB<typename acc_of<TI>::type> *__restrict__ vb,
                                                 int nx, int ny, int nz, int nviews, int nu, int nv,
                                                 typename acc_of<TI>::type ipp, int ntx, int nty,
                                                 int ntz, uint32_t nxcc, int s0, const int *kdev,
                                                 const int *active) {
    typedef typename acc_of<TI>::type T;
    const uint32_t w = cremap(blockIdx.x, gridDim.x, nxcc);
    const int txi = (int)(w % (uint32_t)ntx);
    const uint32_t w2 = w / (uint32_t)ntx;
    const int tyi = (int)(w2 % (uint32_t)nty);
    const uint32_t w3 = w2 / (uint32_t)nty;
    const int tzi = (int)(w3 % (uint32_t)ntz);
    const int s = s0 + (int)(w3 / (uint32_t)ntz);
    if (active && !active[s]) return;
    const int k = kdev ? *kdev : 0;
    const int j = txi * 16 + (threadIdx.x & 15), i = tyi * 16 + (threadIdx.x >> 4), z0 = tzi * CZT;
    const T X = (T)j - (T)0.5 * (T)(nx - 1), Y = (T)i - (T)0.5 * (T)(ny - 1);
    T Z[CZT], acc[CZT];
#pragma unroll
    for (int m = 0; m < CZT; ++m) {
        Z[m] = (T)(z0 + m) - (T)0.5 * (T)(nz - 1);
        acc[m] = 0;
    }
    const int Lu = nu + 2 * CPAD, Lv = nv + 2 * CPAD;
    const T umax = (T)(nu + CPAD), vmax = (T)(nv + CPAD);
    const T *Ys = yp + (int64_t)s * ss;
    const uint32_t rowb = (uint32_t)Lu * (uint32_t)(2 * sizeof(T));   // bytes per padded row of pairs
    for (int vw = 0; vw < nviews; ++vw) {
        const ConeB<T> b = vb[vw];
        // the detector normal and column axis have no z part (checked when
        // the operator is built), so the magnification M, the column u and
        // the weight are those of the whole column of voxels
        const T den = fma(X, b.n[0], fma(Y, b.n[1], -b.Sn));
        const T bu = fma(X, b.eup[0], fma(Y, b.eup[1], -b.Su));
        const T bv = fma(X, b.evp[0], fma(Y, b.evp[1], -b.Sv));
        const T M = cdiv(b.dist, den);
        const T u = fma(M, bu, b.cu);   // padded coordinates
        const T fu = cfract(u);
        const uint32_t ub = (uint32_t)cclamp(u, (T)0, umax) * (uint32_t)(2 * sizeof(T));
        const T wgt = (MP == 2 ? M * M : M) * ipp;
        // the view is the same for the whole workgroup: 32-bit byte offsets
        // from its base (the launcher requires a padded pair view of < 2^32
        // bytes and rows of < 2^24 bytes); the pairs (v, u) and (v, u + 1)
        // are the four taps
        const T *view = Ys + 2 * (int64_t)vw * Lv * Lu;
#pragma unroll
        for (int m = 0; m < CZT; ++m) {
            const T v = fma(M, fma(Z[m], b.evp[2], bv), b.cv);
            const T fv = cfract(v);
            const uint32_t iv = (uint32_t)cclamp(v, (T)0, vmax);
            const T *e = reinterpret_cast<const T *>(reinterpret_cast<const char *>(view) + __umul24(iv, rowb) + ub);
            const T a00 = e[0], a10 = e[1], a01 = e[2], a11 = e[3];
            const T lo = fma(fu, a01 - a00, a00), hi = fma(fu, a11 - a10, a10);
            acc[m] = fma(wgt, fma(fv, hi - lo, lo), acc[m]);
        }
    }
    if (i < ny && j < nx) {
        TI *xo = vec_ptr<TI>(xr, s, k);
#pragma unroll
        for (int m = 0; m < CZT; ++m)
            if (z0 + m < nz) xo[((int64_t)(z0 + m) * ny + i) * nx + j] = (TI)acc[m];
    }
}

// ------------------------------------------------------------ launchers ---
constexpr uint32_t CMAX_GROUPS = (1u << 31) / 256;

template <typename T>
static int fill(T *p, int64_t n, hipStream_t st) {
    if (n <= 0) return ABBA_OK;
    hipLaunchKernelGGL(cfill_k<T>, dim3((unsigned)std::min<int64_t>(4096, (n + 255) / 256)), dim3(256), 0, st, p, n);
    ABBA_LAUNCHED("cfill_k");
    return ABBA_OK;
}

template <typename TI, typename TO>
static int cone_fwd_t(const abba_op *op, VecRef x, VecRef y, int batch, void *scratch, const Launch &L) {
    const abba_geometry &g = op->g;
    const ConeCopies cc = cone_copies(op);
    TI *base = (TI *)scratch;
    TI *vx = cc.vx ? base : nullptr;
    TI *vy = cc.vy ? base + (size_t)batch * cc.vx : nullptr;
    TI *vz = cc.vz ? base + (size_t)batch * (cc.vx + cc.vy) : nullptr;
    int rc;
    if ((rc = fill<TI>(base, (int64_t)batch * (cc.vx + cc.vy + cc.vz), L.stream))) return rc;
    for (int s0 = 0; s0 < batch; s0 += std::max(1, 65535 / g.nz)) {
        const int nb = std::min(std::max(1, 65535 / g.nz), batch - s0);
        dim3 grid((g.nx + 31) / 32, (g.ny + 31) / 32, nb * g.nz);
        hipLaunchKernelGGL(cone_pad_vol_k<TI>, grid, dim3(256), 0, L.stream, x, vx, vy, vz, g.nx, g.ny, g.nz, s0,
                           (int64_t)cc.vx, (int64_t)cc.vy, (int64_t)cc.vz, L.kdev, L.active);
        ABBA_LAUNCHED("cone_pad_vol_k");
    }
    // pair indices within one slice's copy in 32 bits (two elements per pair)
    if (std::max({cc.vx, cc.vy, cc.vz}) >= (size_t)1 << 33) return ABBA_ERR_UNSUPPORTED;
    // 32-bit byte offsets within one slice's copy, built from 24-bit products
    // (row index plane * rows + row, and row length, below 2^24)
    const size_t rows = (size_t)(std::max({g.nx, g.ny, g.nz}) + 1) * (size_t)(std::max({g.nx, g.ny, g.nz}) + 2 * CPAD);
    const int off32 = std::max({cc.vx, cc.vy, cc.vz}) * sizeof(TI) < ((size_t)1 << 32) && rows < ((size_t)1 << 24) ? 1 : 0;
    int nbu = (g.det_u + 255) / 256;
    int rb = g.det_v;
    // built-in: 16 x 16 detector tiles with waves of 16 x 4, groups of 24
    // views per tile, at most 6 workgroups per CU.  Measured at 256^3 / 360 x
    // 384^2 (pair copies): 256-column rows 14.7 ms; tiles with groups of 8 /
    // 16 / 24 / 32 / 48 / 64 views 4.84 / 4.56 / 4.37 / 4.52 / 4.40 / 5.17 ms
    // (8 x 8 waves 0.4-0.6 ms slower).  Detectors of fewer than 16 rows (the
    // fan beam has one) keep the rows of 256 columns.
    int tile = g.det_v >= 16 ? 16 : 0, vg = 24;
    size_t cap_lds = tile ? (size_t)op->lds_cu / 6 / 512 * 512 : 0;   // unused LDS that caps the workgroups per CU
    if (const TuneEntry *t = tune_for(op, batch)) {
        if (t->a_vg >= 1) vg = t->a_vg;
        if (t->a_rb >= 1) rb = std::min(t->a_rb, g.det_v);
        if (t->a_occ >= 1) cap_lds = std::min<size_t>(65536, (size_t)op->lds_cu / (size_t)t->a_occ / 512 * 512);
        else if (t->a_tile != 0 || t->a_rb >= 1) cap_lds = 0;
        if (t->a_tile == -1 || t->a_rb >= 1) tile = 0;
        else if (t->a_tile == 8 || t->a_tile == 16) tile = t->a_tile;
    }
    int nrb = (g.det_v + rb - 1) / rb;
    if (tile) {   // tiles per detector row (nbu) and per column (rb); one band
        nbu = (g.det_u + 15) / 16;
        rb = (g.det_v + 15) / 16;
        nrb = 1;
    } else {
        vg = 1;
    }
    vg = std::min(vg, g.n_angles);
    const int ngv = (g.n_angles + vg - 1) / vg;   // groups of views (the rows order keeps vg = 1)
    const uint64_t per = (uint64_t)nbu * nrb * rb * ngv * vg;
    if (per > CMAX_GROUPS) return ABBA_ERR_UNSUPPORTED;
    const int ch = (int)std::min<uint64_t>((uint64_t)batch, CMAX_GROUPS / per);
    for (int s0 = 0; s0 < batch; s0 += ch) {
        const int nb = std::min(ch, batch - s0);
#define CONE_FWD(TL)                                                                                              \
    hipLaunchKernelGGL((cone_fwd_k<TI, TO, TL>), dim3((uint32_t)(per * nb)), dim3(256), cap_lds, L.stream, vx, vy, vz, \
                       (int64_t)cc.vx, (int64_t)cc.vy, (int64_t)cc.vz, y, (const ConeView *)op->tab, g.nx, g.ny,     \
                       g.nz, g.n_angles, g.det_u, g.det_v, g.det_pitch_u, g.det_pitch_v, nbu, rb, nrb, vg, ngv,      \
                       off32, (uint32_t)op->nxcc, s0, L.kdev, L.active)
        if (tile == 16) CONE_FWD(16);
        else if (tile == 8) CONE_FWD(8);
        else CONE_FWD(0);
#undef CONE_FWD
        ABBA_LAUNCHED("cone_fwd_k");
    }
    return ABBA_OK;
}

int cone_forward(const abba_op *op, VecRef x, VecRef y, int y_dtype, int batch, void *scratch, const Launch &L) {
    if (batch <= 0) return ABBA_OK;
    if (op->img_dtype == ABBA_F64) {
        if (y_dtype != ABBA_F64) return ABBA_ERR_DTYPE;
        return cone_fwd_t<double, double>(op, x, y, batch, scratch, L);
    }
    if (y_dtype == ABBA_F32) return cone_fwd_t<float, float>(op, x, y, batch, scratch, L);
    if (y_dtype == ABBA_BF16) return cone_fwd_t<float, bf16>(op, x, y, batch, scratch, L);
    return ABBA_ERR_DTYPE;
}

template <typename TI, int CZT>
static int cone_bp_launch(const abba_op *op, const typename acc_of<TI>::type *yp, VecRef x, int batch,
                          const Launch &L) {
    typedef typename acc_of<TI>::type T;
    const abba_geometry &g = op->g;
    const ConeCopies cc = cone_copies(op);
    const int ntx = (g.nx + 15) / 16, nty = (g.ny + 15) / 16, ntz = (g.nz + CZT - 1) / CZT;
    const uint64_t per = (uint64_t)ntx * nty * ntz;
    if (per > CMAX_GROUPS) return ABBA_ERR_UNSUPPORTED;
    // byte offsets within one padded view in 32 bits, its rows (and row
    // indices) within the 24 bits of one multiply
    if ((int64_t)(g.det_u + 2 * CPAD) * (g.det_v + 2 * CPAD) * (int64_t)(2 * sizeof(T)) >= (int64_t)1 << 32 ||
        (int64_t)(g.det_u + 2 * CPAD) * (int64_t)(2 * sizeof(T)) >= (int64_t)1 << 24 ||
        g.det_v + 2 * CPAD >= (1 << 24))
        return ABBA_ERR_UNSUPPORTED;
    const int ch = (int)std::min<uint64_t>((uint64_t)batch, CMAX_GROUPS / per);
    const size_t bytes_d = sizeof(ConeView) * g.n_angles;
    const ConeB<T> *vb = reinterpret_cast<const ConeB<T> *>((const unsigned char *)op->tab + bytes_d);
    for (int s0 = 0; s0 < batch; s0 += ch) {
        const int nb = std::min(ch, batch - s0);
        const T ipp = (T)(1.0 / (g.det_pitch_u * g.det_pitch_v));
        if (g.kind == ABBA_GEOM_FAN2D)
            hipLaunchKernelGGL((cone_bp_k<TI, CZT, 1>), dim3((uint32_t)(per * nb)), dim3(256), 0, L.stream, yp,
                               (int64_t)cc.sino, x, vb, g.nx, g.ny, g.nz, g.n_angles, g.det_u, g.det_v, ipp, ntx,
                               nty, ntz, (uint32_t)op->nxcc, s0, L.kdev, L.active);
        else
            hipLaunchKernelGGL((cone_bp_k<TI, CZT, 2>), dim3((uint32_t)(per * nb)), dim3(256), 0, L.stream, yp,
                               (int64_t)cc.sino, x, vb, g.nx, g.ny, g.nz, g.n_angles, g.det_u, g.det_v, ipp, ntx,
                               nty, ntz, (uint32_t)op->nxcc, s0, L.kdev, L.active);
        ABBA_LAUNCHED("cone_bp_k");
    }
    return ABBA_OK;
}

template <typename TIN, typename TI>
static int cone_bp_t(const abba_op *op, VecRef y, VecRef x, int batch, void *scratch, const Launch &L) {
    typedef typename acc_of<TI>::type T;
    const abba_geometry &g = op->g;
    const ConeCopies cc = cone_copies(op);
    T *yp = (T *)scratch;   // every pair is written by the padding kernel
    if ((uint64_t)g.n_angles * (g.det_v + 2 * CPAD) > 0x7fffffffull) return ABBA_ERR_UNSUPPORTED;
    for (int s0 = 0; s0 < batch; s0 += 65535) {
        const int nb = std::min(65535, batch - s0);
        hipLaunchKernelGGL((cone_pad_sino_k<TIN, T>), dim3(g.n_angles * (g.det_v + 2 * CPAD), nb), dim3(256), 0,
                           L.stream, y, yp,
                           g.n_angles, g.det_u, g.det_v, s0, (int64_t)cc.sino, L.kdev, L.active);
        ABBA_LAUNCHED("cone_pad_sino_k");
    }
    int czt = CZT_DEFAULT;
    if (const TuneEntry *t = tune_for(op, batch))
        if (t->czt == 2 || t->czt == 4 || t->czt == 8) czt = t->czt;
    if (czt == 2) return cone_bp_launch<TI, 2>(op, yp, x, batch, L);
    if (czt == 8) return cone_bp_launch<TI, 8>(op, yp, x, batch, L);
    return cone_bp_launch<TI, 4>(op, yp, x, batch, L);
}

int cone_tune_candidates(const abba_op *op, TuneEntry *out, int cap) {
    int n = 0;
    if (op->kind == ABBA_OP_PIXEL)
        for (int c : {2, 4, 8})
            if (n < cap) out[n++] = TuneEntry{0, 0, 0, 0, c, 0};
    if (op->kind == ABBA_OP_JOSEPH) {
        // 256-column rows (views outermost, or bands of rows), 16 x 16 tiles
        // with waves of 16 x 4 or 8 x 8, caps of the workgroups per CU, and
        // groups of neighbouring views per tile
        if (n < cap) out[n++] = TuneEntry{0, 0, 0, 0, 0, 0, 5, -1};
        for (int r : {8, 32})
            if (n < cap && r < op->g.det_v) out[n++] = TuneEntry{0, 0, 0, 0, 0, r, 5};
        for (int c : {5, 0})
            if (n < cap) out[n++] = TuneEntry{0, 0, 0, 0, 0, 0, c, 16};
        for (int v : {16, 48})
            if (n < cap) out[n++] = TuneEntry{0, 0, 0, 0, 0, 0, 6, 16, v};
        for (int c : {5, 0})
            if (n < cap) out[n++] = TuneEntry{0, 0, 0, 0, 0, 0, c, 8};
        if (n < cap) out[n++] = TuneEntry{0, 0, 0, 0, 0, 0, 5, 8, 48};
    }
    return n;
}

int cone_back(const abba_op *op, VecRef y, int y_dtype, VecRef x, int batch, void *scratch, const Launch &L) {
    if (batch <= 0) return ABBA_OK;
    if (op->kind != ABBA_OP_PIXEL) return ABBA_ERR_UNSUPPORTED;
    if (op->img_dtype == ABBA_F64) {
        if (y_dtype != ABBA_F64) return ABBA_ERR_DTYPE;
        return cone_bp_t<double, double>(op, y, x, batch, scratch, L);
    }
    if (y_dtype == ABBA_F32) return cone_bp_t<float, float>(op, y, x, batch, scratch, L);
    if (y_dtype == ABBA_BF16) return cone_bp_t<bf16, float>(op, y, x, batch, scratch, L);
    return ABBA_ERR_DTYPE;
}

}  // namespace abba
