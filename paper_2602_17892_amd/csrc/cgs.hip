// Arnoldi orthogonalisation (eq. (8)) with classical Gram-Schmidt and one
// re-orthogonalisation pass (CGS2), plus the other HBM-streaming kernels of
// the solver: residual / norm formation and the assembly of x_k (eq. (13)).
//
// Every kernel streams basis vectors of one or many slices with 16-byte
// vector loads (float4 / double2); the padded vector stride is a multiple of
// 256 elements so every vector load is aligned.  Products are accumulated in
// FP64.  Reductions are two-stage with a fixed order (per-block partials,
// then one ordered pass), so results do not depend on scheduling.
#include "solve.h"

namespace abba {

template <typename T> struct vec16;
template <> struct vec16<float> { typedef float4 type; static constexpr int N = 4; };
template <> struct vec16<double> { typedef double2 type; static constexpr int N = 2; };

__device__ __forceinline__ void unpack(const float4 &v, double *o) { o[0] = v.x; o[1] = v.y; o[2] = v.z; o[3] = v.w; }
__device__ __forceinline__ void unpack(const double2 &v, double *o) { o[0] = v.x; o[1] = v.y; }
__device__ __forceinline__ float4 pack_f(const double *o) { return make_float4((float)o[0], (float)o[1], (float)o[2], (float)o[3]); }

// A basis column read once per sweep (the basis is far larger than the
// caches): a load with the non-temporal hint.
__device__ __forceinline__ float4 ld_stream(const float4 *p) {
    typedef float f4 __attribute__((ext_vector_type(4)));
    const f4 v = __builtin_nontemporal_load(reinterpret_cast<const f4 *>(p));
    return make_float4(v.x, v.y, v.z, v.w);
}
__device__ __forceinline__ double2 ld_stream(const double2 *p) {
    typedef double d2 __attribute__((ext_vector_type(2)));
    const d2 v = __builtin_nontemporal_load(reinterpret_cast<const d2 *>(p));
    return make_double2(v.x, v.y);
}

template <typename T> __device__ __forceinline__ typename vec16<T>::type pack(const double *o);
template <> __device__ __forceinline__ float4 pack<float>(const double *o) { return pack_f(o); }
template <> __device__ __forceinline__ double2 pack<double>(const double *o) { return make_double2(o[0], o[1]); }

// Block chunk of `nvec` vectors split into `nblk` contiguous pieces.
__device__ __forceinline__ void chunk_of(int64_t nvec, int nblk, int blk, int64_t &v0, int64_t &v1) {
    const int64_t per = (nvec + nblk - 1) / nblk;
    v0 = (int64_t)blk * per;
    v1 = min(nvec, v0 + per);
}

// part[s][blk][j] = sum over this block's elements of W_j . q, for
// j in [j0, j0+DOT_JT) and j < k + extra, where q = W_k (k read on device).
template <typename TW>
__global__ __launch_bounds__(256) void dots_k(const TW *__restrict__ W, int64_t slice_stride, int64_t ldw,
                                              double *__restrict__ part, int nblk, int pstride, int extra,
                                              const int *kdev, const int *active) {
    typedef typename vec16<TW>::type V;
    constexpr int N = vec16<TW>::N;
    const int s = blockIdx.z;
    if (active && !active[s]) return;
    const int k = kdev ? *kdev : 0;
    const int jcount = k + extra;
    const int j0 = blockIdx.y * DOT_JT;
    if (j0 >= jcount) return;
    const int jn = min(DOT_JT, jcount - j0);
    const TW *Ws = W + (int64_t)s * slice_stride;
    const V *q = reinterpret_cast<const V *>(Ws + (int64_t)k * ldw);
    int64_t v0, v1;
    chunk_of(ldw / N, nblk, blockIdx.x, v0, v1);
    double acc[DOT_JT];
#pragma unroll
    for (int jj = 0; jj < DOT_JT; ++jj) acc[jj] = 0.0;
    for (int64_t v = v0 + threadIdx.x; v < v1; v += blockDim.x) {
        double qv[N];
        unpack(q[v], qv);
#pragma unroll
        for (int jj = 0; jj < DOT_JT; ++jj) {
            if (jj < jn) {
                double wv[N];
                unpack(reinterpret_cast<const V *>(Ws + (int64_t)(j0 + jj) * ldw)[v], wv);
#pragma unroll
                for (int e = 0; e < N; ++e) acc[jj] = fma(wv[e], qv[e], acc[jj]);
            }
        }
    }
    __shared__ double red[DOT_JT][4];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
    for (int jj = 0; jj < DOT_JT; ++jj) {
        double t = wave_sum(acc[jj]);
        if (lane == 0) red[jj][wid] = t;
    }
    __syncthreads();
    if (threadIdx.x < jn) {
        const int jj = threadIdx.x;
        double t = 0.0;
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) t += red[jj][w];
        part[((int64_t)s * pstride + j0 + jj) * nblk + blockIdx.x] = t;
    }
}

// out[s][j] = sum over blocks of part[s][j][blk]: one wave per vector j,
// lanes stride over the (contiguous) block partials, then a fixed-order
// butterfly, so the result does not depend on scheduling.
__global__ __launch_bounds__(256) void reduce_k(const double *__restrict__ part, int nblk, int pstride,
                                                double *__restrict__ out, int ostride, int extra, int kfixed,
                                                const int *kdev, const int *active) {
    const int s = blockIdx.x;
    if (active && !active[s]) return;
    const int jcount = (kdev ? *kdev : kfixed) + extra;
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
    for (int j = wid; j < jcount; j += nw) {
        const double *p = part + ((int64_t)s * pstride + j) * nblk;
        double t = 0.0;
        for (int b = lane; b < nblk; b += 64) t += p[b];
        t = wave_sum(t);
        if (lane == 0) out[(int64_t)s * ostride + j] = t;
    }
}

// q := q - sum_{j<k} coef[s][j] W_j  (q = W_k), accumulated in FP64; with
// NORM, also npart[s][blk] = this block's share of ||q||^2.
template <typename TW, bool NORM>
__global__ __launch_bounds__(256) void update_k(TW *__restrict__ W, int64_t slice_stride, int64_t ldw,
                                                const double *__restrict__ coef, int cstride,
                                                double *__restrict__ npart, int nblk,
                                                const int *kdev, const int *active) {
    typedef typename vec16<TW>::type V;
    constexpr int N = vec16<TW>::N;
    const int s = blockIdx.z;
    if (active && !active[s]) return;
    const int k = *kdev;
    TW *Ws = W + (int64_t)s * slice_stride;
    V *q = reinterpret_cast<V *>(Ws + (int64_t)k * ldw);
    const double *cf = coef + (int64_t)s * cstride;
    int64_t v0, v1;
    chunk_of(ldw / N, nblk, blockIdx.x, v0, v1);
    double nrm = 0.0;
    for (int64_t v = v0 + threadIdx.x; v < v1; v += blockDim.x) {
        double qv[N];
        unpack(q[v], qv);
        int j = 0;
        for (; j + 4 <= k; j += 4) {
            double w0[N], w1[N], w2[N], w3[N];
            unpack(reinterpret_cast<const V *>(Ws + (int64_t)(j + 0) * ldw)[v], w0);
            unpack(reinterpret_cast<const V *>(Ws + (int64_t)(j + 1) * ldw)[v], w1);
            unpack(reinterpret_cast<const V *>(Ws + (int64_t)(j + 2) * ldw)[v], w2);
            unpack(reinterpret_cast<const V *>(Ws + (int64_t)(j + 3) * ldw)[v], w3);
            const double c0 = cf[j], c1 = cf[j + 1], c2 = cf[j + 2], c3 = cf[j + 3];
#pragma unroll
            for (int e = 0; e < N; ++e) {
                qv[e] = fma(-c0, w0[e], qv[e]);
                qv[e] = fma(-c1, w1[e], qv[e]);
                qv[e] = fma(-c2, w2[e], qv[e]);
                qv[e] = fma(-c3, w3[e], qv[e]);
            }
        }
        for (; j < k; ++j) {
            double w0[N];
            unpack(reinterpret_cast<const V *>(Ws + (int64_t)j * ldw)[v], w0);
            const double c0 = cf[j];
#pragma unroll
            for (int e = 0; e < N; ++e) qv[e] = fma(-c0, w0[e], qv[e]);
        }
        V out = pack<TW>(qv);
        q[v] = out;
        if (NORM) {
            double r[N];
            unpack(out, r);   // the norm of the stored (rounded) vector
#pragma unroll
            for (int e = 0; e < N; ++e) nrm = fma(r[e], r[e], nrm);
        }
    }
    if (NORM) {
        __shared__ double red[4];
        const double t = block_sum(nrm, red);
        if (threadIdx.x == 0) npart[(int64_t)s * nblk + blockIdx.x] = t;
    }
}

// Close Arnoldi step k of every active slice: H(0:k-1, k-1) = h + c,
// h_{k+1,k} = ||q||, breakdown test against ||M w_k||, 1/h_{k+1,k}.
__global__ void arnoldi_close_k(const double *__restrict__ h, const double *__restrict__ c, int hstride,
                                const double *__restrict__ npart, int nblk, double *__restrict__ H, int K,
                                double *__restrict__ sc, int *__restrict__ flags, const int *kdev,
                                const int *active) {
    const int s = blockIdx.x;
    if (active && !active[s]) return;
    const int k = *kdev;
    double *col = H + ((int64_t)s * K + (k - 1)) * (K + 1);
    const double *hs = h + (int64_t)s * hstride, *cs = c + (int64_t)s * hstride;
    for (int i = threadIdx.x; i < k; i += blockDim.x) col[i] = hs[i] + cs[i];
    if (threadIdx.x == 0) {
        double n2 = 0.0;
        for (int b = 0; b < nblk; ++b) n2 += npart[(int64_t)s * nblk + b];
        const double hk = sqrt(n2);
        const double mw = sqrt(hs[k]);   // NaN stays NaN
        double *S = sc + (int64_t)s * SC_COUNT;
        S[SC_MW] = mw;
        int fl = 0;
        if (!isfinite(hk) || !isfinite(mw)) fl |= FL_NONFINITE;
        if (hk <= 1e-14 * mw) {
            fl |= FL_BREAK;
            col[k] = 0.0;
            S[SC_HK] = 0.0;
            S[SC_INV] = 0.0;
        } else {
            col[k] = hk;
            S[SC_HK] = hk;
            S[SC_INV] = 1.0 / hk;
        }
        flags[s] |= fl;
    }
}

// W_k *= sc[SC_INV] (no-op on breakdown).
template <typename TW>
__global__ __launch_bounds__(256) void scale_k(TW *__restrict__ W, int64_t slice_stride, int64_t ldw,
                                               const double *__restrict__ sc, int kfixed, const int *kdev,
                                               const int *active) {
    typedef typename vec16<TW>::type V;
    constexpr int N = vec16<TW>::N;
    const int s = blockIdx.z;
    if (active && !active[s]) return;
    const int k = kdev ? *kdev : kfixed;
    const double inv = sc[(int64_t)s * SC_COUNT + SC_INV];
    if (inv == 0.0) return;
    V *q = reinterpret_cast<V *>(W + (int64_t)s * slice_stride + (int64_t)k * ldw);
    const int64_t nvec = ldw / N;
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < nvec; v += (int64_t)gridDim.x * blockDim.x) {
        double a[N];
        unpack(q[v], a);
#pragma unroll
        for (int e = 0; e < N; ++e) a[e] *= inv;
        q[v] = pack<TW>(a);
    }
}

// out[s] = b[s] - ax[s] over the first `len` entries, zero on the padding.
template <typename TS, typename TO>
__global__ __launch_bounds__(256) void sub_k(const TS *__restrict__ b, int64_t bstride, const TS *__restrict__ ax,
                                             int64_t axstride, TO *__restrict__ out, int64_t ostride, int64_t len,
                                             int64_t ld) {
    const int s = blockIdx.y;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < ld; e += (int64_t)gridDim.x * blockDim.x) {
        typename acc_of<TO>::type v = 0;
        if (e < len) v = (typename acc_of<TO>::type)load_as<TS>(b + s * bstride, e) -
                         (typename acc_of<TO>::type)load_as<TS>(ax + s * axstride, e);
        store_as<TO>(out + s * ostride, e, v);
    }
}

// npart[s][blk] = partial ||v_s||^2 over `len` entries (any storage type).
template <typename T>
__global__ __launch_bounds__(256) void sqnorm_k(const T *__restrict__ v, int64_t stride, int64_t len,
                                                double *__restrict__ npart, int nblk) {
    const int s = blockIdx.y;
    int64_t e0, e1;
    chunk_of(len, nblk, blockIdx.x, e0, e1);
    double acc = 0.0;
    for (int64_t e = e0 + threadIdx.x; e < e1; e += blockDim.x) {
        const double a = (double)load_as<T>(v + s * stride, e);
        acc = fma(a, a, acc);
    }
    __shared__ double red[4];
    const double t = block_sum(acc, red);
    if (threadIdx.x == 0) npart[(int64_t)s * nblk + blockIdx.x] = t;
}

// Zero the padding [len, ld) of `nv` vectors of every slice.
template <typename T>
__global__ void zero_pad_k(T *__restrict__ base, int64_t slice_stride, int nv, int64_t ld, int64_t len) {
    const int s = blockIdx.y;
    const int64_t padn = ld - len;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < padn * nv; t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t j = t / padn, e = len + t % padn;
        base[s * slice_stride + j * ld + e] = (T)0;
    }
}
template <>
__global__ void zero_pad_k<bf16>(bf16 *__restrict__ base, int64_t slice_stride, int nv, int64_t ld, int64_t len) {
    const int s = blockIdx.y;
    const int64_t padn = ld - len;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < padn * nv; t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t j = t / padn, e = len + t % padn;
        base[s * slice_stride + j * ld + e].bits = 0;
    }
}

// x_s += sum_{j < iters_s} y[s][j] V_j  (eq. (13): V = B W_k in AB mode,
// V = W_k in BA mode); FP64 accumulation, one rounding at the store.
template <typename TV, typename TX>
__global__ __launch_bounds__(256) void assemble_k(TX *__restrict__ x, int64_t xstride, const TV *__restrict__ Vb,
                                                  int64_t vslice, int64_t ldv, const double *__restrict__ y,
                                                  int ystride, const int *__restrict__ iters, int64_t n) {
    const int s = blockIdx.y;
    const int k = iters[s];
    if (k <= 0) return;
    const TV *Vs = Vb + (int64_t)s * vslice;
    const double *ys = y + (int64_t)s * ystride;
    TX *xs = x + (int64_t)s * xstride;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
        double acc = (double)xs[e];
        int j = 0;
        for (; j + 4 <= k; j += 4) {
            const double a0 = Vs[(int64_t)(j + 0) * ldv + e], a1 = Vs[(int64_t)(j + 1) * ldv + e];
            const double a2 = Vs[(int64_t)(j + 2) * ldv + e], a3 = Vs[(int64_t)(j + 3) * ldv + e];
            acc = fma(ys[j], a0, acc);
            acc = fma(ys[j + 1], a1, acc);
            acc = fma(ys[j + 2], a2, acc);
            acc = fma(ys[j + 3], a3, acc);
        }
        for (; j < k; ++j) acc = fma(ys[j], (double)Vs[(int64_t)j * ldv + e], acc);
        xs[e] = (TX)acc;
    }
}

// BA data residual: npart[s][blk] = partial ||r0 - sum_{j<k} y_j Z_j||^2
// with r0 = b - A x_0 and Z_j = A w_j (sinogram storage type).
template <typename TS>
__global__ __launch_bounds__(256) void resid_k(const TS *__restrict__ r0, int64_t rstride, const TS *__restrict__ Z,
                                               int64_t zslice, int64_t ldz, const double *__restrict__ y, int ystride,
                                               int64_t len, double *__restrict__ npart, int nblk, const int *kdev,
                                               const int *active) {
    const int s = blockIdx.y;
    if (active && !active[s]) return;
    const int k = *kdev;
    int64_t e0, e1;
    chunk_of(len, nblk, blockIdx.x, e0, e1);
    const TS *Zs = Z + (int64_t)s * zslice;
    const double *ys = y + (int64_t)s * ystride;
    double acc = 0.0;
    for (int64_t e = e0 + threadIdx.x; e < e1; e += blockDim.x) {
        double r = (double)load_as<TS>(r0 + s * rstride, e);
        for (int j = 0; j < k; ++j) r = fma(-ys[j], (double)load_as<TS>(Zs + (int64_t)j * ldz, e), r);
        acc = fma(r, r, acc);
    }
    __shared__ double red[4];
    const double t = block_sum(acc, red);
    if (threadIdx.x == 0) npart[(int64_t)s * nblk + blockIdx.x] = t;
}

// ------------------------------------------------------- delayed CGS2 ---
// Step k of CGS2 with the second pass delayed by one step (Arnoldi, eq. (8)).
// On entry W_0..W_{k-1} are final, v = W_k is the once-orthogonalised next
// vector and z = W_{k+1} = M v.  One sweep gives, for i <= k,
//   a_i = W_i . v   (a_k = v.v)        b_i = W_i . z   (b_k = v.z)
// part rows [0, K+2) hold the a partials, rows [K+2, 2K+4) the b partials.
template <typename TW>
__global__ __launch_bounds__(256) void ddots_k(const TW *__restrict__ W, int64_t slice_stride, int64_t ldw,
                                               double *__restrict__ part, int nblk, int pstride, int boff,
                                               const int *kdev, const int *active) {
    typedef typename vec16<TW>::type V;
    constexpr int N = vec16<TW>::N;
    const int s = blockIdx.z;
    if (active && !active[s]) return;
    const int k = kdev ? *kdev : 0;
    const int jcount = k + 1;
    const int j0 = blockIdx.y * DOT_JT;
    if (j0 >= jcount) return;
    const int jn = min(DOT_JT, jcount - j0);
    const TW *Ws = W + (int64_t)s * slice_stride;
    const V *vp = reinterpret_cast<const V *>(Ws + (int64_t)k * ldw);
    const V *zp = reinterpret_cast<const V *>(Ws + (int64_t)(k + 1) * ldw);
    int64_t v0, v1;
    chunk_of(ldw / N, nblk, blockIdx.x, v0, v1);
    double acc[DOT_JT], bcc[DOT_JT];
#pragma unroll
    for (int jj = 0; jj < DOT_JT; ++jj) acc[jj] = bcc[jj] = 0.0;
    for (int64_t e = v0 + threadIdx.x; e < v1; e += blockDim.x) {
        double vv[N], zv[N];
        unpack(vp[e], vv);
        unpack(zp[e], zv);
#pragma unroll
        for (int jj = 0; jj < DOT_JT; ++jj) {
            if (jj < jn) {
                double wv[N];
                unpack(ld_stream(reinterpret_cast<const V *>(Ws + (int64_t)(j0 + jj) * ldw) + e), wv);
#pragma unroll
                for (int q = 0; q < N; ++q) {
                    acc[jj] = fma(wv[q], vv[q], acc[jj]);
                    bcc[jj] = fma(wv[q], zv[q], bcc[jj]);
                }
            }
        }
    }
    __shared__ double red[2][DOT_JT][4];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
    for (int jj = 0; jj < DOT_JT; ++jj) {
        const double ta = wave_sum(acc[jj]);
        const double tb = wave_sum(bcc[jj]);
        if (lane == 0) {
            red[0][jj][wid] = ta;
            red[1][jj][wid] = tb;
        }
    }
    __syncthreads();
    if (threadIdx.x < 2 * jn) {
        const int which = threadIdx.x / jn, jj = threadIdx.x % jn;
        double t = 0.0;
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) t += red[which][jj][w];
        part[((int64_t)s * pstride + which * boff + j0 + jj) * nblk + blockIdx.x] = t;
    }
}

// Per slice, from a and b of step k (k on the device):
//  * k >= 1: complete column k-1 of H: H[:k, k-1] += a[:k],
//    h_{k+1,k} = alpha = sqrt(v.v - |a[:k]|^2), the breakdown test against
//    ||M w_k|| = ||H[:, k-1]|| (the Arnoldi relation), 1/alpha in SC_INV;
//    k = 0: nothing to complete, alpha = 1 (w_1 is final).
//  * T[:, k] = (e_k - T[:, :k] a[:k]) / alpha: the final basis is
//    W = V T with V the vectors as they were when M was applied to them.
//  * the first pass of step k+1: with t = H[:k+1, :k] a[:k] and
//    w_{k+1}.z = (b_k - a[:k].b[:k]) / alpha,
//    h1 = ([b[:k] ; w_{k+1}.z] - t) / alpha   (column k of H, if k < K)
//    gd = t / alpha + h1                      (coefficients of the update)
__global__ __launch_bounds__(128) void dclose_k(const double *__restrict__ a, const double *__restrict__ bv,
                                                int astride, double *__restrict__ H, double *__restrict__ T,
                                                double *__restrict__ gd, int gstride, int K,
                                                double *__restrict__ sc, int *__restrict__ flags, const int *kdev,
                                                const int *active) {
    const int s = blockIdx.x;
    if (active && !active[s]) return;
    const int k = *kdev;
    const double *as = a + (int64_t)s * astride, *bs = bv + (int64_t)s * astride;
    double *Hs = H + (int64_t)s * K * (K + 1);
    double *Ts = T + (int64_t)s * K * K;
    double *S = sc + (int64_t)s * SC_COUNT;
    __shared__ double tt[KMAX_SMALL + 2];
    __shared__ double sh[2];   // alpha (0 on breakdown), w_{k+1}.z
    if (k >= 1) {
        double *col = Hs + (int64_t)(k - 1) * (K + 1);
        for (int i = threadIdx.x; i < k; i += blockDim.x) col[i] += as[i];
        __syncthreads();
        if (threadIdx.x == 0) {
            double a2 = 0.0, m2 = 0.0;
            for (int i = 0; i < k; ++i) {
                a2 = fma(as[i], as[i], a2);
                m2 = fma(col[i], col[i], m2);
            }
            const double al2 = as[k] - a2;
            const double alpha = al2 > 0.0 ? sqrt(al2) : (al2 == al2 ? 0.0 : al2);   // NaN stays NaN
            const double mw = sqrt(fma(alpha, alpha, m2));
            S[SC_MW] = mw;
            int fl = 0;
            if (!isfinite(alpha) || !isfinite(mw)) fl |= FL_NONFINITE;
            if (!(alpha > 1e-14 * mw)) {
                fl |= FL_BREAK;
                col[k] = 0.0;
                S[SC_HK] = 0.0;
                S[SC_INV] = 0.0;
                sh[0] = 0.0;
            } else {
                col[k] = alpha;
                S[SC_HK] = alpha;
                S[SC_INV] = 1.0 / alpha;
                sh[0] = alpha;
            }
            flags[s] |= fl;
        }
        __syncthreads();
    } else {
        if (threadIdx.x == 0) {
            S[SC_INV] = 1.0;
            sh[0] = 1.0;
        }
        __syncthreads();
    }
    const double alpha = sh[0];
    if (alpha == 0.0) return;   // breakdown: no next vector
    if (k < K) {
        for (int r = threadIdx.x; r <= k; r += blockDim.x) {
            double v = r == k ? 1.0 : 0.0;
            for (int i = r; i < k; ++i) v = fma(-as[i], Ts[(int64_t)i * K + r], v);
            Ts[(int64_t)k * K + r] = v / alpha;
        }
    }
    for (int r = threadIdx.x; r <= k; r += blockDim.x) {
        double t = 0.0;
        for (int l = r > 0 ? r - 1 : 0; l < k; ++l) t = fma(Hs[(int64_t)l * (K + 1) + r], as[l], t);
        tt[r] = t;
    }
    if (threadIdx.x == 0) {
        double ab = 0.0;
        for (int i = 0; i < k; ++i) ab = fma(as[i], bs[i], ab);
        sh[1] = (bs[k] - ab) / alpha;
    }
    __syncthreads();
    for (int r = threadIdx.x; r <= k; r += blockDim.x) {
        const double h1 = ((r < k ? bs[r] : sh[1]) - tt[r]) / alpha;
        gd[(int64_t)s * gstride + r] = tt[r] / alpha + h1;
        if (k < K) Hs[(int64_t)k * (K + 1) + r] = h1;
    }
}

// The update sweep of step k (slices with 1/alpha = 0 are skipped):
//   W_k     := (v - sum_{i<k} a_i W_i) / alpha                      (= w_{k+1})
//   W_{k+1} := z / alpha - sum_{i<k} gd_i W_i - gd_k w_{k+1}        (next v)
template <typename TW>
__global__ __launch_bounds__(256) void dupdate_k(TW *__restrict__ W, int64_t slice_stride, int64_t ldw,
                                                 const double *__restrict__ a, int astride,
                                                 const double *__restrict__ gd, int gstride,
                                                 const double *__restrict__ sc, int nblk, const int *kdev,
                                                 const int *active) {
    typedef typename vec16<TW>::type V;
    constexpr int N = vec16<TW>::N;
    const int s = blockIdx.z;
    if (active && !active[s]) return;
    const double inv = sc[(int64_t)s * SC_COUNT + SC_INV];
    if (inv == 0.0) return;
    const int k = kdev ? *kdev : 0;
    TW *Ws = W + (int64_t)s * slice_stride;
    V *vp = reinterpret_cast<V *>(Ws + (int64_t)k * ldw);
    V *zp = reinterpret_cast<V *>(Ws + (int64_t)(k + 1) * ldw);
    const double *as = a + (int64_t)s * astride, *gs = gd + (int64_t)s * gstride;
    const double gk = gs[k];
    int64_t v0, v1;
    chunk_of(ldw / N, nblk, blockIdx.x, v0, v1);
    for (int64_t e = v0 + threadIdx.x; e < v1; e += blockDim.x) {
        double wv[N], zv[N];
        unpack(vp[e], wv);
        unpack(zp[e], zv);
#pragma unroll
        for (int q = 0; q < N; ++q) zv[q] *= inv;
        int i = 0;
        for (; i + 4 <= k; i += 4) {
            double w0[N], w1[N], w2[N], w3[N];
            unpack(ld_stream(reinterpret_cast<const V *>(Ws + (int64_t)(i + 0) * ldw) + e), w0);
            unpack(ld_stream(reinterpret_cast<const V *>(Ws + (int64_t)(i + 1) * ldw) + e), w1);
            unpack(ld_stream(reinterpret_cast<const V *>(Ws + (int64_t)(i + 2) * ldw) + e), w2);
            unpack(ld_stream(reinterpret_cast<const V *>(Ws + (int64_t)(i + 3) * ldw) + e), w3);
            const double a0 = as[i], a1 = as[i + 1], a2 = as[i + 2], a3 = as[i + 3];
            const double g0 = gs[i], g1 = gs[i + 1], g2 = gs[i + 2], g3 = gs[i + 3];
#pragma unroll
            for (int q = 0; q < N; ++q) {
                wv[q] = fma(-a0, w0[q], wv[q]);
                zv[q] = fma(-g0, w0[q], zv[q]);
                wv[q] = fma(-a1, w1[q], wv[q]);
                zv[q] = fma(-g1, w1[q], zv[q]);
                wv[q] = fma(-a2, w2[q], wv[q]);
                zv[q] = fma(-g2, w2[q], zv[q]);
                wv[q] = fma(-a3, w3[q], wv[q]);
                zv[q] = fma(-g3, w3[q], zv[q]);
            }
        }
        for (; i < k; ++i) {
            double w0[N];
            unpack(ld_stream(reinterpret_cast<const V *>(Ws + (int64_t)i * ldw) + e), w0);
            const double a0 = as[i], g0 = gs[i];
#pragma unroll
            for (int q = 0; q < N; ++q) {
                wv[q] = fma(-a0, w0[q], wv[q]);
                zv[q] = fma(-g0, w0[q], zv[q]);
            }
        }
#pragma unroll
        for (int q = 0; q < N; ++q) {
            wv[q] *= inv;
            zv[q] = fma(-gk, wv[q], zv[q]);
        }
        vp[e] = pack<TW>(wv);
        zp[e] = pack<TW>(zv);
    }
}

// y2[s][l] = sum_{l <= i < k} T[l][i] y[i]: the coefficients of x (or of the
// data residual) in the vectors kept when M was applied to them.  k = iters
// (final assembly) or the device counter.
__global__ void ty_k(const double *__restrict__ T, const double *__restrict__ y, double *__restrict__ y2, int K,
                     const int *__restrict__ iters, const int *kdev, const int *active) {
    const int s = blockIdx.x;
    if (active && !active[s]) return;
    const int k = iters ? iters[s] : *kdev;
    const double *Ts = T + (int64_t)s * K * K;
    const double *ys = y + (int64_t)s * K;
    for (int l = threadIdx.x; l < k; l += blockDim.x) {
        double v = 0.0;
        for (int i = l; i < k; ++i) v = fma(Ts[(int64_t)i * K + l], ys[i], v);
        y2[(int64_t)s * K + l] = v;
    }
}

// ------------------------------------------------------------ launchers ---
static inline int nblk_for(int64_t nvec) {
    int64_t b = (nvec + 511) / 512;
    if (b < 1) b = 1;
    if (b > 1024) b = 1024;
    return (int)b;
}

// 16-byte vectors of each basis vector that one block of the dot-product
// sweeps handles (the partial sums depend on it, so it is fixed: a single
// slice and a batch get the same bits), and that one block of the delayed
// update sweep handles (elementwise, any value gives the same bits; long
// chunks keep more loads in flight per thread).
#ifndef ABBA_CGS_CHUNK
#define ABBA_CGS_CHUNK 4096
#endif
#ifndef ABBA_CGS_UPD_CHUNK
#define ABBA_CGS_UPD_CHUNK 4096
#endif
static int sweep_blocks(int64_t ldw, int w_dt, int64_t chunk) {
    const int64_t nvec = ldw / (w_dt == ABBA_F64 ? 2 : 4);
    const int64_t b = (nvec + chunk - 1) / chunk;
    return (int)std::min<int64_t>(1024, std::max<int64_t>(1, b));
}
int cgs_nblk(int64_t ldw, int w_dt) { return sweep_blocks(ldw, w_dt, ABBA_CGS_CHUNK); }

template <typename TW>
static int launch_dots(TW *W, const SolveDims &d, double *part, int nblk, int extra, int jtiles,
                       const int *kdev, const int *active, hipStream_t st) {
    dim3 grid(nblk, jtiles, d.S);
    hipLaunchKernelGGL(dots_k<TW>, grid, dim3(256), 0, st, (const TW *)W, (int64_t)d.wslots * d.ldw, d.ldw,
                       part, nblk, d.K + 1, extra, kdev, active);
    ABBA_LAUNCHED("dots_k");
    return ABBA_OK;
}

template <typename TW>
static int launch_update(TW *W, const SolveDims &d, const double *coef, double *npart, int nblk, bool norm,
                         const int *kdev, const int *active, hipStream_t st) {
    dim3 grid(nblk, 1, d.S);
    if (norm)
        hipLaunchKernelGGL((update_k<TW, true>), grid, dim3(256), 0, st, W, (int64_t)d.wslots * d.ldw, d.ldw,
                           coef, d.K + 1, npart, nblk, kdev, active);
    else
        hipLaunchKernelGGL((update_k<TW, false>), grid, dim3(256), 0, st, W, (int64_t)d.wslots * d.ldw, d.ldw,
                           coef, d.K + 1, npart, nblk, kdev, active);
    ABBA_LAUNCHED("update_k");
    return ABBA_OK;
}

// One CGS2 Arnoldi step on W_k for every active slice (k on the device).
template <typename TW>
static int cgs2_step_t(const SolveDims &d, const SolveWS &ws, hipStream_t st) {
    TW *W = (TW *)ws.W;
    const int nblk = cgs_nblk(d.ldw, d.w_dt);
    const int jt = (d.K + 1 + DOT_JT - 1) / DOT_JT;
    int rc;
    // pass 1: h = W_k^T q (and q.q for the breakdown reference)
    if ((rc = launch_dots<TW>(W, d, ws.part, nblk, 1, jt, ws.kdev, ws.active, st))) return rc;
    hipLaunchKernelGGL(reduce_k, dim3(d.S), dim3(256), 0, st, ws.part, nblk, d.K + 1, ws.h, d.K + 1, 1, 0,
                       ws.kdev, ws.active);
    ABBA_LAUNCHED("reduce_k");
    if ((rc = launch_update<TW>(W, d, ws.h, ws.npart, nblk, false, ws.kdev, ws.active, st))) return rc;
    // pass 2: c = W_k^T q, q -= W_k c, ||q||^2
    if ((rc = launch_dots<TW>(W, d, ws.part, nblk, 0, jt, ws.kdev, ws.active, st))) return rc;
    hipLaunchKernelGGL(reduce_k, dim3(d.S), dim3(256), 0, st, ws.part, nblk, d.K + 1, ws.c, d.K + 1, 0, 0,
                       ws.kdev, ws.active);
    ABBA_LAUNCHED("reduce_k");
    if ((rc = launch_update<TW>(W, d, ws.c, ws.npart, nblk, true, ws.kdev, ws.active, st))) return rc;
    hipLaunchKernelGGL(arnoldi_close_k, dim3(d.S), dim3(64), 0, st, ws.h, ws.c, d.K + 1, ws.npart, nblk, ws.H,
                       d.K, ws.sc, ws.flags, ws.kdev, ws.active);
    ABBA_LAUNCHED("arnoldi_close_k");
    dim3 sg(std::min<int64_t>(1024, (d.ldw / vec16<TW>::N + 255) / 256), 1, d.S);
    hipLaunchKernelGGL(scale_k<TW>, sg, dim3(256), 0, st, W, (int64_t)d.wslots * d.ldw, d.ldw, ws.sc, 0,
                       ws.kdev, ws.active);
    ABBA_LAUNCHED("scale_k");
    return ABBA_OK;
}

// One delayed-CGS2 step (both sweeps and the small per-slice algebra) on
// the vectors W_k, W_{k+1} of every active slice; `kdev` = nullptr means k = 0.
template <typename TW>
static int dcgs2_step_t(const SolveDims &d, const SolveWS &ws, const int *kdev, hipStream_t st) {
    TW *W = (TW *)ws.W;
    const int nblk = cgs_nblk(d.ldw, d.w_dt);
    const int jt = (d.K + 2 + DOT_JT - 1) / DOT_JT;
    const int boff = d.K + 2, pstride = 2 * (d.K + 2);
    const int64_t wsl = (int64_t)d.wslots * d.ldw;
    hipLaunchKernelGGL(ddots_k<TW>, dim3(nblk, jt, d.S), dim3(256), 0, st, (const TW *)W, wsl, d.ldw, ws.part, nblk,
                       pstride, boff, kdev, ws.active);
    ABBA_LAUNCHED("ddots_k");
    hipLaunchKernelGGL(reduce_k, dim3(d.S), dim3(256), 0, st, ws.part, nblk, pstride, ws.c, d.K + 2, 1, 0, kdev,
                       ws.active);
    ABBA_LAUNCHED("reduce_k");
    hipLaunchKernelGGL(reduce_k, dim3(d.S), dim3(256), 0, st, ws.part + (size_t)boff * nblk, nblk, pstride, ws.h,
                       d.K + 2, 1, 0, kdev, ws.active);
    ABBA_LAUNCHED("reduce_k");
    hipLaunchKernelGGL(dclose_k, dim3(d.S), dim3(128), 0, st, ws.c, ws.h, d.K + 2, ws.H, ws.T, ws.gd, d.K + 2, d.K,
                       ws.sc, ws.flags, kdev ? kdev : ws.kdev, ws.active);
    ABBA_LAUNCHED("dclose_k");
    // the update has no sums across elements, so its blocks per slice may
    // follow the batch (the same bits): at least 1,024 blocks in all where the
    // vectors allow, one slice alone would otherwise have 32 (one 16-byte
    // vector per thread at most)
    const int64_t nvec = d.ldw / (d.w_dt == ABBA_F64 ? 2 : 4);
    const int nblk_u = (int)std::min<int64_t>(
        std::max<int64_t>(sweep_blocks(d.ldw, d.w_dt, ABBA_CGS_UPD_CHUNK), (1024 + d.S - 1) / d.S),
        std::max<int64_t>(1, std::min<int64_t>(1024, nvec / 256)));
    hipLaunchKernelGGL(dupdate_k<TW>, dim3(nblk_u, 1, d.S), dim3(256), 0, st, W, wsl, d.ldw, (const double *)ws.c,
                       d.K + 2, (const double *)ws.gd, d.K + 2, (const double *)ws.sc, nblk_u, kdev, ws.active);
    ABBA_LAUNCHED("dupdate_k");
    return ABBA_OK;
}

int dcgs2_step(const SolveDims &d, const SolveWS &ws, const int *kdev, hipStream_t st) {
    return d.w_dt == ABBA_F64 ? dcgs2_step_t<double>(d, ws, kdev, st) : dcgs2_step_t<float>(d, ws, kdev, st);
}

int launch_ty(const SolveDims &d, const SolveWS &ws, const int *iters, const int *kdev, const int *active,
              hipStream_t st) {
    hipLaunchKernelGGL(ty_k, dim3(d.S), dim3(128), 0, st, ws.T, ws.y, ws.y2, d.K, iters, kdev, active);
    ABBA_LAUNCHED("ty_k");
    return ABBA_OK;
}

int cgs2_step(const SolveDims &d, const SolveWS &ws, hipStream_t st) {
    return d.w_dt == ABBA_F64 ? cgs2_step_t<double>(d, ws, st) : cgs2_step_t<float>(d, ws, st);
}

// beta = ||W_0||, W_0 /= beta (k fixed at 0); sets sc[SC_BETA] via init_beta_k.
__global__ void init_beta_k(const double *__restrict__ h, int hstride, double *__restrict__ sc, double *__restrict__ g,
                            int K, int *__restrict__ active, int *__restrict__ flags, int *__restrict__ iters,
                            int *__restrict__ status, const int *__restrict__ alive, int S) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= S) return;
    if (alive && !alive[s]) {   // a slice that finished in an earlier restart cycle
        sc[(int64_t)s * SC_COUNT + SC_INV] = 0.0;
        flags[s] = 0;
        iters[s] = 0;
        status[s] = 0;
        active[s] = 0;
        return;
    }
    const double b2 = h[(int64_t)s * hstride];
    const double beta = sqrt(b2);   // NaN stays NaN (no fmax: it would drop it)
    double *Sc = sc + (int64_t)s * SC_COUNT;
    Sc[SC_BETA] = beta;
    g[(int64_t)s * (K + 1)] = beta;
    flags[s] = 0;
    iters[s] = 0;
    if (!isfinite(beta)) {
        Sc[SC_INV] = 0.0;
        active[s] = 0;
        status[s] = ABBA_ST_NONFINITE;
    } else if (beta == 0.0) {
        Sc[SC_INV] = 0.0;
        active[s] = 0;
        status[s] = ABBA_ST_BREAKDOWN;
    } else {
        Sc[SC_INV] = 1.0 / beta;
        active[s] = 1;
        status[s] = 0;
    }
}

template <typename TW>
static int normalize_first_t(const SolveDims &d, const SolveWS &ws, int *iters, int *status, const int *alive,
                             hipStream_t st) {
    TW *W = (TW *)ws.W;
    const int nblk = cgs_nblk(d.ldw, d.w_dt);
    int rc;
    if ((rc = launch_dots<TW>(W, d, ws.part, nblk, 1, 1, nullptr, nullptr, st))) return rc;
    hipLaunchKernelGGL(reduce_k, dim3(d.S), dim3(64), 0, st, ws.part, nblk, d.K + 1, ws.h, d.K + 1, 1, 0,
                       nullptr, nullptr);
    ABBA_LAUNCHED("reduce_k");
    hipLaunchKernelGGL(init_beta_k, dim3((d.S + 63) / 64), dim3(64), 0, st, ws.h, d.K + 1, ws.sc, ws.g, d.K,
                       ws.active, ws.flags, iters, status, alive, d.S);
    ABBA_LAUNCHED("init_beta_k");
    dim3 sg(std::min<int64_t>(1024, (d.ldw / vec16<TW>::N + 255) / 256), 1, d.S);
    hipLaunchKernelGGL(scale_k<TW>, sg, dim3(256), 0, st, W, (int64_t)d.wslots * d.ldw, d.ldw, ws.sc, 0,
                       nullptr, ws.active);
    ABBA_LAUNCHED("scale_k");
    return ABBA_OK;
}

int normalize_first(const SolveDims &d, const SolveWS &ws, int *iters, int *status, const int *alive,
                    hipStream_t st) {
    return d.w_dt == ABBA_F64 ? normalize_first_t<double>(d, ws, iters, status, alive, st)
                              : normalize_first_t<float>(d, ws, iters, status, alive, st);
}

// out = b - ax (first `len` entries, padding zeroed); dtypes by tag.
int launch_sub(int in_dt, const void *b, int64_t bstride, const void *ax, int64_t axstride, int out_dt, void *out,
               int64_t ostride, int64_t len, int64_t ld, int S, hipStream_t st) {
    dim3 grid((unsigned)std::min<int64_t>(2048, (ld + 255) / 256), S);
#define SUBL(TS, TO) hipLaunchKernelGGL((sub_k<TS, TO>), grid, dim3(256), 0, st, (const TS *)b, bstride, \
                                        (const TS *)ax, axstride, (TO *)out, ostride, len, ld)
    if (in_dt == ABBA_F64 && out_dt == ABBA_F64) SUBL(double, double);
    else if (in_dt == ABBA_F32 && out_dt == ABBA_F32) SUBL(float, float);
    else if (in_dt == ABBA_BF16 && out_dt == ABBA_F32) SUBL(bf16, float);
    else if (in_dt == ABBA_BF16 && out_dt == ABBA_BF16) SUBL(bf16, bf16);
    else return ABBA_ERR_DTYPE;
#undef SUBL
    ABBA_LAUNCHED("sub_k");
    return ABBA_OK;
}

// out[s] = ||v_s|| (reduced in block order) into dst[s*dstride].
__global__ void finish_norm_k(const double *__restrict__ npart, int nblk, double *__restrict__ dst, int dstride,
                              int S) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= S) return;
    double t = 0.0;
    for (int b = 0; b < nblk; ++b) t += npart[(int64_t)s * nblk + b];
    dst[(int64_t)s * dstride] = sqrt(t);
}

int launch_norm(int dt, const void *v, int64_t stride, int64_t len, int S, double *npart, double *dst, int dstride,
                hipStream_t st) {
    const int nblk = nblk_for(len / 4);
    dim3 grid(nblk, S);
    if (dt == ABBA_F64) hipLaunchKernelGGL(sqnorm_k<double>, grid, dim3(256), 0, st, (const double *)v, stride, len, npart, nblk);
    else if (dt == ABBA_F32) hipLaunchKernelGGL(sqnorm_k<float>, grid, dim3(256), 0, st, (const float *)v, stride, len, npart, nblk);
    else hipLaunchKernelGGL(sqnorm_k<bf16>, grid, dim3(256), 0, st, (const bf16 *)v, stride, len, npart, nblk);
    ABBA_LAUNCHED("sqnorm_k");
    hipLaunchKernelGGL(finish_norm_k, dim3((S + 63) / 64), dim3(64), 0, st, npart, nblk, dst, dstride, S);
    ABBA_LAUNCHED("finish_norm_k");
    return ABBA_OK;
}

int launch_zero_pad(int dt, void *base, int64_t slice_stride, int nv, int64_t ld, int64_t len, int S,
                    hipStream_t st) {
    if (ld == len || nv <= 0) return ABBA_OK;
    dim3 grid((unsigned)std::min<int64_t>(1024, ((ld - len) * nv + 255) / 256), S);
    if (dt == ABBA_F64) hipLaunchKernelGGL(zero_pad_k<double>, grid, dim3(256), 0, st, (double *)base, slice_stride, nv, ld, len);
    else if (dt == ABBA_F32) hipLaunchKernelGGL(zero_pad_k<float>, grid, dim3(256), 0, st, (float *)base, slice_stride, nv, ld, len);
    else hipLaunchKernelGGL(zero_pad_k<bf16>, grid, dim3(256), 0, st, (bf16 *)base, slice_stride, nv, ld, len);
    ABBA_LAUNCHED("zero_pad_k");
    return ABBA_OK;
}

int launch_assemble(int v_dt, const void *Vb, int64_t vslice, int64_t ldv, int x_dt, void *x, int64_t n,
                    const double *y, int ystride, const int *iters, int S, hipStream_t st) {
    dim3 grid((unsigned)std::min<int64_t>(1024, (n + 255) / 256), S);
    if (v_dt == ABBA_F64 && x_dt == ABBA_F64)
        hipLaunchKernelGGL((assemble_k<double, double>), grid, dim3(256), 0, st, (double *)x, n, (const double *)Vb,
                           vslice, ldv, y, ystride, iters, n);
    else if (v_dt == ABBA_F32 && x_dt == ABBA_F32)
        hipLaunchKernelGGL((assemble_k<float, float>), grid, dim3(256), 0, st, (float *)x, n, (const float *)Vb,
                           vslice, ldv, y, ystride, iters, n);
    else
        return ABBA_ERR_DTYPE;
    ABBA_LAUNCHED("assemble_k");
    return ABBA_OK;
}

int launch_resid(int s_dt, const void *r0, int64_t rstride, const void *Z, int64_t zslice, int64_t ldz,
                 const double *y, int ystride, int64_t len, double *npart, int S, const int *kdev,
                 const int *active, hipStream_t st) {
    const int nblk = nblk_for(len / 4);
    dim3 grid(nblk, S);
    if (s_dt == ABBA_F64)
        hipLaunchKernelGGL(resid_k<double>, grid, dim3(256), 0, st, (const double *)r0, rstride, (const double *)Z,
                           zslice, ldz, y, ystride, len, npart, nblk, kdev, active);
    else if (s_dt == ABBA_F32)
        hipLaunchKernelGGL(resid_k<float>, grid, dim3(256), 0, st, (const float *)r0, rstride, (const float *)Z,
                           zslice, ldz, y, ystride, len, npart, nblk, kdev, active);
    else
        hipLaunchKernelGGL(resid_k<bf16>, grid, dim3(256), 0, st, (const bf16 *)r0, rstride, (const bf16 *)Z,
                           zslice, ldz, y, ystride, len, npart, nblk, kdev, active);
    ABBA_LAUNCHED("resid_k");
    return nblk;
}

}  // namespace abba
