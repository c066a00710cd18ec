// Learned lambda / stop-index rule (not a method of the paper: an optional
// rule that keeps GCV, eq. (15), as fallback and judge and the discrepancy
// principle of Sec. 3.2 as the first stop).
//
//   features  64 per slice and iteration from sigma(H_k) and the plain GMRES
//             residual history (eq. (9)), FP64 then FP32:
//               f[i]    = log10(sigma_(i)/sigma_(1)) / 8, sorted decreasing,
//                         -16/8 past k or below 1e-16;
//               f[32+t] = log10(r_j / r_0) / 8, j = k - 31 + t, 0 for j < 1;
//   network   64 -> 128 -> 128 -> 128 -> 2, ReLU, FP32, one flat parameter
//             vector W1 [128][64], b1, W2 [128][128], b2, W3, b3, W4 [2][128], b4;
//   outputs   o0 = log10(lam/sigma_1)/8, o1 = k_stop/K;
//   judge     lam^ = sigma_1 10^(8 o0) is used when GCV(lam^) <= (1 + delta)
//             GCV(lam_GCV), else lam_GCV; stop at the first k >= K o1;
//   training  mean squared error, hand-written backward pass, Adam (Kingma
//             and Ba 2015); labels from RRE_k(lam) on a 64-point lambda grid,
//             formed from a Gram matrix of P_k = B W_k and the true image.
//
// The network kernels take 64 samples per workgroup with all activations in
// LDS; every sum runs in a fixed order, so results are bitwise reproducible.
// Per-tile weight gradients are reduced over tiles in FP64, in tile order.
#include <atomic>
#include <cmath>

#include "solve.h"

namespace abba {

constexpr int NF = 64, NH = 128, NO = 2;
constexpr int OFF_W1 = 0, OFF_B1 = OFF_W1 + NH * NF, OFF_W2 = OFF_B1 + NH, OFF_B2 = OFF_W2 + NH * NH,
              OFF_W3 = OFF_B2 + NH, OFF_B3 = OFF_W3 + NH * NH, OFF_W4 = OFF_B3 + NH, OFF_B4 = OFF_W4 + NO * NH,
              NPARAM = OFF_B4 + NO;
static_assert(NPARAM == ABBA_MLP_PARAMS, "parameter layout");
static_assert(NF == ABBA_MLP_FEATURES, "feature count");
constexpr int TILE = 64;      // samples per workgroup of the network kernels
constexpr int NT = 256;       // threads per workgroup of the network kernels
constexpr int LGRID = ABBA_LABEL_GRID;
constexpr double FSCALE = 0.125;
constexpr double PADV = -16.0;
constexpr double LOG_LAM_MIN = -12.0, LOG_LAM_MAX = 4.0;

// LDS of the forward kernel: a0 [TILE][NF], two [TILE][NH] buffers, y [TILE][NO]
constexpr size_t FWD_LDS = sizeof(float) * (TILE * NF + 2 * TILE * NH + TILE * NO);
// backward: a0, h1, h2, h3, y
constexpr size_t BWD_LDS = sizeof(float) * (TILE * NF + 3 * TILE * NH + TILE * NO);

// ------------------------------------------------------------ network ----
__device__ __forceinline__ void load_tile(const float *__restrict__ X, int nrows, const int *__restrict__ idx, int n, int base,
                          float *a0) {
    for (int e = threadIdx.x; e < TILE * NF; e += NT) {
        const int sl = e / NF, f = e % NF, i = base + sl;
        float v = 0.f;
        if (i < n) {
            const int r = idx ? idx[i] : i;
            if (r >= 0 && r < nrows) v = X[(int64_t)r * NF + f];
        }
        a0[e] = v;
    }
}

// out[s][o] = relu(b[o] + sum_i W[o][i] in[s][i]), s < TILE, o < NH; thread
// (o, half) computes 32 samples in two passes of 16, summing i in increasing
// order.
template <int NIN>
__device__ __forceinline__ void dense_relu(const float *__restrict__ W, const float *__restrict__ b, const float *in, float *out) {
    const int o = threadIdx.x & (NH - 1);
    const float bo = b[o];
    const float *Wo = W + (int64_t)o * NIN;
    for (int s0 = (threadIdx.x >> 7) * 32, e = s0 + 32; s0 < e; s0 += 16) {
        float acc[16];
#pragma unroll
        for (int q = 0; q < 16; ++q) acc[q] = bo;
        for (int i0 = 0; i0 < NIN; i0 += 16) {
            float w[16];
#pragma unroll
            for (int u = 0; u < 16; ++u) w[u] = Wo[i0 + u];
#pragma unroll
            for (int q = 0; q < 16; ++q) {
                const float *x = in + (s0 + q) * NIN + i0;
                float a = acc[q];
#pragma unroll
                for (int u = 0; u < 16; ++u) a = fmaf(w[u], x[u], a);
                acc[q] = a;
            }
        }
#pragma unroll
        for (int q = 0; q < 16; ++q) out[(s0 + q) * NH + o] = fmaxf(acc[q], 0.f);
    }
}

__device__ __forceinline__ void dense_out(const float *__restrict__ W4, const float *__restrict__ b4, const float *in, float *y) {
    if (threadIdx.x < TILE * NO) {
        const int s = threadIdx.x >> 1, o = threadIdx.x & 1;
        float acc = b4[o];
        for (int i = 0; i < NH; ++i) acc = fmaf(W4[o * NH + i], in[s * NH + i], acc);
        y[s * NO + o] = acc;
    }
}

// Forward of one tile; returns the LDS pointer of the last hidden layer.
__device__ __forceinline__ const float *forward_tile(const float *__restrict__ P, float *a0, float *hA, float *hB, float *hC,
                                     float *y) {
    dense_relu<NF>(P + OFF_W1, P + OFF_B1, a0, hA);
    __syncthreads();
    dense_relu<NH>(P + OFF_W2, P + OFF_B2, hA, hB);
    __syncthreads();
    dense_relu<NH>(P + OFF_W3, P + OFF_B3, hB, hC);
    __syncthreads();
    dense_out(P + OFF_W4, P + OFF_B4, hC, y);
    __syncthreads();
    return hC;
}

__global__ __launch_bounds__(NT) void mlp_fwd_k(const float *__restrict__ P, const float *__restrict__ X, int nrows,
                                                const int *__restrict__ idx, int n, float *__restrict__ Y) {
    extern __shared__ float lds[];
    float *a0 = lds, *hA = a0 + TILE * NF, *hB = hA + TILE * NH, *y = hB + TILE * NH;
    const int base = blockIdx.x * TILE;
    load_tile(X, nrows, idx, n, base, a0);
    __syncthreads();
    forward_tile(P, a0, hA, hB, hA, y);
    if (threadIdx.x < TILE * NO && base + (int)(threadIdx.x >> 1) < n)
        Y[(int64_t)base * NO + threadIdx.x] = y[threadIdx.x];
}

// gW[o][i] = sum_s d[s][o] a[s][i] and gb[o] = sum_s d[s][o] (s in order).
template <int NIN>
__device__ __forceinline__ void weight_grad(const float *d, const float *a, float *__restrict__ gW, float *__restrict__ gb) {
    constexpr int G = NT / NIN;           // thread groups, each over NH / G outputs
    const int i = threadIdx.x % NIN, grp = threadIdx.x / NIN;
    for (int o0 = grp * (NH / G); o0 < (grp + 1) * (NH / G); o0 += 16) {
        float acc[16];
#pragma unroll
        for (int u = 0; u < 16; ++u) acc[u] = 0.f;
        for (int s = 0; s < TILE; ++s) {
            const float av = a[s * NIN + i];
#pragma unroll
            for (int u = 0; u < 16; ++u) acc[u] = fmaf(d[s * NH + o0 + u], av, acc[u]);
        }
#pragma unroll
        for (int u = 0; u < 16; ++u) gW[(o0 + u) * NIN + i] = acc[u];
    }
    if (threadIdx.x < NH) {
        float acc = 0.f;
        for (int s = 0; s < TILE; ++s) acc += d[s * NH + threadIdx.x];
        gb[threadIdx.x] = acc;
    }
}

// a[s][i] := (sum_o W[o][i] d[s][o]) * (a[s][i] > 0), in place (o in order).
__device__ __forceinline__ void back_relu(const float *__restrict__ W, const float *d, float *a) {
    const int i = threadIdx.x & (NH - 1);
    for (int s0 = (threadIdx.x >> 7) * 32, e = s0 + 32; s0 < e; s0 += 16) {
        float acc[16];
#pragma unroll
        for (int q = 0; q < 16; ++q) acc[q] = 0.f;
        for (int o = 0; o < NH; ++o) {
            const float w = W[o * NH + i];
#pragma unroll
            for (int q = 0; q < 16; ++q) acc[q] = fmaf(w, d[(s0 + q) * NH + o], acc[q]);
        }
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            float &v = a[(s0 + q) * NH + i];
            v = v > 0.f ? acc[q] : 0.f;
        }
    }
}

// Loss and per-tile parameter gradients of L = (1/n) sum_s |net(x_s) - t_s|^2.
__global__ __launch_bounds__(NT) void mlp_bwd_k(const float *__restrict__ P, const float *__restrict__ X,
                                                const float *__restrict__ Tg, int nrows, const int *__restrict__ idx,
                                                int n, float *__restrict__ part, double *__restrict__ lpart) {
    extern __shared__ float lds[];
    float *a0 = lds, *h1 = a0 + TILE * NF, *h2 = h1 + TILE * NH, *h3 = h2 + TILE * NH, *y = h3 + TILE * NH;
    __shared__ double lred[NT / 64];
    const int base = blockIdx.x * TILE;
    load_tile(X, nrows, idx, n, base, a0);
    __syncthreads();
    forward_tile(P, a0, h1, h2, h3, y);
    // output error: d4 = 2 (y - t) / n, over the samples of this tile
    double l = 0.0;
    if (threadIdx.x < TILE * NO) {
        const int s = threadIdx.x >> 1, o = threadIdx.x & 1, i = base + s;
        float d = 0.f;
        if (i < n) {
            const int r = idx ? idx[i] : i;
            if (r >= 0 && r < nrows) {
                const float e = y[threadIdx.x] - Tg[(int64_t)r * NO + o];
                l = (double)e * (double)e;
                d = 2.f * e / (float)n;
            }
        }
        y[threadIdx.x] = d;
    }
    l = wave_sum(l);
    if ((threadIdx.x & 63) == 0) lred[threadIdx.x >> 6] = l;
    __syncthreads();
    float *g = part + (int64_t)blockIdx.x * NPARAM;
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int w = 0; w < NT / 64; ++w) t += lred[w];
        lpart[blockIdx.x] = t / (double)n;
    }
    // layer 4
    {
        const int o = threadIdx.x >> 7, i = threadIdx.x & (NH - 1);
        float acc = 0.f;
        for (int s = 0; s < TILE; ++s) acc = fmaf(y[s * NO + o], h3[s * NH + i], acc);
        g[OFF_W4 + o * NH + i] = acc;
        if (threadIdx.x < NO) {
            float b = 0.f;
            for (int s = 0; s < TILE; ++s) b += y[s * NO + threadIdx.x];
            g[OFF_B4 + threadIdx.x] = b;
        }
    }
    __syncthreads();
    const float *W4 = P + OFF_W4;
    for (int e = threadIdx.x; e < TILE * NH; e += NT) {
        const int s = e / NH, i = e % NH;
        const float v = h3[e];
        h3[e] = v > 0.f ? fmaf(W4[i], y[s * NO], W4[NH + i] * y[s * NO + 1]) : 0.f;
    }
    __syncthreads();
    weight_grad<NH>(h3, h2, g + OFF_W3, g + OFF_B3);
    __syncthreads();
    back_relu(P + OFF_W3, h3, h2);
    __syncthreads();
    weight_grad<NH>(h2, h1, g + OFF_W2, g + OFF_B2);
    __syncthreads();
    back_relu(P + OFF_W2, h2, h1);
    __syncthreads();
    weight_grad<NF>(h1, a0, g + OFF_W1, g + OFF_B1);
}

__global__ __launch_bounds__(256) void greduce_k(const float *__restrict__ part, int ntiles,
                                                 const double *__restrict__ lpart, float *__restrict__ grad,
                                                 double *__restrict__ loss) {
    const int p = blockIdx.x * 256 + threadIdx.x;
    if (p < NPARAM) {
        double acc = 0.0;
        for (int t = 0; t < ntiles; ++t) acc += (double)part[(int64_t)t * NPARAM + p];
        grad[p] = (float)acc;
    }
    if (p == 0 && loss) {
        double l = 0.0;
        for (int t = 0; t < ntiles; ++t) l += lpart[t];
        *loss = l;
    }
}

__global__ __launch_bounds__(256) void adam_k(float *__restrict__ th, const float *__restrict__ g,
                                              float *__restrict__ m, float *__restrict__ v, int n, float lr, float b1,
                                              float b2, float eps, float c1, float c2) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = fmaf(b1, m[i], (1.f - b1) * gi);
    const float vi = fmaf(b2, v[i], (1.f - b2) * gi * gi);
    m[i] = mi;
    v[i] = vi;
    th[i] -= lr * (mi * c1) / (sqrtf(vi * c2) + eps);
}

// --------------------------------------------------- solver integration ----
__global__ void gres0_k(const double *__restrict__ sc, double *__restrict__ gres, int K, int S) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s < S) gres[(int64_t)s * (K + 1)] = sc[(int64_t)s * SC_COUNT + SC_BETA];
}

__device__ __forceinline__ double clamp_log(double v) { return v < PADV ? PADV : v; }

// Features of every active slice at iteration k (after the small solve).
__global__ __launch_bounds__(128) void feat_k(const double *__restrict__ sig, const double *__restrict__ sc,
                                             double *__restrict__ gres, const double *__restrict__ noise,
                                             const double *__restrict__ rhoh, float *__restrict__ feat,
                                             float *__restrict__ fhist, int K, const int *kdev, const int *active) {
    const int s = blockIdx.x;
    if (!active[s]) return;
    const int k = *kdev;
    __shared__ double ls[KMAX_SMALL];
    __shared__ double srt[32];
    const double *sg = sig + (int64_t)s * K;
    double *gr = gres + (int64_t)s * (K + 1);
    for (int i = threadIdx.x; i < k; i += blockDim.x) ls[i] = sg[i];
    for (int i = threadIdx.x; i < 32; i += blockDim.x) srt[i] = 0.0;
    if (threadIdx.x == 0) gr[k] = sc[(int64_t)s * SC_COUNT + SC_UK1];
    __syncthreads();
    // rank sort (decreasing, ties by index); only the 32 largest are kept
    for (int i = threadIdx.x; i < k; i += blockDim.x) {
        const double v = ls[i];
        int rank = 0;
        for (int j = 0; j < k; ++j) rank += (ls[j] > v) || (ls[j] == v && j < i);
        if (rank < 32) srt[rank] = v;
    }
    __syncthreads();
    const int t = threadIdx.x;
    if (t < 64) {
        double f;
        if (t < 32) {
            const double s1 = srt[0];
            f = (t < k && s1 > 0.0 && srt[t] > 0.0) ? clamp_log(log10(srt[t] / s1)) : PADV;
        } else if (t == 32) {
            // ||e|| relative to the initial data residual, when ||e|| is given
            const double e = noise ? noise[s] : 0.0, r0 = rhoh[(int64_t)s * (K + 1)];
            f = (e > 0.0 && r0 > 0.0) ? clamp_log(log10(e / r0)) : PADV;
        } else {
            const int j = k - 31 + (t - 32);
            f = 0.0;
            if (j >= 1) f = gr[j] > 0.0 ? clamp_log(log10(gr[j] / gr[0])) : PADV;
        }
        const float fv = (float)(f * FSCALE);
        feat[(int64_t)s * NF + t] = fv;
        if (fhist) fhist[((int64_t)s * K + (k - 1)) * NF + t] = fv;
    }
}

__device__ __forceinline__ double wave_gcv(double lam, const double *sig, const double *uh, int k, double uk1) {
    const double l2 = lam * lam;
    double a = 0.0, b = 0.0;
    for (int i = threadIdx.x; i < k; i += 64) {
        const double ph = l2 / (sig[i] * sig[i] + l2);
        const double t = ph * uh[i];
        a = fma(t, t, a);
        b += ph;
    }
    a = wave_sum(a);
    b = wave_sum(b);
    const double d = 1.0 + b;
    return (a + uk1 * uk1) / (d * d);
}

// The judge (one wave per active slice): keep GCV's lambda unless the
// network's lambda^ is within (1 + delta) of the GCV minimum; record the
// predicted stop index K o1 (clamped to [1, K]).
__global__ __launch_bounds__(64) void judge_k(const float *__restrict__ pred, const double *__restrict__ sig,
                                              const double *__restrict__ uh, const double *__restrict__ Vj,
                                              double *__restrict__ y, double *__restrict__ sc,
                                              double *__restrict__ lamh, double *__restrict__ rhoh, int ab_resid,
                                              int K, double delta, const int *kdev, const int *active) {
    const int s = blockIdx.x;
    if (!active[s]) return;
    const int k = *kdev;
    const double *sg = sig + (int64_t)s * K, *u = uh + (int64_t)s * K;
    double *Sc = sc + (int64_t)s * SC_COUNT;
    double mx = 0.0;
    for (int i = threadIdx.x; i < k; i += 64) mx = fmax(mx, sg[i]);
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) mx = fmax(mx, __shfl_xor(mx, off, 64));
    const double s1 = mx;
    const double uk1 = Sc[SC_UK1];
    const double lam_g = Sc[SC_LAM];
    const double o0 = (double)pred[(int64_t)s * NO], o1 = (double)pred[(int64_t)s * NO + 1];
    const double lg = fmin(fmax(o0 / FSCALE, LOG_LAM_MIN), LOG_LAM_MAX);
    const double lam = s1 * pow(10.0, lg);
    const double g_hat = wave_gcv(lam, sg, u, k, uk1);
    const double g_gcv = wave_gcv(lam_g, sg, u, k, uk1);
    const bool ok = s1 > 0.0 && g_hat <= (1.0 + delta) * g_gcv;
    if (threadIdx.x == 0) {
        // the stop index is the largest prediction made so far: the run stops
        // once it has passed every estimate of the best iteration
        const double kn = fmin(fmax(o1 * (double)K, 1.0), (double)K);
        Sc[SC_KLEARN] = k <= 1 ? kn : fmax(Sc[SC_KLEARN], kn);
        Sc[SC_LAMLEARN] = lam;
    }
    if (!ok) return;
    __shared__ double cf[KMAX_SMALL];
    const double l2 = lam * lam;
    double part = 0.0;
    for (int i = threadIdx.x; i < k; i += 64) {
        const double d = sg[i] * sg[i] + l2;
        cf[i] = sg[i] * u[i] / d;
        const double rem = l2 / d * u[i];
        part = fma(rem, rem, part);
    }
    part = wave_sum(part);
    __syncthreads();
    const double *V = Vj + (int64_t)s * K * K;
    for (int r = threadIdx.x; r < k; r += 64) {
        double acc = 0.0;
        for (int i = 0; i < k; ++i) acc = fma(V[(int64_t)i * K + r], cf[i], acc);
        y[(int64_t)s * K + r] = acc;
    }
    if (threadIdx.x == 0) {
        const double rho = sqrt(part + uk1 * uk1);
        Sc[SC_LAM] = lam;
        Sc[SC_RHOHAT] = rho;
        lamh[(int64_t)s * K + k - 1] = lam;
        if (ab_resid) rhoh[(int64_t)s * (K + 1) + k] = rho;
    }
}

// ---------------------------------------------------------- labels (AB) ----
// ||x_true - x_0||^2 and ||x_true||^2 per slice.
template <typename T>
__global__ __launch_bounds__(256) void enorm_k(const T *__restrict__ xt, const T *__restrict__ x0, int64_t n,
                                               double *__restrict__ en) {
    const int s = blockIdx.x;
    __shared__ double red[8];
    double a = 0.0, b = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += 256) {
        const double t = (double)xt[(int64_t)s * n + i];
        const double e = t - (double)x0[(int64_t)s * n + i];
        a = fma(e, e, a);
        b = fma(t, t, b);
    }
    a = block_sum(a, red);
    b = block_sum(b, red);
    if (threadIdx.x == 0) {
        en[2 * s] = a;
        en[2 * s + 1] = b;
    }
}

// Row k-1 of the Gram matrix of P' (the kept B-images whose combination with
// coefficients z gives x - x_0) and its product with e = x_true - x_0:
// gram[s][k-1][j] = p_{k-1} . p_j (j < k), gram[s][k-1][K] = p_{k-1} . e.
template <typename T>
__global__ __launch_bounds__(256) void gram_k(const T *__restrict__ Pb, int64_t pslice, int64_t ldn,
                                              const T *__restrict__ xt, const T *__restrict__ x0, int64_t n,
                                              double *__restrict__ gram, int K, const int *kdev,
                                              const int *active) {
    const int j = blockIdx.x, s = blockIdx.y;
    if (!active[s]) return;
    const int k = *kdev;
    if (j > k) return;
    __shared__ double red[8];
    const T *pk = Pb + (int64_t)s * pslice + (int64_t)(k - 1) * ldn;
    double acc = 0.0;
    if (j < k) {
        const T *pj = Pb + (int64_t)s * pslice + (int64_t)j * ldn;
        for (int64_t i = threadIdx.x; i < n; i += 256) acc = fma((double)pk[i], (double)pj[i], acc);
    } else {
        const T *a = xt + (int64_t)s * n, *b = x0 + (int64_t)s * n;
        for (int64_t i = threadIdx.x; i < n; i += 256) acc = fma((double)pk[i], (double)a[i] - (double)b[i], acc);
    }
    acc = block_sum(acc, red);
    if (threadIdx.x == 0) gram[((int64_t)s * K + (k - 1)) * (K + 1) + (j < k ? j : K)] = acc;
}

// RRE_k(lam_g) = ||P' z_g - e|| / ||x_true|| with z_g = T y_g (delayed
// schedule) or y_g, y_g = V diag(sigma uhat / (sigma^2 + lam_g^2)):
// ||P' z - e||^2 = z'Gz - 2 z'c + ||e||^2.
__global__ __launch_bounds__(256) void rre_k(const double *__restrict__ sig, const double *__restrict__ uh,
                                             const double *__restrict__ Vj, const double *__restrict__ Tm,
                                             int delayed, const double *__restrict__ gram,
                                             const double *__restrict__ en, double *__restrict__ out, int K,
                                             const int *kdev, const int *active) {
    const int s = blockIdx.x;
    if (!active[s]) return;
    const int k = *kdev;
    __shared__ double ls[KMAX_SMALL], lu[KMAX_SMALL], cf[KMAX_SMALL], yv[KMAX_SMALL], z[KMAX_SMALL], red[8];
    const double *V = Vj + (int64_t)s * K * K, *Ts = Tm + (int64_t)s * K * K;
    const double *G = gram + (int64_t)s * K * (K + 1);
    const int t = threadIdx.x;
    for (int i = t; i < k; i += 256) {
        ls[i] = sig[(int64_t)s * K + i];
        lu[i] = uh[(int64_t)s * K + i];
    }
    __syncthreads();
    double s1 = 0.0;
    for (int i = 0; i < k; ++i) s1 = fmax(s1, ls[i]);
    const double e2 = en[2 * s], xt2 = en[2 * s + 1];
    for (int g = 0; g < LGRID; ++g) {
        const double lam = s1 * pow(10.0, -8.0 + 8.0 * (double)g / (double)(LGRID - 1));
        const double l2 = lam * lam;
        for (int i = t; i < k; i += 256) cf[i] = ls[i] * lu[i] / (ls[i] * ls[i] + l2);
        __syncthreads();
        for (int r = t; r < k; r += 256) {
            double a = 0.0;
            for (int i = 0; i < k; ++i) a = fma(V[(int64_t)i * K + r], cf[i], a);
            yv[r] = a;
        }
        __syncthreads();
        for (int l = t; l < k; l += 256) {
            double a = yv[l];
            if (delayed) {
                a = 0.0;
                for (int i = l; i < k; ++i) a = fma(Ts[(int64_t)i * K + l], yv[i], a);
            }
            z[l] = a;
        }
        __syncthreads();
        double part = 0.0;
        for (int i = t; i < k; i += 256) {
            double u = 0.0;
            for (int j = 0; j < k; ++j) {
                const int hi = i > j ? i : j, lo = i > j ? j : i;
                u = fma(G[(int64_t)hi * (K + 1) + lo], z[j], u);
            }
            part = fma(z[i], u - 2.0 * G[(int64_t)i * (K + 1) + K], part);
        }
        part = block_sum(part, red);
        if (t == 0) out[((int64_t)s * K + (k - 1)) * LGRID + g] = sqrt(fmax(part + e2, 0.0)) / sqrt(xt2);
        __syncthreads();
    }
}

// Targets of each run from its RRE grid: row k < iters holds
// ((-8 + 8 g*_k / 63) / 8, k* / K); rows past iters are NaN.
__global__ __launch_bounds__(128) void labels_k(const double *__restrict__ rre, int K, const int *__restrict__ iters,
                                               float *__restrict__ tgt, int *__restrict__ kstar) {
    const int s = blockIdx.x;
    const int it = iters ? min(max(iters[s], 0), K) : K;
    __shared__ double best[KMAX_SMALL];
    __shared__ int gbest[KMAX_SMALL];
    __shared__ int ks;
    for (int k = threadIdx.x; k < it; k += blockDim.x) {
        const double *r = rre + ((int64_t)s * K + k) * LGRID;
        double bv = r[0];
        int bg = 0;
        for (int g = 1; g < LGRID; ++g)
            if (r[g] < bv) {
                bv = r[g];
                bg = g;
            }
        best[k] = bv;
        gbest[k] = bg;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        int kb = 0;
        for (int k = 1; k < it; ++k)
            if (best[k] < best[kb]) kb = k;
        ks = it > 0 ? kb + 1 : 0;
        if (kstar) kstar[s] = ks;
    }
    __syncthreads();
    for (int k = threadIdx.x; k < K; k += blockDim.x) {
        float a = NAN, b = NAN;
        if (k < it) {
            a = (float)((-8.0 + 8.0 * (double)gbest[k] / (double)(LGRID - 1)) * FSCALE);
            b = (float)((double)ks / (double)K);
        }
        tgt[((int64_t)s * K + k) * NO] = a;
        tgt[((int64_t)s * K + k) * NO + 1] = b;
    }
}

// ------------------------------------------------------------ launchers ---
static int set_lds_attrs() {
    // host threads driving sub-batches may get here together; setting the
    // attribute twice is harmless
    static std::atomic<int> done{-1};
    int dev = 0;
    ABBA_HIP(hipGetDevice(&dev));
    if (done.load() == dev) return ABBA_OK;
    ABBA_HIP(hipFuncSetAttribute((const void *)mlp_fwd_k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)FWD_LDS));
    ABBA_HIP(hipFuncSetAttribute((const void *)mlp_bwd_k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)BWD_LDS));
    done.store(dev);
    return ABBA_OK;
}

static int launch_fwd(const float *P, const float *X, int nrows, const int *idx, int n, float *Y, hipStream_t st) {
    int rc;
    if ((rc = set_lds_attrs())) return rc;
    hipLaunchKernelGGL(mlp_fwd_k, dim3((n + TILE - 1) / TILE), dim3(NT), FWD_LDS, st, P, X, nrows, idx, n, Y);
    ABBA_LAUNCHED("mlp_fwd_k");
    return ABBA_OK;
}

int learned_prepare(const SolveDims &d, const SolveWS &ws, const void *x0, const abba_out *out, hipStream_t st) {
    int rc;
    if ((rc = set_lds_attrs())) return rc;   // before any graph capture of the iteration
    hipLaunchKernelGGL(gres0_k, dim3((d.S + 255) / 256), dim3(256), 0, st, ws.sc, ws.gres, d.K, d.S);
    ABBA_LAUNCHED("gres0_k");
    if (d.labels) {
        if (d.img_dt == ABBA_F64)
            hipLaunchKernelGGL(enorm_k<double>, dim3(d.S), dim3(256), 0, st, (const double *)out->x_true,
                               (const double *)x0, d.n, ws.enorm);
        else
            hipLaunchKernelGGL(enorm_k<float>, dim3(d.S), dim3(256), 0, st, (const float *)out->x_true,
                               (const float *)x0, d.n, ws.enorm);
        ABBA_LAUNCHED("enorm_k");
    }
    return ABBA_OK;
}

int learned_step(const SolveDims &d, const SolveWS &ws, const abba_reg *reg, int learned, const void *x0,
                 const abba_out *out, const double *noise, hipStream_t st) {
    int rc;
    hipLaunchKernelGGL(feat_k, dim3(d.S), dim3(128), 0, st, ws.sig, ws.sc, ws.gres, noise, ws.rhoh, ws.feat,
                       d.feat_out ? out->features : nullptr, d.K, ws.kdev, ws.active);
    ABBA_LAUNCHED("feat_k");
    if (learned) {
        if ((rc = launch_fwd((const float *)reg->mlp, ws.feat, d.S, nullptr, d.S, ws.pred, st))) return rc;
        hipLaunchKernelGGL(judge_k, dim3(d.S), dim3(64), 0, st, ws.pred, ws.sig, ws.uh, ws.Vj, ws.y, ws.sc, ws.lamh,
                           ws.rhoh, d.mode == ABBA_MODE_AB ? 1 : 0, d.K, reg->judge_delta, ws.kdev, ws.active);
        ABBA_LAUNCHED("judge_k");
    }
    if (d.labels) {
        dim3 grid(d.K + 1, d.S);
        if (d.img_dt == ABBA_F64)
            hipLaunchKernelGGL(gram_k<double>, grid, dim3(256), 0, st, (const double *)ws.P, (int64_t)d.pslots * d.ldn,
                               d.ldn, (const double *)out->x_true, (const double *)x0, d.n, ws.gram, d.K, ws.kdev,
                               ws.active);
        else
            hipLaunchKernelGGL(gram_k<float>, grid, dim3(256), 0, st, (const float *)ws.P, (int64_t)d.pslots * d.ldn,
                               d.ldn, (const float *)out->x_true, (const float *)x0, d.n, ws.gram, d.K, ws.kdev,
                               ws.active);
        ABBA_LAUNCHED("gram_k");
        hipLaunchKernelGGL(rre_k, dim3(d.S), dim3(256), 0, st, ws.sig, ws.uh, ws.Vj, ws.T,
                           d.ortho == ABBA_ORTHO_DELAYED ? 1 : 0, ws.gram, ws.enorm, out->rre, d.K, ws.kdev,
                           ws.active);
        ABBA_LAUNCHED("rre_k");
    }
    return ABBA_OK;
}

}  // namespace abba

using namespace abba;

extern "C" int abba_mlp_forward(const float *params, const float *X, int n, float *Y, void *stream) {
    if (n < 0 || (n > 0 && (!params || !X || !Y))) {
        set_error("abba_mlp_forward: params, X and Y are required and n >= 0");
        return ABBA_ERR_ARG;
    }
    if (n == 0) return ABBA_OK;
    return launch_fwd(params, X, n, nullptr, n, Y, (hipStream_t)stream);
}

// Per-tile partial gradients and losses of abba_mlp_loss_grad for n samples.
static size_t loss_grad_bytes(int n, size_t *pbytes) {
    const int ntiles = (n + TILE - 1) / TILE;
    *pbytes = ((size_t)ntiles * NPARAM * sizeof(float) + 255) / 256 * 256;
    return *pbytes + (size_t)ntiles * sizeof(double);
}

extern "C" int abba_mlp_loss_grad_workspace(int n, size_t *bytes) {
    if (n < 1 || !bytes) {
        set_error("abba_mlp_loss_grad_workspace: n >= 1 and bytes are required");
        return ABBA_ERR_ARG;
    }
    size_t p;
    *bytes = loss_grad_bytes(n, &p);
    return ABBA_OK;
}

extern "C" int abba_mlp_loss_grad(const float *params, const float *X, const float *T, int nrows, const int *idx,
                                  int n, float *grad, double *loss, void *workspace, size_t ws_bytes,
                                  void *stream) {
    if (!params || !X || !T || !grad || n < 1 || nrows < 1 || (!idx && n > nrows)) {
        set_error("abba_mlp_loss_grad: params, X, T, grad are required, n >= 1, and n <= nrows without idx");
        return ABBA_ERR_ARG;
    }
    size_t pbytes;
    const size_t need = loss_grad_bytes(n, &pbytes);
    if (!workspace || ws_bytes < need) {
        set_error("abba_mlp_loss_grad: workspace of %zu bytes is smaller than the %zu needed", ws_bytes, need);
        return ABBA_ERR_ARG;
    }
    int rc;
    if ((rc = set_lds_attrs())) return rc;
    hipStream_t st = (hipStream_t)stream;
    const int ntiles = (n + TILE - 1) / TILE;
    float *part = (float *)workspace;
    double *lpart = (double *)((char *)workspace + pbytes);
    hipLaunchKernelGGL(mlp_bwd_k, dim3(ntiles), dim3(NT), BWD_LDS, st, params, X, T, nrows, idx, n, part, lpart);
    ABBA_LAUNCHED("mlp_bwd_k");
    hipLaunchKernelGGL(greduce_k, dim3((NPARAM + 255) / 256), dim3(256), 0, st, part, ntiles, lpart, grad, loss);
    ABBA_LAUNCHED("greduce_k");
    return ABBA_OK;
}

extern "C" int abba_mlp_adam(float *params, const float *grad, float *m, float *v, int step, double lr, double beta1,
                             double beta2, double eps, void *stream) {
    if (!params || !grad || !m || !v || step < 1 || !(lr > 0.0) || !(beta1 >= 0.0 && beta1 < 1.0) ||
        !(beta2 >= 0.0 && beta2 < 1.0) || !(eps > 0.0)) {
        set_error("abba_mlp_adam: invalid argument");
        return ABBA_ERR_ARG;
    }
    const double c1 = 1.0 / (1.0 - std::pow(beta1, step)), c2 = 1.0 / (1.0 - std::pow(beta2, step));
    hipLaunchKernelGGL(adam_k, dim3((NPARAM + 255) / 256), dim3(256), 0, (hipStream_t)stream, params, grad, m, v,
                       NPARAM, (float)lr, (float)beta1, (float)beta2, (float)eps, (float)c1, (float)c2);
    ABBA_LAUNCHED("adam_k");
    return ABBA_OK;
}

extern "C" int abba_mlp_labels(const double *rre, int batch, int k, const int *iters, float *targets, int *k_star,
                               void *stream) {
    if (!rre || !targets || batch < 1 || k < 1 || k > KMAX_SMALL) {
        set_error("abba_mlp_labels: rre and targets are required, batch >= 1, 1 <= k <= %d", KMAX_SMALL);
        return ABBA_ERR_ARG;
    }
    hipLaunchKernelGGL(labels_k, dim3(batch), dim3(128), 0, (hipStream_t)stream, rre, k, iters, targets, k_star);
    ABBA_LAUNCHED("labels_k");
    return ABBA_OK;
}
