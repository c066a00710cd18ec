// The normalised cumulative periodogram (NCP) stopping rule (Sec. 3.2; the
// paper names it without defining it -- the definition here is Hansen's,
// "Discrete Inverse Problems", 2010).
//
// Per active slice and iteration k:
//   1. the data residual r_k = b - A x_k as a vector: in AB mode through the
//      Arnoldi relation, r_k = W_{k+1} (beta e_1 - H_k y_k); in BA mode from
//      the kept operator outputs, r_k = (b - A x_0) - Z_k y_k;
//   2. r_k read as rows of det bins (one row per detector row); the
//      periodogram of each row, P_f = |sum_d r_d e^{-2 pi i f d / det}|^2 at
//      frequencies f = 1..q, q = det / 2 (the mean left out), summed over rows;
//   3. the distance max_f |c_f - f/q| of the NCP c_f = sum_{j<=f} P_j / sum P
//      from the straight line of white noise, which the stopping kernel
//      compares with the 5 % Kolmogorov-Smirnov band 1.36 / sqrt(q).
// Each frequency of a row is evaluated by Goertzel's recurrence (FP64), one
// frequency per thread; the periodogram costs rows * q * det multiply-adds per
// slice and iteration, which the rule adds only when it is selected.
#include <algorithm>
#include <cmath>

#include "solve.h"

namespace abba {

constexpr int NCP_THREADS = 256;
constexpr int NCP_FU = 4;                       // frequencies per thread: q <= 1024

int ncp_row_chunks(int rows) { return (rows + NCP_RC - 1) / NCP_RC; }

// t = beta e_1 - H_k y_k (k+1 entries), AB mode.  Only the Hessenberg part of
// H is stored (entries below the subdiagonal are never written), so row i
// takes columns j >= i - 1.
__global__ void ncp_coef_ab_k(const double *__restrict__ H, const double *__restrict__ y,
                              const double *__restrict__ sc, double *__restrict__ t, int K, const int *kdev,
                              const int *active) {
    const int s = blockIdx.x;
    if (!active[s]) return;
    const int k = *kdev;
    const double *Hs = H + (int64_t)s * K * (K + 1);
    const double *ys = y + (int64_t)s * K;
    for (int i = threadIdx.x; i <= k; i += blockDim.x) {
        double v = i == 0 ? sc[(int64_t)s * SC_COUNT + SC_BETA] : 0.0;
        for (int j = i > 0 ? i - 1 : 0; j < k; ++j) v = fma(-Hs[(int64_t)j * (K + 1) + i], ys[j], v);
        t[(int64_t)s * (K + 1) + i] = v;
    }
}

// r = base - sum_{j<kk} c_j V_j (BA: base = b - A x_0, kk = k) or
// r = sum_{j<kk} c_j V_j (AB: base = nullptr, kk = k + 1).
template <typename TV, typename T>
__global__ __launch_bounds__(256) void ncp_resid_k(const TV *__restrict__ V, int64_t vslice, int64_t ldv,
                                                   const TV *__restrict__ base, int64_t bstride,
                                                   const double *__restrict__ c, int cstride, int extra,
                                                   T *__restrict__ r, int64_t ldr, int64_t len, const int *kdev,
                                                   const int *active) {
    const int s = blockIdx.y;
    if (!active[s]) return;
    const int kk = *kdev + extra;
    const TV *Vs = V + (int64_t)s * vslice;
    const double *cs = c + (int64_t)s * cstride;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < len; e += (int64_t)gridDim.x * blockDim.x) {
        double acc = 0.0;
        for (int j = 0; j < kk; ++j) acc = fma(cs[j], (double)load_as<TV>(Vs, (size_t)((int64_t)j * ldv + e)), acc);
        if (base) acc = (double)load_as<TV>(base, (size_t)((int64_t)s * bstride + e)) - acc;
        r[(int64_t)s * ldr + e] = (T)acc;
    }
}

// Periodogram partial sums over NCP_RC detector rows per workgroup, one
// frequency per thread, by Goertzel's recurrence in FP64:
//   s_d = r_d + c s_{d-1} - s_{d-2}, c = 2 cos(2 pi f / det),
//   |sum_d r_d e^{-2 pi i f d / det}|^2 = s_{N-1}^2 + s_{N-2}^2 - c s_{N-1} s_{N-2}
// (one multiply-add per sample and frequency; the row is read from LDS by
// all lanes at once).
template <typename T>
__global__ __launch_bounds__(NCP_THREADS) void ncp_spec_k(const T *__restrict__ r, int64_t ldr, int rows, int det,
                                                          int q, int nrch, float *__restrict__ spec,
                                                          const int *active) {
    const int s = blockIdx.y, ch = blockIdx.x;
    if (!active[s]) return;
    extern __shared__ __align__(16) unsigned char smem[];
    double *row = reinterpret_cast<double *>(smem);
    double pw[NCP_FU], cf[NCP_FU];
#pragma unroll
    for (int u = 0; u < NCP_FU; ++u) {
        const int f = (int)threadIdx.x + 1 + u * NCP_THREADS;
        pw[u] = 0.0;
        cf[u] = 2.0 * cos(2.0 * M_PI * (double)f / (double)det);
    }
    const T *rs = r + (int64_t)s * ldr;
    for (int rr = 0; rr < NCP_RC; ++rr) {
        const int a = ch * NCP_RC + rr;
        if (a >= rows) break;
        __syncthreads();   // the previous row is no longer read
        for (int d = threadIdx.x; d < det; d += NCP_THREADS) row[d] = (double)rs[(int64_t)a * det + d];
        __syncthreads();
#pragma unroll
        for (int u = 0; u < NCP_FU; ++u) {
            const int f = (int)threadIdx.x + 1 + u * NCP_THREADS;
            if (f > q) continue;
            const double c = cf[u];
            double s1 = 0.0, s2 = 0.0;
            for (int d = 0; d < det; ++d) {
                const double s0 = fma(c, s1, row[d] - s2);
                s2 = s1;
                s1 = s0;
            }
            pw[u] += fma(s1, s1, fma(s2, s2, -c * s1 * s2));
        }
    }
#pragma unroll
    for (int u = 0; u < NCP_FU; ++u) {
        const int f = (int)threadIdx.x + 1 + u * NCP_THREADS;
        if (f <= q) spec[((int64_t)s * nrch + ch) * q + (f - 1)] = (float)pw[u];
    }
}

// Distance of the NCP from the white-noise line; into ncpd[s] and the history.
__global__ __launch_bounds__(256) void ncp_dist_k(const float *__restrict__ spec, int nrch, int q,
                                                  double *__restrict__ ncpd, double *__restrict__ ncph, int K,
                                                  const int *kdev, const int *active) {
    const int s = blockIdx.x;
    if (!active[s]) return;
    const int k = *kdev;
    __shared__ double P[NCP_FU * NCP_THREADS];
    for (int f = threadIdx.x; f < q; f += blockDim.x) {
        double v = 0.0;
        for (int ch = 0; ch < nrch; ++ch) v += (double)spec[((int64_t)s * nrch + ch) * q + f];
        P[f] = v;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double tot = 0.0;
        for (int f = 0; f < q; ++f) tot += P[f];
        double dist = 0.0;
        if (tot > 0.0) {
            double c = 0.0;
            for (int f = 0; f < q; ++f) {
                c += P[f];
                dist = fmax(dist, fabs(c / tot - (double)(f + 1) / (double)q));
            }
        }
        ncpd[s] = dist;
        ncph[(int64_t)s * K + (k - 1)] = dist;
    }
}

template <typename T>
static int ncp_tail(const SolveDims &d, const SolveWS &ws, hipStream_t st) {
    const int rows = (int)(d.m / d.det), q = d.det / 2;
    const size_t lds = (size_t)d.det * sizeof(double);
    hipLaunchKernelGGL(ncp_spec_k<T>, dim3(d.nrch, d.S), dim3(NCP_THREADS), lds, st, (const T *)ws.rvec, d.ldm, rows,
                       d.det, q, d.nrch, ws.spec, ws.active);
    ABBA_LAUNCHED("ncp_spec_k");
    hipLaunchKernelGGL(ncp_dist_k, dim3(d.S), dim3(256), 0, st, ws.spec, d.nrch, q, ws.ncpd, ws.ncph, d.K, ws.kdev,
                       ws.active);
    ABBA_LAUNCHED("ncp_dist_k");
    return ABBA_OK;
}

int launch_ncp(const SolveDims &d, const SolveWS &ws, const double *coef_ba, hipStream_t st) {
    const bool f64 = d.w_dt == ABBA_F64;
    dim3 grid((unsigned)std::min<int64_t>(1024, (d.m + 255) / 256), d.S);
    if (d.mode == ABBA_MODE_AB) {
        hipLaunchKernelGGL(ncp_coef_ab_k, dim3(d.S), dim3(128), 0, st, ws.H, ws.y, ws.sc, ws.tcoef, d.K, ws.kdev,
                           ws.active);
        ABBA_LAUNCHED("ncp_coef_ab_k");
        const int64_t wsl = (int64_t)d.wslots * d.ldw;
        if (f64)
            hipLaunchKernelGGL((ncp_resid_k<double, double>), grid, dim3(256), 0, st, (const double *)ws.W, wsl, d.ldw,
                               (const double *)nullptr, (int64_t)0, ws.tcoef, d.K + 1, 1, (double *)ws.rvec, d.ldm,
                               d.m, ws.kdev, ws.active);
        else
            hipLaunchKernelGGL((ncp_resid_k<float, float>), grid, dim3(256), 0, st, (const float *)ws.W, wsl, d.ldw,
                               (const float *)nullptr, (int64_t)0, ws.tcoef, d.K + 1, 1, (float *)ws.rvec, d.ldm,
                               d.m, ws.kdev, ws.active);
    } else {
        const int64_t zsl = (int64_t)d.pslots * d.ldm;
        if (d.sino_dt == ABBA_F64)
            hipLaunchKernelGGL((ncp_resid_k<double, double>), grid, dim3(256), 0, st, (const double *)ws.Z, zsl, d.ldm,
                               (const double *)ws.sino, d.ldm, coef_ba, d.K, 0, (double *)ws.rvec, d.ldm, d.m,
                               ws.kdev, ws.active);
        else if (d.sino_dt == ABBA_F32)
            hipLaunchKernelGGL((ncp_resid_k<float, float>), grid, dim3(256), 0, st, (const float *)ws.Z, zsl, d.ldm,
                               (const float *)ws.sino, d.ldm, coef_ba, d.K, 0, (float *)ws.rvec, d.ldm, d.m, ws.kdev,
                               ws.active);
        else
            hipLaunchKernelGGL((ncp_resid_k<bf16, float>), grid, dim3(256), 0, st, (const bf16 *)ws.Z, zsl, d.ldm,
                               (const bf16 *)ws.sino, d.ldm, coef_ba, d.K, 0, (float *)ws.rvec, d.ldm, d.m, ws.kdev,
                               ws.active);
    }
    ABBA_LAUNCHED("ncp_resid_k");
    return f64 ? ncp_tail<double>(d, ws, st) : ncp_tail<float>(d, ws, st);
}

}  // namespace abba
