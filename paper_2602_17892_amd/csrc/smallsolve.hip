// The projected problem of hybrid AB-/BA-GMRES, one workgroup per slice, FP64.
//
// At iteration k the Arnoldi step has appended column k of the (k+1) x k
// Hessenberg matrix H_k (eq. (8)).  This kernel
//   1. extends the Givens QR of H_k by one rotation, giving R_k and
//      Q^T beta e_1 = (g, u_{k+1}); |u_{k+1}| is the GMRES residual (eq. (9));
//   2. updates the SVD R_{k-1} = U S V^T to R_k: with the new column
//      (r; rho) of R_k,
//        R_k = diag(U, 1) N diag(V, 1)^T,   N = [S  U^T r; 0  rho],
//      and N, with its last row and column moved first, has a full first
//      column z = (rho, U^T r) and the diagonal (0, s): N N^T = D^2 + z z^T.
//      Its singular values are the roots of the secular equation
//        1 + sum_i z_i^2 / (d_i^2 - w^2) = 0,
//      one in each gap of 0 = d_0 < d_1 <= ... < d_{k-1} and one above; its
//      singular vectors are u_j ~ (z_i / (d_i^2 - w_j^2))_i and
//      v_j ~ (-1, (d_i z_i / (d_i^2 - w_j^2))_{i>0}) (Gu and Eisenstat's
//      divide-and-conquer SVD, SIAM J. Matrix Anal. Appl. 16 (1995)).
//      Entries with z_i at rounding level, and equal d_i (after a rotation
//      that moves their z into one of them), deflate: d_i is then a
//      singular value with unit vectors.  Each root is found in the
//      variable mu - d_K^2, K the nearer pole, from a rational model with
//      the two poles of its gap (Bunch, Nielsen and Sorensen 1978) inside a
//      shrinking bracket; z is then recomputed from the roots (Loewner's
//      formula), which keeps the vectors orthogonal to working precision.
//      U_k = diag(U, 1) U_N and V_k = diag(V, 1) V_N (two k x k products),
//      uhat_k = U_N^T (uhat_{k-1}; g_k) with g = Q^T beta e_1;
//   3. picks lambda (Sec. 3.1): none, fixed, GCV (eq. (15)), the discrepancy
//      principle, or the L-curve corner (eq. (14));
//   4. solves eq. (12): y = V diag(s/(s^2+lam^2)) uhat, and the projected
//      residual rho^2 = sum (lam^2/(s^2+lam^2))^2 uhat^2 + u_{k+1}^2.
// U and V of the previous iteration stay in the workspace (k x k FP64,
// column-major, columns in descending order of s); one k x k FP64 matrix of
// the update (U_N, then V_N) lives in LDS.
//
// Readings where the paper is silent: GCV on a 256-point log grid over
// [1e-8 s_1, s_1], global grid minimum (first index on ties), 60
// golden-section steps in log(lambda) on the neighbouring grid cells, the
// refined point kept unless it is worse; discrepancy principle by 100
// bisection steps in log(lambda) on [1e-12 s_1, 1e8 s_1]; lambda = 0 drops
// singular values below 1e-14 s_1.
#include <atomic>

#include "solve.h"

namespace abba {

constexpr int SS_THREADS = 1024;
constexpr int SS_ROOT_LANES = 8;                   // lanes per secular root
constexpr int SS_ROOT_ITERS = 100;                 // bound on the root iterations
constexpr int SS_COLS = 10;                        // output columns per thread of the updates
constexpr double SS_EPS = 2.220446049250313e-16;   // 2^-52
constexpr int GCV_GRID = 256;
constexpr int GOLDEN_STEPS = 60;
constexpr int DP_STEPS = 100;

struct SmallArgs {
    const double *H;
    double *gc, *gs, *g, *Uj, *Vj, *y, *sig, *uh, *sc, *lamh, *rhoh;
    int *flags;
    int *active;
    const int *kdev;
    int K;
    int rule;
    double lam_fixed;
    double tau;
    const double *noise;     // [S] or nullptr
    int ab_resid;            // 1: rho_k = projected residual (AB mode)
};

// Sum over the 8 lanes of a root group (aligned groups of 8 lanes of a wave).
__device__ __forceinline__ double group8_sum(double v) {
    v += __shfl_xor(v, 1, 64);
    v += __shfl_xor(v, 2, 64);
    v += __shfl_xor(v, 4, 64);
    return v;
}

// 1/x to within an ulp or two: the hardware estimate and two Newton steps.
__device__ __forceinline__ double recip(double x) {
    double r = __builtin_amdgcn_rcp(x);
    double e = fma(-x, r, 1.0);
    r = fma(r, e, r);
    e = fma(-x, r, 1.0);
    return fma(r, e, r);
}

__device__ __forceinline__ double grid_lambda(double s1, int gi) {
    // s1 * 10^(-8 (1 - gi/255))
    return s1 * pow(10.0, -8.0 * (1.0 - (double)gi / (double)(GCV_GRID - 1)));
}

// rho(lam)^2 and the GCV denominator's sum, by one wave (lanes over i).
__device__ __forceinline__ void wave_filter_sums(double lam, const double *sig, const double *uh, int k,
                                                 double &num, double &den) {
    const int lane = threadIdx.x & 63;
    const double l2 = lam * lam;
    double a = 0.0, b = 0.0;
    for (int i = lane; i < k; i += 64) {
        const double s2 = sig[i] * sig[i];
        const double ph = l2 / (s2 + l2);
        const double t = ph * uh[i];
        a = fma(t, t, a);
        b += ph;
    }
    num = wave_sum(a);
    den = wave_sum(b);
}

__device__ __forceinline__ double wave_gcv(double lam, const double *sig, const double *uh, int k, double uk1) {
    double num, den;
    wave_filter_sums(lam, sig, uh, k, num, den);
    const double d = 1.0 + den;
    return (num + uk1 * uk1) / (d * d);
}

__device__ double serial_gcv(double lam, const double *sig, const double *uh, int k, double uk1) {
    const double l2 = lam * lam;
    double num = 0.0, den = 0.0;
    for (int i = 0; i < k; ++i) {
        const double s2 = sig[i] * sig[i];
        const double ph = l2 / (s2 + l2);
        const double t = ph * uh[i];
        num = fma(t, t, num);
        den += ph;
    }
    const double d = 1.0 + den;
    return (num + uk1 * uk1) / (d * d);
}

// L-curve curvature of (log rho, log ||y||) in t = ln(lambda) (closed form).
__device__ double serial_lcurve(double lam, const double *sig, const double *uh, int k, double uk1) {
    const double l2 = lam * lam;
    double R = uk1 * uk1, E = 0.0, R1 = 0.0, R2 = 0.0, E1 = 0.0, E2 = 0.0;
    for (int i = 0; i < k; ++i) {
        const double s2 = sig[i] * sig[i];
        const double phi = s2 / (s2 + l2);
        const double u2 = uh[i] * uh[i];
        const double w = u2 / (s2 + l2);
        const double om = 1.0 - phi;
        R += om * om * u2;
        E += phi * w;
        R1 += 4.0 * phi * om * om * u2;
        R2 += -8.0 * phi * om * om * (1.0 - 3.0 * phi) * u2;
        E1 += -4.0 * phi * om * w;
        E2 += 8.0 * phi * om * (2.0 - 3.0 * phi) * w;
    }
    if (R <= 0.0 || E <= 0.0) return -INFINITY;
    const double a1 = R1 / (2.0 * R), b1 = E1 / (2.0 * E);
    const double a2 = (R2 * R - R1 * R1) / (2.0 * R * R);
    const double b2 = (E2 * E - E1 * E1) / (2.0 * E * E);
    const double den = pow(a1 * a1 + b1 * b1, 1.5);
    if (den == 0.0) return -INFINITY;
    return (a1 * b2 - a2 * b1) / den;
}

// LDS of one slice's small solve (doubles): the k x k update matrix, the new
// column, reduction slots, the secular problem's vectors, and the lambda
// search's arrays; then ints.
struct SsLds {
    double *M, *col, *red, *dsec, *zsec, *dk, *zk, *tau, *zh, *nu, *nv, *sgo, *gh, *rc, *rs, *rcol;
    double *lsig, *luh, *lcf, *lgv;
    int *keep, *basek, *pos, *roti, *rotj, *defl;
};

__device__ __forceinline__ SsLds ss_lds(double *smem, int K) {
    SsLds L;
    double *p = smem;
    L.M = p; p += (size_t)K * K;
    L.col = p; p += K + 1;
    L.red = p; p += 64;
    L.dsec = p; p += K;
    L.zsec = p; p += K;
    L.dk = p; p += K;
    L.zk = p; p += K;
    L.tau = p; p += K;
    L.zh = p; p += K;
    L.nu = p; p += K;
    L.nv = p; p += K;
    L.sgo = p; p += K;
    L.gh = p; p += K;
    L.rc = p; p += K;
    L.rs = p; p += K;
    L.rcol = p; p += K;
    L.lsig = p; p += K;
    L.luh = p; p += K;
    L.lcf = p; p += K;
    L.lgv = p; p += GCV_GRID;
    int *q = reinterpret_cast<int *>(p);
    L.keep = q; q += K;
    L.basek = q; q += K;
    L.pos = q; q += K;
    L.roti = q; q += K;
    L.rotj = q; q += K;
    L.defl = q; q += K;
    return L;
}

size_t smallsolve_lds_bytes(int K) {
    return sizeof(double) * ((size_t)K * K + (K + 1) + 64 + 16 * (size_t)K + GCV_GRID) + sizeof(int) * 6 * (size_t)K;
}

// d_i^2 - w_j^2 for kept entry i and root j (w_j^2 = d_K^2 + eta_j), formed
// as (d_i - d_K)(d_i + d_K) - eta_j so that it is accurate near the pole.
__device__ __forceinline__ double sec_diff(const double *dk, int i, int K, double eta) {
    return (dk[i] - dk[K]) * (dk[i] + dk[K]) - eta;
}

__global__ __launch_bounds__(SS_THREADS) void smallsolve_k(SmallArgs a) {
    const int s = blockIdx.x;
    if (!a.active[s]) return;
    const int k = *a.kdev;
    const int K = a.K;
    const int j = k - 1;          // the new column; k - 1 old singular triplets
    const int tid = threadIdx.x;
    extern __shared__ double smem[];
    const SsLds L = ss_lds(smem, K);
    double *col = L.col;
    __shared__ int s_m, s_nd, s_nrot, s_maxit;
    __shared__ int s_idx;
    __shared__ double s_val[4];
    __shared__ double s_uk1;

    double *Sc = a.sc + (size_t)s * SC_COUNT;
    const double *Hcol = a.H + ((size_t)s * K + j) * (K + 1);
    double *Us = a.Uj + (size_t)s * K * K;    // U_{k-1}, column-major, stride K
    double *Vs = a.Vj + (size_t)s * K * K;
    double *gs = a.g + (size_t)s * (K + 1);
    double *sig = a.sig + (size_t)s * K;      // descending
    double *uh = a.uh + (size_t)s * K;

    for (int t = tid; t <= k; t += SS_THREADS) col[t] = Hcol[t];
    __syncthreads();

    // ---- Givens: previous rotations on the new column, then a new one
    if (tid == 0) {
        double *gcs = a.gc + (size_t)s * K, *gsn = a.gs + (size_t)s * K;
        for (int i = 0; i < j; ++i) {
            const double c = gcs[i], sn = gsn[i];
            const double u = col[i], v = col[i + 1];
            col[i] = c * u + sn * v;
            col[i + 1] = -sn * u + c * v;
        }
        const double p = col[j], q = col[j + 1];
        const double r = hypot(p, q);
        double c = 1.0, sn = 0.0;
        if (r != 0.0) {
            c = p / r;
            sn = q / r;
        }
        gcs[j] = c;
        gsn[j] = sn;
        col[j] = r;
        col[j + 1] = 0.0;
        const double u = gs[j];
        gs[j] = c * u;           // g[j+1] was 0
        gs[j + 1] = -sn * u;
        Sc[SC_UK1] = fabs(gs[j + 1]);
        s_uk1 = fabs(gs[j + 1]);
        // the secular problem, index 0 = the new direction, then the old
        // singular values ascending (stored descending): i <-> p = k - 1 - i
        L.zsec[0] = col[j];
        L.dsec[0] = 0.0;
        L.gh[0] = gs[j];
        for (int i = 0; i < j; ++i) L.rcol[i] = col[i];
    }
    __syncthreads();

    // ---- z = U^T r for the old directions
    for (int p = tid; p < j; p += SS_THREADS) {
        const double *up = Us + (size_t)p * K;
        double acc = 0.0;
        for (int r = 0; r < j; ++r) acc = fma(up[r], L.rcol[r], acc);
        const int i = k - 1 - p;
        L.zsec[i] = acc;
        L.dsec[i] = sig[p];
        L.gh[i] = uh[p];
    }
    __syncthreads();

    // ---- deflation (one lane): small z_i, and equal d_i rotated together
    if (tid == 0) {
        double zz = 0.0;
        for (int i = 0; i < k; ++i) zz = fma(L.zsec[i], L.zsec[i], zz);
        const double nrm = fmax(L.dsec[k - 1], sqrt(zz));
        const double tol = 8.0 * SS_EPS * nrm;
        int m = 0, nd = 0, nrot = 0;
        if (!(nrm > 0.0)) {
            // R_k = 0 (or not finite): every direction deflates
            for (int i = 0; i < k; ++i) L.defl[nd++] = i;
        } else {
            if (fabs(L.zsec[0]) <= tol) L.zsec[0] = tol;
            L.keep[m++] = 0;
        }
        for (int i = m > 0 ? 1 : k; i < k; ++i) {
            if (fabs(L.zsec[i]) <= tol) {
                L.defl[nd++] = i;
                continue;
            }
            const int jj = L.keep[m - 1];
            if (jj > 0 && L.dsec[i] - L.dsec[jj] <= tol) {
                const double r = hypot(L.zsec[i], L.zsec[jj]);
                L.rc[nrot] = L.zsec[jj] / r;
                L.rs[nrot] = L.zsec[i] / r;
                L.roti[nrot] = i;
                L.rotj[nrot] = jj;
                ++nrot;
                L.zsec[jj] = r;
                L.zsec[i] = 0.0;
                L.defl[nd++] = i;
                continue;
            }
            L.keep[m++] = i;
        }
        for (int i = 0; i < m; ++i) {
            L.dk[i] = L.dsec[L.keep[i]];
            L.zk[i] = L.zsec[L.keep[i]];
        }
        s_m = m;
        s_nd = nd;
        s_nrot = nrot;
        s_maxit = 0;
    }
    __syncthreads();
    const int m = s_m, nd = s_nd, nrot = s_nrot;

    // ---- the roots w_j^2 = d_K^2 + eta_j, eight lanes per root
    {
        double zn2 = 0.0;
        for (int i = 0; i < m; ++i) zn2 = fma(L.zk[i], L.zk[i], zn2);
        const int gl = tid & (SS_ROOT_LANES - 1);
        // the eight lanes of a root are an aligned group of a wave, so they
        // take the same branches and exchange values only among themselves
        for (int r0 = tid / SS_ROOT_LANES; r0 < m; r0 += SS_THREADS / SS_ROOT_LANES) {
            const int jr = r0;
            const bool last = jr == m - 1;
            double lo, hi;
            int Kb;
            const double Dhi = last ? L.dk[m - 1] * L.dk[m - 1] + zn2 : L.dk[jr + 1] * L.dk[jr + 1];
            if (last) {
                Kb = jr;
            } else {
                // the nearer pole: the sign of f at the middle of the gap
                const double mid = 0.5 * (L.dk[jr] * L.dk[jr] + Dhi);
                double f = 0.0;
                for (int i = gl; i < m; i += SS_ROOT_LANES) f += L.zk[i] * L.zk[i] / (L.dk[i] * L.dk[i] - mid);
                f = 1.0 + group8_sum(f);
                Kb = f > 0.0 ? jr : jr + 1;
            }
            const double dK = L.dk[Kb];
            lo = (L.dk[jr] - dK) * (L.dk[jr] + dK);
            hi = last ? (L.dk[m - 1] * L.dk[m - 1] + zn2) - dK * dK : (L.dk[jr + 1] - dK) * (L.dk[jr + 1] + dK);
            double eta = 0.5 * (lo + hi);
            int it = 0;
            for (; it < SS_ROOT_ITERS; ++it) {
                double f = 0.0, fa = 0.0, dps = 0.0, dph = 0.0;
                for (int i = gl; i < m; i += SS_ROOT_LANES) {
                    const double dm = sec_diff(L.dk, i, Kb, eta);
                    const double inv = recip(dm);
                    const double t = L.zk[i] * L.zk[i] * inv;
                    f += t;
                    fa += fabs(t);
                    const double dv = t * inv;
                    if (i <= jr) dps += dv;
                    else dph += dv;
                }
                f = 1.0 + group8_sum(f);
                fa = group8_sum(fa);
                dps = group8_sum(dps);
                dph = group8_sum(dph);
                if (f > 0.0) hi = eta;
                else lo = eta;
                if (fabs(f) <= 8.0 * SS_EPS * (1.0 + fa)) break;
                const double Dj = sec_diff(L.dk, jr, Kb, eta);
                double stp;
                if (last) {
                    const double C = f - dps * Dj;
                    stp = Dj + dps * Dj * Dj / C;
                } else {
                    const double Dj1 = sec_diff(L.dk, jr + 1, Kb, eta);
                    const double b = dps * Dj * Dj, e = dph * Dj1 * Dj1;
                    const double C = f - dps * Dj - dph * Dj1;
                    const double a1 = -(C * (Dj + Dj1) + b + e), a0 = C * Dj * Dj1 + b * Dj1 + e * Dj;
                    if (C == 0.0) {
                        stp = -a0 / a1;
                    } else {
                        const double sq = sqrt(fmax(a1 * a1 - 4.0 * C * a0, 0.0));
                        const double q = -0.5 * (a1 + copysign(sq, a1));
                        const double r1 = q / C, r2 = q != 0.0 ? a0 / q : INFINITY;
                        stp = (r1 > Dj && r1 < Dj1) ? r1 : r2;
                    }
                }
                double en = eta + stp;
                if (!(en > lo && (en < hi || (last && en == hi))) || !isfinite(en)) en = 0.5 * (lo + hi);
                if (en == eta) break;
                eta = en;
            }
            if (gl == 0) {
                L.tau[jr] = eta;
                L.basek[jr] = Kb;
                atomicMax(&s_maxit, it + 1);
            }
        }
    }
    __syncthreads();

    // ---- Loewner: zhat from the roots; then the vector norms
    for (int i = tid; i < m; i += SS_THREADS) {
        const double di = L.dk[i];
        double p = -sec_diff(L.dk, i, L.basek[m - 1], L.tau[m - 1]);   // w_{m-1}^2 - d_i^2
        for (int jj = 0; jj < i; ++jj)
            p *= -sec_diff(L.dk, i, L.basek[jj], L.tau[jj]) / ((L.dk[jj] - di) * (L.dk[jj] + di));
        for (int jj = i; jj < m - 1; ++jj)
            p *= -sec_diff(L.dk, i, L.basek[jj], L.tau[jj]) / ((L.dk[jj + 1] - di) * (L.dk[jj + 1] + di));
        L.zh[i] = copysign(sqrt(fmax(p, 0.0)), L.zk[i]);
    }
    __syncthreads();
    for (int jr = tid; jr < m; jr += SS_THREADS) {
        double su = 0.0, sv = 1.0;
        for (int i = 0; i < m; ++i) {
            const double q = L.zh[i] / sec_diff(L.dk, i, L.basek[jr], L.tau[jr]);
            su = fma(q, q, su);
            if (i > 0) sv = fma(L.dk[i] * q, L.dk[i] * q, sv);
        }
        L.nu[jr] = 1.0 / sqrt(su);
        L.nv[jr] = 1.0 / sqrt(sv);
        const double dK = L.dk[L.basek[jr]];
        L.sgo[jr] = sqrt(fma(dK, dK, L.tau[jr]));
    }
    for (int c = tid; c < nd; c += SS_THREADS) L.sgo[m + c] = L.dsec[L.defl[c]];
    __syncthreads();
    // output slot c (roots, then deflated values) -> column pos[c] in
    // descending order of the singular values (ties by slot)
    for (int c = tid; c < k; c += SS_THREADS) {
        const double v = L.sgo[c];
        int r = 0;
        for (int c2 = 0; c2 < k; ++c2) {
            const double w = L.sgo[c2];
            r += (w > v || (w == v && c2 < c)) ? 1 : 0;
        }
        L.pos[c] = r;
    }
    __syncthreads();

    // ---- U_N then V_N into L.M (row-major [secular index][column]), each
    // followed by its product with diag(U, 1) (diag(V, 1)) written in place
    for (int which = 0; which < 2; ++which) {
        const bool isu = which == 0;
        double *M = L.M;
        for (int t = tid; t < k * k; t += SS_THREADS) M[(t / k) * K + (t % k)] = 0.0;
        __syncthreads();
        for (int t = tid; t < m * m; t += SS_THREADS) {
            const int i = t / m, jr = t % m;
            const double q = L.zh[i] / sec_diff(L.dk, i, L.basek[jr], L.tau[jr]);
            double v;
            if (isu) v = q * L.nu[jr];
            else v = (i == 0 ? -1.0 : L.dk[i] * q) * L.nv[jr];
            M[(size_t)L.keep[i] * K + L.pos[jr]] = v;
        }
        for (int c = tid; c < nd; c += SS_THREADS) M[(size_t)L.defl[c] * K + L.pos[m + c]] = 1.0;
        __syncthreads();
        // the rotations of equal d_i, last one first, on the rows
        if (tid < 64) {
            for (int t = nrot - 1; t >= 0; --t) {
                const int ri = L.roti[t], rj = L.rotj[t];
                const double c = L.rc[t], sn = L.rs[t];
                for (int col2 = tid; col2 < k; col2 += 64) {
                    const double xj = M[(size_t)rj * K + col2], xi = M[(size_t)ri * K + col2];
                    M[(size_t)rj * K + col2] = c * xj - sn * xi;
                    M[(size_t)ri * K + col2] = sn * xj + c * xi;
                }
            }
        }
        __syncthreads();
        if (isu) {
            // uhat_k = U_N^T (secular-order uhat_{k-1}; g_k), and the new sigma
            for (int c = tid; c < k; c += SS_THREADS) {
                double acc = 0.0;
                for (int i = 0; i < k; ++i) acc = fma(M[(size_t)i * K + c], L.gh[i], acc);
                L.luh[c] = acc;
            }
            for (int c = tid; c < k; c += SS_THREADS) L.lsig[L.pos[c]] = L.sgo[c];
        }
        // X_new[r][c] = sum_{p<k-1} X[r][p] M[k-1-p][c] + [r == k-1] M[0][c]:
        // thread (r, column group) keeps SS_COLS sums; all reads of X happen
        // before the barrier, all writes of the new X after it
        double *X = isu ? Us : Vs;
        const int ngrp = (k + SS_COLS - 1) / SS_COLS;
        double acc[SS_COLS];
        const int r = tid % K, cg = tid / K;
        const bool mine = r < k && cg < ngrp && tid < K * ngrp;
#pragma unroll
        for (int u = 0; u < SS_COLS; ++u) acc[u] = 0.0;
        if (mine) {
            const int c0 = cg * SS_COLS;
            for (int p = 0; p < j; ++p) {
                const double xv = X[(size_t)p * K + r];
                const double *mr = M + (size_t)(k - 1 - p) * K + c0;
#pragma unroll
                for (int u = 0; u < SS_COLS; ++u)
                    if (c0 + u < k) acc[u] = fma(xv, mr[u], acc[u]);
            }
            if (r == k - 1) {
#pragma unroll
                for (int u = 0; u < SS_COLS; ++u)
                    if (c0 + u < k) acc[u] = M[c0 + u];
            }
        }
        __syncthreads();
        if (mine) {
            const int c0 = cg * SS_COLS;
#pragma unroll
            for (int u = 0; u < SS_COLS; ++u)
                if (c0 + u < k) X[(size_t)(c0 + u) * K + r] = acc[u];
        }
        __syncthreads();
    }
    for (int i = tid; i < k; i += SS_THREADS) {
        sig[i] = L.lsig[i];
        uh[i] = L.luh[i];
    }
    double *lsig = L.lsig, *luh = L.luh, *lcf = L.lcf, *lgv = L.lgv;
    // sigma_1
    const double s1 = lsig[0];
    const double uk1 = s_uk1;
    const double beta = Sc[SC_BETA];
    __syncthreads();

    // ---- lambda
    double lam = 0.0;
    const int rule = a.rule;
    if (rule == ABBA_REG_FIXED) {
        lam = a.lam_fixed;
    } else if ((rule == ABBA_REG_GCV || rule == ABBA_REG_LCURVE || rule == ABBA_REG_LEARNED) && s1 > 0.0) {
        const bool gcv = rule != ABBA_REG_LCURVE;
        if (tid < GCV_GRID) {
            const double lg = grid_lambda(s1, tid);
            lgv[tid] = gcv ? serial_gcv(lg, lsig, luh, k, uk1) : -serial_lcurve(lg, lsig, luh, k, uk1);
        }
        __syncthreads();
        if (tid < 64) {
            // argmin over 256 values, first index on ties
            double bv = INFINITY;
            int bi = GCV_GRID;
            for (int g = tid; g < GCV_GRID; g += 64) {
                const double v = lgv[g];
                if (v < bv || (v == bv && g < bi)) {
                    bv = v;
                    bi = g;
                }
            }
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) {
                const double ov = __shfl_xor(bv, off, 64);
                const int oi = __shfl_xor(bi, off, 64);
                if (ov < bv || (ov == bv && oi < bi)) {
                    bv = ov;
                    bi = oi;
                }
            }
            if (tid == 0) {
                s_idx = bi;
                s_val[0] = bv;
            }
        }
        __syncthreads();
        const int gi = s_idx;
        if (!gcv) {
            lam = grid_lambda(s1, gi);
        } else {
            if (tid < 64) {
                double lo = log(grid_lambda(s1, max(gi - 1, 0)));
                double hi = log(grid_lambda(s1, min(gi + 1, GCV_GRID - 1)));
                const double invphi = (sqrt(5.0) - 1.0) / 2.0;
                double c = hi - invphi * (hi - lo);
                double d = lo + invphi * (hi - lo);
                double fc = wave_gcv(exp(c), lsig, luh, k, uk1);
                double fd = wave_gcv(exp(d), lsig, luh, k, uk1);
                for (int it = 0; it < GOLDEN_STEPS; ++it) {
                    if (fc <= fd) {
                        hi = d;
                        d = c;
                        fd = fc;
                        c = hi - invphi * (hi - lo);
                        fc = wave_gcv(exp(c), lsig, luh, k, uk1);
                    } else {
                        lo = c;
                        c = d;
                        fc = fd;
                        d = lo + invphi * (hi - lo);
                        fd = wave_gcv(exp(d), lsig, luh, k, uk1);
                    }
                }
                double lr = exp(0.5 * (lo + hi));
                const double fr = wave_gcv(lr, lsig, luh, k, uk1);
                if (!(fr <= s_val[0])) lr = grid_lambda(s1, gi);
                if (tid == 0) s_val[1] = lr;
            }
            __syncthreads();
            lam = s_val[1];
        }
    } else if (rule == ABBA_REG_DP) {
        const double target = a.tau * (a.noise ? a.noise[s] : 0.0);
        const double t2 = target * target;
        if (uk1 * uk1 >= t2) {
            lam = 0.0;
        } else if (beta * beta <= t2 || s1 == 0.0) {
            lam = INFINITY;
        } else {
            if (tid < 64) {
                double lo = log(1e-12 * s1), hi = log(1e8 * s1);
                for (int it = 0; it < DP_STEPS; ++it) {
                    const double mid = 0.5 * (lo + hi);
                    double num, den;
                    wave_filter_sums(exp(mid), lsig, luh, k, num, den);
                    if (num + uk1 * uk1 < t2) lo = mid;
                    else hi = mid;
                }
                if (tid == 0) s_val[1] = exp(0.5 * (lo + hi));
            }
            __syncthreads();
            lam = s_val[1];
        }
    }

    // ---- coefficients, y = V coef, projected residual
    const double l2 = lam * lam;
    const bool inf = isinf(lam);
    for (int i = tid; i < k; i += SS_THREADS) {
        const double sg = lsig[i], u = luh[i];
        double cf;
        if (inf) cf = 0.0;
        else if (lam == 0.0) cf = (sg >= 1e-14 * s1 && sg > 0.0) ? u / sg : 0.0;
        else cf = sg * u / (sg * sg + l2);
        lcf[i] = cf;
    }
    __syncthreads();
    double *ys = a.y + (size_t)s * K;
    for (int r = tid; r < k; r += SS_THREADS) {
        double acc = 0.0;
        for (int i = 0; i < k; ++i) acc = fma(Vs[(size_t)i * K + r], lcf[i], acc);
        ys[r] = acc;
    }
    if (tid < 64) {
        double part = 0.0;
        for (int i = tid; i < k; i += 64) {
            const double sg = lsig[i], u = luh[i];
            double rem;
            if (inf) rem = u;
            else if (lam == 0.0) rem = (sg >= 1e-14 * s1 && sg > 0.0) ? 0.0 : u;
            else rem = l2 / (sg * sg + l2) * u;
            part = fma(rem, rem, part);
        }
        part = wave_sum(part);
        if (tid == 0) {
            const double rho = sqrt(part + uk1 * uk1);
            Sc[SC_LAM] = lam;
            Sc[SC_RHOHAT] = rho;
            Sc[SC_SWEEPS] = (double)s_maxit;
            a.lamh[(size_t)s * K + j] = lam;
            if (a.ab_resid) a.rhoh[(size_t)s * (K + 1) + k] = rho;
            if (!isfinite(rho) || !isfinite(s1)) a.flags[s] |= FL_NONFINITE;
        }
    }
}

// Stopping rules (Sec. 3.2) for every slice, then advance the iteration
// counter.  One block; also counts the slices still active.
__global__ __launch_bounds__(1024) void stop_k(int S, int K, int stop_kind, double tau, double rns_eps,
                                               const double *__restrict__ noise, const double *__restrict__ rhoh,
                                               int *__restrict__ active, const int *__restrict__ flags,
                                               int *__restrict__ iters, int *__restrict__ status,
                                               int *__restrict__ kdev, int *__restrict__ nact,
                                               const double *__restrict__ sc, int has_rho,
                                               const double *__restrict__ ncpd, double ncp_thr,
                                               double learned_gate) {
    const int k = *kdev;
    int cnt = 0;
    for (int s = threadIdx.x; s < S; s += blockDim.x) {
        if (!active[s]) continue;
        // rho_k is formed in AB mode (the projected residual) and in BA mode
        // when Z is kept; otherwise only the small solve's flags are tested
        const double rho = has_rho ? rhoh[(size_t)s * (K + 1) + k] : 0.0;
        const double rprev = has_rho ? rhoh[(size_t)s * (K + 1) + k - 1] : 0.0;
        int st = 0;
        const int fl = flags[s];
        if ((fl & FL_NONFINITE) || !isfinite(rho)) st = ABBA_ST_NONFINITE;
        else if (fl & FL_BREAK) st = ABBA_ST_BREAKDOWN;
        else if ((stop_kind == ABBA_STOP_DP || (stop_kind == ABBA_STOP_LEARNED && noise)) && rho <= tau * noise[s])
            st = ABBA_ST_STOP_DP;
        else if (stop_kind == ABBA_STOP_RNS && fabs(rprev - rho) / rprev < rns_eps) st = ABBA_ST_STOP_RNS;
        else if (stop_kind == ABBA_STOP_LEARNED && sc && (double)k >= sc[(size_t)s * SC_COUNT + SC_KLEARN] &&
                 (!(learned_gate > 0.0) || !noise || rho <= learned_gate * tau * noise[s]))
            st = ABBA_ST_STOP_LEARNED;
        else if (stop_kind == ABBA_STOP_NCP && ncpd && ncpd[s] <= ncp_thr)
            st = ABBA_ST_STOP_NCP;
        else if (k >= K) st = ABBA_ST_KMAX;
        iters[s] = k;
        if (st) {
            status[s] |= st;
            active[s] = 0;
        } else {
            ++cnt;
        }
    }
    __shared__ int red[16];
    int v = cnt;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        int t = 0;
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) t += red[w];
        *nact = t;
        *kdev = k + 1;
    }
}

// rho_k = ||b - A x_k|| from the BA residual partials, into rhoh[s][k].
__global__ void finish_resid_k(const double *__restrict__ npart, int nblk, double *__restrict__ rhoh, int K, int S,
                               const int *kdev, const int *active) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= S || !active[s]) return;
    const int k = *kdev;
    double t = 0.0;
    for (int b = 0; b < nblk; ++b) t += npart[(size_t)s * nblk + b];
    rhoh[(size_t)s * (K + 1) + k] = sqrt(t);
}


int launch_smallsolve(const SolveDims &d, const SolveWS &ws, int rule, double lam_fixed, double tau,
                      const double *noise, hipStream_t st) {
    SmallArgs a;
    a.H = ws.H;
    a.gc = ws.gc;
    a.gs = ws.gs;
    a.g = ws.g;
    a.Uj = ws.Uj;
    a.Vj = ws.Vj;
    a.y = ws.y;
    a.sig = ws.sig;
    a.uh = ws.uh;
    a.sc = ws.sc;
    a.lamh = ws.lamh;
    a.rhoh = ws.rhoh;
    a.flags = ws.flags;
    a.active = ws.active;
    a.kdev = ws.kdev;
    a.K = d.K;
    a.rule = rule;
    a.lam_fixed = lam_fixed;
    a.tau = tau;
    a.noise = noise;
    a.ab_resid = d.mode == ABBA_MODE_AB;
    const size_t lds = smallsolve_lds_bytes(d.K);
    hipLaunchKernelGGL(smallsolve_k, dim3(d.S), dim3(SS_THREADS), lds, st, a);
    ABBA_LAUNCHED("smallsolve_k");
    return ABBA_OK;
}

// Allow the small-solve kernel the dynamic LDS of the largest supported k
// (once per device; call outside stream capture).
int smallsolve_prepare() {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    static std::atomic<bool> done[64];
    if (dev >= 0 && dev < 64 && done[dev]) return ABBA_OK;
    e = hipFuncSetAttribute((const void *)smallsolve_k, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)smallsolve_lds_bytes(KMAX_SMALL));
    if (e != hipSuccess) return hip_fail(e, "hipFuncSetAttribute(smallsolve_k)");
    if (dev >= 0 && dev < 64) done[dev] = true;
    return ABBA_OK;
}

int launch_stop(const SolveDims &d, const SolveWS &ws, int stop_kind, double tau, double rns_eps,
                const double *noise, double learned_gate, int *iters, int *status, hipStream_t st) {
    hipLaunchKernelGGL(stop_k, dim3(1), dim3(1024), 0, st, d.S, d.K, stop_kind, tau, rns_eps, noise, ws.rhoh,
                       ws.active, ws.flags, iters, status, ws.kdev, ws.nact, ws.sc,
                       (d.mode == ABBA_MODE_AB || d.keepZ) ? 1 : 0, d.ncp ? ws.ncpd : nullptr,
                       d.ncp ? 1.36 / sqrt((double)(d.det / 2)) : 0.0, learned_gate);
    ABBA_LAUNCHED("stop_k");
    return ABBA_OK;
}

int launch_finish_resid(const SolveDims &d, const SolveWS &ws, int nblk, hipStream_t st) {
    hipLaunchKernelGGL(finish_resid_k, dim3((d.S + 63) / 64), dim3(64), 0, st, ws.npart, nblk, ws.rhoh, d.K, d.S,
                       ws.kdev, ws.active);
    ABBA_LAUNCHED("finish_resid_k");
    return ABBA_OK;
}

}  // namespace abba
