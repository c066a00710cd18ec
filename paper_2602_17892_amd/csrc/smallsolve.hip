// The projected problem of hybrid AB-/BA-GMRES, one workgroup per slice, FP64.
//
// At iteration k the Arnoldi step has appended column k of the (k+1) x k
// Hessenberg matrix H_k (eq. (8)).  This kernel
//   1. extends the Givens QR of H_k by one rotation, giving R_k and
//      Q^T beta e_1 = (g, u_{k+1}); |u_{k+1}| is the GMRES residual (eq. (9));
//   2. extends the SVD R_k = U S V^T by one-sided (Hestenes) Jacobi, warm
//      started from the previous iteration: with A = R V the first k-1
//      columns of [R_{k-1} V_{k-1}, r; 0, rho] are already orthogonal;
//   3. forms uhat = U^T g and picks lambda (Sec. 3.1): none, fixed, GCV
//      (eq. (15)), the discrepancy principle, or the L-curve corner (eq. (14));
//   4. solves eq. (12): y = V diag(s/(s^2+lam^2)) uhat, and the projected
//      residual rho^2 = sum (lam^2/(s^2+lam^2))^2 uhat^2 + u_{k+1}^2.
// Both Jacobi matrices (k x k FP64) live in LDS: 2 * 100^2 * 8 B = 156 KB at
// k = 100, within gfx950's 160 KB per workgroup.
//
// Readings where the paper is silent: GCV on a 256-point log grid over
// [1e-8 s_1, s_1], global grid minimum (first index on ties), 60
// golden-section steps in log(lambda) on the neighbouring grid cells, the
// refined point kept unless it is worse; discrepancy principle by 100
// bisection steps in log(lambda) on [1e-12 s_1, 1e8 s_1]; lambda = 0 drops
// singular values below 1e-14 s_1.
#include "solve.h"

namespace abba {

constexpr int SS_THREADS = 1024;
constexpr int SS_GROUP = 16;                       // lanes per Jacobi pair
constexpr int SS_PAIRS = SS_THREADS / SS_GROUP;    // pairs in flight
constexpr int GCV_GRID = 256;
constexpr int GOLDEN_STEPS = 60;
constexpr int DP_STEPS = 100;
constexpr int MAX_SWEEPS = 30;

struct SmallArgs {
    const double *H;
    double *gc, *gs, *g, *Aj, *Vj, *y, *sig, *uh, *sc, *lamh, *rhoh;
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

constexpr int SS_NR = (KMAX_SMALL + SS_GROUP - 1) / SS_GROUP;   // column entries per lane

// The value of the partner lane inside a row of 16 lanes (a DPP row).
template <int CTRL>
__device__ __forceinline__ double dpp_peer(double v) {
    return __builtin_amdgcn_update_dpp(0.0, v, CTRL, 0xF, 0xF, false);
}

// Sum over the 16 lanes of a Jacobi group, which is one DPP row: quad
// swaps, then the half-row and row mirrors.  Each stage adds two values that
// the partner lane adds as well, so every lane ends with the same bits.
__device__ __forceinline__ double group_sum(double v) {
    static_assert(SS_GROUP == 16, "a Jacobi group is one DPP row");
    v += dpp_peer<0xB1>(v);    // quad_perm [1,0,3,2]
    v += dpp_peer<0x4E>(v);    // quad_perm [2,3,0,1]
    v += dpp_peer<0x141>(v);   // row_half_mirror
    v += dpp_peer<0x140>(v);   // row_mirror
    return v;
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

__global__ __launch_bounds__(SS_THREADS) void smallsolve_k(SmallArgs a) {
    const int s = blockIdx.x;
    if (!a.active[s]) return;
    const int k = *a.kdev;
    const int K = a.K;
    const int j = k - 1;
    const int tid = threadIdx.x;
    extern __shared__ double smem[];
    double *A = smem;                  // [K][K] column-major, column stride K
    double *V = smem + (size_t)K * K;  // [K][K]
    double *col = V + (size_t)K * K;   // [K+1]
    double *red = col + (K + 1);       // [64]
    double *xtra = red + 64;           // small-K overflow area
    __shared__ int s_rot, s_big;
    __shared__ int s_idx;
    __shared__ double s_val[4];
    __shared__ double s_uk1;

    double *Sc = a.sc + (size_t)s * SC_COUNT;
    const double *Hcol = a.H + ((size_t)s * K + j) * (K + 1);
    double *Ajs = a.Aj + (size_t)s * K * K;
    double *Vjs = a.Vj + (size_t)s * K * K;
    double *gs = a.g + (size_t)s * (K + 1);

    // ---- load warm start: A = [A_prev 0; . .], V = diag(V_prev, 1); new H column
    for (int t = tid; t < k * k; t += SS_THREADS) {
        const int c = t / k, r = t % k;
        double av = 0.0, vv = 0.0;
        if (c < j) {
            if (r < j) {
                av = Ajs[(size_t)c * K + r];
                vv = Vjs[(size_t)c * K + r];
            }
        } else {
            vv = (r == j) ? 1.0 : 0.0;
        }
        A[(size_t)c * K + r] = av;
        V[(size_t)c * K + r] = vv;
    }
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
        for (int i = 0; i <= j; ++i) A[(size_t)j * K + i] = col[i];
        // col now holds g (first k entries) for the other waves
        for (int i = 0; i < k; ++i) col[i] = gs[i];
    }
    __syncthreads();

    // ---- one-sided Jacobi on A (k x k), accumulating V
    const int grp = tid / SS_GROUP, gl = tid % SS_GROUP;
    const int n = k + (k & 1);           // even number of players (one dummy if k odd)
    // A pair whose columns are off-orthogonal by delta perturbs the singular
    // values only at O(delta^2) and the vectors at O(delta): 1e-12 is far
    // below what any consumer of y needs, and well above the rounding noise
    // of the computed inner products (which a k*eps threshold would chase).
    // One-sided Jacobi converges quadratically: after a sweep in which every
    // pair was off-orthogonal by at most sqrt(tol), what remains is O(tol),
    // so that sweep is the last one (the confirmation sweep is skipped).
    const double tol = 1e-12, tol_last = 1e-6;
    int sweeps = 0;
    for (int sweep = 0; sweep < MAX_SWEEPS && k > 1; ++sweep) {
        ++sweeps;
        if (tid == 0) s_rot = s_big = 0;
        __syncthreads();
        for (int rnd = 0; rnd < n - 1; ++rnd) {
            for (int pi = grp; pi < n / 2; pi += SS_PAIRS) {
                int p, q;
                if (pi == 0) {
                    p = n - 1;
                    q = rnd;
                } else {
                    p = (rnd + pi) % (n - 1);
                    q = (rnd - pi + n - 1) % (n - 1);
                }
                if (p >= k || q >= k) continue;
                double *ap = A + (size_t)p * K, *aq = A + (size_t)q * K;
                double *vp = V + (size_t)p * K, *vq = V + (size_t)q * K;
                // the four columns' entries of this lane, all loads in flight
                // at once (entries past k read as zero and are not stored)
                double xr[SS_NR], zr[SS_NR], vx[SS_NR], vz[SS_NR];
#pragma unroll
                for (int u = 0; u < SS_NR; ++u) {
                    const int r = gl + u * SS_GROUP;
                    const bool in = r < k;
                    xr[u] = in ? ap[r] : 0.0;
                    zr[u] = in ? aq[r] : 0.0;
                    vx[u] = in ? vp[r] : 0.0;
                    vz[u] = in ? vq[r] : 0.0;
                }
                double al = 0.0, be = 0.0, ga = 0.0;
#pragma unroll
                for (int u = 0; u < SS_NR; ++u) {
                    al = fma(xr[u], xr[u], al);
                    be = fma(zr[u], zr[u], be);
                    ga = fma(xr[u], zr[u], ga);
                }
                al = group_sum(al);
                be = group_sum(be);
                ga = group_sum(ga);
                if (al > 0.0 && be > 0.0 && fabs(ga) > tol * sqrt(al * be)) {
                    const double zeta = (be - al) / (2.0 * ga);
                    const double t = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
                    const double c = 1.0 / sqrt(1.0 + t * t);
                    const double sn = c * t;
#pragma unroll
                    for (int u = 0; u < SS_NR; ++u) {
                        const int r = gl + u * SS_GROUP;
                        if (r < k) {
                            ap[r] = c * xr[u] - sn * zr[u];
                            aq[r] = sn * xr[u] + c * zr[u];
                            vp[r] = c * vx[u] - sn * vz[u];
                            vq[r] = sn * vx[u] + c * vz[u];
                        }
                    }
                    if (gl == 0) {
                        s_rot = 1;
                        if (fabs(ga) > tol_last * sqrt(al * be)) s_big = 1;
                    }
                }
            }
            __syncthreads();
        }
        const int rot = s_rot, big = s_big;
        __syncthreads();
        if (!rot || !big) break;
    }

    // ---- sigma_i = ||A_i||, uhat_i = A_i . g / sigma_i; save the warm start
    double *sig = a.sig + (size_t)s * K;
    double *uh = a.uh + (size_t)s * K;
    for (int i = tid; i < k; i += SS_THREADS) {
        const double *ai = A + (size_t)i * K;
        double n2 = 0.0, d = 0.0;
        for (int r = 0; r < k; ++r) {
            n2 = fma(ai[r], ai[r], n2);
            d = fma(ai[r], col[r], d);
        }
        const double sgm = sqrt(n2);
        sig[i] = sgm;
        uh[i] = sgm > 0.0 ? d / sgm : 0.0;
    }
    for (int t = tid; t < k * k; t += SS_THREADS) {
        const int c = t / k, r = t % k;
        Ajs[(size_t)c * K + r] = A[(size_t)c * K + r];
        Vjs[(size_t)c * K + r] = V[(size_t)c * K + r];
    }
    __syncthreads();
    // reuse A's LDS for sigma / uhat / coefficients / grid values
    double *lsig = (K * K >= 3 * K + GCV_GRID) ? A : xtra;
    double *luh = lsig + K, *lcf = luh + K, *lgv = lcf + K;
    for (int i = tid; i < k; i += SS_THREADS) {
        lsig[i] = sig[i];
        luh[i] = uh[i];
    }
    // sigma_1
    double mx = 0.0;
    for (int i = tid; i < k; i += SS_THREADS) mx = fmax(mx, sig[i]);
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) mx = fmax(mx, __shfl_xor(mx, off, 64));
    if ((tid & 63) == 0) red[tid >> 6] = mx;
    __syncthreads();
    double s1 = 0.0;
    for (int w = 0; w < SS_THREADS / 64; ++w) s1 = fmax(s1, red[w]);
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
        for (int i = 0; i < k; ++i) acc = fma(V[(size_t)i * K + r], lcf[i], acc);
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
            Sc[SC_SWEEPS] = (double)sweeps;
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
                                               const double *__restrict__ ncpd, double ncp_thr) {
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
        else if (stop_kind == ABBA_STOP_LEARNED && sc && (double)k >= sc[(size_t)s * SC_COUNT + SC_KLEARN])
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

size_t smallsolve_lds_bytes(int K) {
    size_t extra = (size_t)K * K >= (size_t)(3 * K + GCV_GRID) ? 0 : (size_t)(3 * K + GCV_GRID);
    return sizeof(double) * (2 * (size_t)K * K + (K + 1) + 64 + extra);
}

int launch_smallsolve(const SolveDims &d, const SolveWS &ws, int rule, double lam_fixed, double tau,
                      const double *noise, hipStream_t st) {
    SmallArgs a;
    a.H = ws.H;
    a.gc = ws.gc;
    a.gs = ws.gs;
    a.g = ws.g;
    a.Aj = ws.Aj;
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
    static bool done[64] = {false};
    if (dev >= 0 && dev < 64 && done[dev]) return ABBA_OK;
    e = hipFuncSetAttribute((const void *)smallsolve_k, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)smallsolve_lds_bytes(KMAX_SMALL));
    if (e != hipSuccess) return hip_fail(e, "hipFuncSetAttribute(smallsolve_k)");
    if (dev >= 0 && dev < 64) done[dev] = true;
    return ABBA_OK;
}

int launch_stop(const SolveDims &d, const SolveWS &ws, int stop_kind, double tau, double rns_eps,
                const double *noise, int *iters, int *status, hipStream_t st) {
    hipLaunchKernelGGL(stop_k, dim3(1), dim3(1024), 0, st, d.S, d.K, stop_kind, tau, rns_eps, noise, ws.rhoh,
                       ws.active, ws.flags, iters, status, ws.kdev, ws.nact, ws.sc,
                       (d.mode == ABBA_MODE_AB || d.keepZ) ? 1 : 0, d.ncp ? ws.ncpd : nullptr,
                       d.ncp ? 1.36 / sqrt((double)(d.det / 2)) : 0.0);
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
