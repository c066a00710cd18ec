// abba_solve: hybrid AB-GMRES (Algorithm 1) and BA-GMRES (Algorithm 2) on a
// batch of independent slices.
//
// Per iteration k (one pass for all active slices, k kept on the device):
//   AB: p_k = B w_k (kept: P_k = B W_k), q = A p_k       (Alg. 1, M = AB)
//   BA: z_k = A w_k (kept when the data residual is needed), q = B z_k
//   CGS2 Arnoldi step (eq. (8)), FP64 accumulation
//   small FP64 solve per slice: Givens, SVD, lambda, y_k, rho_k (eq. (12))
//   BA only: rho_k = ||b - A x_k|| = ||(b - A x_0) - Z_k y_k||
//   stopping rules, then k := k + 1
// At the end x_k = x_0 + P_k y_k (AB; equal to x_0 + B W_k y_k, eq. (13)) or
// x_0 + W_k y_k (BA) at each slice's own stopping iteration.
//
// The per-iteration launch sequence depends on nothing but device state, so
// it can be captured once in a hipGraph and replayed.  The host reads the
// number of active slices only every `poll_every` iterations.
#include <algorithm>
#include <cstring>
#include <string>
#include <system_error>
#include <thread>
#include <vector>

#include "solve.h"

namespace abba {

int cgs2_step(const SolveDims &d, const SolveWS &ws, hipStream_t st);
int dcgs2_step(const SolveDims &d, const SolveWS &ws, const int *kdev, hipStream_t st);
int launch_ty(const SolveDims &d, const SolveWS &ws, const int *iters, const int *kdev, const int *active,
              hipStream_t st);
int normalize_first(const SolveDims &d, const SolveWS &ws, int *iters, int *status, const int *alive,
                    hipStream_t st);
int launch_sub(int in_dt, const void *b, int64_t bstride, const void *ax, int64_t axstride, int out_dt, void *out,
               int64_t ostride, int64_t len, int64_t ld, int S, hipStream_t st);
int launch_norm(int dt, const void *v, int64_t stride, int64_t len, int S, double *npart, double *dst, int dstride,
                hipStream_t st);
int launch_zero_pad(int dt, void *base, int64_t slice_stride, int nv, int64_t ld, int64_t len, int S,
                    hipStream_t st);
int launch_assemble(int v_dt, const void *Vb, int64_t vslice, int64_t ldv, int x_dt, void *x, int64_t n,
                    const double *y, int ystride, const int *iters, int S, hipStream_t st);
int launch_resid(int s_dt, const void *r0, int64_t rstride, const void *Z, int64_t zslice, int64_t ldz,
                 const double *y, int ystride, int64_t len, double *npart, int S, const int *kdev,
                 const int *active, hipStream_t st);
int launch_smallsolve(const SolveDims &d, const SolveWS &ws, int rule, double lam_fixed, double tau,
                      const double *noise, hipStream_t st);
int launch_stop(const SolveDims &d, const SolveWS &ws, int stop_kind, double tau, double rns_eps,
                const double *noise, double learned_gate, int *iters, int *status, hipStream_t st);
int launch_finish_resid(const SolveDims &d, const SolveWS &ws, int nblk, hipStream_t st);
int smallsolve_prepare();
int learned_prepare(const SolveDims &d, const SolveWS &ws, const void *x0, const abba_out *out, hipStream_t st);
int launch_ncp(const SolveDims &d, const SolveWS &ws, const double *coef_ba, hipStream_t st);
int learned_step(const SolveDims &d, const SolveWS &ws, const abba_reg *reg, int learned, const void *x0,
                 const abba_out *out, const double *noise, hipStream_t st);

static inline int64_t round_up(int64_t v, int64_t a) { return (v + a - 1) / a * a; }

// Stream-time accounting of the phases of a solve (exec.phase_ms): an event
// is recorded at every phase change; interval i runs from event i to event
// i + 1 and belongs to phase ph[i].
struct PhaseClock {
    hipStream_t st = nullptr;
    std::vector<hipEvent_t> ev;
    std::vector<int> ph;
    int mark(int phase) {
        hipEvent_t e;
        hipError_t r = hipEventCreate(&e);
        if (r != hipSuccess) return hip_fail(r, "hipEventCreate");
        ev.push_back(e);
        ph.push_back(phase);
        r = hipEventRecord(e, st);
        if (r != hipSuccess) return hip_fail(r, "hipEventRecord");
        return ABBA_OK;
    }
    // Synchronise and add each interval's time to ms[phase].
    int finish(double *ms) {
        int rc = mark(-1);
        if (!rc) {
            hipError_t r = hipEventSynchronize(ev.back());
            if (r != hipSuccess) rc = hip_fail(r, "hipEventSynchronize");
        }
        for (size_t i = 0; !rc && i + 1 < ev.size(); ++i) {
            if (ph[i] < 0) continue;
            float t = 0.f;
            hipError_t r = hipEventElapsedTime(&t, ev[i], ev[i + 1]);
            if (r != hipSuccess) rc = hip_fail(r, "hipEventElapsedTime");
            else ms[ph[i]] += t;
        }
        release();
        return rc;
    }
    void release() {
        for (hipEvent_t e : ev) (void)hipEventDestroy(e);
        ev.clear();
        ph.clear();
    }
    ~PhaseClock() { release(); }
};

static inline int clock_mark(PhaseClock *c, int phase) { return c ? c->mark(phase) : ABBA_OK; }

// Scratch the operators of one solve need for `batch` slices.
static size_t op_scratch_bytes(const abba_op *A, const abba_op *B, int batch) {
    size_t b = 0;
    for (const abba_op *op : {A, B})
        b = std::max(b, cone_path(op) ? cone_scratch_bytes(op, batch) : par2d_scratch_bytes(op, batch));
    return b;
}

size_t solve_workspace_bytes(const SolveDims &d, SolveWS *ws, void *base, size_t scratch_bytes) {
    const size_t wsz = dtype_size(d.w_dt), isz = dtype_size(d.img_dt), ssz = dtype_size(d.sino_dt);
    const size_t S = d.S, K = d.K;
    size_t off = 0;
    auto take = [&](size_t bytes) -> void * {
        void *p = base ? (char *)base + off : nullptr;
        off += (bytes + 255) / 256 * 256;
        return p;
    };
    SolveWS w;
    std::memset(&w, 0, sizeof(w));
    w.W = take(S * d.wslots * d.ldw * wsz);
    w.P = d.mode == ABBA_MODE_AB ? take(S * d.pslots * d.ldn * isz) : nullptr;
    w.Z = d.mode == ABBA_MODE_BA ? take(S * (d.keepZ ? d.pslots : 1) * d.ldm * ssz) : nullptr;
    w.sino = take(S * d.ldm * ssz);
    w.scratch = take(scratch_bytes);
    w.part = (double *)take(S * 1024 * 2 * (K + 2) * 8);
    w.h = (double *)take(S * (K + 2) * 8);
    w.c = (double *)take(S * (K + 2) * 8);
    w.npart = (double *)take(S * 1024 * 8);
    w.H = (double *)take(S * K * (K + 1) * 8);
    w.gc = (double *)take(S * K * 8);
    w.gs = (double *)take(S * K * 8);
    w.g = (double *)take(S * (K + 1) * 8);
    w.Uj = (double *)take(S * K * K * 8);
    w.Vj = (double *)take(S * K * K * 8);
    w.y = (double *)take(S * K * 8);
    w.y2 = (double *)take(S * K * 8);
    w.T = (double *)take(S * K * K * 8);
    w.gd = (double *)take(S * (K + 2) * 8);
    w.sig = (double *)take(S * K * 8);
    w.uh = (double *)take(S * K * 8);
    w.sc = (double *)take(S * SC_COUNT * 8);
    w.lamh = (double *)take(S * K * 8);
    w.rhoh = (double *)take(S * (K + 1) * 8);
    w.feat = (float *)take(S * 64 * 4);
    w.pred = (float *)take(S * 2 * 4);
    w.gres = (double *)take(S * (K + 1) * 8);
    w.gram = d.labels ? (double *)take(S * K * (K + 1) * 8) : nullptr;
    w.enorm = d.labels ? (double *)take(S * 2 * 8) : nullptr;
    if (d.ncp) {
        w.rvec = take(S * d.ldm * (d.w_dt == ABBA_F64 ? 8 : 4));
        w.tcoef = (double *)take(S * (K + 1) * 8);
        w.spec = (float *)take(S * d.nrch * (d.det / 2) * 4);
        w.ncpd = (double *)take(S * 8);
        w.ncph = (double *)take(S * K * 8);
    }
    w.citers = (int *)take(S * 4);
    w.cstatus = (int *)take(S * 4);
    w.alive = (int *)take(S * 4);
    w.active = (int *)take(S * 4);
    w.flags = (int *)take(S * 4);
    w.kdev = (int *)take(4);
    w.nact = (int *)take(4);
    if (ws) *ws = w;
    return off;
}

static int make_dims(const abba_op *A, const abba_op *B, int batch, int mode, int k, const abba_stop *stop,
                     const abba_out *out, SolveDims *d) {
    if (!A || !B) {
        set_error("A or B is NULL");
        return ABBA_ERR_ARG;
    }
    if (A->kind != ABBA_OP_JOSEPH || (B->kind != ABBA_OP_PIXEL && B->kind != ABBA_OP_JOSEPH_T)) {
        set_error("A must be ABBA_OP_JOSEPH and B ABBA_OP_PIXEL or ABBA_OP_JOSEPH_T");
        return ABBA_ERR_ARG;
    }
    if (A->n != B->n || A->m != B->m || A->g.kind != B->g.kind) {
        set_error("A is R^%lld -> R^%lld but B is R^%lld -> R^%lld", (long long)A->n, (long long)A->m,
                  (long long)B->m, (long long)B->n);
        return ABBA_ERR_SHAPE;
    }
    if (A->img_dtype != B->img_dtype || A->sino_dtype != B->sino_dtype) {
        set_error("A and B must use the same dtypes");
        return ABBA_ERR_DTYPE;
    }
    if (batch < 1) {
        set_error("batch must be >= 1");
        return ABBA_ERR_ARG;
    }
    if (mode != ABBA_MODE_AB && mode != ABBA_MODE_BA) {
        set_error("unknown mode %d", mode);
        return ABBA_ERR_ARG;
    }
    const int64_t kmax = A->n < A->m ? A->n : A->m;
    if (k < 1 || (int64_t)k > kmax) {
        set_error("k = %d outside [1, min(m, n) = %lld]", k, (long long)kmax);
        return ABBA_ERR_ARG;
    }
    if (k > KMAX_SMALL) {
        set_error("k = %d exceeds the small-solve limit %d (use restarts)", k, KMAX_SMALL);
        return ABBA_ERR_UNSUPPORTED;
    }
    std::memset(d, 0, sizeof(*d));
    d->S = batch;
    d->K = k;
    d->mode = mode;
    d->n = A->n;
    d->m = A->m;
    d->len = mode == ABBA_MODE_AB ? A->m : A->n;
    d->ldw = round_up(d->len, 256);
    d->ldn = round_up(A->n, 256);
    d->ldm = round_up(A->m, 256);
    d->img_dt = A->img_dtype;
    d->sino_dt = A->sino_dtype;
    d->w_dt = A->img_dtype == ABBA_F64 ? ABBA_F64 : ABBA_F32;
    const bool stop_rule = stop && stop->kind != ABBA_STOP_NONE;
    d->keepZ = mode == ABBA_MODE_BA && (stop_rule || (out && out->resid));
    d->wslots = k + 2;
    d->pslots = k + 1;
    d->ortho = ABBA_ORTHO_DELAYED;
    if (stop && stop->kind == ABBA_STOP_NCP) {
        const int det = A->g.det_u;
        if (det < 2 || det > NCP_MAX_DET || A->m % det) {
            set_error("the NCP rule reads rows of 2..%d detector bins (det_u = %d)", NCP_MAX_DET, det);
            return ABBA_ERR_UNSUPPORTED;
        }
        d->ncp = 1;
        d->det = det;
        d->nrch = ncp_row_chunks((int)(A->m / det));
    }
    return ABBA_OK;
}

__global__ void set_int_k(int *p, int v) { *p = v; }

__global__ void fill_k(double *__restrict__ p, int64_t n, double v) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

static int apply_op(const abba_op *op, bool forward, VecRef in, int in_dt, VecRef out, int out_dt,
                    const SolveDims &d, const SolveWS &ws, const Launch &L, PhaseClock *clk) {
    int rc = clock_mark(clk, forward ? ABBA_PHASE_A : ABBA_PHASE_B);
    if (rc) return rc;
    if (forward)
        rc = cone_path(op) ? cone_forward(op, in, out, out_dt, d.S, ws.scratch, L)
                           : par2d_forward(op, in, out, out_dt, d.S, ws.scratch, L);
    else
        rc = cone_path(op) ? cone_back(op, in, in_dt, out, d.S, ws.scratch, L)
                           : par2d_back(op, in, in_dt, out, d.S, ws.scratch, L);
    if (rc) return rc;
    return clock_mark(clk, ABBA_PHASE_OTHER);
}

struct IterCfg {
    const abba_op *A, *B;
    int rule;
    double lam_fixed, tau;
    const double *noise_reg;
    int stop_kind;
    double stop_tau, rns_eps;
    const double *noise_stop;
    double learned_gate;
    int *iters, *status;
    int learned;
    const abba_reg *reg;
    const abba_out *out;
    const void *x0;
    PhaseClock *clk;     // exec.phase_ms accounting, or nullptr
};

// The operator step of iteration k: q = M (input vector) into W, keeping
// the intermediate (AB: B w in P, BA: A w in Z).  Two-pass CGS2 applies M to
// the final w_k = W_{k-1} and writes W_k; the delayed schedule applies it to
// the once-orthogonalised W_k and writes W_{k+1}.
static int apply_M(const SolveDims &d, const SolveWS &ws, const IterCfg &c, const Launch &L) {
    const bool delayed = d.ortho == ABBA_ORTHO_DELAYED;
    const int in_off = delayed ? 0 : -1, out_off = delayed ? 1 : 0;
    const int64_t wsl = (int64_t)d.wslots * d.ldw;
    VecRef win{ws.W, wsl, d.ldw, in_off};
    VecRef wout{ws.W, wsl, d.ldw, out_off};
    int rc;
    if (d.mode == ABBA_MODE_AB) {
        VecRef p{ws.P, (int64_t)d.pslots * d.ldn, d.ldn, in_off};
        if ((rc = apply_op(c.B, false, win, d.w_dt, p, d.img_dt, d, ws, L, c.clk))) return rc;
        return apply_op(c.A, true, p, d.img_dt, wout, d.w_dt, d, ws, L, c.clk);
    }
    VecRef z{ws.Z, (int64_t)(d.keepZ ? d.pslots : 1) * d.ldm, d.keepZ ? d.ldm : 0, d.keepZ ? in_off : 0};
    if ((rc = apply_op(c.A, true, win, d.w_dt, z, d.sino_dt, d, ws, L, c.clk))) return rc;
    return apply_op(c.B, false, z, d.sino_dt, wout, d.w_dt, d, ws, L, c.clk);
}

// Launch one iteration for all active slices on `st`.
static int one_iteration(const SolveDims &d, const SolveWS &ws, const IterCfg &c, hipStream_t st) {
    Launch L{st, ws.kdev, ws.active};
    const bool delayed = d.ortho == ABBA_ORTHO_DELAYED;
    int rc;
    if ((rc = apply_M(d, ws, c, L))) return rc;
    if ((rc = clock_mark(c.clk, ABBA_PHASE_ORTHO))) return rc;
    if ((rc = delayed ? dcgs2_step(d, ws, ws.kdev, st) : cgs2_step(d, ws, st))) return rc;
    if ((rc = clock_mark(c.clk, ABBA_PHASE_SMALL))) return rc;
    if ((rc = launch_smallsolve(d, ws, c.rule, c.lam_fixed, c.tau, c.noise_reg, st))) return rc;
    if (c.learned || d.feat_out || d.labels) {
        if ((rc = learned_step(d, ws, c.reg, c.learned, c.x0, c.out, c.noise_stop ? c.noise_stop : c.noise_reg,
                               st)))
            return rc;
    }
    const double *yk = ws.y;
    if (d.mode == ABBA_MODE_BA && d.keepZ) {
        // rho_k = ||(b - A x_0) - Z_k y_k||; with the delayed schedule Z holds
        // A applied to the vectors before their second pass: Z_k y = Z' (T y)
        if (delayed) {
            if ((rc = launch_ty(d, ws, nullptr, ws.kdev, ws.active, st))) return rc;
            yk = ws.y2;
        }
        const int nb = launch_resid(d.sino_dt, ws.sino, d.ldm, ws.Z, (int64_t)d.pslots * d.ldm, d.ldm, yk, d.K, d.m,
                                    ws.npart, d.S, ws.kdev, ws.active, st);
        if (nb < 0) return nb;
        if ((rc = launch_finish_resid(d, ws, nb, st))) return rc;
    }
    if (d.ncp && (rc = launch_ncp(d, ws, yk, st))) return rc;
    if ((rc = launch_stop(d, ws, c.stop_kind, c.stop_tau, c.rns_eps, c.noise_stop, c.learned_gate, c.iters,
                          c.status, st)))
        return rc;
    return clock_mark(c.clk, ABBA_PHASE_OTHER);
}

__global__ void cycle_begin_k(int *__restrict__ alive, int *__restrict__ iters, int *__restrict__ status, int S) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= S) return;
    alive[s] = 1;
    iters[s] = 0;
    status[s] = 0;
}

// End of a restart cycle that started `done` iterations in (one block):
// every slice that took part adds its cycle's iteration count and histories
// to the run's; it goes on to the next cycle if no rule ended the cycle and
// iterations are left, else its status becomes final.  *nalive receives the
// number of slices that go on.
__global__ __launch_bounds__(1024) void cycle_end_k(int *__restrict__ alive, const int *__restrict__ citers,
                                                    const int *__restrict__ cstatus, const double *__restrict__ lamh,
                                                    const double *__restrict__ rhoh, const double *__restrict__ ncph,
                                                    int K, int *__restrict__ iters, int *__restrict__ status,
                                                    double *__restrict__ out_lam, double *__restrict__ out_rho,
                                                    double *__restrict__ out_ncp, int ktot, int done,
                                                    int *__restrict__ nalive, int S) {
    int cnt = 0;
    for (int s = threadIdx.x; s < S; s += blockDim.x) {
        if (!alive[s]) continue;
        const int kc = citers[s], st = cstatus[s];
        if (out_lam)
            for (int j = 0; j < kc; ++j) out_lam[(int64_t)s * ktot + done + j] = lamh[(int64_t)s * K + j];
        if (out_ncp && ncph)
            for (int j = 0; j < kc; ++j) out_ncp[(int64_t)s * ktot + done + j] = ncph[(int64_t)s * K + j];
        if (out_rho) {
            if (done == 0) out_rho[(int64_t)s * (ktot + 1)] = rhoh[(int64_t)s * (K + 1)];
            for (int j = 1; j <= kc; ++j)
                out_rho[(int64_t)s * (ktot + 1) + done + j] = rhoh[(int64_t)s * (K + 1) + j];
        }
        iters[s] = done + kc;
        if ((st == 0 || st == ABBA_ST_KMAX) && kc > 0 && done + kc < ktot) {
            ++cnt;
        } else {
            status[s] = st ? st : ABBA_ST_KMAX;
            alive[s] = 0;
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
        *nalive = t;
    }
}

__global__ void copy_hist_k(const double *__restrict__ src, int sstride, double *__restrict__ dst, int dstride,
                            int cols, int S) {
    const int s = blockIdx.x;
    if (s >= S) return;
    for (int j = threadIdx.x; j < cols; j += blockDim.x) dst[(size_t)s * dstride + j] = src[(size_t)s * sstride + j];
}

// One cycle of the method for every slice with alive[s] (all if alive is
// NULL): r_0, beta, w_1 from the current x, then up to kcap iterations, each
// ending in the stopping rules; cfg.iters / cfg.status receive the iteration
// count and status of the cycle.
static int run_cycle(const SolveDims &d, const SolveWS &ws, const IterCfg &cfg, const void *b, void *x,
                     const int *alive, int kcap, const abba_exec &ex, hipGraphExec_t *gexec, hipGraph_t *graph,
                     hipStream_t st) {
    Launch L0{st, nullptr, nullptr};
    const int64_t wsl = (int64_t)d.wslots * d.ldw;
    int rc;
    // histories past a slice's stopping iteration read as NaN
    hipLaunchKernelGGL(fill_k, dim3(64), dim3(256), 0, st, ws.lamh, (int64_t)d.S * d.K, (double)NAN);
    ABBA_LAUNCHED("fill_k");
    hipLaunchKernelGGL(fill_k, dim3(64), dim3(256), 0, st, ws.rhoh, (int64_t)d.S * (d.K + 1), (double)NAN);
    ABBA_LAUNCHED("fill_k");
    if (d.ncp) {
        hipLaunchKernelGGL(fill_k, dim3(64), dim3(256), 0, st, ws.ncph, (int64_t)d.S * d.K, (double)NAN);
        ABBA_LAUNCHED("fill_k");
    }

    // ---- initialisation: r_0, beta, w_1 (Alg. 1 lines 1-3, Alg. 2 lines 1-3)
    if ((rc = launch_zero_pad(d.w_dt, ws.W, wsl, d.wslots, d.ldw, d.len, d.S, st))) return rc;
    if (ws.P && (rc = launch_zero_pad(d.img_dt, ws.P, (int64_t)d.pslots * d.ldn, d.pslots, d.ldn, d.n, d.S, st)))
        return rc;
    VecRef xin{x, d.n, 0, 0};
    VecRef sino{ws.sino, d.ldm, 0, 0};
    if ((rc = clock_mark(cfg.clk, ABBA_PHASE_OTHER))) return rc;
    if ((rc = apply_op(cfg.A, true, xin, d.img_dt, sino, d.sino_dt, d, ws, L0, cfg.clk))) return rc;
    if (d.mode == ABBA_MODE_AB) {
        // r_0 = b - A x_0 (basis storage), rho_0 = beta
        if ((rc = launch_sub(d.sino_dt, b, d.m, ws.sino, d.ldm, d.w_dt, ws.W, wsl, d.m, d.ldw, d.S, st))) return rc;
        if ((rc = launch_norm(d.w_dt, ws.W, wsl, d.m, d.S, ws.npart, ws.rhoh, d.K + 1, st))) return rc;
    } else {
        // b - A x_0 kept in `sino` (data residual); r_0 = B(b - A x_0)
        if ((rc = launch_sub(d.sino_dt, b, d.m, ws.sino, d.ldm, d.sino_dt, ws.sino, d.ldm, d.m, d.ldm, d.S, st)))
            return rc;
        if ((rc = launch_norm(d.sino_dt, ws.sino, d.ldm, d.m, d.S, ws.npart, ws.rhoh, d.K + 1, st))) return rc;
        VecRef w0{ws.W, wsl, 0, 0};
        if ((rc = apply_op(cfg.B, false, sino, d.sino_dt, w0, d.w_dt, d, ws, L0, cfg.clk))) return rc;
    }
    if ((rc = normalize_first(d, ws, cfg.iters, cfg.status, alive, st))) return rc;
    if ((cfg.learned || d.feat_out || d.labels) && (rc = learned_prepare(d, ws, x, cfg.out, st))) return rc;
    if (d.ortho == ABBA_ORTHO_DELAYED) {
        // step 0 of the delayed schedule: M w_1 and its first pass, giving
        // the once-orthogonalised second vector (no projected problem yet)
        hipLaunchKernelGGL(set_int_k, dim3(1), dim3(1), 0, st, ws.kdev, 0);
        ABBA_LAUNCHED("set_int_k");
        Launch L1{st, ws.kdev, ws.active};
        if ((rc = apply_M(d, ws, cfg, L1))) return rc;
        if ((rc = clock_mark(cfg.clk, ABBA_PHASE_ORTHO))) return rc;
        if ((rc = dcgs2_step(d, ws, ws.kdev, st))) return rc;
        if ((rc = clock_mark(cfg.clk, ABBA_PHASE_OTHER))) return rc;
    }
    hipLaunchKernelGGL(set_int_k, dim3(1), dim3(1), 0, st, ws.kdev, 1);
    ABBA_LAUNCHED("set_int_k");

    // ---- iterations
    if (ex.use_graph && !cfg.clk && !*gexec) {
        hipStream_t cap;
        ABBA_HIP(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
        hipError_t e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess) {
            (void)hipStreamDestroy(cap);
            return hip_fail(e, "hipStreamBeginCapture");
        }
        rc = one_iteration(d, ws, cfg, cap);
        e = hipStreamEndCapture(cap, graph);
        (void)hipStreamDestroy(cap);
        if (rc) return rc;
        if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
        e = hipGraphInstantiate(gexec, *graph, nullptr, nullptr, 0);
        if (e != hipSuccess) return hip_fail(e, "hipGraphInstantiate");
    }
    const bool polling = cfg.stop_kind != ABBA_STOP_NONE;
    int host_nact = d.S;
    for (int it = 1; it <= kcap; ++it) {
        if (*gexec) {
            hipError_t e = hipGraphLaunch(*gexec, st);
            if (e != hipSuccess) return hip_fail(e, "hipGraphLaunch");
        } else if ((rc = one_iteration(d, ws, cfg, st))) {
            return rc;
        }
        if (polling && (it % ex.poll_every == 0) && it < kcap) {
            hipError_t e = hipMemcpyAsync(&host_nact, ws.nact, sizeof(int), hipMemcpyDeviceToHost, st);
            if (e == hipSuccess) e = hipStreamSynchronize(st);
            if (e != hipSuccess) return hip_fail(e, "active-slice poll");
            if (host_nact == 0) break;
        }
    }
    return ABBA_OK;
}

// x += P_k y_k (AB) or W_k y_k (BA) with each slice's own k = iters[s].
static int assemble_cycle(const SolveDims &d, const SolveWS &ws, void *x, const int *iters, hipStream_t st) {
    int rc;
    if (d.mode == ABBA_MODE_AB) {
        // delayed schedule: P holds B applied to the vectors before their
        // second pass, B W_k y = P' (T y)
        const double *yk = ws.y;
        if (d.ortho == ABBA_ORTHO_DELAYED) {
            if ((rc = launch_ty(d, ws, iters, nullptr, nullptr, st))) return rc;
            yk = ws.y2;
        }
        return launch_assemble(d.img_dt, ws.P, (int64_t)d.pslots * d.ldn, d.ldn, d.img_dt, x, d.n, yk, d.K, iters,
                               d.S, st);
    }
    return launch_assemble(d.w_dt, ws.W, (int64_t)d.wslots * d.ldw, d.ldw, d.img_dt, x, d.n, ws.y, d.K, iters,
                           d.S, st);
}

}  // namespace abba

using namespace abba;

// Sub-batches of exec.streams: part i holds slices [first[i], first[i] + count[i]).
static int split_parts(int batch, const abba_exec *exec, std::vector<int> &first, std::vector<int> &count) {
    const int p = exec && exec->streams > 1 ? std::min(exec->streams, batch) : 1;
    first.assign(p, 0);
    count.assign(p, 0);
    for (int i = 0, s0 = 0; i < p; ++i) {
        count[i] = batch / p + (i < batch % p ? 1 : 0);
        first[i] = s0;
        s0 += count[i];
    }
    return p;
}

static size_t solve_one_bytes(const abba_op *A, const abba_op *B, int batch, int mode, int k, const abba_stop *stop,
                              const abba_exec *exec, int *rc);

extern "C" int abba_solve_workspace(const abba_op *A, const abba_op *B, int batch, int mode, int k,
                                    const abba_stop *stop, const abba_exec *exec, size_t *bytes) {
    if (!bytes) {
        set_error("bytes is NULL");
        return ABBA_ERR_ARG;
    }
    if (exec && exec->streams < 0) {
        set_error("exec.streams must be >= 0");
        return ABBA_ERR_ARG;
    }
    std::vector<int> first, count;
    const int p = split_parts(batch, exec, first, count);
    if (p > 1) {   // the sub-batches' workspaces one after another, each 256-byte aligned
        size_t total = 0;
        for (int i = 0; i < p; ++i) {
            int rc = ABBA_OK;
            const size_t b = solve_one_bytes(A, B, count[i], mode, k, stop, exec, &rc);
            if (rc) return rc;
            total += (b + 255) / 256 * 256;
        }
        *bytes = total;
        return ABBA_OK;
    }
    int rc = ABBA_OK;
    *bytes = solve_one_bytes(A, B, batch, mode, k, stop, exec, &rc);
    return rc;
}

static size_t solve_one_bytes(const abba_op *A, const abba_op *B, int batch, int mode, int k, const abba_stop *stop,
                              const abba_exec *exec, int *rcp) {
    SolveDims d;
    abba_out dummy;
    std::memset(&dummy, 0, sizeof(dummy));
    dummy.resid = (double *)1;   // size for the worst case (Z kept in BA mode)
    const int kc = exec && exec->restart > 0 && exec->restart < k ? exec->restart : k;
    int rc = make_dims(A, B, batch, mode, kc, stop, &dummy, &d);
    *rcp = rc;
    if (rc) return 0;
    d.labels = exec && (exec->features & ABBA_FEAT_LABELS) && mode == ABBA_MODE_AB;
    return solve_workspace_bytes(d, nullptr, nullptr, op_scratch_bytes(A, B, batch));
}

extern "C" int abba_solve_layout(const abba_op *A, const abba_op *B, int batch, int mode, int k,
                                 const abba_stop *stop, const abba_exec *exec, abba_basis_layout *layout) {
    if (!layout) {
        set_error("layout is NULL");
        return ABBA_ERR_ARG;
    }
    if (exec && exec->streams > 1) {
        set_error("abba_solve_layout describes the workspace of one stream (exec.streams <= 1)");
        return ABBA_ERR_UNSUPPORTED;
    }
    SolveDims d;
    abba_out dummy;
    std::memset(&dummy, 0, sizeof(dummy));
    dummy.resid = (double *)1;   // the carve-up abba_solve_workspace sizes
    const int kc = exec && exec->restart > 0 && exec->restart < k ? exec->restart : k;
    int rc = make_dims(A, B, batch, mode, kc, stop, &dummy, &d);
    if (rc) return rc;
    d.labels = exec && (exec->features & ABBA_FEAT_LABELS) && mode == ABBA_MODE_AB;
    SolveWS ws;
    // carve from a fake base address 0 + 256 so that offsets come out as
    // pointers (a null base would leave every pointer null)
    char *base = reinterpret_cast<char *>(256);
    const size_t bytes = solve_workspace_bytes(d, &ws, base, op_scratch_bytes(A, B, batch));
    std::memset(layout, 0, sizeof(*layout));
    layout->bytes = bytes;
    layout->basis = (size_t)((char *)ws.W - base);
    layout->hessenberg = (size_t)((char *)ws.H - base);
    layout->singular_values = (size_t)((char *)ws.sig - base);
    layout->ldw = d.ldw;
    layout->len = d.len;
    layout->basis_dtype = d.w_dt;
    layout->basis_slots = d.wslots;
    layout->k = d.K;
    return ABBA_OK;
}

static int solve_one(const abba_op *A, const abba_op *B, const void *b, void *x, int batch, int mode, int k,
                     const abba_reg *reg, const abba_stop *stop, const abba_out *out, const abba_exec *exec,
                     void *workspace, size_t ws_bytes, void *stream) {
    if (!b || !x || !reg || !out || !out->iters || !out->status || !workspace) {
        set_error("abba_solve: b, x, reg, out.iters, out.status and workspace are required");
        return ABBA_ERR_ARG;
    }
    abba_exec ex{0, 1, 0, 0, ABBA_ORTHO_DELAYED, nullptr, 1};
    if (exec) ex = *exec;
    if (ex.restart < 0) {
        set_error("restart cycle length must be >= 0");
        return ABBA_ERR_ARG;
    }
    if (k < 1) {
        set_error("k = %d must be >= 1", k);
        return ABBA_ERR_ARG;
    }
    // restarted runs keep a basis of one cycle (Sec. 3.3); k is then the total
    const bool restarting = ex.restart > 0 && ex.restart < k;
    const int kc = restarting ? ex.restart : k;
    SolveDims d;
    int rc = make_dims(A, B, batch, mode, kc, stop, out, &d);
    if (rc) return rc;
    const int rule = reg->kind;
    if (rule < ABBA_REG_NONE || rule > ABBA_REG_LEARNED) {
        set_error("unknown lambda rule %d", rule);
        return ABBA_ERR_ARG;
    }
    if (rule == ABBA_REG_FIXED && !(reg->lambda >= 0.0)) {
        set_error("fixed lambda must be >= 0");
        return ABBA_ERR_ARG;
    }
    if (rule == ABBA_REG_DP) {
        if (mode != ABBA_MODE_AB) {
            set_error("the discrepancy-principle lambda rule needs AB mode (projected residual = data residual)");
            return ABBA_ERR_UNSUPPORTED;
        }
        if (!reg->noise_norm || !(reg->tau > 0.0)) {
            set_error("the discrepancy-principle lambda rule needs noise_norm and tau > 0");
            return ABBA_ERR_ARG;
        }
    }
    if (rule == ABBA_REG_LEARNED && !reg->mlp) {
        set_error("the learned lambda rule needs model parameters");
        return ABBA_ERR_ARG;
    }
    const int stop_kind = stop ? stop->kind : ABBA_STOP_NONE;
    if (stop_kind < ABBA_STOP_NONE || stop_kind > ABBA_STOP_NCP) {
        set_error("unknown stopping rule %d", stop_kind);
        return ABBA_ERR_ARG;
    }
    if (stop_kind == ABBA_STOP_DP && (!stop->noise_norm || !(stop->tau > 0.0))) {
        set_error("the discrepancy-principle stop needs noise_norm and tau > 0");
        return ABBA_ERR_ARG;
    }
    if (stop_kind == ABBA_STOP_RNS && !(stop->rns_eps > 0.0)) {
        set_error("residual-norm stagnation needs rns_eps > 0");
        return ABBA_ERR_ARG;
    }
    if (stop_kind == ABBA_STOP_LEARNED && stop->noise_norm && !(stop->tau > 0.0)) {
        set_error("the discrepancy-principle check of the learned stop needs tau > 0");
        return ABBA_ERR_ARG;
    }
    if (stop_kind == ABBA_STOP_LEARNED && rule != ABBA_REG_LEARNED) {
        set_error("the learned stop needs the learned lambda rule (it shares the model)");
        return ABBA_ERR_ARG;
    }
    if (ex.ortho != ABBA_ORTHO_DELAYED && ex.ortho != ABBA_ORTHO_CGS2) {
        set_error("unknown Gram-Schmidt schedule %d", ex.ortho);
        return ABBA_ERR_ARG;
    }
    d.ortho = ex.ortho;
    if (ex.poll_every < 1) ex.poll_every = 1;
    if (restarting && (rule == ABBA_REG_LEARNED || ex.features)) {
        set_error("the learned rule, features and labels are defined for unrestarted runs");
        return ABBA_ERR_UNSUPPORTED;
    }
    if (ex.features & ~(ABBA_FEAT_OUT | ABBA_FEAT_LABELS)) {
        set_error("unknown feature bits %d", ex.features);
        return ABBA_ERR_ARG;
    }
    d.feat_out = (ex.features & ABBA_FEAT_OUT) != 0;
    d.labels = (ex.features & ABBA_FEAT_LABELS) != 0;
    if (d.feat_out && !out->features) {
        set_error("exec.features asks for features but out.features is NULL");
        return ABBA_ERR_ARG;
    }
    if (d.labels) {
        if (mode != ABBA_MODE_AB) {
            set_error("RRE labels are formed in AB mode only");
            return ABBA_ERR_UNSUPPORTED;
        }
        if (!out->x_true || !out->rre) {
            set_error("RRE labels need out.x_true and out.rre");
            return ABBA_ERR_ARG;
        }
    }
    SolveWS ws;
    const size_t need = solve_workspace_bytes(d, &ws, workspace, op_scratch_bytes(A, B, batch));
    if (ws_bytes < need) {
        set_error("workspace of %zu bytes is smaller than the %zu needed", ws_bytes, need);
        return ABBA_ERR_ARG;
    }
    if ((uintptr_t)workspace & 255) {
        set_error("the workspace must be 256-byte aligned");
        return ABBA_ERR_ARG;
    }
    hipStream_t st = (hipStream_t)stream;
    if ((rc = smallsolve_prepare())) return rc;

    IterCfg cfg;
    cfg.A = A;
    cfg.B = B;
    cfg.rule = rule;
    cfg.lam_fixed = reg->lambda;
    cfg.tau = reg->tau;
    cfg.noise_reg = reg->noise_norm;
    cfg.stop_kind = stop_kind;
    cfg.stop_tau = stop ? stop->tau : 0.0;
    cfg.rns_eps = stop ? stop->rns_eps : 0.0;
    cfg.noise_stop = stop ? stop->noise_norm : nullptr;
    cfg.learned_gate = stop ? stop->learned_gate : 0.0;
    // a restarted run counts iterations and status per cycle, then merges them
    cfg.iters = restarting ? ws.citers : out->iters;
    cfg.status = restarting ? ws.cstatus : out->status;
    cfg.learned = rule == ABBA_REG_LEARNED;
    cfg.reg = reg;
    cfg.out = out;
    cfg.x0 = x;
    PhaseClock clock;
    clock.st = st;
    cfg.clk = ex.phase_ms ? &clock : nullptr;
    hipGraphExec_t gexec = nullptr;
    hipGraph_t graph = nullptr;
    auto cleanup = [&]() {
        if (gexec) (void)hipGraphExecDestroy(gexec);
        if (graph) (void)hipGraphDestroy(graph);
    };
    // the phase times of a finished run (the call then waits for the stream)
    auto timed = [&](int rc_) {
        if (!rc_ && cfg.clk) rc_ = clock.finish(ex.phase_ms);
        return rc_;
    };

    if (!restarting) {
        rc = run_cycle(d, ws, cfg, b, x, nullptr, d.K, ex, &gexec, &graph, st);
        if (!rc) rc = assemble_cycle(d, ws, x, out->iters, st);
        cleanup();
        if (rc) return rc;
        if (out->lambda) {
            hipLaunchKernelGGL(copy_hist_k, dim3(d.S), dim3(128), 0, st, ws.lamh, d.K, out->lambda, d.K, d.K, d.S);
            ABBA_LAUNCHED("copy_hist_k");
        }
        if (out->resid) {
            hipLaunchKernelGGL(copy_hist_k, dim3(d.S), dim3(128), 0, st, ws.rhoh, d.K + 1, out->resid, d.K + 1,
                               d.K + 1, d.S);
            ABBA_LAUNCHED("copy_hist_k");
        }
        if (out->ncp && d.ncp) {
            hipLaunchKernelGGL(copy_hist_k, dim3(d.S), dim3(128), 0, st, ws.ncph, d.K, out->ncp, d.K, d.K, d.S);
            ABBA_LAUNCHED("copy_hist_k");
        }
        return timed(ABBA_OK);
    }

    // ---- restarted cycles (Sec. 3.3): x_0 <- the last cycle's iterate
    if (out->lambda) {
        hipLaunchKernelGGL(fill_k, dim3(64), dim3(256), 0, st, out->lambda, (int64_t)d.S * k, (double)NAN);
        ABBA_LAUNCHED("fill_k");
    }
    if (out->resid) {
        hipLaunchKernelGGL(fill_k, dim3(64), dim3(256), 0, st, out->resid, (int64_t)d.S * (k + 1), (double)NAN);
        ABBA_LAUNCHED("fill_k");
    }
    if (out->ncp && d.ncp) {
        hipLaunchKernelGGL(fill_k, dim3(64), dim3(256), 0, st, out->ncp, (int64_t)d.S * k, (double)NAN);
        ABBA_LAUNCHED("fill_k");
    }
    hipLaunchKernelGGL(cycle_begin_k, dim3((d.S + 255) / 256), dim3(256), 0, st, ws.alive, out->iters, out->status,
                       d.S);
    ABBA_LAUNCHED("cycle_begin_k");
    for (int done = 0; done < k && !rc;) {
        const int pc = std::min(d.K, k - done);
        rc = run_cycle(d, ws, cfg, b, x, ws.alive, pc, ex, &gexec, &graph, st);
        if (!rc) rc = assemble_cycle(d, ws, x, ws.citers, st);
        if (rc) break;
        hipLaunchKernelGGL(cycle_end_k, dim3(1), dim3(1024), 0, st, ws.alive, ws.citers, ws.cstatus, ws.lamh,
                           ws.rhoh, d.ncp ? ws.ncph : nullptr, d.K, out->iters, out->status, out->lambda, out->resid,
                           d.ncp ? out->ncp : nullptr, k, done, ws.nact, d.S);
        ABBA_LAUNCHED("cycle_end_k");
        done += pc;
        if (done < k) {
            int alive = 0;
            hipError_t e = hipMemcpyAsync(&alive, ws.nact, sizeof(int), hipMemcpyDeviceToHost, st);
            if (e == hipSuccess) e = hipStreamSynchronize(st);
            if (e != hipSuccess) {
                rc = hip_fail(e, "alive-slice poll");
                break;
            }
            if (alive == 0) break;
        }
    }
    cleanup();
    return timed(rc);
}

// ------------------------------------------------ concurrent sub-batches --
// exec.streams > 1: the slices are independent, so the batch splits into
// sub-batches of consecutive slices, each solved by solve_one on a stream of
// its own from a host thread of its own (a thread drives its sub-batch's
// launches and active-slice polls); projector launches, sweeps and small
// solves of the sub-batches then overlap on the device.
extern "C" int abba_solve(const abba_op *A, const abba_op *B, const void *b, void *x, int batch, int mode, int k,
                          const abba_reg *reg, const abba_stop *stop, const abba_out *out, const abba_exec *exec,
                          void *workspace, size_t ws_bytes, void *stream) {
    if (exec && exec->streams < 0) {
        set_error("exec.streams must be >= 0");
        return ABBA_ERR_ARG;
    }
    std::vector<int> first, count;
    const int p = batch > 0 ? split_parts(batch, exec, first, count) : 1;
    if (p <= 1) return solve_one(A, B, b, x, batch, mode, k, reg, stop, out, exec, workspace, ws_bytes, stream);
    if (!A || !B || !b || !x || !reg || !out || !out->iters || !out->status || !workspace) {
        set_error("abba_solve: A, B, b, x, reg, out.iters, out.status and workspace are required");
        return ABBA_ERR_ARG;
    }
    if (exec->phase_ms) {
        set_error("exec.phase_ms times one stream (exec.streams <= 1)");
        return ABBA_ERR_UNSUPPORTED;
    }
    size_t need = 0;
    int rc = abba_solve_workspace(A, B, batch, mode, k, stop, exec, &need);
    if (rc) return rc;
    if (ws_bytes < need) {
        set_error("workspace of %zu bytes is smaller than the %zu needed", ws_bytes, need);
        return ABBA_ERR_ARG;
    }
    if ((uintptr_t)workspace & 255) {
        set_error("the workspace must be 256-byte aligned");
        return ABBA_ERR_ARG;
    }
    if ((rc = smallsolve_prepare())) return rc;
    int dev = 0;
    ABBA_HIP(hipGetDevice(&dev));
    const size_t bsz = dtype_size(A->sino_dtype), xsz = dtype_size(A->img_dtype);
    const size_t kk = (size_t)k;
    abba_exec ex1 = *exec;
    ex1.streams = 1;
    struct Part {
        abba_reg reg;
        abba_stop stop;
        abba_out out;
        void *ws;
        size_t ws_bytes;
        hipStream_t st;
        hipEvent_t done;
        int rc;
        std::string err;
    };
    std::vector<Part> parts(p);
    char *wp = (char *)workspace;
    for (int i = 0; i < p; ++i) {
        Part &q = parts[i];
        const size_t s0 = (size_t)first[i];
        q.reg = *reg;
        if (reg->noise_norm) q.reg.noise_norm = reg->noise_norm + s0;
        if (stop) {
            q.stop = *stop;
            if (stop->noise_norm) q.stop.noise_norm = stop->noise_norm + s0;
        }
        q.out = *out;
        q.out.iters = out->iters + s0;
        q.out.status = out->status + s0;
        if (out->lambda) q.out.lambda = out->lambda + s0 * kk;
        if (out->resid) q.out.resid = out->resid + s0 * (kk + 1);
        if (out->features) q.out.features = out->features + s0 * kk * ABBA_MLP_FEATURES;
        if (out->x_true) q.out.x_true = (const char *)out->x_true + s0 * (size_t)A->n * xsz;
        if (out->ncp) q.out.ncp = out->ncp + s0 * kk;
        if (out->rre) q.out.rre = out->rre + s0 * kk * ABBA_LABEL_GRID;
        size_t wb = 0;
        if ((rc = abba_solve_workspace(A, B, count[i], mode, k, stop, &ex1, &wb))) return rc;
        q.ws = wp;
        q.ws_bytes = wb;
        wp += (wb + 255) / 256 * 256;
        q.st = nullptr;
        q.done = nullptr;
        q.rc = ABBA_OK;
    }
    // the library's streams start after the work already on `stream`
    hipStream_t cst = (hipStream_t)stream;
    hipEvent_t start = nullptr;
    auto release = [&]() {
        for (Part &q : parts) {
            if (q.done) (void)hipEventDestroy(q.done);
            if (q.st) (void)hipStreamDestroy(q.st);
        }
        if (start) (void)hipEventDestroy(start);
    };
    hipError_t e = hipEventCreateWithFlags(&start, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventRecord(start, cst);
    for (int i = 0; i < p && e == hipSuccess; ++i) {
        e = hipStreamCreateWithFlags(&parts[i].st, hipStreamNonBlocking);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&parts[i].done, hipEventDisableTiming);
        if (e == hipSuccess) e = hipStreamWaitEvent(parts[i].st, start, 0);
    }
    if (e != hipSuccess) {
        rc = hip_fail(e, "abba_solve: sub-batch streams");
        release();
        return rc;
    }
    auto run_part = [&](int i) {
        Part &q = parts[i];
        const hipError_t se = hipSetDevice(dev);
        if (se != hipSuccess) {
            q.rc = hip_fail(se, "hipSetDevice");
        } else {
            const size_t s0 = (size_t)first[i];
            q.rc = solve_one(A, B, (const char *)b + s0 * (size_t)A->m * bsz, (char *)x + s0 * (size_t)A->n * xsz,
                             count[i], mode, k, &q.reg, stop ? &q.stop : nullptr, &q.out, &ex1, q.ws, q.ws_bytes,
                             q.st);
        }
        if (q.rc) q.err = abba_last_error();
    };
    std::vector<std::thread> threads;
    threads.reserve(p);
    for (int i = 0; i < p; ++i) {
        // a thread that cannot be started: its sub-batch runs on this one
        try {
            threads.emplace_back(run_part, i);
        } catch (const std::system_error &) {
            run_part(i);
        }
    }
    for (std::thread &t : threads) t.join();
    // `stream` waits for every sub-batch
    for (int i = 0; i < p; ++i) {
        e = hipEventRecord(parts[i].done, parts[i].st);
        if (e == hipSuccess) e = hipStreamWaitEvent(cst, parts[i].done, 0);
        if (e != hipSuccess) break;
    }
    for (int i = 0; i < p; ++i)
        if (parts[i].rc) {
            rc = parts[i].rc;
            set_error("sub-batch %d (slices %d..%d): %s", i, first[i], first[i] + count[i] - 1, parts[i].err.c_str());
            break;
        }
    if (!rc && e != hipSuccess) rc = hip_fail(e, "abba_solve: joining the sub-batch streams");
    release();
    return rc;
}
