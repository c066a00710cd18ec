/*
 * abba.h -- C ABI of the MI355X (gfx950) implementation of hybrid AB-/BA-GMRES
 * for X-ray CT with an unmatched backprojector (Bentley, Pasha, Sabate
 * Landman, Yang, Zhang, "Hybrid ABBA-GMRES for Unmatched Backprojectors in
 * Large Scale X-Ray Computerized Tomography").
 *
 * The problem (Sec. 1, eq. (1)): A x ~ b with a forward projector
 * A : R^n -> R^m, data b in R^m, and a backprojector B : R^m -> R^n that is
 * not the transpose of A (Sec. 2, eqs. (4)-(5)).  Hybrid AB-GMRES
 * (Algorithm 1) runs the Arnoldi process on AB, hybrid BA-GMRES
 * (Algorithm 2) on BA; each iteration solves the Tikhonov-regularised
 * projected problem of eq. (12) with a per-iteration lambda (Sec. 3.1) and
 * tests a stopping rule (Sec. 3.2).
 *
 * Conventions for every function:
 *   - Returns 0 (ABBA_OK) or a negative abba_status.  Nothing throws or
 *     aborts; abba_last_error() gives a thread-local message for the last
 *     failure on the calling thread.
 *   - Pointers named x, y, b and the abba_out arrays are DEVICE pointers
 *     (HIP memory of the current device).  The caller owns them; the library
 *     never frees them.  Op handles are owned by the library
 *     (abba_op_create / abba_op_destroy).
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *     Work is enqueued on it; see abba_solve for when the host waits.
 *   - Layouts are dense, row-major, batch-leading:
 *       2D image    [batch][ny][nx]          sinogram [batch][n_angles][det_u]
 *       3D volume   [batch][nz][ny][nx]      sinogram [batch][views][det_v][det_u]
 *   - Supported (image, sinogram) dtype pairs: (F64, F64), (F32, F32),
 *     (F32, BF16).  BF16 values are stored round-to-nearest-even and widened
 *     to FP32 on load; all accumulation is FP32 (FP64 for the F64 pair).
 *
 * Discretisation (the paper leaves it open; it calls the ASTRA toolbox):
 *   2D parallel beam.  Pixel (i,j) centre (j-(nx-1)/2, i-(ny-1)/2), unit
 *   pixels; bin d at s_d = (d-(det_u-1)/2)*det_pitch_u; angle
 *   t_a = a*pi/n_angles unless `angles` is given.  A ray marches over rows
 *   when |cos t| is the larger direction cosine (for the default angles:
 *   4a <= n_angles or 4a >= 3 n_angles).
 *     ABBA_OP_JOSEPH    A: Joseph -- per row (column) linear interpolation at
 *                       the ray crossing, times 1/|cos t| (1/|sin t|).
 *     ABBA_OP_JOSEPH_T  A^T: the exact transpose of A (matched pair).
 *     ABBA_OP_PIXEL     B: pixel driven -- per angle, linear interpolation of
 *                       the sinogram row at (X cos t + Y sin t), times
 *                       1/det_pitch_u.  B != A^T (the unmatched pair).
 *   3D circular cone beam.  Voxel (k,i,j) centre (j-(nx-1)/2, i-(ny-1)/2,
 *   k-(nz-1)/2); view v at b_v = 2*pi*v/views; source sid*(cos b, sin b, 0);
 *   flat detector at distance sdd from the source, columns along
 *   (-sin b, cos b, 0) with pitch det_pitch_u, rows along z with pitch
 *   det_pitch_v, centred on the central ray.
 *     ABBA_OP_JOSEPH    A: Joseph along the dominant axis of each
 *                       source-to-pixel ray, bilinear in the plane.
 *     ABBA_OP_PIXEL     B: voxel driven, bilinear on the detector, weight
 *                       (M/det_pitch_u)(M/det_pitch_v), M the magnification.
 *   2D fan beam, flat detector (the image plane of the cone geometry: nz and
 *   det_v are 1).  View v at b_v = 2*pi*v/views; source sid*(cos b, sin b);
 *   detector at distance sdd from the source, bins along (-sin b, cos b) with
 *   pitch det_pitch_u, centred on the central ray.
 *     ABBA_OP_JOSEPH    A: Joseph along the dominant axis of each
 *                       source-to-bin ray, linear interpolation, step weight.
 *     ABBA_OP_PIXEL     B: pixel driven, linear on the detector, weight
 *                       M/det_pitch_u.
 *   Outside the image or detector everything reads as zero.
 */
#ifndef ABBA_H
#define ABBA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    ABBA_OK = 0,
    ABBA_ERR_ARG = -1,          /* bad argument value (NULL, k out of range, small workspace) */
    ABBA_ERR_SHAPE = -2,        /* A and B sizes do not fit together                         */
    ABBA_ERR_DTYPE = -3,        /* unsupported dtype pair                                     */
    ABBA_ERR_NOMEM = -4,        /* host allocation failed or size overflow                    */
    ABBA_ERR_HIP = -5,          /* a HIP call or kernel launch failed                         */
    ABBA_ERR_NONFINITE = -6,    /* non-finite value found where a check was requested        */
    ABBA_ERR_UNSUPPORTED = -7   /* valid request that this library does not implement        */
} abba_status;

typedef enum { ABBA_F64 = 0, ABBA_F32 = 1, ABBA_BF16 = 2 } abba_dtype;
typedef enum { ABBA_GEOM_PAR2D = 0, ABBA_GEOM_CONE3D = 1, ABBA_GEOM_FAN2D = 2 } abba_geom_kind;
typedef enum { ABBA_OP_JOSEPH = 0, ABBA_OP_PIXEL = 1, ABBA_OP_JOSEPH_T = 2 } abba_op_kind;

typedef struct {
    int kind;                  /* abba_geom_kind                                         */
    int nx, ny, nz;            /* image size; nz = 1 for 2D                               */
    int n_angles;              /* 2D angles or 3D views                                   */
    int det_u, det_v;          /* detector bins (2D: det_v = 1)                           */
    double det_pitch_u;        /* > 0                                                     */
    double det_pitch_v;        /* > 0 (3D)                                                */
    double sid, sdd;           /* source-isocentre and source-detector distance (3D)     */
    const double *angles;      /* host array [n_angles] in radians, or NULL for defaults */
} abba_geometry;

typedef struct abba_op abba_op;

/* Create an operator on the current HIP device.  Geometry tables are built
 * in FP64 on the host and rounded to the storage type (for the 2D
 * pixel-driven B also the detector-window start of every 32 x 64 pixel tile
 * and angle); they are the only device memory the library allocates itself.  `img_dtype` and
 * `sino_dtype` must be one of the supported pairs.  *out receives the handle;
 * apart from its launch tuning (abba_autotune, abba_op_set_tuning) it is
 * immutable and may be used from several streams at once. */
int abba_op_create(abba_op **out, int kind, const abba_geometry *geom,
                   int img_dtype, int sino_dtype);
/* Frees the operator's device tables (hipFree, which waits for the device);
 * no work that uses the operator may still be queued.  NULL is a no-op. */
void abba_op_destroy(abba_op *op);
/* Image length n and sinogram length m of one slice. */
int abba_op_sizes(const abba_op *op, int64_t *n_img, int64_t *n_sino);

/* Device scratch, in bytes, that abba_project (abba_backproject) needs for
 * `batch` slices of this operator: zero-padded copies of the input that the
 * kernels read (2D A: the image rows with pads, row-major and transposed;
 * cone and fan A: the volume per dominant axis; cone and fan B: the views).
 * 0 for the 2D parallel-beam B and A^T, which stage their input in LDS.
 * `bytes` is a host pointer. */
int abba_project_workspace(const abba_op *A, int batch, size_t *bytes);
int abba_backproject_workspace(const abba_op *B, int batch, size_t *bytes);

/* y_s = A x_s for s < batch (eq. (1)); `A` must be ABBA_OP_JOSEPH.  x is
 * [batch][n] in the image dtype, y [batch][m] in the sinogram dtype.
 * workspace: a caller-owned device buffer of at least abba_project_workspace
 * bytes, 256-byte aligned (NULL when that size is 0), overwritten by the call
 * and free again once the stream has passed it; a smaller or misaligned one
 * is ABBA_ERR_ARG.  The call allocates nothing.  Asynchronous on `stream`.
 * Two kernels compute A with identical results: one per ray from global
 * memory, and one that streams the image through LDS, used when the batch is
 * large enough to fill the device; the environment variable
 * ABBA_JOSEPH_PATH=gather|lds forces one of them. */
int abba_project(const abba_op *A, const void *x, void *y, int batch, void *workspace, size_t ws_bytes,
                 void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): y = A x as
 * abba_project computes it (the same kernels, the same result bits), with its
 * scratch in a static device buffer of ABBA_NOALLOC_SCRATCH_BYTES that the
 * library holds on each device it runs on until the process ends.  The call
 * allocates nothing; the caller passes inputs and outputs.  A batch whose
 * scratch (abba_project_workspace) exceeds the buffer is ABBA_ERR_ARG.  Every
 * call on one device shares that device's buffer: calls that overlap on one
 * device (on different streams, or from several threads) race and must be
 * ordered by the caller.  Asynchronous on `stream`. */
#define ABBA_NOALLOC_SCRATCH_BYTES (64u << 20)
#define ABBA_MAX_DEVICES 64
int abba_project_noalloc(const abba_op *A, const void *x, void *y, int batch, void *stream);

/* x_s = B y_s for s < batch; `B` is ABBA_OP_PIXEL (unmatched B of
 * eqs. (4)-(5)) or ABBA_OP_JOSEPH_T (exact A^T).  y is [batch][m] in the
 * sinogram dtype, x [batch][n] in the image dtype.  workspace as for
 * abba_project, sized by abba_backproject_workspace.  The call allocates
 * nothing.  Asynchronous on `stream`. */
int abba_backproject(const abba_op *B, const void *y, void *x, int batch, void *workspace, size_t ws_bytes,
                     void *stream);

/* ---- Launch tuning (tile shapes and kernel choices of the projectors).
 * Every choice computes the same result bits: it changes how work is split
 * over workgroups, never the order of any sum. */
typedef struct {
    int a_path;        /* 2D A: 0 per-ray gather kernel, 1 LDS-band kernel, -1 built-in rule */
    int a_jb;          /* 2D A, LDS kernel: bins per thread and angle, 2..4 (0: 3)           */
    int b_g;           /* 2D B: angles per LDS chunk (0: built-in, at most 64 KB of LDS)      */
    int czt;           /* 3D B: voxels per thread along z, 2, 4 or 8 (0: 4)                   */
    int a_rb;          /* 3D A, rows of 256 columns: detector rows per band of the work
                          order (0: all rows, the views outermost); the views of a band
                          run before the next band                                        */
    int a_occ;         /* 3D A: at most this many workgroups per compute unit, held by
                          reserving unused LDS (at most 64 KB per workgroup, so
                          a_occ >= 3 on 160 KB of LDS per CU; smaller values are
                          ABBA_ERR_ARG): fewer rays in flight share the caches.
                          0: no cap when a_tile or a_rb is set, else the built-in cap
                          (6 for detector tiles)                                          */
    double ms;         /* abba_autotune: mean time of one apply with the chosen launch       */
    double default_ms; /* abba_autotune: the same with the built-in rules                    */
    int candidates;    /* abba_autotune: launch choices timed besides the built-in rules     */
    int a_tile;        /* 3D A: a workgroup per 16 x 16 tile of detector pixels with waves of
                          16 x 4 (16, and the built-in 0 for detectors of 16 rows or more)
                          or 8 x 8 (8); -1: per 256 columns of one detector row (also
                          chosen by a_rb >= 1, and the built-in for shorter detectors)     */
    int a_vg;          /* 3D A, detector tiles: views per group of the work order, 1..4096
                          (0: built-in, 24); the views of a group run next to each other
                          for each tile, so neighbouring views share the voxels in cache  */
} abba_tune;

/* Device bytes abba_autotune needs for `batch` slices: an input and an output
 * of the operator and the scratch of one apply. */
int abba_autotune_workspace(const abba_op *op, int batch, size_t *bytes);

/* Times the launch choices of `op` for `batch` slices (reps applies each,
 * after one warm-up; reps < 1 means 3) on a fixed input pattern written into
 * the caller's workspace (at least abba_autotune_workspace bytes, 256-byte
 * aligned), with HIP events on `stream`, and keeps the fastest (the built-in
 * rules included) in the operator for that batch size; later calls with that
 * batch size, abba_solve included, use it.  `best` (host) may be NULL.
 * Synchronises `stream`; allocates no device memory.  An operator keeps 8
 * batch sizes (the oldest is dropped); changing them while the operator runs
 * is a race. */
int abba_autotune(abba_op *op, int batch, int reps, void *workspace, size_t ws_bytes, void *stream,
                  abba_tune *best);

/* Sets the launch choices of `op` for `batch` (t NULL: forget them). */
int abba_op_set_tuning(abba_op *op, int batch, const abba_tune *t);

/* 1 and *t filled if `op` has launch choices for `batch`, 0 if not. */
int abba_op_get_tuning(const abba_op *op, int batch, abba_tune *t);

typedef enum { ABBA_MODE_AB = 0, ABBA_MODE_BA = 1 } abba_mode;

/* Lambda rules for the projected problem (Sec. 3.1): none (plain AB/BA-GMRES,
 * eqs. (6)-(7)), fixed, GCV (eq. (15)), discrepancy principle (AB only),
 * L-curve corner (eq. (14)), learned (MLP prediction, judged by GCV). */
typedef enum {
    ABBA_REG_NONE = 0, ABBA_REG_FIXED = 1, ABBA_REG_GCV = 2, ABBA_REG_DP = 3,
    ABBA_REG_LCURVE = 4, ABBA_REG_LEARNED = 5
} abba_reg_kind;

/* Stopping rules (Sec. 3.2): none (run k iterations), discrepancy principle,
 * residual-norm stagnation, learned stop index, normalised cumulative
 * periodogram.  NCP reads the data residual b - A x_k as rows of det_u
 * detector bins; each row's periodogram |DFT|^2 at frequencies 1..q,
 * q = det_u / 2, is summed over the rows; the run stops at the first k whose
 * NCP c_f = sum_{j<=f} P_j / sum_j P_j stays within the 5 % Kolmogorov-Smirnov
 * band of white noise: max_f |c_f - f/q| <= 1.36 / sqrt(q). */
typedef enum {
    ABBA_STOP_NONE = 0, ABBA_STOP_DP = 1, ABBA_STOP_RNS = 2, ABBA_STOP_LEARNED = 3, ABBA_STOP_NCP = 4
} abba_stop_kind;

/* Per-slice status bits written to abba_out.status. */
enum {
    ABBA_ST_KMAX = 1, ABBA_ST_STOP_DP = 2, ABBA_ST_STOP_RNS = 4, ABBA_ST_BREAKDOWN = 8,
    ABBA_ST_NONFINITE = 16, ABBA_ST_STOP_LEARNED = 32, ABBA_ST_STOP_NCP = 64
};

typedef struct {
    int kind;                  /* abba_reg_kind                                            */
    double lambda;             /* ABBA_REG_FIXED                                           */
    double tau;                /* DP safety factor (> 1), e.g. 1.01                        */
    const double *noise_norm;  /* device [batch]: ||e|| per slice (DP rule / DP stop)       */
    const void *mlp;           /* device: learned-model parameters (ABBA_REG_LEARNED)      */
    double judge_delta;        /* learned lambda accepted if GCV <= (1+delta) min GCV       */
} abba_reg;

typedef struct {
    int kind;                  /* abba_stop_kind                                           */
    double tau;                /* DP safety factor                                         */
    double rns_eps;            /* RNS tolerance                                            */
    const double *noise_norm;  /* device [batch]: ||e|| per slice (DP)                      */
    double learned_gate;       /* ABBA_STOP_LEARNED with noise_norm: the learned stop fires
                                  only once rho_k <= learned_gate * tau * ||e|| as well
                                  (<= 0: no such condition)                                 */
} abba_stop;

typedef struct {
    int *iters;                /* device [batch]: stopping iteration k (0 if beta = 0)    */
    int *status;               /* device [batch]: ABBA_ST_* bits                           */
    double *lambda;            /* device [batch*k] or NULL: lambda_j, j = 1..k             */
    double *resid;             /* device [batch*(k+1)] or NULL: rho_j = ||b - A x_j||       */
    float *features;           /* device [batch][k][ABBA_MLP_FEATURES] (exec.features bit
                                  ABBA_FEAT_OUT): the learned-rule features of iteration j
                                  in row j-1; rows past a slice's stop are left as they are */
    const void *x_true;        /* device [batch][n], image dtype (bit ABBA_FEAT_LABELS)    */
    double *ncp;               /* device [batch*k] or NULL (ABBA_STOP_NCP): the NCP distance
                                  max_f |c_f - f/q| of r_j, j = 1..k                        */
    double *rre;               /* device [batch][k][ABBA_LABEL_GRID] (bit ABBA_FEAT_LABELS):
                                  ||x_j(lam_g) - x_true|| / ||x_true|| for the grid
                                  lam_g = sigma_1(H_j) 10^(-8 + 8 g / 63), AB mode only   */
} abba_out;

typedef struct {
    int use_graph;             /* capture one iteration in a hipGraph and replay it        */
    int poll_every;            /* host reads the active-slice count every this many
                                  iterations (>= 1); ignored without a stopping rule       */
    int restart;               /* restart cycle length p (Sec. 3.3); 0 = no restart: with
                                  0 < p < k the run is cycles of at most p iterations, each
                                  started from the previous cycle's iterate, k in all      */
    int features;              /* bits ABBA_FEAT_*: write the learned-rule features
                                  (out.features) and/or training labels (out.rre)          */
    int ortho;                 /* Gram-Schmidt schedule, ABBA_ORTHO_*                        */
    double *phase_ms;          /* host [ABBA_PHASES] or NULL: add the stream time of each
                                  phase of the solve (ms, from HIP events recorded between
                                  the phases); the iterations then run without a graph and
                                  the call synchronises `stream` before it returns          */
    int streams;               /* run the batch as this many sub-batches of consecutive
                                  slices (sizes differing by at most one), each on a stream
                                  of its own and driven by a host thread of its own, the
                                  library's streams waiting on `stream` and `stream` on
                                  them; every slice gets the bits it gets alone.  0 or 1:
                                  one.  The workspace is the sub-batches' workspaces one
                                  after another (abba_solve_workspace with the same exec);
                                  not with phase_ms or abba_solve_layout                    */
} abba_exec;

/* Phases timed by exec.phase_ms: the forward projector A (its padded input
 * copies included), the backprojector B, the Gram-Schmidt sweeps with their
 * reductions and per-slice algebra (eq. (8)), the small solve with the lambda
 * rule, learned rule and stopping tests (eq. (12)), and the rest
 * (initialisation, residual formation, assembly of x). */
enum { ABBA_PHASE_A = 0, ABBA_PHASE_B = 1, ABBA_PHASE_ORTHO = 2, ABBA_PHASE_SMALL = 3, ABBA_PHASE_OTHER = 4,
       ABBA_PHASES = 5 };

/* exec.features bits.  Labels need AB mode, out.x_true and out.rre; they add a
 * [batch][k][k+1] FP64 Gram matrix to the workspace. */
enum { ABBA_FEAT_OUT = 1, ABBA_FEAT_LABELS = 2 };

/* Both schedules are CGS2 (classical Gram-Schmidt with one re-orthogonalisation,
 * FP64 accumulation) and give the same iterates in exact arithmetic.
 *   ABBA_ORTHO_DELAYED  the second pass of step k is done in the sweep of step
 *                       k+1 (two sweeps over the basis per iteration instead of
 *                       four; the projected problem of iteration k is completed
 *                       after the operator has been applied to the next vector,
 *                       so a slice stopping at iteration k applies M k+1 times).
 *   ABBA_ORTHO_CGS2     both passes in step k (four sweeps per iteration). */
enum { ABBA_ORTHO_DELAYED = 0, ABBA_ORTHO_CGS2 = 1 };

/* Bytes of device workspace abba_solve needs for (A, B, batch, mode, k, stop). */
int abba_solve_workspace(const abba_op *A, const abba_op *B, int batch, int mode, int k,
                         const abba_stop *stop, const abba_exec *exec, size_t *bytes);

/* Where abba_solve keeps the Arnoldi quantities of eq. (8), M W_k = W_{k+1} H_k,
 * inside its workspace, for callers that inspect them (the same arguments as
 * abba_solve_workspace; `layout` is a host struct).  After abba_solve has
 * finished on the stream, for slice s stopped at iteration k_s (the last
 * cycle's count for restarted runs):
 *   basis  vector j (0 <= j <= k_s) holds w_{j+1}, the orthonormal basis
 *          vector, at byte offset basis + ((s basis_slots + j) ldw) * esize,
 *          len entries of basis_dtype (ABBA_F64 for the F64 pair, else
 *          ABBA_F32); when slice s ended in a breakdown, vector k_s is not a
 *          basis vector (h_{k_s+1,k_s} = 0 and M W_k = W_k H_k(1:k, :)).
 *   H      FP64 [batch][k][k+1] at byte offset hessenberg, column-major per
 *          slice: entry (i, j) of H_k at ((s k + j)(k + 1) + i) * 8; columns
 *          j < k_s are those of H_{k_s}, rows past j + 1 are not defined.
 *   sigma  FP64 [batch][k] at byte offset singular_values: the singular
 *          values of H_{k_s} in descending order (k_s entries of slice s).
 * All offsets are within the workspace of abba_solve_workspace bytes. */
typedef struct {
    size_t bytes;              /* workspace size (as abba_solve_workspace)           */
    size_t basis;              /* byte offset of the basis                           */
    size_t hessenberg;         /* byte offset of H                                   */
    size_t singular_values;    /* byte offset of sigma                               */
    int64_t ldw;               /* elements between consecutive basis vectors         */
    int64_t len;               /* basis vector length: m (AB) or n (BA)              */
    int basis_dtype;           /* abba_dtype of the basis                            */
    int basis_slots;           /* basis vectors per slice                            */
    int k;                     /* Hessenberg columns per slice (one cycle)           */
} abba_basis_layout;

int abba_solve_layout(const abba_op *A, const abba_op *B, int batch, int mode, int k,
                      const abba_stop *stop, const abba_exec *exec, abba_basis_layout *layout);

/* Hybrid AB-GMRES (mode AB, Algorithm 1) or BA-GMRES (mode BA, Algorithm 2)
 * on `batch` independent slices.
 *   A       ABBA_OP_JOSEPH; B: ABBA_OP_PIXEL or ABBA_OP_JOSEPH_T; same geometry
 *           sizes, else ABBA_ERR_SHAPE.
 *   b       device [batch][m], sinogram dtype.
 *   x       device [batch][n], image dtype; in: x_0; out: x_k at each slice's
 *           stopping iteration.
 *   k       iteration budget K, 1 <= k <= min(m, n) (ABBA_ERR_ARG otherwise).
 *           With exec.restart = p, 0 < p < k (Sec. 3.3): the basis holds one
 *           cycle of p vectors (the workspace is sized for p), k is the total
 *           over all cycles and may exceed 100; iters, status and the
 *           histories count iterations over the whole run.  A stopping rule,
 *           a breakdown or non-finite data end a slice's run inside any
 *           cycle; the learned rule, features and labels need unrestarted
 *           runs (ABBA_ERR_UNSUPPORTED).
 *   reg, stop, out, exec as above; `out.iters` and `out.status` are required.
 *   workspace, ws_bytes  device buffer of at least abba_solve_workspace bytes,
 *           256-byte aligned.
 * The Arnoldi process uses classical Gram-Schmidt with one re-orthogonalisation
 * (CGS2, schedule exec.ortho) with FP64 accumulation; H_k, its SVD and lambda
 * are FP64.  A
 * breakdown (h_{k+1,k} <= 1e-14 ||M w_k||) ends that slice with the k-th
 * iterate and ABBA_ST_BREAKDOWN; it is not an error.
 * Without a stopping rule the call only enqueues work.  With one, the host
 * synchronises `stream` every exec.poll_every iterations to read how many
 * slices are still active, and returns when none is or k is reached; the
 * final assembly of x is still enqueued asynchronously. */
int abba_solve(const abba_op *A, const abba_op *B, const void *b, void *x, int batch,
               int mode, int k, const abba_reg *reg, const abba_stop *stop,
               const abba_out *out, const abba_exec *exec,
               void *workspace, size_t ws_bytes, void *stream);

/* ---- Learned lambda / stop index (an optional rule beside those of Sec. 3.1-3.2).
 * Features (per slice and iteration k, from quantities the method produces
 * regardless of lambda): the 32 largest singular values of H_k as
 * log10(sigma_i/sigma_1), padded with -16; log10(||e|| / ||b - A x_0||) when
 * the noise norm is given (reg or stop noise_norm), else -16; and the plain
 * GMRES residuals (eq. (9)) of iterations k-30..k as log10(r_j/r_0), 0 before
 * iteration 1; all scaled by 1/8.  Network: 64 -> 128 -> 128 -> 128 -> 2 with ReLU, FP32;
 * parameters are one flat device array of ABBA_MLP_PARAMS floats:
 * W1 [128][64], b1 [128], W2 [128][128], b2 [128], W3 [128][128], b3 [128],
 * W4 [2][128], b4 [2].  Outputs: o0 = log10(lambda/sigma_1)/8, o1 = k_stop/K.
 * In abba_solve with ABBA_REG_LEARNED the small solve first picks GCV's
 * lambda (eq. (15)); the predicted lambda^ replaces it when
 * GCV(lambda^) <= (1 + judge_delta) GCV(lambda_GCV).  ABBA_STOP_LEARNED stops
 * at the first k >= k^_k, where k^_k is the largest of the predictions K o1
 * (each clamped to [1, K]) made at iterations 1..k, after the discrepancy principle
 * when noise_norm is given, and then, with stop.learned_gate = c > 0, only
 * once the data residual is within the factor c of the discrepancy level
 * (rho_k <= c tau ||e||).  All four calls are asynchronous on `stream`. */
#define ABBA_MLP_FEATURES 64
#define ABBA_MLP_PARAMS 41602
#define ABBA_LABEL_GRID 64

/* Y [n][2] = network(X [n][64]).  Bitwise the same as the inference inside
 * abba_solve. */
int abba_mlp_forward(const float *params, const float *X, int n, float *Y, void *stream);

/* Device bytes of per-tile partial gradients abba_mlp_loss_grad needs for n
 * samples. */
int abba_mlp_loss_grad_workspace(int n, size_t *bytes);

/* Mean squared error L = (1/n) sum_i |net(X[r_i]) - T[r_i]|^2 with r_i =
 * idx[i] (device int32 [n], or NULL for r_i = i) and its gradient `grad`
 * [ABBA_MLP_PARAMS] (device); `loss` is a device double or NULL.  X is
 * [nrows][64], T [nrows][2]; rows r_i outside [0, nrows) count as absent.
 * workspace: device, at least abba_mlp_loss_grad_workspace(n) bytes (the
 * per-tile partial gradients); the call allocates nothing.  Deterministic:
 * the partials are summed in tile order. */
int abba_mlp_loss_grad(const float *params, const float *X, const float *T, int nrows, const int *idx, int n,
                       float *grad, double *loss, void *workspace, size_t ws_bytes, void *stream);

/* One Adam step (Kingma and Ba 2015, Algorithm 1, bias-corrected), step >= 1,
 * on params with moment buffers m, v (device, ABBA_MLP_PARAMS each). */
int abba_mlp_adam(float *params, const float *grad, float *m, float *v, int step, double lr, double beta1,
                  double beta2, double eps, void *stream);

/* Training targets from abba_solve's out.rre of `batch` runs of budget k:
 * targets [batch][k][2] row j-1 = (log10(lambda*_j / sigma_1)/8, k* / k) with
 * lambda*_j the grid minimiser of the RRE at iteration j (first index on
 * ties) and k* the iteration of the smallest of those minima; rows past
 * iters[s] (device, or NULL for k) are NaN.  k_star (device [batch]) may be
 * NULL. */
int abba_mlp_labels(const double *rre, int batch, int k, const int *iters, float *targets, int *k_star,
                    void *stream);

const char *abba_status_str(int status);
const char *abba_last_error(void);
/* Library version string. */
const char *abba_version(void);

#ifdef __cplusplus
}
#endif
#endif /* ABBA_H */
