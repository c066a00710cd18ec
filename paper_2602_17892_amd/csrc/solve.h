// Internal interfaces of the hybrid AB-/BA-GMRES driver.
#pragma once

#include "ops.h"

namespace abba {

// Number of element chunks (blocks) the reductions over a basis vector use.
constexpr int RED_BLOCKS = 128;
// Vectors handled per block of the multi-dot kernel.
constexpr int DOT_JT = 8;
// Largest Krylov dimension handled by the small-solve kernel.
constexpr int KMAX_SMALL = 100;
// NCP stopping rule: detector rows per workgroup of the periodogram kernel,
// and the longest detector row it handles (q = det / 2 <= 1024).
constexpr int NCP_RC = 16;
constexpr int NCP_MAX_DET = 2049;
int ncp_row_chunks(int rows);

// Per-slice scalars kept by the small solve, FP64.
enum {
    SC_BETA = 0,      // ||r_0||
    SC_UK1 = 1,       // GMRES residual component |(Q^T beta e1)_{k+1}|
    SC_MW = 2,        // ||M w_k|| (breakdown reference)
    SC_HK = 3,        // h_{k+1,k}
    SC_INV = 4,       // 1/h_{k+1,k} (0 on breakdown)
    SC_NOISE = 5,     // ||e|| (DP)
    SC_LAM = 6,       // last lambda
    SC_RHOHAT = 7,    // last projected residual
    SC_RHO0 = 8,      // ||b - A x_0||
    SC_LAMLEARN = 9,  // learned log10(lambda/sigma_1) prediction
    SC_KLEARN = 10,   // learned stop index prediction
    SC_SWEEPS = 11,   // most root iterations of the last SVD update (diagnostic)
    SC_COUNT = 16
};

enum { FL_BREAK = 1, FL_NONFINITE = 2 };

struct SolveDims {
    int S;          // batch
    int K;          // iteration budget
    int mode;       // ABBA_MODE_*
    int64_t n, m;   // image / sinogram length of a slice
    int64_t len;    // basis vector length (m for AB, n for BA)
    int64_t ldw;    // padded basis stride (multiple of 256 elements)
    int64_t ldn;    // padded image stride
    int64_t ldm;    // padded sinogram stride
    int keepZ;      // BA: keep Z = A W for the data residual
    int img_dt, sino_dt, w_dt;
    int wslots;     // basis vectors per slice (K + 2: the delayed step also holds M v)
    int pslots;     // kept operator outputs per slice (K + 1)
    int ortho;      // ABBA_ORTHO_*
    int feat_out;   // write the learned-rule features to out.features
    int labels;     // write RRE label grids to out.rre (AB mode)
    int ncp;        // the NCP stopping rule: residual vectors and periodograms
    int det;        // NCP: bins per detector row
    int nrch;       // NCP: row chunks per slice of the periodogram kernel
};

// Workspace carve-up (device pointers).
struct SolveWS {
    void *W;        // [S][K+2][ldw]  basis (w_dt)
    void *P;        // [S][K+1][ldn]  AB: B w_j (img_dt)
    void *Z;        // [S][K+1 or 1][ldm] BA: A w_j (sino_dt)
    void *sino;     // [S][ldm]       b - A x0 (sino_dt)
    void *scratch;  // zero-padded operator input (A and B take turns)
    double *part;   // [S][2(K+2)][nblk] partial dot products (vector-major)
    double *h;      // [S][K+2]
    double *c;      // [S][K+2]
    double *npart;  // [S][RED_BLOCKS] partial squared norms
    double *H;      // [S][K][K+1] column-major Hessenberg
    double *gc, *gs;// [S][K] Givens rotations
    double *g;      // [S][K+1] rotated beta e1
    double *Uj, *Vj;// [S][K][K] U and V of the SVD of R_k (column-major, stride K)
    double *y;      // [S][K]
    double *y2;     // [S][K]         delayed CGS2: T y
    double *T;      // [S][K][K]      delayed CGS2: W = V T (column-major, upper triangular)
    double *gd;     // [S][K+2]       delayed CGS2: update coefficients
    double *sig;    // [S][K]
    double *uh;     // [S][K]
    double *sc;     // [S][SC_COUNT]
    double *lamh;   // [S][K]
    double *rhoh;   // [S][K+1]
    float *feat;    // [S][64] learned-rule features of the current iteration
    float *pred;    // [S][2]  network outputs
    double *gres;   // [S][K+1] plain GMRES residual history (r_0 = beta)
    double *gram;   // [S][K][K+1] labels: Gram matrix of P' and P'^T (x_true - x_0)
    double *enorm;  // [S][2]  labels: ||x_true - x_0||^2, ||x_true||^2
    void *rvec;     // [S][ldm]  NCP: the data residual r_k (accumulation type)
    double *tcoef;  // [S][K+1]  NCP: coefficients of r_k in the kept vectors
    float *spec;    // [S][nrch][q] NCP: periodogram partial sums
    double *ncpd;   // [S]       NCP: distance of the current iteration
    double *ncph;   // [S][K]    NCP: distance history of the cycle
    int *citers;    // [S] restarted runs: iterations of the current cycle
    int *cstatus;   // [S] restarted runs: status of the current cycle
    int *alive;     // [S] restarted runs: the slice takes part in the next cycle
    int *active;    // [S]
    int *flags;     // [S]
    int *kdev;      // [1] current iteration (1-based)
    int *nact;      // [1] active slice count
};

size_t solve_workspace_bytes(const SolveDims &d, SolveWS *ws, void *base, size_t scratch_bytes);

}  // namespace abba
