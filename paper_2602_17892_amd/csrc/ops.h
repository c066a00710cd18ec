// Operator handles and internal launch interfaces of the HIP library.
#pragma once

#include <vector>

#include "common.h"

namespace abba {

// Per-angle constants of the 2D parallel-beam operators, computed in FP64 on
// the host and rounded to T.  A dominant-axis march over "rows" of the
// marched image (x itself for row-march angles, its transpose otherwise):
//   u_r = (s_d * inv_c + off) - r * slope   (interpolation coordinate in row r)
//   y   = w * sum_r lerp(row r, u_r)
template <typename T>
struct AngleTab {
    T inv_c;   // 1/cos (row march) or 1/sin (column march)
    T slope;   // sin/cos or cos/sin
    T off;     // c_r * slope + c_c (centre offsets of the marched image)
    T w;       // 1/|cos| or 1/|sin|: ray length per step
    T cb, sb;  // cos/ds, sin/ds: detector coordinate of a pixel in bins (B)
    T cs, sn;  // cos, sin (exact transpose)
    T absc;    // |dominant direction cosine|
    int rowmarch;
    int pad;
};

// Angles per workgroup of the LDS-band Joseph projector; its angle groups
// hold angles of one march direction only.
constexpr int JOSEPH_GA = 8;
// Zeros on each side of a row of the padded image copies read by the 2D
// Joseph projector: at least twice the rows of its bands (8).
constexpr int JPAD = 16;

// Per-view constants of the 3D cone beam, FP64 (ray set-up is FP64; the
// voxel-driven B rounds them to its accumulation type).
struct ConeView {
    double S[3];     // source position
    double D[3];     // detector centre
    double eu[3];    // column axis (unit)
    double ev[3];    // row axis (unit)
    double n[3];     // detector normal eu x ev
    double dist;     // (D - S) . n: magnification numerator
    double Sn;       // S . n
    double Su, Sv;   // S . eu / pu, S . ev / pv
    double cu, cv;   // (S - D) . eu / pu + (nu - 1)/2, the same for v
};

// Where one vector of a slice lives: base + s*slice_stride +
// (k + k_off)*k_stride elements, with k read from a device counter (or 0).
struct VecRef {
    void *base;
    int64_t slice_stride;
    int64_t k_stride;
    int k_off;
};

// Launch choices of one operator at one batch size (from abba_autotune or
// abba_op_set_tuning).  Every choice computes the same result bits; -1 or 0
// leaves a choice to the built-in rule.
struct TuneEntry {
    int batch;
    int a_path;   // 2D A: 0 gather kernel, 1 LDS-band kernel
    int a_jb;     // 2D A, LDS kernel: bins per thread and angle (2, 3 or 4)
    int b_g;      // 2D B: angles per LDS chunk
    int czt;      // 3D B: voxels per thread along z (2, 4 or 8)
    int a_rb;     // 3D A: detector rows per band of the work order (1 to 64)
    int a_occ;    // 3D A: workgroups per compute unit at most (0: no cap)
    int a_tile;   // 3D A: 0 detector rows per workgroup, 16: 16 x 16 detector tiles
    int a_vg;     // 3D A, tiles: views per group of the work order (0: built-in)
};
constexpr int MAX_TUNE = 8;

struct Launch {
    hipStream_t stream;
    const int *kdev;      // device iteration counter, or nullptr (k = 0)
    const int *active;    // device [batch] flags, or nullptr (all active)
};

}  // namespace abba

struct abba_op {
    int kind;
    abba_geometry g;
    std::vector<double> angles;
    int img_dtype, sino_dtype;
    int64_t n, m;
    int device;
    int nxcc;              // XCDs of the device (workgroups are dealt to them round-robin)
    int ncu;               // compute units of the device
    int lds_cu;            // LDS bytes per compute unit
    void *tab;             // AngleTab<float|double>[n_angles] or ConeView[views]
    int *agrp;             // 2D: [ngroups][4] {first, count, rowmarch, 0}, then the angle order [n_angles]
    int ngroups;
    void *bpw;             // 2D B: per (tile of 32 x 64 pixels, angle), the window start (pixbp_build_table)
    int cone_axes;         // 3D: bit a set if some ray has dominant axis a (0 x, 1 y, 2 z)
    abba::TuneEntry tune[abba::MAX_TUNE];   // per batch size (not thread-safe to change
    int ntune;                              // while the operator is in use)
    abba::TuneEntry trial;                  // abba_autotune's candidate under test
    int trial_on;
};

namespace abba {

// 2D parallel beam (proj2d.hip).  `scratch` holds the zero-padded copy of the
// operator input: at least par2d_scratch_bytes(op, batch) bytes.  A and B of
// one geometry may share it when they run in turn on one stream.
int par2d_forward(const abba_op *op, VecRef x, VecRef y, int y_dtype, int batch, void *scratch,
                  const Launch &L);
int par2d_back(const abba_op *op, VecRef y, int y_dtype, VecRef x, int batch, void *scratch, const Launch &L);
size_t par2d_scratch_bytes(const abba_op *op, int batch);
int pixbp_build_table(abba_op *op);

// 3D cone beam (cone3d.hip).
int cone_forward(const abba_op *op, VecRef x, VecRef y, int y_dtype, int batch, void *scratch, const Launch &L);
int cone_back(const abba_op *op, VecRef y, int y_dtype, VecRef x, int batch, void *scratch, const Launch &L);
size_t cone_scratch_bytes(const abba_op *op, int batch);

int op_build_tables(abba_op *op);

// Cone beam and 2D fan beam run the same kernels (a fan-beam image is the
// z = 0 plane of a cone-beam volume with one detector row).
static inline bool cone_path(const abba_op *op) { return op->g.kind != ABBA_GEOM_PAR2D; }

// Launch choices abba_autotune times (each computes the same result bits).
int par2d_tune_candidates(const abba_op *op, TuneEntry *out, int cap);
int cone_tune_candidates(const abba_op *op, TuneEntry *out, int cap);

// The launch choices for `batch`: the candidate under test, else the stored
// entry for that batch size, else nullptr (built-in rules).
static inline const TuneEntry *tune_for(const abba_op *op, int batch) {
    if (op->trial_on) return &op->trial;
    for (int i = 0; i < op->ntune; ++i)
        if (op->tune[i].batch == batch) return &op->tune[i];
    return nullptr;
}

static inline size_t dtype_size(int dt) { return dt == ABBA_F64 ? 8 : dt == ABBA_F32 ? 4 : 2; }

template <typename T>
__device__ __forceinline__ T *vec_ptr(const VecRef &r, int s, int k) {
    return reinterpret_cast<T *>(r.base) + (int64_t)s * r.slice_stride + (int64_t)(k + r.k_off) * r.k_stride;
}

}  // namespace abba
