// C ABI: status handling, operator handles, abba_project / abba_backproject.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>

#include "ops.h"

namespace abba {

static thread_local char g_err[512] = "";

void set_error(const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
}

int hip_fail(hipError_t e, const char *what) {
    set_error("%s: %s", what, hipGetErrorString(e));
    return ABBA_ERR_HIP;
}

static int supported_pair(int img, int sino) {
    return (img == ABBA_F64 && sino == ABBA_F64) || (img == ABBA_F32 && sino == ABBA_F32) ||
           (img == ABBA_F32 && sino == ABBA_BF16);
}

int validate_geometry(const abba_geometry *g, int kind) {
    if (!g) {
        set_error("geometry is NULL");
        return ABBA_ERR_ARG;
    }
    if (g->kind != ABBA_GEOM_PAR2D && g->kind != ABBA_GEOM_CONE3D && g->kind != ABBA_GEOM_FAN2D) {
        set_error("unknown geometry kind %d", g->kind);
        return ABBA_ERR_ARG;
    }
    const bool fan = g->kind == ABBA_GEOM_FAN2D;
    const bool cone = g->kind == ABBA_GEOM_CONE3D;
    if (g->nx <= 0 || g->ny <= 0 || g->n_angles <= 0 || g->det_u <= 0 || (cone && (g->nz <= 0 || g->det_v <= 0))) {
        set_error("geometry sizes must be positive");
        return ABBA_ERR_ARG;
    }
    if (!cone && ((g->nz != 1 && g->nz != 0) || (g->det_v != 1 && g->det_v != 0))) {
        set_error("2D geometry needs nz = det_v = 1");
        return ABBA_ERR_ARG;
    }
    if (fan && 2.0 * g->sid <= std::sqrt((double)g->nx * g->nx + (double)g->ny * g->ny)) {
        set_error("fan beam: the source (at distance sid from the centre) must lie outside the image");
        return ABBA_ERR_ARG;
    }
    if (fan && !(g->sid > 0.0 && g->sdd > g->sid)) {
        set_error("fan beam needs 0 < sid < sdd");
        return ABBA_ERR_ARG;
    }
    if (fan && kind == ABBA_OP_JOSEPH_T) {
        set_error("the exact transpose is implemented for parallel beams only");
        return ABBA_ERR_UNSUPPORTED;
    }
    if (!(g->det_pitch_u > 0.0) || (cone && !(g->det_pitch_v > 0.0))) {
        set_error("detector pitch must be positive");
        return ABBA_ERR_ARG;
    }
    if (cone && 2.0 * g->sid <= std::sqrt((double)g->nx * g->nx + (double)g->ny * g->ny + (double)g->nz * g->nz)) {
        set_error("cone beam: the source (at distance sid from the centre) must lie outside the volume");
        return ABBA_ERR_ARG;
    }
    if (cone && !(g->sid > 0.0 && g->sdd > g->sid)) {
        set_error("cone beam needs 0 < sid < sdd");
        return ABBA_ERR_ARG;
    }
    const double n = (double)g->nx * g->ny * (cone ? g->nz : 1);
    const double m = (double)g->n_angles * g->det_u * (cone ? g->det_v : 1);
    if (n > 4.0e9 || m > 4.0e9) {
        set_error("problem too large for 32-bit per-slice indexing");
        return ABBA_ERR_NOMEM;
    }
    if (cone && kind == ABBA_OP_JOSEPH_T) {
        set_error("the exact transpose is implemented for 2D geometries only");
        return ABBA_ERR_UNSUPPORTED;
    }
    if (g->angles) {
        for (int a = 0; a < g->n_angles; ++a)
            if (!std::isfinite(g->angles[a])) {
                set_error("angle %d is not finite", a);
                return ABBA_ERR_ARG;
            }
    }
    return ABBA_OK;
}

// March direction of angle a: over rows when |cos| is the larger direction
// cosine; for the default equispaced angles the integer rule 4a <= N or
// 4a >= 3N (no floating-point tie at 45 degrees).
static int rowmarch_of(const abba_geometry &g, int a) {
    if (g.angles) return std::fabs(std::cos(g.angles[a])) >= std::fabs(std::sin(g.angles[a]));
    return (4 * a <= g.n_angles) || (4 * a >= 3 * g.n_angles);
}

template <typename T>
static void fill_tab2d(const abba_op *op, AngleTab<T> *t) {
    const abba_geometry &g = op->g;
    const double cx = 0.5 * (g.nx - 1), cy = 0.5 * (g.ny - 1), ds = g.det_pitch_u;
    for (int a = 0; a < g.n_angles; ++a) {
        const double th = g.angles ? g.angles[a] : a * M_PI / g.n_angles;
        const double cs = std::cos(th), sn = std::sin(th);
        const int rowmarch = rowmarch_of(g, a);
        AngleTab<T> &e = t[a];
        if (rowmarch) {
            e.inv_c = (T)(1.0 / cs);
            e.slope = (T)(sn / cs);
            e.off = (T)(cy * (sn / cs) + cx);
            e.w = (T)(1.0 / std::fabs(cs));
            e.absc = (T)std::fabs(cs);
        } else {
            e.inv_c = (T)(1.0 / sn);
            e.slope = (T)(cs / sn);
            e.off = (T)(cx * (cs / sn) + cy);
            e.w = (T)(1.0 / std::fabs(sn));
            e.absc = (T)std::fabs(sn);
        }
        e.cb = (T)(cs / ds);
        e.sb = (T)(sn / ds);
        e.cs = (T)cs;
        e.sn = (T)sn;
        e.rowmarch = rowmarch;
        e.pad = 0;
    }
}

int build_cone_tables(abba_op *op);   // cone3d.hip

int op_build_tables(abba_op *op) {
    if (cone_path(op)) return build_cone_tables(op);
    const int na = op->g.n_angles;
    size_t bytes;
    void *host;
    if (op->img_dtype == ABBA_F64) {
        bytes = sizeof(AngleTab<double>) * na;
        host = new (std::nothrow) AngleTab<double>[na];
        if (!host) return ABBA_ERR_NOMEM;
        fill_tab2d(op, (AngleTab<double> *)host);
    } else {
        bytes = sizeof(AngleTab<float>) * na;
        host = new (std::nothrow) AngleTab<float>[na];
        if (!host) return ABBA_ERR_NOMEM;
        fill_tab2d(op, (AngleTab<float> *)host);
    }
    hipError_t e = hipMalloc(&op->tab, bytes);
    if (e == hipSuccess) e = hipMemcpy(op->tab, host, bytes, hipMemcpyHostToDevice);
    if (op->img_dtype == ABBA_F64) delete[] (AngleTab<double> *)host;
    else delete[] (AngleTab<float> *)host;
    if (e != hipSuccess) return hip_fail(e, "operator table upload");
    // angle groups of one march direction for the LDS-band projector
    std::vector<int> order, grp;
    for (int pass = 1; pass >= 0; --pass) {
        const int first = (int)order.size();
        for (int a = 0; a < na; ++a)
            if (rowmarch_of(op->g, a) == pass) order.push_back(a);
        for (int i = first; i < (int)order.size(); i += JOSEPH_GA) {
            grp.push_back(i);
            grp.push_back(std::min(JOSEPH_GA, (int)order.size() - i));
            grp.push_back(pass);
            grp.push_back(0);
        }
    }
    op->ngroups = (int)grp.size() / 4;
    grp.insert(grp.end(), order.begin(), order.end());
    e = hipMalloc(&op->agrp, grp.size() * sizeof(int));
    if (e == hipSuccess) e = hipMemcpy(op->agrp, grp.data(), grp.size() * sizeof(int), hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(e, "angle group upload");
    return op->kind == ABBA_OP_PIXEL ? pixbp_build_table(op) : ABBA_OK;
}

}  // namespace abba

using namespace abba;

extern "C" {

const char *abba_version(void) { return "abba-mi355x 0.1 (gfx950)"; }

const char *abba_last_error(void) { return g_err; }

const char *abba_status_str(int s) {
    switch (s) {
    case ABBA_OK: return "ok";
    case ABBA_ERR_ARG: return "invalid argument";
    case ABBA_ERR_SHAPE: return "shape mismatch";
    case ABBA_ERR_DTYPE: return "unsupported dtype";
    case ABBA_ERR_NOMEM: return "out of memory";
    case ABBA_ERR_HIP: return "HIP error";
    case ABBA_ERR_NONFINITE: return "non-finite value";
    case ABBA_ERR_UNSUPPORTED: return "unsupported";
    default: return "unknown status";
    }
}

int abba_op_create(abba_op **out, int kind, const abba_geometry *geom, int img_dtype, int sino_dtype) {
    if (!out) {
        set_error("out is NULL");
        return ABBA_ERR_ARG;
    }
    *out = nullptr;
    if (kind != ABBA_OP_JOSEPH && kind != ABBA_OP_PIXEL && kind != ABBA_OP_JOSEPH_T) {
        set_error("unknown operator kind %d", kind);
        return ABBA_ERR_ARG;
    }
    int rc = validate_geometry(geom, kind);
    if (rc) return rc;
    if (!supported_pair(img_dtype, sino_dtype)) {
        set_error("unsupported (image, sinogram) dtype pair (%d, %d)", img_dtype, sino_dtype);
        return ABBA_ERR_DTYPE;
    }
    abba_op *op = new (std::nothrow) abba_op();
    if (!op) return ABBA_ERR_NOMEM;
    op->kind = kind;
    op->g = *geom;
    if (op->g.kind != ABBA_GEOM_CONE3D) {
        op->g.nz = 1;
        op->g.det_v = 1;
    }
    if (op->g.kind == ABBA_GEOM_FAN2D) op->g.det_pitch_v = 1.0;
    if (geom->angles) {
        op->angles.assign(geom->angles, geom->angles + geom->n_angles);
        op->g.angles = op->angles.data();
    }
    op->img_dtype = img_dtype;
    op->sino_dtype = sino_dtype;
    op->n = (int64_t)op->g.nx * op->g.ny * op->g.nz;
    op->m = (int64_t)op->g.n_angles * op->g.det_u * op->g.det_v;
    op->tab = nullptr;
    op->bpw = nullptr;
    op->agrp = nullptr;
    op->ngroups = 0;
    op->cone_axes = 0;
    hipError_t e = hipGetDevice(&op->device);
    if (e != hipSuccess) {
        delete op;
        return hip_fail(e, "hipGetDevice");
    }
    // workgroups are dealt round-robin to the XCDs; the projectors renumber
    // them so that each XCD (own L2) works on a contiguous range of slices
    int nxcc = 1;
    if (hipDeviceGetAttribute(&nxcc, hipDeviceAttributeNumberOfXccs, op->device) != hipSuccess || nxcc < 1)
        nxcc = 1;
    int ncu = 0;
    if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, op->device) != hipSuccess || ncu < 1)
        ncu = 1;
    (void)hipGetLastError();
    int lds_cu = 0;
    if (hipDeviceGetAttribute(&lds_cu, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, op->device) !=
            hipSuccess || lds_cu < 1)
        lds_cu = 65536;
    op->nxcc = nxcc;
    op->ncu = ncu;
    op->lds_cu = lds_cu;
    rc = op_build_tables(op);
    if (rc) {
        if (op->tab) (void)hipFree(op->tab);
        if (op->bpw) (void)hipFree(op->bpw);
        if (op->agrp) (void)hipFree(op->agrp);
        delete op;
        return rc;
    }
    *out = op;
    return ABBA_OK;
}

void abba_op_destroy(abba_op *op) {
    if (!op) return;
    if (op->tab) (void)hipFree(op->tab);
    if (op->bpw) (void)hipFree(op->bpw);
    if (op->agrp) (void)hipFree(op->agrp);
    delete op;
}

int abba_op_sizes(const abba_op *op, int64_t *n_img, int64_t *n_sino) {
    if (!op) {
        set_error("op is NULL");
        return ABBA_ERR_ARG;
    }
    if (n_img) *n_img = op->n;
    if (n_sino) *n_sino = op->m;
    return ABBA_OK;
}

// Device scratch of one apply: the zero-padded copies the forward projectors
// read (2D: the image rows with pads, row-major and transposed; 3D: the
// volume per dominant axis), the zero-padded views the voxel- and
// pixel-driven backprojectors of the cone and fan geometries read, and none
// for the 2D parallel-beam backprojectors (they stage in LDS).
static size_t apply_scratch_bytes(const abba_op *op, int batch) {
    if (op->kind == ABBA_OP_JOSEPH_T) return 0;
    if (cone_path(op)) return cone_scratch_bytes(op, batch);
    return op->kind == ABBA_OP_JOSEPH ? par2d_scratch_bytes(op, batch) : 0;
}

static int check_ws(const char *who, size_t need, const void *ws, size_t ws_bytes) {
    if (need > 0 && (!ws || ws_bytes < need)) {
        set_error("%s: workspace of %zu bytes%s is smaller than the %zu needed", who, ws_bytes,
                  ws ? "" : " (NULL)", need);
        return ABBA_ERR_ARG;
    }
    if (need > 0 && ((uintptr_t)ws & 255)) {
        set_error("%s: the workspace must be 256-byte aligned", who);
        return ABBA_ERR_ARG;
    }
    return ABBA_OK;
}

int abba_project_workspace(const abba_op *A, int batch, size_t *bytes) {
    if (!A || !bytes || batch < 0 || A->kind != ABBA_OP_JOSEPH) {
        set_error("abba_project_workspace: an ABBA_OP_JOSEPH operator, batch >= 0 and bytes are required");
        return ABBA_ERR_ARG;
    }
    *bytes = batch ? apply_scratch_bytes(A, batch) : 0;
    return ABBA_OK;
}

int abba_backproject_workspace(const abba_op *B, int batch, size_t *bytes) {
    if (!B || !bytes || batch < 0 || (B->kind != ABBA_OP_PIXEL && B->kind != ABBA_OP_JOSEPH_T)) {
        set_error("abba_backproject_workspace: an ABBA_OP_PIXEL or ABBA_OP_JOSEPH_T operator, batch >= 0 and "
                  "bytes are required");
        return ABBA_ERR_ARG;
    }
    *bytes = batch ? apply_scratch_bytes(B, batch) : 0;
    return ABBA_OK;
}

int abba_project(const abba_op *A, const void *x, void *y, int batch, void *workspace, size_t ws_bytes,
                 void *stream) {
    if (!A || batch < 0 || (batch > 0 && (!x || !y))) {
        set_error("abba_project: NULL argument or negative batch");
        return ABBA_ERR_ARG;
    }
    if (A->kind != ABBA_OP_JOSEPH) {
        set_error("abba_project needs an ABBA_OP_JOSEPH operator");
        return ABBA_ERR_ARG;
    }
    if (batch == 0) return ABBA_OK;
    int rc = check_ws("abba_project", apply_scratch_bytes(A, batch), workspace, ws_bytes);
    if (rc) return rc;
    Launch L{(hipStream_t)stream, nullptr, nullptr};
    VecRef xr{const_cast<void *>(x), A->n, 0, 0};
    VecRef yr{y, A->m, 0, 0};
    return cone_path(A) ? cone_forward(A, xr, yr, A->sino_dtype, batch, workspace, L)
                        : par2d_forward(A, xr, yr, A->sino_dtype, batch, workspace, L);
}

int abba_backproject(const abba_op *B, const void *y, void *x, int batch, void *workspace, size_t ws_bytes,
                     void *stream) {
    if (!B || batch < 0 || (batch > 0 && (!x || !y))) {
        set_error("abba_backproject: NULL argument or negative batch");
        return ABBA_ERR_ARG;
    }
    if (B->kind != ABBA_OP_PIXEL && B->kind != ABBA_OP_JOSEPH_T) {
        set_error("abba_backproject needs an ABBA_OP_PIXEL or ABBA_OP_JOSEPH_T operator");
        return ABBA_ERR_ARG;
    }
    if (batch == 0) return ABBA_OK;
    int rc = check_ws("abba_backproject", apply_scratch_bytes(B, batch), workspace, ws_bytes);
    if (rc) return rc;
    Launch L{(hipStream_t)stream, nullptr, nullptr};
    VecRef yr{const_cast<void *>(y), B->m, 0, 0};
    VecRef xr{x, B->n, 0, 0};
    if (B->kind != ABBA_OP_JOSEPH_T && cone_path(B)) return cone_back(B, yr, B->sino_dtype, xr, batch, workspace, L);
    return par2d_back(B, yr, B->sino_dtype, xr, batch, nullptr, L);
}

// ------------------------------------------- allocation-free projection ---
// abba_project_noalloc keeps the scratch of abba_project (the padded image
// copies, which the padding kernel writes in full, pads included, before the
// projector reads them, so nothing needs clearing) in this file-scope device
// array instead of a caller workspace.  In host code the name `scratch` is a
// host-side stand-in, never a device address: each device's copy is located
// once with hipGetSymbolAddress and only that pointer is used.
static __device__ __align__(256) unsigned char scratch[ABBA_NOALLOC_SCRATCH_BYTES];

static std::mutex g_scratch_mu;
static void *g_scratch_dev[ABBA_MAX_DEVICES];   // the array's address on each device

// The address of `scratch` on the current device (looked up on the first
// call on that device, with that device current).
static int noalloc_scratch(void **out) {
    int dev = -1;
    ABBA_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= ABBA_MAX_DEVICES) {
        set_error("device %d is beyond the %d devices this library tracks", dev, ABBA_MAX_DEVICES);
        return ABBA_ERR_UNSUPPORTED;
    }
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void *p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
        if (!p) {
            set_error("hipGetSymbolAddress(scratch) returned a null address");
            return ABBA_ERR_HIP;
        }
        g_scratch_dev[dev] = p;
    }
    *out = g_scratch_dev[dev];
    return ABBA_OK;
}

int abba_project_noalloc(const abba_op *A, const void *x, void *y, int batch, void *stream) {
    if (!A || batch < 0 || (batch > 0 && (!x || !y))) {
        set_error("abba_project_noalloc: NULL argument or negative batch");
        return ABBA_ERR_ARG;
    }
    if (A->kind != ABBA_OP_JOSEPH) {
        set_error("abba_project_noalloc needs an ABBA_OP_JOSEPH operator");
        return ABBA_ERR_ARG;
    }
    if (batch == 0) return ABBA_OK;
    const size_t need = apply_scratch_bytes(A, batch);
    if (need > (size_t)ABBA_NOALLOC_SCRATCH_BYTES) {
        set_error("abba_project_noalloc: %d slices need %zu bytes of scratch, beyond its %zu-byte static buffer "
                  "(use abba_project with a workspace, or fewer slices per call)",
                  batch, need, (size_t)ABBA_NOALLOC_SCRATCH_BYTES);
        return ABBA_ERR_ARG;
    }
    void *scr = nullptr;
    int rc = noalloc_scratch(&scr);
    if (rc) return rc;
    return abba_project(A, x, y, batch, scr, ABBA_NOALLOC_SCRATCH_BYTES, stream);
}

// ------------------------------------------------------------ tuning ------
static void to_c(const TuneEntry &t, abba_tune *o) {
    o->a_path = t.a_path;
    o->a_jb = t.a_jb;
    o->b_g = t.b_g;
    o->czt = t.czt;
    o->a_rb = t.a_rb;
    o->a_occ = t.a_occ;
    o->a_tile = t.a_tile;
    o->a_vg = t.a_vg;
}

static void store_tuning(abba_op *op, const TuneEntry &e) {
    for (int i = 0; i < op->ntune; ++i)
        if (op->tune[i].batch == e.batch) {
            op->tune[i] = e;
            return;
        }
    if (op->ntune == MAX_TUNE) {   // forget the oldest entry
        for (int i = 1; i < MAX_TUNE; ++i) op->tune[i - 1] = op->tune[i];
        --op->ntune;
    }
    op->tune[op->ntune++] = e;
}

int abba_op_set_tuning(abba_op *op, int batch, const abba_tune *t) {
    if (!op || batch < 1) {
        set_error("abba_op_set_tuning: NULL operator or batch < 1");
        return ABBA_ERR_ARG;
    }
    if (!t) {
        for (int i = 0; i < op->ntune; ++i)
            if (op->tune[i].batch == batch) {
                for (int j = i + 1; j < op->ntune; ++j) op->tune[j - 1] = op->tune[j];
                --op->ntune;
                break;
            }
        return ABBA_OK;
    }
    if (t->a_occ < 0 || (t->a_occ > 0 && op->lds_cu / t->a_occ > 65536)) {
        set_error("abba_op_set_tuning: a_occ must be 0 or at least %d (LDS per CU / 64 KB)",
                  (op->lds_cu + 65535) / 65536);
        return ABBA_ERR_ARG;
    }
    if (t->a_tile != 0 && t->a_tile != -1 && t->a_tile != 8 && t->a_tile != 16) {
        set_error("abba_op_set_tuning: a_tile must be 0 (built-in), -1 (rows), 8 or 16");
        return ABBA_ERR_ARG;
    }
    if (t->a_vg < 0 || t->a_vg > 4096) {
        set_error("abba_op_set_tuning: a_vg must be 0 (built-in) or 1..4096 views per group");
        return ABBA_ERR_ARG;
    }
    store_tuning(op, TuneEntry{batch, t->a_path, t->a_jb, t->b_g, t->czt, t->a_rb, t->a_occ, t->a_tile, t->a_vg});
    return ABBA_OK;
}

int abba_op_get_tuning(const abba_op *op, int batch, abba_tune *t) {
    if (!op || !t) {
        set_error("abba_op_get_tuning: NULL argument");
        return ABBA_ERR_ARG;
    }
    for (int i = 0; i < op->ntune; ++i)
        if (op->tune[i].batch == batch) {
            to_c(op->tune[i], t);
            return 1;
        }
    return 0;
}

__global__ void tune_fill_k(float *p, int64_t n, int dt) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const float v = (float)((i * 2654435761ull) % 1000ull) * 1e-3f;   // a fixed pattern in [0, 1)
        if (dt == ABBA_F64) reinterpret_cast<double *>(p)[i] = v;
        else if (dt == ABBA_F32) p[i] = v;
        else reinterpret_cast<uint16_t *>(p)[i] = (uint16_t)(__float_as_uint(v) >> 16);
    }
}

// The autotuner's buffers: an input and an output of `batch` slices and the
// scratch of one apply, each 256-byte aligned.
static size_t tune_bytes(const abba_op *op, int batch, size_t *in_b, size_t *out_b) {
    const bool fwd = op->kind == ABBA_OP_JOSEPH;
    const int in_dt = fwd ? op->img_dtype : op->sino_dtype, out_dt = fwd ? op->sino_dtype : op->img_dtype;
    auto al = [](size_t v) { return (v + 255) / 256 * 256; };
    *in_b = al((size_t)batch * (fwd ? op->n : op->m) * dtype_size(in_dt));
    *out_b = al((size_t)batch * (fwd ? op->m : op->n) * dtype_size(out_dt));
    return *in_b + *out_b + al(apply_scratch_bytes(op, batch));
}

int abba_autotune_workspace(const abba_op *op, int batch, size_t *bytes) {
    if (!op || !bytes || batch < 1) {
        set_error("abba_autotune_workspace: operator and bytes are required, batch >= 1");
        return ABBA_ERR_ARG;
    }
    size_t a, b;
    *bytes = tune_bytes(op, batch, &a, &b);
    return ABBA_OK;
}

int abba_autotune(abba_op *op, int batch, int reps, void *workspace, size_t ws_bytes, void *stream,
                  abba_tune *best) {
    if (!op || batch < 1) {
        set_error("abba_autotune: NULL operator or batch < 1");
        return ABBA_ERR_ARG;
    }
    size_t in_b = 0, out_b = 0;
    const size_t need = tune_bytes(op, batch, &in_b, &out_b);
    if (check_ws("abba_autotune", need, workspace, ws_bytes)) return ABBA_ERR_ARG;

    if (!op || batch < 1) {
        set_error("abba_autotune: NULL operator or batch < 1");
        return ABBA_ERR_ARG;
    }
    if (reps < 1) reps = 3;
    const bool fwd = op->kind == ABBA_OP_JOSEPH;
    const int in_dt = fwd ? op->img_dtype : op->sino_dtype;
    const int64_t in_len = (int64_t)batch * (fwd ? op->n : op->m);
    TuneEntry cand[16];
    const int nc = cone_path(op) ? cone_tune_candidates(op, cand, 16)
                                                  : par2d_tune_candidates(op, cand, 16);
    hipStream_t st = (hipStream_t)stream;
    void *in = workspace, *out = (char *)workspace + in_b, *scr = (char *)workspace + in_b + out_b;
    const size_t scr_b = ws_bytes - in_b - out_b;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    int rc = ABBA_OK;
    double best_ms = 1e300, def_ms = 0.0;
    TuneEntry win{batch, -1, 0, 0, 0, 0};
    auto run = [&]() {
        return fwd ? abba_project(op, in, out, batch, scr, scr_b, stream)
                   : abba_backproject(op, in, out, batch, scr, scr_b, stream);
    };
    auto timed = [&](const TuneEntry &t, double *ms) -> int {
        op->trial = t;
        op->trial_on = 1;
        int r = run();   // warm-up (first launches of a kernel variant load its code)
        if (!r && hipEventRecord(e0, st) != hipSuccess) r = hip_fail(hipGetLastError(), "hipEventRecord");
        for (int i = 0; i < reps && !r; ++i) r = run();
        if (!r && hipEventRecord(e1, st) != hipSuccess) r = hip_fail(hipGetLastError(), "hipEventRecord");
        if (!r && hipEventSynchronize(e1) != hipSuccess) r = hip_fail(hipGetLastError(), "hipEventSynchronize");
        float f = 0.f;
        if (!r && hipEventElapsedTime(&f, e0, e1) != hipSuccess) r = hip_fail(hipGetLastError(), "hipEventElapsedTime");
        op->trial_on = 0;
        *ms = (double)f / reps;
        return r;
    };
    hipError_t e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    if (e != hipSuccess) rc = hip_fail(e, "abba_autotune set-up");
    if (!rc) {
        hipLaunchKernelGGL(tune_fill_k, dim3(1024), dim3(256), 0, st, (float *)in, in_len, in_dt);
        e = hipGetLastError();
        if (e != hipSuccess) rc = hip_fail(e, "tune_fill_k");
    }
    // the built-in rules twice: the first pass also brings the clocks up
    if (!rc) rc = timed(TuneEntry{batch, -1, 0, 0, 0, 0}, &def_ms);
    if (!rc) rc = timed(TuneEntry{batch, -1, 0, 0, 0, 0}, &def_ms);
    if (!rc) best_ms = def_ms;
    for (int i = 0; i < nc && !rc; ++i) {
        TuneEntry t = cand[i];
        t.batch = batch;
        double ms = 0.0;
        rc = timed(t, &ms);
        if (!rc && ms < best_ms) {
            best_ms = ms;
            win = t;
        }
    }
    op->trial_on = 0;
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (rc) return rc;
    store_tuning(op, win);
    if (best) {
        to_c(win, best);
        best->ms = best_ms;
        best->default_ms = def_ms;
        best->candidates = nc;
    }
    return ABBA_OK;
}

}  // extern "C"
