// Shared definitions of the hfmm HIP library (gfx950).
//
// Internal expansion basis.  The device keeps expansions in the basis of the
// Cartesian solid harmonics
//     R_n^m(v) = r^n P_n^m(cos a) e^{i m b} / (n+m)!          (regular)
//     S_n^m(v) = (n-m)! P_n^m(cos a) e^{i m b} / r^{n+1}       (irregular)
// (P_n^m with the Condon-Shortley phase of Eq. 8).  In the paper's
// normalisation (Eqs. 2, 3, 5, 6) r^n Y_n^m = R_n^m / A_n^m and
// Y_n^m / r^{n+1} = A_n^m S_n^m for m >= 0 (the quantity tabulated for M2L in
// Sec. 5.2 is S_n^m), so the device coefficients are
//     Mb_n^m = A_n^m M_n^m = sum_j q_j conj(R_n^m(x_j - c))
//     Lb_n^m = L_n^m / A_n^m = sum_j q_j conj(S_n^m(x_j - c))
// and, per level, they are scaled by the cell side h:
//     Mt_n = Mb_n / h^n,   Lt_n = Lb_n h^{n+1}.
// In these variables every translation is independent of the level, P2M and
// L2P work on (x - c)/h, and all magnitudes stay O(1).  Only m >= 0 is
// stored: X_n^{-m} = (-1)^m conj(X_n^m).  Real layout per cell, degree by
// degree: [Re X_n^0, Re X_n^1, Im X_n^1, ..., Re X_n^n, Im X_n^n], i.e. p*p
// reals; index n*n for m = 0 and n*n + 2m - 1 (Re), n*n + 2m (Im) for m > 0.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stddef.h>

#include <algorithm>
#include <vector>

#include "../../include/hfmm.h"

#define HFMM_ALIGN 256

namespace hfmm {

// ---------------------------------------------------------------------
// error handling
// ---------------------------------------------------------------------
struct HipError {
    hipError_t e;
};

#define HIP_TRY(expr)                              \
    do {                                           \
        hipError_t _e = (expr);                    \
        if (_e != hipSuccess) throw ::hfmm::HipError{_e}; \
    } while (0)

#define LAUNCH_CHECK() HIP_TRY(hipGetLastError())

// Wait for the work enqueued on s before a small read back is used.  A
// blocking wait wakes the host tens of microseconds after the copy lands;
// polling the stream for a short while returns within a few, and only
// longer work falls back to the blocking wait.
void stream_wait(hipStream_t s);

struct Status {
    int code;
};

// ---------------------------------------------------------------------
// arena: persistent allocations grow upwards, per-call temporaries grow
// downwards from the top and are released at the end of each call.
// ---------------------------------------------------------------------
struct Arena {
    char* base = nullptr;
    size_t cap = 0, lo = 0, hi = 0;
    size_t need = 0;  // bytes that would have sufficed (after a failure)
    size_t peak = 0;  // the most bytes in use at once so far

    static size_t align(size_t b) { return (b + HFMM_ALIGN - 1) / HFMM_ALIGN * HFMM_ALIGN; }

    void init(void* p, size_t bytes) {
        base = (char*)p;
        size_t skew = (HFMM_ALIGN - ((uintptr_t)base % HFMM_ALIGN)) % HFMM_ALIGN;
        base += skew;
        cap = bytes > skew ? (bytes - skew) / HFMM_ALIGN * HFMM_ALIGN : 0;
        lo = 0;
        hi = cap;
        need = 0;
        peak = 0;
    }
    void fail(size_t bytes) {
        size_t want = lo + align(bytes) + (cap - hi) + HFMM_ALIGN;
        if (want > need) need = want;
        throw Status{HFMM_E_NOMEM};
    }
    template <typename T>
    T* up(size_t count) {
        size_t b = align(count * sizeof(T) + 1);
        if (lo + b > hi) fail(count * sizeof(T));
        T* p = (T*)(base + lo);
        lo += b;
        peak = std::max(peak, used());
        return p;
    }
    template <typename T>
    T* down(size_t count) {
        size_t b = align(count * sizeof(T) + 1);
        if (lo + b > hi) fail(count * sizeof(T));
        hi -= b;
        peak = std::max(peak, used());
        return (T*)(base + hi);
    }
    size_t free_bytes() const { return hi - lo; }
    void release_temps() { hi = cap; }
    size_t used() const { return lo + (cap - hi); }
};

// ---------------------------------------------------------------------
// tree records
// ---------------------------------------------------------------------
struct Cell {
    int32_t first, count;   // particle range in sorted order
    int32_t parent, child;  // parent cell, first child (-1 for a leaf)
    int32_t ix, iy, iz;     // integer coordinates at this level
    int16_t level;
    int8_t nchild;
    uint8_t mask;           // bit o set when the child of octant o exists
};
static_assert(sizeof(Cell) == 32, "Cell must be 32 bytes");

// A target box.  Every target is evaluated in the box it is binned into:
// a leaf of the source tree (kind 0: leaf = host = that cell), a
// source-free leaf added under a split cell, the octant of the split cell
// that holds the target (kind 1: leaf = -1, host = the split cell), or,
// outside the root cube, the level-0 cube of the extended grid holding it
// (kind 2: leaf = host = -1).  The host is the cell whose local expansion
// covers the box.  For self-evaluation the boxes are the leaves.
struct TBox {
    int32_t first, count;   // targets [first, first + count) in sorted order
    int32_t host, leaf;
    int32_t ix, iy, iz;     // coordinates at `level` (any sign outside the root)
    int16_t level;
    int16_t kind;
};
static_assert(sizeof(TBox) == 32, "TBox must be 32 bytes");

// The box's geometry as a cell record (for adjacency and centres).
__host__ __device__ inline Cell box_cell(const TBox& b) {
    Cell c;
    c.first = c.count = 0;
    c.parent = c.child = -1;
    c.ix = b.ix;
    c.iy = b.iy;
    c.iz = b.iz;
    c.level = b.level;
    c.nchild = 0;
    c.mask = 0;
    return c;
}

// The targets of one evaluation as the kernels see them.  Lists are rows of
// a CSR either by box (separate targets) or by the box's own leaf (self-
// evaluation: the tree's lists).
struct Targets {
    const TBox* box;
    const int32_t* box_of;   // sorted target -> box
    const float4* p32;       // sorted targets, FP32 relative to their box centre
    const double4* p64;      // sorted targets, FP64
    const int32_t* perm;     // sorted target -> output index
    int64_t n;
    int32_t nbox;
    int32_t by_leaf;
};
__device__ __forceinline__ int list_row(const Targets& tg, int b, const TBox& bx) {
    return tg.by_leaf ? bx.leaf : b;
}

// Device status word: data errors found by the kernels (hfmm_status).
enum StatusBits : int32_t {
    ST_SRC_NONFINITE = 1,    // a source coordinate is NaN or infinite
    ST_TGT_NONFINITE = 2,    // a target coordinate is NaN or infinite
    ST_MASS_NONFINITE = 4,   // a mass is NaN or infinite
    ST_OVERFLOW = 8          // a traversal stack overflowed (lists incomplete)
};

struct Root {
    double b[3];   // lower corner of the root cube
    double R;      // half width
    double scale;  // 2^21 / (2R)
    int32_t nbad;  // non-finite input coordinates
    int32_t pad_i;
    double pad[2];
};

// per-call timing of the phases (host wall clock around synchronised steps
// is not used; these are filled from hip events when enabled)
struct Tree {
    int device = 0;
    int64_t n = 0;                   // sources (the particles of the tree)
    int leaf_max = 64;
    Arena arena;
    Root root_h;
    Root* root = nullptr;            // device copy
    // particles, sorted
    uint64_t* keys = nullptr;
    int32_t* perm = nullptr;
    double *xs = nullptr, *ys = nullptr, *zs = nullptr;
    float4* p32 = nullptr;           // x, y, z, m (FP32)
    double4* p64 = nullptr;          // x, y, z, m (FP64)
    int32_t* leaf_of = nullptr;      // sorted particle -> leaf cell
    int32_t* status = nullptr;       // device status word (StatusBits)
    int32_t* moved = nullptr;        // device flag of the last refit
    bool stale = false;              // a refit left the tree unusable
    // self-evaluation view: one box per leaf, sorted particle -> leaf index
    TBox* leaf_boxes = nullptr;
    int32_t* leaf_box_of = nullptr;
    int sort_bits = 0;
    // cells
    Cell* cells = nullptr;
    int32_t ncells = 0, depth = 0;
    std::vector<int32_t> level_start;  // host, depth + 2 entries
    int32_t* leaves = nullptr;
    int32_t nleaves = 0;
    size_t mark_tree = 0;
    // upward state
    int up_p = 0, up_method = -1, up_prec = -1;
    int ldm = 0;                     // row length of M and L: p*p padded to 16
    double* M = nullptr;             // [ncells + 1][ldm] FP64 scaled R-basis, last row 0
    double* cen = nullptr;           // [ncells][4] expansion centre, 1 / side
    void* Mk = nullptr;              // M2L operand copy [(ncells+1)][Kp]
    size_t mark_up = 0;
    // FMM lists (independent of p and masses)
    bool fmm_lists = false;
    int32_t* coll = nullptr;         // [ncells][27] colleagues, -1 padded
    int32_t* vsrc = nullptr;         // [ncells][216] V list by slot, -1 empty
    uint8_t* cflag = nullptr;        // [ncells] bit 0: a colleague is a leaf;
                                     // bit 1: so is one of a proper ancestor
    // U, W, X share one item array; offsets are absolute into it
    int32_t *u_off = nullptr, *u_items = nullptr;
    int32_t *w_off = nullptr, *w_items = nullptr;
    int32_t *x_off = nullptr, *x_items = nullptr;
    int32_t* v_off = nullptr;        // V counts as offsets (items: vsrc)
    int32_t* x_cells = nullptr;  // cells with an X list (P2L targets)
    int32_t n_xcells = 0;
    int64_t n_u = 0, n_v = 0, n_w = 0, n_x = 0;
    int32_t* m2l_order = nullptr;    // targets (level >= 2) by (level, octant)
    int32_t* m2l_torder = nullptr;   // the same targets by (octant, level)
    int32_t* m2l_tiles = nullptr;    // per tile: start into m2l_torder, count, octant
    std::vector<int32_t> m2l_tiles_h;  // host copy (the source of the upload)
    int32_t n_m2l_tiles = 0;
    uint32_t* m2l_tmask = nullptr;   // per tile: slots with a source (8 words)
    int32_t* m2l_tpre = nullptr;     // per tile: M2L work items before it (+ total)
    size_t mark_lists = 0;
    // treecode lists (bh_theta = kFmmListTheta: built from the FMM lists)
    double bh_theta = -1.0;
    int32_t *a_off = nullptr, *a_items = nullptr;   // accepted (M2P)
    int32_t *b_off = nullptr, *b_items = nullptr;   // P2P
    int64_t n_a = 0, n_b = 0;
    // operator tables (per p and precision)
    int ops_p = 0, ops_prec = -1;
    bool ops_rot = false;            // the tables are the rotation M2L's
    void* T = nullptr;               // M2L matrices
    size_t mark_ops = 0;
    int32_t* bexp = nullptr;         // low-precision M2L row exponents
    size_t mark_bh = 0;
    // last evaluation
    double* L = nullptr;             // [ncells + 1][ldm] FP64 local expansions
    double* xl_m2m = nullptr;        // 8 octant operators, matrix-core layout
    double* xl_l2l = nullptr;
    std::vector<int32_t> m2l_level_start;  // host: level -> start in m2l_order
    int ev_p = 0, ev_method = -1;
    int64_t p2p_pairs = 0, m2l_pairs = 0;
    // the last evaluation's targets (separate targets: boxes, sorted
    // positions and lists live in the arena until the next upward pass or
    // evaluation)
    bool tg_sep = false;
    Targets tg{};
    int64_t tg_near = 0, tg_far = 0;     // list entries of the separate targets
    int32_t *tn_off = nullptr, *tn_items = nullptr;  // near (P2P) lists by box
    int32_t *tf_off = nullptr, *tf_items = nullptr;  // far (M2P) lists by box
    // phase timers (HIP events on the caller's stream)
    bool timing = false;
    hipEvent_t ev[2 * HFMM_PHASES] = {};
    bool ev_used[HFMM_PHASES] = {};
};

enum Phase {
    PH_BUILD = 0, PH_LISTS, PH_UPWARD, PH_OPS, PH_M2L, PH_DOWN, PH_FAR, PH_P2P, PH_BH, PH_M2L_PREP
};

// records an event pair around a scope when the tree is timed
struct PhaseTimer {
    Tree& t;
    int ph;
    hipStream_t s;
    PhaseTimer(Tree& t_, int ph_, hipStream_t s_) : t(t_), ph(ph_), s(s_) {
        if (t.timing) HIP_TRY(hipEventRecord(t.ev[2 * ph], s));
    }
    ~PhaseTimer() {
        if (t.timing) {
            if (hipEventRecord(t.ev[2 * ph + 1], s) == hipSuccess) t.ev_used[ph] = true;
        }
    }
};

// ---------------------------------------------------------------------
// device helpers
// ---------------------------------------------------------------------
__host__ __device__ constexpr int tri(int n, int m) { return n * (n + 1) / 2 + m; }
__host__ __device__ constexpr int ntri(int p) { return p * (p + 1) / 2; }
__host__ __device__ constexpr int round_up(int a, int b) { return (a + b - 1) / b * b; }

// real-layout index of (n, m >= 0, part) with part 0 = Re, 1 = Im
__host__ __device__ constexpr int ridx(int n, int m, int part) {
    return m == 0 ? n * n : n * n + 2 * m - 1 + part;
}

// Reciprocal square root: FP32 from the hardware estimate (1 ulp); FP64 from
// the estimate refined by two Newton steps y <- y + y (1 - x y^2) / 2 (each
// squares the relative error), full double precision at a fraction of a
// correctly rounded sqrt and divide.  x = 0 gives inf (FP32) or NaN (FP64);
// callers mask such pairs.
// four-wide vector of the compute type
template <typename T>
struct Vec4;
template <>
struct Vec4<float> {
    using type = float4;
};
template <>
struct Vec4<double> {
    using type = double4;
};

__device__ __forceinline__ float rsqrt_fast(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ __forceinline__ double rsqrt_fast(double x) {
    double y = __builtin_amdgcn_rsq(x);
#pragma unroll
    for (int it = 0; it < 2; ++it) {
        const double e = fma(-x, y * y, 1.0);
        y = fma(0.5 * y, e, y);
    }
    return y;
}

// wave-level helpers (64 lanes): lanes below this one, an exclusive scan
// over the wave, and an LDS fence between lanes of one wave
__device__ __forceinline__ uint64_t lanes_below(int lane) {
    return lane == 0 ? 0ull : (~0ull >> (64 - lane));
}
__device__ __forceinline__ int wave_excl_scan(int v, int lane, int& total) {
    int x = v;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const int u = __shfl_up(x, d, 64);
        if (lane >= d) x += u;
    }
    total = __shfl(x, 63, 64);
    return x - v;
}
__device__ __forceinline__ void wave_lds_fence() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}
// The owner lane of each of `width` consecutive slots of a packed sequence:
// lane j holds a run [off, off + cnt) of it; the runs are in lane order.  The
// lane whose run starts in the window (or covers its first slot) marks that
// slot in own[], then a running maximum over the lanes fills the rest.
// Returns the owner of slot pb + lane (meaningful for slots < total).
__device__ __forceinline__ int wave_run_owner(int* own, int off, int cnt, int pb, int width,
                                              int lane) {
    wave_lds_fence();
    own[lane] = -1;
    if (cnt > 0 && off < pb + width && off + cnt > pb) own[max(off - pb, 0)] = lane;
    wave_lds_fence();
    int o = own[lane];
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const int u = __shfl_up(o, d, 64);
        if (lane >= d) o = max(o, u);
    }
    return o;
}

// Exponent of the low-precision M2L operand scale of one level; the
// per-level maxima start at the byte-fill sentinel 0x80808080, which a level
// without a nonzero coefficient keeps: its scale is then 2^0.
__device__ __forceinline__ int level_exp(const int32_t* levexp, int level) {
    const int e = levexp[level];
    return e == (int32_t)0x80808080 ? 0 : e;
}

// cell side and centre from the integer coordinates (FP64, no contraction so
// that host and device agree bit for bit)
#pragma clang fp contract(off)
__host__ __device__ inline double cell_side(const Root& r, int level) {
    return (2.0 * r.R) / (double)(1u << level);
}
__host__ __device__ inline void cell_centre(const Root& r, const Cell& c,
                                            double out[3]) {
    double h = cell_side(r, c.level);
    out[0] = r.b[0] + ((double)c.ix + 0.5) * h;
    out[1] = r.b[1] + ((double)c.iy + 0.5) * h;
    out[2] = r.b[2] + ((double)c.iz + 0.5) * h;
}
// a position within (1/2 + slack) sides of the centre of cell c along each
// axis (false for non-finite positions)
__host__ __device__ inline bool within_cell(const Root& r, const Cell& c, double slack,
                                            double x, double y, double z) {
    double o[3];
    cell_centre(r, c, o);
    const double lim = (0.5 + slack) * cell_side(r, c.level);
    return fabs(x - o[0]) <= lim && fabs(y - o[1]) <= lim && fabs(z - o[2]) <= lim;
}
#pragma clang fp contract(on)

// closed boxes of two cells intersect (levels may differ)
__device__ inline bool cells_adjacent(const Cell& a, const Cell& b) {
    const Cell& A = a.level <= b.level ? a : b;
    const Cell& B = a.level <= b.level ? b : a;
    int64_t f = (int64_t)1 << (B.level - A.level);
    int64_t ia[3] = {A.ix, A.iy, A.iz}, ib[3] = {B.ix, B.iy, B.iz};
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        if (ib[k] > (ia[k] + 1) * f) return false;
        if (ib[k] + 1 < ia[k] * f) return false;
    }
    return true;
}

// Regular solid harmonics R_n^m(x, y, z), n < NP, m = 0..n (triangular).
//   R_0^0 = 1,  R_m^m = -(x + i y) / (2m) R_{m-1}^{m-1},
//   R_{n+1}^m = ((2n+1) z R_n^m - r^2 R_{n-1}^m) / ((n+1)^2 - m^2)
template <typename T, int NP>
__device__ inline void solid_regular(T x, T y, T z, T* re, T* im) {
    const T r2 = x * x + y * y + z * z;
    re[0] = T(1);
    im[0] = T(0);
#pragma unroll
    for (int m = 0; m < NP; ++m) {
        const int d = tri(m, m);
        if (m > 0) {
            const int s = tri(m - 1, m - 1);
            const T c = T(-1) / T(2 * m);
            re[d] = c * (x * re[s] - y * im[s]);
            im[d] = c * (x * im[s] + y * re[s]);
        }
        if (m + 1 < NP) {
            const int u = tri(m + 1, m);
            const T c = T(2 * m + 1) / T((m + 1) * (m + 1) - m * m);
            re[u] = c * z * re[d];
            im[u] = c * z * im[d];
        }
#pragma unroll
        for (int n = m + 1; n + 1 < NP; ++n) {
            const int a = tri(n, m), b = tri(n - 1, m), u = tri(n + 1, m);
            const T c = T(1) / T((n + 1) * (n + 1) - m * m);
            re[u] = (T(2 * n + 1) * z * re[a] - r2 * re[b]) * c;
            im[u] = (T(2 * n + 1) * z * im[a] - r2 * im[b]) * c;
        }
    }
}

// Irregular solid harmonics S_n^m(x, y, z), n < NP, m = 0..n.
//   S_0^0 = 1/r,  S_m^m = -(2m-1)(x + i y)/r^2 S_{m-1}^{m-1},
//   S_{n+1}^m = ((2n+1) z S_n^m - (n^2 - m^2) S_{n-1}^m) / r^2
template <typename T, int NP>
__device__ inline void solid_irregular(T x, T y, T z, T* re, T* im) {
    const T r2 = x * x + y * y + z * z;
    const T ir2 = T(1) / r2;
    re[0] = sqrt(ir2);
    im[0] = T(0);
#pragma unroll
    for (int m = 0; m < NP; ++m) {
        const int d = tri(m, m);
        if (m > 0) {
            const int s = tri(m - 1, m - 1);
            const T c = T(-(2 * m - 1)) * ir2;
            re[d] = c * (x * re[s] - y * im[s]);
            im[d] = c * (x * im[s] + y * re[s]);
        }
        if (m + 1 < NP) {
            const int u = tri(m + 1, m);
            const T c = T(2 * m + 1) * z * ir2;
            re[u] = c * re[d];
            im[u] = c * im[d];
        }
#pragma unroll
        for (int n = m + 1; n + 1 < NP; ++n) {
            const int a = tri(n, m), b = tri(n - 1, m), u = tri(n + 1, m);
            re[u] = (T(2 * n + 1) * z * re[a] - T(n * n - m * m) * re[b]) * ir2;
            im[u] = (T(2 * n + 1) * z * im[a] - T(n * n - m * m) * im[b]) * ir2;
        }
    }
}

// ---------------------------------------------------------------------
// host helpers (implemented in the .hip files)
// ---------------------------------------------------------------------
inline int grid_for(int64_t n, int block) { return (int)((n + block - 1) / block); }

// device-wide exclusive scan of int32 (returns nothing; total written to
// out[n] when out has n+1 entries)
void scan_exclusive_i32(const int32_t* in, int32_t* out, int64_t n, Arena& A,
                        hipStream_t s, int32_t* total2 = nullptr);
// stable LSD radix sort of key bits [lo_bit, hi_bit); the input pairs are
// only read, the sorted pairs land in (keys_out, vals_out)
void radix_sort_pairs(const uint64_t* keys, const int32_t* vals, uint64_t* keys_out,
                      int32_t* vals_out, int64_t n, int lo_bit, int hi_bit, Arena& A,
                      hipStream_t s);

void build_tree(Tree& t, const double* x, const double* y, const double* z, hipStream_t s);
bool refit_tree(Tree& t, const double* x, const double* y, const double* z, double slack,
                hipStream_t s);
void build_fmm_lists(Tree& t, hipStream_t s);
void build_bh_lists(Tree& t, double theta, hipStream_t s);
void set_last_required(size_t bytes);  // for hfmm_last_required_bytes
void build_fmmlist_treecode_lists(Tree& t, bool fill_far, hipStream_t s);
void fill_fmmlist_far_items(const Tree& t, int32_t* dst, hipStream_t s);
constexpr double kFmmListTheta = -2.0;
void upward_pass(Tree& t, const double* m, int p, int method, int precision,
                 hipStream_t s);
void evaluate(Tree& t, const double* tx, const double* ty, const double* tz, int64_t nt,
              int p, double theta, int method, int precision, double eps2, void* phi,
              void* ax, void* ay, void* az, hipStream_t s);
void direct_sum(const double* x, const double* y, const double* z,
                const double* m, int64_t ns, const double* tx, const double* ty,
                const double* tz, int64_t nt, int precision, double eps2,
                Arena& A, void* phi, void* ax, void* ay, void* az,
                hipStream_t s);

// far-field and near-field kernels (launch wrappers)
void launch_p2p(const Tree& t, const Targets& tg, int precision, double eps2,
                const int32_t* src_off, const int32_t* src_items, const void* far,
                void* phi, void* ax, void* ay, void* az, hipStream_t s);

// separate targets (targets.hip)
Targets self_targets(const Tree& t);
Targets bin_targets(Tree& t, const double* tx, const double* ty, const double* tz,
                    int64_t nt, hipStream_t s);
enum BoxListMode { BOX_FMM = 0, BOX_TREECODE = 1, BOX_TREECODE_FULL = 2 };
void build_box_lists(Tree& t, const Targets& tg, int mode, hipStream_t s);
void build_bh_box_lists(Tree& t, const Targets& tg, double theta, hipStream_t s);

}  // namespace hfmm
