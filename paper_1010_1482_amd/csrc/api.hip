// C ABI of the hfmm library: argument checks, arena layout and the order of
// the passes (Sec. 2, Fig. 1):
//   build:    bbox, keys, sort, cells                       (tree.hip)
//   upward:   P2M at the leaves, M2M to the root            (expansions.hip)
//   evaluate: the targets (the sources, or separate points binned into the
//             tree: targets.hip), then
//             FMM      M2L (+P2L), L2L, L2P (+M2P), P2P     (m2l, expansions, p2p)
//             treecode M2P, P2P (Barnes-Hut lists, or the FMM lists)
#include "common.hpp"
#include "expansions.hpp"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdlib>
#include <new>
#include <vector>

namespace hfmm {

__global__ void k_export_cells(const Cell* __restrict__ cells, int nc, int32_t* __restrict__ o) {
    int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= nc) return;
    Cell x = cells[c];
    int32_t* d = o + (int64_t)c * 9;
    d[0] = x.level;
    d[1] = x.ix;
    d[2] = x.iy;
    d[3] = x.iz;
    d[4] = x.first;
    d[5] = x.count;
    d[6] = x.parent;
    d[7] = x.child;
    d[8] = x.nchild;
}

__global__ void k_v_count(const int32_t* __restrict__ vsrc, int nc, int32_t* __restrict__ cnt) {
    int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= nc) return;
    int k = 0;
    for (int q = 0; q < 216; ++q) k += vsrc[(int64_t)c * 216 + q] >= 0;
    cnt[c] = k;
}

__global__ void k_v_fill(const int32_t* __restrict__ vsrc, int nc, const int32_t* __restrict__ off,
                         int32_t* __restrict__ items) {
    int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= nc) return;
    int k = off[c];
    for (int q = 0; q < 216; ++q) {
        int v = vsrc[(int64_t)c * 216 + q];
        if (v >= 0) items[k++] = v;
    }
}

__global__ void k_offsets_minus(const int32_t* __restrict__ in, int64_t n, int32_t base,
                                int32_t* __restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = in[i] - base;
}

__global__ void k_status_clear(int32_t* status, int32_t bits) {
    if (threadIdx.x == 0) atomicAnd(status, ~bits);
}

// per target, in the caller's order: kind, level, ix, iy, iz, host, leaf and
// the index of its box
__global__ void k_export_targets(Targets tg, int32_t* __restrict__ o) {
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= tg.n) return;
    const int b = tg.box_of[s];
    const TBox x = tg.box[b];
    int32_t* d = o + (int64_t)tg.perm[s] * 8;
    d[0] = x.kind;
    d[1] = x.level;
    d[2] = x.ix;
    d[3] = x.iy;
    d[4] = x.iz;
    d[5] = x.host;
    d[6] = x.leaf;
    d[7] = b;
}

static void clear_status(Tree& t, int32_t bits, hipStream_t s) {
    hipLaunchKernelGGL(k_status_clear, dim3(1), dim3(64), 0, s, t.status, bits);
    LAUNCH_CHECK();
}

static void check_p(int p) {
    if (p < 1 || p > HFMM_MAX_P) throw Status{HFMM_E_UNSUPPORTED};
}
// the FMM with the dense (matrix-core) or the rotation-based M2L
static bool is_fmm(int method) { return method == HFMM_FMM || method == HFMM_FMM_ROT; }
// the methods whose upward pass is the FMM's (geometric centres, FMM lists)
static bool fmm_upward(int method) {
    return is_fmm(method) || method == HFMM_TREECODE_FMMLIST;
}
static bool tree_method(int method) {
    return is_fmm(method) || method == HFMM_TREECODE || method == HFMM_TREECODE_FMMLIST;
}

static void check_precision(int precision) {
    if (precision < HFMM_FP64 || precision > HFMM_M2L_FP16X3) throw Status{HFMM_E_UNSUPPORTED};
}

void upward_pass(Tree& t, const double* m, int p, int method, int precision, hipStream_t s) {
    check_p(p);
    check_precision(precision);
    if (!tree_method(method)) throw Status{HFMM_E_UNSUPPORTED};
    if (method == HFMM_FMM_ROT && precision != HFMM_FP64 && precision != HFMM_FP32)
        throw Status{HFMM_E_UNSUPPORTED};
    if (!m && t.n > 0) throw Status{HFMM_E_INVAL};
    Arena& A = t.arena;
    A.release_temps();
    clear_status(t, ST_MASS_NONFINITE, s);
    t.tg_sep = false;
    t.tg = Targets{};
    if (fmm_upward(method)) {
        if (!t.fmm_lists) {
            A.lo = t.mark_tree;
            PhaseTimer pt(t, PH_LISTS, s);
            build_fmm_lists(t, s);
        }
        A.lo = t.mark_lists;
    } else {
        A.lo = t.mark_tree;
        t.fmm_lists = false;
    }
    t.a_off = nullptr;
    t.bh_theta = -1.0;
    t.T = nullptr;
    t.ops_p = 0;
    t.up_p = 0;
    const int P = p * p;
    int RB, KQ, ld;
    m2l_layout(p, precision, RB, KQ, ld);
    t.ldm = (P + 15) / 16 * 16;
    PhaseTimer pt(t, PH_UPWARD, s);
    if (fmm_upward(method)) prepare_xlat_ops(t, p, s);
    t.cen = (double*)A.up<double4>(t.ncells);
    t.M = A.up<double>((size_t)(t.ncells + 1) * t.ldm);
    HIP_TRY(hipMemsetAsync(t.M + (size_t)t.ncells * t.ldm, 0, sizeof(double) * t.ldm, s));
    t.Mk = nullptr;
    t.mark_up = A.lo;
    fill_masses(t, m, s);
    compute_centres(t, method, s);
    const bool fp64 = precision == HFMM_FP64;
    run_p2m(t, p, fp64, s);
    if (fmm_upward(method))
        run_m2m_mfma(t, p, s);
    else
        run_m2m(t, p, s);
    A.release_temps();
    t.up_p = p;
    t.up_method = method;
    t.up_prec = precision;
}

// M2L (+ P2L) and L2L: the local expansions of every cell; rot: the
// rotation-based M2L instead of the dense operators
static void downward_pass(Tree& t, int p, int precision, bool rot, hipStream_t s) {
    Arena& A = t.arena;
    const bool fp64 = precision == HFMM_FP64;
    {
        PhaseTimer pt(t, PH_OPS, s);
        if (rot)
            prepare_rot_ops(t, p, precision, s);
        else
            prepare_m2l_ops(t, p, precision, s);
    }
    t.L = A.up<double>((size_t)(t.ncells + 1) * t.ldm);
    const size_t row = sizeof(double) * t.ldm;
    HIP_TRY(hipMemsetAsync(t.L + (size_t)t.ncells * t.ldm, 0, row, s));
    if (t.depth >= 2) {
        // M2L partial results: at most as many as half the free arena holds
        // (up to 64: small problems spread their few tiles over more blocks),
        // as many as the launch uses
        const bool mf = !rot && m2l_uses_mfma(p, precision);
        int max_parts = 64;
        const size_t esz = fp64 ? 8 : 4;
        while (max_parts > 1 &&
               (size_t)max_parts * t.ncells * t.ldm * esz > A.free_bytes() / 2)
            --max_parts;
        int nb_unused = 0;
        const int parts_cap =
            mf ? std::max(1, m2l_plan(t, p, precision, max_parts, nb_unused)) : 1;
        void* lm = A.down<char>((size_t)parts_cap * t.ncells * t.ldm * esz);
        int32_t* levexp = A.down<int32_t>(32);
        double* LX = nullptr;
        if (t.n_x > 0) LX = A.down<double>((size_t)t.ncells * t.ldm);
        int64_t stride = 0;
        int parts;
        parts = rot ? run_m2l_rot(t, p, precision, lm, stride, s)
                    : run_m2l(t, p, precision, lm, stride, mf ? max_parts : 1, levexp, s);
        PhaseTimer pt(t, PH_DOWN, s);
        if (LX) {
            HIP_TRY(hipMemsetAsync(LX, 0, row * t.ncells, s));
            run_p2l(t, p, fp64, LX, s);
        }
        HIP_TRY(hipMemsetAsync(t.L, 0, row * t.level_start[2], s));
        const bool lowp = mf && precision >= HFMM_M2L_BF16;
        run_l2l_mfma(t, p, lm, fp64, parts, stride, LX, lowp ? t.bexp : nullptr,
                     lowp ? levexp : nullptr, s);
    } else {
        HIP_TRY(hipMemsetAsync(t.L, 0, row * t.ncells, s));
    }
    A.release_temps();
}

// HFMM_VALIDATE=1: the separate targets' boxes and lists are read back and
// checked on the host before any kernel uses them (ranges, kinds, cell
// indices, the permutation, list offsets and items); a violation returns
// HFMM_E_STATE.  A debugging aid, off by default.
static bool validate_on() {
    static const bool on = [] {
        const char* e = std::getenv("HFMM_VALIDATE");
        return e && e[0] == '1';
    }();
    return on;
}

template <typename X>
static std::vector<X> fetch(const X* d, int64_t n, hipStream_t s) {
    std::vector<X> h((size_t)std::max<int64_t>(n, 0));
    if (n > 0) HIP_TRY(hipMemcpyAsync(h.data(), d, sizeof(X) * n, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    return h;
}

static void validate_targets(const Tree& t, const Targets& tg, const int32_t* off_a,
                             const int32_t* items_a, int64_t na, const int32_t* off_b,
                             const int32_t* items_b, int64_t nb, hipStream_t s) {
    const auto box = fetch(tg.box, tg.nbox, s);
    const auto box_of = fetch(tg.box_of, tg.n, s);
    const auto perm = fetch(tg.perm, tg.n, s);
    auto bad = [] { throw Status{HFMM_E_STATE}; };
    int64_t next = 0;
    for (int b = 0; b < tg.nbox; ++b) {
        const TBox& x = box[b];
        if (x.first != next || x.count < 1 || x.first + (int64_t)x.count > tg.n) bad();
        next = x.first + (int64_t)x.count;
        if (x.host < -1 || x.host >= t.ncells || x.leaf < -1 || x.leaf >= t.ncells) bad();
        if (x.kind == 0 && (x.leaf < 0 || x.host != x.leaf)) bad();
        if (x.kind == 1 && (x.leaf != -1 || x.host < 0)) bad();
        if (x.kind == 2 && (x.leaf != -1 || x.host != -1 || x.level != 0)) bad();
        if (x.kind < 0 || x.kind > 2) bad();
        for (int64_t k = x.first; k < next; ++k)
            if (box_of[k] != b) bad();
    }
    if (next != tg.n) bad();
    std::vector<char> seen((size_t)tg.n, 0);
    for (int64_t k = 0; k < tg.n; ++k) {
        if (perm[k] < 0 || perm[k] >= tg.n || seen[perm[k]]) bad();
        seen[perm[k]] = 1;
    }
    const int32_t* offs[2] = {off_a, off_b};
    const int32_t* its[2] = {items_a, items_b};
    const int64_t tots[2] = {na, nb};
    for (int w = 0; w < 2; ++w) {
        const auto off = fetch(offs[w], (int64_t)tg.nbox + 1, s);
        const auto it = fetch(its[w], tots[w], s);
        if (off[0] != 0 || off[tg.nbox] != tots[w]) bad();
        for (int b = 0; b < tg.nbox; ++b)
            if (off[b + 1] < off[b]) bad();
        for (int64_t e = 0; e < tots[w]; ++e)
            if (it[e] < 0 || it[e] >= t.ncells) bad();
    }
}

// One evaluation at the sources (tx == nullptr) or at nt separate targets
// binned into the tree.  FMM: M2L, L2L, then per target box L2P of its host
// cell's local expansion, M2P over its far list and P2P over its near list
// (the tree's W and U lists for the leaves; for separate targets the lists
// of every box, with V by M2P and X by P2P for a box without sources).
// Treecode: M2P and P2P over the boxes' Barnes-Hut lists, or over the FMM
// lists (the treecode of Sec. 4).
void evaluate(Tree& t, const double* tx, const double* ty, const double* tz, int64_t nt, int p,
              double theta, int method, int precision, double eps2, void* phi, void* ax,
              void* ay, void* az, hipStream_t s) {
    Arena& A = t.arena;
    A.release_temps();
    const bool sep = tx != nullptr;
    const bool fp64 = precision == HFMM_FP64;
    clear_status(t, ST_TGT_NONFINITE | ST_OVERFLOW, s);
    t.tg_sep = false;
    t.tg = Targets{};
    if (sep || is_fmm(method)) {
        // separate targets live above the upward data (and the local
        // expansions); the treecodes' cached self lists are given up
        A.lo = t.mark_up;
        t.a_off = nullptr;
        t.bh_theta = -1.0;
    }
    // the rotation M2L where the matrix cores take no dense operator (FP32
    // above p = 13, FP64 above p = 11): O(p^3) beats the vector units' p^4
    const bool rot = method == HFMM_FMM_ROT ||
                     ((precision == HFMM_FP32 || precision == HFMM_FP64) &&
                      !m2l_uses_mfma(p, precision));
    if (is_fmm(method)) downward_pass(t, p, precision, rot, s);
    Targets tg;
    const int32_t *far_off, *far_items, *near_off, *near_items;
    int64_t n_far;
    bool walk = false;
    {
        PhaseTimer pt(t, PH_BH, s);
        if (sep) {
            tg = bin_targets(t, tx, ty, tz, nt, s);
            if (is_fmm(method))
                build_box_lists(t, tg, BOX_FMM, s);
            else if (method == HFMM_TREECODE_FMMLIST)
                build_box_lists(t, tg, p == 3 ? BOX_TREECODE : BOX_TREECODE_FULL, s);
            else
                build_bh_box_lists(t, tg, theta, s);
            far_off = t.tf_off;
            far_items = t.tf_items;
            n_far = t.tg_far;
            near_off = t.tn_off;
            near_items = t.tn_items;
            walk = method == HFMM_TREECODE_FMMLIST && p == 3;
            if (validate_on())
                validate_targets(t, tg, far_off, far_items, n_far, near_off, near_items,
                                 t.tg_near, s);
        } else {
            tg = self_targets(t);
            if (is_fmm(method)) {
                far_off = t.w_off;
                far_items = t.w_items;
                n_far = t.n_w;
                near_off = t.u_off;
                near_items = t.u_items;
            } else {
                if (method == HFMM_TREECODE_FMMLIST)
                    build_fmmlist_treecode_lists(t, p != 3, s);
                else
                    build_bh_lists(t, theta, s);
                walk = method == HFMM_TREECODE_FMMLIST && p == 3;
                // at p = 3 over the FMM lists the far kernel takes W and
                // reads the V lists itself
                far_off = walk ? t.w_off : t.a_off;
                far_items = walk ? t.w_items : t.a_items;
                n_far = walk ? t.n_w : t.n_a;
                near_off = t.b_off;
                near_items = t.b_items;
            }
        }
    }
    void* far = A.down<char>((size_t)4 * tg.n * (fp64 ? 8 : 4));
    {
        PhaseTimer pt(t, PH_FAR, s);
        if (is_fmm(method))
            run_far(t, tg, p, fp64, far_off, far_items, n_far, far, s);
        else
            run_treecode_far(t, tg, p, fp64, walk, far_off, far_items, far, s);
    }
    {
        PhaseTimer pt(t, PH_P2P, s);
        launch_p2p(t, tg, precision, eps2, near_off, near_items, far, phi, ax, ay, az, s);
    }
    t.tg = tg;
    t.tg_sep = sep;
    t.ev_p = p;
    t.ev_method = method;
    if (is_fmm(method)) t.m2l_pairs = t.n_v;
    A.release_temps();
}

static size_t estimate_bytes(int64_t n_src, int64_t n_tgt, int leaf_max, int p, int method,
                             int precision) {
    // separate targets: sorted copies (88 bytes), sort and box temporaries,
    // and up to one box each with its lists (counted as cells below)
    const int64_t n = n_src + n_tgt;
    const int64_t nc = 4 * n / std::max(1, leaf_max) + 4096;
    const int P = p * p;
    int RB, KQ, ld;
    m2l_layout(p, precision, RB, KQ, ld);
    size_t per_particle = 8 + 4 + 24 + 16 + 32 + 4 + 8 + 4 + 8 + 4 * 8 + 64 + 32;
    // M, L, LX (FP64), the M2L operand and the FP32 copy of M for the
    // far field (FP32), room for twelve M2L partial results (the launch plans
    // fewer for large trees, more for small ones when the arena has room)
    size_t per_cell = 32 + 27 * 4 + 216 * 4 + 3 * 4 + 200 + 16 + 32 + (size_t)ld * 8 * 3 +
                      (size_t)ld * 4 * 2 + (size_t)12 * ld * 4 + 64;
    if (method == HFMM_TREECODE) per_cell = 32 + 32 + 32 + (size_t)P * 8 + 512 + 64;
    // FMM lists and upward data, the FP32 copy of M and the treecode lists:
    // up to 189 M2P items per level from a leaf to the root (levels taken
    // as those of a uniform tree plus two)
    if (method == HFMM_TREECODE_FMMLIST) {
        const double leaves = std::max(1.0, (double)n / std::max(1, leaf_max));
        const int levels = (int)std::ceil(std::log(leaves) / std::log(8.0)) + 2;
        per_cell = 32 + 27 * 4 + 216 * 4 + 3 * 4 + 200 + 16 + 32 + (size_t)ld * 8 +
                   (size_t)ld * 4 + 64 + (size_t)4 * 189 * std::max(levels, 3);
    }
    size_t ops = method == HFMM_FMM ? std::max(m2l_ops_bytes(p, precision), rot_ops_bytes(p, precision))
                 : method == HFMM_FMM_ROT ? rot_ops_bytes(p, precision) : 0;
    if (is_fmm(method)) ops += (size_t)2 * 8 * ld * ld * sizeof(double);
    if (method == HFMM_FMM && precision != HFMM_FP64 && !m2l_uses_mfma(p, precision))
        ops += (size_t)343 * P * P * 8;
    size_t tot = per_particle * (size_t)n + per_cell * (size_t)nc + ops;
    return tot + tot / 4 + ((size_t)64 << 20);
}

static thread_local size_t g_last_required = 0;
static bool g_timing = false;

void set_last_required(size_t bytes) { g_last_required = bytes; }

void stream_wait(hipStream_t s) {
    const auto t0 = std::chrono::steady_clock::now();
    for (;;) {
        const hipError_t e = hipStreamQuery(s);
        if (e == hipSuccess) return;
        if (e != hipErrorNotReady) throw HipError{e};
        if (std::chrono::steady_clock::now() - t0 > std::chrono::microseconds(500)) break;
    }
    HIP_TRY(hipStreamSynchronize(s));
}

}  // namespace hfmm

using namespace hfmm;

struct hfmm_tree_s {
    Tree t;
    ~hfmm_tree_s() {
        for (auto& e : t.ev)
            if (e) (void)hipEventDestroy(e);
    }
};

#define API_BEGIN try {
#define API_END                                   \
    }                                             \
    catch (const Status& st) {                    \
        return st.code;                           \
    }                                             \
    catch (const HipError&) {                     \
        return HFMM_E_HIP;                        \
    }                                             \
    catch (const std::bad_alloc&) {               \
        return HFMM_E_NOMEM;                      \
    }                                             \
    catch (...) {                                 \
        return HFMM_E_HIP;                        \
    }                                             \
    return HFMM_OK;

extern "C" {

int hfmm_arena_bytes(int64_t n_src, int64_t n_tgt, int leaf_max, int p, int method,
                     int precision, size_t* bytes) {
    if (!bytes || n_src < 0 || n_tgt < 0 || leaf_max < 1) return HFMM_E_INVAL;
    if (p < 1 || p > HFMM_MAX_P) return HFMM_E_UNSUPPORTED;
    if (precision < HFMM_FP64 || precision > HFMM_M2L_FP16X3) return HFMM_E_UNSUPPORTED;
    if (method == HFMM_DIRECT) return hfmm_direct_bytes(n_src, n_tgt, precision, bytes);
    if (!tree_method(method)) return HFMM_E_UNSUPPORTED;
    *bytes = estimate_bytes(n_src, n_tgt, leaf_max, p, method, precision);
    return HFMM_OK;
}

int hfmm_build_tree(const double* x, const double* y, const double* z, int64_t n_src,
                    int leaf_max, void* arena, size_t arena_bytes, void* stream,
                    hfmm_tree* out) {
    if (!out) return HFMM_E_INVAL;
    *out = nullptr;
    if (n_src < 0 || leaf_max < 1 || !arena) return HFMM_E_INVAL;
    if (n_src > 0 && (!x || !y || !z)) return HFMM_E_INVAL;
    if (n_src > (int64_t)INT32_MAX / 2) return HFMM_E_UNSUPPORTED;
    hfmm_tree_s* h = new (std::nothrow) hfmm_tree_s();
    if (!h) return HFMM_E_NOMEM;
    Tree& t = h->t;
    hipStream_t s = (hipStream_t)stream;
    try {
        HIP_TRY(hipGetDevice(&t.device));
        t.n = n_src;
        t.leaf_max = leaf_max;
        t.arena.init(arena, arena_bytes);
        if (g_timing) {
            for (auto& e : t.ev) HIP_TRY(hipEventCreate(&e));
            t.timing = true;
        }
        if (t.n > 0) {
            PhaseTimer pt(t, PH_BUILD, s);
            build_tree(t, x, y, z, s);
        } else {
            t.status = t.arena.up<int32_t>(1);
            HIP_TRY(hipMemsetAsync(t.status, 0, sizeof(int32_t), s));
        }
        t.mark_tree = t.arena.lo;
        t.mark_lists = t.mark_up = t.arena.lo;
    } catch (const Status& st) {
        g_last_required = t.arena.need;
        delete h;
        return st.code;
    } catch (...) {
        delete h;
        return HFMM_E_HIP;
    }
    *out = h;
    return HFMM_OK;
}

int hfmm_upward(hfmm_tree h, const double* m, int p, int method, int precision,
                void* stream) {
    if (!h) return HFMM_E_INVAL;
    if (h->t.stale) return HFMM_E_STATE;
    API_BEGIN
    check_p(p);
    check_precision(precision);
    if (!tree_method(method)) throw Status{HFMM_E_UNSUPPORTED};
    if (h->t.n == 0) {
        h->t.up_p = p;
        h->t.up_method = method;
        h->t.up_prec = precision;
        return HFMM_OK;
    }
    upward_pass(h->t, m, p, method, precision, (hipStream_t)stream);
    API_END
}

int hfmm_evaluate(hfmm_tree h, const double* tx, const double* ty, const double* tz,
                  int64_t n_tgt, int p, double theta, int method, int precision, double eps2,
                  void* phi, void* ax, void* ay, void* az, void* stream) {
    if (!h) return HFMM_E_INVAL;
    Tree& t = h->t;
    const bool sep = tx != nullptr;
    if (sep && (n_tgt < 0 || !ty || !tz)) return HFMM_E_INVAL;
    if (!sep && n_tgt != 0) return HFMM_E_INVAL;  // targets given without coordinates
    if (sep && n_tgt > (int64_t)INT32_MAX / 2) return HFMM_E_UNSUPPORTED;
    const int64_t nt = sep ? n_tgt : t.n;
    if (nt > 0 && (!phi || !ax || !ay || !az)) return HFMM_E_INVAL;
    if (!(eps2 >= 0.0) || !std::isfinite(eps2)) return HFMM_E_INVAL;
    if (t.up_p != p || t.up_method != method || t.up_prec != precision) return HFMM_E_STATE;
    if (method == HFMM_TREECODE && !(theta >= 0.0)) return HFMM_E_INVAL;
    API_BEGIN
    hipStream_t s = (hipStream_t)stream;
    if (nt == 0) return HFMM_OK;
    if (t.n == 0) {  // no sources: a zero field
        const size_t e = precision == HFMM_FP64 ? 8 : 4;
        for (void* o : {phi, ax, ay, az}) HIP_TRY(hipMemsetAsync(o, 0, e * nt, s));
        return HFMM_OK;
    }
    evaluate(t, tx, ty, tz, nt, p, theta, method, precision, eps2, phi, ax, ay, az, s);
    API_END
}

int hfmm_solve(const double* x, const double* y, const double* z, const double* m,
               int64_t n_src, const double* tx, const double* ty, const double* tz,
               int64_t n_tgt, int leaf_max, int p, double theta, int method, int precision,
               double eps2, void* arena, size_t arena_bytes, void* phi, void* ax, void* ay,
               void* az, void* stream) {
    if (method == HFMM_DIRECT)
        return hfmm_direct(x, y, z, m, n_src, tx, ty, tz, n_tgt, precision, eps2, arena,
                           arena_bytes, phi, ax, ay, az, stream);
    hfmm_tree h = nullptr;
    int rc = hfmm_build_tree(x, y, z, n_src, leaf_max, arena, arena_bytes, stream, &h);
    if (rc != HFMM_OK) return rc;
    rc = hfmm_upward(h, m, p, method, precision, stream);
    if (rc == HFMM_OK)
        rc = hfmm_evaluate(h, tx, ty, tz, n_tgt, p, theta, method, precision, eps2, phi, ax, ay,
                           az, stream);
    if (rc == HFMM_OK) rc = hfmm_status(h, stream, nullptr);
    if (rc == HFMM_E_NOMEM) g_last_required = h->t.arena.need;
    hfmm_tree_release(h);
    return rc;
}

int hfmm_refit(hfmm_tree h, const double* x, const double* y, const double* z, double slack,
               void* stream, int* kept) {
    if (kept) *kept = 0;
    if (!h || !kept) return HFMM_E_INVAL;
    Tree& t = h->t;
    if (t.n > 0 && (!x || !y || !z)) return HFMM_E_INVAL;
    if (!(slack >= 0.0) || !std::isfinite(slack)) return HFMM_E_INVAL;
    if (t.stale) return HFMM_E_STATE;
    API_BEGIN
    // the expansions, centres of mass and lists of the old positions go
    t.up_p = 0;
    t.up_method = t.up_prec = -1;
    t.tg_sep = false;
    t.tg = Targets{};
    if (t.n == 0) {
        *kept = 1;
        return HFMM_OK;
    }
    t.stale = true;
    const bool k = refit_tree(t, x, y, z, slack, (hipStream_t)stream);
    t.stale = !k;
    *kept = k ? 1 : 0;
    API_END
}

int hfmm_status(hfmm_tree h, void* stream, uint32_t* flags) {
    if (flags) *flags = 0;
    if (!h) return HFMM_E_INVAL;
    const Tree& t = h->t;
    int32_t w = 0;
    if (t.status) {
        hipStream_t s = (hipStream_t)stream;
        if (hipMemcpyAsync(&w, t.status, sizeof(w), hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess)
            return HFMM_E_HIP;
    }
    if (flags) *flags = (uint32_t)w;
    if (w & (ST_SRC_NONFINITE | ST_TGT_NONFINITE | ST_MASS_NONFINITE)) return HFMM_E_DATA;
    if (w & ST_OVERFLOW) return HFMM_E_OVERFLOW;
    return HFMM_OK;
}

int hfmm_direct_bytes(int64_t n_src, int64_t n_tgt, int precision, size_t* bytes) {
    if (!bytes || n_src < 0 || n_tgt < 0) return HFMM_E_INVAL;
    if (precision != HFMM_FP64 && precision != HFMM_FP32) return HFMM_E_UNSUPPORTED;
    size_t e = precision == HFMM_FP64 ? 32 : 16;
    *bytes = e * (size_t)(n_src + n_tgt) + 4 * HFMM_ALIGN;
    return HFMM_OK;
}

int hfmm_direct(const double* x, const double* y, const double* z, const double* m,
                int64_t n_src, const double* tx, const double* ty, const double* tz,
                int64_t n_tgt, int precision, double eps2, void* arena, size_t arena_bytes,
                void* phi, void* ax, void* ay, void* az, void* stream) {
    if (n_src < 0 || n_tgt < 0) return HFMM_E_INVAL;
    if (precision != HFMM_FP64 && precision != HFMM_FP32) return HFMM_E_UNSUPPORTED;
    const bool self = tx == nullptr;
    if (self && n_tgt != 0) return HFMM_E_INVAL;  // targets given without coordinates
    const int64_t nt = self ? n_src : n_tgt;
    if (n_src > 0 && (!x || !y || !z || !m)) return HFMM_E_INVAL;
    if (!self && (!ty || !tz)) return HFMM_E_INVAL;
    if (nt > 0 && (!phi || !ax || !ay || !az || !arena)) return HFMM_E_INVAL;
    if (!(eps2 >= 0.0) || !std::isfinite(eps2)) return HFMM_E_INVAL;
    Arena A;
    A.init(arena, arena_bytes);
    try {
        direct_sum(x, y, z, m, n_src, tx, ty, tz, nt, precision, eps2, A, phi, ax, ay, az,
                   (hipStream_t)stream);
    } catch (const Status& st) {
        g_last_required = A.need;
        return st.code;
    } catch (...) {
        return HFMM_E_HIP;
    }
    return HFMM_OK;
}

void hfmm_tree_release(hfmm_tree h) { delete h; }

size_t hfmm_required_bytes(hfmm_tree h) {
    if (!h) return 0;
    return h->t.arena.need ? h->t.arena.need : h->t.arena.peak;
}

size_t hfmm_last_required_bytes(void) { return g_last_required; }

int hfmm_get_stats(hfmm_tree h, hfmm_stats* st) {
    if (!h || !st) return HFMM_E_INVAL;
    const Tree& t = h->t;
    st->n_particles = t.n;
    st->n_targets = t.tg_sep ? t.tg.n : t.n;
    st->n_target_boxes = t.tg_sep ? t.tg.nbox : t.nleaves;
    st->target_near = t.tg_sep ? t.tg_near : 0;
    st->target_far = t.tg_sep ? t.tg_far : 0;
    st->n_cells = t.ncells;
    st->n_leaves = t.nleaves;
    st->depth = t.depth;
    st->sort_bits = t.sort_bits;
    for (int a = 0; a < 3; ++a) st->root[a] = t.root_h.b[a];
    st->root[3] = t.root_h.R;
    st->list_u = t.fmm_lists ? t.n_u : 0;
    st->list_v = t.fmm_lists ? t.n_v : 0;
    st->list_w = t.fmm_lists ? t.n_w : 0;
    st->list_x = t.fmm_lists ? t.n_x : 0;
    st->list_m2p = t.a_off ? t.n_a : 0;
    st->list_p2p = t.a_off ? t.n_b : 0;
    st->p2p_pairs = t.p2p_pairs;
    st->m2l_pairs = t.m2l_pairs;
    st->arena_used = t.arena.used();
    for (int k = 0; k < HFMM_PHASES; ++k) {
        st->phase_ms[k] = -1.0;
        if (t.timing && t.ev_used[k]) {
            float ms = 0.f;
            if (hipEventSynchronize(t.ev[2 * k + 1]) == hipSuccess &&
                hipEventElapsedTime(&ms, t.ev[2 * k], t.ev[2 * k + 1]) == hipSuccess)
                st->phase_ms[k] = ms;
        }
    }
    return HFMM_OK;
}

void hfmm_set_timing(int on) { g_timing = on != 0; }

const char* hfmm_strerror(int code) {
    switch (code) {
        case HFMM_OK: return "ok";
        case HFMM_E_INVAL: return "invalid argument";
        case HFMM_E_NOMEM: return "arena too small";
        case HFMM_E_UNSUPPORTED: return "unsupported order, method or precision";
        case HFMM_E_HIP: return "HIP runtime error";
        case HFMM_E_STATE: return "call order violated";
        case HFMM_E_DATA: return "non-finite coordinates or masses";
        case HFMM_E_OVERFLOW: return "traversal stack overflow (lists incomplete)";
        default: return "unknown error";
    }
}

int hfmm_export_perm(hfmm_tree h, int32_t* dst, void* stream) {
    if (!h || (!dst && h->t.n > 0)) return HFMM_E_INVAL;
    API_BEGIN
    if (h->t.n > 0)
        HIP_TRY(hipMemcpyAsync(dst, h->t.perm, sizeof(int32_t) * h->t.n,
                               hipMemcpyDeviceToDevice, (hipStream_t)stream));
    API_END
}

int hfmm_export_cells(hfmm_tree h, int32_t* dst, void* stream) {
    if (!h || (!dst && h->t.ncells > 0)) return HFMM_E_INVAL;
    API_BEGIN
    const Tree& t = h->t;
    if (t.ncells > 0) {
        hipLaunchKernelGGL(k_export_cells, dim3(grid_for(t.ncells, 256)), dim3(256), 0,
                           (hipStream_t)stream, t.cells, t.ncells, dst);
        LAUNCH_CHECK();
    }
    API_END
}

int hfmm_export_list(hfmm_tree h, int which, int32_t* off, int32_t* items, void* stream) {
    if (!h || !off || !items || which < 0 || which > 3) return HFMM_E_INVAL;
    Tree& t = h->t;
    if (!t.fmm_lists) return HFMM_E_STATE;
    API_BEGIN
    hipStream_t s = (hipStream_t)stream;
    const int nc = t.ncells;
    if (which == 1) {
        t.arena.release_temps();
        int32_t* cnt = t.arena.down<int32_t>(nc + 1);
        hipLaunchKernelGGL(k_v_count, dim3(grid_for(nc, 256)), dim3(256), 0, s, t.vsrc, nc, cnt);
        LAUNCH_CHECK();
        scan_exclusive_i32(cnt, off, nc, t.arena, s);
        hipLaunchKernelGGL(k_v_fill, dim3(grid_for(nc, 256)), dim3(256), 0, s, t.vsrc, nc, off,
                           items);
        LAUNCH_CHECK();
        HIP_TRY(hipStreamSynchronize(s));
        t.arena.release_temps();
    } else {
        // U, W and X share one item array with absolute offsets: export the
        // list's own slice with offsets starting at 0
        const int32_t* o = which == 0 ? t.u_off : which == 2 ? t.w_off : t.x_off;
        const int32_t* it = which == 0 ? t.u_items : which == 2 ? t.w_items : t.x_items;
        const int64_t nn = which == 0 ? t.n_u : which == 2 ? t.n_w : t.n_x;
        const int64_t base = which == 0 ? 0 : which == 2 ? t.n_u : t.n_u + t.n_w;
        hipLaunchKernelGGL(k_offsets_minus, dim3(grid_for(nc + 1, 256)), dim3(256), 0, s, o,
                           (int64_t)nc + 1, (int32_t)base, off);
        LAUNCH_CHECK();
        if (nn > 0)
            HIP_TRY(hipMemcpyAsync(items, it + base, sizeof(int32_t) * nn,
                                   hipMemcpyDeviceToDevice, s));
    }
    API_END
}

int hfmm_export_bh_list(hfmm_tree h, int which, int32_t* off, int32_t* items, void* stream) {
    if (!h || !off || which < 0 || which > 1) return HFMM_E_INVAL;
    Tree& t = h->t;
    if (!t.a_off) return HFMM_E_STATE;
    API_BEGIN
    hipStream_t s = (hipStream_t)stream;
    const int32_t* o = which == 0 ? t.a_off : t.b_off;
    const int32_t* it = which == 0 ? t.a_items : t.b_items;
    const int64_t nn = which == 0 ? t.n_a : t.n_b;
    HIP_TRY(hipMemcpyAsync(off, o, sizeof(int32_t) * (t.ncells + 1), hipMemcpyDeviceToDevice, s));
    if (nn > 0 && items) {
        if (it)
            HIP_TRY(hipMemcpyAsync(items, it, sizeof(int32_t) * nn, hipMemcpyDeviceToDevice, s));
        else  // over the FMM lists at p = 3 the M2P items are not kept
            fill_fmmlist_far_items(t, items, s);
    }
    API_END
}

int hfmm_export_targets(hfmm_tree h, int32_t* dst, void* stream) {
    if (!h) return HFMM_E_INVAL;
    const Tree& t = h->t;
    if (!t.tg.box) return HFMM_E_STATE;
    if (!dst && t.tg.n > 0) return HFMM_E_INVAL;
    API_BEGIN
    if (t.tg.n > 0) {
        hipLaunchKernelGGL(k_export_targets, dim3(grid_for(t.tg.n, 256)), dim3(256), 0,
                           (hipStream_t)stream, t.tg, dst);
        LAUNCH_CHECK();
    }
    API_END
}

int hfmm_export_target_lists(hfmm_tree h, int which, int32_t* off, int32_t* items,
                             void* stream) {
    if (!h || !off || which < 0 || which > 1) return HFMM_E_INVAL;
    const Tree& t = h->t;
    if (!t.tg_sep) return HFMM_E_STATE;
    API_BEGIN
    hipStream_t s = (hipStream_t)stream;
    const int32_t* o = which == 0 ? t.tf_off : t.tn_off;
    const int32_t* it = which == 0 ? t.tf_items : t.tn_items;
    const int64_t nn = which == 0 ? t.tg_far : t.tg_near;
    HIP_TRY(hipMemcpyAsync(off, o, sizeof(int32_t) * (t.tg.nbox + 1), hipMemcpyDeviceToDevice,
                           s));
    if (nn > 0 && items)
        HIP_TRY(hipMemcpyAsync(items, it, sizeof(int32_t) * nn, hipMemcpyDeviceToDevice, s));
    API_END
}

int hfmm_export_expansions(hfmm_tree h, int which, double* dst, void* stream) {
    if (!h || !dst || which < 0 || which > 1) return HFMM_E_INVAL;
    Tree& t = h->t;
    if (t.up_p == 0 || !t.M) return HFMM_E_STATE;
    if (which == 1 && (!is_fmm(t.up_method) || !t.L || t.ev_p != t.up_p)) return HFMM_E_STATE;
    API_BEGIN
    run_export(which == 0 ? t.M : t.L, t.ldm, t.ncells, t.up_p, t.cen, which, dst,
               (hipStream_t)stream);
    API_END
}

}  // extern "C"
