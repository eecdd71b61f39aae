// C ABI of the hfmm library: argument checks, arena layout and the order of
// the passes (Sec. 2, Fig. 1):
//   build:    bbox, keys, sort, cells                       (tree.hip)
//   upward:   P2M at the leaves, M2M to the root            (expansions.hip)
//   evaluate: FMM      M2L (+P2L), L2L, L2P (+M2P), P2P     (m2l, expansions, p2p)
//             treecode M2P, P2P (Barnes-Hut lists, or the FMM lists)
#include "common.hpp"
#include "expansions.hpp"

#include <algorithm>
#include <cmath>
#include <new>

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

static void check_p(int p) {
    if (p < 1 || p > HFMM_MAX_P) throw Status{HFMM_E_UNSUPPORTED};
}
// the methods whose upward pass is the FMM's (geometric centres, FMM lists)
static bool fmm_upward(int method) {
    return method == HFMM_FMM || method == HFMM_TREECODE_FMMLIST;
}
static bool tree_method(int method) {
    return method == HFMM_FMM || method == HFMM_TREECODE || method == HFMM_TREECODE_FMMLIST;
}

static void check_precision(int precision) {
    if (precision < HFMM_FP64 || precision > HFMM_M2L_FP16X3) throw Status{HFMM_E_UNSUPPORTED};
}

void upward_pass(Tree& t, const double* m, int p, int method, int precision, hipStream_t s) {
    check_p(p);
    check_precision(precision);
    if (!tree_method(method)) throw Status{HFMM_E_UNSUPPORTED};
    if (!m && t.ns > 0) throw Status{HFMM_E_INVAL};
    Arena& A = t.arena;
    A.release_temps();
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

void evaluate_fmm(Tree& t, int p, int precision, double eps2, void* phi, void* ax, void* ay,
                  void* az, hipStream_t s) {
    Arena& A = t.arena;
    A.release_temps();
    A.lo = t.mark_up;
    const int P = p * p;
    const bool fp64 = precision == HFMM_FP64;
    {
        PhaseTimer pt(t, PH_OPS, s);
        prepare_m2l_ops(t, p, precision, s);
    }
    int RB, KQ, ld;
    m2l_layout(p, precision, RB, KQ, ld);
    t.L = A.up<double>((size_t)(t.ncells + 1) * t.ldm);
    const size_t row = sizeof(double) * t.ldm;
    HIP_TRY(hipMemsetAsync(t.L + (size_t)t.ncells * t.ldm, 0, row, s));
    if (t.depth >= 2) {
        // M2L partial results
        const bool mf = m2l_uses_mfma(p, precision);
        int max_parts = 12;
        const size_t esz = fp64 ? 8 : 4;
        while (max_parts > 1 &&
               (size_t)max_parts * t.ncells * t.ldm * esz > A.free_bytes() / 2)
            --max_parts;
        const int parts_cap = mf ? max_parts : 1;
        void* lm = A.down<char>((size_t)parts_cap * t.ncells * t.ldm * esz);
        int32_t* levexp = A.down<int32_t>(32);
        double* LX = nullptr;
        if (t.n_x > 0) LX = A.down<double>((size_t)t.ncells * t.ldm);
        int64_t stride = 0;
        int parts;
        parts = run_m2l(t, p, precision, lm, stride, parts_cap, levexp, s);
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
    void* far = A.down<char>((size_t)4 * t.n * (fp64 ? 8 : 4));
    {
        PhaseTimer pt(t, PH_FAR, s);
        run_far(t, p, fp64, far, s);
    }
    {
        PhaseTimer pt(t, PH_P2P, s);
        launch_p2p(t, precision, eps2, t.leaves, t.nleaves, t.u_off, t.u_items, far, phi, ax,
                   ay, az, s);
    }
    t.ev_p = p;
    t.m2l_pairs = t.n_v;
    A.release_temps();
}

// fmm_lists: the treecode of Sec. 4 (M2P and P2P over the FMM lists, theta
// unused); otherwise Barnes-Hut lists with acceptance theta
void evaluate_treecode(Tree& t, int p, double theta, bool fmm_lists, int precision, double eps2,
                       void* phi, void* ax, void* ay, void* az, hipStream_t s) {
    Arena& A = t.arena;
    A.release_temps();
    {
        PhaseTimer pt(t, PH_BH, s);
        if (fmm_lists)
            build_fmmlist_treecode_lists(t, p != 3, s);
        else
            build_bh_lists(t, theta, s);
    }
    const bool fp64 = precision == HFMM_FP64;
    void* far = A.down<char>((size_t)4 * t.n * (fp64 ? 8 : 4));
    {
        PhaseTimer pt(t, PH_FAR, s);
        run_treecode_far(t, p, fp64, far, s);
    }
    {
        PhaseTimer pt(t, PH_P2P, s);
        launch_p2p(t, precision, eps2, t.leaves, t.nleaves, t.b_off, t.b_items, far, phi, ax,
                   ay, az, s);
    }
    t.ev_p = p;
    A.release_temps();
}

static size_t estimate_bytes(int64_t n_src, int64_t n_tgt, int leaf_max, int p, int method,
                             int precision) {
    const int64_t n = n_src + n_tgt;
    const int64_t nc = 4 * n / std::max(1, leaf_max) + 4096;
    const int P = p * p;
    int RB, KQ, ld;
    m2l_layout(p, precision, RB, KQ, ld);
    size_t per_particle = 8 + 4 + 24 + 16 + 32 + 4 + 8 + 4 + 8 + 4 * 8 + 64;
    // M, L, LX (FP64), the M2L operand and the FP32 copy of M for the
    // far field (FP32), up to twelve M2L partial results
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
    size_t ops = method == HFMM_FMM ? m2l_ops_bytes(p, precision) : 0;
    if (method == HFMM_FMM) ops += (size_t)2 * 8 * ld * ld * sizeof(double);
    if (method == HFMM_FMM && precision != HFMM_FP64 && !m2l_uses_mfma(p, precision))
        ops += (size_t)343 * P * P * 8;
    size_t tot = per_particle * (size_t)n + per_cell * (size_t)nc + ops;
    return tot + tot / 4 + ((size_t)64 << 20);
}

static thread_local size_t g_last_required = 0;
static bool g_timing = false;

void set_last_required(size_t bytes) { g_last_required = bytes; }

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
                    const double* tx, const double* ty, const double* tz, int64_t n_tgt,
                    int leaf_max, void* arena, size_t arena_bytes, void* stream,
                    hfmm_tree* out) {
    if (!out) return HFMM_E_INVAL;
    *out = nullptr;
    if (n_src < 0 || n_tgt < 0 || leaf_max < 1 || !arena) return HFMM_E_INVAL;
    if (n_src > 0 && (!x || !y || !z)) return HFMM_E_INVAL;
    const bool self = tx == nullptr;
    if (!self && n_tgt > 0 && (!ty || !tz)) return HFMM_E_INVAL;
    if (n_src + (self ? 0 : n_tgt) > (int64_t)INT32_MAX / 2) return HFMM_E_UNSUPPORTED;
    hfmm_tree_s* h = new (std::nothrow) hfmm_tree_s();
    if (!h) return HFMM_E_NOMEM;
    Tree& t = h->t;
    hipStream_t s = (hipStream_t)stream;
    try {
        HIP_TRY(hipGetDevice(&t.device));
        t.ns = n_src;
        t.nt = self ? n_src : n_tgt;
        t.self = self;
        t.n = n_src + (self ? 0 : n_tgt);
        t.leaf_max = leaf_max;
        t.arena.init(arena, arena_bytes);
        if (g_timing) {
            for (auto& e : t.ev) HIP_TRY(hipEventCreate(&e));
            t.timing = true;
        }
        if (t.n > 0) {
            PhaseTimer pt(t, PH_BUILD, s);
            build_tree(t, x, y, z, tx, ty, tz, s);
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
    API_BEGIN
    if (h->t.n == 0) {
        h->t.up_p = p;
        h->t.up_method = method;
        h->t.up_prec = precision;
        return HFMM_OK;
    }
    upward_pass(h->t, m, p, method, precision, (hipStream_t)stream);
    API_END
}

int hfmm_evaluate(hfmm_tree h, int p, double theta, int method, int precision, double eps2,
                  void* phi, void* ax, void* ay, void* az, void* stream) {
    if (!h) return HFMM_E_INVAL;
    Tree& t = h->t;
    if (t.nt > 0 && (!phi || !ax || !ay || !az)) return HFMM_E_INVAL;
    if (!(eps2 >= 0.0) || !std::isfinite(eps2)) return HFMM_E_INVAL;
    if (t.up_p != p || t.up_method != method || t.up_prec != precision) return HFMM_E_STATE;
    if (method == HFMM_TREECODE && !(theta >= 0.0)) return HFMM_E_INVAL;
    API_BEGIN
    if (t.n == 0 || t.nt == 0) return HFMM_OK;
    hipStream_t s = (hipStream_t)stream;
    if (method == HFMM_FMM)
        evaluate_fmm(t, p, precision, eps2, phi, ax, ay, az, s);
    else
        evaluate_treecode(t, p, theta, method == HFMM_TREECODE_FMMLIST, precision, eps2, phi,
                          ax, ay, az, s);
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
    int rc = hfmm_build_tree(x, y, z, n_src, tx, ty, tz, n_tgt, leaf_max, arena, arena_bytes,
                             stream, &h);
    if (rc != HFMM_OK) return rc;
    rc = hfmm_upward(h, m, p, method, precision, stream);
    if (rc == HFMM_OK) rc = hfmm_evaluate(h, p, theta, method, precision, eps2, phi, ax, ay, az,
                                          stream);
    if (rc == HFMM_E_NOMEM) g_last_required = h->t.arena.need;
    hfmm_tree_release(h);
    return rc;
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
    return h->t.arena.need ? h->t.arena.need : h->t.arena.used();
}

size_t hfmm_last_required_bytes(void) { return g_last_required; }

int hfmm_get_stats(hfmm_tree h, hfmm_stats* st) {
    if (!h || !st) return HFMM_E_INVAL;
    const Tree& t = h->t;
    st->n_particles = t.n;
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
        case HFMM_E_DATA: return "non-finite coordinates";
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

int hfmm_export_expansions(hfmm_tree h, int which, double* dst, void* stream) {
    if (!h || !dst || which < 0 || which > 1) return HFMM_E_INVAL;
    Tree& t = h->t;
    if (t.up_p == 0 || !t.M) return HFMM_E_STATE;
    if (which == 1 && (t.up_method != HFMM_FMM || !t.L || t.ev_p != t.up_p)) return HFMM_E_STATE;
    API_BEGIN
    run_export(which == 0 ? t.M : t.L, t.ldm, t.ncells, t.up_p, t.cen, which, dst,
               (hipStream_t)stream);
    API_END
}

}  // extern "C"
