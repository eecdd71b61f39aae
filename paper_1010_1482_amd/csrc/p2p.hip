// Near field (P2P, Sec. 5.1) and the direct sum.
//
// Per pair: a_i += m_j (x_j - x_i) / r^3 and phi_i += m_j / r with one
// reciprocal square root (Listing 1 of Sec. 5.1 plus the potential), pairs
// at r^2 == 0 skipped.  The paper gives each target cell a thread block and
// pads the targets to the block size (Secs. 3 and 5.1); leaves here hold up
// to ~32 particles (clustered data: ~10 on average), so one 64-lane wave
// takes one target leaf and, when the leaf has at most 32 (16, 8) targets,
// splits the sources over 2 (4, 8) lane groups that are summed with
// cross-lane shuffles at the end.  The sources of consecutive list cells are
// packed into chunks of 64 (x, y, z, m) records in LDS, so a chunk is full
// however few particles each cell holds; the target leaf itself, whose
// coincident points need the r^2 == 0 test, is taken on its own.  Each wave
// owns its LDS slice, so there is no block-wide barrier.
#include "common.hpp"
#include "expansions.hpp"

namespace hfmm {


// ZERO: the pair may coincide (r^2 == 0, skipped).  Coincident points share
// a key, hence a leaf, so only a leaf with itself needs the test.  Across
// leaves FP64 separations are never 0; FP32 ones can round to 0 for points
// closer than FP32 resolves at the leaf size, and r^2 starts from 1e-24
// there so that the (then meaningless) pair stays finite: r^2 (+ eps^2) is
// one chain of fused multiply-adds from that start, which leaves r^2 above
// 2e-17 unchanged and needs no separate clamp instruction in the loop.
template <typename T, bool SOFT, bool ZERO>
__device__ __forceinline__ void pair(T xi, T yi, T zi, const typename Vec4<T>::type& s,
                                     T eps2, T& phi, T& ax, T& ay, T& az) {
    const T dx = s.x - xi, dy = s.y - yi, dz = s.z - zi;
    T rinv;
    if (ZERO) {  // the test is on the unsoftened r^2
        const T r2 = fma(dx, dx, fma(dy, dy, dz * dz));
        rinv = rsqrt_fast(SOFT ? r2 + eps2 : r2);
        rinv = r2 > T(0) ? rinv : T(0);
    } else {
        const T r0 = SOFT ? eps2 : (sizeof(T) == 4 ? T(1e-24) : T(0));
        rinv = rsqrt_fast(fma(dx, dx, fma(dy, dy, fma(dz, dz, r0))));
    }
    const T mr = s.w * rinv;
    phi += mr;
    const T sc = mr * rinv * rinv;
    ax += dx * sc;
    ay += dy * sc;
    az += dz * sc;
}

// Sum over the sources staged in sh[0, nl): lane layout TW = 64 / G
// targets, lane = g * TW + t, group g takes sources g, g + G, ...  Entries
// past nl up to the next multiple of G are padding (mass 0, far away).
template <typename T, int G, bool SOFT, bool ZERO>
__device__ __forceinline__ void p2p_staged(const typename Vec4<T>::type* sh, int nl, int g,
                                           T xi, T yi, T zi, T eps2, T& phi, T& ax, T& ay,
                                           T& az) {
    const int steps = (nl + G - 1) / G;
#pragma unroll 8
    for (int q = 0; q < steps; ++q) {
        const typename Vec4<T>::type s = sh[q * G + g];
        pair<T, SOFT, ZERO>(xi, yi, zi, s, eps2, phi, ax, ay, az);
    }
}

// Padding record: zero mass far from every target (its terms are exactly 0).
template <typename T>
__device__ __forceinline__ typename Vec4<T>::type p2p_pad() {
    return typename Vec4<T>::type{T(1e18), T(1e18), T(1e18), T(0)};
}

// The target box's own leaf as a source (coincident points possible): the
// sources of cell c against targets me.  In FP32 both are relative to the
// same centre (the box is the leaf), so no offset is added.
template <typename T, int G, bool SOFT>
__device__ __forceinline__ void p2p_self(const Cell& c, const typename Vec4<T>::type* __restrict__ P,
                                         typename Vec4<T>::type* sh, T xi, T yi, T zi, T eps2,
                                         T& phi, T& ax, T& ay, T& az) {
    constexpr int TW = 64 / G;
    const int lane = threadIdx.x & 63, g = lane / TW;
    const int end = c.first + c.count;
    for (int base = c.first; base < end; base += 64) {
        const int k = base + lane;
        const typename Vec4<T>::type v = k < end ? P[k] : p2p_pad<T>();
        wave_lds_fence();
        sh[lane] = v;
        wave_lds_fence();
        p2p_staged<T, G, SOFT, true>(sh, min(64, end - base), g, xi, yi, zi, eps2, phi, ax, ay,
                                     az);
    }
}

// Sum over the list cells items[e0, e1) other than the target leaf `self`.
// Per batch of 64 cells, lane j holds cell j's range and (FP32) the offset
// between its centre and the target leaf's centre, formed in FP64; a scan
// over the counts places the batch's particles in one sequence, which is
// staged 64 at a time.
template <typename T, int G, bool SOFT>
__device__ __forceinline__ void p2p_packed(const Cell* __restrict__ cells, int self,
                                           const int32_t* __restrict__ items, int e0, int e1,
                                           const typename Vec4<T>::type* __restrict__ P,
                                           typename Vec4<T>::type* sh, int* own,
                                           const Root& root, const double cb[3], T xi, T yi,
                                           T zi, T eps2, T& phi, T& ax, T& ay, T& az) {
    using V = typename Vec4<T>::type;
    constexpr int TW = 64 / G;
    constexpr bool REL = sizeof(T) == 4;
    const int lane = threadIdx.x & 63, g = lane / TW;
    for (int eb = e0; eb < e1; eb += 64) {
        int first = 0, cnt = 0;
        T ox = T(0), oy = T(0), oz = T(0);
        if (eb + lane < e1) {
            const int ci = items[eb + lane];
            if (ci != self) {
                const Cell c = cells[ci];
                first = c.first;
                cnt = c.count;
                if (REL) {
                    double cc[3];
                    cell_centre(root, c, cc);
                    ox = (T)(cc[0] - cb[0]);
                    oy = (T)(cc[1] - cb[1]);
                    oz = (T)(cc[2] - cb[2]);
                }
            }
        }
        int tot;
        const int off = wave_excl_scan(cnt, lane, tot);
        // lane's source of the run [pb, pb + 64) of the batch's particles;
        // the next run's load is issued before the current run's pairs
        auto fetch = [&](int pb, V& v, T& sx, T& sy, T& sz) {
            int o = wave_run_owner(own, off, cnt, pb, 64, lane);
            const bool ok = pb + lane < tot;
            o = ok ? o : 0;
            const int f = __shfl(first, o, 64), fo = __shfl(off, o, 64);
            v = p2p_pad<T>();
            if (REL) {
                sx = __shfl(ox, o, 64);
                sy = __shfl(oy, o, 64);
                sz = __shfl(oz, o, 64);
            }
            if (ok) v = P[f + (pb + lane - fo)];
            if (!ok) sx = sy = sz = T(0);
        };
        V v;
        T sx = T(0), sy = T(0), sz = T(0);
        if (tot > 0) fetch(0, v, sx, sy, sz);
        for (int pb = 0; pb < tot; pb += 64) {
            V cur = v;
            if (REL) {
                cur.x += sx;
                cur.y += sy;
                cur.z += sz;
            }
            if (pb + 64 < tot) fetch(pb + 64, v, sx, sy, sz);
            wave_lds_fence();
            sh[lane] = cur;
            wave_lds_fence();
            p2p_staged<T, G, SOFT, false>(sh, min(64, tot - pb), g, xi, yi, zi, eps2, phi, ax,
                                          ay, az);
        }
    }
}

// The targets of one box against the list cells items[e0, e1) (the box's
// own leaf, when it is in the list, summed on its own with the r^2 == 0
// test).  TP: the sorted targets, P: the sorted sources.
template <typename T, typename O, int G, bool SOFT>
__device__ __forceinline__ void p2p_box(const TBox& bx, bool in_list, const Root& root,
                                        const Cell* __restrict__ cells,
                                        const int32_t* __restrict__ items, int e0, int e1,
                                        const typename Vec4<T>::type* __restrict__ P,
                                        const typename Vec4<T>::type* __restrict__ TP,
                                        typename Vec4<T>::type* sh, int* own,
                                        const T* __restrict__ far, int64_t n,
                                        const int32_t* __restrict__ perm, T eps2,
                                        O* __restrict__ phi_o, O* __restrict__ ax_o,
                                        O* __restrict__ ay_o, O* __restrict__ az_o) {
    using V = typename Vec4<T>::type;
    constexpr int TW = 64 / G;
    const int lane = threadIdx.x & 63;
    const int t = lane % TW;
    double cb[3];
    cell_centre(root, box_cell(bx), cb);
    Cell own_leaf;
    if (in_list) own_leaf = cells[bx.leaf];
    for (int c0 = 0; c0 < bx.count; c0 += TW) {
        const int s = bx.first + c0 + t;
        const bool ok = c0 + t < bx.count;
        V me = ok ? TP[s] : V{T(0), T(0), T(0), T(0)};
        T phi = T(0), ax = T(0), ay = T(0), az = T(0);
        if (in_list)
            p2p_self<T, G, SOFT>(own_leaf, P, sh, me.x, me.y, me.z, eps2, phi, ax, ay, az);
        p2p_packed<T, G, SOFT>(cells, bx.leaf, items, e0, e1, P, sh, own, root, cb, me.x, me.y,
                               me.z, eps2, phi, ax, ay, az);
#pragma unroll
        for (int d = TW; d < 64; d <<= 1) {
            phi += __shfl_xor(phi, d, 64);
            ax += __shfl_xor(ax, d, 64);
            ay += __shfl_xor(ay, d, 64);
            az += __shfl_xor(az, d, 64);
        }
        if (ok && lane < TW) {
            const int64_t oi = perm[s];
            if (far) {
                phi += far[s];
                ax += far[n + s];
                ay += far[2 * n + s];
                az += far[3 * n + s];
            }
            phi_o[oi] = (O)phi;
            ax_o[oi] = (O)ax;
            ay_o[oi] = (O)ay;
            az_o[oi] = (O)az;
        }
    }
}

// One wave per target box; sources from the box's CSR list row.
template <typename T, typename O, bool SOFT>
__global__ void __launch_bounds__(256, 8)
k_p2p(const Cell* __restrict__ cells, const Root* __restrict__ rootp, Targets tg,
      const int32_t* __restrict__ off, const int32_t* __restrict__ items,
      const typename Vec4<T>::type* __restrict__ P, const T* __restrict__ far, T eps2,
      O* __restrict__ phi_o, O* __restrict__ ax_o, O* __restrict__ ay_o, O* __restrict__ az_o) {
    using V = typename Vec4<T>::type;
    __shared__ V shm[4][64];
    __shared__ int owm[4][64];
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int li = blockIdx.x * 4 + w;
    if (li >= tg.nbox) return;
    const TBox bx = tg.box[li];
    const int row = list_row(tg, li, bx);
    const Root root = *rootp;
    const int e0 = off[row], e1 = off[row + 1];
    const V* TP = sizeof(T) == 4 ? (const V*)tg.p32 : (const V*)tg.p64;
    V* sh = shm[w];
    int* own = owm[w];
    // is the box's own leaf in its list (then it is summed on its own)
    bool mine = false;
    if (bx.leaf >= 0)
        for (int e = e0 + lane; e < e1; e += 64) mine |= items[e] == bx.leaf;
    const bool in_list = __ballot(mine) != 0ull;
#define P2P_BOX(G)                                                                              \
    p2p_box<T, O, G, SOFT>(bx, in_list, root, cells, items, e0, e1, P, TP, sh, own, far, tg.n, \
                           tg.perm, eps2, phi_o, ax_o, ay_o, az_o)
    if (bx.count <= 8)
        P2P_BOX(8);
    else if (bx.count <= 16)
        P2P_BOX(4);
    else if (bx.count <= 32)
        P2P_BOX(2);
    else
        P2P_BOX(1);
#undef P2P_BOX
}

void launch_p2p(const Tree& t, const Targets& tg, int precision, double eps2,
                const int32_t* src_off, const int32_t* src_items, const void* far, void* phi,
                void* ax, void* ay, void* az, hipStream_t s) {
    if (tg.nbox == 0) return;
    dim3 grid((tg.nbox + 3) / 4), block(256);
    const bool soft = eps2 != 0.0;
#define P2P_LAUNCH(T, SOFT, P)                                                                \
    hipLaunchKernelGGL((k_p2p<T, T, SOFT>), grid, block, 0, s, t.cells, t.root, tg, src_off, \
                       src_items, P, (const T*)far, (T)eps2, (T*)phi, (T*)ax, (T*)ay, (T*)az)
    if (precision == HFMM_FP64) {
        if (soft)
            P2P_LAUNCH(double, true, t.p64);
        else
            P2P_LAUNCH(double, false, t.p64);
    } else {
        if (soft)
            P2P_LAUNCH(float, true, t.p32);
        else
            P2P_LAUNCH(float, false, t.p32);
    }
#undef P2P_LAUNCH
    LAUNCH_CHECK();
}

// ---------------------------------------------------------------------
// direct sum: targets in chunks of 64 per wave, all sources streamed
// ---------------------------------------------------------------------
template <typename T>
__global__ void k_pack_points(const double* __restrict__ x, const double* __restrict__ y,
                              const double* __restrict__ z, const double* __restrict__ m,
                              int64_t n, typename Vec4<T>::type* __restrict__ out) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    out[i] = typename Vec4<T>::type{(T)x[i], (T)y[i], (T)z[i], m ? (T)m[i] : T(0)};
}

template <typename T, bool SOFT>
__global__ void __launch_bounds__(256)
k_direct(const typename Vec4<T>::type* __restrict__ src, int64_t ns,
         const typename Vec4<T>::type* __restrict__ tgt, int64_t nt, T eps2,
         T* __restrict__ phi_o, T* __restrict__ ax_o, T* __restrict__ ay_o,
         T* __restrict__ az_o) {
    using V = typename Vec4<T>::type;
    __shared__ V shm[4][64];
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int64_t i = ((int64_t)blockIdx.x * 4 + w) * 64 + lane;
    if (((int64_t)blockIdx.x * 4 + w) * 64 >= nt) return;
    V me = i < nt ? tgt[i] : V{T(0), T(0), T(0), T(0)};
    V* sh = shm[w];
    T phi = T(0), ax = T(0), ay = T(0), az = T(0);
    for (int64_t base = 0; base < ns; base += 64) {
        const int64_t k = base + lane;
        V v = k < ns ? src[k] : V{T(0), T(0), T(0), T(0)};
        wave_lds_fence();
        sh[lane] = v;
        wave_lds_fence();
        const int nl = (int)min((int64_t)64, ns - base);
#pragma unroll 8
        for (int q = 0; q < nl; ++q)
            pair<T, SOFT, true>(me.x, me.y, me.z, sh[q], eps2, phi, ax, ay, az);
    }
    if (i < nt) {
        phi_o[i] = phi;
        ax_o[i] = ax;
        ay_o[i] = ay;
        az_o[i] = az;
    }
}

template <typename T>
static void direct_t(const double* x, const double* y, const double* z, const double* m,
                     int64_t ns, const double* tx, const double* ty, const double* tz,
                     int64_t nt, double eps2, Arena& A, void* phi, void* ax, void* ay,
                     void* az, hipStream_t s) {
    using V = typename Vec4<T>::type;
    V* src = A.down<V>(ns);
    V* tgt = tx ? A.down<V>(nt) : src;
    hipLaunchKernelGGL((k_pack_points<T>), dim3(grid_for(ns, 256)), dim3(256), 0, s, x, y, z,
                       m, ns, src);
    LAUNCH_CHECK();
    if (tx) {
        hipLaunchKernelGGL((k_pack_points<T>), dim3(grid_for(nt, 256)), dim3(256), 0, s, tx, ty,
                           tz, (const double*)nullptr, nt, tgt);
        LAUNCH_CHECK();
    }
    dim3 grid((unsigned)((nt + 255) / 256)), block(256);
    if (eps2 != 0.0)
        hipLaunchKernelGGL((k_direct<T, true>), grid, block, 0, s, src, ns, tgt, nt, (T)eps2,
                           (T*)phi, (T*)ax, (T*)ay, (T*)az);
    else
        hipLaunchKernelGGL((k_direct<T, false>), grid, block, 0, s, src, ns, tgt, nt, (T)eps2,
                           (T*)phi, (T*)ax, (T*)ay, (T*)az);
    LAUNCH_CHECK();
}

void direct_sum(const double* x, const double* y, const double* z, const double* m, int64_t ns,
                const double* tx, const double* ty, const double* tz, int64_t nt,
                int precision, double eps2, Arena& A, void* phi, void* ax, void* ay, void* az,
                hipStream_t s) {
    if (nt == 0) return;
    if (precision == HFMM_FP64)
        direct_t<double>(x, y, z, m, ns, tx, ty, tz, nt, eps2, A, phi, ax, ay, az, s);
    else
        direct_t<float>(x, y, z, m, ns, tx, ty, tz, nt, eps2, A, phi, ax, ay, az, s);
}

}  // namespace hfmm
