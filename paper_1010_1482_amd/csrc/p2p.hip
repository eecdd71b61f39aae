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
// closer than FP32 resolves at the leaf size, and r^2 is clamped there so
// that the (then meaningless) pair stays finite.
template <typename T, bool SOFT, bool ZERO>
__device__ __forceinline__ void pair(T xi, T yi, T zi, const typename Vec4<T>::type& s,
                                     T eps2, T& phi, T& ax, T& ay, T& az) {
    const T dx = s.x - xi, dy = s.y - yi, dz = s.z - zi;
    T r2 = dx * dx + dy * dy + dz * dz;
    if (!ZERO && sizeof(T) == 4) r2 = fmaxf(r2, 1e-24f);
    T rinv = rsqrt_fast(SOFT ? r2 + eps2 : r2);
    if (ZERO) rinv = r2 > T(0) ? rinv : T(0);
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

// The target leaf as its own source (coincident points possible).  In FP32
// positions are relative to the leaf centre, so no offset is added.
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
        for (int pb = 0; pb < tot; pb += 64) {
            int o = wave_run_owner(own, off, cnt, pb, 64, lane);
            const bool ok = pb + lane < tot;
            o = ok ? o : 0;
            const int f = __shfl(first, o, 64), fo = __shfl(off, o, 64);
            V v = p2p_pad<T>();
            if (REL) {
                const T sx = __shfl(ox, o, 64), sy = __shfl(oy, o, 64), sz = __shfl(oz, o, 64);
                if (ok) {
                    v = P[f + (pb + lane - fo)];
                    v.x += sx;
                    v.y += sy;
                    v.z += sz;
                }
            } else if (ok) {
                v = P[f + (pb + lane - fo)];
            }
            wave_lds_fence();
            sh[lane] = v;
            wave_lds_fence();
            p2p_staged<T, G, SOFT, false>(sh, min(64, tot - pb), g, xi, yi, zi, eps2, phi, ax,
                                          ay, az);
        }
    }
}

template <typename T, typename O, int G, bool SOFT>
__device__ __forceinline__ void p2p_leaf(const Cell& leaf, int self, bool in_list,
                                         const Root& root,
                                         const Cell* __restrict__ cells,
                                         const int32_t* __restrict__ items, int e0, int e1,
                                         const typename Vec4<T>::type* __restrict__ P,
                                         typename Vec4<T>::type* sh, int* own,
                                         const T* __restrict__ far,
                                         int64_t n, const int32_t* __restrict__ perm,
                                         int64_t out_shift, T eps2, O* __restrict__ phi_o,
                                         O* __restrict__ ax_o, O* __restrict__ ay_o,
                                         O* __restrict__ az_o) {
    using V = typename Vec4<T>::type;
    constexpr int TW = 64 / G;
    const int lane = threadIdx.x & 63;
    const int t = lane % TW;
    double cb[3];
    cell_centre(root, leaf, cb);
    for (int c0 = 0; c0 < leaf.count; c0 += TW) {
        const int s = leaf.first + c0 + t;
        const bool ok = c0 + t < leaf.count;
        V me = ok ? P[s] : V{T(0), T(0), T(0), T(0)};
        T phi = T(0), ax = T(0), ay = T(0), az = T(0);
        if (in_list)
            p2p_self<T, G, SOFT>(leaf, P, sh, me.x, me.y, me.z, eps2, phi, ax, ay, az);
        p2p_packed<T, G, SOFT>(cells, self, items, e0, e1, P, sh, own, root, cb, me.x, me.y, me.z,
                               eps2, phi, ax, ay, az);
#pragma unroll
        for (int d = TW; d < 64; d <<= 1) {
            phi += __shfl_xor(phi, d, 64);
            ax += __shfl_xor(ax, d, 64);
            ay += __shfl_xor(ay, d, 64);
            az += __shfl_xor(az, d, 64);
        }
        if (ok && lane < TW) {
            const int64_t oi = (int64_t)perm[s] - out_shift;
            if (oi >= 0) {
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
}

// One wave per target leaf; sources from the CSR list (off/items indexed by
// cell id).  out index = perm[s] - out_shift, skipped when negative.
template <typename T, typename O, bool SOFT>
__global__ void __launch_bounds__(256)
k_p2p(const Cell* __restrict__ cells, const Root* __restrict__ rootp,
      const int32_t* __restrict__ tgt, int ntgt,
      const int32_t* __restrict__ off, const int32_t* __restrict__ items,
      const typename Vec4<T>::type* __restrict__ P, const T* __restrict__ far, int64_t n,
      const int32_t* __restrict__ perm, int64_t out_shift, T eps2, O* __restrict__ phi_o,
      O* __restrict__ ax_o, O* __restrict__ ay_o, O* __restrict__ az_o) {
    using V = typename Vec4<T>::type;
    __shared__ V shm[4][64];
    __shared__ int owm[4][64];
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int li = blockIdx.x * 4 + w;
    if (li >= ntgt) return;
    const int b = tgt[li];
    const Cell leaf = cells[b];
    const Root root = *rootp;
    const int e0 = off[b], e1 = off[b + 1];
    V* sh = shm[w];
    int* own = owm[w];
    // is the target leaf in its own list (then it is summed on its own)
    bool mine = false;
    for (int e = e0 + lane; e < e1; e += 64) mine |= items[e] == b;
    const bool in_list = __ballot(mine) != 0ull;
#define P2P_LEAF(G)                                                                            \
    p2p_leaf<T, O, G, SOFT>(leaf, b, in_list, root, cells, items, e0, e1, P, sh, own, far, n, \
                            perm, out_shift, eps2, phi_o, ax_o, ay_o, az_o)
    if (leaf.count <= 8)
        P2P_LEAF(8);
    else if (leaf.count <= 16)
        P2P_LEAF(4);
    else if (leaf.count <= 32)
        P2P_LEAF(2);
    else
        P2P_LEAF(1);
#undef P2P_LEAF
}

void launch_p2p(const Tree& t, int precision, double eps2, const int32_t* tgt_cells,
                int32_t n_tgt_cells, const int32_t* src_off, const int32_t* src_items,
                const void* far, void* phi, void* ax, void* ay, void* az, hipStream_t s) {
    if (n_tgt_cells == 0) return;
    const int64_t shift = t.self ? 0 : t.ns;
    dim3 grid((n_tgt_cells + 3) / 4), block(256);
    const bool soft = eps2 != 0.0;
    if (precision == HFMM_FP64) {
        if (soft)
            hipLaunchKernelGGL((k_p2p<double, double, true>), grid, block, 0, s, t.cells,
                               t.root, tgt_cells, n_tgt_cells, src_off, src_items, t.p64,
                               (const double*)far, t.n, t.perm, shift, eps2, (double*)phi,
                               (double*)ax, (double*)ay, (double*)az);
        else
            hipLaunchKernelGGL((k_p2p<double, double, false>), grid, block, 0, s, t.cells,
                               t.root, tgt_cells, n_tgt_cells, src_off, src_items, t.p64,
                               (const double*)far, t.n, t.perm, shift, eps2, (double*)phi,
                               (double*)ax, (double*)ay, (double*)az);
    } else {
        if (soft)
            hipLaunchKernelGGL((k_p2p<float, float, true>), grid, block, 0, s, t.cells,
                               t.root, tgt_cells, n_tgt_cells, src_off, src_items, t.p32,
                               (const float*)far, t.n, t.perm, shift, (float)eps2, (float*)phi,
                               (float*)ax, (float*)ay, (float*)az);
        else
            hipLaunchKernelGGL((k_p2p<float, float, false>), grid, block, 0, s, t.cells,
                               t.root, tgt_cells, n_tgt_cells, src_off, src_items, t.p32,
                               (const float*)far, t.n, t.perm, shift, (float)eps2, (float*)phi,
                               (float*)ax, (float*)ay, (float*)az);
    }
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
