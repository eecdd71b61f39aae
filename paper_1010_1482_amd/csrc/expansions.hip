// Expansion kernels: P2M, M2M, L2L, P2L, L2P and M2P (Sec. 2), the M2L
// operator tables built from Eq. 4, and conversion to the paper's
// normalisation for inspection.  See common.hpp for the basis.
#include "common.hpp"
#include "expansions.hpp"

#include <algorithm>

namespace hfmm {

// ---------------------------------------------------------------------
// streaming solid harmonics: f(n, m, re, im) for every n < ND, 0 <= m <= n,
// column by column, so only a few values are live at a time
// ---------------------------------------------------------------------
template <typename T, int ND, typename F>
__device__ __forceinline__ void stream_regular(T x, T y, T z, F&& f) {
    const T r2 = x * x + y * y + z * z;
    T dre = T(1), dim = T(0);
#pragma unroll
    for (int m = 0; m < ND; ++m) {
        if (m > 0) {
            const T c = T(-1) / T(2 * m);
            T nr = c * (x * dre - y * dim);
            T ni = c * (x * dim + y * dre);
            dre = nr;
            dim = ni;
        }
        f(m, m, dre, dim);
        T pr = T(0), pi = T(0), cr = dre, ci = dim;
#pragma unroll
        for (int n = m; n + 1 < ND; ++n) {
            const T c = T(1) / T((n + 1) * (n + 1) - m * m);
            const T a = T(2 * n + 1) * z;
            T nr = (a * cr - r2 * pr) * c;
            T ni = (a * ci - r2 * pi) * c;
            pr = cr;
            pi = ci;
            cr = nr;
            ci = ni;
            f(n + 1, m, cr, ci);
        }
    }
}

template <typename T, int ND, typename F>
__device__ __forceinline__ void stream_irregular(T x, T y, T z, F&& f) {
    const T r2 = x * x + y * y + z * z;
    const T ir = rsqrt_fast(r2);
    const T ir2 = ir * ir;
    T dre = ir, dim = T(0);
#pragma unroll
    for (int m = 0; m < ND; ++m) {
        if (m > 0) {
            const T c = T(-(2 * m - 1)) * ir2;
            T nr = c * (x * dre - y * dim);
            T ni = c * (x * dim + y * dre);
            dre = nr;
            dim = ni;
        }
        f(m, m, dre, dim);
        T pr = T(0), pi = T(0), cr = dre, ci = dim;
#pragma unroll
        for (int n = m; n + 1 < ND; ++n) {
            const T a = T(2 * n + 1) * z;
            const T b = T(n * n - m * m);
            T nr = (a * cr - b * pr) * ir2;
            T ni = (a * ci - b * pi) * ir2;
            pr = cr;
            pi = ci;
            cr = nr;
            ci = ni;
            f(n + 1, m, cr, ci);
        }
    }
}

template <typename T>
__device__ __forceinline__ T cre(const double* X, int n, int m) {
    return (T)X[ridx(n, m, 0)];
}
template <typename T>
__device__ __forceinline__ T cim(const double* X, int n, int m) {
    return m == 0 ? T(0) : (T)X[ridx(n, m, 1)];
}
template <typename T>
__device__ __forceinline__ T cre(const float* X, int n, int m) {
    return (T)X[ridx(n, m, 0)];
}
template <typename T>
__device__ __forceinline__ T cim(const float* X, int n, int m) {
    return m == 0 ? T(0) : (T)X[ridx(n, m, 1)];
}

// ---------------------------------------------------------------------
// masses and centres
// ---------------------------------------------------------------------
// masses in sorted order into the FP32 and FP64 records; non-finite masses
// are flagged in the status word
__global__ void k_fill_masses(int64_t n, const int32_t* __restrict__ perm,
                              const double* __restrict__ m, const double* __restrict__ xs,
                              const double* __restrict__ ys, const double* __restrict__ zs,
                              float4* __restrict__ p32, double4* __restrict__ p64,
                              int32_t* __restrict__ status) {
    int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    bool bad = false;
    if (s < n) {
        const double q = m[perm[s]];
        bad = !isfinite(q);
        p32[s].w = (float)q;
        p64[s] = make_double4(xs[s], ys[s], zs[s], q);
    }
    if (__ballot(bad) && (threadIdx.x & 63) == 0) atomicOr(status, (int32_t)ST_MASS_NONFINITE);
}

__global__ void k_centres_geometric(const Cell* __restrict__ cells, int nc,
                                    const Root* __restrict__ root, double4* __restrict__ cen) {
    int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= nc) return;
    double o[3];
    Cell cell = cells[c];
    cell_centre(*root, cell, o);
    cen[c] = make_double4(o[0], o[1], o[2], 1.0 / cell_side(*root, cell.level));
}

// centres of mass (weights |m|), leaves from particles and parents from
// children, one level at a time (deepest first); w4 = (sum |m| x, y, z, |m|)
__global__ void k_com_level(const Cell* __restrict__ cells, int c0, int c1,
                            const double4* __restrict__ p64, const Root* __restrict__ root,
                            double4* __restrict__ w4, double4* __restrict__ cen) {
#pragma clang fp contract(off)
    int c = c0 + blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= c1) return;
    Cell cell = cells[c];
    double sx = 0, sy = 0, sz = 0, sw = 0;
    if (cell.nchild == 0) {
        for (int s = cell.first; s < cell.first + cell.count; ++s) {
            double4 q = p64[s];
            double a = fabs(q.w);
            sw += a;
            sx += a * q.x;
            sy += a * q.y;
            sz += a * q.z;
        }
    } else {
        for (int k = 0; k < cell.nchild; ++k) {
            double4 q = w4[cell.child + k];
            sx += q.x;
            sy += q.y;
            sz += q.z;
            sw += q.w;
        }
    }
    w4[c] = make_double4(sx, sy, sz, sw);
    double h = cell_side(*root, cell.level);
    if (sw > 0.0) {
        cen[c] = make_double4(sx / sw, sy / sw, sz / sw, 1.0 / h);
    } else {
        double o[3];
        cell_centre(*root, cell, o);
        cen[c] = make_double4(o[0], o[1], o[2], 1.0 / h);
    }
}

// ---------------------------------------------------------------------
// shift tables: R_n^m(u) for the M2M / L2L vectors in units of the child
// side, u = (c_child - c_parent) / h_child.  Octant table (geometric
// centres): u = (ox - 1/2, oy - 1/2, oz - 1/2); per-child table (centres of
// mass).  Stored as (re, im) pairs, triangular, FP64.
// ---------------------------------------------------------------------
template <int NP>
__global__ void k_shift_octants(double2* __restrict__ tab) {
    int o = threadIdx.x;
    if (o >= 8) return;
    double u[3] = {((o >> 2) & 1) - 0.5, ((o >> 1) & 1) - 0.5, (o & 1) - 0.5};
    double2* out = tab + o * ntri(NP);
    stream_regular<double, NP>(u[0], u[1], u[2], [&](int n, int m, double re, double im) {
        out[tri(n, m)] = make_double2(re, im);
    });
}

template <int NP>
__global__ void k_shift_children(const Cell* __restrict__ cells, int nc,
                                 const double4* __restrict__ cen, double2* __restrict__ tab) {
    int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= nc) return;
    Cell cell = cells[c];
    if (cell.parent < 0) return;
    double4 a = cen[c], b = cen[cell.parent];
    double ih = a.w;
    double u[3] = {(a.x - b.x) * ih, (a.y - b.y) * ih, (a.z - b.z) * ih};
    double2* out = tab + (int64_t)c * ntri(NP);
    stream_regular<double, NP>(u[0], u[1], u[2], [&](int n, int m, double re, double im) {
        out[tri(n, m)] = make_double2(re, im);
    });
}

__device__ inline int octant_idx(const Cell& c) {
    return ((c.ix & 1) << 2) | ((c.iy & 1) << 1) | (c.iz & 1);
}

// X_n^m of a stored m >= 0 triangle with X_n^{-m} = (-1)^m conj(X_n^m)
__device__ inline double2 tri_get(const double2* X, int n, int m) {
    if (m >= 0) return X[tri(n, m)];
    double2 v = X[tri(n, -m)];
    double s = (m & 1) ? -1.0 : 1.0;
    return make_double2(s * v.x, -s * v.y);
}
__device__ inline double2 real_get(const double* X, int n, int m) {
    int a = m < 0 ? -m : m;
    double re = X[ridx(n, a, 0)], im = a == 0 ? 0.0 : X[ridx(n, a, 1)];
    if (m >= 0) return make_double2(re, im);
    double s = (a & 1) ? -1.0 : 1.0;
    return make_double2(s * re, -s * im);
}

// ---------------------------------------------------------------------
// P2M: Mt_n^m = sum_j q_j conj(R_n^m((x_j - c) / h)) (Eq. 2 in the device
// basis).  G lanes per leaf, lanes stride over the leaf's particles, then a
// butterfly reduction across the G lanes.
// ---------------------------------------------------------------------
template <typename T, int NP>
__global__ void __launch_bounds__(256)
k_p2m(const Cell* __restrict__ cells, const int32_t* __restrict__ leaves, int nleaves,
      const double4* __restrict__ cen, const double4* __restrict__ p64,
      double* __restrict__ M, int ld) {
    constexpr int G = 8, P = NP * NP;
    const int gid = (blockIdx.x * blockDim.x + threadIdx.x) / G;
    const int sub = threadIdx.x % G;
    const bool active = gid < nleaves;
    const int c = active ? leaves[gid] : 0;
    T acc[P];
#pragma unroll
    for (int k = 0; k < P; ++k) acc[k] = T(0);
    if (active) {
        const Cell cell = cells[c];
        const double4 q = cen[c];
        const double ih = q.w;
        for (int j = cell.first + sub; j < cell.first + cell.count; j += G) {
            const double4 pj = p64[j];
            const T ux = (T)((pj.x - q.x) * ih), uy = (T)((pj.y - q.y) * ih),
                    uz = (T)((pj.z - q.z) * ih), mj = (T)pj.w;
            stream_regular<T, NP>(ux, uy, uz, [&](int n, int m, T re, T im) {
                acc[ridx(n, m, 0)] += mj * re;
                if (m > 0) acc[ridx(n, m, 1)] -= mj * im;
            });
        }
    }
#pragma unroll
    for (int d = 1; d < G; d <<= 1)
#pragma unroll
        for (int k = 0; k < P; ++k) acc[k] += __shfl_xor(acc[k], d, 64);
    if (active && sub == 0) {
        double* out = M + (int64_t)c * ld;
#pragma unroll
        for (int k = 0; k < P; ++k) out[k] = (double)acc[k];
        for (int k = P; k < ld; ++k) out[k] = 0.0;
    }
}

// ---------------------------------------------------------------------
// M2M (FP64): Mt_p[n,m] = 2^-n sum_children sum_{k,l} conj(R_k^l(u))
//                         Mt_c[n-k, m-l]
// one thread per (parent, output (n, m >= 0))
// ---------------------------------------------------------------------
template <int NP>
__global__ void k_m2m(const Cell* __restrict__ cells, int c0, int c1,
                      const double2* __restrict__ shift, int per_child,
                      double* __restrict__ M, int ld) {
    constexpr int P = NP * NP, NT = ntri(NP);
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int c = c0 + (int)(gid / NT);
    if (c >= c1) return;
    const int t = (int)(gid % NT);
    int n = 0;
    while (tri(n + 1, 0) <= t) ++n;
    const int m = t - tri(n, 0);
    const Cell cell = cells[c];
    if (cell.nchild == 0) return;
    double sr = 0.0, si = 0.0;
    for (int q = 0; q < cell.nchild; ++q) {
        const int ch = cell.child + q;
        const double2* R = per_child ? shift + (int64_t)ch * NT
                                     : shift + octant_idx(cells[ch]) * NT;
        const double* Mc = M + (int64_t)ch * ld;
        for (int k = 0; k <= n; ++k)
            for (int l = -k; l <= k; ++l) {
                const int mm = m - l;
                if (mm > n - k || mm < -(n - k)) continue;
                double2 r = tri_get(R, k, l);  // conj below
                double2 x = real_get(Mc, n - k, mm);
                sr += r.x * x.x + r.y * x.y;
                si += r.x * x.y - r.y * x.x;
            }
    }
    const double sc = ldexp(1.0, -n);
    double* out = M + (int64_t)c * ld;
    out[ridx(n, m, 0)] = sr * sc;
    if (m > 0) out[ridx(n, m, 1)] = si * sc;
}

// ---------------------------------------------------------------------
// P2L for the X list (Eq. 3 in the device basis, FP64):
//   Lt_n^m(B) += sum_j q_j conj(S_n^m((x_j - c_B) / h_B))
// One 64-lane wave per target cell with an X list (from the compact array
// of such cells; the others keep LX = 0).  The particles
// of the cell's X-list leaves are packed into chunks of CH (a lane per list
// leaf, a scan of the counts, the owner of each slot from wave_run_owner);
// lane j evaluates
// particle j of the chunk and stores its P weighted terms in LDS
// (coefficient-major, so the stores of one term are consecutive), then lane
// k adds coefficient k (and k + 64, ...) over the chunk: no cross-lane
// reduction, and every lane is busy however few particles a leaf holds.
// T: the type of the terms (FP32 for the FP32 path, whose chunks then hold
// twice as many particles in the same LDS; the sums over chunks are FP64).
// ---------------------------------------------------------------------
template <typename T, int NP, int CH, int RS, int KPL>
__device__ __forceinline__ void p2l_cell(const Cell* __restrict__ cells, int b,
                                         const int32_t* __restrict__ x_off,
                                         const int32_t* __restrict__ x_items,
                                         const double4* __restrict__ cen,
                                         const double4* __restrict__ p64,
                                         double* __restrict__ LX, int ld, T* sh, int* own,
                                         int lane) {
    constexpr int P = NP * NP;
    const int e0 = x_off[b], e1 = x_off[b + 1];
    double acc[KPL];
#pragma unroll
    for (int k = 0; k < KPL; ++k) acc[k] = 0.0;
    const double4 q = cen[b];
    const double ih = q.w;
    for (int eb = e0; eb < e1; eb += 64) {
        int first = 0, cnt = 0;
        if (eb + lane < e1) {
            const Cell src = cells[x_items[eb + lane]];
            first = src.first;
            cnt = src.count;
        }
        int tot;
        const int off = wave_excl_scan(cnt, lane, tot);
        for (int pb = 0; pb < tot; pb += CH) {
            int o = wave_run_owner(own, off, cnt, pb, CH, lane);
            const bool ok = lane < CH && pb + lane < tot;
            o = ok ? o : 0;
            const int f = __shfl(first, o, 64), fo = __shfl(off, o, 64);
            const int nv = min(CH, tot - pb);
            wave_lds_fence();
            if (ok) {
                const double4 pj = p64[f + (pb + lane - fo)];
                const T w = (T)pj.w;
                stream_irregular<T, NP>((T)((pj.x - q.x) * ih), (T)((pj.y - q.y) * ih),
                                        (T)((pj.z - q.z) * ih), [&](int n, int m, T re, T im) {
                                            sh[ridx(n, m, 0) * RS + lane] = w * re;
                                            if (m > 0) sh[ridx(n, m, 1) * RS + lane] = -w * im;
                                        });
            }
            wave_lds_fence();
#pragma unroll
            for (int kk = 0; kk < KPL; ++kk) {
                const int k = lane + 64 * kk;
                if (k < P) {
                    double a = 0.0;
                    for (int j = 0; j < nv; ++j) a += (double)sh[k * RS + j];
                    acc[kk] += a;
                }
            }
        }
    }
    double* out = LX + (int64_t)b * ld;
#pragma unroll
    for (int kk = 0; kk < KPL; ++kk) {
        const int k = lane + 64 * kk;
        if (k < P) out[k] = acc[kk];
    }
    wave_lds_fence();  // the next cell reuses sh and own
}

template <typename T, int NP>
__global__ void __launch_bounds__(64)
k_p2l(const Cell* __restrict__ cells, const int32_t* __restrict__ x_cells,
      const int32_t* __restrict__ x_off, const int32_t* __restrict__ x_items,
      const double4* __restrict__ cen, const double4* __restrict__ p64,
      double* __restrict__ LX, int ld) {
    constexpr int P = NP * NP;
    constexpr int PER = 8192 / (int)sizeof(T) / P;     // particles per chunk (<= 9 KB)
    constexpr int CH = PER < 64 ? PER : 64;
    constexpr int RS = CH + 1;                         // LDS row stride (bank spread)
    constexpr int KPL = (P + 63) / 64;                 // coefficients per lane
    __shared__ T sh[P * RS];
    __shared__ int own[64];
    p2l_cell<T, NP, CH, RS, KPL>(cells, x_cells[blockIdx.x], x_off, x_items, cen, p64, LX, ld,
                                 sh, own, threadIdx.x);
}


// ---------------------------------------------------------------------
// M2P of one expansion (Eq. 2 with its gradient) at u = (x - c) / h:
//   phi = sum Mt S(u) / h,  grad phi from dS_n^m/dz = -S_{n+1}^m and
//   (d/dx + i d/dy) S_n^m = S_{n+1}^{m+1}
// ---------------------------------------------------------------------
template <typename T, int NP, typename MT>
__device__ __forceinline__ void m2p_accumulate(const MT* Mc, T ux, T uy, T uz, T ih,
                                               T& phi, T& ax, T& ay, T& az) {
    T f = T(0), dz = T(0), hr = T(0), hi = T(0);
    stream_irregular<T, NP + 1>(ux, uy, uz, [&](int k, int l, T sr, T si) {
        const T w = l == 0 ? T(1) : T(2);
        if (k < NP) {
            T mr = cre<T>(Mc, k, l), mi = cim<T>(Mc, k, l);
            f += w * (mr * sr - mi * si);
        }
        if (k >= 1) {
            if (l <= k - 1) {
                T mr = cre<T>(Mc, k - 1, l), mi = cim<T>(Mc, k - 1, l);
                dz -= w * (mr * sr - mi * si);
            }
            if (l >= 1) {
                T mr = cre<T>(Mc, k - 1, l - 1), mi = cim<T>(Mc, k - 1, l - 1);
                hr += mr * sr - mi * si;
                hi += mr * si + mi * sr;
            }
            if (l + 1 <= k - 1) {
                T mr = cre<T>(Mc, k - 1, l + 1), mi = cim<T>(Mc, k - 1, l + 1);
                hr -= mr * sr - mi * si;
                hi += mr * si + mi * sr;
            }
        }
    });
    const T ih2 = ih * ih;
    phi += f * ih;
    ax += hr * ih2;
    ay += hi * ih2;
    az += dz * ih2;
}

// ---------------------------------------------------------------------
// Far field of one target leaf per wave, any p.  A batch of up to 64 list
// cells is packed with a ballot: the cell ids and, per cell, the offset from
// its centre to the leaf's reference point cb in units of its side (formed
// in FP64) with 1/h.  Their coefficient rows are then staged FB at a time in
// the wave's LDS slice (the wave copies the rows with 16-byte loads), and
// lane g * TW + t evaluates cells g, g + G, ... of the slice at target t.
// ---------------------------------------------------------------------
template <int NP, typename MT>
struct FarShape {
    static constexpr int LD = (NP * NP + 15) / 16 * 16;  // row length of M
    // rows staged at once: at most 8 KB of coefficients per wave
    static constexpr int FB = (8192 / (LD * (int)sizeof(MT))) < 16
                                  ? (8192 / (LD * (int)sizeof(MT)) < 2 ? 2 : 8192 / (LD * (int)sizeof(MT)))
                                  : 16;
};

template <typename T, int NP, typename MT, int G>
__device__ __forceinline__ void farp_batch(bool valid, int k, const double4& cb,
                                           const double4* __restrict__ cen,
                                           const MT* __restrict__ M, int32_t* ids,
                                           typename Vec4<T>::type* offs, MT* rows, T rx, T ry,
                                           T rz, T& phi, T& ax, T& ay, T& az) {
    using V = typename Vec4<T>::type;
    using S = FarShape<NP, MT>;
    constexpr int TW = 64 / G, Q = S::LD * (int)sizeof(MT) / 16;  // 16-byte chunks per row
    const int lane = threadIdx.x & 63, g = lane / TW;
    const uint64_t bal = __ballot(valid);
    const int nb = __popcll(bal);
    if (nb == 0) return;  // uniform per wave
    V o{};
    if (valid) {
        const double4 qc = cen[k];
        o = V{(T)((cb.x - qc.x) * qc.w), (T)((cb.y - qc.y) * qc.w), (T)((cb.z - qc.z) * qc.w),
              (T)qc.w};
    }
    const int pos = __popcll(bal & lanes_below(lane));
    wave_lds_fence();
    if (valid) {
        ids[pos] = k;
        offs[pos] = o;
    }
    wave_lds_fence();
    for (int sb = 0; sb < nb; sb += S::FB) {
        const int ns = min(S::FB, nb - sb);
        // rows of cells sb .. sb + ns, 16 bytes per lane and load
        for (int c = lane; c < ns * Q; c += 64) {
            const int i = c / Q, q = c - i * Q;
            const uint4 v = *((const uint4*)(M + (int64_t)ids[sb + i] * S::LD) + q);
            *((uint4*)(rows + i * S::LD) + q) = v;
        }
        wave_lds_fence();
        for (int j0 = 0; j0 < ns; j0 += G) {
            const int j = j0 + g;
            if (j < ns) {
                const V d = offs[sb + j];
                m2p_accumulate<T, NP>(rows + j * S::LD, rx * d.w + d.x, ry * d.w + d.y,
                                      rz * d.w + d.z, d.w, phi, ax, ay, az);
            }
        }
        wave_lds_fence();
    }
}

// The M2P terms of the box's list items[e0, e1) (the FMM's W list, and V
// for a box without sources) at its targets.
template <typename T, int NP, typename MT, int G>
__device__ __forceinline__ void farp_box(const TBox& leaf, const double4& cb,
                                          const double4* __restrict__ cen,
                                          const double4* __restrict__ p64,
                                          const int32_t* __restrict__ items, int e0, int e1,
                                          const MT* __restrict__ M, int32_t* ids,
                                          typename Vec4<T>::type* offs, MT* rows,
                                          T* __restrict__ far, int64_t n) {
    constexpr int TW = 64 / G;
    const int lane = threadIdx.x & 63, t = lane % TW;
    for (int c0 = 0; c0 < leaf.count; c0 += TW) {
        const bool ok = c0 + t < leaf.count;
        const int64_t s = (int64_t)leaf.first + c0 + t;
        T rx = T(0), ry = T(0), rz = T(0);
        if (ok) {
            const double4 pj = p64[s];
            rx = (T)(pj.x - cb.x);
            ry = (T)(pj.y - cb.y);
            rz = (T)(pj.z - cb.z);
        }
        T phi = T(0), ax = T(0), ay = T(0), az = T(0);
        for (int eb = e0; eb < e1; eb += 64) {
            const bool v = eb + lane < e1;
            farp_batch<T, NP, MT, G>(v, v ? items[eb + lane] : 0, cb, cen, M, ids, offs, rows,
                                     rx, ry, rz, phi, ax, ay, az);
        }
#pragma unroll
        for (int d = TW; d < 64; d <<= 1) {
            phi += __shfl_xor(phi, d, 64);
            ax += __shfl_xor(ax, d, 64);
            ay += __shfl_xor(ay, d, 64);
            az += __shfl_xor(az, d, 64);
        }
        if (ok && lane < TW) {
            far[s] = phi;
            far[n + s] = ax;
            far[2 * n + s] = ay;
            far[3 * n + s] = az;
        }
    }
}

// L2P at every target (Eq. 3 with its gradient, dR_n^m/dz = R_{n-1}^m,
// (d/dx + i d/dy) R_n^m = R_{n-1}^{m+1}) from the local expansion of its
// box's host cell (none outside the root), one thread per sorted target;
// ADD: add to far (the M2P terms written there first) instead of storing.
template <typename T, int NP, bool ADD>
__global__ void __launch_bounds__(256)
k_l2p(Targets tg, const double4* __restrict__ cen, const double* __restrict__ L, int ld,
      T* __restrict__ far) {
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t n = tg.n;
    if (s >= n) return;
    const int b = tg.box[tg.box_of[s]].host;
    T phi = T(0), ax = T(0), ay = T(0), az = T(0);
    if (b >= 0) {
        const double4 pj = tg.p64[s];
        const double4 q = cen[b];
        const double ihd = q.w;
        const T ux = (T)((pj.x - q.x) * ihd), uy = (T)((pj.y - q.y) * ihd),
                uz = (T)((pj.z - q.z) * ihd);
        const double* Lb = L + (int64_t)b * ld;
        T f = T(0), gz = T(0), gr = T(0), gi = T(0);
        stream_regular<T, NP>(ux, uy, uz, [&](int k, int l, T rr, T ri) {
            const T w = l == 0 ? T(1) : T(2);
            {
                T lr = cre<T>(Lb, k, l), li = cim<T>(Lb, k, l);
                f += w * (lr * rr - li * ri);
            }
            if (k + 1 < NP) {
                T ar = cre<T>(Lb, k + 1, l), ai = cim<T>(Lb, k + 1, l);
                gz += w * (ar * rr - ai * ri);
                if (l >= 1) {
                    T br = cre<T>(Lb, k + 1, l - 1), bi = cim<T>(Lb, k + 1, l - 1);
                    gr += br * rr - bi * ri;
                    gi += br * ri + bi * rr;
                }
                T cr = cre<T>(Lb, k + 1, l + 1), ci = cim<T>(Lb, k + 1, l + 1);
                gr -= cr * rr - ci * ri;
                gi += cr * ri + ci * rr;
            }
        });
        const T ih = (T)ihd, ih2 = ih * ih;
        phi = f * ih;
        ax = gr * ih2;
        ay = gi * ih2;
        az = gz * ih2;
    }
    if (ADD) {
        phi += far[s];
        ax += far[n + s];
        ay += far[2 * n + s];
        az += far[3 * n + s];
    }
    far[s] = phi;
    far[n + s] = ax;
    far[2 * n + s] = ay;
    far[3 * n + s] = az;
}

// geometric centre of a box as the reference point of its targets' offsets
__device__ inline double4 box_ref(const Root& r, const TBox& bx) {
    double c[3];
    cell_centre(r, box_cell(bx), c);
    return make_double4(c[0], c[1], c[2], 0.0);
}

// W-list M2P of the FMM, one wave per target leaf; MT: the multipoles'
// type (an FP32 copy for the FP32 path).  Short, uneven lists: a wave per
// leaf replaces the divergent per-particle loops.  (The treecode's long,
// even lists keep one thread per particle, k_treecode_far: there every lane
// has a target, while a wave per leaf of ~10 particles leaves lanes idle.)
template <typename T, int NP, typename MT>
__global__ void __launch_bounds__(256, sizeof(T) == 4 ? 6 : 1)
k_farp(const Root* __restrict__ root, Targets tg, const double4* __restrict__ cen,
       const int32_t* __restrict__ off, const int32_t* __restrict__ items,
       const MT* __restrict__ M, T* __restrict__ far) {
    using V = typename Vec4<T>::type;
    using S = FarShape<NP, MT>;
    __shared__ int32_t sid[4][64];
    __shared__ V soff[4][64];
    __shared__ __align__(16) MT srow[4][S::FB * S::LD];
    const int w = threadIdx.x >> 6;
    const int li = blockIdx.x * 4 + w;
    if (li >= tg.nbox) return;  // uniform per wave
    const TBox bx = tg.box[li];
    const int row = list_row(tg, li, bx);
    const double4 cb = box_ref(*root, bx);
    const int e0 = off[row], e1 = off[row + 1];
#define FARP_BOX(G)                                                                           \
    farp_box<T, NP, MT, G>(bx, cb, cen, tg.p64, items, e0, e1, M, sid[w], soff[w], srow[w], \
                           far, tg.n)
    if (bx.count <= 4)
        FARP_BOX(16);
    else if (bx.count <= 8)
        FARP_BOX(8);
    else if (bx.count <= 16)
        FARP_BOX(4);
    else if (bx.count <= 32)
        FARP_BOX(2);
    else
        FARP_BOX(1);
#undef FARP_BOX
}

// Treecode far field: M2P over the accepted list of the target's box, one
// thread per sorted target (neighbouring threads share a box and read the
// same cells); MT: FP32 copy of the multipoles for the FP32 path.
template <typename T, int NP, typename MT>
__global__ void __launch_bounds__(256)
k_treecode_far(Targets tg, const double4* __restrict__ cen, const int32_t* __restrict__ a_off,
               const int32_t* __restrict__ a_items, const MT* __restrict__ M, int ld,
               T* __restrict__ far) {
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t n = tg.n;
    if (s >= n) return;
    const int b = tg.box_of[s];
    const int row = list_row(tg, b, tg.box[b]);
    const double4 pj = tg.p64[s];
    T phi = T(0), ax = T(0), ay = T(0), az = T(0);
    for (int e = a_off[row]; e < a_off[row + 1]; ++e) {
        const int C = a_items[e];
        const double4 qc = cen[C];
        const double ic = qc.w;
        m2p_accumulate<T, NP>(M + (int64_t)C * ld, (T)((pj.x - qc.x) * ic),
                              (T)((pj.y - qc.y) * ic), (T)((pj.z - qc.z) * ic), (T)ic, phi, ax,
                              ay, az);
    }
    far[s] = phi;
    far[n + s] = ax;
    far[2 * n + s] = ay;
    far[3 * n + s] = az;
}

// ---------------------------------------------------------------------
// M2P at p = 3 (monopole, dipole, quadrupole: the treecode's quadrupole
// moments) in Cartesian form.  With the irregular harmonics of degree <= 2
// written out, S_0^0 = 1/r, S_1^0 = z/r^3, S_1^1 = -(x + iy)/r^3,
// S_2^0 = (3z^2 - r^2)/r^5, S_2^1 = -3z(x + iy)/r^5, S_2^2 = 3(x + iy)^2/r^5,
// the truncated expansion of a cell is
//   f(u) = q/r + (D.u)/r^3 + (u.Q.u)/r^5,
// q = M00, D = (-2 Re M11, 2 Im M11, M10) and the traceless symmetric
//   Q = [[6 Re M22 - M20, -6 Im M22, -3 Re M21],
//        [-6 Im M22, -6 Re M22 - M20, 3 Im M21],
//        [-3 Re M21, 3 Im M21, 2 M20]],
// the same function the degree-by-degree sum evaluates, and its gradient is
//   D/r^3 + 2 Q.u/r^5 - u (q/r^3 + 3 (D.u)/r^5 + 5 (u.Q.u)/r^7).
// Per cell: (q, Dx, Dy, Dz), (Qxx, Qyy, Qzz, Qxy), (Qxz, Qyz, 0, 0).
// ---------------------------------------------------------------------
template <typename TC>
__global__ void k_cart3(const double* __restrict__ M, int ld, int ncells, TC* __restrict__ C) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= ncells) return;
    const double* X = M + (int64_t)c * ld;
    const double m00 = X[ridx(0, 0, 0)], m10 = X[ridx(1, 0, 0)];
    const double m11r = X[ridx(1, 1, 0)], m11i = X[ridx(1, 1, 1)];
    const double m20 = X[ridx(2, 0, 0)], m21r = X[ridx(2, 1, 0)], m21i = X[ridx(2, 1, 1)];
    const double m22r = X[ridx(2, 2, 0)], m22i = X[ridx(2, 2, 1)];
    TC* o = C + (int64_t)c * 12;
    o[0] = (TC)m00;
    o[1] = (TC)(-2.0 * m11r);
    o[2] = (TC)(2.0 * m11i);
    o[3] = (TC)m10;
    o[4] = (TC)(6.0 * m22r - m20);
    o[5] = (TC)(-6.0 * m22r - m20);
    o[6] = (TC)(2.0 * m20);
    o[7] = (TC)(-6.0 * m22i);
    o[8] = (TC)(-3.0 * m21r);
    o[9] = (TC)(3.0 * m21i);
    o[10] = TC(0);
    o[11] = TC(0);
}

// one evaluation from the moments r0 = (q, D), r1 = (Qxx, Qyy, Qzz, Qxy),
// r2 = (Qxz, Qyz, -, -) at u (in units of the cell side h, ih = 1/h)
template <typename T, typename V>
__device__ __forceinline__ void m2p_cart3(const V& r0, const V& r1, const V& r2, T ux, T uy,
                                          T uz, T ih, T& phi, T& ax, T& ay, T& az) {
    const T q = r0.x, dx = r0.y, dy = r0.z, dz = r0.w;
    const T qxx = r1.x, qyy = r1.y, qzz = r1.z, qxy = r1.w, qxz = r2.x, qyz = r2.y;
    const T r2n = ux * ux + uy * uy + uz * uz;
    const T ir = rsqrt_fast(r2n), ir2 = ir * ir;
    const T ir3 = ir * ir2, ir5 = ir3 * ir2, ir7 = ir5 * ir2;
    const T du = dx * ux + dy * uy + dz * uz;
    const T qx = qxx * ux + qxy * uy + qxz * uz;
    const T qy = qxy * ux + qyy * uy + qyz * uz;
    const T qz = qxz * ux + qyz * uy + qzz * uz;
    const T uqu = ux * qx + uy * qy + uz * qz;
    phi += (q * ir + du * ir3 + uqu * ir5) * ih;
    const T sc = q * ir3 + T(3) * du * ir5 + T(5) * uqu * ir7;
    const T ih2 = ih * ih;
    ax += (dx * ir3 + T(2) * qx * ir5 - ux * sc) * ih2;
    ay += (dy * ir3 + T(2) * qy * ir5 - uy * sc) * ih2;
    az += (dz * ir3 + T(2) * qz * ir5 - uz * sc) * ih2;
}

// One batch of list cells of a target leaf: lane j (j < B) offers cell k
// when `valid`; the valid cells are packed at the front of the wave's LDS
// slice, each as its moments and (r3) the offset from the cell's centre to
// the leaf's reference point cb in units of the cell side, formed in FP64,
// with 1/h.  The offset of a target from cell C is then (x - cb) / h_C + r3,
// one multiply-add per axis from the target's own FP64-formed offset.  Lane
// g * TW + t (g < G) takes target t and the packed cells g, g + G, ...; the
// slots past the batch up to the next multiple of G (at most B <= 64, a
// multiple of G) hold zero moments at unit distance with 1/h = 0, whose
// terms are exactly zero.  Lanes past G * TW compute on clamped slots and
// are never summed.
template <typename T>
__device__ __forceinline__ void far3_batch(bool valid, int k, const double4& cb,
                                           const double4* __restrict__ cen,
                                           const T* __restrict__ C,
                                           typename Vec4<T>::type* sh, int G, int g, T rx, T ry,
                                           T rz, T& phi, T& ax, T& ay, T& az) {
    using V = typename Vec4<T>::type;
    const int lane = threadIdx.x & 63;
    const uint64_t bal = __ballot(valid);
    const int nb = __popcll(bal);
    if (nb == 0) return;  // uniform per wave
    V r0{}, r1{}, r2{}, r3{};
    if (valid) {
        const V* ck = (const V*)(C + (int64_t)k * 12);
        r0 = ck[0];
        r1 = ck[1];
        r2 = ck[2];
        const double4 qc = cen[k];
        r3 = V{(T)((cb.x - qc.x) * qc.w), (T)((cb.y - qc.y) * qc.w), (T)((cb.z - qc.z) * qc.w),
               (T)qc.w};
    }
    const int pos = __popcll(bal & lanes_below(lane));
    const int nr = (nb + G - 1) / G * G;
    wave_lds_fence();
    if (valid) {
        sh[pos] = r0;
        sh[64 + pos] = r1;
        sh[128 + pos] = r2;
        sh[192 + pos] = r3;
    }
    if (lane >= nb && lane < nr) {
        const V z{};
        sh[lane] = z;
        sh[64 + lane] = z;
        sh[128 + lane] = z;
        sh[192 + lane] = V{T(1), T(0), T(0), T(0)};
    }
    wave_lds_fence();
#pragma unroll 2
    for (int j0 = 0; j0 < nr; j0 += G) {
        const int j = min(j0 + g, 63);
        const V a = sh[j], b = sh[64 + j], c = sh[128 + j], d = sh[192 + j];
        m2p_cart3<T>(a, b, c, rx * d.w + d.x, ry * d.w + d.y, rz * d.w + d.z, d.w, phi, ax,
                     ay, az);
    }
}

// The far field of one target box.  Lane groups are sized to the box:
// TW = min(count, 64) lanes per group, G = 64 / TW groups (a leaf of 10
// particles keeps 60 lanes busy where power-of-two groups of 16 kept 40),
// batches of B = G * (64 / G) cells.  WALK: the M2P cells are read from the
// FMM lists (the box's CSR items: W, and V for a box without sources; then
// the V slots of cell b, the box's leaf or its host, and of each ancestor,
// the non-empty ones queued in the wave's id ring `q` so that every batch
// but the last is full); otherwise from the box's CSR list items[e0, e1).
template <typename T, bool WALK>
__device__ __forceinline__ void far3_box(const Cell* __restrict__ cells, int b, const TBox& leaf,
                                          const double4& cb, const double4* __restrict__ cen,
                                          const double4* __restrict__ p64,
                                          const int32_t* __restrict__ items, int e0, int e1,
                                          const int32_t* __restrict__ vsrc,
                                          const T* __restrict__ C,
                                          typename Vec4<T>::type* sh, int* q,
                                          T* __restrict__ far, int64_t n) {
    const int lane = threadIdx.x & 63;
    const int TW = leaf.count < 64 ? leaf.count : 64;
    const int G = 64 / TW, B = G * (64 / G);
    const int g = lane / TW, t = lane - g * TW;  // g == G: an idle lane
    for (int c0 = 0; c0 < leaf.count; c0 += TW) {
        const bool ok = g < G && c0 + t < leaf.count;
        const int64_t s = (int64_t)leaf.first + c0 + t;
        T rx = T(0), ry = T(0), rz = T(0);
        if (ok) {
            const double4 pj = p64[s];
            rx = (T)(pj.x - cb.x);
            ry = (T)(pj.y - cb.y);
            rz = (T)(pj.z - cb.z);
        }
        T phi = T(0), ax = T(0), ay = T(0), az = T(0);
        for (int eb = e0; eb < e1; eb += B) {
            const bool v = lane < B && eb + lane < e1;
            far3_batch<T>(v, v ? items[eb + lane] : 0, cb, cen, C, sh, G, g, rx, ry, rz, phi,
                          ax, ay, az);
        }
        if (WALK) {
            // ring of 256 ids: at most B - 1 + 64 <= 127 are queued at once
            const uint64_t below = lanes_below(lane);
            int head = 0, tail = 0;
            for (int a = b; a >= 0; a = cells[a].parent) {
                const int32_t* row = vsrc + (int64_t)a * 216;
                for (int q0 = 0; q0 < 216; q0 += 64) {
                    const int k = q0 + lane < 216 ? row[q0 + lane] : -1;
                    const uint64_t bal = __ballot(k >= 0);
                    wave_lds_fence();
                    if (k >= 0) q[(tail + __popcll(bal & below)) & 255] = k;
                    tail += __popcll(bal);
                    wave_lds_fence();
                    while (tail - head >= B) {
                        const int kk = q[(head + lane) & 255];
                        far3_batch<T>(lane < B, kk, cb, cen, C, sh, G, g, rx, ry, rz, phi, ax,
                                      ay, az);
                        head += B;
                    }
                }
            }
            if (tail > head) {
                const int kk = q[(head + lane) & 255];
                far3_batch<T>(lane < tail - head, kk, cb, cen, C, sh, G, g, rx, ry, rz, phi, ax,
                              ay, az);
            }
        }
        // group 0 adds the other groups' partial sums of its target
        T sphi = phi, sax = ax, say = ay, saz = az;
        for (int h = 1; h < G; ++h) {
            const int src = h * TW + (t < TW ? t : 0);
            sphi += __shfl(phi, src, 64);
            sax += __shfl(ax, src, 64);
            say += __shfl(ay, src, 64);
            saz += __shfl(az, src, 64);
        }
        if (ok && g == 0) {
            far[s] = sphi;
            far[n + s] = sax;
            far[2 * n + s] = say;
            far[3 * n + s] = saz;
        }
    }
}

// Treecode far field at p = 3 from the Cartesian moments (k_cart3), one
// wave per target box, lane groups sized to its target count.  off/items:
// the box's M2P list (Barnes-Hut), or with WALK its FMM-list part (W, and V
// for a box without sources), the V lists of the cells above being read
// from vsrc.
template <typename T, bool WALK>
__global__ void __launch_bounds__(256, 6)
k_treecode_far3(const Cell* __restrict__ cells, const Root* __restrict__ root, Targets tg,
                const double4* __restrict__ cen, const int32_t* __restrict__ off,
                const int32_t* __restrict__ items, const int32_t* __restrict__ vsrc,
                const T* __restrict__ C, T* __restrict__ far) {
    using V = typename Vec4<T>::type;
    __shared__ V shm[4][256];
    __shared__ int idq[4][WALK ? 256 : 1];
    const int w = threadIdx.x >> 6;
    const int li = blockIdx.x * 4 + w;
    if (li >= tg.nbox) return;  // uniform per wave
    const TBox bx = tg.box[li];
    if (bx.count <= 0) return;
    const int row = list_row(tg, li, bx);
    const double4 cb = box_ref(*root, bx);
    const int walk_from = bx.leaf >= 0 ? bx.leaf : bx.host;
    far3_box<T, WALK>(cells, walk_from, bx, cb, cen, tg.p64, items, off[row], off[row + 1], vsrc,
                      C, shm[w], idq[w], far, tg.n);
}

__global__ void k_to_float(const double* __restrict__ a, int64_t n, float* __restrict__ b) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) b[i] = (float)a[i];
}

// ---------------------------------------------------------------------
// M2L operator of one offset class from Eq. 4.  With the identity of Sec. 5.2,
// Y_N^M / (A_N^M rho^{N+1}) = (N-|M|)! P_N^|M|(cos a) e^{iM b} / rho^{N+1},
// and the change to the device basis (Lb = L / A_j^k, Mb = A_n^m M), the
// factors A_n^m A_j^k of Eq. 4 cancel and the complex coefficient of
// M_n^m in L_j^k becomes
//   c(j,k,n,m) = i^{|k-m|-|k|-|m|} (-1)^j (N-|M|)! P_N^|M| e^{iM b} / rho^{N+1}
// with N = j + n, M = m - k, (rho, a, b) the spherical coordinates of
// c_target - c_source in cell units (offsets are source minus target, so the
// vector is -d).  Conjugate symmetry of M folds m and -m into real entries.
// ---------------------------------------------------------------------
__device__ inline double factorial_d(int n) {
    double f = 1.0;
    for (int i = 2; i <= n; ++i) f *= (double)i;
    return f;
}

// real-layout index -> (n, m, part)
__device__ inline void rdecode(int r, int& n, int& m, int& part) {
    n = 0;
    while ((n + 1) * (n + 1) <= r) ++n;
    int o = r - n * n;
    if (o == 0) {
        m = 0;
        part = 0;
    } else {
        m = (o + 1) / 2;
        part = (o + 1) % 2;
    }
}

// One block per offset class (343 blocks, 27 of them adjacent offsets that
// stay zero).  The block tabulates, for this class, the Sec. 5.2 quantity
// (N-|M|)! P_N^|M|(cos a) / rho^{N+1} for N <= 2p-2 (Eqs. 7-9) and
// cos(M b), sin(M b) in LDS, then threads fill the real entries.  Writes the
// FP64 layout T64[cls][ri][ro] and/or the FP32 matrix-core layout
// Tsw[cls][rb][q][lane][4] with T[16 rb + (lane & 15)][16 q + 4 (lane >> 4) + r].
constexpr int kNmax = 2 * HFMM_MAX_P - 1;

// LDS table of one offset class; returns false for the 27 adjacent offsets
__device__ inline bool m2l_class_table(int p, int cls, double (*pt)[kNmax],
                                       double (*cs)[2]) {
    const int ND = 2 * p - 1;
    const int dx = cls / 49 - 3, dy = (cls / 7) % 7 - 3, dz = cls % 7 - 3;
    const bool far = max(abs(dx), max(abs(dy), abs(dz))) >= 2;
    if (far && (int)threadIdx.x < ND) {
        const int a = threadIdx.x;  // order |M|
        const double vx = -dx, vy = -dy, vz = -dz;
        const double rxy = sqrt(vx * vx + vy * vy);
        const double rho = sqrt(vx * vx + vy * vy + vz * vz);
        const double x = vz / rho, sn = rxy / rho;
        const double beta = (vx == 0.0 && vy == 0.0) ? 0.0 : atan2(vy, vx);
        cs[a][0] = cos(a * beta);
        cs[a][1] = sin(a * beta);
        double pmm = 1.0;  // Eq. 8
        for (int i = 1; i <= a; ++i) pmm *= -(double)(2 * i - 1) * sn;
        double rinv = 1.0 / rho, rpow = rinv;  // 1 / rho^{N+1}
        for (int i = 0; i < a; ++i) rpow *= rinv;
        double pm1 = 0.0, pc = pmm, fct = 1.0;  // P_{N-1}, P_N, (N - a)!
        for (int N = a; N < ND; ++N) {
            pt[N][a] = fct * pc * rpow;
            const double pn = N == a ? x * (2 * a + 1) * pmm                                 // Eq. 9
                                     : (x * (2 * N + 1) * pc - (N + a) * pm1) / (N - a + 1);  // Eq. 7
            pm1 = pc;
            pc = pn;
            fct *= (double)(N - a + 1);
            rpow *= rinv;
        }
    }
    __syncthreads();
    return far;
}

// real entry (row ro, column ri) of the class operator from its table:
// c(j,k,n,+-m) = i^{|k-m|-|k|-|m|} (-1)^j pt[j+n][|m-k|] e^{i (m-k) b}
__device__ inline double m2l_entry(int ro, int ri, const double (*pt)[kNmax],
                                   const double (*cs)[2]) {
    int j, k, po, n, m, pi;
    rdecode(ro, j, k, po);
    rdecode(ri, n, m, pi);
    auto coef = [&](int mm) {
        const int M = mm - k, aM = M < 0 ? -M : M;
        const int ev = abs(k - mm) - abs(k) - abs(mm);
        const double sg = (((ev / 2) & 1) ? -1.0 : 1.0) * ((j & 1) ? -1.0 : 1.0);
        const double v = sg * pt[j + n][aM];
        return make_double2(v * cs[aM][0], v * (M < 0 ? -cs[aM][1] : cs[aM][1]));
    };
    if (m == 0) {
        double2 c0 = coef(0);
        return pi == 0 ? (po == 0 ? c0.x : c0.y) : 0.0;
    }
    double2 cp = coef(m), cm = coef(-m);
    if (po == 0) return pi == 0 ? cp.x + cm.x : -(cp.y - cm.y);
    return pi == 0 ? cp.y + cm.y : cp.x - cm.x;
}

// gridDim.y blocks per offset class (343 classes, 27 of them adjacent
// offsets that stay zero).  Each block tabulates, for its class, the Sec. 5.2
// quantity (N-|M|)! P_N^|M|(cos a) / rho^{N+1} for N <= 2p-2 (Eqs. 7-9) and
// cos(M b), sin(M b) in LDS, then its threads fill a share of the real
// entries in the order they are stored (consecutive threads, consecutive
// addresses; the padding is written as zeros).  Layouts: FP64
// T64[cls][ri][ro], or the matrix-core chunks [cls][rb][q][lane][E] holding
// T[16 rb + (lane & 15)][KS q + 4 r + (lane >> 4)] at element r.
__global__ void __launch_bounds__(256)
k_m2l_ops(int p, int layout, void* __restrict__ T, int RB, int KQ) {
    // layout 0: FP64 [class][ri][ro] (vector units); 1: FP32 matrix-core
    // chunks (E = 4, KS = 16); 2: FP64 matrix-core chunks (E = 2, KS = 8).
    // The r-major order puts the padding of the last block into whole
    // products, which the kernel skips.
    __shared__ double pt[kNmax][kNmax];
    __shared__ double cs[kNmax][2];
    const int P = p * p;
    const int cls = blockIdx.x;
    const bool far = m2l_class_table(p, cls, pt, cs);
    const int64_t per = (int64_t)P * P;
    const int64_t step = (int64_t)gridDim.y * blockDim.x;
    const int64_t first = (int64_t)blockIdx.y * blockDim.x + threadIdx.x;
    if (layout == 0) {
        for (int64_t e = first; e < per; e += step) {
            const int ri = (int)(e / P), ro = (int)(e % P);
            ((double*)T)[(int64_t)cls * per + e] = far ? m2l_entry(ro, ri, pt, cs) : 0.0;
        }
        return;
    }
    const int E = layout == 1 ? 4 : 2, KS = layout == 1 ? 16 : 8;
    const int64_t tot = (int64_t)RB * KQ * 64 * E;
    for (int64_t o = first; o < tot; o += step) {
        const int r = (int)(o % E);
        const int64_t u = o / E;
        const int lane = (int)(u % 64), q = (int)((u / 64) % KQ), rb = (int)(u / (64 * KQ));
        const int ro = 16 * rb + (lane & 15), ri = KS * q + 4 * r + (lane >> 4);
        const double val = (far && ro < P && ri < P) ? m2l_entry(ro, ri, pt, cs) : 0.0;
        if (layout == 1)
            ((float*)T)[(int64_t)cls * tot + o] = (float)val;
        else
            ((double*)T)[(int64_t)cls * tot + o] = val;
    }
}

__device__ inline int mu_exp_d(int n) {  // floor(log2((sqrt3/2)^n / n!))
    double v = 1.0;
    for (int i = 1; i <= n; ++i) v *= 0.8660254037844386 / (double)i;
    return ilogb(v);
}

// Low-precision operators.  pass 0: bexp[j] = max exponent of T_{jn} 2^{mu_n}
// over classes and columns; pass 1: T' = T 2^{mu_n - b_j}, b_j = bexp[j] + 1,
// split into hi and lo (lo may be null) in the layout
// [cls][rb][q][lane][8], element (16 rb + (lane & 15), 32 q + 8 (lane >> 4) + j).
template <typename T16>
__global__ void __launch_bounds__(256)
k_m2l_ops_lp(int p, int pass, int RB, int KQ, int32_t* __restrict__ bexp,
             T16* __restrict__ hi, T16* __restrict__ lo) {
    __shared__ double pt[kNmax][kNmax];
    __shared__ double cs[kNmax][2];
    __shared__ int bmax[kNmax];  // pass 0: block maximum per output degree
    const int P = p * p;
    const int cls = blockIdx.x;
    if (threadIdx.x < kNmax) bmax[threadIdx.x] = INT_MIN;
    const bool far = m2l_class_table(p, cls, pt, cs);
    const int R = 16 * RB, K = 32 * KQ;
    const int64_t per = (int64_t)R * K;
    for (int64_t e = threadIdx.x; e < per; e += blockDim.x) {
        const int ro = (int)(e / K), ri = (int)(e % K);
        double val = 0.0;
        int j = 0, n = 0;
        if (far && ro < P && ri < P) {
            val = m2l_entry(ro, ri, pt, cs);
            j = 0;
            while ((j + 1) * (j + 1) <= ro) ++j;
            while ((n + 1) * (n + 1) <= ri) ++n;
        }
        if (pass == 0) {
            if (val != 0.0) atomicMax(&bmax[j], ilogb(fabs(val)) + mu_exp_d(n));
            continue;
        }
        double t = val == 0.0 ? 0.0 : ldexp(val, mu_exp_d(n) - (bexp[j] + 1));
        const int rb = ro / 16, il = ro % 16;
        const int q = ri / 32, g = (ri % 32) / 8, jj = ri % 8;
        const int64_t idx = ((((int64_t)cls * RB + rb) * KQ + q) * 64 + g * 16 + il) * 8 + jj;
        const T16 h = (T16)(float)t;
        hi[idx] = h;
        if (lo) lo[idx] = (T16)(float)(t - (double)(float)h);
    }
    if (pass == 0) {
        __syncthreads();
        if ((int)threadIdx.x < p && bmax[threadIdx.x] != INT_MIN)
            atomicMax(&bexp[threadIdx.x], bmax[threadIdx.x]);
    }
}

void run_m2l_ops_lp(int p, int precision, int RB, int KQ, int32_t* bexp, void* hi, void* lo,
                    hipStream_t s) {
    const bool bf = precision == HFMM_M2L_BF16 || precision == HFMM_M2L_BF16X3;
    for (int pass = 0; pass < 2; ++pass) {
        if (bf)
            hipLaunchKernelGGL((k_m2l_ops_lp<__bf16>), dim3(343), dim3(256), 0, s, p, pass, RB,
                               KQ, bexp, (__bf16*)hi, (__bf16*)lo);
        else
            hipLaunchKernelGGL((k_m2l_ops_lp<_Float16>), dim3(343), dim3(256), 0, s, p, pass,
                               RB, KQ, bexp, (_Float16*)hi, (_Float16*)lo);
        LAUNCH_CHECK();
    }
}

// pack Mt (FP64, p*p per cell) into the M2L operand: ld = Kp (zero padded),
// one extra zero row at index ncells for absent sources
template <typename TO>
// Rows of the matrix-core M2L operand.  Within each block of 4 NR (NR = 4
// floats or 2 doubles per 16-byte chunk), position NR g + r holds element
// 4 NR q + 4 r + g (the operator's r-major contraction order); the zero row
// ncells stands for an absent source.
__global__ void k_pack(const double* __restrict__ M, int ldm, int ncells, int P, int ld,
                       TO* __restrict__ out) {
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t tot = (int64_t)(ncells + 1) * ld;
    if (gid >= tot) return;
    const int c = (int)(gid / ld), pos = (int)(gid % ld);
    // blocks of 16 floats (4 lane groups x 4 products) or 8 doubles (x 2)
    constexpr int NR = 16 / sizeof(TO);
    const int blk = pos / (4 * NR), w = pos % (4 * NR);
    const int k = blk * 4 * NR + 4 * (w % NR) + w / NR;
    double v = (c < ncells && k < P) ? M[(int64_t)c * ldm + k] : 0.0;
    out[gid] = (TO)v;
}

// device basis -> the paper's normalisation:
//   M_n^m = h^n Mt_n^m / A_n^m,  L_n^m = A_n^m Lt_n^m / h^{n+1}
__global__ void k_export(const double* __restrict__ X, int ld, int ncells, int p,
                         const double4* __restrict__ cen, int which,
                         double* __restrict__ out) {
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int NT = p * (p + 1) / 2;
    if (gid >= (int64_t)ncells * NT) return;
    const int c = (int)(gid / NT), t = (int)(gid % NT);
    int n = 0;
    while ((n + 1) * (n + 2) / 2 <= t) ++n;
    const int m = t - n * (n + 1) / 2;
    const double h = 1.0 / cen[c].w;
    const double A = 1.0 / sqrt(factorial_d(n - m) * factorial_d(n + m));
    double hn = 1.0;
    for (int i = 0; i < n; ++i) hn *= h;
    const double f = which == 0 ? hn / A : A / (hn * h);
    const double* Xc = X + (int64_t)c * ld;
    out[gid * 2] = f * Xc[ridx(n, m, 0)];
    out[gid * 2 + 1] = m == 0 ? 0.0 : f * Xc[ridx(n, m, 1)];
}

// ---------------------------------------------------------------------
// dispatch over p
// ---------------------------------------------------------------------
#define HFMM_DISPATCH_P(p, F)  \
    switch (p) {               \
        case 1: F(1); break;   \
        case 2: F(2); break;   \
        case 3: F(3); break;   \
        case 4: F(4); break;   \
        case 5: F(5); break;   \
        case 6: F(6); break;   \
        case 7: F(7); break;   \
        case 8: F(8); break;   \
        case 9: F(9); break;   \
        case 10: F(10); break; \
        case 11: F(11); break; \
        case 12: F(12); break; \
        case 13: F(13); break; \
        case 14: F(14); break; \
        case 15: F(15); break; \
        case 16: F(16); break; \
        default: throw Status{HFMM_E_UNSUPPORTED}; \
    }

void fill_masses(Tree& t, const double* m, hipStream_t s) {
    hipLaunchKernelGGL(k_fill_masses, dim3(grid_for(t.n, 256)), dim3(256), 0, s, t.n, t.perm,
                       m, t.xs, t.ys, t.zs, t.p32, t.p64, t.status);
    LAUNCH_CHECK();
}

void compute_centres(Tree& t, int method, hipStream_t s) {
    double4* cen = (double4*)t.cen;
    if (method == HFMM_TREECODE) {
        double4* w4 = t.arena.down<double4>(t.ncells);
        for (int l = t.depth; l >= 0; --l) {
            int c0 = t.level_start[l], c1 = t.level_start[l + 1];
            hipLaunchKernelGGL(k_com_level, dim3(grid_for(c1 - c0, 128)), dim3(128), 0, s,
                               t.cells, c0, c1, t.p64, t.root, w4, cen);
            LAUNCH_CHECK();
        }
    } else {
        hipLaunchKernelGGL(k_centres_geometric, dim3(grid_for(t.ncells, 256)), dim3(256), 0, s,
                           t.cells, t.ncells, t.root, cen);
        LAUNCH_CHECK();
    }
}

void run_p2m(Tree& t, int p, bool fp64, hipStream_t s) {
    const int threads = t.nleaves * 8;
#define P2M_CASE(NP)                                                                       \
    if (fp64)                                                                              \
        hipLaunchKernelGGL((k_p2m<double, NP>), dim3(grid_for(threads, 256)), dim3(256), 0, \
                           s, t.cells, t.leaves, t.nleaves, (const double4*)t.cen, t.p64,   \
                           t.M, t.ldm);                                                     \
    else                                                                                    \
        hipLaunchKernelGGL((k_p2m<float, NP>), dim3(grid_for(threads, 256)), dim3(256), 0,  \
                           s, t.cells, t.leaves, t.nleaves, (const double4*)t.cen, t.p64,   \
                           t.M, t.ldm);
    HFMM_DISPATCH_P(p, P2M_CASE);
#undef P2M_CASE
    LAUNCH_CHECK();
}

void run_shift_octants(int p, double2* tab, hipStream_t s) {
#define SH_CASE(NP) hipLaunchKernelGGL((k_shift_octants<NP>), dim3(1), dim3(64), 0, s, tab);
    HFMM_DISPATCH_P(p, SH_CASE);
#undef SH_CASE
    LAUNCH_CHECK();
}

// M2M with a shift vector per child (centres of mass, treecode)
void run_m2m(Tree& t, int p, hipStream_t s) {
    const int NT = p * (p + 1) / 2;
    double2* tab = t.arena.down<double2>((size_t)t.ncells * NT);
#define SH_CASE(NP)                                                                           \
    hipLaunchKernelGGL((k_shift_children<NP>), dim3(grid_for(t.ncells, 128)), dim3(128), 0, s, \
                       t.cells, t.ncells, (const double4*)t.cen, tab);
    HFMM_DISPATCH_P(p, SH_CASE);
#undef SH_CASE
    LAUNCH_CHECK();
    for (int l = t.depth - 1; l >= 0; --l) {
        int c0 = t.level_start[l], c1 = t.level_start[l + 1];
        int64_t threads = (int64_t)(c1 - c0) * NT;
#define M2M_CASE(NP)                                                                     \
    hipLaunchKernelGGL((k_m2m<NP>), dim3(grid_for(threads, 128)), dim3(128), 0, s, t.cells, \
                       c0, c1, tab, 1, t.M, t.ldm);
        HFMM_DISPATCH_P(p, M2M_CASE);
#undef M2M_CASE
        LAUNCH_CHECK();
    }
}

void run_m2l_ops(Tree& t, int p, int layout, void* T, int RB, int KQ, hipStream_t s) {
    // several blocks per class for the larger tables (each recomputes the
    // class's small Legendre table)
    const int split = p >= 6 ? 4 : 1;
    hipLaunchKernelGGL(k_m2l_ops, dim3(343, split), dim3(256), 0, s, p, layout, T, RB, KQ);
    LAUNCH_CHECK();
}

void run_pack(const double* M, int ldm, int ncells, int P, int ld, void* out, bool fp64,
              hipStream_t s) {
    const int64_t tot = (int64_t)(ncells + 1) * ld;
    if (fp64)
        hipLaunchKernelGGL((k_pack<double>), dim3(grid_for(tot, 256)), dim3(256), 0, s, M, ldm,
                           ncells, P, ld, (double*)out);
    else
        hipLaunchKernelGGL((k_pack<float>), dim3(grid_for(tot, 256)), dim3(256), 0, s, M, ldm,
                           ncells, P, ld, (float*)out);
    LAUNCH_CHECK();
}

void run_p2l(Tree& t, int p, bool fp64, double* LX, hipStream_t s) {
    if (t.n_x == 0 || t.n_xcells == 0) return;
#define P2L_CASE(NP)                                                                         \
    if (fp64)                                                                                \
        hipLaunchKernelGGL((k_p2l<double, NP>), dim3(t.n_xcells), dim3(64), 0, s, t.cells,   \
                           t.x_cells, t.x_off, t.x_items, (const double4*)t.cen, t.p64, LX,  \
                           t.ldm);                                                           \
    else                                                                                     \
        hipLaunchKernelGGL((k_p2l<float, NP>), dim3(t.n_xcells), dim3(64), 0, s, t.cells,    \
                           t.x_cells, t.x_off, t.x_items, (const double4*)t.cen, t.p64, LX,  \
                           t.ldm);
    HFMM_DISPATCH_P(p, P2L_CASE);
#undef P2L_CASE
    LAUNCH_CHECK();
}

// FP32 copy of the multipoles (same layout) for the FP32 M2P
static const float* m_as_float(Tree& t, hipStream_t s) {
    const int64_t nel = (int64_t)t.ncells * t.ldm;
    float* m = t.arena.down<float>(nel);
    hipLaunchKernelGGL(k_to_float, dim3(grid_for(nel, 256)), dim3(256), 0, s, t.M, nel, m);
    LAUNCH_CHECK();
    return m;
}

// FMM far field: M2P over the boxes' far lists (the W lists; V too for
// boxes without sources), one wave per target box, then L2P added at every
// target
void run_far(Tree& t, const Targets& tg, int p, bool fp64, const int32_t* off,
             const int32_t* items, int64_t nitems, void* far, hipStream_t s) {
    if (tg.n == 0) return;
    const bool w = nitems > 0;
    const float* M32 = (!fp64 && w) ? m_as_float(t, s) : nullptr;
    const dim3 grid(grid_for(tg.nbox, 4)), block(256), pgrid(grid_for(tg.n, 256));
    const double4* cen = (const double4*)t.cen;
#define FAR_CASE(NP)                                                                          \
    if (fp64) {                                                                               \
        if (w)                                                                                \
            hipLaunchKernelGGL((k_farp<double, NP, double>), grid, block, 0, s, t.root, tg,     \
                               cen, off, items, t.M, (double*)far);                            \
        if (w)                                                                                \
            hipLaunchKernelGGL((k_l2p<double, NP, true>), pgrid, block, 0, s, tg, cen, t.L,     \
                               t.ldm, (double*)far);                                           \
        else                                                                                  \
            hipLaunchKernelGGL((k_l2p<double, NP, false>), pgrid, block, 0, s, tg, cen, t.L,    \
                               t.ldm, (double*)far);                                           \
    } else {                                                                                  \
        if (w)                                                                                \
            hipLaunchKernelGGL((k_farp<float, NP, float>), grid, block, 0, s, t.root, tg, cen,  \
                               off, items, M32, (float*)far);                                  \
        if (w)                                                                                \
            hipLaunchKernelGGL((k_l2p<float, NP, true>), pgrid, block, 0, s, tg, cen, t.L,      \
                               t.ldm, (float*)far);                                            \
        else                                                                                  \
            hipLaunchKernelGGL((k_l2p<float, NP, false>), pgrid, block, 0, s, tg, cen, t.L,     \
                               t.ldm, (float*)far);                                            \
    }
    HFMM_DISPATCH_P(p, FAR_CASE);
#undef FAR_CASE
    LAUNCH_CHECK();
}

// Treecode far field over the boxes' M2P lists off/items; walk: over the FMM
// lists at p = 3 the lists hold only the boxes' own part and the V lists of
// the cells above are read directly
void run_treecode_far(Tree& t, const Targets& tg, int p, bool fp64, bool walk,
                      const int32_t* off, const int32_t* items, void* far, hipStream_t s) {
    if (tg.n == 0) return;
    const double4* cen = (const double4*)t.cen;
    if (p == 3) {  // quadrupole moments: the Cartesian form
        const int64_t nel = (int64_t)t.ncells * 12;
        const dim3 grid(grid_for(tg.nbox, 4)), block(256);
#define FAR3(TT, W)                                                                            \
    hipLaunchKernelGGL((k_treecode_far3<TT, W>), grid, block, 0, s, t.cells, t.root, tg, cen,   \
                       off, items, t.vsrc, c, (TT*)far)
        if (fp64) {
            double* c = t.arena.down<double>(nel);
            hipLaunchKernelGGL(k_cart3<double>, dim3(grid_for(t.ncells, 256)), dim3(256), 0, s,
                               t.M, t.ldm, t.ncells, c);
            LAUNCH_CHECK();
            if (walk)
                FAR3(double, true);
            else
                FAR3(double, false);
        } else {
            float* c = t.arena.down<float>(nel);
            hipLaunchKernelGGL(k_cart3<float>, dim3(grid_for(t.ncells, 256)), dim3(256), 0, s,
                               t.M, t.ldm, t.ncells, c);
            LAUNCH_CHECK();
            if (walk)
                FAR3(float, true);
            else
                FAR3(float, false);
        }
#undef FAR3
        LAUNCH_CHECK();
        return;
    }
    if (walk) throw Status{HFMM_E_STATE};  // other orders take full lists
    // other orders: the spherical form, one thread per target
    const float* M32 = fp64 ? nullptr : m_as_float(t, s);
#define TF_CASE(NP)                                                                            \
    if (fp64)                                                                                  \
        hipLaunchKernelGGL((k_treecode_far<double, NP, double>), dim3(grid_for(tg.n, 256)),     \
                           dim3(256), 0, s, tg, cen, off, items, t.M, t.ldm, (double*)far);    \
    else                                                                                       \
        hipLaunchKernelGGL((k_treecode_far<float, NP, float>), dim3(grid_for(tg.n, 256)),       \
                           dim3(256), 0, s, tg, cen, off, items, M32, t.ldm, (float*)far);
    HFMM_DISPATCH_P(p, TF_CASE);
#undef TF_CASE
    LAUNCH_CHECK();
}

void run_export(const double* X, int ld, int ncells, int p, const double* cen, int which,
                double* out, hipStream_t s) {
    const int64_t tot = (int64_t)ncells * p * (p + 1) / 2;
    hipLaunchKernelGGL(k_export, dim3(grid_for(tot, 256)), dim3(256), 0, s, X, ld, ncells, p,
                       (const double4*)cen, which, out);
    LAUNCH_CHECK();
}

}  // namespace hfmm
