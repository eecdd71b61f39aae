// M2M and L2L of the FMM (Sec. 2) as FP64 matrix-core products.
//
// With geometric centres, a child sits at u = (ox - 1/2, oy - 1/2, oz - 1/2)
// child sides from its parent, so in the level-scaled device basis both
// translations are one of 8 fixed real p^2 x p^2 operators:
//   M2M  Mt_p[n,m]  = 2^-n      sum_{k,l} conj(R_k^l(u)) Mt_c[n-k, m-l]
//   L2L  Lt_c[j,i]  = sum_{n,m} 2^-(n+1) Lt_p[n,m] R_{n-j}^{m-i}(u)
// (R addition theorem).  The operators are built once per order from R(u)
// and applied with v_mfma_f64_16x16x4f64: one wave takes 16 targets
// (columns), rows are output coefficients in blocks of 16, the contraction
// runs over input coefficients k = 16 q + 4 g + r as in the M2L kernel.
// M2M: targets = parents, one product per child octant; L2L: targets =
// children, one product with the operator of the child's octant, plus the
// M2L partial sums and the X-list P2L in the epilogue.
#include "common.hpp"
#include "expansions.hpp"

namespace hfmm {

typedef double doublex4 __attribute__((ext_vector_type(4)));

// R_k^l from the stored m >= 0 triangle: R_k^{-l} = (-1)^l conj(R_k^l);
// zero when |l| > k
__device__ inline double2 rget(const double2* R, int k, int l) {
    const int a = l < 0 ? -l : l;
    if (k < 0 || a > k) return make_double2(0.0, 0.0);
    double2 v = R[tri(k, a)];
    if (l >= 0) return v;
    const double s = (a & 1) ? -1.0 : 1.0;
    return make_double2(s * v.x, -s * v.y);
}

__device__ inline void rdecode2(int r, int& n, int& m, int& part) {
    n = 0;
    while ((n + 1) * (n + 1) <= r) ++n;
    const int o = r - n * n;
    if (o == 0) {
        m = 0;
        part = 0;
    } else {
        m = (o + 1) / 2;
        part = (o + 1) % 2;
    }
}

// real entry of the map X -> c+ X + c- conj(X) for (output part, input part)
__device__ inline double real_entry(double2 cp, double2 cm, int m_in, int po, int pi) {
    if (m_in == 0) return pi == 0 ? (po == 0 ? cp.x : cp.y) : 0.0;
    if (po == 0) return pi == 0 ? cp.x + cm.x : -(cp.y - cm.y);
    return pi == 0 ? cp.y + cm.y : cp.x - cm.x;
}

// one thread per (octant, padded output row, padded input column)
__global__ void k_xlat_ops(int p, int RB, int KQ, const double2* __restrict__ tab,
                           double* __restrict__ m2m, double* __restrict__ l2l) {
    const int P = p * p, NT = p * (p + 1) / 2;
    const int R = 16 * RB, K = 16 * KQ;
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (gid >= (int64_t)8 * R * K) return;
    const int o = (int)(gid / ((int64_t)R * K));
    const int rem = (int)(gid % ((int64_t)R * K));
    const int ro = rem / K, ri = rem % K;
    double vm = 0.0, vl = 0.0;
    if (ro < P && ri < P) {
        const double2* Rt = tab + o * NT;
        int n, m, po, n2, m2, pi;
        rdecode2(ro, n, m, po);
        rdecode2(ri, n2, m2, pi);
        // M2M: output (n, m), input (n2, m2), k = n - n2
        {
            const int k = n - n2;
            const double sc = ldexp(1.0, -n);
            double2 a = rget(Rt, k, m - m2);
            double2 cp = make_double2(sc * a.x, -sc * a.y);
            double2 cm = make_double2(0.0, 0.0);
            if (m2 > 0) {
                double2 b = rget(Rt, k, m + m2);
                const double sg = (m2 & 1) ? -sc : sc;
                cm = make_double2(sg * b.x, -sg * b.y);
            }
            vm = real_entry(cp, cm, m2, po, pi);
        }
        // L2L: output (j = n, i = m), input (n2, m2), k = n2 - j
        {
            const int k = n2 - n;
            const double sc = ldexp(1.0, -(n2 + 1));
            double2 a = rget(Rt, k, m2 - m);
            double2 cp = make_double2(sc * a.x, sc * a.y);
            double2 cm = make_double2(0.0, 0.0);
            if (m2 > 0) {
                double2 b = rget(Rt, k, -m2 - m);
                const double sg = (m2 & 1) ? -sc : sc;
                cm = make_double2(sg * b.x, sg * b.y);
            }
            vl = real_entry(cp, cm, m2, po, pi);
        }
    }
    const int rb = ro / 16, il = ro % 16, q = ri / 16, g = (ri % 16) / 4, r = ri % 4;
    const int64_t idx = ((((int64_t)o * RB + rb) * KQ + q) * 64 + (g * 16 + il)) * 4 + r;
    m2m[idx] = vm;
    l2l[idx] = vl;
}

__device__ inline int degree_of_row(int r) {
    int n = 0;
    while ((n + 1) * (n + 1) <= r) ++n;
    return n;
}

__device__ inline int child_by_octant(const Cell& c, int o) {
    if (!((c.mask >> o) & 1)) return -1;
    return c.child + __popc((unsigned)c.mask & ((1u << o) - 1u));
}

__device__ inline int octant_of_cell(const Cell& c) {
    return ((c.ix & 1) << 2) | ((c.iy & 1) << 1) | (c.iz & 1);
}

__host__ __device__ constexpr int isqrt_c(int r) {
    int n = 0;
    while ((n + 1) * (n + 1) <= r) ++n;
    return n;
}

// Block (rb, q) of an operator is structurally zero when no output degree of
// rows 16 rb .. 16 rb + 15 can draw on an input degree of columns
// 16 q .. 16 q + 15: M2M maps degree n2 into degrees n >= n2, L2L degree n2
// into degrees j <= n2.
template <int MODE>
__host__ __device__ constexpr bool block_live(int rb, int q) {
    return MODE == 0 ? isqrt_c(16 * q) <= isqrt_c(16 * rb + 15)
                     : isqrt_c(16 * q + 15) >= isqrt_c(16 * rb);
}

// acc[rb] += A(cls) * B over the live blocks; independent accumulators are
// interleaved so that consecutive matrix-core instructions do not depend on
// each other.
template <int RB, int KQ, int MODE>
__device__ __forceinline__ void xlat_accumulate(doublex4 (&acc)[RB], const double4* A,
                                                const double* B, int lane) {
#pragma unroll
    for (int q = 0; q < KQ; ++q) {
        const double4 b = *(const double4*)(B + 16 * q);
        double4 a[RB];
#pragma unroll
        for (int rb = 0; rb < RB; ++rb)
            if (block_live<MODE>(rb, q)) a[rb] = A[(rb * KQ + q) * 64 + lane];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const double bv = r == 0 ? b.x : r == 1 ? b.y : r == 2 ? b.z : b.w;
#pragma unroll
            for (int rb = 0; rb < RB; ++rb) {
                if (!block_live<MODE>(rb, q)) continue;
                const double av = r == 0 ? a[rb].x : r == 1 ? a[rb].y : r == 2 ? a[rb].z : a[rb].w;
                acc[rb] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc[rb], 0, 0, 0);
            }
        }
    }
}

// M2M: a block of 8 waves takes 16 parents of one level; wave w applies the
// operator of child octant w, the 8 results are summed in LDS in a fixed
// order and written as whole rows.  Leaves keep their P2M expansion.
template <int RB, int KQ>
__global__ void __launch_bounds__(512)
k_m2m_f64(const Cell* __restrict__ cells, int c0, int ntargets,
          const double* __restrict__ Tsw, double* __restrict__ M, int ld, int zero_row) {
    constexpr int NTE = RB * KQ * 64;
    constexpr int LDR = 16 * RB + 1;  // padded LDS row
    __shared__ double red[16 * LDR];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int g = lane >> 4, col = lane & 15;
    const int ti = blockIdx.x * 16 + col;
    const int tgt = ti < ntargets ? c0 + ti : -1;
    int src = -1;
    if (tgt >= 0) src = child_by_octant(cells[tgt], wave);
    doublex4 acc[RB];
#pragma unroll
    for (int rb = 0; rb < RB; ++rb) acc[rb] = doublex4{0.0, 0.0, 0.0, 0.0};
    if (__ballot(src >= 0))
        xlat_accumulate<RB, KQ, 0>(acc, (const double4*)Tsw + (int64_t)wave * NTE,
                                   M + (int64_t)(src >= 0 ? src : zero_row) * ld + 4 * g, lane);
    for (int w = 0; w < 8; ++w) {
        if (wave == w) {
#pragma unroll
            for (int rb = 0; rb < RB; ++rb)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int row = 16 * rb + 4 * r + g;  // f64 16x16x4 output layout
                    double* d = &red[col * LDR + row];
                    *d = (w == 0 ? 0.0 : *d) + acc[rb][r];
                }
        }
        __syncthreads();
    }
    for (int e = threadIdx.x; e < 16 * 16 * RB; e += blockDim.x) {
        const int c = e / (16 * RB), row = e % (16 * RB);
        const int t = blockIdx.x * 16 + c;
        if (t >= ntargets) continue;
        const int cell = c0 + t;
        if (cells[cell].nchild == 0) continue;
        M[(int64_t)cell * ld + row] = red[c * LDR + row];
    }
}

// M2M for levels with few parents: block (x, rb) takes 16 parents and only
// the output rows 16 rb .. 16 rb + 15, so that a level of a few hundred
// parents still spreads over the GPU (the whole-row kernel above would run
// one long block per 16 parents).  Same products in the same order, so the
// same bits.
template <int RB, int KQ>
__global__ void __launch_bounds__(512)
k_m2m_f64_rows(const Cell* __restrict__ cells, int c0, int ntargets,
               const double* __restrict__ Tsw, double* __restrict__ M, int ld, int zero_row) {
    constexpr int NTE = RB * KQ * 64;
    constexpr int LDR = 17;
    __shared__ double red[16 * LDR];
    const int rb = blockIdx.y;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int g = lane >> 4, col = lane & 15;
    const int ti = blockIdx.x * 16 + col;
    const int tgt = ti < ntargets ? c0 + ti : -1;
    int src = -1;
    if (tgt >= 0) src = child_by_octant(cells[tgt], wave);
    doublex4 acc = doublex4{0.0, 0.0, 0.0, 0.0};
    if (__ballot(src >= 0)) {
        const double4* A = (const double4*)Tsw + (int64_t)wave * NTE;
        const double* B = M + (int64_t)(src >= 0 ? src : zero_row) * ld + 4 * g;
        for (int q = 0; q < KQ; ++q) {
            if (!block_live<0>(rb, q)) continue;
            const double4 b = *(const double4*)(B + 16 * q);
            const double4 a = A[(rb * KQ + q) * 64 + lane];
            acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a.x, b.x, acc, 0, 0, 0);
            acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a.y, b.y, acc, 0, 0, 0);
            acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a.z, b.z, acc, 0, 0, 0);
            acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a.w, b.w, acc, 0, 0, 0);
        }
    }
    for (int w = 0; w < 8; ++w) {
        if (wave == w) {
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                double* d = &red[col * LDR + 4 * r + g];  // f64 16x16x4 output layout
                *d = (w == 0 ? 0.0 : *d) + acc[r];
            }
        }
        __syncthreads();
    }
    if (threadIdx.x < 256) {
        const int c = threadIdx.x >> 4, row = threadIdx.x & 15;
        const int t = blockIdx.x * 16 + c;
        if (t < ntargets) {
            const int cell = c0 + t;
            if (cells[cell].nchild != 0) M[(int64_t)cell * ld + 16 * rb + row] = red[c * LDR + row];
        }
    }
}

// L2L: a block of 4 waves takes 64 children (16 per wave, listed grouped by
// octant); out = L2L(parent) + sum of the M2L partial results (+ P2L),
// combined through LDS so that the partials are read along whole rows.
// Low-precision M2L partials are rescaled by 2^(b_j + e_level + 1).
template <int RB, int KQ, typename TB>
__global__ void __launch_bounds__(256)
k_l2l_f64(const Cell* __restrict__ cells, const int32_t* __restrict__ targets, int ntargets,
          int with_parent, const double* __restrict__ Tsw, double* __restrict__ L, int ld,
          int zero_row, const TB* __restrict__ parts, int nparts, int64_t part_stride,
          const double* __restrict__ lx, int P, const int32_t* __restrict__ bexp,
          const int32_t* __restrict__ levexp, int level) {
    constexpr int NTE = RB * KQ * 64;
    constexpr int LDR = 16 * RB + 1;
    __shared__ double red[64 * LDR];
    __shared__ int scell[64];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int g = lane >> 4, col = lane & 15;
    const int ti = blockIdx.x * 64 + wave * 16 + col;
    const int tgt = ti < ntargets ? targets[ti] : -1;
    int src = -1, cls = 0;
    if (tgt >= 0 && with_parent) {
        const Cell tc = cells[tgt];
        cls = octant_of_cell(tc);
        src = tc.parent;
    }
    doublex4 acc[RB];
#pragma unroll
    for (int rb = 0; rb < RB; ++rb) acc[rb] = doublex4{0.0, 0.0, 0.0, 0.0};
    uint64_t todo = __ballot(src >= 0);
    while (todo) {  // one product per distinct child octant in the wave
        const int leader = __ffsll((unsigned long long)todo) - 1;
        const int c = __shfl(cls, leader, 64);
        const bool mine = src >= 0 && cls == c;
        todo &= ~__ballot(mine);
        doublex4 part[RB];
#pragma unroll
        for (int rb = 0; rb < RB; ++rb) part[rb] = doublex4{0.0, 0.0, 0.0, 0.0};
        xlat_accumulate<RB, KQ, 1>(part, (const double4*)Tsw + (int64_t)c * NTE,
                                   L + (int64_t)(mine ? src : zero_row) * ld + 4 * g, lane);
#pragma unroll
        for (int rb = 0; rb < RB; ++rb)
            if (mine) acc[rb] += part[rb];
    }
    const int lc = wave * 16 + col;
#pragma unroll
    for (int rb = 0; rb < RB; ++rb)
#pragma unroll
        for (int r = 0; r < 4; ++r) red[lc * LDR + 16 * rb + 4 * r + g] = acc[rb][r];
    if (g == 0) scell[lc] = tgt;
    __syncthreads();
    // epilogue: thread -> elements threadIdx.x + 256 k of the 64 x (16 RB)
    // block, in 4 chunks of RB; the partial results are read four parts at
    // a time with every load of a batch in flight (the loads are not
    // predicated: a missing part or element re-reads a valid address)
    const int sc_lev = bexp ? level_exp(levexp, level) + 2 : 0;
#pragma unroll
    for (int ch = 0; ch < 4; ++ch) {
        int64_t off[RB];
        double ps[RB];
#pragma unroll
        for (int k = 0; k < RB; ++k) {
            const int e = (ch * RB + k) * 256 + threadIdx.x;
            const int cell = scell[e / (16 * RB)];
            off[k] = cell >= 0 ? (int64_t)cell * ld + e % (16 * RB) : -1;
            ps[k] = 0.0;
        }
        for (int q0 = 0; q0 < nparts; q0 += 4) {
            TB v[4][RB];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const TB* pp = parts + (int64_t)min(q0 + u, nparts - 1) * part_stride;
#pragma unroll
                for (int k = 0; k < RB; ++k) v[u][k] = pp[off[k] >= 0 ? off[k] : 0];
            }
#pragma unroll
            for (int u = 0; u < 4; ++u)
#pragma unroll
                for (int k = 0; k < RB; ++k)
                    if (q0 + u < nparts) ps[k] += (double)v[u][k];
        }
#pragma unroll
        for (int k = 0; k < RB; ++k) {
            if (off[k] < 0) continue;
            const int e = (ch * RB + k) * 256 + threadIdx.x;
            const int c = e / (16 * RB), row = e % (16 * RB);
            double v = ps[k];
            if (bexp && row < P) v = ldexp(v, bexp[isqrt_c(row)] + sc_lev);
            v += red[c * LDR + row];
            if (lx) v += lx[off[k]];
            L[off[k]] = v;
        }
    }
}

#define HFMM_DISPATCH_RB16(R, F) \
    switch (R) {                 \
        case 1: F(1); break;     \
        case 2: F(2); break;     \
        case 3: F(3); break;     \
        case 4: F(4); break;     \
        case 5: F(5); break;     \
        case 6: F(6); break;     \
        case 7: F(7); break;     \
        case 8: F(8); break;     \
        case 9: F(9); break;     \
        case 10: F(10); break;   \
        case 11: F(11); break;   \
        case 12: F(12); break;   \
        case 13: F(13); break;   \
        case 14: F(14); break;   \
        case 15: F(15); break;   \
        case 16: F(16); break;   \
        default: throw Status{HFMM_E_UNSUPPORTED}; \
    }

void prepare_xlat_ops(Tree& t, int p, hipStream_t s) {
    const int RB = (p * p + 15) / 16;
    const size_t per = (size_t)8 * RB * RB * 64 * 4;
    t.xl_m2m = t.arena.up<double>(per);
    t.xl_l2l = t.arena.up<double>(per);
    double2* tab = t.arena.down<double2>((size_t)8 * p * (p + 1) / 2);
    run_shift_octants(p, tab, s);
    const int64_t threads = (int64_t)8 * 16 * RB * 16 * RB;
    hipLaunchKernelGGL(k_xlat_ops, dim3(grid_for(threads, 256)), dim3(256), 0, s, p, RB, RB,
                       (const double2*)tab, t.xl_m2m, t.xl_l2l);
    LAUNCH_CHECK();
}

void run_m2m_mfma(Tree& t, int p, hipStream_t s) {
    const int RB = (p * p + 15) / 16;
    for (int l = t.depth - 1; l >= 0; --l) {
        const int c0 = t.level_start[l], c1 = t.level_start[l + 1];
        const int nt = c1 - c0;
        // few parents: one block per 16 parents and output row block
        const bool rows = nt < 2048;
        dim3 grid((nt + 15) / 16, rows ? RB : 1), block(512);
#define M2M_CASE(R)                                                                        \
    if (rows)                                                                              \
        hipLaunchKernelGGL((k_m2m_f64_rows<R, R>), grid, block, 0, s, t.cells, c0, nt,     \
                           t.xl_m2m, t.M, t.ldm, t.ncells);                                \
    else                                                                                   \
        hipLaunchKernelGGL((k_m2m_f64<R, R>), grid, block, 0, s, t.cells, c0, nt, t.xl_m2m, \
                           t.M, t.ldm, t.ncells);
        HFMM_DISPATCH_RB16(RB, M2M_CASE);
#undef M2M_CASE
        LAUNCH_CHECK();
    }
}

// L2L for levels with few children: block (x, rb) takes 64 children and only
// the output rows 16 rb .. 16 rb + 15 (the same products and sums, in the
// same order, as the whole-row kernel above).
template <int RB, int KQ, typename TB>
__global__ void __launch_bounds__(256)
k_l2l_f64_rows(const Cell* __restrict__ cells, const int32_t* __restrict__ targets,
               int ntargets, int with_parent, const double* __restrict__ Tsw,
               double* __restrict__ L, int ld, int zero_row, const TB* __restrict__ parts,
               int nparts, int64_t part_stride, const double* __restrict__ lx, int P,
               const int32_t* __restrict__ bexp, const int32_t* __restrict__ levexp,
               int level) {
    constexpr int NTE = RB * KQ * 64;
    constexpr int LDR = 17;
    __shared__ double red[64 * LDR];
    __shared__ int scell[64];
    const int rb = blockIdx.y;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int g = lane >> 4, col = lane & 15;
    const int ti = blockIdx.x * 64 + wave * 16 + col;
    const int tgt = ti < ntargets ? targets[ti] : -1;
    int src = -1, cls = 0;
    if (tgt >= 0 && with_parent) {
        const Cell tc = cells[tgt];
        cls = octant_of_cell(tc);
        src = tc.parent;
    }
    doublex4 acc = doublex4{0.0, 0.0, 0.0, 0.0};
    uint64_t todo = __ballot(src >= 0);
    while (todo) {  // one product per distinct child octant in the wave
        const int leader = __ffsll((unsigned long long)todo) - 1;
        const int c = __shfl(cls, leader, 64);
        const bool mine = src >= 0 && cls == c;
        todo &= ~__ballot(mine);
        doublex4 part = doublex4{0.0, 0.0, 0.0, 0.0};
        const double4* A = (const double4*)Tsw + (int64_t)c * NTE;
        const double* B = L + (int64_t)(mine ? src : zero_row) * ld + 4 * g;
        for (int q = 0; q < KQ; ++q) {
            if (!block_live<1>(rb, q)) continue;
            const double4 b = *(const double4*)(B + 16 * q);
            const double4 a = A[(rb * KQ + q) * 64 + lane];
            part = __builtin_amdgcn_mfma_f64_16x16x4f64(a.x, b.x, part, 0, 0, 0);
            part = __builtin_amdgcn_mfma_f64_16x16x4f64(a.y, b.y, part, 0, 0, 0);
            part = __builtin_amdgcn_mfma_f64_16x16x4f64(a.z, b.z, part, 0, 0, 0);
            part = __builtin_amdgcn_mfma_f64_16x16x4f64(a.w, b.w, part, 0, 0, 0);
        }
        if (mine) acc += part;
    }
    const int lc = wave * 16 + col;
#pragma unroll
    for (int r = 0; r < 4; ++r) red[lc * LDR + 4 * r + g] = acc[r];
    if (g == 0) scell[lc] = tgt;
    __syncthreads();
    // epilogue: thread -> elements threadIdx.x + 256 k of the 64 x 16 block
    const int sc_lev = bexp ? level_exp(levexp, level) + 2 : 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int e = k * 256 + threadIdx.x;
        const int c = e >> 4, row = 16 * rb + (e & 15);
        const int cell = scell[c];
        if (cell < 0) continue;
        const int64_t off = (int64_t)cell * ld + row;
        double ps = 0.0;
        for (int q = 0; q < nparts; ++q) ps += (double)parts[(int64_t)q * part_stride + off];
        double v = ps;
        if (bexp && row < P) v = ldexp(v, bexp[isqrt_c(row)] + sc_lev);
        v += red[c * LDR + (e & 15)];
        if (lx) v += lx[off];
        L[off] = v;
    }
}

void run_l2l_mfma(Tree& t, int p, const void* parts, bool parts_fp64, int nparts,
                  int64_t part_stride, const double* LX, const int32_t* bexp,
                  const int32_t* levexp, hipStream_t s) {
    const int RB = (p * p + 15) / 16;
    for (int l = 2; l <= t.depth; ++l) {
        const int i0 = t.m2l_level_start[l], i1 = t.m2l_level_start[l + 1];
        const int nt = i1 - i0;
        if (nt == 0) continue;
        // few children: one block per 64 children and output row block
        const bool rows = nt < 8192;
        dim3 grid((nt + 63) / 64, rows ? RB : 1), block(256);
        const int wp = l >= 3 ? 1 : 0;
#define L2L_CASE(R)                                                                         \
    if (rows && parts_fp64)                                                                 \
        hipLaunchKernelGGL((k_l2l_f64_rows<R, R, double>), grid, block, 0, s, t.cells,       \
                           t.m2l_order + i0, nt, wp, t.xl_l2l, t.L, t.ldm, t.ncells,         \
                           (const double*)parts, nparts, part_stride, LX, p * p, bexp,      \
                           levexp, l);                                                      \
    else if (rows)                                                                          \
        hipLaunchKernelGGL((k_l2l_f64_rows<R, R, float>), grid, block, 0, s, t.cells,        \
                           t.m2l_order + i0, nt, wp, t.xl_l2l, t.L, t.ldm, t.ncells,         \
                           (const float*)parts, nparts, part_stride, LX, p * p, bexp,       \
                           levexp, l);                                                      \
    else if (parts_fp64)                                                                    \
        hipLaunchKernelGGL((k_l2l_f64<R, R, double>), grid, block, 0, s, t.cells,            \
                           t.m2l_order + i0, nt, wp, t.xl_l2l, t.L, t.ldm, t.ncells,         \
                           (const double*)parts, nparts, part_stride, LX, p * p, bexp,      \
                           levexp, l);                                                      \
    else                                                                                    \
        hipLaunchKernelGGL((k_l2l_f64<R, R, float>), grid, block, 0, s, t.cells,             \
                           t.m2l_order + i0, nt, wp, t.xl_l2l, t.L, t.ldm, t.ncells,         \
                           (const float*)parts, nparts, part_stride, LX, p * p, bexp, levexp,  \
                           l);
        HFMM_DISPATCH_RB16(RB, L2L_CASE);
#undef L2L_CASE
        LAUNCH_CHECK();
    }
}

}  // namespace hfmm
