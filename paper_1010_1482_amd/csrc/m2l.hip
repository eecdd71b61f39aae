// M2L (Eq. 4) as dense products batched by offset class.
//
// In the device basis every V pair at offset class d (316 classes, |d|_inf
// in {2, 3}) applies the same real p^2 x p^2 matrix T_d (built from Eq. 4 in
// expansions.hip), independent of the level.  Targets of one (level, octant)
// see the same 189 classes in the same slots, so a tile of targets of one
// octant runs, slot by slot, C[:, tile] += T_d * M[:, sources(tile, d)] on the
// matrix cores: the paper's thread-per-coefficient loop (Sec. 5.2) becomes a
// GEMM with T_d shared by all targets of the tile.
//
// Matrix-core mapping (v_mfma_f32_16x16x4f32, one 16x16 output block per
// instruction): rows = output coefficients in blocks of 16 (RB blocks, p^2
// padded), columns = 16 targets, contraction over input coefficients in
// steps of 4.  The contraction index k = 16 q + 4 g + r is split so that lane
// group g = lane / 16 loads four consecutive coefficients of its column with
// one 16-byte load; T_d is stored pre-swizzled to match, so both operands
// arrive with 16-byte loads.
#include "common.hpp"
#include "expansions.hpp"

#include <algorithm>
#include <atomic>
#include <cmath>
#include <optional>
#include <type_traits>

namespace hfmm {

typedef float floatx4 __attribute__((ext_vector_type(4)));

// ---------------------------------------------------------------------
// VALU M2L: one 64-lane block per target cell, lanes over output rows
// T64 layout [cls][ri][ro]
// ---------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(64)
k_m2l_valu(const Cell* __restrict__ cells, int c0, int c1, const int32_t* __restrict__ vsrc,
           const double* __restrict__ M, int P, int ld, const T* __restrict__ Tm,
           T* __restrict__ out) {
    extern __shared__ char smem[];
    T* ms = (T*)smem;
    const int c = c0 + blockIdx.x;
    if (c >= c1) return;
    const Cell B = cells[c];
    const int ox = B.ix & 1, oy = B.iy & 1, oz = B.iz & 1;
    T acc[4] = {T(0), T(0), T(0), T(0)};
    const int64_t per = (int64_t)P * P;
    for (int slot = 0; slot < 216; ++slot) {
        const int src = vsrc[(int64_t)c * 216 + slot];
        if (src < 0) continue;
        const int dx = slot / 36 - 2 - ox, dy = (slot / 6) % 6 - 2 - oy, dz = slot % 6 - 2 - oz;
        const int cls = (dx + 3) * 49 + (dy + 3) * 7 + (dz + 3);
        __syncthreads();
        for (int k = threadIdx.x; k < P; k += 64) ms[k] = (T)M[(int64_t)src * ld + k];
        __syncthreads();
        const T* Tc = Tm + cls * per;
        for (int ri = 0; ri < P; ++ri) {
            const T mv = ms[ri];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int ro = threadIdx.x + 64 * u;
                if (ro < P) acc[u] += Tc[(int64_t)ri * P + ro] * mv;
            }
        }
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const int ro = threadIdx.x + 64 * u;
        if (ro < ld) out[(int64_t)c * ld + ro] = ro < P ? acc[u] : T(0);
    }
}



// ---------------------------------------------------------------------
// Low-precision matrix-core M2L (BF16 or FP16 operands, FP32 accumulate),
// with an optional hi/lo split: x3 forms hi*hi + hi*lo + lo*hi.
// v_mfma_f32_16x16x32_{bf16,f16}: each lane holds 8 consecutive contraction
// elements, k = 32 q + 8 g + j, for both operands.
// Range: the scaled operator spans ~2^-2 .. 2^66 and the multipoles decay
// like (sqrt3/2)^n / n!, beyond FP16.  Both are rescaled by powers of two,
//   M'_n = Mt_n 2^{-mu_n} 2^{-e_l},   T'_{jn} = T_{jn} 2^{mu_n - b_j},
// mu_n = floor(log2((sqrt3/2)^n / n!)), b_j from the largest scaled entry of
// output degree j, e_l from the largest monopole of level l, and undone
// exactly (powers of two) in the FP64 L2L epilogue.
// ---------------------------------------------------------------------
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 halfx8 __attribute__((ext_vector_type(8)));

template <typename T16>
struct LowP;
template <>
struct LowP<__bf16> {
    using vec = bf16x8;
    static __device__ __forceinline__ floatx4 mma(vec a, vec b, floatx4 c) {
        return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
    }
};
template <>
struct LowP<_Float16> {
    using vec = halfx8;
    static __device__ __forceinline__ floatx4 mma(vec a, vec b, floatx4 c) {
        return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
    }
};

__device__ inline int mu_exp(int n) {
    double v = 1.0;
    for (int i = 1; i <= n; ++i) v *= 0.8660254037844386 / (double)i;
    return ilogb(v);
}

__device__ inline int degree_of(int r) {
    int n = 0;
    while ((n + 1) * (n + 1) <= r) ++n;
    return n;
}

// Per level: the largest exponent of the scaled coefficients
// Mt_k 2^{-mu_n}, over every cell and every coefficient of the level (not
// only the monopole: with masses of both signs a near-neutral cell has a
// small M_0 and larger higher-degree terms), so that every packed entry is
// below 1 in magnitude.  Block maxima in LDS first: one global atomic per
// block and level.  A level whose coefficients are all zero keeps the
// sentinel, which level_exp() reads as 0.
__global__ void k_level_exp(const Cell* __restrict__ cells, int nc, const double* __restrict__ M,
                            int ldm, int p, int32_t* __restrict__ levexp) {
    __shared__ int bmax[32];
    if (threadIdx.x < 32) bmax[threadIdx.x] = INT_MIN;
    __syncthreads();
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c < nc) {
        const double* row = M + (int64_t)c * ldm;
        int e = INT_MIN;
        for (int n = 0; n < p; ++n) {
            const int mu = mu_exp(n);
            for (int k = n * n; k < (n + 1) * (n + 1); ++k) {
                const double v = fabs(row[k]);
                if (v > 0.0) e = max(e, ilogb(v) - mu);
            }
        }
        if (e != INT_MIN) atomicMax(&bmax[cells[c].level], e);
    }
    __syncthreads();
    if (threadIdx.x < 32 && bmax[threadIdx.x] != INT_MIN)
        atomicMax(&levexp[threadIdx.x], bmax[threadIdx.x]);
}

template <typename T16>
__global__ void k_pack_lp(const Cell* __restrict__ cells, const double* __restrict__ M, int ldm,
                          int ncells, int P, int ld, const int32_t* __restrict__ levexp,
                          T16* __restrict__ hi, T16* __restrict__ lo) {
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (gid >= (int64_t)(ncells + 1) * ld) return;
    const int c = (int)(gid / ld), k = (int)(gid % ld);
    double v = 0.0;
    if (c < ncells && k < P) {
        const int e = level_exp(levexp, cells[c].level);
        v = ldexp(M[(int64_t)c * ldm + k], -mu_exp(degree_of(k)) - (e + 1));
    }
    const T16 h = (T16)(float)v;
    hi[gid] = h;
    if (lo) lo[gid] = (T16)(float)(v - (double)(float)h);
}

// ---------------------------------------------------------------------
// Matrix-core M2L.  Block = 8 waves, tile = up to 256 targets of one
// octant (levels mixed), 32 per wave (two column blocks of 16).  The work
// items are the (tile, slot) pairs in which some target of the tile has a
// source, tile by tile (a tile without any counts as one item, which writes
// zeros); tpre[t] is the number of items before tile t.  Block b takes items
// [b W / NB, (b + 1) W / NB) of the W items, so every block has the same
// share of the products.  The consecutive items of one tile in one block
// are a segment; segment k of a tile (k-th block that touches it) writes
// partial result k, and the tile's last segment writes zeros to the partial
// results after its own; the downward pass sums them (deterministic, no
// atomics).
//
// Both operands travel in 16-byte chunks: chunk 4 q + g of a row holds the
// contraction elements that lane group g feeds to step q.  For FP32 a chunk
// is 4 floats (four 16x16x4 products), for BF16/FP16 8 halves (one 16x16x32
// product).  Per slot the operator T_d sits in LDS: FP32, FP64 and the split
// forms stage the next slot's operator through registers; the single-product
// forms and the largest orders copy it with direct global-to-LDS loads.  The
// source chunks of the next contraction steps are in flight while a step
// runs on the matrix cores.
// ---------------------------------------------------------------------
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

struct OpF32 {
    using E = float;
    using O = float;  // partial results
    using Acc = floatx4;
    static constexpr bool X3 = false;
    static constexpr int S = 4;  // products per (q, rb, cb)
    static __device__ __forceinline__ Acc zero() { return floatx4{0.f, 0.f, 0.f, 0.f}; }
    // output block rb of one target row: rows 16 rb + 4 g + (0..3)
    static __device__ __forceinline__ void store(O* o, int rb, int g, Acc c) {
        *(float4*)(o + 16 * rb + 4 * g) = make_float4(c[0], c[1], c[2], c[3]);
    }
    template <int s>
    static __device__ __forceinline__ floatx4 mma(u32x4 ah, u32x4, u32x4 bh, u32x4,
                                                  floatx4 c) {
        // whole-vector casts: a bit_cast of one vector element loses its
        // index with this compiler (every s would read element 0)
        return __builtin_amdgcn_mfma_f32_16x16x4f32(__builtin_bit_cast(floatx4, ah)[s],
                                                    __builtin_bit_cast(floatx4, bh)[s], c, 0, 0,
                                                    0);
    }
};

template <typename T16, bool SPLIT>
struct OpLow {
    using E = T16;
    using O = float;
    using Acc = floatx4;
    static constexpr bool X3 = SPLIT;
    static constexpr int S = SPLIT ? 3 : 1;  // hi*hi (+ hi*lo + lo*hi)
    static __device__ __forceinline__ Acc zero() { return floatx4{0.f, 0.f, 0.f, 0.f}; }
    static __device__ __forceinline__ void store(O* o, int rb, int g, Acc c) {
        *(float4*)(o + 16 * rb + 4 * g) = make_float4(c[0], c[1], c[2], c[3]);
    }
    template <int s>
    static __device__ __forceinline__ floatx4 mma(u32x4 ah, u32x4 al, u32x4 bh, u32x4 bl,
                                                  floatx4 c) {
        using V = typename LowP<T16>::vec;
        const u32x4 a = s == 2 ? al : ah;
        const u32x4 b = s == 1 ? bl : bh;
        return LowP<T16>::mma(__builtin_bit_cast(V, a), __builtin_bit_cast(V, b), c);
    }
};

// column blocks of 16 targets per wave (8 waves per 256-target tile)
constexpr int kM2LCB = 2;
// contraction steps whose source chunks are loaded ahead of use (with
// register-staged operators: across slot boundaries, 3 for the split forms'
// shorter steps; measured on the device)
constexpr int kM2LAhead = 2;
constexpr int m2l_ahead_staged(bool x3) { return x3 ? 3 : 2; }
// Two operator buffers (the next slot's operator streams in during the
// products, one barrier per slot), used when both copies fit in 144 KiB of
// LDS.
constexpr bool m2l_double_buffer(int rb, int kq, int ns) {
    return 2 * ns * rb * kq * 64 * 16 <= 144 * 1024;
}
// Registers (per lane) of a register-staged operator pipeline: the wave's
// share of the next operator, the accumulators and the source chunks in
// flight.  With one LDS buffer the staging is used when this stays within
// 160 of the 256 a wave has at two waves per SIMD (beyond, the compiler
// spills); otherwise the operator is copied straight to LDS.
constexpr int m2l_staged_regs(int rb, int npw, int ns, int cb, int acc_regs, int ahead) {
    return 4 * npw * ns + cb * rb * acc_regs + 4 * (ahead + 1) * cb * ns;
}
// FP64: a 16-byte chunk holds 2 doubles (two 16x16x4 FP64 products); the
// output rows of a block are 16 rb + 4 r + g (the FP64 product's layout)
typedef double doublex2 __attribute__((ext_vector_type(2)));
typedef double doublex4 __attribute__((ext_vector_type(4)));
struct OpF64 {
    using E = double;
    using O = double;
    using Acc = doublex4;
    static constexpr bool X3 = false;
    static constexpr int S = 2;
    static __device__ __forceinline__ Acc zero() { return doublex4{0.0, 0.0, 0.0, 0.0}; }
    template <int s>
    static __device__ __forceinline__ Acc mma(u32x4 ah, u32x4, u32x4 bh, u32x4, Acc c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(__builtin_bit_cast(doublex2, ah)[s],
                                                    __builtin_bit_cast(doublex2, bh)[s], c, 0,
                                                    0, 0);
    }
    static __device__ __forceinline__ void store(O* o, int rb, int g, Acc c) {
#pragma unroll
        for (int r = 0; r < 4; ++r) o[16 * rb + 4 * r + g] = c[r];
    }
};

// bits of m whose rank among the set bits, counted from `base`, lies in
// [lo, hi)
__device__ inline uint32_t m2l_rank_range(uint32_t m, int base, int lo, int hi) {
    for (int k = base; m && k < lo; ++k) m &= m - 1u;  // drop ranks below lo
    uint32_t keep = 0u;
    for (int k = max(base, lo); m && k < hi; ++k) {
        const uint32_t low = m & (0u - m);
        keep |= low;
        m ^= low;
    }
    return keep;
}

// This block's range of work items and the tile of its first item (the
// items and blocks are described at k_m2l_mma).  Workgroups are handed to
// the 8 XCDs round-robin; they are renumbered so that each XCD (own L2)
// runs one contiguous range of blocks, i.e. of items: the blocks resident
// on an XCD then share tiles and source expansions.
struct M2lItems {
    int b, item, iend, tile;
    int64_t W;
};
__device__ inline M2lItems m2l_items(const int32_t* __restrict__ tpre, int ntiles) {
    M2lItems it;
    const int nb = gridDim.x, lin = blockIdx.x;
    const int xcd = lin & 7, q8 = nb >> 3, r8 = nb & 7;
    it.b = xcd * q8 + min(xcd, r8) + (lin >> 3);
    it.W = tpre[ntiles];
    it.item = (int)((int64_t)it.b * it.W / nb);
    it.iend = (int)((int64_t)(it.b + 1) * it.W / nb);
    // the last tile with tpre[tile] <= item: a 64-way search, every lane
    // probing one point of [lo, hi) per round (tpre[lo] <= item < tpre[hi])
    const int lane = threadIdx.x & 63;
    int lo = 0, hi = ntiles;
    while (hi - lo > 1) {
        const int step = (hi - lo + 63) / 64;
        const int idx = lo + lane * step;
        const bool le = idx < hi && tpre[idx] <= it.item;
        const int k = __popcll(__ballot(le));  // lanes 0 .. k-1 (lane 0 always)
        hi = min(hi, lo + k * step);
        lo = lo + (k - 1) * step;
    }
    it.tile = lo;
    return it;
}

// The segment of tile it.tile that starts at it.item: its partial-result
// number (blocks before this one that hold items of the tile), whether it
// is the tile's last, and its slots (the tile's slots with a source whose
// ranks fall in the segment) as a mask, the same in every lane.  Moves
// it.item to the segment's end.
__device__ inline void m2l_segment(const uint32_t* __restrict__ tmask,
                                   const int32_t* __restrict__ tpre, M2lItems& it, int& part,
                                   bool& last, uint32_t (&mw)[7]) {
    const int nb = gridDim.x;
    const int p0 = tpre[it.tile], p1 = tpre[it.tile + 1];
    const int seg_end = min(it.iend, p1);
    part = it.b - (int)((((int64_t)p0 + 1) * nb - 1) / it.W);
    last = seg_end == p1;
    int base = 0;
#pragma unroll
    for (int w = 0; w < 7; ++w) {
        const uint32_t m = tmask[8 * it.tile + w];
        mw[w] = __builtin_amdgcn_readfirstlane(
            m2l_rank_range(m, base, it.item - p0, seg_end - p0));
        base += __popc(m);
    }
    it.item = seg_end;
}

// first slot >= j of the mask, else 216
__device__ inline int m2l_next_slot(const uint32_t (&mw)[7], int j) {
#pragma unroll
    for (int w = 0; w < 7; ++w) {
        if (j < 32 * w + 32) {
            const uint32_t bb = j > 32 * w ? mw[w] & (~0u << (j - 32 * w)) : mw[w];
            if (bb) return 32 * w + __builtin_ctz(bb);
        }
    }
    return 216;
}

typedef __attribute__((address_space(3))) void* lds_ptr;
typedef const __attribute__((address_space(1))) void* gbl_ptr;

// LASTS: products of the last contraction step that carry data (FP32:
// ceil((p^2 - 16 (KQ - 1)) / 4), the rest are padding and skipped).
// LASTR: rows of the last output block that carry data (p^2 - 16 (RB - 1)).
template <int RB, int KQ, int CB, bool DB, class Op, int LASTS = Op::S, int LASTR = 16>
__global__ void __launch_bounds__(1024 / CB)
k_m2l_mma(const int32_t* __restrict__ tiles, const uint32_t* __restrict__ tmask,
          const int32_t* __restrict__ tpre, int ntiles, int nparts,
          const int32_t* __restrict__ order, const int32_t* __restrict__ vsrc,
          const typename Op::E* __restrict__ Mhi, const typename Op::E* __restrict__ Mlo,
          int ncells, const typename Op::E* __restrict__ Thi,
          const typename Op::E* __restrict__ Tlo, typename Op::O* __restrict__ out,
          int64_t part_stride, int zero_fill) {
    constexpr int NT = RB * KQ * 64;  // 16-byte chunks of one operator
    constexpr int CPR = 4 * KQ;       // 16-byte chunks per operand row
    constexpr int LDO = 16 * RB;      // output row length (floats)
    constexpr int NS = Op::X3 ? 2 : 1;
    constexpr int NW = 16 / CB;       // waves per block (CB column blocks each)
    __shared__ u32x4 sT[NS * NT];
    __shared__ u32x4 sT2[DB ? NS * NT : 1];
    M2lItems it = m2l_items(tpre, ntiles);
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int g = lane >> 4, col = lane & 15;
    constexpr int s0 = 0, ns = 216;
    for (; it.item < it.iend; ++it.tile) {
        const int tile = it.tile;
        int part;
        bool last_seg;
        uint32_t mw[7];
        m2l_segment(tmask, tpre, it, part, last_seg, mw);
        const int start = tiles[4 * tile], count = tiles[4 * tile + 1], oct = tiles[4 * tile + 2];
        const int ox = (oct >> 2) & 1, oy = (oct >> 1) & 1, oz = oct & 1;
        auto next_slot = [&](int j) -> int { return m2l_next_slot(mw, j); };
        // the previous segment's products are done before its buffers are
        // written again
        __syncthreads();

        int tgt[CB];
#pragma unroll
        for (int cb = 0; cb < CB; ++cb) {
            const int i = (wave * CB + cb) * 16 + col;
            tgt[cb] = i < count ? order[start + i] : -1;
        }
        // waves past the tile's last target skip the products (small tiles:
        // edges and corners of the box, the last tile of a group)
        const bool busy = wave * CB * 16 < count;
        typename Op::Acc acc[CB][RB];
#pragma unroll
        for (int cb = 0; cb < CB; ++cb)
#pragma unroll
            for (int rb = 0; rb < RB; ++rb) acc[cb][rb] = Op::zero();

        const u32x4* Mh = (const u32x4*)Mhi;
        const u32x4* Ml = (const u32x4*)Mlo;
        // operator of relative slot jj -> LDS buffer (each wave copies every
        // NW-th 1-KiB chunk with direct global-to-LDS loads)
        auto stage = [&](u32x4* buf, int jj) {
            const int slot = s0 + jj;
            const int dx = slot / 36 - 2 - ox, dy = (slot / 6) % 6 - 2 - oy, dz = slot % 6 - 2 - oz;
            const int cls = (dx + 3) * 49 + (dy + 3) * 7 + (dz + 3);
            const u32x4* th = (const u32x4*)Thi + (int64_t)cls * NT;
            for (int k = wave; k < RB * KQ; k += NW)
                __builtin_amdgcn_global_load_lds((gbl_ptr)(th + k * 64 + lane),
                                                 (lds_ptr)(buf + k * 64), 16, 0, 0);
            if (Op::X3) {
                const u32x4* tl = (const u32x4*)Tlo + (int64_t)cls * NT;
                for (int k = wave; k < RB * KQ; k += NW)
                    __builtin_amdgcn_global_load_lds((gbl_ptr)(tl + k * 64 + lane),
                                                     (lds_ptr)(buf + NT + k * 64), 16, 0, 0);
            }
        };
        auto load_src = [&](int jj, int (&sv)[CB]) {
#pragma unroll
            for (int cb = 0; cb < CB; ++cb)
                sv[cb] = (jj < ns && tgt[cb] >= 0) ? vsrc[(int64_t)tgt[cb] * 216 + s0 + jj] : -1;
        };
        // the same, issued unconditionally (a valid row stands in), so that every
        // call issues CB loads
        auto load_src_u = [&](int jj, int (&sv)[CB]) {
#pragma unroll
            for (int cb = 0; cb < CB; ++cb) {
                const bool ok = jj < ns && tgt[cb] >= 0;
                const int v = vsrc[(int64_t)(tgt[cb] >= 0 ? tgt[cb] : 0) * 216 + s0 +
                                   (jj < ns ? jj : 0)];
                sv[cb] = ok ? v : -1;
            }
        };
        auto set_boff = [&](const int (&sv)[CB], int64_t (&boff)[CB]) {
#pragma unroll
            for (int cb = 0; cb < CB; ++cb)
                boff[cb] = (int64_t)(sv[cb] >= 0 ? sv[cb] : ncells) * CPR + g;
        };
        // source chunks of step q live in bh[q]; kM2LAhead steps are in flight
        // ahead of the matrix cores (registers are only allocated for the live
        // ones, every index being a constant after unrolling)
        auto first_chunks = [&](const int (&sv)[CB], int64_t (&boff)[CB], u32x4 (&bh)[KQ][CB],
                                u32x4 (&bl)[KQ][CB]) {
            set_boff(sv, boff);
#pragma unroll
            for (int q = 0; q < KQ && q < kM2LAhead; ++q)
#pragma unroll
                for (int cb = 0; cb < CB; ++cb) {
                    bh[q][cb] = Mh[boff[cb] + 4 * q];
                    if (Op::X3) bl[q][cb] = Ml[boff[cb] + 4 * q];
                }
        };
        // The single-product forms (BF16/FP16 x1) and FP32 with one operator
        // buffer read the A chunks of step q + 1 from LDS while step q runs (kept
        // there by a scheduling barrier); the other forms load A where it is
        // used, which schedules better for them (measured on the device).
        constexpr bool kPinA = Op::S == 1 || (Op::S == 4 && !DB);
        auto products = [&](const u32x4* buf, const int64_t (&boff)[CB], u32x4 (&bh)[KQ][CB],
                            u32x4 (&bl)[KQ][CB]) {
            u32x4 ah[2][RB], al[2][RB];
            if (kPinA) {
#pragma unroll
                for (int rb = 0; rb < RB; ++rb) {
                    ah[0][rb] = buf[rb * KQ * 64 + lane];
                    al[0][rb] = Op::X3 ? buf[NT + rb * KQ * 64 + lane] : ah[0][rb];
                }
            }
#pragma unroll
            for (int q = 0; q < KQ; ++q) {
                const int cur = q & 1, nxt = cur ^ 1;
                if (q + kM2LAhead < KQ) {
#pragma unroll
                    for (int cb = 0; cb < CB; ++cb) {
                        bh[q + kM2LAhead][cb] = Mh[boff[cb] + 4 * (q + kM2LAhead)];
                        if (Op::X3) bl[q + kM2LAhead][cb] = Ml[boff[cb] + 4 * (q + kM2LAhead)];
                    }
                }
                if (kPinA) {
                    if (q + 1 < KQ) {
#pragma unroll
                        for (int rb = 0; rb < RB; ++rb) {
                            ah[nxt][rb] = buf[(rb * KQ + q + 1) * 64 + lane];
                            al[nxt][rb] =
                                Op::X3 ? buf[NT + (rb * KQ + q + 1) * 64 + lane] : ah[nxt][rb];
                        }
                    }
                    __builtin_amdgcn_sched_barrier(0);
                }
#pragma unroll
                for (int rb = 0; rb < RB; ++rb) {
                    if (!kPinA) {
                        ah[cur][rb] = buf[(rb * KQ + q) * 64 + lane];
                        al[cur][rb] = Op::X3 ? buf[NT + (rb * KQ + q) * 64 + lane] : ah[cur][rb];
                    }
#define M2L_STEP(s)                                                                        \
    if (s < Op::S && (q + 1 < KQ || s < LASTS)) {                                          \
        _Pragma("unroll") for (int cb = 0; cb < CB; ++cb) acc[cb][rb] =                     \
            Op::template mma<(s < Op::S ? s : 0)>(ah[cur][rb], al[cur][rb], bh[q][cb],      \
                                                  bl[q][cb], acc[cb][rb]);                  \
    }
                    M2L_STEP(0)
                    M2L_STEP(1)
                    M2L_STEP(2)
                    M2L_STEP(3)
#undef M2L_STEP
                }
            }
        };

        // Register-staged operators (FP32, FP64 and the split forms).  The
        // operator of the next active slot is read into registers (each wave its
        // NPW chunks) while this slot runs, and written to the other LDS buffer
        // before the slot's barrier (with one buffer: between two barriers after
        // the products): the compiler then tracks every wait itself.  (A direct global-to-LDS copy
        // would make it wait for the copy before the first LDS read of the
        // products, since it cannot tell the two buffers apart.)  The source
        // chunks run kAhead contraction steps ahead across slot boundaries: the
        // last steps of a slot request the first chunks of the next one.
        constexpr int kAhead = KQ < m2l_ahead_staged(Op::X3) ? KQ : m2l_ahead_staged(Op::X3);
        constexpr int NCH = RB * KQ, NPW = (NCH + NW - 1) / NW;
        constexpr bool kStaged =
            Op::S != 1 && (DB || m2l_staged_regs(RB, NPW, NS, CB, sizeof(typename Op::Acc) / 4,
                                                 kAhead) <= 160);
        // FP32: a last output block with at most 12 rows of data runs as
        // 4-row products (v_mfma_f32_4x4x1f32, 16 blocks of 4 x 4: a quarter of
        // a 16 x 16 x 4 product's cycles) instead of a padded 16-row block.
        // Lane (g, col) feeds row 4 u + (col & 3) of the operator and element
        // 16 q + 4 r + g of target col; each block (4 lanes of one g) sums over
        // its own contraction elements, and the four lane groups are added at
        // the end.
        constexpr int NQ = (kStaged && std::is_same<Op, OpF32>::value && LASTR <= 12)
                               ? (LASTR + 3) / 4 : 0;
        constexpr int RBM = NQ > 0 ? RB - 1 : RB;  // row blocks on 16 x 16 products
        floatx4 accq[CB][NQ > 0 ? NQ : 1];
#pragma unroll
        for (int cb = 0; cb < CB; ++cb)
#pragma unroll
            for (int u = 0; u < (NQ > 0 ? NQ : 1); ++u) accq[cb][u] = floatx4{0.f, 0.f, 0.f, 0.f};
        auto load_op = [&](int jj, u32x4 (&r)[NPW][NS]) {
            const int slot = s0 + jj;
            const int dx = slot / 36 - 2 - ox, dy = (slot / 6) % 6 - 2 - oy, dz = slot % 6 - 2 - oz;
            const int cls = (dx + 3) * 49 + (dy + 3) * 7 + (dz + 3);
            const u32x4* th = (const u32x4*)Thi + (int64_t)cls * NT;
            const u32x4* tl = (const u32x4*)Tlo + (int64_t)cls * NT;
#pragma unroll
            for (int i = 0; i < NPW; ++i) {
                const int k = min(wave + NW * i, NCH - 1);
                r[i][0] = th[k * 64 + lane];
                if (Op::X3) r[i][NS - 1] = tl[k * 64 + lane];
            }
        };
        // (no branches: the loads would be sunk into a conditional store's
        // block, i.e. issued just before the store; the waves past the last
        // chunk write that chunk's bytes again)
        auto store_op = [&](u32x4* buf, const u32x4 (&r)[NPW][NS]) {
#pragma unroll
            for (int i = 0; i < NPW; ++i) {
                const int k = min(wave + NW * i, NCH - 1);
                buf[k * 64 + lane] = r[i][0];
                if (Op::X3) buf[NT + k * 64 + lane] = r[i][NS - 1];
            }
        };
        // products of one slot from operator `buf` and source offsets boff; the
        // first kAhead chunks arrive in bf, which on return holds the first
        // chunks of the slot at offsets boffn
        auto products_db = [&](const u32x4* buf, const int64_t (&boff)[CB],
                               const int64_t (&boffn)[CB], u32x4 (&bfh)[kAhead][CB],
                               u32x4 (&bfl)[kAhead][CB]) {
            u32x4 bh[KQ][CB], bl[KQ][CB];
#pragma unroll
            for (int q = 0; q < kAhead; ++q)
#pragma unroll
                for (int cb = 0; cb < CB; ++cb) {
                    bh[q][cb] = bfh[q][cb];
                    bl[q][cb] = bfl[q][cb];
                }
#pragma unroll
            for (int q = 0; q < KQ; ++q) {
#pragma unroll
                for (int cb = 0; cb < CB; ++cb) {
                    if (q + kAhead < KQ) {
                        bh[q + kAhead][cb] = Mh[boff[cb] + 4 * (q + kAhead)];
                        if (Op::X3) bl[q + kAhead][cb] = Ml[boff[cb] + 4 * (q + kAhead)];
                    } else {
                        const int qn = q + kAhead - KQ;
                        bfh[qn][cb] = Mh[boffn[cb] + 4 * qn];
                        if (Op::X3) bfl[qn][cb] = Ml[boffn[cb] + 4 * qn];
                    }
                }
                // keeps the optimiser from sinking the next slot's loads to
                // their use after the barrier (an empty statement, no wait)
                if (q + kAhead >= KQ) asm volatile("" ::: "memory");
                if constexpr (NQ > 0) {
#pragma unroll
                    for (int u = 0; u < NQ; ++u) {
                        const floatx4 aq = __builtin_bit_cast(
                            floatx4, buf[(RBM * KQ + q) * 64 + 16 * g + 4 * u + (lane & 3)]);
#pragma unroll
                        for (int r = 0; r < 4; ++r) {
                            if (q + 1 < KQ || r < LASTS) {
#pragma unroll
                                for (int cb = 0; cb < CB; ++cb)
                                    accq[cb][u] = __builtin_amdgcn_mfma_f32_4x4x1f32(
                                        aq[r], __builtin_bit_cast(floatx4, bh[q][cb])[r],
                                        accq[cb][u], 0, 0, 0);
                            }
                        }
                    }
                }
#pragma unroll
                for (int rb = 0; rb < RBM; ++rb) {
                    const u32x4 ah = buf[(rb * KQ + q) * 64 + lane];
                    const u32x4 al = Op::X3 ? buf[NT + (rb * KQ + q) * 64 + lane] : ah;
#define M2L_STEP(s)                                                                        \
    if (s < Op::S && (q + 1 < KQ || s < LASTS)) {                                          \
        _Pragma("unroll") for (int cb = 0; cb < CB; ++cb) acc[cb][rb] =                     \
            Op::template mma<(s < Op::S ? s : 0)>(ah, al, bh[q][cb], bl[q][cb], acc[cb][rb]); \
    }
                    M2L_STEP(0)
                    M2L_STEP(1)
                    M2L_STEP(2)
                    M2L_STEP(3)
#undef M2L_STEP
                }
                // the step's loads stay in the step (the scheduler would move
                // them down to their use, shortening the distance ahead)
                __builtin_amdgcn_sched_barrier(0);
            }
        };

        int j = next_slot(0);
        int src[CB];
        load_src(j, src);
        if constexpr (kStaged) {
            // state at the top of a slot j: its operator in `cur`, its source
            // offsets in boff and first chunks in flight (bfh/bfl), the source
            // indices of the next active slot jn in srcn
            int64_t boff[CB];
            u32x4 bfh[kAhead][CB], bfl[kAhead][CB];
            u32x4 opr[NPW][NS];
            int srcn[CB];
            int jn = next_slot(j + 1);
            load_src_u(jn, srcn);
            set_boff(src, boff);
#pragma unroll
            for (int q = 0; q < kAhead; ++q)
#pragma unroll
                for (int cb = 0; cb < CB; ++cb) {
                    bfh[q][cb] = Mh[boff[cb] + 4 * q];
                    bfl[q][cb] = Op::X3 ? Ml[boff[cb] + 4 * q] : bfh[q][cb];
                }
            if (j < ns) {
                load_op(j, opr);
                store_op(sT, opr);
            }
            __syncthreads();
            auto body = [&](const u32x4* cur, u32x4* nxt) {
                const int jnn = jn < ns ? next_slot(jn + 1) : ns;
                int srcnn[CB];
                load_src_u(jnn, srcnn);
                // unconditional loads (past the last slot, the last slot's
                // operator again), and every wave runs the products, so that
                // the number of loads in flight is the same on every path and
                // each wait covers only the load it is for
                load_op(jn < ns ? jn : j, opr);
                __builtin_amdgcn_sched_barrier(0);  // issued here, not at their use
                int64_t boffn[CB];
                set_boff(srcn, boffn);
                products_db(cur, boff, boffn, bfh, bfl);
                if (!DB) __syncthreads();  // the one buffer is no longer read
                store_op(nxt, opr);
                __syncthreads();  // nxt holds slot jn; cur is no longer read
                j = jn;
                jn = jnn;
#pragma unroll
                for (int cb = 0; cb < CB; ++cb) {
                    boff[cb] = boffn[cb];
                    srcn[cb] = srcnn[cb];
                }
            };
            // one body per iteration, the buffers swapped by parity (with the
            // loop unrolled by two, the next slot's first loads would be sunk
            // past the barrier into the second half)
            if (DB) {
                for (int par = 0; j < ns; par ^= 1) body(par ? sT2 : sT, par ? sT : sT2);
            } else {
                for (; j < ns;) body(sT, sT);
            }
        } else if constexpr (DB) {
            // single-product forms (short slots): two operator buffers filled
            // by direct global-to-LDS copies, the next active slot's operator
            // streaming in while this one is on the matrix cores (the compiler
            // waits for the copy before the first LDS read, which costs less
            // here than the register staging's shorter reach ahead); one
            // barrier per slot
            if (j < ns) stage(sT, j);
            while (j < ns) {
                {
                    int64_t boff[CB];
                    u32x4 bh[KQ][CB], bl[KQ][CB];
                    first_chunks(src, boff, bh, bl);
                    const int jn = next_slot(j + 1);
                    load_src(jn, src);
                    __syncthreads();  // sT holds slot j, sT2 is no longer read
                    if (jn < ns) stage(sT2, jn);
                    if (busy) products(sT, boff, bh, bl);
                    j = jn;
                }
                if (j >= ns) break;
                {
                    int64_t boff[CB];
                    u32x4 bh[KQ][CB], bl[KQ][CB];
                    first_chunks(src, boff, bh, bl);
                    const int jn = next_slot(j + 1);
                    load_src(jn, src);
                    __syncthreads();  // sT2 holds slot j, sT is no longer read
                    if (jn < ns) stage(sT, jn);
                    if (busy) products(sT2, boff, bh, bl);
                    j = jn;
                }
            }
        } else {
            while (j < ns) {
                stage(sT, j);
                int64_t boff[CB];
                u32x4 bh[KQ][CB], bl[KQ][CB];
                first_chunks(src, boff, bh, bl);
                const int jn = next_slot(j + 1);
                load_src(jn, src);
                __syncthreads();  // operator in LDS
                if (busy) products(sT, boff, bh, bl);
                __syncthreads();  // LDS free for the next operator
                j = jn;
            }
        }
        if constexpr (NQ > 0) {
            // sum the four lane groups; lane group g keeps rows 4 g .. 4 g + 3
            // of the last block (the 16 x 16 layout the store expects)
#pragma unroll
            for (int cb = 0; cb < CB; ++cb) {
                floatx4 v = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
                for (int u = 0; u < NQ; ++u) {
                    floatx4 t = accq[cb][u];
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        t[i] += __shfl_xor(t[i], 16, 64);
                        t[i] += __shfl_xor(t[i], 32, 64);
                    }
                    if (g == u) v = t;
                }
                acc[cb][RB - 1] = v;
            }
        }
        // output block (rb) of column col: the rows this lane holds; with
        // zero_fill, the last segment of the tile clears the partial results
        // after its own (without, k_m2l_sum_parts adds the tile's own ones)
#pragma unroll
        for (int cb = 0; cb < CB; ++cb) {
            if (tgt[cb] < 0) continue;
            typename Op::O* o = out + part * part_stride + (int64_t)tgt[cb] * LDO;
#pragma unroll
            for (int rb = 0; rb < RB; ++rb) Op::store(o, rb, g, acc[cb][rb]);
            if (last_seg && zero_fill)
                for (int q = part + 1; q < nparts; ++q) {
                    o += part_stride;
#pragma unroll
                    for (int rb = 0; rb < RB; ++rb) Op::store(o, rb, g, Op::zero());
                }
        }
    }
}

// Many partial results (small problems spread over many blocks): instead of
// clearing the partial results its segments did not write, each tile's
// segments 1 .. S-1 are added to partial result 0, in order (S = the blocks
// that held the tile's items, from the same item ranges as the M2L launch of
// nb blocks).  Block (t, y) takes elements 4 y .. 4 y + 3 of the rows of tile
// t's targets, one thread per target, eight partial results in flight.
template <typename TO>
__global__ void __launch_bounds__(256)
k_m2l_sum_parts(const int32_t* __restrict__ tiles, const int32_t* __restrict__ tpre, int nb,
                const int32_t* __restrict__ order, TO* __restrict__ out, int64_t part_stride,
                int ldo) {
    const int t = blockIdx.x;
    const int64_t W = tpre[gridDim.x];
    const int p0 = tpre[t], p1 = tpre[t + 1];
    const int b0 = (int)((((int64_t)p0 + 1) * nb - 1) / W);
    const int b1 = (int)((((int64_t)p1) * nb - 1) / W);  // block of item p1 - 1
    const int segs = b1 - b0 + 1;
    const int start = tiles[4 * t], count = tiles[4 * t + 1];
    if (segs <= 1 || (int)threadIdx.x >= count) return;
    const int64_t off = (int64_t)order[start + threadIdx.x] * ldo + 4 * blockIdx.y;
    double acc[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) acc[k] = (double)out[off + k];
    int q = 1;
    for (; q + 7 < segs; q += 8) {
        TO v[8][4];
#pragma unroll
        for (int u = 0; u < 8; ++u)
#pragma unroll
            for (int k = 0; k < 4; ++k) v[u][k] = out[(q + u) * part_stride + off + k];
#pragma unroll
        for (int u = 0; u < 8; ++u)
#pragma unroll
            for (int k = 0; k < 4; ++k) acc[k] += (double)v[u][k];
    }
    for (; q < segs; ++q)
#pragma unroll
        for (int k = 0; k < 4; ++k) acc[k] += (double)out[q * part_stride + off + k];
#pragma unroll
    for (int k = 0; k < 4; ++k) out[off + k] = (TO)acc[k];
}

// ---------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------
static bool is_lowp(int precision) { return precision >= HFMM_M2L_BF16; }
static bool is_x3(int precision) {
    return precision == HFMM_M2L_BF16X3 || precision == HFMM_M2L_FP16X3;
}
static bool is_bf16(int precision) {
    return precision == HFMM_M2L_BF16 || precision == HFMM_M2L_BF16X3;
}

// matrix cores for p <= 13 (FP32, BF16, FP16) and p <= 11 (FP64, whose
// operator must fit in LDS: 16 ceil(p^2/16) x 8 ceil(p^2/8) doubles)
// compute units of a device (cached per device; calls from several host
// threads store the same value)
static int m2l_cus(int device) {
    static std::atomic<int> cached[64];
    if (device < 0 || device >= 64) return 256;
    int n = cached[device].load(std::memory_order_relaxed);
    if (n <= 0) {
        if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, device) !=
                hipSuccess ||
            n <= 0)
            n = 256;
        cached[device].store(n, std::memory_order_relaxed);
    }
    return n;
}

bool m2l_uses_mfma(int p, int precision) {
    return precision == HFMM_FP64 ? p <= 11 : p <= 13;
}

// RB: output row blocks of 16; KQ: contraction blocks (16 for FP32, 32 for
// BF16/FP16); ld: row length of the packed operand
void m2l_layout(int p, int precision, int& RB, int& KQ, int& ld) {
    const int P = p * p;
    RB = (P + 15) / 16;
    if (!m2l_uses_mfma(p, precision)) {
        KQ = 0;
        ld = 16 * RB;
    } else if (is_lowp(precision)) {
        KQ = (P + 31) / 32;
        ld = 32 * KQ;
    } else if (precision == HFMM_FP64) {
        KQ = (P + 7) / 8;
        ld = 8 * KQ;
    } else {
        KQ = RB;
        ld = 16 * KQ;
    }
}

size_t m2l_ops_bytes(int p, int precision) {
    int RB, KQ, ld;
    m2l_layout(p, precision, RB, KQ, ld);
    const int P = p * p;
    if (!m2l_uses_mfma(p, precision))
        return (size_t)343 * P * P * (precision == HFMM_FP64 ? sizeof(double) : sizeof(float));
    if (precision == HFMM_FP64) return (size_t)343 * RB * KQ * 64 * 16;
    if (is_lowp(precision))
        return (size_t)343 * RB * KQ * 64 * 16 * (is_x3(precision) ? 2 : 1) + 256;
    return (size_t)343 * RB * KQ * 64 * 4 * sizeof(float);
}

#define HFMM_DISPATCH_P13(P_, F) \
    switch (P_) {                \
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
        default: throw Status{HFMM_E_UNSUPPORTED}; \
    }

#define HFMM_DISPATCH_RB(R, F) \
    switch (R) {               \
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
        default: throw Status{HFMM_E_UNSUPPORTED}; \
    }

template <typename T>
__global__ void k_cast_ops(const double* __restrict__ a, int64_t n, T* __restrict__ b) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) b[i] = (T)a[i];
}

void prepare_m2l_ops(Tree& t, int p, int precision, hipStream_t s) {
    if (t.ops_p == p && t.ops_prec == precision && t.T && !t.ops_rot) {
        t.arena.lo = t.mark_ops;
        return;
    }
    int RB, KQ, ld;
    m2l_layout(p, precision, RB, KQ, ld);
    const size_t bytes = m2l_ops_bytes(p, precision);
    t.T = t.arena.up<char>(bytes);
    t.bexp = nullptr;
    if (precision == HFMM_FP64 && !m2l_uses_mfma(p, precision)) {
        run_m2l_ops(t, p, 0, t.T, 0, 0, s);
    } else if (precision == HFMM_FP64) {
        run_m2l_ops(t, p, 2, t.T, RB, KQ, s);  // (padding written as zeros)
    } else if (!m2l_uses_mfma(p, precision)) {
        const int64_t nn = (int64_t)343 * p * p * p * p;
        double* tmp = t.arena.down<double>(nn);
        run_m2l_ops(t, p, 0, tmp, 0, 0, s);
        hipLaunchKernelGGL((k_cast_ops<float>), dim3(grid_for(nn, 256)), dim3(256), 0, s, tmp,
                           nn, (float*)t.T);
        LAUNCH_CHECK();
    } else if (is_lowp(precision)) {
        const size_t half = (size_t)343 * RB * KQ * 64 * 8;  // 16-bit elements per operand set
        char* hi = (char*)t.T;
        char* lo = is_x3(precision) ? hi + half * 2 : nullptr;
        t.bexp = (int32_t*)(hi + half * 2 * (is_x3(precision) ? 2 : 1));
        HIP_TRY(hipMemsetAsync(t.bexp, 0x80, 64 * sizeof(int32_t), s));
        run_m2l_ops_lp(p, precision, RB, KQ, t.bexp, hi, lo, s);
    } else {
        run_m2l_ops(t, p, 1, t.T, RB, KQ, s);  // (padding written as zeros)
    }
    t.ops_p = p;
    t.ops_prec = precision;
    t.ops_rot = false;
    t.mark_ops = t.arena.lo;
}

// the rotation M2L's tables, cached like the dense operators
void prepare_rot_ops(Tree& t, int p, int precision, hipStream_t s) {
    if (t.ops_p == p && t.ops_prec == precision && t.T && t.ops_rot) {
        t.arena.lo = t.mark_ops;
        return;
    }
    t.T = t.arena.up<char>(rot_ops_bytes(p, precision));
    t.bexp = nullptr;
    run_rot_ops(p, precision, t.T, s);
    t.ops_p = p;
    t.ops_prec = precision;
    t.ops_rot = true;
    t.mark_ops = t.arena.lo;
}

// Blocks and partial results of the matrix-core M2L.  The W work items
// (tile slots with a source, at least one per tile) number at least n_v / c,
// c the largest tile, since a slot of a tile covers at most c V pairs;
// blocks get at least m = floor(W_lb / NB) items each, so a tile's at most
// 216 items fall into at most 1 + ceil(215 / m) blocks, the number of partial
// results.  One block per CU (two when the operator buffers take at most
// 80 KiB of LDS), fewer when the partial results would exceed max_parts.
// Returns the number of partial results (0 without M2L targets).
int m2l_plan(const Tree& t, int p, int precision, int max_parts, int& nb) {
    const int ntiles = t.n_m2l_tiles;
    nb = 0;
    if (t.depth < 2 || ntiles == 0) return 0;
    int RB, KQ, ld;
    m2l_layout(p, precision, RB, KQ, ld);
    const int lds_kb = (m2l_double_buffer(RB, KQ, is_x3(precision) ? 2 : 1) ? 2 : 1) *
                       (is_x3(precision) ? 2 : 1) * RB * KQ;
    int cmax = 1;
    for (int k = 0; k < ntiles; ++k) cmax = std::max(cmax, t.m2l_tiles_h[4 * k + 1]);
    const int64_t w_lb = std::max<int64_t>(ntiles, (t.n_v + cmax - 1) / cmax);
    nb = m2l_cus(t.device) * (lds_kb <= 80 ? 2 : 1);
    if (max_parts <= 1) {
        nb = 1;
    } else {
        const int m_min = (215 + max_parts - 2) / (max_parts - 1);
        nb = (int)std::max<int64_t>(1, std::min<int64_t>(nb, w_lb / m_min));
    }
    const int m_lb = (int)(w_lb / nb);
    return std::min(nb, 1 + (215 + m_lb - 1) / m_lb);
}

// Runs M2L for every cell of level >= 2 into `out` (rows of t.ldm); returns
// the number of partial results (summed in the L2L epilogue) and their
// stride.  Low precision also fills levexp (per-level monopole exponents).
int run_m2l(Tree& t, int p, int precision, void* out, int64_t& part_stride, int max_parts,
            int32_t* levexp, hipStream_t s) {
    const int P = p * p;
    if (t.depth < 2) {
        part_stride = 0;
        return 0;
    }
    Arena& A = t.arena;
    const int c0 = t.level_start[2], c1 = t.ncells;
    if (!m2l_uses_mfma(p, precision)) {
        PhaseTimer pt(t, PH_M2L, s);
        const size_t sm = (size_t)P * (precision == HFMM_FP64 ? 8 : 4);
        if (precision == HFMM_FP64)
            hipLaunchKernelGGL((k_m2l_valu<double>), dim3(c1 - c0), dim3(64), sm, s, t.cells, c0,
                               c1, t.vsrc, t.M, P, t.ldm, (const double*)t.T, (double*)out);
        else
            hipLaunchKernelGGL((k_m2l_valu<float>), dim3(c1 - c0), dim3(64), sm, s, t.cells, c0,
                               c1, t.vsrc, t.M, P, t.ldm, (const float*)t.T, (float*)out);
        LAUNCH_CHECK();
        part_stride = (int64_t)t.ncells * t.ldm;
        return 1;
    }
    int RB, KQ, ld;
    m2l_layout(p, precision, RB, KQ, ld);
    const int ntiles = t.n_m2l_tiles;
    int nb;
    const int parts = m2l_plan(t, p, precision, max_parts, nb);
    if (parts == 0) {
        part_stride = 0;
        return 0;
    }
    part_stride = (int64_t)t.ncells * t.ldm;
    dim3 grid(nb), block(1024 / kM2LCB);
    // up to kDirectParts partial results go to the L2L epilogue as they are
    // (the segments clear the ones they do not write); more are first summed
    // into the first
    constexpr int kDirectParts = 4;
    const int fill = parts <= kDirectParts ? 1 : 0;
    auto finish = [&](auto* o) -> int {
        if (fill) return parts;
        hipLaunchKernelGGL(k_m2l_sum_parts, dim3(ntiles, 4 * RB), dim3(256), 0, s,
                           t.m2l_tiles, t.m2l_tpre, nb, t.m2l_torder, o, part_stride, 16 * RB);
        LAUNCH_CHECK();
        return 1;
    };
    if (precision == HFMM_FP64) {
        double* Mk = A.down<double>((size_t)(t.ncells + 1) * ld);
        {
            PhaseTimer pp(t, PH_M2L_PREP, s);
            run_pack(t.M, t.ldm, t.ncells, P, ld, Mk, true, s);
        }
        PhaseTimer pt(t, PH_M2L, s);
#define MFMA64_CASE(PP)                                                                       \
    {                                                                                         \
        constexpr int R = ((PP) * (PP) + 15) / 16;                                            \
        constexpr int K = ((PP) * (PP) + 7) / 8;                                              \
        constexpr int LS = ((PP) * (PP) - 8 * (K - 1) + 3) / 4;                               \
        hipLaunchKernelGGL((k_m2l_mma<R, K, kM2LCB, m2l_double_buffer(R, K, 1), OpF64, LS>),  \
                           grid, block, 0, s, t.m2l_tiles, t.m2l_tmask, t.m2l_tpre, ntiles,  \
                           parts, t.m2l_torder, t.vsrc, (const double*)Mk,                    \
                           (const double*)nullptr, t.ncells, (const double*)t.T,              \
                           (const double*)nullptr, (double*)out, part_stride, fill);          \
    }
        switch (p) {
            case 1: MFMA64_CASE(1); break;
            case 2: MFMA64_CASE(2); break;
            case 3: MFMA64_CASE(3); break;
            case 4: MFMA64_CASE(4); break;
            case 5: MFMA64_CASE(5); break;
            case 6: MFMA64_CASE(6); break;
            case 7: MFMA64_CASE(7); break;
            case 8: MFMA64_CASE(8); break;
            case 9: MFMA64_CASE(9); break;
            case 10: MFMA64_CASE(10); break;
            case 11: MFMA64_CASE(11); break;
            default: throw Status{HFMM_E_UNSUPPORTED};
        }
#undef MFMA64_CASE
        LAUNCH_CHECK();
        return finish((double*)out);
    }
    if (!is_lowp(precision)) {
        float* Mk = A.down<float>((size_t)(t.ncells + 1) * ld);
        {
            PhaseTimer pp(t, PH_M2L_PREP, s);
            run_pack(t.M, t.ldm, t.ncells, P, ld, Mk, false, s);
        }
        PhaseTimer pt(t, PH_M2L, s);
#define MFMA_CASE(PP)                                                                        \
    {                                                                                        \
        constexpr int R = ((PP) * (PP) + 15) / 16;                                           \
        constexpr int LS = ((PP) * (PP) - 16 * (R - 1) + 3) / 4;                             \
        constexpr int LR = (PP) * (PP) - 16 * (R - 1);                                       \
        hipLaunchKernelGGL((k_m2l_mma<R, R, kM2LCB, m2l_double_buffer(R, R, 1), OpF32, LS,   \
                                      LR>),                                                  \
                           grid, block, 0, s, t.m2l_tiles, t.m2l_tmask, t.m2l_tpre, ntiles, \
                           parts, t.m2l_torder, t.vsrc, (const float*)Mk,                    \
                           (const float*)nullptr, t.ncells, (const float*)t.T,               \
                           (const float*)nullptr, (float*)out, part_stride, fill);          \
    }
        HFMM_DISPATCH_P13(p, MFMA_CASE);
#undef MFMA_CASE
        LAUNCH_CHECK();
        return finish((float*)out);
    }
    // low precision: per-level scale, packed hi/lo operand, matrix cores
    const bool x3 = is_x3(precision);
    std::optional<PhaseTimer> tm;  // operand preparation, then the products
    tm.emplace(t, PH_M2L_PREP, s);
    HIP_TRY(hipMemsetAsync(levexp, 0x80, 32 * sizeof(int32_t), s));
    hipLaunchKernelGGL(k_level_exp, dim3(grid_for(t.ncells, 256)), dim3(256), 0, s, t.cells,
                       t.ncells, t.M, t.ldm, p, levexp);
    LAUNCH_CHECK();
    const size_t nel = (size_t)(t.ncells + 1) * ld;
    const size_t half = (size_t)343 * RB * KQ * 64 * 8;
    const int64_t tot = (int64_t)nel;
    if (is_bf16(precision)) {
        __bf16* mh = A.down<__bf16>(nel);
        __bf16* ml = x3 ? A.down<__bf16>(nel) : nullptr;
        hipLaunchKernelGGL((k_pack_lp<__bf16>), dim3(grid_for(tot, 256)), dim3(256), 0, s,
                           t.cells, t.M, t.ldm, t.ncells, P, ld, levexp, mh, ml);
        LAUNCH_CHECK();
        tm.reset();
        tm.emplace(t, PH_M2L, s);
        const __bf16* th = (const __bf16*)t.T;
        const __bf16* tl = x3 ? th + half : nullptr;
#define LP_CASE(R)                                                                             \
    if (x3)                                                                                    \
        hipLaunchKernelGGL((k_m2l_mma<R, (R + 1) / 2, kM2LCB, m2l_double_buffer(R, (R + 1) / 2, 2), OpLow<__bf16, true>>), grid, block, 0, s,    \
                           t.m2l_tiles, t.m2l_tmask, t.m2l_tpre, ntiles, parts, t.m2l_torder,    \
                           t.vsrc, mh, ml, t.ncells, th, tl, (float*)out, part_stride, fill);   \
    else                                                                                       \
        hipLaunchKernelGGL((k_m2l_mma<R, (R + 1) / 2, kM2LCB, m2l_double_buffer(R, (R + 1) / 2, 1), OpLow<__bf16, false>>), grid, block, 0, s,   \
                           t.m2l_tiles, t.m2l_tmask, t.m2l_tpre, ntiles, parts, t.m2l_torder,    \
                           t.vsrc, mh, ml, t.ncells, th, tl, (float*)out, part_stride, fill);
        HFMM_DISPATCH_RB(RB, LP_CASE);
#undef LP_CASE
    } else {
        _Float16* mh = A.down<_Float16>(nel);
        _Float16* ml = x3 ? A.down<_Float16>(nel) : nullptr;
        hipLaunchKernelGGL((k_pack_lp<_Float16>), dim3(grid_for(tot, 256)), dim3(256), 0, s,
                           t.cells, t.M, t.ldm, t.ncells, P, ld, levexp, mh, ml);
        LAUNCH_CHECK();
        tm.reset();
        tm.emplace(t, PH_M2L, s);
        const _Float16* th = (const _Float16*)t.T;
        const _Float16* tl = x3 ? th + half : nullptr;
#define LP_CASE(R)                                                                             \
    if (x3)                                                                                    \
        hipLaunchKernelGGL((k_m2l_mma<R, (R + 1) / 2, kM2LCB, m2l_double_buffer(R, (R + 1) / 2, 2), OpLow<_Float16, true>>), grid, block, 0, s,  \
                           t.m2l_tiles, t.m2l_tmask, t.m2l_tpre, ntiles, parts, t.m2l_torder,    \
                           t.vsrc, mh, ml, t.ncells, th, tl, (float*)out, part_stride, fill);   \
    else                                                                                       \
        hipLaunchKernelGGL((k_m2l_mma<R, (R + 1) / 2, kM2LCB, m2l_double_buffer(R, (R + 1) / 2, 1), OpLow<_Float16, false>>), grid, block, 0, s, \
                           t.m2l_tiles, t.m2l_tmask, t.m2l_tpre, ntiles, parts, t.m2l_torder,    \
                           t.vsrc, mh, ml, t.ncells, th, tl, (float*)out, part_stride, fill);
        HFMM_DISPATCH_RB(RB, LP_CASE);
#undef LP_CASE
    }
    LAUNCH_CHECK();
    return finish((float*)out);
}

}  // namespace hfmm
