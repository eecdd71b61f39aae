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
// FP32 matrix-core M2L.  Block = 4 waves, tile = up to 256 targets of one
// (level, octant), 64 per wave (4 column blocks of 16).  blockIdx.y selects a
// contiguous range of slots; each range writes its own partial result,
// summed later in the downward pass (deterministic, no atomics).
// ---------------------------------------------------------------------
template <int RB, int KQ>
__global__ void __launch_bounds__(256)
k_m2l_mfma(const int32_t* __restrict__ tiles, const int32_t* __restrict__ order,
           const int32_t* __restrict__ vsrc, const float* __restrict__ Mk, int ncells,
           const float* __restrict__ Tsw, float* __restrict__ out, int64_t part_stride,
           int slots_per_part) {
    constexpr int KP = 16 * KQ;
    constexpr int NT = RB * KQ * 64;  // float4 entries of one T_d
    __shared__ float4 sT[NT];
    const int tile = blockIdx.x, part = blockIdx.y;
    const int start = tiles[4 * tile], count = tiles[4 * tile + 1], oct = tiles[4 * tile + 2];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int g = lane >> 4, col = lane & 15;
    int tgt[4];
#pragma unroll
    for (int cb = 0; cb < 4; ++cb) {
        const int i = wave * 64 + cb * 16 + col;
        tgt[cb] = i < count ? order[start + i] : -1;
    }
    floatx4 acc[4][RB];
#pragma unroll
    for (int cb = 0; cb < 4; ++cb)
#pragma unroll
        for (int rb = 0; rb < RB; ++rb) acc[cb][rb] = floatx4{0.f, 0.f, 0.f, 0.f};
    const int ox = (oct >> 2) & 1, oy = (oct >> 1) & 1, oz = oct & 1;
    const int s0 = part * slots_per_part, s1 = min(216, s0 + slots_per_part);
    for (int slot = s0; slot < s1; ++slot) {
        const int dx = slot / 36 - 2 - ox, dy = (slot / 6) % 6 - 2 - oy, dz = slot % 6 - 2 - oz;
        if (max(abs(dx), max(abs(dy), abs(dz))) <= 1) continue;  // adjacent: never in V
        const int cls = (dx + 3) * 49 + (dy + 3) * 7 + (dz + 3);
        int src[4];
        bool any = false;
#pragma unroll
        for (int cb = 0; cb < 4; ++cb) {
            src[cb] = tgt[cb] >= 0 ? vsrc[(int64_t)tgt[cb] * 216 + slot] : -1;
            any |= src[cb] >= 0;
        }
        if (!__syncthreads_or(any)) continue;
        const float4* Tg = (const float4*)Tsw + (int64_t)cls * NT;
        for (int i = threadIdx.x; i < NT; i += 256) sT[i] = Tg[i];
        __syncthreads();
        bool act[4];
        const float* Bp[4];
#pragma unroll
        for (int cb = 0; cb < 4; ++cb) {
            act[cb] = __ballot(src[cb] >= 0) != 0;
            Bp[cb] = Mk + (int64_t)(src[cb] >= 0 ? src[cb] : ncells) * KP + 4 * g;
        }
#pragma unroll
        for (int q = 0; q < KQ; ++q) {
            float4 b4[4];
#pragma unroll
            for (int cb = 0; cb < 4; ++cb) b4[cb] = *(const float4*)(Bp[cb] + 16 * q);
#pragma unroll
            for (int rb = 0; rb < RB; ++rb) {
                const float4 a4 = sT[(rb * KQ + q) * 64 + lane];
                // the four column blocks are independent accumulators:
                // interleave them so no instruction waits on the previous one
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const float av = r == 0 ? a4.x : r == 1 ? a4.y : r == 2 ? a4.z : a4.w;
#pragma unroll
                    for (int cb = 0; cb < 4; ++cb) {
                        if (!act[cb]) continue;
                        const float bv = r == 0   ? b4[cb].x
                                         : r == 1 ? b4[cb].y
                                         : r == 2 ? b4[cb].z
                                                  : b4[cb].w;
                        acc[cb][rb] =
                            __builtin_amdgcn_mfma_f32_16x16x4f32(av, bv, acc[cb][rb], 0, 0, 0);
                    }
                }
            }
        }
        __syncthreads();
    }
    // output block (rb): lane holds rows 16 rb + 4 g + (0..3) of column col
#pragma unroll
    for (int cb = 0; cb < 4; ++cb) {
        if (tgt[cb] < 0) continue;
        float* o = out + part * part_stride + (int64_t)tgt[cb] * KP + 4 * g;
#pragma unroll
        for (int rb = 0; rb < RB; ++rb) {
            floatx4 c = acc[cb][rb];
            *(float4*)(o + 16 * rb) = make_float4(c[0], c[1], c[2], c[3]);
        }
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

// largest monopole exponent per level
__global__ void k_level_exp(const Cell* __restrict__ cells, int nc, const double* __restrict__ M,
                            int ldm, int32_t* __restrict__ levexp) {
    int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= nc) return;
    double v = fabs(M[(int64_t)c * ldm]);
    if (v > 0.0) atomicMax(&levexp[cells[c].level], ilogb(v));
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
        const int e = levexp[cells[c].level];
        v = ldexp(M[(int64_t)c * ldm + k], -mu_exp(degree_of(k)) - (e + 1));
    }
    const T16 h = (T16)(float)v;
    hi[gid] = h;
    if (lo) lo[gid] = (T16)(float)(v - (double)(float)h);
}

template <int RB, int KQ, typename T16, bool X3>
__global__ void __launch_bounds__(256)
k_m2l_mfma_lp(const int32_t* __restrict__ tiles, const int32_t* __restrict__ order,
              const int32_t* __restrict__ vsrc, const T16* __restrict__ Mhi,
              const T16* __restrict__ Mlo, int ncells, const T16* __restrict__ Thi,
              const T16* __restrict__ Tlo, float* __restrict__ out, int64_t part_stride,
              int slots_per_part) {
    using V = typename LowP<T16>::vec;
    constexpr int KP = 32 * KQ;        // padded contraction length of the operand
    constexpr int LDO = 16 * RB;       // output row length
    constexpr int NT = RB * KQ * 64;   // 16-byte entries of one operator
    __shared__ V sT[(X3 ? 2 : 1) * NT];
    const int tile = blockIdx.x, part = blockIdx.y;
    const int start = tiles[4 * tile], count = tiles[4 * tile + 1], oct = tiles[4 * tile + 2];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int g = lane >> 4, col = lane & 15;
    int tgt[4];
#pragma unroll
    for (int cb = 0; cb < 4; ++cb) {
        const int i = wave * 64 + cb * 16 + col;
        tgt[cb] = i < count ? order[start + i] : -1;
    }
    floatx4 acc[4][RB];
#pragma unroll
    for (int cb = 0; cb < 4; ++cb)
#pragma unroll
        for (int rb = 0; rb < RB; ++rb) acc[cb][rb] = floatx4{0.f, 0.f, 0.f, 0.f};
    const int ox = (oct >> 2) & 1, oy = (oct >> 1) & 1, oz = oct & 1;
    const int s0 = part * slots_per_part, s1 = min(216, s0 + slots_per_part);
    for (int slot = s0; slot < s1; ++slot) {
        const int dx = slot / 36 - 2 - ox, dy = (slot / 6) % 6 - 2 - oy, dz = slot % 6 - 2 - oz;
        if (max(abs(dx), max(abs(dy), abs(dz))) <= 1) continue;
        const int cls = (dx + 3) * 49 + (dy + 3) * 7 + (dz + 3);
        int src[4];
        bool any = false;
#pragma unroll
        for (int cb = 0; cb < 4; ++cb) {
            src[cb] = tgt[cb] >= 0 ? vsrc[(int64_t)tgt[cb] * 216 + slot] : -1;
            any |= src[cb] >= 0;
        }
        if (!__syncthreads_or(any)) continue;
        {
            const V* th = (const V*)Thi + (int64_t)cls * NT;
            for (int i = threadIdx.x; i < NT; i += 256) sT[i] = th[i];
            if (X3) {
                const V* tl = (const V*)Tlo + (int64_t)cls * NT;
                for (int i = threadIdx.x; i < NT; i += 256) sT[NT + i] = tl[i];
            }
        }
        __syncthreads();
        bool act[4];
        int64_t boff[4];
#pragma unroll
        for (int cb = 0; cb < 4; ++cb) {
            act[cb] = __ballot(src[cb] >= 0) != 0;
            boff[cb] = (int64_t)(src[cb] >= 0 ? src[cb] : ncells) * KP + 8 * g;
        }
#pragma unroll
        for (int q = 0; q < KQ; ++q) {
            V bh[4], bl[4];
#pragma unroll
            for (int cb = 0; cb < 4; ++cb) {
                bh[cb] = *(const V*)(Mhi + boff[cb] + 32 * q);
                if (X3) bl[cb] = *(const V*)(Mlo + boff[cb] + 32 * q);
            }
#pragma unroll
            for (int rb = 0; rb < RB; ++rb) {
                const V ah = sT[(rb * KQ + q) * 64 + lane];
                V al;
                if (X3) al = sT[NT + (rb * KQ + q) * 64 + lane];
#pragma unroll
                for (int cb = 0; cb < 4; ++cb)
                    if (act[cb]) acc[cb][rb] = LowP<T16>::mma(ah, bh[cb], acc[cb][rb]);
                if (X3) {
#pragma unroll
                    for (int cb = 0; cb < 4; ++cb)
                        if (act[cb]) acc[cb][rb] = LowP<T16>::mma(ah, bl[cb], acc[cb][rb]);
#pragma unroll
                    for (int cb = 0; cb < 4; ++cb)
                        if (act[cb]) acc[cb][rb] = LowP<T16>::mma(al, bh[cb], acc[cb][rb]);
                }
            }
        }
        __syncthreads();
    }
#pragma unroll
    for (int cb = 0; cb < 4; ++cb) {
        if (tgt[cb] < 0) continue;
        float* o = out + part * part_stride + (int64_t)tgt[cb] * LDO + 4 * g;
#pragma unroll
        for (int rb = 0; rb < RB; ++rb) {
            floatx4 c = acc[cb][rb];
            *(float4*)(o + 16 * rb) = make_float4(c[0], c[1], c[2], c[3]);
        }
    }
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

bool m2l_uses_mfma(int p, int precision) { return precision != HFMM_FP64 && p <= 13; }

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
    } else {
        KQ = RB;
        ld = 16 * KQ;
    }
}

size_t m2l_ops_bytes(int p, int precision) {
    int RB, KQ, ld;
    m2l_layout(p, precision, RB, KQ, ld);
    const int P = p * p;
    if (precision == HFMM_FP64) return (size_t)343 * P * P * sizeof(double);
    if (!m2l_uses_mfma(p, precision)) return (size_t)343 * P * P * sizeof(float);
    if (is_lowp(precision))
        return (size_t)343 * RB * KQ * 64 * 16 * (is_x3(precision) ? 2 : 1) + 256;
    return (size_t)343 * RB * KQ * 64 * 4 * sizeof(float);
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
    if (t.ops_p == p && t.ops_prec == precision && t.T) {
        t.arena.lo = t.mark_ops;
        return;
    }
    int RB, KQ, ld;
    m2l_layout(p, precision, RB, KQ, ld);
    const size_t bytes = m2l_ops_bytes(p, precision);
    t.T = t.arena.up<char>(bytes);
    t.bexp = nullptr;
    if (precision == HFMM_FP64) {
        run_m2l_ops(t, p, true, (double*)t.T, nullptr, 0, 0, s);
    } else if (!m2l_uses_mfma(p, precision)) {
        const int64_t nn = (int64_t)343 * p * p * p * p;
        double* tmp = t.arena.down<double>(nn);
        run_m2l_ops(t, p, true, tmp, nullptr, 0, 0, s);
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
        // the kernel fills the p^2 x p^2 block; the padding must read as zero
        HIP_TRY(hipMemsetAsync(t.T, 0, bytes, s));
        run_m2l_ops(t, p, false, nullptr, (float*)t.T, RB, KQ, s);
    }
    t.ops_p = p;
    t.ops_prec = precision;
    t.mark_ops = t.arena.lo;
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
    int parts = std::max(1, std::min(max_parts, (2048 + ntiles - 1) / std::max(ntiles, 1)));
    const int spp = (216 + parts - 1) / parts;
    parts = (216 + spp - 1) / spp;
    part_stride = (int64_t)t.ncells * t.ldm;
    dim3 grid(ntiles, parts), block(256);
    if (!is_lowp(precision)) {
        float* Mk = A.down<float>((size_t)(t.ncells + 1) * ld);
        run_pack(t.M, t.ldm, t.ncells, P, ld, Mk, false, s);
#define MFMA_CASE(R)                                                                          \
    hipLaunchKernelGGL((k_m2l_mfma<R, R>), grid, block, 0, s, t.m2l_tiles, t.m2l_order, t.vsrc, \
                       (const float*)Mk, t.ncells, (const float*)t.T, (float*)out, part_stride, \
                       spp);
        HFMM_DISPATCH_RB(RB, MFMA_CASE);
#undef MFMA_CASE
        LAUNCH_CHECK();
        return parts;
    }
    // low precision: per-level scale, packed hi/lo operand, matrix cores
    const bool x3 = is_x3(precision);
    HIP_TRY(hipMemsetAsync(levexp, 0x80, 32 * sizeof(int32_t), s));
    hipLaunchKernelGGL(k_level_exp, dim3(grid_for(t.ncells, 256)), dim3(256), 0, s, t.cells,
                       t.ncells, t.M, t.ldm, levexp);
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
        const __bf16* th = (const __bf16*)t.T;
        const __bf16* tl = x3 ? th + half : nullptr;
#define LP_CASE(R)                                                                             \
    if (x3)                                                                                    \
        hipLaunchKernelGGL((k_m2l_mfma_lp<R, (R + 1) / 2, __bf16, true>), grid, block, 0, s,    \
                           t.m2l_tiles, t.m2l_order, t.vsrc, mh, ml, t.ncells, th, tl,          \
                           (float*)out, part_stride, spp);                                      \
    else                                                                                       \
        hipLaunchKernelGGL((k_m2l_mfma_lp<R, (R + 1) / 2, __bf16, false>), grid, block, 0, s,   \
                           t.m2l_tiles, t.m2l_order, t.vsrc, mh, ml, t.ncells, th, tl,          \
                           (float*)out, part_stride, spp);
        HFMM_DISPATCH_RB(RB, LP_CASE);
#undef LP_CASE
    } else {
        _Float16* mh = A.down<_Float16>(nel);
        _Float16* ml = x3 ? A.down<_Float16>(nel) : nullptr;
        hipLaunchKernelGGL((k_pack_lp<_Float16>), dim3(grid_for(tot, 256)), dim3(256), 0, s,
                           t.cells, t.M, t.ldm, t.ncells, P, ld, levexp, mh, ml);
        LAUNCH_CHECK();
        const _Float16* th = (const _Float16*)t.T;
        const _Float16* tl = x3 ? th + half : nullptr;
#define LP_CASE(R)                                                                             \
    if (x3)                                                                                    \
        hipLaunchKernelGGL((k_m2l_mfma_lp<R, (R + 1) / 2, _Float16, true>), grid, block, 0, s,  \
                           t.m2l_tiles, t.m2l_order, t.vsrc, mh, ml, t.ncells, th, tl,          \
                           (float*)out, part_stride, spp);                                      \
    else                                                                                       \
        hipLaunchKernelGGL((k_m2l_mfma_lp<R, (R + 1) / 2, _Float16, false>), grid, block, 0, s, \
                           t.m2l_tiles, t.m2l_order, t.vsrc, mh, ml, t.ncells, th, tl,          \
                           (float*)out, part_stride, spp);
        HFMM_DISPATCH_RB(RB, LP_CASE);
#undef LP_CASE
    }
    LAUNCH_CHECK();
    return parts;
}

}  // namespace hfmm
