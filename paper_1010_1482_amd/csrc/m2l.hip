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
           const double* __restrict__ M, int P, const T* __restrict__ Tm,
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
        for (int k = threadIdx.x; k < P; k += 64) ms[k] = (T)M[(int64_t)src * P + k];
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
        if (ro < P) out[(int64_t)c * P + ro] = acc[u];
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
#pragma unroll
                for (int cb = 0; cb < 4; ++cb) {
                    if (!act[cb]) continue;
                    floatx4 c = acc[cb][rb];
                    c = __builtin_amdgcn_mfma_f32_16x16x4f32(a4.x, b4[cb].x, c, 0, 0, 0);
                    c = __builtin_amdgcn_mfma_f32_16x16x4f32(a4.y, b4[cb].y, c, 0, 0, 0);
                    c = __builtin_amdgcn_mfma_f32_16x16x4f32(a4.z, b4[cb].z, c, 0, 0, 0);
                    c = __builtin_amdgcn_mfma_f32_16x16x4f32(a4.w, b4[cb].w, c, 0, 0, 0);
                    acc[cb][rb] = c;
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
// host side
// ---------------------------------------------------------------------
bool m2l_uses_mfma(int p, int precision) {
    return precision != HFMM_FP64 && p <= 13;
}

void m2l_layout(int p, int precision, int& RB, int& KQ, int& ld) {
    const int P = p * p;
    if (m2l_uses_mfma(p, precision)) {
        RB = (P + 15) / 16;
        KQ = (P + 15) / 16;
        ld = 16 * KQ;
    } else {
        RB = KQ = 0;
        ld = P;
    }
}

size_t m2l_ops_bytes(int p, int precision) {
    int RB, KQ, ld;
    m2l_layout(p, precision, RB, KQ, ld);
    const int P = p * p;
    if (precision == HFMM_FP64) return (size_t)343 * P * P * sizeof(double);
    if (m2l_uses_mfma(p, precision)) return (size_t)343 * RB * KQ * 64 * 4 * sizeof(float);
    return (size_t)343 * P * P * sizeof(float);
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
    if (precision == HFMM_FP64) {
        run_m2l_ops(t, p, true, (double*)t.T, nullptr, 0, 0, s);
    } else if (m2l_uses_mfma(p, precision)) {
        HIP_TRY(hipMemsetAsync(t.T, 0, bytes, s));
        run_m2l_ops(t, p, false, nullptr, (float*)t.T, RB, KQ, s);
    } else {
        const int64_t nn = (int64_t)343 * p * p * p * p;
        double* tmp = t.arena.down<double>(nn);
        run_m2l_ops(t, p, true, tmp, nullptr, 0, 0, s);
        hipLaunchKernelGGL((k_cast_ops<float>), dim3(grid_for(nn, 256)), dim3(256), 0, s, tmp,
                           nn, (float*)t.T);
        LAUNCH_CHECK();
    }
    t.ops_p = p;
    t.ops_prec = precision;
    t.mark_ops = t.arena.lo;
}

// Runs M2L for every cell of level >= 2 into `out`; returns the number of
// partial results written (summed by the downward pass) and their stride.
int run_m2l(Tree& t, int p, int precision, void* out, int64_t& part_stride, int max_parts,
            hipStream_t s) {
    const int P = p * p;
    if (t.depth < 2) {
        part_stride = 0;
        return 0;
    }
    const int c0 = t.level_start[2], c1 = t.ncells;
    if (!m2l_uses_mfma(p, precision)) {
        part_stride = 0;
        const size_t sm = (size_t)P * (precision == HFMM_FP64 ? 8 : 4);
        if (precision == HFMM_FP64)
            hipLaunchKernelGGL((k_m2l_valu<double>), dim3(c1 - c0), dim3(64), sm, s, t.cells, c0,
                               c1, t.vsrc, t.M, P, (const double*)t.T, (double*)out);
        else
            hipLaunchKernelGGL((k_m2l_valu<float>), dim3(c1 - c0), dim3(64), sm, s, t.cells, c0,
                               c1, t.vsrc, t.M, P, (const float*)t.T, (float*)out);
        LAUNCH_CHECK();
        return 1;
    }
    int RB, KQ, ld;
    m2l_layout(p, precision, RB, KQ, ld);
    const int ntiles = t.n_m2l_tiles;
    int parts = std::max(1, std::min(max_parts, (2048 + ntiles - 1) / std::max(ntiles, 1)));
    const int spp = (216 + parts - 1) / parts;
    parts = (216 + spp - 1) / spp;
    part_stride = (int64_t)t.ncells * ld;
    dim3 grid(ntiles, parts), block(256);
#define MFMA_CASE(R)                                                                          \
    hipLaunchKernelGGL((k_m2l_mfma<R, R>), grid, block, 0, s, t.m2l_tiles, t.m2l_order, t.vsrc, \
                       (const float*)t.Mk, t.ncells, (const float*)t.T, (float*)out,         \
                       part_stride, spp);
    HFMM_DISPATCH_RB(RB, MFMA_CASE);
#undef MFMA_CASE
    LAUNCH_CHECK();
    return parts;
}

}  // namespace hfmm
