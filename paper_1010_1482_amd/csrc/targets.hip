// Separate targets: every target point is binned into the source tree and
// evaluated in its box.  A target's key prefix is followed down the tree as
// far as cells exist: it ends in a leaf (the box is that leaf), or in a
// split cell whose octant holding the target is empty (the box is that
// octant, a source-free leaf added under the cell), or the target lies
// outside the root cube (the box is the root-sized cube of the extended grid
// that holds it).  The evaluation then follows the paper's method (Sec. 2)
// with the adaptive lists it cites (Sec. 6) for these boxes.
//
// Targets are sorted by a key that keeps each box contiguous (the Morton
// key inside the root; outside, a key of the level-0 cube), the box of every
// sorted target is found by a descent from the root, runs of equal boxes
// become the box records, and the targets are gathered in sorted order (FP64,
// and FP32 relative to their box centre).
#include "common.hpp"

#include <algorithm>

namespace hfmm {

#pragma clang fp contract(off)

__device__ inline uint64_t spread21(uint32_t v) {
    uint64_t x = v & 0x1fffffu;
    x = (x | (x << 32)) & 0x1f00000000ffffull;
    x = (x | (x << 16)) & 0x1f0000ff0000ffull;
    x = (x | (x << 8)) & 0x100f00f00f00f00full;
    x = (x | (x << 4)) & 0x10c30c30c30c30c3ull;
    x = (x | (x << 2)) & 0x1249249249249249ull;
    return x;
}

constexpr double kTop = 2097152.0;    // 2^21
constexpr int64_t kFar = 1 << 20;     // outside cubes clamped to +-2^20 root widths
constexpr int kKeyOut = 512;          // outside cubes in the sort key: +-2^9

// Where a target lies relative to the root cube.  Per axis f = floor((x - b)
// s); inside when 0 <= f <= 2^21 on every axis (the upper face belongs to
// the cube, as for the sources' keys), with q = min(f, 2^21 - 1); outside,
// the level-0 cube c = floor(f / 2^21).  A non-finite coordinate is read as
// the root's lower corner (the status word reports it).
struct TPos {
    bool inside;
    int64_t q[3];  // finest-level coordinates (inside) or level-0 cube (outside)
};

__device__ inline TPos target_pos(const Root& r, double x, double y, double z) {
    const double v[3] = {x, y, z};
    double f[3];
    TPos t;
    t.inside = true;
    for (int a = 0; a < 3; ++a) {
        const double va = isfinite(v[a]) ? v[a] : r.b[a];
        f[a] = floor((va - r.b[a]) * r.scale);
        if (!(f[a] >= 0.0 && f[a] <= kTop)) t.inside = false;
    }
    for (int a = 0; a < 3; ++a) {
        if (t.inside) {
            t.q[a] = f[a] > kTop - 1.0 ? (int64_t)kTop - 1 : (int64_t)f[a];
        } else {
            double c = floor(f[a] / kTop);
            c = fmin(fmax(c, -(double)kFar), (double)kFar);
            t.q[a] = (int64_t)c;
        }
    }
    return t;
}

__global__ void k_tkeys(const double* __restrict__ tx, const double* __restrict__ ty,
                        const double* __restrict__ tz, int64_t n, const Root* __restrict__ root,
                        uint64_t* __restrict__ keys, int32_t* __restrict__ idx,
                        int32_t* __restrict__ status) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    bool bad = false;
    if (i < n) {
        const double x = tx[i], y = ty[i], z = tz[i];
        bad = !(isfinite(x) && isfinite(y) && isfinite(z));
        const TPos p = target_pos(*root, x, y, z);
        uint64_t k;
        if (p.inside) {
            k = (spread21((uint32_t)p.q[0]) << 2) | (spread21((uint32_t)p.q[1]) << 1) |
                spread21((uint32_t)p.q[2]);
        } else {
            uint32_t c[3];
            for (int a = 0; a < 3; ++a)
                c[a] = (uint32_t)(min(max(p.q[a], (int64_t)-kKeyOut), (int64_t)kKeyOut - 1) +
                                  kKeyOut);
            k = (1ull << 63) |
                (((spread21(c[0]) << 2) | (spread21(c[1]) << 1) | spread21(c[2])) << 33);
        }
        keys[i] = k;
        idx[i] = (int32_t)i;
    }
    if (__ballot(bad) && (threadIdx.x & 63) == 0) atomicOr(status, (int32_t)ST_TGT_NONFINITE);
}

// The box of every sorted target: g[6 s ..] = (kind | level << 8, ix, iy,
// iz, host, leaf); the FP64 positions in sorted order.
__global__ void k_tbox_find(const double* __restrict__ tx, const double* __restrict__ ty,
                            const double* __restrict__ tz, int64_t n,
                            const int32_t* __restrict__ sidx, const Root* __restrict__ root,
                            const Cell* __restrict__ cells, int32_t* __restrict__ g,
                            double4* __restrict__ p64) {
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    const int64_t i = sidx[s];
    const double x = tx[i], y = ty[i], z = tz[i];
    p64[s] = make_double4(x, y, z, 0.0);
    const TPos p = target_pos(*root, x, y, z);
    int kind, level, host, leaf;
    int64_t c[3];
    if (!p.inside) {
        kind = 2;
        level = 0;
        host = leaf = -1;
        for (int a = 0; a < 3; ++a) c[a] = p.q[a];
    } else {
        int C = 0;
        for (;;) {
            const Cell cc = cells[C];
            if (cc.nchild == 0) {
                kind = 0;
                level = cc.level;
                host = leaf = C;
                c[0] = cc.ix;
                c[1] = cc.iy;
                c[2] = cc.iz;
                break;
            }
            const int lev = cc.level + 1, sh = HFMM_KEY_LEVELS - lev;
            for (int a = 0; a < 3; ++a) c[a] = p.q[a] >> sh;
            const int o = (int)(((c[0] & 1) << 2) | ((c[1] & 1) << 1) | (c[2] & 1));
            if ((cc.mask >> o) & 1) {
                C = cc.child + __popc((unsigned)cc.mask & ((1u << o) - 1u));
            } else {
                kind = 1;
                level = lev;
                host = C;
                leaf = -1;
                break;
            }
        }
    }
    int32_t* o = g + 6 * s;
    o[0] = kind | (level << 8);
    o[1] = (int32_t)c[0];
    o[2] = (int32_t)c[1];
    o[3] = (int32_t)c[2];
    o[4] = host;
    o[5] = leaf;
}

// 1 where a run of equal boxes starts
__global__ void k_tbox_flags(const int32_t* __restrict__ g, int64_t n, int32_t* __restrict__ flag) {
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    bool start = s == 0;
    if (!start)
        for (int k = 0; k < 4; ++k) start |= g[6 * s + k] != g[6 * (s - 1) + k];
    flag[s] = start ? 1 : 0;
}

__global__ void k_tbox_write(const int32_t* __restrict__ g, const int32_t* __restrict__ flag,
                             const int32_t* __restrict__ bidx, int64_t n,
                             TBox* __restrict__ box, int32_t* __restrict__ end,
                             int32_t* __restrict__ box_of) {
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    // bidx is the exclusive scan of the run starts: within a run it already
    // counts the run's own start
    const int b = bidx[s] + flag[s] - 1;
    box_of[s] = b;
    if (flag[s]) {
        const int32_t* o = g + 6 * s;
        TBox bx;
        bx.first = (int32_t)s;
        bx.count = 0;
        bx.kind = (int16_t)(o[0] & 255);
        bx.level = (int16_t)(o[0] >> 8);
        bx.ix = o[1];
        bx.iy = o[2];
        bx.iz = o[3];
        bx.host = o[4];
        bx.leaf = o[5];
        box[b] = bx;
    }
    if (s == n - 1 || flag[s + 1]) end[b] = (int32_t)(s + 1);
}

// counts from the run ends; FP32 targets relative to their box centre
__global__ void k_tbox_count(TBox* __restrict__ box, const int32_t* __restrict__ end, int nbox) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b < nbox) box[b].count = end[b] - box[b].first;
}

__global__ void k_tgather32(const double4* __restrict__ p64, const TBox* __restrict__ box,
                            const int32_t* __restrict__ box_of, int64_t n,
                            const Root* __restrict__ root, float4* __restrict__ p32) {
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    double c[3];
    cell_centre(*root, box_cell(box[box_of[s]]), c);
    const double4 v = p64[s];
    p32[s] = make_float4((float)(v.x - c[0]), (float)(v.y - c[1]), (float)(v.z - c[2]), 0.0f);
}

#pragma clang fp contract(on)

Targets self_targets(const Tree& t) {
    Targets tg{};
    tg.box = t.leaf_boxes;
    tg.box_of = t.leaf_box_of;
    tg.p32 = t.p32;
    tg.p64 = t.p64;
    tg.perm = t.perm;
    tg.n = t.n;
    tg.nbox = t.nleaves;
    tg.by_leaf = 1;
    return tg;
}

Targets bin_targets(Tree& t, const double* tx, const double* ty, const double* tz, int64_t nt,
                    hipStream_t s) {
    Arena& A = t.arena;
    const int64_t n = nt;
    // persistent for the evaluation: sorted index, positions, boxes
    int32_t* sidx = A.up<int32_t>(n);
    double4* p64 = A.up<double4>(n);
    float4* p32 = A.up<float4>(n);
    int32_t* box_of = A.up<int32_t>(n);
    uint64_t* k0 = A.down<uint64_t>(n);
    int32_t* i0 = A.down<int32_t>(n);
    uint64_t* k1 = A.down<uint64_t>(n);
    hipLaunchKernelGGL(k_tkeys, dim3(grid_for(n, 256)), dim3(256), 0, s, tx, ty, tz, n, t.root,
                       k0, i0, t.status);
    LAUNCH_CHECK();
    // boxes are at most one level below the deepest cell; outside keys use
    // bits 33..63
    const int levels = std::min(HFMM_KEY_LEVELS, t.depth + 1);
    const int lo_bit = std::min(33, 3 * (HFMM_KEY_LEVELS - levels));
    radix_sort_pairs(k0, i0, k1, sidx, n, lo_bit, 64, A, s);
    int32_t* g = A.down<int32_t>((size_t)6 * n);
    int32_t* flag = A.down<int32_t>(n + 1);
    int32_t* bidx = A.down<int32_t>(n + 1);
    hipLaunchKernelGGL(k_tbox_find, dim3(grid_for(n, 256)), dim3(256), 0, s, tx, ty, tz, n, sidx,
                       t.root, t.cells, g, p64);
    LAUNCH_CHECK();
    hipLaunchKernelGGL(k_tbox_flags, dim3(grid_for(n, 256)), dim3(256), 0, s, g, n, flag);
    LAUNCH_CHECK();
    scan_exclusive_i32(flag, bidx, n, A, s);
    int32_t nbox = 0;
    HIP_TRY(hipMemcpyAsync(&nbox, bidx + n, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    stream_wait(s);
    TBox* box = A.up<TBox>(std::max(nbox, 1));
    int32_t* end = A.down<int32_t>(std::max(nbox, 1));
    hipLaunchKernelGGL(k_tbox_write, dim3(grid_for(n, 256)), dim3(256), 0, s, g, flag, bidx, n,
                       box, end, box_of);
    LAUNCH_CHECK();
    hipLaunchKernelGGL(k_tbox_count, dim3(grid_for(nbox, 256)), dim3(256), 0, s, box, end, nbox);
    LAUNCH_CHECK();
    hipLaunchKernelGGL(k_tgather32, dim3(grid_for(n, 256)), dim3(256), 0, s, p64, box, box_of, n,
                       t.root, p32);
    LAUNCH_CHECK();
    Targets tg{};
    tg.box = box;
    tg.box_of = box_of;
    tg.p32 = p32;
    tg.p64 = p64;
    tg.perm = sidx;
    tg.n = n;
    tg.nbox = nbox;
    tg.by_leaf = 0;
    return tg;
}

}  // namespace hfmm
