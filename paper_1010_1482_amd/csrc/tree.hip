// Octree construction on the device: FP64 bounding cube, 63-bit Morton keys,
// stable LSD radix sort, and level-by-level cell splitting.
//
// The paper sorts particles and builds the tree and lists on the host
// (Sec. 4, "sort" and "other" in Fig. 6); here every step is a kernel.  A
// census of the sorted keys gives the number of splitting cells of every
// level before the levels are built, so the level loop runs without host
// round trips: the host reads back twice (the census, then the level
// starts).
// Non-finite source coordinates are recorded in the tree's status word.
#include "common.hpp"

#include <algorithm>
#include <cmath>

namespace hfmm {

constexpr int kBlock = 256;
constexpr int kItems = 4;
constexpr int kTile = kBlock * kItems;  // elements per block in a scan
// radix sort: elements per thread and per block (with 16 per thread a block
// writes runs of about 16 keys per digit, so the scatter's stores coalesce)
constexpr int kSortItems = 16;
constexpr int kSortTile = kBlock * kSortItems;

// ---------------------------------------------------------------------
// block-level helpers
// ---------------------------------------------------------------------
__device__ inline int wave_inclusive_scan(int v) {
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        int u = __shfl_up(v, d, 64);
        if (lane >= d) v += u;
    }
    return v;
}

// exclusive scan of one value per thread over a 256-thread block; returns
// the block total in *total
__device__ inline int block_exclusive_scan(int v, int* total) {
    __shared__ int wsum[kBlock / 64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    int inc = wave_inclusive_scan(v);
    if (lane == 63) wsum[w] = inc;
    __syncthreads();
    int off = 0, tot = 0;
#pragma unroll
    for (int i = 0; i < kBlock / 64; ++i) {
        if (i < w) off += wsum[i];
        tot += wsum[i];
    }
    __syncthreads();
    *total = tot;
    return off + inc - v;
}

// ---------------------------------------------------------------------
// device-wide exclusive scan (int32): block sums, scan of sums, block scans
// ---------------------------------------------------------------------
__global__ void k_scan_partials(const int32_t* __restrict__ in, int64_t n,
                                int32_t* __restrict__ part) {
    const int64_t base = (int64_t)blockIdx.x * kTile;
    int s = 0;
#pragma unroll
    for (int k = 0; k < kItems; ++k) {
        int64_t i = base + (int64_t)threadIdx.x * kItems + k;
        if (i < n) s += in[i];
    }
    int tot;
    block_exclusive_scan(s, &tot);
    if (threadIdx.x == 0) part[blockIdx.x] = tot;
}

__global__ void k_scan_sums(int32_t* part, int nparts) {
    // single block, sequential over chunks of 256
    int carry = 0;
    for (int c0 = 0; c0 < nparts; c0 += kBlock) {
        int i = c0 + threadIdx.x;
        int v = i < nparts ? part[i] : 0;
        int tot;
        int ex = block_exclusive_scan(v, &tot);
        if (i < nparts) part[i] = carry + ex;
        carry += tot;
        __syncthreads();
    }
    if (threadIdx.x == 0) part[nparts] = carry;
}

__global__ void k_scan_blocks(const int32_t* __restrict__ in, int64_t n,
                              const int32_t* __restrict__ part,
                              int32_t* __restrict__ out, int write_total,
                              int32_t* __restrict__ total2) {
    const int64_t base = (int64_t)blockIdx.x * kTile;
    int v[kItems];
    int s = 0;
#pragma unroll
    for (int k = 0; k < kItems; ++k) {
        int64_t i = base + (int64_t)threadIdx.x * kItems + k;
        v[k] = i < n ? in[i] : 0;
        s += v[k];
    }
    int tot;
    int ex = block_exclusive_scan(s, &tot) + (part ? part[blockIdx.x] : 0);
#pragma unroll
    for (int k = 0; k < kItems; ++k) {
        int64_t i = base + (int64_t)threadIdx.x * kItems + k;
        if (i < n) out[i] = ex;
        ex += v[k];
    }
    if (write_total && blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) {
        out[n] = part ? part[gridDim.x] : tot;
        if (total2) *total2 = out[n];
    }
}

void scan_exclusive_i32(const int32_t* in, int32_t* out, int64_t n, Arena& A,
                        hipStream_t s, int32_t* total2) {
    // out must hold n + 1 entries; out[n] (and *total2 if given) receives
    // the total
    if (n <= 0) {
        HIP_TRY(hipMemsetAsync(out, 0, sizeof(int32_t), s));
        if (total2) HIP_TRY(hipMemsetAsync(total2, 0, sizeof(int32_t), s));
        return;
    }
    int nb = grid_for(n, kTile);
    if (nb == 1) {  // one block: no partial sums needed
        hipLaunchKernelGGL(k_scan_blocks, dim3(1), dim3(kBlock), 0, s, in, n,
                           (const int32_t*)nullptr, out, 1, total2);
        LAUNCH_CHECK();
        return;
    }
    int32_t* part = A.down<int32_t>(nb + 1);
    hipLaunchKernelGGL(k_scan_partials, dim3(nb), dim3(kBlock), 0, s, in, n, part);
    LAUNCH_CHECK();
    hipLaunchKernelGGL(k_scan_sums, dim3(1), dim3(kBlock), 0, s, part, nb);
    LAUNCH_CHECK();
    hipLaunchKernelGGL(k_scan_blocks, dim3(nb), dim3(kBlock), 0, s, in, n, part, out, 1,
                       total2);
    LAUNCH_CHECK();
}

// ---------------------------------------------------------------------
// stable LSD radix sort of (u64 key, i32 value), 8-bit digits
// ---------------------------------------------------------------------
__device__ inline int key_digit(uint64_t k, int shift, int bits) {
    return (int)((k >> shift) & ((1u << bits) - 1u));
}

__global__ void k_radix_hist(const uint64_t* __restrict__ keys, int64_t n,
                             int shift, int bits, int32_t* __restrict__ hist,
                             int nblocks) {
    __shared__ int cnt[256];
    cnt[threadIdx.x] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * kSortTile;
#pragma unroll
    for (int k = 0; k < kSortItems; ++k) {
        int64_t i = base + (int64_t)k * kBlock + threadIdx.x;
        if (i < n) atomicAdd(&cnt[key_digit(keys[i], shift, bits)], 1);
    }
    __syncthreads();
    hist[(int64_t)threadIdx.x * nblocks + blockIdx.x] = cnt[threadIdx.x];
}

// Each wave ranks 4 consecutive runs of 64 elements in order; elements with
// equal digits keep their input order (stable).
__global__ void __launch_bounds__(kBlock)
k_radix_scatter(const uint64_t* __restrict__ kin, const int32_t* __restrict__ vin,
                uint64_t* __restrict__ kout, int32_t* __restrict__ vout,
                int64_t n, int shift, int bits,
                const int32_t* __restrict__ goff, int nblocks) {
    __shared__ int wcount[kBlock / 64][256];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    for (int d = threadIdx.x; d < (kBlock / 64) * 256; d += kBlock)
        (&wcount[0][0])[d] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * kSortTile + (int64_t)w * (64 * kSortItems);
    const uint64_t lt = (lane == 0) ? 0ull : ((~0ull) >> (64 - lane));
    uint64_t key[kSortItems];
    int32_t val[kSortItems];
    int dig[kSortItems], rank[kSortItems];
#pragma unroll
    for (int r = 0; r < kSortItems; ++r) {
        int64_t i = base + (int64_t)r * 64 + lane;
        bool ok = i < n;
        key[r] = ok ? kin[i] : 0ull;
        val[r] = ok ? vin[i] : 0;
        int d = ok ? key_digit(key[r], shift, bits) : 0;
        dig[r] = d;
        uint64_t mask = __ballot(ok);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            uint64_t bal = __ballot((d >> b) & 1);
            mask &= ((d >> b) & 1) ? bal : ~bal;
        }
        int before = wcount[w][d];
        int pre = __popcll(mask & lt);
        rank[r] = before + pre;
        // the lowest lane of each digit group advances the wave's counter
        if (ok && pre == 0) wcount[w][d] = before + __popcll(mask);
        __builtin_amdgcn_wave_barrier();
    }
    __syncthreads();
    // prefix over waves per digit
    {
        int d = threadIdx.x;  // 256 digits, 256 threads
        int acc = 0;
#pragma unroll
        for (int ww = 0; ww < kBlock / 64; ++ww) {
            int c = wcount[ww][d];
            wcount[ww][d] = acc;
            acc += c;
        }
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < kSortItems; ++r) {
        int64_t i = base + (int64_t)r * 64 + lane;
        if (i < n) {
            int d = dig[r];
            int64_t pos = (int64_t)goff[(int64_t)d * nblocks + blockIdx.x] +
                          wcount[w][d] + rank[r];
            kout[pos] = key[r];
            vout[pos] = val[r];
        }
    }
}

void radix_sort_pairs(const uint64_t* keys, const int32_t* vals, uint64_t* keys_out,
                      int32_t* vals_out, int64_t n, int lo_bit, int hi_bit, Arena& A,
                      hipStream_t s) {
    const int passes = hi_bit > lo_bit ? (hi_bit - lo_bit + 7) / 8 : 0;
    if (n <= 1 || passes == 0) {
        if (n > 0 && keys != keys_out) {
            HIP_TRY(hipMemcpyAsync(keys_out, keys, sizeof(uint64_t) * n,
                                   hipMemcpyDeviceToDevice, s));
            HIP_TRY(hipMemcpyAsync(vals_out, vals, sizeof(int32_t) * n,
                                   hipMemcpyDeviceToDevice, s));
        }
        return;
    }
    const int nb = grid_for(n, kSortTile);
    uint64_t* k2 = A.down<uint64_t>(n);
    int32_t* v2 = A.down<int32_t>(n);
    int32_t* hist = A.down<int32_t>((int64_t)256 * nb);
    int32_t* off = A.down<int32_t>((int64_t)256 * nb + 1);
    // ping-pong between the temporary and the output so that the last pass
    // writes the output
    const uint64_t* ki = keys;
    const int32_t* vi = vals;
    for (int pass = 0; pass < passes; ++pass) {
        const int shift = lo_bit + 8 * pass;
        const int bits = std::min(8, hi_bit - shift);
        const bool to_out = ((passes - 1 - pass) & 1) == 0;
        uint64_t* ko = to_out ? keys_out : k2;
        int32_t* vo = to_out ? vals_out : v2;
        hipLaunchKernelGGL(k_radix_hist, dim3(nb), dim3(kBlock), 0, s, ki, n, shift,
                           bits, hist, nb);
        LAUNCH_CHECK();
        scan_exclusive_i32(hist, off, (int64_t)256 * nb, A, s);
        hipLaunchKernelGGL(k_radix_scatter, dim3(nb), dim3(kBlock), 0, s, ki, vi, ko,
                           vo, n, shift, bits, off, nb);
        LAUNCH_CHECK();
        ki = ko;
        vi = vo;
    }
}

// ---------------------------------------------------------------------
// bounding cube and keys (FP64)
// ---------------------------------------------------------------------
__global__ void k_bbox_partial(const double* __restrict__ x, const double* __restrict__ y,
                               const double* __restrict__ z, int64_t n,
                               double* __restrict__ part) {
    double lo[3] = {INFINITY, INFINITY, INFINITY};
    double hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    int nbad = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        double v[3] = {x[i], y[i], z[i]};
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            if (!isfinite(v[a])) {
                ++nbad;
                continue;
            }
            lo[a] = fmin(lo[a], v[a]);
            hi[a] = fmax(hi[a], v[a]);
        }
    }
#pragma unroll
    for (int d = 32; d > 0; d >>= 1) {
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            lo[a] = fmin(lo[a], __shfl_xor(lo[a], d, 64));
            hi[a] = fmax(hi[a], __shfl_xor(hi[a], d, 64));
        }
        nbad += __shfl_xor(nbad, d, 64);
    }
    __shared__ double sl[4][3], sh[4][3];
    __shared__ int sb[4];
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        for (int a = 0; a < 3; ++a) {
            sl[w][a] = lo[a];
            sh[w][a] = hi[a];
        }
        sb[w] = nbad;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        int nb = 0;
        for (int ww = 0; ww < (int)(blockDim.x >> 6); ++ww) {
            for (int a = 0; a < 3; ++a) {
                lo[a] = fmin(lo[a], sl[ww][a]);
                hi[a] = fmax(hi[a], sh[ww][a]);
            }
            nb += sb[ww];
        }
        for (int a = 0; a < 3; ++a) {
            part[blockIdx.x * 8 + a] = lo[a];
            part[blockIdx.x * 8 + 3 + a] = hi[a];
        }
        part[blockIdx.x * 8 + 6] = (double)nb;
    }
}

// Also writes the root cell (all n particles) as cells[0] and flags
// non-finite source coordinates in the status word.
__global__ void k_bbox_final(const double* __restrict__ part, int nparts, int64_t n, Root* root,
                             Cell* __restrict__ cells, int32_t* __restrict__ status) {
#pragma clang fp contract(off)
    // 256 threads: strided partial min/max, then a tree in LDS (min and max
    // are exact, so the order does not matter)
    __shared__ double sm[7][256];
    double lo[3] = {INFINITY, INFINITY, INFINITY};
    double hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    double nbad = 0.0;
    for (int b = threadIdx.x; b < nparts; b += blockDim.x) {
        for (int a = 0; a < 3; ++a) {
            lo[a] = fmin(lo[a], part[b * 8 + a]);
            hi[a] = fmax(hi[a], part[b * 8 + 3 + a]);
        }
        nbad += part[b * 8 + 6];
    }
    for (int a = 0; a < 3; ++a) {
        sm[a][threadIdx.x] = lo[a];
        sm[3 + a][threadIdx.x] = hi[a];
    }
    sm[6][threadIdx.x] = nbad;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            for (int a = 0; a < 3; ++a) {
                sm[a][threadIdx.x] = fmin(sm[a][threadIdx.x], sm[a][threadIdx.x + w]);
                sm[3 + a][threadIdx.x] = fmax(sm[3 + a][threadIdx.x], sm[3 + a][threadIdx.x + w]);
            }
            sm[6][threadIdx.x] += sm[6][threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x != 0) return;
    root->nbad = (int32_t)sm[6][0];
    if (root->nbad) atomicOr(status, (int32_t)ST_SRC_NONFINITE);
    Cell rc;
    rc.first = 0;
    rc.count = (int32_t)n;
    rc.parent = -1;
    rc.child = -1;
    rc.ix = rc.iy = rc.iz = 0;
    rc.level = 0;
    rc.nchild = 0;
    rc.mask = 0;
    cells[0] = rc;
    for (int a = 0; a < 3; ++a) {
        lo[a] = sm[a][0];
        hi[a] = sm[3 + a][0];
    }
    double R = 0.0, c[3];
    for (int a = 0; a < 3; ++a) {
        c[a] = (lo[a] + hi[a]) / 2.0;
        double h = (hi[a] - lo[a]) / 2.0;
        if (h > R) R = h;
    }
    if (!(R > 0.0)) R = 1.0;
    for (int a = 0; a < 3; ++a) root->b[a] = c[a] - R;
    root->R = R;
    root->scale = 2097152.0 / (2.0 * R);
}

__device__ inline uint64_t spread3(uint32_t v) {
    uint64_t x = v & 0x1fffffu;
    x = (x | (x << 32)) & 0x1f00000000ffffull;
    x = (x | (x << 16)) & 0x1f0000ff0000ffull;
    x = (x | (x << 8)) & 0x100f00f00f00f00full;
    x = (x | (x << 4)) & 0x10c30c30c30c30c3ull;
    x = (x | (x << 2)) & 0x1249249249249249ull;
    return x;
}

__device__ inline uint32_t quantise(double v, double b, double s) {
#pragma clang fp contract(off)
    double f = floor((v - b) * s);
    if (!(f >= 0.0)) return 0u;
    if (f > 2097151.0) return 2097151u;
    return (uint32_t)f;
}

// Keys, the identity permutation, and the positions packed as one 32-byte
// record per particle: the gather into key order then reads one record at
// random instead of three coordinates (each a separate cache line).
__global__ void k_keys(const double* __restrict__ x, const double* __restrict__ y,
                       const double* __restrict__ z, int64_t n, const Root* __restrict__ root,
                       uint64_t* __restrict__ keys, int32_t* __restrict__ idx,
                       double4* __restrict__ rec) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double s = root->scale;
    const double a = x[i], b = y[i], c = z[i];
    uint32_t qx = quantise(a, root->b[0], s);
    uint32_t qy = quantise(b, root->b[1], s);
    uint32_t qz = quantise(c, root->b[2], s);
    keys[i] = (spread3(qx) << 2) | (spread3(qy) << 1) | spread3(qz);
    idx[i] = (int32_t)i;
    rec[i] = make_double4(a, b, c, 0.0);
}

// Sorted FP64 positions, and FP32 positions relative to the centre of the
// particle's leaf for the near field: a pair separation is then rounded
// relative to the cell size instead of to |x|.  rec: the positions packed
// by k_keys, in the caller's order.
__global__ void k_gather_positions(const double4* __restrict__ rec, int64_t n,
                                   const int32_t* __restrict__ perm,
                                   const Cell* __restrict__ cells,
                                   const int32_t* __restrict__ leaf_of,
                                   const Root* __restrict__ root, double* __restrict__ xs,
                                   double* __restrict__ ys, double* __restrict__ zs,
                                   float4* __restrict__ p32) {
    int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    const double4 r = rec[perm[s]];
    const double a = r.x, b = r.y, c = r.z;
    xs[s] = a;
    ys[s] = b;
    zs[s] = c;
    double o[3];
    cell_centre(*root, cells[leaf_of[s]], o);
    p32[s] = make_float4((float)(a - o[0]), (float)(b - o[1]), (float)(c - o[2]), 0.0f);
}

// ---------------------------------------------------------------------
// cells, level by level
// ---------------------------------------------------------------------
// Child ranges of the splitting cells of one level, one wave per cell.  The
// seven octant boundaries (first index whose digit is >= o) are narrowed
// together: each round every lane samples one key per boundary inside the
// current bracket, and the ballot of "digit < o" (a prefix, the keys being
// sorted) shrinks the bracket 65-fold; a bracket of <= 64 keys is resolved
// exactly.  The level's cells are [lev[level], lev[level + 1]) (device
// counts, so no host round trip per level; the grid covers a bound).
// bnd[8 c + o - 1] = boundary o, nz[c] = number of nonempty children;
// info[0] |= 1 when the sort did not order the next digit.
__global__ void __launch_bounds__(1024)
k_split_find(const Cell* __restrict__ cells, const int32_t* __restrict__ lev, int level,
             int leaf_max, int sorted_levels, const uint64_t* __restrict__ keys,
             int32_t* __restrict__ nz, int32_t* __restrict__ bnd, int32_t* __restrict__ info) {
    const int lane = threadIdx.x & 63;
    const int c0 = lev[level], c1 = lev[level + 1];
    const int c = c0 + (int)((blockIdx.x * blockDim.x + threadIdx.x) >> 6);
    int nk = 0;
    Cell cell;
    cell.count = 0;
    cell.level = 0;
    if (c < c1) cell = cells[c];
    if (c < c1 && cell.count > leaf_max && cell.level < HFMM_KEY_LEVELS) {
        if (cell.level + 1 > sorted_levels) {
            if (lane == 0) atomicOr(&info[0], 1);
        } else {
            const int shift = 3 * (HFMM_KEY_LEVELS - cell.level - 1);
            const int beg = cell.first, end = cell.first + cell.count;
            int lo[7], hi[7];
#pragma unroll
            for (int o = 0; o < 7; ++o) {
                lo[o] = beg;
                hi[o] = end;
            }
            for (;;) {
                int widest = 0;
#pragma unroll
                for (int o = 0; o < 7; ++o) widest = max(widest, hi[o] - lo[o]);
                if (widest <= 64) break;
                uint32_t dg[7];
#pragma unroll
                for (int o = 0; o < 7; ++o) {
                    const int64_t len = hi[o] - lo[o];
                    const int at = lo[o] + (int)(((int64_t)(lane + 1) * len) / 65);
                    dg[o] = len > 64 ? (uint32_t)(keys[at] >> shift) & 7u : 0u;
                }
#pragma unroll
                for (int o = 0; o < 7; ++o) {
                    const int64_t len = hi[o] - lo[o];
                    if (len <= 64) continue;
                    const int k = __popcll(__ballot(dg[o] < (uint32_t)(o + 1)));
                    const int below = k == 0 ? lo[o] - 1 : lo[o] + (int)(((int64_t)k * len) / 65);
                    const int above = k == 64 ? hi[o] : lo[o] + (int)(((int64_t)(k + 1) * len) / 65);
                    lo[o] = below + 1;
                    hi[o] = above;
                }
            }
            int b[9];
            b[0] = beg;
            b[8] = end;
#pragma unroll
            for (int o = 0; o < 7; ++o) {
                const int at = lo[o] + lane;
                const bool less = at < hi[o] && ((uint32_t)(keys[at] >> shift) & 7u) < (uint32_t)(o + 1);
                b[o + 1] = lo[o] + __popcll(__ballot(less));
            }
#pragma unroll
            for (int o = 0; o < 8; ++o) nk += b[o + 1] > b[o];
#pragma unroll
            for (int o = 0; o < 7; ++o)
                if (lane == o) bnd[(int64_t)(c - c0) * 8 + o] = b[o + 1];
        }
    }
    if (c < c1 && lane == 0) nz[c - c0] = nk;
}

// (cells beyond `cap`, the room reserved from the census, are not written:
// flag = 1 instead)
__global__ void k_split_emit(Cell* __restrict__ cells, const int32_t* __restrict__ lev,
                             int level, const int32_t* __restrict__ bnd,
                             const int32_t* __restrict__ pos, int64_t cap,
                             int32_t* __restrict__ flag) {
    const int c0 = lev[level], c1 = lev[level + 1], next0 = c1;
    int c = c0 + blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= c1) return;
    int k = pos[c - c0];
    int nk = pos[c - c0 + 1] - k;
    if ((int64_t)next0 + k + nk > cap) {
        *flag = 1;
        return;
    }
    if (nk == 0) {
        cells[c].child = -1;
        cells[c].nchild = 0;
        cells[c].mask = 0;
        return;
    }
    const Cell cell = cells[c];
    const int32_t* bc = bnd + (int64_t)(c - c0) * 8;
    int prev = cell.first, out = next0 + k;
    unsigned mask = 0;
    for (int o = 0; o < 8; ++o) {
        const int b = o < 7 ? bc[o] : cell.first + cell.count;
        if (b > prev) {
            Cell ch;
            ch.first = prev;
            ch.count = b - prev;
            ch.parent = c;
            ch.child = -1;
            ch.ix = 2 * cell.ix + ((o >> 2) & 1);
            ch.iy = 2 * cell.iy + ((o >> 1) & 1);
            ch.iz = 2 * cell.iz + (o & 1);
            ch.level = (int16_t)(cell.level + 1);
            ch.nchild = 0;
            ch.mask = 0;
            cells[out++] = ch;
            mask |= 1u << o;
        }
        prev = b;
    }
    cells[c].child = next0 + k;
    cells[c].nchild = (int8_t)nk;
    cells[c].mask = (uint8_t)mask;
}

__global__ void k_leaf_flags(const Cell* __restrict__ cells, int nc, int32_t* __restrict__ f) {
    int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c < nc) f[c] = cells[c].nchild == 0;
}

// leaves in cell order; per sorted particle its leaf cell and leaf index;
// per leaf its box of the self-evaluation (the leaf's own particles)
// (one wave per 64 cells: lane i writes the record of leaf cell 64 w + i,
// then the wave fills the particle range of each of its leaves in turn,
// the lanes over the particles)
__global__ void k_leaf_compact(const Cell* __restrict__ cells, int nc,
                               const int32_t* __restrict__ pos, int32_t* __restrict__ leaves,
                               int32_t* __restrict__ leaf_of, TBox* __restrict__ boxes,
                               int32_t* __restrict__ box_of) {
    const int w = (int)((blockIdx.x * blockDim.x + threadIdx.x) >> 6);
    const int lane = threadIdx.x & 63;
    const int c = w * 64 + lane;
    if (w * 64 >= nc) return;  // uniform per wave
    Cell cell;
    cell.nchild = 1;
    if (c < nc) cell = cells[c];
    const bool leaf = c < nc && cell.nchild == 0;
    const int li = leaf ? pos[c] : 0;
    if (leaf) {
        leaves[li] = c;
        TBox b;
        b.first = cell.first;
        b.count = cell.count;
        b.host = b.leaf = c;
        b.ix = cell.ix;
        b.iy = cell.iy;
        b.iz = cell.iz;
        b.level = cell.level;
        b.kind = 0;
        boxes[li] = b;
    }
    uint64_t todo = __ballot(leaf);
    while (todo) {
        const int j = __ffsll((unsigned long long)todo) - 1;
        todo &= todo - 1;
        const int first = __shfl(cell.first, j, 64), count = __shfl(cell.count, j, 64);
        const int lj = __shfl(li, j, 64), cj = w * 64 + j;
        for (int s = first + lane; s < first + count; s += 64) {
            leaf_of[s] = cj;
            box_of[s] = lj;
        }
    }
}


// Exclusive scan of the children counts of one level's cells, one block
// of 1024 threads looping over the level: pos[0..m] (pos[m] = total), the
// next level's end lev[level + 2] = lev[level + 1] + total, and the level's
// splitting cells in nsplit[level].  m is at most `cap`, the room the
// census gave the level.
__global__ void __launch_bounds__(1024)
k_level_scan(const int32_t* __restrict__ nz, int32_t* __restrict__ lev, int level,
             int32_t* __restrict__ pos, int32_t* __restrict__ nsplit, int cap,
             int32_t* __restrict__ flag) {
    __shared__ int wsum[16];
    __shared__ int carry_s, split_s;
    int m = lev[level + 1] - lev[level];
    if (m > cap) {  // more cells than the census allows: flagged, clamped
        if (threadIdx.x == 0) *flag = 1;
        m = cap;
    }
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (threadIdx.x == 0) {
        carry_s = 0;
        split_s = 0;
    }
    __syncthreads();
    for (int b0 = 0; b0 < m; b0 += 1024) {
        const int i = b0 + (int)threadIdx.x;
        const int v = i < m ? nz[i] : 0;
        int inc = wave_inclusive_scan(v);
        const uint64_t sp = __ballot(v > 0);
        if (lane == 63) wsum[w] = inc;
        __syncthreads();
        int off = carry_s, tot = 0;
        for (int k = 0; k < 16; ++k) {
            if (k < w) off += wsum[k];
            tot += wsum[k];
        }
        if (i < m) pos[i] = off + inc - v;
        __syncthreads();
        if (threadIdx.x == 0) carry_s += tot;
        if (lane == 0 && sp) atomicAdd(&split_s, __popcll(sp));
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        pos[m] = carry_s;
        lev[level + 2] = lev[level + 1] + carry_s;
        nsplit[level] = split_s;
    }
}

// The same scan over several blocks, for levels with many cells (clustered
// data): per tile of kTile counts a partial sum and a split count, one block
// scans the partials, and each tile then scans its counts.  part holds
// 2 (nb + 1) entries: sums, then split counts.
__global__ void k_lscan_part(const int32_t* __restrict__ nz, const int32_t* __restrict__ lev,
                             int level, int cap, int32_t* __restrict__ part, int nb) {
    const int m = min(lev[level + 1] - lev[level], cap);
    const int64_t base = (int64_t)blockIdx.x * kTile;
    int s = 0, c = 0;
#pragma unroll
    for (int k = 0; k < kItems; ++k) {
        const int64_t i = base + (int64_t)threadIdx.x * kItems + k;
        const int v = i < m ? nz[i] : 0;
        s += v;
        c += v > 0;
    }
    int tot, ctot;
    block_exclusive_scan(s, &tot);
    block_exclusive_scan(c, &ctot);
    if (threadIdx.x == 0) {
        part[blockIdx.x] = tot;
        part[nb + 1 + blockIdx.x] = ctot;
    }
}

__global__ void k_lscan_sums(int32_t* __restrict__ part, int nb) {
    int carry = 0, ccarry = 0;
    for (int c0 = 0; c0 < nb; c0 += kBlock) {
        const int i = c0 + threadIdx.x;
        const int v = i < nb ? part[i] : 0;
        const int w = i < nb ? part[nb + 1 + i] : 0;
        int tot, ctot;
        const int ex = block_exclusive_scan(v, &tot);
        block_exclusive_scan(w, &ctot);
        if (i < nb) part[i] = carry + ex;
        carry += tot;
        ccarry += ctot;
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        part[nb] = carry;
        part[2 * nb + 1] = ccarry;
    }
}

__global__ void k_lscan_blocks(const int32_t* __restrict__ nz, int32_t* __restrict__ lev,
                               int level, int cap, const int32_t* __restrict__ part, int nb,
                               int32_t* __restrict__ pos, int32_t* __restrict__ nsplit,
                               int32_t* __restrict__ flag) {
    const int mraw = lev[level + 1] - lev[level];
    const int m = min(mraw, cap);
    const int64_t base = (int64_t)blockIdx.x * kTile;
    int v[kItems];
    int s = 0;
#pragma unroll
    for (int k = 0; k < kItems; ++k) {
        const int64_t i = base + (int64_t)threadIdx.x * kItems + k;
        v[k] = i < m ? nz[i] : 0;
        s += v[k];
    }
    int tot;
    int ex = block_exclusive_scan(s, &tot) + part[blockIdx.x];
#pragma unroll
    for (int k = 0; k < kItems; ++k) {
        const int64_t i = base + (int64_t)threadIdx.x * kItems + k;
        if (i < m) pos[i] = ex;
        ex += v[k];
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        if (mraw > cap) *flag = 1;
        pos[m] = part[nb];
        lev[level + 2] = lev[level + 1] + part[nb];
        nsplit[level] = part[2 * nb + 1];
    }
}

// Census of the splits the tree will make, from the sorted keys alone.  A
// cell of level l splits iff it holds more than leaf_max keys and l < 21,
// i.e. iff some window of leaf_max + 1 consecutive keys shares its l-digit
// prefix.  With w_i the digits keys i and i + leaf_max share (capped at the
// sorted digits) and d_i those keys i - 1 and i share, the window starting
// at i is the first of its level-l run exactly when l <= w_i and
// l > min(w_{i-1}, d_i) (the window at i - 1 would share the prefix
// otherwise), so each i adds 1 to the split count of the levels
// (min(w_{i-1}, d_i), min(w_i, 20)].  Per block (grid-stride over the
// keys) a histogram over levels; part[block * 32 + l].  A window sharing every sorted digit (fewer than 21)
// means the tree needs a deeper sort: part[block * 32 + 31] = 1.
__device__ inline int shared_digits(uint64_t a, uint64_t b, int cap) {
    const uint64_t x = a ^ b;  // 63-bit keys: bit 63 is zero in both
    const int d = x == 0 ? HFMM_KEY_LEVELS : (__clzll((long long)x) - 1) / 3;
    return d < cap ? d : cap;
}

__global__ void __launch_bounds__(256)
k_split_census(const uint64_t* __restrict__ keys, int64_t n, int leaf_max, int sorted_levels,
               int32_t* __restrict__ part) {
    __shared__ int hist[32];
    if (threadIdx.x < 32) hist[threadIdx.x] = 0;
    __syncthreads();
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i + leaf_max < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const uint64_t ki = keys[i];
        const int wi = shared_digits(ki, keys[i + leaf_max], sorted_levels);
        int lo = -1;  // levels above lo are new runs of windows
        if (i > 0) {
            const uint64_t kp = keys[i - 1];
            const int wp = shared_digits(kp, keys[i - 1 + leaf_max], sorted_levels);
            lo = min(wp, shared_digits(kp, ki, sorted_levels));
        }
        const int hi = min(wi, HFMM_KEY_LEVELS - 1);
        for (int l = lo + 1; l <= hi; ++l) atomicAdd(&hist[l], 1);
        if (wi >= sorted_levels && sorted_levels < HFMM_KEY_LEVELS) hist[31] = 1;
    }
    __syncthreads();
    if (threadIdx.x < 32) part[(int64_t)blockIdx.x * 32 + threadIdx.x] = hist[threadIdx.x];
}

// sum of the per-block census rows (the resort flag as a maximum); also
// sets the first level range (the root: lev[0] = 0, lev[1] = 1) and clears
// the level loop's flag
__global__ void k_census_reduce(const int32_t* __restrict__ part, int nblocks,
                                int32_t* __restrict__ census, int32_t* __restrict__ lev,
                                int32_t* __restrict__ flag) {
    if (threadIdx.x == 0) {
        lev[0] = 0;
        lev[1] = 1;
        *flag = 0;
    }
    const int l = threadIdx.x & 31, g = threadIdx.x >> 5;  // 8 groups of 32
    int acc = 0;
#pragma unroll 8
    for (int b = g; b < nblocks; b += 8) {
        const int v = part[(int64_t)b * 32 + l];
        acc = l == 31 ? max(acc, v) : acc + v;
    }
    __shared__ int red[8][32];
    red[g][l] = acc;
    __syncthreads();
    if (g == 0) {
        for (int k = 1; k < 8; ++k) acc = l == 31 ? max(acc, red[k][l]) : acc + red[k][l];
        census[l] = acc;
    }
}

// A kept tree takes new positions: sorted slot s gets the position of its
// particle perm[s] (FP64, and FP32 about its leaf's centre, the mass lane
// kept); *moved = 1 when a particle lies beyond (1/2 + slack) leaf sides of
// its leaf's centre on some axis, or is not finite.
__global__ void k_refit(const double* __restrict__ x, const double* __restrict__ y,
                        const double* __restrict__ z, int64_t n,
                        const int32_t* __restrict__ perm, const Cell* __restrict__ cells,
                        const int32_t* __restrict__ leaf_of, const Root* __restrict__ root,
                        double slack, double* __restrict__ xs, double* __restrict__ ys,
                        double* __restrict__ zs, float4* __restrict__ p32,
                        int32_t* __restrict__ moved, const double4* __restrict__ rec) {
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    const int64_t i = perm[s];
    double a, b, c;
    if (rec) {
        const double4 r = rec[i];
        a = r.x;
        b = r.y;
        c = r.z;
    } else {
        a = x[i];
        b = y[i];
        c = z[i];
    }
    xs[s] = a;
    ys[s] = b;
    zs[s] = c;
    const Root r = *root;
    const Cell cl = cells[leaf_of[s]];
    double o[3];
    cell_centre(r, cl, o);
    float4 q = p32[s];
    q.x = (float)(a - o[0]);
    q.y = (float)(b - o[1]);
    q.z = (float)(c - o[2]);
    p32[s] = q;
    if (!within_cell(r, cl, slack, a, b, c)) *moved = 1;
}

// positions packed as one 32-byte record per particle (caller's order)
__global__ void k_pack_xyz(const double* __restrict__ x, const double* __restrict__ y,
                           const double* __restrict__ z, int64_t n, double4* __restrict__ rec) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) rec[i] = make_double4(x[i], y[i], z[i], 0.0);
}

bool refit_tree(Tree& t, const double* x, const double* y, const double* z, double slack,
                hipStream_t s) {
    Arena& A = t.arena;
    A.release_temps();
    HIP_TRY(hipMemsetAsync(t.moved, 0, sizeof(int32_t), s));
    // with room in the arena the positions are packed first (one record
    // read at random per particle instead of three coordinates)
    double4* rec = nullptr;
    if (A.free_bytes() >= Arena::align(sizeof(double4) * t.n + 1)) {
        rec = A.down<double4>(t.n);
        hipLaunchKernelGGL(k_pack_xyz, dim3(grid_for(t.n, 256)), dim3(256), 0, s, x, y, z, t.n,
                           rec);
        LAUNCH_CHECK();
    }
    hipLaunchKernelGGL(k_refit, dim3(grid_for(t.n, 256)), dim3(256), 0, s, x, y, z, t.n,
                       t.perm, t.cells, t.leaf_of, t.root, slack, t.xs, t.ys, t.zs, t.p32,
                       t.moved, (const double4*)rec);
    LAUNCH_CHECK();
    A.release_temps();
    int32_t h = 1;
    HIP_TRY(hipMemcpyAsync(&h, t.moved, sizeof(h), hipMemcpyDeviceToHost, s));
    stream_wait(s);
    return h == 0;
}

static int sort_levels_guess(int64_t n, int leaf_max) {
    // levels a uniform distribution needs, plus two
    double ratio = (double)n / (double)std::max(1, leaf_max);
    int L = 0;
    while (ratio > 1.0 && L < HFMM_KEY_LEVELS) {
        ratio /= 8.0;
        ++L;
    }
    return std::min(HFMM_KEY_LEVELS, L + 2);
}

void build_tree(Tree& t, const double* x, const double* y, const double* z, hipStream_t s) {
    Arena& A = t.arena;
    const int64_t n = t.n;
    t.status = A.up<int32_t>(1);
    HIP_TRY(hipMemsetAsync(t.status, 0, sizeof(int32_t), s));
    t.moved = A.up<int32_t>(1);
    t.root = A.up<Root>(1);
    t.keys = A.up<uint64_t>(n);
    t.perm = A.up<int32_t>(n);
    t.xs = A.up<double>(n);
    t.ys = A.up<double>(n);
    t.zs = A.up<double>(n);
    t.p32 = A.up<float4>(n);
    t.p64 = A.up<double4>(n);
    t.leaf_of = A.up<int32_t>(n);
    t.leaf_box_of = A.up<int32_t>(n);
    const size_t cells_lo = A.lo;
    t.cells = (Cell*)(A.base + A.lo);
    auto room = [&](int64_t ncell) {
        size_t b = Arena::align((size_t)ncell * sizeof(Cell) + 1);
        if (cells_lo + b > A.hi) A.fail((size_t)ncell * sizeof(Cell));
        A.lo = cells_lo + b;
    };
    room(1);

    // bounding cube (and the root cell)
    const int nbb = (int)std::min<int64_t>(1024, std::max<int64_t>(1, grid_for(n, 256)));
    double* part = A.down<double>((size_t)nbb * 8);
    hipLaunchKernelGGL(k_bbox_partial, dim3(nbb), dim3(256), 0, s, x, y, z, n, part);
    LAUNCH_CHECK();
    hipLaunchKernelGGL(k_bbox_final, dim3(1), dim3(256), 0, s, part, nbb, n, t.root, t.cells,
                       t.status);
    LAUNCH_CHECK();
    // the root is read back with the level-0 counts (non-finite inputs only
    // make meaningless keys until then)
    HIP_TRY(hipMemcpyAsync(&t.root_h, t.root, sizeof(Root), hipMemcpyDeviceToHost, s));

    // keys, sort (top bits first; a full sort if the tree turns out deeper)
    uint64_t* k0 = A.down<uint64_t>(n);
    int32_t* i0 = A.down<int32_t>(n);
    double4* rec = A.down<double4>(n);
    // census: split cells per level (0..20) and the re-sort flag (31)
    int32_t* census = A.down<int32_t>(32);
    // per level: start of the level's cells (lev[l]) and its splitting cells
    // (nsplit[l]), and the level loop's flag: one array, one read back
    constexpr int kLev = HFMM_KEY_LEVELS + 3, kRec = 2 * kLev + 1;
    int32_t* levrec = A.down<int32_t>(kRec);
    int32_t* lev = levrec;
    int32_t* nsplit = levrec + kLev;
    int32_t* flag = levrec + 2 * kLev;
    int sorted_levels = sort_levels_guess(n, t.leaf_max);
    const size_t hi_mark = A.hi;
    int32_t cen_h[32];
    const int ncb = std::min(256, grid_for(n, 256));  // census blocks
    for (int attempt = 0;; ++attempt) {
        if (attempt > 2) throw Status{HFMM_E_STATE};
        if (attempt == 0) {  // (the sort leaves its input keys as they are)
            hipLaunchKernelGGL(k_keys, dim3(grid_for(n, 256)), dim3(256), 0, s, x, y, z, n,
                               t.root, k0, i0, rec);
            LAUNCH_CHECK();
        }
        const int lo_bit = 3 * (HFMM_KEY_LEVELS - sorted_levels);
        radix_sort_pairs(k0, i0, t.keys, t.perm, n, lo_bit, 63, A, s);
        int32_t* part = A.down<int32_t>((size_t)ncb * 32);
        hipLaunchKernelGGL(k_split_census, dim3(ncb), dim3(256), 0, s, t.keys, n, t.leaf_max,
                           sorted_levels, part);
        LAUNCH_CHECK();
        hipLaunchKernelGGL(k_census_reduce, dim3(1), dim3(256), 0, s, part, ncb, census, lev,
                           flag);
        LAUNCH_CHECK();
        // the one read back before the levels (with the root)
        HIP_TRY(hipMemcpyAsync(cen_h, census, sizeof(cen_h), hipMemcpyDeviceToHost, s));
        stream_wait(s);
        A.hi = hi_mark;
        if (t.root_h.nbad) throw Status{HFMM_E_DATA};  // also in the status word
        t.sort_bits = 63 - lo_bit;
        if (cen_h[31]) {  // a cell splits below the sorted digits
            if (sorted_levels >= HFMM_KEY_LEVELS) throw Status{HFMM_E_STATE};
            // six more levels (two more 8-bit passes) first: clustered sets
            // such as a Plummer sphere need a few levels beyond the uniform
            // guess, seldom all 21
            sorted_levels = attempt == 0 ? std::min(HFMM_KEY_LEVELS, sorted_levels + 6)
                                         : HFMM_KEY_LEVELS;
            continue;
        }
        break;
    }
    // levels 0 .. depth - 1 split; a level's cells number at most 8 times
    // the splits of the level above, so every launch is sized on the host
    // while the exact ranges stay on the device
    int depth = 0;
    int64_t splits = 0, bound_max = 1, bound_total = 1;
    for (int l = 0; l < HFMM_KEY_LEVELS; ++l)
        if (cen_h[l] > 0) {
            depth = l + 1;
            splits += cen_h[l];
            bound_max = std::max<int64_t>(bound_max, 8 * (int64_t)cen_h[l]);
            bound_total += 8 * (int64_t)cen_h[l];
        }
    room(bound_total);
    int32_t* nz = A.down<int32_t>(bound_max + 1);
    int32_t* pos = A.down<int32_t>(bound_max + 1);
    int32_t* bnd = A.down<int32_t>((size_t)bound_max * 8);
    int32_t* lpart = A.down<int32_t>(2 * ((size_t)grid_for(bound_max, kTile) + 1));
    for (int l = 0; l < depth; ++l) {
        const int64_t cells_l = l == 0 ? 1 : 8 * (int64_t)cen_h[l - 1];
        hipLaunchKernelGGL(k_split_find, dim3(grid_for(cells_l * 64, 1024)), dim3(1024), 0, s,
                           t.cells, lev, l, t.leaf_max, sorted_levels, t.keys, nz, bnd, flag);
        LAUNCH_CHECK();
        if (cells_l <= 16384) {
            hipLaunchKernelGGL(k_level_scan, dim3(1), dim3(1024), 0, s, nz, lev, l, pos, nsplit,
                               (int)cells_l, flag);
            LAUNCH_CHECK();
        } else {
            const int nb = grid_for(cells_l, kTile);
            hipLaunchKernelGGL(k_lscan_part, dim3(nb), dim3(kBlock), 0, s, nz, lev, l,
                               (int)cells_l, lpart, nb);
            LAUNCH_CHECK();
            hipLaunchKernelGGL(k_lscan_sums, dim3(1), dim3(kBlock), 0, s, lpart, nb);
            LAUNCH_CHECK();
            hipLaunchKernelGGL(k_lscan_blocks, dim3(nb), dim3(kBlock), 0, s, nz, lev, l,
                               (int)cells_l, lpart, nb, pos, nsplit, flag);
            LAUNCH_CHECK();
        }
        hipLaunchKernelGGL(k_split_emit, dim3(grid_for(cells_l, 256)), dim3(256), 0, s, t.cells,
                           lev, l, bnd, pos, bound_total, flag);
        LAUNCH_CHECK();
    }
    // the one read back after the levels: their starts and split counts
    int32_t rec_h[kRec] = {0, 1};
    if (depth > 0) {
        HIP_TRY(hipMemcpyAsync(rec_h, levrec, sizeof(rec_h), hipMemcpyDeviceToHost, s));
        stream_wait(s);
    }
    const int32_t* lev_h = rec_h;
    const int32_t* nsplit_h = rec_h + kLev;
    const int32_t flag_h = rec_h[2 * kLev];
    // the splits the levels made are the census's, level by level
    for (int l = 0; l < depth; ++l)
        if (nsplit_h[l] != cen_h[l]) throw Status{HFMM_E_STATE};
    if (flag_h) throw Status{HFMM_E_STATE};
    t.level_start.assign(lev_h, lev_h + depth + 2);
    t.ncells = lev_h[depth + 1];
    t.depth = depth;
    if (t.ncells > bound_total) throw Status{HFMM_E_STATE};
    room(t.ncells);
    const int64_t nsplit_total = splits;
    // leaves (cells that did not split), in cell order
    t.nleaves = t.ncells - nsplit_total;
    int32_t* f = A.down<int32_t>(t.ncells + 1);
    int32_t* lpos = A.down<int32_t>(t.ncells + 1);
    hipLaunchKernelGGL(k_leaf_flags, dim3(grid_for(t.ncells, 256)), dim3(256), 0, s, t.cells,
                       t.ncells, f);
    LAUNCH_CHECK();
    scan_exclusive_i32(f, lpos, t.ncells, A, s);
    t.leaves = A.up<int32_t>(t.nleaves);
    t.leaf_boxes = A.up<TBox>(t.nleaves);
    hipLaunchKernelGGL(k_leaf_compact, dim3(grid_for((int64_t)grid_for(t.ncells, 64) * 64, 256)), dim3(256), 0, s,
                       t.cells, t.ncells, lpos, t.leaves, t.leaf_of, t.leaf_boxes,
                       t.leaf_box_of);
    LAUNCH_CHECK();
    hipLaunchKernelGGL(k_gather_positions, dim3(grid_for(n, 256)), dim3(256), 0, s, rec, n,
                       t.perm, t.cells, t.leaf_of, t.root, t.xs, t.ys, t.zs, t.p32);
    LAUNCH_CHECK();
    A.release_temps();
}

}  // namespace hfmm
