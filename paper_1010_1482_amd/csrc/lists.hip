// Interaction lists on the device.
//
// FMM lists follow the adaptive scheme the paper cites (Cheng, Greengard and
// Rokhlin; Sec. 6):
//   colleagues(B)  same-level cells adjacent to B (B included): the children
//                  of colleagues(parent(B)) adjacent to B;
//   V(B)           children of colleagues(parent(B)) not adjacent to B (M2L);
//   U(B leaf)      leaves adjacent to B, B included (P2P);
//   W(B leaf)      descendants C of colleagues of B, C not adjacent to B but
//                  parent(C) adjacent to B (M2P);
//   X(B)           leaves C coarser than B, adjacent to parent(B) and not to
//                  B, i.e. the cells with B in W(C) (P2L).
// On a uniform tree these are the 27-cell P2P list of Sec. 5.1 and the
// 189-cell M2L list of Sec. 5.2.  V is stored densely by offset slot: a
// target in octant o of its parent sees its V cells at integer offsets
// d in [-2-o, 3-o]^3 (per axis), 6^3 = 216 slots of which the 27 adjacent
// ones stay empty, so slot -> offset class is the same for all targets of one
// octant; the M2L kernel batches targets of one octant.
//
// Treecode lists follow the Barnes-Hut acceptance of Sec. 4 per target leaf:
// a cell C is accepted when l_C < theta * d, d being the distance from C's
// centre of mass to the target leaf's closed box; C is never accepted when it
// contains the target leaf; a leaf that fails goes to P2P.
//
// The treecode the paper measures (Sec. 4) takes the FMM's lists instead
// (an acceptance of theta = 2/3): for a target leaf B, M2P from V(B), V(A)
// of every ancestor A of B and W(B); P2P with U(B) and X of B and of its
// ancestors (the leaves the FMM reaches through P2L, too close to B's
// particles for their own multipole expansions).
#include "common.hpp"

#include <algorithm>

namespace hfmm {

constexpr int kColl = 27;
constexpr int kSlots = 216;

__device__ inline int octant_of(const Cell& c) {
    return ((c.ix & 1) << 2) | ((c.iy & 1) << 1) | (c.iz & 1);
}

// ---------------------------------------------------------------------
// colleagues, one level at a time (parents first)
// ---------------------------------------------------------------------
// colleagues stored by offset: slot (ex+1)*9 + (ey+1)*3 + (ez+1) holds the
// same-level cell at B + e, or -1.  The cell at B + e is the child of octant
// (B + e) & 1 of the parent-level cell at (B + e) >> 1, which is the parent's
// colleague at offset ((B + e) >> 1) - parent.
// The same rule locates any cell at offset d in [-2, 3]^3 of a child of the
// parent's colleagues (d per axis within [-2 - o, 3 - o], o the octant).
__device__ inline int cell_at_offset(const Cell* __restrict__ cells,
                                     const int32_t* __restrict__ pc, const Cell& B, int dx,
                                     int dy, int dz) {
    const int X = B.ix + dx, Y = B.iy + dy, Z = B.iz + dz;
    if (X < 0 || Y < 0 || Z < 0) return -1;
    const int qx = (X >> 1) - (B.ix >> 1), qy = (Y >> 1) - (B.iy >> 1),
              qz = (Z >> 1) - (B.iz >> 1);
    const int C = pc[(qx + 1) * 9 + (qy + 1) * 3 + (qz + 1)];
    if (C < 0) return -1;
    const Cell cc = cells[C];
    const int o = ((X & 1) << 2) | ((Y & 1) << 1) | (Z & 1);
    if (!((cc.mask >> o) & 1)) return -1;
    return cc.child + __popc((unsigned)cc.mask & ((1u << o) - 1u));
}

// 32 lanes per cell (27 used), cells of one level (parents done before)
__global__ void k_colleagues(const Cell* __restrict__ cells, int c0, int c1,
                             int32_t* __restrict__ coll, uint8_t* __restrict__ cflag) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    const int c = c0 + (e >> 5), q = e & 31;
    const bool ok = c < c1 && q < kColl;
    int res = -1;
    bool leafc = false;
    Cell B;
    if (c < c1) B = cells[c];
    if (ok) {
        const int ex = q / 9 - 1, ey = (q / 3) % 3 - 1, ez = q % 3 - 1;
        if (B.parent < 0)
            res = q == 13 ? c : -1;
        else
            res = cell_at_offset(cells, coll + (int64_t)B.parent * kColl, B, ex, ey, ez);
        coll[(int64_t)c * kColl + q] = res;
        leafc = res >= 0 && cells[res].nchild == 0;
    }
    const uint64_t bl = __ballot(leafc);
    if (c < c1 && q == 0) {
        const uint32_t mine = (uint32_t)(bl >> (threadIdx.x & 32));
        uint8_t f = mine ? 1 : 0;
        if (B.parent >= 0) {
            const uint8_t pf = cflag[B.parent];
            if (pf & 3) f |= 2;
        }
        cflag[c] = f;
    }
}

// V list by slot, two cells per wave.  27 lanes per cell fetch the parent's
// colleagues (child mask and first child) once; each slot then takes the
// entry of its parent-level offset from the owning lane with a shuffle.
// Rows of levels 0 and 1 stay empty; cv[c] = number of entries.
// vcls[c] (0..26) records on which sides of the parent the list has
// sources: per axis 0 = only above, 1 = both sides (or neither), 2 = only
// below, the axes' digits in snake order (consecutive values differ on one
// side of one axis).  Cells with equal values have their sources in the same
// slab of slots: in a uniform tree the value is the position of the parent
// against the faces of the domain, which decides every empty slot.
__global__ void __launch_bounds__(256)
k_vlist(const Cell* __restrict__ cells, int nc, const int32_t* __restrict__ coll,
        int32_t* __restrict__ vsrc, int32_t* __restrict__ cv, uint8_t* __restrict__ vcls,
        uint32_t* __restrict__ vmask) {
    // two cells per wave: the dependent loads of both (cell, its parent's
    // colleagues, their child masks) are in flight together, lanes 32 h ..
    // 32 h + 26 fetching the colleagues of cell 2 w + h
    const int lane = threadIdx.x & 63, half = lane >> 5;
    const int w = (int)((blockIdx.x * blockDim.x + threadIdx.x) >> 6);
    const int cfirst = 2 * w;
    if (cfirst >= nc) return;  // uniform per wave
    const int cmine = cfirst + half;
    Cell Bm;
    Bm.level = 0;
    Bm.parent = -1;
    if (cmine < nc) Bm = cells[cmine];
    int cm = 0, cch = 0;
    if ((lane & 31) < kColl && cmine < nc && Bm.level >= 2) {
        const int C = coll[(int64_t)Bm.parent * kColl + (lane & 31)];
        if (C >= 0) {
            const Cell cc = cells[C];
            cm = cc.mask;
            cch = cc.child;
        }
    }
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int c = cfirst + h;
        if (c >= nc) break;  // uniform
        Cell B;
        B.ix = __shfl(Bm.ix, 32 * h, 64);
        B.iy = __shfl(Bm.iy, 32 * h, 64);
        B.iz = __shfl(Bm.iz, 32 * h, 64);
        B.level = (int16_t)__shfl((int)Bm.level, 32 * h, 64);
        int32_t* out = vsrc + (int64_t)c * kSlots;
        if (B.level < 2) {
            for (int q = lane; q < kSlots; q += 64) out[q] = -1;
            if (lane == 0) {
                cv[c] = 0;
                vcls[c] = 0;
            }
            if (lane < 8) vmask[(int64_t)c * 8 + lane] = 0u;
            continue;
        }
        const int ox = B.ix & 1, oy = B.iy & 1, oz = B.iz & 1;
        int cnt = 0;
        uint32_t sides = 0;  // bit 2a: a source below on axis a, bit 2a + 1: above
        uint64_t occ[4];     // slots with a source, 64 per word
#pragma unroll
        for (int s0 = 0; s0 < kSlots; s0 += 64) {
            const int slot = s0 + lane;
            const int dx = slot / 36 - 2 - ox, dy = (slot / 6) % 6 - 2 - oy,
                      dz = slot % 6 - 2 - oz;
            const int X = B.ix + dx, Y = B.iy + dy, Z = B.iz + dz;
            const bool ok = slot < kSlots && max(abs(dx), max(abs(dy), abs(dz))) > 1 &&
                            X >= 0 && Y >= 0 && Z >= 0;
            const int q = ok ? ((X >> 1) - (B.ix >> 1) + 1) * 9 +
                                   ((Y >> 1) - (B.iy >> 1) + 1) * 3 +
                                   ((Z >> 1) - (B.iz >> 1) + 1)
                             : 0;
            const int m = __shfl(cm, 32 * h + q, 64), ch = __shfl(cch, 32 * h + q, 64);
            const int o = ((X & 1) << 2) | ((Y & 1) << 1) | (Z & 1);
            const int res =
                ok && ((m >> o) & 1) ? ch + __popc((unsigned)m & ((1u << o) - 1u)) : -1;
            if (slot < kSlots) out[slot] = res;
            occ[s0 / 64] = __ballot(res >= 0);
            cnt += __popcll(occ[s0 / 64]);
            if (res >= 0) {
                const int qa[3] = {(X >> 1) - (B.ix >> 1), (Y >> 1) - (B.iy >> 1),
                                   (Z >> 1) - (B.iz >> 1)};
#pragma unroll
                for (int a = 0; a < 3; ++a)
                    sides |= (qa[a] < 0 ? 1u : 0u) << (2 * a) |
                             (qa[a] > 0 ? 1u : 0u) << (2 * a + 1);
            }
        }
        uint32_t all = 0;
#pragma unroll
        for (int b = 0; b < 6; ++b) all |= (__ballot((sides >> b) & 1u) ? 1u : 0u) << b;
        if (lane < 8) {
            const uint64_t o = occ[min(lane >> 1, 3)];
            vmask[(int64_t)c * 8 + lane] = lane < 7 ? (uint32_t)(o >> (32 * (lane & 1))) : 0u;
        }
        if (lane == 0) {
            cv[c] = cnt;
            int d[3];
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                const bool lo = (all >> (2 * a)) & 1u, hi = (all >> (2 * a + 1)) & 1u;
                d[a] = lo == hi ? 1 : (hi ? 0 : 2);
            }
            const int k1 = d[0] * 3 + ((d[0] & 1) ? 2 - d[1] : d[1]);
            vcls[c] = (uint8_t)(k1 * 3 + ((k1 & 1) ? 2 - d[2] : d[2]));
        }
    }
}

// ---------------------------------------------------------------------
// U, W (leaves) and X (level >= 2): count pass (items == nullptr) and fill
// pass over the same traversal
// ---------------------------------------------------------------------
constexpr int kStack = 8 * (HFMM_KEY_LEVELS + 1);

__device__ inline bool is_ancestor_or_self(const Cell& A, const Cell& B) {
    if (A.level > B.level) return false;
    int s = B.level - A.level;
    return (B.ix >> s) == A.ix && (B.iy >> s) == A.iy && (B.iz >> s) == A.iz;
}

// U, W, X of cell b: counted (items == nullptr) or written at the offsets.
// Ancestor chains are walked only when some ancestor has a leaf colleague
// (cflag bit 1).
__device__ inline void uwx_cell(const Cell* __restrict__ cells, int b,
                                const int32_t* __restrict__ coll,
                                const uint8_t* __restrict__ cflag, bool fill,
                                const int32_t* __restrict__ ou, const int32_t* __restrict__ ow,
                                const int32_t* __restrict__ ox, int32_t* __restrict__ iu,
                                int32_t* __restrict__ iw, int32_t* __restrict__ ix, int& nu,
                                int& nw, int& nx) {
    Cell B = cells[b];
    const bool walk = (cflag[b] & 2) != 0;
    int32_t* pu = fill ? iu + ou[b] : nullptr;
    int32_t* pw = fill ? iw + ow[b] : nullptr;
    int32_t* px = fill ? ix + ox[b] : nullptr;
    const bool leaf = B.nchild == 0;
    // X(B): leaves C coarser than B in colleagues of ancestors, adjacent to
    // parent(B) and not to B
    if (B.level >= 2 && walk) {
        Cell P = cells[B.parent];
        for (int A = B.parent; A >= 0; A = cells[A].parent) {
            const int32_t* ca = coll + (int64_t)A * kColl;
            for (int q = 0; q < kColl; ++q) {
                int C = ca[q];
                if (C < 0) continue;
                Cell cc = cells[C];
                if (cc.nchild != 0) continue;
                if (cells_adjacent(cc, P) && !cells_adjacent(cc, B)) {
                    if (fill) px[nx] = C;
                    ++nx;
                }
            }
        }
    }
    if (leaf) {
        // coarser adjacent leaves: leaf colleagues of proper ancestors
        for (int A = walk ? B.parent : -1; A >= 0; A = cells[A].parent) {
            const int32_t* ca = coll + (int64_t)A * kColl;
            for (int q = 0; q < kColl; ++q) {
                int C = ca[q];
                if (C < 0) continue;
                Cell cc = cells[C];
                if (cc.nchild == 0 && cells_adjacent(cc, B)) {
                    if (fill) pu[nu] = C;
                    ++nu;
                }
            }
        }
        // same level, then finer adjacent leaves (U) and W by descent
        const int32_t* cb = coll + (int64_t)b * kColl;
        int stack[kStack];
        for (int q = 0; q < kColl; ++q) {
            int C = cb[q];
            if (C < 0) continue;
            Cell cc = cells[C];
            if (cc.nchild == 0) {
                if (fill) pu[nu] = C;
                ++nu;
                continue;
            }
            if (C == b) continue;
            int sp = 0;
            stack[sp++] = C;
            while (sp > 0) {
                Cell cur = cells[stack[--sp]];
                for (int i = cur.nchild - 1; i >= 0; --i) {
                    int D = cur.child + i;
                    Cell d = cells[D];
                    if (cells_adjacent(d, B)) {
                        if (d.nchild == 0) {
                            if (fill) pu[nu] = D;
                            ++nu;
                        } else if (sp < kStack) {
                            stack[sp++] = D;
                        }
                    } else {
                        if (fill) pw[nw] = D;
                        ++nw;
                    }
                }
            }
        }
    }
}

// Count pass (iu == nullptr): cu, cw, cx per cell (entry nc of these and
// of cv set to 0); fill pass: the items.
__global__ void k_uwx(const Cell* __restrict__ cells, int nc, const int32_t* __restrict__ coll,
                      const uint8_t* __restrict__ cflag, int32_t* __restrict__ cu,
                      int32_t* __restrict__ cw, int32_t* __restrict__ cx,
                      int32_t* __restrict__ cv, int32_t* __restrict__ cf,
                      const int32_t* __restrict__ ou,
                      const int32_t* __restrict__ ow, const int32_t* __restrict__ ox,
                      int32_t* __restrict__ iu, int32_t* __restrict__ iw,
                      int32_t* __restrict__ ix) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    const bool fill = iu != nullptr;
    int nu = 0, nw = 0, nx = 0;
    if (b < nc) uwx_cell(cells, b, coll, cflag, fill, ou, ow, ox, iu, iw, ix, nu, nw, nx);
    if (fill) return;
    if (b <= nc) {  // entry nc is 0: the five arrays are scanned as one
        cu[b] = nu;
        cw[b] = nw;
        cx[b] = nx;
        cf[b] = nx > 0 ? 1 : 0;  // cells with an X list (P2L targets)
        if (b == nc) cv[b] = 0;
    }
}

// list totals from the joint offsets [U | W | X | V | X flags], each nc + 1
// long (the last total: cells with an X list)
__global__ void k_list_totals(const int32_t* __restrict__ off, int nc, int32_t* __restrict__ tot) {
    if (threadIdx.x < 5) {
        const int64_t a = (int64_t)threadIdx.x * (nc + 1);
        tot[threadIdx.x] = off[a + nc] - off[a];
    }
}

// compact array of the cells with an X list, from the scanned flags
__global__ void k_x_cells(const int32_t* __restrict__ foff, int nc, int32_t* __restrict__ xc) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c < nc && foff[c + 1] > foff[c]) xc[foff[c] - foff[0]] = c;
}

// ---------------------------------------------------------------------
// lists of target boxes (separate targets)
// ---------------------------------------------------------------------
// A box without sources is a leaf added to the tree, so its lists follow
// the same definitions as a leaf's.  near: U (+ X for a box without
// sources, whose P2L the FMM cannot hold in an expansion of its own);
// far: W (+ V for a box without sources, by M2P at its targets).  For the
// treecode over the FMM lists (mode != BOX_FMM) near also takes X of the
// box's own leaf (or host) and of every cell above it, and with
// BOX_TREECODE_FULL far takes their V lists too (at p = 3 the far kernel
// reads those from the V table itself).
__device__ void box_lists_one(const Cell* __restrict__ cells, int ncells,
                              const int32_t* __restrict__ coll,
                              const int32_t* __restrict__ vsrc,
                              const int32_t* __restrict__ x_off,
                              const int32_t* __restrict__ x_items, const TBox& bx, int mode,
                              int32_t* pn, int32_t* pf, int& nn, int& nf, bool& over) {
    const Cell B = box_cell(bx);
    const bool src = bx.leaf >= 0;
    const int P = src ? cells[bx.leaf].parent : bx.host;
    // coarser adjacent leaves: leaf colleagues of the cells above the box
    for (int A = P; A >= 0; A = cells[A].parent) {
        const int32_t* ca = coll + (int64_t)A * kColl;
        for (int q = 0; q < kColl; ++q) {
            const int C = ca[q];
            if (C < 0) continue;
            const Cell cc = cells[C];
            if (cc.nchild == 0 && cells_adjacent(cc, B)) {
                if (pn) pn[nn] = C;
                ++nn;
            }
        }
    }
    // colleagues of the box: leaves (U), and below the others finer
    // adjacent leaves (U) and the first non-adjacent cells (W)
    int stack[kStack];
    for (int q = 0; q < kColl; ++q) {
        const int ex = q / 9 - 1, ey = (q / 3) % 3 - 1, ez = q % 3 - 1;
        int C;
        if (P >= 0)
            C = cell_at_offset(cells, coll + (int64_t)P * kColl, B, ex, ey, ez);
        else  // level 0: the root is the only cell
            C = (ncells > 0 && B.ix + ex == 0 && B.iy + ey == 0 && B.iz + ez == 0) ? 0 : -1;
        if (C < 0) continue;
        const Cell cc = cells[C];
        if (cc.nchild == 0) {
            if (pn) pn[nn] = C;
            ++nn;
            continue;
        }
        int sp = 0;
        stack[sp++] = C;
        while (sp > 0) {
            const Cell cur = cells[stack[--sp]];
            for (int i = cur.nchild - 1; i >= 0; --i) {
                const int D = cur.child + i;
                const Cell d = cells[D];
                if (cells_adjacent(d, B)) {
                    if (d.nchild == 0) {
                        if (pn) pn[nn] = D;
                        ++nn;
                    } else if (sp < kStack) {
                        stack[sp++] = D;
                    } else {
                        over = true;
                    }
                } else {
                    if (pf) pf[nf] = D;
                    ++nf;
                }
            }
        }
    }
    if (!src) {
        // V: children of the colleagues of P not adjacent to the box
        // (outside the root: the root when it is not adjacent)
        if (P >= 0) {
            if (B.level >= 2) {
                const int32_t* cp = coll + (int64_t)P * kColl;
                for (int q = 0; q < kColl; ++q) {
                    const int K = cp[q];
                    if (K < 0) continue;
                    const Cell kc = cells[K];
                    for (int i = 0; i < kc.nchild; ++i) {
                        const int D = kc.child + i;
                        if (!cells_adjacent(cells[D], B)) {
                            if (pf) pf[nf] = D;
                            ++nf;
                        }
                    }
                }
            }
        } else if (ncells > 0 && !cells_adjacent(cells[0], B)) {
            if (pf) pf[nf] = 0;
            ++nf;
        }
        // X: leaf colleagues of P and of the cells above it, adjacent to P
        // and not to the box
        if (P >= 0 && B.level >= 2) {
            const Cell Pc = cells[P];
            for (int A = P; A >= 0; A = cells[A].parent) {
                const int32_t* ca = coll + (int64_t)A * kColl;
                for (int q = 0; q < kColl; ++q) {
                    const int C = ca[q];
                    if (C < 0) continue;
                    const Cell cc = cells[C];
                    if (cc.nchild == 0 && cells_adjacent(cc, Pc) && !cells_adjacent(cc, B)) {
                        if (pn) pn[nn] = C;
                        ++nn;
                    }
                }
            }
        }
    }
    if (mode != BOX_FMM) {
        for (int A = src ? bx.leaf : P; A >= 0; A = cells[A].parent) {
            for (int e = x_off[A]; e < x_off[A + 1]; ++e) {
                if (pn) pn[nn] = x_items[e];
                ++nn;
            }
            if (mode == BOX_TREECODE_FULL)
                for (int q = 0; q < kSlots; ++q) {
                    const int v = vsrc[(int64_t)A * kSlots + q];
                    if (v >= 0) {
                        if (pf) pf[nf] = v;
                        ++nf;
                    }
                }
        }
    }
}

// count pass (in == nullptr): cn, cf per box; fill pass: the items
__global__ void k_box_lists(const Cell* __restrict__ cells, int ncells, Targets tg,
                            const int32_t* __restrict__ coll, const int32_t* __restrict__ vsrc,
                            const int32_t* __restrict__ x_off,
                            const int32_t* __restrict__ x_items, int mode,
                            int32_t* __restrict__ cn, int32_t* __restrict__ cf,
                            const int32_t* __restrict__ on, const int32_t* __restrict__ of,
                            int32_t* __restrict__ in, int32_t* __restrict__ inf,
                            int32_t* __restrict__ status) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= tg.nbox) return;
    const TBox bx = tg.box[b];
    int nn = 0, nf = 0;
    bool over = false;
    box_lists_one(cells, ncells, coll, vsrc, x_off, x_items, bx, mode, in ? in + on[b] : nullptr,
                  inf ? inf + of[b] : nullptr, nn, nf, over);
    if (!in) {
        cn[b] = nn;
        cf[b] = nf;
        if (over) atomicOr(status, (int32_t)ST_OVERFLOW);
    }
}

void build_box_lists(Tree& t, const Targets& tg, int mode, hipStream_t s) {
    if (!t.fmm_lists) throw Status{HFMM_E_STATE};
    Arena& A = t.arena;
    const int nb = tg.nbox;
    int32_t* cnt = A.down<int32_t>(2 * (size_t)(nb + 1));
    int32_t *cn = cnt, *cf = cnt + nb + 1;
    hipLaunchKernelGGL(k_box_lists, dim3(grid_for(nb, 64)), dim3(64), 0, s, t.cells, t.ncells,
                       tg, t.coll, t.vsrc, t.x_off, t.x_items, mode, cn, cf, nullptr, nullptr,
                       nullptr, nullptr, t.status);
    LAUNCH_CHECK();
    t.tn_off = A.up<int32_t>(nb + 1);
    t.tf_off = A.up<int32_t>(nb + 1);
    scan_exclusive_i32(cn, t.tn_off, nb, A, s);
    scan_exclusive_i32(cf, t.tf_off, nb, A, s);
    int32_t h[2];
    HIP_TRY(hipMemcpyAsync(&h[0], t.tn_off + nb, 4, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(&h[1], t.tf_off + nb, 4, hipMemcpyDeviceToHost, s));
    stream_wait(s);
    t.tg_near = h[0];
    t.tg_far = h[1];
    t.tn_items = A.up<int32_t>(std::max<int64_t>(t.tg_near, 1));
    t.tf_items = A.up<int32_t>(std::max<int64_t>(t.tg_far, 1));
    hipLaunchKernelGGL(k_box_lists, dim3(grid_for(nb, 64)), dim3(64), 0, s, t.cells, t.ncells,
                       tg, t.coll, t.vsrc, t.x_off, t.x_items, mode, nullptr, nullptr, t.tn_off,
                       t.tf_off, t.tn_items, t.tf_items, t.status);
    LAUNCH_CHECK();
}

// ---------------------------------------------------------------------
// M2L tiles: targets of level >= 2 ordered by (level, octant)
// ---------------------------------------------------------------------
constexpr int kGroups = 8 * (HFMM_KEY_LEVELS + 2);

// keys (level, octant) for the L2L order and (octant, V-list sides) for
// the M2L tiles (the sort keeps the cells' order, level by level, within
// one key), with the counts per (level, octant)
__global__ void k_m2l_keys(const Cell* __restrict__ cells, const uint8_t* __restrict__ vcls,
                           int c0, int nc, uint64_t* __restrict__ keys,
                           uint64_t* __restrict__ keys2, int32_t* __restrict__ vals,
                           int32_t* __restrict__ counts) {
    __shared__ int hist[kGroups];
    for (int k = threadIdx.x; k < kGroups; k += blockDim.x) hist[k] = 0;
    __syncthreads();
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    int c = c0 + i;
    if (c < nc) {
        Cell B = cells[c];
        int k = B.level * 8 + octant_of(B);
        keys[i] = (uint64_t)k;
        keys2[i] = (uint64_t)(octant_of(B) * 27 + vcls[c]);
        vals[i] = c;
        atomicAdd(&hist[k], 1);
    }
    __syncthreads();
    for (int k = threadIdx.x; k < kGroups; k += blockDim.x)
        if (hist[k]) atomicAdd(&counts[k], hist[k]);
}

// Per M2L tile: the slots (of 216) in which some target of the tile has a
// source (the OR of the targets' slot masks, bit j % 32 of word j / 32, 8
// words, 7 used), and the tile's number of work items, max(1, that many
// slots).  One wave per tile.
__global__ void __launch_bounds__(256)
k_tile_masks(const int32_t* __restrict__ tiles, int ntiles, const int32_t* __restrict__ order,
             const uint32_t* __restrict__ vmask, uint32_t* __restrict__ tmask,
             int32_t* __restrict__ items) {
    const int t = (int)((blockIdx.x * blockDim.x + threadIdx.x) >> 6), lane = threadIdx.x & 63;
    if (t >= ntiles) return;  // uniform per wave
    const int start = tiles[4 * t], count = tiles[4 * t + 1];
    uint32_t m[8] = {0u, 0u, 0u, 0u, 0u, 0u, 0u, 0u};
    for (int i = lane; i < count; i += 64) {
        const uint4* r = (const uint4*)(vmask + (int64_t)order[start + i] * 8);
        const uint4 a = r[0], b = r[1];
        m[0] |= a.x, m[1] |= a.y, m[2] |= a.z, m[3] |= a.w;
        m[4] |= b.x, m[5] |= b.y, m[6] |= b.z, m[7] |= b.w;
    }
    int n = 0;
#pragma unroll
    for (int w = 0; w < 8; ++w) {
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) m[w] |= __shfl_xor(m[w], off, 64);
        n += __popc(m[w]);
    }
    if (lane < 8) {
        uint32_t v = m[0];
#pragma unroll
        for (int w = 1; w < 8; ++w)
            if (lane == w) v = m[w];
        tmask[8 * t + lane] = v;
    }
    if (lane == 0) items[t] = max(1, n);
}

void build_fmm_lists(Tree& t, hipStream_t s) {
    if (t.fmm_lists) return;
    Arena& A = t.arena;
    const int nc = t.ncells;
    t.coll = A.up<int32_t>((size_t)nc * kColl);
    t.vsrc = A.up<int32_t>((size_t)nc * kSlots);
    t.cflag = A.up<uint8_t>(nc);
    // read back once: [0..3] U, W, X, V totals, [4] cells with an X list,
    // [5..) group counts
    int32_t* hr = A.down<int32_t>(5 + kGroups);
    HIP_TRY(hipMemsetAsync(hr, 0, sizeof(int32_t) * (5 + kGroups), s));
    for (int l = 0; l <= t.depth; ++l) {
        const int c0 = t.level_start[l], c1 = t.level_start[l + 1];
        hipLaunchKernelGGL(k_colleagues, dim3(grid_for((int64_t)(c1 - c0) * 32, 256)),
                           dim3(256), 0, s, t.cells, c0, c1, t.coll, t.cflag);
        LAUNCH_CHECK();
    }
    // per-cell counts as one array [U | W | X | V | X flag] of 5 (nc + 1),
    // one scan: the offsets of U, W and X index one shared item array (V is
    // stored densely by slot, only its total is used); the flags place the
    // cells with an X list in a compact array
    const int64_t n4 = 5 * (int64_t)(nc + 1);
    int32_t* cnt = A.down<int32_t>(n4);
    int32_t *cu = cnt, *cw = cnt + (nc + 1), *cx = cnt + 2 * (nc + 1), *cv = cnt + 3 * (nc + 1),
            *cf = cnt + 4 * (nc + 1);
    uint8_t* vcls = A.down<uint8_t>(std::max(nc, 1));
    uint32_t* vmask = A.down<uint32_t>((size_t)std::max(nc, 1) * 8);
    hipLaunchKernelGGL(k_vlist, dim3(grid_for((int64_t)(nc + 1) / 2 * 64, 256)), dim3(256), 0,
                       s, t.cells, nc, t.coll, t.vsrc, cv, vcls, vmask);
    LAUNCH_CHECK();
    hipLaunchKernelGGL(k_uwx, dim3(grid_for(nc + 1, 64)), dim3(64), 0, s, t.cells, nc, t.coll,
                       t.cflag, cu, cw, cx, cv, cf, nullptr, nullptr, nullptr, nullptr,
                       nullptr, nullptr);
    LAUNCH_CHECK();
    int32_t* off = A.up<int32_t>(n4 + 1);
    scan_exclusive_i32(cnt, off, n4, A, s);
    hipLaunchKernelGGL(k_list_totals, dim3(1), dim3(64), 0, s, off, nc, hr);
    LAUNCH_CHECK();
    t.u_off = off;
    t.w_off = off + (nc + 1);
    t.x_off = off + 2 * (nc + 1);
    t.v_off = off + 3 * (nc + 1);
    // M2L target order
    const int c2 = t.depth >= 2 ? t.level_start[2] : nc;
    const int nm = nc - c2;
    uint64_t* mk = A.down<uint64_t>(std::max(nm, 1));
    uint64_t* mk2 = A.down<uint64_t>(std::max(nm, 1));
    uint64_t* mk3 = A.down<uint64_t>(std::max(nm, 1));
    int32_t* mv = A.down<int32_t>(std::max(nm, 1));
    t.m2l_order = A.up<int32_t>(std::max(nm, 1));
    t.m2l_torder = A.up<int32_t>(std::max(nm, 1));
    if (nm > 0) {
        hipLaunchKernelGGL(k_m2l_keys, dim3(grid_for(nm, 256)), dim3(256), 0, s, t.cells,
                           vcls, c2, nc, mk, mk3, mv, hr + 5);
        LAUNCH_CHECK();
        radix_sort_pairs(mk, mv, mk2, t.m2l_order, nm, 0, 8, A, s);
        radix_sort_pairs(mk3, mv, mk2, t.m2l_torder, nm, 0, 8, A, s);
    }
    std::vector<int32_t> h(5 + kGroups);
    HIP_TRY(hipMemcpyAsync(h.data(), hr, sizeof(int32_t) * h.size(), hipMemcpyDeviceToHost, s));
    stream_wait(s);
    t.n_u = h[0];
    t.n_w = h[1];
    t.n_x = h[2];
    t.n_v = h[3];
    t.n_xcells = h[4];
    std::vector<int32_t> gc(h.begin() + 5, h.end());
    int32_t* items = A.up<int32_t>(std::max<int64_t>(t.n_u + t.n_w + t.n_x, 1));
    t.u_items = t.w_items = t.x_items = items;
    hipLaunchKernelGGL(k_uwx, dim3(grid_for(nc, 64)), dim3(64), 0, s, t.cells, nc, t.coll,
                       t.cflag, nullptr, nullptr, nullptr, nullptr, nullptr, t.u_off, t.w_off,
                       t.x_off, items, items, items);
    LAUNCH_CHECK();
    t.x_cells = A.up<int32_t>(std::max(t.n_xcells, 1));
    if (t.n_xcells > 0) {
        hipLaunchKernelGGL(k_x_cells, dim3(grid_for(nc, 256)), dim3(256), 0, s, off + 4 * (nc + 1),
                           nc, t.x_cells);
        LAUNCH_CHECK();
    }
    t.m2l_level_start.assign(t.depth + 2, 0);
    for (int l = 0; l <= t.depth; ++l) {
        int acc = t.m2l_level_start[l];
        for (int o = 0; o < 8; ++o) acc += gc[l * 8 + o];
        t.m2l_level_start[l + 1] = acc;
    }
    // M2L tiles: runs of up to 256 targets of one octant, levels mixed (the
    // scaled operators do not depend on the level and every source is read
    // by index), so only the last tile of an octant is partly filled.  Within
    // an octant the targets come by the sides of their V-list sources, so
    // that a tile's targets mostly lack the same slots (a tile skips a slot
    // only when none of its targets has a source there).  Tiles are listed
    // as (k, octant) for the k-th tile of each octant: the eight tiles of one
    // k cover about the same stretch of the order and read nearly the same
    // source expansions.
    std::vector<int32_t>& tiles = t.m2l_tiles_h;
    tiles.clear();
    int ocount[8] = {0}, ostart[9] = {0};
    for (int o = 0; o < 8; ++o)
        for (int l = 0; l <= HFMM_KEY_LEVELS + 1; ++l) ocount[o] += gc[l * 8 + o];
    for (int o = 0; o < 8; ++o) ostart[o + 1] = ostart[o] + ocount[o];
    const int kmax = *std::max_element(ocount, ocount + 8);
    for (int k = 0; k < kmax; k += 256)
        for (int o = 0; o < 8; ++o) {
            if (k >= ocount[o]) continue;
            tiles.push_back(ostart[o] + k);
            tiles.push_back(std::min(256, ocount[o] - k));
            tiles.push_back(o);
            tiles.push_back(0);
        }
    t.n_m2l_tiles = (int32_t)(tiles.size() / 4);
    t.m2l_tiles = A.up<int32_t>(std::max<size_t>(tiles.size(), 4));
    if (!tiles.empty())  // (the host copy lives as long as the tree)
        HIP_TRY(hipMemcpyAsync(t.m2l_tiles, tiles.data(), sizeof(int32_t) * tiles.size(),
                               hipMemcpyHostToDevice, s));
    // the M2L's work items: slot masks of the tiles and their prefix sums
    t.m2l_tmask = A.up<uint32_t>((size_t)std::max(t.n_m2l_tiles, 1) * 8);
    t.m2l_tpre = A.up<int32_t>((size_t)t.n_m2l_tiles + 1);
    if (t.n_m2l_tiles > 0) {
        int32_t* titems = A.down<int32_t>(t.n_m2l_tiles);
        hipLaunchKernelGGL(k_tile_masks, dim3(grid_for((int64_t)t.n_m2l_tiles * 64, 256)),
                           dim3(256), 0, s, t.m2l_tiles, t.n_m2l_tiles, t.m2l_torder, vmask,
                           t.m2l_tmask, titems);
        LAUNCH_CHECK();
        scan_exclusive_i32(titems, t.m2l_tpre, t.n_m2l_tiles, A, s);
    }
    A.release_temps();
    t.fmm_lists = true;
    t.mark_lists = A.lo;
}

// ---------------------------------------------------------------------
// Barnes-Hut group lists (needs the centres of mass in t.cen)
// ---------------------------------------------------------------------
#pragma clang fp contract(off)
__device__ inline double dist_point_box(const double p[3], const double lo[3], double side) {
    double d2 = 0.0;
    for (int a = 0; a < 3; ++a) {
        double hi = lo[a] + side;
        double e = 0.0;
        if (p[a] < lo[a]) e = lo[a] - p[a];
        if (p[a] > hi) e = p[a] - hi;
        d2 += e * e;
    }
    return sqrt(d2);
}
#pragma clang fp contract(on)

// Barnes-Hut lists, one wave per group of target leaves: a depth-first
// traversal from the root with the stack shared by the wave in LDS (up to 64
// nodes are tested per step, opened nodes push their children).  A node containing the
// target leaf is opened (the leaf itself goes to P2P); otherwise it is
// accepted (M2P) when side < theta * distance(centre of mass, leaf box),
// else a leaf goes to P2P and an inner node is opened.  Item order within a list is
// free (sums over a list are order-insensitive up to rounding).  When a push
// would overflow the LDS stack, each lane finishes its own node's subtree
// with a private stack (counted, then written at scanned offsets).  The
// traversal is bound by the latency of its dependent steps, so the stack is
// sized for occupancy: 1024 entries (5 KB per wave) let 7 blocks share a CU
// (2048: 3 blocks, 9.4 -> 8.1 ms at N = 2^22 Plummer); at 512 the private
// stacks take over and it runs 5x slower.
constexpr int kBhCap = 1024;

// 0: open, 1: accept (M2P), 2: P2P
__device__ __forceinline__ int bh_class(const Cell& cc, int C, const Cell& B, int b,
                                        const Root& r, const double4* __restrict__ cen,
                                        const double lo[3], double hb, double theta) {
#pragma clang fp contract(off)
    if (is_ancestor_or_self(cc, B)) return C == b ? 2 : 0;
    const double4 q = cen[C];
    const double pc[3] = {q.x, q.y, q.z};
    const double d = dist_point_box(pc, lo, hb);
    if (cell_side(r, cc.level) < theta * d) return 1;
    return cc.nchild == 0 ? 2 : 0;
}

// subtree of an opened node C0 with a private stack: counts (or writes);
// returns true when the stack overflowed (entries were dropped)
__device__ inline bool bh_subtree(const Cell* __restrict__ cells, int C0, const Cell& B, int b,
                                  const Root& r, const double4* __restrict__ cen,
                                  const double lo[3], double hb, double theta, int32_t* pa,
                                  int32_t* pb, int& na, int& np) {
    int stack[kStack];
    int sp = 0;
    bool over = false;
    const Cell c0 = cells[C0];
    for (int i = c0.nchild - 1; i >= 0; --i) {
        if (sp < kStack)
            stack[sp++] = c0.child + i;
        else
            over = true;
    }
    while (sp > 0) {
        const int C = stack[--sp];
        const Cell cc = cells[C];
        const int k = bh_class(cc, C, B, b, r, cen, lo, hb, theta);
        if (k == 1) {
            if (pa) pa[na] = C;
            ++na;
        } else if (k == 2) {
            if (pb) pb[np] = C;
            ++np;
        } else {
            for (int i = cc.nchild - 1; i >= 0; --i) {
                if (sp < kStack)
                    stack[sp++] = cc.child + i;
                else
                    over = true;
            }
        }
    }
    return over;
}

// Sibling boxes (the target boxes under one cell, at most 8) are traversed
// together by one wave: a stack entry carries a node and the set of the
// group's boxes for which it is visited (all its ancestors opened for
// them).  Each box's lists are exactly those of its own traversal; the tree
// is read once per group instead of once per box.  A box's own leaf (a
// leaf of the tree) goes to P2P; a box outside the root has no ancestor.
constexpr int kBhGroup = 8;

// the cell above a box (-1 for the root leaf and for boxes outside the root)
__device__ __forceinline__ int box_parent(const Cell* __restrict__ cells, const TBox& b) {
    return b.leaf >= 0 ? cells[b.leaf].parent : b.host;
}

__global__ void __launch_bounds__(256)
k_bh_group(const Cell* __restrict__ cells, Targets tg, const int32_t* __restrict__ gstart,
           const int32_t* __restrict__ ngroups, const Root* __restrict__ root,
           const double4* __restrict__ cen, double theta, int32_t* __restrict__ ca,
           int32_t* __restrict__ cb, const int32_t* __restrict__ oa,
           const int32_t* __restrict__ ob, int32_t* __restrict__ ia, int32_t* __restrict__ ib,
           int32_t* __restrict__ status) {
#pragma clang fp contract(off)
    __shared__ int stk[4][kBhCap];
    __shared__ uint8_t msk[4][kBhCap];
    // per wave: the group's boxes, their corners, own leaves and list offsets
    __shared__ double glo[4][kBhGroup][3];
    __shared__ int gbl[4][kBhGroup], grow[4][kBhGroup], goa[4][kBhGroup], gob[4][kBhGroup];
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int gi = blockIdx.x * 4 + w;
    if (gi >= *ngroups) return;  // uniform per wave; no block-wide barrier below
    const bool fill = ia != nullptr;
    const int l0 = gstart[gi], nl = gstart[gi + 1] - l0;
    const Root r = *root;
    const TBox B0 = tg.box[l0];
    const int lv = B0.level;
    const double hb = cell_side(r, lv);
    if (lane < nl) {
        const TBox Bi = tg.box[l0 + lane];
        const int row = list_row(tg, l0 + lane, Bi);
        gbl[w][lane] = Bi.leaf;
        grow[w][lane] = row;
        glo[w][lane][0] = r.b[0] + (double)Bi.ix * hb;
        glo[w][lane][1] = r.b[1] + (double)Bi.iy * hb;
        glo[w][lane][2] = r.b[2] + (double)Bi.iz * hb;
        goa[w][lane] = fill ? oa[row] : 0;
        gob[w][lane] = fill ? ob[row] : 0;
    }
    int na[kBhGroup], np[kBhGroup];
#pragma unroll
    for (int i = 0; i < kBhGroup; ++i) na[i] = np[i] = 0;
    // the common parent contains every box of the group (none outside the
    // root or for the root leaf)
    const int pid = box_parent(cells, B0);
    Cell P;
    if (pid >= 0) P = cells[pid];
    const uint32_t all = (1u << nl) - 1u;
    int* st = stk[w];
    uint8_t* sm = msk[w];
    int sp = 1;
    if (lane == 0) {
        st[0] = 0;
        sm[0] = (uint8_t)all;
    }
    wave_lds_fence();
    bool overflow = false;
    while (sp > 0) {
        const int k = min(sp, 64), base = sp - k;
        const int C = lane < k ? st[base + lane] : -1;
        const uint32_t m = lane < k ? sm[base + lane] : 0u;
        wave_lds_fence();
        sp = base;
        uint32_t am = 0u, pm = 0u, om = 0u;
        int nch = 0, child = 0;
        if (C >= 0) {
            const Cell cc = cells[C];
            if (pid >= 0 && cc.level < lv && is_ancestor_or_self(cc, P)) {
                om = m;  // contains every box of the group
            } else {
                const double4 q = cen[C];
                const double pc[3] = {q.x, q.y, q.z};
                const double side = cell_side(r, cc.level);
#pragma unroll 1
                for (int i = 0; i < nl; ++i) {
                    if (!((m >> i) & 1u)) continue;
                    if (C == gbl[w][i]) {
                        pm |= 1u << i;  // the box's own leaf
                    } else if (side < theta * dist_point_box(pc, glo[w][i], hb)) {
                        am |= 1u << i;
                    } else if (cc.nchild == 0) {
                        pm |= 1u << i;
                    } else {
                        om |= 1u << i;
                    }
                }
            }
            if (om) {
                nch = cc.nchild;
                child = cc.child;
            }
        }
        const uint64_t lt = lanes_below(lane);
#pragma unroll
        for (int i = 0; i < kBhGroup; ++i) {
            if (i >= nl) break;
            const bool a = (am >> i) & 1u, pp = (pm >> i) & 1u;
            const uint64_t ab = __ballot(a), pb = __ballot(pp);
            if (fill && a) ia[goa[w][i] + na[i] + __popcll(ab & lt)] = C;
            if (fill && pp) ib[gob[w][i] + np[i] + __popcll(pb & lt)] = C;
            na[i] += __popcll(ab);
            np[i] += __popcll(pb);
        }
        int total;
        const int off = wave_excl_scan(nch, lane, total);
        if (sp + total <= kBhCap) {
            for (int c = 0; c < nch; ++c) {
                st[sp + off + c] = child + c;
                sm[sp + off + c] = (uint8_t)om;
            }
            sp += total;
        } else {
            // stack full: every lane finishes the subtree of its opened node,
            // box by box, with a private stack
#pragma unroll
            for (int i = 0; i < kBhGroup; ++i) {
                if (i >= nl) break;
                const TBox Bi = tg.box[l0 + i];
                const Cell Bc = box_cell(Bi);
                int ka = 0, kp = 0;
                const bool mine = (om >> i) & 1u;
                if (mine)
                    overflow |= bh_subtree(cells, C, Bc, gbl[w][i], r, cen, glo[w][i], hb,
                                           theta, nullptr, nullptr, ka, kp);
                int ta, tp;
                const int oa_l = wave_excl_scan(ka, lane, ta);
                const int ob_l = wave_excl_scan(kp, lane, tp);
                if (fill && mine) {
                    int xa = 0, xp = 0;
                    bh_subtree(cells, C, Bc, gbl[w][i], r, cen, glo[w][i], hb, theta,
                               ia + goa[w][i] + na[i] + oa_l, ib + gob[w][i] + np[i] + ob_l, xa,
                               xp);
                }
                na[i] += ta;
                np[i] += tp;
            }
        }
        wave_lds_fence();
    }
    if (status && __ballot(overflow)) {
        if (lane == 0) atomicOr(status, (int32_t)ST_OVERFLOW);
    }
    if (!fill) {
#pragma unroll
        for (int i = 0; i < kBhGroup; ++i)
            if (i < nl && lane == i) {
                ca[grow[w][i]] = na[i];
                cb[grow[w][i]] = np[i];
            }
    }
}

// groups of sibling boxes: a flag where a box's parent differs from the
// previous box's (sibling boxes are adjacent in box order); boxes outside
// the root each form their own group
__global__ void k_bh_group_flags(const Cell* __restrict__ cells, Targets tg,
                                 int32_t* __restrict__ flag) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= tg.nbox) return;
    const int pi = box_parent(cells, tg.box[i]);
    flag[i] = (i == 0 || pi < 0 || pi != box_parent(cells, tg.box[i - 1])) ? 1 : 0;
}

__global__ void k_bh_group_starts(const int32_t* __restrict__ flag,
                                  const int32_t* __restrict__ gidx, int nleaves,
                                  int32_t* __restrict__ gstart) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nleaves) return;
    if (flag[i]) gstart[gidx[i]] = i;
    if (i == nleaves - 1) gstart[gidx[nleaves]] = nleaves;
}

// Barnes-Hut lists of the boxes of tg into rows of nrows (+1) offsets:
// counts, scan, one read-back of the totals, fill
static void bh_lists_rows(Tree& t, const Targets& tg, double theta, int nrows, int32_t*& a_off,
                          int32_t*& b_off, int32_t*& a_items, int32_t*& b_items, int64_t& n_a,
                          int64_t& n_b, hipStream_t s) {
    Arena& A = t.arena;
    int32_t* cnt = A.down<int32_t>(2 * (size_t)(nrows + 1));
    int32_t *ca = cnt, *cb = cnt + nrows + 1;
    HIP_TRY(hipMemsetAsync(cnt, 0, sizeof(int32_t) * 2 * (nrows + 1), s));
    // sibling groups (at most 8 boxes each); the launches cover one wave
    // per box, the waves past the group count exit
    const int nb = tg.nbox;
    int32_t* gflag = A.down<int32_t>(nb);
    int32_t* gidx = A.down<int32_t>(nb + 1);
    int32_t* gstart = A.down<int32_t>(nb + 1);
    hipLaunchKernelGGL(k_bh_group_flags, dim3(grid_for(nb, 256)), dim3(256), 0, s, t.cells, tg,
                       gflag);
    LAUNCH_CHECK();
    scan_exclusive_i32(gflag, gidx, nb, A, s);
    hipLaunchKernelGGL(k_bh_group_starts, dim3(grid_for(nb, 256)), dim3(256), 0, s, gflag,
                       gidx, nb, gstart);
    LAUNCH_CHECK();
    const int32_t* ngroups = gidx + nb;
    hipLaunchKernelGGL(k_bh_group, dim3(grid_for(nb, 4)), dim3(256), 0, s, t.cells, tg, gstart,
                       ngroups, t.root, (const double4*)t.cen, theta, ca, cb, nullptr, nullptr,
                       nullptr, nullptr, t.status);
    LAUNCH_CHECK();
    a_off = A.up<int32_t>(nrows + 1);
    b_off = A.up<int32_t>(nrows + 1);
    scan_exclusive_i32(ca, a_off, nrows, A, s);
    scan_exclusive_i32(cb, b_off, nrows, A, s);
    int32_t h[2];
    HIP_TRY(hipMemcpyAsync(&h[0], a_off + nrows, 4, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(&h[1], b_off + nrows, 4, hipMemcpyDeviceToHost, s));
    stream_wait(s);
    n_a = h[0];
    n_b = h[1];
    a_items = A.up<int32_t>(std::max<int64_t>(n_a, 1));
    b_items = A.up<int32_t>(std::max<int64_t>(n_b, 1));
    hipLaunchKernelGGL(k_bh_group, dim3(grid_for(nb, 4)), dim3(256), 0, s, t.cells, tg, gstart,
                       ngroups, t.root, (const double4*)t.cen, theta, nullptr, nullptr, a_off,
                       b_off, a_items, b_items, nullptr);
    LAUNCH_CHECK();
}

void build_bh_lists(Tree& t, double theta, hipStream_t s) {
    Arena& A = t.arena;
    if (t.bh_theta == theta && t.a_off) {
        A.lo = t.mark_bh;
        return;
    }
    A.lo = t.mark_up;  // lists live above the upward data
    t.fmm_lists = false;
    bh_lists_rows(t, self_targets(t), theta, t.ncells, t.a_off, t.b_off, t.a_items, t.b_items,
                  t.n_a, t.n_b, s);
    A.release_temps();
    t.bh_theta = theta;
    t.mark_bh = A.lo;
}

// Barnes-Hut lists of separate target boxes (rows by box), above the
// current arena mark
void build_bh_box_lists(Tree& t, const Targets& tg, double theta, hipStream_t s) {
    bh_lists_rows(t, tg, theta, tg.nbox, t.tf_off, t.tn_off, t.tf_items, t.tn_items, t.tg_far,
                  t.tg_near, s);
}

// ---------------------------------------------------------------------
// Treecode lists from the FMM lists (the treecode of Sec. 4)
// ---------------------------------------------------------------------
// per leaf B: M2P count |W(B)| + sum over A in {B, ancestors} of |V(A)|,
// P2P count |U(B)| + sum over the same A of |X(A)|; tot[0..1] receive the
// 64-bit totals (one atomic per block), so that the host can refuse lists
// whose int32 offsets would overflow
__global__ void __launch_bounds__(256)
k_tl_count(const Cell* __restrict__ cells, const int32_t* __restrict__ leaves, int nleaves,
           const int32_t* __restrict__ u_off, const int32_t* __restrict__ w_off,
           const int32_t* __restrict__ x_off, const int32_t* __restrict__ v_off,
           int32_t* __restrict__ ca, int32_t* __restrict__ cb,
           unsigned long long* __restrict__ tot) {
    __shared__ int sa[4], sb[4];
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    int na = 0, nb = 0;
    if (i < nleaves) {
        const int b = leaves[i];
        na = w_off[b + 1] - w_off[b];
        nb = u_off[b + 1] - u_off[b];
        for (int a = b; a >= 0; a = cells[a].parent) {
            na += v_off[a + 1] - v_off[a];
            nb += x_off[a + 1] - x_off[a];
        }
        ca[b] = na;
        cb[b] = nb;
    }
    for (int d = 32; d > 0; d >>= 1) {
        na += __shfl_xor(na, d, 64);
        nb += __shfl_xor(nb, d, 64);
    }
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        sa[w] = na;
        sb[w] = nb;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        atomicAdd(&tot[0], (unsigned long long)((int64_t)sa[0] + sa[1] + sa[2] + sa[3]));
        atomicAdd(&tot[1], (unsigned long long)((int64_t)sb[0] + sb[1] + sb[2] + sb[3]));
    }
}

// a run of list items copied by the wave's lanes
__device__ __forceinline__ int wave_copy(const int32_t* __restrict__ src, int e0, int e1,
                                         int32_t* __restrict__ dst, int at, int lane) {
    for (int e = e0 + lane; e < e1; e += 64) dst[at + e - e0] = src[e];
    return at + (e1 - e0);
}

// one wave per leaf: the M2P items in the order W(B), then V(A) slot by slot
// from B up to the root; the P2P items U(B), then X(A) from B up (either
// output may be null, uniformly)
__global__ void __launch_bounds__(256)
k_tl_fill(const Cell* __restrict__ cells, const int32_t* __restrict__ leaves, int nleaves,
          const int32_t* __restrict__ vsrc, const int32_t* __restrict__ u_off,
          const int32_t* __restrict__ w_off, const int32_t* __restrict__ x_off,
          const int32_t* __restrict__ items, const int32_t* __restrict__ a_off,
          const int32_t* __restrict__ b_off, int32_t* __restrict__ a_items,
          int32_t* __restrict__ b_items) {
    const int li = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
    if (li >= nleaves) return;
    const int b = leaves[li];
    const uint64_t below = lanes_below(lane);
    if (a_items) {
        int fa = wave_copy(items, w_off[b], w_off[b + 1], a_items, a_off[b], lane);
        for (int a = b; a >= 0; a = cells[a].parent)
            for (int q0 = 0; q0 < kSlots; q0 += 64) {
                const int q = q0 + lane;
                const int v = q < kSlots ? vsrc[(int64_t)a * kSlots + q] : -1;
                const uint64_t bal = __ballot(v >= 0);
                if (v >= 0) a_items[fa + __popcll(bal & below)] = v;
                fa += __popcll(bal);
            }
    }
    if (b_items) {
        int fb = wave_copy(items, u_off[b], u_off[b + 1], b_items, b_off[b], lane);
        for (int a = b; a >= 0; a = cells[a].parent)
            fb = wave_copy(items, x_off[a], x_off[a + 1], b_items, fb, lane);
    }
}

// fill_far: also write the M2P items (the p = 3 far field reads V and W
// directly and needs only their offsets, for the statistics)
void build_fmmlist_treecode_lists(Tree& t, bool fill_far, hipStream_t s) {
    Arena& A = t.arena;
    if (t.a_off && t.bh_theta == kFmmListTheta && (t.a_items || !fill_far)) {
        A.lo = t.mark_bh;
        return;
    }
    if (!t.fmm_lists) throw Status{HFMM_E_STATE};
    A.lo = t.mark_up;  // above the FMM lists and the upward data
    const int nc = t.ncells, nlv = t.nleaves;
    int32_t* cnt = A.down<int32_t>(2 * (size_t)(nc + 1));
    int32_t *ca = cnt, *cb = cnt + nc + 1;
    unsigned long long* tot = A.down<unsigned long long>(2);
    HIP_TRY(hipMemsetAsync(cnt, 0, sizeof(int32_t) * 2 * (nc + 1), s));
    HIP_TRY(hipMemsetAsync(tot, 0, 2 * sizeof(unsigned long long), s));
    hipLaunchKernelGGL(k_tl_count, dim3(grid_for(nlv, 256)), dim3(256), 0, s, t.cells, t.leaves,
                       nlv, t.u_off, t.w_off, t.x_off, t.v_off, ca, cb, tot);
    LAUNCH_CHECK();
    unsigned long long h[2];
    HIP_TRY(hipMemcpyAsync(h, tot, sizeof(h), hipMemcpyDeviceToHost, s));
    stream_wait(s);
    if (h[0] > (unsigned long long)INT32_MAX || h[1] > (unsigned long long)INT32_MAX)
        throw Status{HFMM_E_UNSUPPORTED};  // list offsets are int32
    t.n_a = (int64_t)h[0];
    t.n_b = (int64_t)h[1];
    t.a_off = A.up<int32_t>(nc + 1);
    t.b_off = A.up<int32_t>(nc + 1);
    scan_exclusive_i32(ca, t.a_off, nc, A, s);
    scan_exclusive_i32(cb, t.b_off, nc, A, s);
    t.a_items = fill_far ? A.up<int32_t>(std::max<int64_t>(t.n_a, 1)) : nullptr;
    t.b_items = A.up<int32_t>(std::max<int64_t>(t.n_b, 1));
    hipLaunchKernelGGL(k_tl_fill, dim3(grid_for(nlv, 4)), dim3(256), 0, s, t.cells, t.leaves,
                       nlv, t.vsrc, t.u_off, t.w_off, t.x_off, t.u_items, t.a_off, t.b_off,
                       t.a_items, t.b_items);
    LAUNCH_CHECK();
    A.release_temps();
    t.bh_theta = kFmmListTheta;
    t.mark_bh = A.lo;
}

// the M2P items of the lists above written to dst (n_a entries, device)
void fill_fmmlist_far_items(const Tree& t, int32_t* dst, hipStream_t s) {
    hipLaunchKernelGGL(k_tl_fill, dim3(grid_for(t.nleaves, 4)), dim3(256), 0, s, t.cells,
                       t.leaves, t.nleaves, t.vsrc, t.u_off, t.w_off, t.x_off, t.u_items,
                       t.a_off, t.b_off, dst, nullptr);
    LAUNCH_CHECK();
}

}  // namespace hfmm
