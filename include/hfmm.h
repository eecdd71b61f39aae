/*
 * hfmm: treecode and fast multipole method for the Laplace / gravitational
 * N-body problem on AMD Instinct MI355X (gfx950).
 *
 * The library evaluates, for every target particle i,
 *     phi_i = sum_j m_j / r_ij          a_i = sum_j m_j (x_j - x_i) / r_ij^3
 * (Eq. 1 of Yokota & Barba, "Treecode and fast multipole method for N-body
 * simulation with CUDA", taken per unit target mass with the sign of the
 * single-pair kernel of Sec. 5.1: a_i is the gradient of phi_i).  Pairs at
 * zero separation are skipped.  eps2 is added to r^2 as in the P2P kernel of
 * Sec. 5.1, in the pairs summed directly (P2P, and every pair of
 * HFMM_DIRECT) only: the far field (M2L, L2L, L2P, M2P, P2L) is the
 * expansion of the unsoftened 1/r.
 *
 * Methods (Sec. 2, Fig. 1):
 *   HFMM_DIRECT    all pairs (the P2P kernel of Sec. 5.1 over one source set)
 *   HFMM_TREECODE  Barnes-Hut: P2M, M2M, M2P under the acceptance criterion
 *                  l < theta * d of Sec. 4 (d from the cell's centre of mass to
 *                  the target leaf), P2P for the rest
 *   HFMM_FMM       P2M, M2M, M2L (Eq. 4), L2L, L2P and P2P over the adaptive
 *                  U/V/W/X lists (Sec. 6 cites Cheng, Greengard and Rokhlin);
 *                  on uniform data these are the 27-cell P2P and 189-cell M2L
 *                  lists of Secs. 5.1 and 5.2
 *   HFMM_FMM_ROT   the FMM with the rotation-based M2L Sec. 6 names among
 *                  the advanced techniques: each multipole expansion rotated
 *                  to the axis of its translation, translated along it
 *                  (order by order, O(p^3)) and rotated back; the same
 *                  result as HFMM_FMM up to rounding (FP64 or FP32 only).
 *                  HFMM_FMM itself takes this M2L where the matrix cores
 *                  hold no dense operator (FP32 above p = 13, FP64 above
 *                  p = 11)
 *   HFMM_TREECODE_FMMLIST
 *                  the treecode the paper measures (Sec. 4): the FMM's upward
 *                  pass (geometric centres) and lists, with M2P at the targets
 *                  in place of M2L + L2L + L2P: M2P from V of the target leaf
 *                  and of its ancestors and from W of the leaf, P2P with U of
 *                  the leaf and X of the leaf and its ancestors (an acceptance
 *                  of theta = 2/3; theta is not used)
 * p is the number of expansion terms: degrees n = 0..p-1 (Eq. 4).
 *
 * Targets.  A tree is built over the sources only.  An evaluation is at the
 * sources themselves (tx == NULL) or at separate target points, each binned
 * into the resident tree: its key is followed down the tree to a leaf (the
 * target is evaluated as that leaf's particles are), to an empty octant of
 * a split cell (a source-free leaf added to the tree: L2P of the split
 * cell's local expansion, M2P over the octant's V and W lists and P2P over
 * its U and X lists, the adaptive lists of Cheng, Greengard and Rokhlin that
 * Sec. 6 cites), or it lies outside the root cube (a root-sized cube of the
 * extended grid, no local expansion).  One tree may be evaluated at any
 * number of target sets.
 *
 * Memory and streams.  Every pointer argument named x, y, z, tx, ty, tz, m,
 * phi, ax, ay, az, arena, off, items or dst is a DEVICE pointer.  The caller
 * allocates all device memory: inputs, outputs and one arena per tree; the
 * library never allocates device memory.  Every call enqueues its work on
 * `stream` (a hipStream_t passed as void*); build and evaluate also
 * synchronise that stream for small size read-backs, other streams are
 * never touched.  A tree handle is used by one stream at a time; different
 * handles are independent and may run concurrently on different streams.
 *
 * Layouts.  Inputs are FP64 structure-of-arrays in the caller's order.
 * Outputs are structure-of-arrays in the caller's order, FP64 when precision
 * is HFMM_FP64 and FP32 otherwise.
 *
 * Errors.  Every function returns HFMM_OK (0) or a negative hfmm_status.  No
 * function aborts or throws.  Argument errors are reported at the call;
 * HFMM_E_NOMEM means the arena is too small and hfmm_required_bytes() then
 * gives a size that is enough for the work done so far (retry with at least
 * that much).  HIP runtime failures return HFMM_E_HIP.  Errors in the data
 * (non-finite coordinates or masses, an overflowing traversal) are found by
 * the kernels and kept in the tree's device status word, read with
 * hfmm_status(); the build also returns HFMM_E_DATA for non-finite source
 * coordinates, and hfmm_solve reads the status word before it returns.
 */
#ifndef HFMM_H
#define HFMM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct hfmm_tree_s* hfmm_tree;

enum hfmm_method {
    HFMM_DIRECT = 0,
    HFMM_TREECODE = 1,
    HFMM_FMM = 2,
    HFMM_TREECODE_FMMLIST = 3,
    HFMM_FMM_ROT = 4
};

/* Arithmetic of the far field.  P2P, P2M, L2P, M2P run in FP32 for every
 * precision but HFMM_FP64, and P2L forms its terms in FP32 there (summed in
 * FP64); M2M and L2L always run in FP64; the M2L variants differ only in the
 * multipole-to-local product:
 *   HFMM_FP32        FP32 matrix-core products
 *   HFMM_M2L_BF16    BF16 operands, FP32 accumulation
 *   HFMM_M2L_BF16X3  BF16 hi/lo split: hi*hi + hi*lo + lo*hi, FP32 accumulation
 *   HFMM_M2L_FP16    FP16 operands (per-degree scaled), FP32 accumulation
 *   HFMM_M2L_FP16X3  FP16 hi/lo split, FP32 accumulation
 *   HFMM_FP64        everything in FP64 (outputs FP64)                      */
enum hfmm_precision {
    HFMM_FP64 = 0,
    HFMM_FP32 = 1,
    HFMM_M2L_BF16 = 2,
    HFMM_M2L_BF16X3 = 3,
    HFMM_M2L_FP16 = 4,
    HFMM_M2L_FP16X3 = 5
};

enum hfmm_status {
    HFMM_OK = 0,
    HFMM_E_INVAL = -1,       /* bad argument (null pointer, n < 0, ...) */
    HFMM_E_NOMEM = -2,       /* arena too small, see hfmm_required_bytes */
    HFMM_E_UNSUPPORTED = -3, /* p outside [1, HFMM_MAX_P] or unknown mode */
    HFMM_E_HIP = -4,         /* HIP runtime error */
    HFMM_E_STATE = -5,       /* call order violated (e.g. evaluate before upward) */
    HFMM_E_DATA = -6,        /* non-finite coordinates or masses */
    HFMM_E_OVERFLOW = -7     /* a traversal stack overflowed: lists incomplete */
};

/* bits of the device status word (hfmm_status) */
#define HFMM_ST_SRC_NONFINITE 1u   /* a source coordinate is NaN or infinite */
#define HFMM_ST_TGT_NONFINITE 2u   /* a target coordinate is NaN or infinite */
#define HFMM_ST_MASS_NONFINITE 4u  /* a mass is NaN or infinite */
#define HFMM_ST_OVERFLOW 8u        /* a traversal stack overflowed */

#define HFMM_MAX_P 16
#define HFMM_KEY_LEVELS 21   /* octree depth limit: 21 bits per axis */
#define HFMM_PHASES 10

/* Upper estimate of the arena bytes for one tree over n_src sources,
 * evaluated at up to n_tgt separate targets at a time (0 for
 * self-evaluation only), at order p.  Host only.  The estimate covers
 * uniform and moderately clustered inputs; a tree that needs more returns
 * HFMM_E_NOMEM. */
int hfmm_arena_bytes(int64_t n_src, int64_t n_tgt, int leaf_max, int p,
                     int method, int precision, size_t* bytes);

/* Build the octree over the n_src sources (Sec. 4, "sort" and "other" of
 * Fig. 6): FP64 bounding cube and 63-bit Morton keys, radix sort, cells
 * split while count > leaf_max (and level < 21).  HFMM_E_DATA for
 * non-finite coordinates.  The handle refers to the arena, which must stay
 * alive and untouched until hfmm_tree_release. */
int hfmm_build_tree(const double* x, const double* y, const double* z,
                    int64_t n_src, int leaf_max, void* arena,
                    size_t arena_bytes, void* stream, hfmm_tree* out);

/* Upward pass: P2M at the leaves and M2M to the root (Sec. 2), FP64
 * translation.  m holds the n_src source masses.  method selects the
 * expansion centres: geometric cell centres (FMM, and the treecode over the
 * FMM lists, which also builds those lists here) or centres of mass
 * (treecode).  A later call with new masses replaces the expansions. */
int hfmm_upward(hfmm_tree t, const double* m, int p, int method,
                int precision, void* stream);

/* Far and near field at the targets (Sec. 2): FMM (M2L, L2L, L2P, P2P) or
 * treecode (M2P, P2P) with acceptance parameter theta (not used by
 * HFMM_TREECODE_FMMLIST).  Targets: tx == NULL evaluates at the sources
 * (outputs hold n_src values in the sources' order); otherwise at the n_tgt
 * points tx, ty, tz (outputs hold n_tgt values in their order), binned into
 * the tree as described above (tx == NULL with n_tgt != 0 is
 * HFMM_E_INVAL; an empty target set needs no call).  p, method and
 * precision must match the last hfmm_upward.  The tree may be evaluated again, at the same or other
 * targets; each evaluation needs arena space for its targets
 * (hfmm_arena_bytes with n_tgt). */
int hfmm_evaluate(hfmm_tree t, const double* tx, const double* ty,
                  const double* tz, int64_t n_tgt, int p, double theta,
                  int method, int precision, double eps2, void* phi, void* ax,
                  void* ay, void* az, void* stream);

/* build_tree + upward + evaluate in one call (self-evaluation when tx ==
 * NULL); reads the status word before it returns (HFMM_E_DATA,
 * HFMM_E_OVERFLOW).  The tree handle is released before returning. */
int hfmm_solve(const double* x, const double* y, const double* z,
               const double* m, int64_t n_src, const double* tx,
               const double* ty, const double* tz, int64_t n_tgt, int leaf_max,
               int p, double theta, int method, int precision, double eps2,
               void* arena, size_t arena_bytes, void* phi, void* ax, void* ay,
               void* az, void* stream);

/* Move the tree's sources to new positions x, y, z (device, FP64, n_src
 * each, in the order given to hfmm_build_tree) keeping the tree: the root,
 * the cells, which sources each holds and in what order, and the FMM lists
 * stay as built, which lets a time step of the N-body simulation skip the
 * build.  The expansions of a kept tree stay about the cell centres of the
 * build and converge only while each source stays near its leaf, hence the
 * rule: when every source lies within (1/2 + slack) leaf sides of its
 * leaf's centre along each axis (slack >= 0; 0 is the leaf's closed box),
 * *kept = 1 and the tree holds the new positions; hfmm_upward (new
 * expansions, centres of mass and treecode lists) must then run before the
 * next hfmm_evaluate (HFMM_E_STATE otherwise).  Otherwise, and for
 * non-finite positions, *kept = 0 and the handle holds no usable tree:
 * hfmm_upward and hfmm_evaluate return HFMM_E_STATE, and the caller
 * releases it and builds a new one.  With the one-cell separation of the
 * FMM lists the kept expansions converge for slack below sqrt(3)/3 - 1/2
 * (about 0.077); 1/16 keeps the accuracy close to that of a new tree.
 * Waits for the stream (a 4-byte read back).  HFMM_E_INVAL for null
 * pointers or a negative or non-finite slack. */
int hfmm_refit(hfmm_tree t, const double* x, const double* y, const double* z,
               double slack, void* stream, int* kept);

/* The tree's device status word: waits for the work enqueued on `stream`
 * and reads it.  Returns HFMM_OK, HFMM_E_DATA (non-finite source or target
 * coordinates or masses: the results are meaningless) or HFMM_E_OVERFLOW (a
 * traversal stack overflowed: lists, hence results, are incomplete); *flags
 * (may be NULL) receives the HFMM_ST_* bits.  Source bits stay for the
 * tree's life, mass bits until the next hfmm_upward, target and overflow
 * bits until the next hfmm_evaluate. */
int hfmm_status(hfmm_tree t, void* stream, uint32_t* flags);

/* Direct sum of Eq. 1 (all pairs, P2P kernel of Sec. 5.1) over n sources at
 * the n_tgt points (tx == NULL: at the sources).  precision HFMM_FP64 or
 * HFMM_FP32.  Needs hfmm_direct_bytes() of arena. */
int hfmm_direct_bytes(int64_t n_src, int64_t n_tgt, int precision,
                      size_t* bytes);
int hfmm_direct(const double* x, const double* y, const double* z,
                const double* m, int64_t n_src, const double* tx,
                const double* ty, const double* tz, int64_t n_tgt,
                int precision, double eps2, void* arena, size_t arena_bytes,
                void* phi, void* ax, void* ay, void* az, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the direct
 * sum of hfmm_direct with its staging records in a device array of the
 * library instead of a caller arena.  The array holds HFMM_SCRATCH_BYTES on
 * every GPU the library runs on, from the load of the library until the
 * process ends; its device address is looked up on the first call on each
 * device.  Same arguments (minus the arena), results and errors as
 * hfmm_direct; HFMM_E_NOMEM, before any device work, when
 * hfmm_direct_bytes() of the job exceeds HFMM_SCRATCH_BYTES (2^21 FP64 or
 * 2^22 FP32 points, sources plus distinct targets, less a little alignment).
 * No device memory is allocated or freed.  All calls on one GPU share its
 * array, and nothing in it needs to start at zero: calls that overlap on one
 * GPU (different streams or threads) race and give wrong results, so the
 * caller serialises them. */
#define HFMM_SCRATCH_BYTES (64u << 20)
int hfmm_direct_noalloc(const double* x, const double* y, const double* z,
                        const double* m, int64_t n_src, const double* tx,
                        const double* ty, const double* tz, int64_t n_tgt,
                        int precision, double eps2, void* phi, void* ax,
                        void* ay, void* az, void* stream);

/* N-body time stepping (the simulation of the title; the paper names no
 * integrator, this is kick-drift-kick leapfrog).  Advances x, y, z, vx, vy,
 * vz (device, FP64, n each, in place) by `steps` steps of length dt under
 * the field of all the particles evaluated by `method` (HFMM_DIRECT,
 * HFMM_TREECODE, HFMM_TREECODE_FMMLIST, HFMM_FMM or HFMM_FMM_ROT, with p,
 * theta, precision, eps2 and leaf_max as for hfmm_solve).  Per step:
 * v += a dt/2; x += v dt; a = field(x); v += a dt/2.  The field at the
 * initial positions is evaluated first, so a call makes steps + 1
 * evaluations; on return phi, ax, ay, az (n each, FP64 for HFMM_FP64, FP32
 * otherwise) hold the field at the final positions.  slack < 0 builds a new
 * tree for every evaluation; slack >= 0 keeps the tree across steps while
 * the moved particles pass the rule of hfmm_refit with that slack, and
 * builds a new one when they do not.  The arena holds the evaluation's
 * space (hfmm_arena_bytes, or hfmm_direct_bytes for HFMM_DIRECT) plus 48
 * bytes per particle for the state of the last completed step.  *done (may
 * be NULL) receives the steps completed and *builds (may be NULL) the trees
 * built: after HFMM_E_NOMEM the positions and velocities are those of step
 * *done and hfmm_last_required_bytes() an arena size that would have
 * sufficed, so the caller can continue with the remaining steps (from a new
 * tree). */
int hfmm_leapfrog(double* x, double* y, double* z, double* vx, double* vy,
                  double* vz, const double* m, int64_t n, double dt, int steps,
                  int leaf_max, int p, double theta, int method, int precision,
                  double eps2, double slack, void* arena, size_t arena_bytes,
                  void* phi, void* ax, void* ay, void* az, int* done,
                  int* builds, void* stream);

/* Release the host handle (the arena belongs to the caller). */
void hfmm_tree_release(hfmm_tree t);

/* Arena bytes that would have sufficed for the failed call (after
 * HFMM_E_NOMEM), or otherwise the most bytes the handle's calls have held
 * at once. */
size_t hfmm_required_bytes(hfmm_tree t);
/* same, for a failed build that returned no handle (per thread) */
size_t hfmm_last_required_bytes(void);

typedef struct {
    int64_t n_particles;   /* sources in the tree */
    int64_t n_cells;
    int64_t n_leaves;
    int32_t depth;         /* deepest level (root = 0) */
    int32_t sort_bits;     /* key bits the radix sort ordered */
    double root[4];        /* lower corner of the root cube and half width */
    int64_t list_u, list_v, list_w, list_x;  /* FMM list entries */
    int64_t list_m2p, list_p2p;              /* treecode list entries */
    int64_t p2p_pairs;     /* particle pairs of the last P2P (incl. skipped) */
    int64_t m2l_pairs;     /* cell pairs of the last M2L */
    size_t arena_used;
    /* device time of the phases of the last calls, in ms (-1 when not timed):
     * 0 tree build, 1 FMM lists, 2 upward (P2M, M2M), 3 M2L operator tables,
     * 4 M2L kernel (the matrix products alone), 5 downward (P2L, L2L),
     * 6 far field (L2P, M2P), 7 P2P (+ output scatter), 8 target binning and
     * the targets' lists (treecode lists for self-evaluation),
     * 9 M2L operand preparation (packing, low-precision scaling) */
    double phase_ms[HFMM_PHASES];
    /* the last evaluation's targets: points, boxes, and for separate
     * targets the near (P2P) and far (M2P) list entries of their boxes */
    int64_t n_targets, n_target_boxes, target_near, target_far;
} hfmm_stats;

/* Turn per-phase device timers on or off for trees built afterwards
 * (process-wide; HIP events recorded on the caller's stream around each
 * phase).  Off by default. */
void hfmm_set_timing(int on);

int hfmm_get_stats(hfmm_tree t, hfmm_stats* s);

const char* hfmm_strerror(int code);

/* ---- inspection (tests and tools) ----
 * All dst pointers are device pointers of the stated length; the copies are
 * enqueued on `stream`.  Cells are in level order, Morton order within a
 * level (root first). */
/* perm[s] = caller index of the source at sorted position s (n_particles). */
int hfmm_export_perm(hfmm_tree t, int32_t* dst, void* stream);
/* The boxes of the last evaluation's targets, per target in the caller's
 * order: kind (0 a leaf, 1 an empty octant of a split cell, 2 outside the
 * root cube), level, ix, iy, iz, host (the cell whose local expansion
 * covers the box, -1 none), leaf (the box's own cell, -1 none) and the
 * box's index: 8 int32 per target (n_targets). */
int hfmm_export_targets(hfmm_tree t, int32_t* dst, void* stream);
/* The lists of the last evaluation's separate-target boxes (which 0 far:
 * M2P, 1 near: P2P) as CSR by box index: off (n_target_boxes + 1 int32) and
 * items (target_far or target_near int32; may be NULL). */
int hfmm_export_target_lists(hfmm_tree t, int which, int32_t* off,
                             int32_t* items, void* stream);
/* per cell: level, ix, iy, iz, first, count, parent, first_child, nchild
 * (9 int32 per cell, cell-major) */
int hfmm_export_cells(hfmm_tree t, int32_t* dst, void* stream);
/* FMM list `which` (0 U, 1 V, 2 W, 3 X) as CSR: off (n_cells + 1 int32) and
 * items (hfmm_stats.list_* int32), rows in cell order. */
int hfmm_export_list(hfmm_tree t, int which, int32_t* off, int32_t* items,
                     void* stream);
/* Treecode lists of the last treecode evaluation (0 accepted/M2P, 1 P2P)
 * per cell as CSR, like above; items may be NULL to export the offsets
 * only. */
int hfmm_export_bh_list(hfmm_tree t, int which, int32_t* off, int32_t* items,
                        void* stream);
/* Expansions in the paper's normalisation (Eqs. 2 and 3): which 0 = M
 * (after hfmm_upward), 1 = L (after hfmm_evaluate with HFMM_FMM).  For every
 * cell, n < p, m = 0..n: (Re, Im), i.e. p*(p+1) doubles per cell. */
int hfmm_export_expansions(hfmm_tree t, int which, double* dst, void* stream);

#ifdef __cplusplus
}
#endif
#endif
