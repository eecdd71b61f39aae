/*
 * FP64 CPU oracle for the treecode and fast multipole method of
 * Yokota & Barba, "Treecode and fast multipole method for N-body simulation
 * with CUDA".
 *
 * TEST INFRASTRUCTURE ONLY.  This library exists to check the HIP path.  Only
 * the tests, the smoke check and the CPU-baseline leg of the benchmark may
 * load it.  It shares no code, header, table or constant generator with the
 * HIP library, and the HIP library never calls it.
 *
 * Conventions (all host memory, all FP64):
 *  - Particles are SoA arrays x, y, z, m of length n, in the caller's order.
 *  - Potential phi_i = sum_j m_j / |x_j - x_i| and acceleration
 *    a_i = sum_j m_j (x_j - x_i) / |x_j - x_i|^3 (Eq. 1 per unit target mass,
 *    with the sign of the single-pair kernel of Sec. 5.1); pairs at zero
 *    separation are skipped; eps2 is added to r^2 as in Sec. 5.1.
 *  - Expansion coefficients are complex, all orders m = -n..n stored, index
 *    n*n + n + m, degrees n = 0..p-1 (p = number of terms, Eq. 4).  A complex
 *    value is two doubles (re, im).
 */
#ifndef HFMM_ORACLE_H
#define HFMM_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- special functions (Eqs. 5-9) ---- */
/* P[n*(nmax+1)+m] = P_n^m(x) for 0 <= m <= n <= nmax (Eqs. 7-9). */
void oracle_legendre(int nmax, double x, double* P);
/* Y[n*n+n+m] = Y_n^m(alpha, beta) for n <= nmax (Eq. 6), complex. */
void oracle_ynm(int nmax, double alpha, double beta, double* Y);
/* A_n^m of Eq. 5. */
double oracle_anm(int n, int m);

/* ---- single operators (Eqs. 2-4, translation theorems) ---- */
void oracle_p2m(int p, const double c[3], int64_t n, const double* x,
                const double* y, const double* z, const double* m, double* M);
void oracle_p2l(int p, const double c[3], int64_t n, const double* x,
                const double* y, const double* z, const double* m, double* L);
void oracle_m2m(int p, const double c_child[3], const double c_parent[3],
                const double* Mc, double* Mp /* accumulated */);
void oracle_m2l(int p, const double c_src[3], const double c_tgt[3],
                const double* M, double* L /* accumulated */);
void oracle_l2l(int p, const double c_parent[3], const double c_child[3],
                const double* Lp, double* Lc /* accumulated */);
/* Evaluate at one point: out[0] = phi, out[1..3] = grad phi = acceleration. */
void oracle_l2p(int p, const double c[3], const double* L, const double x[3],
                double out[4]);
void oracle_m2p(int p, const double c[3], const double* M, const double x[3],
                double out[4]);

/* ---- direct sum (Eq. 1) ---- */
/* Targets are source indices tidx[0..nt) (all sources when tidx == NULL,
 * nt == n). Summation over sources in ascending index order. */
void oracle_direct(int64_t n, const double* x, const double* y,
                   const double* z, const double* m, int64_t nt,
                   const int64_t* tidx, double eps2, double* phi, double* ax,
                   double* ay, double* az);
/* Targets given by coordinates (any point; pairs at r == 0 skipped). */
void oracle_direct_points(int64_t n, const double* x, const double* y,
                          const double* z, const double* m, int64_t nt,
                          const double* tx, const double* ty, const double* tz,
                          double eps2, double* phi, double* ax, double* ay,
                          double* az);

/* ---- octree (Morton keys, adaptive split rule) ---- */
typedef struct otree otree;
otree* oracle_tree_build(int64_t n, const double* x, const double* y,
                         const double* z, int leaf_max);
void oracle_tree_free(otree* t);
int64_t oracle_tree_ncells(const otree* t);
int oracle_tree_depth(const otree* t);
/* root[0..2] = lower corner b, root[3] = half width R */
void oracle_tree_root(const otree* t, double root[4]);
/* keys in the caller's order */
void oracle_tree_keys(const otree* t, uint64_t* keys);
/* perm[s] = caller index of the particle at sorted position s */
void oracle_tree_perm(const otree* t, int64_t* perm);
/* Cells in level order, Morton order within a level. */
void oracle_tree_cells(const otree* t, int32_t* level, int32_t* ix,
                       int32_t* iy, int32_t* iz, int64_t* first,
                       int64_t* count, int32_t* parent, int32_t* first_child,
                       int32_t* nchild);
void oracle_tree_centres(const otree* t, double* cx, double* cy, double* cz,
                         double* side);

/* A tree kept while its particles move: new positions (caller order) for
 * the same cells, membership, order, root and lists. */
void oracle_tree_move(otree* t, const double* x, const double* y,
                      const double* z);
/* 1 iff every particle at x, y, z lies within (1/2 + slack) leaf sides of
 * its leaf's centre along each axis (non-finite: 0). */
int oracle_tree_stays(const otree* t, const double* x, const double* y,
                      const double* z, double slack);

/* FMM lists U, V, W, X (which = 0..3). CSR: off[ncells+1], items[off[ncells]].
 * Lists are computed on first request. */
int64_t oracle_list_size(otree* t, int which);
void oracle_list_get(otree* t, int which, int64_t* off, int32_t* items);
/* Brute-force construction of the same lists straight from the definitions
 * (quadratic in the number of cells; for small trees only). */
int64_t oracle_list_size_bruteforce(otree* t, int which);
void oracle_list_get_bruteforce(otree* t, int which, int64_t* off,
                                int32_t* items);

/* Barnes-Hut group lists for a target leaf: accepted cells (M2P, which = 0)
 * and leaves interacted directly (P2P, which = 1).  Needs masses (caller
 * order) for the centres of mass. CSR over all cells; non-leaves are empty. */
int64_t oracle_bh_lists(otree* t, const double* m, double theta, int which,
                        int64_t* off, int32_t* items);

/* FP64 centre of mass of every cell (weights |m|; geometric centre if the
 * cell's |m| sums to zero). */
void oracle_tree_com(otree* t, const double* m, double* comx, double* comy,
                     double* comz);

/* ---- drivers ---- */
/* All multipole (M) and local (L) expansions of the FMM for masses m
 * (caller order); M and L hold ncells * p*p complex values. */
int oracle_fmm_expansions(otree* t, const double* m, int p, double* M,
                          double* L);
/* Full FMM. Targets are caller indices tidx[0..nt) (all when tidx == NULL). */
int oracle_fmm(int64_t n, const double* x, const double* y, const double* z,
               const double* m, int leaf_max, int p, double eps2, int64_t nt,
               const int64_t* tidx, double* phi, double* ax, double* ay,
               double* az);
/* The FMM and the treecode on a given tree (its particles where
 * oracle_tree_build or the last oracle_tree_move put them); masses and
 * target indices in the caller's order. */
int oracle_fmm_tree(otree* t, const double* m, int p, double eps2, int64_t nt,
                    const int64_t* tidx, double* phi, double* ax, double* ay,
                    double* az);
int oracle_treecode_tree(otree* t, const double* m, int p, double theta,
                         int mode, double eps2, int64_t nt,
                         const int64_t* tidx, double* phi, double* ax,
                         double* ay, double* az);
/* Treecode. mode 0: group acceptance per target leaf; mode 1: per target
 * particle; expansions centred at centres of mass.  mode 2: the treecode of
 * Sec. 4, M2P over the FMM's V lists (leaf and ancestors) and W list, P2P
 * over its U list and X lists (leaf and ancestors), expansions about the
 * geometric centres; theta is not used. */
int oracle_treecode(int64_t n, const double* x, const double* y,
                    const double* z, const double* m, int leaf_max, int p,
                    double theta, int mode, double eps2, int64_t nt,
                    const int64_t* tidx, double* phi, double* ax, double* ay,
                    double* az);

/* ---- separate targets, binned into the source tree ---- */
/* Per target point: kind (0 a leaf of the tree, 1 an empty octant of a
 * split cell, 2 outside the root cube), level, ix, iy, iz of its box, host
 * (the cell whose local expansion covers the box, -1 none) and leaf (the
 * box's cell when kind 0, else -1): 7 int64 per target. */
void oracle_target_boxes(otree* t, int64_t nt, const double* tx,
                         const double* ty, const double* tz, int64_t* out);
/* List `which` (0 U, 1 V, 2 W, 3 X) of the box of point xt, from the
 * definitions; returns its length (items may be NULL). */
int64_t oracle_box_list(otree* t, const double xt[3], int which,
                        int32_t* items);
/* FMM and treecode (mode 0 or 2) at separate target points. */
int oracle_fmm_points(int64_t n, const double* x, const double* y,
                      const double* z, const double* m, int leaf_max, int p,
                      double eps2, int64_t nt, const double* tx,
                      const double* ty, const double* tz, double* phi,
                      double* ax, double* ay, double* az);
int oracle_treecode_points(int64_t n, const double* x, const double* y,
                           const double* z, const double* m, int leaf_max,
                           int p, double theta, int mode, double eps2,
                           int64_t nt, const double* tx, const double* ty,
                           const double* tz, double* phi, double* ax,
                           double* ay, double* az);

/* The same on a given tree (see oracle_fmm_tree). */
int oracle_fmm_points_tree(otree* t, const double* m, int p, double eps2,
                           int64_t nt, const double* tx, const double* ty,
                           const double* tz, double* phi, double* ax,
                           double* ay, double* az);
int oracle_treecode_points_tree(otree* t, const double* m, int p, double theta,
                                int mode, double eps2, int64_t nt,
                                const double* tx, const double* ty,
                                const double* tz, double* phi, double* ax,
                                double* ay, double* az);

/* ---- rotation-based M2L (Sec. 6) ---- */
/* M2L by rotation to the translation axis, coaxial translation (Eq. 4 along
 * z) and rotation back; accumulates into L like oracle_m2l. */
void oracle_m2l_rot(int p, const double c_src[3], const double c_tgt[3],
                    const double* M, double* L);
/* Coefficients (degrees < p) of the field u -> f(Q u), Q a 3x3 row-major
 * rotation, f given by `in` (complex, index n*n + n + m). */
void oracle_rotate(int p, const double Q[9], const double* in, double* out);

/* Threads OpenMP will use (1 when built without OpenMP); set them (n > 0). */
int oracle_num_threads(void);
void oracle_set_num_threads(int n);
/* Wall-clock seconds of the last oracle_fmm_tree (or oracle_fmm) call:
 * out[0] upward, out[1] downward (the cells the targets need), out[2] the
 * evaluation at the targets. */
void oracle_fmm_phase_seconds(double out[3]);

#ifdef __cplusplus
}
#endif
#endif
