/*
 * FP64 CPU oracle for the treecode and fast multipole method of
 * Yokota & Barba, "Treecode and fast multipole method for N-body simulation
 * with CUDA".
 *
 * TEST INFRASTRUCTURE ONLY: it is the plain, slow reference that the HIP
 * library is checked against.  Only the tests, the smoke check and the
 * CPU-baseline leg of the benchmark may load it.  It shares no code with the
 * HIP library.
 *
 * Everything is scalar FP64 and follows the paper's formulas as printed:
 *   Eq. 1            direct sum (sign and self-pair rule of Sec. 5.1)
 *   Eq. 2            multipole expansion  (P2M, M2P)
 *   Eq. 3            local expansion      (P2L, L2P)
 *   Eq. 4            multipole-to-local translation, evaluated literally as
 *                    complex sums over all orders m = -n..n
 *   Eq. 5, 6         A_n^m, Y_n^m
 *   Eqs. 7-9         Legendre recurrences (Eq. 8 read as a double factorial)
 * The operators the paper names but does not print (M2M, L2L, the gradient
 * of L2P and M2P, the adaptive lists it cites from Cheng, Greengard and
 * Rokhlin) follow the classical translation theorems of Greengard and
 * Rokhlin in the paper's normalisation; each is pinned by an exactness or
 * finite-difference test.  OpenMP only parallelises loops over independent
 * outputs; it never changes the order of a sum.
 */
#define _POSIX_C_SOURCE 199309L /* clock_gettime under -std=c99 */
#include "hfmm_oracle.h"

#include <complex.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>
#include <time.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define KBITS 21                     /* key depth: 21 bits per axis */
#define CI(n, m) ((n) * (n) + (n) + (m))

typedef double complex cplx;

int oracle_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void oracle_set_num_threads(int n) {
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

/* wall-clock seconds of the phases of the last oracle_fmm_tree call:
 * upward, downward, evaluation at the targets (timing only; no result
 * depends on it) */
static double g_phase_s[3];

static double wall_s(void) {
    struct timespec ts;
    clock_gettime(CLOCK_MONOTONIC, &ts);
    return (double)ts.tv_sec + 1e-9 * (double)ts.tv_nsec;
}

void oracle_fmm_phase_seconds(double out[3]) {
    for (int i = 0; i < 3; i++) out[i] = g_phase_s[i];
}

/* ------------------------------------------------------------------ */
/* special functions                                                   */
/* ------------------------------------------------------------------ */

static double factorial(int n) {
    double f = 1.0;
    for (int i = 2; i <= n; i++) f *= (double)i;
    return f;
}

static double double_factorial(int n) { /* n!! with (-1)!! = 1 */
    double f = 1.0;
    for (int i = n; i > 1; i -= 2) f *= (double)i;
    return f;
}

/* x^e for integer e by repeated multiplication (exactly covariant under
 * power-of-two scaling of x, unlike a library pow). */
static double ipow(double x, int e) {
    double r = 1.0;
    for (int i = 0; i < (e < 0 ? -e : e); i++) r *= x;
    return e < 0 ? 1.0 / r : r;
}

/* Eq. 5 */
double oracle_anm(int n, int m) {
    if (m < 0) m = -m;
    if (m > n) return 0.0;
    return 1.0 / sqrt(factorial(n - m) * factorial(n + m));
}

/* Eqs. 7-9 with x = cos(alpha) and s = sin(alpha) = (1 - x^2)^{1/2}.
 * Eq. 8 is read with the double factorial (2m-1)!!, which is what its
 * recurrence multiplies by (1, 3, 5, ...).  s is passed in rather than
 * formed from x, which would lose digits near the poles. */
static void legendre_xs(int nmax, double x, double s, double* P) {
    const int w = nmax + 1;
    for (int i = 0; i < w * w; i++) P[i] = 0.0;
    for (int m = 0; m <= nmax; m++) {
        /* Eq. 8: P_m^m = (-1)^m (2m-1)!! (1-x^2)^{m/2} */
        double pmm = ((m & 1) ? -1.0 : 1.0) * double_factorial(2 * m - 1) *
                     ipow(s, m);
        P[m * w + m] = pmm;
        /* Eq. 9: P_{m+1}^m = x (2m+1) P_m^m */
        if (m + 1 <= nmax) P[(m + 1) * w + m] = x * (2 * m + 1) * pmm;
        /* Eq. 7: (n-m+1) P_{n+1}^m = x (2n+1) P_n^m - (n+m) P_{n-1}^m */
        for (int n = m + 1; n < nmax; n++)
            P[(n + 1) * w + m] = (x * (2 * n + 1) * P[n * w + m] -
                                  (n + m) * P[(n - 1) * w + m]) /
                                 (double)(n - m + 1);
    }
}

void oracle_legendre(int nmax, double x, double* P) {
    double s2 = 1.0 - x * x;
    legendre_xs(nmax, x, sqrt(s2 < 0.0 ? 0.0 : s2), P);
}

/* Eq. 6 for all n <= nmax, m = -n..n.  Y is complex. */
static void ynm_table(int nmax, double alpha, double beta, cplx* Y) {
    const int w = nmax + 1;
    double* P = (double*)malloc(sizeof(double) * w * w);
    legendre_xs(nmax, cos(alpha), sin(alpha), P);
    for (int n = 0; n <= nmax; n++)
        for (int m = -n; m <= n; m++) {
            int am = m < 0 ? -m : m;
            double nrm = sqrt(factorial(n - am) / factorial(n + am));
            Y[CI(n, m)] = nrm * P[n * w + am] * cexp(I * (double)m * beta);
        }
    free(P);
}

void oracle_ynm(int nmax, double alpha, double beta, double* Y) {
    ynm_table(nmax, alpha, beta, (cplx*)Y);
}

/* spherical coordinates (rho, alpha, beta) of v; alpha = beta = 0 at the
 * origin and on the z axis. */
static void cart2sph(const double v[3], double* rho, double* alpha,
                     double* beta) {
    double r = sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
    *rho = r;
    if (r == 0.0) {
        *alpha = 0.0;
        *beta = 0.0;
        return;
    }
    /* polar angle from atan2: well conditioned near the z axis, where
     * acos(z / r) loses half the digits */
    *alpha = atan2(sqrt(v[0] * v[0] + v[1] * v[1]), v[2]);
    *beta = (v[0] == 0.0 && v[1] == 0.0) ? 0.0 : atan2(v[1], v[0]);
}

/* i^e for even e */
static double ipow_even(int e) { return ((e / 2) & 1) ? -1.0 : 1.0; }

static double neg1pow(int e) { return (e & 1) ? -1.0 : 1.0; }


/* ------------------------------------------------------------------ */
/* operators                                                           */
/* ------------------------------------------------------------------ */

/* Eq. 2: M_n^m += m_j rho_j^n Y_n^{-m}(alpha_j, beta_j), about centre c */
static void p2m_c(int p, const double c[3], int64_t n, const double* x,
                  const double* y, const double* z, const double* q,
                  cplx* M) {
    cplx* Y = (cplx*)malloc(sizeof(cplx) * p * p);
    for (int64_t j = 0; j < n; j++) {
        double v[3] = {x[j] - c[0], y[j] - c[1], z[j] - c[2]};
        double rho, al, be;
        cart2sph(v, &rho, &al, &be);
        ynm_table(p - 1, al, be, Y);
        for (int nn = 0; nn < p; nn++)
            for (int m = -nn; m <= nn; m++)
                M[CI(nn, m)] += q[j] * ipow(rho, nn) * Y[CI(nn, -m)];
    }
    free(Y);
}

void oracle_p2m(int p, const double c[3], int64_t n, const double* x,
                const double* y, const double* z, const double* m, double* M) {
    memset(M, 0, sizeof(cplx) * p * p);
    p2m_c(p, c, n, x, y, z, m, (cplx*)M);
}

/* Eq. 3: L_n^m += m_j rho_j^{-n-1} Y_n^{-m}(alpha_j, beta_j) */
static void p2l_c(int p, const double c[3], int64_t n, const double* x,
                  const double* y, const double* z, const double* q,
                  cplx* L) {
    cplx* Y = (cplx*)malloc(sizeof(cplx) * p * p);
    for (int64_t j = 0; j < n; j++) {
        double v[3] = {x[j] - c[0], y[j] - c[1], z[j] - c[2]};
        double rho, al, be;
        cart2sph(v, &rho, &al, &be);
        if (rho == 0.0) continue;
        ynm_table(p - 1, al, be, Y);
        for (int nn = 0; nn < p; nn++)
            for (int m = -nn; m <= nn; m++)
                L[CI(nn, m)] +=
                    q[j] * ipow(rho, -nn - 1) * Y[CI(nn, -m)];
    }
    free(Y);
}

void oracle_p2l(int p, const double c[3], int64_t n, const double* x,
                const double* y, const double* z, const double* m, double* L) {
    memset(L, 0, sizeof(cplx) * p * p);
    p2l_c(p, c, n, x, y, z, m, (cplx*)L);
}

/* M2M (paper-silent; Greengard-Rokhlin), vector = c_child - c_parent:
 * M_j^k += sum_{n<=j} sum_m M_{j-n}^{k-m} i^{|k|-|m|-|k-m|} A_n^m A_{j-n}^{k-m}
 *          rho^n Y_n^{-m}(alpha, beta) / A_j^k                               */
static void m2m_c(int p, const double cc[3], const double cp[3],
                  const cplx* Mc, cplx* Mp) {
    double v[3] = {cc[0] - cp[0], cc[1] - cp[1], cc[2] - cp[2]};
    double rho, al, be;
    cart2sph(v, &rho, &al, &be);
    cplx* Y = (cplx*)malloc(sizeof(cplx) * p * p);
    ynm_table(p - 1, al, be, Y);
    for (int j = 0; j < p; j++)
        for (int k = -j; k <= j; k++) {
            cplx s = 0.0;
            for (int n = 0; n <= j; n++)
                for (int m = -n; m <= n; m++) {
                    int km = k - m;
                    if (abs(km) > j - n) continue;
                    s += Mc[CI(j - n, km)] *
                         ipow_even(abs(k) - abs(m) - abs(km)) *
                         oracle_anm(n, m) * oracle_anm(j - n, km) *
                         ipow(rho, n) * Y[CI(n, -m)] /
                         oracle_anm(j, k);
                }
            Mp[CI(j, k)] += s;
        }
    free(Y);
}

void oracle_m2m(int p, const double c_child[3], const double c_parent[3],
                const double* Mc, double* Mp) {
    m2m_c(p, c_child, c_parent, (const cplx*)Mc, (cplx*)Mp);
}

/* Eq. 4, literally.  (rho, alpha, beta) are the spherical coordinates of
 * c_target - c_source: with the (-1)^j of Eq. 4 this is the direction for
 * which a unit mass at the source centre gives exactly its P2L expansion.
 * Y_{j+n} is needed up to degree 2p-2. */
static void m2l_c(int p, const double cs[3], const double ct[3],
                  const cplx* M, cplx* L) {
    double v[3] = {ct[0] - cs[0], ct[1] - cs[1], ct[2] - cs[2]};
    double rho, al, be;
    cart2sph(v, &rho, &al, &be);
    const int nmax = 2 * p - 2;
    cplx* Y = (cplx*)malloc(sizeof(cplx) * (nmax + 1) * (nmax + 1));
    ynm_table(nmax, al, be, Y);
    for (int j = 0; j < p; j++)
        for (int k = -j; k <= j; k++) {
            cplx s = 0.0;
            for (int n = 0; n < p; n++)
                for (int m = -n; m <= n; m++) {
                    s += M[CI(n, m)] * ipow_even(abs(k - m) - abs(k) - abs(m)) *
                         oracle_anm(n, m) * oracle_anm(j, k) *
                         Y[CI(j + n, m - k)] /
                         (neg1pow(j) * oracle_anm(j + n, m - k) *
                          ipow(rho, j + n + 1));
                }
            L[CI(j, k)] += s;
        }
    free(Y);
}

void oracle_m2l(int p, const double c_src[3], const double c_tgt[3],
                const double* M, double* L) {
    m2l_c(p, c_src, c_tgt, (const cplx*)M, (cplx*)L);
}

/* L2L (paper-silent; Greengard-Rokhlin), vector = c_parent - c_child:
 * L_j^k += sum_{n>=j} sum_m L_n^m i^{|m|-|m-k|-|k|} A_{n-j}^{m-k} A_j^k
 *          Y_{n-j}^{m-k}(alpha, beta) rho^{n-j} / ((-1)^{n+j} A_n^m)         */
static void l2l_c(int p, const double cp[3], const double cc[3],
                  const cplx* Lp, cplx* Lc) {
    double v[3] = {cp[0] - cc[0], cp[1] - cc[1], cp[2] - cc[2]};
    double rho, al, be;
    cart2sph(v, &rho, &al, &be);
    cplx* Y = (cplx*)malloc(sizeof(cplx) * p * p);
    ynm_table(p - 1, al, be, Y);
    for (int j = 0; j < p; j++)
        for (int k = -j; k <= j; k++) {
            cplx s = 0.0;
            for (int n = j; n < p; n++)
                for (int m = -n; m <= n; m++) {
                    int mk = m - k;
                    if (abs(mk) > n - j) continue;
                    s += Lp[CI(n, m)] * ipow_even(abs(m) - abs(mk) - abs(k)) *
                         oracle_anm(n - j, mk) * oracle_anm(j, k) *
                         Y[CI(n - j, mk)] * ipow(rho, n - j) /
                         (neg1pow(n + j) * oracle_anm(n, m));
                }
            Lc[CI(j, k)] += s;
        }
    free(Y);
}

void oracle_l2l(int p, const double c_parent[3], const double c_child[3],
                const double* Lp, double* Lc) {
    l2l_c(p, c_parent, c_child, (const cplx*)Lp, (cplx*)Lc);
}

/* Gradient helpers (paper-silent).  Spherical chain rule with the
 * pole-free Legendre identities (Condon-Shortley phase):
 *   dP_n^mu/dtheta = 1/2 [P_n^{mu+1} - (n+mu)(n-mu+1) P_n^{mu-1}],  mu >= 1
 *   dP_n^0/dtheta  = P_n^1
 *   mu P_n^mu / sin(theta) = -1/2 [P_{n+1}^{mu+1}
 *                                  + (n-mu+1)(n-mu+2) P_{n+1}^{mu-1}]
 * P is tabulated to degree p so the second identity is available. */
static double dP_dtheta(const double* P, int w, int n, int mu) {
    if (mu == 0) return (n >= 1) ? P[n * w + 1] : 0.0;
    double up = (mu + 1 <= n) ? P[n * w + mu + 1] : 0.0;
    return 0.5 * (up - (double)(n + mu) * (n - mu + 1) * P[n * w + mu - 1]);
}

static double muP_over_sin(const double* P, int w, int n, int mu) {
    if (mu == 0) return 0.0;
    return -0.5 * (P[(n + 1) * w + mu + 1] +
                   (double)(n - mu + 1) * (n - mu + 2) * P[(n + 1) * w + mu - 1]);
}

/* Evaluate sum_n sum_m C_n^m f_n(r) Y_n^m(theta, phi) and its gradient, where
 * f_n(r) = r^n (local) or r^{-n-1} (multipole). */
static void eval_expansion(int p, const double c[3], const cplx* C,
                           const double x[3], int local, double out[4]) {
    double v[3] = {x[0] - c[0], x[1] - c[1], x[2] - c[2]};
    double r, th, ph;
    cart2sph(v, &r, &th, &ph);
    const int w = p + 1;
    double* P = (double*)malloc(sizeof(double) * w * w);
    legendre_xs(p, cos(th), sin(th), P);
    const double st = sin(th), ct = cos(th), sp = sin(ph), cp = cos(ph);
    cplx f = 0.0, gr = 0.0, gt = 0.0, gp = 0.0;
    for (int n = 0; n < p; n++) {
        double fr, dfr, fr_over_r;
        if (local) {
            fr = ipow(r, n);
            dfr = (n == 0) ? 0.0 : n * ipow(r, n - 1);
            fr_over_r = (n == 0) ? 0.0 : ipow(r, n - 1);
        } else {
            fr = ipow(r, -n - 1);
            dfr = -(n + 1) * ipow(r, -n - 2);
            fr_over_r = ipow(r, -n - 2);
        }
        for (int m = -n; m <= n; m++) {
            int mu = m < 0 ? -m : m;
            double nrm = sqrt(factorial(n - mu) / factorial(n + mu));
            cplx e = cexp(I * (double)m * ph);
            cplx cf = C[CI(n, m)] * nrm * e;
            double Pnm = P[n * w + mu];
            f += cf * fr * Pnm;
            gr += cf * dfr * Pnm;
            gt += cf * fr_over_r * dP_dtheta(P, w, n, mu);
            /* (1/(r sin theta)) d/dphi: the phi-derivative brings i m */
            double sgn = m < 0 ? -1.0 : 1.0;
            gp += cf * fr_over_r * I * sgn * muP_over_sin(P, w, n, mu);
        }
    }
    free(P);
    double g_r = creal(gr), g_t = creal(gt), g_p = creal(gp);
    out[0] = creal(f);
    out[1] = st * cp * g_r + ct * cp * g_t - sp * g_p;
    out[2] = st * sp * g_r + ct * sp * g_t + cp * g_p;
    out[3] = ct * g_r - st * g_t;
}

void oracle_l2p(int p, const double c[3], const double* L, const double x[3],
                double out[4]) {
    eval_expansion(p, c, (const cplx*)L, x, 1, out);
}

void oracle_m2p(int p, const double c[3], const double* M, const double x[3],
                double out[4]) {
    eval_expansion(p, c, (const cplx*)M, x, 0, out);
}

/* ------------------------------------------------------------------ */
/* direct sum                                                          */
/* ------------------------------------------------------------------ */

/* One target against sources [0, n) in ascending order; pairs with
 * r^2 == 0 skipped (the single-pair kernel of Sec. 5.1 plus potential). */
static void p2p_point(const double t[3], int64_t j0, int64_t j1,
                      const double* x, const double* y, const double* z,
                      const double* m, double eps2, double acc[4]) {
    for (int64_t j = j0; j < j1; j++) {
        double dx = x[j] - t[0], dy = y[j] - t[1], dz = z[j] - t[2];
        double r2 = dx * dx + dy * dy + dz * dz;
        if (r2 == 0.0) continue;
        r2 += eps2;
        double rinv = 1.0 / sqrt(r2);
        double s = m[j] * rinv * rinv * rinv;
        acc[0] += m[j] * rinv;
        acc[1] += dx * s;
        acc[2] += dy * s;
        acc[3] += dz * s;
    }
}

void oracle_direct_points(int64_t n, const double* x, const double* y,
                          const double* z, const double* m, int64_t nt,
                          const double* tx, const double* ty, const double* tz,
                          double eps2, double* phi, double* ax, double* ay,
                          double* az) {
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < nt; i++) {
        double t[3] = {tx[i], ty[i], tz[i]};
        double acc[4] = {0, 0, 0, 0};
        p2p_point(t, 0, n, x, y, z, m, eps2, acc);
        phi[i] = acc[0];
        ax[i] = acc[1];
        ay[i] = acc[2];
        az[i] = acc[3];
    }
}

void oracle_direct(int64_t n, const double* x, const double* y,
                   const double* z, const double* m, int64_t nt,
                   const int64_t* tidx, double eps2, double* phi, double* ax,
                   double* ay, double* az) {
    if (tidx == NULL) nt = n;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t k = 0; k < nt; k++) {
        int64_t i = tidx ? tidx[k] : k;
        double t[3] = {x[i], y[i], z[i]};
        double acc[4] = {0, 0, 0, 0};
        p2p_point(t, 0, n, x, y, z, m, eps2, acc);
        phi[k] = acc[0];
        ax[k] = acc[1];
        ay[k] = acc[2];
        az[k] = acc[3];
    }
}

/* ------------------------------------------------------------------ */
/* octree                                                              */
/* ------------------------------------------------------------------ */

typedef struct {
    int level;
    int ix, iy, iz;
    int64_t first, count;
    int parent;
    int first_child, nchild;
} ocell;

struct otree {
    int64_t n;
    int leaf_max;
    double b[3], R;
    uint64_t* keys;  /* caller order */
    int64_t* perm;   /* sorted position -> caller index */
    double *xs, *ys, *zs; /* sorted positions */
    ocell* c;
    int64_t ncells, cap;
    int depth;
    int* leaf_of;    /* sorted position -> leaf cell */
    /* lists: 0 U, 1 V, 2 W, 3 X */
    int lists_done;
    int64_t* loff[4];
    int32_t* litem[4];
};

/* Appendix-B style root cube and 63-bit Morton key: q_a =
 * clamp(floor((x_a - b_a) * s), 0, 2^21 - 1), s = 2^21 / (2R); bit 3t+2 of
 * the key is bit t of q_x, bit 3t+1 of q_y, bit 3t of q_z. */
static uint64_t spread3(uint64_t v) {
    uint64_t r = 0;
    for (int t = 0; t < KBITS; t++) r |= ((v >> t) & 1ull) << (3 * t);
    return r;
}

static int64_t quantise(double xa, double ba, double s) {
    double f = floor((xa - ba) * s);
    int64_t q = (int64_t)f;
    if (f < 0.0) q = 0;
    if (q > (1 << KBITS) - 1) q = (1 << KBITS) - 1;
    return q;
}

typedef struct {
    uint64_t key;
    int64_t idx;
} keyidx;

static int cmp_keyidx(const void* a, const void* b) {
    const keyidx* u = (const keyidx*)a;
    const keyidx* v = (const keyidx*)b;
    if (u->key != v->key) return u->key < v->key ? -1 : 1;
    return (u->idx > v->idx) - (u->idx < v->idx);
}

static int push_cell(otree* t, ocell cell) {
    if (t->ncells == t->cap) {
        t->cap = t->cap ? 2 * t->cap : 1024;
        t->c = (ocell*)realloc(t->c, sizeof(ocell) * t->cap);
    }
    t->c[t->ncells] = cell;
    return (int)t->ncells++;
}

otree* oracle_tree_build(int64_t n, const double* x, const double* y,
                         const double* z, int leaf_max) {
    otree* t = (otree*)calloc(1, sizeof(otree));
    t->n = n;
    t->leaf_max = leaf_max;
    /* root cube */
    double lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
    const double* X[3] = {x, y, z};
    for (int a = 0; a < 3; a++) {
        if (n > 0) lo[a] = hi[a] = X[a][0];
        for (int64_t i = 1; i < n; i++) {
            if (X[a][i] < lo[a]) lo[a] = X[a][i];
            if (X[a][i] > hi[a]) hi[a] = X[a][i];
        }
    }
    double R = 0.0, c[3];
    for (int a = 0; a < 3; a++) {
        c[a] = (lo[a] + hi[a]) / 2.0;
        double h = (hi[a] - lo[a]) / 2.0;
        if (h > R) R = h;
    }
    if (R == 0.0) R = 1.0;
    for (int a = 0; a < 3; a++) t->b[a] = c[a] - R;
    t->R = R;
    const double s = (double)(1 << KBITS) / (2.0 * R);
    /* keys and stable sort */
    t->keys = (uint64_t*)malloc(sizeof(uint64_t) * (n ? n : 1));
    keyidx* ki = (keyidx*)malloc(sizeof(keyidx) * (n ? n : 1));
    for (int64_t i = 0; i < n; i++) {
        uint64_t qx = (uint64_t)quantise(x[i], t->b[0], s);
        uint64_t qy = (uint64_t)quantise(y[i], t->b[1], s);
        uint64_t qz = (uint64_t)quantise(z[i], t->b[2], s);
        t->keys[i] = (spread3(qx) << 2) | (spread3(qy) << 1) | spread3(qz);
        ki[i].key = t->keys[i];
        ki[i].idx = i;
    }
    qsort(ki, (size_t)n, sizeof(keyidx), cmp_keyidx);
    t->perm = (int64_t*)malloc(sizeof(int64_t) * (n ? n : 1));
    t->xs = (double*)malloc(sizeof(double) * (n ? n : 1));
    t->ys = (double*)malloc(sizeof(double) * (n ? n : 1));
    t->zs = (double*)malloc(sizeof(double) * (n ? n : 1));
    for (int64_t i = 0; i < n; i++) {
        t->perm[i] = ki[i].idx;
        t->xs[i] = x[ki[i].idx];
        t->ys[i] = y[ki[i].idx];
        t->zs[i] = z[ki[i].idx];
    }
    /* cells, level by level: split iff count > leaf_max and level < 21 */
    t->depth = 0;
    if (n > 0) {
        ocell root = {0, 0, 0, 0, 0, n, -1, -1, 0};
        push_cell(t, root);
        int64_t lev_begin = 0, lev_end = 1;
        for (int lev = 0; lev_begin < lev_end; lev++) {
            for (int64_t ci = lev_begin; ci < lev_end; ci++) {
                ocell cc = t->c[ci];
                if (!(cc.count > leaf_max && lev < KBITS)) continue;
                int shift = 3 * (KBITS - lev - 1);
                int64_t j = cc.first, end = cc.first + cc.count;
                for (int o = 0; o < 8; o++) {
                    int64_t j0 = j;
                    while (j < end && (int)((ki[j].key >> shift) & 7u) == o) j++;
                    if (j == j0) continue;
                    ocell ch = {lev + 1,
                                2 * cc.ix + ((o >> 2) & 1),
                                2 * cc.iy + ((o >> 1) & 1),
                                2 * cc.iz + (o & 1),
                                j0, j - j0, (int)ci, -1, 0};
                    int id = push_cell(t, ch);
                    if (t->c[ci].nchild == 0) t->c[ci].first_child = id;
                    t->c[ci].nchild++;
                    if (lev + 1 > t->depth) t->depth = lev + 1;
                }
            }
            lev_begin = lev_end;
            lev_end = t->ncells;
        }
    }
    free(ki);
    t->leaf_of = (int*)malloc(sizeof(int) * (n ? n : 1));
    for (int64_t ci = 0; ci < t->ncells; ci++)
        if (t->c[ci].nchild == 0)
            for (int64_t i = t->c[ci].first; i < t->c[ci].first + t->c[ci].count;
                 i++)
                t->leaf_of[i] = (int)ci;
    return t;
}

void oracle_tree_free(otree* t) {
    if (!t) return;
    free(t->keys);
    free(t->perm);
    free(t->xs);
    free(t->ys);
    free(t->zs);
    free(t->c);
    free(t->leaf_of);
    for (int w = 0; w < 4; w++) {
        free(t->loff[w]);
        free(t->litem[w]);
    }
    free(t);
}

int64_t oracle_tree_ncells(const otree* t) { return t->ncells; }
int oracle_tree_depth(const otree* t) { return t->depth; }

void oracle_tree_root(const otree* t, double root[4]) {
    root[0] = t->b[0];
    root[1] = t->b[1];
    root[2] = t->b[2];
    root[3] = t->R;
}

void oracle_tree_keys(const otree* t, uint64_t* keys) {
    memcpy(keys, t->keys, sizeof(uint64_t) * t->n);
}

void oracle_tree_perm(const otree* t, int64_t* perm) {
    memcpy(perm, t->perm, sizeof(int64_t) * t->n);
}

void oracle_tree_cells(const otree* t, int32_t* level, int32_t* ix,
                       int32_t* iy, int32_t* iz, int64_t* first,
                       int64_t* count, int32_t* parent, int32_t* first_child,
                       int32_t* nchild) {
    for (int64_t i = 0; i < t->ncells; i++) {
        level[i] = t->c[i].level;
        ix[i] = t->c[i].ix;
        iy[i] = t->c[i].iy;
        iz[i] = t->c[i].iz;
        first[i] = t->c[i].first;
        count[i] = t->c[i].count;
        parent[i] = t->c[i].parent;
        first_child[i] = t->c[i].first_child;
        nchild[i] = t->c[i].nchild;
    }
}

static double cell_side(const otree* t, int level) {
    return 2.0 * t->R / (double)(1 << level);
}

static void cell_centre(const otree* t, const ocell* c, double out[3]) {
    double h = cell_side(t, c->level);
    out[0] = t->b[0] + (c->ix + 0.5) * h;
    out[1] = t->b[1] + (c->iy + 0.5) * h;
    out[2] = t->b[2] + (c->iz + 0.5) * h;
}

void oracle_tree_centres(const otree* t, double* cx, double* cy, double* cz,
                         double* side) {
    for (int64_t i = 0; i < t->ncells; i++) {
        double cc[3];
        cell_centre(t, &t->c[i], cc);
        cx[i] = cc[0];
        cy[i] = cc[1];
        cz[i] = cc[2];
        side[i] = cell_side(t, t->c[i].level);
    }
}

/* ---- a tree kept while its particles move (time stepping) ---- */

/* The particles of the tree take new positions (caller order): the cells,
 * their membership and order, the root and the lists stay as built, and the
 * expansions about the unchanged cell centres are formed from the new
 * positions by the drivers on this tree. */
void oracle_tree_move(otree* t, const double* x, const double* y,
                      const double* z) {
    for (int64_t s = 0; s < t->n; s++) {
        t->xs[s] = x[t->perm[s]];
        t->ys[s] = y[t->perm[s]];
        t->zs[s] = z[t->perm[s]];
    }
}

/* 1 when every particle at the new positions (caller order) lies within
 * (1/2 + slack) leaf sides of the centre of the leaf it was built into,
 * along each axis, else 0 (non-finite positions give 0).  slack = 0 is the
 * leaf's own closed box; a kept tree's expansions converge while the slack
 * leaves room inside the one-cell separation of the lists. */
int oracle_tree_stays(const otree* t, const double* x, const double* y,
                      const double* z, double slack) {
    for (int64_t s = 0; s < t->n; s++) {
        const ocell* c = &t->c[t->leaf_of[s]];
        double cc[3];
        cell_centre(t, c, cc);
        const double lim = (0.5 + slack) * cell_side(t, c->level);
        const int64_t i = t->perm[s];
        const double d[3] = {x[i] - cc[0], y[i] - cc[1], z[i] - cc[2]};
        for (int a = 0; a < 3; a++)
            if (!(fabs(d[a]) <= lim)) return 0;
    }
    return 1;
}

/* Closed boxes of A and B intersect (integer test, levels may differ). */
static int adjacent(const ocell* A, const ocell* B) {
    if (A->level > B->level) {
        const ocell* T = A;
        A = B;
        B = T;
    }
    int64_t f = (int64_t)1 << (B->level - A->level);
    int64_t ia[3] = {A->ix, A->iy, A->iz}, ib[3] = {B->ix, B->iy, B->iz};
    for (int a = 0; a < 3; a++) {
        if (ib[a] > (ia[a] + 1) * f) return 0;
        if (ib[a] + 1 < ia[a] * f) return 0;
    }
    return 1;
}

static int is_leaf(const ocell* c) { return c->nchild == 0; }

/* dynamic int list */
typedef struct {
    int32_t* v;
    int64_t n, cap;
} ivec;

static void ivec_push(ivec* a, int32_t x) {
    if (a->n == a->cap) {
        a->cap = a->cap ? 2 * a->cap : 32;
        a->v = (int32_t*)realloc(a->v, sizeof(int32_t) * a->cap);
    }
    a->v[a->n++] = x;
}

static void lists_from_vecs(otree* t, int w, ivec* L) {
    t->loff[w] = (int64_t*)malloc(sizeof(int64_t) * (t->ncells + 1));
    int64_t tot = 0;
    for (int64_t i = 0; i < t->ncells; i++) {
        t->loff[w][i] = tot;
        tot += L[i].n;
    }
    t->loff[w][t->ncells] = tot;
    t->litem[w] = (int32_t*)malloc(sizeof(int32_t) * (tot ? tot : 1));
    for (int64_t i = 0; i < t->ncells; i++) {
        if (L[i].n)
            memcpy(t->litem[w] + t->loff[w][i], L[i].v, sizeof(int32_t) * L[i].n);
        free(L[i].v);
    }
}

static void w_descend(const otree* t, int B, int C, ivec* U, ivec* W) {
    const ocell* cb = &t->c[B];
    for (int k = 0; k < t->c[C].nchild; k++) {
        int D = t->c[C].first_child + k;
        if (adjacent(&t->c[D], cb)) {
            if (is_leaf(&t->c[D]))
                ivec_push(U, D);
            else
                w_descend(t, B, D, U, W);
        } else {
            ivec_push(W, D);
        }
    }
}

/* Adaptive FMM lists (Cheng, Greengard and Rokhlin), built from colleagues:
 *   colleagues(B) = same-level cells adjacent to B (B included), found as the
 *                   children of colleagues(parent(B)) adjacent to B;
 *   U(B leaf)     = leaves adjacent to B (B included);
 *   V(B)          = children of colleagues(parent(B)) not adjacent to B;
 *   W(B leaf)     = descendants C of colleagues of B, C not adjacent to B,
 *                   parent(C) adjacent to B;
 *   X(B)          = cells C with B in W(C).                                 */
static void build_lists(otree* t) {
    if (t->lists_done) return;
    const int64_t nc = t->ncells;
    ivec* col = (ivec*)calloc(nc ? nc : 1, sizeof(ivec));
    if (nc > 0) ivec_push(&col[0], 0);
    for (int64_t b = 1; b < nc; b++) {
        int P = t->c[b].parent;
        for (int64_t k = 0; k < col[P].n; k++) {
            int C = col[P].v[k];
            for (int q = 0; q < t->c[C].nchild; q++) {
                int D = t->c[C].first_child + q;
                if (adjacent(&t->c[D], &t->c[b])) ivec_push(&col[b], D);
            }
        }
    }
    ivec* U = (ivec*)calloc(nc ? nc : 1, sizeof(ivec));
    ivec* V = (ivec*)calloc(nc ? nc : 1, sizeof(ivec));
    ivec* W = (ivec*)calloc(nc ? nc : 1, sizeof(ivec));
    ivec* X = (ivec*)calloc(nc ? nc : 1, sizeof(ivec));
    for (int64_t b = 0; b < nc; b++) {
        const ocell* cb = &t->c[b];
        if (b > 0) {
            int P = cb->parent;
            for (int64_t k = 0; k < col[P].n; k++) {
                int C = col[P].v[k];
                for (int q = 0; q < t->c[C].nchild; q++) {
                    int D = t->c[C].first_child + q;
                    if (!adjacent(&t->c[D], cb)) ivec_push(&V[b], D);
                }
            }
        }
        if (!is_leaf(cb)) continue;
        /* coarser adjacent leaves: leaf colleagues of proper ancestors */
        for (int A = cb->parent; A >= 0; A = t->c[A].parent)
            for (int64_t k = 0; k < col[A].n; k++) {
                int C = col[A].v[k];
                if (C != A && is_leaf(&t->c[C]) && adjacent(&t->c[C], cb))
                    ivec_push(&U[b], C);
            }
        /* same level, then finer adjacent leaves and W */
        for (int64_t k = 0; k < col[b].n; k++) {
            int C = col[b].v[k];
            if (is_leaf(&t->c[C]))
                ivec_push(&U[b], C);
            else if (C != b)
                w_descend(t, (int)b, C, &U[b], &W[b]);
        }
    }
    for (int64_t b = 0; b < nc; b++)
        for (int64_t k = 0; k < W[b].n; k++) ivec_push(&X[W[b].v[k]], (int32_t)b);
    for (int64_t b = 0; b < nc; b++) free(col[b].v);
    free(col);
    lists_from_vecs(t, 0, U);
    lists_from_vecs(t, 1, V);
    lists_from_vecs(t, 2, W);
    lists_from_vecs(t, 3, X);
    free(U);
    free(V);
    free(W);
    free(X);
    t->lists_done = 1;
}

int64_t oracle_list_size(otree* t, int which) {
    build_lists(t);
    return t->loff[which][t->ncells];
}

void oracle_list_get(otree* t, int which, int64_t* off, int32_t* items) {
    build_lists(t);
    memcpy(off, t->loff[which], sizeof(int64_t) * (t->ncells + 1));
    memcpy(items, t->litem[which], sizeof(int32_t) * t->loff[which][t->ncells]);
}

/* Brute force straight from the definitions, for cross-checking the
 * colleague-based construction on small trees. */
static int ancestor_at(const otree* t, int C, int level) {
    while (C >= 0 && t->c[C].level > level) C = t->c[C].parent;
    return C;
}

static int in_list_bf(const otree* t, int which, int B, int C) {
    const ocell *cb = &t->c[B], *cc = &t->c[C];
    switch (which) {
        case 0: /* U */
            return is_leaf(cb) && is_leaf(cc) && adjacent(cb, cc);
        case 1: /* V */
            return cb->level >= 1 && cc->level == cb->level &&
                   !adjacent(cb, cc) &&
                   adjacent(&t->c[cb->parent], &t->c[cc->parent]);
        case 2: { /* W */
            if (!is_leaf(cb) || cc->level <= cb->level) return 0;
            int A = ancestor_at(t, C, cb->level);
            return A != B && adjacent(&t->c[A], cb) && !adjacent(cc, cb) &&
                   adjacent(&t->c[cc->parent], cb);
        }
        default: { /* X: B in W(C) */
            if (!is_leaf(cc) || cb->level <= cc->level) return 0;
            int A = ancestor_at(t, B, cc->level);
            return A != C && adjacent(&t->c[A], cc) && !adjacent(cb, cc) &&
                   adjacent(&t->c[cb->parent], cc);
        }
    }
}

int64_t oracle_list_size_bruteforce(otree* t, int which) {
    int64_t tot = 0;
    for (int64_t b = 0; b < t->ncells; b++)
        for (int64_t c = 0; c < t->ncells; c++)
            tot += in_list_bf(t, which, (int)b, (int)c);
    return tot;
}

void oracle_list_get_bruteforce(otree* t, int which, int64_t* off,
                                int32_t* items) {
    int64_t tot = 0;
    for (int64_t b = 0; b < t->ncells; b++) {
        off[b] = tot;
        for (int64_t c = 0; c < t->ncells; c++)
            if (in_list_bf(t, which, (int)b, (int)c)) items[tot++] = (int32_t)c;
    }
    off[t->ncells] = tot;
}

/* ------------------------------------------------------------------ */
/* centres of mass and Barnes-Hut lists                                */
/* ------------------------------------------------------------------ */

void oracle_tree_com(otree* t, const double* m, double* comx, double* comy,
                     double* comz) {
    for (int64_t ci = 0; ci < t->ncells; ci++) {
        const ocell* c = &t->c[ci];
        double w = 0, sx = 0, sy = 0, sz = 0;
        for (int64_t i = c->first; i < c->first + c->count; i++) {
            double a = fabs(m[t->perm[i]]);
            w += a;
            sx += a * t->xs[i];
            sy += a * t->ys[i];
            sz += a * t->zs[i];
        }
        if (w > 0) {
            comx[ci] = sx / w;
            comy[ci] = sy / w;
            comz[ci] = sz / w;
        } else {
            double cc[3];
            cell_centre(t, c, cc);
            comx[ci] = cc[0];
            comy[ci] = cc[1];
            comz[ci] = cc[2];
        }
    }
}

static double dist_point_box(const double pnt[3], const double lo[3],
                             double side) {
    double d2 = 0;
    for (int a = 0; a < 3; a++) {
        double hi = lo[a] + side;
        double e = 0;
        if (pnt[a] < lo[a]) e = lo[a] - pnt[a];
        if (pnt[a] > hi) e = pnt[a] - hi;
        d2 += e * e;
    }
    return sqrt(d2);
}

static int is_ancestor_or_self(const otree* t, int A, int B) {
    for (int c = B; c >= 0; c = t->c[c].parent)
        if (c == A) return 1;
    return 0;
}

/* Barnes-Hut acceptance l < theta * d with d the distance from the centre of
 * mass of C to the closed box of target leaf B; B and its ancestors are never
 * accepted; a leaf that fails goes to P2P. */
static void bh_group(const otree* t, const double* com, double theta, int B,
                     int C, ivec* acc, ivec* near) {
    const ocell* cc = &t->c[C];
    if (is_ancestor_or_self(t, C, B)) {
        if (C == B) {
            ivec_push(near, C);
            return;
        }
        for (int k = 0; k < cc->nchild; k++)
            bh_group(t, com, theta, B, cc->first_child + k, acc, near);
        return;
    }
    const ocell* cb = &t->c[B];
    double hb = cell_side(t, cb->level);
    double lo[3] = {t->b[0] + cb->ix * hb, t->b[1] + cb->iy * hb,
                    t->b[2] + cb->iz * hb};
    double d = dist_point_box(&com[3 * C], lo, hb);
    if (cell_side(t, cc->level) < theta * d) {
        ivec_push(acc, C);
    } else if (is_leaf(cc)) {
        ivec_push(near, C);
    } else {
        for (int k = 0; k < cc->nchild; k++)
            bh_group(t, com, theta, B, cc->first_child + k, acc, near);
    }
}

static double* com_array(otree* t, const double* m) {
    double* cx = (double*)malloc(sizeof(double) * t->ncells * 3);
    double* tx = (double*)malloc(sizeof(double) * t->ncells);
    double* ty = (double*)malloc(sizeof(double) * t->ncells);
    double* tz = (double*)malloc(sizeof(double) * t->ncells);
    oracle_tree_com(t, m, tx, ty, tz);
    for (int64_t i = 0; i < t->ncells; i++) {
        cx[3 * i] = tx[i];
        cx[3 * i + 1] = ty[i];
        cx[3 * i + 2] = tz[i];
    }
    free(tx);
    free(ty);
    free(tz);
    return cx;
}

int64_t oracle_bh_lists(otree* t, const double* m, double theta, int which,
                        int64_t* off, int32_t* items) {
    double* com = com_array(t, m);
    int64_t tot = 0;
    for (int64_t b = 0; b < t->ncells; b++) {
        if (off) off[b] = tot;
        if (!is_leaf(&t->c[b])) continue;
        ivec acc = {0}, near = {0};
        bh_group(t, com, theta, (int)b, 0, &acc, &near);
        ivec* L = which == 0 ? &acc : &near;
        if (items && L->n) memcpy(items + tot, L->v, sizeof(int32_t) * L->n);
        tot += L->n;
        free(acc.v);
        free(near.v);
    }
    if (off) off[t->ncells] = tot;
    free(com);
    return tot;
}

/* ------------------------------------------------------------------ */
/* drivers                                                             */
/* ------------------------------------------------------------------ */

/* Masses in sorted order. */
static double* sorted_masses(const otree* t, const double* m) {
    double* ms = (double*)malloc(sizeof(double) * (t->n ? t->n : 1));
    for (int64_t i = 0; i < t->n; i++) ms[i] = m[t->perm[i]];
    return ms;
}

/* Upward pass: P2M at leaves about centre cen[3*c], then M2M level by level
 * from the deepest parents to the root. */
static void upward(const otree* t, const double* ms, int p, const double* cen,
                   cplx* M) {
    const int64_t nc = t->ncells, pp = (int64_t)p * p;
    memset(M, 0, sizeof(cplx) * nc * pp);
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t ci = 0; ci < nc; ci++) {
        const ocell* c = &t->c[ci];
        if (!is_leaf(c)) continue;
        p2m_c(p, &cen[3 * ci], c->count, t->xs + c->first, t->ys + c->first,
              t->zs + c->first, ms + c->first, M + ci * pp);
    }
    for (int lev = t->depth - 1; lev >= 0; lev--) {
#pragma omp parallel for schedule(dynamic, 4)
        for (int64_t ci = 0; ci < nc; ci++) {
            const ocell* c = &t->c[ci];
            if (c->level != lev || is_leaf(c)) continue;
            for (int k = 0; k < c->nchild; k++) {
                int64_t ch = c->first_child + k;
                m2m_c(p, &cen[3 * ch], &cen[3 * ci], M + ch * pp, M + ci * pp);
            }
        }
    }
}

static double* geometric_centres(const otree* t) {
    double* cen = (double*)malloc(sizeof(double) * 3 * (t->ncells ? t->ncells : 1));
    for (int64_t i = 0; i < t->ncells; i++) cell_centre(t, &t->c[i], &cen[3 * i]);
    return cen;
}

/* Downward pass into cells flagged in need[]: M2L over V, P2L over X, then
 * L2L from the parent (parents first). */
static void downward(otree* t, const double* ms, int p, const double* cen,
                     const cplx* M, cplx* L, const char* need) {
    const int64_t nc = t->ncells, pp = (int64_t)p * p;
    memset(L, 0, sizeof(cplx) * nc * pp);
#pragma omp parallel for schedule(dynamic, 2)
    for (int64_t b = 0; b < nc; b++) {
        if (need && !need[b]) continue;
        for (int64_t k = t->loff[1][b]; k < t->loff[1][b + 1]; k++) {
            int C = t->litem[1][k];
            m2l_c(p, &cen[3 * C], &cen[3 * b], M + C * pp, L + b * pp);
        }
        for (int64_t k = t->loff[3][b]; k < t->loff[3][b + 1]; k++) {
            const ocell* c = &t->c[t->litem[3][k]];
            p2l_c(p, &cen[3 * b], c->count, t->xs + c->first, t->ys + c->first,
                  t->zs + c->first, ms + c->first, L + b * pp);
        }
    }
    for (int lev = 1; lev <= t->depth; lev++) {
#pragma omp parallel for schedule(dynamic, 4)
        for (int64_t b = 0; b < nc; b++) {
            const ocell* c = &t->c[b];
            if (c->level != lev || (need && !need[b])) continue;
            l2l_c(p, &cen[3 * c->parent], &cen[3 * b], L + c->parent * pp,
                  L + b * pp);
        }
    }
}

int oracle_fmm_expansions(otree* t, const double* m, int p, double* M,
                          double* L) {
    build_lists(t);
    double* ms = sorted_masses(t, m);
    double* cen = geometric_centres(t);
    upward(t, ms, p, cen, (cplx*)M);
    downward(t, ms, p, cen, (const cplx*)M, (cplx*)L, NULL);
    free(ms);
    free(cen);
    return 0;
}

static int64_t* inverse_perm(const otree* t) {
    int64_t* inv = (int64_t*)malloc(sizeof(int64_t) * (t->n ? t->n : 1));
    for (int64_t s = 0; s < t->n; s++) inv[t->perm[s]] = s;
    return inv;
}

int oracle_fmm_tree(otree* t, const double* m, int p, double eps2, int64_t nt,
                    const int64_t* tidx, double* phi, double* ax, double* ay,
                    double* az) {
    if (tidx == NULL) nt = t->n;
    if (t->n == 0 || nt == 0) return 0;
    build_lists(t);
    const int64_t nc = t->ncells, pp = (int64_t)p * p;
    double* ms = sorted_masses(t, m);
    double* cen = geometric_centres(t);
    int64_t* inv = inverse_perm(t);
    char* need = NULL;
    if (tidx) { /* only the leaves holding targets and their ancestors */
        need = (char*)calloc(nc, 1);
        for (int64_t k = 0; k < nt; k++)
            for (int c = t->leaf_of[inv[tidx[k]]]; c >= 0 && !need[c];
                 c = t->c[c].parent)
                need[c] = 1;
    }
    cplx* M = (cplx*)malloc(sizeof(cplx) * nc * pp);
    cplx* L = (cplx*)malloc(sizeof(cplx) * nc * pp);
    double t0 = wall_s();
    upward(t, ms, p, cen, M);
    double t1 = wall_s();
    downward(t, ms, p, cen, M, L, need);
    double t2 = wall_s();
    g_phase_s[0] = t1 - t0;
    g_phase_s[1] = t2 - t1;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t k = 0; k < nt; k++) {
        int64_t s = inv[tidx ? tidx[k] : k];
        int b = t->leaf_of[s];
        double xt[3] = {t->xs[s], t->ys[s], t->zs[s]};
        double acc[4] = {0, 0, 0, 0}, o[4];
        oracle_l2p(p, &cen[3 * b], (const double*)(L + b * pp), xt, o);
        for (int a = 0; a < 4; a++) acc[a] += o[a];
        for (int64_t q = t->loff[2][b]; q < t->loff[2][b + 1]; q++) {
            int C = t->litem[2][q];
            oracle_m2p(p, &cen[3 * C], (const double*)(M + C * pp), xt, o);
            for (int a = 0; a < 4; a++) acc[a] += o[a];
        }
        for (int64_t q = t->loff[0][b]; q < t->loff[0][b + 1]; q++) {
            const ocell* c = &t->c[t->litem[0][q]];
            p2p_point(xt, c->first, c->first + c->count, t->xs, t->ys, t->zs,
                      ms, eps2, acc);
        }
        phi[k] = acc[0];
        ax[k] = acc[1];
        ay[k] = acc[2];
        az[k] = acc[3];
    }
    g_phase_s[2] = wall_s() - t2;
    free(need);
    free(M);
    free(L);
    free(inv);
    free(cen);
    free(ms);
    return 0;
}

int oracle_fmm(int64_t n, const double* x, const double* y, const double* z,
               const double* m, int leaf_max, int p, double eps2, int64_t nt,
               const int64_t* tidx, double* phi, double* ax, double* ay,
               double* az) {
    if (tidx == NULL) nt = n;
    if (n == 0 || nt == 0) return 0;
    otree* t = oracle_tree_build(n, x, y, z, leaf_max);
    int rc = oracle_fmm_tree(t, m, p, eps2, nt, tidx, phi, ax, ay, az);
    oracle_tree_free(t);
    return rc;
}

/* per-particle Barnes-Hut traversal for one target at sorted position s */
static void bh_point(const otree* t, const double* com, const cplx* M, int p,
                     double theta, const double* ms, double eps2, int64_t s,
                     int C, double acc[4]) {
    const ocell* cc = &t->c[C];
    const int64_t pp = (int64_t)p * p;
    double xt[3] = {t->xs[s], t->ys[s], t->zs[s]};
    if (is_ancestor_or_self(t, C, t->leaf_of[s])) {
        if (is_leaf(cc)) {
            p2p_point(xt, cc->first, cc->first + cc->count, t->xs, t->ys,
                      t->zs, ms, eps2, acc);
            return;
        }
        for (int k = 0; k < cc->nchild; k++)
            bh_point(t, com, M, p, theta, ms, eps2, s, cc->first_child + k, acc);
        return;
    }
    double d[3] = {xt[0] - com[3 * C], xt[1] - com[3 * C + 1],
                   xt[2] - com[3 * C + 2]};
    double dist = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
    if (cell_side(t, cc->level) < theta * dist) {
        double o[4];
        oracle_m2p(p, &com[3 * C], (const double*)(M + C * pp), xt, o);
        for (int a = 0; a < 4; a++) acc[a] += o[a];
    } else if (is_leaf(cc)) {
        p2p_point(xt, cc->first, cc->first + cc->count, t->xs, t->ys, t->zs,
                  ms, eps2, acc);
    } else {
        for (int k = 0; k < cc->nchild; k++)
            bh_point(t, com, M, p, theta, ms, eps2, s, cc->first_child + k, acc);
    }
}

/* The treecode of Sec. 4: the FMM's interaction lists with every M2L + L2L +
 * L2P replaced by one M2P at the target.  For a target in leaf B the far
 * field is M2P from the V lists of B and of each ancestor of B and from the
 * W list of B; the near field is P2P with the U list of B and the X lists of
 * B and of each ancestor of B (X sources are leaves too close to B's
 * particles for their multipole expansions, which the FMM reaches through
 * P2L).  Together these cover every source particle once. */
static void fmm_list_point(const otree* t, const double* cen, const cplx* M,
                           int p, const double* ms, double eps2, int64_t s,
                           double acc[4]) {
    const int64_t pp = (int64_t)p * p;
    const int B = t->leaf_of[s];
    double xt[3] = {t->xs[s], t->ys[s], t->zs[s]}, o[4];
    for (int a = B; a >= 0; a = t->c[a].parent) {
        for (int64_t q = t->loff[1][a]; q < t->loff[1][a + 1]; q++) {
            int C = t->litem[1][q];
            oracle_m2p(p, &cen[3 * C], (const double*)(M + C * pp), xt, o);
            for (int i = 0; i < 4; i++) acc[i] += o[i];
        }
        for (int64_t q = t->loff[3][a]; q < t->loff[3][a + 1]; q++) {
            const ocell* c = &t->c[t->litem[3][q]];
            p2p_point(xt, c->first, c->first + c->count, t->xs, t->ys, t->zs,
                      ms, eps2, acc);
        }
    }
    for (int64_t q = t->loff[2][B]; q < t->loff[2][B + 1]; q++) {
        int C = t->litem[2][q];
        oracle_m2p(p, &cen[3 * C], (const double*)(M + C * pp), xt, o);
        for (int i = 0; i < 4; i++) acc[i] += o[i];
    }
    for (int64_t q = t->loff[0][B]; q < t->loff[0][B + 1]; q++) {
        const ocell* c = &t->c[t->litem[0][q]];
        p2p_point(xt, c->first, c->first + c->count, t->xs, t->ys, t->zs, ms,
                  eps2, acc);
    }
}

int oracle_treecode_tree(otree* t, const double* m, int p, double theta,
                         int mode, double eps2, int64_t nt,
                         const int64_t* tidx, double* phi, double* ax,
                         double* ay, double* az) {
    if (tidx == NULL) nt = t->n;
    if (t->n == 0 || nt == 0) return 0;
    const int64_t nc = t->ncells, pp = (int64_t)p * p;
    double* ms = sorted_masses(t, m);
    /* mode 2 expands about the geometric centres, as the FMM does */
    double* com = mode == 2 ? geometric_centres(t) : com_array(t, m);
    int64_t* inv = inverse_perm(t);
    cplx* M = (cplx*)malloc(sizeof(cplx) * nc * pp);
    if (mode == 2) build_lists(t);
    upward(t, ms, p, com, M);
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t k = 0; k < nt; k++) {
        int64_t s = inv[tidx ? tidx[k] : k];
        double acc[4] = {0, 0, 0, 0};
        if (mode == 2) {
            fmm_list_point(t, com, M, p, ms, eps2, s, acc);
        } else if (mode == 1) {
            bh_point(t, com, M, p, theta, ms, eps2, s, 0, acc);
        } else {
            int b = t->leaf_of[s];
            ivec accl = {0}, near = {0};
            bh_group(t, com, theta, b, 0, &accl, &near);
            double xt[3] = {t->xs[s], t->ys[s], t->zs[s]}, o[4];
            for (int64_t q = 0; q < accl.n; q++) {
                int C = accl.v[q];
                oracle_m2p(p, &com[3 * C], (const double*)(M + C * pp), xt, o);
                for (int a = 0; a < 4; a++) acc[a] += o[a];
            }
            for (int64_t q = 0; q < near.n; q++) {
                const ocell* c = &t->c[near.v[q]];
                p2p_point(xt, c->first, c->first + c->count, t->xs, t->ys,
                          t->zs, ms, eps2, acc);
            }
            free(accl.v);
            free(near.v);
        }
        phi[k] = acc[0];
        ax[k] = acc[1];
        ay[k] = acc[2];
        az[k] = acc[3];
    }
    free(M);
    free(inv);
    free(com);
    free(ms);
    return 0;
}

int oracle_treecode(int64_t n, const double* x, const double* y,
                    const double* z, const double* m, int leaf_max, int p,
                    double theta, int mode, double eps2, int64_t nt,
                    const int64_t* tidx, double* phi, double* ax, double* ay,
                    double* az) {
    if (tidx == NULL) nt = n;
    if (n == 0 || nt == 0) return 0;
    otree* t = oracle_tree_build(n, x, y, z, leaf_max);
    int rc = oracle_treecode_tree(t, m, p, theta, mode, eps2, nt, tidx, phi,
                                  ax, ay, az);
    oracle_tree_free(t);
    return rc;
}

/* ------------------------------------------------------------------ */
/* separate targets, binned into the source tree                       */
/* ------------------------------------------------------------------ */

/* The box a target point is binned into.  The point's key prefix is
 * followed down the source tree as far as cells exist:
 *   kind 0: it ends in a leaf L: the box is L (host = leaf = L);
 *   kind 1: it ends in a split cell H whose octant holding the point is
 *           empty: the box is that octant, a source-free leaf child of H
 *           (host = H, leaf = -1);
 *   kind 2: the point lies outside the root cube: the box is the
 *           root-sized cube of the grid extended beyond the root that holds
 *           it, at level 0 (host = leaf = -1; coordinates clamped to
 *           +-2^20 root widths, far beyond any adjacency).
 * A box of kind 1 or 2 is a leaf without sources added to the tree; the
 * lists the adaptive FMM defines for a leaf (Cheng, Greengard and Rokhlin,
 * cited in Sec. 6) are defined for it alike. */
typedef struct {
    int kind, level, host, leaf;
    int64_t q[3];
} obox;

static int adj_g(int la, const int64_t a[3], int lb, const int64_t b[3]) {
    if (la > lb) {
        const int64_t* s = a;
        a = b;
        b = s;
        int l = la;
        la = lb;
        lb = l;
    }
    int64_t f = (int64_t)1 << (lb - la);
    for (int k = 0; k < 3; k++) {
        if (b[k] > (a[k] + 1) * f) return 0;
        if (b[k] + 1 < a[k] * f) return 0;
    }
    return 1;
}

static void cell_q(const ocell* c, int64_t q[3]) {
    q[0] = c->ix;
    q[1] = c->iy;
    q[2] = c->iz;
}

static int adj_box_cell(const otree* t, const obox* B, int C) {
    int64_t q[3];
    cell_q(&t->c[C], q);
    return adj_g(B->level, B->q, t->c[C].level, q);
}

static obox bin_target(const otree* t, const double xt[3]) {
    const double s = (double)(1 << KBITS) / (2.0 * t->R);
    const double top = (double)(1 << KBITS);
    double f[3];
    int outside = 0;
    for (int a = 0; a < 3; a++) {
        f[a] = floor((xt[a] - t->b[a]) * s);
        /* the upper face belongs to the cube, as for the sources' keys */
        if (!(f[a] >= 0.0 && f[a] <= top)) outside = 1;
    }
    obox B;
    if (outside) {
        B.kind = 2;
        B.level = 0;
        B.host = B.leaf = -1;
        for (int a = 0; a < 3; a++) {
            double c = floor(f[a] / top);
            if (c > 1048576.0) c = 1048576.0;
            if (c < -1048576.0) c = -1048576.0;
            B.q[a] = (int64_t)c;
        }
        return B;
    }
    int64_t qf[3];
    for (int a = 0; a < 3; a++) qf[a] = f[a] > top - 1.0 ? (1 << KBITS) - 1 : (int64_t)f[a];
    int C = 0;
    for (;;) {
        const ocell* c = &t->c[C];
        if (is_leaf(c)) {
            B.kind = 0;
            B.level = c->level;
            B.host = B.leaf = C;
            cell_q(c, B.q);
            return B;
        }
        const int lev = c->level + 1;
        int64_t q[3];
        for (int a = 0; a < 3; a++) q[a] = qf[a] >> (KBITS - lev);
        int next = -1;
        for (int k = 0; k < c->nchild; k++) {
            const ocell* d = &t->c[c->first_child + k];
            if (d->ix == q[0] && d->iy == q[1] && d->iz == q[2]) next = c->first_child + k;
        }
        if (next < 0) {
            B.kind = 1;
            B.level = lev;
            B.host = C;
            B.leaf = -1;
            for (int a = 0; a < 3; a++) B.q[a] = q[a];
            return B;
        }
        C = next;
    }
}

/* The parent cell of a box (-1 for the root and for boxes outside it). */
static int box_parent(const otree* t, const obox* B) {
    if (B->kind == 0) return t->c[B->leaf].parent;
    return B->kind == 1 ? B->host : -1;
}

/* Is cell C the box itself or one of its ancestors? */
static int box_within(const otree* t, const obox* B, int C) {
    int A = B->kind == 0 ? B->leaf : B->host;
    for (; A >= 0; A = t->c[A].parent)
        if (A == C) return 1;
    return 0;
}

/* The four lists of box B, straight from their definitions, over every
 * cell:
 *   U: leaves adjacent to B (B included when it is a leaf of the tree);
 *   V: cells of B's level, not adjacent to B, whose parents are adjacent to
 *      B's parent (outside the root: the root when not adjacent to B);
 *   W: cells C finer than B, not adjacent to B, whose parent is adjacent to
 *      B, below a cell of B's level adjacent to B (other than B);
 *   X: leaves C coarser than B, not adjacent to B but adjacent to B's
 *      parent, whose cell at C's level on B's ancestor line is adjacent to
 *      C (and not C): the cells with B in their W list. */
static void box_lists(const otree* t, const obox* B, ivec L[4]) {
    const int P = box_parent(t, B);
    for (int C = 0; C < (int)t->ncells; C++) {
        const ocell* cc = &t->c[C];
        const int adj = adj_box_cell(t, B, C);
        if (is_leaf(cc) && adj) ivec_push(&L[0], C);
        if (cc->level == B->level && !adj) {
            if (B->kind == 2 ? C == 0
                             : (P >= 0 && cc->parent >= 0 && adjacent(&t->c[cc->parent], &t->c[P])))
                ivec_push(&L[1], C);
        }
        if (cc->level > B->level && !adj && adj_box_cell(t, B, cc->parent)) {
            int A = ancestor_at(t, C, B->level);
            if (A != B->leaf && adj_box_cell(t, B, A)) ivec_push(&L[2], C);
        }
        if (is_leaf(cc) && cc->level < B->level && !adj && P >= 0 && adjacent(cc, &t->c[P])) {
            int A = ancestor_at(t, B->kind == 0 ? B->leaf : B->host, cc->level);
            if (A != C && adjacent(&t->c[A], cc)) ivec_push(&L[3], C);
        }
    }
}

void oracle_target_boxes(otree* t, int64_t nt, const double* tx, const double* ty,
                         const double* tz, int64_t* out) {
    for (int64_t k = 0; k < nt; k++) {
        double xt[3] = {tx[k], ty[k], tz[k]};
        obox B = bin_target(t, xt);
        int64_t* o = out + 7 * k;
        o[0] = B.kind;
        o[1] = B.level;
        o[2] = B.q[0];
        o[3] = B.q[1];
        o[4] = B.q[2];
        o[5] = B.host;
        o[6] = B.leaf;
    }
}

int64_t oracle_box_list(otree* t, const double xt[3], int which, int32_t* items) {
    obox B = bin_target(t, xt);
    ivec L[4] = {{0}, {0}, {0}, {0}};
    box_lists(t, &B, L);
    int64_t n = L[which].n;
    if (items && n) memcpy(items, L[which].v, sizeof(int32_t) * n);
    for (int w = 0; w < 4; w++) free(L[w].v);
    return n;
}

static void m2p_cells(const otree* t, const double* cen, const cplx* M, int p, const ivec* l,
                      const double xt[3], double acc[4]) {
    const int64_t pp = (int64_t)p * p;
    double o[4];
    for (int64_t q = 0; q < l->n; q++) {
        int C = l->v[q];
        oracle_m2p(p, &cen[3 * C], (const double*)(M + C * pp), xt, o);
        for (int a = 0; a < 4; a++) acc[a] += o[a];
    }
}

static void p2p_cells(const otree* t, const double* ms, double eps2, const ivec* l,
                      const double xt[3], double acc[4]) {
    for (int64_t q = 0; q < l->n; q++) {
        const ocell* c = &t->c[l->v[q]];
        p2p_point(xt, c->first, c->first + c->count, t->xs, t->ys, t->zs, ms, eps2, acc);
    }
}

/* FMM at separate target points.  For a target in box B with host H (the
 * cell whose local expansion covers B):
 *   phi = L2P(L(H)) + M2P over W(B) + P2P over U(B)          (B a leaf),
 * and for a box without sources, which has no local expansion of its own,
 * its V list by M2P and its X list by P2P as well, at the target itself:
 *   phi = L2P(L(H)) + M2P over V(B), W(B) + P2P over U(B), X(B)
 * (no L2P outside the root).  Every source is reached once. */
int oracle_fmm_points_tree(otree* t, const double* m, int p, double eps2, int64_t nt,
                           const double* tx, const double* ty, const double* tz,
                           double* phi, double* ax, double* ay, double* az) {
    if (nt == 0) return 0;
    if (t->n == 0) {
        for (int64_t k = 0; k < nt; k++) phi[k] = ax[k] = ay[k] = az[k] = 0.0;
        return 0;
    }
    build_lists(t);
    const int64_t nc = t->ncells, pp = (int64_t)p * p;
    double* ms = sorted_masses(t, m);
    double* cen = geometric_centres(t);
    cplx* M = (cplx*)malloc(sizeof(cplx) * nc * pp);
    cplx* L = (cplx*)malloc(sizeof(cplx) * nc * pp);
    upward(t, ms, p, cen, M);
    downward(t, ms, p, cen, M, L, NULL);
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t k = 0; k < nt; k++) {
        double xt[3] = {tx[k], ty[k], tz[k]};
        obox B = bin_target(t, xt);
        ivec l[4] = {{0}, {0}, {0}, {0}};
        box_lists(t, &B, l);
        double acc[4] = {0, 0, 0, 0}, o[4];
        if (B.host >= 0) {
            oracle_l2p(p, &cen[3 * B.host], (const double*)(L + B.host * pp), xt, o);
            for (int a = 0; a < 4; a++) acc[a] += o[a];
        }
        m2p_cells(t, cen, M, p, &l[2], xt, acc);
        p2p_cells(t, ms, eps2, &l[0], xt, acc);
        if (B.kind != 0) {
            m2p_cells(t, cen, M, p, &l[1], xt, acc);
            p2p_cells(t, ms, eps2, &l[3], xt, acc);
        }
        for (int w = 0; w < 4; w++) free(l[w].v);
        phi[k] = acc[0];
        ax[k] = acc[1];
        ay[k] = acc[2];
        az[k] = acc[3];
    }
    free(M);
    free(L);
    free(cen);
    free(ms);
    return 0;
}

int oracle_fmm_points(int64_t n, const double* x, const double* y, const double* z,
                      const double* m, int leaf_max, int p, double eps2, int64_t nt,
                      const double* tx, const double* ty, const double* tz, double* phi,
                      double* ax, double* ay, double* az) {
    if (nt == 0) return 0;
    if (n == 0) {
        for (int64_t k = 0; k < nt; k++) phi[k] = ax[k] = ay[k] = az[k] = 0.0;
        return 0;
    }
    otree* t = oracle_tree_build(n, x, y, z, leaf_max);
    int rc = oracle_fmm_points_tree(t, m, p, eps2, nt, tx, ty, tz, phi, ax, ay, az);
    oracle_tree_free(t);
    return rc;
}

/* Barnes-Hut traversal for a target box (the group acceptance of mode 0):
 * cells containing the box are opened, the box's own leaf goes to P2P, other
 * cells are accepted when l < theta d (d from the centre of mass to the
 * box), else a leaf goes to P2P and a split cell is opened. */
static void bh_box(const otree* t, const double* com, double theta, const obox* B, int C,
                   ivec* acc, ivec* near) {
    const ocell* cc = &t->c[C];
    if (box_within(t, B, C)) {
        if (C == B->leaf) {
            ivec_push(near, C);
            return;
        }
        for (int k = 0; k < cc->nchild; k++)
            bh_box(t, com, theta, B, cc->first_child + k, acc, near);
        return;
    }
    const double hb = cell_side(t, 0) / (double)((int64_t)1 << B->level);
    double lo[3];
    for (int a = 0; a < 3; a++) lo[a] = t->b[a] + (double)B->q[a] * hb;
    double d = dist_point_box(&com[3 * C], lo, hb);
    if (cell_side(t, cc->level) < theta * d) {
        ivec_push(acc, C);
    } else if (is_leaf(cc)) {
        ivec_push(near, C);
    } else {
        for (int k = 0; k < cc->nchild; k++)
            bh_box(t, com, theta, B, cc->first_child + k, acc, near);
    }
}

/* Treecode at separate target points: mode 0, Barnes-Hut group lists of the
 * target's box about the centres of mass; mode 2, the treecode of Sec. 4
 * over the FMM lists of the box: M2P over V and W of the box and V of each
 * ancestor, P2P over U and X of the box and X of each ancestor (expansions
 * about the geometric centres). */
int oracle_treecode_points_tree(otree* t, const double* m, int p, double theta,
                                int mode, double eps2, int64_t nt, const double* tx,
                                const double* ty, const double* tz, double* phi,
                                double* ax, double* ay, double* az) {
    if (nt == 0) return 0;
    if (mode != 0 && mode != 2) return -1;
    if (t->n == 0) {
        for (int64_t k = 0; k < nt; k++) phi[k] = ax[k] = ay[k] = az[k] = 0.0;
        return 0;
    }
    const int64_t nc = t->ncells, pp = (int64_t)p * p;
    double* ms = sorted_masses(t, m);
    double* cen = mode == 2 ? geometric_centres(t) : com_array(t, m);
    cplx* M = (cplx*)malloc(sizeof(cplx) * nc * pp);
    if (mode == 2) build_lists(t);
    upward(t, ms, p, cen, M);
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t k = 0; k < nt; k++) {
        double xt[3] = {tx[k], ty[k], tz[k]};
        obox B = bin_target(t, xt);
        double acc[4] = {0, 0, 0, 0};
        if (mode == 0) {
            ivec a = {0}, b = {0};
            bh_box(t, cen, theta, &B, 0, &a, &b);
            m2p_cells(t, cen, M, p, &a, xt, acc);
            p2p_cells(t, ms, eps2, &b, xt, acc);
            free(a.v);
            free(b.v);
        } else {
            ivec l[4] = {{0}, {0}, {0}, {0}};
            box_lists(t, &B, l);
            ivec far = {0}, near = {0};
            for (int64_t q = 0; q < l[1].n; q++) ivec_push(&far, l[1].v[q]);
            for (int64_t q = 0; q < l[2].n; q++) ivec_push(&far, l[2].v[q]);
            for (int64_t q = 0; q < l[0].n; q++) ivec_push(&near, l[0].v[q]);
            for (int64_t q = 0; q < l[3].n; q++) ivec_push(&near, l[3].v[q]);
            for (int A = box_parent(t, &B); A >= 0; A = t->c[A].parent) {
                for (int64_t q = t->loff[1][A]; q < t->loff[1][A + 1]; q++)
                    ivec_push(&far, t->litem[1][q]);
                for (int64_t q = t->loff[3][A]; q < t->loff[3][A + 1]; q++)
                    ivec_push(&near, t->litem[3][q]);
            }
            m2p_cells(t, cen, M, p, &far, xt, acc);
            p2p_cells(t, ms, eps2, &near, xt, acc);
            for (int w = 0; w < 4; w++) free(l[w].v);
            free(far.v);
            free(near.v);
        }
        phi[k] = acc[0];
        ax[k] = acc[1];
        ay[k] = acc[2];
        az[k] = acc[3];
    }
    free(M);
    free(cen);
    free(ms);
    return 0;
}

int oracle_treecode_points(int64_t n, const double* x, const double* y, const double* z,
                           const double* m, int leaf_max, int p, double theta, int mode,
                           double eps2, int64_t nt, const double* tx, const double* ty,
                           const double* tz, double* phi, double* ax, double* ay,
                           double* az) {
    if (mode != 0 && mode != 2) return -1;
    if (nt == 0) return 0;
    if (n == 0) {
        for (int64_t k = 0; k < nt; k++) phi[k] = ax[k] = ay[k] = az[k] = 0.0;
        return 0;
    }
    otree* t = oracle_tree_build(n, x, y, z, leaf_max);
    int rc = oracle_treecode_points_tree(t, m, p, theta, mode, eps2, nt, tx, ty, tz, phi,
                                          ax, ay, az);
    oracle_tree_free(t);
    return rc;
}

/* ------------------------------------------------------------------ */
/* rotation-based M2L                                                  */
/* ------------------------------------------------------------------ */

#define ORACLE_PI 3.14159265358979323846

/* Gauss-Legendre nodes and weights on [-1, 1] (Newton on P_N from the usual
 * cosine guesses). */
static void gauss_legendre(int N, double* x, double* w) {
    for (int i = 0; i < N; i++) {
        double z = cos(ORACLE_PI * (i + 0.75) / (N + 0.5)), dp = 1.0;
        for (int it = 0; it < 100; it++) {
            double p0 = 1.0, p1 = z;
            for (int k = 2; k <= N; k++) {
                double pk = ((2 * k - 1) * z * p1 - (k - 1) * p0) / k;
                p0 = p1;
                p1 = pk;
            }
            dp = N * (z * p1 - p0) / (z * z - 1.0);
            double dz = p1 / dp;
            z -= dz;
            if (fabs(dz) < 1e-16) break;
        }
        /* final derivative at the converged node */
        double p0 = 1.0, p1 = z;
        for (int k = 2; k <= N; k++) {
            double pk = ((2 * k - 1) * z * p1 - (k - 1) * p0) / k;
            p0 = p1;
            p1 = pk;
        }
        dp = N * (z * p1 - p0) / (z * z - 1.0);
        x[i] = z;
        w[i] = 2.0 / ((1.0 - z * z) * dp * dp);
    }
}

/* out = R v for a 3x3 row-major R */
static void mat3(const double R[9], const double v[3], double out[3]) {
    for (int a = 0; a < 3; a++) out[a] = R[3 * a] * v[0] + R[3 * a + 1] * v[1] + R[3 * a + 2] * v[2];
}

/* Re-expand the degree-n part of an expansion after a rotation of the frame:
 * out^m = (2n+1)/(4 pi) * integral over the unit sphere of
 * g(Q u) conj(Y_n^m(u)), g(v) = sum_k in^k Y_n^k(v), which is exact for the
 * degree-n harmonic g (the Y_n^m are orthogonal with norm 4 pi / (2n+1)).
 * The quadrature, Gauss-Legendre in cos a (n + 1 nodes) times the trapezoid
 * rule in b (2n + 1 nodes), integrates degree 2n exactly. */
static void rotate_degree(int n, const double Q[9], const cplx* in, cplx* out) {
    const int nt = n + 1, nb = 2 * n + 1;
    double* gx = (double*)malloc(sizeof(double) * nt);
    double* gw = (double*)malloc(sizeof(double) * nt);
    gauss_legendre(nt, gx, gw);
    cplx* Yu = (cplx*)malloc(sizeof(cplx) * (n + 1) * (n + 1));
    cplx* Yq = (cplx*)malloc(sizeof(cplx) * (n + 1) * (n + 1));
    for (int m = -n; m <= n; m++) out[m + n] = 0;
    for (int a = 0; a < nt; a++)
        for (int b = 0; b < nb; b++) {
            const double ca = gx[a], sa = sqrt(fmax(0.0, 1.0 - ca * ca));
            const double be = 2.0 * ORACLE_PI * b / nb;
            const double u[3] = {sa * cos(be), sa * sin(be), ca};
            double v[3], rho, al, bq;
            mat3(Q, u, v);
            cart2sph(v, &rho, &al, &bq);
            ynm_table(n, acos(ca), be, Yu);
            ynm_table(n, al, bq, Yq);
            cplx g = 0;
            for (int k = -n; k <= n; k++) g += in[k + n] * Yq[CI(n, k)];
            const double wq = gw[a] * 2.0 * ORACLE_PI / nb;
            for (int m = -n; m <= n; m++) out[m + n] += wq * g * conj(Yu[CI(n, m)]);
        }
    for (int m = -n; m <= n; m++) out[m + n] *= (2.0 * n + 1.0) / (4.0 * ORACLE_PI);
    free(gx);
    free(gw);
    free(Yu);
    free(Yq);
}

/* Rotate a whole expansion (degrees < p): coefficients of the field
 * u -> f(Q u) */
static void rotate_expansion(int p, const double Q[9], const cplx* in, cplx* out) {
    cplx* tmp = (cplx*)malloc(sizeof(cplx) * (2 * p + 1));
    for (int n = 0; n < p; n++) {
        rotate_degree(n, Q, in + n * n, tmp);
        for (int m = -n; m <= n; m++) out[CI(n, m)] = tmp[m + n];
    }
    free(tmp);
}

/* The O(p^3) M2L that Sec. 6 lists among the advanced techniques: rotate the
 * multipole expansion into the frame whose z axis points along
 * c_tgt - c_src, translate along that axis (Eq. 4 with the translation on
 * the z axis couples each order m to itself only), and rotate the local
 * expansion back.  R = R_y(-alpha) R_z(-beta) takes the direction (alpha,
 * beta) to the z axis. */
void oracle_m2l_rot(int p, const double c_src[3], const double c_tgt[3], const double* M,
                    double* L) {
    const double d[3] = {c_tgt[0] - c_src[0], c_tgt[1] - c_src[1], c_tgt[2] - c_src[2]};
    double rho, al, be;
    cart2sph(d, &rho, &al, &be);
    const double ca = cos(al), sa = sin(al), cb = cos(be), sb = sin(be);
    /* R = R_y(-al) R_z(-be) */
    const double Rz[9] = {cb, sb, 0, -sb, cb, 0, 0, 0, 1};
    const double Ry[9] = {ca, 0, -sa, 0, 1, 0, sa, 0, ca};
    double R[9], Rt[9];
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) {
            R[3 * i + j] = 0;
            for (int k = 0; k < 3; k++) R[3 * i + j] += Ry[3 * i + k] * Rz[3 * k + j];
        }
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) Rt[3 * i + j] = R[3 * j + i];
    const int pp = p * p;
    cplx* Mr = (cplx*)calloc(pp, sizeof(cplx));
    cplx* Lr = (cplx*)calloc(pp, sizeof(cplx));
    cplx* Lb = (cplx*)malloc(sizeof(cplx) * pp);
    /* multipole in the rotated frame: the field u -> f(R^T u) */
    rotate_expansion(p, Rt, (const cplx*)M, Mr);
    const double zero[3] = {0, 0, 0}, zt[3] = {0, 0, rho};
    m2l_c(p, zero, zt, Mr, Lr);
    /* local expansion back in the original frame: u -> g(R u) */
    rotate_expansion(p, R, Lr, Lb);
    for (int k = 0; k < pp; k++) ((cplx*)L)[k] += Lb[k];
    free(Mr);
    free(Lr);
    free(Lb);
}

/* One rotation of an expansion, exposed for the pins: out = coefficients of
 * u -> f(Q u). */
void oracle_rotate(int p, const double Q[9], const double* in, double* out) {
    rotate_expansion(p, Q, (const cplx*)in, (cplx*)out);
}
