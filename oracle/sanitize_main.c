/*
 * Driver for a sanitizer build of the oracle (AddressSanitizer and
 * UndefinedBehaviorSanitizer on the CPU): every entry point of
 * hfmm_oracle.h runs once on small seeded inputs (a clustered set, so that
 * the tree is adaptive and every list kind is non-empty, plus the empty and
 * single-particle cases).  It checks nothing numerically (the pinned tests
 * do); a memory or undefined-behaviour error aborts the run with a report.
 *
 * TEST INFRASTRUCTURE ONLY, like the oracle itself.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

#include "hfmm_oracle.h"

static uint64_t g_state = 0x9e3779b97f4a7c15ull;

static double uniform01(void) { /* splitmix64 */
    uint64_t z = (g_state += 0x9e3779b97f4a7c15ull);
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    z ^= z >> 31;
    return (double)(z >> 11) * (1.0 / 9007199254740992.0);
}

static void run_set(int64_t n, int leaf, int p) {
    double* x = malloc(sizeof(double) * (n + 1));
    double* y = malloc(sizeof(double) * (n + 1));
    double* z = malloc(sizeof(double) * (n + 1));
    double* m = malloc(sizeof(double) * (n + 1));
    for (int64_t i = 0; i < n; i++) {
        /* half in a small cluster: an adaptive tree with W and X lists */
        const double s = (i % 2) ? 0.02 : 1.0;
        x[i] = s * uniform01();
        y[i] = s * uniform01();
        z[i] = s * uniform01();
        m[i] = (i % 3 == 0 ? -1.0 : 1.0) * (0.5 + uniform01());
    }
    const int64_t nt = n < 16 ? n : 16;
    int64_t* tidx = malloc(sizeof(int64_t) * (nt + 1));
    for (int64_t k = 0; k < nt; k++) tidx[k] = (k * 7) % (n > 0 ? n : 1);
    double* o[4];
    for (int a = 0; a < 4; a++) o[a] = calloc((size_t)(n + 16), sizeof(double));
    double tx[16], ty[16], tz[16];
    for (int k = 0; k < 16; k++) {
        tx[k] = 3.0 * uniform01() - 1.0;
        ty[k] = 3.0 * uniform01() - 1.0;
        tz[k] = 3.0 * uniform01() - 1.0;
    }

    oracle_direct(n, x, y, z, m, nt, tidx, 0.0, o[0], o[1], o[2], o[3]);
    oracle_direct_points(n, x, y, z, m, 16, tx, ty, tz, 1e-6, o[0], o[1], o[2], o[3]);
    oracle_fmm(n, x, y, z, m, leaf, p, 0.0, nt, tidx, o[0], o[1], o[2], o[3]);
    oracle_fmm(n, x, y, z, m, leaf, p, 0.0, 0, NULL, o[0], o[1], o[2], o[3]);
    for (int mode = 0; mode < 3; mode++)
        oracle_treecode(n, x, y, z, m, leaf, p, 0.5, mode, 0.0, nt, tidx, o[0], o[1],
                        o[2], o[3]);
    oracle_fmm_points(n, x, y, z, m, leaf, p, 0.0, 16, tx, ty, tz, o[0], o[1], o[2], o[3]);
    oracle_treecode_points(n, x, y, z, m, leaf, p, 0.5, 0, 0.0, 16, tx, ty, tz, o[0], o[1],
                           o[2], o[3]);
    oracle_treecode_points(n, x, y, z, m, leaf, p, 0.5, 2, 0.0, 16, tx, ty, tz, o[0], o[1],
                           o[2], o[3]);

    if (n > 0) {
        otree* t = oracle_tree_build(n, x, y, z, leaf);
        const int64_t nc = oracle_tree_ncells(t);
        double root[4];
        oracle_tree_root(t, root);
        uint64_t* keys = malloc(sizeof(uint64_t) * n);
        int64_t* perm = malloc(sizeof(int64_t) * n);
        oracle_tree_keys(t, keys);
        oracle_tree_perm(t, perm);
        int32_t* ci[7];
        int64_t* c64[2];
        for (int a = 0; a < 7; a++) ci[a] = malloc(sizeof(int32_t) * nc);
        for (int a = 0; a < 2; a++) c64[a] = malloc(sizeof(int64_t) * nc);
        oracle_tree_cells(t, ci[0], ci[1], ci[2], ci[3], c64[0], c64[1], ci[4], ci[5], ci[6]);
        double* cc[4];
        for (int a = 0; a < 4; a++) cc[a] = malloc(sizeof(double) * nc);
        oracle_tree_centres(t, cc[0], cc[1], cc[2], cc[3]);
        oracle_tree_com(t, m, cc[0], cc[1], cc[2]);
        int64_t* off = malloc(sizeof(int64_t) * (nc + 1));
        for (int w = 0; w < 4; w++) {
            const int64_t k = oracle_list_size(t, w);
            int32_t* items = malloc(sizeof(int32_t) * (k + 1));
            oracle_list_get(t, w, off, items);
            free(items);
            if (n <= 400) {
                const int64_t kb = oracle_list_size_bruteforce(t, w);
                int32_t* ib = malloc(sizeof(int32_t) * (kb + 1));
                oracle_list_get_bruteforce(t, w, off, ib);
                free(ib);
            }
        }
        for (int w = 0; w < 2; w++) {
            const int64_t k = oracle_bh_lists(t, m, 0.5, w, NULL, NULL);
            int32_t* items = malloc(sizeof(int32_t) * (k + 1));
            oracle_bh_lists(t, m, 0.5, w, off, items);
            free(items);
        }
        const int64_t pp = (int64_t)p * p;
        double* M = malloc(sizeof(double) * 2 * pp * nc);
        double* L = malloc(sizeof(double) * 2 * pp * nc);
        oracle_fmm_expansions(t, m, p, M, L);
        int64_t* boxes = malloc(sizeof(int64_t) * 7 * 16);
        oracle_target_boxes(t, 16, tx, ty, tz, boxes);
        for (int w = 0; w < 4; w++) {
            const double pt[3] = {tx[w], ty[w], tz[w]};
            const int64_t k = oracle_box_list(t, pt, w, NULL);
            int32_t* items = malloc(sizeof(int32_t) * (k + 1));
            oracle_box_list(t, pt, w, items);
            free(items);
        }
        oracle_fmm_points_tree(t, m, p, 0.0, 16, tx, ty, tz, o[0], o[1], o[2], o[3]);
        oracle_treecode_points_tree(t, m, p, 0.5, 0, 0.0, 16, tx, ty, tz, o[0], o[1], o[2],
                                    o[3]);
        /* a kept tree: moved positions, the rule, the drivers on it */
        for (int64_t i = 0; i < n; i++) x[i] += 1e-4 * (uniform01() - 0.5);
        (void)oracle_tree_stays(t, x, y, z, 0.0625);
        oracle_tree_move(t, x, y, z);
        oracle_fmm_tree(t, m, p, 0.0, nt, tidx, o[0], o[1], o[2], o[3]);
        oracle_treecode_tree(t, m, p, 0.5, 0, 0.0, 0, NULL, o[0], o[1], o[2], o[3]);
        double ph[3];
        oracle_fmm_phase_seconds(ph);
        free(boxes);
        free(M);
        free(L);
        free(off);
        for (int a = 0; a < 4; a++) free(cc[a]);
        for (int a = 0; a < 7; a++) free(ci[a]);
        for (int a = 0; a < 2; a++) free(c64[a]);
        free(keys);
        free(perm);
        oracle_tree_free(t);
    }
    for (int a = 0; a < 4; a++) free(o[a]);
    free(tidx);
    free(x);
    free(y);
    free(z);
    free(m);
}

int main(void) {
    /* single operators, special functions and the rotation */
    const int p = 6;
    double P[(2 * 6) * (2 * 6)], Y[2 * 36 * 2];
    oracle_legendre(2 * p - 1, 0.3, P);
    oracle_ynm(p - 1, 0.7, -1.2, Y);
    (void)oracle_anm(5, -3);
    double x[5], y[5], z[5], m[5];
    for (int i = 0; i < 5; i++) {
        x[i] = uniform01();
        y[i] = uniform01();
        z[i] = uniform01();
        m[i] = 1.0;
    }
    const double c0[3] = {0.5, 0.5, 0.5}, c1[3] = {2.5, 0.5, -1.5}, c2[3] = {0.25, 0.75, 0.25};
    double A[2 * 36], B[2 * 36], out[4];
    oracle_p2m(p, c0, 5, x, y, z, m, A);
    oracle_m2m(p, c2, c0, A, B);
    oracle_m2l(p, c0, c1, A, B);
    oracle_m2l_rot(p, c0, c1, A, B);
    oracle_l2l(p, c1, c2, B, A);
    oracle_p2l(p, c1, 5, x, y, z, m, B);
    const double pt[3] = {2.4, 0.6, -1.4};
    oracle_l2p(p, c1, B, pt, out);
    oracle_m2p(p, c0, A, pt, out);
    const double Q[9] = {0.0, -1.0, 0.0, 1.0, 0.0, 0.0, 0.0, 0.0, 1.0};
    oracle_rotate(p, Q, A, B);
    oracle_set_num_threads(oracle_num_threads());

    /* trees: empty, one particle, tiny, deep adaptive */
    run_set(0, 4, 4);
    run_set(1, 4, 4);
    run_set(9, 2, 3);
    run_set(300, 4, 5);
    run_set(2000, 8, 4);
    printf("sanitized oracle run complete\n");
    return 0;
}
