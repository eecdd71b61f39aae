// Driver for a sanitizer build (AddressSanitizer, UndefinedBehaviorSanitizer)
// of the host code of the HIP library, run on a machine without a GPU.  Every
// entry point of include/hfmm.h is called on the paths that end before any
// device work (sizing, argument and state checks, error strings) and, with
// valid arguments, on the path where the runtime reports no device: each
// must return a status code, never crash.  Numerical behaviour is the GPU
// tests' business.
#include <stdint.h>
#include <stdio.h>

#include <initializer_list>

#include "hfmm.h"

static int failures = 0;

static void expect(bool ok, const char* what) {
    if (!ok) {
        fprintf(stderr, "unexpected result: %s\n", what);
        ++failures;
    }
}

int main() {
    // sizing over methods, precisions, orders and sizes (host arithmetic)
    size_t bytes = 0;
    for (int method = 0; method <= 5; ++method)
        for (int prec = -1; prec <= 6; ++prec)
            for (int p = 0; p <= 17; ++p)
                for (int64_t n : {(int64_t)0, (int64_t)1, (int64_t)1000, (int64_t)1 << 22}) {
                    const int rc = hfmm_arena_bytes(n, n / 3, 64, p, method, prec, &bytes);
                    expect(rc <= 0, "arena_bytes returns a status");
                }
    expect(hfmm_arena_bytes(10, 0, 64, 4, HFMM_FMM, HFMM_FP32, nullptr) == HFMM_E_INVAL,
           "arena_bytes null output");
    expect(hfmm_arena_bytes(-1, 0, 64, 4, HFMM_FMM, HFMM_FP32, &bytes) == HFMM_E_INVAL,
           "arena_bytes negative n");
    expect(hfmm_direct_bytes(1000, 0, HFMM_FP64, &bytes) == HFMM_OK, "direct_bytes");
    expect(hfmm_direct_bytes(-5, 0, HFMM_FP64, &bytes) == HFMM_E_INVAL, "direct_bytes n < 0");
    for (int code = -12; code <= 2; ++code) expect(hfmm_strerror(code) != nullptr, "strerror");

    // null handles and outputs
    double d[4] = {0, 0, 0, 0};
    uint32_t flags = 7;
    int kept = 3;
    expect(hfmm_upward(nullptr, d, 4, HFMM_FMM, HFMM_FP32, nullptr) == HFMM_E_INVAL, "upward");
    expect(hfmm_evaluate(nullptr, nullptr, nullptr, nullptr, 0, 4, 0.5, HFMM_FMM, HFMM_FP32,
                         0.0, nullptr, nullptr, nullptr, nullptr, nullptr) == HFMM_E_INVAL,
           "evaluate");
    expect(hfmm_status(nullptr, nullptr, &flags) == HFMM_E_INVAL && flags == 0, "status");
    expect(hfmm_refit(nullptr, d, d, d, 0.1, nullptr, &kept) == HFMM_E_INVAL && kept == 0,
           "refit");
    expect(hfmm_get_stats(nullptr, nullptr) == HFMM_E_INVAL, "get_stats");
    expect(hfmm_required_bytes(nullptr) == 0, "required_bytes");
    expect(hfmm_export_perm(nullptr, nullptr, nullptr) == HFMM_E_INVAL, "export_perm");
    expect(hfmm_export_cells(nullptr, nullptr, nullptr) == HFMM_E_INVAL, "export_cells");
    expect(hfmm_export_targets(nullptr, nullptr, nullptr) == HFMM_E_INVAL, "export_targets");
    expect(hfmm_export_list(nullptr, 0, nullptr, nullptr, nullptr) == HFMM_E_INVAL,
           "export_list");
    expect(hfmm_export_bh_list(nullptr, 0, nullptr, nullptr, nullptr) == HFMM_E_INVAL,
           "export_bh_list");
    expect(hfmm_export_target_lists(nullptr, 0, nullptr, nullptr, nullptr) == HFMM_E_INVAL,
           "export_target_lists");
    expect(hfmm_export_expansions(nullptr, 0, nullptr, nullptr) == HFMM_E_INVAL,
           "export_expansions");
    hfmm_tree_release(nullptr);

    // argument errors before any device work
    hfmm_tree t = reinterpret_cast<hfmm_tree>(1);
    char arena[256];
    expect(hfmm_build_tree(d, d, d, -1, 64, arena, sizeof(arena), nullptr, &t) ==
                   HFMM_E_INVAL &&
               t == nullptr,
           "build_tree n < 0");
    expect(hfmm_build_tree(d, d, d, 4, 0, arena, sizeof(arena), nullptr, &t) == HFMM_E_INVAL,
           "build_tree leaf_max 0");
    expect(hfmm_build_tree(nullptr, d, d, 4, 64, arena, sizeof(arena), nullptr, &t) ==
               HFMM_E_INVAL,
           "build_tree null x");
    expect(hfmm_build_tree(d, d, d, 4, 64, nullptr, 0, nullptr, &t) == HFMM_E_INVAL,
           "build_tree null arena");
    expect(hfmm_build_tree(d, d, d, 4, 64, arena, sizeof(arena), nullptr, nullptr) ==
               HFMM_E_INVAL,
           "build_tree null out");
    expect(hfmm_solve(d, d, d, d, 4, nullptr, nullptr, nullptr, 0, 64, 4, 0.5, 9, HFMM_FP32,
                      0.0, arena, sizeof(arena), d, d, d, d, nullptr) != HFMM_OK,
           "solve unknown method");
    expect(hfmm_direct(d, d, d, d, -1, nullptr, nullptr, nullptr, 0, HFMM_FP32, 0.0, arena,
                       sizeof(arena), d, d, d, d, nullptr) == HFMM_E_INVAL,
           "direct n < 0");
    expect(hfmm_direct_noalloc(d, d, d, d, (int64_t)1 << 40, nullptr, nullptr, nullptr, 0,
                               HFMM_FP32, 0.0, d, d, d, d, nullptr) != HFMM_OK,
           "direct_noalloc beyond its array");
    int done = 9, builds = 9;
    expect(hfmm_leapfrog(d, d, d, d, d, d, d, -1, 1e-3, 1, 64, 4, 0.5, HFMM_FMM, HFMM_FP32, 0.0,
                         -1.0, arena, sizeof(arena), d, d, d, d, &done, &builds, nullptr) ==
                   HFMM_E_INVAL &&
               done == 0 && builds == 0,
           "leapfrog n < 0");
    expect(hfmm_leapfrog(d, d, d, d, d, d, d, 0, 1e-3, 3, 64, 4, 0.5, HFMM_FMM, HFMM_FP32, 0.0,
                         -1.0, arena, sizeof(arena), d, d, d, d, &done, &builds, nullptr) ==
                   HFMM_OK &&
               done == 3,
           "leapfrog n = 0");
    hfmm_set_timing(1);
    hfmm_set_timing(0);
    (void)hfmm_last_required_bytes();

    // valid arguments on a machine without a device: a status, no crash
    const int rc = hfmm_build_tree(d, d, d, 4, 64, arena, sizeof(arena), nullptr, &t);
    if (rc == HFMM_OK) hfmm_tree_release(t);
    expect(rc <= 0, "build_tree without a device returns a status");
    const int rd = hfmm_direct(d, d, d, d, 4, nullptr, nullptr, nullptr, 0, HFMM_FP32, 0.0,
                               arena, sizeof(arena), d, d, d, d, nullptr);
    expect(rd <= 0, "direct without a device returns a status");

    if (failures) return 1;
    printf("sanitized host run complete\n");
    return 0;
}
