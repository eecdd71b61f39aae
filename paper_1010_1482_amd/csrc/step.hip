// Time stepping of the N-body simulation the paper's title names (the text
// gives no integrator): kick-drift-kick leapfrog around the force evaluation,
//   v += a dt/2;  x += v dt;  a = field(x);  v += a dt/2,
// a being the field of all the other particles (Eq. 1 per unit mass, the
// sign of Sec. 5.1).  The tree of the moved particles is either built anew
// in the caller's arena or, while every particle stays near the leaf it was
// built into, kept with the new positions (hfmm_refit); the state of the
// last completed step is kept at the top of the arena, so that an
// evaluation that runs out of arena space leaves the caller a whole step to
// continue from.
#include "common.hpp"

namespace hfmm {

// v += hk * a, then (dt != 0) x += dt * v; one thread per particle
template <typename A>
__global__ void k_kick_drift(int64_t n, double* __restrict__ x, double* __restrict__ y,
                             double* __restrict__ z, double* __restrict__ vx,
                             double* __restrict__ vy, double* __restrict__ vz,
                             const A* __restrict__ ax, const A* __restrict__ ay,
                             const A* __restrict__ az, double hk, double dt) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double ux = vx[i] + hk * (double)ax[i];
    const double uy = vy[i] + hk * (double)ay[i];
    const double uz = vz[i] + hk * (double)az[i];
    vx[i] = ux;
    vy[i] = uy;
    vz[i] = uz;
    if (dt != 0.0) {
        x[i] += dt * ux;
        y[i] += dt * uy;
        z[i] += dt * uz;
    }
}

}  // namespace hfmm

using namespace hfmm;

extern "C" int hfmm_leapfrog(double* x, double* y, double* z, double* vx, double* vy,
                             double* vz, const double* m, int64_t n, double dt, int steps,
                             int leaf_max, int p, double theta, int method, int precision,
                             double eps2, double slack, void* arena, size_t arena_bytes,
                             void* phi, void* ax, void* ay, void* az, int* done, int* builds,
                             void* stream) {
    if (done) *done = 0;
    if (builds) *builds = 0;
    if (n < 0 || steps < 0 || !(dt == dt) || !(slack == slack) || !arena) return HFMM_E_INVAL;
    if (n > 0 && (!x || !y || !z || !vx || !vy || !vz || !m || !phi || !ax || !ay || !az))
        return HFMM_E_INVAL;
    if (n == 0) {
        if (done) *done = steps;
        return HFMM_OK;
    }
    // the saved state (x, y, z, vx, vy, vz) above the evaluation's arena
    const size_t state = Arena::align((size_t)n * 6 * sizeof(double));
    if (arena_bytes < state + ((size_t)1 << 20)) {
        set_last_required(state + ((size_t)64 << 20));
        return HFMM_E_NOMEM;
    }
    const size_t eval_bytes = (arena_bytes - state) / HFMM_ALIGN * HFMM_ALIGN;
    double* keep = (double*)((char*)arena + eval_bytes);
    double* cur[6] = {x, y, z, vx, vy, vz};
    hipStream_t s = (hipStream_t)stream;
    const bool f64 = precision == HFMM_FP64;
    const dim3 grid(grid_for(n, 256)), block(256);
    auto kick = [&](double hk, double d) {
        if (f64)
            hipLaunchKernelGGL(k_kick_drift<double>, grid, block, 0, s, n, x, y, z, vx, vy, vz,
                               (const double*)ax, (const double*)ay, (const double*)az, hk, d);
        else
            hipLaunchKernelGGL(k_kick_drift<float>, grid, block, 0, s, n, x, y, z, vx, vy, vz,
                               (const float*)ax, (const float*)ay, (const float*)az, hk, d);
        return hipGetLastError() == hipSuccess;
    };
    // the tree of the current positions (none for the direct sum)
    hfmm_tree h = nullptr;
    size_t need = 0;  // arena bytes a failed evaluation asked for
    auto release = [&]() {
        if (h) hfmm_tree_release(h);
        h = nullptr;
    };
    auto on_tree = [&]() {
        int rc = hfmm_upward(h, m, p, method, precision, stream);
        if (rc == HFMM_OK)
            rc = hfmm_evaluate(h, nullptr, nullptr, nullptr, 0, p, theta, method, precision,
                               eps2, phi, ax, ay, az, stream);
        if (rc == HFMM_OK) rc = hfmm_status(h, stream, nullptr);
        if (rc == HFMM_E_NOMEM) need = hfmm_required_bytes(h);
        return rc;
    };
    auto field = [&]() {
        need = 0;
        if (method == HFMM_DIRECT) {
            const int rc = hfmm_direct(x, y, z, m, n, nullptr, nullptr, nullptr, 0, precision,
                                       eps2, arena, eval_bytes, phi, ax, ay, az, stream);
            if (rc == HFMM_E_NOMEM) need = hfmm_last_required_bytes();
            return rc;
        }
        if (h && slack >= 0.0) {
            int kept = 0;
            const int rc = hfmm_refit(h, x, y, z, slack, stream, &kept);
            if (rc != HFMM_OK) return rc;
            if (kept) return on_tree();
        }
        release();
        const int rc = hfmm_build_tree(x, y, z, n, leaf_max, arena, eval_bytes, stream, &h);
        if (rc != HFMM_OK) {
            h = nullptr;
            if (rc == HFMM_E_NOMEM) need = hfmm_last_required_bytes();
            return rc;
        }
        if (builds) ++*builds;
        return on_tree();
    };
    auto fail = [&](int rc) {
        release();
        // the arena this call needs: the evaluation's and the saved state
        if (rc == HFMM_E_NOMEM) set_last_required(need + state + (1 << 20));
        return rc;
    };
    int rc = field();
    if (rc != HFMM_OK) return fail(rc);
    for (int k = 0; k < steps; ++k) {
        for (int a = 0; a < 6; ++a)
            if (hipMemcpyAsync(keep + (size_t)a * n, cur[a], sizeof(double) * n,
                               hipMemcpyDeviceToDevice, s) != hipSuccess)
                return fail(HFMM_E_HIP);
        if (!kick(0.5 * dt, dt)) return fail(HFMM_E_HIP);
        rc = field();
        if (rc != HFMM_OK) {
            // back to the state of the last completed step
            for (int a = 0; a < 6; ++a)
                if (hipMemcpyAsync(cur[a], keep + (size_t)a * n, sizeof(double) * n,
                                   hipMemcpyDeviceToDevice, s) != hipSuccess)
                    return fail(HFMM_E_HIP);
            return fail(rc);
        }
        if (!kick(0.5 * dt, 0.0)) return fail(HFMM_E_HIP);
        if (done) *done = k + 1;
    }
    release();
    return HFMM_OK;
}
