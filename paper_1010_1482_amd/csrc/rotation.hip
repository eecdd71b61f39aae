// Rotation-based M2L: the O(p^3) translation Sec. 6 names among the
// advanced techniques (Cheng, Greengard and Rokhlin).  For the offset class
// of a V pair (v = target centre - source centre, in cell units, the reading
// of Eq. 4's (rho, alpha, beta)) the multipole expansion is rotated into the
// frame whose z axis points along v, translated along that axis, where Eq. 4
// couples each order k only to itself (in the device basis)
//     Lt'_j^k = sum_{n >= k} (-1)^{j+k} (j+n)! / |v|^{j+n+1} Mt'_n^k,
// and the local expansion is rotated back.  Per pair that is 2 sum_n
// (2n+1)^2 + ~p^3 / 3 multiply-adds instead of the dense operator's p^4.
//
// The rotation matrices (per class and degree, real layout, independent of
// the level like the dense operators) are computed once per order from
// their definition: the rotated degree-n field projected on the harmonics
// with a quadrature exact to degree 2n (Gauss-Legendre in cos a times the
// trapezoid rule in b), through the biorthogonality of the regular and
// irregular harmonics on the unit sphere,
//     integral of S_n^m conj(R_n^m') = 4 pi / (2n+1) delta_{m m'}.
// Frame: R = R_y(-alpha) R_z(-beta) takes v to the z axis; a multipole field
// f becomes u -> f(R^T u), a local field g in the rotated frame is g(R u)
// in the original one.
#include "common.hpp"
#include "expansions.hpp"

namespace hfmm {

constexpr int kRotNodes = 32;  // quadrature nodes staged per round (32 KiB of LDS)

// sum over degrees below n of (2k+1)^2: offset of degree n's block
__host__ __device__ constexpr int rot_off(int n) { return n * (2 * n - 1) * (2 * n + 1) / 3; }

// P_n^m(x), m = 0..n (Condon-Shortley sign, Eqs. 7-9), at sin = s
__device__ inline void legendre_row(int n, double x, double s, double* P) {
    double pmm = 1.0;
    for (int m = 0; m <= n; ++m) {
        if (m > 0) pmm *= -(double)(2 * m - 1) * s;
        if (m == n) {
            P[m] = pmm;
            continue;
        }
        double p0 = pmm, p1 = x * (2 * m + 1) * pmm;
        for (int l = m + 2; l <= n; ++l) {
            const double pl = (x * (2 * l - 1) * p1 - (l + m - 1) * p0) / (l - m);
            p0 = p1;
            p1 = pl;
        }
        P[m] = p1;
    }
}

// regular (R) and irregular (S) harmonics of degree n at the unit vector v:
// R_n^m = P_n^m e^{i m b} / (n+m)!,  S_n^m = (n-m)! P_n^m e^{i m b}
__device__ inline void harmonics_at(int n, const double v[3], double2* Rv, double2* Sv) {
    const double rxy = sqrt(v[0] * v[0] + v[1] * v[1]);
    const double b = rxy == 0.0 ? 0.0 : atan2(v[1], v[0]);
    double P[HFMM_MAX_P];
    legendre_row(n, v[2], rxy, P);
    for (int m = 0; m <= n; ++m) {
        double fa = 1.0, fb = 1.0;  // (n+m)!, (n-m)!
        for (int i = 2; i <= n + m; ++i) fa *= i;
        for (int i = 2; i <= n - m; ++i) fb *= i;
        const double c = cos(m * b), s = sin(m * b);
        if (Rv) Rv[m] = make_double2(P[m] * c / fa, P[m] * s / fa);
        if (Sv) Sv[m] = make_double2(fb * P[m] * c, fb * P[m] * s);
    }
}

// real-layout index i (degree n) of a unit coefficient -> the real field it
// gives from the complex basis value b at a point
__device__ __forceinline__ double field_of(int i, const double2* b) {
    if (i == 0) return b[0].x;
    const int m = (i + 1) / 2;
    return (i & 1) ? 2.0 * b[m].x : -2.0 * b[m].y;
}
// real-layout output o: Re or Im of the projection on conj(basis)
__device__ __forceinline__ double proj_of(int o, const double2* b) {
    if (o == 0) return b[0].x;
    const int m = (o + 1) / 2;
    return (o & 1) ? b[m].x : -b[m].y;
}

// One block per (class, degree n): the forward (multipole, S basis) and
// backward (local, R basis) rotation blocks of degree n, stored input-major
// [i][o] per block: Tab[cls][0: forward, 1: backward][rot_off(n) + i w + o].
template <typename TO>
__global__ void __launch_bounds__(256) k_rot_ops(int p, TO* __restrict__ tab) {
    const int cls = blockIdx.x, n = blockIdx.y;
    const int w = 2 * n + 1, ww = w * w;
    const int SZ = rot_off(p);
    TO* F = tab + (int64_t)cls * 2 * SZ + rot_off(n);
    TO* B = F + SZ;
    const int dx = cls / 49 - 3, dy = (cls / 7) % 7 - 3, dz = cls % 7 - 3;
    if (max(abs(dx), max(abs(dy), abs(dz))) < 2) {  // adjacent: never used
        for (int e = threadIdx.x; e < ww; e += blockDim.x) F[e] = B[e] = TO(0);
        return;
    }
    // v = target - source = -d; R = R_y(-alpha) R_z(-beta)
    const double vx = -dx, vy = -dy, vz = -dz;
    const double rho = sqrt(vx * vx + vy * vy + vz * vz), rxy = sqrt(vx * vx + vy * vy);
    const double ca = vz / rho, sa = rxy / rho;
    const double cb = rxy == 0.0 ? 1.0 : vx / rxy, sb = rxy == 0.0 ? 0.0 : vy / rxy;
    const double R[9] = {ca * cb, ca * sb, -sa, -sb, cb, 0.0, sa * cb, sa * sb, ca};
    // Gauss-Legendre nodes in cos a, n + 1 of them (Newton on P_{n+1})
    __shared__ double gx[HFMM_MAX_P], gw[HFMM_MAX_P];
    const int N = n + 1;
    if ((int)threadIdx.x < N) {
        const int t = threadIdx.x;
        double z = cos(3.14159265358979323846 * (t + 0.75) / (N + 0.5)), d = 1.0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = z;
            for (int k = 2; k <= N; ++k) {
                const double pk = ((2 * k - 1) * z * p1 - (k - 1) * p0) / k;
                p0 = p1;
                p1 = pk;
            }
            d = N * (z * p1 - p0) / (z * z - 1.0);
            const double dz2 = p1 / d;
            z -= dz2;
            if (fabs(dz2) < 1e-16) break;
        }
        double p0 = 1.0, p1 = z;
        for (int k = 2; k <= N; ++k) {
            const double pk = ((2 * k - 1) * z * p1 - (k - 1) * p0) / k;
            p0 = p1;
            p1 = pk;
        }
        d = N * (z * p1 - p0) / (z * z - 1.0);
        gx[t] = z;
        gw[t] = 2.0 / ((1.0 - z * z) * d * d);
    }
    // per node: S_n(R^T u), R_n(u) (forward); R_n(R u), S_n(u) (backward)
    __shared__ double2 sv1[kRotNodes][HFMM_MAX_P], ru[kRotNodes][HFMM_MAX_P];
    __shared__ double2 rv2[kRotNodes][HFMM_MAX_P], su[kRotNodes][HFMM_MAX_P];
    __shared__ double wq[kRotNodes];
    constexpr int kPer = (2 * (2 * HFMM_MAX_P - 1) * (2 * HFMM_MAX_P - 1) + 255) / 256;
    double acc[kPer];
#pragma unroll
    for (int r = 0; r < kPer; ++r) acc[r] = 0.0;
    __syncthreads();
    const int nq = N * w;
    for (int q0 = 0; q0 < nq; q0 += kRotNodes) {
        const int t = threadIdx.x;
        if (t < kRotNodes && q0 + t < nq) {
            const int q = q0 + t, a = q / w, bq = q % w;
            const double cta = gx[a], sta = sqrt(fmax(0.0, 1.0 - cta * cta));
            const double ph = 2.0 * 3.14159265358979323846 * bq / w;
            const double u[3] = {sta * cos(ph), sta * sin(ph), cta};
            double v1[3], v2[3];
            for (int k = 0; k < 3; ++k) {
                v1[k] = R[k] * u[0] + R[3 + k] * u[1] + R[6 + k] * u[2];      // R^T u
                v2[k] = R[3 * k] * u[0] + R[3 * k + 1] * u[1] + R[3 * k + 2] * u[2];  // R u
            }
            harmonics_at(n, u, ru[t], su[t]);
            harmonics_at(n, v1, nullptr, sv1[t]);
            harmonics_at(n, v2, rv2[t], nullptr);
            wq[t] = gw[a] * 2.0 * 3.14159265358979323846 / w;
        }
        __syncthreads();
        const int nb = min(kRotNodes, nq - q0);
#pragma unroll
        for (int r = 0; r < kPer; ++r) {
            const int e = threadIdx.x + 256 * r;
            if (e >= 2 * ww) continue;
            const int tb = e / ww, i = (e % ww) / w, o = e % w;
            double sacc = 0.0;
            for (int q = 0; q < nb; ++q) {
                const double g = field_of(i, tb == 0 ? sv1[q] : rv2[q]);
                const double c = proj_of(o, tb == 0 ? ru[q] : su[q]);
                sacc += wq[q] * g * c;
            }
            acc[r] += sacc;
        }
        __syncthreads();
    }
    const double sc = (2.0 * n + 1.0) / (4.0 * 3.14159265358979323846);
#pragma unroll
    for (int r = 0; r < kPer; ++r) {
        const int e = threadIdx.x + 256 * r;
        if (e >= 2 * ww) continue;
        const int tb = e / ww;
        (tb == 0 ? F : B)[e % ww] = (TO)(sc * acc[r]);
    }
}

size_t rot_ops_bytes(int p, int precision) {
    return (size_t)343 * 2 * rot_off(p) * (precision == HFMM_FP64 ? 8 : 4);
}

void run_rot_ops(int p, int precision, void* tab, hipStream_t s) {
    if (precision == HFMM_FP64)
        hipLaunchKernelGGL(k_rot_ops<double>, dim3(343, p), dim3(256), 0, s, p, (double*)tab);
    else
        hipLaunchKernelGGL(k_rot_ops<float>, dim3(343, p), dim3(256), 0, s, p, (float*)tab);
    LAUNCH_CHECK();
}

// degree of real-layout row r (r < p^2)
__device__ __forceinline__ int rot_degree(int r) {
    int n = 0;
    while ((n + 1) * (n + 1) <= r) ++n;
    return n;
}

// A block of kRotWaves waves takes kRotWaves targets of one octant (from the
// M2L tiles: targets of one octant see the same offset class in the same V
// slot), one target per wave, lanes over its p^2 real coefficients (up to
// four each).  Per slot the class's forward and backward blocks are staged
// in LDS once for all the block's targets; then each wave rotates its
// source's multipoles, translates them along z order by order and rotates
// the result back into its accumulators.  out: [cell][ld] partial result.
constexpr int kRotWaves = 8;

template <typename T, int NP>
__global__ void __launch_bounds__(64 * kRotWaves)
k_m2l_rot(const int32_t* __restrict__ tiles, const int32_t* __restrict__ torder,
          const int32_t* __restrict__ vsrc, const double* __restrict__ M, int ld,
          const T* __restrict__ tab, T* __restrict__ out) {
    // rows up to ld = 16 ceil(p^2 / 16) <= 64 U are written (padding zero)
    constexpr int P = NP * NP, U = (P + 63) / 64, SZ = rot_off(NP);
    __shared__ T ts[2 * SZ];
    __shared__ T wsm[kRotWaves][3][P];
    __shared__ T ft[2 * NP];
    const int start = tiles[4 * blockIdx.x], count = tiles[4 * blockIdx.x + 1];
    const int oct = tiles[4 * blockIdx.x + 2];
    if ((int)blockIdx.y * kRotWaves >= count) return;  // uniform per block
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int ti = blockIdx.y * kRotWaves + wv;
    const int c = ti < count ? torder[start + ti] : -1;
    const int ox = (oct >> 2) & 1, oy = (oct >> 1) & 1, oz = oct & 1;
    T* ms = wsm[wv][0];
    T* mr = wsm[wv][1];
    T* lr = wsm[wv][2];
    // per output row: degree, index in the degree, order and part
    int deg[U], loc[U], ord[U], prt[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const int r = lane + 64 * u;
        const int n = rot_degree(r < P ? r : 0);
        deg[u] = n;
        loc[u] = r - n * n;
        ord[u] = (loc[u] + 1) / 2;
        prt[u] = loc[u] == 0 ? 0 : (loc[u] + 1) % 2;
    }
    T acc[U];
#pragma unroll
    for (int u = 0; u < U; ++u) acc[u] = T(0);
    for (int slot = 0; slot < 216; ++slot) {
        const int src = c >= 0 ? vsrc[(int64_t)c * 216 + slot] : -1;
        // the block's barrier before the tables are overwritten, and whether
        // any of its targets has a source in this slot
        if (!__syncthreads_or(src >= 0)) continue;
        const int dx = slot / 36 - 2 - ox, dy = (slot / 6) % 6 - 2 - oy, dz = slot % 6 - 2 - oz;
        const int cls = (dx + 3) * 49 + (dy + 3) * 7 + (dz + 3);
        const T* g = tab + (int64_t)cls * 2 * SZ;
        for (int e = threadIdx.x; e < 2 * SZ; e += 64 * kRotWaves) ts[e] = g[e];
        if ((int)threadIdx.x < 2 * NP - 1) {  // N! / |v|^{N+1}
            const double rho = sqrt((double)(dx * dx + dy * dy + dz * dz));
            double f = 1.0 / rho;
            for (int k = 1; k <= (int)threadIdx.x; ++k) f *= k / rho;
            ft[threadIdx.x] = (T)f;
        }
        if (src >= 0) {
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int r = lane + 64 * u;
                if (r < P) ms[r] = (T)M[(int64_t)src * ld + r];
            }
        }
        __syncthreads();
        if (src < 0) continue;  // uniform per wave
        // rotate into the frame of v
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int r = lane + 64 * u;
            if (r >= P) continue;
            const int n = deg[u], w = 2 * n + 1;
            const T* f = ts + rot_off(n) + loc[u];
            T sacc = T(0);
            for (int i = 0; i < w; ++i) sacc += f[i * w] * ms[n * n + i];
            mr[r] = sacc;
        }
        wave_lds_fence();
        // translate along z: order k to order k
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int r = lane + 64 * u;
            if (r >= P) continue;
            const int j = deg[u], k = ord[u];
            const int col = k == 0 ? 0 : 2 * k - 1 + prt[u];
            T sacc = T(0);
            for (int n = k; n < NP; ++n) sacc += ft[j + n] * mr[n * n + col];
            lr[r] = ((j + k) & 1) ? -sacc : sacc;
        }
        wave_lds_fence();
        // rotate back and accumulate
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int r = lane + 64 * u;
            if (r >= P) continue;
            const int j = deg[u], w = 2 * j + 1;
            const T* bb = ts + SZ + rot_off(j) + loc[u];
            T sacc = T(0);
            for (int i = 0; i < w; ++i) sacc += bb[i * w] * lr[j * j + i];
            acc[u] += sacc;
        }
    }
    if (c < 0) return;
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const int r = lane + 64 * u;
        if (r < ld) out[(int64_t)c * ld + r] = r < P ? acc[u] : T(0);
    }
}

int run_m2l_rot(Tree& t, int p, int precision, void* out, int64_t& part_stride, hipStream_t s) {
    part_stride = (int64_t)t.ncells * t.ldm;
    if (t.depth < 2 || t.n_m2l_tiles == 0) return 0;
    PhaseTimer pt(t, PH_M2L, s);
    const dim3 grid(t.n_m2l_tiles, (256 + kRotWaves - 1) / kRotWaves), block(64 * kRotWaves);
#define ROT_CASE(NP)                                                                          \
    if (precision == HFMM_FP64)                                                               \
        hipLaunchKernelGGL((k_m2l_rot<double, NP>), grid, block, 0, s, t.m2l_tiles,            \
                           t.m2l_torder, t.vsrc, t.M, t.ldm, (const double*)t.T, (double*)out); \
    else                                                                                      \
        hipLaunchKernelGGL((k_m2l_rot<float, NP>), grid, block, 0, s, t.m2l_tiles,             \
                           t.m2l_torder, t.vsrc, t.M, t.ldm, (const float*)t.T, (float*)out);
    switch (p) {
        case 1: ROT_CASE(1) break;
        case 2: ROT_CASE(2) break;
        case 3: ROT_CASE(3) break;
        case 4: ROT_CASE(4) break;
        case 5: ROT_CASE(5) break;
        case 6: ROT_CASE(6) break;
        case 7: ROT_CASE(7) break;
        case 8: ROT_CASE(8) break;
        case 9: ROT_CASE(9) break;
        case 10: ROT_CASE(10) break;
        case 11: ROT_CASE(11) break;
        case 12: ROT_CASE(12) break;
        case 13: ROT_CASE(13) break;
        case 14: ROT_CASE(14) break;
        case 15: ROT_CASE(15) break;
        case 16: ROT_CASE(16) break;
        default: throw Status{HFMM_E_UNSUPPORTED};
    }
#undef ROT_CASE
    LAUNCH_CHECK();
    return 1;
}

}  // namespace hfmm
