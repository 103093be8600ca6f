// rt_profile.hpp -- device side of the intensity profiles: the photons that
// passed through each particle during the last RT step, per unit time, summed
// or averaged over thin spherical shells around a point (section 3, radial
// profiles of the Stromgren tests) or thin cylindrical shells around an axis
// (section 4, shadow-test profiles).  One pass over the particles of one
// instance: positions and passing photons are read once, coalesced; each
// workgroup bins its particles into an LDS histogram and adds that to the
// global one with one atomic per nonzero entry.
//
// Shell membership is an integer decided by FP64 arithmetic, so it is written
// as plain IEEE operations in a fixed order (the library is built without FMA
// contraction; sqrt and division are correctly rounded): the same order gives
// the same shell on any IEEE FP64 implementation.
#pragma once

#include <hip/hip_runtime.h>

namespace trt {

constexpr int kProfMaxShells = 2048;   // shells per profile
constexpr int kProfMaxCells = 6144;    // shells x bins (LDS: 48 KB of sums + 8 KB of counts)
constexpr int kProfBlock = 256;

struct ProfileArgs {
    const double* pos;            // [N][3] particle positions, cm
    const double* P;              // [N][nf] photons that passed each particle in the last step
    long long j0, j1;             // particles of the instance: j0 .. j1-1
    int nf, n_shells, cyl;        // bins, shells, 1 for cylindrical shells
    double c0, c1, c2;            // centre (a point on the axis for cylinders), cm
    double a0, a1, a2;            // axis direction, any nonzero length (cylinders)
    double half_height;           // > 0: keep |(x - centre) . axis| <= half_height (cylinders)
    double r_max, dt;             // outer radius of the last shell, cm; RT step, s
    double* sum;                  // [n_shells][nf] photons per second, zero on entry
    unsigned long long* cnt;      // [n_shells] particles, zero on entry
};

__global__ __launch_bounds__(kProfBlock) void k_shell_profile(ProfileArgs a) {
    extern __shared__ double s_sum[];  // [n_shells * nf], then the counts as u32
    const int ncell = a.n_shells * a.nf;
    unsigned* s_cnt = reinterpret_cast<unsigned*>(s_sum + ncell);
    for (int k = threadIdx.x; k < ncell; k += blockDim.x) s_sum[k] = 0.0;
    for (int k = threadIdx.x; k < a.n_shells; k += blockDim.x) s_cnt[k] = 0u;
    __syncthreads();

    double u0 = 0.0, u1 = 0.0, u2 = 0.0;
    if (a.cyl) {
        const double an = sqrt(a.a0 * a.a0 + a.a1 * a.a1 + a.a2 * a.a2);
        u0 = a.a0 / an;
        u1 = a.a1 / an;
        u2 = a.a2 / an;
    }
    const double ns = static_cast<double>(a.n_shells);
    const double dr = a.r_max / ns;
    const long long stride = static_cast<long long>(gridDim.x) * blockDim.x;
    for (long long j = a.j0 + static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x; j < a.j1; j += stride) {
        const double d0 = a.pos[3 * j] - a.c0;
        const double d1 = a.pos[3 * j + 1] - a.c1;
        const double d2 = a.pos[3 * j + 2] - a.c2;
        double r2;
        bool keep = true;
        if (a.cyl) {
            const double t = d0 * u0 + d1 * u1 + d2 * u2;
            keep = !(a.half_height > 0.0 && fabs(t) > a.half_height);
            const double q0 = d0 - t * u0, q1 = d1 - t * u1, q2 = d2 - t * u2;
            r2 = q0 * q0 + q1 * q1 + q2 * q2;
        } else {
            r2 = d0 * d0 + d1 * d1 + d2 * d2;
        }
        const double s = floor(sqrt(r2) / dr);
        if (keep && s < ns) {
            const int k = static_cast<int>(s);
            atomicAdd(&s_cnt[k], 1u);
            for (int nu = 0; nu < a.nf; ++nu) atomicAdd(&s_sum[k * a.nf + nu], a.P[j * a.nf + nu] / a.dt);
        }
    }
    __syncthreads();
    for (int k = threadIdx.x; k < ncell; k += blockDim.x)
        if (s_sum[k] != 0.0) atomicAdd(&a.sum[k], s_sum[k]);
    for (int k = threadIdx.x; k < a.n_shells; k += blockDim.x)
        if (s_cnt[k]) atomicAdd(&a.cnt[k], static_cast<unsigned long long>(s_cnt[k]));
}

}  // namespace trt
