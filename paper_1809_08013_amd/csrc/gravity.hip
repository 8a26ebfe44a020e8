// Algorithm 1, step 4 on the GPU (self-gravity; Sec. 5.2.5 phase I), by
// direct summation in FP64 with Plummer softening (G = 1):
//   g_i = - sum_{j != i} m_j (x_i - x_j) / (|x_i - x_j|^2 + eps^2)^{3/2}.
//
// One lane per particle i. The wave walks every j in array order,
// wave-uniformly: each record {x, y, z, m} is one scalar load into SGPRs
// (all waves walk the same sequence at about the same time, so the records
// are served by the scalar cache), four records in flight. j = i adds an
// exact zero when eps > 0 (dx = dy = dz = 0) and is dropped by the d2 > 0
// test when eps = 0. O(n^2) work: the reference the parent codes' tree
// multipoles approximate, not a fast solver.
#include "sph_internal.h"

namespace sph {
namespace {

constexpr int kThreads = 256;

// 1/sqrt(x), x > 0: the hardware estimate and two Newton steps (about one
// ulp in FP64).
__device__ __forceinline__ double rsq_newton(double x)
{
    double y = __builtin_amdgcn_rsq(x);
    const double h = 0.5 * x;
    y = y * __builtin_fma(-h * y, y, 1.5);
    return y * __builtin_fma(-h * y, y, 1.5);
}

__global__ void __launch_bounds__(256)
pack_grav_kernel(int64_t n, const double *__restrict__ x, const double *__restrict__ y,
                 const double *__restrict__ z, const double *__restrict__ m,
                 DensRec *__restrict__ out)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = DensRec{x[i], y[i], z[i], m[i]};
}

__global__ void __launch_bounds__(kThreads)
gravity_direct_kernel(int64_t n, const DensRec *__restrict__ rec, double e2,
                      double *__restrict__ gx, double *__restrict__ gy,
                      double *__restrict__ gz)
{
    const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    const bool active = i < n;
    const DensRec me = rec[active ? i : 0];
    double sx = 0.0, sy = 0.0, sz = 0.0;
    auto term = [&](const DensRec &o) {
        const double dx = me.x - o.x, dy = me.y - o.y, dz = me.z - o.z;
        const double d2 = __builtin_fma(dz, dz, __builtin_fma(dy, dy, __builtin_fma(dx, dx, e2)));
        const double rs = d2 > 0.0 ? rsq_newton(d2) : 0.0;
        const double t = o.m * (rs * rs * rs);
        sx = __builtin_fma(-t, dx, sx);
        sy = __builtin_fma(-t, dy, sy);
        sz = __builtin_fma(-t, dz, sz);
    };
    int64_t j = 0;
    if (n >= 4) {
        DensRec a0 = rec[0], a1 = rec[1], a2 = rec[2], a3 = rec[3];
        j = 4;
        while (n - j >= 4) {
            const DensRec b0 = rec[j], b1 = rec[j + 1], b2 = rec[j + 2], b3 = rec[j + 3];
            term(a0);
            term(a1);
            term(a2);
            term(a3);
            // the wait for b0..b3 goes after the work on a0..a3
            __builtin_amdgcn_sched_barrier(0);
            a0 = b0;
            a1 = b1;
            a2 = b2;
            a3 = b3;
            j += 4;
        }
        term(a0);
        term(a1);
        term(a2);
        term(a3);
    }
    for (; j < n; ++j) term(rec[j]);
    if (active) {
        gx[i] = sx;
        gy[i] = sy;
        gz[i] = sz;
    }
}

inline unsigned blocks_for(int64_t n, int t) { return (unsigned)((n + t - 1) / t); }

}  // namespace

hipError_t launch_gravity_direct(sph_ctx ctx, const sph_particles &p, double eps, double *gx,
                                 double *gy, double *gz)
{
    pack_grav_kernel<<<blocks_for(p.n, 256), 256, 0, ctx->stream>>>(p.n, p.x, p.y, p.z, p.m,
                                                                    ctx->drec);
    gravity_direct_kernel<<<blocks_for(p.n, kThreads), kThreads, 0, ctx->stream>>>(
        p.n, ctx->drec, eps * eps, gx, gy, gz);
    return hipGetLastError();
}

}  // namespace sph
