// Algorithm 1, steps 2 and 3 on the GPU: neighbour search over the cell
// grid, summation density, EOS, momentum and energy with artificial
// viscosity. Gather form throughout: each particle owns its outputs and sums
// its own pairs, so there are no atomics on floating-point values and every
// result is the same from run to run.
//
// The pair arithmetic comes in two forms (template parameter Real):
//   double: everything FP64;
//   float:  separations and velocity differences formed in FP64 and rounded
//           to FP32, FP32 copies of h, m, rho, P/rho^2 and c, FP32 sums,
//           outputs widened to FP64.
#include "sph_internal.h"

namespace sph {
namespace {

constexpr double kInvPi = 0.318309886183790671537767526745;

__device__ __forceinline__ uint32_t compact3(uint32_t v)
{
    v &= 0x09249249u;
    v = (v | (v >> 2)) & 0x030C30C3u;
    v = (v | (v >> 4)) & 0x0300F00Fu;
    v = (v | (v >> 8)) & 0x030000FFu;
    v = (v | (v >> 16)) & 0x000003FFu;
    return v;
}

// Distinct cells around c along one axis (periodic axes wrap; with fewer
// than three cells on a periodic axis every cell is listed once).
__device__ __forceinline__ int axis_cells(int c, int nc, int periodic, int out[3])
{
    int k = 0;
    if (periodic) {
        if (nc >= 3) {
            out[0] = c == 0 ? nc - 1 : c - 1;
            out[1] = c;
            out[2] = c == nc - 1 ? 0 : c + 1;
            k = 3;
        } else {
            for (int v = 0; v < nc; ++v) out[k++] = v;
        }
    } else {
        if (c > 0) out[k++] = c - 1;
        out[k++] = c;
        if (c < nc - 1) out[k++] = c + 1;
    }
    return k;
}

__device__ __forceinline__ double min_image(double d, int periodic, double len, double half)
{
    if (periodic) {
        if (d > half) d -= len;
        else if (d < -half) d += len;
    }
    return d;
}

// M4 spline shape w(q) and slope w'(q).
template <typename R>
__device__ __forceinline__ R m4_w(R q)
{
    const R one = R(1), two = R(2);
    R t = two - q;
    R inner = one + q * q * (R(-1.5) + R(0.75) * q);
    R outer = R(0.25) * t * t * t;
    return q < one ? inner : (q < two ? outer : R(0));
}

template <typename R>
__device__ __forceinline__ R m4_dw(R q)
{
    const R one = R(1), two = R(2);
    R t = two - q;
    R inner = q * (R(-3) + R(2.25) * q);
    R outer = R(-0.75) * t * t;
    return q < one ? inner : (q < two ? outer : R(0));
}

// ---------------------------------------------------------------------------
// Neighbour search: one lane per particle, the 27 cells around its cell,
// exact FP64 relation, ELL column-major output.
__global__ void __launch_bounds__(256)
find_neighbors_kernel(int64_t n, const double *__restrict__ x, const double *__restrict__ y,
                      const double *__restrict__ z, const double *__restrict__ h,
                      const uint32_t *__restrict__ keys, const int32_t *__restrict__ cstart,
                      const int32_t *__restrict__ cend, Grid g, int max_nb,
                      int32_t *__restrict__ count, int32_t *__restrict__ idx,
                      uint32_t *status)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double xi = x[i], yi = y[i], zi = z[i], hi = h[i];
    const uint32_t key = keys[i];
    int cxs[3], cys[3], czs[3];
    const int kx = axis_cells((int)compact3(key), g.nc[0], g.periodic[0], cxs);
    const int ky = axis_cells((int)compact3(key >> 1), g.nc[1], g.periodic[1], cys);
    const int kz = axis_cells((int)compact3(key >> 2), g.nc[2], g.periodic[2], czs);
    int cnt = 0;
    for (int a = 0; a < kz; ++a) {
        for (int b = 0; b < ky; ++b) {
            const int64_t row = ((int64_t)czs[a] * g.nc[1] + cys[b]) * g.nc[0];
            for (int c = 0; c < kx; ++c) {
                const int64_t cell = row + cxs[c];
                const int32_t s = cstart[cell], e = cend[cell];
                for (int32_t j = s; j < e; ++j) {
                    if (j == i) continue;
                    const double dx = min_image(xi - x[j], g.periodic[0], g.len[0], g.half[0]);
                    const double dy = min_image(yi - y[j], g.periodic[1], g.len[1], g.half[1]);
                    const double dz = min_image(zi - z[j], g.periodic[2], g.len[2], g.half[2]);
                    const double r2 = __builtin_fma(dz, dz, __builtin_fma(dy, dy, dx * dx));
                    const double sr = 2.0 * fmax(hi, h[j]);
                    if (r2 < sr * sr) {
                        if (cnt < max_nb) idx[(int64_t)cnt * n + i] = j;
                        ++cnt;
                    }
                }
            }
        }
    }
    count[i] = cnt;
    if (cnt > max_nb) atomicOr(status, ST_CAPACITY);
}

// ---------------------------------------------------------------------------
// Summation density, FP64 pair arithmetic.
__global__ void __launch_bounds__(256)
density_fp64_kernel(int64_t n, const double *__restrict__ x, const double *__restrict__ y,
                    const double *__restrict__ z, const double *__restrict__ h,
                    const double *__restrict__ m, const int32_t *__restrict__ count,
                    const int32_t *__restrict__ idx, int max_nb, Grid g,
                    double *__restrict__ rho)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double xi = x[i], yi = y[i], zi = z[i], hi = h[i];
    const double inv_h = 1.0 / hi;
    double sum = m[i];  // w(0) = 1
    const int cnt = min(count[i], max_nb);
    for (int k = 0; k < cnt; ++k) {
        const int32_t j = idx[(int64_t)k * n + i];
        const double dx = min_image(xi - x[j], g.periodic[0], g.len[0], g.half[0]);
        const double dy = min_image(yi - y[j], g.periodic[1], g.len[1], g.half[1]);
        const double dz = min_image(zi - z[j], g.periodic[2], g.len[2], g.half[2]);
        const double r = sqrt(__builtin_fma(dz, dz, __builtin_fma(dy, dy, dx * dx)));
        sum += m[j] * m4_w(r * inv_h);
    }
    rho[i] = sum * (kInvPi * inv_h * inv_h * inv_h);
}

// Summation density, FP32 pair arithmetic.
__global__ void __launch_bounds__(256)
density_fp32_kernel(int64_t n, const double *__restrict__ x, const double *__restrict__ y,
                    const double *__restrict__ z, const float *__restrict__ hf,
                    const float *__restrict__ mf, const int32_t *__restrict__ count,
                    const int32_t *__restrict__ idx, int max_nb, Grid g,
                    double *__restrict__ rho)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double xi = x[i], yi = y[i], zi = z[i];
    const float inv_h = 1.0f / hf[i];
    float sum = mf[i];
    const int cnt = min(count[i], max_nb);
    for (int k = 0; k < cnt; ++k) {
        const int32_t j = idx[(int64_t)k * n + i];
        const float dx = (float)min_image(xi - x[j], g.periodic[0], g.len[0], g.half[0]);
        const float dy = (float)min_image(yi - y[j], g.periodic[1], g.len[1], g.half[1]);
        const float dz = (float)min_image(zi - z[j], g.periodic[2], g.len[2], g.half[2]);
        const float r = sqrtf(__builtin_fmaf(dz, dz, __builtin_fmaf(dy, dy, dx * dx)));
        sum = __builtin_fmaf(mf[j], m4_w(r * inv_h), sum);
    }
    rho[i] = (double)(sum * ((float)kInvPi * inv_h * inv_h * inv_h));
}

// ---------------------------------------------------------------------------
// EOS; also the FP32 copies of rho, P/rho^2 and c.
__global__ void __launch_bounds__(256)
eos_kernel(int64_t n, int eos, double rho0, double c0, double gamma_tait,
           double gamma_gas, const double *__restrict__ rho, const double *__restrict__ u,
           const double *__restrict__ rho_ref, const double *__restrict__ p_bg,
           double *__restrict__ p, double *__restrict__ c, double *__restrict__ pr2,
           float *__restrict__ rhof, float *__restrict__ pr2f, float *__restrict__ cf)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double r = rho[i];
    double P, C;
    if (eos == SPH_EOS_TAIT) {
        const double B = rho0 * c0 * c0 / gamma_tait;
        const double xr = r / rho_ref[i];
        const double x2 = xr * xr, x4 = x2 * x2, x6 = x4 * x2, x7 = x6 * xr;
        const double x3 = x2 * xr;
        P = p_bg[i] + B * (x7 - 1.0);
        C = c0 * x3;
    } else {
        P = (gamma_gas - 1.0) * r * u[i];
        C = sqrt(gamma_gas * (gamma_gas - 1.0) * u[i]);
    }
    const double q = P / (r * r);
    p[i] = P;
    c[i] = C;
    pr2[i] = q;
    rhof[i] = (float)r;
    pr2f[i] = (float)q;
    cf[i] = (float)C;
}

// ---------------------------------------------------------------------------
// Momentum and energy with Monaghan artificial viscosity, FP64.
__global__ void __launch_bounds__(256)
momentum_fp64_kernel(int64_t n, const double *__restrict__ x, const double *__restrict__ y,
                     const double *__restrict__ z, const double *__restrict__ vx,
                     const double *__restrict__ vy, const double *__restrict__ vz,
                     const double *__restrict__ h, const double *__restrict__ m,
                     const double *__restrict__ rho, const double *__restrict__ cs,
                     const double *__restrict__ pr2, const int32_t *__restrict__ count,
                     const int32_t *__restrict__ idx, int max_nb, Grid g, double alpha,
                     double beta, double eta2, double *__restrict__ ax,
                     double *__restrict__ ay, double *__restrict__ az,
                     double *__restrict__ dudt, double *__restrict__ mumax)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double xi = x[i], yi = y[i], zi = z[i];
    const double vxi = vx[i], vyi = vy[i], vzi = vz[i];
    const double hi = h[i], rhoi = rho[i], ci = cs[i], pi = pr2[i];
    const double inv_hi = 1.0 / hi;
    const double fi = kInvPi * (inv_hi * inv_hi) * (inv_hi * inv_hi);
    double sx = 0.0, sy = 0.0, sz = 0.0, su = 0.0, mum = 0.0;
    const int cnt = min(count[i], max_nb);
    for (int k = 0; k < cnt; ++k) {
        const int32_t j = idx[(int64_t)k * n + i];
        const double dx = min_image(xi - x[j], g.periodic[0], g.len[0], g.half[0]);
        const double dy = min_image(yi - y[j], g.periodic[1], g.len[1], g.half[1]);
        const double dz = min_image(zi - z[j], g.periodic[2], g.len[2], g.half[2]);
        const double r2 = __builtin_fma(dz, dz, __builtin_fma(dy, dy, dx * dx));
        const double r = sqrt(r2);
        const double hj = h[j];
        const double inv_hj = 1.0 / hj;
        const double fj = kInvPi * (inv_hj * inv_hj) * (inv_hj * inv_hj);
        const double dwbar = 0.5 * (fi * m4_dw(r * inv_hi) + fj * m4_dw(r * inv_hj));
        const double F = r > 0.0 ? dwbar / r : 0.0;
        const double wx = vxi - vx[j], wy = vyi - vy[j], wz = vzi - vz[j];
        const double vdotr = __builtin_fma(wz, dz, __builtin_fma(wy, dy, wx * dx));
        const double hbar = 0.5 * (hi + hj);
        double mu = 0.0;
        if (vdotr < 0.0) mu = hbar * vdotr / __builtin_fma(eta2 * hbar, hbar, r2);
        const double cbar = 0.5 * (ci + cs[j]);
        const double rhobar = 0.5 * (rhoi + rho[j]);
        const double Pi = mu * (beta * mu - alpha * cbar) / rhobar;
        const double mG = m[j] * (pi + pr2[j] + Pi) * F;
        sx = __builtin_fma(-mG, dx, sx);
        sy = __builtin_fma(-mG, dy, sy);
        sz = __builtin_fma(-mG, dz, sz);
        su = __builtin_fma(mG, vdotr, su);
        mum = fmax(mum, fabs(mu));
    }
    ax[i] = sx;
    ay[i] = sy;
    az[i] = sz;
    dudt[i] = 0.5 * su;
    mumax[i] = mum;
}

// Momentum and energy, FP32 pair arithmetic.
__global__ void __launch_bounds__(256)
momentum_fp32_kernel(int64_t n, const double *__restrict__ x, const double *__restrict__ y,
                     const double *__restrict__ z, const double *__restrict__ vx,
                     const double *__restrict__ vy, const double *__restrict__ vz,
                     const float *__restrict__ h, const float *__restrict__ m,
                     const float *__restrict__ rho, const float *__restrict__ cs,
                     const float *__restrict__ pr2, const int32_t *__restrict__ count,
                     const int32_t *__restrict__ idx, int max_nb, Grid g, float alpha,
                     float beta, float eta2, double *__restrict__ ax,
                     double *__restrict__ ay, double *__restrict__ az,
                     double *__restrict__ dudt, double *__restrict__ mumax)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double xi = x[i], yi = y[i], zi = z[i];
    const double vxi = vx[i], vyi = vy[i], vzi = vz[i];
    const float hi = h[i], rhoi = rho[i], ci = cs[i], pi = pr2[i];
    const float inv_hi = 1.0f / hi;
    const float fi = (float)kInvPi * (inv_hi * inv_hi) * (inv_hi * inv_hi);
    float sx = 0.f, sy = 0.f, sz = 0.f, su = 0.f, mum = 0.f;
    const int cnt = min(count[i], max_nb);
    for (int k = 0; k < cnt; ++k) {
        const int32_t j = idx[(int64_t)k * n + i];
        const float dx = (float)min_image(xi - x[j], g.periodic[0], g.len[0], g.half[0]);
        const float dy = (float)min_image(yi - y[j], g.periodic[1], g.len[1], g.half[1]);
        const float dz = (float)min_image(zi - z[j], g.periodic[2], g.len[2], g.half[2]);
        const float r2 = __builtin_fmaf(dz, dz, __builtin_fmaf(dy, dy, dx * dx));
        const float r = sqrtf(r2);
        const float hj = h[j];
        const float inv_hj = 1.0f / hj;
        const float fj = (float)kInvPi * (inv_hj * inv_hj) * (inv_hj * inv_hj);
        const float dwbar = 0.5f * (fi * m4_dw(r * inv_hi) + fj * m4_dw(r * inv_hj));
        const float F = r > 0.f ? dwbar / r : 0.f;
        const float wx = (float)(vxi - vx[j]), wy = (float)(vyi - vy[j]),
                    wz = (float)(vzi - vz[j]);
        const float vdotr = __builtin_fmaf(wz, dz, __builtin_fmaf(wy, dy, wx * dx));
        const float hbar = 0.5f * (hi + hj);
        float mu = 0.f;
        if (vdotr < 0.f) mu = hbar * vdotr / __builtin_fmaf(eta2 * hbar, hbar, r2);
        const float cbar = 0.5f * (ci + cs[j]);
        const float rhobar = 0.5f * (rhoi + rho[j]);
        const float Pi = mu * (beta * mu - alpha * cbar) / rhobar;
        const float mG = m[j] * (pi + pr2[j] + Pi) * F;
        sx = __builtin_fmaf(-mG, dx, sx);
        sy = __builtin_fmaf(-mG, dy, sy);
        sz = __builtin_fmaf(-mG, dz, sz);
        su = __builtin_fmaf(mG, vdotr, su);
        mum = fmaxf(mum, fabsf(mu));
    }
    ax[i] = (double)sx;
    ay[i] = (double)sy;
    az[i] = (double)sz;
    dudt[i] = 0.5 * (double)su;
    mumax[i] = (double)mum;
}

inline unsigned blocks_for(int64_t n, int t) { return (unsigned)((n + t - 1) / t); }

}  // namespace

hipError_t launch_find_neighbors(sph_ctx ctx, const sph_particles &p, const sph_nbrs &nb)
{
    find_neighbors_kernel<<<blocks_for(p.n, 256), 256, 0, ctx->stream>>>(
        p.n, p.x, p.y, p.z, p.h, ctx->sorted_keys, ctx->cell_start, ctx->cell_end, ctx->grid,
        nb.max_nb, nb.count, nb.idx, ctx->status_dev);
    return hipGetLastError();
}

hipError_t launch_density(sph_ctx ctx, const sph_particles &p, const sph_nbrs &nb,
                          int precision, double *rho)
{
    if (precision == SPH_FP32_PAIR) {
        density_fp32_kernel<<<blocks_for(p.n, 256), 256, 0, ctx->stream>>>(
            p.n, p.x, p.y, p.z, ctx->hf, ctx->mf, nb.count, nb.idx, nb.max_nb, ctx->grid, rho);
    } else {
        density_fp64_kernel<<<blocks_for(p.n, 256), 256, 0, ctx->stream>>>(
            p.n, p.x, p.y, p.z, p.h, p.m, nb.count, nb.idx, nb.max_nb, ctx->grid, rho);
    }
    return hipGetLastError();
}

hipError_t launch_eos(sph_ctx ctx, const sph_particles &p, const sph_params &prm,
                      const sph_fields &f)
{
    eos_kernel<<<blocks_for(p.n, 256), 256, 0, ctx->stream>>>(
        p.n, prm.eos, prm.rho0, prm.c0, prm.gamma_tait, prm.gamma_gas, f.rho, p.u, p.rho_ref,
        p.p_bg, f.p, f.c, f.pr2, ctx->rhof, ctx->pr2f, ctx->cf);
    return hipGetLastError();
}

hipError_t launch_momentum(sph_ctx ctx, const sph_particles &p, const sph_nbrs &nb,
                           const sph_params &prm, const sph_fields &f, const sph_accel &a)
{
    if (prm.precision == SPH_FP32_PAIR) {
        momentum_fp32_kernel<<<blocks_for(p.n, 256), 256, 0, ctx->stream>>>(
            p.n, p.x, p.y, p.z, p.vx, p.vy, p.vz, ctx->hf, ctx->mf, ctx->rhof, ctx->cf,
            ctx->pr2f, nb.count, nb.idx, nb.max_nb, ctx->grid, (float)prm.alpha,
            (float)prm.beta, (float)prm.eta2, a.ax, a.ay, a.az, a.dudt, a.mumax);
    } else {
        momentum_fp64_kernel<<<blocks_for(p.n, 256), 256, 0, ctx->stream>>>(
            p.n, p.x, p.y, p.z, p.vx, p.vy, p.vz, p.h, p.m, f.rho, f.c, f.pr2, nb.count,
            nb.idx, nb.max_nb, ctx->grid, prm.alpha, prm.beta, prm.eta2, a.ax, a.ay, a.az,
            a.dudt, a.mumax);
    }
    return hipGetLastError();
}

}  // namespace sph
