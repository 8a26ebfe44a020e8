// Algorithm 1, steps 5 and 6 on the GPU: kick-drift-kick update with a
// global dt held in device memory, and the global dt itself as a two-level
// min reduction (wavefront shuffles, then LDS, then one block over the block
// partials). The same pass sums the conserved totals in FP64 in a fixed tree
// order, so they are identical from run to run.
#include <algorithm>

#include "sph_internal.h"

namespace sph {
namespace {

__global__ void __launch_bounds__(256)
integrate_kernel(int64_t n, int stage, const double *__restrict__ dt_dev, Grid g,
                 double *__restrict__ x, double *__restrict__ y, double *__restrict__ z,
                 double *__restrict__ vx, double *__restrict__ vy, double *__restrict__ vz,
                 double *__restrict__ u, const double *__restrict__ ax,
                 const double *__restrict__ ay, const double *__restrict__ az,
                 const double *__restrict__ dudt, const double *__restrict__ gx,
                 const double *__restrict__ gy, const double *__restrict__ gz,
                 uint32_t *status)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double dt = dt_dev[0];
    const double half = 0.5 * dt;
    double tx = ax[i], ty = ay[i], tz = az[i];
    if (gx) {
        tx += gx[i];
        ty += gy[i];
        tz += gz[i];
    }
    const double nvx = vx[i] + half * tx;
    const double nvy = vy[i] + half * ty;
    const double nvz = vz[i] + half * tz;
    const double nu = u[i] + half * dudt[i];
    vx[i] = nvx;
    vy[i] = nvy;
    vz[i] = nvz;
    u[i] = nu;
    if (stage == SPH_KICK_DRIFT) {
        double p[3] = {x[i] + dt * nvx, y[i] + dt * nvy, z[i] + dt * nvz};
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            if (!g.periodic[a]) continue;
            if (p[a] >= g.hi[a]) p[a] -= g.len[a];
            else if (p[a] < g.lo[a]) p[a] += g.len[a];
        }
        x[i] = p[0];
        y[i] = p[1];
        z[i] = p[2];
    } else {
        const double s = x[i] + y[i] + z[i] + nvx + nvy + nvz + nu;
        if (!isfinite(s)) atomicOr(status, ST_NONFINITE);
    }
}

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    return v;
}

__device__ __forceinline__ double wave_min(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_down(v, o, 64));
    return v;
}

// Block-level combine of kRedFields values (field 0 by min, the others by
// sum), fixed order; result valid in thread 0.
__device__ __forceinline__ void block_combine(double v[kRedFields],
                                              double (*lds)[kRedThreads / 64])
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    v[0] = wave_min(v[0]);
#pragma unroll
    for (int k = 1; k < kRedFields; ++k) v[k] = wave_sum(v[k]);
    if (lane == 0) {
#pragma unroll
        for (int k = 0; k < kRedFields; ++k) lds[k][wave] = v[k];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double r0 = lds[0][0];
        for (int w = 1; w < kRedThreads / 64; ++w) r0 = fmin(r0, lds[0][w]);
        v[0] = r0;
#pragma unroll
        for (int k = 1; k < kRedFields; ++k) {
            double s = lds[k][0];
            for (int w = 1; w < kRedThreads / 64; ++w) s += lds[k][w];
            v[k] = s;
        }
    }
}

// Per-block partials: dt candidate min and the 8 conserved totals.
__global__ void __launch_bounds__(kRedThreads)
timestep_partial_kernel(int64_t n, const double *__restrict__ h, const double *__restrict__ c,
                        const double *__restrict__ mumax, const double *__restrict__ ax,
                        const double *__restrict__ ay, const double *__restrict__ az,
                        const double *__restrict__ gx, const double *__restrict__ gy,
                        const double *__restrict__ gz, const double *__restrict__ x,
                        const double *__restrict__ y, const double *__restrict__ z,
                        const double *__restrict__ vx, const double *__restrict__ vy,
                        const double *__restrict__ vz, const double *__restrict__ u,
                        const double *__restrict__ m, double alpha, double beta,
                        double c_cfl, double c_force, double *__restrict__ part)
{
    __shared__ double lds[kRedFields][kRedThreads / 64];
    double v[kRedFields];
    v[0] = INFINITY;
#pragma unroll
    for (int k = 1; k < kRedFields; ++k) v[k] = 0.0;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const double hi = h[i], ci = c[i];
        double d = c_cfl * hi / (ci + 1.2 * (alpha * ci + beta * mumax[i]));
        double tx = ax[i], ty = ay[i], tz = az[i];
        if (gx) {
            tx += gx[i];
            ty += gy[i];
            tz += gz[i];
        }
        const double amag = sqrt(tx * tx + ty * ty + tz * tz);
        if (amag > 0.0) d = fmin(d, c_force * sqrt(hi / amag));
        v[0] = fmin(v[0], d);
        const double mi = m[i], px = x[i], py = y[i], pz = z[i];
        const double qx = vx[i], qy = vy[i], qz = vz[i];
        v[1] += mi;
        v[2] += mi * qx;
        v[3] += mi * qy;
        v[4] += mi * qz;
        v[5] += mi * (py * qz - pz * qy);
        v[6] += mi * (pz * qx - px * qz);
        v[7] += mi * (px * qy - py * qx);
        v[8] += mi * (0.5 * (qx * qx + qy * qy + qz * qz) + u[i]);
    }
    block_combine(v, lds);
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < kRedFields; ++k) part[(int64_t)k * kRedMaxBlocks + blockIdx.x] = v[k];
    }
}

__global__ void __launch_bounds__(kRedThreads)
timestep_final_kernel(int nblocks, const double *__restrict__ part,
                      double *__restrict__ dt_dev, double *__restrict__ diag)
{
    __shared__ double lds[kRedFields][kRedThreads / 64];
    double v[kRedFields];
    v[0] = INFINITY;
#pragma unroll
    for (int k = 1; k < kRedFields; ++k) v[k] = 0.0;
    for (int b = threadIdx.x; b < nblocks; b += kRedThreads) {
        v[0] = fmin(v[0], part[b]);
#pragma unroll
        for (int k = 1; k < kRedFields; ++k) v[k] += part[(int64_t)k * kRedMaxBlocks + b];
    }
    block_combine(v, lds);
    if (threadIdx.x == 0) {
        dt_dev[0] = v[0];
        if (diag) {
#pragma unroll
            for (int k = 1; k < kRedFields; ++k) diag[k - 1] = v[k];
        }
    }
}

// ---------------------------------------------------------------------------
// Ensemble: the same update and reductions per run. A particle is advanced
// only when its run is stepping (not at its t = 0 evaluation, not when it is
// being dropped), with its run's dt and box.
__global__ void __launch_bounds__(256)
integrate_batch_kernel(BatchDev b, int stage, double *__restrict__ F,
                       const double *__restrict__ ax, const double *__restrict__ ay,
                       const double *__restrict__ az, const double *__restrict__ dudt)
{
    const int64_t cap = b.cap;
    const int64_t n = stage == SPH_KICK_DRIFT ? b.hdr->n_in : b.hdr->n_out;
    double *x = F, *y = F + cap, *z = F + 2 * cap;
    double *vx = F + 3 * cap, *vy = F + 4 * cap, *vz = F + 5 * cap, *u = F + 6 * cap;
    const int64_t step = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += step) {
        const int s = b.slot[i];
        const RunDev &r = b.runs[s];
        if (r.phase != RUN_STEP) continue;
        const Grid &g = r.grid;
        const double dt = b.dt[s];
        const double half = 0.5 * dt;
        const double tx = ax[i], ty = ay[i], tz = az[i];
        const double nvx = vx[i] + half * tx;
        const double nvy = vy[i] + half * ty;
        const double nvz = vz[i] + half * tz;
        const double nu = u[i] + half * dudt[i];
        vx[i] = nvx;
        vy[i] = nvy;
        vz[i] = nvz;
        u[i] = nu;
        if (stage == SPH_KICK_DRIFT) {
            double p[3] = {x[i] + dt * nvx, y[i] + dt * nvy, z[i] + dt * nvz};
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                if (!g.periodic[a]) continue;
                if (p[a] >= g.hi[a]) p[a] -= g.len[a];
                else if (p[a] < g.lo[a]) p[a] += g.len[a];
            }
            x[i] = p[0];
            y[i] = p[1];
            z[i] = p[2];
        } else {
            const double sm = x[i] + y[i] + z[i] + nvx + nvy + nvz + nu;
            if (!isfinite(sm)) atomicOr(&b.status[s], ST_NONFINITE);
        }
    }
}

// Partials per run: reduction block q of a run covers its particles
// [256 q, 256 q + 256), the same blocks and the same tree as the single-run
// reduction of that run (which covers 256 consecutive particles per block
// whenever the run has at most kRedMaxBlocks * 256 particles).
__global__ void __launch_bounds__(kRedThreads)
timestep_partial_batch_kernel(BatchDev b, const double *__restrict__ F,
                              const double *__restrict__ c, const double *__restrict__ mumax,
                              const double *__restrict__ ax, const double *__restrict__ ay,
                              const double *__restrict__ az, double *__restrict__ part)
{
    __shared__ double lds[kRedFields][kRedThreads / 64];
    const BatchHdr *hd = b.hdr;
    const int64_t cap = b.cap;
    const double *x = F, *y = F + cap, *z = F + 2 * cap;
    const double *vx = F + 3 * cap, *vy = F + 4 * cap, *vz = F + 5 * cap, *u = F + 6 * cap;
    const double *h = F + 7 * cap, *m = F + 8 * cap;
    const int64_t nred = hd->nred;
    const int nlive = hd->nlive;
    for (int64_t vb = blockIdx.x; vb < nred; vb += gridDim.x) {
        int lo = 0, hi = nlive - 1;
        while (lo < hi) {  // last live run with red_base <= vb
            const int mid = (lo + hi + 1) >> 1;
            if (hd->live_red_base[mid] <= vb) lo = mid; else hi = mid - 1;
        }
        const RunDev &r = b.runs[hd->live_slot[lo]];
        const int64_t q = vb - r.red_base;
        const int64_t i = (int64_t)r.start + q * kRedThreads + threadIdx.x;
        const int64_t end = (int64_t)r.start + r.n;
        double v[kRedFields];
        v[0] = INFINITY;
#pragma unroll
        for (int k = 1; k < kRedFields; ++k) v[k] = 0.0;
        if (i < end) {
            const double hi_ = h[i], ci = c[i];
            double d = r.c_cfl * hi_ / (ci + 1.2 * (r.alpha * ci + r.beta * mumax[i]));
            const double tx = ax[i], ty = ay[i], tz = az[i];
            const double amag = sqrt(tx * tx + ty * ty + tz * tz);
            if (amag > 0.0) d = fmin(d, r.c_force * sqrt(hi_ / amag));
            v[0] = fmin(v[0], d);
            const double mi = m[i], px = x[i], py = y[i], pz = z[i];
            const double qx = vx[i], qy = vy[i], qz = vz[i];
            v[1] += mi;
            v[2] += mi * qx;
            v[3] += mi * qy;
            v[4] += mi * qz;
            v[5] += mi * (py * qz - pz * qy);
            v[6] += mi * (pz * qx - px * qz);
            v[7] += mi * (px * qy - py * qx);
            v[8] += mi * (0.5 * (qx * qx + qy * qy + qz * qz) + u[i]);
        }
        block_combine(v, lds);
        if (threadIdx.x == 0) {
#pragma unroll
            for (int k = 0; k < kRedFields; ++k) part[(int64_t)k * b.nred_cap + vb] = v[k];
        }
        __syncthreads();
    }
}

// One block per live run: its partials in the single-run final order.
__global__ void __launch_bounds__(kRedThreads)
timestep_final_batch_kernel(BatchDev b, const double *__restrict__ part)
{
    __shared__ double lds[kRedFields][kRedThreads / 64];
    const BatchHdr *hd = b.hdr;
    for (int k = blockIdx.x; k < hd->nlive; k += gridDim.x) {
        const int s = hd->live_slot[k];
        const int64_t base = hd->live_red_base[k];
        const int nb = hd->live_red_base[k + 1] - hd->live_red_base[k];
        double v[kRedFields];
        v[0] = INFINITY;
#pragma unroll
        for (int f = 1; f < kRedFields; ++f) v[f] = 0.0;
        for (int q = threadIdx.x; q < nb; q += kRedThreads) {
            v[0] = fmin(v[0], part[base + q]);
#pragma unroll
            for (int f = 1; f < kRedFields; ++f) v[f] += part[(int64_t)f * b.nred_cap + base + q];
        }
        block_combine(v, lds);
        if (threadIdx.x == 0) {
            b.dt[s] = v[0];
#pragma unroll
            for (int f = 1; f < kRedFields; ++f) b.diag[(int64_t)s * 8 + f - 1] = v[f];
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// Individual time steps in power-of-two bins. The per-particle criterion is
// the global one's (same operations), its min and max give the largest step
// D = min(max, min 2^max_bin), and a particle's bin is the smallest b with
// D / 2^b <= its criterion (exact: scaling by a power of two).
__global__ void __launch_bounds__(256)
block_criterion_kernel(int64_t n, const double *__restrict__ h, const double *__restrict__ c,
                       const double *__restrict__ mumax, const double *__restrict__ ax,
                       const double *__restrict__ ay, const double *__restrict__ az,
                       const double *__restrict__ gx, const double *__restrict__ gy,
                       const double *__restrict__ gz, double alpha, double beta, double c_cfl,
                       double c_force, double *__restrict__ dtc, double *__restrict__ part)
{
    __shared__ double lo[256], hi[256];
    double mn = INFINITY, mx = -INFINITY;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const double hi_ = h[i], ci = c[i];
        double d = c_cfl * hi_ / (ci + 1.2 * (alpha * ci + beta * mumax[i]));
        double tx = ax[i], ty = ay[i], tz = az[i];
        if (gx) {
            tx += gx[i];
            ty += gy[i];
            tz += gz[i];
        }
        const double amag = sqrt(tx * tx + ty * ty + tz * tz);
        if (amag > 0.0) d = fmin(d, c_force * sqrt(hi_ / amag));
        dtc[i] = d;
        mn = fmin(mn, d);
        mx = fmax(mx, d);
    }
    lo[threadIdx.x] = mn;
    hi[threadIdx.x] = mx;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            lo[threadIdx.x] = fmin(lo[threadIdx.x], lo[threadIdx.x + w]);
            hi[threadIdx.x] = fmax(hi[threadIdx.x], hi[threadIdx.x + w]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = lo[0];
        part[2 * blockIdx.x + 1] = hi[0];
    }
}

// D from the block partials (one wave; min and max are exact in any order)
__global__ void __launch_bounds__(64)
block_step_kernel(int nblk, const double *__restrict__ part, int max_bin,
                  double *__restrict__ dt_dev)
{
    double mn = INFINITY, mx = -INFINITY;
    for (int b = threadIdx.x; b < nblk; b += 64) {
        mn = fmin(mn, part[2 * b]);
        mx = fmax(mx, part[2 * b + 1]);
    }
    for (int o = 32; o > 0; o >>= 1) {
        mn = fmin(mn, __shfl_xor(mn, o, 64));
        mx = fmax(mx, __shfl_xor(mx, o, 64));
    }
    if (threadIdx.x == 0) dt_dev[0] = fmin(mx, ldexp(mn, max_bin));
}

__global__ void __launch_bounds__(256)
block_bins_kernel(int64_t n, const double *__restrict__ dtc, int max_bin,
                  const double *__restrict__ dt_dev, double *__restrict__ bin,
                  uint32_t *__restrict__ words)
{
    const double D = dt_dev[0];
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int b = 0;
    if (i < n) {
        b = max_bin;
        for (int k = max_bin; k >= 0; --k)
            if (ldexp(D, -k) <= dtc[i]) b = k;
        bin[i] = (double)b;
    }
    // deepest bin: one atomic per wave (every lane takes part in the
    // reduction), and only above the value already there (same-address
    // atomics serialise in their L2 channel)
    int m = b;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) m = max(m, __shfl_xor(m, o, 64));
    if ((threadIdx.x & 63) == 0 &&
        (uint32_t)m > __hip_atomic_load(&words[0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
        atomicMax(&words[0], (uint32_t)m);
}

__global__ void __launch_bounds__(64)
clear_words2_kernel(uint32_t *__restrict__ w)
{
    if (threadIdx.x < 2) w[threadIdx.x] = 0u;
}

// Half kick of the particles of bin b whose step opens (stage 0: sub mod
// 2^(B-b) == 0) or closes (stage 1: (sub + 1) mod 2^(B-b) == 0), with their
// step D / 2^b; the same operations as the global kick.
__global__ void __launch_bounds__(256)
kick_bins_kernel(int64_t n, int stage, int sub, int B, const double *__restrict__ dt_dev,
                 const double *__restrict__ bin, double *__restrict__ vx, double *__restrict__ vy,
                 double *__restrict__ vz, double *__restrict__ u, const double *__restrict__ ax,
                 const double *__restrict__ ay, const double *__restrict__ az,
                 const double *__restrict__ dudt, const double *__restrict__ gx,
                 const double *__restrict__ gy, const double *__restrict__ gz,
                 uint32_t *status)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int b = (int)bin[i];
    const int mask = (1 << (B - b)) - 1;
    if (((stage == 0 ? sub : sub + 1) & mask) != 0) return;
    const double dt = ldexp(dt_dev[0], -b);
    const double half = 0.5 * dt;
    double tx = ax[i], ty = ay[i], tz = az[i];
    if (gx) {
        tx += gx[i];
        ty += gy[i];
        tz += gz[i];
    }
    const double nvx = vx[i] + half * tx;
    const double nvy = vy[i] + half * ty;
    const double nvz = vz[i] + half * tz;
    const double nu = u[i] + half * dudt[i];
    vx[i] = nvx;
    vy[i] = nvy;
    vz[i] = nvz;
    u[i] = nu;
    if (stage == 1 && !isfinite(nvx + nvy + nvz + nu)) atomicOr(status, ST_NONFINITE);
}

__global__ void __launch_bounds__(256)
drift_kernel(int64_t n, int B, const double *__restrict__ dt_dev, Grid g,
             double *__restrict__ x, double *__restrict__ y, double *__restrict__ z,
             const double *__restrict__ vx, const double *__restrict__ vy,
             const double *__restrict__ vz)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double dt = ldexp(dt_dev[0], -B);
    double p[3] = {x[i] + dt * vx[i], y[i] + dt * vy[i], z[i] + dt * vz[i]};
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        if (!g.periodic[a]) continue;
        if (p[a] >= g.hi[a]) p[a] -= g.len[a];
        else if (p[a] < g.lo[a]) p[a] += g.len[a];
    }
    x[i] = p[0];
    y[i] = p[1];
    z[i] = p[2];
}

__global__ void copy_kernel(int64_t n, double *__restrict__ dst, const double *__restrict__ src)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = src[i];
}

inline unsigned blocks_for(int64_t n, int t) { return (unsigned)((n + t - 1) / t); }

}  // namespace

hipError_t launch_integrate(sph_ctx ctx, const sph_particles &p, const Grid &g, int stage,
                            const double *dt_dev, const sph_accel &a)
{
    integrate_kernel<<<blocks_for(p.n, 256), 256, 0, ctx->stream>>>(
        p.n, stage, dt_dev, g, p.x, p.y, p.z, p.vx, p.vy, p.vz, p.u, a.ax, a.ay, a.az, a.dudt,
        p.gx, p.gy, p.gz, ctx->status_dev);
    return hipGetLastError();
}

hipError_t launch_timestep(sph_ctx ctx, const sph_particles &p, const sph_params &prm,
                           const sph_fields &f, const sph_accel &a, double *dt_dev,
                           double *diag_dev)
{
    int64_t nb = (p.n + kRedThreads - 1) / kRedThreads;
    if (nb > kRedMaxBlocks) nb = kRedMaxBlocks;
    if (nb > 0) {
        timestep_partial_kernel<<<(unsigned)nb, kRedThreads, 0, ctx->stream>>>(
            p.n, p.h, f.c, a.mumax, a.ax, a.ay, a.az, p.gx, p.gy, p.gz, p.x, p.y, p.z, p.vx,
            p.vy, p.vz, p.u, p.m, prm.alpha, prm.beta, prm.c_cfl, prm.c_force, ctx->red_part);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    timestep_final_kernel<<<1, kRedThreads, 0, ctx->stream>>>((int)nb, ctx->red_part, dt_dev,
                                                              diag_dev);
    return hipGetLastError();
}

hipError_t launch_block_bins(sph_ctx ctx, const sph_particles &p, const sph_params &prm,
                             const sph_fields &f, const sph_accel &a, int max_bin, double *bin,
                             double *dt_dev)
{
    const int nblk = (int)std::min<int64_t>(kRedMaxBlocks, (p.n + 255) / 256);
    clear_words2_kernel<<<1, 64, 0, ctx->stream>>>(ctx->blk_words);
    block_criterion_kernel<<<(unsigned)nblk, 256, 0, ctx->stream>>>(
        p.n, p.h, f.c, a.mumax, a.ax, a.ay, a.az, p.gx, p.gy, p.gz, prm.alpha, prm.beta,
        prm.c_cfl, prm.c_force, ctx->dtc, ctx->red_part);
    block_step_kernel<<<1, 64, 0, ctx->stream>>>(nblk, ctx->red_part, max_bin, dt_dev);
    block_bins_kernel<<<blocks_for(p.n, 256), 256, 0, ctx->stream>>>(
        p.n, ctx->dtc, max_bin, dt_dev, bin, ctx->blk_words);
    return hipGetLastError();
}

hipError_t launch_kick_bins(sph_ctx ctx, const sph_particles &p, int stage, int sub, int B,
                            const double *dt_dev, const double *bin, const sph_accel &a)
{
    kick_bins_kernel<<<blocks_for(p.n, 256), 256, 0, ctx->stream>>>(
        p.n, stage, sub, B, dt_dev, bin, p.vx, p.vy, p.vz, p.u, a.ax, a.ay, a.az, a.dudt, p.gx,
        p.gy, p.gz, ctx->status_dev);
    return hipGetLastError();
}

hipError_t launch_drift(sph_ctx ctx, const sph_particles &p, const Grid &g, int B,
                        const double *dt_dev)
{
    drift_kernel<<<blocks_for(p.n, 256), 256, 0, ctx->stream>>>(p.n, B, dt_dev, g, p.x, p.y, p.z,
                                                                 p.vx, p.vy, p.vz);
    return hipGetLastError();
}

hipError_t launch_copy(sph_ctx ctx, double *dst, const double *src, int64_t n)
{
    if (n <= 0) return hipSuccess;
    copy_kernel<<<blocks_for(n, 256), 256, 0, ctx->stream>>>(n, dst, src);
    return hipGetLastError();
}

hipError_t launch_integrate_batch(sph_ctx ctx, const BatchDev &b, int stage, double *F,
                                  const double *ax, const double *ay, const double *az,
                                  const double *dudt)
{
    const unsigned g = std::min<unsigned>(blocks_for(b.cap, 256), 4096u);
    integrate_batch_kernel<<<g, 256, 0, ctx->stream>>>(b, stage, F, ax, ay, az, dudt);
    return hipGetLastError();
}

hipError_t launch_timestep_batch(sph_ctx ctx, const BatchDev &b, const double *F,
                                 const double *c, const double *mumax, const double *ax,
                                 const double *ay, const double *az, double *part)
{
    const unsigned g = (unsigned)std::min<int64_t>(b.nred_cap, 2048);
    timestep_partial_batch_kernel<<<g, kRedThreads, 0, ctx->stream>>>(b, F, c, mumax, ax, ay,
                                                                       az, part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    timestep_final_batch_kernel<<<kEnsMaxSlots, kRedThreads, 0, ctx->stream>>>(b, part);
    return hipGetLastError();
}

}  // namespace sph
