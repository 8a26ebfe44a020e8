// Algorithm 1, step 3 on the GPU: summation density, EOS, and momentum and
// energy with artificial viscosity.
//
// Gather form throughout: each particle owns its outputs and sums its own
// pairs in the order of its neighbour list, so there are no atomics on
// floating-point values and every result is the same from run to run.
//
// One lane per particle; at step k every lane needs the record of its own
// k-th neighbour. Loaded lane by lane, each load instruction touches 64
// different cache lines, and the L1 resolves about one line per clock. So
// the records are packed (one aligned record per particle) and fetched
// cooperatively: a group of lanes loads the 16-byte chunks of ONE record, so
// an instruction touches one line per group, and the chunks are then passed
// to their owner lanes through a small per-wave LDS buffer whose padded
// stride keeps both the writes and the reads free of bank conflicts.
//
// The density and momentum pair arithmetic comes in two forms:
//   FP64:      everything FP64;
//   FP32-pair: separations and velocity differences formed in FP64 and
//              rounded to FP32, FP32 copies of h, m, rho, P/rho^2 and c, FP32
//              sums, outputs widened to FP64.
#include <algorithm>
#include <mutex>
#include <type_traits>

#include "sph_internal.h"

namespace sph {
namespace {

constexpr double kInvPi = 0.318309886183790671537767526745;
constexpr int kThreads = 256;

__device__ __forceinline__ double min_image(double d, int periodic, double len, double half)
{
    if (periodic) {
        d = d > half ? d - len : d;
        d = d < -half ? d + len : d;
    }
    return d;
}

__device__ __forceinline__ double fma_r(double a, double b, double c) { return __builtin_fma(a, b, c); }
__device__ __forceinline__ float fma_r(float a, float b, float c) { return __builtin_fmaf(a, b, c); }

// Reciprocal and reciprocal square root from the hardware estimates. The
// FP64 estimates are good to about 2^-25 relative; two Newton steps bring
// them to about one ulp (measured on MI355X), far inside the FP64 form's
// tolerance and far cheaper than the correctly rounded division and square
// root. The FP32 estimates are used as they are (about one ulp).
__device__ __forceinline__ double fast_rcp(double a)
{
    double y = __builtin_amdgcn_rcp(a);
    double e = __builtin_fma(-a, y, 1.0);
    y = __builtin_fma(y, e, y);
    e = __builtin_fma(-a, y, 1.0);
    return __builtin_fma(y, e, y);
}
__device__ __forceinline__ float fast_rcp(float a) { return __builtin_amdgcn_rcpf(a); }

// 1/sqrt(x) for x > 0: y <- y (3/2 - x/2 y^2), twice.
__device__ __forceinline__ double fast_rsq(double x)
{
    double y = __builtin_amdgcn_rsq(x);
    const double h = 0.5 * x;
    y = y * __builtin_fma(-h * y, y, 1.5);
    return y * __builtin_fma(-h * y, y, 1.5);
}
__device__ __forceinline__ float fast_rsq(float x) { return __builtin_amdgcn_rsqf(x); }

// sqrt(x) for x >= 0 (exactly 0 at 0).
template <typename R>
__device__ __forceinline__ R fast_sqrt(R x)
{
    return x > R(0) ? x * fast_rsq(x) : R(0);
}

// M4 spline shape w(q) and slope w'(q).
// (2 - q) is clamped at 0, so the outer piece is zero beyond the support and
// one select suffices.
template <typename R>
__device__ __forceinline__ R m4_w(R q)
{
    const R one = R(1);
    const R t = fmax(R(2) - q, R(0));
    const R inner = one + q * q * (R(-1.5) + R(0.75) * q);
    const R outer = R(0.25) * t * t * t;
    return q < one ? inner : outer;
}

template <typename R>
__device__ __forceinline__ R m4_dw(R q)
{
    const R one = R(1);
    const R t = fmax(R(2) - q, R(0));
    const R inner = q * (R(-3) + R(2.25) * q);
    const R outer = R(-0.75) * t * t;
    return q < one ? inner : outer;
}

// The other kernels of the interchangeable set, as shapes w(q) and dw/dq
// with W = sigma w(q) / h^3 (sigma passed in): Wendland C2,
// w = (1 - q/2)^4 (1 + 2q), and the sinc family, w = S(pi q / 2)^n with
// S(x) = sin(x)/x. Both vanish for q >= 2 and have w(0) = 1, like M4.
enum { KF_M4 = 0, KF_WENDLAND = 1, KF_SINC = 2 };

__device__ __forceinline__ void sin_cos(double x, double *s, double *c) { sincos(x, s, c); }
__device__ __forceinline__ void sin_cos(float x, float *s, float *c) { sincosf(x, s, c); }

template <int KF, typename R>
__device__ __forceinline__ R shape_w(R q, int n)
{
    if constexpr (KF == KF_M4) {
        return m4_w(q);
    } else if constexpr (KF == KF_WENDLAND) {
        const R t = fmax(R(1) - R(0.5) * q, R(0));
        const R t2 = t * t;
        return t2 * t2 * fma_r(R(2), q, R(1));
    } else {
        if (!(q < R(2))) return R(0);
        const R x = R(1.5707963267948966) * q;
        R sx;
        if (x < R(1e-4)) {
            sx = R(1) - x * x * R(1.0 / 6.0);
        } else {
            sx = sin(x) / x;
        }
        R pw = sx;
        for (int k = 1; k < n; ++k) pw *= sx;
        return pw;
    }
}

template <int KF, typename R>
__device__ __forceinline__ R shape_dw(R q, int n)
{
    if constexpr (KF == KF_M4) {
        return m4_dw(q);
    } else if constexpr (KF == KF_WENDLAND) {
        const R t = fmax(R(1) - R(0.5) * q, R(0));
        return R(-5) * q * (t * t * t);
    } else {
        if (!(q < R(2))) return R(0);
        const R x = R(1.5707963267948966) * q;
        R sx, dsx;
        // (x cos x - sin x) / x^2 cancels for small x: FP32 takes its series
        // up to x^7 below x = 0.6 (truncation below 1e-8 relative there)
        const R small = sizeof(R) == 4 ? R(0.6) : R(1e-4);
        if (x < small) {
            const R x2 = x * x;
            sx = R(1) - x2 * (R(1.0 / 6.0) - x2 * (R(1.0 / 120.0) - x2 * R(1.0 / 5040.0)));
            dsx = -x * (R(1.0 / 3.0) - x2 * (R(1.0 / 30.0) - x2 * (R(1.0 / 840.0) -
                                                                    x2 * R(1.0 / 45360.0))));
        } else {
            R sn, cs;
            sin_cos(x, &sn, &cs);
            sx = sn / x;
            dsx = (x * cs - sn) / (x * x);
        }
        R pw = R(1);
        for (int k = 1; k < n; ++k) pw *= sx;  // S^(n-1)
        return R(n) * pw * dsx * R(1.5707963267948966);
    }
}

// 16 bytes at byte c of record j of an array of Size-byte records. Arrays
// below 4 GiB use a 32-bit offset from the uniform base (the load then takes
// the base from SGPRs and needs no 64-bit address arithmetic).
template <bool Big, int Size>
__device__ __forceinline__ double2 rec_chunk(const char *__restrict__ base, int j, uint32_t c)
{
    if constexpr (Big)
        return *reinterpret_cast<const double2 *>(base + (int64_t)j * Size + c);
    else
        return *reinterpret_cast<const double2 *>(base + ((uint32_t)j * (uint32_t)Size + c));
}

// ---------------------------------------------------------------------------
// Order the compiler's LDS accesses around the cooperative loads (LDS
// operations of one wave complete in order).
__device__ __forceinline__ void wave_lds_fence()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ double4 lds_load4(const char *p)
{
    return *reinterpret_cast<const double4 *>(p);
}

// ---------------------------------------------------------------------------
// Summation density: rho_i = (m_i + sum_j m_j w(r_ij / h_i)) / (pi h_i^3).
// Records: DensRec {x, y, z, m}, 32 B; two lanes fetch one record.
constexpr int kDensStride = 48;  // LDS bytes per record: 32 + 16 padding

// Minimum-image parameters of the wave's run. Single run: the kernel's
// grid. Ensemble: the run of the wave's particles (the waves are cut per
// run), read once into wave-uniform registers.
struct Img {
    bool per[3];
    double len[3], half[3];
};

__device__ __forceinline__ double uniform_f64(double v)
{
    const uint64_t u = (uint64_t)__double_as_longlong(v);
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)u);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(u >> 32));
    return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}

// Run slot of a wave's particles (lane 0's: every lane of a wave belongs to
// the same run).
__device__ __forceinline__ int run_slot(const BatchDev &b, int64_t ii)
{
    return __builtin_amdgcn_readfirstlane(b.slot[ii]);
}

// First particle of the calling lane and end of its wave's particles. One
// run: blocks of kThreads consecutive particles (wave w of block `tile`
// takes its 64). Ensemble: `tile` is the wave's 64-particle tile of one run.
template <bool Multi>
__device__ __forceinline__ void lane_span(int64_t tile, int64_t n, const BatchDev &b,
                                          int64_t &i, int64_t &end)
{
    if constexpr (Multi) {
        int64_t t0;
        tile_span<true>(tile, n, b, t0, end);
        i = t0 + (threadIdx.x & 63);
    } else {
        i = tile * kThreads + threadIdx.x;
        end = n;
    }
}

template <bool Multi>
__device__ __forceinline__ Img lane_img(const Grid &g, const BatchDev &b, int64_t ii)
{
    Img m;
    if constexpr (Multi) {
        const Grid &rg = b.runs[run_slot(b, ii)].grid;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            m.per[a] = __builtin_amdgcn_readfirstlane(rg.periodic[a]) != 0;
            m.len[a] = uniform_f64(rg.len[a]);
            m.half[a] = uniform_f64(rg.half[a]);
        }
    } else {
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            m.per[a] = g.periodic[a] != 0;
            m.len[a] = g.len[a];
            m.half[a] = g.half[a];
        }
    }
    return m;
}

// Per >= 0: the periodic axes are known at compile time (bit a set for a
// periodic axis a), so the other axes carry no image code; Per = -1: decided
// at run time from m.
template <int Per>
__device__ __forceinline__ double img(double d, const Img &m, int a)
{
    if constexpr (Per >= 0)
        return ((Per >> a) & 1) ? min_image(d, 1, m.len[a], m.half[a]) : d;
    else
        return min_image(d, m.per[a], m.len[a], m.half[a]);
}

// Compile-time periodic mask for a single run's grid: the common cases get
// their own kernels, any other mix is decided at run time.
inline int per_mask(const Grid &g)
{
    const int m = (g.periodic[0] ? 1 : 0) | (g.periodic[1] ? 2 : 0) | (g.periodic[2] ? 4 : 0);
    return (m == 0 || m == 4 || m == 7) ? m : -1;
}

template <bool F32, bool Multi, bool Big, int Per, int KF>
__device__ __forceinline__ void density_tile(int64_t tile, int64_t n, int64_t ld,
                                             const DensRec *__restrict__ drec,
                                             const double *__restrict__ h,
                                             const int32_t *__restrict__ count,
                                             const int32_t *__restrict__ idx, int max_nb,
                                             const Grid &g, double *__restrict__ rho,
                                             const BatchDev &b, char *buf, double sigma,
                                             int sinc_n, const StepMask &mask)
{
    using R = typename std::conditional<F32, float, double>::type;
    const int lane = threadIdx.x & 63;
    int64_t i, iend;
    lane_span<Multi>(tile, n, b, i, iend);
    const bool active = i < iend;
    const int64_t ii = active ? i : (Multi ? i - lane : 0);
    // individual time steps: only particles whose step closes are evaluated
    const bool closes = Multi || step_closes(mask, ii);
    if (!Multi && mask.bin && __ballot(active && closes) == 0ull) return;
    const Img im = lane_img<Multi>(g, b, ii);
    const DensRec me = drec[ii];
    const R inv_h = R(1) / (R)h[ii];
    R sum = (R)me.m;  // w(0) = 1
    const int cnt = active ? min(count[ii], max_nb) : 0;
    int maxc = cnt;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) maxc = max(maxc, __shfl_xor(maxc, o, 64));
    const int s = lane & 1;
    const char *src_base = reinterpret_cast<const char *>(drec);
    const uint32_t chunk = 16u * (uint32_t)s;
    char *dst_own = buf + lane * kDensStride;
    char *dst_a = buf + (lane & ~1) * kDensStride + 16 * s;
    // Lanes 2g and 2g+1 fetch chunk s of the records of both.
    auto fetch = [&](int jk, double2 &a, double2 &b) {
        const int jp = __shfl_xor(jk, 1, 64);
        const int j0 = s == 0 ? jk : jp, j1 = s == 0 ? jp : jk;
        a = rec_chunk<Big, (int)sizeof(DensRec)>(src_base, j0, chunk);
        b = rec_chunk<Big, (int)sizeof(DensRec)>(src_base, j1, chunk);
    };
    // Two steps in flight: the records of step k + 2 are requested while
    // step k is computed, alternating between two register sets (the loop
    // runs two steps per pass, so no set is copied and every wait counts only
    // the requests issued before the one it needs). Indices are read two
    // steps before their records; steps past a lane's count fetch its own
    // record (in bounds, unused).
    // Index of step k: the list row min(k, max_nb - 1) is read whatever the
    // lane's count (rows at or past the count hold stale values); the value
    // is clamped to a valid record only when it is used, so that the read
    // itself carries no condition.
    const int krow = max_nb - 1;
    // The list is read once per call: non-temporal loads keep its 4 B per
    // pair from evicting the neighbour records from L2.
    auto jat = [&](int k) -> int {
        return __builtin_nontemporal_load(&idx[(int64_t)min(k, krow) * ld + ii]);
    };
    const uint32_t jmax = (uint32_t)(n - 1);
    auto jfix = [&](int j) -> int { return (int)min((uint32_t)j, jmax); };
    auto step = [&](int k) {
        const double2 lo = *reinterpret_cast<const double2 *>(dst_own);
        const double2 hi = *reinterpret_cast<const double2 *>(dst_own + 16);
        if (k < cnt) {
            const R dx = (R)img<Per>(me.x - lo.x, im, 0);
            const R dy = (R)img<Per>(me.y - lo.y, im, 1);
            const R dz = (R)img<Per>(me.z - hi.x, im, 2);
            const R r = fast_sqrt(fma_r(dz, dz, fma_r(dy, dy, dx * dx)));
            sum = fma_r((R)hi.y, shape_w<KF>(r * inv_h, sinc_n), sum);
        }
    };
    double2 a0, a1, b0, b1;
    // (issued in the loop's order: the first set is waited for first)
    const int j0 = jat(0), j1 = jat(1);
    fetch(jfix(j0), a0, a1);
    int ja = jat(2);
    __builtin_amdgcn_sched_barrier(0);
    fetch(jfix(j1), b0, b1);
    int jb = jat(3);
    __builtin_amdgcn_sched_barrier(0);
    // The requests are unconditional (the last pass fetches records that
    // are never used), so the loop body is straight-line code and each wait
    // names an exact count.
    for (int k = 0; k < maxc; k += 2) {
        wave_lds_fence();
        *reinterpret_cast<double2 *>(dst_a) = a0;
        *reinterpret_cast<double2 *>(dst_a + kDensStride) = a1;
        wave_lds_fence();
        fetch(jfix(ja), a0, a1);
        ja = jat(k + 4);
        step(k);
        wave_lds_fence();
        *reinterpret_cast<double2 *>(dst_a) = b0;
        *reinterpret_cast<double2 *>(dst_a + kDensStride) = b1;
        wave_lds_fence();
        fetch(jfix(jb), b0, b1);
        jb = jat(k + 5);
        step(k + 1);
    }
    const R sg = KF == KF_M4 ? (R)kInvPi : (R)sigma;
    if (active && closes) rho[i] = (double)(sum * (sg * inv_h * inv_h * inv_h));
}

// Ensemble: the calling wave's 64-particle tile (-1: none). The grid covers
// the capacity's tiles (one per wave); the blocks a step uses are spread
// over the XCDs.
__device__ __forceinline__ int64_t ens_wave_tile(const BatchDev &b)
{
    const int64_t ntile = b.hdr->ntile;
    const int64_t bt = xcd_used_block((ntile + kThreads / 64 - 1) / (kThreads / 64));
    if (bt < 0) return -1;
    const int64_t t = bt * (kThreads / 64) + (threadIdx.x >> 6);
    return t < ntile ? t : -1;
}

template <bool F32, bool Multi, bool Big, int Per, int KF>
__global__ void __launch_bounds__(kThreads)
density_kernel(int64_t n, int64_t ld, const DensRec *__restrict__ drec,
               const double *__restrict__ h, const int32_t *__restrict__ count,
               const int32_t *__restrict__ idx, int max_nb, Grid g, double *__restrict__ rho,
               BatchDev b, double sigma, int sinc_n, StepMask mask)
{
    __shared__ __attribute__((aligned(16))) char lds[kThreads / 64][64 * kDensStride];
    char *buf = lds[threadIdx.x >> 6];
    if constexpr (Multi) {
        // one run-aligned tile per wave over a capacity-sized grid (a loop
        // over tiles keeps the tile body's loop-invariant values live)
        const int64_t t = ens_wave_tile(b);
        if (t >= 0)
            density_tile<F32, true, Big, -1, KF>(t, b.hdr->n_out, ld, drec, h, count, idx,
                                                 max_nb, g, rho,
                                                 b, buf, sigma, sinc_n, mask);
    } else {
        density_tile<F32, false, Big, Per, KF>(xcd_cu_block(), n, ld, drec, h, count, idx,
                                               max_nb, g, rho, b, buf, sigma, sinc_n, mask);
    }
}

// Density records {x, y, z, m}.
__global__ void __launch_bounds__(256)
pack_dens_kernel(int64_t n, const int64_t *n_dev, const double *__restrict__ x,
                 const double *__restrict__ y, const double *__restrict__ z,
                 const double *__restrict__ m, DensRec *__restrict__ out)
{
    if (n_dev) n = *n_dev;
    const int64_t step = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += step)
        out[i] = DensRec{x[i], y[i], z[i], m[i]};
}

// Generalised volume elements: weights X_i = (m_i / rho_i)^e from a density
// estimate, and the density from the weighted sum k_i (which the density
// kernel leaves in rho when its records carry X instead of m):
// rho_i = k_i (m_i / X_i).
__global__ void __launch_bounds__(256)
volume_weights_kernel(int64_t n, const double *__restrict__ m, const double *__restrict__ rho,
                      double e, double *__restrict__ xw)
{
    const int64_t step = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += step)
        xw[i] = pow(m[i] / rho[i], e);
}

__global__ void __launch_bounds__(256)
gve_density_kernel(int64_t n, const double *__restrict__ m, const double *__restrict__ xw,
                   double *__restrict__ rho, StepMask mask)
{
    const int64_t step = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += step)
        if (step_closes(mask, i)) rho[i] = rho[i] * (m[i] / xw[i]);
}

// ---------------------------------------------------------------------------
// EOS.
__global__ void __launch_bounds__(256)
eos_kernel(int64_t n, int eos, double rho0, double c0, double gamma_tait,
           double gamma_gas, const double *__restrict__ rho, const double *__restrict__ u,
           const double *__restrict__ rho_ref, const double *__restrict__ p_bg,
           double *__restrict__ p, double *__restrict__ c, double *__restrict__ pr2,
           StepMask mask)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n || !step_closes(mask, i)) return;
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
    p[i] = P;
    c[i] = C;
    pr2[i] = P / (r * r);
}

// ---------------------------------------------------------------------------
// Momentum and energy with Monaghan artificial viscosity.
// Records: PairRec (96 B used of 128), PairRec32 (80 B): the used 16-byte
// chunks of a step's 64 records are fetched by the wave in sequence, 64 per
// load instruction, and handed to their owners through LDS.
constexpr int kMomStride = 112;  // LDS bytes per record: 96 + 16 padding

struct MomParams {
    double alpha, beta, eta2;
    double sigma;  // W(0, h) h^3 of the kernel (KF != KF_M4)
    int sinc_n;
    const double *iad_c;  // IAD matrices (IAD instances), 6 per particle
    // individual time steps (bin not null): only particles of bin b with
    // ((sub + 1) mod 2^(B - b)) == 0 are evaluated and written
    const double *bin;
    int sub, B;
};

// IAD matrices (integral approach to derivatives, standard volume elements):
// tau_i = sum_j V_j d d^T W(r, h_i) over the lane's list, d = x_i - x_j
// (the sign cancels), c_i = tau_i^{-1} as xx xy xz yy yz zz. The inverse is
// taken only where det tau_i >= kIadCond (tr tau_i / 3)^3: for a positive
// semi-definite tau that ratio lies in [0, 1], is 1 for an isotropic
// neighbourhood and tends to 0 as the neighbours stop spanning three
// dimensions, where the inverse would be set by rounding alone. Below it
// c_i = (tr tau_i / 3)^-1 I (what the inverse is for an isotropic tau), and
// c_i = 0 without a neighbour inside 2 h_i (tr tau_i = 0).
// Records {x, y, z, V = m / rho}, one lane per particle, FP64.
constexpr double kIadCond = 1e-2;
// Near free surfaces tau_i can be close to singular, and its inverse then
// magnifies last-bit differences. So the matrix is formed with correctly
// rounded operations only (sqrt, division, no fused multiply-add), in the
// plain textbook order: r = sqrt(r^2), q = r / h, W = w(q) / (pi h h h),
// tau += (V W d_a) d_b. For the polynomial kernels (M4, Wendland C2) the
// result is then the same number as in any implementation that evaluates
// these expressions in this order.
template <int KF>
__device__ __forceinline__ double kernel_w_plain(double r, double hh, double sigma, int n)
{
    const double q = r / hh;
    if constexpr (KF == KF_M4) {
        double w = 0.0;
        if (q < 1.0) {
            w = 1.0 - 1.5 * q * q + 0.75 * q * q * q;
        } else if (q < 2.0) {
            const double t = 2.0 - q;
            w = 0.25 * t * t * t;
        }
        return w / (M_PI * hh * hh * hh);
    } else if constexpr (KF == KF_WENDLAND) {
        if (q >= 2.0) return 0.0;
        const double t = 1.0 - 0.5 * q;
        return 21.0 / (16.0 * M_PI * hh * hh * hh) * t * t * t * t * (1.0 + 2.0 * q);
    } else {
        if (q >= 2.0) return 0.0;
        const double x = 0.5 * M_PI * q;
        const double sx = x == 0.0 ? 1.0 : sin(x) / x;
        return sigma / (hh * hh * hh) * pow(sx, (double)n);
    }
}

template <int KF>
__global__ void __launch_bounds__(256)
iad_kernel(int64_t n, int64_t ld, const DensRec *__restrict__ vrec,
           const double *__restrict__ h, const int32_t *__restrict__ count,
           const int32_t *__restrict__ idx, int max_nb, Grid g, double sigma, int sinc_n,
           double *__restrict__ c6)
{
    // The records are gathered as in the density kernel: lanes 2g and 2g+1
    // fetch chunk s of the records of both and hand them over through LDS,
    // with two steps in flight (the same index reads, clamped at their use).
    __shared__ __attribute__((aligned(16))) char lds[4][64 * kDensStride];
    char *buf = lds[threadIdx.x >> 6];
    const int lane = threadIdx.x & 63;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool active = i < n;
    const int64_t ii = active ? i : 0;
    const Img im = lane_img<false>(g, BatchDev{}, ii);
    const DensRec me = vrec[ii];
    const double hh = h[ii];
    double a = 0.0, b = 0.0, c = 0.0, d = 0.0, e = 0.0, f = 0.0;
    const int cnt = active ? min(count[ii], max_nb) : 0;
    int maxc = cnt;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) maxc = max(maxc, __shfl_xor(maxc, o, 64));
    const int s = lane & 1;
    const char *src_base = reinterpret_cast<const char *>(vrec);
    const uint32_t chunk = 16u * (uint32_t)s;
    char *dst_own = buf + lane * kDensStride;
    char *dst_a = buf + (lane & ~1) * kDensStride + 16 * s;
    auto fetch = [&](int jk, double2 &x0, double2 &x1) {
        const int jp = __shfl_xor(jk, 1, 64);
        const int j0 = s == 0 ? jk : jp, j1 = s == 0 ? jp : jk;
        x0 = rec_chunk<true, (int)sizeof(DensRec)>(src_base, j0, chunk);
        x1 = rec_chunk<true, (int)sizeof(DensRec)>(src_base, j1, chunk);
    };
    const int krow = max_nb - 1;
    auto jat = [&](int k) -> int {
        return __builtin_nontemporal_load(&idx[(int64_t)min(k, krow) * ld + ii]);
    };
    const uint32_t jmax = (uint32_t)(n - 1);
    auto jfix = [&](int j) -> int { return (int)min((uint32_t)j, jmax); };
    auto step = [&](int k) {
        const double2 lo = *reinterpret_cast<const double2 *>(dst_own);       // x y
        const double2 hi = *reinterpret_cast<const double2 *>(dst_own + 16);  // z V
        if (k < cnt) {
            const double dx = img<-1>(me.x - lo.x, im, 0);
            const double dy = img<-1>(me.y - lo.y, im, 1);
            const double dz = img<-1>(me.z - hi.x, im, 2);
            const double r = sqrt(__builtin_fma(dz, dz, __builtin_fma(dy, dy, dx * dx)));
            const double vw = hi.y * kernel_w_plain<KF>(r, hh, sigma, sinc_n);
            a += vw * dx * dx;
            b += vw * dx * dy;
            c += vw * dx * dz;
            d += vw * dy * dy;
            e += vw * dy * dz;
            f += vw * dz * dz;
        }
    };
    double2 a0, a1, b0, b1;
    // (issued in the loop's order: the first set is waited for first)
    const int j0 = jat(0), j1 = jat(1);
    fetch(jfix(j0), a0, a1);
    int ja = jat(2);
    __builtin_amdgcn_sched_barrier(0);
    fetch(jfix(j1), b0, b1);
    int jb = jat(3);
    __builtin_amdgcn_sched_barrier(0);
    for (int k = 0; k < maxc; k += 2) {
        wave_lds_fence();
        *reinterpret_cast<double2 *>(dst_a) = a0;
        *reinterpret_cast<double2 *>(dst_a + kDensStride) = a1;
        wave_lds_fence();
        fetch(jfix(ja), a0, a1);
        ja = jat(k + 4);
        step(k);
        wave_lds_fence();
        *reinterpret_cast<double2 *>(dst_a) = b0;
        *reinterpret_cast<double2 *>(dst_a + kDensStride) = b1;
        wave_lds_fence();
        fetch(jfix(jb), b0, b1);
        jb = jat(k + 5);
        step(k + 1);
    }
    if (!active) return;
    const double ca = d * f - e * e, cb = c * e - b * f, cc = b * e - c * d;
    const double det = a * ca + b * cb + c * cc;
    const double tr = a + d + f;
    double *o6 = c6 + 6 * i;
    for (int t = 0; t < 6; ++t) o6[t] = 0.0;
    // no neighbour inside 2 h_i: c_i = 0
    if (!(tr > 0.0) || !isfinite(tr) || !isfinite(det)) return;
    // neighbours that do not span three dimensions (det below kIadCond of
    // (tr / 3)^3): the isotropic form (tr / 3)^-1 I
    const double tm = tr / 3.0;
    if (!(det >= kIadCond * (tm * tm * tm))) {
        o6[0] = o6[3] = o6[5] = 3.0 / tr;
        return;
    }
    o6[0] = ca / det;
    o6[1] = cb / det;
    o6[2] = cc / det;
    o6[3] = (a * f - c * c) / det;
    o6[4] = (b * c - a * e) / det;
    o6[5] = (a * d - b * b) / det;
}

// Volume records {x, y, z, m / rho} for the IAD pass.
__global__ void __launch_bounds__(256)
pack_vol_kernel(int64_t n, const double *__restrict__ x, const double *__restrict__ y,
                const double *__restrict__ z, const double *__restrict__ m,
                const double *__restrict__ rho, DensRec *__restrict__ out)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = DensRec{x[i], y[i], z[i], m[i] / rho[i]};
}

// UH: every particle has the same h. Then h_i = h_j bit for bit, the two
// kernel slopes of the mean gradient are the same number t, and
// 0.5 (t + t) = t exactly, so one evaluation gives the general form's result.
// IAD: the pair terms use Abar_ij = -(W(r, h_i) c_i + W(r, h_j) c_j) r_ij / 2
// in place of the mean kernel gradient; c_j of the next step is loaded with
// the records.
template <bool F32, bool Multi, bool Big, int Per, bool UH, int KF, bool IAD = false,
          bool GVE = false>
__device__ __forceinline__ void momentum_tile(
    int64_t tile, int64_t n, int64_t ld, const PairRec *__restrict__ rec,
    const int32_t *__restrict__ count, const int32_t *__restrict__ idx, int max_nb,
    const Grid &g, const MomParams &prm0, double *__restrict__ ax, double *__restrict__ ay,
    double *__restrict__ az, double *__restrict__ dudt, double *__restrict__ mumax,
    const BatchDev &b, char *buf)
{
    using R = typename std::conditional<F32, float, double>::type;
    const int lane = threadIdx.x & 63;
    int64_t i, iend;
    lane_span<Multi>(tile, n, b, i, iend);
    const bool active = i < iend;
    const int64_t ii = active ? i : (Multi ? i - lane : 0);
    const Img im = lane_img<Multi>(g, b, ii);
    MomParams prm = prm0;
    if constexpr (Multi) {
        const RunDev &r = b.runs[run_slot(b, ii)];
        prm = MomParams{uniform_f64(r.alpha), uniform_f64(r.beta), uniform_f64(r.eta2), 0.0, 0,
                        nullptr, nullptr, 0, 0};
    }
    // individual time steps: lanes whose particle's step does not close now
    // write nothing; a wave without any such lane has nothing to do
    bool closes = true;
    if (!Multi && prm.bin) {
        const int b = (int)prm.bin[ii];
        closes = (((prm.sub + 1) & ((1 << (prm.B - b)) - 1)) == 0);
        if (__ballot(active && closes) == 0ull) return;
    }
    // the FP32-pair form with kernel derivatives reads PairRec32 records
    // (FP32 copies of the fields after the position and velocity)
    constexpr bool R32 = F32 && !IAD;
    constexpr int kRecBytes = R32 ? (int)sizeof(PairRec32) : (int)sizeof(PairRec);
    const PairRec *mp = rec + ii;
    const PairRec32 *mp32 = reinterpret_cast<const PairRec32 *>(rec) + ii;
    double mex, mey, mez, mevx, mevy, mevz;
    R hi, inv_hi, rhoi, ci, pi, xim, qim;
    // generalised volume elements: X_i / m_i and Q_i / m_i of the own record
    // (X and Q = m^2 P / (rho^2 X))
    if constexpr (R32) {
        mex = mp32->x; mey = mp32->y; mez = mp32->z;
        mevx = mp32->vx; mevy = mp32->vy; mevz = mp32->vz;
        hi = mp32->h; inv_hi = mp32->inv_h; rhoi = mp32->rho; ci = mp32->c; pi = mp32->pr2;
        xim = GVE ? mp32->X / mp32->m : R(0);
        qim = GVE ? mp32->Q / mp32->m : R(0);
    } else {
        mex = mp->x; mey = mp->y; mez = mp->z;
        mevx = mp->vx; mevy = mp->vy; mevz = mp->vz;
        hi = (R)mp->h; inv_hi = (R)mp->inv_h; rhoi = (R)mp->rho; ci = (R)mp->c;
        pi = (R)mp->pr2;
        xim = GVE ? (R)(mp->pad[0] / mp->m) : R(0);
        qim = GVE ? (R)(mp->pad[1] / mp->m) : R(0);
    }
    const R sg = KF == KF_M4 ? (R)kInvPi : (R)prm.sigma;
    const int sn = prm.sinc_n;
    const R fi = sg * (inv_hi * inv_hi) * (inv_hi * inv_hi);
    const R alpha = (R)prm.alpha, beta = (R)prm.beta, eta2 = (R)prm.eta2;
    R sx = 0, sy = 0, sz = 0, su = 0, mum = 0;
    // IAD: the lane's own matrix, and the next neighbour's. The IAD gradient
    // Abar_ij is formed in FP64 in both forms and rounded to FP32 like r_ij
    // itself: c_i scales W(r, h_i) up to an O(1) weight (c_i ~ 1 / sum of
    // V W r^2), so near the edge of the support, where an FP32 W(r, h) =
    // (2 - q)^3 / 4 ... loses its relative accuracy to cancellation, an FP32
    // gradient would be off by far more than the FP32 rounding of its size.
    double cix = 0, ciy = 0, ciz = 0, ciyy = 0, ciyz = 0, cizz = 0;
    const double inv_hid = IAD ? mp->inv_h : 0.0;  // (IAD: PairRec records)
    if constexpr (IAD) {
        const double *cp = prm.iad_c + 6 * ii;
        cix = cp[0]; ciy = cp[1]; ciz = cp[2];
        ciyy = cp[3]; ciyz = cp[4]; cizz = cp[5];
    }
    const int cnt = active ? min(count[ii], max_nb) : 0;
    int maxc = cnt;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) maxc = max(maxc, __shfl_xor(maxc, o, 64));
    // The 64 records of a step are kChunks x 64 16-byte chunks: load
    // instruction t gives lane L the chunk (64 t + L) of that sequence, chunk
    // c of record r with 64 t + L = kChunks r + c, so every lane of every
    // instruction loads a chunk that is used.
    constexpr int kChunks = R32 ? 5 : (GVE ? 7 : 6);
    int rsrc[kChunks];
#pragma unroll
    for (int t = 0; t < kChunks; ++t) rsrc[t] = (64 * t + lane) / kChunks;
    auto chunk_of = [&](int t) -> uint32_t {
        return 16u * (uint32_t)(64 * t + lane - kChunks * rsrc[t]);
    };
    const char *src_base = reinterpret_cast<const char *>(rec);
    const char *own = buf + lane * kMomStride;
    // Two steps in flight: the records of step k + 2 are requested while
    // step k is computed, alternating between two register sets (the loop
    // runs two steps per pass, so no set is copied and every wait counts only
    // the requests issued before the one it needs). Indices are read two
    // steps before their records: the list row min(k, max_nb - 1) whatever
    // the lane's count (rows at or past the count hold stale values), the
    // value clamped to a valid record only when it is used, so that no read
    // carries a condition. Records fetched for steps past a lane's count are
    // never used.
    const int krow = max_nb - 1;
    auto jat = [&](int k) -> int {
        return __builtin_nontemporal_load(&idx[(int64_t)min(k, krow) * ld + ii]);
    };
    const uint32_t jmax = (uint32_t)(n - 1);
    auto jfix = [&](int j) -> int { return (int)min((uint32_t)j, jmax); };
    struct RecSet {
        double2 c[kChunks];
        double2 e[3] = {};  // IAD: c_j of the set's step (zero otherwise)
    };
    auto fetch_set = [&](int jk, RecSet &S) {
#pragma unroll
        for (int t = 0; t < kChunks; ++t)
            S.c[t] = rec_chunk<Big, kRecBytes>(src_base, __shfl(jk, rsrc[t], 64), chunk_of(t));
        if constexpr (IAD) {
            const double2 *cp = reinterpret_cast<const double2 *>(prm.iad_c + 6 * (int64_t)jk);
            S.e[0] = cp[0];
            S.e[1] = cp[1];
            S.e[2] = cp[2];
        }
    };
    auto put_set = [&](const RecSet &S) {
        wave_lds_fence();
#pragma unroll
        for (int t = 0; t < kChunks; ++t)
            *reinterpret_cast<double2 *>(buf + rsrc[t] * kMomStride + chunk_of(t)) = S.c[t];
        wave_lds_fence();
    };
    auto step = [&](int k, const double2 f0, const double2 f1, const double2 f2) {
        const double2 q0 = *reinterpret_cast<const double2 *>(own);       // x y
        const double2 q1 = *reinterpret_cast<const double2 *>(own + 16);  // z vx
        const double2 q2 = *reinterpret_cast<const double2 *>(own + 32);  // vy vz
        // neighbour fields: h, 1/h, m, rho, c, P/rho^2, X, Q
        R hj_, inv_hj_, mj_, rhoj_, cj_, prj_, Xj_ = R(0), Qj_ = R(0);
        double inv_hjd = 0.0;  // (IAD)
        if constexpr (R32) {
            const float4 a = *reinterpret_cast<const float4 *>(own + 48);  // h 1/h m rho
            const float4 b = *reinterpret_cast<const float4 *>(own + 64);  // c pr2 X Q
            hj_ = a.x; inv_hj_ = a.y; mj_ = a.z; rhoj_ = a.w;
            cj_ = b.x; prj_ = b.y;
            if constexpr (GVE) { Xj_ = b.z; Qj_ = b.w; }
        } else {
            const double2 q3 = *reinterpret_cast<const double2 *>(own + 48);  // h inv_h
            const double2 q4 = *reinterpret_cast<const double2 *>(own + 64);  // m rho
            const double2 q5 = *reinterpret_cast<const double2 *>(own + 80);  // c pr2
            hj_ = (R)q3.x; inv_hj_ = (R)q3.y; mj_ = (R)q4.x; rhoj_ = (R)q4.y;
            cj_ = (R)q5.x; prj_ = (R)q5.y;
            inv_hjd = q3.y;
            if constexpr (GVE) {
                const double2 q6 = *reinterpret_cast<const double2 *>(own + 96);  // X Q
                Xj_ = (R)q6.x; Qj_ = (R)q6.y;
            }
        }
        if (k < cnt) {
            const double dxd = img<Per>(mex - q0.x, im, 0);
            const double dyd = img<Per>(mey - q0.y, im, 1);
            const double dzd = img<Per>(mez - q1.x, im, 2);
            const R dx = (R)dxd, dy = (R)dyd, dz = (R)dzd;
            const R r2 = fma_r(dz, dz, fma_r(dy, dy, dx * dx));
            // 1/r (0 for coincident particles, whose gradient term vanishes)
            const R rinv = r2 > R(0) ? fast_rsq(r2) : R(0);
            const R r = r2 * rinv;
            R dwbar, hbar;
            R gx = 0, gy = 0, gz = 0;  // IAD: Abar_ij
            if constexpr (IAD) {
                const double r2d = fma_r(dzd, dzd, fma_r(dyd, dyd, dxd * dxd));
                const double rd = r2d * (r2d > 0.0 ? fast_rsq(r2d) : 0.0);
                const double sgd = KF == KF_M4 ? kInvPi : prm.sigma;
                const double wi =
                    sgd * (inv_hid * inv_hid * inv_hid) * shape_w<KF>(rd * inv_hid, sn);
                const double wj =
                    sgd * (inv_hjd * inv_hjd * inv_hjd) * shape_w<KF>(rd * inv_hjd, sn);
                const double cjx = f0.x, cjy = f0.y, cjz = f1.x, cjyy = f1.y, cjyz = f2.x,
                             cjzz = f2.y;
                const double tix = fma_r(ciz, dzd, fma_r(ciy, dyd, cix * dxd));
                const double tiy = fma_r(ciyz, dzd, fma_r(ciyy, dyd, ciy * dxd));
                const double tiz = fma_r(cizz, dzd, fma_r(ciyz, dyd, ciz * dxd));
                const double tjx = fma_r(cjz, dzd, fma_r(cjy, dyd, cjx * dxd));
                const double tjy = fma_r(cjyz, dzd, fma_r(cjyy, dyd, cjy * dxd));
                const double tjz = fma_r(cjzz, dzd, fma_r(cjyz, dyd, cjz * dxd));
                gx = (R)(-0.5 * fma_r(wj, tjx, wi * tix));
                gy = (R)(-0.5 * fma_r(wj, tjy, wi * tiy));
                gz = (R)(-0.5 * fma_r(wj, tjz, wi * tiz));
                dwbar = R(0);
                hbar = R(0.5) * (hi + hj_);
            } else if constexpr (UH) {
                dwbar = fi * shape_dw<KF>(r * inv_hi, sn);
                hbar = hi;
            } else {
                const R hj = hj_, inv_hj = inv_hj_;
                const R fj = sg * (inv_hj * inv_hj) * (inv_hj * inv_hj);
                dwbar = R(0.5) * (fi * shape_dw<KF>(r * inv_hi, sn) +
                                  fj * shape_dw<KF>(r * inv_hj, sn));
                hbar = R(0.5) * (hi + hj);
            }
            const R F = dwbar * rinv;
            const R wx = (R)(mevx - q1.y), wy = (R)(mevy - q2.x), wz = (R)(mevz - q2.y);
            const R vdotr = fma_r(wz, dz, fma_r(wy, dy, wx * dx));
            const R cbar = R(0.5) * (ci + cj_);
            const R rhobar = R(0.5) * (rhoi + rhoj_);
            // one reciprocal for both denominators: inv = 1 / (den rhobar)
            const R den = fma_r(eta2 * hbar, hbar, r2);
            const R inv = fast_rcp(den * rhobar);
            const R mu = vdotr < R(0) ? hbar * vdotr * (rhobar * inv) : R(0);
            const R Pi = mu * (beta * mu - alpha * cbar) * (den * inv);
            // pair weight: m_j (P_i/rho_i^2 + P_j/rho_j^2 + Pi), or with
            // generalised volume elements X_j Q_i/m_i + Q_j X_i/m_i + m_j Pi
            R wgt;
            if constexpr (GVE)
                wgt = fma_r(Xj_, qim, fma_r(Qj_, xim, mj_ * Pi));
            else
                wgt = mj_ * (pi + prj_ + Pi);
            if constexpr (IAD) {
                const R mGs = wgt;
                sx = fma_r(-mGs, gx, sx);
                sy = fma_r(-mGs, gy, sy);
                sz = fma_r(-mGs, gz, sz);
                su = fma_r(mGs, fma_r(wz, gz, fma_r(wy, gy, wx * gx)), su);
            } else {
                const R mG = wgt * F;
                sx = fma_r(-mG, dx, sx);
                sy = fma_r(-mG, dy, sy);
                sz = fma_r(-mG, dz, sz);
                su = fma_r(mG, vdotr, su);
            }
            mum = fmax(mum, fabs(mu));
        }
    };
    RecSet A, B;
    // (issued in the loop's order: the first set is waited for first)
    const int j0 = jat(0), j1 = jat(1);
    fetch_set(jfix(j0), A);
    int ja = jat(2);
    __builtin_amdgcn_sched_barrier(0);
    fetch_set(jfix(j1), B);
    int jb = jat(3);
    __builtin_amdgcn_sched_barrier(0);
    for (int k = 0; k < maxc; k += 2) {
        put_set(A);
        double2 f0 = A.e[0], f1 = A.e[1], f2 = A.e[2];
        fetch_set(jfix(ja), A);
        ja = jat(k + 4);
        step(k, f0, f1, f2);
        put_set(B);
        f0 = B.e[0];
        f1 = B.e[1];
        f2 = B.e[2];
        fetch_set(jfix(jb), B);
        jb = jat(k + 5);
        step(k + 1, f0, f1, f2);
    }
    if (active && closes) {
        ax[i] = (double)sx;
        ay[i] = (double)sy;
        az[i] = (double)sz;
        dudt[i] = 0.5 * (double)su;
        mumax[i] = (double)mum;
    }
}

template <bool F32, bool Multi, bool Big, int Per, int KF, bool IAD = false, bool GVE = false>
__global__ void __launch_bounds__(kThreads)
momentum_kernel(int64_t n, int64_t ld, const PairRec *__restrict__ rec,
                const int32_t *__restrict__ count, const int32_t *__restrict__ idx, int max_nb,
                Grid g, MomParams prm, double *__restrict__ ax, double *__restrict__ ay,
                double *__restrict__ az, double *__restrict__ dudt, double *__restrict__ mumax,
                BatchDev b, const uint32_t *__restrict__ hflag)
{
    __shared__ __attribute__((aligned(16))) char lds[kThreads / 64][64 * kMomStride];
    char *buf = lds[threadIdx.x >> 6];
    if constexpr (Multi) {
        const int64_t t = ens_wave_tile(b);
        if (t >= 0)
            momentum_tile<F32, true, Big, -1, false, KF>(t, b.hdr->n_out, ld, rec, count, idx,
                                                         max_nb, g,
                                                         prm, ax, ay, az, dudt, mumax, b, buf);
    } else if constexpr (IAD || GVE) {
        momentum_tile<F32, false, Big, Per, false, KF, IAD, GVE>(xcd_block(), n, ld, rec,
                                                                 count, idx, max_nb, g, prm, ax,
                                                                 ay, az, dudt, mumax, b, buf);
    } else if (hflag[0] == 0u) {
        // uniform h (flag of the last cell build)
        momentum_tile<F32, false, Big, Per, true, KF>(xcd_block(), n, ld, rec, count, idx,
                                                      max_nb, g, prm, ax, ay, az, dudt, mumax,
                                                      b, buf);
    } else {
        momentum_tile<F32, false, Big, Per, false, KF>(xcd_block(), n, ld, rec, count, idx,
                                                       max_nb, g, prm, ax, ay, az, dudt, mumax,
                                                       b, buf);
    }
}

// Pair records {x, y, z, vx, vy, vz, h, 1/h, m, rho, c, P/rho^2}, and with
// generalised volume elements (xw not null) {X, Q = m^2 (P/rho^2) / X}.
// R32 (the FP32-pair form, kernel derivatives): PairRec32 records, the
// fields after the position and velocity rounded to FP32 (1/h from the FP64
// h, Q from the FP64 fields).
template <bool R32>
__global__ void __launch_bounds__(256)
pack_pair_kernel(int64_t n, const int64_t *n_dev, const double *__restrict__ x,
                 const double *__restrict__ y, const double *__restrict__ z,
                 const double *__restrict__ vx, const double *__restrict__ vy,
                 const double *__restrict__ vz, const double *__restrict__ h,
                 const double *__restrict__ m, const double *__restrict__ rho,
                 const double *__restrict__ c, const double *__restrict__ pr2,
                 const double *__restrict__ xw, void *__restrict__ out)
{
    // Each wave forms the records of 64 consecutive particles in LDS (one
    // per lane, stride 17 doubles), then stores them as 16-byte chunks with
    // consecutive lanes on consecutive chunks, so that every store writes
    // 1 KB of contiguous memory. Only the chunks the momentum kernel reads
    // are written: 6 (96 B), or 7 with the volume weights; 5 (80 B) for
    // PairRec32.
    constexpr int kStride = 17;
    constexpr int kRecBytes = R32 ? (int)sizeof(PairRec32) : (int)sizeof(PairRec);
    constexpr int kParts = kRecBytes / 16;  // chunks per record in memory
    __shared__ double lds[4][64 * kStride];
    if (n_dev) n = *n_dev;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    double *buf = lds[wave];
    const int nparts = R32 ? 5 : (xw ? 7 : 6);
    const int64_t wstep = (int64_t)gridDim.x * (blockDim.x >> 6) * 64;
    for (int64_t base = ((int64_t)blockIdx.x * (blockDim.x >> 6) + wave) * 64; base < n;
         base += wstep) {
        const int64_t i = base + lane;
        if (i < n) {
            const double hi = h[i];
            double *r = buf + lane * kStride;
            r[0] = x[i]; r[1] = y[i]; r[2] = z[i];
            r[3] = vx[i]; r[4] = vy[i]; r[5] = vz[i];
            const double q = xw ? m[i] * m[i] * pr2[i] / xw[i] : 0.0;
            if constexpr (R32) {
                float *f = reinterpret_cast<float *>(r + 6);
                f[0] = (float)hi; f[1] = (float)(1.0 / hi); f[2] = (float)m[i];
                f[3] = (float)rho[i]; f[4] = (float)c[i]; f[5] = (float)pr2[i];
                f[6] = xw ? (float)xw[i] : 0.0f;
                f[7] = (float)q;
            } else {
                r[6] = hi; r[7] = 1.0 / hi; r[8] = m[i];
                r[9] = rho[i]; r[10] = c[i]; r[11] = pr2[i];
                if (xw) {
                    r[12] = xw[i];
                    r[13] = q;
                }
            }
        }
        wave_lds_fence();
        char *dst = reinterpret_cast<char *>(out) + base * kRecBytes;
#pragma unroll
        for (int t = 0; t < 8; ++t) {
            const int q = t * 64 + lane;
            const int rec = q >> 3, part = q & 7;
            if (part < nparts && base + rec < n) {
                const double *src = buf + rec * kStride + 2 * part;
                *reinterpret_cast<double2 *>(dst + (int64_t)rec * kRecBytes + 16 * part) =
                    make_double2(src[0], src[1]);
            }
        }
        (void)kParts;
        wave_lds_fence();
    }
}

inline unsigned blocks_for(int64_t n, int t) { return (unsigned)((n + t - 1) / t); }

// Blocks of an ensemble gather: one wave per 64-particle tile, at most one
// partial tile per run beyond the capacity's.
inline unsigned ens_pair_blocks(int64_t cap)
{
    return blocks_for((cap + 63) / 64 + kEnsMaxSlots, kThreads / 64);
}

// Ensemble EOS: each particle with its run's constants. At a run's t = 0
// evaluation with a density reference, rho_ref := rho first (then the Tait
// ratio is exactly one, as in the single-run initial evaluation).
__global__ void __launch_bounds__(256)
eos_batch_kernel(BatchDev b, const double *__restrict__ rho, const double *__restrict__ u,
                 double *__restrict__ rho_ref, const double *__restrict__ p_bg,
                 double *__restrict__ p, double *__restrict__ c, double *__restrict__ pr2)
{
    const int64_t n = b.hdr->n_out;
    const int64_t step = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += step) {
        const RunDev &rd = b.runs[b.slot[i]];
        const double r = rho[i];
        if (rd.phase == RUN_INIT && rd.set_rho_ref) rho_ref[i] = r;
        double P, C;
        if (rd.eos == SPH_EOS_TAIT) {
            const double B = rd.rho0 * rd.c0 * rd.c0 / rd.gamma_tait;
            const double xr = r / rho_ref[i];
            const double x2 = xr * xr, x4 = x2 * x2, x6 = x4 * x2, x7 = x6 * xr;
            const double x3 = x2 * xr;
            P = p_bg[i] + B * (x7 - 1.0);
            C = rd.c0 * x3;
        } else {
            const double g = rd.gamma_gas;
            P = (g - 1.0) * r * u[i];
            C = sqrt(g * (g - 1.0) * u[i]);
        }
        p[i] = P;
        c[i] = C;
        pr2[i] = P / (r * r);
    }
}

// Record arrays of 4 GiB or more need 64-bit element offsets.
inline bool big_records(int64_t n, size_t rec) { return (uint64_t)n * rec >= (1ull << 32); }

template <bool Multi>
void density_launch(hipStream_t st, unsigned blocks, int precision, bool big, int64_t n,
                    int64_t ld, const DensRec *drec, const double *h, const int32_t *count,
                    const int32_t *idx, int max_nb, const Grid &g, double *rho, const BatchDev &b,
                    const KernelSel &ks, const StepMask &mask = StepMask{})
{
#define SPH_DENS_P(F, B, P, K)                                                             \
    density_kernel<F, Multi, B, P, K><<<blocks, kThreads, 0, st>>>(                        \
        n, ld, drec, h, count, idx, max_nb, g, rho, b, ks.sigma, ks.sinc_n, mask)
#define SPH_DENS(F, B)                                                                     \
    do {                                                                                   \
        const int pm = Multi ? -1 : per_mask(g);                                           \
        if constexpr (Multi) SPH_DENS_P(F, B, -1, KF_M4);                                  \
        else if (ks.family == SPH_KERNEL_WENDLAND_C2) SPH_DENS_P(F, B, -1, KF_WENDLAND);    \
        else if (ks.family == SPH_KERNEL_SINC) SPH_DENS_P(F, B, -1, KF_SINC);              \
        else if (pm == 0) SPH_DENS_P(F, B, 0, KF_M4);                                      \
        else if (pm == 4) SPH_DENS_P(F, B, 4, KF_M4);                                      \
        else if (pm == 7) SPH_DENS_P(F, B, 7, KF_M4);                                      \
        else SPH_DENS_P(F, B, -1, KF_M4);                                                  \
    } while (0)
    if (precision == SPH_FP32_PAIR) {
        if (big) SPH_DENS(true, true); else SPH_DENS(true, false);
    } else {
        if (big) SPH_DENS(false, true); else SPH_DENS(false, false);
    }
#undef SPH_DENS
#undef SPH_DENS_P
}

template <bool Multi>
void momentum_launch(hipStream_t st, unsigned blocks, int precision, bool big, int64_t n,
                     int64_t ld, const PairRec *rec, const int32_t *count, const int32_t *idx,
                     int max_nb, const Grid &g, const MomParams &mp, double *ax, double *ay,
                     double *az, double *dudt, double *mumax, const BatchDev &b,
                     const uint32_t *hflag, int family, bool iad, bool gve)
{
#define SPH_MOM_P(F, B, P, K)                                                              \
    momentum_kernel<F, Multi, B, P, K><<<blocks, kThreads, 0, st>>>(                       \
        n, ld, rec, count, idx, max_nb, g, mp, ax, ay, az, dudt, mumax, b, hflag)
#define SPH_MOM_IAD(F, B, K)                                                               \
    momentum_kernel<F, false, B, -1, K, true><<<blocks, kThreads, 0, st>>>(                \
        n, ld, rec, count, idx, max_nb, g, mp, ax, ay, az, dudt, mumax, b, hflag)
#define SPH_MOM_GVE(F, B, K, I)                                                            \
    momentum_kernel<F, false, B, -1, K, I, true><<<blocks, kThreads, 0, st>>>(             \
        n, ld, rec, count, idx, max_nb, g, mp, ax, ay, az, dudt, mumax, b, hflag)
#define SPH_MOM_GVE_K(F, B, I)                                                             \
    do {                                                                                   \
        if (family == SPH_KERNEL_WENDLAND_C2) SPH_MOM_GVE(F, B, KF_WENDLAND, I);            \
        else if (family == SPH_KERNEL_SINC) SPH_MOM_GVE(F, B, KF_SINC, I);                 \
        else SPH_MOM_GVE(F, B, KF_M4, I);                                                  \
    } while (0)
#define SPH_MOM(F, B)                                                                      \
    do {                                                                                   \
        const int pm = Multi ? -1 : per_mask(g);                                           \
        if constexpr (Multi) SPH_MOM_P(F, B, -1, KF_M4);                                   \
        else if (gve && iad) SPH_MOM_GVE_K(F, B, true);                                    \
        else if (gve) SPH_MOM_GVE_K(F, B, false);                                          \
        else if (iad && family == SPH_KERNEL_WENDLAND_C2) SPH_MOM_IAD(F, B, KF_WENDLAND);  \
        else if (iad && family == SPH_KERNEL_SINC) SPH_MOM_IAD(F, B, KF_SINC);             \
        else if (iad) SPH_MOM_IAD(F, B, KF_M4);                                            \
        else if (family == SPH_KERNEL_WENDLAND_C2) SPH_MOM_P(F, B, -1, KF_WENDLAND);        \
        else if (family == SPH_KERNEL_SINC) SPH_MOM_P(F, B, -1, KF_SINC);                  \
        else if (pm == 0) SPH_MOM_P(F, B, 0, KF_M4);                                       \
        else if (pm == 4) SPH_MOM_P(F, B, 4, KF_M4);                                       \
        else if (pm == 7) SPH_MOM_P(F, B, 7, KF_M4);                                       \
        else SPH_MOM_P(F, B, -1, KF_M4);                                                   \
    } while (0)
    if (precision == SPH_FP32_PAIR) {
        if (big) SPH_MOM(true, true); else SPH_MOM(true, false);
    } else {
        if (big) SPH_MOM(false, true); else SPH_MOM(false, false);
    }
#undef SPH_MOM
#undef SPH_MOM_GVE_K
#undef SPH_MOM_GVE
#undef SPH_MOM_IAD
#undef SPH_MOM_P
}

}  // namespace

hipError_t launch_density(sph_ctx ctx, const sph_particles &p, const sph_nbrs &nb,
                          int precision, const KernelSel &ks, bool gve, double *rho,
                          const StepMask &mask)
{
    const unsigned nblk = blocks_for(p.n, kThreads);
    // generalised volume elements: the records carry X in place of m, the
    // kernel leaves k_i in rho, which is then scaled by m_i / X_i
    pack_dens_kernel<<<blocks_for(p.n, 256), 256, 0, ctx->stream>>>(
        p.n, nullptr, p.x, p.y, p.z, gve ? p.xw : p.m, ctx->drec);
    const int tk = ktime_begin(ctx, TK_DENSITY);
    density_launch<false>(ctx->stream, nblk, precision, big_records(p.n, sizeof(DensRec)), p.n,
                          p.n, ctx->drec, p.h, nb.count, nb.idx, nb.max_nb, ctx->grid, rho,
                          BatchDev{}, ks, mask);
    ktime_end(ctx, tk);
    if (gve)
        gve_density_kernel<<<blocks_for(p.n, 256), 256, 0, ctx->stream>>>(p.n, p.m, p.xw, rho,
                                                                          mask);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// The density without allocation (sph_density_noalloc): the neighbour records
// go to a file-scope device array of SPH_DENSITY_NOALLOC_MAX_N records (32 MiB),
// which each GPU the library runs on holds until the process ends. In host
// code the array's name is not a device address: the address is taken once
// per device, with that device current, by hipGetSymbolAddress and kept; the
// kernels receive it as their record pointer. Every call on a device shares
// its array, so calls that overlap on one device race.
static __device__ __align__(256) DensRec scratch[SPH_DENSITY_NOALLOC_MAX_N];

namespace {
constexpr int kNoAllocDevices = 64;
std::mutex g_scratch_mu;
DensRec *g_scratch_ptr[kNoAllocDevices] = {};
}  // namespace

hipError_t density_noalloc_scratch(DensRec **out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kNoAllocDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_ptr[dev] = static_cast<DensRec *>(ptr);
    }
    *out = g_scratch_ptr[dev];
    return hipSuccess;
}

hipError_t launch_density_noalloc(hipStream_t stream, const sph_particles &p, const sph_nbrs &nb,
                                  const Grid &g, int precision, const KernelSel &ks, bool gve,
                                  double *rho, DensRec *recs)
{
    // the same kernels as launch_density, with recs (the device address of
    // the static array) in place of the context's records
    pack_dens_kernel<<<blocks_for(p.n, 256), 256, 0, stream>>>(p.n, nullptr, p.x, p.y, p.z,
                                                                gve ? p.xw : p.m, recs);
    density_launch<false>(stream, blocks_for(p.n, kThreads), precision, false, p.n, p.n, recs,
                          p.h, nb.count, nb.idx, nb.max_nb, g, rho, BatchDev{}, ks);
    if (gve)
        gve_density_kernel<<<blocks_for(p.n, 256), 256, 0, stream>>>(p.n, p.m, p.xw, rho,
                                                                      StepMask{});
    return hipGetLastError();
}

hipError_t launch_volume_weights(sph_ctx ctx, const sph_particles &p, const double *rho,
                                 double exponent)
{
    volume_weights_kernel<<<blocks_for(p.n, 256), 256, 0, ctx->stream>>>(p.n, p.m, rho,
                                                                         exponent, p.xw);
    return hipGetLastError();
}

hipError_t launch_eos(sph_ctx ctx, const sph_particles &p, const sph_params &prm,
                      const sph_fields &f, const StepMask &mask)
{
    eos_kernel<<<blocks_for(p.n, 256), 256, 0, ctx->stream>>>(
        p.n, prm.eos, prm.rho0, prm.c0, prm.gamma_tait, prm.gamma_gas, f.rho, p.u, p.rho_ref,
        p.p_bg, f.p, f.c, f.pr2, mask);
    return hipGetLastError();
}

hipError_t launch_momentum(sph_ctx ctx, const sph_particles &p, const sph_nbrs &nb,
                           const sph_params &prm, const sph_fields &f, const sph_accel &a,
                           const double *bin, int sub, int B)
{
    const unsigned nblk = blocks_for(p.n, kThreads);
    const KernelSel ks = kernel_sel(prm);
    const bool iad = prm.gradient == SPH_GRAD_IAD;
    const MomParams mp{prm.alpha, prm.beta, prm.eta2, ks.sigma, ks.sinc_n, ctx->iad_c, bin, sub,
                       B};
    if (iad) {
        pack_vol_kernel<<<blocks_for(p.n, 256), 256, 0, ctx->stream>>>(p.n, p.x, p.y, p.z, p.m,
                                                                       f.rho, ctx->drec);
#define SPH_IAD(K)                                                                         \
    iad_kernel<K><<<blocks_for(p.n, 256), 256, 0, ctx->stream>>>(                          \
        p.n, p.n, ctx->drec, p.h, nb.count, nb.idx, nb.max_nb, ctx->grid, ks.sigma,        \
        ks.sinc_n, ctx->iad_c)
        const int tk = ktime_begin(ctx, TK_IAD);
        if (ks.family == SPH_KERNEL_WENDLAND_C2) SPH_IAD(KF_WENDLAND);
        else if (ks.family == SPH_KERNEL_SINC) SPH_IAD(KF_SINC);
        else SPH_IAD(KF_M4);
        ktime_end(ctx, tk);
#undef SPH_IAD
    }
    const bool gve = prm.volume == SPH_VOLUME_GENERALISED;
    const bool r32 = prm.precision == SPH_FP32_PAIR && !iad;  // PairRec32 records
    if (r32)
        pack_pair_kernel<true><<<blocks_for(p.n, 256), 256, 0, ctx->stream>>>(
            p.n, nullptr, p.x, p.y, p.z, p.vx, p.vy, p.vz, p.h, p.m, f.rho, f.c, f.pr2,
            gve ? p.xw : nullptr, ctx->prec);
    else
        pack_pair_kernel<false><<<blocks_for(p.n, 256), 256, 0, ctx->stream>>>(
            p.n, nullptr, p.x, p.y, p.z, p.vx, p.vy, p.vz, p.h, p.m, f.rho, f.c, f.pr2,
            gve ? p.xw : nullptr, ctx->prec);
    const int tk = ktime_begin(ctx, TK_MOMENTUM);
    momentum_launch<false>(ctx->stream, nblk, prm.precision,
                           big_records(p.n, r32 ? sizeof(PairRec32) : sizeof(PairRec)),
                           p.n, p.n, ctx->prec, nb.count, nb.idx, nb.max_nb, ctx->grid, mp,
                           a.ax, a.ay, a.az, a.dudt, a.mumax, BatchDev{}, ctx->hflag_dev,
                           ks.family, iad, gve);
    ktime_end(ctx, tk);
    return hipGetLastError();
}

// Ensemble launches: fixed grids sized for the capacity (the elementwise
// kernels loop over the header's count, the gathers take one tile per block
// and leave the blocks past it idle), so that the same captured sequence
// serves every step.
hipError_t launch_density_batch(sph_ctx ctx, const BatchDev &b, int precision, const double *F,
                                const int32_t *count, const int32_t *idx, int max_nb,
                                double *rho)
{
    const int64_t cap = b.cap;
    const int64_t *n_out = &b.hdr->n_out;
    const unsigned g1 = std::min<unsigned>(blocks_for(cap, 256), 4096u);
    const unsigned g2 = ens_pair_blocks(cap);
    pack_dens_kernel<<<g1, 256, 0, ctx->stream>>>(0, n_out, F + 0 * cap, F + 1 * cap,
                                                  F + 2 * cap, F + 8 * cap, ctx->drec);
    density_launch<true>(ctx->stream, g2, precision, big_records(cap, sizeof(DensRec)), 0, cap,
                         ctx->drec, F + 7 * cap, count, idx, max_nb, Grid{}, rho, b,
                         KernelSel{SPH_KERNEL_M4, 0, 0.0});
    return hipGetLastError();
}

hipError_t launch_eos_batch(sph_ctx ctx, const BatchDev &b, double *F, const double *rho,
                            double *p, double *c, double *pr2)
{
    const int64_t cap = b.cap;
    const unsigned g1 = std::min<unsigned>(blocks_for(cap, 256), 4096u);
    eos_batch_kernel<<<g1, 256, 0, ctx->stream>>>(b, rho, F + 6 * cap, F + 10 * cap,
                                                  F + 9 * cap, p, c, pr2);
    return hipGetLastError();
}

hipError_t launch_momentum_batch(sph_ctx ctx, const BatchDev &b, int precision,
                                 const double *F, const int32_t *count, const int32_t *idx,
                                 int max_nb, const double *rho, const double *c,
                                 const double *pr2, double *ax, double *ay, double *az,
                                 double *dudt, double *mumax)
{
    const int64_t cap = b.cap;
    const int64_t *n_out = &b.hdr->n_out;
    const unsigned g1 = std::min<unsigned>(blocks_for(cap, 256), 4096u);
    const unsigned g2 = ens_pair_blocks(cap);
    const bool r32 = precision == SPH_FP32_PAIR;  // PairRec32 records
    if (r32)
        pack_pair_kernel<true><<<g1, 256, 0, ctx->stream>>>(
            0, n_out, F + 0 * cap, F + 1 * cap, F + 2 * cap, F + 3 * cap, F + 4 * cap,
            F + 5 * cap, F + 7 * cap, F + 8 * cap, rho, c, pr2, nullptr, ctx->prec);
    else
        pack_pair_kernel<false><<<g1, 256, 0, ctx->stream>>>(
            0, n_out, F + 0 * cap, F + 1 * cap, F + 2 * cap, F + 3 * cap, F + 4 * cap,
            F + 5 * cap, F + 7 * cap, F + 8 * cap, rho, c, pr2, nullptr, ctx->prec);
    momentum_launch<true>(ctx->stream, g2, precision,
                          big_records(cap, r32 ? sizeof(PairRec32) : sizeof(PairRec)), 0, cap,
                          ctx->prec, count, idx, max_nb, Grid{}, MomParams{}, ax, ay, az, dudt,
                          mumax, b, nullptr, SPH_KERNEL_M4, false, false);
    return hipGetLastError();
}

}  // namespace sph
