// Host side of the C ABI declared in include/sph.h: argument checks, the
// context and its scratch, grid set-up and the order of launches.
#include <algorithm>
#include <array>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <vector>

#include "sph_internal.h"

using namespace sph;

namespace sph {

// Grid of cells of side >= 2 h_max (1 + 1e-9) on every axis, at most
// max_axis cells per axis and cell_cap in total (coarser cells only add
// candidates: the relation test is exact).
// Normalisation of the sinc kernel of exponent n: B_n = 1 / (4 pi I_n) with
// I_n = int_0^2 q^2 (sin(x)/x)^n dq, x = pi q / 2, by the 5-point
// Gauss-Legendre rule on 400 panels (the integrand is analytic; the rule is
// exact to rounding here). One table for n = 3..12, filled once.
static double sinc_norm(int n)
{
    static const double node[5] = {-0.9061798459386640, -0.5384693101056831, 0.0,
                                   0.5384693101056831, 0.9061798459386640};
    static const double wgt[5] = {0.2369268850561891, 0.4786286704993665,
                                  0.5688888888888889, 0.4786286704993665,
                                  0.2369268850561891};
    const int panels = 400;
    const double half = 1.0 / panels;  // half width of a panel of [0, 2]
    double acc = 0.0;
    for (int k = 0; k < panels; ++k) {
        const double mid = (2 * k + 1) * half;
        for (int t = 0; t < 5; ++t) {
            const double q = mid + half * node[t];
            const double x = 0.5 * M_PI * q;
            const double sx = std::sin(x) / x;
            acc += wgt[t] * q * q * std::pow(sx, n);
        }
    }
    return 1.0 / (4.0 * M_PI * acc * half);
}

KernelSel kernel_sel(const sph_params &prm)
{
    static const std::array<double, 13> sinc_b = [] {
        std::array<double, 13> t{};
        for (int n = 3; n <= 12; ++n) t[n] = sinc_norm(n);
        return t;
    }();
    KernelSel k{prm.kernel, prm.sinc_n, 1.0 / M_PI};
    if (prm.kernel == SPH_KERNEL_WENDLAND_C2) k.sigma = 21.0 / (16.0 * M_PI);
    if (prm.kernel == SPH_KERNEL_SINC) k.sigma = sinc_b[prm.sinc_n];
    return k;
}

Grid make_grid(const sph_box &b, double h_max, int64_t cell_cap, int max_axis)
{
    Grid g{};
    const double want = 2.0 * h_max * (1.0 + 1e-9);
    for (int a = 0; a < 3; ++a) {
        g.periodic[a] = b.periodic[a];
        g.lo[a] = b.lo[a];
        g.hi[a] = b.hi[a];
        g.len[a] = b.hi[a] - b.lo[a];
        g.half[a] = 0.5 * g.len[a];
        double nc = std::floor(g.len[a] / want);
        nc = std::min(std::max(nc, 1.0), (double)max_axis);
        g.nc[a] = (int)nc;
    }
    while ((int64_t)g.nc[0] * g.nc[1] * g.nc[2] > cell_cap) {
        int a = 0;
        for (int k = 1; k < 3; ++k)
            if (g.nc[k] > g.nc[a]) a = k;
        g.nc[a] = std::max(1, g.nc[a] / 2);
    }
    int maxc = std::max(g.nc[0], std::max(g.nc[1], g.nc[2]));
    g.bits = 0;
    while ((1 << g.bits) < maxc) ++g.bits;
    // z slices inside a cell, in the key bits the Morton code leaves free
    g.zbits = std::min(kSliceBits, 32 - 3 * g.bits);
    for (int a = 0; a < 3; ++a) g.inv_s[a] = (double)g.nc[a] / g.len[a];
    return g;
}

}  // namespace sph

namespace sph {

const char *const kTimedKernelNames[TK_COUNT] = {"find_neighbors_kernel", "fallback_kernel",
                                                 "density_kernel", "iad_kernel",
                                                 "momentum_kernel"};

int ktime_begin(sph_ctx ctx, int id)
{
    KTimer &t = ctx->timer;
    if (!t.on || ctx->capturing) return -1;
    hipEvent_t a = nullptr, b = nullptr;
    if (t.pool.size() >= 2) {
        a = t.pool.back();
        t.pool.pop_back();
        b = t.pool.back();
        t.pool.pop_back();
    } else if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) {
        (void)hipGetLastError();
        if (a) (void)hipEventDestroy(a);
        return -1;
    }
    if (hipEventRecord(a, ctx->stream) != hipSuccess) {
        (void)hipGetLastError();
        t.pool.push_back(a);
        t.pool.push_back(b);
        return -1;
    }
    t.pending.push_back(KTimer::Pending{id, a, b});
    return (int)t.pending.size() - 1;
}

void ktime_end(sph_ctx ctx, int slot)
{
    if (slot < 0) return;
    KTimer &t = ctx->timer;
    if (hipEventRecord(t.pending[(size_t)slot].b, ctx->stream) != hipSuccess) {
        (void)hipGetLastError();
        t.pending[(size_t)slot].id = -1;  // dropped when read
    }
}

}  // namespace sph

namespace {

// Sum the durations of the pending timed launches (synchronises on each
// closing event) and recycle their events.
void ktime_collect(sph_ctx ctx)
{
    KTimer &t = ctx->timer;
    for (const KTimer::Pending &q : t.pending) {
        float ms = 0.0f;
        if (q.id >= 0 && hipEventSynchronize(q.b) == hipSuccess &&
            hipEventElapsedTime(&ms, q.a, q.b) == hipSuccess) {
            t.sum_ms[q.id] += ms;
            t.launches[q.id] += 1;
        } else {
            (void)hipGetLastError();
        }
        t.pool.push_back(q.a);
        t.pool.push_back(q.b);
    }
    t.pending.clear();
}

void ktime_release(sph_ctx ctx)
{
    KTimer &t = ctx->timer;
    for (const KTimer::Pending &q : t.pending) {
        t.pool.push_back(q.a);
        t.pool.push_back(q.b);
    }
    t.pending.clear();
    for (hipEvent_t e : t.pool) (void)hipEventDestroy(e);
    t.pool.clear();
}

thread_local std::string g_no_ctx_error;

sph_status fail(sph_ctx ctx, sph_status s, const char *fmt, ...)
    __attribute__((format(printf, 3, 4)));

sph_status fail(sph_ctx ctx, sph_status s, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (ctx) ctx->last_error = buf;
    else g_no_ctx_error = buf;
    return s;
}

sph_status hip_fail(sph_ctx ctx, hipError_t e, const char *where)
{
    return fail(ctx, SPH_E_HIP, "%s: %s", where, hipGetErrorString(e));
}

#define SPH_HIP(ctx, call)                                          \
    do {                                                            \
        hipError_t e_ = (call);                                     \
        if (e_ != hipSuccess) return hip_fail((ctx), e_, #call);    \
    } while (0)

sph_status check_particles(sph_ctx ctx, const sph_particles *p, bool need_v)
{
    if (!p) return fail(ctx, SPH_E_INVALID, "particles is NULL");
    if (p->n < 0 || p->n > ctx->n_max)
        return fail(ctx, SPH_E_INVALID, "n = %lld outside [0, n_max = %lld]",
                    (long long)p->n, (long long)ctx->n_max);
    if (p->n > 0) {
        if (!p->x || !p->y || !p->z || !p->h || !p->m || !p->id)
            return fail(ctx, SPH_E_INVALID, "x, y, z, h, m and id are required");
        if (need_v && (!p->vx || !p->vy || !p->vz || !p->u))
            return fail(ctx, SPH_E_INVALID, "vx, vy, vz and u are required");
        const bool any_g = p->gx || p->gy || p->gz, all_g = p->gx && p->gy && p->gz;
        if (any_g && !all_g) return fail(ctx, SPH_E_INVALID, "gx, gy, gz: all or none");
    }
    return SPH_OK;
}

sph_status check_box(sph_ctx ctx, const sph_box *b)
{
    if (!b) return fail(ctx, SPH_E_INVALID, "box is NULL");
    for (int a = 0; a < 3; ++a) {
        if (!(std::isfinite(b->lo[a]) && std::isfinite(b->hi[a]) && b->hi[a] > b->lo[a]))
            return fail(ctx, SPH_E_INVALID, "box axis %d: need finite lo < hi", a);
        if (b->periodic[a] != 0 && b->periodic[a] != 1)
            return fail(ctx, SPH_E_INVALID, "box axis %d: periodic must be 0 or 1", a);
    }
    return SPH_OK;
}

sph_status check_nbrs(sph_ctx ctx, const sph_nbrs *nb, int64_t n)
{
    if (!nb) return fail(ctx, SPH_E_INVALID, "nbrs is NULL");
    if (nb->max_nb < 1 || nb->max_nb > ctx->max_nb)
        return fail(ctx, SPH_E_INVALID, "max_nb = %d outside [1, %d]", nb->max_nb, ctx->max_nb);
    if (n > 0 && (!nb->count || !nb->idx))
        return fail(ctx, SPH_E_INVALID, "count and idx are required");
    return SPH_OK;
}

sph_status check_params(sph_ctx ctx, const sph_params *prm)
{
    if (!prm) return fail(ctx, SPH_E_INVALID, "params is NULL");
    if (prm->precision != SPH_FP64 && prm->precision != SPH_FP32_PAIR)
        return fail(ctx, SPH_E_INVALID, "unknown precision %d", prm->precision);
    if (prm->eos != SPH_EOS_TAIT && prm->eos != SPH_EOS_IDEAL)
        return fail(ctx, SPH_E_INVALID, "unknown eos %d", prm->eos);
    if (prm->kernel != SPH_KERNEL_M4 && prm->kernel != SPH_KERNEL_WENDLAND_C2 &&
        prm->kernel != SPH_KERNEL_SINC)
        return fail(ctx, SPH_E_INVALID, "unknown kernel %d", prm->kernel);
    if (prm->kernel == SPH_KERNEL_SINC && (prm->sinc_n < 3 || prm->sinc_n > 12))
        return fail(ctx, SPH_E_INVALID, "sinc exponent %d outside [3, 12]", prm->sinc_n);
    if (prm->gradient != SPH_GRAD_KERNEL && prm->gradient != SPH_GRAD_IAD)
        return fail(ctx, SPH_E_INVALID, "unknown gradient %d", prm->gradient);
    if (prm->volume != SPH_VOLUME_STANDARD && prm->volume != SPH_VOLUME_GENERALISED)
        return fail(ctx, SPH_E_INVALID, "unknown volume elements %d", prm->volume);
    if (prm->volume == SPH_VOLUME_GENERALISED && !std::isfinite(prm->volume_p))
        return fail(ctx, SPH_E_INVALID, "volume_p must be finite");
    return SPH_OK;
}

Grid box_grid(const sph_box &b)
{
    Grid g{};
    for (int a = 0; a < 3; ++a) {
        g.periodic[a] = b.periodic[a];
        g.lo[a] = b.lo[a];
        g.hi[a] = b.hi[a];
        g.len[a] = b.hi[a] - b.lo[a];
        g.half[a] = 0.5 * g.len[a];
        g.nc[a] = 1;
    }
    return g;
}

bool same_box(const Grid &g, const sph_box &b)
{
    for (int a = 0; a < 3; ++a)
        if (g.lo[a] != b.lo[a] || g.hi[a] != b.hi[a] || g.periodic[a] != b.periodic[a])
            return false;
    return true;
}

template <typename T>
sph_status dev_alloc(sph_ctx ctx, T **p, int64_t count)
{
    const size_t bytes = sizeof(T) * (size_t)std::max<int64_t>(count, 1);
    if (hipMalloc((void **)p, bytes) != hipSuccess) {
        *p = nullptr;
        (void)hipGetLastError();
        return fail(ctx, SPH_E_NOMEM, "hipMalloc of %zu bytes failed", bytes);
    }
    ctx->scratch_bytes += (int64_t)bytes;
    return SPH_OK;
}

void free_ctx(sph_ctx ctx)
{
    ktime_release(ctx);
    release_gravity_tree(ctx);
    if (ctx->step_exec) (void)hipGraphExecDestroy(ctx->step_exec);
    if (ctx->step_graph) (void)hipGraphDestroy(ctx->step_graph);
    void *ptrs[] = {ctx->keys[0], ctx->keys[1], ctx->vals[0], ctx->vals[1], ctx->hist,
                    ctx->scan_part, ctx->cell_start, ctx->cell_end, ctx->perm_tmp,
                    ctx->perm_tmp_id, ctx->red_part, ctx->status_dev, ctx->nb_mask, ctx->hflag_dev,
                    ctx->fb_tiles, ctx->fb_count, ctx->it_words, ctx->it_hmax, ctx->cell_s2max,
                    ctx->iad_c, ctx->dtc, ctx->blk_words,
                    ctx->srec, ctx->drec, ctx->prec};
    for (void *q : ptrs)
        if (q) (void)hipFree(q);
    delete ctx;
}

}  // namespace

extern "C" {

const char *sph_status_string(sph_status s)
{
    switch (s) {
    case SPH_OK: return "ok";
    case SPH_E_INVALID: return "invalid argument";
    case SPH_E_CAPACITY: return "neighbour list capacity exceeded";
    case SPH_E_HIP: return "HIP runtime error";
    case SPH_E_DOMAIN: return "domain error (h above h_max or periodic axis too short)";
    case SPH_E_NOMEM: return "out of device memory";
    case SPH_E_AGAIN: return "not ready";
    case SPH_E_NONFINITE: return "non-finite state";
    default: return "unknown status";
    }
}

const char *sph_last_error(sph_ctx ctx)
{
    return ctx ? ctx->last_error.c_str() : g_no_ctx_error.c_str();
}

const char *sph_version(void)
{
    static char buf[128];
    hipDeviceProp_t prop;
    int dev = 0;
    if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess)
        snprintf(buf, sizeof buf, "libsph 1 %s %d CUs", prop.gcnArchName,
                 prop.multiProcessorCount);
    else
        snprintf(buf, sizeof buf, "libsph 1 (no device)");
    return buf;
}

sph_status sph_ctx_create(sph_ctx *out, int64_t n_max, int32_t max_nb, sph_stream stream)
{
    if (!out) return fail(nullptr, SPH_E_INVALID, "out is NULL");
    *out = nullptr;
    if (n_max < 1 || n_max > ((int64_t)1 << 31) - kSortTile)
        return fail(nullptr, SPH_E_INVALID, "n_max = %lld out of range", (long long)n_max);
    if (max_nb < 1 || max_nb > 4096)
        return fail(nullptr, SPH_E_INVALID, "max_nb = %d out of range [1, 4096]", max_nb);
    if ((int64_t)max_nb * n_max >= ((int64_t)1 << 40))
        return fail(nullptr, SPH_E_INVALID, "max_nb * n_max too large");
    sph_ctx ctx = new (std::nothrow) sph_ctx_s();
    if (!ctx) return fail(nullptr, SPH_E_NOMEM, "host allocation failed");
    if (hipGetDevice(&ctx->device) != hipSuccess) {
        delete ctx;
        return fail(nullptr, SPH_E_HIP, "no HIP device");
    }
    ctx->stream = (hipStream_t)stream;
    ctx->n_max = n_max;
    ctx->max_nb = max_nb;
    ctx->tiles_max = (n_max + kSortTile - 1) / kSortTile;
    ctx->scan_len_max = ctx->tiles_max * kRadixBins;
    ctx->cell_cap = std::max<int64_t>(n_max / 8 + 64, 65536);
    sph_status s = SPH_OK;
#define ALLOC(ptr, count)                                   \
    if (s == SPH_OK) s = dev_alloc(ctx, &(ptr), (count));
    ALLOC(ctx->keys[0], n_max);
    ALLOC(ctx->keys[1], n_max);
    ALLOC(ctx->vals[0], n_max);
    ALLOC(ctx->vals[1], n_max);
    ALLOC(ctx->hist, ctx->scan_len_max);
    ALLOC(ctx->scan_part, (ctx->scan_len_max + kScanChunk - 1) / kScanChunk + 1);
    ALLOC(ctx->cell_start, ctx->cell_cap);
    ALLOC(ctx->cell_end, ctx->cell_cap);
    ALLOC(ctx->cell_s2max, ctx->cell_cap);
    ALLOC(ctx->iad_c, 6 * n_max);
    ALLOC(ctx->nb_mask, (int64_t)kSearchMaskWords * ((n_max + 63) / 64) * 64);
    ALLOC(ctx->fb_tiles, (n_max + 63) / 64);
    ALLOC(ctx->fb_count, 1);
    ALLOC(ctx->it_words, kItWords);
    ALLOC(ctx->it_hmax, 1);
    ALLOC(ctx->srec, n_max);
    ALLOC(ctx->drec, n_max);
    ALLOC(ctx->prec, n_max);
    ALLOC(ctx->perm_tmp, (int64_t)kPermFields * n_max);
    ALLOC(ctx->perm_tmp_id, n_max);
    ALLOC(ctx->red_part, (int64_t)kRedFields * kRedMaxBlocks);
    ALLOC(ctx->dtc, n_max);
    ALLOC(ctx->blk_words, 2);
    ALLOC(ctx->status_dev, 1);
    ALLOC(ctx->hflag_dev, 1);
#undef ALLOC
    if (s != SPH_OK) {
        g_no_ctx_error = ctx->last_error;
        free_ctx(ctx);
        return s;
    }
    if (hipMemsetAsync(ctx->status_dev, 0, sizeof(uint32_t), ctx->stream) != hipSuccess ||
        hipStreamSynchronize(ctx->stream) != hipSuccess) {
        free_ctx(ctx);
        return fail(nullptr, SPH_E_HIP, "status word initialisation failed");
    }
    *out = ctx;
    return SPH_OK;
}

sph_status sph_ctx_destroy(sph_ctx ctx)
{
    if (!ctx) return SPH_OK;
    (void)hipStreamSynchronize(ctx->stream);
    free_ctx(ctx);
    return SPH_OK;
}

int64_t sph_ctx_scratch_bytes(sph_ctx ctx) { return ctx ? ctx->scratch_bytes : 0; }

sph_status sph_ctx_timing(sph_ctx ctx, int32_t enable)
{
    if (!ctx) return fail(nullptr, SPH_E_INVALID, "ctx is NULL");
    if (enable) {
        SPH_HIP(ctx, hipStreamSynchronize(ctx->stream));
        ktime_collect(ctx);
        for (int k = 0; k < TK_COUNT; ++k) {
            ctx->timer.sum_ms[k] = 0.0;
            ctx->timer.launches[k] = 0;
        }
    }
    ctx->timer.on = enable != 0;
    return SPH_OK;
}

sph_status sph_ctx_kernel_time(sph_ctx ctx, const char *kernel, double *avg_ms,
                               int64_t *launches)
{
    if (!ctx) return fail(nullptr, SPH_E_INVALID, "ctx is NULL");
    if (!kernel || !avg_ms || !launches)
        return fail(ctx, SPH_E_INVALID, "kernel, avg_ms and launches are required");
    int id = -1;
    for (int k = 0; k < TK_COUNT; ++k)
        if (std::strcmp(kernel, kTimedKernelNames[k]) == 0) id = k;
    if (id < 0) return fail(ctx, SPH_E_INVALID, "kernel %s is not timed", kernel);
    ktime_collect(ctx);
    *launches = ctx->timer.launches[id];
    *avg_ms = *launches ? ctx->timer.sum_ms[id] / (double)*launches : 0.0;
    return SPH_OK;
}

sph_status sph_ctx_check(sph_ctx ctx)
{
    if (!ctx) return fail(nullptr, SPH_E_INVALID, "ctx is NULL");
    SPH_HIP(ctx, hipStreamSynchronize(ctx->stream));
    uint32_t st = 0;
    SPH_HIP(ctx, hipMemcpy(&st, ctx->status_dev, sizeof st, hipMemcpyDeviceToHost));
    if (st) SPH_HIP(ctx, hipMemset(ctx->status_dev, 0, sizeof st));
    if (st & ST_DOMAIN) return fail(ctx, SPH_E_DOMAIN, "a particle has h > h_max");
    if (st & ST_CAPACITY) return fail(ctx, SPH_E_CAPACITY, "a neighbour list exceeded max_nb");
    if (st & ST_NONFINITE) return fail(ctx, SPH_E_NONFINITE, "NaN or Inf in the state");
    return SPH_OK;
}

}  // extern "C"

namespace {

// sph_build_cells, with up to 6 extra per-particle arrays reordered alongside
sph_status build_cells(sph_ctx ctx, const sph_particles *p, const sph_box *box, double h_max,
                       double *const *extra, int n_extra)
{
    if (!ctx) return fail(nullptr, SPH_E_INVALID, "ctx is NULL");
    sph_status s;
    if ((s = check_particles(ctx, p, false)) != SPH_OK) return s;
    if ((s = check_box(ctx, box)) != SPH_OK) return s;
    if (!(h_max > 0.0) || !std::isfinite(h_max))
        return fail(ctx, SPH_E_INVALID, "h_max must be finite and > 0");
    for (int a = 0; a < 3; ++a)
        if (box->periodic[a] && !(box->hi[a] - box->lo[a] > 4.0 * h_max))
            return fail(ctx, SPH_E_DOMAIN, "periodic axis %d is not longer than 4 h_max", a);
    ctx->grid = make_grid(*box, h_max, ctx->cell_cap, kMaxAxisCells);
    ctx->n_built = p->n;
    if (p->n == 0) return SPH_OK;
    SPH_HIP(ctx, launch_build_cells(ctx, *p, ctx->grid, h_max, extra, n_extra));
    return SPH_OK;
}

}  // namespace

extern "C" {

sph_status sph_build_cells(sph_ctx ctx, const sph_particles *p, const sph_box *box,
                           double h_max)
{
    return build_cells(ctx, p, box, h_max, nullptr, 0);
}

sph_status sph_find_neighbors(sph_ctx ctx, const sph_particles *p, const sph_box *box,
                              const sph_nbrs *nb)
{
    if (!ctx) return fail(nullptr, SPH_E_INVALID, "ctx is NULL");
    sph_status s;
    if ((s = check_particles(ctx, p, false)) != SPH_OK) return s;
    if ((s = check_box(ctx, box)) != SPH_OK) return s;
    if ((s = check_nbrs(ctx, nb, p->n)) != SPH_OK) return s;
    if (ctx->n_built != p->n || !same_box(ctx->grid, *box))
        return fail(ctx, SPH_E_INVALID, "sph_build_cells was not called for these particles/box");
    if (p->n == 0) return SPH_OK;
    SPH_HIP(ctx, launch_find_neighbors(ctx, *p, *nb));
    return SPH_OK;
}

sph_status sph_density(sph_ctx ctx, const sph_particles *p, const sph_box *box,
                       const sph_nbrs *nb, const sph_params *prm, double *rho)
{
    if (!ctx) return fail(nullptr, SPH_E_INVALID, "ctx is NULL");
    sph_status s;
    if ((s = check_particles(ctx, p, false)) != SPH_OK) return s;
    if ((s = check_box(ctx, box)) != SPH_OK) return s;
    if ((s = check_nbrs(ctx, nb, p->n)) != SPH_OK) return s;
    if ((s = check_params(ctx, prm)) != SPH_OK) return s;
    if (p->n > 0 && !rho) return fail(ctx, SPH_E_INVALID, "rho is NULL");
    if (ctx->n_built != p->n || !same_box(ctx->grid, *box))
        return fail(ctx, SPH_E_INVALID, "sph_build_cells was not called for these particles/box");
    if (p->n == 0) return SPH_OK;
    const bool gve = prm->volume == SPH_VOLUME_GENERALISED;
    if (gve && !p->xw)
        return fail(ctx, SPH_E_INVALID, "generalised volume elements need p->xw");
    SPH_HIP(ctx, launch_density(ctx, *p, *nb, prm->precision, kernel_sel(*prm), gve, rho));
    return SPH_OK;
}

sph_status sph_density_noalloc(const sph_particles *p, const sph_box *box, const sph_nbrs *nb,
                               const sph_params *prm, double *rho, sph_stream stream)
{
    if (!p) return fail(nullptr, SPH_E_INVALID, "particles is NULL");
    if (p->n < 0) return fail(nullptr, SPH_E_INVALID, "n = %lld < 0", (long long)p->n);
    if (p->n > SPH_DENSITY_NOALLOC_MAX_N)
        return fail(nullptr, SPH_E_CAPACITY,
                    "n = %lld exceeds the %d particles of the static scratch",
                    (long long)p->n, SPH_DENSITY_NOALLOC_MAX_N);
    sph_status s;
    if ((s = check_box(nullptr, box)) != SPH_OK) return s;
    if ((s = check_params(nullptr, prm)) != SPH_OK) return s;
    if (!nb) return fail(nullptr, SPH_E_INVALID, "nbrs is NULL");
    if (p->n == 0) return SPH_OK;
    if (nb->max_nb < 1) return fail(nullptr, SPH_E_INVALID, "max_nb = %d < 1", nb->max_nb);
    if (!nb->count || !nb->idx) return fail(nullptr, SPH_E_INVALID, "count and idx are required");
    if (!p->x || !p->y || !p->z || !p->h || !p->m || !rho)
        return fail(nullptr, SPH_E_INVALID, "x, y, z, h, m and rho are required");
    const bool gve = prm->volume == SPH_VOLUME_GENERALISED;
    if (gve && !p->xw)
        return fail(nullptr, SPH_E_INVALID, "generalised volume elements need p->xw");
    DensRec *recs = nullptr;
    SPH_HIP(nullptr, density_noalloc_scratch(&recs));
    SPH_HIP(nullptr, launch_density_noalloc(static_cast<hipStream_t>(stream), *p, *nb,
                                            box_grid(*box), prm->precision,
                                            kernel_sel(*prm), gve, rho, recs));
    return SPH_OK;
}

sph_status sph_volume_weights(sph_ctx ctx, const sph_particles *p, const double *rho,
                              double exponent)
{
    if (!ctx) return fail(nullptr, SPH_E_INVALID, "ctx is NULL");
    sph_status s;
    if ((s = check_particles(ctx, p, false)) != SPH_OK) return s;
    if (!std::isfinite(exponent)) return fail(ctx, SPH_E_INVALID, "exponent must be finite");
    if (p->n == 0) return SPH_OK;
    if (!rho || !p->xw) return fail(ctx, SPH_E_INVALID, "rho and p->xw are required");
    SPH_HIP(ctx, launch_volume_weights(ctx, *p, rho, exponent));
    return SPH_OK;
}

sph_status sph_gravity_direct(sph_ctx ctx, const sph_particles *p, double eps, double *gx,
                              double *gy, double *gz)
{
    if (!ctx) return fail(nullptr, SPH_E_INVALID, "ctx is NULL");
    sph_status s;
    if ((s = check_particles(ctx, p, false)) != SPH_OK) return s;
    if (!(eps >= 0.0) || !std::isfinite(eps))
        return fail(ctx, SPH_E_INVALID, "eps must be finite and >= 0");
    if (p->n == 0) return SPH_OK;
    if (!gx || !gy || !gz) return fail(ctx, SPH_E_INVALID, "gx, gy and gz are required");
    SPH_HIP(ctx, launch_gravity_direct(ctx, *p, eps, gx, gy, gz));
    return SPH_OK;
}

sph_status sph_gravity_tree(sph_ctx ctx, const sph_particles *p, double eps, double theta,
                            int32_t leaf_size, double *gx, double *gy, double *gz)
{
    if (!ctx) return fail(nullptr, SPH_E_INVALID, "ctx is NULL");
    sph_status s;
    if ((s = check_particles(ctx, p, false)) != SPH_OK) return s;
    if (!(eps >= 0.0) || !std::isfinite(eps))
        return fail(ctx, SPH_E_INVALID, "eps must be finite and >= 0");
    if (!(theta > 0.0) || !std::isfinite(theta))
        return fail(ctx, SPH_E_INVALID, "theta must be finite and > 0");
    if (leaf_size < 8 || leaf_size > 64)
        return fail(ctx, SPH_E_INVALID, "leaf_size %d outside [8, 64]", leaf_size);
    if (p->n == 0) return SPH_OK;
    if (!gx || !gy || !gz) return fail(ctx, SPH_E_INVALID, "gx, gy and gz are required");
    uint32_t flags = 0;
    const hipError_t e = launch_gravity_tree(ctx, *p, eps, theta, leaf_size, gx, gy, gz, &flags);
    if (e == hipErrorOutOfMemory || (e != hipSuccess && ctx->gt_n_cap == 0))
        return fail(ctx, SPH_E_NOMEM, "octree buffers: %s", hipGetErrorString(e));
    SPH_HIP(ctx, e);
    if (flags & 1u) return fail(ctx, SPH_E_CAPACITY, "octree node capacity exceeded");
    if (flags & 2u) return fail(ctx, SPH_E_CAPACITY, "octree traversal stack exceeded");
    return SPH_OK;
}

sph_status sph_eos(sph_ctx ctx, const sph_particles *p, const sph_params *prm,
                   const sph_fields *f)
{
    if (!ctx) return fail(nullptr, SPH_E_INVALID, "ctx is NULL");
    sph_status s;
    if ((s = check_particles(ctx, p, false)) != SPH_OK) return s;
    if ((s = check_params(ctx, prm)) != SPH_OK) return s;
    if (!f) return fail(ctx, SPH_E_INVALID, "fields is NULL");
    if (p->n == 0) return SPH_OK;
    if (!f->rho || !f->p || !f->c || !f->pr2)
        return fail(ctx, SPH_E_INVALID, "rho, p, c and pr2 are required");
    if (prm->eos == SPH_EOS_TAIT && (!p->rho_ref || !p->p_bg))
        return fail(ctx, SPH_E_INVALID, "the Tait EOS needs rho_ref and p_bg");
    if (prm->eos == SPH_EOS_IDEAL && !p->u)
        return fail(ctx, SPH_E_INVALID, "the ideal-gas EOS needs u");
    SPH_HIP(ctx, launch_eos(ctx, *p, *prm, *f));
    return SPH_OK;
}

sph_status sph_momentum_energy(sph_ctx ctx, const sph_particles *p, const sph_box *box,
                               const sph_nbrs *nb, const sph_params *prm,
                               const sph_fields *f, const sph_accel *a)
{
    if (!ctx) return fail(nullptr, SPH_E_INVALID, "ctx is NULL");
    sph_status s;
    if ((s = check_particles(ctx, p, true)) != SPH_OK) return s;
    if ((s = check_box(ctx, box)) != SPH_OK) return s;
    if ((s = check_nbrs(ctx, nb, p->n)) != SPH_OK) return s;
    if ((s = check_params(ctx, prm)) != SPH_OK) return s;
    if (!f || !a) return fail(ctx, SPH_E_INVALID, "fields and accel are required");
    if (ctx->n_built != p->n || !same_box(ctx->grid, *box))
        return fail(ctx, SPH_E_INVALID, "sph_build_cells was not called for these particles/box");
    if (p->n == 0) return SPH_OK;
    if (!f->rho || !f->c || !f->pr2 || !a->ax || !a->ay || !a->az || !a->dudt || !a->mumax)
        return fail(ctx, SPH_E_INVALID, "rho, c, pr2, ax, ay, az, dudt, mumax are required");
    if (prm->volume == SPH_VOLUME_GENERALISED && !p->xw)
        return fail(ctx, SPH_E_INVALID, "generalised volume elements need p->xw");
    SPH_HIP(ctx, launch_momentum(ctx, *p, *nb, *prm, *f, *a));
    return SPH_OK;
}

sph_status sph_integrate(sph_ctx ctx, const sph_particles *p, const sph_box *box,
                         int32_t stage, const double *dt_dev, const sph_accel *a)
{
    if (!ctx) return fail(nullptr, SPH_E_INVALID, "ctx is NULL");
    sph_status s;
    if ((s = check_particles(ctx, p, true)) != SPH_OK) return s;
    if ((s = check_box(ctx, box)) != SPH_OK) return s;
    if (stage != SPH_KICK_DRIFT && stage != SPH_KICK)
        return fail(ctx, SPH_E_INVALID, "unknown stage %d", stage);
    if (!dt_dev || !a) return fail(ctx, SPH_E_INVALID, "dt_dev and accel are required");
    if (p->n == 0) return SPH_OK;
    if (!a->ax || !a->ay || !a->az || !a->dudt)
        return fail(ctx, SPH_E_INVALID, "ax, ay, az, dudt are required");
    SPH_HIP(ctx, launch_integrate(ctx, *p, box_grid(*box), stage, dt_dev, *a));
    return SPH_OK;
}

sph_status sph_timestep(sph_ctx ctx, const sph_particles *p, const sph_params *prm,
                        const sph_fields *f, const sph_accel *a, double *dt_dev,
                        double *diag_dev)
{
    if (!ctx) return fail(nullptr, SPH_E_INVALID, "ctx is NULL");
    sph_status s;
    if ((s = check_particles(ctx, p, true)) != SPH_OK) return s;
    if ((s = check_params(ctx, prm)) != SPH_OK) return s;
    if (!f || !a || !dt_dev) return fail(ctx, SPH_E_INVALID, "fields, accel, dt_dev required");
    if (p->n > 0 && (!f->c || !a->ax || !a->ay || !a->az || !a->mumax))
        return fail(ctx, SPH_E_INVALID, "c, ax, ay, az, mumax are required");
    SPH_HIP(ctx, launch_timestep(ctx, *p, *prm, *f, *a, dt_dev, diag_dev));
    return SPH_OK;
}

sph_status sph_init_forces(sph_ctx ctx, const sph_particles *p, const sph_box *box,
                           double h_max, const sph_nbrs *nb, const sph_params *prm,
                           const sph_fields *f, const sph_accel *a, int32_t set_rho_ref,
                           double *dt_dev, double *diag_dev)
{
    sph_status s;
    if ((s = sph_build_cells(ctx, p, box, h_max)) != SPH_OK) return s;
    if ((s = sph_find_neighbors(ctx, p, box, nb)) != SPH_OK) return s;
    if (!f) return fail(ctx, SPH_E_INVALID, "fields is NULL");
    if ((s = check_params(ctx, prm)) != SPH_OK) return s;
    if (prm->volume == SPH_VOLUME_GENERALISED) {
        // no previous density yet: seed the weights from the standard one
        sph_params std_prm = *prm;
        std_prm.volume = SPH_VOLUME_STANDARD;
        if ((s = sph_density(ctx, p, box, nb, &std_prm, f->rho)) != SPH_OK) return s;
        if ((s = sph_volume_weights(ctx, p, f->rho, prm->volume_p)) != SPH_OK) return s;
    }
    if ((s = sph_density(ctx, p, box, nb, prm, f->rho)) != SPH_OK) return s;
    if (set_rho_ref && p->n > 0) {
        if (!p->rho_ref) return fail(ctx, SPH_E_INVALID, "set_rho_ref needs rho_ref");
        SPH_HIP(ctx, launch_copy(ctx, p->rho_ref, f->rho, p->n));
    }
    if ((s = sph_eos(ctx, p, prm, f)) != SPH_OK) return s;
    if ((s = sph_momentum_energy(ctx, p, box, nb, prm, f, a)) != SPH_OK) return s;
    return sph_timestep(ctx, p, prm, f, a, dt_dev, diag_dev);
}

sph_status sph_step(sph_ctx ctx, const sph_particles *p, const sph_box *box, double h_max,
                    const sph_nbrs *nb, const sph_params *prm, const sph_fields *f,
                    const sph_accel *a, double *dt_dev, double *diag_dev)
{
    sph_status s;
    if (!prm) return fail(ctx, SPH_E_INVALID, "params is NULL");
    if (prm->volume == SPH_VOLUME_GENERALISED) {
        if (!f) return fail(ctx, SPH_E_INVALID, "fields is NULL");
        if ((s = sph_volume_weights(ctx, p, f->rho, prm->volume_p)) != SPH_OK) return s;
    }
    if ((s = sph_integrate(ctx, p, box, SPH_KICK_DRIFT, dt_dev, a)) != SPH_OK) return s;
    if ((s = sph_build_cells(ctx, p, box, h_max)) != SPH_OK) return s;
    if ((s = sph_find_neighbors(ctx, p, box, nb)) != SPH_OK) return s;
    if (!f) return fail(ctx, SPH_E_INVALID, "fields is NULL");
    if ((s = sph_density(ctx, p, box, nb, prm, f->rho)) != SPH_OK) return s;
    if ((s = sph_eos(ctx, p, prm, f)) != SPH_OK) return s;
    if ((s = sph_momentum_energy(ctx, p, box, nb, prm, f, a)) != SPH_OK) return s;
    if ((s = sph_integrate(ctx, p, box, SPH_KICK, dt_dev, a)) != SPH_OK) return s;
    return sph_timestep(ctx, p, prm, f, a, dt_dev, diag_dev);
}

sph_status sph_step_capture(sph_ctx ctx, const sph_particles *p, const sph_box *box,
                            double h_max, const sph_nbrs *nb, const sph_params *prm,
                            const sph_fields *f, const sph_accel *a, double *dt_dev,
                            double *diag_dev)
{
    if (!ctx) return fail(nullptr, SPH_E_INVALID, "ctx is NULL");
    if (ctx->step_exec) {
        (void)hipGraphExecDestroy(ctx->step_exec);
        ctx->step_exec = nullptr;
    }
    if (ctx->step_graph) {
        (void)hipGraphDestroy(ctx->step_graph);
        ctx->step_graph = nullptr;
    }
    // The caller's stream may be the null stream, which cannot be captured:
    // record on a private stream (the launches take ctx->stream) and launch
    // the graph on the caller's stream afterwards.
    hipStream_t cap = nullptr;
    SPH_HIP(ctx, hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
    hipStream_t own = ctx->stream;
    const hipError_t be = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
    if (be != hipSuccess) {
        (void)hipStreamDestroy(cap);
        return hip_fail(ctx, be, "hipStreamBeginCapture");
    }
    ctx->stream = cap;
    ctx->capturing = true;
    const sph_status s = sph_step(ctx, p, box, h_max, nb, prm, f, a, dt_dev, diag_dev);
    ctx->capturing = false;
    ctx->stream = own;
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(cap, &g);
    (void)hipStreamDestroy(cap);
    if (s != SPH_OK || e != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        if (s != SPH_OK) return s;
        return hip_fail(ctx, e, "hipStreamEndCapture");
    }
    ctx->step_graph = g;
    const hipError_t ie = hipGraphInstantiate(&ctx->step_exec, g, nullptr, nullptr, 0);
    if (ie != hipSuccess) {
        ctx->step_exec = nullptr;
        return hip_fail(ctx, ie, "hipGraphInstantiate");
    }
    return SPH_OK;
}

sph_status sph_step_replay(sph_ctx ctx)
{
    if (!ctx) return fail(nullptr, SPH_E_INVALID, "ctx is NULL");
    if (!ctx->step_exec) return fail(ctx, SPH_E_INVALID, "no step was captured");
    SPH_HIP(ctx, hipGraphLaunch(ctx->step_exec, ctx->stream));
    return SPH_OK;
}

sph_status sph_step_blocks(sph_ctx ctx, const sph_particles *p, const sph_box *box,
                           double h_max, const sph_nbrs *nb, const sph_params *prm,
                           const sph_fields *f, const sph_accel *a, int32_t max_bin,
                           double *bin, double *dt_dev, double *diag_dev, int32_t *substeps)
{
    if (!ctx) return fail(nullptr, SPH_E_INVALID, "ctx is NULL");
    sph_status s;
    if ((s = check_particles(ctx, p, true)) != SPH_OK) return s;
    if ((s = check_box(ctx, box)) != SPH_OK) return s;
    if ((s = check_nbrs(ctx, nb, p->n)) != SPH_OK) return s;
    if ((s = check_params(ctx, prm)) != SPH_OK) return s;
    if (max_bin < 0 || max_bin > 16)
        return fail(ctx, SPH_E_INVALID, "max_bin %d outside [0, 16]", max_bin);
    if (!f || !a || !dt_dev || !substeps)
        return fail(ctx, SPH_E_INVALID, "fields, accel, dt_dev and substeps are required");
    *substeps = 0;
    if (p->n == 0) return SPH_OK;
    if (!bin) return fail(ctx, SPH_E_INVALID, "bin is required");
    if (!f->rho || !f->c || !a->ax || !a->ay || !a->az || !a->dudt || !a->mumax)
        return fail(ctx, SPH_E_INVALID, "rho, c, ax, ay, az, dudt, mumax are required");
    if (prm->volume == SPH_VOLUME_GENERALISED && !p->xw)
        return fail(ctx, SPH_E_INVALID, "generalised volume elements need p->xw");
    if (prm->gradient == SPH_GRAD_IAD)
        return fail(ctx, SPH_E_INVALID, "individual time steps do not support IAD");
    if (!f->p || !f->pr2) return fail(ctx, SPH_E_INVALID, "p and pr2 are required");
    if (prm->eos == SPH_EOS_TAIT && (!p->rho_ref || !p->p_bg))
        return fail(ctx, SPH_E_INVALID, "the Tait EOS needs rho_ref and p_bg");
    SPH_HIP(ctx, launch_block_bins(ctx, *p, *prm, *f, *a, max_bin, bin, dt_dev));
    uint32_t words[2] = {0, 0};
    SPH_HIP(ctx, hipMemcpyAsync(words, ctx->blk_words, sizeof words, hipMemcpyDeviceToHost,
                                ctx->stream));
    SPH_HIP(ctx, hipStreamSynchronize(ctx->stream));
    const int B = (int)words[0];
    // the bins, the last accelerations and the last density, pressure and
    // sound speed travel with the particles through every cell sort
    double *extra[10] = {bin, a->ax, a->ay, a->az, a->dudt, a->mumax,
                         f->rho, f->p, f->c, f->pr2};
    const bool gve = prm->volume == SPH_VOLUME_GENERALISED;
    const KernelSel ks = kernel_sel(*prm);
    for (int sub = 0; sub < (1 << B); ++sub) {
        const StepMask mask{bin, sub, B};
        if (gve) SPH_HIP(ctx, launch_volume_weights(ctx, *p, f->rho, prm->volume_p));
        SPH_HIP(ctx, launch_kick_bins(ctx, *p, 0, sub, B, dt_dev, bin, *a));
        SPH_HIP(ctx, launch_drift(ctx, *p, box_grid(*box), B, dt_dev));
        if ((s = build_cells(ctx, p, box, h_max, extra, 10)) != SPH_OK) return s;
        // lists, density and EOS only where a step closes; the others keep theirs
        SPH_HIP(ctx, launch_find_neighbors(ctx, *p, *nb, mask));
        SPH_HIP(ctx, launch_density(ctx, *p, *nb, prm->precision, ks, gve, f->rho, mask));
        SPH_HIP(ctx, launch_eos(ctx, *p, *prm, *f, mask));
        SPH_HIP(ctx, launch_momentum(ctx, *p, *nb, *prm, *f, *a, bin, sub, B));
        SPH_HIP(ctx, launch_kick_bins(ctx, *p, 1, sub, B, dt_dev, bin, *a));
    }
    *substeps = 1 << B;
    // totals of the synchronised end state (the criterion output goes to scratch)
    SPH_HIP(ctx, launch_timestep(ctx, *p, *prm, *f, *a, ctx->dtc, diag_dev));
    return SPH_OK;
}

sph_status sph_smoothing_length(sph_ctx ctx, sph_particles *p, const sph_box *box,
                                double n_target, int32_t lo_count, int32_t hi_count,
                                int32_t max_iter, int32_t *count, int32_t *iterations)
{
    if (!ctx) return fail(nullptr, SPH_E_INVALID, "ctx is NULL");
    sph_status s;
    if ((s = check_particles(ctx, p, false)) != SPH_OK) return s;
    if ((s = check_box(ctx, box)) != SPH_OK) return s;
    if (!(n_target > 0.0) || !std::isfinite(n_target))
        return fail(ctx, SPH_E_INVALID, "n_target must be finite and > 0");
    if (lo_count < 0 || hi_count < lo_count || max_iter < 0)
        return fail(ctx, SPH_E_INVALID, "need 0 <= lo_count <= hi_count and max_iter >= 0");
    if (!iterations || (p->n > 0 && !count))
        return fail(ctx, SPH_E_INVALID, "count and iterations are required");
    *iterations = 0;
    if (p->n == 0) return SPH_OK;
    // The sweeps run on the device on the cells built for the largest h at
    // the start (a particle may grow to 2 h = two cells); the host steps in
    // only when a particle outgrows that reach (rebuild and continue) and
    // once at the end, to rebuild the cells for the final h.
    auto largest_h = [&](double *h_max) -> sph_status {
        unsigned long long hbits = 0;
        hipError_t e = launch_max_h(ctx, *p, ctx->it_hmax);
        if (e == hipSuccess)
            e = hipMemcpyAsync(&hbits, ctx->it_hmax, sizeof hbits, hipMemcpyDeviceToHost,
                               ctx->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
        if (e != hipSuccess) return hip_fail(ctx, e, "largest h");
        std::memcpy(h_max, &hbits, sizeof *h_max);
        if (!(*h_max > 0.0) || !std::isfinite(*h_max))
            return fail(ctx, SPH_E_NONFINITE, "h is not finite and positive");
        for (int a = 0; a < 3; ++a)
            if (box->periodic[a] && !(box->hi[a] - box->lo[a] > 4.0 * *h_max))
                return fail(ctx, SPH_E_DOMAIN, "periodic axis %d is not longer than 4 h_max", a);
        return SPH_OK;
    };
    auto build = [&](double h_max) -> hipError_t {
        ctx->grid = make_grid(*box, h_max, ctx->cell_cap, kMaxAxisCells);
        ctx->n_built = p->n;
        return launch_build_cells(ctx, *p, ctx->grid, h_max);
    };
    double h_max = 0.0;
    sph_status st;
    int32_t sweep = 0;
    uint32_t words[kItWords] = {};
    for (;;) {
        if ((st = largest_h(&h_max)) != SPH_OK) return st;
        hipError_t e = build(h_max);
        if (e == hipSuccess)
            e = launch_h_iteration(ctx, *p, count, lo_count, hi_count, n_target, sweep, max_iter,
                                   ctx->it_words);
        if (e == hipSuccess)
            e = hipMemcpyAsync(words, ctx->it_words, sizeof words, hipMemcpyDeviceToHost,
                               ctx->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
        if (e != hipSuccess) return hip_fail(ctx, e, "smoothing-length sweeps");
        sweep = (int32_t)words[3];
        if (words[2]) break;      // done: the counts of sweep `sweep` are final
        if (!words[4]) return fail(ctx, SPH_E_HIP, "smoothing-length sweeps did not finish");
    }
    *iterations = sweep;
    // cells for the final h (this may reorder the particles, and the cells'
    // largest (2 h)^2 must follow the grown h); the final counts follow the
    // particles through the build's permutation (the h they were counted
    // with is the final one)
    if ((st = largest_h(&h_max)) != SPH_OK) return st;
    SPH_HIP(ctx, build(h_max));
    SPH_HIP(ctx, launch_permute_like_build(ctx, count, p->n));
    return SPH_OK;
}

sph_status sph_export_neighbors(sph_ctx ctx, const sph_particles *p, const sph_nbrs *nb,
                                int64_t *offsets_host, int32_t *ids_host, int64_t cap,
                                int64_t *total)
{
    if (!ctx) return fail(nullptr, SPH_E_INVALID, "ctx is NULL");
    sph_status s;
    if ((s = check_particles(ctx, p, false)) != SPH_OK) return s;
    if ((s = check_nbrs(ctx, nb, p->n)) != SPH_OK) return s;
    if (!offsets_host || !total || (cap > 0 && !ids_host))
        return fail(ctx, SPH_E_INVALID, "offsets_host, ids_host and total are required");
    const int64_t n = p->n;
    offsets_host[0] = 0;
    *total = 0;
    if (n == 0) return SPH_OK;
    SPH_HIP(ctx, hipStreamSynchronize(ctx->stream));
    std::vector<int32_t> count(n), id(n), idx((size_t)nb->max_nb * n);
    SPH_HIP(ctx, hipMemcpy(count.data(), nb->count, sizeof(int32_t) * n, hipMemcpyDeviceToHost));
    SPH_HIP(ctx, hipMemcpy(id.data(), p->id, sizeof(int32_t) * n, hipMemcpyDeviceToHost));
    SPH_HIP(ctx, hipMemcpy(idx.data(), nb->idx, sizeof(int32_t) * idx.size(),
                           hipMemcpyDeviceToHost));
    std::vector<int64_t> slot_of(n, -1);
    for (int64_t i = 0; i < n; ++i) {
        if (id[i] < 0 || id[i] >= n || slot_of[id[i]] >= 0)
            return fail(ctx, SPH_E_INVALID, "ids are not a permutation of 0..n-1");
        slot_of[id[i]] = i;
    }
    for (int64_t k = 0; k < n; ++k)
        offsets_host[k + 1] = offsets_host[k] + std::min(count[slot_of[k]], nb->max_nb);
    *total = offsets_host[n];
    if (*total > cap) return fail(ctx, SPH_E_CAPACITY, "export needs %lld entries", (long long)*total);
    for (int64_t k = 0; k < n; ++k) {
        const int64_t i = slot_of[k];
        const int c = std::min(count[i], nb->max_nb);
        int32_t *dst = ids_host + offsets_host[k];
        for (int t = 0; t < c; ++t) dst[t] = id[idx[(size_t)t * n + i]];
        std::sort(dst, dst + c);
    }
    return SPH_OK;
}

}  // extern "C"
