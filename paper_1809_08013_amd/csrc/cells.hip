// Algorithm 1, step 1 on the GPU: cell assignment, Morton keys, stable LSD
// radix sort, in-place reorder of the particle arrays and the cell table.
//
// The paper's parent codes build an octree here (Sec. 5.2.5, phase A). A
// uniform grid of cells of side >= 2 h_max sorted along a Morton curve gives
// the same exact candidate set for a fixed-radius search and keeps the
// particles of a cell, and of neighbouring cells, contiguous in memory.
#include <algorithm>

#include "sph_internal.h"

namespace sph {
namespace {

__device__ __forceinline__ uint32_t spread3(uint32_t v)
{
    v &= 0x3ffu;
    v = (v | (v << 16)) & 0x030000FFu;
    v = (v | (v << 8)) & 0x0300F00Fu;
    v = (v | (v << 4)) & 0x030C30C3u;
    v = (v | (v << 2)) & 0x09249249u;
    return v;
}

__device__ __forceinline__ uint32_t compact3(uint32_t v)
{
    v &= 0x09249249u;
    v = (v | (v >> 2)) & 0x030C30C3u;
    v = (v | (v >> 4)) & 0x0300F00Fu;
    v = (v | (v >> 8)) & 0x030000FFu;
    v = (v | (v >> 16)) & 0x000003FFu;
    return v;
}

__device__ __forceinline__ int cell_of(double v, double lo, double inv_s, int nc)
{
    double f = floor((v - lo) * inv_s);
    f = fmin(fmax(f, 0.0), (double)(nc - 1));
    return (int)f;
}

// z slice of a point in its cell (zbits bits): the fractional part of its
// cell coordinate, scaled by 2^zbits, with points outside the box clamped
// to the first or last slice.
__device__ __forceinline__ uint32_t slice_of(double v, double lo, double inv_s, int cz, int zbits)
{
    const double f = (v - lo) * inv_s;
    double q = floor((f - (double)cz) * (double)(1 << zbits));
    q = fmin(fmax(q, 0.0), (double)((1 << zbits) - 1));
    return (uint32_t)q;
}

__global__ void clear_word_kernel(uint32_t *w) { *w = 0u; }

// Sort key of each particle: the Morton key of its cell, then its z slice in
// the cell; vals = current index. Flags h > h_max, and sets *hflag when some
// h differs from h[0] (one atomic per wave: with variable h, one per
// particle on the same word serialised the kernel, 168 us at 1M).
__global__ void __launch_bounds__(256)
keys_kernel(int64_t n, const double *__restrict__ x, const double *__restrict__ y,
            const double *__restrict__ z, const double *__restrict__ h, Grid g,
            double h_max, uint32_t *__restrict__ keys, int32_t *__restrict__ vals,
            uint32_t *hflag, uint32_t *status)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool active = i < n;
    const double hi = active ? h[i] : 0.0;
    // One flag update per block at most, and none once the flag is set: an
    // atomic from every wave to the one word serialises in its L2 channel
    // (~10 ns each, 150 us over 10^6 particles of varying h).
    const int differs = __syncthreads_or(active && hi != h[0]);
    const int above = __syncthreads_or(active && !(hi <= h_max));
    if (threadIdx.x == 0) {
        if (differs && __hip_atomic_load(hflag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0u)
            atomicOr(hflag, 1u);
        if (above) atomicOr(status, ST_DOMAIN);
    }
    if (!active) return;
    uint32_t cx = (uint32_t)cell_of(x[i], g.lo[0], g.inv_s[0], g.nc[0]);
    uint32_t cy = (uint32_t)cell_of(y[i], g.lo[1], g.inv_s[1], g.nc[1]);
    uint32_t cz = (uint32_t)cell_of(z[i], g.lo[2], g.inv_s[2], g.nc[2]);
    const uint32_t zq = slice_of(z[i], g.lo[2], g.inv_s[2], (int)cz, g.zbits);
    keys[i] = ((spread3(cx) | (spread3(cy) << 1) | (spread3(cz) << 2)) << g.zbits) | zq;
    vals[i] = (int32_t)i;
}

// Per-tile digit histogram, digit-major layout hist[d * ntiles + tile].
__global__ void __launch_bounds__(kSortThreads)
radix_hist_kernel(const uint32_t *__restrict__ keys, int64_t n, const int64_t *n_dev, int shift,
                  uint32_t *__restrict__ hist, int64_t ntiles)
{
    __shared__ uint32_t cnt[kRadixBins];
    if (n_dev) n = *n_dev;
    cnt[threadIdx.x] = 0;
    __syncthreads();
    int64_t base = (int64_t)blockIdx.x * kSortTile;
#pragma unroll
    for (int it = 0; it < kSortItems; ++it) {
        int64_t i = base + it * kSortThreads + threadIdx.x;
        if (i < n) atomicAdd(&cnt[(keys[i] >> shift) & (kRadixBins - 1)], 1u);
    }
    __syncthreads();
    hist[(int64_t)threadIdx.x * ntiles + blockIdx.x] = cnt[threadIdx.x];
}

// Block-wide exclusive scan of one value per thread (256 threads, wave64).
__device__ __forceinline__ uint32_t block_exclusive_scan(uint32_t v, uint32_t *total,
                                                         uint32_t *lds /*[4]*/)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    uint32_t incl = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        uint32_t t = __shfl_up(incl, o, 64);
        if (lane >= o) incl += t;
    }
    if (lane == 63) lds[wave] = incl;
    __syncthreads();
    uint32_t before = 0, all = 0;
#pragma unroll
    for (int w = 0; w < kScanThreads / 64; ++w) {
        uint32_t s = lds[w];
        if (w < wave) before += s;
        all += s;
    }
    __syncthreads();
    *total = all;
    return before + incl - v;
}

// Scan phase 1: per-chunk sums.
__global__ void __launch_bounds__(kScanThreads)
scan_reduce_kernel(const uint32_t *__restrict__ a, int64_t len,
                   uint32_t *__restrict__ part)
{
    __shared__ uint32_t lds[4];
    int64_t base = (int64_t)blockIdx.x * kScanChunk + (int64_t)threadIdx.x * kScanItems;
    uint32_t s = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k)
        if (base + k < len) s += a[base + k];
    uint32_t total;
    block_exclusive_scan(s, &total, lds);
    if (threadIdx.x == 0) part[blockIdx.x] = total;
}

// Scan phase 2: exclusive scan of the chunk sums in one block.
__global__ void __launch_bounds__(kScanThreads)
scan_partials_kernel(uint32_t *__restrict__ part, int64_t nparts)
{
    __shared__ uint32_t lds[4];
    uint32_t carry = 0;
    for (int64_t base = 0; base < nparts; base += kScanThreads) {
        int64_t i = base + threadIdx.x;
        uint32_t v = i < nparts ? part[i] : 0u;
        uint32_t total;
        uint32_t ex = block_exclusive_scan(v, &total, lds);
        if (i < nparts) part[i] = carry + ex;
        carry += total;
    }
}

// Scan phase 3: exclusive scan inside each chunk plus the chunk offset.
__global__ void __launch_bounds__(kScanThreads)
scan_down_kernel(uint32_t *__restrict__ a, int64_t len,
                 const uint32_t *__restrict__ part)
{
    __shared__ uint32_t lds[4];
    int64_t base = (int64_t)blockIdx.x * kScanChunk + (int64_t)threadIdx.x * kScanItems;
    uint32_t v[kScanItems];
    uint32_t s = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        v[k] = (base + k < len) ? a[base + k] : 0u;
        s += v[k];
    }
    uint32_t total;
    uint32_t run = block_exclusive_scan(s, &total, lds) + part[blockIdx.x];
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        if (base + k < len) a[base + k] = run;
        run += v[k];
    }
}

// Stable scatter of one radix pass. Elements of a tile are ranked in index
// order: sub-tile by sub-tile, wave by wave, lane by lane. Lanes holding the
// same digit are matched with one ballot per digit bit.
__global__ void __launch_bounds__(kSortThreads)
radix_scatter_kernel(const uint32_t *__restrict__ kin, const int32_t *__restrict__ vin,
                     int64_t n, const int64_t *n_dev, int shift,
                     const uint32_t *__restrict__ hist, int64_t ntiles,
                     uint32_t *__restrict__ kout, int32_t *__restrict__ vout)
{
    if (n_dev) n = *n_dev;
    if ((int64_t)blockIdx.x * kSortTile >= n) return;
    constexpr int kWaves = kSortThreads / 64;
    __shared__ uint32_t base_of[kRadixBins];
    __shared__ uint32_t run[kRadixBins];
    __shared__ uint32_t wcnt[kWaves][kRadixBins];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    base_of[tid] = hist[(int64_t)tid * ntiles + blockIdx.x];
    run[tid] = 0;
#pragma unroll
    for (int w = 0; w < kWaves; ++w) wcnt[w][tid] = 0;
    __syncthreads();
    const uint64_t lt_mask = lane == 0 ? 0ull : (~0ull >> (64 - lane));
    const int64_t tile0 = (int64_t)blockIdx.x * kSortTile;
    for (int it = 0; it < kSortItems; ++it) {
        const int64_t i = tile0 + it * kSortThreads + tid;
        const bool valid = i < n;
        const uint32_t k = valid ? kin[i] : 0u;
        const int32_t v = valid ? vin[i] : 0;
        const uint32_t d = (k >> shift) & (kRadixBins - 1);
        uint64_t same = __ballot(valid);
#pragma unroll
        for (int b = 0; b < kRadixBits; ++b) {
            const bool bit = (d >> b) & 1u;
            const uint64_t ones = __ballot(bit);
            same &= bit ? ones : ~ones;
        }
        const uint32_t rank = __popcll(same & lt_mask);
        if (valid && rank == 0) wcnt[wave][d] = __popcll(same);
        __syncthreads();
        if (valid) {
            uint32_t off = run[d];
            for (int w = 0; w < wave; ++w) off += wcnt[w][d];
            const uint32_t pos = base_of[d] + off + rank;
            kout[pos] = k;
            vout[pos] = v;
        }
        __syncthreads();
        uint32_t tot = 0;
#pragma unroll
        for (int w = 0; w < kWaves; ++w) {
            tot += wcnt[w][tid];
            wcnt[w][tid] = 0;
        }
        run[tid] += tot;
        __syncthreads();
    }
}

// Gather every particle array into scratch in sorted order.
__global__ void __launch_bounds__(256)
permute_gather_kernel(int64_t n, const int64_t *n_dev, int64_t stride,
                      const int32_t *__restrict__ perm, PermFields f,
                      double *__restrict__ tmp, int32_t *__restrict__ tmp_id,
                      int32_t *__restrict__ tmp_slot)
{
    if (n_dev) n = *n_dev;
    const int64_t step = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += step) {
        const int64_t j = perm[i];
        for (int k = 0; k < f.nf; ++k) tmp[k * stride + i] = f.f[k][j];
        tmp_id[i] = f.id[j];
        if (f.slot) tmp_slot[i] = f.slot[j];
    }
}

// Copy the sorted arrays back into the caller's storage and write the
// search records (position and (2h)^2). Fields 0..2 are x, y, z (always
// present).
__global__ void __launch_bounds__(256)
permute_store_kernel(int64_t n, const int64_t *n_dev, int64_t stride, PermFields f,
                     const double *__restrict__ tmp, const int32_t *__restrict__ tmp_id,
                     const int32_t *__restrict__ tmp_slot, int h_field,
                     SearchRec *__restrict__ srec)
{
    if (n_dev) n = *n_dev;
    const int64_t step = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += step) {
        for (int k = 0; k < f.nf; ++k) f.f[k][i] = tmp[k * stride + i];
        f.id[i] = tmp_id[i];
        if (f.slot) f.slot[i] = tmp_slot[i];
        const double x = tmp[i], y = tmp[stride + i], z = tmp[2 * stride + i];
        const double s = 2.0 * tmp[h_field * stride + i];
        srec[i] = SearchRec{x, y, z, s * s};
    }
}

// Cell table by binary search of each cell's key range (all its slices) in
// the sorted keys: every entry is rewritten on every build, empty cells get
// start == end. Also clears the cell's largest (2h)^2.
__global__ void __launch_bounds__(256)
cell_table_kernel(int64_t ncell, Grid g, const uint32_t *__restrict__ keys, int64_t n,
                  int32_t *__restrict__ cstart, int32_t *__restrict__ cend,
                  unsigned long long *__restrict__ s2max)
{
    int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= ncell) return;
    const uint32_t cx = (uint32_t)(c % g.nc[0]);
    const uint32_t cy = (uint32_t)((c / g.nc[0]) % g.nc[1]);
    const uint32_t cz = (uint32_t)(c / ((int64_t)g.nc[0] * g.nc[1]));
    const uint32_t key = (spread3(cx) | (spread3(cy) << 1) | (spread3(cz) << 2)) << g.zbits;
    const uint32_t last = key | ((1u << g.zbits) - 1u);
    int64_t lo = 0, hi = n;
    while (lo < hi) {   // first index with keys[i] >= key
        int64_t mid = (lo + hi) >> 1;
        if (keys[mid] < key) lo = mid + 1; else hi = mid;
    }
    const int64_t s = lo;
    hi = n;
    while (lo < hi) {   // first index with keys[i] > last
        int64_t mid = (lo + hi) >> 1;
        if (keys[mid] <= last) lo = mid + 1; else hi = mid;
    }
    cstart[c] = (int32_t)s;
    cend[c] = (int32_t)lo;
    s2max[c] = 0ull;
}

// Largest (2h)^2 of each cell, as the ordered bit pattern of a positive
// double: a segmented maximum over the wave's lanes (a cell's particles are
// consecutive), then one atomic per cell and wave.
__global__ void __launch_bounds__(256)
cell_s2max_kernel(int64_t n, Grid g, const uint32_t *__restrict__ keys,
                  const SearchRec *__restrict__ srec, unsigned long long *__restrict__ s2max)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int lane = threadIdx.x & 63;
    const bool active = i < n;
    const uint32_t ck = active ? keys[i] >> g.zbits : 0xFFFFFFFFu;
    unsigned long long v = active ? (unsigned long long)__double_as_longlong(srec[i].s2) : 0ull;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const unsigned long long t = __shfl_down(v, o, 64);
        const uint32_t tk = __shfl_down(ck, o, 64);
        if (lane + o < 64 && tk == ck) v = t > v ? t : v;
    }
    const uint32_t pk = __shfl_up(ck, 1, 64);
    if (active && (lane == 0 || pk != ck)) {
        const int64_t cell = ((int64_t)compact3(ck >> 2) * g.nc[1] + compact3(ck >> 1)) * g.nc[0] +
                             compact3(ck);
        atomicMax(&s2max[cell], v);
    }
}

// ---------------------------------------------------------------------------
// Ensemble kernels: the same cell assignment and table per run, with the
// run's slot in the high key bits. Counts come from the step header, so one
// captured launch sequence serves every batch composition.

// Runs admitted before this step: tag their particles with the slot and
// clear the slot's status word.
__global__ void __launch_bounds__(256)
admit_kernel(BatchDev b)
{
    const BatchHdr *hd = b.hdr;
    const int64_t step = (int64_t)gridDim.x * blockDim.x;
    const int64_t t0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (int r = 0; r < hd->nnew; ++r) {
        const int s = hd->new_slot[r];
        const int64_t off = hd->new_off[r], nr = hd->new_n[r];
        for (int64_t i = t0; i < nr; i += step) b.slot[off + i] = s;
        if (t0 == 0) b.status[s] = 0u;
    }
}

__global__ void __launch_bounds__(256)
keys_batch_kernel(BatchDev b, const double *__restrict__ x, const double *__restrict__ y,
                  const double *__restrict__ z, const double *__restrict__ h,
                  uint32_t *__restrict__ keys, int32_t *__restrict__ vals)
{
    const int64_t n = b.hdr->n_in;
    const int64_t step = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += step) {
        const int s = b.slot[i];
        const RunDev &r = b.runs[s];
        uint32_t key = kEnsDropKey;
        if (r.phase == RUN_INIT || r.phase == RUN_STEP) {
            const Grid &g = r.grid;
            const uint32_t cx = (uint32_t)cell_of(x[i], g.lo[0], g.inv_s[0], g.nc[0]);
            const uint32_t cy = (uint32_t)cell_of(y[i], g.lo[1], g.inv_s[1], g.nc[1]);
            const uint32_t cz = (uint32_t)cell_of(z[i], g.lo[2], g.inv_s[2], g.nc[2]);
            const uint32_t zq = slice_of(z[i], g.lo[2], g.inv_s[2], (int)cz, g.zbits);
            key = ((uint32_t)s << kEnsSlotShift) |
                  ((spread3(cx) | (spread3(cy) << 1) | (spread3(cz) << 2)) << kSliceBits) |
                  (zq << (kSliceBits - g.zbits));
            if (!(h[i] <= r.h_max)) atomicOr(&b.status[s], ST_DOMAIN);
        }
        keys[i] = key;
        vals[i] = (int32_t)i;
    }
}

// Cell table of every live run: global cell c belongs to the live run whose
// cell range holds it; its particles are found by binary search inside the
// run's sorted range.
__global__ void __launch_bounds__(256)
cell_table_batch_kernel(BatchDev b, const uint32_t *__restrict__ keys,
                        int32_t *__restrict__ cstart, int32_t *__restrict__ cend)
{
    const BatchHdr *hd = b.hdr;
    const int64_t ncell = hd->ncell;
    const int nlive = hd->nlive;
    const int64_t step = (int64_t)gridDim.x * blockDim.x;
    for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < ncell; c += step) {
        int lo = 0, hi = nlive - 1;
        while (lo < hi) {  // last live run with cell_base <= c
            const int mid = (lo + hi + 1) >> 1;
            if (hd->live_cell_base[mid] <= c) lo = mid; else hi = mid - 1;
        }
        const int s = hd->live_slot[lo];
        const RunDev &r = b.runs[s];
        const Grid &g = r.grid;
        const int64_t lc = c - r.cell_base;
        const uint32_t cx = (uint32_t)(lc % g.nc[0]);
        const uint32_t cy = (uint32_t)((lc / g.nc[0]) % g.nc[1]);
        const uint32_t cz = (uint32_t)(lc / ((int64_t)g.nc[0] * g.nc[1]));
        const uint32_t key = ((uint32_t)s << kEnsSlotShift) |
                             ((spread3(cx) | (spread3(cy) << 1) | (spread3(cz) << 2)) << kSliceBits);
        const uint32_t last = key | ((1u << kSliceBits) - 1u);
        int64_t a = r.start, e = (int64_t)r.start + r.n;
        while (a < e) {
            const int64_t mid = (a + e) >> 1;
            if (keys[mid] < key) a = mid + 1; else e = mid;
        }
        const int64_t first = a;
        e = (int64_t)r.start + r.n;
        while (a < e) {
            const int64_t mid = (a + e) >> 1;
            if (keys[mid] <= last) a = mid + 1; else e = mid;
        }
        cstart[c] = (int32_t)first;
        cend[c] = (int32_t)a;
    }
}

inline unsigned blocks_for(int64_t n, int t) { return (unsigned)((n + t - 1) / t); }

hipError_t exclusive_scan(sph_ctx ctx, uint32_t *a, int64_t len)
{
    const int64_t nparts = (len + kScanChunk - 1) / kScanChunk;
    scan_reduce_kernel<<<(unsigned)nparts, kScanThreads, 0, ctx->stream>>>(a, len, ctx->scan_part);
    scan_partials_kernel<<<1, kScanThreads, 0, ctx->stream>>>(ctx->scan_part, nparts);
    scan_down_kernel<<<(unsigned)nparts, kScanThreads, 0, ctx->stream>>>(a, len, ctx->scan_part);
    return hipGetLastError();
}

}  // namespace

hipError_t radix_sort_pairs(sph_ctx ctx, uint32_t *k[2], int32_t *v[2], int64_t n,
                            int key_bits, int *cur)
{
    hipStream_t s = ctx->stream;
    const int64_t ntiles = (n + kSortTile - 1) / kSortTile;
    hipError_t e;
    for (int shift = 0; shift < key_bits; shift += kRadixBits) {
        radix_hist_kernel<<<(unsigned)ntiles, kSortThreads, 0, s>>>(k[*cur], n, nullptr, shift,
                                                                     ctx->hist, ntiles);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        if ((e = exclusive_scan(ctx, ctx->hist, ntiles * kRadixBins)) != hipSuccess) return e;
        radix_scatter_kernel<<<(unsigned)ntiles, kSortThreads, 0, s>>>(
            k[*cur], v[*cur], n, nullptr, shift, ctx->hist, ntiles, k[*cur ^ 1], v[*cur ^ 1]);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        *cur ^= 1;
    }
    return hipSuccess;
}

hipError_t launch_build_cells(sph_ctx ctx, const sph_particles &p, const Grid &g,
                              double h_max, double *const *extra, int n_extra)
{
    const int64_t n = p.n;
    hipStream_t s = ctx->stream;
    const int64_t ncell = (int64_t)g.nc[0] * g.nc[1] * g.nc[2];
    clear_word_kernel<<<1, 1, 0, s>>>(ctx->hflag_dev);
    keys_kernel<<<blocks_for(n, 256), 256, 0, s>>>(n, p.x, p.y, p.z, p.h, g, h_max,
                                                   ctx->keys[0], ctx->vals[0], ctx->hflag_dev,
                                                   ctx->status_dev);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int key_bits = 3 * g.bits + g.zbits;
    const int64_t ntiles = (n + kSortTile - 1) / kSortTile;
    int cur = 0;
    for (int shift = 0; shift < key_bits; shift += kRadixBits) {
        radix_hist_kernel<<<(unsigned)ntiles, kSortThreads, 0, s>>>(
            ctx->keys[cur], n, nullptr, shift, ctx->hist, ntiles);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        if ((e = exclusive_scan(ctx, ctx->hist, ntiles * kRadixBins)) != hipSuccess) return e;
        radix_scatter_kernel<<<(unsigned)ntiles, kSortThreads, 0, s>>>(
            ctx->keys[cur], ctx->vals[cur], n, nullptr, shift, ctx->hist, ntiles,
            ctx->keys[cur ^ 1], ctx->vals[cur ^ 1]);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        cur ^= 1;
    }
    ctx->sorted_keys = ctx->keys[cur];

    PermFields f{};
    double *fields[kPermFields] = {p.x, p.y, p.z, p.vx, p.vy, p.vz, p.u, p.h, p.m,
                                   p.rho_ref, p.p_bg, p.gx, p.gy, p.gz, p.xw};
    for (int k = 0; k < n_extra && 15 + k < kPermFields; ++k) fields[15 + k] = extra[k];
    int h_field = -1;
    for (int k = 0; k < kPermFields; ++k) {
        if (!fields[k]) continue;
        if (k == 7) h_field = f.nf;
        f.f[f.nf++] = fields[k];
    }
    f.id = p.id;
    permute_gather_kernel<<<blocks_for(n, 256), 256, 0, s>>>(n, nullptr, ctx->n_max,
                                                             ctx->vals[cur], f, ctx->perm_tmp,
                                                             ctx->perm_tmp_id, nullptr);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    permute_store_kernel<<<blocks_for(n, 256), 256, 0, s>>>(n, nullptr, ctx->n_max, f,
                                                            ctx->perm_tmp, ctx->perm_tmp_id,
                                                            nullptr, h_field, ctx->srec);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    unsigned long long *s2max = reinterpret_cast<unsigned long long *>(ctx->cell_s2max);
    cell_table_kernel<<<blocks_for(ncell, 256), 256, 0, s>>>(ncell, g, ctx->sorted_keys, n,
                                                             ctx->cell_start, ctx->cell_end, s2max);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    cell_s2max_kernel<<<blocks_for(n, 256), 256, 0, s>>>(n, g, ctx->sorted_keys, ctx->srec, s2max);
    return hipGetLastError();
}

__global__ void __launch_bounds__(256)
gather_i32_kernel(int64_t n, const int32_t *__restrict__ perm, const int32_t *__restrict__ src,
                  int32_t *__restrict__ dst)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = src[perm[i]];
}

__global__ void __launch_bounds__(256)
copy_i32_kernel(int64_t n, const int32_t *__restrict__ src, int32_t *__restrict__ dst)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = src[i];
}

hipError_t launch_permute_like_build(sph_ctx ctx, int32_t *a, int64_t n)
{
    // the sort's values are the particles' indices before the build, in
    // sorted order, next to the sorted keys
    const int32_t *perm = ctx->sorted_keys == ctx->keys[0] ? ctx->vals[0] : ctx->vals[1];
    gather_i32_kernel<<<blocks_for(n, 256), 256, 0, ctx->stream>>>(n, perm, a, ctx->perm_tmp_id);
    copy_i32_kernel<<<blocks_for(n, 256), 256, 0, ctx->stream>>>(n, ctx->perm_tmp_id, a);
    return hipGetLastError();
}

hipError_t launch_admit_batch(sph_ctx ctx, const BatchDev &b)
{
    admit_kernel<<<256, 256, 0, ctx->stream>>>(b);
    return hipGetLastError();
}

hipError_t launch_build_cells_batch(sph_ctx ctx, const BatchDev &b, double *F, int32_t *id,
                                    int32_t *slot_tmp)
{
    hipStream_t s = ctx->stream;
    const int64_t cap = b.cap;
    const unsigned grid = std::min<unsigned>(blocks_for(cap, 256), 4096u);
    const int64_t *n_in = &b.hdr->n_in;
    keys_batch_kernel<<<grid, 256, 0, s>>>(b, F + 0 * cap, F + 1 * cap, F + 2 * cap,
                                           F + 7 * cap, ctx->keys[0], ctx->vals[0]);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int64_t ntiles = (cap + kSortTile - 1) / kSortTile;
    int cur = 0;
    for (int shift = 0; shift < kEnsKeyBits; shift += kRadixBits) {
        radix_hist_kernel<<<(unsigned)ntiles, kSortThreads, 0, s>>>(
            ctx->keys[cur], cap, n_in, shift, ctx->hist, ntiles);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        if ((e = exclusive_scan(ctx, ctx->hist, ntiles * kRadixBins)) != hipSuccess) return e;
        radix_scatter_kernel<<<(unsigned)ntiles, kSortThreads, 0, s>>>(
            ctx->keys[cur], ctx->vals[cur], cap, n_in, shift, ctx->hist, ntiles,
            ctx->keys[cur ^ 1], ctx->vals[cur ^ 1]);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        cur ^= 1;
    }
    ctx->sorted_keys = ctx->keys[cur];
    PermFields f{};
    for (int k = 0; k < kEnsFields; ++k) f.f[f.nf++] = F + k * cap;
    f.id = id;
    f.slot = b.slot;
    permute_gather_kernel<<<grid, 256, 0, s>>>(cap, n_in, ctx->n_max, ctx->vals[cur], f,
                                               ctx->perm_tmp, ctx->perm_tmp_id, slot_tmp);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    permute_store_kernel<<<grid, 256, 0, s>>>(cap, n_in, ctx->n_max, f, ctx->perm_tmp,
                                              ctx->perm_tmp_id, slot_tmp, 7, ctx->srec);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    const unsigned cgrid = std::min<unsigned>(blocks_for(b.cell_cap, 256), 4096u);
    cell_table_batch_kernel<<<cgrid, 256, 0, s>>>(b, ctx->sorted_keys, ctx->cell_start,
                                                  ctx->cell_end);
    return hipGetLastError();
}

}  // namespace sph
