// Algorithm 1, step 2 on the GPU: the neighbour search.
//
// One wavefront per block of 64 consecutive particles (cell order). The
// wave first builds, in LDS, the union of the 27-cell stencils of the cells
// its particles live in: the non-empty cells, sorted by their first particle
// and without duplicates, so walking them visits candidates in ascending
// index order. It then streams that union wave-uniformly: each candidate's
// record is one scalar load into SGPRs, every lane tests it against its own
// particle with the exact FP64 relation, and the outcome goes into a per-lane
// bit mask (one bit per union position, kept in a global scratch region so
// that the wave's LDS footprint stays small and occupancy high; each 32-bit
// word of 64 lanes is one 256-byte store). A second phase expands the
// masks row by row, so that all lanes write row k of the ELL list together
// (one contiguous 256-byte store per row) instead of scattering 4-byte
// writes.
//
// A wave whose union does not fit (many distinct cells, or more candidates
// than the mask holds) takes the per-lane path instead: each lane walks its
// own stencil and writes its entries directly. Both paths produce the same
// set in the same (ascending) order, so the sums over a list do not depend on
// the path or on where the wave boundaries fall.
#include <algorithm>
#include <climits>

#include "sph_internal.h"

namespace sph {
namespace {

constexpr int kWave = 64;
constexpr int kMaxEntries = 128;        // 27 * distinct cells, before dedup
constexpr int kMaxCandidates = kSearchMaskWords * 32;
constexpr int kMaxWords = kSearchMaskWords;

__device__ __forceinline__ uint32_t compact3(uint32_t v)
{
    v &= 0x09249249u;
    v = (v | (v >> 2)) & 0x030C30C3u;
    v = (v | (v >> 4)) & 0x0300F00Fu;
    v = (v | (v >> 8)) & 0x030000FFu;
    v = (v | (v >> 16)) & 0x000003FFu;
    return v;
}

// Minimum image as a select chain: identical results to
// "if (d > half) d -= len; else if (d < -half) d += len;".
__device__ __forceinline__ double min_image_sel(double d, double len, double half)
{
    d = d > half ? d - len : d;
    return d < -half ? d + len : d;
}

__device__ __forceinline__ int wrap_or_clip(int c, int nc, int periodic, bool &ok)
{
    if (periodic) {
        ok = true;
        return c < 0 ? c + nc : (c >= nc ? c - nc : c);
    }
    ok = c >= 0 && c < nc;
    return c;
}

// Mode of the relation test. Any: r2 < (2h_i)^2 or r2 < (2h_j)^2, i.e.
// r2 < (2 max(h_i, h_j))^2. Uniform: every particle has the same h, so the
// test is one compare against the lane's own (2h)^2.
template <bool Wrap, bool UniformH>
__device__ __forceinline__ bool related(const SearchRec &me, const SearchRec &o, const Grid &g)
{
    double dx = me.x - o.x, dy = me.y - o.y, dz = me.z - o.z;
    if (Wrap) {
        if (g.periodic[0]) dx = min_image_sel(dx, g.len[0], g.half[0]);
        if (g.periodic[1]) dy = min_image_sel(dy, g.len[1], g.half[1]);
        if (g.periodic[2]) dz = min_image_sel(dz, g.len[2], g.half[2]);
    }
    const double r2 = __builtin_fma(dz, dz, __builtin_fma(dy, dy, dx * dx));
    if (UniformH) return r2 < me.s2;
    return (r2 < me.s2) | (r2 < o.s2);
}

// Stream the union (cells[0..nu)) and record, for each candidate u, whether
// it is related to the lane's particle. Masks are 32-bit words bm[word][lane]
// (word = u / 32) filled from the top: candidate u sits at bit 31 - u % 32.
// Within a cell the next four records are loaded while the current four are
// tested, so the scalar-load latency is overlapped with work.
template <bool Wrap, bool UniformH>
__device__ __forceinline__ void stream_union(const SearchRec &me, const SearchRec *__restrict__ srec,
                                             const int2 *cells, int nu, const Grid &g,
                                             uint32_t *__restrict__ bm, int lane, int &cnt,
                                             uint64_t &occ)
{
    uint32_t acc = 0;
    int u = 0;
    auto flush = [&](int w, uint32_t word) {
        bm[w * kWave + lane] = word;
        cnt += __popc(word);
        occ |= word ? (1ull << w) : 0ull;
    };
    auto step = [&](const SearchRec &o) {
        acc = (acc << 1) | (related<Wrap, UniformH>(me, o, g) ? 1u : 0u);
        ++u;
        if ((u & 31) == 0) {
            flush((u >> 5) - 1, acc);
            acc = 0;
        }
    };
    for (int c = 0; c < nu; ++c) {
        const int s = __builtin_amdgcn_readfirstlane(cells[c].x);
        const int e = __builtin_amdgcn_readfirstlane(cells[c].y);
        int j = s;
        if (e - j >= 4) {
            SearchRec a0 = srec[j], a1 = srec[j + 1], a2 = srec[j + 2], a3 = srec[j + 3];
            j += 4;
            while (e - j >= 4) {
                const SearchRec b0 = srec[j], b1 = srec[j + 1], b2 = srec[j + 2],
                                b3 = srec[j + 3];
                step(a0);
                step(a1);
                step(a2);
                step(a3);
                // keep the wait for b0..b3 (scalar loads complete out of order,
                // so it is a full wait) after the work on a0..a3
                __builtin_amdgcn_sched_barrier(0);
                a0 = b0;
                a1 = b1;
                a2 = b2;
                a3 = b3;
                j += 4;
            }
            step(a0);
            step(a1);
            step(a2);
            step(a3);
        }
        for (; j < e; ++j) step(srec[j]);
    }
    if (u & 31) flush(u >> 5, acc << (32 - (u & 31)));
}

struct SearchLds {
    uint32_t dkeys[kWave];
    int2 ent[kMaxEntries];
    int2 cells[kMaxEntries];
    int u0[kMaxEntries + 1];
};

// One tile of 64 particles. Multi: the particles belong to runs of an
// ensemble (slot in the high key bits); a tile whose particles are all of one
// run uses that run's grid and cell range, a tile spanning two runs takes the
// per-lane path with each lane's own run.
template <bool Multi>
__device__ __forceinline__ void search_tile(
    int64_t tile, int64_t n, int64_t ld, const SearchRec *__restrict__ srec,
    const uint32_t *__restrict__ keys, const int32_t *__restrict__ cstart,
    const int32_t *__restrict__ cend, const Grid &g0, int max_nb, int32_t *__restrict__ count,
    int32_t *__restrict__ idx, uint32_t *__restrict__ mask_scratch,
    const uint32_t *__restrict__ hflag, uint32_t *status0, const BatchDev &b, SearchLds &L)
{
    uint32_t *dkeys = L.dkeys;
    int2 *ent = L.ent;
    int2 *cells = L.cells;
    int *u0 = L.u0;

    const int lane = threadIdx.x;
    const int64_t t0 = tile * kWave;
    uint32_t *bm = mask_scratch + tile * (kMaxWords * kWave);
    const int64_t i = t0 + lane;
    const bool active = i < n;
    const uint64_t lt = lane == 0 ? 0ull : (~0ull >> (64 - lane));

    const uint32_t key = active ? keys[i] : 0xFFFFFFFFu;
    const SearchRec me = active ? srec[i] : SearchRec{0.0, 0.0, 0.0, 0.0};
    // run of the tile (lane 0 is always active) and whether all lanes share it
    int my_slot = 0, slot0 = 0;
    bool mixed = false;
    if constexpr (Multi) {
        my_slot = active ? (int)(key >> (3 * kEnsAxisBits)) : 0;
        slot0 = __builtin_amdgcn_readfirstlane(my_slot);
        mixed = __ballot(active && my_slot != slot0) != 0ull;
    }
    const Grid &g = Multi ? b.runs[slot0].grid : g0;
    const int64_t cbase = Multi ? (int64_t)b.runs[slot0].cell_base : 0;
    const uint32_t mkey = Multi ? (key & kEnsMortonMask) : key;
    const uint32_t prev = __shfl_up(key, 1, kWave);
    const bool first = active && (lane == 0 || key != prev);
    const uint64_t fm = __ballot(first);
    const int ndist = __popcll(fm);
    if (first) dkeys[__popcll(fm & lt)] = mkey;

    // The minimum image can be skipped for the whole wave when, on every
    // periodic axis, the union of the stencils spans less than half the box:
    // then |d| < L/2 for every candidate and the image test is a no-op.
    const int cx = (int)compact3(mkey), cy = (int)compact3(mkey >> 1),
              cz = (int)compact3(mkey >> 2);
    bool wrap = false;
    {
        const int cc[3] = {cx, cy, cz};
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            if (!g.periodic[a]) continue;
            int mn = active ? cc[a] : INT_MAX, mx = active ? cc[a] : INT_MIN;
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) {
                mn = min(mn, __shfl_xor(mn, o, kWave));
                mx = max(mx, __shfl_xor(mx, o, kWave));
            }
            // candidates lie in cells [mn - 1, mx + 1]: |d| < (mx - mn + 3) cells
            if (mn < 1 || mx > g.nc[a] - 2 || 2 * (mx - mn + 3) >= g.nc[a]) wrap = true;
        }
    }

    const int nent = ndist * kStencil;
    bool use_union = nent <= kMaxEntries && !mixed;
    int nu = 0, total = 0;
    __syncthreads();
    if (use_union) {
        // stencil cells of every distinct cell; empty ones become sentinels
        for (int e = lane; e < kMaxEntries; e += kWave) {
            int2 v = make_int2(INT_MAX, INT_MAX);
            if (e < nent) {
                const uint32_t k = dkeys[e / kStencil];
                const int s = e % kStencil;
                bool okx, oky, okz;
                const int x = wrap_or_clip((int)compact3(k) + s % 3 - 1, g.nc[0], g.periodic[0], okx);
                const int y = wrap_or_clip((int)compact3(k >> 1) + (s / 3) % 3 - 1, g.nc[1],
                                           g.periodic[1], oky);
                const int z = wrap_or_clip((int)compact3(k >> 2) + s / 9 - 1, g.nc[2],
                                           g.periodic[2], okz);
                if (okx && oky && okz) {
                    const int64_t cell = cbase + ((int64_t)z * g.nc[1] + y) * g.nc[0] + x;
                    const int a = cstart[cell], e2 = cend[cell];
                    if (a < e2) v = make_int2(a, e2);
                }
            }
            ent[e] = v;
        }
        __syncthreads();
        // bitonic sort of the 128 entries by start, one pair per lane per step
        for (int k = 2; k <= kMaxEntries; k <<= 1) {
            for (int j = k >> 1; j > 0; j >>= 1) {
                const int lo_i = ((lane & ~(j - 1)) << 1) | (lane & (j - 1));
                const int hi_i = lo_i | j;
                const int2 ea = ent[lo_i], eb = ent[hi_i];
                const bool up = (lo_i & k) == 0;
                if ((ea.x > eb.x) == up) {
                    ent[lo_i] = eb;
                    ent[hi_i] = ea;
                }
                __syncthreads();
            }
        }
        // drop sentinels and duplicates (a cell listed by several stencils)
        int2 v0 = ent[lane], v1 = ent[lane + kWave];
        const int p0 = lane == 0 ? INT_MIN : ent[lane - 1].x;
        const int p1 = ent[lane + kWave - 1].x;
        const bool k0 = v0.x != INT_MAX && v0.x != p0;
        const bool k1 = v1.x != INT_MAX && v1.x != p1;
        const uint64_t m0 = __ballot(k0), m1 = __ballot(k1);
        const int n0 = __popcll(m0);
        nu = n0 + __popcll(m1);
        int pos0 = __popcll(m0 & lt), pos1 = n0 + __popcll(m1 & lt);
        if (k0) cells[pos0] = v0;
        if (k1) cells[pos1] = v1;
        __syncthreads();
        // u0[c]: exclusive prefix of the cell lengths; lane holds c = lane and
        // c = lane + 64
        const int l0 = lane < nu ? cells[lane].y - cells[lane].x : 0;
        const int l1 = lane + kWave < nu ? cells[lane + kWave].y - cells[lane + kWave].x : 0;
        int s0 = l0, s1 = l1;
#pragma unroll
        for (int o = 1; o < kWave; o <<= 1) {
            const int t0s = __shfl_up(s0, o, kWave), t1s = __shfl_up(s1, o, kWave);
            if (lane >= o) {
                s0 += t0s;
                s1 += t1s;
            }
        }
        const int tot0 = __shfl(s0, kWave - 1, kWave);
        total = tot0 + __shfl(s1, kWave - 1, kWave);
        if (lane < nu) u0[lane] = s0 - l0;
        if (lane + kWave < nu) u0[lane + kWave] = tot0 + s1 - l1;
        if (lane == 0) u0[nu] = total;
        use_union = total <= kMaxCandidates;
        __syncthreads();
    }

    if (use_union) {
        const bool uniform_h = Multi ? b.runs[slot0].uniform_h != 0 : hflag[0] == 0;
        int cnt = 0;
        uint64_t occ = 0;  // bit w: mask word w has at least one bit for this lane
        if (wrap) {
            if (uniform_h) stream_union<true, true>(me, srec, cells, nu, g, bm, lane, cnt, occ);
            else stream_union<true, false>(me, srec, cells, nu, g, bm, lane, cnt, occ);
        } else {
            if (uniform_h) stream_union<false, true>(me, srec, cells, nu, g, bm, lane, cnt, occ);
            else stream_union<false, false>(me, srec, cells, nu, g, bm, lane, cnt, occ);
        }
        // the lane's own particle is in the union: drop its bit
        if (active) {
            int lo = 0, hi = nu - 1;
            while (lo < hi) {  // last cell with start <= i
                const int mid = (lo + hi + 1) >> 1;
                if (cells[mid].x <= i) lo = mid; else hi = mid - 1;
            }
            const int u_self = u0[lo] + (int)(i - cells[lo].x);
            const int ws = u_self >> 5;
            const uint32_t bit = 0x80000000u >> (u_self & 31);
            const uint32_t word = bm[ws * kWave + lane];
            if (word & bit) {
                bm[ws * kWave + lane] = word & ~bit;
                --cnt;
                if ((word & ~bit) == 0) occ &= ~(1ull << ws);
            }
        } else {
            cnt = 0;
        }
        int maxc = cnt;
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) maxc = max(maxc, __shfl_xor(maxc, o, kWave));
        const int rows = min(maxc, max_nb);
        // Expand row by row: row k of every lane is written by one store. Each
        // lane walks its non-empty words (occ) with the next word already in
        // flight, and keeps the current cell's bounds in registers.
        auto pop_word = [&]() -> int {
            if (occ == 0) return -1;
            const int w = __builtin_ctzll(occ);
            occ &= occ - 1;
            return w;
        };
        int w_cur = pop_word();
        uint32_t cur = w_cur >= 0 ? bm[w_cur * kWave + lane] : 0u;
        int w_nxt = pop_word();
        uint32_t nxt = w_nxt >= 0 ? bm[w_nxt * kWave + lane] : 0u;
        int cp = 0;
        int c_start = cells[0].x, c_u0 = 0, c_end_u = u0[1];
        for (int k = 0; k < rows; ++k) {
            if (k < cnt) {
                if (cur == 0) {
                    cur = nxt;
                    w_cur = w_nxt;
                    w_nxt = pop_word();
                    nxt = w_nxt >= 0 ? bm[w_nxt * kWave + lane] : 0u;
                }
                const int t = __builtin_clz(cur);
                const int uu = w_cur * 32 + t;
                cur &= ~(0x80000000u >> t);
                while (uu >= c_end_u) {
                    ++cp;
                    c_start = cells[cp].x;
                    c_u0 = c_end_u;
                    c_end_u = u0[cp + 1];
                }
                idx[(int64_t)k * ld + i] = c_start + (uu - c_u0);
            }
        }
        if (active) {
            count[i] = cnt;
            if (cnt > max_nb) atomicOr(Multi ? &b.status[slot0] : status0, ST_CAPACITY);
        }
        return;
    }

    // Per-lane path: the lane visits its own stencil's non-empty cells in
    // ascending order of their first particle (selecting the next one each
    // time), so its list is ascending too.
    if (!active) return;
    const Grid &gl = Multi ? b.runs[my_slot].grid : g0;
    const int64_t cbl = Multi ? (int64_t)b.runs[my_slot].cell_base : 0;
    int cnt = 0;
    const int32_t ii = (int32_t)i;
    int last = -1;
    for (;;) {
        int best_s = INT_MAX, best_e = 0;
        for (int s = 0; s < kStencil; ++s) {
            bool okx, oky, okz;
            const int x = wrap_or_clip(cx + s % 3 - 1, gl.nc[0], gl.periodic[0], okx);
            const int y = wrap_or_clip(cy + (s / 3) % 3 - 1, gl.nc[1], gl.periodic[1], oky);
            const int z = wrap_or_clip(cz + s / 9 - 1, gl.nc[2], gl.periodic[2], okz);
            if (!(okx && oky && okz)) continue;
            const int64_t cell = cbl + ((int64_t)z * gl.nc[1] + y) * gl.nc[0] + x;
            const int a = cstart[cell], b = cend[cell];
            if (a < b && a > last && a < best_s) {
                best_s = a;
                best_e = b;
            }
        }
        if (best_s == INT_MAX) break;
        for (int32_t j = best_s; j < best_e; ++j) {
            const SearchRec o = srec[j];
            if (related<true, false>(me, o, gl) && j != ii) {
                if (cnt < max_nb) idx[(int64_t)cnt * ld + i] = j;
                ++cnt;
            }
        }
        last = best_s;
    }
    count[i] = cnt;
    if (cnt > max_nb) atomicOr(Multi ? &b.status[my_slot] : status0, ST_CAPACITY);
}

template <bool Multi>
__global__ void __launch_bounds__(kWave)
find_neighbors_kernel(int64_t n, int64_t ld, const SearchRec *__restrict__ srec,
                      const uint32_t *__restrict__ keys, const int32_t *__restrict__ cstart,
                      const int32_t *__restrict__ cend, Grid g, int max_nb,
                      int32_t *__restrict__ count, int32_t *__restrict__ idx,
                      uint32_t *__restrict__ mask_scratch, const uint32_t *__restrict__ hflag,
                      uint32_t *status, BatchDev b)
{
    __shared__ SearchLds L;
    if constexpr (Multi) {
        const int64_t nn = b.hdr->n_out;
        const int64_t ntile = (nn + kWave - 1) / kWave;
        // the loop bound is wave-uniform, and each pass ends with the LDS
        // reuse ordered by the block barriers inside the tile
        for (int64_t tile = xcd_block(); tile < ntile; tile += gridDim.x) {
            search_tile<true>(tile, nn, ld, srec, keys, cstart, cend, g, max_nb, count, idx,
                              mask_scratch, hflag, status, b, L);
            __syncthreads();
        }
    } else {
        search_tile<false>(xcd_block(), n, ld, srec, keys, cstart, cend, g, max_nb, count, idx,
                           mask_scratch, hflag, status, b, L);
    }
}

}  // namespace

hipError_t launch_find_neighbors(sph_ctx ctx, const sph_particles &p, const sph_nbrs &nb)
{
    const unsigned blocks = (unsigned)((p.n + kWave - 1) / kWave);
    find_neighbors_kernel<false><<<blocks, kWave, 0, ctx->stream>>>(
        p.n, p.n, ctx->srec, ctx->sorted_keys, ctx->cell_start, ctx->cell_end, ctx->grid,
        nb.max_nb, nb.count, nb.idx, ctx->nb_mask, ctx->hflag_dev, ctx->status_dev, BatchDev{});
    return hipGetLastError();
}

hipError_t launch_find_neighbors_batch(sph_ctx ctx, const BatchDev &b, int max_nb,
                                       int32_t *count, int32_t *idx)
{
    // the mask scratch holds one region per tile of the capacity
    const unsigned blocks =
        (unsigned)std::min<int64_t>((b.cap + kWave - 1) / kWave, 16384);
    find_neighbors_kernel<true><<<blocks, kWave, 0, ctx->stream>>>(
        0, b.cap, ctx->srec, ctx->sorted_keys, ctx->cell_start, ctx->cell_end, Grid{}, max_nb,
        count, idx, ctx->nb_mask, nullptr, nullptr, b);
    return hipGetLastError();
}

}  // namespace sph
