// Algorithm 1, step 2 on the GPU: the neighbour search.
//
// One wavefront per tile of 64 consecutive particles (cell order), four
// independent wavefronts per block. The wave first builds, in its own LDS
// region, the union of the 27-cell stencils of the cells its particles live
// in: the non-empty cells, sorted by their first particle and without
// duplicates, so walking them visits candidates in ascending index order. It
// then streams that union wave-uniformly: each candidate's record is one
// scalar load into SGPRs, every lane tests it against its own particle with
// the exact FP64 relation, and the outcome goes into a per-lane bit mask (one
// bit per union position, kept in a global scratch region so that the LDS
// footprint stays small and occupancy high; each 32-bit word of 64 lanes is
// one 256-byte store). A second phase expands the masks row by row, so that
// all lanes write row k of the ELL list together (one contiguous 256-byte
// store per row) instead of scattering 4-byte writes; a per-wave table maps
// each union position to its cell, so a set bit becomes an index with two
// LDS reads.
//
// Periodic axes: when no stencil of the tile reaches across a periodic
// boundary the image test is skipped. Otherwise, when every periodic axis has
// at least 5 cells, the image is chosen once per (union cell, lane) from the
// cell indices: a true neighbour lies in an adjacent cell, and for adjacent
// cells the wrapped ones are exactly those whose raw difference exceeds half
// the box, so adding -L, 0 or +L to the raw difference reproduces the
// minimum-image arithmetic (d -= L or d += L) for every true neighbour; for
// any other candidate a wrong image only makes the distance larger than half
// the box, i.e. larger than 2 h_max, and it is rejected either way. With
// fewer cells the image is chosen per candidate.
//
// A wave whose union has more candidates than the masks hold (dense cells)
// streams the same union but lets each lane append its accepted candidates
// directly; when no image is in play it walks, in each cell, only the z
// slices (the lowest key bits order a cell's particles by z) within reach of
// the tile's z extent. A wave with more distinct cells than its union build
// holds (9), or with a union of many dense cells, takes
// the per-lane path instead: each lane walks its own stencil (sorted by
// Morton key) and writes its entries directly. Both paths produce the same set in the
// same (ascending) order, so the sums over a list do not depend on the path
// or on where the tile boundaries fall.
#include <algorithm>
#include <climits>

#include "sph_internal.h"

namespace sph {
namespace {

constexpr int kWave = 64;
constexpr int kWavesPerBlock = 4;
constexpr int kBlock = kWave * kWavesPerBlock;
constexpr int kMaxCandidates = kSearchMaskWords * 32;
// Stencil entries (27 per distinct cell, before dedup) a tile's union build
// holds: 9 distinct cells (tiles of small runs, and tiles of a rotated
// lattice after some steps, span more than four). Tiles with at most 4 sort
// only the first 128 entries.
constexpr int kEntries = 256;
// Cells of a union handed to the second kernel (held two per lane there).
constexpr int kDenseCells = 2 * 64;
constexpr int kMaxWords = kSearchMaskWords;
// Grid of the second kernel: one-wave blocks draining the worklist, up to 32
// per CU (its occupancy limit is 5 waves per SIMD); the blocks past the
// worklist's length exit at once. 2048 blocks left the dense centre of a 1M
// Evrard sphere on 2 waves per SIMD (search 3.9 ms, 3.0 ms with this grid).
constexpr int64_t kFallbackBlocks = 8192;

enum WrapMode { WRAP_NONE = 0, WRAP_CELL = 1, WRAP_PAIR = 2 };

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

// LDS operations of one wave complete in order; this only keeps the
// compiler from moving them across the point (the wave's regions are its own).
__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
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

// Squared separation of the relation test, with the image conventions of
// the mode. sh: the per-cell image shift (WRAP_CELL).
template <int Mode>
__device__ __forceinline__ double sep2(const SearchRec &me, const SearchRec &o, const Grid &g,
                                       const double (&sh)[3])
{
    double dx = me.x - o.x, dy = me.y - o.y, dz = me.z - o.z;
    if (Mode == WRAP_CELL) {
        dx += sh[0];
        dy += sh[1];
        dz += sh[2];
    } else if (Mode == WRAP_PAIR) {
        if (g.periodic[0]) dx = min_image_sel(dx, g.len[0], g.half[0]);
        if (g.periodic[1]) dy = min_image_sel(dy, g.len[1], g.half[1]);
        if (g.periodic[2]) dz = min_image_sel(dz, g.len[2], g.half[2]);
    }
    return __builtin_fma(dz, dz, __builtin_fma(dy, dy, dx * dx));
}

// A double that is the same in every lane, as a wave-uniform value.
__device__ __forceinline__ double uniform_f64(double v)
{
    const unsigned long long u = (unsigned long long)__double_as_longlong(v);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)u);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(u >> 32));
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// acc * 2 + [r2 < s2], s2 wave-uniform: the comparison's lane mask is the
// carry-in of one add (acc + acc + carry), which shifts the bit in.
__device__ __forceinline__ uint32_t shift_in(uint32_t acc, double r2, double s2)
{
    uint32_t out;
    asm("v_cmp_gt_f64 vcc, %2, %1\n\t"
        "v_addc_co_u32 %0, vcc, %3, %3, vcc"
        : "=v"(out)
        : "v"(r2), "s"(s2), "v"(acc)
        : "vcc");
    return out;
}

// acc * 2 + [r2 < s2a or r2 < s2b], s2b wave-uniform: the two lane masks are
// joined on the scalar unit (comparing against the larger of the two would
// cost two more vector instructions).
__device__ __forceinline__ uint32_t shift_in2(uint32_t acc, double r2, double s2a, double s2b)
{
    uint32_t out;
    uint64_t t;
    asm("v_cmp_lt_f64 %1, %2, %3\n\t"
        "v_cmp_gt_f64 vcc, %4, %2\n\t"
        "s_or_b64 vcc, vcc, %1\n\t"
        "v_addc_co_u32 %0, vcc, %5, %5, vcc"
        : "=v"(out), "=&s"(t)
        : "v"(r2), "v"(s2a), "s"(s2b), "v"(acc)
        : "vcc", "scc");
    return out;
}

// Relation test: r2 < (2h_i)^2 or r2 < (2h_j)^2, i.e. r2 < (2 max(h_i,h_j))^2.
// UniformH: every particle has the same h, one compare against the lane's
// own (2h)^2. sh: the per-cell image shift (WRAP_CELL).
template <int Mode, bool UniformH>
__device__ __forceinline__ bool related(const SearchRec &me, const SearchRec &o, const Grid &g,
                                        const double (&sh)[3])
{
    double dx = me.x - o.x, dy = me.y - o.y, dz = me.z - o.z;
    if (Mode == WRAP_CELL) {
        dx += sh[0];
        dy += sh[1];
        dz += sh[2];
    } else if (Mode == WRAP_PAIR) {
        if (g.periodic[0]) dx = min_image_sel(dx, g.len[0], g.half[0]);
        if (g.periodic[1]) dy = min_image_sel(dy, g.len[1], g.half[1]);
        if (g.periodic[2]) dz = min_image_sel(dz, g.len[2], g.half[2]);
    }
    const double r2 = __builtin_fma(dz, dz, __builtin_fma(dy, dy, dx * dx));
    if (UniformH) return r2 < me.s2;
    return (r2 < me.s2) | (r2 < o.s2);
}

// Per-wave LDS, overlaid by lifetime: the union cells are formed from the
// sorted entries (all entries are read before the first cell is written);
// the position -> cell table is filled after the stream and the self-bit
// removal, when the cells are no longer read; the first union positions are
// written once the distinct keys have been read. At 256 entries this is 5 KiB
// per wave, 20 KiB per block: 8 blocks per CU.
template <int E>
struct SearchLds {
    static_assert(E % (2 * kWave) == 0 && E <= 256, "entries: whole pairs per lane, uint8 cells");
    union {
        struct {
            union {
                int2 ent[E];      // stencil entries {first particle, entry index}
                int2 cells[E];    // union cells {first, end}, ascending (formed from ent)
            };
            uint32_t cxyz[E];     // packed cell coordinates x | y << 10 | z << 20
        };
        uint8_t cellof[kMaxCandidates];   // union position -> union cell
    };
    union {
        uint32_t dkeys[kWave];    // keys of the tile's distinct cells
        int u0[E];                // first union position of each cell
    };
    int base[E];                  // first particle minus first union position
};

// Stream the union (cells[0..nu)) and record, for each candidate u, whether
// it is related to the lane's particle. Masks are 32-bit words bm[word][lane]
// (word = u / 32) filled from the top: candidate u sits at bit 31 - u % 32.
// Within a cell the next four records are loaded while the current four are
// tested, so the scalar-load latency is overlapped with work.
template <int Mode, bool UniformH, int E>
__device__ __forceinline__ void stream_union(const SearchRec &me, const int (&myc)[3],
                                             const SearchRec *__restrict__ srec,
                                             const SearchLds<E> &L, int nu, const Grid &g,
                                             uint32_t *__restrict__ bm, int lane, int &cnt,
                                             uint64_t &occ0, uint32_t &occ1)
{
    uint32_t acc = 0;
    int u = 0;
    double sh[3] = {0.0, 0.0, 0.0};
    auto flush = [&](int w, uint32_t word) {
        bm[w * kWave + lane] = word;
        cnt += __popc(word);
        if (w < 64) occ0 |= word ? (1ull << w) : 0ull;
        else occ1 |= word ? (1u << (w - 64)) : 0u;
    };
    auto step = [&](const SearchRec &o) {
        const double r2 = sep2<Mode>(me, o, g, sh);
        // uniform h: every (2h)^2 is the same number, the candidate's is
        // taken (a scalar operand, and the whole record is then loaded in
        // wide scalar loads)
        acc = UniformH ? shift_in(acc, r2, o.s2) : shift_in2(acc, r2, me.s2, o.s2);
        ++u;
        if ((u & 31) == 0) {
            flush((u >> 5) - 1, acc);
            acc = 0;
        }
    };
    for (int c = 0; c < nu; ++c) {
        const int s = __builtin_amdgcn_readfirstlane(L.cells[c].x);
        const int e = __builtin_amdgcn_readfirstlane(L.cells[c].y);
        if (Mode == WRAP_CELL) {
            const uint32_t p = __builtin_amdgcn_readfirstlane(L.cxyz[c]);
            const int cc[3] = {(int)(p & 1023u), (int)((p >> 10) & 1023u), (int)(p >> 20)};
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                const int d = cc[a] - myc[a];
                sh[a] = !g.periodic[a] ? 0.0 : (d >= 2 ? g.len[a] : (d <= -2 ? -g.len[a] : 0.0));
            }
        }
        int j = s;
        if (e - j >= 4) {
            SearchRec a0 = srec[j], a1 = srec[j + 1], a2 = srec[j + 2], a3 = srec[j + 3];
            j += 4;
            while (e - j >= 4) {
                const SearchRec b0 = srec[j], b1 = srec[j + 1], b2 = srec[j + 2],
                                b3 = srec[j + 3];
                // issue the loads of b0..b3 before the work on a0..a3
                __builtin_amdgcn_sched_barrier(0);
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

// Stream a union too large for the masks (dense cells): the same
// wave-uniform walk, each lane appending its accepted candidates to its own
// list as it goes (few candidates pass, so the scattered stores are rare).
// The union is held across the lanes: lane l has cell l in r0/p0 (range,
// packed coordinates) and cell l + 64 in r1/p1.
template <int Mode, bool UniformH>
__device__ __forceinline__ int stream_direct(const SearchRec &me, const int (&myc)[3],
                                             const SearchRec *__restrict__ srec, int2 r0,
                                             int2 r1, uint32_t p0, uint32_t p1, int nu,
                                             const Grid &g, bool active, int64_t i, int64_t ld,
                                             int max_nb, int32_t *__restrict__ idx)
{
    int cnt = 0;
    double sh[3] = {0.0, 0.0, 0.0};
    const int32_t ii = active ? (int32_t)i : -1;
    auto step = [&](const SearchRec &o, int32_t j) {
        if (related<Mode, UniformH>(me, o, g, sh) && j != ii && active) {
            if (cnt < max_nb) idx[(int64_t)cnt * ld + i] = j;
            ++cnt;
        }
    };
    for (int c = 0; c < nu; ++c) {
        const bool hi_half = c >= kWave;
        const int cl = c & (kWave - 1);
        const int s = __builtin_amdgcn_readlane(hi_half ? r1.x : r0.x, cl);
        const int e = __builtin_amdgcn_readlane(hi_half ? r1.y : r0.y, cl);
        if (Mode == WRAP_CELL) {
            const uint32_t p = (uint32_t)__builtin_amdgcn_readlane((int)(hi_half ? p1 : p0), cl);
            const int cc[3] = {(int)(p & 1023u), (int)((p >> 10) & 1023u), (int)(p >> 20)};
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                const int d = cc[a] - myc[a];
                sh[a] = !g.periodic[a] ? 0.0 : (d >= 2 ? g.len[a] : (d <= -2 ? -g.len[a] : 0.0));
            }
        }
        int j = s;
        if (e - j >= 4) {
            SearchRec a0 = srec[j], a1 = srec[j + 1], a2 = srec[j + 2], a3 = srec[j + 3];
            j += 4;
            while (e - j >= 4) {
                const SearchRec b0 = srec[j], b1 = srec[j + 1], b2 = srec[j + 2],
                                b3 = srec[j + 3];
                step(a0, j - 4);
                step(a1, j - 3);
                step(a2, j - 2);
                step(a3, j - 1);
                __builtin_amdgcn_sched_barrier(0);
                a0 = b0;
                a1 = b1;
                a2 = b2;
                a3 = b3;
                j += 4;
            }
            step(a0, j - 4);
            step(a1, j - 3);
            step(a2, j - 2);
            step(a3, j - 1);
        }
        for (; j < e; ++j) step(srec[j], j);
    }
    return cnt;
}

// Window of a union cell for a dense tile (no periodic image in play): the
// sub-range of the cell's particles that can hold a candidate related to a
// particle of the tile, R^2 being the larger of the tile's and the cell's
// largest (2h)^2.
// - The whole cell is skipped when its x or y range lies more than R + a
//   millionth of a cell beyond the tile's extent [lo, hi] on that axis: every
//   candidate is then farther than both smoothing diameters from every
//   particle of the tile (a particle's cell index comes from the same
//   arithmetic, whose rounding is some 1e-13 of a cell).
// - Otherwise only the z slices within R + (one slice) of the tile's z
//   extent are kept, by the same argument; a cell's keys are ordered by
//   slice, so the window is found by binary search.
// The first and last cell of an axis also hold the particles clamped into
// them from outside the box, so their range is taken as unbounded on the
// outer side, and their outer slice is always kept.
// z_window_r: the same for a given reach r (s2max not read).
__device__ __forceinline__ int2 z_window_r(int2 cr, uint32_t p, const Grid &g,
                                           const double (&tlo)[3], const double (&thi)[3],
                                           double r, const uint32_t *__restrict__ keys);

__device__ __forceinline__ int2 z_window(int2 cr, uint32_t p, const Grid &g, const double (&tlo)[3],
                                         const double (&thi)[3], double s2t,
                                         const unsigned long long *__restrict__ s2max,
                                         const uint32_t *__restrict__ keys)
{
    if (cr.x >= cr.y) return cr;
    const int x = (int)(p & 1023u), y = (int)((p >> 10) & 1023u), z = (int)(p >> 20);
    const int64_t cell = ((int64_t)z * g.nc[1] + y) * g.nc[0] + x;
    const double s2c = __longlong_as_double((long long)s2max[cell]);
    return z_window_r(cr, p, g, tlo, thi, sqrt(fmax(s2t, s2c)), keys);
}

__device__ __forceinline__ int2 z_window_r(int2 cr, uint32_t p, const Grid &g,
                                           const double (&tlo)[3], const double (&thi)[3],
                                           double r, const uint32_t *__restrict__ keys)
{
    if (cr.x >= cr.y) return cr;
    const int x = (int)(p & 1023u), y = (int)((p >> 10) & 1023u), z = (int)(p >> 20);
    const int cxy[2] = {x, y};
#pragma unroll
    for (int a = 0; a < 2; ++a) {
        const double fl = (tlo[a] - g.lo[a]) * g.inv_s[a], fh = (thi[a] - g.lo[a]) * g.inv_s[a];
        const double ra = r * g.inv_s[a] + 1e-6;
        const bool above = cxy[a] > 0 && (double)cxy[a] - fh > ra;
        const bool below = cxy[a] < g.nc[a] - 1 && fl - (double)(cxy[a] + 1) > ra;
        if (above || below) return make_int2(cr.x, cr.x);
    }
    const double zlo = tlo[2], zhi = thi[2];
    const double ns = (double)(1 << g.zbits);
    const double fl = ((zlo - r) - g.lo[2]) * g.inv_s[2] - (double)z;
    const double fh = ((zhi + r) - g.lo[2]) * g.inv_s[2] - (double)z;
    double ql = fmax(floor(fl * ns) - 1.0, 0.0);
    double qh = fmin(floor(fh * ns) + 1.0, ns - 1.0);
    if (z == 0) qh = fmax(qh, 0.0);
    if (z == g.nc[2] - 1) ql = fmin(ql, ns - 1.0);
    if (ql > qh) return make_int2(cr.x, cr.x);
    if (ql == 0.0 && qh == ns - 1.0) return cr;
    const uint32_t base = keys[cr.x] & ~((1u << g.zbits) - 1u);
    const uint32_t klo = base | (uint32_t)ql, khi = base | (uint32_t)qh;
    int a = cr.x, e = cr.y;
    while (a < e) {  // first key >= klo
        const int mid = (a + e) >> 1;
        if (keys[mid] < klo) a = mid + 1; else e = mid;
    }
    const int first = a;
    e = cr.y;
    while (a < e) {  // first key > khi
        const int mid = (a + e) >> 1;
        if (keys[mid] <= khi) a = mid + 1; else e = mid;
    }
    return make_int2(first, a);
}

// One tile of 64 particles. Multi: the particles belong to one run of an
// ensemble (slot in the high key bits) and the tile uses that run's grid
// and cell range; a tile found spanning two runs would take the per-lane
// path with each lane's own run.
template <bool Multi>
__device__ __forceinline__ void search_tile(
    int64_t tile, int64_t n, int64_t ld, const SearchRec *__restrict__ srec,
    const uint32_t *__restrict__ keys, const int32_t *__restrict__ cstart,
    const int32_t *__restrict__ cend, const Grid &g0, int max_nb, int32_t *__restrict__ count,
    int32_t *__restrict__ idx, uint32_t *__restrict__ mask_scratch,
    const uint32_t *__restrict__ hflag, uint32_t *status0, const BatchDev &b,
    SearchLds<kEntries> &L,
    int32_t *__restrict__ fb_tiles, uint32_t *fb_count,
    const unsigned long long *__restrict__ s2max)
{
    const int lane = threadIdx.x & (kWave - 1);
    int64_t t0, tend;
    tile_span<Multi>(tile, n, b, t0, tend);
    uint32_t *bm = mask_scratch + tile * (kMaxWords * kWave);
    const int64_t i = t0 + lane;
    const bool active = i < tend;
    const uint64_t lt = lane == 0 ? 0ull : (~0ull >> (64 - lane));

    const uint32_t key = active ? keys[i] : 0xFFFFFFFFu;
    const SearchRec me = active ? srec[i] : SearchRec{0.0, 0.0, 0.0, 0.0};
    // run of the tile (lane 0 is always active) and whether all lanes share it
    int my_slot = 0, slot0 = 0;
    bool mixed = false;
    if constexpr (Multi) {
        my_slot = active ? (int)(key >> kEnsSlotShift) : 0;
        slot0 = __builtin_amdgcn_readfirstlane(my_slot);
        mixed = __ballot(active && my_slot != slot0) != 0ull;
    }
    // the run's grid, read once into wave-uniform registers
    Grid gm;
    if constexpr (Multi) {
        const uint32_t *src = reinterpret_cast<const uint32_t *>(&b.runs[slot0].grid);
        uint32_t *dst = reinterpret_cast<uint32_t *>(&gm);
#pragma unroll
        for (int k = 0; k < (int)(sizeof(Grid) / 4); ++k)
            dst[k] = __builtin_amdgcn_readfirstlane(src[k]);
    }
    const Grid &g = Multi ? gm : g0;
    const int64_t cbase = Multi ? (int64_t)b.runs[slot0].cell_base : 0;
    // cell part of the key (run and Morton code, without the z slice)
    const uint32_t ckey = key >> (Multi ? kSliceBits : g0.zbits);
    const uint32_t mkey = Multi ? (ckey & kEnsMortonMask) : ckey;
    const uint32_t prev = __shfl_up(ckey, 1, kWave);
    const bool first = active && (lane == 0 || ckey != prev);
    const uint64_t fm = __ballot(first);
    const int ndist = __popcll(fm);
    if (first) L.dkeys[__popcll(fm & lt)] = mkey;

    // The image test can be skipped for the whole wave when, on every
    // periodic axis, the union of the stencils spans less than half the box:
    // then |d| < L/2 for every candidate. Per-cell images need >= 5 cells.
    const int myc[3] = {(int)compact3(mkey), (int)compact3(mkey >> 1),
                        (int)compact3(mkey >> 2)};
    bool wrap = false, few_cells = false;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        if (!g.periodic[a]) continue;
        int mn = active ? myc[a] : INT_MAX, mx = active ? myc[a] : INT_MIN;
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            mn = min(mn, __shfl_xor(mn, o, kWave));
            mx = max(mx, __shfl_xor(mx, o, kWave));
        }
        // candidates lie in cells [mn - 1, mx + 1]: |d| < (mx - mn + 3) cells
        if (mn < 1 || mx > g.nc[a] - 2 || 2 * (mx - mn + 3) >= g.nc[a]) wrap = true;
        if (g.nc[a] < 5) few_cells = true;
    }

    constexpr int E = kEntries;
    constexpr int kC = E / kWave;  // entries per lane
    const int nent = ndist * kStencil;
    bool use_union = nent <= E && !mixed;
    int nu = 0, total = 0;
    wave_sync();
    if (use_union) {
        // stencil cells of every distinct cell; empty ones become sentinels
        for (int e = lane; e < E; e += kWave) {
            int2 v = make_int2(INT_MAX, e);
            if (e < nent) {
                const uint32_t k = L.dkeys[e / kStencil];
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
                    if (a < e2) v = make_int2(a, e);
                }
            }
            L.ent[e] = v;
        }
        wave_sync();
        // bitonic sort of the first sortN entries by first particle (the
        // rest are sentinels, already in place): the sortN / 2
        // compare-exchanges of a step are disjoint, up to kC / 2 per lane
        const int sortN = nent <= 2 * kWave ? 2 * kWave : E;
        for (int k = 2; k <= sortN; k <<= 1) {
            for (int j = k >> 1; j > 0; j >>= 1) {
#pragma unroll
                for (int q = 0; q < kC / 2; ++q) {
                    if (2 * kWave * q >= sortN) break;
                    const int p = lane + q * kWave;
                    const int lo_i = ((p & ~(j - 1)) << 1) | (p & (j - 1));
                    const int hi_i = lo_i | j;
                    const int2 ea = L.ent[lo_i], eb = L.ent[hi_i];
                    const bool up = (lo_i & k) == 0;
                    if ((ea.x > eb.x) == up) {
                        L.ent[lo_i] = eb;
                        L.ent[hi_i] = ea;
                    }
                }
                wave_sync();
            }
        }
        // drop sentinels and duplicates (a cell listed by several stencils);
        // a kept entry's cell is recomputed from its entry index. Lane holds
        // entries lane + q * 64.
        int2 v[kC];
        bool kp[kC];
        uint64_t m[kC];
        int off[kC + 1];
        off[0] = 0;
#pragma unroll
        for (int q = 0; q < kC; ++q) {
            const int e = lane + q * kWave;
            v[q] = L.ent[e];
            const int pv = e == 0 ? INT_MIN : L.ent[e - 1].x;
            kp[q] = v[q].x != INT_MAX && v[q].x != pv;
            m[q] = __ballot(kp[q]);
            off[q + 1] = off[q] + __popcll(m[q]);
        }
        nu = off[kC];
        auto keep = [&](const int2 ve, int pos) {
            const uint32_t k = L.dkeys[ve.y / kStencil];
            const int s = ve.y % kStencil;
            bool ok;
            const int x = wrap_or_clip((int)compact3(k) + s % 3 - 1, g.nc[0], g.periodic[0], ok);
            const int y = wrap_or_clip((int)compact3(k >> 1) + (s / 3) % 3 - 1, g.nc[1],
                                       g.periodic[1], ok);
            const int z = wrap_or_clip((int)compact3(k >> 2) + s / 9 - 1, g.nc[2],
                                       g.periodic[2], ok);
            const int64_t cell = cbase + ((int64_t)z * g.nc[1] + y) * g.nc[0] + x;
            L.cells[pos] = make_int2(ve.x, cend[cell]);
            L.cxyz[pos] = (uint32_t)x | ((uint32_t)y << 10) | ((uint32_t)z << 20);
        };
#pragma unroll
        for (int q = 0; q < kC; ++q)
            if (kp[q]) keep(v[q], off[q] + __popcll(m[q] & lt));
        wave_sync();
        if constexpr (!Multi) {
            if (!wrap && g.zbits > 0) {
                // Each union cell only in its window for the tile (as for the
                // dense unions of the second kernel): cells beyond reach in x
                // or y are emptied, the others keep the z slices within reach
                // of the tile's z extent. Windows stay inside their cells, so
                // the cells stay ascending and hold the tile's own particles.
                double tlo[3], thi[3];
                double s2t = active ? me.s2 : 0.0;
                const double mc[3] = {me.x, me.y, me.z};
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    tlo[a] = active ? mc[a] : INFINITY;
                    thi[a] = active ? mc[a] : -INFINITY;
                }
#pragma unroll
                for (int o = 32; o > 0; o >>= 1) {
#pragma unroll
                    for (int a = 0; a < 3; ++a) {
                        tlo[a] = fmin(tlo[a], __shfl_xor(tlo[a], o, kWave));
                        thi[a] = fmax(thi[a], __shfl_xor(thi[a], o, kWave));
                    }
                    s2t = fmax(s2t, __shfl_xor(s2t, o, kWave));
                }
                // the reduced values are the same in every lane: keep them in
                // scalar registers (vector registers bound the occupancy)
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    tlo[a] = uniform_f64(tlo[a]);
                    thi[a] = uniform_f64(thi[a]);
                }
                s2t = uniform_f64(s2t);
#pragma unroll 1
                for (int c = lane; c < nu; c += kWave)
                    L.cells[c] = z_window(L.cells[c], L.cxyz[c], g, tlo, thi, s2t, s2max, keys);
                wave_sync();
            }
        }
        // u0[c]: exclusive prefix of the cell lengths; lane holds cells
        // c = lane + q * 64
#pragma unroll
        for (int q = 0; q < kC; ++q) {
            const int c = lane + q * kWave;
            const int l = c < nu ? L.cells[c].y - L.cells[c].x : 0;
            int sc = l;
#pragma unroll
            for (int o = 1; o < kWave; o <<= 1) {
                const int t = __shfl_up(sc, o, kWave);
                if (lane >= o) sc += t;
            }
            if (c < nu) {
                L.u0[c] = total + sc - l;
                L.base[c] = L.cells[c].x - (total + sc - l);
            }
            total += __shfl(sc, kWave - 1, kWave);
        }
        wave_sync();
        if (total > kMaxCandidates) {
            if (nu <= kDenseCells) {
                // Too large for the masks: the second kernel walks the same
                // union, read from this tile's scratch region (cells, then
                // coordinates, then the count), with each lane appending
                // directly.
                int2 *gc = reinterpret_cast<int2 *>(bm);
                uint32_t *gx = bm + 2 * kDenseCells;
                for (int c = lane; c < nu; c += kWave) {
                    gc[c] = L.cells[c];
                    gx[c] = L.cxyz[c];
                }
                if (lane == 0) {
                    bm[3 * kDenseCells] = (uint32_t)nu;
                    fb_tiles[atomicAdd(fb_count, 1u)] = (int32_t)(0x80000000u | (uint32_t)tile);
                }
                return;
            }
            use_union = false;  // many dense cells: the per-lane path
        }
    }

    if (use_union) {
        const bool uniform_h = Multi ? b.runs[slot0].uniform_h != 0 : hflag[0] == 0;
        const int mode = !wrap ? WRAP_NONE : (few_cells ? WRAP_PAIR : WRAP_CELL);
        int cnt = 0;
        uint64_t occ0 = 0;  // bit w: mask word w has at least one bit for this lane
        uint32_t occ1 = 0;  // the same for words 64..
#define SPH_STREAM(M, U) \
    stream_union<M, U>(me, myc, srec, L, nu, g, bm, lane, cnt, occ0, occ1)
        if (mode == WRAP_NONE) {
            if (uniform_h) SPH_STREAM(WRAP_NONE, true); else SPH_STREAM(WRAP_NONE, false);
        } else if (mode == WRAP_CELL) {
            if (uniform_h) SPH_STREAM(WRAP_CELL, true); else SPH_STREAM(WRAP_CELL, false);
        } else {
            if (uniform_h) SPH_STREAM(WRAP_PAIR, true); else SPH_STREAM(WRAP_PAIR, false);
        }
#undef SPH_STREAM
        // the lane's own particle is in the union: drop its bit
        if (active) {
            int lo = 0, hi = nu - 1;
            while (lo < hi) {  // last cell with start <= i
                const int mid = (lo + hi + 1) >> 1;
                if (L.cells[mid].x <= i) lo = mid; else hi = mid - 1;
            }
            const int u_self = L.u0[lo] + (int)(i - L.cells[lo].x);
            const int ws = u_self >> 5;
            const uint32_t bit = 0x80000000u >> (u_self & 31);
            const uint32_t word = bm[ws * kWave + lane];
            if (word & bit) {
                bm[ws * kWave + lane] = word & ~bit;
                --cnt;
                if ((word & ~bit) == 0) {
                    if (ws < 64) occ0 &= ~(1ull << ws);
                    else occ1 &= ~(1u << (ws - 64));
                }
            }
        } else {
            cnt = 0;
        }
        wave_sync();
        // union position -> union cell, for the expansion (overlays the
        // union-build arrays, which are not read after this point)
        for (int c = 0; c < nu; ++c) {
            const int a = L.u0[c], e = c + 1 < nu ? L.u0[c + 1] : total;
            for (int uu = a + lane; uu < e; uu += kWave) L.cellof[uu] = (uint8_t)c;
        }
        wave_sync();
        int maxc = cnt;
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) maxc = max(maxc, __shfl_xor(maxc, o, kWave));
        const int rows = min(maxc, max_nb);
        // Expand row by row: row k of every lane is written by one store. Each
        // lane walks its non-empty words (occ) with the next word already in
        // flight. Rows go out in chunks: the chunk's entries are formed in
        // registers first, then stored together, so that a wait for a mask
        // word (stores share its counter) waits for the previous chunk's
        // stores once per chunk, not once per row.
        auto pop_word = [&]() -> int {
            if (occ0 != 0) {
                const int w = __builtin_ctzll(occ0);
                occ0 &= occ0 - 1;
                return w;
            }
            if (occ1 == 0) return -1;
            const int w = 64 + __builtin_ctz(occ1);
            occ1 &= occ1 - 1;
            return w;
        };
        int w_cur = pop_word();
        uint32_t cur = w_cur >= 0 ? bm[w_cur * kWave + lane] : 0u;
        int w_nxt = pop_word();
        uint32_t nxt = w_nxt >= 0 ? bm[w_nxt * kWave + lane] : 0u;
        constexpr int kChunk = 16;
        const int mine = min(cnt, max_nb);
        for (int k0 = 0; k0 < rows; k0 += kChunk) {
            int val[kChunk];
#pragma unroll
            for (int r = 0; r < kChunk; ++r) {
                val[r] = 0;
                if (k0 + r < mine) {
                    if (cur == 0) {
                        cur = nxt;
                        w_cur = w_nxt;
                        w_nxt = pop_word();
                        nxt = w_nxt >= 0 ? bm[w_nxt * kWave + lane] : 0u;
                    }
                    const int t = __builtin_clz(cur);
                    val[r] = w_cur * 32 + t;
                    cur &= ~(0x80000000u >> t);
                }
            }
#pragma unroll
            for (int r = 0; r < kChunk; ++r)
                if (k0 + r < mine) val[r] += L.base[L.cellof[val[r]]];
            // Rows of 64 consecutive entries, whole lines: stored
            // non-temporally, the list (read back only by the next calls)
            // does not evict the union's records from L2. The scattered
            // appends of the per-lane walks stay ordinary stores (partial
            // lines written non-temporally double their time).
#pragma unroll
            for (int r = 0; r < kChunk; ++r)
                if (k0 + r < mine)
                    __builtin_nontemporal_store(val[r], &idx[(int64_t)(k0 + r) * ld + i]);
        }
        if (active) {
            count[i] = cnt;
            if (cnt > max_nb) atomicOr(Multi ? &b.status[slot0] : status0, ST_CAPACITY);
        }
        return;
    }

    // The tile takes the per-lane path, in a kernel of its own (its
    // registers would otherwise lower the occupancy of this one).
    if (lane == 0) fb_tiles[atomicAdd(fb_count, 1u)] = (int32_t)tile;
}

// Per-lane path, one wave per listed tile: each lane visits its own
// stencil's cells in ascending Morton order (= ascending order of their
// particles): the 27 keys are sorted in registers, then each cell is walked
// once with the next record already in flight, so the lane's list is
// ascending too.
template <bool Multi>
__global__ void __launch_bounds__(kWave)
fallback_kernel(int64_t n, int64_t ld, const SearchRec *__restrict__ srec,
                const uint32_t *__restrict__ keys, const int32_t *__restrict__ cstart,
                const int32_t *__restrict__ cend, Grid g0, int max_nb,
                int32_t *__restrict__ count, int32_t *__restrict__ idx, uint32_t *status0,
                BatchDev b, const int32_t *__restrict__ fb_tiles, const uint32_t *fb_count,
                const uint32_t *__restrict__ mask_scratch, const uint32_t *__restrict__ hflag,
                const unsigned long long *__restrict__ s2max)
{
    const int lane = threadIdx.x;
    if (Multi) n = b.hdr->n_out;
    const uint32_t nfb = *fb_count;
    for (uint32_t q = blockIdx.x; q < nfb; q += gridDim.x) {
    const uint32_t entry = (uint32_t)fb_tiles[q];
    const int64_t tile = (int64_t)(entry & 0x7FFFFFFFu);
    int64_t t0, tend;
    tile_span<Multi>(tile, n, b, t0, tend);
    const int64_t i = t0 + lane;
    const bool active = i < tend;
    const uint32_t key = active ? keys[i] : 0xFFFFFFFFu;
    const SearchRec me = active ? srec[i] : SearchRec{0.0, 0.0, 0.0, 0.0};
    const int my_slot = Multi && active ? (int)(key >> kEnsSlotShift) : 0;
    const uint32_t mkey = Multi ? ((key >> kSliceBits) & kEnsMortonMask) : (key >> g0.zbits);
    const int myc[3] = {(int)compact3(mkey), (int)compact3(mkey >> 1),
                        (int)compact3(mkey >> 2)};
    if (entry & 0x80000000u) {
        // a union too large for the masks (its particles are of one run)
        const uint32_t *bm = mask_scratch + tile * (kMaxWords * kWave);
        const int nu = (int)__builtin_amdgcn_readfirstlane(bm[3 * kDenseCells]);
        const int slot0 = __builtin_amdgcn_readfirstlane(my_slot);
        const Grid &g = Multi ? b.runs[slot0].grid : g0;
        bool wrap = false, few_cells = false;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            if (!g.periodic[a]) continue;
            int mn = active ? myc[a] : INT_MAX, mx = active ? myc[a] : INT_MIN;
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) {
                mn = min(mn, __shfl_xor(mn, o, kWave));
                mx = max(mx, __shfl_xor(mx, o, kWave));
            }
            if (mn < 1 || mx > g.nc[a] - 2 || 2 * (mx - mn + 3) >= g.nc[a]) wrap = true;
            if (g.nc[a] < 5) few_cells = true;
        }
        const bool uniform_h = Multi ? b.runs[slot0].uniform_h != 0 : hflag[0] == 0;
        const int mode = !wrap ? WRAP_NONE : (few_cells ? WRAP_PAIR : WRAP_CELL);
        const int2 *gc = reinterpret_cast<const int2 *>(bm);
        const uint32_t *gx = bm + 2 * kDenseCells;
        int2 r0 = make_int2(0, 0), r1 = make_int2(0, 0);
        uint32_t p0 = 0u, p1 = 0u;
        if (lane < nu) {
            r0 = gc[lane];
            p0 = gx[lane];
        }
        if (lane + kWave < nu) {
            r1 = gc[lane + kWave];
            p1 = gx[lane + kWave];
        }
        if (!Multi && mode == WRAP_NONE && g.zbits > 0) {
            // walk only each cell's window (single run: the cell table
            // carries the cells' largest (2h)^2)
            const double mc[3] = {me.x, me.y, me.z};
            double tlo[3], thi[3];
            double s2t = active ? me.s2 : 0.0;
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                tlo[a] = active ? mc[a] : INFINITY;
                thi[a] = active ? mc[a] : -INFINITY;
            }
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) {
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    tlo[a] = fmin(tlo[a], __shfl_xor(tlo[a], o, kWave));
                    thi[a] = fmax(thi[a], __shfl_xor(thi[a], o, kWave));
                }
                s2t = fmax(s2t, __shfl_xor(s2t, o, kWave));
            }
            if (lane < nu) r0 = z_window(r0, p0, g, tlo, thi, s2t, s2max, keys);
            if (lane + kWave < nu) r1 = z_window(r1, p1, g, tlo, thi, s2t, s2max, keys);
        }
        int cnt;
#define SPH_DIRECT(M, U) \
    stream_direct<M, U>(me, myc, srec, r0, r1, p0, p1, nu, g, active, i, ld, max_nb, idx)
        if (mode == WRAP_NONE) cnt = uniform_h ? SPH_DIRECT(WRAP_NONE, true) : SPH_DIRECT(WRAP_NONE, false);
        else if (mode == WRAP_CELL) cnt = uniform_h ? SPH_DIRECT(WRAP_CELL, true) : SPH_DIRECT(WRAP_CELL, false);
        else cnt = uniform_h ? SPH_DIRECT(WRAP_PAIR, true) : SPH_DIRECT(WRAP_PAIR, false);
#undef SPH_DIRECT
        if (active) {
            count[i] = cnt;
            if (cnt > max_nb) atomicOr(Multi ? &b.status[slot0] : status0, ST_CAPACITY);
        }
        continue;
    }
    if (!active) continue;
    const Grid &gl = Multi ? b.runs[my_slot].grid : g0;
    const int64_t cbl = Multi ? (int64_t)b.runs[my_slot].cell_base : 0;
    const double no_shift[3] = {0.0, 0.0, 0.0};
    uint32_t ks[32];
#pragma unroll
    for (int s = 0; s < 32; ++s) {
        ks[s] = 0xFFFFFFFFu;
        if (s < kStencil) {
            bool okx, oky, okz;
            const int x = wrap_or_clip(myc[0] + s % 3 - 1, gl.nc[0], gl.periodic[0], okx);
            const int y = wrap_or_clip(myc[1] + (s / 3) % 3 - 1, gl.nc[1], gl.periodic[1], oky);
            const int z = wrap_or_clip(myc[2] + s / 9 - 1, gl.nc[2], gl.periodic[2], okz);
            if (okx && oky && okz)
                ks[s] = spread3((uint32_t)x) | (spread3((uint32_t)y) << 1) |
                        (spread3((uint32_t)z) << 2);
        }
    }
    // bitonic sorting network over the 32 registers (indices are constants)
#pragma unroll
    for (int k = 2; k <= 32; k <<= 1) {
#pragma unroll
        for (int j = k >> 1; j > 0; j >>= 1) {
#pragma unroll
            for (int t = 0; t < 32; ++t) {
                const int p = t ^ j;
                if (p > t) {
                    const uint32_t lo = min(ks[t], ks[p]), hi = max(ks[t], ks[p]);
                    const bool up = (t & k) == 0;
                    ks[t] = up ? lo : hi;
                    ks[p] = up ? hi : lo;
                }
            }
        }
    }
    int cnt = 0;
    const int32_t ii = (int32_t)i;
    uint32_t prev_key = 0xFFFFFFFFu;
#pragma unroll 1
    for (int s = 0; s < kStencil; ++s) {
        const uint32_t kc = ks[s];
        if (kc == 0xFFFFFFFFu) break;
        if (kc == prev_key) continue;  // a short periodic axis lists a cell twice
        prev_key = kc;
        const int x = (int)compact3(kc), y = (int)compact3(kc >> 1), z = (int)compact3(kc >> 2);
        const int64_t cell = cbl + ((int64_t)z * gl.nc[1] + y) * gl.nc[0] + x;
        const int a = cstart[cell], e = cend[cell];
        if (a >= e) continue;
        SearchRec nx = srec[a];
        for (int32_t j = a; j < e; ++j) {
            const SearchRec o = nx;
            if (j + 1 < e) nx = srec[j + 1];
            if (related<WRAP_PAIR, false>(me, o, gl, no_shift) && j != ii) {
                if (cnt < max_nb) idx[(int64_t)cnt * ld + i] = j;
                ++cnt;
            }
        }
    }
    count[i] = cnt;
    if (cnt > max_nb) atomicOr(Multi ? &b.status[my_slot] : status0, ST_CAPACITY);
    }
}

__global__ void clear_count_kernel(uint32_t *c) { *c = 0u; }


// At most 96 SGPRs (a few spill to VGPR lanes): 8 waves per SIMD instead of
// the 7 that the compiler's own choice allows; the stream is latency-bound.
template <bool Multi>
__global__ void __launch_bounds__(kBlock) __attribute__((amdgpu_num_sgpr(96)))
find_neighbors_kernel(int64_t n, int64_t ld, const SearchRec *__restrict__ srec,
                      const uint32_t *__restrict__ keys, const int32_t *__restrict__ cstart,
                      const int32_t *__restrict__ cend, Grid g, int max_nb,
                      int32_t *__restrict__ count, int32_t *__restrict__ idx,
                      uint32_t *__restrict__ mask_scratch, const uint32_t *__restrict__ hflag,
                      uint32_t *status, BatchDev b, int32_t *__restrict__ fb_tiles,
                      uint32_t *fb_count, StepMask mask,
                      const unsigned long long *__restrict__ s2max)
{
    __shared__ SearchLds<kEntries> lds[kWavesPerBlock];
    const int w = threadIdx.x / kWave;
    SearchLds<kEntries> &L = lds[w];
    const int64_t nn = Multi ? b.hdr->n_out : n;
    int64_t tile;
    if constexpr (Multi) {
        // The grid covers the capacity's tiles, the step uses the first
        // ntile: their blocks are spread over the eight XCDs, the rest exit.
        const int64_t ntile = b.hdr->ntile;
        const int64_t bt = xcd_used_block((ntile + kWavesPerBlock - 1) / kWavesPerBlock);
        if (bt < 0) return;
        tile = bt * kWavesPerBlock + w;
        if (tile >= ntile) return;
    } else {
        tile = xcd_block() * kWavesPerBlock + w;
        if (tile >= (nn + kWave - 1) / kWave) return;
        if (mask.bin) {
            // individual time steps: only tiles holding a particle whose step
            // closes need lists (the others keep their stale ones, unread)
            const int64_t i = tile * kWave + (threadIdx.x & (kWave - 1));
            if (__ballot(i < nn && step_closes(mask, i)) == 0ull) return;
        }
    }
    search_tile<Multi>(tile, nn, ld, srec, keys, cstart, cend, g, max_nb, count, idx,
                       mask_scratch, hflag, status, b, L, fb_tiles, fb_count, s2max);
}


// ---------------------------------------------------------------------------
// Smoothing-length iteration (Algorithm 1, step 2, "neighbours and smoothing
// length"; Sec. 3, target neighbour count): gather counts
// N_i = #{j != i : r^2 < (2 h_i)^2}, the number of particles outside the
// accepted band, and the update of h with a cube root computed by a fixed
// rule of IEEE operations (cbrt_newton), so that any implementation of the
// same rule gets the same h.

// Offsets -k..k on one axis, without repeating a cell when a periodic axis
// has fewer than 2k + 1 cells.
__device__ __forceinline__ int axis_offsets(int nc, int periodic, int k, int (&off)[5])
{
    if (periodic && nc < 2 * k + 1) {
        for (int d = 0; d < nc; ++d) off[d] = d;
        return nc;
    }
    for (int d = -k; d <= k; ++d) off[d + k] = d;
    return 2 * k + 1;
}

// Words of the on-device iteration (ctx->it_words): [0] nonzero when a
// particle is outside the band, [1] length of the list of particles that the
// next sweep counts with lane groups, [2] done (the last sweep's counts are final),
// [3] sweeps counted, [4] a particle outside the grid's reach (2 h > 2
// cells): the host rebuilds the cells and continues.
enum { IT_BAD = 0, IT_NLIST = 1, IT_DONE = 2, IT_SWEEP = 3, IT_REACH = 4, IT_WORDS = 5 };

// After the first sweep on a cell build, a wave whose particles include
// fewer than kSweepDense to recount leaves them to the lane-group kernel
// (its slowest lane would set its time); kSweepGroup lanes share each such
// particle's cells.
constexpr int kSweepDense = 32;
constexpr int kSweepGroup = 32;

// Gather count of the lane's particle over the particles [w.x, w.y): the
// records are loaded four at a time, so that a test waits for its load once
// per four (a record per iteration left each test waiting for its own load;
// the next four in flight as well cost the kernel half its occupancy).
template <int Mode>
__device__ __forceinline__ int count_window(const SearchRec &me, const SearchRec *__restrict__ srec,
                                            int2 w, int self, const Grid &g,
                                            const double (&sh)[3])
{
    int cnt = 0;
    auto test = [&](const SearchRec &o, int j) {
        cnt += (j != self && related<Mode, true>(me, o, g, sh)) ? 1 : 0;
    };
    int j = w.x;
    for (; w.y - j >= 4; j += 4) {
        const SearchRec a0 = srec[j], a1 = srec[j + 1], a2 = srec[j + 2], a3 = srec[j + 3];
        test(a0, j);
        test(a1, j + 1);
        test(a2, j + 2);
        test(a3, j + 3);
    }
    for (; j < w.y; ++j) test(srec[j], j);
    return cnt;
}

// Gather counts of one sweep: N_i = #{j != i : r^2 < (2 h_i)^2}. The cells
// were built for a largest h that the sweeps may outgrow: a particle with
// 2 h_i up to two cells walks the 5^3 cells around its own, beyond that the
// sweep raises IT_REACH and counts nothing. Each cell reached without a
// periodic image is walked only in its window for the own sphere (a point
// box of reach 2 h_i): cells beyond it in x or y are skipped, in the others
// only the z slices within reach. Does nothing once IT_DONE or IT_REACH is
// set. Periodic: some axis of the box is periodic (then each pair takes the
// minimum image; else the separation is used as it is).
// recount_all = 0 (every sweep after the first of a run of sweeps on one
// cell build): a particle whose previous count was inside the band kept its
// h, so its count cannot change; a wave holding fewer than kSweepDense
// particles to recount keeps its counts and exits (after the first sweeps
// most waves do), its particles to recount being on the lane-group list.
template <bool Periodic>
__global__ void __launch_bounds__(256)
gather_count_kernel(int64_t n, const SearchRec *__restrict__ srec,
                    const uint32_t *__restrict__ keys, const int32_t *__restrict__ cstart,
                    const int32_t *__restrict__ cend, Grid g, int32_t *__restrict__ count,
                    int32_t lo_count, int32_t hi_count, uint32_t *words, int recount_all)
{
    if (words[IT_DONE] || words[IT_REACH]) return;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    bool active = i < n;
    if (!recount_all) {
        const int prev = active ? count[i] : lo_count;
        const uint64_t redo = __ballot(prev < lo_count || prev > hi_count);
        if (__popcll(redo) < kSweepDense) return;  // the whole wave
    }
    const SearchRec me = active ? srec[i] : SearchRec{0.0, 0.0, 0.0, 0.0};
    const double R = sqrt(me.s2);
    int k[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const double reach = R * g.inv_s[a] * (1.0 + 1e-12);
        k[a] = reach <= 1.0 ? 1 : (reach <= 2.0 ? 2 : 3);
    }
    const bool outgrown = active && (k[0] > 2 || k[1] > 2 || k[2] > 2);
    if (__ballot(outgrown) != 0ull) {
        if ((threadIdx.x & 63) == 0) atomicOr(&words[IT_REACH], 1u);
        return;  // (the whole wave: the sweep is discarded)
    }
    int cnt = 0;
    if (active) {
        const uint32_t key = keys[i] >> g.zbits;
        const int myc[3] = {(int)compact3(key), (int)compact3(key >> 1),
                            (int)compact3(key >> 2)};
        int ox[5], oy[5], oz[5];
        const int nx = axis_offsets(g.nc[0], g.periodic[0], k[0], ox);
        const int ny = axis_offsets(g.nc[1], g.periodic[1], k[1], oy);
        const int nz = axis_offsets(g.nc[2], g.periodic[2], k[2], oz);
        const double no_shift[3] = {0.0, 0.0, 0.0};
        const double pt[3] = {me.x, me.y, me.z};
        // a periodic axis with fewer than 2k + 1 cells: every cell, once
        const bool all_x = g.periodic[0] && g.nc[0] < 2 * k[0] + 1;
        const bool all_y = g.periodic[1] && g.nc[1] < 2 * k[1] + 1;
        const bool all_z = g.periodic[2] && g.nc[2] < 2 * k[2] + 1;
        for (int c = 0; c < nz; ++c) {
            bool okz = true;
            const int zr = all_z ? oz[c] : myc[2] + oz[c];
            const int z = all_z ? zr : wrap_or_clip(zr, g.nc[2], g.periodic[2], okz);
            if (!okz) continue;
            for (int b = 0; b < ny; ++b) {
                bool oky = true;
                const int yr = all_y ? oy[b] : myc[1] + oy[b];
                const int y = all_y ? yr : wrap_or_clip(yr, g.nc[1], g.periodic[1], oky);
                if (!oky) continue;
                for (int a = 0; a < nx; ++a) {
                    bool okx = true;
                    const int xr = all_x ? ox[a] : myc[0] + ox[a];
                    const int x = all_x ? xr : wrap_or_clip(xr, g.nc[0], g.periodic[0], okx);
                    if (!okx) continue;
                    const int64_t cell = ((int64_t)z * g.nc[1] + y) * g.nc[0] + x;
                    int2 w = make_int2(cstart[cell], cend[cell]);
                    // reached without a periodic image: only the window
                    const bool direct = !all_x && !all_y && !all_z && x == xr && y == yr &&
                                        z == zr;
                    if (direct && g.zbits > 0)
                        w = z_window_r(w, (uint32_t)x | ((uint32_t)y << 10) |
                                              ((uint32_t)z << 20),
                                       g, pt, pt, R, keys);
                    cnt += count_window<Periodic ? WRAP_PAIR : WRAP_NONE>(me, srec, w, (int)i,
                                                                           g, no_shift);
                }
            }
        }
        count[i] = cnt;
    }
    // Only whether some particle is outside the band matters: a wave with
    // one sets the flag unless it is already set. (An atomic from every wave
    // to the one word serialises in its L2 channel: ~10 ns each.) The word
    // is only ever set within a sweep, so a stale read costs one atomic.
    const uint64_t bad = __ballot(active && (cnt < lo_count || cnt > hi_count));
    if ((threadIdx.x & 63) == 0 && bad &&
        __hip_atomic_load(&words[IT_BAD], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0u)
        atomicOr(&words[IT_BAD], 1u);
}

// End of a sweep (one thread): the counts of this sweep are final when every
// particle is inside the band or this is sweep max_iter; else the h update
// follows. Clears the band flag for the next sweep.
__global__ void sweep_end_kernel(uint32_t *words, int32_t max_iter)
{
    if (words[IT_DONE] || words[IT_REACH]) return;
    if (words[IT_BAD] == 0 || (int32_t)words[IT_SWEEP] == max_iter) words[IT_DONE] = 1u;
    else words[IT_SWEEP] += 1u;
    words[IT_BAD] = 0u;
    words[IT_NLIST] = 0u;
}

// Cube root of a > 0 by Newton's iteration for y^3 = a in correctly rounded
// IEEE operations only, so that every implementation that performs the same
// operations gets the same number: a is brought into [1, 8) by exact
// factors of 8, y starts at 3/2 and takes seven steps y <- (2 y + a / y^2) / 3
// (the relative error 1/2 of the start squares at each step), and the
// result is scaled back by the matching power of 2.
__device__ __forceinline__ double cbrt_newton(double a)
{
    int k = 0;
    while (a >= 8.0) {
        a *= 0.125;
        ++k;
    }
    while (a < 1.0) {
        a *= 8.0;
        --k;
    }
    double y = 1.5;
    for (int t = 0; t < 7; ++t) y = (2.0 * y + a / (y * y)) / 3.0;
    return ldexp(y, k);
}

// h <- 2 h for an empty sphere, else (h / 2) (1 + (n_target / N)^(1/3)), for
// the particles outside the band; their search records take the new
// (2 h)^2. Does nothing once the counts are final.
// The updated particles of a wave with fewer than kSweepDense of them go on
// the list of the next sweep's lane-group kernel (list, words[IT_NLIST],
// cleared by the sweep's end; one atomic per block).
__global__ void __launch_bounds__(256)
update_h_kernel(int64_t n, const int32_t *__restrict__ count, double *__restrict__ h,
                SearchRec *__restrict__ srec, int32_t lo_count, int32_t hi_count,
                double n_target, uint32_t *words, int32_t *__restrict__ list)
{
    if (words[IT_DONE] || words[IT_REACH]) return;
    __shared__ uint32_t s_cnt[4];
    __shared__ uint32_t s_base;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int c = i < n ? count[i] : lo_count;
    const bool upd = c < lo_count || c > hi_count;
    if (upd) {
        const double hn = c == 0 ? 2.0 * h[i]
                                 : (h[i] * 0.5) * (1.0 + cbrt_newton(n_target / (double)c));
        h[i] = hn;
        const double s = 2.0 * hn;
        srec[i].s2 = s * s;
    }
    const uint64_t m = __ballot(upd);
    const uint32_t nw = (uint32_t)__popcll(m);
    const uint32_t listed = nw < (uint32_t)kSweepDense ? nw : 0u;
    if (lane == 0) s_cnt[wave] = listed;
    __syncthreads();
    if (threadIdx.x == 0) {
        const uint32_t tot = s_cnt[0] + s_cnt[1] + s_cnt[2] + s_cnt[3];
        s_base = tot ? atomicAdd(&words[IT_NLIST], tot) : 0u;
    }
    __syncthreads();
    if (listed && upd) {
        uint32_t off = s_base;
        for (int w = 0; w < wave; ++w) off += s_cnt[w];
        off += (uint32_t)__popcll(m & ((1ull << lane) - 1ull));
        list[off] = (int32_t)i;
    }
}

// Gather counts of the listed particles (the lane-group half of a sweep):
// kSweepGroup lanes per particle, which take its cells in turn and add
// their counts. Same cells, windows and test as gather_count_kernel.
template <bool Periodic>
__global__ void __launch_bounds__(256)
gather_count_list_kernel(const int32_t *__restrict__ list, const SearchRec *__restrict__ srec,
                         const uint32_t *__restrict__ keys, const int32_t *__restrict__ cstart,
                         const int32_t *__restrict__ cend, Grid g, int32_t *__restrict__ count,
                         int32_t lo_count, int32_t hi_count, uint32_t *words)
{
    if (words[IT_DONE] || words[IT_REACH]) return;
    const int64_t nl = words[IT_NLIST];
    const int sub = threadIdx.x % kSweepGroup;
    const int64_t groups = (int64_t)gridDim.x * (blockDim.x / kSweepGroup);
    for (int64_t e = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kSweepGroup; e < nl;
         e += groups) {
        const int64_t i = list[e];
        const SearchRec me = srec[i];
        const double R = sqrt(me.s2);
        int k[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const double reach = R * g.inv_s[a] * (1.0 + 1e-12);
            k[a] = reach <= 1.0 ? 1 : (reach <= 2.0 ? 2 : 3);
        }
        if (k[0] > 2 || k[1] > 2 || k[2] > 2) {
            if (sub == 0) atomicOr(&words[IT_REACH], 1u);
            continue;  // (the sweep is discarded)
        }
        const uint32_t key = keys[i] >> g.zbits;
        const int myc[3] = {(int)compact3(key), (int)compact3(key >> 1), (int)compact3(key >> 2)};
        int ox[5], oy[5], oz[5];
        const int nx = axis_offsets(g.nc[0], g.periodic[0], k[0], ox);
        const int ny = axis_offsets(g.nc[1], g.periodic[1], k[1], oy);
        const int nz = axis_offsets(g.nc[2], g.periodic[2], k[2], oz);
        const double no_shift[3] = {0.0, 0.0, 0.0};
        const double pt[3] = {me.x, me.y, me.z};
        const bool all_x = g.periodic[0] && g.nc[0] < 2 * k[0] + 1;
        const bool all_y = g.periodic[1] && g.nc[1] < 2 * k[1] + 1;
        const bool all_z = g.periodic[2] && g.nc[2] < 2 * k[2] + 1;
        int cnt = 0;
        for (int f = sub; f < nx * ny * nz; f += kSweepGroup) {
            const int c = f / (nx * ny), bb = (f / nx) % ny, a = f % nx;
            bool okx = true, oky = true, okz = true;
            const int zr = all_z ? oz[c] : myc[2] + oz[c];
            const int z = all_z ? zr : wrap_or_clip(zr, g.nc[2], g.periodic[2], okz);
            const int yr = all_y ? oy[bb] : myc[1] + oy[bb];
            const int y = all_y ? yr : wrap_or_clip(yr, g.nc[1], g.periodic[1], oky);
            const int xr = all_x ? ox[a] : myc[0] + ox[a];
            const int x = all_x ? xr : wrap_or_clip(xr, g.nc[0], g.periodic[0], okx);
            if (!okx || !oky || !okz) continue;
            const int64_t cell = ((int64_t)z * g.nc[1] + y) * g.nc[0] + x;
            int2 w = make_int2(cstart[cell], cend[cell]);
            const bool direct = !all_x && !all_y && !all_z && x == xr && y == yr && z == zr;
            if (direct && g.zbits > 0)
                w = z_window_r(w, (uint32_t)x | ((uint32_t)y << 10) | ((uint32_t)z << 20), g, pt,
                               pt, R, keys);
            cnt += count_window<Periodic ? WRAP_PAIR : WRAP_NONE>(me, srec, w, (int)i, g,
                                                                   no_shift);
        }
#pragma unroll
        for (int o = kSweepGroup / 2; o > 0; o >>= 1) cnt += __shfl_xor(cnt, o, kSweepGroup);
        if (sub == 0) {
            count[i] = cnt;
            if ((cnt < lo_count || cnt > hi_count) &&
                __hip_atomic_load(&words[IT_BAD], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) ==
                    0u)
                atomicOr(&words[IT_BAD], 1u);
        }
    }
}

// Largest h, as the ordered bit patterns of positive doubles.
__global__ void __launch_bounds__(256)
max_h_kernel(int64_t n, const double *__restrict__ h, unsigned long long *out)
{
    unsigned long long m = 0;
    const int64_t step = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += step) {
        const unsigned long long v = (unsigned long long)__double_as_longlong(h[i]);
        m = v > m ? v : m;
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const unsigned long long t = __shfl_xor(m, o, 64);
        m = t > m ? t : m;
    }
    // one atomic per block, and none when the word already holds as much
    // (atomics on one word serialise in its L2 channel)
    __shared__ unsigned long long wmax[4];
    if ((threadIdx.x & 63) == 0) wmax[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < 4; ++w) m = wmax[w] > m ? wmax[w] : m;
        if (m > __hip_atomic_load(out, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
            atomicMax(out, m);
    }
}

__global__ void clear_words_kernel(uint32_t *a, int k)
{
    if ((int)threadIdx.x < k) a[threadIdx.x] = 0u;
}

__global__ void set_word_kernel(uint32_t *a, uint32_t v) { *a = v; }

}  // namespace

hipError_t launch_find_neighbors(sph_ctx ctx, const sph_particles &p, const sph_nbrs &nb,
                                 const StepMask &mask)
{
    const int64_t tiles = (p.n + kWave - 1) / kWave;
    const unsigned blocks = (unsigned)((tiles + kWavesPerBlock - 1) / kWavesPerBlock);
    clear_count_kernel<<<1, 1, 0, ctx->stream>>>(ctx->fb_count);
    int tk = ktime_begin(ctx, TK_FIND_NEIGHBORS);
    find_neighbors_kernel<false><<<blocks, kBlock, 0, ctx->stream>>>(
        p.n, p.n, ctx->srec, ctx->sorted_keys, ctx->cell_start, ctx->cell_end, ctx->grid,
        nb.max_nb, nb.count, nb.idx, ctx->nb_mask, ctx->hflag_dev, ctx->status_dev, BatchDev{},
        ctx->fb_tiles, ctx->fb_count, mask,
        reinterpret_cast<const unsigned long long *>(ctx->cell_s2max));
    ktime_end(ctx, tk);
    const unsigned fblocks = (unsigned)std::min<int64_t>(tiles, kFallbackBlocks);
    tk = ktime_begin(ctx, TK_FALLBACK);
    fallback_kernel<false><<<fblocks, kWave, 0, ctx->stream>>>(
        p.n, p.n, ctx->srec, ctx->sorted_keys, ctx->cell_start, ctx->cell_end, ctx->grid,
        nb.max_nb, nb.count, nb.idx, ctx->status_dev, BatchDev{}, ctx->fb_tiles, ctx->fb_count,
        ctx->nb_mask, ctx->hflag_dev,
        reinterpret_cast<const unsigned long long *>(ctx->cell_s2max));
    ktime_end(ctx, tk);
    return hipGetLastError();
}

hipError_t launch_find_neighbors_batch(sph_ctx ctx, const BatchDev &b, int max_nb,
                                       int32_t *count, int32_t *idx)
{
    // the mask scratch holds one region per tile: the capacity's, plus at
    // most one partial tile per run (each run is cut into its own tiles)
    const int64_t tiles = (b.cap + kWave - 1) / kWave + kEnsMaxSlots;
    const unsigned blocks = (unsigned)((tiles + kWavesPerBlock - 1) / kWavesPerBlock);
    clear_count_kernel<<<1, 1, 0, ctx->stream>>>(ctx->fb_count);
    find_neighbors_kernel<true><<<blocks, kBlock, 0, ctx->stream>>>(
        0, b.cap, ctx->srec, ctx->sorted_keys, ctx->cell_start, ctx->cell_end, Grid{}, max_nb,
        count, idx, ctx->nb_mask, nullptr, nullptr, b, ctx->fb_tiles, ctx->fb_count,
        StepMask{}, nullptr);
    const unsigned fblocks = (unsigned)std::min<int64_t>(tiles, kFallbackBlocks);
    fallback_kernel<true><<<fblocks, kWave, 0, ctx->stream>>>(
        0, b.cap, ctx->srec, ctx->sorted_keys, ctx->cell_start, ctx->cell_end, Grid{}, max_nb,
        count, idx, nullptr, b, ctx->fb_tiles, ctx->fb_count, ctx->nb_mask, nullptr, nullptr);
    return hipGetLastError();
}

hipError_t launch_max_h(sph_ctx ctx, const sph_particles &p, unsigned long long *out)
{
    clear_words_kernel<<<1, 64, 0, ctx->stream>>>(reinterpret_cast<uint32_t *>(out), 2);
    const unsigned blocks = (unsigned)std::min<int64_t>((p.n + 255) / 256, 512);
    max_h_kernel<<<blocks, 256, 0, ctx->stream>>>(p.n, p.h, out);
    return hipGetLastError();
}

static void launch_gather(sph_ctx ctx, const sph_particles &p, int32_t *count, int32_t lo_count,
                   int32_t hi_count, uint32_t *words, unsigned blocks, int recount_all)
{
    const Grid &g = ctx->grid;
    // the list kernel's grid: enough lane groups for the lists of the late
    // sweeps (a few thousand particles), the rest loop. The list lives in
    // the reorder scratch's id array (n_max entries), which no kernel uses
    // between two cell builds.
    const unsigned lblocks = std::min<unsigned>(blocks, 1024u);
    if (g.periodic[0] || g.periodic[1] || g.periodic[2]) {
        gather_count_kernel<true><<<blocks, 256, 0, ctx->stream>>>(
            p.n, ctx->srec, ctx->sorted_keys, ctx->cell_start, ctx->cell_end, g, count,
            lo_count, hi_count, words, recount_all);
        gather_count_list_kernel<true><<<lblocks, 256, 0, ctx->stream>>>(
            ctx->perm_tmp_id, ctx->srec, ctx->sorted_keys, ctx->cell_start, ctx->cell_end, g,
            count, lo_count, hi_count, words);
    } else {
        gather_count_kernel<false><<<blocks, 256, 0, ctx->stream>>>(
            p.n, ctx->srec, ctx->sorted_keys, ctx->cell_start, ctx->cell_end, g, count,
            lo_count, hi_count, words, recount_all);
        gather_count_list_kernel<false><<<lblocks, 256, 0, ctx->stream>>>(
            ctx->perm_tmp_id, ctx->srec, ctx->sorted_keys, ctx->cell_start, ctx->cell_end, g,
            count, lo_count, hi_count, words);
    }
}

hipError_t launch_h_iteration(sph_ctx ctx, const sph_particles &p, int32_t *count,
                              int32_t lo_count, int32_t hi_count, double n_target,
                              int32_t first_sweep, int32_t max_iter, uint32_t *words)
{
    // words: IT_WORDS counters, cleared here; sweeps counted from first_sweep
    clear_words_kernel<<<1, 64, 0, ctx->stream>>>(words, IT_WORDS);
    set_word_kernel<<<1, 1, 0, ctx->stream>>>(words + IT_SWEEP, (uint32_t)first_sweep);
    const unsigned blocks = (unsigned)((p.n + 255) / 256);
    for (int32_t it = first_sweep; it <= max_iter; ++it) {
        // the first sweep on these cells counts every particle (the counts
        // in memory may belong to another order); later ones only recount
        // the waves holding a particle whose h was just updated
        launch_gather(ctx, p, count, lo_count, hi_count, words, blocks, it == first_sweep);
        sweep_end_kernel<<<1, 1, 0, ctx->stream>>>(words, max_iter);
        if (it < max_iter)
            update_h_kernel<<<blocks, 256, 0, ctx->stream>>>(p.n, count, p.h, ctx->srec,
                                                            lo_count, hi_count, n_target,
                                                            words, ctx->perm_tmp_id);
    }
    return hipGetLastError();
}

}  // namespace sph
