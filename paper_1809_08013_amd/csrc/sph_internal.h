// Internal declarations of libsph shared by its translation units.
// Not installed, not part of the C ABI (include/sph.h is).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "sph.h"

namespace sph {

// Status bits raised on the device; sph_ctx_check maps them to sph_status.
enum : uint32_t {
    ST_CAPACITY = 1u << 0,
    ST_DOMAIN = 1u << 1,
    ST_NONFINITE = 1u << 2,
};

constexpr int kMaxAxisCells = 1024;   // 10 Morton bits per axis
constexpr int kRadixBits = 8;
constexpr int kRadixBins = 1 << kRadixBits;
constexpr int kSortThreads = 256;
constexpr int kSortItems = 8;
constexpr int kSortTile = kSortThreads * kSortItems;   // keys per tile
constexpr int kScanThreads = 256;
constexpr int kScanItems = 16;
constexpr int kScanChunk = kScanThreads * kScanItems;  // elements per block
constexpr int kRedThreads = 256;
constexpr int kRedMaxBlocks = 2048;
constexpr int kRedFields = 9;   // dt candidate min + 8 totals
constexpr int kPermFields = 25; // x y z vx vy vz u h m rho_ref p_bg gx gy gz xw + 10 extra

// Uniform cell grid of one build (host values, passed to kernels by value).
struct Grid {
    int nc[3];          // cells per axis
    int bits;           // Morton bits per axis
    int zbits;          // key bits below the cell's Morton code: the z slice in the cell
    int periodic[3];
    double lo[3];
    double hi[3];
    double len[3];      // hi - lo
    double half[3];     // 0.5 * len (minimum image threshold)
    double inv_s[3];    // cells per unit length
};

struct PermFields {
    double *f[kPermFields];
    int nf;
    int32_t *id;
    int32_t *slot;      // ensemble only: run slot of each particle (else null)
};

// Below a cell's Morton code the sort key holds the particle's z slice in the
// cell (at most kSliceBits bits), so that each cell's particles are ordered by
// z and a search can skip the slices out of reach.
constexpr int kSliceBits = 6;

// ---------------------------------------------------------------------------
// Ensemble (many independent runs in one arena).
//
// Key of a particle of run slot s:
//   (s << (3 kEnsAxisBits + kSliceBits)) | (Morton(cell) << kSliceBits) | slice,
// so one stable radix sort over kEnsKeyBits bits groups the particles by run
// and, inside a run, by cell and by z slice, exactly as the single-run sort
// does for the same run. A run being dropped gets the all-ones key and sorts
// behind every live particle.
constexpr int kEnsAxisBits = 5;                     // <= 32 cells per axis per run
constexpr int kEnsSlotBits = 9;
constexpr int kEnsMaxSlots = (1 << kEnsSlotBits) - 1;  // slot 511 is the drop key
constexpr int kEnsSlotShift = 3 * kEnsAxisBits + kSliceBits;
constexpr int kEnsKeyBits = kEnsSlotBits + kEnsSlotShift;
constexpr uint32_t kEnsMortonMask = (1u << (3 * kEnsAxisBits)) - 1u;
constexpr uint32_t kEnsDropKey = 0xFFFFFFFFu;
constexpr int kEnsFields = 11;  // x y z vx vy vz u h m p_bg rho_ref (rows of one block)

enum : int32_t { RUN_FREE = 0, RUN_INIT = 1, RUN_STEP = 2, RUN_DROP = 3 };

// Per-slot description of a run for the current step (host-written).
struct RunDev {
    Grid grid;
    double h_max;
    double rho0, c0, gamma_tait, gamma_gas, alpha, beta, eta2, c_cfl, c_force;
    int32_t eos;
    int32_t phase;        // RUN_*
    int32_t set_rho_ref;  // rho_ref := rho at the t = 0 evaluation
    int32_t uniform_h;    // every particle of the run has the same h
    int32_t cell_base;    // first entry of the run in the cell table
    int32_t ncell;
    int32_t start;        // first particle after this step's sort
    int32_t n;
    int32_t red_base;     // first reduction block of the run
    int32_t pad;
};

// Per-step header (host-written): counts, live runs in slot order, and the
// runs admitted before this step with the arena range they were copied to.
struct BatchHdr {
    int64_t n_in;    // particles before the sort (live + dropped + admitted)
    int64_t n_out;   // particles of live runs, after the sort
    int64_t ncell;   // cells of live runs
    int64_t nred;    // reduction blocks of live runs
    int64_t ntile;   // search tiles of live runs
    int32_t nlive;
    int32_t nnew;
    int32_t live_slot[kEnsMaxSlots];
    int32_t live_cell_base[kEnsMaxSlots + 1];
    int32_t live_red_base[kEnsMaxSlots + 1];
    // first search tile of each live run: a run's particles are cut into
    // tiles of 64 from its own first particle, so no tile holds two runs
    int32_t live_tile_base[kEnsMaxSlots + 1];
    int32_t new_slot[kEnsMaxSlots];
    int32_t new_off[kEnsMaxSlots];
    int32_t new_n[kEnsMaxSlots];
};

// Device pointers an ensemble step reads besides the particle arrays.
struct BatchDev {
    const BatchHdr *hdr;
    const RunDev *runs;
    int32_t *slot;       // per particle
    double *dt;          // per slot
    double *diag;        // 8 per slot
    uint32_t *status;    // per slot
    int64_t cap;         // particle capacity (ELL leading dimension)
    int64_t cell_cap;
    int64_t nred_cap;
};

constexpr int kStencil = 27;
constexpr int kSearchMaskWords = 88;  // per lane of a search wave: 2816 candidates

// Neighbour-side records, one per particle in cell order, so that a
// neighbour's data is one aligned block instead of one cache line per array.
//   SearchRec: position and (2h)^2 (the relation test), 32 B;
//   DensRec:   position and mass (density), 32 B;
//   PairRec:   position, velocity, h, 1/h, m, rho, c, P/rho^2 (momentum and
//              energy), 96 B padded to one 128-byte line.
struct __attribute__((aligned(32))) SearchRec { double x, y, z, s2; };
struct __attribute__((aligned(32))) DensRec { double x, y, z, m; };
struct __attribute__((aligned(128))) PairRec {
    double x, y, z, vx, vy, vz, h, inv_h, m, rho, c, pr2;
    double pad[4];
};
static_assert(sizeof(PairRec) == 128, "PairRec is one cache line");
// The FP32-pair form's momentum records: position and velocity in FP64 (the
// separations and velocity differences are formed in FP64, then rounded),
// h, 1/h, m, rho, c, P/rho^2 and the volume weights X, Q as FP32 copies:
// 48 + 32 = 80 B, five 16-byte chunks (with kernel derivatives; the IAD
// instances keep PairRec, their gradient being formed in FP64). Padded to
// one 128-byte line like PairRec: an 80-byte stride makes most records span
// two lines, and the gather then touches 1.6 lines per record instead of one
// (measured slower on the 1M patch: 0.83 against 0.73 ms).
struct __attribute__((aligned(128))) PairRec32 {
    double x, y, z, vx, vy, vz;
    float h, inv_h, m, rho, c, pr2, X, Q;
};
static_assert(sizeof(PairRec32) == 128, "PairRec32 is one cache line");

// Octree gravity node: centre of mass and opening radius s / theta + delta
// (the acceptance test), mass and traceless quadrupole (xx xy xz yy yz zz),
// the node's range of sorted positions, its children (contiguous, octant
// order; nchild = 0 for a leaf), Morton prefix and level.
struct __attribute__((aligned(128))) GNode {
    double cx, cy, cz, ropen;
    double M, q[6];
    double pad0;
    int32_t start, end, child0, nchild;
    uint32_t prefix;
    int32_t level;
    int32_t pad1[2];
};
static_assert(sizeof(GNode) == 128, "GNode is one cache line");

// Individual time steps: with bin set, a call works only on the particles
// of bin b whose step closes at substep sub of 2^B, ((sub + 1) mod 2^(B-b))
// == 0; the others are left as they are.
struct StepMask {
    const double *bin = nullptr;
    int sub = 0, B = 0;
};
__device__ __forceinline__ bool step_closes(const StepMask &m, int64_t i)
{
    if (!m.bin) return true;
    const int b = (int)m.bin[i];
    return ((m.sub + 1) & ((1 << (m.B - b)) - 1)) == 0;
}

// Block index remapped so that each XCD runs one contiguous range of blocks.
// Blocks are dispatched to the 8 XCDs round-robin (block b to XCD b % 8);
// giving XCD x the x-th contiguous slice keeps a Morton-contiguous region of
// particles, and most of its neighbours, in that XCD's L2.
__device__ __forceinline__ int64_t xcd_block()
{
    const uint32_t B = gridDim.x, b = blockIdx.x;
    const uint32_t q = B / 8, r = B % 8, x = b % 8, pos = b / 8;
    return x < r ? (int64_t)x * (q + 1) + pos
                 : (int64_t)r * (q + 1) + (int64_t)(x - r) * q + pos;
}

// xcd_block for a grid sized for a capacity of which a step uses only the
// first `used` blocks (a count read on the device): those blocks, which are
// dispatched first, are mapped as xcd_block maps a grid of `used` blocks, so
// the work is spread over all eight XCDs; the others get -1 and exit.
__device__ __forceinline__ int64_t xcd_used_block(int64_t used)
{
    const int64_t b = blockIdx.x;
    if (b >= used) return -1;
    const int64_t q = used / 8, r = used % 8, x = b % 8, pos = b / 8;
    return x < r ? x * (q + 1) + pos : r * (q + 1) + (x - r) * q + pos;
}

// First particle and end of 64-particle tile `tile` (one wave's particles
// in the search and pair kernels). One run: tiles of 64 from particle 0, the
// last one ending at n. An ensemble: each live run is cut into its own tiles
// from its first particle (the step header's tile bases), so that no tile
// holds particles of two runs and a wave's run parameters are uniform.
template <bool Multi>
__device__ __forceinline__ void tile_span(int64_t tile, int64_t n, const BatchDev &b,
                                          int64_t &t0, int64_t &tend)
{
    if constexpr (!Multi) {
        t0 = tile * 64;
        tend = min(t0 + (int64_t)64, n);
    } else {
        const BatchHdr *hd = b.hdr;
        int lo = 0, hi = hd->nlive - 1;
        while (lo < hi) {  // last live run whose first tile is <= tile
            const int mid = (lo + hi + 1) >> 1;
            if (hd->live_tile_base[mid] <= tile) lo = mid; else hi = mid - 1;
        }
        const RunDev &r = b.runs[hd->live_slot[lo]];
        t0 = (int64_t)r.start + (tile - hd->live_tile_base[lo]) * (int64_t)64;
        tend = min(t0 + (int64_t)64, (int64_t)r.start + r.n);
    }
}

// xcd_block, refined per CU: the blocks an XCD receives are handed out to
// its 32 CUs in turn, so block pos of the XCD is mapped to the pos / 32-th
// entry of CU pos % 32's own contiguous range. Blocks resident on one CU then
// work on neighbouring tiles and share their neighbours' records in its L1.
__device__ __forceinline__ int64_t xcd_cu_block()
{
    const uint32_t B = gridDim.x, b = blockIdx.x;
    const uint32_t q = B / 8, r = B % 8, x = b % 8, pos = b / 8;
    const uint32_t nb = q + (x < r ? 1u : 0u);  // blocks of this XCD
    const int64_t base = x < r ? (int64_t)x * (q + 1) : (int64_t)r * (q + 1) + (int64_t)(x - r) * q;
    constexpr uint32_t kCus = 32;
    const uint32_t qc = nb / kCus, rc = nb % kCus, c = pos % kCus, round = pos / kCus;
    return base + (int64_t)(c * qc + (c < rc ? c : rc)) + round;
}

}  // namespace sph

namespace sph {
// Live kernel timing (sph_ctx_timing): while on, the launches of the timed
// kernels are bracketed by two HIP events on the context's stream; the
// durations are summed when sph_ctx_kernel_time reads them.
enum TimedKernel {
    TK_FIND_NEIGHBORS = 0,  // find_neighbors_kernel
    TK_FALLBACK,            // fallback_kernel
    TK_DENSITY,             // density_kernel
    TK_IAD,                 // iad_kernel
    TK_MOMENTUM,            // momentum_kernel
    TK_COUNT
};
extern const char *const kTimedKernelNames[TK_COUNT];
struct KTimer {
    bool on = false;
    std::vector<hipEvent_t> pool;  // free events
    struct Pending {
        int id;
        hipEvent_t a, b;
    };
    std::vector<Pending> pending;
    double sum_ms[TK_COUNT] = {};
    int64_t launches[TK_COUNT] = {};
};
// Start/stop one timed launch (no-ops while timing is off or while a step is
// being captured). ktime_begin returns the pending slot or -1.
int ktime_begin(sph_ctx ctx, int id);
void ktime_end(sph_ctx ctx, int slot);
}  // namespace sph

struct sph_ctx_s {
    int device = 0;
    hipStream_t stream = nullptr;
    int64_t n_max = 0;
    int32_t max_nb = 0;

    // radix sort
    uint32_t *keys[2] = {nullptr, nullptr};
    int32_t *vals[2] = {nullptr, nullptr};
    uint32_t *hist = nullptr;        // kRadixBins * tiles_max
    uint32_t *scan_part = nullptr;   // block partials of the scan
    int64_t tiles_max = 0;
    int64_t scan_len_max = 0;
    const uint32_t *sorted_keys = nullptr;  // key of each particle after the build

    // cell table, indexed by linear cell id (cz * ny + cy) * nx + cx
    int32_t *cell_start = nullptr;
    int32_t *cell_end = nullptr;
    int64_t cell_cap = 0;
    uint32_t *nb_mask = nullptr;     // search bit masks: kSearchMaskWords words per particle slot
    double *cell_s2max = nullptr;    // per cell: largest (2h)^2 of its particles
    double *iad_c = nullptr;         // IAD matrices, 6 per particle (xx xy xz yy yz zz)
    int32_t *fb_tiles = nullptr;     // search tiles left to the per-lane path
    uint32_t *fb_count = nullptr;
    uint32_t *it_words = nullptr;    // h iteration: out-of-band count, largest count
    unsigned long long *it_hmax = nullptr;  // h iteration: largest h (bit pattern)

    sph::SearchRec *srec = nullptr;  // search records, cell order
    sph::DensRec *drec = nullptr;    // density records (written by sph_density)
    sph::PairRec *prec = nullptr;    // pair records (written by sph_momentum_energy)
    sph::Grid grid{};
    int64_t n_built = -1;

    // permutation scratch
    double *perm_tmp = nullptr;      // kPermFields * n_max
    int32_t *perm_tmp_id = nullptr;  // n_max; also the smoothing-length sweeps' list

    // reductions
    double *red_part = nullptr;      // kRedFields * kRedMaxBlocks

    // octree gravity: allocated by the first sph_gravity_tree call
    int64_t gt_n_cap = 0;            // particles the buffers hold
    int64_t gt_node_cap = 0;
    int64_t gt_fcap = 0;             // stack entries per wave
    int32_t gt_waves = 0;            // resident waves of the force kernel
    uint32_t *gt_keys[2] = {nullptr, nullptr};
    int32_t *gt_vals[2] = {nullptr, nullptr};
    sph::DensRec *gt_pos = nullptr;  // sorted {x, y, z, m}
    sph::GNode *gt_nodes = nullptr;
    int32_t *gt_lvl = nullptr;       // per level: first node, node count (2 x 12); groups
    int2 *gt_groups = nullptr;       // groups: first and end sorted position
    int32_t *gt_front = nullptr;     // per wave: a stack of gt_fcap nodes to visit
    uint32_t *gt_flags = nullptr;    // bit 0: node capacity, bit 1: stack capacity
    double *gt_box = nullptr;        // lo[3], L
    double *gt_part = nullptr;       // bounding-box partials

    // individual time steps: per-particle criterion, {min, max} partials,
    // deepest bin
    double *dtc = nullptr;
    uint32_t *blk_words = nullptr;

    // one captured sph_step (sph_step_capture / sph_step_replay)
    hipGraph_t step_graph = nullptr;
    hipGraphExec_t step_exec = nullptr;

    sph::KTimer timer;
    bool capturing = false;          // inside sph_step_capture

    uint32_t *status_dev = nullptr;
    uint32_t *hflag_dev = nullptr;   // 0 after a build iff every particle has the same h
    std::string last_error;
    int64_t scratch_bytes = 0;
};

namespace sph {

// Launchers (defined in the .hip files); each returns hipSuccess or the
// launch error.
// extra: up to 10 more per-particle FP64 arrays reordered with the particles.
hipError_t launch_build_cells(sph_ctx ctx, const sph_particles &p, const Grid &g,
                              double h_max, double *const *extra = nullptr, int n_extra = 0);
hipError_t launch_find_neighbors(sph_ctx ctx, const sph_particles &p,
                                 const sph_nbrs &nb, const StepMask &mask = StepMask{});
// The interpolation kernel of a pair call: family (SPH_KERNEL_*), sinc
// exponent, and sigma = W(0, h) h^3.
struct KernelSel {
    int family;
    int sinc_n;
    double sigma;
};
KernelSel kernel_sel(const sph_params &prm);

// gve: generalised volume elements with the weights p.xw.
hipError_t launch_density(sph_ctx ctx, const sph_particles &p, const sph_nbrs &nb,
                          int precision, const KernelSel &ks, bool gve, double *rho,
                          const StepMask &mask = StepMask{});
hipError_t launch_volume_weights(sph_ctx ctx, const sph_particles &p, const double *rho,
                                 double exponent);
// The density without allocation: the device address of the static record
// array on the current device (taken once per device and kept), and the
// density kernels run on it.
hipError_t density_noalloc_scratch(DensRec **out);
hipError_t launch_density_noalloc(hipStream_t stream, const sph_particles &p, const sph_nbrs &nb,
                                  const Grid &g, int precision, const KernelSel &ks, bool gve,
                                  double *rho, DensRec *recs);

hipError_t launch_gravity_direct(sph_ctx ctx, const sph_particles &p, double eps, double *gx,
                                 double *gy, double *gz);
// Octree gravity; *flags receives the capacity bits of the call (synchronises).
// Its buffers are allocated by the first call on a context and released by
// release_gravity_tree.
void release_gravity_tree(sph_ctx ctx);
hipError_t launch_gravity_tree(sph_ctx ctx, const sph_particles &p, double eps, double theta,
                               int leaf_size, double *gx, double *gy, double *gz,
                               uint32_t *flags);
// Stable LSD radix sort of (key, value) pairs in k[cur], v[cur] over the low
// key_bits bits, ping-ponging with k[cur ^ 1], v[cur ^ 1]; *cur is updated to
// the buffer holding the result. Uses the context's histogram and scan
// scratch (n <= n_max).
hipError_t radix_sort_pairs(sph_ctx ctx, uint32_t *k[2], int32_t *v[2], int64_t n,
                            int key_bits, int *cur);
hipError_t launch_eos(sph_ctx ctx, const sph_particles &p, const sph_params &prm,
                      const sph_fields &f, const StepMask &mask = StepMask{});
// bin (not null): only the particles whose step closes at substep sub of
// 2^B get new accelerations (individual time steps).
hipError_t launch_momentum(sph_ctx ctx, const sph_particles &p, const sph_nbrs &nb,
                           const sph_params &prm, const sph_fields &f,
                           const sph_accel &a, const double *bin = nullptr, int sub = 0,
                           int B = 0);
hipError_t launch_integrate(sph_ctx ctx, const sph_particles &p, const Grid &g,
                            int stage, const double *dt_dev, const sph_accel &a);
hipError_t launch_timestep(sph_ctx ctx, const sph_particles &p,
                           const sph_params &prm, const sph_fields &f,
                           const sph_accel &a, double *dt_dev, double *diag_dev);
hipError_t launch_copy(sph_ctx ctx, double *dst, const double *src, int64_t n);
// Individual time steps: per-particle criterion, the largest step D into
// dt_dev[0], the bins into bin (as doubles) and the deepest bin into
// ctx->blk_words[0].
hipError_t launch_block_bins(sph_ctx ctx, const sph_particles &p, const sph_params &prm,
                             const sph_fields &f, const sph_accel &a, int max_bin, double *bin,
                             double *dt_dev);
// Half kicks of the particles whose step opens (stage 0) or closes (stage 1)
// at substep sub of 2^B, and the drift of every particle by D / 2^B.
hipError_t launch_kick_bins(sph_ctx ctx, const sph_particles &p, int stage, int sub, int B,
                            const double *dt_dev, const double *bin, const sph_accel &a);
hipError_t launch_drift(sph_ctx ctx, const sph_particles &p, const Grid &g, int B,
                        const double *dt_dev);

Grid make_grid(const sph_box &b, double h_max, int64_t cell_cap, int max_axis);

// Smoothing-length iteration.
hipError_t launch_max_h(sph_ctx ctx, const sph_particles &p, unsigned long long *out);
// Sweeps first_sweep..max_iter of the count-based h iteration on the cells
// last built, on the device: counts, the band test and the h update, with no
// host work between sweeps. words (kItWords): [0] nonzero when a particle
// is outside the band, [1] length of the next sweep's list of particles
// counted by lane groups, [2] done, [3] last sweep, [4] a particle outgrew
// the cells (the host rebuilds and calls again from sweep [3]).
constexpr int kItWords = 5;
// Reorders an int32 per-particle array as the last cell build reordered the
// particles (its sort permutation).
hipError_t launch_permute_like_build(sph_ctx ctx, int32_t *a, int64_t n);
hipError_t launch_h_iteration(sph_ctx ctx, const sph_particles &p, int32_t *count,
                              int32_t lo_count, int32_t hi_count, double n_target,
                              int32_t first_sweep, int32_t max_iter, uint32_t *words);

// Ensemble launchers: fixed grids sized for b.cap; counts are read from the
// step header on the device. F is the block of kEnsFields state rows
// (x y z vx vy vz u h m p_bg rho_ref), each b.cap long.
hipError_t launch_admit_batch(sph_ctx ctx, const BatchDev &b);
hipError_t launch_build_cells_batch(sph_ctx ctx, const BatchDev &b, double *F, int32_t *id,
                                    int32_t *slot_tmp);
hipError_t launch_find_neighbors_batch(sph_ctx ctx, const BatchDev &b, int max_nb,
                                       int32_t *count, int32_t *idx);
hipError_t launch_density_batch(sph_ctx ctx, const BatchDev &b, int precision, const double *F,
                                const int32_t *count, const int32_t *idx, int max_nb,
                                double *rho);
hipError_t launch_eos_batch(sph_ctx ctx, const BatchDev &b, double *F, const double *rho,
                            double *p, double *c, double *pr2);
hipError_t launch_momentum_batch(sph_ctx ctx, const BatchDev &b, int precision,
                                 const double *F, const int32_t *count, const int32_t *idx,
                                 int max_nb, const double *rho, const double *c,
                                 const double *pr2, double *ax, double *ay, double *az,
                                 double *dudt, double *mumax);
hipError_t launch_integrate_batch(sph_ctx ctx, const BatchDev &b, int stage, double *F,
                                  const double *ax, const double *ay, const double *az,
                                  const double *dudt);
hipError_t launch_timestep_batch(sph_ctx ctx, const BatchDev &b, const double *F,
                                 const double *c, const double *mumax, const double *ax,
                                 const double *ay, const double *az, double *part);

}  // namespace sph
