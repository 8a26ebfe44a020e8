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
//
// The same sum approximated by a Morton octree with multipoles to quadrupole
// order (the parent codes' method; SPHYNX keeps quadrupoles), G = 1:
//   cube   lo_a = min_i x_a, L = max_a (max_i x_a - lo_a) (1 if zero);
//   keys   k_a = min(1023, floor((x_a - lo_a) / L * 1024)), 30-bit Morton
//          code; particles sorted by (key, id) (a stable radix sort of the
//          particles arranged by id);
//   nodes  the root holds all particles; a node of level l < 10 with more
//          than leaf_size particles gets one child per non-empty octant, in
//          octant order; side s = L / 2^l, centre lo + (k + 1/2) s;
//   moments M, centre of mass c and traceless quadrupole
//          Q_ab = sum m (3 d_a d_b - |d|^2 delta_ab), d = x - c; leaves sum
//          their particles in sorted order, internal nodes their children in
//          octant order with the parallel-axis shift;
//   groups the root if it holds at most 64 particles; else, for every node
//          with more than 64 particles, its children with at most 64 in
//          octant order, merged while the run holds at most 64 (a larger
//          child ends a run), and a finest-level leaf with more than 64 cut
//          into runs of 64; one wave each. A node N is accepted
//          for the whole group G when dist(c_N, box_G) > s_N / theta +
//          |c_N - centre_N|; otherwise a leaf is summed directly and an
//          internal node opened (the definition walks breadth-first; the
//          kernel visits the same nodes in stack order);
//   terms  direct -m_j d / (|d|^2 + eps^2)^{3/2} (j != i); node
//          -M d / r^3 + Q d / r^5 - 5/2 (d.Q d) d / r^7, d = x_i - c.
// Tree build and moments use plain FP64 operations in the order of their
// definition (no fused multiply-add; correctly rounded division and square
// root), so the tree and every acceptance decision are the definition's; the
// terms use fused multiply-adds and take 1/sqrt from the hardware estimate
// refined by two Newton steps (about one ulp).
#include <algorithm>
#include <cmath>

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


// ------------------------------------------------------------ octree gravity

constexpr int kGLevels = 10;       // key bits per axis
constexpr int kGBoxBlocks = 1024;  // bounding-box partial blocks (at most)

__device__ __forceinline__ uint32_t spread10(uint32_t v)
{
    v &= 0x3ffu;
    v = (v | (v << 16)) & 0x030000FFu;
    v = (v | (v << 8)) & 0x0300F00Fu;
    v = (v | (v << 4)) & 0x030C30C3u;
    v = (v | (v << 2)) & 0x09249249u;
    return v;
}

// per block: min x, y, z then max x, y, z (exact, so any order gives the same)
__global__ void __launch_bounds__(256)
gbox_partial_kernel(int64_t n, const double *__restrict__ x, const double *__restrict__ y,
                    const double *__restrict__ z, double *__restrict__ part)
{
    __shared__ double red[6][256];
    double v[6] = {INFINITY, INFINITY, INFINITY, -INFINITY, -INFINITY, -INFINITY};
    const int64_t step = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += step) {
        v[0] = fmin(v[0], x[i]);
        v[1] = fmin(v[1], y[i]);
        v[2] = fmin(v[2], z[i]);
        v[3] = fmax(v[3], x[i]);
        v[4] = fmax(v[4], y[i]);
        v[5] = fmax(v[5], z[i]);
    }
    for (int a = 0; a < 6; ++a) red[a][threadIdx.x] = v[a];
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w)
            for (int a = 0; a < 6; ++a)
                red[a][threadIdx.x] = a < 3 ? fmin(red[a][threadIdx.x], red[a][threadIdx.x + w])
                                            : fmax(red[a][threadIdx.x], red[a][threadIdx.x + w]);
        __syncthreads();
    }
    if (threadIdx.x == 0)
        for (int a = 0; a < 6; ++a) part[6 * blockIdx.x + a] = red[a][0];
}

// box = {lo_x, lo_y, lo_z, L}; one wave
__global__ void __launch_bounds__(64)
gbox_final_kernel(int nblk, const double *__restrict__ part, double *__restrict__ box)
{
    double v[6] = {INFINITY, INFINITY, INFINITY, -INFINITY, -INFINITY, -INFINITY};
    for (int b = threadIdx.x; b < nblk; b += 64)
        for (int a = 0; a < 6; ++a)
            v[a] = a < 3 ? fmin(v[a], part[6 * b + a]) : fmax(v[a], part[6 * b + a]);
    for (int o = 32; o > 0; o >>= 1)
        for (int a = 0; a < 6; ++a)
            v[a] = a < 3 ? fmin(v[a], __shfl_xor(v[a], o, 64))
                         : fmax(v[a], __shfl_xor(v[a], o, 64));
    if (threadIdx.x != 0) return;
    double L = 0.0;
    for (int a = 0; a < 3; ++a) {
        box[a] = v[a];
        if (v[3 + a] - v[a] > L) L = v[3 + a] - v[a];
    }
    if (!(L > 0.0)) L = 1.0;
    box[3] = L;
}

// Keys, arranged by particle id: slot id[i] holds (key_i, i). Every slot is
// first given its own particle, so that all values stay in [0, n) whatever
// id holds.
__global__ void __launch_bounds__(256)
gkeys_kernel(int64_t n, const double *__restrict__ x, const double *__restrict__ y,
             const double *__restrict__ z, const int32_t *__restrict__ id,
             const double *__restrict__ box, int by_id, uint32_t *__restrict__ keys,
             int32_t *__restrict__ vals)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double L = box[3];
    const double P[3] = {x[i], y[i], z[i]};
    uint32_t k[3];
    for (int a = 0; a < 3; ++a) {
        const double q = floor((P[a] - box[a]) / L * 1024.0);
        k[a] = q >= 1023.0 ? 1023u : (uint32_t)q;
    }
    const uint32_t key = spread10(k[0]) | (spread10(k[1]) << 1) | (spread10(k[2]) << 2);
    int64_t slot = i;
    if (by_id) {
        const int32_t d = id[i];
        if (d < 0 || d >= n) return;
        slot = d;
    }
    keys[slot] = key;
    vals[slot] = (int32_t)i;
}

__global__ void __launch_bounds__(256)
ggather_kernel(int64_t n, const int32_t *__restrict__ order, const double *__restrict__ x,
               const double *__restrict__ y, const double *__restrict__ z,
               const double *__restrict__ m, DensRec *__restrict__ out)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const int32_t i = order[k];
    out[k] = DensRec{x[i], y[i], z[i], m[i]};
}

// lvl[0..11]: first node of each level, lvl[12..23]: node count of each level
__global__ void __launch_bounds__(64)
gtree_init_kernel(int64_t n, GNode *__restrict__ nodes, int32_t *__restrict__ lvl,
                  uint32_t *__restrict__ flags)
{
    const int t = threadIdx.x;
    if (t < 25) lvl[t] = t == 12 ? 1 : 0;  // lvl[24]: group count
    if (t == 0) {
        GNode r{};
        r.start = 0;
        r.end = (int32_t)n;
        r.child0 = -1;
        r.nchild = 0;
        r.prefix = 0;
        r.level = 0;
        nodes[0] = r;
        flags[0] = 0;
    }
}

__device__ __forceinline__ int32_t lower_key(const uint32_t *__restrict__ keys, int32_t lo,
                                             int32_t hi, uint32_t k)
{
    while (lo < hi) {
        const int32_t mid = lo + (hi - lo) / 2;
        if (keys[mid] < k) lo = mid + 1; else hi = mid;
    }
    return lo;
}

// Split the nodes of level l: children get a contiguous block of the next
// level (one atomic per parent; ids vary from run to run, the tree does not).
__global__ void __launch_bounds__(256)
gtree_split_kernel(int l, const uint32_t *__restrict__ keys, GNode *__restrict__ nodes,
                   int32_t *__restrict__ lvl, int64_t node_cap, int leaf_size,
                   uint32_t *__restrict__ flags)
{
    if (flags[0] & 1u) return;  // an earlier level ran out of nodes
    const int32_t base = lvl[l], cnt = lvl[12 + l];
    const int32_t base_next = base + cnt;
    if (blockIdx.x == 0 && threadIdx.x == 0) lvl[l + 1] = base_next;
    const int64_t step = (int64_t)gridDim.x * blockDim.x;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < cnt; t += step) {
        GNode &N = nodes[base + t];
        N.child0 = -1;
        N.nchild = 0;
        if (l >= kGLevels || N.end - N.start <= leaf_size) continue;
        const int shift = 3 * (kGLevels - 1 - l);
        int32_t b[9];
        for (uint32_t o = 0; o <= 8; ++o)
            b[o] = lower_key(keys, N.start, N.end, ((N.prefix << 3) + o) << shift);
        int nch = 0;
        for (int o = 0; o < 8; ++o) nch += b[o + 1] > b[o];
        const int32_t at = atomicAdd(&lvl[12 + l + 1], nch);
        if ((int64_t)base_next + at + nch > node_cap) {
            atomicOr(flags, 1u);
            continue;
        }
        int j = 0;
        for (uint32_t o = 0; o < 8; ++o) {
            if (b[o + 1] == b[o]) continue;
            GNode c{};
            c.start = b[o];
            c.end = b[o + 1];
            c.child0 = -1;
            c.nchild = 0;
            c.prefix = (N.prefix << 3) | o;
            c.level = l + 1;
            nodes[base_next + at + j] = c;
            ++j;
        }
        N.child0 = base_next + at;
        N.nchild = nch;
    }
}

// Moments of the nodes of level l (children already done).
__global__ void __launch_bounds__(256)
gtree_moments_kernel(int l, const DensRec *__restrict__ pos, GNode *__restrict__ nodes,
                     const int32_t *__restrict__ lvl, const double *__restrict__ box,
                     double theta, const uint32_t *__restrict__ flags)
{
    if (flags[0] & 1u) return;
    const int32_t base = lvl[l], cnt = lvl[12 + l];
    const int64_t step = (int64_t)gridDim.x * blockDim.x;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < cnt; t += step) {
        GNode &N = nodes[base + t];
        double M = 0.0, sc[3] = {0.0, 0.0, 0.0}, Q[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
        double c[3];
        if (N.nchild == 0) {
            for (int32_t k = N.start; k < N.end; ++k) {
                const DensRec r = pos[k];
                M += r.m;
                sc[0] += r.m * r.x;
                sc[1] += r.m * r.y;
                sc[2] += r.m * r.z;
            }
            for (int a = 0; a < 3; ++a) c[a] = sc[a] / M;
            for (int32_t k = N.start; k < N.end; ++k) {
                const DensRec r = pos[k];
                const double d0 = r.x - c[0], d1 = r.y - c[1], d2v = r.z - c[2];
                const double d2 = d0 * d0 + d1 * d1 + d2v * d2v;
                Q[0] += r.m * (3.0 * d0 * d0 - d2);
                Q[1] += r.m * (3.0 * d0 * d1);
                Q[2] += r.m * (3.0 * d0 * d2v);
                Q[3] += r.m * (3.0 * d1 * d1 - d2);
                Q[4] += r.m * (3.0 * d1 * d2v);
                Q[5] += r.m * (3.0 * d2v * d2v - d2);
            }
        } else {
            for (int32_t k = N.child0; k < N.child0 + N.nchild; ++k) {
                const GNode &C = nodes[k];
                M += C.M;
                sc[0] += C.M * C.cx;
                sc[1] += C.M * C.cy;
                sc[2] += C.M * C.cz;
            }
            for (int a = 0; a < 3; ++a) c[a] = sc[a] / M;
            for (int32_t k = N.child0; k < N.child0 + N.nchild; ++k) {
                const GNode &C = nodes[k];
                const double e0 = C.cx - c[0], e1 = C.cy - c[1], e2v = C.cz - c[2];
                const double e2 = e0 * e0 + e1 * e1 + e2v * e2v;
                const double Mk = C.M;
                Q[0] += C.q[0] + Mk * (3.0 * e0 * e0 - e2);
                Q[1] += C.q[1] + Mk * (3.0 * e0 * e1);
                Q[2] += C.q[2] + Mk * (3.0 * e0 * e2v);
                Q[3] += C.q[3] + Mk * (3.0 * e1 * e1 - e2);
                Q[4] += C.q[4] + Mk * (3.0 * e1 * e2v);
                Q[5] += C.q[5] + Mk * (3.0 * e2v * e2v - e2);
            }
        }
        const double s = box[3] / (double)(1u << N.level);
        uint32_t kk[3] = {0u, 0u, 0u};
        for (int b = 0; b < N.level; ++b)
            for (int a = 0; a < 3; ++a) kk[a] |= ((N.prefix >> (3 * b + a)) & 1u) << b;
        double dd = 0.0;
        for (int a = 0; a < 3; ++a) {
            const double centre = box[a] + ((double)kk[a] + 0.5) * s;
            const double e = c[a] - centre;
            dd += e * e;
        }
        N.cx = c[0];
        N.cy = c[1];
        N.cz = c[2];
        N.ropen = s / theta + sqrt(dd);
        N.M = M;
        for (int q = 0; q < 6; ++q) N.q[q] = Q[q];
    }
}

__device__ __forceinline__ void wave_fence()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

// The groups of the definition; their order in the list does not matter.
__global__ void __launch_bounds__(256)
gtree_groups_kernel(int64_t n, const GNode *__restrict__ nodes, int32_t *__restrict__ lvl,
                    int2 *__restrict__ groups, const uint32_t *__restrict__ flags)
{
    if (flags[0] & 1u) return;
    constexpr int G = 64;
    const int32_t total = lvl[kGLevels + 1];  // first node past the last level
    const int64_t step = (int64_t)gridDim.x * blockDim.x;
    const int64_t t0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t0 == 0 && n <= G) groups[atomicAdd(&lvl[24], 1)] = make_int2(0, (int32_t)n);
    for (int64_t t = t0; t < total; t += step) {
        const GNode &N = nodes[t];
        if (N.end - N.start <= G) continue;
        if (N.nchild == 0) {
            const int32_t num = (N.end - N.start + G - 1) / G;
            const int32_t at = atomicAdd(&lvl[24], num);
            for (int32_t q = 0; q < num; ++q)
                groups[at + q] = make_int2(N.start + q * G, min(N.start + (q + 1) * G, N.end));
            continue;
        }
        int2 run[8];
        int nr = 0, cs = -1, ce = -1;
        for (int32_t k = N.child0; k < N.child0 + N.nchild; ++k) {
            const int32_t a = nodes[k].start, b = nodes[k].end;
            if (b - a > G) {
                if (cs >= 0) run[nr++] = make_int2(cs, ce);
                cs = -1;
                continue;
            }
            if (cs >= 0 && b - cs <= G) {
                ce = b;
                continue;
            }
            if (cs >= 0) run[nr++] = make_int2(cs, ce);
            cs = a;
            ce = b;
        }
        if (cs >= 0) run[nr++] = make_int2(cs, ce);
        const int32_t at = atomicAdd(&lvl[24], nr);
        for (int q = 0; q < nr; ++q) groups[at + q] = run[q];
    }
}

__device__ __forceinline__ void lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// One wave per group of 64 sorted particles (persistent waves). The nodes
// still to visit sit on a per-wave stack in global scratch: each round pops
// up to 64 of them, one per lane, tests them against the group's box,
// pushes the children of the opened internal nodes and evaluates the
// accepted nodes and the opened leaves in lane order. A round leaves at most
// 8 * 64 - 64 new entries per tree level on the stack, so 11 levels fit in
// fcap >= 5700. The nodes visited are those of the breadth-first walk of the
// definition (the test does not depend on the order), each term is the
// definition's, and only the order of the per-particle sums differs.
// Each lane loads its node whole; the accepted nodes' moments are handed to
// all lanes through LDS, and an opened leaf's particles are staged in LDS by
// one coalesced load, so no term waits on a memory round trip of its own.
__global__ void __launch_bounds__(256)
gravity_tree_kernel(const DensRec *__restrict__ pos, const int32_t *__restrict__ order,
                    const GNode *__restrict__ nodes, const int2 *__restrict__ groups,
                    const int32_t *__restrict__ lvl, int32_t *__restrict__ stack_all,
                    int64_t fcap, double e2, double *__restrict__ gx, double *__restrict__ gy,
                    double *__restrict__ gz, uint32_t *__restrict__ flags)
{
    __shared__ double nd_all[4][10][64];  // per wave: c, M, Q of each lane's node
    __shared__ DensRec lr_all[4][64];     // per wave: staged leaf particles
    __shared__ int32_t lk_all[4][3][64];  // per wave: their positions; leaf starts, ends
    if (flags[0] & 1u) return;  // the tree is incomplete
    const int lane = threadIdx.x & 63;
    const int w = threadIdx.x >> 6;
    double (*nd)[64] = nd_all[w];
    DensRec *lr = lr_all[w];
    int32_t *lpos = lk_all[w][0], *lstart = lk_all[w][1], *lend = lk_all[w][2];
    const int64_t wid = (int64_t)blockIdx.x * 4 + w;
    const int64_t nw = (int64_t)gridDim.x * 4;
    int32_t *stk = stack_all + wid * fcap;
    const int64_t ngroup = lvl[24];
    for (int64_t g = wid; g < ngroup; g += nw) {
        const int2 gr = groups[g];
        const int64_t k = gr.x + lane;
        const bool active = k < gr.y;
        const DensRec me = pos[active ? k : gr.x];
        double blo[3] = {me.x, me.y, me.z}, bhi[3] = {me.x, me.y, me.z};
        for (int o = 32; o > 0; o >>= 1)
            for (int a = 0; a < 3; ++a) {
                blo[a] = fmin(blo[a], __shfl_xor(blo[a], o, 64));
                bhi[a] = fmax(bhi[a], __shfl_xor(bhi[a], o, 64));
            }
        double ax = 0.0, ay = 0.0, az = 0.0;
        int64_t sp = 0;
        bool root = true;
        while (root || sp > 0) {
            const int64_t nb = root ? 1 : (sp < 64 ? sp : 64);
            const bool valid = lane < nb;
            const int32_t nid = (!valid || root) ? 0 : stk[sp - nb + lane];
            sp -= root ? 0 : nb;
            root = false;
            // the node's test fields and links first; its moments only if
            // accepted
            const GNode &N = nodes[nid];
            const double c[3] = {N.cx, N.cy, N.cz};
            const double ropen = N.ropen;
            const int32_t nstart = N.start, nend = N.end, child0 = N.child0, nch = N.nchild;
            double dd = 0.0;
            for (int a = 0; a < 3; ++a) {
                double e = 0.0;
                if (c[a] < blo[a]) e = blo[a] - c[a];
                else if (c[a] > bhi[a]) e = c[a] - bhi[a];
                dd += e * e;
            }
            const bool acc = valid && sqrt(dd) > ropen;
            const bool open_int = valid && !acc && nch > 0;
            // children of the opened internal nodes onto the stack
            const int cnt = open_int ? nch : 0;
            int incl = cnt;
            for (int o = 1; o < 64; o <<= 1) {
                const int v = __shfl_up(incl, o, 64);
                if (lane >= o) incl += v;
            }
            const int total = __shfl(incl, 63, 64);
            if (sp + total > fcap) {
                if (lane == 0) atomicOr(flags, 2u);
                break;
            }
            if (open_int) {
                const int64_t at = sp + incl - cnt;
                for (int q = 0; q < cnt; ++q) stk[at + q] = child0 + q;
            }
            sp += total;
            // moments of the accepted nodes into LDS
            lds_sync();
            if (acc) {
                nd[0][lane] = c[0];
                nd[1][lane] = c[1];
                nd[2][lane] = c[2];
                nd[3][lane] = N.M;
                for (int q = 0; q < 6; ++q) nd[4 + q][lane] = N.q[q];
            }
            lds_sync();
            // the opened leaves' particles, as one run: lane t's leaf covers
            // [lend[t] - its count, lend[t]) of the run
            const bool leaf = valid && !acc && nch == 0;
            const int lcnt = leaf ? nend - nstart : 0;
            int lincl = lcnt;
            for (int o = 1; o < 64; o <<= 1) {
                const int v = __shfl_up(lincl, o, 64);
                if (lane >= o) lincl += v;
            }
            const int ltotal = __shfl(lincl, 63, 64);
            lstart[lane] = nstart;
            lend[lane] = lincl;
            // accepted nodes in lane order
            uint64_t use = __ballot(acc);
            while (use) {
                const int tl = __builtin_ctzll(use);
                use &= use - 1;
                {
                    // -M d / r^3 + Q d / r^5 - 5/2 (d.Q d) d / r^7, as
                    // (Q d) / r^5 + (-M / r^3 - 5/2 (d.Q d) / r^7) d with fused
                    // multiply-adds
                    const double d0 = me.x - nd[0][tl], d1 = me.y - nd[1][tl],
                                 d2 = me.z - nd[2][tl];
                    const double M = nd[3][tl];
                    const double q0 = nd[4][tl], q1 = nd[5][tl], q2 = nd[6][tl],
                                 q3 = nd[7][tl], q4 = nd[8][tl], q5 = nd[9][tl];
                    const double r2 = __builtin_fma(d2, d2, __builtin_fma(d1, d1, d0 * d0));
                    const double rinv = rsq_newton(r2);  // r2 > 0: the node was accepted
                    const double rinv2 = rinv * rinv;
                    const double rinv3 = rinv * rinv2;
                    const double rinv5 = rinv3 * rinv2;
                    const double rinv7 = rinv5 * rinv2;
                    const double Qd0 = __builtin_fma(q2, d2, __builtin_fma(q1, d1, q0 * d0));
                    const double Qd1 = __builtin_fma(q4, d2, __builtin_fma(q3, d1, q1 * d0));
                    const double Qd2 = __builtin_fma(q5, d2, __builtin_fma(q4, d1, q2 * d0));
                    const double dQd = __builtin_fma(d2, Qd2, __builtin_fma(d1, Qd1, d0 * Qd0));
                    const double rad = __builtin_fma(-2.5 * dQd, rinv7, -M * rinv3);
                    ax = __builtin_fma(Qd0, rinv5, __builtin_fma(rad, d0, ax));
                    ay = __builtin_fma(Qd1, rinv5, __builtin_fma(rad, d1, ay));
                    az = __builtin_fma(Qd2, rinv5, __builtin_fma(rad, d2, az));
                }
            }
            // then the leaves' particles, staged 64 at a time by one load each
            for (int base = 0; base < ltotal; base += 64) {
                const int m = min(64, ltotal - base);
                lds_sync();
                if (lane < m) {
                    const int r = base + lane;
                    int lo = 0, hi = 63;  // first lane whose run ends past r
                    while (lo < hi) {
                        const int mid = (lo + hi) >> 1;
                        if (lend[mid] > r) hi = mid; else lo = mid + 1;
                    }
                    const int first = lo == 0 ? 0 : lend[lo - 1];
                    const int32_t q = lstart[lo] + (r - first);
                    lpos[lane] = q;
                    lr[lane] = pos[q];
                }
                lds_sync();
                for (int j = 0; j < m; ++j) {
                    const DensRec o = lr[j];
                    const double dx = me.x - o.x, dy = me.y - o.y, dz = me.z - o.z;
                    const double d2 =
                        __builtin_fma(dz, dz, __builtin_fma(dy, dy, __builtin_fma(dx, dx, e2)));
                    const double rs = rsq_newton(d2);
                    const double t = lpos[j] == k ? 0.0 : o.m * (rs * rs * rs);
                    ax = __builtin_fma(-t, dx, ax);
                    ay = __builtin_fma(-t, dy, ay);
                    az = __builtin_fma(-t, dz, az);
                }
            }
            // the pushed entries are read by other lanes next round
            wave_fence();
        }
        if (active) {
            const int32_t i = order[k];
            gx[i] = ax;
            gy[i] = ay;
            gz[i] = az;
        }
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


namespace {

template <typename T>
hipError_t gt_alloc(sph_ctx ctx, T **p, int64_t count)
{
    const size_t bytes = sizeof(T) * (size_t)std::max<int64_t>(count, 1);
    hipError_t e = hipMalloc((void **)p, bytes);
    if (e != hipSuccess) {
        *p = nullptr;
        return e;
    }
    ctx->scratch_bytes += (int64_t)bytes;
    return hipSuccess;
}

void gt_release(sph_ctx ctx)
{
    void *ptrs[] = {ctx->gt_keys[0], ctx->gt_keys[1], ctx->gt_vals[0], ctx->gt_vals[1],
                    ctx->gt_pos, ctx->gt_nodes, ctx->gt_lvl, ctx->gt_front, ctx->gt_flags,
                    ctx->gt_box, ctx->gt_part, ctx->gt_groups};
    for (void *q : ptrs)
        if (q) (void)hipFree(q);
    ctx->gt_keys[0] = ctx->gt_keys[1] = nullptr;
    ctx->gt_vals[0] = ctx->gt_vals[1] = nullptr;
    ctx->gt_pos = nullptr;
    ctx->gt_nodes = nullptr;
    ctx->gt_lvl = nullptr;
    ctx->gt_front = nullptr;
    ctx->gt_flags = nullptr;
    ctx->gt_box = nullptr;
    ctx->gt_part = nullptr;
    ctx->gt_groups = nullptr;
    ctx->gt_n_cap = 0;
}

hipError_t gt_reserve_all(sph_ctx ctx)
{
    const int64_t n = ctx->n_max;
    ctx->gt_node_cap = n / 2 + 1024;
    ctx->gt_fcap = 8192;
    ctx->gt_waves = 5120;
    hipError_t e;
    if ((e = gt_alloc(ctx, &ctx->gt_keys[0], n)) != hipSuccess) return e;
    if ((e = gt_alloc(ctx, &ctx->gt_keys[1], n)) != hipSuccess) return e;
    if ((e = gt_alloc(ctx, &ctx->gt_vals[0], n)) != hipSuccess) return e;
    if ((e = gt_alloc(ctx, &ctx->gt_vals[1], n)) != hipSuccess) return e;
    if ((e = gt_alloc(ctx, &ctx->gt_pos, n)) != hipSuccess) return e;
    if ((e = gt_alloc(ctx, &ctx->gt_nodes, ctx->gt_node_cap)) != hipSuccess) return e;
    if ((e = gt_alloc(ctx, &ctx->gt_lvl, 25)) != hipSuccess) return e;
    if ((e = gt_alloc(ctx, &ctx->gt_groups, n + 1)) != hipSuccess) return e;
    if ((e = gt_alloc(ctx, &ctx->gt_front, (int64_t)ctx->gt_waves * ctx->gt_fcap)) !=
        hipSuccess)
        return e;
    if ((e = gt_alloc(ctx, &ctx->gt_flags, 1)) != hipSuccess) return e;
    if ((e = gt_alloc(ctx, &ctx->gt_box, 4)) != hipSuccess) return e;
    if ((e = gt_alloc(ctx, &ctx->gt_part, 6 * kGBoxBlocks)) != hipSuccess) return e;
    ctx->gt_n_cap = n;
    return hipSuccess;
}

// The buffers of the octree gravity, allocated once per context (all or
// none).
hipError_t gt_reserve(sph_ctx ctx)
{
    if (ctx->gt_n_cap > 0) return hipSuccess;
    const hipError_t e = gt_reserve_all(ctx);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        gt_release(ctx);
    }
    return e;
}

}  // namespace

void release_gravity_tree(sph_ctx ctx) { gt_release(ctx); }

hipError_t launch_gravity_tree(sph_ctx ctx, const sph_particles &p, double eps, double theta,
                               int leaf_size, double *gx, double *gy, double *gz,
                               uint32_t *flags)
{
    hipError_t e;
    if ((e = gt_reserve(ctx)) != hipSuccess) return e;
    hipStream_t s = ctx->stream;
    const int64_t n = p.n;
    const unsigned nbox = std::min<unsigned>(kGBoxBlocks, blocks_for(n, 256));
    gbox_partial_kernel<<<nbox, 256, 0, s>>>(n, p.x, p.y, p.z, ctx->gt_part);
    gbox_final_kernel<<<1, 64, 0, s>>>((int)nbox, ctx->gt_part, ctx->gt_box);
    // (key, i) at slot i, then at slot id[i]: the sort starts from id order
    gkeys_kernel<<<blocks_for(n, 256), 256, 0, s>>>(n, p.x, p.y, p.z, p.id, ctx->gt_box, 0,
                                                   ctx->gt_keys[0], ctx->gt_vals[0]);
    gkeys_kernel<<<blocks_for(n, 256), 256, 0, s>>>(n, p.x, p.y, p.z, p.id, ctx->gt_box, 1,
                                                   ctx->gt_keys[0], ctx->gt_vals[0]);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    int cur = 0;
    if ((e = radix_sort_pairs(ctx, ctx->gt_keys, ctx->gt_vals, n, 3 * kGLevels, &cur)) !=
        hipSuccess)
        return e;
    const uint32_t *keys = ctx->gt_keys[cur];
    const int32_t *order = ctx->gt_vals[cur];
    ggather_kernel<<<blocks_for(n, 256), 256, 0, s>>>(n, order, p.x, p.y, p.z, p.m,
                                                     ctx->gt_pos);
    gtree_init_kernel<<<1, 64, 0, s>>>(n, ctx->gt_nodes, ctx->gt_lvl, ctx->gt_flags);
    // level l has at most min(8^l, node_cap) nodes
    auto level_blocks = [&](int l) {
        int64_t most = ctx->gt_node_cap;
        if (l < 8) most = std::min<int64_t>(most, (int64_t)1 << (3 * l));
        return std::max(1u, std::min(4096u, blocks_for(most, 256)));
    };
    for (int l = 0; l <= kGLevels; ++l)
        gtree_split_kernel<<<level_blocks(l), 256, 0, s>>>(l, keys, ctx->gt_nodes, ctx->gt_lvl,
                                                           ctx->gt_node_cap, leaf_size,
                                                           ctx->gt_flags);
    for (int l = kGLevels; l >= 0; --l)
        gtree_moments_kernel<<<level_blocks(l), 256, 0, s>>>(l, ctx->gt_pos, ctx->gt_nodes,
                                                             ctx->gt_lvl, ctx->gt_box, theta,
                                                             ctx->gt_flags);
    gtree_groups_kernel<<<std::min(4096u, blocks_for(ctx->gt_node_cap, 256)), 256, 0, s>>>(
        n, ctx->gt_nodes, ctx->gt_lvl, ctx->gt_groups, ctx->gt_flags);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    // groups hold at least one particle each, so at most n of them
    const unsigned gblocks =
        (unsigned)std::min<int64_t>(ctx->gt_waves / 4, (n + 3) / 4);
    gravity_tree_kernel<<<gblocks, 256, 0, s>>>(ctx->gt_pos, order, ctx->gt_nodes,
                                                ctx->gt_groups, ctx->gt_lvl, ctx->gt_front,
                                                ctx->gt_fcap, eps * eps, gx, gy, gz,
                                                ctx->gt_flags);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if ((e = hipMemcpyAsync(flags, ctx->gt_flags, sizeof(uint32_t), hipMemcpyDeviceToHost, s)) !=
        hipSuccess)
        return e;
    return hipStreamSynchronize(s);
}

}  // namespace sph
