/*
 * sph.h -- C ABI of libsph: one SPH hydro step on one MI355X (gfx950).
 *
 * The step is one pass of the generic SPH loop, Algorithm 1 of the paper
 * (Sec. 3): build the spatial structure (step 1), find the neighbours
 * (step 2), evaluate density, pressure, acceleration and the rate of change
 * of internal energy (step 3, as listed in the prose after Algorithm 1),
 * compute the new global time-step (step 5) and update velocity and position
 * (step 6). Self-gravity (step 4) is not computed here; a fixed external
 * acceleration may be supplied instead.
 *
 * The paper names these steps but not their formulas. The library uses:
 *   - M4 cubic-spline kernel (Table 1), W(r,h) = w(r/h)/(pi h^3), kernel
 *     derivatives for gradients and standard volume elements m/rho (Table 1);
 *   - neighbour relation j != i and r^2 < (2 max(h_i,h_j))^2 (strict), with
 *     r^2 = fma(dz,dz,fma(dy,dy,dx*dx)) in FP64 and the minimum image on
 *     periodic axes (d > L/2: d -= L; d < -L/2: d += L);
 *   - density by summation including the self term, gathered with h_i;
 *   - Tait EOS P = p_bg + B((rho/rho_ref)^7 - 1), c = c0 (rho/rho_ref)^3,
 *     B = rho0 c0^2/7, or ideal gas P = (gamma-1) rho u (Sec. 5.1, Evrard);
 *   - momentum a_i = -sum_j m_j (P_i/rho_i^2 + P_j/rho_j^2 + Pi_ij) gradW_ij
 *     with gradW_ij the mean of the gradients at h_i and h_j; energy
 *     du_i = 1/2 sum_j m_j (...) v_ij . gradW_ij; Monaghan viscosity
 *     mu = hbar v.r/(r^2 + eta2 hbar^2) if v.r < 0, Pi = (-alpha cbar mu +
 *     beta mu^2)/rhobar;
 *   - global dt = min_i min(c_cfl h_i/(c_i + 1.2(alpha c_i + beta mumax_i)),
 *     c_force sqrt(h_i/|a_i + g_i|));
 *   - kick-drift-kick leapfrog with that global dt.
 *
 * Conventions
 *   - Every call returns sph_status. No exceptions cross this boundary.
 *   - Every pointer inside the structs below is a DEVICE pointer owned by the
 *     caller (e.g. a torch tensor's storage), unless stated otherwise. Arrays
 *     are structure-of-arrays, FP64 (int32 for id, count and idx), one entry
 *     per particle.
 *   - The library owns only the opaque context and its scratch (sort buffers,
 *     cell table, packed neighbour records with the FP32-pair form's FP32
 *     copies, reduction partials, status word), allocated once by
 *     sph_ctx_create for n_max particles. Step calls never allocate (the
 *     octree gravity's buffers come with its first call).
 *   - Calls are asynchronous and ordered on the context's stream (borrowed,
 *     never destroyed by the library). Host-side argument errors return at
 *     once. Device-side conditions (neighbour overflow, h above the h_max the
 *     caller promised, non-finite state) set a status word on the device;
 *     sph_ctx_check synchronises the stream, returns and clears it.
 *   - sph_build_cells reorders every particle array in place, in lockstep,
 *     into cell (Morton) order; id[] carries the original ids. Neighbour
 *     indices always refer to the current order.
 */
#ifndef SPH_H
#define SPH_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t sph_status;
enum {
    SPH_OK = 0,
    SPH_E_INVALID = 1,   /* bad argument (null pointer, size, enum) */
    SPH_E_CAPACITY = 2,  /* a neighbour list exceeded max_nb (truncated) */
    SPH_E_HIP = 3,       /* a HIP runtime call failed */
    SPH_E_DOMAIN = 4,    /* h_i > h_max, or a periodic axis shorter than 4 h_max */
    SPH_E_NOMEM = 5,     /* device allocation failed */
    SPH_E_AGAIN = 6,     /* result not ready yet (serving) */
    SPH_E_NONFINITE = 7  /* NaN or Inf in the state */
};

enum { SPH_FP64 = 0, SPH_FP32_PAIR = 1 };        /* sph_params.precision */
enum { SPH_EOS_TAIT = 0, SPH_EOS_IDEAL = 1 };    /* sph_params.eos */
enum { SPH_KICK_DRIFT = 0, SPH_KICK = 1 };       /* sph_integrate stage */

typedef struct sph_ctx_s *sph_ctx;
typedef void *sph_stream; /* a hipStream_t; NULL = the null stream */

/* Particle state. gx, gy, gz: optional fixed external acceleration (NULL
 * when absent); they are permuted with the rest. rho_ref and p_bg are the
 * per-particle Tait reference density and background pressure (read only by
 * the Tait EOS; may be NULL for the ideal gas). xw: the weights X of
 * generalised volume elements (see SPH_VOLUME_GENERALISED), required only
 * when sph_params.volume selects them, else may be NULL; permuted with the
 * rest when present. */
typedef struct {
    int64_t n;
    double *x, *y, *z, *vx, *vy, *vz, *u, *h, *m, *rho_ref, *p_bg;
    double *gx, *gy, *gz;
    int32_t *id;
    double *xw;
} sph_particles;

/* Axis-aligned box. On a periodic axis positions live in [lo, hi) and the
 * minimum image applies; on an open axis the box only sizes the cell grid
 * (particles outside it are clamped into the border cells, which keeps the
 * search exact). Host memory. */
typedef struct {
    double lo[3], hi[3];
    int32_t periodic[3];
} sph_box;

/* Neighbour lists, ELL layout, column-major: the k-th neighbour of particle
 * i is idx[k * n + i], k < min(count[i], max_nb). count[i] is the true count,
 * which may exceed max_nb only after SPH_E_CAPACITY was raised. */
typedef struct {
    int32_t max_nb;
    int32_t *count;  /* [n] */
    int32_t *idx;    /* [max_nb * n] */
} sph_nbrs;

/* Per-particle fields from sph_density / sph_eos. pr2 = P / rho^2. */
typedef struct {
    double *rho, *p, *c, *pr2;
} sph_fields;

/* Outputs of sph_momentum_energy: hydrodynamic acceleration (external g not
 * included), du/dt, and the largest |mu| over each particle's pairs. */
typedef struct {
    double *ax, *ay, *az, *dudt, *mumax;
} sph_accel;

/* Interpolation kernels: the interchangeable set of the mini-app (Sec. 4,
 * Table 2; Table 1 lists which parent code uses which). All have support 2h,
 * so the neighbour relation does not depend on the choice; q = r/h:
 *   SPH_KERNEL_M4           W = w(q) / (pi h^3), the M4 cubic spline
 *   SPH_KERNEL_WENDLAND_C2  W = 21 / (16 pi h^3) (1 - q/2)^4 (1 + 2q)
 *   SPH_KERNEL_SINC         W = B_n / h^3 (sin(x)/x)^n, x = pi q / 2, with
 *                           B_n normalising W to unit integral, 3 <= n <= 12 */
enum { SPH_KERNEL_M4 = 0, SPH_KERNEL_WENDLAND_C2 = 1, SPH_KERNEL_SINC = 2 };

/* Gradient estimates of sph_momentum_energy (Table 1: kernel derivatives for
 * ChaNGa and SPH-flow, IAD for SPHYNX; the mini-app keeps both, Table 2):
 *   SPH_GRAD_KERNEL  grad W, the mean of grad W(r, h_i) and grad W(r, h_j)
 *   SPH_GRAD_IAD     the integral approach to derivatives with standard
 *                    volume elements V_j = m_j / rho_j:
 *                    tau_i = sum_j V_j (x_j - x_i)(x_j - x_i)^T W(r_ij, h_i),
 *                    c_i = tau_i^{-1} where det tau_i >= 0.01 (tr tau_i/3)^3;
 *                    below that (neighbours not spanning three dimensions)
 *                    c_i = (tr tau_i / 3)^{-1} I, and c_i = 0 when
 *                    tr tau_i = 0 (no neighbour inside 2 h_i),
 *                    A_ij = c_i (x_j - x_i) W(r_ij, h_i), and the pair terms
 *                    use (A_ij - A_ji) / 2 in place of the kernel gradient. */
enum { SPH_GRAD_KERNEL = 0, SPH_GRAD_IAD = 1 };

/* Volume elements (Table 1: SPHYNX uses generalised ones, the other codes
 * the standard m/rho):
 *   SPH_VOLUME_STANDARD     V_i = m_i / rho_i
 *   SPH_VOLUME_GENERALISED  V_i = X_i / k_i with k_i = sum_j X_j W(r_ij, h_i)
 *                           (self term included) and weights X = p->xw,
 *                           normally X_i = (m_i / rho_i)^volume_p from the
 *                           previous density (sph_volume_weights). Then
 *                           rho_i = k_i (m_i / X_i), and the pair weight
 *                           m_j (P_i/rho_i^2 + P_j/rho_j^2 + Pi_ij) of the
 *                           momentum and energy equations becomes
 *                           (X_j Q_i + X_i Q_j) / m_i + m_j Pi_ij with
 *                           Q_i = m_i^2 P_i / (rho_i^2 X_i), the general form
 *                           of Hopkins (2013). X = m is the standard case. IAD
 *                           keeps V_j = m_j / rho_j (equal to X_j / k_j). */
enum { SPH_VOLUME_STANDARD = 0, SPH_VOLUME_GENERALISED = 1 };

/* Scalar physics constants (host memory). precision selects the pair
 * arithmetic of sph_density and sph_momentum_energy: SPH_FP64, or
 * SPH_FP32_PAIR (separations and velocity differences formed in FP64 and
 * rounded to FP32; sph_momentum_energy packs FP32 copies of h, 1/h, m, rho,
 * c and P/rho^2 next to the FP64 position and velocity into its neighbour
 * records (80 B of a 128-byte line; with IAD the records stay FP64 and the
 * IAD gradient is formed in FP64); FP32 pair arithmetic and accumulation,
 * results widened to FP64;
 * the neighbour relation, the state, the integration and all reductions stay
 * FP64). kernel selects W and its gradient in both pair calls (zero, the
 * default of a zeroed struct, is M4); sinc_n is the sinc exponent, read only
 * for SPH_KERNEL_SINC; gradient selects SPH_GRAD_KERNEL (zero) or
 * SPH_GRAD_IAD for sph_momentum_energy (IAD matrices are formed inside that
 * call, in FP64 for both precisions); volume selects the volume elements of
 * both pair calls and volume_p the exponent used by sph_step and
 * sph_init_forces to form the weights. */
typedef struct {
    int32_t precision;
    int32_t eos;
    double rho0, c0, gamma_tait, gamma_gas;
    double alpha, beta, eta2;
    double c_cfl, c_force;
    int32_t kernel;
    int32_t sinc_n;
    int32_t gradient;
    int32_t volume;
    double volume_p;
} sph_params;

/* Text for a status code (static storage). */
const char *sph_status_string(sph_status s);

/* Detail of the last error seen on ctx (valid until the next call). */
const char *sph_last_error(sph_ctx ctx);

/* Library and device description, e.g. "libsph 1 gfx950 256 CUs" (static). */
const char *sph_version(void);

/* Create a context for up to n_max particles (n_max >= 1) and neighbour
 * lists of width max_nb (1..4096) on the current HIP device; all scratch is
 * allocated here. Returns SPH_E_NOMEM if the device memory is not there. */
sph_status sph_ctx_create(sph_ctx *out, int64_t n_max, int32_t max_nb,
                          sph_stream stream);

/* Release the context and its scratch (synchronises its stream first). */
sph_status sph_ctx_destroy(sph_ctx ctx);

/* Synchronise the stream and return (and clear) the device status word:
 * SPH_OK or the first error raised since the last check. */
sph_status sph_ctx_check(sph_ctx ctx);

/* Bytes of device scratch held by ctx (host value). */
int64_t sph_ctx_scratch_bytes(sph_ctx ctx);

/* Live kernel timing, for measurement. With enable != 0 (which also clears
 * the sums) every later launch, by this context, of the kernels
 * find_neighbors_kernel, fallback_kernel, density_kernel, iad_kernel and
 * momentum_kernel is bracketed by two HIP events on the context's stream (not
 * inside sph_step_capture); enable = 0 stops. sph_ctx_kernel_time waits for
 * the recorded launches and returns the named kernel's mean duration in ms
 * and its launch count since timing was enabled (SPH_E_INVALID for another
 * name). The events are created on the host (hipEventCreate), never
 * device memory. */
sph_status sph_ctx_timing(sph_ctx ctx, int32_t enable);
sph_status sph_ctx_kernel_time(sph_ctx ctx, const char *kernel, double *avg_ms,
                               int64_t *launches);

/* Algorithm 1, step 1. Assign every particle to a cell of side
 * >= 2 h_max (1 + 1e-9), sort the particles by the cell's Morton key and,
 * inside a cell, by the particle's z slice (up to 64 slices per cell; stable
 * LSD radix sort, so equal keys keep their previous order), reorder all
 * particle arrays of p in place and build the cell table. h_max is the
 * caller's bound on h (no device-to-host copy); a particle with h > h_max
 * raises SPH_E_DOMAIN. A periodic axis must be longer than 4 h_max. */
sph_status sph_build_cells(sph_ctx ctx, const sph_particles *p,
                           const sph_box *box, double h_max);

/* Algorithm 1, step 2. Neighbour sets by the relation stated at the top of
 * this file, searched over the 27 cells around each particle's cell. Needs a
 * preceding sph_build_cells on the same particles. Raises SPH_E_CAPACITY on
 * overflow (lists truncated at max_nb, count still exact). */
sph_status sph_find_neighbors(sph_ctx ctx, const sph_particles *p,
                              const sph_box *box, const sph_nbrs *nb);

/* Algorithm 1, step 3: summation density
 * rho_i = m_i W(0,h_i) + sum_{j in N_i} m_j W(r_ij, h_i); with generalised
 * volume elements rho_i = k_i (m_i / X_i), k_i = X_i W(0,h_i) +
 * sum_{j in N_i} X_j W(r_ij, h_i), X = p->xw (SPH_E_INVALID if NULL). */
sph_status sph_density(sph_ctx ctx, const sph_particles *p,
                       const sph_box *box, const sph_nbrs *nb,
                       const sph_params *prm, double *rho);

/* sph_density for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same computation and kernels as sph_density, with no context. It calls
 * no hipMalloc, hipFree or other allocating routine; its scratch (the packed
 * neighbour records, 32 B per particle) is a static device array of
 * SPH_DENSITY_NOALLOC_MAX_N records that every GPU the library runs on holds
 * until the process ends (32 MiB).
 *   p, nb: device arrays in the order the lists refer to (as left by
 *          sph_build_cells and sph_find_neighbors); p->x, y, z, h, m are
 *          read (and p->xw with generalised volume elements);
 *   box:   the box of that build (its periodic axes and lengths are used);
 *   rho:   device output, n doubles, bitwise the values sph_density writes
 *          for the same inputs;
 *   stream: a hipStream_t (NULL = the null stream) for the launches; the
 *          current device must be the stream's.
 * Asynchronous like the other calls. Errors (host-side only, nothing is
 * launched): SPH_E_CAPACITY if p->n > SPH_DENSITY_NOALLOC_MAX_N,
 * SPH_E_INVALID for NULL or malformed arguments, SPH_E_HIP for a launch or
 * symbol failure; sph_last_error(NULL) gives the detail on the calling
 * thread. Every call on one device shares that device's array, which keeps
 * the last call's records: calls that overlap on one device (two streams,
 * two threads) race and must be ordered by the caller. */
#define SPH_DENSITY_NOALLOC_MAX_N 1048576
sph_status sph_density_noalloc(const sph_particles *p, const sph_box *box,
                               const sph_nbrs *nb, const sph_params *prm,
                               double *rho, sph_stream stream);

/* Algorithm 1, step 3: EOS. Reads f->rho and p->u (ideal) or p->rho_ref,
 * p->p_bg (Tait); writes f->p, f->c, f->pr2 (FP64; the FP32-pair form's
 * FP32 copies are made by sph_momentum_energy when it packs its records). */
sph_status sph_eos(sph_ctx ctx, const sph_particles *p, const sph_params *prm,
                   const sph_fields *f);

/* Algorithm 1, step 3: acceleration, du/dt and per-particle max |mu|.
 * Like sph_find_neighbors, it takes h as of the last sph_build_cells (h must
 * not change between the build and the pair calls of a step). With
 * generalised volume elements it reads the weights p->xw (the same the
 * density used; SPH_E_INVALID if NULL). */
sph_status sph_momentum_energy(sph_ctx ctx, const sph_particles *p,
                               const sph_box *box, const sph_nbrs *nb,
                               const sph_params *prm, const sph_fields *f,
                               const sph_accel *a);

/* Algorithm 1, step 4 (self-gravity; Sec. 5.2.5 phase I) by a Morton
 * octree with multipoles to quadrupole order, the parent codes' method
 * (SPHYNX uses quadrupoles), G = 1, in FP64:
 *   - cube lo_a = min x_a, L = largest extent; keys are 30-bit Morton codes of
 *     floor((x - lo) / L * 1024) (clamped to 1023); particles are sorted by
 *     (key, id);
 *   - a node of level l < 10 with more than leaf_size particles is split
 *     into its non-empty octants; every node carries its mass M, centre of
 *     mass c and traceless quadrupole Q = sum m (3 d d^T - |d|^2 I);
 *   - the sorted particles form groups of 64; a node N is accepted for a
 *     whole group when the distance from c_N to the group's bounding box
 *     exceeds s_N / theta + |c_N - centre_N| (s_N the node's side), and then
 *     contributes -M d/r^3 + Q d/r^5 - 5/2 (d.Q d) d/r^7 (d = x_i - c_N,
 *     unsoftened); otherwise a leaf contributes its particles directly with
 *     Plummer softening eps, -m_j d/(|d|^2 + eps^2)^{3/2}, and an internal
 *     node is opened. theta -> 0 gives the direct sum of sph_gravity_direct.
 * Reads p->x, y, z, m, id (device, n, current order; id must be a
 * permutation of 0..n-1) and writes gx, gy, gz (device, n doubles each,
 * caller-owned, same order). The first call on a context allocates the
 * tree's buffers (about 100 bytes per particle of n_max plus 160 MiB of
 * traversal stacks), kept until sph_ctx_destroy; SPH_E_NOMEM if that fails.
 * Synchronises ctx's stream. SPH_E_INVALID for NULL arrays, eps < 0,
 * theta <= 0 or a non-finite value, leaf_size outside [8, 64];
 * SPH_E_CAPACITY if the tree needs more than n_max / 2 + 1024 nodes
 * (outputs undefined). */
sph_status sph_gravity_tree(sph_ctx ctx, const sph_particles *p, double eps, double theta,
                            int32_t leaf_size, double *gx, double *gy, double *gz);

/* Weights of generalised volume elements (Table 1, SPHYNX) from a density
 * estimate: p->xw[i] = (p->m[i] / rho[i])^exponent, FP64, in the current
 * particle order (rho: device, n doubles, e.g. the previous step's density).
 * SPH_E_INVALID for NULL arrays or a non-finite exponent. */
sph_status sph_volume_weights(sph_ctx ctx, const sph_particles *p, const double *rho,
                              double exponent);

/* Algorithm 1, step 4 (self-gravity; Sec. 5.2.5 phase I) by direct
 * summation in FP64, G = 1, Plummer softening eps >= 0:
 *   g_i = - sum_{j != i} m_j (x_i - x_j) / (|x_i - x_j|^2 + eps^2)^{3/2},
 * no periodic images. Reads p->x, y, z, m (device, n, current order; h and
 * id are checked but not read) and writes gx, gy, gz (device, n doubles
 * each, caller-owned, same order); uses the context's density records as
 * scratch. O(n^2) work: the reference the parent codes' tree multipoles
 * approximate, not a fast solver. Asynchronous on ctx's stream;
 * SPH_E_INVALID for NULL arrays or a negative or non-finite eps. */
sph_status sph_gravity_direct(sph_ctx ctx, const sph_particles *p, double eps,
                              double *gx, double *gy, double *gz);

/* Algorithm 1, step 6, one half of a kick-drift-kick step with the global
 * dt read from device memory dt_dev[0]:
 *   SPH_KICK_DRIFT: v += dt/2 (a + g); u += dt/2 du; x += dt v; wrap
 *                   periodic coordinates into [lo, hi);
 *   SPH_KICK:       v += dt/2 (a + g); u += dt/2 du; raises SPH_E_NONFINITE
 *                   if the new state holds a NaN or Inf. */
sph_status sph_integrate(sph_ctx ctx, const sph_particles *p,
                         const sph_box *box, int32_t stage,
                         const double *dt_dev, const sph_accel *a);

/* Algorithm 1, step 5: dt_dev[0] = global minimum of the Courant and force
 * limits (two-level min reduction, exact). If diag_dev is not NULL it
 * receives 8 FP64 totals: M, Px, Py, Pz, Lx, Ly, Lz, E with P = sum m v,
 * L = sum m x cross v, E = sum m (v^2/2 + u), summed in a fixed tree order
 * (deterministic). */
sph_status sph_timestep(sph_ctx ctx, const sph_particles *p,
                        const sph_params *prm, const sph_fields *f,
                        const sph_accel *a, double *dt_dev, double *diag_dev);

/* Forces at the current state: build cells, neighbours, density, EOS (if
 * set_rho_ref, rho_ref := rho first, so that P = p_bg), momentum and energy,
 * then dt. The t = 0 evaluation that precedes the first step. With
 * generalised volume elements the density is first taken with standard
 * elements and the weights p->xw formed from it (sph_volume_weights with
 * prm->volume_p). */
sph_status sph_init_forces(sph_ctx ctx, const sph_particles *p,
                           const sph_box *box, double h_max,
                           const sph_nbrs *nb, const sph_params *prm,
                           const sph_fields *f, const sph_accel *a,
                           int32_t set_rho_ref, double *dt_dev,
                           double *diag_dev);

/* One whole hydro step: sph_integrate(KICK_DRIFT), sph_build_cells,
 * sph_find_neighbors, sph_density, sph_eos, sph_momentum_energy,
 * sph_integrate(KICK), sph_timestep, in that order on ctx's stream. With
 * generalised volume elements the step first forms the weights p->xw from
 * the previous density f->rho (sph_volume_weights with prm->volume_p). */
sph_status sph_step(sph_ctx ctx, const sph_particles *p, const sph_box *box,
                    double h_max, const sph_nbrs *nb, const sph_params *prm,
                    const sph_fields *f, const sph_accel *a, double *dt_dev,
                    double *diag_dev);

/* sph_step captured into a HIP graph kept by the context (replacing any
 * earlier capture): the same kernels with the same arguments, recorded
 * without running. sph_step_replay launches the graph on ctx's stream, one
 * step per call, without the host work of the individual calls. The
 * captured pointers, n, box, h_max and parameters are fixed: the caller keeps
 * the arrays allocated and unmoved and captures again after changing any of
 * them. Errors of the captured calls are returned by sph_step_capture (no
 * graph is kept); SPH_E_INVALID from sph_step_replay without a capture. */
sph_status sph_step_capture(sph_ctx ctx, const sph_particles *p, const sph_box *box,
                            double h_max, const sph_nbrs *nb, const sph_params *prm,
                            const sph_fields *f, const sph_accel *a, double *dt_dev,
                            double *diag_dev);
sph_status sph_step_replay(sph_ctx ctx);

/* One step with individual time steps in power-of-two bins (Table 1 and
 * Table 2: ChaNGa's multiple time-stepping; the paper's other scaling lever
 * besides the global dt). Needs the forces at the current, synchronised
 * state (sph_init_forces or a previous step: f->c, a->ax..a->mumax).
 *   - each particle's criterion is the global one's (sph_timestep); with
 *     its minimum and maximum, the step D = min(max, min 2^max_bin) goes to
 *     dt_dev[0], and particle i gets the smallest bin b in [0, max_bin] with
 *     D / 2^b <= its criterion (written to bin[i] as a double);
 *   - with B the deepest bin, 2^B substeps of D / 2^B follow. In substep s
 *     the particles of bin b with s mod 2^(B-b) == 0 take their opening half
 *     kick of D / 2^(b+1), every particle drifts and the cells are rebuilt;
 *     the particles whose step closes, (s + 1) mod 2^(B-b) == 0, get new
 *     neighbour lists, density, EOS values, a, du/dt and max |mu| (with the
 *     current, half-kicked velocities and energies, as in sph_step) and
 *     their closing half kick; the others keep the density, pressure and
 *     sound speed of their last evaluation (no prediction), and tiles
 *     without a closing particle are skipped by every pair kernel;
 *   - bin, ax, ay, az, dudt, mumax and f->rho, p, c, pr2 are reordered with
 *     the particles by every cell sort; with generalised volume elements the
 *     weights are formed from the current density at every substep.
 * max_bin = 0 is sph_step. *substeps (host) receives 2^B; diag_dev (if not
 * NULL) the totals of the end state. Synchronises once (to read B).
 * SPH_E_INVALID for max_bin outside [0, 16], NULL arrays or IAD gradients
 * (their matrices would need every neighbour's list). */
sph_status sph_step_blocks(sph_ctx ctx, const sph_particles *p, const sph_box *box,
                           double h_max, const sph_nbrs *nb, const sph_params *prm,
                           const sph_fields *f, const sph_accel *a, int32_t max_bin,
                           double *bin, double *dt_dev, double *diag_dev, int32_t *substeps);

/* Algorithm 1, step 2 ("find the neighbours and the smoothing length"); the
 * target neighbour count of Sec. 3. Iterates, for it = 0, 1, ..., max_iter:
 * build the cells for the current largest h (this reorders p as
 * sph_build_cells does), count for every particle the gather neighbours
 * N_i = #{j != i : r^2 < (2 h_i)^2} (exact FP64 test, minimum image on
 * periodic axes) into count[] (DEVICE, n int32, current order); stop when
 * every N_i is in [lo_count, hi_count] or it == max_iter; otherwise, for the
 * particles outside the band, h_i <- 2 h_i if N_i = 0, else
 * h_i <- (h_i / 2) (1 + (n_target / N_i)^(1/3)), the cube root by Newton's
 * iteration in correctly rounded IEEE operations (seven steps from 3/2 after
 * scaling into [1, 8) by powers of 8), evaluated on the device, so that any
 * implementation of the same rule gets the same h. The sweeps run on the
 * device on the cells built for the starting largest h (a particle may grow
 * to 2 h_i = two cells); the host steps in only to rebuild when a particle
 * outgrows that, and once at the end. *iterations (HOST) receives the last
 * it. On return the cells are built for the final h (sph_find_neighbors may
 * follow directly) and count[] is in that order. Synchronising (three times when
 * no particle outgrows the cells); allocates nothing.
 * SPH_E_DOMAIN if a periodic axis is shorter than 4 h_max at the start or
 * the end, SPH_E_NONFINITE if h stops being finite and positive. */
sph_status sph_smoothing_length(sph_ctx ctx, sph_particles *p, const sph_box *box,
                                double n_target, int32_t lo_count, int32_t hi_count,
                                int32_t max_iter, int32_t *count, int32_t *iterations);

/* Test helper (synchronising): neighbour sets in ORIGINAL-id terms.
 * offsets_host[n+1] (int64) and ids_host[cap] (int32) are HOST buffers;
 * the set of original id k is ids_host[offsets_host[k] .. offsets_host[k+1]),
 * sorted ascending. Requires the ids to be a permutation of 0..n-1.
 * *total receives the number of entries (SPH_E_CAPACITY if > cap). */
sph_status sph_export_neighbors(sph_ctx ctx, const sph_particles *p,
                                const sph_nbrs *nb, int64_t *offsets_host,
                                int32_t *ids_host, int64_t cap,
                                int64_t *total);

/* ------------------------------------------------------------------------
 * Ensemble serving: many independent runs of the step above (for instance
 * rotating patches of uneven sizes), advanced together.
 *
 * Not part of the paper, which runs one simulation at a time: this is a
 * serving layer over the same step. Every resident run's state stays in
 * device memory; all resident runs advance together through one captured
 * HIP graph of fused launches per step (each launch covers every resident
 * particle). A persistent host thread admits queued runs in arrival order as
 * soon as a run slot is free and the run's particles and cells fit in the
 * memory budget, and retires runs after their last step. Each run takes its
 * own global dt (Sec. 3, Algorithm 1, step 5, per run) and its own
 * conserved totals, and its results are bitwise those of the same run
 * advanced alone (and of the single-run calls above at the same precision).
 *
 * A run: the t = 0 evaluation (cells, neighbours, density, optionally
 * rho_ref := rho, EOS, momentum and energy, dt), then n_steps kick-drift-kick
 * steps, exactly as sph_init_forces followed by n_steps calls of sph_step.
 * No external acceleration. Cells: side >= 2 h_max, at most 32 per axis.
 *
 * Threads: submit, poll, wait and stats may be called from any thread.
 * Times are seconds on the steady clock that sph_ens_clock reads.
 * ------------------------------------------------------------------------ */
typedef struct sph_ens_s *sph_ens;

typedef struct {
    int32_t device;            /* HIP device ordinal */
    int32_t precision;         /* SPH_FP64 or SPH_FP32_PAIR, for every run */
    int32_t max_nb;            /* neighbour-list capacity per particle, >= 1 */
    int32_t max_slots;         /* runs resident at once, 1..511 */
    int64_t hbm_budget_bytes;  /* device memory for the arena and its scratch */
    int64_t max_n_per_run;     /* largest run accepted, >= 1 */
    int64_t pinned_submit_bytes; /* pinned host memory up to which sph_ens_submit
                                    copies a run straight into a pinned block
                                    (0: 4 GiB; < 0: never, the engine stages
                                    every run itself) */
} sph_ens_config;

typedef struct {
    int64_t n;                 /* particles, >= 1, <= max_n_per_run */
    int32_t n_steps;           /* KDK steps after the t = 0 evaluation, >= 0 */
    int32_t set_rho_ref;       /* Tait: rho_ref := rho at t = 0 */
    sph_params params;         /* params.precision is ignored (engine's);
                                  params.kernel must be SPH_KERNEL_M4 and
                                  params.gradient SPH_GRAD_KERNEL */
    sph_box box;
    double h_max;              /* >= every h (h stays fixed); sets the cells */
    /* HOST arrays of n entries in any order, copied by sph_ens_submit
     * (the caller may free them when it returns) */
    const double *x, *y, *z, *vx, *vy, *vz, *u, *h, *m, *p_bg;
    const double *rho_ref;     /* Tait without set_rho_ref; else may be NULL */
    const int32_t *id;         /* a permutation of 0..n-1 */
} sph_run_request;

typedef struct {
    /* HOST buffers of n entries owned by the caller, each may be NULL;
     * filled in id order (entry k belongs to the particle with id k) */
    double *x, *y, *z, *vx, *vy, *vz, *u, *rho;
    /* filled by the library */
    double diag[8];            /* M, Px, Py, Pz, Lx, Ly, Lz, E after the run */
    double dt;                 /* dt from the run's last force evaluation */
    double t_submit, t_admit, t_done;
    int32_t steps_done;
    sph_status status;         /* the run's own outcome (SPH_OK, SPH_E_CAPACITY,
                                  SPH_E_DOMAIN, SPH_E_NONFINITE, SPH_E_HIP) */
} sph_run_result;

typedef struct {
    int64_t submitted, completed, queued, running;
    int64_t steps;               /* batched steps launched */
    int64_t particle_steps;      /* sum over launched steps of resident live particles */
    int64_t capacity_particles;  /* particles the budget holds */
    int64_t capacity_cells;
    int64_t bytes_per_particle;  /* device bytes per resident particle */
    int64_t bytes_allocated;     /* device bytes held by the engine */
    int64_t peak_particles;      /* most live particles in one step */
    int32_t peak_runs;           /* most live runs in one step */
    int32_t max_slots;
    double busy_seconds;         /* time from the first admission to the last completion */
} sph_ens_counters;

/* Allocate the arena (SPH_E_NOMEM if the budget cannot be allocated,
 * SPH_E_INVALID if it holds no run of max_n_per_run particles), capture the
 * step graph and start the engine thread. */
sph_status sph_ens_create(sph_ens *out, const sph_ens_config *cfg);

/* Queue a run (non-blocking; copies the arrays). *ticket identifies it.
 * The copy goes into a block of the engine's pinned host memory while the
 * engine's pinned pool holds under cfg.pinned_submit_bytes (the block is
 * reused for the results and returned to the pool when they are taken),
 * else into host memory that the engine stages into a pinned block before
 * the run's upload (ahead of its admission while it waits for a step).
 * SPH_E_INVALID for bad arguments, SPH_E_DOMAIN if some h > h_max or a
 * periodic axis is not longer than 4 h_max, SPH_E_CAPACITY if the run could
 * never fit (particles or cells above what the budget holds). */
sph_status sph_ens_submit(sph_ens e, const sph_run_request *req, uint64_t *ticket);

/* Non-blocking: SPH_E_AGAIN while the run is queued or running. When it is
 * finished, fills *res, forgets the ticket and returns SPH_OK (the run's own
 * outcome is res->status). SPH_E_INVALID for an unknown ticket. */
sph_status sph_ens_poll(sph_ens e, uint64_t ticket, sph_run_result *res);

/* As sph_ens_poll, but blocks until the run is finished. */
sph_status sph_ens_wait(sph_ens e, uint64_t ticket, sph_run_result *res);

sph_status sph_ens_stats(sph_ens e, sph_ens_counters *out);

/* Finish every queued and running run, stop the thread, free everything.
 * Results not yet polled are discarded. */
sph_status sph_ens_destroy(sph_ens e);

const char *sph_ens_last_error(sph_ens e);

/* The clock of t_submit, t_admit and t_done (seconds, steady). */
double sph_ens_clock(void);

#ifdef __cplusplus
}
#endif

#endif /* SPH_H */
