// Ensemble serving: many independent SPH runs advanced together on one GPU.
//
// Every resident run lives in one arena of particle arrays. A batched step
// is one captured HIP graph of fused launches over all resident particles:
// the runs are told apart by a per-particle slot id, which also sits in the
// high bits of the Morton sort key, so one radix sort regroups every run by
// cell and packs the live runs to the front of the arena in slot order. The
// launch grids are sized for the arena's capacity and every count is read on
// the device from a per-step header, so the same graph is replayed for every
// batch composition; between replays the host only uploads that header and
// the per-slot run table.
//
// A persistent host thread runs the loop: it admits queued runs in arrival
// order whenever a slot is free and their particles and cells fit in what
// the memory budget left (appending their initial state at the end of the
// arena), retires runs whose last step has been launched (their final state
// is copied back right after that step; the next step's sort drops their
// particles), and keeps at most two steps in flight so that the host's
// bookkeeping overlaps the GPU's work.
//
// A run's arithmetic does not depend on its neighbours in the batch: its
// particles keep their relative order, its neighbour lists, pair sums and
// reductions are formed over its own particles in the same order and with
// the same reduction tree as when it runs alone (and as the single-run calls
// of this library compute them), so its results are bitwise the same.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "sph_internal.h"

using namespace sph;

namespace {

double clock_s()
{
    using namespace std::chrono;
    return duration<double>(steady_clock::now().time_since_epoch()).count();
}

thread_local std::string g_ens_error;

// Pinned host blocks, recycled by size class (powers of two) and released
// only when the engine is destroyed.
struct PinnedPool {
    std::mutex mu;
    std::multimap<size_t, void *> free_;
    std::vector<void *> all;
    std::atomic<size_t> held{0};  // bytes allocated

    static size_t round_up(size_t b)
    {
        size_t c = 1 << 16;
        while (c < b) c <<= 1;
        return c;
    }
    void *get(size_t bytes, size_t *cls)
    {
        *cls = round_up(bytes);
        {
            std::lock_guard<std::mutex> g(mu);
            auto it = free_.find(*cls);
            if (it != free_.end()) {
                void *p = it->second;
                free_.erase(it);
                return p;
            }
        }
        void *p = nullptr;
        if (hipHostMalloc(&p, *cls, hipHostMallocDefault) != hipSuccess) {
            (void)hipGetLastError();
            return nullptr;
        }
        std::lock_guard<std::mutex> g(mu);
        all.push_back(p);
        held += *cls;
        return p;
    }
    void put(void *p, size_t cls)
    {
        if (!p) return;
        std::lock_guard<std::mutex> g(mu);
        free_.emplace(cls, p);
    }
    void release()
    {
        for (void *p : all) (void)hipHostFree(p);
        all.clear();
        free_.clear();
    }
};

enum RunState { QUEUED, RUNNING, DONE, FAILED };

struct Run {
    uint64_t ticket = 0;
    int64_t n = 0;
    int32_t n_steps = 0;
    int32_t set_rho_ref = 0;
    int32_t has_rho_ref = 0;
    int32_t uniform_h = 1;
    sph_params prm{};
    sph_box box{};
    double h_max = 0.0;
    Grid grid{};
    int64_t ncell = 0;
    // initial state, rows x y z vx vy vz u h m p_bg [rho_ref], then id
    std::vector<double> ic;
    std::vector<int32_t> ic_id;
    // engine-thread state
    int slot = -1;
    int32_t launched = 0;    // steps of this run launched so far (the t = 0 evaluation is 0)
    int64_t start = 0;       // first particle in the arena for the current step
    void *blk = nullptr;     // pinned staging: upload, then the results
    size_t blk_cls = 0;
    bool ahead = false;      // staged by the engine before its admission
    // results (valid once DONE)
    RunState state = QUEUED;
    sph_status status = SPH_OK;
    double t_submit = 0, t_admit = 0, t_done = 0;
};

// Bytes of the pinned block of a run: 11 rows of doubles and the ids.
size_t block_bytes(int64_t n) { return (size_t)n * (kEnsFields * 8 + 4) + 256; }

// Result layout inside the block (after the run's last step): rows
// x y z vx vy vz u rho (8 n doubles), id (n int32), then dt, diag[8],
// status (at fixed offsets after the ids).
size_t res_id_off(int64_t n) { return (size_t)n * 8 * 8; }
size_t res_tail_off(int64_t n) { return ((res_id_off(n) + (size_t)n * 4 + 63) / 64) * 64; }

struct Upload {
    BatchHdr hdr;
    RunDev runs[kEnsMaxSlots];
};

}  // namespace

struct sph_ens_s {
    sph_ens_config cfg{};
    hipStream_t stream = nullptr;
    sph_ctx ctx = nullptr;  // sort, cell and record scratch for the capacity
    int64_t cap = 0, cell_cap = 0, nred_cap = 0;
    int64_t bytes_per_particle = 0, bytes_total = 0;

    // arena
    double *F = nullptr;  // kEnsFields rows of cap
    double *rho = nullptr, *p = nullptr, *c = nullptr, *pr2 = nullptr;
    double *ax = nullptr, *ay = nullptr, *az = nullptr, *dudt = nullptr, *mumax = nullptr;
    int32_t *count = nullptr, *idx = nullptr, *id = nullptr, *slot = nullptr,
            *slot_tmp = nullptr;
    double *red_part = nullptr, *dt = nullptr, *diag = nullptr;
    uint32_t *status = nullptr;
    BatchHdr *hdr_dev = nullptr;
    RunDev *runs_dev = nullptr;
    BatchDev bd{};

    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    Upload *up[3] = {nullptr, nullptr, nullptr};
    hipEvent_t ev[3] = {nullptr, nullptr, nullptr};
    PinnedPool pool;

    // shared with clients (under mu)
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<Run *> queue;
    std::unordered_map<uint64_t, std::unique_ptr<Run>> runs;
    uint64_t next_ticket = 1;
    bool stop = false;
    sph_status fatal = SPH_OK;
    std::string fatal_msg;
    sph_ens_counters ctr{};
    double t_first_busy = -1.0;

    std::thread th;
    std::string last_error;
};

namespace {

sph_status efail(sph_ens e, sph_status s, const char *fmt, ...)
    __attribute__((format(printf, 3, 4)));

sph_status efail(sph_ens e, sph_status s, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (e) {
        std::lock_guard<std::mutex> g(e->mu);
        e->last_error = buf;
    } else {
        g_ens_error = buf;
    }
    return s;
}

// Device bytes per particle of the arena plus the context scratch for it.
int64_t arena_bytes_per_particle(int max_nb)
{
    const int64_t arena = kEnsFields * 8      // state rows
                          + 9 * 8             // rho p c pr2 ax ay az dudt mumax
                          + 4 + 4 * max_nb    // count, idx
                          + 3 * 4;            // id, slot, slot_tmp
    const int64_t scratch = 2 * 4 + 2 * 4     // keys, vals (double-buffered)
                            + 1               // sort histograms (256 / 2048 * 4)
                            + 1               // cell table (cap / 8 cells * 8 B)
                            + kSearchMaskWords * 4  // search bit masks
                            + 32 + 32 + 128   // search, density, pair records
                            + kPermFields * 8 + 4;  // reorder scratch
    return arena + scratch;
}

template <typename T>
bool dalloc(sph_ens e, T **ptr, int64_t count)
{
    const size_t bytes = sizeof(T) * (size_t)std::max<int64_t>(count, 1);
    if (hipMalloc((void **)ptr, bytes) != hipSuccess) {
        *ptr = nullptr;
        (void)hipGetLastError();
        return false;
    }
    e->bytes_total += (int64_t)bytes;
    return true;
}

void free_ens(sph_ens e)
{
    if (e->exec) (void)hipGraphExecDestroy(e->exec);
    if (e->graph) (void)hipGraphDestroy(e->graph);
    for (int k = 0; k < 3; ++k) {
        if (e->ev[k]) (void)hipEventDestroy(e->ev[k]);
        if (e->up[k]) (void)hipHostFree(e->up[k]);
    }
    void *ptrs[] = {e->F, e->rho, e->p, e->c, e->pr2, e->ax, e->ay, e->az, e->dudt, e->mumax,
                    e->count, e->idx, e->id, e->slot, e->slot_tmp, e->red_part, e->dt,
                    e->diag, e->status, e->hdr_dev, e->runs_dev};
    for (void *q : ptrs)
        if (q) (void)hipFree(q);
    e->pool.release();
    if (e->ctx) sph_ctx_destroy(e->ctx);
    if (e->stream) (void)hipStreamDestroy(e->stream);
    delete e;
}

// The launch sequence of one batched step, captured once into a graph:
// admit, kick-drift, build, search, density, EOS, momentum, kick, dt.
hipError_t capture_step(sph_ens e)
{
    const BatchDev &b = e->bd;
    const int prec = e->cfg.precision, mnb = e->cfg.max_nb;
    hipError_t r;
    if ((r = hipStreamBeginCapture(e->stream, hipStreamCaptureModeThreadLocal)) != hipSuccess)
        return r;
    auto run = [&]() -> hipError_t {
        hipError_t q;
        if ((q = launch_admit_batch(e->ctx, b)) != hipSuccess) return q;
        if ((q = launch_integrate_batch(e->ctx, b, SPH_KICK_DRIFT, e->F, e->ax, e->ay, e->az,
                                        e->dudt)) != hipSuccess)
            return q;
        if ((q = launch_build_cells_batch(e->ctx, b, e->F, e->id, e->slot_tmp)) != hipSuccess)
            return q;
        if ((q = launch_find_neighbors_batch(e->ctx, b, mnb, e->count, e->idx)) != hipSuccess)
            return q;
        if ((q = launch_density_batch(e->ctx, b, prec, e->F, e->count, e->idx, mnb, e->rho)) !=
            hipSuccess)
            return q;
        if ((q = launch_eos_batch(e->ctx, b, e->F, e->rho, e->p, e->c, e->pr2)) != hipSuccess)
            return q;
        if ((q = launch_momentum_batch(e->ctx, b, prec, e->F, e->count, e->idx, mnb, e->rho,
                                       e->c, e->pr2, e->ax, e->ay, e->az, e->dudt,
                                       e->mumax)) != hipSuccess)
            return q;
        if ((q = launch_integrate_batch(e->ctx, b, SPH_KICK, e->F, e->ax, e->ay, e->az,
                                        e->dudt)) != hipSuccess)
            return q;
        return launch_timestep_batch(e->ctx, b, e->F, e->c, e->mumax, e->ax, e->ay, e->az,
                                     e->red_part);
    };
    hipError_t q = run();
    hipGraph_t g = nullptr;
    r = hipStreamEndCapture(e->stream, &g);
    if (q != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return q;
    }
    if (r != hipSuccess) return r;
    e->graph = g;
    return hipGraphInstantiate(&e->exec, g, nullptr, nullptr, 0);
}

}  // namespace

namespace {

struct InFlight {
    int ring;
    std::vector<Run *> done;  // runs whose final state is copied after this step
};

enum SlotState : uint8_t { SLOT_FREE, SLOT_LIVE, SLOT_DROP };

sph_status device_status(uint32_t st)
{
    if (st & ST_DOMAIN) return SPH_E_DOMAIN;
    if (st & ST_CAPACITY) return SPH_E_CAPACITY;
    if (st & ST_NONFINITE) return SPH_E_NONFINITE;
    return SPH_OK;
}

// Under e->mu: every unfinished run fails with s; the engine stops.
void fail_all_locked(sph_ens e, sph_status s, const std::string &msg)
{
    e->fatal = s;
    e->fatal_msg = msg;
    const double t = clock_s();
    for (auto &kv : e->runs) {
        Run *r = kv.second.get();
        if (r->state == QUEUED || r->state == RUNNING) {
            r->state = FAILED;
            r->status = s;
            r->t_done = t;
        }
    }
    e->queue.clear();
    e->ctr.queued = 0;
    e->ctr.running = 0;
    e->cv_done.notify_all();
}

void fill_run_dev(RunDev &d, const Run &r, int32_t phase)
{
    d = RunDev{};
    d.grid = r.grid;
    d.h_max = r.h_max;
    d.rho0 = r.prm.rho0;
    d.c0 = r.prm.c0;
    d.gamma_tait = r.prm.gamma_tait;
    d.gamma_gas = r.prm.gamma_gas;
    d.alpha = r.prm.alpha;
    d.beta = r.prm.beta;
    d.eta2 = r.prm.eta2;
    d.c_cfl = r.prm.c_cfl;
    d.c_force = r.prm.c_force;
    d.eos = r.prm.eos;
    d.phase = phase;
    d.set_rho_ref = r.set_rho_ref;
    d.uniform_h = r.uniform_h;
    d.ncell = (int32_t)r.ncell;
    d.n = (int32_t)r.n;
}

void engine_main(sph_ens e)
{
    auto die = [&](hipError_t err, const char *where) {
        (void)hipGetLastError();
        char buf[256];
        snprintf(buf, sizeof buf, "%s: %s", where, hipGetErrorString(err));
        std::lock_guard<std::mutex> g(e->mu);
        fail_all_locked(e, SPH_E_HIP, buf);
    };
    hipError_t err = hipSetDevice(e->cfg.device);
    if (err != hipSuccess) return die(err, "hipSetDevice");

    const int S = e->cfg.max_slots;
    const int64_t cap = e->cap;
    // A run is dereferenced only while its slot is live and its last step
    // has not been launched: once that step completes, a client may take
    // (and free) the run at any time.
    std::vector<Run *> slot_run(S, nullptr);
    std::vector<uint8_t> slot_state(S, SLOT_FREE);
    std::vector<uint8_t> slot_final(S, 0);  // last step of the slot's run launched
    int64_t resident = 0;  // particles of the runs live in the last launched step
    std::deque<InFlight> inflight;
    uint64_t stepno = 0;
    bool idle = false;
    // Initial states are staged in pinned memory (a pool block, allocated
    // the first time a size is needed) ahead of admission, while the GPU
    // works on the steps in flight: the queue head is staged in chunks of at
    // most kStageChunk bytes per wait, up to kStageAhead bytes of staged runs
    // not yet admitted. A run admitted unstaged is staged before its upload.
    constexpr size_t kStageChunk = (size_t)64 << 20, kStageAhead = (size_t)1 << 30;
    size_t staged_ahead = 0;
    auto stage = [&](Run *r) -> bool {
        r->blk = e->pool.get(block_bytes(r->n), &r->blk_cls);
        if (!r->blk) return false;
        std::memcpy(r->blk, r->ic.data(), r->ic.size() * sizeof(double));
        std::memcpy((char *)r->blk + (size_t)r->n * kEnsFields * 8, r->ic_id.data(),
                    (size_t)r->n * 4);
        std::vector<double>().swap(r->ic);
        std::vector<int32_t>().swap(r->ic_id);
        return true;
    };
    auto stage_ahead = [&]() -> bool {
        size_t done = 0;
        while (done < kStageChunk && staged_ahead < kStageAhead) {
            Run *r = nullptr;
            {
                std::lock_guard<std::mutex> g(e->mu);
                for (Run *q : e->queue)
                    if (!q->blk) {
                        r = q;
                        break;
                    }
            }
            if (!r) break;  // queued runs are removed by this thread only
            if (!stage(r)) return false;
            r->ahead = true;
            done += block_bytes(r->n);
            staged_ahead += block_bytes(r->n);
        }
        return true;
    };

    for (;;) {
        // 1. Retire finished steps. Block on the oldest when two are in
        // flight, or when nothing can be launched before it completes.
        while (!inflight.empty()) {
            InFlight &f = inflight.front();
            const bool block = inflight.size() >= 2 || idle;
            if (block && !stage_ahead()) {
                std::lock_guard<std::mutex> g(e->mu);
                fail_all_locked(e, SPH_E_NOMEM, "pinned host allocation failed");
                return;
            }
            err = block ? hipEventSynchronize(e->ev[f.ring]) : hipEventQuery(e->ev[f.ring]);
            if (err == hipErrorNotReady) {
                (void)hipGetLastError();
                break;
            }
            if (err != hipSuccess) return die(err, "step completion");
            idle = false;
            const double t = clock_s();
            std::lock_guard<std::mutex> g(e->mu);
            for (Run *r : f.done) {
                const char *tail = (const char *)r->blk + res_tail_off(r->n);
                uint32_t st;
                std::memcpy(&st, tail + 9 * sizeof(double), sizeof st);
                r->status = device_status(st);
                r->state = DONE;
                r->t_done = t;
                e->ctr.completed++;
                e->ctr.running--;
                e->ctr.busy_seconds = t - e->t_first_busy;
            }
            if (!f.done.empty()) e->cv_done.notify_all();
            inflight.pop_front();
        }

        // 2. Compose the next step: runs whose last step was launched are
        // sorted out of the arena by this step, their slots free up after
        // it; queued runs are admitted in order while they fit.
        std::vector<Run *> admitted;
        int64_t n_in = 0;
        {
            std::unique_lock<std::mutex> lk(e->mu);
            int64_t ncell = 0;
            int nlive = 0;
            for (int s = 0; s < S; ++s) {
                if (slot_state[s] == SLOT_DROP) {
                    slot_state[s] = SLOT_FREE;
                    slot_run[s] = nullptr;
                } else if (slot_state[s] == SLOT_LIVE && slot_final[s]) {
                    slot_state[s] = SLOT_DROP;
                    slot_final[s] = 0;
                    slot_run[s] = nullptr;
                } else if (slot_state[s] == SLOT_LIVE) {
                    ncell += slot_run[s]->ncell;
                    ++nlive;
                }
            }
            if (nlive == 0) {
                // nothing stays resident: the arena is empty again
                resident = 0;
                std::fill(slot_state.begin(), slot_state.end(), (uint8_t)SLOT_FREE);
                std::fill(slot_run.begin(), slot_run.end(), nullptr);
            }
            n_in = resident;
            int next_free = 0;
            while (!e->queue.empty()) {
                Run *r = e->queue.front();
                while (next_free < S && slot_state[next_free] != SLOT_FREE) ++next_free;
                if (next_free >= S) break;
                if (n_in + r->n > cap || ncell + r->ncell > e->cell_cap) break;
                e->queue.pop_front();
                r->slot = next_free;
                r->launched = 0;
                r->state = RUNNING;
                r->t_admit = clock_s();
                if (e->t_first_busy < 0) e->t_first_busy = r->t_admit;
                slot_state[next_free] = SLOT_LIVE;
                slot_run[next_free] = r;
                admitted.push_back(r);
                n_in += r->n;
                ncell += r->ncell;
                ++nlive;
                e->ctr.queued--;
                e->ctr.running++;
            }
            if (nlive == 0) {
                if (!inflight.empty()) {
                    idle = true;
                    continue;
                }
                if (e->stop && e->queue.empty()) break;
                e->cv_work.wait(lk, [&] { return e->stop || !e->queue.empty(); });
                continue;
            }
        }
        // the admitted runs' initial state in pinned memory
        for (Run *r : admitted) {
            if (r->blk) {
                if (r->ahead) staged_ahead -= block_bytes(r->n);
                continue;
            }
            if (!stage(r)) {
                std::lock_guard<std::mutex> g(e->mu);
                fail_all_locked(e, SPH_E_NOMEM, "pinned host allocation failed");
                return;
            }
        }

        // 3. Header and run table, in slot order.
        const int ring = (int)(stepno % 3);
        Upload *u = e->up[ring];
        BatchHdr &hd = u->hdr;
        std::vector<Run *> finishing;
        int64_t start = 0, cbase = 0, rbase = 0, tbase = 0;
        int nl = 0;
        for (int s = 0; s < S; ++s) {
            RunDev &d = u->runs[s];
            d = RunDev{};
            if (slot_state[s] == SLOT_DROP) d.phase = RUN_DROP;
            if (slot_state[s] != SLOT_LIVE) continue;
            Run *r = slot_run[s];
            fill_run_dev(d, *r, r->launched == 0 ? RUN_INIT : RUN_STEP);
            d.start = (int32_t)start;
            d.cell_base = (int32_t)cbase;
            d.red_base = (int32_t)rbase;
            r->start = start;
            hd.live_slot[nl] = s;
            hd.live_cell_base[nl] = (int32_t)cbase;
            hd.live_red_base[nl] = (int32_t)rbase;
            hd.live_tile_base[nl] = (int32_t)tbase;
            ++nl;
            start += r->n;
            cbase += r->ncell;
            rbase += (r->n + kRedThreads - 1) / kRedThreads;
            tbase += (r->n + 63) / 64;
            if (r->launched == r->n_steps) finishing.push_back(r);
        }
        hd.live_cell_base[nl] = (int32_t)cbase;
        hd.live_red_base[nl] = (int32_t)rbase;
        hd.live_tile_base[nl] = (int32_t)tbase;
        hd.ntile = tbase;
        hd.n_in = n_in;
        hd.n_out = start;
        hd.ncell = cbase;
        hd.nred = rbase;
        hd.nlive = nl;
        hd.nnew = (int32_t)admitted.size();
        int64_t off = resident;
        for (size_t k = 0; k < admitted.size(); ++k) {
            hd.new_slot[k] = admitted[k]->slot;
            hd.new_off[k] = (int32_t)off;
            hd.new_n[k] = (int32_t)admitted[k]->n;
            off += admitted[k]->n;
        }

        // 4. Uploads, the step, the copies back, the completion event.
        off = resident;
        for (Run *r : admitted) {
            const int rows = r->has_rho_ref ? kEnsFields : kEnsFields - 1;
            err = hipMemcpy2DAsync(e->F + off, (size_t)cap * 8, r->blk, (size_t)r->n * 8,
                                   (size_t)r->n * 8, rows, hipMemcpyHostToDevice, e->stream);
            if (err == hipSuccess)
                err = hipMemcpyAsync(e->id + off,
                                     (const char *)r->blk + (size_t)r->n * kEnsFields * 8,
                                     (size_t)r->n * 4, hipMemcpyHostToDevice, e->stream);
            if (err != hipSuccess) return die(err, "upload of a run");
            off += r->n;
        }
        err = hipMemcpyAsync(e->hdr_dev, &u->hdr, sizeof(BatchHdr), hipMemcpyHostToDevice,
                             e->stream);
        if (err == hipSuccess)
            err = hipMemcpyAsync(e->runs_dev, u->runs, sizeof(RunDev) * (size_t)S,
                                 hipMemcpyHostToDevice, e->stream);
        if (err != hipSuccess) return die(err, "header upload");
        err = hipGraphLaunch(e->exec, e->stream);
        if (err != hipSuccess) return die(err, "hipGraphLaunch");
        for (Run *r : finishing) {
            char *blk = (char *)r->blk;
            const size_t nb = (size_t)r->n * 8;
            err = hipMemcpy2DAsync(blk, nb, e->F + r->start, (size_t)cap * 8, nb, 7,
                                   hipMemcpyDeviceToHost, e->stream);
            if (err == hipSuccess)
                err = hipMemcpyAsync(blk + 7 * nb, e->rho + r->start, nb, hipMemcpyDeviceToHost,
                                     e->stream);
            if (err == hipSuccess)
                err = hipMemcpyAsync(blk + res_id_off(r->n), e->id + r->start, (size_t)r->n * 4,
                                     hipMemcpyDeviceToHost, e->stream);
            char *tail = blk + res_tail_off(r->n);
            if (err == hipSuccess)
                err = hipMemcpyAsync(tail, e->dt + r->slot, 8, hipMemcpyDeviceToHost, e->stream);
            if (err == hipSuccess)
                err = hipMemcpyAsync(tail + 8, e->diag + (size_t)r->slot * 8, 64,
                                     hipMemcpyDeviceToHost, e->stream);
            if (err == hipSuccess)
                err = hipMemcpyAsync(tail + 72, e->status + r->slot, 4, hipMemcpyDeviceToHost,
                                     e->stream);
            if (err != hipSuccess) return die(err, "result copy");
            slot_final[r->slot] = 1;
        }
        err = hipEventRecord(e->ev[ring], e->stream);
        if (err != hipSuccess) return die(err, "hipEventRecord");
        for (int s = 0; s < S; ++s)
            if (slot_state[s] == SLOT_LIVE) slot_run[s]->launched++;
        inflight.push_back(InFlight{ring, std::move(finishing)});
        ++stepno;
        resident = start;
        std::lock_guard<std::mutex> g(e->mu);
        e->ctr.steps++;
        e->ctr.particle_steps += start;
        e->ctr.peak_particles = std::max<int64_t>(e->ctr.peak_particles, start);
        e->ctr.peak_runs = std::max<int32_t>(e->ctr.peak_runs, nl);
    }
    // drain
    while (!inflight.empty()) {
        err = hipEventSynchronize(e->ev[inflight.front().ring]);
        if (err != hipSuccess) return die(err, "drain");
        inflight.pop_front();
    }
}

// Scatter a finished run's results into the caller's buffers.
void fill_result(const Run &r, sph_run_result *res)
{
    const int64_t n = r.n;
    res->t_submit = r.t_submit;
    res->t_admit = r.t_admit;
    res->t_done = r.t_done;
    res->status = r.status;
    res->steps_done = r.state == DONE ? r.n_steps : 0;
    std::memset(res->diag, 0, sizeof res->diag);
    res->dt = 0.0;
    if (r.state != DONE || !r.blk) return;
    const char *blk = (const char *)r.blk;
    const double *rows = (const double *)blk;
    const int32_t *id = (const int32_t *)(blk + res_id_off(n));
    const char *tail = blk + res_tail_off(n);
    std::memcpy(&res->dt, tail, 8);
    std::memcpy(res->diag, tail + 8, 64);
    double *dst[8] = {res->x, res->y, res->z, res->vx, res->vy, res->vz, res->u, res->rho};
    for (int k = 0; k < 8; ++k) {
        if (!dst[k]) continue;
        const double *src = rows + (size_t)k * n;
        double *d = dst[k];
        for (int64_t q = 0; q < n; ++q) d[id[q]] = src[q];
    }
}

sph_status take_result(sph_ens e, uint64_t ticket, sph_run_result *res, bool block)
{
    if (!e) return efail(nullptr, SPH_E_INVALID, "engine is NULL");
    if (!res) return efail(e, SPH_E_INVALID, "result is NULL");
    std::unique_ptr<Run> run;
    {
        std::unique_lock<std::mutex> lk(e->mu);
        auto it = e->runs.find(ticket);
        if (it == e->runs.end()) {
            e->last_error = "unknown ticket";
            return SPH_E_INVALID;
        }
        Run *r = it->second.get();
        if (block)
            e->cv_done.wait(lk, [&] { return r->state == DONE || r->state == FAILED; });
        if (r->state != DONE && r->state != FAILED) return SPH_E_AGAIN;
        run = std::move(it->second);
        e->runs.erase(it);
    }
    fill_result(*run, res);
    e->pool.put(run->blk, run->blk_cls);
    return SPH_OK;
}

}  // namespace

extern "C" {

double sph_ens_clock(void) { return clock_s(); }

const char *sph_ens_last_error(sph_ens e)
{
    if (!e) return g_ens_error.c_str();
    std::lock_guard<std::mutex> g(e->mu);
    thread_local std::string copy;
    copy = e->fatal != SPH_OK && e->last_error.empty() ? e->fatal_msg : e->last_error;
    return copy.c_str();
}

sph_status sph_ens_create(sph_ens *out, const sph_ens_config *cfg)
{
    if (!out || !cfg) return efail(nullptr, SPH_E_INVALID, "out and cfg are required");
    *out = nullptr;
    if (cfg->precision != SPH_FP64 && cfg->precision != SPH_FP32_PAIR)
        return efail(nullptr, SPH_E_INVALID, "unknown precision %d", cfg->precision);
    if (cfg->max_nb < 1 || cfg->max_nb > 4096)
        return efail(nullptr, SPH_E_INVALID, "max_nb = %d outside [1, 4096]", cfg->max_nb);
    if (cfg->max_slots < 1 || cfg->max_slots > kEnsMaxSlots)
        return efail(nullptr, SPH_E_INVALID, "max_slots = %d outside [1, %d]", cfg->max_slots,
                     kEnsMaxSlots);
    if (cfg->max_n_per_run < 1 || cfg->max_n_per_run > ((int64_t)1 << 30))
        return efail(nullptr, SPH_E_INVALID, "max_n_per_run out of range");
    const int64_t bpp = arena_bytes_per_particle(cfg->max_nb);
    const int64_t fixed = (int64_t)16 << 20;
    int64_t cap = (cfg->hbm_budget_bytes - fixed) / bpp;
    cap = std::min<int64_t>(cap, ((int64_t)1 << 31) - kSortTile - 1);
    if (cap < cfg->max_n_per_run)
        return efail(nullptr, SPH_E_INVALID,
                     "a budget of %lld bytes holds %lld particles (%lld B each), less than "
                     "max_n_per_run = %lld",
                     (long long)cfg->hbm_budget_bytes, (long long)std::max<int64_t>(cap, 0),
                     (long long)bpp, (long long)cfg->max_n_per_run);
    hipError_t err = hipSetDevice(cfg->device);
    if (err != hipSuccess)
        return efail(nullptr, SPH_E_HIP, "hipSetDevice: %s", hipGetErrorString(err));

    sph_ens e = new (std::nothrow) sph_ens_s;
    if (!e) return efail(nullptr, SPH_E_NOMEM, "host allocation failed");
    e->cfg = *cfg;
    e->cap = cap;
    e->bytes_per_particle = bpp;
    e->nred_cap = (cap + kRedThreads - 1) / kRedThreads + kEnsMaxSlots;
    auto bail = [&](sph_status s, const char *msg) {
        g_ens_error = msg;
        free_ens(e);
        return s;
    };
    if ((err = hipStreamCreateWithFlags(&e->stream, hipStreamNonBlocking)) != hipSuccess)
        return bail(SPH_E_HIP, "hipStreamCreateWithFlags failed");
    // the search cuts every run into its own tiles of 64: at most one more
    // (partial) tile per run than the arena's capacity holds
    sph_status s = sph_ctx_create(&e->ctx, cap + 64 * (int64_t)kEnsMaxSlots, cfg->max_nb,
                                  e->stream);
    if (s != SPH_OK) {
        std::string m = std::string("scratch: ") + sph_last_error(nullptr);
        return bail(s, m.c_str());
    }
    e->bytes_total = sph_ctx_scratch_bytes(e->ctx);
    e->cell_cap = e->ctx->cell_cap;
    const int64_t nb = cfg->max_nb;
    bool ok = dalloc(e, &e->F, (int64_t)kEnsFields * cap) && dalloc(e, &e->rho, cap) &&
              dalloc(e, &e->p, cap) && dalloc(e, &e->c, cap) && dalloc(e, &e->pr2, cap) &&
              dalloc(e, &e->ax, cap) && dalloc(e, &e->ay, cap) && dalloc(e, &e->az, cap) &&
              dalloc(e, &e->dudt, cap) && dalloc(e, &e->mumax, cap) &&
              dalloc(e, &e->count, cap) && dalloc(e, &e->idx, nb * cap) &&
              dalloc(e, &e->id, cap) && dalloc(e, &e->slot, cap) &&
              dalloc(e, &e->slot_tmp, cap) &&
              dalloc(e, &e->red_part, (int64_t)kRedFields * e->nred_cap) &&
              dalloc(e, &e->dt, kEnsMaxSlots) && dalloc(e, &e->diag, 8 * kEnsMaxSlots) &&
              dalloc(e, &e->status, kEnsMaxSlots) && dalloc(e, &e->hdr_dev, 1) &&
              dalloc(e, &e->runs_dev, kEnsMaxSlots);
    if (!ok) return bail(SPH_E_NOMEM, "device allocation of the arena failed");
    for (int k = 0; k < 3; ++k) {
        if (hipHostMalloc((void **)&e->up[k], sizeof(Upload), hipHostMallocDefault) !=
            hipSuccess) {
            e->up[k] = nullptr;
            return bail(SPH_E_NOMEM, "pinned header allocation failed");
        }
        std::memset(e->up[k], 0, sizeof(Upload));
        if (hipEventCreateWithFlags(&e->ev[k], hipEventDisableTiming) != hipSuccess)
            return bail(SPH_E_HIP, "hipEventCreateWithFlags failed");
    }
    e->bd = BatchDev{e->hdr_dev, e->runs_dev, e->slot, e->dt, e->diag, e->status,
                     cap, e->cell_cap, e->nred_cap};
    if ((err = capture_step(e)) != hipSuccess) {
        (void)hipGetLastError();
        std::string m = std::string("graph capture: ") + hipGetErrorString(err);
        return bail(SPH_E_HIP, m.c_str());
    }
    e->ctr.capacity_particles = cap;
    e->ctr.capacity_cells = e->cell_cap;
    e->ctr.bytes_per_particle = bpp;
    e->ctr.bytes_allocated = e->bytes_total;
    e->ctr.max_slots = cfg->max_slots;
    try {
        e->th = std::thread(engine_main, e);
    } catch (...) {
        return bail(SPH_E_NOMEM, "could not start the engine thread");
    }
    *out = e;
    return SPH_OK;
}

sph_status sph_ens_submit(sph_ens e, const sph_run_request *q, uint64_t *ticket)
{
    if (!e) return efail(nullptr, SPH_E_INVALID, "engine is NULL");
    if (!q || !ticket) return efail(e, SPH_E_INVALID, "request and ticket are required");
    const int64_t n = q->n;
    if (n < 1 || n > e->cfg.max_n_per_run)
        return efail(e, SPH_E_INVALID, "n = %lld outside [1, max_n_per_run = %lld]",
                     (long long)n, (long long)e->cfg.max_n_per_run);
    if (q->n_steps < 0) return efail(e, SPH_E_INVALID, "n_steps < 0");
    if (!q->x || !q->y || !q->z || !q->vx || !q->vy || !q->vz || !q->u || !q->h || !q->m ||
        !q->p_bg || !q->id)
        return efail(e, SPH_E_INVALID, "x, y, z, vx, vy, vz, u, h, m, p_bg and id are required");
    const sph_params &prm = q->params;
    if (prm.eos != SPH_EOS_TAIT && prm.eos != SPH_EOS_IDEAL)
        return efail(e, SPH_E_INVALID, "unknown eos %d", prm.eos);
    if (prm.kernel != SPH_KERNEL_M4 || prm.gradient != SPH_GRAD_KERNEL ||
        prm.volume != SPH_VOLUME_STANDARD)
        return efail(e, SPH_E_INVALID,
                     "the engine runs the M4 kernel with kernel derivatives and standard "
                     "volume elements only (kernel %d, gradient %d, volume %d)", prm.kernel,
                     prm.gradient, prm.volume);
    if (prm.eos == SPH_EOS_TAIT && !q->set_rho_ref && !q->rho_ref)
        return efail(e, SPH_E_INVALID, "the Tait EOS needs rho_ref or set_rho_ref");
    for (int a = 0; a < 3; ++a) {
        if (!(std::isfinite(q->box.lo[a]) && std::isfinite(q->box.hi[a]) &&
              q->box.hi[a] > q->box.lo[a]))
            return efail(e, SPH_E_INVALID, "box axis %d: need finite lo < hi", a);
        if (q->box.periodic[a] != 0 && q->box.periodic[a] != 1)
            return efail(e, SPH_E_INVALID, "box axis %d: periodic must be 0 or 1", a);
    }
    if (!(q->h_max > 0.0) || !std::isfinite(q->h_max))
        return efail(e, SPH_E_INVALID, "h_max must be finite and > 0");
    for (int a = 0; a < 3; ++a)
        if (q->box.periodic[a] && !(q->box.hi[a] - q->box.lo[a] > 4.0 * q->h_max))
            return efail(e, SPH_E_DOMAIN, "periodic axis %d is not longer than 4 h_max", a);
    auto r = std::make_unique<Run>();
    r->n = n;
    r->n_steps = q->n_steps;
    r->prm = prm;
    r->box = q->box;
    r->h_max = q->h_max;
    r->set_rho_ref = q->set_rho_ref ? 1 : 0;
    r->has_rho_ref = q->rho_ref && !q->set_rho_ref ? 1 : 0;
    const double h0 = q->h[0];
    for (int64_t k = 0; k < n; ++k) {
        const double hk = q->h[k];
        if (!(hk > 0.0)) return efail(e, SPH_E_INVALID, "h must be > 0");
        if (!(hk <= q->h_max)) return efail(e, SPH_E_DOMAIN, "some h > h_max");
        if (hk != h0) r->uniform_h = 0;
    }
    {
        std::vector<uint8_t> seen((size_t)n, 0);
        for (int64_t k = 0; k < n; ++k) {
            const int32_t v = q->id[k];
            if (v < 0 || v >= n || seen[(size_t)v])
                return efail(e, SPH_E_INVALID, "id is not a permutation of 0..n-1");
            seen[(size_t)v] = 1;
        }
    }
    r->grid = make_grid(q->box, q->h_max, e->cell_cap, 1 << kEnsAxisBits);
    r->ncell = (int64_t)r->grid.nc[0] * r->grid.nc[1] * r->grid.nc[2];
    if (n > e->cap || r->ncell > e->cell_cap)
        return efail(e, SPH_E_CAPACITY, "the run can never fit the budget");
    // The initial state goes straight into a pinned block while the pool
    // holds less than cfg.pinned_submit_bytes (the engine then only uploads
    // it), else into host vectors that the engine stages before the upload.
    const double *rows[kEnsFields] = {q->x, q->y, q->z, q->vx, q->vy, q->vz, q->u,
                                      q->h, q->m, q->p_bg, q->rho_ref};
    const int64_t lim = e->cfg.pinned_submit_bytes;
    const size_t submit_pinned = lim == 0 ? (size_t)4 << 30 : (lim < 0 ? 0 : (size_t)lim);
    if (e->pool.held.load() + block_bytes(n) <= submit_pinned)
        r->blk = e->pool.get(block_bytes(n), &r->blk_cls);
    if (r->blk) {
        for (int k = 0; k < kEnsFields; ++k) {
            if (!rows[k] || (k == kEnsFields - 1 && !r->has_rho_ref)) continue;
            std::memcpy((double *)r->blk + (size_t)k * n, rows[k], (size_t)n * 8);
        }
        std::memcpy((char *)r->blk + (size_t)n * kEnsFields * 8, q->id, (size_t)n * 4);
    } else {
        r->ic.resize((size_t)n * kEnsFields);
        for (int k = 0; k < kEnsFields; ++k) {
            if (!rows[k] || (k == kEnsFields - 1 && !r->has_rho_ref)) continue;
            std::memcpy(r->ic.data() + (size_t)k * n, rows[k], (size_t)n * 8);
        }
        r->ic_id.assign(q->id, q->id + n);
    }
    std::lock_guard<std::mutex> g(e->mu);
    if (e->fatal != SPH_OK || e->stop) {
        e->pool.put(r->blk, r->blk_cls);
        if (e->fatal != SPH_OK) {
            e->last_error = e->fatal_msg;
            return e->fatal;
        }
        e->last_error = "the engine is shutting down";
        return SPH_E_INVALID;
    }
    r->ticket = e->next_ticket++;
    r->t_submit = clock_s();
    *ticket = r->ticket;
    e->queue.push_back(r.get());
    e->runs.emplace(r->ticket, std::move(r));
    e->ctr.submitted++;
    e->ctr.queued++;
    e->cv_work.notify_one();
    return SPH_OK;
}

sph_status sph_ens_poll(sph_ens e, uint64_t ticket, sph_run_result *res)
{
    return take_result(e, ticket, res, false);
}

sph_status sph_ens_wait(sph_ens e, uint64_t ticket, sph_run_result *res)
{
    return take_result(e, ticket, res, true);
}

sph_status sph_ens_stats(sph_ens e, sph_ens_counters *out)
{
    if (!e || !out) return efail(e, SPH_E_INVALID, "engine and out are required");
    std::lock_guard<std::mutex> g(e->mu);
    *out = e->ctr;
    return e->fatal;
}

sph_status sph_ens_destroy(sph_ens e)
{
    if (!e) return efail(nullptr, SPH_E_INVALID, "engine is NULL");
    {
        std::lock_guard<std::mutex> g(e->mu);
        e->stop = true;
    }
    e->cv_work.notify_all();
    if (e->th.joinable()) e->th.join();
    const sph_status s = e->fatal;
    (void)hipStreamSynchronize(e->stream);
    free_ens(e);
    return s;
}

}  // extern "C"
