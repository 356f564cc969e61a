// Many independent runs advanced together: the batched ensemble (mhd_batch_*) and
// the continuous-batching request loop (mhd_server_*).
//
// Runs are grouped by (precision, tile shape).  Each group has one tile list that
// concatenates the tiles of its runs (XCD-ordered) and one array of run
// descriptors; a substep of the whole group is one kernel launch.  Every run keeps
// its own buffers, forcing blocks, partials and records, so its arithmetic is the
// same cell by cell as when it runs alone.
#include "mhd.h"
#include "mhd_host.h"

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <set>
#include <thread>
#include <vector>

namespace mhd {

// Cells that the runs of one precision in a batch must bring for each of them to take
// the filled-chip tile: 16 ring work-groups of 1024 cells per CU.
constexpr double BATCH_FILL_CELLS = 4096.0 * 1024;

struct Group {
    int prec = 8;
    int shape = 0;
    bool fit = false;
    int upk = 0;               // 4 when the group's runs use upwinding (launch kinds 4-6)
    std::vector<mhd_ctx *> members;
    int ntiles = 0;
    int ntiles_w = 0;          // 64-wide tiles of substeps 1 and 2 (wide shapes)
    int max_nb2 = 0;
    TileEnt *d_tiles = nullptr;
    TileEnt *d_tiles_w = nullptr;
    void *d_descs = nullptr;
    void *h_descs = nullptr;   // pinned staging
    size_t desc_bytes = 0;
};

struct MultiRunner {
    hipStream_t stream = nullptr;
    bool own_stream = false;
    std::vector<Group> groups;
    hipEvent_t stage_evt = nullptr;
    // runs of different power-of-two size classes go to separate groups (so that they can
    // take different numbers of steps per call)
    bool split_by_size = false;
    // captured graphs, keyed by the number of steps of every group
    std::map<std::vector<int64_t>, hipGraphExec_t> graphs;
    // step counts launched once without a graph (capture_on_reuse): captured when seen again
    std::set<std::vector<int64_t>> seen_once;
    // false: capture a graph the first time a step count is run (batches: the caller
    // warms up once and then replays); true: launch directly the first time and capture
    // only when the same step counts come back (the server, whose set of runs changes
    // every few ticks: a graph used once costs its capture and instantiation for nothing)
    bool capture_on_reuse = false;

    ~MultiRunner() { clear(); }

    void clear_graphs()
    {
        for (auto &g : graphs) (void)hipGraphExecDestroy(g.second);
        graphs.clear();
        seen_once.clear();
    }

    void clear()
    {
        if (stream) (void)hipStreamSynchronize(stream);
        clear_graphs();
        for (auto &g : groups) {
            if (g.d_tiles) (void)hipFree(g.d_tiles);
            if (g.d_tiles_w) (void)hipFree(g.d_tiles_w);
            if (g.d_descs) (void)hipFree(g.d_descs);
            if (g.h_descs) (void)hipHostFree(g.h_descs);
        }
        groups.clear();
        if (stage_evt) (void)hipEventDestroy(stage_evt);
        stage_evt = nullptr;
    }

    mhd_status init_stream(void *s)
    {
        if (s) {
            stream = (hipStream_t)s;
        } else {
            // graph capture needs a stream other than the legacy default stream
            if (hipStreamCreateWithFlags(&stream, hipStreamNonBlocking) != hipSuccess)
                return fail(MHD_E_DEVICE, "hipStreamCreate failed");
            own_stream = true;
        }
        return MHD_OK;
    }

    void destroy_stream()
    {
        if (own_stream && stream) (void)hipStreamDestroy(stream);
        stream = nullptr;
        own_stream = false;
    }

    // (Re)build the groups for this set of contexts.
    mhd_status build(const std::vector<mhd_ctx *> &runs)
    {
        if (stream) (void)hipStreamSynchronize(stream);
        clear_graphs();
        for (auto &g : groups) {
            if (g.d_tiles) (void)hipFree(g.d_tiles);
            if (g.d_tiles_w) (void)hipFree(g.d_tiles_w);
            if (g.d_descs) (void)hipFree(g.d_descs);
            if (g.h_descs) (void)hipHostFree(g.h_descs);
        }
        groups.clear();
        if (!stage_evt && hipEventCreateWithFlags(&stage_evt, hipEventDisableTiming) != hipSuccess)
            return fail(MHD_E_DEVICE, "hipEventCreate failed");
        std::map<std::tuple<int, int, bool, int, int>, size_t> index;
        for (mhd_ctx *c : runs) {
            const int upk = c->p.upwind != 0.0 ? 4 : 0;
            const int cls = split_by_size ? (int)std::floor(std::log2((double)c->ncell)) : 0;
            auto key = std::make_tuple(c->p.precision, c->shape, c->fit, upk, cls);
            auto it = index.find(key);
            if (it == index.end()) {
                index[key] = groups.size();
                Group g;
                g.prec = c->p.precision;
                g.shape = c->shape;
                g.fit = c->fit;
                g.upk = upk;
                groups.push_back(g);
                it = index.find(key);
            }
            groups[it->second].members.push_back(c);
        }
        for (auto &g : groups) {
            std::vector<TileEnt> nat;
            for (size_t i = 0; i < g.members.size(); i++) run_tiles(g.members[i]->p, g.shape, (int)i, nat);
            std::vector<TileEnt> ord = xcd_order(nat);
            g.ntiles = (int)ord.size();
            for (mhd_ctx *c : g.members) g.max_nb2 = std::max(g.max_nb2, c->nb2);
            g.desc_bytes = g.members.size() * (g.prec == MHD_FP64 ? sizeof(RunDesc<double>) : sizeof(RunDesc<float>));
            if (hipMalloc(&g.d_tiles, ord.size() * sizeof(TileEnt)) != hipSuccess ||
                hipMalloc(&g.d_descs, g.desc_bytes) != hipSuccess ||
                hipHostMalloc(&g.h_descs, g.desc_bytes, hipHostMallocDefault) != hipSuccess)
                return fail(MHD_E_OOM, "batch: allocating tile lists failed");
            if (hipMemcpy(g.d_tiles, ord.data(), ord.size() * sizeof(TileEnt), hipMemcpyHostToDevice) != hipSuccess)
                return fail(MHD_E_DEVICE, "batch: tile upload failed");
            if (SHAPES[g.shape].wide) {
                nat.clear();
                for (size_t i = 0; i < g.members.size(); i++) run_tiles_wide(g.members[i]->p, (int)i, nat);
                ord = xcd_order(nat);
                g.ntiles_w = (int)ord.size();
                if (hipMalloc(&g.d_tiles_w, ord.size() * sizeof(TileEnt)) != hipSuccess)
                    return fail(MHD_E_OOM, "batch: allocating tile lists failed");
                if (hipMemcpy(g.d_tiles_w, ord.data(), ord.size() * sizeof(TileEnt), hipMemcpyHostToDevice) != hipSuccess)
                    return fail(MHD_E_DEVICE, "batch: tile upload failed");
            }
        }
        return MHD_OK;
    }

    template <typename T>
    hipError_t launch_group_step(Group &g, int s)
    {
        const RunDesc<T> *d = (const RunDesc<T> *)g.d_descs;
        const int nr = (int)g.members.size();
        hipError_t e = launch_substep<T>(g.shape, g.fit, 0 + g.upk, d, g.d_tiles, g.ntiles, g.d_tiles_w, g.ntiles_w, s, stream);
        if (e == hipSuccess) e = launch_finalize<T>(d, nr, g.max_nb2, s, stream);
        if (e == hipSuccess) e = launch_substep<T>(g.shape, g.fit, 1 + g.upk, d, g.d_tiles, g.ntiles, g.d_tiles_w, g.ntiles_w, s, stream);
        if (e == hipSuccess) e = launch_substep<T>(g.shape, g.fit, 2 + g.upk, d, g.d_tiles, g.ntiles, g.d_tiles_w, g.ntiles_w, s, stream);
        return e;
    }

    // Step s of every group that takes more than s steps (mg[g] steps for group g).
    hipError_t launch_steps(const std::vector<int64_t> &mg)
    {
        const int64_t m = *std::max_element(mg.begin(), mg.end());
        for (int64_t s = 0; s < m; s++)
            for (size_t gi = 0; gi < groups.size(); gi++) {
                if (s >= mg[gi]) continue;
                Group &g = groups[gi];
                hipError_t e = g.prec == MHD_FP64 ? launch_group_step<double>(g, (int)s)
                                                  : launch_group_step<float>(g, (int)s);
                if (e != hipSuccess) return e;
            }
        return hipSuccess;
    }

    // Stage forcing blocks and descriptors of every run of group g for mg[g] steps,
    // enqueue the uploads.
    mhd_status stage(const std::vector<int64_t> &mg)
    {
        if (hipEventSynchronize(stage_evt) != hipSuccess) return fail(MHD_E_DEVICE, "staging event failed");
        for (size_t gi = 0; gi < groups.size(); gi++) {
            Group &g = groups[gi];
            const int64_t m = mg[gi];
            for (size_t i = 0; i < g.members.size(); i++) {
                mhd_ctx *c = g.members[i];
                if (c->rcount + m > CHUNK) {
                    mhd_status st = ctx_drain(c);
                    if (st != MHD_OK) return st;
                }
                if (hipEventSynchronize(c->stage_evt) != hipSuccess) return fail(MHD_E_DEVICE, "staging event failed");
                mhd_status st = ctx_forcing_blocks(c, c->step, m, c->h_stage);
                if (st != MHD_OK) return st;
                const size_t fbytes = (size_t)m * c->fstride * c->p.precision;
                if (hipMemcpyAsync(c->d_forcing, c->h_stage, fbytes, hipMemcpyHostToDevice, stream) != hipSuccess ||
                    hipEventRecord(c->stage_evt, stream) != hipSuccess)
                    return fail(MHD_E_DEVICE, "forcing upload failed");
                if (g.prec == MHD_FP64)
                    fill_desc<double>(c, ((RunDesc<double> *)g.h_descs)[i], c->parity, c->step,
                                      (const double *)c->d_forcing, c->d_records + (size_t)c->rcount * DREC,
                                      c->d_partials, 0);
                else
                    fill_desc<float>(c, ((RunDesc<float> *)g.h_descs)[i], c->parity, c->step,
                                     (const float *)c->d_forcing, c->d_records + (size_t)c->rcount * DREC,
                                     c->d_partials, 0);
            }
            if (hipMemcpyAsync(g.d_descs, g.h_descs, g.desc_bytes, hipMemcpyHostToDevice, stream) != hipSuccess)
                return fail(MHD_E_DEVICE, "descriptor upload failed");
        }
        if (hipEventRecord(stage_evt, stream) != hipSuccess) return fail(MHD_E_DEVICE, "event record failed");
        return MHD_OK;
    }

    void advance(const std::vector<int64_t> &mg)
    {
        for (size_t gi = 0; gi < groups.size(); gi++)
            for (mhd_ctx *c : groups[gi].members) {
                c->rcount += mg[gi];
                c->parity ^= (int)(mg[gi] & 1);
                c->step += mg[gi];
            }
    }

    // Advance the runs of group g by mg[g] steps (1 <= mg[g] <= CHUNK), as one captured
    // graph (replayed for the same step counts) or as plain launches.
    mhd_status run_chunk(const std::vector<int64_t> &mg, bool use_graph)
    {
        if (groups.empty()) return MHD_OK;
        if (mg.size() != groups.size()) return fail(MHD_E_INVALID, "batch: one step count per group needed");
        for (int64_t m : mg)
            if (m < 1 || m > CHUNK) return fail(MHD_E_INVALID, "batch: step counts must lie in [1, CHUNK]");
        mhd_status st = stage(mg);
        if (st != MHD_OK) return st;
        if (use_graph && capture_on_reuse && !graphs.count(mg) && seen_once.insert(mg).second) use_graph = false;
        if (use_graph) {
            auto it = graphs.find(mg);
            if (it == graphs.end()) {
                hipGraph_t graph;
                if (hipStreamBeginCapture(stream, hipStreamCaptureModeThreadLocal) != hipSuccess)
                    return fail(MHD_E_DEVICE, "hipStreamBeginCapture failed");
                hipError_t e = launch_steps(mg);
                hipError_t e2 = hipStreamEndCapture(stream, &graph);
                if (e != hipSuccess || e2 != hipSuccess)
                    return fail(MHD_E_DEVICE, std::string("graph capture failed: ") +
                                                  hipGetErrorString(e != hipSuccess ? e : e2));
                hipGraphExec_t exec;
                e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
                (void)hipGraphDestroy(graph);
                if (e != hipSuccess)
                    return fail(MHD_E_DEVICE, std::string("graph instantiate failed: ") + hipGetErrorString(e));
                it = graphs.emplace(mg, exec).first;
            }
            if (hipGraphLaunch(it->second, stream) != hipSuccess) return fail(MHD_E_DEVICE, "graph launch failed");
        } else {
            hipError_t e = launch_steps(mg);
            if (e != hipSuccess) return fail(MHD_E_DEVICE, std::string("kernel launch failed: ") + hipGetErrorString(e));
        }
        advance(mg);
        return MHD_OK;
    }

    // Advance every run by nsteps (chunks of at most CHUNK steps).
    mhd_status run(int64_t nsteps, bool use_graph)
    {
        while (nsteps > 0) {
            const int64_t m = std::min<int64_t>(nsteps, CHUNK);
            mhd_status st = run_chunk(std::vector<int64_t>(groups.size(), m), use_graph);
            if (st != MHD_OK) return st;
            nsteps -= m;
        }
        return MHD_OK;
    }
};

}  // namespace mhd

using namespace mhd;

struct mhd_batch {
    std::vector<mhd_ctx *> runs;
    MultiRunner mr;
};

// ====================================================================== serving

namespace mhd {

struct Request {
    int64_t id = 0;
    mhd_params p{};
    uint64_t seed = 0;
    double a_noise = 0, kf = 0, f0 = 0, sigma = 0;
    int64_t nsteps = 0;
    bool retain = false;
    int state = MHD_RUN_QUEUED;
    double t_submit = 0, t_admit = 0, t_done = 0;
    int64_t steps_done = 0;
    size_t footprint = 0;
    mhd_ctx *ctx = nullptr;
    std::vector<std::vector<char>> kept;   // retained final state (host)
    double em = 0, brms = 0;
    double last_tdev = -1.0;               // device clock of the run's latest record (s)
};

static double pct(std::vector<double> v, double q)
{
    if (v.empty()) return 0.0;
    std::sort(v.begin(), v.end());
    const double pos = q * (double)(v.size() - 1);
    const size_t lo = (size_t)std::floor(pos), hi = std::min(v.size() - 1, lo + 1);
    return v[lo] + (pos - (double)lo) * (v[hi] - v[lo]);
}

}  // namespace mhd

// Fixed cost of one step of a run group, in cells: its four launches cost about as much
// as advancing this many cells.
constexpr double TICK_OVERHEAD_CELLS = 2e5;

struct mhd_server {
    size_t budget = 0;
    int max_slots = 0;
    int steps_per_tick = 1;
    MultiRunner mr;
    std::mutex mu;
    std::condition_variable cv;
    std::thread worker;
    std::atomic<bool> running{false};
    std::atomic<bool> stop_req{false};
    std::map<int64_t, std::unique_ptr<Request>> reqs;
    std::deque<int64_t> queue;
    std::vector<int64_t> active;
    int64_t next_id = 1;
    size_t in_use = 0, peak = 0;
    int64_t n_sub = 0, n_adm = 0, n_done = 0, n_fail = 0, ticks = 0;
    std::vector<double> step_lat_ms;   // one sample per (run, step): device clock between its records
    std::vector<double> queue_s, e2e_s;
    double busy_s = 0, cell_substeps = 0;
    std::chrono::steady_clock::time_point t0 = std::chrono::steady_clock::now();
    double first_submit = -1.0, last_done = 0.0;
    std::string worker_error;

    double now() const
    {
        return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }

    void loop();
};

void mhd_server::loop()
{
    bool set_changed = true;
    std::vector<mhd_ctx *> ctxs;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    const bool have_ev = hipEventCreate(&ev0) == hipSuccess && hipEventCreate(&ev1) == hipSuccess;
    while (!stop_req.load()) {
        // admission (FIFO) by footprint and free slots; admitted runs get their device
        // state at the end of the current tick and join from the next tick on
        std::vector<Request *> admit;
        {
            std::unique_lock<std::mutex> lk(mu);
            if (active.empty() && queue.empty()) {
                cv.wait_for(lk, std::chrono::milliseconds(5));
                continue;
            }
            while (!queue.empty() && (int)(active.size() + admit.size()) < max_slots) {
                Request *r = reqs[queue.front()].get();
                if (in_use + r->footprint > budget) break;
                in_use += r->footprint;
                peak = std::max(peak, in_use);
                queue.pop_front();
                admit.push_back(r);
            }
        }
        std::vector<Request *> act;
        {
            std::lock_guard<std::mutex> lk(mu);
            for (int64_t id : active) act.push_back(reqs[id].get());
        }
        // 1. the tick of the active set goes to the device (replayed as a captured graph
        //    while the set and the step counts are unchanged; rebuilt after an admission
        //    or a retirement).  Runs are grouped by size class; the costliest group takes
        //    steps_per_tick steps and every other group as many more as makes its share of
        //    the tick about as long, so small runs are not held to the pace of large ones.
        std::vector<int64_t> kq;
        std::map<mhd_ctx *, int64_t> kof;
        mhd_status st = MHD_OK;
        if (!act.empty()) {
            if (set_changed) {
                ctxs.clear();
                for (Request *r : act) ctxs.push_back(r->ctx);
                if (mr.build(ctxs) != MHD_OK) {
                    worker_error = g_err;
                    break;
                }
                set_changed = false;
            }
            std::map<mhd_ctx *, int64_t> left;
            for (Request *r : act) left[r->ctx] = r->nsteps - r->steps_done;
            std::vector<double> cost(mr.groups.size(), TICK_OVERHEAD_CELLS);
            for (size_t gi = 0; gi < mr.groups.size(); gi++)
                for (mhd_ctx *c : mr.groups[gi].members) cost[gi] += (double)c->ncell;
            const double cmax = *std::max_element(cost.begin(), cost.end());
            kq.resize(mr.groups.size());
            for (size_t gi = 0; gi < mr.groups.size(); gi++) {
                int64_t k = std::llround((double)steps_per_tick * cmax / cost[gi]);
                k = std::max<int64_t>(1, std::min<int64_t>(k, CHUNK));
                for (mhd_ctx *c : mr.groups[gi].members) k = std::min(k, left[c]);
                kq[gi] = k;
                for (mhd_ctx *c : mr.groups[gi].members) kof[c] = k;
            }
            if (have_ev) (void)hipEventRecord(ev0, mr.stream);
            st = mr.run_chunk(kq, true);
            if (have_ev) (void)hipEventRecord(ev1, mr.stream);
        }
        const double ta = now();
        // 2. the end of the tick
        if (st == MHD_OK && !act.empty() && hipStreamSynchronize(mr.stream) != hipSuccess)
            st = fail(MHD_E_DEVICE, "device error in tick");
        const double tb = now();
        if (st != MHD_OK) {
            worker_error = g_err;
            break;
        }
        float tick_ms = (float)((tb - ta) * 1e3);
        if (have_ev && !act.empty()) (void)hipEventElapsedTime(&tick_ms, ev0, ev1);
        // 3. device state of the admitted runs (the seed field is generated in the stream,
        //    ahead of the next tick).  Each run takes the tile it takes alone: the groups
        //    of a tick (one per size class) are launched one after another, so each must
        //    fill the chip by itself (the filled-chip tile of a batch made the served
        //    trace 25 % slower).
        for (size_t i = 0; i < admit.size(); i++) {
            Request *r = admit[i];
            mhd_ctx *c = new mhd_ctx();
            mhd_status st2 = ctx_init(c, &r->p, mr.stream, nullptr, -1);
            if (st2 == MHD_OK) st2 = ctx_init_seed(c, r->seed, r->a_noise);
            if (st2 == MHD_OK) {
                c->fmode = 2;
                c->kf = r->kf;
                c->f0 = r->f0;
                c->sigma = r->sigma;
                c->fseed = r->seed;
                c->in_batch = true;
            }
            std::lock_guard<std::mutex> lk(mu);
            if (st2 != MHD_OK) {
                ctx_release(c);
                delete c;
                r->state = MHD_RUN_FAILED;
                r->t_done = now();
                in_use -= r->footprint;
                n_fail++;
                cv.notify_all();
                continue;
            }
            r->ctx = c;
            r->state = MHD_RUN_ACTIVE;
            r->t_admit = now();
            queue_s.push_back(r->t_admit - r->t_submit);
            active.push_back(r->id);
            n_adm++;
            set_changed = true;
        }
        if (act.empty()) continue;
        // A run whose state went non-finite is evicted at the tick where it shows.  Every
        // record carries the device clock of the moment its step was reduced on the
        // device; the difference between a run's consecutive records is the time that
        // run took per step, measured, wherever the other runs' launches fell.
        std::vector<Request *> finished;
        std::vector<double> lat_new;
        for (Request *r : act) {
            mhd_ctx *c = r->ctx;
            const size_t n0 = c->host_diag.size();
            if (ctx_drain(c) == MHD_OK) {
                for (size_t i = n0; i < c->host_diag.size(); i++) {
                    const double td = c->host_diag[i].t_device;
                    if (r->last_tdev >= 0.0) lat_new.push_back((td - r->last_tdev) * 1e3);
                    r->last_tdev = td;
                }
                if (!c->host_diag.empty() && c->host_diag.back().nonfinite > 0) r->nsteps = 0;
            }
            if (c->host_diag.size() > 4) c->host_diag.erase(c->host_diag.begin(), c->host_diag.end() - 4);
        }
        {
            std::lock_guard<std::mutex> lk(mu);
            ticks++;
            busy_s += tick_ms * 1e-3;
            step_lat_ms.insert(step_lat_ms.end(), lat_new.begin(), lat_new.end());
            for (Request *r : act) {
                const int64_t k = kof[r->ctx];
                cell_substeps += 3.0 * (double)k * (double)r->ctx->ncell;
                r->steps_done += k;
                if (r->steps_done >= r->nsteps) finished.push_back(r);
            }
        }
        for (Request *r : finished) {
            mhd_ctx *c = r->ctx;
            // last diagnostics (also flags a run that went non-finite)
            (void)ctx_drain(c);
            bool bad = r->steps_done < r->nsteps || r->nsteps == 0;
            if (!c->host_diag.empty()) {
                r->em = c->host_diag.back().em;
                r->brms = c->host_diag.back().brms;
                for (const auto &d : c->host_diag) bad = bad || d.nonfinite > 0;
            }
            if (r->retain) {
                r->kept.resize(NF);
                for (int f = 0; f < NF; f++) {
                    r->kept[f].resize(c->ncell * c->p.precision);
                    (void)hipMemcpy(r->kept[f].data(), c->bufs[c->parity][f], r->kept[f].size(), hipMemcpyDeviceToHost);
                }
            }
            ctx_release(c);
            delete c;
            std::lock_guard<std::mutex> lk(mu);
            r->ctx = nullptr;
            r->state = bad ? MHD_RUN_FAILED : MHD_RUN_DONE;
            r->t_done = now();
            last_done = r->t_done;
            e2e_s.push_back(r->t_done - r->t_submit);
            in_use -= r->footprint;
            if (bad) n_fail++; else n_done++;
            active.erase(std::find(active.begin(), active.end(), r->id));
            set_changed = true;
        }
        if (!finished.empty()) cv.notify_all();
    }
    if (ev0) (void)hipEventDestroy(ev0);
    if (ev1) (void)hipEventDestroy(ev1);
    running.store(false);
    cv.notify_all();
}

extern "C" {

// ---------------------------------------------------------------- batch

mhd_status mhd_batch_create(const mhd_params *runs, int32_t n, void *hip_stream, mhd_batch **out)
{
    if (!runs || n <= 0 || !out) return fail(MHD_E_INVALID, "batch: need n > 0 runs and an out pointer");
    *out = nullptr;
    for (int32_t i = 0; i < n; i++) {
        mhd_status st = check_params(&runs[i]);
        if (st != MHD_OK) return fail(st, "run " + std::to_string(i) + ": " + g_err);
    }
    mhd_batch *b = new (std::nothrow) mhd_batch();
    if (!b) return fail(MHD_E_OOM, "host allocation failed");
    // A grid alone takes the tile that fills the chip with its own work-groups (a small
    // tile at 64^3 and below, the ring kernel up to 128^3); in a batch the runs of one
    // precision fill it together.  When their cells come to BATCH_FILL_CELLS or more,
    // every run of that precision takes the filled-chip choice (the z-marching kernel
    // where the grid allows it: 48 FP32 runs of 64^3 and 128^3 make 12 % more
    // run-steps per second with it than with the ring kernel).
    double cells[2] = {0, 0};
    for (int32_t i = 0; i < n; i++)
        cells[runs[i].precision == MHD_FP64] += (double)runs[i].nx * runs[i].ny * runs[i].nz;
    mhd_status st = b->mr.init_stream(hip_stream);
    for (int32_t i = 0; i < n && st == MHD_OK; i++) {
        mhd_ctx *c = new mhd_ctx();
        const bool filled = cells[runs[i].precision == MHD_FP64] >= BATCH_FILL_CELLS;
        st = ctx_init(c, &runs[i], b->mr.stream, nullptr, filled ? default_shape(runs[i], true, true) : -1);
        c->in_batch = true;
        b->runs.push_back(c);
    }
    if (st == MHD_OK) st = b->mr.build(b->runs);
    if (st != MHD_OK) {
        const std::string msg = g_err;
        mhd_batch_destroy(b);
        return fail(st, msg);
    }
    *out = b;
    return MHD_OK;
}

mhd_status mhd_batch_destroy(mhd_batch *b)
{
    if (!b) return MHD_OK;
    b->mr.clear();
    for (mhd_ctx *c : b->runs) {
        ctx_release(c);
        delete c;
    }
    b->mr.destroy_stream();
    delete b;
    return MHD_OK;
}

mhd_status mhd_batch_ctx(mhd_batch *b, int32_t i, mhd_ctx **ctx)
{
    if (!b || !ctx || i < 0 || i >= (int32_t)b->runs.size()) return fail(MHD_E_INVALID, "batch: run index out of range");
    *ctx = b->runs[(size_t)i];
    return MHD_OK;
}

mhd_status mhd_batch_run(mhd_batch *b, int64_t nsteps, int use_graph)
{
    if (!b || nsteps < 0) return fail(MHD_E_INVALID, "batch: bad arguments");
    return b->mr.run(nsteps, use_graph != 0);
}

// ---------------------------------------------------------------- server

mhd_status mhd_server_create(size_t hbm_budget, int32_t max_slots, int32_t steps_per_tick, void *hip_stream,
                             mhd_server **out)
{
    if (!out || max_slots <= 0 || steps_per_tick <= 0 || hbm_budget == 0)
        return fail(MHD_E_INVALID, "server: need budget > 0, slots > 0, steps_per_tick > 0");
    mhd_server *s = new (std::nothrow) mhd_server();
    if (!s) return fail(MHD_E_OOM, "host allocation failed");
    s->budget = hbm_budget;
    s->max_slots = max_slots;
    s->steps_per_tick = steps_per_tick;
    s->mr.split_by_size = true;
    s->mr.capture_on_reuse = true;
    mhd_status st = s->mr.init_stream(hip_stream);
    if (st != MHD_OK) {
        delete s;
        return st;
    }
    *out = s;
    return MHD_OK;
}

mhd_status mhd_server_start(mhd_server *s)
{
    if (!s) return fail(MHD_E_INVALID, "server is NULL");
    if (s->running.load()) return MHD_OK;
    if (s->worker.joinable()) s->worker.join();
    s->stop_req.store(false);
    s->running.store(true);
    s->worker = std::thread([s]() { s->loop(); });
    return MHD_OK;
}

mhd_status mhd_server_submit(mhd_server *s, const mhd_params *p, uint64_t seed, double a_noise, double kf, double f0,
                             double sigma, int64_t nsteps, int32_t retain, int64_t *id)
{
    if (!s || !id) return fail(MHD_E_INVALID, "NULL argument");
    mhd_status st = check_params(p);
    if (st != MHD_OK) return st;
    if (nsteps <= 0) return fail(MHD_E_INVALID, "nsteps must be > 0");
    if (!(kf >= 1.0) || !std::isfinite(f0) || !std::isfinite(sigma) || !std::isfinite(a_noise))
        return fail(MHD_E_INVALID, "bad forcing or noise parameters");
    auto r = std::make_unique<Request>();
    r->p = *p;
    r->seed = seed;
    r->a_noise = a_noise;
    r->kf = kf;
    r->f0 = f0;
    r->sigma = sigma;
    r->nsteps = nsteps;
    r->retain = retain != 0;
    r->footprint = ctx_footprint(*p);
    if (r->footprint > s->budget) return fail(MHD_E_BUSY, "run footprint exceeds the whole HBM budget");
    std::lock_guard<std::mutex> lk(s->mu);
    r->id = s->next_id++;
    r->t_submit = s->now();
    if (s->first_submit < 0) s->first_submit = r->t_submit;
    *id = r->id;
    s->queue.push_back(r->id);
    s->reqs[r->id] = std::move(r);
    s->n_sub++;
    s->cv.notify_all();
    return MHD_OK;
}

mhd_status mhd_server_poll(mhd_server *s, int64_t id, mhd_run_info *info)
{
    if (!s || !info) return fail(MHD_E_INVALID, "NULL argument");
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->reqs.find(id);
    if (it == s->reqs.end()) return fail(MHD_E_NOTFOUND, "unknown run id");
    const Request &r = *it->second;
    info->state = r.state;
    info->precision = r.p.precision;
    info->steps_done = r.steps_done;
    info->steps_total = r.nsteps;
    info->t_submit = r.t_submit;
    info->t_admit = r.t_admit;
    info->t_done = r.t_done;
    info->em = r.em;
    info->brms = r.brms;
    return MHD_OK;
}

mhd_status mhd_server_wait(mhd_server *s, int64_t id, double timeout_s)
{
    if (!s) return fail(MHD_E_INVALID, "server is NULL");
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->reqs.find(id);
    if (it == s->reqs.end()) return fail(MHD_E_NOTFOUND, "unknown run id");
    Request *r = it->second.get();
    const auto deadline = std::chrono::steady_clock::now() + std::chrono::duration<double>(timeout_s);
    while (r->state != MHD_RUN_DONE && r->state != MHD_RUN_FAILED) {
        if (!s->running.load()) {
            std::string why = s->worker_error.empty() ? "server is not running" : s->worker_error;
            return fail(MHD_E_DEVICE, "server stopped: " + why);
        }
        if (s->cv.wait_until(lk, deadline) == std::cv_status::timeout &&
            r->state != MHD_RUN_DONE && r->state != MHD_RUN_FAILED)
            return fail(MHD_E_BUSY, "timed out waiting for the run");
    }
    return MHD_OK;
}

mhd_status mhd_server_get_field(mhd_server *s, int64_t id, int field, void *dst)
{
    if (!s || !dst || field < 0 || field >= NF) return fail(MHD_E_INVALID, "bad arguments");
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->reqs.find(id);
    if (it == s->reqs.end()) return fail(MHD_E_NOTFOUND, "unknown run id");
    const Request &r = *it->second;
    if (r.state != MHD_RUN_DONE && r.state != MHD_RUN_FAILED) return fail(MHD_E_BUSY, "run has not finished");
    if (r.kept.empty()) return fail(MHD_E_INVALID, "run was not submitted with retain");
    std::memcpy(dst, r.kept[(size_t)field].data(), r.kept[(size_t)field].size());
    return MHD_OK;
}

mhd_status mhd_server_release(mhd_server *s, int64_t id)
{
    if (!s) return fail(MHD_E_INVALID, "server is NULL");
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->reqs.find(id);
    if (it == s->reqs.end()) return fail(MHD_E_NOTFOUND, "unknown run id");
    if (it->second->state != MHD_RUN_DONE && it->second->state != MHD_RUN_FAILED)
        return fail(MHD_E_BUSY, "run has not finished");
    s->reqs.erase(it);
    return MHD_OK;
}

mhd_status mhd_server_stats_get(mhd_server *s, mhd_server_stats *st)
{
    if (!s || !st) return fail(MHD_E_INVALID, "NULL argument");
    std::lock_guard<std::mutex> lk(s->mu);
    std::memset(st, 0, sizeof *st);
    st->submitted = s->n_sub;
    st->admitted = s->n_adm;
    st->completed = s->n_done;
    st->failed = s->n_fail;
    st->ticks = s->ticks;
    st->step_samples = (int64_t)s->step_lat_ms.size();
    st->lat_p50_ms = pct(s->step_lat_ms, 0.50);
    st->lat_p90_ms = pct(s->step_lat_ms, 0.90);
    st->lat_p99_ms = pct(s->step_lat_ms, 0.99);
    st->queue_p50_s = pct(s->queue_s, 0.50);
    st->queue_p99_s = pct(s->queue_s, 0.99);
    st->e2e_p50_s = pct(s->e2e_s, 0.50);
    st->e2e_p99_s = pct(s->e2e_s, 0.99);
    st->busy_s = s->busy_s;
    st->wall_s = s->first_submit < 0 ? 0.0 : std::max(0.0, s->last_done - s->first_submit);
    st->cell_substeps = s->cell_substeps;
    st->hbm_in_use = s->in_use;
    st->hbm_peak = s->peak;
    return MHD_OK;
}

mhd_status mhd_server_stop(mhd_server *s)
{
    if (!s) return fail(MHD_E_INVALID, "server is NULL");
    s->stop_req.store(true);
    s->cv.notify_all();
    if (s->worker.joinable()) s->worker.join();
    s->running.store(false);
    return MHD_OK;
}

mhd_status mhd_server_destroy(mhd_server *s)
{
    if (!s) return MHD_OK;
    mhd_server_stop(s);
    for (auto &kv : s->reqs)
        if (kv.second->ctx) {
            ctx_release(kv.second->ctx);
            delete kv.second->ctx;
        }
    s->mr.clear();
    s->mr.destroy_stream();
    delete s;
    return MHD_OK;
}

}  // extern "C"
