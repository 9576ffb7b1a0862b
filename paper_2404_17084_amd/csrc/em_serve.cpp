// Serving loop: continuous batching of mapping jobs on one device.
//
// One scheduler thread per context makes every device call of the served
// path; map_submit only validates and copies host inputs, map_poll only waits
// on the server's condition variable.  The thread works on two streams of its
// own: the stage stream (inputs, validation, geometry tables and pair set of
// a job; after its integration: fixups, normalisation, reductions, outputs)
// and the batch stream (integration launches).
//
// Jobs are admitted in submission order while a slot is free and the job's
// footprint estimate fits the device-memory budget (the budget bounds the
// estimated footprint of the jobs in flight); a slot keeps its grow-only
// buffers from one job to the next (the memory held is at most the number of
// slots times the largest job's buffers), taken from the device's memory pool
// in stream order, so that a slot that grows does not synchronise the device.  The scheduler works in rounds: it stages every admitted job
// (pair sets), makes one persistent launch of the task-batch kernel over all
// of them (one launch per precision, over a table of the jobs), stages the
// jobs admitted meanwhile while that launch runs, and when it is done
// finishes its jobs (fixups, reductions, outputs) before the next launch.
// Jobs that arrive while others integrate thus join the next launch; the
// persistent kernel holds every compute unit, so the jobs of one launch
// share the device tile by tile instead of queueing behind each other.  The
// kernel computes each pair the same way whatever the table holds, so a
// job's results are bitwise those of a synchronous map_particles call with
// the same launch shape.
//
// Every wait is bounded by the context's job time limit: the stage functions'
// stream waits (thread-local wait limit), the launch completion (polled), the
// drain at shutdown and map_poll.  A launch or stage wait that runs out
// marks the server failed: its jobs and every later job fail with
// MAP_EDEVICE, and the scheduler stops touching the device.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstdio>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <vector>

#include "em_internal.h"
#include "em_runtime.h"

namespace em {

using Clock = std::chrono::steady_clock;

enum Phase { P_QUEUED, P_ADMITTED, P_STAGED, P_INTEGRATING, P_FINISHED };

struct ServeSlot;

struct Job {
    uint64_t id = 0;
    int precision = MAP_FP64;
    int state = MAP_JOB_PENDING;  // as reported by map_poll
    int phase = P_QUEUED;
    int code = MAP_OK;
    std::string msg;
    // library-owned copies of host inputs (device inputs are borrowed)
    std::vector<double> xyz, m, h, plane, verts, vol;
    std::vector<int64_t> cfo, fvo;
    std::vector<int32_t> fv;
    map_particles_in pin{};
    map_cells_in cin{};
    map_out out{};
    map_stats *user_stats = nullptr;
    size_t footprint = 0;
    Clock::time_point t_submit, t_admit, t_done;
    ServeSlot *slot = nullptr;
    JobState js;
};

struct ServeSlot {
    explicit ServeSlot(int device) : ws(device) {}
    Workspace ws;
    Job *job = nullptr;
};

struct Server {
    Ctx *C = nullptr;
    std::mutex mu;
    std::condition_variable cv;  // submissions, finished jobs, stop requests, scheduler exit
    std::deque<Job *> queue;     // submitted, not yet admitted
    std::vector<Job *> admitted; // admitted, in admission order (until finished)
    std::map<uint64_t, std::unique_ptr<Job>> jobs;
    std::vector<std::unique_ptr<ServeSlot>> slots;
    size_t budget = 0, in_use = 0, max_queue = 1024;
    uint64_t next_id = 1;
    bool stopping = false, exited = false, failed = false;
    std::string fail_msg;
    double limit_ms = 120000.0;
    bool trace = false;
    IntegrateTune tune[2];
    Clock::time_point t0;
    std::thread thread;
    // scheduler-thread state
    hipStream_t sstream = nullptr, bstream = nullptr;
    hipEvent_t bevent = nullptr;
    IntJob *d_table = nullptr;  // device job tables, one region of max_jobs entries per precision
    IntJob *h_table = nullptr;  // pinned host copies (rewritten only while no launch is in flight)
    unsigned *d_ctr = nullptr;  // launch counters, 32 per precision
    int table_cap = 0;
    std::vector<Job *> batch;   // jobs of the launch in flight
    Clock::time_point batch_t0;
};

static double ms_since(const Server &S, Clock::time_point t)
{
    return std::chrono::duration<double, std::milli>(t - S.t0).count();
}

static void trace(Server &S, const Job *j, const char *what, const std::string &extra = std::string())
{
    if (!S.trace) return;
    std::fprintf(stderr, "[exactmap serve] %10.3f ms  job %llu  %s%s%s\n", ms_since(S, Clock::now()),
                 (unsigned long long)(j ? j->id : 0), what, extra.empty() ? "" : "  ", extra.c_str());
    std::fflush(stderr);
}

// Footprint estimate of a job on the device: inputs, geometry tables and the
// pair-proportional buffers (about 64 bytes per pair, ~140 pairs per particle
// for smoothing lengths with ~58 neighbours).
size_t job_footprint(const map_particles_in *p, const map_cells_in *c)
{
    const double pairs = 140.0 * (double)p->n + 64.0;
    double b = 40.0 * p->n + 16.0 * c->n_cells + 48.0 * c->n_faces + 100.0 * c->n_face_verts + 24.0 * c->n_verts +
               120.0 * c->n_cells + 64.0 * pairs + (1 << 22);
    return (size_t)b;
}

template <typename T>
static const T *copy_in(std::vector<T> &dst, const T *src, int64_t count, int mem_kind)
{
    if (mem_kind == MAP_MEM_DEVICE) return src;  // borrowed until the job finishes
    dst.resize(count > 0 ? (size_t)count : 0);
    if (count > 0) std::memcpy(dst.data(), src, sizeof(T) * (size_t)count);
    return dst.data();
}

// ---------------------------------------------------------------- under the server lock
static void finish_locked(Server &S, Job *j, int code, const std::string &msg)
{
    j->code = code;
    j->msg = msg;
    j->t_done = Clock::now();
    if (j->user_stats) {
        if (code != MAP_OK) std::memset(j->user_stats, 0, sizeof(map_stats));
        const Clock::time_point adm = j->phase == P_QUEUED ? j->t_done : j->t_admit;
        j->user_stats->ms_queue = std::chrono::duration<double, std::milli>(adm - j->t_submit).count();
        j->user_stats->ms_latency = std::chrono::duration<double, std::milli>(j->t_done - j->t_submit).count();
    }
    if (j->phase != P_QUEUED) {
        S.in_use -= j->footprint;
        if (j->slot) j->slot->job = nullptr;
        j->slot = nullptr;
        S.admitted.erase(std::remove(S.admitted.begin(), S.admitted.end(), j), S.admitted.end());
    }
    j->phase = P_FINISHED;
    j->state = code == MAP_OK ? MAP_JOB_DONE : MAP_JOB_FAILED;
    trace(S, j, code == MAP_OK ? "finished" : "failed", code == MAP_OK ? std::string() : msg);
    S.cv.notify_all();
}

static void admit_locked(Server &S)
{
    if (S.failed) return;
    while (!S.queue.empty()) {
        Job *j = S.queue.front();
        ServeSlot *free_slot = nullptr;
        for (auto &sl : S.slots)
            if (!sl->job) {
                free_slot = sl.get();
                break;
            }
        if (!free_slot || S.in_use + j->footprint > S.budget) break;
        S.queue.pop_front();
        S.in_use += j->footprint;
        j->phase = P_ADMITTED;
        j->state = MAP_JOB_RUNNING;
        j->t_admit = Clock::now();
        j->slot = free_slot;
        free_slot->job = j;
        S.admitted.push_back(j);
        trace(S, j, "admitted", std::to_string(j->footprint) + " bytes estimated");
    }
}

// The device can no longer be trusted: fail everything and stop scheduling.
static void fail_server_locked(Server &S, const std::string &why)
{
    if (!S.failed) {
        S.failed = true;
        S.fail_msg = why;
        std::fprintf(stderr, "[exactmap serve] serving stopped: %s\n", why.c_str());
        std::fflush(stderr);
    }
    std::vector<Job *> all(S.admitted.begin(), S.admitted.end());
    for (Job *j : S.queue) all.push_back(j);
    S.queue.clear();
    for (Job *j : all) finish_locked(S, j, MAP_EDEVICE, "served mapping stopped: " + why);
    S.batch.clear();
}

// ---------------------------------------------------------------- scheduler thread
template <typename F>
static int guarded(F &&fn, std::string &msg)
{
    try {
        fn();
        return MAP_OK;
    } catch (const Error &e) {
        msg = e.msg;
        return e.code;
    } catch (const std::bad_alloc &) {
        msg = "host allocation failed";
        return MAP_ENOMEM;
    } catch (const std::exception &e) {
        msg = e.what();
        return MAP_EDEVICE;
    }
}

static bool is_wait_failure(int code, const std::string &msg)
{
    return code == MAP_EDEVICE && msg.find(kWaitLimitText) != std::string::npos;
}

static void stage_job(Server &S, Job *j)
{
    std::string msg;
    const int code = guarded(
        [&] {
            stage_pairs(*S.C, j->slot->ws, &j->pin, &j->cin, j->precision, j->js, S.sstream);
            stream_sync(S.sstream);
        },
        msg);
    std::unique_lock<std::mutex> lk(S.mu);
    if (j->phase != P_ADMITTED) return;  // failed meanwhile
    if (code != MAP_OK) {
        if (is_wait_failure(code, msg)) fail_server_locked(S, msg);
        else finish_locked(S, j, code, msg);
        return;
    }
    j->phase = P_STAGED;
    trace(S, j, "staged", std::to_string(j->js.ps.n_pairs) + " pairs");
}

static void finish_job(Server &S, Job *j)
{
    std::string msg;
    map_stats st;
    std::memset(&st, 0, sizeof(st));
    const int code = guarded([&] { stage_finish(*S.C, j->slot->ws, j->js, &j->out, S.sstream, &st); }, msg);
    std::unique_lock<std::mutex> lk(S.mu);
    if (j->phase == P_FINISHED) return;
    if (code == MAP_OK && j->user_stats) *j->user_stats = st;
    if (is_wait_failure(code, msg)) {
        fail_server_locked(S, msg);
        return;
    }
    finish_locked(S, j, code, msg);
    // the slot keeps its buffers for its next job: mapping them anew for
    // every job (from the kernel-mode GPU driver, gigabytes for the largest jobs) costs more
    // than the jobs' own stages
}

// One integration launch per precision over every staged job; returns
// whether a launch was made.
static bool launch_batch(Server &S)
{
    std::vector<Job *> staged;
    {
        std::lock_guard<std::mutex> lk(S.mu);
        if (S.failed) return false;
        for (Job *j : S.admitted)
            if (j->phase == P_STAGED) staged.push_back(j);
    }
    if (staged.empty()) return false;
    std::vector<Job *> launched, empty_jobs;
    std::vector<std::pair<Job *, std::string>> bad;
    std::string msg;
    const int code = guarded(
        [&] {
            for (int prec : {MAP_FP64, MAP_MIXED}) {
                IntJob *ht = S.h_table + (size_t)prec * S.table_cap;
                std::vector<Job *> members;
                int64_t tiles = 0;
                int n = 0;
                for (Job *j : staged) {
                    if (j->precision != prec) continue;
                    const JobState &js = j->js;
                    if (js.ps.n_pairs == 0) {
                        empty_jobs.push_back(j);
                        continue;
                    }
                    // host checks of the entry before the kernel reads it
                    const char *why = nullptr;
                    if (!js.ps.pair_p || !js.ps.pair_c || !js.f || !js.edges || !js.in.xyz || !js.in.h || !js.in.cfo ||
                        !js.in.fvo || !js.in.plane || !js.counters || !js.tile_ctr || !js.fix_items ||
                        (prec == MAP_MIXED && !js.err))
                        why = "a device buffer of the job is missing";
                    else if (js.ps.n_pairs >= (int64_t)UINT32_MAX)
                        why = "pair count out of range";
                    else if (js.fix_cap <= 0)
                        why = "fixup list capacity is zero";
                    else if (n >= S.table_cap)
                        why = "more jobs than table entries";
                    if (why) {
                        bad.emplace_back(j, why);
                        continue;
                    }
                    IntJob &e = ht[n++];
                    e = IntJob();
                    e.np = js.ps.n_pairs;
                    e.tile_base = tiles;
                    e.pair_p = js.ps.pair_p;
                    e.pair_c = js.ps.pair_c;
                    e.xyz = js.in.xyz;
                    e.h = js.in.h;
                    e.cfo = js.in.cfo;
                    e.fvo = js.in.fvo;
                    e.plane = js.in.plane;
                    e.edges = js.edges;
                    e.f = js.f;
                    e.err = js.err;
                    e.counters = reinterpret_cast<unsigned long long *>(js.counters);
                    e.fix_count = js.tile_ctr + 1;
                    e.fix_items = js.fix_items;
                    e.fix_cap = (unsigned)std::min<int64_t>(js.fix_cap, 0xffffffffLL);
                    tiles += (e.np + 63) / 64;
                    members.push_back(j);
                }
                if (n == 0) continue;
                IntJob *dt = S.d_table + (size_t)prec * S.table_cap;
                EM_HIP(hipMemcpyAsync(dt, ht, sizeof(IntJob) * (size_t)n, hipMemcpyHostToDevice, S.bstream));
                launch_integrate_jobs(ht, dt, n, prec, S.tune[prec], S.d_ctr + 32 * prec, S.bstream);
                launched.insert(launched.end(), members.begin(), members.end());
            }
            if (!launched.empty()) EM_HIP(hipEventRecord(S.bevent, S.bstream));
        },
        msg);
    std::unique_lock<std::mutex> lk(S.mu);
    for (auto &b : bad)
        if (b.first->phase == P_STAGED) finish_locked(S, b.first, MAP_EDEVICE, std::string("integration table: ") + b.second);
    if (code != MAP_OK) {
        // nothing of this batch can be trusted to have run
        fail_server_locked(S, "integration launch failed: " + msg);
        return true;
    }
    for (Job *j : empty_jobs)
        if (j->phase == P_STAGED) j->phase = P_INTEGRATING;  // nothing to integrate: finished with the batch
    for (Job *j : launched) j->phase = P_INTEGRATING;
    S.batch = launched;
    S.batch.insert(S.batch.end(), empty_jobs.begin(), empty_jobs.end());
    S.batch_t0 = Clock::now();
    for (Job *j : launched) trace(S, j, "integration launched", std::to_string(launched.size()) + " jobs in the launch");
    return true;  // (with only jobs without pairs no launch was made: they finish at once)
}

// Completion of the launch in flight: 1 done, 0 still running, -1 failed.
static int batch_state(Server &S)
{
    bool has_launch = false;
    for (Job *j : S.batch)
        if (j->js.ps.n_pairs > 0) has_launch = true;
    if (!has_launch) return 1;
    const hipError_t e = hipEventQuery(S.bevent);
    if (e == hipSuccess) return 1;
    (void)hipGetLastError();  // a not-ready query is no error of the next call
    if (e != hipErrorNotReady) {
        std::lock_guard<std::mutex> lk(S.mu);
        fail_server_locked(S, std::string("integration launch failed: ") + hipGetErrorString(e));
        return -1;
    }
    const double waited = std::chrono::duration<double, std::milli>(Clock::now() - S.batch_t0).count();
    if (waited > S.limit_ms) {
        std::lock_guard<std::mutex> lk(S.mu);
        fail_server_locked(S, "an integration launch did not complete within " + std::to_string((long long)S.limit_ms) +
                                  " ms");
        return -1;
    }
    return 0;
}

static void serve_loop(Server *Sp)
{
    Server &S = *Sp;
    set_wait_limit_ms(S.limit_ms);
    (void)hipSetDevice(S.C->device);
    for (;;) {
        std::vector<Job *> to_stage;
        {
            std::unique_lock<std::mutex> lk(S.mu);
            admit_locked(S);
            if (S.failed) {
                // nothing is run after a failure (submissions are refused); wait for the stop request
                if (S.stopping) break;
                S.cv.wait_for(lk, std::chrono::milliseconds(20));
                continue;
            }
            if (S.stopping && S.queue.empty() && S.admitted.empty()) break;
            for (Job *j : S.admitted)
                if (j->phase == P_ADMITTED) to_stage.push_back(j);
        }
        bool progress = false;
        // 1. the launch in flight: when it is done, its jobs are finished
        //    (fixups, reductions, outputs) before anything else, so that their
        //    results do not wait behind the next launch, and the slots and
        //    budget they free are used by the next round of admissions
        if (!S.batch.empty()) {
            const int st = batch_state(S);
            if (st < 0) continue;
            if (st == 1) {
                std::vector<Job *> done;
                done.swap(S.batch);
                for (Job *j : done) trace(S, j, "integration done");
                for (Job *j : done) finish_job(S, j);
                continue;
            }
        }
        // 2. every admitted job gets its pair set (while a launch is in flight
        //    the staging kernels fill the compute units its tail frees)
        for (Job *j : to_stage) {
            stage_job(S, j);
            progress = true;
        }
        // 3. one launch over every staged job
        if (S.batch.empty() && launch_batch(S)) progress = true;
        if (!progress) {
            std::unique_lock<std::mutex> lk(S.mu);
            if (!S.batch.empty()) {
                S.cv.wait_for(lk, std::chrono::microseconds(50));
            } else {
                S.cv.wait_for(lk, std::chrono::milliseconds(20), [&] {
                    if (S.stopping || S.failed) return true;
                    for (Job *j : S.admitted)
                        if (j->phase == P_ADMITTED || j->phase == P_STAGED) return true;
                    return !S.queue.empty() && std::any_of(S.slots.begin(), S.slots.end(),
                                                           [](const std::unique_ptr<ServeSlot> &s) { return !s->job; });
                });
            }
        }
    }
    std::lock_guard<std::mutex> lk(S.mu);
    S.exited = true;
    S.cv.notify_all();
}

static Server &server_of(Ctx &C)
{
    if (C.server) return *C.server;
    auto S = std::make_unique<Server>();
    S->C = &C;
    S->t0 = Clock::now();
    size_t free_b = 0, total_b = 0;
    EM_HIP(hipMemGetInfo(&free_b, &total_b));
    S->budget = C.config.hbm_budget_bytes ? (size_t)C.config.hbm_budget_bytes : (size_t)(0.8 * (double)free_b);
    S->max_queue = C.config.max_queue > 0 ? (size_t)C.config.max_queue : 1024;
    S->limit_ms = C.config.serve_timeout_ms > 0 ? (double)C.config.serve_timeout_ms : 120000.0;
    S->trace = C.config.serve_trace != 0;
    const int n_slots = C.config.max_jobs > 0 ? C.config.max_jobs : 8;
    for (int prec : {MAP_FP64, MAP_MIXED}) {
        IntegrateTune t = pick_tune(C, prec, 1 << 24);
        if (t.persistent != 3) t = default_tune(prec);
        S->tune[prec] = t;
    }
    S->table_cap = n_slots;
    EM_HIP(hipStreamCreateWithFlags(&S->sstream, hipStreamNonBlocking));
    EM_HIP(hipStreamCreateWithFlags(&S->bstream, hipStreamNonBlocking));
    EM_HIP(hipEventCreateWithFlags(&S->bevent, hipEventDisableTiming));
    EM_HIP(hipMalloc(&S->d_table, 2 * sizeof(IntJob) * (size_t)S->table_cap));
    EM_HIP(hipHostMalloc(&S->h_table, 2 * sizeof(IntJob) * (size_t)S->table_cap, hipHostMallocDefault));
    EM_HIP(hipMalloc(&S->d_ctr, 64 * sizeof(unsigned)));
    for (int i = 0; i < n_slots; i++) {
        S->slots.push_back(std::make_unique<ServeSlot>(C.device));
        S->slots.back()->ws.use_stream(S->sstream);
    }
    {
        // the pool that serves the slots' buffers keeps what it has while the
        // server runs (a trim would hand memory back to the GPU driver at the next
        // stream synchronisation, and the next job would map it again); the
        // jobs in flight are bounded by the budget, so is what it holds, up
        // to fragmentation.  serve_stop trims it.
        hipMemPool_t pool = nullptr;
        if (hipDeviceGetDefaultMemPool(&pool, C.device) == hipSuccess && pool) {
            uint64_t keep = ~uint64_t(0);
            (void)hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &keep);
        }
        (void)hipGetLastError();
    }
    Server *raw = S.release();
    raw->thread = std::thread(serve_loop, raw);
    C.server = raw;
    return *raw;
}

int serve_stop(Ctx &C)
{
    Server *S = C.server;
    if (!S) return MAP_OK;
    bool exited = false;
    {
        // drain: queued and admitted jobs complete, then the scheduler exits
        std::unique_lock<std::mutex> lk(S->mu);
        S->stopping = true;
        S->cv.notify_all();
        const auto limit = std::chrono::milliseconds((long long)(2.0 * S->limit_ms) + 5000);
        exited = S->cv.wait_for(lk, limit, [&] { return S->exited; });
    }
    if (!exited) {
        // the scheduler is stuck in a device call: leave it (and the context) alone rather than hang
        std::fprintf(stderr, "[exactmap serve] the serving loop did not stop; its resources are left in place\n");
        std::fflush(stderr);
        S->thread.detach();
        return MAP_EDEVICE;
    }
    S->thread.join();
    (void)hipSetDevice(C.device);
    const bool failed = S->failed;
    if (!failed) {
        for (auto &sl : S->slots) sl->ws.release();
        if (S->sstream) (void)hipStreamSynchronize(S->sstream);
        if (S->bstream) (void)hipStreamSynchronize(S->bstream);
        // the pool's cached memory back to the GPU driver, and its default threshold back
        hipMemPool_t pool = nullptr;
        if (hipDeviceGetDefaultMemPool(&pool, C.device) == hipSuccess && pool) {
            (void)hipMemPoolTrimTo(pool, 0);
            uint64_t keep = 0;
            (void)hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &keep);
        }
        (void)hipGetLastError();
        if (S->d_table) (void)hipFree(S->d_table);
        if (S->d_ctr) (void)hipFree(S->d_ctr);
        if (S->h_table) (void)hipHostFree(S->h_table);
        if (S->bevent) (void)hipEventDestroy(S->bevent);
        if (S->sstream) (void)hipStreamDestroy(S->sstream);
        if (S->bstream) (void)hipStreamDestroy(S->bstream);
        delete S;
    }
    // a failed server keeps its device resources: work of it may still be on the device
    C.server = nullptr;
    return failed ? MAP_EDEVICE : MAP_OK;
}

}  // namespace em

using namespace em;

extern "C" int map_submit(map_ctx *h, const map_particles_in *p, const map_cells_in *c, map_out *out,
                          uint64_t *job_id)
{
    if (!h) return MAP_EINVAL;
    Ctx *C = reinterpret_cast<Ctx *>(h);
    std::lock_guard<std::mutex> guard(C->mu);
    try {
        EM_CHECK(serving_enabled(), MAP_ENOTSUP, "served mapping is not available in this build");
        EM_CHECK(C->precision == MAP_FP64 || C->precision == MAP_MIXED, MAP_EINVAL,
                 "served mapping runs at MAP_FP64 or MAP_MIXED");
        EM_CHECK(out && job_id, MAP_EINVAL, "null output descriptor or job id");
        EM_CHECK(out->mem_kind == MAP_MEM_HOST || out->mem_kind == MAP_MEM_DEVICE, MAP_EINVAL, "bad output mem_kind");
        check_host_args(p, c);
        auto j = std::make_unique<Job>();
        j->precision = C->precision;
        j->t_submit = Clock::now();
        j->pin = *p;
        j->pin.xyz = copy_in(j->xyz, p->xyz, 3 * p->n, p->mem_kind);
        j->pin.m = copy_in(j->m, p->m, p->n, p->mem_kind);
        j->pin.h = copy_in(j->h, p->h, p->n, p->mem_kind);
        j->cin = *c;
        j->cin.cell_face_off = copy_in(j->cfo, c->cell_face_off, c->n_cells + 1, c->mem_kind);
        j->cin.face_vert_off = copy_in(j->fvo, c->face_vert_off, c->n_faces + 1, c->mem_kind);
        j->cin.face_vert = copy_in(j->fv, c->face_vert, c->n_face_verts, c->mem_kind);
        j->cin.face_plane = copy_in(j->plane, c->face_plane, 4 * c->n_faces, c->mem_kind);
        j->cin.verts = copy_in(j->verts, c->verts, 3 * c->n_verts, c->mem_kind);
        j->cin.cell_volume = c->cell_volume ? copy_in(j->vol, c->cell_volume, c->n_cells, c->mem_kind) : nullptr;
        j->out = *out;
        j->user_stats = out->stats;
        j->out.stats = nullptr;
        j->footprint = job_footprint(&j->pin, &j->cin);
        Server &S = server_of(*C);
        std::lock_guard<std::mutex> lk(S.mu);
        EM_CHECK(!S.failed, MAP_EDEVICE, "served mapping stopped: " + S.fail_msg);
        EM_CHECK(!S.stopping, MAP_EBUSY, "the serving loop is shutting down");
        EM_CHECK(j->footprint <= S.budget, MAP_ENOMEM,
                 "job footprint " + std::to_string(j->footprint) + " bytes exceeds the device-memory budget");
        EM_CHECK(S.queue.size() < S.max_queue, MAP_EBUSY, "serving queue is full");
        j->id = S.next_id++;
        *job_id = j->id;
        Job *raw = j.get();
        S.jobs[j->id] = std::move(j);
        S.queue.push_back(raw);
        trace(S, raw, "submitted", std::to_string(p->n) + " particles, " + std::to_string(c->n_cells) + " cells");
        admit_locked(S);  // bookkeeping only: the scheduler thread stages it
        S.cv.notify_all();
        C->err.clear();
        return MAP_OK;
    } catch (const Error &e) {
        C->err = e.msg;
        return e.code;
    } catch (const std::bad_alloc &) {
        C->err = "host allocation failed";
        return MAP_ENOMEM;
    } catch (const std::exception &e) {
        C->err = e.what();
        return MAP_EDEVICE;
    }
}

extern "C" int map_poll(map_ctx *h, uint64_t job_id, int64_t timeout_us, int *state)
{
    if (!h || !state) return MAP_EINVAL;
    Ctx *C = reinterpret_cast<Ctx *>(h);
    Server *S = nullptr;
    {
        std::lock_guard<std::mutex> guard(C->mu);
        S = C->server;
        if (!S) {
            C->err = "no job with this id";
            return MAP_ENOTFOUND;
        }
    }
    std::unique_lock<std::mutex> lk(S->mu);
    auto it = S->jobs.find(job_id);
    if (it == S->jobs.end()) {
        lk.unlock();  // never hold the server lock while taking the context lock
        std::lock_guard<std::mutex> guard(C->mu);
        C->err = "no job with this id";
        return MAP_ENOTFOUND;
    }
    Job *j = it->second.get();
    auto finished = [&] { return j->state == MAP_JOB_DONE || j->state == MAP_JOB_FAILED; };
    // "until finished" is bounded too: the scheduler fails a job whose device
    // work outlives the time limit, so a longer wait means the loop itself is stuck
    const int64_t bound_us = (int64_t)(2.0 * S->limit_ms * 1000.0) + 5000000;
    const int64_t wait_us = timeout_us < 0 ? bound_us : timeout_us;
    if (wait_us > 0) S->cv.wait_for(lk, std::chrono::microseconds(wait_us), finished);
    *state = j->state;
    if (!finished()) {
        if (timeout_us < 0) {
            lk.unlock();
            std::lock_guard<std::mutex> guard(C->mu);
            C->err = "the serving loop did not finish the job within its time limit";
            return MAP_EDEVICE;
        }
        return MAP_OK;
    }
    const int code = j->code;
    const std::string msg = j->msg;
    S->jobs.erase(it);
    lk.unlock();
    std::lock_guard<std::mutex> guard(C->mu);
    C->err = msg;
    return code;
}
