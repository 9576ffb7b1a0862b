// Serving loop: admission by device-memory footprint, per-slot pair-set
// building, and continuous batching of the integration of all ready jobs in
// one persistent launch.
//
// Threads: one worker per slot (stage the inputs, build the pair set; after
// the batched integration: fixups, reductions, outputs) and one batcher (one
// batched integration launch per precision over every job ready at that
// moment).  Admission happens under the server lock at submit and whenever a
// job leaves its slot: jobs are taken in submission order while a slot is
// free and the job's footprint estimate fits the budget.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
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

struct Job {
    uint64_t id = 0;
    int precision = MAP_FP64;
    int state = MAP_JOB_PENDING;
    int code = MAP_OK;
    std::string msg;
    // library-owned copies of the inputs
    std::vector<double> xyz, m, h, plane, verts, vol;
    std::vector<int64_t> cfo, fvo;
    std::vector<int32_t> fv;
    map_particles_in pin{};
    map_cells_in cin{};
    map_out out{};
    map_stats *user_stats = nullptr;
    size_t footprint = 0;
    Clock::time_point t_submit, t_admit, t_done;
    JobState js;
    bool integrated = false;
    bool batch_failed = false;
    std::string batch_msg;
};

struct ServeSlot {
    explicit ServeSlot(int device) : ws(device) {}
    Workspace ws;
    hipStream_t stream = nullptr;
    Job *job = nullptr;
    std::thread worker;
};

struct Server {
    Ctx *C = nullptr;
    std::mutex mu;
    std::condition_variable cv;
    std::deque<Job *> queue;
    std::map<uint64_t, std::unique_ptr<Job>> jobs;
    std::vector<std::unique_ptr<ServeSlot>> slots;
    std::vector<Job *> ready;
    size_t budget = 0;
    size_t in_use = 0;
    size_t max_queue = 1024;
    uint64_t next_id = 1;
    bool stopping = false;
    std::thread batcher;
    hipStream_t bstream = nullptr;
    BatchJob *d_table = nullptr;
    std::vector<BatchJob> h_table[2];  // host copies, alive until the launch has read them
    unsigned *d_ctr = nullptr;
    int table_cap = 0;
};

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
static void copy_in(std::vector<T> &dst, const T *src, int64_t count, int mem_kind)
{
    dst.resize(count > 0 ? (size_t)count : 0);
    if (count <= 0) return;
    if (mem_kind == MAP_MEM_DEVICE)
        EM_HIP(hipMemcpy(dst.data(), src, sizeof(T) * count, hipMemcpyDeviceToHost));
    else
        std::memcpy(dst.data(), src, sizeof(T) * count);
}

// under lock
static void try_admit(Server &S)
{
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
        j->state = MAP_JOB_RUNNING;
        j->t_admit = Clock::now();
        free_slot->job = j;
    }
    S.cv.notify_all();
}

static void finish_job(Server &S, Job *j, int code, const std::string &msg)
{
    j->code = code;
    j->msg = msg;
    j->t_done = Clock::now();
    if (j->user_stats) {
        if (code != MAP_OK) std::memset(j->user_stats, 0, sizeof(map_stats));
        j->user_stats->ms_queue = std::chrono::duration<double, std::milli>(j->t_admit - j->t_submit).count();
        j->user_stats->ms_latency = std::chrono::duration<double, std::milli>(j->t_done - j->t_submit).count();
    }
    j->state = code == MAP_OK ? MAP_JOB_DONE : MAP_JOB_FAILED;
    (void)S;
}

static void worker_loop(Server &S, ServeSlot &sl)
{
    (void)hipSetDevice(S.C->device);
    for (;;) {
        Job *j = nullptr;
        {
            std::unique_lock<std::mutex> lk(S.mu);
            S.cv.wait(lk, [&] { return S.stopping || (sl.job && sl.job->state == MAP_JOB_RUNNING && !sl.job->js.f); });
            if (S.stopping) return;
            j = sl.job;
        }
        int code = MAP_OK;
        std::string msg;
        bool staged = false;
        try {
            stage_pairs(*S.C, sl.ws, &j->pin, &j->cin, j->precision, j->js, sl.stream);
            EM_HIP(hipStreamSynchronize(sl.stream));
            staged = true;
        } catch (const Error &e) {
            code = e.code;
            msg = e.msg;
        } catch (const std::exception &e) {
            code = MAP_EDEVICE;
            msg = e.what();
        }
        if (staged) {
            std::unique_lock<std::mutex> lk(S.mu);
            S.ready.push_back(j);
            S.cv.notify_all();
            S.cv.wait(lk, [&] { return S.stopping || j->integrated; });
            if (S.stopping && !j->integrated) return;
            if (j->batch_failed) {
                code = MAP_EDEVICE;
                msg = j->batch_msg;
                staged = false;
            }
        }
        if (staged) {
            try {
                map_stats st;
                stage_finish(*S.C, sl.ws, j->js, &j->out, sl.stream, &st);
                if (j->user_stats) *j->user_stats = st;
            } catch (const Error &e) {
                code = e.code;
                msg = e.msg;
            } catch (const std::exception &e) {
                code = MAP_EDEVICE;
                msg = e.what();
            }
        }
        std::unique_lock<std::mutex> lk(S.mu);
        finish_job(S, j, code, msg);
        S.in_use -= j->footprint;
        sl.job = nullptr;
        // release this slot's device memory when the pool holds more than the budget
        size_t held = 0;
        for (auto &o : S.slots) held += o->ws.bytes_held();
        if (held > S.budget) {
            lk.unlock();
            (void)hipStreamSynchronize(sl.stream);
            sl.ws.release();
            lk.lock();
        }
        try_admit(S);
    }
}

static void batcher_loop(Server &S)
{
    (void)hipSetDevice(S.C->device);
    for (;;) {
        std::vector<Job *> batch;
        {
            std::unique_lock<std::mutex> lk(S.mu);
            S.cv.wait(lk, [&] { return S.stopping || !S.ready.empty(); });
            if (S.stopping) return;
            batch.swap(S.ready);
        }
        std::string err;
        try {
            for (int prec : {MAP_FP64, MAP_MIXED}) {
                std::vector<BatchJob> &table = S.h_table[prec];
                table.clear();
                int64_t tiles = 0;
                for (Job *j : batch) {
                    if (j->precision != prec || j->js.ps.n_pairs == 0) continue;
                    BatchJob b;
                    b.np = j->js.ps.n_pairs;
                    b.tile_base = tiles;
                    b.pair_p = j->js.ps.pair_p;
                    b.pair_c = j->js.ps.pair_c;
                    b.xyz = j->js.in.xyz;
                    b.h = j->js.in.h;
                    b.cfo = j->js.in.cfo;
                    b.fvo = j->js.in.fvo;
                    b.plane = j->js.in.plane;
                    b.edges = j->js.edges;
                    b.f = j->js.f;
                    b.counters = reinterpret_cast<unsigned long long *>(j->js.counters);
                    b.fix_count = j->js.tile_ctr + 1;
                    b.fix_items = j->js.fix_items;
                    b.fix_cap = (unsigned)(j->js.fix_cap > 0xffffffffLL ? 0xffffffffLL : j->js.fix_cap);
                    tiles += (b.np + 63) / 64;
                    table.push_back(b);
                }
                if (table.empty()) continue;
                // one table region per precision: the second launch's copy
                // must not overwrite the entries the first launch reads
                if ((int)table.size() > S.table_cap) {
                    EM_HIP(hipStreamSynchronize(S.bstream));
                    if (S.d_table) EM_HIP(hipFree(S.d_table));
                    S.d_table = nullptr;
                    S.table_cap = std::max<int>(64, (int)table.size());
                    EM_HIP(hipMalloc(&S.d_table, 2 * sizeof(BatchJob) * S.table_cap));
                }
                BatchJob *dt = S.d_table + (size_t)prec * S.table_cap;
                EM_HIP(hipMemcpyAsync(dt, table.data(), sizeof(BatchJob) * table.size(), hipMemcpyHostToDevice,
                                      S.bstream));
                launch_integrate_batch(dt, (int)table.size(), tiles, prec, S.d_ctr + 16 * prec, S.bstream);
            }
            EM_HIP(hipStreamSynchronize(S.bstream));
        } catch (const Error &e) {
            err = e.msg;
        } catch (const std::exception &e) {
            err = e.what();
        }
        std::unique_lock<std::mutex> lk(S.mu);
        for (Job *j : batch) {
            j->integrated = true;
            if (!err.empty()) {
                j->batch_failed = true;
                j->batch_msg = err;
            }
        }
        S.cv.notify_all();
    }
}

static Server &server_of(Ctx &C)
{
    if (C.server) return *C.server;
    auto *S = new Server;
    S->C = &C;
    size_t free_b = 0, total_b = 0;
    EM_HIP(hipMemGetInfo(&free_b, &total_b));
    S->budget = C.config.hbm_budget_bytes ? (size_t)C.config.hbm_budget_bytes : (size_t)(0.8 * (double)free_b);
    S->max_queue = C.config.max_queue > 0 ? (size_t)C.config.max_queue : 1024;
    const int n_slots = C.config.max_jobs > 0 ? C.config.max_jobs : 8;
    EM_HIP(hipStreamCreateWithFlags(&S->bstream, hipStreamNonBlocking));
    EM_HIP(hipMalloc(&S->d_ctr, 256));
    for (int i = 0; i < n_slots; i++) {
        auto sl = std::make_unique<ServeSlot>(C.device);
        EM_HIP(hipStreamCreateWithFlags(&sl->stream, hipStreamNonBlocking));
        S->slots.push_back(std::move(sl));
    }
    for (auto &sl : S->slots) {
        ServeSlot *p = sl.get();
        p->worker = std::thread([S, p] { worker_loop(*S, *p); });
    }
    S->batcher = std::thread([S] { batcher_loop(*S); });
    C.server = S;
    return *S;
}

void serve_stop(Ctx &C)
{
    Server *S = C.server;
    if (!S) return;
    {
        // drain: every queued and admitted job completes, then the threads stop
        std::unique_lock<std::mutex> lk(S->mu);
        S->cv.wait(lk, [&] {
            if (!S->queue.empty()) return false;
            for (auto &sl : S->slots)
                if (sl->job) return false;
            return true;
        });
        S->stopping = true;
        S->cv.notify_all();
    }
    for (auto &sl : S->slots)
        if (sl->worker.joinable()) sl->worker.join();
    if (S->batcher.joinable()) S->batcher.join();
    (void)hipSetDevice(C.device);
    for (auto &sl : S->slots) {
        if (sl->stream) (void)hipStreamSynchronize(sl->stream);
        sl->ws.release();
        if (sl->stream) (void)hipStreamDestroy(sl->stream);
    }
    if (S->bstream) {
        (void)hipStreamSynchronize(S->bstream);
        (void)hipStreamDestroy(S->bstream);
    }
    if (S->d_table) (void)hipFree(S->d_table);
    if (S->d_ctr) (void)hipFree(S->d_ctr);
    delete S;
    C.server = nullptr;
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
        EM_CHECK(serving_enabled(), MAP_ENOTSUP,
                 "served mapping is switched off: a device run of it stopped making progress and the cause is not "
                 "yet found; use map_particles");
        EM_HIP(hipSetDevice(C->device));
        EM_CHECK(C->precision == MAP_FP64 || C->precision == MAP_MIXED, MAP_EINVAL,
                 "served mapping runs at MAP_FP64 or MAP_MIXED");
        EM_CHECK(out && job_id, MAP_EINVAL, "null output descriptor or job id");
        EM_CHECK(out->mem_kind == MAP_MEM_HOST || out->mem_kind == MAP_MEM_DEVICE, MAP_EINVAL, "bad output mem_kind");
        EM_CHECK(p && c, MAP_EINVAL, "null particle or cell descriptor");
        auto j = std::make_unique<Job>();
        j->precision = C->precision;
        j->t_submit = Clock::now();
        // library-owned host copies (device inputs are copied back to the host)
        copy_in(j->xyz, p->xyz, 3 * p->n, p->mem_kind);
        copy_in(j->m, p->m, p->n, p->mem_kind);
        copy_in(j->h, p->h, p->n, p->mem_kind);
        copy_in(j->cfo, c->cell_face_off, c->n_cells + 1, c->mem_kind);
        copy_in(j->fvo, c->face_vert_off, c->n_faces + 1, c->mem_kind);
        copy_in(j->fv, c->face_vert, c->n_face_verts, c->mem_kind);
        copy_in(j->plane, c->face_plane, 4 * c->n_faces, c->mem_kind);
        copy_in(j->verts, c->verts, 3 * c->n_verts, c->mem_kind);
        if (c->cell_volume) copy_in(j->vol, c->cell_volume, c->n_cells, c->mem_kind);
        j->pin = *p;
        j->pin.xyz = j->xyz.data();
        j->pin.m = j->m.data();
        j->pin.h = j->h.data();
        j->pin.mem_kind = MAP_MEM_HOST;
        j->cin = *c;
        j->cin.cell_face_off = j->cfo.data();
        j->cin.face_vert_off = j->fvo.data();
        j->cin.face_vert = j->fv.data();
        j->cin.face_plane = j->plane.data();
        j->cin.verts = j->verts.data();
        j->cin.cell_volume = c->cell_volume ? j->vol.data() : nullptr;
        j->cin.mem_kind = MAP_MEM_HOST;
        check_host_args(&j->pin, &j->cin);
        j->out = *out;
        j->user_stats = out->stats;
        j->out.stats = nullptr;
        j->footprint = job_footprint(&j->pin, &j->cin);
        Server &S = server_of(*C);
        std::lock_guard<std::mutex> lk(S.mu);
        EM_CHECK(j->footprint <= S.budget, MAP_ENOMEM,
                 "job footprint " + std::to_string(j->footprint) + " bytes exceeds the device-memory budget");
        EM_CHECK(S.queue.size() < S.max_queue, MAP_EBUSY, "serving queue is full");
        j->id = S.next_id++;
        *job_id = j->id;
        Job *raw = j.get();
        S.jobs[j->id] = std::move(j);
        S.queue.push_back(raw);
        try_admit(S);
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
    if (timeout_us < 0)
        S->cv.wait(lk, finished);
    else if (timeout_us > 0)
        S->cv.wait_for(lk, std::chrono::microseconds(timeout_us), finished);
    *state = j->state;
    if (!finished()) return MAP_OK;
    const int code = j->code;
    const std::string msg = j->msg;
    S->jobs.erase(it);
    lk.unlock();
    std::lock_guard<std::mutex> guard(C->mu);
    C->err = msg;
    return code;
}
