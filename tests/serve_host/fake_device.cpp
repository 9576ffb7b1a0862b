// Fake device for the serving loop (em_serve.cpp).  The HIP stand-ins of
// hip/hip_runtime.h run stream operations on one fake device thread, in
// order per stream; the pipeline stages the scheduler calls are replaced by
// host code that does a trivial "mapping" (every pair fraction 1, particle
// a's mass to cell a mod n_cells) and records what the scheduler did: the
// order jobs were admitted in, how many jobs and how many bytes of estimated
// footprint were in flight at once, which threads made device calls, and how
// many device-wide synchronisations (hipFree) ran.  A job whose first cell
// volume is zero fails in its first stage, as malformed geometry would; a job
// of g_log.hang_n particles makes its integration launch hang until
// g_log.release_hang() (a device that stops responding).
#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <functional>
#include <mutex>
#include <random>
#include <thread>
#include <vector>

#include "em_runtime.h"
#include "fake_device.h"

// ---------------------------------------------------------------- fake device
struct FakeOp {
    std::function<void()> fn;
};

struct ihipStream_t {
    std::deque<FakeOp> q;
};

struct ihipEvent_t {
    bool done = true;
};

namespace {
struct FakeDevice {
    std::mutex mu;
    std::condition_variable cv;
    std::vector<ihipStream_t *> streams;
    bool stop = false;
    std::thread thread;
    FakeDevice() : thread([this] { run(); }) {}
    ~FakeDevice()
    {
        {
            std::lock_guard<std::mutex> g(mu);
            stop = true;
        }
        cv.notify_all();
        thread.join();
    }
    bool idle_locked() const
    {
        for (auto *s : streams)
            if (!s->q.empty()) return false;
        return true;
    }
    void run()
    {
        size_t rr = 0;
        std::unique_lock<std::mutex> lk(mu);
        for (;;) {
            cv.wait(lk, [&] { return stop || !idle_locked(); });
            if (stop && idle_locked()) return;
            // the next stream with work, round-robin
            ihipStream_t *s = nullptr;
            for (size_t k = 0; k < streams.size(); k++) {
                ihipStream_t *c = streams[(rr + k) % streams.size()];
                if (!c->q.empty()) {
                    s = c;
                    rr = (rr + k + 1) % streams.size();
                    break;
                }
            }
            FakeOp op = s->q.front();
            lk.unlock();
            op.fn();
            lk.lock();
            s->q.pop_front();
            cv.notify_all();
        }
    }
    void enqueue(ihipStream_t *s, std::function<void()> fn)
    {
        std::lock_guard<std::mutex> g(mu);
        s->q.push_back(FakeOp{std::move(fn)});
        cv.notify_all();
    }
    void wait_idle()
    {
        std::unique_lock<std::mutex> lk(mu);
        cv.wait(lk, [&] { return idle_locked(); });
    }
};

FakeDevice &dev()
{
    static FakeDevice d;
    return d;
}
}  // namespace

hipError_t hipStreamCreateWithFlags(hipStream_t *s, unsigned)
{
    auto *st = new ihipStream_t;
    std::lock_guard<std::mutex> g(dev().mu);
    dev().streams.push_back(st);
    *s = st;
    return hipSuccess;
}

hipError_t hipStreamDestroy(hipStream_t s)
{
    hipStreamSynchronize(s);
    std::lock_guard<std::mutex> g(dev().mu);
    auto &v = dev().streams;
    v.erase(std::remove(v.begin(), v.end(), s), v.end());
    delete s;
    return hipSuccess;
}

hipError_t hipStreamSynchronize(hipStream_t s)
{
    std::unique_lock<std::mutex> lk(dev().mu);
    dev().cv.wait(lk, [&] { return s->q.empty(); });
    return hipSuccess;
}

hipError_t hipStreamQuery(hipStream_t s)
{
    std::lock_guard<std::mutex> g(dev().mu);
    return s->q.empty() ? hipSuccess : hipErrorNotReady;
}

hipError_t hipEventCreateWithFlags(hipEvent_t *e, unsigned)
{
    *e = new ihipEvent_t;
    return hipSuccess;
}

hipError_t hipEventDestroy(hipEvent_t e)
{
    delete e;
    return hipSuccess;
}

hipError_t hipEventRecord(hipEvent_t e, hipStream_t s)
{
    {
        std::lock_guard<std::mutex> g(dev().mu);
        e->done = false;
    }
    dev().enqueue(s, [e] {
        std::lock_guard<std::mutex> g(dev().mu);
        e->done = true;
    });
    return hipSuccess;
}

hipError_t hipEventQuery(hipEvent_t e)
{
    std::lock_guard<std::mutex> g(dev().mu);
    return e->done ? hipSuccess : hipErrorNotReady;
}

hipError_t hipFreeVoid(void *p)
{
    dev().wait_idle();  // the real call synchronises the device
    {
        std::lock_guard<std::mutex> g(em::g_log.mu);
        em::g_log.device_syncs++;
    }
    std::free(p);
    return hipSuccess;
}

hipError_t hipHostFree(void *p) { return hipFreeVoid(p); }

namespace em {

FakeLog g_log;

void FakeLog::release_hang()
{
    {
        std::lock_guard<std::mutex> g(mu);
        hang_released = true;
    }
    hang_cv.notify_all();
    dev().wait_idle();
}

static void note_thread()
{
    std::lock_guard<std::mutex> g(g_log.mu);
    const auto id = std::this_thread::get_id();
    if (std::find(g_log.device_threads.begin(), g_log.device_threads.end(), id) == g_log.device_threads.end())
        g_log.device_threads.push_back(id);
}

Workspace::Workspace(int device) : device_(device), bufs_(S_NUM_SLOTS) {}
Workspace::~Workspace() { release(); }
void Workspace::release()
{
    for (Buf &b : bufs_)
        if (b.p) {
            if (stream_) hipFreeAsync(b.p, stream_);
            else hipFree(b.p);
            held_.fetch_sub(b.cap);
            b.p = nullptr;
            b.cap = 0;
        }
}
void *Workspace::get(int slot, size_t bytes)
{
    Buf &b = bufs_.at(slot);
    if (b.cap < bytes) {
        if (b.p) {
            if (stream_) hipFreeAsync(b.p, stream_);
            else hipFree(b.p);
        }
        held_.fetch_sub(b.cap);
        b.p = std::malloc(bytes);
        b.cap = bytes;
        held_.fetch_add(bytes);
    }
    return b.p;
}
size_t Workspace::bytes_held() const { return held_.load(); }

Ctx::Ctx(const map_config *cfg) : ws(0) { config = *cfg; }
Ctx::~Ctx() {}

bool serving_enabled() { return true; }

IntegrateTune default_tune(int precision)
{
    IntegrateTune t;
    t.persistent = 3;
    t.waves = precision == MAP_FP64 ? 2 : 6;
    return t;
}
IntegrateTune pick_tune(const Ctx &, int precision, int64_t) { return default_tune(precision); }

static thread_local double t_limit_ms = 0.0;
void set_wait_limit_ms(double ms) { t_limit_ms = ms; }
void stream_sync(hipStream_t s)
{
    note_thread();
    const auto t0 = std::chrono::steady_clock::now();
    while (hipStreamQuery(s) != hipSuccess) {
        const double ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
        if (t_limit_ms > 0.0 && ms > t_limit_ms) throw Error{MAP_EDEVICE, std::string(kWaitLimitText)};
        std::this_thread::sleep_for(std::chrono::microseconds(50));
    }
}

static void nap()
{
    static thread_local std::mt19937 rng(std::hash<std::thread::id>()(std::this_thread::get_id()));
    std::this_thread::sleep_for(std::chrono::microseconds(g_log.stage_us + (int)(rng() % 500)));
}

void check_host_args(const map_particles_in *p, const map_cells_in *c)
{
    EM_CHECK(p && c && p->n >= 0 && c->n_cells > 0, MAP_EINVAL, "bad sizes");
}

static void enter(const map_particles_in *p, const map_cells_in *c)
{
    std::lock_guard<std::mutex> g(g_log.mu);
    g_log.order.push_back((int)p->h[0]);
    g_log.live++;
    g_log.max_live = std::max(g_log.max_live, g_log.live);
    g_log.bytes += job_footprint(p, c);
    g_log.max_bytes = std::max(g_log.max_bytes, g_log.bytes);
}

static void leave(size_t fp)
{
    std::lock_guard<std::mutex> g(g_log.mu);
    g_log.live--;
    g_log.bytes -= fp;
}

void stage_pairs(Ctx &, Workspace &ws, const map_particles_in *p, const map_cells_in *c, int precision, JobState &js,
                 hipStream_t s)
{
    note_thread();
    enter(p, c);
    const size_t fp = job_footprint(p, c);
    nap();
    if (c->cell_volume && c->cell_volume[0] == 0.0) {
        leave(fp);
        throw Error{MAP_EGEOM, "cell volume must be positive"};
    }
    js.precision = precision;
    js.in.n = p->n;
    js.in.n_cells = c->n_cells;
    double *m = ws.get<double>(S_M, (size_t)p->n + 1);
    std::memcpy(m, p->m, sizeof(double) * (size_t)p->n);
    js.in.m = m;
    // stand-ins for the device buffers the integration reads (checked by the scheduler)
    js.in.xyz = js.in.h = js.in.plane = m;
    js.in.cfo = js.in.fvo = ws.get<int64_t>(S_CFO, 2);
    js.edges = ws.get<EdgeRec>(S_EDGE, 1);
    js.ps.n_pairs = p->n;
    js.ps.pair_p = js.ps.pair_c = ws.get<uint32_t>(S_PAIR_P, (size_t)p->n + 1);
    js.f = ws.get<double>(S_F, (size_t)p->n + 1);
    js.tile_ctr = ws.get<uint32_t>(S_TILE_CTR, 64);
    js.counters = ws.get<int64_t>(S_COUNTERS, C_NUM);
    js.fix_cap = 16;
    js.fix_items = ws.get<uint64_t>(S_FIX_ITEMS, 16);
    // some device work on the stage stream, waited for by the scheduler
    dev().enqueue(s, [] { std::this_thread::sleep_for(std::chrono::microseconds(100)); });
    std::lock_guard<std::mutex> g(g_log.mu);
    g_log.footprint_of[&js] = fp;
}

void launch_integrate_jobs(const IntJob *h_jobs, const IntJob *d_jobs, int n_jobs, int, const IntegrateTune &, unsigned *,
                           hipStream_t s)
{
    note_thread();
    int64_t tiles = 0;
    for (int j = 0; j < n_jobs; j++) {
        EM_CHECK(h_jobs[j].tile_base == tiles, MAP_EINVAL, "tile bases");
        tiles += (h_jobs[j].np + 63) / 64;
    }
    bool hang = false;
    {
        std::lock_guard<std::mutex> g(g_log.mu);
        g_log.batches++;
        g_log.max_batch = std::max(g_log.max_batch, n_jobs);
        for (int j = 0; j < n_jobs; j++) hang = hang || h_jobs[j].np == g_log.hang_n;
    }
    // the kernel reads the device table (copied before the launch on the same stream)
    std::vector<IntJob> table(d_jobs ? d_jobs : h_jobs, (d_jobs ? d_jobs : h_jobs) + n_jobs);
    dev().enqueue(s, [table, hang] {
        if (hang) {
            std::unique_lock<std::mutex> lk(g_log.mu);
            g_log.hang_cv.wait(lk, [] { return g_log.hang_released; });
        }
        nap();
        for (const IntJob &J : table)
            for (int64_t k = 0; k < J.np; k++) J.f[k] = 1.0;
    });
}

int64_t stage_finish(Ctx &, Workspace &, JobState &js, const map_out *out, hipStream_t s, map_stats *st)
{
    note_thread();
    nap();
    stream_sync(s);
    const int64_t nc = js.in.n_cells;
    std::vector<double> M((size_t)nc, 0.0);
    for (int64_t a = 0; a < js.in.n; a++) M[(size_t)(a % nc)] += js.in.m[a] * js.f[a];
    if (out->cell_mass) std::memcpy(out->cell_mass, M.data(), sizeof(double) * (size_t)nc);
    std::memset(st, 0, sizeof(*st));
    st->n_pairs = js.ps.n_pairs;
    size_t fp = 0;
    {
        std::lock_guard<std::mutex> g(g_log.mu);
        fp = g_log.footprint_of[&js];
        g_log.footprint_of.erase(&js);
    }
    leave(fp);
    return 0;
}

}  // namespace em
