// Fake device for the serving loop (em_serve.cpp): the pipeline stages it
// calls are replaced by host code that does a trivial "mapping" (every pair
// fraction 1, particle a's mass to cell a mod n_cells) and records what the
// scheduler did: the order jobs were admitted in, how many jobs and how many
// bytes of estimated footprint were in flight at once.  A job whose first cell
// volume is zero fails in its first stage, as malformed geometry would.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <mutex>
#include <random>
#include <thread>
#include <vector>

#include "em_runtime.h"
#include "fake_device.h"

namespace em {

FakeLog g_log;

Workspace::Workspace(int device) : device_(device), bufs_(S_NUM_SLOTS) {}
Workspace::~Workspace() { release(); }
void Workspace::release()
{
    for (Buf &b : bufs_)
        if (b.p) {
            std::free(b.p);
            held_.fetch_sub(b.cap);
            b.p = nullptr;
            b.cap = 0;
        }
}
void *Workspace::get(int slot, size_t bytes)
{
    Buf &b = bufs_.at(slot);
    if (b.cap < bytes) {
        std::free(b.p);
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
                 hipStream_t)
{
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
    js.ps.n_pairs = p->n;
    js.f = ws.get<double>(S_F, (size_t)p->n + 1);
    js.tile_ctr = ws.get<uint32_t>(S_TILE_CTR, 64);
    js.counters = ws.get<int64_t>(S_COUNTERS, C_NUM);
    js.fix_cap = 16;
    js.fix_items = ws.get<uint64_t>(S_FIX_ITEMS, 16);
    std::lock_guard<std::mutex> g(g_log.mu);
    g_log.footprint_of[&js] = fp;
}

void launch_integrate_batch(const BatchJob *jobs, int n_jobs, int64_t, int, unsigned *, hipStream_t)
{
    {
        std::lock_guard<std::mutex> g(g_log.mu);
        g_log.batches++;
        g_log.max_batch = std::max(g_log.max_batch, n_jobs);
    }
    nap();
    for (int j = 0; j < n_jobs; j++)
        for (int64_t k = 0; k < jobs[j].np; k++) jobs[j].f[k] = 1.0;
}

int64_t stage_finish(Ctx &, Workspace &, JobState &js, const map_out *out, hipStream_t, map_stats *st)
{
    nap();
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
