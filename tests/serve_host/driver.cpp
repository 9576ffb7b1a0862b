// Scheduler scenarios of the serving loop on the fake device.  Each prints
// "ok <name>" or "FAIL <name>: <what>" and the program exits non-zero on the
// first failure.
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <memory>
#include <random>
#include <vector>

#include "em_runtime.h"
#include "fake_device.h"

using namespace em;

extern "C" int map_submit(map_ctx *, const map_particles_in *, const map_cells_in *, map_out *, uint64_t *);
extern "C" int map_poll(map_ctx *, uint64_t, int64_t, int *);

#define CHECK(cond, ...)                                   \
    do {                                                   \
        if (!(cond)) {                                     \
            std::printf("FAIL %s: ", scenario);            \
            std::printf(__VA_ARGS__);                      \
            std::printf(" (%s:%d)\n", __FILE__, __LINE__); \
            std::exit(1);                                  \
        }                                                  \
    } while (0)

static const char *scenario = "";

struct Job {
    std::vector<double> xyz, m, h, vol, M;
    std::vector<int64_t> cfo;
    map_particles_in p{};
    map_cells_in c{};
    map_out o{};
    map_stats st{};
    uint64_t id = 0;
};

static std::unique_ptr<Job> make(int tag, int n, bool bad = false)
{
    auto j = std::make_unique<Job>();
    const int nc = n / 2 + 1;
    j->xyz.assign(3 * (size_t)n, 0.5);
    j->m.assign((size_t)n, 1.0 / n);
    j->h.assign((size_t)n, 0.05);
    j->h[0] = tag + 0.25;  // the fake device reads the tag from h[0]
    j->vol.assign((size_t)nc, 1.0);
    if (bad) j->vol[0] = 0.0;
    j->cfo.assign((size_t)nc + 1, 0);
    j->M.assign((size_t)nc, -1.0);
    j->p.n = n;
    j->p.xyz = j->xyz.data();
    j->p.m = j->m.data();
    j->p.h = j->h.data();
    j->c.n_cells = nc;
    j->c.cell_face_off = j->cfo.data();
    j->c.face_vert_off = j->cfo.data();
    j->c.cell_volume = j->vol.data();
    for (int d = 0; d < 3; d++) j->c.box[3 + d] = 1.0;
    j->o.cell_mass = j->M.data();
    j->o.stats = &j->st;
    return j;
}

static double sum(const std::vector<double> &v)
{
    double s = 0;
    for (double x : v) s += x;
    return s;
}

static Ctx *context(int max_jobs, uint64_t budget = 0, int max_queue = 0)
{
    map_config cfg{};
    cfg.max_jobs = max_jobs;
    cfg.hbm_budget_bytes = budget;
    cfg.max_queue = max_queue;
    g_log.reset();
    return new Ctx(&cfg);
}

static void finish(Ctx *C)
{
    const int rc = serve_stop(*C);
    CHECK(rc == MAP_OK, "serve_stop returned %d", rc);
    delete C;
}

static int threads_used()
{
    std::lock_guard<std::mutex> g(g_log.mu);
    return (int)g_log.device_threads.size();
}

static int submit(Ctx *C, Job &j) { return map_submit(reinterpret_cast<map_ctx *>(C), &j.p, &j.c, &j.o, &j.id); }

static int poll(Ctx *C, Job &j, int64_t us, int *state) { return map_poll(reinterpret_cast<map_ctx *>(C), j.id, us, state); }

int main()
{
    std::setvbuf(stdout, nullptr, _IONBF, 0);  // keep every line if a sanitizer ends the run
    // jobs of one context all complete with the right outputs; slots bound concurrency
    {
        scenario = "complete";
        Ctx *C = context(3);
        std::vector<std::unique_ptr<Job>> js;
        for (int t = 0; t < 10; t++) js.push_back(make(t, 300 + 97 * t));
        for (auto &j : js) CHECK(submit(C, *j) == MAP_OK, "submit");
        for (auto &j : js) {
            int st = -1;
            CHECK(poll(C, *j, 30000000, &st) == MAP_OK && st == MAP_JOB_DONE, "state %d", st);
            CHECK(std::fabs(sum(j->M) - 1.0) < 1e-12, "mass %g", sum(j->M));
            CHECK(j->st.n_pairs == j->p.n, "stats");
            CHECK(j->st.ms_latency >= j->st.ms_queue && j->st.ms_queue >= 0.0, "latency");
        }
        CHECK(g_log.max_live <= 3, "max live %d", g_log.max_live);
        CHECK(threads_used() == 1, "device calls from %d threads", threads_used());
        finish(C);
        std::printf("ok %s (max live %d, batches %d, largest batch %d)\n", scenario, g_log.max_live, g_log.batches,
                    g_log.max_batch);
    }
    // one slot: admission in submission order
    {
        scenario = "fifo";
        Ctx *C = context(1);
        std::vector<std::unique_ptr<Job>> js;
        for (int t = 0; t < 8; t++) js.push_back(make(t, 200 + 50 * (7 - t)));
        for (auto &j : js) CHECK(submit(C, *j) == MAP_OK, "submit");
        for (auto &j : js) {
            int st = -1;
            CHECK(poll(C, *j, 30000000, &st) == MAP_OK && st == MAP_JOB_DONE, "state");
        }
        for (int t = 0; t < 8; t++) CHECK(g_log.order[t] == t, "position %d holds job %d", t, g_log.order[t]);
        finish(C);
        std::printf("ok %s\n", scenario);
    }
    // the budget bounds the footprint in flight, whatever the slot count
    {
        scenario = "budget";
        auto probe = make(0, 20000);
        const size_t F = job_footprint(&probe->p, &probe->c);
        const uint64_t budget = (uint64_t)(2.5 * (double)F);
        Ctx *C = context(8, budget);
        std::vector<std::unique_ptr<Job>> js;
        for (int t = 0; t < 9; t++) js.push_back(make(t, 20000));
        for (auto &j : js) CHECK(submit(C, *j) == MAP_OK, "submit");
        for (auto &j : js) {
            int st = -1;
            CHECK(poll(C, *j, 30000000, &st) == MAP_OK && st == MAP_JOB_DONE, "state");
        }
        CHECK(g_log.max_bytes <= budget, "in flight %zu > budget %llu", g_log.max_bytes, (unsigned long long)budget);
        CHECK(g_log.max_live <= 2, "max live %d", g_log.max_live);
        // a job larger than the whole budget is refused at submit
        auto big = make(99, 100000);
        CHECK(submit(C, *big) == MAP_ENOMEM, "oversized job accepted");
        finish(C);
        std::printf("ok %s (max in flight %zu of %llu)\n", scenario, g_log.max_bytes, (unsigned long long)budget);
    }
    // a full queue refuses; polls with a zero timeout return at once
    {
        scenario = "queue-full";
        g_log.stage_us = 20000;
        Ctx *C = context(1, 0, 2);
        std::vector<std::unique_ptr<Job>> js;
        for (int t = 0; t < 3; t++) js.push_back(make(t, 100));
        for (auto &j : js) CHECK(submit(C, *j) == MAP_OK, "submit");
        auto extra = make(3, 100);
        CHECK(submit(C, *extra) == MAP_EBUSY, "full queue accepted a job");
        int st = -1;
        CHECK(poll(C, *js[2], 0, &st) == MAP_OK && (st == MAP_JOB_PENDING || st == MAP_JOB_RUNNING), "state %d", st);
        for (auto &j : js) CHECK(poll(C, *j, 30000000, &st) == MAP_OK && st == MAP_JOB_DONE, "state");
        finish(C);
        g_log.stage_us = 200;
        std::printf("ok %s\n", scenario);
    }
    // a failing job reports its own error; the others are untouched
    {
        scenario = "isolation";
        Ctx *C = context(2);
        std::vector<std::unique_ptr<Job>> js;
        for (int t = 0; t < 7; t++) js.push_back(make(t, 400 + 10 * t, t == 3));
        for (auto &j : js) CHECK(submit(C, *j) == MAP_OK, "submit");
        for (int t = 0; t < 7; t++) {
            int st = -1;
            const int rc = poll(C, *js[t], 30000000, &st);
            if (t == 3) {
                CHECK(rc == MAP_EGEOM && st == MAP_JOB_FAILED, "bad job rc %d state %d", rc, st);
                CHECK(poll(C, *js[t], 0, &st) == MAP_ENOTFOUND, "failed job still known");
            } else {
                CHECK(rc == MAP_OK && st == MAP_JOB_DONE, "job %d rc %d", t, rc);
                CHECK(std::fabs(sum(js[t]->M) - 1.0) < 1e-12, "mass");
            }
        }
        CHECK(g_log.live == 0 && g_log.bytes == 0, "footprint leaked");
        finish(C);
        std::printf("ok %s\n", scenario);
    }
    // shutting down drains every queued and running job
    {
        scenario = "drain";
        Ctx *C = context(2);
        std::vector<std::unique_ptr<Job>> js;
        for (int t = 0; t < 6; t++) js.push_back(make(t, 500));
        for (auto &j : js) CHECK(submit(C, *j) == MAP_OK, "submit");
        finish(C);
        for (auto &j : js) CHECK(std::fabs(sum(j->M) - 1.0) < 1e-12, "job not finished by shutdown");
        std::printf("ok %s\n", scenario);
    }
    // many contexts with random slots, sizes and failures
    {
        scenario = "stress";
        std::mt19937 rng(7);
        for (int round = 0; round < 25; round++) {
            Ctx *C = context(1 + (int)(rng() % 4));
            std::vector<std::unique_ptr<Job>> js;
            const int nj = 3 + (int)(rng() % 10);
            for (int t = 0; t < nj; t++) js.push_back(make(t, 50 + (int)(rng() % 3000), rng() % 7 == 0));
            for (auto &j : js) CHECK(submit(C, *j) == MAP_OK, "submit");
            for (auto &j : js) {
                int st = -1;
                const int rc = poll(C, *j, 30000000, &st);
                const bool bad = j->vol[0] == 0.0;
                CHECK(bad ? (rc == MAP_EGEOM && st == MAP_JOB_FAILED) : (rc == MAP_OK && st == MAP_JOB_DONE),
                      "round %d rc %d state %d", round, rc, st);
            }
            finish(C);
        }
        std::printf("ok %s\n", scenario);
    }
    // growing and released slot workspaces use stream-ordered allocation: no
    // device-wide synchronisation, and only the scheduler thread makes the calls
    {
        scenario = "device-syncs";
        Ctx *C = context(2);
        std::vector<std::unique_ptr<Job>> js;
        for (int t = 0; t < 8; t++) js.push_back(make(t, 200 + 400 * t));
        for (auto &j : js) CHECK(submit(C, *j) == MAP_OK, "submit");
        for (auto &j : js) {
            int st = -1;
            CHECK(poll(C, *j, 30000000, &st) == MAP_OK && st == MAP_JOB_DONE, "state %d", st);
            CHECK(std::fabs(sum(j->M) - 1.0) < 1e-12, "mass");
        }
        CHECK(g_log.device_syncs == 0, "%d device-wide syncs from slot buffers", g_log.device_syncs);
        CHECK(threads_used() == 1, "device calls from %d threads", threads_used());
        finish(C);
        std::printf("ok %s\n", scenario);
    }
    // a launch that never completes: the jobs in flight and later ones fail
    // with MAP_EDEVICE within the time limit, polls and shutdown return
    {
        scenario = "watchdog";
        map_config cfg{};
        cfg.max_jobs = 2;
        cfg.serve_timeout_ms = 300;
        g_log.reset();
        g_log.hang_n = 777;
        Ctx *C = new Ctx(&cfg);
        auto a = make(0, 300);
        CHECK(submit(C, *a) == MAP_OK, "submit");
        int st = -1;
        CHECK(poll(C, *a, 30000000, &st) == MAP_OK && st == MAP_JOB_DONE, "first job state %d", st);
        auto hung = make(1, 777);
        auto b = make(2, 300);
        CHECK(submit(C, *hung) == MAP_OK && submit(C, *b) == MAP_OK, "submit");
        const auto t0 = std::chrono::steady_clock::now();
        CHECK(poll(C, *hung, -1, &st) == MAP_EDEVICE && st == MAP_JOB_FAILED, "hung job state %d", st);
        CHECK(poll(C, *b, -1, &st) == MAP_EDEVICE && st == MAP_JOB_FAILED, "later job state %d", st);
        const double ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
        CHECK(ms < 5000, "failure took %.0f ms", ms);
        auto c = make(3, 300);
        CHECK(submit(C, *c) == MAP_EDEVICE, "a stopped server accepted a job");
        CHECK(serve_stop(*C) == MAP_EDEVICE, "shutdown of a failed server reported success");
        g_log.release_hang();  // the context is left allocated, as map_shutdown does
        std::printf("ok %s (failed after %.0f ms)\n", scenario, ms);
    }
    std::printf("all scenarios passed\n");
    return 0;
}
