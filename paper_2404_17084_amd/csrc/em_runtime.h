// Library context and the stages shared by the synchronous and served paths.
#pragma once

#include <map>
#include <mutex>
#include <string>
#include <utility>
#include <vector>

#include "em_internal.h"

namespace em {

struct Server;  // serving loop, em_serve.cpp

struct Ctx {
    explicit Ctx(const map_config *cfg);
    ~Ctx();
    int device = 0;
    int precision = MAP_FP64;
    map_config config{};
    hipStream_t stream = nullptr;
    hipEvent_t ev[8] = {};
    std::mutex mu;
    std::string err;
    Workspace ws;
    // launch tuning of the integration kernel, per precision: an explicit
    // map_set_tune wins over the autotuner's table (keyed by precision and
    // the log2 size class of the pair count), which wins over the default
    IntegrateTune tune_explicit[2];
    bool has_explicit[2] = {false, false};
    std::map<std::pair<int, int>, IntegrateTune> tune_table;
    std::string arch;
    // the caller's config.tune_cache_path is borrowed only during map_init: a copy
    std::string tune_cache_path;
    Server *server = nullptr;
    // the last map_particles result, kept in the workspace for map_back: the
    // cell-major pairs, their fractions and S_a (and, once built, the
    // particle-major view of the pairs)
    struct {
        bool valid = false, have_view = false;
        int64_t n = 0, n_cells = 0, n_pairs = 0;
    } back;
    // remembered regions of the adaptive walk (cx, cy, cz, R, s_min per region)
    std::vector<double> regions;
    // the last map_voronoi grid
    VorGrid vor;
    double vor_box[6] = {0, 0, 0, 0, 0, 0};
    // table of the pyramid integral for MAP_TABLE (built on first use)
    struct {
        int n[3] = {64, 64, 64};
        bool built = false;
        double *d64 = nullptr;
        float *d32 = nullptr;
    } table;
};

IntegrateTune default_tune(int precision);
IntegrateTune pick_tune(const Ctx &C, int precision, int64_t n_pairs);
int size_class(int64_t n_pairs);
void tune_cache_load(Ctx &C);
void tune_cache_save(const Ctx &C);

// Device-side state of one mapping between its stages.
struct JobState {
    int precision = MAP_FP64;
    DevInputs in;
    EdgeRec *edges = nullptr;
    double *aabb = nullptr;
    unsigned *flags = nullptr;
    int64_t *counters = nullptr;
    PairSet ps;
    double *f = nullptr;
    float *err = nullptr;  // mixed path: per-pair FP32 error estimates
    uint32_t *tile_ctr = nullptr;
    uint64_t *fix_items = nullptr;
    int64_t fix_cap = 0;
    hipEvent_t ev_setup = nullptr, ev_fix = nullptr, ev_reduce = nullptr;  // optional timing events
};

void check_host_args(const map_particles_in *p, const map_cells_in *c);
void stage_pairs(Ctx &C, Workspace &ws, const map_particles_in *p, const map_cells_in *c, int precision,
                 JobState &js, hipStream_t s);
int64_t stage_finish(Ctx &C, Workspace &ws, JobState &js, const map_out *out, hipStream_t s, map_stats *st);
void prepare(Ctx &C, Workspace &ws, const map_particles_in *p, const map_cells_in *c, DevInputs &in, EdgeRec *&edges,
             double *&aabb, unsigned *&flags, int64_t *&counters, hipStream_t s);
void run_mapping(Ctx &C, Workspace &ws, const map_particles_in *p, const map_cells_in *c, const map_out *out,
                 int precision, hipStream_t s, bool timed);
// Drains and stops the serving loop (bounded wait).  MAP_OK when it stopped
// cleanly; MAP_EDEVICE when it had failed or did not stop: its device work may
// still be pending, so the context must then be left in place (not freed).
int serve_stop(Ctx &C);
// Builds the context's MAP_TABLE table if its size changed or it was never built.
void ensure_table(Ctx &C, hipStream_t s);
// Device-memory footprint estimate of a served job (admission against the budget).
size_t job_footprint(const map_particles_in *p, const map_cells_in *c);
// Whether map_submit accepts jobs (em_api.cpp).
bool serving_enabled();

}  // namespace em
