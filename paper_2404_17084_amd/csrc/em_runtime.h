// Library context and the stages shared by the synchronous and served paths.
#pragma once

#include <mutex>
#include <string>

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
    IntegrateTune tune;
    Server *server = nullptr;
};

void check_host_args(const map_particles_in *p, const map_cells_in *c);
void prepare(Ctx &C, Workspace &ws, const map_particles_in *p, const map_cells_in *c, DevInputs &in, EdgeRec *&edges,
             double *&aabb, unsigned *&flags, int64_t *&counters, hipStream_t s);
void run_mapping(Ctx &C, Workspace &ws, const map_particles_in *p, const map_cells_in *c, const map_out *out,
                 int precision, hipStream_t s, bool timed);
void serve_stop(Ctx &C);

}  // namespace em
