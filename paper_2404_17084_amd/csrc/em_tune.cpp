// Autotuner of the integration kernel's launch shape, with a text cache.
//
// For a given input the pair set is built once; then each candidate launch
// shape integrates every pair twice (the second run timed with HIP events on
// the library stream) and the fastest is stored for the pair count's size
// class.  All candidates produce results within rounding of each other; the
// tuner only chooses among them.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <sstream>

#include "em_internal.h"
#include "em_runtime.h"

namespace em {

// Untuned shape: task batches (distribution 3) for both precisions, with the
// register budgets and workgroup counts measured fastest on MI355X for the
// 262,144-particle clumpy workload (FP64: 3 waves per SIMD, 4 workgroups per
// CU; mixed: 6 and 6).
IntegrateTune default_tune(int precision)
{
    IntegrateTune t;
    t.persistent = 3;
    t.tile_waves = 1;
    t.grid_per_cu = precision == MAP_FP64 ? 4 : 6;
    t.waves = precision == MAP_FP64 ? 3 : 6;
    return t;
}

int size_class(int64_t n_pairs)
{
    int c = 0;
    while (c < 62 && (int64_t(1) << (c + 1)) <= n_pairs) c++;
    return c;
}

IntegrateTune pick_tune(const Ctx &C, int precision, int64_t n_pairs)
{
    if (C.has_explicit[precision]) return C.tune_explicit[precision];
    auto it = C.tune_table.find({precision, size_class(n_pairs)});
    if (it != C.tune_table.end()) return it->second;
    // nearest size class of the same precision
    int best = 1 << 30;
    IntegrateTune t = default_tune(precision);
    for (const auto &kv : C.tune_table) {
        if (kv.first.first != precision) continue;
        int d = std::abs(kv.first.second - size_class(n_pairs));
        if (d < best) {
            best = d;
            t = kv.second;
        }
    }
    return t;
}

// Cache lines: "<arch> <precision> <size class> <waves> <tile_waves> <grid_per_cu> <persistent> <ms>"
void tune_cache_load(Ctx &C)
{
    if (!C.config.tune_cache_path) return;
    std::ifstream in(C.config.tune_cache_path);
    if (!in) return;
    std::string line;
    while (std::getline(in, line)) {
        std::istringstream ss(line);
        std::string arch;
        int prec, cls, w, tw, g, pers;
        double ms;
        if (!(ss >> arch >> prec >> cls >> w >> tw >> g >> pers >> ms)) continue;
        if (arch != C.arch || (prec != MAP_FP64 && prec != MAP_MIXED)) continue;
        if (w < 0 || w > 8 || tw < 1 || tw > 64 || g < 1 || g > 64 || pers < 0 || pers > 3) continue;
        IntegrateTune t;
        t.waves = w;
        t.tile_waves = tw;
        t.grid_per_cu = g;
        t.persistent = pers;
        C.tune_table[{prec, cls}] = t;
    }
}

void tune_cache_save(const Ctx &C)
{
    if (!C.config.tune_cache_path) return;
    std::string tmp = std::string(C.config.tune_cache_path) + ".tmp";
    {
        std::ofstream out(tmp);
        if (!out) return;
        for (const auto &kv : C.tune_table) {
            const IntegrateTune &t = kv.second;
            out << C.arch << ' ' << kv.first.first << ' ' << kv.first.second << ' ' << t.waves << ' ' << t.tile_waves
                << ' ' << t.grid_per_cu << ' ' << t.persistent << ' ' << 0.0 << '\n';
        }
    }
    std::rename(tmp.c_str(), C.config.tune_cache_path);
}

}  // namespace em

using namespace em;

extern "C" int map_autotune(map_ctx *h, const map_particles_in *p, const map_cells_in *c, int precision,
                            int *best_out, double *best_ms)
{
    if (!h) return MAP_EINVAL;
    Ctx *C = reinterpret_cast<Ctx *>(h);
    std::lock_guard<std::mutex> guard(C->mu);
    C->back.valid = false;  // the tuner reuses the workspace
    try {
        EM_HIP(hipSetDevice(C->device));
        EM_CHECK(precision == MAP_FP64 || precision == MAP_MIXED, MAP_EINVAL, "precision must be MAP_FP64 or MAP_MIXED");
        hipStream_t s = C->stream;
        Workspace &ws = C->ws;
        DevInputs in;
        EdgeRec *edges;
        double *aabb;
        unsigned *flags;
        int64_t *counters;
        prepare(*C, ws, p, c, in, edges, aabb, flags, counters, s);
        PairSet ps = build_pairs(ws, in, aabb, edges, counters, s);
        build_tiles(ws, in, ps, s);
        const int64_t np = ps.n_pairs;
        EM_CHECK(np > 0, MAP_EINVAL, "no pairs to tune on");
        double *f = ws.get<double>(S_F, (size_t)np);
        uint32_t *tile_ctr = ws.get<uint32_t>(S_TILE_CTR, 64);
        const int64_t fix_cap = np / 8 + 65536;
        uint64_t *fix_items = ws.get<uint64_t>(S_FIX_ITEMS, (size_t)fix_cap);
        const int wv64[] = {2, 3};
        const int wvmx[] = {3, 6};
        const int tws[] = {1, 2};
        const int grids[] = {4, 8};
        const int dists[] = {1, 2, 3};
        IntegrateTune best = default_tune(precision);
        float best_t = 1e30f;
        for (int wi = 0; wi < 2; wi++)
            for (int d : dists)
                for (int tw : tws)
                    for (int g : grids) {
                        if (d >= 2 && tw != 1) continue;  // cell tiles and task batches ignore tile_waves
                        IntegrateTune t;
                        t.waves = precision == MAP_FP64 ? wv64[wi] : wvmx[wi];
                        t.persistent = d;
                        t.tile_waves = tw;
                        t.grid_per_cu = g;
                        launch_integrate(in, edges, ps, precision, t, f, nullptr, counters, tile_ctr, fix_items, fix_cap, s);
                        EM_HIP(hipEventRecord(C->ev[6], s));
                        launch_integrate(in, edges, ps, precision, t, f, nullptr, counters, tile_ctr, fix_items, fix_cap, s);
                        EM_HIP(hipEventRecord(C->ev[7], s));
                        EM_HIP(hipEventSynchronize(C->ev[7]));
                        float ms = 0.0f;
                        EM_HIP(hipEventElapsedTime(&ms, C->ev[6], C->ev[7]));
                        if (ms < best_t) {
                            best_t = ms;
                            best = t;
                        }
                    }
        C->tune_table[{precision, size_class(np)}] = best;
        tune_cache_save(*C);
        if (best_out) {
            best_out[0] = best.waves;
            best_out[1] = best.tile_waves;
            best_out[2] = best.grid_per_cu;
            best_out[3] = best.persistent;
        }
        if (best_ms) *best_ms = best_t;
        C->err.clear();
        return MAP_OK;
    } catch (const em::Error &e) {
        C->err = e.msg;
        return e.code;
    } catch (const std::exception &e) {
        C->err = e.what();
        return MAP_EDEVICE;
    }
}
