// C ABI of the Exact-mapping library: context, input staging, the synchronous
// mapping pipeline and its statistics.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <vector>
#include <memory>
#include <mutex>
#include <string>

#include "em_internal.h"
#include "em_runtime.h"

using namespace em;

namespace em {

Ctx::Ctx(const map_config *cfg) : ws(cfg ? cfg->device : 0)
{
    device = cfg ? cfg->device : 0;
    precision = cfg ? cfg->precision : MAP_FP64;
    if (cfg) config = *cfg;
    if (config.tune_cache_path) {
        tune_cache_path = config.tune_cache_path;
        config.tune_cache_path = tune_cache_path.c_str();
    }
    EM_HIP(hipSetDevice(device));
    noalloc_attach(device);
    EM_HIP(hipStreamCreateWithFlags(&stream, hipStreamNonBlocking));
    for (auto &e : ev) EM_HIP(hipEventCreate(&e));
    hipDeviceProp_t prop;
    EM_HIP(hipGetDeviceProperties(&prop, device));
    arch = prop.gcnArchName;
    tune_cache_load(*this);
}

Ctx::~Ctx()
{
    (void)hipSetDevice(device);
    if (stream) (void)hipStreamSynchronize(stream);
    ws.release();
    free_voronoi(vor);
    if (table.d64) (void)hipFree(table.d64);
    if (table.d32) (void)hipFree(table.d32);
    for (auto &e : ev)
        if (e) (void)hipEventDestroy(e);
    if (stream) (void)hipStreamDestroy(stream);
}

static const char *flag_text(unsigned f)
{
    if (f & F_CFO_BAD) return "cell_face_off is not a valid offset array (each cell needs >= 4 faces)";
    if (f & F_FVO_BAD) return "face_vert_off is not a valid offset array";
    if (f & F_FACE_SMALL) return "a face has fewer than 3 vertices";
    if (f & F_VID_RANGE) return "face_vert holds a vertex id out of range";
    if (f & F_PLANE_BAD) return "a face plane is not finite or its normal is not of unit length";
    if (f & F_VERT_NONFINITE) return "a vertex coordinate is not finite";
    if (f & F_VOL_BAD) return "a cell volume is not finite and positive";
    if (f & F_PART_NONFINITE) return "a particle position is not finite";
    if (f & F_H_NONPOS) return "a smoothing length is not finite and positive";
    if (f & F_M_BAD) return "a particle mass is not finite and non-negative";
    if (f & F_RESULT_NONFINITE) return "non-finite cell mass";
    return "invalid input";
}

static int flag_code(unsigned f)
{
    if (f & (F_CFO_BAD | F_FVO_BAD | F_FACE_SMALL | F_VID_RANGE | F_PLANE_BAD | F_VERT_NONFINITE | F_VOL_BAD))
        return MAP_EGEOM;
    if (f & F_RESULT_NONFINITE) return MAP_ENUMERIC;
    return MAP_EINVAL;
}

template <typename T>
static const T *stage(Workspace &ws, int slot, const T *src, int64_t count, int mem_kind, hipStream_t s)
{
    if (count <= 0) return ws.get<T>(slot, 1);
    if (mem_kind == MAP_MEM_DEVICE) return src;
    T *dst = ws.get<T>(slot, (size_t)count);
    EM_HIP(hipMemcpyAsync(dst, src, sizeof(T) * count, hipMemcpyHostToDevice, s));
    return dst;
}

void check_host_args(const map_particles_in *p, const map_cells_in *c)
{
    EM_CHECK(p && c, MAP_EINVAL, "null particle or cell descriptor");
    EM_CHECK(p->n >= 0, MAP_EINVAL, "particle count is negative");
    EM_CHECK(c->n_cells >= 0 && c->n_faces >= 0 && c->n_face_verts >= 0 && c->n_verts >= 0, MAP_EGEOM,
             "negative geometry size");
    EM_CHECK(p->n < (int64_t)INT32_MAX && c->n_cells < (int64_t)INT32_MAX && c->n_verts < (int64_t)INT32_MAX &&
                 c->n_faces < (int64_t)INT32_MAX && c->n_face_verts < (int64_t)INT32_MAX,
             MAP_EINVAL, "particle, cell, wall, wall-vertex or vertex count above 2^31-1");
    EM_CHECK(p->mem_kind == MAP_MEM_HOST || p->mem_kind == MAP_MEM_DEVICE, MAP_EINVAL, "bad particle mem_kind");
    EM_CHECK(c->mem_kind == MAP_MEM_HOST || c->mem_kind == MAP_MEM_DEVICE, MAP_EINVAL, "bad cell mem_kind");
    if (p->n > 0) EM_CHECK(p->xyz && p->m && p->h, MAP_EINVAL, "null particle array");
    EM_CHECK(c->cell_face_off && c->face_vert_off, MAP_EGEOM, "null offset array");
    if (c->n_faces > 0) EM_CHECK(c->face_plane, MAP_EGEOM, "null face_plane");
    if (c->n_face_verts > 0) EM_CHECK(c->face_vert, MAP_EGEOM, "null face_vert");
    if (c->n_verts > 0) EM_CHECK(c->verts, MAP_EGEOM, "null verts");
    for (int d = 0; d < 3; d++)
        EM_CHECK(std::isfinite(c->box[d]) && std::isfinite(c->box[3 + d]) && c->box[3 + d] > c->box[d], MAP_EGEOM,
                 "box must be finite with hi > lo");
    // host-resident offsets can be checked here; device ones are checked on the device
    if (c->mem_kind == MAP_MEM_HOST) {
        EM_CHECK(c->cell_face_off[0] == 0 && c->cell_face_off[c->n_cells] == c->n_faces, MAP_EGEOM,
                 "cell_face_off must start at 0 and end at n_faces");
        EM_CHECK(c->face_vert_off[0] == 0 && c->face_vert_off[c->n_faces] == c->n_face_verts, MAP_EGEOM,
                 "face_vert_off must start at 0 and end at n_face_verts");
    }
}

// Stage inputs, validate them on the device, build geometry tables.
void prepare(Ctx &C, Workspace &ws, const map_particles_in *p, const map_cells_in *c, DevInputs &in, EdgeRec *&edges,
             double *&aabb, unsigned *&flags, int64_t *&counters, hipStream_t s)
{
    check_host_args(p, c);
    in.n = p->n;
    in.n_cells = c->n_cells;
    in.n_faces = c->n_faces;
    in.n_face_verts = c->n_face_verts;
    in.n_verts = c->n_verts;
    for (int d = 0; d < 6; d++) in.box[d] = c->box[d];
    in.xyz = stage(ws, S_XYZ, p->xyz, 3 * p->n, p->mem_kind, s);
    in.m = stage(ws, S_M, p->m, p->n, p->mem_kind, s);
    in.h = stage(ws, S_H, p->h, p->n, p->mem_kind, s);
    in.cfo = stage(ws, S_CFO, c->cell_face_off, c->n_cells + 1, c->mem_kind, s);
    in.fvo = stage(ws, S_FVO, c->face_vert_off, c->n_faces + 1, c->mem_kind, s);
    in.fv = stage(ws, S_FV, c->face_vert, c->n_face_verts, c->mem_kind, s);
    in.plane = stage(ws, S_PLANE, c->face_plane, 4 * c->n_faces, c->mem_kind, s);
    in.verts = stage(ws, S_VERTS, c->verts, 3 * c->n_verts, c->mem_kind, s);
    in.vol = c->cell_volume ? stage(ws, S_VOL, c->cell_volume, c->n_cells, c->mem_kind, s) : nullptr;

    flags = ws.get<unsigned>(S_FLAGS, 4);
    counters = ws.get<int64_t>(S_COUNTERS, C_NUM);
    fill_zero_bytes(flags, sizeof(unsigned) * 4, s);
    fill_zero_bytes(counters, sizeof(int64_t) * C_NUM, s);
    launch_validate(in, flags, s);
    unsigned hf = 0;
    EM_HIP(hipMemcpyAsync(&hf, flags, sizeof(unsigned), hipMemcpyDeviceToHost, s));
    stream_sync(s);
    EM_CHECK(hf == 0, flag_code(hf), flag_text(hf));

    edges = ws.get<EdgeRec>(S_EDGE, (size_t)(c->n_face_verts > 0 ? c->n_face_verts : 1));
    aabb = ws.get<double>(S_AABB, (size_t)(11 * (c->n_cells > 0 ? c->n_cells : 1)));
    double *vol_out = nullptr;
    if (!in.vol) {
        vol_out = ws.get<double>(S_VOL, (size_t)(c->n_cells > 0 ? c->n_cells : 1));
        in.vol = vol_out;
    }
    launch_geometry(in, edges, aabb, vol_out, s);
    (void)C;
}

template <typename T>
static void copy_out(T *dst, const T *src, int64_t count, int mem_kind, hipStream_t s)
{
    if (!dst || count <= 0) return;
    EM_HIP(hipMemcpyAsync(dst, src, sizeof(T) * count,
                          mem_kind == MAP_MEM_DEVICE ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, s));
}

__global__ void k_u32_to_i32(const uint32_t *in, int32_t *out, int64_t n)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = (int32_t)in[i];
}

// Stage 1 of a mapping: inputs staged and validated, geometry tables, pair
// set, and the buffers the integration writes.
void stage_pairs(Ctx &C, Workspace &ws, const map_particles_in *p, const map_cells_in *c, int precision,
                 JobState &js, hipStream_t s)
{
    EM_CHECK(precision == MAP_FP64 || precision == MAP_MIXED || precision == MAP_TABLE, MAP_EINVAL,
             "precision must be MAP_FP64, MAP_MIXED or MAP_TABLE");
    js.precision = precision;
    prepare(C, ws, p, c, js.in, js.edges, js.aabb, js.flags, js.counters, s);
    if (js.ev_setup) EM_HIP(hipEventRecord(js.ev_setup, s));
    js.ps = build_pairs(ws, js.in, js.aabb, js.edges, js.counters, s);
    const int64_t np = js.ps.n_pairs;
    js.f = ws.get<double>(S_F, (size_t)(np > 0 ? np : 1));
    js.err = precision == MAP_MIXED ? ws.get<float>(S_ERR, (size_t)(np > 0 ? np : 1)) : nullptr;
    js.tile_ctr = ws.get<uint32_t>(S_TILE_CTR, 64);
    js.fix_cap = C.config.fixup_cap > 0 ? C.config.fixup_cap : np / 8 + 65536;
    js.fix_items = ws.get<uint64_t>(S_FIX_ITEMS, (size_t)js.fix_cap);
    fill_zero_bytes(js.tile_ctr, 2 * sizeof(unsigned), s);
}

// Stage 3: FP64 fixups of flagged edges (mixed path), S_a, M_i, rho_i, output
// copies and statistics.  Returns the number of fixed-up edge terms.
int64_t stage_finish(Ctx &C, Workspace &ws, JobState &js, const map_out *out, hipStream_t s, map_stats *st)
{
    (void)C;
    const DevInputs &in = js.in;
    const PairSet &ps = js.ps;
    const int64_t np = ps.n_pairs;
    double *f = js.f;
    int64_t n_fix = 0;
    if ((js.precision == MAP_MIXED || js.precision == MAP_FP64) && np > 0) {
        // the fixup list: edge terms flagged by the mixed path's conditioning
        // test, and pairs whose particle lies on two or more of the cell's
        // wall planes (winding weight), both precisions
        auto read_count = [&]() -> int64_t {
            unsigned hfix = 0;
            EM_HIP(hipMemcpyAsync(&hfix, js.tile_ctr + 1, sizeof(unsigned), hipMemcpyDeviceToHost, s));
            stream_sync(s);
            return (int64_t)hfix;
        };
        int64_t n_items = read_count();
        n_fix = n_items;
        if (n_items > js.fix_cap) {
            const IntegrateTune t64 = default_tune(MAP_FP64);
            if (js.precision == MAP_MIXED) {
                // too many flagged edges for the list: every pair again in FP64
                // (whose list then holds winding items only)
                launch_integrate(in, js.edges, ps, MAP_FP64, t64, f, nullptr, js.counters, js.tile_ctr,
                                 js.fix_items, js.fix_cap, s);
                n_items = read_count();
                n_fix = np;
                js.err = nullptr;  // FP64 values: nothing left to check
            }
            if (n_items > js.fix_cap) {
                // more winding items than the list holds: a list that fits them, and the FP64 pass again
                js.fix_cap = n_items;
                js.fix_items = ws.get<uint64_t>(S_FIX_ITEMS, (size_t)n_items);
                launch_integrate(in, js.edges, ps, MAP_FP64, t64, f, nullptr, js.counters, js.tile_ctr,
                                 js.fix_items, js.fix_cap, s);
                n_items = read_count();
                js.err = nullptr;
                EM_CHECK(n_items <= js.fix_cap, MAP_EDEVICE, "fixup list overflow after resizing");
                n_fix = np;
            }
        }
        if (js.precision == MAP_FP64 && n_fix != np) n_fix = 0;  // FP64: no edge terms are recomputed
        if (n_items > 0) {
            uint32_t *iv = ws.get<uint32_t>(S_FIX_VAL2, (size_t)n_items);
            uint64_t *k2 = ws.get<uint64_t>(S_FIX_KEY2, (size_t)n_items);
            uint32_t *v2 = reinterpret_cast<uint32_t *>(ws.get<uint64_t>(S_FIX_VALS, (size_t)n_items * 2));
            fill_iota_u32(iv, n_items, s);
            radix_sort_u64(ws, js.fix_items, iv, k2, v2, n_items, 64, s);
            double *fv = reinterpret_cast<double *>(k2);
            launch_fixup(in, js.edges, ps, js.fix_items, n_items, fv, js.counters, s);
            launch_fixup_apply(js.fix_items, fv, n_items, f, s);
        }
    }
    if (js.ev_fix) EM_HIP(hipEventRecord(js.ev_fix, s));
    int64_t n_cells_fp64 = 0;
    if (js.err && np > 0 && C.config.cell_tol >= 0.0) {
        // cells whose estimated FP32 error exceeds the budget: their pairs again in FP64
        const double tol = C.config.cell_tol > 0.0 ? C.config.cell_tol : kDefaultCellTol;
        unsigned *cnt = reinterpret_cast<unsigned *>(ws.get<uint32_t>(S_CHECK, (size_t)in.n_cells + 64));
        uint32_t *list = reinterpret_cast<uint32_t *>(cnt) + 64;
        launch_cell_check(in, ps, js.err, f, tol, cnt, list, in.n_cells, s);
        unsigned hc = 0;
        EM_HIP(hipMemcpyAsync(&hc, cnt, sizeof(unsigned), hipMemcpyDeviceToHost, s));
        stream_sync(s);
        n_cells_fp64 = hc;
        if (hc > 0) launch_recompute_cells(in, js.edges, ps, list, (int64_t)hc, f, js.counters, s);
    }
    double *S = ws.get<double>(S_S, (size_t)(in.n > 0 ? in.n : 1));
    double *M = ws.get<double>(S_MCELL, (size_t)(in.n_cells > 0 ? in.n_cells : 1));
    double *rho = ws.get<double>(S_RHO, (size_t)(in.n_cells > 0 ? in.n_cells : 1));
    double *red = ws.get<double>(S_RED, 16 + 4 * 256);
    EM_HIP(hipMemcpyAsync(red + 4, in.box, sizeof(double) * 6, hipMemcpyHostToDevice, s));
    launch_reduce(in, ps, f, S, M, rho, red, js.flags, s);
    if (js.ev_reduce) EM_HIP(hipEventRecord(js.ev_reduce, s));

    // outputs
    copy_out(out->cell_mass, (const double *)M, in.n_cells, out->mem_kind, s);
    copy_out(out->cell_density, (const double *)rho, in.n_cells, out->mem_kind, s);
    copy_out(out->frac_sum_raw, (const double *)S, in.n, out->mem_kind, s);
    if (out->pair_capacity > 0 && np > 0) {
        int64_t cnt = np < out->pair_capacity ? np : out->pair_capacity;
        copy_out(out->pair_frac, (const double *)f, cnt, out->mem_kind, s);
        if (out->pair_p || out->pair_c) {
            int32_t *tmp = reinterpret_cast<int32_t *>(ws.get<uint32_t>(S_KEY2, (size_t)np));
            if (out->pair_p) {
                hipLaunchKernelGGL(k_u32_to_i32, dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0, s, ps.pair_p, tmp,
                                   cnt);
                copy_out(out->pair_p, (const int32_t *)tmp, cnt, out->mem_kind, s);
            }
            if (out->pair_c) {
                stream_sync(s);
                hipLaunchKernelGGL(k_u32_to_i32, dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0, s, ps.pair_c, tmp,
                                   cnt);
                copy_out(out->pair_c, (const int32_t *)tmp, cnt, out->mem_kind, s);
            }
        }
    }
    double hred[4] = {0, 0, 0, 0};
    int64_t hcnt[C_NUM];
    unsigned hf = 0;
    EM_HIP(hipMemcpyAsync(hred, red, sizeof(hred), hipMemcpyDeviceToHost, s));
    EM_HIP(hipMemcpyAsync(hcnt, js.counters, sizeof(hcnt), hipMemcpyDeviceToHost, s));
    EM_HIP(hipMemcpyAsync(&hf, js.flags, sizeof(unsigned), hipMemcpyDeviceToHost, s));
    stream_sync(s);
    EM_CHECK(hf == 0, flag_code(hf), flag_text(hf));
    if (st) {
        std::memset(st, 0, sizeof(*st));
        st->n_pairs = np;
        st->n_candidates = hcnt[C_CANDIDATES];
        st->n_edge_terms = hcnt[C_EDGE_TERMS];
        st->n_fixup_terms = n_fix;
        st->n_boundary_pairs = hcnt[C_WINDING];
        st->n_fp64_cells = n_cells_fp64;
        st->n_fp64_pairs = hcnt[C_FP64_PAIRS];
        st->n_face_visits = hcnt[C_FACES];
        st->n_edge_visits = hcnt[C_EDGES];
        st->n_moment_evals = hcnt[C_MOMENTS];
        st->n_quad_intervals = hcnt[C_QUADS];
        st->n_angle_evals = hcnt[C_ANGLES];
        st->n_quad_points = hcnt[C_QPOINTS];
        st->mass_out = hred[0];
        st->max_abs_S_minus_1 = hred[1];
        st->mass_in = hred[2];
    }
    return n_fix;
}

// The table of the tabulated variant at the context's size (built once per size).
void ensure_table(Ctx &C, hipStream_t s)
{
    if (C.table.built) return;
    const size_t nodes = (size_t)C.table.n[0] * C.table.n[1] * C.table.n[2];
    if (C.table.d64) EM_HIP(hipFree(C.table.d64));
    if (C.table.d32) EM_HIP(hipFree(C.table.d32));
    C.table.d64 = nullptr;
    C.table.d32 = nullptr;
    EM_HIP(hipMalloc(&C.table.d64, sizeof(double) * nodes));
    EM_HIP(hipMalloc(&C.table.d32, sizeof(float) * nodes));
    launch_table_build(C.table.n[0], C.table.n[1], C.table.n[2], C.table.d64, C.table.d32, s);
    EM_HIP(hipStreamSynchronize(s));
    C.table.built = true;
}

// The whole synchronous mapping of one job on stream s with workspace ws.
void run_mapping(Ctx &C, Workspace &ws, const map_particles_in *p, const map_cells_in *c, const map_out *out,
                 int precision, hipStream_t s, bool timed)
{
    JobState js;
    if (timed) {
        EM_HIP(hipEventRecord(C.ev[0], s));
        js.ev_setup = C.ev[1];
    }
    stage_pairs(C, ws, p, c, precision, js, s);
    if (precision == MAP_TABLE) {
        ensure_table(C, s);
        if (timed) EM_HIP(hipEventRecord(C.ev[2], s));
        launch_integrate_table(js.in, js.edges, js.ps, C.table.d32, C.table.n[0], C.table.n[1], C.table.n[2], js.f,
                               js.counters, s);
    } else {
        const IntegrateTune tune = pick_tune(C, precision, js.ps.n_pairs);
        if (tune.persistent == 2) build_tiles(ws, js.in, js.ps, s);
        if (timed) EM_HIP(hipEventRecord(C.ev[2], s));
        launch_integrate(js.in, js.edges, js.ps, precision, tune, js.f, js.err, js.counters, js.tile_ctr, js.fix_items,
                         js.fix_cap, s);
    }
    if (timed) {
        EM_HIP(hipEventRecord(C.ev[3], s));
        js.ev_fix = C.ev[4];
        js.ev_reduce = C.ev[5];
    }
    map_stats local;
    stage_finish(C, ws, js, out, s, &local);
    if (timed) {
        float t;
        EM_HIP(hipEventElapsedTime(&t, C.ev[0], C.ev[1]));
        local.ms_setup = t;
        EM_HIP(hipEventElapsedTime(&t, C.ev[1], C.ev[2]));
        local.ms_pairs = t;
        EM_HIP(hipEventElapsedTime(&t, C.ev[2], C.ev[3]));
        local.ms_integrate = t;
        EM_HIP(hipEventElapsedTime(&t, C.ev[3], C.ev[4]));
        local.ms_fixup = t;
        EM_HIP(hipEventElapsedTime(&t, C.ev[4], C.ev[5]));
        local.ms_reduce = t;
        EM_HIP(hipEventElapsedTime(&t, C.ev[0], C.ev[5]));
        local.ms_total = t;
    }
    if (out->stats) *out->stats = local;
    C.back.valid = true;
    C.back.have_view = false;
    C.back.n = js.in.n;
    C.back.n_cells = js.in.n_cells;
    C.back.n_pairs = js.ps.n_pairs;
}

}  // namespace em

// The served path (em_serve.cpp) is part of this build; the fake device of
// the serving tests replaces this with its own switch.
bool em::serving_enabled() { return true; }

// Message of the last failed map_init on this thread (map_last_error(NULL)).
static thread_local std::string g_init_err;

// Distinct files of the HIP runtime (libamdhip64) mapped into this process.
// Two runtimes in one process each keep their own device state, and device
// pointers, streams and events of one are not valid in the other.
static std::vector<std::string> hip_runtimes_mapped()
{
    std::vector<std::string> out;
    FILE *fh = std::fopen("/proc/self/maps", "r");
    if (!fh) return out;
    char line[4096];
    while (std::fgets(line, sizeof(line), fh)) {
        const char *path = std::strchr(line, '/');
        if (!path || !std::strstr(path, "libamdhip64")) continue;
        std::string p(path);
        while (!p.empty() && (p.back() == '\n' || p.back() == ' ')) p.pop_back();
        if (std::find(out.begin(), out.end(), p) == out.end()) out.push_back(p);
    }
    std::fclose(fh);
    return out;
}

// ---------------------------------------------------------------- C ABI
#define API_BODY(ctx, body)                          \
    do {                                             \
        if (!(ctx)) return MAP_EINVAL;               \
        std::lock_guard<std::mutex> _g((ctx)->mu);   \
        try {                                        \
            EM_HIP(hipSetDevice((ctx)->device));     \
            body;                                    \
            (ctx)->err.clear();                      \
            return MAP_OK;                           \
        } catch (const em::Error &e) {               \
            (ctx)->err = e.msg;                      \
            return e.code;                           \
        } catch (const std::bad_alloc &) {           \
            (ctx)->err = "host allocation failed";   \
            return MAP_ENOMEM;                       \
        } catch (const std::exception &e) {          \
            (ctx)->err = e.what();                   \
            return MAP_EDEVICE;                      \
        }                                            \
    } while (0)

extern "C" {

int map_init(const map_config *cfg, map_ctx **out)
{
    g_init_err.clear();
    if (!out) return MAP_EINVAL;
    *out = nullptr;
    {
        const std::vector<std::string> rt = hip_runtimes_mapped();
        if (rt.size() > 1) {
            g_init_err = "two HIP runtimes are loaded in this process (" + rt[0] + ", " + rt[1] +
                         "); load the one the library should use first (e.g. import torch before the library)";
            return MAP_EDEVICE;
        }
    }
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0) {
        (void)hipGetLastError();
        return MAP_EDEVICE;
    }
    int dev = cfg ? cfg->device : 0;
    if (dev < 0 || dev >= ndev) return MAP_EINVAL;
    if (cfg && cfg->precision != MAP_FP64 && cfg->precision != MAP_MIXED && cfg->precision != MAP_TABLE)
        return MAP_EINVAL;
    try {
        *out = reinterpret_cast<map_ctx *>(new Ctx(cfg));
    } catch (const em::Error &e) {
        return e.code;
    } catch (...) {
        return MAP_EDEVICE;
    }
    return MAP_OK;
}

int map_shutdown(map_ctx *h)
{
    if (!h) return MAP_EINVAL;
    Ctx *C = reinterpret_cast<Ctx *>(h);
    if (serve_stop(*C) != MAP_OK) {
        // the serving loop failed or is stuck: its device work may still be
        // pending, so the context stays allocated (released at process exit)
        return MAP_EDEVICE;
    }
    delete C;
    return MAP_OK;
}

const char *map_last_error(map_ctx *h)
{
    if (!h) return g_init_err.c_str();
    return reinterpret_cast<Ctx *>(h)->err.c_str();
}

int map_set_precision(map_ctx *h, int precision)
{
    Ctx *C = reinterpret_cast<Ctx *>(h);
    API_BODY(C, {
        EM_CHECK(precision == MAP_FP64 || precision == MAP_MIXED || precision == MAP_TABLE, MAP_EINVAL,
                 "precision must be MAP_FP64, MAP_MIXED or MAP_TABLE");
        C->precision = precision;
    });
}

int map_voronoi(map_ctx *h, int64_t n, const double *sites, int mem_kind, const double box[6], int lloyd_iters,
                double merge_dist, map_voronoi_out *out)
{
    Ctx *C = reinterpret_cast<Ctx *>(h);
    API_BODY(C, {
        C->back.valid = false;
        EM_CHECK(out && box, MAP_EINVAL, "null output or box");
        EM_CHECK(n >= 1 && n < (int64_t)INT32_MAX, MAP_EINVAL, "site count outside [1, 2^31-1)");
        EM_CHECK(sites, MAP_EINVAL, "null sites");
        EM_CHECK(mem_kind == MAP_MEM_HOST || mem_kind == MAP_MEM_DEVICE, MAP_EINVAL, "bad sites mem_kind");
        EM_CHECK(lloyd_iters >= 0 && lloyd_iters <= 1000, MAP_EINVAL, "lloyd_iters outside [0, 1000]");
        EM_CHECK(std::isfinite(merge_dist) && merge_dist >= 0.0, MAP_EINVAL, "merge_dist must be finite and >= 0");
        for (int d = 0; d < 3; d++)
            EM_CHECK(std::isfinite(box[d]) && std::isfinite(box[3 + d]) && box[3 + d] > box[d], MAP_EINVAL,
                     "box must be finite with hi > lo");
        hipStream_t s = C->stream;
        VorGrid &V = C->vor;
        V.n = 0;
        auto grow = [&](double *&p, size_t &cap, size_t count) {
            if (cap < count || !p) {
                if (p) EM_HIP(hipFree(p));
                p = nullptr;
                EM_HIP(hipMalloc(&p, sizeof(double) * count));
                cap = count;
            }
        };
        grow(V.input, V.cap_input, (size_t)(3 * n));
        grow(V.sites, V.cap_sites, (size_t)(3 * n));
        if (V.cap_site_cell < (size_t)n || !V.site_cell) {
            if (V.site_cell) EM_HIP(hipFree(V.site_cell));
            V.site_cell = nullptr;
            EM_HIP(hipMalloc(&V.site_cell, sizeof(int64_t) * n));
            V.cap_site_cell = (size_t)n;
        }
        EM_HIP(hipMemcpyAsync(V.input, sites, sizeof(double) * 3 * n,
                              mem_kind == MAP_MEM_DEVICE ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, s));
        EM_HIP(hipEventRecord(C->ev[0], s));
        // merging of tightly packed sites, then the grid and its Lloyd steps (the sites live in the
        // grid's own buffer: each step replaces them with the centroids)
        int64_t m = n;
        if (merge_dist > 0.0)
            m = merge_sites(C->ws, n, V.input, box, merge_dist, V.sites, s);
        else
            EM_HIP(hipMemcpyAsync(V.sites, V.input, sizeof(double) * 3 * n, hipMemcpyDeviceToDevice, s));
        for (int it = 0; it <= lloyd_iters; it++) {
            V.n = 0;
            build_voronoi(C->ws, V, m, V.sites, box, s);
            if (it < lloyd_iters)
                EM_HIP(hipMemcpyAsync(V.sites, V.cen, sizeof(double) * 3 * m, hipMemcpyDeviceToDevice, s));
        }
        if (lloyd_iters == 0 && merge_dist == 0.0)
            fill_iota_i64(V.site_cell, n, s);  // the sites are the input points, distinct: each is its own nearest
        else
            site_cells(C->ws, V, n, V.input, box, V.site_cell, s);
        V.n_in = n;
        EM_HIP(hipEventRecord(C->ev[1], s));
        EM_HIP(hipEventSynchronize(C->ev[1]));
        float ms = 0.f;
        EM_HIP(hipEventElapsedTime(&ms, C->ev[0], C->ev[1]));
        // the per-cell records of the build (about 5.9 kB per cell) are not kept
        C->ws.drop(S_VOR8);
        for (int d = 0; d < 6; d++) C->vor_box[d] = box[d];
        out->n_cells = m;
        out->n_faces = V.n_faces;
        out->n_face_verts = V.n_slots;
        out->n_verts = V.n_verts;
        map_cells_in &c = out->cells;
        c.n_cells = m;
        c.n_faces = V.n_faces;
        c.n_face_verts = V.n_slots;
        c.n_verts = V.n_verts;
        c.cell_face_off = V.cfo;
        c.face_vert_off = V.fvo;
        c.face_vert = V.fv;
        c.face_plane = V.plane;
        c.verts = V.verts;
        c.cell_volume = V.vol;
        for (int d = 0; d < 6; d++) c.box[d] = box[d];
        c.mem_kind = MAP_MEM_DEVICE;
        out->face_nb = V.fnb;
        out->sites = V.sites;
        out->centroid = V.cen;
        out->n_sites = n;
        out->site_cell = V.site_cell;
        out->ms = ms;
    });
}

int map_voronoi_copy(map_ctx *h, int mem_kind, int64_t *cell_face_off, int64_t *face_vert_off, int32_t *face_vert,
                     double *face_plane, int64_t *face_nb, double *verts, double *cell_volume, double *centroid,
                     double *sites, int64_t *site_cell)
{
    Ctx *C = reinterpret_cast<Ctx *>(h);
    API_BODY(C, {
        EM_CHECK(mem_kind == MAP_MEM_HOST || mem_kind == MAP_MEM_DEVICE, MAP_EINVAL, "bad mem_kind");
        const VorGrid &V = C->vor;
        EM_CHECK(V.n > 0, MAP_EINVAL, "no Voronoi grid in this context");
        const hipMemcpyKind k = mem_kind == MAP_MEM_DEVICE ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
        hipStream_t s = C->stream;
        if (cell_face_off) EM_HIP(hipMemcpyAsync(cell_face_off, V.cfo, sizeof(int64_t) * (V.n + 1), k, s));
        if (face_vert_off) EM_HIP(hipMemcpyAsync(face_vert_off, V.fvo, sizeof(int64_t) * (V.n_faces + 1), k, s));
        if (face_vert) EM_HIP(hipMemcpyAsync(face_vert, V.fv, sizeof(int32_t) * V.n_slots, k, s));
        if (face_plane) EM_HIP(hipMemcpyAsync(face_plane, V.plane, sizeof(double) * 4 * V.n_faces, k, s));
        if (face_nb) EM_HIP(hipMemcpyAsync(face_nb, V.fnb, sizeof(int64_t) * V.n_faces, k, s));
        if (verts) EM_HIP(hipMemcpyAsync(verts, V.verts, sizeof(double) * 3 * V.n_verts, k, s));
        if (cell_volume) EM_HIP(hipMemcpyAsync(cell_volume, V.vol, sizeof(double) * V.n, k, s));
        if (centroid) EM_HIP(hipMemcpyAsync(centroid, V.cen, sizeof(double) * 3 * V.n, k, s));
        if (sites) EM_HIP(hipMemcpyAsync(sites, V.sites, sizeof(double) * 3 * V.n, k, s));
        if (site_cell) EM_HIP(hipMemcpyAsync(site_cell, V.site_cell, sizeof(int64_t) * V.n_in, k, s));
        EM_HIP(hipStreamSynchronize(s));
    });
}

int map_set_table(map_ctx *h, int n0, int n1, int n2)
{
    Ctx *C = reinterpret_cast<Ctx *>(h);
    API_BODY(C, {
        EM_CHECK(n0 >= 8 && n0 <= 1024 && n1 >= 8 && n1 <= 1024 && n2 >= 8 && n2 <= 1024, MAP_EINVAL,
                 "table sizes must be in [8, 1024]");
        EM_CHECK((int64_t)n0 * n1 * n2 <= ((int64_t)1 << 27), MAP_EINVAL, "table larger than 2^27 nodes");
        if (n0 != C->table.n[0] || n1 != C->table.n[1] || n2 != C->table.n[2]) {
            C->table.n[0] = n0;
            C->table.n[1] = n1;
            C->table.n[2] = n2;
            C->table.built = false;
        }
    });
}

int map_get_table(map_ctx *h, double *values)
{
    Ctx *C = reinterpret_cast<Ctx *>(h);
    API_BODY(C, {
        EM_CHECK(values, MAP_EINVAL, "null values buffer");
        ensure_table(*C, C->stream);
        const size_t nodes = (size_t)C->table.n[0] * C->table.n[1] * C->table.n[2];
        EM_HIP(hipMemcpyAsync(values, C->table.d64, sizeof(double) * nodes, hipMemcpyDeviceToHost, C->stream));
        EM_HIP(hipStreamSynchronize(C->stream));
    });
}

int map_set_tune(map_ctx *h, int precision, int waves, int tile_waves, int grid_per_cu, int persistent)
{
    Ctx *C = reinterpret_cast<Ctx *>(h);
    API_BODY(C, {
        EM_CHECK(precision == MAP_FP64 || precision == MAP_MIXED, MAP_EINVAL, "precision must be MAP_FP64 or MAP_MIXED");
        EM_CHECK(persistent >= -1 && persistent <= 3, MAP_EINVAL, "persistent must be -1 (clear), 0, 1, 2 or 3");
        if (persistent < 0) {
            C->has_explicit[precision] = false;
        } else {
            EM_CHECK(waves >= 0 && waves <= 8, MAP_EINVAL, "waves must be in [0, 8]");
            EM_CHECK(tile_waves >= 1 && tile_waves <= 64, MAP_EINVAL, "tile_waves must be in [1, 64]");
            EM_CHECK(grid_per_cu >= 1 && grid_per_cu <= 64, MAP_EINVAL, "grid_per_cu must be in [1, 64]");
            IntegrateTune &t = C->tune_explicit[precision];
            t.waves = waves;
            t.tile_waves = tile_waves;
            t.grid_per_cu = grid_per_cu;
            t.persistent = persistent;
            C->has_explicit[precision] = true;
        }
    });
}

int map_get_tune(map_ctx *h, int precision, int64_t n_pairs, int *waves, int *tile_waves, int *grid_per_cu,
                 int *persistent)
{
    Ctx *C = reinterpret_cast<Ctx *>(h);
    API_BODY(C, {
        EM_CHECK(precision == MAP_FP64 || precision == MAP_MIXED, MAP_EINVAL, "precision must be MAP_FP64 or MAP_MIXED");
        const IntegrateTune t = pick_tune(*C, precision, n_pairs);
        if (waves) *waves = t.waves;
        if (tile_waves) *tile_waves = t.tile_waves;
        if (grid_per_cu) *grid_per_cu = t.grid_per_cu;
        if (persistent) *persistent = t.persistent;
    });
}

int map_pairs(map_ctx *h, const map_particles_in *p, const map_cells_in *c, int64_t *n_pairs, int32_t *pair_p,
              int32_t *pair_c, int64_t capacity)
{
    Ctx *C = reinterpret_cast<Ctx *>(h);
    API_BODY(C, {
        C->back.valid = false;
        EM_CHECK(n_pairs, MAP_EINVAL, "n_pairs is null");
        EM_CHECK(capacity >= 0, MAP_EINVAL, "negative capacity");
        hipStream_t s = C->stream;
        DevInputs in;
        EdgeRec *edges;
        double *aabb;
        unsigned *flags;
        int64_t *counters;
        prepare(*C, C->ws, p, c, in, edges, aabb, flags, counters, s);
        PairSet ps = build_pairs(C->ws, in, aabb, edges, counters, s);
        *n_pairs = ps.n_pairs;
        int64_t cnt = ps.n_pairs < capacity ? ps.n_pairs : capacity;
        if (cnt > 0 && (pair_p || pair_c)) {
            int32_t *tmp = reinterpret_cast<int32_t *>(C->ws.get<uint32_t>(S_KEY2, (size_t)ps.n_pairs));
            if (pair_p) {
                hipLaunchKernelGGL(k_u32_to_i32, dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0, s, ps.pair_p, tmp,
                                   cnt);
                EM_HIP(hipMemcpyAsync(pair_p, tmp, sizeof(int32_t) * cnt, hipMemcpyDeviceToHost, s));
                EM_HIP(hipStreamSynchronize(s));
            }
            if (pair_c) {
                hipLaunchKernelGGL(k_u32_to_i32, dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0, s, ps.pair_c, tmp,
                                   cnt);
                EM_HIP(hipMemcpyAsync(pair_c, tmp, sizeof(int32_t) * cnt, hipMemcpyDeviceToHost, s));
            }
        }
        EM_HIP(hipStreamSynchronize(s));
    });
}

int map_particles(map_ctx *h, const map_particles_in *p, const map_cells_in *c, map_out *out)
{
    Ctx *C = reinterpret_cast<Ctx *>(h);
    API_BODY(C, {
        C->back.valid = false;
        EM_CHECK(out, MAP_EINVAL, "null output descriptor");
        EM_CHECK(out->mem_kind == MAP_MEM_HOST || out->mem_kind == MAP_MEM_DEVICE, MAP_EINVAL, "bad output mem_kind");
        run_mapping(*C, C->ws, p, c, out, C->precision, C->stream, true);
    });
}

int map_back(map_ctx *h, const double *cell_values, int mem_kind, double *particle_values, int out_mem_kind)
{
    Ctx *C = reinterpret_cast<Ctx *>(h);
    API_BODY(C, {
        EM_CHECK(C->back.valid, MAP_EINVAL,
                 "no mapping to invert: map_back uses the pairs of the last successful map_particles call of this "
                 "context, and another call has run since or none has");
        EM_CHECK(mem_kind == MAP_MEM_HOST || mem_kind == MAP_MEM_DEVICE, MAP_EINVAL, "bad input mem_kind");
        EM_CHECK(out_mem_kind == MAP_MEM_HOST || out_mem_kind == MAP_MEM_DEVICE, MAP_EINVAL, "bad output mem_kind");
        const int64_t n = C->back.n;
        const int64_t nc = C->back.n_cells;
        const int64_t np = C->back.n_pairs;
        EM_CHECK(nc == 0 || cell_values, MAP_EINVAL, "null cell values");
        EM_CHECK(n == 0 || particle_values, MAP_EINVAL, "null particle values");
        hipStream_t s = C->stream;
        Workspace &ws = C->ws;
        if (n > 0) {
            uint32_t *perm = ws.get<uint32_t>(S_PERM, (size_t)(np > 0 ? np : 1));
            int64_t *poff = ws.get<int64_t>(S_POFF, (size_t)n + 1);
            const uint32_t *pair_p = ws.get<uint32_t>(S_PAIR_P, (size_t)(np > 0 ? np : 1));
            const uint32_t *pair_c = ws.get<uint32_t>(S_PAIR_C, (size_t)(np > 0 ? np : 1));
            const double *f = ws.get<double>(S_F, (size_t)(np > 0 ? np : 1));
            const double *S = ws.get<double>(S_S, (size_t)n);
            if (!C->back.have_view) {
                build_particle_view(ws, pair_p, np, n, perm, poff, s);
                C->back.have_view = true;
            }
            const double *q = stage(ws, S_BACK_IN, cell_values, nc, mem_kind, s);
            double *out = out_mem_kind == MAP_MEM_DEVICE ? particle_values : ws.get<double>(S_BACK_OUT, (size_t)n);
            launch_map_back(n, poff, perm, pair_c, f, S, q, out, s);
            if (out_mem_kind == MAP_MEM_HOST)
                EM_HIP(hipMemcpyAsync(particle_values, out, sizeof(double) * n, hipMemcpyDeviceToHost, s));
        }
        EM_HIP(hipStreamSynchronize(s));
    });
}

}  // extern "C"

namespace em {

// Arguments shared by map_pseudo and map_pseudo_adaptive.
static void check_pseudo_args(const map_particles_in *p, const double box[6], const double *src_xyz, int n_src,
                              const map_pseudo_params *par, const map_pseudo_out *out)
{
    EM_CHECK(p && box && par && out, MAP_EINVAL, "null argument");
    EM_CHECK(p->n >= 0 && p->n < (int64_t)INT32_MAX, MAP_EINVAL, "particle count outside [0, 2^31-1)");
    EM_CHECK(p->mem_kind == MAP_MEM_HOST || p->mem_kind == MAP_MEM_DEVICE, MAP_EINVAL, "bad particle mem_kind");
    if (p->n > 0) EM_CHECK(p->xyz && p->m && p->h, MAP_EINVAL, "null particle array");
    for (int d = 0; d < 3; d++)
        EM_CHECK(std::isfinite(box[d]) && std::isfinite(box[3 + d]) && box[3 + d] > box[d], MAP_EINVAL,
                 "box must be finite with hi > lo");
    EM_CHECK(src_xyz && n_src >= 1 && n_src <= 64, MAP_EINVAL, "need 1 to 64 sources");
    for (int k = 0; k < 3 * n_src; k++) EM_CHECK(std::isfinite(src_xyz[k]), MAP_EINVAL, "non-finite source");
    EM_CHECK(std::isfinite(par->theta) && par->theta >= 0.0, MAP_EINVAL, "theta must be finite and >= 0");
    EM_CHECK(std::isfinite(par->r_part) && par->r_part >= 0.0 && std::isfinite(par->r_leaf) && par->r_leaf >= 0.0,
             MAP_EINVAL, "r_part and r_leaf must be finite and >= 0");
    EM_CHECK(par->leaf_size >= 1 && par->leaf_size <= 64, MAP_EINVAL, "leaf_size must be in [1, 64]");
    EM_CHECK(std::isfinite(par->h_fact_node) && par->h_fact_node > 0.0, MAP_EINVAL, "h_fact_node must be > 0");
    EM_CHECK(out->capacity >= 0, MAP_EINVAL, "negative capacity");
    EM_CHECK(out->mem_kind == MAP_MEM_HOST || out->mem_kind == MAP_MEM_DEVICE, MAP_EINVAL, "bad output mem_kind");
}

static PseudoDest dest_of(const map_pseudo_out *out)
{
    PseudoDest d;
    d.capacity = out->capacity;
    d.xyz = out->xyz;
    d.m = out->m;
    d.h = out->h;
    d.size = out->size;
    d.kind = out->kind;
    d.ref = out->ref;
    d.mem_kind = out->mem_kind;
    return d;
}

static DevParticles stage_particles(Ctx &C, const map_particles_in *p, hipStream_t s)
{
    DevParticles dp;
    dp.n = p->n;
    dp.xyz = stage(C.ws, S_XYZ, p->xyz, 3 * p->n, p->mem_kind, s);
    dp.m = stage(C.ws, S_M, p->m, p->n, p->mem_kind, s);
    dp.h = stage(C.ws, S_H, p->h, p->n, p->mem_kind, s);
    return dp;
}

}  // namespace em

extern "C" {

int map_pseudo_adaptive(map_ctx *h, const map_particles_in *p, const double box[6], const double *src_xyz,
                        int n_src, const map_pseudo_params *par, const map_adapt_params *ap, map_pseudo_out *out,
                        map_adapt_stats *stats)
{
    Ctx *C = reinterpret_cast<Ctx *>(h);
    API_BODY(C, {
        C->back.valid = false;
        check_pseudo_args(p, box, src_xyz, n_src, par, out);
        EM_CHECK(ap && ap->neutral, MAP_EINVAL, "null adaptive parameters or callback");
        EM_CHECK(std::isfinite(ap->K) && ap->K > 0.0, MAP_EINVAL, "K must be finite and > 0");
        EM_CHECK(ap->max_walks >= 1, MAP_EINVAL, "max_walks must be >= 1");
        hipStream_t s = C->stream;
        const DevParticles dp = stage_particles(*C, p, s);
        map_pseudo_stats st{};
        map_adapt_stats ast{};
        std::vector<double> regions = C->regions;
        const int64_t n_out =
            run_pseudo_adaptive(C->ws, dp, box, src_xyz, n_src, *par, *ap, regions, dest_of(out), &st, &ast, s, C->ev);
        out->n_out = n_out;
        EM_CHECK(out->capacity >= n_out, MAP_EINVAL,
                 "output capacity " + std::to_string(out->capacity) + " below the pseudo count " +
                     std::to_string(n_out));
        C->regions.swap(regions);
        st.ms_tree = ast.ms_tree;
        st.ms_total = ast.ms_total;
        if (out->stats) *out->stats = st;
        if (stats) *stats = ast;
    });
}

int map_get_regions(map_ctx *h, int64_t capacity, double *regions, int64_t *n_regions)
{
    Ctx *C = reinterpret_cast<Ctx *>(h);
    API_BODY(C, {
        EM_CHECK(n_regions && capacity >= 0, MAP_EINVAL, "null count or negative capacity");
        const int64_t n = (int64_t)C->regions.size() / 5;
        *n_regions = n;
        if (capacity >= n && n > 0) {
            EM_CHECK(regions, MAP_EINVAL, "null regions buffer");
            std::memcpy(regions, C->regions.data(), sizeof(double) * 5 * n);
        }
    });
}

int map_set_regions(map_ctx *h, int64_t n_regions, const double *regions)
{
    Ctx *C = reinterpret_cast<Ctx *>(h);
    API_BODY(C, {
        EM_CHECK(n_regions >= 0, MAP_EINVAL, "negative region count");
        EM_CHECK(n_regions <= MAP_MAX_REGIONS, MAP_ENOMEM, "more than MAP_MAX_REGIONS regions");
        EM_CHECK(n_regions == 0 || regions, MAP_EINVAL, "null regions");
        for (int64_t r = 0; r < n_regions; r++) {
            const double *g = regions + 5 * r;
            for (int k = 0; k < 5; k++) EM_CHECK(std::isfinite(g[k]), MAP_EINVAL, "non-finite region value");
            EM_CHECK(g[3] > 0.0 && g[4] >= 0.0, MAP_EINVAL, "region radius must be > 0 and s_min >= 0");
        }
        C->regions.assign(regions, regions + 5 * n_regions);
    });
}

int map_pseudo(map_ctx *h, const map_particles_in *p, const double box[6], const double *src_xyz, int n_src,
               const map_pseudo_params *par, map_pseudo_out *out)
{
    Ctx *C = reinterpret_cast<Ctx *>(h);
    API_BODY(C, {
        C->back.valid = false;
        check_pseudo_args(p, box, src_xyz, n_src, par, out);
        hipStream_t s = C->stream;
        const DevParticles dp = stage_particles(*C, p, s);
        map_pseudo_stats st{};
        const int64_t n_out = run_pseudo(C->ws, dp, box, src_xyz, n_src, *par, dest_of(out), &st, s, C->ev);
        out->n_out = n_out;
        if (p->n > 0) {
            float t = 0.f;
            EM_HIP(hipEventElapsedTime(&t, C->ev[0], C->ev[1]));
            st.ms_tree = t;
            EM_HIP(hipEventElapsedTime(&t, C->ev[1], C->ev[2]));
            st.ms_walk = t;
            EM_HIP(hipEventElapsedTime(&t, C->ev[2], C->ev[3]));
            st.ms_hsolve = t;
            EM_HIP(hipEventElapsedTime(&t, C->ev[0], C->ev[3]));
            st.ms_total = t;
        }
        if (out->stats) *out->stats = st;
        EM_CHECK(out->capacity == 0 || out->capacity >= n_out, MAP_EINVAL,
                 "output capacity " + std::to_string(out->capacity) + " below the pseudo count " +
                     std::to_string(n_out));
    });
}

}  // extern "C"
