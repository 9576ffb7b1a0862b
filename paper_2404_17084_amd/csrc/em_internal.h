// Internal declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <atomic>
#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/exactmap.h"

namespace em {

// ---------------------------------------------------------------- errors
struct Error {
    int code;
    std::string msg;
};

#define EM_HIP(expr)                                                                          \
    do {                                                                                      \
        hipError_t _e = (expr);                                                               \
        if (_e != hipSuccess)                                                                 \
            throw ::em::Error{MAP_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(_e)}; \
    } while (0)

#define EM_CHECK(cond, code, msg)                  \
    do {                                           \
        if (!(cond)) throw ::em::Error{(code), (msg)}; \
    } while (0)

// ---------------------------------------------------------------- device memory
// A grow-only set of device buffers.  get() returns a buffer of at least
// `bytes`, reallocating (and discarding contents) when it is too small.
// get() and release() belong to the owning thread; bytes_held() may be read
// from any thread (the slot table is sized once and never reallocated).
//
// Arena mode (use_arena): get() hands out 256-byte aligned pieces of one
// fixed device buffer instead, a slot that needs more than its piece getting
// a new piece further on; it never allocates or frees device memory and
// throws MAP_ENOMEM when the buffer is used up.
class Workspace {
public:
    explicit Workspace(int device);
    ~Workspace();
    Workspace(const Workspace &) = delete;
    Workspace &operator=(const Workspace &) = delete;

    void *get(int slot, size_t bytes);
    template <typename T>
    T *get(int slot, size_t count) { return static_cast<T *>(get(slot, count * sizeof(T))); }
    size_t bytes_held() const;
    void release();
    // frees one slot's buffer (not in arena mode, where it stays reserved)
    void drop(int slot);
    void use_arena(void *base, size_t bytes);
    // Stream-ordered mode: buffers come from the device's memory pool with
    // hipMallocAsync / hipFreeAsync on stream s (no device-wide
    // synchronisation when a buffer is replaced or released).
    void use_stream(hipStream_t s) { stream_ = s; }
    bool is_arena() const { return arena_base_ != nullptr; }
    // bytes still free in arena mode (SIZE_MAX otherwise)
    size_t arena_free() const;
    size_t arena_used() const { return arena_used_; }

private:
    struct Buf {
        void *p = nullptr;
        size_t cap = 0;
    };
    int device_;
    std::vector<Buf> bufs_;
    std::atomic<size_t> held_{0};
    char *arena_base_ = nullptr;
    size_t arena_cap_ = 0, arena_used_ = 0;
    hipStream_t stream_ = nullptr;
};

// Buffer slots of one mapping job.
enum Slot : int {
    S_XYZ, S_M, S_H,
    S_CFO, S_FVO, S_FV, S_PLANE, S_VERTS, S_VOL,
    S_EDGE, S_AABB, S_CBIN,
    S_FLAGS, S_COUNTERS,
    S_BINCNT, S_BINOFF, S_BINKEY, S_BINVAL, S_BINKEY2, S_BINVAL2, S_BINLIST, S_BINCNT64, S_BINOFF_G,
    S_PCNT, S_POFF, S_PC_PM, S_PP_PM, S_IOTA,
    S_KEY2, S_PERM, S_PAIR_C, S_PAIR_P, S_CCNT, S_CCNT64, S_COFF,
    S_F, S_F_PM, S_S, S_MCELL, S_RHO, S_RED,
    S_FIX_ITEMS, S_FIX_VALS, S_FIX_KEY2, S_FIX_VAL2,
    S_SCAN_TMP, S_SORT_HIST, S_TILE_CTR, S_TILE_CNT, S_TILE_OFF, S_TILES,
    S_CAND_BUF, S_CAND_MAX, S_PBOX, S_NCNT, S_NOFF, S_QCNT, S_ECNT, S_PCNT2, S_BACK_IN, S_BACK_OUT,
    S_PSEUDO0, S_PSEUDO1, S_PSEUDO2, S_PSEUDO3, S_PSEUDO4, S_PSEUDO5, S_PSEUDO6, S_PSEUDO7,
    S_PSEUDO8, S_PSEUDO9, S_PSEUDO10, S_PSEUDO11, S_PSEUDO12, S_PSEUDO13, S_PSEUDO14, S_PSEUDO15,
    S_ADAPT0, S_ADAPT1, S_ADAPT2, S_ADAPT3, S_ADAPT4, S_ADAPT5, S_ADAPT6, S_ADAPT7,
    S_VOR0, S_VOR1, S_VOR2, S_VOR3, S_VOR4, S_VOR5, S_VOR6, S_VOR7, S_VOR8, S_VOR9, S_VOR10, S_VOR11, S_VOR12,
    S_VOR13, S_VOR14,
    S_ERR, S_CHECK,
    S_NUM_SLOTS
};

// Default per-cell error budget of the mixed path (relative to the cell's mass).
constexpr double kDefaultCellTol = 2e-6;

// Size of the fixed device scratch array of map_particles_noalloc (em_noalloc.hip).
constexpr size_t kNoallocScratchBytes = size_t(128) << 20;
// Looks up (once per device; the device must be current) the device address
// of that array.
void noalloc_attach(int device);

// ---------------------------------------------------------------- geometry records
// One directed wall edge v_k -> v_{k+1} of a face (slot of face_vert):
// start vertex v, unit direction e, in-plane inward normal m = n x e, length L.
struct alignas(16) EdgeRec {
    double vx, vy, vz, L;
    double ex, ey, ez, mx;
    double my, mz;
};
static_assert(sizeof(EdgeRec) == 80, "edge record layout");

// Validation flag bits (device-side checks)
enum : unsigned {
    F_PART_NONFINITE = 1u << 0,
    F_H_NONPOS = 1u << 1,
    F_M_BAD = 1u << 2,
    F_CFO_BAD = 1u << 3,
    F_FVO_BAD = 1u << 4,
    F_FACE_SMALL = 1u << 5,
    F_VID_RANGE = 1u << 6,
    F_PLANE_BAD = 1u << 7,
    F_VERT_NONFINITE = 1u << 8,
    F_VOL_BAD = 1u << 9,
    F_RESULT_NONFINITE = 1u << 10,
};

// Counters written by kernels (int64 each)
enum : int {
    C_CANDIDATES = 0,
    C_EDGE_TERMS = 1,
    C_FIXUPS = 2,
    C_FACES = 3,
    C_EDGES = 4,
    C_MOMENTS = 5,
    C_QUADS = 6,
    C_ANGLES = 7,
    C_QPOINTS = 8,
    C_WINDING = 9,  // pairs whose winding weight was recomputed (particle on two or more wall planes)
    C_FP64_PAIRS = 10,  // mixed path: pairs recomputed in FP64 because their cell's error estimate was too large
    C_NUM = 11
};

// Device-resident view of one job's inputs.
struct DevInputs {
    int64_t n = 0;
    const double *xyz = nullptr, *m = nullptr, *h = nullptr;
    int64_t n_cells = 0, n_faces = 0, n_face_verts = 0, n_verts = 0;
    const int64_t *cfo = nullptr, *fvo = nullptr;
    const int32_t *fv = nullptr;
    const double *plane = nullptr, *verts = nullptr, *vol = nullptr;
    double box[6] = {0, 0, 0, 1, 1, 1};
};

// Launch tuning of the integration kernel.
struct IntegrateTune {
    int block = 256;       // threads per workgroup
    int tile_waves = 1;    // wavefronts of pairs per tile taken from the queue
    int grid_per_cu = 8;   // persistent workgroups per compute unit
    int persistent = 1;    // 2: persistent queue of cell tiles, 1: persistent queue of pair tiles,
                           // 0: one thread per pair
    int waves = 0;         // register budget as waves per SIMD (FP64: 2-4, mixed: 4-6; 0 = lowest)
};

// ---------------------------------------------------------------- primitives (em_primitives.hip)
// Exclusive scan of int64 counts: out[0] = 0, out[i+1] = out[i] + in[i]; out has n+1 entries.
void scan_counts(Workspace &ws, const int64_t *in, int64_t *out, int64_t n, hipStream_t s);
// Stable LSD radix sort by the low `bits` bits of 32-bit keys, carrying 32-bit values.
// Results end in (keys, vals); (keys2, vals2) are scratch of the same size.
void radix_sort_u32(Workspace &ws, uint32_t *keys, uint32_t *vals, uint32_t *keys2, uint32_t *vals2, int64_t n,
                    int bits, hipStream_t s);
// The same for 64-bit keys.
void radix_sort_u64(Workspace &ws, uint64_t *keys, uint32_t *vals, uint64_t *keys2, uint32_t *vals2, int64_t n,
                    int bits, hipStream_t s);
void fill_iota_u32(uint32_t *p, int64_t n, hipStream_t s);
void fill_iota_i64(int64_t *p, int64_t n, hipStream_t s);
// Waits until the work queued on stream s has finished.  On a thread that set
// a wait limit (set_wait_limit_ms > 0; the serving thread does) the wait polls
// and throws MAP_EDEVICE with a message containing kWaitLimitText once the
// limit has passed; otherwise it is hipStreamSynchronize.
void stream_sync(hipStream_t s);
void set_wait_limit_ms(double ms);
constexpr const char *kWaitLimitText = "device work did not finish within the wait limit";
void fill_zero_bytes(void *p, size_t bytes, hipStream_t s);
int device_cu_count();

// ---------------------------------------------------------------- stages
// em_geometry.hip
void launch_validate(const DevInputs &in, unsigned *flags, hipStream_t s);
void launch_geometry(const DevInputs &in, EdgeRec *edges, double *aabb, double *vol_out, hipStream_t s);

// em_pairs.hip: builds the cell-ordered pair set; returns the pair count.
struct PairSet {
    int64_t n_pairs = 0;
    const uint32_t *pair_c = nullptr;  // cell-major order
    const uint32_t *pair_p = nullptr;
    const int64_t *coff = nullptr;     // cell-major offsets (n_cells+1)
    const uint64_t *tiles = nullptr;   // cell tiles of <= 64 pairs (cell << 32 | index)
    int64_t n_tiles = 0;
};
PairSet build_pairs(Workspace &ws, const DevInputs &in, const double *aabb, const EdgeRec *edges,
                    int64_t *counters, hipStream_t s);
// Particle-major view of cell-major pairs: perm (particle-major position ->
// cell-major index, cells ascending within a particle) and poff (n+1).
void build_particle_view(Workspace &ws, const uint32_t *pair_p, int64_t n_pairs, int64_t n, uint32_t *perm,
                         int64_t *poff, hipStream_t s);
// Inverse mapping: q_part[a] = sum over a's pairs of q_cell[c] f / S_a (0 when S_a = 0).
void launch_map_back(int64_t n, const int64_t *poff, const uint32_t *perm, const uint32_t *pair_c, const double *f,
                     const double *S, const double *q_cell, double *q_part, hipStream_t s);

// em_pseudo.hip: pseudo-particle front end (tree, walk, node smoothing lengths).
struct DevParticles {
    int64_t n = 0;
    const double *xyz = nullptr, *m = nullptr, *h = nullptr;
};
struct PseudoDest {
    int64_t capacity = 0;
    double *xyz = nullptr, *m = nullptr, *h = nullptr, *size = nullptr;
    int32_t *kind = nullptr;
    int64_t *ref = nullptr;
    int mem_kind = MAP_MEM_HOST;
};
// Returns the pseudo count; writes the outputs when dest.capacity suffices.
// ev (optional): 4 events recorded at start, after the tree, after the walk
// and after the h-solve.
int64_t run_pseudo(Workspace &ws, const DevParticles &p, const double box[6], const double *src, int n_src,
                   const map_pseudo_params &par, const PseudoDest &dest, map_pseudo_stats *st, hipStream_t s,
                   hipEvent_t *ev);
// Adaptive walk (Sec. III-B, Eq. (6)): walks until the set passes the check or
// ap.max_walks walks ran; `regions` (5 doubles each) is read and replaced.
// ev: at least 2 events (tree timing).  Returns the count of the last set.
int64_t run_pseudo_adaptive(Workspace &ws, const DevParticles &p, const double box[6], const double *src, int n_src,
                            const map_pseudo_params &par, const map_adapt_params &ap, std::vector<double> &regions,
                            const PseudoDest &dest, map_pseudo_stats *st, map_adapt_stats *ast, hipStream_t s,
                            hipEvent_t *ev);

// One job of an integration launch of the task-batch kernels: its pairs
// (cell-major), inputs, geometry tables and outputs.  tile_base is the job's
// first tile (64 pairs each) in the launch's tile space, the running sum of
// the tiles of the jobs before it.
struct IntJob {
    int64_t np = 0;
    int64_t tile_base = 0;
    const uint32_t *pair_p = nullptr, *pair_c = nullptr;
    const double *xyz = nullptr, *h = nullptr;
    const int64_t *cfo = nullptr, *fvo = nullptr;
    const double *plane = nullptr;
    const EdgeRec *edges = nullptr;
    double *f = nullptr;
    float *err = nullptr;  // mixed path: FP32 error estimate per pair (units of f)
    unsigned long long *counters = nullptr;
    unsigned *fix_count = nullptr;
    uint64_t *fix_items = nullptr;
    unsigned fix_cap = 0;
};
// Kernel argument: one job by value (n = 1) or a device table of n jobs.
struct JobsArg {
    const IntJob *table;
    int n;
    int64_t n_tiles;
    IntJob one;
};
// One persistent launch of the task-batch kernel (distribution 3) of
// `precision` over n_jobs jobs: h_jobs is the host table (checked: tile bases
// are the running tile counts), d_jobs its device copy (needed when
// n_jobs > 1, read by the kernel).  tile_ctr: 24 counters of the launch,
// zeroed here.  A pair's result does not depend on the other jobs.
void launch_integrate_jobs(const IntJob *h_jobs, const IntJob *d_jobs, int n_jobs, int precision,
                           const IntegrateTune &tune, unsigned *tile_ctr, hipStream_t s);

// em_integrate.hip: raw f per pair (cell-major order).
void build_tiles(Workspace &ws, const DevInputs &in, PairSet &ps, hipStream_t s);
// err: MAP_MIXED: per-pair FP32 error estimates (units of f) are written there
// (may be null; ignored for MAP_FP64).
void launch_integrate(const DevInputs &in, const EdgeRec *edges, const PairSet &ps, int precision,
                      const IntegrateTune &tune, double *f, float *err, int64_t *counters, uint32_t *tile_ctr,
                      uint64_t *fix_items, int64_t fix_cap, hipStream_t s);
// FP64 recomputation (the whole pair, winding weight included) of every pair
// of the n_cells listed cells, written over f; counters[C_FP64_PAIRS] counts them.
void launch_recompute_cells(const DevInputs &in, const EdgeRec *edges, const PairSet &ps, const uint32_t *cells,
                            int64_t n_cells, double *f, int64_t *counters, hipStream_t s);
// FP64 values of the fixup items: flagged edge terms, and the winding
// correction of pairs whose particle lies on two or more wall planes of the
// cell (counted in counters[C_WINDING]).
void launch_fixup(const DevInputs &in, const EdgeRec *edges, const PairSet &ps, const uint64_t *fix_items,
                  int64_t n_fix, double *fix_vals, int64_t *counters, hipStream_t s);
// adds sorted fixup values into f
void launch_fixup_apply(const uint64_t *keys, const double *vals, int64_t n_fix, double *f, hipStream_t s);

// em_integrate.hip: node values of the tabulated pyramid integral (FP64 and FP32 copies)
void launch_table_build(int n0, int n1, int n2, double *tab64, float *tab32, hipStream_t s);
// em_table.hip: raw f per pair through the table (cell-major order)
void launch_integrate_table(const DevInputs &in, const EdgeRec *edges, const PairSet &ps, const float *tab, int n0,
                            int n1, int n2, double *f, int64_t *counters, hipStream_t s);

// em_voronoi.hip: the box-clipped Voronoi grid of a site set, in the cell
// format of map_cells_in, in device buffers owned by the context
struct VorGrid {
    int64_t n = 0, n_faces = 0, n_slots = 0, n_verts = 0;
    int64_t *cfo = nullptr, *fvo = nullptr, *fnb = nullptr;
    int32_t *fv = nullptr;
    double *plane = nullptr, *verts = nullptr, *vol = nullptr, *cen = nullptr, *sites = nullptr;
    double *input = nullptr;      // the call's input sites (3 n_in)
    int64_t *site_cell = nullptr; // cell holding each input site (n_in)
    int64_t n_in = 0;
    size_t cap_cells = 0, cap_vol = 0, cap_cen = 0, cap_fvo = 0, cap_fnb = 0, cap_plane = 0, cap_fv = 0,
           cap_verts = 0, cap_sites = 0, cap_input = 0, cap_site_cell = 0;
};
void build_voronoi(Workspace &ws, VorGrid &V, int64_t n, const double *sites, const double box[6], hipStream_t s);
// merging of tightly packed sites; returns the number kept (written to out, input order)
int64_t merge_sites(Workspace &ws, int64_t n_in, const double *in, const double box[6], double d, double *out,
                    hipStream_t s);
// the cell of grid V holding each input point (its nearest site, ties to the lower index)
void site_cells(Workspace &ws, const VorGrid &V, int64_t n_in, const double *in, const double box[6],
                int64_t *site_cell, hipStream_t s);
void free_voronoi(VorGrid &V);

// em_reduce.hip
void launch_reduce(const DevInputs &in, const PairSet &ps, const double *f, double *S, double *M,
                   double *rho, double *red, unsigned *flags, hipStream_t s);
// Mixed path, before the reduction: lists the cells whose estimated FP32
// error, sqrt(sum over their pairs of (m_a err_ai)^2), exceeds tol times their
// raw mass |sum m_a f_ai| (count in *count, at most cap cells listed; count
// may exceed cap).
void launch_cell_check(const DevInputs &in, const PairSet &ps, const float *err, const double *f, double tol,
                       unsigned *count, uint32_t *list, int64_t cap, hipStream_t s);

}  // namespace em
