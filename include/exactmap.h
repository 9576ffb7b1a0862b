/*
 * exactmap.h -- C ABI of the MI355X (gfx950) Exact-mapping library.
 *
 * The library maps SPH particles (positions, masses, smoothing lengths) onto a
 * grid of convex cells (a box-clipped Voronoi tessellation) as in Sec. II-B of
 * Lau, Petkova & Bonnell, "Hybrid Radiation Hydrodynamics scheme with gravity
 * tree-based adaptive optimization algorithm" (arXiv 2404.17084), Eq. (1)-(3):
 *
 *     f_ai  = integral over cell V_i of W(|r - r_a|, h_a) dV      (per pair)
 *     S_a   = sum_i f_ai                                            (per particle)
 *     M_i   = sum_a m_a f_ai / S_a,   rho_i = M_i / V_i             (per cell)
 *
 * W is the M4 cubic spline with support 2h (Sec. III-C, III-D).  A pair (a, i)
 * exists iff the distance from r_a to the closed cell i is strictly below 2h_a.
 * The integral is evaluated in closed form as a signed sum over vertex
 * pyramids (particle apex, one cell wall as base, split into right triangles
 * about the particle's projection point on the wall), Sec. II-B.
 *
 * Conventions for every entry point:
 *  - Return value: MAP_OK (0) on success, a negative MAP_E* code on failure.
 *    map_last_error(ctx) then returns a NUL-terminated message owned by ctx,
 *    valid until the next call on that ctx.  Calls on one ctx are serialised
 *    by an internal mutex; different ctx objects are independent.
 *  - Pointers in the *_in structs are borrowed for the duration of the call
 *    (map_submit copies them before it returns).  mem_kind says where they
 *    live: MAP_MEM_HOST (pageable or pinned host memory) or MAP_MEM_DEVICE
 *    (device memory of ctx's device, e.g. torch data_ptr(), fully written
 *    before the call: the library does not synchronise with other streams).
 *  - All device memory used internally is owned by the library (per-ctx pool,
 *    grown on demand, released by map_shutdown).
 *  - Validation failures are reported before any device work: n < 0, bad
 *    offsets, faces with fewer than 3 vertices, vertex ids out of range ->
 *    MAP_EINVAL / MAP_EGEOM; non-finite values, h <= 0, non-unit normals ->
 *    MAP_EINVAL / MAP_EGEOM (checked on the device, before integration).
 */
#ifndef EXACTMAP_H
#define EXACTMAP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    MAP_OK = 0,
    MAP_EINVAL = -1,    /* bad argument or particle data */
    MAP_ENOMEM = -2,    /* device or host allocation failed, or job larger than the budget */
    MAP_EDEVICE = -3,   /* HIP runtime or kernel error */
    MAP_EBUSY = -4,     /* serving queue full */
    MAP_ENOTFOUND = -5, /* unknown job id */
    MAP_EGEOM = -6,     /* malformed cell geometry */
    MAP_ENUMERIC = -7,  /* non-finite result */
    MAP_ENOTSUP = -8    /* entry point switched off in this build */
};

/* Arithmetic of the per-triangle closed-form terms. */
enum {
    MAP_FP64 = 0,  /* everything in FP64 */
    MAP_MIXED = 1, /* FP64 wall distance, foot point and edge projections; FP32
                      closed-form terms accumulated in FP64; FP64 recomputation
                      of terms flagged by a conditioning test; FP64
                      normalisation and reductions */
    MAP_TABLE = 2  /* the pyramid integral read from a table (map_set_table):
                      FP64 geometry, FP32 solid angle and trilinear
                      interpolation, FP64 sums; an approximation whose error
                      is set by the table size, not a precision of the
                      closed form */
};

enum { MAP_MEM_HOST = 0, MAP_MEM_DEVICE = 1 };

typedef struct map_ctx map_ctx;

typedef struct map_config {
    int device;                /* HIP device ordinal */
    int precision;             /* MAP_FP64, MAP_MIXED or MAP_TABLE, default for map_particles */
    uint64_t hbm_budget_bytes; /* serving admission budget; 0 = 80% of free device memory */
    int max_jobs;              /* serving: jobs resident on the device at once (0 = 8) */
    int max_queue;             /* serving: jobs waiting for admission (0 = 1024) */
    const char *tune_cache_path; /* autotuner cache file (text); NULL = no cache; copied by map_init */
    int serve_timeout_ms;      /* serving: time limit of every device wait of a job (0 = 120000) */
    int serve_trace;           /* serving: nonzero = one line per job event on stderr */
    int64_t fixup_cap;         /* MAP_MIXED: capacity of the list of edge terms recomputed in
                                  FP64 (0 = n_pairs / 8 + 65536); when more edges are flagged,
                                  every pair of the call is recomputed in FP64 instead */
    double cell_tol;           /* MAP_MIXED: per-cell error budget.  Each pair carries an
                                  estimate e_ai of the error of its FP32 terms; a cell with
                                  sqrt(sum_a (m_a e_ai / S_a)^2) > cell_tol |M_i| has all its
                                  pairs recomputed in FP64 (0 = 2e-6; negative = never) */
} map_config;

/* Particles: structure of arrays, FP64. */
typedef struct map_particles_in {
    int64_t n;
    const double *xyz; /* 3n, x0 y0 z0 x1 y1 z1 ... */
    const double *m;   /* n, masses */
    const double *h;   /* n, smoothing lengths (> 0) */
    int mem_kind;
} map_particles_in;

/* Convex cells in CSR form (FP64 coordinates). */
typedef struct map_cells_in {
    int64_t n_cells;
    int64_t n_faces;
    int64_t n_face_verts;          /* length of face_vert */
    int64_t n_verts;
    const int64_t *cell_face_off;  /* n_cells+1: faces of cell i are [off[i], off[i+1]) */
    const int64_t *face_vert_off;  /* n_faces+1: slots of face j in face_vert */
    const int32_t *face_vert;      /* vertex ids, counter-clockwise seen from outside the cell */
    const double *face_plane;      /* 4 per face: outward unit normal n and c with n.x = c */
    const double *verts;           /* 3 per vertex */
    const double *cell_volume;     /* n_cells, or NULL: computed on the device */
    double box[6];                 /* xlo ylo zlo xhi yhi zhi: bounding box of all cells */
    int mem_kind;
} map_cells_in;

typedef struct map_stats {
    int64_t n_pairs;        /* exact pair set size */
    int64_t n_candidates;   /* cells tested by the exact meet test */
    int64_t n_edge_terms;   /* edge terms integrated (faces and edges inside the support) */
    int64_t n_fixup_terms;  /* MAP_MIXED: edge terms recomputed in FP64 */
    int64_t n_face_visits;  /* wall planes tested (all walls of every pair's cell) */
    int64_t n_edge_visits;  /* wall edges projected (walls closer than 2h) */
    int64_t n_moment_evals; /* closed-form evaluations (asinh, angle difference and polynomial) */
    int64_t n_quad_intervals; /* MAP_MIXED: Gauss-Legendre sub-intervals of the shell piece (4 points each
                                 in the task-batch distribution 3, 8 in distributions 0-2) */
    int64_t n_angle_evals;  /* angles of edge parts beyond the support or with a piece correction */
    int64_t n_quad_points;  /* Gauss-Legendre points of the shell quadrature (mixed path) */
    int64_t n_boundary_pairs; /* pairs whose particle lies on two or more wall planes of the cell
                                 (an edge or a vertex): winding weight recomputed in FP64 */
    int64_t n_fp64_cells;   /* MAP_MIXED: cells over the error budget (cfg->cell_tol) */
    int64_t n_fp64_pairs;   /* MAP_MIXED: their pairs, recomputed in FP64 */
    double mass_in;         /* sum of m_a */
    double mass_out;        /* sum of M_i */
    double max_abs_S_minus_1; /* over particles whose support lies inside box */
    double ms_setup;        /* device time: validation and geometry tables */
    double ms_pairs;        /* device time: pair search and cell ordering */
    double ms_integrate;    /* device time: the integration kernel(s) */
    double ms_fixup;        /* device time: FP64 recomputation of flagged terms */
    double ms_reduce;       /* device time: S_a, normalisation, M_i, rho_i */
    double ms_total;        /* device time of the whole call */
    double ms_queue;        /* served jobs: host time from map_submit to admission */
    double ms_latency;      /* served jobs: host time from map_submit to completion */
} map_stats;

/* Outputs: caller-owned, caller-sized, in mem_kind memory.  Any may be NULL. */
typedef struct map_out {
    double *cell_mass;     /* n_cells */
    double *cell_density;  /* n_cells */
    double *frac_sum_raw;  /* n particles: S_a before normalisation */
    double *pair_frac;     /* raw f_ai in the order map_pairs returns (cell, then particle) */
    int32_t *pair_p;       /* particle of each pair, same order */
    int32_t *pair_c;       /* cell of each pair, same order */
    int64_t pair_capacity; /* length of pair_frac / pair_p / pair_c */
    int mem_kind;
    map_stats *stats;      /* host memory; may be NULL */
} map_out;

/* Create a context on cfg->device (cfg may be NULL: device 0, FP64).
 * MAP_EDEVICE when no device is visible or when two HIP runtimes (two
 * libamdhip64 files) are mapped into the process: the library uses the
 * runtime it was loaded against, and device pointers of another runtime are
 * not valid in it.  On failure map_last_error(NULL) has the message. */
int map_init(const map_config *cfg, map_ctx **out);
/* Drain the serving loop, free all device memory and the context. */
int map_shutdown(map_ctx *ctx);
const char *map_last_error(map_ctx *ctx);
/* Change the default precision of map_particles (MAP_FP64 / MAP_MIXED / MAP_TABLE). */
int map_set_precision(map_ctx *ctx, int precision);

/*
 * Tabulated variant (Sec. II-B: the vertex-pyramid integral pre-computed and
 * interpolated).  The table holds I(r0, R0, phi) of the M4 kernel (lengths in
 * units of h) on a uniform grid of n0 x n1 x n2 nodes,
 *     r0 = 2 i / (n0 - 1),  R0 = 2 j / (n1 - 1),  phi = (pi/2) k / (n2 - 1)
 * (the last phi plane at pi/2 - 1e-12), node (i, j, k) at index
 * (i n1 + j) n2 + k, computed on the device from the FP64 closed form and
 * read in FP32 by trilinear interpolation.  Outside the grid the pyramid's
 * mass follows exactly from its triangle's solid angle: beyond r0 = 2 the
 * pyramid holds its whole cone, and beyond R0 = 2 the mass cut off by the
 * wall no longer depends on R0.  MAP_TABLE mappings assemble the cell
 * integrals from it (no FP64 fixups); S_a then deviates from 1 in the interior
 * by the table's error and the sum-to-one normalisation keeps the total mass.
 * map_set_table: each size in [8, 1024] and at most 2^27 nodes (default
 * 64 x 64 x 64); the table is rebuilt on the next MAP_TABLE mapping.
 * map_get_table: the FP64 node values of the current size (host memory,
 * n0 n1 n2 doubles; built if needed).
 */
int map_set_table(map_ctx *ctx, int n0, int n1, int n2);
int map_get_table(map_ctx *ctx, double *values);

/*
 * Launch shape of the integration kernel for one precision (the autotuner's
 * knobs): register budget as resident wavefronts per SIMD (0 = compiler
 * default; FP64 kernels 2..4, mixed kernels 4..6; the mixed task-batch
 * kernel has budgets for 2, 3 and 6), wavefronts of consecutive
 * pairs taken per queue pop (1..64), persistent workgroups of 256 threads per
 * compute unit (1..64), and the work distribution: 1 = persistent queue of
 * pair tiles, 2 = persistent queue of single-cell tiles, 3 = persistent queue
 * of pair tiles whose edge terms are run as wavefront-wide task batches, 0 =
 * one thread per pair, -1 = clear the explicit setting (back to the tuned
 * table/default).
 * Untuned default: distribution 3 for both precisions.  For a given
 * distribution, results are bitwise independent of the other knobs and of
 * scheduling.  At MAP_FP64 every distribution evaluates the same closed forms
 * and they differ by rounding only.  At MAP_MIXED they differ also in the
 * shell piece (1 <= s <= 2), integrated by Gauss-Legendre: distribution 3
 * uses 4 points on sub-intervals of at most 0.4 times the distance to the
 * integrand's branch points (and at most 2 - r0), distributions 0-2 use 8
 * points on sub-intervals of at most 0.8 times that distance; both
 * truncations are below 1e-8 of a pair fraction per sub-interval (Gauss-
 * Legendre error bound on a Bernstein ellipse), far below the FP32 rounding
 * of the terms.
 * map_get_tune reports the shape used for n_pairs pairs.
 */
int map_set_tune(map_ctx *ctx, int precision, int waves, int tile_waves, int grid_per_cu, int persistent);
int map_get_tune(map_ctx *ctx, int precision, int64_t n_pairs, int *waves, int *tile_waves, int *grid_per_cu,
                 int *persistent);

/*
 * Autotuner: builds the pair set of (p, c), times every candidate launch shape
 * of the integration kernel at the given precision on the device, and stores
 * the fastest for the pair count's size class (and in cfg->tune_cache_path,
 * one line per entry, when set; the file is read back by map_init).  best[4]
 * receives (waves, tile_waves, grid_per_cu, persistent); *best_ms the
 * integration time of that shape.  Either may be NULL.
 */
int map_autotune(map_ctx *ctx, const map_particles_in *p, const map_cells_in *c, int precision, int *best,
                 double *best_ms);

/*
 * Pair set of Sec. II-B: every (particle a, cell i) with dist(r_a, cell i) < 2h_a,
 * sorted by cell, then by particle.  Count-then-fill: with pair_p/pair_c NULL
 * only *n_pairs is written; otherwise up to capacity pairs are written (host
 * memory) and *n_pairs is the full count.
 */
int map_pairs(map_ctx *ctx, const map_particles_in *p, const map_cells_in *c, int64_t *n_pairs,
              int32_t *pair_p, int32_t *pair_c, int64_t capacity);

/* Synchronous Exact mapping, Eq. (1)-(3) with sum-to-one normalisation. */
int map_particles(map_ctx *ctx, const map_particles_in *p, const map_cells_in *c, map_out *out);

/*
 * map_particles without any device allocation, for callers that cannot
 * allocate device memory (code under graph capture, tight serving loops,
 * harnesses that forbid hipMalloc): the same mapping, results bitwise equal
 * to map_particles with the same launch shape, but every intermediate buffer
 * lives in one fixed 128 MiB device array that the library holds on each
 * device it runs on until the process ends (its address is looked up when a
 * context is created on the device).  Inputs and outputs must be device
 * memory (mem_kind MAP_MEM_DEVICE for p, c and out; out->stats is host
 * memory); precision MAP_FP64 or MAP_MIXED.  No hipMalloc, hipFree or other
 * allocating call is made.  All calls on one device share the array: calls
 * that overlap in time on one device (other contexts, other threads) race and
 * must not be made.  The call leaves nothing for map_back.
 * Errors: those of map_particles; MAP_EINVAL for host memory or MAP_TABLE;
 * MAP_ENOMEM when the input does not fit the array (about 10,000 Voronoi
 * cells and their particles fit; checked before any device work from the
 * geometry sizes, and again as the pair set is built).
 */
int map_particles_noalloc(map_ctx *ctx, const map_particles_in *p, const map_cells_in *c, map_out *out);

/*
 * Inverse mapping, Sec. II-B Eq. (4): particle values from cell values with
 * the pair weights of this context's last successful map_particles call,
 * normalised as in the forward mapping,
 *   q_a = sum_i q_i f_ai / S_a          (0 for a particle that meets no cell),
 * so that sum_a m_a q_a = sum_i q_i M_i (the mapped quantity's mass is kept).
 * cell_values: n_cells doubles of that mapping's cells (host or device memory,
 * mem_kind, borrowed); particle_values: n doubles written in cell-index order
 * of summation per particle (out_mem_kind; caller-owned).  The first call
 * after a mapping also builds the particle-major view of its pairs (a stable
 * sort, kept until the next call that reuses the context's workspace).
 * Errors: MAP_EINVAL when no mapping of this context can be inverted (none
 * yet, or map_pairs, map_pseudo, map_autotune or a failed map_particles ran
 * since), for NULL buffers with nonzero counts or a bad mem_kind.  Values are
 * not checked: a non-finite cell value gives non-finite particle values.
 */
int map_back(map_ctx *ctx, const double *cell_values, int mem_kind, double *particle_values, int out_mem_kind);

/*
 * Pseudo-particles (Sec. III): the gravity-tree front end that lowers the
 * resolution away from the ionising sources before the mapping.
 *
 *  Tree (Sec. III-A): an octree over 63-bit Morton keys of the positions in
 *  `box` (21 bits per axis, key = floor((x - lo) / extent * 2^21) per axis,
 *  clamped, octal digits (x, y, z) from the most significant).  A node holds
 *  the particles sharing its first L digits and is a leaf when it holds at
 *  most leaf_size particles or L = 21.  Node position = centre of mass, size s
 *  = distance from it to the furthest member.  Node label = (1 << 3L) | prefix
 *  (ancestor k levels up = label >> 3k).
 *  Walk (Sec. III-B, Eq. (5)): r = smallest distance from the node's centre of
 *  mass to the sources; a node "comes within" R when r - s < R.  A leaf within
 *  r_part is replaced by its particles; any other node within r_part or r_leaf
 *  is opened; otherwise a node is opened when s > theta * r; a leaf is never
 *  opened otherwise.  Accepted nodes and extracted particles partition the
 *  particles (mass is conserved).
 *  Smoothing lengths (Sec. III-C, Eq. (7)-(9)): a node pseudo-particle's h is
 *  the unique root of (1/pi) sum_b w(|r - r_b| / h) = h_fact_node^3 (that is,
 *  h = h_fact_node n^(-1/3)), the sum running over the node pseudo-particles
 *  and, standing in for extracted particles, the leaves they came from; the
 *  node itself is included.  Newton steps safeguarded by bisection from the
 *  initial guess h0 = 2 h_fact_node s (zero-size nodes: their particles'
 *  largest h); h0 itself when there is no root.  Extracted particles keep
 *  their own h.
 *
 * Output: pseudo-particles in Morton order of their first particle.  Per
 * pseudo-particle: position (3 doubles), mass, h, size s (0 for particles),
 * kind (MAP_PSEUDO_NODE / MAP_PSEUDO_PARTICLE) and ref (the node label, or the
 * particle's index in the input).  out->n_out is always set; when
 * out->capacity < n_out nothing else is written and the call returns MAP_OK if
 * capacity == 0 (count only) or MAP_EINVAL otherwise.  capacity >= p->n always
 * suffices.  Output buffers live in out->mem_kind memory.  Sources src_xyz
 * (3 * n_src doubles, 1 <= n_src <= 64) are host memory.
 * Errors: MAP_EINVAL for n < 0 or n >= 2^31, non-finite or non-positive
 * masses or h, non-finite positions, a box without positive extent, theta,
 * r_part or r_leaf negative or non-finite, leaf_size outside [1, 64],
 * h_fact_node <= 0.
 */
enum { MAP_PSEUDO_NODE = 0, MAP_PSEUDO_PARTICLE = 1 };
typedef struct map_pseudo_params {
    double theta;       /* opening angle of Eq. (5) */
    double r_part;      /* leaves within r_part of a source become their particles */
    double r_leaf;      /* nodes within r_leaf of a source are opened down to leaves */
    int leaf_size;      /* maximum particles per leaf (the paper's tree stops below 10) */
    double h_fact_node; /* h_fact of Eq. (7) and (9), 1.1 in the paper */
} map_pseudo_params;

typedef struct map_pseudo_stats {
    int64_t n_tree_nodes, n_leaves, max_level;
    int64_t n_pseudo, n_pseudo_nodes, n_particles, n_substitute_leaves;
    int64_t n_fallbacks;     /* node h taken from Eq. (9) because no root exists */
    int64_t n_h_evals;       /* evaluations of the number sum over all nodes */
    int64_t n_neighbours;    /* points within 2h of the nodes, summed */
    double ms_tree, ms_walk, ms_hsolve, ms_total;
} map_pseudo_stats;

typedef struct map_pseudo_out {
    int64_t capacity;
    double *xyz;      /* 3 * capacity */
    double *m, *h, *size;
    int32_t *kind;
    int64_t *ref;
    int mem_kind;
    int64_t n_out;    /* written by the call */
    map_pseudo_stats *stats; /* host memory, may be NULL */
} map_pseudo_out;

int map_pseudo(map_ctx *ctx, const map_particles_in *p, const double box[6], const double *src_xyz, int n_src,
               const map_pseudo_params *par, map_pseudo_out *out);

/*
 * Adaptive tree walk (Sec. III-B, Eq. (6)): pseudo-particles refined until
 * every node pseudo-particle is resolved for the neutral fractions that the
 * radiative transfer returns for it.
 *
 * The tree is built once; then walk after walk: the walk of map_pseudo, with
 * internal nodes also opened when their label failed an earlier walk of this
 * call or when they come within a remembered region (below); node smoothing
 * lengths; `neutral` is called with the set (host memory, valid during the
 * call) and fills the neutral fraction of each pseudo-particle; the check of
 * Eq. (6): a node pseudo-particle of size s > 0 fails when
 *     f_neu < f_neu,limit = (K - s_root / s) / K,
 * s_root being the root node's size (extracted particles and zero-size nodes
 * are not checked).  Failing internal nodes are opened in the next walk; when
 * a leaf fails, r_part grows to (1 + 2^-30) times the largest r - s among the
 * failing leaves (r: the leaf's distance to the nearest source), so that each
 * of them is extracted, and r_leaf by the same factor (to at least r_part when
 * r_part was 0).  The walks stop at the first set that passes or after
 * max_walks walks; `out` receives the last set (as map_pseudo; out->capacity
 * must be at least its count, and p->n always suffices).
 *
 * Remembered regions (the memory across steps): the context keeps a list of
 * regions, 5 doubles each (centre x, y, z, radius R, smallest descendant size
 * s_min).  A node "comes within" a region when |com - c| - s < R and is then
 * opened while s > s_min (leaves only by r_part).  At the end of the call a
 * region is dropped when no pseudo-particle of the final set lies inside it
 * (|x - c| < R) or when the smallest neutral fraction inside is at least the
 * limit of Eq. (6) for a node of size R (the node it stands for would pass:
 * it has become shielded), and every node that failed during the call adds a
 * region: its centre of mass, its size, and the smallest size among the
 * final set's node pseudo-particles that descend from it (0 if none).  The
 * list is read and replaced with map_get_regions / map_set_regions (at most
 * MAP_MAX_REGIONS regions; the call fails with MAP_ENOMEM beyond).
 *
 * `neutral` must not call into the library with the same context.  A nonzero
 * return from it stops the call with MAP_EINVAL (regions unchanged).
 * Errors: those of map_pseudo; MAP_EINVAL for K <= 0 or non-finite, max_walks
 * < 1, a NULL callback, or neutral fractions that are not finite.
 */
typedef int (*map_neutral_fn)(void *user, int64_t n_pseudo, const double *xyz, const double *m, const double *h,
                              const double *size, const int32_t *kind, double *f_neu);

typedef struct map_adapt_params {
    double K;               /* Eq. (6); 100 in the paper's runs */
    int max_walks;          /* walks per call, >= 1 */
    map_neutral_fn neutral; /* the radiative-transfer step */
    void *user;             /* passed to neutral */
} map_adapt_params;

typedef struct map_adapt_stats {
    int64_t n_walks;           /* walks run (1: the first set passed) */
    int64_t converged;         /* 1 when the last set passed */
    int64_t n_failed;          /* node pseudo-particles that failed, over all walks */
    int64_t n_r_part_growths;  /* walks after which r_part grew */
    int64_t n_regions_in, n_regions_dropped, n_regions_out;
    double r_part, r_leaf;     /* radii for a next walk: those of the last walk, grown if a leaf failed in it */
    double s_root;             /* size of the root node */
    double ms_tree;            /* tree build (device) */
    double ms_walks;           /* walks, smoothing lengths and checks (host clock, callback excluded) */
    double ms_callback;        /* time spent in `neutral` */
    double ms_total;           /* the whole call (host clock) */
} map_adapt_stats;

#define MAP_MAX_REGIONS 1048576
int map_pseudo_adaptive(map_ctx *ctx, const map_particles_in *p, const double box[6], const double *src_xyz,
                        int n_src, const map_pseudo_params *par, const map_adapt_params *ap, map_pseudo_out *out,
                        map_adapt_stats *stats);
/* Count-then-fill read of the context's regions (host memory, 5 doubles each):
 * *n_regions is always set; regions are written when capacity >= *n_regions. */
int map_get_regions(map_ctx *ctx, int64_t capacity, double *regions, int64_t *n_regions);
/* Replaces the context's regions (host memory; n_regions = 0 clears them).
 * MAP_EINVAL for non-finite values, R <= 0 or s_min < 0; MAP_ENOMEM beyond
 * MAP_MAX_REGIONS. */
int map_set_regions(map_ctx *ctx, int64_t n_regions, const double *regions);

/*
 * Voronoi grid (Sec. II-A): the box-clipped Voronoi cells of n sites (the
 * particle positions, or any points in the box), with tightly packed sites
 * merged and lloyd_iters Lloyd iterations (each site moved to its cell's
 * centroid, the grid rebuilt; the paper applies 5).  Merging (merge_dist > 0):
 * a site is dropped when a site of lower index lies closer than merge_dist
 * (coinciding sites included); the grid is built from the rest, in input
 * order, and site_cell[i] names the cell that holds input site i (its
 * nearest grid site, ties to the lower index; after Lloyd steps a site may lie
 * in a neighbour's cell).  Without merging cell i belongs to site i.  Each cell is
 * the box cut by the bisector planes of its nearest sites, taken nearest
 * first until no farther site can reach it; a vertex within 1e-12 of a
 * cutting plane counts as on it.  Output in the cell format of
 * map_cells_in: faces counter-clockwise about outward unit normals (n.x = c),
 * vertices per cell (shared by its faces), volumes; plus the site or wall
 * across each face (-1 - w for walls x-, x+, y-, y+, z-, z+), the sites after
 * the Lloyd iterations and the cell centroids.
 * The arrays are device memory owned by the context (out->cells has mem_kind
 * MAP_MEM_DEVICE and can be passed to map_particles as it is), valid until the
 * next map_voronoi or map_shutdown; map_voronoi_copy copies them into caller
 * buffers (NULL skips an array) sized by the counts in out.
 * sites: 3 n doubles in mem_kind memory.  Errors: MAP_EINVAL for n < 1, a
 * site outside the box or not finite, two coinciding sites when merge_dist
 * is 0, lloyd_iters outside [0, 1000], merge_dist negative or not finite;
 * MAP_EDEVICE for a cell with more than 64 faces or 128 vertices.  Uses
 * about 7 kB of device memory per site while building (a 5.9 kB record per
 * cell, released when the grid is done).
 */
typedef struct map_voronoi_out {
    int64_t n_cells, n_faces, n_face_verts, n_verts;
    map_cells_in cells;        /* device memory owned by the context */
    const int64_t *face_nb;    /* n_faces */
    const double *sites;       /* 3 n_cells: the sites of the cells */
    const double *centroid;    /* 3 n_cells */
    int64_t n_sites;           /* input sites */
    const int64_t *site_cell;  /* n_sites: the cell holding each input site */
    double ms;                 /* device time of the call */
} map_voronoi_out;
int map_voronoi(map_ctx *ctx, int64_t n, const double *sites, int mem_kind, const double box[6], int lloyd_iters,
                double merge_dist, map_voronoi_out *out);
int map_voronoi_copy(map_ctx *ctx, int mem_kind, int64_t *cell_face_off, int64_t *face_vert_off, int32_t *face_vert,
                     double *face_plane, int64_t *face_nb, double *verts, double *cell_volume, double *centroid,
                     double *sites, int64_t *site_cell);

/*
 * Served mapping (continuous batching; not in the paper, whose mapping runs
 * once per hydro step).  map_submit queues one mapping job at the context's
 * current precision (MAP_FP64 or MAP_MIXED) and returns at once; *job_id
 * identifies it.  Host inputs are copied before map_submit returns; device
 * inputs (mem_kind MAP_MEM_DEVICE) are borrowed, like the outputs: they must
 * stay valid and unchanged until map_poll reports the job finished.
 * Jobs are admitted in submission order while a slot (cfg->max_jobs) and
 * device memory (cfg->hbm_budget_bytes bounds the estimated footprint of the
 * jobs in flight) are free; an admitted job's geometry stays resident on the
 * device until it completes.  Each slot keeps its grow-only buffers from one
 * job to the next (memory held: at most max_jobs times the largest job's
 * buffers, returned at map_shutdown).  One scheduler thread per context makes
 * all the device calls, in rounds: it builds the pair set of every admitted
 * job, integrates all of them in one persistent launch of the task-batch
 * kernel (a table of the jobs), builds the pair sets of the jobs admitted
 * meanwhile while that launch runs, and finishes the launch's jobs
 * (fixups, reductions, outputs) before the next launch; jobs arriving while
 * others integrate join the next launch.  A job's results are bitwise those
 * of map_particles on the same inputs with the default launch shape, alone or
 * in any mix.
 * The out buffers (and out->stats) are caller-owned and must stay valid until
 * map_poll reports MAP_JOB_DONE or MAP_JOB_FAILED.
 * Errors at submit: MAP_EINVAL/MAP_EGEOM (malformed input), MAP_ENOMEM (job
 * larger than the whole budget), MAP_EBUSY (queue holds cfg->max_queue jobs,
 * or the context is shutting down), MAP_EDEVICE (serving stopped after a
 * device failure).  A job that fails later does not affect the others.  Every
 * device wait of the served path is bounded by cfg->serve_timeout_ms; when
 * one runs out, the jobs in flight and all later ones fail with MAP_EDEVICE
 * (the device cannot be trusted any more) and map_shutdown returns
 * MAP_EDEVICE, leaving the context's memory in place.
 */
enum { MAP_JOB_PENDING = 0, MAP_JOB_RUNNING = 1, MAP_JOB_DONE = 2, MAP_JOB_FAILED = 3 };
int map_submit(map_ctx *ctx, const map_particles_in *p, const map_cells_in *c, map_out *out, uint64_t *job_id);
/*
 * Waits up to timeout_us microseconds (0: no wait, negative: until finished,
 * but at most twice cfg->serve_timeout_ms plus 5 s, after which MAP_EDEVICE
 * is returned with the job still running) and writes the job's state.  Once DONE or FAILED has been reported the job
 * is forgotten (a later poll returns MAP_ENOTFOUND).  For a failed job the
 * return value is the job's error code and map_last_error has its message.
 */
int map_poll(map_ctx *ctx, uint64_t job_id, int64_t timeout_us, int *state);

#ifdef __cplusplus
}
#endif

#endif /* EXACTMAP_H */
