/*
 * gp.h -- C ABI of the MI355X refinement library for grid-filtered spatial joins.
 *
 * The library computes the two refinement operations of Zhang & You, "Large-Scale
 * Geospatial Processing on Multi-Core and Many-Core Processors" (arXiv 1403.0802):
 *
 *   PIP  (Sec. III.C, Fig. 3): for each point, the polygon that contains it, by the
 *        even-odd ray-crossing rule over every ring (outer ring and holes).
 *   P2P  (Sec. III.B, Fig. 2): for each point, the nearest polyline within range D,
 *        where a polyline's distance is the minimum point-segment distance over its
 *        segments (perpendicular distance when the projection falls on the segment,
 *        else the nearer endpoint).
 *
 * Both sit behind the paper's filter (Sec. III.A): a uniform grid pairs each point
 * cell with the features whose MBB (expanded by D for P2P) touches that cell, and
 * only those (cell, {feature}) pairs are refined.
 *
 * Exact definitions used by the library (the paper leaves these open):
 *   - Grid: cell = (floor((x-x0)/cs), floor((y-y0)/cs)), row-major id cy*nx+cx; a
 *     point outside [0,nx)x[0,ny) or with a non-finite coordinate is unpaired.
 *     Each MBB is padded by cs*2^-20 on every side (after the +-D expansion for
 *     P2P) before it is rasterised; cells are clamped to the grid.
 *   - PIP crossing of edge (a,b): none if a.y == b.y; else with lo/hi the lower and
 *     upper endpoint, lo.y <= p.y < hi.y and
 *     (p.x-lo.x)*(hi.y-lo.y) < (hi.x-lo.x)*(p.y-lo.y), each product rounded once.
 *     A point takes the SMALLEST polygon id with odd crossing parity, else -1.
 *   - P2P segment distance: dx=b.x-a.x, dy=b.y-a.y, wx=p.x-a.x, wy=p.y-a.y,
 *     L2=dx*dx+dy*dy, t=wx*dx+wy*dy; t<=0: wx*wx+wy*wy; t>=L2: |p-b|^2;
 *     else (wx*dy-wy*dx)^2/L2.  A point takes the polyline with the smallest d^2
 *     among those with d^2 <= D*D (ties: smallest id) and distance sqrt(d^2); with
 *     no such polyline, id -1 and distance +inf.
 *
 * Precision forms:
 *   GP_FP64  every test in FP64 with exactly the operation order above (results are
 *            bitwise reproducible against a scalar FP64 implementation).
 *   GP_MIXED tests in FP32 on coordinates rebased to each grid cell's centre, with a
 *            per-edge guard band; any point whose FP32 decision could differ from the
 *            FP64 one is recomputed in FP64 on the GPU.  PIP ids, P2P ids and P2P
 *            distances are identical to GP_FP64: the winning polylines' distances are
 *            always evaluated in FP64, in the operation order above.
 *
 * Conventions:
 *   - All calls return a gp_status; 0 is success.  gp_last_error() returns a
 *     thread-local message for the last failing call on the calling thread.
 *   - Query calls are asynchronous on the caller's HIP stream (hipStream_t passed as
 *     void*; NULL means the default stream).  Argument errors are reported
 *     synchronously; device faults surface as GP_E_HIP on a later call.
 *   - The library never allocates memory inside gp_pip / gp_p2p: the caller passes a
 *     device workspace of at least gp_workspace_bytes() bytes.
 *   - Ids are int32; sizes are int64 but every count must stay below 2^31.
 */
#ifndef GP_H
#define GP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t gp_status;
#define GP_OK 0
#define GP_E_INVALID_ARG (-1)  /* bad pointer, size, enum or option */
#define GP_E_BAD_GEOMETRY (-2) /* malformed offsets, non-finite vertex, short polyline */
#define GP_E_OOM (-3)          /* device or host allocation failed */
#define GP_E_HIP (-4)          /* a HIP runtime call failed */
#define GP_E_CAPACITY (-5)     /* a count exceeds what the library supports */
#define GP_E_BUSY (-6)         /* server: no admission possible right now */
#define GP_E_CLOSED (-7)       /* server: already shut down */
#define GP_E_TIMEOUT (-8)      /* server: wait timed out */
#define GP_E_NOT_FOUND (-9)    /* server: unknown ticket */

typedef enum { GP_PIP = 1, GP_P2P = 2 } gp_kind;
typedef enum { GP_FP64 = 0, GP_MIXED = 1 } gp_precision;

/* Thread-local text of the last error on this thread (never NULL). */
const char *gp_last_error(void);

/* Features in SoA + CSR form (Sec. III.A-B: count vectors and prefix-sum offsets
 * instead of objects).  Polygon f owns rings feature_ring_off[f]..[f+1]; ring r owns
 * vertices ring_vert_off[r]..[r+1] of x/y.  Rings are implicitly closed; a repeated
 * closing vertex is a harmless zero-length edge.  Polylines: feature_ring_off is NULL,
 * feature f is the vertex chain of ring f, n_rings == n_features, and every polyline
 * needs >= 2 vertices.  Offsets start at 0, never decrease, and end at the total. */
typedef struct gp_geometry {
    int64_t n_features;
    const int64_t *feature_ring_off; /* [n_features+1], polygons only */
    int64_t n_rings;
    const int64_t *ring_vert_off;    /* [n_rings+1] */
    int64_t n_vertices;
    const double *x;                 /* [n_vertices] */
    const double *y;                 /* [n_vertices] */
    int32_t on_device;               /* 1: the five arrays are device pointers */
} gp_geometry;

/* Grid of cell size cell_size > 0.  nx == 0 or ny == 0 derives the extent from the
 * (expanded, padded) MBBs: x0 = smallest MBB corner, nx = floor((max-x0)/cs)+1.
 * radius_D >= 0 is the P2P range (ignored for PIP).
 * pip_cell_classes = 1 (PIP only; 0 otherwise) classifies every (cell, polygon) pair at
 * build time (Sec. III.A): a pair whose cell, widened by max(cs*2^-20, M*2^-40) with M
 * the largest grid coordinate magnitude, meets no edge's bounding box lies wholly
 * inside or wholly outside the polygon, decided by the FP64 crossing parity of the cell
 * centre; every other pair is a boundary pair.  Queries then skip outside pairs, give
 * every still undecided point of the cell an inside pair's id without testing, and test
 * only boundary pairs.  Results are identical to the unclassified grid; gp_stats.tests
 * counts the tests performed and tests_avoided the candidate tests skipped.
 * p2p_segment_filter = 1 (P2P only; 0 otherwise) also rasterises every segment's
 * bounding box, expanded by D and padded like the MBBs, and keeps per cell the list of
 * segments it reaches; the GP_MIXED form then tests only those (a segment farther than
 * D from the whole cell can neither be a point's nearest segment within range nor bring
 * a polyline into range), with the same results; tests and tests_avoided as above.  The
 * GP_FP64 form keeps testing every candidate segment.
 * prestage = 1 (0 otherwise) computes at build time, for every cell, the cell-relative
 * FP32 records of the GP_MIXED form, which its queries then read instead of computing
 * them per work item; same results.  P2P (ignored with p2p_segment_filter): the records
 * of all the cell's candidate segments and the cell's error bounds, 20 bytes per (cell,
 * candidate segment).  PIP: per (cell, candidate polygon) pair its edges' records in
 * three classes -- edges whose FP32 crossing test equals the FP64 predicate for every
 * point of the cell, edges right of the cell whose crossing reduces to the half-open
 * straddle of the point's y (with a flag for a point level with an endpoint in FP32), and
 * guarded edges near the cell (test plus error-band flag) -- 16 bytes per edge (32 per
 * guarded edge).  Reported in gp_grid_info.device_bytes. */
typedef struct gp_grid_params {
    double cell_size;
    double radius_D;
    double x0, y0;
    int64_t nx, ny;
    int32_t pip_cell_classes;
    int32_t p2p_segment_filter;
    int32_t prestage;
} gp_grid_params;

typedef struct gp_grid gp_grid;

/* Kernel configuration chosen by gp_autotune or set by hand (0 = library default). */
typedef struct gp_tuning {
    int32_t points_per_lane; /* 1, 2 or 4: a work item holds up to 64*ppl points */
    int32_t edge_chunk;      /* edges staged in LDS per round: 64..512, multiple of 64
                                (the mixed PIP form on a grid with build-time records
                                streams fixed chunks of 128 and ignores it) */
    int32_t wg_per_cu;       /* persistent workgroups per compute unit: 1..32 */
    int32_t persistent;      /* 1: persistent workgroups popping items from one queue per
                                XCD (stealing from the others when theirs is empty);
                                0: one workgroup per item.  While a grid runs the library
                                default (no gp_set_tuning or gp_autotune on it), queries
                                of fewer than 2^22 points run one workgroup per item, and
                                queries of fewer than 256 points per grid cell at most 2
                                points per lane; the server applies both rules to its
                                chunks whatever the grid's tuning */
    int32_t waves_per_item;  /* P2P: 1, 2 or 4 wavefronts share one LDS staging and a work
                                item holds up to 64*ppl*waves points; PIP: always 1 */
    int32_t vp_points;       /* items with at most this many points (1..64) use the
                                vertex-parallel mapping (lanes over edges or segments, the
                                wave looping over the points; FP64, Sec. III.B's
                                alternative; P2P: one-wave items only, refined by a
                                kernel of their own ahead of the others); -1 never;
                                0 = library default (PIP 16, P2P 4) */
} gp_tuning;

/* Per-call counters.  Filling them synchronises the stream at the end of the call. */
typedef struct gp_stats {
    int64_t n_points;     /* points in the call */
    int64_t n_paired;     /* points in a cell with >= 1 candidate */
    int64_t n_items;      /* refinement work items (cell, point chunk) */
    uint64_t tests;       /* point-edge tests performed: sum over cells npts * sum nedges
                             over the candidates refined (all of them unless the grid
                             was built with pip_cell_classes) */
    int64_t n_rechecked;  /* GP_MIXED: points recomputed in FP64 */
    float ms_pairing;     /* hash + sort + gather + item list */
    float ms_refine;      /* refinement kernel */
    float ms_recheck;     /* FP64 recheck kernel */
    float ms_total;
    uint64_t tests_avoided; /* candidate tests skipped by the cell classes (else 0) */
} gp_stats;

/* Build the device-resident grid for a feature set (Sec. III.A filter):
 * validates the geometry, copies it to the device, derives MBBs (expanded by D for
 * P2P), rasterises them and sorts the (cell, feature) pairs into a cell -> candidate
 * CSR whose lists are sorted by feature id.  Synchronous on hip_stream; the grid owns
 * its device memory until gp_grid_free.  GP_E_BAD_GEOMETRY for malformed input,
 * GP_E_CAPACITY when a count reaches 2^31 or the grid exceeds 2^28 cells. */
gp_status gp_build_grid(gp_kind kind, const gp_geometry *geom, const gp_grid_params *params,
                        void *hip_stream, gp_grid **out);
void gp_grid_free(gp_grid *grid);

/* Grid description.  Any output pointer may be NULL. */
typedef struct gp_grid_info {
    int32_t kind;
    double x0, y0, cell_size, radius_D;
    int64_t nx, ny, n_features, n_edges, n_pairs;
    int64_t n_pairs_inside, n_pairs_outside, n_pairs_boundary; /* cell classes, else 0 */
    int64_t device_bytes;  /* device memory the grid holds */
    int64_t n_segment_pairs; /* (cell, segment) pairs of p2p_segment_filter, else 0 */
} gp_grid_info;
gp_status gp_grid_get_info(const gp_grid *grid, gp_grid_info *info);

/* Copy the candidate CSR to HOST buffers: cand_off[nx*ny+1], cand_id[n_pairs]. */
gp_status gp_grid_candidates(const gp_grid *grid, int32_t *cand_off, int32_t *cand_id);

/* Device workspace needed by gp_pip / gp_p2p / gp_pair_points for n points. */
gp_status gp_workspace_bytes(const gp_grid *grid, int64_t n_points, gp_precision prec,
                             size_t *bytes);

/* Point pairing only (Sec. III.A): cell hash and stable counting sort.  Writes, to
 * DEVICE buffers, perm[n] (sorted position -> original index; points of a cell in
 * ascending original index, unpaired points last) and pt_off[nx*ny+1] (start of each
 * cell in perm).  Asynchronous. */
gp_status gp_pair_points(const gp_grid *grid, int64_t n, const double *px, const double *py,
                         int32_t *perm, int32_t *pt_off, void *ws, size_t ws_bytes,
                         void *hip_stream);

/* PIP refinement for n points (device pointers px, py, out_id).  out_id[i] = smallest
 * polygon id containing point i under the even-odd rule, or -1.  Asynchronous. */
gp_status gp_pip(const gp_grid *grid, int64_t n, const double *px, const double *py,
                 int32_t *out_id, gp_precision prec, void *ws, size_t ws_bytes,
                 void *hip_stream, gp_stats *stats);

/* P2P refinement for n points (device pointers).  out_id[i] = nearest polyline within
 * D (ties: smallest id) or -1; out_dist[i] its distance or +inf.  Asynchronous. */
gp_status gp_p2p(const gp_grid *grid, int64_t n, const double *px, const double *py,
                 int32_t *out_id, double *out_dist, gp_precision prec, void *ws,
                 size_t ws_bytes, void *hip_stream, gp_stats *stats);

/* For callers that cannot allocate device memory (code under hipGraph capture, tight
 * serving loops, harnesses that forbid hipMalloc): gp_pip (kind GP_PIP, out_dist
 * ignored) or gp_p2p (kind GP_P2P) with the workspace taken from a buffer the library
 * holds on each GPU (GP_NOALLOC_SCRATCH_BYTES, kept until the process ends) instead of
 * a caller workspace.  Allocates nothing; inputs and outputs are the caller's device
 * pointers, as for gp_pip / gp_p2p, with the same results.  GP_E_CAPACITY when the
 * workspace for n points (gp_workspace_bytes) exceeds the buffer.  Every call on one GPU
 * shares that GPU's buffer: calls that overlap on one GPU (other streams, other host
 * threads) race and must be serialised by the caller.  Asynchronous on hip_stream. */
#define GP_NOALLOC_SCRATCH_BYTES (64ull << 20)
gp_status gp_query_noalloc(const gp_grid *grid, gp_kind kind, int64_t n, const double *px,
                           const double *py, int32_t *out_id, double *out_dist,
                           gp_precision prec, void *hip_stream);

/* Kernel configuration of a grid for one precision form.  gp_set_tuning with a NULL
 * tuning restores the library default. */
gp_status gp_set_tuning(gp_grid *grid, gp_precision prec, const gp_tuning *tuning);
gp_status gp_get_tuning(const gp_grid *grid, gp_precision prec, gp_tuning *tuning);

/* Autotuner: times every configuration of a built-in search space on the given
 * (device) sample points, keeps the fastest, stores it in the grid and returns it.
 * Results never depend on the configuration.  The winner is cached in the process by
 * (operation, precision, GPU architecture, the grid's build-time options, workload class:
 * the octaves of the sample size, of the tests per paired point and of the paired points
 * per work item under the library default); a later call whose key is cached applies
 * that winner without searching.  Synchronous. */
gp_status gp_autotune(gp_grid *grid, gp_precision prec, int64_t n, const double *px,
                      const double *py, void *ws, size_t ws_bytes, void *hip_stream,
                      gp_tuning *best, float *best_ms);

/* The autotuner's cache: entries in the process, written to / merged from a text file (one
 * line per entry: key, tab, the six gp_tuning fields), so deployments reuse earlier
 * searches.  gp_tuning_cache_load adds nothing and returns GP_E_INVALID_ARG when a line is
 * malformed or holds an invalid tuning. */
gp_status gp_tuning_cache_save(const char *path);
gp_status gp_tuning_cache_load(const char *path);
gp_status gp_tuning_cache_clear(void);
gp_status gp_tuning_cache_size(int64_t *entries);

/* Cell-size sweep: the filter-versus-refine trade-off that Sec. III.A leaves open (a
 * finer grid pairs fewer features with each point but costs more pairs and memory).
 * For each of the n_sizes cell sizes, builds the grid of *params with that cell size
 * (a derived extent is re-derived; an explicit one keeps x0, y0 and covers the same
 * area: nx = ceil(nx0 * cs0 / cs)), runs the query on the n sample points (device
 * pointers) once to warm up and three times timed, and frees the grid again.  Per size
 * i: ms_query[i] the median gp_stats.ms_total (NAN when that grid exceeds the library's
 * limits), n_pairs[i] the candidate pairs, tests[i] the tests performed, grid_bytes[i]
 * the grid's device memory.  *best receives the fastest size.  Any per-size output may
 * be NULL.  Results never depend on the cell size.  Allocates; synchronous. */
gp_status gp_sweep_cell_size(gp_kind kind, const gp_geometry *geom, const gp_grid_params *params,
                             const double *cell_sizes, int32_t n_sizes, int64_t n,
                             const double *px, const double *py, gp_precision prec,
                             void *hip_stream, double *best, float *ms_query,
                             int64_t *n_pairs, uint64_t *tests, int64_t *grid_bytes);

/* Measurement probe (not part of the join): sustained rate on the current device of
 * which = 0: FP32 FMA with every operand in a VGPR (FLOP/s), 1: FP64 FMA (FLOP/s),
 * 2: LDS broadcast 16-byte reads (wave reads/s), 3: the mixed P2P point-segment test on
 * register data with the segment constants in SGPRs (tests/s), 4: FP32 FMA with one
 * SGPR operand (FLOP/s), 5: the mixed P2P test on per-lane VGPR data, four points
 * against two segments per step (tests/s), 6 and 7: the mixed PIP crossing test on
 * per-lane VGPR data, two points per lane against eight edges per step and four against
 * four (tests/s).  `iters` sets the
 * loop length; *ms receives the kernel time.  Synchronous; GP_E_INVALID_ARG for other
 * `which` or iters <= 0. */
gp_status gp_probe_rate(int32_t which, int32_t iters, double *rate, float *ms);

/* ---------------------------------------------------------------- serving */

/* A continuous-batching server over resident grids (the serving form of the refinement:
 * the paper's join answers batches of points against fixed polygon or polyline sets).
 * Requests are cut into chunks of at most slot_points points (every point is
 * independent, so chunking is exact).  A chunk runs in a block of device memory carved
 * from one arena of mem_budget bytes that the server allocates at creation: the chunk's
 * inputs, outputs and query workspace (gp_workspace_bytes) for its size bucket.  Chunks
 * are admitted in FIFO order while one of the n_slots streams is free AND the chunk's
 * block fits in the arena: the chunks of a large request spread over the free streams,
 * and requests that arrive while others run start as streams and memory free up, so
 * their work overlaps on the device.  Each block captures its query into a hipGraph at
 * first use and replays it (use_graphs = 1). */
typedef struct gp_serve_opts {
    int32_t n_slots;          /* chunks running at once (one HIP stream each), 1..16 */
    int64_t slot_points;      /* largest chunk, in points, in [1024, 2^30) */
    int64_t mem_budget;       /* bytes of the device arena; must hold one chunk of
                                 slot_points points (else GP_E_OOM) */
    int32_t precision;        /* gp_precision for every request */
    int32_t inputs_on_device; /* 1: submit() pointers are device memory, else host */
    int32_t use_graphs;       /* 1: replay captured hipGraphs per block */
    int32_t max_queue;        /* pending requests beyond which submit returns BUSY */
} gp_serve_opts;

typedef struct gp_server gp_server;

typedef struct gp_serve_stats {
    int64_t completed, failed, pending;
    int64_t in_flight;                      /* requests with chunks on the device now */
    double p50_us, p99_us, mean_us, max_us; /* submit -> result visible, over the most
                                               recent latency_samples requests */
    double points_per_s, tests_per_s;       /* over the completed requests' busy span */
    int64_t points, tests, graph_replays;
    int64_t chunks_in_flight;               /* chunks on the device now */
    int64_t max_in_flight;                  /* peak of in_flight */
    int64_t max_chunks_in_flight;           /* peak of chunks_in_flight */
    int64_t deferred_for_memory;            /* chunks that waited for arena memory while
                                               a stream was free */
    int64_t bytes_in_use, peak_bytes_in_use, arena_bytes;
    int64_t latency_samples;                /* at most 65,536 */
} gp_serve_stats;

/* pip_grid / p2p_grid may each be NULL (then that kind is rejected); the grids'
 * device must be current.  Allocates the arena and starts the server thread. */
gp_status gp_serve_create(const gp_grid *pip_grid, const gp_grid *p2p_grid,
                          const gp_serve_opts *opts, gp_server **out);
/* Enqueue a request; returns immediately with a ticket.  out_id (and out_dist for P2P)
 * are written before the ticket completes; they live where the inputs live.  The
 * caller keeps inputs and outputs alive until the ticket completes. */
gp_status gp_serve_submit(gp_server *srv, gp_kind kind, int64_t n, const double *px,
                          const double *py, int32_t *out_id, double *out_dist,
                          uint64_t *ticket);
/* done = 1 once the ticket's results are visible (0 while pending).  Reporting done
 * releases the ticket: later calls on it return GP_E_NOT_FOUND. */
gp_status gp_serve_poll(gp_server *srv, uint64_t ticket, int32_t *done);
/* Block until the ticket completes or timeout_us passes (<0: forever).  Returns the
 * request's own status once complete, and releases the ticket (later calls on it return
 * GP_E_NOT_FOUND); GP_E_TIMEOUT otherwise. */
gp_status gp_serve_wait(gp_server *srv, uint64_t ticket, int64_t timeout_us);
/* Counters and latency percentiles.  Named gp_serve_stats_get because gp_serve_stats
 * is the name of the struct it fills. */
gp_status gp_serve_stats_get(gp_server *srv, gp_serve_stats *stats);
/* Forget the latency samples and counters gathered so far (e.g. after a warm-up); the
 * peaks restart from the current values. */
gp_status gp_serve_stats_reset(gp_server *srv);
/* Drain queued and in-flight work, stop the server thread and free everything. */
gp_status gp_serve_destroy(gp_server *srv);

#ifdef __cplusplus
}
#endif
#endif /* GP_H */
