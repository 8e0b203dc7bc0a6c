// Internal interface between the host runtime (gp_api.cpp, gp_serve.cpp) and the HIP
// kernels (gp_kernels.hip).  Not installed; the public ABI is include/gp.h.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "../../include/gp.h"

namespace gp {

// Consecutive segments covered by one bounding circle of the P2P exact-distance pass.
constexpr int P2P_BLOCK = 8;

// Work item of the refinement: a grid cell and a chunk of its (sorted) points.  The
// cell's whole candidate list is refined by one workgroup, so per-point results never
// need a cross-workgroup merge.
struct Item {
  int32_t cell;
  int32_t pt_lo;
  int32_t npts;
  int32_t cost_rank;  // PIP: cost bucket (4 per octave of npts * cell edges) of the
                      // longest-first order
};

// Everything the refinement kernels read.  Passed by value as the kernel argument.
struct RefineArgs {
  // work queue
  const Item *items;
  const uint32_t *n_items;   // device scalar written by the item builder
  uint32_t *item_counter;    // [GP_XCDS] device counters of the item queues, zeroed before
                             // the launch
  // grid
  const int32_t *cand_off;   // [ncells+1]
  const int32_t *cand_id;    // [npairs]
  const int32_t *eoff;       // [nf+1] edge (PIP) or segment (P2P) range of a feature
  const double4 *edge64;     // PIP: (lo.x, lo.y, hi.x, hi.y); P2P: (a.x, a.y, b.x, b.y)
  const float *k32;          // PIP: fl32(w/h), 0 for horizontal edges
  const double4 *frame64;    // P2P: (u.x, u.y, -m.u, -m.v) of each segment, absolute m
  const float4 *frame32;     // P2P: (u.x*scale, u.y*scale, |d|/2*scale, |d|)
  const double4 *circ;       // P2P: per block of P2P_BLOCK segments (centre x, y, radius, 0)
  const uint8_t *cand_class; // PIP, optional: per candidate pair 0 outside, 1 inside, 2 boundary
  const int32_t *cseg_off;   // P2P mixed, optional: [ncells+1] into cseg
  const int32_t *cseg;       // the segments that reach each cell, ascending
  const int32_t *seg2f;      // [nseg] polyline of each segment
  const float4 *recU;        // P2P mixed, optional build-time staging: per (cell, segment)
  const float *recV;         //   records in refinement order, from rec_off[cell]
  const int64_t *rec_off;    //   [ncells+1]
  const float2 *cellE;       //   [ncells] E over near segments, E over all
  const int2 *near;          // P2P: [npairs] near-segment range of each (cell, candidate)
  const float4 *precs;       // PIP mixed, optional build-time records: per (cell, candidate)
  const int64_t *prec_off;   //   pair its edges' records from prec_off[k] (float4 slots):
  const int2 *pcnt;          //   pcnt[k].x plain, pcnt[k].y band, then from the next even
                             //   slot the guarded ones (two slots each) up to prec_off[k+1]
  double x0, y0, cs;
  int32_t nx, ncells;
  double D, D2, D2_next;     // P2P: D, fl(D*D), the smallest double above fl(D*D)
  float half_box;            // bound on |rebased point coordinate| inside its cell
  float p2p_margin;          // P2P: T, the "near the cell" margin (distance units)
  float p2p_scale;           // P2P mixed: power of two; |rebased coordinate| * scale < 1/4
  // points, sorted by cell
  const uint32_t *skey;      // sorted cell ids
  const uint32_t *perm;      // sorted position -> caller index
  const double2 *xy;         // FP64 points in sorted order
  // outputs (caller order)
  int32_t *out_id;
  double *out_dist;
  // FP64 recheck queue (sorted positions)
  uint32_t *rq;
  uint32_t *rq_count;
  int32_t edge_chunk;
  int32_t vp_points;         // items with at most this many points go vertex-parallel
  uint32_t *vp_list;         // P2P: indices of those items, collected before the
  uint32_t *vp_count;        //   refinement (count zeroed with the counters)
};

// Device-resident grid.
// Queries of fewer points than this run one workgroup per item when the tuning in effect
// is the library default (or, in the server, for every chunk): a persistent launch pays
// a fixed cost at its end, when every workgroup finds the queues empty, that only larger
// queries amortise (measured: 1M points 0.61 against 1.38 ms, 10K 0.78 against 1.43;
// from 4M points on the two are level).
constexpr int64_t kPersistentMinPoints = int64_t(1) << 22;
// Likewise 4 points per lane pay only when a cell holds a full item of them: with fewer
// than this many points per grid cell on average the default takes 2 (measured on P2P,
// 1M points with 6 per cell 0.55 against 0.59 ms, 1M with 25 per cell 2.28 against 2.70).
constexpr int64_t kFourPerLaneMinPointsPerCell = 256;

struct Grid {
  gp_kind kind;
  int device;
  double x0, y0, cs, D, D2;
  int32_t nx, ny, ncells;
  int32_t nf, nedges, npairs;
  int32_t *d_eoff;
  double4 *d_edge64;
  float *d_k32;
  double4 *d_frame64;
  float4 *d_frame32;
  double4 *d_circ;
  int32_t *d_cand_off;
  int32_t *d_cand_id;
  int64_t *d_cell_edges;  // [ncells] sum of nedges over the candidates a query refines
  int64_t *d_cell_edges_all;  // [ncells] over all candidates (only with cell classes)
  uint8_t *d_cand_class;  // [npairs] PIP cell classes, or null
  int64_t npairs_class[3];  // outside, inside, boundary
  int32_t *d_cseg_off;    // P2P segment filter: [ncells+1]
  int32_t *d_cseg;        // [ncseg]
  int32_t *d_seg2f;       // [nedges]
  int64_t *d_cell_segs;   // [ncells] segments per cell
  int64_t ncseg;
  int2 *d_near;           // P2P: near-segment range per (cell, candidate) pair
  float4 *d_recU;         // P2P build-time staging (prestage)
  float *d_recV;
  int64_t *d_rec_off;
  float2 *d_cellE;
  int64_t nrec;
  float p2p_scale;        // see RefineArgs
  float4 *d_precs;        // PIP build-time records (prestage), see RefineArgs
  int64_t *d_prec_off;
  int2 *d_pcnt;
  int64_t nprec;
  gp_tuning tune[2];
  bool tune_explicit[2];  // tune[prec] was set by gp_set_tuning or gp_autotune
  int num_cu;
};

// Workspace layout for n points.
struct Workspace {
  uint32_t *keyA, *keyB, *valA, *valB;
  uint32_t *hist;        // radix histogram [256 * nblk]
  uint32_t *scan_tmp;    // scan partials
  int32_t *pt_off;       // [ncells+1]
  double2 *xyA, *xyB;    // FP64 point payload of the sort (ping-pong)
  uint32_t *item_cnt;    // [ncells+1] -> exclusive offsets
  Item *items;
  uint32_t *ikA, *ikB, *ivA, *ivB;  // PIP: sort of the items by cost (max_items each)
  Item *items_sorted;
  uint32_t *vp_list;     // P2P: the vertex-parallel items (max_items)
  uint32_t *rq;
  uint32_t *counters;    // [16]: 0 item counter, 1 rq count, 2 n_items(copy), ...
  unsigned long long *tests;  // [1]
  size_t bytes;
};

// C_ITEM .. C_ITEM + GP_XCDS - 1: the item queues of the persistent launches, one per XCD.
enum Counter { C_RQ = 1, C_NITEMS = 2, C_NPAIRED = 3, C_NVP = 4, C_ITEM = 8, C_COUNT = 16 };

size_t workspace_layout(const Grid &g, int64_t n, gp_precision prec, void *base, Workspace *ws);
size_t scan_tmp_elems(size_t n);

// ---- launchers (gp_kernels.hip); all enqueue on `s` and return hipGetLastError()
hipError_t launch_fill_u32(uint32_t *p, uint32_t v, size_t n, hipStream_t s);
hipError_t launch_exclusive_scan_u32(const uint32_t *in, uint32_t *out, size_t n,
                                     uint32_t *tmp, hipStream_t s);
// Stable sort of (key, value) by key.  With pl_out != NULL the FP64 point (px[i], py[i])
// of every record travels with it (ping-pong through plA/plB; *pl_out = sorted copy).
hipError_t launch_radix_sort(uint32_t *keyA, uint32_t *keyB, uint32_t *valA, uint32_t *valB,
                             size_t n, int nbits, bool values_are_identity, uint32_t *hist,
                             uint32_t *scan_tmp, hipStream_t s, uint32_t **keys_out,
                             uint32_t **vals_out, const double *px = nullptr,
                             const double *py = nullptr, double2 *plA = nullptr,
                             double2 *plB = nullptr, double2 **pl_out = nullptr);
size_t radix_hist_elems(size_t n);

// grid build
hipError_t launch_build_edges(const int32_t *ring_vert_off, const int32_t *feature_ring_off,
                              const double *x, const double *y, int32_t nf, int32_t nrings,
                              int32_t nverts, gp_kind kind, double4 *edge64, float *k32,
                              int32_t *eoff, hipStream_t s);
hipError_t launch_build_frames(const double4 *seg64, int32_t nseg, float scale,
                               double4 *frame64, float4 *frame32, hipStream_t s);
hipError_t launch_build_circles(const double4 *seg64, int32_t nseg, double4 *circ,
                                hipStream_t s);
hipError_t launch_mbb(const int32_t *ring_vert_off, const int32_t *feature_ring_off,
                      const double *x, const double *y, int32_t nf, gp_kind kind, double D,
                      double cs, double *mbb, hipStream_t s);
hipError_t launch_extent(const double *mbb, int32_t nf, double *out4, hipStream_t s);
hipError_t launch_raster_count(const double *mbb, int32_t nf, double x0, double y0, double cs,
                               int32_t nx, int32_t ny, uint32_t *cnt, hipStream_t s);
// out[0] = sum of v[0..n) in 64 bits (out is zeroed first).
hipError_t launch_sum_u32(const uint32_t *v, size_t n, unsigned long long *out, hipStream_t s);
hipError_t launch_raster_emit(const double *mbb, int32_t nf, double x0, double y0, double cs,
                              int32_t nx, int32_t ny, const uint32_t *off, uint32_t *pair_cell,
                              uint32_t *pair_fid, hipStream_t s);
hipError_t launch_histogram(const uint32_t *keys, size_t n, uint32_t *cnt, hipStream_t s);
hipError_t launch_cell_edges(const int32_t *cand_off, const int32_t *cand_id,
                             const int32_t *eoff, const uint8_t *cand_class, int32_t ncells,
                             int64_t *cell_edges, hipStream_t s);
hipError_t launch_near_ranges(const double4 *seg64, int32_t nseg, double D, double pad,
                              double x0, double y0, double cs, int32_t nx, int32_t ny,
                              const uint32_t *pair_cell, const int32_t *cand_id, int32_t npairs,
                              const int32_t *eoff, int4 *rc, int2 *near, hipStream_t s);
hipError_t launch_prestage(const int32_t *cand_off, const int32_t *cand_id, const int32_t *eoff,
                           const double4 *frame64, const float4 *frame32, double x0, double y0,
                           double cs, int32_t nx, int32_t ncells, double D, float hb, float T,
                           float sc, const int64_t *rec_off, float4 *recU, float *recV,
                           float2 *cellE, hipStream_t s);
// PIP build-time records: (band, guarded) counts of every (cell, candidate polygon) pair,
// then the records at the per-pair slot offsets off[] with the (plain, band) counts pc[].
hipError_t launch_pip_rec_count(const uint32_t *pair_cell, const int32_t *cand_id,
                                int32_t npairs, const int32_t *eoff, const double4 *edge64,
                                const float *k32, double x0, double y0, double cs, int32_t nx,
                                float hb, int2 *cnt, hipStream_t s);
hipError_t launch_pip_rec_emit(const uint32_t *pair_cell, const int32_t *cand_id,
                               int32_t npairs, const int32_t *eoff, const double4 *edge64,
                               const float *k32, double x0, double y0, double cs, int32_t nx,
                               float hb, const int64_t *off, const int2 *pc, float4 *recs,
                               hipStream_t s);
hipError_t launch_seg_boxes(const double4 *seg64, int32_t nseg, double D, double pad,
                            double *box, hipStream_t s);
hipError_t launch_seg2f(const int32_t *eoff, int32_t nf, int32_t *seg2f, hipStream_t s);
hipError_t launch_cell_counts(const int32_t *off, int32_t ncells, int64_t *cnt, hipStream_t s);
hipError_t launch_classify_pairs(const uint32_t *pair_cell, const int32_t *cand_id,
                                 int32_t npairs, const int32_t *eoff, const double4 *edge64,
                                 double x0, double y0, double cs, int32_t nx, double margin,
                                 uint8_t *cand_class, hipStream_t s);

// query pipeline
hipError_t launch_hash(const double *px, const double *py, int64_t n, double x0, double y0,
                       double cs, int32_t nx, int32_t ny, uint32_t *key, hipStream_t s);
hipError_t launch_offsets(const uint32_t *skey, int64_t n, int32_t ncells, int32_t *pt_off,
                          hipStream_t s);
hipError_t launch_unpaired(const RefineArgs &a, int64_t n, uint32_t *n_paired, hipStream_t s);
hipError_t launch_items(const int32_t *pt_off, const int32_t *cand_off,
                        const int64_t *cell_edges, const int64_t *cell_edges_all,
                        int32_t ncells, int32_t chunk,
                        uint32_t *item_cnt, uint32_t *scan_tmp, Item *items, uint32_t *counters,
                        unsigned long long *tests, hipStream_t s);
// Items in longest-first order into out[0 .. *n_items), with their cost buckets.
hipError_t launch_order_items(Item *items, const uint32_t *n_items, int64_t max_items,
                              const int64_t *cell_edges, uint32_t *kA, uint32_t *kB,
                              uint32_t *vA, uint32_t *vB, uint32_t *hist, uint32_t *scan_tmp,
                              Item *out, hipStream_t s);
hipError_t launch_refine(gp_kind kind, gp_precision prec, const RefineArgs &a,
                         const gp_tuning &t, int num_cu, int64_t max_items, hipStream_t s);
hipError_t launch_recheck(gp_kind kind, const RefineArgs &a, int num_cu, hipStream_t s);
hipError_t launch_copy_perm(const uint32_t *perm, int64_t n, int32_t *out, hipStream_t s);

}  // namespace gp
