// Host runtime behind include/gp.h: argument checks, the device-resident grid, the
// workspace layout, launch sequencing of the query pipeline, and the autotuner.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "gp_internal.h"

using namespace gp;

struct gp_grid : public gp::Grid {};

// ------------------------------------------------------------------------- errors

static thread_local char g_err[512] = "no error";

extern "C" const char *gp_last_error(void) { return g_err; }

namespace gp {
gp_status set_error(gp_status code, const char *fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
  return code;
}
}  // namespace gp

#define GP_TRY_HIP(expr)                                                                  \
  do {                                                                                    \
    hipError_t e_ = (expr);                                                               \
    if (e_ != hipSuccess)                                                                 \
      return set_error(GP_E_HIP, "%s failed: %s", #expr, hipGetErrorString(e_));          \
  } while (0)

static const int64_t kMaxCount = 0x7fffffffLL;
static const int64_t kMaxCells = (int64_t)1 << 28;

// ------------------------------------------------------------------------- helpers

static int bits_for(uint64_t v) {
  int b = 0;
  while (v) { ++b; v >>= 1; }
  return b;
}

static size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

namespace {
struct DevBuf {
  void *p = nullptr;
  ~DevBuf() { if (p) (void)hipFree(p); }
  hipError_t alloc(size_t bytes) { return hipMalloc(&p, bytes ? bytes : 16); }
  template <class T> T *as() const { return (T *)p; }
};
}  // namespace

// Defaults from full-size sweeps on the configuration-3/4 workloads (gp_autotune
// re-tunes): P2P from a persistent queue, the mixed form with 4 points per lane, the FP64
// form with 2 (it carries three doubles per point from segment to segment) and 64-segment
// chunks (its 64-byte LDS records otherwise limit the waves per CU); PIP 2 points per lane
// and one workgroup per item.
static gp_tuning default_tuning(gp_kind kind, gp_precision prec) {
  gp_tuning t;
  if (kind == GP_P2P) {
    t.points_per_lane = prec == GP_MIXED ? 4 : 2;
    t.edge_chunk = prec == GP_MIXED ? 128 : 64;
    t.wg_per_cu = 32;
    t.persistent = 1;
  } else {
    t.points_per_lane = 2;
    t.edge_chunk = 128;
    t.wg_per_cu = 16;
    t.persistent = 0;
  }
  t.waves_per_item = 1;
  // few-point items vertex-parallel: PIP up to 16 points (its FP64 edge test is cheap
  // next to the staging a point-parallel item needs), P2P up to 4 (each point's polyline
  // minimum is a serial cross-lane reduction)
  t.vp_points = kind == GP_PIP ? 16 : 4;
  return t;
}

static bool tuning_valid(const gp_tuning &t, gp_kind kind) {
  const int w = t.waves_per_item;
  return (t.points_per_lane == 1 || t.points_per_lane == 2 || t.points_per_lane == 4) &&
         t.edge_chunk >= 64 && t.edge_chunk <= 512 && t.edge_chunk % 64 == 0 &&
         t.wg_per_cu >= 1 && t.wg_per_cu <= 32 && (t.persistent == 0 || t.persistent == 1) &&
         (w == 1 || (kind == GP_P2P && (w == 2 || w == 4))) &&
         (t.vp_points == -1 || (t.vp_points >= 1 && t.vp_points <= 64));
}

// ------------------------------------------------------------------------- geometry checks

namespace {
struct HostGeom {
  std::vector<int64_t> fro, rvo;
  std::vector<double> x, y;
};
}  // namespace

template <class T>
static hipError_t fetch(std::vector<T> &dst, const T *src, size_t n, bool on_device) {
  dst.resize(n);
  if (n == 0) return hipSuccess;
  if (on_device) return hipMemcpy(dst.data(), src, n * sizeof(T), hipMemcpyDeviceToHost);
  memcpy(dst.data(), src, n * sizeof(T));
  return hipSuccess;
}

static gp_status check_offsets(const std::vector<int64_t> &off, int64_t end, const char *what) {
  if (off.empty() || off[0] != 0)
    return set_error(GP_E_BAD_GEOMETRY, "%s must start at 0", what);
  for (size_t i = 1; i < off.size(); ++i)
    if (off[i] < off[i - 1])
      return set_error(GP_E_BAD_GEOMETRY, "%s decreases at %zu", what, i);
  if (off.back() != end)
    return set_error(GP_E_BAD_GEOMETRY, "%s ends at %lld, expected %lld", what,
                     (long long)off.back(), (long long)end);
  return GP_OK;
}

// ------------------------------------------------------------------------- grid build

// Half the side of a cell, rounded up, plus the rounding of the FP32 cell-relative
// coordinates: every point of a cell lies within this box around the cell centre.
static float half_box(const Grid &g) {
  double hb = 0.5 * g.cs * (1.0 + 0x1p-18) +
              0x1p-48 * (std::fabs(g.x0) + std::fabs(g.y0) + g.cs * (double)(g.nx + g.ny));
  return (float)(hb * (1.0 + 0x1p-20));
}

// FP32 margin T of the mixed P2P test: a polyline is kept while its FP32 distance is
// within D + T.
static float p2p_margin(const Grid &g) { return (float)std::max(0.01 * g.D, g.cs * 0x1p-10); }

// 64-bit sum of the n per-feature pair counts at cnt (device); -1 (with the error set)
// when a HIP call fails.  Synchronises the stream.
static int64_t pair_total(const uint32_t *cnt, size_t n, hipStream_t s) {
  DevBuf d_sum;
  unsigned long long total = 0;
  hipError_t e = d_sum.alloc(16);
  if (e == hipSuccess) e = launch_sum_u32(cnt, n, (unsigned long long *)d_sum.p, s);
  if (e == hipSuccess) e = hipMemcpyAsync(&total, d_sum.p, 8, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) {
    set_error(GP_E_HIP, "pair count failed: %s", hipGetErrorString(e));
    return -1;
  }
  return total > (unsigned long long)INT64_MAX ? INT64_MAX : (int64_t)total;
}

extern "C" gp_status gp_build_grid(gp_kind kind, const gp_geometry *geom,
                                   const gp_grid_params *params, void *hip_stream,
                                   gp_grid **out) {
  if (!out || !geom || !params) return set_error(GP_E_INVALID_ARG, "null argument");
  *out = nullptr;
  if (kind != GP_PIP && kind != GP_P2P) return set_error(GP_E_INVALID_ARG, "bad kind");
  const double cs = params->cell_size;
  if (!(cs > 0.0) || !std::isfinite(cs))
    return set_error(GP_E_INVALID_ARG, "cell_size must be finite and > 0");
  const double D = kind == GP_P2P ? params->radius_D : 0.0;
  if (!(D >= 0.0) || !std::isfinite(D))
    return set_error(GP_E_INVALID_ARG, "radius_D must be finite and >= 0");
  if (params->nx < 0 || params->ny < 0) return set_error(GP_E_INVALID_ARG, "negative nx/ny");
  if (params->pip_cell_classes != 0 && params->pip_cell_classes != 1)
    return set_error(GP_E_INVALID_ARG, "pip_cell_classes must be 0 or 1");
  if (params->p2p_segment_filter != 0 && params->p2p_segment_filter != 1)
    return set_error(GP_E_INVALID_ARG, "p2p_segment_filter must be 0 or 1");
  if (params->prestage != 0 && params->prestage != 1)
    return set_error(GP_E_INVALID_ARG, "prestage must be 0 or 1");
  const bool derive = params->nx == 0 || params->ny == 0;
  if (!derive && (!std::isfinite(params->x0) || !std::isfinite(params->y0)))
    return set_error(GP_E_INVALID_ARG, "non-finite grid origin");
  const int64_t nf = geom->n_features, nr = geom->n_rings, nv = geom->n_vertices;
  if (nf < 0 || nr < 0 || nv < 0) return set_error(GP_E_INVALID_ARG, "negative count");
  if (nf >= kMaxCount || nr >= kMaxCount || nv >= kMaxCount)
    return set_error(GP_E_CAPACITY, "counts must stay below 2^31");
  if (kind == GP_PIP && nf > 0 && !geom->feature_ring_off)
    return set_error(GP_E_INVALID_ARG, "polygons need feature_ring_off");
  if (kind == GP_P2P && nr != nf)
    return set_error(GP_E_INVALID_ARG, "polylines need n_rings == n_features");
  if (!geom->ring_vert_off || (nv > 0 && (!geom->x || !geom->y)))
    return set_error(GP_E_INVALID_ARG, "null geometry array");
  hipStream_t s = (hipStream_t)hip_stream;
  const bool dev = geom->on_device != 0;

  HostGeom h;
  GP_TRY_HIP(fetch(h.rvo, geom->ring_vert_off, (size_t)nr + 1, dev));
  if (kind == GP_PIP && geom->feature_ring_off)
    GP_TRY_HIP(fetch(h.fro, geom->feature_ring_off, (size_t)nf + 1, dev));
  else if (kind == GP_PIP)
    h.fro.assign(1, 0);  // no polygons: the offsets are the single 0
  GP_TRY_HIP(fetch(h.x, geom->x, (size_t)nv, dev));
  GP_TRY_HIP(fetch(h.y, geom->y, (size_t)nv, dev));
  gp_status st = check_offsets(h.rvo, nv, "ring_vert_off");
  if (st) return st;
  if (kind == GP_PIP) {
    st = check_offsets(h.fro, nr, "feature_ring_off");
    if (st) return st;
  } else {
    for (int64_t f = 0; f < nf; ++f)
      if (h.rvo[f + 1] - h.rvo[f] < 2)
        return set_error(GP_E_BAD_GEOMETRY, "polyline %lld has fewer than 2 vertices",
                         (long long)f);
  }
  for (int64_t v = 0; v < nv; ++v)
    if (!std::isfinite(h.x[v]) || !std::isfinite(h.y[v]))
      return set_error(GP_E_BAD_GEOMETRY, "vertex %lld is not finite", (long long)v);

  int device = 0;
  GP_TRY_HIP(hipGetDevice(&device));
  int num_cu = 0;
  GP_TRY_HIP(hipDeviceGetAttribute(&num_cu, hipDeviceAttributeMultiprocessorCount, device));

  std::vector<int32_t> rvo32(h.rvo.begin(), h.rvo.end());
  std::vector<int32_t> fro32(h.fro.begin(), h.fro.end());
  if (fro32.empty()) fro32.push_back(0);
  const int64_t nedges = kind == GP_PIP ? nv : nv - nf;

  DevBuf d_rvo, d_fro, d_x, d_y, d_mbb;
  GP_TRY_HIP(d_rvo.alloc(rvo32.size() * 4));
  GP_TRY_HIP(d_fro.alloc(fro32.size() * 4));
  GP_TRY_HIP(d_x.alloc((size_t)nv * 8));
  GP_TRY_HIP(d_y.alloc((size_t)nv * 8));
  GP_TRY_HIP(d_mbb.alloc((size_t)std::max<int64_t>(nf, 1) * 32));
  GP_TRY_HIP(hipMemcpyAsync(d_rvo.p, rvo32.data(), rvo32.size() * 4, hipMemcpyHostToDevice, s));
  GP_TRY_HIP(hipMemcpyAsync(d_fro.p, fro32.data(), fro32.size() * 4, hipMemcpyHostToDevice, s));
  if (nv) {
    GP_TRY_HIP(hipMemcpyAsync(d_x.p, h.x.data(), (size_t)nv * 8, hipMemcpyHostToDevice, s));
    GP_TRY_HIP(hipMemcpyAsync(d_y.p, h.y.data(), (size_t)nv * 8, hipMemcpyHostToDevice, s));
  }

  gp_grid *g = new gp_grid();
  memset((gp::Grid *)g, 0, sizeof(gp::Grid));
  auto fail = [&](gp_status code) {
    gp_grid_free(g);
    return code;
  };
  g->kind = kind;
  g->device = device;
  g->num_cu = num_cu;
  g->cs = cs;
  g->D = D;
  g->D2 = D * D;
  g->nf = (int32_t)nf;
  g->nedges = (int32_t)nedges;
  g->tune[GP_FP64] = default_tuning(kind, GP_FP64);
  g->tune[GP_MIXED] = default_tuning(kind, GP_MIXED);
  g->tune_explicit[GP_FP64] = g->tune_explicit[GP_MIXED] = false;

#define GP_TRY_HIP_G(expr)                                                                \
  do {                                                                                    \
    hipError_t e_ = (expr);                                                               \
    if (e_ != hipSuccess)                                                                 \
      return fail(set_error(GP_E_HIP, "%s failed: %s", #expr, hipGetErrorString(e_)));    \
  } while (0)

  GP_TRY_HIP_G(hipMalloc(&g->d_eoff, ((size_t)nf + 1) * 4));
  GP_TRY_HIP_G(hipMalloc(&g->d_edge64, (size_t)std::max<int64_t>(nedges, 1) * sizeof(double4)));
  GP_TRY_HIP_G(hipMalloc(&g->d_k32, (size_t)std::max<int64_t>(nedges, 1) * 4));
  GP_TRY_HIP_G(launch_build_edges(d_rvo.as<int32_t>(), d_fro.as<int32_t>(), d_x.as<double>(),
                                  d_y.as<double>(), (int32_t)nf, (int32_t)nr, (int32_t)nv, kind,
                                  g->d_edge64, g->d_k32, g->d_eoff, s));
  GP_TRY_HIP_G(launch_mbb(d_rvo.as<int32_t>(), d_fro.as<int32_t>(), d_x.as<double>(),
                          d_y.as<double>(), (int32_t)nf, kind, D, cs, d_mbb.as<double>(), s));
  {
    // Bound on |coordinate - cell centre| over every segment of every candidate of a
    // cell: the largest feature MBB diagonal plus D plus a cell diagonal.  The mixed
    // P2P kernel scales its frame constants by a power of two below 1/(4 * bound).
    double diag = 0.0;
    for (int64_t f = 0; f < nf; ++f) {
      int64_t v0 = h.rvo[kind == GP_PIP ? h.fro[f] : f];
      int64_t v1 = h.rvo[kind == GP_PIP ? h.fro[f + 1] : f + 1];
      double lx = INFINITY, ly = INFINITY, hx = -INFINITY, hy = -INFINITY;
      for (int64_t v = v0; v < v1; ++v) {
        lx = std::min(lx, h.x[v]); hx = std::max(hx, h.x[v]);
        ly = std::min(ly, h.y[v]); hy = std::max(hy, h.y[v]);
      }
      if (v1 > v0) diag = std::max(diag, std::hypot(hx - lx, hy - ly));
    }
    const double bound = diag + D + 2.0 * cs;
    int e = (int)std::ceil(std::log2(4.0 * bound));
    e = std::max(-100, std::min(100, e));
    g->p2p_scale = (float)std::ldexp(1.0, -e);
  }
  if (kind == GP_P2P) {
    const size_t ns = (size_t)std::max<int64_t>(nedges, 1);
    GP_TRY_HIP_G(hipMalloc(&g->d_frame64, ns * sizeof(double4)));
    GP_TRY_HIP_G(hipMalloc(&g->d_frame32, ns * sizeof(float4)));
    GP_TRY_HIP_G(launch_build_frames(g->d_edge64, (int32_t)nedges, g->p2p_scale, g->d_frame64,
                                     g->d_frame32, s));
    const size_t nb = (ns + P2P_BLOCK - 1) / P2P_BLOCK;
    GP_TRY_HIP_G(hipMalloc(&g->d_circ, nb * sizeof(double4)));
    GP_TRY_HIP_G(launch_build_circles(g->d_edge64, (int32_t)nedges, g->d_circ, s));
  }

  // extent
  double x0 = params->x0, y0 = params->y0;
  int64_t nx = params->nx, ny = params->ny;
  if (derive) {
    if (nf == 0) {
      x0 = 0.0; y0 = 0.0; nx = 1; ny = 1;
    } else {
      DevBuf d_ext;
      GP_TRY_HIP_G(d_ext.alloc(32));
      GP_TRY_HIP_G(launch_extent(d_mbb.as<double>(), (int32_t)nf, d_ext.as<double>(), s));
      double ext[4];
      GP_TRY_HIP_G(hipMemcpyAsync(ext, d_ext.p, 32, hipMemcpyDeviceToHost, s));
      GP_TRY_HIP_G(hipStreamSynchronize(s));
      x0 = ext[0];
      y0 = ext[1];
      double fx = std::floor((ext[2] - x0) / cs), fy = std::floor((ext[3] - y0) / cs);
      if (!(fx < (double)kMaxCells && fy < (double)kMaxCells))
        return fail(set_error(GP_E_CAPACITY, "derived grid is too large"));
      nx = (int64_t)fx + 1;
      ny = (int64_t)fy + 1;
    }
  }
  if (nx * ny > kMaxCells || nx > kMaxCells || ny > kMaxCells)
    return fail(set_error(GP_E_CAPACITY, "grid of %lld x %lld cells exceeds 2^28 cells",
                          (long long)nx, (long long)ny));
  g->x0 = x0;
  g->y0 = y0;
  g->nx = (int32_t)nx;
  g->ny = (int32_t)ny;
  g->ncells = (int32_t)(nx * ny);
  const int32_t ncells = g->ncells;

  // rasterise the MBBs: per-feature counts, offsets, emit, stable sort by cell
  {
    DevBuf d_cnt, d_tmp;
    const size_t nfe = (size_t)nf + 1;
    GP_TRY_HIP_G(d_cnt.alloc(nfe * 4));
    GP_TRY_HIP_G(d_tmp.alloc(scan_tmp_elems(std::max(nfe, (size_t)ncells + 1)) * 4));
    GP_TRY_HIP_G(launch_raster_count(d_mbb.as<double>(), (int32_t)nf, x0, y0, cs, g->nx, g->ny,
                                     d_cnt.as<uint32_t>(), s));
    // the total in 64 bits first: the 32-bit scan below wraps once it passes 2^32
    const int64_t total = pair_total(d_cnt.as<uint32_t>(), (size_t)nf, s);
    if (total < 0) return fail(GP_E_HIP);
    if (total >= kMaxCount)
      return fail(set_error(GP_E_CAPACITY, "%lld (cell, feature) pairs exceed 2^31 - 1",
                            (long long)total));
    GP_TRY_HIP_G(launch_exclusive_scan_u32(d_cnt.as<uint32_t>(), d_cnt.as<uint32_t>(), nfe,
                                           d_tmp.as<uint32_t>(), s));
    const uint32_t npairs = (uint32_t)total;
    g->npairs = (int32_t)npairs;
    DevBuf kA, kB, vA, vB, hist, stmp;
    const size_t np = std::max<size_t>(npairs, 1);
    GP_TRY_HIP_G(kA.alloc(np * 4));
    GP_TRY_HIP_G(kB.alloc(np * 4));
    GP_TRY_HIP_G(vA.alloc(np * 4));
    GP_TRY_HIP_G(vB.alloc(np * 4));
    GP_TRY_HIP_G(hist.alloc(radix_hist_elems(np) * 4));
    GP_TRY_HIP_G(stmp.alloc(scan_tmp_elems(std::max(radix_hist_elems(np), (size_t)ncells + 1)) * 4));
    GP_TRY_HIP_G(launch_raster_emit(d_mbb.as<double>(), (int32_t)nf, x0, y0, cs, g->nx, g->ny,
                                    d_cnt.as<uint32_t>(), kA.as<uint32_t>(), vA.as<uint32_t>(), s));
    uint32_t *skeys = nullptr, *svals = nullptr;
    GP_TRY_HIP_G(launch_radix_sort(kA.as<uint32_t>(), kB.as<uint32_t>(), vA.as<uint32_t>(),
                                   vB.as<uint32_t>(), npairs, bits_for((uint64_t)ncells - 1),
                                   false, hist.as<uint32_t>(), stmp.as<uint32_t>(), s, &skeys,
                                   &svals));
    GP_TRY_HIP_G(hipMalloc(&g->d_cand_off, ((size_t)ncells + 1) * 4));
    GP_TRY_HIP_G(hipMalloc(&g->d_cand_id, np * 4));
    GP_TRY_HIP_G(hipMalloc(&g->d_cell_edges, std::max<size_t>(ncells, 1) * 8));
    GP_TRY_HIP_G(launch_fill_u32((uint32_t *)g->d_cand_off, 0u, (size_t)ncells + 1, s));
    GP_TRY_HIP_G(launch_histogram(skeys, npairs, (uint32_t *)g->d_cand_off, s));
    GP_TRY_HIP_G(launch_exclusive_scan_u32((uint32_t *)g->d_cand_off, (uint32_t *)g->d_cand_off,
                                           (size_t)ncells + 1, stmp.as<uint32_t>(), s));
    if (npairs)
      GP_TRY_HIP_G(hipMemcpyAsync(g->d_cand_id, svals, (size_t)npairs * 4,
                                  hipMemcpyDeviceToDevice, s));
    if (kind == GP_P2P) {
      // near-segment range of each (cell, candidate) pair, for the mixed form's exact pass
      DevBuf rc;
      GP_TRY_HIP_G(rc.alloc((size_t)std::max<int64_t>(nedges, 1) * 16));
      GP_TRY_HIP_G(hipMalloc(&g->d_near, np * 8));
      GP_TRY_HIP_G(launch_near_ranges(g->d_edge64, (int32_t)nedges, D, cs * 0x1p-20, x0, y0, cs,
                                      g->nx, g->ny, skeys, g->d_cand_id, (int32_t)npairs,
                                      g->d_eoff, (int4 *)rc.p, g->d_near, s));
      GP_TRY_HIP_G(hipStreamSynchronize(s));
    }
    if (kind == GP_PIP && params->pip_cell_classes) {
      // margin of the cell classes: the MBB pad, or more where coordinates are large
      const double M = std::max({std::fabs(x0), std::fabs(y0), std::fabs(x0 + (double)nx * cs),
                                 std::fabs(y0 + (double)ny * cs)});
      const double margin = std::max(cs * 0x1p-20, M * 0x1p-40);
      GP_TRY_HIP_G(hipMalloc(&g->d_cand_class, np));
      GP_TRY_HIP_G(hipMalloc(&g->d_cell_edges_all, std::max<size_t>(ncells, 1) * 8));
      GP_TRY_HIP_G(launch_classify_pairs(skeys, g->d_cand_id, (int32_t)npairs, g->d_eoff,
                                         g->d_edge64, x0, y0, cs, g->nx, margin,
                                         g->d_cand_class, s));
      GP_TRY_HIP_G(launch_cell_edges(g->d_cand_off, g->d_cand_id, g->d_eoff, nullptr, ncells,
                                     g->d_cell_edges_all, s));
      std::vector<uint8_t> cls(npairs);
      if (npairs)
        GP_TRY_HIP_G(hipMemcpyAsync(cls.data(), g->d_cand_class, npairs, hipMemcpyDeviceToHost, s));
      GP_TRY_HIP_G(hipStreamSynchronize(s));
      for (uint8_t c : cls) g->npairs_class[c < 3 ? c : 2] += 1;
    }
    GP_TRY_HIP_G(launch_cell_edges(g->d_cand_off, g->d_cand_id, g->d_eoff, g->d_cand_class,
                                   ncells, g->d_cell_edges, s));
    GP_TRY_HIP_G(hipStreamSynchronize(s));
    if (kind == GP_PIP && params->prestage && npairs > 0) {
      // every (cell, candidate polygon) pair's edge records for the mixed test: classes
      // counted on the device, slot offsets summed here in 64 bits, records emitted
      const float hb = half_box(*g);
      DevBuf d_cnt;
      GP_TRY_HIP_G(d_cnt.alloc((size_t)npairs * sizeof(int2)));
      GP_TRY_HIP_G(launch_pip_rec_count(skeys, g->d_cand_id, (int32_t)npairs, g->d_eoff,
                                        g->d_edge64, g->d_k32, x0, y0, cs, g->nx, hb,
                                        d_cnt.as<int2>(), s));
      std::vector<int2> cnt(npairs), pc(npairs);
      std::vector<int32_t> cid(npairs);
      GP_TRY_HIP_G(hipMemcpyAsync(cnt.data(), d_cnt.p, (size_t)npairs * sizeof(int2),
                                  hipMemcpyDeviceToHost, s));
      GP_TRY_HIP_G(hipMemcpyAsync(cid.data(), g->d_cand_id, (size_t)npairs * 4,
                                  hipMemcpyDeviceToHost, s));
      GP_TRY_HIP_G(hipStreamSynchronize(s));
      std::vector<int64_t> off((size_t)npairs + 1, 0);
      for (size_t k = 0; k < npairs; ++k) {
        const int32_t f = cid[k];
        const int64_t ne = h.rvo[h.fro[f + 1]] - h.rvo[h.fro[f]];
        const int32_t nb = cnt[k].x, ng = cnt[k].y, np = (int32_t)(ne - nb - ng);
        pc[k] = make_int2(np, nb);
        off[k + 1] = off[k] + ((np + nb + 1) & ~1) + 2 * (int64_t)ng;
      }
      g->nprec = off[npairs];
      {
        // the refinement addresses a cell's records relative to its first one in 32 bits
        std::vector<int32_t> co((size_t)ncells + 1);
        GP_TRY_HIP_G(hipMemcpy(co.data(), g->d_cand_off, co.size() * 4, hipMemcpyDeviceToHost));
        for (size_t c = 0; c < (size_t)ncells; ++c)
          if (off[(size_t)co[c + 1]] - off[(size_t)co[c]] >= kMaxCount)
            return fail(set_error(GP_E_CAPACITY, "cell %zu holds 2^31 or more PIP records", c));
      }
      GP_TRY_HIP_G(hipMalloc(&g->d_prec_off, off.size() * 8));
      GP_TRY_HIP_G(hipMalloc(&g->d_pcnt, (size_t)npairs * sizeof(int2)));
      if (hipMalloc(&g->d_precs, (size_t)std::max<int64_t>(g->nprec, 1) * sizeof(float4)) !=
          hipSuccess) {
        g->d_precs = nullptr;
        return fail(set_error(GP_E_OOM, "%lld PIP records (%lld bytes) do not fit",
                              (long long)g->nprec, (long long)g->nprec * 16));
      }
      GP_TRY_HIP_G(hipMemcpyAsync(g->d_prec_off, off.data(), off.size() * 8,
                                  hipMemcpyHostToDevice, s));
      GP_TRY_HIP_G(hipMemcpyAsync(g->d_pcnt, pc.data(), (size_t)npairs * sizeof(int2),
                                  hipMemcpyHostToDevice, s));
      GP_TRY_HIP_G(launch_pip_rec_emit(skeys, g->d_cand_id, (int32_t)npairs, g->d_eoff,
                                       g->d_edge64, g->d_k32, x0, y0, cs, g->nx, hb,
                                       g->d_prec_off, g->d_pcnt, g->d_precs, s));
      GP_TRY_HIP_G(hipStreamSynchronize(s));
    }
  }
  if (kind == GP_P2P && params->p2p_segment_filter && nedges > 0) {
    // (cell, segment) pairs: every segment's box, expanded by D and padded like the MBBs,
    // rasterised and stably sorted by cell, so each cell lists its segments ascending
    const int32_t ns = (int32_t)nedges;
    DevBuf box, cnt, tmp;
    GP_TRY_HIP_G(box.alloc((size_t)ns * 32));
    GP_TRY_HIP_G(cnt.alloc(((size_t)ns + 1) * 4));
    GP_TRY_HIP_G(tmp.alloc(scan_tmp_elems(std::max((size_t)ns + 1, (size_t)ncells + 1)) * 4));
    GP_TRY_HIP_G(launch_seg_boxes(g->d_edge64, ns, D, cs * 0x1p-20, box.as<double>(), s));
    GP_TRY_HIP_G(launch_raster_count(box.as<double>(), ns, x0, y0, cs, g->nx, g->ny,
                                     cnt.as<uint32_t>(), s));
    const int64_t total = pair_total(cnt.as<uint32_t>(), (size_t)ns, s);
    if (total < 0) return fail(GP_E_HIP);
    if (total >= kMaxCount)
      return fail(set_error(GP_E_CAPACITY, "%lld (cell, segment) pairs exceed 2^31 - 1",
                            (long long)total));
    GP_TRY_HIP_G(launch_exclusive_scan_u32(cnt.as<uint32_t>(), cnt.as<uint32_t>(),
                                           (size_t)ns + 1, tmp.as<uint32_t>(), s));
    const uint32_t np2 = (uint32_t)total;
    g->ncseg = np2;
    const size_t n2 = std::max<size_t>(np2, 1);
    DevBuf kA, kB, vA, vB, hist, stmp;
    GP_TRY_HIP_G(kA.alloc(n2 * 4));
    GP_TRY_HIP_G(kB.alloc(n2 * 4));
    GP_TRY_HIP_G(vA.alloc(n2 * 4));
    GP_TRY_HIP_G(vB.alloc(n2 * 4));
    GP_TRY_HIP_G(hist.alloc(radix_hist_elems(n2) * 4));
    GP_TRY_HIP_G(stmp.alloc(scan_tmp_elems(std::max(radix_hist_elems(n2), (size_t)ncells + 1)) * 4));
    GP_TRY_HIP_G(launch_raster_emit(box.as<double>(), ns, x0, y0, cs, g->nx, g->ny,
                                    cnt.as<uint32_t>(), kA.as<uint32_t>(), vA.as<uint32_t>(), s));
    uint32_t *skeys = nullptr, *svals = nullptr;
    GP_TRY_HIP_G(launch_radix_sort(kA.as<uint32_t>(), kB.as<uint32_t>(), vA.as<uint32_t>(),
                                   vB.as<uint32_t>(), np2, bits_for((uint64_t)ncells - 1), false,
                                   hist.as<uint32_t>(), stmp.as<uint32_t>(), s, &skeys, &svals));
    GP_TRY_HIP_G(hipMalloc(&g->d_cseg_off, ((size_t)ncells + 1) * 4));
    GP_TRY_HIP_G(hipMalloc(&g->d_cseg, n2 * 4));
    GP_TRY_HIP_G(hipMalloc(&g->d_seg2f, (size_t)ns * 4));
    GP_TRY_HIP_G(hipMalloc(&g->d_cell_segs, std::max<size_t>(ncells, 1) * 8));
    GP_TRY_HIP_G(launch_fill_u32((uint32_t *)g->d_cseg_off, 0u, (size_t)ncells + 1, s));
    GP_TRY_HIP_G(launch_histogram(skeys, np2, (uint32_t *)g->d_cseg_off, s));
    GP_TRY_HIP_G(launch_exclusive_scan_u32((uint32_t *)g->d_cseg_off, (uint32_t *)g->d_cseg_off,
                                           (size_t)ncells + 1, stmp.as<uint32_t>(), s));
    if (np2)
      GP_TRY_HIP_G(hipMemcpyAsync(g->d_cseg, svals, (size_t)np2 * 4, hipMemcpyDeviceToDevice, s));
    GP_TRY_HIP_G(launch_seg2f(g->d_eoff, (int32_t)nf, g->d_seg2f, s));
    GP_TRY_HIP_G(launch_cell_counts(g->d_cseg_off, ncells, g->d_cell_segs, s));
    GP_TRY_HIP_G(hipStreamSynchronize(s));
  }
  if (kind == GP_P2P && params->prestage && !params->p2p_segment_filter && nedges > 0) {
    // every cell's segment records, in the order the refinement reads them, at offsets
    // from the prefix sum of the cells' candidate segment counts
    std::vector<int64_t> off((size_t)ncells + 1);
    GP_TRY_HIP_G(hipMemcpyAsync(off.data() + 1, g->d_cell_edges, (size_t)ncells * 8,
                                hipMemcpyDeviceToHost, s));
    GP_TRY_HIP_G(hipStreamSynchronize(s));
    off[0] = 0;
    for (size_t c = 1; c <= (size_t)ncells; ++c) off[c] += off[c - 1];
    g->nrec = off[(size_t)ncells];
    const size_t nrec = (size_t)std::max<int64_t>(g->nrec, 1);
    GP_TRY_HIP_G(hipMalloc(&g->d_rec_off, off.size() * 8));
    GP_TRY_HIP_G(hipMalloc(&g->d_recU, nrec * sizeof(float4)));
    GP_TRY_HIP_G(hipMalloc(&g->d_recV, nrec * sizeof(float)));
    GP_TRY_HIP_G(hipMalloc(&g->d_cellE, (size_t)ncells * sizeof(float2)));
    GP_TRY_HIP_G(hipMemcpyAsync(g->d_rec_off, off.data(), off.size() * 8, hipMemcpyHostToDevice, s));
    GP_TRY_HIP_G(launch_prestage(g->d_cand_off, g->d_cand_id, g->d_eoff, g->d_frame64,
                                 g->d_frame32, g->x0, g->y0, g->cs, g->nx, ncells, g->D,
                                 half_box(*g), p2p_margin(*g), g->p2p_scale, g->d_rec_off,
                                 g->d_recU, g->d_recV, g->d_cellE, s));
    GP_TRY_HIP_G(hipStreamSynchronize(s));
  }
#undef GP_TRY_HIP_G
  *out = g;
  return GP_OK;
}

extern "C" void gp_grid_free(gp_grid *g) {
  if (!g) return;
  (void)hipFree(g->d_eoff);
  (void)hipFree(g->d_edge64);
  (void)hipFree(g->d_k32);
  (void)hipFree(g->d_frame64);
  (void)hipFree(g->d_frame32);
  (void)hipFree(g->d_circ);
  (void)hipFree(g->d_cand_off);
  (void)hipFree(g->d_cand_id);
  (void)hipFree(g->d_cell_edges);
  (void)hipFree(g->d_cell_edges_all);
  (void)hipFree(g->d_cand_class);
  (void)hipFree(g->d_cseg_off);
  (void)hipFree(g->d_cseg);
  (void)hipFree(g->d_seg2f);
  (void)hipFree(g->d_cell_segs);
  (void)hipFree(g->d_near);
  (void)hipFree(g->d_rec_off);
  (void)hipFree(g->d_recU);
  (void)hipFree(g->d_recV);
  (void)hipFree(g->d_cellE);
  (void)hipFree(g->d_precs);
  (void)hipFree(g->d_prec_off);
  (void)hipFree(g->d_pcnt);
  delete g;
}

// Device bytes held by a grid (the allocations of gp_build_grid).
static int64_t grid_device_bytes(const Grid &g) {
  const int64_t ne = std::max<int64_t>(g.nedges, 1), nc = std::max<int64_t>(g.ncells, 1);
  const int64_t np = std::max<int64_t>(g.npairs, 1);
  int64_t b = ((int64_t)g.nf + 1) * 4 + ne * (32 + 4) + (nc + 1) * 4 + np * 4 + nc * 8;
  if (g.kind == GP_P2P) b += ne * (32 + 16) + (ne + P2P_BLOCK - 1) / P2P_BLOCK * 32 + np * 8;
  if (g.d_cand_class) b += np + nc * 8;
  if (g.d_cseg_off) b += (nc + 1) * 4 + std::max<int64_t>(g.ncseg, 1) * 4 + ne * 4 + nc * 8;
  if (g.d_recU) b += (nc + 1) * 8 + std::max<int64_t>(g.nrec, 1) * 20 + nc * 8;
  if (g.d_precs) b += (np + 1) * 8 + np * 8 + std::max<int64_t>(g.nprec, 1) * 16;
  return b;
}

extern "C" gp_status gp_grid_get_info(const gp_grid *g, gp_grid_info *info) {
  if (!g || !info) return set_error(GP_E_INVALID_ARG, "null argument");
  info->kind = g->kind;
  info->x0 = g->x0;
  info->y0 = g->y0;
  info->cell_size = g->cs;
  info->radius_D = g->D;
  info->nx = g->nx;
  info->ny = g->ny;
  info->n_features = g->nf;
  info->n_edges = g->nedges;
  info->n_pairs = g->npairs;
  info->n_pairs_outside = g->npairs_class[0];
  info->n_pairs_inside = g->npairs_class[1];
  info->n_pairs_boundary = g->d_cand_class ? g->npairs_class[2] : 0;
  info->device_bytes = grid_device_bytes(*g);
  info->n_segment_pairs = g->ncseg;
  return GP_OK;
}

extern "C" gp_status gp_grid_candidates(const gp_grid *g, int32_t *cand_off, int32_t *cand_id) {
  if (!g || !cand_off || (!cand_id && g->npairs)) return set_error(GP_E_INVALID_ARG, "null argument");
  GP_TRY_HIP(hipMemcpy(cand_off, g->d_cand_off, ((size_t)g->ncells + 1) * 4, hipMemcpyDeviceToHost));
  if (g->npairs)
    GP_TRY_HIP(hipMemcpy(cand_id, g->d_cand_id, (size_t)g->npairs * 4, hipMemcpyDeviceToHost));
  return GP_OK;
}

// ------------------------------------------------------------------------- workspace

static int64_t max_items(const Grid &g, int64_t n) {
  return n / 64 + std::min<int64_t>(g.ncells, n) + 1;
}

namespace gp {
size_t workspace_layout(const Grid &g, int64_t n, gp_precision prec, void *base, Workspace *ws) {
  size_t off = 0;
  auto take = [&](size_t bytes) -> void * {
    size_t o = off;
    off = align_up(off + std::max<size_t>(bytes, 16), 256);
    return base ? (void *)((char *)base + o) : nullptr;
  };
  const size_t un = (size_t)std::max<int64_t>(n, 1);
  const size_t mi = (size_t)max_items(g, n);
  const size_t hist = radix_hist_elems(std::max(un, mi));
  const size_t nc1 = (size_t)g.ncells + 1;
  Workspace w;
  w.keyA = (uint32_t *)take(un * 4);
  w.keyB = (uint32_t *)take(un * 4);
  w.valA = (uint32_t *)take(un * 4);
  w.valB = (uint32_t *)take(un * 4);
  w.hist = (uint32_t *)take(hist * 4);
  w.scan_tmp = (uint32_t *)take(scan_tmp_elems(std::max(hist, nc1)) * 4);
  w.pt_off = (int32_t *)take(nc1 * 4);
  w.item_cnt = (uint32_t *)take(nc1 * 4);
  w.items = (Item *)take(mi * sizeof(Item));
  if (g.kind == GP_PIP) {
    w.ikA = (uint32_t *)take(mi * 4);
    w.ikB = (uint32_t *)take(mi * 4);
    w.ivA = (uint32_t *)take(mi * 4);
    w.ivB = (uint32_t *)take(mi * 4);
    w.items_sorted = (Item *)take(mi * sizeof(Item));
  } else {
    w.ikA = w.ikB = w.ivA = w.ivB = nullptr;
    w.items_sorted = nullptr;
  }
  w.vp_list = g.kind == GP_P2P ? (uint32_t *)take(mi * 4) : nullptr;
  w.counters = (uint32_t *)take(C_COUNT * 4);
  w.tests = (unsigned long long *)take(16);
  w.xyA = (double2 *)take(un * 16);
  w.xyB = (double2 *)take(un * 16);
  w.rq = prec == GP_MIXED ? (uint32_t *)take(un * 4) : nullptr;
  w.bytes = off;
  if (ws) *ws = w;
  return off;
}
}  // namespace gp

extern "C" gp_status gp_workspace_bytes(const gp_grid *g, int64_t n, gp_precision prec,
                                        size_t *bytes) {
  if (!g || !bytes) return set_error(GP_E_INVALID_ARG, "null argument");
  if (n < 0 || n >= kMaxCount) return set_error(GP_E_CAPACITY, "n must be in [0, 2^31)");
  if (prec != GP_FP64 && prec != GP_MIXED) return set_error(GP_E_INVALID_ARG, "bad precision");
  *bytes = workspace_layout(*g, n, prec, nullptr, nullptr);
  return GP_OK;
}

// ------------------------------------------------------------------------- queries

namespace gp {

struct QueryPlan {
  RefineArgs a;
  Workspace w;
  uint32_t *perm;
  int32_t nbits;
};

// Hash, sort and offsets: the point side of the filter.  With xy != NULL the FP64
// points travel through the sort and *xy receives them in sorted order.
static hipError_t pair_points(const Grid &g, int64_t n, const double *px, const double *py,
                              Workspace &w, hipStream_t s, uint32_t **skey, uint32_t **perm,
                              double2 **xy) {
  hipError_t e = launch_hash(px, py, n, g.x0, g.y0, g.cs, g.nx, g.ny, w.keyA, s);
  if (e != hipSuccess) return e;
  e = launch_radix_sort(w.keyA, w.keyB, w.valA, w.valB, (size_t)n, bits_for((uint64_t)g.ncells),
                        true, w.hist, w.scan_tmp, s, skey, perm, px, py, w.xyA, w.xyB, xy);
  if (e != hipSuccess) return e;
  return launch_offsets(*skey, n, g.ncells, w.pt_off, s);
}

static gp_status run_query(const gp_grid *g, gp_kind kind, int64_t n, const double *px,
                           const double *py, int32_t *out_id, double *out_dist,
                           gp_precision prec, void *ws, size_t ws_bytes, hipStream_t s,
                           gp_stats *stats, const gp_tuning *override_tuning) {
  if (!g) return set_error(GP_E_INVALID_ARG, "null grid");
  if (g->kind != kind)
    return set_error(GP_E_INVALID_ARG, "grid was built for the other operation");
  if (prec != GP_FP64 && prec != GP_MIXED) return set_error(GP_E_INVALID_ARG, "bad precision");
  if (n < 0 || n >= kMaxCount) return set_error(GP_E_CAPACITY, "n must be in [0, 2^31)");
  if (stats) memset(stats, 0, sizeof(*stats));
  if (n == 0) return GP_OK;
  if (!px || !py || !out_id || (kind == GP_P2P && !out_dist))
    return set_error(GP_E_INVALID_ARG, "null point or output pointer");
  int cur = 0;
  if (hipGetDevice(&cur) != hipSuccess || cur != g->device)
    return set_error(GP_E_INVALID_ARG, "the grid lives on device %d; make it current", g->device);
  Workspace w;
  const size_t need = workspace_layout(*g, n, prec, ws, &w);
  if (!ws || ws_bytes < need)
    return set_error(GP_E_INVALID_ARG, "workspace too small: %zu bytes needed", need);
  gp_tuning t = override_tuning ? *override_tuning : g->tune[prec];
  // The library default's persistent queue has a cost at the end of every launch (each
  // workgroup finds the queues empty) that only a large query amortises: below
  // kPersistentMinPoints the default runs one workgroup per item instead.
  if (!override_tuning && !g->tune_explicit[prec]) {
    if (n < kPersistentMinPoints) t.persistent = 0;
    if (t.points_per_lane > 2 && n < kFourPerLaneMinPointsPerCell * g->ncells)
      t.points_per_lane = 2;
  }
  if (!tuning_valid(t, g->kind)) return set_error(GP_E_INVALID_ARG, "invalid tuning");

  hipEvent_t ev[5] = {};
  if (stats) {
    for (auto &e : ev) GP_TRY_HIP(hipEventCreate(&e));
    GP_TRY_HIP(hipEventRecord(ev[0], s));
  }
  GP_TRY_HIP(launch_fill_u32(w.counters, 0u, C_COUNT, s));
  GP_TRY_HIP(launch_fill_u32((uint32_t *)w.tests, 0u, 4, s));
  uint32_t *skey = nullptr, *perm = nullptr;
  double2 *xy = nullptr;
  GP_TRY_HIP(pair_points(*g, n, px, py, w, s, &skey, &perm, &xy));

  RefineArgs a;
  memset(&a, 0, sizeof(a));
  a.items = w.items;
  a.n_items = w.item_cnt + g->ncells;
  a.item_counter = w.counters + C_ITEM;
  a.cand_off = g->d_cand_off;
  a.cand_id = g->d_cand_id;
  a.eoff = g->d_eoff;
  a.edge64 = g->d_edge64;
  a.k32 = g->d_k32;
  a.frame64 = g->d_frame64;
  a.frame32 = g->d_frame32;
  a.circ = g->d_circ;
  a.near = g->d_near;
  a.cand_class = g->d_cand_class;
  const bool segf = prec == GP_MIXED && g->d_cseg_off != nullptr;
  a.cseg_off = segf ? g->d_cseg_off : nullptr;
  a.cseg = segf ? g->d_cseg : nullptr;
  a.seg2f = segf ? g->d_seg2f : nullptr;
  const bool pre = prec == GP_MIXED && !segf && g->d_recU != nullptr;
  a.recU = pre ? g->d_recU : nullptr;
  a.recV = pre ? g->d_recV : nullptr;
  a.rec_off = pre ? g->d_rec_off : nullptr;
  a.cellE = pre ? g->d_cellE : nullptr;
  const bool pip_pre = prec == GP_MIXED && g->d_precs != nullptr;
  a.precs = pip_pre ? g->d_precs : nullptr;
  a.prec_off = pip_pre ? g->d_prec_off : nullptr;
  a.pcnt = pip_pre ? g->d_pcnt : nullptr;
  a.x0 = g->x0;
  a.y0 = g->y0;
  a.cs = g->cs;
  a.nx = g->nx;
  a.ncells = g->ncells;
  a.D = g->D;
  a.D2 = g->D2;
  a.D2_next = std::nextafter(g->D2, INFINITY);
  a.half_box = half_box(*g);
  a.p2p_margin = p2p_margin(*g);
  a.p2p_scale = g->p2p_scale;
  a.skey = skey;
  a.perm = perm;
  a.xy = xy;
  a.out_id = out_id;
  a.out_dist = kind == GP_P2P ? out_dist : nullptr;
  a.rq = w.rq;
  a.rq_count = w.counters + C_RQ;
  a.edge_chunk = t.edge_chunk;
  a.vp_points = t.vp_points;
  a.vp_list = w.vp_list;
  a.vp_count = w.counters + C_NVP;

  GP_TRY_HIP(launch_unpaired(a, n, w.counters + C_NPAIRED, s));
  GP_TRY_HIP(launch_items(w.pt_off, g->d_cand_off, segf ? g->d_cell_segs : g->d_cell_edges,
                          segf ? g->d_cell_edges : g->d_cell_edges_all, g->ncells,
                          64 * t.points_per_lane * t.waves_per_item, w.item_cnt, w.scan_tmp,
                          w.items, w.counters, w.tests, s));
  const int64_t mi = n / (64 * t.points_per_lane * t.waves_per_item) +
                    std::min<int64_t>(g->ncells, n) + 1;
  if (kind == GP_PIP) {
    // PIP items run one workgroup each: longest first, so the items of cells under the
    // largest polygons start early and the launch does not end on them
    GP_TRY_HIP(launch_order_items(w.items, a.n_items, mi, g->d_cell_edges, w.ikA, w.ikB, w.ivA,
                                  w.ivB, w.hist, w.scan_tmp, w.items_sorted, s));
    a.items = w.items_sorted;
  }
  if (stats) GP_TRY_HIP(hipEventRecord(ev[1], s));
  GP_TRY_HIP(launch_refine(kind, prec, a, t, g->num_cu, mi, s));
  if (stats) GP_TRY_HIP(hipEventRecord(ev[2], s));
  if (prec == GP_MIXED) GP_TRY_HIP(launch_recheck(kind, a, g->num_cu, s));
  if (stats) {
    GP_TRY_HIP(hipEventRecord(ev[3], s));
    GP_TRY_HIP(hipEventSynchronize(ev[3]));
    uint32_t cnt[C_COUNT];
    unsigned long long tests[2] = {0, 0};
    uint32_t nitems = 0;
    GP_TRY_HIP(hipMemcpy(cnt, w.counters, sizeof(cnt), hipMemcpyDeviceToHost));
    GP_TRY_HIP(hipMemcpy(tests, w.tests, 16, hipMemcpyDeviceToHost));
    GP_TRY_HIP(hipMemcpy(&nitems, a.n_items, 4, hipMemcpyDeviceToHost));
    float m01 = 0, m12 = 0, m23 = 0, m03 = 0;
    GP_TRY_HIP(hipEventElapsedTime(&m01, ev[0], ev[1]));
    GP_TRY_HIP(hipEventElapsedTime(&m12, ev[1], ev[2]));
    GP_TRY_HIP(hipEventElapsedTime(&m23, ev[2], ev[3]));
    GP_TRY_HIP(hipEventElapsedTime(&m03, ev[0], ev[3]));
    stats->n_points = n;
    stats->n_paired = cnt[C_NPAIRED];
    stats->n_items = nitems;
    stats->tests = tests[0];
    stats->tests_avoided = (g->d_cell_edges_all || segf) ? tests[1] - tests[0] : 0;
    stats->n_rechecked = prec == GP_MIXED ? cnt[C_RQ] : 0;
    stats->ms_pairing = m01;
    stats->ms_refine = m12;
    stats->ms_recheck = m23;
    stats->ms_total = m03;
    for (auto &e : ev) (void)hipEventDestroy(e);
  }
  return GP_OK;
}

gp_status run_query_tuned(const gp_grid *g, gp_kind kind, int64_t n, const double *px,
                          const double *py, int32_t *out_id, double *out_dist,
                          gp_precision prec, void *ws, size_t ws_bytes, hipStream_t s,
                          gp_stats *stats, const gp_tuning *t) {
  return run_query(g, kind, n, px, py, out_id, out_dist, prec, ws, ws_bytes, s, stats, t);
}

}  // namespace gp

extern "C" gp_status gp_pair_points(const gp_grid *g, int64_t n, const double *px,
                                    const double *py, int32_t *perm_out, int32_t *pt_off_out,
                                    void *ws, size_t ws_bytes, void *hip_stream) {
  if (!g) return set_error(GP_E_INVALID_ARG, "null grid");
  if (n < 0 || n >= kMaxCount) return set_error(GP_E_CAPACITY, "n must be in [0, 2^31)");
  if (!pt_off_out || (n > 0 && (!px || !py || !perm_out)))
    return set_error(GP_E_INVALID_ARG, "null pointer");
  Workspace w;
  const size_t need = workspace_layout(*g, n, GP_FP64, ws, &w);
  if (!ws || ws_bytes < need)
    return set_error(GP_E_INVALID_ARG, "workspace too small: %zu bytes needed", need);
  hipStream_t s = (hipStream_t)hip_stream;
  uint32_t *skey = w.keyA, *perm = w.valA;
  if (n > 0) GP_TRY_HIP(pair_points(*g, n, px, py, w, s, &skey, &perm, nullptr));
  else GP_TRY_HIP(launch_offsets(skey, 0, g->ncells, w.pt_off, s));
  GP_TRY_HIP(launch_copy_perm(perm, n, perm_out, s));
  GP_TRY_HIP(hipMemcpyAsync(pt_off_out, w.pt_off, ((size_t)g->ncells + 1) * 4,
                            hipMemcpyDeviceToDevice, s));
  return GP_OK;
}

extern "C" gp_status gp_pip(const gp_grid *g, int64_t n, const double *px, const double *py,
                            int32_t *out_id, gp_precision prec, void *ws, size_t ws_bytes,
                            void *hip_stream, gp_stats *stats) {
  return run_query(g, GP_PIP, n, px, py, out_id, nullptr, prec, ws, ws_bytes,
                   (hipStream_t)hip_stream, stats, nullptr);
}

extern "C" gp_status gp_p2p(const gp_grid *g, int64_t n, const double *px, const double *py,
                            int32_t *out_id, double *out_dist, gp_precision prec, void *ws,
                            size_t ws_bytes, void *hip_stream, gp_stats *stats) {
  return run_query(g, GP_P2P, n, px, py, out_id, out_dist, prec, ws, ws_bytes,
                   (hipStream_t)hip_stream, stats, nullptr);
}

// ------------------------------------------------------------------------- tuning

extern "C" gp_status gp_set_tuning(gp_grid *g, gp_precision prec, const gp_tuning *t) {
  if (!g) return set_error(GP_E_INVALID_ARG, "null argument");
  if (prec != GP_FP64 && prec != GP_MIXED) return set_error(GP_E_INVALID_ARG, "bad precision");
  if (!t) {  // back to the library default
    g->tune[prec] = default_tuning(g->kind, prec);
    g->tune_explicit[prec] = false;
    return GP_OK;
  }
  gp_tuning v = *t;
  gp_tuning d = default_tuning(g->kind, prec);
  if (v.points_per_lane == 0) v.points_per_lane = d.points_per_lane;
  if (v.edge_chunk == 0) v.edge_chunk = d.edge_chunk;
  if (v.wg_per_cu == 0) v.wg_per_cu = d.wg_per_cu;
  if (v.waves_per_item == 0) v.waves_per_item = d.waves_per_item;
  if (v.vp_points == 0) v.vp_points = d.vp_points;
  if (!tuning_valid(v, g->kind)) return set_error(GP_E_INVALID_ARG, "invalid tuning");
  g->tune[prec] = v;
  g->tune_explicit[prec] = true;
  return GP_OK;
}

extern "C" gp_status gp_get_tuning(const gp_grid *g, gp_precision prec, gp_tuning *t) {
  if (!g || !t) return set_error(GP_E_INVALID_ARG, "null argument");
  if (prec != GP_FP64 && prec != GP_MIXED) return set_error(GP_E_INVALID_ARG, "bad precision");
  *t = g->tune[prec];
  return GP_OK;
}

// ------------------------------------------------------------------------- tuning cache
// Winners of gp_autotune by (operation, precision, GPU architecture, grid records, workload
// class); the class is the octave of the sample size, of the tests per paired point and of
// the paired points per work item under the library default tuning.  A text line per entry:
// the key, a tab, then points_per_lane edge_chunk wg_per_cu persistent waves_per_item
// vp_points.

namespace {
std::mutex g_tune_mu;
std::map<std::string, gp_tuning> g_tune_cache;

int octave(double v) { return v >= 1.0 ? (int)std::floor(std::log2(v)) : 0; }
}  // namespace

static std::string device_arch(int dev) {
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return "unknown";
  std::string a = prop.gcnArchName;
  const size_t c = a.find(':');
  return c == std::string::npos ? a : a.substr(0, c);
}

static std::string tune_key(const Grid &g, gp_precision prec, int64_t n, const gp_stats &st) {
  char buf[256];
  const double paired = (double)std::max<int64_t>(st.n_paired, 1);
  snprintf(buf, sizeof(buf), "%s %s %s rec=%d seg=%d cls=%d n=%d tpp=%d ppi=%d",
           g.kind == GP_PIP ? "pip" : "p2p", prec == GP_MIXED ? "mixed" : "fp64",
           device_arch(g.device).c_str(), (g.d_precs || g.d_recU) ? 1 : 0,
           g.d_cseg_off ? 1 : 0, g.d_cand_class ? 1 : 0, octave((double)n),
           octave((double)st.tests / paired), octave(paired / (double)std::max<int64_t>(st.n_items, 1)));
  return buf;
}

extern "C" gp_status gp_tuning_cache_clear(void) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_tune_cache.clear();
  return GP_OK;
}

extern "C" gp_status gp_tuning_cache_size(int64_t *entries) {
  if (!entries) return set_error(GP_E_INVALID_ARG, "null argument");
  std::lock_guard<std::mutex> lk(g_tune_mu);
  *entries = (int64_t)g_tune_cache.size();
  return GP_OK;
}

extern "C" gp_status gp_tuning_cache_save(const char *path) {
  if (!path) return set_error(GP_E_INVALID_ARG, "null path");
  FILE *f = fopen(path, "w");
  if (!f) return set_error(GP_E_INVALID_ARG, "cannot write %s", path);
  std::lock_guard<std::mutex> lk(g_tune_mu);
  for (const auto &kv : g_tune_cache) {
    const gp_tuning &t = kv.second;
    fprintf(f, "%s\t%d %d %d %d %d %d\n", kv.first.c_str(), t.points_per_lane, t.edge_chunk,
            t.wg_per_cu, t.persistent, t.waves_per_item, t.vp_points);
  }
  const bool ok = fclose(f) == 0;
  return ok ? GP_OK : set_error(GP_E_INVALID_ARG, "cannot write %s", path);
}

// Adds the file's entries to the cache (replacing equal keys).  Nothing is added when a
// line is malformed or holds an invalid tuning.
extern "C" gp_status gp_tuning_cache_load(const char *path) {
  if (!path) return set_error(GP_E_INVALID_ARG, "null path");
  FILE *f = fopen(path, "r");
  if (!f) return set_error(GP_E_INVALID_ARG, "cannot read %s", path);
  std::map<std::string, gp_tuning> add;
  char line[512];
  int lineno = 0;
  gp_status st = GP_OK;
  while (fgets(line, sizeof(line), f)) {
    ++lineno;
    std::string l(line);
    while (!l.empty() && (l.back() == '\n' || l.back() == '\r')) l.pop_back();
    if (l.empty()) continue;
    const size_t tab = l.find('\t');
    gp_tuning t;
    char tail = 0;
    if (tab == std::string::npos || tab == 0 ||
        sscanf(l.c_str() + tab + 1, "%d %d %d %d %d %d %c", &t.points_per_lane, &t.edge_chunk,
               &t.wg_per_cu, &t.persistent, &t.waves_per_item, &t.vp_points, &tail) != 6) {
      st = set_error(GP_E_INVALID_ARG, "%s:%d: malformed tuning cache line", path, lineno);
      break;
    }
    const std::string key = l.substr(0, tab);
    const gp_kind kind = key.rfind("pip ", 0) == 0 ? GP_PIP : key.rfind("p2p ", 0) == 0 ? GP_P2P
                                                                                       : (gp_kind)0;
    if (!kind || !tuning_valid(t, kind)) {
      st = set_error(GP_E_INVALID_ARG, "%s:%d: invalid tuning cache entry", path, lineno);
      break;
    }
    add[key] = t;
  }
  fclose(f);
  if (st) return st;
  std::lock_guard<std::mutex> lk(g_tune_mu);
  for (const auto &kv : add) g_tune_cache[kv.first] = kv.second;
  return GP_OK;
}

static gp_status autotune_search(gp_grid *g, gp_precision prec, int64_t n, const double *px,
                                 const double *py, int32_t *id, double *dist, void *ws,
                                 size_t ws_bytes, hipStream_t s, gp_tuning *best,
                                 float *best_ms);

// Median of three timed queries (after one untimed) of one configuration.
static gp_status time_config(gp_grid *g, gp_precision prec, int64_t n, const double *px,
                             const double *py, int32_t *id, double *dist, void *ws,
                             size_t ws_bytes, hipStream_t s, const gp_tuning &t, float *ms,
                             gp_stats *first) {
  float times[3];
  for (int r = 0; r < 4; ++r) {
    gp_stats st;
    gp_status rc = run_query(g, g->kind, n, px, py, id, dist, prec, ws, ws_bytes, s, &st, &t);
    if (rc) return rc;
    if (r == 0 && first) *first = st;
    if (r > 0) times[r - 1] = st.ms_total;
  }
  std::sort(times, times + 3);
  *ms = times[1];
  return GP_OK;
}

// Grid search over points per lane, LDS edge chunk, persistent workgroups per CU and the
// queue mode; each configuration is timed (median of 3 after one warm-up) on the sample.
// A cached winner for the sample's workload class is taken without the search.
extern "C" gp_status gp_autotune(gp_grid *g, gp_precision prec, int64_t n, const double *px,
                                 const double *py, void *ws, size_t ws_bytes, void *hip_stream,
                                 gp_tuning *best, float *best_ms) {
  if (!g) return set_error(GP_E_INVALID_ARG, "null grid");
  if (prec != GP_FP64 && prec != GP_MIXED) return set_error(GP_E_INVALID_ARG, "bad precision");
  if (n <= 0) return set_error(GP_E_INVALID_ARG, "autotune needs sample points");
  hipStream_t s = (hipStream_t)hip_stream;
  DevBuf d_id, d_dist;
  GP_TRY_HIP(d_id.alloc((size_t)n * 4));
  GP_TRY_HIP(d_dist.alloc((size_t)n * 8));
  {
    // the workload class, from a query with the library default
    const gp_tuning def = default_tuning(g->kind, prec);
    gp_stats st0;
    float ms0 = 0.f;
    gp_status rc = time_config(g, prec, n, px, py, d_id.as<int32_t>(), d_dist.as<double>(), ws,
                               ws_bytes, s, def, &ms0, &st0);
    if (rc) return rc;
    const std::string key = tune_key(*g, prec, n, st0);
    gp_tuning hit;
    bool found = false;
    {
      std::lock_guard<std::mutex> lk(g_tune_mu);
      auto it = g_tune_cache.find(key);
      if (it != g_tune_cache.end()) {
        hit = it->second;
        found = true;
      }
    }
    if (found) {
      float ms = 0.f;
      rc = time_config(g, prec, n, px, py, d_id.as<int32_t>(), d_dist.as<double>(), ws,
                       ws_bytes, s, hit, &ms, nullptr);
      if (rc) return rc;
      g->tune[prec] = hit;
      g->tune_explicit[prec] = true;
      if (best) *best = hit;
      if (best_ms) *best_ms = ms;
      return GP_OK;
    }
    rc = autotune_search(g, prec, n, px, py, d_id.as<int32_t>(), d_dist.as<double>(), ws,
                         ws_bytes, s, best, best_ms);
    if (rc) return rc;
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune_cache[key] = g->tune[prec];
    return GP_OK;
  }
}

static gp_status autotune_search(gp_grid *g, gp_precision prec, int64_t n, const double *px,
                                 const double *py, int32_t *id, double *dist, void *ws,
                                 size_t ws_bytes, hipStream_t s, gp_tuning *best,
                                 float *best_ms) {
  std::vector<gp_tuning> space;
  const int ppls[3] = {1, 2, 4}, wgs[4] = {8, 12, 16, 32};
  // the mixed PIP refinement over build-time records streams chunks of a fixed size, so
  // the LDS chunk is no axis there
  const bool fixed_chunk = g->kind == GP_PIP && prec == GP_MIXED && g->d_precs != nullptr;
  const std::vector<int> ecs =
      fixed_chunk ? std::vector<int>{128} : std::vector<int>{128, 256, 512};
  for (int p : ppls)
    for (int e : ecs)
      for (int wgc : wgs) space.push_back(gp_tuning{p, e, wgc, 1, 1, 0});
  for (int p : ppls)
    for (int e : ecs) space.push_back(gp_tuning{p, e, 16, 0, 1, 0});
  if (g->kind == GP_P2P)
    for (int wv : {2, 4})
      for (int p : ppls)
        for (int e : ecs)
          for (int wgc : {4, 8, 16}) space.push_back(gp_tuning{p, e, wgc, 1, wv, 0});
  const int vp_default = default_tuning(g->kind, prec).vp_points;
  for (gp_tuning &t : space) t.vp_points = vp_default;
  float best_t = INFINITY;
  gp_tuning best_cfg = g->tune[prec];
  auto consider = [&](const gp_tuning &t) -> gp_status {
    float ms = 0.f;
    gp_status rc = time_config(g, prec, n, px, py, id, dist, ws, ws_bytes, s, t, &ms, nullptr);
    if (!rc && ms < best_t) {
      best_t = ms;
      best_cfg = t;
    }
    return rc;
  };
  for (const gp_tuning &t : space) {
    gp_status rc = consider(t);
    if (rc) return rc;
  }
  {
    // then the vertex-parallel threshold, on the best configuration (P2P: one-wave items)
    for (int vp : {-1, 4, 8, 16, 32, 64}) {
      if (vp == best_cfg.vp_points || (g->kind == GP_P2P && best_cfg.waves_per_item != 1))
        continue;
      gp_tuning t = best_cfg;
      t.vp_points = vp;
      gp_status rc = consider(t);
      if (rc) return rc;
    }
  }
  g->tune[prec] = best_cfg;
  g->tune_explicit[prec] = true;
  if (best) *best = best_cfg;
  if (best_ms) *best_ms = best_t;
  return GP_OK;
}

extern "C" gp_status gp_sweep_cell_size(gp_kind kind, const gp_geometry *geom,
                                        const gp_grid_params *params, const double *cell_sizes,
                                        int32_t n_sizes, int64_t n, const double *px,
                                        const double *py, gp_precision prec, void *hip_stream,
                                        double *best, float *ms_query, int64_t *n_pairs,
                                        uint64_t *tests, int64_t *grid_bytes) {
  if (!geom || !params || !cell_sizes || n_sizes <= 0 || n <= 0 || !px || !py)
    return set_error(GP_E_INVALID_ARG, "bad sweep arguments");
  if (prec != GP_FP64 && prec != GP_MIXED) return set_error(GP_E_INVALID_ARG, "bad precision");
  for (int32_t i = 0; i < n_sizes; ++i)
    if (!(cell_sizes[i] > 0.0) || !std::isfinite(cell_sizes[i]))
      return set_error(GP_E_INVALID_ARG, "cell sizes must be finite and > 0");
  hipStream_t s = (hipStream_t)hip_stream;
  DevBuf d_id, d_dist;
  GP_TRY_HIP(d_id.alloc((size_t)n * 4));
  GP_TRY_HIP(d_dist.alloc((size_t)n * 8));
  const bool derive = params->nx == 0 || params->ny == 0;
  double best_cs = NAN;
  float best_t = INFINITY;
  for (int32_t i = 0; i < n_sizes; ++i) {
    gp_grid_params p = *params;
    p.cell_size = cell_sizes[i];
    if (!derive) {
      p.nx = (int64_t)std::ceil((double)params->nx * params->cell_size / p.cell_size);
      p.ny = (int64_t)std::ceil((double)params->ny * params->cell_size / p.cell_size);
    }
    if (ms_query) ms_query[i] = NAN;
    if (n_pairs) n_pairs[i] = -1;
    if (tests) tests[i] = 0;
    if (grid_bytes) grid_bytes[i] = -1;
    gp_grid *g = nullptr;
    gp_status rc = gp_build_grid(kind, geom, &p, hip_stream, &g);
    if (rc == GP_E_CAPACITY) continue;  // this size exceeds the limits: skipped
    if (rc) return rc;
    size_t wsb = 0;
    rc = gp_workspace_bytes(g, n, prec, &wsb);
    DevBuf ws;
    if (!rc && ws.alloc(wsb) != hipSuccess) rc = set_error(GP_E_OOM, "sweep workspace");
    float times[3] = {0, 0, 0};
    gp_stats st;
    for (int r = 0; r < 4 && !rc; ++r) {
      rc = run_query(g, kind, n, px, py, d_id.as<int32_t>(), d_dist.as<double>(), prec, ws.p,
                     wsb, s, &st, nullptr);
      if (r > 0) times[r - 1] = st.ms_total;
    }
    if (!rc) {
      std::sort(times, times + 3);
      if (ms_query) ms_query[i] = times[1];
      if (n_pairs) n_pairs[i] = g->npairs;
      if (tests) tests[i] = st.tests;
      if (grid_bytes) grid_bytes[i] = grid_device_bytes(*g);
      if (times[1] < best_t) {
        best_t = times[1];
        best_cs = cell_sizes[i];
      }
    }
    gp_grid_free(g);
    if (rc) return rc;
  }
  if (best) *best = best_cs;
  return GP_OK;
}
