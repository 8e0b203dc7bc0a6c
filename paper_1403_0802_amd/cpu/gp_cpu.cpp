// Host implementation of the grid-filtered PIP and P2P refinements: the paper's
// multi-core and SIMD CPU designs (Sec. III.B-C; Tables 2-5 compare single core,
// multi-core, and both with SIMD).  Cells are the unit of multi-core work (OpenMP,
// dynamic schedule); within a cell eight points share one AVX-512 instruction while
// the candidate's edges stream past them, the paper's points-to-lanes mapping.
//
// Arithmetic is FP64 in the operation order of the definitions in gp.h, built with
// -ffp-contract=off and explicit AVX-512 add/sub/mul/div (never FMA), so every mode
// returns exactly the bits of the GPU library's GP_FP64 form.
#include <immintrin.h>
#include <omp.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>

#include "../../include/gp_cpu.h"

namespace {

constexpr int64_t kMaxCells = int64_t(1) << 28;

// PIP edge as the crossing predicate uses it: lower endpoint, x and y extents, top.
struct EdgeP {
  double lox, loy, w, hiy, h;
};
// P2P segment with the quantities the distance cases use.
struct SegD {
  double ax, ay, bx, by, dx, dy, L2;
};

struct HostGrid {
  double x0 = 0, y0 = 0, cs = 1;
  int64_t nx = 0, ny = 0;
  std::vector<int64_t> cand_off;  // [ncells+1]
  std::vector<int32_t> cand_id;
  std::vector<int64_t> foff;      // [nf+1] edge/segment range of each feature
  std::vector<EdgeP> edges;       // PIP
  std::vector<SegD> segs;         // P2P
};

double now_ms() {
  return std::chrono::duration<double, std::milli>(
             std::chrono::steady_clock::now().time_since_epoch())
      .count();
}

// ---------------------------------------------------------------- grid (Sec. III.A)

gp_status build_grid(gp_kind kind, const gp_geometry &g, const gp_grid_params &p, HostGrid &G) {
  const int64_t nf = g.n_features;
  const bool pip = kind == GP_PIP;
  const int64_t *fro = g.feature_ring_off, *rvo = g.ring_vert_off;
  if (nf < 0 || !rvo || (pip && !fro) || (!pip && g.n_rings != nf))
    return GP_E_INVALID_ARG;
  if (g.n_vertices > 0 && (!g.x || !g.y)) return GP_E_INVALID_ARG;
  const int64_t nr = g.n_rings;
  if (rvo[0] != 0 || rvo[nr] != g.n_vertices) return GP_E_BAD_GEOMETRY;
  for (int64_t r = 0; r < nr; ++r)
    if (rvo[r + 1] < rvo[r]) return GP_E_BAD_GEOMETRY;
  if (pip) {
    if (fro[0] != 0 || fro[nf] != nr) return GP_E_BAD_GEOMETRY;
    for (int64_t f = 0; f < nf; ++f)
      if (fro[f + 1] < fro[f]) return GP_E_BAD_GEOMETRY;
  } else {
    for (int64_t f = 0; f < nf; ++f)
      if (rvo[f + 1] - rvo[f] < 2) return GP_E_BAD_GEOMETRY;
  }
  for (int64_t v = 0; v < g.n_vertices; ++v)
    if (!std::isfinite(g.x[v]) || !std::isfinite(g.y[v])) return GP_E_BAD_GEOMETRY;
  const double cs = p.cell_size, D = pip ? 0.0 : p.radius_D;
  const double pad = cs * 0x1p-20;
  auto ring_lo = [&](int64_t f) { return pip ? fro[f] : f; };
  auto ring_hi = [&](int64_t f) { return pip ? fro[f + 1] : f + 1; };

  // edges / segments, feature by feature
  G.foff.assign(nf + 1, 0);
  for (int64_t f = 0; f < nf; ++f) {
    for (int64_t r = ring_lo(f); r < ring_hi(f); ++r) {
      const int64_t v0 = rvo[r], v1 = rvo[r + 1];
      if (pip) {
        for (int64_t v = v0; v < v1; ++v) {
          const int64_t u = v + 1 < v1 ? v + 1 : v0;  // the ring closes itself
          const double ax = g.x[v], ay = g.y[v], bx = g.x[u], by = g.y[u];
          const bool a_low = ay < by;
          const double lox = a_low ? ax : bx, loy = a_low ? ay : by;
          const double hix = a_low ? bx : ax, hiy = a_low ? by : ay;
          G.edges.push_back(EdgeP{lox, loy, hix - lox, hiy, hiy - loy});
        }
      } else {
        for (int64_t v = v0; v + 1 < v1; ++v) {
          SegD s;
          s.ax = g.x[v]; s.ay = g.y[v]; s.bx = g.x[v + 1]; s.by = g.y[v + 1];
          s.dx = s.bx - s.ax;
          s.dy = s.by - s.ay;
          s.L2 = s.dx * s.dx + s.dy * s.dy;
          G.segs.push_back(s);
        }
      }
    }
    G.foff[f + 1] = pip ? (int64_t)G.edges.size() : (int64_t)G.segs.size();
  }

  // MBBs: expanded by D (P2P), then padded
  std::vector<double> mbb(4 * (size_t)nf);
  for (int64_t f = 0; f < nf; ++f) {
    double lx = INFINITY, ly = INFINITY, hx = -INFINITY, hy = -INFINITY;
    for (int64_t v = rvo[ring_lo(f)]; v < rvo[ring_hi(f)]; ++v) {
      lx = std::min(lx, g.x[v]); hx = std::max(hx, g.x[v]);
      ly = std::min(ly, g.y[v]); hy = std::max(hy, g.y[v]);
    }
    if (!pip) { lx = lx - D; ly = ly - D; hx = hx + D; hy = hy + D; }
    mbb[4 * f + 0] = lx - pad;
    mbb[4 * f + 1] = ly - pad;
    mbb[4 * f + 2] = hx + pad;
    mbb[4 * f + 3] = hy + pad;
  }
  double x0 = p.x0, y0 = p.y0;
  int64_t nx = p.nx, ny = p.ny;
  if (nx == 0 || ny == 0) {  // derived extent
    double lx = INFINITY, ly = INFINITY, hx = -INFINITY, hy = -INFINITY;
    for (int64_t f = 0; f < nf; ++f) {
      if (!(mbb[4 * f] <= mbb[4 * f + 2])) continue;  // a feature without vertices
      lx = std::min(lx, mbb[4 * f]); ly = std::min(ly, mbb[4 * f + 1]);
      hx = std::max(hx, mbb[4 * f + 2]); hy = std::max(hy, mbb[4 * f + 3]);
    }
    if (!(lx <= hx)) { lx = ly = 0.0; hx = hy = 0.0; }
    x0 = lx;
    y0 = ly;
    const double fx = std::floor((hx - x0) / cs), fy = std::floor((hy - y0) / cs);
    if (!(fx < (double)kMaxCells && fy < (double)kMaxCells)) return GP_E_CAPACITY;
    nx = (int64_t)fx + 1;
    ny = (int64_t)fy + 1;
  }
  if (nx <= 0 || ny <= 0 || nx * ny > kMaxCells) return GP_E_CAPACITY;
  G.x0 = x0; G.y0 = y0; G.cs = cs; G.nx = nx; G.ny = ny;

  // rasterise: count, offsets, fill (features in ascending id, so lists are sorted)
  const int64_t nc = nx * ny;
  auto span = [&](double lo, double hi, double o, int64_t n, int64_t &c0, int64_t &c1) {
    const double a = std::floor((lo - o) / cs), b = std::floor((hi - o) / cs);
    c0 = a < 0 ? 0 : (a > (double)(n - 1) ? n : (int64_t)a);
    c1 = b < 0 ? -1 : (b > (double)(n - 1) ? n - 1 : (int64_t)b);
  };
  G.cand_off.assign(nc + 1, 0);
  for (int pass = 0; pass < 2; ++pass) {
    std::vector<int64_t> fill;
    if (pass == 1) {
      for (int64_t c = 0; c < nc; ++c) G.cand_off[c + 1] += G.cand_off[c];
      G.cand_id.resize(G.cand_off[nc]);
      fill.assign(G.cand_off.begin(), G.cand_off.end() - 1);
    }
    for (int64_t f = 0; f < nf; ++f) {
      if (!(mbb[4 * f] <= mbb[4 * f + 2])) continue;
      int64_t ax, bx, ay, by;
      span(mbb[4 * f], mbb[4 * f + 2], x0, nx, ax, bx);
      span(mbb[4 * f + 1], mbb[4 * f + 3], y0, ny, ay, by);
      for (int64_t cy = ay; cy <= by; ++cy)
        for (int64_t cx = ax; cx <= bx; ++cx) {
          const int64_t c = cy * nx + cx;
          if (pass == 0) G.cand_off[c + 1] += 1;
          else G.cand_id[fill[c]++] = (int32_t)f;
        }
    }
  }
  return GP_OK;
}

// ---------------------------------------------------------------- refinement, scalar

void pip_scalar(const HostGrid &G, int64_t c, const int64_t *idx, int64_t np, const double *px,
                const double *py, int32_t *out) {
  for (int64_t i = 0; i < np; ++i) {
    const double x = px[idx[i]], y = py[idx[i]];
    int32_t best = -1;
    for (int64_t k = G.cand_off[c]; k < G.cand_off[c + 1]; ++k) {
      const int32_t f = G.cand_id[k];
      bool odd = false;
      for (int64_t e = G.foff[f]; e < G.foff[f + 1]; ++e) {
        const EdgeP &q = G.edges[e];
        const bool st = q.loy <= y && y < q.hiy;
        const double lhs = (x - q.lox) * q.h;
        const double rhs = q.w * (y - q.loy);
        odd ^= st && lhs < rhs;
      }
      if (odd && best < 0) best = f;
    }
    out[idx[i]] = best;
  }
}

inline double seg_d2(const SegD &s, double x, double y) {
  const double wx = x - s.ax, wy = y - s.ay;
  const double t = wx * s.dx + wy * s.dy;
  if (t <= 0.0) return wx * wx + wy * wy;
  if (t >= s.L2) {
    const double ex = x - s.bx, ey = y - s.by;
    return ex * ex + ey * ey;
  }
  const double cr = wx * s.dy - wy * s.dx;
  return (cr * cr) / s.L2;
}

void p2p_scalar(const HostGrid &G, double D2, int64_t c, const int64_t *idx, int64_t np,
                const double *px, const double *py, int32_t *oid, double *od) {
  for (int64_t i = 0; i < np; ++i) {
    const double x = px[idx[i]], y = py[idx[i]];
    int32_t bid = -1;
    double best = INFINITY;
    for (int64_t k = G.cand_off[c]; k < G.cand_off[c + 1]; ++k) {
      const int32_t f = G.cand_id[k];
      double pd = INFINITY;
      for (int64_t e = G.foff[f]; e < G.foff[f + 1]; ++e) pd = std::min(pd, seg_d2(G.segs[e], x, y));
      if (pd <= D2 && pd < best) {  // ascending ids: a tie keeps the smaller id
        best = pd;
        bid = f;
      }
    }
    oid[idx[i]] = bid;
    od[idx[i]] = bid >= 0 ? std::sqrt(best) : INFINITY;
  }
}

// ---------------------------------------------------------------- refinement, AVX-512

__attribute__((target("avx512f,avx512dq"))) void pip_simd(const HostGrid &G, int64_t c,
                                                          const int64_t *idx, int64_t np,
                                                          const double *px, const double *py,
                                                          int32_t *out) {
  for (int64_t i0 = 0; i0 < np; i0 += 8) {
    const int m = (int)std::min<int64_t>(8, np - i0);
    alignas(64) double xs[8], ys[8];
    for (int l = 0; l < 8; ++l) {
      const int64_t j = idx[i0 + (l < m ? l : 0)];
      xs[l] = px[j];
      ys[l] = py[j];
    }
    const __m512d vx = _mm512_load_pd(xs), vy = _mm512_load_pd(ys);
    __mmask8 decided = 0;
    int32_t best[8];
    for (int l = 0; l < 8; ++l) best[l] = -1;
    for (int64_t k = G.cand_off[c]; k < G.cand_off[c + 1]; ++k) {
      const int32_t f = G.cand_id[k];
      __mmask8 par = 0;
      for (int64_t e = G.foff[f]; e < G.foff[f + 1]; ++e) {
        const EdgeP &q = G.edges[e];
        const __m512d loy = _mm512_set1_pd(q.loy);
        const __mmask8 st = _mm512_cmp_pd_mask(loy, vy, _CMP_LE_OQ) &
                            _mm512_cmp_pd_mask(vy, _mm512_set1_pd(q.hiy), _CMP_LT_OQ);
        const __m512d lhs = _mm512_mul_pd(_mm512_sub_pd(vx, _mm512_set1_pd(q.lox)),
                                          _mm512_set1_pd(q.h));
        const __m512d rhs = _mm512_mul_pd(_mm512_set1_pd(q.w), _mm512_sub_pd(vy, loy));
        par ^= st & _mm512_cmp_pd_mask(lhs, rhs, _CMP_LT_OQ);
      }
      const __mmask8 take = par & (__mmask8)~decided;
      for (int l = 0; l < 8; ++l)
        if ((take >> l) & 1) best[l] = f;
      decided |= par;
    }
    for (int l = 0; l < m; ++l) out[idx[i0 + l]] = best[l];
  }
}

__attribute__((target("avx512f,avx512dq"))) void p2p_simd(const HostGrid &G, double D2,
                                                          int64_t c, const int64_t *idx,
                                                          int64_t np, const double *px,
                                                          const double *py, int32_t *oid,
                                                          double *od) {
  const __m512d zero = _mm512_setzero_pd(), inf = _mm512_set1_pd(INFINITY);
  const __m512d vD2 = _mm512_set1_pd(D2);
  for (int64_t i0 = 0; i0 < np; i0 += 8) {
    const int m = (int)std::min<int64_t>(8, np - i0);
    alignas(64) double xs[8], ys[8];
    for (int l = 0; l < 8; ++l) {
      const int64_t j = idx[i0 + (l < m ? l : 0)];
      xs[l] = px[j];
      ys[l] = py[j];
    }
    const __m512d vx = _mm512_load_pd(xs), vy = _mm512_load_pd(ys);
    __m512d best = inf;
    __m512i bid = _mm512_set1_epi64(-1);
    for (int64_t k = G.cand_off[c]; k < G.cand_off[c + 1]; ++k) {
      const int32_t f = G.cand_id[k];
      __m512d pd = inf;
      for (int64_t e = G.foff[f]; e < G.foff[f + 1]; ++e) {
        const SegD &s = G.segs[e];
        const __m512d wx = _mm512_sub_pd(vx, _mm512_set1_pd(s.ax));
        const __m512d wy = _mm512_sub_pd(vy, _mm512_set1_pd(s.ay));
        const __m512d dx = _mm512_set1_pd(s.dx), dy = _mm512_set1_pd(s.dy);
        const __m512d t = _mm512_add_pd(_mm512_mul_pd(wx, dx), _mm512_mul_pd(wy, dy));
        const __m512d da = _mm512_add_pd(_mm512_mul_pd(wx, wx), _mm512_mul_pd(wy, wy));
        const __m512d ex = _mm512_sub_pd(vx, _mm512_set1_pd(s.bx));
        const __m512d ey = _mm512_sub_pd(vy, _mm512_set1_pd(s.by));
        const __m512d db = _mm512_add_pd(_mm512_mul_pd(ex, ex), _mm512_mul_pd(ey, ey));
        const __m512d cr = _mm512_sub_pd(_mm512_mul_pd(wx, dy), _mm512_mul_pd(wy, dx));
        const __m512d L2 = _mm512_set1_pd(s.L2);
        __m512d d = _mm512_div_pd(_mm512_mul_pd(cr, cr), L2);
        d = _mm512_mask_blend_pd(_mm512_cmp_pd_mask(t, L2, _CMP_GE_OQ), d, db);
        d = _mm512_mask_blend_pd(_mm512_cmp_pd_mask(t, zero, _CMP_LE_OQ), d, da);
        pd = _mm512_min_pd(pd, d);
      }
      const __mmask8 win = _mm512_cmp_pd_mask(pd, vD2, _CMP_LE_OQ) &
                           _mm512_cmp_pd_mask(pd, best, _CMP_LT_OQ);
      best = _mm512_mask_blend_pd(win, best, pd);
      bid = _mm512_mask_blend_epi64(win, bid, _mm512_set1_epi64(f));
    }
    alignas(64) double b[8];
    alignas(64) int64_t ids[8];
    _mm512_store_pd(b, best);
    _mm512_store_si512((void *)ids, bid);
    for (int l = 0; l < m; ++l) {
      oid[idx[i0 + l]] = (int32_t)ids[l];
      od[idx[i0 + l]] = ids[l] >= 0 ? std::sqrt(b[l]) : INFINITY;
    }
  }
}

bool host_has_simd() {
  __builtin_cpu_init();
  return __builtin_cpu_supports("avx512f") && __builtin_cpu_supports("avx512dq");
}

}  // namespace

extern "C" int32_t gp_cpu_has_simd(void) { return host_has_simd() ? 1 : 0; }

extern "C" gp_status gp_cpu_join(gp_kind kind, const gp_geometry *geom,
                                 const gp_grid_params *params, int64_t n, const double *px,
                                 const double *py, int32_t *out_id, double *out_dist,
                                 int32_t mode, int32_t threads, gp_cpu_stats *stats) {
  if (!geom || !params || n < 0 || (n > 0 && (!px || !py || !out_id)) ||
      (kind == GP_P2P && n > 0 && !out_dist) || (kind != GP_PIP && kind != GP_P2P) ||
      mode < GP_CPU_SC || mode > GP_CPU_MC_SIMD || geom->on_device)
    return GP_E_INVALID_ARG;
  if (!(params->cell_size > 0.0) || !std::isfinite(params->cell_size) ||
      (kind == GP_P2P && !(params->radius_D >= 0.0)) || params->nx < 0 || params->ny < 0)
    return GP_E_INVALID_ARG;
  const double t0 = now_ms();
  HostGrid G;
  gp_status rc = build_grid(kind, *geom, *params, G);
  if (rc) return rc;
  // pair the points: cell of each point, stable counting sort by cell
  const int64_t nc = G.nx * G.ny;
  std::vector<int64_t> cell(n), off(nc + 2, 0), order(n);
  for (int64_t i = 0; i < n; ++i) {
    const double fx = std::floor((px[i] - G.x0) / G.cs), fy = std::floor((py[i] - G.y0) / G.cs);
    int64_t c = nc;  // unpaired
    if (fx >= 0 && fx < (double)G.nx && fy >= 0 && fy < (double)G.ny)
      c = (int64_t)fy * G.nx + (int64_t)fx;
    cell[i] = c;
    off[c + 1] += 1;
  }
  for (int64_t c = 0; c <= nc; ++c) off[c + 1] += off[c];
  {
    std::vector<int64_t> fill(off.begin(), off.end() - 1);
    for (int64_t i = 0; i < n; ++i) order[fill[cell[i]]++] = i;
  }
  for (int64_t j = off[nc]; j < n; ++j) {
    out_id[order[j]] = -1;
    if (kind == GP_P2P) out_dist[order[j]] = INFINITY;
  }
  std::vector<int64_t> work;  // cells with points and candidates
  uint64_t tests = 0;
  for (int64_t c = 0; c < nc; ++c) {
    const int64_t np = off[c + 1] - off[c];
    if (np == 0) continue;
    if (G.cand_off[c + 1] == G.cand_off[c]) {
      for (int64_t j = off[c]; j < off[c + 1]; ++j) {
        out_id[order[j]] = -1;
        if (kind == GP_P2P) out_dist[order[j]] = INFINITY;
      }
      continue;
    }
    int64_t ne = 0;
    for (int64_t k = G.cand_off[c]; k < G.cand_off[c + 1]; ++k)
      ne += G.foff[G.cand_id[k] + 1] - G.foff[G.cand_id[k]];
    tests += (uint64_t)np * (uint64_t)ne;
    work.push_back(c);
  }
  const double t1 = now_ms();
  const bool simd = (mode == GP_CPU_SC_SIMD || mode == GP_CPU_MC_SIMD) && host_has_simd();
  const bool mc = mode == GP_CPU_MC || mode == GP_CPU_MC_SIMD;
  const int nt = mc ? (threads > 0 ? threads : omp_get_max_threads()) : 1;
  const double D2 = params->radius_D * params->radius_D;
  const int64_t nw = (int64_t)work.size();
#pragma omp parallel for schedule(dynamic, 1) num_threads(nt)
  for (int64_t w = 0; w < nw; ++w) {
    const int64_t c = work[w];
    const int64_t *idx = order.data() + off[c];
    const int64_t np = off[c + 1] - off[c];
    if (kind == GP_PIP) {
      if (simd) pip_simd(G, c, idx, np, px, py, out_id);
      else pip_scalar(G, c, idx, np, px, py, out_id);
    } else {
      if (simd) p2p_simd(G, D2, c, idx, np, px, py, out_id, out_dist);
      else p2p_scalar(G, D2, c, idx, np, px, py, out_id, out_dist);
    }
  }
  const double t2 = now_ms();
  if (stats) {
    stats->tests = tests;
    stats->threads = nt;
    stats->simd = simd ? 1 : 0;
    stats->ms_filter = t1 - t0;
    stats->ms_refine = t2 - t1;
  }
  return GP_OK;
}
