/*
 * CPU oracle for grid-filtered point-in-polygon (PIP) and point-to-polyline nearest
 * distance (P2P) -- TEST INFRASTRUCTURE ONLY.
 *
 * This file is the plain, slow, obviously correct reference that the GPU path is
 * checked against.  It shares no code, header or table with the GPU library and is
 * only ever loaded by the test suite, the smoke check and the CPU-baseline leg of
 * the benchmark.  Everything is scalar IEEE binary64, round-to-nearest-even, built
 * with -O2 -ffp-contract=off so that no multiply-add is fused.
 *
 * What it computes (Zhang & You, "Large-Scale Geospatial Processing on Multi-Core
 * and Many-Core Processors", Sec. II problem statement, Sec. III.A-C):
 *
 *  - Filter (Sec. III.A): a uniform grid.  A point falls in cell
 *    (floor((x-x0)/cs), floor((y-y0)/cs)); a feature is paired with every cell its
 *    MBB touches.  For P2P the MBB is first expanded by the query radius
 *    (x1-R, y1-R, x2+R, y2+R), the necessary condition stated in Sec. III.A.
 *    Both kinds add a pad of cs*2^-20 on every side.
 *  - PIP refinement (Sec. III.C, Fig. 3): the even-odd ray-crossing rule over every
 *    ring of the polygon, holes included.  An edge (a,b) with a.y == b.y never
 *    counts; otherwise, with lo/hi its lower/upper endpoint, it counts when
 *      lo.y <= p.y < hi.y  and  (p.x-lo.x)*(hi.y-lo.y) < (hi.x-lo.x)*(p.y-lo.y),
 *    i.e. the +x ray from p crosses it strictly right of p (half-open in y).
 *    A point takes the smallest polygon id whose parity is odd, else -1.
 *  - P2P refinement (Sec. III.B, Fig. 2): the distance from p to a segment is the
 *    perpendicular distance when the projection falls on the segment, else the
 *    distance to the nearer endpoint; a polyline's distance is the minimum over its
 *    segments.  A point takes the polyline with the smallest squared distance among
 *    those with d^2 <= D*D (ties: smallest id), else (-1, +inf).
 *
 * Points outside the grid extent, or with non-finite coordinates, are unpaired by
 * the filter and get -1 (and +inf).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_PAD_SCALE 0x1p-20

/* ------------------------------------------------------------------ the two tests */

/* Even-odd parity of the crossings of the +x ray from (px,py) with one closed ring
 * of m vertices (the closing edge last->first is implied). */
static int ring_parity(double px, double py, const double *x, const double *y, int64_t m)
{
    int odd = 0;
    for (int64_t i = 0; i < m; ++i) {
        int64_t j = (i + 1 == m) ? 0 : i + 1;
        double ax = x[i], ay = y[i], bx = x[j], by = y[j];
        if (ay == by)
            continue;
        double lox, loy, hix, hiy;
        if (ay < by) {
            lox = ax; loy = ay; hix = bx; hiy = by;
        } else {
            lox = bx; loy = by; hix = ax; hiy = ay;
        }
        if (loy <= py && py < hiy) {
            double lhs = (px - lox) * (hiy - loy);
            double rhs = (hix - lox) * (py - loy);
            if (lhs < rhs)
                odd ^= 1;
        }
    }
    return odd;
}

/* Inside test of polygon f: XOR of the ring parities over all of its rings. */
static int polygon_inside(double px, double py, int64_t f, const int64_t *fro,
                          const int64_t *rvo, const double *x, const double *y)
{
    int odd = 0;
    for (int64_t r = fro[f]; r < fro[f + 1]; ++r) {
        int64_t v0 = rvo[r], v1 = rvo[r + 1];
        odd ^= ring_parity(px, py, x + v0, y + v0, v1 - v0);
    }
    return odd;
}

/* Squared distance from p to segment (a,b), three cases, fixed operation order. */
static double segment_d2(double px, double py, double ax, double ay, double bx, double by)
{
    double dx = bx - ax, dy = by - ay;
    double wx = px - ax, wy = py - ay;
    double L2 = dx * dx + dy * dy;
    double t = wx * dx + wy * dy;
    if (t <= 0.0)
        return wx * wx + wy * wy; /* nearer to a (also a zero-length segment) */
    if (t >= L2) {
        double ex = px - bx, ey = py - by;
        return ex * ex + ey * ey; /* nearer to b */
    }
    double c = wx * dy - wy * dx; /* perpendicular foot inside the segment */
    return (c * c) / L2;
}

/* Minimum squared distance from p to polyline f (vertices v0..v1-1). */
static double polyline_d2(double px, double py, int64_t f, const int64_t *rvo,
                          const double *x, const double *y)
{
    double best = INFINITY;
    for (int64_t v = rvo[f]; v + 1 < rvo[f + 1]; ++v) {
        double d2 = segment_d2(px, py, x[v], y[v], x[v + 1], y[v + 1]);
        if (d2 < best)
            best = d2;
    }
    return best;
}

/* ------------------------------------------------------------------ the grid filter */

/* Feature MBBs, padded by cs*2^-20 and, for P2P (kind 2), expanded by D first.
 * mbb[4f..4f+3] = (lo.x, lo.y, hi.x, hi.y). */
int or_mbb(int kind, int64_t nf, const int64_t *fro, const int64_t *rvo, const double *x,
           const double *y, double D, double cs, double *mbb)
{
    double pad = cs * OR_PAD_SCALE;
    for (int64_t f = 0; f < nf; ++f) {
        int64_t r0 = fro ? fro[f] : f, r1 = fro ? fro[f + 1] : f + 1;
        double mnx = INFINITY, mny = INFINITY, mxx = -INFINITY, mxy = -INFINITY;
        for (int64_t v = rvo[r0]; v < rvo[r1]; ++v) {
            if (x[v] < mnx) mnx = x[v];
            if (x[v] > mxx) mxx = x[v];
            if (y[v] < mny) mny = y[v];
            if (y[v] > mxy) mxy = y[v];
        }
        if (kind == 2) {
            mnx = mnx - D; mny = mny - D; mxx = mxx + D; mxy = mxy + D;
        }
        mbb[4 * f + 0] = mnx - pad;
        mbb[4 * f + 1] = mny - pad;
        mbb[4 * f + 2] = mxx + pad;
        mbb[4 * f + 3] = mxy + pad;
    }
    return 0;
}

/* Extent covering every MBB: origin at the smallest corner, and enough cells that the
 * largest corner maps inside.  out = (x0, y0, nx, ny). */
int or_extent(int64_t nf, const double *mbb, double cs, double *x0, double *y0, int64_t *nx,
              int64_t *ny)
{
    if (nf == 0) {
        *x0 = 0.0; *y0 = 0.0; *nx = 1; *ny = 1;
        return 0;
    }
    double lx = INFINITY, ly = INFINITY, hx = -INFINITY, hy = -INFINITY;
    for (int64_t f = 0; f < nf; ++f) {
        if (mbb[4 * f + 0] < lx) lx = mbb[4 * f + 0];
        if (mbb[4 * f + 1] < ly) ly = mbb[4 * f + 1];
        if (mbb[4 * f + 2] > hx) hx = mbb[4 * f + 2];
        if (mbb[4 * f + 3] > hy) hy = mbb[4 * f + 3];
    }
    *x0 = lx;
    *y0 = ly;
    *nx = (int64_t)floor((hx - lx) / cs) + 1;
    *ny = (int64_t)floor((hy - ly) / cs) + 1;
    return 0;
}

/* Cell of a point, or -1 when it is outside the extent or not finite. */
static int64_t cell_of(double px, double py, double x0, double y0, double cs, int64_t nx,
                       int64_t ny)
{
    double fx = floor((px - x0) / cs);
    double fy = floor((py - y0) / cs);
    if (!(fx >= 0.0 && fx < (double)nx && fy >= 0.0 && fy < (double)ny))
        return -1;
    return (int64_t)fy * nx + (int64_t)fx;
}

void or_point_cells(int64_t n, const double *px, const double *py, double x0, double y0,
                    double cs, int64_t nx, int64_t ny, int64_t *cell)
{
    for (int64_t i = 0; i < n; ++i)
        cell[i] = cell_of(px[i], py[i], x0, y0, cs, nx, ny);
}

/* Index range [lo, hi] of the cells an interval [a, b] touches along one axis, clamped
 * to the grid.  Returns 0 when the interval misses the grid. */
static int axis_range(double a, double b, double o, double cs, int64_t n, int64_t *lo,
                      int64_t *hi)
{
    double fa = floor((a - o) / cs);
    double fb = floor((b - o) / cs);
    if (fb < 0.0 || fa > (double)(n - 1))
        return 0;
    *lo = fa < 0.0 ? 0 : (int64_t)fa;
    *hi = fb > (double)(n - 1) ? n - 1 : (int64_t)fb;
    return 1;
}

/* Cell -> candidate CSR.  With cand_id == NULL only cand_off is filled (counts, then
 * prefix sums); the return value is the number of (cell, feature) pairs.  Features are
 * visited in ascending id, so every cell's list is sorted by id. */
int64_t or_candidates(int64_t nf, const double *mbb, double x0, double y0, double cs,
                      int64_t nx, int64_t ny, int64_t *cand_off, int32_t *cand_id)
{
    int64_t ncells = nx * ny;
    int64_t *fill = NULL;
    if (cand_id == NULL) {
        memset(cand_off, 0, sizeof(int64_t) * (size_t)(ncells + 1));
    } else {
        fill = (int64_t *)malloc(sizeof(int64_t) * (size_t)(ncells + 1));
        memcpy(fill, cand_off, sizeof(int64_t) * (size_t)(ncells + 1));
    }
    for (int64_t f = 0; f < nf; ++f) {
        int64_t ixl, ixh, iyl, iyh;
        if (!axis_range(mbb[4 * f + 0], mbb[4 * f + 2], x0, cs, nx, &ixl, &ixh))
            continue;
        if (!axis_range(mbb[4 * f + 1], mbb[4 * f + 3], y0, cs, ny, &iyl, &iyh))
            continue;
        for (int64_t iy = iyl; iy <= iyh; ++iy)
            for (int64_t ix = ixl; ix <= ixh; ++ix) {
                int64_t c = iy * nx + ix;
                if (cand_id == NULL)
                    cand_off[c + 1] += 1;
                else
                    cand_id[fill[c]++] = (int32_t)f;
            }
    }
    if (cand_id == NULL) {
        for (int64_t c = 0; c < ncells; ++c)
            cand_off[c + 1] += cand_off[c];
    } else {
        free(fill);
    }
    return cand_off[ncells];
}

/* Stable grouping of points by cell: points of cell c are perm[pt_off[c]..pt_off[c+1])
 * in ascending original index; points outside the extent come last. */
void or_sort_points(int64_t n, const int64_t *cell, int64_t ncells, int64_t *pt_off,
                    int64_t *perm)
{
    int64_t *pos = (int64_t *)calloc((size_t)(ncells + 2), sizeof(int64_t));
    for (int64_t i = 0; i < n; ++i) {
        int64_t c = cell[i] < 0 ? ncells : cell[i];
        pos[c + 1] += 1;
    }
    for (int64_t c = 0; c <= ncells; ++c)
        pos[c + 1] += pos[c];
    for (int64_t c = 0; c <= ncells; ++c)
        pt_off[c] = pos[c];
    for (int64_t i = 0; i < n; ++i) {
        int64_t c = cell[i] < 0 ? ncells : cell[i];
        perm[pos[c]++] = i;
    }
    free(pos);
}

/* Point-edge tests the refinement performs: sum over cells of
 * npts(cell) * sum over its candidates of nedges(feature). */
uint64_t or_test_count(int64_t ncells, const int64_t *pt_off, const int64_t *cand_off,
                       const int32_t *cand_id, const int64_t *nedges)
{
    uint64_t total = 0;
    for (int64_t c = 0; c < ncells; ++c) {
        uint64_t np = (uint64_t)(pt_off[c + 1] - pt_off[c]);
        if (np == 0)
            continue;
        uint64_t e = 0;
        for (int64_t k = cand_off[c]; k < cand_off[c + 1]; ++k)
            e += (uint64_t)nedges[cand_id[k]];
        total += np * e;
    }
    return total;
}

/* ------------------------------------------------------------------ the joins */

static void set_threads(int nthreads)
{
#ifdef _OPENMP
    if (nthreads > 0)
        omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
}

/* PIP.  With cand_off == NULL every polygon is tried (brute force, no extent);
 * otherwise only the candidates of the point's cell. */
void or_pip(int64_t n, const double *px, const double *py, int64_t nf, const int64_t *fro,
            const int64_t *rvo, const double *x, const double *y, double x0, double y0,
            double cs, int64_t nx, int64_t ny, const int64_t *cand_off, const int32_t *cand_id,
            int32_t *out_id, int nthreads)
{
    set_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t i = 0; i < n; ++i) {
        int32_t best = -1;
        if (cand_off == NULL) {
            for (int64_t f = 0; f < nf; ++f)
                if (polygon_inside(px[i], py[i], f, fro, rvo, x, y)) {
                    best = (int32_t)f;
                    break;
                }
        } else {
            int64_t c = cell_of(px[i], py[i], x0, y0, cs, nx, ny);
            if (c >= 0)
                for (int64_t k = cand_off[c]; k < cand_off[c + 1]; ++k)
                    if (polygon_inside(px[i], py[i], cand_id[k], fro, rvo, x, y)) {
                        best = cand_id[k];
                        break;
                    }
        }
        out_id[i] = best;
    }
}

/* Number of polygons whose inside test is true, over all polygons (no grid). */
void or_pip_count(int64_t n, const double *px, const double *py, int64_t nf,
                  const int64_t *fro, const int64_t *rvo, const double *x, const double *y,
                  int32_t *out_count, int nthreads)
{
    set_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t i = 0; i < n; ++i) {
        int32_t cnt = 0;
        for (int64_t f = 0; f < nf; ++f)
            cnt += polygon_inside(px[i], py[i], f, fro, rvo, x, y);
        out_count[i] = cnt;
    }
}

/* P2P.  Brute force over all polylines when cand_off == NULL. */
void or_p2p(int64_t n, const double *px, const double *py, int64_t nf, const int64_t *rvo,
            const double *x, const double *y, double D, double x0, double y0, double cs,
            int64_t nx, int64_t ny, const int64_t *cand_off, const int32_t *cand_id,
            int32_t *out_id, double *out_dist, int nthreads)
{
    double D2 = D * D;
    set_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t i = 0; i < n; ++i) {
        int32_t best_id = -1;
        double best = INFINITY;
        int64_t k0 = 0, k1 = nf;
        if (cand_off != NULL) {
            int64_t c = cell_of(px[i], py[i], x0, y0, cs, nx, ny);
            if (c < 0) {
                k0 = 0;
                k1 = 0;
            } else {
                k0 = cand_off[c];
                k1 = cand_off[c + 1];
            }
        }
        for (int64_t k = k0; k < k1; ++k) {
            int64_t f = cand_off != NULL ? cand_id[k] : k;
            double d2 = polyline_d2(px[i], py[i], f, rvo, x, y);
            if (d2 <= D2 && d2 < best) {
                best = d2;
                best_id = (int32_t)f;
            }
        }
        out_id[i] = best_id;
        out_dist[i] = best_id >= 0 ? sqrt(best) : INFINITY;
    }
}

/* Single-pair entry points, for pins that probe the two tests directly. */
int or_polygon_inside(double px, double py, int64_t f, const int64_t *fro, const int64_t *rvo,
                      const double *x, const double *y)
{
    return polygon_inside(px, py, f, fro, rvo, x, y);
}

double or_segment_d2(double px, double py, double ax, double ay, double bx, double by)
{
    return segment_d2(px, py, ax, ay, bx, by);
}

int or_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
