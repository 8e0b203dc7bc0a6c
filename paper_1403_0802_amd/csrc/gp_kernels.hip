// HIP kernels for gfx950 (MI355X): grid pairing and PIP / P2P refinement.
//
// Paper: Zhang & You, arXiv 1403.0802.  Sec. III.A (grid filter built from sorts,
// scans and MBB rasterisation), Sec. III.B (P2P: a (cell, {polyline}) pair per thread
// block, a point per thread, looping over the polylines' vertices; Fig. 2 distance
// cases), Sec. III.C (PIP: same mapping, ray crossing over every ring, Fig. 3).
//
// MI355X mapping.  A work item is one grid cell plus a chunk of up to 64*PPL of its
// points; one 64-lane wavefront owns the item, holds PPL points per lane in VGPRs, and
// walks the cell's whole candidate list in ascending feature id, staging each
// feature's edges through LDS in chunks (every lane then reads the same LDS word, a
// broadcast).  Because a single wave sees all candidates of its points, results need
// no cross-workgroup merge and ties resolve to the smallest id by visiting order.
// Items are pulled from a device-side queue by a persistent grid sized to the CUs.
//
// Compiled with -ffp-contract=off: every FP64 expression is evaluated exactly as
// written (no fused multiply-add), which is what makes the FP64 forms bitwise
// reproducible against a scalar FP64 implementation.  The FP32 forms request fused
// multiply-adds explicitly with fmaf().
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "gp_internal.h"

namespace gp {

#define GP_WAVE 64
#define GP_XCDS 8     // XCDs of an MI355X, each with its own L2
#define GP_XBLOCK 32  // consecutive work items per block of an XCD's queue
#define SCAN_THREADS 256
#define SCAN_ITEMS 16
#define SCAN_TILE (SCAN_THREADS * SCAN_ITEMS)
#define RS_THREADS 256
#define RS_ITEMS 8
#define RS_TILE (RS_THREADS * RS_ITEMS)
#define RS_MAX_BITS 9
#define RS_MAX_BUCKETS (1 << RS_MAX_BITS)
static_assert(RS_THREADS == SCAN_THREADS, "the tile scan uses the block scan");

__device__ __forceinline__ uint64_t ballot(bool c) { return __builtin_amdgcn_ballot_w64(c); }
__device__ __forceinline__ uint32_t lane_id() { return __lane_id(); }
__device__ __forceinline__ uint64_t lanemask_lt() {
  return (1ull << lane_id()) - 1ull;
}
__device__ __forceinline__ uint32_t uniform(uint32_t v) {
  return __builtin_amdgcn_readfirstlane(v);
}

static inline unsigned grid_for(size_t n, unsigned threads, unsigned cap = 65535u * 16u) {
  size_t g = (n + threads - 1) / threads;
  if (g == 0) g = 1;
  if (g > cap) g = cap;
  return (unsigned)g;
}

// ------------------------------------------------------------------------- fill

__global__ void k_fill_u32(uint32_t *p, uint32_t v, size_t n) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x)
    p[i] = v;
}

hipError_t launch_fill_u32(uint32_t *p, uint32_t v, size_t n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_u32, dim3(grid_for(n, 256, 4096)), dim3(256), 0, s, p, v, n);
  return hipGetLastError();
}

// ------------------------------------------------------------------------- scan
// Exclusive prefix sum of uint32 in three phases (tile reduce, scan of tile sums,
// tile scan + offset), recursive over the tile sums.  Deterministic.

// Orders a wave's LDS accesses: every lane's earlier LDS writes are visible to every
// lane's later reads (one wave executes its LDS instructions in order; the fence keeps
// the compiler from moving them).
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v) {
  const uint32_t lane = lane_id();
#pragma unroll
  for (int off = 1; off < GP_WAVE; off <<= 1) {
    uint32_t u = __shfl_up(v, off, GP_WAVE);
    if (lane >= (uint32_t)off) v += u;
  }
  return v;
}

// Block-wide exclusive scan of one value per thread (256 threads); returns the block
// total through *total.
__device__ uint32_t block_excl_scan(uint32_t v, uint32_t *total) {
  __shared__ uint32_t wsum[SCAN_THREADS / GP_WAVE];
  const uint32_t lane = lane_id(), wave = threadIdx.x / GP_WAVE;
  uint32_t inc = wave_incl_scan(v);
  if (lane == GP_WAVE - 1) wsum[wave] = inc;
  __syncthreads();
  uint32_t base = 0, tot = 0;
#pragma unroll
  for (int w = 0; w < SCAN_THREADS / GP_WAVE; ++w) {
    uint32_t x = wsum[w];
    if (w < (int)wave) base += x;
    tot += x;
  }
  __syncthreads();
  *total = tot;
  return base + inc - v;
}

__global__ __launch_bounds__(SCAN_THREADS) void k_scan_reduce(const uint32_t *in, size_t n,
                                                              uint32_t *sums) {
  const size_t base = (size_t)blockIdx.x * SCAN_TILE;
  uint32_t acc = 0;
  for (int r = 0; r < SCAN_ITEMS; ++r) {
    size_t i = base + (size_t)r * SCAN_THREADS + threadIdx.x;
    if (i < n) acc += in[i];
  }
  uint32_t tot;
  block_excl_scan(acc, &tot);
  if (threadIdx.x == 0) sums[blockIdx.x] = tot;
}

__global__ __launch_bounds__(SCAN_THREADS) void k_scan_apply(const uint32_t *in, uint32_t *out,
                                                             size_t n, const uint32_t *offs) {
  __shared__ uint32_t tile[SCAN_TILE + SCAN_TILE / 32];
  const size_t base = (size_t)blockIdx.x * SCAN_TILE;
  for (int r = 0; r < SCAN_ITEMS; ++r) {
    int li = r * SCAN_THREADS + threadIdx.x;
    size_t i = base + li;
    tile[li + li / 32] = i < n ? in[i] : 0u;
  }
  __syncthreads();
  uint32_t loc[SCAN_ITEMS];
  uint32_t acc = 0;
  for (int k = 0; k < SCAN_ITEMS; ++k) {
    int li = threadIdx.x * SCAN_ITEMS + k;
    loc[k] = tile[li + li / 32];
    acc += loc[k];
  }
  uint32_t tot;
  uint32_t pre = block_excl_scan(acc, &tot) + (offs ? offs[blockIdx.x] : 0u);
  for (int k = 0; k < SCAN_ITEMS; ++k) {
    int li = threadIdx.x * SCAN_ITEMS + k;
    tile[li + li / 32] = pre;
    pre += loc[k];
  }
  __syncthreads();
  for (int r = 0; r < SCAN_ITEMS; ++r) {
    int li = r * SCAN_THREADS + threadIdx.x;
    size_t i = base + li;
    if (i < n) out[i] = tile[li + li / 32];
  }
}

size_t scan_tmp_elems(size_t n) {
  size_t total = 0;
  while (n > SCAN_TILE) {
    n = (n + SCAN_TILE - 1) / SCAN_TILE;
    total += n + 64;
  }
  return total + 64;
}

hipError_t launch_exclusive_scan_u32(const uint32_t *in, uint32_t *out, size_t n, uint32_t *tmp,
                                     hipStream_t s) {
  if (n == 0) return hipSuccess;
  if (n <= SCAN_TILE) {
    hipLaunchKernelGGL(k_scan_apply, dim3(1), dim3(SCAN_THREADS), 0, s, in, out, n,
                       (const uint32_t *)nullptr);
    return hipGetLastError();
  }
  size_t nb = (n + SCAN_TILE - 1) / SCAN_TILE;
  uint32_t *sums = tmp;
  hipLaunchKernelGGL(k_scan_reduce, dim3((unsigned)nb), dim3(SCAN_THREADS), 0, s, in, n, sums);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  e = launch_exclusive_scan_u32(sums, sums, nb, tmp + nb + 64, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_scan_apply, dim3((unsigned)nb), dim3(SCAN_THREADS), 0, s, in, out, n,
                     (const uint32_t *)sums);
  return hipGetLastError();
}

// ------------------------------------------------------------------------- radix sort
// Stable LSD radix sort of (uint32 key, uint32 value[, FP64 (x, y) payload]) records.
// Digits are at most 8 bits wide and the pass count is the least that covers the key
// width.  Each pass: per-tile digit histogram, exclusive scan of the digit-major
// histogram, then a stable scatter in which every key's rank among equal digits of its
// tile comes from wavefront ballots (peer masks), not from atomics, so the output
// order is fixed.

size_t radix_hist_elems(size_t n) {
  size_t nblk = (n + RS_TILE - 1) / RS_TILE;
  if (nblk == 0) nblk = 1;
  return (size_t)RS_MAX_BUCKETS * nblk;
}

// Digit histograms of tpw (1 .. RS_HIST_TILES) consecutive tiles per workgroup, written
// digit-major (hist[d * nblk + tile]).  A workgroup takes several tiles, so its counts of
// one digit are adjacent and the writes come in runs instead of one scattered word per
// (digit, tile).  Each thread loads its RS_ITEMS keys of a tile before counting them, so
// that they are in flight together (a load-then-count loop waits on every load).
#define RS_HIST_TILES 16
__global__ __launch_bounds__(RS_THREADS) void k_rs_hist(const uint32_t *keys, size_t n,
                                                        int shift, int bits, uint32_t *hist,
                                                        uint32_t nblk, uint32_t tpw) {
  extern __shared__ uint32_t cnt[];  // [tpw][nb]
  const uint32_t nb = 1u << bits, mask = nb - 1u;
  const uint32_t t0 = blockIdx.x * tpw;
  const uint32_t nt = nblk - t0 < tpw ? nblk - t0 : tpw;
  for (uint32_t d = threadIdx.x; d < nt * nb; d += RS_THREADS) cnt[d] = 0;
  __syncthreads();
  // the workgroup's keys are contiguous
  const size_t base = (size_t)t0 * RS_TILE;
  const uint32_t nk =
      (uint32_t)((size_t)nt * RS_TILE < n - base ? (size_t)nt * RS_TILE : n - base);
  for (uint32_t t = 0; t < nt; ++t) {
    uint32_t kv[RS_ITEMS];
#pragma unroll
    for (int r = 0; r < RS_ITEMS; ++r) {
      const uint32_t j = t * RS_TILE + r * RS_THREADS + threadIdx.x;
      kv[r] = j < nk ? keys[base + j] : 0u;
    }
#pragma unroll
    for (int r = 0; r < RS_ITEMS; ++r) {
      const uint32_t j = t * RS_TILE + r * RS_THREADS + threadIdx.x;
      if (j < nk) atomicAdd(&cnt[t * nb + ((kv[r] >> shift) & mask)], 1u);
    }
  }
  __syncthreads();
  for (uint32_t j = threadIdx.x; j < nt * nb; j += RS_THREADS) {
    const uint32_t d = j / nt, t = j % nt;
    hist[(size_t)d * nblk + t0 + t] = cnt[t * nb + d];
  }
}

// Payload: pass 0 reads it from the caller's separate x/y arrays (px0, py0), later
// passes from the interleaved array pin; it is written interleaved to pout.
//
// Each tile is first sorted by digit in LDS, then written out in that order, so
// consecutive threads store consecutive records of one digit: the global writes form runs
// instead of single scattered records.  The order is stable: a record's rank among equal
// digits comes from ballot peer masks within its wave, and the waves' per-digit counts,
// kept for every round of the tile, are turned into offsets in record order (round, then
// wave, then lane) by one pass per digit -- five barriers per tile.
__global__ __launch_bounds__(RS_THREADS) void k_rs_scatter(
    const uint32_t *kin, const uint32_t *vin, uint32_t *kout, uint32_t *vout, size_t n,
    int shift, int bits, const uint32_t *offs, uint32_t nblk, const double *px0,
    const double *py0, const double2 *pin, double2 *pout) {
  constexpr int NW = RS_THREADS / GP_WAVE;
  // the per-(round, wave, digit) counts, then offsets, share LDS with the sorted tile
  __shared__ union {
    struct {
      uint32_t k[RS_TILE], v[RS_TILE];
      double2 p[RS_TILE];
    } t;
    uint16_t wo[RS_ITEMS * NW * RS_MAX_BUCKETS];
  } sm;
  __shared__ uint32_t lpos[RS_MAX_BUCKETS];   // local start of each digit
  __shared__ uint32_t delta[RS_MAX_BUCKETS];  // global start - local start of each digit
  const uint32_t tid = threadIdx.x, wave = tid / GP_WAVE;
  const uint32_t nb = 1u << bits, mask = nb - 1u;
  // Workgroup b runs on XCD b mod 8; each XCD takes a contiguous range of tiles, so the
  // runs that neighbouring tiles write for one digit (adjacent in the output, sharing
  // cache lines at their ends) are merged in one L2.  The grid covers 8 ranges of
  // ceil(nblk / 8) tiles; the few workgroups past the last tile exit.
  const uint32_t per = (nblk + GP_XCDS - 1) / GP_XCDS;
  const uint32_t tile = (blockIdx.x % GP_XCDS) * per + blockIdx.x / GP_XCDS;
  if (tile >= nblk) return;
  const size_t base = (size_t)tile * RS_TILE;
  const int tn = (int)((n - base) < (size_t)RS_TILE ? (n - base) : (size_t)RS_TILE);
  // the tile's records, in registers
  uint32_t k[RS_ITEMS], v[RS_ITEMS];
  double2 pl[RS_ITEMS];
#pragma unroll
  for (int r = 0; r < RS_ITEMS; ++r) {
    const int li = r * RS_THREADS + (int)tid;
    const size_t i = base + (size_t)li;
    const bool valid = li < tn;
    k[r] = valid ? kin[i] : 0u;
    v[r] = valid ? (vin ? vin[i] : (uint32_t)i) : 0u;
    pl[r] = make_double2(0.0, 0.0);
    if (valid && pout) pl[r] = pin ? pin[i] : make_double2(px0[i], py0[i]);
  }
  for (uint32_t j = tid; j < RS_ITEMS * NW * nb / 2; j += RS_THREADS) ((uint32_t *)sm.wo)[j] = 0u;
  __syncthreads();
  // rank of every record among the equal digits of its wave and round; the first such
  // lane records their count
  uint32_t rank[RS_ITEMS];
#pragma unroll
  for (int r = 0; r < RS_ITEMS; ++r) {
    const bool valid = r * RS_THREADS + (int)tid < tn;
    const uint32_t d = (k[r] >> shift) & mask;
    uint64_t peers = ballot(valid);
    for (int b = 0; b < bits; ++b) {
      const uint64_t m = ballot((d >> b) & 1u);
      peers &= ((d >> b) & 1u) ? m : ~m;
    }
    rank[r] = (uint32_t)__popcll(peers & lanemask_lt());
    if (valid && rank[r] == 0)
      sm.wo[(r * NW + (int)wave) * (int)nb + (int)d] = (uint16_t)__popcll(peers);
  }
  __syncthreads();
  // per digit: counts -> offsets within the digit, in record order; the tile's digit
  // histogram -> local starts and the global placement of each digit's run.  Thread t
  // takes digits dpt*t .. dpt*t + dpt - 1.
  {
    constexpr int DPT = RS_MAX_BUCKETS / RS_THREADS > 1 ? RS_MAX_BUCKETS / RS_THREADS : 1;
    const uint32_t dpt = nb > RS_THREADS ? nb / RS_THREADS : 1u;
    uint32_t run[DPT], sum = 0;
#pragma unroll
    for (int i = 0; i < DPT; ++i) {
      run[i] = 0;
      const uint32_t d = tid * dpt + (uint32_t)i;
      if ((uint32_t)i < dpt && d < nb) {
        for (int q = 0; q < RS_ITEMS * NW; ++q) {
          const uint32_t c = sm.wo[q * nb + d];
          sm.wo[q * nb + d] = (uint16_t)run[i];
          run[i] += c;
        }
      }
      sum += run[i];
    }
    uint32_t tot;
    uint32_t pre = block_excl_scan(sum, &tot);
#pragma unroll
    for (int i = 0; i < DPT; ++i) {
      const uint32_t d = tid * dpt + (uint32_t)i;
      if ((uint32_t)i < dpt && d < nb) {
        lpos[d] = pre;
        delta[d] = offs[(size_t)d * nblk + tile] - pre;
        pre += run[i];
      }
    }
  }
  __syncthreads();
  uint32_t pos[RS_ITEMS];
#pragma unroll
  for (int r = 0; r < RS_ITEMS; ++r) {
    const uint32_t d = (k[r] >> shift) & mask;
    pos[r] = lpos[d] + sm.wo[(r * NW + (int)wave) * nb + d] + rank[r];
  }
  __syncthreads();  // the offsets are read; the tile may now overwrite them
#pragma unroll
  for (int r = 0; r < RS_ITEMS; ++r) {
    if (r * RS_THREADS + (int)tid < tn) {
      sm.t.k[pos[r]] = k[r];
      sm.t.v[pos[r]] = v[r];
      if (pout) sm.t.p[pos[r]] = pl[r];
    }
  }
  __syncthreads();
  // write out in local order: global slot = local slot + (global - local start) of the digit
  for (int j = (int)tid; j < tn; j += RS_THREADS) {
    const uint32_t key = sm.t.k[j];
    const uint32_t gpos = delta[(key >> shift) & mask] + (uint32_t)j;
    kout[gpos] = key;
    vout[gpos] = sm.t.v[j];
    if (pout) pout[gpos] = sm.t.p[j];
  }
}

hipError_t launch_radix_sort(uint32_t *keyA, uint32_t *keyB, uint32_t *valA, uint32_t *valB,
                             size_t n, int nbits, bool values_are_identity, uint32_t *hist,
                             uint32_t *scan_tmp, hipStream_t s, uint32_t **keys_out,
                             uint32_t **vals_out, const double *px, const double *py,
                             double2 *plA, double2 *plB, double2 **pl_out) {
  *keys_out = keyA;
  *vals_out = valA;
  if (pl_out) *pl_out = plA;
  if (n == 0) return hipSuccess;
  const uint32_t nblk = (uint32_t)((n + RS_TILE - 1) / RS_TILE);
  int passes = (nbits + RS_MAX_BITS - 1) / RS_MAX_BITS;
  if (passes < 1) passes = 1;
  const int bits = nbits < 1 ? 1 : (nbits + passes - 1) / passes;
  uint32_t *ki = keyA, *ko = keyB, *vi = valA, *vo = valB;
  double2 *pi = nullptr, *po = pl_out ? plA : nullptr;
  bool ident = values_are_identity;
  for (int p = 0; p < passes; ++p) {
    const int shift = p * bits;
    const uint32_t tpw = RS_HIST_TILES;
    hipLaunchKernelGGL(k_rs_hist, dim3((nblk + tpw - 1) / tpw), dim3(RS_THREADS),
                       (size_t)tpw * ((size_t)1 << bits) * 4, s, ki, n, shift, bits, hist, nblk,
                       tpw);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    e = launch_exclusive_scan_u32(hist, hist, ((size_t)1 << bits) * nblk, scan_tmp, s);
    if (e != hipSuccess) return e;
    const uint32_t sgrid = (nblk + GP_XCDS - 1) / GP_XCDS * GP_XCDS;
    hipLaunchKernelGGL(k_rs_scatter, dim3(sgrid), dim3(RS_THREADS), 0, s, ki,
                       ident ? (const uint32_t *)nullptr : vi, ko, vo, n, shift, bits, hist,
                       nblk, px, py, (const double2 *)pi, po);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    ident = false;
    uint32_t *t = ki; ki = ko; ko = t;
    t = vi; vi = vo; vo = t;
    if (po) {
      pi = po;
      po = (po == plA) ? plB : plA;
    }
  }
  *keys_out = ki;
  *vals_out = vi;
  if (pl_out) *pl_out = pi;
  return hipSuccess;
}

// ------------------------------------------------------------------------- grid build

__device__ __forceinline__ int32_t upper_bound_i32(const int32_t *a, int32_t n, int32_t v) {
  int32_t lo = 0, hi = n;  // first index with a[i] > v
  while (lo < hi) {
    int32_t mid = (lo + hi) >> 1;
    if (a[mid] > v) hi = mid; else lo = mid + 1;
  }
  return lo;
}

// PIP: edge e = ring vertex e and its successor in the ring (the closing edge wraps).
// Stored as (lo.x, lo.y, hi.x, hi.y) with lo the endpoint of smaller y (for equal y the
// successor is lo, which is immaterial: such an edge never crosses) and the FP32 slope
// k = fl32((hi.x-lo.x)/(hi.y-lo.y)) used by the mixed form.
// P2P: segment s of polyline f joins vertices v and v+1, s = v - f.
__global__ void k_build_edges(const int32_t *rvo, const int32_t *fro, const double *x,
                              const double *y, int32_t nf, int32_t nrings, int32_t nverts,
                              int kind, double4 *edge64, float *k32, int32_t *eoff) {
  const int32_t stride = gridDim.x * blockDim.x;
  for (int32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < nverts; v += stride) {
    int32_t r = upper_bound_i32(rvo, nrings + 1, v) - 1;
    int32_t r0 = rvo[r], r1 = rvo[r + 1];
    if (kind == GP_PIP) {
      int32_t nx = (v + 1 < r1) ? v + 1 : r0;
      double ax = x[v], ay = y[v], bx = x[nx], by = y[nx];
      double lox, loy, hix, hiy;
      if (ay < by) { lox = ax; loy = ay; hix = bx; hiy = by; }
      else { lox = bx; loy = by; hix = ax; hiy = ay; }
      edge64[v] = make_double4(lox, loy, hix, hiy);
      k32[v] = (hiy == loy) ? 0.0f : (float)((hix - lox) / (hiy - loy));
    } else {
      if (v + 1 < r1) edge64[v - r] = make_double4(x[v], y[v], x[v + 1], y[v + 1]);
    }
  }
  for (int32_t f = blockIdx.x * blockDim.x + threadIdx.x; f <= nf; f += stride) {
    if (kind == GP_PIP) eoff[f] = rvo[fro[f]];
    else eoff[f] = rvo[f] - f;
  }
}

hipError_t launch_build_edges(const int32_t *rvo, const int32_t *fro, const double *x,
                              const double *y, int32_t nf, int32_t nrings, int32_t nverts,
                              gp_kind kind, double4 *edge64, float *k32, int32_t *eoff,
                              hipStream_t s) {
  size_t work = (size_t)(nverts > nf + 1 ? nverts : nf + 1);
  hipLaunchKernelGGL(k_build_edges, dim3(grid_for(work, 256, 8192)), dim3(256), 0, s, rvo, fro,
                     x, y, nf, nrings, nverts, (int)kind, edge64, k32, eoff);
  return hipGetLastError();
}

// P2P segment frames: u = d/|d| (u = (1, 0) for a zero-length segment), the absolute
// midpoint projections -m.u and -m.v with v = (-u.y, u.x), and the scaled FP32 constants
// the mixed kernel stages unchanged for every cell.
__global__ void k_build_frames(const double4 *seg, int32_t nseg, float scale, double4 *f64,
                               float4 *f32) {
  for (int32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < nseg; i += gridDim.x * blockDim.x) {
    const double4 r = seg[i];
    const double dx = r.z - r.x, dy = r.w - r.y;
    const double L = sqrt(dx * dx + dy * dy);
    const double ux = L > 0.0 ? dx / L : 1.0, uy = L > 0.0 ? dy / L : 0.0;
    const double mx = r.x + 0.5 * dx, my = r.y + 0.5 * dy;
    f64[i] = make_double4(ux, uy, -(mx * ux + my * uy), mx * uy - my * ux);
    const double sc = (double)scale;
    f32[i] = make_float4((float)(ux * sc), (float)(uy * sc), (float)(0.5 * L * sc), (float)L);
  }
}

hipError_t launch_build_frames(const double4 *seg64, int32_t nseg, float scale,
                               double4 *frame64, float4 *frame32, hipStream_t s) {
  if (nseg <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_build_frames, dim3(grid_for(nseg, 256, 8192)), dim3(256), 0, s, seg64, nseg,
                     scale, frame64, frame32);
  return hipGetLastError();
}

// Bounding circle of each block of P2P_BLOCK consecutive segments (blocks may span two
// polylines; the circle still contains every segment of the block): centre of the
// endpoints' box, radius the largest endpoint distance, widened by 2^-40 relative so
// that the FP64 rounding of its computation cannot make it too small.
__global__ void k_build_circles(const double4 *seg, int32_t nseg, double4 *circ) {
  const int32_t nb = (nseg + P2P_BLOCK - 1) / P2P_BLOCK;
  for (int32_t b = blockIdx.x * blockDim.x + threadIdx.x; b < nb; b += gridDim.x * blockDim.x) {
    const int32_t e0 = b * P2P_BLOCK, e1 = min(e0 + P2P_BLOCK, nseg);
    double lx = INFINITY, ly = INFINITY, hx = -INFINITY, hy = -INFINITY;
    for (int32_t e = e0; e < e1; ++e) {
      const double4 r = seg[e];
      lx = fmin(lx, fmin(r.x, r.z)); hx = fmax(hx, fmax(r.x, r.z));
      ly = fmin(ly, fmin(r.y, r.w)); hy = fmax(hy, fmax(r.y, r.w));
    }
    const double cx = 0.5 * (lx + hx), cy = 0.5 * (ly + hy);
    double r2 = 0.0;
    for (int32_t e = e0; e < e1; ++e) {
      const double4 r = seg[e];
      const double ax = r.x - cx, ay = r.y - cy, bx = r.z - cx, by = r.w - cy;
      r2 = fmax(r2, fmax(ax * ax + ay * ay, bx * bx + by * by));
    }
    circ[b] = make_double4(cx, cy, sqrt(r2) * (1.0 + 0x1p-40), 0.0);
  }
}

hipError_t launch_build_circles(const double4 *seg64, int32_t nseg, double4 *circ,
                                hipStream_t s) {
  if (nseg <= 0) return hipSuccess;
  const int32_t nb = (nseg + P2P_BLOCK - 1) / P2P_BLOCK;
  hipLaunchKernelGGL(k_build_circles, dim3(grid_for(nb, 256, 8192)), dim3(256), 0, s, seg64,
                     nseg, circ);
  return hipGetLastError();
}

// Bounding box of a segment, expanded by D and padded like the feature MBBs:
// (min x, min y, max x, max y).
__device__ __forceinline__ double4 seg_box(const double4 r, double D, double pad) {
  return make_double4((fmin(r.x, r.z) - D) - pad, (fmin(r.y, r.w) - D) - pad,
                      (fmax(r.x, r.z) + D) + pad, (fmax(r.y, r.w) + D) + pad);
}

// Each segment's box, in the MBB layout the rasteriser takes.
__global__ void k_seg_boxes(const double4 *seg, int32_t nseg, double D, double pad, double *box) {
  for (int32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < nseg; i += gridDim.x * blockDim.x) {
    const double4 b = seg_box(seg[i], D, pad);
    box[4 * (size_t)i + 0] = b.x;
    box[4 * (size_t)i + 1] = b.y;
    box[4 * (size_t)i + 2] = b.z;
    box[4 * (size_t)i + 3] = b.w;
  }
}

hipError_t launch_seg_boxes(const double4 *seg64, int32_t nseg, double D, double pad,
                            double *box, hipStream_t s) {
  if (nseg <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_seg_boxes, dim3(grid_for(nseg, 256, 8192)), dim3(256), 0, s, seg64, nseg,
                     D, pad, box);
  return hipGetLastError();
}

// Polyline of each segment (segments are stored polyline by polyline).
__global__ void k_seg2f(const int32_t *eoff, int32_t nf, int32_t *seg2f) {
  for (int32_t f = blockIdx.x * blockDim.x + threadIdx.x; f < nf; f += gridDim.x * blockDim.x)
    for (int32_t e = eoff[f]; e < eoff[f + 1]; ++e) seg2f[e] = f;
}

hipError_t launch_seg2f(const int32_t *eoff, int32_t nf, int32_t *seg2f, hipStream_t s) {
  if (nf <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_seg2f, dim3(grid_for(nf, 256, 8192)), dim3(256), 0, s, eoff, nf, seg2f);
  return hipGetLastError();
}

__global__ void k_cell_counts(const int32_t *off, int32_t ncells, int64_t *cnt) {
  for (int32_t c = blockIdx.x * blockDim.x + threadIdx.x; c < ncells; c += gridDim.x * blockDim.x)
    cnt[c] = (int64_t)(off[c + 1] - off[c]);
}

hipError_t launch_cell_counts(const int32_t *off, int32_t ncells, int64_t *cnt, hipStream_t s) {
  hipLaunchKernelGGL(k_cell_counts, dim3(grid_for(ncells, 256, 8192)), dim3(256), 0, s, off,
                     ncells, cnt);
  return hipGetLastError();
}

// Feature MBB over all of its vertices; P2P expands by D; both pad by cs*2^-20.
__global__ void k_mbb(const int32_t *rvo, const int32_t *fro, const double *x, const double *y,
                      int32_t nf, int kind, double D, double cs, double *mbb) {
  const double pad = cs * 0x1p-20;
  for (int32_t f = blockIdx.x * blockDim.x + threadIdx.x; f < nf;
       f += gridDim.x * blockDim.x) {
    int32_t v0 = kind == GP_PIP ? rvo[fro[f]] : rvo[f];
    int32_t v1 = kind == GP_PIP ? rvo[fro[f + 1]] : rvo[f + 1];
    double mnx = INFINITY, mny = INFINITY, mxx = -INFINITY, mxy = -INFINITY;
    for (int32_t v = v0; v < v1; ++v) {
      double a = x[v], b = y[v];
      if (a < mnx) mnx = a;
      if (a > mxx) mxx = a;
      if (b < mny) mny = b;
      if (b > mxy) mxy = b;
    }
    if (kind == GP_P2P) {
      mnx = mnx - D; mny = mny - D; mxx = mxx + D; mxy = mxy + D;
    }
    mbb[4 * (size_t)f + 0] = mnx - pad;
    mbb[4 * (size_t)f + 1] = mny - pad;
    mbb[4 * (size_t)f + 2] = mxx + pad;
    mbb[4 * (size_t)f + 3] = mxy + pad;
  }
}

hipError_t launch_mbb(const int32_t *rvo, const int32_t *fro, const double *x, const double *y,
                      int32_t nf, gp_kind kind, double D, double cs, double *mbb,
                      hipStream_t s) {
  if (nf == 0) return hipSuccess;
  hipLaunchKernelGGL(k_mbb, dim3(grid_for(nf, 64, 8192)), dim3(64), 0, s, rvo, fro, x, y, nf,
                     (int)kind, D, cs, mbb);
  return hipGetLastError();
}

__global__ __launch_bounds__(1024) void k_extent(const double *mbb, int32_t nf, double *out) {
  __shared__ double red[4][1024];
  double lx = INFINITY, ly = INFINITY, hx = -INFINITY, hy = -INFINITY;
  for (int32_t f = threadIdx.x; f < nf; f += blockDim.x) {
    lx = fmin(lx, mbb[4 * (size_t)f + 0]);
    ly = fmin(ly, mbb[4 * (size_t)f + 1]);
    hx = fmax(hx, mbb[4 * (size_t)f + 2]);
    hy = fmax(hy, mbb[4 * (size_t)f + 3]);
  }
  red[0][threadIdx.x] = lx; red[1][threadIdx.x] = ly;
  red[2][threadIdx.x] = hx; red[3][threadIdx.x] = hy;
  __syncthreads();
  for (int w = 512; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      red[0][threadIdx.x] = fmin(red[0][threadIdx.x], red[0][threadIdx.x + w]);
      red[1][threadIdx.x] = fmin(red[1][threadIdx.x], red[1][threadIdx.x + w]);
      red[2][threadIdx.x] = fmax(red[2][threadIdx.x], red[2][threadIdx.x + w]);
      red[3][threadIdx.x] = fmax(red[3][threadIdx.x], red[3][threadIdx.x + w]);
    }
    __syncthreads();
  }
  if (threadIdx.x < 4) out[threadIdx.x] = red[threadIdx.x][0];
}

hipError_t launch_extent(const double *mbb, int32_t nf, double *out4, hipStream_t s) {
  hipLaunchKernelGGL(k_extent, dim3(1), dim3(1024), 0, s, mbb, nf, out4);
  return hipGetLastError();
}

// Cell index range [lo, hi] an interval [a, b] touches on one axis, clamped to the grid;
// false when it misses the grid.
__device__ __forceinline__ bool axis_range(double a, double b, double o, double cs, int32_t n,
                                           int32_t *lo, int32_t *hi) {
  double fa = floor((a - o) / cs);
  double fb = floor((b - o) / cs);
  if (fb < 0.0 || fa > (double)(n - 1)) return false;
  *lo = fa < 0.0 ? 0 : (int32_t)fa;
  *hi = fb > (double)(n - 1) ? n - 1 : (int32_t)fb;
  return true;
}

__global__ void k_raster_count(const double *mbb, int32_t nf, double x0, double y0, double cs,
                               int32_t nx, int32_t ny, uint32_t *cnt) {
  for (int32_t f = blockIdx.x * blockDim.x + threadIdx.x; f < nf;
       f += gridDim.x * blockDim.x) {
    int32_t ax, bx, ay, by;
    uint32_t c = 0;
    if (axis_range(mbb[4 * (size_t)f + 0], mbb[4 * (size_t)f + 2], x0, cs, nx, &ax, &bx) &&
        axis_range(mbb[4 * (size_t)f + 1], mbb[4 * (size_t)f + 3], y0, cs, ny, &ay, &by))
      c = (uint32_t)(bx - ax + 1) * (uint32_t)(by - ay + 1);
    cnt[f] = c;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) cnt[nf] = 0;
}

hipError_t launch_raster_count(const double *mbb, int32_t nf, double x0, double y0, double cs,
                               int32_t nx, int32_t ny, uint32_t *cnt, hipStream_t s) {
  hipLaunchKernelGGL(k_raster_count, dim3(grid_for(nf + 1, 256, 8192)), dim3(256), 0, s, mbb,
                     nf, x0, y0, cs, nx, ny, cnt);
  return hipGetLastError();
}

// 64-bit total of n u32 counts (the (cell, feature) pair count before the 32-bit scan:
// a per-feature count is at most the grid's 2^28 cells, but their sum may pass 2^32).
__global__ __launch_bounds__(256) void k_sum_u32(const uint32_t *v, size_t n,
                                                 unsigned long long *out) {
  unsigned long long t = 0;
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x)
    t += v[i];
  for (int off = 32; off > 0; off >>= 1) t += __shfl_xor(t, off, GP_WAVE);
  if (lane_id() == 0 && t) atomicAdd(out, t);
}

hipError_t launch_sum_u32(const uint32_t *v, size_t n, unsigned long long *out, hipStream_t s) {
  hipError_t e = launch_fill_u32((uint32_t *)out, 0u, 2, s);
  if (e != hipSuccess || n == 0) return e;
  hipLaunchKernelGGL(k_sum_u32, dim3(grid_for(n, 256, 4096)), dim3(256), 0, s, v, n, out);
  return hipGetLastError();
}

// The cells every segment's box reaches (the rasteriser's ranges of seg_box, so exactly
// the cells a segment list would hold it in): (x lo, x hi, y lo, y hi), empty when the
// box misses the grid.
__global__ void k_seg_cells(const double4 *seg, int32_t nseg, double D, double pad, double x0,
                            double y0, double cs, int32_t nx, int32_t ny, int4 *rc) {
  for (int32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < nseg; i += gridDim.x * blockDim.x) {
    const double4 b = seg_box(seg[i], D, pad);
    int32_t ax, bx, ay, by;
    if (axis_range(b.x, b.z, x0, cs, nx, &ax, &bx) && axis_range(b.y, b.w, y0, cs, ny, &ay, &by))
      rc[i] = make_int4(ax, bx, ay, by);
    else
      rc[i] = make_int4(1, 0, 1, 0);
  }
}

// Near-segment range of every (cell, candidate polyline) pair: from the first to one past
// the last of the polyline's segments whose box reaches the cell; the polyline's first
// segment alone when none does (then every segment is farther than D from the whole
// cell).  A segment within D of a point of the cell is inside the range, so the exact
// pass's minimum over the range equals the polyline's whenever that minimum is in range.
// One wave per pair, lanes over segments.
__global__ __launch_bounds__(256) void k_near_ranges(const uint32_t *pair_cell,
                                                     const int32_t *cand_id, int32_t npairs,
                                                     const int32_t *eoff, const int4 *rc,
                                                     int32_t nx, int2 *near) {
  const uint32_t lane = lane_id();
  const int32_t nw = (int32_t)(gridDim.x * (blockDim.x / GP_WAVE));
  for (int32_t k = (int32_t)(blockIdx.x * (blockDim.x / GP_WAVE) + threadIdx.x / GP_WAVE);
       k < npairs; k += nw) {
    const int32_t cell = (int32_t)pair_cell[k];
    const int32_t cx = cell % nx, cy = cell / nx;
    const int32_t f = cand_id[k];
    const int32_t s0 = eoff[f], s1 = eoff[f + 1];
    int32_t lo = -1, hi = -1;
    for (int32_t base = s0; base < s1; base += GP_WAVE) {
      const int32_t sg = base + (int32_t)lane;
      bool nr = false;
      if (sg < s1) {
        const int4 r = rc[sg];
        nr = cx >= r.x && cx <= r.y && cy >= r.z && cy <= r.w;
      }
      const uint64_t m = ballot(nr);
      if (m) {
        if (lo < 0) lo = base + (int32_t)__builtin_ctzll(m);
        hi = base + 63 - (int32_t)__builtin_clzll(m);
      }
    }
    if (lane == 0) near[k] = lo < 0 ? make_int2(s0, s0 + 1) : make_int2(lo, hi + 1);
  }
}

hipError_t launch_near_ranges(const double4 *seg64, int32_t nseg, double D, double pad,
                              double x0, double y0, double cs, int32_t nx, int32_t ny,
                              const uint32_t *pair_cell, const int32_t *cand_id, int32_t npairs,
                              const int32_t *eoff, int4 *rc, int2 *near, hipStream_t s) {
  if (nseg <= 0 || npairs <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_seg_cells, dim3(grid_for(nseg, 256, 8192)), dim3(256), 0, s, seg64, nseg,
                     D, pad, x0, y0, cs, nx, ny, rc);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int64_t blocks = std::min<int64_t>(((int64_t)npairs + 3) / 4, 65536);
  hipLaunchKernelGGL(k_near_ranges, dim3((unsigned)blocks), dim3(256), 0, s, pair_cell, cand_id,
                     npairs, eoff, rc, nx, near);
  return hipGetLastError();
}

// One wavefront per feature: its cells are written row by row, lanes across a row.
__global__ __launch_bounds__(64) void k_raster_emit(const double *mbb, int32_t nf, double x0,
                                                    double y0, double cs, int32_t nx,
                                                    int32_t ny, const uint32_t *off,
                                                    uint32_t *pcell, uint32_t *pfid) {
  for (int32_t f = blockIdx.x; f < nf; f += gridDim.x) {
    int32_t ax, bx, ay, by;
    if (!axis_range(mbb[4 * (size_t)f + 0], mbb[4 * (size_t)f + 2], x0, cs, nx, &ax, &bx) ||
        !axis_range(mbb[4 * (size_t)f + 1], mbb[4 * (size_t)f + 3], y0, cs, ny, &ay, &by))
      continue;
    uint32_t o = off[f];
    int32_t w = bx - ax + 1;
    for (int32_t iy = ay; iy <= by; ++iy)
      for (int32_t k = threadIdx.x; k < w; k += 64) {
        uint32_t pos = o + (uint32_t)(iy - ay) * (uint32_t)w + (uint32_t)k;
        pcell[pos] = (uint32_t)iy * (uint32_t)nx + (uint32_t)(ax + k);
        pfid[pos] = (uint32_t)f;
      }
  }
}

hipError_t launch_raster_emit(const double *mbb, int32_t nf, double x0, double y0, double cs,
                              int32_t nx, int32_t ny, const uint32_t *off, uint32_t *pcell,
                              uint32_t *pfid, hipStream_t s) {
  if (nf == 0) return hipSuccess;
  hipLaunchKernelGGL(k_raster_emit, dim3(nf < 65536 ? nf : 65536), dim3(64), 0, s, mbb, nf, x0,
                     y0, cs, nx, ny, off, pcell, pfid);
  return hipGetLastError();
}

__global__ void k_histogram(const uint32_t *keys, size_t n, uint32_t *cnt) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x)
    atomicAdd(&cnt[keys[i]], 1u);
}

hipError_t launch_histogram(const uint32_t *keys, size_t n, uint32_t *cnt, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_histogram, dim3(grid_for(n, 256, 8192)), dim3(256), 0, s, keys, n, cnt);
  return hipGetLastError();
}

// Crossing of the +x ray from p with edge (lo, hi): half-open in y, strictly right.
__device__ __forceinline__ bool cross64(double px, double py, double lox, double loy, double w,
                                        double hiy, double h) {
  bool st = (loy <= py) & (py < hiy);
  double lhs = (px - lox) * h;
  double rhs = w * (py - loy);
  return st & (lhs < rhs);
}

// Edges a query tests per point of each cell: all candidates' edges, or with cell
// classes only the boundary pairs' edges up to the first inside pair (which decides
// every point still undecided, so the refinement stops there).
__global__ void k_cell_edges(const int32_t *cand_off, const int32_t *cand_id, const int32_t *eoff,
                             const uint8_t *cls, int32_t ncells, int64_t *cell_edges) {
  for (int32_t c = blockIdx.x * blockDim.x + threadIdx.x; c < ncells;
       c += gridDim.x * blockDim.x) {
    int64_t e = 0;
    for (int32_t k = cand_off[c]; k < cand_off[c + 1]; ++k) {
      if (cls && cls[k] == 1) break;
      if (cls && cls[k] == 0) continue;
      int32_t f = cand_id[k];
      e += (int64_t)(eoff[f + 1] - eoff[f]);
    }
    cell_edges[c] = e;
  }
}

// Cell classes of PIP candidate pairs (Sec. III.A), one wavefront per pair.  Boundary
// (2) when any edge's bounding box meets the cell widened by `margin`; else the cell
// lies wholly inside (1) or outside (0) the polygon, and the FP64 crossing parity of its
// centre says which: with every edge at least `margin` from the cell, each crossing
// predicate is exact for every point of the cell, so all of them share the centre's
// parity.
__global__ void k_classify_pairs(const uint32_t *pair_cell, const int32_t *cand_id,
                                 int32_t npairs, const int32_t *eoff, const double4 *edge64,
                                 double x0, double y0, double cs, int32_t nx, double margin,
                                 uint8_t *cls) {
  const uint32_t lane = lane_id();
  const int32_t nw = (int32_t)(gridDim.x * (blockDim.x / GP_WAVE));
  for (int32_t p = (int32_t)(blockIdx.x * (blockDim.x / GP_WAVE) + threadIdx.x / GP_WAVE);
       p < npairs; p += nw) {
    const uint32_t c = pair_cell[p];
    const int32_t f = cand_id[p];
    const double bx0 = x0 + (double)(c % (uint32_t)nx) * cs;
    const double by0 = y0 + (double)(c / (uint32_t)nx) * cs;
    const double bx1 = bx0 + cs, by1 = by0 + cs;
    const double qx = bx0 + 0.5 * cs, qy = by0 + 0.5 * cs;
    bool touch = false;
    uint64_t par = 0;
    const int32_t e1 = eoff[f + 1];
    for (int32_t e = eoff[f] + (int32_t)lane; e - (int32_t)lane < e1; e += GP_WAVE) {
      bool cr = false;
      if (e < e1) {
        const double4 r = edge64[e];  // (lo.x, lo.y, hi.x, hi.y)
        const double mnx = fmin(r.x, r.z), mxx = fmax(r.x, r.z);
        touch |= !(mxx < bx0 - margin || mnx > bx1 + margin || r.w < by0 - margin ||
                   r.y > by1 + margin);
        cr = cross64(qx, qy, r.x, r.y, r.z - r.x, r.w, r.w - r.y);
      }
      par ^= ballot(cr);
    }
    const bool bd = ballot(touch) != 0;
    if (lane == 0) cls[p] = bd ? 2 : (__popcll(par) & 1 ? 1 : 0);
  }
}

hipError_t launch_classify_pairs(const uint32_t *pair_cell, const int32_t *cand_id,
                                 int32_t npairs, const int32_t *eoff, const double4 *edge64,
                                 double x0, double y0, double cs, int32_t nx, double margin,
                                 uint8_t *cand_class, hipStream_t s) {
  if (npairs <= 0) return hipSuccess;
  const unsigned g = grid_for((size_t)npairs * GP_WAVE, 256, 8192);
  hipLaunchKernelGGL(k_classify_pairs, dim3(g), dim3(256), 0, s, pair_cell, cand_id, npairs,
                     eoff, edge64, x0, y0, cs, nx, margin, cand_class);
  return hipGetLastError();
}

hipError_t launch_cell_edges(const int32_t *cand_off, const int32_t *cand_id,
                             const int32_t *eoff, const uint8_t *cand_class, int32_t ncells,
                             int64_t *cell_edges, hipStream_t s) {
  hipLaunchKernelGGL(k_cell_edges, dim3(grid_for(ncells, 256, 8192)), dim3(256), 0, s, cand_off,
                     cand_id, eoff, cand_class, ncells, cell_edges);
  return hipGetLastError();
}

// ------------------------------------------------------------------------- point pipeline

// Cell id of each point; ncells (sorts last) when outside the extent or not finite.
__global__ void k_hash(const double *px, const double *py, int64_t n, double x0, double y0,
                       double cs, int32_t nx, int32_t ny, uint32_t *key) {
  const uint32_t ncells = (uint32_t)nx * (uint32_t)ny;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    double fx = floor((px[i] - x0) / cs);
    double fy = floor((py[i] - y0) / cs);
    bool ok = fx >= 0.0 && fx < (double)nx && fy >= 0.0 && fy < (double)ny;
    key[i] = ok ? (uint32_t)fy * (uint32_t)nx + (uint32_t)fx : ncells;
  }
}

hipError_t launch_hash(const double *px, const double *py, int64_t n, double x0, double y0,
                       double cs, int32_t nx, int32_t ny, uint32_t *key, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_hash, dim3(grid_for(n, 256, 16384)), dim3(256), 0, s, px, py, n, x0, y0,
                     cs, nx, ny, key);
  return hipGetLastError();
}

// pt_off[c] = number of sorted keys < c, for c in [0, ncells].
__global__ void k_offsets(const uint32_t *skey, int64_t n, int32_t ncells, int32_t *pt_off) {
  for (int32_t c = blockIdx.x * blockDim.x + threadIdx.x; c <= ncells;
       c += gridDim.x * blockDim.x) {
    int64_t lo = 0, hi = n;
    while (lo < hi) {
      int64_t mid = (lo + hi) >> 1;
      if (skey[mid] < (uint32_t)c) lo = mid + 1; else hi = mid;
    }
    pt_off[c] = (int32_t)lo;
  }
}

hipError_t launch_offsets(const uint32_t *skey, int64_t n, int32_t ncells, int32_t *pt_off,
                          hipStream_t s) {
  hipLaunchKernelGGL(k_offsets, dim3(grid_for((size_t)ncells + 1, 256, 8192)), dim3(256), 0, s,
                     skey, n, ncells, pt_off);
  return hipGetLastError();
}

__device__ __forceinline__ double cell_cx(const RefineArgs &a, uint32_t cell) {
  return a.x0 + ((double)(cell % (uint32_t)a.nx) + 0.5) * a.cs;
}
__device__ __forceinline__ double cell_cy(const RefineArgs &a, uint32_t cell) {
  return a.y0 + ((double)(cell / (uint32_t)a.nx) + 0.5) * a.cs;
}

// Points the filter leaves unpaired (outside the extent, or in a cell without
// candidates) get their final (-1, +inf) here; the rest are counted.
__global__ __launch_bounds__(256) void k_unpaired(RefineArgs a, int64_t n, uint32_t *n_paired) {
  __shared__ uint32_t wsum[256 / GP_WAVE];
  uint32_t cnt = 0;  // per-wave count (uniform), one atomic per block at the end
  for (int64_t i0 = blockIdx.x * (int64_t)blockDim.x; i0 < n;
       i0 += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = i0 + threadIdx.x;
    const bool in = i < n;
    const uint32_t k = in ? a.skey[i] : 0u;
    const bool paired = in && k < (uint32_t)a.ncells && a.cand_off[k + 1] > a.cand_off[k];
    cnt += (uint32_t)__popcll(ballot(paired));
    if (in && !paired) {
      const uint32_t j = a.perm[i];
      a.out_id[j] = -1;
      if (a.out_dist) a.out_dist[j] = INFINITY;
    }
  }
  if (lane_id() == 0) wsum[threadIdx.x / GP_WAVE] = cnt;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t t = 0;
    for (int w = 0; w < 256 / GP_WAVE; ++w) t += wsum[w];
    if (t) atomicAdd(n_paired, t);
  }
}

hipError_t launch_unpaired(const RefineArgs &a, int64_t n, uint32_t *n_paired, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_unpaired, dim3(grid_for(n, 256, 4096)), dim3(256), 0, s, a, n, n_paired);
  return hipGetLastError();
}

// Items per cell, and the test counts: tests[0] over the candidates a query refines,
// tests[1] over all candidates (only when cell_edges_all is given, i.e. cell classes).
__global__ void k_item_count(const int32_t *pt_off, const int32_t *cand_off,
                             const int64_t *cell_edges, const int64_t *cell_edges_all,
                             int32_t ncells, int32_t chunk, uint32_t *cnt,
                             unsigned long long *tests) {
  // the loop bound is uniform per block so that every lane joins the wave reduction
  for (int32_t c0 = blockIdx.x * blockDim.x; c0 <= ncells; c0 += gridDim.x * blockDim.x) {
    const int32_t c = c0 + (int32_t)threadIdx.x;
    uint32_t q = 0;
    unsigned long long t = 0, ta = 0;
    if (c < ncells) {
      int32_t np = pt_off[c + 1] - pt_off[c];
      int32_t nc = cand_off[c + 1] - cand_off[c];
      if (np > 0 && nc > 0) {
        q = (uint32_t)((np + chunk - 1) / chunk);
        t = (unsigned long long)np * (unsigned long long)cell_edges[c];
        if (cell_edges_all) ta = (unsigned long long)np * (unsigned long long)cell_edges_all[c];
      }
    }
    if (c <= ncells) cnt[c] = q;
    // wavefront reductions of the test counts, one atomic per wave
    for (int off = 32; off > 0; off >>= 1) {
      t += __shfl_xor(t, off, GP_WAVE);
      ta += __shfl_xor(ta, off, GP_WAVE);
    }
    if (lane_id() == 0 && t) atomicAdd(tests, t);
    if (lane_id() == 0 && ta) atomicAdd(tests + 1, ta);
  }
}

__global__ void k_item_emit(const int32_t *pt_off, int32_t ncells, int32_t chunk,
                            const uint32_t *item_off, Item *items) {
  for (int32_t c = blockIdx.x * blockDim.x + threadIdx.x; c < ncells;
       c += gridDim.x * blockDim.x) {
    uint32_t o = item_off[c], q = item_off[c + 1] - o;
    int32_t p0 = pt_off[c], np = pt_off[c + 1] - p0;
    for (uint32_t k = 0; k < q; ++k) {
      int32_t lo = p0 + (int32_t)k * chunk;
      int32_t cnt = np - (int32_t)k * chunk;
      items[o + k] = Item{c, lo, cnt < chunk ? cnt : chunk, 0};
    }
  }
}

hipError_t launch_items(const int32_t *pt_off, const int32_t *cand_off,
                        const int64_t *cell_edges, const int64_t *cell_edges_all,
                        int32_t ncells, int32_t chunk,
                        uint32_t *item_cnt, uint32_t *scan_tmp, Item *items, uint32_t *counters,
                        unsigned long long *tests, hipStream_t s) {
  (void)counters;
  unsigned g = grid_for((size_t)ncells + 1, 256, 8192);
  hipLaunchKernelGGL(k_item_count, dim3(g), dim3(256), 0, s, pt_off, cand_off, cell_edges,
                     cell_edges_all, ncells, chunk, item_cnt, tests);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  e = launch_exclusive_scan_u32(item_cnt, item_cnt, (size_t)ncells + 1, scan_tmp, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_item_emit, dim3(g), dim3(256), 0, s, pt_off, ncells, chunk, item_cnt,
                     items);
  return hipGetLastError();
}

// Longest-first order of the items (the classic rule for scheduling jobs of unequal
// length on parallel machines): a cost bucket per item, 4 per octave of its test count
// npts * cell_edges, kept in Item::cost_rank; sort keys put large buckets first and the
// slots beyond the item count (key 255) last.
__device__ __forceinline__ uint32_t cost_bucket(uint64_t c) {
  if (c == 0) return 0;
  const uint32_t e = 63u - (uint32_t)__clzll(c);  // floor(log2 c)
  const uint32_t frac = e >= 2 ? (uint32_t)(c >> (e - 2)) & 3u : (uint32_t)(c << (2 - e)) & 3u;
  const uint32_t b = 4u * e + frac;
  return b < 254u ? b : 254u;
}

__global__ void k_item_keys(Item *items, const uint32_t *n_items, int64_t max_items,
                            const int64_t *cell_edges, uint32_t *keys) {
  const uint32_t n = *n_items;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < max_items;
       i += (int64_t)gridDim.x * blockDim.x) {
    uint32_t key = 255u;
    if (i < (int64_t)n) {
      Item it = items[i];
      const uint32_t b = cost_bucket((uint64_t)it.npts * (uint64_t)cell_edges[it.cell]);
      items[i].cost_rank = (int32_t)b;
      key = 254u - b;
    }
    keys[i] = key;
  }
}

__global__ void k_item_gather(const Item *items, const uint32_t *idx, int64_t max_items,
                              const uint32_t *n_items, Item *out) {
  const uint32_t n = *n_items;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < (int64_t)n;
       i += (int64_t)gridDim.x * blockDim.x)
    out[i] = items[idx[i]];
}

hipError_t launch_order_items(Item *items, const uint32_t *n_items, int64_t max_items,
                              const int64_t *cell_edges, uint32_t *kA, uint32_t *kB,
                              uint32_t *vA, uint32_t *vB, uint32_t *hist, uint32_t *scan_tmp,
                              Item *out, hipStream_t s) {
  if (max_items <= 0) return hipSuccess;
  const unsigned g = grid_for((size_t)max_items, 256, 8192);
  hipLaunchKernelGGL(k_item_keys, dim3(g), dim3(256), 0, s, items, n_items, max_items,
                     cell_edges, kA);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  uint32_t *ks = nullptr, *vs = nullptr;
  e = launch_radix_sort(kA, kB, vA, vB, (size_t)max_items, 8, true, hist, scan_tmp, s, &ks, &vs);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_item_gather, dim3(g), dim3(256), 0, s, items, vs, max_items, n_items, out);
  return hipGetLastError();
}

__global__ void k_copy_perm(const uint32_t *perm, int64_t n, int32_t *out) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    out[i] = (int32_t)perm[i];
}

hipError_t launch_copy_perm(const uint32_t *perm, int64_t n, int32_t *out, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_copy_perm, dim3(grid_for(n, 256, 16384)), dim3(256), 0, s, perm, n, out);
  return hipGetLastError();
}

// ------------------------------------------------------------------------- FP64 tests
// The two refinement predicates in plain FP64, in the operation order of the
// definitions (Sec. III.C crossing, Sec. III.B / Fig. 2 segment distance).


// Squared distance from p to segment (a, b): endpoint a when t <= 0, endpoint b when
// t >= L2, else the perpendicular foot.
__device__ __forceinline__ double seg_d2_64(double px, double py, double ax, double ay,
                                            double bx, double by) {
  double dx = bx - ax, dy = by - ay;
  double wx = px - ax, wy = py - ay;
  double L2 = dx * dx + dy * dy;
  double t = wx * dx + wy * dy;
  if (t <= 0.0) return wx * wx + wy * wy;
  if (t >= L2) {
    double ex = px - bx, ey = py - by;
    return ex * ex + ey * ey;
  }
  double c = wx * dy - wy * dx;
  return (c * c) / L2;
}

// ------------------------------------------------------------------------- work queue

// Work queue of the persistent launches, with XCD locality.  Items come in cell order;
// blocks of GP_XBLOCK consecutive items go round-robin to GP_XCDS queues, and a
// workgroup pops from the queue of its XCD (workgroups are placed on the XCDs
// round-robin by index), so the items of one cell share an L2 and its staged edges or
// segment records are fetched from HBM once.  A workgroup whose queue is exhausted takes
// items from the next queues: every item is handed out exactly once, and each pop ends
// after at most GP_XCDS exhausted queues.  Returns n_items when nothing is left.  dead
// (one bit per queue, kept by the caller across its pops) marks the queues this
// workgroup has found exhausted, so that it asks each of them once: at the end of a
// launch the failed atomics of all workgroups queue up on the few counter addresses.
__device__ __forceinline__ uint32_t pop_item(const RefineArgs &a, uint32_t n_items,
                                             uint32_t &dead) {
  const uint32_t home = blockIdx.x % GP_XCDS;
  for (uint32_t k = 0; k < GP_XCDS; ++k) {
    const uint32_t q = (home + k) % GP_XCDS;
    if ((dead >> q) & 1u) continue;
    const uint32_t c = atomicAdd(a.item_counter + q, 1u);
    // the c-th item of queue q; increasing in c, so the first miss exhausts the queue
    const uint64_t it = ((uint64_t)(c / GP_XBLOCK) * GP_XCDS + q) * GP_XBLOCK + c % GP_XBLOCK;
    if (it < n_items) return (uint32_t)it;
    dead |= 1u << q;
  }
  return n_items;
}

__device__ __forceinline__ uint32_t next_item(const RefineArgs &a, uint32_t n_items,
                                              uint32_t &dead) {
  uint32_t it = 0;
  if (lane_id() == 0) it = pop_item(a, n_items, dead);
  return uniform(it);
}

// Append the flagged lanes' sorted positions to the FP64 recheck queue.
__device__ __forceinline__ void push_recheck(const RefineArgs &a, bool flag, uint32_t pos) {
  uint64_t m = ballot(flag);
  if (!m) return;
  uint32_t base = 0;
  if (lane_id() == 0) base = atomicAdd(a.rq_count, (uint32_t)__popcll(m));
  base = uniform(base);
  if (flag) a.rq[base + __popcll(m & lanemask_lt())] = pos;
}

// ------------------------------------------------------------------------- points

template <int PPL>
__device__ __forceinline__ void load_points64(const RefineArgs &a, const Item it,
                                              double (&px)[PPL], double (&py)[PPL]) {
  const uint32_t lane = lane_id();
#pragma unroll
  for (int j = 0; j < PPL; ++j) {
    const int idx = (int)lane + GP_WAVE * j;
    const double2 p = idx < it.npts ? a.xy[it.pt_lo + idx] : make_double2(0.0, 0.0);
    px[j] = p.x;
    py[j] = p.y;
  }
}

// FP32 coordinates rebased to the cell centre: fl32(fl64(p - c)).
template <int PPL>
__device__ __forceinline__ void load_points32(const RefineArgs &a, const Item it, double cx,
                                              double cy, float (&px)[PPL], float (&py)[PPL]) {
  const uint32_t lane = lane_id();
#pragma unroll
  for (int j = 0; j < PPL; ++j) {
    const int idx = (int)lane + GP_WAVE * j;
    const double2 p = idx < it.npts ? a.xy[it.pt_lo + idx] : make_double2(cx, cy);
    // + 0 turns a rebased -0 into +0, so the tests on bit patterns (u32 compares of
    // p.y - lo.y) see a point level with an endpoint as t = +0
    px[j] = (float)(p.x - cx) + 0.0f;
    py[j] = (float)(p.y - cy) + 0.0f;
  }
}

// ------------------------------------------------------------------------- PIP, FP64

struct alignas(16) PipRec64 {
  double lox, loy, hiy, w, h, pad;
};

// Vertex-parallel refinement of an item with few points (the alternative mapping of
// Sec. III.B): lanes take the edges of a candidate polygon, the wave loops over the
// item's points (lane p holds point p and its parity), and a point's crossing parity
// over a chunk of 64 edges is the popcount of one ballot.  FP64 in the definition's
// operation order, so its results are final in both precision forms.
__device__ void pip_vp_item(const RefineArgs &a, const Item it) {
  const uint32_t lane = lane_id();
  const int np = it.npts;  // <= a.vp_points <= 64
  double qx = 0.0, qy = 0.0;
  if ((int)lane < np) {
    const double2 p = a.xy[it.pt_lo + (int)lane];
    qx = p.x;
    qy = p.y;
  }
  int32_t best = -1;
  const int32_t k0 = a.cand_off[it.cell], k1 = a.cand_off[it.cell + 1];
  for (int32_t k = k0; k < k1; ++k) {
    const int32_t f = a.cand_id[k];
    const int cls = a.cand_class ? a.cand_class[k] : 2;
    if (cls == 0) continue;  // the cell lies outside polygon f
    if (cls == 1) {          // inside: every undecided point takes f
      if (best < 0) best = f;
      break;
    }
    uint32_t par = 0;
    const int32_t e1 = a.eoff[f + 1];
    for (int32_t e0 = a.eoff[f]; e0 < e1; e0 += GP_WAVE) {
      const int32_t e = e0 + (int32_t)lane;
      const bool act = e < e1;
      double lox = 0.0, loy = 0.0, w = 0.0, hiy = 0.0, h = 0.0;
      if (act) {
        const double4 r = a.edge64[e];
        lox = r.x;
        loy = r.y;
        w = r.z - r.x;
        hiy = r.w;
        h = r.w - r.y;
      }
      for (int p = 0; p < np; ++p) {
        const double px = __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(qx), p),
                                           __builtin_amdgcn_readlane(__double2loint(qx), p));
        const double py = __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(qy), p),
                                           __builtin_amdgcn_readlane(__double2loint(qy), p));
        const bool c = act && cross64(px, py, lox, loy, w, hiy, h);
        const uint32_t odd = (uint32_t)__popcll(ballot(c)) & 1u;
        if ((int)lane == p) par ^= odd;
      }
    }
    if ((int)lane < np && best < 0 && par) best = f;
  }
  if ((int)lane < np) a.out_id[a.perm[it.pt_lo + (int)lane]] = best;
}

template <int PPL>
__device__ void pip64_item(const RefineArgs &a, const Item it, PipRec64 *lds) {
  if (it.npts <= a.vp_points) {
    pip_vp_item(a, it);
    return;
  }
  const uint32_t lane = lane_id();
  const int EC = a.edge_chunk;
  double px[PPL], py[PPL];
  int32_t best[PPL];
  load_points64<PPL>(a, it, px, py);
#pragma unroll
  for (int j = 0; j < PPL; ++j) best[j] = -1;
  const int32_t k0 = a.cand_off[it.cell], k1 = a.cand_off[it.cell + 1];
  for (int32_t k = k0; k < k1; ++k) {
    const int32_t f = a.cand_id[k];
    const int cls = a.cand_class ? a.cand_class[k] : 2;
    if (cls == 0) continue;  // the cell lies outside polygon f
    if (cls == 1) {          // inside: every undecided point takes f, and all are decided
#pragma unroll
      for (int j = 0; j < PPL; ++j)
        if (best[j] < 0) best[j] = f;
      break;
    }
    const int32_t e0 = a.eoff[f], e1 = a.eoff[f + 1];
    uint64_t par[PPL];
#pragma unroll
    for (int j = 0; j < PPL; ++j) par[j] = 0;
    for (int32_t s = e0; s < e1; s += EC) {
      const int cnt = (e1 - s) < EC ? (e1 - s) : EC;
      __syncthreads();
      for (int t = lane; t < cnt; t += GP_WAVE) {
        const double4 r = a.edge64[s + t];
        PipRec64 q;
        q.lox = r.x; q.loy = r.y; q.hiy = r.w;
        q.w = r.z - r.x;
        q.h = r.w - r.y;
        q.pad = 0.0;
        lds[t] = q;
      }
      __syncthreads();
      for (int t = 0; t < cnt; ++t) {
        const PipRec64 q = lds[t];
#pragma unroll
        for (int j = 0; j < PPL; ++j) {
          const double lhs = (px[j] - q.lox) * q.h;
          const double rhs = q.w * (py[j] - q.loy);
          par[j] ^= ballot(q.loy <= py[j]) & ballot(py[j] < q.hiy) & ballot(lhs < rhs);
        }
      }
    }
#pragma unroll
    for (int j = 0; j < PPL; ++j)
      if (best[j] < 0 && ((par[j] >> lane) & 1ull)) best[j] = f;
  }
#pragma unroll
  for (int j = 0; j < PPL; ++j) {
    const int idx = (int)lane + GP_WAVE * j;
    if (idx < it.npts) a.out_id[a.perm[it.pt_lo + idx]] = best[j];
  }
}

// ------------------------------------------------------------------------- PIP, mixed
// FP32 on cell-rebased coordinates.  Each staged edge is classified for the cell:
//  * "plain": for every point of the cell the FP32 decision provably equals the FP64
//    one -- the edge lies wholly above or below the cell's y band, or wholly left of
//    the cell, or spans the band strictly while lying wholly right of the cell.  These
//    run the 4-instruction test (sub, fma, u32 straddle compare, x compare).
//  * "guarded": the rest (edges through or near the cell, endpoints inside its band).
//    Their test also raises a flag when the point is within the edge's error bound G
//    of the edge, or level with an endpoint in FP32; a flagged (point, polygon) pair
//    sends the point to the FP64 recheck when that polygon could still decide it.
// G = 2^-22 * (|k| (3B + 3|lo.y|) + |lo.x| + 3B), B the cell half-width bound: four
// times the rounding error of the FP32 intercept test against the FP64 predicate.

// Lane mask of the crossings of one edge.  Each compare is balloted on its own and
// the masks are combined on the scalar unit (a ballot of a combined predicate would
// cost two extra vector instructions per test).
__device__ __forceinline__ uint64_t plain_cross(float px, float py, const float4 e) {
  const float ty = py - e.y;
  const float xi = fmaf(ty, e.w, e.x);
  return ballot(__float_as_uint(ty) < __float_as_uint(e.z)) & ballot(px < xi);
}

template <int PPL>
__device__ void pipmix_item(const RefineArgs &a, const Item it, float4 *ldsA, float4 *ldsB,
                            float *ldsG) {
  if (it.npts <= a.vp_points) {
    pip_vp_item(a, it);
    return;
  }
  const uint32_t lane = lane_id();
  const int EC = a.edge_chunk;
  const double cx = cell_cx(a, (uint32_t)it.cell), cy = cell_cy(a, (uint32_t)it.cell);
  const float hb = a.half_box;
  float px[PPL], py[PPL];
  int32_t best[PPL];
  bool rq[PPL];
  load_points32<PPL>(a, it, cx, cy, px, py);
#pragma unroll
  for (int j = 0; j < PPL; ++j) {
    best[j] = -1;
    rq[j] = false;
  }
  const int32_t k0 = a.cand_off[it.cell], k1 = a.cand_off[it.cell + 1];
  for (int32_t k = k0; k < k1; ++k) {
    const int32_t f = a.cand_id[k];
    const int cls = a.cand_class ? a.cand_class[k] : 2;
    if (cls == 0) continue;  // the cell lies outside polygon f
    if (cls == 1) {          // inside: every undecided point takes f, and all are decided
#pragma unroll
      for (int j = 0; j < PPL; ++j)
        if (best[j] < 0 && !rq[j]) best[j] = f;
      break;
    }
    const int32_t e0 = a.eoff[f], e1 = a.eoff[f + 1];
    uint64_t par[PPL], flg[PPL];
#pragma unroll
    for (int j = 0; j < PPL; ++j) { par[j] = 0; flg[j] = 0; }
    for (int32_t s = e0; s < e1; s += EC) {
      const int cnt = (e1 - s) < EC ? (e1 - s) : EC;
      __syncthreads();
      uint32_t nA = 0, nB = 0;
      for (int base = 0; base < cnt; base += GP_WAVE) {
        const int t = base + (int)lane;
        const bool act = t < cnt;
        bool careful = false;
        float4 recA = make_float4(0.f, 0.f, 0.f, 0.f), recB = recA;
        float G = 0.f;
        if (act) {
          const double4 r = a.edge64[s + t];
          const float kk = a.k32[s + t];
          const float lx = (float)(r.x - cx), ly = (float)(r.y - cy);
          const float hy = (float)(r.w - cy);
          const bool horiz = r.y == r.w;
          const float h32 = hy - ly;
          G = 0x1p-22f * (fabsf(kk) * (3.0f * hb + 3.0f * fabsf(ly)) + fabsf(lx) + 3.0f * hb);
          const bool yout = (ly > hb) || (hy < -hb);
          const bool ystrict = (ly < -hb) && (hy > hb + 0x1p-20f * h32);
          const float ya = fmaxf(ly, -hb), yb = fminf(hy, hb);
          const float xa = fmaf(ya - ly, kk, lx), xb = fmaf(yb - ly, kk, lx);
          const bool xleft = fmaxf(xa, xb) < -hb - 2.0f * G;
          const bool xright = fminf(xa, xb) > hb + 2.0f * G;
          careful = !(horiz || yout || xleft || (ystrict && xright));
          recA = horiz ? make_float4(0.f, 3.0e38f, 0.f, 0.f) : make_float4(lx, ly, h32, kk);
          recB = make_float4(lx, ly, hy, kk);
        }
        const uint64_t mB = ballot(act && careful), mA = ballot(act && !careful);
        if (act && careful) {
          const uint32_t p = nB + __popcll(mB & lanemask_lt());
          ldsB[p] = recB;
          ldsG[p] = G;
        }
        if (act && !careful) ldsA[nA + __popcll(mA & lanemask_lt())] = recA;
        nA += __popcll(mA);
        nB += __popcll(mB);
      }
      __syncthreads();
      uint32_t t = 0;
      // eight or four edges per step: their LDS reads are in flight together, so a wave
      // waits on the LDS once per 8 * PPL (4 * PPL) tests
      for (; t + 8 <= nA; t += 8) {
        float4 e[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) e[q] = ldsA[t + q];
#pragma unroll
        for (int j = 0; j < PPL; ++j) {
          uint64_t m = 0;
#pragma unroll
          for (int q = 0; q < 8; ++q) m ^= plain_cross(px[j], py[j], e[q]);
          par[j] ^= m;
        }
      }
      for (; t + 4 <= nA; t += 4) {
        const float4 e0 = ldsA[t], e1 = ldsA[t + 1], e2 = ldsA[t + 2], e3 = ldsA[t + 3];
#pragma unroll
        for (int j = 0; j < PPL; ++j)
          par[j] ^= plain_cross(px[j], py[j], e0) ^ plain_cross(px[j], py[j], e1) ^
                    plain_cross(px[j], py[j], e2) ^ plain_cross(px[j], py[j], e3);
      }
      for (; t + 2 <= nA; t += 2) {
        const float4 e0 = ldsA[t], e1 = ldsA[t + 1];
#pragma unroll
        for (int j = 0; j < PPL; ++j)
          par[j] ^= plain_cross(px[j], py[j], e0) ^ plain_cross(px[j], py[j], e1);
      }
      if (t < nA) {
        const float4 e0 = ldsA[t];
#pragma unroll
        for (int j = 0; j < PPL; ++j) par[j] ^= plain_cross(px[j], py[j], e0);
      }
      auto guarded = [&](const float4 e, const float G) {
#pragma unroll
        for (int j = 0; j < PPL; ++j) {
          const float ty = py[j] - e.y;
          const float d = fmaf(ty, e.w, e.x) - px[j];
          const uint64_t st = ballot(ty >= 0.0f) & ballot(py[j] < e.z);
          const uint64_t eq = ballot(ty == 0.0f) | ballot(py[j] == e.z);
          par[j] ^= st & ballot(d > 0.0f);
          flg[j] |= (eq & ballot(!(d < -G))) | (st & ballot(!(fabsf(d) > G)));
        }
      };
      for (t = 0; t + 2 <= nB; t += 2) {  // two edges per step, reads in flight together
        const float4 ea = ldsB[t], eb = ldsB[t + 1];
        const float Ga = ldsG[t], Gb = ldsG[t + 1];
        guarded(ea, Ga);
        guarded(eb, Gb);
      }
      if (t < nB) guarded(ldsB[t], ldsG[t]);
    }
#pragma unroll
    for (int j = 0; j < PPL; ++j) {
      const bool odd = (par[j] >> lane) & 1ull;
      const bool fl = (flg[j] >> lane) & 1ull;
      if (best[j] < 0 && !rq[j]) {
        if (fl) rq[j] = true;
        else if (odd) best[j] = f;
      }
    }
  }
#pragma unroll
  for (int j = 0; j < PPL; ++j) {
    const int idx = (int)lane + GP_WAVE * j;
    const bool v = idx < it.npts;
    if (v && !rq[j]) a.out_id[a.perm[it.pt_lo + idx]] = best[j];
    push_recheck(a, v && rq[j], (uint32_t)(it.pt_lo + idx));
  }
}

// ------------------------------------------------------------------------- PIP, build-time records
// With prestage the grid build classifies every edge of every (cell, candidate polygon)
// pair once, for the mixed test of that cell (FP32 on coordinates rebased to the cell
// centre, hb the bound on a point's rebased coordinates), and stores the records the
// refinement reads:
//  PIP_PLAIN   horizontal, wholly above or below the cell's y band, wholly left of the
//              cell, or spanning the band strictly while right of it: the 4-instruction
//              test (subtract, FMA, straddle and x compares) equals the FP64 predicate for
//              every point of the cell.  Record (lo.x, lo.y, hi.y - lo.y, slope).
//  PIP_BAND    right of the cell by more than 2G over the band, with an endpoint inside it:
//              for every point of the cell the x part of the predicate holds in FP32 and
//              in FP64, so the crossing is the half-open straddle lo.y <= p.y < hi.y.  With
//              t = fl32(p.y - lo.y) and h = fl32(hi.y - lo.y) (rebased values), 0 < t < h
//              implies the FP64 straddle and t < 0 or t > h rules it out (rounding is
//              monotone); t = 0 or t = h is ambiguous and flags the (point, polygon) pair.
//              Record (lo.y, bits(h) - 1, bits(h), 0): the open straddle is one unsigned
//              compare of bits(t) - 1, the closed one of bits(t).
//  PIP_GUARDED everything else: the full test and the error-band flag, two slots
//              (lo.x, lo.y, hi.y, slope), (G, 0, 0, 0).
enum { PIP_PLAIN = 0, PIP_BAND = 1, PIP_GUARDED = 2 };

struct PipEdge {
  int cls;
  float4 rec;
  float G;
};

__device__ __forceinline__ PipEdge pip_classify(const double4 r, float kk, double cx, double cy,
                                                float hb) {
  PipEdge o;
  const float lx = (float)(r.x - cx), ly = (float)(r.y - cy), hy = (float)(r.w - cy);
  const bool horiz = r.y == r.w;
  const float h32 = hy - ly;
  o.G = 0x1p-22f * (fabsf(kk) * (3.0f * hb + 3.0f * fabsf(ly)) + fabsf(lx) + 3.0f * hb);
  const bool yout = (ly > hb) || (hy < -hb);
  const bool ystrict = (ly < -hb) && (hy > hb + 0x1p-20f * h32);
  const float ya = fmaxf(ly, -hb), yb = fminf(hy, hb);
  const float xa = fmaf(ya - ly, kk, lx), xb = fmaf(yb - ly, kk, lx);
  const bool xleft = fmaxf(xa, xb) < -hb - 2.0f * o.G;
  const bool xright = fminf(xa, xb) > hb + 2.0f * o.G;
  if (horiz || yout || xleft || (ystrict && xright)) {
    o.cls = PIP_PLAIN;
    o.rec = horiz ? make_float4(0.f, 3.0e38f, 0.f, 0.f) : make_float4(lx, ly, h32, kk);
  } else if (xright) {
    o.cls = PIP_BAND;
    const uint32_t hbits = __float_as_uint(h32);
    o.rec = make_float4(ly, __uint_as_float(hbits ? hbits - 1u : 0u), __uint_as_float(hbits),
                        0.f);
  } else {
    o.cls = PIP_GUARDED;
    o.rec = make_float4(lx, ly, hy, kk);
  }
  return o;
}

// One wave per (cell, candidate) pair, lanes over the polygon's edges.
__global__ __launch_bounds__(256) void k_pip_rec_count(const uint32_t *pair_cell,
                                                       const int32_t *cand_id, int32_t npairs,
                                                       const int32_t *eoff, const double4 *edge64,
                                                       const float *k32, double x0, double y0,
                                                       double cs, int32_t nx, float hb,
                                                       int2 *cnt) {
  const uint32_t lane = lane_id();
  const int32_t nw = (int32_t)(gridDim.x * (blockDim.x / GP_WAVE));
  for (int32_t k = (int32_t)(blockIdx.x * (blockDim.x / GP_WAVE) + threadIdx.x / GP_WAVE);
       k < npairs; k += nw) {
    const uint32_t cell = pair_cell[k];
    const double cx = x0 + ((double)(cell % (uint32_t)nx) + 0.5) * cs;
    const double cy = y0 + ((double)(cell / (uint32_t)nx) + 0.5) * cs;
    const int32_t f = cand_id[k], e1 = eoff[f + 1];
    int32_t nb = 0, ng = 0;
    for (int32_t base = eoff[f]; base < e1; base += GP_WAVE) {
      const int32_t e = base + (int32_t)lane;
      int cls = -1;
      if (e < e1) cls = pip_classify(edge64[e], k32[e], cx, cy, hb).cls;
      nb += __popcll(ballot(cls == PIP_BAND));
      ng += __popcll(ballot(cls == PIP_GUARDED));
    }
    if (lane == 0) cnt[k] = make_int2(nb, ng);
  }
}

__global__ __launch_bounds__(256) void k_pip_rec_emit(const uint32_t *pair_cell,
                                                      const int32_t *cand_id, int32_t npairs,
                                                      const int32_t *eoff, const double4 *edge64,
                                                      const float *k32, double x0, double y0,
                                                      double cs, int32_t nx, float hb,
                                                      const int64_t *off, const int2 *pc,
                                                      float4 *recs) {
  const uint32_t lane = lane_id();
  const uint64_t lt = lanemask_lt();
  const int32_t nw = (int32_t)(gridDim.x * (blockDim.x / GP_WAVE));
  for (int32_t k = (int32_t)(blockIdx.x * (blockDim.x / GP_WAVE) + threadIdx.x / GP_WAVE);
       k < npairs; k += nw) {
    const uint32_t cell = pair_cell[k];
    const double cx = x0 + ((double)(cell % (uint32_t)nx) + 0.5) * cs;
    const double cy = y0 + ((double)(cell / (uint32_t)nx) + 0.5) * cs;
    const int32_t f = cand_id[k], e1 = eoff[f + 1];
    const int64_t r0 = off[k], r1 = off[k + 1];
    const int32_t np = pc[k].x, nb = pc[k].y;
    const int64_t gs = r0 + ((np + nb + 1) & ~1);
    if (lane == 0 && ((np + nb) & 1)) recs[r0 + np + nb] = make_float4(0.f, 0.f, 0.f, 0.f);
    int32_t iP = 0, iB = 0, iG = 0;
    for (int32_t base = eoff[f]; base < e1; base += GP_WAVE) {
      const int32_t e = base + (int32_t)lane;
      PipEdge q;
      q.cls = -1;
      if (e < e1) q = pip_classify(edge64[e], k32[e], cx, cy, hb);
      const uint64_t mP = ballot(q.cls == PIP_PLAIN), mB = ballot(q.cls == PIP_BAND),
                     mG = ballot(q.cls == PIP_GUARDED);
      // the classes repeat the counting kernel's bit for bit; the bounds keep every
      // write inside the pair's slots regardless
      const int32_t jP = iP + __popcll(mP & lt), jB = iB + __popcll(mB & lt);
      if (q.cls == PIP_PLAIN && jP < np) recs[r0 + jP] = q.rec;
      if (q.cls == PIP_BAND && jB < nb) recs[r0 + np + jB] = q.rec;
      if (q.cls == PIP_GUARDED) {
        const int64_t g = gs + 2 * (int64_t)(iG + __popcll(mG & lt));
        if (g + 1 < r1) {
          recs[g] = q.rec;
          recs[g + 1] = make_float4(q.G, 0.f, 0.f, 0.f);
        }
      }
      iP += __popcll(mP);
      iB += __popcll(mB);
      iG += __popcll(mG);
    }
  }
}

hipError_t launch_pip_rec_count(const uint32_t *pair_cell, const int32_t *cand_id,
                                int32_t npairs, const int32_t *eoff, const double4 *edge64,
                                const float *k32, double x0, double y0, double cs, int32_t nx,
                                float hb, int2 *cnt, hipStream_t s) {
  if (npairs <= 0) return hipSuccess;
  const int64_t blocks = std::min<int64_t>(((int64_t)npairs + 3) / 4, 65536);
  hipLaunchKernelGGL(k_pip_rec_count, dim3((unsigned)blocks), dim3(256), 0, s, pair_cell,
                     cand_id, npairs, eoff, edge64, k32, x0, y0, cs, nx, hb, cnt);
  return hipGetLastError();
}

hipError_t launch_pip_rec_emit(const uint32_t *pair_cell, const int32_t *cand_id,
                               int32_t npairs, const int32_t *eoff, const double4 *edge64,
                               const float *k32, double x0, double y0, double cs, int32_t nx,
                               float hb, const int64_t *off, const int2 *pc, float4 *recs,
                               hipStream_t s) {
  if (npairs <= 0) return hipSuccess;
  const int64_t blocks = std::min<int64_t>(((int64_t)npairs + 3) / 4, 65536);
  hipLaunchKernelGGL(k_pip_rec_emit, dim3((unsigned)blocks), dim3(256), 0, s, pair_cell,
                     cand_id, npairs, eoff, edge64, k32, x0, y0, cs, nx, hb, off, pc, recs);
  return hipGetLastError();
}

// Band test of one edge record: the open straddle 0 < t < h of each lane's point (the
// crossing, as a lane mask).  A point level with an endpoint (t = 0 or t = h, closed but
// not open) is ambiguous: amb, per lane, keeps the minimum of t and t ^ h as bit
// patterns, which is zero once that has happened.  Kept in a VGPR, the ambiguity costs
// vector instructions only; the scalar unit, which bounds this kernel, sees one XOR.
__device__ __forceinline__ uint64_t band_cross(float py, const float4 e, uint32_t &amb) {
  const uint32_t tb = __float_as_uint(py - e.x);
  amb = min(amb, min(tb, tb ^ __float_as_uint(e.z)));
  return ballot(tb - 1u < __float_as_uint(e.y));
}

// Mixed PIP refinement of one item from the grid's records.  The cell's candidate
// polygons are visited in order, each polygon's records in chunks of PIP_PRE_CHUNK slots;
// the records of the next chunk (of this polygon or the next one still to be tested) are
// loaded into registers while the current chunk, already in LDS, is tested, so the
// item waits on one load round trip only at its start.  Each chunk's plain, band and
// guarded parts run their own loops.
#define PIP_PRE_CHUNK 128
template <int PPL>
__device__ void pipmix_pre_item(const RefineArgs &a, const Item it, float4 *lds) {
  if (it.npts <= a.vp_points) {
    pip_vp_item(a, it);
    return;
  }
  constexpr int CH = PIP_PRE_CHUNK, PF = CH / GP_WAVE;
  const uint32_t lane = lane_id();
  const double cx = cell_cx(a, (uint32_t)it.cell), cy = cell_cy(a, (uint32_t)it.cell);
  float px[PPL], py[PPL];
  int32_t best[PPL];
  bool rq[PPL];
  load_points32<PPL>(a, it, cx, cy, px, py);
#pragma unroll
  for (int j = 0; j < PPL; ++j) {
    best[j] = -1;
    rq[j] = false;
  }
  constexpr int U = PPL >= 4 ? 4 : 8;  // plain edges per step
  const int32_t k0 = a.cand_off[it.cell], k1 = a.cand_off[it.cell + 1];
  // the metadata of the cell's first 64 candidate pairs, one pair per lane, in one round
  // trip, kept in LDS after the chunk: polygon id, first record slot relative to the
  // cell's first, (plain, band) counts
  int4 *meta = (int4 *)(lds + CH);
  const int64_t rbase = a.prec_off[k0], rend = a.prec_off[k1];
  if ((int)lane < k1 - k0) {
    const int32_t k = k0 + (int32_t)lane;
    const int2 pc = a.pcnt[k];
    meta[lane] = make_int4(a.cand_id[k], (int32_t)(a.prec_off[k] - rbase), pc.x, pc.y);
  }
  __syncthreads();
  // candidate pair k: polygon, class, first slot, slots, plain and plain+band counts
  struct Cand {
    int32_t f, cls;
    int64_t r0;
    int32_t nsl, nP, nPB;
  };
  auto cand = [&](int32_t k) {
    Cand c;
    const int32_t q = k - k0;
    c.cls = a.cand_class ? a.cand_class[k] : 2;
    if (q < GP_WAVE) {
      const int4 m = meta[q];
      c.f = __builtin_amdgcn_readfirstlane(m.x);
      c.r0 = rbase + __builtin_amdgcn_readfirstlane(m.y);
      c.nP = __builtin_amdgcn_readfirstlane(m.z);
      c.nPB = c.nP + __builtin_amdgcn_readfirstlane(m.w);
    } else {
      c.f = a.cand_id[k];
      c.r0 = a.prec_off[k];
      const int2 pc = a.pcnt[k];
      c.nP = pc.x;
      c.nPB = pc.x + pc.y;
    }
    const int64_t r1 = k + 1 == k1 ? rend
                       : (q + 1 < GP_WAVE ? rbase + __builtin_amdgcn_readfirstlane(meta[q + 1].y)
                                          : a.prec_off[k + 1]);
    c.nsl = (int32_t)(r1 - c.r0);
    return c;
  };
  // the first candidate at or after k that is not wholly outside the cell (k1 if none)
  auto next_tested = [&](int32_t k, Cand &c) {
    for (; k < k1; ++k) {
      c = cand(k);
      if (c.cls != 0) break;
    }
    return k;
  };
  float4 pf[PF];
  auto prefetch = [&](int64_t r, int cnt) {
#pragma unroll
    for (int i = 0; i < PF; ++i) {
      const int t = (int)lane + GP_WAVE * i;
      pf[i] = t < cnt ? a.precs[r + t] : make_float4(0.f, 0.f, 0.f, 0.f);
    }
  };
  Cand cur;
  int32_t k = next_tested(k0, cur);
  int32_t s = 0;
  if (k < k1 && cur.cls == 2) prefetch(cur.r0, cur.nsl < CH ? cur.nsl : CH);
  uint64_t par[PPL], flg[PPL];
  uint32_t ambv[PPL];  // per lane: zero once the point is level with a band endpoint
#pragma unroll
  for (int j = 0; j < PPL; ++j) { par[j] = 0; flg[j] = 0; ambv[j] = ~0u; }
  while (k < k1) {
    if (cur.cls == 1) {  // inside: every undecided point takes f, and all are decided
#pragma unroll
      for (int j = 0; j < PPL; ++j)
        if (best[j] < 0 && !rq[j]) best[j] = cur.f;
      break;
    }
    const int cnt = (cur.nsl - s) < CH ? (cur.nsl - s) : CH;
    __syncthreads();
#pragma unroll
    for (int i = 0; i < PF; ++i) {
      const int t = (int)lane + GP_WAVE * i;
      if (t < cnt) lds[t] = pf[i];
    }
    __syncthreads();
    // the next chunk: the rest of this polygon, else the next polygon to test
    Cand nxt = cur;
    int32_t nk = k, ns = s + CH;
    if (ns >= cur.nsl) {
      nk = next_tested(k + 1, nxt);
      ns = 0;
    }
    if (nk < k1 && nxt.cls == 2)
      prefetch(nxt.r0 + ns, (nxt.nsl - ns) < CH ? (nxt.nsl - ns) : CH);
    const int32_t nP = cur.nP, nPB = cur.nPB, gs = (nPB + 1) & ~1;
    auto clampc = [&](int32_t v) { return v < 0 ? 0 : (v > cnt ? cnt : v); };
    // plain records [0, p1)
    const int p1 = clampc(nP - s);
    int t = 0;
    for (; t + U <= p1; t += U) {
      float4 e[U];
#pragma unroll
      for (int q = 0; q < U; ++q) e[q] = lds[t + q];
#pragma unroll
      for (int j = 0; j < PPL; ++j) {
        uint64_t m = 0;
#pragma unroll
        for (int q = 0; q < U; ++q) m ^= plain_cross(px[j], py[j], e[q]);
        par[j] ^= m;
      }
    }
    for (; t + 2 <= p1; t += 2) {
      const float4 e0 = lds[t], e1 = lds[t + 1];
#pragma unroll
      for (int j = 0; j < PPL; ++j)
        par[j] ^= plain_cross(px[j], py[j], e0) ^ plain_cross(px[j], py[j], e1);
    }
    if (t < p1) {
      const float4 e0 = lds[t];
#pragma unroll
      for (int j = 0; j < PPL; ++j) par[j] ^= plain_cross(px[j], py[j], e0);
    }
    // band records [p1, b1)
    const int b1 = clampc(nPB - s);
    for (t = p1; t + 4 <= b1; t += 4) {
      const float4 e0 = lds[t], e1 = lds[t + 1], e2 = lds[t + 2], e3 = lds[t + 3];
#pragma unroll
      for (int j = 0; j < PPL; ++j)
        par[j] ^= band_cross(py[j], e0, ambv[j]) ^ band_cross(py[j], e1, ambv[j]) ^
                  band_cross(py[j], e2, ambv[j]) ^ band_cross(py[j], e3, ambv[j]);
    }
    for (; t < b1; ++t) {
      const float4 e0 = lds[t];
#pragma unroll
      for (int j = 0; j < PPL; ++j) par[j] ^= band_cross(py[j], e0, ambv[j]);
    }
    // guarded records, two slots each, from the first even slot after the band ones
    for (t = clampc(gs - s); t + 2 <= cnt; t += 2) {
      const float4 e = lds[t];
      const float G = lds[t + 1].x;
#pragma unroll
      for (int j = 0; j < PPL; ++j) {
        const float ty = py[j] - e.y;
        const float d = fmaf(ty, e.w, e.x) - px[j];
        const uint64_t st = ballot(ty >= 0.0f) & ballot(py[j] < e.z);
        const uint64_t eq = ballot(ty == 0.0f) | ballot(py[j] == e.z);
        par[j] ^= st & ballot(d > 0.0f);
        flg[j] |= (eq & ballot(!(d < -G))) | (st & ballot(!(fabsf(d) > G)));
      }
    }
    if (nk != k) {  // the polygon is done
#pragma unroll
      for (int j = 0; j < PPL; ++j) {
        const bool odd = (par[j] >> lane) & 1ull;
        const bool fl = ((flg[j] >> lane) & 1ull) || ambv[j] == 0u;
        if (best[j] < 0 && !rq[j]) {
          if (fl) rq[j] = true;
          else if (odd) best[j] = cur.f;
        }
        par[j] = 0;
        flg[j] = 0;
        ambv[j] = ~0u;
      }
    }
    k = nk;
    s = ns;
    cur = nxt;
  }
#pragma unroll
  for (int j = 0; j < PPL; ++j) {
    const int idx = (int)lane + GP_WAVE * j;
    const bool v = idx < it.npts;
    if (v && !rq[j]) a.out_id[a.perm[it.pt_lo + idx]] = best[j];
    push_recheck(a, v && rq[j], (uint32_t)(it.pt_lo + idx));
  }
}

// ------------------------------------------------------------------------- P2P staging
// A chunk holds the segments of consecutive candidate polylines (a polyline longer
// than the chunk continues in the next one).  tab[q] = (fid, end slot | continues<<31).

struct alignas(16) SegRec64 {
  double ax, ay, bx, by, dx, dy, L2, L2p;
};

// ------------------------------------------------------------------------- P2P, vertex-parallel

__device__ __forceinline__ double wave_min_f64(double v) {
  for (int off = 32; off > 0; off >>= 1) v = fmin(v, __shfl_xor(v, off, GP_WAVE));
  return v;
}

__device__ __forceinline__ int32_t wave_min_i32(int32_t v) {
  for (int off = 32; off > 0; off >>= 1) v = min(v, __shfl_xor(v, off, GP_WAVE));
  return v;
}

// Vertex-parallel refinement of a P2P item with few points (the alternative mapping of
// Sec. III.B, with the cross-lane minimum): lanes take the segments of the cell's
// candidate polylines, four of the item's points at a time.  Each lane keeps, per point,
// the smallest distance it has seen within range and the polyline it came from (a lane
// meets the segments in ascending polyline order, so a later equal distance keeps the
// smaller id); the point's answer is the smallest (distance, id) pair over the lanes,
// which is the nearest polyline in range with ties to the smaller id.  FP64 in the
// definition's operation order; a perpendicular quotient is divided out only when it
// could still beat the lane's best, itself at most next(D*D) (cc >= fl(thr*L2)*(1+2^-49)
// implies cc/L2 > thr), so the results are the definition's in both precision forms.
// The segments of 64 candidates at a time are laid end to end and the lanes walk that
// list 64 segments per step (short polylines do not leave lanes idle); each lane finds
// its segment's polyline from the window's start offsets in LDS (win: this wave's 3 x 64
// words), and the only cross-lane steps are the window scan and the final minima.
__device__ void p2p_vp_item(const RefineArgs &a, const Item it, int32_t *win) {
  const uint32_t lane = lane_id();
  int32_t *wid = win, *wseg = win + GP_WAVE, *wstart = win + 2 * GP_WAVE;
  const int np = it.npts;  // 1 .. a.vp_points (<= 64)
  const int32_t k0 = a.cand_off[it.cell], k1 = a.cand_off[it.cell + 1];
  for (int g = 0; g < np; g += 4) {
    double px[4], py[4], best[4];
    int32_t bid[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const double2 p = a.xy[it.pt_lo + min(g + j, np - 1)];
      px[j] = p.x;
      py[j] = p.y;
      best[j] = a.D2_next;  // accept d2 <= fl(D*D); later only strictly smaller
      bid[j] = -1;
    }
    for (int32_t kw = k0; kw < k1; kw += GP_WAVE) {
      const int32_t kk = kw + (int32_t)lane;
      const int nk = min(GP_WAVE, k1 - kw);
      int32_t wf = 0, w0 = 0, len = 0;
      if (kk < k1) {
        wf = a.cand_id[kk];
        w0 = a.eoff[wf];
        len = a.eoff[wf + 1] - w0;
      }
      const uint32_t incl = wave_incl_scan((uint32_t)len);
      const int32_t total = (int32_t)__builtin_amdgcn_readlane(incl, GP_WAVE - 1);
      wave_lds_sync();  // the previous window's reads are done
      wid[lane] = wf;
      wseg[lane] = w0;
      wstart[lane] = (int32_t)incl - len;
      wave_lds_sync();
      int c = 0;  // this lane's candidate in the window (its flat indices only grow)
      for (int32_t F = (int32_t)lane; F < total; F += GP_WAVE) {
        while (c + 1 < nk && wstart[c + 1] <= F) ++c;
        const int32_t f = wid[c];
        const double4 r = a.edge64[wseg[c] + (F - wstart[c])];
        const double dx = r.z - r.x, dy = r.w - r.y;
        const double L2 = dx * dx + dy * dy;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const double wx = px[j] - r.x, wy = py[j] - r.y;
          const double t = wx * dx + wy * dy;
          double d2;
          if (t <= 0.0) {
            d2 = wx * wx + wy * wy;
          } else if (t >= L2) {
            const double ex = px[j] - r.z, ey = py[j] - r.w;
            d2 = ex * ex + ey * ey;
          } else {
            const double cr = wx * dy - wy * dx;
            const double cc = cr * cr;
            d2 = cc < (best[j] * L2) * (1.0 + 0x1p-49) ? cc / L2 : INFINITY;
          }
          if (d2 < best[j]) {
            best[j] = d2;
            bid[j] = f;
          }
        }
      }
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const double m = wave_min_f64(best[j]);
      const int32_t b = wave_min_i32(best[j] == m && bid[j] >= 0 ? bid[j] : INT32_MAX);
      if (lane == 0 && g + j < np) {
        const uint32_t o = a.perm[it.pt_lo + g + j];
        a.out_id[o] = b == INT32_MAX ? -1 : b;
        a.out_dist[o] = b == INT32_MAX ? INFINITY : sqrt(m);
      }
    }
  }
}

// ------------------------------------------------------------------------- P2P, FP64
// P2P work items may span W wavefronts (W*64*PPL points) that share one LDS staging of
// the segments; every wave owns its own points and results.

template <int PPL, int W>
__device__ __forceinline__ void load_points64w(const RefineArgs &a, const Item it,
                                               double (&px)[PPL], double (&py)[PPL]) {
  const int base = (int)(threadIdx.x / GP_WAVE) * GP_WAVE * PPL + (int)lane_id();
#pragma unroll
  for (int j = 0; j < PPL; ++j) {
    const int idx = base + GP_WAVE * j;
    const double2 p = idx < it.npts ? a.xy[it.pt_lo + idx] : make_double2(0.0, 0.0);
    px[j] = p.x;
    py[j] = p.y;
  }
}

template <int PPL, int W>
__device__ void p2p64_item(const RefineArgs &a, const Item it, SegRec64 *lds, int2 *tab) {
  if (W == 1 && it.npts <= a.vp_points) return;  // refined by k_p2p_vp
  const int tid = (int)threadIdx.x;
  const int wbase = (int)(threadIdx.x / GP_WAVE) * GP_WAVE * PPL;
  const bool wave_live = wbase < it.npts;
  const int EC = a.edge_chunk;
  double px[PPL], py[PPL], best[PPL];
  int32_t bid[PPL];
  load_points64w<PPL, W>(a, it, px, py);
#pragma unroll
  for (int j = 0; j < PPL; ++j) {
    best[j] = a.D2_next;  // accept d2 <= fl(D*D); later only strictly smaller
    bid[j] = -1;
  }
  int32_t k = a.cand_off[it.cell];
  const int32_t k1 = a.cand_off[it.cell + 1];
  int32_t soff = 0;
  while (k < k1) {
    __syncthreads();
    int filled = 0, ntab = 0;
    while (k < k1 && filled < EC) {
      const int32_t f = a.cand_id[k];
      const int32_t s0 = a.eoff[f] + soff, s1 = a.eoff[f + 1];
      const int take = (s1 - s0) < (EC - filled) ? (s1 - s0) : (EC - filled);
      for (int t = tid; t < take; t += GP_WAVE * W) {
        const double4 r = a.edge64[s0 + t];
        SegRec64 q;
        q.ax = r.x; q.ay = r.y; q.bx = r.z; q.by = r.w;
        q.dx = r.z - r.x;
        q.dy = r.w - r.y;
        q.L2 = q.dx * q.dx + q.dy * q.dy;
        // fl(L2 (1 + 2^-48)): best * L2p >= best * L2 (1 + 2^-49) after rounding, the
        // bound that decides whether a perpendicular quotient can still win
        q.L2p = q.L2 * (1.0 + 0x1p-48);
        lds[filled + t] = q;
      }
      filled += take;
      const bool cont = s0 + take < s1;
      if (tid == 0) tab[ntab] = make_int2(f, filled | (cont ? (int)0x80000000 : 0));
      ++ntab;
      if (cont) soff += take;
      else { ++k; soff = 0; }
    }
    __syncthreads();
    if (!wave_live) continue;
    int start = 0;
    for (int q = 0; q < ntab; ++q) {
      const int2 te = tab[q];
      const int32_t f = te.x;
      const int end = te.y & 0x7fffffff;
      // The slots of one table entry are consecutive segments of polyline f, so the b
      // endpoint of slot t is the a endpoint of slot t + 1: its difference to the point
      // and squared distance are computed once and carried (bitwise the same values the
      // definition computes for both segments).
      double wx[PPL], wy[PPL], da[PPL];
      if (start < end) {
        const double ax = lds[start].ax, ay = lds[start].ay;
#pragma unroll
        for (int j = 0; j < PPL; ++j) {
          wx[j] = px[j] - ax;
          wy[j] = py[j] - ay;
          da[j] = wx[j] * wx[j] + wy[j] * wy[j];
        }
      }
      for (int t = start; t < end; ++t) {
        const SegRec64 r = lds[t];
#pragma unroll
        for (int j = 0; j < PPL; ++j) {
          const double tt = wx[j] * r.dx + wy[j] * r.dy;
          const double ex = px[j] - r.bx, ey = py[j] - r.by;
          const double db = ex * ex + ey * ey;
          const double c = wx[j] * r.dy - wy[j] * r.dx;
          const double cc = c * c;
          const bool ca = tt <= 0.0;
          const bool cb = !ca & (tt >= r.L2);
          double d2 = ca ? da[j] : db;
          const bool cp = !ca & !cb;
          // The perpendicular case divides only when its quotient could still beat the
          // current best: cc >= fl(best * L2p) >= fl(best*L2)*(1+2^-49) implies
          // cc/L2 > best.
          d2 = cp ? INFINITY : d2;
          if (cp && cc < best[j] * r.L2p) d2 = cc / r.L2;
          if (d2 < best[j]) { best[j] = d2; bid[j] = f; }
          wx[j] = ex;
          wy[j] = ey;
          da[j] = db;
        }
      }
      start = end;
    }
  }
#pragma unroll
  for (int j = 0; j < PPL; ++j) {
    const int idx = wbase + (int)lane_id() + GP_WAVE * j;
    if (idx < it.npts) {
      const uint32_t o = a.perm[it.pt_lo + idx];
      a.out_id[o] = bid[j];
      a.out_dist[o] = bid[j] >= 0 ? sqrt(best[j]) : INFINITY;
    }
  }
}

// ------------------------------------------------------------------------- P2P, mixed
// FP32 on cell-rebased coordinates, in each segment's own frame.  With u = d/|d|,
// v = (-u.y, u.x), m the segment midpoint and h = |d|/2, the point-segment distance is
// sqrt(e^2 + r^2) with s = (p - m).u, r = (p - m).v and e = max(0, |s| - h).  The LDS
// holds u, v, -m.u, -m.v and h, all multiplied by a per-grid power of two `scale` that
// keeps |s| * scale below 1/2; then s and r are two FMAs each, e is one subtract with
// the |.| and clamp-to-[0,1] modifiers (the upper clamp never binds), and e^2 + r^2 is
// two more -- 7 VALU operations per test, plus half a v_min3_u32 (minimum on the float
// bits as unsigned integers, valid for d^2 >= 0).  Scaling by a power of two is exact.
// The frame (u, h, and the absolute -m.u, -m.v) is precomputed per segment when the
// grid is built; staging for a cell c only adds c.u and c.v in FP64.
//
// Per point the wave tracks the three best polylines (distinct ids; ids of the first
// two).  E is the largest error bound e_s = 48*2^-24*(B*sqrt2 + |m - c| + |d|) over the
// segments near the cell (48 is four times the constant of the rounding analysis).
//  * best > D + E: nothing within D (FP64 agrees);
//  * second > best + 2E: only the best polyline can be the answer; its exact FP64
//    distance decides (within D or not);
//  * third > best + 2E: only the best two can be the answer; their exact FP64
//    distances decide (smaller distance, then smaller id);
//  * otherwise (a three-way near-tie): the point goes to the FP64 recheck queue.
// Reported distances are therefore always FP64 values.

// U = (u.x, u.y, -(m-c).u, h) * scale and R = -(m-c).v * scale; v = (-u.y, u.x) comes
// from U through the FMA's negate modifier, so a segment costs 20 bytes of LDS.
__device__ __forceinline__ uint32_t seg_d2_bits(float px, float py, const float4 U,
                                                const float R) {
  const float s = fmaf(px, U.x, fmaf(py, U.y, U.z));
  const float r = fmaf(px, -U.y, fmaf(py, U.x, R));
  const float e = __builtin_amdgcn_fmed3f(fabsf(s) - U.w, 0.0f, 1.0f);
  return __float_as_uint(fmaf(e, e, r * r));
}

// LDS of the exact-distance pass per wave: for up to two pairs per lane the result,
// descriptor and threshold, the lanes' points, and a queue of 128 (pair, block) entries.
#define P2P_EPI_BYTES (2 * GP_WAVE * (8 + 16 + 8 + 8) + GP_WAVE * 16)

// One segment's record for a cell with centre c: its frame constants relative to c
// (s_c = -(m - c).u, r_c = -(m - c).v, scaled), its error bound e_s in distance units,
// and whether it counts as near the cell.  e_s carries a factor 4 over the rounding
// analysis, which also covers the few ulps of the hardware square root here; "near"
// compares squares against a limit widened by 2^-16.  Used by the refinement's own
// staging and by the build-time staging, which must agree bit for bit.
struct SegStage {
  float4 U;
  float V;
  float es;
  bool nearc;
};
__device__ __forceinline__ SegStage stage_segment(const double4 F, const float4 G, double cx,
                                                  double cy, double sc, float hb, float T,
                                                  float near_lim2) {
  SegStage r;
  const double sC = F.z + (cx * F.x + cy * F.y);
  const double rC = F.w + (cy * F.x - cx * F.y);
  r.U = make_float4(G.x, G.y, (float)(sC * sc), G.z);
  r.V = (float)(rC * sc);
  const float fs = fabsf((float)sC), fr = fabsf((float)rC);
  r.es = 48.0f * 0x1p-24f * (hb * 1.4143f + __builtin_amdgcn_sqrtf(fs * fs + fr * fr) + G.w);
  const float ex = fmaxf(0.0f, fs - 0.5f * G.w);
  r.nearc = !(ex * ex + fr * fr > near_lim2) || !(r.es <= 0.5f * T);
  return r;
}

__device__ __forceinline__ float p2p_near_lim2(double D, float T, float hb) {
  const float near_lim = (float)D + T + hb * 1.4143f;
  return near_lim * near_lim * (1.0f + 0x1p-16f);
}

// Build-time staging: the records of every candidate segment of every cell, in the
// order the refinement consumes them (candidates by id, each polyline's segments in
// order), with the cell's E over its near segments and over all of them.  One
// workgroup per cell.
__global__ __launch_bounds__(256) void k_prestage(const int32_t *cand_off, const int32_t *cand_id,
                                                  const int32_t *eoff, const double4 *frame64,
                                                  const float4 *frame32, double x0, double y0,
                                                  double cs, int32_t nx, int32_t ncells,
                                                  double D, float hb, float T, float sc,
                                                  const int64_t *rec_off, float4 *recU,
                                                  float *recV, float2 *cellE) {
  __shared__ float red[2][256 / GP_WAVE];
  const float near_lim2 = p2p_near_lim2(D, T, hb);
  for (int32_t c = blockIdx.x; c < ncells; c += gridDim.x) {
    const double cx = x0 + ((double)(c % nx) + 0.5) * cs;
    const double cy = y0 + ((double)(c / nx) + 0.5) * cs;
    int64_t pos = rec_off[c];
    float emax = 0.0f, eall = 0.0f;
    for (int32_t k = cand_off[c]; k < cand_off[c + 1]; ++k) {
      const int32_t f = cand_id[k];
      const int32_t s0 = eoff[f], s1 = eoff[f + 1];
      for (int32_t t = (int32_t)threadIdx.x; t < s1 - s0; t += blockDim.x) {
        const SegStage r = stage_segment(frame64[s0 + t], frame32[s0 + t], cx, cy, (double)sc,
                                         hb, T, near_lim2);
        recU[pos + t] = r.U;
        recV[pos + t] = r.V;
        if (r.nearc) emax = fmaxf(emax, r.es);
        eall = fmaxf(eall, r.es);
      }
      pos += s1 - s0;
    }
    for (int off = 32; off > 0; off >>= 1) {
      emax = fmaxf(emax, __shfl_xor(emax, off, GP_WAVE));
      eall = fmaxf(eall, __shfl_xor(eall, off, GP_WAVE));
    }
    if (lane_id() == 0) {
      red[0][threadIdx.x / GP_WAVE] = emax;
      red[1][threadIdx.x / GP_WAVE] = eall;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      for (int w = 1; w < (int)(blockDim.x / GP_WAVE); ++w) {
        emax = fmaxf(emax, red[0][w]);
        eall = fmaxf(eall, red[1][w]);
      }
      cellE[c] = make_float2(emax, eall);
    }
    __syncthreads();
  }
}

hipError_t launch_prestage(const int32_t *cand_off, const int32_t *cand_id, const int32_t *eoff,
                           const double4 *frame64, const float4 *frame32, double x0, double y0,
                           double cs, int32_t nx, int32_t ncells, double D, float hb, float T,
                           float sc, const int64_t *rec_off, float4 *recU, float *recV,
                           float2 *cellE, hipStream_t s) {
  if (ncells <= 0) return hipSuccess;
  const unsigned g = (unsigned)std::min<int64_t>(ncells, 65536);
  hipLaunchKernelGGL(k_prestage, dim3(g), dim3(256), 0, s, cand_off, cand_id, eoff, frame64,
                     frame32, x0, y0, cs, nx, ncells, D, hb, T, sc, rec_off, recU, recV, cellE);
  return hipGetLastError();
}

// PRE: the grid carries build-time segment records (and no segment lists); the kernel
// then holds no FP64 staging code, which keeps it within 96 VGPRs (5 waves per SIMD).
template <int PPL, int W, bool PRE>
__device__ void p2pmix_item(const RefineArgs &a, const Item it, float4 *ldsU, float *ldsV,
                            int2 *tab, int *slotseg, int *slotf, float *red, unsigned char *epi) {
  const int tid = (int)threadIdx.x;
  const uint32_t lane = lane_id();
  const int wave = (int)(threadIdx.x / GP_WAVE);
  const int wbase = wave * GP_WAVE * PPL;
  const bool wave_live = wbase < it.npts;
  const int EC = a.edge_chunk;
  const double cx = cell_cx(a, (uint32_t)it.cell), cy = cell_cy(a, (uint32_t)it.cell);
  const float hb = a.half_box;
  const float T = a.p2p_margin;
  const float near_lim2 = p2p_near_lim2(a.D, T, hb);
  const double sc = (double)a.p2p_scale;
  const double inv_sc = 1.0 / sc;
  float px[PPL], py[PPL];
  uint32_t b1[PPL], b2[PPL], b3[PPL], pm[PPL];
  int32_t f1[PPL], f2[PPL];
#pragma unroll
  for (int j = 0; j < PPL; ++j) {
    const int idx = wbase + (int)lane + GP_WAVE * j;
    const double2 p = idx < it.npts ? a.xy[it.pt_lo + idx] : make_double2(cx, cy);
    px[j] = (float)(p.x - cx);
    py[j] = (float)(p.y - cy);
  }
  const uint32_t INFB = 0x7f800000u;
#pragma unroll
  for (int j = 0; j < PPL; ++j) {
    b1[j] = INFB;
    b2[j] = INFB;
    b3[j] = INFB;
    pm[j] = INFB;
    f1[j] = -1;
    f2[j] = -1;
  }
  float emax = 0.0f;  // per-thread partial of E over the segments this thread staged
  float eall = 0.0f;  // the same over every staged segment, near the cell or not
  // Stage one segment into chunk slot t: its frame constants relative to the cell centre
  // c (s_c = -(m - c).u, r_c = -(m - c).v, scaled), and its share of the error bound E.
  auto stage = [&](int t, const double4 F, const float4 G) {
    const SegStage r = stage_segment(F, G, cx, cy, sc, hb, T, near_lim2);
    ldsU[2 * t] = r.U;
    ldsV[8 * t] = r.V;
    if (r.nearc) emax = fmaxf(emax, r.es);
    eall = fmaxf(eall, r.es);
  };
  // With build-time staging the cell's records are read as they are, in order.
  constexpr bool prestaged = PRE;
  int64_t rpos = prestaged ? a.rec_off[it.cell] : 0;
  // With a segment filter the cell's chunks are slices of its list of reaching segments;
  // otherwise they are cut from its candidate polylines' whole segment ranges.
  const bool seglist = !PRE && a.cseg_off != nullptr;
  int32_t k = seglist ? a.cseg_off[it.cell] : a.cand_off[it.cell];
  const int32_t k1 = seglist ? a.cseg_off[it.cell + 1] : a.cand_off[it.cell + 1];
  int32_t soff = 0;
  // Candidate window: lane i of each wave holds candidate kw + i (id, first and end
  // segment), fetched in one round trip, so planning a chunk issues no dependent loads.
  int32_t kw = k1, wf = 0, we0 = 0, we1 = 0;
  while (k < k1) {
    __syncthreads();
    int filled = 0, ntab = 0;
    if (seglist) {
      // the slot map is the list slice; a polyline's entries are consecutive (segments
      // are stored polyline by polyline), so it ends where the next entry's polyline
      // differs, or continues into the next chunk
      filled = (k1 - k) < EC ? (k1 - k) : EC;
      for (int t = tid; t < filled; t += GP_WAVE * W) {
        const int32_t sg = a.cseg[k + t];
        slotseg[t] = sg;
        slotf[t] = a.seg2f[sg];
      }
      const int32_t fnext = k + filled < k1 ? a.seg2f[a.cseg[k + filled]] : -1;
      __syncthreads();
      for (int base = 0; base < filled; base += GP_WAVE) {
        const int t = base + (int)lane;
        int32_t ft = -1;
        bool mark = false, cont = false;
        if (t < filled) {
          ft = slotf[t];
          const int32_t fn = t + 1 < filled ? slotf[t + 1] : fnext;
          mark = fn != ft || t == filled - 1;
          cont = t == filled - 1 && fn == ft;
        }
        const uint64_t m = ballot(mark);
        if (mark && wave == 0)
          tab[ntab + (int)__popcll(m & lanemask_lt())] =
              make_int2(ft, (t + 1) | (cont ? (int)0x80000000 : 0));
        ntab += (int)__popcll(m);
      }
      k += filled;
    }
    while (!seglist && k < k1 && filled < EC) {
      if (k >= kw + GP_WAVE || kw == k1) {
        kw = k;
        const int32_t kk = kw + (int)lane;
        wf = kk < k1 ? a.cand_id[kk] : 0;
        we0 = a.eoff[wf];
        we1 = a.eoff[wf + 1];
      }
      const int q = k - kw;
      const int32_t s0 = __builtin_amdgcn_readlane(we0, q) + soff;
      const int32_t s1 = __builtin_amdgcn_readlane(we1, q);
      const int take = (s1 - s0) < (EC - filled) ? (s1 - s0) : (EC - filled);
      if (!prestaged)
        for (int t = tid; t < take; t += GP_WAVE * W) slotseg[filled + t] = s0 + t;
      filled += take;
      const bool cont = s0 + take < s1;
      // the table names the candidate by its index k (ids ascend with k within a cell)
      if (tid == 0) tab[ntab] = make_int2(k, filled | (cont ? (int)0x80000000 : 0));
      ++ntab;
      if (cont) soff += take;
      else { ++k; soff = 0; }
    }
    __syncthreads();
    if (prestaged) {
      for (int t = tid; t < filled; t += GP_WAVE * W) {
        ldsU[2 * t] = a.recU[rpos + t];
        ldsV[8 * t] = a.recV[rpos + t];
      }
      rpos += filled;
    }
    // fill the chunk: two slots per thread per step, all four loads issued together
    if constexpr (!PRE) {
      for (int t = tid; t < filled; t += 2 * GP_WAVE * W) {
        const int t2 = t + GP_WAVE * W;
        const bool two = t2 < filled;
        const int sa = slotseg[t], sb = slotseg[two ? t2 : t];
        const double4 Fa = a.frame64[sa], Fb = a.frame64[sb];
        const float4 Ga = a.frame32[sa], Gb = a.frame32[sb];
        stage(t, Fa, Ga);
        if (two) stage(t2, Fb, Gb);
      }
    }
    __syncthreads();
    if (!wave_live) continue;
    int start = 0;
    for (int q = 0; q < ntab; ++q) {
      const int2 te = tab[q];
      const int32_t f = te.x;
      const int end = te.y & 0x7fffffff;
      int t = start;
      for (; t + 2 <= end; t += 2) {
        // two slots per step: four LDS reads off one address (32-byte slots)
        const float4 u0 = ldsU[2 * t], u1 = ldsU[2 * t + 2];
        const float v0 = ldsV[8 * t], v1 = ldsV[8 * t + 8];
#pragma unroll
        for (int j = 0; j < PPL; ++j)
          pm[j] = min(pm[j], min(seg_d2_bits(px[j], py[j], u0, v0),
                                 seg_d2_bits(px[j], py[j], u1, v1)));
      }
      if (t < end) {
        const float4 u0 = ldsU[2 * t];
        const float v0 = ldsV[8 * t];
#pragma unroll
        for (int j = 0; j < PPL; ++j) pm[j] = min(pm[j], seg_d2_bits(px[j], py[j], u0, v0));
      }
      if (!(te.y & (int)0x80000000)) {
        // merge the polyline into the running top three; skipped when it cannot enter
        // any lane's top three (the common case once the near polylines are seen)
        bool any = false;
#pragma unroll
        for (int j = 0; j < PPL; ++j) any |= pm[j] < b3[j];
        if (ballot(any)) {
#pragma unroll
          for (int j = 0; j < PPL; ++j) {
            if (pm[j] < b1[j]) {
              b3[j] = b2[j]; b2[j] = b1[j]; f2[j] = f1[j]; b1[j] = pm[j]; f1[j] = f;
            } else if (pm[j] < b2[j]) {
              b3[j] = b2[j]; b2[j] = pm[j]; f2[j] = f;
            } else if (pm[j] < b3[j]) {
              b3[j] = pm[j];
            }
          }
        }
#pragma unroll
        for (int j = 0; j < PPL; ++j) pm[j] = INFB;
      }
      start = end;
    }
  }
  if constexpr (PRE) {  // the cell's bounds, from the build-time staging
    const float2 ce = a.cellE[it.cell];
    emax = ce.x;
    eall = ce.y;
    // the exact pass reuses the chunk's LDS: every wave of the item must be done with it
    if (W > 1) __syncthreads();
  } else {
    // E = maximum over the whole workgroup's staged segments
    for (int off = 32; off > 0; off >>= 1) {
      emax = fmaxf(emax, __shfl_xor(emax, off, GP_WAVE));
      eall = fmaxf(eall, __shfl_xor(eall, off, GP_WAVE));
    }
    if (W > 1) {
      if (lane == 0) {
        red[wave] = emax;
        red[4 + wave] = eall;
      }
      __syncthreads();
      for (int w = 0; w < W; ++w) {
        emax = fmaxf(emax, red[w]);
        eall = fmaxf(eall, red[4 + w]);
      }
      __syncthreads();
    }
  }
  if (!wave_live) return;
  const double E = (double)emax;
  const double D = a.D;
  // Exact FP64 distances of each point's one or two candidate polylines.  With d_c the
  // FP32-derived distance of candidate c, the exact minimum over its segments is at most
  // d_c + E', E' the largest error bound of any staged segment (its FP32-best segment
  // is one of them).  A block of P2P_BLOCK segments whose bounding circle lies farther
  // than d_c + E' cannot hold the minimum.  The wave tests the blocks of all its
  // (point, polyline) pairs together, queues the blocks that pass in LDS, and evaluates
  // them 64 at a time, one per lane; each block's minimum joins its pair's result by an
  // LDS atomic minimum.  Non-negative doubles order like their bit patterns, so the
  // result is the exact minimum over the polyline's segments whatever the order.
  const double Ep = (double)eall;
  // f1/f2 hold candidate indices, or polyline ids when the chunks come from segment lists
  const bool byk = !seglist;
  // results are stored after all point slots: on this GPU a store holds back every later
  // load's wait (one counter covers both), so stores between slots would stall the
  // next slot's loads on their scattered writes
  int32_t rid[PPL];
  double rdd[PPL];
  bool rw[PPL];
#pragma unroll
  for (int j = 0; j < PPL; ++j) { rid[j] = -1; rdd[j] = INFINITY; rw[j] = false; }
  wave_lds_sync();  // with one wave per item the chunk's LDS is reused without a barrier
  unsigned char *wepi = epi + wave * P2P_EPI_BYTES;
  uint64_t *res = (uint64_t *)wepi;                  // [2*64] result bits per pair
  int4 *pinfo = (int4 *)(res + 2 * GP_WAVE);         // [2*64] {first seg, end seg, first unit, lane}
  double *pthr = (double *)(pinfo + 2 * GP_WAVE);    // [2*64] d_c + E'
  double2 *pts = (double2 *)(pthr + 2 * GP_WAVE);    // [64] the lanes' points
  int2 *uq = (int2 *)(pts + GP_WAVE);                // [2*64] queued (pair, block)
  auto unit_pair = [&](int u, int npairs) {  // the last pair whose first unit is <= u
    int lo = 0, hi = npairs - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (pinfo[mid].z <= u) lo = mid;
      else hi = mid - 1;
    }
    return lo;
  };
  auto eval_block = [&](int2 qb) {
    const int4 P = pinfo[qb.x];
    const double2 p = pts[P.w];
    const int32_t e0 = max(P.x, qb.y * P2P_BLOCK), e1 = min(P.y, (qb.y + 1) * P2P_BLOCK);
    double pd = INFINITY;
    for (int32_t e = e0; e < e1; ++e) {
      const double4 r = a.edge64[e];
      pd = fmin(pd, seg_d2_64(p.x, p.y, r.x, r.y, r.z, r.w));
    }
    atomicMin((unsigned long long *)&res[qb.x], (unsigned long long)__double_as_longlong(pd));
  };
#pragma unroll
  for (int j = 0; j < PPL; ++j) {
    const int idx = wbase + (int)lane + GP_WAVE * j;
    const bool v = idx < it.npts;
    const double d1 = (double)sqrtf(__uint_as_float(b1[j])) * inv_sc;
    const double d2 = (double)sqrtf(__uint_as_float(b2[j])) * inv_sc;
    const double d3 = (double)sqrtf(__uint_as_float(b3[j])) * inv_sc;
    const bool miss = d1 > D + E;
    // candidates for the answer: f1 alone, or f1 and f2 (every other polyline is
    // provably farther than both); their exact FP64 distances decide
    const int ncand = miss ? 0 : (d2 - d1 > 2.0 * E) ? 1 : (d3 - d1 > 2.0 * E) ? 2 : 3;
    const int nc = (v && (ncand == 1 || ncand == 2)) ? ncand : 0;
    int32_t s00 = 0, s01 = 0, s10 = 0, s11 = 0;
    // with candidate indices (no segment lists) only the candidate's near-segment range
    // of this cell can hold a minimum within D; with segment lists, the whole polyline
    if (byk) {
      if (nc >= 1) { const int2 r = a.near[f1[j]]; s00 = r.x; s01 = r.y; }
      if (nc >= 2) { const int2 r = a.near[f2[j]]; s10 = r.x; s11 = r.y; }
    } else {
      if (nc >= 1) { s00 = a.eoff[f1[j]]; s01 = a.eoff[f1[j] + 1]; }
      if (nc >= 2) { s10 = a.eoff[f2[j]]; s11 = a.eoff[f2[j] + 1]; }
    }
    // blocks overlapped by a pair's segments (every polyline has at least one segment)
    const int u0 = nc >= 1 ? (s01 - 1) / P2P_BLOCK - s00 / P2P_BLOCK + 1 : 0;
    const int u1 = nc >= 2 ? (s11 - 1) / P2P_BLOCK - s10 / P2P_BLOCK + 1 : 0;
    const uint32_t pinc = wave_incl_scan((uint32_t)nc);
    const uint32_t uinc = wave_incl_scan((uint32_t)(u0 + u1));
    const int npairs = (int)__builtin_amdgcn_readlane(pinc, GP_WAVE - 1);
    const int nunits = (int)__builtin_amdgcn_readlane(uinc, GP_WAVE - 1);
    const int pid = (int)pinc - nc, uoff = (int)uinc - (u0 + u1);
    if (npairs > 0) {
      if (nc >= 1) {
        res[pid] = 0x7ff0000000000000ull;  // +inf
        pinfo[pid] = make_int4(s00, s01, uoff, (int)lane);
        pthr[pid] = d1 + Ep;
        pts[lane] = a.xy[it.pt_lo + idx];
      }
      if (nc >= 2) {
        res[pid + 1] = 0x7ff0000000000000ull;
        pinfo[pid + 1] = make_int4(s10, s11, uoff + u0, (int)lane);
        pthr[pid + 1] = d2 + Ep;
      }
      wave_lds_sync();
      int qn = 0;  // queued blocks (uniform)
      for (int ub = 0; ub < nunits; ub += GP_WAVE) {
        const int u = ub + (int)lane;
        bool pass = false;
        int2 qb = make_int2(0, 0);
        if (u < nunits) {
          const int q = unit_pair(u, npairs);
          const int4 P = pinfo[q];
          const int blk = P.x / P2P_BLOCK + (u - P.z);
          const double2 p = pts[P.w];
          const double4 C = a.circ[blk];
          const double dx = p.x - C.x, dy = p.y - C.y;
          const double R = (C.z + pthr[q]) * (1.0 + 0x1p-40);
          pass = !(dx * dx + dy * dy > R * R);
          qb = make_int2(q, blk);
        }
        const uint64_t m = ballot(pass);
        if (pass) uq[qn + (int)__popcll(m & lanemask_lt())] = qb;
        qn += (int)__popcll(m);
        wave_lds_sync();
        if (qn >= GP_WAVE) {
          eval_block(uq[lane]);
          const int rest = qn - GP_WAVE;
          const int2 tail = (int)lane < rest ? uq[GP_WAVE + lane] : make_int2(0, 0);
          wave_lds_sync();
          if ((int)lane < rest) uq[lane] = tail;
          qn = rest;
          wave_lds_sync();
        }
      }
      if ((int)lane < qn) eval_block(uq[lane]);
      wave_lds_sync();
    }
    if (nc) {
      int32_t bid = -1;
      double best = INFINITY;
      for (int c = 0; c < nc; ++c) {
        const int32_t fk = c == 0 ? f1[j] : f2[j];
        const int32_t f = byk ? a.cand_id[fk] : fk;
        const double pd = __longlong_as_double((long long)res[pid + c]);
        if (pd <= a.D2 && (pd < best || (pd == best && f < bid))) { best = pd; bid = f; }
      }
      rid[j] = bid;
      rdd[j] = bid >= 0 ? sqrt(best) : INFINITY;
      rw[j] = true;
    } else if (v && miss) {
      rid[j] = -1;
      rdd[j] = INFINITY;
      rw[j] = true;
    }
    push_recheck(a, v && ncand == 3, (uint32_t)(it.pt_lo + idx));
    wave_lds_sync();  // the next point slot reuses the pass's LDS
  }
#pragma unroll
  for (int j = 0; j < PPL; ++j) {
    if (rw[j]) {
      const uint32_t o = a.perm[wbase + (int)lane + GP_WAVE * j + it.pt_lo];
      a.out_id[o] = rid[j];
      a.out_dist[o] = rdd[j];
    }
  }
}

// ------------------------------------------------------------------------- refine kernels

template <int PPL>
__global__ __launch_bounds__(64) void k_pip64(RefineArgs a, int persistent) {
  extern __shared__ __align__(16) unsigned char smem[];
  PipRec64 *lds = (PipRec64 *)smem;
  const uint32_t n_items = *a.n_items;
  uint32_t dead = 0;  // queues this workgroup has found exhausted
  uint32_t it = persistent ? next_item(a, n_items, dead) : blockIdx.x;
  while (it < n_items) {
    pip64_item<PPL>(a, a.items[it], lds);
    if (!persistent) break;
    it = next_item(a, n_items, dead);
  }
}

template <int PPL>
__global__ __launch_bounds__(64) void k_pipmix(RefineArgs a, int persistent) {
  extern __shared__ __align__(16) unsigned char smem[];
  float4 *A = (float4 *)smem;
  float4 *B = A + a.edge_chunk;
  float *G = (float *)(B + a.edge_chunk);
  const uint32_t n_items = *a.n_items;
  uint32_t dead = 0;  // queues this workgroup has found exhausted
  uint32_t it = persistent ? next_item(a, n_items, dead) : blockIdx.x;
  while (it < n_items) {
    // A cell's last item holds the remainder of its points: it runs with the fewest
    // points per lane that hold them, so its idle point slots cost no tests.
    const Item item = a.items[it];
    if (PPL >= 4 && item.npts > 64 && item.npts <= 128) pipmix_item<2>(a, item, A, B, G);
    else if (PPL >= 2 && item.npts <= 64) pipmix_item<1>(a, item, A, B, G);
    else pipmix_item<PPL>(a, item, A, B, G);
    if (!persistent) break;
    it = next_item(a, n_items, dead);
  }
}

// Item of a non-persistent launch with XCD locality: workgroup b runs on XCD b mod 8
// (the hardware places workgroups round-robin), and blocks of GP_XBLOCK consecutive items
// go round-robin to the XCDs, so the items of one cell share an L2.  A bijection of
// [0, G) for grids G that are multiples of GP_XCDS * GP_XBLOCK.
__device__ __forceinline__ uint32_t xcd_item(uint32_t b) {
  const uint32_t x = b % GP_XCDS, j = b / GP_XCDS;
  return (j / GP_XBLOCK) * (GP_XCDS * GP_XBLOCK) + x * GP_XBLOCK + j % GP_XBLOCK;
}

// Wave priority of an item from its cost bucket (4 per octave of tests): the few items of
// 2^18 tests and more -- cells under the largest polygons -- take the SIMD's issue slots
// first, so they end with the bulk instead of after it.
__device__ __forceinline__ void item_priority(const Item &it) {
  if (it.cost_rank >= 4 * 22) __builtin_amdgcn_s_setprio(3);
  else if (it.cost_rank >= 4 * 20) __builtin_amdgcn_s_setprio(2);
  else if (it.cost_rank >= 4 * 18) __builtin_amdgcn_s_setprio(1);
}

template <int PPL>
__global__ __launch_bounds__(64) void k_pipmix_pre(RefineArgs a, int persistent) {
  extern __shared__ __align__(16) unsigned char smem[];
  float4 *lds = (float4 *)smem;
  const uint32_t n_items = *a.n_items;
  uint32_t dead = 0;  // queues this workgroup has found exhausted
  uint32_t it = persistent ? next_item(a, n_items, dead) : xcd_item(blockIdx.x);
  while (it < n_items) {
    // a cell's last item runs with the fewest points per lane that hold its points
    const Item item = a.items[it];
    item_priority(item);
    if (PPL >= 4 && item.npts > 64 && item.npts <= 128) pipmix_pre_item<2>(a, item, lds);
    else if (PPL >= 2 && item.npts <= 64) pipmix_pre_item<1>(a, item, lds);
    else pipmix_pre_item<PPL>(a, item, lds);
    __builtin_amdgcn_s_setprio(0);
    if (!persistent) break;
    it = next_item(a, n_items, dead);
  }
}

// Work-queue pop for a workgroup of several waves (broadcast through LDS).
__device__ __forceinline__ uint32_t next_item_wg(const RefineArgs &a, uint32_t n_items,
                                                 uint32_t *slot, uint32_t &dead) {
  __syncthreads();
  if (threadIdx.x == 0) *slot = pop_item(a, n_items, dead);
  __syncthreads();
  return *slot;
}

template <int PPL, int W>
__global__ __launch_bounds__(64 * W) void k_p2p64(RefineArgs a, int persistent) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ uint32_t s_item;
  SegRec64 *lds = (SegRec64 *)smem;
  int2 *tab = (int2 *)(lds + a.edge_chunk);
  const uint32_t n_items = *a.n_items;
  uint32_t dead = 0;  // queues this workgroup has found exhausted
  uint32_t it = persistent ? (W == 1 ? next_item(a, n_items, dead)
                                      : next_item_wg(a, n_items, &s_item, dead))
                           : blockIdx.x;
  while (it < n_items) {
    p2p64_item<PPL, W>(a, a.items[it], lds, tab);
    if (!persistent) break;
    it = W == 1 ? next_item(a, n_items, dead) : next_item_wg(a, n_items, &s_item, dead);
  }
}

template <int PPL, int W, bool PRE>
__device__ __forceinline__ void p2pmix_loop(const RefineArgs &a, int persistent) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ uint32_t s_item;
  __shared__ float red[8];
  // slot t of the chunk is 32 bytes at U + 2t: the record's float4 U, then its V, so one
  // address register serves both reads of a slot and of its neighbour
  float4 *U = (float4 *)smem;
  float *V = (float *)(U + 1);
  int2 *tab = (int2 *)(U + 2 * a.edge_chunk);
  int *slotseg = (int *)(tab + a.edge_chunk);
  int *slotf = slotseg + a.edge_chunk;
  const uint32_t n_items = *a.n_items;
  uint32_t dead = 0;  // queues this workgroup has found exhausted
  uint32_t it = persistent ? (W == 1 ? next_item(a, n_items, dead)
                                      : next_item_wg(a, n_items, &s_item, dead))
                           : blockIdx.x;
  while (it < n_items) {
    // A cell's last item holds the remainder of its points: with one wave per item it
    // runs with the fewest points per lane that hold them, so its idle point slots cost
    // no tests.
    const Item item = a.items[it];
    if (W == 1 && item.npts <= a.vp_points) {
      // refined by k_p2p_vp
    } else if (W == 1 && PPL >= 4 && item.npts <= 128 && item.npts > 64)
      p2pmix_item<2, W, PRE>(a, item, U, V, tab, slotseg, slotf, red, smem);
    else if (W == 1 && PPL >= 2 && item.npts <= 64)
      p2pmix_item<1, W, PRE>(a, item, U, V, tab, slotseg, slotf, red, smem);
    else
      p2pmix_item<PPL, W, PRE>(a, item, U, V, tab, slotseg, slotf, red, smem);
    if (!persistent) break;
    it = W == 1 ? next_item(a, n_items, dead) : next_item_wg(a, n_items, &s_item, dead);
  }
}

// P2P's vertex-parallel items (at most vp_points points) run in a kernel of their own,
// in both precision forms (inlined into the refinement loops, their code would cost those
// loops registers and with them resident waves): k_vp_collect lists them (one atomic per
// wave), k_p2p_vp gives each a wave.
__global__ __launch_bounds__(256) void k_vp_collect(RefineArgs a) {
  const uint32_t n_items = *a.n_items;
  for (uint32_t base = blockIdx.x * blockDim.x; base < n_items; base += gridDim.x * blockDim.x) {
    const uint32_t i = base + threadIdx.x;
    const bool vp = i < n_items && a.items[i].npts <= a.vp_points;
    const uint64_t m = ballot(vp);
    if (m == 0) continue;
    uint32_t first = 0;
    if (lane_id() == 0) first = atomicAdd(a.vp_count, (uint32_t)__popcll(m));
    first = (uint32_t)__builtin_amdgcn_readfirstlane((int)first);
    if (vp) a.vp_list[first + (uint32_t)__popcll(m & lanemask_lt())] = i;
  }
}

__global__ __launch_bounds__(256) void k_p2p_vp(RefineArgs a) {
  __shared__ int32_t win[256 / GP_WAVE][3 * GP_WAVE];
  const uint32_t nvp = *a.vp_count;
  const uint32_t waves = gridDim.x * (blockDim.x / GP_WAVE);
  for (uint32_t q = blockIdx.x * (blockDim.x / GP_WAVE) + threadIdx.x / GP_WAVE; q < nvp;
       q += waves)
    p2p_vp_item(a, a.items[a.vp_list[q]], win[threadIdx.x / GP_WAVE]);
}

template <int PPL, int W>
__global__ __launch_bounds__(64 * W) void k_p2pmix(RefineArgs a, int persistent) {
  p2pmix_loop<PPL, W, false>(a, persistent);
}

// The same refinement on a grid with build-time segment records.
template <int PPL, int W>
__global__ __launch_bounds__(64 * W) void k_p2pmix_pre(RefineArgs a, int persistent) {
  p2pmix_loop<PPL, W, true>(a, persistent);
}

static size_t refine_lds_bytes(gp_kind kind, gp_precision prec, int ec, int W, bool pre) {
  if (kind == GP_PIP && prec == GP_MIXED && pre) return (size_t)PIP_PRE_CHUNK * 16 + GP_WAVE * 16;
  if (kind == GP_PIP)
    return prec == GP_FP64 ? (size_t)ec * sizeof(PipRec64) : (size_t)ec * (16 + 16 + 4);
  if (prec == GP_FP64) return (size_t)ec * (sizeof(SegRec64) + sizeof(int2));
  // the chunk (segment records, polyline table, slot map), reused by the exact pass
  const size_t chunk = (size_t)ec * (32 + sizeof(int2) + 2 * sizeof(int));
  const size_t epi = (size_t)W * P2P_EPI_BYTES;
  return chunk > epi ? chunk : epi;
}

#define GP_DISPATCH(KERNEL, PPLV, ...)                                             \
  do {                                                                             \
    if ((PPLV) == 1) hipLaunchKernelGGL(KERNEL<1>, __VA_ARGS__);                   \
    else if ((PPLV) == 2) hipLaunchKernelGGL(KERNEL<2>, __VA_ARGS__);              \
    else hipLaunchKernelGGL(KERNEL<4>, __VA_ARGS__);                               \
  } while (0)

#define GP_DISPATCH_W(KERNEL, PPLV, WV, ...)                                       \
  do {                                                                             \
    if ((WV) == 1) {                                                               \
      if ((PPLV) == 1) hipLaunchKernelGGL((KERNEL<1, 1>), __VA_ARGS__);              \
      else if ((PPLV) == 2) hipLaunchKernelGGL((KERNEL<2, 1>), __VA_ARGS__);         \
      else hipLaunchKernelGGL((KERNEL<4, 1>), __VA_ARGS__);                          \
    } else if ((WV) == 2) {                                                        \
      if ((PPLV) == 1) hipLaunchKernelGGL((KERNEL<1, 2>), __VA_ARGS__);              \
      else if ((PPLV) == 2) hipLaunchKernelGGL((KERNEL<2, 2>), __VA_ARGS__);         \
      else hipLaunchKernelGGL((KERNEL<4, 2>), __VA_ARGS__);                          \
    } else {                                                                       \
      if ((PPLV) == 1) hipLaunchKernelGGL((KERNEL<1, 4>), __VA_ARGS__);              \
      else if ((PPLV) == 2) hipLaunchKernelGGL((KERNEL<2, 4>), __VA_ARGS__);         \
      else hipLaunchKernelGGL((KERNEL<4, 4>), __VA_ARGS__);                          \
    }                                                                              \
  } while (0)

hipError_t launch_refine(gp_kind kind, gp_precision prec, const RefineArgs &a,
                         const gp_tuning &t, int num_cu, int64_t max_items, hipStream_t s) {
  const int ppl = t.points_per_lane;

  const bool pip_pre = kind == GP_PIP && prec == GP_MIXED && a.precs != nullptr;
  unsigned grid;
  if (t.persistent) {
    int64_t g = (int64_t)num_cu * t.wg_per_cu;
    if (g > max_items) g = max_items;
    grid = (unsigned)(g < 1 ? 1 : g);
  } else if (pip_pre) {
    // xcd_item maps whole blocks of GP_XCDS * GP_XBLOCK workgroups
    const int64_t blk = GP_XCDS * GP_XBLOCK;
    grid = (unsigned)(((max_items < 1 ? 1 : max_items) + blk - 1) / blk * blk);
  } else {
    grid = (unsigned)(max_items < 1 ? 1 : max_items);
  }
  const int pers = t.persistent ? 1 : 0;
  const int W = kind == GP_P2P ? t.waves_per_item : 1;
  const size_t lds = refine_lds_bytes(kind, prec, a.edge_chunk, W, pip_pre);
  const dim3 blk(64 * W);
  if (kind == GP_PIP && prec == GP_FP64)
    GP_DISPATCH(k_pip64, ppl, dim3(grid), blk, lds, s, a, pers);
  else if (pip_pre)
    GP_DISPATCH(k_pipmix_pre, ppl, dim3(grid), blk, lds, s, a, pers);
  else if (kind == GP_PIP)
    GP_DISPATCH(k_pipmix, ppl, dim3(grid), blk, lds, s, a, pers);
  else {
    if (W == 1 && t.vp_points > 0) {
      const unsigned gc = (unsigned)std::min<int64_t>((max_items + 255) / 256, 4096);
      hipLaunchKernelGGL(k_vp_collect, dim3(gc < 1 ? 1 : gc), dim3(256), 0, s, a);
      hipLaunchKernelGGL(k_p2p_vp, dim3((unsigned)num_cu * 8), dim3(256), 0, s, a);
    }
    if (prec == GP_FP64)
      GP_DISPATCH_W(k_p2p64, ppl, W, dim3(grid), blk, lds, s, a, pers);
    else if (a.recU)
      GP_DISPATCH_W(k_p2pmix_pre, ppl, W, dim3(grid), blk, lds, s, a, pers);
    else
      GP_DISPATCH_W(k_p2pmix, ppl, W, dim3(grid), blk, lds, s, a, pers);
  }
  return hipGetLastError();
}

// ------------------------------------------------------------------------- FP64 recheck
// Each queued point gets its full result over all candidates of its cell, in FP64 with
// the definitions' operation order, straight from the edge records.  Threads take the
// edges of a feature; parity combines by counting odd threads (XOR), distance by an
// exact wave minimum -- both independent of order.

// PIP: one workgroup per queued point.  Its threads split each candidate polygon's
// edges; the polygon's parity is that of the number of threads with an odd count of
// crossings, so even the longest rings take a few dozen steps per point.
__global__ __launch_bounds__(1024) void k_recheck_pip(RefineArgs a) {
  const uint32_t nq = *a.rq_count;
  for (uint32_t q = blockIdx.x; q < nq; q += gridDim.x) {
    const uint32_t i = a.rq[q];
    const uint32_t j = a.perm[i], cell = a.skey[i];
    const double2 p = a.xy[i];
    int32_t best = -1;
    for (int32_t k = a.cand_off[cell]; k < a.cand_off[cell + 1]; ++k) {
      const int32_t f = a.cand_id[k];
      const int32_t e1 = a.eoff[f + 1];
      int odd = 0;
#pragma unroll 4
      for (int32_t e = a.eoff[f] + (int32_t)threadIdx.x; e < e1; e += (int32_t)blockDim.x) {
        const double4 r = a.edge64[e];
        odd ^= cross64(p.x, p.y, r.x, r.y, r.z - r.x, r.w, r.w - r.y) ? 1 : 0;
      }
      // the count is the same in every thread, so the exit is uniform
      if (__syncthreads_count(odd) & 1) {
        best = f;
        break;
      }
    }
    if (threadIdx.x == 0) a.out_id[j] = best;
  }
}

__global__ __launch_bounds__(256) void k_recheck_p2p(RefineArgs a) {
  const uint32_t nq = *a.rq_count;
  const uint32_t lane = lane_id();
  const uint32_t waves = gridDim.x * (blockDim.x / GP_WAVE);
  for (uint32_t q = blockIdx.x * (blockDim.x / GP_WAVE) + threadIdx.x / GP_WAVE; q < nq;
       q += waves) {
    const uint32_t i = a.rq[q];
    const uint32_t j = a.perm[i], cell = a.skey[i];
    const double2 p = a.xy[i];
    const double x = p.x, y = p.y;
    int32_t bid = -1;
    double best = INFINITY;
    for (int32_t k = a.cand_off[cell]; k < a.cand_off[cell + 1]; ++k) {
      const int32_t f = a.cand_id[k];
      // a segment matters only if its d2 can beat thr = min(best, next(D2)); its
      // perpendicular quotient is divided out only when cc < fl(thr*L2)*(1+2^-49)
      const double thr = fmin(best, a.D2_next);
      double pd = INFINITY;
      for (int32_t e = a.eoff[f] + (int32_t)lane; e < a.eoff[f + 1]; e += GP_WAVE) {
        const double4 r = a.edge64[e];
        const double dx = r.z - r.x, dy = r.w - r.y;
        const double wx = x - r.x, wy = y - r.y;
        const double L2 = dx * dx + dy * dy;
        const double t = wx * dx + wy * dy;
        double d2;
        if (t <= 0.0) {
          d2 = wx * wx + wy * wy;
        } else if (t >= L2) {
          const double ex = x - r.z, ey = y - r.w;
          d2 = ex * ex + ey * ey;
        } else {
          const double c = wx * dy - wy * dx;
          const double cc = c * c;
          d2 = cc < (thr * L2) * (1.0 + 0x1p-49) ? cc / L2 : INFINITY;
        }
        pd = fmin(pd, d2);
      }
      pd = wave_min_f64(pd);
      if (pd <= a.D2 && pd < best) { best = pd; bid = f; }
    }
    if (lane == 0) {
      a.out_id[j] = bid;
      a.out_dist[j] = bid >= 0 ? sqrt(best) : INFINITY;
    }
  }
}

hipError_t launch_recheck(gp_kind kind, const RefineArgs &a, int num_cu, hipStream_t s) {
  const unsigned ncu = (unsigned)(num_cu > 0 ? num_cu : 256);
  if (kind == GP_PIP) hipLaunchKernelGGL(k_recheck_pip, dim3(ncu), dim3(1024), 0, s, a);
  else hipLaunchKernelGGL(k_recheck_p2p, dim3(ncu * 4), dim3(256), 0, s, a);
  return hipGetLastError();
}

}  // namespace gp
