// Measurement probes for the roofline: sustained vector FP32 / FP64 FMA rate (FP32 with
// VGPR operands and with an SGPR operand), LDS broadcast-read rate, and the P2P
// inner-loop instruction mix on register data.  Used by
// bench.py to report the peaks the refinement kernels are measured against; not part of
// the join itself.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "gp_internal.h"

namespace gp {
gp_status set_error(gp_status code, const char *fmt, ...);
}
using namespace gp;

namespace {

// 8 independent FMA chains per lane; the result is stored so nothing is dead code.
// VGPR_OPS: every operand in a VGPR (or an inline literal), the form the refinement
// kernels' inner loops take; otherwise one operand comes from an SGPR, which gfx950
// issues at about half the rate.
template <bool VGPR_OPS>
__global__ __launch_bounds__(256) void k_fma_f32(float *out, int iters, float a, float b) {
  float x[8], y[8];
#pragma unroll
  for (int c = 0; c < 8; ++c) {
    x[c] = threadIdx.x * 1e-7f + c;
    y[c] = VGPR_OPS ? 0.5f + 1e-3f * (float)(threadIdx.x & 7) + 1e-4f * c : a;
  }
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int c = 0; c < 8; ++c) x[c] = VGPR_OPS ? fmaf(x[c], y[c], x[c ^ 1]) : fmaf(x[c], a, b);
  }
  float s = 0.f;
#pragma unroll
  for (int c = 0; c < 8; ++c) s += x[c];
  out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

__global__ __launch_bounds__(256) void k_fma_f64(double *out, int iters, double a, double b) {
  double x0 = threadIdx.x * 1e-7, x1 = x0 + 1., x2 = x0 + 2., x3 = x0 + 3.;
  double x4 = x0 + 4., x5 = x0 + 5., x6 = x0 + 6., x7 = x0 + 7.;
  for (int i = 0; i < iters; ++i) {
    x0 = fma(x0, a, b); x1 = fma(x1, a, b); x2 = fma(x2, a, b); x3 = fma(x3, a, b);
    x4 = fma(x4, a, b); x5 = fma(x5, a, b); x6 = fma(x6, a, b); x7 = fma(x7, a, b);
  }
  out[blockIdx.x * blockDim.x + threadIdx.x] = x0 + x1 + x2 + x3 + x4 + x5 + x6 + x7;
}

// LDS broadcast: 4 x ds_read_b128 per iteration, every lane of a wave at the same
// address (within a 4 KB buffer); the wait for the reads is inside the same asm block.
__global__ __launch_bounds__(256) void k_lds_bcast(float *out, int iters) {
  __shared__ float4 buf[256];
  buf[threadIdx.x] = make_float4(threadIdx.x, 1.f, 2.f, 3.f);
  __syncthreads();
  float acc0 = 0.f, acc1 = 0.f, acc2 = 0.f, acc3 = 0.f;
  const uint32_t base = (threadIdx.x / 64) * 8 * 16;
  for (int i = 0; i < iters; ++i) {
    const uint32_t addr = base + (uint32_t)(i & 3) * 256u;  // + 48 + 16 < 4096
    float4 p, q, r, u;
    asm volatile(
        "ds_read_b128 %0, %4\n"
        "ds_read_b128 %1, %4 offset:16\n"
        "ds_read_b128 %2, %4 offset:32\n"
        "ds_read_b128 %3, %4 offset:48\n"
        "s_waitcnt lgkmcnt(0)\n"
        : "=v"(p), "=v"(q), "=v"(r), "=v"(u)
        : "v"(addr)
        : "memory");
    acc0 += p.x + p.w; acc1 += q.y + q.z; acc2 += r.z + r.x; acc3 += u.w + u.y;
  }
  out[blockIdx.x * blockDim.x + threadIdx.x] = acc0 + acc1 + acc2 + acc3;
}

__device__ __forceinline__ uint32_t probe_seg(float px, float py, const float4 U, float R) {
  const float s = fmaf(px, U.x, fmaf(py, U.y, U.z));
  const float r = fmaf(px, -U.y, fmaf(py, U.x, R));
  const float e = __builtin_amdgcn_fmed3f(fabsf(s) - U.w, 0.0f, 1.0f);
  return __float_as_uint(fmaf(e, e, r * r));
}

// The P2P test on segment constants held in registers (no LDS): the VALU-only cost.
__global__ __launch_bounds__(256) void k_p2p_mix_regs(uint32_t *out, int iters, float4 U0,
                                                      float4 U1, float R0, float R1) {
  float px0 = threadIdx.x * 1e-3f, py0 = blockIdx.x * 1e-3f;
  float px1 = px0 + 0.5f, py1 = py0 + 0.25f;
  uint32_t m0 = 0x7f800000u, m1 = 0x7f800000u;
  for (int i = 0; i < iters; ++i) {
    m0 = min(m0, min(probe_seg(px0, py0, U0, R0), probe_seg(px0, py0, U1, R1)));
    m1 = min(m1, min(probe_seg(px1, py1, U0, R0), probe_seg(px1, py1, U1, R1)));
    // perturb every constant so nothing is loop-invariant (4 extra adds per 4 tests)
    U0.z += 1e-6f;
    U1.z -= 1e-6f;
    R0 += 1e-6f;
    R1 -= 1e-6f;
  }
  out[blockIdx.x * blockDim.x + threadIdx.x] = m0 ^ m1;
}

// The same test in the refinement loop's shape: four points per lane against two
// segments per step, every operand in a VGPR (the segment constants differ per lane,
// as after an LDS read), the running minimum with v_min3.
__global__ __launch_bounds__(256) void k_p2p_mix_vregs(uint32_t *out, int iters, float4 U0,
                                                       float4 U1, float R0, float R1) {
  const float o = (float)(threadIdx.x & 63) * 1e-6f;
  U0.x += o; U0.y -= o; U0.z += o; U0.w += o;
  U1.x -= o; U1.y += o; U1.z -= o; U1.w += o;
  R0 += o;
  R1 -= o;
  float px[4], py[4];
  uint32_t m[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    px[j] = threadIdx.x * 1e-3f + 0.25f * j;
    py[j] = blockIdx.x * 1e-3f - 0.125f * j;
    m[j] = 0x7f800000u;
  }
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int j = 0; j < 4; ++j)
      m[j] = min(m[j], min(probe_seg(px[j], py[j], U0, R0), probe_seg(px[j], py[j], U1, R1)));
    // perturb the constants so nothing is loop-invariant (4 extra adds per 8 tests, in
    // place of the loop's address moves)
    U0.z += 1e-6f;
    U1.z -= 1e-6f;
    R0 += 1e-6f;
    R1 -= 1e-6f;
  }
  out[blockIdx.x * blockDim.x + threadIdx.x] = m[0] ^ m[1] ^ m[2] ^ m[3];
}

// The mixed PIP crossing test on per-lane VGPR data in the refinement loop's shape:
// PPL points per lane against E edges per step, each test a subtract, an FMA and two
// compares whose lane masks combine on the scalar unit (AND, then XOR into the parity).
template <int PPL, int E>
__global__ __launch_bounds__(256) void k_pip_mix_vregs(uint32_t *out, int iters, float4 e0) {
  // every edge value differs per lane and per edge, as after an LDS read
  const uint32_t l = threadIdx.x & 63;
  const float o = (float)l * 1e-6f;
  float4 e[E];
#pragma unroll
  for (int q = 0; q < E; ++q)
    e[q] = make_float4(e0.x + o * (float)(q + 1), e0.y - o * (float)(q + 2),
                       __uint_as_float(0x3f000000u + 4u * l + (uint32_t)q),
                       e0.w + o * (float)(2 * q + 1));
  float px[PPL], py[PPL];
  uint64_t par[PPL];
#pragma unroll
  for (int j = 0; j < PPL; ++j) {
    px[j] = threadIdx.x * 1e-4f + 0.25f * j;
    py[j] = blockIdx.x * 1e-4f - 0.125f * j;
    par[j] = 0;
  }
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int j = 0; j < PPL; ++j) {
      uint64_t m = 0;
#pragma unroll
      for (int q = 0; q < E; ++q) {
        const float ty = py[j] - e[q].y;
        const float xi = fmaf(ty, e[q].w, e[q].x);
        m ^= __builtin_amdgcn_ballot_w64(__float_as_uint(ty) < __float_as_uint(e[q].z)) &
             __builtin_amdgcn_ballot_w64(px[j] < xi);
      }
      par[j] ^= m;
      // move the point so nothing is loop-invariant (one add per E tests, about the
      // loop's LDS address move)
      py[j] += 1e-7f;
    }
  }
  uint64_t r = 0;
#pragma unroll
  for (int j = 0; j < PPL; ++j) r ^= par[j];
  out[blockIdx.x * blockDim.x + threadIdx.x] = (uint32_t)(r >> (threadIdx.x & 63)) & 1u;
}

}  // namespace

// which: 0 FP32 FMA on VGPR operands, 1 FP64 FMA, 2 LDS broadcast 16-byte reads, 3 the
// P2P test on register data with the segment constants in SGPRs, 4 FP32 FMA with an
// SGPR operand, 5 the P2P test on per-lane VGPR data in the refinement loop's shape, 6 and
// 7 the PIP crossing test on per-lane VGPR data (2 points per lane x 8 edges per step,
// 4 points per lane x 4 edges).  Returns the achieved rate: FLOP/s (0, 1, 4), wave-level
// broadcast reads per second (2) or tests per second (3, 5, 6, 7).
extern "C" gp_status gp_probe_rate(int32_t which, int32_t iters, double *rate, float *ms) {
  if (!rate || iters <= 0 || which < 0 || which > 7)
    return set_error(GP_E_INVALID_ARG, "bad probe arguments");
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return set_error(GP_E_HIP, "no device");
  const int blocks = cus * 32, threads = 256;
  void *buf = nullptr;
  if (hipMalloc(&buf, (size_t)blocks * threads * 8) != hipSuccess)
    return set_error(GP_E_OOM, "probe buffer");
  hipEvent_t e0, e1;
  (void)hipEventCreate(&e0);
  (void)hipEventCreate(&e1);
  double work = 0.0;
  for (int rep = 0; rep < 2; ++rep) {  // first launch warms up
    (void)hipEventRecord(e0, nullptr);
    const double nthr = (double)blocks * threads;
    switch (which) {
      case 0:
      case 4:
        if (which == 0)
          hipLaunchKernelGGL(k_fma_f32<true>, dim3(blocks), dim3(threads), 0, nullptr,
                             (float *)buf, iters, 0.999f, 1e-3f);
        else
          hipLaunchKernelGGL(k_fma_f32<false>, dim3(blocks), dim3(threads), 0, nullptr,
                             (float *)buf, iters, 0.999f, 1e-3f);
        work = nthr * iters * 8 * 2;
        break;
      case 1:
        hipLaunchKernelGGL(k_fma_f64, dim3(blocks), dim3(threads), 0, nullptr, (double *)buf, iters,
                           0.999, 1e-3);
        work = nthr * iters * 8 * 2;
        break;
      case 2:
        hipLaunchKernelGGL(k_lds_bcast, dim3(blocks), dim3(threads), 0, nullptr, (float *)buf, iters);
        work = nthr / 64.0 * iters * 4;  // wave-level broadcast reads
        break;
      case 6:
        hipLaunchKernelGGL((k_pip_mix_vregs<2, 8>), dim3(blocks), dim3(threads), 0, nullptr,
                           (uint32_t *)buf, iters, make_float4(0.1f, 0.2f, 0.0f, 0.4f));
        work = nthr * iters * 16;
        break;
      case 7:
        hipLaunchKernelGGL((k_pip_mix_vregs<4, 4>), dim3(blocks), dim3(threads), 0, nullptr,
                           (uint32_t *)buf, iters, make_float4(0.1f, 0.2f, 0.0f, 0.4f));
        work = nthr * iters * 16;
        break;
      case 5:
        hipLaunchKernelGGL(k_p2p_mix_vregs, dim3(blocks), dim3(threads), 0, nullptr,
                           (uint32_t *)buf, iters, make_float4(0.1f, 0.2f, 0.3f, 0.4f),
                           make_float4(0.5f, 0.6f, 0.7f, 0.8f), 0.9f, 1.1f);
        work = nthr * iters * 8;
        break;
      default:
        hipLaunchKernelGGL(k_p2p_mix_regs, dim3(blocks), dim3(threads), 0, nullptr,
                           (uint32_t *)buf, iters, make_float4(0.1f, 0.2f, 0.3f, 0.4f),
                           make_float4(0.5f, 0.6f, 0.7f, 0.8f), 0.9f, 1.1f);
        work = nthr * iters * 4;  // point-segment tests
        break;
    }
    (void)hipEventRecord(e1, nullptr);
  }
  hipError_t err = hipEventSynchronize(e1);
  float t = 0.f;
  (void)hipEventElapsedTime(&t, e0, e1);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  (void)hipFree(buf);
  if (err != hipSuccess) return set_error(GP_E_HIP, "probe failed: %s", hipGetErrorString(err));
  *rate = work / (t * 1e-3);
  if (ms) *ms = t;
  return GP_OK;
}
