// bfp_tune.hip -- autotuning of bfp_binop's launch configuration.
//
// For one (op, format, rounding mode) every candidate
//   words_per_lane in {1, 2}      (W = 32 or 64 elements per lane word)
//   block          in {64, 128, 256, 512}
//   blocks_per_cu  in {0, 4, 8}   (0: one thread per slice; else a
//                                   grid-stride loop of that depth)
// is timed on a probe vector with HIP events, median of `reps` runs, each run
// preceded by a read sweep over a 512 MiB buffer so the probe's operands are
// not served from the 256 MB last-level cache (a read sweep leaves clean
// lines, so the timed kernel pays no write-back of someone else's data).  The
// circuits are data-oblivious, so random bits serve as operands.  The winner
// is installed with bfp_launch_set.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <vector>

#include "bfp.h"
#include "bfp_kernels.hpp"

namespace bfp {
namespace {

__global__ void k_fill_random(uint32_t* p, uint64_t n, uint32_t seed) {
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x) {
    uint32_t x = (uint32_t)i * 2654435761u ^ seed;
    x ^= x >> 16;
    x *= 0x7feb352du;
    x ^= x >> 15;
    x *= 0x846ca68bu;
    x ^= x >> 16;
    p[i] = x;
  }
}

__global__ void k_sweep_read(const u32x4* p, uint64_t n4, uint32_t* sink) {
  uint32_t acc = 0;
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n4; i += (uint64_t)gridDim.x * blockDim.x) {
    const u32x4 v = p[i];
    acc ^= v.x ^ v.y ^ v.z ^ v.w;
  }
  if (acc == 0x9E3779B9u) sink[threadIdx.x & 63] = acc;  // keeps the loads live; practically never taken
}

// Plain copy, 16 bytes per lane per iteration, grid-stride: the practical
// HBM ceiling the kernels' fractions are read against.
__global__ void k_copy16(const u32x4* src, u32x4* dst, uint64_t n4) {
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n4; i += (uint64_t)gridDim.x * blockDim.x)
    dst[i] = src[i];
}

struct DevBuf {
  void* p = nullptr;
  ~DevBuf() {
    if (p) (void)hipFree(p);
  }
};

}  // namespace
}  // namespace bfp

using namespace bfp;

extern "C" bfp_status bfp_measure_copy(uint64_t bytes, int reps, void* stream, double* gbps) {
  if (!gbps) return BFP_E_NULL;
  if (bytes < (1u << 20) || bytes > (1ull << 36) || (bytes & 15u) || reps < 1 || reps > 1000) return BFP_E_ARG;
  hipStream_t s = (hipStream_t)stream;
  DevBuf src, dst;
  if (hipMalloc(&src.p, bytes) != hipSuccess || hipMalloc(&dst.p, bytes) != hipSuccess) return BFP_E_NOMEM;
  const uint64_t n4 = bytes / 16;
  hipLaunchKernelGGL(k_fill_random, dim3(2048), dim3(256), 0, s, (uint32_t*)src.p, bytes / 4, 0x4242u);
  const unsigned grid = (unsigned)std::min<uint64_t>((n4 + 255) / 256, 256ull * 64);
  for (int w = 0; w < 2; ++w)
    hipLaunchKernelGGL(k_copy16, dim3(grid), dim3(256), 0, s, (const u32x4*)src.p, (u32x4*)dst.p, n4);
  if (hipGetLastError() != hipSuccess) return BFP_E_HIP;
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess) return BFP_E_HIP;
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return BFP_E_HIP;
  }
  bfp_status st = BFP_OK;
  float ms = 0.f;
  if (hipEventRecord(e0, s) != hipSuccess) st = BFP_E_HIP;
  for (int r = 0; r < reps && st == BFP_OK; ++r)
    hipLaunchKernelGGL(k_copy16, dim3(grid), dim3(256), 0, s, (const u32x4*)src.p, (u32x4*)dst.p, n4);
  if (st == BFP_OK && hipGetLastError() != hipSuccess) st = BFP_E_HIP;
  if (st == BFP_OK && hipEventRecord(e1, s) != hipSuccess) st = BFP_E_HIP;
  if (st == BFP_OK && hipEventSynchronize(e1) != hipSuccess) st = BFP_E_HIP;
  if (st == BFP_OK && hipEventElapsedTime(&ms, e0, e1) != hipSuccess) st = BFP_E_HIP;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (st == BFP_OK) *gbps = 2.0 * (double)bytes / ((double)ms / reps * 1e-3) / 1e9;
  return st;
}

extern "C" bfp_status bfp_autotune(int op, bfp_format f, uint64_t n_probe, int words_per_lane_mask, int reps,
                                   void* stream, bfp_launch* best_out, double* best_us_out) {
  if (!op_valid(op)) return BFP_E_OP;
  if (!bfp_format_supported(f)) return BFP_E_FORMAT;
  if (n_probe == 0 || n_probe > (1ull << 30)) return BFP_E_ARG;
  if ((words_per_lane_mask & 3) == 0) return BFP_E_ARG;
  if (reps < 1 || reps > 1000) return BFP_E_ARG;
  hipStream_t s = (hipStream_t)stream;
  const size_t vec_bytes = bfp_bitslice_bytes(f, n_probe);
  const uint64_t sweep_bytes = 512ull << 20;
  DevBuf a, b, c, sweep, sink;
  if (hipMalloc(&a.p, vec_bytes) != hipSuccess || hipMalloc(&b.p, vec_bytes) != hipSuccess ||
      hipMalloc(&c.p, vec_bytes) != hipSuccess || hipMalloc(&sweep.p, sweep_bytes) != hipSuccess ||
      hipMalloc(&sink.p, 256) != hipSuccess)
    return BFP_E_NOMEM;
  hipLaunchKernelGGL(k_fill_random, dim3(2048), dim3(256), 0, s, (uint32_t*)a.p, vec_bytes / 4, 0x1234u);
  hipLaunchKernelGGL(k_fill_random, dim3(2048), dim3(256), 0, s, (uint32_t*)b.p, vec_bytes / 4, 0x9876u);
  hipLaunchKernelGGL(k_fill_random, dim3(2048), dim3(256), 0, s, (uint32_t*)sweep.p, sweep_bytes / 4, 0x5555u);
  if (hipGetLastError() != hipSuccess) return BFP_E_HIP;

  bfp_launch saved;
  bfp_status st = bfp_launch_get(op, f, &saved);
  if (st != BFP_OK) return st;
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess) return BFP_E_HIP;
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return BFP_E_HIP;
  }
  const int blocks[] = {64, 128, 256, 512};
  const int bpcs[] = {0, 4, 8};
  double best = 1e30;
  bfp_launch best_cfg = saved;
  std::vector<float> ts;
  bool any = false;
  for (int wpl = 1; wpl <= 2 && st == BFP_OK; ++wpl) {
    if (!(words_per_lane_mask & wpl)) continue;
    if (!registry().binop[f.e][f.m][opclass_of(op)][f.round][wpl - 1]) continue;  // not compiled
    any = true;
    for (int blk : blocks) {
      if (blk > registry().max_block[f.e][f.m]) continue;  // not compiled for such blocks
      for (int bpc : bpcs) {
        bfp_launch cfg;
        cfg.words_per_lane = wpl;
        cfg.block = blk;
        cfg.blocks_per_cu = bpc;
        cfg.pad = 0;
        st = bfp_launch_set(op, f, &cfg);
        if (st != BFP_OK) break;
        ts.clear();
        for (int r = 0; r <= reps && st == BFP_OK; ++r) {
          hipLaunchKernelGGL(k_sweep_read, dim3(4096), dim3(256), 0, s, (const u32x4*)sweep.p, sweep_bytes / 16,
                             (uint32_t*)sink.p);
          if (hipEventRecord(e0, s) != hipSuccess) st = BFP_E_HIP;
          if (st == BFP_OK) st = bfp_binop(op, f, a.p, b.p, c.p, n_probe, stream);
          if (st == BFP_OK && hipEventRecord(e1, s) != hipSuccess) st = BFP_E_HIP;
          if (st == BFP_OK && hipEventSynchronize(e1) != hipSuccess) st = BFP_E_HIP;
          float ms = 0.f;
          if (st == BFP_OK && hipEventElapsedTime(&ms, e0, e1) != hipSuccess) st = BFP_E_HIP;
          if (r > 0) ts.push_back(ms);  // first run warms the code path
        }
        if (st != BFP_OK) break;
        std::nth_element(ts.begin(), ts.begin() + ts.size() / 2, ts.end());
        const double med = ts[ts.size() / 2] * 1e3;
        if (med < best) {
          best = med;
          best_cfg = cfg;
        }
      }
      if (st != BFP_OK) break;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (st == BFP_OK && !any) st = BFP_E_ARG;  // no allowed word width is compiled for f
  if (st != BFP_OK) {
    (void)bfp_launch_set(op, f, &saved);
    return st;
  }
  st = bfp_launch_set(op, f, &best_cfg);
  if (best_out) *best_out = best_cfg;
  if (best_us_out) *best_us_out = best;
  return st;
}
