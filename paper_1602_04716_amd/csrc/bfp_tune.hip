// bfp_tune.hip -- autotuning of bfp_binop's launch configuration.
//
// For one (op, format, rounding mode) every compiled candidate
//   words_per_lane in {1, 2, 4}   (W = 32, 64 or 128 elements per lane word;
//                                   4 for formats of at most 10 bits)
//   unroll         in {1, 2}      (units per lane per loop step)
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
#include <mutex>
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

// Ceiling probes: plain read, write and copy sweeps, and a sweep that reads
// two streams and writes their XOR to a third (the traffic of an elementwise
// binary op), with U independent 16-byte accesses per stream in flight per
// lane (each wave instruction covers 1 KiB contiguous; the U accesses of a
// lane are a grid stride apart), with ordinary or non-temporal accesses.
// The best launch shape over a sweep of grids (1 to 32 blocks per CU) and
// block sizes (256 to 1024 threads for 1 or 2 blocks per CU) is the
// practical HBM ceiling the kernels' fractions are read against: writes in
// particular go fastest from few waves (one 256-thread block per CU), not
// from a full grid.  In mode 3 `src` holds the two read streams back to back,
// n4 16-byte words each.
template <int MODE, int U, bool NT>  // MODE 0 read, 1 write, 2 copy, 3 two reads + one write; NT: non-temporal
__global__ void __launch_bounds__(1024) k_bw(const u32x4* __restrict__ src, u32x4* __restrict__ dst, uint64_t n4,
                                            uint32_t* sink) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
  uint32_t acc = 0;
  for (; i + (U - 1) * stride < n4; i += U * stride) {
    u32x4 v[U];
    if constexpr (MODE == 3) {
      u32x4 w[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        v[u] = NT ? __builtin_nontemporal_load(src + i + u * stride) : src[i + u * stride];
        w[u] = NT ? __builtin_nontemporal_load(src + n4 + i + u * stride) : src[n4 + i + u * stride];
      }
#pragma unroll
      for (int u = 0; u < U; ++u) v[u] = u32x4{v[u].x ^ w[u].x, v[u].y ^ w[u].y, v[u].z ^ w[u].z, v[u].w ^ w[u].w};
    } else if constexpr (MODE != 1) {
#pragma unroll
      for (int u = 0; u < U; ++u) v[u] = NT ? __builtin_nontemporal_load(src + i + u * stride) : src[i + u * stride];
    } else {
#pragma unroll
      for (int u = 0; u < U; ++u) v[u] = u32x4{(uint32_t)i, (uint32_t)u, 0u, 0u};
    }
    if constexpr (MODE == 0) {
#pragma unroll
      for (int u = 0; u < U; ++u) acc ^= v[u].x ^ v[u].y ^ v[u].z ^ v[u].w;
    } else {
#pragma unroll
      for (int u = 0; u < U; ++u) {
        if constexpr (NT) __builtin_nontemporal_store(v[u], dst + i + u * stride);
        else dst[i + u * stride] = v[u];
      }
    }
  }
  for (; i < n4; i += stride) {  // the last partial round
    if constexpr (MODE == 0) {
      const u32x4 v = src[i];
      acc ^= v.x ^ v.y ^ v.z ^ v.w;
    } else if constexpr (MODE == 1) {
      dst[i] = u32x4{(uint32_t)i, 0u, 0u, 0u};
    } else if constexpr (MODE == 2) {
      dst[i] = src[i];
    } else {
      const u32x4 v = src[i], w = src[n4 + i];
      dst[i] = u32x4{v.x ^ w.x, v.y ^ w.y, v.z ^ w.z, v.w ^ w.w};
    }
  }
  if (MODE == 0 && acc == 0x9E3779B9u) sink[threadIdx.x & 63] = acc;  // keeps the loads live
}

using BwLauncher = void (*)(unsigned grid, unsigned block, hipStream_t s, const u32x4* src, u32x4* dst, uint64_t n4,
                           uint32_t* sink);
template <int MODE, int U, bool NT>
void launch_bw(unsigned grid, unsigned block, hipStream_t s, const u32x4* src, u32x4* dst, uint64_t n4,
               uint32_t* sink) {
  hipLaunchKernelGGL((k_bw<MODE, U, NT>), dim3(grid), dim3(block), 0, s, src, dst, n4, sink);
}

struct DevBuf {
  void* p = nullptr;
  ~DevBuf() {
    if (p) (void)hipFree(p);
  }
};

// Median microseconds of `reps` runs of `run`, each after a read sweep of
// the 512 MiB `sweep` buffer (plus one untimed warm-up run).
template <class Run>
bfp_status median_cold_us(Run run, int reps, hipStream_t s, const DevBuf& sweep, const DevBuf& sink, double* us) {
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess) return BFP_E_HIP;
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return BFP_E_HIP;
  }
  const uint64_t sweep_bytes = 512ull << 20;
  bfp_status st = BFP_OK;
  std::vector<float> ts;
  for (int r = 0; r <= reps && st == BFP_OK; ++r) {
    hipLaunchKernelGGL(k_sweep_read, dim3(4096), dim3(256), 0, s, (const u32x4*)sweep.p, sweep_bytes / 16,
                       (uint32_t*)sink.p);
    if (hipEventRecord(e0, s) != hipSuccess) st = BFP_E_HIP;
    if (st == BFP_OK) st = run();
    if (st == BFP_OK && hipEventRecord(e1, s) != hipSuccess) st = BFP_E_HIP;
    if (st == BFP_OK && hipEventSynchronize(e1) != hipSuccess) st = BFP_E_HIP;
    float ms = 0.f;
    if (st == BFP_OK && hipEventElapsedTime(&ms, e0, e1) != hipSuccess) st = BFP_E_HIP;
    if (r > 0) ts.push_back(ms);  // the first run warms the code path
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (st != BFP_OK) return st;
  std::nth_element(ts.begin(), ts.begin() + ts.size() / 2, ts.end());
  *us = ts[ts.size() / 2] * 1e3;
  return BFP_OK;
}

// Time `run` under every block x grid depth (words per lane fixed at wpl),
// each configuration installed by `set` first; the fastest is left in
// *best_cfg and *best_us.
template <class Set, class Run>
bfp_status tune_block_grid(Set set, Run run, int wpl, int reps, hipStream_t s, const DevBuf& sweep,
                           const DevBuf& sink, bfp_launch* best_cfg, double* best_us) {
  const int blocks[] = {64, 128, 256, 512};
  const int bpcs[] = {0, 4, 8};
  *best_us = 1e30;
  for (int blk : blocks)
    for (int bpc : bpcs) {
      const bfp_launch cfg{wpl, blk, bpc, 1};
      bfp_status st = set(cfg);
      double us = 0;
      if (st == BFP_OK) st = median_cold_us(run, reps, s, sweep, sink, &us);
      if (st != BFP_OK) return st;
      if (us < *best_us) {
        *best_us = us;
        *best_cfg = cfg;
      }
    }
  return BFP_OK;
}

}  // namespace
}  // namespace bfp

using namespace bfp;

extern "C" bfp_status bfp_measure_hbm(uint64_t bytes, int mode, int reps, void* stream, double* gbps,
                                     int* best_grid, int* best_block, int* best_unroll) {
  if (!gbps) return BFP_E_NULL;
  if (bytes < (1u << 20) || bytes > (1ull << 36) || (bytes & 15u) || reps < 1 || reps > 1000) return BFP_E_ARG;
  if (mode < 0 || mode > 3) return BFP_E_ARG;
  hipStream_t s = (hipStream_t)stream;
  DevBuf src, dst, sink;
  const uint64_t src_bytes = mode == 3 ? 2 * bytes : bytes;  // mode 3: two read streams of `bytes` each
  if (hipMalloc(&src.p, src_bytes) != hipSuccess || hipMalloc(&dst.p, bytes) != hipSuccess ||
      hipMalloc(&sink.p, 256) != hipSuccess)
    return BFP_E_NOMEM;
  const uint64_t n4 = bytes / 16;
  hipLaunchKernelGGL(k_fill_random, dim3(2048), dim3(256), 0, s, (uint32_t*)src.p, src_bytes / 4, 0x4242u);
  if (hipGetLastError() != hipSuccess) return BFP_E_HIP;
  static const BwLauncher table[4][8] = {
#define BFP_BW_ROW(MODE)                                                                                      \
  {launch_bw<MODE, 1, false>, launch_bw<MODE, 2, false>, launch_bw<MODE, 4, false>, launch_bw<MODE, 8, false>, \
   launch_bw<MODE, 1, true>, launch_bw<MODE, 2, true>, launch_bw<MODE, 4, true>, launch_bw<MODE, 8, true>}
      BFP_BW_ROW(0), BFP_BW_ROW(1), BFP_BW_ROW(2), BFP_BW_ROW(3)};
#undef BFP_BW_ROW
  const int unrolls[8] = {1, 2, 4, 8, 1, 2, 4, 8};
  struct Shape {
    int blocks_per_cu, block;
  };
  static const Shape shapes[] = {{1, 256}, {1, 512}, {1, 1024}, {2, 256}, {2, 512}, {4, 256},
                                 {8, 256}, {16, 256}, {32, 256}};
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1)
    return BFP_E_NODEV;
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess) return BFP_E_HIP;
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return BFP_E_HIP;
  }
  bfp_status st = BFP_OK;
  double best = 0.0;
  for (int ui = 0; ui < 8 && st == BFP_OK; ++ui) {
    for (const Shape& sh : shapes) {
      const BwLauncher L = table[mode][ui];
      const unsigned grid = (unsigned)(cus * sh.blocks_per_cu), block = (unsigned)sh.block;
      L(grid, block, s, (const u32x4*)src.p, (u32x4*)dst.p, n4, (uint32_t*)sink.p);  // warm-up
      float ms = 0.f;
      if (hipEventRecord(e0, s) != hipSuccess) st = BFP_E_HIP;
      for (int r = 0; r < reps && st == BFP_OK; ++r)
        L(grid, block, s, (const u32x4*)src.p, (u32x4*)dst.p, n4, (uint32_t*)sink.p);
      if (st == BFP_OK && hipGetLastError() != hipSuccess) st = BFP_E_HIP;
      if (st == BFP_OK && hipEventRecord(e1, s) != hipSuccess) st = BFP_E_HIP;
      if (st == BFP_OK && hipEventSynchronize(e1) != hipSuccess) st = BFP_E_HIP;
      if (st == BFP_OK && hipEventElapsedTime(&ms, e0, e1) != hipSuccess) st = BFP_E_HIP;
      if (st != BFP_OK) break;
      const double moved = (mode == 2 ? 2.0 : (mode == 3 ? 3.0 : 1.0)) * (double)bytes;
      const double g = moved / ((double)ms / reps * 1e-3) / 1e9;
      if (g > best) {
        best = g;
        if (best_grid) *best_grid = (int)grid;
        if (best_block) *best_block = (int)block;
        if (best_unroll) *best_unroll = unrolls[ui];
      }
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (st == BFP_OK) *gbps = best;
  return st;
}

extern "C" bfp_status bfp_measure_copy(uint64_t bytes, int reps, void* stream, double* gbps) {
  return bfp_measure_hbm(bytes, 2, reps, stream, gbps, nullptr, nullptr, nullptr);
}

// Read sweep over `bytes` of a library buffer, so that what a following
// kernel reads comes from HBM rather than the 256 MB last-level cache.
extern "C" bfp_status bfp_flush_llc(uint64_t bytes, void* stream) {
  static std::mutex mu;
  static void* buf[64] = {};
  static uint64_t cap[64] = {};
  if (bytes < (1u << 20) || bytes > (1ull << 34)) return BFP_E_ARG;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return BFP_E_NODEV;
  std::lock_guard<std::mutex> lk(mu);
  bytes = (bytes + 15) / 16 * 16;
  if (cap[dev] < bytes + 256) {
    if (buf[dev]) (void)hipFree(buf[dev]);
    buf[dev] = nullptr;
    cap[dev] = 0;
    if (hipMalloc(&buf[dev], bytes + 256) != hipSuccess) return BFP_E_NOMEM;
    cap[dev] = bytes + 256;
    hipLaunchKernelGGL(k_fill_random, dim3(2048), dim3(256), 0, (hipStream_t)stream, (uint32_t*)buf[dev],
                       bytes / 4, 0x7777u);
  }
  uint8_t* b = static_cast<uint8_t*>(buf[dev]);
  hipLaunchKernelGGL(k_sweep_read, dim3(4096), dim3(256), 0, (hipStream_t)stream, (const u32x4*)b, bytes / 16,
                     (uint32_t*)(b + bytes));
  return hipGetLastError() == hipSuccess ? BFP_OK : BFP_E_HIP;
}

// One wave running a dependent chain of fused multiply-adds: the kernel's
// duration is that wave's lifetime.
__global__ void __launch_bounds__(64) k_wave_clock(float* out, int iters) {
  float x = (float)threadIdx.x;
  for (int i = 0; i < iters; ++i) x = __builtin_fmaf(x, 0.999f, 0.001f);
  out[threadIdx.x] = x;
}

extern "C" bfp_status bfp_wave_clock(int iters, void* stream) {
  static std::mutex mu;
  static void* buf[64] = {};
  if (iters < 1 || iters > (1 << 26)) return BFP_E_ARG;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return BFP_E_NODEV;
  std::lock_guard<std::mutex> lk(mu);
  if (!buf[dev] && hipMalloc(&buf[dev], 256) != hipSuccess) {
    buf[dev] = nullptr;
    return BFP_E_NOMEM;
  }
  hipLaunchKernelGGL(k_wave_clock, dim3(1), dim3(64), 0, (hipStream_t)stream, static_cast<float*>(buf[dev]), iters);
  return hipGetLastError() == hipSuccess ? BFP_OK : BFP_E_HIP;
}

extern "C" bfp_status bfp_autotune(int op, bfp_format f, uint64_t n_probe, int words_per_lane_mask, int reps,
                                   void* stream, bfp_launch* best_out, double* best_us_out) {
  if (!op_valid(op)) return BFP_E_OP;
  if (!bfp_format_supported(f)) return BFP_E_FORMAT;
  if (n_probe == 0 || n_probe > (1ull << 30)) return BFP_E_ARG;
  if ((words_per_lane_mask & 7) == 0) return BFP_E_ARG;
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
  for (int wi = 0; wi < kWordChoices && st == BFP_OK; ++wi) {
    const int wpl = 1 << wi;
    if (!(words_per_lane_mask & (1 << wi))) continue;
    for (int unroll = 1; unroll <= kUnrollChoices && st == BFP_OK; ++unroll) {
      if (!registry().binop[f.e][f.m][opclass_of(op)][f.round][wi][unroll - 1]) continue;  // not compiled
      any = true;
      for (int blk : blocks) {
        if (blk > registry().max_block[f.e][f.m]) continue;  // not compiled for such blocks
        for (int bpc : bpcs) {
          bfp_launch cfg;
          cfg.words_per_lane = wpl;
          cfg.block = blk;
          cfg.blocks_per_cu = bpc;
          cfg.unroll = unroll;
          st = bfp_launch_set(op, f, &cfg);
          if (st != BFP_OK) break;
          ts.clear();
          for (int r = 0; r <= reps && st == BFP_OK; ++r) {
            hipLaunchKernelGGL(k_sweep_read, dim3(4096), dim3(256), 0, s, (const u32x4*)sweep.p,
                               sweep_bytes / 16, (uint32_t*)sink.p);
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

extern "C" bfp_status bfp_autotune_chain(int op1, int op2, bfp_format f, uint64_t n_probe, int reps, void* stream,
                                         bfp_launch* best_out, double* best_us_out) {
  bfp_launch saved;
  bfp_status st = bfp_chain_launch_get(op1, op2, f, &saved);
  if (st != BFP_OK) return st;
  if (n_probe == 0 || n_probe > (1ull << 30) || reps < 1 || reps > 1000) return BFP_E_ARG;
  hipStream_t s = (hipStream_t)stream;
  const size_t vec_bytes = bfp_bitslice_bytes(f, n_probe);
  DevBuf a, b, c, d, sweep, sink;
  if (hipMalloc(&a.p, vec_bytes) != hipSuccess || hipMalloc(&b.p, vec_bytes) != hipSuccess ||
      hipMalloc(&c.p, vec_bytes) != hipSuccess || hipMalloc(&d.p, vec_bytes) != hipSuccess ||
      hipMalloc(&sweep.p, 512ull << 20) != hipSuccess || hipMalloc(&sink.p, 256) != hipSuccess)
    return BFP_E_NOMEM;
  hipLaunchKernelGGL(k_fill_random, dim3(2048), dim3(256), 0, s, (uint32_t*)a.p, vec_bytes / 4, 0x1234u);
  hipLaunchKernelGGL(k_fill_random, dim3(2048), dim3(256), 0, s, (uint32_t*)b.p, vec_bytes / 4, 0x9876u);
  hipLaunchKernelGGL(k_fill_random, dim3(2048), dim3(256), 0, s, (uint32_t*)c.p, vec_bytes / 4, 0x4321u);
  hipLaunchKernelGGL(k_fill_random, dim3(2048), dim3(256), 0, s, (uint32_t*)sweep.p, (512ull << 20) / 4, 0x5555u);
  if (hipGetLastError() != hipSuccess) return BFP_E_HIP;
  bfp_launch best = saved;
  double us = 0;
  st = tune_block_grid([&](const bfp_launch& cfg) { return bfp_chain_launch_set(op1, op2, f, &cfg); },
                       [&]() { return bfp_chain2(op1, op2, f, a.p, b.p, c.p, d.p, n_probe, stream); }, 1, reps, s,
                       sweep, sink, &best, &us);
  if (st != BFP_OK) {
    (void)bfp_chain_launch_set(op1, op2, f, &saved);
    return st;
  }
  st = bfp_chain_launch_set(op1, op2, f, &best);
  if (best_out) *best_out = best;
  if (best_us_out) *best_us_out = us;
  return st;
}

extern "C" bfp_status bfp_autotune_int(int op, int k, int kind, uint64_t n_probe, int reps, void* stream,
                                       bfp_launch* best_out, double* best_us_out) {
  bfp_launch saved;
  bfp_status st = bfp_int_launch_get(op, k, kind, &saved);
  if (st != BFP_OK) return st;
  if (n_probe == 0 || n_probe > (1ull << 30) || reps < 1 || reps > 1000) return BFP_E_ARG;
  hipStream_t s = (hipStream_t)stream;
  const size_t vec_bytes = bfp_int_bitslice_bytes(k, n_probe);
  DevBuf a, b, c, sweep, sink;
  if (hipMalloc(&a.p, vec_bytes) != hipSuccess || hipMalloc(&b.p, vec_bytes) != hipSuccess ||
      hipMalloc(&c.p, vec_bytes) != hipSuccess || hipMalloc(&sweep.p, 512ull << 20) != hipSuccess ||
      hipMalloc(&sink.p, 256) != hipSuccess)
    return BFP_E_NOMEM;
  hipLaunchKernelGGL(k_fill_random, dim3(2048), dim3(256), 0, s, (uint32_t*)a.p, vec_bytes / 4, 0x1234u);
  hipLaunchKernelGGL(k_fill_random, dim3(2048), dim3(256), 0, s, (uint32_t*)b.p, vec_bytes / 4, 0x9876u);
  hipLaunchKernelGGL(k_fill_random, dim3(2048), dim3(256), 0, s, (uint32_t*)sweep.p, (512ull << 20) / 4, 0x5555u);
  if (hipGetLastError() != hipSuccess) return BFP_E_HIP;
  bfp_launch best = saved;
  double us = 0;
  st = tune_block_grid([&](const bfp_launch& cfg) { return bfp_int_launch_set(op, k, kind, &cfg); },
                       [&]() { return bfp_int_binop(op, k, kind, a.p, b.p, c.p, n_probe, stream); },
                       saved.words_per_lane, reps, s, sweep, sink, &best, &us);
  if (st != BFP_OK) {
    (void)bfp_int_launch_set(op, k, kind, &saved);
    return st;
  }
  st = bfp_int_launch_set(op, k, kind, &best);
  if (best_out) *best_out = best;
  if (best_us_out) *best_us_out = us;
  return st;
}

extern "C" bfp_status bfp_autotune_layout(int direction, bfp_format f, uint64_t n_probe, int reps, void* stream,
                                          int* best_method, double* best_us_out) {
  if (direction != 0 && direction != 1) return BFP_E_ARG;
  if (!bfp_format_supported(f)) return BFP_E_FORMAT;
  const int cb = (int)bfp_container_bytes(f);
  const int saved = bfp_layout_method_get(direction, cb);
  if (saved < 0) return saved;
  if (n_probe == 0 || n_probe > (1ull << 30) || reps < 1 || reps > 1000) return BFP_E_ARG;
  hipStream_t s = (hipStream_t)stream;
  const size_t bs_bytes = bfp_bitslice_bytes(f, n_probe), std_bytes = (size_t)n_probe * cb;
  DevBuf bs, sd, sweep, sink;
  if (hipMalloc(&bs.p, bs_bytes) != hipSuccess || hipMalloc(&sd.p, std_bytes + 16) != hipSuccess ||
      hipMalloc(&sweep.p, 512ull << 20) != hipSuccess || hipMalloc(&sink.p, 256) != hipSuccess)
    return BFP_E_NOMEM;
  hipLaunchKernelGGL(k_fill_random, dim3(2048), dim3(256), 0, s, (uint32_t*)sd.p, (std_bytes + 3) / 4, 0x1234u);
  hipLaunchKernelGGL(k_fill_random, dim3(2048), dim3(256), 0, s, (uint32_t*)sweep.p, (512ull << 20) / 4, 0x5555u);
  if (hipGetLastError() != hipSuccess) return BFP_E_HIP;
  bfp_status st = direction == 0 ? BFP_OK : bfp_pack(f, sd.p, bs.p, n_probe, stream);  // valid planes to unpack
  int best = saved;
  double best_us = 1e30;
  const int methods[2] = {BFP_TRANSPOSE_LANE, BFP_TRANSPOSE_XLANE};
  for (int meth : methods) {
    if (st != BFP_OK) break;
    if (cb == 8 && meth != BFP_TRANSPOSE_LANE) continue;
    st = bfp_layout_method_set(direction, cb, meth);
    double us = 0;
    if (st == BFP_OK)
      st = median_cold_us([&]() { return direction == 0 ? bfp_pack(f, sd.p, bs.p, n_probe, stream)
                                                        : bfp_unpack(f, bs.p, sd.p, n_probe, stream); },
                          reps, s, sweep, sink, &us);
    if (st == BFP_OK && us < best_us) {
      best_us = us;
      best = meth;
    }
  }
  if (st != BFP_OK) {
    (void)bfp_layout_method_set(direction, cb, saved);
    return st;
  }
  st = bfp_layout_method_set(direction, cb, best);
  if (best_method) *best_method = best;
  if (best_us_out) *best_us_out = best_us;
  return st;
}
