// bfp_runtime.hip -- the C ABI of include/bfp.h: argument checks, dispatch
// to the compiled kernel variants, launch configuration table.
#include <hip/hip_runtime.h>

#include <mutex>
#include <stdio.h>
#include <string.h>

#include "bfp.h"
#include "bfp_formats.hpp"
#include "bfp_int_kernels.hpp"
#include "bfp_kernels.hpp"
#include "bfp_layout.hpp"
#include "bfp_xlane.hpp"

namespace bfp {

Registry& registry() {
  static Registry r;
  return r;
}

namespace {

// Elements per vector are limited so that a lane's byte offset inside one
// plane fits in 32 bits (planes of at most 2^32 bytes).
constexpr uint64_t kMaxN = 1ull << 36;

bool format_ok(const bfp_format& f) {
  if (f.pad != 0 || (f.round != BFP_RNE && f.round != BFP_RZ)) return false;
  if (f.e < 2 || f.e > kMaxE || f.m < 1 || f.m > kMaxM) return false;
  return registry().binop[f.e][f.m][0][0][0][0] != nullptr;
}

int bits_of(const bfp_format& f) { return 1 + f.e + f.m; }
int cbytes_of(const bfp_format& f) {
  const int B = bits_of(f);
  return B <= 8 ? 1 : (B <= 16 ? 2 : (B <= 32 ? 4 : 8));
}
bool aligned16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }
bool overlap(const void* a, size_t na, const void* b, size_t nb) {
  const uintptr_t a0 = reinterpret_cast<uintptr_t>(a), b0 = reinterpret_cast<uintptr_t>(b);
  return a0 < b0 + nb && b0 < a0 + na;
}

// Compute units of the current device (cached per device).
int cu_count() {
  static int cache[64] = {0};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
  if (cache[dev] == 0) {
    hipDeviceProp_t p;
    if (hipGetDeviceProperties(&p, dev) != hipSuccess) return 256;
    cache[dev] = p.multiProcessorCount > 0 ? p.multiProcessorCount : 256;
  }
  return cache[dev];
}

unsigned grid_for(uint64_t items, int block, int blocks_per_cu) {
  uint64_t g = (items + block - 1) / block;
  if (blocks_per_cu > 0) {
    const uint64_t cap = (uint64_t)cu_count() * blocks_per_cu;
    if (g > cap) g = cap;
  }
  if (g < 1) g = 1;
  if (g > 0x7FFFFFFFull) g = 0x7FFFFFFFull;
  return (unsigned)g;
}

// Launch configuration table: [opclass][e][m][round]
std::mutex g_cfg_mu;
bfp_launch g_cfg[kOpClasses][kMaxE + 1][kMaxM + 1][2];
bool g_cfg_init = false;

// Defaults before tuning (measured on MI355X at 2^26 elements): circuits
// that move more bytes than they compute run best with 64-element lane words
// (two dwords per lane per plane); 8-bit formats with 32-element words in
// blocks of 128; circuits with many gates per bit (VALU-bound) with 32.
void cfg_init_locked() {
  if (g_cfg_init) return;
  for (int o = 0; o < kOpClasses; ++o)
    for (int e = 0; e <= kMaxE; ++e)
      for (int m = 0; m <= kMaxM; ++m)
        for (int r = 0; r < 2; ++r) {
          bfp_launch& c = g_cfg[o][e][m][r];
          const int B = 1 + e + m;
          const bool valu_heavy = (o == 1 && m >= 15) || (o == 2 && m >= 10);
          const bool one_word_only = !registry().binop[e][m][o][r][1][0];
          c.words_per_lane = (B <= 8 || valu_heavy || one_word_only) ? 1 : 2;
          c.block = B <= 8 ? 128 : 256;  // within every format's max_block
          c.blocks_per_cu = 0;
          c.unroll = 1;
        }
  g_cfg_init = true;
}

// Chain kernels [e][m][opclass 1][opclass 2][round] and integer kernels
// [k][op][kind]: block and grid depth (their words per lane are fixed).
bfp_launch g_chain_cfg[kMaxE + 1][kMaxM + 1][2][2][2];
bfp_launch g_int_cfg[kMaxIntBits + 1][3][3];
bool g_aux_init = false;

void aux_init_locked() {
  if (g_aux_init) return;
  for (auto& a : g_chain_cfg)
    for (auto& b : a)
      for (auto& c : b)
        for (auto& d : c)
          for (auto& x : d) x = bfp_launch{1, 256, 0, 1};
  for (int k = 0; k <= kMaxIntBits; ++k)
    for (int o = 0; o < 3; ++o)
      for (int kd = 0; kd < 3; ++kd) g_int_cfg[k][o][kd] = bfp_launch{int_registry().words[k][o], 256, 0, 1};
  g_aux_init = true;
}

bfp_launch cfg_get(int opc, const bfp_format& f) {
  std::lock_guard<std::mutex> lk(g_cfg_mu);
  cfg_init_locked();
  return g_cfg[opc][f.e][f.m][f.round];
}

bool cfg_valid(const bfp_launch& c) {
  if (c.unroll < 0 || c.unroll > 2) return false;
  if (c.words_per_lane != 1 && c.words_per_lane != 2 && c.words_per_lane != 4) return false;
  if (c.block != 64 && c.block != 128 && c.block != 256 && c.block != 512) return false;
  if (c.blocks_per_cu < 0 || c.blocks_per_cu > 64) return false;
  return true;
}

bfp_status hip_status(hipError_t e) { return e == hipSuccess ? BFP_OK : BFP_E_HIP; }

typedef hipError_t (*PackLauncher)(const void*, void*, uint64_t, uint64_t, int, unsigned, unsigned, hipStream_t);

template <int C>
hipError_t launch_pack(const void* src, void* dst, uint64_t n, uint64_t gpad, int B, unsigned grid,
                       unsigned block, hipStream_t s) {
  const size_t lds = (size_t)(block / 64) * 2048 * C;
  hipLaunchKernelGGL((k_pack<C>), dim3(grid), dim3(block), lds, s, static_cast<const uint8_t*>(src),
                     static_cast<uint32_t*>(dst), n, gpad, B);
  return hipGetLastError();
}
template <int C>
hipError_t launch_unpack(const void* src, void* dst, uint64_t n, uint64_t gpad, int B, unsigned grid,
                         unsigned block, hipStream_t s) {
  const size_t lds = (size_t)(block / 64) * 2048 * C;
  hipLaunchKernelGGL((k_unpack<C>), dim3(grid), dim3(block), lds, s, static_cast<const uint32_t*>(src),
                     static_cast<uint8_t*>(dst), n, gpad, B);
  return hipGetLastError();
}

template <int C>
hipError_t launch_pack_x(const void* src, void* dst, uint64_t n, uint64_t gpad, int B, unsigned grid, unsigned block,
                         hipStream_t s) {
  const size_t lds = (size_t)(block / 64) * 32 * kXlaneRow * 4;
  hipLaunchKernelGGL((k_pack_x<C>), dim3(grid), dim3(block), lds, s, static_cast<const uint8_t*>(src),
                     static_cast<uint32_t*>(dst), n, gpad, B);
  return hipGetLastError();
}
template <int C>
hipError_t launch_unpack_x(const void* src, void* dst, uint64_t n, uint64_t gpad, int B, unsigned grid,
                           unsigned block, hipStream_t s) {
  const size_t lds = (size_t)(block / 64) * 32 * kXlaneRow * 4;
  hipLaunchKernelGGL((k_unpack_x<C>), dim3(grid), dim3(block), lds, s, static_cast<const uint32_t*>(src),
                     static_cast<uint8_t*>(dst), n, gpad, B);
  return hipGetLastError();
}

// Transpose method of pack [0] and unpack [1] per container size (1, 2, 4
// bytes): BFP_TRANSPOSE_LANE or BFP_TRANSPOSE_XLANE; 8-byte containers have
// the per-lane method only.
int g_layout_method[2][3] = {};
int cidx(int C) { return C == 1 ? 0 : (C == 2 ? 1 : (C == 4 ? 2 : -1)); }
int layout_method(int dir, int C) {
  const int ci = cidx(C);
  if (ci < 0) return BFP_TRANSPOSE_LANE;
  std::lock_guard<std::mutex> lk(g_cfg_mu);
  return g_layout_method[dir][ci];
}

bfp_status check_op(int op) { return op_valid(op) ? BFP_OK : BFP_E_OP; }

// Ops a two-op chain accepts: add, sub, mul (division is not chained).
bool chain_op_ok(int op) { return op == BFP_ADD || op == BFP_SUB || op == BFP_MUL; }

// d = (a op1 b) op2 c; a == nullptr broadcasts the pattern alpha.
bfp_status chain_impl(int op1, int op2, bfp_format f, const void* a, uint32_t alpha, const void* b, const void* c,
                      void* d, uint64_t n, void* stream) {
  if (!chain_op_ok(op1) || !chain_op_ok(op2)) return BFP_E_OP;
  if (!format_ok(f)) return BFP_E_FORMAT;
  ChainLauncher L = registry().chain[f.e][f.m][opclass_of(op1)][opclass_of(op2)][f.round];
  if (!L) return BFP_E_FORMAT;  // the wide formats have no chain kernels
  if (n == 0) return BFP_OK;
  if (n > kMaxN) return BFP_E_ARG;
  if (!b || !c || !d) return BFP_E_NULL;
  if ((a && !aligned16(a)) || !aligned16(b) || !aligned16(c) || !aligned16(d)) return BFP_E_ALIGN;
  const uint64_t gpad = gpad_of(n);
  const size_t bytes = (size_t)bits_of(f) * gpad * 4;
  const void* in[3] = {a, b, c};
  for (const void* p : in)
    if (p && p != d && overlap(d, bytes, p, bytes)) return BFP_E_ALIAS;
  bfp_launch cfg;
  {
    std::lock_guard<std::mutex> lk(g_cfg_mu);
    aux_init_locked();
    cfg = g_chain_cfg[f.e][f.m][opclass_of(op1)][opclass_of(op2)][f.round];
  }
  const unsigned block = (unsigned)cfg.block;
  const unsigned grid = grid_for(gpad, (int)block, cfg.blocks_per_cu);
  const uint32_t alpha_b = alpha & (uint32_t)((1ull << bits_of(f)) - 1u);
  const uint32_t negb1 = op1 == BFP_SUB ? 0xFFFFFFFFu : 0u, negb2 = op2 == BFP_SUB ? 0xFFFFFFFFu : 0u;
  return hip_status(L(a, alpha_b, b, c, d, gpad, n, negb1, negb2, grid, block, (hipStream_t)stream));
}

}  // namespace
}  // namespace bfp

using namespace bfp;

extern "C" {

const char* bfp_status_string(bfp_status s) {
  switch (s) {
    case BFP_OK: return "ok";
    case BFP_E_FORMAT: return "unsupported format (e, m) or rounding mode";
    case BFP_E_NULL: return "null pointer";
    case BFP_E_ALIGN: return "pointer not 16-byte aligned";
    case BFP_E_OP: return "unknown operation";
    case BFP_E_HIP: return "HIP runtime error";
    case BFP_E_ARG: return "invalid argument";
    case BFP_E_ALIAS: return "input and output overlap";
    case BFP_E_BUDGET: return "memory budget exceeded";
    case BFP_E_NOMEM: return "out of memory";
    case BFP_E_NODEV: return "no usable device";
    default: return "unknown status";
  }
}

const char* bfp_version(void) { return "0.1.0"; }

int bfp_format_supported(bfp_format f) { return format_ok(f) ? 1 : 0; }

size_t bfp_container_bytes(bfp_format f) { return format_ok(f) ? (size_t)cbytes_of(f) : 0; }

uint64_t bfp_plane_stride_words(uint64_t n) { return gpad_of(n); }

size_t bfp_bitslice_bytes(bfp_format f, uint64_t n) {
  if (!format_ok(f)) return 0;
  return (size_t)bits_of(f) * gpad_of(n) * 4u;
}

}  // extern "C"

namespace bfp {
namespace {

int cbytes_of_bits(int B) { return B <= 8 ? 1 : (B <= 16 ? 2 : (B <= 32 ? 4 : 8)); }

// Standard containers <-> B planes, 1 <= B <= 32 (format checked by the caller).
bfp_status pack_impl(int B, const void* std_in, void* bs_out, uint64_t n, void* stream) {
  if (n == 0) return BFP_OK;
  if (n > kMaxN) return BFP_E_ARG;
  if (!std_in || !bs_out) return BFP_E_NULL;
  if (!aligned16(std_in) || !aligned16(bs_out)) return BFP_E_ALIGN;
  const int C = cbytes_of_bits(B);
  const uint64_t gpad = gpad_of(n);
  if (overlap(std_in, n * C, bs_out, (size_t)B * gpad * 4)) return BFP_E_ALIAS;
  const int block = 256;
  const unsigned grid = grid_for(gpad, block, 0);
  PackLauncher L = C == 1 ? launch_pack<1> : (C == 2 ? launch_pack<2> : (C == 4 ? launch_pack<4> : launch_pack<8>));
  if (layout_method(0, C) == BFP_TRANSPOSE_XLANE)
    L = C == 1 ? launch_pack_x<1> : (C == 2 ? launch_pack_x<2> : launch_pack_x<4>);
  return hip_status(L(std_in, bs_out, n, gpad, B, grid, block, (hipStream_t)stream));
}

bfp_status unpack_impl(int B, const void* bs_in, void* std_out, uint64_t n, void* stream) {
  if (n == 0) return BFP_OK;
  if (n > kMaxN) return BFP_E_ARG;
  if (!bs_in || !std_out) return BFP_E_NULL;
  if (!aligned16(bs_in) || !aligned16(std_out)) return BFP_E_ALIGN;
  const int C = cbytes_of_bits(B);
  const uint64_t gpad = gpad_of(n);
  if (overlap(std_out, n * C, bs_in, (size_t)B * gpad * 4)) return BFP_E_ALIAS;
  const int block = 256;
  const uint64_t tiles = ((n + 31) / 32 + 63) / 64;  // 64 groups per wave tile
  const unsigned grid = grid_for(tiles * 64, block, 0);
  PackLauncher L =
      C == 1 ? launch_unpack<1> : (C == 2 ? launch_unpack<2> : (C == 4 ? launch_unpack<4> : launch_unpack<8>));
  if (layout_method(1, C) == BFP_TRANSPOSE_XLANE)
    L = C == 1 ? launch_unpack_x<1> : (C == 2 ? launch_unpack_x<2> : launch_unpack_x<4>);
  return hip_status(L(bs_in, std_out, n, gpad, B, grid, block, (hipStream_t)stream));
}

bool int_bits_ok(int k) { return k >= 1 && k <= kMaxIntBits && int_registry().op[k][0][0] != nullptr; }

}  // namespace

IntRegistry& int_registry() {
  static IntRegistry r;
  return r;
}

}  // namespace bfp

extern "C" {

bfp_status bfp_pack(bfp_format f, const void* std_in, void* bs_out, uint64_t n, void* stream) {
  if (!format_ok(f)) return BFP_E_FORMAT;
  return pack_impl(bits_of(f), std_in, bs_out, n, stream);
}

bfp_status bfp_unpack(bfp_format f, const void* bs_in, void* std_out, uint64_t n, void* stream) {
  if (!format_ok(f)) return BFP_E_FORMAT;
  return unpack_impl(bits_of(f), bs_in, std_out, n, stream);
}

size_t bfp_int_container_bytes(int k) { return int_bits_ok(k) ? (size_t)cbytes_of_bits(k) : 0; }

size_t bfp_int_bitslice_bytes(int k, uint64_t n) { return int_bits_ok(k) ? (size_t)k * gpad_of(n) * 4u : 0; }

bfp_status bfp_int_pack(int k, const void* std_in, void* bs_out, uint64_t n, void* stream) {
  if (!int_bits_ok(k)) return BFP_E_FORMAT;
  return pack_impl(k, std_in, bs_out, n, stream);
}

bfp_status bfp_int_unpack(int k, const void* bs_in, void* std_out, uint64_t n, void* stream) {
  if (!int_bits_ok(k)) return BFP_E_FORMAT;
  return unpack_impl(k, bs_in, std_out, n, stream);
}

bfp_status bfp_int_binop(int op, int k, int kind, const void* a, const void* b, void* c, uint64_t n,
                         void* stream) {
  if (op != BFP_ADD && op != BFP_SUB && op != BFP_MUL) return BFP_E_OP;
  if (!int_bits_ok(k) || kind < BFP_INT_WRAP || kind > BFP_INT_SAT_S) return BFP_E_FORMAT;
  if (n == 0) return BFP_OK;
  if (n > kMaxN) return BFP_E_ARG;
  if (!a || !b || !c) return BFP_E_NULL;
  if (!aligned16(a) || !aligned16(b) || !aligned16(c)) return BFP_E_ALIGN;
  const uint64_t gpad = gpad_of(n);
  const size_t bytes = (size_t)k * gpad * 4;
  if ((c != a && overlap(c, bytes, a, bytes)) || (c != b && overlap(c, bytes, b, bytes))) return BFP_E_ALIAS;
  IntLauncher L = int_registry().op[k][op][kind];
  if (!L) return BFP_E_FORMAT;
  bfp_launch cfg;
  {
    std::lock_guard<std::mutex> lk(g_cfg_mu);
    aux_init_locked();
    cfg = g_int_cfg[k][op][kind];
  }
  const unsigned grid = grid_for(gpad / cfg.words_per_lane, cfg.block, cfg.blocks_per_cu);
  return hip_status(L(a, b, c, gpad, grid, (unsigned)cfg.block, (hipStream_t)stream));
}

bfp_status bfp_binop(int op, bfp_format f, const void* a, const void* b, void* c, uint64_t n, void* stream) {
  bfp_status st = check_op(op);
  if (st != BFP_OK) return st;
  if (!format_ok(f)) return BFP_E_FORMAT;
  if (n == 0) return BFP_OK;
  if (n > kMaxN) return BFP_E_ARG;
  if (!a || !b || !c) return BFP_E_NULL;
  if (!aligned16(a) || !aligned16(b) || !aligned16(c)) return BFP_E_ALIGN;
  const uint64_t gpad = gpad_of(n);
  const size_t bytes = (size_t)bits_of(f) * gpad * 4;
  if ((c != a && overlap(c, bytes, a, bytes)) || (c != b && overlap(c, bytes, b, bytes))) return BFP_E_ALIAS;
  const int opc = opclass_of(op);
  const bfp_launch cfg = cfg_get(opc, f);
  const int U = cfg.unroll > 1 ? 2 : 1;
  BinopLauncher L = registry().binop[f.e][f.m][opc][f.round][r_index(cfg.words_per_lane)][U - 1];
  if (!L) return BFP_E_FORMAT;
  const uint64_t units = gpad / cfg.words_per_lane;
  const unsigned grid = grid_for((units + U - 1) / U, cfg.block, cfg.blocks_per_cu);
  const uint32_t negb = op == BFP_SUB ? 0xFFFFFFFFu : 0u;
  return hip_status(L(a, b, c, gpad, n, negb, grid, (unsigned)cfg.block, (hipStream_t)stream));
}

bfp_status bfp_add(bfp_format f, const void* a, const void* b, void* c, uint64_t n, void* stream) {
  return bfp_binop(BFP_ADD, f, a, b, c, n, stream);
}
bfp_status bfp_sub(bfp_format f, const void* a, const void* b, void* c, uint64_t n, void* stream) {
  return bfp_binop(BFP_SUB, f, a, b, c, n, stream);
}
bfp_status bfp_mul(bfp_format f, const void* a, const void* b, void* c, uint64_t n, void* stream) {
  return bfp_binop(BFP_MUL, f, a, b, c, n, stream);
}
bfp_status bfp_div(bfp_format f, const void* a, const void* b, void* c, uint64_t n, void* stream) {
  return bfp_binop(BFP_DIV, f, a, b, c, n, stream);
}

bfp_status bfp_chain2(int op1, int op2, bfp_format f, const void* a, const void* b, const void* c, void* d,
                      uint64_t n, void* stream) {
  if (!a && n > 0) return BFP_E_NULL;
  return chain_impl(op1, op2, f, a, 0u, b, c, d, n, stream);
}

bfp_status bfp_axpy(bfp_format f, uint32_t alpha, const void* x, const void* y, void* d, uint64_t n,
                    void* stream) {
  return chain_impl(BFP_MUL, BFP_ADD, f, nullptr, alpha, x, y, d, n, stream);
}

bfp_status bfp_binop_std(int op, bfp_format f, const void* a, const void* b, void* c, uint64_t n,
                         void* stream) {
  bfp_status st = check_op(op);
  if (st != BFP_OK) return st;
  if (!format_ok(f)) return BFP_E_FORMAT;
  if (n == 0) return BFP_OK;
  if (n > kMaxN) return BFP_E_ARG;
  if (!a || !b || !c) return BFP_E_NULL;
  if (!aligned16(a) || !aligned16(b) || !aligned16(c)) return BFP_E_ALIGN;
  const size_t bytes = (size_t)n * cbytes_of(f);
  if ((c != a && overlap(c, bytes, a, bytes)) || (c != b && overlap(c, bytes, b, bytes))) return BFP_E_ALIAS;
  StdLauncher L = registry().std_op[f.e][f.m][opclass_of(op)][f.round];
  if (!L) return BFP_E_FORMAT;
  // one 32-element group per lane, 256-thread blocks (for 65,536 elements,
  // 32 blocks of one wave measured no faster than 8 blocks of four: the
  // kernel is bound by one lane's chain of loads, circuit and stores)
  const int block = 256;
  const unsigned grid = grid_for((n + 31) / 32, block, 0);
  const uint32_t negb = op == BFP_SUB ? 0xFFFFFFFFu : 0u;
  return hip_status(L(a, b, c, n, negb, grid, block, (hipStream_t)stream));
}

bfp_status bfp_launch_get(int op, bfp_format f, bfp_launch* out) {
  bfp_status st = check_op(op);
  if (st != BFP_OK) return st;
  if (!format_ok(f)) return BFP_E_FORMAT;
  if (!out) return BFP_E_NULL;
  *out = cfg_get(opclass_of(op), f);
  return BFP_OK;
}

bfp_status bfp_launch_set(int op, bfp_format f, const bfp_launch* cfg) {
  bfp_status st = check_op(op);
  if (st != BFP_OK) return st;
  if (!format_ok(f)) return BFP_E_FORMAT;
  if (!cfg) return BFP_E_NULL;
  if (!cfg_valid(*cfg)) return BFP_E_ARG;
  // the wide formats have one-word kernels only, compiled for blocks of at most 256
  if (!registry().binop[f.e][f.m][opclass_of(op)][f.round][r_index(cfg->words_per_lane)]
                       [cfg->unroll > 1 ? 1 : 0])
    return BFP_E_ARG;
  if (cfg->block > registry().max_block[f.e][f.m]) return BFP_E_ARG;
  std::lock_guard<std::mutex> lk(g_cfg_mu);
  cfg_init_locked();
  g_cfg[opclass_of(op)][f.e][f.m][f.round] = *cfg;
  return BFP_OK;
}

bfp_status bfp_chain_launch_get(int op1, int op2, bfp_format f, bfp_launch* out) {
  if (!chain_op_ok(op1) || !chain_op_ok(op2)) return BFP_E_OP;
  if (!format_ok(f) || !registry().chain[f.e][f.m][0][0][0]) return BFP_E_FORMAT;
  if (!out) return BFP_E_NULL;
  std::lock_guard<std::mutex> lk(g_cfg_mu);
  aux_init_locked();
  *out = g_chain_cfg[f.e][f.m][opclass_of(op1)][opclass_of(op2)][f.round];
  return BFP_OK;
}

bfp_status bfp_chain_launch_set(int op1, int op2, bfp_format f, const bfp_launch* cfg) {
  if (!chain_op_ok(op1) || !chain_op_ok(op2)) return BFP_E_OP;
  if (!format_ok(f) || !registry().chain[f.e][f.m][0][0][0]) return BFP_E_FORMAT;
  if (!cfg) return BFP_E_NULL;
  if (!cfg_valid(*cfg) || cfg->words_per_lane != 1 || cfg->unroll > 1) return BFP_E_ARG;
  std::lock_guard<std::mutex> lk(g_cfg_mu);
  aux_init_locked();
  g_chain_cfg[f.e][f.m][opclass_of(op1)][opclass_of(op2)][f.round] = *cfg;
  return BFP_OK;
}

bfp_status bfp_int_launch_get(int op, int k, int kind, bfp_launch* out) {
  if (op != BFP_ADD && op != BFP_SUB && op != BFP_MUL) return BFP_E_OP;
  if (!int_bits_ok(k) || kind < BFP_INT_WRAP || kind > BFP_INT_SAT_S) return BFP_E_FORMAT;
  if (!out) return BFP_E_NULL;
  std::lock_guard<std::mutex> lk(g_cfg_mu);
  aux_init_locked();
  *out = g_int_cfg[k][op][kind];
  return BFP_OK;
}

bfp_status bfp_int_launch_set(int op, int k, int kind, const bfp_launch* cfg) {
  if (op != BFP_ADD && op != BFP_SUB && op != BFP_MUL) return BFP_E_OP;
  if (!int_bits_ok(k) || kind < BFP_INT_WRAP || kind > BFP_INT_SAT_S) return BFP_E_FORMAT;
  if (!cfg) return BFP_E_NULL;
  if (!cfg_valid(*cfg) || cfg->words_per_lane != int_registry().words[k][op] || cfg->unroll > 1) return BFP_E_ARG;
  std::lock_guard<std::mutex> lk(g_cfg_mu);
  aux_init_locked();
  g_int_cfg[k][op][kind] = *cfg;
  return BFP_OK;
}

bfp_status bfp_layout_method_set(int direction, int cbytes, int method) {
  if (direction != 0 && direction != 1) return BFP_E_ARG;
  if (method != BFP_TRANSPOSE_LANE && method != BFP_TRANSPOSE_XLANE) return BFP_E_ARG;
  const int ci = cidx(cbytes);
  if (ci < 0) return cbytes == 8 && method == BFP_TRANSPOSE_LANE ? BFP_OK : BFP_E_ARG;
  std::lock_guard<std::mutex> lk(g_cfg_mu);
  g_layout_method[direction][ci] = method;
  return BFP_OK;
}

int bfp_layout_method_get(int direction, int cbytes) {
  if ((direction != 0 && direction != 1) || (cidx(cbytes) < 0 && cbytes != 8)) return BFP_E_ARG;
  return layout_method(direction, cbytes);
}

bfp_status bfp_launch_load(const char* path) {
  if (!path) return BFP_E_NULL;
  FILE* fp = fopen(path, "r");
  if (!fp) return BFP_E_ARG;
  char line[256];
  bfp_status st = BFP_OK;
  while (fgets(line, sizeof line, fp)) {
    if (line[0] == '#' || line[0] == '\n') continue;
    if (line[0] == 'l') {  // "layout direction cbytes method"
      int dir, cb, meth;
      if (sscanf(line, "layout %d %d %d", &dir, &cb, &meth) != 3 || bfp_layout_method_set(dir, cb, meth) != BFP_OK) {
        st = BFP_E_ARG;
        break;
      }
      continue;
    }
    if (line[0] == 'c' || line[0] == 'i') {  // "chain op1 op2 e m round block bpc" / "int op k kind block bpc"
      int v[6] = {0};
      bfp_launch c{1, 256, 0, 1};
      bfp_status s2 = BFP_E_ARG;
      if (line[0] == 'c' && sscanf(line, "chain %d %d %d %d %d %d %d", &v[0], &v[1], &v[2], &v[3], &v[4], &c.block,
                                   &c.blocks_per_cu) == 7) {
        bfp_format f{(uint8_t)v[2], (uint8_t)v[3], (uint8_t)v[4], 0};
        if (!format_ok(f) || !registry().chain[f.e][f.m][0][0][0]) continue;
        s2 = bfp_chain_launch_set(v[0], v[1], f, &c);
      } else if (line[0] == 'i' && sscanf(line, "int %d %d %d %d %d", &v[0], &v[1], &v[2], &c.block,
                                          &c.blocks_per_cu) == 5) {
        if (!int_bits_ok(v[1]) || v[0] < 0 || v[0] > 2) continue;
        c.words_per_lane = int_registry().words[v[1]][v[0]];
        s2 = bfp_int_launch_set(v[0], v[1], v[2], &c);
      }
      if (s2 != BFP_OK) {
        st = s2;
        break;
      }
      continue;
    }
    int op, e, m, r, wpl, block, bpc, unroll = 1;
    const int got = sscanf(line, "%d %d %d %d %d %d %d %d", &op, &e, &m, &r, &wpl, &block, &bpc, &unroll);
    if (got != 7 && got != 8) {  // the unroll column may be absent (one unit per step)
      st = BFP_E_ARG;
      break;
    }
    bfp_format f;
    f.e = (uint8_t)e;
    f.m = (uint8_t)m;
    f.round = (uint8_t)r;
    f.pad = 0;
    if (e < 0 || e > 255 || m < 0 || m > 255 || !format_ok(f)) continue;
    bfp_launch c;
    c.words_per_lane = wpl;
    c.block = block;
    c.blocks_per_cu = bpc;
    c.unroll = unroll;
    const bfp_status s2 = bfp_launch_set(op, f, &c);
    if (s2 != BFP_OK) {
      st = s2;
      break;
    }
  }
  fclose(fp);
  return st;
}

bfp_status bfp_launch_save(const char* path) {
  if (!path) return BFP_E_NULL;
  FILE* fp = fopen(path, "w");
  if (!fp) return BFP_E_ARG;
  fprintf(fp, "# op e m round words_per_lane block blocks_per_cu unroll\n");
  {
    std::lock_guard<std::mutex> lk(g_cfg_mu);
    cfg_init_locked();
    for (int o = 0; o < kOpClasses; ++o)
      for (int e = 0; e <= kMaxE; ++e)
        for (int m = 0; m <= kMaxM; ++m)
          for (int r = 0; r < 2; ++r) {
            if (!registry().binop[e][m][0][0][0][0]) continue;
            const bfp_launch& c = g_cfg[o][e][m][r];
            const int op = o == 1 ? BFP_MUL : (o == 2 ? BFP_DIV : BFP_ADD);
            fprintf(fp, "%d %d %d %d %d %d %d %d\n", op, e, m, r, c.words_per_lane, c.block,
                    c.blocks_per_cu, c.unroll > 1 ? 2 : 1);
          }
    aux_init_locked();
    fprintf(fp, "# chain op1 op2 e m round block blocks_per_cu (op classes: 0 add/sub, 2 mul)\n");
    for (int e = 0; e <= kMaxE; ++e)
      for (int m = 0; m <= kMaxM; ++m) {
        if (!registry().chain[e][m][0][0][0]) continue;
        for (int o1 = 0; o1 < 2; ++o1)
          for (int o2 = 0; o2 < 2; ++o2)
            for (int r = 0; r < 2; ++r) {
              const bfp_launch& c = g_chain_cfg[e][m][o1][o2][r];
              fprintf(fp, "chain %d %d %d %d %d %d %d\n", o1 ? BFP_MUL : BFP_ADD, o2 ? BFP_MUL : BFP_ADD, e, m, r,
                      c.block, c.blocks_per_cu);
            }
      }
    fprintf(fp, "# layout direction(0 pack, 1 unpack) cbytes method(0 per lane, 1 across lanes)\n");
    for (int dir = 0; dir < 2; ++dir)
      for (int cb : {1, 2, 4}) fprintf(fp, "layout %d %d %d\n", dir, cb, g_layout_method[dir][cidx(cb)]);
    fprintf(fp, "# int op k kind block blocks_per_cu\n");
    for (int k = 1; k <= kMaxIntBits; ++k)
      for (int o = 0; o < 3; ++o)
        for (int kd = 0; kd < 3; ++kd) {
          if (!int_registry().op[k][o][kd]) continue;
          const bfp_launch& c = g_int_cfg[k][o][kd];
          fprintf(fp, "int %d %d %d %d %d\n", o, k, kd, c.block, c.blocks_per_cu);
        }
  }
  fclose(fp);
  return BFP_OK;
}

}  // extern "C"
