// host_check.cpp -- test driver built with AddressSanitizer and
// UndefinedBehaviorSanitizer: the oracle against the host build of the
// circuits (the GPU kernels' gate code compiled for the CPU) on random and
// special operands of every format and op, the integer vectors, the
// transposes against the oracle's pack, and a single-threaded fuzz of the
// serving scheduler through the host simulator.  Exits 0 when every
// comparison agrees and no sanitizer reports an error.
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

#include <random>
#include <vector>

extern "C" {
uint64_t oracle_op1_64(int op, int e, int m, int mode, uint64_t a, uint64_t b);
int oracle_int_binop(int op, int k, int kind, const uint32_t* a, const uint32_t* b, uint32_t* c, uint64_t n);
int oracle_pack(int B, int cbytes, const void* x, uint32_t* planes, uint64_t n, uint64_t gpad);
int bfpsim_binop(int op, int e, int m, int mode, int wbits, const uint32_t* a, const uint32_t* b, uint32_t* c,
                 uint64_t n);
int bfpsim_binop64(int op, int e, int m, int mode, int wbits, const uint64_t* a, const uint64_t* b, uint64_t* c,
                   uint64_t n);
int bfpsim_int_binop(int op, int k, int kind, int wbits, const uint32_t* a, const uint32_t* b, uint32_t* c,
                     uint64_t n);
int bfpsim_transpose(int C, int inverse, const uint32_t* in, uint32_t* out);
void* simsrv_create(uint64_t budget, int slots);
void simsrv_destroy(void* p);
uint64_t simsrv_put(void* p, uint64_t bytes, uint64_t n);
int simsrv_free(void* p, uint64_t h);
int64_t simsrv_submit(void* p, uint64_t a, uint64_t b, uint64_t n, uint64_t c_bytes);
int simsrv_cancel(void* p, uint64_t id);
int simsrv_step(void* p);
void simsrv_release(void* p, int k);
int simsrv_take(void* p, uint64_t* ids, uint64_t* handles, int32_t* status, int max);
}

static int failures = 0;
static int formats_run = 0, ints_run = 0;
#define CHECK(c, ...)                      \
  do {                                     \
    if (!(c)) {                            \
      if (failures++ < 20) {               \
        fprintf(stderr, __VA_ARGS__);      \
        fprintf(stderr, "\n");             \
      }                                    \
    }                                      \
  } while (0)

static void formats_vs_oracle(std::mt19937_64& rng) {
  const int es[5] = {3, 4, 5, 6, 8}, ms[8] = {1, 2, 3, 5, 7, 10, 15, 23};
  const int n = 256;
  std::vector<uint32_t> a(n), b(n), c(n);
  for (int e : es)
    for (int m : ms) {
      const int B = 1 + e + m;
      const uint64_t mask = B == 64 ? ~0ull : ((1ull << B) - 1);
      for (int i = 0; i < n; ++i) {
        a[i] = (uint32_t)(rng() & mask);
        b[i] = (uint32_t)(rng() & mask);
      }
      a[0] = 0;  // zeros, infinities and a NaN among the operands
      b[1] = 0;
      a[2] = (uint32_t)(((1ull << e) - 1) << m);
      b[3] = (uint32_t)((((1ull << e) - 1) << m) | 1);
      for (int op = 0; op < 4; ++op)
        for (int mode = 0; mode < 2; ++mode)
          for (int wbits : {32, 64}) {
            if (bfpsim_binop(op, e, m, mode, wbits, a.data(), b.data(), c.data(), n) != 0) continue;  // not built
            formats_run++;
            for (int i = 0; i < n; ++i) {
              const uint64_t want = oracle_op1_64(op, e, m, mode, a[i], b[i]);
              CHECK(c[i] == want, "(%d,%d) op %d mode %d w%d: %x op %x = %x, oracle %llx", e, m, op, mode, wbits,
                    a[i], b[i], c[i], (unsigned long long)want);
            }
          }
    }
  const int wide[4][2] = {{8, 31}, {11, 20}, {11, 40}, {11, 52}};
  std::vector<uint64_t> a6(64), b6(64), c6(64);
  for (auto& f : wide) {
    const int e = f[0], m = f[1], B = 1 + e + m;
    const uint64_t mask = B == 64 ? ~0ull : ((1ull << B) - 1);
    for (int i = 0; i < 64; ++i) {
      a6[i] = rng() & mask;
      b6[i] = rng() & mask;
    }
    for (int op = 0; op < 4; ++op)
      for (int mode = 0; mode < 2; ++mode) {
        if (bfpsim_binop64(op, e, m, mode, 32, a6.data(), b6.data(), c6.data(), 64) != 0) continue;
        formats_run++;
        for (int i = 0; i < 64; ++i)
          CHECK(c6[i] == oracle_op1_64(op, e, m, mode, a6[i], b6[i]), "wide (%d,%d) op %d", e, m, op);
      }
  }
}

static void ints_vs_oracle(std::mt19937_64& rng) {
  const int n = 200;
  std::vector<uint32_t> a(n), b(n), c(n), w(n);
  for (int k = 1; k <= 32; ++k) {
    const uint32_t mask = k == 32 ? 0xFFFFFFFFu : ((1u << k) - 1);
    for (int i = 0; i < n; ++i) {
      a[i] = (uint32_t)rng() & mask;
      b[i] = (uint32_t)rng() & mask;
    }
    for (int op = 0; op < 3; ++op)
      for (int kind = 0; kind < 3; ++kind) {
        CHECK(oracle_int_binop(op, k, kind, a.data(), b.data(), w.data(), n) == 0, "oracle int");
        if (bfpsim_int_binop(op, k, kind, 32, a.data(), b.data(), c.data(), n) != 0) continue;
        ints_run++;
        for (int i = 0; i < n; ++i) CHECK(c[i] == w[i], "int k %d op %d kind %d", k, op, kind);
      }
  }
}

static void transposes_vs_oracle(std::mt19937_64& rng) {
  for (int C : {1, 2, 4}) {
    std::vector<uint8_t> x(32 * C);
    for (auto& v : x) v = (uint8_t)rng();
    std::vector<uint32_t> in(8 * C), planes(8 * C), back(8 * C), want(8 * C * 64, 0);
    for (int i = 0; i < 8 * C; ++i) in[i] = (uint32_t)x[4 * i] | (uint32_t)x[4 * i + 1] << 8 |
                                             (uint32_t)x[4 * i + 2] << 16 | (uint32_t)x[4 * i + 3] << 24;
    CHECK(bfpsim_transpose(C, 0, in.data(), planes.data()) == 0, "transpose");
    CHECK(oracle_pack(8 * C, C, x.data(), want.data(), 32, 64) == 0, "oracle pack");
    for (int k = 0; k < 8 * C; ++k) CHECK(planes[k] == want[(size_t)k * 64], "pack C %d plane %d", C, k);
    CHECK(bfpsim_transpose(C, 1, planes.data(), back.data()) == 0, "untranspose");
    for (int i = 0; i < 8 * C; ++i) CHECK(back[i] == in[i], "unpack C %d word %d", C, i);
  }
}

static void scheduler_fuzz(std::mt19937_64& rng) {
  void* s = simsrv_create(1 << 22, 16);
  std::vector<uint64_t> live;
  uint64_t ids[64], hs[64];
  int32_t st[64];
  for (int it = 0; it < 20000; ++it) {
    const unsigned x = (unsigned)(rng() % 100);
    if (x < 25 || live.empty()) {
      const uint64_t h = simsrv_put(s, 256 * (1 + rng() % 32), 1 + rng() % 4000);
      if (h) live.push_back(h);
    } else if (x < 40) {
      const size_t i = rng() % live.size();
      CHECK(simsrv_free(s, live[i]) == 0, "free");
      live.erase(live.begin() + i);
    } else if (x < 75) {
      const uint64_t a = live[rng() % live.size()], b = live[rng() % live.size()];
      (void)simsrv_submit(s, a, b, 1, 256 * (1 + rng() % 8));
    } else if (x < 80) {
      (void)simsrv_cancel(s, 1 + rng() % 5000);
    } else {
      simsrv_release(s, (int)(rng() % 3));
    }
    simsrv_step(s);
    const int k = simsrv_take(s, ids, hs, st, 64);
    for (int i = 0; i < k; ++i)
      if (st[i] == 0) CHECK(simsrv_free(s, hs[i]) == 0, "free result");
  }
  simsrv_destroy(s);
}

int main() {
  std::mt19937_64 rng(12345);
  formats_vs_oracle(rng);
  ints_vs_oracle(rng);
  transposes_vs_oracle(rng);
  scheduler_fuzz(rng);
  if (failures) {
    fprintf(stderr, "%d failures\n", failures);
    return 1;
  }
  printf("host_check ok: %d format/op/mode/word cases, %d integer cases\n", formats_run, ints_run);
  return 0;
}
