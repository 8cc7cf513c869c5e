/*
 * A plain C99 consumer of libbfp: it includes only include/bfp.h and the HIP
 * runtime's C API and links libbfp.so, with no Python and no C++ on its side
 * of the boundary.  The tests run it in two modes:
 *
 *   abi_consumer host
 *       Sizing, gate counts and status strings, no device call; prints one
 *       "key value" line each.
 *   abi_consumer run E M OP N IN OUT
 *       Reads N operand containers a, then N containers b (format (E, M),
 *       nearest-even) from file IN; on the device packs both, applies OP
 *       (add, sub, mul or div) to the bitslice vectors, unpacks into c, and
 *       runs the fused standard-in/standard-out op into d; writes c to OUT.
 *       Exits 3 if c and d differ, 1 on any library or runtime error.
 */
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <hip/hip_runtime_api.h>

#include "bfp.h"

static int fail(const char* what, int st) {
  fprintf(stderr, "%s failed: %d (%s)\n", what, st, st < 0 ? bfp_status_string(st) : "runtime");
  return 1;
}

static int op_code(const char* s) {
  if (!strcmp(s, "add")) return BFP_ADD;
  if (!strcmp(s, "sub")) return BFP_SUB;
  if (!strcmp(s, "mul")) return BFP_MUL;
  if (!strcmp(s, "div")) return BFP_DIV;
  return -1;
}

static int host_mode(void) {
  bfp_format f = {5, 10, BFP_RNE, 0};
  const uint64_t ns[4] = {1, 2048, 65000, 66000};
  int i;
  printf("version %s\n", bfp_version());
  printf("container_bytes_5_10 %u\n", (unsigned)bfp_container_bytes(f));
  for (i = 0; i < 4; ++i)
    printf("stride_%llu %llu\n", (unsigned long long)ns[i], (unsigned long long)bfp_plane_stride_words(ns[i]));
  printf("bitslice_bytes_5_10_65000 %llu\n", (unsigned long long)bfp_bitslice_bytes(f, 65000));
  printf("gates_add_5_10 %ld\n", bfp_gate_count(BFP_ADD, f));
  printf("gates_mul_5_10 %ld\n", bfp_gate_count(BFP_MUL, f));
  printf("format_7_4_supported %d\n", (int)bfp_format_supported((bfp_format){7, 4, BFP_RNE, 0}));
  printf("pack_bad_format %d\n", (int)bfp_pack((bfp_format){7, 4, BFP_RNE, 0}, NULL, NULL, 10, NULL));
  printf("status_null %s\n", bfp_status_string(BFP_E_NULL));
  return 0;
}

static int run_mode(int e, int m, const char* opname, uint64_t n, const char* in_path, const char* out_path) {
  const bfp_format f = {(uint8_t)e, (uint8_t)m, BFP_RNE, 0};
  const int op = op_code(opname);
  size_t cb, bs;
  unsigned char *ha = NULL, *hc = NULL, *hd = NULL;
  void *a = NULL, *b = NULL, *c = NULL, *d = NULL, *pa = NULL, *pb = NULL, *pc = NULL;
  FILE* fp;
  int rc = 1, st;
  if (op < 0 || !bfp_format_supported(f) || n == 0) return fail("arguments", BFP_E_ARG);
  cb = bfp_container_bytes(f);
  bs = bfp_bitslice_bytes(f, n);
  ha = malloc(2 * n * cb);
  hc = malloc(n * cb);
  hd = malloc(n * cb);
  if (!ha || !hc || !hd) return fail("malloc", BFP_E_NOMEM);
  fp = fopen(in_path, "rb");
  if (!fp || fread(ha, cb, 2 * n, fp) != 2 * n) {
    if (fp) fclose(fp);
    return fail("read input", BFP_E_ARG);
  }
  fclose(fp);
  if (hipMalloc(&a, n * cb) != hipSuccess || hipMalloc(&b, n * cb) != hipSuccess ||
      hipMalloc(&c, n * cb) != hipSuccess || hipMalloc(&d, n * cb) != hipSuccess ||
      hipMalloc(&pa, bs) != hipSuccess || hipMalloc(&pb, bs) != hipSuccess || hipMalloc(&pc, bs) != hipSuccess) {
    rc = fail("hipMalloc", BFP_E_NOMEM);
    goto done;
  }
  if (hipMemcpy(a, ha, n * cb, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(b, ha + n * cb, n * cb, hipMemcpyHostToDevice) != hipSuccess) {
    rc = fail("hipMemcpy in", BFP_E_HIP);
    goto done;
  }
  if ((st = bfp_pack(f, a, pa, n, NULL)) != BFP_OK || (st = bfp_pack(f, b, pb, n, NULL)) != BFP_OK) {
    rc = fail("bfp_pack", st);
    goto done;
  }
  if ((st = bfp_binop(op, f, pa, pb, pc, n, NULL)) != BFP_OK) {
    rc = fail("bfp_binop", st);
    goto done;
  }
  if ((st = bfp_unpack(f, pc, c, n, NULL)) != BFP_OK) {
    rc = fail("bfp_unpack", st);
    goto done;
  }
  if ((st = bfp_binop_std(op, f, a, b, d, n, NULL)) != BFP_OK) {
    rc = fail("bfp_binop_std", st);
    goto done;
  }
  if (hipDeviceSynchronize() != hipSuccess || hipMemcpy(hc, c, n * cb, hipMemcpyDeviceToHost) != hipSuccess ||
      hipMemcpy(hd, d, n * cb, hipMemcpyDeviceToHost) != hipSuccess) {
    rc = fail("hipMemcpy out", BFP_E_HIP);
    goto done;
  }
  fp = fopen(out_path, "wb");
  if (!fp || fwrite(hc, cb, n, fp) != n) {
    if (fp) fclose(fp);
    rc = fail("write output", BFP_E_ARG);
    goto done;
  }
  fclose(fp);
  rc = memcmp(hc, hd, n * cb) ? 3 : 0;
  if (rc) fprintf(stderr, "bitslice and fused results differ\n");
done:
  (void)hipFree(a);
  (void)hipFree(b);
  (void)hipFree(c);
  (void)hipFree(d);
  (void)hipFree(pa);
  (void)hipFree(pb);
  (void)hipFree(pc);
  free(ha);
  free(hc);
  free(hd);
  return rc;
}

int main(int argc, char** argv) {
  if (argc == 2 && !strcmp(argv[1], "host")) return host_mode();
  if (argc == 8 && !strcmp(argv[1], "run"))
    return run_mode(atoi(argv[2]), atoi(argv[3]), argv[4], strtoull(argv[5], NULL, 10), argv[6], argv[7]);
  fprintf(stderr, "usage: %s host | run E M OP N IN OUT\n", argv[0]);
  return 2;
}
