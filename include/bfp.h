/*
 * bfp.h -- C ABI of libbfp: bitslice custom-precision floating point on
 * AMD MI355X (gfx950).
 *
 * A custom format has 1 sign bit, e exponent bits and m mantissa bits
 * (B = 1 + e + m).  The paper offers its operations as intrinsic-style C
 * functions generated for one (exponent bits, mantissa bits, rounding mode)
 * configuration (Section 1 contributions; Section 5.1); here the same three
 * numbers are a runtime argument, `bfp_format`, and the library carries the
 * compiled circuits of every format e in {3,4,5,6,8} x m in
 * {1,2,3,5,7,10,15,23} and of the wide formats (8,31), (11,20), (11,40) and
 * (11,52) = binary64 (the wide formats have the elementwise and fused
 * standard ops, not the chain, batch and serving calls).  k-bit integer
 * vectors share the layout (see bfp_int_binop).
 *
 * Layouts (Section 2, Figure 1; Section 4, Figure 3):
 *   standard  one element per unsigned container of 1, 2, 4 or 8 bytes
 *             (B <= 8, <= 16, <= 32, <= 64), value in the low B bits: mantissa in
 *             bits [0,m), exponent in [m,m+e), sign in bit m+e.  Bits above B
 *             are ignored on input and written as zero on output.
 *   bitslice  B planes of G_pad 32-bit words each, plane k first
 *             (plane-major).  Plane k holds bit k of every element; element
 *             i sits in word i/32 of its plane at bit i%32.
 *             G_pad = bfp_plane_stride_words(n) = ceil(n/32) rounded up to a
 *             multiple of 64, plus 256 when that is a multiple of 2048: every
 *             plane starts 256-byte aligned, and plane strides that are
 *             multiples of 8 KiB (which send all planes of one word group to
 *             the same HBM channels) are avoided.  The layout is the same for
 *             any word width a kernel uses (32 or 64 elements per lane
 *             word).  Padding bits past element n are zero after bfp_pack
 *             and stay zero through every operation.
 *
 * Semantics: each result is the exact sum, difference, product or quotient
 * rounded once, to nearest with ties to even (BFP_RNE) or toward zero
 * (BFP_RZ) -- the two modes of Section 4.  Exponent bias 2^(e-1)-1; exponent field 0 holds
 * zero and subnormals; all ones holds Inf (mantissa 0) and NaN.  Overflow
 * gives Inf (RNE) or the largest finite value (RZ).  An exact zero sum of
 * opposite-signed operands is +0.  NaN results are the canonical quiet NaN
 * (sign 0, exponent all ones, mantissa 2^(m-1)); payloads do not propagate.
 * sub(a, b) = add(a, b with its sign flipped).
 *
 * Conventions common to every call:
 *   - Pointers named as device pointers are device memory (hipMalloc or a
 *     torch CUDA tensor's data pointer), 16-byte aligned, owned by the
 *     caller; calls never take ownership and op calls never allocate.
 *   - `stream` is a hipStream_t passed as void*; NULL is the null stream.
 *     Calls are asynchronous with respect to the host: they enqueue work and
 *     return.  A fault inside a kernel surfaces at the caller's next
 *     synchronisation of that stream.
 *   - n == 0 is a no-op that returns BFP_OK.
 *   - Errors are returned as negative bfp_status codes; nothing aborts and no
 *     C++ exception crosses this interface.
 *   - The library is thread-safe; the launch-configuration table is guarded
 *     by a lock.
 */
#ifndef BFP_H
#define BFP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int bfp_status;

#define BFP_OK 0
#define BFP_E_FORMAT (-1)   /* (e, m) not compiled, or round not RNE/RZ */
#define BFP_E_NULL (-2)     /* null pointer with n > 0 */
#define BFP_E_ALIGN (-3)    /* pointer not 16-byte aligned */
#define BFP_E_OP (-4)       /* op not BFP_ADD/BFP_SUB/BFP_MUL/BFP_DIV */
#define BFP_E_HIP (-5)      /* HIP runtime error on launch */
#define BFP_E_ARG (-6)      /* other invalid argument (size, count, handle) */
#define BFP_E_ALIAS (-7)    /* forbidden overlap of input and output */
#define BFP_E_BUDGET (-8)   /* serving: memory budget exceeded */
#define BFP_E_NOMEM (-9)    /* host or device allocation failed */
#define BFP_E_NODEV (-10)   /* no usable gfx950 device */
#define BFP_E_CANCELLED (-11) /* serving: request withdrawn by bfp_server_cancel */
#define BFP_E_TIMEOUT (-12) /* serving: request not launched within the queue timeout */
#define BFP_E_BUSY (-13)    /* serving: request already on the device */

#define BFP_RNE 0 /* round to nearest, ties to even (Section 4) */
#define BFP_RZ 1  /* round toward zero (Section 4) */

/* Operation codes (Section 4, Table 1: Add/Sub, Mul, Div).  Division is
 * correctly rounded in both modes: an operand pair gives the pattern that
 * rounding the exact quotient once gives (x / 0 = signed Inf for finite
 * nonzero x, 0 / 0 and Inf / Inf = NaN, x / Inf = signed zero). */
#define BFP_ADD 0
#define BFP_SUB 1
#define BFP_MUL 2
#define BFP_DIV 3

/* A custom format: e exponent bits, m mantissa bits, rounding mode. */
typedef struct {
  uint8_t e;
  uint8_t m;
  uint8_t round; /* BFP_RNE or BFP_RZ */
  uint8_t pad;   /* must be 0 */
} bfp_format;

/* Text of a status code (static storage). */
const char* bfp_status_string(bfp_status s);

/* Library version, e.g. "0.1.0". */
const char* bfp_version(void);

/* 1 if (e, m, round) is compiled into this library, else 0. */
int bfp_format_supported(bfp_format f);

/* ---- sizing -------------------------------------------------------------- */

/* Bytes of one standard container: 1, 2, 4 or 8; 0 for an invalid format. */
size_t bfp_container_bytes(bfp_format f);

/* G_pad: 32-bit words per plane for n elements (ceil(n/32) rounded up to a
 * multiple of 64, plus 256 if that is a multiple of 2048). */
uint64_t bfp_plane_stride_words(uint64_t n);

/* Bytes of one bitslice vector: B * G_pad * 4; 0 for an invalid format. */
size_t bfp_bitslice_bytes(bfp_format f, uint64_t n);

/* ---- layout transforms (Section 4 helper transforms; Figure 1) ------------ */

/* Standard -> bitslice.  std_in: device, n containers.  bs_out: device,
 * bfp_bitslice_bytes(f, n) bytes, fully written (padding words zero).  The
 * two buffers must not overlap (BFP_E_ALIAS). */
bfp_status bfp_pack(bfp_format f, const void* std_in, void* bs_out, uint64_t n, void* stream);

/* Bitslice -> standard.  bs_in: device, bitslice vector of n elements.
 * std_out: device, n containers written (upper bits zero); no byte past
 * container n-1 is written.  No overlap allowed. */
bfp_status bfp_unpack(bfp_format f, const void* bs_in, void* std_out, uint64_t n, void* stream);

/* ---- arithmetic on resident bitslice vectors (Section 4, Table 1) --------- */

/* c = a op b elementwise, op in {BFP_ADD, BFP_SUB, BFP_MUL, BFP_DIV}.  a, b, c:
 * device bitslice vectors of n elements in format f (same G_pad); all
 * G_pad words of every plane of c are written, and bits of elements at and
 * above n are zero (as bfp_pack leaves them).  c may be the same buffer as
 * a or b (each lane reads all of its words before writing); partial
 * overlaps are not allowed. */
bfp_status bfp_binop(int op, bfp_format f, const void* a, const void* b, void* c, uint64_t n,
                     void* stream);
bfp_status bfp_add(bfp_format f, const void* a, const void* b, void* c, uint64_t n, void* stream);
bfp_status bfp_sub(bfp_format f, const void* a, const void* b, void* c, uint64_t n, void* stream);
bfp_status bfp_mul(bfp_format f, const void* a, const void* b, void* c, uint64_t n, void* stream);
bfp_status bfp_div(bfp_format f, const void* a, const void* b, void* c, uint64_t n, void* stream);

/* ---- two-op chains on resident bitslice vectors ---------------------------- */
/* d = (a op1 b) op2 c elementwise in one kernel, op1, op2 in {BFP_ADD,
 * BFP_SUB, BFP_MUL} (BFP_E_OP otherwise).  Each op rounds on its own in
 * format f, so d equals bfp_binop(op1, ...) into a temporary followed by
 * bfp_binop(op2, ...) bit for bit; the temporary stays in registers, so 4
 * vectors cross HBM instead of 6.  (Section 4 merges the steps of one
 * operation to avoid storing intermediate results; this applies the same
 * idea across operations.)  a, b, c, d: device bitslice vectors of n
 * elements in format f; d may be the same buffer as a, b or c; partial
 * overlaps are not allowed; bits of elements at and above n in d are zero. */
bfp_status bfp_chain2(int op1, int op2, bfp_format f, const void* a, const void* b, const void* c, void* d,
                      uint64_t n, void* stream);

/* d = alpha * x + y (multiply, then add, each rounded), alpha one standard
 * pattern of format f broadcast to every element (bits above 1+e+m are
 * ignored).  x, y, d as for bfp_chain2. */
bfp_status bfp_axpy(bfp_format f, uint32_t alpha, const void* x, const void* y, void* d, uint64_t n,
                    void* stream);

/* Fused standard-in / standard-out op: pack both operands in registers, run
 * the circuit, unpack, in one kernel with no bitslice round trip to memory.
 * a, b, c: device, n containers each (bfp_container_bytes).  c may equal a
 * or b; partial overlaps are not allowed. */
bfp_status bfp_binop_std(int op, bfp_format f, const void* a, const void* b, void* c, uint64_t n,
                         void* stream);

/* ---- k-bit integer vectors (Section 3, Figure 2) ------------------------------ */
/* Vectors of k-bit integers, 1 <= k <= 32, in the same plane-major bitslice
 * layout with k planes (plane i = bit i).  Standard containers are
 * bfp_int_container_bytes(k) = 1, 2 or 4 bytes holding the k-bit pattern:
 * bits above k-1 are ignored on input and zero on output (a signed value is
 * its k-bit two's complement pattern).  Kinds: */
#define BFP_INT_WRAP 0  /* result modulo 2^k (same bits signed or unsigned) */
#define BFP_INT_SAT_U 1 /* unsigned operands, result clamped to [0, 2^k - 1] */
#define BFP_INT_SAT_S 2 /* signed operands, result clamped to [-2^(k-1), 2^(k-1) - 1] */

/* 1, 2 or 4; 0 if k is not compiled. */
size_t bfp_int_container_bytes(int k);
/* k * G_pad * 4; 0 if k is not compiled. */
size_t bfp_int_bitslice_bytes(int k, uint64_t n);
/* Standard <-> bitslice, with the rules of bfp_pack / bfp_unpack. */
bfp_status bfp_int_pack(int k, const void* std_in, void* bs_out, uint64_t n, void* stream);
bfp_status bfp_int_unpack(int k, const void* bs_in, void* std_out, uint64_t n, void* stream);
/* c = a op b elementwise on k-bit bitslice vectors, op in {BFP_ADD, BFP_SUB,
 * BFP_MUL} (the exact sum, difference or product mapped to k bits by the
 * kind).  a, b, c: device bitslice vectors of n elements (same G_pad); c may
 * be the same buffer as a or b; partial overlaps are not allowed; padding
 * bits of c are zero.  Errors: BFP_E_OP, BFP_E_FORMAT (k or kind), as
 * bfp_binop otherwise. */
bfp_status bfp_int_binop(int op, int k, int kind, const void* a, const void* b, void* c, uint64_t n,
                         void* stream);

/* ---- launch configuration (autotuning) ------------------------------------ */

/* One kernel variant: words per lane per plane (1: W = 32 elements,
 * 2: W = 64, 4: W = 128, the last for formats of at most 10 bits), threads
 * per block, blocks per compute unit for the grid-stride grid (0: one
 * thread per work item, no stride loop), and units per loop step (2: a lane
 * runs two independent circuit instances a grid stride apart). */
typedef struct {
  int32_t words_per_lane; /* 1, 2 or 4 */
  int32_t block;          /* 64, 128, 256 or 512 */
  int32_t blocks_per_cu;  /* 0 or 1..64 */
  int32_t unroll;         /* 0 or 1 (one unit per step) or 2 */
} bfp_launch;

/* Current configuration used for (op, f) by bfp_binop (op BFP_SUB shares
 * BFP_ADD's).  Returns BFP_OK and fills *out. */
bfp_status bfp_launch_get(int op, bfp_format f, bfp_launch* out);

/* Set the configuration for (op, f).  Invalid values give BFP_E_ARG. */
bfp_status bfp_launch_set(int op, bfp_format f, const bfp_launch* cfg);

/* Load / save the whole table as text, one line per entry:
 * "op e m round words_per_lane block blocks_per_cu unroll" (a missing unroll
 * column reads as 1).  Lines starting with '#' are comments.  Unknown
 * formats are skipped on load. */
bfp_status bfp_launch_load(const char* path);
bfp_status bfp_launch_save(const char* path);

/* Autotune bfp_binop for (op, f): time every compiled words_per_lane
 * allowed by `words_per_lane_mask` (bit 0: 1 word, bit 1: 2 words, bit 2:
 * 4 words) x unroll {1,2} x block {64,128,256,512} x blocks_per_cu {0,4,8}
 * on a probe vector of n_probe
 * random elements (median of `reps` runs, each after a 512 MiB read sweep
 * that clears the last-level cache), install the fastest with
 * bfp_launch_set and return it in *best (and its median microseconds in
 * *best_us; either may be NULL).  Allocates and frees its own probe buffers
 * (about 3 * bfp_bitslice_bytes(f, n_probe) + 512 MiB) and synchronises
 * `stream`.  1 <= n_probe <= 2^30, 1 <= reps <= 1000.  On error the previous
 * configuration stays in place. */
bfp_status bfp_autotune(int op, bfp_format f, uint64_t n_probe, int words_per_lane_mask, int reps, void* stream,
                        bfp_launch* best, double* best_us);

/* Practical HBM ceiling of this device: `mode` 0 reads, 1 writes, 2 copies
 * `bytes`, 3 reads two streams of `bytes` and writes their XOR to a third
 * (an elementwise binary op's traffic) (>= 1 GiB recommended, so the 256 MB
 * last-level cache cannot hold the buffers) with 16-byte accesses, every
 * wave instruction covering 1 KiB contiguous.  Every launch shape of a sweep
 * (1, 2, 4, 8, 16 or 32 blocks per CU of 256 threads, and 1 or 2 blocks per
 * CU of 512 or 1024 threads; 1, 2, 4 or 8 accesses per stream in flight per
 * lane; ordinary or non-temporal accesses) is timed over `reps` launches
 * between events on `stream`, and the best rate is returned in *gbps (bytes
 * moved per second, everything read + written, 1e9 units); the winning grid
 * (blocks), block (threads) and accesses in flight go to *best_grid,
 * *best_block and *best_unroll when not NULL.  Allocates its buffers.
 * 2^20 <= bytes <= 2^36, bytes a multiple of 16, 1 <= reps <= 1000. */
bfp_status bfp_measure_hbm(uint64_t bytes, int mode, int reps, void* stream, double* gbps, int* best_grid,
                           int* best_block, int* best_unroll);

/* bfp_measure_hbm in copy mode (read + write GB/s). */
bfp_status bfp_measure_copy(uint64_t bytes, int reps, void* stream, double* gbps);

/* Enqueue a read sweep over `bytes` (2^20 .. 2^34) of a buffer the library
 * keeps per device (allocated on first use or growth), so that the data a
 * following kernel reads comes from HBM rather than the 256 MB last-level
 * cache: the "cold" measurements use it between timed launches. */
bfp_status bfp_flush_llc(uint64_t bytes, void* stream);

/* Enqueue one kernel of a single wave (64 threads) that runs a dependent
 * chain of `iters` fused multiply-adds (1 <= iters <= 2^26) into a 256-byte
 * buffer the library keeps per device.  The kernel lasts as long as its one
 * wave, so its traced duration times the shader clock, set against the
 * profiler's per-wave cycle counter for the same dispatch, gives the
 * counter's unit; the profile summaries use it to turn wave-cycle counts
 * into time.  Returns BFP_E_ARG for `iters` out of range. */
bfp_status bfp_wave_clock(int iters, void* stream);


/* Gate count of one circuit instance (one group of 32 elements per word),
 * constants folded: the cost model of Table 1.  Returns -1 if the format
 * is not compiled. */
long bfp_gate_count(int op, bfp_format f);

/* Launch configuration of the two-op chain kernels for (op1, op2, f) (ops
 * share entries by class: add/sub, mul) and of the integer kernels for
 * (op, k, kind): block and blocks_per_cu are free, words_per_lane is the
 * compiled one (1 for chains; 2, or 1 for the multipliers from k = 13, for
 * integers) and unroll 1.  Default: 256-thread blocks, one thread per work
 * item.  Errors: BFP_E_OP, BFP_E_FORMAT, BFP_E_NULL, BFP_E_ARG. */
bfp_status bfp_chain_launch_get(int op1, int op2, bfp_format f, bfp_launch* out);
bfp_status bfp_chain_launch_set(int op1, int op2, bfp_format f, const bfp_launch* cfg);
bfp_status bfp_int_launch_get(int op, int k, int kind, bfp_launch* out);
bfp_status bfp_int_launch_set(int op, int k, int kind, const bfp_launch* cfg);

/* Autotune bfp_chain2 for (op1, op2, f), or bfp_int_binop for (op, k,
 * kind), as bfp_autotune does bfp_binop: every block {64,128,256,512} x
 * blocks_per_cu {0,4,8}, median of `reps` cold runs on n_probe random
 * elements; installs and returns the fastest.  bfp_launch_save writes these
 * entries too ("chain ..." and "int ..." lines) and bfp_launch_load reads
 * them. */
bfp_status bfp_autotune_chain(int op1, int op2, bfp_format f, uint64_t n_probe, int reps, void* stream,
                              bfp_launch* best, double* best_us);
bfp_status bfp_autotune_int(int op, int k, int kind, uint64_t n_probe, int reps, void* stream, bfp_launch* best,
                            double* best_us);

/* Transpose method of bfp_pack / bfp_unpack (direction 0 / 1) for one
 * container size (1, 2 or 4 bytes; 8-byte containers have the per-lane
 * method only), both computing the layout of Figure 1:
 *   BFP_TRANSPOSE_LANE   each lane transposes one 32-element group in its
 *                        registers (the default);
 *   BFP_TRANSPOSE_XLANE  each lane holds one element and the 32 lanes of a
 *                        half-wave transpose their words together (ds_swizzle
 *                        exchanges), plane rows gathered in LDS.
 * The get call returns the method or BFP_E_ARG. */
#define BFP_TRANSPOSE_LANE 0
#define BFP_TRANSPOSE_XLANE 1
bfp_status bfp_layout_method_set(int direction, int cbytes, int method);
int bfp_layout_method_get(int direction, int cbytes);

/* Time pack (direction 0) or unpack (1) of n_probe elements of format f with
 * each method (median of `reps` cold runs), install the faster for f's
 * container size and return it in *best_method (and its microseconds in
 * *best_us; either may be NULL). */
bfp_status bfp_autotune_layout(int direction, bfp_format f, uint64_t n_probe, int reps, void* stream,
                               int* best_method, double* best_us);

/* ---- batched persistent launch --------------------------------------------- */
/* Many vectors of uneven length and mixed formats in one persistent kernel,
 * captured once in a HIP graph.  (Not in the paper, whose operations act on
 * one vector type at a time; this batches its Section 4 operations.)
 *
 * A task is c = a op b on bitslice vectors of n elements in format f, with
 * the same layout and rules as bfp_binop (c may equal a or b).  The plan
 * copies the descriptors to device memory and captures the graph at
 * creation; the caller keeps every a, b, c allocated and unmoved for the
 * plan's lifetime.  Runs of one plan must not overlap in time (they share
 * the plan's work counter): issue them on one stream, or synchronise. */
typedef struct {
  const void* a; /* device, bitslice, format f, n elements */
  const void* b;
  void* c;
  uint64_t n;
  bfp_format f;
  int32_t op; /* BFP_ADD, BFP_SUB, BFP_MUL or BFP_DIV */
} bfp_task;

typedef struct bfp_batch_plan bfp_batch_plan;

/* Validate `count` tasks, cut them into chunks grouped by circuit variant
 * (slowest variants per word first, division last), upload the descriptors and capture the graph on the current device.
 * Errors: BFP_E_ARG (count 0, n 0), BFP_E_FORMAT, BFP_E_OP, BFP_E_NULL,
 * BFP_E_ALIGN, BFP_E_NOMEM, BFP_E_HIP.  On error *out is NULL. */
bfp_status bfp_batch_plan_create(const bfp_task* tasks, uint32_t count, bfp_batch_plan** out);

/* Launch the captured graph on `stream` (one hipGraphLaunch). */
bfp_status bfp_batch_run(bfp_batch_plan* plan, void* stream);

/* The same two kernels launched directly on `stream`, without the graph. */
bfp_status bfp_batch_run_eager(bfp_batch_plan* plan, void* stream);

/* Baseline: one bfp_binop launch per task, in task order, on `stream`. */
bfp_status bfp_batch_run_per_vector(bfp_batch_plan* plan, void* stream);

/* The same per-task launches captured once (on the first call) in a HIP
 * graph and replayed with one hipGraphLaunch: the baseline without the
 * host's launch overhead. */
bfp_status bfp_batch_run_per_vector_graph(bfp_batch_plan* plan, void* stream);

/* Chunks, persistent grid size and total plane words per operand
 * (sum over tasks of B * G_pad); any pointer may be NULL. */
bfp_status bfp_batch_plan_info(const bfp_batch_plan* plan, uint32_t* nchunks, uint32_t* grid,
                               uint64_t* words_per_operand);

/* Free the plan's device memory and graph (NULL is a no-op).  Wait for its
 * runs to finish first. */
void bfp_batch_plan_destroy(bfp_batch_plan* plan);

/* For callers that cannot allocate -- code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc: the batched launch of
 * bfp_batch_plan_create + bfp_batch_run in one call that allocates nothing.
 * `tasks_dev` is an array of `count` bfp_task in DEVICE memory (8-byte
 * aligned, caller-owned, read on `stream`).  A one-block kernel checks every
 * task as bfp_batch_plan_create does, writes the descriptors and the chunk
 * index into a static device array of the library (about 1.4 MB per device,
 * held until the process ends), and the two persistent kernels then run the
 * chunks in task order.  The status of the check (BFP_OK, or the error of the
 * first invalid task: BFP_E_FORMAT, BFP_E_OP, BFP_E_ARG, BFP_E_NULL,
 * BFP_E_ALIGN) is written to *status_dev (device int32) on `stream`; with any
 * invalid task nothing is computed.  Host-side errors: BFP_E_NULL, BFP_E_ARG
 * (count 0 or above 16384 tasks), BFP_E_ALIGN, BFP_E_HIP.  Every call on one
 * device shares that device's array: calls that overlap on one device (two
 * streams, or two threads) race and must be serialised by the caller. */
bfp_status bfp_batch_run_noalloc(const bfp_task* tasks_dev, uint32_t count, int32_t* status_dev, void* stream);

/* ---- serving loop ---------------------------------------------------------- */
/* A request loop over device-resident bitslice vectors (not in the paper;
 * it serves the Section 4 operations).  The server owns one device arena of
 * `hbm_budget_bytes` (allocated at creation): every resident vector -- the
 * caller's operands and every request's result -- is carved from it, so the
 * memory in use never exceeds the budget.  Requests wait in FIFO order and
 * are admitted when one of `slots` request slots is free and the arena can
 * hold the result.  A worker thread launches all requests admitted since its
 * last launch as one batched persistent kernel on whichever of two streams
 * is free (continuous batching: requests that arrive while a batch runs join
 * the next one, which may start before the first ends).
 *
 * Handles are 64-bit (0 is never a handle): the low half names a slot of the
 * server's vector table and the high half that slot's generation, so the
 * handle of a freed vector stays invalid after its slot is reused.  A
 * request computes its op on the first n elements of both operands (same
 * format as the request's e, m; the rounding mode comes from the request);
 * its result is a new resident vector of n elements whose padding bits are
 * zero, whatever the operands hold past n.  Every vector counts the queued,
 * admitted and running requests that use it: freeing a vector retires its
 * handle at once and returns its memory when the last of them completes.
 * Times are steady-clock nanoseconds. */
typedef struct bfp_server bfp_server;
typedef uint64_t bfp_handle;

typedef struct {
  uint64_t req_id;
  bfp_handle result; /* handle of the result vector (0 on error or with autofree) */
  int32_t status;    /* BFP_OK, an error, BFP_E_CANCELLED or BFP_E_TIMEOUT */
  uint32_t _pad;
  uint64_t n;
  int64_t t_submit_ns, t_admit_ns, t_launch_ns, t_done_ns; /* t_done: completion observed */
} bfp_completion;

typedef struct {
  uint64_t budget, used, high_water;            /* arena bytes */
  uint64_t submitted, admitted, completed, ticks;
  uint64_t max_tick_requests, max_inflight_ticks, deferred_budget;
  uint64_t pending, inflight;
  uint64_t deferred_frees; /* frees whose memory waited for running requests */
  uint64_t cancelled, timed_out;
  uint64_t live_vectors, table_slots; /* resident vectors now, and table slots ever used */
} bfp_server_stats;

/* Create a server on the current device.  Errors: BFP_E_ARG (budget < 256
 * bytes, slots outside 1..2^20), BFP_E_NOMEM (arena), BFP_E_HIP. */
bfp_status bfp_server_create(uint64_t hbm_budget_bytes, int32_t slots, bfp_server** out);

/* Pack n standard containers (device memory, read in order on `stream`)
 * into a new resident vector; synchronises `stream` before returning, so the
 * vector is ready for any later request.  BFP_E_BUDGET if the arena is full. */
bfp_status bfp_server_put(bfp_server* s, bfp_format f, const void* std_dev, uint64_t n, void* stream,
                          bfp_handle* handle);

/* Queue c = a op b on the first n elements of resident vectors a and b
 * (n <= both lengths).  Returns at once with the request id.  BFP_E_ARG for
 * a handle that is not live or a bad length, BFP_E_FORMAT if an operand's
 * format differs from f, BFP_E_BUDGET if the result could never fit in the
 * arena. */
bfp_status bfp_server_submit(bfp_server* s, int op, bfp_format f, bfp_handle a, bfp_handle b, uint64_t n,
                             uint64_t* req_id);

/* Withdraw a request that is queued or admitted but not yet launched: it
 * completes with status BFP_E_CANCELLED and holds nothing afterwards.
 * BFP_E_BUSY if it is already on the device (it completes normally),
 * BFP_E_ARG if no request with this id is queued or running. */
bfp_status bfp_server_cancel(bfp_server* s, uint64_t req_id);

/* Requests not launched within `timeout_ns` of their submission complete
 * with status BFP_E_TIMEOUT (0 or negative: no limit, the default).  A
 * request on the device always runs to completion. */
bfp_status bfp_server_set_queue_timeout(bfp_server* s, int64_t timeout_ns);

/* Largest tick: the worker launches the admitted requests in FIFO order up
 * to `max_bytes` of operand and result planes per tick (a, b and c of each
 * request; at least one request per tick), so that a backlog runs as a
 * sequence of bounded launches that complete their requests progressively
 * and alternate between the two streams.  The default is 4 GiB; 0 puts
 * every admitted request in the next tick. */
bfp_status bfp_server_set_tick_limit(bfp_server* s, uint64_t max_bytes);

/* Move up to `max` completions (oldest first) to `out`; *count is set. */
bfp_status bfp_server_poll(bfp_server* s, bfp_completion* out, uint32_t max, uint32_t* count);

/* One entry of an arrival schedule for bfp_server_replay. */
typedef struct {
  int32_t op;
  bfp_format f;
  bfp_handle a, b;     /* operand handles */
  uint64_t n;
  int64_t arrival_ns;  /* submission time, ns after the replay call starts; non-decreasing */
} bfp_request;

/* Submit `count` requests from the calling thread, each at its arrival time
 * (the thread sleeps until shortly before and then spins), so an arrival
 * process is driven at native speed.  Ids are consecutive from *first_id.
 * Ops, formats and the arrival order are checked before the first entry is
 * submitted; an invalid handle or length stops the replay at that entry
 * with its error (earlier entries stay submitted).  Returns when the last
 * entry is submitted; completions are polled as usual. */
bfp_status bfp_server_replay(bfp_server* s, const bfp_request* reqs, uint32_t count, uint64_t* first_id);

/* With `on` nonzero, each result vector is returned to the arena as soon as
 * its request completes (its completion reports result 0). */
bfp_status bfp_server_set_autofree(bfp_server* s, int32_t on);

/* Wait until no request is queued, admitted or running (BFP_E_TIMEOUT on
 * timeout). */
bfp_status bfp_server_wait_idle(bfp_server* s, int64_t timeout_ms);

/* Device address and length of a resident vector.  The address stays valid
 * only while the caller keeps the handle live (until bfp_server_free). */
bfp_status bfp_server_view(bfp_server* s, bfp_handle handle, void** bitslice_dev, uint64_t* n);

/* Unpack a resident vector of format f into its n standard containers at
 * std_dev_out (device), on `stream`, and synchronise `stream`.  The vector
 * is held for the duration of the call, so a concurrent free cannot hand its
 * memory to another vector mid-unpack.  Call it only for vectors whose
 * request has completed. */
bfp_status bfp_server_get(bfp_server* s, bfp_handle handle, bfp_format f, void* std_dev_out, void* stream);

/* Retire a resident vector (operand or result): the handle is invalid from
 * now on, and the memory returns to the arena once no queued, admitted or
 * running request uses it.  BFP_E_ARG if the handle is not live. */
bfp_status bfp_server_free(bfp_server* s, bfp_handle handle);

bfp_status bfp_server_stats_get(bfp_server* s, bfp_server_stats* out);

/* Stop the worker (running batches finish first) and free everything. */
void bfp_server_destroy(bfp_server* s);

#ifdef __cplusplus
}
#endif

#endif /* BFP_H */
