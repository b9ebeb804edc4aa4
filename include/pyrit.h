/*
 * pyrit.h: C ABI of the MI355X (gfx950) erasure-coding library.
 *
 * Systematic MDS erasure codes over GF(2^w) = F_2[x]/(p(x)), computed in the
 * polynomial ring R_{2,n} = F_2[x]/(x^n + 1) with n odd and p dividing
 * x^n + 1, after Detchart & Lacan, "Improving the coding speed of erasure
 * codes with polynomial ring transforms":
 *   - each generator coefficient u is replaced by its sparsest ring
 *     representative c (c = u mod p, fewest nonzero coefficients; the
 *     "sparse transform" of Sec. II-B);
 *   - each data block is embedded in the ring by padding its w slices with
 *     n - w zero slices (the embedding transform of Sec. II-C.2 / II-D.2);
 *   - multiplying by x^s rotates slice indices by s modulo n, so a product is
 *     an XOR of rotated slices, and the n ring slices of each output are
 *     reduced modulo p back to w field slices (inverse embedding, Prop. 2).
 * Plans may instead use the paper's parity transform (Sec. II-C.1 / II-D.1,
 * see PYRIT_TRANSFORM_PARITY), a different MDS code of the same shape.
 *
 * Data layout.  A block is w slices of S bytes ("slice_bytes"), contiguous,
 * or slice_pitch bytes apart in the *_ex calls and in batches.
 * Slice t holds coefficient t of every symbol: symbol (o, b), for byte offset
 * o < S and bit b < 8, is sum_t bit b of byte o of slice t, times x^t.  S must
 * be a positive multiple of 64, every block pointer 16-byte aligned, and
 * (w - 1) * pitch + S < 2^31 (w * S for packed slices).
 *
 * Integers that encode polynomials over GF(2) use bit i for the coefficient
 * of x^i (p includes its x^w term: x^8+x^5+x^4+x^3+1 is 0x139).
 *
 * Conventions.  Every entry point returns PYRIT_OK (0) or a negative
 * PYRIT_E* code; no C++ exception crosses this boundary (a failed host
 * allocation inside the library returns PYRIT_ENOMEM, leaving every object
 * as it was before the call).  Pointer arrays
 * (data[], parity[], blocks[]) are host arrays of device pointers; the
 * library copies them before returning.  Device work is enqueued on the
 * caller's stream (a hipStream_t passed as void*, NULL = the null stream)
 * and runs asynchronously: device faults surface at the caller's next
 * synchronisation.  The caller owns every device buffer and stream.  Plans
 * are immutable after creation (their decode cache is internally locked), so
 * several streams may use one plan at once.
 */
#ifndef PYRIT_H
#define PYRIT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  PYRIT_OK = 0,
  PYRIT_EINVAL = -1,       /* bad argument: size, count, NULL pointer */
  PYRIT_ENOTIRRED = -2,    /* p is not irreducible of degree w */
  PYRIT_ENOTDIV = -3,      /* n even, or p does not divide x^n + 1 */
  PYRIT_ETOOLONG = -4,     /* k + m exceeds 2^w (Cauchy code length limit) */
  PYRIT_ERANGE = -5,       /* a generator coefficient is >= 2^w */
  PYRIT_ETOOMANY = -6,     /* more erasures than parity blocks */
  PYRIT_ESINGULAR = -7,    /* surviving rows of [I; G] are not invertible */
  PYRIT_EALIGN = -8,       /* slice size or pointer alignment */
  PYRIT_EUNSUPPORTED = -9, /* no device kernel for this (w, n, p) ring */
  PYRIT_EHIP = -10,        /* a HIP runtime call failed */
  PYRIT_ENOMEM = -11,      /* host or device allocation failed */
  PYRIT_EBUSY = -12,       /* resource cap reached (serving admission) */
  PYRIT_EINTERNAL = -13,   /* an unexpected internal failure (a bug) */
  PYRIT_ETOOBIG = -14      /* work exceeds a fixed-size library buffer */
};

#define PYRIT_KMAX 64      /* maximum data blocks per stripe */
#define PYRIT_MMAX 64      /* maximum parity blocks per stripe */
#define PYRIT_SMAX_TOTAL 0x7fffffffu /* (w - 1) * pitch + S must stay below this */

/* Text for an error code (static storage). */
const char *pyrit_strerror(int code);

/* Library version string, e.g. "pyrit-mi355x 0.1". */
const char *pyrit_version(void);

/* ------------------------------------------------------------------ algebra
 * Host-side helpers; no device work, usable without a GPU.
 */

/* Check a field/ring pair (Sec. II-A): 1 <= w <= 16, deg p = w, p
 * irreducible, w < n <= 24, n odd, p divides x^n + 1.  Returns PYRIT_OK,
 * PYRIT_EINVAL, PYRIT_ENOTIRRED or PYRIT_ENOTDIV. */
int pyrit_ring_check(int w, int n, uint32_t p);

/* Whether a device kernel exists for this ring with the embedding transform
 * (1) or not (0).  The parity transform has kernels for (4,5,0x1F),
 * (10,11,0x7FF) and (6,9,0x49). */
int pyrit_ring_supported(int w, int n, uint32_t p);

/* Sparse transform of one field element (Sec. II-B): among the 2^(n-w) ring
 * elements c with c mod p == u (deg c < n), return in *c one of least
 * Hamming weight, the numerically smallest on ties. */
int pyrit_lift(int w, int n, uint32_t p, uint32_t u, uint32_t *c);

/* Inverse embedding (Prop. 2, Sec. II-C.2): *u = c mod p for a ring element
 * c of degree < n. */
int pyrit_ring_reduce(int w, int n, uint32_t p, uint32_t c, uint32_t *u);

/* Product in R_{2,n} = F_2[x]/(x^n + 1): the cyclic convolution of a and b. */
int pyrit_ring_mul(int n, uint32_t a, uint32_t b, uint32_t *c);

/* Product in GF(2^w) = F_2[x]/(p). */
int pyrit_gf_mul(int w, uint32_t p, uint32_t a, uint32_t b, uint32_t *c);

/* Plain Cauchy parity matrix (Sec. III uses Cauchy-type MDS generators):
 * G[i*k + j] = 1 / (i + (m + j)) in GF(2^w), i < m, j < k.  Requires
 * k + m <= 2^w.  G is a host array of m*k entries. */
int pyrit_cauchy(int w, uint32_t p, int k, int m, uint16_t *G);

/* Generalized Cauchy parity matrix of small ring weight (Sec. III codes with
 * generalized Cauchy matrices; Sec. II-B: the XOR count is the number of
 * ones of the lifted matrix):
 *   G[i*k + j] = row_scale[i] * C[i][j] * col_scale[j],  C = pyrit_cauchy,
 * with nonzero multipliers chosen by coordinate descent to lower the total
 * weight of the lifted matrix in R_{2,n}.  Scaling rows and columns by
 * nonzero elements keeps every square submatrix nonsingular, so G is MDS.
 * row_scale (m entries), col_scale (k entries) and weight (the total lifted
 * weight) may be NULL.  Deterministic.  Errors as pyrit_ring_check and
 * pyrit_cauchy. */
int pyrit_cauchy_light(int w, int n, uint32_t p, int k, int m, uint16_t *G, uint16_t *row_scale,
                       uint16_t *col_scale, int *weight);

/* -------------------------------------------------------------------- plans */
/* Generalized Cauchy parity matrix with its points chosen as well (the
 * generalized Cauchy codes of Sec. III; Sec. II-B: fewer ones in the lifted
 * matrix mean fewer XORs):
 *   G[i*k + j] = row_scale[i] * col_scale[j] / (X[i] + Y[j]),
 * X (m points) and Y (k points) distinct elements of GF(2^w).  Start: X =
 * {0..m-1}, Y = {m..m+k-1} and the multipliers of pyrit_cauchy_light.  Each
 * sweep offers every point, in turn, every field element not in use, taking
 * it (with that row's or column's best multiplier) when the total lifted
 * weight drops, then re-chooses all multipliers by coordinate descent; it
 * stops after `sweeps` sweeps or a sweep without a gain.  Any distinct
 * points and nonzero multipliers give a Cauchy matrix scaled by rows and
 * columns, whose square submatrices are all nonsingular: G is MDS.  X, Y,
 * row_scale, col_scale and weight (the total lifted weight) may be NULL.
 * Deterministic.  w <= 10 (PYRIT_EUNSUPPORTED above).  Errors as
 * pyrit_cauchy_light, plus PYRIT_EINVAL for sweeps < 0. */
int pyrit_cauchy_search(int w, int n, uint32_t p, int k, int m, int sweeps, uint16_t *G,
                        uint16_t *X, uint16_t *Y, uint16_t *row_scale, uint16_t *col_scale,
                        int *weight);

typedef struct pyrit_plan pyrit_plan;

/* How data enter and leave the ring.
 *   EMBEDDING (Sec. II-C.2, II-D.2): a symbol is padded with n - w zero
 *     coefficients; results are reduced modulo p.  The code is exactly the
 *     field code [I_k; G].
 *   PARITY (Sec. II-C.1, II-D.1): a symbol b enters as the element of the
 *     ideal isomorphic to the field whose low w coefficients are b (for the
 *     AOP, one parity bit; for x^6+x^3+1, three interleaved parity bits);
 *     results leave by dropping the n - w high coefficients.  This is a
 *     different code: with psi(b) = phi_P(b) mod p, parity_i =
 *     psi^-1(sum_j G[i][j] psi(d_j)) symbol by symbol, still MDS; encoder and
 *     decoder must both use it.  Kernels exist for the AOP rings (4,5),
 *     (10,11) and the ESP ring (6,9). */
enum { PYRIT_TRANSFORM_EMBEDDING = 0, PYRIT_TRANSFORM_PARITY = 1 };

/* Build the lifted XOR schedule of the systematic code [I_k; G] (G is the
 * m x k row-major parity part, host memory, copied).
 *   Follows Sec. II-A (the field F_2[x]/(p) inside R_{2,n} = F_2[x]/(x^n+1)
 *   when p divides x^n + 1, n odd) and Sec. II-B (the sparse transform: each
 *   coefficient G[i][j] is replaced by a ring element of least Hamming
 *   weight congruent to it mod p, so the product by it costs one rotated
 *   copy of the block per nonzero coefficient); the code is the systematic
 *   MDS code of Sec. III, whose parity part is G.
 *   Validates the ring (pyrit_ring_check), 1 <= k <= PYRIT_KMAX,
 *   1 <= m <= PYRIT_MMAX, k + m <= 2^w and every G entry < 2^w.  A plan for
 *   a ring without a device kernel is still created (host queries work);
 *   device calls on it return PYRIT_EUNSUPPORTED.
 *   Ownership: *out receives a plan the caller releases with
 *   pyrit_plan_destroy; G is not referenced after the call.
 *   Errors: PYRIT_EINVAL (NULL G or out, k or m out of range),
 *   PYRIT_ENOTIRRED, PYRIT_ENOTDIV, PYRIT_ETOOLONG, PYRIT_ERANGE,
 *   PYRIT_ENOMEM; *out is NULL after any error. */
int pyrit_plan_create(int w, int n, uint32_t p, int k, int m, const uint16_t *G,
                      pyrit_plan **out);

/* pyrit_plan_create with a choice of transform (PYRIT_TRANSFORM_*); an
 * unknown transform is PYRIT_EINVAL.  pyrit_plan_create is the EMBEDDING
 * case.  Decoding with a PARITY plan undoes the PARITY code. */
int pyrit_plan_create_ex(int w, int n, uint32_t p, int k, int m, const uint16_t *G, int transform,
                         pyrit_plan **out);

/* The plan's transform (PYRIT_TRANSFORM_*). */
int pyrit_plan_transform(const pyrit_plan *plan, int *transform);

/* Release a plan and its device copies.  NULL is ignored.  The caller must
 * ensure no stream still runs work that uses the plan. */
void pyrit_plan_destroy(pyrit_plan *plan);

/* Code parameters of a plan (any pointer may be NULL). */
int pyrit_plan_params(const pyrit_plan *plan, int *w, int *n, uint32_t *p, int *k, int *m);

/* The m*k lifted ring elements (row-major, host array of m*k uint32). */
int pyrit_plan_lifted(const pyrit_plan *plan, uint32_t *C);

/* Total Hamming weight of the lifted matrix: the number of rotated-slice
 * XOR terms per output column ("number of ones", Sec. II-B). */
int pyrit_plan_weight(const pyrit_plan *plan, int *weight);

/* Decoding matrix for an erasure pattern (Sec. IV-C): survivors are the first
 * k block ids in 0..k+m-1 that are not erased; D (n_erased x k, row-major,
 * host) maps the survivors to the erased blocks in the listed order:
 * D = G_E * A^{-1} with A the survivors' rows of [I; G] and G_E the erased
 * rows.  survivors (k ints) and D may be NULL. */
int pyrit_decode_matrix(const pyrit_plan *plan, const int *erased, int n_erased,
                        int *survivors, uint16_t *D);

/* ------------------------------------------------------------- device calls */

/* Encode: parity[i] = sum_j G[i][j] * data[j] for i < m, symbol by symbol.
 *   Follows Sec. II-B (each G[i][j] is its sparse ring representative c_ij,
 *   and multiplying by x^s in R_{2,n} rotates the n ring slices by s), the
 *   embedding transform of Sec. II-C.2 / II-D.2 (a block enters the ring as
 *   its w slices followed by n - w zero slices, which are never stored or
 *   loaded) and Prop. 2 (reduction mod p maps the ring sum back to the field
 *   product, so each parity's n ring slices are reduced once, after its last
 *   input).  A PARITY plan computes the parity-transform code instead
 *   (Sec. II-C.1 / II-D.1, PYRIT_TRANSFORM_PARITY).
 *   data: k device pointers, parity: m device pointers (host arrays, copied
 *   before the call returns); each block is w slices of slice_bytes bytes,
 *   packed.  Outputs must not alias inputs.  Enqueued on `stream`; the
 *   caller keeps the buffers alive until it completes.
 *   Errors: PYRIT_EINVAL (NULL plan, array or entry), PYRIT_EALIGN (slice
 *   size not a positive multiple of 64, pointer not 16-byte aligned),
 *   PYRIT_EUNSUPPORTED (no kernel for the ring), PYRIT_EHIP (launch). */
int pyrit_encode(const pyrit_plan *plan, const uint8_t *const *data, uint8_t *const *parity,
                 size_t slice_bytes, void *stream);

/* Decode: blocks holds k + m device pointers (data then parity).  Entries
 * listed in erased[] (distinct ids, n_erased <= m) are outputs; the first k
 * non-erased entries are read.
 *   Follows Sec. IV-C: the decoding matrix depends on the loss pattern.  It
 *   is built on the host (pyrit_decode_matrix: the survivors' rows A of
 *   [I; G] inverted over GF(2^w), D = G_E * A^-1, cached per pattern on the
 *   plan), lifted by the sparse transform of Sec. II-B, and the encode
 *   kernels run with D in place of G, the survivors as inputs and the
 *   erased blocks as outputs.
 *   Layout, ownership and asynchrony as pyrit_encode; entries that are
 *   neither read nor written may be NULL.
 *   Errors: those of pyrit_encode, PYRIT_EINVAL (erased id out of range or
 *   repeated), PYRIT_ETOOMANY (n_erased > m), PYRIT_ESINGULAR (a user G
 *   whose surviving rows are not invertible), PYRIT_ENOMEM. */
int pyrit_decode(const pyrit_plan *plan, const int *erased, int n_erased,
                 uint8_t *const *blocks, size_t slice_bytes, void *stream);

/* pyrit_encode with two layout/launch options:
 *   slice_pitch: bytes from the start of one slice of a block to the next
 *     (0 = slice_bytes, the packed layout).  A pitch P >= S, multiple of 64,
 *     places slice t at t*P; the P - S bytes after each slice are never read
 *     or written, and (w-1)*P + S must stay below 2^31.  A pitch that is not
 *     a large power of two keeps the slices of a block off the same HBM
 *     channel and bank (measured on MI355X: 8 MiB slices at a pitch of
 *     8 MiB + 4 KiB stream 8% faster than packed).  Slices that start on
 *     128-byte boundaries (block and P multiples of 128) keep every wave
 *     access within whole 128-byte cache lines: a batch of mixed slice sizes
 *     measured 5% faster than with 64-byte aligned packed slices.
 *   vec_bytes: column bytes per lane (4, 8 or 16; 0 = library choice, a
 *     per-ring table measured on MI355X: 4 for the 8-slice field; 8 for
 *     the 4-slice field up to four outputs per pass; 16, 8 or 4 for the
 *     6- and 10-slice fields at one, up to four, or more outputs). */
int pyrit_encode_ex(const pyrit_plan *plan, const uint8_t *const *data, uint8_t *const *parity,
                    size_t slice_bytes, size_t slice_pitch, int vec_bytes, void *stream);

/* pyrit_decode with a slice pitch (as in pyrit_encode_ex). */
int pyrit_decode_ex(const pyrit_plan *plan, const int *erased, int n_erased,
                    uint8_t *const *blocks, size_t slice_bytes, size_t slice_pitch, void *stream);

/* ------------------------------------------------ symbol <-> bit-sliced layout
 * The coding calls take bit-sliced blocks (a block as w chunks, Sec. III):
 * slice t holds bit t of every symbol, symbol s at bit s mod 8 of byte s div 8
 * of the slice.  These two calls convert a block of n_symbols ordinary
 * symbols (one byte each for w <= 8, the low w bits; one little-endian 16-bit
 * word each for 8 < w <= 16) to and from that layout on the device.
 *   symbols: device pointer, n_symbols * (w <= 8 ? 1 : 2) bytes;
 *   sliced:  device pointer, w slices of n_symbols / 8 bytes, slice t at
 *            sliced + t * slice_pitch (0 = n_symbols / 8).
 * n_symbols must be a positive multiple of 512 (whole 64-byte slice rows);
 * both pointers 16-byte aligned; slice_pitch a multiple of 64.  Symbol bits at
 * or above w are ignored on the way in and written as zero on the way out.
 * Asynchronous on `stream`.  Errors: PYRIT_EINVAL, PYRIT_EALIGN, PYRIT_EHIP. */
int pyrit_to_sliced(int w, const void *symbols, size_t n_symbols, uint8_t *sliced,
                    size_t slice_pitch, void *stream);
int pyrit_from_sliced(int w, const uint8_t *sliced, size_t slice_pitch, size_t n_symbols,
                      void *symbols, void *stream);

/* Fill nbytes of device memory with the seeded SplitMix64 stream (word q of
 * the buffer is mix64(key + (q+1) * 0x9E3779B97F4A7C15), little endian) for
 * bytes < nrandom, zero beyond.  nbytes must be a multiple of 8. */
int pyrit_fill_random(uint8_t *dst, size_t nbytes, size_t nrandom, uint64_t key, void *stream);

/* pyrit_fill_random for n buffers in one kernel launch: buffer i is
 * dst[i] (device, 8-byte aligned), nbytes[i] bytes (a multiple of 8), filled
 * with the stream of key keys[i], random for bytes < nrandom[i] (nrandom
 * NULL: all bytes) and zero beyond; a buffer of 0 bytes is skipped and its
 * address may be NULL.  The host arrays are copied to a device table that
 * the call allocates and frees; the call returns once the fill
 * has completed on `stream`.  Buffers must not overlap.  Errors:
 * PYRIT_EINVAL, PYRIT_ENOMEM, PYRIT_EHIP. */
int pyrit_fill_random_blocks(uint8_t *const *dst, const size_t *nbytes, const size_t *nrandom,
                             const uint64_t *keys, int n, void *stream);

/* Device-to-device copy with the library's streaming copy kernel (16-byte
 * non-temporal loads, each 16 bytes stored as two 8-byte stores with the
 * default cache policy); src and dst 16-byte aligned, nbytes a multiple of
 * 16.  A bandwidth reference for equal read and write traffic. */
int pyrit_copy(uint8_t *dst, const uint8_t *src, size_t nbytes, void *stream);

/* ------------------------------------------------------------------ batches
 * Many stripes (any mix of supported rings and transforms, k, m, slice sizes,
 * encodes and decodes) coded by ONE kernel launch.  Each stripe is split into
 * passes of at most four outputs and each pass into column tiles; the tiles
 * form a work queue that the launch drains (see pyrit_tune.mode).  The launch
 * is instantiated as a hipGraph with a single kernel node, replayed by
 * pyrit_batch_launch; pyrit_batch_launch_direct dispatches the same kernel
 * without the graph.  The output bytes of every stripe equal those of
 * pyrit_encode / pyrit_decode on the same inputs.
 */
typedef struct {
  const pyrit_plan *plan;   /* code of this stripe (must outlive the batch) */
  int n_erased;             /* 0: encode all m parity blocks; else: decode */
  const int *erased;        /* n_erased distinct block ids (host, copied) */
  uint8_t *const *blocks;   /* k + m device pointers (host array, copied):
                               data then parity; outputs are the parity
                               blocks (encode) or the erased blocks (decode);
                               the first k non-erased blocks are inputs */
  size_t slice_bytes;       /* S of this stripe */
  size_t slice_pitch;       /* slice stride, 0 = slice_bytes (see pyrit_encode_ex) */
} pyrit_batch_item;

/* How the work queue is drained.
 *   PYRIT_BATCH_GRID:   one workgroup per queue item, the hardware dispatcher
 *                       hands items to CUs in queue order (default).
 *   PYRIT_BATCH_QUEUE:  persistent: a resident grid of waves; each wave takes
 *                       one item from a static slot, then claims items from
 *                       one of eight atomic sub-queues.
 *   PYRIT_BATCH_STATIC: persistent: the host assigns items to waves ahead of
 *                       time, longest first, balancing bytes per wave. */
enum { PYRIT_BATCH_GRID = 0, PYRIT_BATCH_QUEUE = 1, PYRIT_BATCH_STATIC = 2 };

typedef struct {
  int mode;         /* PYRIT_BATCH_* */
  int tile_bytes;   /* persistent modes: column bytes per item; 0 = library choice */
  int grid;         /* persistent modes: resident workgroups; 0 = CUs x occupancy */
  int wg_threads;   /* 64, 128 or 256 threads per workgroup; 0 = 128 */
  int xcd_order;    /* grid mode, 0 or 1.  Workgroups are dealt round-robin
                       over the 8 XCDs; with 1 the workgroup-to-item map is
                       permuted so that each XCD codes a contiguous range of
                       the queue, the ranges cut to equal bytes moved (0:
                       workgroup i codes item i).  Persistent modes ignore
                       it. */
  int split_k;      /* grid mode: waves sharing one column chunk, each coding
                       every split_k-th input block, partial sums combined in
                       LDS before the stores: 1, or 2 (128-thread workgroups:
                       one pair of waves on one chunk; 256-thread: two pairs
                       on adjacent chunks); 0 = 2 for 128-thread grid
                       workgroups, else 1.  Persistent modes take 0 or 1. */
} pyrit_tune;

typedef struct pyrit_batch pyrit_batch;

/* Validate every item, build the work queue (host), upload descriptors and
 * pointer tables to device memory (one allocation owned by the batch) and
 * instantiate the hipGraph.  Nothing runs on the GPU yet.  tune may be NULL.
 * Items are validated like pyrit_encode / pyrit_decode; the first failing
 * item's code is returned and no batch is created.  A batch whose launch
 * would exceed 2^32 - 1 threads (grid mode: one workgroup per work item) is
 * PYRIT_EINVAL; split it into several batches.  The items of one batch
 * run concurrently: no item may write a block (or slice bytes) that another
 * item of the same batch reads or writes. */
int pyrit_batch_create(const pyrit_batch_item *items, int n_items, const pyrit_tune *tune,
                       pyrit_batch **out);

/* Enqueue one execution of the batch on stream (graph replay).  A batch
 * must not run concurrently with itself (its queue counters are shared);
 * distinct batches may run concurrently on distinct streams. */
int pyrit_batch_launch(pyrit_batch *batch, void *stream);

/* Same work as pyrit_batch_launch, as a direct kernel launch (no graph). */
int pyrit_batch_launch_direct(pyrit_batch *batch, void *stream);

/* Facts about a batch (any pointer may be NULL): passes, work items, bytes
 * the batch reads and writes ((k + outputs) * w * S summed), and the
 * workgroups and threads per workgroup it launches. */
int pyrit_batch_info(const pyrit_batch *batch, int *n_passes, int *n_work_items,
                     uint64_t *moved_bytes, int *grid, int *wg_threads);

/* Release the batch.  The caller must ensure no stream still runs it. */
void pyrit_batch_destroy(pyrit_batch *batch);

/* The work pyrit_batch_create would set up for the same items and tune,
 * computed on the host only: nothing is allocated on or sent to the device
 * and the block pointers are not dereferenced (they must still be 16-byte
 * aligned), so it serves capacity planning.  The persistent modes need
 * tune->grid > 0, since their resident grid is otherwise a device query.
 * Outputs as pyrit_batch_info (any pointer may be NULL); xcd_bytes (8
 * entries) receives the bytes moved by each XCD's contiguous item range in
 * grid mode with xcd_order = 1 (the ranges are cut to equal bytes), zeros
 * otherwise.  Errors as pyrit_batch_create, without the device ones. */
int pyrit_batch_describe(const pyrit_batch_item *items, int n_items, const pyrit_tune *tune,
                         int *n_passes, int *n_work_items, uint64_t *moved_bytes, int *grid,
                         uint64_t *xcd_bytes);

/* A batch run that allocates nothing: for callers that cannot allocate
 * device memory (tight serving loops, hosts that forbid hipMalloc).  It
 * does the work of pyrit_batch_create followed by one
 * pyrit_batch_launch_direct and pyrit_batch_destroy, with the same outputs,
 * but the batch's device image (work queue, pass descriptors, pointer and
 * lift tables, queue counters) goes into a fixed device array of the
 * library instead of a new allocation.  That array holds
 * PYRIT_SCRATCH_BYTES bytes on each GPU the library runs on, from the
 * first call on that GPU until the process ends; a batch whose image is
 * larger returns PYRIT_ETOOBIG (split its items over several calls).
 *
 * Each call builds the image in host memory and copies it into the array on
 * `stream`, ahead of the kernel (the copy also zeroes the queue counters).
 * The copy is from pageable host memory, which HIP performs synchronously,
 * so the call returns after the copy has completed.  Calls on one stream are
 * ordered.  Every call on one GPU shares that GPU's array, which keeps the
 * last call's image: calls that overlap on one GPU (from several host
 * threads, or on several streams whose work may run at the same time) race
 * on it, and the caller must serialise them.  The current device must be
 * the stream's device.  A stream that is being captured into a graph is
 * PYRIT_EINVAL: the captured copy would read host memory the call has
 * released.  Errors as pyrit_batch_create, plus PYRIT_ETOOBIG. */
#define PYRIT_SCRATCH_BYTES (8u << 20)
int pyrit_batch_run_noalloc(const pyrit_batch_item *items, int n_items, const pyrit_tune *tune,
                            void *stream);

/* ------------------------------------------------------------------ serving
 * A request loop with continuous batching.  Requests arrive over time; each
 * is admitted (FIFO) once its output blocks fit in the server's device pool,
 * which caps the working set; whenever a launch slot (a stream) is free, all
 * admitted requests not yet launched go to the GPU as one batch (the batch
 * kernels above), so requests arriving while earlier ones run are coded in
 * overlapping launches.  Plans and input buffers stay resident; the server
 * owns the output pool, the per-slot descriptor buffers and the streams.
 * Queued small requests that the idle slots can hold go out one per slot;
 * beyond that they go out together on one slot.  A launch that carries at
 * most four requests runs the plain kernel once per request, back to back
 * on its stream (arguments in the kernel-argument segment, nothing uploaded
 * first); larger ones run one batch kernel.
 */
typedef struct {
  double arrival_s;             /* seconds after the start of the run */
  const pyrit_plan *plan;
  int n_erased;                 /* 0: encode the m parity blocks; else decode */
  const int *erased;            /* n_erased distinct block ids (host) */
  const uint8_t *const *inputs; /* k device pointers: the data blocks (encode)
                                   or the first k non-erased blocks (decode) */
  size_t slice_bytes;
  size_t slice_pitch;           /* 0 = slice_bytes; also the pitch of outputs */
} pyrit_request;

typedef struct {
  double admit_s;       /* outputs allocated from the pool */
  double launch_s;      /* its launch was enqueued */
  double done_s;        /* the launch was seen complete */
  uint64_t out_offset;  /* pool offset of its first output block; output r
                           starts at out_offset + r * out_stride */
  uint64_t out_stride;
  int launch;           /* index of the launch that carried it */
} pyrit_request_result;

typedef struct {
  size_t pool_bytes;     /* output pool = working-set cap (bytes) */
  int slots;             /* launches in flight at once (1..16) */
  int max_batch;         /* requests per launch, 0 = unlimited */
  int per_request;       /* 1: one request per launch, plain kernel (baseline) */
  int release_outputs;   /* 1: outputs return to the pool at completion */
  size_t block_skew;     /* bytes left unused after each output block */
  size_t slot_bytes;     /* descriptor buffer per slot, 0 = 64 MiB */
  size_t large_bytes;    /* requests moving at least this many bytes launch
                            alone, on at most slots-1 slots, so that small
                            requests never wait behind them; 0 = off */
  pyrit_tune tune;       /* batch executor (pyrit_batch_create's) */
} pyrit_serve_config;

typedef struct {
  double elapsed_s;         /* first arrival to last completion */
  int launches;
  int max_batch_seen;
  double mean_batch;
  uint64_t peak_pool_bytes; /* largest pool occupancy */
  int admission_waits;      /* requests that waited for pool space */
  uint64_t moved_bytes;     /* (k + outputs) * w * S over all requests */
} pyrit_serve_stats;

typedef struct pyrit_server pyrit_server;

/* Allocate the pool, slot streams, events and descriptor buffers. */
int pyrit_server_create(const pyrit_serve_config *cfg, pyrit_server **out);

/* Device address of the output pool (outputs are read from there). */
void *pyrit_server_pool(const pyrit_server *server);

/* Serve n requests (sorted by arrival_s) in real time from now; returns when
 * all have completed.  res[i] receives request i's timings and output place.
 * Returns PYRIT_EBUSY if a request can never fit (pool too small with
 * release_outputs = 0), or the first request validation error. */
int pyrit_server_run(pyrit_server *server, const pyrit_request *reqs, int n,
                     pyrit_request_result *res, pyrit_serve_stats *stats);

void pyrit_server_destroy(pyrit_server *server);

#ifdef __cplusplus
}
#endif
#endif /* PYRIT_H */
