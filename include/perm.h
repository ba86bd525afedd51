/*
 * perm.h -- C ABI of libperm: Gray-code Glynn permanents on AMD MI355X (gfx950).
 *
 * The permanent of an n x n matrix A is
 *     perm(A) = sum over permutations s of {0..n-1} of  prod_i a[i][s(i)]
 * (arXiv 2602.10141, Sec. 1).  Every entry point below evaluates it with
 * Glynn's formula over 2^(n-1) sign vectors, walked in reflected Gray-code
 * order in contiguous per-thread blocks (Sec. 1 Note; Sec. 2.2-2.3):
 *     perm(A) = 2^-(n-1) * sum_{x < 2^(n-1)} (-1)^x prod_i r_i(x),
 *     r_i(x)  = a[i][0] + sum_{k>=1} d_k(x) a[i][k],
 *     d_k(x)  = 1 - 2*bit_{k-1}(x XOR (x >> 1)),
 * over C (complex128), R (float64) and F_p (p odd, p < 2^31), and lifts
 * residues modulo several primes to a signed integer with the Chinese
 * remainder theorem (Sec. 2.1).
 *
 * Conventions shared by all entry points
 * --------------------------------------
 * - Matrices are dense, row-major, n x n.  complex128 is interleaved
 *   (re, im) binary64, the layout of numpy/torch complex128.  F_p matrices are
 *   uint32 residues; entries >= p are taken mod p.
 * - n = 0 gives perm = 1 (empty product); 0 <= n <= PERM_NMAX (48).
 * - Pointers are host pointers unless PERM_DEVICE_PTRS is set in `flags`, in
 *   which case matrices and outputs named "dev-or-host" are device pointers
 *   (e.g. torch tensor data_ptr()) and the call is asynchronous on `stream`
 *   except where noted.  `stream` is a hipStream_t; NULL is HIP's null
 *   (legacy default) stream, the one PyTorch uses as its default stream, so
 *   such a call is ordered with PyTorch's work there and with every blocking
 *   stream.  A single-matrix call's device output aligned to its element
 *   type is written by the kernels directly (exactly its bytes), otherwise
 *   through a device copy; a host output is written by the kernels into a
 *   pinned slot of the context and copied from there once they are done.
 * - The caller owns every buffer it passes.  The context owns only its
 *   device scratch (staged matrices, partial sums, plans), which grows on
 *   demand up to the context's HBM budget and is reused across calls.
 * - Return value: PERM_OK (0) or a negative-free status code below.  Outputs
 *   are written only on PERM_OK.  perm_last_error() gives a message for the
 *   calling thread's last failure.  No C++ exception crosses this interface.
 * - A context serialises its calls: a call on a different stream than the
 *   previous one first waits (on the device) for the previous call's work.
 *   A context may be used by one host thread at a time.
 * - Work partition.  A permanent's Gray range is split into wave items of
 *   64 lanes x 2^c indices.  Batches (perm_batch, the server) use the
 *   partition of (field, n) in the tuning table, or the library default,
 *   whatever else the batch holds, so a float result has the same bits in
 *   every batch and in the server.  A call whose items at that length would
 *   leave resident waves idle (one matrix of order 10 to about 27, a few
 *   F_p residue matrices) instead uses the latency partition: the chunk
 *   length that minimises the call's time, down to 2^3 (a table entry for
 *   (field, n) turns it off).  F_p results are exact under any partition.  A single
 *   float call (perm_c128, perm_f64) therefore agrees with the same matrix
 *   in a batch to within rounding (1e-10 of prod_i ||row_i||_2 is the tested
 *   bound), and bit for bit when called with PERM_SHARED_PARTITION, which
 *   makes it use the batch partition.
 * - Floating-point results are bit-identical for the same matrix, device and
 *   work partition.
 */
#ifndef PERM_H
#define PERM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define PERM_NMAX 48

/* status codes */
#define PERM_OK        0
#define PERM_EINVAL    1   /* bad argument (see each function) */
#define PERM_ERANGE    2   /* CRT modulus too small for the bound, or output too small */
#define PERM_ENOMEM    3   /* device or host allocation failed, or HBM budget exceeded */
#define PERM_EDEVICE   4   /* HIP runtime error (message in perm_last_error) */
#define PERM_EAGAIN    5   /* server queue full: try again later */
#define PERM_ENOTFOUND 6   /* unknown server ticket */
#define PERM_ECANCELED 7   /* request was cancelled */

/* fields */
#define PERM_C128 0        /* complex128 */
#define PERM_F64  1        /* float64 */
#define PERM_MODP 2        /* integers mod an odd p < 2^31 */

/* flags */
#define PERM_DEVICE_PTRS 0x1u  /* matrix/output pointers are device pointers */
#define PERM_NO_KAHAN    0x2u  /* plain instead of Kahan-compensated float sums */
#define PERM_MONTGOMERY  0x4u  /* F_p: 32-bit Montgomery walk instead of the FP64 Barrett walk */
#define PERM_SHARED_PARTITION 0x8u  /* single float calls: the batch partition (see below) */

typedef struct perm_ctx perm_ctx;

/* Create a context on HIP device `device`.  hbm_budget: most bytes of device
 * scratch the context may hold (0 = 1/4 of the device memory).
 * Errors: PERM_EINVAL (out == NULL), PERM_EDEVICE (no such device). */
int perm_ctx_create(int device, size_t hbm_budget, perm_ctx **out);
void perm_ctx_destroy(perm_ctx *ctx);

/* Text for a status code, and the calling thread's last error message. */
const char *perm_strerror(int status);
const char *perm_last_error(void);

/* perm of one complex128 matrix (paper Sec. 1 definition; Glynn walk, Sec.
 * 2.2-2.3, with Kahan summation, Sec. 1 Note).
 * A: dev-or-host, n*n complex128 row-major.  out: dev-or-host, 2 doubles (re, im).
 * Errors: PERM_EINVAL (n out of range, NULL pointer), PERM_ENOMEM, PERM_EDEVICE. */
int perm_c128(perm_ctx *ctx, const double *A, int n, double *out, unsigned flags, void *stream);

/* perm_c128 for callers that cannot allocate device memory: code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc.  The
 * call makes no hipMalloc, hipFree or host-to-device copy: its scratch
 * (work counters, the work partition, partial sums, staged columns) is a
 * static device array of 2 MiB per device, which the library holds until the
 * process ends, and a kernel writes the partition into it.  Same partition
 * and kernels as perm_c128, so the same bits.
 * A: device, n*n complex128 row-major, 8-byte aligned.  out: device, 2
 * doubles (re, im), 8-byte aligned.  flags must contain PERM_DEVICE_PTRS
 * (PERM_NO_KAHAN, PERM_SHARED_PARTITION allowed); asynchronous on `stream`
 * (NULL: HIP's null stream).
 * 0 <= n <= 32.  Every call on a device shares that device's scratch: calls
 * that overlap on one device (different streams, contexts or threads) race;
 * calls on one stream are ordered.
 * Errors: PERM_EINVAL (host pointers, other flags, n out of range,
 * misalignment, NULL), PERM_ENOMEM (the tuning table's chunk length for n
 * needs more wave items than the scratch holds), PERM_EDEVICE. */
int perm_c128_noalloc(perm_ctx *ctx, const double *A, int n, double *out, unsigned flags,
                      void *stream);

/* perm of one float64 matrix.  A: dev-or-host n*n.  out: dev-or-host, 1 double. */
int perm_f64(perm_ctx *ctx, const double *A, int n, double *out, unsigned flags, void *stream);

/* perm(A) mod p for one residue matrix (paper Sec. 2.1: Ryser's sum over
 * Z/pZ; here Glynn's, which needs p odd).  A: dev-or-host n*n uint32.
 * out: dev-or-host, 1 uint32 in [0, p).
 * Errors: PERM_EINVAL (p even, p < 3 or p >= 2^31; n out of range). */
int perm_modp(perm_ctx *ctx, const uint32_t *A, int n, uint32_t p, uint32_t *out, unsigned flags,
              void *stream);

/* Exact integer permanent through the Chinese remainder theorem (paper Sec.
 * 2.1).  mats: dev-or-host, k matrices of n*n uint32, matrix i reduced mod
 * primes[i] (host array of k distinct primes, 2 < p < 2^31).  log2_bound: an
 * upper bound on log2|perm| (Schur matrices: (n/2) log2 n, from |perm U| <= 1
 * for unitary U; integer matrices: sum_i log2 of the row 1-norms).
 * The residues are lifted by Garner's algorithm to the unique X with
 * |X| < M/2, M = prod primes; PERM_ERANGE if M <= 2^(log2_bound + 1).
 * Outputs (host): |X| as little-endian uint64 limbs in limbs[0..*nlimbs),
 * *sign in {-1, 0, 1}, and, if residues_out != NULL, the k residues.
 * Synchronous.  Errors: PERM_EINVAL (k < 1, a modulus that is not an odd
 * prime below 2^31, duplicate primes), PERM_ERANGE (bound, or max_limbs too
 * small). */
int perm_crt_int(perm_ctx *ctx, const uint32_t *mats, const uint32_t *primes, int k, int n,
                 double log2_bound, uint64_t *limbs, int max_limbs, int *nlimbs, int *sign,
                 uint32_t *residues_out, unsigned flags, void *stream);

/* One matrix of a ragged batch. */
typedef struct {
    uint64_t offset;   /* byte offset of the matrix inside `data` */
    int32_t n;         /* order, 0..PERM_NMAX */
    int32_t field;     /* PERM_C128, PERM_F64 or PERM_MODP */
    uint32_t p;        /* modulus for PERM_MODP (odd, 3 <= p < 2^31), else ignored */
    uint32_t reserved; /* must be 0 */
} perm_item;

/* Ragged batch in one persistent launch (paper Sec. 3.1 samples many
 * matrices of one size; here any mix of fields and orders).
 * items: host array of `count`.  data: dev-or-host buffer holding every
 * matrix (offset aligned to 8 bytes for floats, 4 for F_p).  out: dev-or-host,
 * 16 bytes per item: c128 (re, im); f64 (value, 0.0); F_p (uint32 residue,
 * then 12 zero bytes).  On PERM_EINVAL, *bad_index (if non-NULL) names the
 * first offending item, or -1 for a bad non-item argument. */
int perm_batch(perm_ctx *ctx, const perm_item *items, int count, const void *data, void *out,
               int *bad_index, unsigned flags, void *stream);

/* Unscaled Glynn partial sum over Gray indices [x0, x1) of one matrix:
 *   S = sum_{x0 <= x < x1} (-1)^x prod_i r_i(x)
 * (so perm = 2^-(n-1) S over the full range [0, 2^(n-1))).  Additive over
 * disjoint ranges: the hook for splitting one permanent across calls or
 * devices and for resuming long runs.  out16: host, 16 bytes in the perm_batch
 * slot format (F_p: S mod p).  Synchronous.
 * Errors: PERM_EINVAL (n < 1, x0 > x1, x1 > 2^(n-1)). */
int perm_range(perm_ctx *ctx, const perm_item *item, const void *data, uint64_t x0, uint64_t x1,
               void *out16, unsigned flags, void *stream);

/* Walk-kernel timing.  While enabled, the context records a pair of HIP
 * events around every walk-kernel launch, on the stream the kernel runs on
 * (a launch of one block that stages and finalizes its call's matrices
 * includes that work; a server created on the context records its walk
 * launches too).  Enabling creates events for max(256, on) launches up front
 * (at most 65,536); past that, library calls create more while a server's
 * launches go unrecorded;
 * recording a pair still adds about 9 us to a call's turnaround on the
 * stream, so time small calls' throughput with timing off.  perm_prof_read waits for the
 * recorded launches, returns their summed device time in milliseconds and
 * their count, and clears the record.  Errors: PERM_EINVAL (NULL),
 * PERM_EDEVICE (event creation or timing failed). */
int perm_prof_enable(perm_ctx *ctx, int on);
int perm_prof_read(perm_ctx *ctx, double *walk_ms, uint64_t *launches);

/* ---------------------------------------------------------------- helpers
 * Host-only; no device needed. */

/* The smallest primes p = 1 (mod n) with 2^30 < p < 2^31, ascending: the
 * least count whose product M satisfies M^2 > 4 n^n (i.e. M > 2 n^(n/2), the
 * Schur bound of paper Sec. 2.1), plus `extra` more.  *k receives the count.
 * Errors: PERM_EINVAL (n < 1), PERM_ERANGE (max_primes too small). */
int perm_schur_primes(int n, int extra, uint32_t *primes, int max_primes, int *k);
/* The same primes under the name the interface plan gives the helper. */
int perm_pick_primes(int n, int extra, uint32_t *primes, int max_primes, int *k);

/* The Schur residue matrix (g^(jk) mod p), j,k = 0..n-1, with g the primitive
 * n-th root of unity h^((p-1)/n) for the smallest h >= 2 of exact order n
 * (paper Sec. 2.1).  out: host, n*n uint32.
 * Errors: PERM_EINVAL (p not prime, p != 1 mod n). */
int perm_schur_residues(int n, uint32_t p, uint32_t *out);

/* Garner lift of k residues to the signed integer X, |X| < M/2 (the host
 * step of perm_crt_int, exposed for testing and for residues computed
 * elsewhere, e.g. by perm_range over split ranges). */
int perm_crt_lift(const uint32_t *residues, const uint32_t *primes, int k, double log2_bound,
                  uint64_t *limbs, int max_limbs, int *nlimbs, int *sign);

/* Redundant-prime check of a CRT result, for long exact runs (paper Sec. 2.1
 * lifts one residue per prime; with one prime more than the bound needs, a
 * residue corrupted by a device or memory fault is detected and named).
 * Lifts all k residues and each of the k subsets that leave one out; every
 * such subset's product must still exceed 2^(log2_bound + 1) (else
 * PERM_ERANGE).  All k + 1 lifts equal: *bad = -1 and the value.  Otherwise,
 * if exactly one left-out residue j gives a lift with |X| <= 2^log2_bound,
 * residue j is the corrupted one: *bad = j and that lift is the value.
 * Otherwise PERM_ERANGE ("residues inconsistent").  Outputs as in
 * perm_crt_lift.  Host-only. */
int perm_crt_check(const uint32_t *residues, const uint32_t *primes, int k, double log2_bound,
                   uint64_t *limbs, int max_limbs, int *nlimbs, int *sign, int *bad);

/* -------------------------------------------------------- checkpointed job
 * An exact integer permanent from k residue matrices (as perm_crt_int) for
 * runs too long for one call: the Glynn index range [0, 2^(n-1)) of every
 * prime is cut into pieces of 2^piece_log2 indices, each piece's unscaled
 * partial sum mod p (perm_range) is appended to a checkpoint file as soon as
 * it is known, and a job created on an existing file resumes where it
 * stopped.  Pieces of all primes run together in one persistent launch per
 * batch.  The result is exact and independent of the piece size and of how
 * often the run was interrupted (paper Sec. 2.1 and 2.3: CRT over primes
 * and the multi-hour exact runs).
 *
 * perm_job_create: mats host, k x n x n uint32 (entries < p_i), copied.
 *   primes distinct odd primes < 2^31 with product M > 2^(log2_bound + 1).
 *   piece_log2 in [10, n - 1] (0: n - 9, at least 10).  checkpoint_path NULL
 *   or "": no file.  A file that exists must have been written for the same
 *   (n, primes, matrices, piece_log2), else PERM_EINVAL; a torn last line
 *   (no newline, from a write cut short) is cut off the file.  The file is
 *   held open for appending.
 * perm_job_run: runs batches of pieces until all are done or `seconds` of
 *   wall time have passed (at least one batch); *done / *total receive the
 *   piece counts (either may be NULL).  Every finished batch is on disk
 *   (fflush + fsync) before it returns.
 * perm_job_result: residues (k, may be NULL) and the signed integer as in
 *   perm_crt_int; PERM_EAGAIN while pieces remain.
 * Errors: PERM_EINVAL, PERM_ERANGE, PERM_ENOMEM, PERM_EDEVICE; file errors
 * are PERM_EINVAL with the reason in perm_last_error. */
typedef struct perm_job perm_job;
int perm_job_create(perm_ctx *ctx, const uint32_t *mats, const uint32_t *primes, int k, int n,
                    double log2_bound, int piece_log2, const char *checkpoint_path,
                    perm_job **out);
int perm_job_run(perm_job *job, double seconds, uint64_t *done, uint64_t *total);
int perm_job_result(perm_job *job, uint32_t *residues, uint64_t *limbs, int max_limbs,
                    int *nlimbs, int *sign);
void perm_job_destroy(perm_job *job);

/* ------------------------------------------------------------ tuning table
 * The work partition of a permanent: each wavefront item covers 64 lanes x
 * 2^log2_chunk Gray indices.  The table maps (field, n) to log2_chunk; it
 * changes float results in the last bits (summation order) and nothing
 * else. */
typedef struct {
    int log2_chunk;    /* per-lane chunk length, 0..24 (0 = library default) */
    int grid_per_cu;   /* persistent blocks per compute unit (0 = occupancy limit) */
} perm_tune;

int perm_tune_get(perm_ctx *ctx, int field, int n, perm_tune *out);
int perm_tune_set(perm_ctx *ctx, int field, int n, const perm_tune *t);

/* Measure candidate chunk lengths for `field` at orders n_lo..n_hi on the
 * context's device (batches of `batch` random matrices per order, or one
 * matrix when batch <= 1) and store the fastest in the table.  Jobs below
 * 2^28 Glynn terms try every length from 3 up and keep the best of five
 * timings; larger ones try the default +-4, timed once. */
int perm_autotune(perm_ctx *ctx, int field, int n_lo, int n_hi, int batch);

/* Save / load the table as text lines "field n log2_chunk grid_per_cu",
 * keyed by the header lines "# arch <gcnArchName>" and "# hip <HIP runtime
 * version>".  Loading checks the key against the context's device and the
 * running HIP runtime, and every line (F_p chunk lengths at most 20): a
 * table without the key lines, tuned for another architecture or runtime,
 * or with a bad line is refused with PERM_EINVAL and the context's table is
 * left as it was. */
int perm_tune_save(perm_ctx *ctx, const char *path);
int perm_tune_load(perm_ctx *ctx, const char *path);

/* ---------------------------------------------------------------- serving
 * A request loop with continuous batching.  Requests (one matrix each) are
 * admitted while the HBM and in-flight budgets allow, their work is split
 * into wavefront items and executed in bounded-duration slices that mix all
 * admitted requests, so requests arriving while others run join the next
 * slice.  Each result is bit-identical to perm_batch on the same matrix. */
typedef struct perm_srv perm_srv;

typedef struct {
    size_t hbm_budget;      /* device bytes for admitted requests (0 = 1 GiB) */
    int max_inflight;       /* admitted requests at once (0 = 4096) */
    int max_pending;        /* queued, not yet admitted; submit beyond -> PERM_EAGAIN (0 = 65536) */
    double slice_us;        /* target GPU time per slice in microseconds (0 = 500) */
    unsigned flags;         /* PERM_NO_KAHAN, PERM_MONTGOMERY */
} perm_srv_cfg;

typedef struct {
    uint64_t submitted, admitted, completed, failed, canceled;
    uint64_t slices;
    double p50_us, p99_us, mean_us, max_us;   /* submit -> result visible, completed requests */
    double terms;                             /* Glynn terms executed */
    double busy_s;                            /* wall time with work on the device */
    uint64_t items;                           /* wave items launched (all slices) */
    double rate;                              /* current calibrated device rate, work units/s
                                                 (a unit: one lane-step of an order-n walk = n) */
} perm_srv_stats;

int perm_srv_create(perm_ctx *ctx, const perm_srv_cfg *cfg, perm_srv **out);
/* Copy one matrix (host memory, layout as in perm_batch with offset 0) into
 * the server; *ticket identifies the request.  Errors: PERM_EINVAL,
 * PERM_EAGAIN (pending queue full), PERM_ENOMEM (matrix larger than the
 * whole budget). */
int perm_srv_submit(perm_srv *srv, const perm_item *item, const void *matrix, uint64_t *ticket);
/* *done = 1 and out16 filled (perm_batch slot format) once finished; returns
 * the request's status (PERM_OK, PERM_ECANCELED, PERM_EDEVICE) when done,
 * PERM_OK with *done = 0 while running, PERM_ENOTFOUND for an unknown or
 * already collected ticket.  latency_us (optional) receives the time from
 * submit to the result becoming visible on the host.  A finished ticket is
 * forgotten after it is reported done. */
int perm_srv_poll(perm_srv *srv, uint64_t ticket, void *out16, int *done, double *latency_us);
/* Block until the ticket finishes or timeout_s passes (then *done = 0). */
int perm_srv_wait(perm_srv *srv, uint64_t ticket, double timeout_s, void *out16, int *done,
                  double *latency_us);
/* Where a request's time went, in microseconds of host time: queued_us from
 * submit to admission (device memory and a descriptor slot granted),
 * admitted_us from admission to the launch of the first slice carrying its
 * work, running_us from that launch to the result becoming visible on the
 * host; latency_us is their sum.  A phase the request never reached (it
 * was cancelled or failed before) is 0 and the time goes to the last phase
 * it reached. */
typedef struct {
    double queued_us, admitted_us, running_us, latency_us;
} perm_srv_times;
/* perm_srv_wait, reporting the phases of the request's latency in *times
 * (optional, filled once *done = 1). */
int perm_srv_wait_times(perm_srv *srv, uint64_t ticket, double timeout_s, void *out16, int *done,
                        perm_srv_times *times);
int perm_srv_cancel(perm_srv *srv, uint64_t ticket);
int perm_srv_get_stats(perm_srv *srv, perm_srv_stats *out);
/* Stop accepting, finish or cancel everything, join the worker. */
void perm_srv_destroy(perm_srv *srv);

#ifdef __cplusplus
}
#endif
#endif /* PERM_H */
