/*
 * adanns.h - C ABI of the MI355X (gfx950) AdANNS-IVF / IVF-PQ search library.
 *
 * The operations follow the paper's problem statement and Algorithm 1
 * (AdANNS, arXiv 2305.19435): a database of N points embedded in R^d by a
 * Matryoshka representation (Section 3), an IVF index built by clustering
 * the first d_c coordinates (Section 4.1; Algorithm 1, construction), and a
 * search that assigns each query to its nprobe nearest centroids on the
 * first d_c coordinates, scans the probed inverted lists with the first d_s
 * coordinates and returns the k nearest (Algorithm 1, inference; Appendix A,
 * Table "formula", AdANNS-IVF and AdANNS-IVF-D rows).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Pointers named as "device" must point to memory of the current HIP
 *   device (e.g. torch tensors); "host" pointers to ordinary host memory.
 *   Caller-owned buffers stay owned by the caller; the library copies what
 *   it keeps into its own device memory, owned by the index object.
 * - Matrices are row-major; ``ld*`` is the row stride in elements.
 * - ``stream`` is a hipStream_t (NULL = the default stream). Searches are
 *   enqueued on it and return without waiting for the device, except that a
 *   call may synchronise ``stream`` once to grow its scratch memory.
 * - Distances are squared L2 in FP32, ascending, ties broken by the smaller
 *   id. When fewer than k candidates exist the trailing slots hold id -1 and
 *   distance +inf. Probe lists are sorted by (centroid distance, list index).
 * - Every function returns an adanns_status and never throws. Arguments are
 *   validated before any device work; on error the outputs are untouched and
 *   adanns_last_error() (thread-local) says why. A HIP failure of an earlier
 *   asynchronous launch surfaces as ADANNS_EHIP. nq = 0 is a no-op.
 * - A built index is read-only during searches; searches on different
 *   streams may run concurrently (each stream gets its own scratch memory).
 */
#ifndef ADANNS_H
#define ADANNS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct adanns_index adanns_index; /* opaque, library-owned */

typedef enum adanns_status {
  ADANNS_OK = 0,
  ADANNS_EINVAL = -1,      /* invalid argument */
  ADANNS_ENOMEM = -2,      /* device or host allocation failed */
  ADANNS_EHIP = -3,        /* a HIP runtime call or kernel launch failed */
  ADANNS_EUNSUPPORTED = -4,/* valid request this library does not support */
  ADANNS_EBUDGET = -5,     /* request exceeds an admission budget */
  ADANNS_EIO = -6          /* a file could not be opened, read or written, or is malformed */
} adanns_status;

/* Element type of a database matrix handed to the library. Half elements
 * convert exactly to FP32; the index stores FP32. */
typedef enum adanns_dtype {
  ADANNS_DTYPE_F32 = 0,
  ADANNS_DTYPE_F16 = 1     /* IEEE binary16 */
} adanns_dtype;

typedef enum adanns_format {
  ADANNS_FP32 = 0,
  ADANNS_BF16 = 1,         /* round-to-nearest-even bfloat16 */
  ADANNS_FP8_E4M3 = 2      /* OCP e4m3, one FP32 scale per vector */
} adanns_format;

/* Thread-local text of the last error ("" if none). Never NULL. */
const char *adanns_last_error(void);

/* Library version string. */
const char *adanns_version(void);

/*
 * Import an IVF index whose clustering was computed elsewhere (Section 3,
 * "Inverted File Index": centroids plus the inverted file of each cluster's
 * members; Algorithm 1, construction on the d_c_build prefix).
 *   X         device, [n x d] rows of element type ``dtype`` (adanns_dtype),
 *             row stride ldx >= d elements. Copied (converted to FP32).
 *   centroids device, [nlist x d_c_build] FP32, row stride d_c_build. Copied.
 *   assign    device, [n] int32, the list of each row, each in [0, nlist).
 * Lists keep their members in ascending row order; a row's id is its index
 * in X. Requirements: n >= 1, 1 <= d <= 8192, 1 <= nlist <= 65536,
 * 1 <= d_c_build <= d, n < 2^31. Synchronises ``stream``.
 * On success *out owns the index; release it with adanns_index_free().
 */
adanns_status adanns_ivf_import(const void *X, int64_t n, int32_t d, int64_t ldx, int32_t dtype,
                                const float *centroids, int32_t nlist, int32_t d_c_build,
                                const int32_t *assign, void *stream, adanns_index **out);

/*
 * Build an IVF index on the GPU: Lloyd's k-means on X[:, :d_c] (Section 3,
 * "Inverted File Index"; Section 4.1; Algorithm 1, construction), then one
 * final assignment of every row, which defines the inverted lists.
 *   X          device, [n x d] of element type ``dtype``, row stride ldx >= d
 *              elements. Copied (converted to FP32).
 *   train_rows host, [n_train] int64 rows of X the iterations run on, or
 *              NULL for all rows (then n_train is ignored).
 *   init_rows  host, [nlist] int32 indices into the training rows: the
 *              initial centroids (the caller draws them, e.g. the first
 *              nlist entries of a seeded permutation).
 *   iters      assign/update rounds, 0..1000. Assignment ties go to the
 *              smaller centroid index; an empty cluster keeps its centroid.
 *   objective  host, [iters + 1] doubles or NULL: the k-means objective on
 *              the training rows after each assignment, the last entry after
 *              the final assignment.
 * Centroids are FP32 (each update is a compensated-sum mean rounded to
 * FP32). Limits as adanns_ivf_import; the training set must hold at least
 * nlist rows. Synchronises ``stream``; allocates temporary device memory.
 */
adanns_status adanns_build_ivf(const void *X, int64_t n, int32_t d, int64_t ldx, int32_t dtype,
                               int32_t nlist, int32_t d_c, int32_t iters, const int32_t *init_rows,
                               const int64_t *train_rows, int64_t n_train, double *objective,
                               void *stream, adanns_index **out);

/* Search scratch (staged queries, scores, buckets and every candidate's
 * first-pass value) grows with nq. adanns_search, adanns_search_probes,
 * adanns_search_pq and adanns_search_precision split a batch whose scratch
 * would exceed ``bytes`` into query chunks run one after another on the
 * stream (results unchanged). 0 restores the default of 32 GiB.
 * Process-wide; affects calls made afterwards. */
adanns_status adanns_set_search_scratch_cap(size_t bytes);

/*
 * AdANNS-IVF search (Algorithm 1, inference; Appendix A, Table "formula"):
 * probes = the nprobe clusters nearest to Q[i, :d_c] on the centroids'
 * first d_c coordinates; result = the k rows of the probed lists nearest to
 * Q[i, :d_s] on their first d_s coordinates. d_c < d_c_build searches a
 * prefix of the built centroids (AdANNS-IVF-D, Section 5.1).
 *   Q      device, [nq x ldq] FP32, ldq >= max(d_c, d_s).
 *   dist   device, [nq x k] FP32 out.
 *   ids    device, [nq x k] int64 out.
 *   probes device, [nq x nprobe] int32 out, or NULL.
 * Limits: 1 <= d_c <= d_c_build, 1 <= d_s <= d, 1 <= nprobe <= nlist,
 * 1 <= k <= 1024.
 */
adanns_status adanns_search(const adanns_index *index, const float *Q, int64_t nq, int64_t ldq,
                            int32_t d_c, int32_t d_s, int32_t nprobe, int32_t k,
                            float *dist, int64_t *ids, int32_t *probes, void *stream);

/*
 * adanns_search for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same kernels and results, bit for bit, but the search scratch (staged
 * queries, coarse scores, probes, buckets, first-pass values, re-selection
 * list) lives in a fixed device array of adanns_search_noalloc_max_bytes()
 * = 64 MiB that the library holds on every GPU it runs on until the process
 * ends, instead of the index's per-stream workspace. The call allocates
 * nothing (no hipMalloc / hipFree, no torch allocation, no events: kernel
 * timing is suspended for it); its first call on a device looks up the
 * array's device address once.
 *   Arguments, limits and result conventions: as adanns_search.
 * Errors: as adanns_search, and ADANNS_EBUDGET (outputs untouched) when the
 * batch needs more scratch than the array holds (about nq * (top-nprobe list
 * lengths + nlist + max(d_c, d_s)) * 4 bytes): search fewer queries per call.
 * Every call on a GPU shares that GPU's array, so calls that overlap on one
 * GPU (several streams or threads at once) race and must be serialised by
 * the caller; the array keeps the last call's contents, and every search
 * clears what it needs cleared itself.
 */
adanns_status adanns_search_noalloc(const adanns_index *index, const float *Q, int64_t nq,
                                    int64_t ldq, int32_t d_c, int32_t d_s, int32_t nprobe,
                                    int32_t k, float *dist, int64_t *ids, int32_t *probes,
                                    void *stream);

/* Bytes of the fixed scratch array of adanns_search_noalloc (64 MiB). */
size_t adanns_search_noalloc_max_bytes(void);

/*
 * Same as adanns_search with the probe lists given instead of computed:
 *   probes device, [nq x nprobe] int32, each in [0, nlist), no repeats
 *          within a row; both are checked (ADANNS_EINVAL), which copies the
 *          probes to the host and synchronises ``stream``.
 * Used to check the list scan on its own.
 */
adanns_status adanns_search_probes(const adanns_index *index, const float *Q, int64_t nq,
                                   int64_t ldq, int32_t d_s, int32_t nprobe,
                                   const int32_t *probes, int32_t k, float *dist,
                                   int64_t *ids, void *stream);

/*
 * Attach a product-quantisation codec to an index (Section 3, "Optimized
 * Product Quantization"; Section 4.2 AdANNS-OPQ; Section 4.3 AdANNS-IVFOPQ):
 * the first d_s coordinates of a vector, rotated by R, are split into M
 * blocks of d_s/M coordinates and each block is replaced by the index of
 * its nearest codeword (256 per block, one byte).
 *   R         device, [d_s x d_s] FP32 row-major (q' = q[:d_s] R), or NULL
 *             for the identity (plain PQ). Copied.
 *   codebooks device, [M x 256 x d_s/M] FP32. Copied.
 *   codes     device, [n x M] uint8, row j = database row j. Copied into
 *             list order.
 * Limits: M a multiple of 4 in [4, 64], M divides d_s, d_s <= min(d, 2048),
 * one codec per M. Synchronises ``stream``.
 */
adanns_status adanns_pq_import(adanns_index *index, int32_t M, int32_t d_s, const float *R,
                               const float *codebooks, const uint8_t *codes, void *stream);

/*
 * Train and attach a PQ codec on the GPU for a given rotation R (device
 * [d_s x d_s] row-major, or NULL for the identity): the training rows'
 * first d_s coordinates are rotated (y = x[:d_s] R, compensated FP32), then
 * for each of the M blocks of d_s/M coordinates Lloyd's k-means with 256
 * codewords runs on them (as adanns_build_ivf: init_rows, host [256] int32,
 * index the training rows; train_rows host [n_train] int64 or NULL = all
 * rows; iters rounds); then every row of X is rotated and encoded by its
 * nearest codeword per block (FP32 difference form, ties to the smaller
 * index). The rotation is not learned here (no Procrustes step); a learned
 * OPQ rotation and its codebooks can be attached with adanns_pq_import.
 *   X  device, the index's database [n x d] of element type ``dtype`` (row j =
 *      id j), stride ldx elements.
 * Limits: as adanns_pq_import, and d_s / M <= 32. Synchronises ``stream``.
 */
adanns_status adanns_pq_train(adanns_index *index, const void *X, int64_t ldx, int32_t dtype,
                              int32_t M, int32_t d_s, const float *R, int32_t iters,
                              const int32_t *init_rows, const int64_t *train_rows,
                              int64_t n_train, void *stream);

/*
 * Optimized product quantisation trained on the GPU (Section 3, "Optimized
 * Product Quantization": a learned orthonormal rotation before PQ, the
 * non-parametric method of Ge et al. that the paper names; Section 4.3
 * AdANNS-IVFOPQ). On the training rows' first d_s coordinates X:
 *   R = R_init; then ``outer`` times { Y = X R; PQ k-means on Y (pq_iters Lloyd
 *   rounds per block, from init_rows the first time, then from the previous
 *   codebooks); Yhat = the decoded codes of Y; R = the orthonormal R that
 *   minimises |X R - Yhat|_F, the orthogonal polar factor of X^T Yhat
 *   (adanns_polar_factor) }; then a last PQ k-means on X R from the previous
 *   codebooks. Every row of the index is then rotated and encoded and the
 *   codec attached as by adanns_pq_import (R, codebooks, codes).
 *   X          device, the index's database [n x d] of element type ``dtype``
 *              (row j = id j), stride ldx elements.
 *   R_init     device [d_s x d_s] FP32 orthonormal starting rotation, or NULL
 *              for the identity (the alternation only lowers the distortion
 *              from where it starts, so a start that spreads the variance
 *              over the blocks, e.g. a random rotation, matters).
 *   init_rows  host [256] int32, indices into the training rows.
 *   train_rows host [n_train] int64 rows of X to train on, or NULL (all).
 *   distortion host [outer + 1] or NULL: sum over the training rows of
 *              |Y - Yhat|^2 after each PQ training (non-increasing: each step
 *              minimises it with the other held fixed).
 * Rotations and products accumulate in FP64; codebooks are FP32.
 * Limits: as adanns_pq_train; 0 <= outer <= 100; 0 <= pq_iters <= 1000.
 * Errors: ADANNS_EINVAL, ADANNS_ENOMEM, ADANNS_EHIP, ADANNS_EUNSUPPORTED (the
 * rotation step met a singular X^T Yhat). Synchronises ``stream``.
 */
adanns_status adanns_opq_train(adanns_index *index, const void *X, int64_t ldx, int32_t dtype,
                               int32_t M, int32_t d_s, const float *R_init, int32_t outer,
                               int32_t pq_iters, const int32_t *init_rows,
                               const int64_t *train_rows, int64_t n_train, double *distortion,
                               void *stream);

/*
 * The orthogonal polar factor of a square matrix (the solution of the
 * orthogonal Procrustes problem inside OPQ training): for A = U S V^T
 * (S > 0), R = U V^T, the orthonormal matrix nearest to A.
 *   A, R       device, [d x d] FP64 row-major (A unchanged).
 *   iterations host out or NULL: Newton-Schulz steps taken.
 * Computed by the Newton-Schulz iteration Z <- 1.5 Z - 0.5 Z Z^T Z from
 * A / |A|_F in FP64 until a step changes Z by less than 1e-13 |Z|_F (at most
 * 200 steps). Limits: 1 <= d <= 4096. Errors: ADANNS_EINVAL, ADANNS_ENOMEM,
 * ADANNS_EHIP, ADANNS_EUNSUPPORTED (Z^T Z not the identity to 1e-9 at the end:
 * A singular or too ill-conditioned). Synchronises ``stream``.
 */
adanns_status adanns_polar_factor(const double *A, int32_t d, double *R, int32_t *iterations,
                                  void *stream);

/* A codec as stored: R host [d_s x d_s], codebooks host [M x 256 x d_s/M],
 * codes host [n x M] in database-id order. Any may be NULL. Synchronous. */
adanns_status adanns_pq_codec(const adanns_index *index, int32_t M, float *R, float *codebooks,
                              uint8_t *codes);

/*
 * AdANNS-IVF-PQ search (Section 4.3; Appendix A, Table "formula", IVFOPQ
 * row, read with an unquantised query): probes from the unrotated d_c
 * prefix as in adanns_search; the probed lists are scanned with the
 * asymmetric distance D(x) = sum_m |q'_m - C_m[code_m(x)]|^2 (tables held
 * in LDS); with rerank_k > 0 the rerank_k best by that distance are
 * re-ranked by the exact squared L2 distance on the first d_rerank
 * coordinates of the index's FP32 vectors (shortlist, then re-rank with the
 * high-dimensional representation) and dist holds those exact distances.
 *   M      selects the codec. k in [1, 1016]; rerank_k 0 or in [k, 1016].
 * Other arguments and conventions as adanns_search.
 */
adanns_status adanns_search_pq(const adanns_index *index, const float *Q, int64_t nq, int64_t ldq,
                               int32_t d_c, int32_t nprobe, int32_t M, int32_t k,
                               int32_t rerank_k, int32_t d_rerank, float *dist, int64_t *ids,
                               int32_t *probes, void *stream);

/*
 * Precision form (Section 4.3: a cheap first pass builds a shortlist that is
 * re-ranked with the full-precision representation). Builds a low-precision
 * copy of the index's vectors and centroids: fmt ADANNS_BF16 (round to
 * nearest even) or ADANNS_FP8_E4M3 (OCP e4m3, one FP32 scale per vector,
 * scale = max|x| / 448 over the vector's d coordinates, codes of
 * x * (448 / max|x|) rounded to nearest even, saturating). Idempotent.
 * Synchronises ``stream``.
 */
adanns_status adanns_set_precision(adanns_index *index, int32_t fmt, void *stream);

/*
 * Optional row-major FP32 copy of the index's vectors (rows in list order,
 * d_pad floats each), read by every exact re-measurement of a shortlist
 * (the FP32 distance of Appendix A's formula table, after any first pass)
 * instead of the list slab layout: each candidate then becomes one
 * contiguous read instead of one 128-byte piece per 32 coordinates. Costs
 * rows_pad x d_pad x 4 bytes of device memory, held until the index is
 * freed; results are bit-identical with and without it. Searches and
 * batches created after this call use it; batches created before keep
 * reading the slab layout. Idempotent. Synchronises ``stream``.
 * Errors: ADANNS_EINVAL (NULL index, no FP32 vectors), ADANNS_ENOMEM,
 * ADANNS_EHIP.
 */
adanns_status adanns_index_add_row_copy(adanns_index *index, void *stream);

/*
 * Precision-form search. Queries are quantised the same way (one scale per
 * query over its first d coordinates, so ldq >= d). Coarse: first-pass
 * scores of quantised query and centroid prefixes on BF16 / FP8 MFMA with
 * FP32 accumulation; the nprobe + coarse_margin best by the exact distance
 * between the quantised values, then the nprobe nearest by exact FP32
 * centroid distance. Scan: first-pass distances of quantised query and
 * vectors on MFMA; the rerank_k best by the exact distance between the
 * quantised values; those re-ranked by the exact squared L2 distance on the
 * FP32 vectors' first d_s coordinates; dist holds those exact distances.
 * Needs adanns_set_precision(fmt) first. 1 <= k <= rerank_k <= 1016,
 * nprobe + coarse_margin <= 1016. Other conventions as adanns_search.
 */
adanns_status adanns_search_precision(const adanns_index *index, const float *Q, int64_t nq,
                                      int64_t ldq, int32_t d_c, int32_t d_s, int32_t nprobe,
                                      int32_t k, int32_t fmt, int32_t rerank_k,
                                      int32_t coarse_margin, float *dist, int64_t *ids,
                                      int32_t *probes, void *stream);

/*
 * adanns_search's result (Algorithm 1, inference: the exact k nearest in
 * FP32 of the probed lists' rows on their first d_s coordinates; the same
 * FP32 coarse step and probes) computed with a quantised first pass over
 * the lists: the list scan runs on the BF16 or e4m3 copy
 * (adanns_set_precision) on BF16 / FP8 matrix cores, and only candidates
 * whose FP32 distance can still be among the k nearest are measured exactly
 * in FP32. A candidate's FP32 distance lies within
 * (sqrt(D^) -/+ (|q - q^| + |x - x^|))^2 of the exact distance D^ between the
 * quantised values (triangle inequality; |x - x^| is the row's own
 * quantisation error, stored with the copy), and D^ within the first pass's
 * rounding bound of its first-pass value; candidates whose lower bound
 * exceeds the k-th smallest FP32 distance found so far are skipped. The
 * exact measure is the one adanns_search uses, so dist, ids and probes equal
 * adanns_search's bit for bit. Needs adanns_set_precision(fmt) first;
 * ldq >= d (queries are quantised over all d coordinates); 1 <= k <= 128.
 * Other arguments and conventions as adanns_search. Errors: ADANNS_EINVAL
 * (arguments out of range, fmt not 1 or 2, no copy in fmt), ADANNS_ENOMEM
 * (search scratch), ADANNS_EHIP.
 */
adanns_status adanns_search_filtered(const adanns_index *index, const float *Q, int64_t nq,
                                     int64_t ldq, int32_t d_c, int32_t d_s, int32_t nprobe,
                                     int32_t k, int32_t fmt, float *dist, int64_t *ids,
                                     int32_t *probes, void *stream);

/*
 * The low-precision copy as stored, in database-id order: values host/*
 * The low-precision copy as stored, in database-id order: values host
 * [n x d] (uint16 bf16 bits, or e4m3 bytes), scales host [n] FP32 (1 for
 * bf16). Either may be NULL. Synchronous; for tests and tools.
 */
adanns_status adanns_index_quantized(const adanns_index *index, int32_t fmt, void *values,
                                     float *scales);

/*
 * Kernel timing with HIP events, for measurement tools. While enabled, every
 * search records an event pair around each of its kernel groups on its
 * stream ("tile_dist_coarse", "select_coarse", "bucketing",
 * "tile_dist_scan", "select_scan", and the variants of the other search
 * forms). adanns_timing_read() waits for the recorded events and returns the
 * number of timed launches and their total milliseconds since the last
 * reset; unknown names read as 0 launches. Process-wide; thread-safe.
 */
adanns_status adanns_timing_enable(int32_t enable);
adanns_status adanns_timing_reset(void);
adanns_status adanns_timing_read(const char *kernel, int64_t *launches, double *total_ms);

/*
 * Certificate counters of the shortlists (Algorithm 1's linear scan returns
 * the exact k nearest of the candidates; here a cheaper first pass orders
 * them and only a shortlist is re-measured exactly). Every selection keeps
 * the candidates whose first-pass value, widened by the first pass's
 * rounding-error bound (or IVF-PQ's table-sum bound), can still reach the
 * k nearest (the nprobe nearest centroids, the rerank_k nearest by the
 * quantised measure), however many there are; a query whose band outgrows
 * the one-wave list is selected again by a re-selection launch with up to
 * 4096 slots (LDS permitting). Counts since the last reset, over every search
 * on the current device:
 *   reselected   host out, queries handed to the re-selection launch (or NULL);
 *   uncertified  host out, queries whose band held more candidates than the
 *                largest shortlist (those results are the nearest of the
 *                first-pass best only), or NULL.
 * reset != 0 zeroes both after reading. Synchronises the current device.
 * Errors: ADANNS_EHIP.
 */
adanns_status adanns_selection_stats(int64_t *reselected, int64_t *uncertified, int32_t reset);

/*
 * Diagnostics of adanns_search_filtered (the work its filter leaves, not a
 * result): counts since the last reset over every such search on the current
 * device:
 *   measured  host out, candidates measured exactly in FP32 (or NULL);
 *   windowed  host out, queries whose candidates that can still reach the k
 *             nearest outgrew the free slots, so that they were taken in
 *             several windows of increasing lower bound (or NULL).
 * reset != 0 zeroes both after reading. Synchronises the current device.
 * Errors: ADANNS_EHIP.
 */
adanns_status adanns_filtered_stats(int64_t *measured, int64_t *windowed, int32_t reset);

/*
 * Measurement utility (not part of the method): reads ``bytes`` of device
 * memory ``buf`` once with 16-byte non-temporal loads (streamed past the
 * caches; a grid of tens of thousands of workgroups reaches the highest
 * rate) and writes one partial sum per
 * workgroup to ``partial`` (device, [grid] FP32), the achievable read-only
 * bandwidth to set beside the scans' rates. Timed under the name
 * "stream_read" when kernel timing is on (adanns_timing_*).
 * Requirements: buf 16-byte aligned, bytes a multiple of 16, 1 <= grid <= 65536.
 * Asynchronous on ``stream``. Errors: ADANNS_EINVAL, ADANNS_EHIP.
 */
adanns_status adanns_stream_read(const void *buf, size_t bytes, float *partial, int32_t grid,
                                 void *stream);

/*
 * Batching form: many search configurations, each with its own index,
 * (d_c, d_s, nprobe, k) and query batch, run as one set of persistent
 * launches over a descriptor table (coarse tiles of every configuration in
 * one launch, list-scan tiles of every configuration in one launch, one
 * selection launch per step), optionally captured into a hipGraph.
 * Results equal those of adanns_search on each configuration alone.
 *
 * Queries are one row-major array holding the configurations' queries one
 * after another (config 0 first), row stride ldq >= every max(d_c, d_s);
 * dist / ids are [total queries x ldk] with ldk >= every k; row r of a
 * configuration with k < ldk fills its first k entries. probes (optional)
 * is [sum of nq * nprobe] int32 in configuration order.
 */
typedef struct adanns_batch_config {
  const adanns_index *index;
  int64_t nq;
  int32_t d_c, d_s, nprobe, k;
} adanns_batch_config;

typedef struct adanns_batch adanns_batch; /* opaque, library-owned */

/* Validates the configurations, sizes and allocates the batch's scratch
 * memory and uploads the descriptors. Synchronises ``stream``. The indices
 * must outlive the batch. Uses the autotune cache if it knows the shape. */
adanns_status adanns_batch_create(const adanns_batch_config *cfgs, int32_t ncfg, int64_t ldq,
                                  int64_t ldk, void *stream, adanns_batch **out);

/* Enqueues the batch on ``stream``: no allocation, no host synchronisation
 * (capturable). */
adanns_status adanns_batch_run(adanns_batch *batch, const float *Q, float *dist, int64_t *ids,
                               int32_t *probes, void *stream);

/* Like adanns_batch_run, through a hipGraph captured on first use (and
 * again whenever Q, dist or ids change) and replayed afterwards. The graph
 * runs on a private stream of the batch, ordered after the work already on
 * ``stream`` and before work enqueued on it later (events), so ``stream`` may
 * be the default stream. Kernel timing must be off. */
adanns_status adanns_batch_run_graph(adanns_batch *batch, const float *Q, float *dist,
                                     int64_t *ids, void *stream);

/* Scan tile shape: query-tile height tq (32, 64, 128), vector-tile width tv
 * (64, 128) and persistent grid. Results do not depend on the shape. Until
 * set or autotuned, a batch (and adanns_search) uses the autotune cache's
 * shape for its key, else 64 x 128 tiles when probed lists meet at least 32
 * queries on average, else 32 x 64. */
adanns_status adanns_batch_set_shape(adanns_batch *batch, int32_t tq, int32_t tv, int32_t grid);

/* Autotuner: times every (tq, tv, grid) candidate on this batch (one warm-up and
 * ``reps`` timed runs each, HIP events), keeps the fastest for the batch and
 * records it in the process-wide autotune cache under the batch's shape key
 * (d_s, nprobe and queries per list, bucketed by powers of two), which
 * adanns_search and adanns_batch_create consult. Writes dist / ids. */
adanns_status adanns_batch_autotune(adanns_batch *batch, const float *Q, float *dist,
                                    int64_t *ids, int32_t reps, int32_t *tq, int32_t *tv,
                                    int32_t *grid, void *stream);

/* Total queries, current shape and scratch bytes of a batch (NULL-able). */
adanns_status adanns_batch_info(const adanns_batch *batch, int64_t *queries, int32_t *tq,
                                int32_t *tv, int32_t *grid, size_t *scratch_bytes);

/* Releases a batch (waits for the device; NULL is a no-op). */
void adanns_batch_free(adanns_batch *batch);

/* Forgets every autotuned shape. */
adanns_status adanns_autotune_clear(void);

/*
 * Serving form: an open-loop request loop over the index's PQ codecs
 * (search as adanns_search_pq). Request i (query row i of Q, device
 * [n x ldq]) arrives arrival_s[i] seconds after the call starts (host clock;
 * non-decreasing) with its own budget (d_c[i], nprobe[i], M[i]) (host
 * arrays). hbm_budget bytes of device memory are allocated once, as one
 * region; every search step's scratch (staged queries, coarse scores,
 * probes, buckets, candidate distances, rotated queries, tables: exactly what
 * the search carves) is a piece of it. A host loop admits arrived requests
 * while their step's scratch fits a free piece of the region, batches
 * admitted requests of one budget into a step (the oldest pending request's
 * budget first, at most max_batch requests, as many as the largest free
 * piece holds), runs up to nstreams steps concurrently on streams of their
 * own, and on each step's completion event records the latency of its
 * requests and returns its piece, while newer requests keep being admitted
 * (continuous batching). The memory in use by searches therefore never
 * exceeds hbm_budget (the per-stream step buffers for max_batch staged
 * queries and results, max_batch * (ldq + 3k + 2) * 4 bytes per stream, are
 * outside it). A request whose step alone exceeds the budget is rejected
 * (latency -1). Results go to row i of dist / ids (device [n x k]); latency_s
 * (host [n]) is completion minus arrival. Before the clock starts one request
 * of each budget runs on every stream (kernel loading). Blocks until every
 * request completed; synchronises the device.
 */
typedef struct adanns_serve_stats {
  double wall_s;               /* first arrival window start to last completion */
  int64_t steps;               /* search steps launched */
  double mean_batch;           /* requests per step */
  size_t max_inflight_bytes;   /* peak search scratch in use (never above hbm_budget) */
  int32_t max_streams_busy;    /* peak concurrent steps */
  int64_t rejected;            /* requests larger than the budget */
} adanns_serve_stats;

adanns_status adanns_serve(const adanns_index *index, const float *Q, int64_t ldq, int64_t n,
                           const double *arrival_s, const int32_t *d_c, const int32_t *nprobe,
                           const int32_t *M, int32_t k, int32_t rerank_k, int32_t d_rerank,
                           int32_t nstreams, int32_t max_batch, size_t hbm_budget, float *dist,
                           int64_t *ids, double *latency_s, adanns_serve_stats *stats);

/* Sizes of an index. Any out pointer may be NULL. */
adanns_status adanns_index_info(const adanns_index *index, int64_t *n, int32_t *d,
                                int32_t *nlist, int32_t *d_c_build);

/* The inverted lists as stored: offsets host [nlist + 1] int64, ids host [n]
 * int64 (member ids grouped by list). Either may be NULL. Synchronous. */
adanns_status adanns_index_lists(const adanns_index *index, int64_t *offsets, int64_t *ids);

/* The centroids as stored: host [nlist x d_c_build] FP32. Synchronous. */
adanns_status adanns_index_centroids(const adanns_index *index, float *centroids);

/* Persistence of a built index (the stored form of what Algorithm 1's
 * construction returns: centroids and inverted lists, plus the vectors in
 * their list layout and every PQ codec). adanns_index_save waits for the
 * device, then writes ``path`` (created or truncated). adanns_index_load
 * reads such a file onto the current device on ``stream`` and returns a new
 * index in *out (release with adanns_index_free). Low-precision copies and
 * the row-major re-measure copy are not stored: call adanns_set_precision /
 * adanns_index_add_row_copy again after a load. A file that is
 * not a complete index of this format version gives ADANNS_EIO and leaves
 * *out untouched. */
adanns_status adanns_index_save(const adanns_index *index, const char *path);
adanns_status adanns_index_load(const char *path, void *stream, adanns_index **out);

/* Device bytes held by the index, scratch memory included. */
size_t adanns_index_device_bytes(const adanns_index *index);

/* Release an index and all its device memory (NULL is a no-op). Waits for
 * the device first. */
void adanns_index_free(adanns_index *index);

#ifdef __cplusplus
}
#endif
#endif /* ADANNS_H */
