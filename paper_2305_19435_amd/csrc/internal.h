// Internal declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "adanns.h"

namespace adanns {

// ---- layout constants ------------------------------------------------------
// Vectors are stored per inverted list in "slabs" of SLAB consecutive
// coordinates: element (list h, slab s, row r, t) lives at
//   vec[poff[h] * d_pad + (s * npad_h + r) * SLAB + t],
// with npad_h = poff[h+1] - poff[h] the list's row count rounded up to ROWPAD.
// The first d_s coordinates of a list (d_s a multiple of SLAB) are therefore
// one contiguous span, and a tile of rows x SLAB coordinates is one
// contiguous block of rows * 128 bytes.
constexpr int SLAB = 32;
constexpr int ROWPAD = 64;
constexpr int TILE_Q = 64;     // queries per distance tile
constexpr int TILE_V = 64;     // vectors per distance tile
constexpr int MAX_SHORTLIST = 1024;
constexpr int REFINE_MARGIN = 8;   // extra first-pass candidates re-measured exactly
constexpr int PERSIST_WG = 2048;   // workgroups of the persistent tile kernel (multiple of 8)
// Default largest per-call search scratch before a batch is split into
// query chunks (adanns_set_search_scratch_cap changes it).
constexpr size_t kSearchScratchCap = size_t(32) << 30;

inline int64_t round_up(int64_t a, int64_t b) { return (a + b - 1) / b * b; }
inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

// ---- error handling ----------------------------------------------------------
void set_error(const char *fmt, ...);
void clear_error();

#define ADANNS_HIP(call)                                                          \
  do {                                                                            \
    hipError_t e_ = (call);                                                       \
    if (e_ != hipSuccess) {                                                       \
      ::adanns::set_error("%s failed: %s (%s:%d)", #call, hipGetErrorString(e_), \
                          __FILE__, __LINE__);                                    \
      return ADANNS_EHIP;                                                         \
    }                                                                             \
  } while (0)

#define ADANNS_REQUIRE(cond, ...)         \
  do {                                    \
    if (!(cond)) {                        \
      ::adanns::set_error(__VA_ARGS__);   \
      return ADANNS_EINVAL;               \
    }                                     \
  } while (0)

// ---- per-stream scratch memory ---------------------------------------------
struct Scratch {
  void *base = nullptr;
  size_t bytes = 0;
};

// Carves aligned sub-buffers out of one allocation.
struct Carver {
  char *base;
  size_t off = 0;
  size_t cap;
  template <class T>
  T *take(size_t count) {
    off = (size_t)round_up((int64_t)off, 256);
    T *p = reinterpret_cast<T *>(base + off);
    off += count * sizeof(T);
    return p;
  }
};

}  // namespace adanns

namespace adanns {
// Product-quantisation codec attached to an index (one per M).
struct PqCodec {
  int32_t M = 0, d_s = 0, dsub = 0;
  float *R = nullptr;        // [d_s][d_s] row-major, q' = q[:d_s] R
  float *cb = nullptr;       // [M][256][dsub]
  uint8_t *codes = nullptr;  // [rows_pad][M], layout-row order, zero on padding rows
};
// Low-precision copies of the vectors and centroids (precision form): same
// slab indexing as the FP32 layout, 2-byte (bf16) or 1-byte (e4m3) elements,
// one FP32 scale per stored row for e4m3.
struct QuantStore {
  void *vec = nullptr;
  float *scale = nullptr;       // [rows_pad] (e4m3 only)
  void *cent = nullptr;         // one-list slab layout of nl_pad rows
  float *cent_scale = nullptr;  // [nl_pad] (e4m3 only)
  float *emax = nullptr;        // [1] largest |x - dequantised x| over the rows
  float *rerr = nullptr;        // [rows_pad] |x - dequantised x| of each row (layout order)
  float *cent_emax = nullptr;   // [1] the same over the centroids
};
}  // namespace adanns

struct adanns_index {
  int device = 0;
  int64_t n = 0;
  int32_t d = 0, d_pad = 0, nlist = 0, d_cb = 0, d_cb_pad = 0, nl_pad = 0;
  int64_t rows_pad = 0;
  int32_t max_len = 0;
  std::vector<int64_t> h_off, h_poff;
  std::vector<int32_t> h_len;
  std::vector<int64_t> h_ids;          // member ids grouped by list
  std::vector<int64_t> top_prefix;     // sum of the p largest list lengths, p = 0..nlist
  // device memory owned by the index
  float *vec = nullptr;                // slab layout, rows_pad * d_pad floats
  float *rows = nullptr;               // optional row-major copy of vec [rows_pad][d_pad]
                                       // (list order) read by the exact re-measures
  int64_t *poff = nullptr;             // [nlist + 1]
  int32_t *len = nullptr;              // [nlist]
  int64_t *rowid = nullptr;            // [rows_pad], -1 on padding rows
  float *cent = nullptr;               // [nlist][d_cb_pad] row-major, zero padded
  float *cent_slab = nullptr;          // centroids as one slab-layout list of nl_pad rows
  float *xmax2 = nullptr;              // [1] largest squared row norm of vec, once vec is
                                       // filled (bounds the first pass's rounding error)
  float *cmax2 = nullptr;              // [1] largest squared norm of the centroids
  std::map<int32_t, adanns::PqCodec> pq;   // keyed by M
  adanns::QuantStore quant[3];             // indexed by adanns_format (1 bf16, 2 e4m3)
  size_t own_bytes = 0;
  std::mutex mu;
  std::map<hipStream_t, adanns::Scratch> scratch;
};

namespace adanns {

// Grows (if needed) and returns the scratch memory of ``stream``.
adanns_status get_scratch(adanns_index *ix, hipStream_t stream, size_t bytes, void **out);

// ---- kernel timing with HIP events ------------------------------------------
// When timing is on, a KernelTimer records an event pair around the launches
// in its scope on ``stream``; adanns_timing_read() resolves them.
bool timing_on();
struct KernelTimer {
  const char *name;
  hipStream_t st;
  hipEvent_t a = nullptr, b = nullptr;
  KernelTimer(const char *name, hipStream_t st);
  void stop();
  ~KernelTimer() { stop(); }
};

// ---- batched (multi-configuration) search -----------------------------------
// Descriptor of one search configuration inside a batch; an ordinary search
// is a batch of one. Lives in device memory; the kernels find the
// configuration of a query, pair, list or tile by binary search over the
// prefix fields.
struct CfgDev {
  const float *vec;        // the configuration's index
  const float *rows;       // its row-major copy, or NULL
  const float *xmax2;      // its largest squared row norm, or NULL
  const float *cmax2;      // its largest squared centroid norm, or NULL
  const int64_t *poff;
  const int32_t *len;
  const int64_t *rowid;
  const float *cent;
  const float *cent_slab;
  int32_t d_pad, d_cb_pad, nlist, nl_pad;
  int32_t d_c, d_s, nprobe, k;
  int64_t q0, nq;          // its query rows [q0, q0 + nq) of the batch
  int64_t S0;              // its coarse scores start at S + S0 (row stride nlist)
  int64_t pair0;           // its (query, probe) pairs [pair0, pair0 + nq * nprobe)
  int32_t vl0;             // its lists are virtual lists [vl0, vl0 + nlist)
  int32_t ct0;             // its coarse tiles [ct0, ct0 + qtiles * vtiles)
  int32_t qtiles;          // coarse query tiles
  int32_t pad_;
};

CfgDev make_cfg(const adanns_index *ix, int32_t d_c, int32_t d_s, int32_t nprobe, int32_t k,
                int64_t nq);

// Selection counters of the current device (synchronises it): [0] queries
// re-selected with a wider shortlist, [1] queries left uncertified.
// Reads (and with reset zeroes) selection counters first, first + 1.
hipError_t read_selection_stats(unsigned long long out[2], int first, bool reset);

// IVF-PQ search (adanns_search_pq) and the scratch bytes it needs for nq
// queries of one budget (0 for an invalid budget). With fixed_base the
// scratch is that caller-owned region of fixed_cap bytes: no allocation, no
// query chunks, ADANNS_EBUDGET if it does not fit.
size_t pq_search_scratch_bytes(const adanns_index *ix, int64_t nq, int32_t d_c, int32_t nprobe,
                               int32_t M, int32_t rerank_k, int32_t d_rerank);
adanns_status search_pq_impl(const adanns_index *ix, const float *Q, int64_t nq, int64_t ldq,
                             int32_t d_c, int32_t nprobe, int32_t M, int32_t k, int32_t rerank_k,
                             int32_t d_rerank, float *dist, int64_t *ids, int32_t *probes,
                             void *stream, void *fixed_base, size_t fixed_cap);

// Read-only streaming probe over bytes (a multiple of 16) of buf; out holds
// one float per workgroup of the grid.
hipError_t launch_stream_read(const void *buf, size_t bytes, float *out, int32_t grid,
                              hipStream_t st);

// ---- launch wrappers (kernels.hip) -----------------------------------------
struct SearchBufs {
  CfgDev *cfg;        // device descriptors (one for an ordinary search)
  int32_t ncfg;
  int32_t V;          // virtual lists (sum of nlist over configurations)
  int32_t ct_total;   // coarse tiles over configurations
  int64_t Qtot;       // query rows over configurations
  int64_t pairs;      // pairs over configurations
  int32_t max_nprobe, max_k, max_nlist;  // maxima over configurations (LDS sizing)
  int64_t max_items;  // upper bound on the scan's work items (caps its grid); 0 = none
  float *Qs;          // [nq][dq_pad]
  int64_t ldqs;
  float *S;           // [nq][nlist] coarse first-pass scores
  int32_t *probes;    // [nq][nprobe]
  int32_t *cnt;       // [nlist]
  int32_t *cursor;    // [nlist]
  int32_t *work;      // [8] scan work counters, one per XCD
  int32_t *bkt_off;   // [nlist]
  int32_t *tile_off;  // [nlist + 1]
  int32_t *bucket;    // [nq * nprobe]
  int64_t *seg_off;   // [nq + 1]
  int64_t *pair_base; // [nq * nprobe]
  float *D;           // first-pass distances, query-segmented
  int32_t *redo;      // [2 + Qtot] re-selection counters (coarse, scan) and list, or NULL
};

// A row-major matrix of FP32 or IEEE-half elements (the caller's database,
// or an internal FP32 buffer). Half elements convert exactly to FP32.
struct Mat {
  const void *p = nullptr;
  int64_t ld = 0;
  int32_t type = 0;  // adanns_dtype: 0 FP32, 1 FP16
  size_t esize() const { return type ? 2 : 4; }
  Mat rows(int64_t r0) const { return Mat{(const char *)p + r0 * ld * esize(), ld, type}; }
  Mat cols(int64_t c0) const { return Mat{(const char *)p + c0 * esize(), ld, type}; }
};
inline Mat f32mat(const float *p, int64_t ld) { return Mat{p, ld, 0}; }

// Lloyd's k-means on the GPU (abi.hip): nlist centroids of the first d_c
// columns of X's training rows (all n, or train_rows), from init_rows (indices
// into the training rows) or, if init_centroids (device [nlist x d_c]) is
// given, from those; iters rounds. *C_out (device, [nlist x round_up(d_c, 32)],
// caller frees) holds the centroids; with final_all_rows every row of X is
// then assigned (assign_all) and objective gets the objective per round.
adanns_status kmeans_gpu(const Mat &X, int64_t n, int32_t nlist, int32_t d_c, int32_t iters,
                         const int32_t *init_rows, const int64_t *train_rows, int64_t n_train,
                         double *objective, hipStream_t st, std::vector<int32_t> &assign_all,
                         float **C_out, bool final_all_rows, const float *init_centroids);


hipError_t launch_stage_queries(const float *Q, int64_t nq, int64_t ldq, int32_t dq,
                                float *Qs, int64_t ldqs, hipStream_t st);
hipError_t launch_layout(const Mat &src, int32_t dsrc, const int64_t *src_row,
                         const int32_t *row_list, const int64_t *poff, int64_t rows_pad,
                         int32_t d_pad, float *dst, hipStream_t st);
hipError_t launch_store_cfg(const CfgDev &c, CfgDev *dst, hipStream_t st);
// Scan tile shape from the autotune cache for this search shape (unchanged
// if the shape has not been tuned).
void tuned_shape(const adanns_index *ix, int32_t d_s, int32_t nprobe, int64_t nq, int32_t *tq,
                 int32_t *tv, int32_t *grid);
// Single-configuration helpers (the descriptor is written into b.cfg first).
hipError_t launch_coarse(const adanns_index *ix, const SearchBufs &b, int64_t nq, int32_t d_c,
                         int32_t nprobe, int32_t *user_probes, hipStream_t st,
                         float *out_min_dist = nullptr);
// Batched FP32 search over b.ncfg configurations (descriptors already in
// b.cfg). tq = query-tile height of the scan (32, 64 or 128), grid = number
// of persistent workgroups. Enqueue only: no allocation, no host sync.
hipError_t launch_search_multi(const SearchBufs &b, const float *Q, int64_t ldq, float *dist,
                               int64_t *ids, int64_t ldk, int32_t *user_probes, int32_t tq,
                               int32_t tv, int32_t grid, hipStream_t st, bool do_coarse = true);
hipError_t launch_stage_rows(const Mat &X, const int64_t *rows, const int32_t *rows32,
                             int64_t nrows, int32_t dcols, float *out, int64_t ldo,
                             hipStream_t st);
hipError_t launch_centroid_update(const float *X, int64_t ldx, const int32_t *perm,
                                  const int64_t *off, int32_t nlist, int32_t dcols, float *C,
                                  int64_t ldc, hipStream_t st);
hipError_t launch_bucketing(const adanns_index *ix, const SearchBufs &b, int64_t nq,
                            int32_t nprobe, hipStream_t st,
                            int32_t tq = TILE_Q, int32_t tv = TILE_V);
constexpr int PQ_ENCODE_MAX_DSUB = 32;
// q' = q[:d_s] R (FP64 accumulation), rows of Qs -> (hi, lo) FP32 pairs.
hipError_t launch_rotate(const float *Qs, int64_t ldqs, int64_t nq, const float *R, int32_t d_s,
                         float *qh, float *ql, int64_t ldqr, hipStream_t st);
hipError_t launch_pq_encode(const Mat &X, int64_t n, int32_t M, int32_t dsub, const float *cb,
                            uint8_t *codes, hipStream_t st);
hipError_t launch_gather_codes(const uint8_t *codes, int32_t M, const int64_t *rowid,
                               int64_t rows_pad, uint8_t *out, hipStream_t st);
// Precision form: quantised copies, quantised queries, first passes, selection.
// Row-major copy of the index's slab layout into rows [rows_pad][d_pad].
hipError_t launch_slab_to_rows(const adanns_index *ix, float *rows, hipStream_t st);
// Largest |x - dequantised x| over the rows of the index's quantised copy
// (fmt 1 bf16, 2 e4m3) into qs.emax.
hipError_t launch_quant_err_max(const adanns_index *ix, int32_t fmt, const QuantStore &qs,
                                hipStream_t st);
// The same over the quantised centroids (one-list layout, offsets poff2) into
// qs.cent_emax.
hipError_t launch_quant_err_max_cent(const adanns_index *ix, int32_t fmt, const int64_t *poff2,
                                     const QuantStore &qs, hipStream_t st);
// Largest squared row norm of a slab layout of nlists lists (offsets poff)
// into *out.
hipError_t launch_row_norm_max(const float *vec, const int64_t *poff, int32_t nlists,
                               int32_t d_pad, float *out, hipStream_t st);
hipError_t launch_quantize_store(const adanns_index *ix, int32_t fmt, QuantStore &qs,
                                 hipStream_t st);
hipError_t launch_quantize_cent_fp8(const adanns_index *ix, const int64_t *poff2, QuantStore &qs,
                                    hipStream_t st);
hipError_t launch_quantize_queries(const float *Q, int64_t nq, int64_t ldq, int32_t d,
                                   int32_t fmt, void *Qq, int64_t ldqq, float *qscale,
                                   hipStream_t st);
hipError_t launch_precision_search(const adanns_index *ix, int32_t fmt, const SearchBufs &b,
                                   const void *Qq, int64_t ldqq, const float *qscale, int64_t nq,
                                   int32_t d_c, int32_t d_s, int32_t nprobe, int32_t k,
                                   int32_t rerank_k, int32_t coarse_margin, float *dist,
                                   int64_t *ids, int32_t *user_probes, hipStream_t st);
// adanns_search's exact result from a quantised first pass (fmt 1 bf16, 2
// e4m3): FP32 coarse step, quantised list scan, FP32 re-measure of the
// candidates whose quantisation bound reaches the k-th.
hipError_t launch_filtered_search(const adanns_index *ix, int32_t fmt, const SearchBufs &b,
                                  const void *Qq, int64_t ldqq, const float *qscale, int64_t nq,
                                  int32_t d_c, int32_t d_s, int32_t nprobe, int32_t k,
                                  float *dist, int64_t *ids, int32_t *user_probes,
                                  hipStream_t st);
// IVF-PQ: rotation (compensated), tables, ADC scan and selection.
hipError_t launch_pq_search(const adanns_index *ix, const PqCodec &pq, const SearchBufs &b,
                            int64_t nq, int32_t nprobe, int32_t k, int32_t rerank_k,
                            int32_t d_rerank, float *qr_hi, float *qr_lo, float *lut, float *dist,
                            int64_t *ids, hipStream_t st);

}  // namespace adanns
