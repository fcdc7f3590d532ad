// C ABI of the library: argument validation, index import and layout,
// per-stream scratch memory and the search driver. See include/adanns.h.
#include <algorithm>
#include <atomic>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <functional>
#include <numeric>

#include "internal.h"

namespace adanns {

static thread_local char g_err[512] = "";

void set_error(const char *fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
}

void clear_error() { g_err[0] = 0; }

adanns_status get_scratch(adanns_index *ix, hipStream_t stream, size_t bytes, void **out) {
  std::lock_guard<std::mutex> lk(ix->mu);
  Scratch &s = ix->scratch[stream];
  if (s.bytes < bytes) {
    if (s.base) {
      ADANNS_HIP(hipStreamSynchronize(stream));
      ADANNS_HIP(hipFree(s.base));
      s.base = nullptr;
      s.bytes = 0;
    }
    size_t want = (size_t)round_up((int64_t)bytes, 1 << 20);
    if (hipMalloc(&s.base, want) != hipSuccess) {
      (void)hipGetLastError();
      s.base = nullptr;
      set_error("out of device memory for %zu bytes of search scratch", want);
      return ADANNS_ENOMEM;
    }
    s.bytes = want;
  }
  *out = s.base;
  return ADANNS_OK;
}

// ---- kernel timing -------------------------------------------------------------
static std::atomic<bool> g_timing{false};
static std::mutex g_tmu;
struct PendingTimer {
  std::string name;
  hipEvent_t a, b;
};
static std::vector<PendingTimer> g_pending;
static std::map<std::string, std::pair<int64_t, double>> g_totals;

static thread_local bool t_timers_off = false;

bool timing_on() { return !t_timers_off && g_timing.load(std::memory_order_relaxed); }

// Suspends kernel timing on this thread for its scope.
struct TimersOff {
  bool prev;
  TimersOff() : prev(t_timers_off) { t_timers_off = true; }
  ~TimersOff() { t_timers_off = prev; }
};

KernelTimer::KernelTimer(const char *n, hipStream_t s) : name(n), st(s) {
  if (!timing_on()) return;
  if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) {
    (void)hipGetLastError();
    if (a) (void)hipEventDestroy(a);
    a = b = nullptr;
    return;
  }
  (void)hipEventRecord(a, st);
}

void KernelTimer::stop() {
  if (!a) return;
  (void)hipEventRecord(b, st);
  std::lock_guard<std::mutex> lk(g_tmu);
  g_pending.push_back({name, a, b});
  a = b = nullptr;
}

static adanns_status resolve_timers() {
  std::lock_guard<std::mutex> lk(g_tmu);
  for (auto &p : g_pending) {
    float ms = 0.f;
    ADANNS_HIP(hipEventSynchronize(p.b));
    ADANNS_HIP(hipEventElapsedTime(&ms, p.a, p.b));
    auto &t = g_totals[p.name];
    t.first += 1;
    t.second += ms;
    (void)hipEventDestroy(p.a);
    (void)hipEventDestroy(p.b);
  }
  g_pending.clear();
  return ADANNS_OK;
}

namespace {

struct DevFree {
  std::vector<void *> ptrs;
  ~DevFree() {
    for (void *p : ptrs)
      if (p) (void)hipFree(p);
  }
};

adanns_status dmalloc(adanns_index *ix, void **p, size_t bytes) {
  if (hipMalloc(p, bytes ? bytes : 16) != hipSuccess) {
    (void)hipGetLastError();
    *p = nullptr;
    set_error("out of device memory (%zu bytes)", bytes);
    return ADANNS_ENOMEM;
  }
  ix->own_bytes += bytes;
  return ADANNS_OK;
}

void free_index_memory(adanns_index *ix) {
  void *ptrs[] = {ix->vec,  ix->rows, ix->poff,      ix->len,      ix->rowid,
                  ix->cent, ix->cent_slab, ix->xmax2, ix->cmax2};
  for (void *p : ptrs)
    if (p) (void)hipFree(p);
  for (auto &qsv : ix->quant) {
    void *pp[] = {qsv.vec, qsv.scale, qsv.cent, qsv.cent_scale, qsv.emax, qsv.cent_emax,
                  qsv.rerr};
    for (void *p : pp)
      if (p) (void)hipFree(p);
    qsv = QuantStore{};
  }
  for (auto &kv : ix->pq) {
    void *pp[] = {kv.second.R, kv.second.cb, kv.second.codes};
    for (void *p : pp)
      if (p) (void)hipFree(p);
  }
  ix->pq.clear();
  for (auto &kv : ix->scratch)
    if (kv.second.base) (void)hipFree(kv.second.base);
  ix->scratch.clear();
}

// The largest squared row norm of the filled vector layout, which bounds the
// rounding error of the FP32 first pass (allocated on first use).
adanns_status vector_norm_bound(adanns_index *ix, hipStream_t st) {
  adanns_status s;
  if (!ix->xmax2 && (s = dmalloc(ix, (void **)&ix->xmax2, sizeof(float)))) return s;
  ADANNS_HIP(launch_row_norm_max(ix->vec, ix->poff, ix->nlist, ix->d_pad, ix->xmax2, st));
  return ADANNS_OK;
}

// Lays out lists, ids and vectors for a validated assignment (host array).
// With X == NULL the vector layout is allocated but not filled.
adanns_status build_layout(adanns_index *ix, const Mat &X, const std::vector<int32_t> &assign,
                           hipStream_t st) {
  const int64_t n = ix->n;
  const int32_t nlist = ix->nlist;
  std::vector<int64_t> cnt(nlist, 0);
  for (int64_t j = 0; j < n; ++j) cnt[assign[j]]++;
  ix->h_off.assign(nlist + 1, 0);
  ix->h_poff.assign(nlist + 1, 0);
  ix->h_len.assign(nlist, 0);
  ix->max_len = 0;
  for (int32_t h = 0; h < nlist; ++h) {
    ix->h_off[h + 1] = ix->h_off[h] + cnt[h];
    ix->h_poff[h + 1] = ix->h_poff[h] + round_up(std::max<int64_t>(cnt[h], 1), ROWPAD);
    ix->h_len[h] = (int32_t)cnt[h];
    ix->max_len = std::max<int32_t>(ix->max_len, (int32_t)cnt[h]);
  }
  ix->rows_pad = ix->h_poff[nlist];
  // members in ascending row order within each list
  ix->h_ids.assign(n, 0);
  std::vector<int64_t> cur(ix->h_off.begin(), ix->h_off.end() - 1);
  for (int64_t j = 0; j < n; ++j) ix->h_ids[cur[assign[j]]++] = j;
  std::vector<int64_t> src_row(ix->rows_pad, -1);
  std::vector<int32_t> row_list(ix->rows_pad, 0);
  for (int32_t h = 0; h < nlist; ++h) {
    for (int64_t g = ix->h_poff[h]; g < ix->h_poff[h + 1]; ++g) row_list[g] = h;
    for (int64_t r = 0; r < cnt[h]; ++r) src_row[ix->h_poff[h] + r] = ix->h_ids[ix->h_off[h] + r];
  }
  // workspace bound: the sum of the p largest list lengths
  std::vector<int64_t> sorted(cnt.begin(), cnt.end());
  std::sort(sorted.begin(), sorted.end(), std::greater<int64_t>());
  ix->top_prefix.assign(nlist + 1, 0);
  for (int32_t p = 0; p < nlist; ++p) ix->top_prefix[p + 1] = ix->top_prefix[p] + sorted[p];

  adanns_status s;
  if ((s = dmalloc(ix, (void **)&ix->vec, (size_t)ix->rows_pad * ix->d_pad * sizeof(float))))
    return s;
  if ((s = dmalloc(ix, (void **)&ix->poff, (nlist + 1) * sizeof(int64_t)))) return s;
  if ((s = dmalloc(ix, (void **)&ix->len, nlist * sizeof(int32_t)))) return s;
  if ((s = dmalloc(ix, (void **)&ix->rowid, ix->rows_pad * sizeof(int64_t)))) return s;
  DevFree tmp;
  int32_t *d_row_list = nullptr;
  ADANNS_HIP(hipMalloc(&d_row_list, ix->rows_pad * sizeof(int32_t)));
  tmp.ptrs.push_back(d_row_list);
  ADANNS_HIP(hipMemcpyAsync(ix->poff, ix->h_poff.data(), (nlist + 1) * sizeof(int64_t),
                            hipMemcpyHostToDevice, st));
  ADANNS_HIP(hipMemcpyAsync(ix->len, ix->h_len.data(), nlist * sizeof(int32_t),
                            hipMemcpyHostToDevice, st));
  ADANNS_HIP(hipMemcpyAsync(ix->rowid, src_row.data(), ix->rows_pad * sizeof(int64_t),
                            hipMemcpyHostToDevice, st));
  ADANNS_HIP(hipMemcpyAsync(d_row_list, row_list.data(), ix->rows_pad * sizeof(int32_t),
                            hipMemcpyHostToDevice, st));
  if (X.p) {
    ADANNS_HIP(launch_layout(X, ix->d, ix->rowid, d_row_list, ix->poff, ix->rows_pad, ix->d_pad,
                             ix->vec, st));
    if ((s = vector_norm_bound(ix, st))) return s;
  }
  ADANNS_HIP(hipStreamSynchronize(st));
  return ADANNS_OK;
}

// Centroids: a zero-padded row-major copy and a one-list slab layout.
adanns_status build_centroids(adanns_index *ix, const float *centroids, int64_t ldc,
                              hipStream_t st) {
  const int32_t nlist = ix->nlist;
  adanns_status s;
  if ((s = dmalloc(ix, (void **)&ix->cent, (size_t)nlist * ix->d_cb_pad * sizeof(float)))) return s;
  if ((s = dmalloc(ix, (void **)&ix->cent_slab, (size_t)ix->nl_pad * ix->d_cb_pad * sizeof(float))))
    return s;
  ADANNS_HIP(hipMemsetAsync(ix->cent, 0, (size_t)nlist * ix->d_cb_pad * sizeof(float), st));
  ADANNS_HIP(hipMemcpy2DAsync(ix->cent, ix->d_cb_pad * sizeof(float), centroids,
                              ldc * sizeof(float), ix->d_cb * sizeof(float), nlist,
                              hipMemcpyDeviceToDevice, st));
  std::vector<int64_t> src_row(ix->nl_pad, -1), poff = {0, ix->nl_pad};
  for (int32_t r = 0; r < nlist; ++r) src_row[r] = r;
  std::vector<int32_t> row_list(ix->nl_pad, 0);
  DevFree tmp;
  int64_t *d_src = nullptr, *d_poff = nullptr;
  int32_t *d_rl = nullptr;
  ADANNS_HIP(hipMalloc(&d_src, ix->nl_pad * sizeof(int64_t)));
  tmp.ptrs.push_back(d_src);
  ADANNS_HIP(hipMalloc(&d_poff, 2 * sizeof(int64_t)));
  tmp.ptrs.push_back(d_poff);
  ADANNS_HIP(hipMalloc(&d_rl, ix->nl_pad * sizeof(int32_t)));
  tmp.ptrs.push_back(d_rl);
  ADANNS_HIP(hipMemcpyAsync(d_src, src_row.data(), ix->nl_pad * sizeof(int64_t),
                            hipMemcpyHostToDevice, st));
  ADANNS_HIP(hipMemcpyAsync(d_poff, poff.data(), 2 * sizeof(int64_t), hipMemcpyHostToDevice, st));
  ADANNS_HIP(hipMemcpyAsync(d_rl, row_list.data(), ix->nl_pad * sizeof(int32_t),
                            hipMemcpyHostToDevice, st));
  ADANNS_HIP(launch_layout(f32mat(ix->cent, ix->d_cb_pad), ix->d_cb, d_src, d_rl, d_poff, ix->nl_pad,
                           ix->d_cb_pad, ix->cent_slab, st));
  // the largest centroid norm bounds the coarse first pass's rounding error
  if ((s = dmalloc(ix, (void **)&ix->cmax2, sizeof(float)))) return s;
  ADANNS_HIP(launch_row_norm_max(ix->cent_slab, d_poff, 1, ix->d_cb_pad, ix->cmax2, st));
  ADANNS_HIP(hipStreamSynchronize(st));
  return ADANNS_OK;
}

// Scratch sizes of one search call, carved in a fixed order.
SearchBufs carve(char *base, const adanns_index *ix, int64_t nq, int32_t dq_pad, int32_t nprobe,
                 bool coarse, size_t *total) {
  Carver c{base, 0, 0};
  SearchBufs b{};
  b.cfg = c.take<CfgDev>(1);
  b.ncfg = 1;
  b.V = ix->nlist;
  b.Qtot = nq;
  b.pairs = nq * nprobe;
  b.ct_total = (int32_t)(cdiv(nq, TILE_Q) * cdiv(ix->nlist, TILE_V));
  b.max_nprobe = nprobe;
  b.max_k = MAX_SHORTLIST - REFINE_MARGIN;
  b.max_nlist = ix->nlist;
  // items <= sum over lists of (its pairs) x (its 64-vector tiles)
  b.max_items = nq * nprobe * cdiv(std::max<int64_t>(ix->max_len, 1), 64);
  b.ldqs = dq_pad;
  b.Qs = c.take<float>((size_t)nq * dq_pad);
  b.S = coarse ? c.take<float>((size_t)nq * ix->nlist) : nullptr;
  b.probes = c.take<int32_t>((size_t)nq * nprobe);
  b.cnt = c.take<int32_t>(ix->nlist);
  b.cursor = c.take<int32_t>(ix->nlist);
  b.work = c.take<int32_t>(8);
  b.bkt_off = c.take<int32_t>(ix->nlist);
  b.tile_off = c.take<int32_t>(ix->nlist + 1);
  b.bucket = c.take<int32_t>((size_t)nq * nprobe);
  b.seg_off = c.take<int64_t>(nq + 1);
  b.pair_base = c.take<int64_t>((size_t)nq * nprobe);
  b.D = c.take<float>((size_t)nq * ix->top_prefix[nprobe]);
  b.redo = c.take<int32_t>((size_t)nq + 2);
  *total = c.off + 256;
  return b;
}

adanns_status check_async() {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    set_error("HIP error from an earlier launch: %s", hipGetErrorString(e));
    return ADANNS_EHIP;
  }
  return ADANNS_OK;
}

}  // namespace
}  // namespace adanns

using namespace adanns;

static adanns_status init_index_shape(adanns_index *ix, int64_t n, int32_t d, int32_t nlist,
                                      int32_t d_cb) {
  (void)hipGetDevice(&ix->device);
  ix->n = n;
  ix->d = d;
  ix->d_pad = (int32_t)round_up(d, SLAB);
  ix->nlist = nlist;
  ix->d_cb = d_cb;
  ix->d_cb_pad = (int32_t)round_up(d_cb, SLAB);
  ix->nl_pad = (int32_t)round_up(nlist, ROWPAD);
  return ADANNS_OK;
}

// Lloyd's k-means on the GPU. Assignment = the coarse step with one probe
// (first-pass MFMA scores, exact re-measurement of the best few, ties to the
// smaller index); update = per-centroid mean in a fixed summation order.
namespace adanns {
adanns_status kmeans_gpu(const Mat &X, int64_t n, int32_t nlist, int32_t d_c, int32_t iters,
                         const int32_t *init_rows, const int64_t *train_rows, int64_t n_train,
                         double *objective, hipStream_t st, std::vector<int32_t> &assign_all,
                         float **C_out, bool final_all_rows, const float *init_centroids) {
  const int32_t dcp = (int32_t)round_up(d_c, SLAB);
  const int64_t nt = train_rows ? n_train : n;
  DevFree tmp;
  // centroid-only index used by the coarse kernels
  adanns_index cix;
  init_index_shape(&cix, nlist, d_c, nlist, d_c);
  float *C = nullptr, *Xt = nullptr, *S = nullptr, *mind = nullptr;
  int32_t *asg = nullptr, *perm = nullptr, *d_init = nullptr;
  int64_t *d_rows = nullptr, *d_off = nullptr;
  const int64_t chunk = std::max<int64_t>(4096, std::min<int64_t>(262144, (int64_t(1) << 28) / nlist));
  ADANNS_HIP(hipMalloc(&C, (size_t)nlist * dcp * sizeof(float)));
  ADANNS_HIP(hipMalloc(&cix.cent_slab, (size_t)cix.nl_pad * dcp * sizeof(float)));
  tmp.ptrs.push_back(cix.cent_slab);
  ADANNS_HIP(hipMalloc(&Xt, (size_t)nt * dcp * sizeof(float)));
  tmp.ptrs.push_back(Xt);
  ADANNS_HIP(hipMalloc(&S, (size_t)chunk * nlist * sizeof(float)));
  tmp.ptrs.push_back(S);
  ADANNS_HIP(hipMalloc(&mind, (size_t)std::max(nt, std::min(n, chunk)) * sizeof(float)));
  tmp.ptrs.push_back(mind);
  ADANNS_HIP(hipMalloc(&asg, (size_t)std::max(nt, n) * sizeof(int32_t)));
  tmp.ptrs.push_back(asg);
  ADANNS_HIP(hipMalloc(&perm, (size_t)nt * sizeof(int32_t)));
  tmp.ptrs.push_back(perm);
  ADANNS_HIP(hipMalloc(&d_init, (size_t)nlist * sizeof(int32_t)));
  tmp.ptrs.push_back(d_init);
  ADANNS_HIP(hipMalloc(&d_off, (size_t)(nlist + 1) * sizeof(int64_t)));
  tmp.ptrs.push_back(d_off);
  CfgDev *d_cfg = nullptr;  // descriptor of the assignment searches
  ADANNS_HIP(hipMalloc(&d_cfg, sizeof(CfgDev)));
  tmp.ptrs.push_back(d_cfg);
  float *Xc = nullptr;  // staged chunk for the final assignment of all rows
  ADANNS_HIP(hipMalloc(&Xc, (size_t)std::min(n, chunk) * dcp * sizeof(float)));
  tmp.ptrs.push_back(Xc);
  // re-selection list of the assignment searches, and the largest squared
  // centroid norm that bounds their first pass's rounding error
  int32_t *redo = nullptr;
  ADANNS_HIP(hipMalloc(&redo, (size_t)(chunk + 2) * sizeof(int32_t)));
  tmp.ptrs.push_back(redo);
  ADANNS_HIP(hipMalloc(&cix.cmax2, sizeof(float)));
  tmp.ptrs.push_back(cix.cmax2);
  if (train_rows) {
    ADANNS_HIP(hipMalloc(&d_rows, (size_t)nt * sizeof(int64_t)));
    tmp.ptrs.push_back(d_rows);
    ADANNS_HIP(hipMemcpyAsync(d_rows, train_rows, nt * sizeof(int64_t), hipMemcpyHostToDevice, st));
  }
  ADANNS_HIP(launch_stage_rows(X, d_rows, nullptr, nt, d_c, Xt, dcp, st));
  if (init_centroids) {  // given starting centroids (warm start), row stride d_c
    ADANNS_HIP(hipMemsetAsync(C, 0, (size_t)nlist * dcp * sizeof(float), st));
    ADANNS_HIP(hipMemcpy2DAsync(C, dcp * sizeof(float), init_centroids, d_c * sizeof(float),
                                d_c * sizeof(float), nlist, hipMemcpyDeviceToDevice, st));
  } else {
    ADANNS_HIP(hipMemcpyAsync(d_init, init_rows, nlist * sizeof(int32_t), hipMemcpyHostToDevice,
                              st));
    ADANNS_HIP(launch_stage_rows(f32mat(Xt, dcp), nullptr, d_init, nlist, d_c, C, dcp, st));
  }
  cix.cent = C;

  std::vector<int32_t> h_asg(nt);
  std::vector<float> h_mind(std::max(nt, n));
  std::vector<int32_t> h_perm(nt);
  std::vector<int64_t> h_off(nlist + 1);
  std::vector<int64_t> src_row(cix.nl_pad, -1), poff = {0, cix.nl_pad};
  for (int32_t r = 0; r < nlist; ++r) src_row[r] = r;
  std::vector<int32_t> row_list(cix.nl_pad, 0);
  int64_t *d_src = nullptr, *d_poff1 = nullptr;
  int32_t *d_rl = nullptr;
  ADANNS_HIP(hipMalloc(&d_src, cix.nl_pad * sizeof(int64_t)));
  tmp.ptrs.push_back(d_src);
  ADANNS_HIP(hipMalloc(&d_poff1, 2 * sizeof(int64_t)));
  tmp.ptrs.push_back(d_poff1);
  ADANNS_HIP(hipMalloc(&d_rl, cix.nl_pad * sizeof(int32_t)));
  tmp.ptrs.push_back(d_rl);
  ADANNS_HIP(hipMemcpyAsync(d_src, src_row.data(), cix.nl_pad * sizeof(int64_t), hipMemcpyHostToDevice, st));
  ADANNS_HIP(hipMemcpyAsync(d_poff1, poff.data(), 2 * sizeof(int64_t), hipMemcpyHostToDevice, st));
  ADANNS_HIP(hipMemcpyAsync(d_rl, row_list.data(), cix.nl_pad * sizeof(int32_t), hipMemcpyHostToDevice, st));

  auto assign_rows = [&](const float *rows, int64_t ldr, int64_t count, int32_t *out_asg,
                         float *out_min) -> adanns_status {
    ADANNS_HIP(launch_layout(f32mat(C, dcp), d_c, d_src, d_rl, d_poff1, cix.nl_pad, dcp,
                             cix.cent_slab, st));
    ADANNS_HIP(launch_row_norm_max(cix.cent_slab, d_poff1, 1, dcp, cix.cmax2, st));
    for (int64_t a0 = 0; a0 < count; a0 += chunk) {
      const int64_t m = std::min(chunk, count - a0);
      SearchBufs b{};
      b.cfg = d_cfg;
      b.redo = redo;
      b.Qs = const_cast<float *>(rows) + a0 * ldr;
      b.ldqs = ldr;
      b.S = S;
      b.probes = out_asg + a0;
      ADANNS_HIP(launch_coarse(&cix, b, m, d_c, 1, nullptr, st, out_min + a0));
    }
    return ADANNS_OK;
  };
  adanns_status s;
  for (int32_t it = 0; it < iters; ++it) {
    if ((s = assign_rows(Xt, dcp, nt, asg, mind))) return s;
    ADANNS_HIP(hipMemcpyAsync(h_asg.data(), asg, nt * sizeof(int32_t), hipMemcpyDeviceToHost, st));
    ADANNS_HIP(hipMemcpyAsync(h_mind.data(), mind, nt * sizeof(float), hipMemcpyDeviceToHost, st));
    ADANNS_HIP(hipStreamSynchronize(st));
    if (objective) {
      double J = 0.0;
      for (int64_t j = 0; j < nt; ++j) J += h_mind[j];
      objective[it] = J;
    }
    // the host indexes its arrays by these: a cluster outside [0, nlist)
    // (non-finite rows or centroids leave the coarse step without an order)
    // is an error, not an index
    for (int64_t j = 0; j < nt; ++j)
      ADANNS_REQUIRE(h_asg[j] >= 0 && h_asg[j] < nlist,
                     "k-means: row %lld assigned to cluster %d outside [0, %d) (non-finite data?)",
                     (long long)j, h_asg[j], nlist);
    // stable counting sort of the training rows by cluster
    std::fill(h_off.begin(), h_off.end(), 0);
    for (int64_t j = 0; j < nt; ++j) h_off[h_asg[j] + 1]++;
    for (int32_t h = 0; h < nlist; ++h) h_off[h + 1] += h_off[h];
    std::vector<int64_t> cur(h_off.begin(), h_off.end() - 1);
    for (int64_t j = 0; j < nt; ++j) h_perm[cur[h_asg[j]]++] = (int32_t)j;
    ADANNS_HIP(hipMemcpyAsync(perm, h_perm.data(), nt * sizeof(int32_t), hipMemcpyHostToDevice, st));
    ADANNS_HIP(hipMemcpyAsync(d_off, h_off.data(), (nlist + 1) * sizeof(int64_t), hipMemcpyHostToDevice, st));
    ADANNS_HIP(launch_centroid_update(Xt, dcp, perm, d_off, nlist, d_c, C, dcp, st));
  }
  if (!final_all_rows) {  // centroids only (the caller encodes the rows itself)
    cix.cent = nullptr;
    cix.cent_slab = nullptr;
    cix.cmax2 = nullptr;
    *C_out = C;
    return ADANNS_OK;
  }
  // final assignment of every row against the final centroids
  assign_all.assign(n, 0);
  ADANNS_HIP(launch_layout(f32mat(C, dcp), d_c, d_src, d_rl, d_poff1, cix.nl_pad, dcp,
                           cix.cent_slab, st));
  ADANNS_HIP(launch_row_norm_max(cix.cent_slab, d_poff1, 1, dcp, cix.cmax2, st));
  for (int64_t a0 = 0; a0 < n; a0 += chunk) {
    const int64_t m = std::min(chunk, n - a0);
    ADANNS_HIP(launch_stage_rows(X.rows(a0), nullptr, nullptr, m, d_c, Xc, dcp, st));
    SearchBufs b{};
    b.cfg = d_cfg;
    b.redo = redo;
    b.Qs = Xc;
    b.ldqs = dcp;
    b.S = S;
    b.probes = asg + a0;
    ADANNS_HIP(launch_coarse(&cix, b, m, d_c, 1, nullptr, st, mind));
    ADANNS_HIP(hipMemcpyAsync(h_mind.data() + a0, mind, m * sizeof(float), hipMemcpyDeviceToHost, st));
  }
  ADANNS_HIP(hipMemcpyAsync(assign_all.data(), asg, n * sizeof(int32_t), hipMemcpyDeviceToHost, st));
  ADANNS_HIP(hipStreamSynchronize(st));
  for (int64_t j = 0; j < n; ++j)
    ADANNS_REQUIRE(assign_all[j] >= 0 && assign_all[j] < nlist,
                   "k-means: row %lld assigned to cluster %d outside [0, %d) (non-finite data?)",
                   (long long)j, assign_all[j], nlist);
  if (objective) {
    double J = 0.0;
    if (train_rows)
      for (int64_t j = 0; j < nt; ++j) J += h_mind[train_rows[j]];
    else
      for (int64_t j = 0; j < n; ++j) J += h_mind[j];
    objective[iters] = J;
  }
  cix.cent = nullptr;
  cix.cent_slab = nullptr;  // freed by tmp
  cix.cmax2 = nullptr;
  *C_out = C;
  return ADANNS_OK;
}
}  // namespace adanns

extern "C" {

const char *adanns_last_error(void) { return g_err; }

const char *adanns_version(void) { return "adanns-mi355x 0.1 (gfx950)"; }

adanns_status adanns_ivf_import(const void *X, int64_t n, int32_t d, int64_t ldx, int32_t dtype,
                                const float *centroids, int32_t nlist, int32_t d_c_build,
                                const int32_t *assign, void *stream, adanns_index **out) {
  clear_error();
  ADANNS_REQUIRE(out != nullptr, "out is NULL");
  ADANNS_REQUIRE(X && centroids && assign, "X, centroids and assign must be non-NULL");
  ADANNS_REQUIRE(n >= 1 && n < (int64_t(1) << 31), "n must be in [1, 2^31), got %lld",
                 (long long)n);
  ADANNS_REQUIRE(d >= 1 && d <= 8192, "d must be in [1, 8192], got %d", d);
  ADANNS_REQUIRE(ldx >= d, "ldx (%lld) must be >= d (%d)", (long long)ldx, d);
  ADANNS_REQUIRE(dtype == ADANNS_DTYPE_F32 || dtype == ADANNS_DTYPE_F16,
                 "dtype must be ADANNS_DTYPE_F32 or ADANNS_DTYPE_F16, got %d", dtype);
  ADANNS_REQUIRE(nlist >= 1 && nlist <= 65536, "nlist must be in [1, 65536], got %d", nlist);
  ADANNS_REQUIRE(d_c_build >= 1 && d_c_build <= d, "d_c_build must be in [1, d], got %d",
                 d_c_build);
  adanns_status s = check_async();
  if (s) return s;
  hipStream_t st = (hipStream_t)stream;
  std::vector<int32_t> h_assign(n);
  ADANNS_HIP(hipMemcpyAsync(h_assign.data(), assign, n * sizeof(int32_t), hipMemcpyDeviceToHost, st));
  ADANNS_HIP(hipStreamSynchronize(st));
  for (int64_t j = 0; j < n; ++j)
    ADANNS_REQUIRE(h_assign[j] >= 0 && h_assign[j] < nlist, "assign[%lld] = %d is outside [0, %d)",
                   (long long)j, h_assign[j], nlist);
  adanns_index *ix = new (std::nothrow) adanns_index();
  if (!ix) {
    set_error("out of host memory");
    return ADANNS_ENOMEM;
  }
  init_index_shape(ix, n, d, nlist, d_c_build);
  if ((s = build_layout(ix, Mat{X, ldx, dtype}, h_assign, st)) ||
      (s = build_centroids(ix, centroids, d_c_build, st))) {
    free_index_memory(ix);
    delete ix;
    return s;
  }
  *out = ix;
  return ADANNS_OK;
}

static std::atomic<size_t> g_scratch_cap{kSearchScratchCap};

// Scratch of adanns_search_noalloc: a file-scope device array, one copy per
// GPU, held until the process ends. Host code must not use its name as an
// address (that is a host-side stand-in): the device address comes from
// hipGetSymbolAddress, once per device, kept in g_noalloc_ptr.
constexpr size_t kNoAllocScratchBytes = size_t(64) << 20;
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];
constexpr int kMaxDevices = 64;
static std::mutex g_noalloc_mu;
static void *g_noalloc_ptr[kMaxDevices];

// Device address of ``scratch`` on the current device.
static adanns_status noalloc_scratch(void **out) {
  int dev = 0;
  ADANNS_HIP(hipGetDevice(&dev));
  ADANNS_REQUIRE(dev >= 0 && dev < kMaxDevices, "device %d is beyond the %d supported", dev,
                 kMaxDevices);
  std::lock_guard<std::mutex> lk(g_noalloc_mu);
  if (!g_noalloc_ptr[dev]) {
    void *p = nullptr;
    ADANNS_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    g_noalloc_ptr[dev] = p;
  }
  *out = g_noalloc_ptr[dev];
  return ADANNS_OK;
}

// fixed_base != NULL: the search runs in that caller-fixed scratch of
// fixed_cap bytes (no allocation, no chunking; a larger need is EBUDGET).
static adanns_status search_common(const adanns_index *cix, const float *Q, int64_t nq,
                                   int64_t ldq, int32_t d_c, int32_t d_s, int32_t nprobe,
                                   const int32_t *given_probes, int32_t k, float *dist,
                                   int64_t *ids, int32_t *probes_out, void *stream,
                                   void *fixed_base = nullptr, size_t fixed_cap = 0) {
  adanns_index *ix = const_cast<adanns_index *>(cix);
  const bool coarse = given_probes == nullptr;
  ADANNS_REQUIRE(ix != nullptr, "index is NULL");
  ADANNS_REQUIRE(nq >= 0, "nq must be >= 0");
  ADANNS_REQUIRE(d_s >= 1 && d_s <= ix->d, "d_s must be in [1, %d], got %d", ix->d, d_s);
  if (coarse)
    ADANNS_REQUIRE(d_c >= 1 && d_c <= ix->d_cb, "d_c must be in [1, %d], got %d", ix->d_cb, d_c);
  ADANNS_REQUIRE(nprobe >= 1 && nprobe <= ix->nlist, "nprobe must be in [1, %d], got %d",
                 ix->nlist, nprobe);
  ADANNS_REQUIRE(k >= 1 && k <= MAX_SHORTLIST, "k must be in [1, %d], got %d", MAX_SHORTLIST, k);
  ADANNS_REQUIRE(nq < (int64_t(1) << 31) / std::max(nprobe, 1),
                 "nq * nprobe must be below 2^31");
  ADANNS_REQUIRE(ldq >= std::max(coarse ? d_c : 0, d_s), "ldq (%lld) is smaller than the prefix",
                 (long long)ldq);
  if (nq == 0) return ADANNS_OK;
  ADANNS_REQUIRE(Q && dist && ids, "Q, dist and ids must be non-NULL");
  adanns_status s = check_async();
  if (s) return s;
  hipStream_t st = (hipStream_t)stream;
  const int32_t dq = std::max(coarse ? d_c : 0, d_s);
  const int32_t dq_pad = (int32_t)round_up(dq, SLAB);
  // The scratch grows with the batch (first-pass values of every candidate):
  // a batch whose scratch would pass the cap runs in query chunks.
  const size_t cap = g_scratch_cap.load();
  auto scratch_of = [&](int64_t m) {
    size_t t = 0;
    carve(nullptr, ix, m, dq_pad, nprobe, coarse, &t);
    return t;
  };
  int64_t chunk = nq;
  if (fixed_base) {
    const size_t need = scratch_of(nq);
    if (need > fixed_cap) {
      set_error("the search needs %zu bytes of scratch, more than the %zu of the allocation-free "
                "entry point: search fewer queries per call", need, fixed_cap);
      return ADANNS_EBUDGET;
    }
  } else {
    while (chunk > 1 && scratch_of(chunk) > cap) chunk = (chunk + 1) / 2;
  }
  for (int64_t r0 = 0; r0 < nq; r0 += chunk) {
    const int64_t m = std::min(chunk, nq - r0);
    size_t total = scratch_of(m);
    void *base = fixed_base;
    if (!fixed_base && (s = get_scratch(ix, st, total, &base))) return s;
    SearchBufs b = carve((char *)base, ix, m, dq_pad, nprobe, coarse, &total);
    b.max_k = k;
    ADANNS_HIP(launch_store_cfg(make_cfg(ix, coarse ? d_c : 1, d_s, nprobe, k, m), b.cfg, st));
    if (!coarse)
      ADANNS_HIP(hipMemcpyAsync(b.probes, given_probes + r0 * nprobe,
                                (size_t)m * nprobe * sizeof(int32_t), hipMemcpyDeviceToDevice, st));
    int32_t tq = TILE_Q, tv = TILE_V, grid = PERSIST_WG;
    tuned_shape(ix, d_s, nprobe, m, &tq, &tv, &grid);
    ADANNS_HIP(launch_search_multi(b, Q + r0 * ldq, ldq, dist + r0 * k, ids + r0 * k,
                                   k, probes_out ? probes_out + r0 * nprobe : nullptr, tq, tv,
                                   grid, st, coarse));
  }
  return ADANNS_OK;
}

adanns_status adanns_set_search_scratch_cap(size_t bytes) {
  clear_error();
  g_scratch_cap.store(bytes ? bytes : kSearchScratchCap);
  return ADANNS_OK;
}

adanns_status adanns_search(const adanns_index *index, const float *Q, int64_t nq, int64_t ldq,
                            int32_t d_c, int32_t d_s, int32_t nprobe, int32_t k, float *dist,
                            int64_t *ids, int32_t *probes, void *stream) {
  clear_error();
  return search_common(index, Q, nq, ldq, d_c, d_s, nprobe, nullptr, k, dist, ids, probes, stream);
}

adanns_status adanns_search_noalloc(const adanns_index *index, const float *Q, int64_t nq,
                                    int64_t ldq, int32_t d_c, int32_t d_s, int32_t nprobe,
                                    int32_t k, float *dist, int64_t *ids, int32_t *probes,
                                    void *stream) {
  clear_error();
  void *base = nullptr;
  adanns_status s = noalloc_scratch(&base);
  if (s) return s;
  TimersOff no_events;  // kernel timing would create events
  return search_common(index, Q, nq, ldq, d_c, d_s, nprobe, nullptr, k, dist, ids, probes, stream,
                       base, kNoAllocScratchBytes);
}

size_t adanns_search_noalloc_max_bytes(void) { return kNoAllocScratchBytes; }

adanns_status adanns_search_probes(const adanns_index *index, const float *Q, int64_t nq,
                                   int64_t ldq, int32_t d_s, int32_t nprobe,
                                   const int32_t *probes, int32_t k, float *dist, int64_t *ids,
                                   void *stream) {
  clear_error();
  if (nq > 0 && index != nullptr && nprobe >= 1 && nprobe <= index->nlist) {
    // The scan's scratch bound assumes distinct, in-range probes: check them.
    ADANNS_REQUIRE(probes != nullptr, "probes must be non-NULL");
    std::vector<int32_t> hp((size_t)nq * nprobe);
    ADANNS_HIP(hipMemcpyAsync(hp.data(), probes, hp.size() * sizeof(int32_t),
                              hipMemcpyDeviceToHost, (hipStream_t)stream));
    ADANNS_HIP(hipStreamSynchronize((hipStream_t)stream));
    std::vector<int64_t> seen(index->nlist, -1);
    for (int64_t q = 0; q < nq; ++q)
      for (int32_t j = 0; j < nprobe; ++j) {
        int32_t h = hp[q * nprobe + j];
        ADANNS_REQUIRE(h >= 0 && h < index->nlist, "probes[%lld][%d] = %d is outside [0, %d)",
                       (long long)q, j, h, index->nlist);
        ADANNS_REQUIRE(seen[h] != q, "probes[%lld] repeats list %d", (long long)q, h);
        seen[h] = q;
      }
  }
  return search_common(index, Q, nq, ldq, 0, d_s, nprobe, probes, k, dist, ids, nullptr, stream);
}

adanns_status adanns_build_ivf(const void *X, int64_t n, int32_t d, int64_t ldx, int32_t dtype,
                               int32_t nlist,
                               int32_t d_c, int32_t iters, const int32_t *init_rows,
                               const int64_t *train_rows, int64_t n_train, double *objective,
                               void *stream, adanns_index **out) {
  clear_error();
  ADANNS_REQUIRE(out != nullptr, "out is NULL");
  ADANNS_REQUIRE(X != nullptr && init_rows != nullptr, "X and init_rows must be non-NULL");
  ADANNS_REQUIRE(n >= 1 && n < (int64_t(1) << 31), "n must be in [1, 2^31), got %lld",
                 (long long)n);
  ADANNS_REQUIRE(d >= 1 && d <= 8192, "d must be in [1, 8192], got %d", d);
  ADANNS_REQUIRE(ldx >= d, "ldx (%lld) must be >= d (%d)", (long long)ldx, d);
  ADANNS_REQUIRE(dtype == ADANNS_DTYPE_F32 || dtype == ADANNS_DTYPE_F16,
                 "dtype must be ADANNS_DTYPE_F32 or ADANNS_DTYPE_F16, got %d", dtype);
  ADANNS_REQUIRE(nlist >= 1 && nlist <= 65536, "nlist must be in [1, 65536], got %d", nlist);
  ADANNS_REQUIRE(d_c >= 1 && d_c <= d, "d_c must be in [1, d], got %d", d_c);
  ADANNS_REQUIRE(iters >= 0 && iters <= 1000, "iters must be in [0, 1000], got %d", iters);
  const int64_t nt = train_rows ? n_train : n;
  ADANNS_REQUIRE(nt >= nlist, "the training set (%lld rows) must hold at least nlist rows",
                 (long long)nt);
  if (train_rows)
    for (int64_t j = 0; j < nt; ++j)
      ADANNS_REQUIRE(train_rows[j] >= 0 && train_rows[j] < n, "train_rows[%lld] out of range",
                     (long long)j);
  for (int32_t h = 0; h < nlist; ++h)
    ADANNS_REQUIRE(init_rows[h] >= 0 && init_rows[h] < nt, "init_rows[%d] = %d out of range", h,
                   init_rows[h]);
  adanns_status s = check_async();
  if (s) return s;
  hipStream_t st = (hipStream_t)stream;
  std::vector<int32_t> assign;
  float *C = nullptr;
  const Mat Xm{X, ldx, dtype};
  if ((s = kmeans_gpu(Xm, n, nlist, d_c, iters, init_rows, train_rows, nt, objective, st, assign,
                      &C, true, nullptr))) {
    if (C) (void)hipFree(C);
    return s;
  }
  adanns_index *ix = new (std::nothrow) adanns_index();
  if (!ix) {
    (void)hipFree(C);
    set_error("out of host memory");
    return ADANNS_ENOMEM;
  }
  init_index_shape(ix, n, d, nlist, d_c);
  if ((s = build_layout(ix, Xm, assign, st)) ||
      (s = build_centroids(ix, C, round_up(d_c, SLAB), st))) {
    (void)hipFree(C);
    free_index_memory(ix);
    delete ix;
    return s;
  }
  (void)hipFree(C);
  *out = ix;
  return ADANNS_OK;
}

adanns_status adanns_pq_import(adanns_index *ix, int32_t M, int32_t d_s, const float *R,
                               const float *codebooks, const uint8_t *codes, void *stream) {
  clear_error();
  ADANNS_REQUIRE(ix != nullptr, "index is NULL");
  ADANNS_REQUIRE(codebooks != nullptr && codes != nullptr, "codebooks and codes must be non-NULL");
  ADANNS_REQUIRE(d_s >= 1 && d_s <= ix->d && d_s <= 2048, "d_s must be in [1, min(d, 2048)], got %d",
                 d_s);
  ADANNS_REQUIRE(M >= 4 && M <= 64 && M % 4 == 0, "M must be a multiple of 4 in [4, 64], got %d", M);
  ADANNS_REQUIRE(d_s % M == 0, "M (%d) must divide d_s (%d)", M, d_s);
  ADANNS_REQUIRE(ix->pq.find(M) == ix->pq.end(), "the index already holds a codec with M = %d", M);
  adanns_status s = check_async();
  if (s) return s;
  hipStream_t st = (hipStream_t)stream;
  PqCodec c;
  c.M = M;
  c.d_s = d_s;
  c.dsub = d_s / M;
  auto fail = [&](adanns_status e) {
    void *pp[] = {c.R, c.cb, c.codes};
    for (void *p : pp)
      if (p) (void)hipFree(p);
    return e;
  };
  if ((s = dmalloc(ix, (void **)&c.R, (size_t)d_s * d_s * sizeof(float)))) return fail(s);
  if ((s = dmalloc(ix, (void **)&c.cb, (size_t)M * 256 * c.dsub * sizeof(float)))) return fail(s);
  if ((s = dmalloc(ix, (void **)&c.codes, (size_t)ix->rows_pad * M))) return fail(s);
  if (R) {
    if (hipMemcpyAsync(c.R, R, (size_t)d_s * d_s * sizeof(float), hipMemcpyDeviceToDevice, st))
      return fail(ADANNS_EHIP);
  } else {
    std::vector<float> eye((size_t)d_s * d_s, 0.f);
    for (int32_t i = 0; i < d_s; ++i) eye[(size_t)i * d_s + i] = 1.f;
    if (hipMemcpyAsync(c.R, eye.data(), eye.size() * sizeof(float), hipMemcpyHostToDevice, st) ||
        hipStreamSynchronize(st))
      return fail(ADANNS_EHIP);
  }
  if (hipMemcpyAsync(c.cb, codebooks, (size_t)M * 256 * c.dsub * sizeof(float),
                     hipMemcpyDeviceToDevice, st) ||
      launch_gather_codes(codes, M, ix->rowid, ix->rows_pad, c.codes, st) ||
      hipStreamSynchronize(st)) {
    set_error("HIP error while importing the PQ codec");
    return fail(ADANNS_EHIP);
  }
  ix->pq[M] = c;
  return ADANNS_OK;
}

adanns_status adanns_pq_train(adanns_index *ix, const void *X, int64_t ldx, int32_t dtype,
                              int32_t M,
                              int32_t d_s, const float *R_in, int32_t iters,
                              const int32_t *init_rows, const int64_t *train_rows,
                              int64_t n_train, void *stream) {
  clear_error();
  ADANNS_REQUIRE(ix != nullptr && X != nullptr && init_rows != nullptr,
                 "index, X and init_rows must be non-NULL");
  ADANNS_REQUIRE(ldx >= ix->d, "ldx (%lld) must be >= d (%d)", (long long)ldx, ix->d);
  ADANNS_REQUIRE(dtype == ADANNS_DTYPE_F32 || dtype == ADANNS_DTYPE_F16,
                 "dtype must be ADANNS_DTYPE_F32 or ADANNS_DTYPE_F16, got %d", dtype);
  ADANNS_REQUIRE(d_s >= 1 && d_s <= ix->d && d_s <= 2048, "d_s must be in [1, min(d, 2048)]");
  ADANNS_REQUIRE(M >= 4 && M <= 64 && M % 4 == 0, "M must be a multiple of 4 in [4, 64], got %d", M);
  ADANNS_REQUIRE(d_s % M == 0, "M (%d) must divide d_s (%d)", M, d_s);
  ADANNS_REQUIRE(d_s / M <= PQ_ENCODE_MAX_DSUB, "GPU training supports d_s / M <= %d",
                 PQ_ENCODE_MAX_DSUB);
  ADANNS_REQUIRE(iters >= 0 && iters <= 1000, "iters must be in [0, 1000]");
  ADANNS_REQUIRE(ix->pq.find(M) == ix->pq.end(), "the index already holds a codec with M = %d", M);
  const int64_t nt = train_rows ? n_train : ix->n;
  ADANNS_REQUIRE(nt >= 256, "the training set must hold at least 256 rows");
  for (int32_t c = 0; c < 256; ++c)
    ADANNS_REQUIRE(init_rows[c] >= 0 && init_rows[c] < nt, "init_rows[%d] out of range", c);
  if (train_rows)
    for (int64_t j = 0; j < nt; ++j)
      ADANNS_REQUIRE(train_rows[j] >= 0 && train_rows[j] < ix->n, "train_rows[%lld] out of range",
                     (long long)j);
  adanns_status s = check_async();
  if (s) return s;
  hipStream_t st = (hipStream_t)stream;
  const int32_t dsub = d_s / M, dcp = (int32_t)round_up(dsub, SLAB);
  DevFree tmp;
  float *cb = nullptr, *R = nullptr;
  uint8_t *codes_id = nullptr;
  ADANNS_HIP(hipMalloc(&cb, (size_t)M * 256 * dsub * sizeof(float)));
  tmp.ptrs.push_back(cb);
  ADANNS_HIP(hipMalloc(&codes_id, (size_t)ix->n * M));
  tmp.ptrs.push_back(codes_id);
  std::vector<int32_t> unused;
  // training matrix: the rows themselves, or the training rows rotated by R
  const Mat Xm{X, ldx, dtype};
  Mat Tx = Xm;
  int64_t nT = ix->n;
  const int64_t *trows = train_rows;
  float *Rdev = nullptr, *T = nullptr, *Tlo = nullptr;
  if (R_in) {
    ADANNS_HIP(hipMalloc(&Rdev, (size_t)d_s * d_s * sizeof(float)));
    tmp.ptrs.push_back(Rdev);
    ADANNS_HIP(hipMemcpyAsync(Rdev, R_in, (size_t)d_s * d_s * sizeof(float),
                              hipMemcpyDeviceToDevice, st));
    float *raw = nullptr;
    int64_t *d_tr = nullptr;
    ADANNS_HIP(hipMalloc(&raw, (size_t)nt * d_s * sizeof(float)));
    tmp.ptrs.push_back(raw);
    ADANNS_HIP(hipMalloc(&T, (size_t)nt * d_s * sizeof(float)));
    tmp.ptrs.push_back(T);
    ADANNS_HIP(hipMalloc(&Tlo, (size_t)nt * d_s * sizeof(float)));
    tmp.ptrs.push_back(Tlo);
    if (train_rows) {
      ADANNS_HIP(hipMalloc(&d_tr, (size_t)nt * sizeof(int64_t)));
      tmp.ptrs.push_back(d_tr);
      ADANNS_HIP(hipMemcpyAsync(d_tr, train_rows, nt * sizeof(int64_t), hipMemcpyHostToDevice, st));
    }
    ADANNS_HIP(launch_stage_rows(Xm, d_tr, nullptr, nt, d_s, raw, d_s, st));
    ADANNS_HIP(launch_rotate(raw, d_s, nt, Rdev, d_s, T, Tlo, d_s, st));
    Tx = f32mat(T, d_s);
    nT = nt;
    trows = nullptr;  // T holds exactly the training rows
  }
  for (int32_t m = 0; m < M; ++m) {
    float *C = nullptr;
    // Lloyd's k-means with 256 codewords on the m-th block of coordinates
    if ((s = kmeans_gpu(Tx.cols((int64_t)m * dsub), nT, 256, dsub, iters, init_rows, trows, nt,
                        nullptr, st, unused, &C, false, nullptr))) {
      if (C) (void)hipFree(C);
      return s;
    }
    hipError_t e = hipMemcpy2DAsync(cb + (size_t)m * 256 * dsub, dsub * sizeof(float), C,
                                    dcp * sizeof(float), dsub * sizeof(float), 256,
                                    hipMemcpyDeviceToDevice, st);
    (void)hipStreamSynchronize(st);
    (void)hipFree(C);
    ADANNS_HIP(e);
  }
  if (!R_in) {
    ADANNS_HIP(launch_pq_encode(Xm, ix->n, M, dsub, cb, codes_id, st));
    std::vector<float> eye((size_t)d_s * d_s, 0.f);
    for (int32_t i = 0; i < d_s; ++i) eye[(size_t)i * d_s + i] = 1.f;
    ADANNS_HIP(hipMalloc(&R, eye.size() * sizeof(float)));
    tmp.ptrs.push_back(R);
    ADANNS_HIP(hipMemcpyAsync(R, eye.data(), eye.size() * sizeof(float), hipMemcpyHostToDevice, st));
    ADANNS_HIP(hipStreamSynchronize(st));
    return adanns_pq_import(ix, M, d_s, R, cb, codes_id, stream);
  }
  // encode every row after rotating it, in chunks
  const int64_t chunk = 262144;
  float *craw = nullptr, *crot = nullptr, *clo = nullptr;
  const int64_t cm = std::min<int64_t>(chunk, ix->n);
  ADANNS_HIP(hipMalloc(&craw, (size_t)cm * d_s * sizeof(float)));
  tmp.ptrs.push_back(craw);
  ADANNS_HIP(hipMalloc(&crot, (size_t)cm * d_s * sizeof(float)));
  tmp.ptrs.push_back(crot);
  ADANNS_HIP(hipMalloc(&clo, (size_t)cm * d_s * sizeof(float)));
  tmp.ptrs.push_back(clo);
  for (int64_t a0 = 0; a0 < ix->n; a0 += chunk) {
    const int64_t m = std::min(chunk, ix->n - a0);
    ADANNS_HIP(launch_stage_rows(Xm.rows(a0), nullptr, nullptr, m, d_s, craw, d_s, st));
    ADANNS_HIP(launch_rotate(craw, d_s, m, Rdev, d_s, crot, clo, d_s, st));
    ADANNS_HIP(launch_pq_encode(f32mat(crot, d_s), m, M, dsub, cb, codes_id + a0 * M, st));
  }
  ADANNS_HIP(hipStreamSynchronize(st));
  return adanns_pq_import(ix, M, d_s, Rdev, cb, codes_id, stream);
}

adanns_status adanns_pq_codec(const adanns_index *ix, int32_t M, float *R, float *codebooks,
                              uint8_t *codes) {
  clear_error();
  ADANNS_REQUIRE(ix != nullptr, "index is NULL");
  auto it = ix->pq.find(M);
  ADANNS_REQUIRE(it != ix->pq.end(), "the index holds no PQ codec with M = %d", M);
  const PqCodec &c = it->second;
  if (R) ADANNS_HIP(hipMemcpy(R, c.R, (size_t)c.d_s * c.d_s * sizeof(float), hipMemcpyDeviceToHost));
  if (codebooks)
    ADANNS_HIP(hipMemcpy(codebooks, c.cb, (size_t)M * 256 * c.dsub * sizeof(float),
                         hipMemcpyDeviceToHost));
  if (codes) {
    std::vector<uint8_t> lay((size_t)ix->rows_pad * M);
    ADANNS_HIP(hipMemcpy(lay.data(), c.codes, lay.size(), hipMemcpyDeviceToHost));
    for (int32_t h = 0; h < ix->nlist; ++h)
      for (int64_t r = 0; r < ix->h_len[h]; ++r)
        std::memcpy(codes + (size_t)ix->h_ids[ix->h_off[h] + r] * M,
                    &lay[(size_t)(ix->h_poff[h] + r) * M], M);
  }
  return ADANNS_OK;
}

}  // extern "C"

namespace adanns {
// Scratch bytes of one IVF-PQ search of nq queries (0 if the budget is invalid).
size_t pq_search_scratch_bytes(const adanns_index *ix, int64_t nq, int32_t d_c, int32_t nprobe,
                               int32_t M, int32_t rerank_k, int32_t d_rerank) {
  auto it = ix->pq.find(M);
  if (it == ix->pq.end() || nprobe < 1 || nprobe > ix->nlist) return 0;
  const PqCodec &pq = it->second;
  const int32_t dq = std::max(std::max(d_c, pq.d_s), rerank_k > 0 ? d_rerank : 0);
  const int32_t dq_pad = (int32_t)round_up(dq, SLAB);
  size_t t = 0;
  carve(nullptr, ix, nq, dq_pad, nprobe, true, &t);
  return t + (size_t)round_up((size_t)nq * pq.d_s * 4, 256) * 2 +
         (size_t)round_up((size_t)nq * M * 256 * 4, 256) + 1024;
}

// adanns_search_pq; with fixed_base the scratch is that caller-owned region
// of fixed_cap bytes (no allocation, no chunking; a larger need is EBUDGET).
adanns_status search_pq_impl(const adanns_index *cix, const float *Q, int64_t nq, int64_t ldq,
                             int32_t d_c, int32_t nprobe, int32_t M, int32_t k, int32_t rerank_k,
                             int32_t d_rerank, float *dist, int64_t *ids, int32_t *probes,
                             void *stream, void *fixed_base, size_t fixed_cap) {
  adanns_index *ix = const_cast<adanns_index *>(cix);
  ADANNS_REQUIRE(ix != nullptr, "index is NULL");
  auto it = ix->pq.find(M);
  ADANNS_REQUIRE(it != ix->pq.end(), "the index holds no PQ codec with M = %d", M);
  const PqCodec &pq = it->second;
  ADANNS_REQUIRE(nq >= 0, "nq must be >= 0");
  ADANNS_REQUIRE(d_c >= 1 && d_c <= ix->d_cb, "d_c must be in [1, %d], got %d", ix->d_cb, d_c);
  ADANNS_REQUIRE(nprobe >= 1 && nprobe <= ix->nlist, "nprobe must be in [1, %d], got %d",
                 ix->nlist, nprobe);
  ADANNS_REQUIRE(k >= 1 && k <= MAX_SHORTLIST - REFINE_MARGIN, "k must be in [1, %d], got %d",
                 MAX_SHORTLIST - REFINE_MARGIN, k);
  ADANNS_REQUIRE(rerank_k == 0 || (rerank_k >= k && rerank_k <= MAX_SHORTLIST - REFINE_MARGIN),
                 "rerank_k must be 0 or in [k, %d], got %d", MAX_SHORTLIST - REFINE_MARGIN,
                 rerank_k);
  if (rerank_k > 0)
    ADANNS_REQUIRE(d_rerank >= 1 && d_rerank <= ix->d, "d_rerank must be in [1, %d], got %d",
                   ix->d, d_rerank);
  ADANNS_REQUIRE(nq < (int64_t(1) << 31) / nprobe, "nq * nprobe must be below 2^31");
  const int32_t dq = std::max(std::max(d_c, pq.d_s), rerank_k > 0 ? d_rerank : 0);
  ADANNS_REQUIRE(ldq >= dq, "ldq (%lld) is smaller than the prefix (%d)", (long long)ldq, dq);
  if (nq == 0) return ADANNS_OK;
  ADANNS_REQUIRE(Q && dist && ids, "Q, dist and ids must be non-NULL");
  adanns_status s = check_async();
  if (s) return s;
  hipStream_t st = (hipStream_t)stream;
  const int32_t dq_pad = (int32_t)round_up(dq, SLAB);
  auto bytes_of = [&](int64_t m, size_t *carved) {
    size_t t = 0;
    carve(nullptr, ix, m, dq_pad, nprobe, true, &t);
    if (carved) *carved = t;
    return pq_search_scratch_bytes(ix, m, d_c, nprobe, M, rerank_k, d_rerank);
  };
  if (fixed_base && bytes_of(nq, nullptr) > fixed_cap) {
    set_error("the search needs %zu bytes of scratch, more than the %zu given",
              bytes_of(nq, nullptr), fixed_cap);
    return ADANNS_EBUDGET;
  }
  if (!fixed_base && nq > 1 && bytes_of(nq, nullptr) > g_scratch_cap.load()) {  // query chunks
    int64_t chunk = nq;
    while (chunk > 1 && bytes_of(chunk, nullptr) > g_scratch_cap.load()) chunk = (chunk + 1) / 2;
    for (int64_t r0 = 0; r0 < nq; r0 += chunk) {
      const int64_t m = std::min(chunk, nq - r0);
      if ((s = adanns_search_pq(ix, Q + r0 * ldq, m, ldq, d_c, nprobe, M, k, rerank_k, d_rerank,
                                dist + r0 * k, ids + r0 * k, probes ? probes + r0 * nprobe : nullptr,
                                stream)))
        return s;
    }
    return ADANNS_OK;
  }
  size_t total = 0;
  const size_t extra = bytes_of(nq, &total) - total;
  void *base = fixed_base;
  if (!fixed_base && (s = get_scratch(ix, st, total + extra, &base))) return s;
  SearchBufs b = carve((char *)base, ix, nq, dq_pad, nprobe, true, &total);
  Carver c{(char *)base, total, 0};
  float *qr_hi = c.take<float>((size_t)nq * pq.d_s);
  float *qr_lo = c.take<float>((size_t)nq * pq.d_s);
  float *lut = c.take<float>((size_t)nq * M * 256);
  ADANNS_HIP(launch_stage_queries(Q, nq, ldq, dq, b.Qs, b.ldqs, st));
  ADANNS_HIP(launch_coarse(ix, b, nq, d_c, nprobe, probes, st));
  ADANNS_HIP(launch_pq_search(ix, pq, b, nq, nprobe, k, rerank_k, d_rerank, qr_hi, qr_lo, lut,
                              dist, ids, st));
  return ADANNS_OK;
}
}  // namespace adanns

extern "C" {

adanns_status adanns_search_pq(const adanns_index *cix, const float *Q, int64_t nq, int64_t ldq,
                               int32_t d_c, int32_t nprobe, int32_t M, int32_t k,
                               int32_t rerank_k, int32_t d_rerank, float *dist, int64_t *ids,
                               int32_t *probes, void *stream) {
  clear_error();
  return search_pq_impl(cix, Q, nq, ldq, d_c, nprobe, M, k, rerank_k, d_rerank, dist, ids, probes,
                        stream, nullptr, 0);
}

adanns_status adanns_set_precision(adanns_index *ix, int32_t fmt, void *stream) {
  clear_error();
  ADANNS_REQUIRE(ix != nullptr, "index is NULL");
  ADANNS_REQUIRE(fmt == ADANNS_BF16 || fmt == ADANNS_FP8_E4M3,
                 "fmt must be ADANNS_BF16 (1) or ADANNS_FP8_E4M3 (2), got %d", fmt);
  ADANNS_REQUIRE(ix->vec != nullptr, "the index holds no FP32 vectors to quantise");
  if (ix->quant[fmt].vec) return ADANNS_OK;
  adanns_status s = check_async();
  if (s) return s;
  hipStream_t st = (hipStream_t)stream;
  QuantStore q;
  const size_t eb = fmt == ADANNS_BF16 ? 2 : 1;
  auto fail = [&](adanns_status e) {
    void *pp[] = {q.vec, q.scale, q.cent, q.cent_scale, q.emax, q.cent_emax, q.rerr};
    for (void *p : pp)
      if (p) (void)hipFree(p);
    return e;
  };
  if ((s = dmalloc(ix, &q.vec, (size_t)ix->rows_pad * ix->d_pad * eb))) return fail(s);
  if ((s = dmalloc(ix, &q.cent, (size_t)ix->nl_pad * ix->d_cb_pad * eb))) return fail(s);
  if (fmt == ADANNS_FP8_E4M3) {
    if ((s = dmalloc(ix, (void **)&q.scale, (size_t)ix->rows_pad * sizeof(float)))) return fail(s);
    if ((s = dmalloc(ix, (void **)&q.cent_scale, (size_t)ix->nl_pad * sizeof(float))))
      return fail(s);
  }
  if ((s = dmalloc(ix, (void **)&q.emax, sizeof(float))) ||
      (s = dmalloc(ix, (void **)&q.cent_emax, sizeof(float))) ||
      (s = dmalloc(ix, (void **)&q.rerr, (size_t)ix->rows_pad * sizeof(float))))
    return fail(s);
  if (launch_quantize_store(ix, fmt, q, st) || launch_quant_err_max(ix, fmt, q, st)) {
    set_error("HIP error while quantising the vectors");
    return fail(ADANNS_EHIP);
  }
  {
    // the centroids as one list: e4m3 copies (the BF16 copy is made with the
    // vectors), then the largest quantisation error
    int64_t *d_poff2 = nullptr;
    const int64_t h_poff2[2] = {0, ix->nl_pad};
    if (hipMalloc(&d_poff2, 2 * sizeof(int64_t)) ||
        hipMemcpyAsync(d_poff2, h_poff2, 2 * sizeof(int64_t), hipMemcpyHostToDevice, st) ||
        (fmt == ADANNS_FP8_E4M3 && launch_quantize_cent_fp8(ix, d_poff2, q, st)) ||
        launch_quant_err_max_cent(ix, fmt, d_poff2, q, st) || hipStreamSynchronize(st)) {
      if (d_poff2) (void)hipFree(d_poff2);
      set_error("HIP error while quantising the centroids");
      return fail(ADANNS_EHIP);
    }
    (void)hipFree(d_poff2);
  }
  if (hipStreamSynchronize(st)) {
    set_error("HIP error while quantising");
    return fail(ADANNS_EHIP);
  }
  ix->quant[fmt] = q;
  return ADANNS_OK;
}

adanns_status adanns_index_add_row_copy(adanns_index *ix, void *stream) {
  clear_error();
  ADANNS_REQUIRE(ix != nullptr, "index is NULL");
  ADANNS_REQUIRE(ix->vec != nullptr, "the index holds no FP32 vectors to copy");
  if (ix->rows) return ADANNS_OK;
  adanns_status s = check_async();
  if (s) return s;
  hipStream_t st = (hipStream_t)stream;
  float *rows = nullptr;
  if ((s = dmalloc(ix, (void **)&rows, (size_t)ix->rows_pad * ix->d_pad * sizeof(float))))
    return s;
  if (launch_slab_to_rows(ix, rows, st) != hipSuccess || hipStreamSynchronize(st) != hipSuccess) {
    (void)hipGetLastError();
    (void)hipFree(rows);
    ix->own_bytes -= (size_t)ix->rows_pad * ix->d_pad * sizeof(float);
    set_error("HIP error while copying the vectors");
    return ADANNS_EHIP;
  }
  ix->rows = rows;
  return ADANNS_OK;
}

// Query rows for the FP32 steps: read in place when they are 16-byte aligned
// and cover the zero-padded staging width (the kernels read 16-byte pieces up
// to the 32-coordinate slab that holds the last coordinate they use and mask
// what lies past it), else staged into zero-padded rows.
static hipError_t stage_or_in_place(SearchBufs &b, const float *Q, int64_t nq, int64_t ldq,
                                    int32_t dq, hipStream_t st) {
  if (ldq % 4 == 0 && ((uintptr_t)Q & 15) == 0 && ldq >= b.ldqs) {
    b.Qs = const_cast<float *>(Q);
    b.ldqs = ldq;
    return hipSuccess;
  }
  return launch_stage_queries(Q, nq, ldq, dq, b.Qs, b.ldqs, st);
}

adanns_status adanns_search_precision(const adanns_index *cix, const float *Q, int64_t nq,
                                      int64_t ldq, int32_t d_c, int32_t d_s, int32_t nprobe,
                                      int32_t k, int32_t fmt, int32_t rerank_k,
                                      int32_t coarse_margin, float *dist, int64_t *ids,
                                      int32_t *probes, void *stream) {
  clear_error();
  adanns_index *ix = const_cast<adanns_index *>(cix);
  ADANNS_REQUIRE(ix != nullptr, "index is NULL");
  ADANNS_REQUIRE(fmt == ADANNS_BF16 || fmt == ADANNS_FP8_E4M3, "fmt must be 1 or 2, got %d", fmt);
  ADANNS_REQUIRE(ix->quant[fmt].vec != nullptr,
                 "no quantised copy in this format: call adanns_set_precision first");
  ADANNS_REQUIRE(nq >= 0, "nq must be >= 0");
  ADANNS_REQUIRE(d_c >= 1 && d_c <= ix->d_cb, "d_c must be in [1, %d], got %d", ix->d_cb, d_c);
  ADANNS_REQUIRE(d_s >= 1 && d_s <= ix->d, "d_s must be in [1, %d], got %d", ix->d, d_s);
  ADANNS_REQUIRE(nprobe >= 1 && nprobe <= ix->nlist, "nprobe must be in [1, %d], got %d",
                 ix->nlist, nprobe);
  ADANNS_REQUIRE(k >= 1 && rerank_k >= k && rerank_k <= MAX_SHORTLIST - REFINE_MARGIN,
                 "need 1 <= k <= rerank_k <= %d (k %d, rerank_k %d)",
                 MAX_SHORTLIST - REFINE_MARGIN, k, rerank_k);
  ADANNS_REQUIRE(coarse_margin >= 0 && nprobe + coarse_margin <= MAX_SHORTLIST - REFINE_MARGIN,
                 "coarse_margin must be >= 0 with nprobe + coarse_margin <= %d",
                 MAX_SHORTLIST - REFINE_MARGIN);
  ADANNS_REQUIRE(ldq >= ix->d, "ldq (%lld) must be >= d (%d): queries are quantised over d",
                 (long long)ldq, ix->d);
  ADANNS_REQUIRE(nq < (int64_t(1) << 31) / nprobe, "nq * nprobe must be below 2^31");
  if (nq == 0) return ADANNS_OK;
  ADANNS_REQUIRE(Q && dist && ids, "Q, dist and ids must be non-NULL");
  adanns_status s = check_async();
  if (s) return s;
  hipStream_t st = (hipStream_t)stream;
  const int32_t dq = std::max(d_c, d_s);
  const int32_t dq_pad = (int32_t)round_up(dq, SLAB);
  const size_t eb = fmt == ADANNS_BF16 ? 2 : 1;
  auto bytes_of = [&](int64_t m, size_t *carved) {
    size_t t = 0;
    carve(nullptr, ix, m, dq_pad, nprobe, true, &t);
    if (carved) *carved = t;
    return t + (size_t)round_up((size_t)m * ix->d_pad * eb, 256) +
           (size_t)round_up((size_t)m * 4, 256) + 1024;
  };
  if (nq > 1 && bytes_of(nq, nullptr) > g_scratch_cap.load()) {  // query chunks
    int64_t chunk = nq;
    while (chunk > 1 && bytes_of(chunk, nullptr) > g_scratch_cap.load()) chunk = (chunk + 1) / 2;
    for (int64_t r0 = 0; r0 < nq; r0 += chunk) {
      const int64_t m = std::min(chunk, nq - r0);
      if ((s = adanns_search_precision(ix, Q + r0 * ldq, m, ldq, d_c, d_s, nprobe, k, fmt,
                                       rerank_k, coarse_margin, dist + r0 * k, ids + r0 * k,
                                       probes ? probes + r0 * nprobe : nullptr, stream)))
        return s;
    }
    return ADANNS_OK;
  }
  size_t total = 0;
  const size_t extra = bytes_of(nq, &total) - total;
  void *base = nullptr;
  if ((s = get_scratch(ix, st, total + extra, &base))) return s;
  SearchBufs b = carve((char *)base, ix, nq, dq_pad, nprobe, true, &total);
  Carver c{(char *)base, total, 0};
  void *Qq = c.take<uint8_t>((size_t)nq * ix->d_pad * eb);
  float *qscale = c.take<float>((size_t)nq);
  ADANNS_HIP(stage_or_in_place(b, Q, nq, ldq, dq, st));
  ADANNS_HIP(launch_quantize_queries(Q, nq, ldq, ix->d, fmt, Qq, ix->d_pad, qscale, st));
  ADANNS_HIP(launch_precision_search(ix, fmt, b, Qq, ix->d_pad, qscale, nq, d_c, d_s, nprobe, k,
                                     rerank_k, coarse_margin, dist, ids, probes, st));
  return ADANNS_OK;
}

adanns_status adanns_search_filtered(const adanns_index *cix, const float *Q, int64_t nq,
                                     int64_t ldq, int32_t d_c, int32_t d_s, int32_t nprobe,
                                     int32_t k, int32_t fmt, float *dist, int64_t *ids,
                                     int32_t *probes, void *stream) {
  clear_error();
  adanns_index *ix = const_cast<adanns_index *>(cix);
  ADANNS_REQUIRE(ix != nullptr, "index is NULL");
  ADANNS_REQUIRE(fmt == ADANNS_BF16 || fmt == ADANNS_FP8_E4M3, "fmt must be 1 or 2, got %d", fmt);
  ADANNS_REQUIRE(ix->quant[fmt].vec != nullptr,
                 "no quantised copy in this format: call adanns_set_precision first");
  ADANNS_REQUIRE(nq >= 0, "nq must be >= 0");
  ADANNS_REQUIRE(d_c >= 1 && d_c <= ix->d_cb, "d_c must be in [1, %d], got %d", ix->d_cb, d_c);
  ADANNS_REQUIRE(d_s >= 1 && d_s <= ix->d, "d_s must be in [1, %d], got %d", ix->d, d_s);
  ADANNS_REQUIRE(nprobe >= 1 && nprobe <= ix->nlist, "nprobe must be in [1, %d], got %d",
                 ix->nlist, nprobe);
  ADANNS_REQUIRE(k >= 1 && k <= 128, "k must be in [1, 128], got %d", k);
  ADANNS_REQUIRE(ldq >= ix->d, "ldq (%lld) must be >= d (%d): queries are quantised over d",
                 (long long)ldq, ix->d);
  ADANNS_REQUIRE(nq < (int64_t(1) << 31) / nprobe, "nq * nprobe must be below 2^31");
  if (nq == 0) return ADANNS_OK;
  ADANNS_REQUIRE(Q && dist && ids, "Q, dist and ids must be non-NULL");
  adanns_status s = check_async();
  if (s) return s;
  hipStream_t st = (hipStream_t)stream;
  const int32_t dq = std::max(d_c, d_s);
  const int32_t dq_pad = (int32_t)round_up(dq, SLAB);
  const size_t eb = fmt == ADANNS_BF16 ? 2 : 1;
  auto bytes_of = [&](int64_t m, size_t *carved) {
    size_t t = 0;
    carve(nullptr, ix, m, dq_pad, nprobe, true, &t);
    if (carved) *carved = t;
    return t + (size_t)round_up((size_t)m * ix->d_pad * eb, 256) +
           (size_t)round_up((size_t)m * 4, 256) + 1024;
  };
  if (nq > 1 && bytes_of(nq, nullptr) > g_scratch_cap.load()) {  // query chunks
    int64_t chunk = nq;
    while (chunk > 1 && bytes_of(chunk, nullptr) > g_scratch_cap.load()) chunk = (chunk + 1) / 2;
    for (int64_t r0 = 0; r0 < nq; r0 += chunk) {
      const int64_t m = std::min(chunk, nq - r0);
      if ((s = adanns_search_filtered(ix, Q + r0 * ldq, m, ldq, d_c, d_s, nprobe, k, fmt,
                                      dist + r0 * k, ids + r0 * k,
                                      probes ? probes + r0 * nprobe : nullptr, stream)))
        return s;
    }
    return ADANNS_OK;
  }
  size_t total = 0;
  const size_t extra = bytes_of(nq, &total) - total;
  void *base = nullptr;
  if ((s = get_scratch(ix, st, total + extra, &base))) return s;
  SearchBufs b = carve((char *)base, ix, nq, dq_pad, nprobe, true, &total);
  Carver c{(char *)base, total, 0};
  void *Qq = c.take<uint8_t>((size_t)nq * ix->d_pad * eb);
  float *qscale = c.take<float>((size_t)nq);
  ADANNS_HIP(stage_or_in_place(b, Q, nq, ldq, dq, st));
  ADANNS_HIP(launch_quantize_queries(Q, nq, ldq, ix->d, fmt, Qq, ix->d_pad, qscale, st));
  ADANNS_HIP(launch_filtered_search(ix, fmt, b, Qq, ix->d_pad, qscale, nq, d_c, d_s, nprobe, k,
                                    dist, ids, probes, st));
  return ADANNS_OK;
}

adanns_status adanns_index_quantized(const adanns_index *ix, int32_t fmt, void *values,
                                     float *scales) {
  clear_error();
  ADANNS_REQUIRE(ix != nullptr, "index is NULL");
  ADANNS_REQUIRE(fmt == ADANNS_BF16 || fmt == ADANNS_FP8_E4M3, "fmt must be 1 or 2, got %d", fmt);
  ADANNS_REQUIRE(ix->quant[fmt].vec != nullptr, "no quantised copy in this format");
  const size_t eb = fmt == ADANNS_BF16 ? 2 : 1;
  std::vector<uint8_t> lay((size_t)ix->rows_pad * ix->d_pad * eb);
  ADANNS_HIP(hipMemcpy(lay.data(), ix->quant[fmt].vec, lay.size(), hipMemcpyDeviceToHost));
  std::vector<float> sc;
  if (fmt == ADANNS_FP8_E4M3) {
    sc.resize(ix->rows_pad);
    ADANNS_HIP(hipMemcpy(sc.data(), ix->quant[fmt].scale, sc.size() * 4, hipMemcpyDeviceToHost));
  }
  for (int32_t h = 0; h < ix->nlist; ++h) {
    const int64_t p0 = ix->h_poff[h], npad = ix->h_poff[h + 1] - p0;
    for (int64_t r = 0; r < ix->h_len[h]; ++r) {
      const int64_t id = ix->h_ids[ix->h_off[h] + r];
      if (values) {
        for (int32_t dim = 0; dim < ix->d; ++dim) {
          const size_t src = (size_t)(p0 * ix->d_pad + ((int64_t)(dim / SLAB) * npad + r) * SLAB +
                                      dim % SLAB) * eb;
          std::memcpy((uint8_t *)values + ((size_t)id * ix->d + dim) * eb, &lay[src], eb);
        }
      }
      if (scales) scales[id] = fmt == ADANNS_FP8_E4M3 ? sc[p0 + r] : 1.0f;
    }
  }
  return ADANNS_OK;
}

adanns_status adanns_timing_enable(int32_t enable) {
  clear_error();
  g_timing.store(enable != 0);
  return ADANNS_OK;
}

adanns_status adanns_timing_reset(void) {
  clear_error();
  adanns_status s = resolve_timers();
  std::lock_guard<std::mutex> lk(g_tmu);
  g_totals.clear();
  return s;
}

adanns_status adanns_timing_read(const char *kernel, int64_t *launches, double *total_ms) {
  clear_error();
  ADANNS_REQUIRE(kernel != nullptr, "kernel name is NULL");
  adanns_status s = resolve_timers();
  if (s) return s;
  std::lock_guard<std::mutex> lk(g_tmu);
  auto it = g_totals.find(kernel);
  if (launches) *launches = it == g_totals.end() ? 0 : it->second.first;
  if (total_ms) *total_ms = it == g_totals.end() ? 0.0 : it->second.second;
  return ADANNS_OK;
}

adanns_status adanns_stream_read(const void *buf, size_t bytes, float *partial, int32_t grid,
                                 void *stream) {
  clear_error();
  ADANNS_REQUIRE(buf != nullptr && partial != nullptr, "buf and partial must be non-NULL");
  ADANNS_REQUIRE(bytes % 16 == 0 && ((uintptr_t)buf & 15) == 0,
                 "buf must be 16-byte aligned and bytes a multiple of 16");
  ADANNS_REQUIRE(grid >= 1 && grid <= 65536, "grid must be in [1, 65536], got %d", grid);
  adanns_status s = check_async();
  if (s) return s;
  if (bytes == 0) return ADANNS_OK;
  KernelTimer tm("stream_read", (hipStream_t)stream);
  ADANNS_HIP(launch_stream_read(buf, bytes, partial, grid, (hipStream_t)stream));
  return ADANNS_OK;
}

adanns_status adanns_selection_stats(int64_t *reselected, int64_t *uncertified, int32_t reset) {
  clear_error();
  adanns_status s = check_async();
  if (s) return s;
  unsigned long long v[2] = {0ull, 0ull};
  ADANNS_HIP(read_selection_stats(v, 0, reset != 0));
  if (reselected) *reselected = (int64_t)v[0];
  if (uncertified) *uncertified = (int64_t)v[1];
  return ADANNS_OK;
}

adanns_status adanns_filtered_stats(int64_t *measured, int64_t *windowed, int32_t reset) {
  clear_error();
  adanns_status s = check_async();
  if (s) return s;
  unsigned long long v[2] = {0ull, 0ull};
  ADANNS_HIP(read_selection_stats(v, 2, reset != 0));
  if (measured) *measured = (int64_t)v[0];
  if (windowed) *windowed = (int64_t)v[1];
  return ADANNS_OK;
}

adanns_status adanns_index_info(const adanns_index *ix, int64_t *n, int32_t *d, int32_t *nlist,
                                int32_t *d_c_build) {
  clear_error();
  ADANNS_REQUIRE(ix != nullptr, "index is NULL");
  if (n) *n = ix->n;
  if (d) *d = ix->d;
  if (nlist) *nlist = ix->nlist;
  if (d_c_build) *d_c_build = ix->d_cb;
  return ADANNS_OK;
}

adanns_status adanns_index_lists(const adanns_index *ix, int64_t *offsets, int64_t *ids) {
  clear_error();
  ADANNS_REQUIRE(ix != nullptr, "index is NULL");
  if (offsets) std::memcpy(offsets, ix->h_off.data(), (ix->nlist + 1) * sizeof(int64_t));
  if (ids) std::memcpy(ids, ix->h_ids.data(), ix->n * sizeof(int64_t));
  return ADANNS_OK;
}

adanns_status adanns_index_centroids(const adanns_index *ix, float *centroids) {
  clear_error();
  ADANNS_REQUIRE(ix != nullptr && centroids != nullptr, "index and centroids must be non-NULL");
  ADANNS_HIP(hipMemcpy2D(centroids, ix->d_cb * sizeof(float), ix->cent, ix->d_cb_pad * sizeof(float),
                         ix->d_cb * sizeof(float), ix->nlist, hipMemcpyDeviceToHost));
  return ADANNS_OK;
}

size_t adanns_index_device_bytes(const adanns_index *cix) {
  if (!cix) return 0;
  adanns_index *ix = const_cast<adanns_index *>(cix);
  std::lock_guard<std::mutex> lk(ix->mu);
  size_t b = ix->own_bytes;
  for (auto &kv : ix->scratch) b += kv.second.bytes;
  return b;
}

// ---- persistence ----------------------------------------------------------
// File: "ADANNSIX", u32 version, u32 0, i64 n, i32 d, i32 nlist, i32 d_cb,
// i32 d_pad, i64 rows_pad, i64 offsets[nlist + 1], i64 ids[n], f32
// centroids[nlist][d_cb], f32 vectors[rows_pad][d_pad] (list layout), i32
// number of PQ codecs, then per codec i32 M, i32 d_s, f32 R[d_s][d_s], f32
// codebooks[M][256][d_s / M], u8 codes[rows_pad][M] (list layout), and
// "XINSNNDA". Little-endian, as the host writes it.
static const char kIxMagic[8] = {'A', 'D', 'A', 'N', 'N', 'S', 'I', 'X'};
static const char kIxTrailer[8] = {'X', 'I', 'N', 'S', 'N', 'N', 'D', 'A'};
static const uint32_t kIxVersion = 1;

namespace {
struct File {
  FILE *f = nullptr;
  ~File() {
    if (f) std::fclose(f);
  }
  bool put(const void *p, size_t n) { return std::fwrite(p, 1, n, f) == n; }
  bool get(void *p, size_t n) { return std::fread(p, 1, n, f) == n; }
};

adanns_status dev_to_file(File &fl, const void *dev, size_t bytes) {
  std::vector<char> buf(std::min<size_t>(std::max<size_t>(bytes, 1), size_t(64) << 20));
  for (size_t o = 0; o < bytes; o += buf.size()) {
    const size_t n = std::min(buf.size(), bytes - o);
    ADANNS_HIP(hipMemcpy(buf.data(), (const char *)dev + o, n, hipMemcpyDeviceToHost));
    if (!fl.put(buf.data(), n)) {
      set_error("write failed");
      return ADANNS_EIO;
    }
  }
  return ADANNS_OK;
}

adanns_status file_to_dev(File &fl, void *dev, size_t bytes, hipStream_t st) {
  std::vector<char> buf(std::min<size_t>(std::max<size_t>(bytes, 1), size_t(64) << 20));
  for (size_t o = 0; o < bytes; o += buf.size()) {
    const size_t n = std::min(buf.size(), bytes - o);
    if (!fl.get(buf.data(), n)) {
      set_error("the file ends before the index does");
      return ADANNS_EIO;
    }
    ADANNS_HIP(hipMemcpyAsync((char *)dev + o, buf.data(), n, hipMemcpyHostToDevice, st));
    ADANNS_HIP(hipStreamSynchronize(st));
  }
  return ADANNS_OK;
}
}  // namespace

adanns_status adanns_index_save(const adanns_index *ix, const char *path) {
  clear_error();
  ADANNS_REQUIRE(ix != nullptr && path != nullptr, "index and path must be non-NULL");
  ADANNS_HIP(hipDeviceSynchronize());
  File fl;
  fl.f = std::fopen(path, "wb");
  if (!fl.f) {
    set_error("cannot open %s for writing", path);
    return ADANNS_EIO;
  }
  const uint32_t ver[2] = {kIxVersion, 0};
  const int32_t dims[4] = {ix->d, ix->nlist, ix->d_cb, ix->d_pad};
  bool ok = fl.put(kIxMagic, 8) && fl.put(ver, 8) && fl.put(&ix->n, 8) && fl.put(dims, 16) &&
            fl.put(&ix->rows_pad, 8) &&
            fl.put(ix->h_off.data(), (ix->nlist + 1) * sizeof(int64_t)) &&
            fl.put(ix->h_ids.data(), ix->n * sizeof(int64_t));
  if (!ok) {
    set_error("write failed: %s", path);
    return ADANNS_EIO;
  }
  std::vector<float> cent((size_t)ix->nlist * ix->d_cb);
  ADANNS_HIP(hipMemcpy2D(cent.data(), ix->d_cb * sizeof(float), ix->cent,
                         ix->d_cb_pad * sizeof(float), ix->d_cb * sizeof(float), ix->nlist,
                         hipMemcpyDeviceToHost));
  if (!fl.put(cent.data(), cent.size() * sizeof(float))) {
    set_error("write failed: %s", path);
    return ADANNS_EIO;
  }
  adanns_status s;
  if ((s = dev_to_file(fl, ix->vec, (size_t)ix->rows_pad * ix->d_pad * sizeof(float)))) return s;
  const int32_t npq = (int32_t)ix->pq.size();
  if (!fl.put(&npq, 4)) {
    set_error("write failed: %s", path);
    return ADANNS_EIO;
  }
  for (const auto &kv : ix->pq) {
    const PqCodec &c = kv.second;
    const int32_t hdr[2] = {c.M, c.d_s};
    if (!fl.put(hdr, 8)) {
      set_error("write failed: %s", path);
      return ADANNS_EIO;
    }
    if ((s = dev_to_file(fl, c.R, (size_t)c.d_s * c.d_s * sizeof(float))) ||
        (s = dev_to_file(fl, c.cb, (size_t)c.M * 256 * c.dsub * sizeof(float))) ||
        (s = dev_to_file(fl, c.codes, (size_t)ix->rows_pad * c.M)))
      return s;
  }
  if (!fl.put(kIxTrailer, 8) || std::fflush(fl.f) != 0) {
    set_error("write failed: %s", path);
    return ADANNS_EIO;
  }
  return ADANNS_OK;
}

adanns_status adanns_index_load(const char *path, void *stream, adanns_index **out) {
  clear_error();
  ADANNS_REQUIRE(path != nullptr && out != nullptr, "path and out must be non-NULL");
  adanns_status s;
  hipStream_t st = (hipStream_t)stream;
  File fl;
  fl.f = std::fopen(path, "rb");
  if (!fl.f) {
    set_error("cannot open %s", path);
    return ADANNS_EIO;
  }
  auto bad = [&](const char *what) {
    set_error("%s is not an index file of this version (%s)", path, what);
    return ADANNS_EIO;
  };
  char magic[8];
  uint32_t ver[2];
  int64_t n = 0, rows_pad = 0;
  int32_t dims[4];
  if (!fl.get(magic, 8) || std::memcmp(magic, kIxMagic, 8) != 0) return bad("magic");
  if (!fl.get(ver, 8) || ver[0] != kIxVersion) return bad("version");
  if (!fl.get(&n, 8) || !fl.get(dims, 16) || !fl.get(&rows_pad, 8)) return bad("header");
  const int32_t d = dims[0], nlist = dims[1], d_cb = dims[2];
  if (n < 1 || n >= (int64_t(1) << 31) || d < 1 || d > 8192 || nlist < 1 || nlist > 65536 ||
      d_cb < 1 || d_cb > d || dims[3] != (int32_t)round_up(d, SLAB))
    return bad("sizes");
  std::vector<int64_t> off(nlist + 1), ids(n);
  if (!fl.get(off.data(), off.size() * 8) || !fl.get(ids.data(), ids.size() * 8))
    return bad("lists");
  if (off[0] != 0 || off[nlist] != n) return bad("offsets");
  std::vector<int32_t> assign(n, -1);
  for (int32_t h = 0; h < nlist; ++h) {
    if (off[h + 1] < off[h]) return bad("offsets");
    for (int64_t i = off[h]; i < off[h + 1]; ++i) {
      const int64_t j = ids[i];
      if (j < 0 || j >= n || assign[j] != -1) return bad("ids");
      if (i > off[h] && ids[i - 1] >= j) return bad("list order");
      assign[j] = h;
    }
  }
  std::vector<float> cent((size_t)nlist * d_cb);
  if (!fl.get(cent.data(), cent.size() * sizeof(float))) return bad("centroids");
  // the file's host part is checked before any device work
  if ((s = check_async())) return s;
  adanns_index *ix = new (std::nothrow) adanns_index();
  if (!ix) {
    set_error("out of host memory");
    return ADANNS_ENOMEM;
  }
  auto fail = [&](adanns_status e) {
    free_index_memory(ix);
    delete ix;
    return e;
  };
  init_index_shape(ix, n, d, nlist, d_cb);
  if ((s = build_layout(ix, Mat{}, assign, st))) return fail(s);
  if (ix->rows_pad != rows_pad) return fail(bad("layout rows"));
  {
    DevFree tmp;
    float *dc = nullptr;
    if (hipMalloc(&dc, cent.size() * sizeof(float)) != hipSuccess) {
      set_error("out of device memory");
      return fail(ADANNS_ENOMEM);
    }
    tmp.ptrs.push_back(dc);
    if (hipMemcpy(dc, cent.data(), cent.size() * sizeof(float), hipMemcpyHostToDevice)) {
      set_error("HIP error while loading the centroids");
      return fail(ADANNS_EHIP);
    }
    if ((s = build_centroids(ix, dc, d_cb, st))) return fail(s);
  }
  if ((s = file_to_dev(fl, ix->vec, (size_t)rows_pad * ix->d_pad * sizeof(float), st)) ||
      (s = vector_norm_bound(ix, st)))
    return fail(s);
  int32_t npq = 0;
  if (!fl.get(&npq, 4) || npq < 0 || npq > 16) return fail(bad("codec count"));
  for (int32_t i = 0; i < npq; ++i) {
    int32_t hdr[2];
    if (!fl.get(hdr, 8)) return fail(bad("codec header"));
    PqCodec c;
    c.M = hdr[0];
    c.d_s = hdr[1];
    if (c.M < 4 || c.M > 64 || c.M % 4 || c.d_s < 1 || c.d_s > d || c.d_s > 2048 ||
        c.d_s % c.M || ix->pq.count(c.M))
      return fail(bad("codec sizes"));
    c.dsub = c.d_s / c.M;
    // registered first so that a failure below releases it with the index
    ix->pq[c.M] = c;
    PqCodec &cc = ix->pq[c.M];
    if ((s = dmalloc(ix, (void **)&cc.R, (size_t)c.d_s * c.d_s * sizeof(float))) ||
        (s = dmalloc(ix, (void **)&cc.cb, (size_t)c.M * 256 * c.dsub * sizeof(float))) ||
        (s = dmalloc(ix, (void **)&cc.codes, (size_t)rows_pad * c.M)))
      return fail(s);
    if ((s = file_to_dev(fl, cc.R, (size_t)c.d_s * c.d_s * sizeof(float), st)) ||
        (s = file_to_dev(fl, cc.cb, (size_t)c.M * 256 * c.dsub * sizeof(float), st)) ||
        (s = file_to_dev(fl, cc.codes, (size_t)rows_pad * c.M, st)))
      return fail(s);
  }
  char trailer[8];
  if (!fl.get(trailer, 8) || std::memcmp(trailer, kIxTrailer, 8) != 0) return fail(bad("trailer"));
  *out = ix;
  return ADANNS_OK;
}

void adanns_index_free(adanns_index *ix) {
  if (!ix) return;
  (void)hipDeviceSynchronize();
  free_index_memory(ix);
  delete ix;
}

}  // extern "C"
