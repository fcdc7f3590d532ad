// C ABI of the library: argument validation, index import and layout,
// per-stream scratch memory and the search driver. See include/adanns.h.
#include <algorithm>
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
  void *ptrs[] = {ix->vec, ix->poff, ix->len, ix->rowid, ix->cent, ix->cent_slab};
  for (void *p : ptrs)
    if (p) (void)hipFree(p);
  for (auto &kv : ix->scratch)
    if (kv.second.base) (void)hipFree(kv.second.base);
  ix->scratch.clear();
}

// Lays out lists, ids and vectors for a validated assignment (host array).
adanns_status build_layout(adanns_index *ix, const float *X, int64_t ldx,
                           const std::vector<int32_t> &assign, hipStream_t st) {
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
  ADANNS_HIP(launch_layout(X, ldx, ix->d, ix->rowid, d_row_list, ix->poff, ix->rows_pad, ix->d_pad,
                           ix->vec, st));
  ADANNS_HIP(hipStreamSynchronize(st));
  return ADANNS_OK;
}

// Centroids: a zero-padded row-major copy and a one-list slab layout.
adanns_status build_centroids(adanns_index *ix, const float *centroids, hipStream_t st) {
  const int32_t nlist = ix->nlist;
  adanns_status s;
  if ((s = dmalloc(ix, (void **)&ix->cent, (size_t)nlist * ix->d_cb_pad * sizeof(float)))) return s;
  if ((s = dmalloc(ix, (void **)&ix->cent_slab, (size_t)ix->nl_pad * ix->d_cb_pad * sizeof(float))))
    return s;
  ADANNS_HIP(hipMemsetAsync(ix->cent, 0, (size_t)nlist * ix->d_cb_pad * sizeof(float), st));
  ADANNS_HIP(hipMemcpy2DAsync(ix->cent, ix->d_cb_pad * sizeof(float), centroids,
                              ix->d_cb * sizeof(float), ix->d_cb * sizeof(float), nlist,
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
  ADANNS_HIP(launch_layout(ix->cent, ix->d_cb_pad, ix->d_cb, d_src, d_rl, d_poff, ix->nl_pad,
                           ix->d_cb_pad, ix->cent_slab, st));
  ADANNS_HIP(hipStreamSynchronize(st));
  return ADANNS_OK;
}

// Scratch sizes of one search call, carved in a fixed order.
SearchBufs carve(char *base, const adanns_index *ix, int64_t nq, int32_t dq_pad, int32_t nprobe,
                 bool coarse, size_t *total) {
  Carver c{base, 0, 0};
  SearchBufs b{};
  b.ldqs = dq_pad;
  b.Qs = c.take<float>((size_t)nq * dq_pad);
  b.S = coarse ? c.take<float>((size_t)nq * ix->nlist) : nullptr;
  b.probes = c.take<int32_t>((size_t)nq * nprobe);
  b.cnt = c.take<int32_t>(ix->nlist);
  b.cursor = c.take<int32_t>(ix->nlist);
  b.bkt_off = c.take<int32_t>(ix->nlist);
  b.tile_off = c.take<int32_t>(ix->nlist + 1);
  b.bucket = c.take<int32_t>((size_t)nq * nprobe);
  b.seg_off = c.take<int64_t>(nq + 1);
  b.pair_base = c.take<int64_t>((size_t)nq * nprobe);
  b.D = c.take<float>((size_t)nq * ix->top_prefix[nprobe]);
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

extern "C" {

const char *adanns_last_error(void) { return g_err; }

const char *adanns_version(void) { return "adanns-mi355x 0.1 (gfx950)"; }

adanns_status adanns_ivf_import(const float *X, int64_t n, int32_t d, int64_t ldx,
                                const float *centroids, int32_t nlist, int32_t d_c_build,
                                const int32_t *assign, void *stream, adanns_index **out) {
  clear_error();
  ADANNS_REQUIRE(out != nullptr, "out is NULL");
  ADANNS_REQUIRE(X && centroids && assign, "X, centroids and assign must be non-NULL");
  ADANNS_REQUIRE(n >= 1 && n < (int64_t(1) << 31), "n must be in [1, 2^31), got %lld",
                 (long long)n);
  ADANNS_REQUIRE(d >= 1 && d <= 8192, "d must be in [1, 8192], got %d", d);
  ADANNS_REQUIRE(ldx >= d, "ldx (%lld) must be >= d (%d)", (long long)ldx, d);
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
  (void)hipGetDevice(&ix->device);
  ix->n = n;
  ix->d = d;
  ix->d_pad = (int32_t)round_up(d, SLAB);
  ix->nlist = nlist;
  ix->d_cb = d_c_build;
  ix->d_cb_pad = (int32_t)round_up(d_c_build, SLAB);
  ix->nl_pad = (int32_t)round_up(nlist, ROWPAD);
  if ((s = build_layout(ix, X, ldx, h_assign, st)) || (s = build_centroids(ix, centroids, st))) {
    free_index_memory(ix);
    delete ix;
    return s;
  }
  *out = ix;
  return ADANNS_OK;
}

static adanns_status search_common(const adanns_index *cix, const float *Q, int64_t nq,
                                   int64_t ldq, int32_t d_c, int32_t d_s, int32_t nprobe,
                                   const int32_t *given_probes, int32_t k, float *dist,
                                   int64_t *ids, int32_t *probes_out, void *stream) {
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
  size_t total = 0;
  carve(nullptr, ix, nq, dq_pad, nprobe, coarse, &total);
  void *base = nullptr;
  if ((s = get_scratch(ix, st, total, &base))) return s;
  SearchBufs b = carve((char *)base, ix, nq, dq_pad, nprobe, coarse, &total);
  ADANNS_HIP(launch_stage_queries(Q, nq, ldq, dq, b.Qs, b.ldqs, st));
  if (coarse) {
    ADANNS_HIP(launch_coarse(ix, b, nq, d_c, nprobe, probes_out, st));
  } else {
    ADANNS_HIP(hipMemcpyAsync(b.probes, given_probes, (size_t)nq * nprobe * sizeof(int32_t),
                              hipMemcpyDeviceToDevice, st));
  }
  ADANNS_HIP(launch_scan(ix, b, nq, d_s, nprobe, k, dist, ids, st));
  return ADANNS_OK;
}

adanns_status adanns_search(const adanns_index *index, const float *Q, int64_t nq, int64_t ldq,
                            int32_t d_c, int32_t d_s, int32_t nprobe, int32_t k, float *dist,
                            int64_t *ids, int32_t *probes, void *stream) {
  clear_error();
  return search_common(index, Q, nq, ldq, d_c, d_s, nprobe, nullptr, k, dist, ids, probes, stream);
}

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

void adanns_index_free(adanns_index *ix) {
  if (!ix) return;
  (void)hipDeviceSynchronize();
  free_index_memory(ix);
  delete ix;
}

}  // extern "C"
