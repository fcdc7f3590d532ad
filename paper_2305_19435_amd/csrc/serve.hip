// Serving form: an open-loop request loop over an IVF-PQ index with
// admission by an HBM budget, continuous batching into per-budget steps,
// several streams in flight, completion events, and per-request latency.
#include <algorithm>
#include <chrono>
#include <cstring>
#include <deque>
#include <thread>

#include "internal.h"

namespace adanns {
namespace {

__global__ void k_scatter_rows(const float *__restrict__ sd, const int64_t *__restrict__ si,
                               int64_t nrows, int32_t k, const int64_t *__restrict__ rows,
                               float *__restrict__ dd, int64_t *__restrict__ di) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nrows * k) return;
  int64_t r = i / k, j = i % k;
  dd[rows[r] * k + j] = sd[i];
  di[rows[r] * k + j] = si[i];
}

// First-fit allocator over one device region (offsets only; 256-byte units).
struct Pool {
  std::vector<std::pair<size_t, size_t>> free_;  // (offset, size), by offset
  explicit Pool(size_t cap) { free_.push_back({0, cap / 256 * 256}); }
  static size_t unit(size_t b) { return (b + 255) / 256 * 256; }
  size_t largest() const {
    size_t m = 0;
    for (const auto &f : free_) m = std::max(m, f.second);
    return m;
  }
  bool alloc(size_t bytes, size_t *off) {
    bytes = unit(bytes);
    for (size_t i = 0; i < free_.size(); ++i)
      if (free_[i].second >= bytes) {
        *off = free_[i].first;
        free_[i].first += bytes;
        free_[i].second -= bytes;
        if (free_[i].second == 0) free_.erase(free_.begin() + i);
        return true;
      }
    return false;
  }
  void release(size_t off, size_t bytes) {
    bytes = unit(bytes);
    size_t i = 0;
    while (i < free_.size() && free_[i].first < off) ++i;
    free_.insert(free_.begin() + i, {off, bytes});
    if (i + 1 < free_.size() && free_[i].first + free_[i].second == free_[i + 1].first) {
      free_[i].second += free_[i + 1].second;
      free_.erase(free_.begin() + i + 1);
    }
    if (i > 0 && free_[i - 1].first + free_[i - 1].second == free_[i].first) {
      free_[i - 1].second += free_[i].second;
      free_.erase(free_.begin() + i);
    }
  }
};

struct Slot {
  hipStream_t st = nullptr;
  hipEvent_t done = nullptr;
  float *Qstep = nullptr;
  float *dstep = nullptr;
  int64_t *istep = nullptr;
  int64_t *rows_dev = nullptr;
  int64_t *rows_host = nullptr;  // pinned
  std::vector<int64_t> reqs;     // requests of the step in flight
  size_t bytes = 0;              // its search scratch: a region of the pool
  size_t off = 0;
  bool busy = false;
};

}  // namespace
}  // namespace adanns

using namespace adanns;

extern "C" {

adanns_status adanns_serve(const adanns_index *index, const float *Q, int64_t ldq, int64_t n,
                           const double *arrival_s, const int32_t *d_c, const int32_t *nprobe,
                           const int32_t *M, int32_t k, int32_t rerank_k, int32_t d_rerank,
                           int32_t nstreams, int32_t max_batch, size_t hbm_budget, float *dist,
                           int64_t *ids, double *latency_s, adanns_serve_stats *stats) {
  clear_error();
  adanns_index *ix = const_cast<adanns_index *>(index);
  ADANNS_REQUIRE(ix != nullptr, "index is NULL");
  ADANNS_REQUIRE(n >= 0, "n must be >= 0");
  ADANNS_REQUIRE(nstreams >= 1 && nstreams <= 16, "nstreams must be in [1, 16]");
  ADANNS_REQUIRE(max_batch >= 1 && max_batch <= 65536, "max_batch must be in [1, 65536]");
  ADANNS_REQUIRE(k >= 1 && k <= MAX_SHORTLIST - REFINE_MARGIN, "k out of range");
  if (n == 0) return ADANNS_OK;
  ADANNS_REQUIRE(Q && arrival_s && d_c && nprobe && M && dist && ids && latency_s,
                 "Q, arrival_s, budgets, dist, ids and latency_s must be non-NULL");
  int32_t dq = 1, max_np = 1, max_M = 4, max_ds = 1;
  for (int64_t i = 0; i < n; ++i) {
    auto it = ix->pq.find(M[i]);
    ADANNS_REQUIRE(it != ix->pq.end(), "request %lld: no PQ codec with M = %d", (long long)i, M[i]);
    ADANNS_REQUIRE(d_c[i] >= 1 && d_c[i] <= ix->d_cb, "request %lld: d_c out of range", (long long)i);
    ADANNS_REQUIRE(nprobe[i] >= 1 && nprobe[i] <= ix->nlist, "request %lld: nprobe out of range",
                   (long long)i);
    ADANNS_REQUIRE(i == 0 || arrival_s[i] >= arrival_s[i - 1], "arrival times must not decrease");
    dq = std::max(dq, std::max(d_c[i], it->second.d_s));
    max_np = std::max(max_np, nprobe[i]);
    max_M = std::max(max_M, M[i]);
    max_ds = std::max(max_ds, it->second.d_s);
  }
  if (rerank_k > 0) dq = std::max(dq, d_rerank);
  ADANNS_REQUIRE(ldq >= dq, "ldq (%lld) is smaller than the widest prefix (%d)", (long long)ldq, dq);
  adanns_status s = ADANNS_OK;
  {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
      set_error("HIP error from an earlier launch: %s", hipGetErrorString(e));
      return ADANNS_EHIP;
    }
  }

  // step bytes of ``cnt`` requests of request r's budget: the search scratch
  // exactly as the search carves it
  auto step_bytes = [&](int64_t r, int64_t cnt) {
    return pq_search_scratch_bytes(ix, cnt, d_c[r], nprobe[r], M[r], rerank_k, d_rerank);
  };
  // the budget is one device region: every step's search scratch is carved
  // out of it, so the admitted bytes are the bytes in use
  void *pool_base = nullptr;
  Pool pool(hbm_budget);
  std::vector<Slot> slots(nstreams);
  auto cleanup = [&]() {
    for (Slot &sl : slots) {
      if (sl.st) (void)hipStreamSynchronize(sl.st);
      if (sl.done) (void)hipEventDestroy(sl.done);
      void *pp[] = {sl.Qstep, sl.dstep, sl.istep, sl.rows_dev};
      for (void *p : pp)
        if (p) (void)hipFree(p);
      if (sl.rows_host) (void)hipHostFree(sl.rows_host);
      if (sl.st) (void)hipStreamDestroy(sl.st);
    }
    if (pool_base) (void)hipFree(pool_base);
  };
  if (hbm_budget >= 256 && hipMalloc(&pool_base, hbm_budget / 256 * 256) != hipSuccess) {
    (void)hipGetLastError();
    pool_base = nullptr;
    set_error("could not allocate the %zu-byte serving budget", hbm_budget);
    return ADANNS_ENOMEM;
  }
  for (Slot &sl : slots) {
    if (hipStreamCreateWithFlags(&sl.st, hipStreamNonBlocking) ||
        hipEventCreateWithFlags(&sl.done, hipEventDisableTiming) ||
        hipMalloc(&sl.Qstep, (size_t)max_batch * ldq * sizeof(float)) ||
        hipMalloc(&sl.dstep, (size_t)max_batch * k * sizeof(float)) ||
        hipMalloc(&sl.istep, (size_t)max_batch * k * sizeof(int64_t)) ||
        hipMalloc(&sl.rows_dev, (size_t)max_batch * sizeof(int64_t)) ||
        hipHostMalloc(&sl.rows_host, (size_t)max_batch * sizeof(int64_t), 0)) {
      (void)hipGetLastError();
      cleanup();
      set_error("could not create the serving streams and step buffers");
      return ADANNS_ENOMEM;
    }
  }
  // launch one step of ``cnt`` requests (same budget) on a slot, its search
  // scratch the pool region [off, off + bytes)
  auto launch = [&](Slot &sl, const std::vector<int64_t> &reqs, size_t off,
                    size_t bytes) -> adanns_status {
    const int64_t cnt = (int64_t)reqs.size();
    std::memcpy(sl.rows_host, reqs.data(), cnt * sizeof(int64_t));
    ADANNS_HIP(hipMemcpyAsync(sl.rows_dev, sl.rows_host, cnt * sizeof(int64_t),
                              hipMemcpyHostToDevice, sl.st));
    ADANNS_HIP(launch_stage_rows(f32mat(Q, ldq), sl.rows_dev, nullptr, cnt, (int32_t)ldq, sl.Qstep,
                                 ldq, sl.st));
    const int64_t r0 = reqs[0];
    adanns_status e = search_pq_impl(ix, sl.Qstep, cnt, ldq, d_c[r0], nprobe[r0], M[r0], k,
                                     rerank_k, d_rerank, sl.dstep, sl.istep, nullptr, sl.st,
                                     (char *)pool_base + off, bytes);
    if (e) return e;
    hipLaunchKernelGGL(k_scatter_rows, dim3((unsigned)cdiv(cnt * k, 256)), dim3(256), 0, sl.st,
                       sl.dstep, sl.istep, cnt, k, sl.rows_dev, dist, ids);
    ADANNS_HIP(hipGetLastError());
    ADANNS_HIP(hipEventRecord(sl.done, sl.st));
    return ADANNS_OK;
  };
  // warm-up (kernels loaded before the clock starts): one request of each
  // budget that fits, on every stream; results are overwritten later
  {
    std::vector<int64_t> seen;
    for (int64_t i = 0; i < n; ++i) {
      bool dup = false;
      for (int64_t j : seen)
        dup = dup || (d_c[j] == d_c[i] && nprobe[j] == nprobe[i] && M[j] == M[i]);
      if (dup) continue;
      seen.push_back(i);
      const size_t b = step_bytes(i, 1);
      if (b > hbm_budget / 256 * 256) continue;
      for (Slot &sl : slots) {
        if ((s = launch(sl, std::vector<int64_t>{i}, 0, b))) {
          cleanup();
          return s;
        }
        (void)hipStreamSynchronize(sl.st);
      }
    }
  }

  std::vector<size_t> need(n);
  for (int64_t i = 0; i < n; ++i) need[i] = step_bytes(i, 1);
  for (int64_t i = 0; i < n; ++i) latency_s[i] = -1.0;
  std::deque<int64_t> pending;
  int64_t next = 0, done_cnt = 0, steps = 0, batched = 0, rejected = 0;
  size_t inflight = 0, max_inflight = 0;
  int32_t max_slots_busy = 0;
  using clk = std::chrono::steady_clock;
  const auto t0 = clk::now();
  auto now_s = [&]() { return std::chrono::duration<double>(clk::now() - t0).count(); };

  while (done_cnt + rejected < n) {
    bool progress = false;
    // completions
    for (Slot &sl : slots) {
      if (!sl.busy) continue;
      hipError_t q = hipEventQuery(sl.done);
      if (q == hipErrorNotReady) continue;
      if (q != hipSuccess) {
        cleanup();
        set_error("serving step failed: %s", hipGetErrorString(q));
        return ADANNS_EHIP;
      }
      const double t = now_s();
      for (int64_t r : sl.reqs) latency_s[r] = t - arrival_s[r];
      done_cnt += (int64_t)sl.reqs.size();
      inflight -= sl.bytes;
      pool.release(sl.off, sl.bytes);
      sl.busy = false;
      sl.reqs.clear();
      progress = true;
    }
    // arrivals
    const double t = now_s();
    while (next < n && arrival_s[next] <= t) pending.push_back(next++);
    // admission and batching: the oldest pending request's budget group
    // first (no starvation), as many of that group as fit the budget
    for (Slot &sl : slots) {
      if (sl.busy || pending.empty()) continue;
      const int64_t head = pending.front();
      if (Pool::unit(need[head]) > hbm_budget / 256 * 256) {  // can never be admitted
        pending.pop_front();
        ++rejected;
        progress = true;
        continue;
      }
      const size_t avail = pool.largest();
      if (Pool::unit(need[head]) > avail) break;  // wait for memory to free up
      // the head's budget group, as many as the largest free region holds
      std::vector<int64_t> take;
      for (auto it = pending.begin(); it != pending.end() && (int64_t)take.size() < max_batch;) {
        const int64_t r = *it;
        if (d_c[r] == d_c[head] && nprobe[r] == nprobe[head] && M[r] == M[head] &&
            Pool::unit(step_bytes(head, (int64_t)take.size() + 1)) <= avail) {
          take.push_back(r);
          it = pending.erase(it);
        } else {
          ++it;
        }
      }
      const size_t bytes = Pool::unit(step_bytes(head, (int64_t)take.size()));
      size_t off = 0;
      if (!pool.alloc(bytes, &off)) {  // cannot happen: bytes <= the largest free region
        cleanup();
        set_error("serving pool allocation failed");
        return ADANNS_EBUDGET;
      }
      if ((s = launch(sl, take, off, bytes))) {
        cleanup();
        return s;
      }
      sl.reqs = std::move(take);
      sl.bytes = bytes;
      sl.off = off;
      sl.busy = true;
      inflight += bytes;
      max_inflight = std::max(max_inflight, inflight);
      ++steps;
      batched += (int64_t)sl.reqs.size();
      progress = true;
    }
    int32_t busy = 0;
    for (Slot &sl : slots) busy += sl.busy;
    max_slots_busy = std::max(max_slots_busy, busy);
    if (!progress) std::this_thread::sleep_for(std::chrono::microseconds(20));
  }
  const double wall = now_s();
  cleanup();
  if (stats) {
    stats->wall_s = wall;
    stats->steps = steps;
    stats->mean_batch = steps ? (double)batched / steps : 0.0;
    stats->max_inflight_bytes = max_inflight;
    stats->max_streams_busy = max_slots_busy;
    stats->rejected = rejected;
  }
  return ADANNS_OK;
}

}  // extern "C"
