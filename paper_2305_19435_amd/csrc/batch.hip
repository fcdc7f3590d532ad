// Batching form: many (index, d_c, d_s, nprobe, k) search configurations with
// uneven query batches run as one set of persistent launches over a
// descriptor table, optionally captured once into a hipGraph and replayed;
// plus the tile-shape autotuner and its cache.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>

#include "internal.h"

namespace adanns {

// ---- autotune cache ------------------------------------------------------------
// Key: the search shape bucketed by powers of two (d_s, nprobe and the
// expected number of queries probing a list), since that decides which
// query-tile height and grid size keep the matrix cores busy.
static std::mutex g_tune_mu;
struct Shape {
  int32_t tq, tv, grid;
};
static std::map<std::string, Shape> g_tune;

static int log2_bucket(double v) { return v <= 1.0 ? 0 : (int)std::floor(std::log2(v)); }

static std::string tune_key(int32_t d_s, int32_t nprobe, double per_list) {
  char buf[96];
  snprintf(buf, sizeof(buf), "gfx950/ivf-fp32/ds%d/np%d/qpl%d", log2_bucket(d_s),
           log2_bucket(nprobe), log2_bucket(per_list));
  return buf;
}

}  // namespace adanns

using namespace adanns;

struct adanns_batch {
  std::vector<CfgDev> cfg;
  CfgDev *d_cfg = nullptr;
  void *scratch = nullptr;
  size_t scratch_bytes = 0;
  SearchBufs b{};
  int64_t ldq = 0, ldk = 0;
  int32_t tq = TILE_Q, tv = TILE_V, grid = PERSIST_WG;
  double per_list = 0;      // mean queries per probed list
  int32_t max_ds = 0, max_np = 0;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  const void *g_Q = nullptr, *g_dist = nullptr, *g_ids = nullptr;
  // graphs are captured and replayed on a private stream (the caller's may
  // be the legacy default stream, which cannot be captured), ordered after
  // and before the caller's work by events
  hipStream_t priv = nullptr;
  hipEvent_t ev_in = nullptr, ev_out = nullptr;
};

namespace adanns {

// Untuned scan shape: 64 x 128 tiles once a probed list meets a few dozen
// queries (the autotuner's usual pick there), else 32 x 64 (fewer padded
// query rows; at the ImageNet-1K shape with 8 to 2,048 queries it was within
// 5 % of the best shape at every size, where 64 x 64 was 5-10 % slower).
static void default_shape(double per_list, int32_t *tq, int32_t *tv) {
  if (per_list >= 32) {
    *tq = 64;
    *tv = 128;
  } else {
    *tq = 32;
    *tv = 64;
  }
}

void tuned_shape(const adanns_index *ix, int32_t d_s, int32_t nprobe, int64_t nq, int32_t *tq,
                 int32_t *tv, int32_t *grid) {
  const double per_list = (double)nq * nprobe / std::max(1, ix->nlist);
  default_shape(per_list, tq, tv);
  std::lock_guard<std::mutex> lk(g_tune_mu);
  auto it = g_tune.find(tune_key(d_s, nprobe, per_list));
  if (it != g_tune.end()) {
    *tq = it->second.tq;
    *tv = it->second.tv;
    *grid = it->second.grid;
  }
}

static void drop_graph(adanns_batch *p) {
  if (p->exec && p->priv) (void)hipStreamSynchronize(p->priv);  // no replay still in flight
  if (p->exec) (void)hipGraphExecDestroy(p->exec);
  if (p->graph) (void)hipGraphDestroy(p->graph);
  p->exec = nullptr;
  p->graph = nullptr;
}

}  // namespace adanns

extern "C" {

adanns_status adanns_batch_create(const adanns_batch_config *cfgs, int32_t ncfg, int64_t ldq,
                                  int64_t ldk, void *stream, adanns_batch **out) {
  clear_error();
  ADANNS_REQUIRE(out != nullptr && cfgs != nullptr, "cfgs and out must be non-NULL");
  ADANNS_REQUIRE(ncfg >= 1 && ncfg <= 4096, "ncfg must be in [1, 4096], got %d", ncfg);
  adanns_batch *p = new (std::nothrow) adanns_batch();
  if (!p) {
    set_error("out of host memory");
    return ADANNS_ENOMEM;
  }
  int64_t q0 = 0, S0 = 0, pair0 = 0, D = 0;
  int32_t vl0 = 0, ct0 = 0, dq = 1, kmax = 1;
  double probed = 0, lists = 0;
  int64_t max_items = 0;  // upper bound on the scan's work items
  for (int32_t c = 0; c < ncfg; ++c) {
    const adanns_batch_config &u = cfgs[c];
    const adanns_index *ix = u.index;
    auto bad = [&](const char *why) {
      set_error("config %d: %s", c, why);
      delete p;
      return ADANNS_EINVAL;
    };
    if (!ix) return bad("index is NULL");
    if (!ix->vec) return bad("index holds no FP32 vectors");
    if (u.nq < 0) return bad("nq < 0");
    if (u.d_c < 1 || u.d_c > ix->d_cb) return bad("d_c outside [1, d_c_build]");
    if (u.d_s < 1 || u.d_s > ix->d) return bad("d_s outside [1, d]");
    if (u.nprobe < 1 || u.nprobe > ix->nlist) return bad("nprobe outside [1, nlist]");
    if (u.k < 1 || u.k > MAX_SHORTLIST) return bad("k outside [1, 1024]");
    CfgDev g = make_cfg(ix, u.d_c, u.d_s, u.nprobe, u.k, u.nq);
    max_items += u.nq * u.nprobe * cdiv(std::max<int64_t>(ix->max_len, 1), 64);
    g.q0 = q0;
    g.S0 = S0;
    g.pair0 = pair0;
    g.vl0 = vl0;
    g.ct0 = ct0;
    p->cfg.push_back(g);
    q0 += u.nq;
    S0 += u.nq * ix->nlist;
    pair0 += u.nq * u.nprobe;
    vl0 += ix->nlist;
    ct0 += (int32_t)(g.qtiles * cdiv(ix->nlist, TILE_V));
    D += u.nq * ix->top_prefix[u.nprobe];
    dq = std::max(dq, std::max(u.d_c, u.d_s));
    kmax = std::max(kmax, u.k);
    p->max_ds = std::max(p->max_ds, u.d_s);
    p->max_np = std::max(p->max_np, u.nprobe);
    probed += (double)u.nq * u.nprobe;
    lists += ix->nlist;
  }
  if (pair0 >= (int64_t(1) << 31) || q0 >= (int64_t(1) << 31)) {
    set_error("the batch is too large (pairs or queries >= 2^31)");
    delete p;
    return ADANNS_EINVAL;
  }
  if (ldq < dq || ldk < kmax) {
    set_error("ldq (%lld) must be >= max(d_c, d_s) = %d and ldk (%lld) >= max k = %d",
              (long long)ldq, dq, (long long)ldk, kmax);
    delete p;
    return ADANNS_EINVAL;
  }
  p->ldq = ldq;
  p->ldk = ldk;
  p->per_list = probed / std::max(1.0, lists);
  const int32_t dq_pad = (int32_t)round_up(dq, SLAB);
  const int32_t V = vl0;
  // scratch carve, sizes first
  for (int pass = 0; pass < 2; ++pass) {
    Carver cv{(char *)p->scratch, 0, 0};
    SearchBufs b{};
    b.cfg = cv.take<CfgDev>(ncfg);
    b.ncfg = ncfg;
    b.V = V;
    b.ct_total = ct0;
    b.Qtot = q0;
    b.pairs = pair0;
    b.ldqs = dq_pad;
    b.max_nprobe = p->max_np;
    b.max_k = kmax;
    b.max_nlist = 1;
    for (const CfgDev &g : p->cfg) b.max_nlist = std::max(b.max_nlist, g.nlist);
    b.max_items = max_items;
    b.Qs = cv.take<float>((size_t)q0 * dq_pad);
    b.S = cv.take<float>((size_t)S0);
    b.probes = cv.take<int32_t>((size_t)pair0);
    b.cnt = cv.take<int32_t>(V);
    b.cursor = cv.take<int32_t>(V);
    b.work = cv.take<int32_t>(8);
    b.bkt_off = cv.take<int32_t>(V);
    b.tile_off = cv.take<int32_t>(V + 1);
    b.bucket = cv.take<int32_t>((size_t)pair0);
    b.seg_off = cv.take<int64_t>(q0 + 1);
    b.pair_base = cv.take<int64_t>((size_t)pair0);
    b.D = cv.take<float>((size_t)D);
    b.redo = cv.take<int32_t>((size_t)q0 + 2);
    if (pass == 0) {
      p->scratch_bytes = cv.off + 256;
      if (hipMalloc(&p->scratch, p->scratch_bytes) != hipSuccess) {
        (void)hipGetLastError();
        set_error("out of device memory for %zu bytes of batch scratch", p->scratch_bytes);
        delete p;
        return ADANNS_ENOMEM;
      }
    } else {
      p->b = b;
    }
  }
  p->d_cfg = p->b.cfg;
  if (hipMemcpyAsync(p->d_cfg, p->cfg.data(), ncfg * sizeof(CfgDev), hipMemcpyHostToDevice,
                     (hipStream_t)stream) != hipSuccess ||
      hipStreamSynchronize((hipStream_t)stream) != hipSuccess) {
    set_error("HIP error while uploading the batch descriptors");
    (void)hipFree(p->scratch);
    delete p;
    return ADANNS_EHIP;
  }
  default_shape(p->per_list, &p->tq, &p->tv);
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tune.find(tune_key(p->max_ds, p->max_np, p->per_list));
    if (it != g_tune.end()) {
      p->tq = it->second.tq;
      p->tv = it->second.tv;
      p->grid = it->second.grid;
    }
  }
  *out = p;
  return ADANNS_OK;
}

adanns_status adanns_batch_run(adanns_batch *p, const float *Q, float *dist, int64_t *ids,
                               int32_t *probes, void *stream) {
  clear_error();
  ADANNS_REQUIRE(p != nullptr, "batch is NULL");
  if (p->b.Qtot == 0) return ADANNS_OK;
  ADANNS_REQUIRE(Q && dist && ids, "Q, dist and ids must be non-NULL");
  ADANNS_HIP(launch_search_multi(p->b, Q, p->ldq, dist, ids, p->ldk, probes, p->tq, p->tv,
                                 p->grid, (hipStream_t)stream, true));
  return ADANNS_OK;
}

adanns_status adanns_batch_run_graph(adanns_batch *p, const float *Q, float *dist, int64_t *ids,
                                     void *stream) {
  clear_error();
  ADANNS_REQUIRE(p != nullptr, "batch is NULL");
  if (p->b.Qtot == 0) return ADANNS_OK;
  ADANNS_REQUIRE(Q && dist && ids, "Q, dist and ids must be non-NULL");
  ADANNS_REQUIRE(!timing_on(), "kernel timing must be off while a graph is captured");
  hipStream_t st = (hipStream_t)stream;
  if (!p->priv) {
    ADANNS_HIP(hipStreamCreateWithFlags(&p->priv, hipStreamNonBlocking));
    ADANNS_HIP(hipEventCreateWithFlags(&p->ev_in, hipEventDisableTiming));
    ADANNS_HIP(hipEventCreateWithFlags(&p->ev_out, hipEventDisableTiming));
  }
  if (!p->exec || p->g_Q != Q || p->g_dist != dist || p->g_ids != ids) {
    drop_graph(p);
    ADANNS_HIP(hipStreamBeginCapture(p->priv, hipStreamCaptureModeThreadLocal));
    hipError_t e = launch_search_multi(p->b, Q, p->ldq, dist, ids, p->ldk, nullptr, p->tq, p->tv,
                                       p->grid, p->priv, true);
    hipGraph_t g = nullptr;
    hipError_t e2 = hipStreamEndCapture(p->priv, &g);
    if (e != hipSuccess || e2 != hipSuccess) {
      if (g) (void)hipGraphDestroy(g);
      set_error("graph capture failed: %s", hipGetErrorString(e != hipSuccess ? e : e2));
      return ADANNS_EHIP;
    }
    p->graph = g;
    ADANNS_HIP(hipGraphInstantiate(&p->exec, p->graph, nullptr, nullptr, 0));
    p->g_Q = Q;
    p->g_dist = dist;
    p->g_ids = ids;
  }
  ADANNS_HIP(hipEventRecord(p->ev_in, st));
  ADANNS_HIP(hipStreamWaitEvent(p->priv, p->ev_in, 0));
  ADANNS_HIP(hipGraphLaunch(p->exec, p->priv));
  ADANNS_HIP(hipEventRecord(p->ev_out, p->priv));
  ADANNS_HIP(hipStreamWaitEvent(st, p->ev_out, 0));
  return ADANNS_OK;
}

adanns_status adanns_batch_set_shape(adanns_batch *p, int32_t tq, int32_t tv, int32_t grid) {
  clear_error();
  ADANNS_REQUIRE(p != nullptr, "batch is NULL");
  ADANNS_REQUIRE(tq == 32 || tq == 64 || tq == 128, "tq must be 32, 64 or 128, got %d", tq);
  ADANNS_REQUIRE(tv == 64 || tv == 128, "tv must be 64 or 128, got %d", tv);
  ADANNS_REQUIRE(grid >= 8 && grid <= 65536, "grid must be in [8, 65536], got %d", grid);
  grid = (int32_t)round_up(grid, 8);
  if (p->tq != tq || p->tv != tv || p->grid != grid) drop_graph(p);
  p->tq = tq;
  p->tv = tv;
  p->grid = grid;
  return ADANNS_OK;
}

adanns_status adanns_batch_autotune(adanns_batch *p, const float *Q, float *dist, int64_t *ids,
                                    int32_t reps, int32_t *tq_out, int32_t *tv_out,
                                    int32_t *grid_out, void *stream) {
  clear_error();
  ADANNS_REQUIRE(p != nullptr, "batch is NULL");
  ADANNS_REQUIRE(Q && dist && ids, "Q, dist and ids must be non-NULL");
  ADANNS_REQUIRE(reps >= 1 && reps <= 100, "reps must be in [1, 100]");
  hipStream_t st = (hipStream_t)stream;
  static const int32_t tqs[] = {32, 64, 128};
  static const int32_t tvs[] = {64, 128};
  static const int32_t grids[] = {1024, 2048, 4096};
  hipEvent_t e0, e1;
  ADANNS_HIP(hipEventCreate(&e0));
  ADANNS_HIP(hipEventCreate(&e1));
  float best = 1e30f;
  int32_t btq = p->tq, btv = p->tv, bgrid = p->grid;
  for (int32_t tq : tqs) {
    for (int32_t tv : tvs) {
      for (int32_t grid : grids) {
        // warm-up, then timed repetitions
        if (launch_search_multi(p->b, Q, p->ldq, dist, ids, p->ldk, nullptr, tq, tv, grid, st,
                                true) ||
            hipEventRecord(e0, st)) {
          (void)hipEventDestroy(e0);
          (void)hipEventDestroy(e1);
          set_error("launch failed during autotuning");
          return ADANNS_EHIP;
        }
        for (int32_t r = 0; r < reps; ++r)
          (void)launch_search_multi(p->b, Q, p->ldq, dist, ids, p->ldk, nullptr, tq, tv, grid, st,
                                    true);
        float ms = 0.f;
        if (hipEventRecord(e1, st) || hipEventSynchronize(e1) || hipEventElapsedTime(&ms, e0, e1)) {
          (void)hipEventDestroy(e0);
          (void)hipEventDestroy(e1);
          set_error("timing failed during autotuning");
          return ADANNS_EHIP;
        }
        if (ms < best) {
          best = ms;
          btq = tq;
          btv = tv;
          bgrid = grid;
        }
      }
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (p->tq != btq || p->tv != btv || p->grid != bgrid) drop_graph(p);
  p->tq = btq;
  p->tv = btv;
  p->grid = bgrid;
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune[tune_key(p->max_ds, p->max_np, p->per_list)] = {btq, btv, bgrid};
  }
  if (tq_out) *tq_out = btq;
  if (tv_out) *tv_out = btv;
  if (grid_out) *grid_out = bgrid;
  return ADANNS_OK;
}

adanns_status adanns_batch_info(const adanns_batch *p, int64_t *queries, int32_t *tq,
                                int32_t *tv, int32_t *grid, size_t *scratch_bytes) {
  clear_error();
  ADANNS_REQUIRE(p != nullptr, "batch is NULL");
  if (queries) *queries = p->b.Qtot;
  if (tq) *tq = p->tq;
  if (tv) *tv = p->tv;
  if (grid) *grid = p->grid;
  if (scratch_bytes) *scratch_bytes = p->scratch_bytes;
  return ADANNS_OK;
}

void adanns_batch_free(adanns_batch *p) {
  if (!p) return;
  (void)hipDeviceSynchronize();
  drop_graph(p);
  if (p->ev_in) (void)hipEventDestroy(p->ev_in);
  if (p->ev_out) (void)hipEventDestroy(p->ev_out);
  if (p->priv) (void)hipStreamDestroy(p->priv);
  if (p->scratch) (void)hipFree(p->scratch);
  delete p;
}

adanns_status adanns_autotune_clear(void) {
  clear_error();
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_tune.clear();
  return ADANNS_OK;
}

}  // extern "C"
