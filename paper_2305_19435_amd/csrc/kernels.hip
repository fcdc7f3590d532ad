// Device kernels of the AdANNS search paths for gfx950 (CDNA4) and their
// host-side launch wrappers.
//
//   k_stage_multi    query prefix staging (zero-padded, 16-byte aligned rows)
//   k_tile_multi     first-pass distances |x|^2 - 2 q.x on FP32 MFMA over a
//                    batch of configurations, persistent: the coarse step
//                    (all queries against the centroids) and the list scan
//                    (each list against the queries probing it; TQ x TV
//                    tiles, operands copied global -> LDS, per-XCD work
//                    counters)
//   k_select_wave / k_select_multi / k_select_refine(_wave)
//                    per query: the shortlist by first-pass value, exact
//                    re-measurement in compensated FP32, sort by (distance,
//                    id), top-k / top-nprobe out (one wave or one workgroup
//                    per query)
//   k_count / k_list_scan / k_scatter / k_seg_len / k_pair_base
//                    probe bucketing: (query, probe) pairs grouped per list,
//                    tile counts per list and the output segment of each pair
//   k_rotate / k_pq_lut / k_adc_scan
//                    IVF-PQ: query rotation (FP64 MFMA), distance tables,
//                    table-lookup scan with the tables in LDS
//   k_quant_* / k_tile_dist_q / k_tile_q_scan
//                    precision form: BF16 / e4m3 copies and their first pass
//                    on BF16 / FP8 MFMA (coarse, scan)
//
// The coarse step follows Algorithm 1's inference loop (distances to every
// centroid on the d_c prefix, then the nprobe nearest); the scan is its
// linear scan of the probed lists on the d_s prefix (Appendix A, Table
// "formula", AdANNS-IVF row).
#include "internal.h"

#include <algorithm>
#include <cstdio>
#include <mutex>
#include <type_traits>

namespace adanns {
namespace {

typedef float floatx4 __attribute__((ext_vector_type(4)));

// Loads through a pointer that the compiler cannot prove global (one read
// from a configuration record in memory, or chosen between LDS and global
// memory) become flat loads, which also hold the LDS wait counter: every
// LDS wait then waits for them too and prefetches stop overlapping. ldg
// reads such a pointer as global memory.
#define ADANNS_GLOBAL_AS __attribute__((address_space(1)))
template <class T>
__device__ __forceinline__ T ldg(const T *p) {
  return *(const T ADANNS_GLOBAL_AS *)p;
}
// float4 is a class type whose copy goes through a generic reference, so the
// 16-byte load is made on the native vector type.
__device__ __forceinline__ float4 ldg4(const float *p) {
  const floatx4 v = *(const floatx4 ADANNS_GLOBAL_AS *)p;
  return make_float4(v[0], v[1], v[2], v[3]);
}

// Monotone map from float to uint32 (total order, -0 < +0).
__device__ __forceinline__ uint32_t order_key(float f) {
  uint32_t u = __float_as_uint(f);
  return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}

// ---- compensated arithmetic for the exact re-measurement ---------------------
// Knuth's TwoSum: s + e == a + b exactly.
__device__ __forceinline__ void two_sum(float a, float b, float &s, float &e) {
#pragma clang fp contract(off)
  s = a + b;
  float bb = s - a;
  e = (a - (s - bb)) + (b - bb);
}

// Adds (q - x)^2 to the unevaluated sum S + C. q - x = d + de exactly
// (TwoSum), d*d = p + pe exactly (FMA), so only the tiny terms 2*d*de and
// de^2 (dropped, below u^2 of the term) and the rounding of C are inexact.
__device__ __forceinline__ void acc_sq_diff(float q, float x, float &S, float &C) {
#pragma clang fp contract(off)
  float d, de;
  two_sum(q, -x, d, de);
  float p = d * d;
  float pe = __builtin_fmaf(d, d, -p);
  float t, te;
  two_sum(S, p, t, te);
  S = t;
  C = C + (te + (pe + 2.0f * d * de));
}

__device__ __forceinline__ void wave_reduce_pair(float &S, float &C) {
#pragma clang fp contract(off)
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    float S2 = __shfl_xor(S, off);
    float C2 = __shfl_xor(C, off);
    float t, te;
    two_sum(S, S2, t, te);
    S = t;
    C = C + (C2 + te);
  }
  float hi, lo;
  two_sum(S, C, hi, lo);
  S = hi;
  C = lo;
}

// Exclusive prefix sum over the block (blockDim.x a multiple of 64).
template <class T>
__device__ __forceinline__ T block_excl_scan(T v, T *sh /* >= blockDim.x / 64 */, T *total) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
  T inc = v;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    T t = __shfl_up(inc, off);
    if (lane >= off) inc += t;
  }
  if (lane == 63) sh[wv] = inc;
  __syncthreads();
  T before = 0, all = 0;
  for (int w = 0; w < nw; ++w) {
    T s = sh[w];
    if (w < wv) before += s;
    all += s;
  }
  __syncthreads();
  if (total) *total = all;
  return before + inc - v;
}

// ---------------------------------------------------------------------------
__global__ void k_fill_i32(int32_t *p, int64_t n, int32_t v) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

__global__ void k_stage_queries(const float *__restrict__ Q, int64_t nq, int64_t ldq, int32_t dq,
                                float *__restrict__ Qs, int64_t ldqs) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t row = i / ldqs, col = i % ldqs;
  if (row >= nq) return;
  Qs[i] = col < dq ? Q[row * ldq + col] : 0.0f;
}

// Rows (optionally gathered through ``rows``) copied to a zero-padded buffer.
template <class T>
__global__ void k_stage_rows(const T *__restrict__ X, int64_t ldx, const int64_t *__restrict__ rows,
                             const int32_t *__restrict__ rows32, int64_t nrows, int32_t dcols,
                             float *__restrict__ out, int64_t ldo) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t r = i / ldo, c = i % ldo;
  if (r >= nrows) return;
  int64_t src = rows ? rows[r] : (rows32 ? (int64_t)rows32[r] : r);
  out[i] = c < dcols ? (float)X[src * ldx + c] : 0.0f;
}

// Lloyd update: centroid h becomes the mean of its members (perm[off[h] ..
// off[h+1]) rows of X), summed in a fixed order in compensated FP32; a
// centroid without members keeps its value.
__global__ __launch_bounds__(256) void k_centroid_update(const float *__restrict__ X, int64_t ldx,
                                                         const int32_t *__restrict__ perm,
                                                         const int64_t *__restrict__ off,
                                                         int32_t dcols, float *__restrict__ C,
                                                         int64_t ldc) {
#pragma clang fp contract(off)
  const int32_t h = blockIdx.x;
  const int32_t dim = blockIdx.y * blockDim.x + threadIdx.x;
  if (dim >= dcols) return;
  const int64_t a0 = off[h], a1 = off[h + 1];
  if (a1 == a0) return;
  float S = 0.f, E = 0.f;
  for (int64_t i = a0; i < a1; ++i) {
    float t, te;
    two_sum(S, X[(int64_t)perm[i] * ldx + dim], t, te);
    S = t;
    E = E + te;
  }
  float hi, lo;
  two_sum(S, E, hi, lo);
  const float cnt = (float)(a1 - a0);
  float m = hi / cnt;
  // one correction step: (hi + lo - m * cnt) / cnt
  float r = __builtin_fmaf(-m, cnt, hi) + lo;
  C[(int64_t)h * ldc + dim] = m + r / cnt;
}

// Slab layout writer: one thread per destination element.
template <class T>
__global__ void k_layout(const T *__restrict__ src, int64_t ldsrc, int32_t dsrc,
                         const int64_t *__restrict__ src_row, const int32_t *__restrict__ row_list,
                         const int64_t *__restrict__ poff, int64_t rows_pad, int32_t d_pad,
                         float *__restrict__ dst) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= rows_pad * d_pad) return;
  int64_t g = i / d_pad;
  int32_t dim = (int32_t)(i % d_pad);
  int32_t h = row_list[g];
  int64_t p0 = poff[h];
  int64_t npad = poff[h + 1] - p0;
  int64_t r = g - p0;
  int64_t sr = src_row[g];
  float v = (sr >= 0 && dim < dsrc) ? (float)src[sr * ldsrc + dim] : 0.0f;
  dst[p0 * d_pad + ((int64_t)(dim / SLAB) * npad + r) * SLAB + (dim % SLAB)] = v;
}

// ---- first-pass distance tiles ------------------------------------------------
// Finds the configuration whose prefix field ``off`` (a member pointer)
// covers value v: the largest c with cfg[c].*off <= v.
template <class T>
__device__ __forceinline__ int cfg_of(const CfgDev *cfg, int ncfg, T CfgDev::*off, int64_t v) {
  int lo = 0, hi = ncfg - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if ((int64_t)(cfg[mid].*off) <= v) lo = mid; else hi = mid - 1;
  }
  return lo;
}

struct TileArgs {
  const CfgDev *cfg;
  int32_t ncfg;
  const float *Qs;         // staged queries of the whole batch
  int64_t ldqs;
  int32_t V;               // virtual lists
  const int32_t *tile_off; // scan: [V + 1] tile prefix over virtual lists
  const int32_t *bkt_off;  // scan: start of each virtual list's bucket
  const int32_t *cnt;      // scan: pairs per virtual list
  const int32_t *bucket;   // scan: global pair ids grouped by virtual list
  const int64_t *pair_base;// scan: output offset of each pair
  float *S;                // coarse output
  float *D;                // scan output
  int32_t ct_total;        // coarse: tiles over configurations
  int32_t *work;           // scan: [8] work counters, zero at launch
};

__device__ __forceinline__ float f4(const float4 &v, int e) {
  return e == 0 ? v.x : e == 1 ? v.y : e == 2 ? v.z : v.w;
}

// One TV-vector tile of a list against TQ query rows:
// out[rbase[row] + v] = |x_v[:d]|^2 - 2 q_row[:d] . x_v[:d] for valid rows/vectors.
// rq[] holds the staged-query row of each tile row (-1 = none); the valid
// rows are the first nrow. This register-staged form serves the narrow
// tiles (TQ = 32): four waves in a 2 x 2 grid, each computing (TQ/2) x (TV/2)
// with 16x16x4 FP32 MFMA blocks; wider tiles use tile_compute_dma below.
template <int TQ, int TV>
__device__ __forceinline__ void tile_compute(const float *__restrict__ Qs, int64_t ldqs,
                                             const float *vp, int64_t npad, int nvec_left,
                                             int nrow, int d_dot, const int32_t *rq,
                                             const int64_t *rbase, float *__restrict__ out,
                                             float (*As)[SLAB + 4], float (*Bs)[SLAB + 4],
                                             float *cn) {
  constexpr int NA = TQ / 32;        // float4 of A per thread per slab
  constexpr int NBV = TV / 32;       // float4 of B per thread per slab
  constexpr int NB = TQ / 32;        // MFMA row blocks per wave
  constexpr int NC = TV / 32;        // MFMA column blocks per wave
  const int tid = threadIdx.x, lane = tid & 63;
  const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int rbw = (wv >> 1) * (TQ / 2), cbw = (wv & 1) * (TV / 2);
  const int ncol = nvec_left < TV ? nvec_left : TV;
  // a wave whose rows or vectors all lie past the valid ones skips its MFMAs
  const bool active = nrow > rbw && ncol > cbw;
  const int fr = lane & 15, fk = (lane >> 4) * 8;
  const int lr = tid >> 3, lc = (tid & 7) * 4;
  const int nslab = (d_dot + SLAB - 1) / SLAB;

  floatx4 acc[NB][NC];
#pragma unroll
  for (int i = 0; i < NB; ++i)
#pragma unroll
    for (int j = 0; j < NC; ++j) acc[i][j] = (floatx4){0.f, 0.f, 0.f, 0.f};
  float nrm[NBV];
#pragma unroll
  for (int u = 0; u < NBV; ++u) nrm[u] = 0.f;
  // Loads are unconditional so that they stay in flight across the MFMAs of
  // the previous slab: a row past the tile's valid queries reads staged row 0
  // and a vector past the list's length re-reads its last vector (the list's
  // padding ends at a multiple of ROWPAD, which a TV = 128 tile can overrun);
  // neither result is written out. Coordinates past d_dot are zeroed when
  // the query slab is staged into LDS.
  float4 ra[NA], rb[NBV];
  const float *qp[NA];
#pragma unroll
  for (int u = 0; u < NA; ++u) {
    const int q = rq[lr + 32 * u];
    qp[u] = Qs + (int64_t)(q >= 0 ? q : 0) * ldqs + lc;
  }
  int vrow[NBV];
#pragma unroll
  for (int u = 0; u < NBV; ++u) vrow[u] = min(lr + 32 * u, ncol - 1) * SLAB + lc;

  auto load = [&](int s) {
#pragma unroll
    for (int u = 0; u < NA; ++u) ra[u] = ldg4(qp[u] + s * SLAB);
    const float *src = vp + (int64_t)s * npad * SLAB;
#pragma unroll
    for (int u = 0; u < NBV; ++u) rb[u] = ldg4(src + vrow[u]);
  };

  // Registers -> LDS: slab s + 1 is in flight while slab s is multiplied.
  // (A second LDS stage, prefetching one slab further, measured slower.)
  auto stage = [&](int s) {
    const int dim = s * SLAB + lc;
#pragma unroll
    for (int u = 0; u < NA; ++u) {
      float4 v = ra[u];
      if (dim + 4 > d_dot) {
        if (dim + 0 >= d_dot) v.x = 0.f;
        if (dim + 1 >= d_dot) v.y = 0.f;
        if (dim + 2 >= d_dot) v.z = 0.f;
        if (dim + 3 >= d_dot) v.w = 0.f;
      }
      *(float4 *)&As[lr + 32 * u][lc] = v;
    }
#pragma unroll
    for (int u = 0; u < NBV; ++u) *(float4 *)&Bs[lr + 32 * u][lc] = rb[u];
    // vector norms over the same prefix, from the registers just stored
#pragma unroll
    for (int u = 0; u < NBV; ++u) {
      const float x[4] = {rb[u].x, rb[u].y, rb[u].z, rb[u].w};
#pragma unroll
      for (int e = 0; e < 4; ++e)
        if (dim + e < d_dot) nrm[u] += x[e] * x[e];
    }
  };

  load(0);
  for (int s = 0; s < nslab; ++s) {
    __syncthreads();
    stage(s);
    __syncthreads();
    if (s + 1 < nslab) load(s + 1);
    if (active) {
      // two halves of the slab: MFMA k-slot (lane >> 4) carries coordinate
      // 8 * (lane >> 4) + 4 * half + kb for both operands, so every
      // coordinate of the slab is used exactly once
#pragma unroll
      for (int half = 0; half < 2; ++half) {
        float4 af[NB], bf[NC];
#pragma unroll
        for (int i = 0; i < NB; ++i) af[i] = *(const float4 *)&As[rbw + i * 16 + fr][fk + 4 * half];
#pragma unroll
        for (int j = 0; j < NC; ++j) bf[j] = *(const float4 *)&Bs[cbw + j * 16 + fr][fk + 4 * half];
#pragma unroll
        for (int kb = 0; kb < 4; ++kb)
#pragma unroll
          for (int i = 0; i < NB; ++i)
#pragma unroll
            for (int j = 0; j < NC; ++j)
              acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(f4(af[i], kb), f4(bf[j], kb),
                                                               acc[i][j], 0, 0, 0);
      }
    }
  }
  // norms: 8 consecutive threads share a vector row
#pragma unroll
  for (int u = 0; u < NBV; ++u) {
    nrm[u] += __shfl_xor(nrm[u], 1);
    nrm[u] += __shfl_xor(nrm[u], 2);
    nrm[u] += __shfl_xor(nrm[u], 4);
    if ((tid & 7) == 0) cn[lr + 32 * u] = nrm[u];
  }
  __syncthreads();
  // 16x16 f32 MFMA result: lane holds column (lane & 15), rows 4*(lane>>4)+e
#pragma unroll
  for (int i = 0; i < NB; ++i)
#pragma unroll
    for (int j = 0; j < NC; ++j)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int row = rbw + i * 16 + (lane >> 4) * 4 + e;
        const int col = cbw + j * 16 + (lane & 15);
        if (rq[row] >= 0 && col < nvec_left) out[rbase[row] + col] = cn[col] - 2.0f * acc[i][j][e];
      }
}

// LDS-DMA form of the tile for TQ, TV >= 64. Every lane copies 16-byte
// chunks from global memory straight into LDS (global_load_lds_dwordx4); two
// LDS stages alternate, so one barrier per slab remains and no registers
// carry the next slab. A stage holds each operand row as 32 floats without
// padding; 16-byte chunk c of row r sits at position c ^ f(r), with
// f(r) = (r & 7) ^ ((r >> 3) & 1), which spreads the 16-byte reads of 8 or 16
// consecutive rows over all LDS banks. Four waves in a 2 x 2 grid compute
// (TQ/2) x (TV/2) each with 16x16x4 FP32 MFMA blocks. Vector norms are summed
// from the B fragments the MFMAs read.
__device__ __forceinline__ int swz(int r) { return (r & 7) ^ ((r >> 3) & 1); }
// s_waitcnt immediate for vmcnt(n) with the other counters left free
constexpr int vm_wait_imm(int n) { return 0x0F70 | (n & 15) | ((n >> 4) << 14); }
template <int I> using ic = std::integral_constant<int, I>;

template <int TQ, int TV>
__device__ __forceinline__ void tile_compute_dma(const float *__restrict__ Qs, int64_t ldqs,
                                                 const float *vp, int64_t npad, int nvec_left,
                                                 int nrow, int d_dot, const int32_t *rq,
                                                 const int64_t *rbase, float *__restrict__ out,
                                                 float *A0, float *B0, float *A1, float *B1,
                                                 float *cn) {
  static_assert(TQ >= 64 && TV >= 64, "LDS-DMA tile needs TQ, TV >= 64");
  constexpr int NA = TQ / 32;   // 16-byte copies of A per lane per slab
  constexpr int NBV = TV / 32;  // 16-byte copies of B per lane per slab
  constexpr int NB16 = TQ / 32, NC16 = TV / 32;  // 16x16 blocks per wave
  const int tid = threadIdx.x, lane = tid & 63;
  const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int rbw = (wv >> 1) * (TQ / 2), cbw = (wv & 1) * (TV / 2);
  const int ncol = nvec_left < TV ? nvec_left : TV;
  // a wave whose rows or vectors all lie past the valid ones skips its MFMAs
  const bool active = nrow > rbw && ncol > cbw;
  const int nslab = (d_dot + SLAB - 1) / SLAB;

  // Copy side: wave instruction u fills rows (4u + wv) * 8 .. + 7, lane l
  // writing LDS chunk (l & 7) of row (l >> 3) of that block. Copies are
  // unconditional: a row past the tile's valid queries reads staged row 0 and
  // a vector past the list's length re-reads its last vector; neither result
  // is written out.
  const int lrow = lane >> 3;
  const int gch = (lane & 7) ^ lrow ^ (wv & 1);  // global chunk: (l & 7) ^ f(row)
  const float *qp[NA];
#pragma unroll
  for (int u = 0; u < NA; ++u) {
    const int q = rq[(4 * u + wv) * 8 + lrow];
    qp[u] = Qs + (int64_t)(q >= 0 ? q : 0) * ldqs + gch * 4;
  }
  int vrow[NBV];
#pragma unroll
  for (int u = 0; u < NBV; ++u) vrow[u] = min((4 * u + wv) * 8 + lrow, ncol - 1) * SLAB + gch * 4;
  auto issue = [&](int s, float *A, float *B) {
#pragma unroll
    for (int u = 0; u < NA; ++u)
      __builtin_amdgcn_global_load_lds(
          (const void *)(qp[u] + s * SLAB),
          (__attribute__((address_space(3))) void *)(A + (4 * u + wv) * 8 * SLAB), 16, 0, 0);
    const float *src = vp + (int64_t)s * npad * SLAB;
#pragma unroll
    for (int u = 0; u < NBV; ++u)
      __builtin_amdgcn_global_load_lds(
          (const void *)(src + vrow[u]),
          (__attribute__((address_space(3))) void *)(B + (4 * u + wv) * 8 * SLAB), 16, 0, 0);
  };
  // The last slab of a prefix that ends inside it: every lane zeroes, in the
  // stage just filled, the coordinates past the prefix of the chunks it
  // copied (both operands, so that values past the prefix never meet), then
  // the workgroup synchronises again.
  auto clip = [&](float *A, float *B, int lim) {
    const int c = (lane & 7) * 4;  // LDS position of this lane's chunks
#pragma unroll
    for (int e = 0; e < 4; ++e)
      if (gch * 4 + e >= lim) {
#pragma unroll
        for (int u = 0; u < NA; ++u) A[((4 * u + wv) * 8 + lrow) * SLAB + c + e] = 0.f;
#pragma unroll
        for (int u = 0; u < NBV; ++u) B[((4 * u + wv) * 8 + lrow) * SLAB + c + e] = 0.f;
      }
    __syncthreads();
  };

  floatx4 acc[NB16][NC16];
#pragma unroll
  for (int i = 0; i < NB16; ++i)
#pragma unroll
    for (int j = 0; j < NC16; ++j) acc[i][j] = (floatx4){0.f, 0.f, 0.f, 0.f};
  float nrm[NC16];
#pragma unroll
  for (int j = 0; j < NC16; ++j) nrm[j] = 0.f;
  // Read side: in half h of a slab, lane l reads row (l & 15) of each
  // 16-row block, global chunk 2 (l >> 4) + h; MFMA k-slot (l >> 4) at step t
  // then carries coordinate 8 (l >> 4) + 4 h + t for both operands.
  const int r16 = lane & 15, g16 = lane >> 4;
  const int sw16 = swz(r16);
  auto compute = [&](const float *A, const float *B) {
    float4 af[2][NB16], bf[2][NC16];
    auto fetch = [&](int h) {
      const int off = (((2 * g16 + h) ^ sw16) << 2);
#pragma unroll
      for (int i = 0; i < NB16; ++i) af[h][i] = *(const float4 *)&A[(rbw + i * 16 + r16) * SLAB + off];
#pragma unroll
      for (int j = 0; j < NC16; ++j) bf[h][j] = *(const float4 *)&B[(cbw + j * 16 + r16) * SLAB + off];
    };
    fetch(0);
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      if (h == 0) fetch(1);
#pragma unroll
      for (int j = 0; j < NC16; ++j)
        nrm[j] += bf[h][j].x * bf[h][j].x + bf[h][j].y * bf[h][j].y + bf[h][j].z * bf[h][j].z +
                  bf[h][j].w * bf[h][j].w;
#pragma unroll
      for (int kb = 0; kb < 4; ++kb)
#pragma unroll
        for (int i = 0; i < NB16; ++i)
#pragma unroll
          for (int j = 0; j < NC16; ++j)
            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(f4(af[h][i], kb), f4(bf[h][j], kb),
                                                             acc[i][j], 0, 0, 0);
    }
    // Schedule: the first half's reads, then the second half's reads spread
    // over the first half's MFMAs (six MFMAs after each), then the remaining
    // MFMAs, the norms last.
    constexpr int NR = NB16 + NC16, NM = NB16 * NC16 * 4, SPREAD = NM / NR < 6 ? NM / NR : 6;
    __builtin_amdgcn_sched_group_barrier(0x100, NR, 0);
#pragma unroll
    for (int t = 0; t < NR; ++t) {
      __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);
      __builtin_amdgcn_sched_group_barrier(0x008, SPREAD, 0);
    }
    __builtin_amdgcn_sched_group_barrier(0x008, 2 * NM - NR * SPREAD, 0);
    __builtin_amdgcn_sched_group_barrier(0x002, 64, 0);
  };

  // Stage J holds slab s; the copy of slab s + 1 is in flight meanwhile.
  __builtin_amdgcn_s_waitcnt(vm_wait_imm(0));  // the previous item's stores first
  issue(0, A0, B0);
  int s = 0;
  auto step = [&](auto J) -> bool {
    constexpr int j = decltype(J)::value;
    float *A = j == 0 ? A0 : A1, *B = j == 0 ? B0 : B1;
    __builtin_amdgcn_s_waitcnt(vm_wait_imm(0));  // this wave's copies of slab s have landed
    __syncthreads();  // slab s is in stage j; every wave is done with stage 1 - j
    if (s + 1 < nslab) issue(s + 1, j == 0 ? A1 : A0, j == 0 ? B1 : B0);
    if (d_dot - s * SLAB < SLAB) clip(A, B, d_dot - s * SLAB);
    if (active) compute(A, B);
    return ++s >= nslab;
  };
  for (;;) {
    if (step(ic<0>{})) break;
    if (step(ic<1>{})) break;
  }
  // norms: the four lane groups of a column hold its four coordinate ranges;
  // waves 0 and 1 cover every column (wave 0 is always active, wave 1
  // whenever its columns hold vectors)
#pragma unroll
  for (int j = 0; j < NC16; ++j) {
    nrm[j] += __shfl_xor(nrm[j], 16);
    nrm[j] += __shfl_xor(nrm[j], 32);
    if (wv < 2 && active && lane < 16) cn[cbw + j * 16 + lane] = nrm[j];
  }
  __syncthreads();
  // 16x16 f32 MFMA result: lane holds column (lane & 15), rows 4 (lane >> 4) + e
#pragma unroll
  for (int i = 0; i < NB16; ++i)
#pragma unroll
    for (int j = 0; j < NC16; ++j)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int row = rbw + i * 16 + 4 * (lane >> 4) + e;
        const int col = cbw + j * 16 + (lane & 15);
        if (rq[row] >= 0 && col < nvec_left) out[rbase[row] + col] = cn[col] - 2.0f * acc[i][j][e];
      }
}

// Persistent tile kernel over a batch (two workgroups per CU: the register
// budget is held to 256 per lane). COARSE: every configuration's queries
// against its centroids (tiles numbered per configuration); otherwise every
// virtual list against the queries probing it.
constexpr int SCAN_CHUNK = 64;  // consecutive scan items an XCD takes in a row

template <int TQ, int TV, int COARSE>
__global__ __launch_bounds__(256, 2) void k_tile_multi(TileArgs a) {
  constexpr bool DMA = TQ >= 64 && TV >= 64;
  // two unpadded stages for the LDS-DMA tile, one padded stage otherwise
  __shared__ __attribute__((aligned(16))) float As[DMA ? TQ * SLAB : TQ * (SLAB + 4)];
  __shared__ __attribute__((aligned(16))) float Bs[DMA ? TV * SLAB : TV * (SLAB + 4)];
  __shared__ __attribute__((aligned(16))) float As1[DMA ? TQ * SLAB : 4];
  __shared__ __attribute__((aligned(16))) float Bs1[DMA ? TV * SLAB : 4];
  __shared__ int64_t rbase[TQ];
  __shared__ int32_t rq[TQ];
  __shared__ float cn[TV];
  const int tid = threadIdx.x;
  const int total = COARSE ? a.ct_total : a.tile_off[a.V];
  const int G = gridDim.x;
  // XCD-aware order: workgroup b runs on XCD b % 8. Coarse: each XCD gets a
  // contiguous run of work items. Scan: the items (lists in order, query
  // tile fastest) are dealt to the XCDs in chunks of SCAN_CHUNK consecutive
  // items, chunk c to XCD c % 8, and an XCD's workgroups take its items one
  // at a time from the XCD's counter. The items in flight on one XCD thus
  // stay a window of consecutive items however unevenly they last (the query
  // and vector tiles they share meet in that XCD's L2), and regions of the
  // item order that cost more (longer prefixes, longer lists) are spread
  // over every XCD.
  const int xcd = blockIdx.x & 7;
  __shared__ int s_item;
  for (int w = COARSE ? xcd * (G >> 3) + (blockIdx.x >> 3) : 0;; w += G) {
    if (!COARSE) {
      __syncthreads();  // every thread has read the previous s_item
      if (tid == 0) {
        const int k = atomicAdd(&a.work[xcd], 1);
        s_item = ((k / SCAN_CHUNK) * 8 + xcd) * SCAN_CHUNK + k % SCAN_CHUNK;
      }
      __syncthreads();
      w = s_item;
    }
    if (w >= total) break;
    int c, qt, vt, m, nvec, d_dot;
    int64_t npad;
    const float *vbase;
    int h = 0, v = 0;
    if (COARSE) {
      c = cfg_of(a.cfg, a.ncfg, &CfgDev::ct0, w);
      const CfgDev &g = a.cfg[c];
      const int local = w - g.ct0;
      qt = local % g.qtiles;
      vt = local / g.qtiles;
      m = (int)g.nq;
      nvec = g.nlist;
      npad = g.nl_pad;
      vbase = g.cent_slab;
      d_dot = g.d_c;
    } else {
      int lo = 0, hi = a.V - 1;
      while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (a.tile_off[mid] <= w) lo = mid; else hi = mid - 1;
      }
      v = lo;
      c = cfg_of(a.cfg, a.ncfg, &CfgDev::vl0, v);
      const CfgDev &g = a.cfg[c];
      h = v - g.vl0;
      m = a.cnt[v];
      nvec = ldg(g.len + h);
      const int64_t p0 = ldg(g.poff + h);
      npad = ldg(g.poff + h + 1) - p0;
      const int qts = (m + TQ - 1) / TQ;
      const int rem = w - a.tile_off[v];
      qt = rem % qts;
      vt = rem / qts;
      vbase = g.vec + p0 * g.d_pad;
      d_dot = g.d_s;
    }
    __syncthreads();  // previous item's epilogue is done with rq / rbase / cn
    if (tid < TQ) {
      const CfgDev &g = a.cfg[c];
      const int i = qt * TQ + tid;
      if (i < m) {
        if (COARSE) {
          rq[tid] = (int32_t)(g.q0 + i);
          rbase[tid] = g.S0 + (int64_t)i * g.nlist;
        } else {
          const int32_t pair = a.bucket[a.bkt_off[v] + i];
          rq[tid] = (int32_t)(g.q0 + (pair - g.pair0) / g.nprobe);
          rbase[tid] = a.pair_base[pair];
        }
      } else {
        rq[tid] = -1;
        rbase[tid] = 0;
      }
    }
    __syncthreads();
    if constexpr (DMA)
      tile_compute_dma<TQ, TV>(a.Qs, a.ldqs, vbase + (int64_t)vt * TV * SLAB, npad,
                               nvec - vt * TV, min(TQ, m - qt * TQ), d_dot, rq, rbase,
                               (COARSE ? a.S : a.D) + (int64_t)vt * TV, As, Bs, As1, Bs1, cn);
    else
      tile_compute<TQ, TV>(a.Qs, a.ldqs, vbase + (int64_t)vt * TV * SLAB, npad, nvec - vt * TV,
                           min(TQ, m - qt * TQ), d_dot, rq, rbase,
                           (COARSE ? a.S : a.D) + (int64_t)vt * TV,
                           (float(*)[SLAB + 4])As, (float(*)[SLAB + 4])Bs, cn);
  }
}

// ---- per-query selection and exact re-measurement ----------------------------
// Candidate measures used after the first-pass selection. Each returns the
// exact value of a distance the method defines, as an unevaluated FP32 pair.
enum SelMode : int32_t {
  SEL_COARSE = 0,        // centroid distance on d_c, FP32 centroids
  SEL_L2 = 1,            // vector distance on d_s, FP32 slab layout
  SEL_ADC = 2,           // asymmetric PQ distance (rotated query vs codebooks)
  SEL_QUANT = 3,         // distance between quantised query and quantised vector
  SEL_COARSE_QUANT = 4,  // distance between quantised query and quantised centroid
};

struct SelArgs {
  int32_t mode;
  const float *D;
  const int64_t *seg_off;  // scan modes: [nq + 1]
  int32_t nl;              // coarse modes: scores per query
  int32_t K1;              // first-pass shortlist length
  int32_t K2;              // kept after the first exact measure
  int32_t kout;            // results per query
  int32_t stageB;          // re-measure the K2 kept with exact FP32 L2, keep kout
  const float *Qs;
  int64_t ldqs;
  int32_t d_dot;           // coordinates of the first measure
  int32_t d_B;             // coordinates of the second measure
  const float *cent;       // coarse: [nl][ld_cent]
  int32_t ld_cent;
  const float *vec;        // scan: slab layout
  const float *rows;       // scan: row-major copy of vec, or NULL
  int32_t d_pad;
  const int64_t *poff;
  const int64_t *rowid;
  const int32_t *probes;   // scan: [nq][nprobe]
  int32_t nprobe;
  const int64_t *pair_base;
  // ADC
  const uint8_t *codes;    // [rows_pad][M]
  int32_t M, dsub;
  const float *cb;         // [M][256][dsub]
  const float *qr_hi, *qr_lo;  // rotated queries as pairs, [nq][ldqr]
  int64_t ldqr;
  // quantised operands (precision form)
  int32_t qfmt;            // 1 = bf16, 2 = fp8 e4m3
  const void *qvec;        // slab layout of the quantised vectors (or centroids)
  const float *qscale;     // per layout row (fp8)
  int32_t qd_pad;          // padded width of the quantised layout
  const void *qQ;          // quantised queries [nq][ldqq]
  const float *qQscale;    // per query (fp8)
  int64_t ldqq;
  const float *qemax;      // largest |x - dequantised x| of the stored rows, or NULL
                           // (enables the FP32 re-rank's quantisation bound)
  const float *qrerr;      // |x - dequantised x| of each stored row (layout order), or NULL
  const float *qerr;       // the same, for the first pass's rounding bound, or NULL
  const float *xmax2;      // largest squared FP32 row norm (with qerr), or NULL
  int64_t qnpad;           // coarse-quant: rows of the one-list layout
  float *out_dist;
  int64_t *out_ids;
  int32_t *out_probes;
  int32_t *out_probes2;
  int64_t ldo;             // output row stride (0 = kout)
  int32_t lcap;            // segment floats staged in LDS (0 = none)
  int32_t kcap;            // candidate slots in LDS (power of two >= K1)
  // Queries whose shortlist cannot be certified here are appended to
  // redo_list (count in *redo_cnt) and left for the re-selection launch; NULL
  // in that launch itself.
  int32_t *redo_cnt;
  int32_t *redo_list;
  int64_t redo_q0;         // added to a query's index in redo_list
  // k_select_filtered_wave: > 0 also certifies that every result lies in the
  // shortlist of this many nearest candidates by exact quantised distance
  int32_t shortlist;
};

// Process-wide selection counters (per device): [0] queries handed to the
// re-selection launch, [1] queries whose band of possible nearest candidates
// held more than the largest shortlist (result not certified exact); exact
// search with a quantised first pass: [2] candidates measured exactly, [3]
// queries that needed more than one window of candidates.
__device__ unsigned long long g_sel_stats[4];

// Bound on |first-pass value - exact value| of a candidate, as a function of
// the first-pass value f. kind 0: none known; 1: a constant B; 2: IVF-PQ's
// B(f) = c1 f + c2 (2 sqrt(f) + 2^-24 |q'|) (see wave_fp_bound). Both grow
// with f no faster than f, so f - B(f) is non-decreasing and a candidate that
// can still reach the kv nearest is one with f - B(f) <= v_kv + B(v_kv),
// v_kv the kv-th smallest first-pass value: every other one is farther than
// kv candidates in exact arithmetic.
struct FpBound {
  int32_t kind;
  float B, c1, c2, qn;
  float eq;  // quantised modes: |q - q^| over the first measure's prefix, else -1
  float qq;  // quantised modes: |q^|^2 over that prefix (FP32; the first pass omits it)
  __device__ float of(float f) const {
    if (kind == 1) return B;
    f = fmaxf(f, 0.f);
    return c1 * f + c2 * (2.f * sqrtf(f) + 0x1p-24f * qn);
  }
  __device__ float upper(float v) const { return v + of(v); }
  __device__ bool keep(float f, float up) const { return f - of(f) <= up; }
};

// First-pass value of a (order_key << 32 | position) composite.
__device__ __forceinline__ float comp_value(uint64_t comp) {
  const uint32_t kk = (uint32_t)(comp >> 32);
  return __uint_as_float((kk & 0x80000000u) ? (kk & 0x7FFFFFFFu) : ~kk);
}

__device__ __forceinline__ int64_t min64(int64_t a, int64_t b) { return a < b ? a : b; }

__device__ __forceinline__ bool pair_less(float ah, float al, int64_t ai, float bh, float bl,
                                          int64_t bi) {
  if (ah != bh) return ah < bh;
  if (al != bl) return al < bl;
  return ai < bi;
}

// Adds ((qh + ql) - x)^2 for a query coordinate given as a pair.
__device__ __forceinline__ void acc_sq_diff2(float qh, float ql, float x, float &S, float &C) {
#pragma clang fp contract(off)
  float d, de;
  two_sum(qh, -x, d, de);
  de = de + ql;
  float p = d * d;
  float pe = __builtin_fmaf(d, d, -p);
  float t, te;
  two_sum(S, p, t, te);
  S = t;
  C = C + (te + (pe + 2.0f * d * de));
}

// Exact product a*b as a pair.
__device__ __forceinline__ void two_prod(float a, float b, float &p, float &e) {
#pragma clang fp contract(off)
  p = a * b;
  e = __builtin_fmaf(a, b, -p);
}

// Value of an OCP e4m3 byte (finite codes only; 0x7F/0xFF never stored).
__device__ __forceinline__ float e4m3_to_float(uint32_t c) {
  const uint32_t s = c & 0x80u, e = (c >> 3) & 0xFu, f = c & 7u;
  float v = e == 0 ? (float)f * 0.001953125f
                   : __uint_as_float(((e + 120u) << 23) | (f << 20));
  return s ? -v : v;
}

__device__ __forceinline__ float bf16_to_float(uint16_t b) {
  return __uint_as_float((uint32_t)b << 16);
}

// Quantised value (as an exact pair) of coordinate ``i`` of a quantised row.
template <class P>
__device__ __forceinline__ void quant_value(int32_t fmt, P base, int64_t idx, float scale,
                                            float &hi, float &lo) {
  if (fmt == 1) {
    hi = bf16_to_float(ldg((const uint16_t *)base + idx));
    lo = 0.f;
  } else {
    two_prod(scale, e4m3_to_float(ldg((const uint8_t *)base + idx)), hi, lo);
  }
}
// The staged quantised query row in LDS.
__device__ __forceinline__ void quant_value(int32_t fmt, const uint8_t *lds, int64_t idx,
                                            float scale, float &hi, float &lo, bool) {
  if (fmt == 1) {
    hi = bf16_to_float(((const uint16_t *)lds)[idx]);
    lo = 0.f;
  } else {
    two_prod(scale, e4m3_to_float(lds[idx]), hi, lo);
  }
}

__device__ __forceinline__ void bitonic_sort(float *chi, float *clo, int64_t *cid, int64_t *cg,
                                             int P2) {
  const int tid = threadIdx.x;
  for (int size = 2; size <= P2; size <<= 1) {
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      __syncthreads();
      for (int t = tid; t < (P2 >> 1); t += blockDim.x) {
        const int i = 2 * t - (t & (stride - 1));
        const int j = i + stride;
        const bool up = (i & size) == 0;
        const bool gt = pair_less(chi[j], clo[j], cid[j], chi[i], clo[i], cid[i]);
        if (gt == up) {
          float th = chi[i]; chi[i] = chi[j]; chi[j] = th;
          float tl = clo[i]; clo[i] = clo[j]; clo[j] = tl;
          int64_t ti = cid[i]; cid[i] = cid[j]; cid[j] = ti;
          int64_t tg = cg[i]; cg[i] = cg[j]; cg[j] = tg;
        }
      }
    }
  }
  __syncthreads();
}

// Dynamic LDS of the selection kernels: histogram (reused for the staged
// query row), the query's first-pass segment when it fits (lcap floats), and
// the candidate arrays (kcap entries).
__host__ __device__ inline size_t sel_smem_bytes(int32_t lcap, int32_t kcap) {
  return 2048 * 4 + 4096 + (size_t)lcap * 4 + (size_t)kcap * (8 + 4 + 4 + 8 + 8);
}

// Where a candidate lives. Coarse modes: a centroid (id = gpack = row = h).
// Scan modes: row r of list h, at layout row p0 + r.
struct CandLoc {
  int64_t id, gpack, row, p0, npad;
};

__device__ __forceinline__ CandLoc locate(const SelArgs &a, bool coarse, int64_t q, int64_t seg0,
                                          int64_t pos) {
  CandLoc L{pos, pos, pos, 0, 0};
  if (coarse) return L;
  const int64_t pabs = seg0 + pos;
  const int64_t *pb = a.pair_base + q * a.nprobe;
  int lo = 0, hi = a.nprobe - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (ldg(pb + mid) <= pabs) lo = mid; else hi = mid - 1;
  }
  const int32_t h = ldg(a.probes + q * a.nprobe + lo);
  const int64_t r = pabs - ldg(pb + lo);
  L.p0 = ldg(a.poff + h);
  L.npad = ldg(a.poff + h + 1) - L.p0;
  L.id = ldg(a.rowid + L.p0 + r);
  L.gpack = ((int64_t)h << 32) | r;
  L.row = L.p0 + r;
  return L;
}

__device__ __forceinline__ CandLoc locate_packed(const SelArgs &a, bool coarse, int64_t gpack) {
  CandLoc L{0, gpack, gpack, 0, 0};
  if (coarse) return L;
  const int32_t h = (int32_t)(gpack >> 32);
  L.p0 = ldg(a.poff + h);
  L.npad = ldg(a.poff + h + 1) - L.p0;
  L.row = L.p0 + (gpack & 0xffffffffll);
  return L;
}

// First exact measure of one candidate over the lanes of a wave: the value
// the method ranks by (SelMode), as the unevaluated pair S + C. ``qrow`` is
// the FP32 query row (LDS or global); ``qq_lds`` the staged quantised query
// row in LDS, or NULL to read it from global memory. Each lane accumulates
// its coordinates lane, lane + 64, ... in increasing order; loads are
// issued in batches so that several are in flight.
// Exact distance between the quantised query and G quantised stored rows
// (SEL_QUANT), the rows' loads in flight together: lane l takes 16-byte
// chunks l, l + 64, ... of each row inside its slabs, QB chunks per row
// loaded before any is used; each row accumulates its coordinates in the
// same order as with G = 1, so the results do not depend on G.
template <int G>
__device__ __forceinline__ void measure_quant_rows(const SelArgs &a, int64_t q, const CandLoc *L,
                                                   const uint8_t *qq_lds, int lane, float *S,
                                                   float *C) {
  const int d = a.d_dot;
  const float qs = a.qfmt == 2 ? ldg(a.qQscale + q) : 1.f;
  const int qeb = a.qfmt == 1 ? 2 : 1;
  const int per = 16 / qeb;
  float xs[G];
  const uint8_t *vb[G];
#pragma unroll
  for (int g = 0; g < G; ++g) {
    xs[g] = a.qfmt == 2 ? ldg(a.qscale + L[g].row) : 1.f;
    vb[g] = (const uint8_t *)a.qvec + (L[g].p0 * a.qd_pad + (L[g].row - L[g].p0) * SLAB) * qeb;
  }
  typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
  constexpr int QB = 4;
  for (int e00 = lane * per; e00 < d; e00 += 64 * per * QB) {
    u32x4 w4s[G][QB], q4s[QB];
#pragma unroll
    for (int b = 0; b < QB; ++b) {
      const int e0 = e00 + 64 * per * b;
      if (e0 < d) {
#pragma unroll
        for (int g = 0; g < G; ++g)
          w4s[g][b] = ldg((const u32x4 *)(vb[g] + ((int64_t)(e0 / SLAB) * L[g].npad * SLAB +
                                                   e0 % SLAB) * qeb));
        // the query's bytes at the same coordinates (rows are 16-byte aligned)
        q4s[b] = qq_lds ? *(const u32x4 *)(qq_lds + (int64_t)e0 * qeb)
                        : ldg((const u32x4 *)((const uint8_t *)a.qQ + (q * a.ldqq + e0) * qeb));
      }
    }
#pragma unroll
    for (int b = 0; b < QB; ++b) {
      const int e0 = e00 + 64 * per * b;
      if (e0 >= d) break;
      const u32x4 q4 = q4s[b];
      const uint32_t qds[4] = {q4[0], q4[1], q4[2], q4[3]};
      const uint32_t msk = qeb == 2 ? 0xffffu : 0xffu;
#pragma unroll
      for (int g = 0; g < G; ++g) {
        const u32x4 w4 = w4s[g][b];
        const uint32_t wds[4] = {w4[0], w4[1], w4[2], w4[3]};
        for (int u = 0; u < per && e0 + u < d; ++u) {
          const int sh = ((u * qeb) % 4) * 8;
          const uint32_t bits = (wds[(u * qeb) / 4] >> sh) & msk;
          const uint32_t qbits = (qds[(u * qeb) / 4] >> sh) & msk;
          float qh, ql, xh, xl;
          if (a.qfmt == 1) {
            qh = bf16_to_float((uint16_t)qbits);
            ql = 0.f;
            xh = bf16_to_float((uint16_t)bits);
            xl = 0.f;
          } else {
            two_prod(qs, e4m3_to_float(qbits), qh, ql);
            two_prod(xs[g], e4m3_to_float(bits), xh, xl);
          }
          acc_sq_diff2(qh, ql - xl, xh, S[g], C[g]);
        }
      }
    }
  }
}

template <class QP>
__device__ __forceinline__ void measure1(const SelArgs &a, int64_t q, const CandLoc &L, QP qrow,
                                         const uint8_t *qq_lds, int lane, float &S, float &C) {
  const int d = a.d_dot;
  if (a.mode == SEL_COARSE) {
    const float *x = a.cent + L.row * a.ld_cent;
    for (int d0 = lane; d0 < d; d0 += 64 * 8) {
      float xv[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) xv[u] = d0 + 64 * u < d ? ldg(x + d0 + 64 * u) : 0.f;
#pragma unroll
      for (int u = 0; u < 8; ++u)
        if (d0 + 64 * u < d) acc_sq_diff(qrow[d0 + 64 * u], xv[u], S, C);
    }
  } else if (a.mode == SEL_L2) {
    // lane l takes coordinates 4l + 256u + e (u = 0, 1, ..., e = 0..3) in
    // that order, read as 16-byte pieces: in the slab layout coordinate dim
    // of the row sits at (dim / SLAB) * npad * SLAB + dim % SLAB, in the
    // row-major copy at dim (npad = 1). k_select_wave accumulates in the
    // same order, so both give the same bits.
    const float *base = a.rows ? a.rows + L.row * a.d_pad
                               : a.vec + L.p0 * a.d_pad + (L.row - L.p0) * SLAB;
    const int64_t np = a.rows ? 1 : L.npad;
    for (int d0 = 4 * lane; d0 < d; d0 += 256 * 4) {
      float4 xv[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int dim = d0 + 256 * u;
        xv[u] = dim < d ? ldg4(base + (int64_t)(dim / SLAB) * np * SLAB + dim % SLAB)
                        : make_float4(0.f, 0.f, 0.f, 0.f);
      }
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int dim = d0 + 256 * u + e;
          if (dim < d) acc_sq_diff(qrow[dim], f4(xv[u], e), S, C);
        }
    }
  } else if (a.mode == SEL_ADC) {
    const uint8_t *code = a.codes + L.row * a.M;
    const float *qh = a.qr_hi + q * a.ldqr, *ql = a.qr_lo + q * a.ldqr;
    for (int d0 = lane; d0 < d; d0 += 64 * 8) {
      uint32_t cm[8];
      float x[8], h8[8], l8[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int dim = d0 + 64 * u;
        cm[u] = dim < d ? ldg(code + dim / a.dsub) : 0u;
        h8[u] = dim < d ? ldg(qh + dim) : 0.f;
        l8[u] = dim < d ? ldg(ql + dim) : 0.f;
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int dim = d0 + 64 * u;
        const int m = dim / a.dsub, t = dim - m * a.dsub;
        x[u] = dim < d ? ldg(a.cb + ((int64_t)m * 256 + cm[u]) * a.dsub + t) : 0.f;
      }
#pragma unroll
      for (int u = 0; u < 8; ++u)
        if (d0 + 64 * u < d) acc_sq_diff2(h8[u], l8[u], x[u], S, C);
    }
  } else {  // SEL_QUANT, SEL_COARSE_QUANT: quantised query vs quantised row
    const bool cq = a.mode == SEL_COARSE_QUANT;
    const float xs = a.qfmt == 2 ? ldg(a.qscale + L.row) : 1.f;
    const float qs = a.qfmt == 2 ? ldg(a.qQscale + q) : 1.f;
    if (!cq) {  // 16-byte chunks of the stored row, inside one slab
      measure_quant_rows<1>(a, q, &L, qq_lds, lane, &S, &C);
    } else {
      for (int dim = lane; dim < d; dim += 64) {
        float qh, ql, xh, xl;
        if (qq_lds)
          quant_value(a.qfmt, qq_lds, dim, qs, qh, ql, true);
        else
          quant_value(a.qfmt, a.qQ, q * a.ldqq + dim, qs, qh, ql);
        quant_value(a.qfmt, a.qvec,
                    ((int64_t)(dim / SLAB) * a.qnpad + L.row) * SLAB + (dim % SLAB), xs, xh, xl);
        acc_sq_diff2(qh, ql - xl, xh, S, C);  // (qh + ql) - (xh + xl)
      }
    }
  }
}

// Second exact measure: FP32 squared L2 on the first d_B coordinates
// (centroid rows, or the slab layout).
template <class QP>
__device__ __forceinline__ void measureB(const SelArgs &a, bool coarse, const CandLoc &L, QP qrow,
                                         int lane, float &S, float &C) {
  const int d = a.d_B;
  if (coarse) {
    const float *x = a.cent + L.row * a.ld_cent;
    for (int d0 = lane; d0 < d; d0 += 64 * 8) {
      float xv[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) xv[u] = d0 + 64 * u < d ? ldg(x + d0 + 64 * u) : 0.f;
#pragma unroll
      for (int u = 0; u < 8; ++u)
        if (d0 + 64 * u < d) acc_sq_diff(qrow[d0 + 64 * u], xv[u], S, C);
    }
  } else {
    // lane l takes coordinates 4l + 256u + e in that order, read as 16-byte
    // pieces, 2048 coordinates per pass
    const float *base = a.rows ? a.rows + L.row * a.d_pad
                               : a.vec + L.p0 * a.d_pad + (L.row - L.p0) * SLAB;
    const int64_t np = a.rows ? 1 : L.npad;
    for (int d0 = 4 * lane; d0 < d; d0 += 256 * 8) {
      float4 xv[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int dim = d0 + 256 * u;
        xv[u] = dim < d ? ldg4(base + (int64_t)(dim / SLAB) * np * SLAB + dim % SLAB)
                        : make_float4(0.f, 0.f, 0.f, 0.f);
      }
#pragma unroll
      for (int u = 0; u < 8; ++u)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int dim = d0 + 256 * u + e;
          if (dim < d) acc_sq_diff(qrow[dim], f4(xv[u], e), S, C);
        }
    }
  }
}

// G centroid candidates at once, their loads in flight together, each in the
// order of its single measure: measure1's quantised coarse case (STAGE 0)
// or measureB's centroid case (STAGE 1). Same bits as one at a time.
template <int G, int STAGE, class QP>
__device__ __forceinline__ void measure_cent_g(const SelArgs &a, int64_t q, const CandLoc *L,
                                               QP qrow, int lane, float *S, float *C) {
  if constexpr (STAGE == 0) {
    const int d = a.d_dot;
    const float qs = a.qfmt == 2 ? ldg(a.qQscale + q) : 1.f;
    float xs[G];
#pragma unroll
    for (int g = 0; g < G; ++g) xs[g] = a.qfmt == 2 ? ldg(a.qscale + L[g].row) : 1.f;
    for (int dim = lane; dim < d; dim += 64) {
      float qh, ql, xh[G], xl[G];
      quant_value(a.qfmt, a.qQ, q * a.ldqq + dim, qs, qh, ql);
#pragma unroll
      for (int g = 0; g < G; ++g)
        quant_value(a.qfmt, a.qvec,
                    ((int64_t)(dim / SLAB) * a.qnpad + L[g].row) * SLAB + (dim % SLAB), xs[g],
                    xh[g], xl[g]);
#pragma unroll
      for (int g = 0; g < G; ++g) acc_sq_diff2(qh, ql - xl[g], xh[g], S[g], C[g]);
    }
  } else {
    const int d = a.d_B;
    const float *x[G];
#pragma unroll
    for (int g = 0; g < G; ++g) x[g] = a.cent + L[g].row * a.ld_cent;
    for (int d0 = lane; d0 < d; d0 += 64 * 8) {
      float xv[G][8];
#pragma unroll
      for (int g = 0; g < G; ++g)
#pragma unroll
        for (int u = 0; u < 8; ++u) xv[g][u] = d0 + 64 * u < d ? ldg(x[g] + d0 + 64 * u) : 0.f;
#pragma unroll
      for (int u = 0; u < 8; ++u)
        if (d0 + 64 * u < d)
#pragma unroll
          for (int g = 0; g < G; ++g) acc_sq_diff(qrow[d0 + 64 * u], xv[g][u], S[g], C[g]);
    }
  }
}

// measureB's vector case (d_B <= 2048) with this lane's query coordinates
// 4l + 256u .. 4l + 256u + 3 already in registers (q4[u]); the same order of
// accumulation, so the same bits.
__device__ __forceinline__ void measureB_vec_rq(const SelArgs &a, const CandLoc &L,
                                                const float4 *q4, int lane, float &S,
                                                float &C) {
  const int d = a.d_B;
  const float *base = a.rows ? a.rows + L.row * a.d_pad
                             : a.vec + L.p0 * a.d_pad + (L.row - L.p0) * SLAB;
  const int64_t np = a.rows ? 1 : L.npad;
  float4 xv[8];
#pragma unroll
  for (int u = 0; u < 8; ++u) {
    const int dim = 4 * lane + 256 * u;
    xv[u] = dim < d ? ldg4(base + (int64_t)(dim / SLAB) * np * SLAB + dim % SLAB)
                    : make_float4(0.f, 0.f, 0.f, 0.f);
  }
#pragma unroll
  for (int u = 0; u < 8; ++u)
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int dim = 4 * lane + 256 * u + e;
      if (dim < d) acc_sq_diff(f4(q4[u], e), f4(xv[u], e), S, C);
    }
}

// The first-pass error bound of query q's candidates (one wave; every lane
// gets the same value).
//  * FP32 first pass |x|^2 - 2 q.x on d coordinates (SEL_COARSE, SEL_L2):
//    off its exact value by at most B = 4 (d + 2) 2^-24 (X^2 + 2 |q| X), X the
//    largest norm of the stored rows (xmax2 = X^2): four times the classical
//    bound of a length-d dot product and sum of squares in FP32 plus the final
//    rounding (the factor covers the matrix cores' undocumented internal
//    accumulation order).
//  * quantised first pass (SEL_QUANT, SEL_COARSE_QUANT): the same expression
//    for the dequantised operands, X = (largest FP32 norm) + (largest
//    |x - x^|), |q| replaced by |q^|.
//  * ADC (SEL_ADC): the first pass sums M table entries, each the FP32 sum over
//    dsub coordinates of (q'_hi - c)^2; against the exact asymmetric distance
//    (rotated query q'_hi + q'_lo) it is off by at most
//    B(f) = 4 (dsub + M + 4) 2^-24 f + 4 2^-24 |q'| (2 sqrt(f) + 2^-24 |q'|):
//    four times the classical bounds for the entries and their sum, plus the
//    dropped q'_lo (|q'_lo| <= 2^-24 |q'_hi|).
// Norms are rounded up by 1e-3 relative where the bound is not already four
// times the classical one.
__device__ FpBound wave_fp_bound(const SelArgs &a, int64_t q, int lane) {
  FpBound fb{0, 0.f, 0.f, 0.f, 0.f, -1.f, 0.f};
  const int d = a.d_dot;
  if (a.mode == SEL_ADC) {
    const float ADANNS_GLOBAL_AS *qh = (const float ADANNS_GLOBAL_AS *)(a.qr_hi + q * a.ldqr);
    float qq = 0.f;
    for (int dim = lane; dim < d; dim += 64) qq = fmaf(qh[dim], qh[dim], qq);
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) qq += __shfl_xor(qq, o);
    fb.qn = sqrtf(qq) * 1.001f;
    fb.c1 = 4.f * (float)(a.dsub + a.M + 4) * 0x1p-24f;
    fb.c2 = 4.f * 0x1p-24f * fb.qn;
    fb.kind = 2;
  } else if (a.mode == SEL_QUANT || a.mode == SEL_COARSE_QUANT) {
    const float ADANNS_GLOBAL_AS *qrow = (const float ADANNS_GLOBAL_AS *)(a.Qs + q * a.ldqs);
    float qq = 0.f, ee = 0.f;
    for (int dim = lane; dim < d; dim += 64) {
      const int64_t qi = q * a.ldqq + dim;
      const float qh = a.qfmt == 1
                           ? bf16_to_float(ldg((const uint16_t *)a.qQ + qi))
                           : ldg(a.qQscale + q) * e4m3_to_float(ldg((const uint8_t *)a.qQ + qi));
      const float df = qrow[dim] - qh;
      qq = fmaf(qh, qh, qq);
      ee = fmaf(df, df, ee);
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      qq += __shfl_xor(qq, o);
      ee += __shfl_xor(ee, o);
    }
    fb.eq = sqrtf(ee);
    fb.qq = qq;
    if (a.qerr != nullptr && a.xmax2 != nullptr) {
      const float X = (sqrtf(ldg(a.xmax2)) + ldg(a.qerr)) * 1.001f, qn = sqrtf(qq) * 1.001f;
      fb.B = 4.f * (float)(d + 2) * 0x1p-24f * (X * X + 2.f * qn * X);
      fb.kind = 1;
    }
  } else if (a.xmax2 != nullptr) {  // FP32 first pass
    const float ADANNS_GLOBAL_AS *qrow = (const float ADANNS_GLOBAL_AS *)(a.Qs + q * a.ldqs);
    float qq = 0.f;
    for (int dim = lane; dim < d; dim += 64) qq = fmaf(qrow[dim], qrow[dim], qq);
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) qq += __shfl_xor(qq, o);
    const float X2 = ldg(a.xmax2), X = sqrtf(X2), qn = sqrtf(qq);
    fb.B = 4.f * (float)(d + 2) * 0x1p-24f * (X2 + 2.f * qn * X);
    fb.kind = 1;
  }
  if (!(fb.B <= __FLT_MAX__) || !(fb.qn <= __FLT_MAX__)) fb.kind = 0;  // overflowed
  return fb;
}

// wave_fp_bound for the quantised modes with the query's coordinates read
// as 16-byte pieces, eight in flight per lane (the same bound; the sums'
// order differs, which their 1.001 margins cover). For the kernels whose
// registers allow it.
__device__ __forceinline__ FpBound wave_fp_bound_quant_vec(const SelArgs &a, int64_t q, int lane) {
  FpBound fb{0, 0.f, 0.f, 0.f, 0.f, -1.f, 0.f};
  const int d = a.d_dot;
  // lane l takes coordinates 4l + 256u .. +3 (16-byte query loads, eight
  // in flight; the staged rows are padded past d to a multiple of 4)
  const float *qrow = a.Qs + q * a.ldqs;
  const float qs = a.qfmt == 1 ? 1.f : ldg(a.qQscale + q);
  float qq = 0.f, ee = 0.f;
  for (int d0 = 4 * lane; d0 < d; d0 += 256 * 8) {
    float4 xv[8];
    uint2 hv[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int dim = d0 + 256 * u;
      const int64_t qi = q * a.ldqq + dim;
      xv[u] = dim < d ? ldg4(qrow + dim) : make_float4(0.f, 0.f, 0.f, 0.f);
      if (dim >= d) hv[u] = make_uint2(0u, 0u);
      else if (a.qfmt == 1) hv[u] = *(const uint2 *)((const uint16_t *)a.qQ + qi);
      else hv[u] = make_uint2(*(const uint32_t *)((const uint8_t *)a.qQ + qi), 0u);
    }
#pragma unroll
    for (int u = 0; u < 8; ++u)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int dim = d0 + 256 * u + e;
        if (dim < d) {
          const uint32_t w = e < 2 ? hv[u].x : hv[u].y;
          const float qh = a.qfmt == 1
                               ? __uint_as_float((e & 1 ? w >> 16 : w & 0xffffu) << 16)
                               : qs * e4m3_to_float((uint8_t)(hv[u].x >> (8 * e)));
          const float df = f4(xv[u], e) - qh;
          qq = fmaf(qh, qh, qq);
          ee = fmaf(df, df, ee);
        }
      }
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    qq += __shfl_xor(qq, o);
    ee += __shfl_xor(ee, o);
  }
  fb.eq = sqrtf(ee);
  fb.qq = qq;
  if (a.qerr != nullptr && a.xmax2 != nullptr) {
    const float X = (sqrtf(ldg(a.xmax2)) + ldg(a.qerr)) * 1.001f, qn = sqrtf(qq) * 1.001f;
    fb.B = 4.f * (float)(d + 2) * 0x1p-24f * (X * X + 2.f * qn * X);
    fb.kind = 1;
  }
  if (!(fb.B <= __FLT_MAX__)) fb.kind = 0;  // overflowed
  return fb;
}

// Hands query q to the re-selection launch (one lane / thread calls this).
__device__ __forceinline__ void push_redo(int32_t *cnt, int32_t *list, int64_t q) {
  const int slot = atomicAdd(cnt, 1);
  list[slot] = (int32_t)q;
  atomicAdd(&g_sel_stats[0], 1ull);
}

// measureB_vec_rq for two candidates at once (both rows' loads in flight);
// each row's order of accumulation as in measureB_vec_rq, so the same bits.
__device__ __forceinline__ void measureB_vec_rq2(const SelArgs &a, const CandLoc &L0,
                                                 const CandLoc &L1, const float4 *q4, int lane,
                                                 float &S0, float &C0, float &S1, float &C1) {
  const int d = a.d_B;
  const float *b0 = a.rows ? a.rows + L0.row * a.d_pad
                           : a.vec + L0.p0 * a.d_pad + (L0.row - L0.p0) * SLAB;
  const float *b1 = a.rows ? a.rows + L1.row * a.d_pad
                           : a.vec + L1.p0 * a.d_pad + (L1.row - L1.p0) * SLAB;
  const int64_t n0 = a.rows ? 1 : L0.npad, n1 = a.rows ? 1 : L1.npad;
  float4 x0[8], x1[8];
#pragma unroll
  for (int u = 0; u < 8; ++u) {
    const int dim = 4 * lane + 256 * u;
    const bool in = dim < d;
    x0[u] = in ? ldg4(b0 + (int64_t)(dim / SLAB) * n0 * SLAB + dim % SLAB)
               : make_float4(0.f, 0.f, 0.f, 0.f);
    x1[u] = in ? ldg4(b1 + (int64_t)(dim / SLAB) * n1 * SLAB + dim % SLAB)
               : make_float4(0.f, 0.f, 0.f, 0.f);
  }
#pragma unroll
  for (int u = 0; u < 8; ++u)
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int dim = 4 * lane + 256 * u + e;
      if (dim < d) {
        acc_sq_diff(f4(q4[u], e), f4(x0[u], e), S0, C0);
        acc_sq_diff(f4(q4[u], e), f4(x1[u], e), S1, C1);
      }
    }
}

__device__ __forceinline__ void select_body(const SelArgs &a, const int64_t q) {
  extern __shared__ __attribute__((aligned(16))) unsigned char sel_smem[];
  uint32_t *hist = (uint32_t *)sel_smem;
  float *qstage = (float *)sel_smem;  // reuses the histogram after selection
  uint8_t *qqstage = sel_smem + 2048 * 4;  // quantised query bytes (precision form)
  float *segbuf = (float *)(sel_smem + 2048 * 4 + 4096);
  int64_t *cpos = (int64_t *)(sel_smem + 2048 * 4 + 4096 + (size_t)a.lcap * 4);
  int64_t *cid = cpos + a.kcap;
  int64_t *cg = cid + a.kcap;         // coarse: h; scan: (h << 32) | row in list
  float *chi = (float *)(cg + a.kcap);
  float *clo = chi + a.kcap;
  __shared__ uint32_t sh32[16];
  __shared__ uint32_t s_bin, s_before, s_min, s_max;
  __shared__ int s_slot;

  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6, nwv = blockDim.x >> 6;
  const bool coarse = a.mode == SEL_COARSE || a.mode == SEL_COARSE_QUANT;
  const int64_t ldo = a.ldo ? a.ldo : a.kout;
  const float *seg;
  int64_t L, seg0 = 0;
  if (coarse) {
    seg = a.D + q * a.nl;
    L = a.nl;
  } else {
    seg0 = a.seg_off[q];
    seg = a.D + seg0;
    L = a.seg_off[q + 1] - seg0;
  }
  __shared__ FpBound s_fb;
  __shared__ int s_ncand, s_nkeep;
  __shared__ float s_up;
  int ncand;
  // the segment is staged in LDS when it fits: every pass below reads it
  const bool staged = L > a.K1 && L <= a.lcap;
  bool rounds = false;  // band wider than the slots: measured in rounds
  if (L <= a.K1) {
    ncand = (int)L;
    for (int i = tid; i < ncand; i += blockDim.x) cpos[i] = i;
  } else {
    // the first-pass error bound of this query (one wave computes it)
    if (wv == 0) {
      const FpBound fb = wave_fp_bound(a, q, lane);
      if (lane == 0) s_fb = fb;
    }
    if (staged) {  // eight independent loads in flight per thread
      for (int64_t base = tid; base < L; base += (int64_t)blockDim.x * 8) {
        float v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const int64_t i = base + (int64_t)blockDim.x * u;
          v[u] = i < L ? seg[i] : 0.f;
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const int64_t i = base + (int64_t)blockDim.x * u;
          if (i < L) segbuf[i] = v[u];
        }
      }
    }
    // The segment is read from LDS or from global memory; the generic lambda
    // is instantiated for each so that neither becomes a flat access.
    auto select_from = [&](auto src) {
      // key range of the segment
      uint32_t kmin = 0xffffffffu, kmax = 0u;
      if (tid == 0) {
        s_min = 0xffffffffu;
        s_max = 0u;
      }
      __syncthreads();
      for (int64_t i = tid; i < L; i += blockDim.x) {
        const uint32_t kk = order_key(src[i]);
        kmin = kk < kmin ? kk : kmin;
        kmax = kk > kmax ? kk : kmax;
      }
      atomicMin(&s_min, kmin);
      atomicMax(&s_max, kmax);
      __syncthreads();
      // radix selection of the K-th smallest key over an adaptive window
      // [lo, hi): each pass splits the window into at most 2048 bins; the
      // last pass has unit bins, so T is exact; on return need counts the
      // keys equal to T that belong to the K smallest and n_eq all of them
      auto radix = [&](uint32_t K, uint32_t &T, uint32_t &need, uint32_t &n_eq) {
        uint64_t lo = s_min, hi = (uint64_t)s_max + 1;
        need = K;
        for (int pass = 0; pass < 4; ++pass) {
          const uint64_t width = hi - lo;
          const int shift = width <= 2048 ? 0 : (64 - __clzll((long long)(width - 1))) - 11;
          for (int i = tid; i < 2048; i += blockDim.x) hist[i] = 0;
          __syncthreads();
          for (int64_t i = tid; i < L; i += blockDim.x) {
            const uint64_t kk = order_key(src[i]);
            if (kk >= lo && kk < hi) atomicAdd(&hist[(uint32_t)((kk - lo) >> shift)], 1u);
          }
          __syncthreads();
          const int per = 2048 / blockDim.x;
          uint32_t local = 0;
          for (int e = 0; e < per; ++e) local += hist[tid * per + e];
          uint32_t excl = block_excl_scan<uint32_t>(local, sh32, nullptr);
          if (excl < need && need <= excl + local) {
            uint32_t c = excl;
            for (int e = 0; e < per; ++e) {
              uint32_t hb = hist[tid * per + e];
              if (c + hb >= need) {
                s_bin = (uint32_t)(tid * per + e);
                s_before = c;
                break;
              }
              c += hb;
            }
          }
          __syncthreads();
          const uint64_t nlo = lo + ((uint64_t)s_bin << shift);
          const uint64_t nhi = nlo + ((uint64_t)1 << shift);
          need -= s_before;
          lo = nlo;
          hi = nhi < hi ? nhi : hi;
          __syncthreads();
          if (shift == 0) break;
        }
        T = (uint32_t)lo;
        n_eq = hist[s_bin];
        __syncthreads();
      };
      // the K smallest (key, position) composites, in slots 0..K-1
      auto take_smallest = [&](int K) {
        uint32_t T, need, n_eq;
        radix((uint32_t)K, T, need, n_eq);
        if (tid == 0) s_slot = 0;
        __syncthreads();
        if (n_eq == need) {
          // every key equal to T is taken: one coalesced pass, any slot order
          for (int64_t i = tid; i < L; i += blockDim.x) {
            if (order_key(src[i]) <= T) {
              const int slot = atomicAdd(&s_slot, 1);
              cpos[slot] = i;
            }
          }
        } else {
          // take every key below T and the first ``need`` equal ones in
          // position order
          const int64_t chunk = (L + blockDim.x - 1) / blockDim.x;
          const int64_t a0 = tid * chunk, a1 = min64(L, a0 + chunk);
          uint32_t ne = 0;
          for (int64_t i = a0; i < a1; ++i) ne += order_key(src[i]) == T;
          uint32_t eq_before = block_excl_scan<uint32_t>(ne, sh32, nullptr);
          const int nlt = K - (int)need;
          for (int64_t i = a0; i < a1; ++i) {
            uint32_t kk = order_key(src[i]);
            if (kk < T) {
              int slot = atomicAdd(&s_slot, 1);
              cpos[slot] = i;
            } else if (kk == T) {
              if (eq_before < need) cpos[nlt + eq_before] = i;
              ++eq_before;
            }
          }
        }
      };
      const FpBound fb = s_fb;
      // Precision form (quantised first pass, then the exact FP32 distance
      // re-ranks the K2 nearest by exact quantised distance): the final k
      // are found without materialising that shortlist S*. With B the first
      // pass's bound, a candidate with f < v_{K2+1} - 2B is surely in S*
      // (nearer than every candidate outside the first pass's K2 smallest)
      // and one with f > v_K2 + 2B surely not. Its FP32 distance is at least
      // (sqrt(f - B) - |q - q^| - |x - x^|)^2 (triangle inequality; the
      // second norm is the candidate's own row's quantisation error). The k
      // nearest by first pass (surely in S*) are measured in FP32; U, the
      // largest of those, bounds the k-th FP32 distance of S* from above, so
      // only sure candidates whose lower bound reaches U are measured. If a
      // candidate that is not surely in S* could reach U, the general path
      // below decides S* exactly instead.
      if (a.mode == SEL_QUANT && a.stageB && a.qrerr != nullptr && a.qerr != nullptr &&
          a.d_B == a.d_dot && fb.kind == 1 && L > a.K2 && a.kout <= a.K2 && a.kout <= a.kcap) {
        __shared__ int s_qr;
        __shared__ uint32_t s_above;
        const float B = fb.B;
        uint32_t T2, need2, neq2;
        radix((uint32_t)a.K2, T2, need2, neq2);
        const float vK2 = comp_value((uint64_t)T2 << 32);
        if (tid == 0) s_above = 0xffffffffu;
        __syncthreads();
        if (neq2 <= need2) {  // the smallest key above T2 is v_{K2+1}
          uint32_t mk = 0xffffffffu;
          for (int64_t i = tid; i < L; i += blockDim.x) {
            const uint32_t kk = order_key(src[i]);
            if (kk > T2 && kk < mk) mk = kk;
          }
          atomicMin(&s_above, mk);
        }
        __syncthreads();
        const float vK2p1 = neq2 > need2 ? vK2 : comp_value((uint64_t)s_above << 32);
        const float sure_thr = vK2p1 - 2.f * B, amb_hi = vK2 + 2.f * B;
        // the k nearest by first pass, measured in FP32
        take_smallest(a.kout);
        if (tid == 0) s_qr = 1;
        __syncthreads();
        const float ADANNS_GLOBAL_AS *qg = (const float ADANNS_GLOBAL_AS *)(a.Qs + q * a.ldqs);
        for (int c = wv; c < a.kout; c += nwv) {
          const CandLoc Lc = locate(a, false, q, seg0, cpos[c]);
          float S = 0.f, C = 0.f;
          measureB(a, false, Lc, qg, lane, S, C);
          wave_reduce_pair(S, C);
          if (lane == 0) {
            chi[c] = S;
            clo[c] = C;
            if (!(src[cpos[c]] < sure_thr)) s_qr = 0;  // not surely in S*: general path
          }
        }
        __syncthreads();
        if (tid == 0) {
          float u = 0.f;
          for (int c = 0; c < a.kout; ++c) u = fmaxf(u, chi[c] + clo[c]);
          s_up = u * (1.f + 0x1p-20f);
          s_slot = 0;
        }
        __syncthreads();
        if (s_qr) {
          // the first pass omits |q^|^2: the exact quantised distance is at
          // least f - B + |q^|^2, the FP32 sum of squares |q^|^2 being off by
          // at most 4 (d + 2) 2^-24 of itself
          const float qlo = fb.qq * (1.f - 4.f * (float)(a.d_dot + 2) * 0x1p-24f);
          const float sU = sqrtf(s_up);
          const float eq = fb.eq * 1.001f;
          const float reach = sU + eq + ldg(a.qerr) * 1.001f;
          const float fmax = fminf(amb_hi, reach * reach * 1.001f + B - qlo);
          for (int64_t i = tid; i < L; i += blockDim.x) {
            const float f = src[i];
            if (!(f <= fmax)) continue;
            const CandLoc Lc = locate(a, false, q, seg0, i);
            const float lo = sqrtf(fmaxf(f - B + qlo, 0.f)) - eq - ldg(a.qrerr + Lc.row) * 1.001f;
            if (lo <= sU) {
              const int slot = atomicAdd(&s_slot, 1);
              if (slot < a.kcap) cpos[slot] = i;
              if (!(f < sure_thr)) s_qr = 0;
            }
          }
        }
        __syncthreads();
        const int nM = s_slot;
        if (s_qr && nM <= a.kcap && nM >= a.kout) {
          for (int c = wv; c < nM; c += nwv) {
            const CandLoc Lc = locate(a, false, q, seg0, cpos[c]);
            float S = 0.f, C = 0.f;
            measureB(a, false, Lc, qg, lane, S, C);
            wave_reduce_pair(S, C);
            if (lane == 0) {
              chi[c] = S;
              clo[c] = C;
              cid[c] = Lc.id;
              cg[c] = Lc.gpack;
            }
          }
          int P2 = 1;
          while (P2 < nM) P2 <<= 1;
          for (int c = nM + tid; c < P2; c += blockDim.x) {
            chi[c] = __builtin_inff();
            clo[c] = 0.f;
            cid[c] = INT64_MAX;
            cg[c] = -1;
          }
          bitonic_sort(chi, clo, cid, cg, P2);
          const int64_t ldo_ = a.ldo ? a.ldo : a.kout;
          for (int j = tid; j < a.kout; j += blockDim.x) {
            a.out_dist[q * ldo_ + j] = chi[j];
            a.out_ids[q * ldo_ + j] = cid[j];
          }
          if (tid == 0) s_ncand = -4;  // done
          return;
        }
        __syncthreads();
      }
      if (fb.kind == 0) {
        // no error bound known: the plain margin, not certified
        take_smallest(a.K1);
        if (tid == 0) {
          s_ncand = a.K1;
          atomicAdd(&g_sel_stats[1], 1ull);
        }
        return;
      }
      // Certified shortlist: every candidate whose first-pass value can still
      // reach the kv nearest (FpBound::keep against the kv-th smallest value),
      // however many there are.
      const int kv = a.stageB ? a.K2 : a.kout;
      uint32_t T, need, n_eq;
      radix((uint32_t)kv, T, need, n_eq);
      const float up = fb.upper(comp_value((uint64_t)T << 32));
      if (tid == 0) s_slot = 0;
      __syncthreads();
      int nk = 0;
      for (int64_t i = tid; i < L; i += blockDim.x) nk += fb.keep(src[i], up);
      atomicAdd(&s_slot, nk);
      __syncthreads();
      const int n_keep = s_slot;
      __syncthreads();
      if (n_keep <= a.kcap) {
        if (tid == 0) s_slot = 0;
        __syncthreads();
        for (int64_t i = tid; i < L; i += blockDim.x)
          if (fb.keep(src[i], up)) cpos[atomicAdd(&s_slot, 1)] = i;
        if (tid == 0) s_ncand = n_keep;
      } else if (a.redo_list != nullptr) {
        // more than this launch's slots: the re-selection launch takes it
        if (tid == 0) {
          push_redo(a.redo_cnt, a.redo_list, q + a.redo_q0);
          s_ncand = -1;
        }
      } else if (a.kcap - kv >= 1) {
        // more than this launch's slots: the band is measured in rounds of
        // kcap - kv candidates, keeping the kv best (see below)
        if (tid == 0) {
          s_ncand = -2;
          s_nkeep = n_keep;
          s_up = up;
        }
      } else {
        // no room for rounds (kv fills the slots): the kcap nearest by first
        // pass, counted as not certified
        take_smallest(a.kcap);
        if (tid == 0) {
          s_ncand = a.kcap;
          atomicAdd(&g_sel_stats[1], 1ull);
        }
      }
    };
    __syncthreads();  // s_fb
    if (staged)
      select_from(segbuf);
    else
      select_from((const float ADANNS_GLOBAL_AS *)seg);
    __syncthreads();
    ncand = s_ncand;
    if (ncand == -1 || ncand == -4) return;  // handed over / done (uniform over the block)
    rounds = ncand == -2;
  }
  __syncthreads();
  // stage the query row (coordinates of both measures) in LDS
  const int dq_stage = a.d_dot > a.d_B ? a.d_dot : a.d_B;
  const bool qstaged = dq_stage <= 2048;
  if (qstaged)
    for (int i = tid; i < dq_stage; i += blockDim.x) qstage[i] = a.Qs[q * a.ldqs + i];
  const int qeb = a.qfmt == 1 ? 2 : 1;
  const bool qqstaged = (a.mode == SEL_QUANT || a.mode == SEL_COARSE_QUANT) &&
                        (int64_t)a.d_dot * qeb <= 4096;
  if (qqstaged) {
    const uint8_t *src = (const uint8_t *)a.qQ + q * a.ldqq * qeb;
    for (int i = tid; i < a.d_dot * qeb; i += blockDim.x) qqstage[i] = src[i];
  }
  __syncthreads();

  // first exact measure, one wave per candidate; the query row is read from
  // LDS when staged, else from global memory (one instantiation each)
  const float ADANNS_GLOBAL_AS *qglob = (const float ADANNS_GLOBAL_AS *)(a.Qs + q * a.ldqs);
  auto run1 = [&](auto qrow, int c0, int c1) {
    for (int c = c0 + wv; c < c1; c += nwv) {
      const CandLoc Lc = locate(a, coarse, q, seg0, cpos[c]);
      float S = 0.f, C = 0.f;
      measure1(a, q, Lc, qrow, qqstaged ? qqstage : nullptr, lane, S, C);
      wave_reduce_pair(S, C);
      if (lane == 0) {
        chi[c] = S;
        clo[c] = C;
        cid[c] = Lc.id;
        cg[c] = Lc.gpack;
      }
    }
  };
  auto sort_first = [&](int n) {  // sorts slots [0, n) by (distance pair, id)
    int P2 = 1;
    while (P2 < n) P2 <<= 1;
    for (int c = n + tid; c < P2; c += blockDim.x) {
      chi[c] = __builtin_inff();
      clo[c] = 0.f;
      cid[c] = INT64_MAX;
      cg[c] = -1;
    }
    bitonic_sort(chi, clo, cid, cg, P2);
  };
  if (!rounds) {
    if (qstaged)
      run1(qstage, 0, ncand);
    else
      run1(qglob, 0, ncand);
    sort_first(ncand);
  } else {
    // The band holds n_keep > kcap candidates: in position order, rounds of
    // kcap - kv of them are measured into the slots after the kv best so
    // far, and the slots re-sorted, so that the kv best of the whole band
    // remain. Every candidate of the band is measured exactly once.
    const int kv = a.stageB ? a.K2 : a.kout;
    const int C = a.kcap - kv;
    const int nk = s_nkeep;
    auto band_rounds = [&](auto src) {
      const FpBound fb = s_fb;
      const float up = s_up;
      const int64_t chunk = (L + blockDim.x - 1) / blockDim.x;
      const int64_t a0 = tid * chunk, a1 = min64(L, a0 + chunk);
      int have = 0;
      for (int lo = 0; lo < nk; lo += C) {
        const int cnt = min(C, nk - lo);
        uint32_t ne = 0;
        for (int64_t i = a0; i < a1; ++i) ne += fb.keep(src[i], up);
        uint32_t r = block_excl_scan<uint32_t>(ne, sh32, nullptr);
        for (int64_t i = a0; i < a1 && r < (uint32_t)(lo + cnt); ++i)
          if (fb.keep(src[i], up)) {
            if (r >= (uint32_t)lo) cpos[have + (r - lo)] = i;
            ++r;
          }
        __syncthreads();
        if (qstaged)
          run1(qstage, have, have + cnt);
        else
          run1(qglob, have, have + cnt);
        sort_first(have + cnt);
        have = min(kv, have + cnt);
      }
      ncand = have;
    };
    if (staged)
      band_rounds(segbuf);
    else
      band_rounds((const float ADANNS_GLOBAL_AS *)seg);
  }

  int nres = ncand;
  if (a.stageB) {
    // second exact measure (FP32 L2 on d_B coordinates) of the K2 best
    nres = ncand < a.K2 ? ncand : a.K2;
    // quantised rows: as in wave_select, only the prefix within
    // (sqrt(D^_k) + 2e)^2, e = |q - q^| + the largest |x - x^|, is re-measured
    // (both measures on the same prefix: distances on different prefixes do
    // not bound each other)
    if ((a.mode == SEL_QUANT || a.mode == SEL_COARSE_QUANT) && a.qemax != nullptr &&
        a.d_B == a.d_dot && nres > a.kout) {
      __shared__ float s_eq[16];
      __shared__ int s_nres;
      float eq = 0.f;
      for (int dim = tid; dim < a.d_B; dim += blockDim.x) {
        const int64_t qi = q * a.ldqq + dim;
        const float qh = a.qfmt == 1 ? bf16_to_float(ldg((const uint16_t *)a.qQ + qi))
                                     : ldg(a.qQscale + q) * e4m3_to_float(ldg((const uint8_t *)a.qQ + qi));
        const float df = ldg(a.Qs + q * a.ldqs + dim) - qh;
        eq = fmaf(df, df, eq);
      }
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) eq += __shfl_xor(eq, o);
      if (lane == 0) s_eq[wv] = eq;
      __syncthreads();
      if (tid == 0) {
        float t = 0.f;
        for (int w = 0; w < nwv; ++w) t += s_eq[w];
        // a margin of 1e-3 relative covers the FP32 rounding of these bounds
        const float e = (sqrtf(t) + ldg(a.qemax)) * 1.001f;
        const float up = (sqrtf(fmaxf(chi[a.kout - 1], 0.f)) + 2.f * e) * 1.001f;
        int lo = a.kout, hi = nres;  // the first position past the bound
        while (lo < hi) {
          const int mid = (lo + hi) >> 1;
          if (sqrtf(fmaxf(chi[mid], 0.f)) <= up) lo = mid + 1; else hi = mid;
        }
        s_nres = lo;
      }
      __syncthreads();
      nres = s_nres;
    }
    auto run2 = [&](auto qrow) {
      for (int c = wv; c < nres; c += nwv) {
        float S = 0.f, C = 0.f;
        measureB(a, coarse, locate_packed(a, coarse, cg[c]), qrow, lane, S, C);
        wave_reduce_pair(S, C);
        if (lane == 0) {
          chi[c] = S;
          clo[c] = C;
        }
      }
    };
    if (qstaged)
      run2(qstage);
    else
      run2(qglob);
    __syncthreads();
    int P3 = 1;
    while (P3 < nres) P3 <<= 1;
    for (int c = nres + tid; c < P3; c += blockDim.x) {
      chi[c] = __builtin_inff();
      clo[c] = 0.f;
      cid[c] = INT64_MAX;
      cg[c] = -1;
    }
    bitonic_sort(chi, clo, cid, cg, P3);
  }
  for (int j = tid; j < a.kout; j += blockDim.x) {
    const bool has = j < nres;
    if (coarse) {
      const int32_t hsel = has ? (int32_t)cid[j] : -1;
      a.out_probes[q * a.kout + j] = hsel;
      if (a.out_probes2) a.out_probes2[q * a.kout + j] = hsel;
      // coarse distance output: the nearest centroid's distance per query
      if (a.out_dist && j == 0) a.out_dist[q * ldo] = has ? chi[0] : __builtin_inff();
    } else {
      a.out_dist[q * ldo + j] = has ? chi[j] : __builtin_inff();
      a.out_ids[q * ldo + j] = has ? cid[j] : -1;
    }
  }
}

__global__ __launch_bounds__(512) void k_select_refine(SelArgs a) { select_body(a, blockIdx.x); }

// Re-selection of the queries a previous selection launch handed over (their
// first shortlist could not be certified): the certified band selection of
// select_body with this launch's larger candidate capacity. The grid strides
// over the list; its length is read from device memory, so the launch needs
// no host synchronisation.
__global__ __launch_bounds__(512) void k_select_refine_redo(SelArgs a) {
  const int32_t n = *(volatile const int32_t *)a.redo_cnt;
  const int32_t *list = a.redo_list;
  SelArgs b = a;
  b.redo_cnt = nullptr;
  b.redo_list = nullptr;
  for (int32_t i = blockIdx.x; i < n; i += gridDim.x) {
    select_body(b, list[i]);
    __syncthreads();  // LDS reused by the next query
  }
}

// Precision-form re-rank of a deep shortlist (SEL_QUANT with the FP32
// re-rank, K2 > the one-wave list), one 256-thread workgroup per query, in
// the common case; every other case is handed to the re-selection launch
// (select_body: the same reasoning with exact order statistics, else the
// shortlist decided exactly). With f the quantised first-pass values of the
// query's candidates and B their error bound (wave_fp_bound):
//  * one 2048-bin histogram of f (equal widths between the segment's min and
//    max) places ranks kout, K2 and K2 + 1 in bins; bin edges widened by one
//    bin on each side give v_{K2+1} >= lo and v_K2 <= hi, so a candidate with
//    f < lo - 2B is surely in the shortlist S* (the K2 nearest by exact
//    quantised distance) and one with f > hi + 2B surely not;
//  * the candidates in the bins up to rank kout (all surely in S*, else the
//    query is handed over) are measured in FP32; U, their kout-th smallest
//    distance, bounds the kout-th FP32 distance of S* from above;
//  * a candidate's FP32 distance is at least
//    (sqrt(f - B + |q^|^2) - |q - q^| - |x - x^|)^2, so only those whose
//    bound reaches U are measured (all must be surely in S*), and the kout
//    nearest of them are the result.
constexpr int QRR_BINS = 2048;
constexpr int QRR_CAP = 256;

__global__ __launch_bounds__(256) void k_select_qrerank(SelArgs a) {
  __shared__ uint32_t hist[QRR_BINS];
  __shared__ int64_t cpos[QRR_CAP], cid[QRR_CAP], cg[QRR_CAP];
  __shared__ float chi[QRR_CAP], clo[QRR_CAP];
  __shared__ uint32_t sh32[16];
  __shared__ FpBound s_fb;
  __shared__ uint32_t s_kmin, s_kmax;
  __shared__ int s_cnt, s_bad, s_bk, s_b2, s_b3;
  __shared__ float s_U;
  const int64_t q = blockIdx.x;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6, nwv = blockDim.x >> 6;
  const int kout = a.kout, K2 = a.K2;
  const int64_t seg0 = a.seg_off[q], L = a.seg_off[q + 1] - seg0;
  const float ADANNS_GLOBAL_AS *src = (const float ADANNS_GLOBAL_AS *)(a.D + seg0);
  const int64_t ldo = a.ldo ? a.ldo : a.kout;
  auto hand_over = [&]() {
    if (tid == 0) push_redo(a.redo_cnt, a.redo_list, q + a.redo_q0);
  };
  if (L <= (int64_t)K2 + REFINE_MARGIN) {  // short segments: the general path
    hand_over();
    return;
  }
  if (wv == 0) {
    const FpBound fb = wave_fp_bound(a, q, lane);
    if (lane == 0) s_fb = fb;
  }
  if (tid == 0) {
    s_kmin = 0xffffffffu;
    s_kmax = 0u;
    s_cnt = 0;
    s_bad = 0;
  }
  for (int i = tid; i < QRR_BINS; i += blockDim.x) hist[i] = 0;
  __syncthreads();
  const FpBound fb = s_fb;
  if (fb.kind != 1) {
    hand_over();
    return;
  }
  // passes over the segment: eight loads in flight per thread (positions
  // past the end re-read the last value and are not visited)
  auto each_f = [&](auto fn) {
    for (int64_t base = tid; base < L; base += (int64_t)blockDim.x * 8) {
      float v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) v[u] = src[min64(base + (int64_t)blockDim.x * u, L - 1)];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int64_t i = base + (int64_t)blockDim.x * u;
        if (i < L) fn(i, v[u]);
      }
    }
  };
  {
    uint32_t kmin = 0xffffffffu, kmax = 0u;
    each_f([&](int64_t, float f) {
      const uint32_t kk = order_key(f);
      kmin = kk < kmin ? kk : kmin;
      kmax = kk > kmax ? kk : kmax;
    });
    atomicMin(&s_kmin, kmin);
    atomicMax(&s_kmax, kmax);
  }
  __syncthreads();
  const float fmin = comp_value((uint64_t)s_kmin << 32), fmax = comp_value((uint64_t)s_kmax << 32);
  const float w = (fmax - fmin) / (float)QRR_BINS;
  const float inv = fmax > fmin ? (float)QRR_BINS / (fmax - fmin) : 0.f;
  auto bin_of = [&](float f) { return min(QRR_BINS - 1, max(0, (int)((f - fmin) * inv))); };
  each_f([&](int64_t, float f) { atomicAdd(&hist[bin_of(f)], 1u); });
  __syncthreads();
  {
    constexpr int per = QRR_BINS / 256;
    uint32_t local = 0;
    for (int e = 0; e < per; ++e) local += hist[tid * per + e];
    uint32_t c = block_excl_scan<uint32_t>(local, sh32, nullptr);
    for (int e = 0; e < per; ++e) {
      const uint32_t hb = hist[tid * per + e], b = tid * per + e;
      if (c < (uint32_t)kout && (uint32_t)kout <= c + hb) s_bk = b;
      if (c < (uint32_t)K2 && (uint32_t)K2 <= c + hb) s_b2 = b;
      if (c < (uint32_t)K2 + 1 && (uint32_t)K2 + 1 <= c + hb) s_b3 = b;
      c += hb;
    }
  }
  __syncthreads();
  const float B = fb.B;
  const float sure_thr = (fmin + (float)(s_b3 - 1) * w) - 2.f * B;  // below: surely in S*
  const float amb_hi = (fmin + (float)(s_b2 + 2) * w) + 2.f * B;    // above: surely not
  const int bk = s_bk;
  // the candidates of the bins up to rank kout
  each_f([&](int64_t i, float f) {
    if (bin_of(f) <= bk) {
      const int slot = atomicAdd(&s_cnt, 1);
      if (slot < QRR_CAP) cpos[slot] = i;
      if (!(f < sure_thr)) s_bad = 1;
    }
  });
  __syncthreads();
  const int c0 = s_cnt;
  if (s_bad || c0 > QRR_CAP || c0 < kout) {
    hand_over();
    return;
  }
  const float ADANNS_GLOBAL_AS *qg = (const float ADANNS_GLOBAL_AS *)(a.Qs + q * a.ldqs);
  // this lane's query coordinates 4 lane + 256 u (+0..3), read once
  const bool rq = a.d_B <= 2048;
  float4 q4[8];
  if (rq) {
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      float v[4];
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int dim = 4 * lane + 256 * u + e;
        v[e] = dim < a.d_B ? qg[dim] : 0.f;
      }
      q4[u] = make_float4(v[0], v[1], v[2], v[3]);
    }
  }
  auto measure = [&](int n) {  // FP32 distances of slots [0, n), sorted
    if (rq) {  // two candidates per wave at a time
      for (int c = 2 * wv; c < n; c += 2 * nwv) {
        const int c1 = c + 1 < n ? c + 1 : c;
        const CandLoc L0 = locate(a, false, q, seg0, cpos[c]);
        const CandLoc L1 = locate(a, false, q, seg0, cpos[c1]);
        float S0 = 0.f, C0 = 0.f, S1 = 0.f, C1 = 0.f;
        measureB_vec_rq2(a, L0, L1, q4, lane, S0, C0, S1, C1);
        wave_reduce_pair(S0, C0);
        wave_reduce_pair(S1, C1);
        if (lane == 0) {
          chi[c] = S0;
          clo[c] = C0;
          cid[c] = L0.id;
          cg[c] = L0.gpack;
          if (c1 != c) {
            chi[c1] = S1;
            clo[c1] = C1;
            cid[c1] = L1.id;
            cg[c1] = L1.gpack;
          }
        }
      }
    } else {
      for (int c = wv; c < n; c += nwv) {
        const CandLoc Lc = locate(a, false, q, seg0, cpos[c]);
        float S = 0.f, C = 0.f;
        measureB(a, false, Lc, qg, lane, S, C);
        wave_reduce_pair(S, C);
        if (lane == 0) {
          chi[c] = S;
          clo[c] = C;
          cid[c] = Lc.id;
          cg[c] = Lc.gpack;
        }
      }
    }
    int P2 = 1;
    while (P2 < n) P2 <<= 1;
    __syncthreads();
    for (int c = n + tid; c < P2; c += blockDim.x) {
      chi[c] = __builtin_inff();
      clo[c] = 0.f;
      cid[c] = INT64_MAX;
      cg[c] = -1;
    }
    bitonic_sort(chi, clo, cid, cg, P2);
  };
  measure(c0);
  if (tid == 0) {
    s_U = (chi[kout - 1] + clo[kout - 1]) * (1.f + 0x1p-20f);
    s_cnt = 0;
  }
  __syncthreads();
  // the candidates whose FP32 lower bound reaches U
  {
    const float qlo = fb.qq * (1.f - 4.f * (float)(a.d_dot + 2) * 0x1p-24f);
    const float sU = sqrtf(s_U);
    const float eq = fb.eq * 1.001f;
    const float reach = sU + eq + ldg(a.qerr) * 1.001f;
    const float flim = fminf(amb_hi, reach * reach * 1.001f + B - qlo);
    each_f([&](int64_t i, float f) {
      if (!(f <= flim)) return;
      const CandLoc Lc = locate(a, false, q, seg0, i);
      const float lo = sqrtf(fmaxf(f - B + qlo, 0.f)) - eq - ldg(a.qrerr + Lc.row) * 1.001f;
      if (lo <= sU) {
        const int slot = atomicAdd(&s_cnt, 1);
        if (slot < QRR_CAP) cpos[slot] = i;
        if (!(f < sure_thr)) s_bad = 1;
      }
    });
  }
  __syncthreads();
  const int nM = s_cnt;
  if (s_bad || nM > QRR_CAP || nM < kout) {
    hand_over();
    return;
  }
  measure(nM);
  for (int j = tid; j < kout; j += blockDim.x) {
    a.out_dist[q * ldo + j] = chi[j];
    a.out_ids[q * ldo + j] = cid[j];
  }
}

// Exact FP32 k nearest of every candidate with a quantised first pass
// (adanns_search_filtered: the same result as adanns_search, bit for bit), one
// 256-thread workgroup per query. With f the quantised first-pass values and
// B their error bound, a candidate's FP32 distance is at least
// lo = sqrt(f - B + |q^|^2) - |q - q^| - |x - x^| (triangle inequality, the
// last norm the candidate's own row's quantisation error).
//  1. The candidates of the f-histogram bins up to rank k (set 1) are
//     measured exactly in FP32; U, their k-th smallest distance, bounds the
//     k-th nearest's from above.
//  2. Every other candidate whose lo reaches sqrt(U) is measured and the k
//     nearest of all measured ones returned. When more than the free slots
//     qualify, they are taken in windows of increasing lo (a histogram of lo
//     picks each window), U tightening after each; a window that cannot be
//     split falls back to rounds in position order.
// Candidates are located through the query's probe table staged in LDS
// (position -> probe by binary search); queries with more probes than the
// table holds locate through global memory. g_sel_stats[2] counts exact
// measures, g_sel_stats[3] queries that needed more than one window.
// Exact FP32 measure (compensated, as measureB) of two vector rows at once
// against the query row qrow (16-byte aligned, padded to a multiple of 4):
// lane l takes coordinates 4l + 256u + e in that order, 1024 per pass, the
// query's pieces re-read from L2 each pass (fewer registers than holding
// them), so each row's sum has measureB's order and bits. xp / np: the rows'
// first slab piece and slab stride in rows (1 for the row-major copy).
__device__ __forceinline__ void measure2_rows(const float *qrow, int d, const float *const xp[2],
                                              const int64_t np[2], int lane, float S[2],
                                              float C[2]) {
  constexpr int PP = 4;
  for (int d0 = 4 * lane; d0 < d; d0 += 256 * PP) {
    float4 qv[PP], xv[2][PP];
#pragma unroll
    for (int u = 0; u < PP; ++u) {
      const int dim = d0 + 256 * u;
      qv[u] = dim < d ? ldg4(qrow + dim) : make_float4(0.f, 0.f, 0.f, 0.f);
    }
#pragma unroll
    for (int gi = 0; gi < 2; ++gi)
#pragma unroll
      for (int u = 0; u < PP; ++u) {
        const int dim = d0 + 256 * u;
        xv[gi][u] = dim < d ? ldg4(xp[gi] + (int64_t)(dim / SLAB) * np[gi] * SLAB + dim % SLAB)
                            : make_float4(0.f, 0.f, 0.f, 0.f);
      }
#pragma unroll
    for (int u = 0; u < PP; ++u)
#pragma unroll
      for (int e = 0; e < 4; ++e)
        if (d0 + 256 * u + e < d)
#pragma unroll
          for (int gi = 0; gi < 2; ++gi) acc_sq_diff(f4(qv[u], e), f4(xv[gi][u], e), S[gi], C[gi]);
  }
}

constexpr int FLT_NPT = 256;
constexpr int FLT_LIST = 1024;  // candidates listed for the bound test

__device__ __forceinline__ void filtered_block(const SelArgs &a, const int64_t q) {
  __shared__ uint32_t hist[QRR_BINS];
  __shared__ int32_t s_lpos[FLT_LIST];
  __shared__ float s_lf[FLT_LIST];
  __shared__ int64_t cpos[QRR_CAP], cid[QRR_CAP], cg[QRR_CAP];
  __shared__ float chi[QRR_CAP], clo[QRR_CAP];
  __shared__ int64_t t_start[FLT_NPT + 1], t_p0[FLT_NPT], t_np[FLT_NPT];
  __shared__ int32_t t_h[FLT_NPT];
  __shared__ uint32_t sh32[16];
  __shared__ FpBound s_fb;
  __shared__ uint32_t s_kmin, s_kmax;
  __shared__ int s_cnt, s_bk, s_c1, s_nl;
  __shared__ float s_t;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6, nwv = blockDim.x >> 6;
  const int kout = a.kout, np = a.nprobe;
  const int64_t seg0 = a.seg_off[q], L = a.seg_off[q + 1] - seg0;
  const float ADANNS_GLOBAL_AS *src = (const float ADANNS_GLOBAL_AS *)(a.D + seg0);
  const int64_t ldo = a.ldo ? a.ldo : a.kout;
  const bool tab = np <= FLT_NPT;
  if (wv == 0) {
    const FpBound fb = wave_fp_bound_quant_vec(a, q, lane);
    if (lane == 0) s_fb = fb;
  }
  if (tid == 0) {
    s_kmin = 0xffffffffu;
    s_kmax = 0u;
    s_cnt = 0;
  }
  if (tab) {
    for (int p = tid; p < np; p += blockDim.x) {
      const int32_t h = ldg(a.probes + q * np + p);
      t_start[p] = ldg(a.pair_base + q * np + p) - seg0;
      t_h[p] = h;
      t_p0[p] = ldg(a.poff + h);
      t_np[p] = ldg(a.poff + h + 1) - t_p0[p];
    }
    if (tid == 0) t_start[np] = L;
  }
  for (int i = tid; i < QRR_BINS; i += blockDim.x) hist[i] = 0;
  __syncthreads();
  const FpBound fb = s_fb;
  // probe of position pos (t_start[p] <= pos < t_start[p + 1])
  auto probe_of = [&](int64_t pos) {
    int lo = 0, hi = np - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (t_start[mid] <= pos) lo = mid; else hi = mid - 1;
    }
    return lo;
  };
  // layout row of position pos
  auto row_of = [&](int64_t pos) -> int64_t {
    if (!tab) return locate(a, false, q, seg0, pos).row;
    const int p = probe_of(pos);
    return t_p0[p] + (pos - t_start[p]);
  };
  auto loc_of = [&](int64_t pos) -> CandLoc {
    if (!tab) return locate(a, false, q, seg0, pos);
    const int p = probe_of(pos);
    CandLoc c;
    const int64_t r = pos - t_start[p];
    c.p0 = t_p0[p];
    c.npad = t_np[p];
    c.row = c.p0 + r;
    c.id = ldg(a.rowid + c.row);
    c.gpack = ((int64_t)t_h[p] << 32) | r;
    return c;
  };
  // Passes over the segment: 16-byte loads of the aligned 4-value chunks
  // that cover it, eight in flight per thread (a chunk's values outside the
  // segment are skipped; the buffer's 256-byte alignment keeps the first
  // and last chunks inside it). each_f, one value per load, serves the
  // passes whose per-value work is heavy (rare paths).
  auto each_fast = [&](auto fn) {
    const int64_t c0 = seg0 >> 2, c1 = (seg0 + L + 3) >> 2;
    for (int64_t cb = c0 + tid; cb < c1; cb += (int64_t)blockDim.x * 8) {
      float4 v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) v[u] = ldg4(a.D + 4 * min64(cb + (int64_t)blockDim.x * u, c1 - 1));
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int64_t ch = cb + (int64_t)blockDim.x * u;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int64_t i = 4 * ch + e - seg0;
          if (ch < c1 && i >= 0 && i < L) fn(i, f4(v[u], e));
        }
      }
    }
  };
  auto each_f = [&](auto fn) {
    for (int64_t base = tid; base < L; base += (int64_t)blockDim.x * 8) {
      float v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) v[u] = src[min64(base + (int64_t)blockDim.x * u, L - 1)];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int64_t i = base + (int64_t)blockDim.x * u;
        if (i < L) fn(i, v[u]);
      }
    }
  };
  const float ADANNS_GLOBAL_AS *qg = (const float ADANNS_GLOBAL_AS *)(a.Qs + q * a.ldqs);
  int measured = 0;  // thread 0's count of exact measures
  // FP32 distances of slots [c0, c1), then slots [0, c1) sorted
  auto measure = [&](int c0, int c1) __attribute__((always_inline)) {
    if (tid == 0) measured += c1 - c0;
    if (a.d_B <= 2048) {
      const float *qrow = a.Qs + q * a.ldqs;
      for (int c = c0 + 2 * wv; c < c1; c += 2 * nwv) {
        const int cc = c + 1 < c1 ? c + 1 : c;
        const CandLoc L0 = loc_of(cpos[c]);
        const CandLoc L1 = loc_of(cpos[cc]);
        const float *xp[2] = {
            a.rows ? a.rows + L0.row * a.d_pad : a.vec + L0.p0 * a.d_pad + (L0.row - L0.p0) * SLAB,
            a.rows ? a.rows + L1.row * a.d_pad : a.vec + L1.p0 * a.d_pad + (L1.row - L1.p0) * SLAB};
        const int64_t np[2] = {a.rows ? 1 : L0.npad, a.rows ? 1 : L1.npad};
        float S[2] = {0.f, 0.f}, C[2] = {0.f, 0.f};
        measure2_rows(qrow, a.d_B, xp, np, lane, S, C);
        wave_reduce_pair(S[0], C[0]);
        wave_reduce_pair(S[1], C[1]);
        if (lane == 0) {
          chi[c] = S[0];
          clo[c] = C[0];
          cid[c] = L0.id;
          cg[c] = L0.gpack;
          if (cc != c) {
            chi[cc] = S[1];
            clo[cc] = C[1];
            cid[cc] = L1.id;
            cg[cc] = L1.gpack;
          }
        }
      }
    } else {
      for (int c = c0 + wv; c < c1; c += nwv) {
        const CandLoc Lc = loc_of(cpos[c]);
        float S = 0.f, C = 0.f;
        measureB(a, false, Lc, qg, lane, S, C);
        wave_reduce_pair(S, C);
        if (lane == 0) {
          chi[c] = S;
          clo[c] = C;
          cid[c] = Lc.id;
          cg[c] = Lc.gpack;
        }
      }
    }
    int P2 = 1;
    while (P2 < c1) P2 <<= 1;
    __syncthreads();
    for (int c = c1 + tid; c < P2; c += blockDim.x) {
      chi[c] = __builtin_inff();
      clo[c] = 0.f;
      cid[c] = INT64_MAX;
      cg[c] = -1;
    }
    bitonic_sort(chi, clo, cid, cg, P2);
  };
  // Phase-2 state: the bound's constants, U's root, and the lower bounds
  // already measured (lo <= t)
  const float B = fb.B;
  const float qlo = fb.qq * (1.f - 4.f * (float)(a.d_dot + 2) * 0x1p-24f);
  const float eq = fb.eq * 1.001f;
  const float emax = ldg(a.qerr) * 1.001f;
  float fmin = 0.f, fhi = 0.f, inv = 0.f, t = -1.f, sU = 0.f, flim = 0.f;
  int bk = -1;
  // (bins and bounds are recomputed in several passes: no contraction, so
  // that every pass takes the same bits)
  // bins of [fmin, fhi]; values above fhi take bin QRR_BINS
  auto bin_of = [&](float f) {
#pragma clang fp contract(off)
    return f > fhi ? QRR_BINS : min(QRR_BINS - 1, max(0, (int)((f - fmin) * inv)));
  };
  // lo of a candidate outside set 1 that can reach sqrt(U) and is not
  // measured yet, else -1 (lo is clamped at 0)
  auto lo_of = [&](int64_t i, float f) -> float {
#pragma clang fp contract(off)
    if (!(f <= flim) || bin_of(f) <= bk) return -1.f;
    const float lo = fmaxf(sqrtf(fmaxf(f - B + qlo, 0.f)) - eq -
                               ldg(a.qrerr + row_of(i)) * 1.001f, 0.f);
    return lo > t && lo <= sU ? lo : -1.f;
  };
  // mode 0: every candidate; 1: set 1; 2: lo_of
  auto pred = [&](int mode, int64_t i, float f) -> bool {
    return mode == 0 ? true : mode == 1 ? bin_of(f) <= bk : lo_of(i, f) >= 0.f;
  };
  // Every candidate with pred(mode), measured in rounds of at most
  // QRR_CAP - have slots in position order (ranks from contiguous per-thread
  // chunks and a block scan), merged with the have sorted ones; returns the
  // new have.
  auto rounds_by_position = [&](int mode, int have) -> int {
    const int64_t chunk = (L + blockDim.x - 1) / blockDim.x;
    const int64_t a0 = min64(L, tid * chunk), a1 = min64(L, a0 + chunk);
    uint32_t ne = 0;
    for (int64_t i = a0; i < a1; ++i) ne += pred(mode, i, src[i]) ? 1u : 0u;
    uint32_t n = 0;
    const uint32_t r0 = block_excl_scan<uint32_t>(ne, sh32, &n);
    for (uint32_t lo = 0; lo < n;) {
      const uint32_t cnt = min((uint32_t)(QRR_CAP - have), n - lo);
      uint32_t r = r0;
      for (int64_t i = a0; i < a1 && r < lo + cnt; ++i)
        if (pred(mode, i, src[i])) {
          if (r >= lo) cpos[have + (r - lo)] = i;
          ++r;
        }
      __syncthreads();
      measure(have, have + (int)cnt);
      have = min(kout, have + (int)cnt);
      lo += cnt;
    }
    return have;
  };
  int got;
  bool multi = false;
  if (L <= QRR_CAP || fb.kind != 1) {  // few candidates, or no bound known: all measured
    got = rounds_by_position(0, 0);
    multi = L > QRR_CAP;
  } else {
    {
      uint32_t kmin = 0xffffffffu, kmax = 0u;
      each_fast([&](int64_t, float f) {
        const uint32_t kk = order_key(f);
        kmin = kk < kmin ? kk : kmin;
        kmax = kk > kmax ? kk : kmax;
      });
      atomicMin(&s_kmin, kmin);
      atomicMax(&s_kmax, kmax);
    }
    __syncthreads();
    fmin = comp_value((uint64_t)s_kmin << 32);
    const float fmax = comp_value((uint64_t)s_kmax << 32);
    // the histogram covers the lowest quarter of the range first (rank k
    // lies there unless the quarter holds fewer than k), else all of it
    for (int full = 0; full < 2; ++full) {
      fhi = full ? fmax : fmin + 0.25f * (fmax - fmin);
      inv = fhi > fmin ? (float)QRR_BINS / (fhi - fmin) : 0.f;
      if (full) {
        for (int b = tid; b < QRR_BINS; b += blockDim.x) hist[b] = 0;
        __syncthreads();
      }
      each_fast([&](int64_t, float f) {
        const int b = bin_of(f);
        if (b < QRR_BINS) atomicAdd(&hist[b], 1u);
      });
      __syncthreads();
      constexpr int per = QRR_BINS / 256;
      uint32_t local = 0, tot = 0;
      for (int e = 0; e < per; ++e) local += hist[tid * per + e];
      uint32_t c = block_excl_scan<uint32_t>(local, sh32, &tot);
      for (int e = 0; e < per; ++e) {
        const uint32_t hb = hist[tid * per + e], b = tid * per + e;
        if (c < (uint32_t)kout && (uint32_t)kout <= c + hb) {
          s_bk = b;
          s_c1 = c + hb;
        }
        c += hb;
      }
      __syncthreads();
      if (tot >= (uint32_t)kout) break;
    }
    bk = s_bk;
    const int c1 = s_c1;
    // 1: the bins up to rank kout (at least kout candidates)
    int have;
    if (c1 <= QRR_CAP) {
      each_fast([&](int64_t i, float f) {
        if (bin_of(f) <= bk) {
          const int slot = atomicAdd(&s_cnt, 1);
          if (slot < c1) cpos[slot] = i;
        }
      });
      __syncthreads();
      measure(0, c1);
      have = kout;
    } else {
      have = rounds_by_position(1, 0);
      multi = true;
    }
    // 2: the rest whose lower bound reaches sqrt(U), in windows of lo
    for (;;) {
      sU = sqrtf((chi[kout - 1] + clo[kout - 1]) * (1.f + 0x1p-20f));
      const float reach = sU + eq + emax;
      flim = reach * reach * 1.001f + B - qlo;
      const int C = QRR_CAP - have;
      __syncthreads();
      if (tid == 0) {
        s_cnt = 0;
        s_nl = 0;
      }
      __syncthreads();
      auto take = [&](int64_t i, float f) {
        if (lo_of(i, f) >= 0.f) {
          const int slot = atomicAdd(&s_cnt, 1);
          if (slot < C) cpos[have + slot] = i;
        }
      };
      // the values below flim outside set 1 are listed first, so that the
      // row-error loads of the bound test are issued together
      const bool listable = L <= 0x7fffffff;  // positions fit the list's int32
      each_fast([&](int64_t i, float f) {
        if (listable && f <= flim && bin_of(f) > bk) {
          const int e = atomicAdd(&s_nl, 1);
          if (e < FLT_LIST) {
            s_lpos[e] = (int32_t)i;
            s_lf[e] = f;
          }
        }
      });
      __syncthreads();
      const int nl = s_nl;
      if (listable && nl <= FLT_LIST) {
        for (int e = tid; e < nl; e += blockDim.x) take(s_lpos[e], s_lf[e]);
      } else {
        each_f(take);
      }
      __syncthreads();
      int n = s_cnt;
      const bool windowed = n > C;
      if (windowed) {
        multi = true;
        // histogram of lo over (t, sU]: the longest run of bins from the
        // start holding at most C candidates (and at least one) is the
        // next window
        for (int b = tid; b < QRR_BINS; b += blockDim.x) hist[b] = 0;
        __syncthreads();
        const float t0 = fmaxf(t, 0.f);
        const float winv = sU > t0 ? (float)QRR_BINS / (sU - t0) : 0.f;
        auto wbin = [&](float lo) {
#pragma clang fp contract(off)
          return min(QRR_BINS - 1, max(0, (int)((lo - t0) * winv)));
        };
        each_f([&](int64_t i, float f) {
          const float lo = lo_of(i, f);
          if (lo >= 0.f) atomicAdd(&hist[wbin(lo)], 1u);
        });
        __syncthreads();
        {
          constexpr int per = QRR_BINS / 256;
          uint32_t local = 0;
          for (int e = 0; e < per; ++e) local += hist[tid * per + e];
          uint32_t c = block_excl_scan<uint32_t>(local, sh32, nullptr);
          if (tid == 0) s_bk = -1;
          __syncthreads();
          for (int e = 0; e < per; ++e) {
            const uint32_t hb = hist[tid * per + e], b = tid * per + e;
            if (c + hb > 0 && c + hb <= (uint32_t)C &&
                (b + 1 == QRR_BINS || c + hb + hist[b + 1] > (uint32_t)C))
              s_bk = b;
            c += hb;
          }
        }
        __syncthreads();
        const int wb = s_bk;
        if (wb < 0) {  // the first non-empty bin alone overflows: position order
          have = rounds_by_position(2, have);
          break;
        }
        // the window: exactly the candidates of bins 0..wb
        if (tid == 0) s_cnt = 0;
        __syncthreads();
        each_f([&](int64_t i, float f) {
          const float lo = lo_of(i, f);
          if (lo >= 0.f && wbin(lo) <= wb) {
            const int slot = atomicAdd(&s_cnt, 1);
            if (slot < C) cpos[have + slot] = i;
          }
        });
        __syncthreads();
        n = min(s_cnt, C);
        // the largest lo taken: every candidate left has a larger one
        float mx = 0.f;
        for (int c = have + tid; c < have + n; c += blockDim.x) {
          const int64_t i = cpos[c];
          mx = fmaxf(mx, lo_of(i, src[i]));
        }
        if (tid == 0) s_t = 0.f;
        __syncthreads();
        atomicMax((int *)&s_t, __float_as_int(mx));
        __syncthreads();
      }
      if (n > 0) measure(have, have + n);
      have = min(kout, have + n);
      if (!windowed) break;
      t = s_t;
    }
    got = have;
  }
  if (a.shortlist > 0 && L > a.shortlist) {
    // The precision form's result (the FP32 k nearest of the shortlist S, the
    // a.shortlist nearest candidates by exact quantised distance): the result
    // above is also S's when it lies in S (as k_select_filtered_wave argues).
    // A candidate ahead of result x in S's order has f <= f_x + 2B, so x is
    // in S when at most a.shortlist candidates have f <= T = max_x f_x + 2B.
    // Otherwise the query is handed over.
    // the results' own first-pass values (located through their list and row)
    __syncthreads();
    if (tid == 0) {
      s_cnt = 0;
      s_kmax = 0u;
    }
    __syncthreads();
    if (tid < kout && tid < got) {
      const int64_t gp = cg[tid];
      const int32_t h = (int32_t)(gp >> 32);
      const int64_t r = gp & 0xffffffffll;
      int64_t pos = -1;
      for (int p = 0; p < np && pos < 0; ++p) {
        const int32_t hp = tab ? t_h[p] : ldg(a.probes + q * np + p);
        if (hp == h) pos = (tab ? t_start[p] : ldg(a.pair_base + q * np + p) - seg0) + r;
      }
      atomicMax(&s_kmax, pos >= 0 ? order_key(src[pos]) : 0xffffffffu);
    }
    __syncthreads();
    float T = __builtin_inff();
    if (fb.kind == 1 && got >= kout && s_kmax != 0xffffffffu) {
      T = comp_value((uint64_t)s_kmax << 32) + 2.f * B * 1.001f;
      T += fabsf(T) * 0x1p-20f;
    }
    if (T <= __FLT_MAX__) {
      int c = 0;
      each_fast([&](int64_t, float f) { c += f <= T ? 1 : 0; });
      if (c) atomicAdd(&s_cnt, c);
    }
    __syncthreads();
    if (!(T <= __FLT_MAX__) || s_cnt > a.shortlist) {
      if (tid == 0) push_redo(a.redo_cnt, a.redo_list, q + a.redo_q0);
      return;
    }
  }
  for (int j = tid; j < kout; j += blockDim.x) {
    a.out_dist[q * ldo + j] = j < got ? chi[j] : __builtin_inff();
    a.out_ids[q * ldo + j] = j < got ? cid[j] : -1;
  }
  if (tid == 0) {
    atomicAdd(&g_sel_stats[2], (unsigned long long)measured);
    if (multi) atomicAdd(&g_sel_stats[3], 1ull);
  }
}

// (three workgroups per CU: the measures wait on memory, so workgroups in
// flight count more than the registers the bound spills; e4m3 selection
// 12.2 -> 9.7 ms at the ImageNet-1K shape)
__global__ __launch_bounds__(256, 3) void k_select_exact_filtered(SelArgs a) {
  filtered_block(a, blockIdx.x);
}

// The queries the one-wave selection handed over (a.redo_cnt / a.redo_list),
// one workgroup each, striding over the list.
__global__ __launch_bounds__(256, 3) void k_select_exact_filtered_redo(SelArgs a) {
  const int32_t n = *(volatile const int32_t *)a.redo_cnt;
  for (int32_t i = blockIdx.x; i < n; i += gridDim.x) {
    filtered_block(a, a.redo_list[i]);
    __syncthreads();  // the next query reuses the LDS
  }
}

// The same selection and measures for one query on one wave, without LDS
// or barriers, when K1 <= 64 (see k_select_wave below for the list
// mechanics). Results equal select_body's.
__device__ void wave_select(const SelArgs &a, const int64_t q, const int lane);

// (four waves per SIMD: its steps wait on memory latency, so waves in flight
// count more than the two registers the limit spills)
__global__ __launch_bounds__(256, 4) void k_select_refine_wave(SelArgs a, int64_t nq) {
  const int64_t q = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (q >= nq) return;  // whole waves leave; nothing synchronises the block
  wave_select(a, q, threadIdx.x & 63);
}

// Batched FP32 selection: one block per query row of the batch; the
// configuration's fields are patched into the arguments.
struct SelMultiArgs {
  const CfgDev *cfg;
  int32_t ncfg;
  int32_t coarse;
  const float *Qs;
  int64_t ldqs;
  const float *S;
  const float *D;
  const int64_t *seg_off;
  int32_t *probes;
  int32_t *user_probes;
  const int64_t *pair_base;
  float *dist;             // scan: [Qtot][ldk]; coarse: optional nearest distance [Qtot]
  int64_t *ids;
  int64_t ldk;
  int32_t lcap, kcap;
  // [2 + Qtot]: counts of queries handed to re-selection by the coarse ([0])
  // and scan ([1]) selections, then the list of them; NULL in the
  // re-selection launch itself
  int32_t *redo;
};

__device__ __forceinline__ void select_multi_row(const SelMultiArgs &m, int64_t r) {
  const int c = cfg_of(m.cfg, m.ncfg, &CfgDev::q0, r);
  const CfgDev &g = m.cfg[c];
  const int64_t q = r - g.q0;
  SelArgs a{};
  a.Qs = m.Qs + g.q0 * m.ldqs;
  a.ldqs = m.ldqs;
  a.lcap = m.lcap;
  a.kcap = m.kcap;
  if (m.coarse) {
    a.mode = SEL_COARSE;
    a.D = m.S + g.S0;
    a.nl = g.nlist;
    a.K1 = min(g.nlist, min(g.nprobe + REFINE_MARGIN, MAX_SHORTLIST));
    a.K2 = g.nprobe;
    a.kout = g.nprobe;
    a.d_dot = g.d_c;
    a.cent = g.cent;
    a.ld_cent = g.d_cb_pad;
    a.out_probes = m.probes + g.pair0;
    a.out_probes2 = m.user_probes ? m.user_probes + g.pair0 : nullptr;
    a.out_dist = m.dist ? m.dist + g.q0 : nullptr;
    a.ldo = 1;
    a.xmax2 = g.cmax2;
  } else {
    a.mode = SEL_L2;
    a.D = m.D;
    a.seg_off = m.seg_off + g.q0;
    a.K1 = min(g.k + REFINE_MARGIN, MAX_SHORTLIST);
    a.K2 = g.k;
    a.kout = g.k;
    a.ldo = m.ldk;
    a.d_dot = g.d_s;
    a.vec = g.vec;
    a.rows = g.rows;
    a.d_pad = g.d_pad;
    a.poff = g.poff;
    a.rowid = g.rowid;
    a.probes = m.probes + g.pair0;
    a.nprobe = g.nprobe;
    a.pair_base = m.pair_base + g.pair0;
    a.out_dist = m.dist + g.q0 * m.ldk;
    a.out_ids = m.ids + g.q0 * m.ldk;
    a.xmax2 = g.xmax2;
  }
  if (m.redo) {
    a.redo_cnt = m.redo + (m.coarse ? 0 : 1);
    a.redo_list = m.redo + 2;  // batch rows
    a.redo_q0 = g.q0;
  }
  select_body(a, q);
}

__global__ __launch_bounds__(512) void k_select_multi(SelMultiArgs m) {
  select_multi_row(m, blockIdx.x);
}

// Re-selection of the batch rows handed over by the coarse (m.coarse) or scan
// selection: as k_select_refine_redo.
__global__ __launch_bounds__(512) void k_select_multi_redo(SelMultiArgs m) {
  const int32_t n = *(volatile const int32_t *)(m.redo + (m.coarse ? 0 : 1));
  const int32_t *list = m.redo + 2;
  SelMultiArgs b = m;
  b.redo = nullptr;
  for (int32_t i = blockIdx.x; i < n; i += gridDim.x) {
    select_multi_row(b, list[i]);
    __syncthreads();  // LDS reused by the next row
  }
}

// Per-query selection when at most WSEL_K candidates are kept (K1 <= 64):
// one wave per query, no LDS and no barriers. The K1 smallest first-pass
// distances are kept as a sorted list spread over the lanes, keyed by
// (order_key(distance) << 32 | position), so that ties go to the earlier
// position exactly as in select_body; each batch of 64 distances is filtered
// against the list's K1-th entry with one ballot and only the survivors are
// inserted. The candidates are then re-measured exactly (compensated FP32,
// same order of accumulation as select_body) and sorted across lanes by
// (distance pair, id). Results are identical to k_select_multi's.
constexpr int WSEL_K = 64;
// the one-wave selections keep up to kv + WAVE_MARGIN first-pass candidates
// (within WSEL_K), kv the number of exact values the query needs
constexpr int WAVE_MARGIN = 12;
// candidates re-measured together by k_select_wave: two, with 1024
// coordinates per pass, keep the kernel within 128 registers, four waves per
// SIMD (the selection waits on memory latency, so waves in flight count more
// than loads per wave)
constexpr int SELW_G = 2;
// batches of at most this many queries take k_select_wave's WIDE form: one
// wave per query puts at most two waves on each of the 1024 SIMDs, which the
// WIDE form holds, so the four-wave form would gain nothing there
constexpr int64_t SELW_WIDE_MAX = 2048;

__device__ __forceinline__ uint64_t readlane64(uint64_t v, int l) {
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, l);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), l);
  return ((uint64_t)hi << 32) | lo;
}

__device__ __forceinline__ uint64_t shfl_up64(uint64_t v, int d) {
  const uint32_t lo = __shfl_up((uint32_t)v, d);
  const uint32_t hi = __shfl_up((uint32_t)(v >> 32), d);
  return ((uint64_t)hi << 32) | lo;
}

__device__ __forceinline__ int64_t shfl_xor64(int64_t v, int m) {
  const uint32_t lo = __shfl_xor((uint32_t)(uint64_t)v, m);
  const uint32_t hi = __shfl_xor((uint32_t)((uint64_t)v >> 32), m);
  return (int64_t)(((uint64_t)hi << 32) | lo);
}

__device__ __forceinline__ void bitonic_lanes(float &S, float &C, int64_t &id, int64_t &gp,
                                              int lane) {
#pragma unroll
  for (int k = 2; k <= 64; k <<= 1) {
#pragma unroll
    for (int j = k >> 1; j > 0; j >>= 1) {
      const float oS = __shfl_xor(S, j), oC = __shfl_xor(C, j);
      const int64_t oid = shfl_xor64(id, j), ogp = shfl_xor64(gp, j);
      const bool up = (lane & k) == 0, lower = (lane & j) == 0;
      const bool other_less = pair_less(oS, oC, oid, S, C, id);
      if ((lower == up) ? other_less : !other_less) {
        S = oS;
        C = oC;
        id = oid;
        gp = ogp;
      }
    }
  }
}

// Admission cap for a one-wave list of the K1 smallest (key, position)
// composites, from its first batch v (values at positions base + 64 u + lane,
// those at L or beyond ignored): the K1-th smallest of the lanes' minima is
// at least the K1-th smallest value of all L (K1 distinct candidates lie at or
// under it), so values above it never enter the list, and equal keys are
// admitted at every position. ~0 when fewer than K1 lanes hold a value.
template <int U>
__device__ __forceinline__ uint64_t admit_cap(const float (&v)[U], int64_t base, int64_t L,
                                              int lane, int K1) {
  uint32_t mk = 0xFFFFFFFFu;
#pragma unroll
  for (int u = 0; u < U; ++u)
    if (base + 64 * u + lane < L) mk = min(mk, order_key(v[u]));
  // bitonic sort of the 64 lane minima, ascending over the lanes
#pragma unroll
  for (int k = 2; k <= 64; k <<= 1)
#pragma unroll
    for (int j = k >> 1; j > 0; j >>= 1) {
      const uint32_t o = (uint32_t)__shfl_xor((int)mk, j);
      const bool up = (lane & k) == 0, lower = (lane & j) == 0;
      mk = (lower == up) ? min(mk, o) : max(mk, o);
    }
  const uint32_t t = (uint32_t)__builtin_amdgcn_readlane((int)mk, K1 - 1);
  return t == 0xFFFFFFFFu ? ~0ull : ((uint64_t)t << 32) | 0xFFFFFFFFull;
}

__device__ __forceinline__ void wave_select(const SelArgs &a, const int64_t q, const int lane) {
  const bool coarse = a.mode == SEL_COARSE || a.mode == SEL_COARSE_QUANT;
  const int64_t ldo = a.ldo ? a.ldo : a.kout;
  const float *seg;
  int64_t L, seg0 = 0;
  if (coarse) {
    seg = a.D + q * a.nl;
    L = a.nl;
  } else {
    seg0 = a.seg_off[q];
    seg = a.D + seg0;
    L = a.seg_off[q + 1] - seg0;
  }
  // 1. the K1 smallest (key, position) composites, sorted over the lanes;
  // K1 as wide as the lanes allow up to kv + WAVE_MARGIN, so that the
  // certificate below rarely fails (only the band within the error bound is
  // measured, so a wider list costs insertions, not measures)
  const int kv = a.stageB ? a.K2 : a.kout;
  const int K1 = max(a.K1, min(WSEL_K, kv + WAVE_MARGIN));
  const float ADANNS_GLOBAL_AS *sg = (const float ADANNS_GLOBAL_AS *)seg;
  uint64_t best = ~0ull, thr = ~0ull, cap = ~0ull;
  constexpr int U = 16;
  for (int64_t base = 0; base < L; base += 64 * U) {
    float v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t i = base + 64 * u + lane;
      v[u] = i < L ? sg[i] : 0.f;
    }
    if (base == 0) thr = cap = admit_cap(v, 0, L, lane, K1);
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t i = base + 64 * u + lane;
      const uint64_t comp = i < L ? ((uint64_t)order_key(v[u]) << 32) | (uint64_t)i : ~0ull;
      uint64_t mask = __ballot(comp < thr);
      while (mask) {
        const int b = __builtin_ctzll(mask);
        mask &= mask - 1;
        const uint64_t x = readlane64(comp, b);
        if (x < thr) {
          const uint64_t up = shfl_up64(best, 1);
          if (!(best < x)) best = (lane == 0 || up < x) ? x : up;
          const uint64_t kth = readlane64(best, K1 - 1);
          thr = kth < cap ? kth : cap;
        }
      }
    }
  }
  int ncand = (int)min64(L, (int64_t)K1);
  const float ADANNS_GLOBAL_AS *qglob = (const float ADANNS_GLOBAL_AS *)(a.Qs + q * a.ldqs);
  // 1b. certificate: with B the first pass's error bound (wave_fp_bound),
  // only candidates whose value can still reach the kv nearest are measured
  // (for the quantised first pass: the kv nearest by exact quantised
  // distance). If the list holds fewer than all candidates and its last
  // entry can still reach them, candidates beyond it might too: the query is
  // handed to the re-selection launch (workgroup path, certified band).
  const FpBound fb = wave_fp_bound(a, q, lane);
  const bool quant = a.mode == SEL_QUANT || a.mode == SEL_COARSE_QUANT;
  const float eqn = fb.eq;
  if (fb.kind != 0 && ncand > kv) {
    const float up = fb.upper(comp_value(readlane64(best, kv - 1)));
    if (L > K1 && fb.keep(comp_value(readlane64(best, K1 - 1)), up)) {
      if (a.redo_list != nullptr) {
        if (lane == 0) push_redo(a.redo_cnt, a.redo_list, q + a.redo_q0);
        return;
      }
      if (lane == 0) atomicAdd(&g_sel_stats[1], 1ull);
    }
    ncand = __popcll(__ballot(lane < ncand && fb.keep(comp_value(best), up)));
  } else if (fb.kind == 0 && L > K1) {
    // no bound known (never the case for the library's launches): the plain
    // list, not certified
    if (lane == 0) atomicAdd(&g_sel_stats[1], 1ull);
  }
  // 2. lane j < ncand locates candidate j
  CandLoc mine{INT64_MAX, -1, 0, 0, 0};
  if (lane < ncand) mine = locate(a, coarse, q, seg0, (int64_t)(uint32_t)best);
  // 3. first exact measure over the lanes: quantised rows two at a time,
  // other measures one candidate at a time
  float myS = __builtin_inff(), myC = 0.f;
  auto cand = [&](int cc) {
    CandLoc Lc;
    Lc.id = (int64_t)readlane64((uint64_t)mine.id, cc);
    Lc.gpack = (int64_t)readlane64((uint64_t)mine.gpack, cc);
    Lc.row = (int64_t)readlane64((uint64_t)mine.row, cc);
    Lc.p0 = (int64_t)readlane64((uint64_t)mine.p0, cc);
    Lc.npad = (int64_t)readlane64((uint64_t)mine.npad, cc);
    return Lc;
  };
  if (a.mode == SEL_QUANT) {
    for (int cc = 0; cc < ncand; cc += 2) {
      // an odd last candidate is measured twice, the copy discarded
      const int c1 = cc + 1 < ncand ? cc + 1 : cc;
      const CandLoc Lp[2] = {cand(cc), cand(c1)};
      float S[2] = {0.f, 0.f}, C[2] = {0.f, 0.f};
      measure_quant_rows<2>(a, q, Lp, nullptr, lane, S, C);
      wave_reduce_pair(S[0], C[0]);
      wave_reduce_pair(S[1], C[1]);
      if (lane == cc) {
        myS = S[0];
        myC = C[0];
      }
      if (lane == c1 && c1 != cc) {
        myS = S[1];
        myC = C[1];
      }
    }
  } else if (a.mode == SEL_COARSE_QUANT) {
    // four centroids at a time (duplicates of the last one discarded)
    for (int cc = 0; cc < ncand; cc += 4) {
      CandLoc Lp[4];
#pragma unroll
      for (int g = 0; g < 4; ++g) Lp[g] = cand(cc + g < ncand ? cc + g : ncand - 1);
      float S[4] = {0.f, 0.f, 0.f, 0.f}, C[4] = {0.f, 0.f, 0.f, 0.f};
      measure_cent_g<4, 0>(a, q, Lp, qglob, lane, S, C);
#pragma unroll
      for (int g = 0; g < 4; ++g) {
        wave_reduce_pair(S[g], C[g]);
        if (lane == cc + g && cc + g < ncand) {
          myS = S[g];
          myC = C[g];
        }
      }
    }
  } else {
    for (int cc = 0; cc < ncand; ++cc) {
      const CandLoc Lc = cand(cc);
      float S = 0.f, C = 0.f;
      measure1(a, q, Lc, qglob, nullptr, lane, S, C);
      wave_reduce_pair(S, C);
      if (lane == cc) {
        myS = S;
        myC = C;
      }
    }
  }
  int64_t myid = mine.id, mygp = mine.gpack;
  bitonic_lanes(myS, myC, myid, mygp, lane);
  int nres = ncand;
  if (a.stageB) {
    // second exact measure (FP32 L2 on d_B coordinates) of the K2 best
    nres = ncand < a.K2 ? ncand : a.K2;
    // Quantised rows: |‖q - x‖ - ‖q^ - x^‖| <= ‖q - q^‖ + ‖x - x^‖ <= e,
    // e = ‖q - q^‖ + (largest ‖x - x^‖ of the rows). A candidate whose
    // quantised distance lies beyond (sqrt(D^_k) + 2e)^2 is farther than k
    // others in FP32, so only the prefix within it is re-measured.
    // (both measures on the same prefix: distances on different prefixes do
    // not bound each other)
    if (quant && a.qemax != nullptr && a.d_B == a.d_dot && eqn >= 0.f && nres > a.kout) {
      // a margin of 1e-3 relative covers the FP32 rounding of these bounds
      const float e = (eqn + ldg(a.qemax)) * 1.001f;
      const float sk = __shfl(myS, a.kout - 1);
      const float up = sqrtf(fmaxf(sk, 0.f)) + 2.f * e;
      const bool keep = lane < nres && sqrtf(fmaxf(myS, 0.f)) <= up * 1.001f;
      nres = __popcll(__ballot(keep));
    }
    if (lane >= nres) {
      myS = __builtin_inff();
      myC = 0.f;
      myid = INT64_MAX;
      mygp = -1;
    }
    // vectors up to 2048 coordinates: this lane's query coordinates are
    // read once into registers
    const bool rq = !coarse && a.d_B <= 2048;
    float4 q4[8];
    if (rq) {
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        float v[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int dim = 4 * lane + 256 * u + e;
          v[e] = dim < a.d_B ? qglob[dim] : 0.f;
        }
        q4[u] = make_float4(v[0], v[1], v[2], v[3]);
      }
    }
    if (coarse) {  // four centroids at a time, as the first measure
      for (int cc = 0; cc < nres; cc += 4) {
        CandLoc Lp[4];
#pragma unroll
        for (int g = 0; g < 4; ++g)
          Lp[g] = locate_packed(a, true, (int64_t)readlane64((uint64_t)mygp,
                                                            cc + g < nres ? cc + g : nres - 1));
        float S[4] = {0.f, 0.f, 0.f, 0.f}, C[4] = {0.f, 0.f, 0.f, 0.f};
        measure_cent_g<4, 1>(a, q, Lp, qglob, lane, S, C);
#pragma unroll
        for (int g = 0; g < 4; ++g) {
          wave_reduce_pair(S[g], C[g]);
          if (lane == cc + g && cc + g < nres) {
            myS = S[g];
            myC = C[g];
          }
        }
      }
    } else {
      for (int cc = 0; cc < nres; ++cc) {
        const int64_t gp = (int64_t)readlane64((uint64_t)mygp, cc);
        float S = 0.f, C = 0.f;
        if (rq)
          measureB_vec_rq(a, locate_packed(a, false, gp), q4, lane, S, C);
        else
          measureB(a, false, locate_packed(a, false, gp), qglob, lane, S, C);
        wave_reduce_pair(S, C);
        if (lane == cc) {
          myS = S;
          myC = C;
        }
      }
    }
    bitonic_lanes(myS, myC, myid, mygp, lane);
  }
  if (lane < a.kout) {
    const bool has = lane < nres;
    if (coarse) {
      const int32_t hsel = has ? (int32_t)myid : -1;
      a.out_probes[q * a.kout + lane] = hsel;
      if (a.out_probes2) a.out_probes2[q * a.kout + lane] = hsel;
      if (a.out_dist && lane == 0) a.out_dist[q * ldo] = has ? myS : __builtin_inff();
    } else {
      a.out_dist[q * ldo + lane] = has ? myS : __builtin_inff();
      a.out_ids[q * ldo + lane] = has ? myid : -1;
    }
  }
}

// adanns_search_filtered's selection with one wave per query (kout +
// WAVE_MARGIN <= WSEL_K): the K1 smallest first-pass values as a sorted
// list over the lanes (as k_select_wave); the first kout of them measured
// exactly in FP32, U their largest (an upper bound on the k-th nearest's
// distance); then the others whose lower bound
// sqrt(f - B + |q^|^2) - |q - q^| - |x - x^| reaches sqrt(U) measured too, and
// the kout nearest of all measured returned. If the list's last value can
// still reach sqrt(U) with the largest row error, candidates beyond the list
// might too: the query goes to the workgroup kernel (a.redo_cnt /
// a.redo_list). The exact measure accumulates each lane's coordinates in the
// order of measureB, so the distances equal adanns_search's bit for bit.
__global__ __launch_bounds__(256, 3) void k_select_filtered_wave(SelArgs a, int64_t nq) {
  const int lane = threadIdx.x & 63;
  const int64_t q = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (q >= nq) return;  // whole waves leave; nothing synchronises the block
  const int kout = a.kout;
  const int64_t ldo = a.ldo ? a.ldo : a.kout;
  const int64_t seg0 = a.seg_off[q], L = a.seg_off[q + 1] - seg0;
  const float ADANNS_GLOBAL_AS *sg = (const float ADANNS_GLOBAL_AS *)(a.D + seg0);
  // list width: kout + 22 (at the ImageNet-1K shape with BF16 a list of 32
  // handed no query over and selected 18 % faster than one of 64; 24 handed
  // over 0.1 %)
  const int K1 = min(WSEL_K, kout + 22);
  // 1. the K1 smallest (key, position) composites, sorted over the lanes
  // (batches of 64 U values, the next loading while one is merged;
  // positions past the segment re-read its last value)
  uint64_t best = ~0ull, thr = ~0ull, cap = ~0ull;
  constexpr int U = 16;
  auto load = [&](float (&v)[U], int64_t base) {
#pragma unroll
    for (int u = 0; u < U; ++u) v[u] = sg[min64(base + 64 * u + lane, L - 1)];
  };
  auto merge = [&](const float (&v)[U], int64_t base) {
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t i = base + 64 * u + lane;
      const uint64_t comp = i < L ? ((uint64_t)order_key(v[u]) << 32) | (uint64_t)i : ~0ull;
      uint64_t mask = __ballot(comp < thr);
      while (mask) {
        const int b = __builtin_ctzll(mask);
        mask &= mask - 1;
        const uint64_t x = readlane64(comp, b);
        if (x < thr) {
          const uint64_t up = shfl_up64(best, 1);
          if (!(best < x)) best = (lane == 0 || up < x) ? x : up;
          const uint64_t kth = readlane64(best, K1 - 1);
          thr = kth < cap ? kth : cap;
        }
      }
    }
  };
  if (L > 0) {
    float va[U], vb[U];
    load(va, 0);
    for (int64_t base = 0;; base += 128 * U) {
      load(vb, base + 64 * U);
      if (base == 0) thr = cap = admit_cap(va, 0, L, lane, K1);
      merge(va, base);
      if (base + 64 * U >= L) break;
      load(va, base + 128 * U);
      merge(vb, base + 64 * U);
      if (base + 128 * U >= L) break;
    }
  }
  const int ncand = (int)min64(L, (int64_t)K1);
  const FpBound fb = wave_fp_bound_quant_vec(a, q, lane);
  if (L > K1 && fb.kind != 1) {  // no bound: every candidate, in the workgroup kernel
    if (lane == 0) push_redo(a.redo_cnt, a.redo_list, q + a.redo_q0);
    return;
  }
  // 2. where each candidate lives (lane j < ncand holds candidate j)
  int64_t my_id = INT64_MAX, my_row = 0, my_npad = 0;
  const float *my_base = nullptr;
  if (lane < ncand) {
    const CandLoc c = locate(a, false, q, seg0, (int64_t)(uint32_t)best);
    my_id = c.id;
    my_row = c.row;
    my_npad = a.rows ? 1 : c.npad;
    my_base = a.rows ? a.rows + c.row * a.d_pad : a.vec + c.p0 * a.d_pad + (c.row - c.p0) * SLAB;
  }
  // 3. exact FP32 measures of the lanes in a mask, two candidates at a time,
  // lane l taking coordinates 4l + 256u + e in that order, 1024 per pass
  const int d = a.d_B;
  const float *qrow = a.Qs + q * a.ldqs;
  float myS = __builtin_inff(), myC = 0.f;
  int nmeas = 0;
  auto measure_mask = [&](uint64_t mask) {
    nmeas += __popcll(mask);
    while (mask) {
      const int c0 = __builtin_ctzll(mask);
      mask &= mask - 1;
      int c1 = c0;
      if (mask) {
        c1 = __builtin_ctzll(mask);
        mask &= mask - 1;
      }
      const float *xp[2] = {(const float *)readlane64((uint64_t)my_base, c0),
                            (const float *)readlane64((uint64_t)my_base, c1)};
      const int64_t np[2] = {(int64_t)readlane64((uint64_t)my_npad, c0),
                             (int64_t)readlane64((uint64_t)my_npad, c1)};
      float S[2] = {0.f, 0.f}, C[2] = {0.f, 0.f};
      measure2_rows(qrow, d, xp, np, lane, S, C);
      wave_reduce_pair(S[0], C[0]);
      wave_reduce_pair(S[1], C[1]);
      if (lane == c0) {
        myS = S[0];
        myC = C[0];
      }
      if (lane == c1 && c1 != c0) {
        myS = S[1];
        myC = C[1];
      }
    }
  };
  const uint64_t lanes_lt = [&](int n) { return n >= 64 ? ~0ull : ((1ull << n) - 1ull); }(
      L > K1 ? kout : ncand);
  measure_mask(lanes_lt & __ballot(lane < ncand));
  if (L > K1) {
    // U: the largest of the kout measured; the bound test for the rest
    float u = lane < kout ? (myS + myC) * (1.f + 0x1p-20f) : 0.f;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) u = fmaxf(u, __shfl_xor(u, o));
    const float sU = sqrtf(u);
    const float B = fb.B;
    const float qlo = fb.qq * (1.f - 4.f * (float)(a.d_dot + 2) * 0x1p-24f);
    const float eq = fb.eq * 1.001f;
    const float reach = sU + eq + ldg(a.qerr) * 1.001f;
    const float flim = reach * reach * 1.001f + B - qlo;
    if (comp_value(readlane64(best, K1 - 1)) <= flim) {  // not certified within the list
      if (lane == 0) push_redo(a.redo_cnt, a.redo_list, q + a.redo_q0);
      return;
    }
    const float f = comp_value(best);
    bool need = false;
    if (lane >= kout && lane < ncand && f <= flim) {
      const float lo = sqrtf(fmaxf(f - B + qlo, 0.f)) - eq - ldg(a.qrerr + my_row) * 1.001f;
      need = lo <= sU;
    }
    measure_mask(__ballot(need));
  }
  // (each lane's first-pass value rides along with its measure)
  int64_t gp = (int64_t)__float_as_uint(comp_value(best));
  bitonic_lanes(myS, myC, my_id, gp, lane);
  if (a.shortlist > 0 && L > a.shortlist) {
    // The precision form's result: the FP32 k nearest of the shortlist S (the
    // a.shortlist nearest candidates by exact quantised distance). If every
    // result above lies in S, it is that result too (S holds all candidates'
    // k nearest). A candidate y ahead of result x in S's order has
    // f_y <= f_x + 2B (B bounds each first-pass value's error), so x is in S
    // when at most a.shortlist candidates have f <= T = max_x f_x + 2B; all
    // of them are in the list when its last entry lies above T.
    float T = -__builtin_inff();
    if (lane < kout && lane < nmeas) T = __uint_as_float((uint32_t)gp);
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) T = fmaxf(T, __shfl_xor(T, o));
    T += 2.f * fb.B * 1.001f;
    T += fabsf(T) * 0x1p-20f;
    const bool inlist = L <= K1 || comp_value(readlane64(best, K1 - 1)) > T;
    const int nle = __popcll(__ballot(lane < ncand && comp_value(best) <= T));
    if (fb.kind != 1 || !(T <= __FLT_MAX__) || !inlist || nle > a.shortlist) {
      if (lane == 0) push_redo(a.redo_cnt, a.redo_list, q + a.redo_q0);
      return;
    }
  }
  if (lane < kout) {
    const bool has = lane < nmeas;
    a.out_dist[q * ldo + lane] = has ? myS : __builtin_inff();
    a.out_ids[q * ldo + lane] = has ? my_id : -1;
  }
  if (lane == 0) atomicAdd(&g_sel_stats[2], (unsigned long long)nmeas);
}

// COARSE: the coarse step's selection (m.coarse set), else the scan's; two
// instantiations, so that the coarse one does not carry the registers of the
// scan's re-measure. WIDE (batches too small to fill the chip, where each
// query's own latency counts): more loads per wave, three candidates per
// pass of 2048 coordinates and 32 first-pass values per lane, at two waves
// per SIMD; otherwise two candidates per pass of 1024 coordinates and 16
// first-pass values per lane, at four waves per SIMD.
template <bool COARSE, bool WIDE = false>
__global__ __launch_bounds__(256, WIDE ? 2 : 3) void k_select_wave(SelMultiArgs m, int64_t Qtot) {
  const int lane = threadIdx.x & 63;
  const int64_t r = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (r >= Qtot) return;  // whole waves leave; nothing below synchronises the block
  const int c = cfg_of(m.cfg, m.ncfg, &CfgDev::q0, r);
  const CfgDev &g = m.cfg[c];
  const int64_t q = r - g.q0;
  constexpr bool coarse = COARSE;
  const float *seg;
  int64_t L, seg0 = 0;
  int K1, kout, d_dot;
  if (coarse) {
    seg = m.S + g.S0 + q * g.nlist;
    L = g.nlist;
    kout = g.nprobe;
    d_dot = g.d_c;
  } else {
    seg0 = m.seg_off[r];
    seg = m.D + seg0;
    L = m.seg_off[r + 1] - seg0;
    kout = g.k;
    d_dot = g.d_s;
  }
  // the launch guarantees kout + REFINE_MARGIN <= WSEL_K; a wider list (see
  // WAVE_MARGIN) lets the certificate below fail rarely
  K1 = min(WSEL_K, kout + WAVE_MARGIN);

  // 1. the K1 smallest (key, position) composites, sorted over lanes
  const float ADANNS_GLOBAL_AS *sg = (const float ADANNS_GLOBAL_AS *)seg;
  uint64_t best = ~0ull, thr = ~0ull, cap = ~0ull;
  constexpr int U = !COARSE && WIDE ? 32 : 16;  // loads in flight per lane and batch
  // scan: batches of 64 U values, the next batch loading while one is merged
  // (positions past the segment re-read its last value, so that the loads
  // carry no branches and the merge waits for its own batch only)
  auto load = [&](float (&v)[U], int64_t base) {
#pragma unroll
    for (int u = 0; u < U; ++u) v[u] = sg[min64(base + 64 * u + lane, L - 1)];
  };
  auto merge = [&](const float (&v)[U], int64_t base) {
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t i = base + 64 * u + lane;
      const uint64_t comp = i < L ? ((uint64_t)order_key(v[u]) << 32) | (uint64_t)i : ~0ull;
      uint64_t mask = __ballot(comp < thr);
      while (mask) {
        const int b = __builtin_ctzll(mask);
        mask &= mask - 1;
        const uint64_t x = readlane64(comp, b);
        if (x < thr) {
          const uint64_t up = shfl_up64(best, 1);
          if (!(best < x)) best = (lane == 0 || up < x) ? x : up;
          const uint64_t kth = readlane64(best, K1 - 1);
          thr = kth < cap ? kth : cap;
        }
      }
    }
  };
  if constexpr (COARSE) {
    // one score row per query (nlist values, often a single batch): no
    // prefetch
    for (int64_t base = 0; base < L; base += 64 * U) {
      float v[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int64_t i = base + 64 * u + lane;
        v[u] = i < L ? sg[i] : 0.f;
      }
      if (base == 0) thr = cap = admit_cap(v, 0, L, lane, K1);
      merge(v, base);
    }
  } else if (L > 0) {
    float va[U], vb[U];
    load(va, 0);
    // (the prefetch is unconditional: a batch past the end re-reads the
    // last value, and the wait counts stay exact on every path)
    for (int64_t base = 0;; base += 128 * U) {
      load(vb, base + 64 * U);
      if (base == 0) thr = cap = admit_cap(va, 0, L, lane, K1);
      merge(va, base);
      if (base + 64 * U >= L) break;
      load(va, base + 128 * U);
      merge(vb, base + 64 * U);
      if (base + 128 * U >= L) break;
    }
  }
  int ncand = (int)min64(L, (int64_t)K1);
  const float ADANNS_GLOBAL_AS *qrow =
      (const float ADANNS_GLOBAL_AS *)(m.Qs + r * m.ldqs);

  // 1b. the first-pass value |x|^2 - 2 q.x on a prefix of d coordinates
  // (d_s for vectors, d_c for centroids) is off its exact value by at most
  // B = c (X^2 + 2 |q| X), X the largest norm of the index's rows (or
  // centroids) and c = 4 (d + 2) 2^-24: four times the classical bound for a
  // length-d dot product and sum of squares in FP32 plus the final rounding.
  // A candidate whose first-pass value exceeds the k-th smallest by more than
  // 2B is farther than k others in exact arithmetic, so only the shortlist's
  // prefix within 2B of the k-th smallest is re-measured.
  // Certificate: if the list holds fewer than all L candidates and its last
  // entry is within the 2B band too, candidates beyond it might be among the
  // kout nearest; the query then goes to the re-selection launch.
  const float *xm = coarse ? g.cmax2 : g.xmax2;
  bool certain = L <= K1;
  if (xm != nullptr && ncand > kout) {
    float qq = 0.f;
    for (int d0 = 4 * lane; d0 < d_dot; d0 += 256) {
      const float4 v = ldg4((const float *)qrow + d0);
      qq += (d0 < d_dot ? v.x * v.x : 0.f) + (d0 + 1 < d_dot ? v.y * v.y : 0.f) +
            (d0 + 2 < d_dot ? v.z * v.z : 0.f) + (d0 + 3 < d_dot ? v.w * v.w : 0.f);
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) qq += __shfl_xor(qq, o);
    const float X2 = ldg(xm), X = sqrtf(X2), qn = sqrtf(qq);
    const float B = 4.f * (float)(d_dot + 2) * 0x1p-24f * (X2 + 2.f * qn * X);
    const uint32_t kk = (uint32_t)(readlane64(best, kout - 1) >> 32);
    const float vk = __uint_as_float((kk & 0x80000000u) ? (kk & 0x7FFFFFFFu) : ~kk);
    const float T = vk + 2.f * B;
    if (T <= __FLT_MAX__) {
      const uint64_t tcomp = ((uint64_t)order_key(T) << 32) | 0xFFFFFFFFull;
      certain = certain || readlane64(best, K1 - 1) > tcomp;
      ncand = __popcll(__ballot(lane < ncand && best <= tcomp));
    }
  }
  if (!certain) {
    if (m.redo != nullptr) {
      if (lane == 0) push_redo(m.redo + (COARSE ? 0 : 1), m.redo + 2, r);
      return;  // whole waves leave
    }
    if (lane == 0) atomicAdd(&g_sel_stats[1], 1ull);
  }

  // 2. where each candidate lives (lane j < ncand holds candidate j)
  int64_t my_id = INT64_MAX, my_npad = 0;
  const float *my_base = nullptr;
  if (lane < ncand) {
    const int64_t pos = (int64_t)(uint32_t)best;
    if (coarse) {
      my_id = pos;
      my_base = g.cent + pos * g.d_cb_pad;
    } else {
      const int64_t pabs = seg0 + pos;
      const int64_t *pb = m.pair_base + g.pair0 + q * g.nprobe;
      int lo = 0, hi = g.nprobe - 1;
      while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (ldg(pb + mid) <= pabs) lo = mid; else hi = mid - 1;
      }
      const int32_t h = ldg(m.probes + g.pair0 + q * g.nprobe + lo);
      const int64_t rr = pabs - ldg(pb + lo);
      const int64_t p0 = ldg(g.poff + h);
      my_id = ldg(g.rowid + p0 + rr);
      // slab layout, or the row-major copy (read with npad = 1)
      my_npad = g.rows ? 1 : ldg(g.poff + h + 1) - p0;
      my_base = g.rows ? g.rows + (p0 + rr) * g.d_pad : g.vec + p0 * g.d_pad + rr * SLAB;
    }
  }

  // 3. exact re-measurement over the lanes
  float myS = __builtin_inff(), myC = 0.f;
  // vectors: G candidates at a time, lane l taking coordinates
  // 4l + 256u + e in that order (as measure1), 256 PP coordinates per pass
  // read as 16-byte pieces, so that G x PP + PP loads are in flight per lane;
  // the query row's rows are 16-byte aligned and padded to the slab width.
  constexpr int G = WIDE ? 3 : SELW_G, PP = WIDE ? 8 : 4;
  if (!coarse)
  for (int cc = 0; cc < ncand; cc += G) {
    const float ADANNS_GLOBAL_AS *xp[G];
    int64_t np[G];
#pragma unroll
    for (int gi = 0; gi < G; ++gi) {
      const int c = cc + gi < ncand ? cc + gi : ncand - 1;
      xp[gi] = (const float ADANNS_GLOBAL_AS *)readlane64((uint64_t)my_base, c);
      np[gi] = (int64_t)readlane64((uint64_t)my_npad, c);
    }
    float S[G], C[G];
#pragma unroll
    for (int gi = 0; gi < G; ++gi) S[gi] = C[gi] = 0.f;
    for (int d0 = 4 * lane; d0 < d_dot; d0 += 256 * PP) {
      float4 qv[PP], xv[G][PP];
#pragma unroll
      for (int u = 0; u < PP; ++u) {
        const int dim = d0 + 256 * u;
        qv[u] = dim < d_dot ? ldg4((const float *)qrow + dim) : make_float4(0.f, 0.f, 0.f, 0.f);
      }
#pragma unroll
      for (int gi = 0; gi < G; ++gi)
#pragma unroll
        for (int u = 0; u < PP; ++u) {
          const int dim = d0 + 256 * u;
          xv[gi][u] = dim < d_dot
                          ? ldg4((const float *)xp[gi] + (int64_t)(dim / SLAB) * np[gi] * SLAB + dim % SLAB)
                          : make_float4(0.f, 0.f, 0.f, 0.f);
        }
#pragma unroll
      for (int u = 0; u < PP; ++u)
#pragma unroll
        for (int e = 0; e < 4; ++e)
          if (d0 + 256 * u + e < d_dot)
#pragma unroll
            for (int gi = 0; gi < G; ++gi)
              acc_sq_diff(f4(qv[u], e), f4(xv[gi][u], e), S[gi], C[gi]);
    }
#pragma unroll
    for (int gi = 0; gi < G; ++gi) {
      wave_reduce_pair(S[gi], C[gi]);
      if (cc + gi < ncand && lane == cc + gi) {
        myS = S[gi];
        myC = C[gi];
      }
    }
  }
  // centroids: two at a time, lane l taking coordinates l, l + 64, ... (as
  // measure1's coarse measure)
  if (coarse)
  for (int cc = 0; cc < ncand; cc += 2) {
    const bool two = cc + 1 < ncand;
    const float ADANNS_GLOBAL_AS *x0 =
        (const float ADANNS_GLOBAL_AS *)readlane64((uint64_t)my_base, cc);
    const float ADANNS_GLOBAL_AS *x1 =
        (const float ADANNS_GLOBAL_AS *)readlane64((uint64_t)my_base, two ? cc + 1 : cc);
    float S0 = 0.f, C0 = 0.f, S1 = 0.f, C1 = 0.f;
    {
      for (int d0 = lane; d0 < d_dot; d0 += 64 * 8) {
        float xa[8], xb[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const int dim = d0 + 64 * u;
          xa[u] = dim < d_dot ? x0[dim] : 0.f;
          xb[u] = dim < d_dot ? x1[dim] : 0.f;
        }
#pragma unroll
        for (int u = 0; u < 8; ++u)
          if (d0 + 64 * u < d_dot) {
            const float qv = qrow[d0 + 64 * u];
            acc_sq_diff(qv, xa[u], S0, C0);
            acc_sq_diff(qv, xb[u], S1, C1);
          }
      }
    }
    wave_reduce_pair(S0, C0);
    wave_reduce_pair(S1, C1);
    if (lane == cc) {
      myS = S0;
      myC = C0;
    }
    if (two && lane == cc + 1) {
      myS = S1;
      myC = C1;
    }
  }

  // 4. bitonic sort of the 64 lanes by (S, C, id); lanes past ncand hold
  // (+inf, 0, INT64_MAX) and sort last
#pragma unroll
  for (int k = 2; k <= 64; k <<= 1) {
#pragma unroll
    for (int j = k >> 1; j > 0; j >>= 1) {
      const float oS = __shfl_xor(myS, j), oC = __shfl_xor(myC, j);
      const int64_t oid = shfl_xor64(my_id, j);
      const bool up = (lane & k) == 0, lower = (lane & j) == 0;
      const bool other_less = pair_less(oS, oC, oid, myS, myC, my_id);
      if ((lower == up) ? other_less : !other_less) {
        myS = oS;
        myC = oC;
        my_id = oid;
      }
    }
  }

  // 5. outputs
  if (lane < kout) {
    const bool has = lane < ncand;
    if (coarse) {
      const int32_t hsel = has ? (int32_t)my_id : -1;
      m.probes[g.pair0 + q * kout + lane] = hsel;
      if (m.user_probes) m.user_probes[g.pair0 + q * kout + lane] = hsel;
      if (m.dist && lane == 0) m.dist[r] = has ? myS : __builtin_inff();
    } else {
      m.dist[r * m.ldk + lane] = has ? myS : __builtin_inff();
      m.ids[r * m.ldk + lane] = has ? my_id : -1;
    }
  }
}

// ---- IVF-PQ ----------------------------------------------------------------------
// Codes of database row rowid[g] copied to layout row g (zero on padding rows).
__global__ void k_gather_codes(const uint8_t *__restrict__ codes, int32_t M,
                               const int64_t *__restrict__ rowid, int64_t rows_pad,
                               uint8_t *__restrict__ out) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= rows_pad * M) return;
  int64_t g = i / M, m = i % M;
  int64_t src = rowid[g];
  out[i] = src >= 0 ? codes[src * M + m] : 0;
}

// PQ encoding: code[row][m] = the nearest of block m's 256 codewords to
// X[row, m*dsub : (m+1)*dsub] (difference form, ties to the smaller index).
template <class T>
__global__ __launch_bounds__(256) void k_pq_encode(const T *__restrict__ X, int64_t ldx,
                                                   int64_t n, int32_t M, int32_t dsub,
                                                   const float *__restrict__ cb,
                                                   uint8_t *__restrict__ codes) {
  extern __shared__ float cbs[];  // [256][dsub]
  const int m = blockIdx.y;
  for (int i = threadIdx.x; i < 256 * dsub; i += blockDim.x) cbs[i] = cb[(int64_t)m * 256 * dsub + i];
  __syncthreads();
  const int64_t row = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (row >= n) return;
  float y[PQ_ENCODE_MAX_DSUB];
  const T *src = X + row * ldx + (int64_t)m * dsub;
#pragma unroll
  for (int t = 0; t < PQ_ENCODE_MAX_DSUB; ++t) y[t] = t < dsub ? (float)src[t] : 0.f;
  float best = __builtin_inff();
  int bc = 0;
  for (int c = 0; c < 256; ++c) {
    const float *cw = cbs + c * dsub;
    float acc = 0.f;
#pragma unroll
    for (int t = 0; t < PQ_ENCODE_MAX_DSUB; ++t) {
      if (t < dsub) {
        const float dd = y[t] - cw[t];
        acc += dd * dd;
      }
    }
    if (acc < best) {
      best = acc;
      bc = c;
    }
  }
  codes[row * M + m] = (uint8_t)bc;
}

// q' = q[:d_s] R accumulated in FP64 (products of FP32 values are exact in
// FP64), stored as the FP32 pair (hi, lo) with hi + lo = the FP64 sum to
// within 2^-48 relative. FP64 matrix cores: a workgroup computes ROT_Q
// queries x ROT_C output columns, wave w the 16 queries 16w.. against four
// 16-column blocks with v_mfma_f64_16x16x4f64 (lane l supplies A[l % 16][l /
// 16] and B[l / 16][l % 16]; it receives D[l / 16 + 4 r][l % 16], r = 0..3,
// a different row order from the FP32 16x16x4 form). Q and R are staged in
// LDS as FP64, ROT_K coordinates at a time.
constexpr int ROT_Q = 64, ROT_C = 64, ROT_K = 32;
typedef double doublex4 __attribute__((ext_vector_type(4)));
__global__ __launch_bounds__(256) void k_rotate(const float *__restrict__ Qs, int64_t ldqs,
                                                int64_t nq, const float *__restrict__ R,
                                                int32_t d_s, float *__restrict__ qh,
                                                float *__restrict__ ql, int64_t ldqr) {
  constexpr int NPA = ROT_Q * ROT_K / 256, NPB = ROT_K * ROT_C / 256;  // per thread
  __shared__ double As[ROT_K][ROT_Q + 1];  // As[k][query]
  __shared__ double Bs[ROT_K][ROT_C + 1];  // Bs[k][column]
  const int tid = threadIdx.x, lane = tid & 63;
  const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int64_t q0 = (int64_t)blockIdx.x * ROT_Q;
  const int c0 = blockIdx.y * ROT_C;
  doublex4 acc[ROT_C / 16];
#pragma unroll
  for (int j = 0; j < ROT_C / 16; ++j) acc[j] = (doublex4){0.0, 0.0, 0.0, 0.0};
  // the next chunk's values are loaded into registers while this one's
  // MFMAs run
  float pa[NPA], pb[NPB];
  auto load = [&](int k0) {
#pragma unroll
    for (int e = 0; e < NPA; ++e) {
      const int i = tid + 256 * e, qq = i / ROT_K, kk = i % ROT_K;
      const int64_t q = q0 + qq;
      pa[e] = (q < nq && k0 + kk < d_s) ? Qs[q * ldqs + k0 + kk] : 0.f;
    }
#pragma unroll
    for (int e = 0; e < NPB; ++e) {
      const int i = tid + 256 * e, kk = i / ROT_C, cc = i % ROT_C;
      pb[e] = (k0 + kk < d_s && c0 + cc < d_s) ? R[(int64_t)(k0 + kk) * d_s + c0 + cc] : 0.f;
    }
  };
  load(0);
  for (int k0 = 0; k0 < d_s; k0 += ROT_K) {
    __syncthreads();  // the previous chunk is consumed
#pragma unroll
    for (int e = 0; e < NPA; ++e) {
      const int i = tid + 256 * e;
      As[i % ROT_K][i / ROT_K] = (double)pa[e];
    }
#pragma unroll
    for (int e = 0; e < NPB; ++e) {
      const int i = tid + 256 * e;
      Bs[i / ROT_C][i % ROT_C] = (double)pb[e];
    }
    __syncthreads();
    if (k0 + ROT_K < d_s) load(k0 + ROT_K);
#pragma unroll
    for (int ks = 0; ks < ROT_K; ks += 4) {
      const double a = As[ks + (lane >> 4)][16 * wv + (lane & 15)];
#pragma unroll
      for (int j = 0; j < ROT_C / 16; ++j)
        acc[j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, Bs[ks + (lane >> 4)][16 * j + (lane & 15)],
                                                      acc[j], 0, 0, 0);
    }
  }
#pragma unroll
  for (int j = 0; j < ROT_C / 16; ++j)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int64_t q = q0 + 16 * wv + (lane >> 4) + 4 * r;
      const int c = c0 + 16 * j + (lane & 15);
      if (q < nq && c < d_s) {
        const float hi = (float)acc[j][r];
        qh[q * ldqr + c] = hi;
        ql[q * ldqr + c] = (float)(acc[j][r] - (double)hi);
      }
    }
}

// LUT[q][m][c] = |q'_m - C_m[c]|^2 in FP32 (difference form, t = 0..dsub-1
// in order) from the rotated query's high part. A workgroup takes block m
// for LUT_Q queries: block m's 256 codewords are staged in LDS (LUT_T
// coordinates at a time) and thread c fills entry c of every query's table.
constexpr int LUT_Q = 64;
constexpr int LUT_T = 32;
__global__ __launch_bounds__(256) void k_pq_lut(const float *__restrict__ qh, int64_t ldqr,
                                                int64_t nq, const float *__restrict__ cb,
                                                int32_t M, int32_t dsub, float *__restrict__ lut) {
  __shared__ float cw[256][LUT_T + 1];  // odd stride: thread c's row starts in its own bank
  __shared__ float qv[LUT_Q][LUT_T];
  const int m = blockIdx.y, c = threadIdx.x;
  const int64_t q0 = (int64_t)blockIdx.x * LUT_Q;
  float acc[LUT_Q];
#pragma unroll
  for (int a = 0; a < LUT_Q; ++a) acc[a] = 0.f;
  for (int t0 = 0; t0 < dsub; t0 += LUT_T) {
    const int tn = min(LUT_T, dsub - t0);
    __syncthreads();  // the previous chunk is consumed
    for (int i = threadIdx.x; i < 256 * tn; i += blockDim.x)
      cw[i / tn][i % tn] = cb[((int64_t)m * 256 + i / tn) * dsub + t0 + i % tn];
    for (int i = threadIdx.x; i < LUT_Q * tn; i += blockDim.x) {
      const int64_t q = q0 + i / tn;
      qv[i / tn][i % tn] = q < nq ? qh[q * ldqr + (int64_t)m * dsub + t0 + i % tn] : 0.f;
    }
    __syncthreads();
#pragma unroll
    for (int a = 0; a < LUT_Q; ++a)
      for (int t = 0; t < tn; ++t) {
        const float dd = qv[a][t] - cw[c][t];
        acc[a] += dd * dd;
      }
  }
#pragma unroll
  for (int a = 0; a < LUT_Q; ++a)
    if (q0 + a < nq) lut[((q0 + a) * M + m) * 256 + c] = acc[a];
}

// ADC scan: a workgroup holds one query's table in LDS and walks G of its
// probed lists one after another, every thread taking rows of the current
// list; each row sums the M table entries its codes pick (in code order
// m = 0..M-1). 1024 threads share one table, so that a CU holds enough waves
// to hide the table reads' latency. The next list's location is loaded while
// the current one is scanned. MM > 0: M = MM, a multiple of 16, and each
// row's codes are loaded whole (all its 16-byte pieces in flight together)
// before its look-ups: loaded one piece at a time between look-ups, the
// rows' cache lines were evicted and fetched again (1.33x the algorithmic
// bytes at M = 64). MM = 0: any M (a multiple of 4) given at run time.
constexpr int ADC_THREADS = 1024;
template <int MM>
__global__ __launch_bounds__(ADC_THREADS) void k_adc_scan(const float *__restrict__ lut, int32_t M_,
                                                          const uint8_t *__restrict__ codes,
                                                          const int32_t *__restrict__ probes,
                                                          int32_t nprobe, int32_t G,
                                                          const int64_t *__restrict__ poff,
                                                          const int32_t *__restrict__ len,
                                                          const int64_t *__restrict__ pair_base,
                                                          float *__restrict__ D) {
  static_assert(MM % 16 == 0 && MM <= 64, "whole-row loads for M = 16, 32, 64");
  const int M = MM > 0 ? MM : M_;
  extern __shared__ float tab[];  // [M][256]
  const int gpq = (nprobe + G - 1) / G;
  const int64_t q = blockIdx.x / gpq;
  const int j0 = (int)(blockIdx.x % gpq) * G, j1 = min(nprobe, j0 + G);
  const float4 *src = (const float4 *)(lut + q * M * 256);
  for (int i = threadIdx.x; i < M * 64; i += blockDim.x) ((float4 *)tab)[i] = src[i];
  __syncthreads();
  auto where = [&](int j, int32_t &n, const uint8_t *&cbase, float *&out) {
    const int64_t pair = q * nprobe + j;
    const int32_t h = probes[pair];
    n = len[h];
    cbase = codes + poff[h] * M;
    out = D + pair_base[pair];
  };
  int32_t n;
  const uint8_t *cbase;
  float *out;
  where(j0, n, cbase, out);
  for (int j = j0; j < j1; ++j) {
    int32_t n2 = 0;
    const uint8_t *cb2 = nullptr;
    float *out2 = nullptr;
    if (j + 1 < j1) where(j + 1, n2, cb2, out2);
    for (int r = threadIdx.x; r < n; r += blockDim.x) {
      float acc = 0.f;
      if constexpr (MM > 0) {
        constexpr int NW = MM / 16;
        const uint4 *row = (const uint4 *)(cbase + (int64_t)r * MM);
        uint4 c16[NW];
#pragma unroll
        for (int w = 0; w < NW; ++w) c16[w] = row[w];
#pragma unroll
        for (int w = 0; w < NW; ++w) {
          const uint32_t wd[4] = {c16[w].x, c16[w].y, c16[w].z, c16[w].w};
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            const int m = w * 16 + e * 4;
            acc += tab[(m + 0) * 256 + (wd[e] & 0xff)];
            acc += tab[(m + 1) * 256 + ((wd[e] >> 8) & 0xff)];
            acc += tab[(m + 2) * 256 + ((wd[e] >> 16) & 0xff)];
            acc += tab[(m + 3) * 256 + (wd[e] >> 24)];
          }
        }
      } else if ((M & 15) == 0) {  // 16 codes per load (rows are 16-byte aligned)
        const uint4 *row = (const uint4 *)(cbase + (int64_t)r * M);
        for (int w = 0; w < (M >> 4); ++w) {
          const uint4 c16 = row[w];
          const uint32_t wd[4] = {c16.x, c16.y, c16.z, c16.w};
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            const int m = w * 16 + e * 4;
            acc += tab[(m + 0) * 256 + (wd[e] & 0xff)];
            acc += tab[(m + 1) * 256 + ((wd[e] >> 8) & 0xff)];
            acc += tab[(m + 2) * 256 + ((wd[e] >> 16) & 0xff)];
            acc += tab[(m + 3) * 256 + (wd[e] >> 24)];
          }
        }
      } else {
        const uint32_t *row = (const uint32_t *)(cbase + (int64_t)r * M);
        for (int w = 0; w < (M >> 2); ++w) {
          const uint32_t c4 = row[w];
          const int m = w * 4;
          acc += tab[(m + 0) * 256 + (c4 & 0xff)];
          acc += tab[(m + 1) * 256 + ((c4 >> 8) & 0xff)];
          acc += tab[(m + 2) * 256 + ((c4 >> 16) & 0xff)];
          acc += tab[(m + 3) * 256 + (c4 >> 24)];
        }
      }
      out[r] = acc;
    }
    n = n2;
    cbase = cb2;
    out = out2;
  }
}

// ---- precision form ------------------------------------------------------------
// BF16: upper half of the FP32 encoding after round-to-nearest-even.
__device__ __forceinline__ uint16_t bf16_rne(float x) {
  uint32_t u = __float_as_uint(x);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

// OCP e4m3: nearest value, ties to the even code, saturating at +-448; the
// scaling by powers of two is exact, so the only rounding is rint().
__device__ __forceinline__ uint8_t e4m3_encode(float y) {
  const float a = fabsf(y);
  uint32_t code;
  if (!(a < 448.f)) {
    code = 0x7Eu;
  } else if (a < 0.015625f) {
    code = (uint32_t)__builtin_rintf(a * 512.f);
  } else {
    int e = (int)((__float_as_uint(a) >> 23) & 0xFFu) - 127;
    uint32_t m = (uint32_t)__builtin_rintf(a * __uint_as_float((uint32_t)(130 - e) << 23));
    if (m == 16u) {
      m = 8u;
      e += 1;
    }
    code = ((uint32_t)(e + 7) << 3) | (m - 8u);
    if (code > 0x7Eu) code = 0x7Eu;
  }
  const uint32_t sign = (code != 0u && (__float_as_uint(y) >> 31)) ? 0x80u : 0u;
  return (uint8_t)(sign | code);
}

__global__ void k_quant_bf16(const float *__restrict__ src, int64_t n, uint16_t *__restrict__ dst) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = bf16_rne(src[i]);
}

// One wave per slab-layout row: scale = amax / 448 over the row's first
// d_used coordinates, codes of x * (448 / amax).
__global__ __launch_bounds__(256) void k_quant_fp8_slab(const float *__restrict__ src,
                                                        const int64_t *__restrict__ poff,
                                                        int32_t nlist, int64_t rows, int32_t d_pad,
                                                        int32_t d_used, uint8_t *__restrict__ dst,
                                                        float *__restrict__ scale) {
  const int lane = threadIdx.x & 63;
  const int64_t g = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (g >= rows) return;
  int lo = 0, hi = nlist - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (poff[mid] <= g) lo = mid; else hi = mid - 1;
  }
  const int64_t p0 = poff[lo], npad = poff[lo + 1] - p0, r = g - p0;
  const int64_t base = p0 * d_pad + r * SLAB;
  float amax = 0.f;
  for (int dim = lane; dim < d_used; dim += 64)
    amax = fmaxf(amax, fabsf(src[base + (int64_t)(dim / SLAB) * npad * SLAB + (dim % SLAB)]));
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) amax = fmaxf(amax, __shfl_xor(amax, off));
  const float inv = amax > 0.f ? 448.f / amax : 0.f;
  if (lane == 0) scale[g] = amax / 448.f;
  for (int dim = lane; dim < d_pad; dim += 64) {
    const int64_t idx = base + (int64_t)(dim / SLAB) * npad * SLAB + (dim % SLAB);
    dst[idx] = dim < d_used ? e4m3_encode(src[idx] * inv) : (uint8_t)0;
  }
}

// Row-major query quantisation (one wave per row), zero beyond d_used.
__global__ __launch_bounds__(256) void k_quant_rows(const float *__restrict__ Q, int64_t nq,
                                                    int64_t ldq, int32_t d_used, int32_t fmt,
                                                    void *__restrict__ out, int64_t ldo,
                                                    float *__restrict__ scale) {
  const int lane = threadIdx.x & 63;
  const int64_t q = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (q >= nq) return;
  const float *row = Q + q * ldq;
  // Rows that are 16-byte aligned and at least ldo wide (ldo a multiple of 8):
  // eight coordinates per lane and step, 16-byte loads, four steps in flight
  // (values past d_used are written as zero, the same per coordinate as
  // below); other rows one coordinate per lane and step.
  const bool vec = ((uintptr_t)Q & 15) == 0 && ldq % 4 == 0 && ldq >= ldo && ldo % 8 == 0;
  if (fmt == 1) {
    uint16_t *o = (uint16_t *)out + q * ldo;
    if (vec) {
      for (int c0 = 8 * lane; c0 < ldo; c0 += 512 * 4) {
        float4 v[4][2];
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
          for (int h = 0; h < 2; ++h) {
            const int dim = c0 + 512 * u + 4 * h;
            v[u][h] = dim < ldo ? *(const float4 *)(row + dim) : make_float4(0.f, 0.f, 0.f, 0.f);
          }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int dim = c0 + 512 * u;
          if (dim >= ldo) break;
          uint32_t w[4];
#pragma unroll
          for (int t = 0; t < 4; ++t) {
            const float x0 = f4(v[u][t >> 1], 2 * (t & 1)), x1 = f4(v[u][t >> 1], 2 * (t & 1) + 1);
            const uint32_t b0 = dim + 2 * t < d_used ? bf16_rne(x0) : 0u;
            const uint32_t b1 = dim + 2 * t + 1 < d_used ? bf16_rne(x1) : 0u;
            w[t] = b0 | (b1 << 16);
          }
          *(uint4 *)(o + dim) = make_uint4(w[0], w[1], w[2], w[3]);
        }
      }
    } else {
      for (int dim = lane; dim < ldo; dim += 64) o[dim] = dim < d_used ? bf16_rne(row[dim]) : 0;
    }
    if (lane == 0 && scale) scale[q] = 1.f;
    return;
  }
  uint8_t *o = (uint8_t *)out + q * ldo;
  float amax = 0.f;
  if (vec) {
    for (int c0 = 8 * lane; c0 < ldo; c0 += 512 * 4) {
      float4 v[4][2];
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const int dim = c0 + 512 * u + 4 * h;
          v[u][h] = dim < ldo ? *(const float4 *)(row + dim) : make_float4(0.f, 0.f, 0.f, 0.f);
        }
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int t = 0; t < 8; ++t)
          if (c0 + 512 * u + t < d_used) amax = fmaxf(amax, fabsf(f4(v[u][t >> 2], t & 3)));
    }
  } else {
    for (int dim = lane; dim < d_used; dim += 64) amax = fmaxf(amax, fabsf(row[dim]));
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) amax = fmaxf(amax, __shfl_xor(amax, off));
  const float inv = amax > 0.f ? 448.f / amax : 0.f;
  if (lane == 0) scale[q] = amax / 448.f;
  if (vec) {
    for (int c0 = 8 * lane; c0 < ldo; c0 += 512 * 4) {
      float4 v[4][2];
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const int dim = c0 + 512 * u + 4 * h;
          v[u][h] = dim < ldo ? *(const float4 *)(row + dim) : make_float4(0.f, 0.f, 0.f, 0.f);
        }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int dim = c0 + 512 * u;
        if (dim >= ldo) break;
        uint32_t w[2] = {0u, 0u};
#pragma unroll
        for (int t = 0; t < 8; ++t)
          if (dim + t < d_used)
            w[t >> 2] |= (uint32_t)e4m3_encode(f4(v[u][t >> 2], t & 3) * inv) << (8 * (t & 3));
        *(uint2 *)(o + dim) = make_uint2(w[0], w[1]);
      }
    }
  } else {
    for (int dim = lane; dim < ldo; dim += 64) o[dim] = dim < d_used ? e4m3_encode(row[dim] * inv) : 0;
  }
}

__device__ __forceinline__ float qdecode(int FMT, uint32_t bits) {
  return FMT == 1 ? __uint_as_float(bits << 16) : e4m3_to_float(bits);
}

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

struct TileQArgs {
  const uint8_t *Qq;       // quantised queries, row-major, ldqq elements per row
  int64_t ldqq;
  const float *qscale;     // per query (e4m3), else unused
  int32_t d_dot;
  const uint8_t *vec;      // quantised slab layout
  const float *vscale;     // per layout row (e4m3)
  int32_t d_pad;
  const int64_t *poff;
  const int32_t *len;
  int32_t nlist;
  const int32_t *tile_off;
  const int32_t *bkt_off;
  const int32_t *cnt;
  const int32_t *bucket;
  int32_t pair_div;
  const int64_t *pair_base;
  float *out;
  int64_t nq;
  int32_t nl, nl_pad, qtiles, total_host;
  int32_t *work;           // scan: [8] work counters, zero at launch
};

// First pass of the precision form: s_x^2 |x_hat|^2 - 2 s_q s_x (q_hat . x_hat)
// on BF16 (FMT 1) or e4m3 (FMT 2) MFMA with FP32 accumulation; products of
// these formats are exact in FP32. This kernel serves the coarse step (every
// query against the centroids, stored as one slab-layout list): tiles of 64
// queries x 64 centroids, K steps of 4 slabs (128 coordinates). The scan uses
// k_tile_q_scan.
template <int FMT>
__global__ __launch_bounds__(256) void k_tile_dist_q(TileQArgs a) {
  constexpr int EB = FMT == 1 ? 2 : 1;
  constexpr int KS = 4;
  constexpr int ROWB = SLAB * EB;
  constexpr int STEPB = KS * ROWB;
  constexpr int CPR = STEPB / 16;          // 16-byte chunks per row per step
  constexpr int NU = TILE_Q * CPR / 256;   // chunks per thread per operand
  __shared__ __attribute__((aligned(16))) uint8_t As[TILE_Q][STEPB + 16];
  __shared__ __attribute__((aligned(16))) uint8_t Bs[TILE_V][STEPB + 16];
  __shared__ int64_t rbase[TILE_Q];
  __shared__ int32_t rq[TILE_Q];
  __shared__ float rsc[TILE_Q], csc[TILE_V], cn[TILE_V];

  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int total = a.total_host;
  const int G = gridDim.x;
  const int rb = (wv >> 1) * 32, cb = (wv & 1) * 32;
  const int fr = lane & 15, fg = lane >> 4;
  const int nslab_dot = (a.d_dot + SLAB - 1) / SLAB;
  const int nsteps = (nslab_dot + KS - 1) / KS;

  // XCD-aware order: workgroup b runs on XCD b % 8; each XCD gets a
  // contiguous run of work items
  const int L = (blockIdx.x & 7) * (G >> 3) + (blockIdx.x >> 3);
  for (int w = L; w < total; w += G) {
    const int qt = w % a.qtiles, vt = w / a.qtiles;
    const int m = (int)a.nq, nvec = a.nl;
    const int64_t npad = a.nl_pad, p0 = 0;
    __syncthreads();
    if (tid < TILE_Q) {
      const int i = qt * TILE_Q + tid;
      if (i < m) {
        const int32_t qq = i;
        rq[tid] = qq;
        rbase[tid] = (int64_t)i * a.nl;
        rsc[tid] = FMT == 2 ? a.qscale[qq] : 1.f;
      } else {
        rq[tid] = -1;
        rbase[tid] = 0;
        rsc[tid] = 0.f;
      }
    } else if (tid < TILE_Q + TILE_V) {
      const int col = tid - TILE_Q;
      csc[col] = FMT == 2 ? a.vscale[p0 + vt * TILE_V + col] : 1.f;
    }
    __syncthreads();
    const uint8_t *vbase = a.vec + (p0 * a.d_pad + (int64_t)vt * TILE_V * SLAB) * EB;

    floatx4 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j) acc[i][j] = (floatx4){0.f, 0.f, 0.f, 0.f};
    float nrm[NU];
#pragma unroll
    for (int u = 0; u < NU; ++u) nrm[u] = 0.f;
    uint4 ra[NU], rbv[NU];

    auto load = [&](int step) {
#pragma unroll
      for (int u = 0; u < NU; ++u) {
        const int idx = tid + 256 * u;
        const int row = idx / CPR, ch = idx % CPR;
        const int byte = ch * 16;
        const int slab = step * KS + byte / ROWB;
        const int inb = byte % ROWB;
        const int e0 = slab * SLAB + inb / EB;  // first coordinate of the chunk
        uint4 va = make_uint4(0, 0, 0, 0), vb = make_uint4(0, 0, 0, 0);
        if (slab < nslab_dot) {
          const int qq = rq[row];
          if (qq >= 0) va = *(const uint4 *)(a.Qq + ((int64_t)qq * a.ldqq + e0) * EB);
          vb = *(const uint4 *)(vbase + ((int64_t)slab * npad * SLAB + (int64_t)row * SLAB) * EB + inb);
          if (e0 + 16 / EB > a.d_dot) {  // zero query coordinates past d_dot
            uint32_t wds[4] = {va.x, va.y, va.z, va.w};
#pragma unroll
            for (int e = 0; e < 16 / EB; ++e) {
              if (e0 + e >= a.d_dot) {
                const int wi = (e * EB) / 4, sh = ((e * EB) % 4) * 8;
                wds[wi] &= ~(((1u << (8 * EB)) - 1u) << sh);
              }
            }
            va = make_uint4(wds[0], wds[1], wds[2], wds[3]);
          }
        }
        ra[u] = va;
        rbv[u] = vb;
      }
    };

    load(0);
    for (int step = 0; step < nsteps; ++step) {
      __syncthreads();
#pragma unroll
      for (int u = 0; u < NU; ++u) {
        const int idx = tid + 256 * u;
        const int row = idx / CPR, ch = idx % CPR;
        *(uint4 *)&As[row][ch * 16] = ra[u];
        *(uint4 *)&Bs[row][ch * 16] = rbv[u];
        // squared norm of the vector chunk, coordinates below d_dot only
        const int byte = ch * 16;
        const int e0 = (step * KS + byte / ROWB) * SLAB + (byte % ROWB) / EB;
        const uint32_t wds[4] = {rbv[u].x, rbv[u].y, rbv[u].z, rbv[u].w};
#pragma unroll
        for (int e = 0; e < 16 / EB; ++e) {
          const uint32_t bits = (wds[(e * EB) / 4] >> (((e * EB) % 4) * 8)) & ((1u << (8 * EB)) - 1u);
          const float v = qdecode(FMT, bits);
          if (e0 + e < a.d_dot) nrm[u] += v * v;
        }
      }
      __syncthreads();
      if (step + 1 < nsteps) load(step + 1);
#pragma unroll
      for (int sl = 0; sl < KS; ++sl) {
        const int off = sl * ROWB + fg * 8 * EB;
        if (FMT == 1) {
          bf16x8 af[2], bfv[2];
#pragma unroll
          for (int i = 0; i < 2; ++i) {
            const uint4 x = *(const uint4 *)&As[rb + i * 16 + fr][off];
            af[i] = __builtin_bit_cast(bf16x8, x);
          }
#pragma unroll
          for (int j = 0; j < 2; ++j) {
            const uint4 x = *(const uint4 *)&Bs[cb + j * 16 + fr][off];
            bfv[j] = __builtin_bit_cast(bf16x8, x);
          }
#pragma unroll
          for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j)
              acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[i], bfv[j], acc[i][j], 0, 0, 0);
        } else {
          long af[2], bfv[2];
#pragma unroll
          for (int i = 0; i < 2; ++i) af[i] = *(const long *)&As[rb + i * 16 + fr][off];
#pragma unroll
          for (int j = 0; j < 2; ++j) bfv[j] = *(const long *)&Bs[cb + j * 16 + fr][off];
#pragma unroll
          for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j)
              acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8(af[i], bfv[j], acc[i][j], 0, 0, 0);
        }
      }
    }
    // norms: CPR consecutive threads share a row
#pragma unroll
    for (int u = 0; u < NU; ++u) {
#pragma unroll
      for (int off = 1; off < CPR; off <<= 1) nrm[u] += __shfl_xor(nrm[u], off);
      const int idx = tid + 256 * u;
      if ((idx % CPR) == 0) cn[idx / CPR] = nrm[u];
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int row = rb + i * 16 + (lane >> 4) * 4 + e;
          const int col = cb + j * 16 + (lane & 15);
          const int v = vt * TILE_V + col;
          if (rq[row] >= 0 && v < nvec) {
            const float sx = csc[col], sq = rsc[row];
            a.out[rbase[row] + v] = sx * sx * cn[col] - 2.0f * sq * sx * acc[i][j][e];
          }
        }
  }
}

// LDS-DMA form of the precision form's scan tile (TQ x TV = 128 x 64),
// built like tile_compute_dma: every stage holds 128 bytes of each operand
// row (SC = 64 BF16 or 128 e4m3 coordinates, KS slabs), copied straight into
// LDS by 16-byte global_load_lds_dwordx4 with chunk c of row r at position
// c ^ f(r); four waves in a 2 x 2 grid, each (TQ/2) x (TV/2) in 16x16x32
// MFMA blocks. Lane l reads, per k-step of 32 coordinates, the 8 values at
// coordinates 8 (l >> 4) .. of row l & 15, for both operands. Quantised
// norms are summed from the decoded B fragments. Coordinates past d_dot are
// zeroed in LDS on the last stage (both operands); copies that would start
// past a row's stored width re-read an earlier piece of it, which is zeroed
// too.
// The copies run in a ring of three stages, two ahead of the one being
// read: the scan waits on copy latency (its MFMA work per stage is short), so
// bytes in flight set its pace. The barrier that hands a stage over waits
// for LDS work only, and the fragment reads are inline-asm ds_read groups
// that wait for their own results: LDS reads that the compiler sees make it
// wait for every copy still in flight (it cannot tell the stage being read
// from the stages being filled), which would drain the ring at every stage.
constexpr int QTILE_Q = 128, QTILE_V = 64;  // precision-form scan tile

typedef int v4i32 __attribute__((ext_vector_type(4)));
// LDS address of p, as ds_read takes it
__device__ __forceinline__ uint32_t lds_off(const uint8_t *p) {
  return (uint32_t)(uintptr_t)(const __attribute__((address_space(3))) uint8_t *)p;
}
// Four A-operand reads at la and two B-operand reads at lb, rows 16 apart
// (2048 bytes), 16 bytes each; one group that waits for its own results.
__device__ __forceinline__ void lds_frags_b128(uint32_t la, uint32_t lb, v4i32 (&ra)[4],
                                               v4i32 (&rb)[2]) {
  asm volatile(
      "ds_read_b128 %0, %6\n"
      "ds_read_b128 %1, %6 offset:2048\n"
      "ds_read_b128 %2, %6 offset:4096\n"
      "ds_read_b128 %3, %6 offset:6144\n"
      "ds_read_b128 %4, %7\n"
      "ds_read_b128 %5, %7 offset:2048\n"
      "s_waitcnt lgkmcnt(0)"
      : "=&v"(ra[0]), "=&v"(ra[1]), "=&v"(ra[2]), "=&v"(ra[3]), "=&v"(rb[0]), "=&v"(rb[1])
      : "v"(la), "v"(lb));
}
// The same with 8-byte reads.
__device__ __forceinline__ void lds_frags_b64(uint32_t la, uint32_t lb, long (&ra)[4],
                                              long (&rb)[2]) {
  asm volatile(
      "ds_read_b64 %0, %6\n"
      "ds_read_b64 %1, %6 offset:2048\n"
      "ds_read_b64 %2, %6 offset:4096\n"
      "ds_read_b64 %3, %6 offset:6144\n"
      "ds_read_b64 %4, %7\n"
      "ds_read_b64 %5, %7 offset:2048\n"
      "s_waitcnt lgkmcnt(0)"
      : "=&v"(ra[0]), "=&v"(ra[1]), "=&v"(ra[2]), "=&v"(ra[3]), "=&v"(rb[0]), "=&v"(rb[1])
      : "v"(la), "v"(lb));
}

template <int FMT, int TQ, int TV>
__global__ __launch_bounds__(256, 2) void k_tile_q_scan(TileQArgs a) {
  static_assert(TQ == 128 && TV == 64, "fragment reads written for 128 x 64 tiles");
  constexpr int NST = 3;  // stages in the copy ring (3 x 24 KB at 128 x 64)
  constexpr int EB = FMT == 1 ? 2 : 1;
  constexpr int KS = 128 / (SLAB * EB);    // slabs per stage
  constexpr int SC = KS * SLAB;            // coordinates per stage
  constexpr int CPS = SLAB * EB / 16;      // 16-byte chunks per slab row
  constexpr int EPC = 16 / EB;             // coordinates per chunk
  constexpr int NA = TQ / 32, NBV = TV / 32;
  constexpr int NB16 = TQ / 32, NC16 = TV / 32;
  constexpr int NKS = SC / 32;             // MFMA k-steps per stage
  __shared__ __attribute__((aligned(16))) uint8_t Ar[NST][TQ * 128];
  __shared__ __attribute__((aligned(16))) uint8_t Br[NST][TV * 128];
  __shared__ int64_t rbase[TQ];
  __shared__ int32_t rq[TQ];
  __shared__ float rsc[TQ], csc[TV], cn[TV];
  __shared__ int s_item;

  const int tid = threadIdx.x, lane = tid & 63;
  const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int rbw = (wv >> 1) * (TQ / 2), cbw = (wv & 1) * (TV / 2);
  const int total = a.tile_off[a.nlist];
  const int xcd = blockIdx.x & 7;
  const int nstage = (a.d_dot + SC - 1) / SC;
  const int nslab_dot = (a.d_dot + SLAB - 1) / SLAB;
  const int lrow = lane >> 3;
  const int gch = (lane & 7) ^ lrow ^ (wv & 1);  // global chunk of this lane's copies
  const int r16 = lane & 15, g16 = lane >> 4;
  const int sw16 = swz(r16);

  for (;;) {
    __syncthreads();  // every thread has read the previous s_item; epilogue done
    if (tid == 0) {
      const int k = atomicAdd(&a.work[xcd], 1);
      s_item = ((k / SCAN_CHUNK) * 8 + xcd) * SCAN_CHUNK + k % SCAN_CHUNK;
    }
    __syncthreads();
    const int w = s_item;
    if (w >= total) break;
    int lo = 0, hi = a.nlist - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (ldg(a.tile_off + mid) <= w) lo = mid; else hi = mid - 1;
    }
    const int h = lo;
    const int m = ldg(a.cnt + h), nvec = ldg(a.len + h);
    const int64_t p0 = ldg(a.poff + h), npad = ldg(a.poff + h + 1) - p0;
    const int qts = (m + TQ - 1) / TQ;
    const int rem = w - ldg(a.tile_off + h);
    const int qt = rem % qts, vt = rem / qts;
    const int ncol = min(TV, nvec - vt * TV);
    const int nrow = min(TQ, m - qt * TQ);
    if (tid < TQ) {
      const int i = qt * TQ + tid;
      if (i < m) {
        const int32_t pair = ldg(a.bucket + ldg(a.bkt_off + h) + i);
        const int32_t qq = pair / a.pair_div;
        rq[tid] = qq;
        rbase[tid] = ldg(a.pair_base + pair);
        rsc[tid] = FMT == 2 ? ldg(a.qscale + qq) : 1.f;
      } else {
        rq[tid] = -1;
        rbase[tid] = 0;
        rsc[tid] = 0.f;
      }
    } else if (tid < TQ + TV) {
      const int col = tid - TQ;
      csc[col] = (FMT == 2 && col < ncol) ? ldg(a.vscale + p0 + vt * TV + col) : 1.f;
    }
    __syncthreads();
    const bool active = nrow > rbw && ncol > cbw;
    const uint8_t *vbase = a.vec + (p0 * a.d_pad + (int64_t)vt * TV * SLAB) * EB;
    // copy side: wave instruction u fills rows (4u + wv) * 8 .. + 7
    const uint8_t *qp[NA];
#pragma unroll
    for (int u = 0; u < NA; ++u) {
      const int q = rq[(4 * u + wv) * 8 + lrow];
      qp[u] = a.Qq + (int64_t)(q >= 0 ? q : 0) * a.ldqq * EB;
    }
    int vrow[NBV];
#pragma unroll
    for (int u = 0; u < NBV; ++u) vrow[u] = min((4 * u + wv) * 8 + lrow, ncol - 1);
    auto issue = [&](int s, uint8_t *A, uint8_t *B) {
      // this lane's chunk: coordinates s * SC + gch * EPC .., in slab sl
      int sl = s * KS + gch / CPS;
      int c0 = s * SC + gch * EPC;
      if (sl >= nslab_dot) {  // past the prefix: re-read the first piece (zeroed)
        sl = 0;
        c0 = 0;
      }
#pragma unroll
      for (int u = 0; u < NA; ++u)
        __builtin_amdgcn_global_load_lds(
            (const void *)(qp[u] + (int64_t)c0 * EB),
            (__attribute__((address_space(3))) void *)(A + (4 * u + wv) * 8 * 128), 16, 0, 0);
#pragma unroll
      for (int u = 0; u < NBV; ++u)
        __builtin_amdgcn_global_load_lds(
            (const void *)(vbase + ((int64_t)sl * npad * SLAB + (int64_t)vrow[u] * SLAB) * EB +
                           (gch % CPS) * 16),
            (__attribute__((address_space(3))) void *)(B + (4 * u + wv) * 8 * 128), 16, 0, 0);
    };
    auto clip = [&](uint8_t *A, uint8_t *B, int lim) {
      const int c = (lane & 7) * 16;  // LDS position of this lane's chunks
#pragma unroll
      for (int e = 0; e < EPC; ++e)
        if (gch * EPC + e >= lim) {
#pragma unroll
          for (int u = 0; u < NA; ++u)
#pragma unroll
            for (int b = 0; b < EB; ++b) A[((4 * u + wv) * 8 + lrow) * 128 + c + e * EB + b] = 0;
#pragma unroll
          for (int u = 0; u < NBV; ++u)
#pragma unroll
            for (int b = 0; b < EB; ++b) B[((4 * u + wv) * 8 + lrow) * 128 + c + e * EB + b] = 0;
        }
      __syncthreads();
    };
    floatx4 acc[NB16][NC16];
#pragma unroll
    for (int i = 0; i < NB16; ++i)
#pragma unroll
      for (int j = 0; j < NC16; ++j) acc[i][j] = (floatx4){0.f, 0.f, 0.f, 0.f};
    float nrm[NC16];
#pragma unroll
    for (int j = 0; j < NC16; ++j) nrm[j] = 0.f;
    auto compute = [&](const uint8_t *A, const uint8_t *B) {
#pragma unroll
      for (int ks = 0; ks < NKS; ++ks) {
        // chunk and byte of this lane's 8 values at k-step ks
        const int ch = FMT == 1 ? 4 * ks + g16 : 2 * ks + (g16 >> 1);
        const int inner = FMT == 1 ? 0 : (g16 & 1) * 8;
        const int off = ((ch ^ sw16) << 4) + inner;
        const uint32_t la = lds_off(A + (rbw + r16) * 128 + off);
        const uint32_t lb = lds_off(B + (cbw + r16) * 128 + off);
        if constexpr (FMT == 1) {
          v4i32 ra[NB16], rb[NC16];
          lds_frags_b128(la, lb, ra, rb);
          bf16x8 af[NB16], bfv[NC16];
#pragma unroll
          for (int i = 0; i < NB16; ++i) af[i] = __builtin_bit_cast(bf16x8, ra[i]);
#pragma unroll
          for (int j = 0; j < NC16; ++j) {
            const uint4 x = __builtin_bit_cast(uint4, rb[j]);
            bfv[j] = __builtin_bit_cast(bf16x8, x);
            const uint32_t wd[4] = {x.x, x.y, x.z, x.w};
#pragma unroll
            for (int t = 0; t < 4; ++t) {
              const float v0 = __uint_as_float(wd[t] << 16), v1 = __uint_as_float(wd[t] & 0xffff0000u);
              nrm[j] += v0 * v0 + v1 * v1;
            }
          }
#pragma unroll
          for (int i = 0; i < NB16; ++i)
#pragma unroll
            for (int j = 0; j < NC16; ++j)
              acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[i], bfv[j], acc[i][j], 0, 0, 0);
        } else {
          long af[NB16], bfv[NC16];
          lds_frags_b64(la, lb, af, bfv);
#pragma unroll
          for (int j = 0; j < NC16; ++j) {
            const int lo32 = (int)(uint32_t)bfv[j], hi32 = (int)(uint32_t)((uint64_t)bfv[j] >> 32);
            const float v[8] = {
                __builtin_amdgcn_cvt_f32_fp8(lo32, 0), __builtin_amdgcn_cvt_f32_fp8(lo32, 1),
                __builtin_amdgcn_cvt_f32_fp8(lo32, 2), __builtin_amdgcn_cvt_f32_fp8(lo32, 3),
                __builtin_amdgcn_cvt_f32_fp8(hi32, 0), __builtin_amdgcn_cvt_f32_fp8(hi32, 1),
                __builtin_amdgcn_cvt_f32_fp8(hi32, 2), __builtin_amdgcn_cvt_f32_fp8(hi32, 3)};
#pragma unroll
            for (int t = 0; t < 8; ++t) nrm[j] += v[t] * v[t];
          }
#pragma unroll
          for (int i = 0; i < NB16; ++i)
#pragma unroll
            for (int j = 0; j < NC16; ++j)
              acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8(af[i], bfv[j], acc[i][j], 0, 0, 0);
        }
      }
    };
    __builtin_amdgcn_s_waitcnt(vm_wait_imm(0));  // the previous item's stores first
    constexpr int NCOPY = NA + NBV;  // copies per lane and stage
    for (int p = 0; p < NST - 1 && p < nstage; ++p) issue(p, Ar[p], Br[p]);
    for (int s = 0; s < nstage; ++s) {
      const int j = s % NST;
      // this wave's copies of stage s have landed; those of stage s + 1 (issued
      // after them, and counted in order) may still be in flight
      if (s + 1 < nstage) __builtin_amdgcn_s_waitcnt(vm_wait_imm(NCOPY));
      else __builtin_amdgcn_s_waitcnt(vm_wait_imm(0));
      // LDS-only barrier: stage s has landed for every wave, and every wave's
      // reads of stage s - 1 (whose buffer is refilled next) have returned
      __builtin_amdgcn_s_waitcnt(0xC07F);  // lgkmcnt(0), other counters free
      __builtin_amdgcn_s_barrier();
      if (s + NST - 1 < nstage) issue(s + NST - 1, Ar[(s + NST - 1) % NST], Br[(s + NST - 1) % NST]);
      if (a.d_dot - s * SC < SC) clip(Ar[j], Br[j], a.d_dot - s * SC);
      if (active) compute(Ar[j], Br[j]);
    }
    // norms: the four lane groups of a column hold its coordinate ranges
#pragma unroll
    for (int j = 0; j < NC16; ++j) {
      nrm[j] += __shfl_xor(nrm[j], 16);
      nrm[j] += __shfl_xor(nrm[j], 32);
      if (wv < 2 && active && lane < 16) cn[cbw + j * 16 + lane] = nrm[j];
    }
    __syncthreads();
    // 16x16 f32 MFMA result: lane holds column (lane & 15), rows 4 (lane >> 4) + e
#pragma unroll
    for (int i = 0; i < NB16; ++i)
#pragma unroll
      for (int j = 0; j < NC16; ++j)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int row = rbw + i * 16 + 4 * (lane >> 4) + e;
          const int col = cbw + j * 16 + (lane & 15);
          if (rq[row] >= 0 && col < ncol) {
            const float sx = csc[col], sq = rsc[row];
            a.out[rbase[row] + vt * TV + col] = sx * sx * cn[col] - 2.0f * sq * sx * acc[i][j][e];
          }
        }
  }
}

// ---- probe bucketing (batched) -------------------------------------------------
__global__ void k_store_cfg(CfgDev c, CfgDev *dst) { *dst = c; }

// cnt[virtual list of each pair] += 1
__global__ void k_count(const int32_t *__restrict__ probes, int64_t npairs, const CfgDev *cfg,
                        int32_t ncfg, int32_t *__restrict__ cnt) {
  int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= npairs) return;
  const int c = cfg_of(cfg, ncfg, &CfgDev::pair0, p);
  atomicAdd(&cnt[cfg[c].vl0 + probes[p]], 1);
}

// The same two passes with the counting done per workgroup in LDS first
// (BKT_CHUNK pairs per workgroup), so that each workgroup makes one global
// atomic per list it touches instead of one per pair: the list counters
// share few cache lines, and per-pair atomics on them serialise.
constexpr int BKT_CHUNK = 8192;       // pairs per workgroup
constexpr int BKT_LDS_BINS = 8192;    // virtual lists an LDS histogram holds (32 KB)

__global__ __launch_bounds__(1024) void k_count_lds(const int32_t *__restrict__ probes,
                                                    int64_t npairs, const CfgDev *cfg,
                                                    int32_t ncfg, int32_t V,
                                                    int32_t *__restrict__ cnt) {
  extern __shared__ int32_t hist[];  // [V]
  const int tid = threadIdx.x;
  for (int i = tid; i < V; i += 1024) hist[i] = 0;
  __syncthreads();
  const int64_t p0 = (int64_t)blockIdx.x * BKT_CHUNK, p1 = min64(npairs, p0 + BKT_CHUNK);
  for (int64_t p = p0 + tid; p < p1; p += 1024) {
    const int c = cfg_of(cfg, ncfg, &CfgDev::pair0, p);
    atomicAdd(&hist[cfg[c].vl0 + probes[p]], 1);
  }
  __syncthreads();
  for (int i = tid; i < V; i += 1024) {
    const int32_t h = hist[i];
    if (h) atomicAdd(&cnt[i], h);
  }
}

// bucket[bkt_off[v] + slot] = p for the pairs p of virtual list v: a
// workgroup ranks its pairs per list in LDS, reserves one run of slots per
// list with one atomic on cursor[v], then writes.
__global__ __launch_bounds__(1024) void k_scatter_lds(const int32_t *__restrict__ probes,
                                                      int64_t npairs, const CfgDev *cfg,
                                                      int32_t ncfg, int32_t V,
                                                      const int32_t *__restrict__ bkt_off,
                                                      int32_t *__restrict__ cursor,
                                                      int32_t *__restrict__ bucket) {
  extern __shared__ int32_t hist[];  // [V]: counts, then each list's run start
  constexpr int PER = BKT_CHUNK / 1024;
  const int tid = threadIdx.x;
  for (int i = tid; i < V; i += 1024) hist[i] = 0;
  __syncthreads();
  const int64_t p0 = (int64_t)blockIdx.x * BKT_CHUNK, p1 = min64(npairs, p0 + BKT_CHUNK);
  int32_t vv[PER], rk[PER];
#pragma unroll
  for (int j = 0; j < PER; ++j) {
    const int64_t p = p0 + tid + 1024 * j;
    vv[j] = -1;
    rk[j] = 0;
    if (p < p1) {
      const int c = cfg_of(cfg, ncfg, &CfgDev::pair0, p);
      vv[j] = cfg[c].vl0 + probes[p];
      rk[j] = atomicAdd(&hist[vv[j]], 1);
    }
  }
  __syncthreads();
  for (int i = tid; i < V; i += 1024) {
    const int32_t h = hist[i];
    if (h) hist[i] = atomicAdd(&cursor[i], h);
  }
  __syncthreads();
#pragma unroll
  for (int j = 0; j < PER; ++j)
    if (vv[j] >= 0) bucket[bkt_off[vv[j]] + hist[vv[j]] + rk[j]] = (int32_t)(p0 + tid + 1024 * j);
}

// One workgroup of 1024 threads: bucket offsets, tile prefix (query tiles of
// height tq x tv-vector tiles per virtual list), cursor and scan work counter
// reset.
__global__ __launch_bounds__(1024) void k_list_scan(const int32_t *__restrict__ cnt,
                                                    const CfgDev *cfg, int32_t ncfg, int32_t V,
                                                    int32_t tq, int32_t tv,
                                                    int32_t *__restrict__ bkt_off,
                                                    int32_t *__restrict__ tile_off,
                                                    int32_t *__restrict__ cursor,
                                                    int32_t *__restrict__ work) {
  __shared__ int32_t sh[16];
  const int tid = threadIdx.x;
  if (tid < 8) work[tid] = 0;
  const int chunk = (V + blockDim.x - 1) / blockDim.x;
  const int v0 = tid * chunk, v1 = min(V, v0 + chunk);
  auto tiles = [&](int v) {
    const int c = cfg_of(cfg, ncfg, &CfgDev::vl0, v);
    const int32_t len = cfg[c].len[v - cfg[c].vl0];
    return ((cnt[v] + tq - 1) / tq) * ((len + tv - 1) / tv);
  };
  int32_t sc = 0, st = 0;
  for (int v = v0; v < v1; ++v) {
    sc += cnt[v];
    st += tiles(v);
  }
  int32_t tot_t;
  int32_t ec = block_excl_scan<int32_t>(sc, sh, nullptr);
  int32_t et = block_excl_scan<int32_t>(st, sh, &tot_t);
  for (int v = v0; v < v1; ++v) {
    bkt_off[v] = ec;
    tile_off[v] = et;
    cursor[v] = 0;
    ec += cnt[v];
    et += tiles(v);
  }
  if (tid == 0) tile_off[V] = tot_t;
}

__global__ void k_scatter(const int32_t *__restrict__ probes, int64_t npairs, const CfgDev *cfg,
                          int32_t ncfg, const int32_t *__restrict__ bkt_off,
                          int32_t *__restrict__ cursor, int32_t *__restrict__ bucket) {
  int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= npairs) return;
  const int c = cfg_of(cfg, ncfg, &CfgDev::pair0, p);
  const int32_t v = cfg[c].vl0 + probes[p];
  bucket[bkt_off[v] + atomicAdd(&cursor[v], 1)] = (int32_t)p;
}

// Candidates of every query row of the batch (sum of its probed list lengths).
__global__ void k_seg_len(const int32_t *__restrict__ probes, int64_t Qtot, const CfgDev *cfg,
                          int32_t ncfg, int64_t *__restrict__ seg_len) {
  int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= Qtot) return;
  const int c = cfg_of(cfg, ncfg, &CfgDev::q0, r);
  const CfgDev &g = cfg[c];
  const int32_t *pr = probes + g.pair0 + (r - g.q0) * g.nprobe;
  int64_t s = 0;
  for (int j = 0; j < g.nprobe; ++j) s += g.len[pr[j]];
  seg_len[r] = s;
}

// One workgroup: out[0..n] = exclusive prefix of in[0..n).
__global__ __launch_bounds__(1024) void k_scan_i64(const int64_t *__restrict__ in, int64_t n,
                                                   int64_t *__restrict__ out) {
  // tiles of 1024 x R values: thread t holds R consecutive values of a tile
  // (coalesced across the block, every load of a tile in flight at once)
  __shared__ int64_t sh[16];
  constexpr int R = 8;
  const int tid = threadIdx.x;
  int64_t carry = 0;
  for (int64_t base = 0; base < n; base += 1024 * R) {
    int64_t v[R], s = 0;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int64_t i = base + (int64_t)tid * R + r;
      v[r] = i < n ? in[i] : 0;
      s += v[r];
    }
    int64_t tot;
    int64_t e = carry + block_excl_scan<int64_t>(s, sh, &tot);
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int64_t i = base + (int64_t)tid * R + r;
      if (i < n) out[i] = e;
      e += v[r];
    }
    carry += tot;
  }
  if (tid == 0) out[n] = carry;
}

__global__ void k_pair_base(const int32_t *__restrict__ probes, int64_t Qtot, const CfgDev *cfg,
                            int32_t ncfg, const int64_t *__restrict__ seg_off,
                            int64_t *__restrict__ pair_base) {
  int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= Qtot) return;
  const int c = cfg_of(cfg, ncfg, &CfgDev::q0, r);
  const CfgDev &g = cfg[c];
  const int64_t p0 = g.pair0 + (r - g.q0) * g.nprobe;
  int64_t s = seg_off[r];
  for (int j = 0; j < g.nprobe; ++j) {
    pair_base[p0 + j] = s;
    s += g.len[probes[p0 + j]];
  }
}

inline unsigned blocks_for(int64_t n, int t) { return (unsigned)((n + t - 1) / t); }

}  // namespace

// ---- launch wrappers -------------------------------------------------------------
__global__ void k_stage_multi(const float *__restrict__ Q, int64_t ldq, const CfgDev *cfg,
                              int32_t ncfg, int64_t Qtot, float *__restrict__ Qs, int64_t ldqs) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t r = i / ldqs, col = i % ldqs;
  if (r >= Qtot) return;
  const int c = cfg_of(cfg, ncfg, &CfgDev::q0, r);
  const int32_t dq = max(cfg[c].d_c, cfg[c].d_s);
  Qs[i] = col < dq ? Q[r * ldq + col] : 0.0f;
}

static int32_t next_pow2(int32_t v) {
  int32_t p = 1;
  while (p < v) p <<= 1;
  return p;
}

constexpr int32_t SEG_LDS_CAP = 16384;   // at most this many first-pass distances staged

// Dynamic LDS a selection workgroup may use: the device's per-workgroup limit
// less the kernels' static LDS (the function attribute is raised to it when it
// exceeds the 64 KB default; if that fails, 64 KB less the static LDS).
static size_t sel_smem_budget() {
  static std::once_flag once;
  static size_t budget = 48 * 1024;
  std::call_once(once, [] {
    const void *fns[] = {(const void *)k_select_refine, (const void *)k_select_multi,
                         (const void *)k_select_refine_redo, (const void *)k_select_multi_redo};
    int dev = 0, v = 0;
    size_t per_block = 64 * 1024, stat = 0;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) == hipSuccess &&
        v > 0)
      per_block = (size_t)v;
    for (const void *f : fns) {
      hipFuncAttributes fa;
      if (hipFuncGetAttributes(&fa, f) == hipSuccess) stat = std::max(stat, fa.sharedSizeBytes);
    }
    stat = (stat + 255) / 256 * 256;
    const size_t dflt = 64 * 1024 - stat;
    size_t dyn = per_block > stat ? per_block - stat : 0;
    if (dyn > dflt) {
      bool ok = true;
      for (const void *f : fns)
        ok = ok && hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)dyn) ==
                       hipSuccess;
      if (!ok) dyn = dflt;
    }
    budget = dyn;
    (void)hipGetLastError();
  });
  return budget;
}

// Segment floats that fit beside the histogram and kcap candidate slots.
static int32_t seg_cap(int32_t kcap, int64_t max_len) {
  const int64_t room = ((int64_t)sel_smem_budget() - (int64_t)sel_smem_bytes(0, kcap)) / 4;
  const int64_t cap = std::min<int64_t>({(int64_t)SEG_LDS_CAP, room / 256 * 256, max_len});
  return (int32_t)std::max<int64_t>(cap, 0);
}

// Candidate slots of the re-selection launches: the most that fit the LDS
// budget (up to 4096), so that only a band of more candidates than that
// leaves a result uncertified.
static int32_t redo_kcap() {
  int32_t k = 4096;
  while (k > 64 && sel_smem_bytes(0, k) > sel_smem_budget()) k >>= 1;
  return k;
}

hipError_t read_selection_stats(unsigned long long out[2], int first, bool reset) {
  const size_t off = (size_t)first * sizeof(unsigned long long), n = 2 * sizeof(unsigned long long);
  hipError_t e = hipDeviceSynchronize();
  if (e == hipSuccess) e = hipMemcpyFromSymbol(out, HIP_SYMBOL(g_sel_stats), n, off);
  if (e == hipSuccess && reset) {
    const unsigned long long z[2] = {0ull, 0ull};
    e = hipMemcpyToSymbol(HIP_SYMBOL(g_sel_stats), z, n, off);
  }
  return e;
}

// Workgroups of a re-selection launch (it strides over its list).
static unsigned redo_grid(int64_t nq) { return (unsigned)std::max<int64_t>(1, std::min<int64_t>(nq, 512)); }

// Zeroes the two re-selection counters of a search (a fill kernel, not a
// memset: searches may be captured into graphs).
static void reset_redo(int32_t *redo, hipStream_t st) {
  if (redo) hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(64), 0, st, redo, (int64_t)2, 0);
}

// One query per wave when the first shortlist fits the lanes and either the
// exact measures are short (one wave measures the candidates one after
// another) or the batch holds enough queries to give every SIMD two waves
// (measured: the precision form's re-rank of 32 at d_s 2048, 147k
// coordinates per query, 24 % faster than one workgroup per query on 50k
// queries); else one workgroup of eight waves per query.
// ``redo_cnt`` / ``redo_list`` (nq entries) collect the queries whose
// shortlist the first launch cannot certify; the re-selection launch that
// follows takes them with the widest shortlist. NULL: no re-selection.
static void launch_select(SelArgs s, int64_t nq, size_t smem, int32_t *redo_cnt,
                          int32_t *redo_list, hipStream_t st) {
  if (nq == 0) return;
  const int64_t measure = (int64_t)s.K1 * s.d_dot + (s.stageB ? (int64_t)s.K2 * s.d_B : 0);
  const bool many = nq >= 2048;
  s.redo_cnt = redo_cnt;
  s.redo_list = redo_cnt ? redo_list : nullptr;
  s.redo_q0 = 0;
  if (s.K1 <= WSEL_K && s.kout <= WSEL_K &&
      (measure <= 96 * 1024 || (many && measure <= 512 * 1024)))
    hipLaunchKernelGGL(k_select_refine_wave, dim3((unsigned)cdiv(nq, 4)), dim3(256), 0, st, s, nq);
  else if (s.mode == SEL_QUANT && s.stageB && s.qrerr != nullptr && s.qerr != nullptr &&
           s.d_B == s.d_dot && s.kout <= s.K2 && s.kout <= QRR_CAP && redo_cnt != nullptr)
    hipLaunchKernelGGL(k_select_qrerank, dim3((unsigned)nq), dim3(256), 0, st, s);
  else
    hipLaunchKernelGGL(k_select_refine, dim3((unsigned)nq), dim3(512), smem, st, s);
  if (redo_cnt) {
    s.kcap = redo_kcap();
    s.lcap = seg_cap(s.kcap, SEG_LDS_CAP);
    hipLaunchKernelGGL(k_select_refine_redo, dim3(redo_grid(nq)), dim3(512),
                       sel_smem_bytes(s.lcap, s.kcap), st, s);
  }
}

// Sets the LDS caps of a single-configuration selection; returns its bytes.
static size_t sel_caps(SelArgs &s, int64_t max_len) {
  s.kcap = next_pow2(std::max(std::max(s.K1, s.kout), 1));
  s.lcap = seg_cap(s.kcap, max_len);
  return sel_smem_bytes(s.lcap, s.kcap);
}

CfgDev make_cfg(const adanns_index *ix, int32_t d_c, int32_t d_s, int32_t nprobe, int32_t k,
                int64_t nq) {
  CfgDev c{};
  c.vec = ix->vec;
  c.rows = ix->rows;
  c.xmax2 = ix->xmax2;
  c.cmax2 = ix->cmax2;
  c.poff = ix->poff;
  c.len = ix->len;
  c.rowid = ix->rowid;
  c.cent = ix->cent;
  c.cent_slab = ix->cent_slab;
  c.d_pad = ix->d_pad;
  c.d_cb_pad = ix->d_cb_pad;
  c.nlist = ix->nlist;
  c.nl_pad = ix->nl_pad;
  c.d_c = d_c;
  c.d_s = d_s;
  c.nprobe = nprobe;
  c.k = k;
  c.q0 = 0;
  c.nq = nq;
  c.S0 = 0;
  c.pair0 = 0;
  c.vl0 = 0;
  c.ct0 = 0;
  c.qtiles = (int32_t)cdiv(nq, TILE_Q);
  return c;
}

hipError_t launch_store_cfg(const CfgDev &c, CfgDev *dst, hipStream_t st) {
  hipLaunchKernelGGL(k_store_cfg, dim3(1), dim3(1), 0, st, c, dst);
  return hipGetLastError();
}

hipError_t launch_stage_queries(const float *Q, int64_t nq, int64_t ldq, int32_t dq, float *Qs,
                                int64_t ldqs, hipStream_t st) {
  int64_t n = nq * ldqs;
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_stage_queries, dim3(blocks_for(n, 256)), dim3(256), 0, st, Q, nq, ldq, dq,
                     Qs, ldqs);
  return hipGetLastError();
}

hipError_t launch_layout(const Mat &src, int32_t dsrc, const int64_t *src_row,
                         const int32_t *row_list, const int64_t *poff, int64_t rows_pad,
                         int32_t d_pad, float *dst, hipStream_t st) {
  int64_t n = rows_pad * d_pad;
  if (n == 0) return hipSuccess;
  if (src.type == 1)
    hipLaunchKernelGGL(k_layout<_Float16>, dim3(blocks_for(n, 256)), dim3(256), 0, st,
                       (const _Float16 *)src.p, src.ld, dsrc, src_row, row_list, poff, rows_pad,
                       d_pad, dst);
  else
    hipLaunchKernelGGL(k_layout<float>, dim3(blocks_for(n, 256)), dim3(256), 0, st,
                       (const float *)src.p, src.ld, dsrc, src_row, row_list, poff, rows_pad,
                       d_pad, dst);
  return hipGetLastError();
}

hipError_t launch_stage_rows(const Mat &X, const int64_t *rows, const int32_t *rows32,
                             int64_t nrows, int32_t dcols, float *out, int64_t ldo,
                             hipStream_t st) {
  int64_t n = nrows * ldo;
  if (n == 0) return hipSuccess;
  if (X.type == 1)
    hipLaunchKernelGGL(k_stage_rows<_Float16>, dim3(blocks_for(n, 256)), dim3(256), 0, st,
                       (const _Float16 *)X.p, X.ld, rows, rows32, nrows, dcols, out, ldo);
  else
    hipLaunchKernelGGL(k_stage_rows<float>, dim3(blocks_for(n, 256)), dim3(256), 0, st,
                       (const float *)X.p, X.ld, rows, rows32, nrows, dcols, out, ldo);
  return hipGetLastError();
}

hipError_t launch_centroid_update(const float *X, int64_t ldx, const int32_t *perm,
                                  const int64_t *off, int32_t nlist, int32_t dcols, float *C,
                                  int64_t ldc, hipStream_t st) {
  KernelTimer tm("kmeans_update", st);
  hipLaunchKernelGGL(k_centroid_update, dim3(nlist, blocks_for(dcols, 256)), dim3(256), 0, st, X,
                     ldx, perm, off, dcols, C, ldc);
  return hipGetLastError();
}

// Coarse step of a batch whose descriptors are in b.cfg (b.Qs already staged).
static hipError_t coarse_multi(const SearchBufs &b, int32_t *user_probes, float *out_min_dist,
                               int32_t grid_cap, hipStream_t st) {
  TileArgs t{};
  t.cfg = b.cfg;
  t.ncfg = b.ncfg;
  t.Qs = b.Qs;
  t.ldqs = b.ldqs;
  t.S = b.S;
  t.ct_total = b.ct_total;
  const int grid = (int)std::min<int64_t>(grid_cap, round_up(b.ct_total, 8));
  {
    KernelTimer tm("tile_dist_coarse", st);
    hipLaunchKernelGGL((k_tile_multi<TILE_Q, TILE_V, 1>), dim3(grid), dim3(256), 0, st, t);
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  SelMultiArgs m{};
  m.cfg = b.cfg;
  m.ncfg = b.ncfg;
  m.coarse = 1;
  m.Qs = b.Qs;
  m.ldqs = b.ldqs;
  m.S = b.S;
  m.probes = b.probes;
  m.user_probes = user_probes;
  m.dist = out_min_dist;
  m.kcap = next_pow2(std::min(b.max_nlist, std::min(b.max_nprobe + REFINE_MARGIN, MAX_SHORTLIST)));
  m.lcap = seg_cap(m.kcap, b.max_nlist);
  m.redo = b.redo;
  {
    KernelTimer tm("select_coarse", st);
    if (b.max_nprobe + REFINE_MARGIN <= WSEL_K)
      hipLaunchKernelGGL(k_select_wave<true>, dim3((unsigned)cdiv(b.Qtot, 4)), dim3(256), 0, st, m,
                         b.Qtot);
    else
      hipLaunchKernelGGL(k_select_multi, dim3((unsigned)b.Qtot), dim3(512),
                         sel_smem_bytes(m.lcap, m.kcap), st, m);
    if (b.redo) {
      m.kcap = redo_kcap();
      m.lcap = seg_cap(m.kcap, b.max_nlist);
      hipLaunchKernelGGL(k_select_multi_redo, dim3(redo_grid(b.Qtot)), dim3(512),
                         sel_smem_bytes(m.lcap, m.kcap), st, m);
    }
  }
  return hipGetLastError();
}

static hipError_t bucketing_multi(const SearchBufs &b, int32_t tq, int32_t tv, hipStream_t st) {
  KernelTimer tmb("bucketing", st);
  hipLaunchKernelGGL(k_fill_i32, dim3(blocks_for(b.V, 256)), dim3(256), 0, st, b.cnt,
                     (int64_t)b.V, 0);
  const bool lds = b.V <= BKT_LDS_BINS;
  const unsigned gl = (unsigned)std::max<int64_t>(1, cdiv(b.pairs, BKT_CHUNK));
  const size_t hb = (size_t)b.V * sizeof(int32_t);
  if (lds)
    hipLaunchKernelGGL(k_count_lds, dim3(gl), dim3(1024), hb, st, b.probes, b.pairs, b.cfg, b.ncfg,
                       b.V, b.cnt);
  else
    hipLaunchKernelGGL(k_count, dim3(blocks_for(b.pairs, 256)), dim3(256), 0, st, b.probes,
                       b.pairs, b.cfg, b.ncfg, b.cnt);
  hipLaunchKernelGGL(k_list_scan, dim3(1), dim3(1024), 0, st, b.cnt, b.cfg, b.ncfg, b.V, tq, tv,
                     b.bkt_off, b.tile_off, b.cursor, b.work);
  if (lds)
    hipLaunchKernelGGL(k_scatter_lds, dim3(gl), dim3(1024), hb, st, b.probes, b.pairs, b.cfg,
                       b.ncfg, b.V, b.bkt_off, b.cursor, b.bucket);
  else
    hipLaunchKernelGGL(k_scatter, dim3(blocks_for(b.pairs, 256)), dim3(256), 0, st, b.probes,
                       b.pairs, b.cfg, b.ncfg, b.bkt_off, b.cursor, b.bucket);
  // per-query segment lengths go to pair_base as a temporary, then the scan
  hipLaunchKernelGGL(k_seg_len, dim3(blocks_for(b.Qtot, 256)), dim3(256), 0, st, b.probes, b.Qtot,
                     b.cfg, b.ncfg, b.pair_base);
  hipLaunchKernelGGL(k_scan_i64, dim3(1), dim3(1024), 0, st, b.pair_base, b.Qtot, b.seg_off);
  hipLaunchKernelGGL(k_pair_base, dim3(blocks_for(b.Qtot, 256)), dim3(256), 0, st, b.probes,
                     b.Qtot, b.cfg, b.ncfg, b.seg_off, b.pair_base);
  tmb.stop();
  return hipGetLastError();
}

hipError_t launch_coarse(const adanns_index *ix, const SearchBufs &b, int64_t nq, int32_t d_c,
                         int32_t nprobe, int32_t *user_probes, hipStream_t st,
                         float *out_min_dist) {
  const CfgDev c = make_cfg(ix, d_c, 0, nprobe, 0, nq);
  hipError_t e = launch_store_cfg(c, b.cfg, st);
  if (e != hipSuccess) return e;
  reset_redo(b.redo, st);
  SearchBufs bb = b;
  bb.ncfg = 1;
  bb.Qtot = nq;
  bb.ct_total = c.qtiles * (int32_t)cdiv(ix->nlist, TILE_V);
  bb.max_nlist = ix->nlist;
  bb.max_nprobe = nprobe;
  return coarse_multi(bb, user_probes, out_min_dist, PERSIST_WG, st);
}

hipError_t launch_bucketing(const adanns_index *ix, const SearchBufs &b, int64_t nq,
                            int32_t nprobe, hipStream_t st, int32_t tq, int32_t tv) {
  SearchBufs bb = b;
  bb.ncfg = 1;
  bb.V = ix->nlist;
  bb.Qtot = nq;
  bb.pairs = nq * nprobe;
  return bucketing_multi(bb, tq, tv, st);
}

template <int TQ, int TV>
static void launch_scan_tiles(const TileArgs &t, int grid, hipStream_t st) {
  hipLaunchKernelGGL((k_tile_multi<TQ, TV, 0>), dim3(grid), dim3(256), 0, st, t);
}

hipError_t launch_search_multi(const SearchBufs &b, const float *Q, int64_t ldq, float *dist,
                               int64_t *ids, int64_t ldk, int32_t *user_probes, int32_t tq,
                               int32_t tv, int32_t grid, hipStream_t st, bool do_coarse) {
  if (tq != 32 && tq != 128) tq = 64;
  if (tv != 128) tv = 64;
  reset_redo(b.redo, st);
  // The kernels read query rows through 16-byte loads up to the 32-coordinate
  // slab that holds the last coordinate they use, and mask what lies past it;
  // rows that are 16-byte aligned and at least that wide are read in place,
  // others are first staged into zero-padded rows.
  SearchBufs bq = b;
  if (ldq % 4 == 0 && ((uintptr_t)Q & 15) == 0 && ldq >= b.ldqs) {
    bq.Qs = const_cast<float *>(Q);
    bq.ldqs = ldq;
  } else {
    const int64_t n = b.Qtot * b.ldqs;
    KernelTimer tm("stage_queries", st);
    hipLaunchKernelGGL(k_stage_multi, dim3(blocks_for(n, 256)), dim3(256), 0, st, Q, ldq, b.cfg,
                       b.ncfg, b.Qtot, b.Qs, b.ldqs);
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (do_coarse && (e = coarse_multi(bq, user_probes, nullptr, PERSIST_WG, st)) != hipSuccess)
    return e;
  if ((e = bucketing_multi(bq, tq, tv, st)) != hipSuccess) return e;
  TileArgs t{};
  t.cfg = b.cfg;
  t.ncfg = b.ncfg;
  t.Qs = bq.Qs;
  t.ldqs = bq.ldqs;
  t.V = b.V;
  t.tile_off = b.tile_off;
  t.bkt_off = b.bkt_off;
  t.cnt = b.cnt;
  t.bucket = b.bucket;
  t.pair_base = b.pair_base;
  t.D = b.D;
  t.work = b.work;
  grid = (int)round_up(std::max(8, grid), 8);
  // no more workgroups than the work items can occupy (small batches)
  if (b.max_items > 0) grid = (int)std::min<int64_t>(grid, round_up(std::max<int64_t>(8, b.max_items), 8));
  {
    KernelTimer tm("tile_dist_scan", st);
    if (tv == 128) {
      if (tq == 32) launch_scan_tiles<32, 128>(t, grid, st);
      else if (tq == 128) launch_scan_tiles<128, 128>(t, grid, st);
      else launch_scan_tiles<64, 128>(t, grid, st);
    } else {
      if (tq == 32) launch_scan_tiles<32, 64>(t, grid, st);
      else if (tq == 128) launch_scan_tiles<128, 64>(t, grid, st);
      else launch_scan_tiles<64, 64>(t, grid, st);
    }
  }
  if ((e = hipGetLastError()) != hipSuccess) return e;
  SelMultiArgs m{};
  m.cfg = b.cfg;
  m.ncfg = b.ncfg;
  m.coarse = 0;
  m.Qs = bq.Qs;
  m.ldqs = bq.ldqs;
  m.D = b.D;
  m.seg_off = b.seg_off;
  m.probes = b.probes;
  m.pair_base = b.pair_base;
  m.dist = dist;
  m.ids = ids;
  m.ldk = ldk;
  m.kcap = next_pow2(std::min(b.max_k + REFINE_MARGIN, MAX_SHORTLIST));
  m.lcap = seg_cap(m.kcap, SEG_LDS_CAP);
  m.redo = b.redo;
  {
    KernelTimer tm("select_scan", st);
    if (b.max_k + REFINE_MARGIN <= WSEL_K && b.Qtot <= SELW_WIDE_MAX)
      hipLaunchKernelGGL((k_select_wave<false, true>), dim3((unsigned)cdiv(b.Qtot, 4)), dim3(256),
                         0, st, m, b.Qtot);
    else if (b.max_k + REFINE_MARGIN <= WSEL_K)
      hipLaunchKernelGGL(k_select_wave<false>, dim3((unsigned)cdiv(b.Qtot, 4)), dim3(256), 0, st, m,
                         b.Qtot);
    else
      hipLaunchKernelGGL(k_select_multi, dim3((unsigned)b.Qtot), dim3(512),
                         sel_smem_bytes(m.lcap, m.kcap), st, m);
  }
  if (b.redo) {
    KernelTimer tm("select_redo", st);
    m.kcap = redo_kcap();
    m.lcap = seg_cap(m.kcap, SEG_LDS_CAP);
    hipLaunchKernelGGL(k_select_multi_redo, dim3(redo_grid(b.Qtot)), dim3(512),
                       sel_smem_bytes(m.lcap, m.kcap), st, m);
  }
  return hipGetLastError();
}

// Row-major copy of the slab layout: rows[g][dim] = coordinate dim of layout
// row g (list order). One block column per list; coalesced writes.
__global__ void k_slab_to_rows(const float *__restrict__ vec, const int64_t *__restrict__ poff,
                               int32_t d_pad, float *__restrict__ rows) {
  const int h = blockIdx.y;
  const int64_t p0 = poff[h], np = poff[h + 1] - p0;
  const float *src = vec + p0 * d_pad;
  float *dst = rows + p0 * d_pad;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < np * d_pad;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = i / d_pad;
    const int dim = (int)(i - r * d_pad);
    dst[i] = src[(int64_t)(dim / SLAB) * np * SLAB + r * SLAB + dim % SLAB];
  }
}

hipError_t launch_slab_to_rows(const adanns_index *ix, float *rows, hipStream_t st) {
  if (ix->nlist == 0) return hipSuccess;
  const int64_t per_list = std::max<int64_t>(1, (int64_t)ix->max_len * ix->d_pad);
  const unsigned bx = (unsigned)std::min<int64_t>(64, cdiv(per_list, 256));
  hipLaunchKernelGGL(k_slab_to_rows, dim3(bx, (unsigned)ix->nlist), dim3(256), 0, st, ix->vec,
                     ix->poff, ix->d_pad, rows);
  return hipGetLastError();
}

// Largest squared norm over the rows of the slab layout (padding rows are
// zero): block h covers list h, each half-wave one row at a time with its 32
// lanes across the slab width. Non-negative floats order as their bit
// patterns, so the maximum is taken with an integer atomic.
__global__ __launch_bounds__(256) void k_row_norm_max(const float *__restrict__ vec,
                                                      const int64_t *__restrict__ poff,
                                                      int32_t d_pad, uint32_t *__restrict__ out) {
  __shared__ float sh[8];
  const int h = blockIdx.x, half = threadIdx.x >> 5, l = threadIdx.x & 31;
  const int64_t p0 = poff[h], np = poff[h + 1] - p0;
  const float *src = vec + p0 * d_pad;
  const int nslab = d_pad / SLAB;
  float best = 0.f;
  for (int64_t r = half; r < np; r += 8) {
    float s = 0.f;
    for (int k = 0; k < nslab; ++k) {
      const float x = src[((int64_t)k * np + r) * SLAB + l];
      s = fmaf(x, x, s);
    }
    for (int o = 16; o > 0; o >>= 1) s += __shfl_xor(s, o, 32);
    best = fmaxf(best, s);
  }
  if (l == 0) sh[half] = best;
  __syncthreads();
  if (threadIdx.x == 0) {
    float m = sh[0];
    for (int i = 1; i < 8; ++i) m = fmaxf(m, sh[i]);
    atomicMax(out, __float_as_uint(m));
  }
}

// Read-only streaming probe: every byte of buf read once with 16-byte
// non-temporal loads (streamed past the caches), four in flight per thread,
// consecutive threads on consecutive 16-byte pieces (each wave reads 1 KB
// contiguous per load); each workgroup writes the sum of what it read, so
// that no load can be dropped. (Measured on 4 GiB: plain loads reach 5.3 TB/s
// with 1024 workgroups and 6.2 TB/s with 32768; non-temporal loads 5.7 and
// 7.0 TB/s.)
__global__ __launch_bounds__(256) void k_stream_read(const floatx4 *__restrict__ buf, int64_t n4,
                                                     float *__restrict__ out) {
  __shared__ float sh[4];
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  floatx4 acc = {0.f, 0.f, 0.f, 0.f};
  for (; i + 3 * stride < n4; i += 4 * stride) {
    const floatx4 a = __builtin_nontemporal_load(buf + i);
    const floatx4 b = __builtin_nontemporal_load(buf + i + stride);
    const floatx4 c = __builtin_nontemporal_load(buf + i + 2 * stride);
    const floatx4 d = __builtin_nontemporal_load(buf + i + 3 * stride);
    acc += (a + b) + (c + d);
  }
  for (; i < n4; i += stride) acc += __builtin_nontemporal_load(buf + i);
  float v = (acc[0] + acc[1]) + (acc[2] + acc[3]);
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) out[blockIdx.x] = (sh[0] + sh[1]) + (sh[2] + sh[3]);
}

hipError_t launch_stream_read(const void *buf, size_t bytes, float *out, int32_t grid,
                              hipStream_t st) {
  hipLaunchKernelGGL(k_stream_read, dim3((unsigned)grid), dim3(256), 0, st, (const floatx4 *)buf,
                     (int64_t)(bytes / 16), out);
  return hipGetLastError();
}

hipError_t launch_row_norm_max(const float *vec, const int64_t *poff, int32_t nlists,
                               int32_t d_pad, float *out, hipStream_t st) {
  hipError_t e = hipMemsetAsync(out, 0, sizeof(float), st);
  if (e != hipSuccess || nlists == 0) return e;
  hipLaunchKernelGGL(k_row_norm_max, dim3((unsigned)nlists), dim3(256), 0, st, vec, poff, d_pad,
                     (uint32_t *)out);
  return hipGetLastError();
}

hipError_t launch_quantize_store(const adanns_index *ix, int32_t fmt, QuantStore &qs,
                                 hipStream_t st) {
  if (fmt == 1) {
    const int64_t nv = ix->rows_pad * ix->d_pad, nc = (int64_t)ix->nl_pad * ix->d_cb_pad;
    hipLaunchKernelGGL(k_quant_bf16, dim3(blocks_for(nv, 256)), dim3(256), 0, st, ix->vec, nv,
                       (uint16_t *)qs.vec);
    hipLaunchKernelGGL(k_quant_bf16, dim3(blocks_for(nc, 256)), dim3(256), 0, st, ix->cent_slab,
                       nc, (uint16_t *)qs.cent);
    return hipGetLastError();
  }
  hipLaunchKernelGGL(k_quant_fp8_slab, dim3(blocks_for(ix->rows_pad, 4)), dim3(256), 0, st,
                     ix->vec, ix->poff, ix->nlist, ix->rows_pad, ix->d_pad, ix->d,
                     (uint8_t *)qs.vec, qs.scale);
  // the centroids are quantised by launch_quantize_cent_fp8
  return hipGetLastError();
}

hipError_t launch_quantize_cent_fp8(const adanns_index *ix, const int64_t *poff2, QuantStore &qs,
                                    hipStream_t st) {
  hipLaunchKernelGGL(k_quant_fp8_slab, dim3(blocks_for(ix->nl_pad, 4)), dim3(256), 0, st,
                     ix->cent_slab, poff2, 1, (int64_t)ix->nl_pad, ix->d_cb_pad, ix->d_cb,
                     (uint8_t *)qs.cent, qs.cent_scale);
  return hipGetLastError();
}

// Largest |x - dequantised x| over the rows of the quantised slab layout
// (as k_row_norm_max: block h covers list h, a half-wave per row). The
// dequantised value is the bf16 value, or scale x e4m3 value.
__global__ __launch_bounds__(256) void k_quant_err_max(const float *__restrict__ vec,
                                                       const void *__restrict__ qvec,
                                                       const float *__restrict__ qscale,
                                                       int32_t fmt, const int64_t *__restrict__ poff,
                                                       int32_t d_pad, uint32_t *__restrict__ out,
                                                       float *__restrict__ rerr) {
  __shared__ float sh[8];
  const int h = blockIdx.x, half = threadIdx.x >> 5, l = threadIdx.x & 31;
  const int64_t p0 = poff[h], np = poff[h + 1] - p0;
  const int nslab = d_pad / SLAB;
  float best = 0.f;
  for (int64_t r = half; r < np; r += 8) {
    const float xs = fmt == 2 ? qscale[p0 + r] : 1.f;
    float s = 0.f;
    for (int k = 0; k < nslab; ++k) {
      const int64_t i = p0 * d_pad + ((int64_t)k * np + r) * SLAB + l;
      const float xq = fmt == 1 ? bf16_to_float(((const uint16_t *)qvec)[i])
                                : xs * e4m3_to_float(((const uint8_t *)qvec)[i]);
      const float df = vec[i] - xq;
      s = fmaf(df, df, s);
    }
    for (int o = 16; o > 0; o >>= 1) s += __shfl_xor(s, o, 32);
    best = fmaxf(best, sqrtf(s));
    if (rerr != nullptr && l == 0) rerr[p0 + r] = sqrtf(s);
  }
  if (l == 0) sh[half] = best;
  __syncthreads();
  if (threadIdx.x == 0) {
    float m = sh[0];
    for (int i = 1; i < 8; ++i) m = fmaxf(m, sh[i]);
    atomicMax(out, __float_as_uint(m));
  }
}

hipError_t launch_quant_err_max(const adanns_index *ix, int32_t fmt, const QuantStore &qs,
                                hipStream_t st) {
  hipError_t e = hipMemsetAsync(qs.emax, 0, sizeof(float), st);
  if (e != hipSuccess || ix->nlist == 0) return e;
  hipLaunchKernelGGL(k_quant_err_max, dim3((unsigned)ix->nlist), dim3(256), 0, st, ix->vec,
                     qs.vec, qs.scale, fmt, ix->poff, ix->d_pad, (uint32_t *)qs.emax, qs.rerr);
  return hipGetLastError();
}

hipError_t launch_quant_err_max_cent(const adanns_index *ix, int32_t fmt, const int64_t *poff2,
                                     const QuantStore &qs, hipStream_t st) {
  hipError_t e = hipMemsetAsync(qs.cent_emax, 0, sizeof(float), st);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_quant_err_max, dim3(1), dim3(256), 0, st, ix->cent_slab, qs.cent,
                     qs.cent_scale, fmt, poff2, ix->d_cb_pad, (uint32_t *)qs.cent_emax,
                     (float *)nullptr);
  return hipGetLastError();
}

hipError_t launch_quantize_queries(const float *Q, int64_t nq, int64_t ldq, int32_t d,
                                   int32_t fmt, void *Qq, int64_t ldqq, float *qscale,
                                   hipStream_t st) {
  if (nq == 0) return hipSuccess;
  KernelTimer tm("quantize_queries", st);
  hipLaunchKernelGGL(k_quant_rows, dim3(blocks_for(nq, 4)), dim3(256), 0, st, Q, nq, ldq, d, fmt,
                     Qq, ldqq, qscale);
  return hipGetLastError();
}

// The quantised list scan's first pass (precision and filtered searches):
// each probed list's quantised vectors against the quantised queries probing
// it, into b.D (tiles and buckets from launch_bucketing with QTILE shapes).
static hipError_t launch_q_scan(const adanns_index *ix, int32_t fmt, const SearchBufs &b,
                                const void *Qq, int64_t ldqq, const float *qscale,
                                int32_t nprobe, int32_t d_s, hipStream_t st) {
  const QuantStore &qs = ix->quant[fmt];
  hipError_t e;
  TileQArgs u{};
  u.Qq = (const uint8_t *)Qq;
  u.ldqq = ldqq;
  u.qscale = qscale;
  u.d_dot = d_s;
  u.vec = (const uint8_t *)qs.vec;
  u.vscale = qs.scale;
  u.d_pad = ix->d_pad;
  u.poff = ix->poff;
  u.len = ix->len;
  u.nlist = ix->nlist;
  u.tile_off = b.tile_off;
  u.bkt_off = b.bkt_off;
  u.cnt = b.cnt;
  u.work = b.work;
  u.bucket = b.bucket;
  u.pair_div = nprobe;
  u.pair_base = b.pair_base;
  u.out = b.D;
  {
    KernelTimer tm("tile_q_scan", st);
    const int qgrid = (int)(b.max_items > 0 ? std::min<int64_t>(PERSIST_WG, round_up(std::max<int64_t>(8, b.max_items), 8))
                                            : PERSIST_WG);
    if (fmt == 1)
      hipLaunchKernelGGL((k_tile_q_scan<1, QTILE_Q, QTILE_V>), dim3(qgrid), dim3(256), 0, st, u);
    else
      hipLaunchKernelGGL((k_tile_q_scan<2, QTILE_Q, QTILE_V>), dim3(qgrid), dim3(256), 0, st, u);
  }
  e = hipGetLastError();
  return e;
}

hipError_t launch_precision_search(const adanns_index *ix, int32_t fmt, const SearchBufs &b,
                                   const void *Qq, int64_t ldqq, const float *qscale, int64_t nq,
                                   int32_t d_c, int32_t d_s, int32_t nprobe, int32_t k,
                                   int32_t rerank_k, int32_t coarse_margin, float *dist,
                                   int64_t *ids, int32_t *user_probes, hipStream_t st) {
  const QuantStore &qs = ix->quant[fmt];
  hipError_t e0 = launch_store_cfg(make_cfg(ix, d_c, d_s, nprobe, k, nq), b.cfg, st);
  if (e0 != hipSuccess) return e0;
  reset_redo(b.redo, st);
  // coarse first pass on the quantised centroids
  TileQArgs t{};
  t.Qq = (const uint8_t *)Qq;
  t.ldqq = ldqq;
  t.qscale = qscale;
  t.d_dot = d_c;
  t.vec = (const uint8_t *)qs.cent;
  t.vscale = qs.cent_scale;
  t.d_pad = ix->d_cb_pad;
  t.pair_div = 1;
  t.out = b.S;
  t.nq = nq;
  t.nl = ix->nlist;
  t.nl_pad = ix->nl_pad;
  t.qtiles = (int32_t)cdiv(nq, TILE_Q);
  t.total_host = t.qtiles * (int32_t)cdiv(ix->nlist, TILE_V);
  int grid = (int)std::min<int64_t>(PERSIST_WG, round_up(t.total_host, 8));
  {
    KernelTimer tm("tile_q_coarse", st);
    if (fmt == 1)
      hipLaunchKernelGGL(k_tile_dist_q<1>, dim3(grid), dim3(256), 0, st, t);
    else
      hipLaunchKernelGGL(k_tile_dist_q<2>, dim3(grid), dim3(256), 0, st, t);
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  SelArgs s{};
  s.mode = SEL_COARSE_QUANT;
  s.D = b.S;
  s.nl = ix->nlist;
  s.K2 = std::min<int32_t>(ix->nlist, nprobe + coarse_margin);
  s.K1 = std::min<int32_t>(ix->nlist, s.K2 + REFINE_MARGIN);
  s.kout = nprobe;
  s.stageB = 1;
  s.Qs = b.Qs;
  s.ldqs = b.ldqs;
  s.d_dot = d_c;
  s.d_B = d_c;
  s.cent = ix->cent;
  s.ld_cent = ix->d_cb_pad;
  s.qfmt = fmt;
  s.qvec = qs.cent;
  s.qscale = qs.cent_scale;
  s.qQ = Qq;
  s.qQscale = qscale;
  s.ldqq = ldqq;
  s.qnpad = ix->nl_pad;
  s.qemax = fmt == 1 ? qs.cent_emax : nullptr;
  s.qerr = qs.cent_emax;
  s.xmax2 = ix->cmax2;
  s.out_probes = b.probes;
  s.out_probes2 = user_probes;
  {
    const size_t smem = sel_caps(s, ix->nlist);
    KernelTimer tm("select_q_coarse", st);
    launch_select(s, nq, smem, b.redo, b.redo ? b.redo + 2 : nullptr, st);
  }
  e = launch_bucketing(ix, b, nq, nprobe, st, QTILE_Q, QTILE_V);
  if (e != hipSuccess) return e;
  if ((e = launch_q_scan(ix, fmt, b, Qq, ldqq, qscale, nprobe, d_s, st)) != hipSuccess) return e;
  SelArgs r{};  r.mode = SEL_QUANT;
  r.D = b.D;
  r.seg_off = b.seg_off;
  r.K2 = rerank_k;
  r.K1 = std::min<int32_t>(rerank_k + REFINE_MARGIN, MAX_SHORTLIST);
  r.kout = k;
  r.stageB = 1;
  r.Qs = b.Qs;
  r.ldqs = b.ldqs;
  r.d_dot = d_s;
  r.d_B = d_s;
  r.vec = ix->vec;
  r.rows = ix->rows;
  r.d_pad = ix->d_pad;
  r.poff = ix->poff;
  r.rowid = ix->rowid;
  r.probes = b.probes;
  r.nprobe = nprobe;
  r.pair_base = b.pair_base;
  r.qfmt = fmt;
  r.qvec = qs.vec;
  r.qscale = qs.scale;
  r.qd_pad = ix->d_pad;
  r.qQ = Qq;
  r.qQscale = qscale;
  r.ldqq = ldqq;
  // (e4m3's quantisation error spans the whole shortlist: no bound)
  r.qemax = fmt == 1 ? qs.emax : nullptr;
  r.qerr = qs.emax;
  r.qrerr = qs.rerr;
  r.xmax2 = ix->xmax2;
  r.out_dist = dist;
  r.out_ids = ids;
  {
    const size_t smem = sel_caps(r, SEG_LDS_CAP);
    KernelTimer tm("select_q_scan", st);
    if (nq > 0 && fmt == 1 && k + WAVE_MARGIN <= WSEL_K && b.redo != nullptr) {
      // BF16: the exact search's one-wave selection (FP32 k nearest of all
      // candidates, per-row quantisation bound), certified to return only
      // shortlist members, which makes it the shortlist's k nearest; the
      // queries it cannot certify go to the general re-selection launch
      SelArgs w = r;
      w.shortlist = rerank_k;
      w.redo_cnt = b.redo + 1;
      w.redo_list = b.redo + 2;
      w.redo_q0 = 0;
      hipLaunchKernelGGL(k_select_filtered_wave, dim3((unsigned)cdiv(nq, 4)), dim3(256), 0, st, w,
                         nq);
      w.shortlist = 0;
      w.kcap = redo_kcap();
      w.lcap = seg_cap(w.kcap, SEG_LDS_CAP);
      hipLaunchKernelGGL(k_select_refine_redo, dim3(redo_grid(nq)), dim3(512),
                         sel_smem_bytes(w.lcap, w.kcap), st, w);
    } else if (nq > 0 && fmt == 2 && r.K1 > WSEL_K && k <= 128 && b.redo != nullptr) {
      // e4m3, deep shortlist: the exact search's workgroup selection, with the
      // same shortlist certificate; the rest to the general re-selection
      SelArgs w = r;
      w.shortlist = rerank_k;
      w.redo_cnt = b.redo + 1;
      w.redo_list = b.redo + 2;
      w.redo_q0 = 0;
      hipLaunchKernelGGL(k_select_exact_filtered, dim3((unsigned)nq), dim3(256), 0, st, w);
      w.shortlist = 0;
      w.kcap = redo_kcap();
      w.lcap = seg_cap(w.kcap, SEG_LDS_CAP);
      hipLaunchKernelGGL(k_select_refine_redo, dim3(redo_grid(nq)), dim3(512),
                         sel_smem_bytes(w.lcap, w.kcap), st, w);
    } else {
      launch_select(r, nq, smem, b.redo ? b.redo + 1 : nullptr, b.redo ? b.redo + 2 : nullptr, st);
    }
  }
  return hipGetLastError();
}

hipError_t launch_filtered_search(const adanns_index *ix, int32_t fmt, const SearchBufs &b,
                                  const void *Qq, int64_t ldqq, const float *qscale, int64_t nq,
                                  int32_t d_c, int32_t d_s, int32_t nprobe, int32_t k,
                                  float *dist, int64_t *ids, int32_t *user_probes,
                                  hipStream_t st) {
  const QuantStore &qs = ix->quant[fmt];
  // the FP32 coarse step, exactly as adanns_search runs it
  hipError_t e = launch_coarse(ix, b, nq, d_c, nprobe, user_probes, st);
  if (e != hipSuccess) return e;
  if ((e = launch_bucketing(ix, b, nq, nprobe, st, QTILE_Q, QTILE_V)) != hipSuccess) return e;
  if ((e = launch_q_scan(ix, fmt, b, Qq, ldqq, qscale, nprobe, d_s, st)) != hipSuccess) return e;
  SelArgs r{};
  r.mode = SEL_QUANT;
  r.D = b.D;
  r.seg_off = b.seg_off;
  r.K2 = k;
  r.K1 = k;
  r.kout = k;
  r.stageB = 1;
  r.Qs = b.Qs;
  r.ldqs = b.ldqs;
  r.d_dot = d_s;
  r.d_B = d_s;
  r.vec = ix->vec;
  r.rows = ix->rows;
  r.d_pad = ix->d_pad;
  r.poff = ix->poff;
  r.rowid = ix->rowid;
  r.probes = b.probes;
  r.nprobe = nprobe;
  r.pair_base = b.pair_base;
  r.qfmt = fmt;
  r.qvec = qs.vec;
  r.qscale = qs.scale;
  r.qd_pad = ix->d_pad;
  r.qQ = Qq;
  r.qQscale = qscale;
  r.ldqq = ldqq;
  r.qerr = qs.emax;
  r.qrerr = qs.rerr;
  r.xmax2 = ix->xmax2;
  r.out_dist = dist;
  r.out_ids = ids;
  {
    KernelTimer tm("select_filtered", st);
    if (nq > 0 && fmt == 1 && k + WAVE_MARGIN <= WSEL_K && b.redo != nullptr) {
      // BF16: one wave per query; the queries it cannot certify within its
      // list go to the workgroup kernel. (e4m3's bound band outgrows the
      // list for most queries at d_s 2048: the workgroup kernel directly.)
      r.redo_cnt = b.redo + 1;
      r.redo_list = b.redo + 2;
      r.redo_q0 = 0;
      hipLaunchKernelGGL(k_select_filtered_wave, dim3((unsigned)cdiv(nq, 4)), dim3(256), 0, st, r,
                         nq);
      hipLaunchKernelGGL(k_select_exact_filtered_redo, dim3(redo_grid(nq)), dim3(256), 0, st, r);
    } else if (nq > 0) {
      hipLaunchKernelGGL(k_select_exact_filtered, dim3((unsigned)nq), dim3(256), 0, st, r);
    }
  }
  return hipGetLastError();
}

hipError_t launch_rotate(const float *Qs, int64_t ldqs, int64_t nq, const float *R, int32_t d_s,
                         float *qh, float *ql, int64_t ldqr, hipStream_t st) {
  if (nq == 0) return hipSuccess;
  KernelTimer tm("pq_rotate", st);
  hipLaunchKernelGGL(k_rotate, dim3((unsigned)cdiv(nq, ROT_Q), (unsigned)cdiv(d_s, ROT_C)),
                     dim3(256), 0, st, Qs, ldqs, nq, R, d_s, qh, ql, ldqr);
  return hipGetLastError();
}

hipError_t launch_pq_encode(const Mat &X, int64_t n, int32_t M, int32_t dsub, const float *cb,
                            uint8_t *codes, hipStream_t st) {
  if (n == 0) return hipSuccess;
  if (X.type == 1)
    hipLaunchKernelGGL(k_pq_encode<_Float16>, dim3(blocks_for(n, 256), M), dim3(256),
                       256 * dsub * sizeof(float), st, (const _Float16 *)X.p, X.ld, n, M, dsub, cb,
                       codes);
  else
    hipLaunchKernelGGL(k_pq_encode<float>, dim3(blocks_for(n, 256), M), dim3(256),
                       256 * dsub * sizeof(float), st, (const float *)X.p, X.ld, n, M, dsub, cb,
                       codes);
  return hipGetLastError();
}

hipError_t launch_gather_codes(const uint8_t *codes, int32_t M, const int64_t *rowid,
                               int64_t rows_pad, uint8_t *out, hipStream_t st) {
  int64_t n = rows_pad * M;
  hipLaunchKernelGGL(k_gather_codes, dim3(blocks_for(n, 256)), dim3(256), 0, st, codes, M, rowid,
                     rows_pad, out);
  return hipGetLastError();
}

hipError_t launch_pq_search(const adanns_index *ix, const PqCodec &pq, const SearchBufs &b,
                            int64_t nq, int32_t nprobe, int32_t k, int32_t rerank_k,
                            int32_t d_rerank, float *qr_hi, float *qr_lo, float *lut, float *dist,
                            int64_t *ids, hipStream_t st) {
  reset_redo(b.redo, st);
  hipError_t e = launch_bucketing(ix, b, nq, nprobe, st);
  if (e != hipSuccess) return e;
  const int64_t ldqr = pq.d_s;
  e = launch_rotate(b.Qs, b.ldqs, nq, pq.R, pq.d_s, qr_hi, qr_lo, ldqr, st);
  if (e != hipSuccess) return e;
  {
    KernelTimer tm("pq_lut", st);
    if (nq > 0)
      hipLaunchKernelGGL(k_pq_lut, dim3((unsigned)cdiv(nq, LUT_Q), (unsigned)pq.M), dim3(256), 0,
                         st, qr_hi, ldqr, nq, pq.cb, pq.M, pq.dsub, lut);
  }
  {
    KernelTimer tm("adc_scan", st);
    // lists per workgroup: as many as keep about 512 workgroups in flight
    const int32_t G = (int32_t)std::max<int64_t>(1, std::min<int64_t>(nprobe, nq * nprobe / 512));
    if (nq > 0)
    {
      const dim3 grid((unsigned)(nq * cdiv(nprobe, G)));
      const size_t tb = pq.M * 256 * sizeof(float);
      auto go = [&](auto kern) {
        hipLaunchKernelGGL(kern, grid, dim3(ADC_THREADS), tb, st, lut, pq.M, pq.codes, b.probes,
                           nprobe, G, ix->poff, ix->len, b.pair_base, b.D);
      };
      switch (pq.M) {
        case 16: go(k_adc_scan<16>); break;
        case 32: go(k_adc_scan<32>); break;
        case 64: go(k_adc_scan<64>); break;
        default: go(k_adc_scan<0>);
      }
    }
  }
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  SelArgs s{};
  s.mode = SEL_ADC;
  s.D = b.D;
  s.seg_off = b.seg_off;
  const int32_t keep = rerank_k > 0 ? rerank_k : k;
  s.K1 = std::min<int32_t>(keep + REFINE_MARGIN, MAX_SHORTLIST);
  s.K2 = keep;
  s.kout = k;
  s.stageB = rerank_k > 0;
  s.Qs = b.Qs;
  s.ldqs = b.ldqs;
  s.d_dot = pq.d_s;
  s.d_B = d_rerank;
  s.vec = ix->vec;
  s.rows = ix->rows;
  s.d_pad = ix->d_pad;
  s.poff = ix->poff;
  s.rowid = ix->rowid;
  s.probes = b.probes;
  s.nprobe = nprobe;
  s.pair_base = b.pair_base;
  s.codes = pq.codes;
  s.M = pq.M;
  s.dsub = pq.dsub;
  s.cb = pq.cb;
  s.qr_hi = qr_hi;
  s.qr_lo = qr_lo;
  s.ldqr = ldqr;
  s.out_dist = dist;
  s.out_ids = ids;
  {
    const size_t smem = sel_caps(s, SEG_LDS_CAP);
    KernelTimer tm("select_adc", st);
    launch_select(s, nq, smem, b.redo ? b.redo + 1 : nullptr, b.redo ? b.redo + 2 : nullptr, st);
  }
  return hipGetLastError();
}

}  // namespace adanns
