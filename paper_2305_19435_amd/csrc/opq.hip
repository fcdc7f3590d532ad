// Optimized product quantisation on the GPU: the orthonormal rotation R
// learned together with the PQ codebooks (Section 3, "Optimized Product
// Quantization", the non-parametric method of Ge et al. that the paper
// names; Section 4.3 AdANNS-IVFOPQ). Alternation on the training rows X:
//   R = R_init (or I); repeat { Y = X R; PQ k-means on Y (warm-started from the previous
//   codebooks); Yhat = decode(encode(Y)); R = argmin over orthonormal R of
//   |X R - Yhat|_F = the orthogonal polar factor of X^T Yhat }
// then a last PQ training on X R, and every row is encoded.
//
//   k_gemm64         C = alpha op(A) B + beta C with FP64 accumulation (64x64
//                    tiles staged in LDS, k split over workgroups)
//   k_polar_*        the orthogonal polar factor by the Newton-Schulz
//                    iteration Z <- 1.5 Z - 0.5 Z (Z^T Z), FP64
//   k_pq_decode      codes -> reconstructed rows
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "internal.h"

namespace adanns {
namespace {

constexpr int GT = 64;   // output tile edge
constexpr int GK = 16;   // k-chunk staged per step

// Partial products of C = op(A) B over the k-range of blockIdx.z:
// op(A) is m x k (A row-major m x k, or A^T with A row-major k x m), B is
// k x n row-major; FP64 accumulation; partial [z][m][n].
template <class TA, class TB, bool TRANS_A>
__global__ __launch_bounds__(256) void k_gemm64(int m, int n, int64_t k, int64_t kchunk,
                                                 const TA *__restrict__ A, int64_t lda,
                                                 const TB *__restrict__ B, int64_t ldb,
                                                 double *__restrict__ part) {
  __shared__ double As[GK][GT + 1];
  __shared__ double Bs[GK][GT + 1];
  const int i0 = blockIdx.y * GT, j0 = blockIdx.x * GT;
  const int tx = threadIdx.x % 16, ty = threadIdx.x / 16;
  const int64_t k0 = (int64_t)blockIdx.z * kchunk, k1 = std::min<int64_t>(k, k0 + kchunk);
  double acc[4][4];
#pragma unroll
  for (int r = 0; r < 4; ++r)
#pragma unroll
    for (int c = 0; c < 4; ++c) acc[r][c] = 0.0;
  for (int64_t kk0 = k0; kk0 < k1; kk0 += GK) {
    for (int e = threadIdx.x; e < GK * GT; e += blockDim.x) {
      int kk, ii;
      if (TRANS_A) {  // A[(kk0 + kk) * lda + i0 + ii]: consecutive threads, consecutive ii
        kk = e / GT;
        ii = e % GT;
      } else {        // A[(i0 + ii) * lda + kk0 + kk]: consecutive threads, consecutive kk
        ii = e / GK;
        kk = e % GK;
      }
      const int64_t kg = kk0 + kk;
      const int ig = i0 + ii;
      double v = 0.0;
      if (kg < k1 && ig < m) v = TRANS_A ? (double)A[kg * lda + ig] : (double)A[(int64_t)ig * lda + kg];
      As[kk][ii] = v;
      const int kb = e / GT, jj = e % GT;
      const int64_t kbg = kk0 + kb;
      const int jg = j0 + jj;
      Bs[kb][jj] = (kbg < k1 && jg < n) ? (double)B[kbg * ldb + jg] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < GK; ++kk) {
      double a[4], b[4];
#pragma unroll
      for (int r = 0; r < 4; ++r) a[r] = As[kk][ty * 4 + r];
#pragma unroll
      for (int c = 0; c < 4; ++c) b[c] = Bs[kk][tx * 4 + c];
#pragma unroll
      for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int c = 0; c < 4; ++c) acc[r][c] = fma(a[r], b[c], acc[r][c]);
    }
    __syncthreads();
  }
  double *P = part + (int64_t)blockIdx.z * m * n;
#pragma unroll
  for (int r = 0; r < 4; ++r)
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const int i = i0 + ty * 4 + r, j = j0 + tx * 4 + c;
      if (i < m && j < n) P[(int64_t)i * n + j] = acc[r][c];
    }
}

// C = alpha * (sum of the nz partials, in order) + beta * C.
__global__ void k_gemm_reduce(int64_t mn, int nz, const double *__restrict__ part, double alpha,
                              double beta, double *__restrict__ C) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= mn) return;
  double s = 0.0;
  for (int z = 0; z < nz; ++z) s += part[(int64_t)z * mn + i];
  C[i] = alpha * s + (beta != 0.0 ? beta * C[i] : 0.0);
}

// Sum of squares of v[0..n) (or of v - w when w is given) into *out
// (atomic FP64 add; *out zeroed by the caller).
__global__ void k_sumsq64(const double *__restrict__ v, const double *__restrict__ w, int64_t n,
                          double *__restrict__ out) {
  __shared__ double sh[4];
  double s = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const double x = w ? v[i] - w[i] : v[i];
    s = fma(x, x, s);
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) atomicAdd(out, (sh[0] + sh[1]) + (sh[2] + sh[3]));
}

// Largest |P - I| over a d x d matrix (as an order-preserving bit pattern of
// a non-negative double) into *out (zeroed by the caller).
__global__ void k_max_off_identity(const double *__restrict__ P, int d,
                                   unsigned long long *__restrict__ out) {
  const int64_t n = (int64_t)d * d;
  double m = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const double x = P[i] - ((i / d == i % d) ? 1.0 : 0.0);
    m = x == x ? fmax(m, fabs(x)) : __builtin_inf();  // NaN counts as infinitely far
  }
  atomicMax(out, (unsigned long long)__double_as_longlong(m));
}

__global__ void k_scale64(const double *__restrict__ src, int64_t n, const double *__restrict__ s2,
                          double *__restrict__ dst) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = src[i] / sqrt(*s2);
}

__global__ void k_to_f32(const double *__restrict__ src, int64_t n, float *__restrict__ dst) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = (float)src[i];
}

// out[j][m * dsub + t] = cb[m][codes[j][m]][t]
__global__ void k_pq_decode(const uint8_t *__restrict__ codes, int64_t n, int32_t M, int32_t dsub,
                            const float *__restrict__ cb, float *__restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t d = (int64_t)M * dsub;
  if (i >= n * d) return;
  const int64_t j = i / d;
  const int32_t c = (int32_t)(i % d), m = c / dsub, t = c % dsub;
  out[i] = cb[((int64_t)m * 256 + codes[j * M + m]) * dsub + t];
}

// Sum of squared differences of two FP32 arrays of n elements into *out
// (FP64; *out zeroed by the caller).
__global__ void k_sqdiff_sum(const float *__restrict__ a, const float *__restrict__ b, int64_t n,
                             double *__restrict__ out) {
  __shared__ double sh[4];
  double s = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const double x = (double)a[i] - (double)b[i];
    s = fma(x, x, s);
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) atomicAdd(out, (sh[0] + sh[1]) + (sh[2] + sh[3]));
}

unsigned blocks(int64_t n, int b) { return (unsigned)std::max<int64_t>(1, (n + b - 1) / b); }

// C[m x n] = alpha op(A) B + beta C (FP64), k split over workgroups.
template <class TA, class TB, bool TRANS_A>
hipError_t gemm64(int m, int n, int64_t k, const TA *A, int64_t lda, const TB *B, int64_t ldb,
                  double alpha, double beta, double *C, double *part, int64_t part_cap,
                  hipStream_t st) {
  const int gx = (n + GT - 1) / GT, gy = (m + GT - 1) / GT;
  // enough workgroups for the chip, each with a k-range of whole chunks
  int nz = (int)std::max<int64_t>(1, std::min<int64_t>((k + 255) / 256, 2048 / (gx * gy) + 1));
  nz = (int)std::min<int64_t>(nz, part_cap / ((int64_t)m * n));
  nz = std::max(nz, 1);
  int64_t kchunk = (k + nz - 1) / nz;
  kchunk = (kchunk + GK - 1) / GK * GK;
  nz = (int)((k + kchunk - 1) / kchunk);
  hipLaunchKernelGGL((k_gemm64<TA, TB, TRANS_A>), dim3(gx, gy, nz), dim3(256), 0, st, m, n, k,
                     kchunk, A, lda, B, ldb, part);
  hipLaunchKernelGGL(k_gemm_reduce, dim3(blocks((int64_t)m * n, 256)), dim3(256), 0, st,
                     (int64_t)m * n, nz, part, alpha, beta, C);
  return hipGetLastError();
}

// Scratch (doubles) of polar(): Z, Zn, P, the norm, and the k-split partials.
int64_t polar_scratch(int32_t d) { return (int64_t)d * d * (3 + 16) + 8; }

// The orthogonal polar factor of the d x d matrix A (FP64, device): for
// A = U S V^T with S > 0, U V^T, the orthonormal matrix nearest to A, which
// also maximises tr(R^T A) (orthogonal Procrustes). Newton-Schulz from
// Z = A / |A|_F (singular values in (0, 1]): every singular value follows
// s <- 1.5 s - 0.5 s^3, which rises to 1 (by about 1.5x while small, then
// quadratically) while the singular vectors stay fixed. Stops when a step
// changes Z by less than 1e-13 |Z|_F; fails (returns false) if Z^T Z is then
// not the identity to 1e-9 (A singular or too ill-conditioned for the
// iteration limit).
bool polar(const double *A, int32_t d, double *R, double *scr, int32_t max_iter, int32_t *iters,
           hipStream_t st) {
  const int64_t dd = (int64_t)d * d;
  double *Z = scr, *Zn = scr + dd, *P = scr + 2 * dd, *nrm = scr + 3 * dd,
         *part = scr + 3 * dd + 8;
  const int64_t part_cap = 16 * dd;
  if (hipMemsetAsync(nrm, 0, sizeof(double), st) != hipSuccess) return false;
  hipLaunchKernelGGL(k_sumsq64, dim3(blocks(dd, 256 * 8)), dim3(256), 0, st, A,
                     (const double *)nullptr, dd, nrm);
  hipLaunchKernelGGL(k_scale64, dim3(blocks(dd, 256)), dim3(256), 0, st, A, dd, nrm, Z);
  int32_t it = 0;
  for (; it < max_iter; ++it) {
    // P = Z^T Z; Zn = 1.5 Z - 0.5 Z P
    if (gemm64<double, double, true>(d, d, d, Z, d, Z, d, 1.0, 0.0, P, part, part_cap, st) ||
        hipMemcpyAsync(Zn, Z, dd * sizeof(double), hipMemcpyDeviceToDevice, st) ||
        gemm64<double, double, false>(d, d, d, Z, d, P, d, -0.5, 1.5, Zn, part, part_cap, st))
      return false;
    double h[2] = {0.0, 0.0};
    if (hipMemsetAsync(nrm, 0, 2 * sizeof(double), st) != hipSuccess) return false;
    hipLaunchKernelGGL(k_sumsq64, dim3(blocks(dd, 256 * 8)), dim3(256), 0, st, Zn, Z, dd, nrm);
    hipLaunchKernelGGL(k_sumsq64, dim3(blocks(dd, 256 * 8)), dim3(256), 0, st, Zn,
                       (const double *)nullptr, dd, nrm + 1);
    if (hipMemcpyAsync(h, nrm, 2 * sizeof(double), hipMemcpyDeviceToHost, st) ||
        hipStreamSynchronize(st))
      return false;
    std::swap(Z, Zn);
    if (!std::isfinite(h[0]) || !std::isfinite(h[1]) || h[1] == 0.0) return false;
    if (std::sqrt(h[0]) <= 1e-13 * std::sqrt(h[1])) {
      ++it;
      break;
    }
  }
  if (iters) *iters = it;
  if (it >= max_iter) return false;  // did not settle
  // orthogonality check: max |Z^T Z - I|
  unsigned long long bits = 0;
  if (gemm64<double, double, true>(d, d, d, Z, d, Z, d, 1.0, 0.0, P, part, part_cap, st) ||
      hipMemsetAsync(nrm, 0, sizeof(double), st))
    return false;
  hipLaunchKernelGGL(k_max_off_identity, dim3(blocks(dd, 256 * 8)), dim3(256), 0, st, P, d,
                     (unsigned long long *)nrm);
  if (hipMemcpyAsync(&bits, nrm, sizeof(bits), hipMemcpyDeviceToHost, st) ||
      hipMemcpyAsync(R, Z, dd * sizeof(double), hipMemcpyDeviceToDevice, st) ||
      hipStreamSynchronize(st))
    return false;
  double off;
  std::memcpy(&off, &bits, sizeof(off));
  return off <= 1e-9;
}

}  // namespace
}  // namespace adanns

using namespace adanns;

extern "C" {

adanns_status adanns_polar_factor(const double *A, int32_t d, double *R, int32_t *iterations,
                                  void *stream) {
  clear_error();
  ADANNS_REQUIRE(A != nullptr && R != nullptr, "A and R must be non-NULL");
  ADANNS_REQUIRE(d >= 1 && d <= 4096, "d must be in [1, 4096], got %d", d);
  hipStream_t st = (hipStream_t)stream;
  double *scr = nullptr;
  if (hipMalloc(&scr, (size_t)polar_scratch(d) * sizeof(double)) != hipSuccess) {
    (void)hipGetLastError();
    set_error("out of device memory for the polar factor's scratch");
    return ADANNS_ENOMEM;
  }
  const bool ok = polar(A, d, R, scr, 200, iterations, st);
  (void)hipStreamSynchronize(st);
  (void)hipFree(scr);
  if (!ok) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
      set_error("HIP error in the polar factor: %s", hipGetErrorString(e));
      return ADANNS_EHIP;
    }
    set_error("the Newton-Schulz iteration did not reach an orthonormal matrix (the matrix is "
              "singular or too ill-conditioned)");
    return ADANNS_EUNSUPPORTED;
  }
  return ADANNS_OK;
}

adanns_status adanns_opq_train(adanns_index *ix, const void *X, int64_t ldx, int32_t dtype,
                               int32_t M, int32_t d_s, const float *R_init, int32_t outer,
                               int32_t pq_iters, const int32_t *init_rows,
                               const int64_t *train_rows, int64_t n_train, double *distortion,
                               void *stream) {
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
  ADANNS_REQUIRE(outer >= 0 && outer <= 100, "outer must be in [0, 100]");
  ADANNS_REQUIRE(pq_iters >= 0 && pq_iters <= 1000, "pq_iters must be in [0, 1000]");
  ADANNS_REQUIRE(ix->pq.find(M) == ix->pq.end(), "the index already holds a codec with M = %d", M);
  const int64_t nt = train_rows ? n_train : ix->n;
  ADANNS_REQUIRE(nt >= 256, "the training set must hold at least 256 rows");
  for (int32_t c = 0; c < 256; ++c)
    ADANNS_REQUIRE(init_rows[c] >= 0 && init_rows[c] < nt, "init_rows[%d] out of range", c);
  if (train_rows)
    for (int64_t j = 0; j < nt; ++j)
      ADANNS_REQUIRE(train_rows[j] >= 0 && train_rows[j] < ix->n, "train_rows[%lld] out of range",
                     (long long)j);
  {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
      set_error("HIP error from an earlier launch: %s", hipGetErrorString(e));
      return ADANNS_EHIP;
    }
  }
  hipStream_t st = (hipStream_t)stream;
  const int32_t dsub = d_s / M, dcp = (int32_t)round_up(dsub, SLAB);
  const int64_t dd = (int64_t)d_s * d_s;
  std::vector<void *> owned;
  auto cleanup = [&]() {
    (void)hipStreamSynchronize(st);
    for (void *p : owned)
      if (p) (void)hipFree(p);
  };
  auto alloc = [&](void **p, size_t bytes) {
    if (hipMalloc(p, bytes) != hipSuccess) {
      (void)hipGetLastError();
      *p = nullptr;
      return false;
    }
    owned.push_back(*p);
    return true;
  };
  float *raw = nullptr, *T = nullptr, *Tlo = nullptr, *Yh = nullptr, *cb = nullptr, *R32 = nullptr;
  double *Mt = nullptr, *R64 = nullptr, *scr = nullptr, *dist_d = nullptr;
  uint8_t *codes_t = nullptr, *codes_id = nullptr;
  int64_t *d_tr = nullptr;
  if (!alloc((void **)&raw, (size_t)nt * d_s * 4) || !alloc((void **)&T, (size_t)nt * d_s * 4) ||
      !alloc((void **)&Tlo, (size_t)nt * d_s * 4) || !alloc((void **)&Yh, (size_t)nt * d_s * 4) ||
      !alloc((void **)&cb, (size_t)M * 256 * dsub * 4) || !alloc((void **)&R32, (size_t)dd * 4) ||
      !alloc((void **)&Mt, (size_t)dd * 8) || !alloc((void **)&R64, (size_t)dd * 8) ||
      !alloc((void **)&scr, (size_t)polar_scratch(d_s) * 8) ||
      !alloc((void **)&dist_d, sizeof(double)) || !alloc((void **)&codes_t, (size_t)nt * M) ||
      !alloc((void **)&codes_id, (size_t)ix->n * M) ||
      (train_rows && !alloc((void **)&d_tr, (size_t)nt * 8))) {
    cleanup();
    set_error("out of device memory for OPQ training");
    return ADANNS_ENOMEM;
  }
  const Mat Xm{X, ldx, dtype};
  auto fail_hip = [&](const char *what) {
    hipError_t e = hipGetLastError();
    cleanup();
    set_error("%s failed: %s", what, hipGetErrorString(e));
    return ADANNS_EHIP;
  };
  if (train_rows &&
      hipMemcpyAsync(d_tr, train_rows, nt * sizeof(int64_t), hipMemcpyHostToDevice, st))
    return fail_hip("copying the training rows");
  if (launch_stage_rows(Xm, d_tr, nullptr, nt, d_s, raw, d_s, st))
    return fail_hip("staging the training rows");
  if (R_init) {  // the given starting rotation
    if (hipMemcpyAsync(R32, R_init, dd * 4, hipMemcpyDeviceToDevice, st) ||
        hipStreamSynchronize(st))
      return fail_hip("copying R_init");
  } else {  // R = I
    std::vector<float> eye((size_t)dd, 0.f);
    for (int32_t i = 0; i < d_s; ++i) eye[(size_t)i * d_s + i] = 1.f;
    if (hipMemcpyAsync(R32, eye.data(), dd * 4, hipMemcpyHostToDevice, st) ||
        hipStreamSynchronize(st))
      return fail_hip("setting R = I");
  }
  std::vector<int32_t> unused;
  for (int32_t t = 0; t <= outer; ++t) {
    // Y = X R on the training rows (FP64 accumulation, the high part kept)
    if (launch_rotate(raw, d_s, nt, R32, d_s, T, Tlo, d_s, st))
      return fail_hip("rotating the training rows");
    // PQ k-means per block: from init_rows the first time, then warm-started
    for (int32_t m = 0; m < M; ++m) {
      float *C = nullptr;
      adanns_status s = kmeans_gpu(f32mat(T, d_s).cols((int64_t)m * dsub), nt, 256, dsub, pq_iters,
                                   init_rows, nullptr, nt, nullptr, st, unused, &C, false,
                                   t == 0 ? nullptr : cb + (size_t)m * 256 * dsub);
      if (s) {
        if (C) (void)hipFree(C);
        cleanup();
        return s;
      }
      hipError_t e = hipMemcpy2DAsync(cb + (size_t)m * 256 * dsub, dsub * sizeof(float), C,
                                      dcp * sizeof(float), dsub * sizeof(float), 256,
                                      hipMemcpyDeviceToDevice, st);
      (void)hipStreamSynchronize(st);
      (void)hipFree(C);
      if (e != hipSuccess) return fail_hip("copying the codebooks");
    }
    // encode, decode, distortion sum |Y - Yhat|^2
    if (launch_pq_encode(f32mat(T, d_s), nt, M, dsub, cb, codes_t, st))
      return fail_hip("encoding the training rows");
    hipLaunchKernelGGL(k_pq_decode, dim3(blocks(nt * d_s, 256)), dim3(256), 0, st, codes_t, nt, M,
                       dsub, cb, Yh);
    double dist_h = 0.0;
    if (hipMemsetAsync(dist_d, 0, sizeof(double), st)) return fail_hip("clearing the distortion");
    hipLaunchKernelGGL(k_sqdiff_sum, dim3(std::min<unsigned>(2048, blocks(nt * d_s, 256))),
                       dim3(256), 0, st, T, Yh, nt * d_s, dist_d);
    if (hipMemcpyAsync(&dist_h, dist_d, sizeof(double), hipMemcpyDeviceToHost, st) ||
        hipStreamSynchronize(st))
      return fail_hip("the distortion");
    if (distortion) distortion[t] = dist_h;
    if (t == outer) break;
    // R = polar factor of X^T Yhat (orthogonal Procrustes)
    if (gemm64<float, float, true>(d_s, d_s, nt, raw, d_s, Yh, d_s, 1.0, 0.0, Mt, scr,
                                   16 * dd, st))
      return fail_hip("X^T Yhat");
    if (!polar(Mt, d_s, R64, scr, 200, nullptr, st)) {
      hipError_t e = hipGetLastError();
      cleanup();
      if (e != hipSuccess) {
        set_error("HIP error in the rotation step: %s", hipGetErrorString(e));
        return ADANNS_EHIP;
      }
      set_error("the rotation step did not converge to an orthonormal matrix");
      return ADANNS_EUNSUPPORTED;
    }
    hipLaunchKernelGGL(k_to_f32, dim3(blocks(dd, 256)), dim3(256), 0, st, R64, dd, R32);
  }
  // encode every row with the final rotation and codebooks, in chunks
  const int64_t chunk = 262144;
  const int64_t cm = std::min<int64_t>(chunk, ix->n);
  float *craw = nullptr, *crot = nullptr, *clo = nullptr;
  if (!alloc((void **)&craw, (size_t)cm * d_s * 4) || !alloc((void **)&crot, (size_t)cm * d_s * 4) ||
      !alloc((void **)&clo, (size_t)cm * d_s * 4)) {
    cleanup();
    set_error("out of device memory for OPQ encoding");
    return ADANNS_ENOMEM;
  }
  for (int64_t a0 = 0; a0 < ix->n; a0 += chunk) {
    const int64_t m = std::min(chunk, ix->n - a0);
    if (launch_stage_rows(Xm.rows(a0), nullptr, nullptr, m, d_s, craw, d_s, st) ||
        launch_rotate(craw, d_s, m, R32, d_s, crot, clo, d_s, st) ||
        launch_pq_encode(f32mat(crot, d_s), m, M, dsub, cb, codes_id + a0 * M, st))
      return fail_hip("encoding the rows");
  }
  if (hipStreamSynchronize(st)) return fail_hip("OPQ training");
  adanns_status s = adanns_pq_import(ix, M, d_s, R32, cb, codes_id, stream);
  cleanup();
  return s;
}

}  // extern "C"
