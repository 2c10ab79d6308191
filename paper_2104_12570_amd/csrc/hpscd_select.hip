// Column-wise inner products X^T v of a whole matrix, and the two users of
// them: the gradient stop rule of a single-system solve and feature
// selection with HPSCD (Section 8, Algorithm 3).
//
// X^T v is the "first step of the inner loop for every column at once" of
// Algorithm 3: one pass over X, HBM-bound (4 bytes of X per inner-product
// term), FP64 sums of the FP32 products.  The pass writes one FP64 partial
// sum per (row strip, column); a second kernel adds the strips in a fixed
// order, so every result is bitwise reproducible.
//
// Feature selection keeps its residual e in FP64 (m doubles; X stays FP32),
// so the choice of each column (an argmax) is taken on FP64 values.
#include "hpscd_device.hpp"
#include "hpscd_internal.hpp"

#include <float.h>

namespace hpscd {

namespace {

constexpr int TILE = 64;                               // columns per reduction workgroup
constexpr int XTV_CHUNKS = 4;                          // chunks of 4 rows per lane per sub-strip
constexpr int XTV_SUB = WAVE * XTV_CHUNKS * 4;         // 1024 rows per sub-strip
constexpr int XTV_CPW = 16;                            // columns per wave
constexpr int XTV_COLS = 4 * XTV_CPW;                  // columns per workgroup (four waves)
constexpr int XTV_U = 4;                               // columns whose loads are issued together

template <typename TV>
__device__ inline double as_f64(TV v) { return (double)v; }

// Workgroup (s, g): rows [s*rows_per, (s+1)*rows_per) in sub-strips of 1024,
// columns [g*64, g*64 + 64), sixteen per wave.  Lane L owns rows
// sub + k*256 + 4L .. +3 (k < 4) of every sub-strip: each load of a wave is
// 1 KB of one column, contiguous.  partial[s*n + j] = sum_rows X_ij v_i;
// workgroups with g == 0 also write vnorm[s] = sum_rows v_i^2.
template <typename TV>
__global__ void __launch_bounds__(256) k_xtv(const float* X, int64_t ldx, int64_t m, int64_t n, const TV* v,
                                             int64_t rows_per, double* partial, double* vnorm,
                                             const int32_t* done) {
  if (done && load_flag(done)) return;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t s = blockIdx.x;
  const int64_t r_begin = s * rows_per, r_end = min(m, r_begin + rows_per);
  const int64_t jw = (int64_t)blockIdx.y * XTV_COLS + (int64_t)wave * XTV_CPW;
  double acc[XTV_CPW];
#pragma unroll
  for (int c = 0; c < XTV_CPW; ++c) acc[c] = 0.0;
  double vsq = 0.0;
  for (int64_t sub = r_begin; sub < r_end; sub += XTV_SUB) {
    double vv[XTV_CHUNKS][4];
    int lim[XTV_CHUNKS];
#pragma unroll
    for (int k = 0; k < XTV_CHUNKS; ++k) {
      const int64_t r0 = sub + (int64_t)k * (WAVE * 4) + 4 * lane;
      const int64_t left = r_end - r0;
      lim[k] = left <= 0 ? 0 : (left >= 4 ? 4 : (int)left);
#pragma unroll
      for (int i = 0; i < 4; ++i) vv[k][i] = i < lim[k] ? as_f64(v[r0 + i]) : 0.0;
      if (blockIdx.y == 0 && wave == 0) {
#pragma unroll
        for (int i = 0; i < 4; ++i) vsq = fma(vv[k][i], vv[k][i], vsq);
      }
    }
#pragma unroll
    for (int c0 = 0; c0 < XTV_CPW; c0 += XTV_U) {
      float4 x[XTV_U][XTV_CHUNKS];
#pragma unroll
      for (int u = 0; u < XTV_U; ++u) {
        const int64_t j = jw + c0 + u;
#pragma unroll
        for (int k = 0; k < XTV_CHUNKS; ++k) {
          const int64_t r0 = sub + (int64_t)k * (WAVE * 4) + 4 * lane;
          x[u][k] = (j < n && lim[k] > 0) ? load_chunk<F32>(X, j * ldx + r0) : F32::zero();
          if (lim[k] < 4) x[u][k] = mask_chunk<F32>(x[u][k], lim[k]);
        }
      }
#pragma unroll
      for (int u = 0; u < XTV_U; ++u)
#pragma unroll
        for (int k = 0; k < XTV_CHUNKS; ++k) {
          acc[c0 + u] = fma((double)x[u][k].x, vv[k][0], acc[c0 + u]);
          acc[c0 + u] = fma((double)x[u][k].y, vv[k][1], acc[c0 + u]);
          acc[c0 + u] = fma((double)x[u][k].z, vv[k][2], acc[c0 + u]);
          acc[c0 + u] = fma((double)x[u][k].w, vv[k][3], acc[c0 + u]);
        }
    }
  }
#pragma unroll
  for (int c = 0; c < XTV_CPW; ++c) {
    const double t = wave_sum(acc[c]);
    const int64_t j = jw + c;
    if (lane == 0 && j < n) partial[s * n + j] = t;
  }
  if (blockIdx.y == 0 && wave == 0) {
    const double t = wave_sum(vsq);
    if (lane == 0) vnorm[s] = t;
  }
}

// Tile t = 64 columns, one workgroup: thread (q, c) (q = wave, c = lane)
// sums the strips s = q, q+4, ... of column j = 64t + c with eight loads in
// flight (eight running sums, added in a fixed order), then the four strip
// groups are added in order through LDS: g_j.  Tile t then writes
//   mode 0 (gradient): tsum[t] = sum_j g_j^2 (fixed order);
//   mode 1 (selection): the best candidate of the tile, score_j =
//     g_j^2 / <X_j,X_j> (as g_j^2 * rdn_j) over columns not selected with
//     rdn_j > 0, ties to the lower index: tscore[t], tidx[t] (-1: none).
__global__ void __launch_bounds__(256) k_xtv_tiles(const double* partial, int64_t S, int64_t n, int mode,
                                                   const double* rdn, const int32_t* selected, double* g,
                                                   double* tsum, double* tscore, int64_t* tidx,
                                                   const int32_t* done) {
  if (done && load_flag(done)) return;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t j = (int64_t)blockIdx.x * TILE + lane;
  __shared__ double part[4][TILE];
  {
    double acc[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    if (j < n) {
      int64_t s = wave;
      for (; s + 28 < S; s += 32) {
#pragma unroll
        for (int u = 0; u < 8; ++u) acc[u] += partial[(s + 4 * u) * n + j];
      }
      for (; s < S; s += 4) acc[0] += partial[s * n + j];
    }
    part[wave][lane] = ((acc[0] + acc[1]) + (acc[2] + acc[3])) + ((acc[4] + acc[5]) + (acc[6] + acc[7]));
  }
  __syncthreads();
  if (wave != 0) return;
  const double gj = (part[0][lane] + part[1][lane]) + (part[2][lane] + part[3][lane]);
  if (j < n && g) g[j] = gj;
  if (mode == 0) {
    const double t = wave_sum(j < n ? gj * gj : 0.0);
    if (lane == 0) tsum[blockIdx.x] = t;
    return;
  }
  double sc = -1.0;
  int64_t id = -1;
  if (j < n && !selected[j] && rdn[j] > 0.0) {
    sc = gj * gj * rdn[j];
    id = j;
  }
  // wave argmax, ties to the lower index
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    const double os = __shfl_xor(sc, off);
    const int64_t oi = __shfl_xor(id, off);
    const bool take = (oi >= 0) && (id < 0 || os > sc || (os == sc && oi < id));
    sc = take ? os : sc;
    id = take ? oi : id;
  }
  if (lane == 0) {
    tscore[blockIdx.x] = sc;
    tidx[blockIdx.x] = id;
  }
}

// Fixed-order sum of v[0..count) by one workgroup of 256 threads; every
// thread returns the total.
__device__ inline double block_sum_f64(const double* v, int64_t count, double* red) {
  double acc = 0.0;
  for (int64_t i = threadIdx.x; i < count; i += 256) acc += v[i];
  const double t = wave_sum(acc);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = t;
  __syncthreads();
  const double tot = (red[0] + red[1]) + (red[2] + red[3]);
  __syncthreads();
  return tot;
}

// Gradient stop rule (one workgroup).  init: ||X^T y||^2 into st->xty2.
// Otherwise, after sweep `sweep`: rel = ||X^T e|| / ||X^T y|| into
// fstat[2]; when ||e|| = 0, ||X^T e|| = 0 or rel < tol the solve ends here:
// the control words take the sweep count, the stop and the column count,
// and hist[sweep] = ||e|| (FP64 sum of the running residual).
__global__ void __launch_bounds__(256) k_grad_stop(const double* tsum, int64_t T, const double* vnorm, int64_t S,
                                                   int init, int32_t sweep, int64_t n, double tol, int32_t* ctl,
                                                   int64_t* ctl64, double* fstat, double* hist) {
  if (load_flag(&ctl[CTL_DONE])) return;
  __shared__ double red[4];
  const double g2 = block_sum_f64(tsum, T, red);
  if (init) {
    if (threadIdx.x == 0) fstat[3] = g2;
    return;
  }
  const double e2 = block_sum_f64(vnorm, S, red);
  if (threadIdx.x != 0) return;
  const double rel = fstat[3] > 0.0 ? sqrt(g2) / sqrt(fstat[3]) : sqrt(g2);
  fstat[2] = rel;
  if (e2 == 0.0 || g2 == 0.0 || rel < tol) {
    const double nrm = sqrt(e2);
    hist[sweep] = nrm;
    fstat[0] = e2;
    fstat[1] = nrm;
    ctl[CTL_SWEEPS] = sweep;
    ctl[CTL_CONVERGED] = 1;
    ctl64[C64_COLS] = (int64_t)sweep * n;
    store_flag(&ctl[CTL_DONE], 1);
  }
}

// Selection step f (one workgroup): the best of the tiles (ties to the lower
// index).  Records hist[f] = ||e|| (before the step); under tol > 0 stops
// when the best score < tol * ||e||^2; else J[f] = j^, da[f] = g_j^ rdn_j^,
// a64[j^] += da, selected[j^] = 1, count = f + 1, and the step (j^, da) for
// the residual update.
__global__ void __launch_bounds__(256) k_select_pick(const double* tscore, const int64_t* tidx, int64_t T,
                                                     const double* vnorm, int64_t S, const double* g,
                                                     const double* rdn, int32_t f, double tol, int32_t* selected,
                                                     double* a64, int32_t* Jd, double* dad, double* hist,
                                                     int32_t* ctl, int64_t* step_j, double* step_da) {
  if (load_flag(&ctl[CTL_DONE])) return;
  __shared__ double red[4];
  __shared__ double bs[256];
  __shared__ int64_t bi[256];
  const double e2 = block_sum_f64(vnorm, S, red);
  double b = -1.0;
  int64_t k = -1;
  for (int64_t t = threadIdx.x; t < T; t += 256) {
    const bool take = (tidx[t] >= 0) && (k < 0 || tscore[t] > b || (tscore[t] == b && tidx[t] < k));
    if (take) { b = tscore[t]; k = tidx[t]; }
  }
  bs[threadIdx.x] = b;
  bi[threadIdx.x] = k;
  __syncthreads();
  if (threadIdx.x != 0) return;
  for (int w = 1; w < 256; ++w) {
    const bool take = (bi[w] >= 0) && (k < 0 || bs[w] > b || (bs[w] == b && bi[w] < k));
    if (take) { b = bs[w]; k = bi[w]; }
  }
  hist[f] = sqrt(e2);
  if (k < 0 || (tol > 0.0 && b < tol * e2)) {
    ctl[CTL_CONVERGED] = k >= 0 ? 1 : 0;
    store_flag(&ctl[CTL_DONE], 1);
    return;
  }
  const double da = g[k] * rdn[k];
  Jd[f] = (int32_t)k;
  dad[f] = da;
  a64[k] += da;
  selected[k] = 1;
  ctl[CTL_SWEEPS] = f + 1;
  *step_j = k;
  *step_da = da;
}

// e <- e - X_j da (FP64 residual, FP32 column) for the step just chosen.
__global__ void __launch_bounds__(256) k_select_axpy(const float* X, int64_t ldx, int64_t m, double* e,
                                                     const int64_t* step_j, const double* step_da,
                                                     const int32_t* ctl) {
  if (load_flag(&ctl[CTL_DONE])) return;
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= m) return;
  const int64_t j = *step_j;
  e[i] = fma(-(double)X[j * ldx + i], *step_da, e[i]);
}

// ||e||^2 partial sums of an FP64 vector (one per workgroup of 1024 rows).
__global__ void __launch_bounds__(256) k_sumsq_f64(const double* e, int64_t m, double* part) {
  double acc = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * 1024 + threadIdx.x; i < min(m, (int64_t)(blockIdx.x + 1) * 1024); i += 256)
    acc = fma(e[i], e[i], acc);
  __shared__ double red[4];
  const double t = wave_sum(acc);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = t;
  __syncthreads();
  if (threadIdx.x == 0) part[blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
}

__global__ void __launch_bounds__(256) k_sqrt_sum(const double* part, int64_t count, double* out) {
  __shared__ double red[4];
  const double t = block_sum_f64(part, count, red);
  if (threadIdx.x == 0) *out = sqrt(t);
}

__global__ void k_to_f64(const float* src, double* dst, int64_t m) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < m) dst[i] = (double)src[i];
}

inline dim3 grid1(int64_t n) { return dim3((unsigned)std::max<int64_t>(1, (n + 255) / 256)); }

}  // namespace

XtvPlan plan_xtv(int64_t m, int64_t n, int64_t cap) {
  // Row strips of whole 1024-row sub-strips: about 2048 workgroups (eight
  // per CU, four waves each with sixteen 16-byte loads in flight), within
  // the partial-sum space.
  XtvPlan p{};
  const int64_t G = (n + XTV_COLS - 1) / XTV_COLS;
  const int64_t subs = (m + XTV_SUB - 1) / XTV_SUB;
  int64_t S = std::max<int64_t>(1, std::min<int64_t>(subs, (2048 + G - 1) / G));
  const int64_t T = (n + TILE - 1) / TILE;
  while (S > 1 && S * n + S + 3 * T > cap) --S;
  const int64_t per = (subs + S - 1) / S;
  p.rows_per = per * XTV_SUB;
  p.S = (m + p.rows_per - 1) / p.rows_per;
  p.G = G;
  p.T = T;
  p.need = p.S * n + p.S + 3 * p.T;
  return p;
}

hipError_t launch_xtv(const float* X, int64_t ldx, int64_t m, int64_t n, const void* v, bool v_f64,
                      const XtvPlan& p, double* partial, double* vnorm, const int32_t* done, hipStream_t s) {
  if (p.G > 65535) return hipErrorInvalidValue;
  const dim3 grid((unsigned)p.S, (unsigned)p.G);
  if (v_f64)
    hipLaunchKernelGGL(k_xtv<double>, grid, dim3(256), 0, s, X, ldx, m, n, static_cast<const double*>(v),
                       p.rows_per, partial, vnorm, done);
  else
    hipLaunchKernelGGL(k_xtv<float>, grid, dim3(256), 0, s, X, ldx, m, n, static_cast<const float*>(v),
                       p.rows_per, partial, vnorm, done);
  return hipGetLastError();
}

hipError_t launch_grad_stop(const float* X, int64_t ldx, int64_t m, int64_t n, const float* e, bool init,
                            int32_t sweep, double tol, double* ws, int64_t cap, int32_t* ctl, int64_t* ctl64,
                            double* fstat, double* hist, hipStream_t s) {
  const XtvPlan p = plan_xtv(m, n, cap);
  if (p.need > cap) return hipErrorInvalidValue;
  double* partial = ws;
  double* vnorm = ws + p.S * n;
  double* tsum = vnorm + p.S;
  hipError_t err = launch_xtv(X, ldx, m, n, e, false, p, partial, vnorm, &ctl[CTL_DONE], s);
  if (err != hipSuccess) return err;
  hipLaunchKernelGGL(k_xtv_tiles, dim3((unsigned)p.T), dim3(256), 0, s, partial, p.S, n, 0, nullptr, nullptr, nullptr,
                     tsum, nullptr, nullptr, &ctl[CTL_DONE]);
  hipLaunchKernelGGL(k_grad_stop, dim3(1), dim3(256), 0, s, tsum, p.T, vnorm, p.S, init ? 1 : 0, sweep, n, tol, ctl,
                     ctl64, fstat, hist);
  return hipGetLastError();
}

hipError_t launch_select_step(const float* X, int64_t ldx, int64_t m, int64_t n, double* e, const XtvPlan& p,
                              double* partial, double* vnorm, double* g, double* tscore, int64_t* tidx,
                              const double* rdn, int32_t f, double tol, int32_t* selected, double* a64, int32_t* Jd,
                              double* dad, double* hist, int32_t* ctl, int64_t* step_j, double* step_da,
                              hipStream_t s) {
  hipError_t err = launch_xtv(X, ldx, m, n, e, true, p, partial, vnorm, &ctl[CTL_DONE], s);
  if (err != hipSuccess) return err;
  hipLaunchKernelGGL(k_xtv_tiles, dim3((unsigned)p.T), dim3(256), 0, s, partial, p.S, n, 1, rdn, selected, g,
                     nullptr, tscore, tidx, &ctl[CTL_DONE]);
  hipLaunchKernelGGL(k_select_pick, dim3(1), dim3(256), 0, s, tscore, tidx, p.T, vnorm, p.S, g, rdn, f, tol,
                     selected, a64, Jd, dad, hist, ctl, step_j, step_da);
  hipLaunchKernelGGL(k_select_axpy, grid1(m), dim3(256), 0, s, X, ldx, m, e, step_j, step_da, ctl);
  return hipGetLastError();
}

hipError_t launch_norm_f64(const double* e, int64_t m, double* part, double* out, hipStream_t s) {
  const int64_t blocks = (m + 1023) / 1024;
  hipLaunchKernelGGL(k_sumsq_f64, dim3((unsigned)blocks), dim3(256), 0, s, e, m, part);
  hipLaunchKernelGGL(k_sqrt_sum, dim3(1), dim3(256), 0, s, part, blocks, out);
  return hipGetLastError();
}

hipError_t launch_to_f64(const float* src, double* dst, int64_t m, hipStream_t s) {
  hipLaunchKernelGGL(k_to_f64, grid1(m), dim3(256), 0, s, src, dst, m);
  return hipGetLastError();
}

}  // namespace hpscd
