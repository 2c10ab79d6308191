// Auxiliary kernels of the HPSCD solver: column statistics, FP64 residuals,
// bfloat16 conversion and small fills.
//
// Column statistics.  Algorithm 1 divides by <X_j, X_j> at every step; the
// value is constant, so it is computed once per solve (FP64 sums) and stored
// as its reciprocal (0 for a zero column, which the solver then skips).  For
// blocks of B > 1 columns the sweep kernels also need the strictly-lower
// in-block Gram entries <X_l, X_i>, i < l, computed in the same pass.
//
// Residual.  r = y - X·a with FP64 accumulation is used for the initial
// residual of a warm start (Algorithm 1 forms e = y - X·a from the initial
// guess), for the periodic refresh of the bfloat16-storage form, and for the
// final FP64 check ||y - X·a||_2.
#include "hpscd_device.hpp"
#include "hpscd_internal.hpp"

#include <float.h>

namespace hpscd {

template <class S>
__device__ inline float chunk_at(const typename S::raw_t& r, int i) { return S::get(r, i); }

// ------------------------------------------------------------- column stats
// Grid (PR, NBG) of 256-thread workgroups.  Wave w of workgroup (rx, gy)
// handles column blocks b = gy*4 + w (+ strides) over rows
// [rx*rows_per, (rx+1)*rows_per) and writes its FP64 partial sums to
// partial[(rx*nb + b)*NPX + q]: first the NP = B(B+1)/2 in-block pairs (l, i<=l)
// at l(l+1)/2 + i, then (CROSS) the B*B pairs <X_{b,l}, X_{b-1,i}> with the
// previous block at NP + l*B + i (zero for b = 0).
template <class S, int B, bool CROSS>
__global__ void __launch_bounds__(256) k_colgram(const void* X, int64_t ldx, int64_t m, int64_t n,
                                                 int64_t rows_per, double* partial) {
  using raw = typename S::raw_t;
  constexpr int VEC = S::VEC, NP = B * (B + 1) / 2, NX = CROSS ? B * B : 0, NPX = NP + NX;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t nb = (n + B - 1) / B;
  const int64_t r0 = (int64_t)blockIdx.x * rows_per;
  const int64_t r1 = min(m, r0 + rows_per);
  for (int64_t b = (int64_t)blockIdx.y * 4 + wave; b < nb; b += (int64_t)gridDim.y * 4) {
    double acc[NPX];
#pragma unroll
    for (int q = 0; q < NPX; ++q) acc[q] = 0.0;
    for (int64_t row = r0 + (int64_t)lane * VEC; row < r1; row += 64 * VEC) {
      const int lim = (int)min((int64_t)VEC, r1 - row);
      raw x[B], xp[CROSS ? B : 1];
#pragma unroll
      for (int l = 0; l < B; ++l) {
        const int64_t j = b * B + l;
        x[l] = (j < n) ? load_chunk<S>(X, j * ldx + row) : S::zero();
        if (lim < VEC) x[l] = mask_chunk<S>(x[l], lim);
      }
      if constexpr (CROSS) {
#pragma unroll
        for (int l = 0; l < B; ++l) {
          const int64_t j = (b - 1) * B + l;
          xp[l] = (b > 0) ? load_chunk<S>(X, j * ldx + row) : S::zero();
          if (lim < VEC) xp[l] = mask_chunk<S>(xp[l], lim);
        }
      }
#pragma unroll
      for (int i = 0; i < VEC; ++i) {
        double v[B];
#pragma unroll
        for (int l = 0; l < B; ++l) v[l] = (double)chunk_at<S>(x[l], i);
#pragma unroll
        for (int l = 0; l < B; ++l)
#pragma unroll
          for (int k = 0; k <= l; ++k) acc[l * (l + 1) / 2 + k] = fma(v[l], v[k], acc[l * (l + 1) / 2 + k]);
        if constexpr (CROSS) {
#pragma unroll
          for (int l = 0; l < B; ++l)
#pragma unroll
            for (int k = 0; k < B; ++k)
              acc[NP + l * B + k] = fma(v[l], (double)chunk_at<S>(xp[k], i), acc[NP + l * B + k]);
        }
      }
    }
#pragma unroll
    for (int q = 0; q < NPX; ++q) {
      const double sum = wave_sum(acc[q]);
      if (lane == q % 64) partial[((int64_t)blockIdx.x * nb + b) * NPX + q] = sum;
    }
  }
}

// The same statistics for blocks of 16 columns on the matrix cores: the
// block's Gram matrix X_b^T X_b is a dense contraction over the rows, summed
// with v_mfma_f64_16x16x4 (FP64 products of the FP32 or BF16 values, exact,
// and FP64 sums).  Lane (j, k) = (lane % 16, lane / 16) loads 16 bytes of
// column j at rows row + k*VEC ..; multiply-add t takes element t of every
// lane, i.e. rows {row + k*VEC + t : k < 4} as its K = 4 slice, and the
// same register is both operands (A = X^T, B = X).  The accumulator holds
// G[lane/16 + 4*v][lane % 16] in element v (the instruction's result layout,
// checked on the device); the entries (l, i <= l) go to the partial sums in
// the layout of k_colgram.
// With a column order `map`, block position p = b*16 + j holds column
// map[p] (the blocks of one sweep in that order).  While ctl[CTL_DONE] is set
// (`done`), the kernel returns at once.
template <class S>
__global__ void __launch_bounds__(256) k_colgram16_mfma(const void* X, int64_t ldx, int64_t m, int64_t n,
                                                        int64_t rows_per, double* partial, const int32_t* map,
                                                        const int32_t* done) {
  using raw = typename S::raw_t;
  constexpr int VEC = S::VEC, B = 16, NP = B * (B + 1) / 2;
  if (done && load_flag(done)) return;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int j = lane & 15, kq = lane >> 4;
  const int64_t nb = (n + B - 1) / B;
  const int64_t r0 = (int64_t)blockIdx.x * rows_per;
  const int64_t r1 = min(m, r0 + rows_per);
  for (int64_t b = (int64_t)blockIdx.y * 4 + wave; b < nb; b += (int64_t)gridDim.y * 4) {
    const int64_t pos = b * B + j;
    const int64_t col = pos < n ? (map ? (int64_t)map[pos] : pos) : n;
    typedef double d4 __attribute__((ext_vector_type(4)));
    d4 acc = {0.0, 0.0, 0.0, 0.0};
    int64_t row = r0;
    // U row steps per round with all their loads issued first: one load in
    // flight per wave leaves the matrix cores idle for most of each load's
    // latency
    constexpr int U = 8;
    for (; row + U * 4 * VEC <= r1; row += U * 4 * VEC) {
      raw xs[U];
#pragma unroll
      for (int u = 0; u < U; ++u)
        xs[u] = col < n ? load_chunk<S>(X, col * ldx + row + (int64_t)(u * 4 + kq) * VEC) : S::zero();
#pragma unroll
      for (int u = 0; u < U; ++u)
#pragma unroll
        for (int t = 0; t < VEC; ++t) {
          const double v = (double)chunk_at<S>(xs[u], t);
          acc = __builtin_amdgcn_mfma_f64_16x16x4f64(v, v, acc, 0, 0, 0);
        }
    }
    for (; row < r1; row += 4 * VEC) {
      const int64_t rr = row + (int64_t)kq * VEC;
      const int64_t left = r1 - rr;
      const int lim = left <= 0 ? 0 : (left >= VEC ? VEC : (int)left);
      raw x = (col < n && lim > 0) ? load_chunk<S>(X, col * ldx + rr) : S::zero();
      if (lim < VEC) x = mask_chunk<S>(x, lim);
#pragma unroll
      for (int t = 0; t < VEC; ++t) {
        const double v = (double)chunk_at<S>(x, t);
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(v, v, acc, 0, 0, 0);
      }
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int l = kq + 4 * v, i = j;
      if (i <= l) partial[((int64_t)blockIdx.x * nb + b) * NP + l * (l + 1) / 2 + i] = acc[v];
    }
  }
}

// Sum the PR partials (fixed order) into rdn[nb*B], gram[nb*NG] and (CROSS)
// cross[nb*B*B].  WAVE: one wave per output, its lanes striding over the
// partials (many partials: tall systems); else one thread per output adding
// them in turn (a few partials: short, wide systems with many blocks).
template <int B, bool CROSS, bool WAVE>
__global__ void __launch_bounds__(256) k_colgram_reduce(const double* partial, int PR, int64_t n, double* rdn,
                                                        double* gram, double* cross, int32_t* ctl,
                                                        int64_t* zero_cols, const int32_t* done) {
  constexpr int NP = B * (B + 1) / 2, NG = B * (B - 1) / 2, NX = CROSS ? B * B : 0, NPX = NP + NX;
  if (done && load_flag(done)) return;
  const int64_t nb = (n + B - 1) / B;
  int64_t idx;
  double s = 0.0;
  if constexpr (WAVE) {
    const int lane = threadIdx.x & 63;
    idx = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (idx >= nb * NPX) return;
    const int64_t b = idx / NPX;
    const int q = (int)(idx % NPX);
    double acc = 0.0;
    for (int r = lane; r < PR; r += 64) acc += partial[((int64_t)r * nb + b) * NPX + q];
    s = wave_sum(acc);
    if (lane != 0) return;
  } else {
    idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (idx >= nb * NPX) return;
    for (int r = 0; r < PR; ++r) s += partial[(int64_t)r * nb * NPX + idx];
  }
  const int64_t b = idx / NPX;
  const int q = (int)(idx % NPX);
  if (q >= NP) {
    cross[b * NX + (q - NP)] = s;
    return;
  }
  int l = 0;
  while ((l + 1) * (l + 2) / 2 <= q) ++l;
  const int i = q - l * (l + 1) / 2;
  const int64_t j = b * B + l;
  if (i == l) {
    double r = 0.0;
    if (j < n) {
      if (!(s <= DBL_MAX)) store_flag(&ctl[CTL_NONFINITE], 1);
      else if (s == 0.0) { if (zero_cols) atomicAdd((unsigned long long*)zero_cols, 1ull); }
      else r = 1.0 / s;
    }
    rdn[b * B + l] = r;
  } else {
    gram[b * NG + l * (l - 1) / 2 + i] = (j < n) ? s : 0.0;
  }
}

template <int B, bool CROSS>
static void launch_colgram_reduce(const double* partial, int PR, int64_t n, double* rdn, double* gram,
                                  double* cross, int32_t* ctl, int64_t* zero_cols, const int32_t* done,
                                  hipStream_t s) {
  constexpr int NPX = B * (B + 1) / 2 + (CROSS ? B * B : 0);
  const int64_t total = (n + B - 1) / B * NPX;
  if (PR > 16)
    hipLaunchKernelGGL((k_colgram_reduce<B, CROSS, true>), dim3((unsigned)((total + 3) / 4)), dim3(256), 0, s,
                       partial, PR, n, rdn, gram, cross, ctl, zero_cols, done);
  else
    hipLaunchKernelGGL((k_colgram_reduce<B, CROSS, false>), dim3((unsigned)((total + 255) / 256)), dim3(256), 0,
                       s, partial, PR, n, rdn, gram, cross, ctl, zero_cols, done);
}

// Tables of 16-column blocks from those of 8-column blocks: the strictly
// lower in-block Gram of block b holds the in-block Gram entries of its two
// halves and the Gram of the second half against the first.  One thread per
// entry (l, i), i < l, at l(l-1)/2 + i.
__global__ void __launch_bounds__(256) k_gram16(const double* gram8, const double* cross8, int64_t nb8,
                                                int64_t nb16, double* gram16) {
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (t >= nb16 * 120) return;
  const int64_t b = t / 120;
  const int q = (int)(t % 120);
  int l = 1;
  while (l * (l - 1) / 2 + l <= q) ++l;
  const int i = q - l * (l - 1) / 2;
  const int64_t h0 = 2 * b, h1 = 2 * b + 1;
  double v = 0.0;
  if (l < 8) v = gram8[h0 * 28 + l * (l - 1) / 2 + i];
  else if (h1 < nb8) v = (i >= 8) ? gram8[h1 * 28 + (l - 8) * (l - 9) / 2 + (i - 8)] : cross8[h1 * 64 + (l - 8) * 8 + i];
  gram16[b * 120 + q] = v;
}

// Step matrix of each 16-column block.  With D = diag(<X_l,X_l>) and L the
// strictly lower in-block Gram, the block's sequential steps satisfy
// (D + L) da = g for the dots g taken against the residual at the start of
// the block (the forward substitution of the sweep kernels), so da = M g with
// M = (D + L)^{-1}, lower triangular.  Column k of M is that substitution
// applied to the unit vector e_k; a zero or padding column (reciprocal norm 0)
// gives a zero row, i.e. da_l = 0 as in the substitution.  One thread per
// (block, k); M of block b is row-major at minv[(b*16 + l)*16 + k].
//
// Algorithm 2 (Section 7, thr > 1): the columns of a sweep form consecutive
// blocks of thr, and every column of such a block steps against the residual
// at that block's start.  Within the 16-column block b (columns j0 .. j0+15)
// column l belongs to the thr-block starting at s_l = floor((j0+l)/thr)*thr.
// If s_l < j0 the sweep kernel takes its dot against the residual saved at
// s_l, so da_l = g_l / <X_l,X_l>.  Otherwise the kernel's dot is against the
// residual at j0, which still lacks the steps of the columns j0 .. s_l - 1 of
// this block; the substitution removes exactly those:
//     da_l = (g_l - sum_{i < s_l - j0} <X_l, X_i> da_i) / <X_l, X_l>.
// thr = 1 is the substitution of Algorithm 1.
template <bool PAR>
__global__ void __launch_bounds__(256) k_block_inverse16(const double* rdn, const double* gram, int64_t nb,
                                                         double* minv, int32_t thr, const int32_t* done) {
  if (done && load_flag(done)) return;
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (t >= nb * 16) return;
  const int64_t b = t / 16;
  const int k = (int)(t % 16);
  double x[16];
#pragma unroll
  for (int l = 0; l < 16; ++l) {
    double acc = (l == k) ? 1.0 : 0.0;
    if constexpr (PAR) {
      const int64_t j0 = b * 16;
      const int64_t s_l = (j0 + l) / thr * thr;
      const int upto = s_l < j0 ? 0 : (int)(s_l - j0);
#pragma unroll
      for (int i = 0; i < l; ++i)
        if (i < upto) acc -= gram[b * 120 + l * (l - 1) / 2 + i] * x[i];
    } else {
      // Algorithm 1: every earlier column of the block
#pragma unroll
      for (int i = 0; i < l; ++i) acc -= gram[b * 120 + l * (l - 1) / 2 + i] * x[i];
    }
    x[l] = acc * rdn[b * 16 + l];
    minv[(b * 16 + l) * 16 + k] = x[l];
  }
}

hipError_t launch_colgram_reduce32(const double* partial, int PR, int64_t n, double* rdn, double* gram, int32_t* ctl,
                                   int64_t* zero_cols, hipStream_t s) {
  launch_colgram_reduce<32, false>(partial, PR, n, rdn, gram, nullptr, ctl, zero_cols, nullptr, s);
  return hipGetLastError();
}

static hipError_t block_inverse16(const double* rdn, const double* gram, int64_t n, double* minv, hipStream_t s,
                                  int32_t thr = 0, const int32_t* done = nullptr) {
  const int64_t nb = (n + 15) / 16;
  const dim3 grid((unsigned)((nb * 16 + 255) / 256));
  if (thr > 1)
    hipLaunchKernelGGL(k_block_inverse16<true>, grid, dim3(256), 0, s, rdn, gram, nb, minv, thr, done);
  else
    hipLaunchKernelGGL(k_block_inverse16<false>, grid, dim3(256), 0, s, rdn, gram, nb, minv, thr, done);
  return hipGetLastError();
}

template <class S, int B, bool CROSS>
static hipError_t colgram_impl(const void* X, int64_t ldx, int64_t m, int64_t n, double* rdn, double* gram,
                               double* cross, double* partial, int64_t partial_cap, int32_t* ctl,
                               int64_t* zero_cols, hipStream_t s) {
  constexpr int NPX = B * (B + 1) / 2 + (CROSS ? B * B : 0);
  const int64_t nb = (n + B - 1) / B;
  // Enough waves to fill the chip (~8192), rows split only when the columns
  // alone cannot provide them.
  int64_t PR = 1;
  if (nb < 8192) PR = (8192 + nb - 1) / nb;
  const int64_t min_rows = 64 * S::VEC * 4;
  PR = std::max<int64_t>(1, std::min<int64_t>(PR, (m + min_rows - 1) / min_rows));
  while (PR > 1 && PR * nb * NPX > partial_cap) --PR;
  if (PR * nb * NPX > partial_cap) return hipErrorInvalidValue;
  int64_t rows_per = (m + PR - 1) / PR;
  rows_per = (rows_per + S::VEC - 1) / S::VEC * S::VEC;
  PR = (m + rows_per - 1) / rows_per;
  const int64_t NBG = std::min<int64_t>((nb + 3) / 4, 65535);
  hipLaunchKernelGGL((k_colgram<S, B, CROSS>), dim3((unsigned)PR, (unsigned)NBG), dim3(256), 0, s, X, ldx, m, n,
                     rows_per, partial);
  hipError_t err = hipGetLastError();
  if (err != hipSuccess) return err;
  launch_colgram_reduce<B, CROSS>(partial, (int)PR, n, rdn, gram, cross, ctl, zero_cols, nullptr, s);
  return hipGetLastError();
}

// As colgram_impl for blocks of 16 columns, the partial sums on the matrix
// cores (k_colgram16_mfma); the same reduction.
template <class S>
static hipError_t colgram16_mfma(const void* X, int64_t ldx, int64_t m, int64_t n, double* rdn, double* gram,
                                 double* partial, int64_t partial_cap, int32_t* ctl, int64_t* zero_cols,
                                 hipStream_t s, const int32_t* map, const int32_t* done) {
  constexpr int B = 16, NPX = B * (B + 1) / 2;
  const int64_t nb = (n + B - 1) / B;
  int64_t PR = 1;
  if (nb < 8192) PR = (8192 + nb - 1) / nb;
  const int64_t min_rows = 4 * S::VEC * 16;
  PR = std::max<int64_t>(1, std::min<int64_t>(PR, (m + min_rows - 1) / min_rows));
  while (PR > 1 && PR * nb * NPX > partial_cap) --PR;
  if (PR * nb * NPX > partial_cap) return hipErrorInvalidValue;
  int64_t rows_per = (m + PR - 1) / PR;
  rows_per = (rows_per + 4 * S::VEC - 1) / (4 * S::VEC) * (4 * S::VEC);
  PR = (m + rows_per - 1) / rows_per;
  const int64_t NBG = std::min<int64_t>((nb + 3) / 4, 65535);
  hipLaunchKernelGGL((k_colgram16_mfma<S>), dim3((unsigned)PR, (unsigned)NBG), dim3(256), 0, s, X, ldx, m, n,
                     rows_per, partial, map, done);
  hipError_t err = hipGetLastError();
  if (err != hipSuccess) return err;
  launch_colgram_reduce<B, false>(partial, (int)PR, n, rdn, gram, nullptr, ctl, zero_cols, done, s);
  return hipGetLastError();
}

hipError_t launch_colgram(const void* X, bool bf16, int64_t ldx, int64_t m, int64_t n, int B, double* rdn,
                          double* gram, double* cross, double* partial, int64_t partial_cap, int32_t* ctl,
                          int64_t* zero_cols, hipStream_t s, const int32_t* map, int32_t thr) {
  if ((map || thr > 1) && (B != 16 || bf16)) return hipErrorInvalidValue;
#define HPSCD_CG(BB)                                                                                           \
  case BB:                                                                                                     \
    if (cross)                                                                                                 \
      return bf16 ? colgram_impl<BF16, BB, true>(X, ldx, m, n, rdn, gram, cross, partial, partial_cap, ctl,     \
                                                 zero_cols, s)                                                 \
                  : colgram_impl<F32, BB, true>(X, ldx, m, n, rdn, gram, cross, partial, partial_cap, ctl,      \
                                                zero_cols, s);                                                 \
    return bf16 ? colgram_impl<BF16, BB, false>(X, ldx, m, n, rdn, gram, cross, partial, partial_cap, ctl,      \
                                                zero_cols, s)                                                  \
                : colgram_impl<F32, BB, false>(X, ldx, m, n, rdn, gram, cross, partial, partial_cap, ctl,       \
                                               zero_cols, s);
  switch (B) {
    HPSCD_CG(1) HPSCD_CG(2) HPSCD_CG(4) HPSCD_CG(8)
    case 16: {
      // FP32: one pass of the 16-column statistics.  BF16: the 16-column
      // tables from one pass of the 8-column statistics with the Gram of each
      // block against the previous one (cross must hold nb16 * 256 doubles:
      // the 8-column cross Gram, then the 8-column in-block Gram).  Then the
      // step matrices into cross.
      if (cross == nullptr) return hipErrorInvalidValue;
      if (!bf16) {
        const int32_t* done = map ? &ctl[CTL_DONE] : nullptr;
        hipError_t err =
            colgram16_mfma<F32>(X, ldx, m, n, rdn, gram, partial, partial_cap, ctl, zero_cols, s, map, done);
        return err != hipSuccess ? err : block_inverse16(rdn, gram, n, cross, s, thr, done);
      }
      const int64_t nb8 = (n + 7) / 8, nb16 = (n + 15) / 16;
      double* cross8 = cross;
      double* gram8 = cross + nb8 * 64;
      hipError_t err = launch_fill_f64(rdn + nb8 * 8, nb16 * 16 - nb8 * 8, 0.0, s);
      if (err != hipSuccess) return err;
      err = colgram_impl<BF16, 8, true>(X, ldx, m, n, rdn, gram8, cross8, partial, partial_cap, ctl, zero_cols, s);
      if (err != hipSuccess) return err;
      const int64_t total = nb16 * 120;
      hipLaunchKernelGGL(k_gram16, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, gram8, cross8, nb8, nb16,
                         gram);
      err = hipGetLastError();
      return err != hipSuccess ? err : block_inverse16(rdn, gram, n, cross, s);
    }
    default: return hipErrorInvalidValue;
  }
#undef HPSCD_CG
}

// Batched column statistics: one wave per (system, column block), all rows.
template <int B>
__global__ void __launch_bounds__(256) k_colgram_batched(const float* Xpool, const SysDesc* sys, int32_t count,
                                                         int64_t nblk_total, const int64_t* blk_first,
                                                         double* rdn, double* gram, int32_t* ctl) {
  using S = F32;
  using raw = S::raw_t;
  constexpr int VEC = S::VEC, NP = B * (B + 1) / 2, NG = B * (B - 1) / 2;
  const int lane = threadIdx.x & 63;
  const int64_t g = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (g >= nblk_total) return;
  int lo = 0, hi = count - 1;  // last system with blk_first <= g
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (blk_first[mid] <= g) lo = mid; else hi = mid - 1;
  }
  const SysDesc sd = sys[lo];
  const int64_t b = g - blk_first[lo];
  const float* X = Xpool + sd.x_off;
  double acc[NP];
#pragma unroll
  for (int q = 0; q < NP; ++q) acc[q] = 0.0;
  for (int64_t row = (int64_t)lane * VEC; row < sd.m; row += 64 * VEC) {
    const int lim = (int)min((int64_t)VEC, sd.m - row);
    raw x[B];
#pragma unroll
    for (int l = 0; l < B; ++l) {
      const int64_t j = b * B + l;
      x[l] = (j < sd.n) ? load_chunk<S>(X, j * sd.ldx + row) : S::zero();
      if (lim < VEC) x[l] = mask_chunk<S>(x[l], lim);
    }
#pragma unroll
    for (int i = 0; i < VEC; ++i) {
      double v[B];
#pragma unroll
      for (int l = 0; l < B; ++l) v[l] = (double)S::get(x[l], i);
#pragma unroll
      for (int l = 0; l < B; ++l)
#pragma unroll
        for (int k = 0; k <= l; ++k) acc[l * (l + 1) / 2 + k] = fma(v[l], v[k], acc[l * (l + 1) / 2 + k]);
    }
  }
  double* r = rdn + sd.g_off + b * B;
  double* gm = gram + (sd.g_off / B + b) * NG;
#pragma unroll
  for (int l = 0; l < B; ++l) {
#pragma unroll
    for (int k = 0; k <= l; ++k) {
      const double s = wave_sum(acc[l * (l + 1) / 2 + k]);
      if (lane == 0) {
        const bool valid = (b * B + l) < sd.n;
        if (k == l) {
          if (valid && !(s <= DBL_MAX)) store_flag(&ctl[CTL_NONFINITE], 1);
          r[l] = (valid && s > 0.0 && s <= DBL_MAX) ? 1.0 / s : 0.0;
        } else {
          gm[l * (l - 1) / 2 + k] = valid ? s : 0.0;
        }
      }
    }
  }
}

hipError_t launch_colgram_batched(const float* Xpool, const SysDesc* sys, int32_t count, int64_t nblk_total,
                                  const int64_t* blk_first, int B, double* rdn, double* gram, int32_t* ctl,
                                  hipStream_t s) {
  const dim3 grid((unsigned)((nblk_total + 3) / 4));
#define HPSCD_CGB(BB)                                                                                   \
  case BB:                                                                                              \
    hipLaunchKernelGGL((k_colgram_batched<BB>), grid, dim3(256), 0, s, Xpool, sys, count, nblk_total,    \
                       blk_first, rdn, gram, ctl);                                                      \
    return hipGetLastError();
  switch (B) {
    HPSCD_CGB(1) HPSCD_CGB(2) HPSCD_CGB(4) HPSCD_CGB(8)
    default: return hipErrorInvalidValue;
  }
#undef HPSCD_CGB
}

// ---------------------------------------------------------------- residual
// Tall layout: one thread per chunk of 4 rows, looping over the columns.
__global__ void __launch_bounds__(256) k_resid_rows(const float* X, int64_t ldx, int64_t m, int64_t ncols,
                                                    const float* y, const double* a64, const float* a32,
                                                    float* e_out, double* partial, const int32_t* skip_if,
                                                    double* e64_out) {
  if (skip_if && *skip_if) return;
  const int64_t row = ((int64_t)blockIdx.x * 256 + threadIdx.x) * 4;
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  const int lim = row < m ? (int)min((int64_t)4, m - row) : 0;
  if (lim > 0) {
    for (int i = 0; i < lim; ++i) acc[i] = (double)y[row + i];
    int64_t j = 0;
    if (!a64 && !a32) ncols = 0;
    for (; j + 4 <= ncols; j += 4) {
      float4 x[4];
      double aj[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        x[u] = load_chunk<F32>(X, (j + u) * ldx + row);
        aj[u] = a64 ? a64[j + u] : (double)a32[j + u];
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        acc[0] = fma(-(double)x[u].x, aj[u], acc[0]);
        acc[1] = fma(-(double)x[u].y, aj[u], acc[1]);
        acc[2] = fma(-(double)x[u].z, aj[u], acc[2]);
        acc[3] = fma(-(double)x[u].w, aj[u], acc[3]);
      }
    }
    for (; j < ncols; ++j) {
      const float4 x = load_chunk<F32>(X, j * ldx + row);
      const double aj = a64 ? a64[j] : (double)a32[j];
      acc[0] = fma(-(double)x.x, aj, acc[0]);
      acc[1] = fma(-(double)x.y, aj, acc[1]);
      acc[2] = fma(-(double)x.z, aj, acc[2]);
      acc[3] = fma(-(double)x.w, aj, acc[3]);
    }
  }
  double sq = 0.0;
  for (int i = 0; i < 4; ++i) {
    if (i < lim) {
      sq = fma(acc[i], acc[i], sq);
      if (e_out) e_out[row + i] = (float)acc[i];
      if (e64_out) e64_out[row + i] = acc[i];
    }
  }
  __shared__ double wsum[4];
  sq = wave_sum(sq);
  if ((threadIdx.x & 63) == 0) wsum[threadIdx.x >> 6] = sq;
  __syncthreads();
  if (threadIdx.x == 0) partial[blockIdx.x] = (wsum[0] + wsum[1]) + (wsum[2] + wsum[3]);
}

// Wide layout: workgroup g accumulates X[:, cols of g]·a for a tile of rows
// into partial[g*tile + row] (FP64, columns in order); k_resid_cols_reduce
// adds the partials.  RC_U columns are requested before their products are
// added, so a thread keeps RC_U * RC_CHUNKS 16-byte loads in flight.
constexpr int RC_CHUNKS = 2;  // chunks per thread per row tile: 2048 rows per tile
constexpr int RC_U = 8;
__global__ void __launch_bounds__(256) k_resid_cols(const float* X, int64_t ldx, int64_t m, int64_t row0,
                                                    int64_t ncols, int64_t cols_per, const double* a64,
                                                    const float* a32, double* partial, int64_t tile,
                                                    const int32_t* skip_if) {
  if (skip_if && *skip_if) return;
  const int64_t c0 = (int64_t)blockIdx.x * cols_per, c1 = min(ncols, c0 + cols_per);
  double acc[RC_CHUNKS][4];
  int64_t rr[RC_CHUNKS];
  int lim[RC_CHUNKS];
#pragma unroll
  for (int q = 0; q < RC_CHUNKS; ++q) {
    rr[q] = row0 + ((int64_t)threadIdx.x + 256 * q) * 4;
    lim[q] = rr[q] < m ? (int)min((int64_t)4, m - rr[q]) : 0;
    for (int i = 0; i < 4; ++i) acc[q][i] = 0.0;
  }
  auto coef = [&](int64_t j) { return a64 ? a64[j] : (a32 ? (double)a32[j] : 0.0); };
  auto add = [&](const float4 (&x)[RC_CHUNKS], double aj) {
#pragma unroll
    for (int q = 0; q < RC_CHUNKS; ++q) {
      const float4 v = lim[q] < 4 ? mask_chunk<F32>(x[q], lim[q]) : x[q];
      acc[q][0] = fma((double)v.x, aj, acc[q][0]);
      acc[q][1] = fma((double)v.y, aj, acc[q][1]);
      acc[q][2] = fma((double)v.z, aj, acc[q][2]);
      acc[q][3] = fma((double)v.w, aj, acc[q][3]);
    }
  };
  int64_t j = c0;
  for (; j + RC_U <= c1; j += RC_U) {
    float4 x[RC_U][RC_CHUNKS];
#pragma unroll
    for (int u = 0; u < RC_U; ++u)
#pragma unroll
      for (int q = 0; q < RC_CHUNKS; ++q)
        x[u][q] = lim[q] > 0 ? load_chunk<F32>(X, (j + u) * ldx + rr[q]) : make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
    for (int u = 0; u < RC_U; ++u) add(x[u], coef(j + u));
  }
  for (; j < c1; ++j) {
    float4 x[RC_CHUNKS];
#pragma unroll
    for (int q = 0; q < RC_CHUNKS; ++q)
      x[q] = lim[q] > 0 ? load_chunk<F32>(X, j * ldx + rr[q]) : make_float4(0.f, 0.f, 0.f, 0.f);
    add(x, coef(j));
  }
#pragma unroll
  for (int q = 0; q < RC_CHUNKS; ++q)
    for (int i = 0; i < 4; ++i) {
      const int64_t r = rr[q] - row0 + i;
      if (r < tile) partial[(int64_t)blockIdx.x * tile + r] = acc[q][i];
    }
}

// Rows of a tile, 64 per workgroup (lane = row): y_r minus the sum of the G
// partials, wave w adding those of g in [w*GQ, (w+1)*GQ) in order (eight
// loads in flight), the four wave sums then added in order; writes e (FP32
// and/or FP64) and the workgroup's sum of squares.
__global__ void __launch_bounds__(256) k_resid_cols_reduce(const double* partial, int G, int64_t tile, int64_t row0,
                                                           int64_t m, const float* y, float* e_out,
                                                           double* sq_partial, const int32_t* skip_if,
                                                           double* e64_out) {
  if (skip_if && *skip_if) return;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int64_t r = (int64_t)blockIdx.x * 64 + lane;
  const int GQ = (G + 3) / 4;
  const int g0 = w * GQ, g1 = min(G, g0 + GQ);
  double s = 0.0;
  if (r < tile) {
    int g = g0;
    for (; g + 8 <= g1; g += 8) {
      double v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) v[u] = partial[(int64_t)(g + u) * tile + r];
#pragma unroll
      for (int u = 0; u < 8; ++u) s += v[u];
    }
    for (; g < g1; ++g) s += partial[(int64_t)g * tile + r];
  }
  __shared__ double ws[4][64];
  ws[w][lane] = s;
  __syncthreads();
  if (w != 0) return;
  double v = 0.0;
  if (r < tile && row0 + r < m) {
    const double tot = ((ws[0][lane] + ws[1][lane]) + ws[2][lane]) + ws[3][lane];
    v = (double)y[row0 + r] - tot;
    if (e_out) e_out[row0 + r] = (float)v;
    if (e64_out) e64_out[row0 + r] = v;
  }
  const double sq = wave_sum(v * v);
  if (lane == 0) sq_partial[blockIdx.x] = sq;
}

// Fixed-order sum of `count` doubles into *out (single workgroup).
__global__ void __launch_bounds__(256) k_sum_f64(const double* v, int64_t count, double* out, int accumulate,
                                                 const int32_t* skip_if) {
  if (skip_if && *skip_if) return;
  double s = 0.0;
  for (int64_t i = threadIdx.x; i < count; i += 256) s += v[i];
  __shared__ double wsum[4];
  s = wave_sum(s);
  if ((threadIdx.x & 63) == 0) wsum[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    const double t = (wsum[0] + wsum[1]) + (wsum[2] + wsum[3]);
    *out = accumulate ? *out + t : t;
  }
}

hipError_t launch_residual(const float* X, int64_t ldx, int64_t m, int64_t ncols, const float* y,
                           const double* a64, const float* a32, float* e_out, double* norm2, double* partial,
                           int64_t partial_cap, const int32_t* skip_if, hipStream_t s, double* e64_out) {
  if (ncols == 0 || m >= 65536) {
    const int64_t G = (m + 1023) / 1024;
    if (G > partial_cap) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_resid_rows, dim3((unsigned)G), dim3(256), 0, s, X, ldx, m, ncols, y, a64, a32, e_out,
                       partial, skip_if, e64_out);
    hipError_t err = hipGetLastError();
    if (err != hipSuccess) return err;
    if (norm2) hipLaunchKernelGGL(k_sum_f64, dim3(1), dim3(256), 0, s, partial, G, norm2, 0, skip_if);
    return hipGetLastError();
  }
  // Column-split form for short, wide systems: up to 256 workgroups of at
  // least 32 columns each.
  const int64_t tile = 256 * RC_CHUNKS * 4;
  int64_t G = std::min<int64_t>(256, std::max<int64_t>(1, ncols / 32));
  const int64_t sqn = (tile + 63) / 64;
  while (G > 1 && G * tile + sqn * ((m + tile - 1) / tile) > partial_cap) G /= 2;
  const int64_t cols_per = (ncols + G - 1) / G;
  G = (ncols + cols_per - 1) / cols_per;
  const int64_t ntiles = (m + tile - 1) / tile;
  if (G * tile + sqn * ntiles > partial_cap) return hipErrorInvalidValue;
  double* sqp = partial + G * tile;
  for (int64_t t = 0; t < ntiles; ++t) {
    hipLaunchKernelGGL(k_resid_cols, dim3((unsigned)G), dim3(256), 0, s, X, ldx, m, t * tile, ncols, cols_per,
                       a64, a32, partial, tile, skip_if);
    hipLaunchKernelGGL(k_resid_cols_reduce, dim3((unsigned)sqn), dim3(256), 0, s, partial, (int)G, tile,
                       t * tile, m, y, e_out, sqp + t * sqn, skip_if, e64_out);
  }
  hipError_t err = hipGetLastError();
  if (err != hipSuccess) return err;
  if (norm2) hipLaunchKernelGGL(k_sum_f64, dim3(1), dim3(256), 0, s, sqp, sqn * ntiles, norm2, 0, skip_if);
  return hipGetLastError();
}

// Batched residual: one workgroup per system.
__global__ void __launch_bounds__(256) k_resid_batched(const float* Xpool, const float* ypool, const SysDesc* sys,
                                                       const double* a64pool, const float* a32pool, float* e_out,
                                                       double* norm2) {
  const SysDesc sd = sys[blockIdx.x];
  const float* X = Xpool + sd.x_off;
  double sq = 0.0;
  for (int64_t row = (int64_t)threadIdx.x * 4; row < sd.m; row += 1024) {
    const int lim = (int)min((int64_t)4, sd.m - row);
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    for (int i = 0; i < lim; ++i) acc[i] = (double)ypool[sd.y_off + row + i];
    if (a64pool || a32pool) {
      auto coef = [&](int64_t j) { return a64pool ? a64pool[sd.a_off + j] : (double)a32pool[sd.a_off + j]; };
      auto add = [&](float4 x, double aj) {
        if (lim < 4) x = mask_chunk<F32>(x, lim);
        acc[0] = fma(-(double)x.x, aj, acc[0]);
        acc[1] = fma(-(double)x.y, aj, acc[1]);
        acc[2] = fma(-(double)x.z, aj, acc[2]);
        acc[3] = fma(-(double)x.w, aj, acc[3]);
      };
      // (eight columns requested before their products are added, columns
      // in order)
      int64_t j = 0;
      for (; j + 8 <= sd.n; j += 8) {
        float4 x[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) x[u] = load_chunk<F32>(X, (j + u) * sd.ldx + row);
#pragma unroll
        for (int u = 0; u < 8; ++u) add(x[u], coef(j + u));
      }
      for (; j < sd.n; ++j) add(load_chunk<F32>(X, j * sd.ldx + row), coef(j));
    }
    for (int i = 0; i < lim; ++i) {
      sq = fma(acc[i], acc[i], sq);
      if (e_out) e_out[sd.y_off + row + i] = (float)acc[i];
    }
  }
  __shared__ double wsum[4];
  sq = wave_sum(sq);
  if ((threadIdx.x & 63) == 0) wsum[threadIdx.x >> 6] = sq;
  __syncthreads();
  if (threadIdx.x == 0 && norm2) norm2[blockIdx.x] = (wsum[0] + wsum[1]) + (wsum[2] + wsum[3]);
}

hipError_t launch_residual_batched(const float* Xpool, const float* ypool, const SysDesc* sys, int32_t count,
                                   const double* a64pool, const float* a32pool, float* e_out, double* norm2,
                                   hipStream_t s) {
  hipLaunchKernelGGL(k_resid_batched, dim3((unsigned)count), dim3(256), 0, s, Xpool, ypool, sys, a64pool, a32pool,
                     e_out, norm2);
  return hipGetLastError();
}

// --------------------------------------------------------------- conversion
// FP32 -> bfloat16, round to nearest with ties to even on the 16 discarded
// bits; NaN stays a quiet NaN.
__device__ inline uint16_t to_bf16_rne(float f) {
  const uint32_t u = __float_as_uint(f);
  if ((u & 0x7F800000u) == 0x7F800000u && (u & 0x007FFFFFu) != 0u) return (uint16_t)((u >> 16) | 0x0040u);
  const uint32_t bias = 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)((u + bias) >> 16);
}

__global__ void __launch_bounds__(256) k_f32_to_bf16(const float* src, uint16_t* dst, int64_t rows, int64_t cols,
                                                     int64_t lds, int64_t ldd) {
  const int64_t per_col = (rows + 7) / 8;
  const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (idx >= per_col * cols) return;
  const int64_t j = idx / per_col, r = (idx % per_col) * 8;
  uint16_t out[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) out[i] = (r + i < rows) ? to_bf16_rne(src[j * lds + r + i]) : (uint16_t)0;
  uint4 w;
  w.x = (uint32_t)out[0] | ((uint32_t)out[1] << 16);
  w.y = (uint32_t)out[2] | ((uint32_t)out[3] << 16);
  w.z = (uint32_t)out[4] | ((uint32_t)out[5] << 16);
  w.w = (uint32_t)out[6] | ((uint32_t)out[7] << 16);
  *reinterpret_cast<uint4*>(dst + j * ldd + r) = w;
}

hipError_t launch_f32_to_bf16(const float* src, uint16_t* dst, int64_t rows, int64_t cols, int64_t lds, int64_t ldd,
                              hipStream_t s) {
  const int64_t total = (rows + 7) / 8 * cols;
  hipLaunchKernelGGL(k_f32_to_bf16, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, src, dst, rows, cols,
                     lds, ldd);
  return hipGetLastError();
}

// ------------------------------------------------------------ read stream
// Reads every 16-byte chunk of a buffer once per pass, the bandwidth a pure
// read stream of HBM reaches: the measured denominator of the sweep kernels'
// roofline.  Each workgroup streams one contiguous segment, a wave reading
// 1 KB per load, sixteen 128-bit loads in flight per thread (the pattern
// that measured fastest: 6.2-6.3 TB/s on 1 GiB, against 5.1 TB/s for a
// grid-stride loop).  The loaded values only feed a sum that is stored when
// it is NaN (never for the finite data it is used on), so no load can be
// dropped.
__global__ void __launch_bounds__(256) k_read_stream(const float4* __restrict__ p, int64_t n4, float* sink) {
  constexpr int U = 16, T = 256;
  const int64_t per = (n4 + gridDim.x - 1) / gridDim.x;
  const int64_t b0 = (int64_t)blockIdx.x * per, b1 = min(n4, b0 + per);
  float acc = 0.f;
  int64_t i = b0 + threadIdx.x;
  for (; i + (U - 1) * T < b1; i += U * T) {
    float4 v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) v[u] = p[i + u * T];
#pragma unroll
    for (int u = 0; u < U; ++u) acc += (v[u].x + v[u].y) + (v[u].z + v[u].w);
  }
  for (; i < b1; i += T) {
    const float4 v = p[i];
    acc += (v.x + v.y) + (v.z + v.w);
  }
  if (acc != acc) sink[blockIdx.x * T + threadIdx.x] = acc;
}

hipError_t launch_read_stream(const void* p, int64_t bytes, int grid, float* sink, hipStream_t s) {
  hipLaunchKernelGGL(k_read_stream, dim3((unsigned)grid), dim3(256), 0, s, static_cast<const float4*>(p), bytes / 16,
                     sink);
  return hipGetLastError();
}

// -------------------------------------------------------------------- small
__global__ void k_a_out(const double* a64, float* a, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) a[i] = (float)a64[i];
}
__global__ void k_a_init(double* a64, const float* a0, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) a64[i] = a0 ? (double)a0[i] : 0.0;
}
__global__ void k_fill_u64(uint64_t* p, int64_t n, uint64_t v) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) p[i] = v;
}
__global__ void k_fill_i32(int32_t* p, int64_t n, int32_t v) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) p[i] = v;
}
__global__ void k_fill_f64(double* p, int64_t n, double v) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) p[i] = v;
}
__global__ void k_copy_f32(const float* s, float* d, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) d[i] = s[i];
}

__global__ void k_a_out_batched(const double* a64pool, float* apool, const SysDesc* sys) {
  const SysDesc sd = sys[blockIdx.x];
  for (int64_t j = threadIdx.x; j < sd.n; j += 256) apool[sd.a_off + j] = (float)a64pool[sd.a_off + j];
}

static inline dim3 g1(int64_t n) { return dim3((unsigned)std::max<int64_t>(1, (n + 255) / 256)); }

hipError_t launch_a_out(const double* a64, float* a, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_a_out, g1(n), dim3(256), 0, s, a64, a, n);
  return hipGetLastError();
}
hipError_t launch_a_out_batched(const double* a64pool, float* apool, const SysDesc* sys, int32_t count, hipStream_t s) {
  hipLaunchKernelGGL(k_a_out_batched, dim3((unsigned)count), dim3(256), 0, s, a64pool, apool, sys);
  return hipGetLastError();
}
hipError_t launch_a_init(double* a64, const float* a0, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_a_init, g1(n), dim3(256), 0, s, a64, a0, n);
  return hipGetLastError();
}
hipError_t launch_fill_u64(uint64_t* p, int64_t n, uint64_t v, hipStream_t s) {
  hipLaunchKernelGGL(k_fill_u64, g1(n), dim3(256), 0, s, p, n, v);
  return hipGetLastError();
}
hipError_t launch_fill_i32(int32_t* p, int64_t n, int32_t v, hipStream_t s) {
  hipLaunchKernelGGL(k_fill_i32, g1(n), dim3(256), 0, s, p, n, v);
  return hipGetLastError();
}
hipError_t launch_fill_f64(double* p, int64_t n, double v, hipStream_t s) {
  hipLaunchKernelGGL(k_fill_f64, g1(n), dim3(256), 0, s, p, n, v);
  return hipGetLastError();
}
hipError_t launch_copy_f32(const float* src, float* dst, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_copy_f32, g1(n), dim3(256), 0, s, src, dst, n);
  return hipGetLastError();
}

}  // namespace hpscd
