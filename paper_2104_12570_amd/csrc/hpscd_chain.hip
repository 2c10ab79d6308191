// Column chain of a short system (m <= 2048 rows) on one workgroup: the
// bfloat16-storage form and the FP32 form of Algorithm 1 (Section 2) on
// short wide systems, where the columns form one long sequential chain and
// no other workgroup can share it.
//
// The chain's speed is set by the time per block of B columns: the block's
// loads, one reduction of the B dots (plus ||e||^2) over the workgroup, the
// block's steps da = M g through its precomputed step matrix
// M = (D + L)^{-1} (the exact Algorithm 1 steps of the block, as in the
// grid kernels), and the axpy.  Here:
//  * all 512 threads hold 4 rows each (2048 rows), so a 2000-row system
//    keeps every thread busy: a column is one 16-byte (FP32) or 8-byte
//    (bfloat16) load per thread;
//  * the columns of the next two blocks are in flight while the current one
//    is reduced (a ring of three register blocks, every load unconditional):
//    a lone workgroup's loads take longer than one block's arithmetic;
//  * the block is as wide as the registers allow: 16 FP32 columns or 32
//    bfloat16 columns (the same registers for the ring) -- halving the
//    bytes halves a block's register footprint, so the storage form takes
//    half as many reductions per sweep;
//  * the step matrix of the next block is staged in LDS (double buffer) by
//    all threads; after the partial sums every wave computes four rows of
//    da = M g (16 lanes a row), wave 0 also the stop tests; one barrier
//    after the partial sums, one after da.
#include "hpscd_device.hpp"
#include "hpscd_internal.hpp"

#include <float.h>

namespace hpscd {

namespace {

// Four rows of a column per thread.
template <class S> struct Quad;
template <> struct Quad<F32> {
  using raw = float4;  // 16 bytes
  static constexpr int BYTES = 4;
  __device__ static inline raw load(__amdgpu_buffer_rsrc_t rs, int voff, int soff) {
    return __builtin_bit_cast(raw, __builtin_amdgcn_raw_buffer_load_b128(rs, voff, soff, 0));
  }
  __device__ static inline float get(const raw& r, int i) { return i == 0 ? r.x : i == 1 ? r.y : i == 2 ? r.z : r.w; }
  __device__ static inline void refresh(raw&) {}
  __device__ static inline raw mask(raw r, int lim) {
    if (lim < 1) r.x = 0.f;
    if (lim < 2) r.y = 0.f;
    if (lim < 3) r.z = 0.f;
    if (lim < 4) r.w = 0.f;
    return r;
  }
};
template <> struct Quad<BF16> {
  using raw = uint2;  // 8 bytes: four bfloat16 rows
  static constexpr int BYTES = 2;
  __device__ static inline raw load(__amdgpu_buffer_rsrc_t rs, int voff, int soff) {
    return __builtin_bit_cast(raw, __builtin_amdgcn_raw_buffer_load_b64(rs, voff, soff, 0));
  }
  __device__ static inline float get(const raw& r, int i) {
    const uint32_t w = (i >> 1) == 0 ? r.x : r.y;
    return __uint_as_float((i & 1) ? (w & 0xFFFF0000u) : (w << 16));
  }
  // (the packed words are declared changed, so the conversions are redone
  // from them instead of 128 converted values staying live)
  __device__ static inline void refresh(raw& r) { asm volatile("" : "+v"(r.x), "+v"(r.y)); }
  __device__ static inline raw mask(raw r, int lim) {
    if (lim < 1) r.x &= 0xFFFF0000u;
    if (lim < 2) r.x &= 0x0000FFFFu;
    if (lim < 3) r.y &= 0xFFFF0000u;
    if (lim < 4) r.y &= 0x0000FFFFu;
    return r;
  }
};

__device__ inline void chain_barrier() {
  asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
  __builtin_amdgcn_s_barrier();
  asm volatile("" ::: "memory");
}

typedef const SolveArgs __attribute__((address_space(4)))* KArgs;
__device__ inline KArgs kargs() {
  KArgs p = (KArgs)__builtin_amdgcn_kernarg_segment_ptr();
  asm volatile("" : "+s"(p));
  return p;
}

constexpr int CT = 512;            // threads
constexpr int CNW = CT / WAVE;     // waves
constexpr int CROWS = 4 * CT;      // rows held by the workgroup

template <class S, int B>
__global__ void __launch_bounds__(CT) k_sweep_chain(SolveArgs A) {
  using Q = Quad<S>;
  using raw = typename Q::raw;
  constexpr int NV = B + 1;
  __shared__ float red[CNW][NV];
  __shared__ double msh[2][B * B];  // step matrices of the current and the next block
  __shared__ float dash[B];
  __shared__ int flag;

  const int tid = threadIdx.x, lane = tid & (WAVE - 1);
  const int wave = __builtin_amdgcn_readfirstlane(tid / WAVE);
  const int64_t m = A.m, n = A.n;
  const int nb = (int)((n + B - 1) / B);
  if (A.ctl[CTL_NONFINITE] != 0 || A.ctl[CTL_DONE] != 0) return;

  // rows 4*tid .. 4*tid+3; a thread with no valid row rereads rows 0..3
  // (masked to zero), so no load leaves the column
  const int64_t r0 = 4 * (int64_t)tid;
  const int lim = r0 >= m ? 0 : (m - r0 >= 4 ? 4 : (int)(m - r0));
  const int64_t roff = lim > 0 ? r0 : 0;
  const bool straddle = __ballot(lim < 4) != 0;  // (wave-uniform)
  float e[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) e[i] = i < lim ? A.e0[r0 + i] : 0.f;

  const int64_t nblocks = A.blk_end - A.blk_begin;
  int bi = (int)(A.blk_begin % nb);
  int sdone = (int)(A.blk_begin / nb);
  double prev_norm = A.fstat[1];
  const double ynorm = sqrt(*A.ynorm2);
  const bool col_checks = A.check_cols > 0 && A.stop == STOP_REL_RESID;

  // column loads of block b through one buffer resource based at the
  // block's first column and spanning its valid columns (the range check
  // counts the scalar offset too): the row offset in a vector register, the
  // column offset as a scalar (a column past n reads column n-1 again: its
  // step-matrix rows and columns are zero, and it stays inside X)
  const int64_t col_bytes = A.ldx * (int64_t)Q::BYTES;
  const int voff = (int)(roff * Q::BYTES);
  struct BlockRef {
    __amdgpu_buffer_rsrc_t rs;
    int nvalid;
  };
  auto block_ref = [&](int b) {
    b = __builtin_amdgcn_readfirstlane(b);
    const int64_t j0 = (int64_t)b * B;
    const int nvalid = n - j0 < B ? (int)(n - j0) : B;
    const uint32_t nrec = (uint32_t)((int64_t)nvalid * col_bytes);  // (< 2^32: B * col_bytes is checked by the host)
    return BlockRef{__builtin_amdgcn_make_buffer_rsrc(
                        const_cast<char*>(reinterpret_cast<const char*>(A.X) + j0 * col_bytes), 0, (int)nrec,
                        0x00020000),
                    nvalid};
  };
  auto load_col = [&](const BlockRef& r, int l) {
    const int lc = l < r.nvalid ? l : r.nvalid - 1;
    return Q::load(r.rs, voff, (int)(lc * col_bytes));
  };
  auto load_block = [&](raw (&xb)[B], int b) {
    const BlockRef r = block_ref(b);
#pragma unroll
    for (int l = 0; l < B; ++l) xb[l] = load_col(r, l);
  };
  // the step matrix of block b: B*B doubles, MPT per thread
  constexpr int MPT = (B * B + CT - 1) / CT;  // (2 for B = 32, 1 for 16)
  auto load_m = [&](double (&mv)[MPT], int b) {
#pragma unroll
    for (int k = 0; k < MPT; ++k) {
      const int idx = (tid * MPT + k) % (B * B);
      mv[k] = A.minv[(int64_t)b * B * B + idx];
    }
  };
  auto store_m = [&](const double (&mv)[MPT], int buf) {
#pragma unroll
    for (int k = 0; k < MPT; ++k) {
      const int idx = tid * MPT + k;
      if (idx < B * B) msh[buf][idx] = mv[k];
    }
  };
  // block index k blocks after b (k small, wave-uniform)
  auto adv = [&](int b, int k) {
    b += k;
    while (b >= nb) b -= nb;
    return b;
  };

  // A ring of three register blocks.  Step t (block t in slot t mod 3)
  // requests block t + 2 into the slot that block t - 1 has just left,
  // spread over its dot products (one column load between the arithmetic of
  // two columns, so the memory pipeline works while the ALUs do); its step
  // matrix M(t + 3) goes into the register slot whose matrix was staged in
  // LDS at the end of step t - 1, and M(t + 1) is staged at the end of
  // step t.
  constexpr int NR = 3;
  raw xr[NR][B];
  double mr[NR][MPT];
  {
    double m0[MPT];
    load_m(m0, bi);
    store_m(m0, 0);
  }
  load_m(mr[1], adv(bi, 1));
  load_block(xr[0], bi);
  load_m(mr[2], adv(bi, 2));
  load_block(xr[1], adv(bi, 1));
  int mcur = 0;

  auto finalize = [&](int sd, bool conv, int64_t cols, double nrm2) {
    const KArgs K = kargs();
    K->ctl[CTL_SWEEPS] = sd;
    K->ctl[CTL_CONVERGED] = conv ? 1 : 0;
    K->ctl[CTL_DONE] = 1;
    K->ctl64[C64_COLS] = cols;
    K->fstat[0] = nrm2;
  };

  // da of the block is shared out as 16 lanes per row of M, four rows per
  // wave (waves 0 .. B/4 - 1); each lane takes B/16 entries of its row
  constexpr int QL = B / 16;
  const int mrow = 4 * wave + (lane >> 4);
  const int q0 = (lane & 15) * QL;
  const bool owns = wave < B / 4 && (lane & 15) == 0;

  // One block on the ring buffer x (which holds block bi); mnext holds the
  // step matrix of the next block.  Returns true when the solve stops.
  auto step = [&](raw(&x)[B], raw(&xfree)[B], double(&mload)[MPT], double(&mnext)[MPT]) -> bool {
    bi = __builtin_amdgcn_readfirstlane(bi);
    const int64_t j0 = (int64_t)bi * B;
    // a cancel request, looked at by wave 0 at a sweep's first block: read
    // before the block's work so that its trip to host memory overlaps it
    int32_t cancel_req = 0;
    if (bi == 0 && wave == 0) cancel_req = load_cancel(kargs()->cancel);
    load_m(mload, adv(bi, 3));
    const BlockRef ahead = block_ref(adv(bi, 2));
    // partial sums of this thread's rows: the B dots and ||e||^2
    {
      if (straddle) {
#pragma unroll
        for (int l = 0; l < B; ++l) x[l] = Q::mask(x[l], lim);
      }
      // sixteen dots at a time through one scattered wave sum (lane L holds
      // the total of dot h*16 + ((L >> 2) & 15))
#pragma unroll
      for (int h = 0; h < B / 16; ++h) {
        float p[16];
#pragma unroll
        for (int l = 0; l < 16; ++l) {
          float acc = 0.f;
#pragma unroll
          for (int i = 0; i < 4; ++i) acc = fmaf(Q::get(x[16 * h + l], i), e[i], acc);
          p[l] = acc;
          xfree[16 * h + l] = load_col(ahead, 16 * h + l);
          __builtin_amdgcn_sched_barrier(0);
        }
        const float t = wave_sum16_scatter(p);
        if ((lane & 3) == 0) red[wave][16 * h + (lane >> 2)] = t;
      }
      float pn = 0.f;
#pragma unroll
      for (int i = 0; i < 4; ++i) pn = fmaf(e[i], e[i], pn);
      const float tn = wave_sum(pn);
      if (lane == 0) red[wave][B] = tn;
    }
    chain_barrier();
    // da = M g: the totals g_q (FP64, fixed order) a lane needs, its terms
    // of row mrow, and the row's sum over its 16 lanes
    double da = 0.0;
    if (wave < B / 4) {
      double part = 0.0;
#pragma unroll
      for (int u = 0; u < QL; ++u) {
        double gq = 0.0;
#pragma unroll
        for (int w = 0; w < CNW; ++w) gq += (double)red[w][q0 + u];
        part = fma(msh[mcur][mrow * B + q0 + u], gq, part);
      }
      part += dpp_f64<0xB1>(part);   // quad_perm [1,0,3,2]
      part += dpp_f64<0x4E>(part);   // quad_perm [2,3,0,1]
      part += dpp_f64<0x141>(part);  // row_half_mirror
      part += dpp_f64<0x140>(part);  // row_mirror: every lane of the row holds the sum
      da = part;
      if ((lane & 15) == 0) dash[mrow] = (float)part;
    }
    // wave 0: ||e||^2 and the stop tests
    if (wave == 0) {
      double nrm2 = 0.0;
#pragma unroll
      for (int w = 0; w < CNW; ++w) nrm2 += (double)red[w][B];
      int stop = 0;  // 1: stop before this block, 2: non-finite, 3: aborted
      if (!(nrm2 <= DBL_MAX)) {
        stop = 2;
      } else if (bi == 0) {
        const KArgs K = kargs();
        const double nrm = sqrt(nrm2);
        bool conv = false, st = false;
        if (K->stop != STOP_NONE && nrm2 == 0.0) st = conv = true;
        else if (K->stop == STOP_REL_CHANGE && sdone >= 1 && (prev_norm - nrm) < K->tol * nrm) st = conv = true;
        else if (K->stop == STOP_REL_RESID && nrm < K->tol * ynorm) st = conv = true;
        if (!st && sdone >= K->max_sweeps) st = true;
        asm volatile("" : "+v"(cancel_req));  // (keeps the test, and the wait for the load, here)
        if (!st && cancel_req != 0) stop = 3;
        if (lane == 0) {
          K->hist[sdone] = nrm;
          K->fstat[1] = nrm;
          if (st) finalize(sdone, conv, (int64_t)sdone * n, nrm2);
        }
        prev_norm = nrm;
        if (st) stop = 1;
      } else if (col_checks) {
        const KArgs K = kargs();
        const int64_t cols = (int64_t)sdone * n + j0;
        if (cols % K->check_cols == 0 && (nrm2 == 0.0 || sqrt(nrm2) < K->tol * ynorm)) {
          if (lane == 0) finalize(sdone, true, cols, nrm2);
          stop = 1;
        }
      }
      if (stop >= 2 && lane == 0) {
        const KArgs K = kargs();
        store_flag(&K->ctl[CTL_ERR], stop == 3 ? ERR_ABORTED : ERR_NONFINITE);
        finalize(sdone, false, (int64_t)sdone * n + j0, nrm2);
      }
      if (lane == 0) flag = stop;
    }
    chain_barrier();
    if (flag) return true;
    // (an atomic add without return: no load to wait for, which would also
    // wait for the columns in flight)
    if (owns && j0 + mrow < n)
      (void)__hip_atomic_fetch_add(&A.a64[j0 + mrow], da, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    // the axpy with the block's B steps
#pragma unroll
    for (int l = 0; l < B; ++l) Q::refresh(x[l]);
#pragma unroll
    for (int l = 0; l < B; ++l) {
      const float f = dash[l];
#pragma unroll
      for (int i = 0; i < 4; ++i) e[i] = fmaf(-f, Q::get(x[l], i), e[i]);
    }
    if (straddle) {
#pragma unroll
      for (int i = 0; i < 4; ++i) e[i] = i < lim ? e[i] : 0.f;
    }
    // next: stage the next block's step matrix
    store_m(mnext, mcur ^ 1);
    mcur ^= 1;
    bi = adv(bi, 1);
    if (bi == 0) ++sdone;
    return false;
  };
  // (NR steps per iteration, so each ring buffer is a fixed register array)
  static_assert(NR == 3, "the loop below is written for a ring of three");
  for (int64_t k = 0; k < nblocks; k += NR) {
    if (step(xr[0], xr[2], mr[0], mr[1])) break;
    if (k + 1 >= nblocks || step(xr[1], xr[0], mr[1], mr[2])) break;
    if (k + 2 >= nblocks || step(xr[2], xr[1], mr[2], mr[0])) break;
  }
  for (int i = 0; i < 4; ++i)
    if (i < lim) A.e_out[r0 + i] = e[i];
}

// ----------------------------------------------------------- 32-column Gram
// The Gram matrix X_b^T X_b of 32-column blocks on the FP64 matrix cores, as
// k_colgram16_mfma does for 16 columns: wave w of workgroup (rx, gy) takes
// block b = gy*4 + w over the rows of strip rx; lane (j, k) loads 16 bytes of
// columns j and 16 + j at rows row + k*VEC.., and three 16 x 16 x 4
// multiply-adds per element build the tiles (0,0), (1,1) and (1,0) (A = the
// first operand's columns).  The entries (l, i <= l) go to
// partial[(rx*nb + b)*528 + l(l+1)/2 + i] (FP64 products of the stored
// values, exact; FP64 sums).
template <class S>
__global__ void __launch_bounds__(256) k_colgram32_mfma(const void* X, int64_t ldx, int64_t m, int64_t n,
                                                        int64_t rows_per, double* partial) {
  using raw = typename S::raw_t;
  constexpr int VEC = S::VEC, B = 32, NP = B * (B + 1) / 2;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int j = lane & 15, kq = lane >> 4;
  const int64_t nb = (n + B - 1) / B;
  const int64_t r0 = (int64_t)blockIdx.x * rows_per;
  const int64_t r1 = min(m, r0 + rows_per);
  typedef double d4 __attribute__((ext_vector_type(4)));
  for (int64_t b = (int64_t)blockIdx.y * 4 + wave; b < nb; b += (int64_t)gridDim.y * 4) {
    const int64_t c0 = b * B + j, c1 = b * B + 16 + j;
    d4 t00 = {0.0, 0.0, 0.0, 0.0}, t11 = t00, t10 = t00;
    for (int64_t row = r0; row < r1; row += 4 * VEC) {
      const int64_t rr = row + (int64_t)kq * VEC;
      const int64_t left = r1 - rr;
      const int lim = left <= 0 ? 0 : (left >= VEC ? VEC : (int)left);
      raw a = (c0 < n && lim > 0) ? load_chunk<S>(X, c0 * ldx + rr) : S::zero();
      raw c = (c1 < n && lim > 0) ? load_chunk<S>(X, c1 * ldx + rr) : S::zero();
      if (lim < VEC) {
        a = mask_chunk<S>(a, lim);
        c = mask_chunk<S>(c, lim);
      }
#pragma unroll
      for (int t = 0; t < VEC; ++t) {
        const double va = (double)S::get(a, t), vc = (double)S::get(c, t);
        t00 = __builtin_amdgcn_mfma_f64_16x16x4f64(va, va, t00, 0, 0, 0);
        t11 = __builtin_amdgcn_mfma_f64_16x16x4f64(vc, vc, t11, 0, 0, 0);
        t10 = __builtin_amdgcn_mfma_f64_16x16x4f64(vc, va, t10, 0, 0, 0);
      }
    }
    // element v of a tile: row lane/16 + 4v, column lane mod 16
    double* out = partial + ((int64_t)blockIdx.x * nb + b) * NP;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int rl = kq + 4 * v, ci = j;
      if (ci <= rl) {
        out[rl * (rl + 1) / 2 + ci] = t00[v];
        out[(16 + rl) * (17 + rl) / 2 + 16 + ci] = t11[v];
      }
      out[(16 + rl) * (17 + rl) / 2 + ci] = t10[v];
    }
  }
}

// Step matrices of 32-column blocks: M = (D + L)^{-1}, column k of M by
// forward substitution on the unit vector e_k (as k_block_inverse16).
__global__ void __launch_bounds__(256) k_block_inverse32(const double* rdn, const double* gram, int64_t nb,
                                                         double* minv) {
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (t >= nb * 32) return;
  const int64_t b = t / 32;
  const int k = (int)(t % 32);
  double x[32];
#pragma unroll
  for (int l = 0; l < 32; ++l) {
    double acc = (l == k) ? 1.0 : 0.0;
#pragma unroll
    for (int i = 0; i < l; ++i) acc -= gram[b * 496 + l * (l - 1) / 2 + i] * x[i];
    x[l] = acc * rdn[b * 32 + l];
    minv[(b * 32 + l) * 32 + k] = x[l];
  }
}

}  // namespace

bool chain_variant_exists(bool bf16, int B) { return bf16 ? B == 32 : B == 16; }
int chain_max_rows() { return CROWS; }

hipError_t launch_chain(bool bf16, int B, const SolveArgs& a, hipStream_t s) {
  SolveArgs args = a;
  if (bf16 && B == 32) hipLaunchKernelGGL((k_sweep_chain<BF16, 32>), dim3(1), dim3(CT), 0, s, args);
  else if (!bf16 && B == 16) hipLaunchKernelGGL((k_sweep_chain<F32, 16>), dim3(1), dim3(CT), 0, s, args);
  else return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_colgram32(const void* X, bool bf16, int64_t ldx, int64_t m, int64_t n, double* rdn, double* gram,
                            double* minv, double* partial, int64_t partial_cap, int32_t* ctl, int64_t* zero_cols,
                            hipStream_t s) {
  constexpr int B = 32, NP = B * (B + 1) / 2;
  const int64_t nb = (n + B - 1) / B;
  const int vec = bf16 ? 8 : 4;
  int64_t PR = 1;
  if (nb < 8192) PR = (8192 + nb - 1) / nb;
  const int64_t min_rows = 4 * vec * 16;
  PR = std::max<int64_t>(1, std::min<int64_t>(PR, (m + min_rows - 1) / min_rows));
  while (PR > 1 && PR * nb * NP > partial_cap) --PR;
  if (PR * nb * NP > partial_cap) return hipErrorInvalidValue;
  int64_t rows_per = (m + PR - 1) / PR;
  rows_per = (rows_per + 4 * vec - 1) / (4 * vec) * (4 * vec);
  PR = (m + rows_per - 1) / rows_per;
  const int64_t NBG = std::min<int64_t>((nb + 3) / 4, 65535);
  if (bf16)
    hipLaunchKernelGGL(k_colgram32_mfma<BF16>, dim3((unsigned)PR, (unsigned)NBG), dim3(256), 0, s, X, ldx, m, n,
                       rows_per, partial);
  else
    hipLaunchKernelGGL(k_colgram32_mfma<F32>, dim3((unsigned)PR, (unsigned)NBG), dim3(256), 0, s, X, ldx, m, n,
                       rows_per, partial);
  hipError_t err = hipGetLastError();
  if (err != hipSuccess) return err;
  err = launch_colgram_reduce32(partial, (int)PR, n, rdn, gram, ctl, zero_cols, s);
  if (err != hipSuccess) return err;
  hipLaunchKernelGGL(k_block_inverse32, dim3((unsigned)((nb * 32 + 255) / 256)), dim3(256), 0, s, rdn, gram, nb,
                     minv);
  return hipGetLastError();
}

}  // namespace hpscd
