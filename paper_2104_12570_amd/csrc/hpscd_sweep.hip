// Sweep kernels of the HPSCD solver (paper, Section 2, Algorithm 1).
//
// One step of Algorithm 1 for column j is
//     da = <X_j, e> / <X_j, X_j>,   e <- e - X_j da,   a_j <- a_j + da
// (Section 3 derives da as the one-column least-squares fit of e and the
// update as the residual recursion e_{k+1} = e_k - X da_k).
//
// Data flow on the GPU.  The residual e never leaves registers: the rows of
// the system are split over the threads of a "team" (a wave, a workgroup, or
// every workgroup of a persistent grid), each thread owning R chunks of VEC
// consecutive rows.  X is column-major and is streamed exactly once per sweep
// with 128-bit loads; the columns of the next block are loaded while the
// current block is being reduced, so the loads overlap the reduction.
//
// Columns are processed in blocks of B.  The team reduces the B dot products
// <X_l, e> of a block (against the residual at the start of the block) plus
// ||e||^2 in one round, then every thread recovers the exact sequential steps
// of the block by forward substitution with the block's Gram entries
//     da_l = (<X_l, e> - sum_{i<l} <X_l, X_i> da_i) / <X_l, X_l>,
// which is algebraically identical to running the B steps one after another
// (the residual after step i is e - sum_{i'<=i} X_i' da_i').  B = 1 is the
// literal per-column reduction.  The axpy of block b is fused with the dots of
// block b+1 in the same pass over the register-resident residual.
//
// The reduction of one block is: wave DPP sums -> LDS across the waves of a
// workgroup -> (grid teams only) one 64-bit {sequence, value} word per value
// and workgroup, published with a relaxed agent-scope atomic store and read
// back by every workgroup, summed in a fixed order so all workgroups compute
// bitwise identical da.
#include "hpscd_device.hpp"
#include "hpscd_internal.hpp"

#include <float.h>

#include <atomic>

namespace hpscd {

// Coefficients of one block (B reciprocal norms, then the strictly-lower
// Gram entries) are held one per lane across NCR registers and broadcast with
// readlane when the block is solved.
template <int B>
struct Coef {
  static constexpr int NG = B * (B - 1) / 2;
  static constexpr int NGD = NG + B;
  static constexpr int NCR = (B + WAVE - 1) / WAVE;                     // registers of reciprocal norms
  static constexpr int NCG = NG > 0 ? (NG + WAVE - 1) / WAVE : 0;       // registers of Gram entries
  double vr[NCR];
  double vg[NCG > 0 ? NCG : 1];

  // Every lane issues the same loads (indices clamped into range; lanes past
  // the last entry hold a copy that is never read), and nothing selects on
  // the loaded values, so the compiler can leave the loads in flight and
  // count them exactly when it waits.
  __device__ inline void load(const double* rdn, const double* gram, int64_t bi, int lane) {
    // bi: block index within the sweep
#pragma unroll
    for (int r = 0; r < NCR; ++r) {
      const int q = r * WAVE + lane;
      vr[r] = rdn[bi * B + (q < B ? q : B - 1)];
    }
#pragma unroll
    for (int r = 0; r < NCG; ++r) {
      const int q = r * WAVE + lane;
      vg[r] = gram[bi * NG + (q < NG ? q : NG - 1)];
    }
  }
  // Entry q of the block's table (q < B: reciprocal norm, then the Gram
  // entries); q is a compile-time constant after unrolling.
  __device__ inline double get(int q) const {
    return q < B ? readlane_f64(vr[q / WAVE], q % WAVE) : readlane_f64(vg[(q - B) / WAVE], (q - B) % WAVE);
  }
};

template <int B>
__device__ inline void forward_substitute(const double (&tot)[B + 1], const Coef<B>& cf, double (&da)[B]) {
#pragma unroll
  for (int l = 0; l < B; ++l) {
    double acc = tot[l];
#pragma unroll
    for (int i = 0; i < l; ++i) acc -= cf.get(B + l * (l - 1) / 2 + i) * da[i];
    da[l] = uniform_f64(acc * cf.get(l));
  }
}

// --------------------------------------------------------------------------
// Single-system kernel: a persistent grid (GRID) or one workgroup.
// --------------------------------------------------------------------------
template <class S, int T, int R, int B, bool GRID, int D>
__global__ void __launch_bounds__(T) k_sweep(SolveArgs A) {
  static_assert(D == 2 || D == 3 || (D == 4 && !GRID), "prefetch ring of 2 or 3 blocks (4 for one workgroup)");
  using raw = typename S::raw_t;
  constexpr int VEC = S::VEC;
  constexpr int NW = T / WAVE;
  constexpr int NV = B + 1;
  constexpr int MAXC = 8;                       // up to 512 workgroups in a grid team
  constexpr int MAXT = (NV * MAXC + NW - 1) / NW < 8 ? (NV * MAXC + NW - 1) / NW : 8;  // poll tasks per wave
  constexpr int CPW = (MAXC + NW - 1) / NW;  // chunks of 64 workgroups polled by one wave
  constexpr int NWD = NV * CPW;              // poll words per lane
  __shared__ float red[2][NW][NV];
  __shared__ double gsum[2][NV][MAXC];
  __shared__ int sflag;

  const int tid = threadIdx.x, lane = tid & (WAVE - 1), wave = tid / WAVE;
  const int wg = GRID ? (int)blockIdx.x : 0;
  const int64_t m = A.m, n = A.n;
  const int nb = (int)((n + B - 1) / B);
  if (A.ctl[CTL_NONFINITE] != 0 || A.ctl[CTL_DONE] != 0) return;
  if (tid == 0) sflag = 0;

  float e[R][VEC];
  int lim[R];
  int64_t rof[R];
  uint32_t boff[R];  // byte offset of the chunk inside a column (columns are < 4 GiB)
#pragma unroll
  for (int c = 0; c < R; ++c) {
    rof[c] = (int64_t)wg * (T * R * VEC) + (int64_t)VEC * (tid + T * c);
    const int64_t left = m - rof[c];
    lim[c] = left <= 0 ? 0 : (left >= VEC ? VEC : (int)left);
    boff[c] = (uint32_t)(rof[c] * (16 / VEC));
#pragma unroll
    for (int i = 0; i < VEC; ++i) e[c][i] = (i < lim[c]) ? A.e0[rof[c] + i] : 0.f;
  }

  double prev_norm = A.fstat[1];
  const double ynorm = sqrt(*A.ynorm2);
  const int64_t nblocks = A.blk_end - A.blk_begin;
  const int64_t col_bytes = A.ldx * (int64_t)(16 / VEC);
  // Ring of D register buffers: the current block and the next D-1 blocks,
  // whose loads are in flight while the current block is reduced.
  raw x0[B][R], x1[B][R], x2[D >= 3 ? B : 1][R], x3[D >= 4 ? B : 1][R];
  Coef<B> c0, c1, c2, c3;

  // Columns of one block are read through a buffer resource based at the
  // block's first column: one 32-bit lane offset per chunk, one scalar offset
  // per column, and loads past the last column of the system return zero.
  auto load_cols = [&](raw (&x)[B][R], int bi) {
    bi = __builtin_amdgcn_readfirstlane(bi);  // (uniform: keeps the resource in scalar registers)
    const int j0 = bi * B;
    const int nvalid = (n - j0) < B ? (int)(n - j0) : B;
    const int64_t span = (int64_t)(nvalid - 1) * col_bytes + A.ldx * (int64_t)(16 / VEC);
    const uint32_t nrec = span > 0xFFFFFFFFll ? 0xFFFFFFFFu : (uint32_t)span;
    const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
        const_cast<char*>(reinterpret_cast<const char*>(A.X) + (int64_t)j0 * col_bytes), 0, (int)nrec, 0x00020000);
    // Unconditional loads: rows past m read padding, the next column or (past
    // the resource's range) zero, and are masked before use; a fixed number
    // of loads per block keeps the compiler's wait counts exact.
#pragma unroll
    for (int l = 0; l < B; ++l) {
#pragma unroll
      for (int c = 0; c < R; ++c)
        x[l][c] = __builtin_bit_cast(raw, __builtin_amdgcn_raw_buffer_load_b128(rs, (int)boff[c], (int)(l * col_bytes), 0));
    }
  };
  auto load_block = [&](raw (&x)[B][R], Coef<B>& cf, int bi) {
    load_cols(x, bi);
    cf.load(A.rdn, A.gram, bi, lane);
  };

  auto finalize = [&](int sdone, bool conv, int64_t cols, double nrm2) {
    if (wg == 0 && tid == 0) {
      A.ctl[CTL_SWEEPS] = sdone;
      A.ctl[CTL_CONVERGED] = conv ? 1 : 0;
      A.ctl[CTL_DONE] = 1;
      A.ctl64[C64_COLS] = cols;
      A.fstat[0] = nrm2;
    }
  };

  // Position of the current block: global index k, index in the sweep bi,
  // complete sweeps before it sdone.
  int bi = (int)(A.blk_begin % nb);
  int sdone = (int)(A.blk_begin / nb);
  uint32_t seq = (uint32_t)(A.blk_begin + 1);

  // One block: returns true when the solve is over.  `pf` receives the
  // block D-1 ahead (when has_next).
  auto step = [&](raw (&cur)[B][R], auto& pf, Coef<B>& ccur, Coef<B>& cpf, bool has_next) -> bool {
    const int j0 = bi * B;
    const int nbi = (bi + 1 == nb) ? 0 : bi + 1;
    int pbi = bi + D - 1;
    while (pbi >= nb) pbi -= nb;
    auto prefetch = [&]() {
      if constexpr (sizeof(pf) == sizeof(cur)) load_block(pf, cpf, pbi);
    };
    // The block D-1 ahead is requested even past the end of the launch (it is
    // a valid block of the sweep, never used), so every step issues the same
    // loads.
    (void)has_next;
    if constexpr (!GRID) prefetch();

    float p[NV];
#pragma unroll
    for (int l = 0; l < B; ++l) {
      float acc = 0.f;
#pragma unroll
      for (int c = 0; c < R; ++c) {
        if (lim[c] < VEC) cur[l][c] = mask_chunk<S>(cur[l][c], lim[c]);
#pragma unroll
        for (int i = 0; i < VEC; ++i) acc = fmaf(S::get(cur[l][c], i), e[c][i], acc);
      }
      p[l] = acc;
    }
    {
      float acc = 0.f;
#pragma unroll
      for (int c = 0; c < R; ++c)
#pragma unroll
        for (int i = 0; i < VEC; ++i) acc = fmaf(e[c][i], e[c][i], acc);
      p[B] = acc;
    }
    // Cancellation: workgroup 0 turns its norm partial into NaN at a sweep
    // boundary, which every workgroup then sees in the reduced norm.
    bool aborting = false;
    if (bi == 0 && wg == 0 && tid == 0 && load_cancel(A.cancel) != 0) {
      p[B] = __int_as_float(0x7fc00000);
      aborting = true;
    }

    const int par = (int)(seq & 1u);
#pragma unroll
    for (int l = 0; l < NV; ++l) {
      const float v = wave_sum(p[l]);
      if (lane == 0) red[par][wave][l] = v;
    }
    __syncthreads();
    double tot[NV];
    if constexpr (GRID) {
      // Slots are [parity][value][workgroup], so the 64 lanes of a poll load
      // read 512 contiguous bytes.  Poll task t covers value l = t / ncn of
      // the 64 workgroups of chunk c = t % ncn; each wave issues all its task
      // loads at once, then the next block's loads, then re-polls only words
      // whose sequence number is not yet current.
      uint64_t* slot_base = A.slots + (int64_t)par * NV * A.P;
      // With two blocks resident, the next block's coefficients are requested
      // first and its columns right behind this wave's first poll loads: the
      // wait for the poll words then leaves the columns in flight.  (Vector
      // loads return in issue order, so a re-poll does wait behind them.)
      if constexpr (D == 2) {
        if constexpr (sizeof(pf) == sizeof(cur)) cpf.load(A.rdn, A.gram, pbi, lane);
      }
      if (tid < NV) {
        float sacc = 0.f;
#pragma unroll
        for (int w = 0; w < NW; ++w) sacc += red[par][w][tid];
        publish(slot_base + (int64_t)tid * A.P + wg, seq, sacc);
      }
      if (A.poll_delay) {
        const uint64_t t0d = now_ticks();
        while (now_ticks() - t0d < A.poll_delay) __builtin_amdgcn_s_sleep(2);
      }
      const int ncn = (A.P + WAVE - 1) / WAVE;
      bool timed_out = false;
      // Wave w reads chunk c = w (+ NW, ...) of 64 workgroups for every value:
      // word (l, c*64 + lane).  Every lane issues the same loads (lanes past
      // the last workgroup read a valid word and ignore it), no index needs a
      // division, and nothing selects on a loaded value before the wait, so
      // the wait for the poll words is an exact count that leaves the column
      // loads behind them in flight.
      uint64_t w[NWD];
#pragma unroll
      for (int k = 0; k < CPW; ++k) {
        const int idx = (wave + k * NW) * WAVE + lane;
        const bool live = wave + k * NW < MAXC && idx < A.P;
#pragma unroll
        for (int l = 0; l < NV; ++l) w[k * NV + l] = peek(slot_base + (int64_t)l * A.P + (live ? idx : 0));
      }
      if constexpr (D == 2) {
        if constexpr (sizeof(pf) == sizeof(cur)) load_cols(pf, pbi);
      }
#pragma unroll
      for (int k = 0; k < CPW; ++k) {
        const int idx = (wave + k * NW) * WAVE + lane;
        const bool live = wave + k * NW < MAXC && idx < A.P;
#pragma unroll
        for (int l = 0; l < NV; ++l)
          if (!live) w[k * NV + l] = (uint64_t)seq << 32;
      }
      uint64_t tstart = 0;
      for (int spin = 0;; ++spin) {
        bool ready = true;
#pragma unroll
        for (int q = 0; q < NWD; ++q) ready = ready && ((uint32_t)(w[q] >> 32) == seq);
        if (ready) break;
        if (spin == 0) tstart = now_ticks();
        else if (now_ticks() - tstart > A.timeout_ticks) {
          timed_out = true;
          break;
        }
        __builtin_amdgcn_s_sleep(1);
#pragma unroll
        for (int k = 0; k < CPW; ++k) {
          const int idx = (wave + k * NW) * WAVE + lane;
#pragma unroll
          for (int l = 0; l < NV; ++l)
            if ((uint32_t)(w[k * NV + l] >> 32) != seq) w[k * NV + l] = peek(slot_base + (int64_t)l * A.P + idx);
        }
      }
#pragma unroll
      for (int k = 0; k < CPW; ++k) {
        const int c = wave + k * NW;
        if (c < ncn) {  // wave-uniform
          const int idx = c * WAVE + lane;
#pragma unroll
          for (int l = 0; l < NV; ++l) {
            const double v = wave_sum(idx < A.P ? (double)__uint_as_float((uint32_t)w[k * NV + l]) : 0.0);
            if (lane == 0) gsum[par][l][c] = v;
          }
        }
      }
      if constexpr (D != 2) prefetch();
      if (timed_out) sflag = 1;
      __syncthreads();
      if (sflag) {
        if (tid == 0) store_flag(&A.ctl[CTL_ERR], ERR_TIMEOUT);
        return true;
      }
#pragma unroll
      for (int l = 0; l < NV; ++l) {
        double sacc = 0.0;
        for (int c = 0; c < ncn; ++c) sacc += gsum[par][l][c];
        tot[l] = uniform_f64(sacc);
      }
    } else {
#pragma unroll
      for (int l = 0; l < NV; ++l) {
        double sacc = 0.0;
#pragma unroll
        for (int w = 0; w < NW; ++w) sacc += (double)red[par][w][l];
        tot[l] = uniform_f64(sacc);
      }
    }

    const double nrm2 = tot[B];
    const double nrm = sqrt(nrm2);
    if (!(nrm2 <= DBL_MAX)) {  // NaN or Inf: cancelled, or the data overflowed
      if (wg == 0 && tid == 0) store_flag(&A.ctl[CTL_ERR], aborting ? ERR_ABORTED : ERR_NONFINITE);
      finalize(sdone, false, (int64_t)sdone * n + j0, nrm2);
      return true;
    }
    if (bi == 0) {
      if (wg == 0 && tid == 0) { A.hist[sdone] = nrm; A.fstat[1] = nrm; }
      bool stop = false, conv = false;
      if (A.stop != STOP_NONE && nrm2 == 0.0) stop = conv = true;
      else if (A.stop == STOP_REL_CHANGE && sdone >= 1 && (prev_norm - nrm) < A.tol * nrm) stop = conv = true;
      else if (A.stop == STOP_REL_RESID && nrm < A.tol * ynorm) stop = conv = true;
      if (!stop && sdone >= A.max_sweeps) stop = true;
      prev_norm = nrm;
      if (stop) { finalize(sdone, conv, (int64_t)sdone * n, nrm2); return true; }
    } else if (A.check_cols > 0 && A.stop == STOP_REL_RESID) {
      const int64_t cols = (int64_t)sdone * n + j0;
      if (cols % A.check_cols == 0 && (nrm2 == 0.0 || nrm < A.tol * ynorm)) {
        finalize(sdone, true, cols, nrm2);
        return true;
      }
    }

    double da[B];
    forward_substitute<B>(tot, ccur, da);
#pragma unroll
    for (int l = 0; l < B; ++l) {
      const float f = (float)da[l];
#pragma unroll
      for (int c = 0; c < R; ++c)
#pragma unroll
        for (int i = 0; i < VEC; ++i) e[c][i] = fmaf(-f, S::get(cur[l][c], i), e[c][i]);
    }
    // Every workgroup holds the same da; coefficient j is accumulated by
    // workgroup j mod P (one writer per coefficient, no return value waited for).
    if (tid < B) {
      const int64_t j = j0 + tid;
      if (j < n && (int)(j % A.P) == wg) {
        double d = 0.0;
#pragma unroll
        for (int l = 0; l < B; ++l) if (tid == l) d = da[l];
        (void)__hip_atomic_fetch_add(&A.a64[j], d, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
    }
    // advance to the next block
    bi = nbi;
    if (bi == 0) ++sdone;
    ++seq;
    return false;
  };

  if (nblocks > 0) load_block(x0, c0, bi);
  if constexpr (D >= 3) {
    if (nblocks > 1) load_block(x1, c1, bi + 1 == nb ? 0 : bi + 1);
  }
  if constexpr (D >= 4) {
    int b2 = bi + 2;
    while (b2 >= nb) b2 -= nb;
    if (nblocks > 2) load_block(x2, c2, b2);
  }
  __syncthreads();
  for (int64_t k = 0; k < nblocks;) {
    if constexpr (D == 2) {
      if (step(x0, x1, c0, c1, k + 1 < nblocks)) break;
      if (++k >= nblocks) break;
      if (step(x1, x0, c1, c0, k + 1 < nblocks)) break;
      ++k;
    } else if constexpr (D == 3) {
      if (step(x0, x2, c0, c2, k + 2 < nblocks)) break;
      if (++k >= nblocks) break;
      if (step(x1, x0, c1, c0, k + 2 < nblocks)) break;
      if (++k >= nblocks) break;
      if (step(x2, x1, c2, c1, k + 2 < nblocks)) break;
      ++k;
    } else {
      if (step(x0, x3, c0, c3, k + 3 < nblocks)) break;
      if (++k >= nblocks) break;
      if (step(x1, x0, c1, c0, k + 3 < nblocks)) break;
      if (++k >= nblocks) break;
      if (step(x2, x1, c2, c1, k + 3 < nblocks)) break;
      if (++k >= nblocks) break;
      if (step(x3, x2, c3, c2, k + 3 < nblocks)) break;
      ++k;
    }
  }
#pragma unroll
  for (int c = 0; c < R; ++c)
#pragma unroll
    for (int i = 0; i < VEC; ++i)
      if (i < lim[c]) A.e_out[rof[c] + i] = e[c][i];
}

// --------------------------------------------------------------------------
// Grid kernel with a polling wave that never waits behind column data.
//
// Vector loads of a wave return in issue order, so a wave that has requested
// the next block's columns sees the result of a later poll of the exchange
// words only after those columns have arrived: streaming and reduction
// latency add up.  Here the last wave of each workgroup does all the polling
// and issues no column loads of its own; its rows of every block are brought
// into LDS by the other waves with direct-to-LDS buffer loads, issued with
// their own column loads for the next block right after the partial sums are
// published.  The next block's columns then stream in while the exchange is
// in flight.  Arithmetic, reduction order and stop logic are those of k_sweep.
template <class S, int T, int R, int B, int NPW>
__global__ void __launch_bounds__(T) k_sweep_px(SolveArgs A) {
  using raw = typename S::raw_t;
  constexpr int VEC = S::VEC;
  constexpr int NW = T / WAVE;
  constexpr int NV = B + 1;
  constexpr int NH = NW - NPW;         // waves that stream columns
  constexpr int MAXC = 4;              // up to 256 workgroups
  constexpr int CPP = MAXC / NPW;      // chunks of 64 workgroups per polling wave
  static_assert(NW > NPW && MAXC % NPW == 0, "wave split");
  __shared__ float red[2][NW][NV];
  __shared__ raw pbuf[2][NPW][B][R][WAVE];  // the polling waves' rows of two blocks
  __shared__ double tpart[NPW][NV];
  __shared__ int sflag;

  const int tid = threadIdx.x, lane = tid & (WAVE - 1), wave = tid / WAVE;
  const bool pollw = wave >= NH;
  const int pw = pollw ? wave - NH : 0;
  const int wg = (int)blockIdx.x;
  const int64_t m = A.m, n = A.n;
  const int nb = (int)((n + B - 1) / B);
  if (A.ctl[CTL_NONFINITE] != 0 || A.ctl[CTL_DONE] != 0) return;
  if (tid == 0) sflag = 0;

  float e[R][VEC];
  int lim[R];
  int64_t rof[R];
  uint32_t boff[R];   // own rows
  uint32_t boffp[NPW][R];  // the polling waves' rows, lane for lane
#pragma unroll
  for (int c = 0; c < R; ++c) {
    rof[c] = (int64_t)wg * (T * R * VEC) + (int64_t)VEC * (tid + T * c);
    const int64_t left = m - rof[c];
    lim[c] = left <= 0 ? 0 : (left >= VEC ? VEC : (int)left);
    boff[c] = (uint32_t)(rof[c] * (16 / VEC));
#pragma unroll
    for (int q = 0; q < NPW; ++q) {
      const int64_t rofp = (int64_t)wg * (T * R * VEC) + (int64_t)VEC * ((NH + q) * WAVE + lane + T * c);
      boffp[q][c] = (uint32_t)(rofp * (16 / VEC));
    }
#pragma unroll
    for (int i = 0; i < VEC; ++i) e[c][i] = (i < lim[c]) ? A.e0[rof[c] + i] : 0.f;
  }

  double prev_norm = A.fstat[1];
  const double ynorm = sqrt(*A.ynorm2);
  const int64_t nblocks = A.blk_end - A.blk_begin;
  const int64_t col_bytes = A.ldx * (int64_t)(16 / VEC);
  raw x0[B][R], x1[B][R];
  Coef<B> c0, c1;

  auto rsrc = [&](int bi) {
    bi = __builtin_amdgcn_readfirstlane(bi);  // (uniform: keeps the resource in scalar registers)
    const int j0 = bi * B;
    const int nvalid = (n - j0) < B ? (int)(n - j0) : B;
    const int64_t span = (int64_t)(nvalid - 1) * col_bytes + A.ldx * (int64_t)(16 / VEC);
    const uint32_t nrec = span > 0xFFFFFFFFll ? 0xFFFFFFFFu : (uint32_t)span;
    return __builtin_amdgcn_make_buffer_rsrc(
        const_cast<char*>(reinterpret_cast<const char*>(A.X) + (int64_t)j0 * col_bytes), 0, (int)nrec, 0x00020000);
  };
  // Streaming waves: their own columns into registers and their share of the
  // polling wave's columns into LDS buffer `pb` (unconditional loads; rows
  // past m are masked before use).
  auto load_block = [&](raw (&x)[B][R], int bi, int pb) {
    const __amdgpu_buffer_rsrc_t rs = rsrc(bi);
#pragma unroll
    for (int l = 0; l < B; ++l)
#pragma unroll
      for (int c = 0; c < R; ++c)
        x[l][c] = __builtin_bit_cast(raw, __builtin_amdgcn_raw_buffer_load_b128(rs, (int)boff[c], (int)(l * col_bytes), 0));
#pragma unroll
    for (int q = 0; q < NPW * B * R; ++q) {
      if (q % NH == wave) {  // wave-uniform
        const int v = q / (B * R), l = (q / R) % B, c = q % R;
        __builtin_amdgcn_raw_ptr_buffer_load_lds(rs, (__attribute__((address_space(3))) void*)&pbuf[pb][v][l][c][0],
                                                  16, (int)boffp[v][c], (int)(l * col_bytes), 0, 0);
      }
    }
  };

  auto finalize = [&](int sdone, bool conv, int64_t cols, double nrm2) {
    if (wg == 0 && tid == 0) {
      A.ctl[CTL_SWEEPS] = sdone;
      A.ctl[CTL_CONVERGED] = conv ? 1 : 0;
      A.ctl[CTL_DONE] = 1;
      A.ctl64[C64_COLS] = cols;
      A.fstat[0] = nrm2;
    }
  };

  int bi = (int)(A.blk_begin % nb);
  int sdone = (int)(A.blk_begin / nb);
  uint32_t seq = (uint32_t)(A.blk_begin + 1);

  auto step = [&](raw (&cur)[B][R], raw (&pf)[B][R], Coef<B>& ccur, Coef<B>& cpf, int64_t k) -> bool {
    const int j0 = bi * B;
    const int nbi = (bi + 1 == nb) ? 0 : bi + 1;
    const int pb = (int)(k & 1);
    // this block's columns (registers, and the polling wave's rows in LDS) have landed
    if (!pollw) asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    __syncthreads();
    // the polling wave's ring registers are otherwise unused: its rows land there
    if (pollw) {
#pragma unroll
      for (int l = 0; l < B; ++l)
#pragma unroll
        for (int c = 0; c < R; ++c) cur[l][c] = pbuf[pb][pw][l][c][lane];
    }
    auto& xl = cur;
#pragma unroll
    for (int l = 0; l < B; ++l)
#pragma unroll
      for (int c = 0; c < R; ++c)
        if (lim[c] < VEC) xl[l][c] = mask_chunk<S>(xl[l][c], lim[c]);
    float p[NV];
#pragma unroll
    for (int l = 0; l < B; ++l) {
      float acc = 0.f;
#pragma unroll
      for (int c = 0; c < R; ++c)
#pragma unroll
        for (int i = 0; i < VEC; ++i) acc = fmaf(S::get(xl[l][c], i), e[c][i], acc);
      p[l] = acc;
    }
    {
      float acc = 0.f;
#pragma unroll
      for (int c = 0; c < R; ++c)
#pragma unroll
        for (int i = 0; i < VEC; ++i) acc = fmaf(e[c][i], e[c][i], acc);
      p[B] = acc;
    }
    bool aborting = false;
    if (bi == 0 && wg == 0 && tid == 0 && load_cancel(A.cancel) != 0) {
      p[B] = __int_as_float(0x7fc00000);
      aborting = true;
    }
    const int par = (int)(seq & 1u);
#pragma unroll
    for (int l = 0; l < NV; ++l) {
      const float v = wave_sum(p[l]);
      if (lane == 0) red[par][wave][l] = v;
    }
    __syncthreads();
    uint64_t* slot_base = A.slots + (int64_t)par * NV * A.P;
    if (!pollw) {
      // next block: columns in flight during the exchange (the block after the
      // last one of the launch is a valid block, requested and never used)
      int pbi = bi + 1;
      if (pbi >= nb) pbi -= nb;
      load_block(pf, pbi, pb ^ 1);
      cpf.load(A.rdn, A.gram, pbi, lane);
    } else {
      if (pw == 0 && lane < NV) {
        float sacc = 0.f;
#pragma unroll
        for (int w = 0; w < NW; ++w) sacc += red[par][w][lane];
        publish(slot_base + (int64_t)lane * A.P + wg, seq, sacc);
      }
      if (A.poll_delay) {
        const uint64_t t0d = now_ticks();
        while (now_ticks() - t0d < A.poll_delay) __builtin_amdgcn_s_sleep(2);
      }
      // polling wave pw reads chunks pw*CPP .. of 64 workgroups: word
      // (l, c*64 + lane); lanes past the last workgroup read a valid word
      const int ncn = (A.P + WAVE - 1) / WAVE;
      uint64_t w[NV][CPP];
#pragma unroll
      for (int k = 0; k < CPP; ++k) {
        const int c = pw * CPP + k;
        const int idx = c * WAVE + lane;
        const bool live = c < ncn && idx < A.P;
#pragma unroll
        for (int l = 0; l < NV; ++l) w[l][k] = peek(slot_base + (int64_t)l * A.P + (live ? idx : 0));
      }
#pragma unroll
      for (int k = 0; k < CPP; ++k) {
        const int c = pw * CPP + k;
        const int idx = c * WAVE + lane;
        const bool live = c < ncn && idx < A.P;
#pragma unroll
        for (int l = 0; l < NV; ++l)
          if (!live) w[l][k] = (uint64_t)seq << 32;
      }
      uint64_t tstart = 0;
      bool timed_out = false;
      for (int spin = 0;; ++spin) {
        bool ready = true;
#pragma unroll
        for (int l = 0; l < NV; ++l)
#pragma unroll
          for (int k = 0; k < CPP; ++k) ready = ready && ((uint32_t)(w[l][k] >> 32) == seq);
        if (ready) break;
        if (spin == 0) tstart = now_ticks();
        else if (now_ticks() - tstart > A.timeout_ticks) {
          timed_out = true;
          break;
        }
        __builtin_amdgcn_s_sleep(1);
#pragma unroll
        for (int k = 0; k < CPP; ++k) {
          const int idx = (pw * CPP + k) * WAVE + lane;
#pragma unroll
          for (int l = 0; l < NV; ++l)
            if ((uint32_t)(w[l][k] >> 32) != seq) w[l][k] = peek(slot_base + (int64_t)l * A.P + idx);
        }
      }
      // fixed order: per lane over its chunks, across the lanes, then over
      // the polling waves
#pragma unroll
      for (int l = 0; l < NV; ++l) {
        double acc = 0.0;
#pragma unroll
        for (int k = 0; k < CPP; ++k) {
          const int c = pw * CPP + k;
          const int idx = c * WAVE + lane;
          acc += (c < ncn && idx < A.P) ? (double)__uint_as_float((uint32_t)w[l][k]) : 0.0;
        }
        const double tl = wave_sum(acc);
        if (lane == 0) tpart[pw][l] = tl;
      }
      if (timed_out && lane == 0) sflag = 1;
      int pbi = bi + 1;
      if (pbi >= nb) pbi -= nb;
      cpf.load(A.rdn, A.gram, pbi, lane);
    }
    __syncthreads();
    if (sflag) {
      if (tid == 0) store_flag(&A.ctl[CTL_ERR], ERR_TIMEOUT);
      return true;
    }
    double tot[NV];
#pragma unroll
    for (int l = 0; l < NV; ++l) {
      double acc = 0.0;
#pragma unroll
      for (int q = 0; q < NPW; ++q) acc += tpart[q][l];
      tot[l] = uniform_f64(acc);
    }

    const double nrm2 = tot[B];
    const double nrm = sqrt(nrm2);
    if (!(nrm2 <= DBL_MAX)) {
      if (wg == 0 && tid == 0) store_flag(&A.ctl[CTL_ERR], aborting ? ERR_ABORTED : ERR_NONFINITE);
      finalize(sdone, false, (int64_t)sdone * n + j0, nrm2);
      return true;
    }
    if (bi == 0) {
      if (wg == 0 && tid == 0) { A.hist[sdone] = nrm; A.fstat[1] = nrm; }
      bool stop = false, conv = false;
      if (A.stop != STOP_NONE && nrm2 == 0.0) stop = conv = true;
      else if (A.stop == STOP_REL_CHANGE && sdone >= 1 && (prev_norm - nrm) < A.tol * nrm) stop = conv = true;
      else if (A.stop == STOP_REL_RESID && nrm < A.tol * ynorm) stop = conv = true;
      if (!stop && sdone >= A.max_sweeps) stop = true;
      prev_norm = nrm;
      if (stop) { finalize(sdone, conv, (int64_t)sdone * n, nrm2); return true; }
    } else if (A.check_cols > 0 && A.stop == STOP_REL_RESID) {
      const int64_t cols = (int64_t)sdone * n + j0;
      if (cols % A.check_cols == 0 && (nrm2 == 0.0 || nrm < A.tol * ynorm)) {
        finalize(sdone, true, cols, nrm2);
        return true;
      }
    }
    double da[B];
    forward_substitute<B>(tot, ccur, da);
#pragma unroll
    for (int l = 0; l < B; ++l) {
      const float f = (float)da[l];
#pragma unroll
      for (int c = 0; c < R; ++c)
#pragma unroll
        for (int i = 0; i < VEC; ++i) e[c][i] = fmaf(-f, S::get(xl[l][c], i), e[c][i]);
    }
    if (tid < B) {
      const int64_t j = j0 + tid;
      if (j < n && (int)(j % A.P) == wg) {
        double d = 0.0;
#pragma unroll
        for (int l = 0; l < B; ++l) if (tid == l) d = da[l];
        (void)__hip_atomic_fetch_add(&A.a64[j], d, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
    }
    bi = nbi;
    if (bi == 0) ++sdone;
    ++seq;
    return false;
  };

  if (nblocks > 0) {
    if (!pollw) load_block(x0, bi, 0);
    c0.load(A.rdn, A.gram, bi, lane);
  }
  for (int64_t k = 0; k < nblocks;) {
    if (step(x0, x1, c0, c1, k)) break;
    if (++k >= nblocks) break;
    if (step(x1, x0, c1, c0, k)) break;
    ++k;
  }
  // no direct-to-LDS load may still be in flight when the workgroup ends
  asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
#pragma unroll
  for (int c = 0; c < R; ++c)
#pragma unroll
    for (int i = 0; i < VEC; ++i)
      if (i < lim[c]) A.e_out[rof[c] + i] = e[c][i];
}

// First row of a chunk that holds only rows below m, read in place of a
// chunk with no valid row (finite data, whose residual is held at zero).
// With m below one chunk there is none: every chunk is then masked.
__device__ inline int64_t full_chunk_row(int64_t m, int vec) { return m >= vec ? (m / vec - 1) * vec : 0; }

// Barrier that orders LDS only (an LDS wait and s_barrier): a barrier with
// memory fences would also wait for the column loads in flight.
__device__ inline void lds_barrier() {
  asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
  __builtin_amdgcn_s_barrier();
  asm volatile("" ::: "memory");
}

// The kernel's SolveArgs read again from the argument segment where they are
// used, for fields needed only off the per-block path (stop tests, history,
// control words): the pointer is opaque to the optimiser, so these loads are
// not hoisted and the values do not occupy scalar registers across the loop.
typedef const SolveArgs __attribute__((address_space(4)))* KArgs;
__device__ inline KArgs cold_args() {
  KArgs p = (KArgs)__builtin_amdgcn_kernarg_segment_ptr();
  asm volatile("" : "+s"(p));
  return p;
}

// --------------------------------------------------------------------------
// Grid kernel with wide blocks.
//
// One grid-wide reduction per block of B = 16 columns instead of 8: every
// wave loads its rows of the block, computes the partial sums, and the
// workgroup then exchanges them with the grid while no column load is in
// flight, so the exchange's loads and stores never queue behind column data
// (nor behind other CUs' column bursts in the memory fabric).  The next
// block's first PF columns are requested as soon as the exchange has
// completed, into registers of their own, and stream while the totals, the
// step and the axpy run; its other columns are requested after the axpy.
// On the 1M x 256 system the column stream of a 16-column block (256 KB per
// CU) plus one exchange takes less than two exchanges of 8-column blocks,
// each overlapped with the next block's loads in the same CU memory pipeline.
// The exchange is spread over the waves: value v of the block is polled and
// summed by wave v mod NW.  The block's B steps come from its step matrix
// M = (D + L)^{-1} (precomputed, FP64): da = M g with g the grid-summed dots,
// the same values as the forward substitution of k_sweep (only the rounding
// order differs), but 16 independent FP64 dot products, one per lane,
// instead of a serial chain run redundantly by every wave.  Stop logic is
// that of k_sweep.
//
// Method variants (V):
//  0  Algorithm 1.
//  1  Algorithm 2 (Section 7) with blocks of A.thr columns: every column of
//     such a block steps against the residual at the block's start.  The
//     kernel keeps a copy es of the residual taken where the current
//     thr-block began; a column whose thr-block began in an earlier
//     16-column block takes its dot against es, the others against e, and
//     the block's step matrix (k_block_inverse16 with thr) removes the steps
//     of this block that such a column must not see.
//  2  Column order: sweep s visits the columns A.order[s-1][0..n-1]; block
//     position p of the sweep is column A.order[s-1][p] (the step matrices of
//     the sweep's blocks are computed for that order before the sweep).
// Columns past n in the last block read the block's last valid column
// again (finite data; their step-matrix rows and columns are zero).
template <class S, int T, int R, int B, int V>
__global__ void __launch_bounds__(T) k_sweep_wide(SolveArgs A) {
  constexpr bool PAR = V == 1, ORD = V == 2;
  using raw = typename S::raw_t;
  constexpr int VEC = S::VEC;
  constexpr int NW = T / WAVE;
  constexpr int NV = B + 1;
  constexpr int MAXC = 4;                      // up to 256 workgroups
  constexpr int VPW = (NV + NW - 1) / NW;      // values summed by one wave, at most
  constexpr long long TIMED_OUT = 0x7ff8000000000001ll;  // a NaN no arithmetic here produces
  static_assert(B == 16, "the scattered wave sums and the step matrix rows are laid out for 16 columns");
  // next-block columns requested after the exchange (Algorithm 1 form; the
  // 1024-thread shape has no registers to spare)
  constexpr int PF = (V == 0 && T <= 512) ? 2 : 0;
  __shared__ float red[NW][NV];
  __shared__ double stot[NV];

  const int tid = threadIdx.x, lane = tid & (WAVE - 1);
  const int wave = __builtin_amdgcn_readfirstlane(tid / WAVE);
  const int wg = (int)blockIdx.x;
  const int64_t m = A.m, n = A.n;
  const int nb = (int)((n + B - 1) / B);
  if (A.ctl[CTL_NONFINITE] != 0 || A.ctl[CTL_DONE] != 0) return;

  const int64_t col_bytes = A.ldx * (int64_t)(16 / VEC);
  float e[R][VEC];
  int lim[R];
  uint32_t boff[R];
  // This workgroup owns rows [wg_row0, wg_end): rows_per_wg (a multiple of
  // VEC, at most T*R*VEC) per workgroup, so a grid can spread over every CU.
  const int64_t wg_row0 = (int64_t)wg * A.rows_per_wg;
  const int64_t wg_end = min(m, wg_row0 + (int64_t)A.rows_per_wg);
  // A chunk with no valid row is read at an offset past the block's buffer
  // range, which returns zero and moves no data, when the 32-bit offsets
  // leave room for it (a block spans at most 16 column strides); otherwise
  // (and under a column order, whose buffer range is all of X) it reads a
  // chunk of valid rows.  Its residual is held at zero either way.
  const bool oob = !ORD && 31 * col_bytes < 0xFFFFFFFFll;
#pragma unroll
  for (int c = 0; c < R; ++c) {
    const int64_t r0 = wg_row0 + (int64_t)VEC * (tid + T * c);
    const int64_t left = wg_end - r0;
    lim[c] = left <= 0 ? 0 : (left >= VEC ? VEC : (int)left);
    boff[c] = lim[c] > 0 ? (uint32_t)(r0 * (16 / VEC))
                         : (oob ? (uint32_t)(16 * col_bytes) : (uint32_t)(full_chunk_row(m, VEC) * (16 / VEC)));
#pragma unroll
    for (int i = 0; i < VEC; ++i) e[c][i] = (i < lim[c]) ? A.e0[r0 + i] : 0.f;
  }
  const bool ragged = wg_end - wg_row0 < (int64_t)(T * R * VEC);
  const bool tiny = m < VEC && !oob;  // no chunk of valid rows to read: every chunk is masked
  // Algorithm 2: the residual where the current thr-block began
  float es[PAR ? R : 1][PAR ? VEC : 1];
  if constexpr (PAR) {
#pragma unroll
    for (int c = 0; c < R; ++c)
#pragma unroll
      for (int i = 0; i < VEC; ++i) es[c][i] = e[c][i];
  }
  const int64_t thr = PAR ? (int64_t)A.thr : 1;
  bool straddle[R];
#pragma unroll
  for (int c = 0; c < R; ++c) straddle[c] = __ballot(lim[c] < VEC && (lim[c] > 0 || tiny)) != 0;

  double prev_norm = A.fstat[1];
  const double ynorm = sqrt(*A.ynorm2);
  const int64_t nblocks = A.blk_end - A.blk_begin;
  int bi = (int)(A.blk_begin % nb);
  int sdone = (int)(A.blk_begin / nb);
  uint32_t seq = (uint32_t)(A.blk_begin + 1);
  const bool col_checks = A.check_cols > 0 && A.stop == STOP_REL_RESID;

  auto finalize = [&](int sd, bool conv, int64_t cols, double nrm2) {
    if (wg == 0 && tid == 0) {
      const KArgs K = cold_args();
      K->ctl[CTL_SWEEPS] = sd;
      K->ctl[CTL_CONVERGED] = conv ? 1 : 0;
      K->ctl[CTL_DONE] = 1;
      K->ctl64[C64_COLS] = cols;
      K->fstat[0] = nrm2;
    }
  };

  // the first PF columns of block b into xn (the same unconditional,
  // range-checked loads as the block's other columns)
  raw xn[PF > 0 ? PF : 1][R];
  auto prefetch = [&](int b) {
    b = __builtin_amdgcn_readfirstlane(b);
    const int jb = b * B;
    const int nv = (n - jb) < B ? (int)(n - jb) : B;
    char* base = const_cast<char*>(reinterpret_cast<const char*>(A.X)) + (int64_t)jb * col_bytes;
    const int64_t span = (int64_t)(nv - 1) * col_bytes + A.ldx * (int64_t)(16 / VEC);
    const uint32_t nrec = span > 0xFFFFFFFFll ? 0xFFFFFFFFu : (uint32_t)span;
    const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(base, 0, (int)nrec, 0x00020000);
#pragma unroll
    for (int l = 0; l < (PF > 0 ? PF : 1); ++l) {
      const int lc = l < nv ? l : nv - 1;
      const int coff = (int)((int64_t)lc * col_bytes);
#pragma unroll
      for (int c = 0; c < R; ++c)
        xn[l][c] = __builtin_bit_cast(raw, __builtin_amdgcn_raw_buffer_load_b128(rs, (int)boff[c], coff, 0));
    }
  };
  if constexpr (PF > 0) {
    if (nblocks > 0) prefetch(bi);
  }

  for (int64_t k = 0; k < nblocks; ++k) {
    // (uniform; said explicitly so the column resource stays in scalar
    // registers instead of a per-load loop over distinct values)
    bi = __builtin_amdgcn_readfirstlane(bi);
    const int j0 = bi * B;
    const int nbi = (bi + 1 == nb) ? 0 : bi + 1;  // (the block after the launch's last: requested, never used)
    // a cancel request is looked at by one lane of workgroup 0 at a sweep's
    // first block, read here so that its trip to host memory overlaps the
    // column stream
    int32_t cancel_req = 0;
    if (bi == 0 && wg == 0 && tid == B) cancel_req = load_cancel(cold_args()->cancel);
    // (its value is hidden from the optimiser until it is used below, so the
    // test is not hoisted here, where it would wait for the load at once)
    // row (lane mod B) of the block's step matrix M: da = M g
    double mr[B];
    {
      const double2* src = reinterpret_cast<const double2*>(A.minv + ((int64_t)bi * B + (lane & (B - 1))) * B);
#pragma unroll
      for (int t = 0; t < B / 2; ++t) {
        const double2 v = src[t];
        mr[2 * t] = v.x;
        mr[2 * t + 1] = v.y;
      }
    }
    // the block's columns; a column past n reads the last valid one again
    const int nvalid = (n - j0) < B ? (int)(n - j0) : B;
    raw x[B][R];
    const int32_t* ordr = nullptr;
    if constexpr (ORD) {
      // (the stop test of the last sweep runs on one more block: its loads
      // reuse the last sweep's order)
      const int64_t srow = sdone < A.max_sweeps ? sdone : (A.max_sweeps > 0 ? A.max_sweeps - 1 : 0);
      ordr = A.order + srow * n;
    }
    {
      char* base = const_cast<char*>(reinterpret_cast<const char*>(A.X));
      uint32_t nrec;
      if constexpr (ORD) {
        const int64_t span = n * col_bytes;  // (below 4 GiB: checked by the host)
        nrec = (uint32_t)span;
      } else {
        base += (int64_t)j0 * col_bytes;
        const int64_t span = (int64_t)(nvalid - 1) * col_bytes + A.ldx * (int64_t)(16 / VEC);
        nrec = span > 0xFFFFFFFFll ? 0xFFFFFFFFu : (uint32_t)span;
      }
      const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(base, 0, (int)nrec, 0x00020000);
#pragma unroll
      for (int l = PF; l < B; ++l) {
        const int lc = l < nvalid ? l : nvalid - 1;
        int coff;
        if constexpr (ORD) coff = __builtin_amdgcn_readfirstlane((int)((int64_t)ordr[j0 + lc] * col_bytes));
        else coff = (int)((int64_t)lc * col_bytes);
#pragma unroll
        for (int c = 0; c < R; ++c)
          x[l][c] = __builtin_bit_cast(raw, __builtin_amdgcn_raw_buffer_load_b128(rs, (int)boff[c], coff, 0));
      }
    }
    if constexpr (PF > 0) {
      // (after the other columns are requested, so their loads are not held
      // back by a wait for these)
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int l = 0; l < PF; ++l)
#pragma unroll
        for (int c = 0; c < R; ++c) x[l][c] = xn[l][c];
    }
#pragma unroll
    for (int c = 0; c < R; ++c)
      if (straddle[c]) {  // wave-uniform
#pragma unroll
        for (int l = 0; l < B; ++l)
          if (lim[c] < VEC && (lim[c] > 0 || tiny)) x[l][c] = mask_chunk<S>(x[l][c], lim[c]);
      }
    // partial sums of this wave's rows: the B dots (summed over the wave
    // with one scattered reduction) and ||e||^2
    {
      float p[B];
#pragma unroll
      for (int l = 0; l < B; ++l) {
        float acc = 0.f;
        // Algorithm 2: a column whose thr-block began before this block
        // takes its dot against the residual saved at that block's start
        const bool cont = PAR && (j0 + l) / thr * thr < j0;
        if (cont) {
#pragma unroll
          for (int c = 0; c < R; ++c)
#pragma unroll
            for (int i = 0; i < VEC; ++i) acc = fmaf(S::get(x[l][c], i), es[PAR ? c : 0][PAR ? i : 0], acc);
        } else {
#pragma unroll
          for (int c = 0; c < R; ++c)
#pragma unroll
            for (int i = 0; i < VEC; ++i) acc = fmaf(S::get(x[l][c], i), e[c][i], acc);
        }
        p[l] = acc;
      }
      float pn = 0.f;
#pragma unroll
      for (int c = 0; c < R; ++c)
#pragma unroll
        for (int i = 0; i < VEC; ++i) pn = fmaf(e[c][i], e[c][i], pn);
      const float t = wave_sum16_scatter(p);
      if ((lane & 3) == 0) red[wave][lane >> 2] = t;
      const float tn = wave_sum(pn);
      if (lane == 0) red[wave][B] = tn;
    }
    lds_barrier();
    asm volatile("" : "+v"(cancel_req));
    bool aborting = false;
    if (A.P == 1) {
      if constexpr (PF > 0) prefetch(nbi);
      // one workgroup (a system of at most T*R*VEC rows): its sums are the
      // totals, no exchange; a cancel request rides the norm as a NaN
      if (tid < NV) {
        double acc = 0.0;
#pragma unroll
        for (int w = 0; w < NW; ++w) acc += (double)red[w][tid];
        if (tid == B && bi == 0 && cancel_req != 0)
          acc = __longlong_as_double(0x7ff8000000000000ll);
        stot[tid] = acc;
      }
    } else {
      // exchange with the grid: wave 0 publishes the workgroup's sums; value v
      // is polled and summed by wave v mod NW
      const uint64_t* slot_base = A.slots + (int64_t)(seq & 1u) * NV * A.P;
      bool injected = false;
      if (wave == 0 && lane < NV) {
        float sacc = 0.f;
  #pragma unroll
        for (int w = 0; w < NW; ++w) sacc += red[w][lane];
        // a cancel request rides the norm of a sweep's first block as a NaN
        if (lane == B && bi == 0 && wg == 0 && cancel_req != 0) {
          sacc = __int_as_float(0x7fc00000);
          injected = true;
        }
        publish(const_cast<uint64_t*>(slot_base) + (int64_t)lane * A.P + wg, seq, sacc);
      }
      aborting = __ballot(injected) != 0;  // (meaningful in wave 0 of workgroup 0)
      if (A.poll_delay) {
        const uint64_t t0d = now_ticks();
        while (now_ticks() - t0d < A.poll_delay) __builtin_amdgcn_s_sleep(2);
      }
      const int ncn = (A.P + WAVE - 1) / WAVE;
      uint64_t w[VPW][MAXC];
  #pragma unroll
      for (int q = 0; q < VPW; ++q) {
        const int v = wave + NW * q;
        const int vv = v < NV ? v : NV - 1;  // (rounds past the last value reread a valid word)
  #pragma unroll
        for (int c = 0; c < MAXC; ++c) {
          const int idx = c * WAVE + lane;
          const bool live = c < ncn && idx < A.P;
          w[q][c] = live ? peek(slot_base + (int64_t)vv * A.P + idx) : ((uint64_t)seq << 32);
        }
      }
      // a wave-uniform spin: every exit follows a completed check of the
      // words, so nothing of the poll is still in flight after the loop
      auto all_ready = [&]() {
        bool ready = true;
  #pragma unroll
        for (int q = 0; q < VPW; ++q)
  #pragma unroll
          for (int c = 0; c < MAXC; ++c) ready = ready && ((uint32_t)(w[q][c] >> 32) == seq);
        return __ballot(!ready) == 0;
      };
      bool timed_out = false;
      if (!all_ready()) {
        const uint64_t tstart = now_ticks();
        do {
          if (now_ticks() - tstart > A.timeout_ticks) {
            timed_out = true;
            break;
          }
          __builtin_amdgcn_s_sleep(1);
  #pragma unroll
          for (int q = 0; q < VPW; ++q) {
            const int v = wave + NW * q;
            const int vv = v < NV ? v : NV - 1;
  #pragma unroll
            for (int c = 0; c < MAXC; ++c) {
              const int idx = c * WAVE + lane;
              if ((uint32_t)(w[q][c] >> 32) != seq) w[q][c] = peek(slot_base + (int64_t)vv * A.P + idx);
            }
          }
        } while (!all_ready());
      }
      const bool any_timeout = __ballot(timed_out) != 0;
      if constexpr (PF > 0) {
        // the exchange is done: the next block's first columns stream while
        // the totals, the step and the axpy run (requested earlier, during
        // the exchange, they would slow every other CU's polls)
        __builtin_amdgcn_sched_barrier(0);
        prefetch(nbi);
        __builtin_amdgcn_sched_barrier(0);
      }
      // fixed order: per lane over its chunks, then across the lanes
  #pragma unroll
      for (int q = 0; q < VPW; ++q) {
        const int v = wave + NW * q;
        double acc = 0.0;
  #pragma unroll
        for (int c = 0; c < MAXC; ++c) {
          const int idx = c * WAVE + lane;
          acc += (c < ncn && idx < A.P) ? (double)__uint_as_float((uint32_t)w[q][c]) : 0.0;
        }
        const double tv = wave_sum(acc);
        if (v < NV && lane == 0) stot[v] = any_timeout ? __longlong_as_double(TIMED_OUT) : tv;
      }
    }
    lds_barrier();
    // some wave's poll timed out
    const bool tmo = __ballot(lane < NV && __double_as_longlong(stot[lane < NV ? lane : 0]) == TIMED_OUT) != 0;
    if (tmo) {
      if (tid == 0) store_flag(&cold_args()->ctl[CTL_ERR], ERR_TIMEOUT);
      break;
    }
    const double nrm2 = uniform_f64(stot[B]);
    const double nrm = sqrt(nrm2);
    if (!(nrm2 <= DBL_MAX)) {
      if (wg == 0 && tid == 0) {
        const bool ab = aborting || (A.P == 1 && load_cancel(cold_args()->cancel) != 0);
        store_flag(&cold_args()->ctl[CTL_ERR], ab ? ERR_ABORTED : ERR_NONFINITE);
      }
      finalize(sdone, false, (int64_t)sdone * n + j0, nrm2);
      break;
    }
    if (bi == 0) {
      const KArgs K = cold_args();
      if (wg == 0 && tid == 0) { K->hist[sdone] = nrm; K->fstat[1] = nrm; }
      bool stop = false, conv = false;
      if (K->stop != STOP_NONE && nrm2 == 0.0) stop = conv = true;
      else if (K->stop == STOP_REL_CHANGE && sdone >= 1 && (prev_norm - nrm) < K->tol * nrm) stop = conv = true;
      else if (K->stop == STOP_REL_RESID && nrm < K->tol * ynorm) stop = conv = true;
      if (!stop && sdone >= K->max_sweeps) stop = true;
      prev_norm = nrm;
      if (stop) { finalize(sdone, conv, (int64_t)sdone * n, nrm2); break; }
    } else if (col_checks) {
      const KArgs K = cold_args();
      const int64_t cols = (int64_t)sdone * n + j0;
      if (cols % K->check_cols == 0 && (nrm2 == 0.0 || nrm < K->tol * ynorm)) {
        finalize(sdone, true, cols, nrm2);
        break;
      }
    }
    // da = M g: lane l of every wave computes da_l (fixed order), the axpy
    // takes the B steps as scalars
    double dl = 0.0;
#pragma unroll
    for (int q = 0; q < B; ++q) dl = fma(mr[q], stot[q], dl);
    const int fl = __float_as_int((float)dl);
#pragma unroll
    for (int l = 0; l < B; ++l) {
      if constexpr (PAR) {
        // a thr-block begins at this column: keep the residual it starts from
        if ((j0 + l) % thr == 0 && j0 + l < n) {
#pragma unroll
          for (int c = 0; c < R; ++c)
#pragma unroll
            for (int i = 0; i < VEC; ++i) es[c][i] = e[c][i];
        }
      }
      const float f = __int_as_float(__builtin_amdgcn_readlane(fl, l));
#pragma unroll
      for (int c = 0; c < R; ++c)
#pragma unroll
        for (int i = 0; i < VEC; ++i) e[c][i] = fmaf(-f, S::get(x[l][c], i), e[c][i]);
    }
    if (ragged) {
#pragma unroll
      for (int c = 0; c < R; ++c)
#pragma unroll
        for (int i = 0; i < VEC; ++i) e[c][i] = (i < lim[c]) ? e[c][i] : 0.f;
    }
    if (tid < B) {  // lane tid of wave 0 holds da_tid
      const int64_t p = j0 + tid;
      if (p < n && (int)(p % A.P) == wg) {
        const int64_t j = ORD ? (int64_t)ordr[p] : p;
        (void)__hip_atomic_fetch_add(&A.a64[j], dl, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
    }
    bi = nbi;
    if (bi == 0) ++sdone;
    ++seq;
  }
  // no prefetched column may still be in flight when the workgroup ends
  if constexpr (PF > 0) asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
#pragma unroll
  for (int c = 0; c < R; ++c) {
    const int64_t r0 = wg_row0 + (int64_t)VEC * (tid + T * c);
#pragma unroll
    for (int i = 0; i < VEC; ++i)
      if (i < lim[c]) A.e_out[r0 + i] = e[c][i];
  }
}

// --------------------------------------------------------------------------
// Batched kernel: a persistent grid of workgroups pulls work items from an
// atomic queue.  An item is either one system solved by the whole workgroup
// (rows over T threads, reductions through LDS) or up to NW systems solved
// by one wave each (rows over 64 lanes, reductions by DPP only, no barrier).
// --------------------------------------------------------------------------
// Workgroup shapes (both 8192 rows): four waves of eight FP32 chunks per
// thread (2048 rows per wave team), or eight waves of four (1024 rows per
// wave team, twice the column chains resident per CU in the same registers).
template <int W> struct BShape {
  static constexpr int T = W ? 512 : 256;  // threads per workgroup
  static constexpr int R = W ? 4 : 8;      // chunks per thread
};

template <int TT, int R, int B, int NWG>
__device__ inline void team_solve(const BatchArgs& A, int sidx, int ttid, float (&red)[2][NWG][B + 1]) {
  using S = F32;
  using raw = S::raw_t;
  constexpr int VEC = S::VEC;
  constexpr int NW = TT / WAVE;
  constexpr int NV = B + 1;
  const int lane = ttid & (WAVE - 1), wave = ttid / WAVE;
  const SysDesc sd = A.sys[sidx];
  const int64_t m = sd.m, n = sd.n, nb = (n + B - 1) / B;
  const float* X = A.Xpool + sd.x_off;
  const double* rdn = A.rdn + sd.g_off;
  const double* gram = A.gram + sd.g_off / B * Coef<B>::NG;
  double* hist = A.hist + sd.h_off;

  // Columns are read through a buffer resource based at the block's first
  // column (built from values equal across the team, made explicitly
  // uniform so the resource stays in scalar registers).  Every load is
  // issued unconditionally, so the compiler can wait for the current block
  // with an exact count while the next one is in flight: a chunk with no
  // valid row is read past the block's range (zero, no data moved) when the
  // 32-bit offsets leave room, else at row 0; columns past n lie past the
  // range too; partly or wholly invalid chunks are masked before use.
  const uint32_t col_bytes = (uint32_t)__builtin_amdgcn_readfirstlane((int)(sd.ldx * 4));
  const bool oob = (int64_t)(2 * B) * sd.ldx * 4 < 0xFFFFFFFFll;
  float e[R][VEC];
  int lim[R];
  uint32_t boff[R];
#pragma unroll
  for (int c = 0; c < R; ++c) {
    const int64_t rof = (int64_t)VEC * (ttid + TT * c);
    const int64_t left = m - rof;
    lim[c] = left <= 0 ? 0 : (left >= VEC ? VEC : (int)left);
    boff[c] = lim[c] > 0 ? (uint32_t)(rof * 4) : (oob ? (uint32_t)B * col_bytes : 0u);
#pragma unroll
    for (int i = 0; i < VEC; ++i) e[c][i] = (i < lim[c]) ? A.e0pool[sd.y_off + rof + i] : 0.f;
  }
  const double ynorm = sqrt(A.ynorm2[sidx]);
  double prev_norm = 0.0;
  const int64_t ke = (int64_t)A.max_sweeps * nb + 1;
  raw xa[B][R], xb[B][R];
  Coef<B> ca, cb;

  auto block_rsrc = [&](int64_t k) {
    const int64_t bi = k % nb, j0 = bi * B;
    const int nvalid = (n - j0) < B ? (int)(n - j0) : B;
    const int64_t span = (int64_t)nvalid * sd.ldx * 4;
    const uint64_t base = (uint64_t)(X + j0 * sd.ldx);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)base);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(base >> 32));
    const uint32_t nrec = (uint32_t)__builtin_amdgcn_readfirstlane(
        (int)(span > 0xFFFFFFFFll ? 0xFFFFFFFFu : (uint32_t)span));
    return __builtin_amdgcn_make_buffer_rsrc(reinterpret_cast<void*>(((uint64_t)hi << 32) | lo), 0, (int)nrec,
                                             0x00020000);
  };
  auto load_chunk_at = [&](const __amdgpu_buffer_rsrc_t& rs, int l, int c) {
    return __builtin_bit_cast(raw, __builtin_amdgcn_raw_buffer_load_b128(rs, (int)boff[c], (int)(l * col_bytes), 0));
  };
  auto load_block = [&](raw (&x)[B][R], Coef<B>& cf, int64_t k) {
    const __amdgpu_buffer_rsrc_t rs = block_rsrc(k);
#pragma unroll
    for (int l = 0; l < B; ++l)
#pragma unroll
      for (int c = 0; c < R; ++c) x[l][c] = load_chunk_at(rs, l, c);
    cf.load(rdn, gram, k % nb, lane);
  };

  auto step = [&](raw (&cur)[B][R], raw (&nxt)[B][R], Coef<B>& ccur, Coef<B>& cnxt, int64_t k) -> bool {
    const int64_t bi = k % nb, j0 = bi * B;
    const int sdone = (int)(k / nb);
    // the next block (past the last step: a harmless reread, issued so every
    // path loads alike): its coefficients now, its columns spread over this
    // block's dot products, one chunk load between the arithmetic of two
    // chunks, so the memory pipeline works while the ALUs do
    cnxt.load(rdn, gram, (k + 1) % nb, lane);
    const __amdgpu_buffer_rsrc_t rsn = block_rsrc(k + 1);
    float p[NV];
#pragma unroll
    for (int l = 0; l < B; ++l) {
      float acc = 0.f;
#pragma unroll
      for (int c = 0; c < R; ++c) {
        if (lim[c] < VEC) cur[l][c] = mask_chunk<S>(cur[l][c], lim[c]);
#pragma unroll
        for (int i = 0; i < VEC; ++i) acc = fmaf(S::get(cur[l][c], i), e[c][i], acc);
        nxt[l][c] = load_chunk_at(rsn, l, c);
        __builtin_amdgcn_sched_barrier(0);
      }
      p[l] = acc;
    }
    {
      float acc = 0.f;
#pragma unroll
      for (int c = 0; c < R; ++c)
#pragma unroll
        for (int i = 0; i < VEC; ++i) acc = fmaf(e[c][i], e[c][i], acc);
      p[B] = acc;
    }
    double tot[NV];
    if constexpr (NW == 1) {
#pragma unroll
      for (int l = 0; l < NV; ++l) tot[l] = uniform_f64((double)wave_sum(p[l]));
    } else {
      const int par = (int)(k & 1);
#pragma unroll
      for (int l = 0; l < NV; ++l) {
        const float v = wave_sum(p[l]);
        if (lane == 0) red[par][wave][l] = v;
      }
      __syncthreads();
#pragma unroll
      for (int l = 0; l < NV; ++l) {
        double s = 0.0;
#pragma unroll
        for (int w = 0; w < NW; ++w) s += (double)red[par][w][l];
        tot[l] = uniform_f64(s);
      }
    }
    const double nrm2 = tot[B], nrm = sqrt(nrm2);
    if (bi == 0) {
      if (ttid == 0) hist[sdone] = nrm;
      bool stop = false, conv = false;
      if (!(nrm2 <= DBL_MAX)) stop = true;
      else if (A.stop != STOP_NONE && nrm2 == 0.0) stop = conv = true;
      else if (A.stop == STOP_REL_CHANGE && sdone >= 1 && (prev_norm - nrm) < sd.tol * nrm) stop = conv = true;
      else if (A.stop == STOP_REL_RESID && nrm < sd.tol * ynorm) stop = conv = true;
      if (!stop && sdone >= A.max_sweeps) stop = true;
      prev_norm = nrm;
      if (stop) {
        if (ttid == 0) { A.sweeps[sidx] = sdone; A.converged[sidx] = conv ? 1 : 0; }
        return true;
      }
    }
    double da[B];
    forward_substitute<B>(tot, ccur, da);
#pragma unroll
    for (int l = 0; l < B; ++l) {
      const float f = (float)da[l];
#pragma unroll
      for (int c = 0; c < R; ++c)
#pragma unroll
        for (int i = 0; i < VEC; ++i) e[c][i] = fmaf(-f, S::get(cur[l][c], i), e[c][i]);
    }
    if (ttid < B) {
      double d = 0.0;
#pragma unroll
      for (int l = 0; l < B; ++l) if (ttid == l) d = da[l];
      if (j0 + ttid < n) {
        // only this lane touches a_j of this system; no return value is waited for
        (void)__hip_atomic_fetch_add(A.a64pool + sd.a_off + j0 + ttid, d, __ATOMIC_RELAXED,
                                     __HIP_MEMORY_SCOPE_AGENT);
      }
    }
    return false;
  };

  load_block(xa, ca, 0);
  for (int64_t k = 0; k < ke;) {
    if (step(xa, xb, ca, cb, k)) break;
    if (++k >= ke) break;
    if (step(xb, xa, cb, ca, k)) break;
    ++k;
  }
}

template <int B, int W>
__global__ void __launch_bounds__(BShape<W>::T) k_batched(BatchArgs A) {
  constexpr int BT = BShape<W>::T, BR = BShape<W>::R;
  constexpr int NW = BT / WAVE;
  __shared__ float red[2][NW][B + 1];
  __shared__ int s_item;
  const int tid = threadIdx.x, wave = tid / WAVE;
  for (;;) {
    // the next item is taken only once every wave is done with the last one:
    // taken as soon as wave 0 was done, it waited, reserved, for the
    // workgroup's slowest wave while other workgroups ran out of work
    __syncthreads();
    if (tid == 0) s_item = atomicAdd(A.queue, 1);
    __syncthreads();
    const int it = s_item;
    if (it >= A.nitems) break;
    const WorkItem w = A.items[it];
    if (w.mode == 0) {
      team_solve<BT, BR, B, NW>(A, w.sys[0], tid, red);
    } else if (wave < w.count) {
      team_solve<WAVE, BR, B, NW>(A, w.sys[wave], tid & (WAVE - 1), red);
    }
  }
}

// --------------------------------------------------------------------------
// Variant registry
// --------------------------------------------------------------------------
#define HPSCD_SWEEP_VARIANTS(X_)                                                              \
  X_(F32, 1024, 1, 1, true, 2) X_(F32, 1024, 1, 2, true, 2) X_(F32, 1024, 1, 4, true, 2)      \
  X_(F32, 1024, 1, 4, true, 3) X_(F32, 512, 2, 4, true, 3) X_(F32, 512, 2, 8, true, 3)        \
  X_(F32, 512, 2, 2, true, 2) X_(F32, 512, 2, 4, true, 2) X_(F32, 512, 2, 8, true, 2)         \
  X_(F32, 256, 4, 8, true, 2) X_(F32, 256, 4, 8, true, 3) X_(F32, 256, 4, 4, true, 3)         \
  X_(BF16, 512, 1, 4, true, 2) X_(BF16, 512, 1, 8, true, 2) X_(BF16, 1024, 1, 4, true, 2)     \
  X_(BF16, 512, 1, 8, true, 3) X_(BF16, 256, 2, 8, true, 3)                                    \
  X_(F32, 256, 1, 1, true, 2) X_(F32, 256, 1, 2, true, 2) X_(F32, 256, 1, 4, true, 2)         \
  X_(F32, 256, 1, 8, true, 2)                                                                  \
  X_(F32, 256, 2, 1, false, 2) X_(F32, 256, 2, 2, false, 2) X_(F32, 256, 2, 4, false, 2)      \
  X_(F32, 256, 2, 8, false, 2)                                                                 \
  X_(F32, 256, 4, 1, false, 2) X_(F32, 256, 4, 2, false, 2) X_(F32, 256, 4, 4, false, 2)      \
  X_(F32, 256, 4, 8, false, 2)                                                                 \
  X_(BF16, 1024, 1, 1, true, 2) X_(BF16, 1024, 1, 8, true, 2)                                 \
  X_(BF16, 256, 1, 1, false, 2) X_(BF16, 256, 1, 4, false, 2) X_(BF16, 256, 1, 8, false, 2)   \
  X_(BF16, 256, 2, 1, false, 2) X_(BF16, 256, 2, 4, false, 2) X_(BF16, 256, 2, 8, false, 2)   \
  X_(F32, 256, 2, 8, false, 3) X_(F32, 256, 2, 8, false, 4) X_(F32, 256, 2, 4, false, 4)       \
  X_(BF16, 256, 1, 8, false, 3) X_(BF16, 256, 1, 8, false, 4) X_(BF16, 256, 1, 4, false, 4)

#define HPSCD_IS_BF16_F32 false
#define HPSCD_IS_BF16_BF16 true

struct Variant {
  int T, R, B;
  bool bf16, grid;
  int D;           // 2, 3, 4: prefetch ring (k_sweep); 5: polling waves (k_sweep_px); 8: wide blocks
  const void* fn;
  int threads;     // launch width
  int V;           // method variant of the wide-block kernel (0: Algorithm 1)
};

#define HPSCD_ENTRY(S, T, R, B, G, D) \
  {T, R, B, HPSCD_IS_BF16_##S, G, D, reinterpret_cast<const void*>(&k_sweep<S, T, R, B, G, D>), T, 0},
#define HPSCD_PX_VARIANTS(X_) \
  X_(F32, 512, 2, 8, 2) X_(F32, 512, 2, 4, 1) X_(F32, 256, 4, 4, 1) X_(F32, 256, 4, 8, 2) X_(BF16, 512, 1, 8, 2)
#define HPSCD_XENTRY(S, T, R, B, NPW) \
  {T, R, B, HPSCD_IS_BF16_##S, true, 5, reinterpret_cast<const void*>(&k_sweep_px<S, T, R, B, NPW>), T, 0},
// kind 8: wide blocks (the next block's first columns requested after each exchange)
#define HPSCD_WIDE_VARIANTS(X_) X_(F32, 512, 2, 16) X_(BF16, 512, 1, 16) X_(F32, 256, 4, 16) X_(F32, 1024, 1, 16) \
  X_(F32, 512, 1, 16) X_(F32, 256, 1, 16)
#define HPSCD_WBENTRY(S, T, R, B) \
  {T, R, B, HPSCD_IS_BF16_##S, true, 8, reinterpret_cast<const void*>(&k_sweep_wide<S, T, R, B, 0>), T, 0},
#define HPSCD_WB1ENTRY(S, T, R, B) \
  {T, R, B, HPSCD_IS_BF16_##S, false, 8, reinterpret_cast<const void*>(&k_sweep_wide<S, T, R, B, 0>), T, 0},
// the method variants (Algorithm 2, column order) of the FP32 shapes
#define HPSCD_WIDE_F32_VARIANTS(X_) X_(512, 2, 1) X_(256, 4, 1) X_(1024, 1, 1) X_(512, 1, 1) X_(256, 1, 1) \
  X_(512, 2, 2) X_(256, 4, 2) X_(1024, 1, 2) X_(512, 1, 2) X_(256, 1, 2)
#define HPSCD_WVENTRY(T, R, V) \
  {T, R, 16, false, true, 8, reinterpret_cast<const void*>(&k_sweep_wide<F32, T, R, 16, V>), T, V}, \
  {T, R, 16, false, false, 8, reinterpret_cast<const void*>(&k_sweep_wide<F32, T, R, 16, V>), T, V},
static const Variant kVariants[] = {HPSCD_SWEEP_VARIANTS(HPSCD_ENTRY) HPSCD_PX_VARIANTS(HPSCD_XENTRY)
                                        HPSCD_WIDE_VARIANTS(HPSCD_WBENTRY) HPSCD_WIDE_VARIANTS(HPSCD_WB1ENTRY)
                                            HPSCD_WIDE_F32_VARIANTS(HPSCD_WVENTRY)};

// The deepest prefetch ring built for the shape (D = 0: any).
static const Variant* find_variant(int T, int R, int B, bool bf16, bool grid, int D = 0, int V = 0) {
  const Variant* best = nullptr;
  for (const Variant& v : kVariants)
    if (v.T == T && v.R == R && v.B == B && v.bf16 == bf16 && v.grid == grid && (D == 0 || v.D == D) && v.V == V)
      if (!best || v.D > best->D) best = &v;
  return best;
}

bool sweep_variant_exists(int T, int R, int B, bool bf16, bool grid, int D, int V) {
  return find_variant(T, R, B, bf16, grid, D, V) != nullptr;
}

int sweep_max_workgroups(int T, int R, int B, bool bf16, bool grid, int D, int V) {
  const Variant* v = find_variant(T, R, B, bf16, grid, D, V);
  if (!v) return 0;
  return v->D >= 5 ? 256 : 512;
}

// Resident workgroups per CU of a compiled kernel at its launch width: a
// property of the code object, asked of the runtime once per variant (every
// planned solve needs it; the query is not free).  0 in a slot = not asked yet.
static int occupancy_once(std::atomic<int>& slot, const void* fn, int threads) {
  const int c = slot.load(std::memory_order_relaxed);
  if (c > 0) return c - 1;
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, fn, threads, 0) != hipSuccess) return 0;
  slot.store(nb + 1, std::memory_order_relaxed);
  return nb;
}

int sweep_max_blocks_per_cu(int T, int R, int B, bool bf16, bool grid, int D, int V) {
  static std::atomic<int> occ[sizeof(kVariants) / sizeof(kVariants[0])];
  const Variant* v = find_variant(T, R, B, bf16, grid, D, V);
  if (!v) return 0;
  return occupancy_once(occ[v - kVariants], v->fn, v->threads);
}

hipError_t launch_sweep(int T, int R, int B, bool bf16, bool grid, int D, const SolveArgs& a, hipStream_t s,
                        bool cooperative, int V) {
  const Variant* v = find_variant(T, R, B, bf16, grid, D, V);
  if (!v) return hipErrorInvalidValue;
  SolveArgs args = a;
  void* kargs[] = {&args};
  const dim3 g(grid ? (unsigned)a.P : 1u), b((unsigned)v->threads);
  if (cooperative) return hipLaunchCooperativeKernel(v->fn, g, b, kargs, 0, s);
  return hipLaunchKernel(v->fn, g, b, kargs, 0, s);
}

#define HPSCD_BATCHED_VARIANTS(X_) X_(1, 0) X_(2, 0) X_(4, 0) X_(1, 1) X_(2, 1) X_(4, 1)
struct BVariant { int code; const void* fn; int threads, R; };
#define HPSCD_BENTRY(B, W) \
  {B + (W ? kBatchWide : 0), reinterpret_cast<const void*>(&k_batched<B, W>), BShape<W>::T, BShape<W>::R},
static const BVariant kBVariants[] = {HPSCD_BATCHED_VARIANTS(HPSCD_BENTRY)};

static const BVariant* find_bvariant(int code) {
  for (const BVariant& v : kBVariants) if (v.code == code) return &v;
  return nullptr;
}
bool batched_variant_exists(int code) { return find_bvariant(code) != nullptr; }
int batched_threads(int code) {
  const BVariant* v = find_bvariant(code);
  return v ? v->threads : 0;
}
int batched_rows_per_wave(int code) {
  const BVariant* v = find_bvariant(code);
  return v ? WAVE * v->R * F32::VEC : 0;
}
int batched_rows_per_wg(int code) {
  const BVariant* v = find_bvariant(code);
  return v ? v->threads * v->R * F32::VEC : 0;
}
int batched_max_blocks_per_cu(int code) {
  static std::atomic<int> occ[sizeof(kBVariants) / sizeof(kBVariants[0])];
  const BVariant* v = find_bvariant(code);
  if (!v) return 0;
  return occupancy_once(occ[v - kBVariants], v->fn, v->threads);
}
hipError_t launch_batched(int code, const BatchArgs& a, int grid, hipStream_t s) {
  const BVariant* v = find_bvariant(code);
  if (!v) return hipErrorInvalidValue;
  BatchArgs args = a;
  void* kargs[] = {&args};
  return hipLaunchKernel(v->fn, dim3((unsigned)grid), dim3((unsigned)v->threads), kargs, 0, s);
}

}  // namespace hpscd
