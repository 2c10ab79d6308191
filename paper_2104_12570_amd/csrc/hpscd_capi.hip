// C ABI of libhpscd: argument validation, workspace, launch planning.
#include "hpscd.h"
#include "hpscd_device.hpp"
#include "hpscd_internal.hpp"

#include <algorithm>
#include <cfloat>
#include <cmath>
#include <cstdlib>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <limits>
#include <map>
#include <mutex>
#include <string>
#include <vector>

using namespace hpscd;

namespace {
thread_local std::string g_err;
}

void hpscd::set_last_error(const char* msg) { g_err = msg; }

namespace {

hpscd_status fail(hpscd_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return st;
}

#define HIP_TRY(expr)                                                                        \
  do {                                                                                       \
    hipError_t _e = (expr);                                                                  \
    if (_e != hipSuccess) return fail(HPSCD_EDEVICE, "%s: %s", #expr, hipGetErrorString(_e)); \
  } while (0)

// Grow-only device buffer.
struct DevBuf {
  void* p = nullptr;
  size_t cap = 0;
  hipError_t ensure(size_t bytes) {
    if (bytes <= cap) return hipSuccess;
    if (p) (void)hipFree(p);
    p = nullptr;
    cap = 0;
    size_t want = std::max(bytes, (size_t)256);
    hipError_t e = hipMalloc(&p, want);
    if (e == hipSuccess) cap = want;
    return e;
  }
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    cap = 0;
  }
  template <class T> T* as() const { return reinterpret_cast<T*>(p); }
};

// Control block (one device allocation, read back with one copy).
struct CtlBlock {
  int32_t ctl[8];
  int64_t ctl64[4];
  double fstat[4];
  double ynorm2;
  double fnorm2;
  double pad[2];
};
static_assert(sizeof(CtlBlock) == 128, "control block layout");

constexpr uint64_t kTimeoutTicks = 1000000000ull;  // 10 s of the 100 MHz clock

struct Tuned {
  int B;
  int64_t wave_max_m;            // systems with m <= this share a workgroup, one per wave
  std::vector<int32_t> sweeps;   // sweeps each system took when tuned (order hint; empty: none)
};

// Device workspace of one batched solve (the context's, or a plan's own).
struct BatchWork {
  DevBuf sys, items, blk, rdn, gram, a64, e0, hist, i32, f64;
  void release() {
    for (DevBuf* b : {&sys, &items, &blk, &rdn, &gram, &a64, &e0, &hist, &i32, &f64}) b->release();
  }
};

}  // namespace

// Fixed workspace of hpscd_solve_f32_noalloc: one array per device, loaded
// with the library's code object and kept until the process ends.  In host
// code the name is a stand-in, not a device address: the address is taken
// per device with hipGetSymbolAddress (hpscd_create) and only that pointer
// is used.
constexpr size_t kScratchBytes = (size_t)HPSCD_NOALLOC_SCRATCH_BYTES;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

struct hpscd_ctx {
  int device = 0;
  int cus = 0;
  unsigned char* scratch_ptr = nullptr;  // this device's copy of `scratch`
  DevBuf ctlb, e0, eo, a64, rdn, gram, cross, partial, slots, hist;
  DevBuf selw;  // feature selection: FP64 residual, inner products, flags, results
  BatchWork bw;
  void* host = nullptr;
  size_t host_cap = 0;
  int32_t* cancel_h = nullptr;        // cancel word, pinned host memory mapped into the device
  const int32_t* cancel_d = nullptr;  // its device address
  hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
  std::map<std::string, Tuned> tuned;

  hpscd_status host_ensure(size_t bytes) {
    if (bytes <= host_cap) return HPSCD_OK;
    if (host) (void)hipHostFree(host);
    host = nullptr;
    host_cap = 0;
    if (hipHostMalloc(&host, bytes, hipHostMallocDefault) != hipSuccess)
      return fail(HPSCD_ENOMEM, "pinned host buffer of %zu bytes", bytes);
    host_cap = bytes;
    return HPSCD_OK;
  }
};

namespace {

hpscd_status ensure(DevBuf& b, size_t bytes, const char* what) {
  if (b.ensure(bytes) != hipSuccess) return fail(HPSCD_ENOMEM, "device workspace '%s' (%zu bytes)", what, bytes);
  return HPSCD_OK;
}

bool aligned16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }

}  // namespace

int hpscd::ctx_device(const hpscd_ctx* c) { return c->device; }

namespace {

hpscd_status validate_opts(const hpscd_opts* o) {
  if (!o) return fail(HPSCD_EINVAL, "opts is NULL");
  if (o->max_sweeps < 0) return fail(HPSCD_EINVAL, "max_sweeps must be >= 0 (got %d)", o->max_sweeps);
  if (o->stop < HPSCD_STOP_NONE || o->stop > HPSCD_STOP_REL_GRAD)
    return fail(HPSCD_EINVAL, "unknown stop rule %d", o->stop);
  if (o->thr < 0) return fail(HPSCD_EINVAL, "thr must be >= 0 (got %d)", o->thr);
  if (o->spin_timeout_us < 0) return fail(HPSCD_EINVAL, "spin_timeout_us must be >= 0 (got %d)", o->spin_timeout_us);
  if (o->thr > 1 && o->order) return fail(HPSCD_EINVAL, "thr > 1 (Algorithm 2) and a column order are exclusive");
  if ((o->thr > 1 || o->order) && o->depth != 0 && o->depth != 8)
    return fail(HPSCD_EINVAL, "Algorithm 2 and column orders run on the wide-block kernel (depth 8) only");
  if ((o->thr > 1 || o->order) && o->block != 0 && o->block != 16)
    return fail(HPSCD_EINVAL, "Algorithm 2 and column orders use blocks of 16 columns");
  if ((o->thr > 1 || o->order) && o->refresh_cols > 0)
    return fail(HPSCD_EINVAL, "Algorithm 2 and column orders are single-precision solves without refreshes");
  if (!std::isfinite(o->tol) || o->tol < 0.0) return fail(HPSCD_EINVAL, "tol must be finite and >= 0");
  if (o->check_cols < 0) return fail(HPSCD_EINVAL, "check_cols must be >= 0");
  if (o->refresh_cols < 0) return fail(HPSCD_EINVAL, "refresh_cols must be >= 0");
  if (o->block != 0 && o->block != 1 && o->block != 2 && o->block != 4 && o->block != 8 && o->block != 16 &&
      o->block != 32)
    return fail(HPSCD_EINVAL, "block must be 0, 1, 2, 4, 8, 16 or 32 (got %d)", o->block);
  if (o->depth != 0 && o->depth != 2 && o->depth != 3 && o->depth != 4 && o->depth != 5 && o->depth != 8 &&
      o->depth != 9)
    return fail(HPSCD_EINVAL, "depth (kernel kind) must be 0, 2, 3, 4, 5, 8 or 9 (got %d)", o->depth);
  if (o->block == 16 && o->depth != 0 && o->depth != 8 && o->depth != 9)
    return fail(HPSCD_EINVAL, "block 16 runs only on the wide-block kernel (depth 8) or the chain kernel (depth 9)");
  if (o->block == 32 && o->depth != 0 && o->depth != 9)
    return fail(HPSCD_EINVAL, "block 32 runs only on the chain kernel (depth 9)");
  if (o->depth == 9 && o->block != 0 && o->block != 16 && o->block != 32)
    return fail(HPSCD_EINVAL, "the chain kernel (depth 9) takes blocks of 16 or 32 columns");
  if ((o->flags & HPSCD_F_FORCE_GRID) && (o->flags & HPSCD_F_FORCE_WG))
    return fail(HPSCD_EINVAL, "FORCE_GRID and FORCE_WG are exclusive");
  if ((int64_t)o->max_sweeps + 1 > (int64_t)1 << 30) return fail(HPSCD_EINVAL, "max_sweeps too large");
  return HPSCD_OK;
}

// Largest block size <= want that divides every positive constraint.
int pick_block(int want, std::initializer_list<int64_t> divides) {
  for (int B = want; B >= 1; B /= 2) {
    bool ok = true;
    for (int64_t d : divides)
      if (d > 0 && d % B != 0) ok = false;
    if (ok) return B;
  }
  return 1;
}

struct Plan {
  bool grid;
  int T, R, B, P, D;
  int rpw;  // rows per workgroup
  int V;    // method variant of the wide-block kernel
};

// One planning attempt; `wide` selects the wide-block kernel (16 columns per
// reduction).
static hpscd_status plan_try(hpscd_ctx* c, int64_t m, int64_t n, bool bf16, const hpscd_opts* o, bool wide,
                             Plan* pl) {
  const int V = o->order ? 2 : (o->thr > 1 ? 1 : 0);
  const int VEC = bf16 ? 8 : 4;
  bool grid;
  if (o->flags & HPSCD_F_FORCE_GRID) grid = true;
  else if (o->flags & HPSCD_F_FORCE_WG) grid = false;
  else grid = m > 256 * (bf16 ? 2 : 4) * VEC;
  std::vector<std::pair<int, int>> shapes;  // (T, R) candidates, smallest first
  if (wide) {
    // FP32: the fewest rows per workgroup that keep the grid within 256
    // workgroups (one per CU), so a smaller system still spreads over the chip
    if (bf16) shapes = {{512, 1}};
    else shapes = {{256, 1}, {512, 1}, {512, 2}, {256, 4}, {1024, 1}};
  } else if (grid) {
    // FP32: the polling-wave kernel (kind 5) with 256 threads x 4 chunks first
    // (up to 256 workgroups, 1,048,576 rows), then the plain grid kernel
    if (bf16) shapes = {{1024, 1}, {512, 1}};
    else if (m >= 256 * 1024 * 4) shapes = {{256, 4}, {512, 2}, {1024, 1}};
    else shapes = {{256, 4}, {256, 1}, {256, 2}, {512, 2}, {1024, 1}};
  } else {
    if (bf16) shapes = {{256, 1}, {256, 2}};
    else shapes = {{256, 2}, {256, 4}};
  }
  const int want = o->block > 0 ? o->block : (wide ? 16 : (grid ? 8 : 4));
  // Stop checks and refreshes fall at block starts, counted in column steps
  // from the start of the solve: the block must divide n for those to land
  // on every multiple of check_cols (refresh_cols).
  const bool checks = o->check_cols > 0 && o->stop == HPSCD_STOP_REL_RESID;
  const int64_t need_n = (o->refresh_cols > 0 || checks) ? n : 0;
  int B = pick_block(want, {o->check_cols, o->refresh_cols, need_n});
  if (o->block > 0 && B != o->block)
    return fail(HPSCD_EINVAL, "block %d must divide check_cols, refresh_cols and (with either) n", o->block);
  if (o->team_threads > 0) {
    std::vector<std::pair<int, int>> keep;
    for (int R : {1, 2, 4}) keep.push_back({o->team_threads, R});
    shapes = keep;
  }
  // Kernel kinds in order of preference (see launch_sweep).
  std::vector<int> kinds;
  if (grid && o->depth == 4)
    return fail(HPSCD_EINVAL, "depth 4 (a ring of four blocks) exists for one workgroup only");
  if (o->depth != 0) kinds = {o->depth};
  else if (wide) kinds = {8};
  else if (grid) kinds = {5, 2, 3};
  else kinds = {4, 3, 2};         // one workgroup: the deepest ring hides the most load latency
  auto kind_of = [&](int T, int R, int b) {
    for (int k : kinds)
      if (sweep_variant_exists(T, R, b, bf16, grid, k, k == 8 ? V : 0)) return k;
    return 0;
  };
  for (auto [T, R] : shapes) {
    const int64_t rows = (int64_t)T * R * VEC;
    if (!grid && m > rows) continue;
    int b = B;
    while (b >= 1 && !kind_of(T, R, b)) b /= 2;
    if (b < 1) continue;
    if (o->block > 0 && b != o->block) continue;
    const int kind = kind_of(T, R, b);
    int64_t P = grid ? (m + rows - 1) / rows : 1;
    int64_t rpw = rows;
    if (grid) {
      const int maxw = sweep_max_workgroups(T, R, b, bf16, true, kind, V);
      if (P > maxw) continue;
      const int per_cu = sweep_max_blocks_per_cu(T, R, b, bf16, true, kind, V);
      if (per_cu <= 0 || P > (int64_t)per_cu * c->cus) continue;
      if (kind == 8 && 4 * P >= 3 * (int64_t)c->cus) {
        // a grid that already covers most CUs spreads its rows over one
        // workgroup per CU (at least half the capacity of a workgroup each);
        // on the 1M x 256 system 256 workgroups instead of 245 measured 1.5 %
        // faster, on a 100k-row system twice the workgroups at half the rows
        // measured 5 % slower, so smaller grids are left as they are
        const int64_t Pw = std::min<int64_t>({(int64_t)c->cus, (int64_t)maxw, (m + rows / 2 - 1) / (rows / 2)});
        if (Pw > P) {
          rpw = ((m + Pw - 1) / Pw + VEC - 1) / VEC * VEC;
          P = (m + rpw - 1) / rpw;
        }
      }
    }
    *pl = Plan{grid, T, R, b, (int)P, kind, (int)rpw, V};
    return HPSCD_OK;
  }
  return fail(HPSCD_EINVAL, "no kernel variant fits m=%lld (%s team, block %d)", (long long)m,
              grid ? "grid" : "workgroup", B);
}

// The column chain on one workgroup (kind 9) for systems of at most 2048
// rows: 16-column FP32 or 32-column bfloat16 blocks.  Returns false when it
// does not fit the options (and, when it was asked for, sets the error).
bool plan_chain(int64_t m, int64_t n, int64_t ldx, bool bf16, const hpscd_opts* o, Plan* pl, hpscd_status* rc) {
  const bool asked = o->depth == 9 || o->block == 32;
  *rc = HPSCD_OK;
  const int B = bf16 ? 32 : 16;
  const char* why = nullptr;
  const bool checks = o->check_cols > 0 && o->stop == HPSCD_STOP_REL_RESID;
  if (m > chain_max_rows()) why = "the chain kernel (depth 9, block 32) holds at most 2048 rows";
  else if (o->team_threads > 0 && o->team_threads != 512) why = "the chain kernel (depth 9) runs 512 threads";
  else if ((int64_t)B * ldx * (bf16 ? 2 : 4) > (int64_t)INT32_MAX)
    why = "the chain kernel (depth 9) addresses a block's columns with 32-bit offsets (ldx too large)";
  else if (o->flags & HPSCD_F_FORCE_GRID) why = "the chain kernel (depth 9) is one workgroup";
  else if (o->thr > 1 || o->order) why = "Algorithm 2 and column orders run on the wide-block kernel (depth 8)";
  else if (o->block > 0 && o->block != B) why = "the chain kernel takes 16 FP32 or 32 bfloat16 columns per block";
  else if ((checks && o->check_cols % B) || (o->refresh_cols > 0 && o->refresh_cols % B) ||
           ((checks || o->refresh_cols > 0) && n % B))
    why = "the chain kernel's block must divide check_cols, refresh_cols and (with either) n";
  if (why) {
    if (asked) *rc = fail(HPSCD_EINVAL, "%s", why);
    return false;
  }
  *pl = Plan{false, 512, 1, B, 1, 9, chain_max_rows(), 0};
  return true;
}

hpscd_status plan_single(hpscd_ctx* c, int64_t m, int64_t n, int64_t ldx, bool bf16, const hpscd_opts* o, Plan* pl) {
  // Short systems (one workgroup holds every row): the column chain kernel
  // by default, unless the options ask for another kernel.
  if (o->depth == 9 || o->block == 32 || (o->depth == 0 && m <= chain_max_rows())) {
    hpscd_status rc;
    if (plan_chain(m, n, ldx, bf16, o, pl, &rc)) return HPSCD_OK;
    if (rc != HPSCD_OK) return rc;
  }
  // The wide-block kernel when asked for; by default for FP32 grids, where it
  // measured fastest from 100k to 1M rows (a reduction per 16 columns, none
  // of the exchange's memory operations queued behind column loads), unless
  // the block cannot be 16 (column checks, refreshes) or the grid would
  // exceed 256 workgroups.
  if (o->depth == 8 || (o->depth == 0 && o->block == 16) || o->thr > 1 || o->order)
    return plan_try(c, m, n, bf16, o, true, pl);
  if (o->depth == 0 && o->block == 0 && o->team_threads == 0 && !bf16) {
    Plan wp;
    if (plan_try(c, m, n, bf16, o, true, &wp) == HPSCD_OK && wp.grid) {
      *pl = wp;
      return HPSCD_OK;
    }
  }
  return plan_try(c, m, n, bf16, o, false, pl);
}

// Wait between publishing a grid reduction's words and the first poll of
// the others' words.  A poll that arrives before the slowest workgroup's
// words are visible costs a second round trip (and, in the plain grid kernel,
// waits behind the next block's column loads); the wait that minimised the
// block time grows with the number of workgroups (measured on the 1M x 256
// system and on 64k..500k-row systems).
uint32_t poll_delay_ticks(const Plan& pl) {
  if (!pl.grid) return 0;
  if (pl.D == 5) return (uint32_t)std::min(240.0, 80.0 + 0.6 * pl.P);
  if (pl.D == 8) return (uint32_t)std::min(200.0, 65.0 + 0.22 * pl.P);
  if (pl.D == 2 || pl.D == 3) return (uint32_t)std::min(160.0, 0.65 * pl.P);
  return 0;
}

hpscd_status validate_single(int64_t m, int64_t n, const void* X, int64_t ldx, int vec, const void* y,
                             const hpscd_opts* o, const void* a_out) {
  if (m < 1) return fail(HPSCD_EINVAL, "m must be >= 1 (got %lld)", (long long)m);
  if (n < 1) return fail(HPSCD_EINVAL, "n must be >= 1 (got %lld)", (long long)n);
  if (!X) return fail(HPSCD_EINVAL, "X is NULL");
  if (!y) return fail(HPSCD_EINVAL, "y is NULL");
  if (!a_out) return fail(HPSCD_EINVAL, "a_out is NULL");
  if (ldx < m) return fail(HPSCD_EINVAL, "ldx (%lld) < m (%lld)", (long long)ldx, (long long)m);
  if (ldx % vec != 0) return fail(HPSCD_EINVAL, "ldx (%lld) must be a multiple of %d", (long long)ldx, vec);
  if (!aligned16(X)) return fail(HPSCD_EINVAL, "X must be 16-byte aligned");
  if (n > (int64_t)1 << 40 || m > (int64_t)1 << 40) return fail(HPSCD_EINVAL, "system too large");
  return validate_opts(o);
}

float elapsed(hipEvent_t a, hipEvent_t b) {
  float ms = 0.f;
  if (hipEventElapsedTime(&ms, a, b) != hipSuccess) return -1.f;
  return ms;
}

// Device workspace of one single-system solve: the context's grow-only
// buffers, or regions of a fixed scratch area.
struct Work {
  CtlBlock* cb;
  float *e0, *eo;
  double *a64, *rdn, *gram, *cross, *partial, *hist;
  uint64_t* slots;
  int64_t partial_cap;
};

// Sizes (bytes) of the workspace regions of a solve planned as `pl`.
struct WorkSizes {
  size_t ctl, e0, eo, a64, rdn, gram, cross, partial, slots, hist;
  int64_t partial_cap;
  size_t total() const { return ctl + e0 + eo + a64 + rdn + gram + cross + partial + slots + hist; }
};

WorkSizes work_sizes(const Plan& pl, int64_t m, int64_t n, const hpscd_opts* o) {
  const int B = pl.B;
  const int64_t nb = (n + B - 1) / B;
  const int NG = B * (B - 1) / 2;
  auto r256 = [](size_t b) { return (b + 255) / 256 * 256; };
  WorkSizes w{};
  // partial sums of the column statistics (rows split ~8192 ways over the
  // blocks, at most), of the residual passes, and of X^T e (gradient rule)
  int64_t cap = std::max<int64_t>({(int64_t)1 << 21, nb * B * 80, (m + 1023) / 1024 + 8});
  if (o->stop == HPSCD_STOP_REL_GRAD) cap = std::max<int64_t>(cap, plan_xtv(m, n, (int64_t)1 << 22).need);
  w.partial_cap = cap;
  w.ctl = r256(sizeof(CtlBlock));
  w.e0 = r256((size_t)m * 4);
  w.eo = r256((size_t)m * 4);
  w.a64 = r256((size_t)n * 8);
  w.rdn = r256((size_t)nb * B * 8);
  w.gram = r256((size_t)std::max<int64_t>(1, nb * NG) * 8);
  w.cross = r256((size_t)nb * B * B * 8);
  w.partial = r256((size_t)cap * 8);
  w.slots = r256((size_t)4 * (B + 1) * std::max(1, pl.P) * 8);
  w.hist = r256((size_t)((int64_t)o->max_sweeps + 1) * 8);
  return w;
}

hpscd_status work_from_ctx(hpscd_ctx* c, const WorkSizes& z, Work* w) {
  hpscd_status rc;
  if ((rc = ensure(c->ctlb, z.ctl, "ctl")) || (rc = ensure(c->e0, z.e0, "e0")) || (rc = ensure(c->eo, z.eo, "e")) ||
      (rc = ensure(c->a64, z.a64, "a64")) || (rc = ensure(c->rdn, z.rdn, "rdn")) ||
      (rc = ensure(c->gram, z.gram, "gram")) || (rc = ensure(c->cross, z.cross, "cross")) ||
      (rc = ensure(c->partial, z.partial, "partial")) || (rc = ensure(c->slots, z.slots, "slots")) ||
      (rc = ensure(c->hist, z.hist, "hist")))
    return rc;
  *w = Work{c->ctlb.as<CtlBlock>(), c->e0.as<float>(), c->eo.as<float>(), c->a64.as<double>(),
            c->rdn.as<double>(), c->gram.as<double>(), c->cross.as<double>(), c->partial.as<double>(),
            c->hist.as<double>(), c->slots.as<uint64_t>(), (int64_t)(c->partial.cap / 8)};
  return HPSCD_OK;
}

// Host-side landing area of a solve's results: the control block and hist.
struct HostOut {
  CtlBlock* cb;
  double* hist;  // max_sweeps + 1 doubles
};

hpscd_status solve_single(hpscd_ctx* c, int64_t m, int64_t n, const void* Xs, int64_t ldxs, bool bf16,
                          const float* X32, int64_t ldx32, const float* y, const float* a0, const hpscd_opts* o,
                          float* a_out, double* hist, hpscd_info* info, hipStream_t st, const Plan& pl,
                          const Work& w, const HostOut& ho) {
  HIP_TRY(hipSetDevice(c->device));
  const int B = pl.B;
  const int64_t nb = (n + B - 1) / B;
  const int64_t hist_len = (int64_t)o->max_sweeps + 1;
  const int64_t partial_cap = w.partial_cap;
  const bool grad_rule = o->stop == HPSCD_STOP_REL_GRAD;
  const bool ordered = pl.V == 2;

  CtlBlock* cb = w.cb;
  int32_t* ctl = reinterpret_cast<int32_t*>(cb);
  int64_t* ctl64 = reinterpret_cast<int64_t*>(reinterpret_cast<char*>(cb) + offsetof(CtlBlock, ctl64));
  double* fstat = reinterpret_cast<double*>(reinterpret_cast<char*>(cb) + offsetof(CtlBlock, fstat));
  double* ynorm2 = reinterpret_cast<double*>(reinterpret_cast<char*>(cb) + offsetof(CtlBlock, ynorm2));
  double* fnorm2 = reinterpret_cast<double*>(reinterpret_cast<char*>(cb) + offsetof(CtlBlock, fnorm2));
  double* partial = w.partial;

  // a cancel request concerns the solve running when it is made
  __atomic_store_n(c->cancel_h, 0, __ATOMIC_SEQ_CST);
  HIP_TRY(hipEventRecord(c->ev[0], st));
  HIP_TRY(launch_fill_i32(ctl, sizeof(CtlBlock) / 4, 0, st));
  HIP_TRY(launch_fill_f64(w.hist, hist_len, std::numeric_limits<double>::quiet_NaN(), st));
  if (pl.grid) HIP_TRY(launch_fill_u64(w.slots, 4 * (int64_t)(B + 1) * pl.P, 0, st));
  HIP_TRY(launch_a_init(w.a64, a0, n, st));
  HIP_TRY(launch_residual(X32, ldx32, m, 0, y, nullptr, nullptr, nullptr, ynorm2, partial, partial_cap, nullptr, st));
  const float* e0 = y;
  if (a0) {
    HIP_TRY(launch_residual(X32, ldx32, m, n, y, nullptr, a0, w.e0, nullptr, partial, partial_cap, nullptr, st));
    e0 = w.e0;
  }
  // column statistics (under a column order: before every sweep, below)
  if (!ordered)
  {
    if (pl.D == 9 && B == 32)
      HIP_TRY(launch_colgram32(Xs, bf16, ldxs, m, n, w.rdn, w.gram, w.cross, partial, partial_cap, ctl,
                               &ctl64[C64_ZERO_COLS], st));
    else
      HIP_TRY(launch_colgram(Xs, bf16, ldxs, m, n, B, w.rdn, w.gram, B == 16 ? w.cross : nullptr, partial,
                             partial_cap, ctl, &ctl64[C64_ZERO_COLS], st, nullptr, pl.V == 1 ? o->thr : 0));
  }
  if (grad_rule)
    HIP_TRY(launch_grad_stop(X32, ldx32, m, n, y, true, 0, o->tol, partial, partial_cap, ctl, ctl64, fstat, w.hist,
                             st));
  HIP_TRY(hipEventRecord(c->ev[1], st));

  SolveArgs A{};
  A.X = Xs;
  A.ldx = ldxs;
  A.m = m;
  A.n = n;
  A.rdn = w.rdn;
  A.gram = w.gram;
  A.minv = B >= 16 ? w.cross : nullptr;
  A.a64 = w.a64;
  A.e_out = w.eo;
  A.hist = w.hist;
  A.slots = w.slots;
  A.ctl = ctl;
  A.fstat = fstat;
  A.ctl64 = ctl64;
  A.max_sweeps = o->max_sweeps;
  A.stop = o->stop;
  A.tol = o->tol;
  A.ynorm2 = ynorm2;
  A.check_cols = (o->stop == HPSCD_STOP_REL_RESID) ? o->check_cols : 0;
  A.P = pl.P;
  A.rows_per_wg = pl.rpw;
  // every spin-wait is bounded: 10 s of the 100 MHz clock, or the caller's
  // bound (a bound below two first-poll pauses also halves that pause)
  A.timeout_ticks = o->spin_timeout_us > 0 ? (uint64_t)o->spin_timeout_us * 100 : kTimeoutTicks;
  A.poll_delay = (uint32_t)std::min<uint64_t>(poll_delay_ticks(pl), A.timeout_ticks / 2);
  A.thr = o->thr;
  A.order = o->order;
  A.cancel = c->cancel_d;
  const int64_t total = (int64_t)o->max_sweeps * nb + 1;
  // launch segments: a refresh period, or one sweep when something runs
  // between sweeps (the gradient rule's pass, a column order's statistics)
  const int64_t seg = (grad_rule || ordered) ? nb
                      : (o->refresh_cols > 0) ? std::max<int64_t>(1, o->refresh_cols / B) : total;
  const bool coop = pl.grid && !(o->flags & HPSCD_F_NO_COOP);
  int refreshes = 0;
  // Refreshes with the relative-residual rule: the running residual drifts
  // from y - X·a (bfloat16 columns, or FP32 rounding over many steps), so a
  // stop it signals is confirmed on the residual recomputed from X32 (FP64
  // sums); if that one is not yet under the tolerance, the sweeps resume
  // where they stopped.
  const bool confirm = o->refresh_cols > 0 && o->stop == HPSCD_STOP_REL_RESID;
  CtlBlock* hcb = ho.cb;
  bool resumed = false;
  for (int64_t kb = 0; kb < total;) {
    A.e0 = (kb == 0 && !resumed) ? e0 : w.eo;
    A.blk_begin = kb;
    A.blk_end = std::min(total, (kb / seg + 1) * seg);  // refreshes stay on multiples of refresh_cols
    const int64_t sweep = kb / nb;                       // (segments of one sweep: the sweep it runs)
    if (ordered && sweep < o->max_sweeps)
      HIP_TRY(launch_colgram(Xs, false, ldxs, m, n, B, w.rdn, w.gram, w.cross, partial, partial_cap, ctl,
                             sweep == 0 ? &ctl64[C64_ZERO_COLS] : nullptr, st, o->order + sweep * n, 0));
    if (pl.D == 9) HIP_TRY(launch_chain(bf16, B, A, st));
    else HIP_TRY(launch_sweep(pl.T, pl.R, B, bf16, pl.grid, pl.D, A, st, coop, pl.V));
    if (grad_rule && A.blk_end < total)
      HIP_TRY(launch_grad_stop(X32, ldx32, m, n, w.eo, false, (int32_t)(sweep + 1), o->tol, partial, partial_cap, ctl,
                               ctl64, fstat, w.hist, st));
    if ((grad_rule || ordered) && A.blk_end < total) {
      // stop queueing sweeps once the solve has ended
      HIP_TRY(hipMemcpyAsync(hcb, cb, sizeof(CtlBlock), hipMemcpyDeviceToHost, st));
      HIP_TRY(hipStreamSynchronize(st));
      if (hcb->ctl[CTL_DONE]) break;
    }
    if (confirm) {
      HIP_TRY(hipMemcpyAsync(hcb, cb, sizeof(CtlBlock), hipMemcpyDeviceToHost, st));
      HIP_TRY(hipStreamSynchronize(st));
      if (hcb->ctl[CTL_DONE]) {
        if (!hcb->ctl[CTL_CONVERGED] || hcb->ctl[CTL_ERR] || hcb->ctl[CTL_NONFINITE]) break;
        const int64_t cs = hcb->ctl64[C64_COLS];
        const int64_t touched = a0 ? n : std::min(n, cs);
        HIP_TRY(launch_residual(X32, ldx32, m, touched, y, w.a64, nullptr, w.eo, fnorm2, partial, partial_cap, nullptr,
                                st));
        ++refreshes;
        HIP_TRY(hipMemcpyAsync(hcb, cb, sizeof(CtlBlock), hipMemcpyDeviceToHost, st));
        HIP_TRY(hipStreamSynchronize(st));
        const double ynorm = std::sqrt(hcb->ynorm2);
        if (hcb->fnorm2 == 0.0 || std::sqrt(hcb->fnorm2) < o->tol * ynorm) break;
        // not yet: clear the stop and resume at the block where it fired
        HIP_TRY(launch_fill_i32(&ctl[CTL_CONVERGED], 1, 0, st));
        HIP_TRY(launch_fill_i32(&ctl[CTL_DONE], 1, 0, st));
        if (pl.grid) HIP_TRY(launch_fill_u64(w.slots, 4 * (int64_t)(B + 1) * pl.P, 0, st));
        kb = (cs / n) * nb + (cs % n) / B;
        resumed = true;
        continue;
      }
    }
    if (o->refresh_cols > 0 && A.blk_end < total) {
      const int64_t cols = (A.blk_end / nb) * n + (A.blk_end % nb) * B;
      const int64_t touched = a0 ? n : std::min(n, cols);
      HIP_TRY(launch_residual(X32, ldx32, m, touched, y, w.a64, nullptr, w.eo, nullptr, partial, partial_cap,
                              &ctl[CTL_DONE], st));
      ++refreshes;
    }
    kb = A.blk_end;
  }
  HIP_TRY(hipEventRecord(c->ev[2], st));
  HIP_TRY(launch_a_out(w.a64, a_out, n, st));
  // the final check judges the coefficients returned (single precision)
  const bool check = !(o->flags & HPSCD_F_NO_FINAL_CHECK);
  if (check)
    HIP_TRY(launch_residual(X32, ldx32, m, n, y, nullptr, a_out, nullptr, fnorm2, partial, partial_cap, nullptr, st));
  HIP_TRY(hipEventRecord(c->ev[3], st));
  CtlBlock* hc = ho.cb;
  double* hh = ho.hist;
  HIP_TRY(hipMemcpyAsync(hc, cb, sizeof(CtlBlock), hipMemcpyDeviceToHost, st));
  if (hh) HIP_TRY(hipMemcpyAsync(hh, w.hist, (size_t)hist_len * 8, hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));

  if (hist && hh && hist != hh) std::memcpy(hist, hh, (size_t)hist_len * 8);
  if (info) {
    std::memset(info, 0, sizeof *info);
    info->sweeps_done = hc->ctl[CTL_SWEEPS];
    info->converged = hc->ctl[CTL_CONVERGED];
    info->cols_done = hc->ctl64[C64_COLS];
    info->zero_cols = hc->ctl64[C64_ZERO_COLS];
    info->final_norm = std::sqrt(hc->fstat[0]);
    info->y_norm = std::sqrt(hc->ynorm2);
    info->final_rel_resid = check ? (info->y_norm > 0 ? std::sqrt(hc->fnorm2) / info->y_norm : std::sqrt(hc->fnorm2))
                                  : std::numeric_limits<double>::quiet_NaN();
    info->block_used = B;
    info->team_wgs = pl.P;
    info->team_threads = pl.T;
    info->refreshes = refreshes;
    info->sweep_ms = elapsed(c->ev[1], c->ev[2]);
    info->total_ms = elapsed(c->ev[0], c->ev[3]);
    info->kernel_kind = pl.D;
    // ||e|| grew over a sweep (by more than 0.1 %)
    if (hh)
      for (int32_t k = 1; k <= info->sweeps_done && k < hist_len; ++k)
        if (hh[k] > hh[k - 1] * 1.001) info->diverged = 1;
    info->rel_grad = (grad_rule && info->sweeps_done > 0) ? hc->fstat[2] : std::numeric_limits<double>::quiet_NaN();
  }
  if (hc->ctl[CTL_NONFINITE]) return fail(HPSCD_ENONFINITE, "X or y holds a non-finite value");
  if (hc->ctl[CTL_ERR] == ERR_TIMEOUT) return fail(HPSCD_ETIMEOUT, "grid reduction timed out");
  if (hc->ctl[CTL_ERR] == ERR_ABORTED) return fail(HPSCD_EABORTED, "solve aborted");
  if (hc->ctl[CTL_ERR] == ERR_NONFINITE) return fail(HPSCD_ENONFINITE, "the iteration produced a non-finite residual");
  g_err.clear();
  return HPSCD_OK;
}

// Regions of the fixed scratch area for a solve planned as `pl`: the
// context-path layout, with the partial sums limited to what the column
// statistics of one 8192-way row split, the residual passes and the
// gradient rule use, and no starting-residual buffer when a0 is absent.
hpscd_status work_from_scratch(hpscd_ctx* c, const Plan& pl, int64_t m, int64_t n, const hpscd_opts* o, bool has_a0,
                               Work* w) {
  WorkSizes z = work_sizes(pl, m, n, o);
  const int B = pl.B;
  const int64_t nb = (n + B - 1) / B, NPX = B * (B + 1) / 2;
  int64_t cap = std::max<int64_t>({(int64_t)8192 * NPX, nb * NPX, (m + 1023) / 1024 + 8});
  if (o->stop == HPSCD_STOP_REL_GRAD) cap = std::max<int64_t>(cap, plan_xtv(m, n, (int64_t)1 << 22).need);
  z.partial_cap = cap;
  z.partial = (size_t)cap * 8;
  if (!has_a0) z.e0 = 0;
  if (B != 16) z.cross = 0;  // (step matrices: 16-column blocks only)
  if (z.total() > kScratchBytes)
    return fail(HPSCD_EINVAL, "the solve needs %zu bytes of workspace, more than the %zu-byte scratch area of the "
                "allocation-free entry point", z.total(), kScratchBytes);
  unsigned char* p = c->scratch_ptr;
  auto take = [&](size_t b) { unsigned char* q = p; p += b; return q; };
  w->cb = reinterpret_cast<CtlBlock*>(take(z.ctl));
  w->e0 = reinterpret_cast<float*>(take(z.e0));
  w->eo = reinterpret_cast<float*>(take(z.eo));
  w->a64 = reinterpret_cast<double*>(take(z.a64));
  w->rdn = reinterpret_cast<double*>(take(z.rdn));
  w->gram = reinterpret_cast<double*>(take(z.gram));
  w->cross = reinterpret_cast<double*>(take(z.cross));
  w->partial = reinterpret_cast<double*>(take(z.partial));
  w->slots = reinterpret_cast<uint64_t*>(take(z.slots));
  w->hist = reinterpret_cast<double*>(take(z.hist));
  w->partial_cap = cap;
  return HPSCD_OK;
}

// Plan, size the context's workspace and solve.
hpscd_status solve_single_ctx(hpscd_ctx* c, int64_t m, int64_t n, const void* Xs, int64_t ldxs, bool bf16,
                              const float* X32, int64_t ldx32, const float* y, const float* a0, const hpscd_opts* o,
                              float* a_out, double* hist, hpscd_info* info, hipStream_t st) {
  hpscd_opts oo = *o;
  if (oo.max_sweeps == 0) oo.order = nullptr;  // (no sweep: the order is not read)
  o = &oo;
  Plan pl;
  hpscd_status rc = plan_single(c, m, n, ldxs, bf16, o, &pl);
  if (rc != HPSCD_OK) return rc;
  HIP_TRY(hipSetDevice(c->device));
  if (pl.V == 2 && n * (int64_t)(ldxs * 4) > (int64_t)0xFFFFFFFF)
    return fail(HPSCD_EINVAL, "a column order needs X below 4 GiB");
  const WorkSizes z = work_sizes(pl, m, n, o);
  Work w;
  if ((rc = work_from_ctx(c, z, &w)) != HPSCD_OK) return rc;
  const int64_t hist_len = (int64_t)o->max_sweeps + 1;
  if ((rc = c->host_ensure(sizeof(CtlBlock) + (size_t)hist_len * 8))) return rc;
  HostOut ho{reinterpret_cast<CtlBlock*>(c->host),
             reinterpret_cast<double*>(reinterpret_cast<char*>(c->host) + sizeof(CtlBlock))};
  return solve_single(c, m, n, Xs, ldxs, bf16, X32, ldx32, y, a0, o, a_out, hist, info, st, pl, w, ho);
}

}  // namespace

extern "C" {

int hpscd_version(void) { return HPSCD_VERSION; }

const char* hpscd_last_error(void) { return g_err.c_str(); }

void hpscd_default_opts(hpscd_opts* o) {
  if (!o) return;
  std::memset(o, 0, sizeof *o);
  o->max_sweeps = 100;
  o->stop = HPSCD_STOP_NONE;
}

hpscd_status hpscd_create(int device, hpscd_ctx** out) {
  try {
    if (!out) return fail(HPSCD_EINVAL, "out is NULL");
    *out = nullptr;
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || count <= 0) return fail(HPSCD_EDEVICE, "no HIP device");
    if (device < 0 || device >= count) return fail(HPSCD_EDEVICE, "device %d out of range (%d devices)", device, count);
    HIP_TRY(hipSetDevice(device));
    hipDeviceProp_t prop;
    HIP_TRY(hipGetDeviceProperties(&prop, device));
    hpscd_ctx* c = new hpscd_ctx();
    c->device = device;
    c->cus = prop.multiProcessorCount;
    {
      void* sp = nullptr;
      const hipError_t e = hipGetSymbolAddress(&sp, HIP_SYMBOL(scratch));
      if (e != hipSuccess || !sp) {
        delete c;
        return fail(HPSCD_EDEVICE, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
      }
      c->scratch_ptr = static_cast<unsigned char*>(sp);
    }
    for (auto& e : c->ev)
      if (hipEventCreate(&e) != hipSuccess) { delete c; return fail(HPSCD_EDEVICE, "hipEventCreate"); }
    {
      void* hp = nullptr;
      void* dp = nullptr;
      if (hipHostMalloc(&hp, 64, hipHostMallocMapped | hipHostMallocCoherent) != hipSuccess) {
        delete c;
        return fail(HPSCD_ENOMEM, "pinned cancel word");
      }
      c->cancel_h = static_cast<int32_t*>(hp);
      *c->cancel_h = 0;
      if (hipHostGetDevicePointer(&dp, hp, 0) != hipSuccess || !dp) {
        (void)hipHostFree(hp);
        delete c;
        return fail(HPSCD_EDEVICE, "hipHostGetDevicePointer(cancel word)");
      }
      c->cancel_d = static_cast<const int32_t*>(dp);
    }
    *out = c;
    g_err.clear();
    return HPSCD_OK;
  } catch (...) {
    return fail(HPSCD_ENOMEM, "allocation failure");
  }
}

void hpscd_destroy(hpscd_ctx* c) {
  if (!c) return;
  (void)hipSetDevice(c->device);
  (void)hipDeviceSynchronize();
  for (DevBuf* b : {&c->ctlb, &c->e0, &c->eo, &c->a64, &c->rdn, &c->gram, &c->cross, &c->partial, &c->slots, &c->hist,
                    &c->selw})
    b->release();
  c->bw.release();
  if (c->host) (void)hipHostFree(c->host);
  for (auto& e : c->ev) if (e) (void)hipEventDestroy(e);
  if (c->cancel_h) (void)hipHostFree(c->cancel_h);
  delete c;
}

hpscd_status hpscd_validate(int64_t m, int64_t n, const void* X, int64_t ldx, int elem_bytes, const void* y,
                            const hpscd_opts* opts, const void* a_out) {
  if (elem_bytes != 4 && elem_bytes != 2) return fail(HPSCD_EINVAL, "elem_bytes must be 4 or 2");
  return validate_single(m, n, X, ldx, elem_bytes == 4 ? 4 : 8, y, opts, a_out);
}

hpscd_status hpscd_solve_f32(hpscd_ctx* ctx, int64_t m, int64_t n, const float* X, int64_t ldx, const float* y,
                             const float* a0, const hpscd_opts* opts, float* a_out, double* hist, hpscd_info* info,
                             void* stream) {
  try {
    hpscd_status rc = validate_single(m, n, X, ldx, 4, y, opts, a_out);
    if (rc != HPSCD_OK) return rc;
    if (!ctx) return fail(HPSCD_EINVAL, "ctx is NULL");
    return solve_single_ctx(ctx, m, n, X, ldx, false, X, ldx, y, a0, opts, a_out, hist, info, (hipStream_t)stream);
  } catch (...) {
    return fail(HPSCD_ENOMEM, "host allocation failure");
  }
}

hpscd_status hpscd_solve_f32_noalloc(hpscd_ctx* ctx, int64_t m, int64_t n, const float* X, int64_t ldx,
                                     const float* y, const float* a0, const hpscd_opts* opts, float* a_out,
                                     double* hist, hpscd_info* info, void* stream) {
  try {
    hpscd_status rc = validate_single(m, n, X, ldx, 4, y, opts, a_out);
    if (rc != HPSCD_OK) return rc;
    if (!ctx) return fail(HPSCD_EINVAL, "ctx is NULL");
    if (!ctx->scratch_ptr) return fail(HPSCD_EDEVICE, "the context has no scratch area");
    hpscd_opts oo = *opts;
    if (oo.max_sweeps == 0) oo.order = nullptr;
    Plan pl;
    if ((rc = plan_single(ctx, m, n, ldx, false, &oo, &pl)) != HPSCD_OK) return rc;
    if (pl.V == 2 && n * (int64_t)(ldx * 4) > (int64_t)0xFFFFFFFF)
      return fail(HPSCD_EINVAL, "a column order needs X below 4 GiB");
    Work w;
    if ((rc = work_from_scratch(ctx, pl, m, n, &oo, a0 != nullptr, &w)) != HPSCD_OK) return rc;
    // results come back through pageable copies into the caller's memory
    CtlBlock hcb;
    HostOut ho{&hcb, hist};
    return solve_single(ctx, m, n, X, ldx, false, X, ldx, y, a0, &oo, a_out, hist, info, (hipStream_t)stream, pl,
                        w, ho);
  } catch (...) {
    return fail(HPSCD_ENOMEM, "host allocation failure");
  }
}

hpscd_status hpscd_solve_bf16(hpscd_ctx* ctx, int64_t m, int64_t n, const uint16_t* Xb, int64_t ldxb, const float* X32,
                              int64_t ldx, const float* y, const float* a0, const hpscd_opts* opts, float* a_out,
                              double* hist, hpscd_info* info, void* stream) {
  try {
    hpscd_status rc = validate_single(m, n, Xb, ldxb, 8, y, opts, a_out);
    if (rc != HPSCD_OK) return rc;
    if (!X32) return fail(HPSCD_EINVAL, "X32 is NULL");
    if (ldx < m || ldx % 4 != 0 || !aligned16(X32))
      return fail(HPSCD_EINVAL, "X32 needs ldx >= m, ldx %% 4 == 0 and 16-byte alignment");
    if (!ctx) return fail(HPSCD_EINVAL, "ctx is NULL");
    return solve_single_ctx(ctx, m, n, Xb, ldxb, true, X32, ldx, y, a0, opts, a_out, hist, info, (hipStream_t)stream);
  } catch (...) {
    return fail(HPSCD_ENOMEM, "host allocation failure");
  }
}

hpscd_status hpscd_convert_bf16(hpscd_ctx* ctx, int64_t rows, int64_t cols, const float* src, int64_t lds,
                                uint16_t* dst, int64_t ldd, void* stream) {
  if (!ctx) return fail(HPSCD_EINVAL, "ctx is NULL");
  if (rows < 1 || cols < 1) return fail(HPSCD_EINVAL, "rows and cols must be >= 1");
  if (!src || !dst) return fail(HPSCD_EINVAL, "NULL array");
  if (lds < rows || ldd < rows || ldd % 8 != 0 || !aligned16(dst))
    return fail(HPSCD_EINVAL, "need lds >= rows, ldd >= rows, ldd %% 8 == 0, dst 16-byte aligned");
  HIP_TRY(hipSetDevice(ctx->device));
  HIP_TRY(launch_f32_to_bf16(src, dst, rows, cols, lds, ldd, (hipStream_t)stream));
  return HPSCD_OK;
}

hpscd_status hpscd_residual_f64(hpscd_ctx* ctx, int64_t m, int64_t n, const float* X, int64_t ldx, const float* y,
                                const float* a, float* e_out, double* norm_out, void* stream) {
  if (!ctx) return fail(HPSCD_EINVAL, "ctx is NULL");
  if (m < 1 || n < 1 || !X || !y || !a) return fail(HPSCD_EINVAL, "bad residual arguments");
  if (ldx < m || ldx % 4 != 0 || !aligned16(X)) return fail(HPSCD_EINVAL, "X layout");
  HIP_TRY(hipSetDevice(ctx->device));
  const int64_t cap = std::max<int64_t>((int64_t)1 << 21, (m + 1023) / 1024 + 8);
  hpscd_status rc;
  if ((rc = ensure(ctx->partial, (size_t)cap * 8, "partial")) || (rc = ensure(ctx->ctlb, sizeof(CtlBlock), "ctl")))
    return rc;
  if ((rc = ctx->host_ensure(64))) return rc;
  double* d = reinterpret_cast<double*>(reinterpret_cast<char*>(ctx->ctlb.p) + offsetof(CtlBlock, fnorm2));
  hipStream_t st = (hipStream_t)stream;
  HIP_TRY(launch_residual(X, ldx, m, n, y, nullptr, a, e_out, d, ctx->partial.as<double>(), cap, nullptr, st));
  if (norm_out) {
    HIP_TRY(hipMemcpyAsync(ctx->host, d, 8, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    *norm_out = std::sqrt(*reinterpret_cast<double*>(ctx->host));
  }
  return HPSCD_OK;
}

hpscd_status hpscd_select_f32(hpscd_ctx* ctx, int64_t m, int64_t n, const float* X, int64_t ldx, const float* y,
                              const float* a0, int32_t F, double tol, float* a_out, int32_t* J_out,
                              double* da_out, double* hist, int32_t* selected, void* stream) {
  try {
    if (!ctx) return fail(HPSCD_EINVAL, "ctx is NULL");
    if (m < 1 || n < 1) return fail(HPSCD_EINVAL, "m and n must be >= 1");
    if (!X || !y || !a_out) return fail(HPSCD_EINVAL, "X, y and a_out must not be NULL");
    if (!J_out || !selected) return fail(HPSCD_EINVAL, "J_out and selected must not be NULL");
    if (ldx < m || ldx % 4 != 0 || !aligned16(X))
      return fail(HPSCD_EINVAL, "X needs ldx >= m, ldx %% 4 == 0 and 16-byte alignment");
    if (F < 0) return fail(HPSCD_EINVAL, "F must be >= 0");
    if (!std::isfinite(tol) || tol < 0.0) return fail(HPSCD_EINVAL, "tol must be finite and >= 0");
    if (n > (int64_t)65535 * 64) return fail(HPSCD_EINVAL, "n above %lld", (long long)65535 * 64);
    if (m > (int64_t)1 << 40) return fail(HPSCD_EINVAL, "system too large");
    hipStream_t st = (hipStream_t)stream;
    hpscd_ctx* c = ctx;
    HIP_TRY(hipSetDevice(c->device));
    const int32_t Fe = (int32_t)std::min<int64_t>(F, n);
    // workspace: the column statistics and the residual passes share the
    // partial sums with X^T e
    int64_t cap = std::max<int64_t>({(int64_t)1 << 21, n * 80, (m + 1023) / 1024 + 8});
    const XtvPlan xp = plan_xtv(m, n, cap);
    cap = std::max<int64_t>(cap, xp.need);
    hpscd_status rc;
    if ((rc = ensure(c->ctlb, sizeof(CtlBlock), "ctl")) || (rc = ensure(c->a64, (size_t)n * 8, "a64")) ||
        (rc = ensure(c->rdn, (size_t)n * 8, "rdn")) || (rc = ensure(c->gram, 8, "gram")) ||
        (rc = ensure(c->partial, (size_t)cap * 8, "partial")))
      return rc;
    // selection region: e64[m], g[n], tscore[T], tidx[T], flags[n], J[F], da[F], hist[F+1], part[m/1024+1],
    // step (j, da), final norm
    const int64_t nparts = (m + 1023) / 1024;
    auto al = [](int64_t b) { return (b + 255) / 256 * 256; };
    const int64_t o_e = 0, o_g = o_e + al(m * 8), o_ts = o_g + al(n * 8), o_ti = o_ts + al(xp.T * 8),
                  o_fl = o_ti + al(xp.T * 8), o_J = o_fl + al(n * 4), o_da = o_J + al((int64_t)Fe * 4 + 4),
                  o_h = o_da + al((int64_t)Fe * 8 + 8), o_p = o_h + al(((int64_t)Fe + 1) * 8), o_s = o_p + al(nparts * 8),
                  o_end = o_s + 256;
    if ((rc = ensure(c->selw, (size_t)o_end, "selection workspace"))) return rc;
    const size_t host_bytes = sizeof(CtlBlock) + ((size_t)Fe + 1) * 8 * 2 + (size_t)Fe * 4 + 64;
    if ((rc = c->host_ensure(host_bytes))) return rc;
    char* sw = reinterpret_cast<char*>(c->selw.p);
    double* e64 = reinterpret_cast<double*>(sw + o_e);
    double* g = reinterpret_cast<double*>(sw + o_g);
    double* tsc = reinterpret_cast<double*>(sw + o_ts);
    int64_t* tid = reinterpret_cast<int64_t*>(sw + o_ti);
    int32_t* flags = reinterpret_cast<int32_t*>(sw + o_fl);
    int32_t* Jd = reinterpret_cast<int32_t*>(sw + o_J);
    double* dad = reinterpret_cast<double*>(sw + o_da);
    double* hd = reinterpret_cast<double*>(sw + o_h);
    double* parts = reinterpret_cast<double*>(sw + o_p);
    int64_t* step_j = reinterpret_cast<int64_t*>(sw + o_s);
    double* step_da = reinterpret_cast<double*>(sw + o_s + 8);
    double* fin = reinterpret_cast<double*>(sw + o_s + 16);
    CtlBlock* cb = c->ctlb.as<CtlBlock>();
    int32_t* ctl = reinterpret_cast<int32_t*>(cb);
    int64_t* ctl64 = reinterpret_cast<int64_t*>(reinterpret_cast<char*>(cb) + offsetof(CtlBlock, ctl64));
    double* ynorm2 = reinterpret_cast<double*>(reinterpret_cast<char*>(cb) + offsetof(CtlBlock, ynorm2));
    double* partial = c->partial.as<double>();
    const int64_t pcap = (int64_t)(c->partial.cap / 8);

    HIP_TRY(launch_fill_i32(ctl, sizeof(CtlBlock) / 4, 0, st));
    HIP_TRY(launch_fill_i32(flags, n, 0, st));
    HIP_TRY(launch_fill_i32(Jd, Fe + 1, -1, st));
    HIP_TRY(launch_fill_f64(hd, Fe + 1, std::numeric_limits<double>::quiet_NaN(), st));
    HIP_TRY(launch_a_init(c->a64.as<double>(), a0, n, st));
    HIP_TRY(launch_residual(X, ldx, m, 0, y, nullptr, nullptr, nullptr, ynorm2, partial, pcap, nullptr, st));
    // <X_j, X_j> (as 1/<X_j, X_j>, 0 for a zero column) with FP64 sums
    HIP_TRY(launch_colgram(X, false, ldx, m, n, 1, c->rdn.as<double>(), c->gram.as<double>(), nullptr, partial, pcap,
                           ctl, &ctl64[C64_ZERO_COLS], st));
    if (a0)
      HIP_TRY(launch_residual(X, ldx, m, n, y, nullptr, a0, nullptr, nullptr, partial, pcap, nullptr, st, e64));
    else
      HIP_TRY(launch_to_f64(y, e64, m, st));
    for (int32_t f = 0; f < Fe; ++f)
      HIP_TRY(launch_select_step(X, ldx, m, n, e64, xp, partial, partial + xp.S * n, g, tsc, tid, c->rdn.as<double>(),
                                 f, tol, flags, c->a64.as<double>(), Jd, dad, hd, ctl, step_j, step_da, st));
    HIP_TRY(launch_norm_f64(e64, m, parts, fin, st));
    HIP_TRY(launch_a_out(c->a64.as<double>(), a_out, n, st));
    char* h = reinterpret_cast<char*>(c->host);
    CtlBlock* hcb = reinterpret_cast<CtlBlock*>(h);
    double* hh = reinterpret_cast<double*>(h + sizeof(CtlBlock));
    double* hda = hh + Fe + 1;
    int32_t* hJ = reinterpret_cast<int32_t*>(hda + Fe + 1);
    double* hfin = reinterpret_cast<double*>(hJ + Fe + 2);
    HIP_TRY(hipMemcpyAsync(hcb, cb, sizeof(CtlBlock), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipMemcpyAsync(hh, hd, ((size_t)Fe + 1) * 8, hipMemcpyDeviceToHost, st));
    if (Fe > 0) HIP_TRY(hipMemcpyAsync(hda, dad, (size_t)Fe * 8, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipMemcpyAsync(hJ, Jd, ((size_t)Fe + 1) * 4, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipMemcpyAsync(hfin, fin, 8, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    if (hcb->ctl[CTL_NONFINITE] || !(hcb->ynorm2 <= DBL_MAX))
      return fail(HPSCD_ENONFINITE, "X or y holds a non-finite value");
    const int32_t cnt = hcb->ctl[CTL_SWEEPS];
    *selected = cnt;
    for (int32_t f = 0; f < F; ++f) J_out[f] = f < cnt ? hJ[f] : -1;
    if (da_out)
      for (int32_t f = 0; f < F; ++f) da_out[f] = f < cnt ? hda[f] : std::numeric_limits<double>::quiet_NaN();
    if (hist) {
      for (int32_t f = 0; f <= F; ++f) hist[f] = f < cnt ? hh[f] : std::numeric_limits<double>::quiet_NaN();
      hist[cnt] = *hfin;
    }
    g_err.clear();
    return HPSCD_OK;
  } catch (...) {
    return fail(HPSCD_ENOMEM, "host allocation failure");
  }
}

hpscd_status hpscd_read_stream(hpscd_ctx* ctx, const void* buf, int64_t bytes, int32_t passes, double* ms_per_pass,
                               void* stream) {
  if (!ctx) return fail(HPSCD_EINVAL, "ctx is NULL");
  if (!buf || !ms_per_pass) return fail(HPSCD_EINVAL, "NULL argument");
  if (bytes < 16 || bytes % 16 != 0 || !aligned16(buf))
    return fail(HPSCD_EINVAL, "need a 16-byte aligned buffer of a positive multiple of 16 bytes");
  if (passes < 1) return fail(HPSCD_EINVAL, "passes must be >= 1");
  HIP_TRY(hipSetDevice(ctx->device));
  const int grid = 16 * ctx->cus;  // sixteen workgroups of 256 threads per CU
  hpscd_status rc;
  if ((rc = ensure(ctx->partial, (size_t)grid * 256 * 4, "sink"))) return rc;
  hipStream_t st = (hipStream_t)stream;
  HIP_TRY(launch_read_stream(buf, bytes, grid, ctx->partial.as<float>(), st));  // (first touch)
  HIP_TRY(hipEventRecord(ctx->ev[0], st));
  for (int32_t k = 0; k < passes; ++k) HIP_TRY(launch_read_stream(buf, bytes, grid, ctx->partial.as<float>(), st));
  HIP_TRY(hipEventRecord(ctx->ev[1], st));
  HIP_TRY(hipEventSynchronize(ctx->ev[1]));
  *ms_per_pass = elapsed(ctx->ev[0], ctx->ev[1]) / passes;
  return HPSCD_OK;
}

hpscd_status hpscd_abort(hpscd_ctx* ctx) {
  if (!ctx) return fail(HPSCD_EINVAL, "ctx is NULL");
  __atomic_store_n(ctx->cancel_h, 1, __ATOMIC_SEQ_CST);
  return HPSCD_OK;
}

}  // extern "C"

// ---------------------------------------------------------------- batched
namespace {

struct BatchPlan {
  std::vector<SysDesc> sd;
  std::vector<WorkItem> items;
  std::vector<int64_t> blk_first;
  int64_t nblk = 0, a_size = 0, y_size = 0, rdn_size = 0, gram_size = 0;
};

hpscd_status validate_batch(int32_t count, const hpscd_sys* sys, const float* Xpool, const float* ypool,
                            const hpscd_opts* o, const float* apool) {
  if (count < 1) return fail(HPSCD_EINVAL, "count must be >= 1");
  if (!sys) return fail(HPSCD_EINVAL, "sys is NULL");
  if (!Xpool || !ypool || !apool) return fail(HPSCD_EINVAL, "NULL pool");
  if (!aligned16(Xpool)) return fail(HPSCD_EINVAL, "Xpool must be 16-byte aligned");
  const int64_t max_m = batched_rows_per_wg(1);  // (every shape holds 8192 rows)
  for (int32_t i = 0; i < count; ++i) {
    const hpscd_sys& s = sys[i];
    if (s.m < 1 || s.n < 1) return fail(HPSCD_EINVAL, "system %d: m and n must be >= 1", i);
    if (s.m > max_m) return fail(HPSCD_EINVAL, "system %d: m=%lld exceeds %lld", i, (long long)s.m, (long long)max_m);
    if (s.ldx < s.m || s.ldx % 4 != 0) return fail(HPSCD_EINVAL, "system %d: need ldx >= m and ldx %% 4 == 0", i);
    if (s.x_off < 0 || s.x_off % 4 != 0) return fail(HPSCD_EINVAL, "system %d: x_off must be >= 0 and %% 4 == 0", i);
    if (s.y_off < 0 || s.a_off < 0) return fail(HPSCD_EINVAL, "system %d: negative offset", i);
    if (!(s.tol >= 0.0) || !std::isfinite(s.tol)) return fail(HPSCD_EINVAL, "system %d: tol must be finite and >= 0", i);
  }
  return validate_opts(o);
}

// Work items in longest-processing-time order: systems that fit one wave are
// grouped as many to an item as the workgroup has waves, by decreasing cost;
// larger systems get a whole workgroup.  The queue hands items out in this
// order.  `code` names the kernel variant (block size and shape).
//
// Cost model: a team's time per block is a latency, nearly independent of
// the rows (measured on the 4096-system batch: about 1.5 us for a one-wave
// team, 2.7 us for a workgroup, over 256 to 8192 rows), so a system costs
// (sweeps + 1) * blocks * t_team.  `sweeps` (optional) are the sweep counts
// the systems took when the batch was tuned; without them every system
// counts one sweep.  Item cost: that of its costliest system.
void plan_batch(int32_t count, const hpscd_sys* sys, int code, int64_t wave_max_m, int hist_len, double tol,
                const std::vector<int32_t>& sweeps, BatchPlan* bp) {
  const int B = batched_block(code);
  bp->sd.resize(count);
  bp->blk_first.resize(count);
  int64_t g = 0, blk = 0;
  for (int32_t i = 0; i < count; ++i) {
    const hpscd_sys& s = sys[i];
    const int64_t nb = (s.n + B - 1) / B;
    bp->sd[i] = SysDesc{s.m, s.n, s.x_off, s.ldx, s.y_off, s.a_off, g, (int64_t)i * hist_len, s.tol > 0.0 ? s.tol : tol};
    bp->blk_first[i] = blk;
    g += nb * B;
    blk += nb;
    bp->a_size = std::max(bp->a_size, s.a_off + s.n);
    bp->y_size = std::max(bp->y_size, s.y_off + s.m);
  }
  bp->nblk = blk;
  bp->rdn_size = g;
  bp->gram_size = g / B * (B * (B - 1) / 2);
  std::vector<int32_t> small, big;
  const int64_t wave_rows = std::min<int64_t>(wave_max_m, batched_rows_per_wave(code));
  for (int32_t i = 0; i < count; ++i) (sys[i].m <= wave_rows ? small : big).push_back(i);
  const bool hint = (int32_t)sweeps.size() == count;
  auto cost = [&](int32_t i, bool wave_team) {
    const double nbi = (double)((sys[i].n + B - 1) / B);
    const double sw = hint ? (double)sweeps[i] + 1.0 : 1.0;
    return sw * nbi * (wave_team ? 1.5 : 2.7) + 1e-9 * (double)sys[i].m;  // (ties: larger first)
  };
  std::sort(small.begin(), small.end(), [&](int32_t a, int32_t b) { return cost(a, true) > cost(b, true); });
  std::sort(big.begin(), big.end(), [&](int32_t a, int32_t b) { return cost(a, false) > cost(b, false); });
  std::vector<std::pair<double, WorkItem>> items;
  for (int32_t i : big) items.push_back({cost(i, false), WorkItem{0, 1, {i}}});
  const int per = std::min<int>(batched_threads(code) / WAVE, (int)(sizeof(WorkItem::sys) / sizeof(int32_t)));
  for (size_t k = 0; k < small.size(); k += per) {
    WorkItem w{1, 0, {}};
    for (int q = 0; q < per && k + q < small.size(); ++q) w.sys[w.count++] = small[k + q];
    items.push_back({cost(small[k], true), w});
  }
  std::stable_sort(items.begin(), items.end(), [](auto& a, auto& b) { return a.first > b.first; });
  bp->items.clear();
  for (auto& it : items) bp->items.push_back(it.second);
}

std::string batch_key(int32_t count, const hpscd_sys* sys) {
  // shape signature: count and a coarse histogram of sizes
  int64_t sm = 0, sn = 0, smn = 0;
  for (int32_t i = 0; i < count; ++i) { sm += sys[i].m; sn += sys[i].n; smn += sys[i].m * sys[i].n; }
  char buf[128];
  snprintf(buf, sizeof buf, "%d:%lld:%lld:%lld", count, (long long)sm, (long long)sn, (long long)smn);
  return buf;
}

// Sizes of the workspace regions of one batched solve.
struct BatchLayout {
  int32_t count = 0;
  int hist_len = 0;
  size_t sys_bytes = 0, item_bytes = 0, blk_bytes = 0;
  size_t i32_n = 0;  // queue[4], ctl[12], sweeps[count], converged[count]
  size_t f64_n = 0;  // ynorm2[count], fnorm2[count]
};

// Plan the batch, size the workspace, and upload the tables (waits for the
// upload: the staging buffer is the context's pinned buffer).
hpscd_status prepare_batch(hpscd_ctx* c, BatchWork& w, int32_t count, const hpscd_sys* sys, bool has_a0,
                           const hpscd_opts* o, int B, int64_t wave_max_m, const std::vector<int32_t>& sweeps,
                           BatchPlan& bp, BatchLayout& L, hipStream_t st) {
  HIP_TRY(hipSetDevice(c->device));
  L.count = count;
  L.hist_len = o->max_sweeps + 1;
  plan_batch(count, sys, B, wave_max_m, L.hist_len, o->tol, sweeps, &bp);
  L.sys_bytes = bp.sd.size() * sizeof(SysDesc);
  L.item_bytes = bp.items.size() * sizeof(WorkItem);
  L.blk_bytes = bp.blk_first.size() * sizeof(int64_t);
  L.i32_n = 16 + 2 * (size_t)count;
  L.f64_n = 2 * (size_t)count;
  hpscd_status rc;
  if ((rc = ensure(w.sys, L.sys_bytes, "sys")) || (rc = ensure(w.items, L.item_bytes, "items")) ||
      (rc = ensure(w.blk, L.blk_bytes, "blk")) || (rc = ensure(w.rdn, (size_t)bp.rdn_size * 8, "rdn")) ||
      (rc = ensure(w.gram, (size_t)std::max<int64_t>(1, bp.gram_size) * 8, "gram")) ||
      (rc = ensure(w.a64, (size_t)bp.a_size * 8, "a64")) ||
      (rc = ensure(w.e0, has_a0 ? (size_t)bp.y_size * 4 : 4, "e0")) ||
      (rc = ensure(w.hist, (size_t)count * L.hist_len * 8, "hist")) || (rc = ensure(w.i32, L.i32_n * 4, "i32")) ||
      (rc = ensure(w.f64, L.f64_n * 8, "f64")))
    return rc;
  const size_t up = L.sys_bytes + L.item_bytes + L.blk_bytes;
  const size_t down = L.i32_n * 4 + L.f64_n * 8 + (size_t)count * L.hist_len * 8;
  if ((rc = c->host_ensure(std::max(up, down) + 64))) return rc;
  char* h = reinterpret_cast<char*>(c->host);
  HIP_TRY(hipStreamSynchronize(st));  // the staging buffer may still feed an earlier copy
  std::memcpy(h, bp.sd.data(), L.sys_bytes);
  std::memcpy(h + L.sys_bytes, bp.items.data(), L.item_bytes);
  std::memcpy(h + L.sys_bytes + L.item_bytes, bp.blk_first.data(), L.blk_bytes);
  HIP_TRY(hipMemcpyAsync(w.sys.p, h, L.sys_bytes, hipMemcpyHostToDevice, st));
  HIP_TRY(hipMemcpyAsync(w.items.p, h + L.sys_bytes, L.item_bytes, hipMemcpyHostToDevice, st));
  HIP_TRY(hipMemcpyAsync(w.blk.p, h + L.sys_bytes + L.item_bytes, L.blk_bytes, hipMemcpyHostToDevice, st));
  HIP_TRY(hipStreamSynchronize(st));
  return HPSCD_OK;
}

// Queue the whole batched solve on `st`: kernels only (no copies, no
// memsets, no host waits), so the sequence can be recorded into a HIP graph.
// Events ev (four, or NULL) bracket setup, sweeps and output.
hpscd_status enqueue_batch(hpscd_ctx* c, BatchWork& w, const BatchPlan& bp, const BatchLayout& L, const float* Xpool,
                           const float* ypool, const float* a0pool, const hpscd_opts* o, int B, float* apool,
                           hipEvent_t* ev, hipStream_t st) {
  const int32_t count = L.count;
  int32_t* i32 = w.i32.as<int32_t>();
  int32_t* queue = i32;
  int32_t* ctl = i32 + 4;
  int32_t* d_sweeps = i32 + 16;
  int32_t* d_conv = d_sweeps + count;
  double* ynorm2 = w.f64.as<double>();
  double* fnorm2 = ynorm2 + count;
  const SysDesc* dsys = w.sys.as<SysDesc>();
  if (ev) HIP_TRY(hipEventRecord(ev[0], st));
  HIP_TRY(launch_fill_i32(i32, (int64_t)L.i32_n, 0, st));
  HIP_TRY(launch_fill_f64(w.hist.as<double>(), (int64_t)count * L.hist_len, std::numeric_limits<double>::quiet_NaN(), st));
  HIP_TRY(launch_a_init(w.a64.as<double>(), a0pool, bp.a_size, st));
  HIP_TRY(launch_residual_batched(Xpool, ypool, dsys, count, nullptr, nullptr, nullptr, ynorm2, st));
  const float* e0 = ypool;
  if (a0pool) {
    HIP_TRY(launch_residual_batched(Xpool, ypool, dsys, count, nullptr, a0pool, w.e0.as<float>(), nullptr, st));
    e0 = w.e0.as<float>();
  }
  HIP_TRY(launch_colgram_batched(Xpool, dsys, count, bp.nblk, w.blk.as<int64_t>(), batched_block(B), w.rdn.as<double>(),
                                 w.gram.as<double>(), ctl + CTL_NONFINITE, st));
  if (ev) HIP_TRY(hipEventRecord(ev[1], st));
  BatchArgs A{};
  A.Xpool = Xpool;
  A.ypool = ypool;
  A.sys = dsys;
  A.items = w.items.as<WorkItem>();
  A.nitems = (int)bp.items.size();
  A.queue = queue;
  A.rdn = w.rdn.as<double>();
  A.gram = w.gram.as<double>();
  A.e0pool = e0;
  A.a64pool = w.a64.as<double>();
  A.hist = w.hist.as<double>();
  A.sweeps = d_sweeps;
  A.converged = d_conv;
  A.max_sweeps = o->max_sweeps;
  A.stop = o->stop;
  A.tol = o->tol;
  A.ynorm2 = ynorm2;
  const int per_cu = batched_max_blocks_per_cu(B);
  if (per_cu <= 0) return fail(HPSCD_EDEVICE, "batched kernel cannot be resident");
  const int grid = std::max(1, std::min(A.nitems, per_cu * c->cus));
  HIP_TRY(launch_batched(B, A, grid, st));
  if (ev) HIP_TRY(hipEventRecord(ev[2], st));
  HIP_TRY(launch_a_out_batched(w.a64.as<double>(), apool, dsys, count, st));
  if (!(o->flags & HPSCD_F_NO_FINAL_CHECK))
    HIP_TRY(launch_residual_batched(Xpool, ypool, dsys, count, nullptr, apool, nullptr, fnorm2, st));
  if (ev) HIP_TRY(hipEventRecord(ev[3], st));
  return HPSCD_OK;
}

// Wait for `st` and copy the per-system results to the host.
hpscd_status collect_batch(hpscd_ctx* c, BatchWork& w, const BatchLayout& L, const hpscd_sys* sys, bool check, int B,
                           int grid, double* hist, int32_t* sweeps_done, int32_t* converged, double* final_rel,
                           hpscd_info* info, hipEvent_t* ev, hipStream_t st) {
  const int32_t count = L.count;
  HIP_TRY(hipStreamSynchronize(st));  // the staging buffer is free once the stream has drained
  char* h = reinterpret_cast<char*>(c->host);
  HIP_TRY(hipMemcpyAsync(h, w.i32.p, L.i32_n * 4, hipMemcpyDeviceToHost, st));
  HIP_TRY(hipMemcpyAsync(h + L.i32_n * 4, w.f64.p, L.f64_n * 8, hipMemcpyDeviceToHost, st));
  if (hist)
    HIP_TRY(hipMemcpyAsync(h + L.i32_n * 4 + L.f64_n * 8, w.hist.p, (size_t)count * L.hist_len * 8,
                           hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  const int32_t* hi = reinterpret_cast<const int32_t*>(h);
  const double* hy = reinterpret_cast<const double*>(h + L.i32_n * 4);
  if (sweeps_done) std::memcpy(sweeps_done, hi + 16, (size_t)count * 4);
  if (converged) std::memcpy(converged, hi + 16 + count, (size_t)count * 4);
  if (final_rel)
    for (int32_t i = 0; i < count; ++i) {
      const double yn = std::sqrt(hy[i]);
      final_rel[i] = check ? (yn > 0 ? std::sqrt(hy[count + i]) / yn : std::sqrt(hy[count + i]))
                           : std::numeric_limits<double>::quiet_NaN();
    }
  if (hist) std::memcpy(hist, h + L.i32_n * 4 + L.f64_n * 8, (size_t)count * L.hist_len * 8);
  if (info) {
    std::memset(info, 0, sizeof *info);
    int64_t swsum = 0, cvsum = 0, cols = 0;
    for (int32_t i = 0; i < count; ++i) {
      swsum += hi[16 + i];
      cvsum += hi[16 + count + i];
      cols += (int64_t)hi[16 + i] * sys[i].n;
    }
    info->sweeps_done = (int32_t)std::min<int64_t>(swsum, INT32_MAX);
    info->converged = (int32_t)cvsum;
    info->cols_done = cols;
    info->block_used = batched_block(B);
    info->team_wgs = grid;
    info->team_threads = batched_threads(B);
    info->sweep_ms = ev ? elapsed(ev[1], ev[2]) : std::numeric_limits<double>::quiet_NaN();
    info->total_ms = ev ? elapsed(ev[0], ev[3]) : std::numeric_limits<double>::quiet_NaN();
    info->final_rel_resid = std::numeric_limits<double>::quiet_NaN();
  }
  if (hi[4 + CTL_NONFINITE]) return fail(HPSCD_ENONFINITE, "a system holds a non-finite value");
  g_err.clear();
  return HPSCD_OK;
}

int batched_grid(hpscd_ctx* c, const BatchPlan& bp, int B) {
  const int per_cu = batched_max_blocks_per_cu(B);
  return std::max(1, std::min((int)bp.items.size(), std::max(1, per_cu) * c->cus));
}

hpscd_status solve_batched(hpscd_ctx* c, int32_t count, const hpscd_sys* sys, const float* Xpool, const float* ypool,
                           const float* a0pool, const hpscd_opts* o, int B, int64_t wave_max_m,
                           const std::vector<int32_t>& hint, float* apool, double* hist, int32_t* sweeps_done,
                           int32_t* converged, double* final_rel, hpscd_info* info, hipStream_t st) {
  BatchPlan bp;
  BatchLayout L;
  hpscd_status rc = prepare_batch(c, c->bw, count, sys, a0pool != nullptr, o, B, wave_max_m, hint, bp, L, st);
  if (rc != HPSCD_OK) return rc;
  if ((rc = enqueue_batch(c, c->bw, bp, L, Xpool, ypool, a0pool, o, B, apool, c->ev, st)) != HPSCD_OK) return rc;
  return collect_batch(c, c->bw, L, sys, !(o->flags & HPSCD_F_NO_FINAL_CHECK), B, batched_grid(c, bp, B), hist,
                       sweeps_done, converged, final_rel, info, c->ev, st);
}

Tuned batched_choice(hpscd_ctx* c, int32_t count, const hpscd_sys* sys, const hpscd_opts* o) {
  auto it = c->tuned.find(batch_key(count, sys));
  Tuned t = it != c->tuned.end() ? it->second : Tuned{1, batched_rows_per_wave(1), {}};
  if (o->block > 0) t.B = o->block + (t.B & kBatchWide);  // (the tuned shape stays)
  // team_threads asks for a workgroup shape: 256 (four waves) or 512 (eight)
  if (o->team_threads == 256) t.B = batched_block(t.B);
  else if (o->team_threads == 512) t.B = batched_block(t.B) + kBatchWide;
  return t;
}

}  // namespace

extern "C" {

hpscd_status hpscd_solve_batched_f32(hpscd_ctx* ctx, int32_t count, const hpscd_sys* sys, const float* Xpool,
                                     const float* ypool, const float* a0pool, const hpscd_opts* opts, float* apool,
                                     double* hist, int32_t* sweeps_done, int32_t* converged,
                                     double* final_rel_resid, hpscd_info* info, void* stream) {
  try {
    hpscd_status rc = validate_batch(count, sys, Xpool, ypool, opts, apool);
    if (rc != HPSCD_OK) return rc;
    if (!ctx) return fail(HPSCD_EINVAL, "ctx is NULL");
    const Tuned t = batched_choice(ctx, count, sys, opts);
    if (!batched_variant_exists(t.B)) return fail(HPSCD_EINVAL, "batched block %d is not built", t.B);
    return solve_batched(ctx, count, sys, Xpool, ypool, a0pool, opts, t.B, t.wave_max_m, t.sweeps, apool, hist,
                         sweeps_done, converged, final_rel_resid, info, (hipStream_t)stream);
  } catch (...) {
    return fail(HPSCD_ENOMEM, "host allocation failure");
  }
}

hpscd_status hpscd_autotune_batched(hpscd_ctx* ctx, int32_t count, const hpscd_sys* sys, const float* Xpool,
                                    const float* ypool, const hpscd_opts* opts, float* apool, void* stream) {
  try {
    hpscd_status rc = validate_batch(count, sys, Xpool, ypool, opts, apool);
    if (rc != HPSCD_OK) return rc;
    if (!ctx) return fail(HPSCD_EINVAL, "ctx is NULL");
    // Candidates: the block size B (columns per reduction round), the
    // workgroup shape (four waves of eight chunks per thread, or eight of
    // four), and the work split (systems small enough for one wave share a
    // workgroup, one per wave, or every system gets a whole workgroup).
    // The first solve records each system's sweep count; every candidate
    // (and every later solve of this batch) orders its work by it.
    std::vector<int32_t> sweeps(count, 0);
    rc = solve_batched(ctx, count, sys, Xpool, ypool, nullptr, opts, 1, batched_rows_per_wave(1), {}, apool,
                       nullptr, sweeps.data(), nullptr, nullptr, nullptr, (hipStream_t)stream);
    if (rc != HPSCD_OK) return rc;
    double best = 1e300;
    Tuned choice{1, batched_rows_per_wave(1), sweeps};
    for (int code : {1, 2, 4, 1 + kBatchWide, 2 + kBatchWide, 4 + kBatchWide}) {
      if (!batched_variant_exists(code)) continue;
      const int B = code;  // (the variant code travels as the block argument)
      for (int64_t split : {(int64_t)batched_rows_per_wave(code), (int64_t)0}) {
        double t = 1e300;
        for (int rep = 0; rep < 2; ++rep) {
          hpscd_info inf;
          rc = solve_batched(ctx, count, sys, Xpool, ypool, nullptr, opts, B, split, sweeps, apool, nullptr,
                             nullptr, nullptr, nullptr, &inf, (hipStream_t)stream);
          if (rc != HPSCD_OK) return rc;
          t = std::min(t, inf.total_ms);
        }
        if (t < best) { best = t; choice.B = B; choice.wave_max_m = split; }
      }
    }
    ctx->tuned[batch_key(count, sys)] = choice;
    g_err.clear();
    return HPSCD_OK;
  } catch (...) {
    return fail(HPSCD_ENOMEM, "host allocation failure");
  }
}

}  // extern "C"

// ------------------------------------------------------- batched graph plan
struct hpscd_batch_plan {
  hpscd_ctx* ctx = nullptr;
  BatchWork w;
  BatchPlan bp;
  BatchLayout L;
  std::vector<hpscd_sys> sys;
  bool check = true;
  int B = 1, grid = 1;
  hipStream_t cap = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

extern "C" {

void hpscd_batched_plan_destroy(hpscd_batch_plan* p) {
  if (!p) return;
  if (p->ctx) (void)hipSetDevice(p->ctx->device);
  if (p->cap) (void)hipStreamSynchronize(p->cap);
  if (p->exec) (void)hipGraphExecDestroy(p->exec);
  if (p->graph) (void)hipGraphDestroy(p->graph);
  if (p->cap) (void)hipStreamDestroy(p->cap);
  p->w.release();
  delete p;
}

hpscd_status hpscd_batched_plan_create(hpscd_ctx* ctx, int32_t count, const hpscd_sys* sys, const float* Xpool,
                                       const float* ypool, const float* a0pool, const hpscd_opts* opts,
                                       float* apool, hpscd_batch_plan** out) {
  if (!out) return fail(HPSCD_EINVAL, "out is NULL");
  *out = nullptr;
  hpscd_batch_plan* p = nullptr;
  try {
    hpscd_status rc = validate_batch(count, sys, Xpool, ypool, opts, apool);
    if (rc != HPSCD_OK) return rc;
    if (!ctx) return fail(HPSCD_EINVAL, "ctx is NULL");
    const Tuned t = batched_choice(ctx, count, sys, opts);
    if (!batched_variant_exists(t.B)) return fail(HPSCD_EINVAL, "batched block %d is not built", t.B);
    HIP_TRY(hipSetDevice(ctx->device));
    p = new hpscd_batch_plan();
    p->ctx = ctx;
    p->sys.assign(sys, sys + count);
    p->check = !(opts->flags & HPSCD_F_NO_FINAL_CHECK);
    p->B = t.B;
    if (hipStreamCreateWithFlags(&p->cap, hipStreamNonBlocking) != hipSuccess) {
      hpscd_batched_plan_destroy(p);
      return fail(HPSCD_EDEVICE, "stream creation failed");
    }
    rc = prepare_batch(ctx, p->w, count, sys, a0pool != nullptr, opts, t.B, t.wave_max_m, t.sweeps, p->bp, p->L,
                       p->cap);
    if (rc != HPSCD_OK) { hpscd_batched_plan_destroy(p); return rc; }
    p->grid = batched_grid(ctx, p->bp, t.B);
    if (hipStreamBeginCapture(p->cap, hipStreamCaptureModeThreadLocal) != hipSuccess) {
      hpscd_batched_plan_destroy(p);
      return fail(HPSCD_EDEVICE, "graph capture could not start");
    }
    rc = enqueue_batch(ctx, p->w, p->bp, p->L, Xpool, ypool, a0pool, opts, t.B, apool, nullptr, p->cap);
    hipGraph_t g = nullptr;
    const hipError_t ec = hipStreamEndCapture(p->cap, &g);
    p->graph = g;
    if (rc != HPSCD_OK) { hpscd_batched_plan_destroy(p); return rc; }
    if (ec != hipSuccess || !g || hipGraphInstantiate(&p->exec, g, nullptr, nullptr, 0) != hipSuccess) {
      hpscd_batched_plan_destroy(p);
      return fail(HPSCD_EDEVICE, "graph capture or instantiation failed");
    }
    *out = p;
    g_err.clear();
    return HPSCD_OK;
  } catch (...) {
    if (p) hpscd_batched_plan_destroy(p);
    return fail(HPSCD_ENOMEM, "host allocation failure");
  }
}

hpscd_status hpscd_batched_plan_launch(hpscd_batch_plan* p, void* stream) {
  if (!p || !p->exec) return fail(HPSCD_EINVAL, "plan is NULL");
  HIP_TRY(hipSetDevice(p->ctx->device));
  HIP_TRY(hipGraphLaunch(p->exec, (hipStream_t)stream));
  return HPSCD_OK;
}

hpscd_status hpscd_batched_plan_results(hpscd_batch_plan* p, double* hist, int32_t* sweeps_done, int32_t* converged,
                                        double* final_rel_resid, hpscd_info* info, void* stream) {
  if (!p) return fail(HPSCD_EINVAL, "plan is NULL");
  try {
    HIP_TRY(hipSetDevice(p->ctx->device));
    return collect_batch(p->ctx, p->w, p->L, p->sys.data(), p->check, p->B, p->grid, hist, sweeps_done, converged,
                         final_rel_resid, info, nullptr, (hipStream_t)stream);
  } catch (...) {
    return fail(HPSCD_ENOMEM, "host allocation failure");
  }
}

}  // extern "C"
