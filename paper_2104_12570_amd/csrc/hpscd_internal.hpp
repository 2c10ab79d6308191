// Host-side declarations shared by the HPSCD translation units.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

struct hpscd_ctx;

namespace hpscd {

// Arguments of one sweep-kernel launch (single system, grid or one workgroup).
struct SolveArgs {
  const void* X;          // column-major m x n, 16-byte aligned columns
  int64_t ldx, m, n;
  const float* e0;        // residual at entry (length m)
  const double* rdn;      // [nb*B] 1/<X_j,X_j> (0 for zero and padding columns)
  const double* gram;     // [nb][B*(B-1)/2] strictly-lower in-block Gram, (l,i) row-major
  const double* minv;     // [nb][B][B] step matrix M = (D+L)^-1 of each block, row-major (B = 16 only)
  double* a64;            // [n] coefficients, accumulated in FP64
  float* e_out;           // [m] residual at exit
  double* hist;           // [max_sweeps+1] ||e||_2 after each complete sweep
  uint64_t* slots;        // grid exchange words [2][B+1][P]
  int32_t* ctl;           // control words (Ctl)
  double* fstat;          // [0] ||e||^2 at exit, [1] last recorded sweep norm
  int64_t* ctl64;         // [C64_COLS] column steps done
  int32_t max_sweeps;
  int32_t stop;
  double tol;
  const double* ynorm2;   // device: ||y||^2
  int64_t check_cols;
  int64_t blk_begin;      // first global block index of this launch
  int64_t blk_end;        // one past the last global block index of this launch
  int32_t P;              // workgroups in the grid (1 for a workgroup team)
  int32_t rows_per_wg;    // rows owned by one workgroup (wide-block kernel; others own T*R*VEC)
  uint64_t timeout_ticks; // bound on any spin-wait (100 MHz ticks)
  uint32_t poll_delay;    // ticks between publishing and the first poll of a grid reduction
  int32_t thr;            // Algorithm 2 block width (wide-block kernel, variant 1)
  const int32_t* order;   // [max_sweeps][n] column order (wide-block kernel, variant 2)
  const int32_t* cancel;  // cancel word in host memory (mapped): non-zero stops the solve at a sweep start
};

// One system of a batch as the batched kernels see it (element offsets).
struct SysDesc {
  int64_t m, n, x_off, ldx, y_off, a_off;
  int64_t g_off;          // offset of this system's rdn/gram region
  int64_t h_off;          // offset of this system's hist region
  double tol;             // stop tolerance of this system
};

// One unit of batched work: a system solved by the whole workgroup, or up to
// eight systems solved by one wave each (as many as the workgroup has waves).
struct WorkItem {
  int32_t mode;           // 0 = workgroup team, 1 = wave teams
  int32_t count;          // systems in the item
  int32_t sys[8];
};

struct BatchArgs {
  const float* Xpool;
  const float* ypool;
  const SysDesc* sys;
  const WorkItem* items;
  int32_t nitems;
  int32_t* queue;          // atomic work counter (zeroed before launch)
  const double* rdn;       // per-system regions at sys.g_off
  const double* gram;      // per-system regions at sys.g_off*(B-1)/2
  const float* e0pool;     // initial residuals (ypool when a0 is absent)
  double* a64pool;         // [a_size]
  double* hist;            // per-system hist regions at sys.h_off
  int32_t* sweeps;         // [count]
  int32_t* converged;      // [count]
  int32_t max_sweeps;
  int32_t stop;
  double tol;
  const double* ynorm2;    // [count] ||y_i||^2
};

// Message returned by hpscd_last_error() on this host thread.
void set_last_error(const char* msg);
// HIP device of a context.
int ctx_device(const struct ::hpscd_ctx* c);

// Kernel launchers (return hipError_t of the launch).
// D: kernel kind (2, 3, 4: k_sweep ring; 5: k_sweep_px; 8: k_sweep_wide).
// V: method variant of the wide-block kernel (0: Algorithm 1, 1: Algorithm 2
// with SolveArgs::thr, 2: column order SolveArgs::order); 0 for other kinds.
hipError_t launch_sweep(int variant_T, int variant_R, int B, bool bf16, bool grid, int D,
                        const SolveArgs& a, hipStream_t s, bool cooperative, int V = 0);
int sweep_max_blocks_per_cu(int T, int R, int B, bool bf16, bool grid, int D, int V = 0);
int sweep_max_workgroups(int T, int R, int B, bool bf16, bool grid, int D, int V = 0);
bool sweep_variant_exists(int T, int R, int B, bool bf16, bool grid, int D, int V = 0);

// Column chain of a short system on one workgroup (kind 9): 16-column FP32
// or 32-column bfloat16 blocks through step matrices in SolveArgs::minv.
bool chain_variant_exists(bool bf16, int B);
int chain_max_rows();
hipError_t launch_chain(bool bf16, int B, const SolveArgs& a, hipStream_t s);
// Reciprocal norms, in-block Gram and step matrices of 32-column blocks.
hipError_t launch_colgram32(const void* X, bool bf16, int64_t ldx, int64_t m, int64_t n, double* rdn, double* gram,
                            double* minv, double* partial, int64_t partial_cap, int32_t* ctl, int64_t* zero_cols,
                            hipStream_t s);
hipError_t launch_colgram_reduce32(const double* partial, int PR, int64_t n, double* rdn, double* gram, int32_t* ctl,
                                   int64_t* zero_cols, hipStream_t s);

hipError_t launch_batched(int B, const BatchArgs& a, int grid, hipStream_t s);
int batched_threads(int code);
// Batched kernel variants are named by a code: the block size (1, 2 or 4),
// plus kBatchWide for workgroups of eight waves with four chunks per thread
// instead of four waves with eight (more column chains resident per CU).
constexpr int kBatchWide = 16;
inline int batched_block(int code) { return code & (kBatchWide - 1); }
int batched_rows_per_wave(int code);
int batched_rows_per_wg(int code);
int batched_max_blocks_per_cu(int code);
bool batched_variant_exists(int code);

// Column statistics: rdn = 1/<X_j,X_j> and the in-block Gram, FP64 sums.
// cross: NULL, or [nb][B*B] receiving <X_{b,l}, X_{b-1,i}> at l*B + i (zero for b = 0).
// B = 16: cross is required and receives each block's step matrix M (see
// k_block_inverse16) instead.
// map: NULL, or (B = 16, FP32 only) the column order of the sweep: block
// position p holds column map[p]; the kernels return at once while
// ctl[CTL_DONE] is set (a solve that has stopped).  thr > 1 (B = 16, FP32):
// the step matrices of Algorithm 2 with blocks of thr columns instead of
// those of Algorithm 1.  zero_cols: NULL or the counter of zero columns.
hipError_t launch_colgram(const void* X, bool bf16, int64_t ldx, int64_t m, int64_t n, int B,
                          double* rdn, double* gram, double* cross, double* partial, int64_t partial_cap,
                          int32_t* ctl, int64_t* zero_cols, hipStream_t s, const int32_t* map = nullptr,
                          int32_t thr = 0);
hipError_t launch_colgram_batched(const float* Xpool, const SysDesc* sys, int32_t count, int64_t nblk_total,
                                  const int64_t* blk_first, int B, double* rdn, double* gram,
                                  int32_t* ctl, hipStream_t s);
// r = y - X[:, :ncols]·a (FP64 accumulation); optional FP32 copy to e_out and
// ||r||^2 into *norm2 (device double).
hipError_t launch_residual(const float* X, int64_t ldx, int64_t m, int64_t ncols, const float* y,
                           const double* a64, const float* a32, float* e_out, double* norm2,
                           double* partial, int64_t partial_cap, const int32_t* skip_if, hipStream_t s,
                           double* e64_out = nullptr);

// X^T v for all n columns (FP64 sums): S row strips of rows_per rows, G
// groups of 64 columns, T tiles of 256 columns; `need` doubles of workspace.
struct XtvPlan {
  int64_t S, G, T, rows_per, need;
};
XtvPlan plan_xtv(int64_t m, int64_t n, int64_t cap);
hipError_t launch_xtv(const float* X, int64_t ldx, int64_t m, int64_t n, const void* v, bool v_f64,
                      const XtvPlan& p, double* partial, double* vnorm, const int32_t* done, hipStream_t s);
// Gradient stop rule after sweep `sweep` on the running residual e (or, with
// init, ||X^T y||^2 from e = y).  ws: workspace of cap doubles.
hipError_t launch_grad_stop(const float* X, int64_t ldx, int64_t m, int64_t n, const float* e, bool init,
                            int32_t sweep, double tol, double* ws, int64_t cap, int32_t* ctl, int64_t* ctl64,
                            double* fstat, double* hist, hipStream_t s);
// One selection step of Algorithm 3 (see hpscd_select.hip).
hipError_t launch_select_step(const float* X, int64_t ldx, int64_t m, int64_t n, double* e, const XtvPlan& p,
                              double* partial, double* vnorm, double* g, double* tscore, int64_t* tidx,
                              const double* rdn, int32_t f, double tol, int32_t* selected, double* a64, int32_t* Jd,
                              double* dad, double* hist, int32_t* ctl, int64_t* step_j, double* step_da,
                              hipStream_t s);
hipError_t launch_norm_f64(const double* e, int64_t m, double* part, double* out, hipStream_t s);
hipError_t launch_to_f64(const float* src, double* dst, int64_t m, hipStream_t s);
hipError_t launch_residual_batched(const float* Xpool, const float* ypool, const SysDesc* sys, int32_t count,
                                   const double* a64pool, const float* a32pool, float* e_out,
                                   double* norm2, hipStream_t s);
hipError_t launch_f32_to_bf16(const float* src, uint16_t* dst, int64_t rows, int64_t cols,
                              int64_t lds, int64_t ldd, hipStream_t s);
hipError_t launch_a_out(const double* a64, float* a, int64_t n, hipStream_t s);
hipError_t launch_a_out_batched(const double* a64pool, float* apool, const SysDesc* sys, int32_t count, hipStream_t s);
hipError_t launch_a_init(double* a64, const float* a0, int64_t n, hipStream_t s);
hipError_t launch_fill_u64(uint64_t* p, int64_t n, uint64_t v, hipStream_t s);
hipError_t launch_fill_i32(int32_t* p, int64_t n, int32_t v, hipStream_t s);
hipError_t launch_fill_f64(double* p, int64_t n, double v, hipStream_t s);
hipError_t launch_copy_f32(const float* src, float* dst, int64_t n, hipStream_t s);
// One pass of 16-byte loads over `bytes` (a multiple of 16) of a buffer; sink:
// grid*256 floats, written only for a NaN sum.
hipError_t launch_read_stream(const void* p, int64_t bytes, int grid, float* sink, hipStream_t s);

}  // namespace hpscd
