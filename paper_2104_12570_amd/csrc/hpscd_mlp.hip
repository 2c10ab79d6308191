// Multilayer perceptron that predicts a warm start a0 for a parametric family
// of systems (the initial guess of Algorithm 1 is free; a good one saves
// sweeps).  Layers: in -> h1 -> h2 -> out, exact GELU after the two hidden
// layers, linear output; loss = mean over the batch of sum_k (out_k - t_k)^2
// / out; training by Adam.  Everything runs in the kernels below (FP32).
//
// Parameter vector (flat, FP32): W1[h1][in], b1[h1], W2[h2][h1], b2[h2],
// W3[out][h2], b3[out]; W[o][i] is row-major (row o = output unit o).
#include "hpscd.h"
#include "hpscd_device.hpp"
#include "hpscd_internal.hpp"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>

namespace hpscd {
namespace mlp {

constexpr int TM = 64, TN = 64, TK = 16;

// C[i][j] (+)= sum_k A(i,k) B(k,j), A(i,k) = A[i*sai + k*sak], B(k,j) = B[k*sbk + j*sbj],
// C[i][j] at C[i*ldc + j].  Epilogue: + bias[j] (bias_on_col) or + bias[i] (row),
// then optional GELU: Z = C + bias, H = gelu(Z).  accumulate: C += result.
enum Epi : int { EPI_NONE = 0, EPI_BIAS_COL = 1, EPI_BIAS_COL_GELU = 2 };

__device__ inline float gelu(float z) { return 0.5f * z * (1.0f + erff(z * 0.70710678118654752f)); }
__device__ inline float gelu_grad(float z) {
  const float cdf = 0.5f * (1.0f + erff(z * 0.70710678118654752f));
  const float pdf = 0.39894228040143268f * expf(-0.5f * z * z);
  return cdf + z * pdf;
}

__global__ void __launch_bounds__(256) k_gemm(int M, int N, int K, const float* A, int64_t sai, int64_t sak,
                                              const float* Bm, int64_t sbk, int64_t sbj, float* C, int64_t ldc,
                                              const float* bias, int epi, float* Z, int accumulate) {
  __shared__ float As[TK][TM + 1];
  __shared__ float Bs[TK][TN + 1];
  const int tx = threadIdx.x % 16, ty = threadIdx.x / 16;
  const int i0 = blockIdx.y * TM, j0 = blockIdx.x * TN;
  float acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = 0.f;
  for (int k0 = 0; k0 < K; k0 += TK) {
    for (int q = threadIdx.x; q < TK * TM; q += 256) {
      const int kk = q / TM, ii = q % TM;
      const int i = i0 + ii, k = k0 + kk;
      As[kk][ii] = (i < M && k < K) ? A[(int64_t)i * sai + (int64_t)k * sak] : 0.f;
    }
    for (int q = threadIdx.x; q < TK * TN; q += 256) {
      const int kk = q / TN, jj = q % TN;
      const int j = j0 + jj, k = k0 + kk;
      Bs[kk][jj] = (j < N && k < K) ? Bm[(int64_t)k * sbk + (int64_t)j * sbj] : 0.f;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < TK; ++kk) {
      float av[4], bv[4];
#pragma unroll
      for (int a = 0; a < 4; ++a) av[a] = As[kk][ty * 4 + a];
#pragma unroll
      for (int b = 0; b < 4; ++b) bv[b] = Bs[kk][tx * 4 + b];
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = fmaf(av[a], bv[b], acc[a][b]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    const int i = i0 + ty * 4 + a;
    if (i >= M) continue;
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const int j = j0 + tx * 4 + b;
      if (j >= N) continue;
      float v = acc[a][b];
      if (epi != EPI_NONE) v += bias[j];
      const int64_t o = (int64_t)i * ldc + j;
      if (epi == EPI_BIAS_COL_GELU) {
        Z[o] = v;
        v = gelu(v);
      }
      C[o] = accumulate ? C[o] + v : v;
    }
  }
}

static hipError_t gemm(hipStream_t s, int M, int N, int K, const float* A, int64_t sai, int64_t sak, const float* B,
                       int64_t sbk, int64_t sbj, float* C, int64_t ldc, const float* bias = nullptr,
                       int epi = EPI_NONE, float* Z = nullptr, bool accumulate = false) {
  const dim3 grid((unsigned)((N + TN - 1) / TN), (unsigned)((M + TM - 1) / TM));
  hipLaunchKernelGGL(k_gemm, grid, dim3(256), 0, s, M, N, K, A, sai, sak, B, sbk, sbj, C, ldc, bias, epi, Z,
                     accumulate ? 1 : 0);
  return hipGetLastError();
}

// dZ = dH * gelu'(Z), elementwise.
__global__ void k_gelu_back(const float* dH, const float* Z, float* dZ, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) dZ[i] = dH[i] * gelu_grad(Z[i]);
}

// Column sums of a [rows][cols] row-major matrix (bias gradients), fixed order.
__global__ void k_colsum(const float* G, int rows, int cols, float* out) {
  const int j = blockIdx.x;
  float acc = 0.f;
  for (int r = threadIdx.x; r < rows; r += 256) acc += G[(int64_t)r * cols + j];
  __shared__ float ws[4];
  acc = wave_sum(acc);
  if ((threadIdx.x & 63) == 0) ws[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) out[j] = (ws[0] + ws[1]) + (ws[2] + ws[3]);
}

// Output gradient of the loss L = sum_{b,k} (o - t)^2 / (batch * out):
// dO = 2 (o - t) / (batch * out); per-block partial sums of (o - t)^2.
// The target enters standardised per output column k = i mod out:
// (t - mu_k) / sd_k with osc = [mu (out), sd (out)] (mu 0, sd 1 until an
// output scaling is fitted).
__global__ void k_mse(const float* O, const float* Tt, float* dO, int64_t n, float scale, float* part,
                      const float* osc, int out) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  float d = 0.f;
  if (i < n) {
    const int k = (int)(i % out);
    d = O[i] - (Tt[i] - osc[k]) / osc[out + k];
    dO[i] = 2.f * d * scale;
  }
  __shared__ float ws[4];
  float sq = wave_sum(d * d);
  if ((threadIdx.x & 63) == 0) ws[threadIdx.x >> 6] = sq;
  __syncthreads();
  if (threadIdx.x == 0) part[blockIdx.x] = (ws[0] + ws[1]) + (ws[2] + ws[3]);
}

__global__ void k_sum_f32(const float* v, int n, float* out, float scale) {
  float acc = 0.f;
  for (int i = threadIdx.x; i < n; i += 256) acc += v[i];
  __shared__ float ws[4];
  acc = wave_sum(acc);
  if ((threadIdx.x & 63) == 0) ws[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) *out = ((ws[0] + ws[1]) + (ws[2] + ws[3])) * scale;
}

// Network output in target units: y = sd_k * o + mu_k.
__global__ void k_affine_out(const float* O, float* Y, int64_t n, const float* osc, int out) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const int k = (int)(i % out);
  Y[i] = fmaf(osc[out + k], O[i], osc[k]);
}

// Output scaling from targets T[count][out]: per column k the mean and the
// sample standard deviation (two passes, FP64 sums; at least 1e-12; 1 for a
// single row).  One workgroup per column.
__global__ void __launch_bounds__(256) k_colstats(const float* T, int64_t count, int out, float* osc) {
  const int k = blockIdx.x;
  __shared__ double ws[4];
  double acc = 0.0;
  for (int64_t b = threadIdx.x; b < count; b += 256) acc += (double)T[b * out + k];
  double t = wave_sum(acc);
  if ((threadIdx.x & 63) == 0) ws[threadIdx.x >> 6] = t;
  __syncthreads();
  const double mean = ((ws[0] + ws[1]) + (ws[2] + ws[3])) / (double)count;
  __syncthreads();
  acc = 0.0;
  for (int64_t b = threadIdx.x; b < count; b += 256) {
    const double d = (double)T[b * out + k] - mean;
    acc = fma(d, d, acc);
  }
  t = wave_sum(acc);
  if ((threadIdx.x & 63) == 0) ws[threadIdx.x >> 6] = t;
  __syncthreads();
  if (threadIdx.x == 0) {
    const double ss = (ws[0] + ws[1]) + (ws[2] + ws[3]);
    const double sd = count > 1 ? sqrt(ss / (double)(count - 1)) : 1.0;
    osc[k] = (float)mean;
    osc[out + k] = (float)(sd > 1e-12 ? sd : 1e-12);
  }
}

__global__ void k_osc_reset(float* osc, int out) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i < 2 * out) osc[i] = i < out ? 0.f : 1.f;
}

// Adam (Kingma & Ba): m = b1 m + (1-b1) g; v = b2 v + (1-b2) g^2;
// p -= lr * (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps).
__global__ void k_adam(float* p, const float* g, float* m, float* v, int64_t n, float lr, float b1, float b2,
                       float eps, float c1, float c2) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

static inline dim3 g1(int64_t n) { return dim3((unsigned)std::max<int64_t>(1, (n + 255) / 256)); }

// Parameters k0 .. k0+count-1 of the flat vector drawn uniform in
// [-bound, bound): value k of the SplitMix64 stream started at `seed`
// (Steele, Lea and Flood, "Fast splittable pseudorandom number generators",
// 2014: state_k = seed + (k+1)*0x9E3779B97F4A7C15, then the finaliser of
// Stafford's Mix13), its top 53 bits taken as u in [0, 1).
__device__ inline uint64_t splitmix64_at(uint64_t seed, uint64_t k) {
  uint64_t z = seed + (k + 1) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

__global__ void k_init_uniform(float* p, int64_t k0, int64_t count, double bound, uint64_t seed) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= count) return;
  const double u = (double)(splitmix64_at(seed, (uint64_t)(k0 + i)) >> 11) * 0x1.0p-53;
  p[k0 + i] = (float)((2.0 * u - 1.0) * bound);
}

}  // namespace mlp
}  // namespace hpscd

using namespace hpscd;
using namespace hpscd::mlp;

struct hpscd_mlp {
  int dev = 0;
  int in = 0, h1 = 0, h2 = 0, out = 0;
  int64_t np = 0;
  float *p = nullptr, *g = nullptr, *m = nullptr, *v = nullptr;  // params, grads, Adam moments
  int cap = 0;                                                    // batch capacity of the activations
  float *z1 = nullptr, *a1 = nullptr, *z2 = nullptr, *a2 = nullptr, *o = nullptr;
  float *d3 = nullptr, *d2 = nullptr, *d1 = nullptr, *part = nullptr, *loss = nullptr;
  float* host_loss = nullptr;
  float* osc = nullptr;  // output scaling [mu (out), sd (out)]
  int64_t t = 0;  // Adam step count

  float* W1() { return p; }
  float* B1() { return p + (int64_t)h1 * in; }
  float* W2() { return B1() + h1; }
  float* B2() { return W2() + (int64_t)h2 * h1; }
  float* W3() { return B2() + h2; }
  float* B3() { return W3() + (int64_t)out * h2; }
};

namespace {
hpscd_status mfail(hpscd_status st, const char* msg) {
  hpscd::set_last_error(msg);
  return st;
}
#define MLP_TRY(expr)                                                 \
  do {                                                                \
    hipError_t _e = (expr);                                           \
    if (_e != hipSuccess) return mfail(HPSCD_EDEVICE, #expr);          \
  } while (0)

int64_t nparams(int in, int h1, int h2, int out) {
  return (int64_t)h1 * in + h1 + (int64_t)h2 * h1 + h2 + (int64_t)out * h2 + out;
}

hpscd_status ensure_batch(hpscd_mlp* n, int batch) {
  if (batch <= n->cap) return HPSCD_OK;
  float** bufs[] = {&n->z1, &n->a1, &n->z2, &n->a2, &n->o, &n->d3, &n->d2, &n->d1, &n->part};
  for (float** b : bufs)
    if (*b) { (void)hipFree(*b); *b = nullptr; }
  const int64_t H = std::max(n->h1, n->h2);
  const size_t sz[] = {(size_t)batch * n->h1, (size_t)batch * n->h1, (size_t)batch * n->h2, (size_t)batch * n->h2,
                       (size_t)batch * n->out, (size_t)batch * std::max<int64_t>(n->out, H),
                       (size_t)batch * H, (size_t)batch * H, (size_t)(batch * n->out + 255) / 256 + 1};
  for (int k = 0; k < 9; ++k)
    if (hipMalloc(bufs[k], sz[k] * sizeof(float)) != hipSuccess) return mfail(HPSCD_ENOMEM, "activation buffers");
  n->cap = batch;
  return HPSCD_OK;
}

// Forward pass for `batch` rows of x [batch][in]; output into n->o.
hpscd_status forward(hpscd_mlp* n, int batch, const float* x, hipStream_t s) {
  // Z1 = x W1^T + b1: A = x (i=b, k=in), B(k, j) = W1[j][k]
  MLP_TRY(gemm(s, batch, n->h1, n->in, x, n->in, 1, n->W1(), 1, n->in, n->a1, n->h1, n->B1(), EPI_BIAS_COL_GELU,
               n->z1));
  MLP_TRY(gemm(s, batch, n->h2, n->h1, n->a1, n->h1, 1, n->W2(), 1, n->h1, n->a2, n->h2, n->B2(), EPI_BIAS_COL_GELU,
               n->z2));
  MLP_TRY(gemm(s, batch, n->out, n->h2, n->a2, n->h2, 1, n->W3(), 1, n->h2, n->o, n->out, n->B3(), EPI_BIAS_COL));
  return HPSCD_OK;
}

// Gradients of the loss into n->g (and the loss into n->loss).
hpscd_status backward(hpscd_mlp* n, int batch, const float* x, const float* target, hipStream_t s) {
  const int64_t no = (int64_t)batch * n->out;
  const float scale = 1.0f / (float)((int64_t)batch * n->out);
  hipLaunchKernelGGL(k_mse, g1(no), dim3(256), 0, s, n->o, target, n->d3, no, scale, n->part, n->osc, n->out);
  hipLaunchKernelGGL(k_sum_f32, dim3(1), dim3(256), 0, s, n->part, (int)g1(no).x, n->loss, scale);
  float* gW1 = n->g;
  float* gB1 = gW1 + (int64_t)n->h1 * n->in;
  float* gW2 = gB1 + n->h1;
  float* gB2 = gW2 + (int64_t)n->h2 * n->h1;
  float* gW3 = gB2 + n->h2;
  float* gB3 = gW3 + (int64_t)n->out * n->h2;
  // layer 3: dW3[o][j] = sum_b d3[b][o] a2[b][j]; db3 = colsum(d3); dA2 = d3 W3
  MLP_TRY(gemm(s, n->out, n->h2, batch, n->d3, 1, n->out, n->a2, n->h2, 1, gW3, n->h2));
  hipLaunchKernelGGL(k_colsum, dim3(n->out), dim3(256), 0, s, n->d3, batch, n->out, gB3);
  MLP_TRY(gemm(s, batch, n->h2, n->out, n->d3, n->out, 1, n->W3(), n->h2, 1, n->d2, n->h2));
  hipLaunchKernelGGL(k_gelu_back, g1((int64_t)batch * n->h2), dim3(256), 0, s, n->d2, n->z2, n->d2,
                     (int64_t)batch * n->h2);
  // layer 2
  MLP_TRY(gemm(s, n->h2, n->h1, batch, n->d2, 1, n->h2, n->a1, n->h1, 1, gW2, n->h1));
  hipLaunchKernelGGL(k_colsum, dim3(n->h2), dim3(256), 0, s, n->d2, batch, n->h2, gB2);
  MLP_TRY(gemm(s, batch, n->h1, n->h2, n->d2, n->h2, 1, n->W2(), n->h1, 1, n->d1, n->h1));
  hipLaunchKernelGGL(k_gelu_back, g1((int64_t)batch * n->h1), dim3(256), 0, s, n->d1, n->z1, n->d1,
                     (int64_t)batch * n->h1);
  // layer 1
  MLP_TRY(gemm(s, n->h1, n->in, batch, n->d1, 1, n->h1, x, n->in, 1, gW1, n->in));
  hipLaunchKernelGGL(k_colsum, dim3(n->h1), dim3(256), 0, s, n->d1, batch, n->h1, gB1);
  return hipGetLastError() == hipSuccess ? HPSCD_OK : mfail(HPSCD_EDEVICE, "backward launch");
}

hpscd_status check_batch(hpscd_mlp* n, int batch, const void* x) {
  if (!n) return mfail(HPSCD_EINVAL, "mlp is NULL");
  if (batch < 1) return mfail(HPSCD_EINVAL, "batch must be >= 1");
  if (!x) return mfail(HPSCD_EINVAL, "input is NULL");
  return HPSCD_OK;
}

hpscd_status read_loss(hpscd_mlp* n, float* loss_out, hipStream_t s) {
  if (!loss_out) return HPSCD_OK;
  MLP_TRY(hipMemcpyAsync(n->host_loss, n->loss, sizeof(float), hipMemcpyDeviceToHost, s));
  MLP_TRY(hipStreamSynchronize(s));
  *loss_out = *n->host_loss;
  return HPSCD_OK;
}
}  // namespace

extern "C" {

hpscd_status hpscd_mlp_create(hpscd_ctx* ctx, int in, int h1, int h2, int out, uint64_t seed, hpscd_mlp** res) {
  if (!res) return mfail(HPSCD_EINVAL, "out pointer is NULL");
  *res = nullptr;
  if (!ctx) return mfail(HPSCD_EINVAL, "ctx is NULL");
  if (in < 1 || h1 < 1 || h2 < 1 || out < 1 || in > 65536 || h1 > 65536 || h2 > 65536 || out > 65536)
    return mfail(HPSCD_EINVAL, "layer widths must be in [1, 65536]");
  const int device = hpscd::ctx_device(ctx);
  MLP_TRY(hipSetDevice(device));
  hpscd_mlp* n = new hpscd_mlp();
  n->dev = device;
  n->in = in; n->h1 = h1; n->h2 = h2; n->out = out;
  n->np = nparams(in, h1, h2, out);
  for (float** b : {&n->p, &n->g, &n->m, &n->v})
    if (hipMalloc(b, n->np * sizeof(float)) != hipSuccess) { hpscd_mlp_destroy(n); return mfail(HPSCD_ENOMEM, "params"); }
  if (hipMalloc(&n->loss, sizeof(float)) != hipSuccess || hipMalloc(&n->osc, 2 * (size_t)out * sizeof(float)) != hipSuccess ||
      hipHostMalloc(&n->host_loss, sizeof(float), hipHostMallocDefault) != hipSuccess) {
    hpscd_mlp_destroy(n);
    return mfail(HPSCD_ENOMEM, "loss");
  }
  MLP_TRY(hipMemset(n->m, 0, n->np * sizeof(float)));
  MLP_TRY(hipMemset(n->v, 0, n->np * sizeof(float)));
  hipLaunchKernelGGL(k_osc_reset, g1(2 * (int64_t)out), dim3(256), 0, 0, n->osc, out);
  // W and b of each layer uniform in +-1/sqrt(fan_in), in the flat order
  const int fan[3] = {in, h1, h2}, rows[3] = {h1, h2, out};
  int64_t k0 = 0;
  for (int l = 0; l < 3; ++l) {
    const int64_t cnt = (int64_t)rows[l] * fan[l] + rows[l];
    hipLaunchKernelGGL(k_init_uniform, g1(cnt), dim3(256), 0, 0, n->p, k0, cnt, 1.0 / std::sqrt((double)fan[l]), seed);
    k0 += cnt;
  }
  MLP_TRY(hipGetLastError());
  MLP_TRY(hipDeviceSynchronize());
  *res = n;
  return HPSCD_OK;
}

void hpscd_mlp_destroy(hpscd_mlp* n) {
  if (!n) return;
  (void)hipSetDevice(n->dev);
  (void)hipDeviceSynchronize();
  for (float* b : {n->p, n->g, n->m, n->v, n->z1, n->a1, n->z2, n->a2, n->o, n->d3, n->d2, n->d1, n->part, n->loss,
                   n->osc})
    if (b) (void)hipFree(b);
  if (n->host_loss) (void)hipHostFree(n->host_loss);
  delete n;
}

int64_t hpscd_mlp_num_params(const hpscd_mlp* n) { return n ? n->np : 0; }

hpscd_status hpscd_mlp_set_params(hpscd_mlp* n, const float* flat, void* stream) {
  if (!n || !flat) return mfail(HPSCD_EINVAL, "NULL argument");
  MLP_TRY(hipMemcpyAsync(n->p, flat, n->np * sizeof(float), hipMemcpyDeviceToDevice, (hipStream_t)stream));
  MLP_TRY(hipMemsetAsync(n->m, 0, n->np * sizeof(float), (hipStream_t)stream));
  MLP_TRY(hipMemsetAsync(n->v, 0, n->np * sizeof(float), (hipStream_t)stream));
  n->t = 0;
  return HPSCD_OK;
}

hpscd_status hpscd_mlp_get_params(hpscd_mlp* n, float* flat, void* stream) {
  if (!n || !flat) return mfail(HPSCD_EINVAL, "NULL argument");
  MLP_TRY(hipMemcpyAsync(flat, n->p, n->np * sizeof(float), hipMemcpyDeviceToDevice, (hipStream_t)stream));
  return HPSCD_OK;
}

hpscd_status hpscd_mlp_forward(hpscd_mlp* n, int batch, const float* x, float* y, void* stream) {
  hpscd_status rc = check_batch(n, batch, x);
  if (rc != HPSCD_OK) return rc;
  if (!y) return mfail(HPSCD_EINVAL, "output is NULL");
  MLP_TRY(hipSetDevice(n->dev));
  if ((rc = ensure_batch(n, batch)) != HPSCD_OK) return rc;
  hipStream_t s = (hipStream_t)stream;
  if ((rc = forward(n, batch, x, s)) != HPSCD_OK) return rc;
  const int64_t no = (int64_t)batch * n->out;
  hipLaunchKernelGGL(k_affine_out, g1(no), dim3(256), 0, s, n->o, y, no, n->osc, n->out);
  MLP_TRY(hipGetLastError());
  return HPSCD_OK;
}

hpscd_status hpscd_mlp_fit_output_scaling(hpscd_mlp* n, int count, const float* target, void* stream) {
  if (!n || !target) return mfail(HPSCD_EINVAL, "NULL argument");
  if (count < 1) return mfail(HPSCD_EINVAL, "count must be >= 1");
  MLP_TRY(hipSetDevice(n->dev));
  hipLaunchKernelGGL(k_colstats, dim3(n->out), dim3(256), 0, (hipStream_t)stream, target, (int64_t)count, n->out,
                     n->osc);
  MLP_TRY(hipGetLastError());
  return HPSCD_OK;
}

hpscd_status hpscd_mlp_get_output_scaling(hpscd_mlp* n, float* mu_sd, void* stream) {
  if (!n || !mu_sd) return mfail(HPSCD_EINVAL, "NULL argument");
  MLP_TRY(hipMemcpyAsync(mu_sd, n->osc, 2 * (size_t)n->out * sizeof(float), hipMemcpyDeviceToDevice,
                         (hipStream_t)stream));
  return HPSCD_OK;
}

hpscd_status hpscd_mlp_set_output_scaling(hpscd_mlp* n, const float* mu_sd, void* stream) {
  if (!n || !mu_sd) return mfail(HPSCD_EINVAL, "NULL argument");
  MLP_TRY(hipMemcpyAsync(n->osc, mu_sd, 2 * (size_t)n->out * sizeof(float), hipMemcpyDeviceToDevice,
                         (hipStream_t)stream));
  return HPSCD_OK;
}

hpscd_status hpscd_mlp_grads(hpscd_mlp* n, int batch, const float* x, const float* target, float* grad_flat,
                             float* loss_out, void* stream) {
  hpscd_status rc = check_batch(n, batch, x);
  if (rc != HPSCD_OK) return rc;
  if (!target) return mfail(HPSCD_EINVAL, "target is NULL");
  MLP_TRY(hipSetDevice(n->dev));
  if ((rc = ensure_batch(n, batch)) != HPSCD_OK) return rc;
  hipStream_t s = (hipStream_t)stream;
  if ((rc = forward(n, batch, x, s)) != HPSCD_OK) return rc;
  if ((rc = backward(n, batch, x, target, s)) != HPSCD_OK) return rc;
  if (grad_flat) MLP_TRY(hipMemcpyAsync(grad_flat, n->g, n->np * sizeof(float), hipMemcpyDeviceToDevice, s));
  return read_loss(n, loss_out, s);
}

hpscd_status hpscd_mlp_train_step(hpscd_mlp* n, int batch, const float* x, const float* target, float lr,
                                  float* loss_out, void* stream) {
  hpscd_status rc = check_batch(n, batch, x);
  if (rc != HPSCD_OK) return rc;
  if (!target) return mfail(HPSCD_EINVAL, "target is NULL");
  if (!(lr > 0.f) || !std::isfinite(lr)) return mfail(HPSCD_EINVAL, "lr must be positive and finite");
  MLP_TRY(hipSetDevice(n->dev));
  if ((rc = ensure_batch(n, batch)) != HPSCD_OK) return rc;
  hipStream_t s = (hipStream_t)stream;
  if ((rc = forward(n, batch, x, s)) != HPSCD_OK) return rc;
  if ((rc = backward(n, batch, x, target, s)) != HPSCD_OK) return rc;
  n->t += 1;
  const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
  const float c1 = 1.f - (float)std::pow(0.9, (double)n->t);
  const float c2 = 1.f - (float)std::pow(0.999, (double)n->t);
  hipLaunchKernelGGL(k_adam, g1(n->np), dim3(256), 0, s, n->p, n->g, n->m, n->v, n->np, lr, b1, b2, eps, c1, c2);
  MLP_TRY(hipGetLastError());
  return read_loss(n, loss_out, s);
}

}  // extern "C"
