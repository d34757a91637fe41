// srmhd_mlp.hip -- training kernels of the learned Newton guess and their C
// ABI entry points (include/srmhd.h): forward with an activation cache, MSE
// loss gradient, backward, Adam on FP32 master weights with BF16 re-
// quantisation.  Every matrix product runs on v_mfma_f32_16x16x16_bf16 with
// FP32 accumulation through one bounds-checked, strided 16x16-tile kernel;
// activations are feature-major ([unit][sample]).
#include "srmhd.h"
#include "srmhd_mlp.hpp"

#include <hip/hip_runtime.h>

#include <cmath>
#include <mutex>

namespace srmhd {

// Message for srmhd_last_error(NULL) (srmhd_api.hip).
void set_call_error(const char* msg);

// Scratch of srmhd_mlp_forward_noalloc: the BF16 activations of one batch
// (input tile X, hidden H1, H2; feature-major, batch padded to 16), for
// batches of up to kNoAllocMaxBatch samples.  Each GPU the library runs on
// holds its own copy until the process ends; host code reaches it only
// through the address hipGetSymbolAddress returns on that device.
constexpr int kNoAllocMaxBatch = 65536;
constexpr size_t kNoAllocBytes = (size_t)(2 * 16 + 2 * 64 + 2 * 64) * kNoAllocMaxBatch;
static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

namespace {

struct GemmArgs {
  int M, N, K;
  const uint16_t* A;
  long long sam, sak;
  const uint16_t* B;
  long long sbk, sbn;
  int mode;  // 0 store, 1 bias + ReLU (z and bf16 h), 2 bias, 3 ReLU-mask of a gradient
  float* Cf;
  long long scm, scn;
  uint16_t* Cb;
  long long sbm, sbn2;
  const float* bias;
  const float* mask;
  long long smm, smn;
};

// C[m][n] = sum_k A(m,k) B(k,n); one wavefront per 16x16 tile of C; elements
// outside M x N x K read as zero and are not written.
__global__ __launch_bounds__(64) void k_gemm(GemmArgs g) {
  const int l = threadIdx.x, col = l & 15, kq = 4 * (l >> 4);
  const int n0 = blockIdx.x * 16, m0 = blockIdx.y * 16;
  f32x4 acc = {0.f, 0.f, 0.f, 0.f};
  const int ma = m0 + col, nb = n0 + col;
  for (int k0 = 0; k0 < g.K; k0 += 16) {
    bf16x4 a, b;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int k = k0 + kq + j;
      a[j] = (ma < g.M && k < g.K) ? (short)g.A[ma * g.sam + k * g.sak] : (short)0;
      b[j] = (nb < g.N && k < g.K) ? (short)g.B[k * g.sbk + nb * g.sbn] : (short)0;
    }
    acc = mfma16(a, b, acc);
  }
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int m = m0 + kq + r, n = n0 + col;
    if (m >= g.M || n >= g.N) continue;
    const float c = acc[r];
    if (g.mode == 0) {
      g.Cf[m * g.scm + n * g.scn] = c;
    } else if (g.mode == 1) {
      const float z = c + g.bias[m];
      if (g.Cf) g.Cf[m * g.scm + n * g.scn] = z;
      g.Cb[m * g.sbm + n * g.sbn2] = f2bf(fmaxf(z, 0.f));
    } else if (g.mode == 2) {
      g.Cf[m * g.scm + n * g.scn] = c + g.bias[m];
    } else {
      const float v = g.mask[m * g.smm + n * g.smn] > 0.f ? c : 0.f;
      if (g.Cf) g.Cf[m * g.scm + n * g.scn] = v;
      if (g.Cb) g.Cb[m * g.sbm + n * g.sbn2] = f2bf(v);
    }
  }
}

void gemm(const GemmArgs& g, hipStream_t s) {
  dim3 grid((g.N + 15) / 16, (g.M + 15) / 16);
  hipLaunchKernelGGL(k_gemm, grid, dim3(64), 0, s, g);
}

GemmArgs gemm_args(int M, int N, int K, const uint16_t* A, long long sam, long long sak,
                   const uint16_t* B, long long sbk, long long sbn) {
  GemmArgs g{};
  g.M = M; g.N = N; g.K = K;
  g.A = A; g.sam = sam; g.sak = sak;
  g.B = B; g.sbk = sbk; g.sbn = sbn;
  return g;
}

// x (batch x 5, row-major) -> X bf16 [5][bp]
__global__ void k_pack_x(const float* x, int batch, int bp, uint16_t* X) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= batch * kMlpIn) return;
  const int b = i / kMlpIn, f = i % kMlpIn;
  X[f * bp + b] = f2bf(x[i]);
}

// dL/dy of the mean squared error over the 2*batch outputs; per-workgroup
// partial sums of (y - t)^2 (fixed order).
__global__ __launch_bounds__(256) void k_loss_grad(const float* y, const float* t, int batch,
                                                   int bp, float* dyf, uint16_t* dyb,
                                                   float* partial) {
  __shared__ float sm[256];
  const int i = blockIdx.x * 256 + threadIdx.x;
  float d2 = 0.f;
  if (i < batch * kMlpOut) {
    const int b = i / kMlpOut, o = i % kMlpOut;
    const float d = y[i] - t[i];
    const float gr = 2.f * d / (float)(batch * kMlpOut);
    dyf[o * bp + b] = gr;
    dyb[o * bp + b] = f2bf(gr);
    d2 = d * d;
  }
  sm[threadIdx.x] = d2;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) sm[threadIdx.x] += sm[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = sm[0];
}

__global__ __launch_bounds__(256) void k_loss_final(const float* partial, int nparts, int nout,
                                                    float* loss) {
  __shared__ float sm[256];
  float a = 0.f;
  for (int i = threadIdx.x; i < nparts; i += 256) a += partial[i];
  sm[threadIdx.x] = a;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) sm[threadIdx.x] += sm[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) *loss = sm[0] / (float)nout;
}

// out[r] = sum_{n < ncols} Z[r * ld + n], one workgroup per row, fixed order
__global__ __launch_bounds__(256) void k_rowsum(const float* Z, long long ld, int ncols,
                                                float* out) {
  __shared__ float sm[256];
  const int r = blockIdx.x;
  float a = 0.f;
  for (int n = threadIdx.x; n < ncols; n += 256) a += Z[r * ld + n];
  sm[threadIdx.x] = a;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) sm[threadIdx.x] += sm[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[r] = sm[0];
}

// Adam (Kingma & Ba 2015) on FP32 master weights; c1 = 1/(1 - b1^t),
// c2 = 1/(1 - b2^t); writes the BF16 copy.
__global__ void k_adam(float* p, uint16_t* w, float* m, float* v, const float* g, int n, float lr,
                       float b1, float b2, float eps, float c1, float c2) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  const float pi = p[i] - lr * (mi * c1) / (sqrtf(vi * c2) + eps);
  p[i] = pi;
  w[i] = f2bf(pi);
}

__global__ void k_quantize(const float* p, uint16_t* w, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) w[i] = f2bf(p[i]);
}

constexpr int kLossParts = 4096;

size_t al(size_t x) { return (x + 255) / 256 * 256; }

// Activation cache, feature-major, batch padded to bp = ceil16(batch).
struct Cache {
  uint16_t *X, *H1, *H2, *dYb, *dZ2b, *dZ1b;
  float *Z1, *Z2, *dYf, *dZ2f, *dZ1f, *part;
  size_t bytes;
};

Cache cache_of(void* base, int batch) {
  const size_t bp = (size_t)((batch + 15) / 16 * 16);
  char* p = (char*)base;
  size_t o = 0;
  Cache c;
  auto take = [&](size_t b) { char* r = p ? p + o : nullptr; o += al(b); return r; };
  c.X = (uint16_t*)take(2 * 16 * bp);
  c.Z1 = (float*)take(4 * kMlpH * bp);
  c.H1 = (uint16_t*)take(2 * kMlpH * bp);
  c.Z2 = (float*)take(4 * kMlpH * bp);
  c.H2 = (uint16_t*)take(2 * kMlpH * bp);
  c.dYb = (uint16_t*)take(2 * 16 * bp);
  c.dYf = (float*)take(4 * kMlpOut * bp);
  c.dZ2f = (float*)take(4 * kMlpH * bp);
  c.dZ2b = (uint16_t*)take(2 * kMlpH * bp);
  c.dZ1f = (float*)take(4 * kMlpH * bp);
  c.dZ1b = (uint16_t*)take(2 * kMlpH * bp);
  c.part = (float*)take(4 * kLossParts);
  c.bytes = o;
  return c;
}

int check() { return hipGetLastError() == hipSuccess ? SRMHD_OK : SRMHD_E_HIP; }

bool batch_ok(int batch) { return batch > 0 && batch <= kLossParts * 256 / kMlpOut; }

// Device address of `scratch` on each device, looked up once per device
// (with that device current) at the first no-alloc call there.
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

int scratch_of_current_device(void** out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return SRMHD_E_HIP;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return SRMHD_E_HIP;
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return SRMHD_OK;
}

// The three network layers of one forward pass: x (batch x 5) -> X -> H1 ->
// H2 -> y (batch x 2).  Z1, Z2 (the FP32 pre-activations, kept for the
// backward pass) are written when non-null.
void forward_layers(const float* params, const uint16_t* w_bf16, const float* x, float* y,
                    uint16_t* X, float* Z1, uint16_t* H1, float* Z2, uint16_t* H2, int batch,
                    hipStream_t s) {
  const long long bp = (batch + 15) / 16 * 16;
  hipLaunchKernelGGL(k_pack_x, dim3((batch * kMlpIn + 255) / 256), dim3(256), 0, s, x, batch,
                     (int)bp, X);
  GemmArgs g = gemm_args(kMlpH, batch, kMlpIn, w_bf16 + kOffW1, kMlpIn, 1, X, bp, 1);
  g.mode = 1; g.Cf = Z1; g.scm = bp; g.scn = 1; g.Cb = H1; g.sbm = bp; g.sbn2 = 1;
  g.bias = params + kOffB1;
  gemm(g, s);
  g = gemm_args(kMlpH, batch, kMlpH, w_bf16 + kOffW2, kMlpH, 1, H1, bp, 1);
  g.mode = 1; g.Cf = Z2; g.scm = bp; g.scn = 1; g.Cb = H2; g.sbm = bp; g.sbn2 = 1;
  g.bias = params + kOffB2;
  gemm(g, s);
  g = gemm_args(kMlpOut, batch, kMlpH, w_bf16 + kOffW3, kMlpH, 1, H2, bp, 1);
  g.mode = 2; g.Cf = y; g.scm = 1; g.scn = kMlpOut; g.bias = params + kOffB3;
  gemm(g, s);
}

}  // namespace
}  // namespace srmhd

using namespace srmhd;

extern "C" {

size_t srmhd_mlp_cache_bytes(int batch) {
  if (!batch_ok(batch)) return 0;
  return cache_of(nullptr, batch).bytes;
}

int srmhd_mlp_quantize(const float* params, uint16_t* w_bf16, int n, void* stream) {
  if (!params || !w_bf16 || n <= 0) return SRMHD_E_INVAL;
  hipLaunchKernelGGL(k_quantize, dim3((n + 255) / 256), dim3(256), 0, (hipStream_t)stream, params,
                     w_bf16, n);
  return check();
}

int srmhd_mlp_forward(const float* params, const uint16_t* w_bf16, const float* x, float* y,
                      void* cache, int batch, void* stream) {
  if (!params || !w_bf16 || !x || !y || !cache || !batch_ok(batch)) return SRMHD_E_INVAL;
  if (((uintptr_t)cache) % 256) return SRMHD_E_INVAL;
  const Cache c = cache_of(cache, batch);
  forward_layers(params, w_bf16, x, y, c.X, c.Z1, c.H1, c.Z2, c.H2, batch, (hipStream_t)stream);
  return check();
}

int srmhd_mlp_forward_noalloc(const float* params, const uint16_t* w_bf16, const float* x,
                              float* y, int batch, void* stream) {
  if (!params || !w_bf16 || !x || !y) {
    set_call_error("mlp_forward_noalloc: a pointer is NULL");
    return SRMHD_E_INVAL;
  }
  if (batch < 1 || batch > kNoAllocMaxBatch) {
    set_call_error("mlp_forward_noalloc: batch must be in 1..65536 (the size of the "
                         "library's static scratch)");
    return SRMHD_E_INVAL;
  }
  void* base = nullptr;
  if (scratch_of_current_device(&base) != SRMHD_OK) {
    set_call_error("mlp_forward_noalloc: hipGetSymbolAddress of the scratch failed");
    return SRMHD_E_HIP;
  }
  // X | H1 | H2, each 256-byte aligned (bp * 2 bytes is a multiple of 32)
  const size_t bp = (size_t)((batch + 15) / 16 * 16);
  uint16_t* X = (uint16_t*)base;
  uint16_t* H1 = X + al(2 * 16 * bp) / 2;
  uint16_t* H2 = H1 + al(2 * kMlpH * bp) / 2;
  forward_layers(params, w_bf16, x, y, X, nullptr, H1, nullptr, H2, batch, (hipStream_t)stream);
  return check();
}

int srmhd_mlp_loss_grad(const float* y, const float* t, void* cache, float* loss, int batch,
                        void* stream) {
  if (!y || !t || !cache || !loss || !batch_ok(batch)) return SRMHD_E_INVAL;
  hipStream_t s = (hipStream_t)stream;
  const Cache c = cache_of(cache, batch);
  const int bp = (batch + 15) / 16 * 16;
  const int nblk = (batch * kMlpOut + 255) / 256;
  hipLaunchKernelGGL(k_loss_grad, dim3(nblk), dim3(256), 0, s, y, t, batch, bp, c.dYf, c.dYb,
                     c.part);
  hipLaunchKernelGGL(k_loss_final, dim3(1), dim3(256), 0, s, c.part, nblk, batch * kMlpOut, loss);
  return check();
}

int srmhd_mlp_backward(const uint16_t* w_bf16, void* cache, float* grad, int batch, void* stream) {
  if (!w_bf16 || !cache || !grad || !batch_ok(batch)) return SRMHD_E_INVAL;
  hipStream_t s = (hipStream_t)stream;
  const Cache c = cache_of(cache, batch);
  const long long bp = (batch + 15) / 16 * 16;
  // layer 3: dW3 = dY H2^T, db3 = sum dY, dZ2 = (W3^T dY) * (Z2 > 0)
  GemmArgs g = gemm_args(kMlpOut, kMlpH, batch, c.dYb, bp, 1, c.H2, 1, bp);
  g.mode = 0; g.Cf = grad + kOffW3; g.scm = kMlpH; g.scn = 1;
  gemm(g, s);
  hipLaunchKernelGGL(k_rowsum, dim3(kMlpOut), dim3(256), 0, s, c.dYf, bp, batch, grad + kOffB3);
  g = gemm_args(kMlpH, batch, kMlpOut, w_bf16 + kOffW3, 1, kMlpH, c.dYb, bp, 1);
  g.mode = 3; g.mask = c.Z2; g.smm = bp; g.smn = 1;
  g.Cf = c.dZ2f; g.scm = bp; g.scn = 1; g.Cb = c.dZ2b; g.sbm = bp; g.sbn2 = 1;
  gemm(g, s);
  // layer 2: dW2 = dZ2 H1^T, db2 = sum dZ2, dZ1 = (W2^T dZ2) * (Z1 > 0)
  g = gemm_args(kMlpH, kMlpH, batch, c.dZ2b, bp, 1, c.H1, 1, bp);
  g.mode = 0; g.Cf = grad + kOffW2; g.scm = kMlpH; g.scn = 1;
  gemm(g, s);
  hipLaunchKernelGGL(k_rowsum, dim3(kMlpH), dim3(256), 0, s, c.dZ2f, bp, batch, grad + kOffB2);
  g = gemm_args(kMlpH, batch, kMlpH, w_bf16 + kOffW2, 1, kMlpH, c.dZ2b, bp, 1);
  g.mode = 3; g.mask = c.Z1; g.smm = bp; g.smn = 1;
  g.Cf = c.dZ1f; g.scm = bp; g.scn = 1; g.Cb = c.dZ1b; g.sbm = bp; g.sbn2 = 1;
  gemm(g, s);
  // layer 1: dW1 = dZ1 X^T, db1 = sum dZ1
  g = gemm_args(kMlpH, kMlpIn, batch, c.dZ1b, bp, 1, c.X, 1, bp);
  g.mode = 0; g.Cf = grad + kOffW1; g.scm = kMlpIn; g.scn = 1;
  gemm(g, s);
  hipLaunchKernelGGL(k_rowsum, dim3(kMlpH), dim3(256), 0, s, c.dZ1f, bp, batch, grad + kOffB1);
  return check();
}

int srmhd_mlp_adam(float* params, uint16_t* w_bf16, float* m, float* v, const float* grad, int n,
                   float lr, float beta1, float beta2, float eps, int t, void* stream) {
  if (!params || !w_bf16 || !m || !v || !grad || n <= 0 || t < 1) return SRMHD_E_INVAL;
  if (!(lr > 0.f) || !(beta1 >= 0.f && beta1 < 1.f) || !(beta2 >= 0.f && beta2 < 1.f) ||
      !(eps > 0.f))
    return SRMHD_E_INVAL;
  const float c1 = (float)(1.0 / (1.0 - std::pow((double)beta1, t)));
  const float c2 = (float)(1.0 / (1.0 - std::pow((double)beta2, t)));
  hipLaunchKernelGGL(k_adam, dim3((n + 255) / 256), dim3(256), 0, (hipStream_t)stream, params,
                     w_bf16, m, v, grad, n, lr, beta1, beta2, eps, c1, c2);
  return check();
}

}  // extern "C"
