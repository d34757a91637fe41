// srmhd_mlp.hpp -- the learned Newton guess: a 5 -> 64 -> 64 -> 2 ReLU network
// with BF16 weights and FP32 accumulation on the CDNA matrix cores
// (v_mfma_f32_16x16x16_bf16).  Device helpers shared by the inversion kernel
// (in-wavefront inference) and the training kernels.
//
// Parameter vector (FP32 master and its BF16 copy share the layout; rows are
// output units): W1[64][5] | b1[64] | W2[64][64] | b2[64] | W3[2][64] | b3[2].
// Features of a conserved state, the invariants the one-unknown inversion
// depends on: log(U/D), |S|/U, B^2/U, tau^2/(S^2 B^2 + 1e-300), log D, with
// tau = S.B.  Outputs: standardised log(p/D) and log Gamma.
//
// MFMA 16x16x16 lane layout (64 lanes, l = lane): A[m][k] holds m = l%16,
// k = 4(l/16)+j; B[k][n] holds n = l%16, k = 4(l/16)+j; D[m][n] holds n = l%16,
// m = 4(l/16)+r (j, r = 0..3).  Activations are kept feature-major (feature =
// k of the next layer, cell = n), so a layer's D tile over output units
// 16t..16t+15 is, element for element, the next layer's B operand for the
// K block t: no transposes between layers.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace srmhd {

constexpr int kMlpIn = 5, kMlpH = 64, kMlpOut = 2;
constexpr int kOffW1 = 0, kOffB1 = 320, kOffW2 = 384, kOffB2 = 4480, kOffW3 = 4544,
              kOffB3 = 4672, kMlpNParam = 4674;

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// float -> bfloat16 bits, round to nearest even (finite inputs)
__device__ __forceinline__ uint16_t f2bf(float f) {
  const uint32_t u = __float_as_uint(f);
  return (uint16_t)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
}

__device__ __forceinline__ float bf2f(uint16_t b) { return __uint_as_float(((uint32_t)b) << 16); }

__device__ __forceinline__ f32x4 mfma16(bf16x4 a, bf16x4 b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}

struct MlpDev {
  const uint16_t* w;  // BF16 parameter vector (weights used)
  const float* p;     // FP32 parameter vector (biases used)
  float fmean[kMlpIn], finv[kMlpIn];  // feature standardisation: (f - mean) * inv
  float omean[kMlpOut], ostd[kMlpOut];  // output de-standardisation
};

// The five invariant features of (D, S^2, B^2, tau, U), in FP64.
__device__ __forceinline__ void mlp_features(double D, double S2, double B2, double tau, double U,
                                             double* f) {
  f[0] = log(U / D);
  f[1] = sqrt(S2) / U;
  f[2] = B2 / U;
  f[3] = tau * tau / (S2 * B2 + 1e-300);
  f[4] = log(D);
}

// One wavefront evaluates the network for its 64 lanes' cells.  `feat` are
// the raw features of this lane's cell; `lx` (64*16 bf16) and `ly` (64*2 f32)
// are this wavefront's LDS scratch.  Must be called by all 64 lanes (MFMA is
// wavefront-wide); `bar` orders the LDS hand-offs (a workgroup barrier).
template <typename Barrier>
__device__ __forceinline__ void mlp_wave(const MlpDev& m, const float* feat, uint16_t* lx, float* ly,
                                         float* out, Barrier bar) {
  const int l = threadIdx.x & 63;
  const int col = l & 15, kq = 4 * (l >> 4);
#pragma unroll
  for (int k = 0; k < 16; ++k) {
    const float v = k < kMlpIn ? (feat[k] - m.fmean[k]) * m.finv[k] : 0.f;
    lx[l * 16 + k] = f2bf(v);
  }
  bar();
  bf16x4 a1[4], a3[4];
  f32x4 b1[4], b2[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) {
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int k = kq + j;
      a1[t][j] = k < kMlpIn ? (short)m.w[kOffW1 + (16 * t + col) * kMlpIn + k] : (short)0;
      a3[t][j] = col < kMlpOut ? (short)m.w[kOffW3 + col * kMlpH + 16 * t + kq + j] : (short)0;
      b1[t][j] = m.p[kOffB1 + 16 * t + kq + j];
      b2[t][j] = m.p[kOffB2 + 16 * t + kq + j];
    }
  }
  const float b30 = m.p[kOffB3 + 0], b31 = m.p[kOffB3 + 1];
#pragma unroll 1
  for (int nb = 0; nb < 4; ++nb) {
    bf16x4 x;
#pragma unroll
    for (int j = 0; j < 4; ++j) x[j] = (short)lx[(16 * nb + col) * 16 + kq + j];
    bf16x4 h1[4], h2[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      f32x4 acc = {0.f, 0.f, 0.f, 0.f};
      acc = mfma16(a1[t], x, acc);
#pragma unroll
      for (int r = 0; r < 4; ++r) h1[t][r] = (short)f2bf(fmaxf(acc[r] + b1[t][r], 0.f));
    }
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int kt = 0; kt < 4; ++kt) {
        bf16x4 a2;
#pragma unroll
        for (int j = 0; j < 4; ++j) a2[j] = (short)m.w[kOffW2 + (16 * t + col) * kMlpH + 16 * kt + kq + j];
        acc = mfma16(a2, h1[kt], acc);
      }
#pragma unroll
      for (int r = 0; r < 4; ++r) h2[t][r] = (short)f2bf(fmaxf(acc[r] + b2[t][r], 0.f));
    }
    f32x4 y = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int kt = 0; kt < 4; ++kt) y = mfma16(a3[kt], h2[kt], y);
    if (l < 16) {
      ly[(16 * nb + l) * 2 + 0] = y[0] + b30;
      ly[(16 * nb + l) * 2 + 1] = y[1] + b31;
    }
  }
  bar();
  out[0] = ly[l * 2 + 0] * m.ostd[0] + m.omean[0];
  out[1] = ly[l * 2 + 1] * m.ostd[1] + m.omean[1];
}

}  // namespace srmhd
