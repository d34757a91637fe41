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

// Two floats to a packed pair of BF16 (round to nearest even; one
// v_cvt_pk_bf16_f32 on gfx950), low half = a.
typedef __bf16 bf16x2v __attribute__((ext_vector_type(2)));
typedef unsigned u32x2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ unsigned pack_bf16(float a, float b) {
  bf16x2v v;
  v[0] = (__bf16)a;
  v[1] = (__bf16)b;
  return __builtin_bit_cast(unsigned, v);
}

// bias + ReLU of an MFMA accumulator tile, packed to the next layer's BF16
// operand
__device__ __forceinline__ bf16x4 relu_bf16(f32x4 acc, f32x4 bias) {
  u32x2 w;
  w[0] = pack_bf16(fmaxf(acc[0] + bias[0], 0.f), fmaxf(acc[1] + bias[1], 0.f));
  w[1] = pack_bf16(fmaxf(acc[2] + bias[2], 0.f), fmaxf(acc[3] + bias[3], 0.f));
  return __builtin_bit_cast(bf16x4, w);
}

// Four consecutive BF16 parameters (8-byte aligned) as an MFMA operand.
__device__ __forceinline__ bf16x4 load_bf16x4(const uint16_t* p) {
  return *reinterpret_cast<const bf16x4*>(p);
}

// The same features for inference: the ratios in FP64, the logarithms and
// the square root in FP32 (the network sees them rounded to BF16).
__device__ __forceinline__ void mlp_features_f32(double D, double S2, double B2, double tau,
                                                 double U, float* f) {
  const double iu = 1.0 / U;
  f[0] = __logf((float)(U / D));
  f[1] = sqrtf((float)S2) * (float)iu;
  f[2] = (float)(B2 * iu);
  f[3] = (float)(tau * tau / (S2 * B2 + 1e-300));
  f[4] = __logf((float)D);
}

// One wavefront evaluates the network for its 64 lanes' cells.  `feat` are
// the raw features of this lane's cell; `lx` (64*16 bf16, 8-byte aligned) and
// `ly` (64*2 f32) are this wavefront's LDS scratch.  Must be called by all 64
// lanes (MFMA is wavefront-wide); `bar` orders the LDS hand-offs (a
// workgroup barrier).  Layer-2 weights are read as 8-byte vectors (they stay
// in the L1 cache); activations are rounded to BF16 by the hardware pack
// conversion.
template <typename Barrier>
__device__ __forceinline__ void mlp_wave(const MlpDev& m, const float* feat, uint16_t* lx, float* ly,
                                         float* out, Barrier bar) {
  const int l = threadIdx.x & 63;
  const int col = l & 15, kq = 4 * (l >> 4);
  float z[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) z[k] = k < kMlpIn ? (feat[k] - m.fmean[k]) * m.finv[k] : 0.f;
  unsigned* lx32 = reinterpret_cast<unsigned*>(lx);
#pragma unroll
  for (int k = 0; k < 4; ++k) lx32[l * 8 + k] = pack_bf16(z[2 * k], z[2 * k + 1]);
#pragma unroll
  for (int k = 4; k < 8; ++k) lx32[l * 8 + k] = 0u;
  bar();
  bf16x4 a1[4], a3[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) {
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int k = kq + j;
      a1[t][j] = k < kMlpIn ? (short)m.w[kOffW1 + (16 * t + col) * kMlpIn + k] : (short)0;
      a3[t][j] = col < kMlpOut ? (short)m.w[kOffW3 + col * kMlpH + 16 * t + kq + j] : (short)0;
    }
  }
  const float b30 = m.p[kOffB3 + 0], b31 = m.p[kOffB3 + 1];
  const uint16_t* w2 = m.w + kOffW2 + col * kMlpH + kq;
  // hidden-layer biases of this lane's four output rows, re-read from the
  // L1 cache per block (16-byte aligned) rather than held in registers
  const f32x4* bias1 = reinterpret_cast<const f32x4*>(m.p + kOffB1 + kq);
  const f32x4* bias2 = reinterpret_cast<const f32x4*>(m.p + kOffB2 + kq);
#pragma unroll 1
  for (int nb = 0; nb < 4; ++nb) {
    const bf16x4 x = *reinterpret_cast<const bf16x4*>(&lx[(16 * nb + col) * 16 + kq]);
    bf16x4 h1[4], h2[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      f32x4 acc = {0.f, 0.f, 0.f, 0.f};
      acc = mfma16(a1[t], x, acc);
      h1[t] = relu_bf16(acc, bias1[4 * t]);
    }
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int kt = 0; kt < 4; ++kt)
        acc = mfma16(load_bf16x4(w2 + 16 * t * kMlpH + 16 * kt), h1[kt], acc);
      h2[t] = relu_bf16(acc, bias2[4 * t]);
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
