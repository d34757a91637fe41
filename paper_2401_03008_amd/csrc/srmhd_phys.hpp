// srmhd_phys.hpp -- point physics and stencil functions of the SRMHD stage,
// as inlined device code templated on the arithmetic type T (double, or float
// for the reconstruction and face fluxes of the mixed form).
//
// Sec. 2 of arXiv 2401.03008 fixes the ideal SRMHD system: D = rho Gamma,
// S = rho h Gamma^2 v + E x B, U = rho h Gamma^2 - p + (E^2 + B^2)/2,
// W_ij = rho h Gamma^2 v_i v_j - E_i E_j - B_i B_j + p_tot delta_ij,
// E = -v x B, h = 1 + g/(g-1) p/rho.  Everything else below is a published
// method named in place (the paper gives no formulas for them).
#pragma once

#include <hip/hip_runtime.h>

#include "srmhd_kernels.hpp"

namespace srmhd {

// Primitive state in a face-normal frame: n is the face normal, (n, t1, t2)
// is a cyclic permutation of (x, y, z), so cross products keep their form.
template <typename T>
struct FaceState {
  T rho, vn, vt1, vt2, p, bn, bt1, bt2;
};

// Conserved variables and normal fluxes of the five fluid components, and the
// fast-speed bounds, for one face state.
template <typename T>
struct FaceEval {
  T u[5];  // D, S_n, S_t1, S_t2, U
  T f[5];  // normal fluxes of the same
  T lm, lp;
};

template <typename T>
__device__ __forceinline__ T sq(T a) { return a * a; }

// 1/x for the face-physics and edge-formula denominators (finite, positive,
// of moderate size: no zero, infinity or denormal handling).  FP64: the
// hardware reciprocal estimate refined by two Newton-Raphson steps for
// f(r) = 1/r - x, r <- r + r (1 - x r), each of which squares the relative
// error; FP32: the hardware reciprocal (within 1 ulp).
__device__ __forceinline__ double recip(double x) {
  double r = __builtin_amdgcn_rcp(x);
  double e = __builtin_fma(-x, r, 1.0);
  r = __builtin_fma(r, e, r);
  e = __builtin_fma(-x, r, 1.0);
  return __builtin_fma(r, e, r);
}
__device__ __forceinline__ float recip(float x) { return __builtin_amdgcn_rcpf(x); }

// Sec. 2 conserved variables and normal fluxes; fast speeds from the quadratic
// bound of Del Zanna et al. (2003): w^2 = c_s^2 + v_A^2 - c_s^2 v_A^2 with
// c_s^2 = g p/(rho h), v_A^2 = b^2/(rho h + b^2), b^2 = B^2/Gamma^2 + (v.B)^2.
template <typename T>
__device__ __forceinline__ void face_eval(const FaceState<T>& s, T g, T g1,
                                          FaceEval<T>& e) {
  const T v2 = s.vn * s.vn + s.vt1 * s.vt1 + s.vt2 * s.vt2;
  const T one_m_v2 = T(1) - v2;
  const T rhoh = s.rho + g1 * s.p;
  // E = -v x B in the (n, t1, t2) frame
  const T En = s.vt2 * s.bt1 - s.vt1 * s.bt2;
  const T Et1 = s.vn * s.bt2 - s.vt2 * s.bn;
  const T Et2 = s.vt1 * s.bn - s.vn * s.bt1;
  const T E2 = En * En + Et1 * Et1 + Et2 * Et2;
  const T B2 = s.bn * s.bn + s.bt1 * s.bt1 + s.bt2 * s.bt2;
  const T vB = s.vn * s.bn + s.vt1 * s.bt1 + s.vt2 * s.bt2;
  const T b2 = B2 * one_m_v2 + vB * vB;  // comoving field strength squared
  // one division for 1/(1 - v^2), 1/(rho h) and 1/(rho h + b^2)
  const T q1 = rhoh * (rhoh + b2);
  const T r = recip(one_m_v2 * q1);
  const T lor2 = q1 * r;                       // 1/(1 - v^2)
  const T inv_rhoh = one_m_v2 * (rhoh + b2) * r;
  const T inv_rhohb = one_m_v2 * rhoh * r;
  const T W = rhoh * lor2;
  const T pm = T(0.5) * (E2 + B2);
  const T D = s.rho * sqrt(lor2);
  const T Sn = W * s.vn + (Et1 * s.bt2 - Et2 * s.bt1);
  e.u[0] = D;
  e.u[1] = Sn;
  e.u[2] = W * s.vt1 + (Et2 * s.bn - En * s.bt2);
  e.u[3] = W * s.vt2 + (En * s.bt1 - Et1 * s.bn);
  e.u[4] = W - s.p + pm;
  const T Wvn = W * s.vn;
  e.f[0] = D * s.vn;
  e.f[1] = Wvn * s.vn - En * En - s.bn * s.bn + (s.p + pm);
  e.f[2] = Wvn * s.vt1 - Et1 * En - s.bt1 * s.bn;
  e.f[3] = Wvn * s.vt2 - Et2 * En - s.bt2 * s.bn;
  e.f[4] = Sn;
  // fast-speed bound
  const T cs2 = g * s.p * inv_rhoh;
  const T va2 = b2 * inv_rhohb;
  const T w2 = cs2 + va2 - cs2 * va2;
  const T den = T(1) - v2 * w2;
  const T inv_den = recip(den);
  T disc = w2 * one_m_v2 * (den - s.vn * s.vn * (T(1) - w2));
  disc = disc > T(0) ? disc : T(0);
  const T sqd = sqrt(disc);
  const T a = s.vn * (T(1) - w2);
  e.lp = (a + sqd) * inv_den;
  e.lm = (a - sqd) * inv_den;
}

template <typename T>
__device__ __forceinline__ bool face_state_ok(const FaceState<T>& s) {
  const T v2 = s.vn * s.vn + s.vt1 * s.vt1 + s.vt2 * s.vt2;
  return s.rho > T(0) && s.p > T(0) && v2 < T(1);
}

// ---------------------------------------------------------------- MP5 (REC)
// Suresh & Huynh (1997) monotonicity-preserving fifth-order interface values,
// alpha = 4, eps = 1e-10.  Left state at x_{i+1/2} (centre v_i): the
// unlimited fifth-order value v_or is kept when (v_or - v_i)(v_or - v_MP) <=
// eps, v_MP = v_i + minmod(v_{i+1} - v_i, alpha (v_i - v_{i-1})); otherwise it
// is limited to [v_min, v_max], the bounds built from v_i, v_{i+1}, the upper
// limit v_UL = v_i + alpha (v_i - v_{i-1}), the median v_MD = (v_i +
// v_{i+1})/2 - d^{M4}_{i+1/2}/2 and the large-curvature value v_LC = v_i +
// (v_i - v_{i-1})/2 + (4/3) d^{M4}_{i-1/2}, with d^{M4} the minmod4 of the
// neighbouring second differences.  The right state is the mirror image
// (centre v_{i+1}, stencil reversed).

// minmod(a, b) = (sgn a + sgn b)/2 * min(|a|, |b|) and
// minmod4(a, b, c, d) = (sgn a + sgn b)/8 * |(sgn a + sgn c)(sgn a + sgn d)| *
// min(|a|, |b|, |c|, |d|): the argument of least magnitude when all have one
// sign, else zero.  Written as max(min, 0) + min(max, 0) over the arguments:
// all positive gives the minimum, all negative the maximum, mixed signs (or a
// zero) give zero -- the same value exactly, in min/max instructions only.
template <typename T>
__device__ __forceinline__ T minmod2(T a, T b) {
  return fmax(fmin(a, b), T(0)) + fmin(fmax(a, b), T(0));
}

template <typename T>
__device__ __forceinline__ T minmod4(T a, T b, T c, T d) {
  const T lo = fmin(fmin(a, b), fmin(c, d)), hi = fmax(fmax(a, b), fmax(c, d));
  return fmax(lo, T(0)) + fmin(hi, T(0));
}

// Both states at the face x_{i+1/2} from s[0..5] = v_{i-2..i+3}: left from
// s0..s4 (centre s2), right from s5..s1 (centre s3).  The curvatures d_i,
// d_{i+1} and d^{M4}_{i+1/2} (minmod4 is symmetric in its pair) are computed
// once for both sides, and only when a side needs its limiter.  The unlimited
// value is written as the centre plus a combination of differences (exact on
// constant data).  POINT: the unlimited value is the fifth-order interpolation of
// point values, (3, -20, 90, 60, -5)/128 (the face point values that the
// sixth-order DER expects), instead of the cell-average kernel.
template <typename T, bool POINT = false>
__device__ __forceinline__ void mp5_pair(T s0, T s1, T s2, T s3, T s4, T s5, T& left, T& right) {
  // left: centre s2; right: centre s3, mirrored
  T vorL, vorR;
  if (POINT) {
    const T c128 = T(1.0 / 128.0);
    vorL = s2 + (T(3) * (s0 - s2) - T(20) * (s1 - s2) + T(60) * (s3 - s2) -
                 T(5) * (s4 - s2)) * c128;
    vorR = s3 + (T(3) * (s5 - s3) - T(20) * (s4 - s3) + T(60) * (s2 - s3) -
                 T(5) * (s1 - s3)) * c128;
  } else {
    const T c60 = T(1.0 / 60.0);
    vorL = s2 + (T(2) * (s0 - s2) - T(13) * (s1 - s2) + T(27) * (s3 - s2) -
                 T(3) * (s4 - s2)) * c60;
    vorR = s3 + (T(2) * (s5 - s3) - T(13) * (s4 - s3) + T(27) * (s2 - s3) -
                 T(3) * (s1 - s3)) * c60;
  }
  const T dlL = s2 - s1, dlR = s3 - s4;
  const T vmpL = s2 + minmod2(s3 - s2, T(4) * dlL);
  const T vmpR = s3 + minmod2(s2 - s3, T(4) * dlR);
  const bool okL = (vorL - s2) * (vorL - vmpL) <= T(1e-10);
  const bool okR = (vorR - s3) * (vorR - vmpR) <= T(1e-10);
  left = vorL;
  right = vorR;
  if (okL && okR) return;
  const T d1 = s0 - T(2) * s1 + s2;  // d_{i-1}
  const T d2 = s1 - T(2) * s2 + s3;  // d_i
  const T d3 = s2 - T(2) * s3 + s4;  // d_{i+1}
  const T d4 = s3 - T(2) * s4 + s5;  // d_{i+2}
  const T m23 = minmod4(T(4) * d2 - d3, T(4) * d3 - d2, d2, d3);  // d^{M4}_{i+1/2}
  if (!okL) {
    const T m12 = minmod4(T(4) * d2 - d1, T(4) * d1 - d2, d2, d1);  // d^{M4}_{i-1/2}
    const T vul = s2 + T(4) * dlL;
    const T vmd = T(0.5) * (s2 + s3) - T(0.5) * m23;
    const T vlc = s2 + T(0.5) * dlL + T(4.0 / 3.0) * m12;
    const T vmin = fmax(fmin(fmin(s2, s3), vmd), fmin(fmin(s2, vul), vlc));
    const T vmax = fmin(fmax(fmax(s2, s3), vmd), fmax(fmax(s2, vul), vlc));
    left = vorL + minmod2(vmin - vorL, vmax - vorL);
  }
  if (!okR) {
    const T m34 = minmod4(T(4) * d3 - d4, T(4) * d4 - d3, d3, d4);  // d^{M4}_{i+3/2}
    const T vul = s3 + T(4) * dlR;
    const T vmd = T(0.5) * (s3 + s2) - T(0.5) * m23;
    const T vlc = s3 + T(0.5) * dlR + T(4.0 / 3.0) * m34;
    const T vmin = fmax(fmin(fmin(s3, s2), vmd), fmin(fmin(s3, vul), vlc));
    const T vmax = fmin(fmax(fmax(s3, s2), vmd), fmax(fmax(s3, vul), vlc));
    right = vorR + minmod2(vmin - vorR, vmax - vorR);
  }
}

// Monotonized-central slope (van Leer 1977): sign(a) min(2|a|, 2|b|, |a+b|/2)
// when a and b have the same sign, else 0.
template <typename T>
__device__ __forceinline__ T mc_slope(T a, T b) {
  const T m = fmin(fmin(T(2) * fabs(a), T(2) * fabs(b)), T(0.5) * fabs(a + b));
  return a * b > T(0) ? copysign(m, a) : T(0);
}

// REC of both states at x_{i+1/2} from v_{i-2..i+3}.  kRecMp5: MP5 (cell-
// average kernel); kRecMc: linear, v_i + MC/2 and v_{i+1} - MC/2 (uses
// v_{i-1..i+2} only); kRecMp5Point: MP5 around the point-value interpolation.

template <int REC, typename T>
__device__ __forceinline__ void rec_pair(T s0, T s1, T s2, T s3, T s4, T s5, T& left, T& right) {
  if (REC == kRecMc) {
    left = s2 + T(0.5) * mc_slope(s2 - s1, s3 - s2);
    right = s3 - T(0.5) * mc_slope(s3 - s2, s4 - s3);
  } else {
    mp5_pair<T, REC == kRecMp5Point>(s0, s1, s2, s3, s4, s5, left, right);
  }
}

// ------------------------------------------------------------- UCT formula
// Londrillo & Del Zanna (2004) upwind edge field for an edge along k with
// (p, q, k) cyclic: four corner values E[ab] (a = side along p, b = side along
// q; 0 = left, 1 = right), p- and q-direction upwind speeds at the edge, B_q
// reconstructed along p (bqL/bqR) and B_p reconstructed along q (bpL/bpR).
template <typename T>
__device__ __forceinline__ T uct_edge(T ELL, T ELR, T ERL, T ERR, T app, T apm,
                                      T aqp, T aqm, T bqL, T bqR, T bpL, T bpR) {
  const T sp = app + apm, sq_ = aqp + aqm;
  if (sp > T(0) && sq_ > T(0)) {
    // one reciprocal for the weights and both dissipation coefficients
    const T inv = recip(sp * sq_);
    const T e = (app * aqp * ELL + app * aqm * ELR + apm * aqp * ERL + apm * aqm * ERR) * inv;
    const T dp = app * apm * sq_ * inv;
    const T dq = aqp * aqm * sp * inv;
    return e + dp * (bqR - bqL) - dq * (bpR - bpL);
  }
  T e;
  if (sp > T(0)) {
    e = (app * (ELL + ELR) + apm * (ERL + ERR)) / (T(2) * sp);
  } else if (sq_ > T(0)) {
    e = (aqp * (ELL + ERL) + aqm * (ELR + ERR)) / (T(2) * sq_);
  } else {
    e = T(0.25) * (ELL + ELR + ERL + ERR);
  }
  const T dp = sp > T(0) ? app * apm / sp : T(0);
  const T dq = sq_ > T(0) ? aqp * aqm / sq_ : T(0);
  return e + dp * (bqR - bqL) - dq * (bpR - bpL);
}

}  // namespace srmhd
