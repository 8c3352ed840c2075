// Per-pair arithmetic of the real-space kernels: radial coefficients of the
// screened, damped and bare kernels and the multipole contractions written
// out in closed form.
//
// Radial coefficients c_n(r) (c_{n+1} = -c_n'/r) define every interaction
// tensor.  Kernels:
//   bare     c0_n = (2n-1)!! / r^(2n+1)
//   Ewald    B_0 = erfc(beta r)/r,
//            B_n = ((2n-1) B_{n-1} + (2 beta^2)^n exp(-beta^2 r^2)/(beta sqrt(pi))) / r^2
//   Thole    damped c_n = lambda_{2n+1} c0_n with 1 - lambda_{2n+1} = P_n(x) exp(-x),
//            x = a r^3 s_i s_j, s = abar^-1/2, and
//            P_1 = 1, P_2 = 1 + x, P_3 = 1 + x + 3x^2/5,
//            P_4 = 1 + x + 18x^2/35 + 9x^3/35
//            (each from the previous by P_{n+1} = P_n + 3x/(2n+1) (P_n - P_n'),
//            which makes each damped tensor the derivative of the one below).
// Class coefficients with E_n the base kernel (B_n periodic, c0_n cluster):
//   excluded pair (same molecule, permanent involved):  c_n = E_n - c0_n
//   damped pair  (polarizable-polarizable):              c_n = E_n - P_n e^-x c0_n
//   plain pair:                                          c_n = E_n
//
// Multipole convention: the potential of site j at R = r - r_j is
// [q_j - d_j.grad + 1/3 Theta_j:grad grad] G(R) and the energy of site i in a
// potential phi is [q_i + d_i.grad + 1/3 Theta_i:grad grad] phi at r_i, with
// Theta the traceless Buckingham quadrupole.  Expanding with
// grad^n G in terms of deltas, R and c_n gives U = sum_n c_n P_n with
//   P0 = qi qj
//   P1 = qi (dj.R) - qj (di.R) + di.dj
//   P2 = (qi R.Tj.R + qj R.Ti.R)/3 - (di.R)(dj.R) + 2/3 (di.Tj.R - dj.Ti.R)
//        + 2/9 Ti:Tj
//   P3 = ((dj.R)(R.Ti.R) - (di.R)(R.Tj.R))/3 - 4/9 (Ti.R).(Tj.R)
//   P4 = (R.Ti.R)(R.Tj.R)/9
// and the force on i, F = -dU/dR = R sum_n c_{n+1} P_n - sum_n c_n grad P_n.
#pragma once
#include "common.h"
#include "erfcx_fit.h"

namespace sibfa {

// erfcx(x) = exp(x^2) erfc(x) for x >= 0: the Chebyshev series of
// erfcx_fit.h in t = 1 / (1 + p x), x clamped to kErfcxMax (past it erfc is
// below 2e-17).  The Ewald recursion multiplies by the exp(-x^2) it needs
// anyway, so erfc costs a reciprocal and a short series.  Relative error
// about 1e-14 (FP64) and 7e-7 (FP32).
template <typename R>
__device__ __forceinline__ R dev_erfcx(R x);
template <>
__device__ __forceinline__ double dev_erfcx<double>(double x) {
  x = fmin(x, kErfcxMax);
  const double d = 1.0 + kErfcxPF64 * x;
  // single-precision reciprocal, then two Newton steps (1e-7 -> 1e-14 -> exact)
  double t = (double)__builtin_amdgcn_rcpf((float)d);
  t = t * fma(-d, t, 2.0);
  t = t * fma(-d, t, 2.0);
  const double u = fma(t - kErfcxT0F64, 2.0 / (1.0 - kErfcxT0F64), -1.0);
  const double u2 = 2.0 * u;
  double b1 = 0.0, b2 = 0.0;
#pragma unroll
  for (int k = kErfcxDegF64; k >= 1; --k) {
    const double b = fma(u2, b1, kErfcxCF64[k] - b2);
    b2 = b1;
    b1 = b;
  }
  return fma(u, b1, kErfcxCF64[0] - b2);
}
template <>
__device__ __forceinline__ float dev_erfcx<float>(float x) {
  x = fminf(x, (float)kErfcxMax);
  const float t = __builtin_amdgcn_rcpf(1.0f + kErfcxPF32 * x);
  const float u = fmaf(t - kErfcxT0F32, 2.0f / (1.0f - kErfcxT0F32), -1.0f);
  const float u2 = 2.0f * u;
  float b1 = 0.0f, b2 = 0.0f;
#pragma unroll
  for (int k = kErfcxDegF32; k >= 1; --k) {
    const float b = fmaf(u2, b1, kErfcxCF32[k] - b2);
    b2 = b1;
    b1 = b;
  }
  return fmaf(u, b1, kErfcxCF32[0] - b2);
}

template <typename R>
__device__ __forceinline__ R dev_exp(R x);
template <>
__device__ __forceinline__ double dev_exp<double>(double x) { return exp(x); }
// FP32: the hardware 2^x (1 ulp) of x log2(e); the rounding of the product
// adds a relative error of at most 2^-24 |x log2 e| (8e-7 at the Ewald
// recursion's largest argument, 13), within the FP32 path's own rounding.
// The arguments here are never positive; below -126 / log2(e) the result
// flushes to zero, as the true values are then under FP32's normal range.
template <>
__device__ __forceinline__ float dev_exp<float>(float x) {
  return __builtin_amdgcn_exp2f(x * 1.44269504088896341f);
}

template <typename R>
__device__ __forceinline__ R dev_rsqrt(R x);
template <>
__device__ __forceinline__ double dev_rsqrt<double>(double x) { return rsqrt(x); }
template <>
__device__ __forceinline__ float dev_rsqrt<float>(float x) { return rsqrtf(x); }

// bare c0_0..c0_N
template <typename R, int N>
__device__ __forceinline__ void bare_coeffs(R rinv, R rinv2, R c[N + 1]) {
  c[0] = rinv;
#pragma unroll
  for (int n = 1; n <= N; ++n) c[n] = R(2 * n - 1) * c[n - 1] * rinv2;
}

// Ewald real-space B_0..B_N
template <typename R, int N>
__device__ __forceinline__ void ewald_coeffs(R r, R rinv, R rinv2, R beta, R B[N + 1]) {
  const R br = beta * r;
  const R ex = dev_exp<R>(-br * br);
  const R g = ex * (R(1) / (beta * R(kSqrtPi)));
  B[0] = ex * dev_erfcx<R>(br) * rinv;
  const R t = R(2) * beta * beta;
  R tn = t;
#pragma unroll
  for (int n = 1; n <= N; ++n) {
    B[n] = (R(2 * n - 1) * B[n - 1] + tn * g) * rinv2;
    tn *= t;
  }
}

// 1 - lambda_{2n+1} = P_n(x) e^-x, n = 1..4 (tp[0] unused, set 0)
template <typename R>
__device__ __forceinline__ void thole_tp(R x, R tp[5]) {
  const R e = dev_exp<R>(-x);
  const R x2 = x * x;
  tp[0] = R(0);
  tp[1] = e;
  tp[2] = (R(1) + x) * e;
  tp[3] = (R(1) + x + R(0.6) * x2) * e;
  tp[4] = (R(1) + x + R(18.0 / 35.0) * x2 + R(9.0 / 35.0) * x2 * x) * e;
}

template <typename R>
struct MP {
  R q;
  R d[3];
  R t[6];   // xx, xy, xz, yy, yz, zz
};

template <typename R>
__device__ __forceinline__ void tvec(const R t[6], const R v[3], R o[3]) {
  o[0] = t[0] * v[0] + t[1] * v[1] + t[2] * v[2];
  o[1] = t[1] * v[0] + t[3] * v[1] + t[4] * v[2];
  o[2] = t[2] * v[0] + t[4] * v[1] + t[5] * v[2];
}

// Energy U and force on i (F = -dU/dR) of multipoles A at r_i and B at
// r_j, R = r_i - r_j, with coefficients c[0..5] (c[5] used by the force).
template <typename R, bool WANT_U, bool WANT_F>
__device__ __forceinline__ void mp_pair(const R c[6], const MP<R>& A, const MP<R>& B,
                                        const R Rv[3], R& U, R F[3]) {
  const R dri = A.d[0] * Rv[0] + A.d[1] * Rv[1] + A.d[2] * Rv[2];
  const R drj = B.d[0] * Rv[0] + B.d[1] * Rv[1] + B.d[2] * Rv[2];
  const R dij = A.d[0] * B.d[0] + A.d[1] * B.d[1] + A.d[2] * B.d[2];
  R qir[3], qjr[3];
  tvec(A.t, Rv, qir);
  tvec(B.t, Rv, qjr);
  const R qrri = qir[0] * Rv[0] + qir[1] * Rv[1] + qir[2] * Rv[2];
  const R qrrj = qjr[0] * Rv[0] + qjr[1] * Rv[1] + qjr[2] * Rv[2];
  const R diqjr = A.d[0] * qjr[0] + A.d[1] * qjr[1] + A.d[2] * qjr[2];
  const R djqir = B.d[0] * qir[0] + B.d[1] * qir[1] + B.d[2] * qir[2];
  const R qq = qir[0] * qjr[0] + qir[1] * qjr[1] + qir[2] * qjr[2];
  const R tt = A.t[0] * B.t[0] + A.t[3] * B.t[3] + A.t[5] * B.t[5] +
               R(2) * (A.t[1] * B.t[1] + A.t[2] * B.t[2] + A.t[4] * B.t[4]);
  const R third = R(1.0 / 3.0);
  const R P0 = A.q * B.q;
  const R P1 = A.q * drj - B.q * dri + dij;
  const R P2 = third * (A.q * qrrj + B.q * qrri) - dri * drj + R(2.0 / 3.0) * (diqjr - djqir) +
               R(2.0 / 9.0) * tt;
  const R P3 = third * (drj * qrri - dri * qrrj) - R(4.0 / 9.0) * qq;
  const R P4 = R(1.0 / 9.0) * qrri * qrrj;
  if (WANT_U) U = c[0] * P0 + c[1] * P1 + c[2] * P2 + c[3] * P3 + c[4] * P4;
  if (WANT_F) {
    const R rad = c[1] * P0 + c[2] * P1 + c[3] * P2 + c[4] * P3 + c[5] * P4;
    R tjdi[3], tidj[3], tiqjr[3], tjqir[3];
    tvec(B.t, A.d, tjdi);
    tvec(A.t, B.d, tidj);
    tvec(A.t, qjr, tiqjr);
    tvec(B.t, qir, tjqir);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const R g1 = A.q * B.d[a] - B.q * A.d[a];
      const R g2 = R(2.0 / 3.0) * (A.q * qjr[a] + B.q * qir[a]) - A.d[a] * drj - B.d[a] * dri +
                   R(2.0 / 3.0) * (tjdi[a] - tidj[a]);
      const R g3 = third * (B.d[a] * qrri - A.d[a] * qrrj) +
                   R(2.0 / 3.0) * (drj * qir[a] - dri * qjr[a]) -
                   R(4.0 / 9.0) * (tiqjr[a] + tjqir[a]);
      const R g4 = R(2.0 / 9.0) * (qir[a] * qrrj + qjr[a] * qrri);
      F[a] = Rv[a] * rad - (c[1] * g1 + c[2] * g2 + c[3] * g3 + c[4] * g4);
    }
  }
}

// Field at r_i of the multipoles B at r_j, R = r_i - r_j, coefficients c[1..3].
template <typename R>
__device__ __forceinline__ void mp_field(const R c[6], const MP<R>& B, const R Rv[3], R E[3]) {
  const R drj = B.d[0] * Rv[0] + B.d[1] * Rv[1] + B.d[2] * Rv[2];
  R qjr[3];
  tvec(B.t, Rv, qjr);
  const R qrrj = qjr[0] * Rv[0] + qjr[1] * Rv[1] + qjr[2] * Rv[2];
  const R rad = B.q * c[1] + drj * c[2] + R(1.0 / 3.0) * qrrj * c[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) E[a] = Rv[a] * rad - (B.d[a] * c[1] + R(2.0 / 3.0) * qjr[a] * c[2]);
}

// Field at r_i of a point dipole p at r_j (coefficients c1, c2).
template <typename R>
__device__ __forceinline__ void dip_field(R c1, R c2, const R p[3], const R Rv[3], R E[3]) {
  const R rp = Rv[0] * p[0] + Rv[1] * p[1] + Rv[2] * p[2];
#pragma unroll
  for (int a = 0; a < 3; ++a) E[a] = c2 * rp * Rv[a] - c1 * p[a];
}

}  // namespace sibfa
