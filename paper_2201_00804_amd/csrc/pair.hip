// Real-space pair kernels over the ELL neighbour lists.
//
// Mapping: G consecutive lanes own one site and stride through its list;
// the G partial sums are folded with cross-lane shuffles.  Same-molecule
// pairs (few per site, short distances where the excluded Ewald part
// E_n - c0_n cancels strongly) are always evaluated in FP64; the
// intermolecular pairs run in the kernel's precision R (double, or float in
// mixed mode) with FP64 accumulation.
//
//  k_perm    : permanent field E at polarizable sites (Thole-damped Mmu
//              class, excluded within a molecule) and the MM real-space
//              energy, plus Ewald self terms.
//  k_matvec  : real-space part of (T p)_i = alpha_i^-1 p_i - [damped dipole
//              field of p + PME field of p + self]; k_matvec_recip gathers
//              the PME field from the potential grid and forms p.Tp.
//  k_force   : real-space forces of MM, Mmu and mumu classes at fixed mu.
#include <hip/hip_ext.h>

#include "common.h"
#include "pairmath.h"
#include "kernels.h"

namespace sibfa {

template <typename R>
__device__ __forceinline__ void load_mp(const SysView& s, int j, MP<R>& M, R x[3]);

template <>
__device__ __forceinline__ void load_mp<double>(const SysView& s, int j, MP<double>& M,
                                                double x[3]) {
  const double4 p = s.sp[j], d = s.sd[j], t = s.sth[j];
  const double2 t2 = s.sth2[j];
  x[0] = p.x; x[1] = p.y; x[2] = p.z;
  M.q = p.w;
  M.d[0] = d.x; M.d[1] = d.y; M.d[2] = d.z;
  M.t[0] = t.x; M.t[1] = t.y; M.t[2] = t.z; M.t[3] = t.w; M.t[4] = t2.x; M.t[5] = t2.y;
}

template <>
__device__ __forceinline__ void load_mp<float>(const SysView& s, int j, MP<float>& M, float x[3]) {
  const float4 p = s.sp32[j], d = s.sd32[j], t = s.sth32[j];
  const float2 t2 = s.sth232[j];
  x[0] = p.x; x[1] = p.y; x[2] = p.z;
  M.q = p.w;
  M.d[0] = d.x; M.d[1] = d.y; M.d[2] = d.z;
  M.t[0] = t.x; M.t[1] = t.y; M.t[2] = t.z; M.t[3] = t.w; M.t[4] = t2.x; M.t[5] = t2.y;
}

template <typename R>
__device__ __forceinline__ R site_s(const SysView& s, int j);
template <>
__device__ __forceinline__ double site_s<double>(const SysView& s, int j) { return s.sd[j].w; }
template <>
__device__ __forceinline__ float site_s<float>(const SysView& s, int j) { return s.sd32[j].w; }

template <typename R>
__device__ __forceinline__ void displacement(const SysView& s, const R xi[3], const R xj[3],
                                             R Rv[3]) {
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    R d = xi[a] - xj[a];
    if (s.periodic) d = min_image<R>(d, R(s.box[a]), R(s.ibox[a]));
    Rv[a] = d;
  }
}

// r_i - r_j from the FP64 positions, rounded to R.  In FP32 this carries
// only the rounding of the separation itself, not that of two coordinates
// as large as the box (about 1e-5 A at 100 A, which would dominate the
// error of the FP32 pair energies and forces); in FP64 it is displacement().
template <typename R>
__device__ __forceinline__ void sep64(const SysView& s, const double xi[3], const double xj[3],
                                      R Rv[3]) {
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    double d = xi[a] - xj[a];
    if (s.periodic) d = min_image<double>(d, s.box[a], s.ibox[a]);
    Rv[a] = R(d);
  }
}

// The multipoles of site j in precision R and its FP64 position (the
// charge comes from the FP64 record too, which holds both).
template <typename R>
__device__ __forceinline__ void load_mp_x64(const SysView& s, int j, MP<R>& M, double x[3]) {
  const double4 p = s.sp[j];
  x[0] = p.x; x[1] = p.y; x[2] = p.z;
  if constexpr (sizeof(R) == sizeof(double)) {
    const double4 d = s.sd[j], t = s.sth[j];
    const double2 t2 = s.sth2[j];
    M.q = p.w;
    M.d[0] = d.x; M.d[1] = d.y; M.d[2] = d.z;
    M.t[0] = t.x; M.t[1] = t.y; M.t[2] = t.z; M.t[3] = t.w; M.t[4] = t2.x; M.t[5] = t2.y;
  } else {
    const float4 d = s.sd32[j], t = s.sth32[j];
    const float2 t2 = s.sth232[j];
    M.q = R(p.w);
    M.d[0] = d.x; M.d[1] = d.y; M.d[2] = d.z;
    M.t[0] = t.x; M.t[1] = t.y; M.t[2] = t.z; M.t[3] = t.w; M.t[4] = t2.x; M.t[5] = t2.y;
  }
}

// base kernel E_0..E_N: Ewald B_n when periodic, bare c0_n for clusters
template <typename R, int N>
__device__ __forceinline__ void base_coeffs(const SysView& s, R r, R rinv, R rinv2, R E[N + 1]) {
  if (s.periodic) ewald_coeffs<R, N>(r, rinv, rinv2, R(s.beta), E);
  else bare_coeffs<R, N>(rinv, rinv2, E);
}

__device__ __forceinline__ double thole_a_pair(const SysView& s, int i, int j) {
  return s.uniform_thole ? s.thole_a : fmin(s.sa[i], s.sa[j]);
}
__device__ __forceinline__ double thole_a_polpair(const SysView& s, int i, int j) {
  return s.uniform_thole ? s.thole_a : fmin(s.pa[i], s.pa[j]);
}

// ------------------------------------------------------------------ E0 + E_elec
// Same-molecule pairs (excluded, E_n - c0_n; FP64; periodic only) and the
// Ewald self terms, one thread per site: writes E0 of polarizable sites
// and the energy partials S_AUX (pairs) and S_ESELF.
__global__ __launch_bounds__(kBlock) void k_perm_intra(SysView s, Reduce red, double4* E0) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int sub = 0, G = 1;
  double acc[3] = {0.0, 0.0, 0.0};
  double U = 0.0, Uself = 0.0;
  int pi = -1;
  if (i < s.n) {
    pi = s.polidx[i];
    if (s.periodic) {
      MP<double> Mi;
      double xi[3];
      load_mp<double>(s, i, Mi, xi);
      const int cnt = s.nc_in[i];
      for (int k = sub; k < cnt; k += G) {
        const int j = s.nb_in[(size_t)i * s.cap_in + k];
        MP<double> Mj;
        double xj[3], Rv[3];
        load_mp<double>(s, j, Mj, xj);
        displacement<double>(s, xi, xj, Rv);
        const double r2 = Rv[0] * Rv[0] + Rv[1] * Rv[1] + Rv[2] * Rv[2];
        const double rinv = rsqrt(r2), r = r2 * rinv, rinv2 = rinv * rinv;
        double B[5], c0[5], c[6];
        ewald_coeffs<double, 4>(r, rinv, rinv2, s.beta, B);
        bare_coeffs<double, 4>(rinv, rinv2, c0);
#pragma unroll
        for (int n = 0; n < 5; ++n) c[n] = B[n] - c0[n];
        c[5] = 0.0;
        double u, fdum[3];
        mp_pair<double, true, false>(c, Mi, Mj, Rv, u, fdum);
        U += 0.5 * u;
        if (pi >= 0) {
          double E[3];
          mp_field<double>(c, Mj, Rv, E);
          acc[0] += E[0]; acc[1] += E[1]; acc[2] += E[2];
        }
      }
    }
  }
  if (i < s.n && s.periodic) {
    const double4 p = s.sp[i], d = s.sd[i], t = s.sth[i];
    const double2 t2 = s.sth2[i];
    const double b = s.beta, b3 = b * b * b, b5 = b3 * b * b;
    const double tt = t.x * t.x + t.w * t.w + t2.y * t2.y +
                      2.0 * (t.y * t.y + t.z * t.z + t2.x * t2.x);
    Uself = -(b / kSqrtPi * p.w * p.w + 2.0 * b3 / (3.0 * kSqrtPi) * (d.x * d.x + d.y * d.y + d.z * d.z) +
              8.0 * b5 / (45.0 * kSqrtPi) * tt);
    const double sf = 4.0 * b3 / (3.0 * kSqrtPi);
    acc[0] += sf * d.x; acc[1] += sf * d.y; acc[2] += sf * d.z;
  }
  if (pi >= 0) E0[pi] = make_double4(acc[0], acc[1], acc[2], 0.0);
  block_partial(U, red, S_AUX);
  block_partial(Uself, red, S_ESELF);
}

// One intermolecular pair of k_perm: MM energy (half, the pair is seen from
// both sites) and, for a polarizable site i, the field of M_j, Thole-damped
// when j is polarizable too.  Far pairs (see the list layout) have x >= 50
// for every polarizable pair, where the damping factor e^-x < 2e-22 is
// dropped, as it is for near pairs with x >= 50.
template <typename R, bool NEAR>
__device__ __forceinline__ void perm_pair(const SysView& s, int i, int j, int pi, const MP<R>& Mi,
                                          const double xi[3], R si, double& U, double acc[3]) {
  MP<R> Mj;
  R Rv[3];
  double xj[3];
  load_mp_x64<R>(s, j, Mj, xj);
  sep64<R>(s, xi, xj, Rv);
  const R r2 = Rv[0] * Rv[0] + Rv[1] * Rv[1] + Rv[2] * Rv[2];
  const R rinv = dev_rsqrt<R>(r2), r = r2 * rinv, rinv2 = rinv * rinv;
  R c[6];
  base_coeffs<R, 4>(s, r, rinv, rinv2, c);
  c[5] = R(0);
  R u, fdum[3];
  mp_pair<R, true, false>(c, Mi, Mj, Rv, u, fdum);
  U += 0.5 * (double)u;
  if (pi >= 0) {
    if (NEAR) {
      const R sj = site_s<R>(s, j);
      R x = R(0);
      if (sj > R(0) && (x = R(thole_a_pair(s, i, j)) * r2 * r * si * sj) < R(50)) {
        R tp[5], c0[4];
        thole_tp<R>(x, tp);
        bare_coeffs<R, 3>(rinv, rinv2, c0);
#pragma unroll
        for (int n = 1; n <= 3; ++n) c[n] -= tp[n] * c0[n];
      }
    }
    R E[3];
    mp_field<R>(c, Mj, Rv, E);
    acc[0] += (double)E[0]; acc[1] += (double)E[1]; acc[2] += (double)E[2];
  }
}

// Intermolecular pairs within the cutoff (precision R): MM energy partials
// (S_EREAL) and the damped field added to E0 of polarizable sites.  Near
// entries first, then far ones (no damping).
template <typename R, int G>
__global__ __launch_bounds__(kBlock) void k_perm(SysView s, Reduce red, double4* E0) {
  const int sub = threadIdx.x % G;
  const int i = blockIdx.x * (kBlock / G) + threadIdx.x / G;
  double acc[3] = {0.0, 0.0, 0.0};
  double U = 0.0;
  int pi = -1;
  if (i < s.n) {
    pi = s.polidx[i];
    MP<R> Mi;
    R xr[3];
    load_mp<R>(s, i, Mi, xr);
    const double4 p4 = s.sp[i];
    const double xi[3] = {p4.x, p4.y, p4.z};
    const R si = site_s<R>(s, i);
    const int* row = s.nb_all + (size_t)i * s.cap_all;
    const int nn = s.nc_near[i], nf = s.nc_all[i] - nn;
    for (int k = sub; k < nn; k += G) perm_pair<R, true>(s, i, row[k], pi, Mi, xi, si, U, acc);
    // far entries two per step (same summation order): the second pair's
    // gathers are issued while the first is evaluated
    const int* far = row + s.cap_all - 1;
    int k = sub;
    for (; k + G < nf; k += 2 * G) {
      const int j0 = far[-k], j1 = far[-(k + G)];
      perm_pair<R, false>(s, i, j0, pi, Mi, xi, si, U, acc);
      perm_pair<R, false>(s, i, j1, pi, Mi, xi, si, U, acc);
    }
    if (k < nf) perm_pair<R, false>(s, i, far[-k], pi, Mi, xi, si, U, acc);
  }
#pragma unroll
  for (int a = 0; a < 3; ++a) acc[a] = group_sum<G>(acc[a]);
  if (sub == 0 && pi >= 0) {
    double4 e = E0[pi];
    e.x += acc[0]; e.y += acc[1]; e.z += acc[2];
    E0[pi] = e;
  }
  block_partial(U, red, S_EREAL);
}

// ------------------------------------------------------------------ matvec
template <typename R>
__device__ __forceinline__ void load_p(const double4* p, const float4* p32, int j, R v[3]);
template <>
__device__ __forceinline__ void load_p<double>(const double4* p, const float4*, int j, double v[3]) {
  const double4 a = p[j];
  v[0] = a.x; v[1] = a.y; v[2] = a.z;
}
template <>
__device__ __forceinline__ void load_p<float>(const double4*, const float4* p32, int j, float v[3]) {
  const float4 a = p32[j];
  v[0] = a.x; v[1] = a.y; v[2] = a.z;
}

template <typename R>
__device__ __forceinline__ void load_pp(const SysView& s, int j, R x[3], R& sj);
template <>
__device__ __forceinline__ void load_pp<double>(const SysView& s, int j, double x[3], double& sj) {
  const double4 a = s.pp[j];
  x[0] = a.x; x[1] = a.y; x[2] = a.z; sj = a.w;
}
template <>
__device__ __forceinline__ void load_pp<float>(const SysView& s, int j, float x[3], float& sj) {
  const float4 a = s.pp32[j];
  x[0] = a.x; x[1] = a.y; x[2] = a.z; sj = a.w;
}

template <typename R>
__device__ __forceinline__ R grid_at(const PmeView& pm, size_t idx);
template <>
__device__ __forceinline__ double grid_at<double>(const PmeView& pm, size_t idx) { return pm.phi[idx]; }
template <>
__device__ __forceinline__ float grid_at<float>(const PmeView& pm, size_t idx) { return pm.phi32[idx]; }

// Damped, screened dipole-dipole coefficients of the intermolecular pol
// pairs, c1 = E_1 - P_1 e^-x c0_1 and c2 = E_2 - P_2 e^-x c0_2, in the
// ELL layout of the pol list.  Positions are fixed during a solve, so the
// matvec reads them instead of re-evaluating erfc/exp per pair.  Computed
// in FP64 (R = double: FP64 table, and its FP32 rounding when out32 is
// given) or in FP32 (R = float: FP32 table only).
template <typename R, int G>
__global__ __launch_bounds__(kBlock) void k_pol_coef(SysView s, double2* out, float2* out32,
                                                     double2* out_in) {
  const int sub = threadIdx.x % G;
  const int pi = blockIdx.x * (kBlock / G) + threadIdx.x / G;
  if (pi >= s.npol) return;
  {
    // same-molecule polarizable pairs, always FP64
    double xi[3], si;
    load_pp<double>(s, pi, xi, si);
    const int cin = s.nc_ipol[pi];
    for (int k = sub; k < cin; k += G) {
      const size_t e = (size_t)pi * s.cap_ipol + k;
      const int j = s.nb_ipol[e];
      double xj[3], sj, Rv[3];
      load_pp<double>(s, j, xj, sj);
      displacement<double>(s, xi, xj, Rv);
      const double r2 = Rv[0] * Rv[0] + Rv[1] * Rv[1] + Rv[2] * Rv[2];
      const double rinv = rsqrt(r2), r = r2 * rinv, rinv2 = rinv * rinv;
      double Eb[3], c0[3], tp[5];
      base_coeffs<double, 2>(s, r, rinv, rinv2, Eb);
      bare_coeffs<double, 2>(rinv, rinv2, c0);
      thole_tp<double>(thole_a_polpair(s, pi, j) * r2 * r * si * sj, tp);
      out_in[e] = make_double2(Eb[1] - tp[1] * c0[1], Eb[2] - tp[2] * c0[2]);
    }
  }
  R xr[3], sr;
  load_pp<R>(s, pi, xr, sr);
  const int cnt = s.nc_pol[pi];
  for (int k = sub; k < cnt; k += G) {
    const size_t e = (size_t)pi * s.cap_pol + k;
    const int j = s.nb_pol[e];
    R xj[3], sj, Rv[3];
    load_pp<R>(s, j, xj, sj);
    displacement<R>(s, xr, xj, Rv);
    const R r2 = Rv[0] * Rv[0] + Rv[1] * Rv[1] + Rv[2] * Rv[2];
    const R rinv = dev_rsqrt<R>(r2), r = r2 * rinv, rinv2 = rinv * rinv;
    R Eb[3];
    base_coeffs<R, 2>(s, r, rinv, rinv2, Eb);
    R c1 = Eb[1], c2 = Eb[2];
    // damping only where it is not negligible (x < 50, as in k_perm)
    const R x = R(thole_a_polpair(s, pi, j)) * r2 * r * sr * sj;
    if (x < R(50)) {
      R c0[3], tp[5];
      bare_coeffs<R, 2>(rinv, rinv2, c0);
      thole_tp<R>(x, tp);
      c1 -= tp[1] * c0[1];
      c2 -= tp[2] * c0[2];
    }
    if (out) out[e] = make_double2((double)c1, (double)c2);
    if (out32) out32[e] = make_float2((float)c1, (float)c2);
  }
}

// The coefficient and index streams are read once per matvec: non-temporal
// loads keep them from evicting the gathered neighbour records from L2.
typedef double nt_double2 __attribute__((ext_vector_type(2)));
typedef float nt_float2 __attribute__((ext_vector_type(2)));
template <typename R>
__device__ __forceinline__ void load_coef(const SysView& s, size_t e, R& c1, R& c2);
template <>
__device__ __forceinline__ void load_coef<double>(const SysView& s, size_t e, double& c1, double& c2) {
  const nt_double2 c = __builtin_nontemporal_load(reinterpret_cast<const nt_double2*>(s.cpol + e));
  c1 = c.x; c2 = c.y;
}
template <>
__device__ __forceinline__ void load_coef<float>(const SysView& s, size_t e, float& c1, float& c2) {
  const nt_float2 c = __builtin_nontemporal_load(reinterpret_cast<const nt_float2*>(s.cpol32 + e));
  c1 = c.x; c2 = c.y;
}

// One intermolecular pol pair of the matvec: field at i of the dipole p_j,
// with the cached coefficients of the entry.
template <typename R>
__device__ __forceinline__ void matvec_pair(const SysView& s, const double4* p, const float4* p32,
                                            size_t e, const R xr[3], double f[3]) {
  const int j = __builtin_nontemporal_load(&s.nb_pol[e]);
  R xj[3], sj, Rv[3], pj[3];
  load_pp<R>(s, j, xj, sj);
  load_p<R>(p, p32, j, pj);
  R c1, c2;
  load_coef<R>(s, e, c1, c2);
  displacement<R>(s, xr, xj, Rv);
  R E[3];
  dip_field<R>(c1, c2, pj, Rv, E);
  f[0] += (double)E[0]; f[1] += (double)E[1]; f[2] += (double)E[2];
}

// Real-space part of (T p)_i = alpha_i^-1 p_i - [real field + self field]
// (minus the reciprocal field, subtracted by k_matvec_recip when periodic;
// clusters finish here, with p.Tp).  Needs the cached coefficients of the
// current positions (k_pol_coef).
template <typename R, int G>
__global__ __launch_bounds__(kBlock) void k_matvec(SysView s, Reduce red, const double4* p,
                                                   const float4* p32, double4* out,
                                                   int dot_slot) {
  if (stopped(red.stop)) return;
  const int sub = threadIdx.x % G;
  const int pi = xcd_block() * (kBlock / G) + threadIdx.x / G;
  double f[3] = {0.0, 0.0, 0.0};
  if (pi < s.npol) {
    double xi[3], si;
    load_pp<double>(s, pi, xi, si);
    // same-molecule polarizable pairs (damped, FP64)
    const int cin = s.nc_ipol[pi];
    for (int k = sub; k < cin; k += G) {
      const size_t e = (size_t)pi * s.cap_ipol + k;
      const int j = s.nb_ipol[e];
      double xj[3], sj, Rv[3], pj[3];
      load_pp<double>(s, j, xj, sj);
      load_p<double>(p, p32, j, pj);
      displacement<double>(s, xi, xj, Rv);
      const double2 cc = s.cipol[e];
      const double c1 = cc.x, c2 = cc.y;
      double E[3];
      dip_field<double>(c1, c2, pj, Rv, E);
      f[0] += E[0]; f[1] += E[1]; f[2] += E[2];
    }
    // intermolecular polarizable pairs within the cutoff, precision R; four
    // entries per lane and step so that their gathers overlap
    R xr[3], sr;
    load_pp<R>(s, pi, xr, sr);
    const int cnt = s.nc_pol[pi];
    const size_t row = (size_t)pi * s.cap_pol;
    int k = sub;
    for (; k + 3 * G < cnt; k += 4 * G) {
      matvec_pair<R>(s, p, p32, row + k, xr, f);
      matvec_pair<R>(s, p, p32, row + k + G, xr, f);
      matvec_pair<R>(s, p, p32, row + k + 2 * G, xr, f);
      matvec_pair<R>(s, p, p32, row + k + 3 * G, xr, f);
    }
    for (; k < cnt; k += G) matvec_pair<R>(s, p, p32, row + k, xr, f);
  }
#pragma unroll
  for (int a = 0; a < 3; ++a) f[a] = group_sum<G>(f[a]);
  double dot = 0.0;
  if (sub == 0 && pi < s.npol) {
    const double4 pv = p[pi];
    if (s.periodic) {
      const double b = s.beta, sf = 4.0 * b * b * b / (3.0 * kSqrtPi);
      f[0] += sf * pv.x; f[1] += sf * pv.y; f[2] += sf * pv.z;
    }
    const double* ai = s.ainv + 6 * (size_t)pi;
    double q[3];
    q[0] = ai[0] * pv.x + ai[1] * pv.y + ai[2] * pv.z - f[0];
    q[1] = ai[1] * pv.x + ai[3] * pv.y + ai[4] * pv.z - f[1];
    q[2] = ai[2] * pv.x + ai[4] * pv.y + ai[5] * pv.z - f[2];
    out[pi] = make_double4(q[0], q[1], q[2], 0.0);
    dot = pv.x * q[0] + pv.y * q[1] + pv.z * q[2];
  }
  if (!s.periodic && dot_slot >= 0) block_partial(dot, red, dot_slot);
}

// Reciprocal part of the matvec: q_i -= E_rec,i = -grad phi(r_i) with phi
// the potential grid of the spread p; then p.Tp.  One thread per site.
template <typename R, int P>
__global__ __launch_bounds__(kBlock) void k_matvec_recip(SysView s, PmeView pm, Reduce red,
                                                         const double4* p, double4* out,
                                                         int dot_slot) {
  if (stopped(red.stop)) return;
  const int pi = blockIdx.x * blockDim.x + threadIdx.x;
  double dot = 0.0;
  if (pi < s.npol) {
    const double4 x = s.pp[pi];
    int base[3];
    R th[3][2][P];
    const double xs[3] = {x.x, x.y, x.z};
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      double fr;
      base[a] = grid_base(xs[a], pm.scale[a], pm.K[a], &fr);
      bspline_weights<R, P, 1>((R)fr, th[a]);
    }
    double g[3] = {0.0, 0.0, 0.0};
    for (int tz = 0; tz < P; ++tz) {
      int iz = base[2] - tz; if (iz < 0) iz += pm.K[2];
      for (int ty = 0; ty < P; ++ty) {
        int iy = base[1] - ty; if (iy < 0) iy += pm.K[1];
        const size_t rowi = ((size_t)iz * pm.K[1] + iy) * pm.K[0];
        R s0 = 0, s1 = 0;
#pragma unroll
        for (int tx = 0; tx < P; ++tx) {
          int ix = base[0] - tx; if (ix < 0) ix += pm.K[0];
          const R v = grid_at<R>(pm, rowi + ix);
          s0 += v * th[0][0][tx];
          s1 += v * th[0][1][tx];
        }
        g[0] += (double)(s1 * th[1][0][ty] * th[2][0][tz]);
        g[1] += (double)(s0 * th[1][1][ty] * th[2][0][tz]);
        g[2] += (double)(s0 * th[1][0][ty] * th[2][1][tz]);
      }
    }
    double4 q = out[pi];
    q.x += g[0] * pm.scale[0];
    q.y += g[1] * pm.scale[1];
    q.z += g[2] * pm.scale[2];
    out[pi] = q;
    const double4 pv = p[pi];
    dot = pv.x * q.x + pv.y * q.y + pv.z * q.z;
  }
  if (dot_slot >= 0) block_partial(dot, red, dot_slot);
}

// ------------------------------------------------------------------ forces
template <typename R>
__device__ __forceinline__ void load_mu(const double4* mu, const float4* mu32, int j, R v[3]);
template <>
__device__ __forceinline__ void load_mu<double>(const double4* mu, const float4*, int j, double v[3]) {
  const double4 a = mu[j];
  v[0] = a.x; v[1] = a.y; v[2] = a.z;
}
template <>
__device__ __forceinline__ void load_mu<float>(const double4*, const float4* mu32, int j, float v[3]) {
  const float4 a = mu32[j];
  v[0] = a.x; v[1] = a.y; v[2] = a.z;
}

template <typename R>
__device__ __forceinline__ MP<R> dipole_only(const R d[3]) {
  MP<R> m;
  m.q = R(0);
  m.d[0] = d[0]; m.d[1] = d[1]; m.d[2] = d[2];
#pragma unroll
  for (int k = 0; k < 6; ++k) m.t[k] = R(0);
  return m;
}

// Real-space forces at fixed mu.  Writing M' = (q, d + mu, Theta) and using
// that every class term is bilinear in the multipoles of the two sites:
//  intermolecular pair: MM(B) + Mmu(cT) + mumu(cT) = F(M', M'; cT)
//                       + F(M, M; B - cT),  cT_n = B_n - P_n e^-x c0_n,
//    and B - cT vanishes unless both sites are polarizable and close enough
//    for the Thole factor to matter (x < 50), so the second term is skipped
//    for almost every pair;
//  same-molecule pair:  MM and Mmu excluded (E - c0), mumu damped
//                       = F(M', M'; E - c0) + F(mu, mu; lambda c0)
//    (the first term is zero for clusters, where E = c0).
// The virial (VIR) of the pair energies under a homogeneous strain
// R -> (1 + eps) R with the multipoles fixed, W_ab = -dE/d eps_ab, is
// 1/2 sum over directed list entries of f_a R_b, f the force on i of the
// entry's pair; each kernel writes its block partials of the nine
// components (row-major) to its own nine reduction slots.
__device__ __forceinline__ void vir_add(double W[9], const double f[3], const double R[3]) {
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) W[3 * a + b] += 0.5 * f[a] * R[b];
}

__device__ __forceinline__ void vir_partials(const double W[9], const Reduce& red, int slot0) {
#pragma unroll
  for (int k = 0; k < 9; ++k) block_partial(W[k], red, slot0 + k);
}

// Same-molecule pairs (FP64, one thread per site); writes Fout.
template <bool VIR>
__global__ __launch_bounds__(kBlock) void k_force_intra(SysView s, Reduce red, const double4* mu,
                                                        double4* Fout) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  double F[3] = {0.0, 0.0, 0.0};
  double W[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
  if (i < s.n) {
    {
      const int sub = 0, G = 1;
      const float4* mu32 = nullptr;
      MP<double> Mi;
      double xi[3], mui[3];
      load_mp<double>(s, i, Mi, xi);
      load_mu<double>(mu, mu32, i, mui);
      MP<double> Pi = Mi;
      Pi.d[0] += mui[0]; Pi.d[1] += mui[1]; Pi.d[2] += mui[2];
      const double si = s.sd[i].w;
      const int cnt = s.nc_in[i];
      for (int k = sub; k < cnt; k += G) {
        const int j = s.nb_in[(size_t)i * s.cap_in + k];
        MP<double> Mj;
        double xj[3], Rv[3], muj[3];
        load_mp<double>(s, j, Mj, xj);
        load_mu<double>(mu, mu32, j, muj);
        displacement<double>(s, xi, xj, Rv);
        const double r2 = Rv[0] * Rv[0] + Rv[1] * Rv[1] + Rv[2] * Rv[2];
        const double rinv = rsqrt(r2), r = r2 * rinv, rinv2 = rinv * rinv;
        double Eb[6], c0[6], c[6];
        base_coeffs<double, 5>(s, r, rinv, rinv2, Eb);
        bare_coeffs<double, 5>(rinv, rinv2, c0);
        double u, f[3];
        if (s.periodic) {
#pragma unroll
          for (int n = 0; n < 6; ++n) c[n] = Eb[n] - c0[n];
          MP<double> Pj = Mj;
          Pj.d[0] += muj[0]; Pj.d[1] += muj[1]; Pj.d[2] += muj[2];
          mp_pair<double, false, true>(c, Pi, Pj, Rv, u, f);
          F[0] += f[0]; F[1] += f[1]; F[2] += f[2];
          if (VIR) vir_add(W, f, Rv);
        }
        const double sj = s.sd[j].w;
        if (si > 0.0 && sj > 0.0) {
          double tp[5];
          thole_tp<double>(thole_a_pair(s, i, j) * r2 * r * si * sj, tp);
          c[0] = 0.0;
          c[5] = 0.0;
#pragma unroll
          for (int n = 1; n <= 4; ++n) c[n] = (1.0 - tp[n]) * c0[n];
          const MP<double> Ui = dipole_only<double>(mui), Uj = dipole_only<double>(muj);
          mp_pair<double, false, true>(c, Ui, Uj, Rv, u, f);
          F[0] += f[0]; F[1] += f[1]; F[2] += f[2];
          if (VIR) vir_add(W, f, Rv);
        }
      }
    }
    Fout[i] = make_double4(F[0], F[1], F[2], 0.0);
  }
  if (VIR) vir_partials(W, red, S_VRI);
}

// ------------------------------------------------------------------ site fields
// Field E and field gradient dE_b/dr_a at every site of the multipoles that
// its own permanent multipoles interact with (local frames: the energy's
// derivative with respect to a site's dipole is -E, with respect to its
// quadrupole -1/3 grad E): the permanent multipoles of the other sites
// (MM class) and the induced dipoles (Mmu class, Thole-damped).  With
// M' = (q, d + mu, Theta) the two classes combine as in the force kernel:
// M' with the damped coefficients, plus M with B - cT where the damping
// matters; same-molecule pairs (periodic only) take M' with E - c0.
// Field and gradient of a source (q, d, Theta) at R = r_i - r_j:
//   E_b       = R_b rad - d_b c1 - 2/3 (Theta R)_b c2,
//   rad       = q c1 + (d.R) c2 + 1/3 (R Theta R) c3,
//   dE_b/dR_a = delta_ab rad - R_a R_b S + c2 (R_b d_a + R_a d_b)
//               + 2/3 c3 (R_b (Theta R)_a + R_a (Theta R)_b) - 2/3 c2 Theta_ab,
//   S         = q c2 + (d.R) c3 + 1/3 (R Theta R) c4
// (from dc_n/dR_a = -R_a c_{n+1}).  Gradients are stored xx xy xz yy yz zz.
template <typename R>
__device__ __forceinline__ void mp_field_grad(const R c[6], const MP<R>& B, const R Rv[3],
                                              double E[3], double G[6]) {
  const R dr = B.d[0] * Rv[0] + B.d[1] * Rv[1] + B.d[2] * Rv[2];
  R tr[3];
  tvec(B.t, Rv, tr);
  const R rtr = tr[0] * Rv[0] + tr[1] * Rv[1] + tr[2] * Rv[2];
  const R third = R(1.0 / 3.0), two3 = R(2.0 / 3.0);
  const R rad = B.q * c[1] + dr * c[2] + third * rtr * c[3];
  const R S = B.q * c[2] + dr * c[3] + third * rtr * c[4];
#pragma unroll
  for (int b = 0; b < 3; ++b) E[b] += (double)(Rv[b] * rad - B.d[b] * c[1] - two3 * tr[b] * c[2]);
  const int ia[6] = {0, 0, 0, 1, 1, 2}, ib[6] = {0, 1, 2, 1, 2, 2};
#pragma unroll
  for (int k = 0; k < 6; ++k) {
    const int a = ia[k], b = ib[k];
    R g = -Rv[a] * Rv[b] * S + c[2] * (Rv[b] * B.d[a] + Rv[a] * B.d[b]) +
          two3 * c[3] * (Rv[b] * tr[a] + Rv[a] * tr[b]) - two3 * c[2] * B.t[k];
    if (a == b) g += rad;
    G[k] += (double)g;
  }
}

// One intermolecular pair of k_force (see the identity above).  NEAR: the
// pair may be damped (x < 50); far pairs never are.
template <typename R, bool NEAR, bool VIR, bool FG>
__device__ __forceinline__ void force_pair(const SysView& s, int i, int j, const MP<R>& Mi,
                                           const MP<R>& Pi, const double xi[3], R si,
                                           const double4* mu, const float4* mu32, double F[3],
                                           double W[9], double E[3], double Gg[6]) {
  MP<R> Mj;
  R Rv[3], muj[3];
  double xj[3];
  load_mp_x64<R>(s, j, Mj, xj);
  load_mu<R>(mu, mu32, j, muj);
  sep64<R>(s, xi, xj, Rv);
  const R r2 = Rv[0] * Rv[0] + Rv[1] * Rv[1] + Rv[2] * Rv[2];
  const R rinv = dev_rsqrt<R>(r2), r = r2 * rinv, rinv2 = rinv * rinv;
  R c[6];
  base_coeffs<R, 5>(s, r, rinv, rinv2, c);
  bool damp = false;
  R D[6] = {R(0), R(0), R(0), R(0), R(0), R(0)};
  if (NEAR) {
    const R sj = site_s<R>(s, j);
    R x = R(0);
    damp = si > R(0) && sj > R(0) && (x = R(thole_a_pair(s, i, j)) * r2 * r * si * sj) < R(50);
    if (damp) {
      R tp[5], c0[5];
      thole_tp<R>(x, tp);
      bare_coeffs<R, 4>(rinv, rinv2, c0);
#pragma unroll
      for (int n = 1; n <= 4; ++n) {
        D[n] = tp[n] * c0[n];
        c[n] -= D[n];
      }
    }
  }
  MP<R> Pj = Mj;
  Pj.d[0] += muj[0]; Pj.d[1] += muj[1]; Pj.d[2] += muj[2];
  if (FG) {
    // site field and gradient of the same pair (see mp_field_grad)
    mp_field_grad<R>(c, Pj, Rv, E, Gg);
    if (NEAR && damp) mp_field_grad<R>(D, Mj, Rv, E, Gg);
  }
  R u, f[3];
  mp_pair<R, false, true>(c, Pi, Pj, Rv, u, f);
  double fd[3] = {(double)f[0], (double)f[1], (double)f[2]};
  F[0] += fd[0]; F[1] += fd[1]; F[2] += fd[2];
  if (NEAR && damp) {
    mp_pair<R, false, true>(D, Mi, Mj, Rv, u, f);
    F[0] += (double)f[0]; F[1] += (double)f[1]; F[2] += (double)f[2];
    if (VIR) {
      fd[0] += (double)f[0]; fd[1] += (double)f[1]; fd[2] += (double)f[2];
    }
  }
  if (VIR) {
    const double Rd[3] = {(double)Rv[0], (double)Rv[1], (double)Rv[2]};
    vir_add(W, fd, Rd);
  }
}

// Intermolecular pairs within the cutoff (precision R); adds to Fout.
// Near entries first (the damped ones are among them), then far ones.
template <typename R, int G, bool VIR, bool FG>
__global__ __launch_bounds__(kBlock) void k_force(SysView s, Reduce red, const double4* mu,
                                                  const float4* mu32, double4* Fout, double4* FS,
                                                  double* GS) {
  const int sub = threadIdx.x % G;
  const int i = blockIdx.x * (kBlock / G) + threadIdx.x / G;
  double F[3] = {0.0, 0.0, 0.0};
  double W[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
  double E[3] = {0.0, 0.0, 0.0}, Gg[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  if (i < s.n) {
    MP<R> Mi;
    R xr[3], mui[3];
    load_mp<R>(s, i, Mi, xr);
    const double4 p4 = s.sp[i];
    const double xi[3] = {p4.x, p4.y, p4.z};
    load_mu<R>(mu, mu32, i, mui);
    MP<R> Pi = Mi;
    Pi.d[0] += mui[0]; Pi.d[1] += mui[1]; Pi.d[2] += mui[2];
    const R si = site_s<R>(s, i);
    const int* row = s.nb_all + (size_t)i * s.cap_all;
    const int nn = s.nc_near[i], nf = s.nc_all[i] - nn;
    for (int k = sub; k < nn; k += G)
      force_pair<R, true, VIR, FG>(s, i, row[k], Mi, Pi, xi, si, mu, mu32, F, W, E, Gg);
    const int* far = row + s.cap_all - 1;
    int k = sub;
    for (; k + G < nf; k += 2 * G) {
      const int j0 = far[-k], j1 = far[-(k + G)];
      force_pair<R, false, VIR, FG>(s, i, j0, Mi, Pi, xi, si, mu, mu32, F, W, E, Gg);
      force_pair<R, false, VIR, FG>(s, i, j1, Mi, Pi, xi, si, mu, mu32, F, W, E, Gg);
    }
    if (k < nf)
      force_pair<R, false, VIR, FG>(s, i, far[-k], Mi, Pi, xi, si, mu, mu32, F, W, E, Gg);
  }
#pragma unroll
  for (int a = 0; a < 3; ++a) F[a] = group_sum<G>(F[a]);
  if (sub == 0 && i < s.n) {
    double4 f = Fout[i];
    f.x += F[0]; f.y += F[1]; f.z += F[2];
    Fout[i] = f;
  }
  if (FG) {
#pragma unroll
    for (int a = 0; a < 3; ++a) E[a] = group_sum<G>(E[a]);
#pragma unroll
    for (int k = 0; k < 6; ++k) Gg[k] = group_sum<G>(Gg[k]);
    if (sub == 0 && i < s.n) {
      double4 e = FS[i];
      e.x += E[0]; e.y += E[1]; e.z += E[2];
      FS[i] = e;
#pragma unroll
      for (int k = 0; k < 6; ++k) GS[6 * (size_t)i + k] += Gg[k];
    }
  }
  if (VIR) vir_partials(W, red, S_VRF);
}

// Same-molecule pairs (FP64, one thread per site): writes FS and GS.
__global__ __launch_bounds__(kBlock) void k_site_fg_intra(SysView s, const double4* mu,
                                                          double4* FS, double* GS) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= s.n) return;
  double E[3] = {0.0, 0.0, 0.0}, G[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  if (s.periodic) {
    MP<double> Mi;
    double xi[3];
    load_mp<double>(s, i, Mi, xi);
    const int cnt = s.nc_in[i];
    for (int k = 0; k < cnt; ++k) {
      const int j = s.nb_in[(size_t)i * s.cap_in + k];
      MP<double> Mj;
      double xj[3], Rv[3];
      load_mp<double>(s, j, Mj, xj);
      const double4 m = mu[j];
      Mj.d[0] += m.x; Mj.d[1] += m.y; Mj.d[2] += m.z;
      displacement<double>(s, xi, xj, Rv);
      const double r2 = Rv[0] * Rv[0] + Rv[1] * Rv[1] + Rv[2] * Rv[2];
      const double rinv = rsqrt(r2), r = r2 * rinv, rinv2 = rinv * rinv;
      double Eb[5], c0[5], c[6];
      ewald_coeffs<double, 4>(r, rinv, rinv2, s.beta, Eb);
      bare_coeffs<double, 4>(rinv, rinv2, c0);
#pragma unroll
      for (int n = 0; n < 5; ++n) c[n] = Eb[n] - c0[n];
      c[5] = 0.0;
      mp_field_grad<double>(c, Mj, Rv, E, G);
    }
  }
  FS[i] = make_double4(E[0], E[1], E[2], 0.0);
#pragma unroll
  for (int k = 0; k < 6; ++k) GS[6 * (size_t)i + k] = G[k];
}

// ------------------------------------------------------------------ launchers
constexpr int kG = 16;

static int blocks_for(int items, int G) {
  const int per = kBlock / G;
  int b = (items + per - 1) / per;
  return b < 1 ? 1 : b;
}

void launch_perm(const SysView& s, Reduce& red, double4* E0, bool mixed, hipStream_t st) {
  const dim3 gi((s.n + kBlock - 1) / kBlock);
  hipLaunchKernelGGL(k_perm_intra, gi, dim3(kBlock), 0, st, s, red, E0);
  red.nparts[S_AUX] = red.nparts[S_ESELF] = (int)gi.x;
  const dim3 g(blocks_for(s.n, kG)), b(kBlock);
  red.nparts[S_EREAL] = (int)g.x;
  if (mixed) hipLaunchKernelGGL((k_perm<float, kG>), g, b, 0, st, s, red, E0);
  else hipLaunchKernelGGL((k_perm<double, kG>), g, b, 0, st, s, red, E0);
}

void launch_matvec_real(const SysView& s, Reduce& red, const double4* p, const float4* p32,
                        double4* out, int dot_slot, bool mixed, hipStream_t st, hipEvent_t done,
                        hipEvent_t t0, hipEvent_t t1) {
  if (s.npol <= 0) {
    if (t0) (void)hipEventRecord(t0, st);
    if (t1) (void)hipEventRecord(t1, st);
    if (done) (void)hipEventRecord(done, st);
    return;
  }
  const dim3 g(blocks_for(s.npol, kG)), b(kBlock);
  // done: recorded by the kernel's own completion (no marker packet),
  // unless the completion event is taken by the timing pair
  hipEvent_t end = t1 ? t1 : done;
  if (mixed)
    hipExtLaunchKernelGGL((k_matvec<float, kG>), g, b, 0, st, t0, end, 0, s, red, p, p32, out,
                          dot_slot);
  else
    hipExtLaunchKernelGGL((k_matvec<double, kG>), g, b, 0, st, t0, end, 0, s, red, p, p32, out,
                          dot_slot);
  if (t1 && done) (void)hipEventRecord(done, st);
  if (!s.periodic && dot_slot >= 0) red.nparts[dot_slot] = (int)g.x;
}

template <int P>
static void matvec_recip_p(const SysView& s, const PmeView& pm, Reduce& red, const double4* p,
                           double4* out, int dot_slot, bool mixed, hipStream_t st) {
  const dim3 g((s.npol + kBlock - 1) / kBlock), b(kBlock);
  if (mixed) hipLaunchKernelGGL((k_matvec_recip<float, P>), g, b, 0, st, s, pm, red, p, out, dot_slot);
  else hipLaunchKernelGGL((k_matvec_recip<double, P>), g, b, 0, st, s, pm, red, p, out, dot_slot);
  if (dot_slot >= 0) red.nparts[dot_slot] = (int)g.x;
}

void launch_matvec_recip(const SysView& s, const PmeView& pm, Reduce& red, const double4* p,
                         double4* out, int dot_slot, bool mixed, hipStream_t st) {
  if (s.npol <= 0 || !s.periodic) return;
  switch (pm.order) {
    case 4: matvec_recip_p<4>(s, pm, red, p, out, dot_slot, mixed, st); break;
    case 6: matvec_recip_p<6>(s, pm, red, p, out, dot_slot, mixed, st); break;
    default: matvec_recip_p<5>(s, pm, red, p, out, dot_slot, mixed, st); break;
  }
}


void launch_pol_coef(const SysView& s, double2* out, float2* out32, double2* out_in,
                     hipStream_t st) {
  if (s.npol <= 0) return;
  const dim3 g(blocks_for(s.npol, kG)), b(kBlock);
  if (out) hipLaunchKernelGGL((k_pol_coef<double, kG>), g, b, 0, st, s, out, out32, out_in);
  else hipLaunchKernelGGL((k_pol_coef<float, kG>), g, b, 0, st, s, nullptr, out32, out_in);
}

template <bool VIR, bool FG>
static void force_kernels(const SysView& s, Reduce& red, const double4* mu, const float4* mu32,
                          double4* F, bool mixed, hipStream_t st, double4* FS, double* GS) {
  const dim3 gi((s.n + kBlock - 1) / kBlock), b(kBlock);
  const dim3 g(blocks_for(s.n, kG));
  if (FG)   // same-molecule part of the site fields first: it overwrites FS and GS
    hipLaunchKernelGGL(k_site_fg_intra, gi, b, 0, st, s, mu, FS, GS);
  hipLaunchKernelGGL(k_force_intra<VIR>, gi, b, 0, st, s, red, mu, F);
  if (mixed)
    hipLaunchKernelGGL((k_force<float, kG, VIR, FG>), g, b, 0, st, s, red, mu, mu32, F, FS, GS);
  else
    hipLaunchKernelGGL((k_force<double, kG, VIR, FG>), g, b, 0, st, s, red, mu, mu32, F, FS, GS);
  if (VIR)
    for (int k = 0; k < 9; ++k) {
      red.nparts[S_VRI + k] = (int)gi.x;
      red.nparts[S_VRF + k] = (int)g.x;
    }
}

void launch_force(const SysView& s, Reduce& red, const double4* mu, const float4* mu32, double4* F,
                  bool mixed, bool virial, hipStream_t st, double4* FS, double* GS) {
  const bool fg = FS != nullptr;
  if (virial) {
    if (fg) force_kernels<true, true>(s, red, mu, mu32, F, mixed, st, FS, GS);
    else force_kernels<true, false>(s, red, mu, mu32, F, mixed, st, FS, GS);
  } else {
    if (fg) force_kernels<false, true>(s, red, mu, mu32, F, mixed, st, FS, GS);
    else force_kernels<false, false>(s, red, mu, mu32, F, mixed, st, FS, GS);
  }
}

}  // namespace sibfa
