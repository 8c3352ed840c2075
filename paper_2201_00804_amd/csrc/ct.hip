// Reduced many-body charge transfer (paper: Many-Body Charge
// Transfer/Charge Delocalization, the reduced expression, Eq. 13-16):
//   E_ct = sum_l sum_k -n(l) (e1 - e2)^2 / dE,
//   e1 = exp(-eta rho1) (V_int(a1) - V_l) (C_s t + C_p m cos alpha),
//   e2 = exp(-eta rho2) (V_int(a2) - V_l) (C_s t + C_p m cos beta),
//   dE = ae(l) + V_l - ah(k),
// over lone pairs l (carried by atom c) and acceptor bonds k = (a1, a2) of
// other molecules with |r_c - r_a1| inside the real-space cutoff; rho the
// distances c-a over 2 sqrt(rvdw_c rvdw_a), alpha and beta the angles at c
// between the lone pair and a1, a2.  V_l is the potential of the other
// molecules' permanent multipoles at the lone pair (Ewald-summed when
// periodic, own molecule excluded); V_int(a) the bare potential at atom a
// of its own molecule's other sites.  Potentials enter in kcal/mol per
// unit charge.  Everything runs in FP64.
//
//  k_ct_flags     : per sorted site, what it is (an a1, a carrier, has
//                   multipoles) and its acceptor and lone-pair ranges, so
//                   list scans test one word per entry.
//  k_ct_records   : per lone pair and per acceptor, one 64-byte record of
//                   what a pair needs from that side.
//  k_ct_vlp       : real-space part of V_l.
//  k_ct_vint      : V_int at the acceptor atoms.
//  k_ct_gather_pot: reciprocal V_l and its gradient from the PME grid.
//  k_ct_pairs_lp  : per lone pair over its carrier's neighbours: the energy,
//                   w_l = dE/dV_l, the direct forces on l and c.
//  k_ct_pairs_acc : per acceptor over a1's neighbours (the same pairs): the
//                   direct forces on a1, a2 and u_a = dE/dV_int(a).
//  k_ct_collect   : per site, its share of all of these (fixed order).
//  k_ct_wforce_*  : -grad of sum_l w_l V_l + sum_a u_a V_int(a) in real
//                   space: point charges w at the lone pairs (and u at the
//                   acceptor atoms, own molecule, bare) against the
//                   permanent multipoles.  The reciprocal part of the w
//                   charges goes through the ordinary PME force gather.
//
// The list passes run one wave per lone pair, acceptor or site.  Only a
// fraction of a site's neighbours take part (acceptor H atoms, lone-pair
// carriers, lone pairs), so the wave compacts the entries that do into a
// ring in LDS, in list order, and evaluates them 64 at a time with every
// lane busy; per-lane sums in a fixed order and a fixed reduction tree keep
// the results reproducible.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "common.h"
#include "pairmath.h"
#include "kernels.h"

namespace sibfa {

namespace {

constexpr int kRing = 128;                 // LDS ring slots per wave
constexpr int kWaves = kBlock / 64;

// bits of CtArgs::flag_s
constexpr int kIsA1 = 1;        // a1 of at least one acceptor
constexpr int kIsCarrier = 2;   // carries at least one lone pair
constexpr int kHasMult = 4;     // nonzero permanent multipoles

// One wave walks entries [0, nt) of a list, kScanU chunks of 64 per step
// (the loads of a step issue together; more chunks hide more latency and
// hold more registers).  hit(k, v) tells whether entry k
// takes part and sets the value v to queue; queued values keep list order
// in a ring of kRing slots, and whenever 64 are queued every lane takes one
// and runs eval(v).  What is left runs at the end on the first lanes.  The
// whole wave calls it with the same nt.
template <int kScanU, class Hit, class Eval>
__device__ __forceinline__ void wave_compact(int nt, int* ring, Hit hit, Eval eval) {
  const int lane = threadIdx.x & 63;
  int head = 0, tail = 0;   // wave-uniform
  for (int base = 0; base < nt; base += 64 * kScanU) {
    int v[kScanU];
    bool h[kScanU];
#pragma unroll
    for (int u = 0; u < kScanU; ++u) {
      const int k = base + 64 * u + lane;
      h[u] = hit(min(k, nt - 1), v[u]) && k < nt;   // clamped: every lane loads
    }
#pragma unroll
    for (int u = 0; u < kScanU; ++u) {
      const unsigned long long m = __ballot(h[u]);
      if (h[u]) ring[(tail + lanes_below(m, 0)) & (kRing - 1)] = v[u];
      tail += __popcll(m);   // at most 63 + 64 < kRing queued
      wave_sync();
      if (tail - head >= 64) {
        eval(ring[(head + lane) & (kRing - 1)]);
        head += 64;
        wave_sync();   // the next chunk may overwrite the slots just read
      }
    }
  }
  if (lane < tail - head) eval(ring[(head + lane) & (kRing - 1)]);
}

__device__ __forceinline__ void site_pos(const SysView& s, int i, double x[3]) {
  const double4 p = s.sp[i];
  x[0] = p.x; x[1] = p.y; x[2] = p.z;
}

__device__ __forceinline__ void rec_mp(const SysView& s, int j, MP<double>& M, double x[3]) {
  const double4 p = s.sp[j], d = s.sd[j], t = s.sth[j];
  const double2 t2 = s.sth2[j];
  x[0] = p.x; x[1] = p.y; x[2] = p.z;
  M.q = p.w;
  M.d[0] = d.x; M.d[1] = d.y; M.d[2] = d.z;
  M.t[0] = t.x; M.t[1] = t.y; M.t[2] = t.z; M.t[3] = t.w; M.t[4] = t2.x; M.t[5] = t2.y;
}

__device__ __forceinline__ void sep(const SysView& s, const double a[3], const double b[3],
                                    double R[3]) {
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    double d = a[k] - b[k];
    if (s.periodic) d = min_image<double>(d, s.box[k], s.ibox[k]);
    R[k] = d;
  }
}

// Potential at R (= r - r_j) of multipoles M: q c0 + (d.R) c1 + 1/3 (R Theta R) c2.
__device__ __forceinline__ double mp_potential(const double c[3], const MP<double>& M,
                                               const double R[3]) {
  double tr[3];
  tvec(M.t, R, tr);
  const double rtr = tr[0] * R[0] + tr[1] * R[1] + tr[2] * R[2];
  return M.q * c[0] + (M.d[0] * R[0] + M.d[1] * R[1] + M.d[2] * R[2]) * c[1] +
         (1.0 / 3.0) * rtr * c[2];
}

// Field at r_i of multipoles M at r_j, R = r_i - r_j, from coefficients
// c[0..3] with grad c_n = -R c_{n+1}: minus the gradient of mp_potential,
//   E = (q c1 + (d.R) c2 + 1/3 (R Theta R) c3) R - d c1 - 2/3 (Theta R) c2.
// A point charge w at r_i feels w E; the multipoles feel the reaction.
__device__ __forceinline__ void mp_field(const double c[4], const MP<double>& M,
                                        const double R[3], double E[3]) {
  double tr[3];
  tvec(M.t, R, tr);
  const double dr = M.d[0] * R[0] + M.d[1] * R[1] + M.d[2] * R[2];
  const double rtr = tr[0] * R[0] + tr[1] * R[1] + tr[2] * R[2];
  const double rad = M.q * c[1] + dr * c[2] + (1.0 / 3.0) * rtr * c[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) E[k] = rad * R[k] - M.d[k] * c[1] - (2.0 / 3.0) * tr[k] * c[2];
}

// Entry k of site i's intermolecular list (near entries, then far ones
// stored from the row's end).
__device__ __forceinline__ int all_entry(const SysView& s, int i, int k, int nn) {
  const int* row = s.nb_all + (size_t)i * s.cap_all;
  return k < nn ? row[k] : row[s.cap_all - 1 - (k - nn)];
}

struct CtPair {
  double E, dV, dVi1, dVi2;
  double gL[3], gC[3], gA1[3], gA2[3];   // dE/dr of l, c, a1, a2
};

// The lone-pair side of a pair (potentials already times the Coulomb
// constant) and the acceptor side.
struct LpSide {
  double xL[3], xc[3], VL, nocc, ae, rvc;
};
struct AccSide {
  double x1[3], x2[3], V1, V2, rv1, rv2, ah;
};

__device__ __forceinline__ void load_lp(const CtArgs& a, int p, LpSide& l) {
  const double4* r = reinterpret_cast<const double4*>(a.lp_rec) + 2 * (size_t)p;
  const double4 r0 = r[0], r1 = r[1];
  l.xL[0] = r0.x; l.xL[1] = r0.y; l.xL[2] = r0.z; l.VL = r0.w;
  l.nocc = r1.x; l.ae = r1.y; l.rvc = r1.z;
}

__device__ __forceinline__ void load_acc(const CtArgs& a, int k, AccSide& q) {
  const double4* r = reinterpret_cast<const double4*>(a.acc_rec) + 2 * (size_t)k;
  const double4 r0 = r[0], r1 = r[1];
  q.x2[0] = r0.x; q.x2[1] = r0.y; q.x2[2] = r0.z; q.V1 = r0.w;
  q.V2 = r1.x; q.rv1 = r1.y; q.rv2 = r1.z; q.ah = r1.w;
}

// Everything of one (lone pair, acceptor) pair.
__device__ __forceinline__ void ct_pair(const SysView& s, const CtArgs& a, const LpSide& l,
                                        const AccSide& q, CtPair& o) {
  double u[3], d1[3], d2[3];
  sep(s, l.xL, l.xc, u);
  sep(s, q.x1, l.xc, d1);
  sep(s, q.x2, l.xc, d2);
  // reciprocal lengths (one rsqrt each) in place of the divisions
  const double inu = rsqrt(u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
  const double ir1 = rsqrt(d1[0] * d1[0] + d1[1] * d1[1] + d1[2] * d1[2]);
  const double ir2 = rsqrt(d2[0] * d2[0] + d2[1] * d2[1] + d2[2] * d2[2]);
  const double r1 = (d1[0] * d1[0] + d1[1] * d1[1] + d1[2] * d1[2]) * ir1;
  const double r2 = (d2[0] * d2[0] + d2[1] * d2[1] + d2[2] * d2[2]) * ir2;
  // eta / s = eta / (2 sqrt(rvdw_c rvdw_a))
  const double es1 = 0.5 * a.eta * rsqrt(l.rvc * q.rv1), es2 = 0.5 * a.eta * rsqrt(l.rvc * q.rv2);
  const double ud1 = u[0] * d1[0] + u[1] * d1[1] + u[2] * d1[2];
  const double ud2 = u[0] * d2[0] + u[1] * d2[1] + u[2] * d2[2];
  const double ca = ud1 * inu * ir1, cb = ud2 * inu * ir2;
  const double ex1 = exp(-es1 * r1), ex2 = exp(-es2 * r2);
  const double VL = l.VL;
  const double X1 = q.V1 - VL, X2 = q.V2 - VL;
  const double g1 = a.cs * a.t + a.cp * a.m * ca, g2 = a.cs * a.t + a.cp * a.m * cb;
  const double e1 = ex1 * X1 * g1, e2 = ex2 * X2 * g2;
  const double nocc = l.nocc, idE = 1.0 / (l.ae + VL - q.ah);
  const double diff = e1 - e2;
  const double G = -2.0 * nocc * diff * idE;   // dE/de1; dE/de2 = -G
  o.E = 0.5 * G * diff;                        // -n (e1 - e2)^2 / dE
  const double GD = -o.E * idE;                // dE/d(dE) = n (e1 - e2)^2 / dE^2
  o.dV = kCoulomb * (-G * ex1 * g1 + G * ex2 * g2 + GD);
  o.dVi1 = kCoulomb * G * ex1 * g1;
  o.dVi2 = -kCoulomb * G * ex2 * g2;
  const double k1 = G * ex1 * X1 * a.cp * a.m;    // dE/dcos(alpha)
  const double k2 = -G * ex2 * X2 * a.cp * a.m;   // dE/dcos(beta)
  const double r1e = -G * es1 * e1;               // dE/dr1
  const double r2e = G * es2 * e2;                // dE/dr2
  const double inu1 = inu * ir1, inu2 = inu * ir2, inu_sq = inu * inu;
  const double ir1_sq = ir1 * ir1, ir2_sq = ir2 * ir2;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const double dca_du = d1[c] * inu1 - ca * u[c] * inu_sq;
    const double dcb_du = d2[c] * inu2 - cb * u[c] * inu_sq;
    const double dca_dd1 = u[c] * inu1 - ca * d1[c] * ir1_sq;
    const double dcb_dd2 = u[c] * inu2 - cb * d2[c] * ir2_sq;
    o.gL[c] = k1 * dca_du + k2 * dcb_du;
    o.gA1[c] = r1e * d1[c] * ir1 + k1 * dca_dd1;
    o.gA2[c] = r2e * d2[c] * ir2 + k2 * dcb_dd2;
    o.gC[c] = -(o.gL[c] + o.gA1[c] + o.gA2[c]);
  }
}

}  // namespace

// What each sorted site is, for the list scans.
__global__ __launch_bounds__(kBlock) void k_ct_flags(SysView s, CtArgs a) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= s.n) return;
  const int c = a.perm[i];
  const double4 p = s.sp[i], d = s.sd[i], t = s.sth[i];
  const double2 t2 = s.sth2[i];
  const bool mult = p.w != 0.0 || d.x != 0.0 || d.y != 0.0 || d.z != 0.0 || t.x != 0.0 ||
                    t.y != 0.0 || t.z != 0.0 || t.w != 0.0 || t2.x != 0.0 || t2.y != 0.0;
  const int a0 = a.a1_start[c], a1 = a.a1_start[c + 1];
  const int c0 = a.car_start[c], c1 = a.car_start[c + 1];
  a.flag_s[i] = (a1 > a0 ? kIsA1 : 0) | (c1 > c0 ? kIsCarrier : 0) | (mult ? kHasMult : 0);
  a.rng_s[i] = make_int4(a0, a1, c0, c1);
}

// The side records of the lone pairs (after V_l is complete) and of the
// acceptors (after V_int).
__global__ __launch_bounds__(kBlock) void k_ct_records(SysView s, CtArgs a) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < a.n_lp) {
    const int c = a.lp[2 * t + 1];
    const double4 x = s.sp[a.inv_perm[a.lp[2 * t]]];
    double4* r = reinterpret_cast<double4*>(a.lp_rec) + 2 * (size_t)t;
    r[0] = make_double4(x.x, x.y, x.z, kCoulomb * a.Vlp[t]);
    r[1] = make_double4(a.lp_par[2 * t], a.lp_par[2 * t + 1], a.rvdw[c], 0.0);
  }
  if (t < a.n_acc) {
    const int a1 = a.acc[2 * t], a2 = a.acc[2 * t + 1];
    const double4 x = s.sp[a.inv_perm[a2]];
    double4* r = reinterpret_cast<double4*>(a.acc_rec) + 2 * (size_t)t;
    r[0] = make_double4(x.x, x.y, x.z, kCoulomb * a.Vint[a1]);
    r[1] = make_double4(kCoulomb * a.Vint[a2], a.rvdw[a1], a.rvdw[a2], a.ah[t]);
  }
}

// Real-space part of V_l: the other molecules within the cutoff (Ewald or
// bare kernel) and, periodic, the excluded own-molecule correction.  One
// wave per lone pair over the neighbours that carry multipoles.
__global__ __launch_bounds__(kBlock) void k_ct_vlp(SysView s, CtArgs a) {
  __shared__ int ring[kWaves][kRing];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int p = blockIdx.x * kWaves + wv;
  if (p >= a.n_lp) return;   // wave-uniform; no block-wide barrier follows
  const int i = a.inv_perm[a.lp[2 * p]];
  double xi[3];
  site_pos(s, i, xi);
  double V = 0.0;
  const int nn = s.nc_near[i];
  wave_compact<4>(
      s.nc_all[i], ring[wv],
      [&](int k, int& v) {
        v = all_entry(s, i, k, nn);
        return (a.flag_s[v] & kHasMult) != 0;
      },
      [&](int j) {
        MP<double> M;
        double xj[3], R[3];
        rec_mp(s, j, M, xj);
        sep(s, xi, xj, R);
        const double r2 = R[0] * R[0] + R[1] * R[1] + R[2] * R[2];
        const double rinv = rsqrt(r2), r = r2 * rinv, rinv2 = rinv * rinv;
        double c[3];
        if (s.periodic) ewald_coeffs<double, 2>(r, rinv, rinv2, s.beta, c);
        else bare_coeffs<double, 2>(rinv, rinv2, c);
        V += mp_potential(c, M, R);
      });
  if (s.periodic)
    for (int k = lane; k < s.nc_in[i]; k += 64) {
      const int j = s.nb_in[(size_t)i * s.cap_in + k];
      MP<double> M;
      double xj[3], R[3];
      rec_mp(s, j, M, xj);
      sep(s, xi, xj, R);
      const double r2 = R[0] * R[0] + R[1] * R[1] + R[2] * R[2];
      const double rinv = rsqrt(r2), r = r2 * rinv, rinv2 = rinv * rinv;
      double B[3], c0[3], c[3];
      ewald_coeffs<double, 2>(r, rinv, rinv2, s.beta, B);
      bare_coeffs<double, 2>(rinv, rinv2, c0);
#pragma unroll
      for (int n = 0; n < 3; ++n) c[n] = B[n] - c0[n];
      V += mp_potential(c, M, R);
    }
  V = wave_sum(V);
  if (lane == 0) a.Vlp[p] = V;
}

// V_int at the acceptor atoms: bare potential of the own molecule's other
// sites.
__global__ __launch_bounds__(kBlock) void k_ct_vint(SysView s, CtArgs a) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= a.n_vint) return;
  const int site = a.vint_sites[t];
  const int i = a.inv_perm[site];
  const double4 pi = s.sp[i];
  const double xi[3] = {pi.x, pi.y, pi.z};
  double V = 0.0;
  for (int k = 0; k < s.nc_in[i]; ++k) {
    const int j = s.nb_in[(size_t)i * s.cap_in + k];
    MP<double> M;
    double xj[3], R[3];
    rec_mp(s, j, M, xj);
    sep(s, xi, xj, R);
    const double r2 = R[0] * R[0] + R[1] * R[1] + R[2] * R[2];
    const double rinv = rsqrt(r2), rinv2 = rinv * rinv;
    double c[3];
    bare_coeffs<double, 2>(rinv, rinv2, c);
    V += mp_potential(c, M, R);
  }
  a.Vint[site] = V;
}

// Reciprocal potential and its gradient at the lone pairs (from the grid of
// the permanent multipoles).
template <int P>
__global__ __launch_bounds__(kBlock) void k_ct_gather_pot(SysView s, PmeView pm, CtArgs a) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= a.n_lp) return;
  const double4 x = s.sp[a.inv_perm[a.lp[2 * p]]];
  int base[3];
  double th[3][2][P];
  site_splines<double, P, 1>(pm, x.x, x.y, x.z, base, th);
  double phi = 0.0, g[3] = {0.0, 0.0, 0.0};
  for (int tz = 0; tz < P; ++tz) {
    int iz = base[2] - tz; if (iz < 0) iz += pm.K[2];
    for (int ty = 0; ty < P; ++ty) {
      int iy = base[1] - ty; if (iy < 0) iy += pm.K[1];
      const size_t row = ((size_t)iz * pm.K[1] + iy) * pm.K[0];
      double s0 = 0.0, s1 = 0.0;
#pragma unroll
      for (int tx = 0; tx < P; ++tx) {
        int ix = base[0] - tx; if (ix < 0) ix += pm.K[0];
        const double v = pm.phi[row + ix];
        s0 += v * th[0][0][tx];
        s1 += v * th[0][1][tx];
      }
      phi += s0 * th[1][0][ty] * th[2][0][tz];
      g[0] += s1 * th[1][0][ty] * th[2][0][tz];
      g[1] += s0 * th[1][1][ty] * th[2][0][tz];
      g[2] += s0 * th[1][0][ty] * th[2][1][tz];
    }
  }
  a.Vlp[p] += phi;
#pragma unroll
  for (int q = 0; q < 3; ++q) a.Gr[3 * (size_t)p + q] = g[q] * pm.scale[q];
}

// Per lone pair (one wave): the acceptors whose a1 is among the carrier's
// neighbours.
__global__ __launch_bounds__(kBlock) void k_ct_pairs_lp(SysView s, CtArgs a, Reduce red) {
  __shared__ int ring[kWaves][kRing];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int p = blockIdx.x * kWaves + wv;
  double E = 0.0, w = 0.0, FL[3] = {0.0, 0.0, 0.0}, FC[3] = {0.0, 0.0, 0.0};
  if (p < a.n_lp) {   // wave-uniform
    const int i = a.inv_perm[a.lp[2 * p + 1]];
    LpSide l;
    load_lp(a, p, l);
    site_pos(s, i, l.xc);
    const int nn = s.nc_near[i];
    const int2* rng = reinterpret_cast<const int2*>(a.rng_s);   // [2 j]: a1 range
    wave_compact<4>(
        s.nc_all[i], ring[wv],
        [&](int e, int& v) {
          v = all_entry(s, i, e, nn);
          const int2 r = rng[2 * (size_t)v];
          return r.y > r.x;
        },
        [&](int j) {
          AccSide q;
          site_pos(s, j, q.x1);
          const int2 rg = rng[2 * (size_t)j];
          for (int r = rg.x; r < rg.y; ++r) {
            load_acc(a, a.a1_ref[r], q);
            CtPair o;
            ct_pair(s, a, l, q, o);
            E += o.E;
            w += o.dV;
#pragma unroll
            for (int c = 0; c < 3; ++c) {
              FL[c] -= o.gL[c];
              FC[c] -= o.gC[c];
            }
          }
        });
  }
  E = wave_sum(E);
  w = wave_sum(w);
#pragma unroll
  for (int q = 0; q < 3; ++q) {
    FL[q] = wave_sum(FL[q]);
    FC[q] = wave_sum(FC[q]);
  }
  if (lane == 0 && p < a.n_lp) {
    a.w[p] = w;
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      a.Fl[3 * (size_t)p + q] = FL[q];
      a.Fc[3 * (size_t)p + q] = FC[q];
    }
  } else {
    E = 0.0;
  }
  block_partial(E, red, S_ECT);
}

// Per acceptor (one wave): the lone pairs carried by a1's neighbours.
__global__ __launch_bounds__(kBlock) void k_ct_pairs_acc(SysView s, CtArgs a) {
  __shared__ int ring[kWaves][kRing];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int k = blockIdx.x * kWaves + wv;
  if (k >= a.n_acc) return;   // wave-uniform; no block-wide barrier follows
  double F1[3] = {0.0, 0.0, 0.0}, F2[3] = {0.0, 0.0, 0.0}, u1 = 0.0, u2 = 0.0;
  const int i = a.inv_perm[a.acc[2 * k]];
  AccSide q;
  load_acc(a, k, q);
  site_pos(s, i, q.x1);
  const int nn = s.nc_near[i];
  const int2* rng = reinterpret_cast<const int2*>(a.rng_s);   // [2 j + 1]: carrier range
  wave_compact<4>(
      s.nc_all[i], ring[wv],
      [&](int e, int& v) {
        v = all_entry(s, i, e, nn);
        const int2 r = rng[2 * (size_t)v + 1];
        return r.y > r.x;
      },
      [&](int j) {
        LpSide l;
        site_pos(s, j, l.xc);
        const int2 rg = rng[2 * (size_t)j + 1];
        for (int r = rg.x; r < rg.y; ++r) {
          load_lp(a, a.car_ref[r], l);
          CtPair o;
          ct_pair(s, a, l, q, o);
          u1 += o.dVi1;
          u2 += o.dVi2;
#pragma unroll
          for (int c = 0; c < 3; ++c) {
            F1[c] -= o.gA1[c];
            F2[c] -= o.gA2[c];
          }
        }
      });
  u1 = wave_sum(u1);
  u2 = wave_sum(u2);
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    F1[c] = wave_sum(F1[c]);
    F2[c] = wave_sum(F2[c]);
  }
  if (lane == 0) {
    a.ua[2 * (size_t)k] = u1;
    a.ua[2 * (size_t)k + 1] = u2;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      a.Fa[6 * (size_t)k + c] = F1[c];
      a.Fa[6 * (size_t)k + 3 + c] = F2[c];
    }
  }
}

// Per site (caller order c): w, u and the direct forces, in sorted order.
// A lone pair also takes the reciprocal part of -w grad V_l here.
__global__ __launch_bounds__(kBlock) void k_ct_collect(CtArgs a) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= a.n) return;
  double F[3] = {0.0, 0.0, 0.0}, W = 0.0, U = 0.0;
  const int p = a.lp_of[c];
  if (p >= 0) {
    W = a.w[p];
#pragma unroll
    for (int q = 0; q < 3; ++q) F[q] += a.Fl[3 * (size_t)p + q] - W * a.Gr[3 * (size_t)p + q];
  }
  for (int r = a.car_start[c]; r < a.car_start[c + 1]; ++r) {
    const int pl = a.car_ref[r];
#pragma unroll
    for (int q = 0; q < 3; ++q) F[q] += a.Fc[3 * (size_t)pl + q];
  }
  for (int r = a.at_start[c]; r < a.at_start[c + 1]; ++r) {
    const int ks = a.at_ref[r];   // 2 k + slot
    U += a.ua[ks];
#pragma unroll
    for (int q = 0; q < 3; ++q) F[q] += a.Fa[3 * (size_t)ks + q];
  }
  const int i = a.inv_perm[c];
  a.W_s[i] = W;
  a.U_s[i] = U;
  a.F_s[i] = make_double4(F[0], F[1], F[2], 0.0);
}

// -grad of sum_l w_l V_l + sum_a u_a V_int(a) in real space, added to F_s
// by three passes: the w of each lone pair against its neighbours'
// multipoles (k_ct_wforce_lp), the multipoles of each site against the
// neighbours' w (k_ct_wforce_mp), and the own-molecule terms, which also
// leave F_s divided by the Coulomb constant, the unit of the reciprocal
// gather that multiplies by it (k_ct_wforce_in).  Split so that each list
// pass holds one set of multipoles in registers.
__global__ __launch_bounds__(kBlock) void k_ct_wforce_lp(SysView s, CtArgs a) {
  __shared__ int ring[kWaves][kRing];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int p = blockIdx.x * kWaves + wv;
  if (p >= a.n_lp) return;   // wave-uniform; no block-wide barrier follows
  const int i = a.inv_perm[a.lp[2 * p]];
  const double Wi = a.W_s[i];
  if (Wi == 0.0) return;
  double xi[3];
  site_pos(s, i, xi);
  double F[3] = {0.0, 0.0, 0.0};
  const int nn = s.nc_near[i];
  wave_compact<4>(
      s.nc_all[i], ring[wv],
      [&](int k, int& v) {
        v = all_entry(s, i, k, nn);
        return (a.flag_s[v] & kHasMult) != 0;
      },
      [&](int j) {
        MP<double> Mj;
        double xj[3], R[3];
        rec_mp(s, j, Mj, xj);
        sep(s, xi, xj, R);
        const double r2 = R[0] * R[0] + R[1] * R[1] + R[2] * R[2];
        const double rinv = rsqrt(r2), r = r2 * rinv, rinv2 = rinv * rinv;
        double c[4], E[3];
        if (s.periodic) ewald_coeffs<double, 3>(r, rinv, rinv2, s.beta, c);
        else bare_coeffs<double, 3>(rinv, rinv2, c);
        mp_field(c, Mj, R, E);
        F[0] += E[0]; F[1] += E[1]; F[2] += E[2];
      });
#pragma unroll
  for (int q = 0; q < 3; ++q) F[q] = Wi * wave_sum(F[q]);
  if (lane == 0) {
    const double4 d = a.F_s[i];
    a.F_s[i] = make_double4(d.x + F[0], d.y + F[1], d.z + F[2], 0.0);
  }
}

// FG: also the field E and field gradient G of the w charges at r_i
// (every site, zero at sites without multipoles), divided by the Coulomb
// constant, into FS, GS.
template <bool FG>
__global__ __launch_bounds__(kBlock) void k_ct_wforce_mp(SysView s, CtArgs a, double4* FS,
                                                         double* GS) {
  __shared__ int ring[kWaves][kRing];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int i = blockIdx.x * kWaves + wv;
  if (i >= s.n) return;   // wave-uniform; no block-wide barrier follows
  if ((a.flag_s[i] & kHasMult) == 0) {
    if (FG && lane < 6) {
      if (lane == 0) FS[i] = make_double4(0.0, 0.0, 0.0, 0.0);
      GS[6 * (size_t)i + lane] = 0.0;
    }
    return;
  }
  MP<double> Mi;
  double xi[3];
  rec_mp(s, i, Mi, xi);
  double F[3] = {0.0, 0.0, 0.0}, E[3] = {0.0, 0.0, 0.0}, G[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  const int nn = s.nc_near[i];
  wave_compact<4>(
      s.nc_all[i], ring[wv],
      [&](int k, int& v) {
        v = all_entry(s, i, k, nn);
        return a.W_s[v] != 0.0;
      },
      [&](int j) {
        double xj[3], R[3];
        site_pos(s, j, xj);
        sep(s, xj, xi, R);   // r_j - r_i: the field of M_i at the charge
        const double r2 = R[0] * R[0] + R[1] * R[1] + R[2] * R[2];
        const double rinv = rsqrt(r2), r = r2 * rinv, rinv2 = rinv * rinv;
        double c[4], Ej[3];
        if (s.periodic) ewald_coeffs<double, 3>(r, rinv, rinv2, s.beta, c);
        else bare_coeffs<double, 3>(rinv, rinv2, c);
        mp_field(c, Mi, R, Ej);
        const double wj = a.W_s[j];
        F[0] -= wj * Ej[0]; F[1] -= wj * Ej[1]; F[2] -= wj * Ej[2];
        if (FG) {   // the charge's field at r_i: -w c1 R, gradient w (c1 I - c2 R R)
          const double w1 = wj * c[1], w2 = wj * c[2];
#pragma unroll
          for (int q = 0; q < 3; ++q) E[q] -= w1 * R[q];
          G[0] += w1 - w2 * R[0] * R[0];
          G[1] -= w2 * R[0] * R[1];
          G[2] -= w2 * R[0] * R[2];
          G[3] += w1 - w2 * R[1] * R[1];
          G[4] -= w2 * R[1] * R[2];
          G[5] += w1 - w2 * R[2] * R[2];
        }
      });
#pragma unroll
  for (int q = 0; q < 3; ++q) F[q] = wave_sum(F[q]);
  if (lane == 0) {
    const double4 d = a.F_s[i];
    a.F_s[i] = make_double4(d.x + F[0], d.y + F[1], d.z + F[2], 0.0);
  }
  if (FG) {
    const double sc = 1.0 / kCoulomb;
#pragma unroll
    for (int q = 0; q < 3; ++q) E[q] = wave_sum(E[q]) * sc;
#pragma unroll
    for (int q = 0; q < 6; ++q) G[q] = wave_sum(G[q]) * sc;
    if (lane == 0) FS[i] = make_double4(E[0], E[1], E[2], 0.0);
    if (lane < 6) {
      double g = G[0];
#pragma unroll
      for (int q = 1; q < 6; ++q) g = lane == q ? G[q] : g;
      GS[6 * (size_t)i + lane] = g;
    }
  }
}

// Own molecule (one thread per site): the u charges of V_int (bare) and,
// periodic, the part of the reciprocal sum of the w charges that V_l
// excludes (coefficients B - c0); then F_s / Coulomb.
template <bool FG>
__global__ __launch_bounds__(kBlock) void k_ct_wforce_in(SysView s, CtArgs a, double4* FS,
                                                         double* GS) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= s.n) return;
  double F[3] = {0.0, 0.0, 0.0}, Ef[3] = {0.0, 0.0, 0.0}, G[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  const double Wi = a.W_s[i], Ui = a.U_s[i];
  for (int k = 0; k < s.nc_in[i]; ++k) {
    const int j = s.nb_in[(size_t)i * s.cap_in + k];
    const double Wj = a.W_s[j], Uj = a.U_s[j];
    // charge at i (u bare; w periodic, B - c0) against the multipoles at j,
    // and the reverse
    const double qi_b = Ui, qj_b = Uj;
    const double qi_x = s.periodic ? Wi : 0.0, qj_x = s.periodic ? Wj : 0.0;
    if (qi_b == 0.0 && qj_b == 0.0 && qi_x == 0.0 && qj_x == 0.0) continue;
    double xi[3], xj[3], R[3];
    site_pos(s, i, xi);
    site_pos(s, j, xj);
    sep(s, xi, xj, R);
    const double r2 = R[0] * R[0] + R[1] * R[1] + R[2] * R[2];
    const double rinv = rsqrt(r2), r = r2 * rinv, rinv2 = rinv * rinv;
    double c0[4], cx[4] = {0.0, 0.0, 0.0, 0.0};
    bare_coeffs<double, 3>(rinv, rinv2, c0);
    if (qi_x != 0.0 || qj_x != 0.0) {
      double B[4];
      ewald_coeffs<double, 3>(r, rinv, rinv2, s.beta, B);
#pragma unroll
      for (int n = 0; n < 4; ++n) cx[n] = B[n] - c0[n];
    }
    if (FG) {   // the field at r_i of the charges at r_j and its gradient
      const double e1 = qj_b * c0[1] + (qj_x != 0.0 ? qj_x * cx[1] : 0.0);
      const double e2 = qj_b * c0[2] + (qj_x != 0.0 ? qj_x * cx[2] : 0.0);
#pragma unroll
      for (int q = 0; q < 3; ++q) Ef[q] += e1 * R[q];
      G[0] += e1 - e2 * R[0] * R[0];
      G[1] -= e2 * R[0] * R[1];
      G[2] -= e2 * R[0] * R[2];
      G[3] += e1 - e2 * R[1] * R[1];
      G[4] -= e2 * R[1] * R[2];
      G[5] += e1 - e2 * R[2] * R[2];
    }
    double E[3];
    if (qi_b != 0.0 || qi_x != 0.0) {   // field of M_j at r_i
      MP<double> Mj;
      double y[3];
      rec_mp(s, j, Mj, y);
      if (qi_b != 0.0) {
        mp_field(c0, Mj, R, E);
#pragma unroll
        for (int q = 0; q < 3; ++q) F[q] += qi_b * E[q];
      }
      if (qi_x != 0.0) {
        mp_field(cx, Mj, R, E);
#pragma unroll
        for (int q = 0; q < 3; ++q) F[q] += qi_x * E[q];
      }
    }
    if (qj_b != 0.0 || qj_x != 0.0) {   // field of M_i at r_j, reaction on i
      MP<double> Mi;
      double y[3];
      rec_mp(s, i, Mi, y);
      const double Rn[3] = {-R[0], -R[1], -R[2]};
      if (qj_b != 0.0) {
        mp_field(c0, Mi, Rn, E);
#pragma unroll
        for (int q = 0; q < 3; ++q) F[q] -= qj_b * E[q];
      }
      if (qj_x != 0.0) {
        mp_field(cx, Mi, Rn, E);
#pragma unroll
        for (int q = 0; q < 3; ++q) F[q] -= qj_x * E[q];
      }
    }
  }
  const double4 d = a.F_s[i];
  const double sc = 1.0 / kCoulomb;
  a.F_s[i] = make_double4((d.x + F[0]) * sc, (d.y + F[1]) * sc, (d.z + F[2]) * sc, 0.0);
  if (FG) {
    const double4 e = FS[i];
    FS[i] = make_double4(e.x + Ef[0] * sc, e.y + Ef[1] * sc, e.z + Ef[2] * sc, 0.0);
#pragma unroll
    for (int q = 0; q < 6; ++q) GS[6 * (size_t)i + q] += G[q] * sc;
  }
}

// The w charges (divided by the Coulomb constant) as the only amplitude of
// an alternative record set for the spreading kernel.
__global__ __launch_bounds__(kBlock) void k_ct_wrecords(SysView s, CtArgs a, double4* sp_w) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= s.n) return;
  const double4 p = s.sp[i];
  sp_w[i] = make_double4(p.x, p.y, p.z, a.W_s[i] * (1.0 / kCoulomb));
}

void launch_ct_potentials(const SysView& s, const CtArgs& a, hipStream_t st) {
  const dim3 b(kBlock);
  hipLaunchKernelGGL(k_ct_flags, dim3((s.n + kBlock - 1) / kBlock), b, 0, st, s, a);
  if (a.n_lp > 0)
    hipLaunchKernelGGL(k_ct_vlp, dim3((a.n_lp + kWaves - 1) / kWaves), b, 0, st, s, a);
  if (a.n_vint > 0)
    hipLaunchKernelGGL(k_ct_vint, dim3((a.n_vint + kBlock - 1) / kBlock), b, 0, st, s, a);
}

void launch_ct_gather_pot(const SysView& s, const PmeView& pm, const CtArgs& a, hipStream_t st) {
  if (a.n_lp <= 0) return;
  const dim3 g((a.n_lp + kBlock - 1) / kBlock), b(kBlock);
  switch (pm.order) {
    case 4: hipLaunchKernelGGL(k_ct_gather_pot<4>, g, b, 0, st, s, pm, a); break;
    case 6: hipLaunchKernelGGL(k_ct_gather_pot<6>, g, b, 0, st, s, pm, a); break;
    default: hipLaunchKernelGGL(k_ct_gather_pot<5>, g, b, 0, st, s, pm, a); break;
  }
}

void launch_ct_pairs(const SysView& s, const CtArgs& a, Reduce& red, hipStream_t st) {
  const dim3 b(kBlock);
  const int nr = std::max(std::max(a.n_lp, a.n_acc), 1);
  hipLaunchKernelGGL(k_ct_records, dim3((nr + kBlock - 1) / kBlock), b, 0, st, s, a);
  const dim3 gl((std::max(a.n_lp, 1) + kWaves - 1) / kWaves);
  hipLaunchKernelGGL(k_ct_pairs_lp, gl, b, 0, st, s, a, red);
  red.nparts[S_ECT] = (int)gl.x;
  if (a.n_acc > 0)
    hipLaunchKernelGGL(k_ct_pairs_acc, dim3((a.n_acc + kWaves - 1) / kWaves), b, 0, st, s, a);
  hipLaunchKernelGGL(k_ct_collect, dim3((a.n + kBlock - 1) / kBlock), b, 0, st, a);
}

void launch_ct_wforce(const SysView& s, const CtArgs& a, double4* sp_w, hipStream_t st,
                      double4* FS, double* GS) {
  const dim3 b(kBlock), gw((s.n + kWaves - 1) / kWaves), gs((s.n + kBlock - 1) / kBlock);
  if (a.n_lp > 0)
    hipLaunchKernelGGL(k_ct_wforce_lp, dim3((a.n_lp + kWaves - 1) / kWaves), b, 0, st, s, a);
  if (FS && GS) {
    hipLaunchKernelGGL(k_ct_wforce_mp<true>, gw, b, 0, st, s, a, FS, GS);
    hipLaunchKernelGGL(k_ct_wforce_in<true>, gs, b, 0, st, s, a, FS, GS);
  } else {
    hipLaunchKernelGGL(k_ct_wforce_mp<false>, gw, b, 0, st, s, a, FS, GS);
    hipLaunchKernelGGL(k_ct_wforce_in<false>, gs, b, 0, st, s, a, FS, GS);
  }
  if (sp_w) hipLaunchKernelGGL(k_ct_wrecords, dim3((s.n + kBlock - 1) / kBlock), b, 0, st, s, a, sp_w);
}

}  // namespace sibfa
