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
//                   multipoles), so list scans test one word per entry.
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
// (the loads of a step issue together).  hit(k, v) tells whether entry k
// takes part and sets the value v to queue; queued values keep list order
// in a ring of kRing slots, and whenever 64 are queued every lane takes one
// and runs eval(v).  What is left runs at the end on the first lanes.  The
// whole wave calls it with the same nt.
constexpr int kScanU = 4;
template <class Hit, class Eval>
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

// Everything of one (lone pair p, acceptor k) pair, given the positions of
// the lone pair, its carrier and the acceptor's a1 and a2.
__device__ __forceinline__ void ct_pair(const SysView& s, const CtArgs& a, int p, int k,
                                        const double xL[3], const double xc[3],
                                        const double x1[3], const double x2[3], CtPair& o) {
  const int c = a.lp[2 * p + 1];
  const int a1 = a.acc[2 * k], a2 = a.acc[2 * k + 1];
  double u[3], d1[3], d2[3];
  sep(s, xL, xc, u);
  sep(s, x1, xc, d1);
  sep(s, x2, xc, d2);
  const double nu = sqrt(u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
  const double r1 = sqrt(d1[0] * d1[0] + d1[1] * d1[1] + d1[2] * d1[2]);
  const double r2 = sqrt(d2[0] * d2[0] + d2[1] * d2[1] + d2[2] * d2[2]);
  const double s1 = 2.0 * sqrt(a.rvdw[c] * a.rvdw[a1]), s2 = 2.0 * sqrt(a.rvdw[c] * a.rvdw[a2]);
  const double ud1 = u[0] * d1[0] + u[1] * d1[1] + u[2] * d1[2];
  const double ud2 = u[0] * d2[0] + u[1] * d2[1] + u[2] * d2[2];
  const double ca = ud1 / (nu * r1), cb = ud2 / (nu * r2);
  const double ex1 = exp(-a.eta * r1 / s1), ex2 = exp(-a.eta * r2 / s2);
  const double VL = kCoulomb * a.Vlp[p];
  const double X1 = kCoulomb * a.Vint[a1] - VL, X2 = kCoulomb * a.Vint[a2] - VL;
  const double g1 = a.cs * a.t + a.cp * a.m * ca, g2 = a.cs * a.t + a.cp * a.m * cb;
  const double e1 = ex1 * X1 * g1, e2 = ex2 * X2 * g2;
  const double nocc = a.lp_par[2 * p], dE = a.lp_par[2 * p + 1] + VL - a.ah[k];
  const double diff = e1 - e2;
  o.E = -nocc * diff * diff / dE;
  const double G = -2.0 * nocc * diff / dE;   // dE/de1; dE/de2 = -G
  const double GD = nocc * diff * diff / (dE * dE);
  o.dV = kCoulomb * (-G * ex1 * g1 + G * ex2 * g2 + GD);
  o.dVi1 = kCoulomb * G * ex1 * g1;
  o.dVi2 = -kCoulomb * G * ex2 * g2;
  const double k1 = G * ex1 * X1 * a.cp * a.m;    // dE/dcos(alpha)
  const double k2 = -G * ex2 * X2 * a.cp * a.m;   // dE/dcos(beta)
  const double r1e = G * (-a.eta / s1) * e1;      // dE/dr1
  const double r2e = -G * (-a.eta / s2) * e2;     // dE/dr2
#pragma unroll
  for (int q = 0; q < 3; ++q) {
    const double dca_du = d1[q] / (nu * r1) - ca * u[q] / (nu * nu);
    const double dcb_du = d2[q] / (nu * r2) - cb * u[q] / (nu * nu);
    const double dca_dd1 = u[q] / (nu * r1) - ca * d1[q] / (r1 * r1);
    const double dcb_dd2 = u[q] / (nu * r2) - cb * d2[q] / (r2 * r2);
    o.gL[q] = k1 * dca_du + k2 * dcb_du;
    o.gA1[q] = r1e * d1[q] / r1 + k1 * dca_dd1;
    o.gA2[q] = r2e * d2[q] / r2 + k2 * dcb_dd2;
    o.gC[q] = -(o.gL[q] + o.gA1[q] + o.gA2[q]);
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
  a.flag_s[i] = (a.a1_start[c + 1] > a.a1_start[c] ? kIsA1 : 0) |
                (a.car_start[c + 1] > a.car_start[c] ? kIsCarrier : 0) | (mult ? kHasMult : 0);
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
  wave_compact(
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
    double xL[3], xc[3];
    site_pos(s, a.inv_perm[a.lp[2 * p]], xL);
    site_pos(s, i, xc);
    const int nn = s.nc_near[i];
    wave_compact(
        s.nc_all[i], ring[wv],
        [&](int e, int& v) {
          v = all_entry(s, i, e, nn);
          return (a.flag_s[v] & kIsA1) != 0;
        },
        [&](int j) {
          double x1[3];
          site_pos(s, j, x1);
          const int cj = a.perm[j];
          for (int r = a.a1_start[cj]; r < a.a1_start[cj + 1]; ++r) {
            const int k = a.a1_ref[r];
            double x2[3];
            site_pos(s, a.inv_perm[a.acc[2 * k + 1]], x2);
            CtPair o;
            ct_pair(s, a, p, k, xL, xc, x1, x2, o);
            E += o.E;
            w += o.dV;
#pragma unroll
            for (int q = 0; q < 3; ++q) {
              FL[q] -= o.gL[q];
              FC[q] -= o.gC[q];
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
  double x1[3], x2[3];
  site_pos(s, i, x1);
  site_pos(s, a.inv_perm[a.acc[2 * k + 1]], x2);
  const int nn = s.nc_near[i];
  wave_compact(
      s.nc_all[i], ring[wv],
      [&](int e, int& v) {
        v = all_entry(s, i, e, nn);
        return (a.flag_s[v] & kIsCarrier) != 0;
      },
      [&](int j) {
        double xc[3];
        site_pos(s, j, xc);
        const int cj = a.perm[j];
        for (int r = a.car_start[cj]; r < a.car_start[cj + 1]; ++r) {
          const int p = a.car_ref[r];
          double xL[3];
          site_pos(s, a.inv_perm[a.lp[2 * p]], xL);
          CtPair o;
          ct_pair(s, a, p, k, xL, xc, x1, x2, o);
          u1 += o.dVi1;
          u2 += o.dVi2;
#pragma unroll
          for (int q = 0; q < 3; ++q) {
            F1[q] -= o.gA1[q];
            F2[q] -= o.gA2[q];
          }
        }
      });
  u1 = wave_sum(u1);
  u2 = wave_sum(u2);
#pragma unroll
  for (int q = 0; q < 3; ++q) {
    F1[q] = wave_sum(F1[q]);
    F2[q] = wave_sum(F2[q]);
  }
  if (lane == 0) {
    a.ua[2 * (size_t)k] = u1;
    a.ua[2 * (size_t)k + 1] = u2;
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      a.Fa[6 * (size_t)k + q] = F1[q];
      a.Fa[6 * (size_t)k + 3 + q] = F2[q];
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
  wave_compact(
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
  wave_compact(
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
