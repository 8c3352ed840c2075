// Batched gas-phase clusters.  One workgroup owns one cluster and runs its
// whole polarization path with direct sums (no cutoff, no neighbour list):
//
//   k_cl_prep  : polarizable-site compaction, alpha^-1 with a positivity
//                check, the Thole-damped permanent field E at the
//                polarizable sites and the multipolar energy E_elec;
//   k_cl_solve : block-Jacobi PCG for T mu = E (Eq. 18) held entirely in
//                the workgroup -- the direction vector lives in LDS, dot
//                products are LDS reductions, and the FP64 true residual
//                (replacing the recurrence residual, as in the context
//                solver) is evaluated in the same launch -- then
//                E_pol = -1/2 mu.E (Eq. 19);
//   k_cl_force : forces at the converged mu through the combined-density
//                identity of the periodic force kernel with the bare kernel.
//
// Each kernel walks the batch with a grid-stride loop over clusters, and
// every reduction runs in a fixed order inside one workgroup, so a cluster's
// results are bitwise independent of which other clusters share the batch.
//
// Pair coefficients of a cluster (bare kernel c0_n = (2n-1)!!/r^(2n+1)):
//   different molecules: MM c0; Mmu and mumu (both sites polarizable)
//                        c0 - P_n e^-x c0 (Thole); same molecule: mumu only,
//                        damped; MM and Mmu excluded.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <mutex>
#include <string>

#include "../../include/sibfa_pol.h"
#include "common.h"
#include "pairmath.h"

namespace sibfa {

constexpr int kClBlock = 256;
constexpr int kClWaves = kClBlock / 64;
constexpr int kClMaxSites = SIBFA_BATCH_MAX_SITES;
constexpr int kClMaxPol = SIBFA_BATCH_MAX_POLARIZABLE;
constexpr int kClOwn = (kClMaxPol + kClBlock - 1) / kClBlock;   // sites per slot, G = 1

struct ClusterArgs {
  int nclusters;
  int nsites;           // sites in the caller arrays (and scratch capacity)
  const int* off;       // [nclusters + 1] site offsets into the caller arrays
  const int* warm;      // [nclusters] 1: start from mu, or nullptr
  const double* xyz;    // caller arrays, concatenated clusters
  const int* mol;
  const double* q;
  const double* dip;
  const double* quad;
  const double* alpha;
  const double* thole;  // [n] or nullptr (uniform thole_a)
  double thole_a;
  double tol;
  int max_iter;
  // scratch, indexed by global site offset; polarizable records are
  // compacted to the front of each cluster's segment
  int* npol;            // [nclusters]
  int* polsite;         // [n] polarizable rank -> global site
  int* prank;           // [n] global site -> polarizable rank, or -1
  double* sval;         // [n] abar^-1/2 per site (0: not polarizable)
  double4* pp;          // [n] x, y, z, s of polarizable rank
  double* pa;           // [n] Thole factor of polarizable rank
  double* palpha;       // [n][6]
  double* painv;        // [n][6]
  double4* E0;          // [n]
  double4* X;           // [n]
  double4* Rr;          // [n]
  // outputs
  double* mu;           // [n][3]
  double* forces;       // [n][3] or nullptr
  double* e_pol;        // [nclusters]
  double* e_elec;
  int* iters;
  double* rms;
  int* status;
};

// ---------------------------------------------------------------- helpers

// Lanes per site: the largest power of two G <= 16 with G * count <= block.
__device__ __forceinline__ int lanes_for(int count) {
  int G = 1;
  while (G < 16 && 2 * G * count <= kClBlock) G *= 2;
  return G;
}

// Cluster c's site range [base, base + n) from the offsets, and whether it
// is a valid one: 1..kClMaxSites sites inside the nsites of the arrays.
// Offsets validated on the host always pass; offsets that the caller
// keeps on the device are checked here, and a cluster whose range fails
// is reported (E_ARG) without touching its rows.
__device__ __forceinline__ bool cluster_range(const ClusterArgs& a, int c, int& base, int& n) {
  base = a.off[c];
  const int end = a.off[c + 1];
  n = end - base;
  return base >= 0 && n >= 1 && n <= kClMaxSites && end <= a.nsites;
}

__device__ __forceinline__ double group_sum_rt(double v, int G) {
  for (int o = G >> 1; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Sums of up to three values over the block, returned to every thread in
// the same fixed order.  All threads must call it.
struct BlockSum {
  double* sh;   // [3][kClWaves] in LDS
  __device__ void operator()(double& a, double& b, double& c) const {
    a = wave_sum(a);
    b = wave_sum(b);
    c = wave_sum(c);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) {
      sh[w] = a;
      sh[kClWaves + w] = b;
      sh[2 * kClWaves + w] = c;
    }
    __syncthreads();
    a = b = c = 0.0;
    for (int k = 0; k < kClWaves; ++k) {
      a += sh[k];
      b += sh[kClWaves + k];
      c += sh[2 * kClWaves + k];
    }
  }
};

template <typename R>
__device__ __forceinline__ void load_site(const ClusterArgs& a, int g, MP<R>& M, double x[3]) {
  x[0] = a.xyz[3 * (size_t)g];
  x[1] = a.xyz[3 * (size_t)g + 1];
  x[2] = a.xyz[3 * (size_t)g + 2];
  M.q = (R)a.q[g];
#pragma unroll
  for (int k = 0; k < 3; ++k) M.d[k] = (R)a.dip[3 * (size_t)g + k];
#pragma unroll
  for (int k = 0; k < 6; ++k) M.t[k] = (R)a.quad[6 * (size_t)g + k];
}

__device__ __forceinline__ double thole_of(const ClusterArgs& a, int g) {
  return a.thole ? a.thole[g] : a.thole_a;
}

// Inverse of a symmetric 3x3 (xx,xy,xz,yy,yz,zz); false unless positive
// definite (leading minors > 0).
__device__ __forceinline__ bool sym_inverse(const double m[6], double inv[6]) {
  const double a = m[0], b = m[1], c = m[2], d = m[3], e = m[4], f = m[5];
  const double m2 = a * d - b * b;
  const double A = d * f - e * e, B = c * e - b * f, C = b * e - c * d;
  const double det = a * A + b * B + c * C;
  if (!(a > 0.0) || !(m2 > 0.0) || !(det > 0.0)) return false;
  const double id = 1.0 / det;
  inv[0] = A * id;
  inv[1] = B * id;
  inv[2] = C * id;
  inv[3] = (a * f - c * c) * id;
  inv[4] = (b * c - a * e) * id;
  inv[5] = m2 * id;
  return true;
}

__device__ __forceinline__ void sym_apply(const double* m, const double v[3], double o[3]) {
  o[0] = m[0] * v[0] + m[1] * v[1] + m[2] * v[2];
  o[1] = m[1] * v[0] + m[3] * v[1] + m[4] * v[2];
  o[2] = m[2] * v[0] + m[4] * v[1] + m[5] * v[2];
}

// ---------------------------------------------------------------- prep
template <typename R>
__global__ __launch_bounds__(kClBlock) void k_cl_prep(ClusterArgs a) {
  __shared__ int wcount[kClWaves];
  __shared__ int bad;
  __shared__ double sh[3 * kClWaves];
  const BlockSum bsum{sh};
  const int t = threadIdx.x, lane64 = t & 63, w = t >> 6;
  for (int c = blockIdx.x; c < a.nclusters; c += gridDim.x) {
    int base, n;
    if (!cluster_range(a, c, base, n)) {
      if (t == 0) {
        a.npol[c] = 0;
        a.status[c] = (int)SIBFA_E_ARG;
        a.e_elec[c] = __longlong_as_double(0x7ff8000000000000ll);
      }
      continue;
    }
    __syncthreads();
    if (t == 0) bad = 0;
    // order-preserving compaction of the polarizable sites, 256 at a time
    int total = 0;
    for (int c0 = 0; c0 < n; c0 += kClBlock) {
      const int i = c0 + t;
      bool is_pol = false;
      double al[6];
      if (i < n) {
        const int g = base + i;
#pragma unroll
        for (int k = 0; k < 6; ++k) {
          al[k] = a.alpha[6 * (size_t)g + k];
          is_pol = is_pol || al[k] != 0.0;
        }
      }
      const unsigned long long m = __ballot(is_pol);
      const int rank_in_wave = __popcll(m & ((1ull << lane64) - 1ull));
      __syncthreads();
      if (lane64 == 0) wcount[w] = __popcll(m);
      __syncthreads();
      int before = total;
      for (int k = 0; k < w; ++k) before += wcount[k];
      if (i < n) {
        const int g = base + i;
        double s = 0.0;
        int rank = -1;
        if (is_pol) {
          const int pk = before + rank_in_wave;
          rank = pk;
          double inv[6];
          if (!sym_inverse(al, inv)) {
            bad = 1;
          } else {
            s = 1.0 / sqrt((al[0] + al[3] + al[5]) / 3.0);
            const size_t o = base + (size_t)pk;
            a.polsite[o] = g;
            a.pp[o] = make_double4(a.xyz[3 * (size_t)g], a.xyz[3 * (size_t)g + 1],
                                   a.xyz[3 * (size_t)g + 2], s);
            a.pa[o] = thole_of(a, g);
#pragma unroll
            for (int k = 0; k < 6; ++k) {
              a.palpha[6 * o + k] = al[k];
              a.painv[6 * o + k] = inv[k];
            }
          }
        }
        a.sval[g] = s;
        a.prank[g] = rank;
      }
      for (int k = 0; k < kClWaves; ++k) total += wcount[k];
    }
    __syncthreads();
    const int np = total;
    if (t == 0) {
      a.npol[c] = np;
      a.status[c] = (bad || np > kClMaxPol) ? (int)SIBFA_E_ARG : 0;
    }
    // permanent field at polarizable sites and the MM energy; G lanes per site
    const int G = lanes_for(n), nslot = kClBlock / G, slot = t / G, lane = t % G;
    double U = 0.0;
    for (int i = slot; i < n; i += nslot) {
      const int gi = base + i;
      MP<R> Mi;
      double xi[3];
      load_site<R>(a, gi, Mi, xi);
      const int mi = a.mol[gi];
      const double si = a.sval[gi];
      const double ai = thole_of(a, gi);
      double acc[3] = {0.0, 0.0, 0.0};
      for (int j = lane; j < n; j += G) {
        const int gj = base + j;
        if (a.mol[gj] == mi) continue;
        MP<R> Mj;
        double xj[3];
        load_site<R>(a, gj, Mj, xj);
        const R Rv[3] = {(R)(xi[0] - xj[0]), (R)(xi[1] - xj[1]), (R)(xi[2] - xj[2])};
        const R r2 = Rv[0] * Rv[0] + Rv[1] * Rv[1] + Rv[2] * Rv[2];
        const R rinv = dev_rsqrt<R>(r2), r = r2 * rinv, rinv2 = rinv * rinv;
        R c0[6];
        bare_coeffs<R, 4>(rinv, rinv2, c0);
        c0[5] = R(0);
        R u, fd[3];
        mp_pair<R, true, false>(c0, Mi, Mj, Rv, u, fd);
        U += 0.5 * (double)u;
        if (si > 0.0) {
          R cc[6] = {c0[0], c0[1], c0[2], c0[3], R(0), R(0)};
          const double sj = a.sval[gj];
          if (sj > 0.0) {
            R tp[5];
            thole_tp<R>(R(fmin(ai, thole_of(a, gj))) * r2 * r * R(si * sj), tp);
#pragma unroll
            for (int k = 1; k <= 3; ++k) cc[k] -= tp[k] * c0[k];
          }
          R E[3];
          mp_field<R>(cc, Mj, Rv, E);
          acc[0] += (double)E[0];
          acc[1] += (double)E[1];
          acc[2] += (double)E[2];
        }
      }
#pragma unroll
      for (int k = 0; k < 3; ++k) acc[k] = group_sum_rt(acc[k], G);
      if (lane == 0 && si > 0.0)
        a.E0[base + a.prank[gi]] = make_double4(acc[0], acc[1], acc[2], 0.0);
    }
    double d1 = 0.0, d2 = 0.0;
    bsum(U, d1, d2);
    if (t == 0) a.e_elec[c] = kCoulomb * U;
  }
}

// ---------------------------------------------------------------- solve
// Field at polarizable rank k of the dipoles v[j], j != k, damped (every
// pair of a cluster's polarizable sites couples, same molecule included).
template <typename RR>
__device__ __forceinline__ void cl_dip_field(const double4* lpos, const double* la,
                                             const double4* lv, int np, int k, int lane, int G,
                                             double f[3]) {
  const double4 pk = lpos[k];
  const double ak = la[k];
  f[0] = f[1] = f[2] = 0.0;
  for (int j = lane; j < np; j += G) {
    if (j == k) continue;
    const double4 pj = lpos[j];
    const double4 vj = lv[j];
    const RR Rv[3] = {(RR)(pk.x - pj.x), (RR)(pk.y - pj.y), (RR)(pk.z - pj.z)};
    const RR r2 = Rv[0] * Rv[0] + Rv[1] * Rv[1] + Rv[2] * Rv[2];
    const RR rinv = dev_rsqrt<RR>(r2), r = r2 * rinv, rinv2 = rinv * rinv;
    const RR c01 = rinv * rinv2, c02 = RR(3) * c01 * rinv2;
    const RR x = RR(fmin(ak, la[j])) * r2 * r * RR(pk.w * pj.w);
    const RR e = dev_exp<RR>(-x);
    const RR c1 = (RR(1) - e) * c01, c2 = (RR(1) - (RR(1) + x) * e) * c02;
    const RR p[3] = {(RR)vj.x, (RR)vj.y, (RR)vj.z};
    RR E[3];
    dip_field<RR>(c1, c2, p, Rv, E);
    f[0] += (double)E[0];
    f[1] += (double)E[1];
    f[2] += (double)E[2];
  }
  f[0] = group_sum_rt(f[0], G);
  f[1] = group_sum_rt(f[1], G);
  f[2] = group_sum_rt(f[2], G);
}

template <typename R>
__global__ __launch_bounds__(kClBlock) void k_cl_solve(ClusterArgs a) {
  __shared__ double4 lpos[kClMaxPol];
  __shared__ double4 lv[kClMaxPol];
  __shared__ double la[kClMaxPol];
  __shared__ double sh[3 * kClWaves];
  const BlockSum bsum{sh};
  const int t = threadIdx.x;
  for (int c = blockIdx.x; c < a.nclusters; c += gridDim.x) {
    int base, n;
    if (!cluster_range(a, c, base, n)) {
      if (t == 0) {
        a.e_pol[c] = __longlong_as_double(0x7ff8000000000000ll);
        a.iters[c] = 0;
        a.rms[c] = 0.0;
      }
      continue;
    }
    const int np = a.npol[c];
    const int st0 = a.status[c];
    if (st0 != 0 || np == 0) {
      for (int i = t; i < n; i += kClBlock)
        for (int k = 0; k < 3; ++k) a.mu[3 * (size_t)(base + i) + k] = 0.0;
      if (t == 0) {
        a.e_pol[c] = st0 != 0 ? __longlong_as_double(0x7ff8000000000000ll) : 0.0;
        a.iters[c] = 0;
        a.rms[c] = 0.0;
      }
      continue;
    }
    const int G = lanes_for(np), nslot = kClBlock / G, slot = t / G, lane = t % G;
    __syncthreads();
    for (int k = t; k < np; k += kClBlock) {
      lpos[k] = a.pp[base + k];
      la[k] = a.pa[base + k];
      const size_t o = base + (size_t)k;
      double x[3];
      if (a.warm && a.warm[c]) {
        const size_t g = a.polsite[o];
        x[0] = a.mu[3 * g];
        x[1] = a.mu[3 * g + 1];
        x[2] = a.mu[3 * g + 2];
      } else {
        const double4 e = a.E0[o];
        const double ev[3] = {e.x, e.y, e.z};
        sym_apply(a.palpha + 6 * o, ev, x);
      }
      a.X[o] = make_double4(x[0], x[1], x[2], 0.0);
    }
    __syncthreads();
    const double tol = a.tol;
    const double zz_stop = (tol / kDebye) * (tol / kDebye) * np;
    int it = 0, restarts = 0, status = 0;
    double rho = 0.0;
    double rz_run = 0.0;            // r.z of the running sequence
    double zz_replace = -1.0;       // see the context solver: one early
    bool fresh = true;              // residual replacement in mixed mode
    double zr[kClOwn][3], ps[kClOwn][3];
    for (;;) {
      // true residual r = E - T x in FP64, z = alpha r; the running search
      // directions of this slot's sites are kept while lv holds x
      if (!fresh) {
#pragma unroll
        for (int kk = 0; kk < kClOwn; ++kk) {
          const int k = slot + kk * nslot;
          if (k < np && lane == 0) {
            const double4 pv = lv[k];
            ps[kk][0] = pv.x; ps[kk][1] = pv.y; ps[kk][2] = pv.z;
          }
        }
      }
      __syncthreads();
      for (int k = t; k < np; k += kClBlock) lv[k] = a.X[base + k];
      __syncthreads();
      double zz = 0.0, rz = 0.0, d = 0.0;
#pragma unroll
      for (int kk = 0; kk < kClOwn; ++kk) {
        const int k = slot + kk * nslot;
        if (k >= np) break;
        double f[3];
        cl_dip_field<double>(lpos, la, lv, np, k, lane, G, f);
        if (lane == 0) {
          const size_t o = base + (size_t)k;
          const double4 xv = lv[k], e = a.E0[o];
          const double xa[3] = {xv.x, xv.y, xv.z};
          double tx[3], r[3], z[3];
          sym_apply(a.painv + 6 * o, xa, tx);
          r[0] = e.x - (tx[0] - f[0]);
          r[1] = e.y - (tx[1] - f[1]);
          r[2] = e.z - (tx[2] - f[2]);
          sym_apply(a.palpha + 6 * o, r, z);
          a.Rr[o] = make_double4(r[0], r[1], r[2], 0.0);
          zz += z[0] * z[0] + z[1] * z[1] + z[2] * z[2];
          rz += r[0] * z[0] + r[1] * z[1] + r[2] * z[2];
          zr[kk][0] = z[0];
          zr[kk][1] = z[1];
          zr[kk][2] = z[2];
        }
      }
      bsum(zz, rz, d);
      rho = kDebye * sqrt(zz / np);
      if (rho <= tol) break;
      if (it >= a.max_iter || restarts > 8) {
        status = (int)SIBFA_E_NOT_CONVERGED;
        break;
      }
      // a new sequence (p = z) at the start; afterwards the true residual
      // replaces the recurrence one and the sequence goes on (p = z + beta p)
      const double beta0 = fresh ? 0.0 : rz / rz_run;
      if (fresh) {
        if (sizeof(R) == 4) zz_replace = 1e-8 * zz;
      } else {
        ++restarts;
      }
#pragma unroll
      for (int kk = 0; kk < kClOwn; ++kk) {
        const int k = slot + kk * nslot;
        if (k < np && lane == 0) {
          const double b0 = fresh ? 0.0 : beta0;
          const double q0 = fresh ? 0.0 : ps[kk][0], q1 = fresh ? 0.0 : ps[kk][1],
                       q2 = fresh ? 0.0 : ps[kk][2];
          lv[k] = make_double4(zr[kk][0] + b0 * q0, zr[kk][1] + b0 * q1, zr[kk][2] + b0 * q2, 0.0);
        }
      }
      fresh = false;
      rz_run = rz;
      __syncthreads();
      while (it < a.max_iter) {
        double pq = 0.0, d1 = 0.0, d2 = 0.0;
        double qr[kClOwn][3];
#pragma unroll
        for (int kk = 0; kk < kClOwn; ++kk) {
          const int k = slot + kk * nslot;
          if (k >= np) break;
          double f[3];
          cl_dip_field<R>(lpos, la, lv, np, k, lane, G, f);
          if (lane == 0) {
            const double4 pv = lv[k];
            const double pa3[3] = {pv.x, pv.y, pv.z};
            double tp[3];
            sym_apply(a.painv + 6 * (base + (size_t)k), pa3, tp);
            qr[kk][0] = tp[0] - f[0];
            qr[kk][1] = tp[1] - f[1];
            qr[kk][2] = tp[2] - f[2];
            pq += pa3[0] * qr[kk][0] + pa3[1] * qr[kk][1] + pa3[2] * qr[kk][2];
          }
        }
        bsum(pq, d1, d2);
        if (!(pq > 0.0)) {
          status = (int)SIBFA_E_NOT_SPD;
          break;
        }
        const double gamma = rz_run / pq;
        double zz2 = 0.0, rz2 = 0.0, d3 = 0.0;
#pragma unroll
        for (int kk = 0; kk < kClOwn; ++kk) {
          const int k = slot + kk * nslot;
          if (k >= np) break;
          if (lane == 0) {
            const size_t o = base + (size_t)k;
            const double4 pv = lv[k];
            double4 xv = a.X[o], rv = a.Rr[o];
            xv.x += gamma * pv.x;
            xv.y += gamma * pv.y;
            xv.z += gamma * pv.z;
            rv.x -= gamma * qr[kk][0];
            rv.y -= gamma * qr[kk][1];
            rv.z -= gamma * qr[kk][2];
            a.X[o] = xv;
            a.Rr[o] = rv;
            const double r[3] = {rv.x, rv.y, rv.z};
            double z[3];
            sym_apply(a.palpha + 6 * o, r, z);
            zz2 += z[0] * z[0] + z[1] * z[1] + z[2] * z[2];
            rz2 += r[0] * z[0] + r[1] * z[1] + r[2] * z[2];
            zr[kk][0] = z[0];
            zr[kk][1] = z[1];
            zr[kk][2] = z[2];
          }
        }
        bsum(zz2, rz2, d3);
        ++it;
        if (zz2 <= zz_stop) break;
        if (zz2 <= zz_replace) {
          zz_replace = -1.0;
          break;
        }
        const double beta = rz2 / rz_run;
        rz_run = rz2;
#pragma unroll
        for (int kk = 0; kk < kClOwn; ++kk) {
          const int k = slot + kk * nslot;
          if (k < np && lane == 0) {
            const double4 pv = lv[k];
            lv[k] = make_double4(zr[kk][0] + beta * pv.x, zr[kk][1] + beta * pv.y,
                                 zr[kk][2] + beta * pv.z, 0.0);
          }
        }
        __syncthreads();
      }
      if (status == (int)SIBFA_E_NOT_SPD) break;
      __syncthreads();
    }
    // outputs: mu in caller order (zero at non-polarizable sites), E_pol
    __syncthreads();
    for (int i = t; i < n; i += kClBlock) {
      if (a.sval[base + i] == 0.0)
        for (int k = 0; k < 3; ++k) a.mu[3 * (size_t)(base + i) + k] = 0.0;
    }
    double me = 0.0, d4 = 0.0, d5 = 0.0;
    for (int k = t; k < np; k += kClBlock) {
      const size_t o = base + (size_t)k;
      const double4 xv = a.X[o], e = a.E0[o];
      const size_t g = a.polsite[o];
      a.mu[3 * g] = xv.x;
      a.mu[3 * g + 1] = xv.y;
      a.mu[3 * g + 2] = xv.z;
      me += xv.x * e.x + xv.y * e.y + xv.z * e.z;
    }
    bsum(me, d4, d5);
    if (t == 0) {
      a.e_pol[c] = -0.5 * kCoulomb * me;
      a.iters[c] = it;
      a.rms[c] = rho;
      a.status[c] = status;
    }
  }
}

// ---------------------------------------------------------------- forces
template <typename R>
__global__ __launch_bounds__(kClBlock) void k_cl_force(ClusterArgs a) {
  const int t = threadIdx.x;
  for (int c = blockIdx.x; c < a.nclusters; c += gridDim.x) {
    int base, n;
    if (!cluster_range(a, c, base, n)) continue;
    if (a.status[c] == (int)SIBFA_E_ARG) {
      for (int i = t; i < n; i += kClBlock)
        for (int k = 0; k < 3; ++k) a.forces[3 * (size_t)(base + i) + k] = 0.0;
      continue;
    }
    const int G = lanes_for(n), nslot = kClBlock / G, slot = t / G, lane = t % G;
    for (int i = slot; i < n; i += nslot) {
      const int gi = base + i;
      MP<R> Mi;
      double xi[3];
      load_site<R>(a, gi, Mi, xi);
      const R mui[3] = {(R)a.mu[3 * (size_t)gi], (R)a.mu[3 * (size_t)gi + 1],
                        (R)a.mu[3 * (size_t)gi + 2]};
      MP<R> Pi = Mi;
      Pi.d[0] += mui[0];
      Pi.d[1] += mui[1];
      Pi.d[2] += mui[2];
      const int mi = a.mol[gi];
      const double si = a.sval[gi];
      const double ai = thole_of(a, gi);
      double F[3] = {0.0, 0.0, 0.0};
      for (int j = lane; j < n; j += G) {
        if (j == i) continue;
        const int gj = base + j;
        MP<R> Mj;
        double xj[3];
        load_site<R>(a, gj, Mj, xj);
        const double sj = a.sval[gj];
        const R Rv[3] = {(R)(xi[0] - xj[0]), (R)(xi[1] - xj[1]), (R)(xi[2] - xj[2])};
        const R r2 = Rv[0] * Rv[0] + Rv[1] * Rv[1] + Rv[2] * Rv[2];
        const R rinv = dev_rsqrt<R>(r2), r = r2 * rinv, rinv2 = rinv * rinv;
        R c0[6];
        bare_coeffs<R, 5>(rinv, rinv2, c0);
        const bool both = si > 0.0 && sj > 0.0;
        const R x = both ? R(fmin(ai, thole_of(a, gj))) * r2 * r * R(si * sj) : R(0);
        R u, f[3];
        if (a.mol[gj] == mi) {
          if (!both) continue;
          // same molecule: damped mu-mu only
          R tp[5], cc[6];
          thole_tp<R>(x, tp);
          cc[0] = R(0);
          cc[5] = R(0);
#pragma unroll
          for (int k = 1; k <= 4; ++k) cc[k] = (R(1) - tp[k]) * c0[k];
          const R muj[3] = {(R)a.mu[3 * (size_t)gj], (R)a.mu[3 * (size_t)gj + 1],
                            (R)a.mu[3 * (size_t)gj + 2]};
          MP<R> Ui, Uj;
          Ui.q = Uj.q = R(0);
#pragma unroll
          for (int k = 0; k < 3; ++k) {
            Ui.d[k] = mui[k];
            Uj.d[k] = muj[k];
          }
#pragma unroll
          for (int k = 0; k < 6; ++k) Ui.t[k] = Uj.t[k] = R(0);
          mp_pair<R, false, true>(cc, Ui, Uj, Rv, u, f);
          F[0] += (double)f[0];
          F[1] += (double)f[1];
          F[2] += (double)f[2];
          continue;
        }
        R cc[6], D[6] = {R(0), R(0), R(0), R(0), R(0), R(0)};
#pragma unroll
        for (int k = 0; k < 6; ++k) cc[k] = c0[k];
        const bool damp = both && x < R(50);
        if (damp) {
          R tp[5];
          thole_tp<R>(x, tp);
#pragma unroll
          for (int k = 1; k <= 4; ++k) {
            D[k] = tp[k] * c0[k];
            cc[k] -= D[k];
          }
        }
        MP<R> Pj = Mj;
        Pj.d[0] += (R)a.mu[3 * (size_t)gj];
        Pj.d[1] += (R)a.mu[3 * (size_t)gj + 1];
        Pj.d[2] += (R)a.mu[3 * (size_t)gj + 2];
        mp_pair<R, false, true>(cc, Pi, Pj, Rv, u, f);
        F[0] += (double)f[0];
        F[1] += (double)f[1];
        F[2] += (double)f[2];
        if (damp) {
          mp_pair<R, false, true>(D, Mi, Mj, Rv, u, f);
          F[0] += (double)f[0];
          F[1] += (double)f[1];
          F[2] += (double)f[2];
        }
      }
#pragma unroll
      for (int k = 0; k < 3; ++k) F[k] = group_sum_rt(F[k], G);
      if (lane == 0)
        for (int k = 0; k < 3; ++k) a.forces[3 * (size_t)gi + k] = kCoulomb * F[k];
    }
  }
}

}  // namespace sibfa

using namespace sibfa;

// Device memory of sibfa_batch_clusters_noalloc: the batch scratch arrays
// for SIBFA_BATCH_NOALLOC_MAX_SITES sites and SIBFA_BATCH_NOALLOC_MAX_CLUSTERS
// clusters, carved as by carve() below (every region rounded up to 256
// bytes).  Each device the library runs on holds its own copy for the life
// of the process; calls on one device share it.
namespace {
constexpr size_t kNaSites = SIBFA_BATCH_NOALLOC_MAX_SITES;
constexpr size_t kNaClusters = SIBFA_BATCH_NOALLOC_MAX_CLUSTERS;
constexpr size_t a256(size_t x) { return (x + 255) & ~(size_t)255; }
constexpr size_t kNaBytes =
    a256((kNaClusters + 1) * sizeof(int)) + 2 * a256(kNaClusters * sizeof(int)) +
    2 * a256(kNaSites * sizeof(int)) + 2 * a256(kNaSites * sizeof(double)) +
    a256(kNaSites * sizeof(double4)) + 2 * a256(kNaSites * 6 * sizeof(double)) +
    3 * a256(kNaSites * sizeof(double4));
}  // namespace

static __device__ __align__(256) unsigned char scratch[kNaBytes];

struct sibfa_batch_s {
  int device = 0;
  hipStream_t stream = nullptr;
  sibfa_alloc_fn af = nullptr;
  sibfa_free_fn ff = nullptr;
  void* user = nullptr;
  std::string err;
  size_t cap_sites = 0, cap_clusters = 0;
  void* scratch = nullptr;   // one device allocation holding every array
  int* h_stage = nullptr;    // pinned staging of offsets and warm flags
  size_t h_cap = 0;
  hipEvent_t staged = nullptr;
  bool staged_pending = false;
  ClusterArgs args{};
};

namespace {

sibfa_status bfail(sibfa_batch b, sibfa_status s, const std::string& msg) {
  if (b) b->err = msg;
  return s;
}

void* balloc(sibfa_batch b, size_t bytes) {
  if (b->af) return b->af(bytes, b->user);
  void* p = nullptr;
  return hipMalloc(&p, bytes) == hipSuccess ? p : nullptr;
}

void bfree(sibfa_batch b, void* p) {
  if (!p) return;
  if (b->ff) b->ff(p, b->user);
  else (void)hipFree(p);
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// Carves the scratch arrays for `sites` sites and `clusters` clusters out of
// one allocation (or only measures it when base is null).
size_t carve(char* base, size_t sites, size_t clusters, ClusterArgs* a) {
  size_t o = 0;
  auto take = [&](size_t bytes) {
    char* p = base ? base + o : nullptr;
    o += align256(bytes);
    return p;
  };
  char* off = take((clusters + 1) * sizeof(int));
  char* warm = take(clusters * sizeof(int));
  char* npol = take(clusters * sizeof(int));
  char* polsite = take(sites * sizeof(int));
  char* prank = take(sites * sizeof(int));
  char* sval = take(sites * sizeof(double));
  char* pp = take(sites * sizeof(double4));
  char* pa = take(sites * sizeof(double));
  char* palpha = take(sites * 6 * sizeof(double));
  char* painv = take(sites * 6 * sizeof(double));
  char* E0 = take(sites * sizeof(double4));
  char* X = take(sites * sizeof(double4));
  char* Rr = take(sites * sizeof(double4));
  if (a) {
    a->off = reinterpret_cast<int*>(off);
    a->warm = reinterpret_cast<int*>(warm);
    a->npol = reinterpret_cast<int*>(npol);
    a->polsite = reinterpret_cast<int*>(polsite);
    a->prank = reinterpret_cast<int*>(prank);
    a->sval = reinterpret_cast<double*>(sval);
    a->pp = reinterpret_cast<double4*>(pp);
    a->pa = reinterpret_cast<double*>(pa);
    a->palpha = reinterpret_cast<double*>(palpha);
    a->painv = reinterpret_cast<double*>(painv);
    a->E0 = reinterpret_cast<double4*>(E0);
    a->X = reinterpret_cast<double4*>(X);
    a->Rr = reinterpret_cast<double4*>(Rr);
  }
  return o;
}

#define BHIP(call)                                                                  \
  do {                                                                              \
    hipError_t e_ = (call);                                                         \
    if (e_ != hipSuccess) return bfail(b, SIBFA_E_DEVICE, hipGetErrorString(e_));   \
  } while (0)

template <typename R>
void launch_batch(const ClusterArgs& a, hipStream_t st) {
  const int grid = std::min(a.nclusters, 16384);
  hipLaunchKernelGGL(k_cl_prep<R>, dim3(grid), dim3(kClBlock), 0, st, a);
  hipLaunchKernelGGL(k_cl_solve<R>, dim3(grid), dim3(kClBlock), 0, st, a);
  if (a.forces) hipLaunchKernelGGL(k_cl_force<R>, dim3(grid), dim3(kClBlock), 0, st, a);
}

}  // namespace

extern "C" {

sibfa_status sibfa_batch_create(sibfa_batch* out, int device, void* hip_stream,
                                sibfa_alloc_fn alloc_fn, sibfa_free_fn free_fn, void* user) {
  if (!out) return SIBFA_E_ARG;
  *out = nullptr;
  if ((alloc_fn == nullptr) != (free_fn == nullptr)) return SIBFA_E_ARG;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return SIBFA_E_DEVICE;
  if (hipSetDevice(device) != hipSuccess) return SIBFA_E_DEVICE;
  sibfa_batch b = new sibfa_batch_s();
  b->device = device;
  b->stream = static_cast<hipStream_t>(hip_stream);
  b->af = alloc_fn;
  b->ff = free_fn;
  b->user = user;
  if (hipEventCreateWithFlags(&b->staged, hipEventDisableTiming) != hipSuccess) {
    delete b;
    return SIBFA_E_DEVICE;
  }
  *out = b;
  return SIBFA_OK;
}

void sibfa_batch_destroy(sibfa_batch b) {
  if (!b) return;
  (void)hipSetDevice(b->device);
  (void)hipStreamSynchronize(b->stream);
  bfree(b, b->scratch);
  if (b->h_stage) (void)hipHostFree(b->h_stage);
  if (b->staged) (void)hipEventDestroy(b->staged);
  delete b;
}

const char* sibfa_batch_last_error(sibfa_batch b) { return b ? b->err.c_str() : "null batch"; }

sibfa_status sibfa_batch_clusters(sibfa_batch b, int n_clusters, const int* site_offsets,
                                  const int* warm_start, const double* xyz, const int32_t* mol,
                                  const double* q, const double* dip, const double* quad,
                                  const double* alpha, const double* thole,
                                  const sibfa_params* params, double* mu, double* forces,
                                  double* e_pol, double* e_elec, int* iterations,
                                  double* rms_debye, int* status) {
  if (!b) return SIBFA_E_ARG;
  if (n_clusters <= 0 || !site_offsets)
    return bfail(b, SIBFA_E_ARG, "n_clusters > 0 and site_offsets required");
  if (!xyz || !mol || !q || !dip || !quad || !alpha || !params || !mu || !e_pol || !e_elec ||
      !iterations || !rms_debye || !status)
    return bfail(b, SIBFA_E_ARG, "a required array is NULL");
  if (!(params->tol_debye > 0.0) || params->max_iter < 1 || !(params->thole_a > 0.0) ||
      (params->precision != SIBFA_FP64 && params->precision != SIBFA_MIXED))
    return bfail(b, SIBFA_E_ARG, "tol_debye > 0, max_iter >= 1, thole_a > 0 and a valid precision required");
  if (site_offsets[0] != 0) return bfail(b, SIBFA_E_ARG, "site_offsets[0] must be 0");
  for (int c = 0; c < n_clusters; ++c) {
    const int nc = site_offsets[c + 1] - site_offsets[c];
    if (nc < 1 || nc > kClMaxSites)
      return bfail(b, SIBFA_E_ARG, "every cluster needs 1 to SIBFA_BATCH_MAX_SITES sites");
  }
  const size_t n = (size_t)site_offsets[n_clusters];
  BHIP(hipSetDevice(b->device));
  // staging: offsets then warm flags; wait for the previous upload first
  const size_t need = 2 * (size_t)n_clusters + 1;
  if (b->staged_pending) {
    BHIP(hipEventSynchronize(b->staged));
    b->staged_pending = false;
  }
  if (need > b->h_cap) {
    if (b->h_stage) BHIP(hipHostFree(b->h_stage));
    b->h_stage = nullptr;
    b->h_cap = 0;
    BHIP(hipHostMalloc(reinterpret_cast<void**>(&b->h_stage), need * sizeof(int),
                       hipHostMallocDefault));
    b->h_cap = need;
  }
  if (n > b->cap_sites || (size_t)n_clusters > b->cap_clusters) {
    // grow: earlier batches on the stream may still read the old arrays
    BHIP(hipStreamSynchronize(b->stream));
    const size_t sites = std::max(n, 2 * b->cap_sites);
    const size_t clusters = std::max<size_t>(n_clusters, std::max<size_t>(64, 2 * b->cap_clusters));
    bfree(b, b->scratch);
    b->scratch = nullptr;
    b->cap_sites = b->cap_clusters = 0;
    void* p = balloc(b, carve(nullptr, sites, clusters, nullptr));
    if (!p) return bfail(b, SIBFA_E_NOMEM, "batch scratch allocation failed");
    b->scratch = p;
    b->cap_sites = sites;
    b->cap_clusters = clusters;
  }
  ClusterArgs a{};
  carve(static_cast<char*>(b->scratch), b->cap_sites, b->cap_clusters, &a);
  for (int c = 0; c <= n_clusters; ++c) b->h_stage[c] = site_offsets[c];
  for (int c = 0; c < n_clusters; ++c)
    b->h_stage[n_clusters + 1 + c] = warm_start ? (warm_start[c] != 0) : 0;
  BHIP(hipMemcpyAsync(const_cast<int*>(a.off), b->h_stage, (n_clusters + 1) * sizeof(int),
                      hipMemcpyHostToDevice, b->stream));
  BHIP(hipMemcpyAsync(const_cast<int*>(a.warm), b->h_stage + n_clusters + 1,
                      n_clusters * sizeof(int), hipMemcpyHostToDevice, b->stream));
  BHIP(hipEventRecord(b->staged, b->stream));
  b->staged_pending = true;
  a.nclusters = n_clusters;
  a.nsites = (int)n;
  a.xyz = xyz;
  a.mol = mol;
  a.q = q;
  a.dip = dip;
  a.quad = quad;
  a.alpha = alpha;
  a.thole = thole;
  a.thole_a = params->thole_a;
  a.tol = params->tol_debye;
  a.max_iter = params->max_iter;
  a.mu = mu;
  a.forces = forces;
  a.e_pol = e_pol;
  a.e_elec = e_elec;
  a.iters = iterations;
  a.rms = rms_debye;
  a.status = status;
  if (params->precision == SIBFA_MIXED) launch_batch<float>(a, b->stream);
  else launch_batch<double>(a, b->stream);
  BHIP(hipGetLastError());
  return SIBFA_OK;
}

}  // extern "C"

namespace {

constexpr int kNaMaxDevices = 64;
std::mutex g_na_mu;
void* g_na_ptr[kNaMaxDevices] = {};

// Device address of `scratch` on `device` (which must be current), looked
// up once per device.  In host code the array's name is only a stand-in
// for the symbol: kernels get this address.
sibfa_status noalloc_scratch(int device, void** out) {
  std::lock_guard<std::mutex> lock(g_na_mu);
  if (!g_na_ptr[device]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return SIBFA_E_DEVICE;
    g_na_ptr[device] = p;
  }
  *out = g_na_ptr[device];
  return SIBFA_OK;
}

}  // namespace

extern "C" sibfa_status sibfa_batch_clusters_noalloc(
    int device, void* hip_stream, int n_clusters, int n_sites, const int* site_offsets,
    const int* warm_start, const double* xyz, const int32_t* mol, const double* q,
    const double* dip, const double* quad, const double* alpha, const double* thole,
    const sibfa_params* params, double* mu, double* forces, double* e_pol, double* e_elec,
    int* iterations, double* rms_debye, int* status) {
  if (n_clusters < 1 || n_clusters > SIBFA_BATCH_NOALLOC_MAX_CLUSTERS || n_sites < 1 ||
      n_sites > SIBFA_BATCH_NOALLOC_MAX_SITES)
    return SIBFA_E_ARG;
  if (!site_offsets || !xyz || !mol || !q || !dip || !quad || !alpha || !params || !mu ||
      !e_pol || !e_elec || !iterations || !rms_debye || !status)
    return SIBFA_E_ARG;
  if (!(params->tol_debye > 0.0) || params->max_iter < 1 || !(params->thole_a > 0.0) ||
      (params->precision != SIBFA_FP64 && params->precision != SIBFA_MIXED))
    return SIBFA_E_ARG;
  if (device < 0 || device >= kNaMaxDevices) return SIBFA_E_DEVICE;
  if (hipSetDevice(device) != hipSuccess) return SIBFA_E_DEVICE;
  // the layout of carve() must fit the static array
  if (carve(nullptr, kNaSites, kNaClusters, nullptr) > kNaBytes) return SIBFA_E_DEVICE;
  void* base = nullptr;
  if (noalloc_scratch(device, &base) != SIBFA_OK) return SIBFA_E_DEVICE;
  ClusterArgs a{};
  carve(static_cast<char*>(base), kNaSites, kNaClusters, &a);
  a.off = site_offsets;   // the caller's device arrays, checked per cluster
  a.warm = warm_start;
  a.nclusters = n_clusters;
  a.nsites = n_sites;
  a.xyz = xyz;
  a.mol = mol;
  a.q = q;
  a.dip = dip;
  a.quad = quad;
  a.alpha = alpha;
  a.thole = thole;
  a.thole_a = params->thole_a;
  a.tol = params->tol_debye;
  a.max_iter = params->max_iter;
  a.mu = mu;
  a.forces = forces;
  a.e_pol = e_pol;
  a.e_elec = e_elec;
  a.iters = iterations;
  a.rms = rms_debye;
  a.status = status;
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  if (params->precision == SIBFA_MIXED) launch_batch<float>(a, st);
  else launch_batch<double>(a, st);
  return hipGetLastError() == hipSuccess ? SIBFA_OK : SIBFA_E_DEVICE;
}
