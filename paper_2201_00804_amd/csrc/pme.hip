// Smooth PME: B-spline spreading of multipoles onto the charge grid and
// gathering of potential derivatives (Essmann et al. 1995, the SPME method
// the paper uses for multipoles and polarization).
//
// With u_a = K_a r_a / L_a and W(k) = prod_a M_p(u_a - k_a), a site adds
//   q W + d.grad W + 1/3 Theta:grad grad W
// to grid point k (gradients with respect to the site position, so a
// derivative along a carries K_a/L_a).  After the convolution the grid holds
// the potential phi(k); a site's potential derivatives are sums of phi(k)
// times derivatives of W.  Grid layout: x fastest, [K2][K1][K0].
// Spreading accumulates in LDS per grid brick (see below); gathering reads
// p^3 points per site in p*p rows of p consecutive addresses.
#include "common.h"
#include "kernels.h"

namespace sibfa {

template <typename R>
__device__ __forceinline__ R grid_phi(const PmeView& pm, size_t idx);
template <>
__device__ __forceinline__ double grid_phi<double>(const PmeView& pm, size_t idx) { return pm.phi[idx]; }
template <>
__device__ __forceinline__ float grid_phi<float>(const PmeView& pm, size_t idx) { return pm.phi32[idx]; }

// ------------------------------------------------------------ spreading
// Sites are binned by home brick, the brick of B^3 grid points (B <= 8, per
// axis; the last brick along an axis never has fewer than p - 1 points)
// holding their base index b.  A site touches points b - t, t = 0..p-1, so
// all contributions of a brick's sites fall in the brick extended by p - 1
// points towards lower indices: its tile, (B + p - 1)^3 points.
//
//  k_spread_tile : one workgroup per brick spreads its own sites into the
//                  tile (every site is evaluated once) and stores the tile;
//  fold          : every grid point sums the tiles that cover it -- its own
//                  brick's and, along each axis where it lies within p - 1
//                  points of the next brick, that brick's -- in a fixed
//                  order.  No global atomics, no clearing, deterministic.
//                  k_spread_fold writes the real grid Q the convolution
//                  starts from.

// Sites come in cell-sorted order, so a wavefront's sites fall in a few
// bricks: one counter atomic per run of equal bricks.
__global__ void k_brick_bin(SysView s, PmeView pm, int pol, int* brick_of, int* counts) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int n = pol ? s.npol : s.n;
  const bool act = i < n;
  int b = 0;
  if (act) {
    double x[3];
    if (pol) { const double4 p = s.pp[i]; x[0] = p.x; x[1] = p.y; x[2] = p.z; }
    else { const double4 p = s.sp[i]; x[0] = p.x; x[1] = p.y; x[2] = p.z; }
    int h[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      double fr;
      h[a] = grid_base(x[a], pm.scale[a], pm.K[a], &fr) / pm.Bb[a];
    }
    b = h[0] + pm.nb[0] * (h[1] + pm.nb[1] * h[2]);
    brick_of[i] = b;
  }
  wave_atomic_inc(counts, b, act);
}

void launch_brick_bin(const SysView& s, const PmeView& pm, int pol, int* brick_of, int* counts,
                      hipStream_t st) {
  const int n = pol ? s.npol : s.n;
  if (n > 0)
    hipLaunchKernelGGL(k_brick_bin, dim3((n + kBlock - 1) / kBlock), dim3(kBlock), 0, st, s, pm,
                       pol, brick_of, counts);
}

template <typename R>
__device__ __forceinline__ R* grid_out(const PmeView& pm);
template <>
__device__ __forceinline__ double* grid_out<double>(const PmeView& pm) { return pm.Q; }
template <>
__device__ __forceinline__ float* grid_out<float>(const PmeView& pm) { return pm.Q32; }
template <typename R>
__device__ __forceinline__ R* tile_buf(const PmeView& pm);
template <>
__device__ __forceinline__ double* tile_buf<double>(const PmeView& pm) { return pm.tiles; }
template <>
__device__ __forceinline__ float* tile_buf<float>(const PmeView& pm) { return pm.tiles32; }

// FULL: multipoles (q, d [+ mu], Theta) of all sites; otherwise the dipoles
// of the polarizable sites.
//
// Owner-computes, no atomics: thread (x, y) of the workgroup owns one tile
// column and keeps its T2 values in registers.  A site's contribution is a
// sum of separable terms  A theta_x^(kx)(x) theta_y^(ky)(y) theta_z^(kz)(z),
// regrouped by kz as  sum_kz U_kz(x, y) theta_z^(kz)(z).  Sites are staged
// in chunks with their B-spline weights expanded to the tile width (zeros
// outside the p-point support), so the inner loop is a few LDS reads (the z
// weights are the same address for every lane) and FMAs.  The brick lists
// are sorted by site index when they are built, so the tile sums -- and the
// grid -- are reproducible bit for bit.
constexpr int kSpreadBlock = 192;      // >= (kBrick + p - 1)^2 columns, p <= 6

template <bool FULL>
struct SpreadShape {
  static constexpr int ND = FULL ? 2 : 1;   // highest derivative order
  static constexpr int NA = FULL ? 10 : 3;  // amplitudes per site
  static constexpr int CH = FULL ? 32 : 64; // sites per staged chunk
};

template <typename R, int P, bool FULL>
__global__ __launch_bounds__(kSpreadBlock) void k_spread_tile(SysView s, PmeView pm,
                                                              const double4* vec) {
  if (stopped(pm.stop)) return;
  using Sh = SpreadShape<FULL>;
  constexpr int ND = Sh::ND, NA = Sh::NA, CH = Sh::CH;
  constexpr int TM = kBrick + P - 1;
  __shared__ R w[3][ND + 1][CH][TM];
  __shared__ R amp[NA][CH];
  const int tid = threadIdx.x;
  const int T0 = pm.Bb[0] + P - 1, T1 = pm.Bb[1] + P - 1, T2 = pm.Bb[2] + P - 1;
  const int nb0 = pm.nb[0], nb1 = pm.nb[1];
  const int b = blockIdx.x;
  const int o[3] = {(b % nb0) * pm.Bb[0], ((b / nb0) % nb1) * pm.Bb[1], (b / (nb0 * nb1)) * pm.Bb[2]};
  const int* start = FULL ? pm.bstart_all : pm.bstart_pol;
  const int* order = FULL ? pm.border_all : pm.border_pol;
  const int s0 = start[b], total = start[b + 1] - s0;
  const bool owner = tid < T0 * T1;
  const int cx = owner ? tid % T0 : 0, cy = owner ? tid / T0 : 0;
  R acc[TM];
#pragma unroll
  for (int z = 0; z < TM; ++z) acc[z] = R(0);
  const R sc[3] = {(R)pm.scale[0], (R)pm.scale[1], (R)pm.scale[2]};
  for (int c0 = 0; c0 < total; c0 += CH) {
    const int n = min(CH, total - c0);
    __syncthreads();
    if (tid < 3 * n) {
      const int j = tid / 3, ax = tid - 3 * j;
      const int idx = order[s0 + c0 + j];
      const double4 p = FULL ? s.sp[idx] : s.pp[idx];
      const double xa = ax == 0 ? p.x : (ax == 1 ? p.y : p.z);
      double fr;
      const int base = grid_base(xa, pm.scale[ax], pm.K[ax], &fr);
      R th[ND + 1][P];
      bspline_weights<R, P, ND>((R)fr, th);
      const int top = base - o[ax] + P - 1;
#pragma unroll
      for (int k = 0; k <= ND; ++k)
#pragma unroll
        for (int z = 0; z < TM; ++z) {
          const int d = top - z;
          R v = R(0);
#pragma unroll
          for (int t = 0; t < P; ++t) v = d == t ? th[k][t] : v;
          w[ax][k][j][z] = v;
        }
      if (ax == 0) {
        if (FULL) {
          const double4 d4 = s.sd[idx], t4 = s.sth[idx];
          const double2 t2 = s.sth2[idx];
          double ddx = d4.x, ddy = d4.y, ddz = d4.z;
          if (vec) {
            const double4 m = vec[idx];
            ddx += m.x; ddy += m.y; ddz += m.z;
          }
          const R third = R(1.0 / 3.0);
          amp[0][j] = (R)p.w;
          amp[1][j] = (R)ddx * sc[0];
          amp[2][j] = (R)ddy * sc[1];
          amp[3][j] = (R)ddz * sc[2];
          amp[4 % NA][j] = (R)t4.x * sc[0] * sc[0] * third;
          amp[5 % NA][j] = (R)t4.w * sc[1] * sc[1] * third;
          amp[6 % NA][j] = (R)t2.y * sc[2] * sc[2] * third;
          amp[7 % NA][j] = R(2) * third * (R)t4.y * sc[0] * sc[1];
          amp[8 % NA][j] = R(2) * third * (R)t4.z * sc[0] * sc[2];
          amp[9 % NA][j] = R(2) * third * (R)t2.x * sc[1] * sc[2];
        } else {
          const double4 pv = vec[idx];
          amp[0][j] = (R)pv.x * sc[0];
          amp[1][j] = (R)pv.y * sc[1];
          amp[2][j] = (R)pv.z * sc[2];
        }
      }
    }
    __syncthreads();
    if (owner) {
      for (int j = 0; j < n; ++j) {
        const R x0 = w[0][0][j][cx], x1 = w[0][1][j][cx];
        const R y0 = w[1][0][j][cy], y1 = w[1][1][j][cy];
        if (FULL) {
          const R x2 = w[0][ND][j][cx], y2 = w[1][ND][j][cy];
          const R U0 = x0 * (amp[0][j] * y0 + amp[2][j] * y1 + amp[5 % NA][j] * y2) +
                       x1 * (amp[1][j] * y0 + amp[7 % NA][j] * y1) + x2 * amp[4 % NA][j] * y0;
          const R U1 = x0 * (amp[3][j] * y0 + amp[9 % NA][j] * y1) + x1 * amp[8 % NA][j] * y0;
          const R U2 = x0 * amp[6 % NA][j] * y0;
          if (U0 == R(0) && U1 == R(0) && U2 == R(0)) continue;
#pragma unroll
          for (int z = 0; z < TM; ++z)
            acc[z] += U0 * w[2][0][j][z] + U1 * w[2][1][j][z] + U2 * w[2][ND][j][z];
        } else {
          const R U0 = amp[0][j] * x1 * y0 + amp[1][j] * x0 * y1;
          const R U1 = amp[2][j] * x0 * y0;
          if (U0 == R(0) && U1 == R(0)) continue;
#pragma unroll
          for (int z = 0; z < TM; ++z) acc[z] += U0 * w[2][0][j][z] + U1 * w[2][1][j][z];
        }
      }
    }
  }
  if (owner) {
    R* out = tile_buf<R>(pm) + (size_t)b * pm.tile_size;
#pragma unroll
    for (int z = 0; z < TM; ++z)
      if (z < T2) out[(z * T1 + cy) * T0 + cx] = acc[z];
  }
}

template <typename R>
__global__ __launch_bounds__(kBlock) void k_spread_fold(PmeView pm) {
  if (stopped(pm.stop)) return;
  const int K0 = pm.K[0], K1 = pm.K[1], K2 = pm.K[2];
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (size_t)K0 * K1 * K2) return;
  grid_out<R>(pm)[idx] = fold_point<R>(pm, (int)(idx % K0), (int)((idx / K0) % K1),
                                       (int)(idx / ((size_t)K0 * K1)));
}

void launch_spread_fold(const PmeView& pm, bool mixed, hipStream_t st) {
  const size_t npts = (size_t)pm.K[0] * pm.K[1] * pm.K[2];
  const dim3 g((unsigned)((npts + kBlock - 1) / kBlock)), b(kBlock);
  if (mixed) hipLaunchKernelGGL(k_spread_fold<float>, g, b, 0, st, pm);
  else hipLaunchKernelGGL(k_spread_fold<double>, g, b, 0, st, pm);
}

// ------------------------------------------------------------ gathering
template <typename R, int P>
__global__ __launch_bounds__(kBlock) void k_gather_field(SysView s, PmeView pm, double4* E0) {
  const int pi = blockIdx.x * blockDim.x + threadIdx.x;
  if (pi >= s.npol) return;
  const double4 x = s.pp[pi];
  int base[3];
  R th[3][2][P];
  site_splines<R, P, 1>(pm, x.x, x.y, x.z, base, th);
  double g[3] = {0.0, 0.0, 0.0};
  for (int tz = 0; tz < P; ++tz) {
    int iz = base[2] - tz; if (iz < 0) iz += pm.K[2];
    for (int ty = 0; ty < P; ++ty) {
      int iy = base[1] - ty; if (iy < 0) iy += pm.K[1];
      const size_t row = ((size_t)iz * pm.K[1] + iy) * pm.K[0];
      R s0 = 0, s1 = 0;
#pragma unroll
      for (int tx = 0; tx < P; ++tx) {
        int ix = base[0] - tx; if (ix < 0) ix += pm.K[0];
        const R v = grid_phi<R>(pm, row + ix);
        s0 += v * th[0][0][tx];
        s1 += v * th[0][1][tx];
      }
      g[0] += (double)(s1 * th[1][0][ty] * th[2][0][tz]);
      g[1] += (double)(s0 * th[1][1][ty] * th[2][0][tz]);
      g[2] += (double)(s0 * th[1][0][ty] * th[2][1][tz]);
    }
  }
  double4 e = E0[pi];
  e.x -= g[0] * pm.scale[0];
  e.y -= g[1] * pm.scale[1];
  e.z -= g[2] * pm.scale[2];
  E0[pi] = e;
}

// index of the (kx, ky, kz) derivative, kx + ky + kz <= 3
__host__ __device__ constexpr int didx(int kx, int ky, int kz) {
  return kx + 4 * (ky + 4 * kz);
}

// Reciprocal forces of the combined density at every site.  VIR: also the
// site terms of the reciprocal virial, sum_j [d'_jb d_a phi(r_j) +
// 2/3 Theta_jbc d_a d_c phi(r_j)] with d' = d + mu (block partials, slots
// S_VRG, row-major).
template <typename R, int P, bool VIR>
__global__ __launch_bounds__(kBlock) void k_gather_force(SysView s, PmeView pm, Reduce red,
                                                         const double4* mu, const double4* Freal,
                                                         const int* perm, double* out,
                                                         double4* FS, double* GS, bool self) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  double W[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
  if (i < s.n) {
    const double4 p = s.sp[i], d4 = s.sd[i], t4 = s.sth[i];
    const double2 t2 = s.sth2[i];
    const double4 m = mu[i];
    int base[3];
    R th[3][4][P];
    site_splines<R, P, 3>(pm, p.x, p.y, p.z, base, th);
    double D[64];
#pragma unroll
    for (int k = 0; k < 64; ++k) D[k] = 0.0;
    for (int tz = 0; tz < P; ++tz) {
      int iz = base[2] - tz; if (iz < 0) iz += pm.K[2];
      for (int ty = 0; ty < P; ++ty) {
        int iy = base[1] - ty; if (iy < 0) iy += pm.K[1];
        const size_t row = ((size_t)iz * pm.K[1] + iy) * pm.K[0];
        R sx[4] = {0, 0, 0, 0};
#pragma unroll
        for (int tx = 0; tx < P; ++tx) {
          int ix = base[0] - tx; if (ix < 0) ix += pm.K[0];
          const R v = grid_phi<R>(pm, row + ix);
#pragma unroll
          for (int k = 0; k < 4; ++k) sx[k] += v * th[0][k][tx];
        }
#pragma unroll
        for (int kz = 0; kz <= 3; ++kz)
#pragma unroll
          for (int ky = 0; ky <= 3 - kz; ++ky) {
            const R yz = th[1][ky][ty] * th[2][kz][tz];
#pragma unroll
            for (int kx = 0; kx <= 3 - ky - kz; ++kx) D[didx(kx, ky, kz)] += (double)(sx[kx] * yz);
          }
      }
    }
    const double sc[3] = {pm.scale[0], pm.scale[1], pm.scale[2]};
    auto der = [&](int a, int b, int c) -> double {   // b, c = -1 for lower order
      int k[3] = {0, 0, 0};
      double f = sc[a];
      k[a]++;
      if (b >= 0) { k[b]++; f *= sc[b]; }
      if (c >= 0) { k[c]++; f *= sc[c]; }
      return D[didx(k[0], k[1], k[2])] * f;
    };
    const double q = p.w;
    const double dd[3] = {d4.x + m.x, d4.y + m.y, d4.z + m.z};
    const double T[3][3] = {{t4.x, t4.y, t4.z}, {t4.y, t4.w, t2.x}, {t4.z, t2.x, t2.y}};
    const double4 fr = Freal[i];
    const double frr[3] = {fr.x, fr.y, fr.z};
    const int c = perm[i];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      double f = q * der(a, -1, -1);
      for (int b = 0; b < 3; ++b) {
        f += dd[b] * der(a, b, -1);
        for (int cc = 0; cc < 3; ++cc) f += T[b][cc] * der(a, b, cc) * (1.0 / 3.0);
      }
      out[3 * (size_t)c + a] = kCoulomb * (frr[a] - f);
    }
    if (FS) {
      // site field E = -grad phi and gradient -grad grad phi, plus the self
      // terms: 4 b^3/(3 sqrt pi) (d + mu) and 16 b^5/(15 sqrt pi) Theta
      // (the latter 3x the quadrupole self derivative, as the field
      // gradient enters the quadrupole energy with 1/3)
      const double b = pm.beta, b3 = b * b * b;
      const double sf = self ? 4.0 * b3 / (3.0 * kSqrtPi) : 0.0;
      const double st = self ? 16.0 * b3 * b * b / (15.0 * kSqrtPi) : 0.0;
      double4 e = FS[i];
      e.x += sf * dd[0] - der(0, -1, -1);
      e.y += sf * dd[1] - der(1, -1, -1);
      e.z += sf * dd[2] - der(2, -1, -1);
      FS[i] = e;
      const int ia[6] = {0, 0, 0, 1, 1, 2}, ib[6] = {0, 1, 2, 1, 2, 2};
#pragma unroll
      for (int k = 0; k < 6; ++k)
        GS[6 * (size_t)i + k] += st * T[ia[k]][ib[k]] - der(ia[k], ib[k], -1);
    }
    if (VIR) {
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        const double da = der(a, -1, -1);
#pragma unroll
        for (int b = 0; b < 3; ++b) {
          double w = dd[b] * da;
#pragma unroll
          for (int cc = 0; cc < 3; ++cc) w += (2.0 / 3.0) * T[b][cc] * der(a, cc, -1);
          W[3 * a + b] = w;
        }
      }
    }
  }
  if (VIR)
#pragma unroll
    for (int k = 0; k < 9; ++k) block_partial(W[k], red, S_VRG + k);
}

// ------------------------------------------------------------ launchers
template <int P, bool FULL>
static void spread_p(const PmeView& pm, const SysView& s, const double4* vec, bool mixed,
                     hipStream_t st) {
  const dim3 g(pm.nb[0] * pm.nb[1] * pm.nb[2]), bt(kSpreadBlock);
  if (mixed) hipLaunchKernelGGL((k_spread_tile<float, P, FULL>), g, bt, 0, st, s, pm, vec);
  else hipLaunchKernelGGL((k_spread_tile<double, P, FULL>), g, bt, 0, st, s, pm, vec);
}

template <bool FULL>
static void spread(const PmeView& pm, const SysView& s, const double4* vec, bool mixed,
                   hipStream_t st) {
  switch (pm.order) {
    case 4: spread_p<4, FULL>(pm, s, vec, mixed, st); break;
    case 6: spread_p<6, FULL>(pm, s, vec, mixed, st); break;
    default: spread_p<5, FULL>(pm, s, vec, mixed, st); break;
  }
}

void launch_spread_mult(const SysView& s, const PmeView& pm, const double4* mu, bool mixed,
                        hipStream_t st) {
  spread<true>(pm, s, mu, mixed, st);
}

void launch_spread_dip(const SysView& s, const PmeView& pm, const double4* p, bool mixed,
                       hipStream_t st) {
  spread<false>(pm, s, p, mixed, st);
}

template <int P>
static void gather_field_p(const SysView& s, const PmeView& pm, double4* E0, bool mixed,
                           hipStream_t st) {
  if (s.npol <= 0) return;
  const dim3 g((s.npol + kBlock - 1) / kBlock), b(kBlock);
  if (mixed) hipLaunchKernelGGL((k_gather_field<float, P>), g, b, 0, st, s, pm, E0);
  else hipLaunchKernelGGL((k_gather_field<double, P>), g, b, 0, st, s, pm, E0);
}

void launch_gather_field(const SysView& s, const PmeView& pm, double4* E0, bool mixed,
                         hipStream_t st) {
  switch (pm.order) {
    case 4: gather_field_p<4>(s, pm, E0, mixed, st); break;
    case 6: gather_field_p<6>(s, pm, E0, mixed, st); break;
    default: gather_field_p<5>(s, pm, E0, mixed, st); break;
  }
}

template <int P, bool VIR>
static void gather_force_pv(const SysView& s, const PmeView& pm, Reduce& red, const double4* mu,
                            const double4* Freal, const int* perm, double* out, bool mixed,
                            hipStream_t st, double4* FS, double* GS, bool self) {
  const dim3 g((s.n + kBlock - 1) / kBlock), b(kBlock);
  if (mixed)
    hipLaunchKernelGGL((k_gather_force<float, P, VIR>), g, b, 0, st, s, pm, red, mu, Freal, perm,
                       out, FS, GS, self);
  else
    hipLaunchKernelGGL((k_gather_force<double, P, VIR>), g, b, 0, st, s, pm, red, mu, Freal, perm,
                       out, FS, GS, self);
  if (VIR)
    for (int k = 0; k < 9; ++k) red.nparts[S_VRG + k] = (int)g.x;
}

template <int P>
static void gather_force_p(const SysView& s, const PmeView& pm, Reduce& red, const double4* mu,
                           const double4* Freal, const int* perm, double* out, bool mixed,
                           bool vir, hipStream_t st, double4* FS, double* GS, bool self) {
  if (vir) gather_force_pv<P, true>(s, pm, red, mu, Freal, perm, out, mixed, st, FS, GS, self);
  else gather_force_pv<P, false>(s, pm, red, mu, Freal, perm, out, mixed, st, FS, GS, self);
}

void launch_gather_force(const SysView& s, const PmeView& pm, Reduce& red, const double4* mu,
                         const double4* Freal, const int* perm, double* out, bool mixed,
                         bool virial, hipStream_t st, double4* FS, double* GS, bool self) {
  switch (pm.order) {
    case 4: gather_force_p<4>(s, pm, red, mu, Freal, perm, out, mixed, virial, st, FS, GS, self); break;
    case 6: gather_force_p<6>(s, pm, red, mu, Freal, perm, out, mixed, virial, st, FS, GS, self); break;
    default: gather_force_p<5>(s, pm, red, mu, Freal, perm, out, mixed, virial, st, FS, GS, self); break;
  }
}

}  // namespace sibfa
