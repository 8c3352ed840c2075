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
// Spreading uses global floating-point atomics; each site touches p^3
// points in p*p rows of p consecutive addresses.
#include "common.h"
#include "kernels.h"

namespace sibfa {

template <typename R>
__device__ __forceinline__ void grid_add(const PmeView& pm, size_t idx, R v);
template <>
__device__ __forceinline__ void grid_add<double>(const PmeView& pm, size_t idx, double v) {
  atomicAdd(pm.Q + idx, v);
}
template <>
__device__ __forceinline__ void grid_add<float>(const PmeView& pm, size_t idx, float v) {
  atomicAdd(pm.Q32 + idx, v);
}

template <typename R>
__device__ __forceinline__ R grid_phi(const PmeView& pm, size_t idx);
template <>
__device__ __forceinline__ double grid_phi<double>(const PmeView& pm, size_t idx) { return pm.phi[idx]; }
template <>
__device__ __forceinline__ float grid_phi<float>(const PmeView& pm, size_t idx) { return pm.phi32[idx]; }

template <typename R, int P, int ND>
__device__ __forceinline__ void site_splines(const PmeView& pm, double x, double y, double z,
                                             int base[3], R th[3][ND + 1][P]) {
  const double xs[3] = {x, y, z};
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const double u = xs[a] * pm.scale[a];
    const double fl = floor(u);
    int k = (int)fl;
    if (k >= pm.K[a]) k -= pm.K[a];
    if (k < 0) k += pm.K[a];
    base[a] = k;
    bspline_weights<R, P, ND>((R)(u - fl), th[a]);
  }
}

// ------------------------------------------------------------ spreading
template <typename R, int P>
__global__ __launch_bounds__(kBlock) void k_spread_mult(SysView s, PmeView pm, const double4* mu) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= s.n) return;
  const double4 p = s.sp[i], d4 = s.sd[i], t4 = s.sth[i];
  const double2 t2 = s.sth2[i];
  double dx = d4.x, dy = d4.y, dz = d4.z;
  if (mu) {
    const double4 m = mu[i];
    dx += m.x; dy += m.y; dz += m.z;
  }
  int base[3];
  R th[3][3][P];
  site_splines<R, P, 2>(pm, p.x, p.y, p.z, base, th);
  const R sx = (R)pm.scale[0], sy = (R)pm.scale[1], sz = (R)pm.scale[2];
  const R q = (R)p.w;
  const R Dx = (R)dx * sx, Dy = (R)dy * sy, Dz = (R)dz * sz;
  const R third = R(1.0 / 3.0);
  const R Txx = (R)t4.x * sx * sx * third, Tyy = (R)t4.w * sy * sy * third,
          Tzz = (R)t2.y * sz * sz * third;
  const R Txy = R(2) * third * (R)t4.y * sx * sy, Txz = R(2) * third * (R)t4.z * sx * sz,
          Tyz = R(2) * third * (R)t2.x * sy * sz;
  for (int tz = 0; tz < P; ++tz) {
    int iz = base[2] - tz; if (iz < 0) iz += pm.K[2];
    const R z0 = th[2][0][tz], z1 = th[2][1][tz], z2 = th[2][2][tz];
    for (int ty = 0; ty < P; ++ty) {
      int iy = base[1] - ty; if (iy < 0) iy += pm.K[1];
      const R y0 = th[1][0][ty], y1 = th[1][1][ty], y2 = th[1][2][ty];
      const R c0 = q * y0 * z0 + Dy * y1 * z0 + Dz * y0 * z1 + Tyy * y2 * z0 + Tzz * y0 * z2 +
                   Tyz * y1 * z1;
      const R c1 = Dx * y0 * z0 + Txy * y1 * z0 + Txz * y0 * z1;
      const R c2 = Txx * y0 * z0;
      const size_t row = ((size_t)iz * pm.K[1] + iy) * pm.K[0];
#pragma unroll
      for (int tx = 0; tx < P; ++tx) {
        int ix = base[0] - tx; if (ix < 0) ix += pm.K[0];
        const R v = c0 * th[0][0][tx] + c1 * th[0][1][tx] + c2 * th[0][2][tx];
        grid_add<R>(pm, row + ix, v);
      }
    }
  }
}

template <typename R, int P>
__global__ __launch_bounds__(kBlock) void k_spread_dip(SysView s, PmeView pm, Reduce red,
                                                       DirUpdate du) {
  const int pi = blockIdx.x * blockDim.x + threadIdx.x;
  if (pi >= s.npol) return;
  double4 pv = du.p[pi];
  if (du.upd) {
    const double beta = red.scalars[du.num] / red.scalars[du.den];
    const double4 z = du.z[pi];
    pv = make_double4(z.x + beta * pv.x, z.y + beta * pv.y, z.z + beta * pv.z, 0.0);
    du.p[pi] = pv;
    du.p32[pi] = make_float4((float)pv.x, (float)pv.y, (float)pv.z, 0.f);
  }
  const double4 x = s.pp[pi];
  int base[3];
  R th[3][2][P];
  site_splines<R, P, 1>(pm, x.x, x.y, x.z, base, th);
  const R Dx = (R)pv.x * (R)pm.scale[0], Dy = (R)pv.y * (R)pm.scale[1],
          Dz = (R)pv.z * (R)pm.scale[2];
  for (int tz = 0; tz < P; ++tz) {
    int iz = base[2] - tz; if (iz < 0) iz += pm.K[2];
    const R z0 = th[2][0][tz], z1 = th[2][1][tz];
    for (int ty = 0; ty < P; ++ty) {
      int iy = base[1] - ty; if (iy < 0) iy += pm.K[1];
      const R y0 = th[1][0][ty], y1 = th[1][1][ty];
      const R c0 = Dy * y1 * z0 + Dz * y0 * z1;
      const R c1 = Dx * y0 * z0;
      const size_t row = ((size_t)iz * pm.K[1] + iy) * pm.K[0];
#pragma unroll
      for (int tx = 0; tx < P; ++tx) {
        int ix = base[0] - tx; if (ix < 0) ix += pm.K[0];
        grid_add<R>(pm, row + ix, c0 * th[0][0][tx] + c1 * th[0][1][tx]);
      }
    }
  }
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

template <typename R, int P>
__global__ __launch_bounds__(kBlock) void k_gather_force(SysView s, PmeView pm, const double4* mu,
                                                         const double4* Freal, const int* perm,
                                                         double* out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= s.n) return;
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
}

// ------------------------------------------------------------ launchers
template <int P>
static void spread_mult_p(const SysView& s, const PmeView& pm, const double4* mu, bool mixed,
                          hipStream_t st) {
  const dim3 g((s.n + kBlock - 1) / kBlock), b(kBlock);
  if (mixed) hipLaunchKernelGGL((k_spread_mult<float, P>), g, b, 0, st, s, pm, mu);
  else hipLaunchKernelGGL((k_spread_mult<double, P>), g, b, 0, st, s, pm, mu);
}

void launch_spread_mult(const SysView& s, const PmeView& pm, const double4* mu, bool mixed,
                        hipStream_t st) {
  switch (pm.order) {
    case 4: spread_mult_p<4>(s, pm, mu, mixed, st); break;
    case 6: spread_mult_p<6>(s, pm, mu, mixed, st); break;
    default: spread_mult_p<5>(s, pm, mu, mixed, st); break;
  }
}

template <int P>
static void spread_dip_p(const SysView& s, const PmeView& pm, const Reduce& red, DirUpdate du,
                         bool mixed, hipStream_t st) {
  const dim3 g((s.npol + kBlock - 1) / kBlock), b(kBlock);
  if (mixed) hipLaunchKernelGGL((k_spread_dip<float, P>), g, b, 0, st, s, pm, red, du);
  else hipLaunchKernelGGL((k_spread_dip<double, P>), g, b, 0, st, s, pm, red, du);
}

void launch_spread_dip(const SysView& s, const PmeView& pm, const Reduce& red, DirUpdate du,
                       bool mixed, hipStream_t st) {
  switch (pm.order) {
    case 4: spread_dip_p<4>(s, pm, red, du, mixed, st); break;
    case 6: spread_dip_p<6>(s, pm, red, du, mixed, st); break;
    default: spread_dip_p<5>(s, pm, red, du, mixed, st); break;
  }
}

template <int P>
static void gather_field_p(const SysView& s, const PmeView& pm, double4* E0, bool mixed,
                           hipStream_t st) {
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

template <int P>
static void gather_force_p(const SysView& s, const PmeView& pm, const double4* mu,
                           const double4* Freal, const int* perm, double* out, bool mixed,
                           hipStream_t st) {
  const dim3 g((s.n + kBlock - 1) / kBlock), b(kBlock);
  if (mixed)
    hipLaunchKernelGGL((k_gather_force<float, P>), g, b, 0, st, s, pm, mu, Freal, perm, out);
  else
    hipLaunchKernelGGL((k_gather_force<double, P>), g, b, 0, st, s, pm, mu, Freal, perm, out);
}

void launch_gather_force(const SysView& s, const PmeView& pm, const double4* mu,
                         const double4* Freal, const int* perm, double* out, bool mixed,
                         hipStream_t st) {
  switch (pm.order) {
    case 4: gather_force_p<4>(s, pm, mu, Freal, perm, out, mixed, st); break;
    case 6: gather_force_p<6>(s, pm, mu, Freal, perm, out, mixed, st); break;
    default: gather_force_p<5>(s, pm, mu, Freal, perm, out, mixed, st); break;
  }
}

}  // namespace sibfa
