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
// One workgroup per brick of B^3 grid points, accumulated in LDS.  A site
// with base index b touches points b - t, t = 0..p-1, so a brick receives
// contributions from the sites whose home brick (the brick holding b) is the
// brick itself or its successor along any axis: 8 home bricks.  Each site
// adds its in-brick points with LDS atomics; the finished tile is stored
// with plain coalesced writes, every grid point by exactly one brick, so the
// grid needs no clearing and no global atomics are used.

__global__ void k_brick_bin(SysView s, PmeView pm, int pol, int* brick_of, int* counts) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int n = pol ? s.npol : s.n;
  if (i >= n) return;
  double x[3];
  if (pol) { const double4 p = s.pp[i]; x[0] = p.x; x[1] = p.y; x[2] = p.z; }
  else { const double4 p = s.sp[i]; x[0] = p.x; x[1] = p.y; x[2] = p.z; }
  int h[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    double fr;
    h[a] = grid_base(x[a], pm.scale[a], pm.K[a], &fr) / pm.Bb[a];
  }
  const int b = h[0] + pm.nb[0] * (h[1] + pm.nb[1] * h[2]);
  brick_of[i] = b;
  atomicAdd(&counts[b], 1);
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

// Per-axis setup of a site against a brick: base index, offset d of the
// base from the brick origin (mod K) and the contributing t range.
struct AxisSpan {
  int d, tlo, thi;
};

template <int P>
__device__ __forceinline__ bool axis_span(int base, int x0, int Bx, int K, AxisSpan& a) {
  int d = base - x0;
  if (d < 0) d += K;
  a.d = d;
  a.tlo = d - Bx + 1 > 0 ? d - Bx + 1 : 0;
  a.thi = d < P - 1 ? d : P - 1;
  return a.tlo <= a.thi;
}

// FULL: multipoles (q, d [+ mu], Theta) of all sites; otherwise dipoles of
// the polarizable sites (with the optional direction update).
//
// Work split: the brick's candidate sites (the 8 home bricks' lists, taken
// as one concatenated range) are handled in chunks of CH per wavefront.  A
// wave stages its chunk in LDS -- the sites that reach the brick, compacted
// with a ballot, with their B-spline weights, amplitudes and in-brick t
// ranges -- and then spreads (site, ty, tz) work items over its 64 lanes,
// each adding one row of up to p points to the LDS tile with LDS atomics.
template <typename R, int P, bool FULL>
struct Stage {
  static constexpr int ND = FULL ? 2 : 1;
  static constexpr int NA = FULL ? 10 : 3;
  static constexpr int CH = FULL ? 16 : 32;
  R th[3][ND + 1][P][CH];
  R amp[NA][CH];
  int d[3][CH];
  int lo[3][CH];
  int hi[3][CH];
};

template <typename R, int P, bool FULL>
__global__ __launch_bounds__(kBlock) void k_spread_brick(SysView s, PmeView pm, Reduce red,
                                                         DirUpdate du, const double4* mu) {
  if (stopped(red.stop)) return;
  using St = Stage<R, P, FULL>;
  constexpr int ND = St::ND, CH = St::CH, NW = kBlock / 64;
  __shared__ R tile[kBrick * kBrick * kBrick];
  __shared__ St stage[NW];
  const int S0 = pm.Bb[0], S1 = pm.Bb[1], S2 = pm.Bb[2];   // full brick sizes (tile strides)
  const int nb0 = pm.nb[0], nb1 = pm.nb[1], nb2 = pm.nb[2];
  const int bx = blockIdx.x % nb0, by = (blockIdx.x / nb0) % nb1, bz = blockIdx.x / (nb0 * nb1);
  const int o[3] = {bx * S0, by * S1, bz * S2};
  const int Bs[3] = {min(S0, pm.K[0] - o[0]), min(S1, pm.K[1] - o[1]), min(S2, pm.K[2] - o[2])};
  const int ntile = S0 * S1 * S2;
  for (int e = threadIdx.x; e < ntile; e += blockDim.x) tile[e] = R(0);
  double beta = 0.0;
  if (!FULL && du.upd) {
    const double num = slot_total(red, du.num);
    const double den = slot_total(red, du.den);
    beta = num / den;
  }
  const int* start = FULL ? pm.bstart_all : pm.bstart_pol;
  const int* order = FULL ? pm.border_all : pm.border_pol;
  // the candidate ranges of the (up to) 8 home bricks, concatenated
  int rs[8], rl[8], total = 0;
#pragma unroll
  for (int h = 0; h < 8; ++h) {
    const int dx = h & 1, dy = (h >> 1) & 1, dz = h >> 2;
    rs[h] = 0; rl[h] = 0;
    if ((dx && nb0 == 1) || (dy && nb1 == 1) || (dz && nb2 == 1)) continue;
    const int hid = (bx + dx) % nb0 + nb0 * ((by + dy) % nb1 + nb1 * ((bz + dz) % nb2));
    rs[h] = start[hid];
    rl[h] = start[hid + 1] - rs[h];
    total += rl[h];
  }
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  St& sg = stage[wv];
  const R sc[3] = {(R)pm.scale[0], (R)pm.scale[1], (R)pm.scale[2]};
  const int rounds = (total + NW * CH - 1) / (NW * CH);
  __syncthreads();
  for (int rd = 0; rd < rounds; ++rd) {
    // ---- stage this wave's chunk
    const int c = (rd * NW + wv) * CH + lane;
    bool contrib = false;
    int idx = -1, hh = 0;
    if (lane < CH && c < total) {
      int rem = c;
#pragma unroll
      for (int h = 0; h < 8; ++h) {
        if (idx < 0) {
          if (rem < rl[h]) { idx = order[rs[h] + rem]; hh = h; }
          else rem -= rl[h];
        }
      }
    }
    double x[3] = {0, 0, 0};
    double4 pv = make_double4(0.0, 0.0, 0.0, 0.0);
    int base[3] = {0, 0, 0};
    double fr[3] = {0, 0, 0};
    AxisSpan sp[3];
    if (idx >= 0) {
      if (FULL) {
        const double4 p = s.sp[idx];
        x[0] = p.x; x[1] = p.y; x[2] = p.z;
      } else {
        const double4 p = s.pp[idx];
        x[0] = p.x; x[1] = p.y; x[2] = p.z;
        pv = du.p_old[idx];
        if (du.upd) {
          const double4 z = du.z[idx];
          pv = make_double4(z.x + beta * pv.x, z.y + beta * pv.y, z.z + beta * pv.z, 0.0);
          if (hh == 0) {
            du.p_new[idx] = pv;
            du.p_new32[idx] = make_float4((float)pv.x, (float)pv.y, (float)pv.z, 0.f);
          }
        }
      }
      contrib = true;
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        base[a] = grid_base(x[a], pm.scale[a], pm.K[a], &fr[a]);
        contrib = contrib && axis_span<P>(base[a], o[a], Bs[a], pm.K[a], sp[a]);
      }
    }
    const unsigned long long mask = __ballot(contrib);
    const int cnt = __popcll(mask);
    if (contrib) {
      const unsigned long long below = lane == 0 ? 0ull : (~0ull >> (64 - lane));
      const int slot = __popcll(mask & below);
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        R th[ND + 1][P];
        bspline_weights<R, P, ND>((R)fr[a], th);
#pragma unroll
        for (int k = 0; k <= ND; ++k)
#pragma unroll
          for (int t = 0; t < P; ++t) sg.th[a][k][t][slot] = th[k][t];
        sg.d[a][slot] = sp[a].d;
        sg.lo[a][slot] = sp[a].tlo;
        sg.hi[a][slot] = sp[a].thi;
      }
      if (FULL) {
        const double4 p = s.sp[idx], d4 = s.sd[idx], t4 = s.sth[idx];
        const double2 t2 = s.sth2[idx];
        double ddx = d4.x, ddy = d4.y, ddz = d4.z;
        if (mu) {
          const double4 m = mu[idx];
          ddx += m.x; ddy += m.y; ddz += m.z;
        }
        const R third = R(1.0 / 3.0);
        sg.amp[0][slot] = (R)p.w;
        sg.amp[1][slot] = (R)ddx * sc[0];
        sg.amp[2][slot] = (R)ddy * sc[1];
        sg.amp[3][slot] = (R)ddz * sc[2];
        sg.amp[4 % St::NA][slot] = (R)t4.x * sc[0] * sc[0] * third;
        sg.amp[5 % St::NA][slot] = (R)t4.w * sc[1] * sc[1] * third;
        sg.amp[6 % St::NA][slot] = (R)t2.y * sc[2] * sc[2] * third;
        sg.amp[7 % St::NA][slot] = R(2) * third * (R)t4.y * sc[0] * sc[1];
        sg.amp[8 % St::NA][slot] = R(2) * third * (R)t4.z * sc[0] * sc[2];
        sg.amp[9 % St::NA][slot] = R(2) * third * (R)t2.x * sc[1] * sc[2];
      } else {
        sg.amp[0][slot] = (R)pv.x * sc[0];
        sg.amp[1][slot] = (R)pv.y * sc[1];
        sg.amp[2][slot] = (R)pv.z * sc[2];
      }
    }
    __syncthreads();
    // ---- spread (site, ty, tz) rows of the staged sites
    for (int it = lane; it < cnt * P * P; it += 64) {
      const int slot = it / (P * P), r = it - slot * (P * P);
      const int ty = r % P, tz = r / P;
      if (ty < sg.lo[1][slot] || ty > sg.hi[1][slot] || tz < sg.lo[2][slot] || tz > sg.hi[2][slot])
        continue;
      const R y0 = sg.th[1][0][ty][slot], y1 = sg.th[1][1][ty][slot];
      const R z0 = sg.th[2][0][tz][slot], z1 = sg.th[2][1][tz][slot];
      R c0, c1, c2 = R(0);
      if (FULL) {
        const R y2 = sg.th[1][ND][ty][slot], z2 = sg.th[2][ND][tz][slot];
        const R* A = &sg.amp[0][0];
        c0 = A[0 * CH + slot] * y0 * z0 + A[2 * CH + slot] * y1 * z0 + A[3 * CH + slot] * y0 * z1 +
             A[5 * CH + slot] * y2 * z0 + A[6 * CH + slot] * y0 * z2 + A[9 * CH + slot] * y1 * z1;
        c1 = A[1 * CH + slot] * y0 * z0 + A[7 * CH + slot] * y1 * z0 + A[8 * CH + slot] * y0 * z1;
        c2 = A[4 * CH + slot] * y0 * z0;
      } else {
        c0 = sg.amp[1][slot] * y1 * z0 + sg.amp[2][slot] * y0 * z1;
        c1 = sg.amp[0][slot] * y0 * z0;
      }
      const int oy = sg.d[1][slot] - ty, oz = sg.d[2][slot] - tz, dx = sg.d[0][slot];
      R* row = tile + (oz * S1 + oy) * S0;
      const int lo = sg.lo[0][slot], hi = sg.hi[0][slot];
      for (int tx = lo; tx <= hi; ++tx) {
        R v = c0 * sg.th[0][0][tx][slot] + c1 * sg.th[0][1][tx][slot];
        if (FULL) v += c2 * sg.th[0][ND][tx][slot];
        atomicAdd(row + (dx - tx), v);
      }
    }
    __syncthreads();
  }
  R* Q = grid_out<R>(pm);
  for (int e = threadIdx.x; e < ntile; e += blockDim.x) {
    const int ox = e % S0, oy = (e / S0) % S1, oz = e / (S0 * S1);
    if (ox < Bs[0] && oy < Bs[1] && oz < Bs[2])
      Q[((size_t)(o[2] + oz) * pm.K[1] + (o[1] + oy)) * pm.K[0] + (o[0] + ox)] = tile[e];
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
template <int P, bool FULL>
static void spread_brick_p(const SysView& s, const PmeView& pm, const Reduce& red, DirUpdate du,
                           const double4* mu, bool mixed, hipStream_t st) {
  const dim3 g(pm.nb[0] * pm.nb[1] * pm.nb[2]), b(kBlock);
  if (mixed) hipLaunchKernelGGL((k_spread_brick<float, P, FULL>), g, b, 0, st, s, pm, red, du, mu);
  else hipLaunchKernelGGL((k_spread_brick<double, P, FULL>), g, b, 0, st, s, pm, red, du, mu);
}

template <bool FULL>
static void spread_brick(const SysView& s, const PmeView& pm, const Reduce& red, DirUpdate du,
                         const double4* mu, bool mixed, hipStream_t st) {
  switch (pm.order) {
    case 4: spread_brick_p<4, FULL>(s, pm, red, du, mu, mixed, st); break;
    case 6: spread_brick_p<6, FULL>(s, pm, red, du, mu, mixed, st); break;
    default: spread_brick_p<5, FULL>(s, pm, red, du, mu, mixed, st); break;
  }
}

void launch_spread_mult(const SysView& s, const PmeView& pm, const double4* mu, bool mixed,
                        hipStream_t st) {
  DirUpdate du{};
  Reduce red{};
  spread_brick<true>(s, pm, red, du, mu, mixed, st);
}

void launch_spread_dip(const SysView& s, const PmeView& pm, const Reduce& red, DirUpdate du,
                       bool mixed, hipStream_t st) {
  spread_brick<false>(s, pm, red, du, nullptr, mixed, st);
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
