// Molecular block preconditioner of the PCG solve (Eq. 18; the paper names
// a preconditioned conjugate gradient without fixing the preconditioner).
// For every molecule with at most kPcMax polarizable sites, M is the
// molecule's block of T in bare form: alpha_i^-1 on the diagonal blocks and
// the Thole-damped bare dipole-dipole tensor -(c2 R R^T - c1 I) between two
// of its sites (the same damping as T's same-molecule pairs, without the
// Ewald split: in a box the molecule's periodic images and the self terms
// are left out, which changes only how well M preconditions).  z = M^-1 r
// replaces z = alpha r; the stop test still measures alpha r.  Larger
// molecules, and a block whose Cholesky factorisation fails, keep alpha
// per site.
//
// Layout: the group of a molecule is kept by its leader, the member with
// the smallest polarizable index (n[leader] = group size, 0 for the other
// members); mem[4 i + k] lists the members in increasing order and
// inv[kPcPacked i + ...] holds the Cholesky factor L of M (M = L L^T),
// lower triangle packed row by row with 1 / L_jj on the diagonal, so that
// z = M^-1 r is a forward and a backward substitution.  A site of a larger
// molecule is a group of its own.  Every size has its own instantiation,
// so the factor stays in registers.
// The vector kernels run one thread per polarizable index; leaders work on
// their whole group (no other thread touches those sites), the rest only
// join the block reductions.
#include <hip/hip_runtime.h>

#include "common.h"
#include "pairmath.h"
#include "kernels.h"

namespace sibfa {

namespace {

__device__ __forceinline__ int tri(int i, int j) { return i * (i + 1) / 2 + j; }   // i >= j

__device__ __forceinline__ double thole_pair(const SysView& s, int i, int j) {
  return s.uniform_thole ? s.thole_a : fmin(s.pa[i], s.pa[j]);
}

// Members of pi's group, or 0 when pi is not the group's leader.
__device__ __forceinline__ int group_of(const SysView& s, int pi, int mem[kPcMax]) {
  const int cin = s.nc_ipol[pi];
  mem[0] = pi;
  if (cin + 1 > kPcMax) return 1;   // a larger molecule: alpha per site
  const int* row = s.nb_ipol + (size_t)pi * s.cap_ipol;
  for (int k = 0; k < cin; ++k) {
    const int j = row[k];
    if (j < pi) return 0;
    // insertion into the sorted tail
    int t = k + 1;
    while (t > 1 && mem[t - 1] > j) {
      mem[t] = mem[t - 1];
      --t;
    }
    mem[t] = j;
  }
  return cin + 1;
}

// y = M^-1 v = L^-T L^-1 v for a group of NG sites (3 NG unknowns).
template <int NG>
__device__ __forceinline__ void apply_inv(const double* L, const double v[3 * NG],
                                          double y[3 * NG]) {
  constexpr int N = 3 * NG;
  double w[N];
#pragma unroll
  for (int i = 0; i < N; ++i) {
    double a = v[i];
#pragma unroll
    for (int k = 0; k < i; ++k) a -= L[tri(i, k)] * w[k];
    w[i] = a * L[tri(i, i)];
  }
#pragma unroll
  for (int i = N - 1; i >= 0; --i) {
    double a = w[i];
#pragma unroll
    for (int k = i + 1; k < N; ++k) a -= L[tri(k, i)] * y[k];
    y[i] = a * L[tri(i, i)];
  }
}

__device__ __forceinline__ double alpha_norm2(const SysView& s, int m, const double r[3]) {
  const double* a = s.alpha + 6 * (size_t)m;
  const double z0 = a[0] * r[0] + a[1] * r[1] + a[2] * r[2];
  const double z1 = a[1] * r[0] + a[3] * r[1] + a[4] * r[2];
  const double z2 = a[2] * r[0] + a[4] * r[1] + a[5] * r[2];
  return z0 * z0 + z1 * z1 + z2 * z2;
}

}  // namespace

namespace {

// M of a group of NG sites (lower packed), then its Cholesky factor with
// 1 / L_jj on the diagonal; a block that is not positive definite is
// replaced by blockdiag(alpha^-1), which is.
template <int NG>
__device__ __forceinline__ void build_group(const SysView& s, const int mem[kPcMax], double* out) {
  constexpr int N = 3 * NG, P = N * (N + 1) / 2;
  double M[P];
  const int ia[6] = {0, 1, 1, 2, 2, 2}, ib[6] = {0, 0, 1, 0, 1, 2};
  const int ka[6] = {0, 1, 3, 2, 4, 5};   // packed (xx,xy,xz,yy,yz,zz) index of (ia, ib)
#pragma unroll
  for (int t = 0; t < P; ++t) M[t] = 0.0;
#pragma unroll
  for (int u = 0; u < NG; ++u) {
    const double* ai = s.ainv + 6 * (size_t)mem[u];
#pragma unroll
    for (int e = 0; e < 6; ++e) M[tri(3 * u + ia[e], 3 * u + ib[e])] = ai[ka[e]];
  }
#pragma unroll
  for (int u = 1; u < NG; ++u) {
    const double4 pu = s.pp[mem[u]];
#pragma unroll
    for (int v = 0; v < u; ++v) {
      const double4 pv = s.pp[mem[v]];
      double R[3] = {pu.x - pv.x, pu.y - pv.y, pu.z - pv.z};
      if (s.periodic)
#pragma unroll
        for (int a = 0; a < 3; ++a) R[a] = min_image<double>(R[a], s.box[a], s.ibox[a]);
      const double r2 = R[0] * R[0] + R[1] * R[1] + R[2] * R[2];
      const double rinv = rsqrt(r2), r = r2 * rinv, rinv2 = rinv * rinv;
      double c0[3], tp[5];
      bare_coeffs<double, 2>(rinv, rinv2, c0);
      thole_tp<double>(thole_pair(s, mem[u], mem[v]) * r2 * r * pu.w * pv.w, tp);
      const double c1 = (1.0 - tp[1]) * c0[1], c2 = (1.0 - tp[2]) * c0[2];
#pragma unroll
      for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b)
          M[tri(3 * u + a, 3 * v + b)] = (a == b ? c1 : 0.0) - c2 * R[a] * R[b];
    }
  }
  bool ok = true;
#pragma unroll
  for (int pass = 0; pass < 2; ++pass) {
    if (pass == 1) {
      if (ok) break;
      // fallback: alpha per site
#pragma unroll
      for (int t = 0; t < P; ++t) M[t] = 0.0;
#pragma unroll
      for (int u = 0; u < NG; ++u) {
        const double* ai = s.ainv + 6 * (size_t)mem[u];
#pragma unroll
        for (int e = 0; e < 6; ++e) M[tri(3 * u + ia[e], 3 * u + ib[e])] = ai[ka[e]];
      }
      ok = true;
    }
#pragma unroll
    for (int j = 0; j < N; ++j) {
      double d = M[tri(j, j)];
#pragma unroll
      for (int k = 0; k < j; ++k) d -= M[tri(j, k)] * M[tri(j, k)];
      ok = ok && d > 0.0;
      const double il = rsqrt(d > 0.0 ? d : 1.0);
      M[tri(j, j)] = il;   // 1 / L_jj
#pragma unroll
      for (int i = j + 1; i < N; ++i) {
        double v = M[tri(i, j)];
#pragma unroll
        for (int k = 0; k < j; ++k) v -= M[tri(i, k)] * M[tri(j, k)];
        M[tri(i, j)] = v * il;
      }
    }
  }
#pragma unroll
  for (int t = 0; t < P; ++t) out[t] = M[t];
}

}  // namespace

// The group of each leader and the Cholesky factor of its M.
__global__ __launch_bounds__(kBlock) void k_pc_build(SysView s, PcView pc) {
  const int pi = blockIdx.x * blockDim.x + threadIdx.x;
  if (pi >= s.npol) return;
  int mem[kPcMax];
  const int ng = group_of(s, pi, mem);
  pc.n[pi] = ng;
  if (ng == 0) return;
  for (int k = 0; k < kPcMax; ++k) pc.mem[kPcMax * (size_t)pi + k] = k < ng ? mem[k] : -1;
  double* out = pc.inv + kPcPacked * (size_t)pi;
  switch (ng) {
    case 1: build_group<1>(s, mem, out); break;
    case 2: build_group<2>(s, mem, out); break;
    case 3: build_group<3>(s, mem, out); break;
    default: build_group<4>(s, mem, out); break;
  }
}

namespace {

template <int NG>
__device__ __forceinline__ void precond_group(const PcView& pc, int pi, const double4* in,
                                              double4* out) {
  const int* mem = pc.mem + kPcMax * (size_t)pi;
  double v[3 * NG], y[3 * NG];
#pragma unroll
  for (int u = 0; u < NG; ++u) {
    const double4 a = in[mem[u]];
    v[3 * u] = a.x; v[3 * u + 1] = a.y; v[3 * u + 2] = a.z;
  }
  apply_inv<NG>(pc.inv + kPcPacked * (size_t)pi, v, y);
#pragma unroll
  for (int u = 0; u < NG; ++u) out[mem[u]] = make_double4(y[3 * u], y[3 * u + 1], y[3 * u + 2], 0.0);
}

// r = E0 - t (or r -= gamma q, x += gamma p) over the group, z = M^-1 r;
// partial sums r.z and |alpha r|^2.
template <int NG, bool INIT>
__device__ __forceinline__ void residual_group(const SysView& s, const PcView& pc, int pi,
                                               const double4* a_in, const double4* b_in,
                                               double gamma, double4* x, const double4* p,
                                               double4* r, double4* z, double4* pz, float4* pz32,
                                               double& rz, double& zz) {
  const int* mem = pc.mem + kPcMax * (size_t)pi;
  double rv[3 * NG], y[3 * NG];
#pragma unroll
  for (int u = 0; u < NG; ++u) {
    const int m = mem[u];
    double4 ro;
    if (INIT) {
      const double4 e = a_in[m], t = b_in[m];
      ro = make_double4(e.x - t.x, e.y - t.y, e.z - t.z, 0.0);
    } else {
      const double4 q = b_in[m], pv = p[m];
      ro = r[m];
      double4 xv = x[m];
      xv.x += gamma * pv.x; xv.y += gamma * pv.y; xv.z += gamma * pv.z;
      ro.x -= gamma * q.x; ro.y -= gamma * q.y; ro.z -= gamma * q.z;
      x[m] = xv;
    }
    r[m] = ro;
    rv[3 * u] = ro.x; rv[3 * u + 1] = ro.y; rv[3 * u + 2] = ro.z;
    zz += alpha_norm2(s, m, rv + 3 * u);
  }
  apply_inv<NG>(pc.inv + kPcPacked * (size_t)pi, rv, y);
#pragma unroll
  for (int u = 0; u < NG; ++u) {
    const int m = mem[u];
    const double4 zo = make_double4(y[3 * u], y[3 * u + 1], y[3 * u + 2], 0.0);
    z[m] = zo;
    if (pz) {
      pz[m] = zo;
      pz32[m] = make_float4((float)zo.x, (float)zo.y, (float)zo.z, 0.f);
    }
    rz += rv[3 * u] * y[3 * u] + rv[3 * u + 1] * y[3 * u + 1] + rv[3 * u + 2] * y[3 * u + 2];
  }
}

}  // namespace

__global__ __launch_bounds__(kBlock) void k_pc_apply(SysView s, PcView pc, const double4* in,
                                                     double4* out) {
  const int pi = blockIdx.x * blockDim.x + threadIdx.x;
  if (pi >= s.npol) return;
  switch (pc.n[pi]) {
    case 1: precond_group<1>(pc, pi, in, out); break;
    case 2: precond_group<2>(pc, pi, in, out); break;
    case 3: precond_group<3>(pc, pi, in, out); break;
    case 4: precond_group<4>(pc, pi, in, out); break;
    default: break;
  }
}

// r = E0 - t, z = M^-1 r (and p = z when p is given); r.z into rz_slot,
// |alpha r|^2 into S_ZZ.
__global__ __launch_bounds__(kBlock) void k_pc_init_residual(SysView s, PcView pc, Reduce red,
                                                             const double4* E0, const double4* t,
                                                             double4* r, double4* z, double4* p,
                                                             float4* p32, int rz_slot) {
  const int pi = blockIdx.x * blockDim.x + threadIdx.x;
  double rz = 0.0, zz = 0.0;
  if (pi < s.npol) {
    switch (pc.n[pi]) {
      case 1: residual_group<1, true>(s, pc, pi, E0, t, 0.0, nullptr, nullptr, r, z, p, p32, rz, zz); break;
      case 2: residual_group<2, true>(s, pc, pi, E0, t, 0.0, nullptr, nullptr, r, z, p, p32, rz, zz); break;
      case 3: residual_group<3, true>(s, pc, pi, E0, t, 0.0, nullptr, nullptr, r, z, p, p32, rz, zz); break;
      case 4: residual_group<4, true>(s, pc, pi, E0, t, 0.0, nullptr, nullptr, r, z, p, p32, rz, zz); break;
      default: break;
    }
  }
  block_partial(rz, red, rz_slot);
  block_partial(zz, red, S_ZZ);
}

// The PCG update with z = M^-1 r: x += gamma p, r -= gamma q over each group.
__global__ __launch_bounds__(kBlock) void k_pc_update(SysView s, PcView pc, Reduce red,
                                                      int rz_slot, int rz_next_slot, double4* x,
                                                      double4* r, double4* z, const double4* p,
                                                      const double4* q) {
  if (stopped(red.stop)) return;
  const int pi = blockIdx.x * blockDim.x + threadIdx.x;
  double rz = 0.0, zz = 0.0;
  const double rzt = slot_total(red, rz_slot);
  const double gamma = rzt == 0.0 ? 0.0 : rzt / slot_total(red, S_PQ);
  if (pi < s.npol) {
    switch (pc.n[pi]) {
      case 1: residual_group<1, false>(s, pc, pi, nullptr, q, gamma, x, p, r, z, nullptr, nullptr, rz, zz); break;
      case 2: residual_group<2, false>(s, pc, pi, nullptr, q, gamma, x, p, r, z, nullptr, nullptr, rz, zz); break;
      case 3: residual_group<3, false>(s, pc, pi, nullptr, q, gamma, x, p, r, z, nullptr, nullptr, rz, zz); break;
      case 4: residual_group<4, false>(s, pc, pi, nullptr, q, gamma, x, p, r, z, nullptr, nullptr, rz, zz); break;
      default: break;
    }
  }
  block_partial(rz, red, rz_next_slot);
  block_partial(zz, red, S_ZZ);
}

void launch_pc_build(const SysView& s, const PcView& pc, hipStream_t st) {
  if (s.npol <= 0) return;
  hipLaunchKernelGGL(k_pc_build, dim3((s.npol + kBlock - 1) / kBlock), dim3(kBlock), 0, st, s, pc);
}

void launch_pc_apply(const SysView& s, const PcView& pc, const double4* in, double4* out,
                     hipStream_t st) {
  if (s.npol <= 0) return;
  hipLaunchKernelGGL(k_pc_apply, dim3((s.npol + kBlock - 1) / kBlock), dim3(kBlock), 0, st, s, pc,
                     in, out);
}

void launch_pc_init_residual(const SysView& s, const PcView& pc, Reduce& red, const double4* E0,
                             const double4* t, double4* r, double4* z, double4* p, float4* p32,
                             int rz_slot, hipStream_t st) {
  const dim3 g((std::max(s.npol, 1) + kBlock - 1) / kBlock);
  hipLaunchKernelGGL(k_pc_init_residual, g, dim3(kBlock), 0, st, s, pc, red, E0, t, r, z, p, p32,
                     rz_slot);
  red.nparts[rz_slot] = (int)g.x;
  red.nparts[S_ZZ] = (int)g.x;
}

void launch_pc_update(const SysView& s, const PcView& pc, Reduce& red, int rz_slot,
                      int rz_next_slot, double4* x, double4* r, double4* z, const double4* p,
                      const double4* q, hipStream_t st) {
  const dim3 g((std::max(s.npol, 1) + kBlock - 1) / kBlock);
  hipLaunchKernelGGL(k_pc_update, g, dim3(kBlock), 0, st, s, pc, red, rz_slot, rz_next_slot, x, r,
                     z, p, q);
  red.nparts[rz_next_slot] = (int)g.x;
  red.nparts[S_ZZ] = (int)g.x;
}

}  // namespace sibfa
