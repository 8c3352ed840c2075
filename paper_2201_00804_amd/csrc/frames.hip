// Molecular local frames: multipoles and polarizabilities given in a frame
// attached to a molecule, rotated to the global frame at the current
// positions, and the forces of that rotation (the torques turned into
// forces on the frame's sites).
//
// Paper, Multipolar Electrostatics: SIBFA stores the distributed multipoles
// (and its anisotropic polarizabilities) in a molecular frame and rotates
// them at every geometry.  The frame used here (the paper names none) is
// built from three sites (o, a, b) of the molecule, for water O, H1, H2:
//   u = (r_a - r_o)/|..|, v = (r_b - r_o)/|..|, e_z = (u + v)/|u + v|,
//   e_x = unit(u - (u.e_z) e_z), e_y = e_z x e_x,  R = [e_x e_y e_z],
//   d = R d_loc, Theta = R Theta_loc R^T, alpha = R alpha_loc R^T.
//
// Forces.  At the converged (stationary) dipoles the energy depends on R
// only through the rotated quantities, with
//   dE/dR = sum_i G^d_i d_loc_i^T + 2 G^Theta_i R Theta_loc_i + 2 G^alpha_i R alpha_loc_i
//   G^d     = -E'          (E' the field that d_i feels: the permanent
//                           multipoles of the other sites, the induced
//                           dipoles (Thole-damped), the reciprocal sum and
//                           the Ewald self field of d_i + mu_i),
//   G^Theta = -1/3 grad E' (the same sources; self term -16 b^5/(45 sqrt pi) Theta),
//   G^alpha = -1/2 (alpha^-1 mu)(alpha^-1 mu)^T,
// so 2 G^alpha R alpha_loc = -(alpha^-1 mu)(R^T mu)^T.  dE/dR is pulled back
// through the frame construction in reverse (adjoint) order to dE/dr of the
// three frame sites.  The site fields E' and gradients come from the pair
// kernels and the reciprocal gather.
//
//  k_rotate       : per site, global d, Theta (and alpha) from the local ones.
//  k_frame_site   : per site, its term of dE/dR.
//  k_frame_group  : per frame, the sum over its sites in a fixed order, the
//                   adjoint pass, the forces on (o, a, b) and the virial
//                   of the frame (sum over its sites of F_k r_k^T, which
//                   with sum F_k = 0 is F_a A^T + F_b B^T).
//  k_frame_scatter: per site, the frame forces that act on it (fixed order)
//                   added to the caller-order forces.
#include <hip/hip_runtime.h>

#include "common.h"
#include "kernels.h"

namespace sibfa {

namespace {

__device__ __forceinline__ double dot3(const double a[3], const double b[3]) {
  return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}

__device__ __forceinline__ void cross3(const double a[3], const double b[3], double o[3]) {
  o[0] = a[1] * b[2] - a[2] * b[1];
  o[1] = a[2] * b[0] - a[0] * b[2];
  o[2] = a[0] * b[1] - a[1] * b[0];
}

// Everything the adjoint pass needs of one frame.
struct Basis {
  double A[3], B[3];        // r_a - r_o, r_b - r_o (minimum image)
  double nA, nB, ns, nw;    // norms of A, B, s = u + v, w
  double u[3], v[3], ex[3], ey[3], ez[3];
  double uz;                // u.e_z
};

__device__ void frame_basis(const FrameArgs& f, int o, int a, int b, Basis& K) {
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    double da = f.xyz[3 * (size_t)a + c] - f.xyz[3 * (size_t)o + c];
    double db = f.xyz[3 * (size_t)b + c] - f.xyz[3 * (size_t)o + c];
    if (f.periodic) {
      da = min_image<double>(da, f.box[c], f.ibox[c]);
      db = min_image<double>(db, f.box[c], f.ibox[c]);
    }
    K.A[c] = da;
    K.B[c] = db;
  }
  K.nA = sqrt(dot3(K.A, K.A));
  K.nB = sqrt(dot3(K.B, K.B));
  double s[3], w[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    K.u[c] = K.A[c] / K.nA;
    K.v[c] = K.B[c] / K.nB;
    s[c] = K.u[c] + K.v[c];
  }
  K.ns = sqrt(dot3(s, s));
#pragma unroll
  for (int c = 0; c < 3; ++c) K.ez[c] = s[c] / K.ns;
  K.uz = dot3(K.u, K.ez);
#pragma unroll
  for (int c = 0; c < 3; ++c) w[c] = K.u[c] - K.uz * K.ez[c];
  K.nw = sqrt(dot3(w, w));
#pragma unroll
  for (int c = 0; c < 3; ++c) K.ex[c] = w[c] / K.nw;
  cross3(K.ez, K.ex, K.ey);
}

// R[p][q]: row p (global axis), column q (local axis)
__device__ __forceinline__ void rot_matrix(const Basis& K, double R[3][3]) {
#pragma unroll
  for (int p = 0; p < 3; ++p) {
    R[p][0] = K.ex[p];
    R[p][1] = K.ey[p];
    R[p][2] = K.ez[p];
  }
}

__device__ __forceinline__ void sym6(const double* t, double M[3][3]) {
  M[0][0] = t[0]; M[0][1] = t[1]; M[0][2] = t[2];
  M[1][0] = t[1]; M[1][1] = t[3]; M[1][2] = t[4];
  M[2][0] = t[2]; M[2][1] = t[4]; M[2][2] = t[5];
}

// R M R^T stored xx xy xz yy yz zz
__device__ void rotate_sym(const double R[3][3], const double* loc, double* out) {
  double M[3][3], RM[3][3];
  sym6(loc, M);
#pragma unroll
  for (int p = 0; p < 3; ++p)
#pragma unroll
    for (int q = 0; q < 3; ++q) RM[p][q] = R[p][0] * M[0][q] + R[p][1] * M[1][q] + R[p][2] * M[2][q];
  const int ia[6] = {0, 0, 0, 1, 1, 2}, ib[6] = {0, 1, 2, 1, 2, 2};
#pragma unroll
  for (int k = 0; k < 6; ++k) {
    const int p = ia[k], q = ib[k];
    out[k] = RM[p][0] * R[q][0] + RM[p][1] * R[q][1] + RM[p][2] * R[q][2];
  }
}

// Adjoint of x/|x|: the gradient with respect to x from the one with
// respect to n = x/|x|: (g - (g.n) n) / |x|.
__device__ __forceinline__ void unit_adjoint(const double g[3], const double n[3], double norm,
                                             double out[3]) {
  const double gn = dot3(g, n);
#pragma unroll
  for (int c = 0; c < 3; ++c) out[c] = (g[c] - gn * n[c]) / norm;
}

}  // namespace

__global__ __launch_bounds__(kBlock) void k_rotate(FrameArgs f) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= f.n) return;
  const int o = f.frames[3 * (size_t)i];
  if (o < 0) {
    // no frame: the local values are the global ones
#pragma unroll
    for (int c = 0; c < 3; ++c) f.dip[3 * (size_t)i + c] = f.dloc[3 * (size_t)i + c];
#pragma unroll
    for (int k = 0; k < 6; ++k) f.quad[6 * (size_t)i + k] = f.qloc[6 * (size_t)i + k];
    if (f.aloc)
#pragma unroll
      for (int k = 0; k < 6; ++k) f.alpha[6 * (size_t)i + k] = f.aloc[6 * (size_t)i + k];
    return;
  }
  Basis K;
  frame_basis(f, o, f.frames[3 * (size_t)i + 1], f.frames[3 * (size_t)i + 2], K);
  double R[3][3];
  rot_matrix(K, R);
  const double* dl = f.dloc + 3 * (size_t)i;
#pragma unroll
  for (int p = 0; p < 3; ++p) f.dip[3 * (size_t)i + p] = R[p][0] * dl[0] + R[p][1] * dl[1] + R[p][2] * dl[2];
  rotate_sym(R, f.qloc + 6 * (size_t)i, f.quad + 6 * (size_t)i);
  if (f.aloc) rotate_sym(R, f.aloc + 6 * (size_t)i, f.alpha + 6 * (size_t)i);
}

__global__ __launch_bounds__(kBlock) void k_frame_site(FrameArgs f) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= f.n) return;
  const int o = f.frames[3 * (size_t)i];
  if (o < 0) return;
  Basis K;
  frame_basis(f, o, f.frames[3 * (size_t)i + 1], f.frames[3 * (size_t)i + 2], K);
  double R[3][3];
  rot_matrix(K, R);
  const int j = f.inv_perm[i];
  const double4 e = f.FS[j];
  const double Gd[3] = {-kCoulomb * e.x, -kCoulomb * e.y, -kCoulomb * e.z};
  double GT[3][3];
  sym6(f.GS + 6 * (size_t)j, GT);
  const double dl[3] = {f.dloc[3 * (size_t)i], f.dloc[3 * (size_t)i + 1], f.dloc[3 * (size_t)i + 2]};
  double TL[3][3];
  sym6(f.qloc + 6 * (size_t)i, TL);
  // GT R (GT scaled below)
  double GR[3][3];
#pragma unroll
  for (int p = 0; p < 3; ++p)
#pragma unroll
    for (int q = 0; q < 3; ++q) GR[p][q] = GT[p][0] * R[0][q] + GT[p][1] * R[1][q] + GT[p][2] * R[2][q];
  const double gts = -2.0 * kCoulomb / 3.0;
  double C[3][3];
#pragma unroll
  for (int p = 0; p < 3; ++p)
#pragma unroll
    for (int q = 0; q < 3; ++q)
      C[p][q] = Gd[p] * dl[q] +
                gts * (GR[p][0] * TL[0][q] + GR[p][1] * TL[1][q] + GR[p][2] * TL[2][q]);
  if (f.aloc) {
    const double* al = f.alpha + 6 * (size_t)i;
    const double4 m = f.mu_s[j];
    const double mu[3] = {m.x, m.y, m.z};
    if (mu[0] != 0.0 || mu[1] != 0.0 || mu[2] != 0.0) {
      // v = alpha^-1 mu from the adjugate (alpha symmetric positive definite)
      const double a00 = al[3] * al[5] - al[4] * al[4], a01 = al[2] * al[4] - al[1] * al[5];
      const double a02 = al[1] * al[4] - al[2] * al[3], a11 = al[0] * al[5] - al[2] * al[2];
      const double a12 = al[1] * al[2] - al[0] * al[4], a22 = al[0] * al[3] - al[1] * al[1];
      const double idet = 1.0 / (al[0] * a00 + al[1] * a01 + al[2] * a02);
      const double inv[3][3] = {{a00 * idet, a01 * idet, a02 * idet},
                                {a01 * idet, a11 * idet, a12 * idet},
                                {a02 * idet, a12 * idet, a22 * idet}};
      double v[3], rm[3];
#pragma unroll
      for (int p = 0; p < 3; ++p) v[p] = inv[p][0] * mu[0] + inv[p][1] * mu[1] + inv[p][2] * mu[2];
#pragma unroll
      for (int q = 0; q < 3; ++q) rm[q] = R[0][q] * mu[0] + R[1][q] * mu[1] + R[2][q] * mu[2];
#pragma unroll
      for (int p = 0; p < 3; ++p)
#pragma unroll
        for (int q = 0; q < 3; ++q) C[p][q] -= kCoulomb * v[p] * rm[q];
    }
  }
#pragma unroll
  for (int p = 0; p < 3; ++p)
#pragma unroll
    for (int q = 0; q < 3; ++q) f.C[9 * (size_t)i + 3 * p + q] = C[p][q];
}

__global__ __launch_bounds__(kBlock) void k_frame_group(FrameArgs f, Reduce red, int vir) {
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  double W[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
  if (g < f.ngroups) {
    double C[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    for (int k = f.gstart[g]; k < f.gstart[g + 1]; ++k) {
      const double* ci = f.C + 9 * (size_t)f.gsites[k];
#pragma unroll
      for (int t = 0; t < 9; ++t) C[t] += ci[t];
    }
    Basis K;
    frame_basis(f, f.gframe[3 * g], f.gframe[3 * g + 1], f.gframe[3 * g + 2], K);
    // dE/d e_x, e_y, e_z: the columns of dE/dR
    double gx[3], gy[3], gz[3];
#pragma unroll
    for (int p = 0; p < 3; ++p) {
      gx[p] = C[3 * p];
      gy[p] = C[3 * p + 1];
      gz[p] = C[3 * p + 2];
    }
    // e_y = e_z x e_x
    double t[3];
    cross3(K.ex, gy, t);
#pragma unroll
    for (int c = 0; c < 3; ++c) gz[c] += t[c];
    cross3(gy, K.ez, t);
#pragma unroll
    for (int c = 0; c < 3; ++c) gx[c] += t[c];
    // e_x = unit(w), w = u - (u.e_z) e_z
    double gw[3];
    unit_adjoint(gx, K.ex, K.nw, gw);
    const double gwz = dot3(gw, K.ez);
    double gu[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      gu[c] = gw[c] - gwz * K.ez[c];
      gz[c] += -gwz * K.u[c] - K.uz * gw[c];
    }
    // e_z = unit(s), s = u + v
    double gs[3];
    unit_adjoint(gz, K.ez, K.ns, gs);
    double gv[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      gu[c] += gs[c];
      gv[c] = gs[c];
    }
    // u = unit(A), v = unit(B); A = r_a - r_o, B = r_b - r_o
    double gA[3], gB[3];
    unit_adjoint(gu, K.u, K.nA, gA);
    unit_adjoint(gv, K.v, K.nB, gB);
    double* out = f.Fg + 9 * (size_t)g;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      out[c] = gA[c] + gB[c];    // o: F = -dE/dr_o
      out[3 + c] = -gA[c];       // a
      out[6 + c] = -gB[c];       // b
    }
    if (vir)
#pragma unroll
      for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) W[3 * a + b] = -gA[a] * K.A[b] - gB[a] * K.B[b];
  }
  if (vir)
#pragma unroll
    for (int k = 0; k < 9; ++k) block_partial(W[k], red, S_VRR + k);
}

__global__ __launch_bounds__(kBlock) void k_frame_scatter(FrameArgs f, double* forces) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= f.n) return;
  const int b = f.sstart[k], e = f.sstart[k + 1];
  if (b == e) return;
  double F[3] = {0.0, 0.0, 0.0};
  for (int r = b; r < e; ++r) {
    const double* fg = f.Fg + 3 * (size_t)f.sref[r];
#pragma unroll
    for (int c = 0; c < 3; ++c) F[c] += fg[c];
  }
#pragma unroll
  for (int c = 0; c < 3; ++c) forces[3 * (size_t)k + c] += F[c];
}

void launch_rotate(const FrameArgs& f, hipStream_t st) {
  hipLaunchKernelGGL(k_rotate, dim3((f.n + kBlock - 1) / kBlock), dim3(kBlock), 0, st, f);
}

void launch_frame_forces(const FrameArgs& f, Reduce& red, double* forces, bool virial,
                         hipStream_t st) {
  const dim3 b(kBlock);
  hipLaunchKernelGGL(k_frame_site, dim3((f.n + kBlock - 1) / kBlock), b, 0, st, f);
  const dim3 gg((std::max(f.ngroups, 1) + kBlock - 1) / kBlock);
  hipLaunchKernelGGL(k_frame_group, gg, b, 0, st, f, red, virial ? 1 : 0);
  if (virial)
    for (int k = 0; k < 9; ++k) red.nparts[S_VRR + k] = (int)gg.x;
  hipLaunchKernelGGL(k_frame_scatter, dim3((f.n + kBlock - 1) / kBlock), b, 0, st, f, forces);
}

}  // namespace sibfa
