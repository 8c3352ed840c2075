// Molecular dynamics driver kernels: the Beeman integrator (Computational
// Details: Beeman, 1 fs steps, the polarization solved at every step), with
// midpoint virtual sites and harmonic bonds that hold the molecules
// together.  The paper's bonded and short-range terms need parameters that
// are not available, so the bonds are a stand-in that keeps a trajectory
// well defined; the step exercises the whole polarization path.
//
// Beeman, for the atoms (mass > 0):
//   x(t+dt) = x + v dt + (4 a - a_prev) dt^2 / 6
//   v(t+dt) = v + (2 a(t+dt) + 5 a - a_prev) dt / 6
// Virtual sites sit at the midpoint of two atoms (minimum image), carry no
// mass, and hand half of their force to each parent.  A soft repulsion
// eps ((rho_i + rho_j)/r)^12 between sites of different molecules stands in
// for the short-range terms, which keeps molecules from falling into each
// other under the bare multipole attraction (virtual sites take part: their
// multipoles would otherwise meet other sites unopposed).  Units: A, fs,
// g/mol, kcal/mol: a = F / m * kAccel.
#include <hip/hip_runtime.h>

#include "common.h"
#include "kernels.h"

namespace sibfa {

namespace {

constexpr double kAccel = 4.184e-4;   // (kcal/mol/A) / (g/mol) in A/fs^2

__device__ __forceinline__ double wrap(const MdArgs& m, double d, int a) {
  return m.periodic ? min_image<double>(d, m.box[a], m.ibox[a]) : d;
}

}  // namespace

// Positions of the atoms at t + dt.
__global__ __launch_bounds__(kBlock) void k_md_positions(MdArgs m, double dt) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= m.n || !(m.mass[i] > 0.0)) return;
  const double h = dt * dt / 6.0;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const size_t k = 3 * (size_t)i + a;
    m.xyz[k] += m.vel[k] * dt + (4.0 * m.acc[k] - m.accp[k]) * h;
  }
}

// Virtual sites at the midpoint of their parents.
__global__ __launch_bounds__(kBlock) void k_md_vsites(MdArgs m) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= m.n) return;
  const int p = m.vpar[2 * (size_t)i], q = m.vpar[2 * (size_t)i + 1];
  if (p < 0) return;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const double xp = m.xyz[3 * (size_t)p + a];
    m.xyz[3 * (size_t)i + a] = xp + 0.5 * wrap(m, m.xyz[3 * (size_t)q + a] - xp, a);
  }
}

// Total force on each atom (its own, half of each virtual site it
// parents, its bonds), the new acceleration and, when dt > 0, the Beeman
// velocity update, scaled by keep = 1 - friction (keep = 1: plain Beeman;
// below 1 a damped relaxation); kinetic and bond energy partials (each
// bond counted half at each end).  dt = 0: the start of a run (a_prev = a).
__global__ __launch_bounds__(kBlock) void k_md_finish(MdArgs m, Reduce red, double dt,
                                                      double keep) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  double ek = 0.0, eb = 0.0;
  if (dt == 0.0 && i < m.n && !(m.mass[i] > 0.0))   // virtual sites do not move by themselves
#pragma unroll
    for (int a = 0; a < 3; ++a) m.vel[3 * (size_t)i + a] = 0.0;
  if (i < m.n && m.mass[i] > 0.0) {
    double F[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) F[a] = m.force[3 * (size_t)i + a];
    for (int r = m.vstart[i]; r < m.vstart[i + 1]; ++r) {
      const int v = m.vref[r];
#pragma unroll
      for (int a = 0; a < 3; ++a) F[a] += 0.5 * m.force[3 * (size_t)v + a];
    }
    for (int r = m.bstart[i]; r < m.bstart[i + 1]; ++r) {
      const int b = m.bref[r];
      const int j = m.bonds[2 * (size_t)b] == i ? m.bonds[2 * (size_t)b + 1] : m.bonds[2 * (size_t)b];
      double d[3];
#pragma unroll
      for (int a = 0; a < 3; ++a) d[a] = wrap(m, m.xyz[3 * (size_t)i + a] - m.xyz[3 * (size_t)j + a], a);
      const double len = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
      const double ext = len - m.bond_r0[b];
      const double fk = -m.bond_k[b] * ext / len;
#pragma unroll
      for (int a = 0; a < 3; ++a) F[a] += fk * d[a];
      eb += 0.25 * m.bond_k[b] * ext * ext;
    }
    const double s = kAccel / m.mass[i];
    double v2 = 0.0;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const size_t k = 3 * (size_t)i + a;
      const double an = F[a] * s;
      if (dt > 0.0) {
        m.vel[k] = keep * (m.vel[k] + (2.0 * an + 5.0 * m.acc[k] - m.accp[k]) * dt / 6.0);
        m.accp[k] = m.acc[k];
      } else {
        m.accp[k] = an;
      }
      m.acc[k] = an;
      v2 += m.vel[k] * m.vel[k];
    }
    ek = 0.5 * m.mass[i] * v2 / kAccel;
  }
  block_partial(ek, red, S_EKIN);
  block_partial(eb, red, S_EBOND);
}

// Stand-in short-range repulsion between sites of different molecules
// that both have a positive radius, within the cutoff:
// eps ((rho_i + rho_j) / r)^12, over the intermolecular neighbour lists
// (sorted order; each site sums its own pairs, G lanes per site).  Adds to
// the caller-order forces (a virtual site's share reaches its parents in
// k_md_finish); energy partials count each ordered pair half.
template <int G>
__global__ __launch_bounds__(kBlock) void k_md_repulsion(SysView s, MdArgs m, Reduce red,
                                                         const int* perm) {
  const int sub = threadIdx.x % G;
  const int i = blockIdx.x * (kBlock / G) + threadIdx.x / G;
  double F[3] = {0.0, 0.0, 0.0}, U = 0.0;
  int ci = -1;
  if (i < s.n) {
    ci = perm[i];
    const double ri = m.rep_rho[ci];
    if (ri > 0.0) {
      const double4 pi = s.sp[i];
      const int* row = s.nb_all + (size_t)i * s.cap_all;
      const int nn = s.nc_near[i], nt = s.nc_all[i];
      for (int k = sub; k < nt; k += G) {
        const int j = k < nn ? row[k] : row[s.cap_all - 1 - (k - nn)];
        const double rj = m.rep_rho[perm[j]];
        if (!(rj > 0.0)) continue;
        const double sig = ri + rj;
        const double4 pj = s.sp[j];
        double d[3] = {pi.x - pj.x, pi.y - pj.y, pi.z - pj.z};
#pragma unroll
        for (int a = 0; a < 3; ++a) d[a] = wrap(m, d[a], a);
        const double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
        const double x2 = sig * sig / r2, x6 = x2 * x2 * x2, e = m.rep_eps * x6 * x6;
        U += 0.5 * e;
        const double f = 12.0 * e / r2;
#pragma unroll
        for (int a = 0; a < 3; ++a) F[a] += f * d[a];
      }
    }
  }
#pragma unroll
  for (int a = 0; a < 3; ++a) F[a] = group_sum<G>(F[a]);
  if (sub == 0 && ci >= 0)
#pragma unroll
    for (int a = 0; a < 3; ++a) m.rep_force[3 * (size_t)ci + a] += F[a];
  block_partial(U, red, S_EREP);
}

void launch_md_repulsion(const SysView& s, const MdArgs& m, Reduce& red, const int* perm,
                         hipStream_t st) {
  constexpr int G = 16;
  const dim3 g((s.n + kBlock / G - 1) / (kBlock / G));
  hipLaunchKernelGGL(k_md_repulsion<G>, g, dim3(kBlock), 0, st, s, m, red, perm);
  red.nparts[S_EREP] = (int)g.x;
}

void launch_md_positions(const MdArgs& m, double dt, hipStream_t st) {
  const dim3 g((m.n + kBlock - 1) / kBlock), b(kBlock);
  hipLaunchKernelGGL(k_md_positions, g, b, 0, st, m, dt);
  hipLaunchKernelGGL(k_md_vsites, g, b, 0, st, m);
}

void launch_md_vsites(const MdArgs& m, hipStream_t st) {
  hipLaunchKernelGGL(k_md_vsites, dim3((m.n + kBlock - 1) / kBlock), dim3(kBlock), 0, st, m);
}

void launch_md_finish(const MdArgs& m, Reduce& red, double dt, double friction,
                      hipStream_t st) {
  const dim3 g((m.n + kBlock - 1) / kBlock);
  hipLaunchKernelGGL(k_md_finish, g, dim3(kBlock), 0, st, m, red, dt, 1.0 - friction);
  red.nparts[S_EKIN] = (int)g.x;
  red.nparts[S_EBOND] = (int)g.x;
}

}  // namespace sibfa
