// Vector kernels of the PCG driver and the reorderings between the caller's
// site order and the library's polarizable-site order.
//
// Vectors over polarizable sites are double4 (w unused).  The block
// preconditioner is z = alpha r with the 3x3 site polarizability
// (the inverse of T's diagonal blocks).  Dot products are reduced per block
// and finalised deterministically by the last block (block_reduce_to_slot).
#include <hip/hip_ext.h>

#include "common.h"
#include "kernels.h"

namespace sibfa {

__device__ __forceinline__ double3 amul(const double* a, double4 v) {
  return make_double3(a[0] * v.x + a[1] * v.y + a[2] * v.z,
                      a[1] * v.x + a[3] * v.y + a[4] * v.z,
                      a[2] * v.x + a[4] * v.y + a[5] * v.z);
}

__global__ __launch_bounds__(kBlock) void k_init_residual(SysView s, Reduce red, const double4* E0,
                                                          const double4* t, double4* r, double4* z,
                                                          double4* p, float4* p32, int rz_slot) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  double rz = 0.0, zz = 0.0;
  if (i < s.npol) {
    const double4 e = E0[i], tv = t[i];
    const double4 rv = make_double4(e.x - tv.x, e.y - tv.y, e.z - tv.z, 0.0);
    const double3 zv = amul(s.alpha + 6 * (size_t)i, rv);
    r[i] = rv;
    const double4 z4 = make_double4(zv.x, zv.y, zv.z, 0.0);
    z[i] = z4;
    if (p) {
      p[i] = z4;
      p32[i] = make_float4((float)zv.x, (float)zv.y, (float)zv.z, 0.f);
    }
    rz = rv.x * zv.x + rv.y * zv.y + rv.z * zv.z;
    zz = zv.x * zv.x + zv.y * zv.y + zv.z * zv.z;
  }
  block_partial(rz, red, rz_slot);
  block_partial(zz, red, S_ZZ);
}

__global__ __launch_bounds__(kBlock) void k_update(SysView s, Reduce red, int rz_slot,
                                                   int rz_next_slot, double4* x, double4* r,
                                                   double4* z, const double4* p, const double4* q) {
  if (stopped(red.stop)) return;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  double rz = 0.0, zz = 0.0;
  // r.z = 0 only for a zero residual (alpha is SPD): nothing to update
  const double rzt = slot_total(red, rz_slot);
  const double gamma = rzt == 0.0 ? 0.0 : rzt / slot_total(red, S_PQ);
  if (i < s.npol) {
    const double4 pv = p[i], qv = q[i];
    double4 xv = x[i], rv = r[i];
    xv.x += gamma * pv.x; xv.y += gamma * pv.y; xv.z += gamma * pv.z;
    rv.x -= gamma * qv.x; rv.y -= gamma * qv.y; rv.z -= gamma * qv.z;
    const double3 zv = amul(s.alpha + 6 * (size_t)i, rv);
    x[i] = xv;
    r[i] = rv;
    z[i] = make_double4(zv.x, zv.y, zv.z, 0.0);
    rz = rv.x * zv.x + rv.y * zv.y + rv.z * zv.z;
    zz = zv.x * zv.x + zv.y * zv.y + zv.z * zv.z;
  }
  block_partial(rz, red, rz_next_slot);
  block_partial(zz, red, S_ZZ);
}

// Stop test of the previous iteration (see k_check), made by every block
// on the same partial sums, so all agree; block 0 raises the flag.  With
// zz_ref (a device total the host has not read), the replacement threshold
// is zz_replace * *zz_ref.
__device__ __forceinline__ bool check_stop(const Reduce& red, int* flag, int iter, double zz_stop,
                                           double zz_replace, const double* zz_ref) {
  const double pq = slot_total(red, S_PQ);
  const double zz = slot_total(red, S_ZZ);
  const double zr = zz_ref ? zz_replace * *zz_ref : zz_replace;
  // a converged residual stops first (a zero residual also has p.Tp = 0)
  int reason = 0;
  if (zz <= zz_stop) reason = 1;
  else if (!(pq > 0.0)) reason = 2;
  else if (zz <= zr) reason = 3;
  if (reason && blockIdx.x == 0 && threadIdx.x == 0) {
    flag[1] = reason; flag[2] = iter; flag[0] = 1;
  }
  return reason != 0;
}

// p = z + beta p with beta = scalars[num] / scalars[den] (no grid to spread),
// after the stop test of the previous iteration when flag is given.
__global__ __launch_bounds__(kBlock) void k_direction(SysView s, Reduce red, int num, int den,
                                                      const double4* z, double4* p, float4* p32,
                                                      int* flag, int iter, double zz_stop,
                                                      double zz_replace, const double* zz_ref) {
  if (stopped(red.stop)) return;
  if (flag && check_stop(red, flag, iter, zz_stop, zz_replace, zz_ref)) return;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  // r.z = 0 only for a zero residual (then z = 0 and p = 0 as well)
  const double rz_old = slot_total(red, den);
  const double beta = rz_old == 0.0 ? 0.0 : slot_total(red, num) / rz_old;
  if (i >= s.npol) return;
  const double4 zv = z[i], pv = p[i];
  const double4 o = make_double4(zv.x + beta * pv.x, zv.y + beta * pv.y, zv.z + beta * pv.z, 0.0);
  p[i] = o;
  p32[i] = make_float4((float)o.x, (float)o.y, (float)o.z, 0.f);
}

// x += w z (the peek step of the truncated solver)
__global__ __launch_bounds__(kBlock) void k_axpy4(SysView s, double4* x, const double4* z,
                                                  double w) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= s.npol) return;
  const double4 zv = z[i];
  double4 xv = x[i];
  xv.x += w * zv.x; xv.y += w * zv.y; xv.z += w * zv.z;
  x[i] = xv;
}

__global__ __launch_bounds__(kBlock) void k_precond(SysView s, const double4* in, double4* out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= s.npol) return;
  const double3 v = amul(s.alpha + 6 * (size_t)i, in[i]);
  out[i] = make_double4(v.x, v.y, v.z, 0.0);
}

// a.b into slot and, when b2 is given, a.b2 into slot2 (one launch)
__global__ __launch_bounds__(kBlock) void k_dot(SysView s, Reduce red, const double4* a,
                                                const double4* b, int slot, const double4* b2,
                                                int slot2) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  double d = 0.0, d2 = 0.0;
  if (i < s.npol) {
    const double4 u = a[i], v = b[i];
    d = u.x * v.x + u.y * v.y + u.z * v.z;
    if (b2) {
      const double4 w = b2[i];
      d2 = u.x * w.x + u.y * w.y + u.z * w.z;
    }
  }
  block_partial(d, red, slot);
  if (b2) block_partial(d2, red, slot2);
}

__global__ __launch_bounds__(kBlock) void k_residual_norm(SysView s, Reduce red, const double4* E0,
                                                          const double4* t) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  double zz = 0.0;
  if (i < s.npol) {
    const double4 e = E0[i], tv = t[i];
    const double4 rv = make_double4(e.x - tv.x, e.y - tv.y, e.z - tv.z, 0.0);
    const double3 zv = amul(s.alpha + 6 * (size_t)i, rv);
    zz = zv.x * zv.x + zv.y * zv.y + zv.z * zv.z;
  }
  block_partial(zz, red, S_ZZ);
}

// Convergence test on the device after iteration `iter`: stop when
// z.z <= zz_stop (the tolerance), p.Tp <= 0 (not positive definite) or
// z.z <= zz_replace (time to replace the recurrence residual by the true
// one; a negative value never triggers).
// flag: [0] stop, [1] reason (1 converged, 2 not SPD, 3 replace),
// [2] iterations done.
__global__ __launch_bounds__(kBlock) void k_check(Reduce red, int* flag, double* zz_out, int iter,
                                                  double zz_stop, double zz_replace,
                                                  const double* zz_ref) {
  // z.z of the last update that ran (kernels after a stop leave the
  // partials alone), for the host's batch sizing
  const double zz = slot_total(red, S_ZZ);
  if (threadIdx.x == 0) *zz_out = zz;
  if (flag[0]) return;
  (void)check_stop(red, flag, iter, zz_stop, zz_replace, zz_ref);
}

__global__ void k_copy4(const double4* in, double4* out, float4* out32, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double4 v = in[i];
  out[i] = v;
  if (out32) out32[i] = make_float4((float)v.x, (float)v.y, (float)v.z, 0.f);
}

__global__ void k_mu_sites(SysView s, const double4* x, double4* mu, float4* mu32) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= s.n) return;
  const int pi = s.polidx[i];
  const double4 v = pi >= 0 ? x[pi] : make_double4(0.0, 0.0, 0.0, 0.0);
  mu[i] = v;
  mu32[i] = make_float4((float)v.x, (float)v.y, (float)v.z, 0.f);
}

__global__ void k_pol_to_caller(SysView s, const int* perm, const double4* v, double* out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= s.n) return;
  const int pi = s.polidx[i];
  const double4 a = pi >= 0 ? v[pi] : make_double4(0.0, 0.0, 0.0, 0.0);
  const size_t c = perm[i];
  out[3 * c] = a.x;
  out[3 * c + 1] = a.y;
  out[3 * c + 2] = a.z;
}

__global__ void k_caller_to_pol(SysView s, const int* perm, const double* in, double4* v,
                                float4* v32) {
  const int pi = blockIdx.x * blockDim.x + threadIdx.x;
  if (pi >= s.npol) return;
  const size_t c = perm[s.polsite[pi]];
  const double4 a = make_double4(in[3 * c], in[3 * c + 1], in[3 * c + 2], 0.0);
  v[pi] = a;
  if (v32) v32[pi] = make_float4((float)a.x, (float)a.y, (float)a.z, 0.f);
}

// out = a x + b y over the polarizable sites (y may be NULL: out = a x).
__global__ __launch_bounds__(kBlock) void k_lincomb4(SysView s, double4* out, double a,
                                                     const double4* x, double b,
                                                     const double4* y) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= s.npol) return;
  const double4 u = x[i];
  double4 o = make_double4(a * u.x, a * u.y, a * u.z, 0.0);
  if (y) {
    const double4 v = y[i];
    o.x += b * v.x; o.y += b * v.y; o.z += b * v.z;
  }
  out[i] = o;
}

// y += a x over count doubles.
__global__ __launch_bounds__(kBlock) void k_axpy_d(size_t count, double a, const double* x,
                                                   double* y) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) y[i] += a * x[i];
}

// Records with the multipoles removed (positions and Thole widths kept).
__global__ __launch_bounds__(kBlock) void k_zero_records(SysView s, double4* sp0, double4* sd0,
                                                         double4* sth0, double2* sth20) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= s.n) return;
  const double4 p = s.sp[i];
  sp0[i] = make_double4(p.x, p.y, p.z, 0.0);
  sd0[i] = make_double4(0.0, 0.0, 0.0, s.sd[i].w);
  sth0[i] = make_double4(0.0, 0.0, 0.0, 0.0);
  sth20[i] = make_double2(0.0, 0.0);
}

// Extrapolated guess: v = sum_j coef_j h_j over the k newest history
// entries (caller order, 3 n doubles each).
__global__ void k_predict(SysView s, const int* perm, const double* hist, size_t stride,
                          PredArgs pa, double4* v, float4* v32) {
  const int pi = blockIdx.x * blockDim.x + threadIdx.x;
  if (pi >= s.npol) return;
  const size_t c = perm[s.polsite[pi]];
  double a[3] = {0.0, 0.0, 0.0};
  for (int j = 0; j < pa.k; ++j) {
    const double* h = hist + (size_t)pa.slot[j] * stride + 3 * c;
#pragma unroll
    for (int d = 0; d < 3; ++d) a[d] += pa.coef[j] * h[d];
  }
  v[pi] = make_double4(a[0], a[1], a[2], 0.0);
  if (v32) v32[pi] = make_float4((float)a[0], (float)a[1], (float)a[2], 0.f);
}

__global__ void k_forces_out(int n, const int* perm, const double4* F, double* out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double4 f = F[i];
  const size_t c = perm[i];
  out[3 * c] = kCoulomb * f.x;
  out[3 * c + 1] = kCoulomb * f.y;
  out[3 * c + 2] = kCoulomb * f.z;
}

__global__ void k_counts_out(int n, const int* perm, const int* counts, int* out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[perm[i]] = counts[i];
}

static dim3 grid_for(int n) { return dim3(n > 0 ? (n + kBlock - 1) / kBlock : 1); }

void launch_init_residual(const SysView& s, Reduce& red, const double4* E0, const double4* t,
                          double4* r, double4* z, double4* p, float4* p32, int rz_slot,
                          hipStream_t st) {
  red.nparts[rz_slot] = red.nparts[S_ZZ] = (int)grid_for(s.npol).x;
  hipLaunchKernelGGL(k_init_residual, grid_for(s.npol), dim3(kBlock), 0, st, s, red, E0, t, r, z,
                     p, p32, rz_slot);
}
void launch_update(const SysView& s, Reduce& red, int rz_slot, int rz_next_slot, double4* x,
                   double4* r, double4* z, const double4* p, const double4* q, hipStream_t st) {
  // reads the totals of rz_slot and S_PQ (launched with the current counts)
  hipLaunchKernelGGL(k_update, grid_for(s.npol), dim3(kBlock), 0, st, s, red, rz_slot,
                     rz_next_slot, x, r, z, p, q);
  red.nparts[rz_next_slot] = red.nparts[S_ZZ] = (int)grid_for(s.npol).x;
}
void launch_direction(const SysView& s, const Reduce& red, int num, int den, const double4* z,
                      double4* p, float4* p32, int* flag, int iter, double zz_stop,
                      double zz_replace, const double* zz_ref, hipStream_t st, hipEvent_t done) {
  if (done)   // the kernel's own completion records the event: no marker packet
    hipExtLaunchKernelGGL(k_direction, grid_for(s.npol), dim3(kBlock), 0, st, nullptr, done, 0, s,
                          red, num, den, z, p, p32, flag, iter, zz_stop, zz_replace, zz_ref);
  else
    hipLaunchKernelGGL(k_direction, grid_for(s.npol), dim3(kBlock), 0, st, s, red, num, den, z, p,
                       p32, flag, iter, zz_stop, zz_replace, zz_ref);
}
// One block per slot: the slot's partials summed in a fixed order.
__global__ __launch_bounds__(kBlock) void k_slot_totals(Reduce red, SlotList sl, double* out) {
  const int k = blockIdx.x;
  const int slot = sl.slot[k], n = sl.nparts[k];
  const double* p = red.partials + (size_t)slot * red.max_blocks;
  double v = 0.0;
  for (int b = threadIdx.x; b < n; b += blockDim.x) v += p[b];
  __shared__ double sh[kBlock / 64];
  v = wave_sum(v);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) t += sh[w];
    out[k] = t;
  }
}

void launch_slot_totals(const Reduce& red, const SlotList& sl, double* out, hipStream_t st) {
  if (sl.n > 0)
    hipLaunchKernelGGL(k_slot_totals, dim3(sl.n), dim3(kBlock), 0, st, red, sl, out);
}

// flag (zeroed by the caller) becomes nonzero if any of v[0..n) is NaN or Inf.
__global__ void k_nonfinite(const double* v, size_t n, int* flag) {
  bool bad = false;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x)
    bad = bad || !isfinite(v[i]);
  if (__any(bad) && (threadIdx.x & 63) == 0) atomicOr(flag, 1);
}

void launch_nonfinite(const double* v, size_t n, int* flag, hipStream_t st) {
  size_t blocks = (n + kBlock - 1) / kBlock;
  if (blocks > 1024) blocks = 1024;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(k_nonfinite, dim3((unsigned)blocks), dim3(kBlock), 0, st, v, n, flag);
}

void launch_check(const Reduce& red, int* flag, double* zz_out, int iter, double zz_stop,
                  double zz_replace, const double* zz_ref, hipStream_t st) {
  hipLaunchKernelGGL(k_check, dim3(1), dim3(kBlock), 0, st, red, flag, zz_out, iter, zz_stop,
                     zz_replace, zz_ref);
}
void launch_axpy4(const SysView& s, double4* x, const double4* z, double w, hipStream_t st) {
  hipLaunchKernelGGL(k_axpy4, grid_for(s.npol), dim3(kBlock), 0, st, s, x, z, w);
}
void launch_precond(const SysView& s, const double4* in, double4* out, hipStream_t st) {
  hipLaunchKernelGGL(k_precond, grid_for(s.npol), dim3(kBlock), 0, st, s, in, out);
}
void launch_dot(const SysView& s, Reduce& red, const double4* a, const double4* b, int slot,
                hipStream_t st, const double4* b2, int slot2) {
  red.nparts[slot] = (int)grid_for(s.npol).x;
  if (b2) red.nparts[slot2] = (int)grid_for(s.npol).x;
  hipLaunchKernelGGL(k_dot, grid_for(s.npol), dim3(kBlock), 0, st, s, red, a, b, slot, b2, slot2);
}
void launch_residual_norm(const SysView& s, Reduce& red, const double4* E0, const double4* t,
                          hipStream_t st) {
  red.nparts[S_ZZ] = (int)grid_for(s.npol).x;
  hipLaunchKernelGGL(k_residual_norm, grid_for(s.npol), dim3(kBlock), 0, st, s, red, E0, t);
}
void launch_copy4(const double4* in, double4* out, float4* out32, int n, hipStream_t st) {
  if (n > 0) hipLaunchKernelGGL(k_copy4, grid_for(n), dim3(kBlock), 0, st, in, out, out32, n);
}
void launch_mu_sites(const SysView& s, const double4* x, double4* mu, float4* mu32, hipStream_t st) {
  hipLaunchKernelGGL(k_mu_sites, grid_for(s.n), dim3(kBlock), 0, st, s, x, mu, mu32);
}
void launch_pol_to_caller(const SysView& s, const int* perm, const double4* v, double* out,
                          hipStream_t st) {
  hipLaunchKernelGGL(k_pol_to_caller, grid_for(s.n), dim3(kBlock), 0, st, s, perm, v, out);
}
void launch_caller_to_pol(const SysView& s, const int* perm, const double* in, double4* v,
                          float4* v32, hipStream_t st) {
  if (s.npol > 0)
    hipLaunchKernelGGL(k_caller_to_pol, grid_for(s.npol), dim3(kBlock), 0, st, s, perm, in, v, v32);
}
void launch_lincomb4(const SysView& s, double4* out, double a, const double4* x, double b,
                     const double4* y, hipStream_t st) {
  if (s.npol > 0)
    hipLaunchKernelGGL(k_lincomb4, grid_for(s.npol), dim3(kBlock), 0, st, s, out, a, x, b, y);
}
void launch_axpy_d(size_t count, double a, const double* x, double* y, hipStream_t st) {
  if (count > 0)
    hipLaunchKernelGGL(k_axpy_d, dim3((unsigned)((count + kBlock - 1) / kBlock)), dim3(kBlock), 0,
                       st, count, a, x, y);
}
void launch_zero_records(const SysView& s, double4* sp0, double4* sd0, double4* sth0,
                         double2* sth20, hipStream_t st) {
  hipLaunchKernelGGL(k_zero_records, grid_for(s.n), dim3(kBlock), 0, st, s, sp0, sd0, sth0, sth20);
}
void launch_predict(const SysView& s, const int* perm, const double* hist, size_t stride,
                    const PredArgs& pa, double4* v, float4* v32, hipStream_t st) {
  if (s.npol > 0)
    hipLaunchKernelGGL(k_predict, grid_for(s.npol), dim3(kBlock), 0, st, s, perm, hist, stride, pa,
                       v, v32);
}
void launch_forces_out(int n, const int* perm, const double4* F, double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_forces_out, grid_for(n), dim3(kBlock), 0, st, n, perm, F, out);
}

void launch_counts_out(int n, const int* perm, const int* counts, int* out, hipStream_t st) {
  hipLaunchKernelGGL(k_counts_out, grid_for(n), dim3(kBlock), 0, st, n, perm, counts, out);
}

}  // namespace sibfa
