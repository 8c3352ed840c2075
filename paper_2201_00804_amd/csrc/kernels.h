// Launchers of the compute kernels (pair.hip, pme.hip, fft.hip, vec.hip).
#pragma once
#include "common.h"

namespace sibfa {

// pair.hip
void launch_perm(const SysView& s, const Reduce& red, double4* E0, bool mixed, hipStream_t st);
void launch_matvec(const SysView& s, const PmeView& pm, const Reduce& red, const double4* p,
                   const float4* p32, double4* out, int dot_slot, bool mixed, hipStream_t st);
void launch_force(const SysView& s, const double4* mu, const float4* mu32, double4* F, bool mixed,
                  hipStream_t st);

// pme.hip
// Spread of the permanent multipoles (with the induced dipoles added to d
// when mu != NULL, sorted-site indexing) onto the real grid.
void launch_spread_mult(const SysView& s, const PmeView& pm, const double4* mu, bool mixed,
                        hipStream_t st);
// Spread of polarizable-site dipoles.  With upd != 0 first sets
// p = z + beta p, beta = scalars[num] / scalars[den], and writes p (and its
// FP32 copy).
struct DirUpdate {
  int upd;
  int num, den;          // reduction slots
  const double4* z;
  double4* p;
  float4* p32;
};
void launch_spread_dip(const SysView& s, const PmeView& pm, const Reduce& red, DirUpdate du,
                       bool mixed, hipStream_t st);
// E0[pi] += -grad phi at polarizable sites.
void launch_gather_field(const SysView& s, const PmeView& pm, double4* E0, bool mixed,
                         hipStream_t st);
// Reciprocal forces of the combined density added to the real-space forces;
// scaled by the Coulomb constant and written in caller order.
void launch_gather_force(const SysView& s, const PmeView& pm, const double4* mu,
                         const double4* Freal, const int* perm, double* out, bool mixed,
                         hipStream_t st);

// fft.hip: full convolution phi = IFFT(G * FFT(Q)) with E_rec into S_EREC;
// Q is zeroed on the way.
void launch_convolution(const PmeView& pm, const Reduce& red, bool mixed, hipStream_t st);

// vec.hip
// PCG kernels over polarizable sites (double4 vectors, w unused).
void launch_init_residual(const SysView& s, const Reduce& red, const double4* E0,
                          const double4* t, double4* r, double4* z, double4* p, float4* p32,
                          int rz_slot, hipStream_t st);
void launch_update(const SysView& s, const Reduce& red, int rz_slot, int rz_next_slot,
                   double4* x, double4* r, double4* z, const double4* p, const double4* q,
                   hipStream_t st);
void launch_direction(const SysView& s, const Reduce& red, int num, int den, const double4* z,
                      double4* p, float4* p32, hipStream_t st);
void launch_precond(const SysView& s, const double4* in, double4* out, hipStream_t st);
void launch_dot(const SysView& s, const Reduce& red, const double4* a, const double4* b, int slot,
                hipStream_t st);
void launch_residual_norm(const SysView& s, const Reduce& red, const double4* E0, const double4* t,
                          hipStream_t st);
void launch_copy4(const double4* in, double4* out, float4* out32, int n, hipStream_t st);
// sorted-site mu (zero at non-polarizable sites) from polarizable-index x
void launch_mu_sites(const SysView& s, const double4* x, double4* mu, float4* mu32, hipStream_t st);
// caller order [n][3] <-> polarizable index vectors
void launch_pol_to_caller(const SysView& s, const int* perm, const double4* v, double* out,
                          hipStream_t st);
void launch_caller_to_pol(const SysView& s, const int* perm, const double* in, double4* v,
                          float4* v32, hipStream_t st);
// Coulomb-scaled forces to caller order (no reciprocal part)
void launch_forces_out(int n, const int* perm, const double4* F, double* out, hipStream_t st);
// neighbour counts to caller order
void launch_counts_out(int n, const int* perm, const int* counts, int* out, hipStream_t st);

}  // namespace sibfa
