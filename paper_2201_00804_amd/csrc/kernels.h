// Launchers of the compute kernels (pair.hip, pme.hip, fft.hip, vec.hip).
#pragma once
#include "common.h"

namespace sibfa {

// pair.hip
void launch_perm(const SysView& s, Reduce& red, double4* E0, bool mixed, hipStream_t st);
// T p in two kernels: real space (reads the cached pair coefficients, which
// must be current) and, for periodic systems, the PME field gather with
// p.Tp.  The dot product's partials come from the last of the two.
// done: recorded when the kernel completes; t0, t1 (both or neither): the
// kernel's own dispatch events, for timing
void launch_matvec_real(const SysView& s, Reduce& red, const double4* p, const float4* p32,
                        double4* out, int dot_slot, bool mixed, hipStream_t st,
                        hipEvent_t done = nullptr, hipEvent_t t0 = nullptr,
                        hipEvent_t t1 = nullptr);
void launch_matvec_recip(const SysView& s, const PmeView& pm, Reduce& red, const double4* p,
                         double4* out, int dot_slot, bool mixed, hipStream_t st);
// cache the pol-list pair coefficients: FP64 into out, or FP32 into out32
// when out is NULL; the same-molecule pol list always in FP64 into out_in
void launch_pol_coef(const SysView& s, double2* out, float2* out32, double2* out_in,
                     hipStream_t st);
// virial: also the real-space virial partials (slots S_VRI, S_VRF).
// FS, GS (may be NULL; local frames): also the field and field gradient
// (xx xy xz yy yz zz) at every site (sorted order) from the real-space
// pairs its permanent multipoles take part in -- the other molecules'
// multipoles, the induced dipoles (damped where the pair is) and, for
// periodic systems, the excluded same-molecule part.  Overwrites FS, GS.
void launch_force(const SysView& s, Reduce& red, const double4* mu, const float4* mu32, double4* F,
                  bool mixed, bool virial, hipStream_t st, double4* FS = nullptr,
                  double* GS = nullptr);

// pme.hip
// Spread of the permanent multipoles (with the induced dipoles added to d
// when mu != NULL, sorted-site indexing) onto the real grid.
void launch_spread_mult(const SysView& s, const PmeView& pm, const double4* mu, bool mixed,
                        hipStream_t st);
// Home-brick binning of the sites for the spreading kernels (counts must be
// zeroed; pol = 1 bins polarizable sites, 0 all sites).
void launch_brick_bin(const SysView& s, const PmeView& pm, int pol, int* brick_of, int* counts,
                      hipStream_t st);
// Real grid Q from the spreading tiles (used by the multi-pass convolution).
void launch_spread_fold(const PmeView& pm, bool mixed, hipStream_t st);
// Spread of the polarizable-site dipoles p (polarizable order).
void launch_spread_dip(const SysView& s, const PmeView& pm, const double4* p, bool mixed,
                       hipStream_t st);
// E0[pi] += -grad phi at polarizable sites.
void launch_gather_field(const SysView& s, const PmeView& pm, double4* E0, bool mixed,
                         hipStream_t st);
// Reciprocal forces of the combined density added to the real-space forces;
// scaled by the Coulomb constant and written in caller order.
// virial: also the site (amplitude) terms of the reciprocal virial (slots
// S_VRG).
// FS, GS (may be NULL): the reciprocal field and field gradient at every
// site plus (self) the Ewald self terms of d + mu and Theta are added to
// them.
void launch_gather_force(const SysView& s, const PmeView& pm, Reduce& red, const double4* mu,
                         const double4* Freal, const int* perm, double* out, bool mixed,
                         bool virial, hipStream_t st, double4* FS = nullptr,
                         double* GS = nullptr, bool self = true);

// fft.hip: full convolution phi = IFFT(G * FFT(Q)) with E_rec partials in
// the slot pm.erec_slot; virial: also the m-space sum of the reciprocal
// virial (slots S_VRK).
void launch_convolution(const PmeView& pm, Reduce& red, bool mixed, hipStream_t st,
                        bool virial = false);

// vec.hip
// PCG kernels over polarizable sites (double4 vectors, w unused).
// r = E0 - t, z = alpha r, p = z (skipped when p is null: the residual of a
// running sequence is replaced), r.z into rz_slot and z.z into S_ZZ.
void launch_init_residual(const SysView& s, Reduce& red, const double4* E0,
                          const double4* t, double4* r, double4* z, double4* p, float4* p32,
                          int rz_slot, hipStream_t st);
void launch_update(const SysView& s, Reduce& red, int rz_slot, int rz_next_slot,
                   double4* x, double4* r, double4* z, const double4* p, const double4* q,
                   hipStream_t st);
// p = z + beta p; with a flag, first the stop test of iteration `iter`
// (that of k_check), and no update when it stops.  zz_ref (may be NULL):
// the replacement threshold is zz_replace * *zz_ref.  done (may be NULL):
// recorded by the kernel's completion.
void launch_direction(const SysView& s, const Reduce& red, int num, int den, const double4* z,
                      double4* p, float4* p32, int* flag, int iter, double zz_stop,
                      double zz_replace, const double* zz_ref, hipStream_t st,
                      hipEvent_t done = nullptr);
void launch_nonfinite(const double* v, size_t n, int* flag, hipStream_t st);
// Totals of up to 8 reduction slots (one block each, fixed order) into out.
struct SlotList {
  int n;
  int slot[8];
  int nparts[8];
};
void launch_slot_totals(const Reduce& red, const SlotList& sl, double* out, hipStream_t st);
// device-side convergence test (see k_check)
void launch_check(const Reduce& red, int* flag, double* zz_out, int iter, double zz_stop,
                  double zz_replace, const double* zz_ref, hipStream_t st);
void launch_precond(const SysView& s, const double4* in, double4* out, hipStream_t st);

// precond.hip: molecular block preconditioner (polarizable order).
constexpr int kPcMax = 4;                               // sites per block
constexpr int kPcPacked = 3 * kPcMax * (3 * kPcMax + 1) / 2;   // packed M^-1
struct PcView {
  int* n;         // [npol] group size at the group's leader, 0 elsewhere
  int* mem;       // [npol][kPcMax] members of the leader's group (increasing)
  double* inv;    // [npol][kPcPacked] M^-1 of the leader's group, lower packed
};
// M and M^-1 for the current positions and polarizabilities (after the
// same-molecule polarizable lists)
void launch_pc_build(const SysView& s, const PcView& pc, hipStream_t st);
// out = M^-1 in
void launch_pc_apply(const SysView& s, const PcView& pc, const double4* in, double4* out,
                     hipStream_t st);
// as launch_init_residual / launch_update with z = M^-1 r; S_ZZ still
// receives |alpha r|^2, the quantity the tolerance measures
void launch_pc_init_residual(const SysView& s, const PcView& pc, Reduce& red, const double4* E0,
                             const double4* t, double4* r, double4* z, double4* p, float4* p32,
                             int rz_slot, hipStream_t st);
void launch_pc_update(const SysView& s, const PcView& pc, Reduce& red, int rz_slot,
                      int rz_next_slot, double4* x, double4* r, double4* z, const double4* p,
                      const double4* q, hipStream_t st);
// x += w z over the polarizable sites
void launch_axpy4(const SysView& s, double4* x, const double4* z, double w, hipStream_t st);
// a.b into slot (and a.b2 into slot2 when b2 is given)
void launch_dot(const SysView& s, Reduce& red, const double4* a, const double4* b, int slot,
                hipStream_t st, const double4* b2 = nullptr, int slot2 = -1);
void launch_residual_norm(const SysView& s, Reduce& red, const double4* E0, const double4* t,
                          hipStream_t st);
void launch_copy4(const double4* in, double4* out, float4* out32, int n, hipStream_t st);
// sorted-site mu (zero at non-polarizable sites) from polarizable-index x
void launch_mu_sites(const SysView& s, const double4* x, double4* mu, float4* mu32, hipStream_t st);
// caller order [n][3] <-> polarizable index vectors
void launch_pol_to_caller(const SysView& s, const int* perm, const double4* v, double* out,
                          hipStream_t st);
void launch_caller_to_pol(const SysView& s, const int* perm, const double* in, double4* v,
                          float4* v32, hipStream_t st);
// out = a x + b y (polarizable order; y may be NULL)
void launch_lincomb4(const SysView& s, double4* out, double a, const double4* x, double b,
                     const double4* y, hipStream_t st);
// y += a x over count doubles
void launch_axpy_d(size_t count, double a, const double* x, double* y, hipStream_t st);
// sorted records without multipoles (positions, Thole widths kept)
void launch_zero_records(const SysView& s, double4* sp0, double4* sd0, double4* sth0,
                         double2* sth20, hipStream_t st);
// Extrapolated initial guess (polarizable order) from k history entries
// of caller-order dipoles (entry j at hist + slot[j] * stride).
constexpr int kPredMax = 6;
struct PredArgs {
  int k;
  int slot[kPredMax];
  double coef[kPredMax];
};
void launch_predict(const SysView& s, const int* perm, const double* hist, size_t stride,
                    const PredArgs& pa, double4* v, float4* v32, hipStream_t st);
// Coulomb-scaled forces to caller order (no reciprocal part)
void launch_forces_out(int n, const int* perm, const double4* F, double* out, hipStream_t st);
// neighbour counts to caller order
void launch_counts_out(int n, const int* perm, const int* counts, int* out, hipStream_t st);

// frames.hip: molecular local frames (caller order throughout, except FS,
// GS and mu_s, which are in sorted order).
struct FrameArgs {
  int n, ngroups;
  int periodic;
  double box[3], ibox[3];
  const double* xyz;     // [n][3]
  const int* frames;     // [n][3] frame sites (o, a, b); o < 0: no frame
  const double* dloc;    // [n][3] local dipoles
  const double* qloc;    // [n][6] local quadrupoles
  const double* aloc;    // [n][6] local polarizabilities (NULL: not rotated)
  double* dip;           // global outputs (the context's caller-order copies)
  double* quad;
  double* alpha;
  const int* inv_perm;   // caller -> sorted
  const double4* FS;     // site field (sorted)
  const double* GS;      // site field gradient (sorted, 6 per site)
  const double4* mu_s;   // induced dipoles (sorted)
  double* C;             // [n][9] per-site dE/dR
  const int* gframe;     // [ngroups][3] distinct frames
  const int* gstart;     // [ngroups + 1] sites of each frame in gsites
  const int* gsites;
  double* Fg;            // [ngroups][3][3] forces on (o, a, b)
  const int* sstart;     // [n + 1] entries of sref per site
  const int* sref;       // 3 g + slot of every frame force acting on the site
};
// md.hip: Beeman steps (caller order).
struct MdArgs {
  int n;
  int periodic;
  double box[3], ibox[3];
  double* xyz;           // the context's positions
  double* vel;           // [n][3] A/fs
  double* acc;           // [n][3] a(t), A/fs^2
  double* accp;          // [n][3] a(t - dt)
  const double* force;   // [n][3] kcal/mol/A of the electrostatics + polarization
  const double* mass;    // [n] g/mol, 0 for a virtual site
  const int* vpar;       // [n][2] parents of a virtual site, -1 -1 otherwise
  const int* vstart;     // [n + 1] virtual sites parented by each atom (vref)
  const int* vref;
  const int* bonds;      // [nb][2]
  const double* bond_k;  // [nb] kcal/mol/A^2
  const double* bond_r0; // [nb] A
  const int* bstart;     // [n + 1] bonds of each atom (bref)
  const int* bref;
  const double* rep_rho; // [n] repulsion radii (A)
  double rep_eps;        // kcal/mol; 0: no repulsion
  double* rep_force;     // where the repulsion forces are added (= force)
};
// stand-in repulsion forces added to m.rep_force, energy partials S_EREP
void launch_md_repulsion(const SysView& s, const MdArgs& m, Reduce& red, const int* perm,
                         hipStream_t st);
void launch_md_positions(const MdArgs& m, double dt, hipStream_t st);
void launch_md_vsites(const MdArgs& m, hipStream_t st);
// dt = 0 starts a run (a_prev = a = F/m, no velocity update); velocities
// are scaled by 1 - friction after each update
void launch_md_finish(const MdArgs& m, Reduce& red, double dt, double friction,
                      hipStream_t st);

// ct.hip: reduced charge transfer (caller-order inputs; sorted-order
// outputs W_s, U_s, F_s).
struct CtArgs {
  int n, n_lp, n_acc, n_vint;
  const int* lp;          // [n_lp][2] lone-pair site, carrier atom
  const double* lp_par;   // [n_lp][2] occupation, ionization energy (kcal/mol)
  const int* acc;         // [n_acc][2] a1 (the H), a2 (the heavy atom)
  const double* ah;       // [n_acc] affinity (kcal/mol)
  const double* rvdw;     // [n] van der Waals radii (A)
  double eta, cs, cp, t, m;
  const int* a1_start;    // [n + 1] acceptors whose a1 is the site (a1_ref)
  const int* a1_ref;
  const int* car_start;   // [n + 1] lone pairs the site carries (car_ref)
  const int* car_ref;
  const int* lp_of;       // [n] lone pair at the site, or -1
  const int* at_start;    // [n + 1] 2 k + slot of the acceptors the site is in
  const int* at_ref;
  const int* vint_sites;  // [n_vint] distinct acceptor atoms
  const int* perm;        // sorted -> caller
  const int* inv_perm;    // caller -> sorted
  int* flag_s;            // [n] sorted: a1 / carrier / has-multipoles bits
  int4* rng_s;            // [n] sorted: a1_start range, car_start range
  double* lp_rec;         // [n_lp][8] x_l, kC V_l, n, ae, rvdw of the carrier, 0
  double* acc_rec;        // [n_acc][8] x_a2, kC V_int(a1), kC V_int(a2), rvdw a1, a2, ah
  double* Vlp;            // [n_lp] V_l (e/A)
  double* Gr;             // [n_lp][3] reciprocal grad V_l
  double* Vint;           // [n] V_int at acceptor atoms (e/A)
  double* w;              // [n_lp] dE/dV_l
  double* Fl;             // [n_lp][3] direct force on the lone pair
  double* Fc;             // [n_lp][3] direct force on its carrier
  double* Fa;             // [n_acc][2][3] direct forces on a1, a2
  double* ua;             // [n_acc][2] dE/dV_int(a1), dE/dV_int(a2)
  double* W_s;            // [n] sorted: w at lone-pair sites
  double* U_s;            // [n] sorted: u at acceptor atoms
  double4* F_s;           // [n] sorted: forces (kcal/mol/A, then / Coulomb)
};
void launch_ct_potentials(const SysView& s, const CtArgs& a, hipStream_t st);
void launch_ct_gather_pot(const SysView& s, const PmeView& pm, const CtArgs& a, hipStream_t st);
// energy partials into S_ECT
void launch_ct_pairs(const SysView& s, const CtArgs& a, Reduce& red, hipStream_t st);
// sp_w (may be NULL): records with the w charges for the reciprocal spread
// FS, GS (may be NULL): also the field and field gradient of the w and u
// charges at every site (sorted, divided by the Coulomb constant), real
// space, for the forces of local frames
void launch_ct_wforce(const SysView& s, const CtArgs& a, double4* sp_w, hipStream_t st,
                      double4* FS = nullptr, double* GS = nullptr);

// global d, Theta (and alpha when aloc is set) from the local ones
void launch_rotate(const FrameArgs& f, hipStream_t st);
// forces of the rotation added to forces (caller order); virial: also the
// frame virial partials (slots S_VRR)
void launch_frame_forces(const FrameArgs& f, Reduce& red, double* forces, bool virial,
                         hipStream_t st);

}  // namespace sibfa
