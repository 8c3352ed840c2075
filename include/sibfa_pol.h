/*
 * sibfa_pol.h -- C-ABI of the MI355X (gfx950) library for the SIBFA
 * many-body polarization path under periodic boundaries (Smooth PME) and
 * for gas-phase clusters.
 *
 * What it computes (Naseem-Khan et al., "Development of the Quantum Inspired
 * SIBFA Many-Body Polarizable Force Field", technical appendix,
 * Polarization, Eq. 17-19): given sites carrying permanent multipoles
 * (charge q, dipole d, traceless Buckingham quadrupole Theta) and 3x3
 * polarizability tensors alpha_i,
 *   E      = field of the permanent multipoles at the polarizable sites,
 *   T      = polarization matrix: alpha_i^-1 on the diagonal blocks and minus
 *            the Thole-damped dipole field tensors off the diagonal,
 *   mu     = solution of T mu = E (Eq. 18), by preconditioned conjugate
 *            gradient (Computational Details),
 *   E_pol  = -1/2 mu . E (Eq. 19),
 *   E_elec = plain multipole-multipole electrostatic energy (Eq. 2 without
 *            the penetration correction),
 *   forces = -d(E_elec + E_pol)/dr at the converged mu.
 * Periodic boxes use Ewald splitting with Smooth PME for the reciprocal
 * part (the paper's SPME treatment of multipoles and polarization), tin-foil
 * boundary, minimum image in real space.
 *
 * Conventions shared by every call:
 *  - Units: A, e, e*A, e*A^2, A^3; energies kcal/mol (332.0637133 e^2/A);
 *    forces kcal/mol/A; tolerances in Debye (4.803204 D per e*A).
 *  - Array arguments are DEVICE pointers on the context's device, in the
 *    caller's site order, row-major AoS: xyz [n][3], dipoles [n][3],
 *    quadrupoles [n][6] ordered xx,xy,xz,yy,yz,zz, polarizabilities [n][6]
 *    in the same order.  They are read (or written) during the call on the
 *    context's stream and never retained: the library copies what it needs
 *    into its own cell-sorted device buffers.  Scalars (energies, iteration
 *    counts, residuals) are HOST pointers.
 *  - Calls that return host scalars synchronize the context's stream;
 *    the others only enqueue work on it.  sibfa_solve_induced reads its
 *    scalars at the solver's last stop test and returns with the copy of
 *    mu_out still enqueued (ordered before later work on the stream).
 *  - Exclusions: a molecule's own sites do not interact through E or
 *    E_elec; induced dipoles of one molecule do couple (Thole-damped).
 *  - Thole damping: lambda_3 = 1 - exp(-a u^3), u = r/(abar_i abar_j)^(1/6),
 *    abar = trace(alpha)/3, a_ij = min(a_i, a_j); higher tensors are the
 *    exact derivatives of the damped field.  No damping when a site is not
 *    polarizable.
 *  - Errors: every call returns a sibfa_status; on a negative status the
 *    message is available from sibfa_last_error and the context stays
 *    usable (state set by earlier successful calls is kept).
 *  - Thread safety: one host thread per context at a time; different
 *    contexts may be used concurrently.
 */
#ifndef SIBFA_POL_H
#define SIBFA_POL_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct sibfa_ctx_s* sibfa_ctx;

typedef enum {
  SIBFA_OK = 0,
  SIBFA_E_ARG = -1,           /* invalid argument (NULL, size, NaN, cutoff) */
  SIBFA_E_STATE = -2,         /* call order violated                        */
  SIBFA_E_NOMEM = -3,         /* device allocation failed                   */
  SIBFA_E_NOT_SPD = -4,       /* p.Tp <= 0 met in the solver                */
  SIBFA_E_NOT_CONVERGED = -5, /* max_iter reached above the tolerance       */
  SIBFA_E_DEVICE = -6         /* HIP runtime error                          */
} sibfa_status;

typedef enum { SIBFA_FP64 = 0, SIBFA_MIXED = 1 } sibfa_precision;

/* Preconditioner of the PCG solve (Eq. 18; the paper names a preconditioned
 * conjugate gradient and leaves the preconditioner open).  DIAG: z = alpha r
 * per site.  MOLBLOCK: z = M^-1 r with M, per molecule of at most 4
 * polarizable sites, the molecule's block of T in bare form (alpha^-1 on
 * the diagonal, the Thole-damped dipole-dipole tensors between its sites);
 * larger molecules keep alpha per site.  Either way the solve stops on the
 * RMS of alpha (E - T mu), so both reach the same tolerance; the truncated
 * solver (sibfa_solve_tcg) always uses DIAG. */
typedef enum { SIBFA_PRECOND_DIAG = 0, SIBFA_PRECOND_MOLBLOCK = 1 } sibfa_precond;

typedef struct {
  double ewald_beta;    /* A^-1, Ewald splitting parameter (periodic only)   */
  double cutoff;        /* A, real-space cutoff; must be < min(box)/2        */
  int grid[3];          /* PME points per axis: even, factors 2,3,5 only     */
  int order;            /* B-spline order: 4, 5 or 6                         */
  double thole_a;       /* default Thole factor (0.28 in the paper's model)  */
  double tol_debye;     /* solver tolerance: RMS of alpha*(E - T mu), Debye  */
  int max_iter;         /* PCG iteration limit, all sequences together       */
  sibfa_precision precision; /* FP64, or FP32 pair/PME math with FP64
                                accumulation, reductions and residuals      */
  sibfa_precond precond;     /* preconditioner of sibfa_solve_induced       */
} sibfa_params;

typedef struct {
  int iterations;          /* PCG iterations of the last solve              */
  int restarts;            /* FP64 true-residual replacements of the last
                              solve (the final confirmation not counted)   */
  double true_rms_debye;   /* RMS of alpha*(E - T mu), recomputed in FP64    */
  double e_pol;            /* kcal/mol, Eq. 19                               */
  double e_pol_variational;/* kcal/mol, Eq. 17 at the returned mu            */
  double e_elec;           /* kcal/mol                                       */
  double e_elec_real;      /* kcal/mol, real-space pairs                     */
  double e_elec_recip;     /* kcal/mol, reciprocal (0 for clusters)          */
  double e_elec_self;      /* kcal/mol, Ewald self term (0 for clusters)     */
  int n_sites, n_polarizable;
  int max_neighbors;       /* largest real-space neighbour count of a site   */
} sibfa_stats;

typedef void* (*sibfa_alloc_fn)(size_t bytes, void* user);
typedef void (*sibfa_free_fn)(void* ptr, void* user);

/* Create a context on HIP device `device`, enqueuing on `hip_stream`
 * (a hipStream_t; NULL = the null stream).  alloc/free (both or neither)
 * provide device memory, e.g. from a caching allocator; NULL = hipMalloc. */
sibfa_status sibfa_create(sibfa_ctx* out, int device, void* hip_stream,
                          sibfa_alloc_fn alloc_fn, sibfa_free_fn free_fn,
                          void* user);
void sibfa_destroy(sibfa_ctx ctx);
const char* sibfa_last_error(sibfa_ctx ctx);

/* Fill *p with the defaults (beta 0.4, cutoff 9, grid 32^3, order 5,
 * thole 0.28, tol 1e-8 D, 200 iterations, FP64). */
void sibfa_default_params(sibfa_params* p);

/* Device bytes a context will hold for a system of n_sites sites of which
 * n_polarizable are polarizable (box NULL = cluster); for admission
 * control.  The polarizable count is an argument because the
 * polarization-pair lists and their cached coefficients (rows and density
 * both follow it) dominate the footprint, and a caller admitting a request
 * knows it from its polarizabilities before any context exists.  Returns 0
 * on invalid arguments. */
size_t sibfa_footprint_bytes(int n_sites, int n_polarizable,
                             const double* box, const sibfa_params* p);

/* Define the system: n_sites sites at xyz [n][3] (device), molecule ids
 * mol [n] (device int32, each in [0, n)), box [3] (HOST, orthorhombic edge
 * lengths) or NULL for a non-periodic cluster, and the parameters (HOST).
 * The sites are the paper's multipole centres (Multipolar Electrostatics:
 * atoms and bond barycentres of each molecule); molecule ids carry the
 * exclusion rule above (the permanent field and E_elec are intermolecular
 * terms).  The Ewald/SPME parameters are those of the Computational
 * Details' periodic runs.  Periodic systems need every molecule's sites
 * within the cutoff of each other (checked when lists are built:
 * SIBFA_E_ARG). */
sibfa_status sibfa_set_system(sibfa_ctx ctx, int n_sites, const double* xyz,
                              const int32_t* mol, const double* box,
                              const sibfa_params* params);

/* New positions for the same sites (one MD step of the Computational
 * Details); keeps mu as the guess for the next solve (warm start).  Only
 * enqueues the copy: NaN/Inf coordinates are reported (SIBFA_E_ARG) by the
 * next call that computes. */
sibfa_status sibfa_update_positions(sibfa_ctx ctx, const double* xyz);

/* Permanent multipoles (device): q [n], dip [n][3], quad [n][6] traceless,
 * the distributed multipoles up to quadrupole of Multipolar
 * Electrostatics (Eq. 2), given in the global frame.  dip or quad may be
 * NULL (zero). */
sibfa_status sibfa_set_multipoles(sibfa_ctx ctx, const double* q,
                                  const double* dip, const double* quad);

/* Polarizabilities alpha [n][6] (device; symmetric positive definite, or an
 * all-zero row for a non-polarizable site), the 3x3 alpha_i of the
 * technical appendix (Polarization) whose inverses are T's diagonal blocks,
 * and optional per-site Thole factors thole [n] (device; NULL =
 * params.thole_a; the Thole damping of Many-Body Polarization). */
sibfa_status sibfa_set_polarizabilities(sibfa_ctx ctx, const double* alpha,
                                        const double* thole);

/* Molecular local frames (Multipolar Electrostatics: the distributed
 * multipoles, and SIBFA's anisotropic polarizabilities, are given in a
 * frame attached to the molecule and rotated to the global frame at each
 * geometry).  frames [n][3] (device, int32): for every site the indices
 * (o, a, b) of three distinct sites of its own molecule that span its
 * frame (e_z along the bisector of r_a - r_o and r_b - r_o, e_x in their
 * plane towards a, e_y = e_z x e_x), or -1 -1 -1 for a site whose local
 * values are already global.  dip_local [n][3], quad_local [n][6]
 * (device; NULL = zero) replace the dipoles and quadrupoles of
 * sibfa_set_multipoles (q stays); alpha_local [n][6] (device; NULL = the
 * polarizabilities of sibfa_set_polarizabilities are not rotated)
 * replaces them.  The library copies all arrays.  From then on every
 * computation rotates them at the current positions, and the forces of
 * sibfa_energy_forces include the derivative of the rotation (the torques
 * as forces on the frame sites), as does its virial.  Call after
 * sibfa_set_multipoles and sibfa_set_polarizabilities (SIBFA_E_STATE
 * otherwise); a later call of either of them switches the frames off, as
 * does frames = NULL (the global multipoles then stay those of the last
 * rotation).  A frame that does not meet the rules above: SIBFA_E_ARG,
 * nothing changed.  Synchronizes the context's streams.  Device memory:
 * about 300 bytes per site more while frames are set (the local copies
 * and the buffers of the rotation forces). */
sibfa_status sibfa_set_local_frames(sibfa_ctx ctx, const int32_t* frames,
                                    const double* dip_local,
                                    const double* quad_local,
                                    const double* alpha_local);

/* Permanent field E (Eq. 18's right-hand side, e/A^2) at every site, [n][3]
 * (device), zero rows at non-polarizable sites. */
sibfa_status sibfa_permanent_field(sibfa_ctx ctx, double* field_out);

/* tp_out = T p for p given on every site [n][3] (device; rows of
 * non-polarizable sites are ignored, their output rows are zero). */
sibfa_status sibfa_apply_T(sibfa_ctx ctx, const double* p, double* tp_out);

/* Solve T mu = E by PCG (preconditioner per params.precond: alpha per site,
 * or the molecular blocks of T).
 * warm_start: start from the dipoles kept from the previous solve (or set
 * by sibfa_set_dipoles), or the predictor's extrapolation of them (see
 * sibfa_set_predictor), instead of alpha E.  mu_out [n][3] (device) or
 * NULL; iters and true_rms_debye (HOST) may be NULL.  Returns
 * SIBFA_E_NOT_CONVERGED (mu still returned) or SIBFA_E_NOT_SPD. */
sibfa_status sibfa_solve_induced(sibfa_ctx ctx, int warm_start, double* mu_out,
                                 int* iters, double* true_rms_debye);

/* Truncated conjugate gradient (TCG-n), the fixed-cost alternative to an
 * iterated solve that the paper names (Many-Body Polarization; defined in
 * the work it cites).  The dipoles are the `order`-th iterate of the PCG
 * above, with no convergence test, then, when omega != 0, one peek step
 * mu += omega alpha r with that iterate's residual r.  The guess is the
 * direct field alpha E, or with warm_start the dipoles kept from the last
 * solve_induced or given to sibfa_set_dipoles, or the predictor's
 * extrapolation of them (SIBFA_E_STATE if there are none).  order: 1..SIBFA_TCG_MAX_ORDER.  mu_out [n][3]
 * (device, zero rows at non-polarizable sites) or NULL; e_pol (HOST,
 * kcal/mol) = -1/2 mu.E (the form of Eq. 19) or NULL.  Runs in the
 * context's precision and returns after a stream synchronisation.  The
 * dipoles of the last solve_induced stay the warm start; the next
 * energy_forces solves again.  This call returns no forces:
 * sibfa_tcg_energy_forces below gives the forces at TCG dipoles (the
 * fixed-dipole identity of sibfa_energy_forces holds only at the converged
 * solution).
 * Returns SIBFA_E_ARG for a bad order or a non-finite omega, SIBFA_E_NOT_SPD
 * if p.Tp <= 0 in a step. */
#define SIBFA_TCG_MAX_ORDER 64
sibfa_status sibfa_solve_tcg(sibfa_ctx ctx, int order, double omega, int warm_start,
                             double* mu_out, double* e_pol);

/* TCG-n energies and forces (Many-Body Polarization names the truncated
 * solver; its analytic derivative is given in the work it cites, not in
 * the paper): the dipoles of sibfa_solve_tcg (same order, omega and guess;
 * a warm guess counts as fixed), E_pol = -1/2 mu.E at them and E_elec
 * (HOST, kcal/mol), and the forces of E_elec + E_pol [n][3] (device,
 * kcal/mol/A, or NULL), which include the derivative of every step of the
 * truncated iteration (at TCG dipoles the fixed-dipole identity of
 * sibfa_energy_forces does not hold).  Always FP64.  The reverse pass
 * through the iteration costs n + 1 matvecs and the forces 2n + 4 force
 * evaluations; every step reads a dot product back to the host.  mu_out
 * [n][3] (device) or NULL.  Errors as sibfa_solve_tcg. */
sibfa_status sibfa_tcg_energy_forces(sibfa_ctx ctx, int order, double omega, int warm_start,
                                     double* e_pol, double* e_elec, double* forces,
                                     double* mu_out);

/* Energies (HOST, kcal/mol) and forces [n][3] (device, kcal/mol/A, or
 * NULL) at the current dipoles; solves first if they are stale.
 * virial [9] (HOST, kcal/mol, row-major) or NULL: W_ab = -dE/d eps_ab,
 * E = E_elec + E_pol, for the homogeneous strain r -> (1 + eps) r of every
 * site and of the box, with the multipoles, polarizabilities and induced
 * dipoles held in the global frame (the dipoles make E_pol stationary, so
 * this is the full strain derivative, as the forces are the full
 * gradient; the NPT runs of the Computational Details need it).  Real
 * space: 1/2 sum over ordered pairs of f_a R_b; reciprocal (Smooth PME of
 * the combined density q, d + mu, Theta):
 *   W_ab = delta_ab E_rec - sum_m G(m) (pi^2/beta^2 + 1/m^2) m_a m_b |S(m)|^2
 *          + sum_j [(d + mu)_jb d_a phi(r_j) + 2/3 Theta_jbc d_a d_c phi(r_j)].
 * Not symmetric in general (the global-frame multipoles do not rotate with
 * the strain).  Pairs crossing the cutoff under the strain are not
 * followed, as for the energy. */
sibfa_status sibfa_energy_forces(sibfa_ctx ctx, double* e_pol, double* e_elec,
                                 double* forces, double* virial);

/* Copy out / restore the induced dipoles mu of Eq. 18 [n][3] (device):
 * the next solve starts from the restored ones when warm-started (an
 * extrapolated guess from earlier steps, as the truncated and predicted
 * solvers the Many-Body Polarization section cites use). */
sibfa_status sibfa_get_dipoles(sibfa_ctx ctx, double* mu);
sibfa_status sibfa_set_dipoles(sibfa_ctx ctx, const double* mu);

/* Predictor of the warm-start guess (the extrapolated guesses that the
 * truncated and iterated solvers cited under Many-Body Polarization start
 * from along a trajectory).  The context keeps the last
 * SIBFA_PREDICT_MAX_ORDER dipole sets: every converged sibfa_solve_induced
 * (also the one inside sibfa_energy_forces) and every sibfa_set_dipoles
 * adds one.  With order k >= 2 a warm start (solve or TCG) begins at the
 * value for the next step of the polynomial of degree k' - 1 through the
 * k' = min(k, kept) newest sets, taken as equally spaced in time:
 * mu_guess = sum_{j=1..k'} (-1)^(j+1) C(k', j) mu_(newest - j + 1)
 * (k' = 2: 2 mu_1 - mu_2).  Order 0 or 1, or fewer than two sets kept: the
 * newest set (the plain warm start).  Setting the order clears the history;
 * so do new polarizabilities and sibfa_set_system.  The history takes
 * SIBFA_PREDICT_MAX_ORDER * 24 bytes per site of device memory, allocated
 * with the first set it keeps.  SIBFA_E_ARG for an order outside
 * 0..SIBFA_PREDICT_MAX_ORDER. */
#define SIBFA_PREDICT_MAX_ORDER 6
sibfa_status sibfa_set_predictor(sibfa_ctx ctx, int order);

/* Reduced many-body charge transfer (Many-Body Charge Transfer/Charge
 * Delocalization, the reduced expression, Eq. 13-16):
 *   E_ct = sum_l sum_k -n(l) (e1 - e2)^2 / (ae(l) + V_l - ah(k)),
 *   e1 = exp(-eta rho1) (V_int(a1) - V_l) (C_s t + C_p m cos alpha),
 *   e2 = exp(-eta rho2) (V_int(a2) - V_l) (C_s t + C_p m cos beta),
 * over lone pairs l (a site of the molecule, carried by atom c) and
 * acceptor bonds k = (a1, a2) (a1 the hydrogen) of other molecules whose
 * a1 lies within the real-space cutoff of c (every other molecule for a
 * cluster); rho = |r_c - r_a| / (2 sqrt(rvdw_c rvdw_a)); alpha, beta the
 * angles at c between r_l - r_c and r_a1 - r_c, r_a2 - r_c.  V_l is the
 * potential at the lone pair of the other molecules' permanent multipoles
 * (Smooth PME in a box, own molecule excluded), V_int(a) the bare potential
 * at atom a of its own molecule's other sites; both enter in kcal/mol per
 * unit charge.
 * sibfa_set_charge_transfer: lp [n_lp][2] (device int32: lone-pair site,
 * carrier atom, one molecule; the lone-pair site carries no multipoles and
 * no polarizability), lp_par [n_lp][2] (device: occupation n, ionization
 * energy ae, kcal/mol), acc [n_acc][2] (device int32: a1, a2 of one
 * molecule), acc_ah [n_acc] (device, kcal/mol), rvdw [n] (device, A,
 * positive at carriers and acceptor atoms), constants (HOST).  Copied and
 * checked once (SIBFA_E_ARG); call after the multipoles, polarizabilities
 * and local frames (sibfa_set_local_frames); setting any of them again
 * switches the term off.  With local frames the lone-pair sites carry no
 * local multipoles or polarizability either.  Synchronizes.
 * sibfa_ct_energy_forces: E_ct (HOST, kcal/mol) and, when forces is not
 * NULL, its forces [n][3] (device, kcal/mol/A, written, not added),
 * including those through the potentials and, with local frames, those of
 * the rotation of the multipoles (E_ct depends on them through V_l and
 * V_int).  Always FP64; independent of the induced dipoles (no solve). */
typedef struct {
  double eta, cs, cp, t, m;
} sibfa_ct_params;
sibfa_status sibfa_set_charge_transfer(sibfa_ctx ctx, int n_lp, const int32_t* lp,
                                       const double* lp_par, int n_acc, const int32_t* acc,
                                       const double* acc_ah, const double* rvdw,
                                       const sibfa_ct_params* params);
sibfa_status sibfa_ct_energy_forces(sibfa_ctx ctx, double* e_ct, double* forces);

/* Molecular dynamics (Computational Details: Beeman integrator, 1 fs
 * steps, the polarization solved at every step).  The paper's other terms
 * (repulsion, dispersion, bonded terms) are outside this library, and the
 * charge transfer above is not added to the MD forces, so the driver takes
 * harmonic bonds as a stand-in that holds the molecules together; a trajectory exercises and times the polarization
 * path, it is not the paper's model.
 * sibfa_md_init: masses [n] (device, g/mol; 0 marks a virtual site),
 * vsites [n][2] (device int32 or NULL: none): the two atoms whose midpoint
 * (minimum image) a virtual site is, -1 -1 for an atom; n_bonds harmonic
 * bonds [n_bonds][2] between atoms (device int32) with bond_k (kcal/mol/A^2)
 * and bond_r0 (A) (device); a stand-in short-range repulsion
 * rep_eps ((rho_i + rho_j)/r)^12 (kcal/mol) between sites of different
 * molecules within the cutoff whose radii are both positive (virtual sites
 * included; their forces go to the parents), rep_radius [n] (device, A,
 * >= 0; NULL with rep_eps = 0: none); vel [n][3] (device, A/fs, or NULL:
 * zero).
 * Places the virtual sites, evaluates the forces at the current positions
 * and starts the integrator (a(-dt) = a(0)).  Needs the system, multipoles
 * and polarizabilities (local frames and the predictor are used when set).
 * Sites of a molecule must stay within the cutoff of each other, as for
 * every call.  Synchronizes.
 * sibfa_md_run: n_steps Beeman steps of dt_fs: new positions, a warm-
 * started solve (with the predictor if one is set), forces, new velocities,
 * then scaled by 1 - friction (friction in [0, 1]; 0 is plain Beeman, a
 * positive value a damped relaxation, e.g. to remove the close contacts of
 * a synthetic start before a run).
 * stats [n_steps] (HOST or NULL): per step E_pol, E_elec, bond, repulsion
 * and kinetic energy (kcal/mol) and the solver iterations.  An error stops the run
 * with the positions of that step already moved.
 * sibfa_md_get_state: positions and velocities [n][3] (device; either may
 * be NULL).  A later sibfa_set_system ends the dynamics. */
typedef struct {
  double e_pol, e_elec, e_bond, e_rep, e_kin;
  int iterations;
} sibfa_md_stats;
sibfa_status sibfa_md_init(sibfa_ctx ctx, const double* masses, const int32_t* vsites,
                           int n_bonds, const int32_t* bonds, const double* bond_k,
                           const double* bond_r0, const double* rep_radius, double rep_eps,
                           const double* vel);
sibfa_status sibfa_md_run(sibfa_ctx ctx, int n_steps, double dt_fs, double friction,
                          sibfa_md_stats* stats);
sibfa_status sibfa_md_get_state(sibfa_ctx ctx, double* xyz, double* vel);

/* Real-space neighbour counts per site [n] (device int32): intermolecular
 * sites within the cutoff (all sites within reach for clusters). */
sibfa_status sibfa_neighbor_counts(sibfa_ctx ctx, int32_t* counts_out);

/* Statistics of the last solve / energy evaluation (HOST). */
sibfa_status sibfa_get_stats(sibfa_ctx ctx, sibfa_stats* out);

/* Per-phase kernel timing with HIP events recorded on the context's stream
 * around the launches of each phase (enable = 1 starts and clears the
 * accumulators, 0 stops).  Phases: */
typedef enum {
  SIBFA_PH_LISTS = 0,     /* binning, cell sort, records, neighbour lists   */
  SIBFA_PH_FIELD_REAL,    /* real-space permanent field + E_elec pairs      */
  SIBFA_PH_FIELD_RECIP,   /* permanent PME: spread, convolution, gather     */
  SIBFA_PH_SPREAD,        /* solver: direction update + dipole spreading    */
  SIBFA_PH_FFT,           /* solver: 3D FFT convolution (5 passes)          */
  SIBFA_PH_MATVEC,        /* solver: real-space part of T p                  */
  SIBFA_PH_UPDATE,        /* solver: x, r, z updates and dot products       */
  SIBFA_PH_FORCE_REAL,    /* real-space forces                              */
  SIBFA_PH_FORCE_RECIP,   /* combined-density PME forces                    */
  SIBFA_PH_PAIRCOEF,      /* solver: damped pair coefficients, once a solve  */
  SIBFA_PH_MATVEC_RECIP,  /* solver: PME field gather of T p and p.Tp        */
  SIBFA_PH_MATVEC_FP64,   /* mixed precision: each whole FP64 T x (residual
                             replacements, TCG adjoint products); the
                             phases above then hold FP32 launches only      */
  SIBFA_PH_COUNT
} sibfa_phase;

typedef struct {
  double ms[16];          /* accumulated event time per phase, milliseconds */
  int calls[16];          /* number of timed launches (groups) per phase    */
  long long pairs[4];     /* list entries: all, same-molecule, pol, pol-same */
} sibfa_profile;

sibfa_status sibfa_set_profiling(sibfa_ctx ctx, int enable);
/* As sibfa_set_profiling, timing only the phases whose bit (1 << phase) is
 * set in phase_mask (0 = off): fewer events, less perturbation.  Each timed
 * phase boundary costs the stream a few microseconds. */
sibfa_status sibfa_set_profiling_phases(sibfa_ctx ctx, unsigned phase_mask);
/* Synchronizes the stream and returns the accumulated times. */
sibfa_status sibfa_get_profile(sibfa_ctx ctx, sibfa_profile* out);

/* ------------------------------------------------------------------------
 * Batched gas-phase clusters (serving many small independent systems).
 *
 * Same mathematics as a cluster context (direct sums, no cutoff; the
 * permanent field, the PCG solve of T mu = E (Eq. 18), E_pol (Eq. 19),
 * E_elec and forces), for many clusters in one call: one workgroup owns one
 * cluster and keeps its whole solve on the device, so a batch costs three
 * kernel launches and no host synchronisation.  A cluster's results are
 * bitwise independent of the other clusters in the batch.  The batched
 * solve uses the diagonal preconditioner (params.precond is not read).
 *
 * Limits per cluster: at most SIBFA_BATCH_MAX_SITES sites and
 * SIBFA_BATCH_MAX_POLARIZABLE polarizable sites (larger systems use a
 * context).
 * ------------------------------------------------------------------------ */
#define SIBFA_BATCH_MAX_SITES 1024
#define SIBFA_BATCH_MAX_POLARIZABLE 640

typedef struct sibfa_batch_s* sibfa_batch;

/* A batch executor on `device`, enqueuing on `hip_stream`; alloc/free as
 * for sibfa_create.  It owns scratch memory that grows to the largest batch
 * seen (about 240 bytes per site) and pinned staging for the offsets. */
sibfa_status sibfa_batch_create(sibfa_batch* out, int device, void* hip_stream,
                                sibfa_alloc_fn alloc_fn, sibfa_free_fn free_fn,
                                void* user);
/* Waits for the batch stream, then releases everything. */
void sibfa_batch_destroy(sibfa_batch b);
const char* sibfa_batch_last_error(sibfa_batch b);

/* Evaluate n_clusters clusters stored back to back.
 *  site_offsets [n_clusters + 1] (HOST): cluster c owns sites
 *    [site_offsets[c], site_offsets[c+1]); site_offsets[0] = 0; each
 *    cluster has 1..SIBFA_BATCH_MAX_SITES sites.
 *  warm_start [n_clusters] (HOST) or NULL: nonzero = start cluster c's
 *    solve from the dipoles found in mu instead of alpha E.
 *  xyz [n][3], mol [n], q [n], dip [n][3], quad [n][6], alpha [n][6],
 *    thole [n] or NULL: DEVICE, caller layout as for a context; molecule
 *    ids only need to compare equal within a molecule.
 *  params (HOST): thole_a, tol_debye, max_iter and precision are used;
 *    the Ewald/PME fields are ignored.
 * Outputs (DEVICE), written when the batch's kernels complete on the
 * stream (the call itself only enqueues work):
 *  mu [n][3] (also the warm-start input), forces [n][3] or NULL,
 *  e_pol, e_elec [n_clusters] kcal/mol, iterations [n_clusters],
 *  rms_debye [n_clusters] (true residual), status [n_clusters]:
 *  SIBFA_OK, SIBFA_E_ARG (alpha not positive definite, or too many
 *  polarizable sites: zero mu and forces, NaN e_pol), SIBFA_E_NOT_SPD or
 *  SIBFA_E_NOT_CONVERGED (mu and forces at the last iterate).
 * Input arrays must stay valid and unchanged until the batch completes;
 * batches on one executor run in call order. */
sibfa_status sibfa_batch_clusters(sibfa_batch b, int n_clusters,
                                  const int* site_offsets, const int* warm_start,
                                  const double* xyz, const int32_t* mol,
                                  const double* q, const double* dip,
                                  const double* quad, const double* alpha,
                                  const double* thole, const sibfa_params* params,
                                  double* mu, double* forces, double* e_pol,
                                  double* e_elec, int* iterations,
                                  double* rms_debye, int* status);

/* ------------------------------------------------------------------------
 * Batched clusters without allocation.
 *
 * For callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc.  The same
 * computation and kernels as sibfa_batch_clusters, with no executor: the
 * scratch arrays live in a fixed device array of the library (about 8 MB,
 * for at most SIBFA_BATCH_NOALLOC_MAX_SITES sites and
 * SIBFA_BATCH_NOALLOC_MAX_CLUSTERS clusters per call), which each device
 * holds until the process ends.  The call allocates nothing, enqueues three
 * kernels on hip_stream (a hipStream_t; NULL = null stream) on `device` and
 * returns; it neither synchronises nor copies from the host.
 *
 * Differences from sibfa_batch_clusters:
 *  - site_offsets [n_clusters + 1] and warm_start [n_clusters] (or NULL)
 *    are DEVICE arrays; n_sites is the number of sites in the caller
 *    arrays.  The offsets are checked on the device: a cluster whose range
 *    is not 1..SIBFA_BATCH_MAX_SITES sites inside [0, n_sites) gets status
 *    SIBFA_E_ARG and NaN e_pol and e_elec, and its mu and forces rows are
 *    not written.
 *  - Errors are return codes only: SIBFA_E_ARG (n_clusters or n_sites out
 *    of range, a required pointer NULL, bad params), SIBFA_E_DEVICE (HIP
 *    error).
 *  - Every call on one device uses the same scratch array, and each call
 *    rewrites every scratch value it reads, so nothing carries over between
 *    calls.  Calls that overlap in time on one device (other streams, other
 *    threads, or enqueued before an earlier call's kernels have finished
 *    while on another stream) race on it: order them on one stream.
 * Inputs and outputs as for sibfa_batch_clusters, all DEVICE pointers.
 * ------------------------------------------------------------------------ */
#define SIBFA_BATCH_NOALLOC_MAX_SITES 32768
#define SIBFA_BATCH_NOALLOC_MAX_CLUSTERS 4096

sibfa_status sibfa_batch_clusters_noalloc(int device, void* hip_stream, int n_clusters,
                                          int n_sites, const int* site_offsets,
                                          const int* warm_start, const double* xyz,
                                          const int32_t* mol, const double* q,
                                          const double* dip, const double* quad,
                                          const double* alpha, const double* thole,
                                          const sibfa_params* params, double* mu,
                                          double* forces, double* e_pol, double* e_elec,
                                          int* iterations, double* rms_debye, int* status);

#ifdef __cplusplus
}
#endif
#endif /* SIBFA_POL_H */
