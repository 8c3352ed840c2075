"""Plain FP64 CPU oracle for the SIBFA many-body polarization path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product library imports, links or
runs this package; only the tests, the smoke check and the benchmark's
CPU-baseline leg do.  It shares no code with the HIP path.

What it computes (paper: "Development of the Quantum Inspired SIBFA
Many-Body Polarizable Force Field", technical appendix, Polarization):
  * the field E of the permanent multipoles (charge, dipole, quadrupole) at
    every polarizable site,
  * the polarization matrix T (inverse polarizabilities on the diagonal
    blocks, minus the dipole-dipole field tensors off the diagonal),
  * the induced dipoles mu solving T mu = E (Eq. 18) by preconditioned
    conjugate gradient or by a dense solve, and the fixed-cost truncated
    conjugate gradient (TCG-n) the paper names as the alternative,
  * E_pol = -1/2 mu.E (Eq. 19) and the variational form
    1/2 mu.T mu - mu.E (Eq. 17),
  * the multipolar electrostatic energy (Eq. 2, without the penetration
    correction) and the forces at fixed mu,
for gas-phase clusters (direct sums), periodic boxes with brute-force Ewald
sums, and periodic boxes with Smooth Particle Mesh Ewald.

Readings where the paper is silent (Thole form and constant, exclusions,
quadrupole convention, Nyquist handling of the B-spline moduli, units of the
solver tolerance) are listed in the module docstrings that use them.
"""
from .model import Params, System, evaluate, permanent_field, apply_T, \
    dense_T_columns, dense_T_blocks, energy_forces, electrostatic_energy, tcg
from .solver import pcg, plain_cg, jacobi
from . import radial, tensors, realspace, recip, units, frames, md, ct

__all__ = ["Params", "System", "evaluate", "permanent_field", "apply_T",
           "dense_T_columns", "dense_T_blocks", "energy_forces",
           "electrostatic_energy", "tcg", "pcg", "plain_cg", "jacobi", "radial",
           "tensors", "realspace", "recip", "units", "frames"]
