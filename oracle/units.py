"""Unit constants of the oracle (the paper states none; Tinker's values).

COULOMB  kcal*A/(mol*e^2): energies are COULOMB * (e^2/A).
DEBYE    Debye per e*A: the solver tolerance is an RMS in Debye.
"""
COULOMB = 332.0637133
DEBYE = 4.803204
