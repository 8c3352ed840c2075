"""Shared helpers of the GPU tests: run the HIP path through the binding and
the oracle on the same seeded inputs."""
import sys

import numpy as np

import oracle
from oracle.model import System, Params


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def oracle_params(sysd, beta=0.4, cutoff=9.0, grid=32, order=5, tol=1e-10):
    if sysd.get("box") is None:
        return Params(method="direct", tol=tol)
    g = (grid, grid, grid) if isinstance(grid, int) else tuple(grid)
    return Params(method="spme", beta=beta, cutoff=cutoff, grid=g, order=order, tol=tol)


def gpu_params(sysd, beta=0.4, cutoff=9.0, grid=32, order=5, tol=1e-10, precision="fp64",
               max_iter=200, **extra):
    from paper_2201_00804_amd import default_params
    return default_params(beta=beta, cutoff=cutoff, grid=grid, order=order, tol=tol,
                          precision=precision, max_iter=max_iter, **extra)


def engine_for(sysd, prm):
    from paper_2201_00804_amd import Engine
    eng = Engine(0)
    eng.load(sysd, prm)
    return eng


def rel_err(a, b):
    """Largest elementwise difference over the largest reference entry
    (absolute when the reference is all zero)."""
    a = np.asarray(a, float)
    b = np.asarray(b, float)
    scale = np.abs(b).max() if b.size else 0.0
    diff = np.abs(a - b).max() if b.size else 0.0
    return float(diff / scale) if scale > 0 else float(diff)


def rms_rel(a, b):
    """Relative RMS difference (absolute RMS when the reference is zero)."""
    a = np.asarray(a, float)
    b = np.asarray(b, float)
    num = np.sqrt(np.mean((a - b) ** 2))
    den = np.sqrt(np.mean(b ** 2))
    return float(num / den) if den > 0 else float(num)


def pol_rows(sysd):
    return np.flatnonzero(np.any(np.asarray(sysd["alpha"]) != 0, axis=1))
