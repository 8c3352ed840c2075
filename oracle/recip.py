"""Reciprocal-space sums: brute-force Ewald k-sum and Smooth PME.

Both compute, for a periodic box with tin-foil boundary, the reciprocal part
of the electrostatics of point multipoles (charge, dipole, traceless
quadrupole) and its derivatives at the sites.  The structure factor is
  S(m) = sum_j [q_j + 2 pi i m.d_j - (4 pi^2/3) m.Theta_j.m] exp(2 pi i m.r_j)
and the energy E_rec = 1/(2 pi V) sum_{m != 0} exp(-pi^2 m^2/beta^2)/m^2 |S(m)|^2.
The reciprocal potential is
  phi(r) = 1/(pi V) sum_{m != 0} exp(-pi^2 m^2/beta^2)/m^2
           Re[conj(S(m)) exp(2 pi i m.r)],
so that E_rec = 1/2 sum_i [q_i + d_i.grad + 1/3 Theta_i:grad grad] phi(r_i).

SPME (Essmann et al. 1995, the method the paper uses for multipoles and
polarization) replaces exp(2 pi i m.r_j) by cardinal B-spline interpolation
of order p on a K1 x K2 x K3 grid:
  Q(k) = sum_j [q_j W_j(k) + d_j.grad_j W_j(k) + 1/3 Theta_j:grad_j grad_j W_j(k)],
  W_j(k) = prod_a M_p(u_ja - k_a),  u_ja = K_a r_ja / L_a  (wrapped),
  E_rec = 1/2 sum_m G(m) |FFT(Q)(m)|^2,
  G(m) = B(m) C(m), C(m) = exp(-pi^2 m^2/beta^2)/(pi V m^2), C(0) = 0,
  B(m) = prod_a 1/|sum_{k=0}^{p-2} M_p(k+1) exp(2 pi i m_a k/K_a)|^2.
For odd p and even K the sum in B vanishes at the Nyquist index m_a = K_a/2.
Reading taken: a (near-)zero |sum|^2 is replaced by the mean of its two
neighbours before inverting (the weight exp(-pi^2 m^2/beta^2) there is below
1e-6, so the choice is immaterial at the tolerances used, but it is fixed).
The potential grid is phi(k) = sum_m G(m) FFT(Q)(m) exp(2 pi i m.k/K) and
site derivatives are gathered with the derivatives of W_j.
"""
import math

import numpy as np
from scipy.special import comb, factorial


# ---------------------------------------------------------------- k-sum
def cell_volume(box):
    box = np.asarray(box, float)
    return float(abs(np.linalg.det(box))) if box.ndim == 2 else float(np.prod(box))


def kvectors(box, beta, tol=1e-18):
    """Reciprocal vectors m != 0 with exp(-pi^2 m^2/beta^2) >= tol.  box:
    (3,) edges of an orthorhombic cell (m = n / L), or (3,3) lattice vectors
    as rows H (m = n inv(H)^T, so that m.a_k = n_k)."""
    box = np.asarray(box, float)
    # exp(-pi^2 m^2/beta^2) < tol  =>  |m| > beta sqrt(-ln tol)/pi
    mmax = beta * math.sqrt(-math.log(tol)) / math.pi
    # |n_k| = |m.a_k| <= |m| |a_k|
    lengths = np.linalg.norm(box, axis=1) if box.ndim == 2 else box
    na = np.ceil(mmax * lengths).astype(int)
    rng = [np.arange(-n, n + 1) for n in na]
    g = np.stack(np.meshgrid(*rng, indexing="ij"), axis=-1).reshape(-1, 3)
    g = g[np.any(g != 0, axis=1)]
    m = g @ np.linalg.inv(box).T if box.ndim == 2 else g / box
    m2 = np.sum(m * m, axis=1)
    keep = m2 <= mmax * mmax
    return m[keep], m2[keep]


def structure_factor(m, pos, q, d, th):
    phase = np.exp(2j * np.pi * (m @ pos.T))          # (M, n)
    amp = np.zeros(phase.shape, dtype=complex)
    if q is not None:
        amp += q[None, :]
    if d is not None:
        amp += 2j * np.pi * (m @ d.T)
    if th is not None:
        amp += -(4 * np.pi ** 2 / 3.0) * np.einsum("ma,nab,mb->mn", m, th, m)
    return np.sum(amp * phase, axis=1)


def ewald_recip(pos, box, beta, mult, at, nderiv, chunk=2000):
    """Brute-force reciprocal energy and potential derivatives.

    mult = (q, d, th) source multipoles (any may be None); at = evaluation
    positions (k, 3).  Returns (E_rec, [phi, grad phi (k,3), grad^2 (k,3,3),
    grad^3 (k,3,3,3)][:nderiv+1])."""
    V = cell_volume(box)
    m, m2 = kvectors(box, beta)
    q, d, th = mult
    energy = 0.0
    derivs = [np.zeros((len(at),) + (3,) * k) for k in range(nderiv + 1)]
    for s in range(0, len(m), chunk):
        mm = m[s:s + chunk]
        w = np.exp(-np.pi ** 2 * m2[s:s + chunk] / beta ** 2) / m2[s:s + chunk]
        S = structure_factor(mm, pos, q, d, th)
        energy += float(np.sum(w * np.abs(S) ** 2)) / (2 * np.pi * V)
        coef = (w * np.conj(S)) / (np.pi * V)                 # (M,)
        ph = np.exp(2j * np.pi * (at @ mm.T))                 # (k, M)
        base = ph * coef[None, :]
        for k in range(nderiv + 1):
            fac = (2j * np.pi) ** k
            if k == 0:
                derivs[0] += np.real(base.sum(axis=1))
            elif k == 1:
                derivs[1] += np.real(fac * np.einsum("km,ma->ka", base, mm))
            elif k == 2:
                derivs[2] += np.real(fac * np.einsum("km,ma,mb->kab", base, mm, mm))
            else:
                derivs[3] += np.real(fac * np.einsum("km,ma,mb,mc->kabc",
                                                     base, mm, mm, mm))
    return energy, derivs


# ------------------------------------------------------------------ SPME
def bspline(u, order, nd=0):
    """nd-th derivative of the cardinal B-spline M_order at u (explicit
    Schoenberg form: M_n(u) = 1/(n-1)! sum_k (-1)^k C(n,k) (u-k)_+^(n-1))."""
    u = np.asarray(u, float)
    n = order
    deg = n - 1 - nd
    out = np.zeros_like(u)
    if deg < 0:
        return out
    for k in range(n + 1):
        t = np.maximum(u - k, 0.0)
        term = (-1.0) ** k * comb(n, k) * (t ** deg if deg > 0 else (u - k > 0).astype(float))
        out += term
    out /= factorial(deg)
    return out


def _site_weights(pos, box, K, order, nd):
    """Per site and axis: grid indices (n, 3, p) and derivative weights
    dW[a][t] (n, 3, p) of M_p(u - k) with respect to r_a (t-th derivative)."""
    box = np.asarray(box, float)
    K = np.asarray(K, int)
    u = np.mod(pos / box, 1.0) * K
    fl = np.floor(u)
    w = u - fl
    t = np.arange(order)
    idx = (fl[:, :, None].astype(int) - t[None, None, :]) % K[None, :, None]
    arg = w[:, :, None] + t[None, None, :]
    scale = (K / box)[None, :, None]
    vals = [bspline(arg, order, k) * scale ** k for k in range(nd + 1)]
    return idx, vals


def _multi_index(nd_axes):
    """Derivative multi-indices (counts per axis) for a tensor index tuple."""
    cnt = [0, 0, 0]
    for a in nd_axes:
        cnt[a] += 1
    return cnt


def spme_spread(pos, box, K, order, mult):
    q, d, th = mult
    n = len(pos)
    nd = 2 if th is not None else (1 if d is not None else 0)
    idx, vals = _site_weights(pos, box, K, order, nd)
    grid = np.zeros(tuple(K))
    # amplitude of each derivative multi-index, per site
    coeff = {}
    if q is not None:
        coeff[(0, 0, 0)] = coeff.get((0, 0, 0), 0) + q
    if d is not None:
        for a in range(3):
            key = tuple(_multi_index([a]))
            coeff[key] = coeff.get(key, 0) + d[:, a]
    if th is not None:
        for a in range(3):
            for b in range(3):
                key = tuple(_multi_index([a, b]))
                coeff[key] = coeff.get(key, 0) + th[:, a, b] / 3.0
    for key, amp in coeff.items():
        wx = vals[key[0]][:, 0, :]
        wy = vals[key[1]][:, 1, :]
        wz = vals[key[2]][:, 2, :]
        W = amp[:, None, None, None] * wx[:, :, None, None] * \
            wy[:, None, :, None] * wz[:, None, None, :]
        ix = idx[:, 0, :][:, :, None, None]
        iy = idx[:, 1, :][:, None, :, None]
        iz = idx[:, 2, :][:, None, None, :]
        ix, iy, iz = np.broadcast_arrays(ix, iy, iz)
        np.add.at(grid, (ix.ravel(), iy.ravel(), iz.ravel()), W.ravel())
    del n
    return grid


def bspline_moduli(K, order):
    """|sum_{k=0}^{p-2} M_p(k+1) exp(2 pi i m k/K)|^2 for m = 0..K-1, with
    (near-)zero entries replaced by the mean of their neighbours."""
    k = np.arange(order - 1)
    Mk = bspline(k + 1.0, order)
    m = np.arange(K)
    s = np.exp(2j * np.pi * np.outer(m, k) / K) @ Mk
    mod = np.abs(s) ** 2
    for i in range(K):
        if mod[i] < 1e-7:
            mod[i] = 0.5 * (mod[(i - 1) % K] + mod[(i + 1) % K])
    return mod


def spme_influence(box, K, order, beta):
    box = np.asarray(box, float)
    K = np.asarray(K, int)
    V = float(np.prod(box))
    freqs = [np.fft.fftfreq(K[a], d=1.0 / K[a]) / box[a] for a in range(3)]
    mx, my, mz = np.meshgrid(*freqs, indexing="ij")
    m2 = mx ** 2 + my ** 2 + mz ** 2
    mods = [bspline_moduli(K[a], order) for a in range(3)]
    Bm = 1.0 / (mods[0][:, None, None] * mods[1][None, :, None] * mods[2][None, None, :])
    with np.errstate(divide="ignore", invalid="ignore"):
        C = np.exp(-np.pi ** 2 * m2 / beta ** 2) / (np.pi * V * m2)
    C[0, 0, 0] = 0.0
    return Bm * C


def spme_potential(grid, G):
    """E_rec and the potential grid phi(k)."""
    F = np.fft.fftn(grid)
    energy = 0.5 * float(np.sum(G * np.abs(F) ** 2))
    phi = np.real(np.fft.ifftn(G * F)) * grid.size
    return energy, phi


def spme_gather(pos, box, K, order, phi, nderiv):
    """[phi, grad, grad^2, grad^3][:nderiv+1] of the interpolated potential
    at each site (derivatives with respect to the site position)."""
    idx, vals = _site_weights(pos, box, K, order, nderiv)
    n = len(pos)
    ix = idx[:, 0, :][:, :, None, None]
    iy = idx[:, 1, :][:, None, :, None]
    iz = idx[:, 2, :][:, None, None, :]
    local = phi[ix, iy, iz]                                   # (n,p,p,p)
    out = [np.zeros((n,) + (3,) * k) for k in range(nderiv + 1)]
    import itertools
    for k in range(nderiv + 1):
        for axes in itertools.product(range(3), repeat=k):
            cnt = _multi_index(axes)
            wx = vals[cnt[0]][:, 0, :]
            wy = vals[cnt[1]][:, 1, :]
            wz = vals[cnt[2]][:, 2, :]
            v = np.einsum("nxyz,nx,ny,nz->n", local, wx, wy, wz)
            out[k][(slice(None),) + axes] = v
    return out


# ---------------------------------------------------------------- virial
# W_ab = -dE_rec/d eps_ab under the homogeneous strain r -> (1 + eps) r of
# every site and of the cell, with the multipoles fixed in the global
# frame.  Fractional coordinates are unchanged, reciprocal vectors go to
# (1 + eps)^-T m (dm_c/d eps_ab = -delta_cb m_a), V to (1 + tr eps) V, and
# the amplitude 2 pi i m.d - (4 pi^2/3) m.Theta.m of each site follows m.
# Differentiating E_rec = 1/(2 pi V) sum_m f(m^2) |S(m)|^2,
# f = exp(-pi^2 m^2/beta^2)/m^2, term by term:
#   volume      -delta_ab E_rec
#   f(m^2)      sum_m C(m) (pi^2/beta^2 + 1/m^2) m_a m_b |S(m)|^2,
#               C = f/(pi V) (twice the energy weight)
#   amplitudes  -sum_j [d_jb d_a phi(r_j) + 2/3 Theta_jbc d_a d_c phi(r_j)]
# so W_ab = delta_ab E_rec - (m-space sum) + sum_j [d_jb d_a phi_j
#           + 2/3 Theta_jbc d_a d_c phi_j].
# For SPME the same steps hold exactly for the interpolated energy: the
# B-spline weights depend only on fractional coordinates, and the dipole
# and quadrupole spread terms carry the Cartesian gradient, which strains
# as the amplitudes above; C(m) becomes G(m) = B(m) C(m) on the grid.
def _site_virial(mult, derivs):
    q, d, th = mult
    W = np.zeros((3, 3))
    if d is not None:
        W += np.einsum("jb,ja->ab", d, derivs[1])
    if th is not None:
        W += (2.0 / 3.0) * np.einsum("jbc,jac->ab", th, derivs[2])
    return W


def ewald_recip_virial(pos, box, beta, mult, chunk=2000):
    """Brute-force reciprocal energy and its virial (3,3) (e^2/A units)."""
    V = cell_volume(box)
    m, m2 = kvectors(box, beta)
    q, d, th = mult
    nd = 2 if th is not None else 1
    energy, derivs = ewald_recip(pos, box, beta, mult, pos, nd, chunk)
    W = energy * np.eye(3) + _site_virial(mult, derivs)
    for s in range(0, len(m), chunk):
        mm = m[s:s + chunk]
        mm2 = m2[s:s + chunk]
        C = np.exp(-np.pi ** 2 * mm2 / beta ** 2) / mm2 / (np.pi * V)
        S = structure_factor(mm, pos, q, d, th)
        wgt = C * (np.pi ** 2 / beta ** 2 + 1.0 / mm2) * np.abs(S) ** 2
        W -= np.einsum("m,ma,mb->ab", wgt, mm, mm)
    return energy, W


def spme_virial(pos, box, K, order, beta, mult):
    """SPME reciprocal energy and its virial (3,3), orthorhombic cell."""
    box = np.asarray(box, float)
    K = np.asarray(K, int)
    q, d, th = mult
    grid = spme_spread(pos, box, K, order, mult)
    G = spme_influence(box, K, order, beta)
    energy, phi = spme_potential(grid, G)
    nd = 2 if th is not None else 1
    derivs = spme_gather(pos, box, K, order, phi, nd)
    F = np.fft.fftn(grid)
    freqs = [np.fft.fftfreq(K[a], d=1.0 / K[a]) / box[a] for a in range(3)]
    m = np.stack(np.meshgrid(*freqs, indexing="ij"), axis=-1)
    m2 = np.sum(m * m, axis=-1)
    with np.errstate(divide="ignore", invalid="ignore"):
        wgt = G * (np.pi ** 2 / beta ** 2 + 1.0 / m2) * np.abs(F) ** 2
    wgt[0, 0, 0] = 0.0
    W = energy * np.eye(3) + _site_virial(mult, derivs)
    W -= np.einsum("xyz,xyza,xyzb->ab", wgt, m, m)
    return energy, W
