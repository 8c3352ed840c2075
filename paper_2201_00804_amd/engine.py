"""Python binding of the C-ABI with torch tensors for device memory and the
current torch stream.  Every computation runs in the HIP library; this
module only checks shapes/dtypes and passes pointers.
"""
import ctypes

import torch

from . import _lib


class SibfaError(RuntimeError):
    def __init__(self, status, message):
        self.status = status
        super().__init__(f"{_lib.STATUS_NAMES.get(status, status)}: {message}")


def default_params(**kw):
    lib = _lib.load()
    p = _lib.Params()
    lib.sibfa_default_params(ctypes.byref(p))
    for k, v in kw.items():
        if k == "grid":
            g = (v, v, v) if isinstance(v, int) else tuple(v)
            p.grid[0], p.grid[1], p.grid[2] = g
        elif k == "precision":
            p.precision = {"fp64": _lib.FP64, "mixed": _lib.MIXED}.get(v, v)
        elif k == "precond":
            p.precond = {"diag": _lib.PRECOND_DIAG, "molblock": _lib.PRECOND_MOLBLOCK}.get(v, v)
        elif k == "beta":
            p.ewald_beta = v
        elif k == "tol":
            p.tol_debye = v
        else:
            setattr(p, k, v)
    return p


def footprint_bytes(n_sites, n_polarizable, box, params):
    lib = _lib.load()
    b = None if box is None else (ctypes.c_double * 3)(*[float(x) for x in box])
    return int(lib.sibfa_footprint_bytes(int(n_sites), int(n_polarizable), b, ctypes.byref(params)))


def _dev(t, dtype, shape, device, name):
    if t is None:
        return None
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if t.dtype != dtype or t.device != device or not t.is_contiguous():
        raise ValueError(f"{name} must be a contiguous {dtype} tensor on {device}")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")
    return t


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


class TorchAllocator:
    """Device memory for the library from torch's caching allocator: the
    alloc/free callbacks of sibfa_create and sibfa_batch_create.  Blocks
    are taken on the stream the library enqueues on."""

    def __init__(self, device, stream):
        self.device = int(device)
        self.stream = stream

        def _alloc(nbytes, user):
            try:
                return int(torch.cuda.caching_allocator_alloc(int(nbytes), self.device,
                                                              self.stream))
            except RuntimeError:   # out of memory: the library reports E_NOMEM
                return None

        def _free(ptr, user):
            try:
                torch.cuda.caching_allocator_delete(int(ptr))
            except Exception:   # interpreter shutdown: torch is gone already
                pass

        # the ctypes callback objects must outlive the library's use of them
        self.alloc_fn = _lib.ALLOC_FN(_alloc)
        self.free_fn = _lib.FREE_FN(_free)


def _callbacks(allocator):
    """The alloc/free arguments of the create calls: the allocator's, or
    null function pointers (the library then calls hipMalloc)."""
    if allocator is None:
        return _lib.ALLOC_FN(), _lib.FREE_FN()
    return allocator.alloc_fn, allocator.free_fn


class Engine:
    """One system (box or cluster) resident on one device.  Device memory
    comes from torch's caching allocator (torch_memory=False: the library
    calls hipMalloc itself)."""

    def __init__(self, device=0, stream=None, torch_memory=True):
        self.lib = _lib.load()
        self.device = torch.device("cuda", device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.allocator = TorchAllocator(device, self.stream) if torch_memory else None
        af, ff = _callbacks(self.allocator)
        h = ctypes.c_void_p()
        st = self.lib.sibfa_create(ctypes.byref(h), int(device),
                                   ctypes.c_void_p(self.stream.cuda_stream), af, ff, None)
        if st != 0:
            raise SibfaError(st, "sibfa_create failed")
        self.h = h
        self.n = 0

    def close(self):
        if getattr(self, "h", None):
            self.lib.sibfa_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, st):
        if st != 0:
            raise SibfaError(st, self.lib.sibfa_last_error(self.h).decode())

    # -- setup ------------------------------------------------------------
    def set_system(self, pos, mol, box, params):
        n = pos.shape[0]
        _dev(pos, torch.float64, (n, 3), self.device, "pos")
        _dev(mol, torch.int32, (n,), self.device, "mol")
        b = None if box is None else (ctypes.c_double * 3)(*[float(x) for x in box])
        self.params = params
        self._check(self.lib.sibfa_set_system(self.h, n, _ptr(pos), _ptr(mol), b,
                                              ctypes.byref(params)))
        self.n = n

    def update_positions(self, pos):
        _dev(pos, torch.float64, (self.n, 3), self.device, "pos")
        self._check(self.lib.sibfa_update_positions(self.h, _ptr(pos)))

    def set_multipoles(self, q, dip=None, quad=None):
        _dev(q, torch.float64, (self.n,), self.device, "q")
        _dev(dip, torch.float64, (self.n, 3), self.device, "dip")
        _dev(quad, torch.float64, (self.n, 6), self.device, "quad")
        self._check(self.lib.sibfa_set_multipoles(self.h, _ptr(q), _ptr(dip), _ptr(quad)))

    def set_polarizabilities(self, alpha, thole=None):
        _dev(alpha, torch.float64, (self.n, 6), self.device, "alpha")
        _dev(thole, torch.float64, (self.n,), self.device, "thole")
        self._check(self.lib.sibfa_set_polarizabilities(self.h, _ptr(alpha), _ptr(thole)))

    def set_local_frames(self, frames, dip_local=None, quad_local=None, alpha_local=None):
        """Frames [n][3] (int32 site indices, -1 rows: none) and the local
        dipoles, quadrupoles and polarizabilities they carry; frames=None
        switches local frames off."""
        if frames is None:
            self._check(self.lib.sibfa_set_local_frames(self.h, None, None, None, None))
            return
        _dev(frames, torch.int32, (self.n, 3), self.device, "frames")
        _dev(dip_local, torch.float64, (self.n, 3), self.device, "dip_local")
        _dev(quad_local, torch.float64, (self.n, 6), self.device, "quad_local")
        _dev(alpha_local, torch.float64, (self.n, 6), self.device, "alpha_local")
        self._check(self.lib.sibfa_set_local_frames(self.h, _ptr(frames), _ptr(dip_local),
                                                    _ptr(quad_local), _ptr(alpha_local)))

    def load(self, sysd, params):
        """Convenience: system dict (numpy arrays as produced by synth)."""
        dev = self.device
        t = lambda a, dt=torch.float64: torch.as_tensor(a, dtype=dt, device=dev).contiguous()
        self.set_system(t(sysd["pos"]), t(sysd["mol"], torch.int32), sysd.get("box"), params)
        self.set_multipoles(t(sysd["q"]), t(sysd["dip"]), t(sysd["quad"]))
        self.set_polarizabilities(t(sysd["alpha"]),
                                  None if sysd.get("thole") is None else t(sysd["thole"]))

    # -- compute ----------------------------------------------------------
    def permanent_field(self):
        out = torch.empty((self.n, 3), dtype=torch.float64, device=self.device)
        self._check(self.lib.sibfa_permanent_field(self.h, _ptr(out)))
        return out

    def apply_T(self, p):
        _dev(p, torch.float64, (self.n, 3), self.device, "p")
        out = torch.empty((self.n, 3), dtype=torch.float64, device=self.device)
        self._check(self.lib.sibfa_apply_T(self.h, _ptr(p), _ptr(out)))
        return out

    def solve(self, warm_start=False):
        mu = torch.empty((self.n, 3), dtype=torch.float64, device=self.device)
        it = ctypes.c_int(0)
        rms = ctypes.c_double(0.0)
        self._check(self.lib.sibfa_solve_induced(self.h, int(bool(warm_start)), _ptr(mu),
                                                 ctypes.byref(it), ctypes.byref(rms)))
        return mu, it.value, rms.value

    def solve_tcg(self, order, omega=0.0, warm_start=False, mu_out=True):
        """TCG-n dipoles (or None) and E_pol at them (kcal/mol)."""
        mu = None
        if mu_out:
            mu = torch.empty((self.n, 3), dtype=torch.float64, device=self.device)
        e = ctypes.c_double(0.0)
        self._check(self.lib.sibfa_solve_tcg(self.h, int(order), float(omega),
                                             int(bool(warm_start)), _ptr(mu), ctypes.byref(e)))
        return mu, e.value

    def tcg_energy_forces(self, order, omega=0.0, warm_start=False, forces=True, mu_out=False):
        """(E_pol, E_elec, forces or None, mu or None) at TCG-n dipoles, with
        the forces of the truncated iteration (FP64)."""
        e_pol = ctypes.c_double(0.0)
        e_elec = ctypes.c_double(0.0)
        f = torch.empty((self.n, 3), dtype=torch.float64, device=self.device) if forces else None
        mu = torch.empty((self.n, 3), dtype=torch.float64, device=self.device) if mu_out else None
        self._check(self.lib.sibfa_tcg_energy_forces(self.h, int(order), float(omega),
                                                     int(bool(warm_start)), ctypes.byref(e_pol),
                                                     ctypes.byref(e_elec), _ptr(f), _ptr(mu)))
        return e_pol.value, e_elec.value, f, mu

    def energy_forces(self, forces=True, out=None, virial=False):
        """(E_pol, E_elec, forces or None), plus the 3x3 virial (a host
        list of rows, kcal/mol) as a fourth item when virial is true."""
        e_pol = ctypes.c_double(0.0)
        e_elec = ctypes.c_double(0.0)
        f = None
        if forces:
            f = out if out is not None else torch.empty((self.n, 3), dtype=torch.float64,
                                                        device=self.device)
            _dev(f, torch.float64, (self.n, 3), self.device, "forces")
        w = (ctypes.c_double * 9)() if virial else None
        self._check(self.lib.sibfa_energy_forces(self.h, ctypes.byref(e_pol), ctypes.byref(e_elec),
                                                 _ptr(f), w))
        if virial:
            return e_pol.value, e_elec.value, f, [[w[3 * a + b] for b in range(3)]
                                                  for a in range(3)]
        return e_pol.value, e_elec.value, f

    def get_dipoles(self):
        mu = torch.empty((self.n, 3), dtype=torch.float64, device=self.device)
        self._check(self.lib.sibfa_get_dipoles(self.h, _ptr(mu)))
        return mu

    def set_dipoles(self, mu):
        _dev(mu, torch.float64, (self.n, 3), self.device, "mu")
        self._check(self.lib.sibfa_set_dipoles(self.h, _ptr(mu)))

    def set_predictor(self, order):
        """Warm starts from the polynomial extrapolation of the last `order`
        dipole sets (0 or 1: the last set)."""
        self._check(self.lib.sibfa_set_predictor(self.h, int(order)))

    # -- reduced charge transfer ------------------------------------------
    def set_charge_transfer(self, lp, lp_par, acc, acc_ah, rvdw, eta, cs, cp, t, m):
        """lp [n_lp][2] (lone-pair site, carrier), lp_par [n_lp][2]
        (occupation, ionization energy), acc [n_acc][2] (a1 = H, a2),
        acc_ah [n_acc], rvdw [n]: device tensors; the constants as floats."""
        nl = lp.shape[0]
        na = acc.shape[0]
        _dev(lp, torch.int32, (nl, 2), self.device, "lp")
        _dev(lp_par, torch.float64, (nl, 2), self.device, "lp_par")
        _dev(acc, torch.int32, (na, 2), self.device, "acc")
        _dev(acc_ah, torch.float64, (na,), self.device, "acc_ah")
        _dev(rvdw, torch.float64, (self.n,), self.device, "rvdw")
        prm = _lib.CtParams(float(eta), float(cs), float(cp), float(t), float(m))
        self._check(self.lib.sibfa_set_charge_transfer(self.h, nl, _ptr(lp), _ptr(lp_par), na,
                                                       _ptr(acc), _ptr(acc_ah), _ptr(rvdw),
                                                       ctypes.byref(prm)))

    def ct_energy_forces(self, forces=True):
        """(E_ct kcal/mol, forces [n][3] or None)."""
        e = ctypes.c_double(0.0)
        f = torch.empty((self.n, 3), dtype=torch.float64, device=self.device) if forces else None
        self._check(self.lib.sibfa_ct_energy_forces(self.h, ctypes.byref(e), _ptr(f)))
        return e.value, f

    # -- dynamics (Beeman) ------------------------------------------------
    def md_init(self, masses, vsites=None, bonds=None, bond_k=None, bond_r0=None,
                rep_radius=None, rep_eps=0.0, vel=None):
        _dev(masses, torch.float64, (self.n,), self.device, "masses")
        _dev(rep_radius, torch.float64, (self.n,), self.device, "rep_radius")
        _dev(vsites, torch.int32, (self.n, 2), self.device, "vsites")
        nb = 0 if bonds is None else bonds.shape[0]
        _dev(bonds, torch.int32, (nb, 2), self.device, "bonds")
        _dev(bond_k, torch.float64, (nb,), self.device, "bond_k")
        _dev(bond_r0, torch.float64, (nb,), self.device, "bond_r0")
        _dev(vel, torch.float64, (self.n, 3), self.device, "vel")
        self._check(self.lib.sibfa_md_init(self.h, _ptr(masses), _ptr(vsites), nb, _ptr(bonds),
                                           _ptr(bond_k), _ptr(bond_r0), _ptr(rep_radius),
                                           float(rep_eps), _ptr(vel)))

    def md_run(self, n_steps, dt_fs=1.0, friction=0.0):
        """Per-step records (E_pol, E_elec, E_bond, E_rep, E_kin, iterations);
        friction > 0 damps the velocities (a relaxation)."""
        st = (_lib.MdStats * max(int(n_steps), 1))()
        self._check(self.lib.sibfa_md_run(self.h, int(n_steps), float(dt_fs), float(friction),
                                          st))
        return [(r.e_pol, r.e_elec, r.e_bond, r.e_rep, r.e_kin, r.iterations)
                for r in list(st)[:int(n_steps)]]

    def md_state(self):
        x = torch.empty((self.n, 3), dtype=torch.float64, device=self.device)
        v = torch.empty_like(x)
        self._check(self.lib.sibfa_md_get_state(self.h, _ptr(x), _ptr(v)))
        return x, v

    def neighbor_counts(self):
        out = torch.empty((self.n,), dtype=torch.int32, device=self.device)
        self._check(self.lib.sibfa_neighbor_counts(self.h, _ptr(out)))
        return out

    def set_profiling(self, enable=True, phases=None):
        """Time every phase (or only the named ones) with HIP events."""
        if phases is None or not enable:
            self._check(self.lib.sibfa_set_profiling(self.h, int(bool(enable))))
        else:
            mask = 0
            for name in phases:
                mask |= 1 << _lib.PHASES.index(name)
            self._check(self.lib.sibfa_set_profiling_phases(self.h, mask))

    def profile(self):
        """Accumulated per-phase event times (ms), launch groups and list sizes."""
        pr = _lib.Profile()
        self._check(self.lib.sibfa_get_profile(self.h, ctypes.byref(pr)))
        return {"ms": {name: pr.ms[k] for k, name in enumerate(_lib.PHASES)},
                "calls": {name: pr.calls[k] for k, name in enumerate(_lib.PHASES)},
                "pairs": {"all": pr.pairs[0], "same_molecule": pr.pairs[1],
                          "pol": pr.pairs[2], "pol_same_molecule": pr.pairs[3]}}

    def stats(self):
        s = _lib.Stats()
        self._check(self.lib.sibfa_get_stats(self.h, ctypes.byref(s)))
        return {name: getattr(s, name) for name, _ in s._fields_}
