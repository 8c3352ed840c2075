"""Python binding of the batched-cluster executor (sibfa_batch_*): many
independent gas-phase clusters evaluated in one call, one workgroup per
cluster.  Only marshalling happens here; the work runs in the HIP library.
"""
import ctypes

import torch

from . import _lib
from .engine import SibfaError, TorchAllocator, _callbacks, _dev, _ptr

MAX_SITES = _lib.BATCH_MAX_SITES
MAX_POLARIZABLE = _lib.BATCH_MAX_POLARIZABLE


class BatchResult:
    """Device outputs of one batch; valid once `event` has completed."""

    def __init__(self, offsets, mu, forces, e_pol, e_elec, iters, rms, status, event):
        self.offsets = offsets
        self.mu = mu
        self.forces = forces
        self.e_pol = e_pol
        self.e_elec = e_elec
        self.iters = iters
        self.rms = rms
        self.status = status
        self.event = event

    def ready(self):
        return self.event.query()

    def wait(self):
        self.event.synchronize()

    def cluster(self, c):
        """Host copies of cluster c's results (synchronizes)."""
        self.wait()
        a, b = self.offsets[c], self.offsets[c + 1]
        return dict(mu=self.mu[a:b].cpu(), forces=None if self.forces is None else self.forces[a:b].cpu(),
                    e_pol=float(self.e_pol[c]), e_elec=float(self.e_elec[c]),
                    iterations=int(self.iters[c]), rms_debye=float(self.rms[c]),
                    status=int(self.status[c]))


class ClusterBatch:
    """Batch executor bound to one device and stream."""

    def __init__(self, device=0, stream=None, torch_memory=True):
        self.lib = _lib.load()
        self.device = torch.device("cuda", device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.allocator = TorchAllocator(device, self.stream) if torch_memory else None
        af, ff = _callbacks(self.allocator)
        h = ctypes.c_void_p()
        st = self.lib.sibfa_batch_create(ctypes.byref(h), int(device),
                                         ctypes.c_void_p(self.stream.cuda_stream), af, ff, None)
        if st != 0:
            raise SibfaError(st, "sibfa_batch_create failed")
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            self.lib.sibfa_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def run(self, offsets, xyz, mol, q, dip, quad, alpha, params, thole=None, warm=None,
            mu=None, forces=True):
        """Enqueue one batch.  offsets: host sequence [n_clusters + 1];
        arrays: device tensors of the concatenated clusters; warm: host
        sequence of flags (mu must then hold the starting dipoles)."""
        offsets = [int(x) for x in offsets]
        nc = len(offsets) - 1
        n = offsets[-1]
        dev = self.device
        for name, t, dt, shape in (("xyz", xyz, torch.float64, (n, 3)),
                                   ("mol", mol, torch.int32, (n,)),
                                   ("q", q, torch.float64, (n,)),
                                   ("dip", dip, torch.float64, (n, 3)),
                                   ("quad", quad, torch.float64, (n, 6)),
                                   ("alpha", alpha, torch.float64, (n, 6)),
                                   ("thole", thole, torch.float64, (n,))):
            _dev(t, dt, shape, dev, name)
        if mu is None:
            mu = torch.zeros((n, 3), dtype=torch.float64, device=dev)
        _dev(mu, torch.float64, (n, 3), dev, "mu")
        f = torch.empty((n, 3), dtype=torch.float64, device=dev) if forces else None
        e_pol = torch.empty(nc, dtype=torch.float64, device=dev)
        e_elec = torch.empty(nc, dtype=torch.float64, device=dev)
        iters = torch.empty(nc, dtype=torch.int32, device=dev)
        rms = torch.empty(nc, dtype=torch.float64, device=dev)
        status = torch.empty(nc, dtype=torch.int32, device=dev)
        off_c = (ctypes.c_int * (nc + 1))(*offsets)
        warm_c = None if warm is None else (ctypes.c_int * nc)(*[int(bool(w)) for w in warm])
        st = self.lib.sibfa_batch_clusters(
            self.h, nc, off_c, warm_c, _ptr(xyz), _ptr(mol), _ptr(q), _ptr(dip), _ptr(quad),
            _ptr(alpha), _ptr(thole), ctypes.byref(params), _ptr(mu), _ptr(f), _ptr(e_pol),
            _ptr(e_elec), _ptr(iters), _ptr(rms), _ptr(status))
        if st != 0:
            raise SibfaError(st, self.lib.sibfa_batch_last_error(self.h).decode())
        ev = torch.cuda.Event()
        ev.record(self.stream)
        return BatchResult(offsets, mu, f, e_pol, e_elec, iters, rms, status, ev)


def concat_clusters(systems, device):
    """Concatenate synth-style cluster dicts into device tensors; returns
    (offsets, tensors dict)."""
    import numpy as np
    offsets = [0]
    for s in systems:
        offsets.append(offsets[-1] + len(s["pos"]))
    cat = lambda k: np.concatenate([s[k] for s in systems])
    t = lambda a, dt=torch.float64: torch.as_tensor(a, dtype=dt, device=device).contiguous()
    mols = np.concatenate([s["mol"] for s in systems]).astype(np.int32)
    return offsets, dict(xyz=t(cat("pos")), mol=t(mols, torch.int32), q=t(cat("q")),
                         dip=t(cat("dip")), quad=t(cat("quad")), alpha=t(cat("alpha")))
