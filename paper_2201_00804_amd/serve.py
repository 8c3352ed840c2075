"""Request-level serving of polarization evaluations on one GPU.

A request names a system (a gas-phase cluster or a periodic box) and its
current positions; the answer is E_pol, E_elec and the forces at the
converged induced dipoles.  The server keeps work resident on the device:

  * periodic boxes run on resident contexts (one per system, each on its
    own stream).  A new box is admitted only if its device footprint
    (sibfa_footprint_bytes) fits the HBM budget next to the resident ones;
    least-recently-used contexts are evicted to make room, and a system
    larger than the whole budget is rejected.  A repeat of a resident
    system (new positions, e.g. the next MD step) updates positions and
    warm-starts the solve from its previous dipoles;
  * several box requests are in flight at once: box_slots worker threads
    each take the oldest queued box request whose system is not already in
    flight (requests of one system stay in arrival order), so the solves of
    different boxes overlap on the device, each on its context's streams;
  * clusters are gathered into batches: every cluster pending when the
    cluster worker becomes free goes into one sibfa_batch_clusters call
    (three launches for the whole batch), warm-started from the dipoles of
    the system's previous request when there was one.  A cluster system's
    multipoles, polarizabilities and last dipoles stay on the device; a
    request brings only its positions.

The box workers and the cluster worker run concurrently on separate
streams; the request clock starts at the request's arrival and stops when
its energies and forces are in host memory.
"""
import collections
import math
import threading
import time

import numpy as np
import torch

from . import engine as _engine
from .batch import ClusterBatch, MAX_SITES


class Request:
    __slots__ = ("rid", "system", "kind", "pos", "arrival", "start", "done", "e_pol", "e_elec",
                 "forces", "iterations", "status", "warm", "batch_size")

    def __init__(self, rid, system, kind, pos, arrival):
        self.rid = rid
        self.system = system
        self.kind = kind
        self.pos = pos
        self.arrival = arrival
        self.start = self.done = None
        self.e_pol = self.e_elec = None
        self.forces = None
        self.iterations = None
        self.status = None
        self.warm = False
        self.batch_size = 1


class _Resident:
    __slots__ = ("engine", "stream", "footprint", "has_mu")


class Server:
    """systems: dict name -> synth-style system dict (pos, mol, q, dip, quad,
    alpha, box or None) plus, for boxes, 'params' (beta, cutoff, grid)."""

    def __init__(self, systems, device=0, precision="mixed", tol=1e-8, hbm_budget=None,
                 max_batch_sites=1 << 18, max_iter=400, box_slots=3, precond="diag"):
        self.systems = systems
        self.dev = torch.device("cuda", device)
        self.precision = precision
        self.precond = precond        # box contexts' PCG preconditioner
        self.tol = tol
        self.max_iter = max_iter
        if hbm_budget is None:
            free, _ = torch.cuda.mem_get_info(self.dev)
            hbm_budget = int(0.5 * free)
        self.budget = int(hbm_budget)
        self.max_batch_sites = max_batch_sites
        self.box_slots = max(1, int(box_slots))
        self.resident = collections.OrderedDict()   # name -> _Resident (LRU order)
        self.resident_bytes = 0
        self.evictions = 0
        self.rejections = 0
        self.inflight = set()                       # box systems being evaluated
        self.box_spans = []                         # (start, done) of box requests
        self._admit_lock = threading.Lock()
        self.cl_static = {}                         # name -> device arrays of a cluster
        self.cluster_mu = {}                        # name -> device mu of the last request
        self.cl_stream = torch.cuda.Stream(self.dev)
        self.batcher = ClusterBatch(device, stream=self.cl_stream)
        self.cl_params = _engine.default_params(tol=tol, precision=precision, max_iter=max_iter)
        self._box_q = collections.deque()
        self._cl_q = collections.deque()
        self._cv = threading.Condition()
        self._stop = False
        self.busy = {"box": 0.0, "cluster": 0.0}
        self.batches = []
        self.errors = []

    # ----------------------------------------------------------- admission
    def _box_params(self, sysd):
        p = sysd["params"]
        return _engine.default_params(beta=p["beta"], cutoff=p["cutoff"], grid=p["grid"],
                                      order=p.get("order", 5), tol=self.tol,
                                      precision=self.precision, max_iter=self.max_iter,
                                      precond=self.precond)

    def _admit(self, name):
        """Resident context of a box system, creating it (and evicting
        least-recently-used contexts that are not in flight) if needed; None
        if it can never fit.  Waits while the contexts in flight hold the
        memory it needs."""
        while True:
            with self._admit_lock:
                r = self._admit_now(name)
            if r is not False:
                return r
            with self._cv:   # a box in flight finishes and notifies
                self._cv.wait(timeout=0.01)

    def _admit_now(self, name):
        if name in self.resident:
            self.resident.move_to_end(name)
            return self.resident[name]
        sysd = self.systems[name]
        prm = self._box_params(sysd)
        n = len(sysd["pos"])
        npol = int(np.count_nonzero(np.any(sysd["alpha"] != 0, axis=1)))
        fp = _engine.footprint_bytes(n, npol, sysd["box"], prm)
        if fp > self.budget:
            self.rejections += 1
            return None
        while self.resident_bytes + fp > self.budget:
            idle = [k for k in self.resident if k not in self.inflight]
            if not idle:
                return False          # only contexts in flight: wait for one
            r = self.resident.pop(idle[0])
            r.stream.synchronize()
            r.engine.close()
            self.resident_bytes -= r.footprint
            self.evictions += 1
        r = _Resident()
        r.stream = torch.cuda.Stream(self.dev)
        r.engine = _engine.Engine(self.dev.index, stream=r.stream)
        with torch.cuda.stream(r.stream):
            r.engine.load(sysd, prm)
        r.footprint = fp
        r.has_mu = False
        self.resident[name] = r
        self.resident_bytes += fp
        return r

    # ------------------------------------------------------------- workers
    def _run_box(self, req):
        r = self._admit(req.system)
        if r is None:
            req.status = "rejected"
            return
        with torch.cuda.stream(r.stream):
            pos = torch.as_tensor(req.pos, dtype=torch.float64, device=self.dev)
            r.engine.update_positions(pos)
            req.warm = r.has_mu
            try:
                _, it, _ = r.engine.solve(warm_start=r.has_mu)
                e_pol, e_elec, F = r.engine.energy_forces()
                req.forces = F.cpu().numpy()
                req.status = 0
            except _engine.SibfaError as e:
                it, e_pol, e_elec = -1, math.nan, math.nan
                req.status = e.status
        r.has_mu = req.status == 0
        req.iterations, req.e_pol, req.e_elec = it, e_pol, e_elec

    def _static(self, name):
        """Device arrays of a cluster system, uploaded on its first request."""
        s = self.cl_static.get(name)
        if s is None:
            d = self.systems[name]
            t = lambda a, dt=torch.float64: torch.as_tensor(a, dtype=dt, device=self.dev)
            s = dict(mol=t(np.asarray(d["mol"]).astype(np.int32), torch.int32), q=t(d["q"]),
                     dip=t(d["dip"]), quad=t(d["quad"]), alpha=t(d["alpha"]))
            self.cl_static[name] = s
        return s

    def _run_clusters(self, reqs):
        offsets = [0]
        for q in reqs:
            offsets.append(offsets[-1] + len(q.pos))
        warm = [q.system in self.cluster_mu for q in reqs]
        with torch.cuda.stream(self.cl_stream):
            # only the positions come from the host; the rest of the batch is
            # laid out from device-resident arrays
            st_ = [self._static(q.system) for q in reqs]
            cat = lambda key: torch.cat([s[key] for s in st_])
            xyz = torch.as_tensor(np.concatenate([q.pos for q in reqs]), dtype=torch.float64,
                                  device=self.dev)
            mu0 = torch.cat([self.cluster_mu[q.system] if w else
                             torch.zeros((len(q.pos), 3), dtype=torch.float64, device=self.dev)
                             for q, w in zip(reqs, warm)])
            res = self.batcher.run(offsets, xyz, cat("mol"), cat("q"), cat("dip"), cat("quad"),
                                   cat("alpha"), self.cl_params, warm=warm, mu=mu0)
            F = res.forces.cpu().numpy()
            e_pol = res.e_pol.cpu().numpy()
            e_elec = res.e_elec.cpu().numpy()
            its = res.iters.cpu().numpy()
            st = res.status.cpu().numpy()
            for c, q in enumerate(reqs):
                if st[c] == 0:   # the dipoles stay on the device for the next request
                    self.cluster_mu[q.system] = res.mu[offsets[c]:offsets[c + 1]].clone()
        for c, q in enumerate(reqs):
            a, b = offsets[c], offsets[c + 1]
            q.forces = F[a:b]
            q.e_pol, q.e_elec = float(e_pol[c]), float(e_elec[c])
            q.iterations, q.status = int(its[c]), int(st[c])
            q.warm = warm[c]
            q.batch_size = len(reqs)
        self.batches.append((len(reqs), offsets[-1]))

    def _next_box(self):
        """The oldest queued box request whose system is not in flight
        (called with the condition held), or None."""
        for k, q in enumerate(self._box_q):
            if q.system not in self.inflight:
                del self._box_q[k]
                self.inflight.add(q.system)
                return q
        return None

    def _box_worker(self):
        while True:
            with self._cv:
                req = self._next_box()
                while req is None and not (self._stop and not self._box_q):
                    self._cv.wait()
                    req = self._next_box()
                if req is None:
                    return
            t0 = time.perf_counter()
            req.start = t0
            try:
                self._run_box(req)
            except Exception as e:   # surfaced to the caller after the run
                self.errors.append(repr(e))
                req.status = "error"
            req.done = time.perf_counter()
            with self._cv:
                self.inflight.discard(req.system)
                self.busy["box"] += req.done - t0
                self.box_spans.append((t0, req.done))
                self._cv.notify_all()

    def _cluster_worker(self):
        while True:
            with self._cv:
                while not self._cl_q and not self._stop:
                    self._cv.wait()
                if not self._cl_q:
                    return
                reqs, sites = [], 0
                while self._cl_q and sites + len(self._cl_q[0].pos) <= self.max_batch_sites:
                    q = self._cl_q.popleft()
                    reqs.append(q)
                    sites += len(q.pos)
            t0 = time.perf_counter()
            for q in reqs:
                q.start = t0
            try:
                self._run_clusters(reqs)
            except Exception as e:
                self.errors.append(repr(e))
                for q in reqs:
                    q.status = "error"
            t1 = time.perf_counter()
            for q in reqs:
                q.done = t1
            self.busy["cluster"] += t1 - t0

    # ----------------------------------------------------------------- run
    def run(self, requests):
        """Serve requests whose .arrival are offsets in seconds from now
        (open loop: arrivals do not wait for completions).  Returns the
        wall time of the run."""
        for q in requests:
            if q.kind == "cluster" and len(q.pos) > MAX_SITES:
                raise ValueError("cluster larger than the batch limit; serve it as a box-less context")
        self._stop = False
        workers = [threading.Thread(target=self._box_worker, daemon=True)
                   for _ in range(self.box_slots)]
        workers.append(threading.Thread(target=self._cluster_worker, daemon=True))
        for w in workers:
            w.start()
        t0 = time.perf_counter()
        for q in requests:
            q.arrival += t0
            delay = q.arrival - time.perf_counter()
            if delay > 0:
                time.sleep(delay)
            with self._cv:
                (self._box_q if q.kind == "box" else self._cl_q).append(q)
                self._cv.notify_all()
        with self._cv:
            self._stop = True
            self._cv.notify_all()
        for w in workers:
            w.join()
        torch.cuda.synchronize(self.dev)
        return time.perf_counter() - t0

    def close(self):
        for r in self.resident.values():
            r.engine.close()
        self.resident.clear()
        self.batcher.close()


# ----------------------------------------------------------------- workload
def serving_pool(seed=0, n_clusters=48, box_sizes=("box216", "box216", "box1024", "box1024",
                                                     "box4096", "box4096")):
    """The request pool: clusters of U{2..64} waters and periodic boxes of
    the named workloads (each box entry gets its own seeded system)."""
    from synth import water_cluster, water_box
    from synth.water import CONFIGS
    rng = np.random.default_rng(seed)
    systems = {}
    for k in range(n_clusters):
        nw = int(rng.integers(2, 65))
        systems[f"cl{k}"] = water_cluster(nw, 500 + 64 * seed + k)
    for k, name in enumerate(box_sizes):
        c = CONFIGS[name]
        d = water_box(c["n_waters"], c["box"], 200 + 16 * seed + k)
        d["params"] = dict(beta=c["beta"], cutoff=c["cutoff"], grid=c["grid"], order=c["order"])
        systems[f"{name}_{k}"] = d
    return systems


def request_stream(systems, n_requests, rate, seed=0, cluster_share=0.7, step=0.01):
    """Poisson arrivals at `rate` per second; each request picks a cluster
    (probability cluster_share) or a box uniformly from the pool, and a
    repeat of a system moves every site by U[-step, step] A from its last
    positions (an MD step)."""
    rng = np.random.default_rng(seed)
    clusters = sorted(k for k, v in systems.items() if v.get("box") is None)
    boxes = sorted(k for k, v in systems.items() if v.get("box") is not None)
    current = {}
    t = 0.0
    out = []
    for rid in range(n_requests):
        t += rng.exponential(1.0 / rate)
        kind = "cluster" if rng.random() < cluster_share else "box"
        pool = clusters if kind == "cluster" else boxes
        name = pool[int(rng.integers(len(pool)))]
        if name in current:
            pos = current[name] + rng.uniform(-step, step, size=current[name].shape)
        else:
            pos = systems[name]["pos"].copy()
        current[name] = pos
        out.append(Request(rid, name, kind, pos, t))
    return out


def box_overlap(spans):
    """How much box evaluations overlapped in time: the share of box
    requests that ran while another box request was running, and the
    largest number in flight at once."""
    if not spans:
        return dict(box_overlap_share=0.0, max_boxes_in_flight=0)
    ev = sorted([(s, 1) for s, _ in spans] + [(d, -1) for _, d in spans])
    cur = best = 0
    for _, k in ev:
        cur += k
        best = max(best, cur)
    s = np.array(sorted(spans))
    overl = 0
    for i, (a, b) in enumerate(s):
        if np.any((s[:, 0] < b) & (s[:, 1] > a) & (np.arange(len(s)) != i)):
            overl += 1
    return dict(box_overlap_share=round(overl / len(s), 3), max_boxes_in_flight=int(best))


def summarize(requests, wall, server=None, skip=0):
    """Latency percentiles (ms) and throughput over requests[skip:]."""
    rs = [q for q in requests[skip:] if q.done is not None]
    lat = np.array([q.done - q.arrival for q in rs]) * 1e3
    out = dict(requests=len(rs), wall_s=round(wall, 3),
               throughput_per_s=round(len(rs) / wall, 1) if wall > 0 else None,
               p50_ms=round(float(np.percentile(lat, 50)), 3) if len(lat) else None,
               p99_ms=round(float(np.percentile(lat, 99)), 3) if len(lat) else None,
               failed=sum(1 for q in rs if q.status not in (0,)))
    for kind in ("cluster", "box"):
        lk = np.array([q.done - q.arrival for q in rs if q.kind == kind]) * 1e3
        if len(lk):
            out[kind] = dict(count=len(lk), p50_ms=round(float(np.percentile(lk, 50)), 3),
                             p99_ms=round(float(np.percentile(lk, 99)), 3),
                             warm_share=round(np.mean([q.warm for q in rs if q.kind == kind]), 3),
                             mean_iterations=round(float(np.mean(
                                 [q.iterations for q in rs if q.kind == kind
                                  and q.iterations is not None])), 2))
    if server is not None:
        out["utilisation"] = {k: round(v / wall, 3) for k, v in server.busy.items()}
        out["box_slots"] = server.box_slots
        out.update(box_overlap(server.box_spans))
        out["evictions"] = server.evictions
        out["rejections"] = server.rejections
        if server.batches:
            out["mean_batch_clusters"] = round(float(np.mean([b[0] for b in server.batches])), 2)
        out["errors"] = server.errors[:3]
    return out
