#!/usr/bin/env python3
"""Benchmark of the polarization path on one MI355X.

One step = one full pol+elec energy/force evaluation of the 32,000-water
periodic box (98.55 A, cutoff 9 A, beta 0.40/A, SPME 96^3 order 5, PCG to a
true-residual RMS of 1e-8 D, cold start): cell sort and neighbour lists,
permanent field (real space + SPME), PCG solve, E_pol, E_elec and all site
forces.  Inputs are resident in HBM before timing starts.  The solve runs
with the molecular block preconditioner (--precond; the tolerance measures
alpha r either way) and the same steps are timed with the diagonal one
beside it.

Prints ONE JSON line.  `value` is evaluations per second of the precision
named in `dtype`; both precisions are reported under "fp64" and "mixed".
The roofline object covers the kernel with the largest share of the timed
region (per-launch durations from HIP events recorded by the library on its
own stream).  The CPU baseline times the FP64 oracle on a bounded sample of
the same workload and scales it to one evaluation.
"""
import argparse
import json
import math
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "pol+elec energy/force evals/s @32k waters, FP32-mixed vs FP64; p50/p99 latency"
PRECOND_NAMES = {"molblock": "molecular block-Jacobi (each water's 9x9 block of T, bare form)",
                 "diag": "diagonal (alpha per site)"}
WORKLOAD = "box32000"

# MI355X published peaks: vector FP64 78.6 TFLOP/s, vector FP32 157.3
# TFLOP/s (the FP32 figure counts packed two-wide FP32 instructions, which
# this build leaves disabled: its FP32 kernels can issue at most half of
# it), HBM 8 TB/s.
PEAK_VALU_TFLOPS = {"fp64": 78.6, "mixed": 157.3}
PEAK_HBM_GBS = 8000.0

# Algorithmic flop counts (FMA = 2, each erfc/exp/rsqrt = 1) of one pair of
# the real-space force and permanent-field kernels.
FLOPS_FORCE_PAIR = 560
FLOPS_FIELD_PAIR = 190
# Algorithmic flops of one unordered polarizable pair of the matvec T p,
# counted for the pair evaluated from scratch (the method's work, whatever
# the kernel caches): separation and r^2 (8), rsqrt and r (2), the Ewald
# B1, B2 with exp(-beta^2 r^2) and erfc (32), the Thole lambda_3,
# lambda_5 and bare coefficients (20), the two screened coefficients (6),
# and the dipole field of each site at the other, R.p and c2 R (R.p) -
# c1 p accumulated (2 x 13).
FLOPS_MATVEC_HALF_PAIR = 95

# Algorithmic bytes of the real-space matvec kernel k_matvec, streamed once
# per launch (operands gathered for neighbour j are shared by every row that
# lists j and are counted once, with the site's own row):
#   per intermolecular polarizable list entry: 4 B neighbour index + the
#     cached coefficient pair (c1, c2): 16 B in FP64, 8 B in FP32;
#   per same-molecule list entry: 4 B index + 16 B FP64 coefficients;
#   per polarizable site: position/Thole record (32 B FP64; + 16 B FP32 in
#     mixed), p (32 B; + 16 B FP32 copy in mixed), alpha^-1 (48 B),
#     T p written (32 B), two list counts (8 B).
MATVEC_ENTRY_BYTES = {"fp64": 20, "mixed": 12}
MATVEC_SAME_BYTES = 20
MATVEC_SITE_BYTES = {"fp64": 152, "mixed": 184}
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_matvec_box32000_traffic.md")


def matvec_bytes(pairs, npol, precision):
    return (pairs["pol"] * MATVEC_ENTRY_BYTES[precision]
            + pairs["pol_same_molecule"] * MATVEC_SAME_BYTES
            + npol * MATVEC_SITE_BYTES[precision])


def measured_traffic(precision):
    """HBM bytes per k_matvec launch from the committed counter summary
    (FETCH_SIZE + WRITE_SIZE, scaled by the copy-kernel factor), or None when
    that summary is absent or was taken from other kernel sources."""
    try:
        txt = open(TRAFFIC_FILE).read()
    except OSError:
        return None
    vals = {}
    for line in txt.splitlines():
        parts = line.strip().strip("|").split("|")
        if len(parts) >= 2:
            vals[parts[0].strip()] = parts[1].strip().strip("`")
    from paper_2201_00804_amd.profsum import source_hash
    if vals.get("kernel sources sha256[:16]") != source_hash("k_matvec"):
        return None
    v = vals.get(f"traffic bytes per launch ({precision})")
    return float(v) if v else None


def _percentile(xs, q):
    xs = sorted(xs)
    if not xs:
        return float("nan")
    k = (len(xs) - 1) * q
    f, c = math.floor(k), math.ceil(k)
    return xs[f] if f == c else xs[f] + (xs[c] - xs[f]) * (k - f)


def run_gpu(sysd, prm, precision, steps, warmup, precond="molblock", profile=True):
    import torch
    from paper_2201_00804_amd import Engine, default_params

    params = default_params(beta=prm["beta"], cutoff=prm["cutoff"], grid=prm["grid"],
                            order=prm["order"], tol=prm["tol"], precision=precision,
                            max_iter=400, precond=precond)
    eng = Engine(0)
    eng.load(sysd, params)
    dev = eng.device
    pos = torch.as_tensor(sysd["pos"], dtype=torch.float64, device=dev).contiguous()
    F = torch.empty_like(pos)

    def step():
        eng.update_positions(pos)
        _, it, rms = eng.solve(warm_start=False)
        e_pol, e_elec, _ = eng.energy_forces(out=F)
        return it, rms, e_pol, e_elec

    for _ in range(warmup):
        step()
    # timed region: nothing but the evaluations
    times = []
    info = None
    torch.cuda.synchronize()
    t_all = time.perf_counter()
    for _ in range(steps):
        t0 = time.perf_counter()
        info = step()
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
    torch.cuda.synchronize()
    total = time.perf_counter() - t_all
    if not profile:
        st = eng.stats()
        out = dict(total_s=total, step_s=times, iters=info[0], true_rms_debye=info[1],
                   e_pol=info[2], e_elec=info[3], stats=st)
        eng.close()
        return out
    # the same steps again with HIP events around the matvec kernel only
    # (roofline), then around every phase (breakdown)
    eng.set_profiling(True, phases=["matvec"])
    for _ in range(steps):
        step()
    prof_mv = eng.profile()
    eng.set_profiling(True)
    for _ in range(steps):
        step()
    prof = eng.profile()
    eng.set_profiling(False)
    st = eng.stats()
    out = dict(total_s=total, step_s=times, iters=info[0], true_rms_debye=info[1],
               e_pol=info[2], e_elec=info[3], profile=prof, profile_matvec=prof_mv, stats=st,
               forces=F.detach().cpu().numpy(), mu=eng.get_dipoles().cpu().numpy())
    eng.close()
    return out


def run_tcg(sysd, prm, precision, steps, warmup, orders=(1, 2), omega=1.0, precond="molblock"):
    """Fixed-cost truncated CG (with the peek step) against the converged
    solve, both without forces: ms per evaluation (positions update, lists,
    field, solve, E_pol) and E_pol; in FP64 also TCG energies with their
    forces (the derivative of the truncated iteration)."""
    import torch
    from paper_2201_00804_amd import Engine, default_params

    params = default_params(beta=prm["beta"], cutoff=prm["cutoff"], grid=prm["grid"],
                            order=prm["order"], tol=prm["tol"], precision=precision,
                            max_iter=400, precond=precond)
    eng = Engine(0)
    eng.load(sysd, params)
    pos = torch.as_tensor(sysd["pos"], dtype=torch.float64, device=eng.device).contiguous()

    def pcg():
        eng.update_positions(pos)
        eng.solve(warm_start=False)
        return eng.energy_forces(forces=False)[0]

    def tcg(n):
        eng.update_positions(pos)
        return eng.solve_tcg(n, omega, mu_out=False)[1]

    def tcg_forces(n):
        eng.update_positions(pos)
        ep, ee, _f, _m = eng.tcg_energy_forces(n, omega)
        return ep

    variants = [("pcg", pcg)] + [(f"tcg{n}_peek", (lambda n=n: tcg(n))) for n in orders]
    if precision == "fp64":
        # energies and forces at TCG dipoles (always FP64)
        variants += [(f"tcg{n}_peek_forces", (lambda n=n: tcg_forces(n))) for n in orders]
    out = {}
    for name, fn in variants:
        for _ in range(warmup):
            fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            e = fn()
        torch.cuda.synchronize()
        out[name] = dict(ms=round(1e3 * (time.perf_counter() - t0) / steps, 3), e_pol=e)
    eng.close()
    ref = out["pcg"]["e_pol"]
    for name in out:
        out[name]["e_pol_rel_err"] = abs(out[name]["e_pol"] - ref) / abs(ref)
    out["omega"] = omega
    return out


def run_md(name, precision, relax_steps, steps, dt=1.0, predictor=3, precond="molblock"):
    """Beeman dynamics demo: the synthetic start relaxed with damped steps
    (0.2 fs, friction 0.3), then `steps` plain Beeman steps of dt fs with
    thermal velocities, warm-started solves with the extrapolating
    predictor; steps/s of the timed part, solver iterations per step and
    the total-energy drift over it."""
    import numpy as np
    import torch
    from synth import config_system, water_md
    from paper_2201_00804_amd import Engine, default_params

    d, cfg = config_system(name)
    m = water_md(d, 3)
    t = lambda a, dt_=torch.float64: torch.as_tensor(np.asarray(a), dtype=dt_,
                                                     device="cuda").contiguous()
    eng = Engine(0)
    eng.load(d, default_params(beta=cfg["beta"], cutoff=cfg["cutoff"], grid=cfg["grid"],
                               order=cfg["order"], tol=cfg["tol"], precision=precision,
                               max_iter=400, precond=precond))
    eng.set_predictor(predictor)
    args = (t(m["masses"]), t(m["vsites"], torch.int32), t(m["bonds"], torch.int32),
            t(m["bond_k"]), t(m["bond_r0"]), t(m["rep_radius"]), m["rep_eps"])
    eng.md_init(*args)
    eng.md_run(relax_steps, 0.2, 0.3)
    eng.md_init(*args, vel=t(m["vel"]))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st = np.array(eng.md_run(steps, dt))
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    eng.close()
    et = st[:, :5].sum(1)
    return dict(workload=name, n_waters=len(d["pos"]) // 5, dt_fs=dt, steps=steps,
                relax_steps=relax_steps, predictor=predictor,
                steps_per_s=round(steps / el, 2), ms_per_step=round(1e3 * el / steps, 3),
                iterations_mean=round(float(st[:, 5].mean()), 2),
                e_tot_drift=round(float(et[-1] - et[0]), 4),
                e_tot_spread=round(float(et.max() - et.min()), 4),
                e_kin_mean=round(float(st[:, 4].mean()), 2))


def run_ct(name, steps=10, warmup=2):
    """Reduced charge transfer on a water box with two lone-pair sites per
    water: ms per E_ct + forces call (potentials, pair passes, potential
    forces, the reciprocal passes), FP64."""
    import numpy as np
    import torch
    from synth import config_system, water_lone_pairs, water_ct
    from paper_2201_00804_amd import Engine, default_params

    d, cfg = config_system(name)
    d = water_lone_pairs(d)
    ct = water_ct(d)
    t = lambda a, dt_=torch.float64: torch.as_tensor(np.asarray(a), dtype=dt_,
                                                     device="cuda").contiguous()
    eng = Engine(0)
    eng.load(d, default_params(beta=cfg["beta"], cutoff=cfg["cutoff"], grid=cfg["grid"],
                               order=cfg["order"], tol=cfg["tol"], max_iter=400))
    eng.set_charge_transfer(t(ct["lp"], torch.int32), t(ct["lp_par"]), t(ct["acc"], torch.int32),
                            t(ct["ah"]), t(ct["rvdw"]), ct["eta"], ct["cs"], ct["cp"], ct["t"],
                            ct["m"])
    for _ in range(warmup):
        e, _f = eng.ct_energy_forces()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        e, _f = eng.ct_energy_forces()
    torch.cuda.synchronize()
    ms = 1e3 * (time.perf_counter() - t0) / steps
    eng.close()
    return dict(workload=name + "+lone_pairs", n_sites=len(d["pos"]), n_lone_pairs=len(ct["lp"]),
                n_acceptors=len(ct["acc"]), ms_energy_forces=round(ms, 3), e_ct=e)


def roofline(res, precision):
    """Roofline point of the kernel with the largest share of the timed
    region, the real-space matvec.  It is priced as vector-ALU work (the
    method's flops per unordered pair times the pairs of one launch, over
    the launch time, against the vector peak of the kernel's precision); the
    HBM rate of the bytes it streams is given beside it.  The force and field
    pair kernels, if they dominate, are priced in flops the same way."""
    prof = res["profile"]
    ms, calls, pairs = prof["ms"], prof["calls"], prof["pairs"]
    npol = res["stats"]["n_polarizable"]
    total = max(sum(ms.values()), 1e-30)
    share = {k: round(v / total, 4) for k, v in ms.items() if v > 0}
    dom = "matvec" if ms["matvec"] > 0 else max(ms, key=lambda k: ms[k])
    if dom == "matvec":
        pm = res["profile_matvec"]
        avg_ms = pm["ms"]["matvec"] / max(pm["calls"]["matvec"], 1)
        launches = pm["calls"]["matvec"]
    else:
        avg_ms = ms[dom] / max(calls[dom], 1)
        launches = calls[dom]
    base = dict(phase=dom, avg_launch_ms=round(avg_ms, 5), launches=launches,
                phase_share=share,
                timing="HIP events around each launch on the library stream, over the "
                       "timed steps repeated with only that phase instrumented")
    peak = PEAK_VALU_TFLOPS[precision]
    if dom == "matvec":
        half_pairs = (pairs["pol"] + pairs["pol_same_molecule"]) / 2.0
        fl = half_pairs * FLOPS_MATVEC_HALF_PAIR
        tf = fl / (avg_ms * 1e-3) / 1e12
        b = matvec_bytes(pairs, npol, precision)
        gbs = b / (avg_ms * 1e-3) / 1e9
        return dict(kernel="k_matvec", bound="alu", achieved=round(tf, 3), peak=peak,
                    unit="TFLOP/s", frac=round(tf / peak, 4),
                    traffic=measured_traffic(precision), flops_per_launch=int(fl),
                    half_pairs_per_launch=int(half_pairs),
                    hbm=dict(achieved=round(gbs, 1), peak=PEAK_HBM_GBS, unit="GB/s",
                             frac=round(gbs / PEAK_HBM_GBS, 4), bytes_per_launch=int(b)),
                    **base)
    if dom in ("force_real", "field_real"):
        fl = (pairs["all"] + pairs["same_molecule"]) * \
            (FLOPS_FORCE_PAIR if dom == "force_real" else FLOPS_FIELD_PAIR)
        tf = fl / (avg_ms * 1e-3) / 1e12
        return dict(kernel="k_force" if dom == "force_real" else "k_perm", bound="alu",
                    achieved=round(tf, 3), peak=peak, unit="TFLOP/s",
                    frac=round(tf / peak, 4), traffic=None,
                    flops_per_launch=int(fl), **base)
    return dict(kernel=dom, bound="hbm", achieved=None, peak=PEAK_HBM_GBS, unit="GB/s",
                frac=None, traffic=None, **base)


def recip_chain(res, precision, K):
    """HBM rate of the solver's reciprocal chain against its algorithmic
    bytes per iteration (grid of K^3 values of w bytes; w = 4 in mixed
    precision, 8 in FP64; N_pol polarizable sites):
      spread (tile + fold)   K^3 w written + position and p read (6 w per site)
      FFT pair (fwd + inv)   two transforms of three read+write passes: 12 K^3 w
      gather (+ p.Tp)        K^3 w read + position (3 w), p (24 B) read and
                             T p read and written (2 x 24 B) per site
    Phase times are the HIP-event means per launch group of the profiled
    steps (the chain runs beside the real-space matvec)."""
    prof = res["profile"]
    npol = res["stats"]["n_polarizable"]
    w = 4 if precision == "mixed" else 8
    grid = K ** 3 * w
    parts = {"spread": grid + 6 * w * npol, "fft": 12 * grid,
             "matvec_recip": grid + (3 * w + 72) * npol}
    out, tb, tt = {}, 0.0, 0.0
    for ph, b in parts.items():
        calls = max(prof["calls"][ph], 1)
        ms = prof["ms"][ph] / calls
        gbs = b / (ms * 1e-3) / 1e9
        out[ph] = dict(avg_ms=round(ms, 5), bytes=int(b), achieved_gbs=round(gbs, 1),
                       frac=round(gbs / PEAK_HBM_GBS, 4))
        tb += b
        tt += ms
    out["chain"] = dict(ms=round(tt, 5), bytes=int(tb), achieved_gbs=round(tb / (tt * 1e-3) / 1e9, 1),
                        frac=round(tb / (tt * 1e-3) / 1e9 / PEAK_HBM_GBS, 4))
    return out


def copy_probe(mib, reps):
    """A plain device copy of known size, the reference point that scales the
    FETCH_SIZE / WRITE_SIZE counters of the kernels to bytes."""
    import torch
    n = mib * (1 << 20) // 4
    x = torch.ones(n, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    for _ in range(reps):
        y.copy_(x)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes_read": n * 4, "copy_probe_bytes_written": n * 4,
                      "reps": reps}), flush=True)


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


# State shared with the forked real-space workers of the CPU baseline.
_MP = {}


def _rs_rows_worker(rows):
    """One worker's share of the oracle's real-space pair sums: rows
    (pol_rows, all_rows) of the sample.  Returns the time of each part."""
    import numpy as np
    from threadpoolctl import threadpool_limits

    from oracle import realspace as rs
    from oracle.model import Context

    s, p, pf = _MP["s"], _MP["p"], _MP["pf"]
    rp, ra = rows
    t = {}
    with threadpool_limits(limits=1):
        # the neighbour search's cost per row: a one-row search measures the
        # fixed part (tree and same-molecule pairs over the whole box)
        t0 = time.perf_counter()
        Context(s, p, subset=np.union1d(rp, ra)[:1])
        t1 = time.perf_counter()
        ctx = Context(s, p, subset=np.union1d(rp, ra))
        t["pairs"] = max((time.perf_counter() - t1) - (t1 - t0), 0.0)
        mult = (s.q, s.dip, s.th)
        none3 = (None, None, None)
        I = ctx.pairs.i
        m_pol = np.isin(I, rp)
        m_all = np.isin(I, ra)
        t0 = time.perf_counter()
        rs.pair_sum(ctx.pairs, "Mmu", ctx.kernel, p.beta, ctx.thole, none3, mult, "field", s.n,
                    pair_mask=m_pol)
        t["real_field"] = time.perf_counter() - t0
        t0 = time.perf_counter()
        rs.pair_sum(ctx.pairs, ctx.mumu_cls, ctx.kernel, p.beta, ctx.thole, none3,
                    (None, pf, None), "field", s.n, pair_mask=m_pol & ctx.is_pol[ctx.pairs.j])
        t["real_matvec"] = time.perf_counter() - t0
        mud = (None, pf, None)
        t0 = time.perf_counter()
        for cls, a, b in (("MM", mult, mult), ("Mmu", mud, mult), ("Mmu", mult, mud),
                          (ctx.mumu_cls, mud, mud)):
            rs.pair_sum(ctx.pairs, cls, ctx.kernel, p.beta, ctx.thole, a, b, "force", s.n,
                        pair_mask=m_all)
        t["real_force"] = time.perf_counter() - t0
        t0 = time.perf_counter()
        rs.pair_sum(ctx.pairs, "MM", ctx.kernel, p.beta, ctx.thole, mult, mult, "energy", s.n,
                    pair_mask=m_all)
        t["real_energy"] = time.perf_counter() - t0
    return t


def cpu_full_eval(name):
    """One whole FP64 oracle evaluation of a small box, on one thread: the
    permanent field, the PCG solve to the tolerance, E_pol, E_elec and all
    forces (the oracle's own evaluate, unsampled)."""
    from threadpoolctl import threadpool_limits

    from oracle.model import System, Params, evaluate
    from synth import config_system

    d, cfg = config_system(name)
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        s = System.from_dict(d)
        p = Params(method="spme", beta=cfg["beta"], cutoff=cfg["cutoff"],
                   grid=(cfg["grid"],) * 3, order=cfg["order"], tol=cfg["tol"])
        r = evaluate(s, p)
        sec = time.perf_counter() - t0
    return dict(workload=name, n_sites=len(d["pos"]), seconds=round(sec, 2), cores=1,
                kind="oracle", iterations=int(r["iters"]), e_pol=float(r["E_pol"]))


def cpu_baseline(sysd, prm, iters, sample=360):
    """The FP64 oracle on a bounded sample of the same box, scaled to one
    evaluation: the oracle's real-space pair sums for `sample` sites
    (polarizable ones for E and T p, arbitrary ones for forces and the MM
    energy) and its neighbour search for them, each scaled by N/sample, plus
    one full-size SPME pass of each kind (permanent field; dipoles, once per
    matvec; combined density for forces).

    Two timings: one process on one thread, and the real-space rows split
    over every host core the process may use (forked worker processes, one
    thread each; each part timed by its slowest worker) with the SPME passes
    (one process, one thread) added unchanged."""
    import multiprocessing

    import numpy as np
    from threadpoolctl import threadpool_limits

    from oracle import realspace as rs
    from oracle.model import System, Params, Context

    with threadpool_limits(limits=1):
        s = System.from_dict(sysd)
        p = Params(method="spme", beta=prm["beta"], cutoff=prm["cutoff"],
                   grid=(prm["grid"],) * 3, order=prm["order"], tol=prm["tol"])
        pol = s.pol
        rng = np.random.default_rng(7)
        samp_pol = np.sort(rng.choice(pol, sample, replace=False))
        samp_all = np.sort(rng.choice(s.n, sample, replace=False))
        both = np.union1d(samp_pol, samp_all)
        t, wall = {}, 0.0

        def timed(fn):
            nonlocal wall
            t0 = time.perf_counter()
            out = fn()
            dt = time.perf_counter() - t0
            wall += dt
            return out, dt

        _, t_fixed = timed(lambda: Context(s, p, subset=both[:1]))
        ctx, t_ctx = timed(lambda: Context(s, p, subset=both))
        t["pairs"] = t_fixed + max(t_ctx - t_fixed, 0.0) * s.n / len(both)
        mult = (s.q, s.dip, s.th)
        none3 = (None, None, None)
        I = ctx.pairs.i
        m_pol = np.isin(I, samp_pol)
        m_all = np.isin(I, samp_all)
        _, dt = timed(lambda: rs.pair_sum(ctx.pairs, "Mmu", ctx.kernel, p.beta, ctx.thole, none3,
                                          mult, "field", s.n, pair_mask=m_pol))
        t["real_field"] = dt * len(pol) / sample
        _, t["spme_field"] = timed(lambda: ctx.recip_derivs(mult, s.pos[samp_pol], 1))
        pv = rng.normal(size=(len(pol), 3)) * 0.05
        pf = ctx.full(pv)
        mask_t = m_pol & ctx.is_pol[ctx.pairs.j]
        _, dt = timed(lambda: rs.pair_sum(ctx.pairs, ctx.mumu_cls, ctx.kernel, p.beta, ctx.thole,
                                          none3, (None, pf, None), "field", s.n, pair_mask=mask_t))
        t["real_matvec"] = dt * len(pol) / sample
        _, t["spme_matvec"] = timed(lambda: ctx.recip_derivs((None, pf, None), s.pos[samp_pol], 1))
        mud = (None, pf, None)

        def forces():
            for cls, a, b in (("MM", mult, mult), ("Mmu", mud, mult), ("Mmu", mult, mud),
                              (ctx.mumu_cls, mud, mud)):
                rs.pair_sum(ctx.pairs, cls, ctx.kernel, p.beta, ctx.thole, a, b, "force", s.n,
                            pair_mask=m_all)

        _, dt = timed(forces)
        t["real_force"] = dt * s.n / sample
        comb = (s.q, s.dip + pf, s.th)
        _, t["spme_force"] = timed(lambda: ctx.recip_derivs(comb, s.pos[samp_all], 3))
        _, dt = timed(lambda: rs.pair_sum(ctx.pairs, "MM", ctx.kernel, p.beta, ctx.thole, mult,
                                          mult, "energy", s.n, pair_mask=m_all))
        t["real_energy"] = dt * s.n / sample

    def per_eval(tt):
        return (tt["pairs"] + tt["real_field"] + t["spme_field"] +
                (iters + 1) * (tt["real_matvec"] + t["spme_matvec"]) + tt["real_force"] +
                t["spme_force"] + tt["real_energy"])

    t_eval1 = per_eval(t)
    # the real-space rows over every usable core
    cores = max(1, len(os.sched_getaffinity(0)))
    _MP.update(s=s, p=p, pf=pf)
    chunks = [(samp_pol[k::cores], samp_all[k::cores]) for k in range(cores)]
    mp = multiprocessing.get_context("fork")
    t0 = time.perf_counter()
    with mp.Pool(cores) as pool:
        parts = pool.map(_rs_rows_worker, chunks, chunksize=1)
    t_map = time.perf_counter() - t0
    _MP.clear()
    tm = {}
    for k in ("pairs", "real_field", "real_matvec", "real_force", "real_energy"):
        slowest = max(w[k] for w in parts)
        rows = len(pol) if k in ("real_field", "real_matvec") else s.n
        tm[k] = slowest * rows / sample
    tm["pairs"] = t_fixed + max(w["pairs"] for w in parts) * s.n / len(both)
    t_eval_mc = per_eval(tm)
    return dict(value=1.0 / t_eval_mc, unit="evals/s", cores=cores, kind="oracle",
                cpu_model=_cpu_model(),
                sample=(f"{sample} polarizable + {sample} arbitrary sites of the "
                        f"{len(np.unique(sysd['mol'])):,}-molecule box (real-space rows and "
                        f"neighbour search scaled by N/sample; rows "
                        f"split over {cores} worker processes, one thread each) plus "
                        f"full-size SPME passes on one thread (permanent; dipole, once per "
                        f"matvec; combined for forces); {iters + 1} matvecs per solve; "
                        f"{wall:.1f} s of single-thread and {t_map:.1f} s of parallel "
                        f"measured CPU work"),
                seconds_per_eval=round(t_eval_mc, 1),
                parts_s={**{k: round(v, 2) for k, v in tm.items()},
                         **{k: round(t[k], 2) for k in ("spme_field", "spme_matvec",
                                                        "spme_force")}},
                single_thread=dict(value=1.0 / t_eval1, cores=1, seconds_per_eval=round(t_eval1, 1),
                                   parts_s={k: round(v, 2) for k, v in t.items()}))


def run_serving(n_requests, n_warmup, utilisation=0.65, seed=0, precond="molblock"):
    """Open-loop serving stream on the synthetic pool (48 clusters of
    U{2..64} waters, boxes of 216, 1,024 and 4,096 waters, two of each;
    70% cluster requests; repeats are MD steps of 0.01 A), mixed precision
    at 1e-8 D.  A warm-up stream at 200 requests/s admits every box and
    measures the box worker's mean service time S; the timed stream then
    arrives at the Poisson rate that loads that worker to `utilisation`
    (rate = utilisation / (0.3 S))."""
    from paper_2201_00804_amd.serve import Server, serving_pool, request_stream, summarize
    systems = serving_pool(seed)
    srv = Server(systems, precision="mixed", tol=1e-8, precond=precond)
    stream = request_stream(systems, n_warmup + n_requests, rate=1.0, seed=seed + 1)
    warm, timed = stream[:n_warmup], stream[n_warmup:]
    for q in warm:
        q.arrival /= 200.0
    srv.run(warm)
    n_box = sum(q.kind == "box" for q in warm)
    s_box = srv.busy["box"] / max(n_box, 1)
    rate = utilisation / (0.3 * s_box)
    t_first = timed[0].arrival
    for q in timed:
        q.arrival = (q.arrival - t_first) / rate
    srv.busy = {"box": 0.0, "cluster": 0.0}
    srv.batches.clear()
    wall = srv.run(timed)
    out = summarize(timed, wall, srv)
    out.update(rate_per_s=round(rate, 1), warmup_requests=n_warmup,
               warmup_box_service_ms=round(1e3 * s_box, 3),
               pool="48 clusters U{2..64} waters + boxes 216, 1024, 4096 (x2); 70% clusters; "
                    "MD steps of 0.01 A; mixed precision, 1e-8 D",
               box_precond=PRECOND_NAMES[precond],
               resident_mb=round(srv.resident_bytes / 2 ** 20, 1))
    srv.close()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--precision", choices=["both", "fp64", "mixed"], default="both")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--serve-requests", type=int, default=2000)
    ap.add_argument("--serve-warmup", type=int, default=300)
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--no-tcg", action="store_true")
    ap.add_argument("--no-md", action="store_true")
    ap.add_argument("--no-ct", action="store_true")
    ap.add_argument("--precond", choices=["molblock", "diag"], default="molblock",
                    help="preconditioner of the PCG solve (the other one is timed beside it)")
    ap.add_argument("--no-alt-precond", action="store_true")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB (counter reference)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the path is built for a single MI355X "
              "(sharding over several GPUs is designed, not built); use --gpus 1",
              file=sys.stderr)
        sys.exit(2)
    if args.copy_probe:
        copy_probe(args.copy_probe, max(args.steps, 1))
        return

    from synth import config_system
    sysd, prm = config_system(WORKLOAD)
    import numpy as np

    precisions = ["fp64", "mixed"] if args.precision == "both" else [args.precision]
    results = {}
    for prec in precisions:
        print(f"[bench] {prec}: {args.warmup} warmup + {args.steps} timed steps", file=sys.stderr,
              flush=True)
        results[prec] = run_gpu(sysd, prm, prec, args.steps, args.warmup, args.precond)
        r = results[prec]
        print(f"[bench] {prec}: {1e3 * r['total_s'] / args.steps:.2f} ms/step, iters "
              f"{r['iters']}, rms {r['true_rms_debye']:.2e} D", file=sys.stderr, flush=True)

    def summary(r):
        return dict(value=round(args.steps / r["total_s"], 3),
                    ms_per_step=round(1e3 * r["total_s"] / args.steps, 3),
                    p50_ms=round(1e3 * _percentile(r["step_s"], 0.5), 3),
                    p99_ms=round(1e3 * _percentile(r["step_s"], 0.99), 3),
                    iterations=r["iters"], restarts=r["stats"]["restarts"],
                    true_rms_debye=r["true_rms_debye"], e_pol=r["e_pol"], e_elec=r["e_elec"],
                    phase_ms_per_step={k: round(v / args.steps, 4)
                                       for k, v in r["profile"]["ms"].items()})

    head = "mixed" if "mixed" in results else precisions[0]
    main_r = results[head]
    out = {
        "metric": METRIC,
        "value": round(args.steps / main_r["total_s"], 3),
        "unit": "evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(1e3 * main_r["total_s"] / args.steps, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64" if head == "mixed" else "f64",
        "data": "synthetic",
        "config": {"workload": "32,000 rigid waters, 98.55 A periodic box, cutoff 9 A, "
                               "beta 0.40/A, SPME 96^3 order 5, PCG to 1e-8 D RMS (cold start)",
                   "n_waters": 32000, "n_sites": len(sysd["pos"]), "precision": head,
                   "precond": PRECOND_NAMES[args.precond]},
        "latency_ms": {"p50": round(1e3 * _percentile(main_r["step_s"], 0.5), 3),
                       "p99": round(1e3 * _percentile(main_r["step_s"], 0.99), 3)},
        "roofline": roofline(main_r, head),
    }
    for k, r in results.items():
        out[k] = summary(r)
        out[k]["recip_chain"] = recip_chain(r, k, prm["grid"])
        if k != head:
            out[k]["roofline"] = roofline(r, k)
    if "fp64" in results and "mixed" in results:
        a, b = results["fp64"], results["mixed"]
        rel = lambda x, y: abs(x - y) / max(abs(y), 1e-300)
        out["mixed_vs_fp64"] = {
            "speedup": round(a["total_s"] / b["total_s"], 3),
            "speedup_target": 2.0,
            "e_pol_rel": rel(b["e_pol"], a["e_pol"]),
            "e_elec_rel": rel(b["e_elec"], a["e_elec"]),
            "e_elec_real_rel": rel(b["stats"]["e_elec_real"], a["stats"]["e_elec_real"]),
            "e_elec_recip_rel": rel(b["stats"]["e_elec_recip"], a["stats"]["e_elec_recip"]),
            "iterations": {"fp64": a["iters"], "mixed": b["iters"]},
            "force_rms_rel": float(np.sqrt(np.mean((b["forces"] - a["forces"]) ** 2) /
                                           np.mean(a["forces"] ** 2))),
            "mu_rms_debye": float(4.803204 * np.sqrt(np.mean(np.sum((b["mu"] - a["mu"]) ** 2, 1)))),
        }
    if not args.no_alt_precond:
        alt = "diag" if args.precond == "molblock" else "molblock"
        out["precond_" + alt] = {"precond": PRECOND_NAMES[alt]}
        for prec in precisions:
            print(f"[bench] {prec} with the {alt} preconditioner", file=sys.stderr, flush=True)
            r = run_gpu(sysd, prm, prec, args.steps, args.warmup, alt, profile=False)
            out["precond_" + alt][prec] = dict(
                value=round(args.steps / r["total_s"], 3),
                ms_per_step=round(1e3 * r["total_s"] / args.steps, 3),
                iterations=r["iters"], true_rms_debye=r["true_rms_debye"], e_pol=r["e_pol"])
            print(f"[bench] {prec} {alt}: {1e3 * r['total_s'] / args.steps:.2f} ms/step, iters "
                  f"{r['iters']}", file=sys.stderr, flush=True)
    if not args.no_tcg:
        out["tcg"] = {}
        for prec in precisions:
            print(f"[bench] tcg {prec}: converged solve vs TCG-1/TCG-2 with peek, no forces",
                  file=sys.stderr, flush=True)
            t = run_tcg(sysd, prm, prec, args.steps, args.warmup, precond=args.precond)
            out["tcg"][prec] = t
            print("[bench] tcg " + prec + ": " + ", ".join(
                f"{k} {v['ms']} ms (E_pol rel err {v['e_pol_rel_err']:.2e})"
                for k, v in t.items() if isinstance(v, dict)), file=sys.stderr, flush=True)
    if not args.no_md:
        out["md"] = []
        for name, relax, nsteps in (("box216", 300, 300), ("box32000", 100, 20)):
            for prec in precisions:
                print(f"[bench] md {name} {prec}: {relax} relaxation + {nsteps} Beeman steps",
                      file=sys.stderr, flush=True)
                r = run_md(name, prec, relax, nsteps, precond=args.precond)
                r["precision"] = prec
                out["md"].append(r)
                print(f"[bench] md {name} {prec}: {r['steps_per_s']} steps/s, "
                      f"{r['iterations_mean']} iterations per step, E_tot drift "
                      f"{r['e_tot_drift']} kcal/mol", file=sys.stderr, flush=True)
    if not args.no_ct:
        out["ct"] = []
        for name in ("box216", "box32000"):
            print(f"[bench] charge transfer {name} + lone pairs", file=sys.stderr, flush=True)
            r = run_ct(name, args.steps, args.warmup)
            out["ct"].append(r)
            print(f"[bench] charge transfer {name}: {r['ms_energy_forces']} ms per E_ct + forces",
                  file=sys.stderr, flush=True)
    if not args.no_serve:
        print(f"[bench] serving: {args.serve_warmup} warm-up + {args.serve_requests} requests",
              file=sys.stderr, flush=True)
        out["serving"] = run_serving(args.serve_requests, args.serve_warmup,
                                     precond=args.precond)
        sv = out["serving"]
        print(f"[bench] serving: {sv['throughput_per_s']} req/s at {sv['rate_per_s']}/s, p50 "
              f"{sv['p50_ms']} ms, p99 {sv['p99_ms']} ms", file=sys.stderr, flush=True)
    if not args.no_cpu_baseline:
        iters = results.get("fp64", main_r)["iters"]
        print("[bench] cpu baseline (oracle, bounded sample)", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(sysd, prm, iters)
        print("[bench] cpu baseline: one whole oracle evaluation of the 216-water box",
              file=sys.stderr, flush=True)
        out["cpu_baseline"]["full_eval"] = cpu_full_eval("box216")
        print("[bench] cpu baseline: the 4,096-water box, same bounded sample",
              file=sys.stderr, flush=True)
        from synth import config_system
        d2, cfg2 = config_system("box4096")
        c2 = cpu_baseline(d2, cfg2, iters)
        out["cpu_baseline"]["box4096"] = dict(
            n_sites=len(d2["pos"]), seconds_per_eval=c2["seconds_per_eval"], cores=c2["cores"],
            single_thread_seconds_per_eval=c2["single_thread"]["seconds_per_eval"],
            sample=c2["sample"])
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
