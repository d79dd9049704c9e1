#!/usr/bin/env python3
"""Benchmark of the staggered even/odd hot path on one MI355X.

One step = one pass of the whole path over one batch of synthetic input:
  1. pack the gauge field (FP64 18-real; the solver converts its FP32 12-real
     inner copy itself),
  2. mixed-precision multi-shift CG for every (right-hand side, shift) to a
     true residual of 1e-10 (FP32 12-real inner iteration, FP64 reliable
     updates, FP64 verification and batched refinement, hipGraph replay,
     right-hand sides batched through each link load),
  3. the rational action S_f,
  4. the fermion force dS_f/dU on the solutions (projected to su(3)).
Inputs (links, pseudofermions) are resident in HBM before the timed region.

Workloads (seeded, synthetic; the paper's thermalised production lattices are
not available):
  c4  48^4, Haar SU(3) links, m = 0.02, 12 shifts in [1e-4, 10], 8 RHS  (default)
  c3  32^4, links exp(0.5 i H), m = 0.02, 12 shifts, 1 RHS

Printed: one JSON line with the step throughput (shift-solves/s), the
time-to-1e-10 of the mixed batched solve next to sequential plain FP64 GPU
solves of the same systems, D_oe/D_eo bandwidth against the 8 TB/s peak and a
STREAM ceiling, the roofline of the dominant kernel measured with HIP events,
and the CPU oracle timed on a bounded sample.

Stencil launch configurations start from the shipped MI355X tuning cache
(paper_1801_01473_amd/tune/gfx950_256cu.txt, written by the stencil tuner on
an MI355X; shapes it lacks are tuned during the warm-up step); --retune tunes
every shape from scratch, LQCD_TUNE_CACHE=<file> uses the caller's cache.

--profile-kernels runs one warm mixed solve of the workload, one measured solve
bracketed by small copy launches (markers in the dispatch list), standalone D_oe
launches and a copy kernel of known size (for rocprofv3 counter collection)
and exits.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Dslash GB/s & % HBM peak; multishift-CG time-to-1e-10, mixed vs FP64, 1 GPU"
HBM_PEAK_GBS = 8000.0

WORKLOADS = {
    "c4": dict(L=(48, 48, 48, 48), links="haar", beta=None, link_seed=104, src_seed=204,
               mass=0.02, nshift=12, nrhs=8,
               name="48^4 (one GPU's share of 96^4), Haar SU(3) links, m=0.02, "
                    "12 shifts log-spaced in [1e-4,10], 8 Gaussian RHS batched, FP32 12-real "
                    "inner / FP64 outer, tol 1e-10; + rational action + fermion force"),
    "c3": dict(L=(32, 32, 32, 32), links="exp", beta=0.5, link_seed=103, src_seed=203,
               mass=0.02, nshift=12, nrhs=1,
               name="32^4, links exp(0.5iH), m=0.02, 12 shifts log-spaced in [1e-4,10], 1 RHS, "
                    "FP32 12-real inner / FP64 reliable updates, tol 1e-10; + action + force"),
}


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def make_inputs(w):
    import numpy as np
    import synth
    L = w["L"]
    t0 = time.time()
    if w["links"] == "haar":
        U = synth.links_haar(L, w["link_seed"])
    else:
        U = synth.links_exp(L, w["beta"], w["link_seed"])
    phi = synth.gaussian_even_source(L, w["nrhs"], w["src_seed"])
    sig = synth.rational_shifts(w["nshift"])
    al = synth.rational_weights(sig)
    log(f"inputs generated in {time.time() - t0:.1f} s")
    return U, phi, np.asarray(sig), np.asarray(al)


def event_time_ms(fn, reps):
    """Median of `reps` individually event-timed launches after 3 warm-ups."""
    import torch
    for _ in range(3):
        fn()
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(reps)]
    for e0, e1 in ev:
        e0.record()
        fn()
        e1.record()
    torch.cuda.synchronize()
    ts = sorted(e0.elapsed_time(e1) for e0, e1 in ev)
    return ts[len(ts) // 2]


def dslash_entry(lq, torch, g, Ul, prec, fmt, n, copy_gbs, label):
    """Standalone D_oe: median launch time, algorithmic GB/s, GFLOP/s (570 per
    output site and RHS; 'executed' adds the row-2 reconstruction per site and
    link load: 336 for 12-real, 384 with the determinant factor, 336 + 8 x 54
    for the U(1) angle format: row 2 and the phase product per link)."""
    cd = torch.complex128 if prec == lq.F64 else torch.complex64
    x = torch.randn(n, 3, g.Vh, dtype=cd, device="cuda")
    y = torch.empty_like(x)
    ms = event_time_ms(lambda: lq.doe(g, Ul, x, out=y), 20)
    byts = g.Vh * dslash_bytes_per_site(prec, fmt, n)
    gbs = byts / (ms * 1e-3) / 1e9
    flops = 570.0 * g.Vh * n
    exe = flops + {lq.LINKS12: 336.0, lq.LINKS12D: 384.0,
                   lq.LINKS12T: 336.0 + 8 * 54.0}.get(fmt, 0.0) * g.Vh
    del x, y
    return dict(what=label, us=1000 * ms, GBps=gbs, frac_hbm_peak=gbs / HBM_PEAK_GBS,
                frac_stream_copy=gbs / copy_gbs, GFLOPs=flops / (ms * 1e-3) / 1e9,
                executed_GFLOPs=exe / (ms * 1e-3) / 1e9)


def dslash_bytes_per_site(prec, fmt, nrhs):
    """Algorithmic bytes per output site: every link once, each input spinor
    once (perfect neighbour reuse), each output once."""
    rb = 8 if prec == 0 else 4
    links = 8 * {0: 18, 1: 12, 2: 14, 3: 13}[fmt] * rb
    return links + nrhs * 2 * (3 * 2 * rb)


def shift_update_bytes(Vh, stats):
    """Algorithmic bytes of the shift-update kernels of a solve, per precision
    and kernel, from the device's counters (per even site, spinor = 3 complex):
      per-iteration update (window 1): r in + per updated shift x, p in and out
      base update (window > 1): r in (the residual ring slot), p in and out
      window flush: each ring slot in + per materialised shift x, p in and out"""
    spin = {"f64": 48, "f32": 24}
    its = {"f64": sum(r[0]["iters_fp64"] for r in stats),
           "f32": sum(r[0]["iters"] - r[0]["iters_fp64"] for r in stats)}
    out = {}
    for prec, sfx in (("f64", "fp64"), ("f32", "fp32")):
        sp = spin[prec]
        if stats[0][0]["shift_window"] > 1:
            out["base_update_" + prec] = Vh * its[prec] * 3 * sp
            out["ms_flush_" + prec] = Vh * sum(r[0]["flush_slots_" + sfx] * sp
                                               + r[0]["flush_shifts_" + sfx] * 4 * sp
                                               for r in stats)
        else:
            upd = sum(r[0]["shift_updates_" + sfx] for r in stats)
            out["ms_update_" + prec] = Vh * (its[prec] * sp + upd * 4 * sp)
    return out


def kernel_table(g, nrhs, stats, ktimes):
    """Per-kernel average launch time (HIP events) and algorithmic bandwidth of
    the main solve's kernels.  Bytes per even/odd site and launch, all RHS live:
      D_oe            links + nrhs (in + out)
      D_eo + CG       links + nrhs (t in + p in + r in + r out)
      shift updates   from the device's counters, see shift_update_bytes."""
    Vh = g.Vh
    upd_bytes = shift_update_bytes(Vh, stats)
    links = {"f64": 8 * 6 * 16, "f32": 8 * 6 * 8}  # 12-real links
    spin = {"f64": 48, "f32": 24}
    out = {}
    for cls, (n, ms) in ktimes.items():
        if "_refine" in cls or not cls.endswith(f"_n{nrhs}"):
            continue
        prec = "f64" if "_f64" in cls else "f32"
        if cls.startswith("dslash_oe"):
            per_launch = Vh * (links[prec] + nrhs * 2 * spin[prec])
            kern = f"k_dslash D_oe {prec} 12-real"
        elif cls.startswith("dslash_eo_cg"):
            per_launch = Vh * (links[prec] + nrhs * 4 * spin[prec])
            kern = f"k_dslash D_eo+CG update {prec} 12-real"
        else:
            base = cls.rsplit("_n", 1)[0]
            if base not in upd_bytes:
                continue
            per_launch = upd_bytes[base] / max(n, 1)
            kern = {"ms_update": "k_ms_update", "base_update": "k_base_update",
                    "ms_flush": "k_ms_flush"}[base.rsplit("_", 1)[0]] + f" {prec}"
        avg_us = 1000.0 * ms / max(n, 1)
        gbs = per_launch / (avg_us * 1e-6) / 1e9
        out[cls] = dict(kernel=kern, launches=n, total_ms=ms, avg_us=avg_us,
                        bytes_per_launch=per_launch, GBps=gbs, frac_hbm_peak=gbs / HBM_PEAK_GBS)
    return out


SHIPPED_TUNE_CACHE = os.path.join(os.path.dirname(os.path.abspath(__file__)),
                                  "paper_1801_01473_amd", "tune", "gfx950_256cu.txt")

# tuning-cache key fields (precision, link format, mode) of the solve's kernel classes
KERNEL_CLASS_KEY = {"dslash_eo_cg_f32": (1, 1, 2), "dslash_oe_f32": (1, 1, 0),
                    "dslash_eo_cg_f64": (0, 1, 2), "dslash_oe_f64": (0, 1, 0)}


def rhs_pairs(kernel_class, nrhs):
    """Whether the multi-shift solve runs this stencil class on interleaved
    right-hand-side pairs: the FP32 classes at an even RHS count, unless
    LQCD_RHS_PAIRS=0 keeps the systems one after the other."""
    base = kernel_class.rsplit("_", 1)[0]
    return (base.endswith("_f32") and nrhs >= 2 and nrhs % 2 == 0
            and not os.environ.get("LQCD_RHS_PAIRS", "").startswith("0"))


def tuned_config(cache, L, kernel_class, nrhs):
    """The configuration the stencil tuner chose for a kernel class in this
    run, read back from the tuning-cache file (the last entry for its key), or
    None."""
    base = kernel_class.rsplit("_", 1)[0]
    if cache is None or base not in KERNEL_CLASS_KEY or not os.path.exists(cache):
        return None
    prec, fmt, mode = KERNEL_CLASS_KEY[base]
    tail = f"/{L[0]}x{L[1]}x{L[2]}x{L[3]}/p{prec}/f{fmt}/n{nrhs}/b0/m{mode}"
    if rhs_pairs(kernel_class, nrhs):
        tail += "/pairs"
    found = None
    with open(cache) as f:
        for line in f:
            key, _, cfg = line.strip().partition(";")
            if key.endswith(tail):
                found = cfg
    return found


def measured_traffic(kernel_class, cfg):
    """HBM bytes per launch of the dominant kernel from the committed rocprofv3
    FETCH_SIZE / WRITE_SIZE passes, with a note.  The bytes are None when the
    dominant kernel is another one, when the stencil sources changed since the
    counters were taken, or when the tuner chose another configuration in this
    run than in the counter runs (the traffic depends on the traversal)."""
    here = os.path.dirname(os.path.abspath(__file__))
    path = os.path.join(here, "profiles", "dominant_kernel_traffic.json")
    if not os.path.exists(path):
        return None, "no counter record"
    with open(path) as f:
        rec = json.load(f)
    if rec.get("kernel_class") != kernel_class:
        return None, f"counters are for {rec.get('kernel_class')}"
    h = hashlib.sha256()
    for src in rec["sources"]:
        with open(os.path.join(here, src), "rb") as f:
            h.update(f.read())
    if h.hexdigest() != rec["source_sha256"]:
        return None, "stencil sources changed since the counters were taken"
    if cfg != rec["tuned_configuration"]:
        return None, (f"counters taken with configuration {rec['tuned_configuration']}, "
                      f"this run tuned {cfg}")
    return (rec["read_bytes_per_launch"] + rec["write_bytes_per_launch"],
            f"configuration {cfg}, as in the counter runs")


def config3_m2(lq, torch):
    """Time-to-1e-10 on the 32^4 single-RHS configuration (links exp(0.5iH),
    m = 0.02, the same 12 shifts): mixed FP32-12 with FP64 reliable updates vs
    plain FP64 18-real, each after one untimed solve (tuning, graph capture)."""
    w = WORKLOADS["c3"]
    U, phi, sig, _ = make_inputs(w)
    g = lq.Geometry(w["L"])
    U64 = lq.pack_links(g, torch.from_numpy(U).to("cuda"))
    b = lq.pack_spinor(g, torch.from_numpy(phi).to("cuda"), 0)
    del U, phi
    out = {}
    for name, kw in (("mixed", dict(inner_prec=lq.F32, inner_fmt=lq.LINKS12)),
                     ("fp64", dict(inner_prec=lq.F64, inner_fmt=lq.LINKS18))):
        p = lq.solver_params(mass=w["mass"], tol=1e-10, **kw)
        lq.cg_multishift(g, p, U64, sig, b)
        torch.cuda.synchronize()
        t0 = time.time()
        _, _, st = lq.cg_multishift(g, p, U64, sig, b)
        torch.cuda.synchronize()
        out[name] = dict(seconds=time.time() - t0, iters=st[0][0]["iters"],
                         refine_iters=sum(s["refine_iters"] for s in st[0]),
                         max_true_rel_residual=max(s["true_rel_residual"] for s in st[0]))
    out["speedup_mixed_vs_fp64"] = out["fp64"]["seconds"] / out["mixed"]["seconds"]
    log(f"config 3 (32^4, 1 RHS): mixed {out['mixed']['seconds']:.3f} s, "
        f"FP64 {out['fp64']['seconds']:.3f} s")
    return out


def config2_overhead(lq, torch):
    """Plain FP64 CG at 24^4 (Haar links, m = 0.05, 1 RHS): time per iteration
    with graph replay and with direct launches, against the standalone FP64
    18-real D_oe; shows how much of an iteration is launch latency at a size
    where each kernel runs only tens of microseconds."""
    import synth
    L = (24, 24, 24, 24)
    g = lq.Geometry(L)
    U64 = lq.pack_links(g, torch.from_numpy(synth.links_haar(L, 102)).to("cuda"))
    b = lq.pack_spinor(g, torch.from_numpy(synth.gaussian_even_source(L, 1, 202)).to("cuda"), 0)
    out = {}
    for name, graph in (("graph", 1), ("direct", 0)):
        p = lq.solver_params(mass=0.05, tol=1e-10, use_graph=graph)
        lq.cg(g, p, U64, b)
        torch.cuda.synchronize()
        t0 = time.time()
        _, _, st = lq.cg(g, p, U64, b)
        torch.cuda.synchronize()
        dt = time.time() - t0
        out[name] = dict(seconds=dt, iters=st[0]["iters"],
                         us_per_iter=1e6 * dt / max(st[0]["iters"], 1),
                         true_rel_residual=st[0]["true_rel_residual"])
    x = torch.randn(1, 3, g.Vh, dtype=torch.complex128, device="cuda")
    y = torch.empty_like(x)
    out["doe_fp64_18_us"] = 1000 * event_time_ms(lambda: lq.doe(g, U64, x, out=y), 20)
    log(f"config 2 (24^4 FP64 CG): {out['graph']['us_per_iter']:.1f} us/iter with graphs, "
        f"{out['direct']['us_per_iter']:.1f} direct")
    return out


def rhmc_heatbath(lq, torch, g, U64, mass, nrhs, degree=14, seed=205):
    """RHMC pseudofermion heatbath and accept/reject action on the workload
    lattice: minimax x^(1/8) and x^(-1/4) of the given degree on the spectral
    interval [m^2, m^2 + 16] (Remez, host); phi = r_{1/8}(A) xi for nrhs
    Gaussian xi (mixed-precision multi-shift solve + combination kernel), then
    S = phi^dag r_{-1/4}(A) phi.  Reports the times, the identity
    S / |xi|^2 - 1 (bounded by 2 eps(1/8) + eps(-1/4) + solver error) and the
    combination kernel's algorithmic bandwidth."""
    import synth
    L = tuple(g.L)
    lo, hi = lq.spectral_bounds(mass)
    t0 = time.time()
    e = lq.minimax(0.125, lo, hi, degree)
    q = lq.minimax(-0.25, lo, hi, degree)
    t_remez = time.time() - t0
    xi = lq.pack_spinor(g, torch.from_numpy(synth.gaussian_even_source(L, nrhs, seed)).to("cuda"),
                        0)
    p = lq.solver_params(mass=mass, tol=1e-10, inner_prec=lq.F32, inner_fmt=lq.LINKS12,
                         reliable_interval=100, use_graph=1)
    lq.pseudofermion_heatbath(g, p, U64, e, xi)  # tuning and graph capture for this shape
    torch.cuda.synchronize()
    t0 = time.time()
    phi, st1 = lq.pseudofermion_heatbath(g, p, U64, e, xi)
    torch.cuda.synchronize()
    t_hb = time.time() - t0
    t0 = time.time()
    S, X, st2 = lq.rational_action(g, p, U64, q, phi)
    torch.cuda.synchronize()
    t_act = time.time() - t0
    xi2 = float((xi.abs() ** 2).sum().item())
    y = torch.empty_like(phi)
    ms = event_time_ms(lambda: lq.rational_combine(g, q.alpha0, q.alpha, phi, X, out=y), 20)
    nbytes = g.Vh * 48 * nrhs * (q.degree + 2)  # b and every X_i read once, y written
    del X, y
    out = dict(degree=degree, interval=[lo, hi], remez_s=t_remez,
               eps_eighth=e.max_rel_error, eps_quarter=q.max_rel_error,
               heatbath_s=t_hb, action_s=t_act,
               identity_dev=abs(S / xi2 - 1.0),
               identity_bound=2 * e.max_rel_error + q.max_rel_error,
               max_true_rel_residual=max(s["true_rel_residual"] for st in (st1, st2)
                                         for row in st for s in row),
               combine_us=1000 * ms, combine_GBps=nbytes / (ms * 1e-3) / 1e9,
               combine_frac_hbm_peak=nbytes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS)
    log(f"RHMC heatbath ({nrhs} RHS, degree {degree}): {t_hb:.3f} s, action {t_act:.3f} s, "
        f"|S/|xi|^2 - 1| = {out['identity_dev']:.2e}, combine {out['combine_GBps']:.0f} GB/s")
    return out


def rhmc_trajectory_bench(lq, torch, g48, U48):
    """RHMC trajectories on a 16^4 lattice (beta = 4.0, m = 0.1, one
    pseudofermion, degree-12 rational approximations, mixed-precision solves).
    The start (links exp(0.3 i H)) is far from equilibrium, so it is first
    thermalised by 40 pure-gauge MD trajectories (tau = 1, 10 Omelyan steps,
    fresh momenta, no accept/reject: thermalisation only, not part of a
    Markov chain).  Then full trajectories (heatbath, tau = 1 of gauge +
    fermion force, accept/reject with u = 0.5) at 20 and 40 Omelyan steps
    (dH(20) / dH(40) ~ 4 for the second-order scheme) and the multi-step
    scheme (10 outer fermion steps, 4 gauge substeps each): time, dH and the
    accept decision.  Then the tree-level Symanzik gauge force kernel alone on
    the workload lattice: 85 SU(3) products (198 flops each) per link, against
    the FP64 vector peak."""
    import synth
    L = (16, 16, 16, 16)
    g = lq.Geometry(L)
    beta, m = 4.0, 0.1
    lo, hi = lq.spectral_bounds(m)
    e8 = lq.minimax(0.125, lo, hi, 12)
    q4 = lq.minimax(-0.25, lo, hi, 12)
    p = lq.solver_params(mass=m, tol=1e-10, inner_prec=lq.F32, inner_fmt=lq.LINKS12,
                         use_graph=1)
    U0 = lq.pack_links(g, torch.from_numpy(synth.links_exp(L, 0.3, 601)).to("cuda"))
    gforce = lambda Ux, F: lq.gauge_force(g, Ux, beta, out=F)
    t0 = time.time()
    for k in range(40):
        Hk = lq.pack_links(g, torch.from_numpy(synth.momenta(L, 700 + k)).to("cuda"))
        lq.md_integrate(g, U0, Hk, 1.0, 10, gforce)
    torch.cuda.synchronize()
    therm_s = time.time() - t0
    H0 = lq.pack_links(g, torch.from_numpy(synth.momenta(L, 602)).to("cuda"))
    xi = lq.pack_spinor(g, torch.from_numpy(synth.gaussian_even_source(L, 1, 603)).to("cuda"), 0)
    lq.rhmc_trajectory(g, p, U0.clone(), beta, e8, q4, xi, H0.clone(), u=0.5, tau=0.05,
                       nsteps=1)  # tuning and graph capture at this shape
    res = {}
    for key, n, sub in ((20, 20, 1), (40, 40, 1), ("nested", 10, 4)):
        torch.cuda.synchronize()
        t0 = time.time()
        r = lq.rhmc_trajectory(g, p, U0.clone(), beta, e8, q4, xi, H0.clone(), u=0.5, tau=1.0,
                               nsteps=n, gauge_substeps=sub)
        torch.cuda.synchronize()
        res[key] = (time.time() - t0, r)
    F = lq.empty_links(g48, lq.F64, lq.LINKS18, "cuda")
    ms = event_time_ms(lambda: lq.gauge_force(g48, U48, 5.0, out=F), 10)
    flops = 8 * g48.Vh * 85 * 198
    # stout smearing (one level) and its chain-rule step on the workload lattice
    chain = lq.stout_smear(g48, U48, 0.15)
    ms_smear = event_time_ms(lambda: lq.stout_smear(g48, U48, 0.15), 10)
    ms_chain = event_time_ms(lambda: lq.stout_force(g48, chain, 0.15, F, mode=1), 5)
    del F, chain
    out = dict(lattice=list(L), beta=beta, mass=m, tau=1.0, integrator="omelyan",
               thermalisation="40 pure-gauge MD trajectories (tau 1, 10 steps, no "
                              "accept/reject)", thermalisation_s=therm_s,
               seconds_20_steps=res[20][0], seconds_40_steps=res[40][0],
               dH_20=res[20][1]["dH"], dH_40=res[40][1]["dH"],
               dH_ratio=res[20][1]["dH"] / res[40][1]["dH"],
               accepted_20=res[20][1]["accepted"], accepted_40=res[40][1]["accepted"],
               force_evaluations_20=res[20][1]["force_evaluations"],
               nested_10x4=dict(seconds=res["nested"][0], dH=res["nested"][1]["dH"],
                                accepted=res["nested"][1]["accepted"],
                                fermion_force_evaluations=res["nested"][1]["force_evaluations"]),
               gauge_force_48x4_ms=ms, gauge_force_TFLOPs=flops / (ms * 1e-3) / 1e12,
               gauge_force_frac_fp64_peak=flops / (ms * 1e-3) / 1e12 / 78.6,
               stout_smear_48x4_ms=ms_smear, stout_chain_rule_48x4_ms=ms_chain)
    log(f"RHMC trajectory 16^4: {res[20][0]:.2f} s (20 Omelyan steps), dH {out['dH_20']:.3e} / "
        f"{out['dH_40']:.3e} at 20 / 40 steps (accepted {out['accepted_20']} / "
        f"{out['accepted_40']}), nested 10x4 dH {out['nested_10x4']['dH']:.3e}; gauge force "
        f"48^4 {ms:.2f} ms ({out['gauge_force_TFLOPs']:.1f} TFLOP/s)")
    return out


def force_roofline(lq, torch, g, U64, al, X):
    """The fermion force kernel on the step's solutions (K = npf x nshift
    pairs), event-timed: per odd site and pair 8 SU(3) mat-vecs of chi = D_oe X
    (8 x 66 flops + 7 x 6 adds) and 8 outer products (8 x 72), FP64; bytes: the
    X vectors once (48 B per even site and pair), the links once (2 x 144 B
    per odd site) and the output once (2 x 144 B).  Its roof is the larger of
    bytes / 8 TB/s and flops / 78.6 TFLOP/s (FP64 vector peak)."""
    F = lq.empty_links(g, lq.F64, lq.LINKS18, "cuda")
    ms = event_time_ms(lambda: lq.fermion_force(g, U64, al, X, mode=0, out=F), 10)
    K = X.shape[0] * X.shape[1]
    flops = g.Vh * K * (8 * 66 + 7 * 6 + 8 * 72)
    byts = g.Vh * (K * 48 + 2 * 144 * 4 + 2 * 144 * 4)
    roof_ms = max(byts / 8e12, flops / 78.6e12) * 1e3
    del F
    return dict(pairs=K, ms=ms, TFLOPs=flops / (ms * 1e-3) / 1e12, GBps=byts / (ms * 1e-3) / 1e9,
                roof_ms=roof_ms, frac_of_roof=roof_ms / ms, bound="fp64-alu" if
                flops / 78.6e12 > byts / 8e12 else "hbm")


def stencil_ab(lq, torch):
    """A/B of the FP32 12-real 8-RHS D_oe at 48^4 (Haar links, seed 104, random
    right-hand sides): the tuned k_dslash against the t-march and matrix-core
    variants pinned in several launch shapes; 3 warm-ups + 20 event-timed
    launches each, the largest relative difference to the tuned result, and
    the tuned configuration (read back from a private tuning-cache file)."""
    import tempfile
    import synth
    L = (48, 48, 48, 48)
    g = lq.Geometry(L)
    U64 = lq.pack_links(g, torch.from_numpy(synth.links_haar(L, 104)).to("cuda"))
    Ul = lq.convert_links(g, U64, lq.F64, lq.LINKS18, lq.F32, lq.LINKS12)
    del U64
    gen = torch.Generator(device="cuda").manual_seed(7)
    x = torch.randn(8, 3, g.Vh, dtype=torch.complex64, device="cuda", generator=gen)
    cache = os.path.join(tempfile.mkdtemp(), "tune.txt")
    os.environ["LQCD_TUNE_CACHE"] = cache
    byts = g.Vh * dslash_bytes_per_site(lq.F32, lq.LINKS12, 8)
    runs = [("tuned", None),
            ("t_march_tm6_tp2_b64", "64,8,1,0,1,0,0,0,0,0,1,6,2"),
            ("t_march_tm12_tp4_b128", "128,8,1,0,1,0,0,0,0,0,1,12,4"),
            ("mfma_b256_lex", "256,8,1,0,1,0,0,0,0,0,1,0,2,1"),
            ("mfma_b256_tz6", "256,8,1,6,1,0,0,0,0,0,1,0,2,1"),
            ("mfma_b128_tz6_ty24", "128,8,1,6,1,0,0,0,0,24,1,0,2,1"),
            ("mfma_b64_tz12_ty24", "64,8,1,12,1,0,0,0,0,24,1,0,2,1")]
    out, ref = {}, None
    for name, cfg in runs:
        if cfg:
            os.environ["LQCD_DSLASH_CFG"] = cfg
        else:
            os.environ.pop("LQCD_DSLASH_CFG", None)
        y = torch.empty_like(x)
        ms = event_time_ms(lambda: lq.doe(g, Ul, x, out=y), 20)
        if ref is None:
            ref = y
        d = float(((y - ref).abs().max() / ref.abs().max()).item())
        out[name] = dict(cfg=cfg, us=1000 * ms, GBps=byts / (ms * 1e-3) / 1e9,
                         max_rel_diff_vs_tuned=d)
        log(f"stencil A/B {name}: {1000 * ms:.1f} us, diff {d:.1e}")
    os.environ.pop("LQCD_DSLASH_CFG", None)
    os.environ.pop("LQCD_TUNE_CACHE", None)
    out["tuned"]["cfg"] = open(cache).read().strip().split(";")[-1] if os.path.exists(cache) else None
    return out


def cpu_baseline(w, U, phi, sig, gpu_iters_per_rhs, gpu_shift_updates_per_rhs, X0=None,
                 budget_s=20.0):
    """Oracle multi-shift CG timed on a bounded sample: a few iterations on one
    right-hand side of the same lattice with all shifts active and with the
    base shift alone, which gives the oracle's cost per iteration and per
    active shifted system; the estimate for the whole batch weights them with
    the GPU run's iteration and active-shift counts (the oracle freezes
    converged shifts the same way).  Also times the oracle's D_oe on all host
    threads and on one, and recomputes with the oracle the FP64 true residual
    of the GPU's solutions for the first right-hand side (X0: natural layout
    [nshift][V][3])."""
    import numpy as np
    import oracle
    L = w["L"]
    threads = len(os.sched_getaffinity(0))
    oracle.set_threads(threads)
    ts = []
    for _ in range(3):
        t0 = time.time()
        oracle.doe(L, U, phi[0])
        ts.append(time.time() - t0)
    doe_all = sorted(ts)[1]
    oracle.set_threads(1)
    t0 = time.time()
    oracle.doe(L, U, phi[0])
    doe_one = time.time() - t0
    oracle.set_threads(threads)
    check = None
    if X0 is not None:
        tr = [oracle.true_residual(L, U, w["mass"], float(sg), phi[0], X0[s])
              for s, sg in enumerate(sig)]
        check = {"rhs": 0, "shifts": len(tr), "max_true_rel_residual": float(np.max(tr)),
                 "all_below_1e-10": bool(np.max(tr) <= 1e-10)}

    def per_iteration(sigmas, n):
        t0 = time.time()
        oracle.cg_multishift(L, U, w["mass"], sigmas, phi[0], tol=1e-10, max_iter=1,
                             verify=False)
        t1 = time.time() - t0
        t0 = time.time()
        oracle.cg_multishift(L, U, w["mass"], sigmas, phi[0], tol=1e-10, max_iter=n,
                             verify=False)
        tn = time.time() - t0
        return (tn - t1) / (n - 1), t1

    _, t1 = per_iteration(sig, 2)
    n = max(2, min(5, int(budget_s / 2 / max(t1, 1e-3))))
    it_all, _ = per_iteration(sig, n)
    it_base, _ = per_iteration(sig[:1], n)
    per_shift = max(it_all - it_base, 0.0) / max(len(sig) - 1, 1)
    est_rhs = (gpu_iters_per_rhs * it_base
               + max(gpu_shift_updates_per_rhs - gpu_iters_per_rhs, 0) * per_shift)
    est_solve = est_rhs * w["nrhs"]
    value = w["nrhs"] * w["nshift"] / est_solve
    return {
        "value": value, "unit": "shift-solves/s", "cores": threads, "kind": "oracle",
        "sample": (f"estimate: oracle FP64 multi-shift CG on 1 RHS of the same "
                   f"{'x'.join(map(str, L))} lattice, {n} iterations with all {w['nshift']} "
                   f"shifts ({it_all:.3f} s/iter) and {n} with the base shift alone "
                   f"({it_base:.3f} s/iter) on {threads} threads "
                   f"({platform.processor() or platform.machine()}), weighted by the GPU run's "
                   f"{gpu_iters_per_rhs} iterations and {gpu_shift_updates_per_rhs} active "
                   f"shifted-system iterations per RHS, x {w['nrhs']} RHS"),
        "seconds_per_iteration_all_shifts": it_all,
        "seconds_per_iteration_base_only": it_base,
        "seconds_per_active_shift_iteration": per_shift,
        "estimated_solve_s": est_solve,
        "doe_s": {"threads": threads, "all_threads": doe_all, "one_thread": doe_one},
        "oracle_true_residual_check": check,
    }


def oracle_config3_solve():
    """The oracle's whole multi-shift solve of the 32^4 single-RHS configuration
    (links exp(0.5iH), m = 0.02, 12 shifts, tol 1e-10, verification and
    refinement included), timed on every host thread: a measured CPU
    time-to-solution next to the GPU's for the same systems."""
    import numpy as np
    import oracle
    w = WORKLOADS["c3"]
    U, phi, sig, _ = make_inputs(w)
    threads = len(os.sched_getaffinity(0))
    oracle.set_threads(threads)
    t0 = time.time()
    _, st, (its, ref), tr = oracle.cg_multishift(w["L"], U, w["mass"], sig, phi[0], tol=1e-10)
    sec = time.time() - t0
    log(f"oracle config 3 solve: {sec:.1f} s on {threads} threads ({its} iterations)")
    return {"seconds": sec, "cores": threads, "status": st, "iters": its, "refine_iters": ref,
            "max_true_rel_residual": float(np.max(tr)),
            "what": "oracle FP64 multi-shift CG, 32^4, 1 RHS x 12 shifts, tol 1e-10, measured"}


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", choices=sorted(WORKLOADS), default="c4")
    ap.add_argument("--no-fp64-baseline", action="store_true")
    ap.add_argument("--stencil-ab", action="store_true",
                    help="only the 48^4 FP32 8-RHS D_oe A/B: tuned VALU stencil vs the "
                         "t-march and matrix-core variants")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-rhmc", action="store_true",
                    help="skip the RHMC heatbath / action measurement")
    ap.add_argument("--rhmc-only", action="store_true",
                    help="only the RHMC measurements (heatbath, action, trajectory, gauge "
                         "force, stout smearing, fermion force), for profiling them")
    ap.add_argument("--retune", action="store_true",
                    help="tune every stencil shape from scratch instead of starting from "
                         "the shipped MI355X tuning cache")
    ap.add_argument("--profile-kernels", action="store_true",
                    help="one solve + standalone D_oe + copy kernel, for counter runs")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(halo exchange across GPUs is out of scope); run with --gpus 1", flush=True)
        sys.exit(2)

    import numpy as np
    import torch
    import paper_1801_01473_amd as lq

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", flush=True)
        sys.exit(2)
    torch.cuda.set_device(0)
    if args.stencil_ab:
        print(json.dumps({"stencil_ab": stencil_ab(lq, torch)}), flush=True)
        return
    # The tuner's choices are read back from the tuning cache: a private file
    # unless the caller names one.  The private file starts from the shipped
    # MI355X cache (the configurations the committed counters were taken
    # with; its keys name gfx950 and 256 CUs, so other devices tune afresh),
    # unless --retune asks for tuning from scratch.
    tune_cache = os.environ.get("LQCD_TUNE_CACHE") or None
    if tune_cache is None:
        import atexit
        import shutil
        import tempfile
        tmp = tempfile.mkdtemp()
        atexit.register(shutil.rmtree, tmp, True)
        tune_cache = os.path.join(tmp, "tune.txt")
        if not args.retune:
            shutil.copyfile(SHIPPED_TUNE_CACHE, tune_cache)
        os.environ["LQCD_TUNE_CACHE"] = tune_cache
    w = WORKLOADS[args.workload]
    L = w["L"]
    g = lq.Geometry(L)
    nrhs, nshift = w["nrhs"], w["nshift"]
    U, phi, sig, al = make_inputs(w)
    U_dev = torch.from_numpy(U).to("cuda")
    phi_p = lq.pack_spinor(g, torch.from_numpy(phi).to("cuda"), 0)
    torch.cuda.synchronize()

    params = lq.solver_params(mass=w["mass"], tol=1e-10, inner_prec=lq.F32,
                              inner_fmt=lq.LINKS12, reliable_interval=100, use_graph=1)
    dom = dict(prec=lq.F32, fmt=lq.LINKS12, nrhs=nrhs)

    if args.rhmc_only:
        U64 = lq.pack_links(g, U_dev)
        rh = rhmc_heatbath(lq, torch, g, U64, w["mass"], nrhs)
        tr = rhmc_trajectory_bench(lq, torch, g, U64)
        # the fermion force on solutions of the step's shape (seeded Gaussian
        # stand-ins: the kernel's cost does not depend on the values)
        gen = torch.Generator(device="cuda").manual_seed(11)
        Xs = torch.randn(nrhs, nshift, 3, g.Vh, dtype=torch.complex128, device="cuda",
                         generator=gen)
        ff = force_roofline(lq, torch, g, U64, al, Xs)
        del Xs
        log(f"fermion force {L[0]}x{L[1]}x{L[2]}x{L[3]}, {ff['pairs']} pairs: {ff['ms']:.2f} ms")
        print(json.dumps({"rhmc_heatbath": rh, "rhmc_trajectory": tr, "fermion_force": ff}),
              flush=True)
        return

    if args.profile_kernels:
        U64 = lq.pack_links(g, U_dev)
        lq.cg_multishift(g, params, U64, sig, phi_p)  # tuning + graph capture
        torch.cuda.synchronize()
        # small copy launches bracket the measured solve in the dispatch list
        lq.stream_bandwidth(1 << 20, 1)
        log("profiled solve")
        _, _, pst = lq.cg_multishift(g, params, U64, sig, phi_p)
        torch.cuda.synchronize()
        lq.stream_bandwidth(1 << 20, 1)
        Uin = lq.convert_links(g, U64, lq.F64, lq.LINKS18, dom["prec"], dom["fmt"])
        x = torch.randn(nrhs, 3, g.Vh, dtype=torch.complex64, device="cuda")
        y = torch.empty_like(x)
        for _ in range(5):
            lq.doe(g, Uin, x, out=y)
        x64 = torch.randn(1, 3, g.Vh, dtype=torch.complex128, device="cuda")
        y64 = torch.empty_like(x64)
        for _ in range(5):
            lq.doe(g, U64, x64, out=y64)
        cb, tb = lq.stream_bandwidth(1 << 30, 5)
        torch.cuda.synchronize()
        print(json.dumps({"profile_kernels": "done", "copy_bytes_per_array": 1 << 30,
                          "profiled_solve_iters_fp64": [r[0]["iters_fp64"] for r in pst],
                          "profiled_solve_iters": [r[0]["iters"] for r in pst],
                          "shift_window": pst[0][0]["shift_window"],
                          "shift_update_algorithmic_bytes": shift_update_bytes(g.Vh, pst)}),
              flush=True)
        return

    state = {}

    def step():
        t0 = time.time()
        U64 = lq.pack_links(g, U_dev)
        torch.cuda.synchronize()
        t1 = time.time()
        X, st, stats = lq.cg_multishift(g, params, U64, sig, phi_p)
        t2 = time.time()
        S = lq.action(g, 0.0, al, phi_p, X)
        F = lq.fermion_force(g, U64, al, X, mode=0)
        torch.cuda.synchronize()
        t3 = time.time()
        state.update(X=X, stats=stats, S=S, F=F, U64=U64,
                     t_pack=t1 - t0, t_solve=t2 - t1, t_force=t3 - t2)

    for i in range(args.warmup):
        log(f"warmup step {i + 1}/{args.warmup}")
        step()
    torch.cuda.synchronize()
    solve_times, force_times = [], []
    t_start = time.time()
    for i in range(args.steps):
        step()
        solve_times.append(state["t_solve"])
        force_times.append(state["t_force"])
        log(f"step {i + 1}/{args.steps}: solve {state['t_solve']:.3f} s, "
            f"action+force {state['t_force']:.3f} s")
    torch.cuda.synchronize()
    elapsed = time.time() - t_start
    ms_per_step = 1000.0 * elapsed / args.steps
    value = nrhs * nshift / (elapsed / args.steps)

    stats = state["stats"]
    max_tr = max(s["true_rel_residual"] for row in stats for s in row)
    all_conv = all(s["converged"] == 1 for row in stats for s in row)
    iters = [row[0]["iters"] for row in stats]
    refine = sum(s["refine_iters"] for row in stats for s in row)
    rel = [row[0]["reliable_updates"] for row in stats]

    # per-kernel timing of the same solve (HIP events around each launch, no graph)
    lq.kernel_timing(True)
    _, _, tstats = lq.cg_multishift(g, params, state["U64"], sig, phi_p)
    lq.kernel_timing(False)
    ktimes = lq.kernel_timing()
    kernels = kernel_table(g, nrhs, tstats, ktimes)
    force_line = force_roofline(lq, torch, g, state["U64"], al, state["X"])
    dominant = max(kernels, key=lambda k: kernels[k]["total_ms"])

    # time-to-1e-10: plain FP64 GPU multi-shift, one RHS at a time
    fp64 = None
    if not args.no_fp64_baseline:
        p64 = lq.solver_params(mass=w["mass"], tol=1e-10, inner_prec=lq.F64,
                               inner_fmt=lq.LINKS18, use_graph=1)
        U64 = state["U64"]
        lq.cg_multishift(g, p64, U64, sig, phi_p[0:1].contiguous())  # tune + graph
        torch.cuda.synchronize()
        t0 = time.time()
        it64, tr64 = [], []
        for j in range(nrhs):
            _, _, s64 = lq.cg_multishift(g, p64, U64, sig, phi_p[j:j + 1].contiguous())
            it64.append(s64[0][0]["iters"])
            tr64.append(max(s["true_rel_residual"] for s in s64[0]))
        torch.cuda.synchronize()
        t64 = time.time() - t0
        fp64 = dict(seconds=t64, iters=it64, max_true_residual=max(tr64))
        log(f"FP64 sequential baseline: {t64:.3f} s")
        # the same FP64 solve with the right-hand sides batched (18-real links, then
        # 12-real): separates the gain of batching from that of mixed precision
        fp64["batched"] = {}
        for fname, fmt in (("links18", lq.LINKS18), ("links12", lq.LINKS12)):
            pb = lq.solver_params(mass=w["mass"], tol=1e-10, inner_prec=lq.F64, inner_fmt=fmt,
                                  use_graph=1)
            lq.cg_multishift(g, pb, U64, sig, phi_p)  # tune + graph
            torch.cuda.synchronize()
            t0 = time.time()
            _, _, sb = lq.cg_multishift(g, pb, U64, sig, phi_p)
            torch.cuda.synchronize()
            fp64["batched"][fname] = dict(
                seconds=time.time() - t0, iters=sb[0][0]["iters"],
                max_true_rel_residual=max(s["true_rel_residual"] for row in sb for s in row))
        log(f"FP64 batched: {fp64['batched']['links18']['seconds']:.3f} s (18-real), "
            f"{fp64['batched']['links12']['seconds']:.3f} s (12-real)")
        # secondary context: each shift of the first RHS by its own plain FP64 CG
        lq.cg(g, p64, U64, phi_p[0:1].contiguous(), sigma=float(sig[-1]))  # graph capture
        torch.cuda.synchronize()
        t0 = time.time()
        cg_it = []
        for sg in sig:
            _, _, sc = lq.cg(g, p64, U64, phi_p[0:1].contiguous(), sigma=float(sg))
            cg_it.append(sc[0]["iters"])
        torch.cuda.synchronize()
        fp64["per_shift_cg_1rhs_s"] = time.time() - t0
        fp64["per_shift_cg_iters"] = cg_it
        log(f"per-shift FP64 CG, 1 RHS: {fp64['per_shift_cg_1rhs_s']:.3f} s")
        fp64["config3_32x4_1rhs"] = config3_m2(lq, torch)
        fp64["config2_24x4_cg"] = config2_overhead(lq, torch)

    # D_oe bandwidth (standalone, HIP events), STREAM ceiling
    copy_gbs, triad_gbs = lq.stream_bandwidth(1 << 30, 20)
    U64 = state["U64"]
    dsl = {}
    lat = "x".join(map(str, L))
    for name, (prec, fmt, n) in {
            "fp64_18_1rhs": (lq.F64, lq.LINKS18, 1),
            "fp64_12_1rhs": (lq.F64, lq.LINKS12, 1),
            "fp32_18_1rhs": (lq.F32, lq.LINKS18, 1),
            "fp32_12_1rhs": (lq.F32, lq.LINKS12, 1),
            f"fp32_12_{nrhs}rhs": (lq.F32, lq.LINKS12, nrhs),
            f"fp32_12d_{nrhs}rhs": (lq.F32, lq.LINKS12D, nrhs),
            f"fp32_12t_{nrhs}rhs": (lq.F32, lq.LINKS12T, nrhs),
            "fp32_12t_1rhs": (lq.F32, lq.LINKS12T, 1),
            "fp32_12d_1rhs": (lq.F32, lq.LINKS12D, 1),
            f"fp64_12_{nrhs}rhs": (lq.F64, lq.LINKS12, nrhs)}.items():
        Ul = U64 if (prec, fmt) == (lq.F64, lq.LINKS18) else lq.convert_links(
            g, U64, lq.F64, lq.LINKS18, prec, fmt)
        dsl[name] = dslash_entry(lq, torch, g, Ul, prec, fmt, n, copy_gbs,
                                 f"{lat}, workload links, {n} RHS")
        del Ul
    # the paper-sized FP64 check at 32^4 (links 604 MB, above the 256 MB MALL)
    g32 = lq.Geometry((32, 32, 32, 32))
    U32 = lq.pack_links(g32, torch.randn(4, g32.V, 3, 3, dtype=torch.complex128,
                                         device="cuda"))
    dsl["fp64_18_1rhs_32x4"] = dslash_entry(lq, torch, g32, U32, lq.F64, lq.LINKS18, 1,
                                            copy_gbs, "32^4, Gaussian 3x3 links (timing only)")
    del U32
    # the paper's own lattice (32^3 x 48, Sec. 5), where its FP64 Dirac figures are quoted
    gp = lq.Geometry((32, 32, 32, 48))
    Up = lq.pack_links(gp, torch.randn(4, gp.V, 3, 3, dtype=torch.complex128, device="cuda"))
    for name, fmt in (("fp64_18_1rhs_32x3x48", lq.LINKS18), ("fp64_12_1rhs_32x3x48", lq.LINKS12)):
        Ul = Up if fmt == lq.LINKS18 else lq.convert_links(gp, Up, lq.F64, lq.LINKS18, lq.F64, fmt)
        dsl[name] = dslash_entry(lq, torch, gp, Ul, lq.F64, fmt, 1, copy_gbs,
                                 "32^3x48 (the paper's lattice), Gaussian 3x3 links (timing only)")
        del Ul
    del Up
    rhmc = traj = None
    if not args.no_rhmc:
        rhmc = rhmc_heatbath(lq, torch, g, U64, w["mass"], nrhs)
        traj = rhmc_trajectory_bench(lq, torch, g, U64)
    kd = kernels[dominant]
    dom_cfg = tuned_config(tune_cache, L, dominant, nrhs)
    traffic, traffic_note = measured_traffic(dominant, dom_cfg)
    roof = {
        "kernel": f"{dominant} ({kd['kernel']})",
        "bound": "hbm",
        "achieved": kd["GBps"],
        "peak": HBM_PEAK_GBS,
        "unit": "GB/s",
        "frac": kd["GBps"] / HBM_PEAK_GBS,
        "traffic": traffic,
        "traffic_source": ("rocprofv3 FETCH_SIZE x 2.00 + WRITE_SIZE x 1.00 per launch from "
                           "profiles/dominant_kernel_traffic.json, taken with the stencil "
                           "sources whose sha256 it records and the tuned configuration it "
                           "names (null when either differs)"),
        "traffic_note": traffic_note,
        "tuned_configuration": dom_cfg,
        "algorithmic_bytes_per_launch": kd["bytes_per_launch"],
        "avg_launch_us": kd["avg_us"],
        "share_of_solve_kernel_time": kd["total_ms"] / sum(v["total_ms"] for v in kernels.values()),
        # the HBM rate the counter traffic implies at this run's launch time, next to the
        # box's STREAM copy: how much of the gap to the peak is re-fetch, how much rate
        "traffic_GBps": (traffic / (kd["avg_us"] * 1e-6) / 1e9) if traffic else None,
    }

    cpu = None
    if not args.no_cpu_baseline:
        log("timing the CPU oracle on a bounded sample")
        X0 = lq.unpack_spinor(g, state["X"][0], 0).cpu().numpy()
        upd = (sum(row[0]["shift_updates_fp64"] + row[0]["shift_updates_fp32"] for row in stats)
               / len(stats))
        cpu = cpu_baseline(w, U, phi, sig, int(round(np.mean(iters))), int(round(upd)), X0=X0)
        del X0
        if fp64 and fp64.get("config3_32x4_1rhs"):
            fp64["config3_32x4_1rhs"]["oracle"] = oracle_config3_solve()
            c3 = fp64["config3_32x4_1rhs"]
            c3["speedup_mixed_vs_oracle"] = c3["oracle"]["seconds"] / c3["mixed"]["seconds"]

    mixed_solve = float(np.median(solve_times))
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "shift-solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic (seeded generators in synth/: Haar links, Gaussian even-site sources)",
        "config": {"workload": w["name"], "lattice": list(L), "nrhs": nrhs, "nshift": nshift,
                   "mass": w["mass"], "tol": 1e-10, "inner": "fp32 12-real",
                   "reliable_interval": 100, "reliable_delta": 1e-3, "mixed_switch": 1e-3,
                   "shift_window": stats[0][0]["shift_window"]},
        "roofline": roof,
        "cpu_baseline": cpu,
        "time_to_1e10": {
            "mixed_batched_s": mixed_solve,
            "fp64_sequential_s": fp64["seconds"] if fp64 else None,
            "speedup_mixed_vs_fp64": (fp64["seconds"] / mixed_solve) if fp64 else None,
            "fp64_batched": fp64["batched"] if fp64 else None,
            "speedup_split": ({
                "batching_fp64_18": fp64["seconds"] / fp64["batched"]["links18"]["seconds"],
                "compression_fp64_12": (fp64["batched"]["links18"]["seconds"]
                                        / fp64["batched"]["links12"]["seconds"]),
                "mixed_precision": fp64["batched"]["links12"]["seconds"] / mixed_solve}
                if fp64 else None),
            "action_plus_force_s": float(np.median(force_times)),
            "fp64_per_shift_cg_1rhs_s": fp64["per_shift_cg_1rhs_s"] if fp64 else None,
            "fp64_per_shift_cg_iters": fp64["per_shift_cg_iters"] if fp64 else None,
            "config3_32x4_1rhs": fp64["config3_32x4_1rhs"] if fp64 else None,
            "config2_24x4_fp64_cg": fp64["config2_24x4_cg"] if fp64 else None,
        },
        "solver": {"iters_per_rhs": iters,
                   "fp64_phase_iters_per_rhs": [row[0]["iters_fp64"] for row in stats],
                   "shift_updates_fp64": sum(row[0]["shift_updates_fp64"] for row in stats),
                   "shift_updates_fp32": sum(row[0]["shift_updates_fp32"] for row in stats),
                   "shift_window": stats[0][0]["shift_window"],
                   "shift_update_algorithmic_GB": {
                       k: v / 1e9 for k, v in shift_update_bytes(g.Vh, stats).items()},
                   "reliable_updates_per_rhs": rel,
                   "refine_iters_total": refine, "max_true_rel_residual": max_tr,
                   "all_converged": all_conv,
                   "fp64_iters_per_rhs": fp64["iters"] if fp64 else None,
                   "fp64_max_true_rel_residual": fp64["max_true_residual"] if fp64 else None},
        "kernels": kernels,
        "dslash": dsl,
        "fermion_force": force_line,
        "rhmc_heatbath": rhmc,
        "rhmc_trajectory": traj,
        "stream": {"copy_GBps": copy_gbs, "triad_GBps": triad_gbs},
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
