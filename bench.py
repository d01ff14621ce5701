"""Benchmark: particle-element passes/s of FP64 thin-lattice tracking on one GPU.

Default workload (the dynamic-aperture scan): a 20,000-element errored thin
ring (2000 FODO cells with order-10 multipoles, 8 RF cavities, circular
apertures), 100,000 protons at 450 GeV on a 2000 x 50 polar grid of 0-10
sigma at delta = 2.7e-4, tracked 10,000 turns = 10 steps of 1,000 turns.
Inputs are seeded and synthetic and are resident in HBM before timing.

Prints ONE JSON line with the throughput, a roofline entry for the dominant
kernel (the tracking kernel, FP64 vector ALU bound) and the CPU oracle timed
on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FP64_VECTOR_PEAK_TFLOPS = 78.6   # 256 CU x 128 FP64 FLOP/clk x 2.4 GHz
KERNEL_NAMES = {4: "k_track4 (element interpreter)"}
for _s in range(8):
    KERNEL_NAMES[5 + _s] = "xtm_line (per-line generated kernel, %s workgroups, parameters %s)" % (
        "one-wave" if _s & 1 else "256-lane",
        ("read at use", "grouped per element", "fetched one element ahead",
         "fetched one element ahead, one loss test per cell")[_s >> 1])
KERNEL_NAMES[13] = ("xtm_line (per-line generated kernel, one-wave workgroups, parameters "
                    "fetched one element ahead, two particles per lane)")
KERNEL_NAMES[14] = ("xtm_line (per-line generated kernel, one-wave workgroups, parameters "
                    "fetched one element ahead, long cells)")

# HBM bytes per tracking-kernel launch, averaged over the timed region of one
# FETCH_SIZE and one WRITE_SIZE counter pass of this benchmark, each scaled by
# what the same counter reads for a plain 1 GiB device copy (x2.000, x1.000).
# A figure holds only for the workload, particle count, turns per step and
# kernel it was taken on, and for the kernel sources: the key carries a hash
# of the sources the per-line kernel is generated from, and any change to them
# makes the bench report no traffic until the counters are taken again.  The
# figure is per launch, so it does not depend on the number of timed steps.
TRAFFIC_SOURCES = ("xtm_jit.cpp", "xtm_maps.h")
MEASURED_TRAFFIC = {
    # (workload, particles, turns per step, kernel variant, source hash):
    #     (bytes per launch, profile)
    ("cfg2", 100000, 1000, 14, "8fc270e379fe13d4"):
        (21432430.0, "profiles/xtm_line_cfg2_hbm_counters.txt"),
    ("cfg1sat", 1048576, 1000, 14, "8fc270e379fe13d4"):
        (189155935.0, "profiles/xtm_line_cfg2_hbm_counters.txt"),
}


def kernel_source_hash() -> str:
    import hashlib
    h = hashlib.sha256()
    for f in TRAFFIC_SOURCES:
        with open(os.path.join(ROOT, "paper_2310_00317_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


# Algorithmic FLOPs per element application: the per-element counts of the
# method's formulas with a square root, a division, a sine and a compare
# counted as one operation and a fused multiply-add as two (drift 23,
# multipole of order N 8 N + 2, RF 17, shift 2, rotation 12, aperture 3).  Two
# counts are this project's: the curvature terms of a thin bend (11) and the
# expanded drift (20).
def element_flops(el) -> np.ndarray:
    from paper_2310_00317_amd import inputs as I
    f = np.zeros(len(el))
    for i, e in enumerate(el):
        t = int(e["type"])
        if t == I.DRIFT:
            f[i] = 23
        elif t == I.DRIFT_EXPANDED:
            f[i] = 20
        elif t == I.MULTIPOLE:
            f[i] = 8 * int(e["order"]) + 2 + (11 if e["hxl"] != 0 else 0)
        elif t == I.RF:
            f[i] = 17
        elif t == I.XYSHIFT:
            f[i] = 2
        elif t == I.SROTATION:
            f[i] = 12
        elif t in (I.AP_CIRCLE, I.AP_ELLIPSE, I.AP_RECT):
            f[i] = 3
        elif t in (I.QUADRUPOLE, I.SBEND):
            # N order-1 kicks (with curvature for a bend) and N + 1 drifts
            n = int(e["p"][2])
            f[i] = (n + 1) * 23 + n * (10 + (11 if t == I.SBEND else 0))
    return f


# Algorithmic HBM bytes per pass of the one-launch-per-element baseline: the
# state word and the FP64 fields each map reads and writes (drift 60 + 24,
# multipole 36 + 16, aperture 20, RF 20 + 32, shift 20 + 16, rotation 36 + 32,
# marker 4); elements read and written whole: 2 x 72 + 4.
def element_bytes(el) -> np.ndarray:
    from paper_2310_00317_amd import inputs as I
    b = np.full(len(el), 148.0)
    for i, e in enumerate(el):
        t = int(e["type"])
        if t == I.DRIFT:
            b[i] = 84
        elif t == I.MULTIPOLE and e["hxl"] == 0 and e["length"] <= 0:
            b[i] = 52
        elif t in (I.AP_CIRCLE, I.AP_ELLIPSE, I.AP_RECT):
            b[i] = 20
        elif t == I.RF:
            b[i] = 52
        elif t == I.XYSHIFT:
            b[i] = 36
        elif t == I.SROTATION:
            b[i] = 68
        elif t == I.MARKER:
            b[i] = 4
    return b


def workload(name: str, n_override: int | None, radiation: int = 2):
    from paper_2310_00317_amd import inputs as I
    if name == "cfg2":
        el = I.cfg2_lattice()
        c, _, _ = I.cfg2_grid(2000, 50, 10.0)
        if n_override:
            c = c[:n_override]   # the first rays of the grid (a timing subset)
        desc = ("DA scan: 20,000-element errored thin ring (order-10 multipoles, 8 RF, "
                "circular apertures), 100,000 protons at 450 GeV on a 2000x50 polar grid "
                "0-10 sigma, delta=2.7e-4")
        return el, c, I.PROTON_450GEV, desc, 1000, 10
    if name == "cfg1":
        el = I.cfg1_lattice()
        c = I.cfg1_particles(n_override or 1000)
        desc = f"thin FODO ring, 801 elements, {len(c)} Gaussian protons at 450 GeV"
        return el, c, I.PROTON_450GEV, desc, 100, 1
    if name == "cfg1sat":
        el = I.cfg1_lattice()
        c = I.cfg1_particles(n_override or (1 << 20))
        desc = f"thin FODO ring, 801 elements, {len(c)} Gaussian protons at 450 GeV"
        return el, c, I.PROTON_450GEV, desc, 100, 1
    if name == "cfg5":
        import paper_2310_00317_amd as P
        el = I.cfg5_lattice()
        n = n_override or 1_000_000
        # electrons matched to the ring's 6D normal form (closed orbit and
        # eigenvectors with the mean energy loss) at the given emittances
        nf = P.twiss6d(P.Lattice(el, I.ELECTRON_45GEV6), radiation=1)
        c = P.matched_gaussian(nf, I.ELECTRON_45GEV6, I.CFG5_EMITTANCES, I.standard_normals(n))
        desc = (f"electron ring, 20,000 thin elements (bends with radiation length, 8 RF), "
                f"{len(c)} electrons at 45.6 GeV matched to the 6D normal form, " +
                ("photon-by-photon radiation (Poisson photon counts, universal spectrum, "
                 "Philox deviates)" if radiation == 3 else
                 "mean + quantum radiation (Philox deviates)"))
        return el, c, I.ELECTRON_45GEV6, desc, 10, 2
    if name == "cfg3":
        counts = I.cfg3_counts()
        if n_override:
            counts = np.maximum(1, (counts * (n_override / counts.sum())).astype(np.int64))
        els, cs = [], []
        for v, n in enumerate(counts):
            e, c = I.cfg3_variant(v, int(n))
            els.append(e)
            cs.append(c)
        desc = (f"64 errored variants of the thin FODO ring (801 elements each), "
                f"{int(counts.sum())} Gaussian protons in total (2,000-50,000 per variant), "
                "one batched launch per chunk")
        return els, (np.concatenate(cs), counts), I.PROTON_450GEV, desc, 200, 2
    if name == "thick":
        el = I.thick_ring()
        c = I.gaussian_particles(n_override or (1 << 20), seed=23,
                                 sigmas=np.array([1.5e-3, 5e-5, 1.2e-3, 5e-5, 0.1, 1e-4]))
        desc = (f"ring of thick quadrupoles and sector bends sliced into drift-kick-drift "
                f"slices (16 cells, 144 elements, 784 after slicing), {len(c)} Gaussian "
                "protons at 450 GeV")
        return el, c, I.PROTON_450GEV, desc, 100, 1
    raise SystemExit(f"unknown workload {name}")


def cpu_baseline(el, c, ref, sample_every: int, turns: int, radiation: int = 0, seed: int = 0):
    import oracle
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    threads = max(1, min(threads, os.cpu_count() or 1))
    sub = c[::sample_every]
    p = oracle.init(sub, ref)
    t = time.perf_counter()
    passes = oracle.track(el, ref, p, turns, nthreads=threads, radiation=radiation, seed=seed)
    dt = time.perf_counter() - t
    return {"value": passes / dt, "unit": "passes/s", "cores": threads, "kind": "oracle",
            "sample": f"every {sample_every}th particle ({len(sub)}) x {turns} turns "
                      f"= {passes} passes in {dt:.1f} s"}


def refine_bench(args):
    """Loss-location refinement of the DA-scan ring's losses: the 100,000-particle
    grid tracked (untimed) for --turns-per-step turns, then the refinement
    kernel launched --steps times on the same losses, each launch timed with
    HIP events on its stream.  Algorithmic FLOPs per polygon test: the
    interpolation of the M vertices (x and y: a subtraction and a fused
    multiply-add each, 6 M), the point on the path and the weight (10) and
    two straddling edges (16)."""
    import torch
    import paper_2310_00317_amd as P
    I = P.inputs
    el = I.cfg2_lattice()
    coords, _, _ = I.cfg2_grid()
    ref = I.PROTON_450GEV
    turns = args.turns_per_step or 1000
    steps = args.steps if args.steps is not None else 3
    M, ds, nb = args.refine_vertices, args.refine_ds, args.refine_bisect
    n = len(coords)
    print(f"[bench] refine: {n} particles, {len(el)} elements, {turns} turns tracked, "
          f"M={M} ds={ds} n_bisect={nb}", file=sys.stderr, flush=True)
    lat = P.Lattice(el, ref)
    parts = P.Particles(n, ref).init(coords)
    P.track(lat, parts, turns)
    torch.cuda.synchronize()
    st = torch.cuda.current_stream()
    for _ in range(args.warmup):
        P.refine_losses(lat, parts, M, ds, nb, stream=st)
    torch.cuda.synchronize()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(steps)]
    t0 = time.perf_counter()
    out = None
    for a, b in evs:
        a.record(st)
        out = P.refine_losses(lat, parts, M, ds, nb, stream=st, with_tests=True)
        b.record(st)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kernel_ms = sum(a.elapsed_time(b) for a, b in evs)
    s_loss, _, _, tests = out
    state = parts.state[:n]
    n_lost = int((state == 0).sum().item())
    total_tests = int(tests.to(torch.int64).sum().item())
    flops_per_test = 6 * M + 26
    avg_ms = kernel_ms / max(steps, 1)
    value = n_lost / (avg_ms / 1e3) if avg_ms > 0 else 0.0
    achieved = total_tests * flops_per_test / (avg_ms / 1e3) / 1e12 if avg_ms > 0 else 0.0
    out_line = {
        "metric": "refined loss locations/s (FP64)",
        "value": value,
        "unit": "losses/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": args.warmup,
        "ms_per_step": avg_ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "loss-location refinement of the DA-scan ring (20,000 elements, "
                               f"100,000-particle grid tracked {turns} turns)",
                   "n_particles": n, "n_lost": n_lost, "n_vertices": M, "ds": ds,
                   "n_bisect": nb, "polygon_tests": total_tests, "wall_s": wall},
        "roofline": {"bound": "alu", "kernel": "k_refine (one wave per lost particle)",
                     "achieved": achieved, "peak": FP64_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / FP64_VECTOR_PEAK_TFLOPS, "traffic": None,
                     "flops_per_test": flops_per_test, "avg_launch_ms": avg_ms,
                     "launches": steps},
    }
    if not args.no_cpu_baseline:
        import oracle
        print("[bench] timing the CPU oracle on a sample of the losses", file=sys.stderr,
              flush=True)
        g = parts.to_numpy()
        lost = np.nonzero(g["state"] == 0)[0]
        pick = lost[:: max(1, len(lost) // 2000)]
        o = oracle.Particles(len(pick))
        for f in oracle.FLOAT_FIELDS + oracle.INT_FIELDS:
            getattr(o, f)[:] = g[f][pick]
        o.particle_id[:] = g["particle_id"][pick]
        t = time.perf_counter()
        oracle.refine_losses(el, ref, o, M, ds, nb)
        dt = time.perf_counter() - t
        out_line["cpu_baseline"] = {"value": len(pick) / dt, "unit": "losses/s", "cores": 1,
                                    "kind": "oracle",
                                    "sample": f"{len(pick)} of the {len(lost)} losses "
                                              f"(every {max(1, len(lost) // 2000)}th) in {dt:.1f} s"}
    print(json.dumps(out_line), flush=True)


def twiss_bench(args):
    """Optics by tracking of the 20,000-element DA-scan ring: the whole
    xtm_twiss call (closed-orbit Newton steps and the final 11-particle
    recorded turn on the GPU, the 4x4 algebra and the table on the host),
    timed on the host clock after one warmup call.  Algorithmic FLOPs: the
    element maps of the tracked turns (apertures are not applied)."""
    import torch
    import paper_2310_00317_amd as P
    I = P.inputs
    el = I.cfg2_lattice()
    ref = I.PROTON_450GEV
    steps = args.steps if args.steps is not None else 5
    lat = P.Lattice(el, ref)
    for _ in range(max(args.warmup, 0)):
        P.twiss(lat)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    tw = None
    for _ in range(steps):
        tw = P.twiss(lat)
    wall = time.perf_counter() - t0
    ms = wall / steps * 1e3
    f = element_flops(el)
    f[np.isin(el["type"], (I.AP_CIRCLE, I.AP_ELLIPSE, I.AP_RECT))] = 0.0
    turns = (tw["iterations"] + 1) * 9 + 11  # particle-turns per call
    flops = turns * float(f.sum())
    achieved = flops / (ms / 1e3) / 1e12
    out = {
        "metric": "optics computations/s (closed orbit, beta, alpha, phase, dispersion)",
        "value": 1e3 / ms,
        "unit": "twiss/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "optics of the DA-scan ring (20,000 thin elements, order-10 "
                               "errors), 4D uncoupled, delta0 = 0",
                   "n_elements": len(el), "newton_steps": tw["iterations"],
                   "particle_turns": turns, "qx": tw["qx"], "qy": tw["qy"], "wall_s": wall},
        "roofline": {"bound": "alu", "kernel": "xtm_record (generated recording kernel, one "
                                               "thread per particle, 9 or 11 particles: one "
                                               "wave, latency-bound)",
                     "achieved": achieved, "peak": FP64_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / FP64_VECTOR_PEAK_TFLOPS, "traffic": None,
                     "flops_per_call": flops},
    }
    if not args.no_cpu_baseline:
        import oracle
        t = time.perf_counter()
        oracle.twiss(el, ref, h=1e-9, hd=1e-8)
        dt = time.perf_counter() - t
        out["cpu_baseline"] = {"value": 1.0 / dt, "unit": "twiss/s", "cores": 1, "kind": "oracle",
                               "sample": f"one optics computation of the same ring in {dt:.2f} s"}
    print(json.dumps(out), flush=True)


def cfg3_separate(args):
    """The 64 lattice variants tracked one after another, each with its own
    lattice, particle set and default launches (the comparison for the
    batched launch): 1 warmup step, then the timed steps on the host clock
    around all variants."""
    import torch
    import paper_2310_00317_amd as P
    I = P.inputs
    els, (coords, counts), ref, _, tps_default, steps_default = workload("cfg3", args.particles)
    tps = args.turns_per_step or tps_default
    steps = args.steps if args.steps is not None else steps_default
    first = np.concatenate([[0], np.cumsum(counts)]).astype(np.int64)
    lats = [P.Lattice(e, ref) for e in els]

    def fresh():
        return [P.Particles(int(counts[v]), ref).init(coords[first[v]:first[v + 1]])
                for v in range(len(els))]

    for _ in range(args.warmup):
        sets = fresh()
        for v in range(len(els)):
            P.track(lats[v], sets[v], tps)
    torch.cuda.synchronize()
    sets = fresh()
    torch.cuda.synchronize()
    passes = 0
    t0 = time.perf_counter()
    for _ in range(steps):
        for v in range(len(els)):
            pv, _ = P.track(lats[v], sets[v], tps)
            passes += pv
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    f = element_flops(els[0])
    fpp = float(f.sum() / len(els[0]))
    achieved = passes * fpp / wall / 1e12
    print(json.dumps({
        "metric": "particle-element passes/s (FP64), lattice variants tracked one after another",
        "value": passes / wall, "unit": "passes/s", "n_gpus": 1, "steps": steps,
        "warmup": args.warmup, "ms_per_step": wall / steps * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"64 errored FODO variants, {int(counts.sum())} protons, each "
                               "variant its own lattice, set and launches", "turns": steps * tps,
                   "passes": int(passes), "wall_s": wall},
        "roofline": {"bound": "alu", "kernel": "xtm_line, one lattice per launch sequence",
                     "achieved": achieved, "peak": FP64_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / FP64_VECTOR_PEAK_TFLOPS, "traffic": None,
                     "flops_per_pass": fpp}}), flush=True)


def learned_da(args):
    """Dynamic-aperture scan of the cfg1 ring: plain tracking to the horizon
    versus learned early stop (network) and the tune-diffusion rule, on the
    same GPU with the same kernels.  Training data: random amplitudes tracked
    to the horizon with the recorder on (reported separately, not part of the
    scan wall time)."""
    import torch
    import paper_2310_00317_amd as P
    from paper_2310_00317_amd import inputs as I
    from paper_2310_00317_amd import learned as L
    el, ref = I.cfg1_lattice(), I.PROTON_450GEV
    tw, emit, rap = I.cfg1_twiss(), I.CFG2_EMIT, I.CFG1_APERTURE
    lat = P.Lattice(el, ref)
    log = lambda m: print(f"[cfg4] {m}", file=sys.stderr, flush=True)
    H = args.horizon
    t = time.perf_counter()
    tc, _, _ = I.random_amplitudes(args.train_particles, args.da_rmax, tw, seed=404)
    data = L.collect(lat, ref, tc, H, tw, emit, rap, first_id=10 ** 9,
                     windows=max(args.windows, args.stages))
    t_label = time.perf_counter() - t
    log(f"labels: {args.train_particles} particles x {H} turns in {t_label:.1f} s; "
        f"stable fraction {data.label.mean():.3f}")
    t = time.perf_counter()
    pred = L.train(data, max_false_rate=args.max_false_rate, epochs=args.epochs)
    t_train = time.perf_counter() - t
    rule = L.rule_threshold(data, max_false_rate=args.max_false_rate)
    log(f"trained in {t_train:.1f} s, tau {pred.tau:.3f} (held-out false rate "
        f"{pred.val_false_rate:.2e}, {pred.val_retired} retired); rule threshold {rule:.3f}")
    gc, gr, _ = I.polar_grid(args.da_radii, args.da_rays, args.da_rmax, tw, emit)
    # compile the kernel forms the scans will use once, outside the timed scans
    warm = P.Particles(4096, ref).init(gc[:4096])
    tt = args.tune_turns
    if tt > 0:
        P.autotune(warm, lattice=lat, probe_turns=1)
    else:
        P.track(lat, warm, 2)
    warm.close()
    plain = L.scan(lat, ref, gc, H, tune_turns=tt)
    log(f"plain scan {plain['wall_s']:.1f} s")
    learned = L.scan(lat, ref, gc, H, tw, emit, rap, predictor=pred, tune_turns=tt,
                     stages=args.stages, keep_decisions=True)
    log(f"learned scan {learned['wall_s']:.1f} s, retired {learned['retired']}")
    if args.no_rule_scan:
        ruled = None
    else:
        ruled = L.scan(lat, ref, gc, H, tw, emit, rap, rule_tau=rule, tune_turns=tt)
        log(f"rule scan {ruled['wall_s']:.1f} s, retired {ruled['retired']}")
    nr, nt = args.da_radii, args.da_rays
    e_l = L.da_error(learned["state"], plain["state"], gr, nr, nt)
    per_ray = L.da_error_per_ray(learned["state"], plain["state"], gr, nr, nt)
    sub = per_ray[::10]   # the 50-ray sub-grid (every 10th angle)
    worst = int(np.argmax(per_ray))
    da_p = P.dynamic_aperture(plain["state"], gr, nr, nt)
    da_l = P.dynamic_aperture(learned["state"], gr, nr, nt)
    # the particles whose retirement moved the worst ray's aperture: lost in
    # plain tracking, retired by the network, inside the learned aperture
    on_ray = np.arange(worst * nr, (worst + 1) * nr)
    culprits = [int(i) for i in on_ray
                if plain["state"][i] in (0, -1) and learned["state"][i] == 2
                and gr[i] < (da_l[worst] if np.isfinite(da_l[worst]) else np.inf)]
    dec = learned["decisions"][0]
    worst_ray = {"ray": worst, "error_sigma": float(per_ray[worst]),
                 "da_plain": float(da_p[worst]), "da_learned": float(da_l[worst]),
                 "falsely_retired": [{"particle": i, "radius_sigma": float(gr[i]),
                                      "lost_at_turn_plain": int(plain["at_turn"][i]),
                                      "logit": float(dec["score"][i]), "tau": float(dec["tau"]),
                                      "features": [float(v) for v in dec["features"][i]]}
                                     for i in culprits[:3]]}
    false_ret = (learned["state"] == 2) & np.isin(plain["state"], (0, -1))
    ray_stats = {"grid_500": {"mean": float(per_ray.mean()), "max": float(per_ray.max()),
                              "q50": float(np.quantile(per_ray, 0.5)),
                              "q90": float(np.quantile(per_ray, 0.9)),
                              "q99": float(np.quantile(per_ray, 0.99)),
                              "rays_above_0.1": int((per_ray > 0.1).sum()),
                              "rays_above_1": int((per_ray > 1.0).sum())},
                 "grid_50": {"mean": float(sub.mean()), "max": float(sub.max()),
                             "rays_above_0.1": int((sub > 0.1).sum())},
                 "falsely_retired_total": int(false_ret.sum()),
                 "worst_ray": worst_ray}
    e_r = L.da_error(ruled["state"], plain["state"], gr, nr, nt) if ruled else (None, None)
    da = P.dynamic_aperture(plain["state"], gr, nr, nt)
    keys = ("retired", "audited", "audit_lost", "audit_upper", "fallback", "wall_s")
    out = {
        "metric": "DA wall-clock speedup, learned early stop vs plain tracking",
        "value": plain["wall_s"] / learned["wall_s"],
        "unit": "x",
        "n_gpus": 1,
        "higher_is_better": True,
        "vs_baseline": None,
        "dtype": "f64 tracking; bf16/fp32 network",
        "data": "synthetic",
        "config": {"workload": f"cfg1 ring DA scan, {nr}x{nt} polar grid 0-{args.da_rmax} sigma, "
                               f"{H} turns; predictor trained on {args.train_particles} random "
                               "amplitudes", "horizon": H, "max_false_rate": args.max_false_rate,
                   "stages": args.stages, "windows": max(args.windows, args.stages)},
        "da_error_sigma": {"network_mean": e_l[0], "network_max": e_l[1],
                           "rule_mean": e_r[0], "rule_max": e_r[1]},
        "da_error_rays": ray_stats,
        "plain": {"wall_s": plain["wall_s"], "da_mean_sigma": float(np.mean(np.where(
            np.isfinite(da), da, args.da_rmax))), "da_min_sigma": float(np.min(da))},
        "network": {k: learned[k] for k in keys if k in learned},
        "rule": {k: ruled[k] for k in keys if k in ruled} if ruled else None,
        "rule_speedup": plain["wall_s"] / ruled["wall_s"] if ruled else None,
        "network_stages": learned.get("stages"),
        "training": {"label_s": t_label, "train_s": t_train, "tau": pred.tau,
                     "taus": [float(t) for t in pred.taus],
                     "val_false_rate": pred.val_false_rate,
                     "loss_first_last": [float(pred.losses[0]), float(pred.losses[-1])]},
    }
    print(json.dumps(out, default=lambda o: bool(o) if isinstance(o, np.bool_) else float(o)),
          flush=True)


def radiation_equilibrium(args):
    """The electron ring's radiation equilibrium at scale: an ensemble matched
    to the 6D normal form, tracked `--eq-turns` turns (five longitudinal
    damping times by default) with quantum excitation (Gaussian or photon by
    photon); the energy spread of the last tenth of the run, the energy loss
    per turn of a particle on the design orbit through the ring without its
    cavities, and the longitudinal damping time of the normal form, each
    beside its closed form: U0 = (2/3) r m gamma^4 sum h^2 L_r, sigma_delta^2 =
    C_q gamma^2 h / J_z (identical bends, C_q = 55 hbar_c / (32 sqrt 3 m c^2)),
    tau_z = 2 E0 / (J_z U0) turns with J_z = 2."""
    import torch
    import paper_2310_00317_amd as P
    from paper_2310_00317_amd import inputs as I
    ref = I.ELECTRON_45GEV6
    el = I.cfg5_lattice()
    lat = P.Lattice(el, ref)
    n = args.particles or 100_000
    nf = P.twiss6d(lat, radiation=1)
    c = P.matched_gaussian(nf, ref, I.CFG5_EMITTANCES, I.standard_normals(n))
    parts = P.Particles(n, ref).init(c)
    seed = 20231003
    turns = args.eq_turns
    chunk = 100
    samples = []
    t0 = time.perf_counter()
    for k in range(turns // chunk):
        P.track(lat, parts, chunk, radiation=args.radiation, seed=seed)
        if (k + 1) * chunk > 0.9 * turns:
            samples.append(float(parts.delta[:n].std().cpu()))
        if k % 10 == 9:
            print(f"[eq] {(k + 1) * chunk} turns, sigma_delta {float(parts.delta[:n].std().cpu()):.4e}",
                  file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    alive = int((parts.state[:n] == 1).sum().cpu())
    # energy loss per turn on the design orbit, cavities removed (mean model)
    no_rf = el[el["type"] != I.RF]
    lat0 = P.Lattice(no_rf, ref)
    one = P.Particles(1, ref).init(np.zeros((1, 6)))
    P.track(lat0, one, 1, radiation=1)
    e0 = math.sqrt(ref.p0c_eV ** 2 + ref.mass0_eV ** 2)
    b0 = ref.p0c_eV / e0
    g0 = e0 / ref.mass0_eV
    u0_meas = -float(one.ptau[0].cpu()) * ref.p0c_eV
    bends = el[(el["type"] == I.MULTIPOLE) & (el["length"] > 0)]
    h = np.abs(bends["knl"][:, 0]) / bends["length"]
    u0_cf = 2.0 / 3.0 * I.R_ELECTRON * I.ELECTRON_MASS_EV * g0 ** 4 * float(np.sum(h * h * bends["length"]))
    cq = 55.0 / (32.0 * math.sqrt(3.0)) * I.HBAR_C_EVM / I.ELECTRON_MASS_EV
    jz = 2.0
    sd_cf = math.sqrt(cq * g0 ** 2 * float(h[0]) / jz)
    tau_nf = 1.0 / nf.damping[2]
    tau_cf = 2.0 * e0 / (jz * u0_cf)
    out = {"metric": "radiation equilibrium of the electron ring against closed forms",
           "value": float(np.mean(samples)) / sd_cf, "unit": "sigma_delta / closed form",
           "n_gpus": 1, "higher_is_better": None, "vs_baseline": None, "dtype": "f64",
           "data": "synthetic",
           "config": {"workload": f"electron ring, 20,000 thin elements, {n} electrons at 45.6 GeV "
                                  f"matched to the 6D normal form, {turns} turns, radiation "
                                  f"{'photon by photon' if args.radiation == 3 else 'mean + Gaussian quantum'}"},
           "sigma_delta": {"tracked": float(np.mean(samples)), "closed_form": sd_cf},
           "u0_eV": {"tracked": u0_meas, "closed_form": u0_cf},
           "tau_z_turns": {"normal_form": tau_nf, "closed_form": tau_cf},
           "partition_numbers": [float(d / (u0_cf / (2 * e0))) for d in nf.damping[:]],
           "alive_at_end": alive, "wall_s": wall,
           "passes_per_s": n * len(el) * turns / wall}
    print(json.dumps(out), flush=True)


def mlp_bench(args):
    """The loss predictor's kernels alone: inference on 2^20 feature rows and
    training steps (gradient + Adam) on batches of 4,096, timed with events;
    BF16 MFMA work per sample 37,120 FLOP forward (2 (16 x 128 + 128 x 128 +
    128)), about three times that for a training sample."""
    import torch
    import paper_2310_00317_amd as P
    rng = np.random.default_rng(5)
    n = args.particles or (1 << 20)
    X = torch.tensor(rng.normal(size=(n, 16)).astype(np.float32), device="cuda")
    Y = torch.tensor((rng.random(4096) < 0.6).astype(np.float32), device="cuda")
    theta = P.mlp_init(3)
    norm = P.feature_stats(X)
    m, v = torch.zeros_like(theta), torch.zeros_like(theta)
    work = torch.empty(P.mlp_workspace(4096), dtype=torch.float32, device="cuda")
    Xb = X[:4096].contiguous()
    for _ in range(3):
        P.mlp_forward(theta, norm, X)
        g, _ = P.mlp_grad(theta, norm, Xb, Y, 1.5, work=work)
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    reps = 20
    a.record()
    for _ in range(reps):
        P.mlp_forward(theta, norm, X)
    b.record()
    torch.cuda.synchronize()
    fwd_ms = a.elapsed_time(b) / reps
    steps = 200
    a.record()
    for k in range(steps):
        g, _ = P.mlp_grad(theta, norm, Xb, Y, 1.5, work=work)
        P.mlp_adam(theta, m, v, g, k + 1, 1e-3)
    b.record()
    torch.cuda.synchronize()
    step_ms = a.elapsed_time(b) / steps
    fwd_flop = 2.0 * (16 * 128 + 128 * 128 + 128)
    peak = 2500.0
    out = {"metric": "loss-predictor inference rows/s (BF16 MFMA, FP32 accumulate)",
           "value": n / (fwd_ms / 1e3), "unit": "rows/s", "n_gpus": 1, "higher_is_better": True,
           "vs_baseline": None, "dtype": "bf16", "data": "synthetic",
           "config": {"workload": f"MLP 16-128-128-1, {n} rows forward; training batches of "
                                  "4096 (gradient + Adam)"},
           "forward_ms": fwd_ms, "train_step_ms": step_ms,
           "roofline": {"bound": "mfma", "achieved": n * fwd_flop / (fwd_ms / 1e3) / 1e12,
                        "peak": peak, "unit": "TFLOP/s",
                        "frac": n * fwd_flop / (fwd_ms / 1e3) / 1e12 / peak,
                        "traffic": None, "kernel": "k_mlp_forward"},
           "train_tflops": 3 * 4096 * fwd_flop / (step_ms / 1e3) / 1e12}
    print(json.dumps(out), flush=True)


def timed_steps(parts, run, steps: int, tps: int, log: bool = False) -> dict:
    """Time `steps` calls of run(parts, tps) between two events on the current
    stream (inputs resident in HBM); the library times each tracking launch
    with HIP events on its stream (time_kernels)."""
    import torch
    torch.cuda.synchronize()
    out = {"passes": 0, "kernel_ms": 0.0, "launches": 0, "variant": 0, "alive": 0}
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    t_wall = time.perf_counter()
    start.record()
    for s in range(steps):
        st = run(parts, tps, time_kernels=True)
        out["passes"] += st.passes
        out["kernel_ms"] += st.kernel_ms
        out["launches"] += st.launches
        out["variant"] = st.variant
        out["alive"] = st.alive
        if log:
            print(f"[bench] step {s + 1}/{steps}: alive {st.alive}", file=sys.stderr, flush=True)
    stop.record()
    torch.cuda.synchronize()
    out["wall"] = time.perf_counter() - t_wall
    out["ms"] = start.elapsed_time(stop)
    out["value"] = out["passes"] / (out["ms"] / 1e3)
    return out


def alu_roofline(m: dict, flops_per_pass: float, traffic, traffic_src) -> dict:
    kms = m["kernel_ms"]
    achieved = m["passes"] * flops_per_pass / (kms / 1e3) / 1e12 if kms > 0 else 0.0
    return {"bound": "alu", "kernel": KERNEL_NAMES.get(m["variant"], "?"),
            "achieved": achieved, "peak": FP64_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
            "frac": achieved / FP64_VECTOR_PEAK_TFLOPS, "traffic": traffic,
            "flops_per_pass": flops_per_pass, "avg_launch_ms": kms / max(m["launches"], 1),
            "launches": m["launches"], "traffic_unit": "bytes per launch",
            "traffic_profile": traffic_src}


def saturated_fodo_leg(P, turns: int, n: int) -> dict:
    """The FODO ring at 2^20 particles (the saturated first configuration):
    one warmup of 20 turns on its own set, then `turns` timed turns of a fresh
    set, with the roofline of its tracking kernel."""
    import torch
    from paper_2310_00317_amd import inputs as I
    el = I.cfg1_lattice()
    ref = I.PROTON_450GEV
    lat = P.Lattice(el, ref)
    coords = torch.from_numpy(np.ascontiguousarray(I.cfg1_particles(n))).to("cuda")
    run = lambda parts, t, **kw: P.track(lat, parts, t, full_stats=True, **kw)
    w = P.Particles(n, ref).init(coords)
    run(w, 20)
    w.close()
    parts = P.Particles(n, ref).init(coords)
    m = timed_steps(parts, run, 1, turns)
    fpp = float(element_flops(el).sum() / len(el))
    key = ("cfg1sat", n, turns, m["variant"], kernel_source_hash())
    traffic, src = MEASURED_TRAFFIC.get(key, (None, None))
    return {"workload": f"thin FODO ring, 801 elements, {n} Gaussian protons at 450 GeV, "
                        f"{turns} turns", "value": m["value"], "unit": "passes/s",
            "ms": m["ms"], "passes": int(m["passes"]), "alive_at_end": int(m["alive"]),
            "roofline": alu_roofline(m, fpp, traffic, src)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--turns-per-step", type=int, default=None)
    ap.add_argument("--workload", default="cfg2",
                    choices=["cfg2", "cfg1", "cfg1sat", "cfg3", "cfg4", "cfg5", "mlp", "refine",
                             "twiss", "thick"])
    ap.add_argument("--refine-vertices", type=int, default=64,
                    help="refine: polygon vertices per aperture")
    ap.add_argument("--refine-ds", type=float, default=0.01, help="refine: sub-step [m]")
    ap.add_argument("--refine-bisect", type=int, default=30, help="refine: bisection steps")
    ap.add_argument("--da-rays", type=int, default=500, help="cfg4: rays of the evaluation grid")
    ap.add_argument("--da-radii", type=int, default=2000, help="cfg4: radii per ray")
    ap.add_argument("--da-rmax", type=float, default=30.0, help="cfg4: grid edge [sigma]")
    ap.add_argument("--train-particles", type=int, default=1200000)
    ap.add_argument("--horizon", type=int, default=100000, help="cfg4: turns")
    ap.add_argument("--epochs", type=int, default=60)
    ap.add_argument("--tune-turns", type=int, default=0,
                    help="cfg4: autotuner probe turns before each long tracking stretch (0 = off)")
    ap.add_argument("--max-false-rate", type=float, default=1.5e-3,
                    help="cfg4: held-out false-retire budget that fixes the threshold")
    ap.add_argument("--stages", type=int, default=1,
                    help="cfg4: retirement decisions at the end of this many 1024-turn windows")
    ap.add_argument("--windows", type=int, default=1,
                    help="cfg4: recorded 1024-turn windows per training particle (pooled)")
    ap.add_argument("--no-rule-scan", action="store_true", help="cfg4: skip the rule-only scan")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="BYTES",
                    help="only run a plain device-to-device copy of BYTES (3 times), the "
                         "reference for scaling HBM byte counters")
    ap.add_argument("--particles", type=int, default=None)
    ap.add_argument("--block", type=int, default=0)
    ap.add_argument("--chunk", type=int, default=0)
    ap.add_argument("--variant", type=int, default=0)
    ap.add_argument("--graph", action="store_true",
                    help="replay each step's chunk sequence as a captured hipGraph")
    ap.add_argument("--per-element", action="store_true",
                    help="time the measurement baseline instead: one kernel launch per element "
                         "and turn, particle state through HBM at every element")
    ap.add_argument("--autotune", action="store_true",
                    help="run the launch-plan autotuner before the warmup and track with its "
                         "pick (reported in config)")
    ap.add_argument("--tune-probe", type=int, default=10,
                    help="--autotune: turns of each probe")
    ap.add_argument("--tune-warm", type=int, default=200,
                    help="--autotune: turns the probe copy is tracked before the probes "
                         "(past the scan's early losses)")
    ap.add_argument("--separate", action="store_true",
                    help="cfg3: track the variants one after another, each with its own "
                         "lattice and particle set, instead of one batched launch per chunk")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--equilibrium", action="store_true",
                    help="cfg5: track a matched ensemble to equilibrium and compare the energy "
                         "spread, energy loss and damping time with their closed forms")
    ap.add_argument("--eq-turns", type=int, default=5000)
    ap.add_argument("--radiation", type=int, default=2, choices=[1, 2, 3],
                    help="cfg5: 1 mean loss, 2 mean + Gaussian quantum excitation, "
                         "3 photon by photon")
    ap.add_argument("--sat-turns", type=int, default=1000,
                    help="default workload: turns of the 2^20-particle FODO leg (0 = skip)")
    ap.add_argument("--cpu-sample-every", type=int, default=100)
    ap.add_argument("--cpu-turns", type=int, default=None,
                    help="turns of the CPU oracle sample (default 1500; 150 with radiation, "
                         "50 photon by photon)")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: this tracker shards particles with no "
              "exchange during tracking, so multi-GPU runs are not part of this build",
              file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2310_00317_amd as P

    if args.copy_calibration:
        n = args.copy_calibration // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": n * 4, "copy_bytes_written": n * 4, "copies": 3}))
        return
    if args.workload == "cfg4":
        return learned_da(args)
    if args.workload == "mlp":
        return mlp_bench(args)
    if args.workload == "cfg5" and args.equilibrium:
        return radiation_equilibrium(args)
    if args.workload == "refine":
        return refine_bench(args)
    if args.workload == "twiss":
        return twiss_bench(args)
    if args.workload == "cfg3" and args.separate:
        return cfg3_separate(args)
    el, coords, ref, desc, tps_default, steps_default = workload(args.workload, args.particles, args.radiation)
    tps = args.turns_per_step or tps_default
    steps = args.steps if args.steps is not None else steps_default
    batched = args.workload == "cfg3"
    if batched:
        coords, counts = coords
        first = np.concatenate([[0], np.cumsum(counts)]).astype(np.int64)
        el_all = np.concatenate(el)
    else:
        el_all = el
    n = len(coords)
    n_el = len(el[0]) if batched else len(el)
    print(f"[bench] workload {args.workload}: {n} particles, {n_el} elements, "
          f"{steps} x {tps} turns (+{args.warmup} warmup steps)", file=sys.stderr, flush=True)

    torch.cuda.set_device(0)
    if batched:
        lats = [P.Lattice(e, ref) for e in el]
        batch = P.Batch(lats)
    else:
        lat = P.Lattice(el, ref)
    n_el_tracked = 0 if batched else lat.n_elements
    coords_dev = torch.from_numpy(np.ascontiguousarray(coords)).to("cuda")
    extra = dict(radiation=args.radiation, seed=20231002) if args.workload == "cfg5" else {}

    if args.per_element and (batched or extra):
        raise SystemExit("--per-element: single-lattice workloads without radiation only")

    def run(parts, turns, **kw):
        if args.per_element:
            return P.track_per_element(lat, parts, turns)
        if batched:
            return P.track_batched(batch, parts, first, turns, block=args.block,
                                   turns_per_chunk=args.chunk, variant=args.variant,
                                   graph=args.graph, full_stats=True, **kw)
        return P.track(lat, parts, turns, block=args.block, turns_per_chunk=args.chunk,
                       variant=args.variant, graph=args.graph, full_stats=True, **extra, **kw)

    plan = None
    if args.autotune:
        # the autotuner times the candidate plans (form, chunk length,
        # compaction period) on a copy of the set, advanced past its first
        # turns, and keeps the fastest as the lattice's (or batch's) plan,
        # which tracking then uses when no variant is forced
        probe = P.Particles(n, ref).init(coords_dev)
        if batched:
            plan = P.autotune(probe, batch=batch, first_slot=first, probe_turns=args.tune_probe,
                              warm_turns=args.tune_warm)
        else:
            plan = P.autotune(probe, lattice=lat, probe_turns=args.tune_probe,
                              warm_turns=args.tune_warm)
        torch.cuda.synchronize()
        del probe
    if args.warmup > 0:
        w = P.Particles(n, ref).init(coords_dev)
        for _ in range(args.warmup):
            run(w, tps)
        w.close()
        del w

    parts = P.Particles(n, ref).init(coords_dev)
    m = timed_steps(parts, run, steps, tps, log=True)
    total_passes, kernel_ms, launches = m["passes"], m["kernel_ms"], m["launches"]
    variant_ran, alive, ms, wall, value = m["variant"], m["alive"], m["ms"], m["wall"], m["value"]

    if args.per_element:
        # the baseline's algorithmic bytes: the fields each element's map reads
        # and writes, averaged over the line
        bytes_per_pass = float(element_bytes(el).mean())
        gbs = total_passes * bytes_per_pass / (kernel_ms / 1e3) / 1e9 if kernel_ms > 0 else 0.0
        out = {
            "metric": "particle-element passes/s (FP64); DA wall-clock learned vs plain at 0.1 sigma",
            "value": value, "unit": "passes/s", "n_gpus": 1, "steps": steps,
            "warmup": args.warmup, "ms_per_step": ms / steps, "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
            "config": {"workload": desc + "; one kernel launch per element (baseline)",
                       "n_particles": n, "n_elements": n_el, "turns": steps * tps,
                       "alive_at_end": int(alive), "passes": int(total_passes), "wall_s": wall},
            "roofline": {"bound": "hbm", "kernel": "k_elem (one launch per element)",
                         "achieved": gbs, "peak": 8000.0, "unit": "GB/s", "frac": gbs / 8000.0,
                         "traffic": None, "bytes_per_pass": bytes_per_pass,
                         "avg_launch_ms": kernel_ms / max(launches, 1), "launches": launches},
        }
        print(json.dumps(out), flush=True)
        return

    flops = element_flops(el_all)
    # per element of the tracked line (thick elements count their slices)
    n_tracked = n_el_tracked if n_el_tracked else len(el_all)
    flops_per_pass = float(flops.sum() / n_tracked)
    key = (args.workload, n, tps, variant_ran, kernel_source_hash())
    traffic, traffic_src = MEASURED_TRAFFIC.get(key, (None, None))
    if args.chunk or args.autotune or args.block:
        # the counters were taken with the default launch shape
        traffic, traffic_src = None, None

    out = {
        "metric": "particle-element passes/s (FP64); DA wall-clock learned vs plain at 0.1 sigma",
        "value": value,
        "unit": "passes/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": args.warmup,
        "ms_per_step": ms / steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": desc, "n_particles": n, "n_elements": n_el,
                   **({"autotune_pick": {"variant": plan.variant, "block": plan.block,
                                         "turns_per_chunk": plan.turns_per_chunk,
                                         "compact_every": plan.compact_every,
                                         "probe_passes_per_s": plan.passes_per_s}}
                      if plan is not None else {}),
                   "turns": steps * tps, "alive_at_end": int(alive),
                   "passes": int(total_passes), "wall_s": wall},
        "roofline": alu_roofline(m, flops_per_pass, traffic, traffic_src),
    }
    if args.workload == "cfg2" and args.sat_turns > 0 and not args.particles:
        print("[bench] saturated FODO leg", file=sys.stderr, flush=True)
        out["cfg1_sat"] = saturated_fodo_leg(P, args.sat_turns, 1 << 20)
    if not args.no_cpu_baseline:
        print("[bench] timing the CPU oracle on a sample", file=sys.stderr, flush=True)
        if args.cpu_turns is None:
            args.cpu_turns = (50 if args.radiation == 3 else 150) if extra else 1500
        if batched:
            out["cpu_baseline"] = cpu_baseline(el[0], coords[: counts[0]], ref,
                                               args.cpu_sample_every, args.cpu_turns)
        else:
            out["cpu_baseline"] = cpu_baseline(el, coords, ref, args.cpu_sample_every,
                                               args.cpu_turns, **extra)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
