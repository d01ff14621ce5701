"""Learned early stop for dynamic-aperture scans, driven through the C ABI.

Every compute step is a library call (tracking with the early-turn recorder,
features, network training and inference, threshold selection, retirement,
dynamic aperture); this module only sequences them and moves small host
arrays (masks, index splits) between the calls.

Labels: a particle is positive (stable) if it is still alive after the
horizon.  The predictor is applied at turn 1024 to the particles still alive;
those with logit >= tau are retired (state 2) unless they fall in the
Philox-drawn audit set, which is tracked to the horizon like the rest and
measures the false-retire rate of the run itself.  If the audit's upper 95 %
bound on that rate exceeds ``fallback_rate``, every retired particle is
resumed from its turn-1024 state and tracked to the horizon (full-tracking
fallback).
"""
from __future__ import annotations

import math
import time
from dataclasses import dataclass

import numpy as np

import paper_2310_00317_amd as P

RECORD_TURNS = P.RECORD_TURNS


@dataclass
class Predictor:
    theta: object          # torch float32 [MLP_PARAMS]
    norm: object           # torch float32 [32]
    tau: float             # retire threshold on the logit
    val_false_rate: float  # held-out false-retire fraction at tau
    val_retired: int       # held-out rows at or above tau
    losses: np.ndarray     # per-epoch mean training loss


@dataclass
class Collected:
    feat: object           # torch float32 [n, 16]
    label: np.ndarray      # int32 (1 = alive after the horizon)
    alive_at_record: np.ndarray  # bool: alive after the record turns
    state: np.ndarray
    at_turn: np.ndarray


def collect(lat, ref, coords, horizon: int, twiss4, emit: float, r_aperture: float,
            first_id: int = 0) -> Collected:
    """Track the set to the horizon with the recorder on; features from the
    first 1024 turns and survival labels."""
    import torch
    n = len(coords)
    parts = P.Particles(n, ref).init(coords, first_id=first_id)
    rec = torch.zeros((RECORD_TURNS, 4, n), dtype=torch.float32, device="cuda")
    P.track(lat, parts, RECORD_TURNS, record=rec)
    st1, _, _ = parts.losses()
    feat = P.features(rec, twiss4, emit, r_aperture)
    del rec
    P.track(lat, parts, horizon - RECORD_TURNS)
    st, at, _ = parts.losses()
    return Collected(feat, (st == 1).astype(np.int32), st1 == 1, st, at)


def train(data: Collected, max_false_rate: float = 1e-3, val_frac: float = 0.1,
          epochs: int = 30, batch: int = 4096, lr: float = 1e-3, seed: int = 1) -> Predictor:
    """Fit the network on the rows alive after the record turns; pick tau on
    a held-out split."""
    import torch
    rows = np.nonzero(data.alive_at_record)[0]
    rng = np.random.default_rng(seed)
    rows = rows[rng.permutation(len(rows))]
    n_val = max(1, int(len(rows) * val_frac))
    val, tr = rows[:n_val], rows[n_val:]
    dev = data.feat.device
    X = data.feat[torch.as_tensor(tr, device=dev)].contiguous()
    Y = torch.as_tensor(data.label[tr].astype(np.float32), device=dev)
    Xv = data.feat[torch.as_tensor(val, device=dev)].contiguous()
    Yv = torch.as_tensor(data.label[val], device=dev)
    norm = P.feature_stats(X)
    theta = P.mlp_init(seed)
    m = torch.zeros_like(theta)
    v = torch.zeros_like(theta)
    n_pos = int(data.label[tr].sum())
    pos_weight = (len(tr) - n_pos) / max(n_pos, 1)
    _, losses = P.mlp_train(theta, m, v, norm, X, Y, pos_weight, epochs, batch, lr, seed)
    z = P.mlp_forward(theta, norm, Xv)
    tau, rate, sel = P.select_threshold(z, Yv, max_false_rate)
    return Predictor(theta, norm, tau, rate, sel, losses)


def rule_threshold(data: Collected, max_false_rate: float = 1e-3, val_frac: float = 0.1,
                   seed: int = 1) -> float:
    """The method without the network: retire iff the larger of the two
    tune-diffusion features (f8, f9) is below a threshold, chosen on the same
    held-out split with the same budget.  Returned as a threshold on the
    score -max(f8, f9)."""
    import torch
    rows = np.nonzero(data.alive_at_record)[0]
    rng = np.random.default_rng(seed)
    rows = rows[rng.permutation(len(rows))]
    val = rows[: max(1, int(len(rows) * val_frac))]
    f = data.feat[torch.as_tensor(val, device=data.feat.device)]
    score = (-torch.maximum(f[:, 8], f[:, 9])).contiguous()
    tau, _, _ = P.select_threshold(score, torch.as_tensor(data.label[val], device=f.device),
                                   max_false_rate)
    return tau


def rule_scores(feat):
    import torch
    return (-torch.maximum(feat[:, 8], feat[:, 9])).contiguous()


def wilson_upper(k: int, n: int, z: float = 1.6449) -> float:
    """One-sided 95 % Wilson upper bound of a binomial proportion."""
    if n == 0:
        return 1.0
    p = k / n
    d = 1 + z * z / n
    c = p + z * z / (2 * n)
    h = z * math.sqrt(p * (1 - p) / n + z * z / (4 * n * n))
    return (c + h) / d


def scan(lat, ref, coords, horizon: int, twiss4=None, emit=None, r_aperture=None,
         predictor: Predictor | None = None, rule_tau: float | None = None,
         audit_fraction: float = 0.05, audit_seed: int = 0x5EED, fallback_rate: float = 5e-3,
         first_id: int = 0, tune_turns: int = 0, variant: int = 0) -> dict:
    """One DA scan.  Plain when neither a predictor nor a rule threshold is
    given; otherwise learned (network) or rule-based early stop.  Returns the
    final states, the GPU wall time and the retire/audit counts.

    tune_turns > 0: before each long tracking stretch (the whole horizon of a
    plain scan; the turns after retirement otherwise) the launch-plan
    autotuner times every kernel form on a scratch copy of the particles
    still tracked, for that many turns, and the stretch runs with the
    fastest (inside the timed wall time; results are the same bit for bit).
    The plan stays set on the lattice afterwards.  variant != 0 runs that
    tracking kernel throughout instead (see xtm_track_opts.variant)."""
    import torch
    n = len(coords)
    coords_dev = torch.as_tensor(np.ascontiguousarray(coords), device="cuda")
    parts = P.Particles(n, ref).init(coords_dev, first_id=first_id)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    out = {"retired": 0, "audited": 0, "audit_lost": 0, "fallback": False}
    if predictor is None and rule_tau is None:
        if tune_turns > 0:
            P.autotune(parts, lattice=lat, probe_turns=tune_turns)
        P.track(lat, parts, horizon, variant=variant)
    else:
        rec = torch.zeros((RECORD_TURNS, 4, n), dtype=torch.float32, device="cuda")
        P.track(lat, parts, RECORD_TURNS, record=rec, variant=variant)
        feat = P.features(rec, twiss4, emit, r_aperture)
        del rec
        if predictor is not None:
            score, tau = P.mlp_forward(predictor.theta, predictor.norm, feat), predictor.tau
        else:
            score, tau = rule_scores(feat), rule_tau
        st_pre, _, _ = parts.losses()
        retired, audited = P.retire(parts, score, tau, audit_seed, audit_fraction)
        st_post, _, _ = parts.losses()
        snap = parts.to_numpy() if retired else None
        sc = score.cpu().numpy()
        audit_mask = (st_pre == 1) & (sc >= tau) & (st_post == 1)
        if tune_turns > 0:
            P.autotune(parts, lattice=lat, probe_turns=tune_turns)
        P.track(lat, parts, horizon - RECORD_TURNS, variant=variant)
        st_end, _, _ = parts.losses()
        lost_audit = int(((st_end != 1) & audit_mask).sum())
        out.update(retired=retired, audited=audited, audit_lost=lost_audit,
                   audit_upper=wilson_upper(lost_audit, int(audit_mask.sum())))
        if retired and out["audit_upper"] > fallback_rate:
            # full-tracking fallback: resume the retired particles from turn 1024
            ret = np.nonzero(st_post == 2)[0]
            c6 = np.stack([snap[f][ret] for f in ("x", "px", "y", "py", "zeta", "delta")], 1)
            res = P.Particles(len(ret), ref).init(c6)
            res.reset(RECORD_TURNS)
            P.track(lat, res, horizon - RECORD_TURNS)
            rs, ra, re = res.losses()
            out["fallback"] = True
            out["resumed"] = (ret, rs, ra, re)
    torch.cuda.synchronize()
    out["wall_s"] = time.perf_counter() - t0
    st, at, ae = parts.losses()
    if out.get("resumed") is not None:
        ret, rs, ra, re = out["resumed"]
        st, at, ae = st.copy(), at.copy(), ae.copy()
        st[ret], at[ret], ae[ret] = rs, ra, re
    out["state"], out["at_turn"], out["at_element"] = st, at, ae
    return out


def da_error(state_a, state_b, radius, n_r: int, n_theta: int) -> tuple[float, float]:
    """Mean and max over rays of |DA_a - DA_b| in sigma (rays with no loss on
    either side are censored at the scan edge)."""
    da_a = P.dynamic_aperture(state_a, radius, n_r, n_theta)
    da_b = P.dynamic_aperture(state_b, radius, n_r, n_theta)
    edge = float(np.max(radius))
    a = np.where(np.isfinite(da_a), da_a, edge)
    b = np.where(np.isfinite(da_b), da_b, edge)
    d = np.abs(a - b)
    return float(d.mean()), float(d.max())
