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
resumed from the state it was retired in and tracked to the horizon
(full-tracking fallback).

Stages (an extension of the single decision at turn 1024): with K stages the
same decision is repeated at the end of each consecutive 1024-turn window
(turns 1024, 2048, ..., K*1024) for the particles still tracked, from the
features of that window.  The network is trained on the windows of the
training set pooled (a window's features and the particle's survival to the
horizon), and each stage has its own threshold from the held-out rows of its
window.  Audited particles stay audited at every stage (the audit draw is a
function of the particle id), so the audit still judges every retirement.
"""
from __future__ import annotations

import time
from dataclasses import dataclass

import numpy as np

import paper_2310_00317_amd as P

RECORD_TURNS = P.RECORD_TURNS


@dataclass
class Predictor:
    theta: object          # torch float32 [MLP_PARAMS]
    norm: object           # torch float32 [32]
    tau: float             # retire threshold on the logit (first window)
    val_false_rate: float  # held-out false-retire fraction at tau
    val_retired: int       # held-out rows at or above tau
    losses: np.ndarray     # per-epoch mean training loss
    taus: tuple = ()       # per-window thresholds (window k: taus[k]); () = (tau,)

    def tau_at(self, k: int) -> float:
        t = self.taus or (self.tau,)
        return float(t[min(k, len(t) - 1)])


@dataclass
class Collected:
    feat: object           # torch float32 [n, 16] (first window)
    label: np.ndarray      # int32 (1 = alive after the horizon)
    alive_at_record: np.ndarray  # bool: alive after the first window
    state: np.ndarray
    at_turn: np.ndarray
    feats: tuple = ()      # per window k: torch float32 [n, 16]
    alive: tuple = ()      # per window k: bool, alive after window k


def collect(lat, ref, coords, horizon: int, twiss4, emit: float, r_aperture: float,
            first_id: int = 0, windows: int = 1) -> Collected:
    """Track the set to the horizon with the recorder on; features from each
    of the first `windows` 1024-turn windows and survival labels."""
    import torch
    n = len(coords)
    parts = P.Particles(n, ref).init(coords, first_id=first_id)
    rec = torch.zeros((windows * RECORD_TURNS, 4, n), dtype=torch.float32, device="cuda")
    feats, alive = [], []
    for k in range(windows):
        P.track(lat, parts, RECORD_TURNS, record=rec)
        st_k, _, _ = parts.losses()
        alive.append(st_k == 1)
        feats.append(P.features(rec[k * RECORD_TURNS:(k + 1) * RECORD_TURNS], twiss4, emit,
                                r_aperture))
    del rec
    P.track(lat, parts, horizon - windows * RECORD_TURNS)
    st, at, _ = parts.losses()
    return Collected(feats[0], (st == 1).astype(np.int32), alive[0], st, at, tuple(feats),
                     tuple(alive))


def train(data: Collected, max_false_rate: float = 1e-3, val_frac: float = 0.1,
          epochs: int = 30, batch: int = 4096, lr: float = 1e-3, seed: int = 1) -> Predictor:
    """Fit the network on the rows alive after each recorded window (pooled
    over the windows); pick each window's threshold on a held-out split of
    the particles."""
    import torch
    feats = data.feats or (data.feat,)
    alive = data.alive or (data.alive_at_record,)
    n = len(data.label)
    rng = np.random.default_rng(seed)
    perm = rng.permutation(n)
    is_val = np.zeros(n, dtype=bool)
    # the held-out particles: val_frac of those alive after the first window
    first = perm[alive[0][perm]]
    is_val[first[: max(1, int(len(first) * val_frac))]] = True
    dev = data.feat.device
    Xs, Ys, val_sets = [], [], []
    for f, a in zip(feats, alive):
        tr = np.nonzero(a & ~is_val)[0]
        tr = tr[rng.permutation(len(tr))]
        Xs.append(f[torch.as_tensor(tr, device=dev)])
        Ys.append(data.label[tr])
        val_sets.append((f, np.nonzero(a & is_val)[0]))
    X = torch.cat(Xs).contiguous()
    y = np.concatenate(Ys)
    Y = torch.as_tensor(y.astype(np.float32), device=dev)
    norm = P.feature_stats(X)
    theta = P.mlp_init(seed)
    m = torch.zeros_like(theta)
    v = torch.zeros_like(theta)
    n_pos = int(y.sum())
    pos_weight = (len(y) - n_pos) / max(n_pos, 1)
    _, losses = P.mlp_train(theta, m, v, norm, X, Y, pos_weight, epochs, batch, lr, seed)
    taus, first_rate, first_sel = [], 0.0, 0
    for k, (f, val) in enumerate(val_sets):
        Xv = f[torch.as_tensor(val, device=dev)].contiguous()
        Yv = torch.as_tensor(data.label[val], device=dev)
        z = P.mlp_forward(theta, norm, Xv)
        tau, rate, sel = P.select_threshold(z, Yv, max_false_rate)
        taus.append(tau)
        if k == 0:
            first_rate, first_sel = rate, sel
    return Predictor(theta, norm, taus[0], first_rate, first_sel, losses, tuple(taus))


def rule_threshold(data: Collected, max_false_rate: float = 1e-3, val_frac: float = 0.1,
                   seed: int = 1) -> float:
    """The method without the network: retire iff the larger of the two
    tune-diffusion features (f8, f9) is below a threshold, chosen on the same
    held-out split with the same budget.  Returned as a threshold on the
    library's rule score (xtm_rule_score, -max(f8, f9))."""
    import torch
    rows = np.nonzero(data.alive_at_record)[0]
    rng = np.random.default_rng(seed)
    rows = rows[rng.permutation(len(rows))]
    val = rows[: max(1, int(len(rows) * val_frac))]
    f = data.feat[torch.as_tensor(val, device=data.feat.device)].contiguous()
    tau, _, _ = P.select_threshold(P.rule_score(f),
                                   torch.as_tensor(data.label[val], device=f.device),
                                   max_false_rate)
    return tau


def rule_scores(feat):
    return P.rule_score(feat.contiguous())


def scan(lat, ref, coords, horizon: int, twiss4=None, emit=None, r_aperture=None,
         predictor: Predictor | None = None, rule_tau: float | None = None,
         audit_fraction: float = 0.05, audit_seed: int = 0x5EED, fallback_rate: float = 5e-3,
         first_id: int = 0, tune_turns: int = 0, variant: int = 0, stages: int = 1,
         keep_decisions: bool = False) -> dict:
    """One DA scan.  Plain when neither a predictor nor a rule threshold is
    given; otherwise learned (network) or rule-based early stop, decided at
    the end of each of the first `stages` 1024-turn windows.  Returns the
    final states, the GPU wall time and the retire/audit counts.

    tune_turns > 0: before each long tracking stretch (the whole horizon of a
    plain scan; the turns after the last stage otherwise) the launch-plan
    autotuner times every kernel form on a scratch copy of the particles
    still tracked, for that many turns, and the stretch runs with the
    fastest (inside the timed wall time; results are the same bit for bit).
    The plan stays set on the lattice afterwards.  variant != 0 runs that
    tracking kernel throughout instead (see xtm_track_opts.variant).
    keep_decisions: also return each decision's scores and features (host
    arrays, indexed by particle) for analysis."""
    import torch
    n = len(coords)
    coords_dev = torch.as_tensor(np.ascontiguousarray(coords), device="cuda")
    parts = P.Particles(n, ref).init(coords_dev, first_id=first_id)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    out = {"retired": 0, "audited": 0, "audit_lost": 0, "fallback": False, "stages": []}
    if predictor is None and rule_tau is None:
        if tune_turns > 0:
            P.autotune(parts, lattice=lat, probe_turns=tune_turns)
        P.track(lat, parts, horizon, variant=variant)
    else:
        stages = max(1, min(int(stages), horizon // RECORD_TURNS))
        rec = torch.zeros((stages * RECORD_TURNS, 4, n), dtype=torch.float32, device="cuda")
        audit_flags = torch.zeros(n, dtype=torch.int32, device="cuda")
        for k in range(stages):
            P.track(lat, parts, RECORD_TURNS, record=rec, variant=variant)
            feat = P.features(rec[k * RECORD_TURNS:(k + 1) * RECORD_TURNS], twiss4, emit,
                              r_aperture)
            if predictor is not None:
                score, tau = P.mlp_forward(predictor.theta, predictor.norm, feat), \
                    predictor.tau_at(k)
            else:
                score, tau = P.rule_score(feat), rule_tau
            retired, audited = P.retire(parts, score, tau, audit_seed, audit_fraction,
                                        audit_flags=audit_flags)
            if keep_decisions:
                out.setdefault("decisions", []).append(
                    {"score": score.cpu().numpy(), "features": feat.cpu().numpy(), "tau": tau})
            out["retired"] += retired
            out["stages"].append({"turn": (k + 1) * RECORD_TURNS, "tau": float(tau),
                                  "retired": retired, "audited": audited,
                                  "tracked_after": int(np.count_nonzero(parts.losses()[0] == 1))})
        del rec
        if tune_turns > 0:
            P.autotune(parts, lattice=lat, probe_turns=tune_turns)
        P.track(lat, parts, horizon - stages * RECORD_TURNS, variant=variant)
        v = P.audit_verdict(parts, audit_flags, fallback_rate)
        out.update(audited=v["audited"], audit_lost=v["lost"], audit_upper=v["upper"])
        if v["fallback"]:
            # full-tracking fallback: every retired particle resumes from the
            # turn it was retired at (inside the library)
            out["fallback"] = True
            out["resumed_passes"], _ = P.resume_retired(lat, parts, variant=variant)
    torch.cuda.synchronize()
    out["wall_s"] = time.perf_counter() - t0
    st, at, ae = parts.losses()
    out["state"], out["at_turn"], out["at_element"] = st, at, ae
    return out


def da_error_per_ray(state_a, state_b, radius, n_r: int, n_theta: int) -> np.ndarray:
    """|DA_a - DA_b| in sigma for every ray (rays with no loss on either side
    censored at the scan edge)."""
    da_a = P.dynamic_aperture(state_a, radius, n_r, n_theta)
    da_b = P.dynamic_aperture(state_b, radius, n_r, n_theta)
    edge = float(np.max(radius))
    a = np.where(np.isfinite(da_a), da_a, edge)
    b = np.where(np.isfinite(da_b), da_b, edge)
    return np.abs(a - b)


def da_error(state_a, state_b, radius, n_r: int, n_theta: int) -> tuple[float, float]:
    """Mean and max over rays of |DA_a - DA_b| in sigma."""
    d = da_error_per_ray(state_a, state_b, radius, n_r, n_theta)
    return float(d.mean()), float(d.max())
