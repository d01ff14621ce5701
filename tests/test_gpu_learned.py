"""GPU parity of the learned early-stop kernels against the oracle: the
early-turn recorder, the 16 features, the 16-128-128-1 network (forward,
gradient, Adam step, initialisation) and the retire policy."""
import math

import numpy as np
import pytest

from paper_2310_00317_amd import inputs as I

pytestmark = pytest.mark.gpu
REF = I.PROTON_450GEV
EMIT = 1e-8


@pytest.fixture(scope="module")
def P():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2310_00317_amd as P
    P.lib()
    return P


def _twiss():
    k = 1 / I.CFG1_F
    return I.cell_twiss_at_qf_entry(k, -k, I.CFG1_HALF)


# ------------------------------------------------------------------ recorder
@pytest.mark.parametrize("variant,chunk", [(0, 100), (4, 0), (0, 0), (5, 50), (6, 30), (7, 0),
                                           (8, 100), (9, 0), (10, 64), (11, 0), (12, 40),
                                           (13, 0), (13, 50), (14, 0), (14, 30)])
def test_recorder_matches_oracle(P, oracle_mod, variant, chunk):
    """cfg1 without RF (bitwise tracking) on a polar grid reaching 32 sigma:
    survivors and particles lost at turns 0..95.  Entries up to the loss turn
    equal the FP32-rounded oracle record bit for bit; later ones stay
    untouched."""
    import torch
    from oracle import features as F
    el = I.cfg1_lattice(rf_on=False)
    c, r, th = I.polar_grid(16, 4, 32.0, _twiss(), EMIT, delta=2.7e-4)
    orec, op = F.record(el, REF, c, fp32=True)
    n = len(c)
    lat = P.Lattice(el, REF)
    parts = P.Particles(n, REF).init(c)
    rec = torch.full((F.WINDOW * 2, 4, n), float("nan"), dtype=torch.float32, device="cuda")
    P.track(lat, parts, 1024, turns_per_chunk=chunk, variant=variant, record=rec)
    g = rec.cpu().numpy().astype(np.float64)
    st, at, _ = parts.losses()
    assert np.array_equal(st, op.state) and np.array_equal(at, op.at_turn)
    assert (op.state != 1).sum() >= 20 and (op.state == 1).sum() >= 20
    for j in range(n):
        last = min(int(op.at_turn[j]), 1023)
        assert np.array_equal(g[: last + 1, :, j], orec[: last + 1, :, j]), j
        assert np.all(np.isnan(g[last + 1:, :, j])), j


def test_recorder_resumes_and_ignores_later_turns(P, oracle_mod):
    """Recording across several track calls equals one call; turns past the
    buffer's length are not written."""
    import torch
    from oracle import features as F
    el = I.cfg1_lattice(rf_on=False)
    c, _, _ = I.polar_grid(6, 3, 14.0, _twiss(), EMIT, delta=2.7e-4)
    orec, _ = F.record(el, REF, c, turns=40, fp32=True)
    lat = P.Lattice(el, REF)
    parts = P.Particles(len(c), REF).init(c)
    rec = torch.full((32, 4, len(c)), float("nan"), dtype=torch.float32, device="cuda")
    for k in (7, 13, 20):
        P.track(lat, parts, k, record=rec)
    assert np.array_equal(rec.cpu().numpy().astype(np.float64), orec[:32])


# ------------------------------------------------------------------ features
FEATURE_TURN_GROUPS = {
    "fp64_stats": [0, 1, 2, 3, 10, 11, 12, 13, 14, 15],
    "tunes": [4, 5, 6, 7],
    "diffusion": [8, 9],
}


def _feature_case(oracle_mod, rf_on=True, n_r=12, n_t=8, rmax=16.0):
    from oracle import features as F
    el = I.cfg1_lattice(rf_on=rf_on)
    c, r, th = I.polar_grid(n_r, n_t, rmax, _twiss(), EMIT, delta=2.7e-4)
    keep = r > 0
    c = c[keep]
    rec, p = F.record(el, REF, c, fp32=True)
    assert np.all(p.state == 1)
    return rec, F.features(rec, _twiss(), EMIT, I.CFG1_APERTURE)


def assert_features_close(g, o):
    """Gates derived from the arithmetic: the action statistics are FP64 on
    both sides and stored in FP32 (relative 1e-6); tunes come from FP32
    512-point FFTs (absolute 1e-6); the tune-diffusion logarithm is compared
    through 10^f (absolute 3e-7, two FP32 tune roundings and the FFT error)."""
    for j in FEATURE_TURN_GROUPS["fp64_stats"]:
        err = np.abs(g[:, j] - o[:, j])
        assert np.all(err <= 1e-6 * np.abs(o[:, j]) + 1e-12), (j, err.max())
    for j in FEATURE_TURN_GROUPS["tunes"]:
        d = np.abs(g[:, j] - o[:, j]) % 1.0
        d = np.minimum(d, 1 - d)
        assert np.all(d <= 1e-6), (j, d.max())
    for j in FEATURE_TURN_GROUPS["diffusion"]:
        err = np.abs(10.0 ** g[:, j] - 10.0 ** o[:, j])
        assert np.all(err <= 3e-7), (j, err.max())


def test_features_match_oracle(P, oracle_mod):
    import torch
    rec, fo = _feature_case(oracle_mod)
    d = torch.tensor(rec.astype(np.float32), device="cuda").contiguous()
    fg = P.features(d, _twiss(), EMIT, I.CFG1_APERTURE).cpu().numpy().astype(np.float64)
    assert fg.shape == fo.shape
    assert_features_close(fg, fo)


def test_features_from_gpu_record(P, oracle_mod):
    """End to end: record on the GPU (cfg1 with RF), features on the GPU,
    against the oracle's record and features."""
    import torch
    from oracle import features as F
    el = I.cfg1_lattice()
    c, r, _ = I.polar_grid(10, 6, 15.0, _twiss(), EMIT, delta=2.7e-4)
    c = c[r > 0]
    orec, _ = F.record(el, REF, c, fp32=True)
    fo = F.features(orec, _twiss(), EMIT, I.CFG1_APERTURE)
    lat = P.Lattice(el, REF)
    parts = P.Particles(len(c), REF).init(c)
    rec = torch.zeros((1024, 4, len(c)), dtype=torch.float32, device="cuda")
    P.track(lat, parts, 1024, record=rec)
    g = rec.cpu().numpy().astype(np.float64)
    # tracking is bitwise (the RF sine is the shared series), so is the record
    assert np.array_equal(g, orec)
    fg = P.features(rec, _twiss(), EMIT, I.CFG1_APERTURE).cpu().numpy().astype(np.float64)
    assert_features_close(fg, fo)


def test_feature_argument_errors(P):
    import torch
    rec = torch.zeros((1024, 4, 3), dtype=torch.float32, device="cuda")
    with pytest.raises(P.XtmError):
        P.features(rec, (0.0, 0.0, 1.0, 0.0), EMIT, 0.04)
    with pytest.raises(P.XtmError):
        P.features(rec, (1.0, 0.0, 1.0, 0.0), -1.0, 0.04)
    assert P.features(rec[:, :, :0].contiguous(), (1.0, 0.0, 1.0, 0.0), EMIT, 0.04).shape == (0, 16)


def test_feature_stats(P):
    import torch
    rng = np.random.default_rng(11)
    f = (rng.normal(size=(3001, 16)) * np.arange(1, 17) + np.arange(16) * 3).astype(np.float32)
    f[:, 7] = 2.5                                   # constant column -> inv std 1
    mask = (rng.random(3001) < 0.7).astype(np.int32)
    g = P.feature_stats(torch.tensor(f, device="cuda"),
                        torch.tensor(mask, device="cuda")).cpu().numpy()
    sel = f[mask != 0].astype(np.float64)
    mean, std = sel.mean(0), sel.std(0)
    inv = np.where(std > 0, 1 / np.where(std > 0, std, 1), 1.0)
    assert np.allclose(g[:16], mean, rtol=1e-6, atol=1e-6)
    assert np.allclose(g[16:], inv, rtol=1e-5)
    assert g[16 + 7] == 1.0
    g2 = P.feature_stats(torch.tensor(f, device="cuda")).cpu().numpy()
    assert np.allclose(g2[:16], f.astype(np.float64).mean(0), rtol=1e-6, atol=1e-6)


# ------------------------------------------------------------------ network
def _net_inputs(B, seed=5):
    from oracle import mlp
    rng = np.random.default_rng(seed)
    theta = np.zeros(mlp.N_PARAMS)
    o = 0
    for name, shape in mlp.SIZES:
        n = int(np.prod(shape))
        std = math.sqrt(2.0 / shape[0]) if name[0] in "Ww" else 0.05
        theta[o:o + n] = rng.normal(0, std, n)
        o += n
    theta = theta.astype(np.float32)
    x = (rng.normal(size=(B, 16)) * np.linspace(0.5, 3, 16) + np.linspace(-2, 2, 16)).astype(np.float32)
    norm = np.concatenate([np.linspace(-2, 2, 16), 1 / np.linspace(0.5, 3, 16)]).astype(np.float32)
    y = (rng.random(B) < 0.3).astype(np.float32)
    return theta, x, norm, y


@pytest.mark.parametrize("B", [1, 63, 64, 1000, 4099])
def test_mlp_forward_matches_oracle(P, B):
    import torch
    from oracle import mlp
    theta, x, norm, _ = _net_inputs(B)
    t = lambda a: torch.tensor(a, device="cuda")
    z = P.mlp_forward(t(theta), t(norm), t(x)).cpu().numpy().astype(np.float64)
    zo = mlp.forward(theta.astype(np.float64), mlp.standardise(x, norm))["z3"]
    err = np.abs(z - zo)
    assert np.all(err <= 1e-3 * (1 + np.abs(zo))), err.max()


@pytest.mark.parametrize("B", [4096, 1000])
def test_mlp_gradient_matches_oracle(P, B):
    import torch
    from oracle import mlp
    theta, x, norm, y = _net_inputs(B, seed=7)
    w = float((y == 0).sum() / max((y == 1).sum(), 1))
    t = lambda a: torch.tensor(a, device="cuda")
    g, loss = P.mlp_grad(t(theta), t(norm), t(x), t(y), w)
    g = g.cpu().numpy().astype(np.float64)
    Lo, go = mlp.backward(theta.astype(np.float64), mlp.standardise(x, norm), y, w)
    assert abs(float(loss.cpu()[0]) - Lo) <= 1e-4 * abs(Lo)
    gp, op = mlp.unpack(g), mlp.unpack(go)
    for name, _ in mlp.SIZES:
        a, b = gp[name].ravel(), op[name].ravel()
        rel = np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30)
        cos = a @ b / max(np.linalg.norm(a) * np.linalg.norm(b), 1e-30)
        assert rel <= 1e-2 and cos >= 0.999, (name, rel, cos)


@pytest.mark.parametrize("B", [4096, 1000])
def test_mlp_gradient_elementwise_bound(P, B):
    """Every gradient element within 2^-7 of its magnitude scale: the same
    backward sums taken over absolute values (|A|^T |D| for a weight, sum |D|
    for a bias, no ReLU masks, so a unit whose sign differs between FP32 and
    FP64 is covered).  Both sides round the GEMM operands to BF16 at the same
    points; what is left is FP32 against FP64 accumulation (about 2^-24 of
    the scale per term) and a BF16 rounding that may fall one ulp (2^-8)
    apart where the value before it differs: together below 2^-8 of the
    scale at each of the two chained products, hence 2^-7.  (Removing every
    BF16 rounding on one side moves the elements by up to 2e-2 of the scale,
    which this bound does not admit.)"""
    import torch
    from oracle import mlp
    theta, x, norm, y = _net_inputs(B, seed=7)
    w = float((y == 0).sum() / max((y == 1).sum(), 1))
    t = lambda a: torch.tensor(a, device="cuda")
    g, _ = P.mlp_grad(t(theta), t(norm), t(x), t(y), w)
    gp = mlp.unpack(g.cpu().numpy().astype(np.float64))
    th = theta.astype(np.float64)
    _, go = mlp.backward(th, mlp.standardise(x, norm), y, w)
    op = mlp.unpack(go)
    f = mlp.forward(th, mlp.standardise(x, norm))
    p = mlp.unpack(th)
    yy = y.astype(np.float64)
    s = 1.0 / (1.0 + np.exp(-f["z3"]))
    m3 = np.abs(s * (w * yy + (1 - yy)) - w * yy) / B
    m2 = np.outer(m3, np.abs(p["w3"]))
    m1 = m2 @ np.abs(p["W2"]).T
    scale = {"b3": np.array([m3.sum()]), "w3": np.abs(f["H2"]).T @ m3,
             "b2": m2.sum(axis=0), "W2": np.abs(f["H1"]).T @ m2,
             "b1": m1.sum(axis=0), "W1": np.abs(f["X"]).T @ m1}
    for name, _ in mlp.SIZES:
        err = np.abs(gp[name] - op[name])
        bound = 2.0 ** -7 * scale[name] + 1e-12
        assert np.all(err <= bound), (name, float((err / bound).max()))


def test_adam_steps_match_oracle(P):
    import torch
    from oracle import mlp
    rng = np.random.default_rng(3)
    theta = rng.normal(0, 0.1, mlp.N_PARAMS).astype(np.float32)
    grads = [rng.normal(0, 1e-2, mlp.N_PARAMS).astype(np.float32) for _ in range(3)]
    tg = torch.tensor(theta, device="cuda")
    m = torch.zeros_like(tg)
    v = torch.zeros_like(tg)
    th, mo, vo = theta.astype(np.float64), np.zeros(mlp.N_PARAMS), np.zeros(mlp.N_PARAMS)
    for k, gr in enumerate(grads, start=1):
        P.mlp_adam(tg, m, v, torch.tensor(gr, device="cuda"), k, 1e-3)
        th, mo, vo = mlp.adam_step(th, mo, vo, gr.astype(np.float64), k, lr=1e-3)
    got = tg.cpu().numpy().astype(np.float64)
    assert np.all(np.abs(got - th) <= 1e-6 * np.abs(th) + 1e-9)
    # the step itself (theta - theta0) to 1e-3 relative
    d_g, d_o = got - theta, th - theta.astype(np.float64)
    assert np.linalg.norm(d_g - d_o) <= 1e-3 * np.linalg.norm(d_o)


def test_mlp_init_matches_oracle(P):
    from oracle import mlp
    seed = 2023
    g = P.mlp_init(seed).cpu().numpy()
    o = mlp.he_init(seed).astype(np.float32)
    ulp = np.abs(g.view(np.int32).astype(np.int64) - o.view(np.int32).astype(np.int64))
    assert np.all(ulp <= 1), ulp.max()
    assert np.all(g[2048:2176] == 0) and g[-1] == 0


# ------------------------------------------------------------------ retire
def test_retire_policy(P, oracle_mod):
    """Retire where logit >= threshold outside the 5 % audit set; retired
    particles keep their coordinates and stop being tracked; the rest
    continue bitwise as without retirement."""
    import torch
    el = I.cfg1_lattice(rf_on=False)
    c, r, _ = I.polar_grid(40, 50, 32.0, _twiss(), EMIT, delta=2.7e-4)
    n = len(c)
    lat = P.Lattice(el, REF)
    a = P.Particles(n, REF).init(c, first_id=1000)
    b = P.Particles(n, REF).init(c, first_id=1000)
    P.track(lat, a, 30)
    P.track(lat, b, 30)
    rng = np.random.default_rng(8)
    logit = torch.tensor(rng.normal(size=n).astype(np.float32), device="cuda")
    st0, _, _ = a.losses()
    seed = 0xC0FFEE
    retired, audited = P.retire(a, logit, 0.0, seed, 0.05)
    lg = logit.cpu().numpy()
    elig = (st0 == 1) & (lg >= 0.0)
    aud = oracle_mod.audit_mask(seed, np.arange(n) + 1000, 0.05)
    exp_ret = elig & ~aud
    st1, at1, _ = a.losses()
    assert retired == exp_ret.sum() and audited == (elig & aud).sum()
    assert np.array_equal(st1 == 2, exp_ret)
    snap = a.to_numpy()
    pa, alive_a = P.track(lat, a, 50)
    pb, alive_b = P.track(lat, b, 50)
    ga, gb = a.to_numpy(), b.to_numpy()
    keep = ~exp_ret
    for f in ("x", "px", "y", "py", "zeta", "delta", "state", "at_turn", "at_element"):
        assert np.array_equal(ga[f][keep], gb[f][keep]), f
        assert np.array_equal(ga[f][exp_ret], snap[f][exp_ret]), f
    assert alive_a == alive_b - int(((gb["state"] == 1) & exp_ret).sum())


def test_retire_infinite_threshold_is_plain_tracking(P):
    import torch
    el = I.cfg1_lattice(rf_on=False)
    c, _, _ = I.polar_grid(20, 10, 30.0, _twiss(), EMIT, delta=2.7e-4)
    lat = P.Lattice(el, REF)
    a = P.Particles(len(c), REF).init(c)
    b = P.Particles(len(c), REF).init(c)
    P.track(lat, a, 10)
    P.track(lat, b, 10)
    logit = torch.full((len(c),), 1e30, dtype=torch.float32, device="cuda")
    assert P.retire(a, logit, float("inf"), 1, 0.05) == (0, 0)
    P.track(lat, a, 40)
    P.track(lat, b, 40)
    ga, gb = a.to_numpy(), b.to_numpy()
    for f in ga:
        assert np.array_equal(ga[f], gb[f]), f


def test_audit_flags_verdict_and_resume_through_the_abi(P, oracle_mod):
    """Two decisions (turns 20 and 45) with audit flags, tracking to turn 120,
    the audit's verdict against the oracle's, then the library's fallback:
    every retired particle resumes from the turn it was retired at, and the
    whole set ends bit for bit as plain tracking to turn 120."""
    import torch
    el = I.cfg1_lattice(rf_on=False)
    c, _, _ = I.polar_grid(40, 50, 32.0, _twiss(), EMIT, delta=2.7e-4)
    n = len(c)
    lat = P.Lattice(el, REF)
    a = P.Particles(n, REF).init(c, first_id=500)
    plain = P.Particles(n, REF).init(c, first_id=500)
    P.track(lat, plain, 120)
    flags = torch.zeros(n, dtype=torch.int32, device="cuda")
    rng = np.random.default_rng(31)
    seed, frac = 0xABCDEF, 0.2
    eligible = np.zeros(n, dtype=bool)
    for t_dec, t_next in ((20, 45), (45, 120)):
        P.track(lat, a, t_dec - a.turn)
        st0, _, _ = a.losses()
        logit = torch.tensor(rng.normal(size=n).astype(np.float32), device="cuda")
        P.retire(a, logit, 0.3, seed, frac, audit_flags=flags)
        eligible |= (st0 == 1) & (logit.cpu().numpy() >= 0.3)
    P.track(lat, a, 120 - a.turn)
    aud = oracle_mod.audit_mask(seed, np.arange(n) + 500, frac)
    fl = flags.cpu().numpy()
    assert np.array_equal(fl != 0, eligible & aud)
    st, _, _ = a.losses()
    assert (st == 2).sum() == (eligible & ~aud).sum() > 0
    for rate in (1.0, 0.0):
        v = P.audit_verdict(a, flags, rate)
        o = oracle_mod.audit_verdict(st, fl, rate)
        assert (v["audited"], v["lost"], v["fallback"]) == (o["audited"], o["lost"], o["fallback"])
        assert abs(v["upper"] - o["upper"]) <= 1e-15
    assert P.audit_verdict(a, flags, 0.0)["fallback"]
    passes, alive = P.resume_retired(lat, a)
    assert a.turn == 120 and passes > 0
    ga, gp = a.to_numpy(), plain.to_numpy()
    for f in ("x", "px", "y", "py", "zeta", "delta", "ptau", "rpp", "rvv", "state", "at_turn",
              "at_element"):
        assert np.array_equal(ga[f].view(np.int64) if ga[f].dtype.kind == "f" else ga[f],
                              gp[f].view(np.int64) if gp[f].dtype.kind == "f" else gp[f]), f
    assert alive == int((gp["state"] == 1).sum())
    # the set goes on as one: 10 more turns equal plain tracking
    P.track(lat, a, 10)
    P.track(lat, plain, 10)
    ga, gp = a.to_numpy(), plain.to_numpy()
    for f in ("x", "state", "at_turn", "at_element"):
        assert np.array_equal(ga[f], gp[f]), f


def test_rule_score_matches_oracle(P, oracle_mod):
    import torch
    rng = np.random.default_rng(4)
    f = rng.normal(size=(1000, 16)).astype(np.float32)
    f[::97, 8] = np.nan
    f[5::101, 9] = np.nan
    got = P.rule_score(torch.tensor(f, device="cuda")).cpu().numpy()
    exp = oracle_mod.rule_score(f)
    assert np.array_equal(np.isnan(got), np.isnan(exp))
    m = ~np.isnan(exp)
    assert np.array_equal(got[m], exp[m])


# ------------------------------------------------------------------ training loop
def test_threshold_selection_matches_oracle(P, oracle_mod):
    import torch
    rng = np.random.default_rng(21)
    z = np.round(rng.normal(size=3000), 2).astype(np.float32)      # many ties
    y = (rng.random(3000) < 1 / (1 + np.exp(-3 * z))).astype(np.int32)
    for rate in (0.0, 1e-3, 0.05, 0.3):
        tau, fr, sel = P.select_threshold(torch.tensor(z, device="cuda"),
                                          torch.tensor(y, device="cuda"), rate)
        exp = oracle_mod.select_threshold(z, y, rate)
        assert tau == np.float32(exp) if np.isfinite(exp) else tau == np.inf, (rate, tau, exp)
        if np.isfinite(exp):
            m = z >= tau
            assert sel == m.sum() and abs(fr - np.mean(y[m] == 0)) < 1e-12


def test_training_loop_full_batch_equals_one_step(P):
    """One epoch with the whole set as the batch is one gradient + Adam step
    (row order changes only the FP32 summation order)."""
    import torch
    theta, x, norm, y = _net_inputs(512, seed=13)
    t = lambda a: torch.tensor(a, device="cuda")
    th1, m1, v1 = t(theta), torch.zeros(len(theta), device="cuda"), torch.zeros(len(theta), device="cuda")
    step, losses = P.mlp_train(th1, m1, v1, t(norm), t(x), t(y), 2.0, 1, 512, 1e-3, 99)
    assert step == 1 and losses.shape == (1,)
    th2, m2, v2 = t(theta), torch.zeros(len(theta), device="cuda"), torch.zeros(len(theta), device="cuda")
    g, loss = P.mlp_grad(th2, t(norm), t(x), t(y), 2.0)
    P.mlp_adam(th2, m2, v2, g, 1, 1e-3)
    a, b = th1.cpu().numpy(), th2.cpu().numpy()
    # Adam's first step is about lr sign(g): only gradients at the FP32
    # summation-noise level may take the other sign
    assert np.mean(np.abs(a - b) > 1e-4) <= 0.01
    assert np.abs(b - theta).max() > 5e-4
    assert abs(losses[0] - float(loss.cpu()[0])) <= 1e-5 * abs(float(loss.cpu()[0]))


def test_training_learns_a_separable_rule(P):
    import torch
    rng = np.random.default_rng(5)
    n = 20000
    x = rng.normal(size=(n, 16)).astype(np.float32)
    y = ((x[:, 0] + 0.5 * x[:, 3] - 0.3 * x[:, 7]) > 0.2).astype(np.float32)
    t = lambda a: torch.tensor(a, device="cuda")
    X = t(x)
    norm = P.feature_stats(X)
    theta = P.mlp_init(7)
    m, v = torch.zeros_like(theta), torch.zeros_like(theta)
    w = float((y == 0).sum() / (y == 1).sum())
    step, losses = P.mlp_train(theta, m, v, norm, X, t(y), w, 8, 1024, 3e-3, 1)
    assert step == 8 * 20 and losses[-1] < 0.5 * losses[0]
    z = P.mlp_forward(theta, norm, X).cpu().numpy()
    acc = np.mean((z > 0) == (y > 0.5))
    assert acc > 0.97, acc
