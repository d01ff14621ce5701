"""GPU parity: the HIP path (through the C ABI) against the CPU oracle on the
same seeded inputs.  Coordinates must agree within 1e-12 relative (with the
1e-3 x RMS floor) and loss records exactly; for drifts, multipoles, shifts,
rotations and apertures the rounding contract makes them bitwise equal."""
import math
import sys

import numpy as np
import pytest

from paper_2310_00317_amd import inputs as I
from parity_util import (REVERSIBILITY_BOUND, assert_bitwise, assert_parity, bitwise_fraction,
                         gpu_run, oracle_run, reversibility_sample)

pytestmark = pytest.mark.gpu
REF = I.PROTON_450GEV


@pytest.fixture(scope="module")
def P():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2310_00317_amd as P
    P.lib()
    return P


def banner(msg):
    print(f"[gpu-parity] {msg}", flush=True)
    sys.stdout.flush()


def test_cfg1_literal_100_turns(P, oracle_mod):
    banner("cfg1 literal: 1000 protons, 801 elements, 100 turns")
    el = I.cfg1_lattice()
    c = I.cfg1_particles(1000)
    g, gpasses, galive, _, _ = gpu_run(P, el, REF, c, 100)
    o, opasses = oracle_run(oracle_mod, el, REF, c, 100)
    worst = assert_parity(g, o, rtol=1e-12)
    assert gpasses == opasses
    assert galive == int((o.state == 1).sum())
    frac = bitwise_fraction(g, o, (o.state == 1))
    banner(f"worst rel err {max(worst.values()):.2e}; bitwise-equal fraction {frac:.4f}")
    assert_bitwise(g, o)


def test_cfg1_regular_orbits_and_losses(P, oracle_mod):
    banner("cfg1 with regular-orbit mask")
    el = I.cfg1_lattice()
    c = I.cfg1_particles(1000)
    g, _, _, _, _ = gpu_run(P, el, REF, c, 100)
    o, _ = oracle_run(oracle_mod, el, REF, c, 100)
    reg = oracle_mod.regular_mask(el, REF, c)
    assert_parity(g, o, rtol=1e-12, mask=reg)
    agree = np.mean((g["state"] == 1) == (o.state == 1))
    assert agree >= 0.999


def test_cfg1_misaligned_shifts_rotations(P, oracle_mod):
    banner("cfg1m: shifted and tilted quads")
    el = I.cfg1m_lattice()
    c = I.cfg1_particles(512, seed=5)
    g, gp, _, _, _ = gpu_run(P, el, REF, c, 50)
    o, op = oracle_run(oracle_mod, el, REF, c, 50)
    assert_parity(g, o, rtol=1e-12)
    assert gp == op


def test_expanded_drift_lattice(P, oracle_mod):
    banner("cfg1 with expanded drifts")
    el = I.cfg1_lattice(expanded_drift=True)
    c = I.cfg1_particles(256, seed=9)
    g, gp, _, _, _ = gpu_run(P, el, REF, c, 100)
    o, op = oracle_run(oracle_mod, el, REF, c, 100)
    assert_parity(g, o, rtol=1e-12)
    assert gp == op


def random_lattice(seed, n=200):
    rng = np.random.default_rng(seed)
    els = []
    for _ in range(n):
        k = rng.integers(0, 10)
        if k == 0:
            els.append(I.drift(rng.uniform(0.05, 0.5)))
        elif k == 1:
            els.append(I.drift(rng.uniform(0.05, 0.5), expanded=True))
        elif k in (2, 3):
            N = int(rng.integers(0, 11))
            # each order kicks by ~1e-7 rad at r = 10 mm
            scale = np.array([1e-7 * math.factorial(n) / 1e-2 ** n for n in range(N + 1)])
            knl = rng.normal(0, 1, N + 1) * scale
            ksl = rng.normal(0, 1, N + 1) * scale
            if k == 3:
                th = rng.normal(0, 1e-3)
                knl[0] = th
                els.append(I.multipole(knl=knl, ksl=ksl, hxl=th, length=rng.uniform(0, 3)))
            else:
                els.append(I.multipole(knl=knl, ksl=ksl))
        elif k == 4:
            els.append(I.rf(rng.uniform(1e5, 1e6), 4e8, rng.uniform(0, 360)))
        elif k == 5:
            els.append(I.xyshift(*rng.normal(0, 1e-4, 2)))
        elif k == 6:
            els.append(I.srotation(rng.normal(0, 0.3)))
        elif k == 7:
            els.append(I.ap_ellipse(0.008, 0.0065))
        elif k == 8:
            els.append(I.ap_rect(-0.0075, 0.008, -0.007, 0.0065))
        else:
            els.append(I.ap_circle(0.0085) if rng.random() < 0.5 else I.marker())
    return I.line(els)


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_every_element_type_random_lattice(P, oracle_mod, seed):
    banner(f"random lattice seed {seed}")
    el = random_lattice(seed)
    rng = np.random.default_rng(seed + 100)
    c = rng.normal(0, [3e-3, 2e-6, 3e-3, 2e-6, 0.05, 1e-3], (700, 6))
    g, gp, _, _, _ = gpu_run(P, el, REF, c, 20)
    o, op = oracle_run(oracle_mod, el, REF, c, 20)
    # the inputs exercise both outcomes
    assert 0.05 < np.mean(o.state == 1) < 0.98
    assert_parity(g, o, rtol=1e-12)
    assert gp == op


def test_resume_bitwise(P):
    banner("resume 37 + 63 == 100")
    el = I.cfg1_lattice()
    c = I.cfg1_particles(1000)
    a, _, _, _, _ = gpu_run(P, el, REF, c, 100)
    lat = P.Lattice(el, REF)
    parts = P.Particles(len(c), REF).init(c)
    P.track(lat, parts, 37)
    P.track(lat, parts, 63)
    assert parts.turn == 100
    b = parts.to_numpy()
    for f in a:
        assert np.array_equal(a[f], b[f], equal_nan=True), f


@pytest.mark.parametrize("opts", [dict(turns_per_chunk=1), dict(turns_per_chunk=7, block=64),
                                  dict(variant=4), dict(variant=4, turns_per_chunk=3, block=128),
                                  dict(turns_per_chunk=100, block=128, compact=False),
                                  dict(turns_per_chunk=33, block=192),
                                  dict(variant=5, turns_per_chunk=11),
                                  dict(variant=5, turns_per_chunk=5, compact=False),
                                  dict(variant=6, turns_per_chunk=11),
                                  dict(variant=7, turns_per_chunk=9),
                                  dict(variant=8), dict(variant=9, turns_per_chunk=4),
                                  dict(variant=10, turns_per_chunk=6, compact=False),
                                  dict(variant=11, turns_per_chunk=8),
                                  dict(variant=12), dict(variant=12, turns_per_chunk=3,
                                                         compact=False),
                                  dict(variant=13), dict(variant=13, turns_per_chunk=5,
                                                         compact=False),
                                  dict(variant=10), dict(variant=14, turns_per_chunk=7),
                                  dict(variant=14, turns_per_chunk=3, compact=False)])
def test_launch_shape_invariance(P, opts):
    banner(f"launch shape {opts}")
    el = I.cfg1_lattice()
    c = I.cfg1_particles(3000, seed=4)
    c[::50, 0] *= 25.0  # some early losses so compaction has work
    a, pa, _, _, _ = gpu_run(P, el, REF, c, 100)
    b, pb, _, _, _ = gpu_run(P, el, REF, c, 100, **opts)
    assert pa == pb
    for f in a:
        assert np.array_equal(a[f], b[f], equal_nan=True), f


@pytest.mark.parametrize("rf_on", [False, True])
def test_backward_parity_and_reversibility(P, oracle_mod, rf_on):
    """Forward 100 turns then backward 100 turns: every map, the RF sine
    included (both sides evaluate the same series), obeys the rounding
    contract, so the GPU equals the oracle bitwise; the 1e-12 gate of
    max(|value|, RMS of the coordinate) is checked as well."""
    banner(f"backward tracking, rf_on={rf_on}")
    el = I.cfg1_lattice(rf_on=rf_on)
    c = reversibility_sample()
    lat = P.Lattice(el, REF)
    parts = P.Particles(len(c), REF).init(c)
    P.track(lat, parts, 100)
    alive = parts.to_numpy()["state"] == 1
    P.track_backward(lat, parts, 100)
    assert parts.turn == 0
    g = parts.to_numpy()
    o = oracle_mod.init(c, REF)
    oracle_mod.track(el, REF, o, 100)
    oracle_mod.track_backward(el, REF, o, 100)
    from parity_util import rel_err
    alive_both = (o.state == 1) & (g["state"] == 1)
    errs = rel_err(g, o, alive_both, floor_frac=1.0)
    for f, e in errs.items():
        assert np.max(e[alive_both]) <= 1e-12, f
    assert_bitwise(g, o)
    # reversibility up to roundoff grown over 200 turns of a sextupolar ring,
    # the bound the oracle's own pin uses on the same sample
    rms = np.sqrt(np.mean(c[alive] ** 2, axis=0))
    for j, f in enumerate(("x", "px", "y", "py", "zeta", "delta")):
        err = np.abs(g[f][alive] - c[alive, j])
        bound = REVERSIBILITY_BOUND * np.maximum(np.abs(c[alive, j]), rms[j])
        assert np.all(err <= bound), (f, np.max(err / bound))


def test_edge_cases(P, oracle_mod):
    banner("edge cases")
    el = I.cfg1_lattice()
    # empty set
    lat = P.Lattice(el, REF)
    e = P.Particles(0, REF).init(np.zeros((0, 6)))
    assert P.track(lat, e, 10) == (0, 0)
    # zero turns leaves everything untouched
    c = I.cfg1_particles(64)
    g0, p0, a0, _, _ = gpu_run(P, el, REF, c, 0)
    assert p0 == 0 and a0 == 64 and np.array_equal(g0["x"], c[:, 0])
    # outside the aperture, NaN, imaginary pz, already lost on entry
    bad = np.array([[0.05, 0, 0, 0, 0, 0], [np.nan, 0, 0, 0, 0, 0], [0, 1.5, 0, 0, 0, 0],
                    [0, 0, np.inf, 0, 0, 0], [1e-3, 0, 1e-3, 0, 0, 0]])
    g, gp, ga, _, _ = gpu_run(P, el, REF, bad, 5)
    o, op = oracle_run(oracle_mod, el, REF, bad, 5)
    assert np.array_equal(g["state"], o.state) and np.array_equal(g["at_element"], o.at_element)
    assert np.array_equal(g["at_turn"], o.at_turn) and gp == op
    assert list(g["state"][:4]) == [0, 0, -1, 0]
    # empty lattice and an apertures-only lattice
    lat0 = P.Lattice(I.line([]), REF)
    p0 = P.Particles(4, REF).init(c[:4])
    assert P.track(lat0, p0, 10) == (0, 4)
    apl = I.line([I.ap_circle(1e-3), I.ap_rect(-1, 1, -1e-4, 1e-4)])
    g, gp, _, _, _ = gpu_run(P, apl, REF, c, 3)
    o, op = oracle_run(oracle_mod, apl, REF, c, 3)
    assert np.array_equal(g["state"], o.state) and gp == op


def test_reference_mismatch_is_an_error(P):
    lat = P.Lattice(I.cfg1_lattice(), REF)
    parts = P.Particles(8, I.Reference(I.PROTON_MASS_EV, 1.0, 451e9)).init(I.cfg1_particles(8))
    with pytest.raises(P.XtmError) as ei:
        P.track(lat, parts, 1)
    assert ei.value.code == -5


def test_cfg2_lattice_reduced(P, oracle_mod):
    banner("cfg2 lattice (20,000 elements), 300 grid particles, 5 turns")
    el = I.cfg2_lattice()
    c, r, th = I.cfg2_grid(n_r=60, n_theta=5, r_max_sigma=12.0)
    g, gp, _, _, _ = gpu_run(P, el, REF, c, 5)
    o, op = oracle_run(oracle_mod, el, REF, c, 5)
    assert_parity(g, o, rtol=1e-12)
    assert gp == op


def test_cfg2_loss_parity_at_da_scale(P, oracle_mod):
    """Lost/surviving agreement on the 20,000-element DA ring at a scan's
    turn count: five rays of the 50-angle grid, 241 radii each from 1.5 to
    9 sigma (spacing 1/32 sigma, straddling every ray's dynamic aperture),
    1,000 turns, the oracle on all host threads.  Gates: >= 99.9 % of the
    particles agree on lost/surviving, and any particle that disagrees lies
    within 0.05 sigma of its ray's dynamic aperture (the smallest radius the
    oracle loses on that ray); particles lost on both sides agree on turn
    and element.  The identity rate of the whole record is reported."""
    banner("cfg2 ring: 5 rays x 241 radii, 1,000 turns (loss parity at DA scale)")
    el = I.cfg2_lattice()
    c_all, r_all, _ = I.cfg2_grid(n_r=321, n_theta=50, r_max_sigma=10.0)
    rays = (5, 15, 25, 35, 45)
    ray_of = np.repeat(np.arange(50), 321)
    sel = np.isin(ray_of, rays) & (r_all >= 1.5) & (r_all <= 9.0)
    c, r, ray = c_all[sel], r_all[sel], ray_of[sel]
    assert len(c) == 5 * 241
    turns = 1000
    g, gp, _, _, _ = gpu_run(P, el, REF, c, turns)
    o, op = oracle_run(oracle_mod, el, REF, c, turns)
    g_alive, o_alive = g["state"] == 1, o.state == 1
    agree = g_alive == o_alive
    same_record = ((g["state"] == o.state) & (g["at_turn"] == o.at_turn)
                   & (g["at_element"] == o.at_element))
    da = {j: float(np.min(r[(ray == j) & ~o_alive], initial=np.inf)) for j in rays}
    banner(f"lost/surviving agreement {agree.mean():.5f}; identical loss records "
           f"{same_record.mean():.5f}; bitwise-equal coordinates "
           f"{bitwise_fraction(g, o, np.ones(len(c), bool)):.5f}; passes gpu {gp} oracle {op}; "
           f"DA per ray " + ", ".join(f"{j}: {da[j]:.3f}" for j in rays))
    assert 0.1 < o_alive.mean() < 0.9   # the radii straddle the aperture
    assert all(1.5 < da[j] < 9.0 for j in rays)
    assert agree.mean() >= 0.999
    for i in np.nonzero(~agree)[0]:
        assert abs(r[i] - da[int(ray[i])]) <= 0.05, (i, r[i], da[int(ray[i])])
    both_lost = ~g_alive & ~o_alive
    assert np.array_equal(g["at_turn"][both_lost], o.at_turn[both_lost])
    assert np.array_equal(g["at_element"][both_lost], o.at_element[both_lost])
    assert np.array_equal(g["state"][both_lost], o.state[both_lost])


@pytest.mark.parametrize("variant", [4, 5, 6, 7, 8, 9, 10, 11, 12, 13, 14])
def test_kernel_variants_on_multisegment_lattice(P, variant):
    """The 20,000-element lattice spans many LDS segments: every kernel variant
    must give bitwise the same result as the default one."""
    banner(f"cfg2 lattice, variant {variant} vs default")
    el = I.cfg2_lattice()
    c, _, _ = I.cfg2_grid(n_r=100, n_theta=6, r_max_sigma=40.0)  # 22% lost within 6 turns
    a, pa, _, _, _ = gpu_run(P, el, REF, c, 6)
    b, pb, _, _, _ = gpu_run(P, el, REF, c, 6, variant=variant, turns_per_chunk=2)
    assert (a["state"] != 1).any()
    assert pa == pb
    for f in a:
        assert np.array_equal(a[f], b[f], equal_nan=True), f


def test_graph_replay_matches_eager(P):
    """The chunk sequence captured as a hipGraph and replayed several times
    (with eager work and synchronisations in between) gives bitwise the eager
    result after every replay."""
    banner("hipGraph replay vs eager")
    el = I.cfg1_lattice()
    c = I.cfg1_particles(3000, seed=21)
    c[::40, 0] *= 25.0
    lat = P.Lattice(el, REF)
    eager = P.Particles(len(c), REF).init(c)
    graph = P.Particles(len(c), REF).init(c)
    for rep in range(4):
        pe = P.track(lat, eager, 30, turns_per_chunk=7)
        pg = P.track(lat, graph, 30, turns_per_chunk=7, graph=True, stats=(rep % 2 == 0))
        if pg is not None:
            assert pg == pe
        a, b = eager.to_numpy(), graph.to_numpy()
        for f in a:
            assert np.array_equal(a[f], b[f], equal_nan=True), (rep, f)
        assert graph.turn == eager.turn == 30 * (rep + 1)


def test_graph_cache_survives_lattice_reuse(P):
    """A particle set keeps the graphs it captured.  After the lattice it
    tracked is destroyed, a new lattice (often at the same host address, the
    heap reuses it) tracked with the same options must capture its own graph:
    the result equals eager tracking through the new lattice, bit for bit."""
    banner("graph cache after lattice destroy and re-create")
    el_a = I.cfg1_lattice()
    el_b = I.cfg1_lattice()
    el_b["knl"][:, 2] *= -1.5  # same structure, other sextupoles
    c = I.cfg1_particles(2000, seed=23)
    c[::50, 0] *= 25.0  # some losses
    lat_a2 = P.Lattice(el_a, REF)
    ref = P.Particles(len(c), REF).init(c)
    P.track(lat_a2, ref, 20, turns_per_chunk=5)
    lat = P.Lattice(el_a, REF)
    parts = P.Particles(len(c), REF).init(c)
    P.track(lat, parts, 20, turns_per_chunk=5, graph=True)
    addr_a = lat.handle.value
    lat.close()
    lat_b = P.Lattice(el_b, REF)
    print(f"handle reused: {lat_b.handle.value == addr_a}", flush=True)
    P.track(lat_b, parts, 20, turns_per_chunk=5, graph=True)
    P.track(lat_b, ref, 20, turns_per_chunk=5)
    a, b = parts.to_numpy(), ref.to_numpy()
    for f in ("x", "px", "y", "py", "zeta", "delta", "state", "at_element"):
        assert np.array_equal(a[f], b[f], equal_nan=True), f


def test_empty_lattice_counts_turns(P, oracle_mod):
    c = I.cfg1_particles(8)
    g, gp, ga, _, _ = gpu_run(P, I.line([]), REF, c, 10)
    o, op = oracle_run(oracle_mod, I.line([]), REF, c, 10)
    assert gp == op == 0 and ga == 8
    assert np.array_equal(g["at_turn"], o.at_turn) and np.all(o.at_turn == 10)


def test_variant_numbers(P):
    """Every per-line form is a kernel number; one past the last is refused."""
    assert P.line_variants() == list(range(5, 15))
    lat = P.Lattice(I.cfg1_lattice(), REF)
    parts = P.Particles(8, REF).init(np.zeros((8, 6)))
    with pytest.raises(P.XtmError) as ei:
        P.track(lat, parts, 1, variant=15)
    assert ei.value.code == -1


def test_line_kernel_unavailable_for_irregular_lattice(P):
    """An irregular 200-element line has no compact cell structure: asking for
    the per-line kernel explicitly is an error, the default falls back."""
    el = random_lattice(1)
    c = np.zeros((64, 6))
    lat = P.Lattice(el, REF)
    parts = P.Particles(64, REF).init(c)
    with pytest.raises(P.XtmError) as ei:
        P.track(lat, parts, 1, variant=5)
    assert ei.value.code == -6
    P.track(lat, parts, 1)
    assert parts.turn == 1


def large_cell_lattice(seed=3, units=30):
    """Repeating 19-element unit [aperture 5 mm, 6 x (order-10 multipole with
    an alternating +-0.8 quadrupole, 1 m drift, order-10 multipole with a
    sextupole)] whose parameters (271 words) exceed one word per lane of a
    256-lane workgroup, with different random strengths in every unit, so the
    per-line kernel stages each cell in several passes and stale or misplaced
    parameters would show."""
    rng = np.random.default_rng(seed)
    err = lambda: rng.normal(0, 1e-5, 11) * 10.0 ** -np.arange(11)
    els = []
    for _ in range(units):
        els.append(I.ap_circle(0.005))
        for k in range(6):
            knl, ksl = err(), err()
            knl[1] += 0.8 if k % 2 == 0 else -0.8
            els.append(I.multipole(knl=knl, ksl=ksl, order=10))
            els.append(I.drift(1.0))
            knl, ksl = err(), err()
            knl[2] += rng.normal(0, 0.5)
            els.append(I.multipole(knl=knl, ksl=ksl, order=10))
    return I.line(els)


@pytest.mark.parametrize("variant", [0, 4, 6, 7, 8, 9, 10, 11, 12, 13, 14])
def test_line_kernel_with_multi_pass_staging(P, oracle_mod, variant):
    banner(f"large-cell lattice, variant {variant}")
    el = large_cell_lattice()
    c = I.gaussian_particles(700, 31, [2e-3, 3e-4, 2e-3, 3e-4, 0.05, 1e-4])
    g, gp, _, _, _ = gpu_run(P, el, REF, c, 30, variant=variant)
    o, op = oracle_run(oracle_mod, el, REF, c, 30)
    assert gp == op
    assert_bitwise(g, o)
    assert 0.05 < np.mean(o.state == 1) < 0.98


@pytest.mark.parametrize("lattice", ["cfg1", "cfg2"])
def test_per_element_baseline_equals_tracking(P, lattice):
    """The one-launch-per-element baseline applies the same maps: every
    coordinate, state, loss turn and element equal the default tracker's bit
    for bit, and so do the pass counts (losses included)."""
    banner(f"per-element baseline, {lattice}")
    if lattice == "cfg1":
        el, turns = I.cfg1_lattice(), 60
        c = I.cfg1_particles(3000, seed=8)
        c[::40, 0] *= 25.0
    else:
        el, turns = I.cfg2_lattice(), 3
        c, _, _ = I.cfg2_grid(n_r=60, n_theta=5, r_max_sigma=40.0)
    a, pa, aa, _, _ = gpu_run(P, el, REF, c, turns)
    lat = P.Lattice(el, REF)
    parts = P.Particles(len(c), REF).init(c)
    st = P.track_per_element(lat, parts, turns)
    b = parts.to_numpy()
    assert (a["state"] != 1).any()
    assert st.passes == pa and st.alive == aa and st.launches == turns * len(el)
    assert parts.turn == turns
    for f in a:
        assert np.array_equal(a[f], b[f], equal_nan=True), f
    # the rebuilt alive list lets ordinary tracking continue from here
    P.track(lat, parts, 2)
    assert parts.turn == turns + 2


def test_drift_domain_edges(P, oracle_mod):
    """The drift's square root and quotients over its whole domain, bit for
    bit equal to the oracle's IEEE operations: momenta from near zero
    (1 + delta = 2^-299) to 2^100, angles up to nearly 90 degrees, the edges
    of the short sequences' window (pz^2 at 2^-600 and 4, numerators of
    d(2+d) - px^2 - py^2 below 2^-600, signed zeros), the divisors with an
    all-ones significand (1 + pz = 2 - 2^-52 with a power-of-two numerator,
    pz = 1 - 2^-53 with power-of-two lengths), lengths from 0 and 1e-200 m
    to 1e80 m, and particles whose pz^2 is not positive (lost)."""
    banner("drift domain edges")
    rng = np.random.default_rng(5)
    deltas = np.array([0.0, -0.0, 1e-300, 1e-3, -0.5, -1 + 2.0 ** -299, -1 + 2.0 ** -300,
                       -1 + 2.0 ** -290, -1 + 2.0 ** -301, 1.0, 1.0 - 2.0 ** -52, 2.0 ** 100,
                       2.0 ** 299, 3.0])
    rows = []
    for d in deltas:
        opd = 1.0 + d
        for frac in (0.0, 1e-9, 0.3, 0.7, 0.999999, 1.0 - 2.0 ** -40, 1.0):
            a = frac * abs(opd)
            phi = rng.uniform(0, 2 * np.pi)
            rows.append([1e-3, a * np.cos(phi), -2e-3, a * np.sin(phi), 0.01, d])
    # pz^2 = 1 - 2^-51, pz = 1 - 2^-52, 1 + pz = 2 - 2^-52, numerator -2^-51
    rows.append([1e-3, 2.0 ** -26, -2e-3, 2.0 ** -26, 0.01, 0.0])
    rows.append([-0.0, 2.0 ** -26, 0.0, -(2.0 ** -26), -0.0, 0.0])
    # pz^2 = 1 - 2^-52, pz = 1 - 2^-53 (all-ones significand)
    rows.append([1e-3, 0.0, -2e-3, 2.0 ** -26, 0.01, 0.0])
    rows.append([1e-3, 2.0 ** -26, -2e-3, 0.0, 0.01, -0.0])
    # pz^2 just below 4 (delta = 1)
    rows.append([1e-3, 2.0 ** -20, -2e-3, 0.0, 0.01, 1.0])
    c = np.array(rows)
    lengths = [1e-200, 1.0, 0.0, 1e80, -1.0, 0.75, -0.0, 2.0 ** -601, 3.0, 0.5, -(2.0 ** 600),
               1e-80]
    el = I.line([I.drift(L) for L in lengths])
    g, gp, _, _, _ = gpu_run(P, el, REF, c, 1, variant=4)
    o, op = oracle_run(oracle_mod, el, REF, c, 1)
    assert gp == op
    assert (o.state != 1).any() and (o.state == 1).sum() > len(c) // 2
    assert_bitwise(g, o)
    for v in (0, 5, 10, 12, 13, 14):
        gv, _, _, _, _ = gpu_run(P, el, REF, c, 1, variant=v)
        for f in g:
            assert np.array_equal(np.asarray(gv[f]).view(np.uint8),
                                  np.asarray(g[f]).view(np.uint8)), (v, f)
