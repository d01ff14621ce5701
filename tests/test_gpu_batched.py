"""Batched tracking of lattice variants and the launch-plan autotuner: the
batch must give, bit for bit, what tracking each variant alone gives, and
the autotuner must leave the set untouched and only change speed."""
import numpy as np
import pytest

from paper_2310_00317_amd import inputs as I
from parity_util import assert_bitwise, assert_parity

pytestmark = pytest.mark.gpu
REF = I.PROTON_450GEV
FIELDS = ("x", "px", "y", "py", "zeta", "delta", "ptau", "rpp", "rvv", "state", "at_turn",
          "at_element", "particle_id")


@pytest.fixture(scope="module")
def P():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2310_00317_amd as P
    P.lib()
    return P


def _variants(counts):
    """Errored cfg1 variants with cfg1 Gaussian beams; the first eighth of
    each beam is pushed out to ~14 sigma so that losses (and the loss replay)
    occur in every variant."""
    lats, coords = [], []
    for v, n in enumerate(counts):
        el, c = I.cfg3_variant(v, n)
        c = c.copy()
        c[: max(1, n // 8), [0, 2]] *= 14.0
        lats.append(el)
        coords.append(c[:n])
    return lats, coords


@pytest.mark.parametrize("chunk,graph,variant", [(64, False, 4), (0, False, 4), (50, True, 4),
                                               (0, False, 0), (64, False, 6), (0, False, 8),
                                               (50, True, 10), (0, False, 12), (7, False, 10),
                                               (0, False, 13), (50, True, 13), (0, False, 14),
                                               (50, True, 14)])
def test_batched_equals_separate(P, chunk, graph, variant):
    """Every batched kernel (the interpreter, and the one-wave per-line forms
    reading each variant's parameters) gives bit for bit what tracking each
    variant alone gives; the slot ranges are uneven, one is empty, and waves
    straddle variant boundaries."""
    counts = [37, 300, 0, 129, 64]
    els, coords = _variants(counts)
    first = np.concatenate([[0], np.cumsum(counts)]).astype(np.int64)
    lats = [P.Lattice(e, REF) for e in els]
    batch = P.Batch(lats)
    allc = np.concatenate(coords)
    big = P.Particles(len(allc), REF).init(allc)
    st = P.track_batched(batch, big, first, 300, turns_per_chunk=chunk, graph=graph,
                         variant=variant, full_stats=not graph)
    if not graph:
        # the default is the long-cell one-wave form
        assert st.variant == (14 if variant == 0 else variant)
    g = big.to_numpy()
    n_lost = 0
    for v, n in enumerate(counts):
        if n == 0:
            continue
        one = P.Particles(n, REF).init(coords[v], first_id=int(first[v]))
        P.track(lats[v], one, 300, variant=4)
        o = one.to_numpy()
        sl = slice(first[v], first[v + 1])
        for f in FIELDS:
            assert np.array_equal(g[f][sl], o[f], equal_nan=True), (v, f)
        n_lost += int((o["state"] != 1).sum())
    assert n_lost >= 40


def test_batched_matches_oracle(P, oracle_mod):
    counts = [50, 80]
    els, coords = _variants(counts)
    first = np.array([0, 50, 130], dtype=np.int64)
    lats = [P.Lattice(e, REF) for e in els]
    big = P.Particles(130, REF).init(np.concatenate(coords))
    P.track_batched(P.Batch(lats), big, first, 200)
    g = big.to_numpy()
    for v in range(2):
        o = oracle_mod.init(coords[v], REF, first_id=int(first[v]))
        oracle_mod.track(els[v], REF, o, 200)
        gv = {f: g[f][first[v]:first[v + 1]] for f in FIELDS}
        assert_parity(gv, o, rtol=1e-12)
        assert_bitwise(gv, o)


def test_batch_argument_errors(P):
    a = P.Lattice(I.cfg1_lattice(), REF)
    b = P.Lattice(I.cfg1_lattice(n_cells=50), REF)
    with pytest.raises(P.XtmError):
        P.Batch([a, b])                                   # element counts differ
    batch = P.Batch([a, a])
    parts = P.Particles(10, REF).init(I.gaussian_particles(10, 1))
    for bad in ([0, 5, 9], [1, 5, 10], [0, 7, 5]):
        with pytest.raises(P.XtmError):
            P.track_batched(batch, parts, bad, 1)
    with pytest.raises(P.XtmError):
        P.track_batched(batch, parts, [0, 5, 10], 1, variant=5)


def test_autotune_leaves_set_and_results_unchanged(P):
    el = I.cfg1_lattice()
    c = I.gaussian_particles(4096, 77)
    c[:300, [0, 2]] *= 14.0
    lat = P.Lattice(el, REF)
    a = P.Particles(len(c), REF).init(c)
    P.track(lat, a, 5)
    before = a.to_numpy()
    plan = P.autotune(a, lattice=lat, probe_turns=3)
    assert plan.variant in [4] + P.line_variants() and plan.block in (64, 128, 256)
    assert plan.passes_per_s > 0
    after = a.to_numpy()
    for f in FIELDS:
        assert np.array_equal(before[f], after[f]), f
    assert a.turn == 5
    b = P.Particles(len(c), REF).init(c)
    P.track(lat, b, 5, variant=4, block=256)
    P.track(lat, a, 100)                  # planned launch
    P.track(lat, b, 100, variant=4, block=256)
    ga, gb = a.to_numpy(), b.to_numpy()
    for f in FIELDS:
        assert np.array_equal(ga[f], gb[f]), f


def test_autotune_searches_chunk_length_and_compaction_period(P):
    """With a warm-up the probes start past the first turns' losses; the plan
    carries a chunk length and a compaction period, and tracking under it
    equals tracking with the defaults bit for bit."""
    el = I.cfg1_lattice()
    c = I.gaussian_particles(6000, 78)
    c[:2000, [0, 2]] *= 16.0            # a third lost within a few dozen turns
    lat = P.Lattice(el, REF)
    a = P.Particles(len(c), REF).init(c)
    plan = P.autotune(a, lattice=lat, probe_turns=20, warm_turns=10)
    assert plan.turns_per_chunk in (0, 1, 4, 16) and plan.compact_every in (1, 2, 4, 8)
    assert plan.passes_per_s > 0 and a.turn == 0
    b = P.Particles(len(c), REF).init(c)
    pa = P.track(lat, a, 150)                              # the plan
    pb = P.track(lat, b, 150, variant=10, turns_per_chunk=0, compact_every=1)
    ga, gb = a.to_numpy(), b.to_numpy()
    assert pa == pb
    for f in FIELDS:
        assert np.array_equal(ga[f], gb[f]), f


@pytest.mark.parametrize("variant", [4, 10, 13, 14])
def test_compaction_period_gives_the_same_results(P, variant):
    """Compacting the alive list only every few chunks (lost particles stay in
    the list in between) changes no result, eager or replayed as a graph."""
    el = I.cfg1_lattice()
    c = I.gaussian_particles(3000, 79)
    c[::3, [0, 2]] *= 16.0
    lat = P.Lattice(el, REF)
    ref_set = P.Particles(len(c), REF).init(c)
    pr = P.track(lat, ref_set, 60, variant=variant, turns_per_chunk=3)
    for every, graph in ((3, False), (7, False), (3, True)):
        x = P.Particles(len(c), REF).init(c)
        px = P.track(lat, x, 60, variant=variant, turns_per_chunk=3, compact_every=every,
                     graph=graph)
        assert px == pr, (every, graph)
        gx, gr = x.to_numpy(), ref_set.to_numpy()
        for f in FIELDS:
            assert np.array_equal(gx[f], gr[f]), (every, graph, f)
        # the set goes on as one after the period's last compaction
        alive_after = P.track(lat, x, 5, variant=variant)[1]
        fresh = P.Particles(len(c), REF).init(c)
        assert alive_after == P.track(lat, fresh, 65, variant=variant)[1]


def test_autotune_batch(P):
    counts = [200, 0, 500]
    els, coords = _variants(counts)
    first = np.array([0, 200, 200, 700], dtype=np.int64)
    batch = P.Batch([P.Lattice(e, REF) for e in els])
    big = P.Particles(700, REF).init(np.concatenate(coords))
    plan = P.autotune(big, batch=batch, first_slot=first, probe_turns=2)
    assert plan.variant in (4, 6, 8, 10, 12, 13, 14) and plan.block in (64, 128, 256)
    assert big.turn == 0


def test_batch_of_different_structures_uses_the_interpreter(P):
    """Variants whose element structures differ (one multipole of another
    order) cannot share a per-line kernel: the default falls back to the
    interpreter, with the same results as separate tracking; asking for a
    per-line form is an error."""
    el_a = I.cfg1_lattice()
    el_b = el_a.copy()
    k = int(np.nonzero(el_b["type"] == I.MULTIPOLE)[0][3])
    el_b["order"][k] = 3
    lats = [P.Lattice(el_a, REF), P.Lattice(el_b, REF)]
    c = I.gaussian_particles(200, 5)
    first = np.array([0, 100, 200], dtype=np.int64)
    big = P.Particles(200, REF).init(c)
    st = P.track_batched(P.Batch(lats), big, first, 50, full_stats=True)
    assert st.variant == 4
    g = big.to_numpy()
    for v in range(2):
        one = P.Particles(100, REF).init(c[100 * v:100 * (v + 1)], first_id=100 * v)
        P.track(lats[v], one, 50, variant=4)
        o = one.to_numpy()
        for f in FIELDS:
            assert np.array_equal(g[f][100 * v:100 * (v + 1)], o[f], equal_nan=True), (v, f)
    big2 = P.Particles(200, REF).init(c)
    with pytest.raises(P.XtmError) as ei:
        P.track_batched(P.Batch(lats), big2, first, 5, variant=10)
    assert ei.value.code == -6
