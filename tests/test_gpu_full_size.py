"""Parity at the configurations' full sizes, in the launch configuration the
benchmark times (default kernel, automatic chunks): the whole ensemble is
tracked on the GPU through the C ABI, and a sample of its particles is
tracked alone by the oracle (each with its own id, so the radiation deviates
are its own) and compared element by element: loss state, turn and element
identical, coordinates bit for bit.  The sample takes particles evenly over
the set plus, where there are losses, some of the lost ones."""
import numpy as np
import pytest

from paper_2310_00317_amd import inputs as I
from parity_util import ALL_FLOAT

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2310_00317_amd as P
    P.lib()
    return P


def banner(msg):
    print(f"[full-size] {msg}", flush=True)


def _sample(g, n_even, n_lost, seed):
    n = len(g["state"])
    rng = np.random.default_rng(seed)
    idx = set(np.linspace(0, n - 1, n_even).astype(np.int64).tolist())
    lost = np.nonzero(g["state"] != 1)[0]
    if len(lost):
        idx |= set(rng.choice(lost, size=min(n_lost, len(lost)), replace=False).tolist())
    return np.array(sorted(idx), dtype=np.int64)


def _compare(g, idx, o, where):
    for f in ("state", "at_turn", "at_element"):
        a, b = g[f][idx], getattr(o, f)
        bad = np.nonzero(a != b)[0]
        assert bad.size == 0, (where, f, idx[bad[:5]], a[bad[:5]], b[bad[:5]])
    for f in ALL_FLOAT:
        a, b = g[f][idx], getattr(o, f)
        same = (a.view(np.int64) == b.view(np.int64)) | (np.isnan(a) & np.isnan(b))
        bad = np.nonzero(~same)[0]
        assert bad.size == 0, (where, f, idx[bad[:5]], a[bad[:5]], b[bad[:5]])


def _oracle_sample(oracle_mod, el, ref, coords, idx, turns, **kw):
    o = oracle_mod.init(coords[idx], ref)
    o.particle_id[:] = idx
    oracle_mod.track(el, ref, o, turns, **kw)
    return o


def test_da_scan_full_grid(P, oracle_mod):
    """The DA-scan workload: 100,000 protons on the 2000 x 50 polar grid of
    the 20,000-element errored ring, two steps of 1,000 turns."""
    banner("DA ring, 100,000 particles, 2 x 1,000 turns")
    el = I.cfg2_lattice()
    c, _, _ = I.cfg2_grid()
    assert len(c) == 100000
    lat = P.Lattice(el, I.PROTON_450GEV)
    parts = P.Particles(len(c), I.PROTON_450GEV).init(c)
    for _ in range(2):
        P.track(lat, parts, 1000)
    g = parts.to_numpy()
    idx = _sample(g, 96, 32, 1)
    banner(f"alive {int((g['state'] == 1).sum())}; oracle on {len(idx)} sampled particles")
    o = _oracle_sample(oracle_mod, el, I.PROTON_450GEV, c, idx, 2000)
    _compare(g, idx, o, "cfg2")
    assert (g["state"][idx] != 1).any() and (g["state"][idx] == 1).any()


def test_saturated_fodo_full(P, oracle_mod):
    """The FODO ring at 2^20 particles, 1,000 turns (the bench's FODO leg)."""
    banner("FODO ring, 2^20 particles, 1,000 turns")
    el = I.cfg1_lattice()
    c = I.cfg1_particles(1 << 20)
    lat = P.Lattice(el, I.PROTON_450GEV)
    parts = P.Particles(len(c), I.PROTON_450GEV).init(c)
    P.track(lat, parts, 1000)
    g = parts.to_numpy()
    idx = _sample(g, 128, 32, 2)
    o = _oracle_sample(oracle_mod, el, I.PROTON_450GEV, c, idx, 1000)
    _compare(g, idx, o, "cfg1sat")


@pytest.mark.parametrize("radiation", [2, 3])
def test_electron_ring_full(P, oracle_mod, radiation):
    """10^6 electrons matched to the electron ring's 6D normal form, two
    steps of 10 turns with quantum excitation (Gaussian, or photon by
    photon), as the radiation benchmark runs them."""
    banner(f"electron ring, 10^6 matched electrons, 2 x 10 turns, radiation {radiation}")
    ref = I.ELECTRON_45GEV6
    el = I.cfg5_lattice()
    lat = P.Lattice(el, ref)
    nf = P.twiss6d(lat, radiation=1)
    c = P.matched_gaussian(nf, ref, I.CFG5_EMITTANCES, I.standard_normals(1_000_000))
    parts = P.Particles(len(c), ref).init(c)
    for _ in range(2):
        P.track(lat, parts, 10, radiation=radiation, seed=20231002)
    g = parts.to_numpy()
    idx = _sample(g, 64, 16, 3)
    o = _oracle_sample(oracle_mod, el, ref, c, idx, 20, radiation=radiation, seed=20231002)
    _compare(g, idx, o, f"cfg5 radiation {radiation}")


def test_batched_variants_full(P, oracle_mod):
    """64 errored variants of the FODO ring with 2,000-50,000 particles each
    (1.76 M in all) in one batched launch per chunk, two steps of 200
    turns; two particles of every variant checked against the oracle
    tracking them through their own variant."""
    banner("64 batched variants, 1.76 M particles, 2 x 200 turns")
    ref = I.PROTON_450GEV
    counts = I.cfg3_counts()
    els, cs = [], []
    for v, n in enumerate(counts):
        e, c = I.cfg3_variant(v, int(n))
        els.append(e)
        cs.append(c)
    first = np.concatenate([[0], np.cumsum(counts)]).astype(np.int64)
    allc = np.concatenate(cs)
    batch = P.Batch([P.Lattice(e, ref) for e in els])
    parts = P.Particles(len(allc), ref).init(allc)
    for _ in range(2):
        P.track_batched(batch, parts, first, 200)
    g = parts.to_numpy()
    rng = np.random.default_rng(4)
    for v in range(len(counts)):
        a, b = int(first[v]), int(first[v + 1])
        idx = np.sort(rng.choice(np.arange(a, b), size=2, replace=False))
        o = _oracle_sample(oracle_mod, els[v], ref, allc, idx, 400)
        _compare(g, idx, o, f"variant {v}")
