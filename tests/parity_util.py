"""Helpers for GPU-vs-oracle parity tests (test infrastructure)."""
import numpy as np

COORDS = ("x", "px", "y", "py", "zeta", "delta")

# Forward 100 turns then backward 100 turns of the FODO ring returns every
# surviving particle of this sample to within this many times
# max(|u0|, RMS of the coordinate): one bound for the oracle's own pin and
# for the GPU, on the same particles.
REVERSIBILITY_BOUND = 1e-11


def reversibility_sample():
    from paper_2310_00317_amd import inputs as I
    return I.cfg1_particles(500, seed=12)
ALL_FLOAT = COORDS + ("ptau", "rpp", "rvv")


def gpu_run(P, elements, ref, coords, n_turns, **kw):
    """Track on the GPU through the C ABI; returns (numpy dict, passes, alive, lattice, particles)."""
    lat = P.Lattice(elements, ref)
    parts = P.Particles(len(coords), ref).init(np.asarray(coords))
    passes, alive = P.track(lat, parts, n_turns, **kw)
    return parts.to_numpy(), passes, alive, lat, parts


def oracle_run(oracle, elements, ref, coords, n_turns):
    p = oracle.init(np.asarray(coords), ref)
    passes = oracle.track(elements, ref, p, n_turns)
    return p, passes


def rel_err(g, o, alive, floor_frac=1e-3):
    """|g - o| / max(|o|, s_c), s_c = floor_frac x RMS of o over alive particles."""
    out = {}
    for f in ALL_FLOAT:
        ov = getattr(o, f) if not isinstance(o, dict) else o[f]
        gv = g[f]
        rms = np.sqrt(np.mean(ov[alive] ** 2)) if alive.any() else 0.0
        sc = floor_frac * rms
        den = np.maximum(np.abs(ov), sc)
        with np.errstate(invalid="ignore", divide="ignore"):
            e = np.where(den > 0, np.abs(gv - ov) / den, np.abs(gv - ov))
        out[f] = e
    return out


def assert_parity(g, o, rtol=1e-12, mask=None, check_ints=True):
    """Coordinates within rtol (relative, with the RMS floor) on `mask`
    (default: particles alive on both sides); loss records identical."""
    ost = o.state
    alive = (ost == 1) & (g["state"] == 1)
    m = alive if mask is None else (mask & alive)
    if check_ints:
        for f in ("state", "at_turn", "at_element"):
            ov = getattr(o, f)
            bad = np.nonzero(g[f] != ov)[0]
            assert bad.size == 0, f"{f} differs at {bad[:10]} gpu={g[f][bad[:5]]} oracle={ov[bad[:5]]}"
        assert np.array_equal(g["particle_id"], o.particle_id)
    errs = rel_err(g, o, alive)
    worst = {}
    for f, e in errs.items():
        w = float(np.max(e[m])) if m.any() else 0.0
        worst[f] = w
        assert w <= rtol, f"{f}: worst relative error {w:.3e} > {rtol:.1e}"
    return worst


def bitwise_fraction(g, o, mask):
    eq = np.ones(len(g["x"]), dtype=bool)
    for f in ALL_FLOAT:
        eq &= (g[f] == getattr(o, f)) | (np.isnan(g[f]) & np.isnan(getattr(o, f)))
    return float(eq[mask].mean()) if mask.any() else 1.0


def assert_bitwise(g, o, fields=ALL_FLOAT + ("state", "at_turn", "at_element")):
    """Every listed field equal bit for bit (signed zeros included; NaN
    matches NaN whatever its payload): the rounding
    contract of the two implementations (same operation order, explicit
    fused multiply-adds, correctly rounded IEEE operations and the same
    series for sin, cos and log)."""
    for f in fields:
        a, b = np.asarray(g[f]), np.asarray(o[f] if isinstance(o, dict) else getattr(o, f))
        if a.dtype.kind == "f":
            # bit patterns (so +0 and -0 differ); any NaN matches any NaN
            same = (a.view(np.int64) == b.view(np.int64)) | (np.isnan(a) & np.isnan(b))
        else:
            same = a == b
        bad = np.nonzero(~same)[0]
        assert bad.size == 0, f"{f}: {bad.size} differ, first {bad[:5]}: {a[bad[:3]]} vs {b[bad[:3]]}"
