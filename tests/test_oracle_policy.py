"""Pins of the retire policy's reference pieces: the audit set drawn from the
Philox stream and the per-ray dynamic aperture of a polar scan."""
import math

import numpy as np

import oracle


def test_audit_fraction_is_binomial():
    for seed in (1, 2):
        ids = np.arange(40000) + 10 ** 6 * seed
        m = oracle.audit_mask(seed, ids, 0.05)
        sd = math.sqrt(0.05 * 0.95 / len(ids))
        assert abs(m.mean() - 0.05) < 4 * sd
    assert not oracle.audit_mask(3, np.arange(1000), 0.0).any()
    assert oracle.audit_mask(3, np.arange(1000), 1.0).all()


def test_audit_mask_uses_the_reserved_counter():
    # the decision is the first Philox word of counter (id_lo, id_hi, 2^32 - 1, 0)
    seed, pid = 0x0123456789ABCDEF, (5 << 32) + 17
    w = oracle.philox((17, 5, 0xFFFFFFFF, 0), (seed & 0xFFFFFFFF, seed >> 32))[0]
    f = (int(w) + 1) / 2.0 ** 32          # smallest fraction that audits it
    assert oracle.audit_mask(seed, [pid], f)[0]
    assert not oracle.audit_mask(seed, [pid], int(w) / 2.0 ** 32)[0]
    # nested sets: a larger fraction audits a superset
    ids = np.arange(5000)
    a, b = oracle.audit_mask(9, ids, 0.05), oracle.audit_mask(9, ids, 0.2)
    assert np.all(b[a])


def test_dynamic_aperture_brute_force():
    rng = np.random.default_rng(4)
    n_r, n_t = 7, 5
    radii = np.tile(np.linspace(0, 6, n_r), n_t)
    state = rng.choice([1, 0, -1, 2], size=n_r * n_t, p=[0.6, 0.2, 0.1, 0.1])
    state[n_r * 2:n_r * 3] = 1                      # a ray with no loss
    da = oracle.dynamic_aperture(state, radii, n_r, n_t)
    for j in range(n_t):
        lost = [radii[j * n_r + i] for i in range(n_r) if state[j * n_r + i] in (0, -1)]
        assert da[j] == (min(lost) if lost else math.inf)


def test_threshold_definition_on_hand_cases():
    z = np.array([3.0, 2.0, 1.0, 0.0, -1.0])
    y = np.array([1, 1, 0, 1, 1])
    assert oracle.select_threshold(z, y, 0.0) == 2.0
    assert oracle.select_threshold(z, y, 0.25) == -1.0      # 1 lost of 5 = 0.2
    assert oracle.select_threshold(z, y, 0.3) == -1.0
    assert oracle.select_threshold(np.array([1.0]), np.array([0]), 0.5) == np.inf


def test_wilson_upper_bound_against_scipy_and_closed_forms():
    """The audit's bound: the upper end of Wilson's score interval at the
    one-sided 95 % normal quantile, i.e. the upper end of scipy's two-sided
    90 % Wilson interval; with no loss it is z^2 / (n + z^2)."""
    from scipy.stats import binomtest, norm
    z = norm.ppf(0.95)
    assert abs(z - 1.6448536269514722) < 1e-15
    for k, n in ((0, 1), (0, 100), (1, 100), (41, 27449), (7, 20), (20, 20), (3, 5000)):
        ci = binomtest(k, n).proportion_ci(confidence_level=0.90, method="wilson")
        assert abs(oracle.wilson_upper(k, n) - ci.high) <= 1e-13, (k, n)
    for n in (1, 10, 1000, 10 ** 6):
        assert abs(oracle.wilson_upper(0, n) - z * z / (n + z * z)) <= 1e-15
    assert oracle.wilson_upper(0, 0) == 1.0
    assert abs(oracle.wilson_upper(5, 5) - 1.0) <= 2e-16
    # more losses, or the same fraction on fewer particles, never lower it
    ups = [oracle.wilson_upper(k, 1000) for k in range(0, 50)]
    assert all(b > a for a, b in zip(ups, ups[1:]))
    assert oracle.wilson_upper(1, 100) > oracle.wilson_upper(10, 1000)


def test_audit_verdict_by_hand():
    st = np.array([1, 1, 0, -1, 2, 2, 1, 0])
    fl = np.array([1, 0, 1, 1, 0, 0, 1, 0])
    v = oracle.audit_verdict(st, fl, 0.5)
    assert (v["audited"], v["lost"]) == (4, 2)
    assert abs(v["upper"] - oracle.wilson_upper(2, 4)) == 0.0
    assert v["fallback"] is (v["upper"] > 0.5)
    assert oracle.audit_verdict(st, fl, 0.99)["fallback"] is False
    # no retired particle: never a fallback, however bad the audit
    assert oracle.audit_verdict(np.array([0, 0]), np.array([1, 1]), 0.0)["fallback"] is False


def test_rule_score_by_hand():
    f = np.zeros((3, 16), dtype=np.float32)
    f[0, 8], f[0, 9] = -3.0, -5.0
    f[1, 8], f[1, 9] = -7.0, -2.5
    f[2, 8], f[2, 9] = np.nan, -1.0
    s = oracle.rule_score(f)
    assert s[0] == 3.0 and s[1] == 2.5 and np.isnan(s[2])
