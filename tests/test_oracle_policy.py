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
