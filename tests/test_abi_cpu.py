"""CPU-side checks of the C-ABI library: it loads, exports every declared
entry point, and validates its arguments before touching a device."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_2310_00317_amd import inputs as I

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "xtm.h")


def declared_functions():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(xtm_[a-z0-9_]+)\s*\(", txt)))


@pytest.fixture(scope="module")
def xtm():
    import paper_2310_00317_amd as P
    if not os.path.exists(P.LIB_PATH):
        pytest.fail("libxtm.so is not built (run __graft_entry__.build())")
    return P


def test_header_declares_the_boundary():
    names = declared_functions()
    for n in ("xtm_lattice_create", "xtm_particles_bind", "xtm_particles_init", "xtm_track",
              "xtm_track_backward", "xtm_get_losses", "xtm_sync"):
        assert n in names


def test_library_exports_every_declared_symbol(xtm):
    L = xtm.lib()
    missing = [n for n in declared_functions() if not hasattr(L, n)]
    assert not missing, missing


def test_element_struct_layout_matches_header():
    # offsets of xtm_element_desc under natural alignment
    d = I.ELEMENT_DTYPE
    assert d.itemsize == 248
    assert [d.fields[k][1] for k in d.names] == [0, 4, 8, 16, 104, 192, 200]


def _create(xtm, els, ref=I.PROTON_450GEV):
    r = xtm._ref_struct(ref)
    h = ctypes.c_void_p()
    code = xtm.lib().xtm_lattice_create(els.ctypes.data_as(ctypes.c_void_p), len(els),
                                        ctypes.byref(r), ctypes.byref(h))
    return code, h


@pytest.mark.parametrize("mutate,expected", [
    (lambda e: e.__setitem__("type", 99), -2),
    (lambda e: (e.__setitem__("type", I.MULTIPOLE), e.__setitem__("order", 11)), -2),
    (lambda e: (e.__setitem__("type", I.MULTIPOLE), e.__setitem__("order", -1)), -2),
    (lambda e: (e.__setitem__("type", I.AP_CIRCLE)), -2),                       # r = 0
    (lambda e: (e.__setitem__("type", I.AP_ELLIPSE), e["p"].__setitem__(0, 1.0)), -2),
    (lambda e: (e.__setitem__("type", I.AP_RECT), e["p"].__setitem__(slice(0, 4), [1, 0, -1, 1])), -2),
    (lambda e: (e.__setitem__("type", I.DRIFT), e.__setitem__("length", np.inf)), -2),
    (lambda e: (e.__setitem__("type", I.RF), e["p"].__setitem__(1, -1.0)), -2),
])
def test_invalid_elements_rejected_before_any_device_work(xtm, mutate, expected):
    els = I.line([I.drift(1.0), I.drift(1.0)])
    e = els[1]
    mutate(e)
    els[1] = e
    code, h = _create(xtm, els)
    assert code == expected
    assert h.value is None
    msg = xtm.lib().xtm_last_error().decode()
    assert "element 1" in msg


def test_bad_reference_and_arguments(xtm):
    els = I.line([I.drift(1.0)])
    code, _ = _create(xtm, els, I.Reference(0.0, 1.0, 1e9))
    assert code == -5
    r = xtm._ref_struct(I.PROTON_450GEV)
    h = ctypes.c_void_p()
    assert xtm.lib().xtm_lattice_create(None, 3, ctypes.byref(r), ctypes.byref(h)) == -1
    assert xtm.lib().xtm_lattice_create(None, 0, ctypes.byref(r), None) == -1
    a = xtm._Arrays()
    a.n = -1
    assert xtm.lib().xtm_particles_bind(ctypes.byref(a), ctypes.byref(r), ctypes.byref(h)) == -1
    a.n = 10  # null arrays
    assert xtm.lib().xtm_particles_bind(ctypes.byref(a), ctypes.byref(r), ctypes.byref(h)) == -1
    assert xtm.lib().xtm_track(None, None, 1, None, None, None) == -1
    assert xtm.lib().xtm_particles_turn(None, None) == -1


def test_version_string(xtm):
    assert b"gfx950" in xtm.lib().xtm_version()


def test_dynamic_aperture_host_function_matches_oracle(oracle_mod):
    """xtm_dynamic_aperture is host-only: checked here against the oracle's
    definition on random scans (retired particles, state 2, are survivors)."""
    import paper_2310_00317_amd as P
    rng = np.random.default_rng(12)
    for n_r, n_t in ((1, 1), (9, 4), (200, 7)):
        st = rng.choice([1, 0, -1, 2], size=n_r * n_t, p=[0.7, 0.15, 0.05, 0.1]).astype(np.int32)
        r = rng.random(n_r * n_t) * 30
        got = P.dynamic_aperture(st, r, n_r, n_t)
        exp = oracle_mod.dynamic_aperture(st, r, n_r, n_t)
        assert np.array_equal(got, exp)
    with pytest.raises(P.XtmError):
        P.lib()
        P.check(P.lib().xtm_dynamic_aperture(None, None, 0, 0, None), "xtm_dynamic_aperture")


def test_noalloc_gradient_checks_its_arguments_before_any_device_work(xtm):
    """The allocation-free gradient rejects batches beyond its fixed
    workspace (and empty ones) before it looks at any pointer or device."""
    L = xtm.lib()
    fake = ctypes.c_void_p(256)   # never dereferenced: the call fails first
    for B in (0, -1, 4097, 1 << 40):
        assert L.xtm_mlp_grad_noalloc(fake, fake, fake, fake, B, 1.0, fake, None, None) == -1
        assert b"4096" in L.xtm_last_error()
    assert L.xtm_mlp_grad_noalloc(None, fake, fake, fake, 8, 1.0, fake, None, None) == -1
    assert L.xtm_mlp_grad_noalloc(fake, fake, fake, fake, 8, 1.0, None, None, None) == -1


def test_audit_upper_bound_host_function_matches_oracle(oracle_mod):
    """xtm_audit_upper_bound is host-only: checked against the oracle's
    Wilson bound, and its argument checks."""
    import paper_2310_00317_amd as P
    for k, n in ((0, 0), (0, 1), (0, 100), (1, 100), (41, 27449), (7, 20), (20, 20)):
        got = P.audit_upper_bound(k, n)
        assert abs(got - oracle_mod.wilson_upper(k, n)) <= 1e-15 * max(1.0, got), (k, n)
    for k, n in ((-1, 5), (6, 5), (0, -1)):
        with pytest.raises(P.XtmError):
            P.audit_upper_bound(k, n)


def test_photon_table_equals_the_oracle_table():
    """The library computes the photon-spectrum table on the host with its own
    quadrature and root finding; rounded to single precision it must equal
    the oracle's independently computed table value for value."""
    import paper_2310_00317_amd as P
    from oracle import photons
    lib_t = P.photon_table()
    orc_t = photons.table()
    assert lib_t.shape == orc_t.shape == (P.PHOTON_TABLE_NODES,)
    bad = np.nonzero(lib_t != orc_t)[0]
    assert bad.size == 0, (bad[:5], lib_t[bad[:5]], orc_t[bad[:5]])
    with pytest.raises(P.XtmError):
        P.check(P.lib().xtm_photon_table(None, P.PHOTON_TABLE_NODES), "xtm_photon_table")


def test_normal_form_and_matched_gaussian_host_functions_match_oracle(oracle_mod):
    """The library's eigen-analysis (Hessenberg + shifted QR, null vectors by
    full pivoting) against LAPACK's on the oracle's one-turn maps, and its
    matched-ensemble arithmetic against the oracle's."""
    import paper_2310_00317_amd as P
    eref = I.ELECTRON_45GEV6
    cases = ((I.cfg1_lattice(), I.PROTON_450GEV, 0),
             (I.cfg5_lattice(100, n_rf=4, apertures=False, sextupoles=False), eref, 1),
             (I.cfg5_lattice(), eref, 1))
    for el, ref, rad in cases:
        nf = oracle_mod.normal_form_6d(el, ref, radiation=rad)
        got = P.normal_form_of_map(nf["J"])
        d = got.as_dict()
        assert np.max(np.abs(d["q"] - nf["q"])) < 1e-13
        assert np.max(np.abs(d["damping"] - nf["damping"])) < 1e-13
        assert np.max(np.abs(d["lam"] - nf["lam"])) < 1e-13
        assert np.max(np.abs(d["v"] - nf["v"])) < 1e-11 * np.max(np.abs(nf["v"]))
        for k in range(6):
            got.co[k] = nf["co"][k]
        g = np.random.default_rng(7).normal(size=(500, 6))
        a = P.matched_gaussian(got, ref, [2e-9, 5e-10, 1e-6], g)
        b = oracle_mod.matched_gaussian(nf, ref, [2e-9, 5e-10, 1e-6], g)
        assert np.max(np.abs(a - b) / np.std(b, axis=0)) < 1e-10
    with pytest.raises(P.XtmError):
        P.normal_form_of_map(np.diag([2.0, 0.5, 1.0, 1.0, 1.0, 1.0]))   # real eigenvalues
