"""GPU parity with thick quadrupoles and sector bends, which the library
slices at lattice creation and the oracle slices with its own code: the
same sliced line, bitwise-equal tracking, the map back to user elements,
and optics on the sliced ring."""
import sys

import numpy as np
import pytest

from paper_2310_00317_amd import inputs as I
from parity_util import assert_bitwise, gpu_run, oracle_run

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


def test_thick_ring_tracking_bitwise(P, oracle_mod):
    print("[gpu-thick] 16-cell ring of thick quadrupoles and bends, 600 protons, 60 turns",
          flush=True)
    el = I.thick_ring()
    thin = oracle_mod.expand_thick(el)
    c = I.gaussian_particles(600, seed=17, sigmas=np.array([6e-3, 5e-4, 4e-3, 5e-4, 0.1, 1e-3]))
    g, gp, _, lat, _ = gpu_run(P, el, REF, c, 60)
    o, op = oracle_run(oracle_mod, el, REF, c, 60)
    assert lat.n_elements == len(thin)
    assert_bitwise(g, o)
    assert gp == op
    assert (o.state == 0).sum() > 20 and (o.state == 1).sum() > 20
    # the map back to user elements: slices of element k report k
    ui = lat.user_index()
    counts = [1 + 2 * int(e["p"][2]) if e["type"] in (I.QUADRUPOLE, I.SBEND) else 1 for e in el]
    assert np.array_equal(ui, np.repeat(np.arange(len(el)), counts))
    lost = o.state == 0
    assert np.isin(el["type"][ui[o.at_element[lost]]], (I.AP_CIRCLE, I.AP_ELLIPSE)).all()


def test_thick_ring_optics(P, oracle_mod):
    el = I.thick_ring()
    g = P.twiss(P.Lattice(el, REF))
    o = oracle_mod.twiss(el, REF, h=1e-9, hd=1e-8)
    for c in ("betx", "bety", "alfx", "alfy", "mux", "muy", "dx", "dpx"):
        scale = np.max(np.abs(o[c]))
        assert np.max(np.abs(g[c] - o[c])) <= 1e-9 * scale + 1e-12, c
    assert abs(g["qx"] - o["qx"]) < 1e-10 and abs(g["qy"] - o["qy"]) < 1e-10
    assert np.max(o["dx"]) > 0.5  # the bends give dispersion


def test_bad_thick_elements(P):
    for bad in (I.quadrupole(0.0, 0.1), I.quadrupole(1.0, 0.1, slices=0), I.sbend(1.0, 0.1, slices=2.5)):
        with pytest.raises(P.XtmError, match="element 1"):
            P.Lattice(I.line([I.marker(), bad]), REF)


def test_refine_on_sliced_line(P, oracle_mod):
    import torch
    el = I.thick_ring()
    c = I.gaussian_particles(600, seed=17, sigmas=np.array([6e-3, 5e-4, 4e-3, 5e-4, 0.1, 1e-3]))
    g, _, _, lat, parts = gpu_run(P, el, REF, c, 30)
    o, _ = oracle_run(oracle_mod, el, REF, c, 30)
    assert_bitwise(g, o)
    s, x, y = P.refine_losses(lat, parts, 64, 0.01, 30)
    torch.cuda.synchronize()
    so, xo, yo = oracle_mod.refine_losses(el, REF, o, 64, 0.01, 30)
    assert_bitwise({"s": s.cpu().numpy(), "x": x.cpu().numpy(), "y": y.cpu().numpy()},
                   {"s": so, "x": xo, "y": yo}, fields=("s", "x", "y"))
    assert (o.state == 0).sum() > 20
