"""MI355X (gfx950) FP64 thin-lattice particle tracker.

Thin Python binding over the C ABI of ``libxtm.so`` (declared in
``include/xtm.h``).  It only marshals arguments: device memory comes from
torch tensors on the ROCm device, every computation runs in the library's
HIP kernels.  Importing the package does not load the library; the first
call that needs it does, and raises if it was not built.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

from . import inputs  # noqa: F401  (seeded input generators)

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libxtm.so")

XTM_OK = 0
STATUS_NAMES = {0: "XTM_OK", -1: "XTM_E_ARG", -2: "XTM_E_ELEMENT", -3: "XTM_E_HIP",
                -4: "XTM_E_NOMEM", -5: "XTM_E_REFERENCE", -6: "XTM_E_UNSUPPORTED",
                -7: "XTM_E_STATE"}

FLOAT_FIELDS = ("x", "px", "y", "py", "zeta", "delta", "ptau", "rpp", "rvv")
INT_FIELDS = ("state", "at_element", "at_turn")


class XtmError(RuntimeError):
    def __init__(self, code: int, where: str, msg: str):
        super().__init__(f"{where}: {STATUS_NAMES.get(code, code)}: {msg}")
        self.code = code


class _TwissSummary(ctypes.Structure):
    _fields_ = [("qx", ctypes.c_double), ("qy", ctypes.c_double), ("co", ctypes.c_double * 4),
                ("iterations", ctypes.c_int32), ("pad", ctypes.c_int32),
                ("residual", ctypes.c_double)]


TWISS_COLUMNS = ("s", "x", "px", "y", "py", "betx", "alfx", "mux", "bety", "alfy", "muy",
                 "dx", "dpx", "dy", "dpy")


class _Reference(ctypes.Structure):
    _fields_ = [("mass0_eV", ctypes.c_double), ("charge0", ctypes.c_double),
                ("p0c_eV", ctypes.c_double)]


class _Arrays(ctypes.Structure):
    _fields_ = [(f, ctypes.c_void_p) for f in FLOAT_FIELDS + INT_FIELDS + ("particle_id",)] + \
        [("n", ctypes.c_int64)]


class TrackOpts(ctypes.Structure):
    _fields_ = [("turns_per_chunk", ctypes.c_int32), ("block", ctypes.c_int32),
                ("no_compact", ctypes.c_int32), ("use_graph", ctypes.c_int32),
                ("time_kernels", ctypes.c_int32), ("variant", ctypes.c_int32),
                ("radiation", ctypes.c_int32), ("record_turns", ctypes.c_int32),
                ("rng_seed", ctypes.c_uint64), ("record_buf", ctypes.c_void_p),
                ("compact_every", ctypes.c_int32), ("pad", ctypes.c_int32)]


class TrackStats(ctypes.Structure):
    _fields_ = [("passes", ctypes.c_int64), ("alive", ctypes.c_int64),
                ("launches", ctypes.c_int32), ("variant", ctypes.c_int32),
                ("kernel_ms", ctypes.c_double)]


class NormalForm6(ctypes.Structure):
    _fields_ = [("co", ctypes.c_double * 6), ("J", ctypes.c_double * 36),
                ("lam_re", ctypes.c_double * 3), ("lam_im", ctypes.c_double * 3),
                ("q", ctypes.c_double * 3), ("damping", ctypes.c_double * 3),
                ("v_re", ctypes.c_double * 18), ("v_im", ctypes.c_double * 18),
                ("iterations", ctypes.c_int32), ("pad", ctypes.c_int32),
                ("residual", ctypes.c_double)]

    def as_dict(self) -> dict:
        v = np.array(self.v_re[:]) + 1j * np.array(self.v_im[:])
        return {"co": np.array(self.co[:]), "J": np.array(self.J[:]).reshape(6, 6),
                "lam": np.array(self.lam_re[:]) + 1j * np.array(self.lam_im[:]),
                "q": np.array(self.q[:]), "damping": np.array(self.damping[:]),
                "v": v.reshape(3, 6), "iterations": int(self.iterations),
                "residual": float(self.residual)}


class Plan(ctypes.Structure):
    _fields_ = [("variant", ctypes.c_int32), ("block", ctypes.c_int32),
                ("passes_per_s", ctypes.c_double), ("turns_per_chunk", ctypes.c_int32),
                ("compact_every", ctypes.c_int32)]


_lib = None


def lib() -> ctypes.CDLL:
    """Load libxtm.so (built by ``paper_2310_00317_amd.build``); no fallback."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_2310_00317_amd.build` (there is no CPU fallback)")
        L = ctypes.CDLL(LIB_PATH)
        vp, i32, i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
        sig = {
            "xtm_last_error": ([], ctypes.c_char_p),
            "xtm_version": ([], ctypes.c_char_p),
            "xtm_max_variant": ([], ctypes.c_int32),
            "xtm_lattice_create": ([vp, i32, vp, vp], i32),
            "xtm_lattice_destroy": ([vp], i32),
            "xtm_lattice_info": ([vp, vp, vp], i32),
            "xtm_lattice_user_index": ([vp, vp], i32),
            "xtm_particles_bind": ([vp, vp, vp], i32),
            "xtm_particles_release": ([vp], i32),
            "xtm_particles_init": ([vp, vp, i64, i32, vp], i32),
            "xtm_particles_reset": ([vp, i32, vp], i32),
            "xtm_particles_turn": ([vp, vp], i32),
            "xtm_track": ([vp, vp, i32, vp, vp, vp], i32),
            "xtm_track_backward": ([vp, vp, i32, vp, vp], i32),
            "xtm_track_per_element": ([vp, vp, i32, vp, vp], i32),
            "xtm_refine_losses": ([vp, vp, i32, ctypes.c_double, i32, vp, vp, vp, vp, vp], i32),
            "xtm_track_record": ([vp, vp, i64, vp, vp], i32),
            "xtm_twiss_open": ([vp, ctypes.c_double, ctypes.c_double, ctypes.c_double, vp, vp,
                                vp], i32),
            "xtm_twiss_coupled": ([vp, ctypes.c_double, ctypes.c_double, ctypes.c_double, i32,
                                   ctypes.c_double, vp, vp, vp], i32),
            "xtm_chromaticity": ([vp, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                  ctypes.c_double, i32, ctypes.c_double, vp, vp], i32),
            "xtm_twiss": ([vp, ctypes.c_double, ctypes.c_double, ctypes.c_double, i32,
                           ctypes.c_double, vp, vp, vp, vp], i32),
            "xtm_get_losses": ([vp, vp, vp, vp, vp], i32),
            "xtm_sync": ([vp], i32),
            "xtm_philox4x32_10": ([ctypes.c_uint64, vp, i64, vp, vp], i32),
            "xtm_batch_create": ([vp, i32, vp], i32),
            "xtm_batch_destroy": ([vp], i32),
            "xtm_track_batched": ([vp, vp, vp, i32, vp, vp, vp], i32),
            "xtm_autotune": ([vp, vp, vp, vp, i32, i32, vp, vp], i32),
            "xtm_features": ([vp, i64, vp, ctypes.c_double, ctypes.c_double, vp, vp], i32),
            "xtm_feature_stats": ([vp, vp, i64, vp, vp], i32),
            "xtm_mlp_init": ([vp, ctypes.c_uint64, vp], i32),
            "xtm_mlp_forward": ([vp, vp, vp, i64, vp, vp], i32),
            "xtm_mlp_workspace": ([i64, vp], i32),
            "xtm_mlp_grad": ([vp, vp, vp, vp, i64, ctypes.c_float, vp, vp, vp, vp], i32),
            "xtm_mlp_grad_noalloc": ([vp, vp, vp, vp, i64, ctypes.c_float, vp, vp, vp], i32),
            "xtm_mlp_adam": ([vp, vp, vp, vp, i32, ctypes.c_float, vp], i32),
            "xtm_mlp_train": ([vp, vp, vp, vp, vp, vp, i64, ctypes.c_float, i32, i32,
                               ctypes.c_float, ctypes.c_uint64, vp, vp, vp], i32),
            "xtm_select_threshold": ([vp, vp, i64, ctypes.c_double, vp, vp, vp, vp], i32),
            "xtm_dynamic_aperture": ([vp, vp, i32, i32, vp], i32),
            "xtm_retire": ([vp, vp, ctypes.c_float, ctypes.c_uint64, ctypes.c_double, vp, vp, vp,
                            vp], i32),
            "xtm_rule_score": ([vp, i64, vp, vp], i32),
            "xtm_photon_table": ([vp, i32], i32),
            "xtm_twiss6d": ([vp, i32, vp, i32, ctypes.c_double, vp, vp], i32),
            "xtm_normal_form_of_map": ([vp, vp], i32),
            "xtm_matched_gaussian": ([vp, vp, vp, vp, i64, vp], i32),
            "xtm_audit_upper_bound": ([i64, i64, vp], i32),
            "xtm_audit_verdict": ([vp, vp, ctypes.c_double, vp, vp, vp, vp, vp], i32),
            "xtm_resume_retired": ([vp, vp, vp, vp, vp], i32),
        }
        for name, (args, res) in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = res
        _lib = L
    return _lib


def check(code: int, where: str) -> None:
    if code != XTM_OK:
        raise XtmError(code, where, lib().xtm_last_error().decode())


def _ref_struct(ref) -> _Reference:
    return _Reference(float(ref.mass0_eV), float(ref.charge0), float(ref.p0c_eV))


def _stream(stream=None):
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


class Lattice:
    """Library-owned element table built from 248-byte element records."""

    def __init__(self, elements: np.ndarray, ref):
        el = np.ascontiguousarray(elements)
        if el.dtype.itemsize != inputs.ELEMENT_DTYPE.itemsize:
            raise ValueError("elements must use inputs.ELEMENT_DTYPE")
        self.ref = ref
        self._el = el
        r = _ref_struct(ref)
        h = ctypes.c_void_p()
        check(lib().xtm_lattice_create(el.ctypes.data_as(ctypes.c_void_p), len(el),
                                       ctypes.byref(r), ctypes.byref(h)), "xtm_lattice_create")
        self._h = h
        n = ctypes.c_int32()
        b = ctypes.c_int64()
        check(lib().xtm_lattice_info(self._h, ctypes.byref(n), ctypes.byref(b)), "xtm_lattice_info")
        # elements of the line the library tracks (thick elements sliced)
        self.n_elements = int(n.value)

    def user_index(self) -> np.ndarray:
        """User element of each element of the sliced line."""
        out = np.zeros(max(self.n_elements, 1), dtype=np.int32)
        check(lib().xtm_lattice_user_index(self._h, out.ctypes.data_as(ctypes.c_void_p)),
              "xtm_lattice_user_index")
        return out[: self.n_elements]

    @property
    def handle(self):
        return self._h

    def table_bytes(self) -> int:
        n = ctypes.c_int32()
        b = ctypes.c_int64()
        check(lib().xtm_lattice_info(self._h, ctypes.byref(n), ctypes.byref(b)), "xtm_lattice_info")
        return int(b.value)

    def close(self):
        if getattr(self, "_h", None):
            lib().xtm_lattice_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Particles:
    """Caller-owned SoA particle arrays (torch tensors on the GPU) bound as a set."""

    def __init__(self, n: int, ref, device="cuda"):
        import torch
        self.n = int(n)
        self.ref = ref
        self.device = torch.device(device)
        m = max(self.n, 1)
        for f in FLOAT_FIELDS:
            setattr(self, f, torch.zeros(m, dtype=torch.float64, device=self.device))
        for f in INT_FIELDS:
            setattr(self, f, torch.zeros(m, dtype=torch.int32, device=self.device))
        self.particle_id = torch.zeros(m, dtype=torch.int64, device=self.device)
        a = _Arrays()
        for f in FLOAT_FIELDS + INT_FIELDS + ("particle_id",):
            setattr(a, f, getattr(self, f).data_ptr())
        a.n = self.n
        r = _ref_struct(ref)
        h = ctypes.c_void_p()
        check(lib().xtm_particles_bind(ctypes.byref(a), ctypes.byref(r), ctypes.byref(h)),
              "xtm_particles_bind")
        self._h = h

    @property
    def handle(self):
        return self._h

    def init(self, coords, first_id: int = 0, stream=None):
        """Set coordinates from an (n, 6) array (numpy: host; torch cuda tensor: device)."""
        import torch
        if isinstance(coords, torch.Tensor):
            c = coords.to(dtype=torch.float64).contiguous()
            if c.shape != (self.n, 6):
                raise ValueError("coords must have shape (n, 6)")
            on_dev = 1 if c.is_cuda else 0
            ptr = ctypes.c_void_p(c.data_ptr())
            keep = c
        else:
            keep = np.ascontiguousarray(coords, dtype=np.float64).reshape(-1, 6)
            if keep.shape[0] != self.n:
                raise ValueError("coords must have shape (n, 6)")
            on_dev = 0
            ptr = keep.ctypes.data_as(ctypes.c_void_p)
        check(lib().xtm_particles_init(self._h, ptr, int(first_id), on_dev, _stream(stream)),
              "xtm_particles_init")
        if on_dev:
            torch.cuda.current_stream().synchronize()
        del keep
        return self

    def reset(self, turn: int, stream=None):
        check(lib().xtm_particles_reset(self._h, int(turn), _stream(stream)), "xtm_particles_reset")

    @property
    def turn(self) -> int:
        t = ctypes.c_int32()
        check(lib().xtm_particles_turn(self._h, ctypes.byref(t)), "xtm_particles_turn")
        return int(t.value)

    def to_numpy(self) -> dict:
        import torch
        torch.cuda.synchronize()
        out = {}
        for f in FLOAT_FIELDS + INT_FIELDS + ("particle_id",):
            out[f] = getattr(self, f)[: self.n].cpu().numpy()
        return out

    def losses(self, stream=None):
        st = np.zeros(max(self.n, 1), dtype=np.int32)
        at = np.zeros_like(st)
        ae = np.zeros_like(st)
        check(lib().xtm_get_losses(self._h, st.ctypes.data_as(ctypes.c_void_p),
                                   at.ctypes.data_as(ctypes.c_void_p),
                                   ae.ctypes.data_as(ctypes.c_void_p), _stream(stream)),
              "xtm_get_losses")
        return st[: self.n], at[: self.n], ae[: self.n]

    def close(self):
        if getattr(self, "_h", None):
            lib().xtm_particles_release(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def line_variants() -> list:
    """Kernel numbers of the per-line kernel's forms (5 .. xtm_max_variant())."""
    return list(range(5, int(lib().xtm_max_variant()) + 1))


def track(lattice: Lattice, particles: Particles, n_turns: int, turns_per_chunk: int = 0,
          block: int = 0, compact: bool = True, graph: bool = False, stats: bool = True,
          time_kernels: bool = False, variant: int = 0, radiation: int = 0, seed: int = 0,
          stream=None, full_stats: bool = False, record=None, compact_every: int = 0):
    """Track ``n_turns`` forward.  With ``stats`` (synchronising) returns
    (passes, alive), or the whole TrackStats if ``full_stats``.  ``record``:
    a float32 cuda tensor [T, 4, n] that receives (x, px, y, py) at the start
    of absolute turns < T."""
    o = _opts(turns_per_chunk, block, compact, graph, time_kernels, variant, radiation, seed,
              record, particles.n, compact_every)
    s = TrackStats()
    check(lib().xtm_track(lattice.handle, particles.handle, int(n_turns), ctypes.byref(o),
                          _stream(stream), ctypes.byref(s) if (stats or full_stats) else None),
          "xtm_track")
    if full_stats:
        return s
    return (int(s.passes), int(s.alive)) if stats else None


class Batch:
    """Lattice variants tracked together; keeps the lattices alive."""

    def __init__(self, lattices):
        self.lattices = list(lattices)
        arr = (ctypes.c_void_p * len(self.lattices))(*[l.handle.value for l in self.lattices])
        h = ctypes.c_void_p()
        check(lib().xtm_batch_create(arr, len(self.lattices), ctypes.byref(h)), "xtm_batch_create")
        self._h = h

    @property
    def handle(self):
        return self._h

    def close(self):
        if getattr(self, "_h", None):
            lib().xtm_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _opts(turns_per_chunk=0, block=0, compact=True, graph=False, time_kernels=False, variant=0,
          radiation=0, seed=0, record=None, n=0, compact_every=0):
    rec_turns, rec_ptr = 0, None
    if record is not None:
        if tuple(record.shape[1:]) != (4, n) or not record.is_contiguous():
            raise ValueError("record must be a contiguous [T, 4, n] tensor")
        rec_turns, rec_ptr = int(record.shape[0]), record.data_ptr()
    return TrackOpts(int(turns_per_chunk), int(block), 0 if compact else 1, 1 if graph else 0,
                     1 if time_kernels else 0, int(variant), int(radiation), rec_turns, int(seed),
                     rec_ptr, int(compact_every), 0)


def track_batched(batch: Batch, particles: Particles, first_slot, n_turns: int,
                  stream=None, full_stats: bool = False, **kw):
    """Track all variants n_turns; variant v owns slots first_slot[v]..first_slot[v+1]-1."""
    fs = np.ascontiguousarray(first_slot, dtype=np.int64)
    o = _opts(n=particles.n, **kw)
    s = TrackStats()
    check(lib().xtm_track_batched(batch.handle, particles.handle,
                                  fs.ctypes.data_as(ctypes.c_void_p), int(n_turns),
                                  ctypes.byref(o), _stream(stream), ctypes.byref(s)),
          "xtm_track_batched")
    return s if full_stats else (int(s.passes), int(s.alive))


def autotune(particles: Particles, lattice: Lattice = None, batch: Batch = None, first_slot=None,
             probe_turns: int = 2, warm_turns: int = 0, stream=None) -> Plan:
    fs = None if first_slot is None else np.ascontiguousarray(first_slot, dtype=np.int64)
    plan = Plan()
    check(lib().xtm_autotune(None if lattice is None else lattice.handle,
                             None if batch is None else batch.handle, particles.handle,
                             None if fs is None else fs.ctypes.data_as(ctypes.c_void_p),
                             int(probe_turns), int(warm_turns), _stream(stream),
                             ctypes.byref(plan)),
          "xtm_autotune")
    return plan


def track_per_element(lattice: Lattice, particles: Particles, n_turns: int, stream=None):
    """Measurement baseline: one kernel launch per element and turn, state
    through HBM each time (same results as track).  Returns TrackStats."""
    s = TrackStats()
    check(lib().xtm_track_per_element(lattice.handle, particles.handle, int(n_turns),
                                      _stream(stream), ctypes.byref(s)), "xtm_track_per_element")
    return s


def refine_losses(lattice: Lattice, particles: Particles, n_vertices: int = 64, ds: float = 0.01,
                  n_bisect: int = 30, stream=None, with_tests: bool = False):
    """Loss locations of the particles lost on an aperture (backtracking
    against a polygon-interpolated aperture; xtm_refine_losses): device
    tensors (s, x, y) of the set's length, NaN for particles not lost on an
    aperture; with_tests adds the int32 tensor of polygon tests per particle."""
    import torch
    m = max(particles.n, 1)
    out = [torch.empty(m, dtype=torch.float64, device=particles.device) for _ in range(3)]
    tests = torch.empty(m, dtype=torch.int32, device=particles.device) if with_tests else None
    check(lib().xtm_refine_losses(lattice.handle, particles.handle, int(n_vertices), float(ds),
                                  int(n_bisect), *[ctypes.c_void_p(t.data_ptr()) for t in out],
                                  ctypes.c_void_p(tests.data_ptr() if with_tests else 0),
                                  _stream(stream)), "xtm_refine_losses")
    res = tuple(t[:particles.n] for t in out)
    return res + (tests[:particles.n],) if with_tests else res


def track_record(lattice: Lattice, coords, stream=None):
    """One turn of the (n, 6) coordinates (x, px, y, py, zeta, delta) with the
    coordinates recorded at every element entry and after the last
    (xtm_track_record): device tensor (n_el + 1, n, 6)."""
    import torch
    c = torch.as_tensor(np.asarray(coords, dtype=np.float64) if not isinstance(coords, torch.Tensor)
                        else coords, dtype=torch.float64).to("cuda").contiguous()
    n = c.shape[0]
    out = torch.empty((lattice.n_elements + 1, max(n, 1), 6), dtype=torch.float64, device="cuda")
    check(lib().xtm_track_record(lattice.handle, ctypes.c_void_p(c.data_ptr()), int(n),
                                 ctypes.c_void_p(out.data_ptr()), _stream(stream)),
          "xtm_track_record")
    return out[:, :n]


def twiss(lattice: Lattice, delta0: float = 0.0, h: float = 1e-9, hd: float = 1e-8,
          max_iter: int = 30, tol: float = 1e-15, guess=None, stream=None) -> dict:
    """Uncoupled linear optics by tracking (xtm_twiss): per-element columns
    (TWISS_COLUMNS, numpy arrays of n_el + 1) plus qx, qy, the closed orbit at
    the start (co), the Newton steps made and the last residual."""
    n = lattice.n_elements
    table = np.zeros((n + 1, len(TWISS_COLUMNS)), dtype=np.float64)
    summ = _TwissSummary()
    g = None if guess is None else np.ascontiguousarray(guess, dtype=np.float64)
    check(lib().xtm_twiss(lattice.handle, float(delta0), float(h), float(hd), int(max_iter),
                          float(tol), None if g is None else g.ctypes.data_as(ctypes.c_void_p),
                          table.ctypes.data_as(ctypes.c_void_p), ctypes.byref(summ),
                          _stream(stream)), "xtm_twiss")
    out = {c: table[:, k].copy() for k, c in enumerate(TWISS_COLUMNS)}
    out.update(qx=summ.qx, qy=summ.qy, co=np.array(summ.co[:]), iterations=summ.iterations,
               residual=summ.residual)
    return out


def twiss_open(lattice: Lattice, init, delta0: float = 0.0, h: float = 1e-9, hd: float = 1e-8,
               stream=None) -> dict:
    """Optics of a line from given initial conditions (xtm_twiss_open): init =
    (x, px, y, py, betx, alfx, bety, alfy, dx, dpx, dy, dpy); the per-element
    columns of TWISS_COLUMNS."""
    n = lattice.n_elements
    table = np.zeros((n + 1, len(TWISS_COLUMNS)), dtype=np.float64)
    iv = np.ascontiguousarray(init, dtype=np.float64)
    if iv.shape != (12,):
        raise ValueError("init must hold 12 values")
    check(lib().xtm_twiss_open(lattice.handle, float(delta0), float(h), float(hd),
                               iv.ctypes.data_as(ctypes.c_void_p),
                               table.ctypes.data_as(ctypes.c_void_p), _stream(stream)),
          "xtm_twiss_open")
    return {c: table[:, k].copy() for k, c in enumerate(TWISS_COLUMNS)}


COUPLED_COLUMNS = ("s", "betx1", "bety1", "betx2", "bety2", "mu1", "mu2")


def twiss_coupled(lattice: Lattice, delta0: float = 0.0, h: float = 1e-9, hd: float = 1e-8,
                  max_iter: int = 30, tol: float = 1e-15, stream=None) -> dict:
    """Transverse optics with linear coupling (xtm_twiss_coupled): per-element
    mode betas and phases (COUPLED_COLUMNS) and the eigen-tunes q1, q2."""
    n = lattice.n_elements
    table = np.zeros((n + 1, len(COUPLED_COLUMNS)), dtype=np.float64)
    q = np.zeros(2, dtype=np.float64)
    check(lib().xtm_twiss_coupled(lattice.handle, float(delta0), float(h), float(hd), int(max_iter),
                                  float(tol), table.ctypes.data_as(ctypes.c_void_p),
                                  q.ctypes.data_as(ctypes.c_void_p), _stream(stream)),
          "xtm_twiss_coupled")
    out = {c: table[:, k].copy() for k, c in enumerate(COUPLED_COLUMNS)}
    out.update(q1=float(q[0]), q2=float(q[1]))
    return out


def chromaticity(lattice: Lattice, delta0: float = 0.0, eps: float = 1e-6, h: float = 1e-9,
                 hd: float = 1e-8, max_iter: int = 30, tol: float = 1e-15, stream=None):
    """(dQx/d delta, dQy/d delta) by central differences of the tracked tunes
    (xtm_chromaticity)."""
    out = np.zeros(2, dtype=np.float64)
    check(lib().xtm_chromaticity(lattice.handle, float(delta0), float(eps), float(h), float(hd),
                                 int(max_iter), float(tol), out.ctypes.data_as(ctypes.c_void_p),
                                 _stream(stream)), "xtm_chromaticity")
    return float(out[0]), float(out[1])


def track_backward(lattice: Lattice, particles: Particles, n_turns: int, stats: bool = True,
                   stream=None):
    s = TrackStats()
    check(lib().xtm_track_backward(lattice.handle, particles.handle, int(n_turns), _stream(stream),
                                   ctypes.byref(s) if stats else None), "xtm_track_backward")
    return (int(s.passes), int(s.alive)) if stats else None


def sync(stream=None):
    check(lib().xtm_sync(_stream(stream)), "xtm_sync")


def philox(seed: int, ctr0, n_blocks: int, stream=None):
    """Raw Philox4x32-10 words (torch uint32-as-int32 tensor of 4 n_blocks) on the GPU."""
    import torch
    out = torch.empty(max(4 * int(n_blocks), 1), dtype=torch.int32, device="cuda")
    c = (ctypes.c_uint32 * 4)(*[int(v) & 0xFFFFFFFF for v in ctr0])
    check(lib().xtm_philox4x32_10(int(seed), c, int(n_blocks), ctypes.c_void_p(out.data_ptr()),
                                  _stream(stream)), "xtm_philox4x32_10")
    return out[: 4 * int(n_blocks)]


# ------------------------------------------------------------ learned early stop
MLP_PARAMS = 18817
N_FEATURES = 16
RECORD_TURNS = 1024


def _p(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def features(record, twiss4, emit: float, r_aperture: float, stream=None):
    """16 FP32 features per particle from a [1024, 4, n] float32 record."""
    import torch
    n = int(record.shape[2])
    out = torch.empty((max(n, 1), N_FEATURES), dtype=torch.float32, device=record.device)
    tw = (ctypes.c_double * 4)(*[float(v) for v in twiss4])
    check(lib().xtm_features(_p(record), n, tw, float(emit), float(r_aperture), _p(out),
                             _stream(stream)), "xtm_features")
    return out[:n]


def feature_stats(feat, mask=None, stream=None):
    """[32] float32: column means then inverse standard deviations."""
    import torch
    norm = torch.empty(32, dtype=torch.float32, device=feat.device)
    check(lib().xtm_feature_stats(_p(feat), _p(mask), int(feat.shape[0]), _p(norm),
                                  _stream(stream)), "xtm_feature_stats")
    return norm


def mlp_init(seed: int, device="cuda", stream=None):
    import torch
    theta = torch.empty(MLP_PARAMS, dtype=torch.float32, device=device)
    check(lib().xtm_mlp_init(_p(theta), int(seed), _stream(stream)), "xtm_mlp_init")
    return theta


def mlp_forward(theta, norm, x, stream=None):
    import torch
    B = int(x.shape[0])
    out = torch.empty(max(B, 1), dtype=torch.float32, device=x.device)
    check(lib().xtm_mlp_forward(_p(theta), _p(norm), _p(x), B, _p(out), _stream(stream)),
          "xtm_mlp_forward")
    return out[:B]


def mlp_workspace(B: int) -> int:
    n = ctypes.c_int64()
    check(lib().xtm_mlp_workspace(int(B), ctypes.byref(n)), "xtm_mlp_workspace")
    return int(n.value)


def mlp_grad(theta, norm, x, y, pos_weight: float, work=None, stream=None):
    """(grad [MLP_PARAMS], loss [1]) float32 tensors."""
    import torch
    B = int(x.shape[0])
    if work is None:
        work = torch.empty(mlp_workspace(B), dtype=torch.float32, device=x.device)
    grad = torch.empty(MLP_PARAMS, dtype=torch.float32, device=x.device)
    loss = torch.empty(1, dtype=torch.float32, device=x.device)
    check(lib().xtm_mlp_grad(_p(theta), _p(norm), _p(x), _p(y), B, float(pos_weight), _p(grad),
                             _p(loss), _p(work), _stream(stream)), "xtm_mlp_grad")
    return grad, loss


MLP_NOALLOC_MAX_BATCH = 4096


def mlp_grad_noalloc(theta, norm, x, y, pos_weight: float, grad, loss=None, stream=None):
    """xtm_mlp_grad_noalloc into caller tensors grad [MLP_PARAMS] and loss
    [1] (or None): the library's fixed workspace, no device allocation."""
    check(lib().xtm_mlp_grad_noalloc(_p(theta), _p(norm), _p(x), _p(y), int(x.shape[0]),
                                     float(pos_weight), _p(grad),
                                     _p(loss), _stream(stream)),
          "xtm_mlp_grad_noalloc")


def mlp_adam(theta, m, v, grad, step: int, lr: float, stream=None):
    check(lib().xtm_mlp_adam(_p(theta), _p(m), _p(v), _p(grad), int(step), float(lr),
                             _stream(stream)), "xtm_mlp_adam")


def retire(particles: Particles, logit, threshold: float, audit_seed: int,
           audit_fraction: float = 0.05, audit_flags=None, stream=None):
    """Retire alive particles with logit >= threshold outside the audit set;
    the audited ones are flagged in audit_flags (int32 tensor, one per slot)
    when given; returns (retired, audited)."""
    r = ctypes.c_int64()
    a = ctypes.c_int64()
    check(lib().xtm_retire(particles.handle, _p(logit), float(threshold), int(audit_seed),
                           float(audit_fraction), _p(audit_flags), ctypes.byref(r),
                           ctypes.byref(a), _stream(stream)), "xtm_retire")
    return int(r.value), int(a.value)


def rule_score(feat, stream=None):
    """-max(f8, f9) per row of a [n, 16] float32 feature tensor (xtm_rule_score)."""
    import torch
    n = int(feat.shape[0])
    out = torch.empty(max(n, 1), dtype=torch.float32, device=feat.device)
    check(lib().xtm_rule_score(_p(feat), n, _p(out), _stream(stream)), "xtm_rule_score")
    return out[:n]


def twiss6d(lattice: Lattice, radiation: int = 0, h=None, max_iter: int = 20,
            tol: float = 1e-15, stream=None) -> NormalForm6:
    """6D linear normal form by tracking (xtm_twiss6d)."""
    out = NormalForm6()
    hh = None if h is None else np.ascontiguousarray(h, dtype=np.float64)
    check(lib().xtm_twiss6d(lattice.handle, int(radiation),
                            None if hh is None else hh.ctypes.data_as(ctypes.c_void_p),
                            int(max_iter), float(tol), ctypes.byref(out), _stream(stream)),
          "xtm_twiss6d")
    return out


def normal_form_of_map(J) -> NormalForm6:
    out = NormalForm6()
    Jc = np.ascontiguousarray(J, dtype=np.float64).reshape(36)
    check(lib().xtm_normal_form_of_map(Jc.ctypes.data_as(ctypes.c_void_p), ctypes.byref(out)),
          "xtm_normal_form_of_map")
    return out


def matched_gaussian(nf: NormalForm6, ref, eps, gauss) -> np.ndarray:
    """(n, 6) coordinates (x, px, y, py, zeta, delta) matched to the normal
    form with mode emittances eps[3], from standard normals gauss (n, 6)."""
    g = np.ascontiguousarray(gauss, dtype=np.float64).reshape(-1, 6)
    e = np.ascontiguousarray(eps, dtype=np.float64)
    out = np.zeros_like(g)
    r = _ref_struct(ref)
    check(lib().xtm_matched_gaussian(ctypes.byref(nf), ctypes.byref(r),
                                     e.ctypes.data_as(ctypes.c_void_p),
                                     g.ctypes.data_as(ctypes.c_void_p), len(g),
                                     out.ctypes.data_as(ctypes.c_void_p)),
          "xtm_matched_gaussian")
    return out


PHOTON_TABLE_NODES = 2433


def photon_table() -> np.ndarray:
    """The library's inverse photon spectrum (xtm_photon_table), host copy."""
    out = np.zeros(PHOTON_TABLE_NODES, dtype=np.float64)
    check(lib().xtm_photon_table(out.ctypes.data_as(ctypes.c_void_p), PHOTON_TABLE_NODES),
          "xtm_photon_table")
    return out


def audit_upper_bound(n_lost: int, n_audited: int) -> float:
    out = ctypes.c_double()
    check(lib().xtm_audit_upper_bound(int(n_lost), int(n_audited), ctypes.byref(out)),
          "xtm_audit_upper_bound")
    return float(out.value)


def audit_verdict(particles: Particles, audit_flags, fallback_rate: float, stream=None) -> dict:
    """xtm_audit_verdict: {audited, lost, upper, fallback}."""
    a, l, f = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int32()
    u = ctypes.c_double()
    check(lib().xtm_audit_verdict(particles.handle, _p(audit_flags), float(fallback_rate),
                                  ctypes.byref(a), ctypes.byref(l), ctypes.byref(u),
                                  ctypes.byref(f), _stream(stream)), "xtm_audit_verdict")
    return {"audited": int(a.value), "lost": int(l.value), "upper": float(u.value),
            "fallback": bool(f.value)}


def resume_retired(lattice: Lattice, particles: Particles, variant: int = 0, stream=None):
    """xtm_resume_retired: the full-tracking fallback; returns (passes, alive)."""
    o = TrackOpts()
    o.variant = int(variant)
    st = TrackStats()
    check(lib().xtm_resume_retired(lattice.handle, particles.handle, ctypes.byref(o),
                                   _stream(stream), ctypes.byref(st)), "xtm_resume_retired")
    return int(st.passes), int(st.alive)


def mlp_train(theta, m, v, norm, x, y, pos_weight: float, epochs: int, batch: int, lr: float,
              shuffle_seed: int, step: int = 0, stream=None):
    """Run the training loop; returns (new Adam step count, per-epoch mean loss)."""
    st = ctypes.c_int32(int(step))
    losses = np.zeros(max(int(epochs), 1), dtype=np.float32)
    check(lib().xtm_mlp_train(_p(theta), _p(m), _p(v), _p(norm), _p(x), _p(y), int(x.shape[0]),
                              float(pos_weight), int(epochs), int(batch), float(lr),
                              int(shuffle_seed), ctypes.byref(st),
                              losses.ctypes.data_as(ctypes.c_void_p), _stream(stream)),
          "xtm_mlp_train")
    return int(st.value), losses[: int(epochs)]


def select_threshold(logit, label, max_false_rate: float, stream=None):
    """(tau, false rate at tau, rows at or above tau); label int32 (1 = survived)."""
    tau = ctypes.c_float()
    rate = ctypes.c_double()
    sel = ctypes.c_int64()
    check(lib().xtm_select_threshold(_p(logit), _p(label), int(logit.shape[0]),
                                     float(max_false_rate), ctypes.byref(tau), ctypes.byref(rate),
                                     ctypes.byref(sel), _stream(stream)), "xtm_select_threshold")
    return float(tau.value), float(rate.value), int(sel.value)


def dynamic_aperture(state, radius, n_r: int, n_theta: int) -> np.ndarray:
    st = np.ascontiguousarray(state, dtype=np.int32)
    r = np.ascontiguousarray(radius, dtype=np.float64)
    if st.size != n_r * n_theta or r.size != n_r * n_theta:
        raise ValueError("state and radius need n_r * n_theta entries")
    out = np.zeros(n_theta)
    check(lib().xtm_dynamic_aperture(st.ctypes.data_as(ctypes.c_void_p),
                                     r.ctypes.data_as(ctypes.c_void_p), int(n_r), int(n_theta),
                                     out.ctypes.data_as(ctypes.c_void_p)), "xtm_dynamic_aperture")
    return out
