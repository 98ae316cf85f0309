"""Thin ctypes binding of ``libhexsv.so`` (C-ABI in ``include/hexsv.h``).

Argument marshalling only: every step of the time stepper runs in the HIP
library.  PyTorch provides the device memory (tensor ``data_ptr()``) and the
stream (``torch.cuda.current_stream().cuda_stream``).  The binding refuses to
work without the built library: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np
import torch

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "lib", "libhexsv.so")

OK, EINVAL, EDOMAIN, ENOMEM, EHIP, ENUMERIC, ESTATE, EUNSUPPORTED = 0, -1, -2, -3, -4, -5, -6, -7
FP64, FP32 = 0, 1
INTERIOR, WALL, OUTFLOW, PERIODIC, DIRICHLET, FLUX = 0, 1, 2, 3, 4, 5
S, E, N, W = 0, 1, 2, 3
MAX_SEGMENTS = 8


class HexsvError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"hexsv error {code}: {msg}")
        self.code = code


class Segment(C.Structure):
    _fields_ = [("side", C.c_int32), ("lo", C.c_int32), ("hi", C.c_int32), ("code", C.c_int32)]


class GridDesc(C.Structure):
    _fields_ = [("nq", C.c_int32), ("nr", C.c_int32), ("edge", C.c_double),
                ("side_bc", C.c_int32 * 4), ("nseg", C.c_int32),
                ("seg", Segment * MAX_SEGMENTS), ("active", C.POINTER(C.c_uint8)),
                ("mask_bc", C.c_int32)]


class Params(C.Structure):
    _fields_ = [("g", C.c_double), ("cfl", C.c_double), ("dt_max", C.c_double),
                ("h_dry", C.c_double), ("precision", C.c_int32), ("steps_per_graph", C.c_int32),
                ("tile", C.c_int32), ("wg_per_cu", C.c_int32),
                ("ensemble_mode", C.c_int32), ("reserved", C.c_int32)]


class Rain(C.Structure):
    _fields_ = [("kind", C.c_int32), ("i_a", C.c_double), ("t_a", C.c_double), ("T_d", C.c_double)]


class Books(C.Structure):
    _fields_ = [("t", C.c_double), ("initial", C.c_double), ("stored", C.c_double),
                ("rain", C.c_double), ("outflow", C.c_double), ("clamp", C.c_double),
                ("residual", C.c_double), ("steps", C.c_int64), ("dt_min", C.c_double),
                ("dt_max_seen", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


# (name, restype, argtypes)
_VP = C.c_void_p
_SIGS = [
    ("hexsv_version", C.c_char_p, []),
    ("hexsv_last_error", C.c_char_p, []),
    ("hexsv_grid_create", C.c_int, [C.POINTER(GridDesc), C.POINTER(_VP)]),
    ("hexsv_grid_destroy", None, [_VP]),
    ("hexsv_grid_counts", C.c_int, [_VP, C.POINTER(C.c_int64), C.POINTER(C.c_int64)]),
    ("hexsv_grid_tables_device", C.c_int, [_VP, _VP, _VP, _VP, _VP, _VP]),
    ("hexsv_grid_tables", C.c_int, [_VP, _VP, _VP, _VP, _VP]),
    ("hexsv_sim_create", C.c_int, [_VP, C.POINTER(Params), C.POINTER(_VP)]),
    ("hexsv_sim_destroy", None, [_VP]),
    ("hexsv_sim_set_fields", C.c_int, [_VP, _VP, _VP, _VP, _VP, C.c_double, _VP]),
    ("hexsv_sim_set_rain", C.c_int, [_VP, C.POINTER(Rain)]),
    ("hexsv_sim_set_linear_friction", C.c_int, [_VP, C.c_double]),
    ("hexsv_sim_set_viscosity", C.c_int, [_VP, C.c_int32]),
    ("hexsv_sim_set_infiltration", C.c_int, [_VP, C.c_double, C.c_double]),
    ("hexsv_sim_set_state", C.c_int, [_VP, C.c_double, _VP, _VP, _VP, _VP]),
    ("hexsv_sim_run", C.c_int, [_VP, C.c_double, C.c_int64, _VP]),
    ("hexsv_sim_get_state", C.c_int, [_VP, _VP, _VP, _VP, _VP, _VP, _VP]),
    ("hexsv_sim_get_books", C.c_int, [_VP, C.POINTER(Books), _VP]),
    ("hexsv_sim_set_books", C.c_int, [_VP, C.POINTER(Books), _VP]),
    ("hexsv_sim_info", C.c_int, [_VP] + [C.POINTER(C.c_int32)] * 5),
    ("hexsv_sim_timing", C.c_int, [_VP, C.c_int32, C.POINTER(C.c_double), C.POINTER(C.c_int64),
                                   C.POINTER(C.c_int64)]),
    ("hexsv_sim_time_kernel", C.c_int, [_VP, C.c_int32, C.POINTER(C.c_double), _VP]),
    ("hexsv_ensemble_create", C.c_int, [C.c_int32, C.POINTER(_VP), C.POINTER(Params),
                                        C.POINTER(_VP)]),
    ("hexsv_ensemble_destroy", None, [_VP]),
    ("hexsv_ensemble_set_scenario", C.c_int, [_VP, C.c_int32, _VP, _VP, _VP, C.c_double,
                                              C.POINTER(Rain), C.c_double, _VP, _VP, _VP, _VP]),
    ("hexsv_ensemble_run", C.c_int, [_VP, C.POINTER(C.c_double), C.c_int64, _VP]),
    ("hexsv_ensemble_set_viscosity", C.c_int, [_VP, C.c_int32]),
    ("hexsv_ensemble_get_state", C.c_int, [_VP, C.c_int32, _VP, _VP, _VP, _VP, _VP, _VP]),
    ("hexsv_ensemble_get_books", C.c_int, [_VP, C.c_int32, C.POINTER(Books), _VP]),
    ("hexsv_ensemble_timing", C.c_int, [_VP, C.c_int32, C.POINTER(C.c_double),
                                        C.POINTER(C.c_int64), C.POINTER(C.c_int64)]),
    ("hexsv_ensemble_autotune", C.c_int, [_VP, C.c_int32, C.c_char_p, C.POINTER(C.c_int32),
                                          C.POINTER(C.c_double), _VP]),
    ("hexsv_ensemble_info", C.c_int, [_VP, C.POINTER(C.c_int32), C.POINTER(C.c_int32),
                                      C.POINTER(C.c_int64), C.POINTER(C.c_int32),
                                      C.POINTER(C.c_int32)]),
    ("hexsv_sim_autotune", C.c_int, [_VP, C.c_int32, C.c_char_p, C.POINTER(C.c_int32),
                                     C.POINTER(C.c_double), _VP]),
    ("hexsv_surrogate_create", C.c_int, [C.c_int32, C.c_int32, C.c_int32, C.POINTER(_VP)]),
    ("hexsv_surrogate_steps", C.c_int32, [_VP]),
    ("hexsv_surrogate_destroy", None, [_VP]),
    ("hexsv_surrogate_num_params", C.c_int64, [_VP]),
    ("hexsv_surrogate_set_params", C.c_int, [_VP, _VP, C.c_int64, _VP]),
    ("hexsv_surrogate_get_params", C.c_int, [_VP, _VP, C.c_int64, _VP]),
    ("hexsv_surrogate_set_scales", C.c_int, [_VP, C.POINTER(C.c_float), C.c_int32]),
    ("hexsv_surrogate_get_scales", C.c_int, [_VP, C.POINTER(C.c_float), C.c_int32]),
    ("hexsv_surrogate_set_fused", C.c_int, [_VP, C.c_int32]),
    ("hexsv_surrogate_forward", C.c_int, [_VP, _VP, C.c_int32, C.c_int32, C.c_int32, _VP, _VP,
                                          _VP]),
    ("hexsv_surrogate_forward_noalloc", C.c_int, [_VP, _VP, C.c_int32, C.c_int32, C.c_int32,
                                                  _VP, _VP, _VP]),
    ("hexsv_surrogate_gradient", C.c_int, [_VP, _VP, C.c_int32, C.c_int32, C.c_int32, _VP, _VP,
                                           _VP, C.POINTER(C.c_double), _VP]),
    ("hexsv_surrogate_train_step", C.c_int, [_VP, _VP, C.c_int32, C.c_int32, C.c_int32, _VP, _VP,
                                             C.c_float, C.POINTER(C.c_double), _VP]),
    ("hexsv_sim_surrogate_features", C.c_int, [_VP, _VP, C.c_double, C.c_int32, _VP, _VP]),
    ("hexsv_sim_run_surrogate", C.c_int, [_VP, _VP, C.c_double, C.c_double, C.c_int32,
                                          C.c_double, C.c_int32, C.POINTER(C.c_int64),
                                          C.POINTER(C.c_int64), _VP]),
    ("hexsv_sim_surrogate_stats", C.c_int, [_VP, C.POINTER(C.c_int64)]),
    ("hexsv_sim_set_surrogate_backoff", C.c_int, [_VP, C.c_int32]),
    ("hexsv_autotune", C.c_int, [C.c_char_p, C.c_int32, C.c_int32, C.c_int64,
                                 C.POINTER(C.c_int32), C.POINTER(C.c_double), _VP]),
    ("hexsv_tile_count", C.c_int, []),
    ("hexsv_tile_shape", C.c_int, [C.c_int32] + [C.POINTER(C.c_int32)] * 3),
]

_lib = None


def lib():
    """Load libhexsv.so; raise if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "`python -m paper_2406_14933_amd.build` (hipcc, gfx950)")
        L = C.CDLL(LIB_PATH)
        for name, res, args in _SIGS:
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def exported_symbols():
    return [s[0] for s in _SIGS]


def _check(rc):
    if rc != OK:
        raise HexsvError(rc, lib().hexsv_last_error().decode())


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dev(x, dtype=torch.float64, n=None):
    """A contiguous CUDA tensor of dtype (copies host data to the device)."""
    if isinstance(x, np.ndarray) or not torch.is_tensor(x):
        x = torch.from_numpy(np.ascontiguousarray(np.asarray(x), dtype=np.float64 if dtype == torch.float64 else None))
    x = x.to(device="cuda", dtype=dtype).contiguous()
    if n is not None and x.numel() != n:
        raise ValueError(f"expected {n} values, got {x.numel()}")
    return x


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else None


TUNE_STEP, TUNE_ENSEMBLE = 0, 1


def autotune(cache_path, kernel="step", precision="fp32", cells_hint=1 << 20):
    """Tune the step (or batched-ensemble) kernel on the library's own workload of about
    cells_hint cells and record the choice in the JSON cache; returns (tile, ms)."""
    k = {"step": TUNE_STEP, "ensemble": TUNE_ENSEMBLE}[kernel]
    prec = {"fp64": FP64, "fp32": FP32}[precision]
    best, ms = C.c_int32(), C.c_double()
    _check(lib().hexsv_autotune(str(cache_path).encode(), k, prec, int(cells_hint),
                                C.byref(best), C.byref(ms), _stream()))
    return best.value, ms.value


def tile_shapes():
    out = []
    for v in range(lib().hexsv_tile_count()):
        a, b, c = C.c_int32(), C.c_int32(), C.c_int32()
        _check(lib().hexsv_tile_shape(v, C.byref(a), C.byref(b), C.byref(c)))
        out.append((a.value, b.value, c.value))
    return out


class Grid:
    """Hexagonal raster handle (axial nq x nr parallelogram, edge a)."""

    def __init__(self, nq, nr, edge, side=(OUTFLOW, WALL, WALL, WALL), segs=(), active=None,
                 mask_bc=WALL):
        d = GridDesc()
        d.nq, d.nr, d.edge = int(nq), int(nr), float(edge)
        for k in range(4):
            d.side_bc[k] = int(side[k])
        segs = list(segs)
        if len(segs) > MAX_SEGMENTS:
            raise ValueError("too many segments")
        d.nseg = len(segs)
        for k, (s_, lo, hi, code) in enumerate(segs):
            d.seg[k] = Segment(int(s_), int(lo), int(hi), int(code))
        self._active = None
        if active is not None:
            # per cell: 0 outside the domain, 1 updated, 2 Dirichlet (held at its state),
            # 3 given flux (prescribes the discharge h v)
            a = np.asarray(active).reshape(-1)
            if a.dtype != bool and a.size and (a.min() < 0 or a.max() > 3):
                raise ValueError("active holds values other than 0, 1, 2, 3")
            self._active = np.ascontiguousarray(a, dtype=np.uint8)
            d.active = self._active.ctypes.data_as(C.POINTER(C.c_uint8))
        d.mask_bc = int(mask_bc)
        h = C.c_void_p()
        _check(lib().hexsv_grid_create(C.byref(d), C.byref(h)))
        self._h = h
        self.nq, self.nr, self.edge = int(nq), int(nr), float(edge)
        n, na = C.c_int64(), C.c_int64()
        _check(lib().hexsv_grid_counts(h, C.byref(n), C.byref(na)))
        self.cells, self.active_cells = n.value, na.value

    @classmethod
    def from_scenario(cls, sc):
        return cls(sc.nq, sc.nr, sc.a, sc.side, sc.segs, sc.active, sc.mask_code)

    def tables(self):
        """Device tensors (nbr int32 (N,6), code uint8 (N,6), q int32 (N,), r int32 (N,))
        computed by the table kernel on the current stream."""
        nbr = torch.empty((self.cells, 6), dtype=torch.int32, device="cuda")
        code = torch.empty((self.cells, 6), dtype=torch.uint8, device="cuda")
        q = torch.empty(self.cells, dtype=torch.int32, device="cuda")
        r = torch.empty(self.cells, dtype=torch.int32, device="cuda")
        _check(lib().hexsv_grid_tables_device(self._h, _ptr(nbr), _ptr(code), _ptr(q), _ptr(r),
                                              _stream()))
        return nbr, code, q, r

    def tables_host(self):
        """The same tables as NumPy arrays, written by the library into host memory."""
        nbr = np.empty((self.cells, 6), np.int32)
        code = np.empty((self.cells, 6), np.uint8)
        q = np.empty(self.cells, np.int32)
        r = np.empty(self.cells, np.int32)
        _check(lib().hexsv_grid_tables(self._h, *(C.c_void_p(a.ctypes.data)
                                                  for a in (nbr, code, q, r))))
        return nbr, code, q, r

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and _lib is not None:
            _lib.hexsv_grid_destroy(h)
            self._h = None


class Sim:
    """Single-catchment time stepper (FP64 or FP32 state, FP64 books and dt)."""

    def __init__(self, grid: Grid, precision="fp32", g=9.81, cfl=0.5, dt_max=1.0, h_dry=0.0,
                 steps_per_graph=100, tile=-1, wg_per_cu=0):
        self.grid = grid
        prec = {"fp64": FP64, "fp32": FP32, FP64: FP64, FP32: FP32}[precision]
        p = Params(float(g), float(cfl), float(dt_max), float(h_dry), prec, int(steps_per_graph),
                   int(tile), int(wg_per_cu), 0, 0)
        h = C.c_void_p()
        _check(lib().hexsv_sim_create(grid._h, C.byref(p), C.byref(h)))
        self._h = h
        self.precision = "fp64" if prec == FP64 else "fp32"

    @classmethod
    def from_scenario(cls, sc, precision="fp32", grid=None, **kw):
        grid = grid or Grid.from_scenario(sc)
        s = cls(grid, precision, g=sc.g, cfl=sc.cfl, dt_max=sc.dt_max, h_dry=sc.h_dry, **kw)
        s.set_fields(sc.z, sc.theta, sc.alpha_p, sc.alpha_s)
        s.set_rain(sc.rain_kind, sc.i_a, sc.t_a, sc.T_d)
        if getattr(sc, "tau_lin", 0.0):
            s.set_linear_friction(sc.tau_lin)
        if getattr(sc, "visc", False):
            s.set_viscosity(True)
        if getattr(sc, "f_inf", 0.0):
            s.set_infiltration(sc.f_inf, sc.h_inf)
        s.set_state(sc.h0, sc.v10, sc.v20, 0.0)
        return s

    def set_fields(self, z, theta, alpha_p, alpha_s):
        """alpha_s: one soil coefficient, or one per cell (an array of the raster's size)."""
        n = self.grid.cells
        z, th, ap = (_dev(x, n=n) for x in (z, theta, alpha_p))
        field, scalar = None, 0.0
        if np.ndim(alpha_s) > 0 or torch.is_tensor(alpha_s):
            field = _dev(alpha_s, n=n)
        else:
            scalar = float(alpha_s)
        _check(lib().hexsv_sim_set_fields(self._h, _ptr(z), _ptr(th), _ptr(ap), _ptr(field),
                                          scalar, _stream()))

    def set_viscosity(self, on):
        """Momentum flux with artificial viscosity (for shocks); off by default."""
        _check(lib().hexsv_sim_set_viscosity(self._h, int(bool(on))))

    def set_infiltration(self, f_inf, h_inf):
        """Infiltration i(h) = f_inf h / (h + h_inf) (m/s) in the mass source; 0 turns it off."""
        _check(lib().hexsv_sim_set_infiltration(self._h, float(f_inf), float(h_inf)))

    def set_linear_friction(self, tau):
        """Linear soil resistance -tau h v (1/s), the Thacker test's law; 0 turns it off."""
        _check(lib().hexsv_sim_set_linear_friction(self._h, float(tau)))

    def set_rain(self, kind=0, i_a=0.0, t_a=0.0, T_d=float("inf")):
        r = Rain(int(kind), float(i_a), float(t_a), float(T_d))
        _check(lib().hexsv_sim_set_rain(self._h, C.byref(r)))

    def set_state(self, h, v1, v2, t0=0.0):
        n = self.grid.cells
        h, v1, v2 = (_dev(x, n=n) for x in (h, v1, v2))
        _check(lib().hexsv_sim_set_state(self._h, float(t0), _ptr(h), _ptr(v1), _ptr(v2),
                                         _stream()))

    def run(self, t_end, max_steps=0):
        _check(lib().hexsv_sim_run(self._h, float(t_end), int(max_steps), _stream()))
        return self

    def state(self):
        n = self.grid.cells
        out = {k: torch.empty(n, dtype=torch.float64, device="cuda")
               for k in ("h", "v1", "v2", "q1", "q2")}
        _check(lib().hexsv_sim_get_state(self._h, *(_ptr(out[k]) for k in
                                                     ("h", "v1", "v2", "q1", "q2")), _stream()))
        return out

    def state_numpy(self):
        st = self.state()
        torch.cuda.synchronize()
        return {k: v.cpu().numpy() for k, v in st.items()}

    def books(self):
        b = Books()
        _check(lib().hexsv_sim_get_books(self._h, C.byref(b), _stream()))
        return b.as_dict()

    def set_books(self, d):
        b = Books(**{k: d[k] for k, _ in Books._fields_})
        _check(lib().hexsv_sim_set_books(self._h, C.byref(b), _stream()))

    def timing(self, enable=None):
        """Totals of the device-timed replays since the last reset; enable=True/False resets."""
        ms, st, rp = C.c_double(), C.c_int64(), C.c_int64()
        en = -1 if enable is None else int(bool(enable))
        _check(lib().hexsv_sim_timing(self._h, en, C.byref(ms), C.byref(st), C.byref(rp)))
        return {"gpu_ms": ms.value, "steps": st.value, "replays": rp.value}

    def time_kernel(self, nlaunch=50):
        """Average duration (ms) of the step kernel alone, from hipEvents on the current stream."""
        ms = C.c_double()
        _check(lib().hexsv_sim_time_kernel(self._h, int(nlaunch), C.byref(ms), _stream()))
        return ms.value

    def autotune(self, nlaunch=30, cache_path=None):
        """Pick the fastest tile variant for this raster (state and books are unchanged)."""
        best, ms = C.c_int32(), C.c_double()
        path = cache_path.encode() if cache_path else None
        _check(lib().hexsv_sim_autotune(self._h, int(nlaunch), path, C.byref(best), C.byref(ms),
                                        _stream()))
        return best.value, ms.value

    def run_surrogate(self, sur, t_end, window, k, residual_tol=1e-3, project=True):
        """Advance with surrogate windows and solver fallback; returns (accepted, fallback)."""
        a, f = C.c_int64(), C.c_int64()
        _check(lib().hexsv_sim_run_surrogate(self._h, sur._h, float(t_end), float(window), int(k),
                                             float(residual_tol), int(bool(project)), C.byref(a),
                                             C.byref(f), _stream()))
        return a.value, f.value

    def set_surrogate_backoff(self, max_spans):
        """Most spans the solver advances after a run of refused windows (0: none)."""
        _check(lib().hexsv_sim_set_surrogate_backoff(self._h, int(max_spans)))

    def surrogate_stats(self):
        """Windows of all run_surrogate calls: kept and refused (by reason)."""
        a = (C.c_int64 * 4)()
        _check(lib().hexsv_sim_surrogate_stats(self._h, a))
        return dict(zip(("kept", "refused_residual", "refused_wave_speed", "refused_nonfinite"),
                        list(a)))

    def surrogate_features(self, sur, window, k):
        """(cells, 11) FP32 network inputs of a window starting at the current state."""
        f = torch.empty((self.grid.cells, Surrogate.FEATURES), dtype=torch.float32, device="cuda")
        _check(lib().hexsv_sim_surrogate_features(self._h, sur._h, float(window), int(k), _ptr(f),
                                                  _stream()))
        return f

    def info(self):
        vals = [C.c_int32() for _ in range(5)]
        _check(lib().hexsv_sim_info(self._h, *(C.byref(v) for v in vals)))
        return dict(zip(("workgroups", "tile", "tq", "tr", "threads"), (v.value for v in vals)))

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and _lib is not None:
            _lib.hexsv_sim_destroy(h)
            self._h = None


class Ensemble:
    """Batch of independent catchments (uneven rasters) advanced by one persistent kernel."""

    MODES = {"auto": 0, "persistent": 1, "batched": 2}

    def __init__(self, grids, precision="fp32", g=9.81, cfl=0.5, dt_max=1.0, h_dry=0.0,
                 steps_per_launch=50, tile=-1, mode="auto"):
        self.grids = list(grids)
        prec = {"fp64": FP64, "fp32": FP32}[precision]
        p = Params(float(g), float(cfl), float(dt_max), float(h_dry), prec, int(steps_per_launch),
                   int(tile), 0, self.MODES[mode], 0)
        arr = (C.c_void_p * len(self.grids))(*[gr._h for gr in self.grids])
        h = C.c_void_p()
        _check(lib().hexsv_ensemble_create(len(self.grids), arr, C.byref(p), C.byref(h)))
        self._h = h
        self.precision = precision

    @classmethod
    def from_scenarios(cls, scs, precision="fp32", **kw):
        s0 = scs[0]
        ens = cls([Grid.from_scenario(sc) for sc in scs], precision, g=s0.g, cfl=s0.cfl,
                  dt_max=s0.dt_max, h_dry=s0.h_dry, **kw)
        if getattr(s0, "visc", False):
            ens.set_viscosity(True)
        for i, sc in enumerate(scs):
            ens.set_scenario(i, sc)
        return ens

    def set_viscosity(self, on):
        """Artificial viscosity for every scenario (batched-step mode only)."""
        _check(lib().hexsv_ensemble_set_viscosity(self._h, int(bool(on))))

    def set_scenario(self, s, sc, t0=0.0):
        n = self.grids[s].cells
        z, th, ap, h, v1, v2 = (_dev(x, n=n) for x in (sc.z, sc.theta, sc.alpha_p, sc.h0, sc.v10,
                                                       sc.v20))
        r = Rain(int(sc.rain_kind), float(sc.i_a), float(sc.t_a), float(sc.T_d))
        _check(lib().hexsv_ensemble_set_scenario(self._h, int(s), _ptr(z), _ptr(th), _ptr(ap),
                                                 float(sc.alpha_s), C.byref(r), float(t0),
                                                 _ptr(h), _ptr(v1), _ptr(v2), _stream()))

    def run(self, t_end, max_steps=0):
        t = np.ascontiguousarray(np.broadcast_to(np.asarray(t_end, np.float64),
                                                 (len(self.grids),)))
        _check(lib().hexsv_ensemble_run(self._h, t.ctypes.data_as(C.POINTER(C.c_double)),
                                        int(max_steps), _stream()))
        return self

    def state(self, s):
        n = self.grids[s].cells
        out = {k: torch.empty(n, dtype=torch.float64, device="cuda")
               for k in ("h", "v1", "v2", "q1", "q2")}
        _check(lib().hexsv_ensemble_get_state(self._h, int(s), *(_ptr(out[k]) for k in
                                                                 ("h", "v1", "v2", "q1", "q2")),
                                              _stream()))
        return out

    def state_numpy(self, s):
        st = self.state(s)
        torch.cuda.synchronize()
        return {k: v.cpu().numpy() for k, v in st.items()}

    def books(self, s):
        b = Books()
        _check(lib().hexsv_ensemble_get_books(self._h, int(s), C.byref(b), _stream()))
        return b.as_dict()

    def timing(self, enable=None):
        ms, cu, ln = C.c_double(), C.c_int64(), C.c_int64()
        en = -1 if enable is None else int(bool(enable))
        _check(lib().hexsv_ensemble_timing(self._h, en, C.byref(ms), C.byref(cu), C.byref(ln)))
        return {"gpu_ms": ms.value, "cell_updates": cu.value, "launches": ln.value}

    def autotune(self, ksteps=5, cache_path=None):
        """Pick the fastest ensemble tile variant (state and books are restored)."""
        best, ms = C.c_int32(), C.c_double()
        path = cache_path.encode() if cache_path else None
        _check(lib().hexsv_ensemble_autotune(self._h, int(ksteps), path, C.byref(best),
                                             C.byref(ms), _stream()))
        return best.value, ms.value

    def info(self):
        wg, tile, spl, mode = C.c_int32(), C.c_int32(), C.c_int32(), C.c_int32()
        cells = C.c_int64()
        _check(lib().hexsv_ensemble_info(self._h, C.byref(wg), C.byref(tile), C.byref(cells),
                                         C.byref(spl), C.byref(mode)))
        return {"workgroups": wg.value, "tile": tile.value, "cells": cells.value,
                "steps_per_launch": spl.value,
                "mode": {1: "persistent", 2: "batched"}.get(mode.value, "?")}

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and _lib is not None:
            _lib.hexsv_ensemble_destroy(h)
            self._h = None


class Surrogate:
    """Hex-convolution residual network (BF16 MFMA kernels, FP32 master weights)."""

    def __init__(self, layers=4, channels=32, k=16):
        h = C.c_void_p()
        _check(lib().hexsv_surrogate_create(int(layers), int(channels), int(k), C.byref(h)))
        self._h = h
        self.layers, self.channels = layers, channels
        self.k = int(lib().hexsv_surrogate_steps(h))
        self.num_params = int(lib().hexsv_surrogate_num_params(h))

    def set_params(self, p):
        t = _dev(p, dtype=torch.float32, n=self.num_params)
        _check(lib().hexsv_surrogate_set_params(self._h, _ptr(t), self.num_params, _stream()))

    def params(self):
        t = torch.empty(self.num_params, dtype=torch.float32, device="cuda")
        _check(lib().hexsv_surrogate_get_params(self._h, _ptr(t), self.num_params, _stream()))
        return t

    def set_scales(self, scales):
        """{H, Q, Z, dH, dQ, S}: input depth, discharge, elevation, output depth and discharge,
        input slope."""
        a = (C.c_float * len(scales))(*[float(x) for x in scales])
        _check(lib().hexsv_surrogate_set_scales(self._h, a, len(scales)))

    def scales(self, n=5):
        a = (C.c_float * n)()
        _check(lib().hexsv_surrogate_get_scales(self._h, a, n))
        return list(a)

    FEATURES = 11

    @staticmethod
    def _shape(x, nq, nr, ch):
        n = x.numel() // ch
        if x.numel() != n * ch or n % (nq * nr):
            raise ValueError("array does not hold whole samples")
        return n // (nq * nr)

    def set_fused(self, on=True):
        """Forward of the 4-layer, 32-channel network as one fused kernel or one launch per
        layer (the default); the outputs are the same bit for bit."""
        _check(lib().hexsv_surrogate_set_fused(self._h, 1 if on else 0))

    # grid (optional): the raster whose neighbour rule the taps follow (periodic sides, the
    # domain mask); without it the raster is a walled nq x nr parallelogram
    def forward(self, features, nq, nr, grid=None):
        f = _dev(features, dtype=torch.float32)
        batch = self._shape(f, nq, nr, self.FEATURES)
        out = torch.empty((batch * nq * nr, 4), dtype=torch.float32, device="cuda")
        _check(lib().hexsv_surrogate_forward(self._h, grid._h if grid else None, batch, int(nq),
                                             int(nr), _ptr(f), _ptr(out), _stream()))
        return out

    def forward_noalloc(self, features, nq, nr, out, grid=None):
        """forward into the caller's `out` ((cells, 4) FP32 on the device; columns 0..2
        written) with the library's static workspace: no allocation inside the call."""
        for name, t in (("features", features), ("out", out)):
            if not (torch.is_tensor(t) and t.is_cuda and t.dtype == torch.float32
                    and t.is_contiguous()):
                raise ValueError(f"{name}: a contiguous FP32 device tensor (no copy is made)")
        batch = self._shape(features, nq, nr, self.FEATURES)
        if out.numel() != 4 * batch * nq * nr:
            raise ValueError("out: 4 floats per cell")
        _check(lib().hexsv_surrogate_forward_noalloc(self._h, grid._h if grid else None, batch,
                                                     int(nq), int(nr), _ptr(features), _ptr(out),
                                                     _stream()))
        return out

    def gradient(self, features, target, nq, nr, grid=None):
        f = _dev(features, dtype=torch.float32)
        t = _dev(target, dtype=torch.float32)
        batch = self._shape(f, nq, nr, self.FEATURES)
        g = torch.empty(self.num_params, dtype=torch.float32, device="cuda")
        loss = C.c_double()
        _check(lib().hexsv_surrogate_gradient(self._h, grid._h if grid else None, batch, int(nq),
                                              int(nr), _ptr(f), _ptr(t), _ptr(g), C.byref(loss),
                                              _stream()))
        return loss.value, g

    def train_step(self, features, target, nq, nr, lr, grid=None):
        batch = self._shape(features, nq, nr, self.FEATURES)
        loss = C.c_double()
        _check(lib().hexsv_surrogate_train_step(self._h, grid._h if grid else None, batch,
                                                int(nq), int(nr), _ptr(features), _ptr(target),
                                                float(lr), C.byref(loss), _stream()))
        return loss.value

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and _lib is not None:
            _lib.hexsv_surrogate_destroy(h)
            self._h = None
