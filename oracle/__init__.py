"""FP64 CPU oracle of the porous Saint-Venant hex-raster scheme — TEST INFRASTRUCTURE.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  It wraps ``libhexsv_oracle.so`` (plain C,
built from ``hexsv_oracle.c`` by :func:`build`) with ctypes and numpy; it shares no
code with the GPU library.  Every function cites the passage of arXiv 2406.14933 it
follows; the C source states the readings taken where the paper is silent.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libhexsv_oracle.so")
SRC_PATH = os.path.join(HERE, "hexsv_oracle.c")

INTERIOR, WALL, OUTFLOW, PERIODIC, DIRICHLET, FLUX = 0, 1, 2, 3, 4, 5
S, E, N, W = 0, 1, 2, 3
DQ = (1, 0, -1, -1, 0, 1)
DR = (0, 1, 1, 0, -1, -1)


def build(quiet: bool = True) -> str:
    """Compile the oracle with gcc: FP64, no fast-math, no FMA contraction."""
    cmd = ["gcc", "-O2", "-fno-fast-math", "-ffp-contract=off", "-fopenmp", "-fPIC",
           "-shared", "-std=c99", "-Wall", "-o", LIB_PATH + ".tmp", SRC_PATH, "-lm"]
    subprocess.run(cmd, check=True, capture_output=quiet)
    os.replace(LIB_PATH + ".tmp", LIB_PATH)
    return LIB_PATH


class RefParams(C.Structure):
    _fields_ = [("g", C.c_double), ("cfl", C.c_double), ("dt_max", C.c_double),
                ("h_dry", C.c_double), ("alpha_s", C.c_double), ("tau_lin", C.c_double),
                ("visc", C.c_int32), ("f_inf", C.c_double), ("h_inf", C.c_double),
                ("alpha_s_cell", C.c_void_p)]


class RefRain(C.Structure):
    _fields_ = [("kind", C.c_int32), ("i_a", C.c_double), ("t_a", C.c_double),
                ("T_d", C.c_double)]


class RefBooks(C.Structure):
    _fields_ = [("t", C.c_double), ("initial", C.c_double), ("stored", C.c_double),
                ("rain", C.c_double), ("outflow", C.c_double), ("clamp", C.c_double),
                ("residual", C.c_double), ("steps", C.c_int64), ("dt_min", C.c_double),
                ("dt_max_seen", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH) or os.path.getmtime(LIB_PATH) < os.path.getmtime(SRC_PATH):
            build()
        L = C.CDLL(LIB_PATH)
        dp = C.POINTER(C.c_double)
        ip = C.POINTER(C.c_int32)
        up = C.POINTER(C.c_uint8)
        L.ref_geometry.argtypes = [C.c_double, dp]
        L.ref_normal.argtypes = [C.c_int, dp]
        L.ref_tables.argtypes = [C.c_int32, C.c_int32, ip, C.c_int32, ip, up, C.c_int32, ip, up]
        L.ref_tables.restype = C.c_int
        L.ref_rain_rate.argtypes = [C.c_int32, C.c_double, C.c_double, C.c_double, C.c_double]
        L.ref_rain_rate.restype = C.c_double
        L.ref_mu.argtypes = [C.c_double] * 4
        L.ref_mu.restype = C.c_double
        L.ref_cell_sums.argtypes = [C.c_int32, ip, up, C.c_double, C.c_double, dp, dp, dp, dp,
                                    dp, C.c_int32, dp]
        L.ref_visc_sums.argtypes = [C.c_int32, ip, up, C.c_double, C.c_double, dp, dp, dp, dp,
                                    C.c_int32, dp]
        L.ref_cmax.argtypes = [C.c_int32, dp, C.c_double, dp, dp, dp]
        L.ref_cmax.restype = C.c_double
        L.ref_dt.argtypes = [C.c_double, C.POINTER(RefParams), C.c_double, C.c_double, C.c_double]
        L.ref_dt.restype = C.c_double
        L.ref_step_cells.argtypes = [C.c_int32, ip, up, C.c_double, dp, dp, dp,
                                     C.POINTER(RefParams), C.POINTER(RefRain), C.c_double,
                                     C.c_double, dp, dp, dp, C.c_int32, ip, dp, dp, dp, dp]
        L.ref_books_init.argtypes = [C.c_int32, C.c_double, dp, dp, C.c_double,
                                     C.POINTER(RefBooks)]
        L.ref_run.argtypes = [C.c_int32, ip, up, C.c_double, dp, dp, dp, C.POINTER(RefParams),
                              C.POINTER(RefRain), C.c_double, C.c_int64, dp, dp, dp,
                              C.POINTER(RefBooks), dp, C.c_int32]
        L.ref_run.restype = C.c_int64
        L.ref_hexconv_fwd.argtypes = [C.c_int32, ip, C.c_int32, C.c_int32, dp, dp, dp, dp]
        L.ref_hexconv_bwd.argtypes = [C.c_int32, ip, C.c_int32, C.c_int32, dp, dp, dp, dp, dp, dp]
        _lib = L
    return _lib


def _d(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _i(a):
    return a.ctypes.data_as(C.POINTER(C.c_int32))


def _u(a):
    return a.ctypes.data_as(C.POINTER(C.c_uint8))


def _f64(a, n=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if n is not None:
        assert a.size == n, (a.size, n)
    return a


# ----------------------------------------------------------------- geometry

def geometry(a: float):
    """(sigma, l, phi_min) of the regular hexagon of edge a (Sec. 2.2 (a); eq. fvm_2D_eq_frac.13)."""
    out = np.zeros(3)
    lib().ref_geometry(a, _d(out))
    return float(out[0]), float(out[1]), float(out[2])


def normal(k: int):
    out = np.zeros(2)
    lib().ref_normal(k, _d(out))
    return float(out[0]), float(out[1])


@dataclass
class RefGrid:
    """Axial nq x nr hex raster with explicit neighbour/edge-code tables (Sec. 2.2 (a))."""
    nq: int
    nr: int
    a: float
    nbr: np.ndarray   # (N, 6) int32, -1 where the edge is not INTERIOR
    code: np.ndarray  # (N, 6) uint8
    active: np.ndarray  # (N,) bool: computational cells
    dirichlet: np.ndarray = None  # (N,) bool: boundary cells whose state is held fixed
    flux: np.ndarray = None       # (N,) bool: boundary cells prescribing the discharge h v

    @property
    def n(self):
        return self.nq * self.nr


def tables(nq, nr, side=(WALL, WALL, WALL, WALL), segs=(), active=None, mask_code=WALL):
    """Neighbour and edge-code tables; see ``ref_tables`` in hexsv_oracle.h."""
    N = nq * nr
    side_a = np.ascontiguousarray(side, dtype=np.int32)
    seg_a = np.ascontiguousarray(np.array(segs, dtype=np.int32).reshape(-1, 4))
    act = None if active is None else np.ascontiguousarray(active, dtype=np.uint8).reshape(N)
    nbr = np.empty((N, 6), np.int32)
    code = np.empty((N, 6), np.uint8)
    rc = lib().ref_tables(nq, nr, _i(side_a), len(seg_a), _i(seg_a) if len(seg_a) else None,
                          _u(act) if act is not None else None, mask_code, _i(nbr), _u(code))
    if rc != 0:
        raise ValueError("invalid grid description")
    return nbr, code


def grid(nq, nr, a, side=(WALL, WALL, WALL, WALL), segs=(), active=None, mask_code=WALL):
    nbr, code = tables(nq, nr, side, segs, active, mask_code)
    if active is None:
        act, dch, flx = np.ones(nq * nr, bool), np.zeros(nq * nr, bool), np.zeros(nq * nr, bool)
    else:
        raw = np.asarray(active).reshape(-1)
        act, dch, flx = raw == 1, raw == 2, raw == 3
    return RefGrid(nq, nr, float(a), nbr, code, act, dch, flx)


# ------------------------------------------------------------ small pieces

def rain_rate(kind, i_a, t_a, T_d, t):
    """r(t): constant on [0, T_d] (kind 0) or the triangular hyetograph of Appendix C (kind 1)."""
    return lib().ref_rain_rate(int(kind), i_a, t_a, T_d, t)


def mu(alpha, beta, g1, g2):
    """Appendix A, miu-formula."""
    return lib().ref_mu(alpha, beta, g1, g2)


def params(g=9.81, cfl=0.5, dt_max=1.0, h_dry=0.0, alpha_s=0.0, tau_lin=0.0, visc=False,
           f_inf=0.0, h_inf=0.0):
    """alpha_s: one Darcy-Weisbach coefficient, or an array of one per cell (eq_tsa_darcy)."""
    field = None
    if np.ndim(alpha_s) > 0:
        field = np.ascontiguousarray(alpha_s, dtype=np.float64).reshape(-1)
        alpha_s = 0.0
    p = RefParams(g, cfl, dt_max, h_dry, float(alpha_s), tau_lin, int(bool(visc)), f_inf, h_inf,
                  field.ctypes.data if field is not None else None)
    p._alpha_s_field = field  # keeps the array alive while the parameters are used
    return p


def rain(kind=0, i_a=0.0, t_a=0.0, T_d=float("inf")):
    return RefRain(int(kind), i_a, t_a, T_d)


def _theta_masked(G: RefGrid, theta):
    th = _f64(theta, G.n).copy()
    dch = G.dirichlet if G.dirichlet is not None else np.zeros(G.n, bool)
    flx = G.flux if G.flux is not None else np.zeros(G.n, bool)
    th[~(G.active | dch | flx)] = 0.0
    th[dch] = -th[dch]  # held fixed: not updated, not booked, read with |theta| by neighbours
    th[flx] = -1.0      # held fixed, not booked; its edges read h, v and z only
    return th


def cell_sums(G: RefGrid, g, z, theta, h, v1, v2, i):
    """{L, J1, J2, S1, S2, F_out} of eq. fvm_2D_eq_frac.01 for cell i."""
    out = np.zeros(6)
    z, th, h, v1, v2 = (_f64(x, G.n) for x in (z, _theta_masked(G, theta), h, v1, v2))
    lib().ref_cell_sums(G.n, _i(G.nbr), _u(G.code), G.a, g, _d(z), _d(th), _d(h), _d(v1),
                        _d(v2), int(i), _d(out))
    return out


def visc_sums(G: RefGrid, g, theta, h, v1, v2, i):
    """The artificial-viscosity part {V1, V2} of the augmented flux J^v for cell i."""
    out = np.zeros(2)
    th, h, v1, v2 = (_f64(x, G.n) for x in (_theta_masked(G, theta), h, v1, v2))
    lib().ref_visc_sums(G.n, _i(G.nbr), _u(G.code), G.a, g, _d(th), _d(h), _d(v1), _d(v2),
                        int(i), _d(out))
    return out


def cmax(G: RefGrid, g, theta, h, v1, v2):
    th, h, v1, v2 = (_f64(x, G.n) for x in (_theta_masked(G, theta), h, v1, v2))
    return lib().ref_cmax(G.n, _d(th), g, _d(h), _d(v1), _d(v2))


def dt(a, p: RefParams, c_max, t, t_end):
    return lib().ref_dt(a, C.byref(p), c_max, t, t_end)


def books_init(G: RefGrid, theta, h, t0=0.0) -> RefBooks:
    b = RefBooks()
    th, h = _f64(_theta_masked(G, theta), G.n), _f64(h, G.n)
    lib().ref_books_init(G.n, G.a, _d(th), _d(h), t0, C.byref(b))
    return b


def step_cells(G: RefGrid, z, theta, alpha_p, p: RefParams, r: RefRain, dt_, t_next,
               h, v1, v2, cells):
    """One step of eq. fvm_2D_eq_frac.07 for the given cells from state n; returns (h, v1, v2, add)."""
    cells = np.ascontiguousarray(cells, dtype=np.int32)
    n = len(cells)
    hn, v1n, v2n, add = np.zeros(n), np.zeros(n), np.zeros(n), np.zeros(3)
    z, th, ap, h, v1, v2 = (_f64(x, G.n) for x in
                            (z, _theta_masked(G, theta), alpha_p, h, v1, v2))
    lib().ref_step_cells(G.n, _i(G.nbr), _u(G.code), G.a, _d(z), _d(th), _d(ap), C.byref(p),
                         C.byref(r), dt_, t_next, _d(h), _d(v1), _d(v2), n, _i(cells),
                         _d(hn), _d(v1n), _d(v2n), _d(add))
    return hn, v1n, v2n, add


def run(G: RefGrid, z, theta, alpha_p, p: RefParams, r: RefRain, h, v1, v2, t_end,
        max_steps=10 ** 9, books: RefBooks | None = None, t0=0.0, log_dt=False, nthreads=0):
    """Advance the state to t_end (or max_steps).  Returns (h, v1, v2, books, dt_log)."""
    z, th, ap = (_f64(x, G.n) for x in (z, _theta_masked(G, theta), alpha_p))
    h, v1, v2 = (_f64(x, G.n).copy() for x in (h, v1, v2))
    if books is None:
        books = books_init(G, theta, h, t0)
    cap = int(min(max_steps, 10 ** 7))
    dlog = np.zeros(cap) if log_dt else None
    rc = lib().ref_run(G.n, _i(G.nbr), _u(G.code), G.a, _d(z), _d(th), _d(ap), C.byref(p),
                       C.byref(r), t_end, cap, _d(h), _d(v1), _d(v2), C.byref(books),
                       _d(dlog) if dlog is not None else None, int(nthreads))
    if rc == -1:
        raise ValueError("oracle rejected the input")
    if rc == -2:
        raise FloatingPointError("non-finite state in the oracle")
    if dlog is not None:
        dlog = dlog[:rc]
    return h, v1, v2, books, dlog


# --------------------------------------------------------------- hex conv

def hexconv_fwd(G: RefGrid, x, W, b):
    """y[o,i] = b[o] + sum_{c,t} W[o,c,t] x[c, nbr_t(i)], zero where a tap has no neighbour."""
    cin, cout = x.shape[0], W.shape[0]
    x = np.ascontiguousarray(x, np.float64)
    W = np.ascontiguousarray(W, np.float64)
    b = np.ascontiguousarray(b, np.float64)
    y = np.zeros((cout, G.n))
    lib().ref_hexconv_fwd(G.n, _i(G.nbr), cin, cout, _d(x), _d(W), _d(b), _d(y))
    return y


def hexconv_bwd(G: RefGrid, x, W, dy):
    """(dx, dW, db) of :func:`hexconv_fwd`."""
    cin, cout = x.shape[0], W.shape[0]
    x = np.ascontiguousarray(x, np.float64)
    W = np.ascontiguousarray(W, np.float64)
    dy = np.ascontiguousarray(dy, np.float64)
    dx = np.zeros_like(x)
    dW = np.zeros_like(W)
    db = np.zeros(cout)
    lib().ref_hexconv_bwd(G.n, _i(G.nbr), cin, cout, _d(x), _d(W), _d(dy), _d(dx), _d(dW),
                          _d(db))
    return dx, dW, db
