"""Seeded synthetic scenarios for the hex-raster Saint-Venant stepper.

This module only draws inputs: terrain, porosity and drag fields, rain forcing,
initial states and boundary descriptions.  It holds none of the scheme's
arithmetic, so the CPU oracle and the GPU library can both consume its output
without sharing code.  Random numbers come from NumPy's PCG64 with the seed
``14933 + 1000 * config + scenario``.

The paper's own workloads (real DEMs and flume measurements) are not available;
the recipes below stand in for them (fractal relief with an outlet, Gaussian
vegetation patches, constant or triangular rain).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field, replace

import numpy as np

INTERIOR, WALL, OUTFLOW, PERIODIC = 0, 1, 2, 3
S, E, N, W = 0, 1, 2, 3

G_ACCEL = 9.81          # m/s^2 (value used by the paper's experiments)
ALPHA_P = 73.39         # 1/m, plant drag coefficient calibrated in the paper's flume study
ALPHA_S = 0.00709       # Darcy-Weisbach soil coefficient calibrated there too
MMH = 1.0e-3 / 3600.0   # 1 mm/h in m/s


def seed_of(config: int, scenario: int = 0) -> int:
    return 14933 + 1000 * config + scenario


def rng_of(config: int, scenario: int = 0) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed_of(config, scenario)))


@dataclass
class Scenario:
    """Everything one run needs; arrays are FP64, index i = r*nq + q."""
    name: str
    nq: int
    nr: int
    a: float
    z: np.ndarray
    theta: np.ndarray
    alpha_p: np.ndarray
    alpha_s: float = ALPHA_S
    side: tuple = (OUTFLOW, WALL, WALL, WALL)
    segs: tuple = ()
    active: np.ndarray | None = None
    mask_code: int = WALL
    rain_kind: int = 0
    i_a: float = 0.0
    t_a: float = 0.0
    T_d: float = float("inf")
    h0: np.ndarray | None = None
    v10: np.ndarray | None = None
    v20: np.ndarray | None = None
    t_end: float = 600.0
    g: float = G_ACCEL
    cfl: float = 0.5
    dt_max: float = 1.0
    h_dry: float = 0.0
    tau_lin: float = 0.0  # linear soil resistance -tau*h*v (1/s); 0: the paper's Darcy-Weisbach law
    visc: bool = False    # augmented momentum flux with artificial viscosity (for shocks)
    f_inf: float = 0.0    # infiltration i(h) = f_inf h / (h + h_inf), m/s; 0: none
    h_inf: float = 0.0    # its half-rate depth, m
    meta: dict = field(default_factory=dict)

    def __post_init__(self):
        n = self.nq * self.nr
        if self.h0 is None:
            self.h0 = np.zeros(n)
        if self.v10 is None:
            self.v10 = np.zeros(n)
        if self.v20 is None:
            self.v20 = np.zeros(n)

    @property
    def n(self) -> int:
        return self.nq * self.nr

    @property
    def rain(self):
        return (self.rain_kind, self.i_a, self.t_a, self.T_d)

    def with_(self, **kw) -> "Scenario":
        return replace(self, **kw)


# ------------------------------------------------------------ raster layout

def centres(nq: int, nr: int, a: float):
    """Hex centre coordinates of the axial parallelogram (pointy-top, edge a)."""
    q = np.tile(np.arange(nq, dtype=np.float64), nr)
    r = np.repeat(np.arange(nr, dtype=np.float64), nq)
    x = a * math.sqrt(3.0) * (q + 0.5 * r)
    y = 1.5 * a * r
    return x, y


# ---------------------------------------------------------------- terrain

def fractal_field(nq, nr, a, rng, beta=2.0):
    """Gaussian random surface with power spectrum ~ |k|^-beta, sampled at hex centres.

    Built by an inverse real FFT on a rectangle covering the parallelogram, with
    random phases, then bilinear interpolation at the centres.  Returned in [0, 1].
    """
    dx, dy = a * math.sqrt(3.0), 1.5 * a
    nx = nq + (nr + 1) // 2 + 2
    ny = nr + 2
    kx = np.fft.rfftfreq(nx, d=dx)
    ky = np.fft.fftfreq(ny, d=dy)
    K = np.sqrt(kx[None, :] ** 2 + ky[:, None] ** 2)
    K[0, 0] = 1.0
    amp = K ** (-beta / 2.0)
    amp[0, 0] = 0.0
    phase = rng.uniform(0.0, 2.0 * math.pi, size=amp.shape)
    spec = (amp * np.exp(1j * phase)).astype(np.complex128)
    f = np.fft.irfft2(spec, s=(ny, nx))
    x, y = centres(nq, nr, a)
    fx, fy = x / dx, y / dy
    i0 = np.clip(np.floor(fx).astype(np.int64), 0, nx - 2)
    j0 = np.clip(np.floor(fy).astype(np.int64), 0, ny - 2)
    tx, ty = fx - i0, fy - j0
    v = ((1 - tx) * (1 - ty) * f[j0, i0] + tx * (1 - ty) * f[j0, i0 + 1]
         + (1 - tx) * ty * f[j0 + 1, i0] + tx * ty * f[j0 + 1, i0 + 1])
    v = (v - v.min()) / max(v.max() - v.min(), 1e-300)
    return v


def carve_outlet(z, nq, nr, a, width=16, radius_cells=256, grade=0.01):
    """Lower the terrain around an outlet in the middle of the S side.

    z <- min(z, z_out + grade * d) within radius_cells*a of the outlet centre, with
    z_out = min(z) - 1 m.  Returns (z, segs) with segs the OUTFLOW segment of the S side.
    """
    x, y = centres(nq, nr, a)
    q0 = nq // 2 - width // 2
    xo = a * math.sqrt(3.0) * (nq // 2)
    d = np.hypot(x - xo, y)
    z_out = z.min() - 1.0
    near = d <= radius_cells * a
    z = z.copy()
    z[near] = np.minimum(z[near], z_out + grade * d[near])
    segs = ((S, q0, q0 + width, OUTFLOW),)
    return z, segs


# ------------------------------------------------------------- vegetation

def vegetation_density(nq, nr, a, rng, n_patches, peak_lo=0.0, peak_hi=0.6, dmax=0.6,
                       sig_lo=4.0, sig_hi=32.0):
    """Sum of Gaussian patches of plant density, capped at dmax.

    Centres uniform over the raster, widths U[sig_lo*a, sig_hi*a], peaks U[peak_lo, peak_hi].
    Each patch is evaluated only within 4 widths of its centre.
    """
    n = nq * nr
    d = np.zeros(n)
    x, y = centres(nq, nr, a)
    sq3 = math.sqrt(3.0)
    cq = rng.uniform(0, nq, size=n_patches)
    cr = rng.uniform(0, nr, size=n_patches)
    sig = rng.uniform(sig_lo * a, sig_hi * a, size=n_patches)
    peak = rng.uniform(peak_lo, peak_hi, size=n_patches)
    d2 = d.reshape(nr, nq)
    for p in range(n_patches):
        cx = a * sq3 * (cq[p] + 0.5 * cr[p])
        cy = 1.5 * a * cr[p]
        R = 4.0 * sig[p]
        r_lo = max(0, int(math.floor((cy - R) / (1.5 * a))))
        r_hi = min(nr, int(math.ceil((cy + R) / (1.5 * a))) + 1)
        if r_lo >= r_hi:
            continue
        q_lo = max(0, int(math.floor((cx - R) / (a * sq3) - 0.5 * (r_hi - 1))))
        q_hi = min(nq, int(math.ceil((cx + R) / (a * sq3) - 0.5 * r_lo)) + 1)
        if q_lo >= q_hi:
            continue
        qq = np.arange(q_lo, q_hi, dtype=np.float64)
        rr = np.arange(r_lo, r_hi, dtype=np.float64)
        X = a * sq3 * (qq[None, :] + 0.5 * rr[:, None])
        Y = 1.5 * a * rr[:, None] + 0.0 * qq[None, :]
        g = peak[p] * np.exp(-((X - cx) ** 2 + (Y - cy) ** 2) / (2.0 * sig[p] ** 2))
        d2[r_lo:r_hi, q_lo:q_hi] += g
    return np.minimum(d, dmax)


# ----------------------------------------------------------------- configs

def c1_planar(nq=64, nr=64, a=1.0, slope=0.05, theta=0.8, rain_mmh=50.0, t_end=600.0):
    """Plain method, FP64: uniform planar slope, porosity 0.8, constant drag, dry start."""
    n = nq * nr
    _, y = centres(nq, nr, a)
    return Scenario(
        name=f"planar{nq}x{nr}", nq=nq, nr=nr, a=a, z=slope * y, theta=np.full(n, theta),
        alpha_p=np.full(n, ALPHA_P), side=(OUTFLOW, WALL, WALL, WALL), rain_kind=0,
        i_a=rain_mmh * MMH, T_d=float("inf"), t_end=t_end,
        meta={"slope": slope, "rain_mmh": rain_mmh})


def catchment(nq, nr, a, config, relief=40.0, rain_mmh=100.0, t_end=3600.0, rain_T=None,
              outlet_width=16, scenario=0):
    """Single fractal catchment with a carved outlet and Gaussian vegetation patches."""
    rng = rng_of(config, scenario)
    z = relief * fractal_field(nq, nr, a, rng)
    z, segs = carve_outlet(z, nq, nr, a, width=outlet_width,
                           radius_cells=min(256, max(nq, nr) // 4))
    n = nq * nr
    d = vegetation_density(nq, nr, a, rng, max(1, n // 2048))
    return Scenario(
        name=f"catchment{nq}x{nr}", nq=nq, nr=nr, a=a, z=z, theta=1.0 - d,
        alpha_p=np.full(n, ALPHA_P), side=(WALL, WALL, WALL, WALL), segs=segs, rain_kind=0,
        i_a=rain_mmh * MMH, T_d=float("inf") if rain_T is None else rain_T, t_end=t_end,
        meta={"relief": relief, "rain_mmh": rain_mmh, "seed": seed_of(config, scenario)})


def c2_catchment(nq=1024, nr=1024, a=2.0, t_end=3600.0):
    """Single catchment, FP64 vs FP32: fractal relief 0-40 m, outlet, 100 mm/h for 3600 s."""
    return catchment(nq, nr, a, config=2, rain_mmh=100.0, t_end=t_end)


def c4_large(nq=4096, nr=4096, a=2.0, t_end=3600.0):
    """Large single domain, FP32: as C2 with a 150 mm/h storm for 1800 s then recession."""
    return catchment(nq, nr, a, config=4, rain_mmh=150.0, t_end=t_end, rain_T=1800.0)


def ensemble_member(s, nmin=128, nmax=512, a=1.0, t_end=1800.0, config=3, size=None):
    """One scenario of the batched ensemble: planar slope, patches, constant or triangular rain."""
    rng = rng_of(config, s)
    ns = int(rng.integers(nmin, nmax + 1)) if size is None else int(size)
    slope = float(rng.uniform(0.01, 0.20))
    peak = float(rng.uniform(0.0, 0.6))
    i_mmh = float(rng.uniform(10.0, 150.0))
    tri = bool(rng.integers(0, 2))
    n = ns * ns
    _, y = centres(ns, ns, a)
    d = vegetation_density(ns, ns, a, rng, max(1, n // 2048), peak_lo=0.0, peak_hi=peak)
    if tri:
        kind, t_a, T_d = 1, 0.25 * t_end, t_end
    else:
        kind, t_a, T_d = 0, 0.0, float("inf")
    return Scenario(
        name=f"ens{config}_{s}_{ns}", nq=ns, nr=ns, a=a, z=slope * y, theta=1.0 - d,
        alpha_p=np.full(n, ALPHA_P), side=(OUTFLOW, WALL, WALL, WALL), rain_kind=kind,
        i_a=i_mmh * MMH, t_a=t_a, T_d=T_d, t_end=t_end,
        meta={"slope": slope, "peak": peak, "rain_mmh": i_mmh, "triangular": tri,
              "seed": seed_of(config, s)})


def c3_ensemble(n_scen=256, nmin=128, nmax=512, t_end=1800.0, config=3):
    return [ensemble_member(s, nmin, nmax, t_end=t_end, config=config) for s in range(n_scen)]


# ------------------------------------------------------- invariant set-ups

def hexagon_mask(nq, nr, R):
    """Active cells within hex distance R of the centre cell (nq//2, nr//2)."""
    q = np.tile(np.arange(nq), nr) - nq // 2
    r = np.repeat(np.arange(nr), nq) - nr // 2
    return (np.maximum(np.maximum(np.abs(q), np.abs(r)), np.abs(q + r)) <= R).astype(np.uint8)


def cone(R=12, a=1.0, H=2.0, crater=False, rain_mmh=200.0, t_end=60.0, rim=WALL, theta=0.9):
    """Six-fold symmetric cone (or crater) on a hexagonal active region of radius R."""
    nq = nr = 2 * R + 3
    act = hexagon_mask(nq, nr, R)
    x, y = centres(nq, nr, a)
    xc, yc = a * math.sqrt(3.0) * (nq // 2 + 0.5 * (nr // 2)), 1.5 * a * (nr // 2)
    rho = np.hypot(x - xc, y - yc)
    rho_max = R * a * math.sqrt(3.0)
    zf = H * (1.0 - rho / rho_max)
    if crater:
        zf = H * rho / rho_max
    n = nq * nr
    return Scenario(
        name=f"cone{R}{'c' if crater else ''}", nq=nq, nr=nr, a=a, z=zf, theta=np.full(n, theta),
        alpha_p=np.full(n, ALPHA_P), side=(WALL, WALL, WALL, WALL), active=act, mask_code=rim,
        rain_kind=0, i_a=rain_mmh * MMH, t_end=t_end, meta={"R": R})


def kinematic_strip(nq=8, nr=64, a=1.0, slope=0.05, theta=0.8, rain_mmh=50.0, t_end=3600.0):
    """Planar slope periodic in q, wall at the top row, free outflow at r = 0."""
    n = nq * nr
    _, y = centres(nq, nr, a)
    return Scenario(
        name=f"strip{nq}x{nr}", nq=nq, nr=nr, a=a, z=slope * y, theta=np.full(n, theta),
        alpha_p=np.full(n, ALPHA_P), side=(OUTFLOW, PERIODIC, WALL, PERIODIC), rain_kind=0,
        i_a=rain_mmh * MMH, t_end=t_end, meta={"slope": slope})


def lake_at_rest(nq=24, nr=20, a=1.0, level=1.0, emerged=False, seed=7):
    """Still water over rough dyadic terrain: w = g*(z+h) is constant on wet cells.

    Terrain values are multiples of 2^-10 below the level so z + h == level exactly.
    With emerged=True some cells rise above the level and stay dry.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    n = nq * nr
    z = np.round(rng.uniform(0.0, 0.75, size=n) * 1024.0) / 1024.0
    if emerged:
        bumps = rng.random(n) < 0.15
        z[bumps] = level + np.round(rng.uniform(0.01, 0.3, size=bumps.sum()) * 1024.0) / 1024.0
    h = np.maximum(level - z, 0.0)
    th = np.round(rng.uniform(0.4, 1.0, size=n) * 256.0) / 256.0
    return Scenario(
        name="lake", nq=nq, nr=nr, a=a, z=z, theta=th, alpha_p=np.full(n, ALPHA_P),
        side=(WALL, WALL, WALL, WALL), rain_kind=0, i_a=0.0, h0=h, t_end=50.0)


def thacker(a=0.888231, half_x=200.0, half_y=150.0, t_end=330.0, tau=0.7, curv=(1.25e-3, 5e-3),
            centre=(500.0, 500.0), w0=15.0, du0=0.02 * G_ACCEL, dv0=-0.1 * G_ACCEL, h_dry=1e-3,
            cfl=0.25):
    """The non-oscillating Thacker problem of Sec. 3.2.2 / Appendix B: paraboloid bed
    z = A (x-x0)^2 + B (y-y0)^2, no vegetation (theta = 1), no rain, linear soil resistance
    -tau h v, velocity initially zero with accelerations (du0, dv0), free surface
    w(0,x,y) = w0 - (x-x0) du0/g - (y-y0) dv0/g (the exact solution at t = 0), h = [w - z]_+.

    The raster is a parallelogram of edge a covering x0 +- half_x, y0 +- half_y (the water
    stays well inside; the extra cells are dry), walls all round.  Below h_dry (1 mm) the
    velocity is set to zero: with only a linear resistance a thin film at the wet/dry front
    would otherwise be accelerated without bound.  The Courant number is 0.25: at 0.5 a mode
    in the 15 m deep centre of the bowl grows slowly and takes over after about 60 s (the
    paper does not give its value for this test).  meta carries the exact solution's
    parameters and the centre coordinates' offset (ox, oy)."""
    A, B = curv
    x0, y0 = centre
    nr = int(math.ceil(2.0 * half_y / (1.5 * a))) + 1
    shift = a * math.sqrt(3.0) * 0.5 * (nr - 1)
    nq = int(math.ceil((2.0 * half_x + shift) / (a * math.sqrt(3.0)))) + 1
    ox, oy = x0 - half_x - shift, y0 - half_y
    x, y = centres(nq, nr, a)
    x, y = x + ox, y + oy
    z = A * (x - x0) ** 2 + B * (y - y0) ** 2
    w = w0 - (x - x0) * du0 / G_ACCEL - (y - y0) * dv0 / G_ACCEL
    n = nq * nr
    return Scenario(
        name=f"thacker-a{a:g}", nq=nq, nr=nr, a=a, z=z, theta=np.ones(n), alpha_p=np.zeros(n),
        alpha_s=0.0, side=(WALL, WALL, WALL, WALL), h0=np.maximum(w - z, 0.0), t_end=t_end,
        tau_lin=tau, h_dry=h_dry, cfl=cfl,
        meta={"A": A, "B": B, "x0": x0, "y0": y0, "ox": ox, "oy": oy, "tau": tau, "w0": w0,
              "u0": 0.0, "v0": 0.0, "du0": du0, "dv0": dv0, "g": G_ACCEL})


def riemann(n_section=1122, length=18.0, width=1.0, x_jump=9.0, t_end=1.5,
            left=(0.8, 1.0, 0.2, 5.00), right=(1.0, 1.2, 0.6, 1.33), cfl=0.5):
    """The Riemann problem with vegetation of Sec. 3.2.3: a horizontal channel of the given
    length and width with a jump of porosity, bed, depth and velocity at x_jump; each side
    is (theta, z, h, u) of the paper's data table (v = 0).  Pointy-top hexes whose rows
    run along the channel, n_section centres per row (the paper's longitudinal section
    has 1122); the rectangle is cut from the axial parallelogram by the active mask.  The
    channel walls are the raster's S and N sides; the cut ends are OUTFLOW (ghost cells
    copy the cell, so the supercritical inflow at x = 0 keeps its state).  No friction
    (the paper gives no coefficients for this test) and the artificial-viscosity flux."""
    a = length / (n_section * math.sqrt(3.0))
    s3a = a * math.sqrt(3.0)
    nr = int(math.floor((width - a) / (1.5 * a))) + 1
    oy = 0.5 * (width - 1.5 * a * (nr - 1))
    ox = 0.5 * s3a - 0.5 * s3a * (nr - 1)
    nq = n_section + (nr - 1 + 1) // 2 + 1
    x, y = centres(nq, nr, a)
    x, y = x + ox, y + oy
    eps = 1e-9 * length
    act = ((x >= 0.5 * s3a - eps) & (x <= length - 0.5 * s3a + eps)).astype(np.uint8)
    L = x <= x_jump
    pick = lambda k: np.where(L, left[k], right[k]).astype(np.float64)
    n = nq * nr
    h0 = np.where(act > 0, pick(2), 0.0)
    v10 = np.where(act > 0, pick(3), 0.0)
    return Scenario(
        name=f"riemann-{n_section}", nq=nq, nr=nr, a=a, z=pick(1), theta=pick(0),
        alpha_p=np.zeros(n), alpha_s=0.0, side=(WALL, OUTFLOW, WALL, OUTFLOW), active=act,
        mask_code=OUTFLOW, h0=h0, v10=v10, t_end=t_end, cfl=cfl, visc=True,
        meta={"ox": ox, "oy": oy, "x_jump": x_jump, "left": left, "right": right})


def radial(kind="crater", a=0.5, r0=10.0, r1=100.0, A=10.0, h0=0.05, v0=1.0, t_end=40.0,
           cfl=0.5, h_dry=1e-5):
    """Flow on a radially symmetric surface (Sec. 3.2.1): an annulus r0 <= r <= r1 with bed
    z = A + s A cos(pi (r - r0) / (r1 - r0)), s = -1 for the crater (its rim r1 is the top)
    and +1 for the hillock (its inner edge r0 is the top).  Water enters through the top
    edge with depth h0 and speed v0 along -n (n the domain's outward normal there) and
    leaves freely through the bottom edge.  The inflow is a ring of Dirichlet cells (active
    code 2) one cell thick just outside the top edge, holding that state; the bottom edge's
    masked neighbours are OUTFLOW.  theta = 1, no friction (the paper gives no coefficients
    for this test), no rain; the annulus starts dry."""
    s = -1.0 if kind == "crater" else 1.0
    R = r1 + 3.0 * a
    nr = int(math.ceil(2.0 * R / (1.5 * a))) + 1
    shift = a * math.sqrt(3.0) * 0.5 * (nr - 1)
    nq = int(math.ceil((2.0 * R + shift) / (a * math.sqrt(3.0)))) + 1
    x, y = centres(nq, nr, a)
    x = x - R - shift
    y = y - R
    rr = np.hypot(x, y)
    ring = a * math.sqrt(3.0)
    act = ((rr >= r0) & (rr <= r1)).astype(np.uint8)
    if kind == "crater":
        inflow, rin = (rr > r1) & (rr <= r1 + ring), r1
    else:
        inflow, rin = (rr < r0) & (rr >= r0 - ring), r0
    act[inflow] = 2
    z = A + s * A * np.cos(math.pi * (rr - r0) / (r1 - r0))
    n = nq * nr
    ux, uy = x / np.maximum(rr, 1e-12), y / np.maximum(rr, 1e-12)
    vdir = -1.0 if kind == "crater" else 1.0  # -v0 n: inward at the rim, outward at r0
    h = np.where(inflow, h0, 0.0)
    return Scenario(
        name=f"radial-{kind}-a{a:g}", nq=nq, nr=nr, a=a, z=z, theta=np.ones(n),
        alpha_p=np.zeros(n), alpha_s=0.0, side=(WALL, WALL, WALL, WALL), active=act,
        mask_code=OUTFLOW, h0=h, v10=np.where(inflow, vdir * v0 * ux, 0.0),
        v20=np.where(inflow, vdir * v0 * uy, 0.0), t_end=t_end, cfl=cfl, h_dry=h_dry,
        meta={"kind": kind, "r0": r0, "r1": r1, "A": A, "s": s, "h0": h0, "v0": v0,
              "r_in": rin, "ox": -R - shift, "oy": -R, "g": G_ACCEL})


def flume(q=0.007, h_in=0.03, theta_v=0.99364, m=0.00105, alpha_s=ALPHA_S, alpha_p=ALPHA_P,
          a=0.05, length=18.0, width=1.0, vegetated="lower", t_end=300.0, inflow="flux"):
    """The sloping laboratory flume of Sec. 3.3.2 (18 m x 1 m, bed z = -m (x - 18), emergent
    vegetation of porosity theta_v on the lower half x in [9, 18] ("lower", theta_1) or the
    upper half ("upper", theta_2)), fed at x = 0 with the discharge q per unit width and
    draining freely at x = 18.  The inflow is a column of boundary cells just upstream of
    x = 0 holding depth h_in and velocity q / h_in along x: given-mass-flux cells (active code
    3, inflow="flux": every edge into one carries the discharge l q cos(angle) and sees the
    cell's own depth) or Dirichlet cells (code 2, inflow="dirichlet": the state h_in is
    imposed).  The channel walls are the raster's S and N sides; the masked cells past
    x = 18 are OUTFLOW.  The channel starts at depth h_in with the same discharge."""
    s3 = math.sqrt(3.0)
    nr = max(2, int(round(width / (1.5 * a))))
    ox = -s3 * a * (2.0 + 0.5 * (nr - 1))
    nq = int(math.ceil((length + 2.0 * s3 * a - ox) / (s3 * a))) + 1
    x, y = centres(nq, nr, a)
    x = x + ox
    act = np.zeros(nq * nr, np.uint8)
    act[(x >= 0.0) & (x <= length)] = 1
    act[(x < 0.0) & (x >= -s3 * a)] = 3 if inflow == "flux" else 2
    veg = (x >= 0.5 * length) if vegetated == "lower" else (x < 0.5 * length)
    theta = np.where(veg, theta_v, 1.0)
    if inflow != "flux":
        theta = np.where(act == 2, 1.0, theta)  # the imposed state carries q = h_in v
    h = np.where(act > 0, h_in, 0.0)
    v1 = np.where(act == 1, q / (theta * h_in), np.where(act > 1, q / h_in, 0.0))
    return Scenario(
        name=f"flume-{vegetated}-q{q:g}", nq=nq, nr=nr, a=a, z=-m * (x - length), theta=theta,
        alpha_p=np.full(nq * nr, float(alpha_p)), alpha_s=float(alpha_s), side=(WALL,) * 4,
        active=act, mask_code=OUTFLOW, h0=h, v10=v1, v20=np.zeros(nq * nr), t_end=t_end,
        meta={"x": x, "q": q, "h_in": h_in, "theta_v": theta_v, "m": m, "length": length,
              "vegetated": vegetated, "veg_zone": (act == 1) & (x >= 0.5 * length)})


def random_state(sc: Scenario, seed: int, depth=0.05, speed=0.3, dry_frac=0.2):
    """A rough wet/dry state on sc's raster (for one-step checks)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    n = sc.n
    h = rng.uniform(0.0, depth, size=n)
    h[rng.random(n) < dry_frac] = 0.0
    v1 = rng.uniform(-speed, speed, size=n)
    v2 = rng.uniform(-speed, speed, size=n)
    v1[h == 0] = 0.0
    v2[h == 0] = 0.0
    return h, v1, v2
