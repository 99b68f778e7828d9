"""Seeded synthetic inputs shared by the oracle and the HIP path.

This module holds problem descriptions (grid, time axis, line geometry),
seeded earth models (a Gaussian low-velocity lens and a layered model with
sinusoidal interfaces and a smooth random perturbation), the Ricker wavelet
and seeded random vectors.  It contains none of the method's arithmetic: no
stencil, no absorbing layer, no injection or sampling rule, no solver step.

Units are SI throughout: metres, seconds, pascals, kg/m^3.

The workloads stand in for the paper's synthetic crosswell examples
(Numerical Examples section: smooth models, 20 m cells, sub-12 Hz wavelets);
the paper uses no public dataset.
"""
from __future__ import annotations

import dataclasses
import math
from dataclasses import dataclass, field

import numpy as np

RHO_WATERLIKE = 1000.0  # 1 g/cm^3, the paper's constant density
BASE_SEED = 20220331


@dataclass(frozen=True)
class Problem:
    """Geometry and discretisation of one surface-source subproblem family.

    The physical grid has ``nz`` rows (depth, slow axis) and ``nx`` columns
    (lateral, fast axis) with spacing ``h`` in both directions; node (i, j)
    sits at depth ``i*h`` and lateral position ``j*h``.  An absorbing layer of
    ``npml`` cells is added outside this grid on all four sides.

    The extended source lives on the horizontal line at depth ``z_src``,
    sampled at ``ns`` positions ``x_src0 + k*h``; receivers sit at depth
    ``z_rec`` at ``nr`` positions ``x_rec0 + k*h``.  ``slab_dz`` is the signed
    datum offset (in cells, positive = deeper) of the thin slab that carries
    the preconditioner; ``rslab_dz`` the same for the thin slab around the
    receiver line that carries the data-space weight of the weighted normal
    equations (0: none).  ``xs`` lists the lateral position of the physical
    point source of each shot (one shot = one subproblem sharing the model).
    """

    nz: int
    nx: int
    h: float
    dt: float
    nt: int
    order: int = 8
    npml: int = 20
    pml_R: float = 1e-3
    z_src: float = 0.0
    x_src0: float = 0.0
    ns: int = 0
    z_rec: float = 0.0
    x_rec0: float = 0.0
    nr: int = 0
    slab_dz: int = 5
    xs: tuple = (0.0,)
    rslab_dz: int = 0

    @property
    def nshots(self) -> int:
        return len(self.xs)

    def replace(self, **kw) -> "Problem":
        return dataclasses.replace(self, **kw)


@dataclass(frozen=True)
class Problem3:
    """Geometry and discretisation of the 3D form: physical grid nz x ny x
    nx (z slowest, x fastest), spacing h on every axis, node (i, k, j) at
    depth i h, y = k h, x = j h; an absorbing layer of npml cells on every
    side.  The source is a plane at depth z_src of nsx x nsy traces at
    (x_src0 + a h, y_src0 + b h), trace index b nsx + a; the receivers a
    plane at z_rec likewise.  slab_dz is the signed datum offset (cells) of
    the thin slab that carries the preconditioner, (x_s, y_s) the physical
    point from which the penalty measures lateral distance."""

    nz: int
    ny: int
    nx: int
    h: float
    dt: float
    nt: int
    order: int = 8
    npml: int = 10
    pml_R: float = 1e-3
    z_src: float = 0.0
    x_src0: float = 0.0
    y_src0: float = 0.0
    nsx: int = 1
    nsy: int = 1
    z_rec: float = 0.0
    x_rec0: float = 0.0
    y_rec0: float = 0.0
    nrx: int = 1
    nry: int = 1
    slab_dz: int = 5        # signed thin-slab datum offset (cells) for M^-1
    x_s: float = 0.0        # the physical point (lateral position) of the
    y_s: float = 0.0        # subproblem, for the penalty A

    @property
    def ns(self) -> int:
        return self.nsx * self.nsy

    @property
    def nr(self) -> int:
        return self.nrx * self.nry

    def replace(self, **kw) -> "Problem3":
        from dataclasses import replace
        return replace(self, **kw)


@dataclass
class Workload:
    """A problem plus its model, wavelet and solver settings."""

    name: str
    prob: Problem
    kappa: np.ndarray  # [nz][nx] bulk modulus, Pa
    rho: float
    freq: float  # Ricker peak frequency, Hz
    K: int  # fixed PCG iteration count
    alpha_rel: float
    dtype: str
    extras: dict = field(default_factory=dict)


# ----------------------------------------------------------------------------
# wavelet

def ricker(t: np.ndarray, f: float, t0: float | None = None) -> np.ndarray:
    """Ricker wavelet (1 - 2 pi^2 f^2 tau^2) exp(-pi^2 f^2 tau^2), tau = t - t0,
    with the default delay t0 = 1.5/f."""
    if t0 is None:
        t0 = 1.5 / f
    a = (math.pi * f * (np.asarray(t, dtype=np.float64) - t0)) ** 2
    return (1.0 - 2.0 * a) * np.exp(-a)


def ricker_deriv(t: np.ndarray, f: float, t0: float | None = None) -> np.ndarray:
    """Time derivative of :func:`ricker`."""
    if t0 is None:
        t0 = 1.5 / f
    tau = np.asarray(t, dtype=np.float64) - t0
    b = (math.pi * f) ** 2
    return (-6.0 * b * tau + 4.0 * b * b * tau ** 3) * np.exp(-b * tau * tau)


# ----------------------------------------------------------------------------
# models

def lens_velocity(nz: int, nx: int, h: float, rng: np.random.Generator,
                  c0: float = 2500.0, dip: float = 500.0, radius: float = 300.0,
                  xc_range=(600.0, 3400.0), zc_range=(600.0, 1400.0)) -> np.ndarray:
    """Background c0 with a Gaussian low-velocity lens of depth ``dip`` and
    radius ``radius``; the centre is drawn uniformly from the given ranges."""
    xc = rng.uniform(*xc_range)
    zc = rng.uniform(*zc_range)
    z = np.arange(nz)[:, None] * h
    x = np.arange(nx)[None, :] * h
    r2 = (x - xc) ** 2 + (z - zc) ** 2
    return c0 - dip * np.exp(-r2 / radius ** 2)


def layered_velocity(nz: int, nx: int, h: float, rng: np.random.Generator,
                     nlayers: int = 12, vmin: float = 1500.0, vmax: float = 4500.0,
                     zrange=(100.0, 3900.0), min_gap: float = 100.0,
                     amp: float = 20.0, pert: float = 0.03,
                     smooth: float = 50.0) -> np.ndarray:
    """Layered model: ``nlayers - 1`` interfaces with depths drawn uniformly
    (sorted, redrawn until separated by ``min_gap``), each bent by a sinusoid
    of amplitude ``amp`` and random wavelength/phase; layer k has velocity
    vmin + (vmax - vmin) k / (nlayers - 1).  The result is multiplied by
    1 + pert * delta with delta a Gaussian-smoothed white field (std 1,
    clipped to +-3)."""
    from scipy.ndimage import gaussian_filter

    nif = nlayers - 1
    for _ in range(1000):
        depths = np.sort(rng.uniform(zrange[0], zrange[1], size=nif))
        if np.all(np.diff(depths) >= min_gap):
            break
    lam = rng.uniform(500.0, 4000.0, size=nif)
    phi = rng.uniform(0.0, 2.0 * math.pi, size=nif)
    z = np.arange(nz)[:, None] * h
    x = np.arange(nx)[None, :] * h
    layer = np.zeros((nz, nx), dtype=np.int64)
    for k in range(nif):
        zk = depths[k] + amp * np.sin(2.0 * math.pi * x / lam[k] + phi[k])
        layer += (z >= zk).astype(np.int64)
    vel = vmin + (vmax - vmin) * layer / (nlayers - 1)
    white = rng.standard_normal((nz, nx))
    sm = gaussian_filter(white, sigma=smooth / h, mode="reflect")
    sm = (sm - sm.mean()) / sm.std()
    sm = np.clip(sm, -3.0, 3.0)
    return vel * (1.0 + pert * sm)


def layered_velocity3(nz: int, ny: int, nx: int, h: float, rng: np.random.Generator,
                      nlayers: int = 8, vmin: float = 1500.0, vmax: float = 4000.0,
                      amp: float = 20.0) -> np.ndarray:
    """3D layered model [nz][ny][nx]: ``nlayers - 1`` interfaces at depths
    drawn uniformly over the grid's depth range (sorted), each bent by a
    sinusoid in x and one in y of amplitude ``amp`` and random
    wavelength/phase; layer k has velocity vmin + (vmax - vmin) k /
    (nlayers - 1)."""
    nif = nlayers - 1
    depths = np.sort(rng.uniform(0.1 * (nz - 1) * h, 0.9 * (nz - 1) * h, size=nif))
    lam = rng.uniform(500.0, 4000.0, size=(nif, 2))
    phi = rng.uniform(0.0, 2.0 * math.pi, size=(nif, 2))
    z = np.arange(nz)[:, None, None] * h
    y = np.arange(ny)[None, :, None] * h
    x = np.arange(nx)[None, None, :] * h
    layer = np.zeros((nz, ny, nx), dtype=np.int64)
    for k in range(nif):
        zk = (depths[k] + amp * np.sin(2.0 * math.pi * x / lam[k, 0] + phi[k, 0])
              + amp * np.sin(2.0 * math.pi * y / lam[k, 1] + phi[k, 1]))
        layer += (z >= zk).astype(np.int64)
    return vmin + (vmax - vmin) * layer / (nlayers - 1)


def kappa_from_velocity(vel: np.ndarray, rho: float = RHO_WATERLIKE) -> np.ndarray:
    """Bulk modulus of a constant-density model with the given velocity."""
    return rho * np.asarray(vel, dtype=np.float64) ** 2


def with_gardner_density(wl: "Workload") -> "Workload":
    """The same workload with a density array instead of the constant
    density: rho = 310 v^(1/4) kg/m^3 (v in m/s, Gardner's empirical rule for
    sedimentary rocks) from the workload's velocity, the velocity kept
    (kappa = rho v^2)."""
    vel = np.sqrt(np.asarray(wl.kappa, dtype=np.float64) / wl.rho)
    rho = 310.0 * vel ** 0.25
    return Workload(wl.name + "+rho", wl.prob, rho * vel ** 2, rho, wl.freq, wl.K,
                    wl.alpha_rel, wl.dtype, dict(wl.extras))


def homogeneous_kappa(nz: int, nx: int, c: float = 2000.0,
                      rho: float = RHO_WATERLIKE) -> np.ndarray:
    return np.full((nz, nx), rho * c * c)


# ----------------------------------------------------------------------------
# workloads (the five benchmark configurations)

def shot_positions(nshots: int, width: float) -> tuple:
    """nshots source positions evenly spread over [0, width] (cell centres)."""
    return tuple((k + 0.5) * width / nshots for k in range(nshots))


_shot_positions = shot_positions


def workload(c: int, **over) -> Workload:
    """Configuration ``c`` in 1..4 (5 is a request generator, see
    :func:`serving_requests`).  Keyword overrides replace Problem fields."""
    rng = np.random.default_rng(BASE_SEED + c)
    if c == 1:
        nz, nx, h = 101, 201, 20.0
        vel = lens_velocity(nz, nx, h, rng)
        prob = Problem(nz=nz, nx=nx, h=h, dt=2e-3, nt=1000, order=4, npml=20,
                       z_src=100.0, x_src0=0.0, ns=nx, z_rec=40.0, x_rec0=0.0,
                       nr=nx, slab_dz=5, xs=(2000.0,))
        wl = Workload("c1", prob, kappa_from_velocity(vel), RHO_WATERLIKE,
                      8.0, 10, 1e-3, "f64")
    elif c in (2, 4):
        nz, nx, h = 801, 1601, 5.0
        rng = np.random.default_rng(BASE_SEED + 2)
        vel = layered_velocity(nz, nx, h, rng)
        prob = Problem(nz=nz, nx=nx, h=h, dt=0.5e-3, nt=4000, order=8, npml=20,
                       z_src=20.0, x_src0=0.0, ns=nx, z_rec=10.0, x_rec0=0.0,
                       nr=nx, slab_dz=5, xs=(4000.0,))
        wl = Workload("c2" if c == 2 else "c4", prob, kappa_from_velocity(vel),
                      RHO_WATERLIKE, 15.0, 30, 1e-3,
                      "f32" if c == 2 else "f16")
    elif c == 3:
        nz, nx, h = 401, 801, 10.0
        vel = layered_velocity(nz, nx, h, rng)
        prob = Problem(nz=nz, nx=nx, h=h, dt=1e-3, nt=2000, order=8, npml=20,
                       z_src=20.0, x_src0=0.0, ns=nx, z_rec=10.0, x_rec0=0.0,
                       nr=nx, slab_dz=5, xs=_shot_positions(64, (nx - 1) * h))
        wl = Workload("c3", prob, kappa_from_velocity(vel), RHO_WATERLIKE,
                      15.0, 20, 1e-3, "f32")
    else:
        raise ValueError(f"unknown configuration {c}")
    if over:
        wl.prob = wl.prob.replace(**over)
    return wl


SERVING_GRIDS = ((201, 401, 20.0), (401, 801, 10.0), (801, 1601, 5.0))


def serving_request(req_id: int, rng: np.random.Generator, max_shots: int = 64,
                    nt_range=(500, 4000)) -> Workload:
    """One request of the serving stream: a grid drawn from SERVING_GRIDS, a
    record length from nt_range in steps of 100, 1..max_shots shots spaced as
    in the batched configuration, and a layered model seeded by the request
    id.  dt = h/10 ms per metre of cell size (2, 1, 0.5 ms)."""
    gi = int(rng.integers(0, len(SERVING_GRIDS)))
    nz, nx, h = SERVING_GRIDS[gi]
    nt = int(rng.integers(nt_range[0] // 100, nt_range[1] // 100 + 1)) * 100
    nshots = int(rng.integers(1, max_shots + 1))
    mrng = np.random.default_rng(BASE_SEED + 1000 + req_id)
    vel = layered_velocity(nz, nx, h, mrng)
    dt = h / 10.0 * 1e-3
    prob = Problem(nz=nz, nx=nx, h=h, dt=dt, nt=nt, order=8, npml=20,
                   z_src=4 * h, x_src0=0.0, ns=nx, z_rec=2 * h, x_rec0=0.0,
                   nr=nx, slab_dz=5, xs=_shot_positions(nshots, (nx - 1) * h))
    return Workload(f"req{req_id}", prob, kappa_from_velocity(vel),
                    RHO_WATERLIKE, 15.0 * 5.0 / h if h > 5.0 else 15.0, 20,
                    1e-3, "f16")


def serving_requests(n: int = 200, seed: int = BASE_SEED + 5, **kw):
    """Seeded request stream: (arrival offset in units of the mean gap, Workload)."""
    rng = np.random.default_rng(seed)
    out = []
    t = 0.0
    for i in range(n):
        t += rng.exponential(1.0)
        out.append((t, serving_request(i, rng, **kw)))
    return out


# ----------------------------------------------------------------------------
# source gathers and random vectors

def spike_gather(prob: Problem, wavelet: np.ndarray, shot: int = 0) -> np.ndarray:
    """Source gather [nt][ns] that is zero except for the trace nearest the
    shot's physical position, which carries ``wavelet`` divided by the cell
    size (a point source on the source line expressed as a line density)."""
    g = np.zeros((prob.nt, prob.ns))
    k = int(round((prob.xs[shot] - prob.x_src0) / prob.h))
    k = min(max(k, 0), prob.ns - 1)
    g[:, k] = wavelet / prob.h
    return g


def source_wavelet(prob: Problem, freq: float) -> np.ndarray:
    """Ricker samples at the half-step times (n + 1/2) dt, the times at
    which the source term enters the leapfrog update n -> n+1."""
    t = (np.arange(prob.nt) + 0.5) * prob.dt
    return ricker(t, freq)


def random_traces(shape, seed: int) -> np.ndarray:
    return np.random.default_rng(seed).standard_normal(shape)


# ----------------------------------------------------------------------------
# the paper's crosswell example (Numerical Examples: 8 km x 4 km at 20 m,
# kappa 4 GPa, rho 1 g/cm^3, a central low-velocity lens down to 1.6 GPa,
# receivers at 1000 m and extended sources at 3000 m over x = 2000..6000 m,
# point source at (3500, 3500) m with a 1 / 2.5 / 7.5 / 12.5 Hz bandpass
# wavelet, auxiliary datums 100 m above both lines)

def bandpass_wavelet(t: np.ndarray, corners=(1.0, 2.5, 7.5, 12.5), t0: float = 0.8,
                     nfft: int = 1 << 16, dtf: float = 1e-3) -> np.ndarray:
    """Zero-phase wavelet with a trapezoidal amplitude spectrum (0 below
    corners[0], linear up to 1 at corners[1], flat to corners[2], linear
    down to 0 at corners[3]), centred at t0 and sampled at times t by linear
    interpolation of an nfft-point inverse FFT at spacing dtf; peak 1."""
    f = np.fft.rfftfreq(nfft, dtf)
    f1, f2, f3, f4 = corners
    amp = np.clip(np.minimum((f - f1) / (f2 - f1), (f4 - f) / (f4 - f3)), 0.0, 1.0)
    w = np.fft.irfft(amp, nfft)
    w = np.roll(w, nfft // 2)
    tw = (np.arange(nfft) - nfft // 2) * dtf + t0
    out = np.interp(np.asarray(t, dtype=np.float64), tw, w, left=0.0, right=0.0)
    return out / np.abs(w).max()


def crosswell_kappa(nz: int = 201, nx: int = 401, h: float = 20.0, lens: bool = True,
                    k0: float = 4.0e9, kmin: float = 1.6e9, radius: float = 500.0):
    """Bulk modulus of the crosswell example: k0 everywhere, minus (when
    lens) a Gaussian of standard deviation ``radius`` centred in the
    rectangle that brings it to kmin at the centre."""
    kap = np.full((nz, nx), k0)
    if lens:
        z = np.arange(nz)[:, None] * h - 0.5 * (nz - 1) * h
        x = np.arange(nx)[None, :] * h - 0.5 * (nx - 1) * h
        kap = kap - (k0 - kmin) * np.exp(-(x * x + z * z) / (2.0 * radius * radius))
    return kap


def crosswell_problem(h: float = 20.0, dt: float = 4e-3, nt: int = 1000, order: int = 8,
                      npml: int = 20) -> Problem:
    """The inversion geometry: extended sources on z = 3000 m and receivers
    on z = 1000 m, both over x = 2000..6000 m; thin-slab datums 100 m above
    each line; penalty centred on x_s = 3500 m."""
    nz, nx = int(round(4000.0 / h)) + 1, int(round(8000.0 / h)) + 1
    n = int(round(4000.0 / h)) + 1
    dz = -int(round(100.0 / h))
    return Problem(nz=nz, nx=nx, h=h, dt=dt, nt=nt, order=order, npml=npml,
                   z_src=3000.0, x_src0=2000.0, ns=n, z_rec=1000.0, x_rec0=2000.0, nr=n,
                   slab_dz=dz, xs=(3500.0,), rslab_dz=dz)


def crosswell_point_problem(prob: Problem) -> Problem:
    """The data geometry: the point source at (3500, 3500) m as a one-sample
    source line, the same receivers."""
    return prob.replace(z_src=3500.0, x_src0=3500.0, ns=1, slab_dz=-1, rslab_dz=0)
