"""Seeded synthetic initial conditions and request traces.

This module only *generates inputs*: phase-space grids of the initial
distribution f(x, p, t=0) and the parameter sets of the workloads.  It holds
none of the arithmetic of the time-split solver (no interpolation, no force,
no reduction order), so both the solver library and the CPU oracle can be fed
from it without sharing any part of the method.

Grid convention (used by every generator): an axis [umin, umax) with n nodes
has spacing du = (umax - umin) / n and nodes u_i = umin + i*du, i = 0..n-1.
Arrays are row-major f[j, i] with j the momentum index and i the position
index, i.e. x is contiguous, as in the data layout of Sec. 3 of the paper.

Initial conditions follow the paper's workloads (Sec. 4):
  * waterbag: f constant on |x| <= x0, |p| <= p0 (Sec. 4.1 uses the inclusive
    bounds), the HMF waterbag being fixed by its magnetization M0 and energy
    per particle U (Sec. 4.2, eqs. hmfpot and mxmydef);
  * homogeneous Gaussian in p with a cos(theta) perturbation;
every one normalised to unit total mass on the grid, which is the mean-field
scaling of the Hamiltonian (Sec. 2, eq. hamgen).  Noise is multiplicative on
the support, f = c (1 + A eta), with eta uniform in [-1, 1) drawn from a
counter-based SplitMix64 stream (Steele, Lea & Flood 2014): the k-th draw of
seed s is mix(s + (k+1) * 0x9E3779B97F4A7C15), top 53 bits.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field, asdict

import numpy as np

MODEL_HMF, MODEL_RING, MODEL_SHEET, MODEL_EXTERNAL = 0, 1, 2, 3
BC_PERIODIC, BC_ZERO = 0, 1
STORAGE_F64, STORAGE_F32 = 0, 1
SPLINE_FD, SPLINE_GS = 0, 1  # f'' by eq. (findif) or by eq. (tridiagsys)
SPLIT_STRANG, SPLIT_TRIPLE_JUMP, SPLIT_SUZUKI = 0, 1, 2  # time splitting: one step, or a 4th-order composition

_GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def splitmix64(seed: int, counter: np.ndarray) -> np.ndarray:
    """k-th outputs of the SplitMix64 stream seeded with `seed` (uint64 array)."""
    with np.errstate(over="ignore"):
        z = np.uint64(seed & 0xFFFFFFFFFFFFFFFF) + (counter.astype(np.uint64) + np.uint64(1)) * _GOLDEN
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        return z ^ (z >> np.uint64(31))


def uniform01(seed: int, counter: np.ndarray) -> np.ndarray:
    """Uniform doubles in [0, 1) from the top 53 bits of SplitMix64."""
    return (splitmix64(seed, counter) >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)


def nodes(n: int, umin: float, umax: float) -> np.ndarray:
    du = (umax - umin) / n
    return umin + np.arange(n, dtype=np.float64) * du


@dataclass
class Params:
    """Physical and numerical parameters of one simulation (one phase-space grid)."""
    model: int
    nx: int
    np_: int
    xmin: float
    xmax: float
    pmin: float
    pmax: float
    dt: float
    bc_x: int = BC_PERIODIC
    bc_p: int = BC_PERIODIC
    storage: int = STORAGE_F64
    ring_eps: float = 0.01
    sheet_G: float = 1.0
    spline: int = SPLINE_FD
    splitting: int = SPLIT_STRANG
    filter_every: int = 0
    filter_strength: float = 0.0

    @property
    def dx(self) -> float:
        return (self.xmax - self.xmin) / self.nx

    @property
    def dp(self) -> float:
        return (self.pmax - self.pmin) / self.np_

    def as_dict(self) -> dict:
        return asdict(self)


# ---------------------------------------------------------------------------
# Waterbag parameter map (Sec. 4.2): a uniform f on |theta| <= theta0,
# |p| <= p0 has M = sin(theta0)/theta0 and energy per particle
# U = p0^2/6 + (1 - M^2)/2 (kinetic <p^2>/2 plus the HMF potential).
# ---------------------------------------------------------------------------

def waterbag_halfwidths(M0: float, U: float) -> tuple[float, float]:
    """(theta0, p0) of the HMF waterbag with magnetization M0 and energy U."""
    if not (0.0 <= M0 < 1.0):
        raise ValueError("M0 must lie in [0, 1)")
    kin = U - 0.5 * (1.0 - M0 * M0)
    if kin < 0.0:
        raise ValueError("U below the potential energy of the waterbag")
    # sin(t)/t decreases monotonically from 1 (t -> 0) to 0 (t = pi): bisection.
    lo, hi = 0.0, math.pi
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        val = math.sin(mid) / mid if mid > 0.0 else 1.0
        if val > M0:
            lo = mid
        else:
            hi = mid
        if hi - lo <= 4e-16 * hi:
            break
    theta0 = 0.5 * (lo + hi)
    p0 = math.sqrt(6.0 * kin)
    return theta0, p0


def _normalise(raw: np.ndarray, dx: float, dp: float) -> np.ndarray:
    """raw / ((S dx) dp), S the sum of raw in index order: each row serially
    from i = 0 (cumsum accumulates in order), then the row sums from j = 0.
    Any generator of the same raw values can reproduce S bit for bit."""
    rows = np.cumsum(raw, axis=1)[:, -1]
    total = float(np.cumsum(rows)[-1]) * dx * dp
    if not total > 0.0:
        raise ValueError("empty initial condition")
    return raw / total


def waterbag(p: Params, x0: float, p0: float, noise: float = 0.0, seed: int = 0) -> np.ndarray:
    """Uniform f on |x| <= x0, |p| <= p0 (inclusive), multiplicative noise, unit mass.

    Each half-width is raised to at least two grid cells so that no parameter
    choice gives an empty support.
    """
    x0 = max(x0, 2.0 * p.dx)
    p0 = max(p0, 2.0 * p.dp)
    x = nodes(p.nx, p.xmin, p.xmax)
    v = nodes(p.np_, p.pmin, p.pmax)
    support = (np.abs(v)[:, None] <= p0) & (np.abs(x)[None, :] <= x0)
    raw = np.where(support, 1.0, 0.0)
    if noise != 0.0:
        # draw k = j nx + i of the stream for the support nodes only
        k = np.flatnonzero(support).astype(np.uint64)
        eta = 2.0 * uniform01(seed, k) - 1.0
        raw.ravel()[k.astype(np.int64)] = 1.0 + noise * eta
    return _normalise(raw, p.dx, p.dp)


def gaussian(p: Params, T: float, amp: float, seed: int = 0) -> np.ndarray:
    """f proportional to exp(-p^2/2T) (1 + amp cos(x - phi)), unit mass.

    phi = 0 for seed 0 (mirror-symmetric state), else 2 pi u(seed).
    """
    phi = 0.0 if seed == 0 else 2.0 * math.pi * float(uniform01(seed, np.zeros(1, np.uint64))[0])
    x = nodes(p.nx, p.xmin, p.xmax)
    v = nodes(p.np_, p.pmin, p.pmax)
    # exp and cos of the C library, once per node
    e = np.array([math.exp(-(vj * vj) / (2.0 * T)) for vj in v.tolist()])
    c = np.array([1.0 + amp * math.cos(xi - phi) for xi in x.tolist()])
    raw = e[:, None] * c[None, :]
    return _normalise(raw, p.dx, p.dp)


# ---------------------------------------------------------------------------
# Workloads.  Domains and sizes of the five workload families.
# ---------------------------------------------------------------------------

def hmf_waterbag_small(seed: int = 0) -> tuple[Params, np.ndarray, int]:
    """HMF, 128 x 128, theta in [-pi, pi), p in [-2.5, 2.5), waterbag M0 = 0.5,
    U = 0.69, noise 1e-4, dt = 0.1, 100 steps."""
    p = Params(MODEL_HMF, 128, 128, -math.pi, math.pi, -2.5, 2.5, 0.1)
    th0, p0 = waterbag_halfwidths(0.5, 0.69)
    return p, waterbag(p, th0, p0, 1e-4, seed), 100


def hmf_gaussian(n: int, T: float, storage: int = STORAGE_F64, seed: int = 0) -> tuple[Params, np.ndarray, int]:
    """HMF, n x n, Gaussian at temperature T with a 1e-3 cos(theta) seed,
    dt = 0.05, 2000 steps."""
    p = Params(MODEL_HMF, n, n, -math.pi, math.pi, -2.5, 2.5, 0.05, storage=storage)
    return p, gaussian(p, T, 1e-3, seed), 2000


def ring_waterbag(n: int = 2048, storage: int = STORAGE_F64, seed: int = 0) -> tuple[Params, np.ndarray, int]:
    """Ring model, n x n, p in [-3, 3), eps = 0.01, waterbag with M0 = 0.8 at the
    paper's energy e = 0.7, noise 1e-4, dt = 0.02, 1000 steps."""
    p = Params(MODEL_RING, n, n, -math.pi, math.pi, -3.0, 3.0, 0.02, storage=storage, ring_eps=0.01)
    th0, p0 = waterbag_halfwidths(0.8, 0.7)
    return p, waterbag(p, th0, p0, 1e-4, seed), 1000


def sheet_waterbag(n: int = 4096, storage: int = STORAGE_F64, seed: int = 0) -> tuple[Params, np.ndarray, int]:
    """Self-gravitating sheets, n x n, x in [-10, 10) with f = 0 outside,
    p in [-4, 4) periodic, G = 1, waterbag x0 = 1, p0 = 0.5, noise 1e-4,
    dt = 0.01, 2000 steps."""
    p = Params(MODEL_SHEET, n, n, -10.0, 10.0, -4.0, 4.0, 0.01, bc_x=BC_ZERO,
               storage=storage, sheet_G=1.0)
    return p, waterbag(p, 1.0, 0.5, 1e-4, seed), 2000


# ---------------------------------------------------------------------------
# Serving trace: parameter-scan requests with Poisson arrivals.
# ---------------------------------------------------------------------------

SERVE_SIDES = (64, 128, 256, 512, 1024, 2048)
_DOMAINS = {
    MODEL_HMF: dict(xmin=-math.pi, xmax=math.pi, pmin=-2.5, pmax=2.5, bc_x=BC_PERIODIC),
    MODEL_RING: dict(xmin=-math.pi, xmax=math.pi, pmin=-3.0, pmax=3.0, bc_x=BC_PERIODIC),
    MODEL_SHEET: dict(xmin=-10.0, xmax=10.0, pmin=-4.0, pmax=4.0, bc_x=BC_ZERO),
}


@dataclass
class Request:
    rid: int
    arrival: float          # seconds after the start of the trace
    params: Params
    U: float
    M0: float
    seed: int
    nsteps: int

    def initial_condition(self) -> np.ndarray:
        th0, p0 = waterbag_halfwidths(self.M0, self.U)
        return waterbag(self.params, th0, p0, 1e-4, self.seed)


def serving_trace(nreq: int = 512, rate: float = math.inf, seed: int = 0,
                  storage: int = STORAGE_F32, sides=SERVE_SIDES,
                  steps_range=(100, 2000)) -> list[Request]:
    """Requests of the batched parameter scan.

    Model uniform over {HMF, ring, sheet} (each with its own domain), grid
    sides drawn independently from `sides`, U ~ U[0.5, 0.8], M0 ~ U[0, 1),
    dt in {0.05, 0.1}, steps uniform in `steps_range`.  rate = inf puts every
    arrival at t = 0 (a saturating burst); otherwise arrivals are Poisson.
    For the ring and the sheet the same (theta0, p0) map is used, x0 = theta0.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    t = 0.0
    out = []
    for r in range(nreq):
        model = int(rng.integers(0, 3))
        nx = int(sides[int(rng.integers(0, len(sides)))])
        npp = int(sides[int(rng.integers(0, len(sides)))])
        U = float(rng.uniform(0.5, 0.8))
        M0 = float(rng.uniform(0.0, 1.0))
        dt = (0.05, 0.1)[int(rng.integers(0, 2))]
        nsteps = int(rng.integers(steps_range[0], steps_range[1] + 1))
        if math.isfinite(rate):
            t += float(rng.exponential(1.0 / rate))
        d = _DOMAINS[model]
        p = Params(model, nx, npp, d["xmin"], d["xmax"], d["pmin"], d["pmax"], dt,
                   bc_x=d["bc_x"], storage=storage)
        out.append(Request(r, t, p, U, M0, r + 1 + (seed << 20), nsteps))
    return out
