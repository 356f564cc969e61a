"""Seeded synthetic inputs shared by the solver's tests, the oracle's tests and the benchmark.

This module holds no arithmetic of the MHD method itself: it only draws random
numbers and lays out arrays.  Everything here is an *input* — the initial state
of a run and the random draws that the forcing of each step consumes
(Section 4, Eqs. forcing and fnorm: a random integer wave vector from a shell,
a random unit vector, a random phase).  How those draws become a forcing field
is method arithmetic and is written separately by the solver and the oracle.

Random numbers come from SplitMix64 (Steele, Lea and Flood, "Fast splittable
pseudorandom number generators", OOPSLA 2014), used as a counter-based
generator: output ``i`` of stream ``(seed, sid)`` is ``mix(key + (i+1)*GAMMA)``
with ``key = mix(seed ^ mix(sid))``.  A uniform double is the top 53 bits
times 2**-53; normals come from the Box-Muller transform of consecutive pairs.

State layout (the same for every consumer): a float array of shape
``(7, nz, ny, nx)`` — fields ln(rho), u_x, u_y, u_z, A_x, A_y, A_z — C-ordered,
so x is the fastest index.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field, asdict
from typing import List, Sequence, Tuple

import numpy as np

GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)

# stream ids
SID_FORCING = 1
SID_FIELD = 100  # + field index 0..6

NFIELDS = 7
FIELD_NAMES = ("lnrho", "ux", "uy", "uz", "ax", "ay", "az")


def _mix(z):
    """SplitMix64 output finaliser on a uint64 scalar or array (wrapping arithmetic)."""
    z = np.asarray(z, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
    return z ^ (z >> np.uint64(31))


def stream_key(seed: int, sid: int) -> np.uint64:
    return np.uint64(_mix(np.uint64(seed & 0xFFFFFFFFFFFFFFFF) ^ _mix(np.uint64(sid))))


def raw64(seed: int, sid: int, counters) -> np.ndarray:
    """Outputs ``counters`` (array of ints) of stream (seed, sid) as uint64."""
    key = stream_key(seed, sid)
    c = np.asarray(counters, dtype=np.uint64)
    with np.errstate(over="ignore"):
        return _mix(key + (c + np.uint64(1)) * GAMMA)


def uniform(seed: int, sid: int, counters) -> np.ndarray:
    """Uniform doubles in [0, 1) from the top 53 bits."""
    x = raw64(seed, sid, counters)
    return (x >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)


def normal(seed: int, sid: int, n: int, start: int = 0) -> np.ndarray:
    """``n`` standard normals: Box-Muller on uniform pairs (2p, 2p+1)."""
    npair = (n + 1) // 2
    p = np.arange(npair, dtype=np.uint64) + np.uint64(start)
    u1 = uniform(seed, sid, 2 * p)
    u2 = uniform(seed, sid, 2 * p + np.uint64(1))
    r = np.sqrt(-2.0 * np.log1p(-u1))
    out = np.empty(2 * npair)
    out[0::2] = r * np.cos(2.0 * math.pi * u2)
    out[1::2] = r * np.sin(2.0 * math.pi * u2)
    return out[:n]


# ---------------------------------------------------------------- forcing draws

def shell_vectors(kf: float) -> np.ndarray:
    """Integer wave vectors with kf-1/2 <= |k| <= kf+1/2, in lexicographic order.

    The shell is the one Section 4 describes for kf = 5 (4.5 <= |k| <= 5.5);
    the same half-width is used for any kf.
    """
    lo2, hi2 = (kf - 0.5) ** 2, (kf + 0.5) ** 2
    m = int(math.floor(kf + 0.5))
    out = []
    for kx in range(-m, m + 1):
        for ky in range(-m, m + 1):
            for kz in range(-m, m + 1):
                q = kx * kx + ky * ky + kz * kz
                if lo2 <= q <= hi2:
                    out.append((kx, ky, kz))
    return np.array(out, dtype=np.int32).reshape(-1, 3)


@dataclass
class ForcingDraw:
    """Random inputs of one step's forcing: wave vector, random unit vector, phase."""
    k: Tuple[int, int, int]
    e: Tuple[float, float, float]
    phi: float


def forcing_draws(seed: int, nsteps: int, kf: float, first_step: int = 0) -> List[ForcingDraw]:
    """Per-step forcing draws; step ``n`` uses counters 8n .. 8n+7 of stream (seed, 1).

    counter 8n   -> shell index (uniform over the shell)
    8n+1, 8n+2   -> first candidate unit vector e (uniform on the sphere)
    8n+3, 8n+4   -> second candidate, used if the first is within 8 degrees of k
    8n+5         -> phase phi, uniform in [-pi, pi)
    If both candidates are nearly parallel to k, e is the coordinate axis least
    parallel to k (ties to the lowest axis).
    """
    shell = shell_vectors(kf)
    out = []
    for n in range(first_step, first_step + nsteps):
        u = uniform(seed, SID_FORCING, np.arange(8 * n, 8 * n + 8))
        k = shell[min(int(u[0] * len(shell)), len(shell) - 1)]
        kn = math.sqrt(float(k[0] ** 2 + k[1] ** 2 + k[2] ** 2))
        khat = k / kn
        chosen = None
        for a, b in ((u[1], u[2]), (u[3], u[4])):
            z = 2.0 * a - 1.0
            s = math.sqrt(max(0.0, 1.0 - z * z))
            ph = 2.0 * math.pi * b
            e = np.array([s * math.cos(ph), s * math.sin(ph), z])
            if abs(float(np.dot(khat, e))) <= 0.99:
                chosen = e
                break
        if chosen is None:
            ax = int(np.argmin(np.abs(khat)))
            chosen = np.zeros(3)
            chosen[ax] = 1.0
        phi = math.pi * (2.0 * u[5] - 1.0)
        out.append(ForcingDraw(k=(int(k[0]), int(k[1]), int(k[2])),
                               e=(float(chosen[0]), float(chosen[1]), float(chosen[2])),
                               phi=float(phi)))
    return out


# ---------------------------------------------------------------- run parameters

TWO_PI = 2.0 * math.pi


@dataclass
class RunParams:
    """Physical and numerical parameters of one run (Section 4 units: L=2pi, cs=1, rho0=1, mu0=1)."""
    nx: int
    ny: int
    nz: int
    nu: float
    eta: float
    dt: float = 1e-3
    cs: float = 1.0
    lx: float = TWO_PI
    ly: float = TWO_PI
    lz: float = TWO_PI
    bext: Tuple[float, float, float] = (0.0, 0.0, 0.0)
    precision: int = 8  # bytes per value: 8 = FP64, 4 = FP32
    upwind: float = 0.0  # upwinding coefficient of the continuity advection (0: off, 1: full)

    @property
    def ncell(self) -> int:
        return self.nx * self.ny * self.nz

    def dict(self):
        return asdict(self)


@dataclass
class Forcing:
    """One step's forcing record: the draw plus helicity sigma and amplitude factor f0."""
    k: Tuple[int, int, int]
    e: Tuple[float, float, float]
    phi: float
    sigma: float
    f0: float


def forcing_schedule(seed: int, nsteps: int, kf: float, f0: float, sigma: float,
                     first_step: int = 0) -> List[Forcing]:
    return [Forcing(k=d.k, e=d.e, phi=d.phi, sigma=sigma, f0=f0)
            for d in forcing_draws(seed, nsteps, kf, first_step)]


def no_forcing(nsteps: int) -> List[Forcing]:
    """Records with f0 = 0: the forcing term vanishes exactly."""
    return [Forcing(k=(1, 0, 0), e=(0.0, 1.0, 0.0), phi=0.0, sigma=0.0, f0=0.0)
            for _ in range(nsteps)]


# ---------------------------------------------------------------- initial states

def ic_seed_noise(p: RunParams, seed: int, amp: float, dtype=np.float64) -> np.ndarray:
    """Section 4 initial condition: ln(rho)=0, u=0, A = amp * N(0,1) per cell and component."""
    st = np.zeros((NFIELDS, p.nz, p.ny, p.nx), dtype=np.float64)
    for c in range(3):
        st[4 + c] = amp * normal(seed, SID_FIELD + 4 + c, p.ncell).reshape(p.nz, p.ny, p.nx)
    return st.astype(dtype)


def smooth_state(p: RunParams, seed: int, kmax: int = 3, amp_lnrho: float = 0.1,
                 amp_u: float = 0.2, amp_a: float = 0.2, nmodes: int = 6,
                 dtype=np.float64) -> np.ndarray:
    """Band-limited random state: per field a sum of ``nmodes`` Fourier modes, |k_i| <= kmax.

    Mode m of field f has integer wave vector, amplitude and phase drawn from
    stream (seed, 100+f); the field is sum_m a_m cos(k_m . x + p_m) on the grid
    x = (i, j, l) * L / N, normalised so its largest |value| is ``amp``.
    """
    amps = [amp_lnrho] + [amp_u] * 3 + [amp_a] * 3
    st = np.zeros((NFIELDS, p.nz, p.ny, p.nx), dtype=np.float64)
    x = np.arange(p.nx) * (TWO_PI / p.nx)
    y = np.arange(p.ny) * (TWO_PI / p.ny)
    z = np.arange(p.nz) * (TWO_PI / p.nz)
    for f in range(NFIELDS):
        if amps[f] == 0.0:
            continue
        u = uniform(seed, SID_FIELD + f, np.arange(5 * nmodes))
        acc = np.zeros((p.nz, p.ny, p.nx))
        for m in range(nmodes):
            k = [int(math.floor(u[5 * m + c] * (2 * kmax + 1))) - kmax for c in range(3)]
            if k == [0, 0, 0]:
                k = [1, 0, 0]
            a = 0.5 + u[5 * m + 3]
            ph = TWO_PI * u[5 * m + 4]
            acc += a * np.cos(k[0] * x[None, None, :] + k[1] * y[None, :, None]
                              + k[2] * z[:, None, None] + ph)
        st[f] = amps[f] * acc / np.max(np.abs(acc))
    return st.astype(dtype)


def uniform_state(p: RunParams, seed: int, lo: float = 0.0, hi: float = 1.0,
                  dtype=np.float64) -> np.ndarray:
    """Every field uniform random in [lo, hi) per cell (the paper's benchmark fields, Appendix A)."""
    st = np.empty((NFIELDS, p.nz, p.ny, p.nx), dtype=np.float64)
    for f in range(NFIELDS):
        st[f] = (lo + (hi - lo) * uniform(seed, SID_FIELD + f, np.arange(p.ncell))).reshape(
            p.nz, p.ny, p.nx)
    return st.astype(dtype)


def noise_state(p: RunParams, seed: int, amp_lnrho: float = 0.05, amp_u: float = 0.05,
                amp_a: float = 0.05, dtype=np.float64) -> np.ndarray:
    """Every field amp * N(0,1) per cell: the rough case, where every stencil weight matters."""
    amps = [amp_lnrho] + [amp_u] * 3 + [amp_a] * 3
    st = np.empty((NFIELDS, p.nz, p.ny, p.nx), dtype=np.float64)
    for f in range(NFIELDS):
        st[f] = amps[f] * normal(seed, SID_FIELD + f, p.ncell).reshape(p.nz, p.ny, p.nx)
    return st.astype(dtype)


# ---------------------------------------------------------------- workloads

def ensemble_runs() -> List[dict]:
    """48 independent runs: 32 at 64^3 then 16 at 128^3, nu = eta log-spaced 5e-3 .. 2e-4,
    sigma = 1 for even i else 0, seed i, FP32, kf = 3, f0 = 0.02, dt = 1e-3."""
    runs = []
    for i in range(48):
        n = 64 if i < 32 else 128
        nu = 5e-3 * (0.04 ** (i / 47.0))
        runs.append(dict(n=n, nu=nu, eta=nu, sigma=1.0 if i % 2 == 0 else 0.0, seed=i,
                         precision=4, kf=3.0, f0=0.02, dt=1e-3, a_noise=1e-5))
    return runs


def serving_trace(nruns: int = 240, rate: float = 4.0, seed: int = 0, nsteps: int = 1000,
                  sizes: Sequence[int] = (32, 64, 128, 256)) -> List[dict]:
    """Poisson arrivals (rate per second) of runs with N uniform in ``sizes``, nu = eta
    log-uniform in [3e-4, 1e-2], sigma uniform in {0, 1}, seed j, FP32, ``nsteps`` steps.

    Draws come from stream (seed, 7) with 4 counters per run: inter-arrival time,
    size index, log-viscosity, helicity.
    """
    out, t = [], 0.0
    for j in range(nruns):
        u = uniform(seed, 7, np.arange(4 * j, 4 * j + 4))
        t += -math.log1p(-u[0]) / rate
        n = sizes[min(int(u[1] * len(sizes)), len(sizes) - 1)]
        nu = math.exp(math.log(3e-4) + u[2] * (math.log(1e-2) - math.log(3e-4)))
        sigma = 1.0 if u[3] >= 0.5 else 0.0
        out.append(dict(arrival=t, n=n, nu=nu, eta=nu, sigma=sigma, seed=j, precision=4,
                        kf=3.0, f0=0.02, dt=1e-3, a_noise=1e-5, nsteps=nsteps))
    return out
