"""FP64 CPU oracle of the forced isothermal MHD update (Section 4 equations, Section 2 methods).

TEST INFRASTRUCTURE.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  The solver package
never imports it, and it imports nothing from the solver.

The magnetic power spectrum (``magnetic_spectrum``) is the discrete curl followed by
a library FFT over the full grid and a shell sum, written from its definition.

Two independent implementations live here:
  * ``mhd_oracle.c`` (built into ``liboracle.so``): plain C loops with periodic
    wrap, OpenMP over z-planes, used at every size;
  * ``numpy_ref.py``: whole-array NumPy with ``np.roll``, used as a brute-force
    cross-check on tiny grids.
Both read the state as a float64 array of shape (7, nz, ny, nx).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from typing import Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")
SRC_PATH = os.path.join(HERE, "mhd_oracle.c")


def build(verbose: bool = False) -> str:
    """Compile the C oracle with gcc (no FMA contraction: plain IEEE double)."""
    cmd = ["gcc", "-O2", "-fopenmp", "-std=c11", "-ffp-contract=off", "-Wall", "-shared",
           "-fPIC", "-o", LIB_PATH + ".tmp", SRC_PATH, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.check_call(cmd)
    os.replace(LIB_PATH + ".tmp", LIB_PATH)
    return LIB_PATH


class _Params(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32), ("pad", C.c_int32),
                ("lx", C.c_double), ("ly", C.c_double), ("lz", C.c_double),
                ("cs", C.c_double), ("nu", C.c_double), ("eta", C.c_double), ("dt", C.c_double),
                ("bext", C.c_double * 3), ("upwind", C.c_double)]


class _Forcing(C.Structure):
    _fields_ = [("k", C.c_int32 * 3), ("pad", C.c_int32), ("e", C.c_double * 3),
                ("phi", C.c_double), ("sigma", C.c_double), ("f0", C.c_double)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH) or os.path.getmtime(LIB_PATH) < os.path.getmtime(SRC_PATH):
            build()
        L = C.CDLL(LIB_PATH)
        dp = C.POINTER(C.c_double)
        L.ora_rhs.argtypes = [dp, C.POINTER(_Params), C.POINTER(_Forcing), dp, dp]
        L.ora_step.argtypes = [dp, C.POINTER(_Params), C.POINTER(_Forcing), C.c_int64, dp]
        L.ora_step_cells.argtypes = [dp, C.POINTER(_Params), C.POINTER(_Forcing), C.c_int64,
                                     C.POINTER(C.c_int64), dp]
        L.ora_terms_cells.argtypes = [dp, C.POINTER(_Params), C.POINTER(_Forcing), C.c_int64,
                                      C.POINTER(C.c_int64), dp]
        L.ora_deriv.argtypes = [dp, C.c_int, C.c_int, C.c_int, C.c_double, C.c_double,
                                C.c_double, C.c_int, C.c_int, C.c_int, C.c_int, dp]
        L.ora_forcing_field.argtypes = [C.POINTER(_Params), C.POINTER(_Forcing), dp]
        L.ora_diag.argtypes = [dp, C.POINTER(_Params), dp]
        L.ora_set_threads.argtypes = [C.c_int]
        L.ora_get_threads.restype = C.c_int
        _lib = L
    return _lib


def _dp(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _params(p) -> _Params:
    q = _Params()
    q.nx, q.ny, q.nz = p.nx, p.ny, p.nz
    q.lx, q.ly, q.lz = p.lx, p.ly, p.lz
    q.cs, q.nu, q.eta, q.dt = p.cs, p.nu, p.eta, p.dt
    for c in range(3):
        q.bext[c] = p.bext[c]
    q.upwind = float(getattr(p, "upwind", 0.0))
    return q


def _forcings(recs: Sequence) -> "C.Array":
    arr = (_Forcing * max(1, len(recs)))()
    for s, r in enumerate(recs):
        for c in range(3):
            arr[s].k[c] = int(r.k[c])
            arr[s].e[c] = float(r.e[c])
        arr[s].phi, arr[s].sigma, arr[s].f0 = float(r.phi), float(r.sigma), float(r.f0)
    return arr


def _state64(state: np.ndarray, p) -> np.ndarray:
    st = np.ascontiguousarray(state, dtype=np.float64)
    assert st.shape == (7, p.nz, p.ny, p.nx), st.shape
    return st


def set_threads(n: int) -> None:
    lib().ora_set_threads(int(n))


def get_threads() -> int:
    return int(lib().ora_get_threads())


def rhs(state, p, rec):
    """(R, termmax): R has the state's shape; termmax is (7, 7) largest |term| per field."""
    st = _state64(state, p)
    R = np.empty_like(st)
    tm = np.zeros(49)
    lib().ora_rhs(_dp(st), C.byref(_params(p)), _forcings([rec]), _dp(R), _dp(tm))
    return R, tm.reshape(7, 7)


def step(state, p, recs):
    """Advance ``len(recs)`` full RK3 steps.  Returns (new_state, tscale[nsteps, 7])."""
    st = _state64(state, p).copy()
    ts = np.zeros((len(recs), 7))
    rc = lib().ora_step(_dp(st), C.byref(_params(p)), _forcings(recs), len(recs), _dp(ts))
    if rc != 0:
        raise MemoryError("oracle step: allocation failed")
    return st, ts


def step_cells(state, p, rec, cells):
    """One RK3 step evaluated only at the given global linear cell indices -> (ncells, 7)."""
    st = _state64(state, p)
    cl = np.ascontiguousarray(cells, dtype=np.int64)
    out = np.empty((len(cl), 7))
    rc = lib().ora_step_cells(_dp(st), C.byref(_params(p)), _forcings([rec]), len(cl),
                              cl.ctypes.data_as(C.POINTER(C.c_int64)), _dp(out))
    if rc != 0:
        raise MemoryError("oracle step_cells: allocation failed")
    return out


def terms_cells(state, p, rec, cells):
    """(ncells, 7, 7): |term| per cell, field and term of the right-hand side at ``state``."""
    st = _state64(state, p)
    cl = np.ascontiguousarray(cells, dtype=np.int64)
    out = np.zeros((len(cl), 7, 7))
    lib().ora_terms_cells(_dp(st), C.byref(_params(p)), _forcings([rec]), len(cl),
                          cl.ctypes.data_as(C.POINTER(C.c_int64)), _dp(out))
    return out


def deriv(f, h, kind, a, b=0, wrap=True):
    """One derivative operator on a scalar array (nz, ny, nx): kind 1 d_a, 2 d_a^2, 3 d_a d_b."""
    g = np.ascontiguousarray(f, dtype=np.float64)
    nz, ny, nx = g.shape
    out = np.empty_like(g)
    lib().ora_deriv(_dp(g), nx, ny, nz, float(h[0]), float(h[1]), float(h[2]), int(kind),
                    int(a), int(b), 1 if wrap else 0, _dp(out))
    return out


def forcing_field(p, rec):
    """The forcing term of one record on the grid, shape (3, nz, ny, nx)."""
    out = np.empty((3, p.nz, p.ny, p.nx))
    lib().ora_forcing_field(C.byref(_params(p)), _forcings([rec]), _dp(out))
    return out


DIAG_KEYS = ("em", "ek", "urms", "brms", "umax", "lnrho_mean", "bx_mean", "by_mean",
             "bz_mean", "nonfinite")


def diag(state, p) -> dict:
    st = _state64(state, p)
    out = np.zeros(10)
    rc = lib().ora_diag(_dp(st), C.byref(_params(p)), _dp(out))
    if rc != 0:
        raise MemoryError("oracle diag: allocation failed")
    return dict(zip(DIAG_KEYS, out.tolist()))


def growth_rate(t, brms, i0=0, i1=None) -> float:
    """Least-squares slope of ln B_rms(t) over samples [i0, i1) (Section 5.1: B_rms ~ exp(lambda t)).

    Solved as the 2x2 normal equations in FP64 after centring t.
    """
    t = np.asarray(t, dtype=np.float64)[i0:i1]
    y = np.log(np.asarray(brms, dtype=np.float64)[i0:i1])
    tc = t - t.mean()
    return float(np.sum(tc * (y - y.mean())) / np.sum(tc * tc))


def magnetic_spectrum(state, p):
    """Shell spectrum E_B(k) of the discrete magnetic field (Section 5.3, power spectra).

    Follows the definition: B = curl A with the sixth-order first derivative (plus
    B_ext), its discrete Fourier transform B_hat(k) = sum_x B(x) exp(-i k.x) (a
    library FFT over the full grid), and the energy of every wavevector summed into
    the shell s with s - 1/2 <= |k|/dk < s + 1/2, dk = 2 pi / max(L).  Normalised
    so that sum_s E_B(s) dk = (1/2) int |B|^2 dV (volume integral, mu0 = 1):
    E_B(s) = V / (2 dk Ncell^2) * sum_{k in s} |B_hat(k)|^2.  The shell index is
    computed from m_a * (max(L) / L_a) in the order x, y, z, squared, summed, square
    root, + 1/2, floor, all in FP64.  Returns (E, dk).
    """
    st = _state64(state, p)
    h = (p.lx / p.nx, p.ly / p.ny, p.lz / p.nz)
    A = st[4:7]
    bext = tuple(getattr(p, "bext", (0.0, 0.0, 0.0)))
    B = np.empty_like(A)
    for c, (a, b) in enumerate(((1, 2), (2, 0), (0, 1))):
        # B_c = d_a A_b - d_b A_a for the cyclic triple (c, a, b)
        B[c] = deriv(A[b], h, 1, a) - deriv(A[a], h, 1, b) + bext[c]
    lmax = max(p.lx, p.ly, p.lz)
    dk = 2.0 * np.pi / lmax
    r = (lmax / p.lx, lmax / p.ly, lmax / p.lz)
    mz, my, mx = np.meshgrid(np.fft.fftfreq(p.nz, 1.0 / p.nz), np.fft.fftfreq(p.ny, 1.0 / p.ny),
                             np.fft.fftfreq(p.nx, 1.0 / p.nx), indexing="ij")
    q = (mx * r[0]) ** 2 + (my * r[1]) ** 2
    q = q + (mz * r[2]) ** 2
    shell = np.floor(np.sqrt(q) + 0.5).astype(np.int64)
    nshell = spectrum_nshell(p)
    power = np.zeros(shell.shape)
    for c in range(3):
        F = np.fft.fftn(B[c])
        power += F.real ** 2 + F.imag ** 2
    E = np.bincount(shell.ravel(), weights=power.ravel(), minlength=nshell)
    vol = p.lx * p.ly * p.lz
    ncell = float(p.nx * p.ny * p.nz)
    return E * (vol / (2.0 * dk * ncell * ncell)), dk


def spectrum_nshell(p) -> int:
    """Number of shells: the shell of the corner wavevector (n_a // 2 per axis), plus one."""
    lmax = max(p.lx, p.ly, p.lz)
    q = ((p.nx // 2) * (lmax / p.lx)) ** 2 + ((p.ny // 2) * (lmax / p.ly)) ** 2
    q = q + ((p.nz // 2) * (lmax / p.lz)) ** 2
    return int(np.floor(np.sqrt(q) + 0.5)) + 1


def spectral_growth_rate(t, ek, i0=0, i1=None) -> float:
    """Growth rate lambda_k of one spectral channel, E_B,k ~ exp(2 lambda_k t) (Section 5.1)."""
    return 0.5 * growth_rate(t, ek, i0, i1)


def tolerance_error(gpu, ora, tscale, dt):
    """Per-field error of one step: ||gpu - ora||_inf / max(||ora||_inf, dt * T_f).

    T_f is the sum over the field's RHS terms of max|term| (from ``step``).  Returns
    (e[7], plain[7]) where plain is ||gpu - ora||_inf / ||ora||_inf.
    """
    g = np.asarray(gpu, dtype=np.float64).reshape(7, -1)
    o = np.asarray(ora, dtype=np.float64).reshape(7, -1)
    d = np.max(np.abs(g - o), axis=1)
    n = np.max(np.abs(o), axis=1)
    den = np.maximum(n, dt * np.asarray(tscale))
    e = np.where(den > 0, d / np.where(den > 0, den, 1.0), d)
    plain = np.where(n > 0, d / np.where(n > 0, n, 1.0), d)
    return e, plain
