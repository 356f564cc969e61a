"""Python binding of ``libmhd.so``, the gfx950 solver for forced isothermal MHD.

Argument marshalling only: every step of the update runs in the HIP kernels of
the library.  Function names are those of the C ABI (``include/mhd.h``).  Device
buffers and streams may be given as torch tensors / ``torch.cuda.Stream``
objects or as raw integers (device pointers, hipStream_t).

Importing this module fails loudly if the library has not been built
(``python -m paper_2012_08758_amd.build``): there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass
from typing import List, Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmhd.so")

MHD_OK, MHD_E_INVALID, MHD_E_OOM, MHD_E_DEVICE, MHD_E_NONFINITE, MHD_E_BUSY, \
    MHD_E_UNSUPPORTED, MHD_E_NOTFOUND = range(8)
MHD_FP32, MHD_FP64 = 4, 8
FIELDS = ("lnrho", "ux", "uy", "uz", "ax", "ay", "az")
MHD_RUN_QUEUED, MHD_RUN_ACTIVE, MHD_RUN_DONE, MHD_RUN_FAILED = range(4)


class MhdError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"mhd status {status}: {msg}")
        self.status = status


class mhd_params(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32), ("precision", C.c_int32),
                ("lx", C.c_double), ("ly", C.c_double), ("lz", C.c_double), ("cs", C.c_double),
                ("nu", C.c_double), ("eta", C.c_double), ("dt", C.c_double), ("bext", C.c_double * 3),
                ("upwind", C.c_double)]


class mhd_forcing(C.Structure):
    _fields_ = [("k", C.c_int32 * 3), ("pad", C.c_int32), ("e", C.c_double * 3),
                ("phi", C.c_double), ("sigma", C.c_double), ("f0", C.c_double)]


class mhd_diag(C.Structure):
    _fields_ = [("step", C.c_int64), ("t", C.c_double), ("em", C.c_double), ("ek", C.c_double),
                ("urms", C.c_double), ("brms", C.c_double), ("umax", C.c_double),
                ("lnrho_mean", C.c_double), ("b_mean", C.c_double * 3), ("nonfinite", C.c_int64),
                ("t_device", C.c_double)]


class mhd_run_info(C.Structure):
    _fields_ = [("state", C.c_int32), ("precision", C.c_int32), ("steps_done", C.c_int64),
                ("steps_total", C.c_int64), ("t_submit", C.c_double), ("t_admit", C.c_double),
                ("t_done", C.c_double), ("em", C.c_double), ("brms", C.c_double)]


class mhd_server_stats(C.Structure):
    _fields_ = [("submitted", C.c_int64), ("admitted", C.c_int64), ("completed", C.c_int64),
                ("failed", C.c_int64), ("ticks", C.c_int64), ("step_samples", C.c_int64),
                ("lat_p50_ms", C.c_double), ("lat_p90_ms", C.c_double), ("lat_p99_ms", C.c_double),
                ("queue_p50_s", C.c_double), ("queue_p99_s", C.c_double),
                ("e2e_p50_s", C.c_double), ("e2e_p99_s", C.c_double),
                ("busy_s", C.c_double), ("wall_s", C.c_double), ("cell_substeps", C.c_double),
                ("hbm_in_use", C.c_size_t), ("hbm_peak", C.c_size_t)]


# exported symbol -> (restype, argtypes)
_P = C.c_void_p
_SIGS = {
    "mhd_create": (C.c_int, [C.POINTER(mhd_params), _P, C.POINTER(_P)]),
    "mhd_create_borrowed": (C.c_int, [C.POINTER(mhd_params), C.POINTER(_P), _P, C.POINTER(_P)]),
    "mhd_destroy": (C.c_int, [_P]),
    "mhd_set_field": (C.c_int, [_P, C.c_int, _P, C.c_int]),
    "mhd_get_field": (C.c_int, [_P, C.c_int, _P, C.c_int]),
    "mhd_init_seed": (C.c_int, [_P, C.c_uint64, C.c_double]),
    "mhd_set_forcing": (C.c_int, [_P, C.POINTER(mhd_forcing), C.c_int64]),
    "mhd_set_forcing_random": (C.c_int, [_P, C.c_double, C.c_double, C.c_double, C.c_uint64]),
    "mhd_clear_forcing": (C.c_int, [_P]),
    "mhd_step": (C.c_int, [_P, C.c_int64]),
    "mhd_reduce": (C.c_int, [_P]),
    "mhd_step_timed": (C.c_int, [_P, C.c_int64, C.POINTER(C.c_double), C.POINTER(C.c_double)]),
    "mhd_get_diag": (C.c_int, [_P, C.POINTER(mhd_diag), C.c_int64, C.POINTER(C.c_int64)]),
    "mhd_clear_diag": (C.c_int, [_P]),
    "mhd_get_time": (C.c_int, [_P, C.POINTER(C.c_int64), C.POINTER(C.c_double)]),
    "mhd_sync": (C.c_int, [_P]),
    "mhd_field_ptr": (C.c_int, [_P, C.c_int, C.POINTER(_P)]),
    "mhd_growth_rate": (C.c_int, [C.POINTER(mhd_diag), C.c_int64, C.c_int64, C.c_int64,
                                  C.POINTER(C.c_double)]),
    "mhd_spectrum": (C.c_int, [_P, C.POINTER(C.c_double), C.c_int32, C.POINTER(C.c_int32),
                               C.POINTER(C.c_double)]),
    "mhd_spectrum_noalloc": (C.c_int, [_P, _P, C.c_int32, C.POINTER(C.c_int32), C.POINTER(C.c_double)]),
    "mhd_spectrum_shells": (C.c_int, [C.POINTER(mhd_params), C.POINTER(C.c_int32),
                                      C.POINTER(C.c_double), C.POINTER(C.c_size_t)]),
    "mhd_channel_growth_rate": (C.c_int, [C.POINTER(C.c_double), C.POINTER(C.c_double), C.c_int64,
                                          C.POINTER(C.c_double)]),
    "mhd_last_error": (C.c_char_p, []),
    "mhd_forcing_draw": (C.c_int, [C.c_double, C.c_double, C.c_double, C.c_uint64, C.c_int64,
                                   C.POINTER(mhd_forcing)]),
    "mhd_num_tile_shapes": (C.c_int32, []),
    "mhd_tile_shape_name": (C.c_int, [C.c_int32, C.c_char_p, C.c_size_t]),
    "mhd_set_tile_shape": (C.c_int, [C.POINTER(mhd_params), C.c_int32]),
    "mhd_tile_config": (C.c_int, [C.POINTER(mhd_params), C.c_char_p, C.c_size_t]),
    "mhd_ctx_tile_config": (C.c_int, [_P, C.c_char_p, C.c_size_t]),
    "mhd_autotune": (C.c_int, [C.POINTER(mhd_params), C.c_int, _P, C.POINTER(C.c_double)]),
    "mhd_batch_create": (C.c_int, [C.POINTER(mhd_params), C.c_int32, _P, C.POINTER(_P)]),
    "mhd_batch_destroy": (C.c_int, [_P]),
    "mhd_batch_ctx": (C.c_int, [_P, C.c_int32, C.POINTER(_P)]),
    "mhd_batch_run": (C.c_int, [_P, C.c_int64, C.c_int]),
    "mhd_server_create": (C.c_int, [C.c_size_t, C.c_int32, C.c_int32, _P, C.POINTER(_P)]),
    "mhd_server_start": (C.c_int, [_P]),
    "mhd_server_submit": (C.c_int, [_P, C.POINTER(mhd_params), C.c_uint64, C.c_double, C.c_double,
                                    C.c_double, C.c_double, C.c_int64, C.c_int32,
                                    C.POINTER(C.c_int64)]),
    "mhd_server_poll": (C.c_int, [_P, C.c_int64, C.POINTER(mhd_run_info)]),
    "mhd_server_wait": (C.c_int, [_P, C.c_int64, C.c_double]),
    "mhd_server_get_field": (C.c_int, [_P, C.c_int64, C.c_int, _P]),
    "mhd_server_release": (C.c_int, [_P, C.c_int64]),
    "mhd_server_stats_get": (C.c_int, [_P, C.POINTER(mhd_server_stats)]),
    "mhd_server_stop": (C.c_int, [_P]),
    "mhd_server_destroy": (C.c_int, [_P]),
}
EXPORTS = tuple(_SIGS)


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(
            f"{LIB_PATH} is missing: build it with `python -m paper_2012_08758_amd.build` "
            "(there is no fallback implementation)")
    lib = C.CDLL(LIB_PATH)
    for name, (res, args) in _SIGS.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


lib = _load()


def _check(st: int):
    if st != MHD_OK:
        raise MhdError(st, lib.mhd_last_error().decode())


def _stream_handle(stream) -> Optional[int]:
    if stream is None:
        return None
    if isinstance(stream, int):
        return stream
    return int(stream.cuda_stream)  # torch.cuda.Stream


def _ptr(buf) -> int:
    if isinstance(buf, int):
        return buf
    return int(buf.data_ptr())  # torch tensor


def make_params(nx, ny=None, nz=None, *, nu, eta, dt=1e-3, cs=1.0, precision=MHD_FP64,
                lx=2 * np.pi, ly=2 * np.pi, lz=2 * np.pi, bext=(0.0, 0.0, 0.0), upwind=0.0) -> mhd_params:
    p = mhd_params()
    p.nx = nx
    p.ny = nx if ny is None else ny
    p.nz = nx if nz is None else nz
    p.precision = precision
    p.lx, p.ly, p.lz = lx, ly, lz
    p.cs, p.nu, p.eta, p.dt = cs, nu, eta, dt
    for a in range(3):
        p.bext[a] = bext[a]
    p.upwind = upwind
    return p


def params_from(rp) -> mhd_params:
    """From any object with the attributes of ``mhd_inputs.RunParams``."""
    return make_params(rp.nx, rp.ny, rp.nz, nu=rp.nu, eta=rp.eta, dt=rp.dt, cs=rp.cs,
                       precision=rp.precision, lx=rp.lx, ly=rp.ly, lz=rp.lz, bext=rp.bext,
                       upwind=getattr(rp, "upwind", 0.0))


def forcing_array(recs: Sequence) -> "C.Array":
    arr = (mhd_forcing * max(1, len(recs)))()
    for i, r in enumerate(recs):
        for a in range(3):
            arr[i].k[a] = int(r.k[a])
            arr[i].e[a] = float(r.e[a])
        arr[i].phi, arr[i].sigma, arr[i].f0 = float(r.phi), float(r.sigma), float(r.f0)
    return arr


# ---------------------------------------------------------------- C ABI, same names

def mhd_create(p: mhd_params, stream=None) -> int:
    h = _P()
    _check(lib.mhd_create(C.byref(p), _stream_handle(stream), C.byref(h)))
    return h.value


def mhd_create_borrowed(p: mhd_params, bufs: Sequence, stream=None) -> int:
    if len(bufs) != 14:
        raise ValueError("need 14 device buffers")
    arr = (_P * 14)(*[_ptr(b) for b in bufs])
    h = _P()
    _check(lib.mhd_create_borrowed(C.byref(p), arr, _stream_handle(stream), C.byref(h)))
    return h.value


def mhd_destroy(ctx: int) -> None:
    _check(lib.mhd_destroy(ctx))


def mhd_set_field(ctx: int, field: int, src, on_device: Optional[bool] = None) -> None:
    """src: numpy array (host, copied synchronously), torch tensor or device pointer."""
    if isinstance(src, np.ndarray):
        a = np.ascontiguousarray(src)
        _check(lib.mhd_set_field(ctx, field, a.ctypes.data, 0))
        return
    dev = True if on_device is None else on_device
    _check(lib.mhd_set_field(ctx, field, _ptr(src), 1 if dev else 0))


def mhd_get_field(ctx: int, field: int, dst, on_device: Optional[bool] = None) -> None:
    if isinstance(dst, np.ndarray):
        if not dst.flags.c_contiguous:
            raise ValueError("dst must be C-contiguous")
        _check(lib.mhd_get_field(ctx, field, dst.ctypes.data, 0))
        return
    dev = True if on_device is None else on_device
    _check(lib.mhd_get_field(ctx, field, _ptr(dst), 1 if dev else 0))


def mhd_init_seed(ctx: int, seed: int, a_noise: float) -> None:
    _check(lib.mhd_init_seed(ctx, seed, a_noise))


def mhd_set_forcing(ctx: int, recs: Sequence) -> None:
    arr = forcing_array(recs)
    _check(lib.mhd_set_forcing(ctx, arr, len(recs)))


def mhd_set_forcing_random(ctx: int, kf: float, f0: float, sigma: float, seed: int) -> None:
    _check(lib.mhd_set_forcing_random(ctx, kf, f0, sigma, seed))


def mhd_clear_forcing(ctx: int) -> None:
    _check(lib.mhd_clear_forcing(ctx))


def mhd_step(ctx: int, nsteps: int) -> None:
    _check(lib.mhd_step(ctx, nsteps))


def mhd_step_timed(ctx: int, nsteps: int):
    """(kernel_ms[4], step_ms[nsteps]): see the header."""
    k = (C.c_double * 4)()
    st = (C.c_double * max(1, nsteps))()
    _check(lib.mhd_step_timed(ctx, nsteps, k, st))
    return list(k), np.array(st[:nsteps])


def mhd_reduce(ctx: int) -> None:
    _check(lib.mhd_reduce(ctx))


def mhd_get_diag(ctx: int) -> List[dict]:
    n = C.c_int64()
    _check(lib.mhd_get_diag(ctx, None, 0, C.byref(n)))
    arr = (mhd_diag * max(1, n.value))()
    _check(lib.mhd_get_diag(ctx, arr, n.value, C.byref(n)))
    return [diag_dict(arr[i]) for i in range(n.value)]


def diag_dict(d: mhd_diag) -> dict:
    return dict(step=d.step, t=d.t, em=d.em, ek=d.ek, urms=d.urms, brms=d.brms, umax=d.umax,
                lnrho_mean=d.lnrho_mean, bx_mean=d.b_mean[0], by_mean=d.b_mean[1],
                bz_mean=d.b_mean[2], nonfinite=d.nonfinite, t_device=d.t_device)


def mhd_clear_diag(ctx: int) -> None:
    _check(lib.mhd_clear_diag(ctx))


def mhd_get_time(ctx: int):
    s, t = C.c_int64(), C.c_double()
    _check(lib.mhd_get_time(ctx, C.byref(s), C.byref(t)))
    return s.value, t.value


def mhd_sync(ctx: int) -> None:
    _check(lib.mhd_sync(ctx))


def mhd_field_ptr(ctx: int, field: int) -> int:
    p = _P()
    _check(lib.mhd_field_ptr(ctx, field, C.byref(p)))
    return p.value


def mhd_growth_rate(records: Sequence[dict], i0: int = 0, i1: Optional[int] = None) -> float:
    n = len(records)
    arr = (mhd_diag * max(1, n))()
    for i, r in enumerate(records):
        arr[i].t, arr[i].brms = r["t"], r["brms"]
    lam = C.c_double()
    _check(lib.mhd_growth_rate(arr, n, i0, n if i1 is None else i1, C.byref(lam)))
    return lam.value


def mhd_spectrum(ctx: int):
    """(E_B[nshell], dk) of the current state: see the header."""
    ns, dk = C.c_int32(), C.c_double()
    _check(lib.mhd_spectrum(ctx, None, 0, C.byref(ns), C.byref(dk)))
    out = (C.c_double * max(1, ns.value))()
    _check(lib.mhd_spectrum(ctx, out, ns.value, C.byref(ns), C.byref(dk)))
    return np.array(out[:ns.value]), dk.value


def mhd_spectrum_noalloc(ctx: int, out_dev: int, cap: int):
    """Spectrum into the device array out_dev (cap doubles) on the run's stream, using
    the library's static device scratch (no allocation, no synchronisation); returns
    (nshell, dk).  See the header."""
    ns, dk = C.c_int32(), C.c_double()
    _check(lib.mhd_spectrum_noalloc(ctx, out_dev, cap, C.byref(ns), C.byref(dk)))
    return ns.value, dk.value


def mhd_spectrum_shells(p: mhd_params):
    """(nshell, dk, workspace_bytes) for runs of this size (host-only)."""
    ns, dk, wb = C.c_int32(), C.c_double(), C.c_size_t()
    _check(lib.mhd_spectrum_shells(C.byref(p), C.byref(ns), C.byref(dk), C.byref(wb)))
    return ns.value, dk.value, wb.value


def mhd_channel_growth_rate(t: Sequence[float], e: Sequence[float]) -> float:
    ta = np.ascontiguousarray(t, dtype=np.float64)
    ea = np.ascontiguousarray(e, dtype=np.float64)
    if ta.shape != ea.shape:
        raise ValueError("t and e must have the same length")
    lam = C.c_double()
    _check(lib.mhd_channel_growth_rate(ta.ctypes.data_as(C.POINTER(C.c_double)),
                                       ea.ctypes.data_as(C.POINTER(C.c_double)), len(ta),
                                       C.byref(lam)))
    return lam.value


def mhd_forcing_draw(kf: float, f0: float, sigma: float, seed: int, n: int) -> mhd_forcing:
    out = mhd_forcing()
    _check(lib.mhd_forcing_draw(kf, f0, sigma, seed, n, C.byref(out)))
    return out


def mhd_num_tile_shapes() -> int:
    return int(lib.mhd_num_tile_shapes())


def mhd_tile_shape_name(i: int) -> str:
    buf = C.create_string_buffer(64)
    _check(lib.mhd_tile_shape_name(i, buf, 64))
    return buf.value.decode()


def mhd_set_tile_shape(p: mhd_params, i: int) -> None:
    _check(lib.mhd_set_tile_shape(C.byref(p), i))


def mhd_tile_config(p: mhd_params) -> str:
    buf = C.create_string_buffer(64)
    _check(lib.mhd_tile_config(C.byref(p), buf, 64))
    return buf.value.decode()


def mhd_ctx_tile_config(ctx: int) -> str:
    buf = C.create_string_buffer(64)
    _check(lib.mhd_ctx_tile_config(ctx, buf, 64))
    return buf.value.decode()


def mhd_autotune(p: mhd_params, reps: int = 3, stream=None) -> float:
    ms = C.c_double()
    _check(lib.mhd_autotune(C.byref(p), reps, _stream_handle(stream), C.byref(ms)))
    return ms.value


def mhd_batch_create(runs: Sequence[mhd_params], stream=None) -> int:
    arr = (mhd_params * len(runs))(*runs)
    h = _P()
    _check(lib.mhd_batch_create(arr, len(runs), _stream_handle(stream), C.byref(h)))
    return h.value


def mhd_batch_destroy(b: int) -> None:
    _check(lib.mhd_batch_destroy(b))


def mhd_batch_ctx(b: int, i: int) -> int:
    h = _P()
    _check(lib.mhd_batch_ctx(b, i, C.byref(h)))
    return h.value


def mhd_batch_run(b: int, nsteps: int, use_graph: bool = True) -> None:
    _check(lib.mhd_batch_run(b, nsteps, 1 if use_graph else 0))


def mhd_server_create(hbm_budget: int, max_slots: int, steps_per_tick: int = 1, stream=None) -> int:
    h = _P()
    _check(lib.mhd_server_create(hbm_budget, max_slots, steps_per_tick, _stream_handle(stream),
                                 C.byref(h)))
    return h.value


def mhd_server_start(s: int) -> None:
    _check(lib.mhd_server_start(s))


def mhd_server_submit(s: int, p: mhd_params, seed: int, a_noise: float, kf: float, f0: float,
                      sigma: float, nsteps: int, retain: bool = False) -> int:
    rid = C.c_int64()
    _check(lib.mhd_server_submit(s, C.byref(p), seed, a_noise, kf, f0, sigma, nsteps,
                                 1 if retain else 0, C.byref(rid)))
    return rid.value


def mhd_server_poll(s: int, rid: int) -> mhd_run_info:
    info = mhd_run_info()
    _check(lib.mhd_server_poll(s, rid, C.byref(info)))
    return info


def mhd_server_wait(s: int, rid: int, timeout_s: float = 600.0) -> None:
    _check(lib.mhd_server_wait(s, rid, timeout_s))


def mhd_server_get_field(s: int, rid: int, field: int, dst: np.ndarray) -> None:
    _check(lib.mhd_server_get_field(s, rid, field, dst.ctypes.data))


def mhd_server_release(s: int, rid: int) -> None:
    _check(lib.mhd_server_release(s, rid))


def mhd_server_stats_get(s: int) -> mhd_server_stats:
    st = mhd_server_stats()
    _check(lib.mhd_server_stats_get(s, C.byref(st)))
    return st


def mhd_server_stop(s: int) -> None:
    _check(lib.mhd_server_stop(s))


def mhd_server_destroy(s: int) -> None:
    _check(lib.mhd_server_destroy(s))


# ---------------------------------------------------------------- convenience

class Run:
    """One solver context with numpy in/out of the whole state (shape (7, nz, ny, nx))."""

    def __init__(self, p: mhd_params, stream=None):
        self.p = p
        self.dtype = np.float64 if p.precision == MHD_FP64 else np.float32
        self.h = mhd_create(p, stream)

    def close(self):
        if self.h:
            mhd_destroy(self.h)
            self.h = 0

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def set_state(self, st: np.ndarray):
        st = np.ascontiguousarray(st, dtype=self.dtype)
        assert st.shape == (7, self.p.nz, self.p.ny, self.p.nx), st.shape
        for f in range(7):
            mhd_set_field(self.h, f, st[f])

    def get_state(self) -> np.ndarray:
        out = np.empty((7, self.p.nz, self.p.ny, self.p.nx), dtype=self.dtype)
        for f in range(7):
            mhd_get_field(self.h, f, out[f])
        return out

    def step(self, n: int):
        mhd_step(self.h, n)

    def set_forcing(self, recs):
        mhd_set_forcing(self.h, recs)

    def diag(self):
        return mhd_get_diag(self.h)

    def spectrum(self):
        return mhd_spectrum(self.h)
