"""Magnetic power spectrum on the GPU vs the oracle's, through the C ABI.

The oracle takes the definition literally (the discrete curl in real space, a library FFT
of the full grid, nearest-integer shells); the device path transforms A with its own FFT
and applies the curl as its Fourier symbol.  Bar, every shell s, both run precisions (the
spectrum is FP64 either way; FP32 runs start from FP32 values the oracle reads promoted
exactly):  |E_gpu(s) - E_oracle(s)| <= 1e-12 * sum_s E_oracle(s).  FFT roundoff is bounded
relative to the norm of the transformed data, about eps * log2(N) per transform, so three
passes at N <= 2048 stay below ~1e-14 of the total; a missing or misplaced mode is O(E_s).
"""
import math

import numpy as np
import pytest

import mhd_inputs as mi
import oracle

pytestmark = pytest.mark.gpu

TOL = 1e-12
TWO_PI = 2.0 * math.pi


@pytest.fixture(scope="module")
def mhd():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2012_08758_amd as m
    return m


def _dtype(prec):
    return np.float64 if prec == 8 else np.float32


def _check(got, dk, rp, st, label):
    want, dk_o = oracle.magnetic_spectrum(st.astype(np.float64), rp)
    assert len(got) == len(want) and dk == dk_o, (label, len(got), len(want), dk, dk_o)
    err = np.max(np.abs(got - want)) / np.sum(want)
    print(f"{label}: {len(got)} shells, max |dE| / sum E = {err:.2e}", flush=True)
    assert err <= TOL, (label, err)


GRIDS = [
    ((32, 32, 32), {}),
    ((48, 40, 36), dict(lx=5.0, ly=TWO_PI, lz=4.0, bext=(0.1, -0.2, 0.05))),
    ((45, 28, 50), {}),
    ((8, 8, 8), dict(bext=(0.0, 0.0, 0.3))),
    ((2048, 8, 8), {}),        # longest x lines: one complex line per block, 1025 shells
    ((8, 1536, 8), {}),        # radix-3 stage on long y lines
    ((12, 8, 1050), {}),       # radices 2, 3, 5, 7 on long z lines
]


@pytest.mark.parametrize("prec", [8, 4])
@pytest.mark.parametrize("dims,kw", GRIDS, ids=[f"{d[0]}x{d[1]}x{d[2]}" for d, _ in GRIDS])
def test_spectrum_parity(mhd, dims, kw, prec):
    rp = mi.RunParams(*dims, nu=1e-3, eta=1e-3, precision=prec, **kw)
    st = mi.noise_state(rp, 11, 0.1, 0.1, 0.3, dtype=_dtype(prec))
    with mhd.Run(mhd.params_from(rp)) as run:
        run.set_state(st)
        got, dk = run.spectrum()
        again, _ = run.spectrum()
    assert np.array_equal(got, again)  # fixed-order sums: bit-reproducible
    _check(got, dk, rp, st, f"spectrum {dims} fp{8 * prec}")


@pytest.mark.parametrize("prec", [8, 4])
def test_spectrum_of_an_evolved_forced_state(mhd, prec):
    rp = mi.RunParams(48, 48, 48, nu=5e-3, eta=5e-3, precision=prec)
    st = mi.noise_state(rp, 4, 0.05, 0.2, 0.2, dtype=_dtype(prec))
    with mhd.Run(mhd.params_from(rp)) as run:
        run.set_state(st)
        run.set_forcing(mi.forcing_schedule(2, 5, 3.0, 0.05, 1.0))
        run.step(5)
        cur = run.get_state()
        got, dk = run.spectrum()
    _check(got, dk, rp, cur, f"evolved 48^3 fp{8 * prec}")


def test_channel_growth_rate_of_a_decaying_beltrami_field(mhd):
    """Spectra taken on the device after every step: the channel k of a decaying Beltrami
    field falls as |G(-eta k2^2 dt)|^2 per step, so lambda_k = ln|G| / dt, equal to the
    B_rms rate from the diagnostics (the factor 2 of E_B,k ~ exp(2 lambda_k t))."""
    rp = mi.RunParams(8, 8, 32, nu=0.1, eta=0.1, dt=0.02, precision=8)
    z = np.arange(32) * (TWO_PI / 32)
    k = 2
    st = np.zeros((7, 32, 8, 8))
    st[4] = (np.sin(k * z) / k)[:, None, None]
    st[5] = (np.cos(k * z) / k)[:, None, None]
    ts, ek = [], []
    with mhd.Run(mhd.params_from(rp)) as run:
        run.set_state(st)
        for n in range(8):
            ts.append(n * rp.dt)
            ek.append(run.spectrum()[0][k])
            run.step(1)
        mhd.mhd_reduce(run.h)
        diag = run.diag()
    w = k * TWO_PI / 32
    k2 = (3 * (1 - math.cos(w)) - 0.3 * (1 - math.cos(2 * w)) + (1 - math.cos(3 * w)) / 45) / (TWO_PI / 32) ** 2
    zz = -rp.eta * k2 * rp.dt
    lam = math.log(abs(1 + zz + zz * zz / 2 + zz ** 3 / 6)) / rp.dt
    assert abs(mhd.mhd_channel_growth_rate(ts, ek) - lam) < 1e-10
    assert abs(mhd.mhd_growth_rate(diag) - lam) < 1e-10


def test_spectrum_of_batched_runs(mhd):
    """Spectra of runs advanced together in one graph-replayed batch (mixed sizes and
    precisions) match the oracle's spectra of their states."""
    specs = [mi.RunParams(16, 16, 16, nu=5e-3, eta=5e-3, precision=8),
             mi.RunParams(24, 20, 16, nu=2e-3, eta=2e-3, precision=8, upwind=1.0),
             mi.RunParams(32, 32, 32, nu=1e-3, eta=1e-3, precision=4)]
    b = mhd.mhd_batch_create([mhd.params_from(rp) for rp in specs])
    try:
        ctxs = [mhd.mhd_batch_ctx(b, i) for i in range(len(specs))]
        for i, (c, rp) in enumerate(zip(ctxs, specs)):
            st = mi.noise_state(rp, 60 + i, 0.05, 0.1, 0.2, dtype=_dtype(rp.precision))
            for f in range(7):
                mhd.mhd_set_field(c, f, np.ascontiguousarray(st[f]))
            mhd.mhd_set_forcing(c, mi.forcing_schedule(70 + i, 6, 3.0, 0.05, float(i % 2)))
        mhd.mhd_batch_run(b, 6, True)
        for i, (c, rp) in enumerate(zip(ctxs, specs)):
            got = np.empty((7, rp.nz, rp.ny, rp.nx), dtype=_dtype(rp.precision))
            for f in range(7):
                mhd.mhd_get_field(c, f, got[f])
            E, dk = mhd.mhd_spectrum(c)
            _check(E, dk, rp, got, f"batch run {i}")
    finally:
        mhd.mhd_batch_destroy(b)


# ------------------------------------------------------------------ full size (512^3)

def test_full_size_beltrami_spectrum_fp64(mhd):
    """512^3 FP64, A = (sin 5z, cos 5z, 0)/5: the whole energy (1/2) V (k_eff/5)^2 in shell 5."""
    n, k = 512, 5
    rp = mi.RunParams(n, n, n, nu=4e-4, eta=4e-4, precision=8)
    z = np.arange(n) * (TWO_PI / n)
    with mhd.Run(mhd.params_from(rp)) as run:
        mhd.mhd_init_seed(run.h, 0, 0.0)
        mhd.mhd_set_field(run.h, 4, np.ascontiguousarray(
            np.broadcast_to((np.sin(k * z) / k)[:, None, None], (n, n, n))))
        mhd.mhd_set_field(run.h, 5, np.ascontiguousarray(
            np.broadcast_to((np.cos(k * z) / k)[:, None, None], (n, n, n))))
        got, dk = run.spectrum()
    h = TWO_PI / n
    w = k * h
    keff = (1.5 * math.sin(w) - 0.3 * math.sin(2 * w) + math.sin(3 * w) / 30.0) / h
    want = 0.5 * TWO_PI ** 3 * (keff / k) ** 2
    print(f"512^3 Beltrami: E[5] rel err {abs(got[k] - want) / want:.2e}, "
          f"max other {np.max(np.abs(np.delete(got, k))) / want:.2e}", flush=True)
    assert dk == 1.0 and len(got) == oracle.spectrum_nshell(rp)
    assert abs(got[k] - want) <= TOL * want
    assert np.max(np.abs(np.delete(got, k))) <= TOL * want


@pytest.mark.parametrize("prec", [8, 4])
def test_full_size_parseval_against_the_energy_diagnostic(mhd, prec):
    """512^3 seed field (A noise 1e-5) plus B_ext: sum_s E(s) dk = V E_M, with E_M the
    device's real-space FP64 diagnostic (itself checked against the oracle)."""
    n = 512
    rp = mi.RunParams(n, n, n, nu=4e-4, eta=4e-4, precision=prec, bext=(1e-5, 0.0, -2e-5))
    with mhd.Run(mhd.params_from(rp)) as run:
        mhd.mhd_init_seed(run.h, 3, 1e-5)
        got, dk = run.spectrum()
        mhd.mhd_reduce(run.h)
        em = run.diag()[-1]["em"]
    vol = TWO_PI ** 3
    err = abs(np.sum(got) * dk - vol * em) / (vol * em)
    print(f"512^3 fp{8 * prec} Parseval: rel err {err:.2e}", flush=True)
    assert err <= TOL
    assert abs(got[0] - 0.5 * vol * (1e-10 + 4e-10)) <= 1e-12 * vol * em
