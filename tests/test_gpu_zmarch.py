"""The z-marching kernel with register queues (tile shape "32x8+zm") against the FP64
oracle, through the C ABI, every step from a shared state.

Bars as in test_gpu_parity: per field and step e_f <= 1e-12 (FP64), 1e-5 (FP32);
diagnostics to 1e-12 relative.  The grids exercise what is particular to this kernel:
a tile as wide as the grid (x and y halos wrapping more than once), z-segments whose
length is not a multiple of the six-step unroll and a ragged last segment, planes that
wrap in z at both ends of a segment, anisotropic spacing, an imposed field, helical and
non-helical forcing, upwinding, and the diagnostics fused into substep 1 plus the
diagnostics-only launch.
"""
import math

import numpy as np
import pytest

import mhd_inputs as mi
import oracle

pytestmark = pytest.mark.gpu

TOL = {8: 1e-12, 4: 1e-5}
ZM, ZMW = 14, 15     # 32x8 tiles; FP32 with substeps 1 and 2 on 64x8 tiles of 1024 threads


@pytest.fixture(scope="module")
def mhd():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2012_08758_amd as m
    return m


def _dtype(prec):
    return np.float64 if prec == 8 else np.float32


def _run(mhd, rp, st, recs, shape=ZM):
    p = mhd.params_from(rp)
    mhd.mhd_set_tile_shape(p, shape)
    want = "64x8+zm" if shape == ZMW and rp.precision == 4 and rp.nx % 64 == 0 else "32x8+zm"
    try:
        with mhd.Run(p) as run:
            assert mhd.mhd_ctx_tile_config(run.h) == want
            run.set_state(st)
            run.set_forcing(recs)
            outs = []
            for _ in recs:
                run.step(1)
                outs.append(run.get_state())
            mhd.mhd_reduce(run.h)
            diag = run.diag()
    finally:
        mhd.mhd_set_tile_shape(p, -1)
    return outs, diag


def _check(got, want, tscale, rp, label):
    e, plain = oracle.tolerance_error(got, want, tscale, rp.dt)
    print(f"{label}: e_f = " + " ".join(f"{n}:{x:.2e}" for n, x in zip(mi.FIELD_NAMES, e)), flush=True)
    assert np.all(e <= TOL[rp.precision]), (label, e, plain)


GRIDS = [
    # (nx, ny, nz), extra parameters
    ((32, 8, 13), dict(bext=(0.02, -0.01, 0.03))),                    # one tile: halos wrap twice
    ((64, 16, 20), dict(lx=5.0, ly=2 * math.pi, lz=4.0)),             # anisotropic spacing
    ((96, 24, 70), dict(bext=(0.0, 0.0, 0.05))),                      # one segment of 70 planes
    ((32, 16, 131), {}),                                              # segments of 66 and 65 planes
]


@pytest.mark.parametrize("prec", [8, 4])
@pytest.mark.parametrize("dims,kw", GRIDS, ids=[f"{d[0]}x{d[1]}x{d[2]}" for d, _ in GRIDS])
def test_zm_every_step(mhd, dims, kw, prec):
    rp = mi.RunParams(*dims, nu=3e-3, eta=2e-3, dt=1e-3, precision=prec, **kw)
    st = mi.noise_state(rp, 40 + dims[2], 0.2, 0.2, 0.2, dtype=_dtype(prec))
    recs = mi.forcing_schedule(7, 3, 3.0, 0.05, 1.0 if dims[0] != 64 else 0.0)
    got, diag = _run(mhd, rp, st, recs)
    inputs = [st.astype(np.float64)] + [g.astype(np.float64) for g in got]
    for n in range(3):
        want, ts = oracle.step(inputs[n], rp, [recs[n]])
        _check(got[n], want, ts[0], rp, f"zm {dims} fp{8 * prec} step {n + 1}")
    # the record of step n reduces that step's input state; the last one (mhd_reduce)
    # comes from the diagnostics-only launch
    assert len(diag) == 4
    for n, rec in enumerate(diag):
        ref = oracle.diag(inputs[n], rp)
        for k in ("em", "ek", "urms", "brms", "umax", "lnrho_mean"):
            assert abs(rec[k] - ref[k]) <= 1e-12 * max(abs(ref[k]), 1e-300), (n, k, rec[k], ref[k])
        for k in ("bx_mean", "by_mean", "bz_mean"):
            assert abs(rec[k] - ref[k]) <= 1e-12 * max(abs(ref[k]), 1e-3 * ref["brms"]), (n, k, rec[k], ref[k])
        assert rec["nonfinite"] == 0


@pytest.mark.parametrize("prec", [8, 4])
def test_zm_upwinding(mhd, prec):
    rp = mi.RunParams(64, 48, 40, nu=3e-3, eta=2e-3, dt=1e-3, precision=prec, upwind=1.0)
    st = mi.noise_state(rp, 95, 0.2, 0.3, 0.2, dtype=_dtype(prec))
    recs = mi.forcing_schedule(5, 2, 3.0, 0.05, 0.5)
    got, _ = _run(mhd, rp, st, recs)
    inputs = [st.astype(np.float64)] + [g.astype(np.float64) for g in got]
    for n in range(2):
        want, ts = oracle.step(inputs[n], rp, [recs[n]])
        _check(got[n], want, ts[0], rp, f"zm upwind fp{8 * prec} step {n + 1}")


WIDE_GRIDS = [
    ((64, 8, 13), dict(bext=(0.02, -0.01, 0.03))),                    # one 64-wide tile: halos wrap twice
    ((128, 16, 20), dict(lx=5.0, ly=2 * math.pi, lz=4.0)),            # anisotropic spacing
    ((192, 24, 70), dict(lx=6 * math.pi, bext=(0.0, 0.0, 0.05))),     # three tiles across, one segment
    ((64, 16, 131), {}),                                              # segments of 66 and 65 planes
]


@pytest.mark.parametrize("dims,kw", WIDE_GRIDS, ids=[f"{d[0]}x{d[1]}x{d[2]}" for d, _ in WIDE_GRIDS])
def test_zm_wide_every_step(mhd, dims, kw):
    """FP32 with substeps 1 and 2 on 64-wide tiles (substep 0 and its diagnostics on the
    32-wide ones), every step against the oracle."""
    rp = mi.RunParams(*dims, nu=3e-3, eta=2e-3, dt=1e-3, precision=4, **kw)
    st = mi.noise_state(rp, 70 + dims[2], 0.2, 0.2, 0.2, dtype=np.float32)
    recs = mi.forcing_schedule(8, 3, 3.0, 0.05, 1.0 if dims[0] != 128 else 0.0)
    got, diag = _run(mhd, rp, st, recs, ZMW)
    inputs = [st.astype(np.float64)] + [g.astype(np.float64) for g in got]
    for n in range(3):
        want, ts = oracle.step(inputs[n], rp, [recs[n]])
        _check(got[n], want, ts[0], rp, f"zm wide {dims} step {n + 1}")
    for n, rec in enumerate(diag):
        ref = oracle.diag(inputs[n], rp)
        for k in ("em", "ek", "urms", "brms", "umax", "lnrho_mean"):
            assert abs(rec[k] - ref[k]) <= 1e-12 * max(abs(ref[k]), 1e-300), (n, k, rec[k], ref[k])


def test_zm_wide_upwinding(mhd):
    rp = mi.RunParams(64, 48, 40, nu=3e-3, eta=2e-3, dt=1e-3, precision=4, upwind=1.0)
    st = mi.noise_state(rp, 96, 0.2, 0.3, 0.2, dtype=np.float32)
    recs = mi.forcing_schedule(6, 2, 3.0, 0.05, 0.5)
    got, _ = _run(mhd, rp, st, recs, ZMW)
    inputs = [st.astype(np.float64)] + [g.astype(np.float64) for g in got]
    for n in range(2):
        want, ts = oracle.step(inputs[n], rp, [recs[n]])
        _check(got[n], want, ts[0], rp, f"zm wide upwind step {n + 1}")


def test_zm_wide_and_narrow_tiles_agree_bit_for_bit(mhd):
    """The 64-wide and 32-wide FP32 kernels do the same arithmetic per cell in the same
    order, so the two tilings give the same bits."""
    rp = mi.RunParams(128, 32, 48, nu=3e-3, eta=2e-3, dt=1e-3, precision=4)
    st = mi.noise_state(rp, 5, 0.2, 0.2, 0.2, dtype=np.float32)
    recs = mi.forcing_schedule(9, 2, 3.0, 0.05, 1.0)
    a, _ = _run(mhd, rp, st, recs, ZM)
    b, _ = _run(mhd, rp, st, recs, ZMW)
    for n in range(2):
        assert np.array_equal(a[n], b[n]), n


def test_zm_counts_nonfinite_cells_once(mhd):
    """A cell whose flow and field values are both non-finite counts once (the two
    halves of a column are combined through LDS)."""
    rp = mi.RunParams(32, 8, 16, nu=1e-3, eta=1e-3, precision=8)
    st = mi.noise_state(rp, 1)
    st[2, 3, 4, 5] = np.nan       # u_y
    st[6, 3, 4, 5] = np.inf       # A_z of the same cell
    st[0, 0, 0, 0] = -np.inf      # ln rho of another cell
    st[5, 9, 7, 31] = np.nan      # A_y of a third
    p = mhd.params_from(rp)
    mhd.mhd_set_tile_shape(p, ZM)
    try:
        with mhd.Run(p) as run:
            run.set_state(st)
            mhd.mhd_reduce(run.h)
            assert run.diag()[-1]["nonfinite"] == 3
    finally:
        mhd.mhd_set_tile_shape(p, -1)
