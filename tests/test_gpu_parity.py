"""HIP path vs the FP64 oracle, through the C ABI, on seeded inputs.

Bars (per field f, per step, from the same input state and forcing records):
    e_f = ||gpu - oracle||_inf / max(||oracle||_inf, dt * T_f)  <= 1e-12 (FP64), 1e-5 (FP32)
with T_f the sum over the field's right-hand-side terms of max|term| (the scale that
roundoff of one step is relative to).  FP32 runs start from FP32 values, which the
oracle reads promoted exactly to FP64.  Diagnostics (FP64 sums at both precisions)
must agree to 1e-12 relative.
"""
import math

import numpy as np
import pytest

import mhd_inputs as mi
import oracle

pytestmark = pytest.mark.gpu

TOL = {8: 1e-12, 4: 1e-5}


@pytest.fixture(scope="module")
def mhd():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2012_08758_amd as m
    return m


def _dtype(prec):
    return np.float64 if prec == 8 else np.float32


def gpu_run(mhd, rp, state, recs, per_step=False, shape=None):
    """Run len(recs) steps on the GPU.  Returns the list of states after each step
    (per_step) or the final state, plus the diagnostic records."""
    p = mhd.params_from(rp)
    if shape is not None:
        mhd.mhd_set_tile_shape(p, shape)
    try:
        with mhd.Run(p) as run:
            run.set_state(state.astype(_dtype(rp.precision)))
            run.set_forcing(recs)
            outs = []
            if per_step:
                for _ in recs:
                    run.step(1)
                    outs.append(run.get_state())
            else:
                run.step(len(recs))
                outs.append(run.get_state())
            mhd.mhd_reduce(run.h)
            diag = run.diag()
    finally:
        if shape is not None:
            mhd.mhd_set_tile_shape(p, -1)
    return outs, diag


def check_step(got, want, tscale, rp, label):
    e, plain = oracle.tolerance_error(got, want, tscale, rp.dt)
    print(f"{label}: e_f = " + " ".join(f"{n}:{x:.2e}" for n, x in zip(mi.FIELD_NAMES, e)), flush=True)
    assert np.all(e <= TOL[rp.precision]), (label, e, plain)
    return e


def oracle_per_step(st, rp, recs):
    outs, scales = [], []
    cur = st.astype(np.float64)
    for r in recs:
        cur, ts = oracle.step(cur, rp, [r])
        outs.append(cur)
        scales.append(ts[0])
    return outs, scales


# ------------------------------------------------------------------ small grids, every step

@pytest.mark.parametrize("prec", [8, 4])
def test_config1_32cubed_every_step(mhd, prec):
    """32^3, nu = eta = 5e-3, non-helical forcing kf = 3, f0 = 0.02, A noise 1e-5, 20 steps.

    Every step is checked from a shared state: the oracle advances the GPU's own state
    of the previous step (FP32 values promoted exactly to FP64) with the same record.
    The diagnostic record of step n is the FP64 reduction of that step's input state,
    so it must equal the oracle's reduction of the same state to 1e-12 at either
    precision (FP32 states are reduced in FP64, with an FP64 curl, on the device)."""
    rp = mi.RunParams(32, 32, 32, nu=5e-3, eta=5e-3, dt=1e-3, precision=prec)
    st = mi.ic_seed_noise(rp, 0, 1e-5, dtype=_dtype(prec))
    recs = mi.forcing_schedule(0, 20, 3.0, 0.02, 0.0)
    got, diag = gpu_run(mhd, rp, st, recs, per_step=True)
    inputs = [st.astype(np.float64)] + [g.astype(np.float64) for g in got]
    for n in range(20):
        want, ts = oracle.step(inputs[n], rp, [recs[n]])
        check_step(got[n], want, ts[0], rp, f"cfg1 fp{8 * prec} step {n + 1}")
    # the whole 20-step trajectory stays within the per-step bar of the oracle's own one
    traj, tsc = oracle_per_step(st, rp, recs)
    check_step(got[-1], traj[-1], tsc[-1], rp, f"cfg1 fp{8 * prec} trajectory")
    # diagnostics of the input state of every step, and of the final state
    assert len(diag) == 21
    for n, rec in enumerate(diag):
        ref = oracle.diag(inputs[n], rp)
        assert rec["step"] == n and abs(rec["t"] - n * rp.dt) < 1e-15
        for k in ("em", "ek", "urms", "brms", "umax"):
            assert abs(rec[k] - ref[k]) <= 1e-12 * abs(ref[k]) + 1e-300, (n, k, rec[k], ref[k])
        assert rec["nonfinite"] == 0


@pytest.mark.parametrize("shape", range(14))
def test_every_tile_shape_ragged_grid_fp64(mhd, shape):
    rp = mi.RunParams(20, 18, 13, nu=4e-3, eta=6e-3, dt=1e-3, precision=8, bext=(0.01, 0.0, -0.02))
    st = mi.noise_state(rp, 5 + shape, 0.2, 0.2, 0.2)
    recs = mi.forcing_schedule(3, 2, 3.0, 0.05, 1.0)
    got, _ = gpu_run(mhd, rp, st, recs, per_step=True, shape=shape)
    want, scales = oracle_per_step(st, rp, recs)
    for n in range(2):
        check_step(got[n], want[n], scales[n], rp, f"shape {shape} step {n + 1}")


@pytest.mark.parametrize("shape", [0, 3, 5, 6, 8, 9, 11])
def test_tile_shapes_fp32(mhd, shape):
    rp = mi.RunParams(24, 20, 17, nu=4e-3, eta=6e-3, dt=1e-3, precision=4)
    st = mi.noise_state(rp, 7, 0.2, 0.2, 0.2, dtype=np.float32)
    recs = mi.forcing_schedule(4, 2, 3.0, 0.05, 0.5)
    got, _ = gpu_run(mhd, rp, st, recs, per_step=True, shape=shape)
    want, scales = oracle_per_step(st, rp, recs)
    for n in range(2):
        check_step(got[n], want[n], scales[n], rp, f"fp32 shape {shape} step {n + 1}")


@pytest.mark.parametrize("prec", [8, 4])
@pytest.mark.parametrize("grid", [(8, 8, 8), (12, 8, 8)])
@pytest.mark.parametrize("shape", [7, 10, 11])
def test_wide_ring_tiles_on_narrow_grids(mhd, shape, grid, prec):
    """Ring tiles 32 cells wide on grids of 8 and 12 points in x: one tile spans the
    periodic x axis several times, so the copies of the s-2 state and of the forcing
    slots wrap x more than once."""
    rp = mi.RunParams(*grid, nu=4e-3, eta=3e-3, dt=1e-3, precision=prec)
    st = mi.noise_state(rp, 200 + shape, 0.2, 0.2, 0.2, dtype=_dtype(prec))
    recs = mi.forcing_schedule(9, 2, 3.0, 0.05, 1.0)
    got, _ = gpu_run(mhd, rp, st, recs, per_step=True, shape=shape)
    cur = st.astype(np.float64)
    for n in range(2):
        want, ts = oracle.step(cur, rp, [recs[n]])
        check_step(got[n], want, ts[0], rp, f"shape {shape} grid {grid} fp{8 * prec} step {n + 1}")
        cur = got[n].astype(np.float64)


@pytest.mark.parametrize("prec", [8, 4])
@pytest.mark.parametrize("shape", range(6, 14))
def test_ring_shapes_wrap_once(mhd, shape, prec):
    """Ring kernels on a grid larger than their halo box (single-wrap offsets)."""
    rp = mi.RunParams(48, 40, 32, nu=3e-3, eta=2e-3, dt=1e-3, precision=prec)
    st = mi.noise_state(rp, 60 + shape, 0.2, 0.2, 0.2, dtype=_dtype(prec))
    recs = mi.forcing_schedule(8, 2, 3.0, 0.05, 1.0)
    got, _ = gpu_run(mhd, rp, st, recs, per_step=True, shape=shape)
    want, scales = oracle_per_step(st, rp, recs)
    for n in range(2):
        check_step(got[n], want[n], scales[n], rp, f"ring shape {shape} fp{8 * prec} step {n + 1}")


@pytest.mark.parametrize("prec", [8, 4])
@pytest.mark.parametrize("shape", [12, 13])
def test_march_shapes_several_slabs(mhd, shape, prec):
    """z-marching kernel on 64x48x40: two z-segments of five slabs per column (the first
    slab, steady slabs and the prefetch past a segment's end); every step and the
    diagnostics of the shared input state against the oracle, then a diagnostics-only
    launch on a later state."""
    rp = mi.RunParams(64, 48, 40, nu=3e-3, eta=2e-3, dt=1e-3, precision=prec, bext=(0.0, 0.02, 0.0))
    st = mi.noise_state(rp, 80 + shape, 0.2, 0.2, 0.2, dtype=_dtype(prec))
    recs = mi.forcing_schedule(9, 3, 3.0, 0.05, 1.0)
    got, diag = gpu_run(mhd, rp, st, recs, per_step=True, shape=shape)
    want, scales = oracle_per_step(st, rp, recs)
    for n in range(3):
        check_step(got[n], want[n], scales[n], rp, f"march shape {shape} fp{8 * prec} step {n + 1}")
    ref = oracle.diag(st.astype(np.float64), rp)
    for k in ("em", "ek", "urms", "brms", "umax"):
        assert abs(diag[0][k] - ref[k]) <= 1e-12 * abs(ref[k]), (k, diag[0][k], ref[k])
    p = mhd.params_from(rp)
    mhd.mhd_set_tile_shape(p, shape)
    try:
        with mhd.Run(p) as run:
            run.set_state(got[-1])
            mhd.mhd_reduce(run.h)
            rec = run.diag()[-1]
    finally:
        mhd.mhd_set_tile_shape(p, -1)
    ref = oracle.diag(got[-1].astype(np.float64), rp)
    for k in ("em", "ek", "urms", "brms", "umax", "lnrho_mean"):
        assert abs(rec[k] - ref[k]) <= 1e-12 * max(abs(ref[k]), 1e-300), (k, rec[k], ref[k])


@pytest.mark.parametrize("prec", [8, 4])
@pytest.mark.parametrize("shape", [0, 9, 10, 12, 13])
def test_upwinding_parity(mhd, shape, prec):
    """Upwinding of the continuity advection on (staged, ring CZ=2, ring, marching)
    kernels: two steps against the oracle, with rough ln rho and u so that the
    sixth-difference correction is far from negligible."""
    rp = mi.RunParams(64, 48, 40, nu=3e-3, eta=2e-3, dt=1e-3, precision=prec, upwind=1.0)
    st = mi.noise_state(rp, 90 + shape, 0.2, 0.3, 0.2, dtype=_dtype(prec))
    recs = mi.forcing_schedule(5, 2, 3.0, 0.05, 0.5)
    got, _ = gpu_run(mhd, rp, st, recs, per_step=True, shape=shape)
    want, scales = oracle_per_step(st, rp, recs)
    for n in range(2):
        check_step(got[n], want[n], scales[n], rp, f"upwind shape {shape} fp{8 * prec} step {n + 1}")
    # and the term is really there: the step without it differs well beyond the bar
    q = mi.RunParams(64, 48, 40, nu=3e-3, eta=2e-3, dt=1e-3, precision=prec)
    plain, _ = oracle.step(st.astype(np.float64), q, recs[:1])
    e, _ = oracle.tolerance_error(plain, want[0], scales[0], rp.dt)
    assert e[0] > 100 * TOL[prec], e


@pytest.mark.parametrize("n", [8, 9, 33])
def test_small_and_odd_grids(mhd, n):
    """Grids smaller than a tile (the halo wraps more than once) and odd sizes."""
    rp = mi.RunParams(n, n, n, nu=1e-2, eta=1e-2, dt=1e-3, precision=8)
    st = mi.smooth_state(rp, 2, kmax=2)
    recs = mi.forcing_schedule(9, 3, 3.0, 0.02, 1.0)
    got, _ = gpu_run(mhd, rp, st, recs, per_step=True)
    want, scales = oracle_per_step(st, rp, recs)
    for k in range(3):
        check_step(got[k], want[k], scales[k], rp, f"{n}^3 step {k + 1}")


def test_forcing_off_and_bext_alfven_state(mhd):
    """No forcing records (f0 = 0) and an imposed field: exercises the Lorentz/induction pair."""
    rp = mi.RunParams(16, 16, 32, nu=1e-2, eta=1e-2, dt=1e-2, precision=8, bext=(0.0, 0.0, 1.0))
    st = mi.smooth_state(rp, 12, kmax=3, amp_lnrho=0.05, amp_u=0.1, amp_a=0.1)
    recs = mi.no_forcing(4)
    got, _ = gpu_run(mhd, rp, st, recs, per_step=True)
    want, scales = oracle_per_step(st, rp, recs)
    for k in range(4):
        check_step(got[k], want[k], scales[k], rp, f"bext step {k + 1}")


# ------------------------------------------------------------------ full sizes, sampled

def _sample_cells(rp, n, seed):
    rng = np.random.default_rng(seed)
    cells = rng.integers(0, rp.ncell, size=n)
    # faces, edges and corners of the periodic box
    corners = []
    for x in (0, rp.nx - 1):
        for y in (0, rp.ny - 1):
            for z in (0, rp.nz - 1):
                corners.append(x + rp.nx * (y + rp.ny * z))
    return np.unique(np.concatenate([cells, corners]))


@pytest.mark.parametrize("n,prec,sigma,nu", [(256, 8, 1.0, 1e-3), (512, 8, 0.0, 4e-4), (512, 4, 0.0, 4e-4)])
def test_full_size_sampled_one_step(mhd, n, prec, sigma, nu):
    """256^3 (helical, nu = eta = 1e-3) and 512^3 (non-helical, 4e-4) in FP64 and FP32, in
    the launch configuration the benchmark uses: one step from a seeded state, compared
    with the oracle's step at sampled cells (its dependency cone, evaluated cell by cell)."""
    rp = mi.RunParams(n, n, n, nu=nu, eta=nu, dt=1e-3, precision=prec)
    print(f"generating {n}^3 state", flush=True)
    st = mi.noise_state(rp, 21, 0.05, 0.05, 0.05, dtype=_dtype(prec))
    rec = mi.forcing_schedule(0, 1, 3.0, 0.02, sigma)[0]
    got, _ = gpu_run(mhd, rp, st, [rec])
    got = got[0].reshape(7, -1)
    cells = _sample_cells(rp, 400, n)
    st64 = st.astype(np.float64) if prec == 4 else st
    want = oracle.step_cells(st64, rp, rec, cells)
    terms = oracle.terms_cells(st64, rp, rec, cells).max(axis=0).sum(axis=1)
    g = got[:, cells].T.astype(np.float64)
    d = np.abs(g - want).max(axis=0)
    den = np.maximum(np.abs(want).max(axis=0), rp.dt * terms)
    e = d / den
    print(f"{n}^3 fp{8 * prec} sampled e_f: " + " ".join(f"{x:.2e}" for x in e), flush=True)
    assert np.all(e <= TOL[prec]), e


@pytest.mark.parametrize("prec", [8, 4])
def test_full_size_band_every_cell(mhd, prec):
    """512^3 FP64 and FP32 in the benchmark's launch configuration (FP32: substeps 2 and 3
    on the 64-wide tiles): one step from a seeded state,
    compared on EVERY cell of a 16-plane z-band (4.2 M cells, all x and y, so every tile
    column including the ones that wrap in x, and the band crosses a z-segment boundary
    of the z-marching kernel at z = 256).  The oracle steps a periodic 34-plane slab cut
    from the same input state (the band plus 9 planes on each side: three substeps of a
    radius-3 stencil reach 9 planes, so the slab's artificial z wrap cannot reach the
    band).  The forcing record is the first draw of the schedule with k_z = 0, whose
    forcing does not depend on z, so that the slab sees the same forcing."""
    n, z0, band, halo = 512, 248, 16, 9
    rp = mi.RunParams(n, n, n, nu=4e-4, eta=4e-4, dt=1e-3, precision=prec)
    rec = next(r for r in mi.forcing_schedule(0, 200, 3.0, 0.02, 0.0) if r.k[2] == 0)
    print(f"generating {n}^3 state", flush=True)
    st = mi.noise_state(rp, 23, 0.05, 0.05, 0.05, dtype=_dtype(prec))
    print("one GPU step", flush=True)
    got, _ = gpu_run(mhd, rp, st, [rec])
    got = got[0]
    print(f"tile config {mhd.mhd_tile_config(mhd.params_from(rp))}; oracle on the slab", flush=True)
    nzs = band + 2 * halo
    planes = [(z0 - halo + j) % n for j in range(nzs)]
    slab = np.ascontiguousarray(st[:, planes]).astype(np.float64)
    del st
    h = rp.lz / n
    sp = mi.RunParams(n, n, nzs, nu=rp.nu, eta=rp.eta, dt=rp.dt, precision=8, lz=nzs * h)
    want, ts = oracle.step(slab, sp, [rec])
    want = want[:, halo:halo + band]
    g = got[:, z0:z0 + band]
    e, _ = oracle.tolerance_error(g, want, ts[0], rp.dt)
    print(f"512^3 fp{8 * prec} band of 16 planes, every cell: e_f = " +
          " ".join(f"{k}:{x:.2e}" for k, x in zip(mi.FIELD_NAMES, e)), flush=True)
    assert np.all(e <= TOL[prec]), e


@pytest.mark.parametrize("n,prec,sigma,nu,checks", [(256, 8, 1.0, 1e-3, (100, 200)),
                                                    (512, 8, 0.0, 4e-4, (100,)), (512, 4, 0.0, 4e-4, (100,))])
def test_full_size_sampled_later_steps(mhd, n, prec, sigma, nu, checks):
    """The 256^3 and 512^3 workloads from their seed field (A noise 1e-5) under the
    forcing schedule, advanced on the GPU: at steps 100 (and 200) the step is checked
    against the oracle's step from the GPU's own state before it, at sampled cells."""
    rp = mi.RunParams(n, n, n, nu=nu, eta=nu, dt=1e-3, precision=prec)
    recs = mi.forcing_schedule(0, max(checks), 3.0, 0.02, sigma)
    cells = _sample_cells(rp, 300, n + 1)
    with mhd.Run(mhd.params_from(rp)) as run:
        mhd.mhd_init_seed(run.h, 0, 1e-5)
        run.set_forcing(recs)
        done = 0
        for c in checks:
            run.step(c - 1 - done)
            before = run.get_state()
            run.step(1)
            done = c
            got = run.get_state().reshape(7, -1)[:, cells].T.astype(np.float64)
            st64 = before.astype(np.float64)
            del before
            want = oracle.step_cells(st64, rp, recs[c - 1], cells)
            terms = oracle.terms_cells(st64, rp, recs[c - 1], cells).max(axis=0).sum(axis=1)
            del st64
            e = np.abs(got - want).max(axis=0) / np.maximum(np.abs(want).max(axis=0), rp.dt * terms)
            print(f"{n}^3 fp{8 * prec} step {c} sampled e_f: " + " ".join(f"{x:.2e}" for x in e), flush=True)
            assert np.all(e <= TOL[prec]), (c, e)


# ------------------------------------------------------------------ diagnostics

@pytest.mark.parametrize("prec", [8, 4])
def test_diagnostics_match_oracle(mhd, prec):
    rp = mi.RunParams(24, 20, 16, nu=1e-3, eta=1e-3, dt=1e-3, precision=prec, bext=(0.1, 0.0, 0.0))
    st = mi.noise_state(rp, 31, 0.3, 0.3, 0.3, dtype=_dtype(prec))
    with mhd.Run(mhd.params_from(rp)) as run:
        run.set_state(st)
        mhd.mhd_reduce(run.h)
        rec = run.diag()[-1]
    ref = oracle.diag(st.astype(np.float64), rp)
    for k in ("em", "ek", "urms", "brms", "umax", "lnrho_mean", "bx_mean", "by_mean", "bz_mean"):
        scale = max(abs(ref[k]), 1e-3 * ref["brms"] if k.startswith("b") else abs(ref[k]))
        assert abs(rec[k] - ref[k]) <= 1e-12 * max(scale, 1e-300), (k, rec[k], ref[k])
    assert rec["nonfinite"] == 0


def test_nonfinite_cells_are_counted(mhd):
    rp = mi.RunParams(16, 16, 16, nu=1e-3, eta=1e-3, precision=8)
    st = mi.noise_state(rp, 1)
    st[2, 3, 4, 5] = np.nan
    st[6, 0, 0, 0] = np.inf
    st[6, 1, 0, 0] = -np.inf
    with mhd.Run(mhd.params_from(rp)) as run:
        run.set_state(st)
        mhd.mhd_reduce(run.h)
        assert run.diag()[-1]["nonfinite"] == 3


def test_beltrami_growth_rate_on_gpu(mhd):
    """Decaying Beltrami field: B_rms falls by |G(-eta k2^2 dt)| per step exactly; the GPU's
    FP64 series and host fit give lambda = ln|G| / dt."""
    rp = mi.RunParams(8, 8, 32, nu=0.1, eta=0.1, dt=0.02, precision=8)
    z = np.arange(32) * (2 * math.pi / 32)
    k = 2
    st = np.zeros((7, 32, 8, 8))
    st[4] = (np.sin(k * z) / k)[:, None, None]
    st[5] = (np.cos(k * z) / k)[:, None, None]
    w = k * 2 * math.pi / 32
    k2 = (3 * (1 - math.cos(w)) - 0.3 * (1 - math.cos(2 * w)) + (1 - math.cos(3 * w)) / 45) / (2 * math.pi / 32) ** 2
    zz = -rp.eta * k2 * rp.dt
    G = 1 + zz + zz * zz / 2 + zz ** 3 / 6
    _, diag = gpu_run(mhd, rp, st, mi.no_forcing(10))
    lam = mhd.mhd_growth_rate(diag)
    assert abs(lam - math.log(abs(G)) / rp.dt) < 1e-10


def test_growth_rate_windows_match_the_oracle(mhd):
    """The 256^3 workload's recipe at 32^3 (FP64, helical forcing at kf = 3, f0 = 0.02,
    nu = eta = 1e-3, seed field 1e-5, 200 steps): the device's B_rms series and the
    growth-rate fits over steps 1-200 and 101-200 agree with the oracle's run."""
    rp = mi.RunParams(32, 32, 32, nu=1e-3, eta=1e-3, dt=1e-3, precision=8)
    st = mi.ic_seed_noise(rp, 0, 1e-5)
    recs = mi.forcing_schedule(0, 200, 3.0, 0.02, 1.0)
    _, diag = gpu_run(mhd, rp, st, recs)
    assert len(diag) == 201
    cur = st.astype(np.float64)
    t, br = [], []
    for n in range(201):
        d = oracle.diag(cur, rp)
        t.append(n * rp.dt)
        br.append(d["brms"])
        if n < 200:
            cur, _ = oracle.step(cur, rp, [recs[n]])
    gb = np.array([r["brms"] for r in diag])
    rel = np.max(np.abs(gb - np.array(br)) / np.array(br))
    print(f"B_rms series max relative difference over 200 steps: {rel:.2e}", flush=True)
    assert rel <= 1e-11
    for i0 in (1, 101):
        lg = mhd.mhd_growth_rate(diag, i0, 201)
        lo = oracle.growth_rate(t, br, i0, 201)
        print(f"lambda over steps {i0}-200: device {lg:.12e} oracle {lo:.12e}", flush=True)
        assert abs(lg - lo) <= 1e-10


def test_autotuner_picks_a_shape_that_runs_correctly(mhd):
    """mhd_autotune times every eligible tile shape on a scratch run and pins the fastest
    for the grid; a run created afterwards uses it and still matches the oracle."""
    rp = mi.RunParams(48, 40, 32, nu=2e-3, eta=2e-3, dt=1e-3, precision=4)
    p = mhd.params_from(rp)
    names = {mhd.mhd_tile_shape_name(i) for i in range(mhd.mhd_num_tile_shapes())}
    try:
        best = mhd.mhd_autotune(p, 2)
        chosen = mhd.mhd_tile_config(p)
        print(f"autotuned {chosen}: {best:.3f} ms per step", flush=True)
        assert best > 0 and any(chosen.startswith(n.split("+")[0]) for n in names)
        st = mi.noise_state(rp, 17, 0.1, 0.1, 0.1, dtype=np.float32)
        recs = mi.forcing_schedule(9, 2, 3.0, 0.05, 1.0)
        got, _ = gpu_run(mhd, rp, st, recs, per_step=True)
        want, scales = oracle_per_step(st, rp, recs)
        for n in range(2):
            check_step(got[n], want[n], scales[n], rp, f"autotuned {chosen} step {n + 1}")
    finally:
        mhd.mhd_set_tile_shape(p, -1)


# ------------------------------------------------------------------ runtime properties

@pytest.mark.parametrize("dims,prec", [((20, 16, 12), 8), ((21, 15, 11), 8), ((21, 15, 11), 4), ((64, 64, 64), 4)])
def test_init_seed_matches_input_generator(mhd, dims, prec):
    """The seed field generated on the device against the input generator: the same
    SplitMix64 counters and Box-Muller pairs (an odd cell count leaves the last pair
    half used); the device and host transcendentals may differ in the last bit, so
    FP64 values agree to a few ulp and FP32 values (rounded once from FP64) to one."""
    rp = mi.RunParams(*dims, nu=1e-3, eta=1e-3, precision=prec)
    want = mi.ic_seed_noise(rp, 42, 1e-5, dtype=_dtype(prec))
    with mhd.Run(mhd.params_from(rp)) as run:
        run.set_state(np.ones_like(want))      # the seed must overwrite all seven fields
        mhd.mhd_init_seed(run.h, 42, 1e-5)
        got = run.get_state()
    assert np.all(got[:4] == 0)
    rel = np.abs(got[4:].astype(np.float64) - want[4:]) / np.abs(want[4:]).astype(np.float64).clip(1e-300)
    bound = 8 * 2.0 ** -52 if prec == 8 else 2.0 ** -23
    assert np.max(rel) <= bound, np.max(rel)


def test_bitwise_deterministic_and_resumable(mhd):
    rp = mi.RunParams(24, 24, 24, nu=2e-3, eta=2e-3, precision=8)
    st = mi.noise_state(rp, 3, 0.1, 0.1, 0.1)
    recs = mi.forcing_schedule(5, 6, 3.0, 0.02, 1.0)
    a, _ = gpu_run(mhd, rp, st, recs)
    b, _ = gpu_run(mhd, rp, st, recs)
    assert np.array_equal(a[0], b[0])
    # checkpoint / resume: 3 steps, copy the state out, new context, 3 more steps
    h1, _ = gpu_run(mhd, rp, st, recs[:3])
    h2, _ = gpu_run(mhd, rp, h1[0], recs[3:])
    assert np.array_equal(h2[0], a[0])


def test_borrowed_torch_buffers(mhd):
    import torch
    rp = mi.RunParams(16, 12, 20, nu=2e-3, eta=2e-3, precision=4)
    st = mi.noise_state(rp, 8, 0.1, 0.1, 0.1, dtype=np.float32)
    recs = mi.forcing_schedule(6, 3, 3.0, 0.02, 0.0)
    ref, _ = gpu_run(mhd, rp, st, recs)
    bufs = torch.zeros((14, rp.ncell), dtype=torch.float32, device="cuda")
    stream = torch.cuda.current_stream()
    h = mhd.mhd_create_borrowed(mhd.params_from(rp), [bufs[i] for i in range(14)], stream)
    try:
        bufs[:7].copy_(torch.from_numpy(st.reshape(7, -1)))
        torch.cuda.synchronize()
        mhd.mhd_set_forcing(h, recs)
        mhd.mhd_step(h, 3)
        mhd.mhd_sync(h)
        par = 1 if mhd.mhd_field_ptr(h, 0) == bufs[7].data_ptr() else 0
        got = bufs[7 * par:7 * par + 7].cpu().numpy().reshape(ref[0].shape)
    finally:
        mhd.mhd_destroy(h)
    assert np.array_equal(got, ref[0])


def _batch_specs():
    # one run per precision with upwinding: those go to launches of their own
    return [mi.RunParams(16, 16, 16, nu=5e-3, eta=5e-3, precision=8),
            mi.RunParams(24, 20, 16, nu=2e-3, eta=2e-3, precision=8, upwind=1.0),
            mi.RunParams(32, 32, 32, nu=1e-3, eta=1e-3, precision=4),
            mi.RunParams(20, 20, 24, nu=4e-4, eta=4e-4, precision=4, upwind=0.5)]


@pytest.mark.parametrize("use_graph", [True, False])
def test_batched_ensemble_equals_runs_alone(mhd, use_graph):
    specs = _batch_specs()
    states = [mi.noise_state(rp, 40 + i, 0.1, 0.1, 0.1, dtype=_dtype(rp.precision)) for i, rp in enumerate(specs)]
    scheds = [mi.forcing_schedule(50 + i, 7, 3.0, 0.02, float(i % 2)) for i in range(len(specs))]
    alone = [gpu_run(mhd, rp, s, r)[0][0] for rp, s, r in zip(specs, states, scheds)]
    b = mhd.mhd_batch_create([mhd.params_from(rp) for rp in specs])
    try:
        ctxs = [mhd.mhd_batch_ctx(b, i) for i in range(len(specs))]
        for c, s, r in zip(ctxs, states, scheds):
            for f in range(7):
                mhd.mhd_set_field(c, f, np.ascontiguousarray(s[f]))
            mhd.mhd_set_forcing(c, r)
        mhd.mhd_batch_run(b, 4, use_graph)
        mhd.mhd_batch_run(b, 3, use_graph)
        for i, (c, rp) in enumerate(zip(ctxs, specs)):
            got = np.empty_like(alone[i])
            for f in range(7):
                mhd.mhd_get_field(c, f, got[f])
            assert np.array_equal(got, alone[i]), f"run {i} differs in the batch"
            assert len(mhd.mhd_get_diag(c)) == 7
    finally:
        mhd.mhd_batch_destroy(b)


def test_a_batch_that_fills_the_chip_gives_small_grids_the_large_tile(mhd):
    """16 FP32 runs of 64^3 bring 2^22 cells, enough to fill the chip together: the batch
    gives them the z-marching tile instead of the small ring tile they take alone, and
    each run still matches the oracle step by step at the FP32 bar.  Two such runs do
    not fill the chip and keep the tile they take alone."""
    rps = [mi.RunParams(64, 64, 64, nu=2e-3, eta=2e-3, dt=1e-3, precision=4) for _ in range(16)]
    alone_cfg = mhd.mhd_tile_config(mhd.params_from(rps[0]))
    b2 = mhd.mhd_batch_create([mhd.params_from(rp) for rp in rps[:2]])
    try:
        assert mhd.mhd_ctx_tile_config(mhd.mhd_batch_ctx(b2, 0)) == alone_cfg
    finally:
        mhd.mhd_batch_destroy(b2)
    states = [mi.noise_state(rp, 80 + i, 0.1, 0.1, 0.1, dtype=np.float32) for i, rp in enumerate(rps)]
    scheds = [mi.forcing_schedule(90 + i, 2, 3.0, 0.05, float(i % 2)) for i in range(len(rps))]
    outs = []
    b = mhd.mhd_batch_create([mhd.params_from(rp) for rp in rps])
    try:
        ctxs = [mhd.mhd_batch_ctx(b, i) for i in range(len(rps))]
        cfg = mhd.mhd_ctx_tile_config(ctxs[0])
        print(f"alone {alone_cfg}, in the batch {cfg}", flush=True)
        assert cfg == "64x8+zm" and cfg != alone_cfg
        for c, st, r in zip(ctxs, states, scheds):
            for f in range(7):
                mhd.mhd_set_field(c, f, np.ascontiguousarray(st[f]))
            mhd.mhd_set_forcing(c, r)
        for _ in range(2):
            mhd.mhd_batch_run(b, 1, False)
            step = []
            for i in (0, 7, 15):
                got = np.empty_like(states[i])
                for f in range(7):
                    mhd.mhd_get_field(ctxs[i], f, got[f])
                step.append(got)
            outs.append(step)
    finally:
        mhd.mhd_batch_destroy(b)
    for j, i in enumerate((0, 7, 15)):
        cur = states[i].astype(np.float64)
        for k in range(2):
            want, ts = oracle.step(cur, rps[i], [scheds[i][k]])
            check_step(outs[k][j], want, ts[0], rps[i], f"batch run {i} step {k + 1}")
            cur = outs[k][j].astype(np.float64)


def test_a_filled_batch_gives_an_8cubed_run_the_large_tile(mhd):
    """An FP32 batch whose large run brings more than 2^22 cells fills the chip, so an 8^3
    run in the same batch (too narrow for the z-marching tile) takes the 32-wide ring tile
    instead of its small one; that run (and a 12 x 8 x 8 one) still meets the FP32 bar
    against the oracle at every step."""
    rps = [mi.RunParams(256, 256, 128, nu=1e-3, eta=1e-3, precision=4),
           mi.RunParams(8, 8, 8, nu=4e-3, eta=3e-3, precision=4),
           mi.RunParams(12, 8, 8, nu=4e-3, eta=3e-3, precision=4)]
    states = [mi.noise_state(rp, 300 + i, 0.1, 0.1, 0.1, dtype=np.float32) for i, rp in enumerate(rps)]
    scheds = [mi.forcing_schedule(310 + i, 2, 3.0, 0.05, 1.0) for i in range(len(rps))]
    outs = []
    b = mhd.mhd_batch_create([mhd.params_from(rp) for rp in rps])
    try:
        ctxs = [mhd.mhd_batch_ctx(b, i) for i in range(len(rps))]
        cfgs = [mhd.mhd_ctx_tile_config(c) for c in ctxs]
        print("tiles in the batch:", cfgs, flush=True)
        assert cfgs[1] == cfgs[2] == "32x4x8/2+ring"
        for c, st, r in zip(ctxs, states, scheds):
            for f in range(7):
                mhd.mhd_set_field(c, f, np.ascontiguousarray(st[f]))
            mhd.mhd_set_forcing(c, r)
        for _ in range(2):
            mhd.mhd_batch_run(b, 1, False)
            step = []
            for i in (1, 2):
                got = np.empty_like(states[i])
                for f in range(7):
                    mhd.mhd_get_field(ctxs[i], f, got[f])
                step.append(got)
            outs.append(step)
    finally:
        mhd.mhd_batch_destroy(b)
    for j, i in enumerate((1, 2)):
        cur = states[i].astype(np.float64)
        for k in range(2):
            want, ts = oracle.step(cur, rps[i], [scheds[i][k]])
            check_step(outs[k][j], want, ts[0], rps[i], f"narrow batch run {i} step {k + 1}")
            cur = outs[k][j].astype(np.float64)


def test_server_continuous_batching_equals_alone(mhd):
    """Runs that arrive while others are in flight are admitted by footprint, advance
    together, and finish with exactly the state they reach alone."""
    specs = [(16, 8, 30), (24, 4, 45), (32, 4, 20), (16, 4, 60), (20, 8, 25), (28, 8, 40)]
    params = [mi.RunParams(n, n, n, nu=3e-3, eta=3e-3, precision=prec) for n, prec, _ in specs]
    budget = 3 * 14 * 8 * 28 ** 3 + (1 << 22)
    srv = mhd.mhd_server_create(budget, 4, 5)
    ids = []
    try:
        mhd.mhd_server_start(srv)
        for j, (rp, (_, _, steps)) in enumerate(zip(params, specs)):
            ids.append(mhd.mhd_server_submit(srv, mhd.params_from(rp), 100 + j, 1e-3, 3.0, 0.02,
                                             float(j % 2), steps, retain=True))
        for rid in ids:
            mhd.mhd_server_wait(srv, rid, 120.0)
        st = mhd.mhd_server_stats_get(srv)
        assert st.completed == len(specs) and st.failed == 0
        assert st.hbm_peak <= budget and st.lat_p99_ms > 0
        # one latency sample per step after each run's first (device clock between records)
        assert st.step_samples == sum(s - 1 for _, _, s in specs)
        for j, (rid, rp, (_, _, steps)) in enumerate(zip(ids, params, specs)):
            info = mhd.mhd_server_poll(srv, rid)
            assert info.state == mhd.MHD_RUN_DONE and info.steps_done == steps
            with mhd.Run(mhd.params_from(rp)) as run:
                mhd.mhd_init_seed(run.h, 100 + j, 1e-3)
                mhd.mhd_set_forcing_random(run.h, 3.0, 0.02, float(j % 2), 100 + j)
                run.step(steps)
                want = run.get_state()
            got = np.empty_like(want)
            for f in range(7):
                mhd.mhd_server_get_field(srv, rid, f, got[f])
            assert np.array_equal(got, want), f"served run {j} differs from the run alone"
    finally:
        mhd.mhd_server_destroy(srv)


def test_server_small_runs_keep_their_own_pace(mhd):
    """A small run submitted after a large one with as many steps finishes first: each
    size class takes steps in proportion to its cost, not one step per large step."""
    big = mi.RunParams(64, 64, 64, nu=3e-3, eta=3e-3, precision=4)
    small = mi.RunParams(16, 16, 16, nu=3e-3, eta=3e-3, precision=4)
    srv = mhd.mhd_server_create(1 << 30, 4, 4)
    try:
        mhd.mhd_server_start(srv)
        ib = mhd.mhd_server_submit(srv, mhd.params_from(big), 1, 1e-3, 3.0, 0.02, 0.0, 300)
        is_ = mhd.mhd_server_submit(srv, mhd.params_from(small), 2, 1e-3, 3.0, 0.02, 1.0, 300)
        mhd.mhd_server_wait(srv, ib, 120.0)
        mhd.mhd_server_wait(srv, is_, 120.0)
        rb, rs = mhd.mhd_server_poll(srv, ib), mhd.mhd_server_poll(srv, is_)
        assert rb.state == rs.state == mhd.MHD_RUN_DONE
        assert rb.steps_done == rs.steps_done == 300
        print(f"large done at {rb.t_done - rb.t_submit:.3f} s, small at {rs.t_done - rs.t_submit:.3f} s", flush=True)
        assert rs.t_done < rb.t_done
    finally:
        mhd.mhd_server_destroy(srv)


def test_server_evicts_a_run_that_goes_nonfinite(mhd):
    """A run with an unstable time step is flagged and evicted; a co-resident run is unaffected."""
    good = mi.RunParams(16, 16, 16, nu=3e-3, eta=3e-3, precision=8)
    bad = mi.RunParams(16, 16, 16, nu=3e-3, eta=3e-3, dt=5.0, precision=8)
    srv = mhd.mhd_server_create(1 << 30, 4, 2)
    try:
        mhd.mhd_server_start(srv)
        ig = mhd.mhd_server_submit(srv, mhd.params_from(good), 1, 1e-3, 3.0, 0.02, 1.0, 40, retain=True)
        ib = mhd.mhd_server_submit(srv, mhd.params_from(bad), 2, 1.0, 3.0, 5.0, 1.0, 4000, retain=False)
        mhd.mhd_server_wait(srv, ig, 60.0)
        mhd.mhd_server_wait(srv, ib, 60.0)
        assert mhd.mhd_server_poll(srv, ib).state == mhd.MHD_RUN_FAILED
        assert mhd.mhd_server_poll(srv, ib).steps_done < 4000
        assert mhd.mhd_server_poll(srv, ig).state == mhd.MHD_RUN_DONE
        with mhd.Run(mhd.params_from(good)) as run:
            mhd.mhd_init_seed(run.h, 1, 1e-3)
            mhd.mhd_set_forcing_random(run.h, 3.0, 0.02, 1.0, 1)
            run.step(40)
            want = run.get_state()
        got = np.empty_like(want)
        for f in range(7):
            mhd.mhd_server_get_field(srv, ig, f, got[f])
        assert np.array_equal(got, want)
    finally:
        mhd.mhd_server_destroy(srv)
