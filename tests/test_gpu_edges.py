"""Edge cases of the HIP path, through the C ABI: zero steps, calls that cross the
staging chunk of 512 steps (alone and in a graph-captured batch), grids that are one
tile thin in two directions and long in the third, and a forcing schedule that runs
out.  Parity bars as in the other GPU tests (per field, per step):
1e-12 (FP64) and 1e-5 (FP32) of the field's scale."""
import numpy as np
import pytest

import mhd_inputs as mi
import oracle

pytestmark = pytest.mark.gpu

TOL = {8: 1e-12, 4: 1e-5}
CHUNK = 512  # staging chunk of the library (steps per staged forcing block)


@pytest.fixture(scope="module")
def mhd():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2012_08758_amd as m
    return m


def _dtype(prec):
    return np.float64 if prec == 8 else np.float32


def _check(got, want, tscale, rp, label):
    e, plain = oracle.tolerance_error(got, want, tscale, rp.dt)
    print(f"{label}: e_f = " + " ".join(f"{n}:{x:.2e}" for n, x in zip(mi.FIELD_NAMES, e)), flush=True)
    assert np.all(e <= TOL[rp.precision]), (label, e, plain)


def test_zero_steps_is_a_no_op(mhd):
    rp = mi.RunParams(16, 12, 10, nu=2e-3, eta=2e-3, precision=8)
    st = mi.noise_state(rp, 11, 0.1, 0.1, 0.1)
    with mhd.Run(mhd.params_from(rp)) as run:
        run.set_state(st)
        run.set_forcing(mi.forcing_schedule(1, 2, 3.0, 0.02, 1.0))
        run.step(0)
        mhd.mhd_sync(run.h)
        assert np.array_equal(run.get_state(), st)
        assert run.diag() == [] and mhd.mhd_get_time(run.h) == (0, 0.0)
    b = mhd.mhd_batch_create([mhd.params_from(rp)])
    try:
        c = mhd.mhd_batch_ctx(b, 0)
        for f in range(7):
            mhd.mhd_set_field(c, f, np.ascontiguousarray(st[f]))
        mhd.mhd_batch_run(b, 0, True)
        got = np.empty_like(st)
        for f in range(7):
            mhd.mhd_get_field(c, f, got[f])
        assert np.array_equal(got, st) and mhd.mhd_get_diag(c) == []
    finally:
        mhd.mhd_batch_destroy(b)


def test_a_call_across_the_staging_chunk(mhd):
    """600 steps in one call (a chunk of 512, then 88) equal the same steps in calls that
    split elsewhere, bit for bit; the four steps around the chunk boundary match the
    oracle one by one; every step keeps its own forcing record and diagnostic record."""
    rp = mi.RunParams(10, 8, 12, nu=2e-2, eta=2e-2, dt=1e-3, precision=8)
    st = mi.smooth_state(rp, 4, kmax=2)
    nst = 600
    recs = mi.forcing_schedule(21, nst, 3.0, 0.05, 1.0)
    p = mhd.params_from(rp)
    with mhd.Run(p) as run:
        run.set_state(st)
        run.set_forcing(recs)
        run.step(nst)
        one_call = run.get_state()
        d1 = run.diag()
    with mhd.Run(p) as run:
        run.set_state(st)
        run.set_forcing(recs)
        run.step(CHUNK - 2)
        mid = run.get_state()
        per = []
        for _ in range(4):
            run.step(1)
            per.append(run.get_state())
        run.step(nst - CHUNK - 2)
        split = run.get_state()
        d2 = run.diag()
    assert np.array_equal(one_call, split)
    assert len(d1) == len(d2) == nst
    assert [r["step"] for r in d1] == list(range(nst))
    diff = [(a["step"], k) for a, b in zip(d1, d2) for k in a if k != "t_device" and a[k] != b[k]]
    assert not diff, diff[:5]
    # the device clock of the records (when each step was reduced) runs forward
    assert all(b["t_device"] > a["t_device"] for a, b in zip(d1, d1[1:]))
    cur = mid.astype(np.float64)
    for k in range(4):
        nxt, ts = oracle.step(cur, rp, [recs[CHUNK - 2 + k]])
        _check(per[k], nxt, ts[0], rp, f"step {CHUNK - 1 + k}")
        cur = per[k].astype(np.float64)


def test_a_graph_captured_batch_across_the_staging_chunk(mhd):
    specs = [mi.RunParams(8, 8, 8, nu=2e-2, eta=2e-2, precision=8),
             mi.RunParams(12, 8, 16, nu=2e-2, eta=2e-2, precision=4)]
    states = [mi.smooth_state(rp, 30 + i, kmax=2).astype(_dtype(rp.precision)) for i, rp in enumerate(specs)]
    nst = 530
    scheds = [mi.forcing_schedule(40 + i, nst, 3.0, 0.05, float(i)) for i in range(len(specs))]
    alone = []
    for rp, s, r in zip(specs, states, scheds):
        with mhd.Run(mhd.params_from(rp)) as run:
            run.set_state(s)
            run.set_forcing(r)
            run.step(nst)
            alone.append(run.get_state())
    b = mhd.mhd_batch_create([mhd.params_from(rp) for rp in specs])
    try:
        ctxs = [mhd.mhd_batch_ctx(b, i) for i in range(len(specs))]
        for c, s, r in zip(ctxs, states, scheds):
            for f in range(7):
                mhd.mhd_set_field(c, f, np.ascontiguousarray(s[f]))
            mhd.mhd_set_forcing(c, r)
        mhd.mhd_batch_run(b, nst, True)
        for i, c in enumerate(ctxs):
            got = np.empty_like(alone[i])
            for f in range(7):
                mhd.mhd_get_field(c, f, got[f])
            assert np.array_equal(got, alone[i]), f"run {i} differs in the batch"
            assert len(mhd.mhd_get_diag(c)) == nst
    finally:
        mhd.mhd_batch_destroy(b)


@pytest.mark.parametrize("prec", [8, 4])
@pytest.mark.parametrize("dims", [(200, 8, 8), (8, 200, 8), (8, 8, 200)])
def test_thin_long_grids(mhd, dims, prec):
    """Two sides at the minimum of 8 (the halo wraps within one tile), the third long
    and not a multiple of any tile side."""
    rp = mi.RunParams(*dims, nu=3e-3, eta=4e-3, dt=1e-3, precision=prec, bext=(0.0, 0.02, 0.0))
    st = mi.noise_state(rp, 60, 0.1, 0.1, 0.1, dtype=_dtype(prec))
    recs = mi.forcing_schedule(61, 2, 3.0, 0.05, 0.5)
    p = mhd.params_from(rp)
    outs = []
    with mhd.Run(p) as run:
        run.set_state(st)
        run.set_forcing(recs)
        for _ in recs:
            run.step(1)
            outs.append(run.get_state())
    cur = st.astype(np.float64)
    for k, r in enumerate(recs):
        nxt, ts = oracle.step(cur, rp, [r])
        _check(outs[k], nxt, ts[0], rp, f"{dims} fp{8 * prec} step {k + 1}")
        cur = outs[k].astype(np.float64)


def test_a_forcing_schedule_that_runs_out_is_an_error(mhd):
    rp = mi.RunParams(12, 12, 12, nu=2e-3, eta=2e-3, precision=8)
    st = mi.noise_state(rp, 70, 0.1, 0.1, 0.1)
    recs = mi.forcing_schedule(71, 3, 3.0, 0.05, 1.0)
    with mhd.Run(mhd.params_from(rp)) as run:
        run.set_state(st)
        run.set_forcing(recs)
        with pytest.raises(mhd.MhdError, match="outside the forcing schedule"):
            run.step(4)
        mhd.mhd_sync(run.h)
        assert np.array_equal(run.get_state(), st) and mhd.mhd_get_time(run.h)[0] == 0
        run.step(3)
        with pytest.raises(mhd.MhdError, match="outside the forcing schedule"):
            run.step(1)
        got = run.get_state()
    with mhd.Run(mhd.params_from(rp)) as run:
        run.set_state(st)
        run.set_forcing(recs)
        run.step(3)
        assert np.array_equal(got, run.get_state())
