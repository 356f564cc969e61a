"""The 48-run ensemble mix and a served run, against the oracle and against runs alone,
through the C ABI.

Bars as in test_gpu_parity: per field and step e_f <= 1e-5 for FP32 runs, from the same
input state and forcing record; runs whose tile shape is the same alone and in the
batch must match their run alone bit for bit.  Initial states come from the input
generator (the library's seed field is checked against it in test_gpu_parity).
"""
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


def _check(got, want, tscale, rp, label):
    e, plain = oracle.tolerance_error(got, want, tscale, rp.dt)
    print(f"{label}: e_f = " + " ".join(f"{n}:{x:.2e}" for n, x in zip(mi.FIELD_NAMES, e)), flush=True)
    assert np.all(e <= TOL[rp.precision]), (label, e, plain)


def _rp(r):
    return mi.RunParams(r["n"], r["n"], r["n"], nu=r["nu"], eta=r["eta"], dt=r["dt"], precision=r["precision"])


def _state(mhd, ctx, rp):
    out = np.empty((7, rp.nz, rp.ny, rp.nx), dtype=np.float32 if rp.precision == 4 else np.float64)
    for f in range(7):
        mhd.mhd_get_field(ctx, f, out[f])
    return out


def test_the_48_run_ensemble_mix(mhd):
    """The ensemble workload (32 x 64^3 + 16 x 128^3, FP32, nu = eta log-spaced, helical and
    non-helical forcing, seeds 0..47) for two graph-replayed steps: sampled 64^3 runs
    against the oracle at every step, sampled 128^3 runs bit for bit against the same runs
    alone with the tile shape pinned to the one they take in the batch (the z-marching
    kernel with 64-wide tiles in substeps 1 and 2, which neither size takes alone)."""
    runs = mi.ensemble_runs()
    rps = [_rp(r) for r in runs]
    check64, check128 = (0, 13, 31), (32, 41, 47)
    outs = {i: [] for i in check64 + check128}
    b = mhd.mhd_batch_create([mhd.params_from(rp) for rp in rps])
    try:
        ctxs = [mhd.mhd_batch_ctx(b, i) for i in range(len(runs))]
        cfg = {mhd.mhd_ctx_tile_config(c) for c in ctxs}
        print("tiles in the 48-run batch:", cfg, flush=True)
        assert cfg == {"64x8+zm"}
        for c, r in zip(ctxs, runs):
            mhd.mhd_init_seed(c, r["seed"], r["a_noise"])
            mhd.mhd_set_forcing_random(c, r["kf"], r["f0"], r["sigma"], r["seed"])
        for _ in range(2):
            mhd.mhd_batch_run(b, 1, True)
            for i in outs:
                outs[i].append(_state(mhd, ctxs[i], rps[i]))
    finally:
        mhd.mhd_batch_destroy(b)
    for i in check64:
        r, rp = runs[i], rps[i]
        recs = mi.forcing_schedule(r["seed"], 2, r["kf"], r["f0"], r["sigma"])
        cur = mi.ic_seed_noise(rp, r["seed"], r["a_noise"], dtype=np.float32).astype(np.float64)
        for k in range(2):
            want, ts = oracle.step(cur, rp, [recs[k]])
            _check(outs[i][k], want, ts[0], rp, f"ensemble run {i} (64^3) step {k + 1}")
            cur = outs[i][k].astype(np.float64)
    names = [mhd.mhd_tile_shape_name(j) for j in range(mhd.mhd_num_tile_shapes())]
    for i in check128:
        r, rp = runs[i], rps[i]
        p = mhd.params_from(rp)
        mhd.mhd_set_tile_shape(p, names.index("64x8+zm"))
        try:
            with mhd.Run(p) as run:
                mhd.mhd_init_seed(run.h, r["seed"], r["a_noise"])
                mhd.mhd_set_forcing_random(run.h, r["kf"], r["f0"], r["sigma"], r["seed"])
                for k in range(2):
                    run.step(1)
                    alone = run.get_state()
                    assert np.array_equal(outs[i][k], alone), f"ensemble run {i} (128^3) step {k + 1} differs from alone"
        finally:
            mhd.mhd_set_tile_shape(p, -1)


def test_a_served_run_matches_the_oracle_on_its_first_step(mhd):
    """A 32^3 FP32 request that arrives while larger requests are being served: its state
    after its first step matches the oracle's step of the same seeded state and forcing
    record at the FP32 bar, and the server's per-step latencies are measured samples
    (one per step after a run's first, from the device clock of its records)."""
    srv = mhd.mhd_server_create(1 << 32, 8, 5)
    reqs = [(64, 3e-3, 0.0, 7, 40), (48, 2e-3, 1.0, 8, 30), (32, 4e-3, 1.0, 9, 1), (64, 1e-3, 1.0, 10, 20)]
    ids = []
    try:
        mhd.mhd_server_start(srv)
        for n, nu, sigma, seed, steps in reqs:
            rp = mi.RunParams(n, n, n, nu=nu, eta=nu, precision=4)
            ids.append(mhd.mhd_server_submit(srv, mhd.params_from(rp), seed, 1e-3, 3.0, 0.05, sigma, steps,
                                             retain=True))
        for rid in ids:
            mhd.mhd_server_wait(srv, rid, 120.0)
        st = mhd.mhd_server_stats_get(srv)
        assert st.completed == len(reqs) and st.failed == 0
        assert st.step_samples == sum(s - 1 for *_, s in reqs)
        assert 0 < st.lat_p50_ms <= st.lat_p99_ms
        n, nu, sigma, seed, steps = reqs[2]
        rp = mi.RunParams(n, n, n, nu=nu, eta=nu, precision=4)
        got = np.empty((7, n, n, n), dtype=np.float32)
        for f in range(7):
            mhd.mhd_server_get_field(srv, ids[2], f, got[f])
    finally:
        mhd.mhd_server_destroy(srv)
    st0 = mi.ic_seed_noise(rp, seed, 1e-3, dtype=np.float32).astype(np.float64)
    want, ts = oracle.step(st0, rp, mi.forcing_schedule(seed, 1, 3.0, 0.05, sigma))
    _check(got, want, ts[0], rp, "served 32^3 run, step 1")
