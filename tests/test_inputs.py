"""The seeded input generator: published SplitMix64 values, shell contents, determinism."""
import math
import os

import numpy as np

import mhd_inputs as mi

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _golden_lines(name):
    with open(os.path.join(GOLD, name)) as fh:
        return [ln.strip() for ln in fh if ln.strip() and not ln.startswith("#")]


def test_splitmix64_matches_published_sequence():
    # the generator seeded with state 0: outputs mix(0 + (i+1)*gamma)
    want = [int(x, 16) for x in _golden_lines("splitmix64_state0.txt")]
    got = [int(mi._mix(np.uint64((i + 1) * 0x9E3779B97F4A7C15 % 2**64))) for i in range(len(want))]
    assert got == want


def test_forcing_shell_counts_match_section4_definition():
    for line in _golden_lines("forcing_shell.txt"):
        kf, count, q = line.split()
        sh = mi.shell_vectors(float(kf))
        assert len(sh) == int(count)
        qs = sorted(set(int(x) for x in (sh.astype(np.int64) ** 2).sum(1)))
        assert qs == [int(x) for x in q.split(",")]
        n = np.sqrt((sh.astype(float) ** 2).sum(1))
        assert np.all(n >= float(kf) - 0.5) and np.all(n <= float(kf) + 0.5)


def test_uniform_range_and_determinism():
    u = mi.uniform(3, 9, np.arange(100000))
    assert u.min() >= 0.0 and u.max() < 1.0
    assert abs(u.mean() - 0.5) < 0.01
    assert np.array_equal(u, mi.uniform(3, 9, np.arange(100000)))
    assert not np.array_equal(u, mi.uniform(4, 9, np.arange(100000)))


def test_normal_moments():
    z = mi.normal(1, 2, 200001)
    assert len(z) == 200001
    assert abs(z.mean()) < 0.01 and abs(z.std() - 1.0) < 0.01


def test_forcing_draws_are_valid():
    draws = mi.forcing_draws(0, 500, 3.0)
    shell = {tuple(k) for k in mi.shell_vectors(3.0).tolist()}
    for d in draws:
        assert tuple(d.k) in shell
        assert abs(np.linalg.norm(d.e) - 1.0) < 1e-14
        kh = np.array(d.k) / np.linalg.norm(d.k)
        assert abs(kh @ np.array(d.e)) <= 0.99
        assert -math.pi <= d.phi < math.pi
    # all shell vectors get drawn eventually, roughly uniformly
    ks = [tuple(d.k) for d in mi.forcing_draws(0, 20000, 3.0)]
    assert len(set(ks)) == 98


def test_ic_seed_noise_layout():
    p = mi.RunParams(8, 10, 12, nu=1e-3, eta=1e-3)
    st = mi.ic_seed_noise(p, 0, 1e-5)
    assert st.shape == (7, 12, 10, 8)
    assert np.all(st[:4] == 0.0)
    assert 0.5e-5 < st[4:].std() < 1.5e-5


def test_workload_recipes():
    runs = mi.ensemble_runs()
    assert len(runs) == 48
    assert sum(r["n"] == 64 for r in runs) == 32 and sum(r["n"] == 128 for r in runs) == 16
    assert abs(runs[0]["nu"] - 5e-3) < 1e-15 and abs(runs[-1]["nu"] - 2e-4) < 1e-15
    tr = mi.serving_trace(240)
    assert len(tr) == 240
    gaps = np.diff([0.0] + [r["arrival"] for r in tr])
    assert 0.15 < gaps.mean() < 0.35
    assert all(3e-4 <= r["nu"] <= 1e-2 for r in tr)
