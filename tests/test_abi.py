"""The C-ABI library loads, exports every symbol the header declares, and its host-only
logic (argument validation, forcing draws, growth-rate fit, tile shapes) behaves.
No device work here."""
import ctypes as C
import math
import os
import re

import numpy as np
import pytest

import mhd_inputs as mi

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mhd.h")


def _mhd():
    import paper_2012_08758_amd as mhd
    return mhd


def header_symbols():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(mhd_[a-z0-9_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    mhd = _mhd()
    lib = C.CDLL(mhd.LIB_PATH)
    syms = header_symbols()
    assert len(syms) >= 30
    missing = [s for s in syms if not hasattr(lib, s)]
    assert not missing, missing
    # and the binding covers exactly the declared API
    assert sorted(mhd.EXPORTS) == syms


def test_struct_layouts_match_header():
    mhd = _mhd()
    assert C.sizeof(mhd.mhd_params) == 4 * 4 + 11 * 8
    assert C.sizeof(mhd.mhd_forcing) == 4 * 4 + 6 * 8
    assert C.sizeof(mhd.mhd_diag) == 8 + 12 * 8


@pytest.mark.parametrize("bad", [
    dict(nx=7), dict(ny=4), dict(precision=2), dict(dt=0.0), dict(dt=-1e-3), dict(nu=-1.0),
    dict(eta=float("nan")), dict(lx=0.0), dict(nx=70000), dict(bext=(0.0, float("inf"), 0.0)),
    dict(upwind=-1.0), dict(upwind=float("nan")),
])
def test_invalid_parameters_are_rejected_before_device_work(bad):
    mhd = _mhd()
    kw = dict(nu=1e-3, eta=1e-3)
    n = dict(nx=16, ny=16, nz=16)
    for k in ("nx", "ny", "nz"):
        if k in bad:
            n[k] = bad.pop(k)
    p = mhd.make_params(n["nx"], n["ny"], n["nz"], **kw)
    for k, v in bad.items():
        if k == "bext":
            for a in range(3):
                p.bext[a] = v[a]
        else:
            setattr(p, k, v)
    with pytest.raises(mhd.MhdError) as ei:
        mhd.mhd_create(p)
    assert ei.value.status == mhd.MHD_E_INVALID
    assert mhd.lib.mhd_last_error().decode()


def test_forcing_draws_match_the_input_generator_bit_for_bit():
    mhd = _mhd()
    for kf in (3.0, 5.0):
        ref = mi.forcing_draws(11, 300, kf)
        for n in range(300):
            f = mhd.mhd_forcing_draw(kf, 0.02, 1.0, 11, n)
            assert tuple(f.k) == ref[n].k
            assert tuple(f.e) == ref[n].e
            assert f.phi == ref[n].phi
            assert f.sigma == 1.0 and f.f0 == 0.02


def test_growth_rate_fit_host_side():
    mhd = _mhd()
    t = np.arange(50) * 1e-3
    recs = [dict(t=float(x), brms=float(2e-5 * math.exp(0.031 * x))) for x in t]
    assert abs(mhd.mhd_growth_rate(recs) - 0.031) < 1e-10
    assert abs(mhd.mhd_growth_rate(recs, 10, 40) - 0.031) < 1e-10
    with pytest.raises(mhd.MhdError):
        mhd.mhd_growth_rate(recs, 5, 6)


def test_tile_shapes_and_pinning():
    mhd = _mhd()
    n = mhd.mhd_num_tile_shapes()
    names = [mhd.mhd_tile_shape_name(i) for i in range(n)]
    assert len(set(names)) == n and all(re.fullmatch(r"\d+x\d+x\d+/\d(\+ring|\+march)?|\d+x\d+\+zm", s) for s in names)
    p = mhd.make_params(96, 80, 72, nu=1e-3, eta=1e-3)
    default = mhd.mhd_tile_config(p)
    mhd.mhd_set_tile_shape(p, 0)              # the register-staged 16x8x4 tile runs on any grid
    assert mhd.mhd_tile_config(p) == names[0] != default
    mhd.mhd_set_tile_shape(p, -1)
    assert mhd.mhd_tile_config(p) == default
    with pytest.raises(mhd.MhdError):
        mhd.mhd_set_tile_shape(p, n)


def test_binding_refuses_to_run_without_the_library(tmp_path, monkeypatch):
    """The product path has no fallback: a missing library is an ImportError."""
    import importlib.util
    src = os.path.join(ROOT, "paper_2012_08758_amd", "__init__.py")
    fake = tmp_path / "pkg"
    fake.mkdir()
    (fake / "__init__.py").write_text(open(src).read())
    spec = importlib.util.spec_from_file_location("mhd_nolib", str(fake / "__init__.py"))
    mod = importlib.util.module_from_spec(spec)
    with pytest.raises(ImportError):
        spec.loader.exec_module(mod)


# ------------------------------------------------------------------ spectrum (host-only parts)

@pytest.mark.parametrize("dims,kw", [((32, 32, 32), {}), ((48, 40, 36), dict(lx=5.0, ly=6.0, lz=4.0)),
                                     ((45, 28, 50), {}), ((2048, 8, 8), {})])
def test_spectrum_shells_match_the_oracle(dims, kw):
    import oracle
    mhd = _mhd()
    rp = mi.RunParams(*dims, nu=1e-3, eta=1e-3, **kw)
    ns, dk, wb = mhd.mhd_spectrum_shells(mhd.params_from(rp))
    assert ns == oracle.spectrum_nshell(rp)
    assert dk == 2 * math.pi / max(rp.lx, rp.ly, rp.lz)
    assert wb >= 48 * (rp.nx // 2 + 1) * rp.ny * rp.nz


@pytest.mark.parametrize("dims", [(37, 32, 32), (32, 22, 32), (32, 32, 8192)])
def test_spectrum_rejects_grids_it_cannot_transform(dims):
    mhd = _mhd()
    rp = mi.RunParams(*dims, nu=1e-3, eta=1e-3)
    with pytest.raises(mhd.MhdError) as ei:
        mhd.mhd_spectrum_shells(mhd.params_from(rp))
    assert ei.value.status == mhd.MHD_E_UNSUPPORTED


def test_channel_growth_rate_is_half_the_log_slope():
    mhd = _mhd()
    t = np.arange(50) * 0.1
    assert abs(mhd.mhd_channel_growth_rate(t, 3e-9 * np.exp(2 * 0.0173 * t)) - 0.0173) < 1e-12
    with pytest.raises(mhd.MhdError):
        mhd.mhd_channel_growth_rate(t[:1], np.ones(1))
    with pytest.raises(mhd.MhdError):
        mhd.mhd_channel_growth_rate(t, np.zeros(50))


def test_null_handles_are_rejected():
    """Every entry point that takes a context, batch or server handle refuses NULL with
    MHD_E_INVALID (no device work: these fail before any HIP call)."""
    mhd = _mhd()
    lib = mhd.lib
    buf = C.create_string_buffer(64)
    d, s, i32 = C.c_double(), C.c_int64(), C.c_int32()
    calls = {
        "mhd_step": lambda: lib.mhd_step(None, 1),
        "mhd_reduce": lambda: lib.mhd_reduce(None),
        "mhd_sync": lambda: lib.mhd_sync(None),
        "mhd_get_time": lambda: lib.mhd_get_time(None, C.byref(s), C.byref(d)),
        "mhd_ctx_tile_config": lambda: lib.mhd_ctx_tile_config(None, buf, 64),
        "mhd_spectrum": lambda: lib.mhd_spectrum(None, None, 0, C.byref(i32), C.byref(d)),
        "mhd_init_seed": lambda: lib.mhd_init_seed(None, 1, 1e-5),
        "mhd_clear_forcing": lambda: lib.mhd_clear_forcing(None),
        "mhd_batch_run": lambda: lib.mhd_batch_run(None, 1, 1),
    }
    for name, call in calls.items():
        assert call() == mhd.MHD_E_INVALID, name
