"""Pins for the FP64 oracle: closed forms, exactness, invariants and an independent brute force.

None of these re-types the oracle's formulas: each checks what the paper's
equations and the mathematics of the discretisation fix (polynomial exactness and
sixth-order convergence of the stencils, exact linear solutions of the discrete
system, the isothermal energy budget, symmetries), so that a dropped term, a wrong
sign, index or coefficient in the oracle fails at least one of them.
"""
import math

import numpy as np
import pytest

import mhd_inputs as mi
import oracle
from oracle import numpy_ref

TWO_PI = 2.0 * math.pi


def _p(nx, ny=None, nz=None, **kw):
    ny = nx if ny is None else ny
    nz = nx if nz is None else nz
    kw.setdefault("nu", 0.0)
    kw.setdefault("eta", 0.0)
    return mi.RunParams(nx, ny, nz, **kw)


def _coords(p):
    x = np.arange(p.nx) * (p.lx / p.nx)
    y = np.arange(p.ny) * (p.ly / p.ny)
    z = np.arange(p.nz) * (p.lz / p.nz)
    return np.meshgrid(z, y, x, indexing="ij")[::-1]  # X, Y, Z each (nz, ny, nx)


# Modified wavenumbers of the explicit sixth-order central schemes (Lele 1992, J. Comput.
# Phys. 103, 16, Section 2): first derivative w' = 3/2 sin w - 3/10 sin 2w + 1/30 sin 3w,
# second derivative w''^2 = 3(1 - cos w) - 3/10 (1 - cos 2w) + 1/45 (1 - cos 3w), w = k h.
def keff(k, h):
    w = k * h
    return (1.5 * math.sin(w) - 0.3 * math.sin(2 * w) + math.sin(3 * w) / 30.0) / h


def k2eff(k, h):
    w = k * h
    return math.sqrt(3 * (1 - math.cos(w)) - 0.3 * (1 - math.cos(2 * w))
                     + (1 - math.cos(3 * w)) / 45.0) / h


def rk3_poly(z):
    """Amplification of any three-stage third-order Runge-Kutta scheme on y' = z y / dt."""
    return np.eye(z.shape[0]) + z + z @ z / 2 + z @ z @ z / 6 if np.ndim(z) == 2 else \
        1 + z + z * z / 2 + z ** 3 / 6


NOFORCE = mi.no_forcing(1)[0]


# ------------------------------------------------------------------ stencils

@pytest.mark.parametrize("axis", [0, 1, 2])
def test_first_derivative_exact_to_degree_6_only(axis):
    h = 0.37
    n = [9, 9, 9]
    n[axis] = 15
    idx = np.meshgrid(np.arange(n[2]), np.arange(n[1]), np.arange(n[0]), indexing="ij")[::-1]
    s = (idx[axis] - 7) * h
    hh = [1.0, 1.0, 1.0]
    hh[axis] = h
    for deg in range(8):
        d = oracle.deriv(s ** deg, hh, 1, axis, wrap=False)
        want = deg * s ** (deg - 1) if deg else 0 * s
        m = ~np.isnan(d)
        err = np.max(np.abs(d[m] - want[m]))
        if deg <= 6:
            assert err <= 1e-12 * max(1.0, np.max(np.abs(s[m] ** deg)) / h)
        else:
            assert err > 1e-6  # not exact at degree 7: truncation error h^6 f^(7) / 140
            # the leading error term of the sixth-order scheme: -h^6/140 * 7!
            assert abs(np.mean(d[m] - want[m]) - h ** 6 * 5040 / 140) < 1e-9


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_second_derivative_exact_to_degree_7(axis):
    h = 0.29
    n = [9, 9, 9]
    n[axis] = 15
    idx = np.meshgrid(np.arange(n[2]), np.arange(n[1]), np.arange(n[0]), indexing="ij")[::-1]
    s = (idx[axis] - 7) * h
    hh = [1.0, 1.0, 1.0]
    hh[axis] = h
    for deg in range(9):
        d = oracle.deriv(s ** deg, hh, 2, axis, wrap=False)
        want = deg * (deg - 1) * s ** (deg - 2) if deg >= 2 else 0 * s
        m = ~np.isnan(d)
        err = np.max(np.abs(d[m] - want[m]))
        if deg <= 7:
            assert err <= 1e-11 * max(1.0, np.max(np.abs(s[m] ** deg)) / h ** 2)
        else:
            assert err > 1e-6


@pytest.mark.parametrize("a,b", [(0, 1), (0, 2), (1, 2), (1, 0), (2, 1)])
def test_mixed_derivative_exact_to_total_degree_7(a, b):
    ha, hb = 0.31, 0.23
    n = [13, 13, 13]
    idx = np.meshgrid(np.arange(n[2]), np.arange(n[1]), np.arange(n[0]), indexing="ij")[::-1]
    hh = [1.0, 1.0, 1.0]
    hh[a], hh[b] = ha, hb
    sa = (idx[a] - 6) * ha
    sb = (idx[b] - 6) * hb
    for p in range(8):
        for q in range(8 - p):
            f = sa ** p * sb ** q
            d = oracle.deriv(f, hh, 3, a, b, wrap=False)
            want = (p * q * sa ** max(p - 1, 0) * sb ** max(q - 1, 0)) if p and q else 0 * f
            m = ~np.isnan(d)
            err = np.max(np.abs(d[m] - want[m]))
            assert err <= 1e-11 * max(1.0, np.max(np.abs(f[m])) / (ha * hb)), (p, q, err)
    # total degree 8 with odd powers is not exact (for even-even powers the two
    # diagonal truncation errors cancel)
    f = sa ** 5 * sb ** 3
    d = oracle.deriv(f, hh, 3, a, b, wrap=False)
    m = ~np.isnan(d)
    assert np.max(np.abs(d[m] - 15 * sa[m] ** 4 * sb[m] ** 2)) > 1e-8


def test_periodic_stencils_converge_at_sixth_order():
    errs = {1: [], 2: [], 3: []}
    for n in (24, 48, 96):
        X, Y, _ = _coords(_p(n, n, 2))
        h = TWO_PI / n
        x = np.arange(n) * h
        f = np.sin(3 * x + 0.4)[None, None, :] * np.ones((2, 2, 1))
        errs[1].append(np.max(np.abs(oracle.deriv(f, (h, 1, 1), 1, 0) - 3 * np.cos(3 * x + 0.4))))
        errs[2].append(np.max(np.abs(oracle.deriv(f, (h, 1, 1), 2, 0) + 9 * np.sin(3 * x + 0.4))))
        g = np.sin(2 * X + 3 * Y + 0.3)
        d = oracle.deriv(g, (h, h, 1.0), 3, 0, 1)
        errs[3].append(np.max(np.abs(d + 6 * np.sin(2 * X + 3 * Y + 0.3))))
    for k, e in errs.items():
        r1, r2 = e[0] / e[1], e[1] / e[2]
        assert 50 < r1 < 75 and 58 < r2 < 70, (k, e)


def test_modified_wavenumbers_match_published_closed_forms():
    n, k = 32, 3
    h = TWO_PI / n
    x = np.arange(n) * h
    f = np.sin(k * x)[None, None, :] * np.ones((2, 2, 1))
    d1 = oracle.deriv(f, (h, 1, 1), 1, 0)[0, 0]
    d2 = oracle.deriv(f, (h, 1, 1), 2, 0)[0, 0]
    assert np.max(np.abs(d1 - keff(k, h) * np.cos(k * x))) < 1e-13
    assert np.max(np.abs(d2 + k2eff(k, h) ** 2 * np.sin(k * x))) < 1e-12
    assert abs(keff(k, h) / k - 0.999721092477) < 1e-12
    assert abs(k2eff(k, h) ** 2 / k ** 2 - 0.999929320612) < 1e-12


def test_periodic_wrap_equals_tiled_patch():
    rng = np.random.default_rng(5)
    f = rng.standard_normal((8, 8, 8))
    big = np.tile(f, (3, 3, 3))
    h = (0.3, 0.5, 0.7)
    for kind, a, b in [(1, 0, 0), (1, 1, 0), (1, 2, 0), (2, 0, 0), (2, 2, 0), (3, 0, 1), (3, 0, 2), (3, 1, 2)]:
        per = oracle.deriv(f, h, kind, a, b, wrap=True)
        pat = oracle.deriv(big, h, kind, a, b, wrap=False)[8:16, 8:16, 8:16]
        assert np.array_equal(per, pat)


# ------------------------------------------------------------------ time stepping

def test_shear_wave_follows_rk3_amplification_exactly():
    # u = (0, U sin kx, 0): advection, pressure, Lorentz and 2 S.grad ln rho vanish identically
    # in the discrete system, so u_y^n = U G(-nu k2^2 dt)^n sin kx with G the RK3 polynomial.
    p = _p(32, 4, 4, nu=0.2, dt=0.05)
    X, _, _ = _coords(p)
    st = np.zeros((7, p.nz, p.ny, p.nx))
    U, k = 0.1, 3
    st[2] = U * np.sin(k * X)
    out, _ = oracle.step(st, p, mi.no_forcing(10))
    z = -p.nu * k2eff(k, TWO_PI / 32) ** 2 * p.dt
    want = U * rk3_poly(z) ** 10 * np.sin(k * X)
    assert np.max(np.abs(out[2] - want)) < 1e-14
    assert np.max(np.abs(out[[0, 1, 3, 4, 5, 6]])) == 0.0
    # the continuous solution differs by the time error z^4/24 per step: the test can tell
    assert np.max(np.abs(want - U * math.exp(10 * z) * np.sin(k * X))) > 1e-7
    # and by the stencil error at fixed dt, within the sixth-order truncation
    zc = -p.nu * k ** 2 * p.dt
    assert np.max(np.abs(out[2] - U * rk3_poly(zc) ** 10 * np.sin(k * X))) < 1e-4 * U


def test_nonlinear_time_convergence_is_third_order():
    p0 = _p(12, nu=0.02, eta=0.02)
    st = mi.smooth_state(p0, 11, kmax=2, amp_lnrho=0.2, amp_u=0.5, amp_a=0.5, nmodes=3)
    T = 0.16
    sols = {}
    for nst in (4, 8, 16, 128):
        p = _p(12, nu=0.02, eta=0.02, dt=T / nst)
        sols[nst], _ = oracle.step(st, p, mi.no_forcing(nst))
    e = [np.max(np.abs(sols[n] - sols[128])) for n in (4, 8, 16)]
    r1, r2 = e[0] / e[1], e[1] / e[2]
    assert 6.5 < r1 < 9.5 and 6.5 < r2 < 9.5, e


def test_beltrami_field_is_force_free_and_decays_at_the_discrete_rate():
    # Section 5: the large-scale field B = (Bx sin(kz + phi), By cos(kz + phi), 0).
    p = _p(8, 8, 32, eta=0.1, nu=0.1, dt=0.02)
    _, _, Z = _coords(p)
    k = 2
    st = np.zeros((7, p.nz, p.ny, p.nx))
    st[4] = np.sin(k * Z) / k
    st[5] = np.cos(k * Z) / k
    h = TWO_PI / 32
    G = rk3_poly(-p.eta * k2eff(k, h) ** 2 * p.dt)
    series = []
    cur = st
    for n in range(11):
        d = oracle.diag(cur, p)
        series.append(d["brms"])
        assert abs(d["em"] - 0.5 * (keff(k, h) / k) ** 2 * G ** (2 * n)) < 1e-14
        assert abs(d["bx_mean"]) < 1e-15 and abs(d["by_mean"]) < 1e-15
        if n < 10:
            cur, _ = oracle.step(cur, p, mi.no_forcing(1))
    assert np.max(np.abs(cur[4:6] - G ** 10 * st[4:6])) < 1e-14
    assert np.max(np.abs(cur[:4])) < 1e-13  # j x B = 0 up to roundoff, so u and ln rho stay 0
    t = np.arange(11) * p.dt
    lam = oracle.growth_rate(t, series)
    assert abs(lam - math.log(abs(G)) / p.dt) < 1e-12


def _linear_evolution(M, dt, nsteps, v0):
    P = rk3_poly(dt * M)
    return np.linalg.matrix_power(P, nsteps) @ v0


def test_alfven_wave_uses_the_second_derivative_wavenumber():
    # B_ext = B0 z, u_x = U cos kz: u_x' = -B0 D2 A_y + nu D2 u_x, A_y' = -B0 u_x + eta D2 A_y
    B0, U, k = 1.0, 1e-7, 4
    p = _p(4, 4, 32, nu=0.01, eta=0.01, dt=0.01, bext=(0.0, 0.0, B0))
    _, _, Z = _coords(p)
    st = np.zeros((7, p.nz, p.ny, p.nx))
    st[1] = U * np.cos(k * Z)
    n = 50
    out, _ = oracle.step(st, p, mi.no_forcing(n))
    h = TWO_PI / 32
    q = k2eff(k, h) ** 2
    M = np.array([[-p.nu * q, B0 * q], [-B0, -p.eta * q]])
    uh, ah = _linear_evolution(M, p.dt, n, np.array([U, 0.0]))
    assert np.max(np.abs(out[1] - uh * np.cos(k * Z))) < 1e-5 * U
    assert np.max(np.abs(out[5] - ah * np.cos(k * Z))) < 1e-5 * U
    # using the first-derivative wavenumber instead would be visibly wrong
    q1 = keff(k, h) ** 2
    M1 = np.array([[-p.nu * q1, B0 * q1], [-B0, -p.eta * q1]])
    uh1, _ = _linear_evolution(M1, p.dt, n, np.array([U, 0.0]))
    assert abs(uh1 - uh) > 1e-3 * U


def test_sound_wave_linear_evolution():
    # ln rho = eps cos kx, u = 0: u_x' = cs^2 keff eps_hat - 4/3 nu k2^2 u_hat, eps' = -keff u_hat
    eps, k = 1e-7, 4
    p = _p(32, 4, 4, nu=0.01, eta=0.01, dt=0.01)
    X, _, _ = _coords(p)
    st = np.zeros((7, p.nz, p.ny, p.nx))
    st[0] = eps * np.cos(k * X)
    n = 50
    out, _ = oracle.step(st, p, mi.no_forcing(n))
    h = TWO_PI / 32
    ke, q = keff(k, h), k2eff(k, h) ** 2
    M = np.array([[-4.0 / 3.0 * p.nu * q, p.cs ** 2 * ke], [-ke, 0.0]])
    uh, eh = _linear_evolution(M, p.dt, n, np.array([0.0, eps]))
    assert np.max(np.abs(out[1] - uh * np.sin(k * X))) < 1e-5 * eps
    assert np.max(np.abs(out[0] - eh * np.cos(k * X))) < 1e-5 * eps


# ------------------------------------------------------------------ forcing

@pytest.mark.parametrize("sigma", [0.0, 0.5, 1.0])
def test_forcing_is_a_single_transverse_unit_mode(sigma):
    p = _p(16, nu=1e-3, eta=1e-3, dt=1e-3)
    rec = mi.Forcing(k=(2, -1, 2), e=(0.6, 0.0, 0.8), phi=0.7, sigma=sigma, f0=0.02)
    F = oracle.forcing_field(p, rec)
    Fh = np.fft.fftn(F, axes=(1, 2, 3)) / (16 ** 3)
    kidx = (rec.k[2] % 16, rec.k[1] % 16, rec.k[0] % 16)
    midx = ((-rec.k[2]) % 16, (-rec.k[1]) % 16, (-rec.k[0]) % 16)
    spec = np.sum(np.abs(Fh) ** 2, axis=0)
    tot = spec.sum()
    assert (spec[kidx] + spec[midx]) / tot > 1 - 1e-15
    K = np.array(rec.k, dtype=float)
    kn = np.linalg.norm(K)
    amp = rec.f0 * p.cs * math.sqrt(kn * p.cs / p.dt)
    # f = Re{amp f_k e^{i(k.x+phi)}}: the FFT coefficient at +k is amp/2 f_k e^{i phi}
    fk = 2.0 * Fh[(slice(None),) + kidx] * np.exp(-1j * rec.phi) / amp
    assert abs(np.linalg.norm(fk) - 1.0) < 1e-13          # |f_k| = 1
    assert abs(K @ fk) < 1e-13                              # transverse: k . f_k = 0
    curl = 1j * np.cross(K, fk)
    if sigma == 1.0:
        assert np.max(np.abs(curl - kn * fk)) < 1e-13      # positive-helicity curl eigenvector
    assert abs(np.mean(np.sum(F * F, axis=0)) - amp ** 2 / 2) < 1e-12 * amp ** 2
    # kinetic helicity of the forcing: <f . curl f> = sigma-dependent, zero for sigma = 0
    hel = np.real(np.vdot(fk, curl)) / kn
    assert abs(hel - 2 * sigma / (1 + sigma ** 2)) < 1e-13
    # the independent NumPy formula (e projected perpendicular to k) agrees
    assert np.max(np.abs(F - numpy_ref.forcing(p, rec))) < 1e-13 * amp


# ------------------------------------------------------------------ whole RHS

def _spec_d(f, a):
    n = f.shape[2 - a]
    k = np.fft.fftfreq(n, d=1.0 / n)
    if n % 2 == 0:
        k[n // 2] = 0.0
    sh = [1, 1, 1]
    sh[2 - a] = n
    return np.real(np.fft.ifft(np.fft.fft(f, axis=2 - a) * (1j * k).reshape(sh), axis=2 - a))


def _curl(V):
    return np.stack([_spec_d(V[2], 1) - _spec_d(V[1], 2), _spec_d(V[0], 2) - _spec_d(V[2], 0),
                     _spec_d(V[1], 0) - _spec_d(V[0], 1)])


def _budget(n, lorentz_sign_flip=False):
    """(dE/dt from the oracle RHS) - (forcing work - viscous - ohmic), and d(mass)/dt.

    E = sum h^3 [rho u^2/2 + cs^2 rho ln rho + |B|^2/2] obeys, for the continuous
    equations of Section 4, dE/dt = sum h^3 [rho u.f - 2 nu rho S:S - eta j.j].
    Derivatives here are spectral (exact for the band-limited fields used), so the
    residual is the oracle's truncation error alone.
    """
    p = _p(n, nu=0.05, eta=0.04, dt=1e-3)
    st = mi.smooth_state(p, 5, kmax=2, amp_lnrho=0.1, amp_u=0.3, amp_a=0.3, nmodes=4)
    rec = mi.Forcing(k=(2, 1, -2), e=(0.0, 0.6, 0.8), phi=0.3, sigma=0.6, f0=0.02)
    R, _ = oracle.rhs(st, p, rec)
    F = oracle.forcing_field(p, rec)
    lnr, u, A = st[0], st[1:4], st[4:7]
    rho = np.exp(lnr)
    B = _curl(A)
    J = _curl(B)
    if lorentz_sign_flip:
        R = R.copy()
        R[1:4] -= 2.0 * np.cross(J, B, axis=0) / rho
    h3 = (TWO_PI / n) ** 3
    u2 = np.sum(u * u, axis=0)
    dEdt = h3 * np.sum(rho * np.sum(u * R[1:4], axis=0)
                       + (0.5 * u2 + p.cs ** 2 * (lnr + 1.0)) * rho * R[0]
                       + np.sum(J * R[4:7], axis=0))
    du = [[_spec_d(u[c], a) for a in range(3)] for c in range(3)]
    divu = du[0][0] + du[1][1] + du[2][2]
    SS = sum((0.5 * (du[a][b] + du[b][a]) - (divu / 3.0 if a == b else 0.0)) ** 2
             for a in range(3) for b in range(3))
    budget = h3 * np.sum(rho * np.sum(u * F, axis=0) - 2 * p.nu * rho * SS
                         - p.eta * np.sum(J * J, axis=0))
    return abs(dEdt - budget) / abs(budget), abs(h3 * np.sum(rho * R[0]))


def test_energy_budget_and_mass_converge_at_sixth_order():
    r16, m16 = _budget(16)
    r32, m32 = _budget(32)
    assert 45 < r16 / r32 < 80, (r16, r32)
    assert 45 < m16 / m32 < 80, (m16, m32)
    assert r32 < 1e-5
    # a sign error in any conservative exchange (here: the Lorentz force) leaves an O(1) residual
    bad, _ = _budget(32, lorentz_sign_flip=True)
    assert bad > 1e-2


def test_div_curl_is_zero_to_roundoff():
    p = _p(16, 12, 10)
    A = mi.noise_state(p, 4, 0.0, 0.0, 1.0)[4:7]
    h = (p.lx / p.nx, p.ly / p.ny, p.lz / p.nz)
    d = lambda f, a: oracle.deriv(f, h, 1, a)
    B = [d(A[2], 1) - d(A[1], 2), d(A[0], 2) - d(A[2], 0), d(A[1], 0) - d(A[0], 1)]
    div = d(B[0], 0) + d(B[1], 1) + d(B[2], 2)
    assert np.max(np.abs(div)) < 1e-13 * np.max(np.abs(B)) / min(h)


def test_uniform_state_is_an_exact_fixed_point():
    p = _p(9, 10, 11, nu=0.01, eta=0.02, dt=1e-3)
    st = np.zeros((7, p.nz, p.ny, p.nx))
    st[0] = 0.3
    st[1], st[2], st[3] = 0.1, -0.2, 0.05
    st[4], st[5], st[6] = 1.0, 2.0, 3.0
    out, _ = oracle.step(st, p, mi.no_forcing(3))
    assert np.array_equal(out, st)


def test_translation_equivariance():
    p = _p(12, 10, 9, nu=0.02, eta=0.03, dt=2e-3)
    st = mi.noise_state(p, 8, 0.2, 0.2, 0.2)
    rec = mi.Forcing(k=(2, -3, 1), e=(0.3, 0.4, 0.866), phi=0.4, sigma=0.8, f0=0.05)
    sh = (3, 5, 7)  # cells along x, y, z
    rolled = np.roll(st, (sh[2], sh[1], sh[0]), axis=(1, 2, 3))
    dphi = -sum(TWO_PI * rec.k[a] * sh[a] / n for a, n in enumerate((p.nx, p.ny, p.nz)))
    rec2 = mi.Forcing(k=rec.k, e=rec.e, phi=rec.phi + dphi, sigma=rec.sigma, f0=rec.f0)
    a, _ = oracle.step(rolled, p, [rec2])
    b, _ = oracle.step(st, p, [rec])
    b = np.roll(b, (sh[2], sh[1], sh[0]), axis=(1, 2, 3))
    assert np.max(np.abs(a - b)) < 1e-13 * np.max(np.abs(b))


def test_cyclic_axis_permutation_equivariance():
    # new x = old z, new y = old x, new z = old y (a proper rotation: helicity is kept)
    p = _p(10, 12, 14, nu=0.02, eta=0.03, dt=2e-3)
    st = mi.noise_state(p, 9, 0.2, 0.2, 0.2)
    rec = mi.Forcing(k=(1, -2, 2), e=(0.48, 0.6, 0.64), phi=-1.1, sigma=1.0, f0=0.05)

    def perm_state(s):
        t = np.transpose(s, (0, 2, 3, 1))  # array axes (z, y, x) -> (old y, old x, old z)
        return np.ascontiguousarray(t[[0, 3, 1, 2, 6, 4, 5]])

    def perm_vec(v):
        return (v[2], v[0], v[1])

    q = _p(p.nz, p.nx, p.ny, nu=p.nu, eta=p.eta, dt=p.dt)
    rq = mi.Forcing(k=perm_vec(rec.k), e=perm_vec(rec.e), phi=rec.phi, sigma=rec.sigma, f0=rec.f0)
    a, _ = oracle.step(perm_state(st), q, [rq])
    b, _ = oracle.step(st, p, [rec])
    assert np.max(np.abs(a - perm_state(b))) < 1e-13 * np.max(np.abs(b))


def test_c_oracle_matches_independent_numpy_brute_force_8cubed():
    p = _p(8, nu=5e-3, eta=7e-3, dt=1e-3, bext=(0.01, -0.02, 0.03))
    st = mi.noise_state(p, 3, 0.3, 0.3, 0.3)
    recs = mi.forcing_schedule(1, 2, 3.0, 0.02, 0.7)
    R, _ = oracle.rhs(st, p, recs[0])
    R2 = numpy_ref.rhs(st, p, recs[0])
    assert np.max(np.abs(R - R2)) <= 1e-13 * np.max(np.abs(R))
    s1, _ = oracle.step(st, p, recs)
    s2 = numpy_ref.step(st, p, recs)
    assert np.max(np.abs(s1 - s2)) <= 1e-13 * np.max(np.abs(s1))


# ------------------------------------------------------------------ upwinding (Section 4)

@pytest.mark.parametrize("c", [1.0, 0.4])
def test_upwinding_matches_one_sided_fifth_order_stencils(c):
    """The C oracle's correction form against the NumPy reference, which takes each
    advective product with the six-point stencil (derived from the Taylor conditions)
    that leans against the flow; random velocities of both signs, ragged grid."""
    p = _p(9, 8, 10, nu=5e-3, eta=7e-3, dt=1e-3, upwind=c)
    st = mi.noise_state(p, 41, 0.3, 0.6, 0.3)
    rec = mi.forcing_schedule(2, 1, 3.0, 0.02, 0.3)[0]
    R, _ = oracle.rhs(st, p, rec)
    R2 = numpy_ref.rhs(st, p, rec)
    assert np.max(np.abs(R[0] - R2[0])) <= 1e-13 * np.max(np.abs(R[0]))
    assert np.max(np.abs(R[1:] - R2[1:])) <= 1e-13 * np.max(np.abs(R[1:]))
    q = _p(9, 8, 10, nu=5e-3, eta=7e-3, dt=1e-3)
    R0, _ = oracle.rhs(st, q, rec)
    assert np.max(np.abs(R[0] - R0[0])) > 1e-6 * np.max(np.abs(R0[0]))  # the term is there
    assert np.array_equal(R[1:], R0[1:])                                 # and nowhere else


def test_upwinding_of_a_single_mode_has_the_sixth_difference_symbol():
    """Uniform u, ln rho = eps sin(k.x): the added term is -|u_a| 64 sin^6(k_a h/2) / (60 h)
    times ln rho per axis (a damping), and it is zero when u = 0."""
    n, eps = 16, 1e-3
    p = _p(n, upwind=1.0)
    X, Y, Z = _coords(p)
    k = (2, 3, 1)
    u = (0.7, -0.4, 0.25)
    lnr = eps * np.sin(k[0] * X + k[1] * Y + k[2] * Z)
    st = np.zeros((7,) + X.shape)
    st[0] = lnr
    for a in range(3):
        st[1 + a] = u[a]
    R, _ = oracle.rhs(st, p, NOFORCE)
    R0, _ = oracle.rhs(st, _p(n), NOFORCE)
    h = TWO_PI / n
    sym = -sum(abs(u[a]) * 64.0 * math.sin(k[a] * h / 2) ** 6 / (60.0 * h) for a in range(3))
    assert np.max(np.abs((R[0] - R0[0]) - sym * lnr)) <= 1e-12 * eps
    st[1:4] = 0.0
    R, _ = oracle.rhs(st, p, NOFORCE)
    assert np.max(np.abs(R[0])) == 0.0


def test_upwinding_correction_vanishes_at_fifth_order():
    ratios = []
    prev = None
    for n in (24, 48):
        p = _p(n, upwind=1.0)
        X, Y, Z = _coords(p)
        st = np.zeros((7,) + X.shape)
        st[0] = 0.1 * np.sin(X) * np.cos(2 * Y + Z)
        st[1] = 0.3 * np.cos(Y)
        st[2] = -0.2 * np.sin(Z + X)
        st[3] = 0.1
        R, _ = oracle.rhs(st, p, NOFORCE)
        R0, _ = oracle.rhs(st, _p(n), NOFORCE)
        e = np.max(np.abs(R[0] - R0[0]))
        if prev is not None:
            ratios.append(prev / e)
        prev = e
    assert 28.0 < ratios[0] < 36.0, ratios  # 2^5 = 32


def test_step_cells_matches_full_step():
    p = _p(12, 11, 13, nu=4e-3, eta=6e-3, dt=1e-3)
    st = mi.noise_state(p, 21, 0.3, 0.3, 0.3)
    rec = mi.forcing_schedule(4, 1, 3.0, 0.02, 1.0)[0]
    full, _ = oracle.step(st, p, [rec])
    cells = np.array([0, 1, p.nx - 1, p.ncell - 1, p.nx * p.ny * 5 + 7, 777, 1234])
    out = oracle.step_cells(st, p, rec, cells)
    assert np.max(np.abs(out - full.reshape(7, -1)[:, cells].T)) <= 1e-15 * np.max(np.abs(full))


# ------------------------------------------------------------------ diagnostics

def test_diagnostics_closed_forms():
    p = _p(16, 16, 32)
    X, _, Z = _coords(p)
    st = np.zeros((7, p.nz, p.ny, p.nx))
    U, c = 0.3, 0.2
    st[0] = c
    st[1] = U * np.sin(2 * X)      # max |u| is attained at x = pi/4 (i = 2)
    k = 3
    st[4] = np.sin(k * Z) / k
    st[5] = np.cos(k * Z) / k
    d = oracle.diag(st, p)
    h = TWO_PI / 32
    assert abs(d["urms"] - U / math.sqrt(2)) < 1e-15
    assert abs(d["ek"] - 0.5 * math.exp(c) * U ** 2 / 2) < 1e-15
    assert abs(d["umax"] - U) < 1e-15
    assert abs(d["lnrho_mean"] - c) < 1e-15
    assert abs(d["em"] - 0.5 * (keff(k, h) / k) ** 2) < 1e-15
    assert abs(d["brms"] - keff(k, h) / k) < 1e-15
    assert d["nonfinite"] == 0
    st[3, 1, 2, 3] = np.nan
    st[6, 4, 5, 6] = np.inf
    assert oracle.diag(st, p)["nonfinite"] == 2


def test_growth_rate_fit_is_exact_on_an_exponential():
    t = np.arange(200) * 1e-3
    lam = 0.0173
    assert abs(oracle.growth_rate(t, 1e-5 * np.exp(lam * t)) - lam) < 1e-10
    assert abs(oracle.growth_rate(t, 3.0 * np.exp(-0.8 * t), 100, 200) + 0.8) < 1e-10


# ------------------------------------------------------------------ magnetic spectrum

@pytest.mark.parametrize("axis", [0, 1, 2])
def test_spectrum_of_a_beltrami_field_is_one_shell(axis):
    # A = (sin kz, cos kz, 0)/k and its cyclic permutations: the discrete B is a
    # single Fourier shell |k| with |B|^2 = (k_eff/k)^2 everywhere, so the whole energy
    # (1/2) V (k_eff/k)^2 sits in shell k (dk = 1 for L = 2 pi).
    p = _p(32, 24, 20)
    X = _coords(p)
    k = 3
    h = (p.lx / p.nx, p.ly / p.ny, p.lz / p.nz)[axis]
    st = np.zeros((7,) + X[0].shape)
    a, b = (axis + 1) % 3, (axis + 2) % 3
    st[4 + a] = np.sin(k * X[axis]) / k
    st[4 + b] = np.cos(k * X[axis]) / k
    E, dk = oracle.magnetic_spectrum(st, p)
    assert dk == 1.0
    assert len(E) == oracle.spectrum_nshell(p) == int(math.floor(math.sqrt(16 ** 2 + 12 ** 2 + 10 ** 2) + 0.5)) + 1
    want = 0.5 * TWO_PI ** 3 * (keff(k, h) / k) ** 2
    assert abs(E[k] - want) <= 1e-13 * want
    assert np.max(np.abs(np.delete(E, k))) <= 1e-14 * want


@pytest.mark.parametrize("kvec,shell", [((1, 2, 2), 3), ((3, 0, -4), 5), ((-2, 3, 6), 7)])
def test_spectrum_of_an_oblique_mode(kvec, shell):
    # A = a cos(k.x + phi): B = -sin(k.x + phi) (kappa x a) with kappa_a the sixth-order
    # modified wavenumber of axis a, so <|B|^2> = |kappa x a|^2 / 2 and the shell |k|
    # holds V |kappa x a|^2 / 4.
    p = _p(16, 12, 14)
    X = _coords(p)
    a = np.array([0.3, -0.2, 0.5])
    th = kvec[0] * X[0] + kvec[1] * X[1] + kvec[2] * X[2] + 0.7
    st = np.zeros((7,) + X[0].shape)
    for c in range(3):
        st[4 + c] = a[c] * np.cos(th)
    hs = (p.lx / p.nx, p.ly / p.ny, p.lz / p.nz)
    kap = np.array([math.copysign(keff(abs(kk), hh), kk) for kk, hh in zip(kvec, hs)])
    want = TWO_PI ** 3 * float(np.sum(np.cross(kap, a) ** 2)) / 4
    E, _ = oracle.magnetic_spectrum(st, p)
    assert abs(E[shell] - want) <= 1e-13 * want
    assert np.max(np.abs(np.delete(E, shell))) <= 1e-14 * want


def test_spectrum_matches_a_direct_fourier_sum_on_a_small_box():
    # Brute force from the definition on a non-cubic box: B from the np.roll stencils,
    # B_hat(k) = sum_x B(x) exp(-i k.x) summed directly with physical k and x, every
    # wavevector placed by |k| / dk rounded to the nearest shell, dk = 2 pi / max(L).
    p = _p(8, 6, 10, lx=TWO_PI, ly=3.1, lz=7.3, bext=(0.05, -0.1, 0.02))
    st = mi.noise_state(p, 5, 0.0, 0.0, 0.4)
    h = (p.lx / p.nx, p.ly / p.ny, p.lz / p.nz)
    A = st[4:7]
    B = np.stack([numpy_ref.d1(A[2], 1, h[1]) - numpy_ref.d1(A[1], 2, h[2]),
                  numpy_ref.d1(A[0], 2, h[2]) - numpy_ref.d1(A[2], 0, h[0]),
                  numpy_ref.d1(A[1], 0, h[0]) - numpy_ref.d1(A[0], 1, h[1])])
    B += np.array(p.bext)[:, None, None, None]
    xs = [np.arange(n) * L / n for n, L in ((p.nx, p.lx), (p.ny, p.ly), (p.nz, p.lz))]
    dk = TWO_PI / max(p.lx, p.ly, p.lz)
    vol = p.lx * p.ly * p.lz
    E = {}
    margin = 1.0
    for mz in range(-(p.nz // 2), (p.nz + 1) // 2):
        for my in range(-(p.ny // 2), (p.ny + 1) // 2):
            for mx in range(-(p.nx // 2), (p.nx + 1) // 2):
                kp = (TWO_PI * mx / p.lx, TWO_PI * my / p.ly, TWO_PI * mz / p.lz)
                ph = np.exp(-1j * (kp[2] * xs[2][:, None, None] + kp[1] * xs[1][None, :, None]
                                   + kp[0] * xs[0][None, None, :]))
                pw = sum(abs(np.sum(B[c] * ph)) ** 2 for c in range(3))
                s = math.sqrt(kp[0] ** 2 + kp[1] ** 2 + kp[2] ** 2) / dk
                margin = min(margin, abs(s - math.floor(s) - 0.5))
                E[int(math.floor(s + 0.5))] = E.get(int(math.floor(s + 0.5)), 0.0) + pw
    assert margin > 1e-6  # no wavevector near a shell boundary: the rounding is unambiguous
    n2 = float(p.ncell) ** 2
    got, dk_o = oracle.magnetic_spectrum(st, p)
    assert abs(dk_o - dk) < 1e-15
    want = np.zeros(len(got))
    for s, v in E.items():
        want[s] = v * vol / (2 * dk * n2)
    assert np.max(np.abs(got - want)) <= 1e-13 * np.sum(want)


def test_spectrum_sums_to_the_magnetic_energy_with_a_mean_field():
    # Parseval: sum_s E_B(s) dk = (1/2) int |B|^2 dV = V E_M, and the uniform field
    # B_ext alone fills shell 0 with (1/2) V |B_ext|^2 / dk.
    p = _p(12, 10, 16, lx=5.0, ly=TWO_PI, lz=4.0, bext=(0.1, -0.2, 0.05))
    st = mi.noise_state(p, 9, 0.2, 0.2, 0.3)
    E, dk = oracle.magnetic_spectrum(st, p)
    vol = p.lx * p.ly * p.lz
    em = oracle.diag(st, p)["em"]
    assert abs(np.sum(E) * dk - vol * em) <= 1e-13 * vol * em
    assert abs(E[0] * dk - 0.5 * vol * (0.1 ** 2 + 0.2 ** 2 + 0.05 ** 2)) <= 1e-13 * vol * em


def test_channel_growth_rate_of_a_decaying_beltrami_field_equals_the_rms_rate():
    # With u = 0 and a Beltrami A the discrete system is linear: each step multiplies A
    # by G(-eta k2^2 dt), the RK3 polynomial.  The channel E_B(k) ~ exp(2 lambda_k t)
    # and B_rms ~ exp(lambda t) then give the same lambda = ln|G| / dt.
    p = _p(16, eta=2e-2, dt=5e-3)
    X = _coords(p)
    k = 2
    st = np.zeros((7,) + X[0].shape)
    st[4] = np.sin(k * X[2]) / k
    st[5] = np.cos(k * X[2]) / k
    ts, ek, br = [], [], []
    for n in range(6):
        ts.append(n * p.dt)
        ek.append(oracle.magnetic_spectrum(st, p)[0][k])
        br.append(oracle.diag(st, p)["brms"])
        st, _ = oracle.step(st, p, [NOFORCE])
    h = TWO_PI / 16
    lam = math.log(abs(rk3_poly(-p.eta * k2eff(k, h) ** 2 * p.dt))) / p.dt
    assert abs(oracle.spectral_growth_rate(ts, ek) - lam) < 1e-10
    assert abs(oracle.growth_rate(ts, br) - lam) < 1e-10


# ------------------------------------------------------------------ tolerance scale T_f
#
# The parity bar divides by max(||f||, dt * T_f) with T_f = sum over the field's
# right-hand-side terms of max |term| (largest over the step's substeps).  These pins
# fix every term slot on states where each term has a closed form in the modified
# wavenumbers of the stencils, so that a term filed under the wrong index, counted
# twice or left out changes a slot that is checked here.
#
# Slots per field: ln rho: |u.grad ln rho|, sum_a |d_a u_a|, |upwinding|;
# u_c: |advection|, |pressure|, |Lorentz|, |nu lap u|, |nu/3 grad div u|,
#      |2 nu S.grad ln rho|, |forcing|;  A_c: |(u x B)_c|, |eta lap A_c|.

def _terms_all(st, p, rec=NOFORCE):
    cells = np.arange(p.ncell, dtype=np.int64)
    t = oracle.terms_cells(st, p, rec, cells)  # (ncell, 7, 7)
    return t.reshape(p.nz, p.ny, p.nx, 7, 7)


def _close(got, want, scale):
    assert np.max(np.abs(got - want)) <= 1e-12 * scale, (np.max(np.abs(got - want)), scale)


def test_term_slots_shear_lorentz_and_induction_closed_forms():
    # ln rho = eps sin(a x), u = (U sin(b y), 0, W), A = (0, 0, al sin(c x))
    p = _p(16, 16, 8, nu=0.03, eta=0.02, cs=1.3)
    X, Y, _ = _coords(p)
    h = TWO_PI / 16
    eps, U, W, al = 0.3, 0.7, 0.4, 0.9
    a, b, c = 2, 3, 1
    st = np.zeros((7, p.nz, p.ny, p.nx))
    st[0] = eps * np.sin(a * X)
    st[1] = U * np.sin(b * Y)
    st[3] = W
    st[6] = al * np.sin(c * X)
    t = _terms_all(st, p)
    a1, b1, c1 = keff(a, h), keff(b, h), keff(c, h)
    b2, c2 = k2eff(b, h) ** 2, k2eff(c, h) ** 2
    dlx = eps * a1 * np.cos(a * X)            # d_x ln rho (the only gradient component)
    dyux = U * b1 * np.cos(b * Y)             # d_y u_x (the only velocity gradient)
    By = -al * c1 * np.cos(c * X)             # B = curl A = (0, B_y, 0)
    jz = al * c2 * np.sin(c * X)              # j = grad div A - lap A = (0, 0, j_z)
    zero = np.zeros_like(X)
    want = {
        (0, 0): np.abs(U * np.sin(b * Y) * dlx), (0, 1): zero, (0, 2): zero,
        (1, 0): zero, (1, 1): p.cs ** 2 * np.abs(dlx),
        (1, 2): np.abs(np.exp(-st[0]) * (-jz * By)), (1, 3): p.nu * b2 * np.abs(U * np.sin(b * Y)),
        (1, 4): zero, (1, 5): zero, (1, 6): zero,
        (2, 0): zero, (2, 1): zero, (2, 2): zero, (2, 3): zero, (2, 4): zero,
        # 2 nu S_yx d_x ln rho, S_yx = (d_y u_x)/2
        (2, 5): p.nu * np.abs(dyux * dlx), (2, 6): zero,
        (3, 0): zero, (3, 1): zero, (3, 2): zero, (3, 3): zero, (3, 4): zero, (3, 5): zero,
        (3, 6): zero,
        (4, 0): np.abs(W * By), (4, 1): zero,                 # (u x B)_x = -u_z B_y
        (5, 0): zero, (5, 1): zero,
        (6, 0): np.abs(U * np.sin(b * Y) * By),               # (u x B)_z = u_x B_y
        (6, 1): p.eta * c2 * np.abs(al * np.sin(c * X)),
    }
    for (f, s), w in want.items():
        _close(t[..., f, s], w, 1.0)
    # slots that no field has are left at zero
    assert np.all(t[..., 0, 3:] == 0.0) and np.all(t[..., 4:, 2:] == 0.0)


def test_term_slots_compressive_flow_closed_forms():
    # u = (U sin(a x), 0, 0), ln rho = eps sin(b y): advection, grad div, the trace part
    # of the strain and the divergence slot of ln rho
    p = _p(16, 16, 8, nu=0.05, cs=0.8)
    X, Y, _ = _coords(p)
    h = TWO_PI / 16
    U, eps, a, b = 0.6, 0.25, 2, 1
    st = np.zeros((7, p.nz, p.ny, p.nx))
    st[1] = U * np.sin(a * X)
    st[0] = eps * np.sin(b * Y)
    t = _terms_all(st, p)
    a1, a2, b1 = keff(a, h), k2eff(a, h) ** 2, keff(b, h)
    dxux = U * a1 * np.cos(a * X)
    dly = eps * b1 * np.cos(b * Y)
    zero = np.zeros_like(X)
    _close(t[..., 0, 0], zero, 1.0)                                   # u_x d_x ln rho = 0
    _close(t[..., 0, 1], np.abs(dxux), 1.0)
    _close(t[..., 1, 0], np.abs(U * np.sin(a * X) * dxux), 1.0)       # u_x d_x u_x
    _close(t[..., 1, 3], p.nu * a2 * np.abs(U * np.sin(a * X)), 1.0)
    _close(t[..., 1, 4], p.nu / 3.0 * a2 * np.abs(U * np.sin(a * X)), 1.0)
    _close(t[..., 1, 5], zero, 1.0)                                   # S_xy = 0, d_x ln rho = 0
    _close(t[..., 2, 1], p.cs ** 2 * np.abs(dly), 1.0)
    # 2 nu S_yy d_y ln rho with the traceless S_yy = -(div u)/3
    _close(t[..., 2, 5], 2.0 * p.nu / 3.0 * np.abs(dxux * dly), 1.0)
    for f, s in [(1, 1), (1, 2), (2, 0), (2, 3), (2, 4), (3, 5)]:
        _close(t[..., f, s], zero, 1.0)


def test_term_slots_upwinding_and_forcing():
    # uniform u_x = U under ln rho = eps sin(a x): the upwinding slot is the sixth-difference
    # symbol; with a forcing record, the forcing slot is |f| of the forcing field
    p = _p(16, 8, 8, upwind=0.7)
    X, _, _ = _coords(p)
    h = TWO_PI / 16
    U, eps, a = 0.5, 0.2, 3
    st = np.zeros((7, p.nz, p.ny, p.nx))
    st[1] = U
    st[0] = eps * np.sin(a * X)
    rec = mi.forcing_schedule(4, 1, 3.0, 0.05, 0.5)[0]
    t = _terms_all(st, p, rec)
    sym = 64.0 * math.sin(a * h / 2) ** 6
    _close(t[..., 0, 2], p.upwind * U * eps * sym * np.abs(np.sin(a * X)) / (60.0 * h), 1.0)
    F = oracle.forcing_field(p, rec)
    for c in range(3):
        _close(t[..., 1 + c, 6], np.abs(F[c]), max(1.0, np.max(np.abs(F))))


def test_rhs_termmax_is_the_largest_term_over_cells():
    p = _p(12, 10, 8, nu=0.02, eta=0.01)
    st = mi.smooth_state(p, 3, kmax=2, amp_lnrho=0.2, amp_u=0.4, amp_a=0.4, nmodes=3)
    rec = mi.forcing_schedule(2, 1, 3.0, 0.05, 1.0)[0]
    _, tm = oracle.rhs(st, p, rec)
    t = _terms_all(st, p, rec)
    assert np.array_equal(tm, t.reshape(-1, 7, 7).max(axis=0))


def test_step_tscale_of_a_shear_wave():
    # u = (0, U sin kx, 0) stays a shear wave: only nu lap u_y is non-zero, largest in
    # substep 1 (the amplitude decays), and its maximum over the grid is nu k2^2 U
    p = _p(32, 4, 4, nu=0.2, eta=0.1, dt=0.01)
    X, _, _ = _coords(p)
    U, k = 0.3, 2  # the grid holds x = pi/4 where sin(2x) = 1
    st = np.zeros((7, p.nz, p.ny, p.nx))
    st[2] = U * np.sin(k * X)
    _, ts = oracle.step(st, p, mi.no_forcing(1))
    want = np.array([0.0, 0.0, p.nu * k2eff(k, TWO_PI / 32) ** 2 * U, 0.0, 0.0, 0.0, 0.0])
    assert np.all(ts[0][want == 0.0] == 0.0), ts
    assert abs(ts[0][2] - want[2]) <= 1e-13 * want[2], ts


def test_step_tscale_of_a_beltrami_field():
    # A = (sin kz, cos kz, 0)/k, u = 0: A decays by diffusion only (T = eta k2^2 / k for
    # A_x and A_y, 0 for A_z); j x B vanishes up to roundoff, so the u and ln rho scales
    # are roundoff-sized
    p = _p(8, 8, 32, eta=0.1, nu=0.05, dt=0.01)
    _, _, Z = _coords(p)
    k = 2
    st = np.zeros((7, p.nz, p.ny, p.nx))
    st[4] = np.sin(k * Z) / k
    st[5] = np.cos(k * Z) / k
    _, ts = oracle.step(st, p, mi.no_forcing(1))
    w = p.eta * k2eff(k, TWO_PI / 32) ** 2 / k
    assert abs(ts[0][4] - w) <= 1e-13 * w and abs(ts[0][5] - w) <= 1e-13 * w, ts
    assert ts[0][6] == 0.0
    assert np.all(ts[0][:4] < 1e-12 * w), ts


def test_step_tscale_sums_the_terms_of_a_field():
    # sound wave ln rho = eps sin(kx), u = 0: in substep 1 only the pressure acts on u_x;
    # later substeps add u_x-driven terms of order dt, so T(u_x) = cs^2 eps keff (1 + O(dt))
    # and T(ln rho) = sum of |u.grad ln rho| and |d_x u_x|, both of order dt
    p = _p(32, 4, 4, nu=0.01, dt=1e-4)
    X, _, _ = _coords(p)
    eps, k = 0.01, 3
    st = np.zeros((7, p.nz, p.ny, p.nx))
    st[0] = eps * np.sin(k * X)
    _, ts = oracle.step(st, p, mi.no_forcing(1))
    h = TWO_PI / 32
    pres = p.cs ** 2 * eps * keff(k, h)
    assert abs(ts[0][1] - pres) <= 2e-3 * pres, ts
    # ln rho: after substep 2, u_x ~ (beta1 + ...) dt * pres; d_x u_x ~ keff u_x
    assert 0.0 < ts[0][0] < 2.0 * p.dt * pres * keff(k, h), ts
    assert np.all(ts[0][2:] == 0.0), ts


def test_tolerance_error_uses_the_larger_of_field_norm_and_term_floor():
    ora = np.zeros((7, 2, 2, 2))
    ora[1, 0, 0, 0] = 2.0          # ||u_x|| = 2
    gpu = ora.copy()
    gpu[1, 1, 1, 1] += 1e-6        # error 1e-6 in u_x
    gpu[0, 0, 0, 1] += 3e-9        # error 3e-9 in ln rho, whose norm is 0
    ts = np.array([5.0, 1e5, 0, 0, 0, 0, 0])
    e, plain = oracle.tolerance_error(gpu, ora, ts, 1e-3)
    assert abs(e[1] - 1e-6 / max(2.0, 1e-3 * 1e5)) < 1e-20   # the term floor 100 wins
    assert abs(e[0] - 3e-9 / (1e-3 * 5.0)) < 1e-20            # norm 0: the floor alone
    assert abs(plain[1] - 5e-7) < 1e-20 and plain[0] == 3e-9
    assert np.all(e[2:] == 0.0)


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_term_slots_compression_along_each_axis(axis):
    # u_a = V sin(k x_a) along one axis a: every slot that holds d_a u_a or d_a d_a u_a
    p = _p(16, 12, 20, nu=0.04)
    C3 = _coords(p)
    n = (p.nx, p.ny, p.nz)[axis]
    h = TWO_PI / n
    V, k = 0.8, 2
    st = np.zeros((7, p.nz, p.ny, p.nx))
    s = np.sin(k * C3[axis])
    st[1 + axis] = V * s
    t = _terms_all(st, p)
    k1, k2 = keff(k, h), k2eff(k, h) ** 2
    dadua = V * k1 * np.cos(k * C3[axis])
    _close(t[..., 0, 1], np.abs(dadua), 1.0)
    _close(t[..., 1 + axis, 0], np.abs(V * s * dadua), 1.0)
    _close(t[..., 1 + axis, 3], p.nu * k2 * np.abs(V * s), 1.0)
    _close(t[..., 1 + axis, 4], p.nu / 3.0 * k2 * np.abs(V * s), 1.0)
    for b in range(3):
        if b != axis:
            assert np.all(t[..., 1 + b, :6] == 0.0)
