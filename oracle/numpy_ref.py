"""Independent whole-array NumPy implementation of the same discrete update (tiny grids only).

TEST INFRASTRUCTURE (see the package docstring).  Written separately from the C
oracle so the two can check each other: stencil weights are *derived* here by
solving the Taylor (moment) conditions instead of being typed in, derivatives use
``np.roll`` on whole arrays, and the forcing uses the unit vector projected
perpendicular to k, for which Eq. feigen reduces to
f_k = -(e' + i sigma k^ x e') / sqrt(1 + sigma^2).
"""
from __future__ import annotations

import math
from fractions import Fraction

import numpy as np


def _solve_exact(rows, rhs):
    """Gaussian elimination over rationals (exact stencil weights)."""
    n = len(rows)
    M = [[Fraction(x) for x in r] + [Fraction(b)] for r, b in zip(rows, rhs)]
    for c in range(n):
        piv = next(r for r in range(c, n) if M[r][c] != 0)
        M[c], M[piv] = M[piv], M[c]
        for r in range(n):
            if r != c and M[r][c] != 0:
                f = M[r][c] / M[c][c]
                M[r] = [a - f * b for a, b in zip(M[r], M[c])]
    return [M[r][n] / M[r][r] for r in range(n)]


def central_weights(order: int, radius: int = 3):
    """Weights w_m (m = -radius..radius) with sum_m w_m m^q / q! = [q == order], q < 2 radius + 1.

    The unique 2r+1 point central stencil for the derivative of that order.
    """
    offs = list(range(-radius, radius + 1))
    rows = [[Fraction(m) ** q / math.factorial(q) for m in offs] for q in range(len(offs))]
    rhs = [1 if q == order else 0 for q in range(len(offs))]
    return dict(zip(offs, _solve_exact(rows, rhs)))


def one_sided_weights(lo: int, hi: int):
    """First-derivative weights on offsets lo..hi (6 points: exact to degree 5)."""
    offs = list(range(lo, hi + 1))
    rows = [[Fraction(m) ** q / math.factorial(q) for m in offs] for q in range(len(offs))]
    rhs = [1 if q == 1 else 0 for q in range(len(offs))]
    return dict(zip(offs, _solve_exact(rows, rhs)))


W1 = {m: float(w) for m, w in central_weights(1).items()}
# fifth-order upwind-biased first derivatives: for flow in +a the stencil leans back
# (offsets -3..2), for flow in -a forward (-2..3)
WUP_POS = {m: float(w) for m, w in one_sided_weights(-3, 2).items()}
WUP_NEG = {m: float(w) for m, w in one_sided_weights(-2, 3).items()}
W2 = {m: float(w) for m, w in central_weights(2).items()}


def _shift(f, axis, m):
    """g[i] = f[i + m] along the given array axis (periodic)."""
    return np.roll(f, -m, axis=axis)


# array axes for spatial directions x, y, z of a (nz, ny, nx) array
_AX = {0: 2, 1: 1, 2: 0}


def d1(f, a, h):
    return sum(w * _shift(f, _AX[a], m) for m, w in W1.items() if w != 0.0) / h


def d2(f, a, h):
    return sum(w * _shift(f, _AX[a], m) for m, w in W2.items()) / (h * h)


def dab(f, a, b, ha, hb):
    """d_a d_b by the diagonal second differences: [D2 along (a+b) - D2 along (a-b)] / (4 ha hb)."""
    acc = np.zeros_like(f)
    for m, w in W2.items():
        if m == 0:
            continue
        pp = _shift(_shift(f, _AX[a], m), _AX[b], m)
        pm = _shift(_shift(f, _AX[a], m), _AX[b], -m)
        acc += w * (pp - pm)
    return acc / (4.0 * ha * hb)


def forcing(p, rec):
    if rec.f0 == 0.0:
        return np.zeros((3, p.nz, p.ny, p.nx))
    K = np.array([2 * math.pi * rec.k[0] / p.lx, 2 * math.pi * rec.k[1] / p.ly,
                  2 * math.pi * rec.k[2] / p.lz])
    kn = float(np.linalg.norm(K))
    kh = K / kn
    e = np.asarray(rec.e, dtype=float)
    ep = e - kh * float(kh @ e)
    ep /= np.linalg.norm(ep)
    fk = -(ep + 1j * rec.sigma * np.cross(kh, ep)) / math.sqrt(1.0 + rec.sigma ** 2)
    amp = rec.f0 * p.cs * math.sqrt(kn * p.cs / p.dt)
    x = np.arange(p.nx) * (p.lx / p.nx)
    y = np.arange(p.ny) * (p.ly / p.ny)
    z = np.arange(p.nz) * (p.lz / p.nz)
    th = (K[0] * x[None, None, :] + K[1] * y[None, :, None] + K[2] * z[:, None, None]) + rec.phi
    ph = np.exp(1j * th)
    return np.stack([np.real(amp * fk[c] * ph) for c in range(3)])


def rhs(state, p, rec):
    h = (p.lx / p.nx, p.ly / p.ny, p.lz / p.nz)
    lnr = state[0]
    u = state[1:4]
    A = state[4:7]
    glnr = [d1(lnr, a, h[a]) for a in range(3)]
    du = [[d1(u[c], a, h[a]) for a in range(3)] for c in range(3)]
    dA = [[d1(A[c], a, h[a]) for a in range(3)] for c in range(3)]
    lap = lambda f: d2(f, 0, h[0]) + d2(f, 1, h[1]) + d2(f, 2, h[2])

    def grad_div(V):
        out = []
        for c in range(3):
            acc = d2(V[c], c, h[c])
            for b in range(3):
                if b != c:
                    acc = acc + dab(V[b], c, b, h[c], h[b])
            out.append(acc)
        return out

    gdu = grad_div(u)
    gdA = grad_div(A)
    lapu = [lap(u[c]) for c in range(3)]
    lapA = [lap(A[c]) for c in range(3)]
    J = [gdA[c] - lapA[c] for c in range(3)]
    B = [dA[2][1] - dA[1][2] + p.bext[0], dA[0][2] - dA[2][0] + p.bext[1],
         dA[1][0] - dA[0][1] + p.bext[2]]
    divu = du[0][0] + du[1][1] + du[2][2]
    S = [[0.5 * (du[a][b] + du[b][a]) - (divu / 3.0 if a == b else 0.0) for b in range(3)]
         for a in range(3)]
    F = forcing(p, rec)
    rho_inv = np.exp(-lnr)
    R = np.empty_like(state)
    R[0] = -(u[0] * glnr[0] + u[1] * glnr[1] + u[2] * glnr[2]) - divu
    c = float(getattr(p, "upwind", 0.0))
    if c != 0.0:
        # the advective products with the upwind-biased stencils, blended by c
        up = np.zeros_like(lnr)
        for a in range(3):
            dpos = sum(w * _shift(lnr, _AX[a], m) for m, w in WUP_POS.items()) / h[a]
            dneg = sum(w * _shift(lnr, _AX[a], m) for m, w in WUP_NEG.items()) / h[a]
            up += u[a] * np.where(u[a] > 0, dpos, dneg)
        R[0] = -(1.0 - c) * (u[0] * glnr[0] + u[1] * glnr[1] + u[2] * glnr[2]) - c * up - divu
    jxB = np.cross(np.stack(J), np.stack(B), axis=0)
    uxB = np.cross(u, np.stack(B), axis=0)
    for c in range(3):
        adv = u[0] * du[c][0] + u[1] * du[c][1] + u[2] * du[c][2]
        visc = p.nu * (lapu[c] + gdu[c] / 3.0
                       + 2.0 * (S[c][0] * glnr[0] + S[c][1] * glnr[1] + S[c][2] * glnr[2]))
        R[1 + c] = -adv - p.cs ** 2 * glnr[c] + rho_inv * jxB[c] + visc + F[c]
        R[4 + c] = uxB[c] + p.eta * lapA[c]
    return R


ALPHA = (0.0, -5.0 / 9.0, -153.0 / 128.0)
BETA = (1.0 / 3.0, 15.0 / 16.0, 8.0 / 15.0)


def step(state, p, recs):
    f = np.array(state, dtype=np.float64, copy=True)
    for rec in recs:
        w = np.zeros_like(f)
        for s in range(3):
            w = ALPHA[s] * w + p.dt * rhs(f, p, rec)
            f = f + BETA[s] * w
    return f
