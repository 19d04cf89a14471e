"""Analytic data for the acoustic wave system (problem data only).

The first-order system (eq. 2.1) is written for (v, sigma) with v = dU/dt and
sigma = -grad U, where U solves the second-order wave equation (eq. 2.2).  Each
field below returns U, v and sigma at space-time points; initial data are the
t = 0 values and Dirichlet data g_D are the values of v on the boundary.

All functions take x of shape (..., n) and t broadcastable to x[..., 0].
"""
from __future__ import annotations

import numpy as np


class Field:
    """A solution of the second-order wave equation with its first-order
    fields.  Subclasses implement ``U``, ``v`` and ``sigma``."""

    def U(self, x, t):  # pragma: no cover - interface
        raise NotImplementedError

    def v(self, x, t):  # pragma: no cover - interface
        raise NotImplementedError

    def sigma(self, x, t):  # pragma: no cover - interface
        raise NotImplementedError


class StandingWave1D(Field):
    """U = sin(pi x) cos(pi t) on [0,1], c = 1 (the 1+1D standing wave)."""

    def U(self, x, t):
        return np.sin(np.pi * x[..., 0]) * np.cos(np.pi * t)

    def v(self, x, t):
        return -np.pi * np.sin(np.pi * x[..., 0]) * np.sin(np.pi * t)

    def sigma(self, x, t):
        return (-np.pi * np.cos(np.pi * x[..., 0]) * np.cos(np.pi * t))[..., None]


class SinSin1D(Field):
    """U = sin(pi x) sin(pi t) (the energy test problem of Sec. 6.5)."""

    def U(self, x, t):
        return np.sin(np.pi * x[..., 0]) * np.sin(np.pi * t)

    def v(self, x, t):
        return np.pi * np.sin(np.pi * x[..., 0]) * np.cos(np.pi * t)

    def sigma(self, x, t):
        return (-np.pi * np.cos(np.pi * x[..., 0]) * np.sin(np.pi * t))[..., None]


class PlaneWave(Field):
    """U = cos(k.x - c|k| t): a plane wave travelling along k."""

    def __init__(self, k, c: float = 1.0):
        self.k = np.asarray(k, dtype=np.float64)
        self.c = float(c)
        self.w = self.c * float(np.linalg.norm(self.k))

    def _arg(self, x, t):
        return x @ self.k - self.w * t

    def U(self, x, t):
        return np.cos(self._arg(x, t))

    def v(self, x, t):
        return self.w * np.sin(self._arg(x, t))

    def sigma(self, x, t):
        return self.k * np.asarray(np.sin(self._arg(x, t)))[..., None]

    @staticmethod
    def seeded(n: int, kmag: float, seed: int, c: float = 1.0):
        rng = np.random.default_rng(seed)
        if n == 1:
            d = np.array([1.0])
        elif n == 2:
            th = rng.uniform(0.0, 2.0 * np.pi)
            d = np.array([np.cos(th), np.sin(th)])
        else:
            v = rng.normal(size=3)
            d = v / np.linalg.norm(v)
        return PlaneWave(kmag * d, c)


class StandingWaveND(Field):
    """U = prod_m sin(pi x_m) * cos(sqrt(n) pi c t) on the unit cube."""

    def __init__(self, n: int, c: float = 1.0):
        self.n = n
        self.c = float(c)
        self.w = np.sqrt(n) * np.pi * self.c

    def _S(self, x):
        return np.prod(np.sin(np.pi * x), axis=-1)

    def U(self, x, t):
        return self._S(x) * np.cos(self.w * t)

    def v(self, x, t):
        return -self.w * self._S(x) * np.sin(self.w * t)

    def sigma(self, x, t):
        s = np.sin(np.pi * x)
        co = np.cos(np.pi * x)
        out = np.empty(x.shape, dtype=np.float64)
        for m in range(x.shape[-1]):
            prod = np.pi * co[..., m]
            for l in range(x.shape[-1]):
                if l != m:
                    prod = prod * s[..., l]
            out[..., m] = -prod
        return out * np.asarray(np.cos(self.w * t))[..., None]


class PaperStandingWave(Field):
    """U = prod_m cos(pi x_m) * sin(pi c sqrt(n) t) / (sqrt(n) pi) (eq. 6.1)."""

    def __init__(self, n: int, c: float = 1.0):
        self.n = n
        self.c = float(c)
        self.w = np.pi * self.c * np.sqrt(n)

    def U(self, x, t):
        return np.prod(np.cos(np.pi * x), axis=-1) * np.sin(self.w * t) / (np.sqrt(self.n) * np.pi)

    def v(self, x, t):
        return np.prod(np.cos(np.pi * x), axis=-1) * np.cos(self.w * t) * self.c

    def sigma(self, x, t):
        co = np.cos(np.pi * x)
        s = np.sin(np.pi * x)
        out = np.empty(x.shape, dtype=np.float64)
        for m in range(x.shape[-1]):
            prod = -np.pi * s[..., m]
            for l in range(x.shape[-1]):
                if l != m:
                    prod = prod * co[..., l]
            out[..., m] = -prod
        return out * np.asarray(np.sin(self.w * t) / (np.sqrt(self.n) * np.pi))[..., None]


class PolynomialPlaneWaves(Field):
    """U = sum_i a_i (d_i . x - c t + s_i)^deg: a polynomial solution of the
    wave equation with speed c built from plane waves f(d.x - c t) with unit
    directions d_i.  It is a degree-``deg`` Trefftz polynomial, constructed
    independently of the Trefftz recursion (eq. 3.1)."""

    def __init__(self, n: int, deg: int, nwaves: int, seed: int, c: float = 1.0):
        rng = np.random.default_rng(seed)
        d = rng.normal(size=(nwaves, n))
        self.d = d / np.linalg.norm(d, axis=1, keepdims=True)
        self.a = rng.uniform(-1.0, 1.0, size=nwaves)
        self.s = rng.uniform(-0.5, 0.5, size=nwaves)
        self.deg = deg
        self.c = float(c)

    def _z(self, x, t):
        return x @ self.d.T - self.c * np.asarray(t)[..., None] + self.s

    def U(self, x, t):
        return (self.a * self._z(x, t) ** self.deg).sum(-1)

    def v(self, x, t):
        if self.deg == 0:
            return np.zeros(np.broadcast(x[..., 0], t).shape)
        return (self.a * self.deg * self._z(x, t) ** (self.deg - 1) * (-self.c)).sum(-1)

    def sigma(self, x, t):
        if self.deg == 0:
            return np.zeros(x.shape)
        g = self.a * self.deg * self._z(x, t) ** (self.deg - 1)  # (..., nw)
        return -(g @ self.d)


class InterfaceQuadratic(Field):
    """U = t^2 + (x_1 - xi)^2 / c(x)^2 for a speed c(x) = c_left for x_1 < xi
    and c_right otherwise.  v = 2t and sigma . e_1 = -2(x_1 - xi)/c^2 are both
    continuous across x_1 = xi (sigma . e_1 = 0 there), so this solves the
    two-material problem exactly."""

    def __init__(self, xi: float, c_left: float, c_right: float):
        self.xi, self.cl, self.cr = float(xi), float(c_left), float(c_right)

    def _c(self, x):
        return np.where(x[..., 0] < self.xi, self.cl, self.cr)

    def U(self, x, t):
        return t * t + (x[..., 0] - self.xi) ** 2 / self._c(x) ** 2

    def v(self, x, t):
        return 2.0 * t * np.ones_like(x[..., 0])

    def sigma(self, x, t):
        out = np.zeros(x.shape)
        out[..., 0] = -2.0 * (x[..., 0] - self.xi) / self._c(x) ** 2
        return out


class GaussianPulse(Field):
    """Initial data only: U0 = exp(-|x - x0|^2 / delta^2), v0 = 0,
    sigma0 = -grad U0 (no closed-form evolution)."""

    def __init__(self, x0, delta: float):
        self.x0 = np.asarray(x0, dtype=np.float64)
        self.delta = float(delta)

    def U(self, x, t):
        r2 = ((x - self.x0) ** 2).sum(-1)
        return np.exp(-r2 / self.delta ** 2)

    def v(self, x, t):
        return np.zeros(x.shape[:-1])

    def sigma(self, x, t):
        return (2.0 * (x - self.x0) / self.delta ** 2) * self.U(x, t)[..., None]


class SinProduct(Field):
    """Initial data only: U0 = prod_m sin(pi x_m), v0 = 0, sigma0 = -grad U0."""

    def U(self, x, t):
        return np.prod(np.sin(np.pi * x), axis=-1)

    def v(self, x, t):
        return np.zeros(x.shape[:-1])

    def sigma(self, x, t):
        s = np.sin(np.pi * x)
        co = np.cos(np.pi * x)
        out = np.empty(x.shape)
        for m in range(x.shape[-1]):
            prod = np.pi * co[..., m]
            for l in range(x.shape[-1]):
                if l != m:
                    prod = prod * s[..., l]
            out[..., m] = -prod
        return out


class CornerBessel(Field):
    """U = cos(a t) sin(nu phi) J_nu(a r) in polar coordinates about the
    origin, phi in [0, 2 pi) (Sec. 6.6: nu = 2/3, a = 10 on the L-shaped
    domain, where phi runs over [0, 3 pi/2] and U vanishes on both edges at
    the re-entrant corner).  J_nu(a r) sin(nu phi) is an eigenfunction of the
    Laplacian with eigenvalue -a^2, so U solves the wave equation with c = 1;
    grad U ~ r^(nu - 1) is singular at the corner."""

    def __init__(self, a: float = 10.0, nu: float = 2.0 / 3.0):
        self.a = float(a)
        self.nu = float(nu)

    def _polar(self, x):
        r = np.hypot(x[..., 0], x[..., 1])
        phi = np.mod(np.arctan2(x[..., 1], x[..., 0]), 2.0 * np.pi)
        return r, phi

    def U(self, x, t):
        from scipy.special import jv

        r, phi = self._polar(x)
        return np.cos(self.a * t) * np.sin(self.nu * phi) * jv(self.nu, self.a * r)

    def v(self, x, t):
        from scipy.special import jv

        r, phi = self._polar(x)
        return -self.a * np.sin(self.a * t) * np.sin(self.nu * phi) * jv(self.nu, self.a * r)

    def sigma(self, x, t):
        from scipy.special import jv, jvp

        r, phi = self._polar(x)
        rs = np.where(r > 0.0, r, 1.0)
        dr = self.a * jvp(self.nu, self.a * r) * np.sin(self.nu * phi)           # dS/dr
        dp = np.where(r > 0.0, self.nu * np.cos(self.nu * phi) * jv(self.nu, self.a * r) / rs, 0.0)  # (1/r) dS/dphi
        cp, sp = np.cos(phi), np.sin(phi)
        gx = dr * cp - dp * sp
        gy = dr * sp + dp * cp
        ct = np.asarray(np.cos(self.a * t))
        return -np.stack([gx * ct, gy * ct], axis=-1)


class Zero(Field):
    def U(self, x, t):
        return np.zeros(x.shape[:-1])

    def v(self, x, t):
        return np.zeros(x.shape[:-1])

    def sigma(self, x, t):
        return np.zeros(x.shape)
