"""Manufactured solutions used as pins (closed forms, not the method).

* PolySolution: u(x, y) = sum a_ij (x - x0)^i (y - y0)^j with i, j <= deg.  On a
  mesh of GLL order N >= deg it lies in Q_N on every element, so the GLL
  discretisation reproduces it exactly when s = -Lap u - c u and
  t = d_n u + i eta u (Sec. 2, Sec. 3.1).
* PlaneWaves: superposition of e^{i kappa d_k . x}, an exact solution of
  -Lap u - kappa^2 u = 0 (b = 0, s = 0).
"""
import numpy as np


class PolySolution:
    def __init__(self, deg, seed=0, x0=0.5, y0=0.5):
        rng = np.random.default_rng(seed)
        a = rng.standard_normal((deg + 1, deg + 1)) + 1j * rng.standard_normal((deg + 1, deg + 1))
        a /= (1.0 + np.add.outer(np.arange(deg + 1), np.arange(deg + 1))) ** 2
        self.a, self.deg, self.x0, self.y0 = a, deg, x0, y0

    def _terms(self, x, y, dx, dy):
        X = np.asarray(x, dtype=float) - self.x0
        Y = np.asarray(y, dtype=float) - self.y0
        out = np.zeros(np.broadcast(X, Y).shape, dtype=complex)
        for i in range(dx, self.deg + 1):
            ci = np.prod(np.arange(i - dx + 1, i + 1)) if dx else 1.0
            for j in range(dy, self.deg + 1):
                cj = np.prod(np.arange(j - dy + 1, j + 1)) if dy else 1.0
                out += self.a[i, j] * ci * cj * X ** (i - dx) * Y ** (j - dy)
        return out

    def u(self, x, y):
        return self._terms(x, y, 0, 0)

    def grad(self, x, y):
        return self._terms(x, y, 1, 0), self._terms(x, y, 0, 1)

    def lap(self, x, y):
        return self._terms(x, y, 2, 0) + self._terms(x, y, 0, 2)

    def source(self, c_fn):
        """s = -Lap u - c u, with c given as a function of (x, y)."""
        return lambda x, y: -self.lap(x, y) - c_fn(x, y) * self.u(x, y)

    def t(self, eta):
        """Incoming impedance data (d_n + i eta) u for outward normal (nx, ny)."""
        def f(x, y, nx, ny):
            gx, gy = self.grad(x, y)
            return gx * nx + gy * ny + 1j * eta * self.u(x, y)
        return f


class PlaneWaves:
    def __init__(self, kappa, count=3, seed=0):
        rng = np.random.default_rng(seed)
        th = rng.uniform(0, 2 * np.pi, count)
        self.d = np.stack([np.cos(th), np.sin(th)], 1)
        self.amp = rng.standard_normal(count) + 1j * rng.standard_normal(count)
        self.kappa = kappa

    def u(self, x, y):
        return sum(a * np.exp(1j * self.kappa * (d[0] * np.asarray(x) + d[1] * np.asarray(y)))
                   for a, d in zip(self.amp, self.d))

    def dn(self, x, y, nx, ny):
        return sum(a * 1j * self.kappa * (d[0] * nx + d[1] * ny)
                   * np.exp(1j * self.kappa * (d[0] * np.asarray(x) + d[1] * np.asarray(y)))
                   for a, d in zip(self.amp, self.d))
