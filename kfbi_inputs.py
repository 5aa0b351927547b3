"""Seeded synthetic workloads shared by the oracle tests, the GPU tests and the benchmark.

This module holds problem *data* only: the box/grid/PDE parameters of each workload, the
shape parameters of the level sets, the manufactured exact solutions (u, p) with their body
forces, and seeded random densities/directions.  It contains none of the method's arithmetic
(no crossings, fits, jumps, corrections, transforms or solves); both the oracle and the GPU
library compute those on their own.

Workloads (the paper uses only analytic, synthetic problems, Section 5; these follow the
same recipe: an irregular domain embedded in a box, a manufactured smooth solution, a
Cartesian MAC grid):

* ``sphere32``    Stokes, mu=1, sphere R=0.5 at the origin, box [-1,1]^3, N=32.
* ``star128``     Stokes, mu=1, star r=0.5+0.1 sin(3 theta) cos(4 phi), N=128.
* ``ellip128``    Navier, lambda=10, mu=1, ellipsoid (0.6,0.45,0.35) rotated 30 deg about z, N=128.
* ``star256``     Stokes, mu=1, star as star128, N=256 (the headline evaluation size).
* ``star512n``    Navier, lambda=100, mu=1, star r=0.5+0.12 sin(5 theta) cos(3 phi), N=512.
* ``ex51`` .. ``ex56``  the six examples of Sec. 5 of the paper, box [-1.2,1.2]^3: Stokes on
  the unit sphere (5.1, the printed u2 corrected to be divergence-free), on the ellipsoid
  x^2 + y^2/0.64 + z^2/0.36 = 1 (5.2) and on the torus a = 0.35, c = 0.7 (5.3); Navier with
  (E, nu) = (1000, 1/10) on the unit sphere (5.4), (4000, 1/20) on the ellipsoid (1, 0.8, 0.6)
  (5.5) and (2000, 2/5) on the torus (5.6); mu = E / (2(1+nu)), lambda = E nu / ((1+nu)(1-2nu)).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field, replace

import numpy as np

STOKES, NAVIER = 0, 1
SPHERE, ELLIPSOID, STAR, TORUS = 0, 1, 2, 3


@dataclass(frozen=True)
class Shape:
    kind: int
    center: tuple = (0.0, 0.0, 0.0)
    param: tuple = (0.0,) * 6   # sphere: R | ellipsoid: a,b,c | star: r0,eps,k,l | torus: a,c
    rot_z_deg: float = 0.0


@dataclass(frozen=True)
class Config:
    N: int
    lo: float = -1.0
    hi: float = 1.0
    pde: int = STOKES
    mu: float = 1.0
    lam: float = 0.0
    shape: Shape = field(default_factory=lambda: Shape(SPHERE, param=(0.5, 0, 0, 0, 0, 0)))
    solution: str = "stokes_trig"     # manufactured solution family

    def with_N(self, N: int) -> "Config":
        return replace(self, N=N)

    @property
    def h(self) -> float:
        return (self.hi - self.lo) / self.N


def sphere(R=0.5, center=(0.0, 0.0, 0.0)):
    return Shape(SPHERE, tuple(center), (R, 0, 0, 0, 0, 0))


def ellipsoid(a, b, c, rot_z_deg=0.0, center=(0.0, 0.0, 0.0)):
    return Shape(ELLIPSOID, tuple(center), (a, b, c, 0, 0, 0), rot_z_deg)


def star(r0, eps, k, l, center=(0.0, 0.0, 0.0)):
    return Shape(STAR, tuple(center), (r0, eps, float(k), float(l), 0, 0))


def torus(a, c, center=(0.0, 0.0, 0.0)):
    return Shape(TORUS, tuple(center), (a, c, 0, 0, 0, 0))


WORKLOADS = {
    "sphere32": Config(N=32, pde=STOKES, mu=1.0, shape=sphere(0.5), solution="stokes_trig"),
    "star128": Config(N=128, pde=STOKES, mu=1.0, shape=star(0.5, 0.1, 3, 4), solution="stokes_trig"),
    "ellip128": Config(N=128, pde=NAVIER, mu=1.0, lam=10.0,
                       shape=ellipsoid(0.6, 0.45, 0.35, 30.0), solution="navier_exp"),
    "star256": Config(N=256, pde=STOKES, mu=1.0, shape=star(0.5, 0.1, 3, 4), solution="stokes_trig"),
    "star512n": Config(N=512, pde=NAVIER, mu=1.0, lam=100.0, shape=star(0.5, 0.12, 5, 3),
                       solution="navier_exp"),
}


def lame(E, nu):
    """(mu, lambda) of Young's modulus E and Poisson ratio nu."""
    return E / (2 * (1 + nu)), E * nu / ((1 + nu) * (1 - 2 * nu))


_BOX = dict(lo=-1.2, hi=1.2)
WORKLOADS.update({
    "ex51": Config(N=64, pde=STOKES, mu=1.0, shape=sphere(1.0), solution="ex51", **_BOX),
    "ex52": Config(N=64, pde=STOKES, mu=1.0, shape=ellipsoid(1.0, 0.8, 0.6), solution="ex52", **_BOX),
    "ex53": Config(N=64, pde=STOKES, mu=1.0, shape=torus(0.35, 0.7), solution="ex53", **_BOX),
    "ex54": Config(N=64, pde=NAVIER, mu=lame(1000, 0.1)[0], lam=lame(1000, 0.1)[1], shape=sphere(1.0),
                   solution="ex54", **_BOX),
    "ex55": Config(N=64, pde=NAVIER, mu=lame(4000, 0.05)[0], lam=lame(4000, 0.05)[1],
                   shape=ellipsoid(1.0, 0.8, 0.6), solution="ex55", **_BOX),
    "ex56": Config(N=64, pde=NAVIER, mu=lame(2000, 0.4)[0], lam=lame(2000, 0.4)[1], shape=torus(0.35, 0.7),
                   solution="ex56", **_BOX),
})


def _paper_example_exprs(name, printed=False):
    """Sympy expressions (u1, u2, u3, p or None) of the exact solutions of Sec. 5.  Example 5.1
    as printed has div u = -2y; printed=False returns it with y^2(2 - y^2) in u2, which makes
    it divergence-free."""
    import sympy as sp
    x, y, z = sp.symbols("x y z", real=True)
    r2 = x ** 2 + y ** 2 + z ** 2
    if name == "ex51":
        u = (x**2 * (2 - x**2) + 4 * x * y * (x**2 + y**2 - 1) + z**2 * (3 * z**2 - 6 * x**2 - 2),
             x**2 * (3 * x**2 - 6 * y**2 - 1) + y**2 * ((1 if printed else 2) - y**2),
             4 * z * x * (z**2 + x**2 - 1))
        p = 8 * y * (3 * x**2 - y**2) + 8 * x * (3 * z**2 - x**2)
    elif name == "ex52":
        u = (2 * x**3 * y / 3 - z**2 * x**2 + sp.exp(z) + sp.sin(sp.pi * z),
             -x**2 * y**2 + sp.cos(sp.pi * x),
             2 * z**3 * x / 3 + sp.exp(x) + sp.sin(sp.pi * x))
        p = (x - 1)**3 * (y - 1)**3 * (z - 1)**3
    elif name == "ex53":
        u = (-4 * x * y * (1 - x**2 - y**2) - x**2 * (x**2 + 6 * z**2 - 2) + z**2 * (3 * z**2 - 2)
             + sp.exp(sp.cos(y)) + sp.exp(sp.sin(z)),
             x**2 * (3 * x**2 - 6 * y**2 - 2) - y**2 * (y**2 - 2) + sp.exp(sp.sin(x)),
             -4 * (1 - x**2 - z**2) * x * z + sp.exp(sp.cos(x)))
        p = sp.exp(1 - y**2 - z**3) * sp.sin(x**2 + 1)
    elif name == "ex54":
        s = sp.sin(2 * sp.pi * r2)
        u = (s * sp.cos(2 * y) * sp.cos(z), s * sp.cos(x) * sp.cos(x + z), s * sp.cos(sp.pi * x) * sp.cos(y))
        p = None
    elif name == "ex55":
        c = sp.cos(x) * sp.cos(y) * sp.cos(z)
        u = (r2 - 4 + c, r2 - 4 + x * y + c, r2 - 4 + y * z + c)
        p = None
    elif name == "ex56":
        u = (sp.exp(1 - y**2 - z**2) * sp.sin(3 * x**2 + 2), sp.sin(1 - r2), 3 * x**2 + 2 * y**2 + z**2)
        p = None
    else:
        raise ValueError(name)
    return (x, y, z), u, p


_PAPER_CACHE = {}


def _paper_example(name, mu, lam):
    """Numpy callables (u, p, f) of a Sec. 5 example: f = -mu lap u + grad p (Stokes) or
    f = -mu lap u - (lambda+mu) grad div u (Navier, with p = -(lambda+mu) div u)."""
    key = (name, mu, lam)
    if key not in _PAPER_CACHE:
        import sympy as sp
        (x, y, z), u, p = _paper_example_exprs(name)
        X = (x, y, z)
        div = sum(sp.diff(u[i], X[i]) for i in range(3))
        lap = [sum(sp.diff(u[i], X[k], 2) for k in range(3)) for i in range(3)]
        if p is not None:  # Stokes
            f = [-mu * lap[i] + sp.diff(p, X[i]) for i in range(3)]
        else:
            p = -(lam + mu) * div
            f = [-mu * lap[i] - (lam + mu) * sp.diff(div, X[i]) for i in range(3)]
        fu = sp.lambdify(X, list(u), "numpy")
        fp = sp.lambdify(X, p, "numpy")
        ff = sp.lambdify(X, f, "numpy")
        stack = lambda g: (lambda a, b, c: np.stack(np.broadcast_arrays(*[np.asarray(v, float) + 0 * a
                                                                           for v in g(a, b, c)]), axis=-1))
        _PAPER_CACHE[key] = (stack(fu), lambda a, b, c: np.asarray(fp(a, b, c), float) + 0 * a, stack(ff))
    return _PAPER_CACHE[key]


# ----------------------------------------------------------------------------------------
# Manufactured exact solutions (problem data).  Each returns arrays shaped like x.
# ----------------------------------------------------------------------------------------
_NAV_A = np.array([1.0, 0.5, -0.3])


def exact_u(sol: str, x, y, z):
    """Exact velocity/displacement, stacked on a trailing axis of length 3."""
    x, y, z = np.asarray(x, float), np.asarray(y, float), np.asarray(z, float)
    if sol == "stokes_trig":
        pi = math.pi
        sx, cx = np.sin(pi * x), np.cos(pi * x)
        sy, cy = np.sin(pi * y), np.cos(pi * y)
        sz, cz = np.sin(pi * z), np.cos(pi * z)
        return np.stack([sx * cy * cz, -2.0 * cx * sy * cz, cx * cy * sz], axis=-1)
    if sol == "navier_exp":
        s = np.exp(x) * np.sin(y + z)
        return s[..., None] * _NAV_A
    if sol.startswith("ex5"):
        return _paper_example(sol, 1.0, 0.0)[0](x, y, z)
    raise ValueError(sol)


def exact_p(sol: str, x, y, z, lam: float = 0.0, mu: float = 1.0):
    """Exact pressure (Stokes) or auxiliary pressure -(lambda+mu) div u (Navier)."""
    x, y, z = np.asarray(x, float), np.asarray(y, float), np.asarray(z, float)
    if sol == "stokes_trig":
        return np.sin(x + y + z)
    if sol == "navier_exp":
        a = _NAV_A
        div = np.exp(x) * (a[0] * np.sin(y + z) + (a[1] + a[2]) * np.cos(y + z))
        return -(lam + mu) * div
    if sol.startswith("ex5"):
        return _paper_example(sol, mu, lam)[1](x, y, z)
    raise ValueError(sol)


def body_force(sol: str, x, y, z, mu: float = 1.0, lam: float = 0.0):
    """f = -mu lap u + grad p (Stokes) or f = -mu lap u - (lambda+mu) grad div u (Navier)."""
    x, y, z = np.asarray(x, float), np.asarray(y, float), np.asarray(z, float)
    if sol == "stokes_trig":
        u = exact_u(sol, x, y, z)
        c = np.cos(x + y + z)
        return 3.0 * math.pi ** 2 * mu * u + c[..., None] * np.ones(3)
    if sol == "navier_exp":
        a = _NAV_A
        e = np.exp(x)
        s, c = np.sin(y + z), np.cos(y + z)
        # lap(e^x sin(y+z)) = -e^x sin(y+z)
        lap_u = -(e * s)[..., None] * a
        b = a[1] + a[2]
        gdiv = np.stack([e * (a[0] * s + b * c), e * (a[0] * c - b * s), e * (a[0] * c - b * s)], axis=-1)
        return -mu * lap_u - (lam + mu) * gdiv
    if sol.startswith("ex5"):
        return _paper_example(sol, mu, lam)[2](x, y, z)
    raise ValueError(sol)


# ----------------------------------------------------------------------------------------
# Seeded random inputs
# ----------------------------------------------------------------------------------------
def random_density(n: int, seed: int = 2) -> np.ndarray:
    """Random density phi ~ N(0,1) i.i.d., shape (n, 3)."""
    return np.random.default_rng(seed).standard_normal((n, 3))


def random_directions(n: int, count: int = 16, seed: int = 1) -> np.ndarray:
    """Unit-norm random directions in R^{n x 3}, shape (count, n, 3)."""
    d = np.random.default_rng(seed).standard_normal((count, n, 3))
    return d / np.linalg.norm(d.reshape(count, -1), axis=1)[:, None, None]


def level_set_value(shape: Shape, x, y, z):
    """Value of the level-set function psi (Omega = {psi <= 0}); problem data for probe sampling."""
    cx, cy, cz = shape.center
    X, Y, Z = np.asarray(x) - cx, np.asarray(y) - cy, np.asarray(z) - cz
    p = shape.param
    if shape.kind == SPHERE:
        return np.sqrt(X * X + Y * Y + Z * Z) - p[0]
    if shape.kind == ELLIPSOID:
        t = math.radians(shape.rot_z_deg)
        xr = math.cos(t) * X + math.sin(t) * Y
        yr = -math.sin(t) * X + math.cos(t) * Y
        return (xr / p[0]) ** 2 + (yr / p[1]) ** 2 + (Z / p[2]) ** 2 - 1.0
    if shape.kind == STAR:
        rho = np.sqrt(X * X + Y * Y + Z * Z)
        th = np.arccos(np.clip(Z / np.where(rho > 0, rho, 1.0), -1, 1))
        ph = np.arctan2(Y, X)
        return rho - (p[0] + p[1] * np.sin(p[2] * th) * np.cos(p[3] * ph))
    if shape.kind == TORUS:
        q = np.sqrt(X * X + Y * Y) - p[1]
        return np.sqrt(q * q + Z * Z) - p[0]
    raise ValueError(shape.kind)


def probe_points(cfg: Config, m: int = 4096, seed: int = 0) -> np.ndarray:
    """m uniform-random interior probe points (seeded).

    A candidate drawn uniformly in the box is kept iff the 8 nodes of its trilinear cell on
    each of the three velocity grids lie in Omega, so trilinear interpolation of a grid field
    at the probe only touches interior nodes.
    """
    rng = np.random.default_rng(seed)
    h, lo = cfg.h, cfg.lo
    out = []
    while sum(len(o) for o in out) < m:
        c = rng.uniform(cfg.lo, cfg.hi, size=(8 * m, 3))
        ok = np.ones(len(c), bool)
        for comp in range(3):
            off = np.array([0.0 if d == comp else 0.5 for d in range(3)])
            base = np.floor((c - lo) / h - off)
            for corner in range(8):
                bits = np.array([(corner >> d) & 1 for d in range(3)])
                node = lo + (base + bits + off) * h
                ok &= level_set_value(cfg.shape, node[:, 0], node[:, 1], node[:, 2]) <= 0
        out.append(c[ok])
    return np.concatenate(out)[:m]


def probe_target(cfg: Config, xyz: np.ndarray) -> np.ndarray:
    """Target field for the probe misfit loss: 0.9 u_exact + 0.05 (1,1,1)."""
    return 0.9 * exact_u(cfg.solution, xyz[:, 0], xyz[:, 1], xyz[:, 2]) + 0.05
