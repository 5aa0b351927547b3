"""Oracle geometry: grids, level sets, crossings, control points, local frames.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Paper: Sec. 4.2 (box, N^3 cells, h, the five grid sets T_h, T_h^0..T_h^3), Algorithm 1 step 1
(mark nodes inside/outside, find intersections of the surface with grid lines, tangential and
normal directions there), Sec. 3 (control points = intersections with grid lines, primary
points).

Readings used here (the paper is silent on them):
* Box [lo,hi]^3 from the workload, h = (hi-lo)/N (the paper's [0,1]^3 of Sec. 4.2 and
  [-1.2,1.2]^3 of Sec. 5 are two instances).
* Omega = {psi <= 0} for an analytic level set psi; n = grad psi/|grad psi| points outward.
* Crossings are taken on the nine families of grid lines used by the MAC stencils: for each
  axis k, the k-lines of the cell grid T^0 (which are also the k-lines of T^k) and the k-lines
  of the two other face grids.  Along a line, psi is sampled on the half-step lattice
  lo + j h/2; every sign change (of the test psi <= 0) brackets one crossing, located by
  bisection until the bracket cannot shrink; the crossing is the bracket midpoint.  A node
  segment (length h, endpoints on the half-step lattice) whose endpoints lie on different
  sides therefore holds exactly one detected crossing; a segment with equal sides holds zero
  or two (a grazing line) and is not used by any stencil.
* Control points are the crossings on the three T^0 line families that are *primary*:
  |n_k| >= (1 - 1e-12) max_j |n_j| for a k-line.  Order: axis k, then the two transverse line
  indices lexicographically, then ascending position.
* Frame: t1 = normalise(e_k x n) with k = argmin |n_k| (lowest index on ties), t2 = n x t1,
  curvature kappa_ab = -t_a^T (hess psi) t_b / |grad psi| so that the surface is
  nu = 1/2 kappa_ab xi_a xi_b + O(|xi|^3) in the frame (a sphere of radius R has kappa = -I/R).
* Star level set: theta = arccos(z/|x|), phi = atan2(y, x), psi = |x| - r(theta, phi).
* Ellipsoid rotated by +rot about z: body coordinates x' = R_z(-rot) (x - c).
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np
import sympy as sp

SPHERE, ELLIPSOID, STAR, TORUS = 0, 1, 2, 3


class GeometryError(RuntimeError):
    pass


# ----------------------------------------------------------------------------------------
# Level sets with analytic gradient and Hessian (derived symbolically, never differenced)
# ----------------------------------------------------------------------------------------
class LevelSet:
    def __init__(self, shape):
        X = sp.symbols("x y z", real=True)
        c = shape.center
        x, y, z = X[0] - c[0], X[1] - c[1], X[2] - c[2]
        p = shape.param
        if shape.kind == SPHERE:
            psi = sp.sqrt(x ** 2 + y ** 2 + z ** 2) - p[0]
            half = (p[0], p[0], p[0])
        elif shape.kind == ELLIPSOID:
            t = sp.pi * sp.Float(shape.rot_z_deg) / 180
            xr = sp.cos(t) * x + sp.sin(t) * y
            yr = -sp.sin(t) * x + sp.cos(t) * y
            psi = (xr / p[0]) ** 2 + (yr / p[1]) ** 2 + (z / p[2]) ** 2 - 1
            a = max(p[0], p[1], p[2])
            half = (a, a, p[2])
        elif shape.kind == STAR:
            rho = sp.sqrt(x ** 2 + y ** 2 + z ** 2)
            th = sp.acos(z / rho)
            ph = sp.atan2(y, x)
            psi = rho - (p[0] + p[1] * sp.sin(p[2] * th) * sp.cos(p[3] * ph))
            r = p[0] + abs(p[1])
            half = (r, r, r)
        elif shape.kind == TORUS:
            q = sp.sqrt(x ** 2 + y ** 2) - p[1]
            psi = sp.sqrt(q ** 2 + z ** 2) - p[0]
            half = (p[0] + p[1], p[0] + p[1], p[0])
        else:
            raise ValueError(shape.kind)
        grad = [sp.diff(psi, v) for v in X]
        hess = [[sp.diff(g, v) for v in X] for g in grad]
        self._psi = sp.lambdify(X, psi, "numpy")
        self._grad = [sp.lambdify(X, g, "numpy") for g in grad]
        self._hess = [[sp.lambdify(X, hh, "numpy") for hh in row] for row in hess]
        self.bbox_lo = np.array(c) - np.array(half)
        self.bbox_hi = np.array(c) + np.array(half)

    @staticmethod
    def _bc(v, like):
        return np.broadcast_to(np.asarray(v, float), like.shape).astype(float)

    def psi(self, P):
        P = np.asarray(P, float)
        return self._bc(self._psi(P[..., 0], P[..., 1], P[..., 2]), P[..., 0])

    def grad(self, P):
        P = np.asarray(P, float)
        return np.stack([self._bc(g(P[..., 0], P[..., 1], P[..., 2]), P[..., 0]) for g in self._grad], -1)

    def hess(self, P):
        P = np.asarray(P, float)
        return np.stack([np.stack([self._bc(h(P[..., 0], P[..., 1], P[..., 2]), P[..., 0])
                                   for h in row], -1) for row in self._hess], -2)

    def inside(self, P):
        return self.psi(P) <= 0.0


# ----------------------------------------------------------------------------------------
# Grids (Sec. 4.2).  Grid ids: -1 = cell centres T^0 (pressure), m = 0,1,2 = face grid T^{m+1}
# (velocity component m).  Arrays are numpy C-order [i][j][k] <-> (x, y, z).
#   p   : (N, N, N),  node (a,b,c) at lo + (a+1/2, b+1/2, c+1/2) h
#   u_m : N+1 along axis m (integer positions lo + a h, a = 0..N; a = 0 and N are the box
#         faces where u_m = 0), N along the two other axes (half positions).
# ----------------------------------------------------------------------------------------
@dataclass
class Grid:
    N: int
    lo: float
    hi: float

    @property
    def h(self):
        return (self.hi - self.lo) / self.N

    def shape(self, g):
        return tuple(self.N + 1 if d == g else self.N for d in range(3))

    def offset(self, g):
        """Per-axis offset in units of h: 0 for integer positions, 1/2 for half positions."""
        return np.array([0.0 if d == g else 0.5 for d in range(3)])

    def coords(self, g, idx):
        idx = np.asarray(idx, float)
        return self.lo + (idx + self.offset(g)) * self.h

    def all_nodes(self, g):
        sh = self.shape(g)
        I = np.stack(np.meshgrid(*[np.arange(s) for s in sh], indexing="ij"), -1)
        return self.coords(g, I)


FAMILIES = [(k, g) for k in range(3) for g in ([-1] + [m for m in range(3) if m != k])]


def transverse_axes(k):
    return [d for d in range(3) if d != k]


@dataclass
class Crossings:
    """All crossings of the surface with the nine line families, in family order."""
    fam: np.ndarray      # (T,) family index into FAMILIES
    line: np.ndarray     # (T, 2) transverse indices
    j: np.ndarray        # (T,) half-step sample interval index
    pos: np.ndarray      # (T,) coordinate along the line axis
    xyz: np.ndarray      # (T, 3)
    normal: np.ndarray   # (T, 3)
    t1: np.ndarray
    t2: np.ndarray
    kappa: np.ndarray    # (T, 2, 2)
    cp: np.ndarray       # (T,) control-point index or -1
    cp_target: np.ndarray  # (n,) crossing index of each control point


def _line_families(grid: Grid, ls: LevelSet, k: int, g: int):
    """Enumerate lines of family (k, g) that can meet the surface; return transverse indices
    and transverse coordinates."""
    N, lo, h = grid.N, grid.lo, grid.h
    ax = transverse_axes(k)
    idx_lists, coord_lists = [], []
    for d in ax:
        if d == g:
            ii = np.arange(N + 1)
            cc = lo + ii * h
        else:
            ii = np.arange(N)
            cc = lo + (ii + 0.5) * h
        keep = (cc >= ls.bbox_lo[d] - h) & (cc <= ls.bbox_hi[d] + h)
        idx_lists.append(ii[keep])
        coord_lists.append(cc[keep])
    I1, I2 = np.meshgrid(idx_lists[0], idx_lists[1], indexing="ij")
    C1, C2 = np.meshgrid(coord_lists[0], coord_lists[1], indexing="ij")
    return ax, I1.ravel(), I2.ravel(), C1.ravel(), C2.ravel()


def find_crossings(grid: Grid, ls: LevelSet):
    N, lo, h = grid.N, grid.lo, grid.h
    out = {key: [] for key in ("fam", "line", "j", "pos")}
    for f, (k, g) in enumerate(FAMILIES):
        ax, I1, I2, C1, C2 = _line_families(grid, ls, k, g)
        if len(I1) == 0:
            continue
        # half-step samples along the line, restricted to the bounding box (psi > 0 outside)
        jlo = max(0, int(math.floor((ls.bbox_lo[k] - h - lo) / (0.5 * h))))
        jhi = min(2 * N, int(math.ceil((ls.bbox_hi[k] + h - lo) / (0.5 * h))))
        js = np.arange(jlo, jhi + 1)
        s = lo + js * (0.5 * h)
        P = np.empty((len(I1), len(js), 3))
        P[:, :, k] = s[None, :]
        P[:, :, ax[0]] = C1[:, None]
        P[:, :, ax[1]] = C2[:, None]
        ins = ls.inside(P)
        chg = ins[:, 1:] != ins[:, :-1]
        L, J = np.nonzero(chg)           # row-major: line order, then ascending position
        if len(L) == 0:
            continue
        a = s[J].copy()
        b = s[J + 1].copy()
        side_a = ins[L, J]
        base = np.empty((len(L), 3))
        base[:, ax[0]] = C1[L]
        base[:, ax[1]] = C2[L]

        def at(t):
            q = base.copy()
            q[:, k] = t
            return q

        # bisection until the bracket stops shrinking
        for _ in range(200):
            m = 0.5 * (a + b)
            active = (m != a) & (m != b)
            if not np.any(active):
                break
            im = ls.inside(at(m))
            left = (im == side_a) & active
            right = (im != side_a) & active
            a = np.where(left, m, a)
            b = np.where(right, m, b)
        pos = 0.5 * (a + b)
        out["fam"].append(np.full(len(L), f))
        out["line"].append(np.stack([I1[L], I2[L]], -1))
        out["j"].append(js[J])
        out["pos"].append(pos)
    fam = np.concatenate(out["fam"])
    line = np.concatenate(out["line"])
    jj = np.concatenate(out["j"])
    pos = np.concatenate(out["pos"])
    # crossing points
    xyz = np.empty((len(fam), 3))
    for f, (k, g) in enumerate(FAMILIES):
        sel = fam == f
        ax = transverse_axes(k)
        xyz[sel, k] = pos[sel]
        for t, d in enumerate(ax):
            off = 0.0 if d == g else 0.5
            xyz[sel, d] = lo + (line[sel, t] + off) * h
    return fam, line, jj, pos, xyz


def frames(ls: LevelSet, X):
    G = ls.grad(X)
    gn = np.linalg.norm(G, axis=-1)
    n = G / gn[:, None]
    kmin = np.argmin(np.abs(n), axis=-1)      # first index on ties
    e = np.eye(3)[kmin]
    t1 = np.cross(e, n)
    t1 /= np.linalg.norm(t1, axis=-1)[:, None]
    t2 = np.cross(n, t1)
    H = ls.hess(X)
    T = np.stack([t1, t2], 1)                  # (M, 2, 3)
    kappa = -np.einsum("mai,mij,mbj->mab", T, H, T) / gn[:, None, None]
    return n, t1, t2, kappa


def build_crossings(grid: Grid, ls: LevelSet) -> Crossings:
    fam, line, jj, pos, xyz = find_crossings(grid, ls)
    n, t1, t2, kappa = frames(ls, xyz)
    cp = np.full(len(fam), -1, dtype=np.int64)
    famk = np.array([FAMILIES[f][0] for f in fam])
    famg = np.array([FAMILIES[f][1] for f in fam])
    absn = np.abs(n)
    primary = (famg == -1) & (absn[np.arange(len(fam)), famk] >= (1.0 - 1e-12) * absn.max(-1))
    cp_target = np.nonzero(primary)[0]         # family order is k = 0,1,2 for the T^0 families
    cp[cp_target] = np.arange(len(cp_target))
    return Crossings(fam, line, jj, pos, xyz, n, t1, t2, kappa, cp, cp_target)


def node_sides(grid: Grid, ls: LevelSet):
    """Boolean inside-masks (psi <= 0) of every node of T^0 (key -1) and T^1..T^3 (keys 0..2).

    Nodes outside the bounding box of Omega have psi > 0 and are marked outside directly."""
    out = {}
    for g in (-1, 0, 1, 2):
        sh = grid.shape(g)
        off = grid.offset(g)
        sl = []
        for d in range(3):
            c = grid.lo + (np.arange(sh[d]) + off[d]) * grid.h
            ok = np.nonzero((c >= ls.bbox_lo[d] - grid.h) & (c <= ls.bbox_hi[d] + grid.h))[0]
            sl.append(slice(ok[0], ok[-1] + 1) if len(ok) else slice(0, 0))
        mask = np.zeros(sh, bool)
        I = np.stack(np.meshgrid(*[np.arange(s.start, s.stop) for s in sl], indexing="ij"), -1)
        if I.size:
            mask[sl[0], sl[1], sl[2]] = ls.inside(grid.coords(g, I))
        out[g] = mask
    return out
