"""Oracle MAC scheme: operators, sine-transform Poisson solver, Schur-complement CG, dense
augmented solve for tiny grids, and the irregular-node corrections.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Paper: Sec. 4.2 (difference operators, the MAC scheme at regular points, the modified scheme
with corrected right-hand sides, the saddle-point system, the augmented system with an
auxiliary mean variable, the Schur complement solved by CG with an FFT-based Poisson solver
inside, and the velocity back-substitution); Sec. 4.3 (correction terms, cases 1-4).

Readings used here:
* Unknowns of u_m are the interior faces (index 1..N-1 along m; 0 and N are the box faces
  where u = 0).  Across the tangential box faces u = 0 is imposed by ghost reflection
  u_ghost = -u_adjacent, so -Delta_h on T^m is diagonalised by DST-I along m and DST-II along
  the two other axes, eigenvalue (4/h^2) sin^2(j pi / 2N) per axis and mode j.
* The system is A_u u + G p = F_u, D u + c p = F_p with A_u = -mu Delta_h, G = delta^+,
  D = delta^- = -G^T; c = 0 (Stokes) or 1/(lambda+mu) (Navier, generalised Stokes form of
  Remark 3.1).  Schur complement S = G^T A_u^{-1} G + c I, S p = P(F_p + G^T A_u^{-1} F_u),
  u = A_u^{-1}(F_u - G p).  For Stokes P removes the mean and p has mean zero (the auxiliary
  mean variable of the augmented system; the printed sign of its rank-one term is garbled,
  and eliminating it this way gives the same velocity for either sign).  The continuity
  residual then reads D u = F_p - mean(F_p).  For Navier there is no projection.
* Correction sign (general rule, Sec. 4.3): for an equation at z0 with stencil coefficient
  c_q on a node z_q across the interface, C = -s(z0) c_q D_q, s = +1 in Omega and -1 outside,
  D_q = [[v]] + xi [[v_k]] + xi^2/2 [[v_kk]] (velocity) or [[p]] + xi [[p_k]] (pressure) at
  the crossing r, xi = (z_q - r)_k.  This reproduces cases 1-3 and the pressure term of
  case 4 as printed; for the velocity term of case 4 it gives the opposite sign to the
  printed one, which is the sign that makes K c = c hold exactly for constant densities.
"""
from __future__ import annotations

import numpy as np
import scipy.fft as sfft
import scipy.sparse as sps
import scipy.linalg as sla

from .geometry import FAMILIES, transverse_axes, GeometryError
from .surface import NJ, jidx_u, jidx_du, jidx_ddu, jidx_p, jidx_dp

STOKES, NAVIER = 0, 1


class MAC:
    def __init__(self, N, lo, hi, pde, mu, lam=0.0, workers=None):
        self.N, self.lo, self.hi = N, lo, hi
        self.h = (hi - lo) / N
        self.pde, self.mu, self.lam = pde, mu, lam
        self.c = 0.0 if pde == STOKES else 1.0 / (lam + mu)
        self.workers = workers
        j = np.arange(1, N + 1)
        lam_half = (4.0 / self.h ** 2) * np.sin(j * np.pi / (2 * N)) ** 2          # DST-II modes 1..N
        lam_int = (4.0 / self.h ** 2) * np.sin(j[:-1] * np.pi / (2 * N)) ** 2       # DST-I modes 1..N-1
        self._eig = []
        for m in range(3):
            ax = [lam_int if d == m else lam_half for d in range(3)]
            self._eig.append(mu * (ax[0][:, None, None] + ax[1][None, :, None] + ax[2][None, None, :]))

    # ---------------- shapes
    def ushape(self, m):
        return tuple(self.N + 1 if d == m else self.N for d in range(3))

    def zeros_u(self):
        return [np.zeros(self.ushape(m)) for m in range(3)]

    @staticmethod
    def interior(m):
        sl = [slice(None)] * 3
        sl[m] = slice(1, -1)
        return tuple(sl)

    # ---------------- operators (Sec. 4.2)
    def G(self, p):
        """MAC gradient delta^+_m p at interior faces (boundary faces zero)."""
        out = self.zeros_u()
        for m in range(3):
            out[m][self.interior(m)] = np.diff(p, axis=m) / self.h
        return out

    def D(self, u):
        """MAC divergence sum_m delta^-_m u_m at cells (u_m zero on the box faces)."""
        return sum(np.diff(u[m], axis=m) for m in range(3)) / self.h

    def lap(self, v, m):
        """Delta_h of u_m (interior faces), ghost reflection across tangential box faces."""
        h2 = self.h ** 2
        out = np.zeros_like(v)
        for d in range(3):
            if d == m:
                pad = v                                              # faces 0 and N are zero
                core = pad[self.interior(m)]
                lo_ = np.take(pad, np.arange(0, self.N - 1), axis=m)
                hi_ = np.take(pad, np.arange(2, self.N + 1), axis=m)
                out[self.interior(m)] += (lo_ - 2 * core + hi_) / h2
            else:
                first = np.take(v, [0], axis=d)
                last = np.take(v, [self.N - 1], axis=d)
                ext = np.concatenate([-first, v, -last], axis=d)
                lo_ = np.take(ext, np.arange(0, self.N), axis=d)
                hi_ = np.take(ext, np.arange(2, self.N + 2), axis=d)
                out += (lo_ - 2 * v + hi_) / h2
        out[tuple(slice(0, 1) if d == m else slice(None) for d in range(3))] = 0
        out[tuple(slice(self.N, self.N + 1) if d == m else slice(None) for d in range(3))] = 0
        return out

    def apply(self, u, p):
        """The full MAC operator: (A_u u + G p, D u + c p)."""
        gp = self.G(p)
        ru = [-self.mu * self.lap(u[m], m) + gp[m] for m in range(3)]
        return ru, self.D(u) + self.c * p

    # ---------------- sine-transform Poisson solver
    def poisson(self, r, m):
        """A_u^{-1} r on T^m by orthonormal DST-I (axis m) / DST-II (other axes)."""
        types = [1 if d == m else 2 for d in range(3)]
        x = r[self.interior(m)]
        for d in range(3):
            x = sfft.dst(x, type=types[d], axis=d, norm="ortho", workers=self.workers)
        x = x / self._eig[m]
        for d in range(3):
            x = sfft.idst(x, type=types[d], axis=d, norm="ortho", workers=self.workers)
        out = np.zeros(self.ushape(m))
        out[self.interior(m)] = x
        return out

    def schur(self, p):
        gp = self.G(p)
        v = [self.poisson(gp[m], m) for m in range(3)]
        return -self.D(v) + self.c * p          # G^T = -D

    def project(self, q):
        return q - q.mean() if self.pde == STOKES else q

    def solve(self, Fu, Fp, rtol=1e-13, maxit=1000):
        """Schur-complement CG (no preconditioner) then velocity back-substitution."""
        w = [self.poisson(Fu[m], m) for m in range(3)]
        b = self.project(Fp - self.D(w))        # F_p + G^T A^{-1} F_u
        x = np.zeros_like(b)
        r = b.copy()
        d = r.copy()
        rr = np.vdot(r, r)
        bn = np.sqrt(rr)
        it = 0
        if bn > 0:
            while it < maxit and np.sqrt(rr) > rtol * bn:
                q = self.project(self.schur(d))
                alpha = rr / np.vdot(d, q)
                x += alpha * d
                r -= alpha * q
                rr_new = np.vdot(r, r)
                d = r + (rr_new / rr) * d
                rr = rr_new
                it += 1
            if np.sqrt(rr) > rtol * bn:
                raise RuntimeError("Schur CG did not converge")
        gp = self.G(x)
        u = [self.poisson(Fu[m] - gp[m], m) for m in range(3)]
        return u, x, it

    def solve_transpose(self, ubar, rtol=1e-13, maxit=1000):
        """Transpose of the map (F_u, F_p) -> u.  The system matrix satisfies
        A^T = diag(I,-I) A diag(I,-I) because D = -G^T, so with (u', p') the solution for
        the right-hand side (ubar, 0), the transpose gives (F_u-bar, F_p-bar) = (u', -p')."""
        u, p, it = self.solve(ubar, np.zeros((self.N,) * 3), rtol, maxit)
        return u, -p, it

    # ---------------- dense augmented solve (tiny grids only)
    def unknown_index(self):
        """Index map of the unknowns (u interior faces, then p) into a flat vector."""
        idx = []
        off = 0
        for m in range(3):
            a = -np.ones(self.ushape(m), dtype=np.int64)
            cnt = int(np.prod([self.N - 1 if d == m else self.N for d in range(3)]))
            a[self.interior(m)] = (off + np.arange(cnt)).reshape(a[self.interior(m)].shape)
            idx.append(a)
            off += cnt
        pidx = (off + np.arange(self.N ** 3)).reshape((self.N,) * 3)
        return idx, pidx, off + self.N ** 3

    def dense_solve(self, Fu, Fp):
        """Direct LU of the assembled system, with the Stokes mean handled by the augmented
        form [A_u G 0; D 0 1; 0 1^T 0] (auxiliary mean variable)."""
        idx, pidx, n = self.unknown_index()
        aug = self.pde == STOKES
        nt = n + (1 if aug else 0)
        A = np.zeros((nt, nt))
        for col in range(n):
            e = np.zeros(n)
            e[col] = 1.0
            u = self.zeros_u()
            for m in range(3):
                u[m][idx[m] >= 0] = e[idx[m][idx[m] >= 0]]
            p = e[pidx]
            ru, rp = self.apply(u, p)
            v = np.zeros(nt)
            for m in range(3):
                v[idx[m][idx[m] >= 0]] = ru[m][idx[m] >= 0]
            v[pidx.ravel()] = rp.ravel()
            A[:, col] = v
        rhs = np.zeros(nt)
        for m in range(3):
            rhs[idx[m][idx[m] >= 0]] = Fu[m][idx[m] >= 0]
        rhs[pidx.ravel()] = Fp.ravel()
        if aug:
            A[pidx.ravel(), n] = 1.0
            A[n, pidx.ravel()] = 1.0
        sol = sla.lu_solve(sla.lu_factor(A), rhs)
        u = self.zeros_u()
        for m in range(3):
            u[m][idx[m] >= 0] = sol[idx[m][idx[m] >= 0]]
        return u, sol[pidx]


# ----------------------------------------------------------------------------------------
# Corrections (Sec. 4.3)
# ----------------------------------------------------------------------------------------
def _crossing_lookup(cr):
    """(family, i1, i2, half-step interval) -> crossing index."""
    return {(int(f), int(a), int(b), int(j)): t
            for t, (f, (a, b), j) in enumerate(zip(cr.fam, cr.line, cr.j))}


def _family_of(k, g):
    return FAMILIES.index((k, g))


def rhs_layout(N):
    """Offsets of F_u0, F_u1, F_u2, F_p in the flat right-hand-side vector."""
    sizes = [(N + 1) * N * N] * 3 + [N ** 3]
    off = np.concatenate([[0], np.cumsum(sizes)])
    return off


def correction_matrix(mac: MAC, sides, cr):
    """Sparse map from the flattened jump vectors (T*34) to the right-hand side
    (F_u0, F_u1, F_u2, F_p flattened), holding every correction term."""
    N, h, lo, mu = mac.N, mac.h, mac.lo, mac.mu
    look = _crossing_lookup(cr)
    off = rhs_layout(N)
    rows, cols, vals = [], [], []

    def find(fam, i1, i2, ja, jb):
        for j in range(ja, jb):
            t = look.get((fam, i1, i2, j))
            if t is not None:
                return t
        raise GeometryError("no crossing on an arm whose end points lie on different sides")

    def arms(g, shape, eq_off, m_eq):
        """Enumerate the stencil arms of the equations on grid g (m_eq = momentum component
        or -1 for continuity)."""
        side0 = sides[g]
        goff = np.array([0.0 if d == g else 0.5 for d in range(3)])
        # valid equation nodes
        valid = np.ones(shape, bool)
        if g >= 0:
            valid[tuple(slice(0, 1) if d == g else slice(None) for d in range(3))] = False
            valid[tuple(slice(N, N + 1) if d == g else slice(None) for d in range(3))] = False
        out = []
        if g >= 0:
            # Laplacian arms along each axis d: neighbour on the same grid, coefficient -mu/h^2
            for d in range(3):
                for sgn in (-1, 1):
                    out.append(("lap", d, sgn))
            # pressure-gradient arms along m: p at -h/2 (coeff -1/h) and +h/2 (coeff +1/h)
            for sgn in (-1, 1):
                out.append(("pg", g, sgn))
        else:
            for d in range(3):
                for sgn in (-1, 1):
                    out.append(("div", d, sgn))
        for kind, d, sgn in out:
            if kind == "lap":
                nb_side = np.zeros(shape, bool)
                src = [slice(None)] * 3
                dst = [slice(None)] * 3
                if sgn > 0:
                    src[d] = slice(1, None)
                    dst[d] = slice(0, -1)
                else:
                    src[d] = slice(0, -1)
                    dst[d] = slice(1, None)
                has = np.zeros(shape, bool)
                has[tuple(dst)] = True
                nb_side[tuple(dst)] = side0[tuple(src)]
                irr = valid & has & (nb_side != side0)
                if d == g:
                    # neighbour on a box face: never crossed when Omega is inside the box
                    pass
                coef = -mu / h ** 2
                fam = _family_of(d, -1 if d == g else g)
                comp = g
            elif kind == "pg":
                # p index along g: node a sits between p[a-1] (sgn -1) and p[a] (sgn +1)
                ps = sides[-1]
                nb_side = np.zeros(shape, bool)
                has = np.zeros(shape, bool)
                src = [slice(None)] * 3
                dst = [slice(None)] * 3
                if sgn > 0:
                    src[d] = slice(0, N)
                    dst[d] = slice(0, N)
                else:
                    src[d] = slice(0, N)
                    dst[d] = slice(1, N + 1)
                nb_side[tuple(dst)] = ps[tuple(src)]
                has[tuple(dst)] = True
                irr = valid & has & (nb_side != side0)
                coef = sgn / h
                fam = _family_of(d, -1)
                comp = -1
            else:  # div: cell a between faces a (sgn -1, coeff -1/h) and a+1 (sgn +1, +1/h)
                us = sides[d]
                nb_side = np.zeros(shape, bool)
                src = [slice(None)] * 3
                if sgn > 0:
                    src[d] = slice(1, N + 1)
                else:
                    src[d] = slice(0, N)
                nb_side[...] = us[tuple(src)]
                irr = nb_side != side0
                coef = sgn / h
                fam = _family_of(d, -1)
                comp = d
            I = np.argwhere(irr)
            if len(I) == 0:
                continue
            flat = np.ravel_multi_index(I.T, shape) + eq_off
            s0 = np.where(side0[tuple(I.T)], 1.0, -1.0)
            ax = transverse_axes(d)
            step = 1.0 if kind == "lap" else 0.5          # arm length in units of h
            for r in range(len(I)):
                node = I[r]
                z0 = lo + (node + goff) * h
                zq = z0.copy()
                zq[d] += sgn * step * h
                # half-step interval range covered by the arm
                ja = int(round((min(z0[d], zq[d]) - lo) / (0.5 * h)))
                jb = int(round((max(z0[d], zq[d]) - lo) / (0.5 * h)))
                t = find(fam, int(node[ax[0]]), int(node[ax[1]]), ja, jb)
                xi = zq[d] - cr.pos[t]
                base = t * NJ
                cC = -s0[r] * coef
                if comp >= 0:
                    ent = [(jidx_u(comp), 1.0), (jidx_du(comp, d), xi), (jidx_ddu(comp, d, d), 0.5 * xi * xi)]
                else:
                    ent = [(jidx_p(), 1.0), (jidx_dp(d), xi)]
                for jj, wgt in ent:
                    rows.append(flat[r])
                    cols.append(base + jj)
                    vals.append(cC * wgt)

    for m in range(3):
        arms(m, mac.ushape(m), off[m], m)
    arms(-1, (N, N, N), off[3], -1)
    T = len(cr.fam)
    return sps.csr_matrix((vals, (rows, cols)), shape=(off[-1], T * NJ))
