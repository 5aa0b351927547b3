"""Oracle boundary integral operator, its transpose, GMRES and the Dirichlet BVP.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Paper: Sec. 3 (representation u = G f - M phi; second-kind BIE 1/2 phi - M phi = g - G f,
solved by GMRES), Prop. 4.1-4.4 (volume and double-layer integrals are solutions of simple
interface problems; the interior trace of the double-layer interface solution is
1/2 phi - M phi), Remark 3.1 (unified interface problem; Navier in generalised Stokes form),
Algorithm 1 (steps 1-3), Sec. 5 (GMRES from a zero guess, stop on the relative residual).

K phi is computed, for a density phi at the control points, as
  fit -> jumps -> corrections -> MAC solve -> interpolation,
i.e. K = W S C J F + E J F, with F the least-squares fit, J the jump relations, C the
corrections, S the Schur-CG MAC solve, W the grid part and E the jump-function part of the
interpolation.  The transpose is the product of the transposes (the MAC solve transposes as
described in mac.MAC.solve_transpose).

GMRES reading: unrestarted, modified Gram-Schmidt Arnoldi, Givens rotations, stop when the
residual norm relative to the initial one (= ||b|| for the zero guess) is below tol.

Two forms of the trace (a reading; the paper interpolates the interior limit only):
  form="interior": K phi = u+, the interior limit interpolated with the jump function built
      from the jumps at the control point, whose value part is the density itself;
  form="average" (default):  K phi = 1/2 phi + (u+ + u-)/2, i.e. 1/2 phi - M phi with the double-layer
      integral -M phi taken as the mean of the two one-sided limits (Prop. 4.2 / 4.4), both
      interpolated from the same ten nodes with the jump function whose value part is the
      least-squares fitted value at the control point (the derivative parts are the same in
      both forms).  For smooth densities the two forms differ by the fit's O(h^3) value error;
      for densities that oscillate on the grid scale (which the grid solution cannot carry)
      the interior form acts like the exterior weight fraction of the stencil, which ranges
      over [0, 1], while the average form acts like 1/2, as the second-kind equation does.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sps

from .geometry import Grid, LevelSet, build_crossings, node_sides
from .surface import fit_matrix, jump_matrix, NJ
from .mac import MAC, correction_matrix, rhs_layout
from .interp import interpolation_matrices

STOKES, NAVIER = 0, 1


def _blockdiag(A):
    """Block-diagonal sparse matrix from a stack of dense blocks (T, r, c)."""
    T, r, c = A.shape
    rows = (np.arange(T)[:, None, None] * r + np.arange(r)[None, :, None]).repeat(c, 2)
    cols = (np.arange(T)[:, None, None] * c + np.arange(c)[None, None, :]).repeat(r, 1)
    return sps.csr_matrix((A.ravel(), (rows.ravel(), cols.ravel())), shape=(T * r, T * c))


class Oracle:
    def __init__(self, cfg, cg_rtol=1e-13, workers=None, form="average"):
        if form not in ("interior", "average"):
            raise ValueError("form must be 'interior' or 'average'")
        self.form = form
        self.cfg = cfg
        self.N, self.lo, self.hi = cfg.N, cfg.lo, cfg.hi
        self.h = (cfg.hi - cfg.lo) / cfg.N
        self.pde, self.mu, self.lam = cfg.pde, cfg.mu, cfg.lam
        self.cg_rtol = cg_rtol
        self.grid = Grid(cfg.N, cfg.lo, cfg.hi)
        self.ls = LevelSet(cfg.shape)
        self.cr = build_crossings(self.grid, self.ls)
        self.sides = node_sides(self.grid, self.ls)
        self.n = len(self.cr.cp_target)
        self.T = len(self.cr.fam)
        P, self.neighbours, Sraw = fit_matrix(self.cr, self.h, raw_values=True)
        self.Fit = sps.kron(P, sps.identity(3), format="csr")            # (18T, 3n)
        A, B = jump_matrix(self.pde, self.mu, self.lam, self.cr)
        self.Jmat = _blockdiag(A)                                          # (34T, 18T)
        self.Bmat = _blockdiag(B)                                          # (34T, 3T)
        self.mac = MAC(cfg.N, cfg.lo, cfg.hi, self.pde, self.mu, self.lam, workers=workers)
        self.Cmat = correction_matrix(self.mac, self.sides, self.cr)
        self.W, self.E, Eall = interpolation_matrices(self.cr, self.sides, cfg.N, cfg.lo, self.h, both_sides=True)
        if form == "average":
            # jump function of the mean limit: exterior nodes +J/2, interior nodes -J/2
            self.Eavg = (self.E - 0.5 * Eall).tocsr()
            # fit with the fitted value (not the density) at the control-point targets
            tgt = np.asarray(self.cr.cp_target)
            Pv = P.tolil()
            for c, t in enumerate(tgt):
                Pv[6 * t] = Sraw[c]
            self.FitRaw = sps.kron(Pv.tocsr(), sps.identity(3), format="csr")
        self.rhs_off = rhs_layout(cfg.N)
        self.last_cg_iters = 0

    # ------------------------------------------------------------------ helpers
    @property
    def points(self):
        return self.cr.xyz[self.cr.cp_target]

    @property
    def normals(self):
        return self.cr.normal[self.cr.cp_target]

    def split_rhs(self, v):
        o, N = self.rhs_off, self.N
        Fu = [v[o[m]:o[m + 1]].reshape(self.mac.ushape(m)) for m in range(3)]
        return Fu, v[o[3]:o[4]].reshape((N, N, N))

    def join_u(self, u):
        return np.concatenate([x.ravel() for x in u])

    def volume_source(self, f):
        """f~ = f in Omega, 0 outside, at the nodes of T^1..T^3 (Prop. 4.1, 4.3), and
        [[f]] = f at every crossing point (f~ jumps from f to 0 across the surface)."""
        Fu = []
        for m in range(3):
            X = self.grid.all_nodes(m)
            v = np.where(self.sides[m], f(X[..., 0], X[..., 1], X[..., 2])[..., m], 0.0)
            Fu.append(v)
        X = self.cr.xyz
        Fj = f(X[:, 0], X[:, 1], X[:, 2])
        return Fu, Fj

    # ------------------------------------------------------------------ operator
    def interface_solve(self, phi, f=None):
        """Solve the unified interface problem ([[u]] = phi, [[sigma n]] = 0, body force
        f~); returns jumps, velocity, pressure."""
        phi = np.asarray(phi, float).reshape(self.n, 3)
        jumps = self.Jmat @ (self.Fit @ phi.ravel())
        vol = None
        if f is not None:
            vol, Fj = self.volume_source(f)
            jumps = jumps + self.Bmat @ Fj.ravel()
        rhs = self.Cmat @ jumps
        Fu, Fp = self.split_rhs(rhs)
        if vol is not None:
            Fu = [Fu[m] + vol[m] for m in range(3)]
        u, p, it = self.mac.solve(Fu, Fp, rtol=self.cg_rtol)
        self.last_cg_iters = it
        return jumps, u, p

    def _trace(self, phi, jumps, u, form, f=None):
        """K phi read off one interface solve (jumps, grid velocity u) in trace form `form`."""
        if form == "interior":
            return (self.W @ self.join_u(u) + self.E @ jumps).reshape(self.n, 3)
        if not hasattr(self, "Eavg"):
            raise ValueError("the average form needs an oracle built with form='average'")
        phi = np.asarray(phi, float).reshape(self.n, 3)
        jr = self.Jmat @ (self.FitRaw @ phi.ravel())
        if f is not None:
            jr = jr + self.Bmat @ self.volume_source(f)[1].ravel()
        return (0.5 * phi.ravel() + self.W @ self.join_u(u) + self.Eavg @ jr).reshape(self.n, 3)

    def eval(self, phi, f=None, form=None):
        """K phi = u+ at the control points for the double-layer interface problem (f None);
        with f, the trace of the unified interface problem (volume + double layer).  form
        overrides the oracle's trace form for this call."""
        jumps, u, p = self.interface_solve(phi, f)
        return self._trace(phi, jumps, u, form or self.form, f)

    def eval_both(self, phi):
        """K phi in both trace forms from one interface solve (the grid solution is common to
        the two forms; they differ only in how the trace is read off it)."""
        jumps, u, p = self.interface_solve(phi)
        return {fm: self._trace(phi, jumps, u, fm) for fm in ("interior", "average")}

    def _adjoint_from(self, w, rhs_bar, form):
        if form == "interior":
            jbar = self.Cmat.T @ rhs_bar + self.E.T @ w
            return (self.Fit.T @ (self.Jmat.T @ jbar)).reshape(self.n, 3)
        if not hasattr(self, "Eavg"):
            raise ValueError("the average form needs an oracle built with form='average'")
        out = self.Fit.T @ (self.Jmat.T @ (self.Cmat.T @ rhs_bar))
        out += self.FitRaw.T @ (self.Jmat.T @ (self.Eavg.T @ w)) + 0.5 * w
        return out.reshape(self.n, 3)

    def _adjoint_solve(self, w):
        ub = self.W.T @ w
        o = self.rhs_off
        ubar = [ub[o[m]:o[m + 1]].reshape(self.mac.ushape(m)) for m in range(3)]
        Fu_bar, Fp_bar, it = self.mac.solve_transpose(ubar, rtol=self.cg_rtol)
        self.last_cg_iters = it
        return np.concatenate([x.ravel() for x in Fu_bar] + [Fp_bar.ravel()])

    def eval_adjoint(self, w, form=None):
        w = np.asarray(w, float).ravel()
        return self._adjoint_from(w, self._adjoint_solve(w), form or self.form)

    def eval_adjoint_both(self, w):
        """K^T w in both trace forms from one transposed MAC solve (W^T w is common)."""
        w = np.asarray(w, float).ravel()
        rb = self._adjoint_solve(w)
        return {fm: self._adjoint_from(w, rb, fm) for fm in ("interior", "average")}

    # ------------------------------------------------------------------ GMRES + BVP
    @staticmethod
    def gmres(apply, b, tol, maxit=200):
        b = np.asarray(b, float).ravel()
        beta = np.linalg.norm(b)
        x = np.zeros_like(b)
        if beta == 0:
            return x, 0, [0.0]
        Q = [b / beta]
        Hh = np.zeros((maxit + 1, maxit))
        cs, sn = np.zeros(maxit), np.zeros(maxit)
        g = np.zeros(maxit + 1)
        g[0] = beta
        hist = [1.0]
        k = 0
        for k in range(maxit):
            v = apply(Q[k])
            for i in range(k + 1):
                Hh[i, k] = np.dot(Q[i], v)
                v = v - Hh[i, k] * Q[i]
            Hh[k + 1, k] = np.linalg.norm(v)
            if Hh[k + 1, k] > 0:
                Q.append(v / Hh[k + 1, k])
            else:
                Q.append(np.zeros_like(v))
            for i in range(k):
                a, c = Hh[i, k], Hh[i + 1, k]
                Hh[i, k] = cs[i] * a + sn[i] * c
                Hh[i + 1, k] = -sn[i] * a + cs[i] * c
            r = np.hypot(Hh[k, k], Hh[k + 1, k])
            cs[k], sn[k] = Hh[k, k] / r, Hh[k + 1, k] / r
            Hh[k, k] = r
            Hh[k + 1, k] = 0.0
            g[k + 1] = -sn[k] * g[k]
            g[k] = cs[k] * g[k]
            hist.append(abs(g[k + 1]) / beta)
            if hist[-1] < tol:
                break
        m = k + 1
        y = np.linalg.solve(np.triu(Hh[:m, :m]), g[:m])
        x = sum(y[i] * Q[i] for i in range(m))
        return x, m, hist

    def solve_bvp(self, g, f=None, tol=1e-8, maxit=200):
        """Dirichlet BVP (Algorithm 1 step 3): b = volume trace, GMRES on K phi = g - b, then
        the unified interface solve gives (u_h, p_h)."""
        g = np.asarray(g, float).reshape(self.n, 3)
        b = self.eval(np.zeros((self.n, 3)), f) if f is not None else np.zeros((self.n, 3))
        phi, iters, hist = self.gmres(lambda v: self.eval(v).ravel(), (g - b).ravel(), tol, maxit)
        phi = phi.reshape(self.n, 3)
        _, u, p = self.interface_solve(phi, f)
        return phi, u, p, iters, hist

    # ------------------------------------------------------------------ errors (Sec. 5)
    def errors(self, u, p, u_exact, p_exact):
        """Normalised max and l2 errors over MAC nodes in Omega; pressures compared after
        shifting both to zero mean over the cells in Omega."""
        res = {}
        for m in range(3):
            X = self.grid.all_nodes(m)
            msk = self.sides[m].copy()
            ue = u_exact(X[..., 0], X[..., 1], X[..., 2])[..., m][msk]
            e = u[m][msk] - ue
            res[f"u{m}_max"] = np.abs(e).max() / np.abs(ue).max()
            res[f"u{m}_l2"] = np.linalg.norm(e) / np.linalg.norm(ue)
        X = self.grid.all_nodes(-1)
        msk = self.sides[-1]
        pe = p_exact(X[..., 0], X[..., 1], X[..., 2])[msk]
        ph = p[msk]
        pe = pe - pe.mean()
        ph = ph - ph.mean()
        res["p_max"] = np.abs(ph - pe).max() / np.abs(pe).max()
        res["p_l2"] = np.linalg.norm(ph - pe) / np.linalg.norm(pe)
        return res
