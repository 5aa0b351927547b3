"""Oracle surface calculus: least-squares surface derivatives and interface jump relations.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The correction terms of Sec. 4.3 need, at each crossing point, the jumps of the velocity and
its first and second derivatives along the line, and of the pressure and its first
derivative; the interpolation of Sec. 4.4 needs the full jumps [[u]], [[grad u]], [[hess u]]
at each control point.  The paper states that they follow from the interface conditions and
the PDE but omits the derivation (end of Sec. 4.3).  The derivation used here:

Surface derivatives (reading; the paper defers "equilibration" to a cited work): the density
is fitted, per component, by an unweighted least-squares quadratic in the tangent-plane
coordinates xi = (t1.(x-x0), t2.(x-x0))/h over the control points x_j with |x_j - x0| <= 2.5h
and n_j.n0 >= 0.5 (radius grown by 0.5h up to 4h until there are at least 12), basis
[1, xi1, xi2, xi1^2/2, xi1 xi2, xi2^2/2].  At a control point the value is the density there.

First order, with w = d[[u]]/dn and s = sum_a t_a . Phi_a:
  [[grad u]] = w n^T + sum_a Phi_a t_a^T (rows = components),
  tangential traction: t_a . w = -n . Phi_a + t_a . T / mu,
  Stokes:  n . w = -s (jump of div u vanishes),  [[p]] = 2 mu n.w - n.T,
  Navier:  n . w = (n.T - lambda s)/(lambda + 2 mu),  [[p]] = -(lambda+mu)[[div u]].
Second order, per component i, H_i = [[hess u_i]] in the frame (t1, t2, n):
  V_ab = Phi_ab - kappa_ab w               (Monge patch identity),
  V_an from the tangential derivative of the traction condition
      (d_a [[sigma]]) n - sum_b kappa_ab [[sigma]] t_b = d_a T,
  plus (Stokes) the tangential derivative of [[div u]] = 0; then V_nn and the normal
  pressure derivative from the momentum jump -mu [[lap u]] + [[grad p]] = [[f]] and (Stokes)
  the normal derivative of [[div u]] = 0.  For Navier [[grad p]] = -(lambda+mu)[[grad div u]].
Every unknown has a closed form (the coefficient matrices are those of a flat interface).
"""
from __future__ import annotations

import numpy as np
from scipy.spatial import cKDTree
import scipy.sparse as sps

from .geometry import GeometryError

STOKES, NAVIER = 0, 1


def fit_matrix(cr, h, raw_values=False):
    """Least-squares fit weights as a sparse matrix of shape (6*T, n).

    Row 6*t+q gives quantity q of target t (0 value, 1-2 first derivatives d/dxi_a in physical
    units, 3-5 second derivatives 11, 12, 22) as a combination of the density at control
    points.  With raw_values, also returns the (n, n) matrix S whose row c is the fitted
    value (before the exact density replaces it) at control point c."""
    X = cr.xyz[cr.cp_target]
    Ncp = cr.normal[cr.cp_target]
    tree = cKDTree(X)
    T = len(cr.fam)
    rows, cols, vals = [], [], []
    # 2.5h plus a relative 1e-9 so that neighbours at exactly 2.5h (symmetric grids) are
    # included whatever the rounding of the distance
    radius = np.full(T, 2.5 * h + 1e-9 * h)
    nb = [None] * T
    pending = np.arange(T)
    while len(pending):
        lists = tree.query_ball_point(cr.xyz[pending], radius[pending])
        still = []
        for t, L in zip(pending, lists):
            L = np.array(sorted(L), dtype=np.int64)
            if len(L):
                L = L[Ncp[L] @ cr.normal[t] >= 0.5]
            if len(L) >= 12:
                nb[t] = L
            elif radius[t] + 0.5 * h <= 4.0 * h + 1e-12 * h:
                radius[t] += 0.5 * h
                still.append(t)
            else:
                raise GeometryError("fewer than 12 control points within 4h of a target")
        pending = np.array(still, dtype=np.int64)
    scale = np.array([1.0, 1 / h, 1 / h, 1 / h ** 2, 1 / h ** 2, 1 / h ** 2])
    Sr, Sc, Sv = [], [], []
    for t in range(T):
        L = nb[t]
        d = X[L] - cr.xyz[t]
        xi1 = d @ cr.t1[t] / h
        xi2 = d @ cr.t2[t] / h
        A = np.stack([np.ones_like(xi1), xi1, xi2, 0.5 * xi1 ** 2, xi1 * xi2, 0.5 * xi2 ** 2], 1)
        P = np.linalg.pinv(A) * scale[:, None]          # (6, K)
        if cr.cp[t] >= 0:                                # control point target: exact value
            Sr.append(np.full(len(L), cr.cp[t]))
            Sc.append(L)
            Sv.append(P[0].copy())
            P[0, :] = 0.0
            P[0, np.nonzero(L == cr.cp[t])[0][0]] = 1.0
        for q in range(6):
            rows.append(np.full(len(L), 6 * t + q))
            cols.append(L)
            vals.append(P[q])
    M = sps.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                       shape=(6 * T, len(cr.cp_target)))
    if raw_values:
        n = len(cr.cp_target)
        S = sps.csr_matrix((np.concatenate(Sv), (np.concatenate(Sr), np.concatenate(Sc))), shape=(n, n))
        return M, nb, S
    return M, nb


def jump_relations(pde, mu, lam, n, t1, t2, kappa, Phi, Phi_a, Phi_ab, F, Tr=None, dTr=None):
    """Jumps at surface points from surface derivatives of [[u]] and the interface data.

    Shapes (M points): n,t1,t2 (M,3); kappa (M,2,2); Phi (M,3); Phi_a (M,2,3) = d/dxi_a;
    Phi_ab (M,3,3) = second derivatives [11, 12, 22] x component; F = [[f]] (M,3);
    Tr = [[sigma n]] (M,3) and dTr (M,2,3) its tangential derivatives (zero if None).
    Returns J0 (M,3), Gu (M,3,3) [i,k] = d_k [[u_i]], H (M,3,3,3) [i,k,l], p (M,), gp (M,3).
    """
    M = len(n)
    Tr = np.zeros((M, 3)) if Tr is None else Tr
    dTr = np.zeros((M, 2, 3)) if dTr is None else dTr
    t = np.stack([t1, t2], 1)                          # (M,2,3)
    dot = lambda a, b: np.einsum("...i,...i->...", a, b)
    # ---- first order
    s = dot(t[:, 0], Phi_a[:, 0]) + dot(t[:, 1], Phi_a[:, 1])
    wt = np.stack([-dot(n, Phi_a[:, a]) + dot(t[:, a], Tr) / mu for a in range(2)], 1)  # (M,2)
    if pde == STOKES:
        wn = -s
        jp = 2 * mu * wn - dot(n, Tr)
    else:
        wn = (dot(n, Tr) - lam * s) / (lam + 2 * mu)
        jdiv = wn + s
        jp = -(lam + mu) * jdiv
    w = wn[:, None] * n + wt[:, 0, None] * t[:, 0] + wt[:, 1, None] * t[:, 1]
    Gu = w[:, :, None] * n[:, None, :] + sum(Phi_a[:, a, :, None] * t[:, a, None, :] for a in range(2))
    I = np.eye(3)
    sym = Gu + np.swapaxes(Gu, 1, 2)
    if pde == STOKES:
        sig = -jp[:, None, None] * I + mu * sym
    else:
        sig = lam * jdiv[:, None, None] * I + mu * sym
    # ---- second order, tangential-tangential block
    ab = {(0, 0): 0, (0, 1): 1, (1, 0): 1, (1, 1): 2}
    V = {(a, b): Phi_ab[:, ab[(a, b)]] - kappa[:, a, b, None] * w for a in range(2) for b in range(2)}
    # ---- tangential-normal block
    Van, pi_a, dlt_a = [], [], []
    for a in range(2):
        Rp = dTr[:, a] + sum(kappa[:, a, b, None] * np.einsum("mij,mj->mi", sig, t[:, b]) for b in range(2))
        tV = dot(t[:, 0], V[(a, 0)]) + dot(t[:, 1], V[(a, 1)])
        if pde == STOKES:
            nVan = -tV
            pi_a.append(2 * mu * nVan - dot(n, Rp))
        else:
            nVan = (dot(n, Rp) - lam * tV) / (lam + 2 * mu)
            dlt_a.append(tV + nVan)
        tc = [dot(t[:, c], Rp) / mu - dot(n, V[(a, c)]) for c in range(2)]
        Van.append(nVan[:, None] * n + tc[0][:, None] * t[:, 0] + tc[1][:, None] * t[:, 1])
    # ---- normal-normal block
    S12 = V[(0, 0)] + V[(1, 1)]
    tVan = dot(t[:, 0], Van[0]) + dot(t[:, 1], Van[1])
    if pde == STOKES:
        nVnn = -tVan
        pin = mu * (nVnn + dot(n, S12)) + dot(n, F)
        gp = pi_a[0][:, None] * t[:, 0] + pi_a[1][:, None] * t[:, 1] + pin[:, None] * n
        Vnn = (gp - F) / mu - S12
    else:
        nVnn = -(dot(n, F) + mu * dot(n, S12) + (lam + mu) * tVan) / (lam + 2 * mu)
        dn = tVan + nVnn
        g = dlt_a[0][:, None] * t[:, 0] + dlt_a[1][:, None] * t[:, 1] + dn[:, None] * n
        Vnn = -(F + (lam + mu) * g) / mu - S12
        gp = -(lam + mu) * g
    outer = lambda a, b: a[:, :, None] * b[:, None, :]
    H = np.zeros((M, 3, 3, 3))
    for i in range(3):
        Hi = np.zeros((M, 3, 3))
        for a in range(2):
            for b in range(2):
                Hi += V[(a, b)][:, i, None, None] * outer(t[:, a], t[:, b])
            Hi += Van[a][:, i, None, None] * (outer(t[:, a], n) + outer(n, t[:, a]))
        Hi += Vnn[:, i, None, None] * outer(n, n)
        H[:, i] = Hi
    return Phi.copy(), Gu, H, jp, gp


# Layout of the flattened jump vector of one surface point (34 entries):
#   0..2   [[u_i]]
#   3..11  [[d_k u_i]]        at 3 + 3 i + k
#   12..29 [[d_k d_l u_i]]     at 12 + 6 i + (00,11,22,12,02,01 -> 0..5)
#   30     [[p]]
#   31..33 [[d_k p]]
NJ = 34
_HIDX = {(0, 0): 0, (1, 1): 1, (2, 2): 2, (1, 2): 3, (2, 1): 3, (0, 2): 4, (2, 0): 4, (0, 1): 5, (1, 0): 5}


def jidx_u(i):
    return i


def jidx_du(i, k):
    return 3 + 3 * i + k


def jidx_ddu(i, k, l):
    return 12 + 6 * i + _HIDX[(k, l)]


def jidx_p():
    return 30


def jidx_dp(k):
    return 31 + k


def flatten_jumps(J0, Gu, H, jp, gp):
    M = len(J0)
    out = np.zeros((M, NJ))
    for i in range(3):
        out[:, jidx_u(i)] = J0[:, i]
        for k in range(3):
            out[:, jidx_du(i, k)] = Gu[:, i, k]
            for l in range(k, 3):
                out[:, jidx_ddu(i, k, l)] = H[:, i, k, l]
    out[:, jidx_p()] = jp
    for k in range(3):
        out[:, jidx_dp(k)] = gp[:, k]
    return out


def jump_matrix(pde, mu, lam, cr):
    """Per-target linear maps from (fit quantities, [[f]]) to the 34 jump values.

    Returns A (T, 34, 18) acting on fit values ordered [q*3 + i] (q = 0..5 as in fit_matrix,
    i = component) and B (T, 34, 3) acting on [[f]].  The jump relations are linear in their
    inputs (with zero traction jump), so each column is the response to one unit input."""
    T = len(cr.fam)
    A = np.zeros((T, NJ, 18))
    B = np.zeros((T, NJ, 3))

    def run(fitvals, F):
        Phi = fitvals[:, 0]
        Phi_a = fitvals[:, 1:3]
        Phi_ab = fitvals[:, 3:6]
        return flatten_jumps(*jump_relations(pde, mu, lam, cr.normal, cr.t1, cr.t2, cr.kappa,
                                              Phi, Phi_a, Phi_ab, F))

    for c in range(18):
        fv = np.zeros((T, 6, 3))
        fv[:, c // 3, c % 3] = 1.0
        A[:, :, c] = run(fv, np.zeros((T, 3)))
    for c in range(3):
        F = np.zeros((T, 3))
        F[:, c] = 1.0
        B[:, :, c] = run(np.zeros((T, 6, 3)), F)
    return A, B
