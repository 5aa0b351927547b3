"""Oracle interpolation of the interior trace u+ at control points (Sec. 4.4).

TEST INFRASTRUCTURE ONLY (see the package docstring).

For a control point x and velocity component m, a quadratic polynomial in (z - x) is fitted
through ten nodes z_i of T^m; at nodes outside Omega the grid value is first shifted by the
jump function J_i (second-order Taylor expansion of the jump from x to z_i), so that all ten
values belong to the interior extension.  The value of the polynomial at x is u+_m(x).

Reading of "ten closest grid nodes" (the literal ten nearest can be eight corners of one cell
plus two nodes, which are not unisolvent for quadratics): z0 is the node of T^m nearest to x
(round half up), s_k = sign((x - z0)_k) with 0 -> +1, and the stencil is
  z0, z0 +- h e_k (k = 1..3), z0 + h(s1 e1 + s2 e2), z0 + h(s1 e1 + s3 e3), z0 + h(s2 e2 + s3 e3),
which matches the one-quadrant picture of the paper's figure and is unisolvent.
Polynomial basis in d = (z - x)/h: [1, d1, d2, d3, d1^2/2, d2^2/2, d3^2/2, d2 d3, d1 d3, d1 d2].
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sps

from .surface import NJ, jidx_u, jidx_du, jidx_ddu


def stencil(x, m, N, lo, h):
    """Ten stencil node indices (10, 3) of T^m for the point x."""
    off = np.array([0.0 if d == m else 0.5 for d in range(3)])
    z0 = np.floor((x - lo) / h - off + 0.5).astype(np.int64)
    zc = lo + (z0 + off) * h
    s = np.where(x - zc >= 0, 1, -1)
    E = np.eye(3, dtype=np.int64)
    nodes = [z0]
    for k in range(3):
        nodes.append(z0 - E[k])
        nodes.append(z0 + E[k])
    nodes.append(z0 + s[0] * E[0] + s[1] * E[1])
    nodes.append(z0 + s[0] * E[0] + s[2] * E[2])
    nodes.append(z0 + s[1] * E[1] + s[2] * E[2])
    return np.array(nodes)


def basis(d):
    d1, d2, d3 = d[..., 0], d[..., 1], d[..., 2]
    return np.stack([np.ones_like(d1), d1, d2, d3, 0.5 * d1 ** 2, 0.5 * d2 ** 2, 0.5 * d3 ** 2,
                     d2 * d3, d1 * d3, d1 * d2], -1)


def weights(x, nodes, m, lo, h):
    off = np.array([0.0 if d == m else 0.5 for d in range(3)])
    z = lo + (nodes + off) * h
    V = basis((z - x) / h)                   # (10, 10)
    e0 = np.zeros(10)
    e0[0] = 1.0
    return np.linalg.solve(V.T, e0), z       # first row of V^{-1}


def interpolation_matrices(cr, sides, N, lo, h, both_sides=False):
    """W (3n x |u|): grid part; E (3n x T*34): jump-function part of the interior limit u+
    (the jump function J_i at the stencil nodes outside Omega).

    With both_sides, also returns E_all: the jump function at every stencil node, so that the
    exterior limit is u- = W u + (E - E_all) jumps (stencil nodes inside Omega carry -J_i).

    The flat velocity vector concatenates u0 (N+1,N,N), u1 (N,N+1,N), u2 (N,N,N+1)."""
    n = len(cr.cp_target)
    sizes = [(N + 1) * N * N] * 3
    uoff = np.concatenate([[0], np.cumsum(sizes)])
    Wr, Wc, Wv, Er, Ec, Ev = [], [], [], [], [], []
    Ar, Ac, Av = [], [], []
    for c in range(n):
        t = cr.cp_target[c]
        x = cr.xyz[t]
        for m in range(3):
            shape = tuple(N + 1 if d == m else N for d in range(3))
            nodes = stencil(x, m, N, lo, h)
            w, z = weights(x, nodes, m, lo, h)
            row = 3 * c + m
            for i in range(10):
                a = nodes[i]
                lo_ok = (a >= 0).all() and all(a[d] < shape[d] for d in range(3))
                inner = (a[m] >= 1) and (a[m] <= N - 1)
                if not (lo_ok and inner):
                    raise RuntimeError("interpolation stencil leaves the interior nodes")
                Wr.append(row)
                Wc.append(uoff[m] + np.ravel_multi_index(tuple(a), shape))
                Wv.append(w[i])
                dz = z[i] - x
                base = t * NJ
                # jump function J_i: second-order Taylor polynomial of the jump from x to z_i
                cols = [base + jidx_u(m)]
                vals = [w[i]]
                for k in range(3):
                    cols.append(base + jidx_du(m, k)); vals.append(w[i] * dz[k])
                    for l in range(3):
                        cols.append(base + jidx_ddu(m, k, l)); vals.append(w[i] * 0.5 * dz[k] * dz[l])
                Ar += [row] * len(cols); Ac += cols; Av += vals
                if not sides[m][tuple(a)]:
                    Er += [row] * len(cols); Ec += cols; Ev += vals
    W = sps.csr_matrix((Wv, (Wr, Wc)), shape=(3 * n, uoff[-1]))
    E = sps.csr_matrix((Ev, (Er, Ec)), shape=(3 * n, len(cr.fam) * NJ))
    if both_sides:
        Eall = sps.csr_matrix((Av, (Ar, Ac)), shape=(3 * n, len(cr.fam) * NJ))
        return W, E, Eall
    return W, E
