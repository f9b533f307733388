"""Implicit Euler time stepping with contact (float64, CPU).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

One frame of Incremental Potential Contact (the loop the paper runs its
examples with, section "Examples": Newton iterations on the incremental
potential until the largest displacement per time step falls below a
tolerance), with the contact set found anew at every Newton iterate and every
line-search trial (``collision.Surface.detect``) and the step bounded by CCD
(``collision.Surface.ccd``):

    x_tilde = x + h v + h^2 g
    repeat: contacts at x; p = -H^-1 grad E (projected Hessian, block-Jacobi
            PCG to rtol); stop when max_v |p_v| / h < tol; alpha = CCD bound
            (<= 1); halve alpha until E(x + alpha p) <= E(x) + c alpha grad.p
            (E with the contacts at the trial positions); x += alpha p
    v = (x - x_start) / h

Only free vertices and affine bodies move; fixed vertices keep their
positions.  With affine bodies (``affine.AffineOracle``) x holds the rows of
degrees of freedom (free vertices, then a_1, a_2, a_3, t per body); a body
vertex sits at r_1 a_1 + r_2 a_2 + r_3 a_3 + t (summed left to right), its
displacement under a row motion is the same map of the motion, gravity moves
the t rows only (M4^-1 of a body's gravity force is e_4 (x) g), and the
stencils that reach a body vertex form the body-contact part.
"""
from __future__ import annotations

import math

import numpy as np

from . import affine as oaff
from . import assemble as oasm
from . import pcg as opcg

GRAVITY = np.array([0.0, 0.0, -9.81])


class Stepper:
    """prob: a problem dict (tets / cloth of ``assemble.Oracle``, without
    contacts; x_tilde is recomputed every frame), surface: collision.Surface."""

    def __init__(self, prob, surface, classic=False, gravity=GRAVITY):
        self.p = dict(prob)
        self.p["static"] = False
        self.surface = surface
        self.classic = classic
        self.n = int(prob["n_free"])
        self.x_fixed = np.asarray(prob["x_fixed"], np.float64).reshape(-1, 3)
        self.dhat = float(prob["dhat"])
        self.g = np.asarray(gravity, np.float64)
        self.nb = int(prob.get("n_bodies", 0))
        self.rows = self.n + 4 * self.nb
        if self.nb:
            self.body_of = np.asarray(prob["abd_body"], np.int64)
            self.rest = np.asarray(prob["abd_rest"], np.float64).reshape(-1, 3)

    def _body_points(self, X):
        """r_1 a_1 + r_2 a_2 + r_3 a_3 + t of every body vertex from rows X."""
        q = X[self.n:].reshape(self.nb, 4, 3)[self.body_of]
        r = self.rest
        return r[:, 0:1] * q[:, 0] + r[:, 1:2] * q[:, 1] + r[:, 2:3] * q[:, 2] + q[:, 3]

    def xall(self, x):
        """Positions of every vertex id (free, fixed, body vertices)."""
        X = np.asarray(x, np.float64).reshape(self.rows, 3)
        parts = [X[:self.n], self.x_fixed]
        if self.nb:
            parts.append(self._body_points(X))
        return np.concatenate(parts)

    def pall(self, p):
        """Displacements of every vertex id under the row motion p."""
        P = np.asarray(p, np.float64).reshape(self.rows, 3)
        parts = [P[:self.n], np.zeros_like(self.x_fixed)]
        if self.nb:
            parts.append(self._body_points(P))
        return np.concatenate(parts)

    def oracle_at(self, x, x_tilde):
        """The oracle with the contacts found at positions x."""
        ct, ci, eps = self.surface.detect(self.xall(x), self.dhat)
        q = dict(self.p)
        if not self.nb:
            q.update(x_tilde=x_tilde, ctype=ct, cidx=ci, ee_eps=eps)
            return oasm.Oracle(q, classic=self.classic), len(ct)
        body = (ci >= self.n + self.x_fixed.shape[0]).any(axis=1)
        e = eps if eps is not None else np.zeros(len(ct))
        q.update(x_tilde=x_tilde[:self.n], body_qt=x_tilde[self.n:].reshape(self.nb, 4, 3),
                 ctype=ct[~body], cidx=ci[~body], ee_eps=e[~body] if eps is not None else None,
                 bctype=ct[body], bcidx=ci[body], bee_eps=e[body] if eps is not None else None)
        return oaff.AffineOracle(q, classic=self.classic), len(ct)

    def energy(self, x, x_tilde):
        o, _ = self.oracle_at(x, x_tilde)
        return o.energy(x)

    def frame(self, x, v, h=None, tol=1e-2, max_newton=50, rtol=1e-8, armijo=1e-4, max_halvings=40, s_ccd=0.1):
        """One time step from (x, v); returns (x1, v1, info)."""
        h = float(self.p["h"]) if h is None else h
        x = np.asarray(x, np.float64).reshape(self.rows, 3).copy()
        v = np.asarray(v, np.float64).reshape(self.rows, 3)
        G = np.zeros((self.rows, 3))
        G[:self.n] = self.g
        G[self.n + 3::4] = self.g  # the bodies' t rows
        x_tilde = x + h * v + h * h * G
        x_start = x.copy()
        info = dict(newton_iters=0, cg_iters=0, alphas=[], ccd=[], contacts=[], trials=[], energies=[])
        for _ in range(max_newton):
            o, nc = self.oracle_at(x, x_tilde)
            ev = o.eval(x)
            asm = o.assemble(ev)
            H = o.csr(asm)
            Minv = opcg.block_inverse(o.diag_blocks(asm))
            g = asm["grad"].ravel()
            p, it, _, status = opcg.pcg(lambda u: H @ u, -g, Minv, rtol, 20000)
            info["cg_iters"] += it
            info["contacts"].append(nc)
            info["energies"].append(ev["E"])
            p = p.reshape(self.rows, 3)
            if np.sqrt((p * p).sum(axis=1)).max() / h < tol:
                break
            info["newton_iters"] += 1
            alpha = self.surface.ccd(self.xall(x), self.pall(p), 1.0, s_ccd, self.dhat)
            info["ccd"].append(alpha)
            E0, gp = ev["E"], float(g @ p.ravel())
            for k in range(max_halvings + 1):
                xt = x + alpha * p
                Et = self.energy(xt, x_tilde)
                if Et <= E0 + armijo * alpha * gp:
                    break
                alpha *= 0.5
            info["alphas"].append(alpha)
            info["trials"].append(k + 1)
            x = xt
        return x, (x - x_start) / h, info


def min_distance2(surface, xall):
    """Smallest squared distance over all point-triangle and edge-edge pairs of
    the surface (no shared vertex), brute force."""
    from . import collision as col
    X = [tuple(float(c) for c in row) for row in np.asarray(xall)]
    best = math.inf
    for v in surface.points:
        for tri in surface.tris:
            if v in tri:
                continue
            best = min(best, col.point_triangle(X[v], X[tri[0]], X[tri[1]], X[tri[2]])[2])
    E = surface.edges
    for i in range(len(E)):
        for j in range(i + 1, len(E)):
            if E[i][0] in E[j] or E[i][1] in E[j]:
                continue
            best = min(best, col.segment_segment(X[E[i][0]], X[E[i][1]], X[E[j][0]], X[E[j][1]])[2])
    return best
