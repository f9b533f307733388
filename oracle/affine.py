"""Affine bodies mixed with free vertices (float64, CPU oracle).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

A vertex of affine body b sits at p = A_b r + t_b (r its rest position): the
paper's example of an alternative parameterisation of a position (section
"Introduction", the Affine Body Dynamics example, and section "UNION").  A
contact stencil gathers its vertex positions from the union of free, fixed and
affine-body vertices; its derivatives with respect to the degrees of freedom
follow the chain rule through that union (section "Differentiation of Unioned
Attributes": the Jacobian of a unioned position is the Jacobian of the
parameterisation it came from).

Degrees of freedom, in rows of 3: the n_free free vertices, then per body the
columns a_1, a_2, a_3 of A and t (rows n_free + 4 b + (0, 1, 2, 3)).  So
p = sum_j r_j a_j + t is linear in the rows, with weights w = (r_1, r_2, r_3, 1).

Vertex ids of a stencil: [0, n_free) free, [n_free, n_free + n_fixed) fixed,
[n_free + n_fixed, ...) affine-body vertex k = id - n_free - n_fixed.

Energies (each a plain definition; derivatives by torch.func):

* body inertia 1/2 (q - q~)^T (M4 (x) I3) (q - q~) with M4 = sum_v m_v w_v w_v^T
  over the body's vertices (= 1/2 sum_v m_v |p_v(q) - p_v(q~)|^2);
* orthogonality h^2 k_b 1/2 |A^T A - I|_F^2 (the paper's E_affine regulariser,
  scaled like the elastic energies), its 9x9 Hessian over (a_1, a_2, a_3)
  projected to the PSD cone;
* the barrier of every contact stencil touching a body: its Hessian over the
  stencil's movable positions (free and affine-body vertices) is projected
  there, then mapped to the degrees of freedom, J^T Proj(H_p) J with J the
  (constant) Jacobian of the positions: the reduced-coordinate projection of
  section "Eigendecomposition (EVD) and PSD Projection" (valid since p is
  linear in the degrees of freedom), 6 x 6 for a free-body point-point
  stencil instead of 15 x 15, and 6 x 6 instead of 24 x 24 for two bodies.

The row list of a stencil: its vertices' rows in vertex order, a body's four
rows once (first occurrence), fixed vertices none; local pairs over this list
follow the canonical rule of ``pattern.py`` (lists up to 8 rows, 36 pairs).
"""
from __future__ import annotations

import numpy as np
import torch
from torch.func import grad, hessian, vmap

from . import energy as en
from . import local, pattern

MAX_ROWS = 8


def body_positions(q, rest):
    """p = A r + t for q (4, 3) rows (a_1, a_2, a_3, t) and rest (3,)."""
    return rest[0] * q[0] + rest[1] * q[1] + rest[2] * q[2] + q[3]


def orthogonality(q):
    """1/2 |A^T A - I|_F^2 with A = [a_1 a_2 a_3] (columns) from the rows of q (4, 3)."""
    A = q[:3].T
    G = A.T @ A - torch.eye(3, dtype=q.dtype)
    return 0.5 * (G * G).sum()


def body_inertia(q, qt, M4):
    """1/2 sum_ab M4[a, b] (q_a - qt_a) . (q_b - qt_b)."""
    d = q - qt
    return 0.5 * torch.einsum("ab,ai,bi->", M4, d, d)


class AffineScene:
    """Contacts touching affine bodies plus the bodies' own energies, over the
    full degree-of-freedom vector X (n_rows, 3) = [free vertices; body rows].

    prob keys: n_free, x_fixed, dhat, kappa, h, and
      n_bodies, body_M4 (nb, 4, 4), body_qt (nb, 4, 3), body_k (nb,),
      abd_body (nv,), abd_rest (nv, 3),
      bctype (ns,), bcidx (ns, 4): the stencils touching bodies."""

    def __init__(self, prob, classic=False):
        self.p = prob
        self.n_free = int(prob["n_free"])
        self.nb = int(prob["n_bodies"])
        self.n_rows = self.n_free + 4 * self.nb
        self.x_fixed = local.T(prob["x_fixed"]).reshape(-1, 3)
        self.n_fixed = self.x_fixed.shape[0]
        self.abd_body = np.asarray(prob["abd_body"], np.int64)
        self.abd_rest = np.asarray(prob["abd_rest"], np.float64).reshape(-1, 3)
        self.M4 = local.T(prob["body_M4"]).reshape(-1, 4, 4)
        self.qt = local.T(prob["body_qt"]).reshape(-1, 4, 3)
        self.k = local.T(prob["body_k"]).reshape(-1)
        self.h = float(prob["h"])
        self.classic = classic
        self.ctype = np.asarray(prob["bctype"], np.int64)
        self.cidx = np.asarray(prob["bcidx"], np.int64).reshape(-1, 4)
        # edge-edge mollifier thresholds of these stencils, or none
        self.ee_eps = np.asarray(prob["bee_eps"], np.float64) if prob.get("bee_eps") is not None else None
        self.rows, self.W = self.row_lists(self.cidx)
        # patterns: the body stencils (4 rows each, static) and the body contacts
        brows = self.n_free + 4 * np.arange(self.nb)[:, None] + np.arange(4)[None, :]
        self.body_rows = brows
        self.rp_b, self.ci_b, (self.slot_b,) = pattern.build(self.n_rows, [self.rows], False)
        self.pairs_b = pattern.stencil_pairs(self.rows)

    # ------------------------------------------------------------ the union
    def row_lists(self, cidx):
        """(ns, 8) row lists (-1 padded) and (ns, 4, 8) weights W[s, a, j]: the
        coefficient of row j of the list in the position of stencil vertex a."""
        ns = cidx.shape[0]
        rows = -np.ones((ns, MAX_ROWS), np.int64)
        W = np.zeros((ns, 4, MAX_ROWS))
        base = self.n_free + self.n_fixed
        for s in range(ns):
            lst = []
            for a in range(4):
                v = int(cidx[s, a])
                if v < 0 or (self.n_free <= v < base):
                    continue  # unused or fixed: no degrees of freedom
                if v < self.n_free:
                    rv, wv = [v], [1.0]
                else:
                    k = v - base
                    b = int(self.abd_body[k])
                    rv = [self.n_free + 4 * b + j for j in range(4)]
                    wv = list(self.abd_rest[k]) + [1.0]
                for r, w in zip(rv, wv):
                    if r not in lst:
                        lst.append(r)
                    W[s, a, lst.index(r)] += w
            if len(lst) > MAX_ROWS:
                raise ValueError(f"stencil {s} reaches {len(lst)} rows (at most {MAX_ROWS})")
            rows[s, :len(lst)] = lst
        return rows, W

    def positions(self, X, cidx=None):
        """Stencil vertex positions (ns, 4, 3) and the movable mask (ns, 4)."""
        cidx = self.cidx if cidx is None else cidx
        X = local.T(X).reshape(self.n_rows, 3)
        base = self.n_free + self.n_fixed
        ns = cidx.shape[0]
        xs = torch.zeros(ns, 4, 3)
        mov = torch.zeros(ns, 4, dtype=torch.bool)
        for s in range(ns):
            for a in range(4):
                v = int(cidx[s, a])
                if v < 0:
                    continue
                if v < self.n_free:
                    xs[s, a] = X[v]
                    mov[s, a] = True
                elif v < base:
                    xs[s, a] = self.x_fixed[v - self.n_free]
                else:
                    k = v - base
                    b = int(self.abd_body[k])
                    xs[s, a] = body_positions(X[self.n_free + 4 * b:self.n_free + 4 * b + 4],
                                              local.T(self.abd_rest[k]))
                    mov[s, a] = True
        return xs, mov

    # ------------------------------------------------------------ energies
    def body_terms(self, X, hess=local.PROJECTED):
        """Per body: energy, gradient (nb, 4, 3) and 12 x 12 Hessian over its
        rows: inertia (M4 (x) I3) plus h^2 k times the orthogonality energy (its
        9 x 9 Hessian over a_1..a_3 projected unless hess=EXACT)."""
        X = local.T(X).reshape(self.n_rows, 3)
        q = X[self.n_free:].reshape(self.nb, 4, 3)
        h2 = self.h * self.h
        E_in = vmap(body_inertia)(q, self.qt, self.M4)
        g_in = vmap(grad(body_inertia))(q, self.qt, self.M4)
        H_in = vmap(hessian(body_inertia))(q, self.qt, self.M4).reshape(self.nb, 12, 12)
        E_or = h2 * self.k * vmap(orthogonality)(q)
        g_or = h2 * self.k.view(-1, 1, 1) * vmap(grad(orthogonality))(q)
        H_or = h2 * self.k.view(-1, 1, 1) * vmap(hessian(orthogonality))(q).reshape(self.nb, 12, 12)
        if hess == local.PROJECTED:
            P = torch.zeros_like(H_or)
            P[:, :9, :9] = local.psd_project(H_or[:, :9, :9])
            H_or = P
        return E_in, E_or, g_in + g_or, local.sym(H_in + H_or)

    def contact_terms(self, X, hess=local.PROJECTED):
        """Per body contact: energy, gradient over its row list (ns, 8, 3), the
        row-list Hessian (ns, 24, 24) J^T Proj(H_p) J, and d."""
        xs, mov = self.positions(X)
        E, gp, Hp, d = local.contact_local(xs, torch.as_tensor(self.ctype), mov, float(self.p["kappa"]),
                                           float(self.p["dhat"]), hess, self.classic, self.ee_eps)
        # J: position (vertex a, axis i) -> row list (j, axis l): W[a, j] delta_il
        W = torch.as_tensor(self.W)
        J = torch.einsum("saj,il->saijl", W, torch.eye(3)).reshape(-1, 12, 3 * MAX_ROWS)
        g = (J.transpose(1, 2) @ gp.reshape(-1, 12, 1)).reshape(-1, MAX_ROWS, 3)
        H = J.transpose(1, 2) @ Hp @ J
        return E, g, local.sym(H), d

    def mollifiers(self, X):
        """m(c) of every body contact (1 except for mollified edge-edge stencils)."""
        m = torch.ones(self.cidx.shape[0])
        if self.ee_eps is None:
            return m
        xs, _ = self.positions(X)
        sel = torch.nonzero(torch.as_tensor(self.ctype) == 1).flatten()
        if sel.numel():
            m[sel] = en.ee_mollifier(vmap(en.ee_cross_norm)(xs[sel]), torch.as_tensor(self.ee_eps)[sel])
        return m

    def distances(self, X):
        xs, _ = self.positions(X)
        d = torch.zeros(xs.shape[0])
        ct = torch.as_tensor(self.ctype)
        for t in range(4):
            sel = torch.nonzero(ct == t).flatten()
            if sel.numel():
                d[sel] = vmap(en.DIST[t])(xs[sel])
        return d.numpy()

    # ------------------------------------------------------------ assembly
    def assemble_body_part(self, H):
        """Scatter-adds the row-list Hessians into the body-contact part's
        blocks (as is when row_a <= row_b, transposed otherwise)."""
        vals = np.zeros((len(self.ci_b), 3, 3))
        H = np.asarray(H)
        for s in range(self.rows.shape[0]):
            for q in range(self.slot_b.shape[1]):
                sl = self.slot_b[s, q]
                if sl < 0:
                    continue
                a, b = self.pairs_b[s, q]
                blk = H[s, 3 * a:3 * a + 3, 3 * b:3 * b + 3]
                if self.rows[s, a] > self.rows[s, b]:
                    blk = blk.T
                vals[sl] += blk
        return vals

    def scatter_grad(self, g):
        out = np.zeros((self.n_rows, 3))
        g = np.asarray(g)
        for s in range(self.rows.shape[0]):
            for j in range(MAX_ROWS):
                r = self.rows[s, j]
                if r >= 0:
                    out[r] += g[s, j]
        return out


class AffineOracle:
    """A scene with free vertices (tets, ordinary contacts: ``assemble.Oracle``)
    and affine bodies (``AffineScene``), over X (n_rows, 3).  Parts, each an
    upper-triangular BSR over n_rows rows: static (tets and the other elastic
    stencils, the bodies' 4-row stencils, every diagonal), dynamic (contacts
    between free and fixed vertices only) and body contacts (stencils touching
    a body).  Same interface as ``Oracle`` for ``newton.newton_step``."""

    def __init__(self, prob, classic=False):
        from . import assemble as oasm
        self.p = prob
        self.base = oasm.Oracle(prob, classic=classic)
        self.scene = AffineScene(prob, classic=classic)
        self.n_free = self.scene.n_free
        self.n = self.scene.n_rows
        nb = self.scene.nb
        shift = 4 * nb  # fixed ids move past the body rows in the row space

        def rowids(idx):
            idx = np.asarray(idx, np.int64).copy()
            fixed = idx >= self.n_free
            idx[fixed] += shift
            return idx

        b = self.base
        self.tet_r, self.tri_r, self.hinge_r = rowids(b.tet_idx), rowids(b.tri_idx), rowids(b.hinge_idx)
        self.rp_s, self.ci_s, (self.slot_t, self.slot_f, self.slot_h, self.slot_bd) = pattern.build(
            self.n, [self.tet_r, self.tri_r, self.hinge_r, self.scene.body_rows], True)
        self.cidx_r = rowids(b.cidx)
        self.rp_d, self.ci_d, (self.slot_c,) = pattern.build(self.n, [self.cidx_r], False)
        self.rp_b, self.ci_b, self.slot_b = self.scene.rp_b, self.scene.ci_b, self.scene.slot_b
        self.mass = np.concatenate([b.mass, np.ones(4 * nb)])  # (only used for damping shifts)
        self.cidx = np.concatenate([b.cidx, self.scene.cidx])

    def _x(self, X):
        X = np.asarray(X, np.float64).reshape(self.n, 3)
        return X, X[:self.n_free]

    def eval(self, X, hess=local.PROJECTED):
        X, xf = self._x(X)
        ev = self.base.eval(xf, hess)
        Ein, Eor, gb, Hb = self.scene.body_terms(X, hess)
        Ec, gc, Hc, d = self.scene.contact_terms(X, hess)
        ev.update(X=X, E_body_inertia=Ein.numpy(), E_orth=Eor.numpy(), g_body=gb.numpy(), H_body=Hb.numpy(),
                  E_bc=Ec.numpy(), g_bc=gc.numpy(), H_bc=Hc.numpy(), d_bc=d.numpy())
        ev["E_elastic"] += float(Eor.sum())
        ev["E_inertia"] += float(Ein.sum())
        ev["E_contact"] += float(Ec.sum())
        ev["E"] = ev["E_inertia"] + ev["E_elastic"] + ev["E_contact"]
        return ev

    def assemble(self, ev):
        b = self.base
        n = self.n
        sb = b._scatter_blocks
        vals_s = sb(len(self.ci_s), self.tet_r, b.pairs_t, self.slot_t, ev["H_t"])
        if len(b.tri_idx):
            vals_s += sb(len(self.ci_s), self.tri_r, b.pairs_f, self.slot_f, ev["H_f"])
        if len(b.hinge_idx):
            vals_s += sb(len(self.ci_s), self.hinge_r, b.pairs_h, self.slot_h, ev["H_h"])
        brows = self.scene.body_rows
        vals_s += sb(len(self.ci_s), brows, pattern.stencil_pairs(brows), self.slot_bd, ev["H_body"])
        if not b.static:
            vals_s[self.rp_s[:self.n_free]] += b.mass[:, None, None] * np.eye(3)[None]
        vals_d = sb(len(self.ci_d), self.cidx_r, b.pairs_c, self.slot_c, ev["H_c"])
        vals_b = self.scene.assemble_body_part(ev["H_bc"])
        g = np.zeros((n, 3))
        g[:self.n_free] = b.assemble(ev)["grad"]
        g[self.n_free:] += ev["g_body"].reshape(-1, 3)
        g += self.scene.scatter_grad(ev["g_bc"])
        return dict(values_s=vals_s, values_d=vals_d, values_b=vals_b, grad=g)

    def _parts(self, asm):
        return ((self.rp_s, self.ci_s, asm["values_s"]), (self.rp_d, self.ci_d, asm["values_d"]),
                (self.rp_b, self.ci_b, asm["values_b"]))

    def csr(self, asm):
        import scipy.sparse as sp
        n = self.n
        H = sp.csr_matrix((3 * n, 3 * n))
        for rp, ci, vals in self._parts(asm):
            rows = np.repeat(np.arange(n), np.diff(rp))
            up = sp.bsr_matrix((vals, ci, rp), shape=(3 * n, 3 * n)).tocsr()
            off = rows != ci
            lo = sp.bsr_matrix((vals[off], ci[off], np.concatenate(
                [[0], np.cumsum(np.bincount(rows[off], minlength=n))])), shape=(3 * n, 3 * n)).tocsr().T
            H = H + up + lo
        return H.tocsr()

    def diag_blocks(self, asm):
        D = np.zeros((self.n, 3, 3))
        for rp, ci, vals in self._parts(asm):
            rows = np.repeat(np.arange(self.n), np.diff(rp))
            dg = rows == ci
            D[rows[dg]] += vals[dg]
        return D

    def energy(self, X):
        X, xf = self._x(X)
        Ein, Eor, _, _ = self.scene.body_terms(X)
        d = torch.as_tensor(self.scene.distances(X))
        dhat, kappa = float(self.p["dhat"]), float(self.p["kappa"])
        bfun = en.barrier_ipc_classic if self.base.classic else en.barrier
        act = d < dhat
        Ec = torch.where(act, bfun(torch.where(act, d, torch.full_like(d, dhat)), dhat, kappa), torch.zeros_like(d))
        Ec = Ec * self.scene.mollifiers(X)
        return self.base.energy(xf) + float(Ein.sum()) + float(Eor.sum()) + float(Ec.sum())

    def distances(self, X):
        X, xf = self._x(X)
        return np.concatenate([self.base.distances(xf), self.scene.distances(X)])

    def sides(self, X):
        X, xf = self._x(X)
        xs, _ = self.scene.positions(X)
        sb = en.signed_side(xs, torch.as_tensor(self.scene.ctype)).numpy()
        return np.concatenate([self.base.sides(xf), sb])
