"""Whole-problem evaluation and assembly (float64, CPU).

``Oracle(problem)`` builds the static (elastic + every free diagonal) and
dynamic (contact) patterns with ``pattern.build`` and then, for positions x:

* ``eval(x)``: per-stencil energies, gradients and local Hessians
  (``local.py``) plus the inertia term 1/2 sum_v m_v |x_v - x_tilde_v|^2
  (or, for a static problem, the gravity potential -sum_v m_v g . x_v);
* ``assemble(ev)``: scatter-adds every local 3x3 block into its slot (as is
  when v_a <= v_b, transposed otherwise), adds m_v I to the static diagonal
  blocks, and sums the gradient per vertex.

The global Hessian is H = H_static + H_dynamic, both upper-triangular BSR with
row-major 3x3 blocks (appendix "Global Hessian Compression").
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import torch

from . import energy as en
from . import local, pattern

F_SPACE, X_SPACE = local.F_SPACE, local.X_SPACE
PROJECTED, EXACT = local.PROJECTED, local.EXACT


class Oracle:
    def __init__(self, prob, proj=F_SPACE, classic=False):
        self.p = prob
        self.n = int(prob["n_free"])
        self.proj = proj
        self.classic = classic
        n = self.n
        self.tet_idx = np.asarray(prob["tet_idx"], np.int64)
        self.cidx = np.asarray(prob["cidx"], np.int64)
        self.ctype = np.asarray(prob["ctype"], np.int64)
        # edge-edge mollifier thresholds (IPC's near-parallel treatment), or none
        self.ee_eps = np.asarray(prob["ee_eps"], np.float64) if prob.get("ee_eps") is not None else None
        nf = len(prob.get("tri_idx", []))
        nh = len(prob.get("hinge_idx", []))
        self.tri_idx = np.full((nf, 4), -1, np.int64)
        if nf:
            self.tri_idx[:, :3] = np.asarray(prob["tri_idx"], np.int64)
        self.hinge_idx = np.asarray(prob["hinge_idx"], np.int64).reshape(-1, 4) if nh else np.zeros((0, 4), np.int64)
        self.rp_s, self.ci_s, (self.slot_t, self.slot_f, self.slot_h) = pattern.build(
            n, [self.tet_idx, self.tri_idx, self.hinge_idx], True)
        self.rp_d, self.ci_d, (self.slot_c,) = pattern.build(n, [self.cidx], False)
        self.pairs_t = pattern.stencil_pairs(self.tet_idx)
        self.pairs_f = pattern.stencil_pairs(self.tri_idx)
        self.pairs_h = pattern.stencil_pairs(self.hinge_idx)
        self.pairs_c = pattern.stencil_pairs(self.cidx)
        t = local.T
        self.x_fixed = t(prob["x_fixed"]).reshape(-1, 3)
        self.dm_inv = t(prob["dm_inv"])
        self.vol = t(prob["vol"])
        nt = self.tet_idx.shape[0]
        if "mu_t" in prob:
            self.mu = t(prob["mu_t"])
            self.lam = t(prob["lam_t"])
        else:
            self.mu = torch.full((nt,), float(prob["mu"]))
            self.lam = torch.full((nt,), float(prob["lam"]))
        self.mass = np.asarray(prob["mass"], np.float64)
        self.x_tilde = np.asarray(prob["x_tilde"], np.float64)
        self.static = bool(prob.get("static", False))
        if nf:
            self.tri_dm_inv = t(prob["tri_dm_inv"]).reshape(-1, 2, 2)
            self.tri_area = t(prob["tri_area"])
        if nh:
            hr = np.asarray(prob["hinge_rest"], np.float64).reshape(-1, 2)
            self.hinge_theta = t(hr[:, 0])
            self.hinge_stiff = t(hr[:, 1])
        self.gravity = np.asarray(prob.get("gravity", [0.0, 0.0, -9.81]), np.float64)

    # ------------------------------------------------------------ pieces
    def inertia(self, x):
        """Inertia (dynamic) or gravity potential (static): energy, gradient."""
        if self.static:
            e = -np.sum(self.mass[:, None] * self.gravity[None, :] * x)
            g = -self.mass[:, None] * self.gravity[None, :] * np.ones_like(x)
            return e, g
        dx = x - self.x_tilde
        return 0.5 * np.sum(self.mass[:, None] * dx * dx), self.mass[:, None] * dx

    def tets(self, x, hess=PROJECTED, mu=None, lam=None):
        if not len(self.tet_idx):  # an empty sum
            return torch.zeros(0), torch.zeros(0, 4, 3), torch.zeros(0, 12, 12)
        xt, free = local.gather_positions(local.T(x), self.x_fixed, self.tet_idx, self.n)
        return local.snh_local(xt, self.dm_inv, self.mu if mu is None else mu,
                               self.lam if lam is None else lam, self.vol,
                               float(self.p["h"]), free, self.proj, hess)

    def tris(self, x, hess=PROJECTED):
        if not len(self.tri_idx):
            return torch.zeros(0), torch.zeros(0, 4, 3), torch.zeros(0, 12, 12)
        xf, free = local.gather_positions(local.T(x), self.x_fixed, self.tri_idx, self.n)
        p = self.p
        return local.membrane_local(xf[:, :3], self.tri_dm_inv, self.tri_area, p["thickness"], p["mu_c"],
                                    p["lam_c"], float(p["h"]), free, hess)

    def hinges(self, x, hess=PROJECTED):
        if not len(self.hinge_idx):
            return torch.zeros(0), torch.zeros(0, 4, 3), torch.zeros(0, 12, 12)
        xh, free = local.gather_positions(local.T(x), self.x_fixed, self.hinge_idx, self.n)
        return local.hinge_local(xh, self.hinge_theta, self.hinge_stiff, float(self.p["h"]), free, hess)

    def contacts(self, x, hess=PROJECTED):
        xc, free = local.gather_positions(local.T(x), self.x_fixed, self.cidx, self.n)
        return local.contact_local(xc, torch.as_tensor(self.ctype), free,
                                   float(self.p["kappa"]), float(self.p["dhat"]), hess,
                                   self.classic, self.ee_eps)

    def mollifiers(self, x):
        """m(c) of every contact stencil (1 except for mollified edge-edge stencils)."""
        m = torch.ones(len(self.ctype))
        if self.ee_eps is None:
            return m
        xc, _ = local.gather_positions(local.T(np.asarray(x).reshape(self.n, 3)), self.x_fixed, self.cidx, self.n)
        sel = torch.nonzero(torch.as_tensor(self.ctype) == 1).flatten()
        if sel.numel():
            c = torch.vmap(en.ee_cross_norm)(xc[sel])
            m[sel] = en.ee_mollifier(c, torch.as_tensor(self.ee_eps)[sel])
        return m

    # ------------------------------------------------------------ whole problem
    def eval(self, x, hess=PROJECTED):
        x = np.asarray(x, np.float64).reshape(self.n, 3)
        e_i, g_i = self.inertia(x)
        Et, gt, Ht = self.tets(x, hess)
        Ef, gf, Hf = self.tris(x, hess)
        Eh, gh, Hh = self.hinges(x, hess)
        Ec, gc, Hc, d = self.contacts(x, hess)
        e_el = float(Et.sum()) + float(Ef.sum()) + float(Eh.sum())
        return dict(x=x, E_inertia=e_i, g_inertia=g_i, E_t=Et.numpy(), g_t=gt.numpy(),
                    H_t=Ht.numpy(), E_f=Ef.numpy(), g_f=gf.numpy(), H_f=Hf.numpy(), E_h=Eh.numpy(),
                    g_h=gh.numpy(), H_h=Hh.numpy(), E_c=Ec.numpy(), g_c=gc.numpy(), H_c=Hc.numpy(),
                    d=d.numpy(), E_elastic=e_el, E_contact=float(Ec.sum()),
                    E=e_i + e_el + float(Ec.sum()))

    def _scatter_blocks(self, nnzb, idx, pairs, slots, H):
        vals = np.zeros((nnzb, 3, 3))
        ok = slots >= 0
        s_i, q_i = np.nonzero(ok)
        a = pairs[s_i, q_i, 0]
        b = pairs[s_i, q_i, 1]
        rr = 3 * a[:, None, None] + np.arange(3)[None, :, None]
        cc = 3 * b[:, None, None] + np.arange(3)[None, None, :]
        blk = H[s_i[:, None, None], rr, cc]  # (m, 3, 3): rows of v_a, cols of v_b
        flip = idx[s_i, a] > idx[s_i, b]
        blk[flip] = blk[flip].transpose(0, 2, 1)
        np.add.at(vals, slots[s_i, q_i], blk)
        return vals

    def _scatter_grad(self, idx, g):
        out = np.zeros((self.n, 3))
        free = (idx >= 0) & (idx < self.n)
        s_i, a = np.nonzero(free)
        np.add.at(out, idx[s_i, a], g[s_i, a])
        return out

    def assemble(self, ev):
        n = self.n
        vals_s = self._scatter_blocks(len(self.ci_s), self.tet_idx, self.pairs_t, self.slot_t, ev["H_t"])
        if len(self.tri_idx):
            vals_s += self._scatter_blocks(len(self.ci_s), self.tri_idx, self.pairs_f, self.slot_f, ev["H_f"])
        if len(self.hinge_idx):
            vals_s += self._scatter_blocks(len(self.ci_s), self.hinge_idx, self.pairs_h, self.slot_h, ev["H_h"])
        vals_d = self._scatter_blocks(len(self.ci_d), self.cidx, self.pairs_c, self.slot_c, ev["H_c"])
        if not self.static:
            vals_s[self.rp_s[:-1]] += self.mass[:, None, None] * np.eye(3)[None]
        g = ev["g_inertia"] + self._scatter_grad(self.tet_idx, ev["g_t"]) + \
            self._scatter_grad(self.cidx, ev["g_c"])
        if len(self.tri_idx):
            g = g + self._scatter_grad(self.tri_idx, ev["g_f"])
        if len(self.hinge_idx):
            g = g + self._scatter_grad(self.hinge_idx, ev["g_h"])
        return dict(values_s=vals_s, values_d=vals_d, grad=g.reshape(n, 3))

    def energy_parts(self, x):
        """Energies only (line search): inertia, tets, membranes, hinges, contacts."""
        x = np.asarray(x, np.float64).reshape(self.n, 3)
        e_i, _ = self.inertia(x)
        xt, _ = local.gather_positions(local.T(x), self.x_fixed, self.tet_idx, self.n)
        h2 = float(self.p["h"]) ** 2
        Et = h2 * float(torch.vmap(en.snh_tet_energy)(xt, self.dm_inv, self.mu, self.lam, self.vol).sum()) \
            if len(self.tet_idx) else 0.0
        Ef = Eh = 0.0
        if len(self.tri_idx):
            p = self.p
            xf, _ = local.gather_positions(local.T(x), self.x_fixed, self.tri_idx, self.n)
            nf = xf.shape[0]
            Ef = h2 * float(torch.vmap(en.stvk_membrane)(
                xf[:, :3], self.tri_dm_inv, self.tri_area, torch.full((nf,), float(p["thickness"])),
                torch.full((nf,), float(p["mu_c"])), torch.full((nf,), float(p["lam_c"]))).sum())
        if len(self.hinge_idx):
            xh, _ = local.gather_positions(local.T(x), self.x_fixed, self.hinge_idx, self.n)
            Eh = h2 * float(torch.vmap(en.hinge_energy)(xh, self.hinge_theta, self.hinge_stiff).sum())
        d = self.distances(x)
        dhat, kappa = float(self.p["dhat"]), float(self.p["kappa"])
        dt = torch.as_tensor(d)
        bfun = en.barrier_ipc_classic if self.classic else en.barrier
        act = dt < dhat
        Ec = torch.where(act, bfun(torch.where(act, dt, torch.full_like(dt, dhat)), dhat, kappa),
                         torch.zeros_like(dt)) * self.mollifiers(x)
        return dict(inertia=e_i, tets=Et, membranes=Ef, hinges=Eh, contacts=float(Ec.sum()),
                    contact_terms=Ec.numpy())

    def energy(self, x):
        """Total energy only (line search)."""
        e = self.energy_parts(x)
        return e["inertia"] + e["tets"] + e["membranes"] + e["hinges"] + e["contacts"]

    def distances(self, x):
        xc, _ = local.gather_positions(local.T(np.asarray(x).reshape(self.n, 3)), self.x_fixed,
                                       self.cidx, self.n)
        d = torch.zeros(xc.shape[0])
        ct = torch.as_tensor(self.ctype)
        for t in range(4):
            sel = torch.nonzero(ct == t).flatten()
            if sel.numel():
                d[sel] = torch.vmap(en.DIST[t])(xc[sel])
        return d.numpy()

    def sides(self, x):
        xc, _ = local.gather_positions(local.T(np.asarray(x).reshape(self.n, 3)), self.x_fixed,
                                       self.cidx, self.n)
        return en.signed_side(xc, torch.as_tensor(self.ctype)).numpy()

    # ------------------------------------------------------------ matrices
    def diag_blocks(self, asm):
        """Sum of the static and dynamic diagonal blocks of every free vertex."""
        D = asm["values_s"][self.rp_s[:-1]].copy()
        rows_d = np.repeat(np.arange(self.n), np.diff(self.rp_d))
        is_diag = rows_d == self.ci_d
        D[rows_d[is_diag]] += asm["values_d"][is_diag]
        return D

    def csr(self, asm):
        """Full symmetric scalar CSR of H = H_s + H_d (both triangles)."""
        n = self.n
        mats = []
        for rp, ci, vals in ((self.rp_s, self.ci_s, asm["values_s"]),
                             (self.rp_d, self.ci_d, asm["values_d"])):
            rows = np.repeat(np.arange(n), np.diff(rp))
            bsr = sp.bsr_matrix((vals, ci, rp), shape=(3 * n, 3 * n))
            upper = bsr.tocsr()
            off = rows != ci
            bsr_off = sp.bsr_matrix((vals[off], ci[off], np.concatenate(
                [[0], np.cumsum(np.bincount(rows[off], minlength=n))])), shape=(3 * n, 3 * n))
            mats.append(upper + bsr_off.tocsr().T)
        return (mats[0] + mats[1]).tocsr()


def to_dense(rp, ci, vals, n):
    """Expand an upper BSR part to a dense symmetric 3n x 3n matrix."""
    D = np.zeros((3 * n, 3 * n))
    rows = np.repeat(np.arange(len(rp) - 1), np.diff(rp))
    for k, (r, c) in enumerate(zip(rows, ci)):
        D[3 * r:3 * r + 3, 3 * c:3 * c + 3] += vals[k]
        if r != c:
            D[3 * c:3 * c + 3, 3 * r:3 * r + 3] += vals[k].T
    return D
