"""Shared helpers of the GPU parity tests: per-entry rounding scales derived
from the oracle's local contributions, the elementwise bar, and the
restriction of a large scene to the stencils around sampled vertices (so the
oracle can check full-size GPU results row by row)."""
import numpy as np
import scipy.sparse as sp
import torch

from oracle import energy as en
from oracle import local as olocal

TOL = 1e-10


def scales(o, ev, x):
    """Per-entry rounding scales: contributing local-Hessian Frobenius norms;
    for gradients the contributing gradient norms, floored for elastic terms
    by their stress scale (tets, membranes) or k |grad theta| (hinges), the
    size of the terms that cancel near rest.  Returns (static values, dynamic
    values, gradient, elastic-energy scale)."""
    def fro(H):
        return np.broadcast_to(np.sqrt((H * H).sum(axis=(1, 2)))[:, None, None], H.shape)

    def gn(g, floor=None):
        s = np.sqrt((g * g).sum(axis=(1, 2)))
        if floor is not None:
            s = np.maximum(s, floor)
        return np.broadcast_to(s[:, None, None], g.shape)

    p = o.p
    h2 = float(p["h"]) ** 2
    nnz = len(o.ci_s)
    vs = o._scatter_blocks(nnz, o.tet_idx, o.pairs_t, o.slot_t, fro(ev["H_t"]))
    dm = o.dm_inv.numpy()
    st_t = h2 * o.vol.numpy() * (o.mu.numpy() + o.lam.numpy()) * np.sqrt((dm * dm).sum(axis=(1, 2))) * 4.0
    g = np.abs(ev["g_inertia"]) + o._scatter_grad(o.tet_idx, gn(ev["g_t"], st_t))
    e = st_t.sum()
    if len(o.tri_idx):
        vs += o._scatter_blocks(nnz, o.tri_idx, o.pairs_f, o.slot_f, fro(ev["H_f"]))
        d2 = o.tri_dm_inv.numpy()
        st_f = (h2 * o.tri_area.numpy() * p["thickness"] * (p["mu_c"] + p["lam_c"]) *
                np.sqrt((d2 * d2).sum(axis=(1, 2))) * 4.0)
        g += o._scatter_grad(o.tri_idx, gn(ev["g_f"], st_f))
        e += st_f.sum() + np.abs(ev["E_f"]).sum()
    if len(o.hinge_idx):
        vs += o._scatter_blocks(nnz, o.hinge_idx, o.pairs_h, o.slot_h, fro(ev["H_h"]))
        xh, _ = olocal.gather_positions(torch.as_tensor(np.asarray(x)), o.x_fixed, o.hinge_idx, o.n)
        gth = torch.vmap(torch.func.grad(en.hinge_angle))(xh).numpy()
        st_h = h2 * o.hinge_stiff.numpy() * np.sqrt((gth * gth).sum(axis=(1, 2))) * 4.0
        g += o._scatter_grad(o.hinge_idx, gn(ev["g_h"], st_h))
        e += st_h.sum() + np.abs(ev["E_h"]).sum()
    if not o.static:
        vs[o.rp_s[:-1]] += np.abs(o.mass)[:, None, None] * np.eye(3)[None]
    vd = o._scatter_blocks(len(o.ci_d), o.cidx, o.pairs_c, o.slot_c, fro(ev["H_c"]))
    g += o._scatter_grad(o.cidx, gn(ev["g_c"]))
    return vs, vd, g, e


def within(gpu, ref, scale, tol=TOL):
    err = np.abs(np.asarray(gpu) - np.asarray(ref))
    bad = err > tol * np.asarray(scale) + 1e-300
    assert not bad.any(), f"{bad.sum()} entries off; worst {err.max():.3e} (scale {np.max(scale):.3e})"


def restrict(p, verts):
    """The scene with only the stencils that touch a vertex of `verts` (same
    vertices and ids): its oracle gives complete gradient rows and BSR rows
    for those vertices."""
    verts = np.asarray(verts)
    mark = np.zeros(p["n_free"] + len(p["x_fixed"]) + 1, bool)
    mark[verts] = True

    def touching(idx):
        idx = np.asarray(idx)
        return mark[np.where(idx >= 0, idx, -1)].any(axis=1) if len(idx) else np.zeros(0, bool)

    q = dict(p)
    k = touching(p["tet_idx"])
    q["tet_idx"], q["dm_inv"], q["vol"] = p["tet_idx"][k], p["dm_inv"][k], p["vol"][k]
    for key in ("mu_t", "lam_t"):
        if key in p:
            q[key] = p[key][k]
    k = touching(p["cidx"])
    q["ctype"], q["cidx"] = p["ctype"][k], p["cidx"][k]
    if len(p.get("tri_idx", [])):
        k = touching(p["tri_idx"])
        q["tri_idx"], q["tri_dm_inv"], q["tri_area"] = p["tri_idx"][k], p["tri_dm_inv"][k], p["tri_area"][k]
    if len(p.get("hinge_idx", [])):
        k = touching(p["hinge_idx"])
        q["hinge_idx"], q["hinge_rest"] = p["hinge_idx"][k], p["hinge_rest"][k]
    return q


def bsr_rows(rp, ci, vals, rows):
    """{row: (cols, blocks)} of an upper BSR part."""
    return {int(r): (ci[rp[r]:rp[r + 1]], vals[rp[r]:rp[r + 1]]) for r in rows}


def gpu_csr(g, out):
    """The GPU's assembled matrix (both parts, both triangles) as SciPy CSR in
    float64 (float32 values convert exactly): each upper part B contributes
    B + (off-diagonal blocks of B)^T."""
    H = None
    for part, key in ((0, "values_s"), (1, "values_d")):
        rp, ci, _ = g.pattern(part)
        if len(ci) == 0:
            continue
        vals = out[key].cpu().numpy().astype(np.float64)
        off = (ci != np.repeat(np.arange(g.n), np.diff(rp)))[:, None, None]
        shape = (3 * g.n, 3 * g.n)
        M = sp.bsr_matrix((vals, ci, rp), shape=shape).tocsr() + sp.bsr_matrix((vals * off, ci, rp), shape=shape).T
        H = M if H is None else H + M
    return H.tocsr()
