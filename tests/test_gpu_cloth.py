"""Cloth (StVK membranes + dihedral hinges) on the HIP path against the oracle:
bit-exact pattern with triangles and hinges in the static part, eval /
assembly parity (projected and exact), PCG and Newton-step parity, and the
same with fixed cloth vertices (hinges with 1..3 free vertices, membranes
with fixed corners).  Bars as in the volumetric parity tests."""
import numpy as np
import pytest
import torch

from oracle import assemble as oasm
from oracle import energy as en
from oracle import local as olocal
from oracle import newton as onewton
from oracle import pcg as opcg
from paper_2605_23088_amd import synth

pytestmark = pytest.mark.gpu
TOL = 1e-10


def with_fixed(p, fixed):
    """The same scene with the vertices `fixed` turned into fixed vertices
    (ids relabelled: remaining free vertices first, then the fixed ones);
    stencils left without a free vertex are dropped."""
    n = p["n_free"]
    fixed = np.unique(fixed)
    keep = np.setdiff1d(np.arange(n), fixed)
    new = np.empty(n, np.int64)
    new[keep] = np.arange(len(keep))
    new[fixed] = len(keep) + np.arange(len(fixed))

    def remap(idx):
        idx = np.asarray(idx, np.int64)
        return np.where(idx >= 0, new[np.maximum(idx, 0)], -1)

    def has_free(idx):
        return ((idx >= 0) & (idx < len(keep))).any(axis=1)

    q = dict(p)
    q["n_free"] = len(keep)
    q["x0"] = p["x0"][keep]
    q["x_fixed"] = p["x0"][fixed]
    q["mass"] = p["mass"][keep]
    q["x_tilde"] = p["x_tilde"][keep]
    q["tet_idx"] = remap(p["tet_idx"]).astype(np.int32)
    q["tri_idx"] = remap(p["tri_idx"]).astype(np.int32)
    hidx = remap(p["hinge_idx"])
    hk = has_free(hidx)
    q["hinge_idx"] = hidx[hk].astype(np.int32)
    q["hinge_rest"] = p["hinge_rest"][hk]
    cidx = remap(p["cidx"])
    ck = has_free(cidx)
    q["cidx"] = cidx[ck].astype(np.int32)
    q["ctype"] = p["ctype"][ck]
    return q


def case(name):
    p = synth.small_cloth()
    if name == "cloth":
        return p
    if name == "cloth_fixed":
        rng = np.random.default_rng(8)
        cloth_v = np.unique(p["tri_idx"])
        return with_fixed(p, rng.choice(cloth_v, 60, replace=False))
    raise KeyError(name)


CASES = ["cloth", "cloth_fixed"]
_cache = {}


def setup(name):
    if name not in _cache:
        from paper_2605_23088_amd.yasps import Yasps
        p = case(name)
        rng = np.random.default_rng(5)
        # perturb positions so that no stencil sits exactly at rest
        x = p["x0"] + 2e-5 * rng.standard_normal(p["x0"].shape)
        o = oasm.Oracle(p)
        assert (o.distances(x) > 0).all()
        _cache[name] = (p, o, Yasps(p), x)
    return _cache[name]


def xdev(x):
    return torch.as_tensor(x, dtype=torch.float64, device="cuda").contiguous()


def scales(o, ev, x):
    """Per-entry rounding scales: contributing local-Hessian Frobenius norms;
    for gradients the contributing gradient norms, floored for elastic terms
    by their stress scale (tets, membranes) or k |grad theta| (hinges), the
    size of the terms that cancel near rest."""
    def fro(H):
        return np.broadcast_to(np.sqrt((H * H).sum(axis=(1, 2)))[:, None, None], H.shape)

    def gn(g, floor=None):
        s = np.sqrt((g * g).sum(axis=(1, 2)))
        if floor is not None:
            s = np.maximum(s, floor)
        return np.broadcast_to(s[:, None, None], g.shape)

    nnz = len(o.ci_s)
    vs = (o._scatter_blocks(nnz, o.tet_idx, o.pairs_t, o.slot_t, fro(ev["H_t"])) +
          o._scatter_blocks(nnz, o.tri_idx, o.pairs_f, o.slot_f, fro(ev["H_f"])) +
          o._scatter_blocks(nnz, o.hinge_idx, o.pairs_h, o.slot_h, fro(ev["H_h"])))
    vd = o._scatter_blocks(len(o.ci_d), o.cidx, o.pairs_c, o.slot_c, fro(ev["H_c"]))
    vs[o.rp_s[:-1]] += np.abs(o.mass)[:, None, None] * np.eye(3)[None]
    p = o.p
    h2 = float(p["h"]) ** 2
    dm = o.dm_inv.numpy()
    st_t = h2 * o.vol.numpy() * (o.mu.numpy() + o.lam.numpy()) * np.sqrt((dm * dm).sum(axis=(1, 2))) * 4.0
    d2 = o.tri_dm_inv.numpy()
    st_f = h2 * o.tri_area.numpy() * p["thickness"] * (p["mu_c"] + p["lam_c"]) * np.sqrt((d2 * d2).sum(axis=(1, 2))) * 4
    xh, _ = olocal.gather_positions(torch.as_tensor(x), o.x_fixed, o.hinge_idx, o.n)
    gth = torch.vmap(torch.func.grad(en.hinge_angle))(xh).numpy()
    st_h = h2 * o.hinge_stiff.numpy() * np.sqrt((gth * gth).sum(axis=(1, 2))) * 4.0
    g = (np.abs(ev["g_inertia"]) + o._scatter_grad(o.tet_idx, gn(ev["g_t"], st_t)) +
         o._scatter_grad(o.tri_idx, gn(ev["g_f"], st_f)) + o._scatter_grad(o.hinge_idx, gn(ev["g_h"], st_h)) +
         o._scatter_grad(o.cidx, gn(ev["g_c"])))
    e = st_t.sum() + st_f.sum() + np.abs(ev["E_h"]).sum() + st_h.sum() + np.abs(ev["E_f"]).sum()
    return vs, vd, g, e


def within(gpu, ref, scale, tol=TOL):
    err = np.abs(np.asarray(gpu) - np.asarray(ref))
    bad = err > tol * np.asarray(scale) + 1e-300
    assert not bad.any(), f"{bad.sum()} entries off; worst {err.max():.3e} (scale {np.max(scale):.3e})"


@pytest.mark.parametrize("name", CASES)
def test_cloth_pattern_bit_exact(name):
    p, o, g, x = setup(name)
    rp, ci, sl = g.pattern(0)
    assert np.array_equal(rp, o.rp_s) and np.array_equal(ci, o.ci_s)
    assert np.array_equal(sl, np.concatenate([o.slot_t, o.slot_f, o.slot_h]))
    rp, ci, sl = g.pattern(1)
    assert np.array_equal(rp, o.rp_d) and np.array_equal(ci, o.ci_d) and np.array_equal(sl, o.slot_c)


@pytest.mark.parametrize("name", CASES)
@pytest.mark.parametrize("exact", [False, True])
def test_cloth_eval_and_assembly_parity(name, exact):
    p, o, g, x = setup(name)
    ev = o.eval(x, oasm.EXACT if exact else oasm.PROJECTED)
    asm = o.assemble(ev)
    info = g.eval(xdev(x), exact=exact)
    vs, vd, gs, e_el = scales(o, ev, x)
    assert abs(info["e_elastic"] - ev["E_elastic"]) <= TOL * e_el
    assert abs(info["e_contact"] - ev["E_contact"]) <= TOL * np.abs(ev["E_c"]).sum()
    out = g.assemble()
    within(out["values_s"].cpu().numpy(), asm["values_s"], vs)
    within(out["values_d"].cpu().numpy(), asm["values_d"], vd)
    within(out["grad"].cpu().numpy(), asm["grad"], gs)
    d = out["values_s"].cpu().numpy()[o.rp_s[:-1]]
    assert np.array_equal(d, d.transpose(0, 2, 1))


@pytest.mark.parametrize("name", CASES)
def test_cloth_pcg_and_newton_parity(name):
    p, o, g, x = setup(name)
    ev = o.eval(x)
    asm = o.assemble(ev)
    H = o.csr(asm)
    Minv = opcg.block_inverse(o.diag_blocks(asm))
    b = -asm["grad"].ravel()
    x_o, it_o, _, st_o = opcg.pcg(lambda v: H @ v, b, Minv, 1e-8, 20000)
    g.eval(xdev(x))
    g.assemble(copy=False)
    xs, info = g.pcg(torch.as_tensor(b, device="cuda").view(-1, 3).contiguous(), rtol=1e-8)
    assert info["status"] == 0 and st_o == "ok"
    assert abs(info["iters"] - it_o) <= 2, (info["iters"], it_o)
    r = np.linalg.norm(H @ xs.cpu().numpy().ravel() - b) / np.linalg.norm(b)
    assert r <= 1e-8 * 1.05
    # one Newton step
    x1_o, info_o = onewton.newton_step(o, x, rtol=1e-10)
    xd = xdev(x)
    ni = g.newton_step(xd, rtol=1e-10)
    a0 = onewton.initial_step(o, x, info_o["p"])
    assert ni["status"] == 0 and ni["alpha0"] == pytest.approx(a0, rel=1e-8)
    assert round(np.log2(ni["alpha0"] / ni["alpha"])) == round(np.log2(a0 / info_o["alpha"]))
    assert abs(ni["e0"] - info_o["E0"]) <= 1e-10 * abs(info_o["E0"])
    assert abs(ni["e1"] - info_o["E1"]) <= 1e-8 * abs(info_o["E0"])
    assert np.abs(xd.cpu().numpy() - x1_o).max() <= 1e-7 * np.abs(info_o["p"]).max()


def test_cloth_hinge_groups_cover_every_free_count():
    p, o, g, x = setup("cloth_fixed")
    nfree = ((o.hinge_idx >= 0) & (o.hinge_idx < o.n)).sum(axis=1)
    assert set(np.unique(nfree).tolist()) == {1, 2, 3, 4}
