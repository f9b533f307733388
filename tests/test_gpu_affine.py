"""Affine bodies mixed with free vertices: parity of the HIP path (through the
C ABI) with ``oracle.affine.AffineOracle``.

Bars as for the free-vertex scenes: bit-exact patterns and slot maps of all
three matrix parts; float64 values within 1e-10 of the summed magnitudes of
the contributions to each entry; PCG iteration counts within +-2; the Newton
step's halvings equal.
"""
import numpy as np
import pytest
import torch

from oracle import affine as oaff
from oracle import newton as onewton
from oracle import pcg as opcg
from paper_2605_23088_amd import synth

pytestmark = pytest.mark.gpu

TOL = 1e-10
CASES = ["affine", "affine_mid", "affine_classic", "affine_mollified"]
_cache = {}


def case(name):
    if name == "affine":
        return synth.affine_block()
    if name == "affine_mid":  # several SpMV chunks per part and a ragged last one
        return synth.affine_block(seed=43, nx=10, ny=9, nz=8, n_pt=500, n_ee=400, n_pp=200, n_pt1=300, n_pp2=150,
                                  n_ee2=150, n_fixed_pt=100)
    if name == "affine_classic":  # about a fifth of the stencils inactive
        return synth.affine_block(seed=44, dhi=1.25e-3)
    if name == "affine_mollified":  # near-parallel free-body edge pairs under the EE mollifier
        return synth.affine_block(seed=45, ee_angle=(0.005, 0.06))
    raise KeyError(name)


def setup(name):
    if name not in _cache:
        from paper_2605_23088_amd.yasps import IPC_CLASSIC, SQLOG, Yasps
        p = case(name)
        classic = name.endswith("classic")
        o = oaff.AffineOracle(p, classic=classic)
        g = Yasps(p, barrier=IPC_CLASSIC if classic else SQLOG)
        _cache[name] = (p, o, g)
    return _cache[name]


def xdev(p, x=None):
    return torch.as_tensor(p["X0"] if x is None else x, dtype=torch.float64, device="cuda").contiguous()


def fro(H):
    H = np.asarray(H)
    return np.broadcast_to(np.sqrt((H * H).sum(axis=(-2, -1)))[..., None, None], H.shape).copy()


def gnorm(g):
    g = np.asarray(g)
    return np.broadcast_to(np.sqrt((g * g).sum(axis=(-2, -1)))[..., None, None], g.shape).copy()


def scales(o, ev):
    """Per-entry error scales: every contribution replaced by the norm of the
    local matrix (or gradient) it came from, assembled the same way."""
    en = dict(ev)
    en["H_t"] = fro(ev["H_t"])
    en["H_c"] = fro(ev["H_c"])
    en["H_body"] = fro(ev["H_body"])
    en["H_bc"] = fro(ev["H_bc"])
    b = o.base
    h2 = float(b.p["h"]) ** 2
    dm = b.dm_inv.numpy()
    st = h2 * b.vol.numpy() * (b.mu.numpy() + b.lam.numpy()) * np.sqrt((dm * dm).sum(axis=(1, 2))) * 4.0
    en["g_t"] = np.maximum(gnorm(ev["g_t"]), st[:, None, None])
    en["g_c"] = gnorm(ev["g_c"])
    en["g_inertia"] = np.abs(ev["g_inertia"])
    en["g_body"] = gnorm(ev["g_body"]) + np.abs(ev["g_body"]).max()
    en["g_bc"] = gnorm(ev["g_bc"])
    return o.assemble(en)


def within(gpu, ref, scale, tol=TOL):
    err = np.abs(np.asarray(gpu) - np.asarray(ref))
    bad = err > tol * np.asarray(scale) + 1e-300
    assert not bad.any(), f"{bad.sum()} entries off; worst {err.max():.3e} (scale {np.max(scale):.3e})"


def test_case_covers_every_mix():
    """Free-body and body-body stencils of every type, and both movable counts."""
    p = case("affine")
    n, nfix = p["n_free"], p["x_fixed"].shape[0]
    kinds = set()
    for t, ids in zip(p["bctype"], p["bcidx"]):
        body = tuple(int(v >= n + nfix) for v in ids if v >= 0)
        kinds.add((int(t), sum(body), len(body) - sum(body)))
    assert {(0, 1, 3), (1, 2, 2), (3, 1, 1), (3, 2, 0), (1, 4, 0)} <= kinds, kinds


@pytest.mark.parametrize("name", CASES)
def test_patterns_bit_exact(name):
    p, o, g = setup(name)
    rp, ci, sl = g.pattern(0)
    assert np.array_equal(rp, o.rp_s) and np.array_equal(ci, o.ci_s)
    assert np.array_equal(sl, np.concatenate([o.slot_t, o.slot_bd]))
    rp, ci, sl = g.pattern(1)
    assert np.array_equal(rp, o.rp_d) and np.array_equal(ci, o.ci_d) and np.array_equal(sl, o.slot_c)
    rp, ci, sl = g.pattern(2)
    assert np.array_equal(rp, o.rp_b) and np.array_equal(ci, o.ci_b) and np.array_equal(sl, o.slot_b)


@pytest.mark.parametrize("name", CASES)
@pytest.mark.parametrize("exact", [False, True])
def test_eval_and_assembly_parity(name, exact):
    p, o, g = setup(name)
    hess = oaff.local.EXACT if exact else oaff.local.PROJECTED
    ev = o.eval(p["X0"], hess)
    asm = o.assemble(ev)
    sc = scales(o, ev)
    info = g.eval(xdev(p), exact=exact)
    mag = (np.abs(ev["E_t"]).sum() + np.abs(ev["E_c"]).sum() + np.abs(ev["E_bc"]).sum() + abs(ev["E_inertia"])
           + np.abs(ev["E_orth"]).sum() + np.abs(ev["E_body_inertia"]).sum())
    assert abs(info["energy"] - ev["E"]) <= TOL * mag
    assert abs(info["e_contact"] - ev["E_contact"]) <= TOL * (np.abs(ev["E_c"]).sum() + np.abs(ev["E_bc"]).sum())
    d = np.concatenate([ev["d"], ev["d_bc"]])
    assert info["min_d"] == pytest.approx(d.min(), rel=1e-12)
    assert info["n_active"] == int((d < p["dhat"]).sum())
    out = g.assemble()
    within(out["values_s"].cpu().numpy(), asm["values_s"], sc["values_s"])
    within(out["values_d"].cpu().numpy(), asm["values_d"], sc["values_d"])
    within(out["values_b"].cpu().numpy(), asm["values_b"], sc["values_b"])
    within(out["grad"].cpu().numpy(), asm["grad"], sc["grad"])
    D = o.diag_blocks(asm)
    Minv = opcg.block_inverse(D)
    bi = out["block_inv"].cpu().numpy()
    cond = np.linalg.cond(D)
    assert np.all(np.abs(bi - Minv) <= 1e-12 * cond[:, None, None] * np.abs(Minv).max(axis=(1, 2))[:, None, None])


@pytest.mark.parametrize("name", CASES)
def test_pcg_parity(name):
    p, o, g = setup(name)
    ev = o.eval(p["X0"])
    asm = o.assemble(ev)
    H = o.csr(asm)
    Minv = opcg.block_inverse(o.diag_blocks(asm))
    b = -asm["grad"].ravel()
    x_o, it_o, rel_o, st_o = opcg.pcg(lambda v: H @ v, b, Minv, 1e-8, 20000)
    g.eval(xdev(p))
    g.assemble(copy=False)
    bd = torch.as_tensor(b, device="cuda").view(-1, 3).contiguous()
    # the three-part SpMV against the oracle's matrix
    u = np.random.default_rng(7).normal(size=b.shape)
    y = g.spmv(torch.as_tensor(u, device="cuda").view(-1, 3).contiguous()).cpu().numpy().ravel()
    Hu = H @ u
    absH = abs(H)
    within(y, Hu, absH @ np.abs(u), tol=1e-12)
    x, info = g.pcg(bd, rtol=1e-8)
    assert info["status"] == 0 and st_o == "ok"
    assert abs(info["iters"] - it_o) <= 2, (info["iters"], it_o)
    r = np.linalg.norm(H @ x.cpu().numpy().ravel() - b) / np.linalg.norm(b)
    assert r <= 1e-8 * 1.05, r


@pytest.mark.parametrize("name", CASES)
def test_newton_step_parity(name):
    p, o, g = setup(name)
    x1_o, info_o = onewton.newton_step(o, p["X0"], rtol=1e-10)
    x = xdev(p)
    info = g.newton_step(x, rtol=1e-10)
    assert info["status"] == 0
    a0 = onewton.initial_step(o, p["X0"], info_o["p"])
    assert info["alpha0"] == pytest.approx(a0, rel=1e-8)
    assert round(np.log2(info["alpha0"] / info["alpha"])) == round(np.log2(a0 / info_o["alpha"]))
    mag = abs(info_o["E0"]) + 1e-300
    assert abs(info["e0"] - info_o["E0"]) <= 1e-10 * mag
    assert abs(info["e1"] - info_o["E1"]) <= 1e-8 * mag
    assert np.abs(x.cpu().numpy() - x1_o).max() <= 1e-7 * np.abs(info_o["p"]).max() + 1e-15


def test_body_contact_errors_and_reset():
    """Rejected sets leave no body contacts; a smaller set reuses the buffers
    and still matches the oracle."""
    from paper_2605_23088_amd.yasps import E_ARG, YaspsError
    p, o, g = setup("affine")
    n, nfix = p["n_free"], p["x_fixed"].shape[0]
    base = n + nfix
    b0 = int(np.flatnonzero(p["abd_body"] == 0)[0]) + base
    b1 = int(np.flatnonzero(p["abd_body"] == 1)[0]) + base
    # 4 + 4 + 1 + 1 = 10 rows
    bad_t = np.array([1], np.int32)
    bad_i = np.array([[b0, b1, 0, 1]], np.int32)
    with pytest.raises(YaspsError) as e:
        g.set_body_contacts(bad_t, bad_i)
    assert e.value.status == E_ARG and "8 rows" in str(e.value)
    # no movable vertex
    with pytest.raises(YaspsError) as e:
        g.set_body_contacts(np.array([3], np.int32), np.array([[n, n + 1, -1, -1]], np.int32))
    assert e.value.status == E_ARG
    # the context holds no body contacts now: energy = the free-vertex part + body terms
    q = dict(p)
    q["bctype"] = p["bctype"][:0]
    q["bcidx"] = p["bcidx"][:0]
    o0 = oaff.AffineOracle(q)
    info = g.eval(xdev(p))
    assert info["energy"] == pytest.approx(o0.eval(p["X0"])["E"], rel=1e-12)
    # a smaller set (every other stencil)
    q["bctype"] = p["bctype"][::2]
    q["bcidx"] = p["bcidx"][::2]
    g.set_body_contacts(q["bctype"], q["bcidx"])
    o2 = oaff.AffineOracle(q)
    ev = o2.eval(p["X0"])
    asm = o2.assemble(ev)
    sc = scales(o2, ev)
    g.eval(xdev(p))
    out = g.assemble()
    rp, ci, sl = g.pattern(2)
    assert np.array_equal(rp, o2.rp_b) and np.array_equal(ci, o2.ci_b) and np.array_equal(sl, o2.slot_b)
    within(out["values_b"].cpu().numpy(), asm["values_b"], sc["values_b"])
    within(out["grad"].cpu().numpy(), asm["grad"], sc["grad"])
    g.set_body_contacts(p["bctype"], p["bcidx"])  # restore


def test_lm_shift_with_bodies():
    """The damping scale takes the free vertices' rows only (bodies have no
    lumped mass), with the body-contact part's diagonal blocks included."""
    p, o, g = setup("affine")
    ev = o.eval(p["X0"])
    asm = o.assemble(ev)
    g.eval(xdev(p))
    g.assemble(copy=False)
    D = o.diag_blocks(asm)[:p["n_free"]]
    tr = np.abs(np.trace(D, axis1=1, axis2=2)) / (3.0 * np.asarray(p["mass"]))
    assert g.lm_shift(1e-2) == pytest.approx(1e-2 * np.median(tr), rel=1e-12)
