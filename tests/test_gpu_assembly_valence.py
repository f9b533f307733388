"""Assembly of slots with very different numbers of contributions: a star of
300 tets around one vertex (its diagonal block and gradient row sum 301
contributions, every other slot one or two), so the LDS-staged block sums take
several rounds for the workgroup that holds the star's centre, next to
workgroups of single-contribution slots.  Values, gradient and block inverses
against the oracle (exact and projected Hessians), and the PCG solution."""
import numpy as np
import pytest
import torch

from oracle import assemble as oasm
from oracle import pcg as opcg
from paper_2605_23088_amd import synth
from test_gpu_parity import abs_sums, tet_stress_scale, within

pytestmark = pytest.mark.gpu


def star_problem(m=300, seed=5):
    """Vertex 0 at the origin; tet i = (0, a_i, b_i, c_i) with three private
    vertices at radius ~0.1, positively oriented; rest shape = the drawn
    positions, x0 = rest + N(0, 1e-3)."""
    rng = np.random.default_rng(seed)
    base = synth.small_block(seed=11, nx=3, ny=3, nz=3, n_pt=20, n_ee=20)
    n = 1 + 3 * m
    X = np.zeros((n, 3))
    tets = np.zeros((m, 4), np.int64)
    for i in range(m):
        while True:
            P = rng.standard_normal((3, 3))
            P = 0.1 * P / np.linalg.norm(P, axis=1, keepdims=True)
            if np.linalg.det(P) > 2e-4:  # positive orientation, not degenerate
                break
        X[1 + 3 * i:4 + 3 * i] = P
        tets[i] = [0, 1 + 3 * i, 2 + 3 * i, 3 + 3 * i]
    Ds = np.stack([X[tets[:, k]] - X[tets[:, 0]] for k in (1, 2, 3)], axis=2)  # columns
    dm_inv = np.linalg.inv(Ds)
    vol = np.abs(np.linalg.det(Ds)) / 6.0
    mass = np.full(n, 1e-3)
    x0 = X + 1e-3 * rng.standard_normal(X.shape)
    h2g = base["h"] ** 2 * np.asarray(base["gravity"])
    p = dict(base)
    p.update(n_free=n, x0=np.ascontiguousarray(x0), x_tilde=np.ascontiguousarray(X + h2g), mass=mass,
             x_fixed=np.zeros((0, 3)), tet_idx=tets.astype(np.int32), dm_inv=np.ascontiguousarray(dm_inv),
             vol=np.ascontiguousarray(vol), ctype=np.zeros(0, np.int32), cidx=np.zeros((0, 4), np.int32),
             name="star")
    for k in ("grid", "spacing"):
        p.pop(k, None)
    return p


@pytest.fixture(scope="module")
def star():
    from paper_2605_23088_amd.yasps import Yasps
    p = star_problem()
    return p, oasm.Oracle(p), Yasps(p)


@pytest.mark.parametrize("exact", [False, True])
def test_high_valence_assembly(star, exact):
    p, o, g = star
    ev = o.eval(p["x0"], oasm.EXACT if exact else oasm.PROJECTED)
    asm = o.assemble(ev)
    g.eval(torch.as_tensor(p["x0"], device="cuda").contiguous(), exact=exact)
    out = g.assemble()
    assert int(o.rp_s[1] - o.rp_s[0]) == 1 + 3 * 300  # the centre's row: its diagonal and 900 neighbours
    vs, _, gs = abs_sums(o, ev)
    within(out["values_s"].cpu().numpy(), asm["values_s"], vs)
    within(out["grad"].cpu().numpy(), asm["grad"], gs)
    D = o.diag_blocks(asm)
    Minv = opcg.block_inverse(D)
    bi = out["block_inv"].cpu().numpy()
    cond = np.linalg.cond(D)
    assert np.all(np.abs(bi - Minv) <= 1e-12 * cond[:, None, None] * np.abs(Minv).max(axis=(1, 2))[:, None, None])
    assert tet_stress_scale(o).shape == (300,)


def test_high_valence_pcg(star):
    p, o, g = star
    ev = o.eval(p["x0"])
    asm = o.assemble(ev)
    H = o.csr(asm)
    g.eval(torch.as_tensor(p["x0"], device="cuda").contiguous())
    g.assemble(copy=False)
    b = -asm["grad"].ravel()
    x, info = g.pcg(torch.as_tensor(b, device="cuda").view(-1, 3).contiguous(), rtol=1e-10)
    assert info["status"] == 0
    r = np.linalg.norm(H @ x.cpu().numpy().ravel() - b) / np.linalg.norm(b)
    assert r <= 1e-9, r
