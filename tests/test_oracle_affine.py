"""Pins of the oracle's affine-body scenes (CPU): positions p = A r + t, the
body inertia against its per-vertex definition, the orthogonality energy's
closed-form gradient and invariances, the chain rule through the union of
free / fixed / body vertices against autodiff of the composed function,
finite differences of the whole scene, the reduced-coordinate projection,
the pattern rule, and a Newton step."""
import numpy as np
import pytest
import torch

from oracle import affine
from oracle import local
from oracle import newton as onewton
from oracle import pattern
from paper_2605_23088_amd import synth


@pytest.fixture(scope="module")
def scene():
    p = synth.affine_block(seed=5, nx=3, ny=3, nz=2, n_pt=30, n_ee=30, n_pp=12, n_pt1=16, n_pp2=10,
                           n_ee2=10, n_fixed_pt=8)
    return p, affine.AffineOracle(p)


def test_body_positions_are_affine():
    rng = np.random.default_rng(1)
    A = rng.normal(size=(3, 3))
    t = rng.normal(size=3)
    r = rng.normal(size=3)
    q = torch.as_tensor(np.concatenate([A.T, t[None]], 0))
    assert np.allclose(affine.body_positions(q, torch.as_tensor(r)).numpy(), A @ r + t, rtol=0, atol=1e-14)


def test_body_inertia_equals_per_vertex_sum():
    """1/2 (q - q~)^T (M4 (x) I3) (q - q~) with M4 = sum m w w^T equals
    1/2 sum_v m_v |p_v(q) - p_v(q~)|^2."""
    rng = np.random.default_rng(2)
    r = rng.normal(size=(7, 3))
    m = rng.uniform(0.5, 2.0, 7)
    w = np.concatenate([r, np.ones((7, 1))], 1)
    M4 = (m[:, None, None] * w[:, :, None] * w[:, None, :]).sum(0)
    q = rng.normal(size=(4, 3))
    qt = rng.normal(size=(4, 3))
    pq = r @ q[:3] + q[3]
    pt = r @ qt[:3] + qt[3]
    ref = 0.5 * np.sum(m * ((pq - pt) ** 2).sum(1))
    got = float(affine.body_inertia(torch.as_tensor(q), torch.as_tensor(qt), torch.as_tensor(M4)))
    assert got == pytest.approx(ref, rel=1e-13)


def test_orthogonality_closed_form_and_invariance():
    rng = np.random.default_rng(3)
    A = np.eye(3) + 0.2 * rng.normal(size=(3, 3))
    q = torch.as_tensor(np.concatenate([A.T, rng.normal(size=(1, 3))], 0))
    G = A.T @ A - np.eye(3)
    assert float(affine.orthogonality(q)) == pytest.approx(0.5 * np.sum(G * G), rel=1e-13)
    # d/dA 1/2 |A^T A - I|^2 = 2 A (A^T A - I); rows of q are the columns of A
    g = torch.func.grad(affine.orthogonality)(q).numpy()
    gA = 2.0 * A @ G
    assert np.allclose(g[:3], gA.T, rtol=1e-12, atol=1e-13) and np.all(g[3] == 0.0)
    # zero with zero gradient on rotations, invariant under A -> R A
    Q, _ = np.linalg.qr(rng.normal(size=(3, 3)))
    R = Q * np.sign(np.linalg.det(Q))
    qr = torch.as_tensor(np.concatenate([R.T, np.zeros((1, 3))], 0))
    assert abs(float(affine.orthogonality(qr))) <= 1e-28
    assert np.abs(torch.func.grad(affine.orthogonality)(qr).numpy()).max() <= 1e-14
    qR = torch.as_tensor(np.concatenate([(R @ A).T, np.zeros((1, 3))], 0))
    assert float(affine.orthogonality(qR)) == pytest.approx(float(affine.orthogonality(q)), rel=1e-12)


def test_row_lists_and_pattern(scene):
    p, o = scene
    s = o.scene
    n, nfix = p["n_free"], p["x_fixed"].shape[0]
    base = n + nfix
    for st in range(s.cidx.shape[0]):
        want = []
        for v in s.cidx[st]:
            if v < 0 or n <= v < base:
                continue
            rows = [int(v)] if v < n else [n + 4 * int(p["abd_body"][v - base]) + j for j in range(4)]
            want += [r for r in rows if r not in want]
        got = s.rows[st][s.rows[st] >= 0].tolist()
        assert got == want
    # set-based brute force of the body-contact pattern and slot map
    keys = set()
    for st in range(s.rows.shape[0]):
        lst = s.rows[st][s.rows[st] >= 0]
        for a in range(len(lst)):
            for b in range(a, len(lst)):
                keys.add((min(lst[a], lst[b]), max(lst[a], lst[b])))
    keys = sorted(keys)
    assert len(keys) == len(s.ci_b)
    rows = np.repeat(np.arange(o.n), np.diff(s.rp_b))
    assert list(zip(rows.tolist(), s.ci_b.tolist())) == keys
    pos = {k: i for i, k in enumerate(keys)}
    for st in range(s.rows.shape[0]):
        lst = s.rows[st][s.rows[st] >= 0]
        q = 0
        for a in range(len(lst)):
            for b in range(a, len(lst)):
                assert s.slot_b[st, q] == pos[(min(lst[a], lst[b]), max(lst[a], lst[b]))]
                q += 1
        assert np.all(s.slot_b[st, q:] == -1)
    # the static part holds every diagonal and each body's 10 blocks
    assert len(o.rp_s) == o.n + 1
    for b in range(p["n_bodies"]):
        r0 = n + 4 * b
        for i in range(4):
            cols = o.ci_s[o.rp_s[r0 + i]:o.rp_s[r0 + i + 1]]
            assert set(range(r0 + i, r0 + 4)) <= set(cols.tolist())


def test_chain_rule_through_the_union(scene):
    """The row-list gradient and (exact) Hessian of every body contact equal
    autodiff of the barrier as a function of the stencil's degree-of-freedom
    rows (positions formed inside the differentiated function)."""
    p, o = scene
    s = o.scene
    X = torch.as_tensor(p["X0"])
    E, g, H, d = s.contact_terms(X, local.EXACT)
    n, nfix = p["n_free"], p["x_fixed"].shape[0]
    base = n + nfix
    kappa, dhat = float(p["kappa"]), float(p["dhat"])
    for st in np.random.default_rng(0).choice(s.cidx.shape[0], 25, replace=False):
        lst = s.rows[st][s.rows[st] >= 0]
        ids = s.cidx[st]

        def f(Y, ids=ids, lst=lst):
            Xl = X.clone()
            Xl = Xl.index_put((torch.as_tensor(lst),), Y)
            xs = []
            for v in ids:
                if v < 0:
                    xs.append(torch.zeros(3))
                elif v < n:
                    xs.append(Xl[v])
                elif v < base:
                    xs.append(torch.as_tensor(p["x_fixed"][v - n]))
                else:
                    b = int(p["abd_body"][v - base])
                    xs.append(affine.body_positions(Xl[n + 4 * b:n + 4 * b + 4], torch.as_tensor(p["abd_rest"][v - base])))
            x4 = torch.stack(xs)
            dd = affine.en.DIST[int(s.ctype[st])](x4)
            return affine.en.barrier(dd, dhat, kappa)

        Y = X[torch.as_tensor(lst)]
        gr = torch.func.grad(f)(Y).numpy()
        Hr = torch.func.hessian(f)(Y).reshape(3 * len(lst), 3 * len(lst)).numpy()
        L = len(lst)
        assert np.allclose(g[st, :L].numpy(), gr, rtol=1e-10, atol=1e-12 * np.abs(gr).max())
        assert np.allclose(H[st, :3 * L, :3 * L].numpy(), Hr, rtol=1e-9, atol=1e-11 * np.abs(Hr).max())


def test_scene_finite_differences(scene):
    """Central differences of the whole scene's energy along random directions
    give g . v, and of the gradient give H v (exact Hessian)."""
    p, o = scene
    X = p["X0"]
    ev = o.eval(X, local.EXACT)
    asm = o.assemble(ev)
    H = o.csr(asm)
    g = asm["grad"].ravel()
    rng = np.random.default_rng(4)
    for _ in range(3):
        v = rng.normal(size=X.shape)
        v /= np.abs(v).max()
        eps = 1e-6
        fd = (o.energy(X + eps * v) - o.energy(X - eps * v)) / (2 * eps)
        assert fd == pytest.approx(g @ v.ravel(), rel=1e-5)
        gp = o.assemble(o.eval(X + eps * v, local.EXACT))["grad"].ravel()
        gm = o.assemble(o.eval(X - eps * v, local.EXACT))["grad"].ravel()
        fdh = (gp - gm) / (2 * eps)
        Hv = H @ v.ravel()
        assert np.linalg.norm(fdh - Hv) <= 1e-5 * np.linalg.norm(Hv)


def test_reduced_projection(scene):
    """J^T Proj(H_p) J: positive semidefinite, equal to the exact mapped
    Hessian wherever H_p is already PSD, and the same result as projecting the
    free principal submatrix when every movable vertex is free."""
    p, o = scene
    s = o.scene
    X = p["X0"]
    _, _, Hp, _ = s.contact_terms(X, local.PROJECTED)
    _, _, He, _ = s.contact_terms(X, local.EXACT)
    for st in range(Hp.shape[0]):
        L = int((s.rows[st] >= 0).sum())
        A = Hp[st, :3 * L, :3 * L].numpy()
        w = np.linalg.eigvalsh(A)
        assert w.min() >= -1e-10 * max(1.0, np.abs(w).max())
    xs, mov = s.positions(X)
    _, _, Hpos, _ = local.contact_local(xs, torch.as_tensor(s.ctype), mov, float(p["kappa"]), float(p["dhat"]),
                                        local.EXACT)
    for st in range(Hp.shape[0]):
        wpos = np.linalg.eigvalsh(Hpos[st].numpy())
        if wpos.min() >= 0.0:
            assert np.allclose(Hp[st].numpy(), He[st].numpy(), rtol=1e-9, atol=1e-12 * np.abs(He[st].numpy()).max())
    # a stencil with free vertices only: the union mapping is the identity
    q = dict(p)
    free_pt = np.array([[0, 1, 2, 3]], np.int32)  # any four free vertices
    q["bctype"], q["bcidx"] = np.array([3], np.int32), np.array([[free_pt[0, 0], free_pt[0, 1], -1, -1]], np.int32)
    sq = affine.AffineScene(q)
    _, _, Hq, _ = sq.contact_terms(X, local.PROJECTED)
    xq, mq = sq.positions(X)
    _, _, Href, _ = local.contact_local(xq, torch.as_tensor(sq.ctype), mq, float(p["kappa"]), float(p["dhat"]))
    assert np.allclose(Hq[0, :6, :6].numpy(), Href[0, :6, :6].numpy(), rtol=0, atol=1e-15 * np.abs(Href).max())


def test_rigid_motion_invariance(scene):
    """Rotating and translating everything (free and fixed vertices, A -> R A,
    t -> R t + c) leaves the barrier and orthogonality energies unchanged."""
    p, o = scene
    rng = np.random.default_rng(6)
    Q, _ = np.linalg.qr(rng.normal(size=(3, 3)))
    R = Q * np.sign(np.linalg.det(Q))
    c = rng.normal(size=3)
    n = p["n_free"]
    X = p["X0"]
    Xr = X.copy()
    Xr[:n] = X[:n] @ R.T + c
    for b in range(p["n_bodies"]):
        rows = X[n + 4 * b:n + 4 * b + 4]
        Xr[n + 4 * b:n + 4 * b + 3] = rows[:3] @ R.T
        Xr[n + 4 * b + 3] = R @ rows[3] + c
    q = dict(p)
    q["x_fixed"] = p["x_fixed"] @ R.T + c
    orot = affine.AffineOracle(q)
    e0 = o.scene.contact_terms(X)[0].numpy()
    e1 = orot.scene.contact_terms(Xr)[0].numpy()
    assert np.allclose(e0, e1, rtol=1e-8, atol=1e-12 * np.abs(e0).max())
    o0 = o.scene.body_terms(X)[1].numpy()
    o1 = orot.scene.body_terms(Xr)[1].numpy()
    assert np.allclose(o0, o1, rtol=1e-8, atol=1e-14)


def test_newton_step_decreases_energy(scene):
    p, o = scene
    X1, info = onewton.newton_step(o, p["X0"], rtol=1e-10)
    assert info["cg_status"] == "ok" and info["alpha"] > 0
    assert info["E1"] < info["E0"]
    assert (o.distances(X1) > 0).all()
    # the PCG direction solves the assembled system
    ev = o.eval(p["X0"])
    asm = o.assemble(ev)
    H = o.csr(asm).toarray()
    pd = np.linalg.solve(H, -asm["grad"].ravel())
    assert np.linalg.norm(info["p"].ravel() - pd) <= 1e-8 * np.linalg.norm(pd)
