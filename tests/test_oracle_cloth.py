"""Pins for the oracle's cloth terms: the StVK membrane and the dihedral
(discrete-shells) hinge.  Closed forms for uniform and uniaxial stretch and
for a hinge folded by a known angle, zero energy and gradient at rest, rigid
motion invariance, central finite differences of energy and gradient, the
F-space projection reducing to the exact Hessian where d2Psi/dF2 is PSD, and a
dense brute-force assembly of a small cloth scene against the BSR."""
import numpy as np
import pytest
import torch

from oracle import assemble, local
from oracle import energy as en
from paper_2605_23088_amd import synth

torch.set_default_dtype(torch.float64)
MU, LAM, THICK = 3.8e4, 3.3e4, 1e-3


def rot(rng):
    q = rng.standard_normal(4)
    q /= np.linalg.norm(q)
    w, x, y, z = q
    return np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)],
                     [2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)],
                     [2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)]])


def rest_triangle(rng):
    P = rng.uniform(-1, 1, (3, 2))
    D = np.stack([P[1] - P[0], P[2] - P[0]], 1)
    if np.linalg.det(D) < 0:
        P[[1, 2]] = P[[2, 1]]
        D = np.stack([P[1] - P[0], P[2] - P[0]], 1)
    return P, np.linalg.inv(D), 0.5 * abs(np.linalg.det(D))


def psi_m(x, Dinv, A):
    return float(en.stvk_membrane(torch.tensor(x), torch.tensor(Dinv), torch.tensor(A), torch.tensor(THICK),
                                  torch.tensor(MU), torch.tensor(LAM)))


def embed(P, R, t, scale=np.eye(2)):
    Q = P @ scale.T
    return np.concatenate([Q, np.zeros((3, 1))], 1) @ R.T + t


@pytest.mark.parametrize("seed", range(4))
def test_membrane_rest_and_rigid_motion(seed):
    rng = np.random.default_rng(seed)
    P, Dinv, A = rest_triangle(rng)
    x = embed(P, rot(rng), rng.standard_normal(3))
    xt = torch.tensor(x, requires_grad=True)
    E = en.stvk_membrane(xt, torch.tensor(Dinv), torch.tensor(A), torch.tensor(THICK), torch.tensor(MU),
                         torch.tensor(LAM))
    E.backward()
    assert abs(float(E.detach())) < 1e-20 and float(xt.grad.abs().max()) < 1e-9
    # a deformed state keeps its energy under any rigid motion
    S = np.array([[1.3, 0.2], [-0.1, 0.8]])
    e1 = psi_m(embed(P, np.eye(3), 0, S), Dinv, A)
    e2 = psi_m(embed(P, rot(rng), rng.standard_normal(3), S), Dinv, A)
    assert abs(e1 - e2) <= 1e-12 * e1


@pytest.mark.parametrize("s", [0.7, 1.0, 1.25])
def test_membrane_closed_forms(s):
    rng = np.random.default_rng(11)
    P, Dinv, A = rest_triangle(rng)
    g = 0.5 * (s * s - 1)
    tol = 1e-12 * A * THICK * (MU + LAM) * max(g * g, 1e-12)
    # uniform in-plane stretch: G = g I -> A t (2 mu + 2 lam) g^2
    e = psi_m(embed(P, np.eye(3), 0, s * np.eye(2)), Dinv, A)
    assert abs(e - A * THICK * 2 * (MU + LAM) * g * g) <= tol
    # uniaxial stretch along the rest x axis: G = diag(g, 0) -> A t (mu + lam/2) g^2
    e = psi_m(embed(P, np.eye(3), 0, np.diag([s, 1.0])), Dinv, A)
    assert abs(e - A * THICK * (MU + 0.5 * LAM) * g * g) <= tol


def membrane_eval(x, Dinv, A, hess):
    E, g, H = local.membrane_local(torch.tensor(x)[None], torch.tensor(Dinv)[None], torch.tensor([A]), THICK,
                                   MU, LAM, 1.0, torch.ones(1, 4, dtype=torch.bool), hess)
    return float(E[0]), g[0, :3].numpy().ravel(), H[0, :9, :9].numpy()


def test_membrane_finite_differences():
    rng = np.random.default_rng(5)
    P, Dinv, A = rest_triangle(rng)
    x = embed(P, rot(rng), 0) + 0.2 * rng.standard_normal((3, 3))
    E, g, H = membrane_eval(x, Dinv, A, assemble.EXACT)
    eps = 1e-6
    for k in range(9):
        dx = np.zeros(9)
        dx[k] = eps
        Ep = membrane_eval(x + dx.reshape(3, 3), Dinv, A, assemble.EXACT)
        Em = membrane_eval(x - dx.reshape(3, 3), Dinv, A, assemble.EXACT)
        assert abs((Ep[0] - Em[0]) / (2 * eps) - g[k]) <= 1e-6 * np.abs(g).max()
        assert np.abs((Ep[1] - Em[1]) / (2 * eps) - H[:, k]).max() <= 1e-6 * np.abs(H).max()


def test_membrane_projection():
    rng = np.random.default_rng(9)
    P, Dinv, A = rest_triangle(rng)
    R = rot(rng)
    # stretched: d2Psi/dF2 is PSD, so the F-space projection is the exact Hessian
    x = embed(P, R, 0, 1.2 * np.eye(2))
    _, _, He = membrane_eval(x, Dinv, A, assemble.EXACT)
    _, _, Hp = membrane_eval(x, Dinv, A, assemble.PROJECTED)
    assert np.abs(He - Hp).max() <= 1e-10 * np.abs(He).max()
    # compressed: the exact Hessian is indefinite, the projection is PSD and
    # still annihilates the three translations
    x = embed(P, R, 0, 0.6 * np.eye(2))
    _, _, He = membrane_eval(x, Dinv, A, assemble.EXACT)
    _, _, Hp = membrane_eval(x, Dinv, A, assemble.PROJECTED)
    assert np.linalg.eigvalsh(He).min() < -1e-6 * np.abs(He).max()
    assert np.linalg.eigvalsh(Hp).min() >= -1e-10 * np.abs(Hp).max()
    T = np.kron(np.ones((3, 1)), np.eye(3))
    assert np.abs(Hp @ T).max() <= 1e-10 * np.abs(Hp).max()


def hinge(phi, edge=1.0):
    """Edge x0 -> x1 on the x axis, wing x2 in the xy plane at height 1, wing x3
    the mirror image rotated about the edge by phi."""
    return np.array([[0.0, 0, 0], [edge, 0, 0], [0.5, 1.0, 0], [0.5, -np.cos(phi), -np.sin(phi)]])


@pytest.mark.parametrize("phi", [0.0, 0.3, -1.1, 2.5, -3.0])
def test_hinge_angle_closed_form_and_symmetries(phi):
    rng = np.random.default_rng(3)
    x = hinge(phi)
    th = float(en.hinge_angle(torch.tensor(x)))
    assert abs(th - phi) <= 1e-13
    # rigid motion and relabelling the hinge (edge reversed, wings swapped)
    y = x @ rot(rng).T + rng.standard_normal(3)
    assert abs(float(en.hinge_angle(torch.tensor(y))) - phi) <= 1e-12
    assert abs(float(en.hinge_angle(torch.tensor(x[[1, 0, 3, 2]]))) - phi) <= 1e-12


def test_hinge_energy_gradient_and_flat_hessian():
    k = 0.37
    x = hinge(0.0, edge=2.0)
    xt = torch.tensor(x)
    E, g, H = local.hinge_local(xt[None], torch.zeros(1), torch.tensor([k]), 1.0,
                                torch.ones(1, 4, dtype=torch.bool), assemble.EXACT)
    assert float(E[0]) == 0.0 and float(g.abs().max()) == 0.0
    # flat hinge: H = 2 k grad(theta) grad(theta)^T, grad(theta) at a wing
    # vertex is along the normal with length |e| / |n| = 1 / (wing height)
    gt = torch.func.grad(en.hinge_angle)(xt).numpy()
    assert abs(abs(gt[2, 2]) - 1.0) <= 1e-12 and abs(abs(gt[3, 2]) - 1.0) <= 1e-12
    assert np.abs(gt[:, :2]).max() <= 1e-12 and np.abs(gt.sum(0)).max() <= 1e-12
    gv = gt.ravel()
    assert np.abs(H[0].numpy() - 2 * k * np.outer(gv, gv)).max() <= 1e-12
    # at a fold the energy is k (theta - theta_bar)^2
    E, _, _ = local.hinge_local(torch.tensor(hinge(0.8))[None], torch.tensor([0.3]), torch.tensor([k]), 1.0,
                                torch.ones(1, 4, dtype=torch.bool), assemble.EXACT)
    assert abs(float(E[0]) - k * 0.5 ** 2) <= 1e-14


def test_hinge_finite_differences_and_projection():
    rng = np.random.default_rng(4)
    x = hinge(0.9) + 0.05 * rng.standard_normal((4, 3))
    tb, k = torch.tensor([0.2]), torch.tensor([0.5])
    one = torch.ones(1, 4, dtype=torch.bool)

    def ev(y, hess=assemble.EXACT):
        E, g, H = local.hinge_local(torch.tensor(y)[None], tb, k, 1.0, one, hess)
        return float(E[0]), g[0].numpy().ravel(), H[0].numpy()

    E, g, H = ev(x)
    eps = 1e-6
    for j in range(12):
        d = np.zeros(12)
        d[j] = eps
        Ep, gp, _ = ev(x + d.reshape(4, 3))
        Em, gm, _ = ev(x - d.reshape(4, 3))
        assert abs((Ep - Em) / (2 * eps) - g[j]) <= 1e-6 * np.abs(g).max()
        assert np.abs((gp - gm) / (2 * eps) - H[:, j]).max() <= 1e-5 * np.abs(H).max()
    _, _, Hp = ev(x, assemble.PROJECTED)
    w = np.linalg.eigvalsh(Hp)
    assert w.min() >= -1e-12 * w.max()
    T = np.kron(np.ones((4, 1)), np.eye(3))
    assert np.abs(Hp @ T).max() <= 1e-10 * np.abs(Hp).max()
    # projection keeps the positive part: Hp - H is PSD
    assert np.linalg.eigvalsh(Hp - H).min() >= -1e-10 * np.abs(H).max()


@pytest.fixture(scope="module")
def cloth():
    p = synth.small_cloth()
    rng = np.random.default_rng(2)
    x = p["x0"] + 1e-4 * rng.standard_normal(p["x0"].shape)
    o = assemble.Oracle(p)
    ev = o.eval(x)
    return p, o, ev, o.assemble(ev), x


def test_cloth_generator_shape(cloth):
    p, o, ev, asm, x = cloth
    n_sheet = 15 * 15
    assert p["n_free"] == 7 * 7 * 3 + 2 * n_sheet
    assert len(p["tri_idx"]) == 2 * 2 * 14 * 14
    assert len(p["hinge_idx"]) == 2 * (3 * 14 * 14 - 2 * 14)
    counts = np.bincount(p["ctype"], minlength=4)
    assert counts.tolist() == [250, 250, 100, 40]
    assert (p["contact_d"] > 0).all() and (p["contact_d"] < p["dhat"]).all()
    # the stored distances are the oracle's distances at x0
    assert np.allclose(o.distances(p["x0"]), p["contact_d"], rtol=1e-10, atol=0)
    # the sheets rest flat: the gap fields stretch and bend them at x0, and a
    # flattened copy has zero membrane and bending energy
    ev0 = o.eval(p["x0"])
    assert (ev0["E_f"] >= 0).all() and (ev0["E_h"] >= 0).all() and ev0["E_f"].max() > 0
    xf = p["x0"].copy()
    cloth_v = np.unique(p["tri_idx"])
    xf[cloth_v, 2] = 0.0
    assert float(o.tris(xf)[0].abs().max()) < 1e-20 and float(o.hinges(xf)[0].abs().max()) < 1e-20


def test_cloth_dense_bruteforce_assembly(cloth):
    p, o, ev, asm, x = cloth
    n = o.n
    Hd = np.zeros((3 * n, 3 * n))
    gd = ev["g_inertia"].copy()
    for idx, Hl, gl in ((o.tet_idx, ev["H_t"], ev["g_t"]), (o.tri_idx, ev["H_f"], ev["g_f"]),
                        (o.hinge_idx, ev["H_h"], ev["g_h"]), (o.cidx, ev["H_c"], ev["g_c"])):
        for s in range(idx.shape[0]):
            for a in range(4):
                va = idx[s, a]
                if not 0 <= va < n:
                    continue
                gd[va] += gl[s, a]
                for b in range(4):
                    vb = idx[s, b]
                    if 0 <= vb < n:
                        Hd[3 * va:3 * va + 3, 3 * vb:3 * vb + 3] += Hl[s, 3 * a:3 * a + 3, 3 * b:3 * b + 3]
    Hd += np.kron(np.diag(p["mass"]), np.eye(3))
    H = o.csr(asm).toarray()
    assert np.abs(H - Hd).max() <= 1e-12 * np.abs(Hd).max()
    assert np.abs(asm["grad"] - gd).max() <= 1e-12 * np.abs(gd).max()
    assert np.array_equal(H, H.T)
    assert np.linalg.eigvalsh(H).min() > 0
