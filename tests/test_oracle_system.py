"""Pins for the oracle's pattern, assembly, block-Jacobi PCG and Newton step:
closed-form block counts, a brute-force set-based pattern builder, dense
brute-force assembly, dense direct solves and SciPy's CG, and the line-search
guarantees."""
import json
import os

import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle import assemble, newton, pattern, pcg
from paper_2605_23088_amd import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.fixture(scope="module")
def c1():
    p = synth.c1_two_cubes()
    o = assemble.Oracle(p)
    ev = o.eval(p["x0"])
    asm = o.assemble(ev)
    return p, o, ev, asm


@pytest.mark.parametrize("dims", [(1, 1, 1), (4, 4, 4), (3, 5, 2), (7, 2, 6)])
def test_static_block_count_closed_form(dims):
    nx, ny, nz = dims
    tets = synth.kuhn_tets(nx, ny, nz)
    n = (nx + 1) * (ny + 1) * (nz + 1)
    rp, ci, _ = pattern.build(n, [tets], True)
    # vertices + axis edges + face diagonals + body diagonals
    assert len(ci) == (2 * nx + 1) * (2 * ny + 1) * (2 * nz + 1)


def test_golden_counts():
    with open(os.path.join(GOLDEN, "counts.json")) as f:
        gold = json.load(f)
    assert [len(pattern.local_pairs(k)) for k in (4, 3, 2)] == gold["upper_pairs_per_stencil"]
    n = 125
    rp, ci, _ = pattern.build(n, [synth.kuhn_tets(4, 4, 4)], True)
    assert len(ci) == gold["nnzb_4x4x4_cube"]
    # one gradient placement index per vertex: 4 for a tet, not 12
    assert pattern.used_vertices(np.array([[0, 1, 2, 3]]))[0] == gold["snh_gradient_indices"]
    # DoF of N free vertices plus one affine body: 3N + 9 + 3
    N = 17
    assert 3 * N + 9 + 3 == gold["dof_example"]["formula_value_at_N17"]


def brute_pattern(n, idx_list, diag):
    keys = set()
    if diag:
        keys |= {(v, v) for v in range(n)}
    for idx in idx_list:
        for row in idx:
            vs = [v for v in row if v >= 0]
            for a in range(len(vs)):
                for b in range(a, len(vs)):
                    if vs[a] < n and vs[b] < n:
                        keys.add((min(vs[a], vs[b]), max(vs[a], vs[b])))
    return sorted(keys)


def test_pattern_matches_brute_force_sets(c1):
    p, o, _, _ = c1
    n = o.n
    for (rp, ci, slots, idx, diag) in ((o.rp_s, o.ci_s, o.slot_t, o.tet_idx, True),
                                       (o.rp_d, o.ci_d, o.slot_c, o.cidx, False)):
        keys = brute_pattern(n, [idx], diag)
        rows = np.repeat(np.arange(n), np.diff(rp))
        assert list(zip(rows.tolist(), ci.tolist())) == keys
        lookup = {k: i for i, k in enumerate(keys)}
        for s, row in enumerate(idx):
            vs = [v for v in row if v >= 0]
            q = 0
            for a in range(len(vs)):
                for b in range(a, len(vs)):
                    want = lookup.get((min(vs[a], vs[b]), max(vs[a], vs[b])), -1) \
                        if vs[a] < n and vs[b] < n else -1
                    assert slots[s, q] == want
                    q += 1
            assert (slots[s, q:] == -1).all()
    # diagonal is the first block of every static row
    assert (o.ci_s[o.rp_s[:-1]] == np.arange(n)).all()


def test_pattern_with_fixed_and_short_stencils():
    n = 6
    idx = np.array([[0, 7, 2, 3], [4, 1, -1, -1], [5, 2, 8, -1], [9, 10, 1, 0]])
    rp, ci, (slot,) = pattern.build(n, [idx], False)
    keys = brute_pattern(n, [idx], False)
    rows = np.repeat(np.arange(n), np.diff(rp))
    assert list(zip(rows.tolist(), ci.tolist())) == keys
    assert (slot[1, 3:] == -1).all() and (slot[2, 6:] == -1).all()
    assert slot[0, 1] == -1 and slot[3, 0] == -1


def test_dense_bruteforce_assembly(c1):
    p, o, ev, asm = c1
    n = o.n
    Hd = np.zeros((3 * n, 3 * n))
    gd = ev["g_inertia"].copy()
    for idx, Hl, gl in ((o.tet_idx, ev["H_t"], ev["g_t"]), (o.cidx, ev["H_c"], ev["g_c"])):
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
    D = o.diag_blocks(asm)
    for v in range(n):
        assert np.allclose(D[v], Hd[3 * v:3 * v + 3, 3 * v:3 * v + 3], rtol=0, atol=1e-12 * np.abs(Hd).max())
    # upper-storage dense expansion agrees with the scalar CSR
    Dn = assemble.to_dense(o.rp_s, o.ci_s, asm["values_s"], n) + assemble.to_dense(o.rp_d, o.ci_d, asm["values_d"], n)
    assert np.array_equal(Dn, Dn.T) and np.abs(Dn - H).max() <= 1e-13 * np.abs(H).max()


def test_pcg_matches_direct_solve_and_scipy(c1):
    p, o, ev, asm = c1
    H = o.csr(asm)
    Hd = H.toarray()
    g = asm["grad"].ravel()
    Minv = pcg.block_inverse(o.diag_blocks(asm))
    x, it, rel, st = pcg.pcg(lambda v: H @ v, -g, Minv, 1e-12, 20000)
    assert st == "ok" and it <= 3 * o.n
    xd = np.linalg.solve(Hd, -g)
    assert np.linalg.norm(x - xd) <= 1e-8 * np.linalg.norm(xd)
    assert np.linalg.norm(Hd @ x + g) <= 1e-12 * np.linalg.norm(g) * (1 + 1e-6)
    Mop = spla.LinearOperator(Hd.shape, matvec=lambda r: np.einsum("vij,vj->vi", Minv, r.reshape(-1, 3)).ravel())
    xs, info = spla.cg(H, -g, rtol=1e-12, atol=0.0, M=Mop, maxiter=20000)
    assert info == 0 and np.linalg.norm(xs - xd) <= 1e-8 * np.linalg.norm(xd)


def test_pcg_status_paths(c1):
    p, o, ev, asm = c1
    H = o.csr(asm)
    g = asm["grad"].ravel()
    Minv = pcg.block_inverse(o.diag_blocks(asm))
    x, it, rel, st = pcg.pcg(lambda v: H @ v, -g, Minv, 1e-8, 1)
    assert st == "noconv" and it == 1 and rel > 1e-8
    x, it, rel, st = pcg.pcg(lambda v: -(H @ v), -g, -Minv, 1e-8, 100)
    assert st == "breakdown"
    x, it, rel, st = pcg.pcg(lambda v: H @ v, np.zeros_like(g), Minv, 1e-8, 100)
    assert st == "ok" and it == 0 and not x.any()


def test_pcg_exact_in_n_steps_for_block_diagonal():
    rng = np.random.default_rng(0)
    n = 30
    A = rng.normal(size=(n, 3, 3))
    D = A @ A.transpose(0, 2, 1) + np.eye(3)
    Hd = np.zeros((3 * n, 3 * n))
    for v in range(n):
        Hd[3 * v:3 * v + 3, 3 * v:3 * v + 3] = D[v]
    b = rng.normal(size=3 * n)
    x, it, rel, st = pcg.pcg(lambda v: Hd @ v, b, pcg.block_inverse(D), 1e-12, 10)
    # block-Jacobi inverts a block-diagonal system exactly (appendix "Preconditioner")
    assert st == "ok" and it == 1


def test_newton_step_decreases_energy_and_stays_feasible(c1):
    p, o, ev, asm = c1
    x1, info = newton.newton_step(o, p["x0"], rtol=1e-8)
    assert info["cg_status"] == "ok"
    assert info["alpha"] > 0 and info["E1"] < info["E0"]
    assert (o.distances(x1) > 0).all()
    assert (np.sign(o.sides(x1)) == np.sign(o.sides(p["x0"]))).all()
    assert abs(o.energy(x1) - info["E1"]) <= 1e-12 * abs(info["E1"])
    # energy-only path agrees with the full evaluation
    assert abs(o.energy(p["x0"]) - ev["E"]) <= 1e-13 * abs(ev["E"])
    # the direction is a descent direction
    assert float(asm["grad"].ravel() @ info["p"].ravel()) < 0


def test_newton_converges_on_c1(c1):
    p, o, _, _ = c1
    x = p["x0"].copy()
    E = []
    for _ in range(8):
        x, info = newton.newton_step(o, x, rtol=1e-10)
        E.append(info["E1"])
    assert all(b <= a for a, b in zip(E, E[1:]))
    g = o.assemble(o.eval(x))["grad"]
    assert np.abs(g).max() < 1e-6 * np.abs(o.assemble(o.eval(p["x0"]))["grad"]).max()
