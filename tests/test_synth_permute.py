"""The seeded vertex relabelling of the benchmark's permuted variant: a
bijection of the free vertices that leaves fixed ids and padding alone, and
under which the oracle's energy is unchanged and its gradient and Hessian
are the relabelled ones."""
import numpy as np
import pytest

from oracle import assemble as oasm
from paper_2605_23088_amd import synth


def test_permute_vertices_relabels_the_free_vertices_only():
    p = synth.small_block()
    q, perm = synth.permute_vertices(p, seed=3)
    n = p["n_free"]
    assert sorted(perm.tolist()) == list(range(n))
    assert np.array_equal(q["x0"][perm], p["x0"])
    assert np.array_equal(q["mass"][perm], p["mass"])
    assert np.array_equal(q["tet_idx"], perm[p["tet_idx"]])
    ci, cq = p["cidx"], q["cidx"]
    free = (ci >= 0) & (ci < n)
    assert np.array_equal(cq[free], perm[ci[free]]) and np.array_equal(cq[~free], ci[~free])


def test_oracle_is_invariant_under_the_relabelling():
    p = synth.small_block()
    q, perm = synth.permute_vertices(p, seed=4)
    op, oq = oasm.Oracle(p), oasm.Oracle(q)
    ep, eq = op.eval(p["x0"]), oq.eval(q["x0"])
    assert eq["E"] == pytest.approx(ep["E"], rel=1e-12)
    ap, aq = op.assemble(ep), oq.assemble(eq)
    gp, gq = np.asarray(ap["grad"]), np.asarray(aq["grad"])
    assert np.abs(gq[perm] - gp).max() <= 1e-11 * np.abs(gp).max()
    Hp, Hq = op.csr(ap).toarray(), oq.csr(aq).toarray()
    P = np.repeat(3 * perm, 3) + np.tile(np.arange(3), len(perm))
    assert np.abs(Hq[np.ix_(P, P)] - Hp).max() <= 1e-11 * np.abs(Hp).max()
