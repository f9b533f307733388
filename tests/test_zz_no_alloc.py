"""The non-allocating solve (yasps_pcg_noalloc) against yasps_pcg.

Both run the same kernels in the same order, so the non-allocating call must
return the same solution bit for bit; its workspace is a fixed per-GPU array
that keeps the previous call's contents, so it is called twice in a row, the
second time on a smaller system, and once on a system too large for the array
(a clear YASPS_E_ARG, after which the array still serves smaller systems).
"""
import numpy as np
import pytest
import torch

from paper_2605_23088_amd import synth

pytestmark = pytest.mark.gpu


def _solve_both(g, b, rtol):
    x_ref, info_ref = g.pcg(b, rtol=rtol)
    x = torch.full_like(b, float("nan"))
    info = g.pcg_noalloc(b, x, rtol=rtol, allow=(-1, -5))
    torch.cuda.synchronize()
    return x_ref, info_ref, x, info, info["rc"]


def _system(p, precision):
    from paper_2605_23088_amd.yasps import Yasps
    g = Yasps(p, precision=precision)
    x0 = torch.as_tensor(p["x0"], dtype=torch.float64, device="cuda").contiguous()
    g.eval(x0)
    out = g.assemble()
    return g, (-out["grad"]).contiguous()


@pytest.mark.parametrize("precision", [0, 1], ids=["fp64", "mixed"])
def test_noalloc_equals_pcg_twice_then_smaller(precision):
    from paper_2605_23088_amd.yasps import OK
    big = synth.small_block(seed=12, nx=10, ny=9, nz=8, n_pt=600, n_ee=500)  # 990 free vertices
    small = synth.c1_two_cubes()                                               # 250 free vertices
    assert small["n_free"] < big["n_free"]
    for p in (big, small):
        g, b = _system(p, precision)
        x_ref, info_ref, x, info, rc = _solve_both(g, b, 1e-10)
        assert rc == OK, rc
        assert info["iters"] == info_ref["iters"] and info["status"] == info_ref["status"]
        assert info["rel_residual"] == info_ref["rel_residual"]
        assert torch.equal(x, x_ref), float((x - x_ref).abs().max())
        g.close()


def test_noalloc_rejects_a_system_beyond_its_array():
    from paper_2605_23088_amd.yasps import E_ARG, OK, Yasps, lib
    n = 320_000  # inertia only: 120 bytes of workspace per free vertex, more than the fixed 32 MiB
    rng = np.random.default_rng(3)
    x0 = rng.uniform(0.0, 1.0, (n, 3))
    p = dict(n_free=n, x0=x0, x_fixed=np.zeros((0, 3)), mass=np.full(n, 0.5), x_tilde=x0 + 1e-3,
             tet_idx=np.zeros((0, 4), np.int32), dm_inv=np.zeros((0, 3, 3)), vol=np.zeros(0),
             mu=1.0, lam=1.0, h=1e-2, kappa=1.0, dhat=1e-3)
    g, b = _system(p, 0)
    x_ref, info_ref, x, info, rc = _solve_both(g, b, 1e-10)
    assert rc == E_ARG
    assert "yasps_pcg_noalloc" in lib().yasps_last_error(g.ctx).decode()
    assert torch.isnan(x).all()  # nothing was written
    # the solve itself is diagonal here: one iteration, x = M^-1 b
    assert info_ref["iters"] <= 2
    g.close()
    # the array still serves a system that fits
    q = synth.small_block(seed=11, nx=5, ny=4, nz=3, n_pt=150, n_ee=150)
    g, b = _system(q, 0)
    x_ref, info_ref, x, info, rc = _solve_both(g, b, 1e-10)
    assert rc == OK and torch.equal(x, x_ref)
    g.close()
