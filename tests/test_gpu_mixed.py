"""Precision form (float32 element Hessians, BSR values and PCG vectors; float64
contact arithmetic, energies, gradient and residual replacement) against the
float64 oracle: gradient rel. error <= 1e-5 and Newton direction rel. error
<= 1e-4 (direction of reference solved to rtol 1e-12)."""
import numpy as np
import pytest
import torch

from oracle import assemble as oasm
from oracle import pcg as opcg
from paper_2605_23088_amd import synth

pytestmark = pytest.mark.gpu


def cases():
    return {
        "block_mid": synth.small_block(seed=12, nx=10, ny=9, nz=8, n_pt=600, n_ee=500),
        "C1": synth.c1_two_cubes(),
    }


@pytest.fixture(scope="module", params=["block_mid", "C1"])
def mixed_case(request):
    from paper_2605_23088_amd.yasps import MIXED, Yasps
    p = cases()[request.param]
    o = oasm.Oracle(p)
    ev = o.eval(p["x0"])
    asm = o.assemble(ev)
    H = o.csr(asm)
    Minv = opcg.block_inverse(o.diag_blocks(asm))
    g_ref = asm["grad"].ravel()
    p_ref, it, _, st = opcg.pcg(lambda v: H @ v, -g_ref, Minv, 1e-12, 50000)
    assert st == "ok"
    gm = Yasps(p, precision=MIXED)
    return p, o, ev, asm, H, g_ref, p_ref, gm


def test_mixed_gradient_and_values(mixed_case):
    p, o, ev, asm, H, g_ref, p_ref, gm = mixed_case
    x = torch.as_tensor(p["x0"], dtype=torch.float64, device="cuda").contiguous()
    info = gm.eval(x)
    assert abs(info["energy"] - ev["E"]) <= 1e-10 * (np.abs(ev["E_t"]).sum() + np.abs(ev["E_c"]).sum()
                                                    + abs(ev["E_inertia"]))
    out = gm.assemble()
    assert out["values_s"].dtype == torch.float32
    g = out["grad"].cpu().numpy().ravel()
    assert np.linalg.norm(g - g_ref) <= 1e-5 * np.linalg.norm(g_ref)
    vs = out["values_s"].cpu().numpy().astype(np.float64)
    assert np.linalg.norm(vs - asm["values_s"]) <= 1e-5 * np.linalg.norm(asm["values_s"])
    if len(o.ci_d):
        vd = out["values_d"].cpu().numpy().astype(np.float64)
        assert np.linalg.norm(vd - asm["values_d"]) <= 1e-5 * np.linalg.norm(asm["values_d"])


def test_mixed_newton_direction(mixed_case):
    p, o, ev, asm, H, g_ref, p_ref, gm = mixed_case
    x = torch.as_tensor(p["x0"], dtype=torch.float64, device="cuda").contiguous()
    gm.eval(x)
    a = gm.assemble()
    pd, info = gm.pcg(-a["grad"].contiguous(), rtol=1e-8)
    assert info["status"] == 0
    pv = pd.cpu().numpy().ravel()
    err = np.linalg.norm(pv - p_ref) / np.linalg.norm(p_ref)
    assert err <= 1e-4, err
    # the reported residual is a float64 true residual of the float32-valued system
    assert info["rel_residual"] <= 1e-8


def test_mixed_newton_step_decreases_energy(mixed_case):
    p, o, ev, asm, H, g_ref, p_ref, gm = mixed_case
    x = torch.as_tensor(p["x0"], dtype=torch.float64, device="cuda").contiguous()
    ni = gm.newton_step(x, rtol=1e-8)
    assert ni["status"] == 0 and ni["e1"] < ni["e0"] and ni["alpha"] > 0
    assert (o.distances(x.cpu().numpy()) > 0).all()
