"""Host-only checks of the C-ABI boundary: the library is built for gfx950,
loads, and exports every entry point the header declares (no compute calls)."""
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "yasps.h")
LIB = os.path.join(ROOT, "paper_2605_23088_amd", "libyasps.so")


def declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(yasps_[a-z_]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = declared()
    for f in ("yasps_create", "yasps_set_contacts", "yasps_eval_stencils", "yasps_assemble_bsr", "yasps_pcg",
              "yasps_newton_step", "yasps_get_pattern", "yasps_destroy", "yasps_last_error"):
        assert f in names


def test_library_exports_every_declared_symbol():
    if not os.path.exists(LIB):
        pytest.fail("libyasps.so is not built (python -m paper_2605_23088_amd.build)")
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True, text=True, check=True).stdout
    exported = set(line.split()[-1] for line in out.splitlines() if line.strip())
    missing = [f for f in declared() if f not in exported]
    assert not missing, missing


def test_library_loads_and_binding_matches_header():
    import torch  # noqa: F401  (load torch's HIP runtime first)
    from paper_2605_23088_amd import yasps
    L = yasps.lib()
    for f in declared():
        assert hasattr(L, f), f
    assert set(yasps.EXPORTS) == set(declared())


def test_library_holds_gfx950_code():
    # the embedded offload bundle names its target triple and processor
    data = open(LIB, "rb").read()
    assert b"amdgcn-amd-amdhsa--gfx950" in data


def test_binding_fails_loudly_without_library(tmp_path, monkeypatch):
    from paper_2605_23088_amd import yasps
    monkeypatch.setattr(yasps, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(yasps, "_lib", None)
    with pytest.raises(RuntimeError):
        yasps.lib()


def _header_struct_fields(name):
    src = re.sub(r"/\*.*?\*/", "", open(HEADER).read(), flags=re.S)
    body = re.search(r"typedef struct \{([^}]*)\}\s*" + name + r"\s*;", src).group(1)
    return [re.findall(r"(\w+)\s*(?:\[[^\]]*\])?\s*$", d.strip())[0] for d in body.split(";") if d.strip()]


@pytest.mark.parametrize("name,cls", [("yasps_params", "Params"), ("yasps_newton_params", "NewtonParams"),
                                      ("yasps_eval_info", "EvalInfo")])
def test_binding_structs_match_header(name, cls):
    from paper_2605_23088_amd import yasps
    fields = [f[0] for f in getattr(yasps, cls)._fields_]
    assert fields == _header_struct_fields(name)
