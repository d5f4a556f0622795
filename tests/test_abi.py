"""The C ABI library loads without a GPU and exports every function declared
in include/nrto.h."""
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2603_02642_amd", "libnrto.so")


def declared():
    src = open(os.path.join(ROOT, "include", "nrto.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(nrto_[a-z_0-9]+)\s*\(", src)))


def test_header_declares_core_entry_points():
    names = declared()
    for n in ["nrto_setup", "nrto_scp_step", "nrto_solve_socp", "nrto_project_soc", "nrto_destroy",
              "nrto_last_error", "nrto_linearize"]:
        assert n in names


def test_library_exports_all_declared_symbols():
    if not os.path.exists(LIB):
        pytest.skip("library not built")
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True, text=True, check=True).stdout
    exported = set(l.split()[-1] for l in out.splitlines() if l.strip())
    missing = [n for n in declared() if n not in exported]
    assert not missing, missing


def test_library_loads_and_defaults_without_gpu():
    if not os.path.exists(LIB):
        pytest.skip("library not built")
    from paper_2603_02642_amd import nrto
    o = nrto.default_options()
    assert o.rho == 40.0 and o.max_admm == 40 and o.max_inner == 100 and o.eps_kkt == 1e-4
