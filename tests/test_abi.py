"""The C-ABI library loads and exports every symbol its header declares, and
argument errors are reported before any device work (CPU-only checks)."""
import ctypes as C
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def dcf():
    from paper_2406_19494_amd import binding
    if not os.path.exists(binding.LIB_PATH):
        from paper_2406_19494_amd import build
        build.build()
    return binding


def test_library_exports_every_declared_symbol(dcf):
    L = dcf.lib()
    declared = dcf.declared_symbols()
    assert "dcf_rk3_step" in declared and "dcf_vjp_step" in declared
    missing = [s for s in declared if not hasattr(L, s)]
    assert not missing, missing


def test_exports_match_nm(dcf):
    out = subprocess.run(["nm", "-D", "--defined-only", dcf.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = {line.split()[-1] for line in out.splitlines() if " T dcf_" in line}
    assert set(dcf.declared_symbols()) <= exported


def test_invalid_arguments_rejected_without_device(dcf):
    L = dcf.lib()
    g = dcf.dcf_grid()
    g.ndim = 3
    g.n[0], g.n[1], g.n[2] = 2, 8, 8   # fewer than 3 cells on an active axis
    for d in range(3):
        g.hi[d] = 1.0
    gas = dcf.dcf_gas(1.4, 1.0, 0.7, 0, 0.0, 1.0, 0.0)
    ctx = C.c_void_p()
    rc = L.dcf_create(C.byref(g), C.byref(gas), C.byref(ctx))
    assert rc == -1 and b"at least 3" in L.dcf_last_error()
    g.n[0] = 8
    gas.gamma = 1.0
    assert L.dcf_create(C.byref(g), C.byref(gas), C.byref(ctx)) == -1
    assert L.dcf_create(None, C.byref(gas), C.byref(ctx)) == -1
    # null context on every stateful call
    assert L.dcf_rk3_step(None, None, None, None) == -1
    assert L.dcf_vjp_step(None, None, None, None, None, None, None, None) == -1
    assert L.dcf_rk3_step_keep(None, None, None, None, None) == -1
    assert L.dcf_rk3_step_noalloc(None, None, None, None, None) == -1
    assert L.dcf_rk3_step_cfl(None, None, None, 0.5, 0.0, None, None) == -1
    # batched stepping: sizes and null arguments are checked first
    nb = C.c_size_t()
    assert L.dcf_batch_table_bytes(0, C.byref(nb)) == -1
    assert L.dcf_batch_table_bytes(3, C.byref(nb)) == 0 and nb.value > 0
    assert L.dcf_batch_rk3_step(None, None, None, 1, 0.0, None, 0, None) == -1


def test_product_path_does_not_import_oracle():
    """The package must not reach the oracle (no CPU fallback)."""
    code = ("import sys; import paper_2406_19494_amd.solver, paper_2406_19494_amd.binding; "
            "assert not any(m.startswith('oracle') for m in sys.modules), "
            "[m for m in sys.modules if m.startswith('oracle')]")
    subprocess.run([sys.executable, "-c", code], cwd=ROOT, check=True)
    import re
    pkg = os.path.join(ROOT, "paper_2406_19494_amd")
    pat = re.compile(r"^\s*(from\s+oracle|import\s+oracle|#include\s+[\"<].*oracle)", re.M)
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".hpp", ".cpp", ".h")):
                text = open(os.path.join(dirpath, f)).read()
                assert not pat.search(text), f
