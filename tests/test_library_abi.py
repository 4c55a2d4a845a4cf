"""The C-ABI library builds for gfx950, loads, and exports every function that
include/lowrank.h declares (no compute calls: these run without a GPU)."""
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lowrank.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(lowrank_[a-z_A-Z0-9]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    from paper_1607_02925_amd import lowrank, build
    if not os.path.exists(lowrank.LIB_PATH):
        build.build()
    return lowrank.load_library()


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ["lowrank_plan", "lowrank_solve", "lowrank_get_schedule", "lowrank_destroy",
                 "lowrank_status_string", "lowrank_last_error", "lowrank_options_default"]:
        assert must in names


def test_every_declared_symbol_is_exported(lib):
    from paper_1607_02925_amd import lowrank
    names = declared_functions()
    out = subprocess.run(["nm", "-D", "--defined-only", lowrank.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = set(line.split()[-1] for line in out.splitlines() if line.strip())
    missing = [n for n in names if n not in exported]
    assert not missing, missing
    # and the binding declares exactly the header's surface
    assert sorted(lowrank.SIGNATURES) == names


def test_status_strings_and_defaults(lib):
    import ctypes
    from paper_1607_02925_amd import lowrank
    assert lib.lowrank_status_string(0) == b"ok"
    assert lib.lowrank_status_string(3).startswith(b"no gap")
    opt = lowrank.lr_options()
    lib.lowrank_options_default(ctypes.byref(opt))
    assert opt.est_iters == 4 and opt.max_epochs == 60 and opt.eta_scale == 1.0


def test_plan_rejects_bad_sizes_without_gpu(lib):
    """Argument validation happens before any device call."""
    import ctypes
    from paper_1607_02925_amd import lowrank
    h = ctypes.c_void_p()
    m = lowrank.lr_matrix(d=100, n=50, ld=100, nnz=0, dtype=1, layout=0, values=1,
                          col_ptr=None, row_idx=None)
    for k, p in [(3, 3), (0, 4), (5, 100), (4, 51), (2, 65)]:
        assert lib.lowrank_plan(ctypes.byref(h), ctypes.byref(m), k, p, 1e-4, None, None) == \
            lowrank.LR_EINVAL
    m.layout = 1
    assert lib.lowrank_plan(ctypes.byref(h), ctypes.byref(m), 2, 4, 1e-4, None, None) == \
        lowrank.LR_EINVAL
    m.layout, m.values = 0, None
    assert lib.lowrank_plan(ctypes.byref(h), ctypes.byref(m), 2, 4, 1e-4, None, None) == \
        lowrank.LR_EINVAL
    assert b"null" in lib.lowrank_last_error()
