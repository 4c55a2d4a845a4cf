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


def test_struct_layouts_match_the_header(tmp_path):
    """The binding's ctypes structures have the header's sizes and field
    offsets (a mismatch would let the library write past a caller's struct)."""
    import ctypes
    import shutil
    from paper_1607_02925_amd import lowrank
    cc = shutil.which("gcc")
    if cc is None:
        pytest.skip("no host C compiler")
    structs = {"lr_matrix": lowrank.lr_matrix, "lr_schedule": lowrank.lr_schedule,
               "lr_options": lowrank.lr_options, "lr_report": lowrank.lr_report,
               "lr_ticket_info": lowrank.lr_ticket_info,
               "lr_server_stats": lowrank.lr_server_stats}
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "lowrank.h"',
             "int main(void) {"]
    for name, cls in structs.items():
        lines.append('  printf("%s size %%zu\\n", sizeof(%s));' % (name, name))
        for f, _ in cls._fields_:
            cf = "lambda" if f == "lam" else f
            lines.append('  printf("%s %s %%zu\\n", offsetof(%s, %s));' % (name, f, name, cf))
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = str(tmp_path / "layout")
    subprocess.run([cc, "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", exe],
                   check=True)
    out = subprocess.run([exe], capture_output=True, text=True, check=True).stdout.split("\n")
    seen = {}
    for line in out:
        if line.strip():
            a, b, c = line.split()
            seen[(a, b)] = int(c)
    for name, cls in structs.items():
        assert seen[(name, "size")] == ctypes.sizeof(cls), name
        for f, _ in cls._fields_:
            assert seen[(name, f)] == getattr(cls, f).offset, (name, f)
