"""Host-side logic of the library that needs no GPU: the server's HBM arena
(first-fit allocator, checked against a brute-force occupancy map), workspace
sizing and the server's argument checks."""
import ctypes
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1607_02925_amd", "csrc")


def test_arena_first_fit_against_brute_force(tmp_path):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("no host C++ compiler")
    exe = str(tmp_path / "arena_check")
    subprocess.run([gxx, "-O1", "-std=c++17", "-Wall", "-Werror", "-I", CSRC,
                    os.path.join(ROOT, "tests", "arena_check.cpp"), "-o", exe], check=True)
    r = subprocess.run([exe], capture_output=True, text=True)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "arena ok" in r.stdout


@pytest.fixture(scope="module")
def lib():
    from paper_1607_02925_amd import lowrank, build
    if not os.path.exists(lowrank.LIB_PATH):
        build.build()
    return lowrank.load_library()


def _mat(d, n, dtype=1):
    from paper_1607_02925_amd import lowrank
    return lowrank.lr_matrix(d=d, n=n, ld=d, nnz=0, dtype=dtype, layout=0, values=1,
                             col_ptr=None, row_idx=None)


def test_plan_bytes(lib):
    """Workspace is dominated by X^T W (n x pad16(p) FP64), the sampling table
    (16 bytes per column) and the minibatch staging; it grows with n and p."""
    from paper_1607_02925_amd import lowrank
    out = ctypes.c_size_t()
    m = _mat(2048, 200000)
    assert lib.lowrank_plan_bytes(ctypes.byref(m), 10, 20, None, ctypes.byref(out)) == 0
    b = out.value
    assert b % 256 == 0
    assert b >= 200000 * 32 * 8 + 200000 * 16
    assert b < 200000 * 32 * 8 + 200000 * 16 + 2 ** 28
    m2 = _mat(2048, 400000)
    assert lib.lowrank_plan_bytes(ctypes.byref(m2), 10, 20, None, ctypes.byref(out)) == 0
    assert out.value > b
    assert lib.lowrank_plan_bytes(ctypes.byref(m), 10, 40, None, ctypes.byref(out)) == 0
    assert out.value > b
    assert lib.lowrank_plan_bytes(ctypes.byref(m), 20, 20, None, ctypes.byref(out)) == \
        lowrank.LR_EINVAL


def test_server_argument_checks_without_gpu(lib):
    """Checks that happen before any device call."""
    from paper_1607_02925_amd import lowrank
    h = ctypes.c_void_p()
    assert lib.lowrank_server_create(ctypes.byref(h), 1 << 30, 0) == lowrank.LR_EINVAL
    assert lib.lowrank_server_create(ctypes.byref(h), 1 << 30, lowrank.LR_MAX_SLOTS + 1) == \
        lowrank.LR_EINVAL
    assert lib.lowrank_server_create(ctypes.byref(h), 16, 1) == lowrank.LR_EINVAL
    assert lib.lowrank_server_create(None, 1 << 30, 1) == lowrank.LR_EINVAL
    t = ctypes.c_uint64()
    m = _mat(100, 50)
    assert lib.lowrank_submit(None, ctypes.byref(m), 2, 4, 1e-4, None, None, None,
                              ctypes.byref(t)) == lowrank.LR_EINVAL
    assert lib.lowrank_poll(None, 1, None, None) == lowrank.LR_EINVAL
    assert lib.lowrank_wait(None, 1, None, None) == lowrank.LR_EINVAL
    lib.lowrank_server_destroy(None)


def test_precision_option_checks(lib):
    """The BF16 matrix-core steps are offered for dense BF16 X only; the check
    happens before any device call."""
    from paper_1607_02925_amd import lowrank
    h = ctypes.c_void_p()
    opt = lowrank.lr_options()
    lib.lowrank_options_default(ctypes.byref(opt))
    assert opt.precision == lowrank.LR_PREC_F64
    opt.precision = lowrank.LR_PREC_BF16_STEPS
    m = _mat(100, 500, dtype=lowrank.LR_F32)
    assert lib.lowrank_plan(ctypes.byref(h), ctypes.byref(m), 2, 4, 1e-4, ctypes.byref(opt),
                            None) == lowrank.LR_EINVAL
    assert b"BF16" in lib.lowrank_last_error()
    opt.precision = 7
    m = _mat(100, 500, dtype=lowrank.LR_BF16)
    assert lib.lowrank_plan(ctypes.byref(h), ctypes.byref(m), 2, 4, 1e-4, ctypes.byref(opt),
                            None) == lowrank.LR_EINVAL
    # the split copies add to the workspace
    out0, out1 = ctypes.c_size_t(), ctypes.c_size_t()
    opt.precision = lowrank.LR_PREC_F64
    assert lib.lowrank_plan_bytes(ctypes.byref(m), 2, 4, ctypes.byref(opt), ctypes.byref(out0)) == 0
    opt.precision = lowrank.LR_PREC_BF16_STEPS
    assert lib.lowrank_plan_bytes(ctypes.byref(m), 2, 4, ctypes.byref(opt), ctypes.byref(out1)) == 0
    assert out1.value > out0.value


def test_f32_steps_option_checks(lib):
    """The FP32 matrix-core steps take dense FP32 or BF16 X; their FP32 tile
    copies (pad16(d) x 16 floats and two pad16(b_max) x 16 partials here) add
    to the workspace."""
    from paper_1607_02925_amd import lowrank
    h = ctypes.c_void_p()
    opt = lowrank.lr_options()
    lib.lowrank_options_default(ctypes.byref(opt))
    opt.precision = lowrank.LR_PREC_F32_STEPS
    m = _mat(100, 500, dtype=lowrank.LR_F64)
    assert lib.lowrank_plan(ctypes.byref(h), ctypes.byref(m), 2, 4, 1e-4, ctypes.byref(opt),
                            None) == lowrank.LR_EINVAL
    assert b"FP32 matrix-core" in lib.lowrank_last_error()
    opt.adaptive = 1
    m = _mat(100, 500, dtype=lowrank.LR_F32)
    assert lib.lowrank_plan(ctypes.byref(h), ctypes.byref(m), 2, 4, 1e-4, ctypes.byref(opt),
                            None) == lowrank.LR_EINVAL
    opt.adaptive = 0
    for dt in (lowrank.LR_F32, lowrank.LR_BF16):
        m = _mat(100, 500, dtype=dt)
        out0, out2 = ctypes.c_size_t(), ctypes.c_size_t()
        opt.precision = lowrank.LR_PREC_F64
        assert lib.lowrank_plan_bytes(ctypes.byref(m), 2, 4, ctypes.byref(opt),
                                      ctypes.byref(out0)) == 0
        opt.precision = lowrank.LR_PREC_F32_STEPS
        assert lib.lowrank_plan_bytes(ctypes.byref(m), 2, 4, ctypes.byref(opt),
                                      ctypes.byref(out2)) == 0
        # 112 x 16 and 4 x 512 x 16 floats, each in place of an empty 256-byte slot
        assert out2.value - out0.value == (112 * 16 * 4 - 256) + (2 * 512 * 16 * 4 - 256)


def test_accel_option_checks(lib):
    """accel takes 0 or 1 and does not combine with a replay schedule; the
    momentum buffers add to the workspace."""
    from paper_1607_02925_amd import lowrank
    h = ctypes.c_void_p()
    opt = lowrank.lr_options()
    lib.lowrank_options_default(ctypes.byref(opt))
    assert opt.accel == 0
    m = _mat(100, 500)
    opt.accel = 2
    assert lib.lowrank_plan(ctypes.byref(h), ctypes.byref(m), 2, 4, 1e-4, ctypes.byref(opt),
                            None) == lowrank.LR_EINVAL
    assert b"accel" in lib.lowrank_last_error()
    opt.accel = 1
    ep = (ctypes.c_int32 * 1)(1)
    opt.replay = ctypes.pointer(lowrank.lr_schedule(lam=1.0, mu_hat=0.1, eta=1e-3, m=4, b=64,
                                                    first_solve=0, outer=1, n_epochs=1,
                                                    epochs=ep))
    assert lib.lowrank_plan(ctypes.byref(h), ctypes.byref(m), 2, 4, 1e-4, ctypes.byref(opt),
                            None) == lowrank.LR_EINVAL
    assert b"replay" in lib.lowrank_last_error()
    opt.replay = None
    out0, out1 = ctypes.c_size_t(), ctypes.c_size_t()
    opt.accel = 0
    assert lib.lowrank_plan_bytes(ctypes.byref(m), 2, 4, ctypes.byref(opt), ctypes.byref(out0)) == 0
    opt.accel = 1
    assert lib.lowrank_plan_bytes(ctypes.byref(m), 2, 4, ctypes.byref(opt), ctypes.byref(out1)) == 0
    # four d x p FP64 buffers; an unused buffer still holds one 256-byte slot
    assert out1.value >= out0.value + 4 * (100 * 4 * 8 - 256)
