"""CPU-side checks of the native library (no GPU needed).

* every function declared in include/bzq.h is exported by libbzq.so;
* argument errors are reported before any device work (status codes, NULL
  plan, message text);
* the device FFT building blocks and the plan's quadrature rules, compiled
  for the host, against direct long-double evaluation and closed forms.
"""
import ctypes
import os
import re
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2004_11239_amd", "libbzq.so")
CSRC = os.path.join(ROOT, "paper_2004_11239_amd", "csrc")
HIPCC = "/opt/rocm/bin/hipcc"


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        if not os.path.exists(HIPCC):
            pytest.skip("library not built and hipcc not available")
        from paper_2004_11239_amd.build import build
        build(verbose=False)
    return ctypes.CDLL(LIB)


def declared_functions():
    text = open(os.path.join(ROOT, "include", "bzq.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(bzq_\w+)\s*\(", text)))


def test_header_symbols_exported(lib):
    names = declared_functions()
    assert len(names) >= 15
    for n in names:
        assert hasattr(lib, n), n
    # every internal symbol resolves inside the library (a lazily bound one
    # would only fail at its first call)
    nm = shutil.which("nm")
    if nm:
        r = subprocess.run([nm, "-D", "--undefined-only", LIB], capture_output=True, text=True)
        assert r.returncode == 0
        assert "bzq" not in r.stdout, r.stdout


def test_argument_validation_without_device(lib):
    f = lib.bzq_plan_create
    f.argtypes = [ctypes.POINTER(ctypes.c_void_p), ctypes.c_int, ctypes.c_double, ctypes.c_double,
                  ctypes.c_double, ctypes.c_double, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                  ctypes.c_int, ctypes.c_void_p]
    f.restype = ctypes.c_int
    lib.bzq_last_error.restype = ctypes.c_char_p
    lib.bzq_status_string.restype = ctypes.c_char_p
    h = ctypes.c_void_p(1234)
    cases = [
        ((15, 8.0, 4.0, 0.0, 0.5, 16, 38, 0), 1),     # odd N
        ((4, 8.0, 4.0, 0.0, 0.5, 16, 38, 0), 1),      # N < 8
        ((16, -1.0, 4.0, 0.0, 0.5, 16, 38, 0), 1),    # L <= 0
        ((16, 8.0, 0.0, 0.0, 0.5, 16, 38, 0), 1),     # R <= 0
        ((16, 8.0, 4.0, -3.5, 0.5, 16, 38, 0), 1),    # gamma out of range
        ((16, 8.0, 4.0, 0.0, 1.0, 16, 38, 0), 1),     # s = 1 (nu = 2)
        ((16, 8.0, 4.0, 0.0, -0.1, 16, 38, 0), 1),    # s < 0
        ((16, 8.0, 4.0, 0.0, 0.5, 0, 38, 0), 1),      # N_rho < 1
        ((16, 8.0, 4.0, 0.0, 0.5, 16, 37, 0), 1),     # no Lebedev rule of size 37
        ((16, 8.0, 4.0, 0.0, 0.5, 16, 38, 7), 1),     # unknown precision
        ((12, 8.0, 4.0, 0.0, 0.5, 16, 38, 0), 4),     # valid but no FFT schedule
        ((96, 8.0, 4.0, 0.0, 0.5, 16, 38, 0), 4),
        ((256, 8.0, 4.0, 0.0, 0.5, 16, 38, 0), 4),
    ]
    # kernel selector (BZQ_KERNEL_POWER = 0, BZQ_KERNEL_CUTOFF_CONST = 1)
    cases = [(a + (0,), c) for a, c in cases] + [
        ((12, 8.0, 4.0, 0.0, 2.0, 16, 38, 0, 1), 4),  # cutoff kernel: s ignored, then no FFT schedule
        ((12, 8.0, 4.0, 0.0, 2.0, 16, 38, 0, 0), 1),  # the same s for the power kernel: invalid
        ((16, 8.0, 4.0, 0.0, 0.5, 16, 38, 0, 2), 1),  # the general selector is not taken here
        ((16, 8.0, 4.0, 0.0, 0.5, 16, 38, 0, 7), 1),  # unknown selector
    ]
    for args, code in cases:
        h.value = 1234
        assert f(ctypes.byref(h), *args, None) == code, args
        assert h.value is None
        assert len(lib.bzq_last_error()) > 0
    assert lib.bzq_status_string(1) == b"invalid argument"
    rb = lib.bzq_request_device_bytes
    rb.restype = ctypes.c_size_t
    rb.argtypes = [ctypes.c_int, ctypes.c_int]
    # state (f_hat, Q_hat) plus a workspace (whose chunk of pairs is capped in
    # bytes, so both precisions come out near the cap), growing with N
    assert rb(32, 1) > 2 * 32 ** 3 * 16 and rb(32, 0) > 2 * 32 ** 3 * 16
    assert rb(64, 1) > rb(32, 1)
    assert rb(7, 0) == 0 and rb(32, 5) == 0
    lib.bzq_collision.argtypes = [ctypes.c_void_p] * 4
    assert lib.bzq_collision(None, None, None, None) == 1
    lib.bzq_plan_destroy.argtypes = [ctypes.c_void_p]
    assert lib.bzq_plan_destroy(None) == 0


def _compile_and_run(src, extra, tmp_path):
    if not os.path.exists(HIPCC):
        pytest.skip("hipcc not available")
    exe = str(tmp_path / "check")
    cmd = [HIPCC, "-O1", "-std=c++17", "-x", "hip", "--offload-host-only", f"-I{CSRC}",
           os.path.join(ROOT, "tests", "native", src)] + extra + ["-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    r = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    print(r.stdout[-3000:])
    return r


def test_fft_building_blocks_on_host(tmp_path):
    r = _compile_and_run("fft_host_check.cpp", [], tmp_path)
    assert r.returncode == 0, r.stdout


def test_xcd_launch_shapes_on_host(tmp_path):
    r = _compile_and_run("xcd_host_check.cpp", [], tmp_path)
    assert r.returncode == 0, r.stdout


def test_plan_quadrature_on_host(tmp_path):
    r = _compile_and_run("quad_host_check.cpp", [os.path.join(CSRC, "quadrature.cpp")], tmp_path)
    assert r.returncode == 0, r.stdout


def test_plan2d_argument_validation_without_device(lib):
    f = lib.bzq_plan2d_create
    d, i = ctypes.c_double, ctypes.c_int
    f.argtypes = [ctypes.POINTER(ctypes.c_void_p), i, d, d, d, d, d, d, i, i, i, i, ctypes.c_void_p]
    f.restype = ctypes.c_int
    c3 = 1.0 / (8.0 * 3.141592653589793)
    ok = (16, 8.0, 4.0, 0.0, c3, 0.0, 0.0, 64, 8, 16, 0)
    cases = [
        ((15,) + ok[1:], 1),                                  # odd N
        (ok[:2] + (0.0,) + ok[3:], 1),                        # R <= 0
        (ok[:4] + (-1.0,) + ok[5:], 1),                       # c <= 0
        (ok[:5] + (0.5,) + ok[6:], 1),                        # s >= 1/2 (F2D needs s < 1/2)
        (ok[:5] + (-1.5,) + ok[6:], 1),                       # s < -1
        (ok[:6] + (0.5,) + ok[7:], 1),                        # r >= 1/2
        (ok[:7] + (4,) + ok[8:], 1),                          # too few Jacobi nodes
        (ok[:9] + (15,) + ok[10:], 1),                        # odd N_sigma
        (ok[:10] + (3,), 1),                                  # unknown precision
        ((12,) + ok[1:], 4),                                  # valid, no FFT schedule
        ((128,) + ok[1:], 4),
    ]
    h = ctypes.c_void_p()
    for args, code in cases:
        h.value = 1234
        assert f(ctypes.byref(h), *args, None) == code, args
        assert h.value is None
    lib.bzq_collision2d.argtypes = [ctypes.c_void_p] * 4
    assert lib.bzq_collision2d(None, None, None, None) == 1
    lib.bzq_plan2d_destroy.argtypes = [ctypes.c_void_p]
    assert lib.bzq_plan2d_destroy(None) == 0


def test_weight_series_on_host(tmp_path):
    r = _compile_and_run("fh_host_check.cpp", [os.path.join(CSRC, "funk_hecke.cpp"),
                                               os.path.join(CSRC, "quadrature.cpp")], tmp_path)
    assert r.returncode == 0, r.stdout


def test_otf_plan_limits_without_device(lib):
    """bzq_plan_create_otf validates like bzq_plan_create_general and refuses,
    before any device work, a geometry whose largest a|k| needs more than 64
    even terms of the weight series."""
    f = lib.bzq_plan_create_otf
    d, i = ctypes.c_double, ctypes.c_int
    f.argtypes = [ctypes.POINTER(ctypes.c_void_p), i, d, d, d, i, d, d, d, i, i, i, ctypes.c_void_p]
    f.restype = ctypes.c_int
    c = 0.02
    h = ctypes.c_void_p()
    # selector 0: the power kernel of order b_s (b_c, b_r ignored); 2: (b_c, b_s, b_r)
    cases = [
        ((15, 8.0, 4.0, 0.0, 0, 0.0, 0.5, 0.0, 16, 38, 0), 1),     # odd N
        ((16, 8.0, 4.0, 0.0, 0, 0.0, 1.0, 0.0, 16, 38, 0), 1),     # s = 1
        ((16, 8.0, 4.0, 0.0, 2, -1.0, 0.5, 0.0, 16, 38, 0), 1),    # general kernel with c <= 0
        ((16, 8.0, 4.0, 0.0, 5, c, 0.5, 0.0, 16, 38, 0), 1),       # unknown selector
        ((16, 8.0, 4.0, 0.0, 0, 0.0, 0.5, 0.0, 16, 37, 0), 1),     # no Lebedev rule of size 37
        ((12, 8.0, 4.0, 0.0, 0, -5.0, 0.5, 9.0, 16, 38, 0), 4),    # b_c, b_r ignored; no FFT schedule
        ((12, 8.0, 4.0, 0.0, 1, 0.0, 7.0, 0.0, 16, 38, 0), 4),     # cutoff: all ignored
        ((12, 8.0, 4.0, 0.0, 2, c, 0.5, 0.0, 16, 38, 0), 4),       # no FFT schedule
        ((64, 2.0, 40.0, 0.0, 0, 0.0, 0.5, 0.0, 8, 38, 0), 4),     # a|k| ~ 840: series too long
    ]
    for args, code in cases:
        h.value = 1234
        assert f(ctypes.byref(h), *args, None) == code, args
        assert h.value is None


def test_chunk_cap_bounds_the_workspace(lib, monkeypatch):
    """The pipeline's chunk of pairs is sized so that its intermediates stay
    below BZQ_CHUNK_MB (default 2048 MB): at 64^3 FP32 one pair-two's A and B
    take 96 x (3984 + 2 x 1984) x 8 bytes, so halving the cap takes about
    1 GB (175 or 176 pair-twos) off the device bytes of a request."""
    rb = lib.bzq_request_device_bytes
    rb.restype = ctypes.c_size_t
    rb.argtypes = [ctypes.c_int, ctypes.c_int]
    monkeypatch.delenv("BZQ_CHUNK_MB", raising=False)
    default = rb(64, 1)
    monkeypatch.setenv("BZQ_CHUNK_MB", "2048")
    assert rb(64, 1) == default
    monkeypatch.setenv("BZQ_CHUNK_MB", "1024")
    half = rb(64, 1)
    per_pt = 96 * (3984 + 2 * 1984) * 8
    assert 175 * per_pt <= default - half <= 177 * per_pt, (default, half)
