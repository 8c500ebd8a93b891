"""The C-ABI library loads, exports every entry point include/tqr.h declares,
and rejects illegal arguments synchronously (no device work).  CPU only."""
import ctypes
import os
import re

import pytest

from conftest import ROOT

HEADER = os.path.join(ROOT, "include", "tqr.h")
LIB = os.path.join(ROOT, "paper_0707_3548_amd", "libtqr.so")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(tqr_[a-z_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.skip("libtqr.so not built")
    from paper_0707_3548_amd import tqr
    return tqr.lib()


def test_every_declared_symbol_is_exported(lib):
    names = declared_functions()
    assert "tqr_factor" in names and "tqr_solve_ls" in names and "tqr_apply_qt" in names
    for name in names:
        assert hasattr(lib, name), f"{name} declared in tqr.h but not exported"


def test_sizes(lib):
    assert lib.tqr_t_elems(512, 512, 64, 16) == 8 * 8 * 16 * 64
    assert lib.tqr_t_elems(100, 70, 32, 16) == 4 * 3 * 16 * 32
    assert lib.tqr_t_elems(10, 20, 32, 16) == -1          # m < n
    assert lib.tqr_t_elems(64, 64, 48, 16) == -1          # unsupported b
    assert lib.tqr_t_elems(64, 64, 256, 64) == -1         # panel too large for the chip
    assert lib.tqr_workspace_bytes(512, 512, 0, 64, 16) >= 512 * 512 * 8
    assert lib.tqr_workspace_bytes(512, 512, 3, 64, 16) > lib.tqr_workspace_bytes(512, 512, 0, 64, 16)


@pytest.mark.parametrize("args,code", [
    ((-1, 0), -1), ((5, 6), -1), ((5, -1), -2),
])
def test_factor_rejects_bad_shapes(lib, args, code):
    m, n = args
    rc = lib.tqr_factor(m, n, None, max(1, m), 64, 16, None, None, 0, None)
    assert rc == code
    assert lib.tqr_last_error_string()


def test_factor_argument_order(lib):
    fake = ctypes.c_void_p(256)  # never dereferenced: validation fails first
    assert lib.tqr_factor(8, 8, None, 8, 64, 16, fake, fake, 1 << 30, None) == -3
    assert lib.tqr_factor(8, 8, fake, 4, 64, 16, fake, fake, 1 << 30, None) == -4
    assert lib.tqr_factor(8, 8, fake, 8, 48, 16, fake, fake, 1 << 30, None) == -5
    assert lib.tqr_factor(8, 8, fake, 8, 64, 24, fake, fake, 1 << 30, None) == -6
    assert lib.tqr_factor(8, 8, fake, 8, 64, 16, None, fake, 1 << 30, None) == -7
    assert lib.tqr_factor(8, 8, fake, 8, 64, 16, fake, None, 1 << 30, None) == -8
    assert lib.tqr_factor(8, 8, fake, 8, 64, 16, fake, fake, 16, None) == -9
    # empty problems return at once
    assert lib.tqr_factor(0, 0, None, 1, 64, 16, None, None, 0, None) == 0
    assert lib.tqr_factor(5, 0, None, 5, 64, 16, None, None, 0, None) == 0


def test_apply_and_solve_argument_checks(lib):
    fake = ctypes.c_void_p(256)
    big = 1 << 40
    assert lib.tqr_apply_qt(8, 8, -1, fake, 8, fake, 64, 16, fake, 8, fake, big, None) == -3
    assert lib.tqr_apply_qt(8, 8, 1, fake, 8, fake, 64, 16, fake, 4, fake, big, None) == -10
    assert lib.tqr_apply_q(8, 8, 1, fake, 8, None, 64, 16, fake, 8, fake, big, None) == -6
    assert lib.tqr_solve_ls(8, 8, 1, fake, 8, fake, 8, 64, 16, fake, fake, big, None, None) == -13
    assert lib.tqr_solve_ls(8, 9, 1, fake, 8, fake, 8, 64, 16, fake, fake, big, fake, None) == -1


def test_form_q_argument_checks(lib):
    fake = ctypes.c_void_p(256)
    big = 1 << 40
    assert lib.tqr_form_q(8, 9, fake, 8, fake, 64, 16, fake, 8, fake, big, None) == -1
    assert lib.tqr_form_q(8, 8, None, 8, fake, 64, 16, fake, 8, fake, big, None) == -3
    assert lib.tqr_form_q(8, 8, fake, 4, fake, 64, 16, fake, 8, fake, big, None) == -4
    assert lib.tqr_form_q(8, 8, fake, 8, None, 64, 16, fake, 8, fake, big, None) == -5
    assert lib.tqr_form_q(8, 8, fake, 8, fake, 48, 16, fake, 8, fake, big, None) == -6
    assert lib.tqr_form_q(8, 8, fake, 8, fake, 64, 24, fake, 8, fake, big, None) == -7
    assert lib.tqr_form_q(8, 8, fake, 8, fake, 64, 16, None, 8, fake, big, None) == -8
    assert lib.tqr_form_q(8, 8, fake, 8, fake, 64, 16, fake, 7, fake, big, None) == -9
    assert lib.tqr_form_q(8, 8, fake, 8, fake, 64, 16, fake, 8, None, big, None) == -10
    assert lib.tqr_form_q(8, 8, fake, 8, fake, 64, 16, fake, 8, fake, 16, None) == -11
    assert lib.tqr_form_q(0, 0, None, 1, None, 64, 16, None, 1, None, 0, None) == 0


def test_solve_ls_ex_option_checks(lib):
    from paper_0707_3548_amd import tqr
    fake = ctypes.c_void_p(256)
    big = 1 << 40
    bad = tqr.Options(ctypes.sizeof(tqr.Options) - 8, 0, 0, 0, None, None, None, 0, None, None)
    assert lib.tqr_solve_ls_ex(8, 8, 1, fake, 8, fake, 8, 64, 16, fake, fake, big, fake, None, ctypes.byref(bad)) == -15
    serial = tqr.Options(ctypes.sizeof(tqr.Options), 0, tqr.MODE_SERIAL, 0, None, None, None, 0, None, None)
    assert lib.tqr_solve_ls_ex(8, 8, 1, fake, 8, fake, 8, 64, 16, fake, fake, big, fake, None, ctypes.byref(serial)) == -15
    # earlier arguments are reported first
    assert lib.tqr_solve_ls_ex(8, 9, 1, fake, 8, fake, 8, 64, 16, fake, fake, big, fake, None, ctypes.byref(bad)) == -1


def test_noalloc_argument_checks_and_scratch_limit(lib):
    """tqr_factor_noalloc validates like tqr_factor and rejects, before any
    device call, a problem whose workspace exceeds the fixed scratch."""
    from paper_0707_3548_amd import tqr
    fake = ctypes.c_void_p(256)  # never dereferenced: validation fails first
    assert lib.tqr_factor_noalloc(5, 6, fake, 5, 64, 16, fake, None) == -1
    assert lib.tqr_factor_noalloc(8, 8, None, 8, 64, 16, fake, None) == -3
    assert lib.tqr_factor_noalloc(8, 8, fake, 4, 64, 16, fake, None) == -4
    assert lib.tqr_factor_noalloc(8, 8, fake, 8, 48, 16, fake, None) == -5
    assert lib.tqr_factor_noalloc(8, 8, fake, 8, 64, 24, fake, None) == -6
    assert lib.tqr_factor_noalloc(8, 8, fake, 8, 64, 16, None, None) == -7
    assert lib.tqr_factor_noalloc(0, 0, None, 1, 64, 16, None, None) == 0
    assert lib.tqr_workspace_bytes(3840, 3840, 0, 256, 16) <= tqr.NOALLOC_SCRATCH_BYTES
    assert lib.tqr_workspace_bytes(4096, 4096, 0, 256, 16) > tqr.NOALLOC_SCRATCH_BYTES
    assert lib.tqr_factor_noalloc(4096, 4096, fake, 4096, 256, 16, fake, None) == tqr.TQR_ESCRATCH
    assert b"scratch" in lib.tqr_last_error_string()


def test_noalloc_scratch_constant_matches_the_header():
    src = open(HEADER).read()
    m = re.search(r"#define TQR_NOALLOC_SCRATCH_BYTES \((\d+)ll << (\d+)\)", src)
    assert m
    from paper_0707_3548_amd import tqr
    assert tqr.NOALLOC_SCRATCH_BYTES == int(m.group(1)) << int(m.group(2))
