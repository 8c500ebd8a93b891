"""The strip updates' LDS operand reads stay inside the buffers they are
meant to read, for every instantiated (tile_b, inner_ib), both directions,
both forms, every inner block and every lane (CPU): the offsets come from the
kernels' own header (csrc/tqr_offsets.h), compiled into a host program."""
import os
import subprocess

import pytest

from conftest import ROOT

CSRC = os.path.join(ROOT, "paper_0707_3548_amd", "csrc")
SRC = os.path.join(ROOT, "tests", "check_lds_offsets.cpp")


def _build(tmp_path, extra=()):
    exe = str(tmp_path / "check_lds_offsets")
    subprocess.check_call(["g++", "-std=c++17", "-O1", "-I", CSRC, *extra, SRC, "-o", exe])
    return exe


def test_every_strip_update_read_is_in_bounds(tmp_path):
    out = subprocess.run([_build(tmp_path)], capture_output=True, text=True)
    assert out.returncode == 0, out.stdout + out.stderr
    assert out.stdout.startswith("OK")
    assert int(out.stdout.split()[1]) > 1_000_000


def test_the_check_catches_a_prefetch_one_block_past_the_end(tmp_path):
    """A checker that also enumerated row block B/16 (the unguarded prefetch
    of the fault once seen) must report it: the check is not vacuous."""
    src = open(SRC).read().replace("rb < B / 16; ++rb", "rb <= B / 16; ++rb")
    bad = tmp_path / "check_bad.cpp"
    bad.write_text(src)
    exe = str(tmp_path / "check_bad")
    subprocess.check_call(["g++", "-std=c++17", "-O1", "-I", CSRC, str(bad), "-o", exe])
    out = subprocess.run([exe], capture_output=True, text=True)
    assert out.returncode == 1 and "VIOLATION" in out.stdout
