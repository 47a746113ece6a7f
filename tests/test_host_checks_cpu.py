"""Host checks of integer helpers the solver kernels share, built with hipcc
and run on the CPU:
- the ghost-image writer (common.h: write_images, which takes a short path
  when a position has at most one image per axis) stores exactly what the
  general form (write_images_any, every combination of each axis's position
  and images) does, for every lattice (cell or vertex centred per axis),
  role, boundary kind and position on 2D and 3D lattices of one to five
  points a side;
- division through one multiply (kernels.h: make_div, div_by) equals
  integer division, exhaustively for small divisors and dividends and at
  random over the whole range, and the point and colour decodes that use it
  give the points of the plain decodes for every box up to 40 x 12 x 6."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


def run_check(tmp_path, name):
    exe = str(tmp_path / name)
    subprocess.check_call(["hipcc", "--offload-arch=gfx950", "-O1", "-std=c++17",
                           "-I", os.path.join(ROOT, "paper_1302_3663_amd", "csrc"),
                           "-I", os.path.join(ROOT, "include"),
                           os.path.join(HERE, name + ".cpp"), "-o", exe])
    out = subprocess.run([exe], capture_output=True, text=True, timeout=600)
    print(out.stdout)
    assert out.returncode == 0 and " 0 mismatches" in out.stdout, out.stdout + out.stderr


needs_hipcc = pytest.mark.skipif(shutil.which("hipcc") is None, reason="needs hipcc to build the host check")


@needs_hipcc
def test_compact_image_writer_matches_general(tmp_path):
    run_check(tmp_path, "images_check")


@needs_hipcc
def test_division_by_multiply_and_decodes(tmp_path):
    run_check(tmp_path, "div_check")
