"""The ghost-image writer of the solver kernels (common.h: write_images,
which takes a short path when a position has at most one image per axis)
stores exactly what the general form (write_images_any, every combination of
each axis's position and images) does.  Checked on the host for every
lattice (cell or vertex centred per axis), role, boundary kind and position,
on 2D and 3D lattices of one to five points a side."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


@pytest.mark.skipif(shutil.which("hipcc") is None, reason="needs hipcc to build the host check")
def test_compact_image_writer_matches_general(tmp_path):
    exe = str(tmp_path / "images_check")
    subprocess.check_call(["hipcc", "--offload-arch=gfx950", "-O1", "-std=c++17",
                           "-I", os.path.join(ROOT, "paper_1302_3663_amd", "csrc"),
                           "-I", os.path.join(ROOT, "include"),
                           os.path.join(HERE, "images_check.cpp"), "-o", exe])
    out = subprocess.run([exe], capture_output=True, text=True, timeout=600)
    print(out.stdout)
    assert out.returncode == 0 and " 0 mismatches" in out.stdout, out.stdout + out.stderr
