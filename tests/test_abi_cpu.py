"""The C interface without a GPU: the library loads, exports every function
that include/ibmg.h declares, agrees with the oracle on lattice sizes, sizes
its workspace, and rejects invalid descriptors before touching a device."""
import ctypes
import os
import re

import pytest

import oracle as O
from paper_1302_3663_amd import _lib as L
from paper_1302_3663_amd import ibmg, synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "ibmg.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ibb_[a-z_0-9]+)\s*\(", text)))


def test_every_declared_symbol_is_exported_and_bound():
    lib = L.load()
    names = declared_functions()
    assert len(names) >= 20
    for n in names:
        assert hasattr(lib, n), n
        assert n in L.ABI_FUNCTIONS, n


CASES = [synth.tiny_2d(), synth.tiny_2d(inout=True), synth.tiny_3d(), synth.tiny_3d(periodic_z=True)]


@pytest.mark.parametrize("ci", range(len(CASES)))
def test_lattice_sizes_match_oracle(ci):
    p = CASES[ci]["params"]
    assert ibmg.face_counts(p) == O.face_counts(p)
    assert ibmg.cell_count(p) == O.cell_count(p)
    assert ibmg.edge_counts(p) == O.edge_counts(p)
    assert len(CASES[ci]["u0"]) == sum(ibmg.face_counts(p))


def test_footprint_grows_with_precision_and_nodes():
    # without the coarse tail (whose matrix is FP64 in FP64 mode and FP32
    # when refined), the refined solver's FP32 copies add to the footprint
    p = dict(synth.tiny_3d()["params"], coarse_tail=-1)
    a = ibmg.footprint_bytes(p, 10, 10)
    b = ibmg.footprint_bytes(p, 1000, 10)
    c = ibmg.footprint_bytes(p, 10, 10, precision=L.IBB_FP32_REFINED, inner_cycles=1)
    assert 0 < a < b and a < c
    # the tail's matrix: 320 velocity and 128 pressure unknowns on level 1
    t64 = ibmg.footprint_bytes(dict(p, coarse_tail=0), 10, 10)
    t32 = ibmg.footprint_bytes(dict(p, coarse_tail=0), 10, 10, precision=L.IBB_FP32_REFINED, inner_cycles=1)
    assert t64 - a >= 8 * (320 ** 2 + 128 ** 2) and t32 - c >= 4 * (320 ** 2 + 128 ** 2)


def test_galerkin_footprint_and_flags():
    """Galerkin levels hold 235 (3D) / 31 (2D) entries per row and lattice
    point of every coarse level (FP64, plus FP32 when refined) and a second
    iterate buffer; the flag takes 0 or 1 and excludes the constant-viscosity
    form."""
    lib = L.load()
    for case, slots in ((synth.tiny_3d(), (235, 235, 235)), (synth.tiny_2d(), (31, 31))):
        p = dict(case["params"], coarse_tail=-1)
        D = p["dim"]
        nel = 0
        n = list(p["n"][:D])
        levels = 1
        while all(v % 2 == 0 and v // 2 >= 2 for v in n):
            n = [v // 2 for v in n]
            levels += 1
            pad = 1
            for v in n:
                pad *= v + 3
            nel += pad
        for prec, w in ((L.IBB_FP64, 8), (L.IBB_FP32_REFINED, 12)):
            base = ibmg.footprint_bytes(p, 10, 10, precision=prec, inner_cycles=1)
            gal = ibmg.footprint_bytes(dict(p, galerkin=1), 10, 10, precision=prec, inner_cycles=1)
            assert gal - base >= w * sum(slots) * nel
        for over in (dict(galerkin=2), dict(galerkin=1, decoupled=1, mu_max=p["mu_out"])):
            d = L.make_desc(dict(p, **over))
            nb = ctypes.c_size_t()
            assert lib.ibb_footprint_bytes(ctypes.byref(d), 10, 10, ctypes.byref(nb)) == L.IBB_EINVAL


@pytest.mark.parametrize("field,value", [("dim", 4), ("h", 0.0), ("omega", -1.0), ("nu1", -1), ("kernel", 7),
                                         ("precision", 5)])
def test_invalid_descriptor_rejected(field, value):
    lib = L.load()
    p = synth.tiny_2d()["params"]
    d = L.make_desc(p)
    setattr(d, field, value)
    n = ctypes.c_size_t()
    assert lib.ibb_footprint_bytes(ctypes.byref(d), 10, 10, ctypes.byref(n)) == L.IBB_EINVAL
    ctx = ctypes.c_void_p()
    buf = ctypes.create_string_buffer(16)
    assert lib.ibb_create(ctypes.byref(d), 10, 10, ctypes.cast(buf, ctypes.c_void_p), 16, None,
                          ctypes.byref(ctx)) == L.IBB_EINVAL
    assert not ctx.value


def test_odd_grid_and_small_workspace_rejected():
    lib = L.load()
    p = dict(synth.tiny_2d()["params"])
    p["n"] = [15, 8, 1]
    d = L.make_desc(p)
    n = ctypes.c_size_t()
    assert lib.ibb_footprint_bytes(ctypes.byref(d), 1, 1, ctypes.byref(n)) == L.IBB_EINVAL
    d = L.make_desc(synth.tiny_2d()["params"])
    ctx = ctypes.c_void_p()
    buf = ctypes.create_string_buffer(64)
    assert lib.ibb_create(ctypes.byref(d), 10, 10, ctypes.cast(buf, ctypes.c_void_p), 64, None,
                          ctypes.byref(ctx)) == L.IBB_ENOMEM


def test_status_strings():
    lib = L.load()
    for s in range(7):
        assert lib.ibb_status_string(s)


@pytest.mark.parametrize("cname,pycls", [("ibb_desc", "Desc"), ("ibb_solve_stats", "SolveStats"),
                                         ("ibb_lag_stats", "LagStats")])
def test_struct_layouts_match_header(cname, pycls, tmp_path):
    """Every field of the binding's ctypes mirror sits at the offset the C
    compiler gives it from include/ibmg.h, and the sizes agree."""
    import subprocess
    cls = getattr(L, pycls)
    names = [f[0] for f in cls._fields_]
    src = tmp_path / "layout.c"
    body = "\n".join(f'    printf("{n} %zu\\n", offsetof({cname}, {n}));' for n in names)
    src.write_text(f'#include <stdio.h>\n#include <stddef.h>\n#include "ibmg.h"\nint main(void) {{\n'
                   f'    printf("sizeof %zu\\n", sizeof({cname}));\n{body}\n    return 0;\n}}\n')
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = dict(line.split() for line in subprocess.run([str(exe)], check=True, capture_output=True,
                                                       text=True).stdout.splitlines())
    assert int(out["sizeof"]) == ctypes.sizeof(cls)
    for n in names:
        assert int(out[n]) == getattr(cls, n).offset, n


def test_decoupled_needs_constant_viscosity():
    lib = L.load()
    p = dict(synth.tiny_2d()["params"], decoupled=1)
    n = ctypes.c_size_t()
    assert p["mu_max"] != p["mu_out"]
    assert lib.ibb_footprint_bytes(ctypes.byref(L.make_desc(p)), 10, 10, ctypes.byref(n)) == L.IBB_EINVAL
    p["mu_max"] = p["mu_out"]
    assert lib.ibb_footprint_bytes(ctypes.byref(L.make_desc(p)), 10, 10, ctypes.byref(n)) == L.IBB_OK


def test_oversized_grid_rejected():
    """Array indices are formed in 32-bit arithmetic: a grid whose padded
    arrays would hold 2^31 entries or more is refused."""
    lib = L.load()
    p = dict(synth.tiny_3d()["params"])
    n = ctypes.c_size_t()
    p["n"] = [1290, 1290, 1290]
    assert lib.ibb_footprint_bytes(ctypes.byref(L.make_desc(p)), 1, 1, ctypes.byref(n)) == L.IBB_EINVAL
    p["n"] = [1024, 1024, 1024]
    assert lib.ibb_footprint_bytes(ctypes.byref(L.make_desc(p)), 1, 1, ctypes.byref(n)) == L.IBB_OK

