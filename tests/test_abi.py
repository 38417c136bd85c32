"""The C ABI without a GPU: libcmlb.so loads, exports every function that
include/cmlb.h declares, the parameter struct layout agrees between C and the
binding, and argument validation happens before any device call."""
import ctypes
import os
import re
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "cmlb.h")
HEADER3 = os.path.join(ROOT, "include", "cmlb3.h")


@pytest.fixture(scope="module")
def lib():
    from paper_2504_09024_amd import build, cmlb
    if build.is_stale():
        build.build()
    return cmlb.load()


def declared_functions(header=HEADER, prefix="cmlb_"):
    text = open(header).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(" + prefix + r"[a-z_0-9]+)\s*\(", text)))


def test_header_declares_the_binding_names():
    from paper_2504_09024_amd import cmlb
    assert declared_functions() == sorted(cmlb.EXPORTS)


def test_header3_declares_the_binding_names():
    from paper_2504_09024_amd import cmlb
    assert declared_functions(HEADER3, "cmlb3_") == sorted(cmlb.EXPORTS3)


def test_library_exports_every_declared_symbol(lib):
    names = declared_functions() + declared_functions(HEADER3, "cmlb3_")
    for name in names:
        assert hasattr(lib, name), name
    out = subprocess.run(["nm", "-D", "--defined-only", lib._name], capture_output=True,
                         text=True, check=True).stdout
    exported = set(re.findall(r"\s(cmlb3?_\w+)$", out, flags=re.M))
    assert set(names) <= exported


def test_param_struct_layout_matches_c():
    from paper_2504_09024_amd import cmlb
    fields = [f for f, _ in cmlb.SimParams._fields_]
    src = ['#include <stdio.h>', '#include <stddef.h>', f'#include "{HEADER}"', "int main(void){",
           'printf("%zu\\n", sizeof(cmlb_sim_params));']
    src += [f'printf("%zu\\n", offsetof(cmlb_sim_params, {f}));' for f in fields]
    src += ["return 0;}"]
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "t.c")
        exe = os.path.join(d, "t")
        open(c, "w").write("\n".join(src))
        subprocess.run(["gcc", c, "-o", exe], check=True)
        vals = [int(v) for v in subprocess.run([exe], capture_output=True, text=True,
                                               check=True).stdout.split()]
    assert vals[0] == ctypes.sizeof(cmlb.SimParams)
    for f, off in zip(fields, vals[1:]):
        assert getattr(cmlb.SimParams, f).offset == off, f


def test_param3_struct_layout_matches_c():
    from paper_2504_09024_amd import cmlb
    fields = [f for f, _ in cmlb.SimParams3._fields_]
    src = ['#include <stdio.h>', '#include <stddef.h>', f'#include "{HEADER3}"', "int main(void){",
           'printf("%zu\\n", sizeof(cmlb3_sim_params));']
    src += [f'printf("%zu\\n", offsetof(cmlb3_sim_params, {f}));' for f in fields]
    src += ["return 0;}"]
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "t.c")
        exe = os.path.join(d, "t")
        open(c, "w").write("\n".join(src))
        subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), c, "-o", exe], check=True)
        vals = [int(v) for v in subprocess.run([exe], capture_output=True, text=True,
                                               check=True).stdout.split()]
    assert vals[0] == ctypes.sizeof(cmlb.SimParams3)
    for f, off in zip(fields, vals[1:]):
        assert getattr(cmlb.SimParams3, f).offset == off, f


def test_validation3_before_device(lib):
    from paper_2504_09024_amd import cmlb
    from paper_2504_09024_amd import workloads as W
    good = dict(W.params(nx=32, ny=16), nz=8)

    def create(plist, prec=0):
        arr = (cmlb.SimParams3 * max(len(plist), 1))(*[cmlb.make_params3(p) for p in plist])
        h = ctypes.c_void_p()
        return lib.cmlb3_create(arr, len(plist), prec, None, ctypes.byref(h))

    assert create([]) == cmlb.EINVAL
    assert create([dict(good, nz=0)]) == cmlb.EINVAL
    assert create([dict(good, ny=2)]) == cmlb.EINVAL
    assert create([good], prec=5) == cmlb.EINVAL
    assert create([good, dict(good, flow="coupled")]) == cmlb.EINVAL
    assert create([dict(good, flow="coupled", omega_zeta=2.5)]) == cmlb.EUNSTABLE
    # a lattice beyond the 32-bit buffer range
    assert create([dict(good, nx=1024, ny=1024, nz=128)], prec=0) == cmlb.EINVAL
    assert lib.cmlb3_step(None, 1) == cmlb.EINVAL
    assert lib.cmlb3_step_count(None) == -1
    assert lib.cmlb3_last_error(None) == b"null context"
    lib.cmlb3_destroy(None)


def _create(lib, plist, prec=0):
    from paper_2504_09024_amd import cmlb
    arr = (cmlb.SimParams * max(len(plist), 1))(*[cmlb.make_params(p) for p in plist])
    h = ctypes.c_void_p()
    rc = lib.cmlb_create(arr, len(plist), prec, None, ctypes.byref(h))
    return rc, h


def test_validation_before_device(lib):
    from paper_2504_09024_amd import cmlb
    from paper_2504_09024_amd import workloads as W
    good = W.params(nx=64, ny=64)
    assert _create(lib, [])[0] == cmlb.EINVAL
    assert _create(lib, [dict(good, nx=2)])[0] == cmlb.EINVAL
    assert _create(lib, [dict(good, phi_a=0.0, phi_b=0.0)])[0] == cmlb.EINVAL
    assert _create(lib, [dict(good, W=0.0)])[0] == cmlb.EINVAL
    assert _create(lib, [good], prec=7)[0] == cmlb.EINVAL
    # sims of one context share flow and boundary type
    assert _create(lib, [good, dict(good, flow="coupled")])[0] == cmlb.EINVAL
    assert _create(lib, [good, dict(good, bc_y="walls")])[0] == cmlb.EINVAL
    # relaxation rates outside (0, 2)
    cpl = dict(good, flow="coupled")
    assert _create(lib, [dict(cpl, omega_zeta=2.5)])[0] == cmlb.EUNSTABLE
    assert _create(lib, [dict(cpl, nu_a=-0.2)])[0] in (cmlb.EINVAL, cmlb.EUNSTABLE)
    assert _create(lib, [dict(good, M_phi=-0.1)])[0] == cmlb.EINVAL
    # a simulation's population block (rows padded to runs of 64 nodes)
    # must fit 2^31 bytes: 27 x 4 B x 4096 x 4800 fits, 4096 x 4864 does not;
    # the padding counts (4033 columns take 64 runs)
    big = dict(cpl, nx=4096, ny=4864)
    assert _create(lib, [big], prec=1)[0] == cmlb.EINVAL
    assert _create(lib, [dict(big, nx=4033)], prec=1)[0] == cmlb.EINVAL
    assert _create(lib, [dict(big, nx=4096, ny=2432)], prec=0)[0] == cmlb.EINVAL
    assert _create(lib, [dict(big, nx=8192, ny=4864)], prec=2)[0] == cmlb.EINVAL
    # null output handle
    arr = (cmlb.SimParams * 1)(cmlb.make_params(good))
    assert lib.cmlb_create(arr, 1, 0, None, None) == cmlb.EINVAL
    # null context everywhere
    assert lib.cmlb_step(None, 1) == cmlb.EINVAL
    assert lib.cmlb_step_count(None) == -1
    assert lib.cmlb_last_error(None) == b"null context"
    lib.cmlb_destroy(None)


def test_copy_validation_before_device(lib):
    """cmlb_copy rejects null or misaligned pointers, sizes that are not a
    multiple of 16 and an unknown cache policy before any device call; an
    empty copy launches nothing."""
    from paper_2504_09024_amd import cmlb
    vp = ctypes.c_void_p
    assert lib.cmlb_copy(None, vp(256), 16, 0, None) == cmlb.EINVAL
    assert lib.cmlb_copy(vp(257), vp(512), 16, 0, None) == cmlb.EINVAL
    assert lib.cmlb_copy(vp(256), vp(520), 16, 0, None) == cmlb.EINVAL
    assert lib.cmlb_copy(vp(256), vp(512), 24, 0, None) == cmlb.EINVAL
    assert lib.cmlb_copy(vp(256), vp(512), -16, 0, None) == cmlb.EINVAL
    assert lib.cmlb_copy(vp(256), vp(512), 16, 2, None) == cmlb.EINVAL
    assert lib.cmlb_copy(vp(256), vp(512), 0, 1, None) == cmlb.OK


def test_copy_planes_validation_before_device(lib):
    """cmlb_copy_planes takes the rules of cmlb_copy and only 9 or 27
    planes, checked before any device call."""
    from paper_2504_09024_amd import cmlb
    vp = ctypes.c_void_p
    for planes in (0, 1, 8, 10, 26, 28, -9):
        assert lib.cmlb_copy_planes(vp(256), vp(512), 16, planes, 0, None) == cmlb.EINVAL
    assert lib.cmlb_copy_planes(None, vp(256), 16, 9, 0, None) == cmlb.EINVAL
    assert lib.cmlb_copy_planes(vp(264), vp(512), 16, 9, 0, None) == cmlb.EINVAL
    assert lib.cmlb_copy_planes(vp(256), vp(512), 24, 27, 0, None) == cmlb.EINVAL
    assert lib.cmlb_copy_planes(vp(256), vp(512), -16, 27, 1, None) == cmlb.EINVAL
    assert lib.cmlb_copy_planes(vp(256), vp(512), 16, 27, 3, None) == cmlb.EINVAL
    assert lib.cmlb_copy_planes(vp(256), vp(512), 0, 27, 1, None) == cmlb.OK
