"""The C ABI library loads and exports every symbol include/ddm.h declares.

CPU only: no compute call is made.  Also checks that the ctypes mirror of
ddm_plan_desc has the C layout, and the validation paths that return before
any HIP call.
"""

import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = [os.path.join(ROOT, "include", f) for f in sorted(os.listdir(os.path.join(ROOT, "include")))
           if f.endswith(".h")]


def declared_functions():
    names = []
    for h in HEADERS:
        text = open(h).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        names += re.findall(r"\b(ddm_[a-z0-9_]+)\s*\(", text)
    return sorted(set(names))


def test_header_declares_entry_points():
    names = declared_functions()
    for n in ["ddm_plan_create", "ddm_structure_function", "ddm_radial_average",
              "ddm_image_spectra", "ddm_structure_from_spectra", "ddm_last_error"]:
        assert n in names


def test_library_exports_every_declared_symbol(libddm_path):
    lib = ctypes.CDLL(libddm_path)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_covers_every_declared_symbol(libddm_path):
    from paper_2012_05695_amd import _lib
    bound = {s[0] for s in _lib.SIGNATURES}
    assert set(declared_functions()) <= bound
    _lib.load(libddm_path)


@pytest.mark.parametrize("cname,pyname", [("ddm_plan_desc", "PlanDesc"), ("ddm_fit_desc", "FitDesc")])
def test_struct_layout_matches_c(tmp_path, cname, pyname):
    from paper_2012_05695_amd import _lib
    cls = getattr(_lib, pyname)
    src = tmp_path / "layout.c"
    src.write_text(
        '#include <stdio.h>\n#include <stddef.h>\n#include "ddm.h"\n'
        "int main(void){printf(\"%%zu\", sizeof(%s));" % cname
        + "".join('printf(" %%zu", offsetof(%s, %s));' % (cname, f) for f, _ in cls._fields_)
        + "return 0;}\n")
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)])
    vals = [int(x) for x in subprocess.check_output([str(exe)]).split()]
    assert vals[0] == ctypes.sizeof(cls)
    offs = [getattr(cls, f).offset for f, _ in cls._fields_]
    assert vals[1:] == offs


def test_host_only_calls(libddm_path):
    from paper_2012_05695_amd import _lib
    lib = _lib.load(libddm_path)
    assert lib.ddm_abi_version() == 1
    d = _lib.PlanDesc()
    lib.ddm_plan_desc_init(ctypes.byref(d))
    assert d.struct_size == ctypes.sizeof(_lib.PlanDesc)
    assert d.k2_max == -1 and d.precondition == 1 and d.pixel == _lib.DDM_PIX_U16
    h = ctypes.c_void_p(1234)
    # validation failures return before any HIP call
    d.struct_size = 3
    assert lib.ddm_plan_create(ctypes.byref(d), ctypes.byref(h)) == _lib.DDM_ERR_INVALID_ARGUMENT
    assert h.value is None
    assert b"struct_size" in lib.ddm_last_error()
    lib.ddm_plan_desc_init(ctypes.byref(d))
    d.width, d.height, d.n_frames = 100, 64, 8
    assert lib.ddm_plan_create(ctypes.byref(d), ctypes.byref(h)) == _lib.DDM_ERR_UNSUPPORTED
    d.width, d.n_frames = 64, 1
    assert lib.ddm_plan_create(ctypes.byref(d), ctypes.byref(h)) == _lib.DDM_ERR_INVALID_ARGUMENT
    d.n_frames, d.max_lag = 8, 9
    assert lib.ddm_plan_create(ctypes.byref(d), ctypes.byref(h)) == _lib.DDM_ERR_INVALID_ARGUMENT
    assert lib.ddm_plan_create(None, ctypes.byref(h)) == _lib.DDM_ERR_INVALID_ARGUMENT
    # step two's method: unknown values, and the lengths each method takes
    lib.ddm_plan_desc_init(ctypes.byref(d))
    assert d.method == _lib.DDM_METHOD_FOURIER and d.padding == _lib.DDM_PAD_POW2
    d.width, d.height, d.n_frames = 64, 64, 8
    d.method = 3
    assert lib.ddm_plan_create(ctypes.byref(d), ctypes.byref(h)) == _lib.DDM_ERR_INVALID_ARGUMENT
    assert b"method" in lib.ddm_last_error()
    d.method, d.n_frames = _lib.DDM_METHOD_FOURIER, 16385
    assert lib.ddm_plan_create(ctypes.byref(d), ctypes.byref(h)) == _lib.DDM_ERR_UNSUPPORTED
    assert b"DDM_METHOD_DIRECT" in lib.ddm_last_error()
    d.method, d.n_frames = _lib.DDM_METHOD_DIRECT, 65537
    assert lib.ddm_plan_create(ctypes.byref(d), ctypes.byref(h)) == _lib.DDM_ERR_UNSUPPORTED
    assert lib.ddm_plan_method(None, None) == _lib.DDM_ERR_INVALID_ARGUMENT
    # batches: every stack descriptor is checked before any HIP call, and
    # batched stacks take the FP32 spectra store only
    descs = (_lib.PlanDesc * 2)()
    for i in range(2):
        lib.ddm_plan_desc_init(ctypes.byref(descs[i]))
        descs[i].width, descs[i].height, descs[i].n_frames = 64, 64, 16
    descs[1].spectrum = _lib.DDM_SPEC_F16_QSCALED
    b = ctypes.c_void_p(1234)
    assert lib.ddm_batch_create(descs, 2, 2, None, ctypes.byref(b)) == _lib.DDM_ERR_UNSUPPORTED
    assert b.value is None and b"stack 1" in lib.ddm_last_error()
    descs[1].spectrum = _lib.DDM_SPEC_F32
    descs[1].n_frames = 1
    assert lib.ddm_batch_create(descs, 2, 2, None, ctypes.byref(b)) == _lib.DDM_ERR_INVALID_ARGUMENT
    assert b"stack 1" in lib.ddm_last_error()
    assert lib.ddm_batch_create(descs, 2, 0, None, ctypes.byref(b)) == _lib.DDM_ERR_INVALID_ARGUMENT
    assert lib.ddm_plan_destroy(None) == _lib.DDM_OK
    assert lib.ddm_structure_function(None, None, None) == _lib.DDM_ERR_INVALID_ARGUMENT


def test_noalloc_scratch_size_matches_header():
    from paper_2012_05695_amd import _lib
    text = open(os.path.join(ROOT, "include", "ddm.h")).read()
    m = re.search(r"#define DDM_NOALLOC_SCRATCH_BYTES \((\d+)u << (\d+)\)", text)
    assert m, "DDM_NOALLOC_SCRATCH_BYTES not found"
    assert int(m.group(1)) << int(m.group(2)) == _lib.DDM_NOALLOC_SCRATCH_BYTES
