"""The C-ABI library loads and exports every entry point of include/ssd.h;
argument checks that return before any device work behave as documented.
No GPU is needed."""
import ctypes
import os
import re

import pytest

from paper_1503_02198_amd import ssd

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ssd.h")


def _declared():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"\b(ssd_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(ssd.LIB_PATH):
        pytest.fail("libssd.so is not built (python -m paper_1503_02198_amd.build)")
    return ssd.lib()


def test_exports_match_header(L):
    names = _declared()
    assert len(names) >= 12
    for n in names:
        assert hasattr(L, n), n
    assert sorted(ssd.EXPORTS) == names


def test_struct_layout_matches_header():
    # ssd_mesh_desc: 2 ints, 6 pointers, 14 doubles (incl. arrays) on LP64
    assert ctypes.sizeof(ssd.MeshDesc) == 8 + 6 * 8 + 14 * 8
    assert ctypes.sizeof(ssd.Info) == 6 * 4 + 2 * 8
    # ssd_batch_group: 7 int32, a float, an int32 and 2 floats
    assert ctypes.sizeof(ssd.BatchGroup) == 11 * 4


def test_struct_layout_matches_c_compiler(tmp_path):
    """The binding's structures against sizeof/offsetof from a C compiler
    reading include/ssd.h."""
    import shutil
    import subprocess
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    src = tmp_path / "layout.c"
    src.write_text('#include <stdio.h>\n#include <stddef.h>\n#include "ssd.h"\n'
                   "int main(void) { printf(\"%zu %zu %zu %zu %zu\\n\", sizeof(ssd_mesh_desc), "
                   "offsetof(ssd_mesh_desc, face_kind), sizeof(ssd_info), offsetof(ssd_info, work_len), "
                   "sizeof(ssd_batch_group)); return 0; }\n")
    exe = tmp_path / "layout"
    include = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include")
    subprocess.run([cc, "-std=c99", "-I", include, "-o", str(exe), str(src)], check=True)
    got = [int(x) for x in subprocess.run([str(exe)], check=True, capture_output=True,
                                          text=True).stdout.split()]
    assert got == [ctypes.sizeof(ssd.MeshDesc), ssd.MeshDesc.face_kind.offset, ctypes.sizeof(ssd.Info),
                   ssd.Info.work_len.offset, ctypes.sizeof(ssd.BatchGroup)]


def test_argument_errors_without_device(L):
    h = ctypes.c_void_p()
    assert L.ssd_create_mesh(None, 0, ctypes.byref(h)) == -1
    assert b"null" in L.ssd_last_error()
    d = ssd.MeshDesc()
    d.N = 7
    d.n_elem = 4
    assert L.ssd_create_mesh(ctypes.byref(d), 0, ctypes.byref(h)) == -1
    assert b"N must be" in L.ssd_last_error()
    d.N = 3
    d.n_elem = 0
    assert L.ssd_create_mesh(ctypes.byref(d), 0, ctypes.byref(h)) == -1
    assert L.ssd_query(None, None) == -1
    assert L.ssd_set_rotation(None, 0.0, 0.0) == -1
    assert L.ssd_residual(None, None, None, None) == -1
    assert L.ssd_rk_step(None, None, None, 0.0, 1.0, 0, None) == -1
    assert L.ssd_destroy_mesh(None) == 0
    # batches
    b = ctypes.c_void_p()
    assert L.ssd_batch_create(None, 1, ctypes.byref(b)) == -1
    arr = (ctypes.c_void_p * 1)(None)
    assert L.ssd_batch_create(arr, 1, ctypes.byref(b)) == -1
    assert b"null mesh" in L.ssd_last_error()
    assert L.ssd_batch_create(arr, 0, ctypes.byref(b)) == -1
    assert L.ssd_batch_rk_steps(None, None, None, None, None, 1, 0, 0, None) == -1
    assert L.ssd_batch_query(None, 0, None) == -1
    assert L.ssd_batch_destroy(None) == 0
    # learned correction
    net = ctypes.c_void_p()
    assert L.ssd_mlp_create(5, 0, ctypes.byref(net)) == -1
    assert b"N = 2..4" in L.ssd_last_error()
    assert L.ssd_mlp_create(3, 0, None) == -1
    assert L.ssd_mlp_destroy(None) == 0
    assert L.ssd_mlp_dims(None, None, None) == -1
    assert L.ssd_mlp_forward(None, None, 0, None, None) == -1
    assert L.ssd_mlp_train_step(None, None, None, 1, None, 1, ctypes.c_float(1e-3),
                                ctypes.c_float(0.0), 0, None) == -1
    assert L.ssd_mlp_loss(None, None, None) == -1
    assert L.ssd_subgrid_features(None, None, None, None) == -1
    assert L.ssd_restrict(None, None, None, None, None, None) == -1
    assert b"null mesh" in L.ssd_last_error()
    assert L.ssd_subgrid_targets(None, None, None, None, None, None, None) == -1
    assert L.ssd_subgrid_attach(None, None, ctypes.c_float(1.0), 0) == -1
