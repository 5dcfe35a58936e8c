"""CPU tests of the C ABI: the library loads, exports every function the
header declares, and rejects bad arguments before launching anything.
No compute call is made here (there is no GPU)."""
import ctypes
import os
import re
from ctypes import byref, c_double, c_size_t, c_void_p

import numpy as np
import pytest

import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "tsvdm.h")


@pytest.fixture(scope="module")
def lib():
    from paper_2605_16058_amd import _lib
    return _lib.load()


def _header_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(tsvdm_[a-z_0-9]+)\s*\(", src)))


def test_header_and_binding_agree():
    from paper_2605_16058_amd import _lib
    assert _header_functions() == sorted(_lib.exported_names())


def test_header_constants_match_binding():
    from paper_2605_16058_amd import _lib
    src = open(HEADER).read()
    m = re.search(r"#define TSVDM_GRAM_MAX_R (\d+)", src)
    assert m and int(m.group(1)) == _lib.GRAM_MAX_R
    m = re.search(r"#define TSVDM_GRAM_LDS_MAX_R (\d+)", src)
    assert m and int(m.group(1)) == _lib.GRAM_LDS_MAX_R
    for name, v in _lib.GRAM_JACOBI.items():
        assert re.search(rf"TSVDM_GRAM_{name.upper()} = {v}\b", src), name


def test_library_exports_every_declared_symbol(lib):
    for name in _header_functions():
        assert hasattr(lib, name), name


def test_version(lib):
    assert lib.tsvdm_version() >= 10000


def _colmajor_bytes(M):
    return np.ascontiguousarray(np.asarray(M, dtype=np.float64).T)


def test_check_transform_accepts_orthogonal_and_scaled(lib):
    for M, c2 in [(synth.dct2_matrix(16), 1.0),
                  (synth.haar_orthogonal(9, np.random.default_rng(0)), 1.0),
                  (3.0 * synth.dct2_matrix(5), 9.0)]:
        Mc = _colmajor_bytes(M)
        out = c_double(0)
        rc = lib.tsvdm_check_transform(c_void_p(Mc.ctypes.data), M.shape[0], 1e-10, byref(out))
        assert rc == 0
        assert abs(out.value - c2) < 1e-12 * c2


def test_check_transform_rejects(lib):
    M = np.array([[1.0, 0.3], [0.0, 1.0]])
    Mc = _colmajor_bytes(M)
    rc = lib.tsvdm_check_transform(c_void_p(Mc.ctypes.data), 2, 1e-10, None)
    assert rc == -3
    assert b"orthogonal" in lib.tsvdm_last_error()
    Z = np.zeros((3, 3))
    assert lib.tsvdm_check_transform(c_void_p(Z.ctypes.data), 3, 1e-10, None) == -3
    assert lib.tsvdm_check_transform(None, 3, 1e-10, None) == -1


DUMMY = c_void_p(256)  # never dereferenced: every call below fails validation


def test_workspace_queries(lib):
    from paper_2605_16058_amd import _lib
    assert _lib.workspace_size("tsvdm_transform_workspace_size", 256) >= 256 * 256 * 8
    assert _lib.workspace_size("tsvdm_slice_svd_workspace_size", 512, 1024, 256, 0) > 0
    assert _lib.workspace_size("tsvdm_truncate_tol_workspace_size", 512, 256) >= 131072 * 8
    assert _lib.workspace_size("tsvdm_pack_workspace_size", 64, 48, 16) >= 48 * 16 * 4
    assert _lib.workspace_size("tsvdm_reconstruct_workspace_size", 64, 48, 16, 0) >= 64 * 48 * 16 * 8
    assert _lib.workspace_size("tsvdm_error_workspace_size", 1000) > 0
    assert _lib.workspace_size("tsvdm_backward_workspace_size", 32, 24, 8, 1) > 0
    out = c_size_t(0)
    assert lib.tsvdm_slice_svd_workspace_size(0, 4, 4, 0, byref(out)) == -2
    assert lib.tsvdm_slice_svd_workspace_size(4, 4, 4, 2, byref(out)) == -8


def test_transform_validation(lib):
    ok = (DUMMY, 1, c_void_p(512), 1, 8, 8, 4, DUMMY, 0, 1.0, 0, 0, DUMMY, 1 << 20, None)
    # null input
    a = list(ok); a[0] = None
    assert lib.tsvdm_transform(*a) == -1
    # bad shape
    a = list(ok); a[4] = 0
    assert lib.tsvdm_transform(*a) == -2
    # bad dtype / compute
    a = list(ok); a[1] = 7
    assert lib.tsvdm_transform(*a) == -8
    a = list(ok); a[10] = 2; a[3] = 0  # bf16 compute into an F64 output
    assert lib.tsvdm_transform(*a) == -8
    # aliasing
    a = list(ok); a[2] = a[0]
    assert lib.tsvdm_transform(*a) == -1
    # unknown tile shape
    for tile in (-1, 9):
        a = list(ok); a[11] = tile
        assert lib.tsvdm_transform(*a) == -1
        assert b"tile" in lib.tsvdm_last_error()
    # workspace too small
    a = list(ok); a[13] = 8
    assert lib.tsvdm_transform(*a) == -4
    assert b"workspace" in lib.tsvdm_last_error()


def test_slice_svd_validation(lib):
    base = [DUMMY, 0, 16, 12, 4, DUMMY, DUMMY, DUMMY, 0, 0, 0.0, 1, DUMMY, 1 << 20, None]
    a = list(base); a[8] = 7
    assert lib.tsvdm_slice_svd(*a) == -1
    a = list(base); a[10] = 1.5
    assert lib.tsvdm_slice_svd(*a) == -1
    a = list(base); a[6] = None
    assert lib.tsvdm_slice_svd(*a) == -1
    a = list(base); a[13] = 0
    assert lib.tsvdm_slice_svd(*a) == -4


def test_slice_svd_gram_validation(lib):
    D2 = c_void_p(256 + 4096)   # B must not alias A_hat
    base = [DUMMY, 200, 150, 4, D2, DUMMY, DUMMY, DUMMY, 0, 0, 0.0, 0, 1, DUMMY, 1 << 30, None]
    a = list(base); a[11] = 3            # unknown placement of the Jacobi
    assert lib.tsvdm_slice_svd_gram(*a) == -1
    assert b"jacobi" in lib.tsvdm_last_error()
    a = list(base); a[11] = 2            # in LDS needs min(m, p) <= 128
    assert lib.tsvdm_slice_svd_gram(*a) == -2
    a = list(base); a[1] = 1030; a[2] = 1040
    assert lib.tsvdm_slice_svd_gram(*a) == -2
    a = list(base); a[4] = DUMMY
    assert lib.tsvdm_slice_svd_gram(*a) == -1
    a = list(base); a[8] = 7
    assert lib.tsvdm_slice_svd_gram(*a) == -1
    a = list(base); a[14] = 8
    assert lib.tsvdm_slice_svd_gram(*a) == -4


def test_truncation_validation(lib):
    assert lib.tsvdm_truncate_rank(0, 4, 4, DUMMY, DUMMY, None) == -1
    assert lib.tsvdm_truncate_rank(2, 0, 4, DUMMY, DUMMY, None) == -2
    base = [DUMMY, 8, 4, 0.1, DUMMY, DUMMY, DUMMY, DUMMY, 1 << 20, None]
    for eps in (0.0, 1.0, -0.5, float("nan")):
        a = list(base); a[3] = eps
        assert lib.tsvdm_truncate_tol(*a) == -1
    a = list(base); a[8] = 16
    assert lib.tsvdm_truncate_tol(*a) == -4


def test_pack_reconstruct_error_backward_validation(lib):
    p = [DUMMY, DUMMY, DUMMY, 0, 8, 6, 3, DUMMY, DUMMY, -1, DUMMY, DUMMY, DUMMY, DUMMY, DUMMY,
         1 << 20, None]
    assert lib.tsvdm_pack(*p) == -1
    p[9] = 4; p[3] = 5
    assert lib.tsvdm_pack(*p) == -8
    rc = [DUMMY, DUMMY, 0, 8, 6, 3, DUMMY, DUMMY, 4, None, 1.0, DUMMY, 0, 0, 0, DUMMY, 1 << 20, None]
    assert lib.tsvdm_reconstruct(*rc) == -1
    rc[9] = DUMMY; rc[10] = float("inf")
    assert lib.tsvdm_reconstruct(*rc) == -1
    rc[10] = 1.0; rc[14] = 9
    assert lib.tsvdm_reconstruct(*rc) == -1
    assert lib.tsvdm_error(DUMMY, 0, DUMMY, 0, 0, DUMMY, DUMMY, 1 << 20, None) == -2
    bw = [DUMMY, 1, 8, 6, 3, DUMMY, 0, 1.0, None, None, DUMMY, DUMMY, DUMMY, 1 << 30, None]
    assert lib.tsvdm_backward(*bw) == -1
    bw[6] = 2; bw[14 - 1] = 1
    assert lib.tsvdm_backward(*bw) == -4


def _header_struct_fields(name):
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    body = re.search(r"typedef struct \{(.*?)\}\s*" + name + r"\s*;", src, flags=re.S).group(1)
    fields = []
    for decl in body.split(";"):
        decl = decl.strip()
        if not decl:
            continue
        names = decl.split(None, 1)[1] if not decl.startswith("const") else decl.split(None, 2)[2]
        for nm in names.split(","):
            fields.append(nm.strip().lstrip("*").strip())
    return fields


def test_batch_item_layout_matches_header(tmp_path):
    """Field names and every offset agree with what a C compiler makes of the header."""
    import shutil
    import subprocess
    from paper_2605_16058_amd import _lib
    names = [f for f, _ in _lib.BatchItem._fields_]
    assert _header_struct_fields("tsvdm_batch_item") == names
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    src = tmp_path / "layout.c"
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "tsvdm.h"', "int main(void) {",
             '  printf("%zu\\n", sizeof(tsvdm_batch_item));']
    lines += [f'  printf("%zu\\n", offsetof(tsvdm_batch_item, {f}));' for f in names]
    lines += ["  return 0;", "}"]
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run([cc, "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)],
                   check=True)
    got = [int(x) for x in subprocess.run([str(exe)], check=True, capture_output=True,
                                          text=True).stdout.split()]
    assert got[0] == ctypes.sizeof(_lib.BatchItem)
    assert got[1:] == [getattr(_lib.BatchItem, f).offset for f in names]


def _item(m=40, p=30, n=6, mode=2):
    from paper_2605_16058_amd import _lib
    it = _lib.BatchItem()
    it.m, it.p, it.n = m, p, n
    it.A = it.M = it.rho = it.offsets = 256
    it.inv_scale = 1.0
    it.mode = mode
    it.k = 4
    it.eps = 0.1
    return it


def test_batch_plan_validation_and_layout(lib):
    """Plan creation only validates and lays out host tables: no device call."""
    from paper_2605_16058_amd import _lib

    def create(items, block=0):
        arr = (_lib.BatchItem * len(items))(*items)
        plan, wsb = c_void_p(), c_size_t(0)
        rc = lib.tsvdm_batch_plan_create(ctypes.cast(arr, c_void_p), len(items), 1, 1, 1, block, 0,
                                         byref(plan), byref(wsb))
        if rc == 0:
            assert wsb.value > 0
            assert lib.tsvdm_batch_plan_destroy(plan) == 0
        return rc, wsb.value

    assert create([_item(), _item(300, 280, 12, 1)])[0] == 0
    # per-item widths and tiles
    a, b = _item(), _item(300, 280, 12, 1)
    a.block, b.block, a.ttm_tile, b.ttm_tile = 16, 32, 3, 1
    assert create([a, b])[0] == 0
    for field, bad in (("block", 8), ("block", 64), ("ttm_tile", 9), ("ttm_tile", -1), ("reserved", 1)):
        it = _item()
        setattr(it, field, bad)
        assert create([it])[0] == -1, field
        assert field.encode() in lib.tsvdm_last_error()
    assert create([_item()], block=8)[0] == -1
    bad = _item(); bad.eps = 1.0
    assert create([bad])[0] == -1
    bad = _item(); bad.n = 0
    assert create([bad])[0] == -2


def test_transform_mode_validation(lib):
    from ctypes import c_int64
    dims = (c_int64 * 4)(5, 4, 3, 2)
    ok = [DUMMY, 1, c_void_p(512), 1, 4, dims, 3, DUMMY, 0, 1.0, 1, 0, DUMMY, 1 << 20, None]
    a = list(ok); a[6] = 2           # mode 2 is never transformed
    assert lib.tsvdm_transform_mode(*a) == -1
    a = list(ok); a[6] = 5           # k > d
    assert lib.tsvdm_transform_mode(*a) == -1
    a = list(ok); a[4] = 2           # d < 3
    assert lib.tsvdm_transform_mode(*a) == -2
    bad = (c_int64 * 4)(5, 0, 3, 2)
    a = list(ok); a[5] = bad
    assert lib.tsvdm_transform_mode(*a) == -2
    a = list(ok); a[5] = None
    assert lib.tsvdm_transform_mode(*a) == -1
    a = list(ok); a[13] = 8          # workspace
    assert lib.tsvdm_transform_mode(*a) == -4
    assert lib.tsvdm_lowrank(DUMMY, DUMMY, 0, 8, 6, 3, DUMMY, DUMMY, -1, DUMMY, None) == -1
    assert lib.tsvdm_lowrank(DUMMY, DUMMY, 5, 8, 6, 3, DUMMY, DUMMY, 4, DUMMY, None) == -8


def test_transform_dct_validation(lib):
    # every rejection happens on the host, before any launch
    from ctypes import c_int64
    dims = (c_int64 * 3)(5, 4, 16)
    ok = [DUMMY, 1, c_void_p(512), 1, 3, dims, 3, 0, 1, None]
    a = list(ok); a[7] = 2           # inverse must be 0 or 1
    assert lib.tsvdm_transform_dct(*a) == -1
    a = list(ok); a[8] = 2           # BF16 arithmetic is not offered
    assert lib.tsvdm_transform_dct(*a) == -8
    a = list(ok); a[6] = 4           # k > d
    assert lib.tsvdm_transform_dct(*a) == -1
    a = list(ok); a[2] = DUMMY       # Y aliases X
    assert lib.tsvdm_transform_dct(*a) == -1
    for n in (1, 12, 2048):          # not a power of two in [2, 1024]
        a = list(ok); a[5] = (c_int64 * 3)(5, 4, n)
        assert lib.tsvdm_transform_dct(*a) == -2
    a = list(ok); a[5] = (c_int64 * 3)(1 << 16, 1 << 15, 2)   # rows before mode 3 >= 2^31
    assert lib.tsvdm_transform_dct(*a) == -2
    a = list(ok); a[5] = None
    assert lib.tsvdm_transform_dct(*a) == -1
