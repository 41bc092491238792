"""The C ABI: exported symbols and host-side error conventions (no GPU needed).

These calls are all rejected on the host before any device work, so they run
in the CPU suite; each must return the documented status and leave a message.
"""
import ctypes
import os
import re
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lpdec.h")
LIB = os.path.join(ROOT, "paper_1204_0556_amd", "liblpdec.so")

EINVAL, ENOMEM, EDEVICE, EUNSUPPORTED = -1, -2, -3, -4


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(lpdec_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.fail("liblpdec.so is not built (run __graft_entry__.build())")
    L = ctypes.CDLL(LIB)
    L.lpdec_last_error.restype = ctypes.c_char_p
    return L


def test_header_declares_the_abi():
    names = declared_functions()
    for must in ("lpdec_code_create", "lpdec_code_destroy", "lpdec_decode", "lpdec_decode_state",
                 "lpdec_decode_multi", "lpdec_project", "lpdec_last_error", "lpdec_default_params",
                 "lpdec_code_get_info"):
        assert must in names


def test_library_exports_every_declared_symbol(lib):
    for name in declared_functions():
        assert hasattr(lib, name), name
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True, text=True).stdout
    for name in declared_functions():
        assert re.search(rf"\bT {name}\b", out), name


def _create(lib, m, n, row_ptr, col_idx):
    rp = np.ascontiguousarray(row_ptr, np.int32)
    ci = np.ascontiguousarray(col_idx, np.int32)
    h = ctypes.c_void_p()
    st = lib.lpdec_code_create(ctypes.c_int32(m), ctypes.c_int32(n), ctypes.c_int64(ci.size),
                               rp.ctypes.data_as(ctypes.c_void_p), ci.ctypes.data_as(ctypes.c_void_p),
                               ctypes.byref(h))
    return st, h, lib.lpdec_last_error().decode()


@pytest.mark.parametrize("case,m,n,rp,ci,status,msg", [
    ("empty column", 2, 4, [0, 2, 4], [0, 1, 0, 1], EINVAL, "column 2"),
    ("degree one row", 2, 3, [0, 1, 3], [0, 1, 2], EINVAL, "degree 1"),
    ("duplicate index", 1, 3, [0, 3], [0, 0, 1], EINVAL, "strictly increasing"),
    ("unsorted row", 1, 3, [0, 3], [2, 0, 1], EINVAL, "strictly increasing"),
    ("index out of range", 1, 3, [0, 3], [0, 1, 3], EINVAL, "out of range"),
    ("bad row_ptr end", 1, 3, [0, 2], [0, 1, 2], EINVAL, "nnz"),
    ("degree above max", 1, 17, [0, 17], list(range(17)), EUNSUPPORTED, "degree 17"),
    ("no rows", 0, 3, [0], [0], EINVAL, "m and n"),
    # size limits: 16-bit variable and slot indices in the edge metadata
    ("n too large", 1, 65537, [0, 2], [0, 1], EUNSUPPORTED, "n > 65536"),
    ("nnz too large", 8193, 65536, list(range(0, 65537, 8)) + [65544], list(range(65536)) + list(range(8)),
     EUNSUPPORTED, "nnz > 65536"),
])
def test_code_create_rejects(lib, case, m, n, rp, ci, status, msg):
    st, h, err = _create(lib, m, n, rp, ci)
    assert st == status, (case, st, err)
    assert h.value is None
    assert msg in err, (case, err)


def test_null_arguments(lib):
    lib.lpdec_decode.argtypes = [ctypes.c_void_p, ctypes.c_int32] + [ctypes.c_void_p] * 6
    assert lib.lpdec_decode(None, 1, None, None, None, None, None, None) == EINVAL
    assert "code" in lib.lpdec_last_error().decode()
    lib.lpdec_code_destroy(None)  # NULL-safe
    lib.lpdec_decode_noalloc.argtypes = [ctypes.c_void_p, ctypes.c_int32] + [ctypes.c_void_p] * 6
    assert lib.lpdec_decode_noalloc(None, 1, None, None, None, None, None, None) == EINVAL
    assert "code" in lib.lpdec_last_error().decode()


def test_project_argument_checks(lib):
    lib.lpdec_project.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
    assert lib.lpdec_project(17, 4, None, None, None) == EINVAL
    assert lib.lpdec_project(1, 4, None, None, None) == EINVAL
    assert lib.lpdec_project(6, -1, None, None, None) == EINVAL
    assert lib.lpdec_project(6, 0, None, None, None) == 0  # empty batch is a no-op
    assert lib.lpdec_project(6, 4, None, None, None) == EINVAL


def test_multi_argument_checks(lib):
    lib.lpdec_decode_multi.restype = ctypes.c_int
    assert lib.lpdec_decode_multi(None, 0, 1, None, None, None, ctypes.c_int64(0), None, None, None,
                                  ctypes.c_int64(0), None, None, None) == EINVAL


def test_multi_autotune_argument_checks(lib):
    vp, i32, i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
    lib.lpdec_autotune_multi.argtypes = [vp, i32, i32, vp, vp, vp, i64, vp, i32, vp, vp, vp]
    assert lib.lpdec_autotune_multi(None, 1, 4, None, None, None, 0, None, 2, None, None, None) == EINVAL
    assert "NULL" in lib.lpdec_last_error().decode()


def test_tuning_argument_checks(lib):
    vp, i32 = ctypes.c_void_p, ctypes.c_int32
    lib.lpdec_code_set_tuning.argtypes = [vp, i32, i32, i32]
    assert lib.lpdec_code_set_tuning(None, 1, 1, -1) == EINVAL
    lib.lpdec_code_set_graph.argtypes = [vp, i32]
    assert lib.lpdec_code_set_graph(None, 1) == EINVAL
    lib.lpdec_code_launch_info.argtypes = [vp, vp, vp]
    assert lib.lpdec_code_launch_info(None, None, None) == EINVAL
    lib.lpdec_autotune.argtypes = [vp, i32, vp, vp, i32, vp, vp, vp]
    assert lib.lpdec_autotune(None, 1, None, None, 2, None, None, None) == EINVAL
    assert "NULL" in lib.lpdec_last_error().decode()


def test_default_params(lib):
    class P(ctypes.Structure):
        _fields_ = [("mu", ctypes.c_float), ("rho", ctypes.c_float), ("max_iter", ctypes.c_int32),
                    ("tol", ctypes.c_float), ("storage", ctypes.c_int32), ("mode", ctypes.c_int32)]
    lib.lpdec_default_params.restype = P
    p = lib.lpdec_default_params()
    # Sec. 5.1: eps = 1e-5, mu = 3, t_max = 1000, rho = 1.9
    assert (p.mu, p.max_iter, p.storage, p.mode) == (3.0, 1000, 0, 0)
    assert abs(p.rho - 1.9) < 1e-6 and abs(p.tol - 1e-5) < 1e-12


def test_sorting_networks_sort_every_binary_input(tmp_path):
    """The kernels' compare-exchange networks (0-1 principle, all 2^d inputs)."""
    inc = os.path.join(ROOT, "paper_1204_0556_amd", "csrc", "sortnet.inc")
    src = tmp_path / "net.cpp"
    src.write_text(f'''
#include <cstdio>
#define LPD_CE(a,b) {{ int p=s[a], q=s[b]; s[a]=p>q?p:q; s[b]=p>q?q:p; }}
#include "{inc}"
template <int D> int check(void (*f)(int*)) {{
  for (int m = 0; m < (1 << D); ++m) {{ int s[16]; for (int k = 0; k < D; ++k) s[k] = (m >> k) & 1; f(s);
    for (int k = 1; k < D; ++k) if (s[k-1] < s[k]) return 0; }}
  return 1; }}
void n2(int*s){{LPD_NET_2}} void n3(int*s){{LPD_NET_3}} void n4(int*s){{LPD_NET_4}} void n5(int*s){{LPD_NET_5}}
void n6(int*s){{LPD_NET_6}} void n7(int*s){{LPD_NET_7}} void n8(int*s){{LPD_NET_8}}
void n9(int*s){{LPD_NET_9}} void n10(int*s){{LPD_NET_10}} void n11(int*s){{LPD_NET_11}} void n12(int*s){{LPD_NET_12}}
void n13(int*s){{LPD_NET_13}} void n14(int*s){{LPD_NET_14}} void n15(int*s){{LPD_NET_15}} void n16(int*s){{LPD_NET_16}}
int main(){{ return !(check<2>(n2)&&check<3>(n3)&&check<4>(n4)&&check<5>(n5)&&check<6>(n6)&&check<7>(n7)&&check<8>(n8)
  &&check<9>(n9)&&check<10>(n10)&&check<11>(n11)&&check<12>(n12)&&check<13>(n13)&&check<14>(n14)
  &&check<15>(n15)&&check<16>(n16)); }}
''')
    exe = tmp_path / "net"
    subprocess.check_call(["g++", "-O1", "-o", str(exe), str(src)])
    assert subprocess.call([str(exe)]) == 0


def test_binding_constants_match_the_header():
    import re
    hdr = open(os.path.join(ROOT, "include", "lpdec.h")).read()
    py = open(os.path.join(ROOT, "paper_1204_0556_amd", "__init__.py")).read()
    h = int(re.search(r"#define LPDEC_TUNE_VARIANTS (\d+)", hdr).group(1))
    b = int(re.search(r"^TUNE_VARIANTS = (\d+)", py, re.M).group(1))
    assert h == b == 4
