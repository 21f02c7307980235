"""C-ABI checks that need no GPU: the library loads, exports every declared symbol, and
rejects bad arguments before any device call."""
import ctypes as C
import os
import re
import subprocess

import numpy as np
import pytest

import paper_2404_16322_amd as P
from paper_2404_16322_amd import binding as B

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = set()
    for f in os.listdir(os.path.join(ROOT, "include")):
        if f.endswith(".h"):
            txt = open(os.path.join(ROOT, "include", f)).read()
            txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
            names |= set(re.findall(r"\b(ddc_[a-z_0-9]+)\s*\(", txt))
    return names


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(P.lib_path()):
        pytest.fail("libddc.so is not built; run __graft_entry__.build()")
    return P.load_library()


def test_exports_every_declared_symbol(lib):
    names = _declared()
    assert len(names) >= 13
    for n in names:
        assert hasattr(lib, n), n
    assert set(B.SYMBOLS) == names


def test_struct_layouts_match_the_c_compiler(tmp_path):
    """sizeof / offsetof of every ABI struct, as gcc lays out include/ddc.h, equal ctypes'."""
    structs = {"ddc_fit_params": B.FitParams, "ddc_artifacts": B.Artifacts,
               "ddc_index_info": B.IndexInfo, "ddc_search_stats": B.SearchStats,
               "ddc_server_params": B.ServerParams, "ddc_server_stats": B.ServerStats,
               "ddc_launch_params": B.LaunchParams}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "ddc.h"', "int main(void){"]
    for cname, cls in structs.items():
        lines.append(f'printf("{cname} %zu\\n", sizeof({cname}));')
        for f, _ in cls._fields_:
            lines.append(f'printf("{cname}.{f} %zu\\n", offsetof({cname}, {f}));')
    lines.append("return 0;}")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c99", f"-I{os.path.join(ROOT, 'include')}", str(src), "-o", str(exe)],
                   check=True)
    got = dict(l.split() for l in subprocess.run([str(exe)], capture_output=True, text=True,
                                                 check=True).stdout.splitlines())
    for cname, cls in structs.items():
        assert int(got[cname]) == C.sizeof(cls), cname
        for f, _ in cls._fields_:
            assert int(got[f"{cname}.{f}"]) == getattr(cls, f).offset, (cname, f)


def test_default_params(lib):
    p = B.default_params()
    assert (p.nlist, p.delta_d, p.block_b, p.lag_l, p.kmeans_iters, p.calib_k, p.calib_max_neg) == \
        (4096, 32, 256, 0, 25, 10, 50)
    assert p.pca_sample == 1_000_000


def _rc(fn, *args):
    return fn(*args)


def test_search_rejects_bad_arguments_without_device(lib):
    q = np.zeros((1, 8), np.float32)
    ids = np.zeros(10, np.int64)
    d = np.zeros(10, np.float32)
    rc = lib.ddc_search(None, q.ctypes.data, 1, 10, 1, 0.1, 0, ids.ctypes.data, d.ctypes.data, None)
    assert rc == -1 and b"NULL" in lib.ddc_last_error()
    rc = lib.ddc_search_device(None, None, 1, None, 10, 10, None, 1, 1, 0.1, 0, None, None, None,
                               None, None)
    assert rc == -1
    rc = lib.ddc_search_device_noalloc(None, None, 1, None, 10, 10, None, 1, 1, 0.1, 0, None, None,
                                       None, None, None)
    assert rc == -1 and b"NULL" in lib.ddc_last_error()
    assert lib.ddc_search_device_noalloc_bytes() == 64 << 20
    rc = lib.ddc_search_estimate(None, q.ctypes.data, 1, 10, 1, 32, 0, ids.ctypes.data, d.ctypes.data)
    assert rc == -1 and b"NULL" in lib.ddc_last_error()
    lp = B.LaunchParams(0, -1, 1, 1, -1, -1, 0, 0, 0)
    assert lib.ddc_set_launch(None, C.byref(lp)) == -1
    w = C.c_int32()
    assert lib.ddc_scan_variant(None, 1, 1, 1, 0, C.byref(w), C.byref(w), None, None, None) == -1


def test_fit_rejects_bad_parameters_without_device(lib):
    base = np.zeros((100, 16), np.float32)
    cal = np.zeros((10, 16), np.float32)
    out = C.c_void_p()
    cases = [dict(nlist=0), dict(nlist=200), dict(delta_d=16), dict(block_b=100), dict(lag_l=-1), dict(lag_l=65),
             dict(calib_k=0), dict(calib_max_neg=0), dict(storage=7)]
    for kw in cases:
        p = B.default_params(nlist=4)
        for k, v in kw.items():
            setattr(p, k, v)
        rc = lib.ddc_fit(base.ctypes.data, 100, 16, cal.ctypes.data, 10, C.byref(p), C.byref(out))
        assert rc in (-1, -6), (kw, rc)
        assert out.value is None
        assert lib.ddc_last_error()
    bad = base.copy()
    bad[3, 3] = np.nan
    rc = lib.ddc_fit(bad.ctypes.data, 100, 16, cal.ctypes.data, 10, C.byref(B.default_params(nlist=4)),
                     C.byref(out))
    assert rc == -1 and b"non-finite" in lib.ddc_last_error()
    rc = lib.ddc_fit(base.ctypes.data, 100, 5000, cal.ctypes.data, 10, C.byref(B.default_params(nlist=4)),
                     C.byref(out))
    assert rc == -1


def test_import_rejects_bad_artifacts_without_device(lib):
    a = B.Artifacts()
    out = C.c_void_p()
    assert lib.ddc_import(None, C.byref(out)) == -1
    a.n, a.dim, a.nlist, a.delta_d, a.block_b = 10, 8, 2, 32, 256
    assert lib.ddc_import(C.byref(a), C.byref(out)) == -1      # missing arrays
    mu, R = np.zeros(8), np.eye(8)
    cent = np.zeros((2, 8), np.float32)
    assign = np.array([0, 1, 2, 0, 0, 0, 0, 0, 0, 0], np.int32)  # 2 is out of range
    y = np.zeros((10, 8), np.float32)
    a.mu, a.rot, a.centroids, a.assign, a.y = mu.ctypes.data, R.ctypes.data, cent.ctypes.data, \
        assign.ctypes.data, y.ctypes.data
    assert lib.ddc_import(C.byref(a), C.byref(out)) == -1
    assert b"assign" in lib.ddc_last_error()
    a.lag_l = 65
    assert lib.ddc_import(C.byref(a), C.byref(out)) == -1
    assert b"lag_l" in lib.ddc_last_error()


def test_correction_rejects_bad_significance(lib):
    m = np.zeros(4)
    assert lib.ddc_correction(None, 10, 0.1, 0, m.ctypes.data, m.ctypes.data) == -1


def test_server_rejects_bad_arguments_without_device(lib):
    out = C.c_void_p()
    p = B.ServerParams(4, 256, 1 << 30, 0.05, 0)
    assert lib.ddc_server_create(None, C.byref(p), C.byref(out)) == -1
    assert out.value is None
    t = C.c_uint64()
    assert lib.ddc_server_submit(None, None, 1, None, None, C.byref(t)) == -1
    done = C.c_int()
    assert lib.ddc_server_poll(None, 1, None, None, C.byref(done), None) == -1
    st = B.ServerStats()
    assert lib.ddc_server_get_stats(None, C.byref(st)) == -1


def test_load_rejects_missing_and_foreign_files_without_device(lib, tmp_path):
    out = C.c_void_p()
    assert lib.ddc_load(str(tmp_path / "none.ddc").encode(), C.byref(out)) == -4
    f = tmp_path / "foreign.ddc"
    f.write_bytes(b"NOTANIDX" + bytes(64))
    assert lib.ddc_load(str(f).encode(), C.byref(out)) == -4
    assert b"not an index file" in lib.ddc_last_error()
    f.write_bytes(b"DDCINDEX" + (1).to_bytes(4, "little") + bytes(10))
    assert lib.ddc_load(str(f).encode(), C.byref(out)) == -4      # truncated header
    assert out.value is None
    assert lib.ddc_save(None, b"x") == -1


def test_fit_rejects_bad_table_and_fp8_parameters_without_device(lib):
    base = np.zeros((100, 16), np.float32)
    cal = np.zeros((10, 16), np.float32)
    out = C.c_void_p()
    for kw in [dict(calib_k_extra=(5, 0, 0)), dict(calib_k_extra=(20, 15, 0)),
               dict(calib_k_extra=(0, 20, 0)), dict(calib_k_extra=(300, 0, 0)),
               dict(fp8_lead_dims=32), dict(fp8_lead_dims=64)]:
        p = B.default_params(nlist=4, **kw)
        rc = lib.ddc_fit(base.ctypes.data, 100, 16, cal.ctypes.data, 10, C.byref(p), C.byref(out))
        assert rc == -1, kw
        assert out.value is None


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    """No fallback: with the library absent the first call raises instead of computing."""
    from paper_2404_16322_amd import binding
    monkeypatch.setattr(binding, "_LIB", None)
    monkeypatch.setattr(binding, "lib_path", lambda: str(tmp_path / "libddc.so"))
    with pytest.raises(RuntimeError, match="not built"):
        binding.load_library()
    with pytest.raises(RuntimeError, match="not built"):
        binding.default_params(nlist=4)


def test_product_package_never_loads_the_oracle():
    """The package and its library load without the oracle (test infrastructure only)."""
    import sys
    code = ("import sys; import paper_2404_16322_amd as P; P.load_library(); "
            "P.binding.default_params(nlist=4); "
            "bad = [m for m in sys.modules if m == 'oracle' or m.startswith('oracle.')]; "
            "assert not bad, bad")
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, "-c", code], cwd=root, capture_output=True, text=True,
                       timeout=120)
    assert r.returncode == 0, r.stderr[-2000:]


def test_oracle_and_product_share_no_code():
    """Neither side imports, includes or links the other: the package's sources never name
    the oracle, and the oracle's sources never name the package, its C++ sources or header."""
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    pkg = os.path.join(root, "paper_2404_16322_amd")
    use_oracle = re.compile(r"^\s*(import\s+oracle\b|from\s+oracle\b|#\s*include\s*[<\"].*oracle)", re.M)
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".cpp", ".hip", ".h")):
                txt = open(os.path.join(dirpath, f), encoding="utf-8").read()
                assert not use_oracle.search(txt), os.path.join(dirpath, f)
    use_pkg = re.compile(r"^\s*(import\s+paper_2404_16322_amd|from\s+paper_2404_16322_amd|"
                         r".*\bcsrc\b|.*ddc\.h|.*libddc)", re.M)
    for f in os.listdir(os.path.join(root, "oracle")):
        if f.endswith(".py"):
            txt = open(os.path.join(root, "oracle", f), encoding="utf-8").read()
            code = "\n".join(l for l in txt.splitlines() if not l.lstrip().startswith("#"))
            code = re.sub(r'"""(?:.|\n)*?"""', "", code)
            assert not use_pkg.search(code), f


def test_fault_injection_spec_and_live_counts_without_device(lib):
    """ddc_set_fault accepts only "alloc:<n>" (n >= 0) and the live-allocation count starts empty
    (no device is touched by either)."""
    for bad in (b"", b"alloc", b"alloc:", b"alloc:-1", b"alloc:3x", b"free:1", None):
        assert lib.ddc_set_fault(bad) == -1
    assert lib.ddc_set_fault(b"alloc:7") == 0
    assert lib.ddc_set_fault(b"alloc:0") == 0
    n, b = C.c_int64(-1), C.c_int64(-1)
    assert lib.ddc_live_allocations(C.byref(n), C.byref(b)) == 0
    assert (n.value, b.value) == (0, 0)
    assert lib.ddc_live_allocations(None, None) == -1
