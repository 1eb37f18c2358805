"""The C-ABI library loads, exports what include/kc.h declares, and rejects
malformed graphs on the host (no GPU needed: validation runs before any
device call)."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def kc():
    import paper_2511_16356_amd as kc
    if not os.path.exists(kc.LIB_PATH):
        from paper_2511_16356_amd import build_lib
        build_lib.build()
    return kc


def declared_functions():
    text = open(os.path.join(ROOT, "include", "kc.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return set(re.findall(r"\b(kc_[a-z0-9_]+)\s*\(", text))


def test_exports_every_declared_symbol(kc):
    lib = kc.library()
    decl = declared_functions()
    assert decl == set(kc.EXPORTS)
    for name in decl:
        assert hasattr(lib, name), name


def test_status_strings(kc):
    lib = kc.library()
    for code in range(8):
        assert lib.kc_status_string(code)


def _create(kc, offsets, indices, root=-1):
    lib = kc.library()
    off = np.ascontiguousarray(offsets, dtype=np.int64)
    idx = np.ascontiguousarray(indices, dtype=np.int32)
    h = ctypes.c_void_p()
    st = lib.kc_graph_create(len(off) - 1, ctypes.c_void_p(off.ctypes.data), 1,
                             ctypes.c_void_p(idx.ctypes.data), root, None, ctypes.byref(h))
    return st, lib.kc_last_error().decode()


def test_rejects_malformed_graphs(kc):
    # path 0-1-2 as a reference shape
    assert _create(kc, [0], [])[0] == 1                                   # n < 2
    assert _create(kc, [0, 1, 3, 4], [1, 2, 0, 1])[0] == 1               # row 1 not ascending
    assert _create(kc, [0, 2, 4, 5], [0, 1, 0, 2, 1])[0] == 1            # self-loop at 0
    assert _create(kc, [0, 1, 3, 4], [1, 0, 0, 1])[0] == 1               # duplicate in row 1
    assert _create(kc, [0, 1, 2, 3], [1, 0, 1])[0] == 1                  # (2,1) has no reverse
    assert _create(kc, [0, 1, 3, 4], [1, 0, 5, 1])[0] == 1               # neighbour out of range
    assert _create(kc, [0, 1, 3, 4], [1, 0, 2, 1], root=7)[0] == 1       # root out of range
    assert _create(kc, [1, 1, 3, 4], [1, 0, 2, 1])[0] == 1               # offsets[0] != 0
    st, msg = _create(kc, [0, 1, 2, 3, 4], [1, 0, 3, 2])                # two components
    assert st == 2 and "reachable" in msg


def test_rejects_huge_degree(kc):
    leaves = 1 << 20
    n = leaves + 1
    off = np.concatenate([[0, leaves], leaves + np.arange(1, leaves + 1)]).astype(np.int64)
    idx = np.concatenate([np.arange(1, n), np.zeros(leaves)]).astype(np.int32)
    assert _create(kc, off, idx)[0] == 7


def test_binding_fails_loudly_without_library(kc, monkeypatch, tmp_path):
    monkeypatch.setattr(kc, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(kc, "_lib", None)
    with pytest.raises(kc.KcError):
        kc.library()


def test_probe_library_exports_its_header():
    """libkc_probe.so (measured memory ceilings) exports what include/kc_probe.h declares."""
    from paper_2511_16356_amd import build_lib
    if not os.path.exists(build_lib.PROBE_LIB):
        build_lib.build()
    text = open(os.path.join(ROOT, "include", "kc_probe.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    decl = set(re.findall(r"\b(kc_[a-z0-9_]+)\s*\(", text))
    assert decl == {"kc_probe_stream_read", "kc_probe_random_read", "kc_probe_stream_sweep", "kc_probe_random_sweep"}
    lib = ctypes.CDLL(build_lib.PROBE_LIB)
    for name in decl:
        assert hasattr(lib, name), name


def _oracle_imports(path):
    """(enclosing function name or None, line) of every import of the oracle in a Python file."""
    import ast
    tree = ast.parse(open(path).read(), filename=path)
    found = []

    def visit(node, func):
        for child in ast.iter_child_nodes(node):
            f = child.name if isinstance(child, (ast.FunctionDef, ast.AsyncFunctionDef)) else func
            if isinstance(child, ast.Import) and any(a.name.split(".")[0] == "oracle" for a in child.names):
                found.append((func, child.lineno))
            if isinstance(child, ast.ImportFrom) and (child.module or "").split(".")[0] == "oracle":
                found.append((func, child.lineno))
            visit(child, f)

    visit(tree, None)
    return found


def test_product_never_reaches_the_oracle():
    """The product path has no route to the CPU oracle: nothing in the package
    (Python, HIP, C++) or the public headers names it, and outside tests/ only
    the build step and smoke check of __graft_entry__.py and the benchmark's
    CPU-baseline leg import it."""
    for top in ("paper_2511_16356_amd", "include", "graphgen"):
        for dirpath, _, files in os.walk(os.path.join(ROOT, top)):
            for name in files:
                if not name.endswith((".py", ".hip", ".cpp", ".h", ".c")):
                    continue
                path = os.path.join(dirpath, name)
                text = open(path, errors="replace").read()
                assert not re.search(r"^\s*(import\s+oracle|from\s+oracle\b)", text, re.M), path
                assert not re.search(r'#\s*include\s*[<"][^>"]*oracle', text), path
                assert "kc_oracle" not in text and "orc_" not in text, path
    assert {f for f, _ in _oracle_imports(os.path.join(ROOT, "bench.py"))} == {"cpu_baseline"}
    assert {f for f, _ in _oracle_imports(os.path.join(ROOT, "__graft_entry__.py"))} <= {"build", "smoke"}


def test_oracle_never_reaches_the_product():
    """The oracle shares no code with the HIP path: nothing under oracle/
    imports the package, includes its headers or loads its library."""
    for dirpath, _, files in os.walk(os.path.join(ROOT, "oracle")):
        for name in files:
            if not name.endswith((".py", ".c", ".h")):
                continue
            path = os.path.join(dirpath, name)
            text = open(path, errors="replace").read()
            assert not re.search(r"^\s*(import\s+paper_2511_16356_amd|from\s+paper_2511_16356_amd\b)", text, re.M), path
            assert "libkc_mi355x.so" not in text and "libkc_probe.so" not in text, path
            assert not re.search(r'#\s*include\s*[<"](kc|kc_internal|kc_host)\.h', text), path
