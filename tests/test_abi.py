"""The C-ABI library loads and exports every symbol include/psi.h declares
(no compute calls: these run without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = [os.path.join(ROOT, "include", h) for h in sorted(os.listdir(os.path.join(ROOT, "include")))
           if h.endswith(".h")]


def declared_functions():
    names = []
    for h in HEADERS:
        text = open(h).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        names += re.findall(r"^\s*(?:const\s+)?[a-z_0-9]+\s*\*?\s*(psi_[a-z0-9_]+)\s*\(", text, flags=re.M)
    return sorted(set(names))


@pytest.fixture(scope="module")
def lib():
    from paper_2206_09960_amd import _ffi
    if not os.path.exists(_ffi.LIB_PATH):
        from paper_2206_09960_amd import build
        build.build()
    return _ffi.load()


def test_header_declares_entry_points():
    names = declared_functions()
    for required in ("psi_build_operator", "psi_solve", "psi_step", "psi_final",
                     "psi_operator_workspace_size", "psi_last_error"):
        assert required in names


def test_every_declared_symbol_is_exported(lib):
    for name in declared_functions():
        assert hasattr(lib, name), name


def test_binding_covers_header(lib):
    from paper_2206_09960_amd import _ffi
    bound = {s[0] for s in _ffi.SIGNATURES}
    assert set(declared_functions()) <= bound


def test_host_only_calls(lib):
    from paper_2206_09960_amd import _ffi
    assert lib.psi_version().decode().startswith("psi-mi355x")
    p = _ffi.Params()
    assert lib.psi_params_default(ctypes.byref(p)) == 0
    assert p.tol == 1e-8 and p.max_iter == 10000
    a, b = ctypes.c_size_t(), ctypes.c_size_t()
    assert lib.psi_operator_workspace_size(1000, 10000, 1, 0, ctypes.byref(a), ctypes.byref(b)) == 0
    assert a.value > 1000 * 8 and b.value > 10000 * 16
    assert lib.psi_operator_workspace_size(0, 10, 1, 0, ctypes.byref(a), ctypes.byref(b)) == 1
    assert b"n_users" in lib.psi_last_error()


def test_struct_sizes_match_header():
    """Compile a tiny C program against the header and compare struct sizes."""
    import subprocess
    import tempfile
    from paper_2206_09960_amd import _ffi
    src = r'''
#include <stdio.h>
#include "psi.h"
int main(void){printf("%zu %zu %zu\n", sizeof(psi_operator_stats), sizeof(psi_params), sizeof(psi_info));return 0;}
'''
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "t.c")
        open(c, "w").write(src)
        exe = os.path.join(d, "t")
        r = subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), "-I", "/opt/rocm/include",
                            c, "-o", exe], capture_output=True, text=True)
        assert r.returncode == 0, r.stderr
        out = subprocess.run([exe], capture_output=True, text=True).stdout.split()
    assert [int(x) for x in out] == [ctypes.sizeof(_ffi.OperatorStats), ctypes.sizeof(_ffi.Params),
                                     ctypes.sizeof(_ffi.Info)]


def test_binding_refuses_mismatched_inputs(lib):
    """Lengths are checked before any pointer reaches the library (no GPU needed)."""
    import numpy as np

    from paper_2206_09960_amd import api
    one = np.ones(3)
    with pytest.raises(ValueError, match="same length"):
        api.Operator(3, np.array([0, 1]), np.array([1]), one, one, device="cuda:0")
    with pytest.raises(ValueError, match="n_users"):
        api.Operator(3, np.array([0, 1]), np.array([1, 2]), np.ones(2), one, device="cuda:0")
    with pytest.raises(ValueError, match="node_offsets"):
        api.Operator(3, np.array([0, 1]), np.array([1, 2]), one, one, node_offsets=[0],
                     device="cuda:0")
    with pytest.raises(ValueError, match="GPU"):
        api.Operator(3, np.array([0, 1]), np.array([1, 2]), one, one, device="cpu")


def test_product_path_never_imports_the_oracle():
    """The package and its HIP sources neither import nor include anything
    under oracle/ (the oracle is test infrastructure only)."""
    import ast

    pkg = os.path.join(ROOT, "paper_2206_09960_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            path = os.path.join(dirpath, f)
            if f.endswith(".py"):
                tree = ast.parse(open(path, encoding="utf-8").read())
                for node in ast.walk(tree):
                    names = []
                    if isinstance(node, ast.Import):
                        names = [a.name for a in node.names]
                    elif isinstance(node, ast.ImportFrom):
                        names = [node.module or ""]
                    assert not any(n.split(".")[0] == "oracle" for n in names), path
            elif f.endswith((".hip", ".h", ".cpp")):
                src = open(path, encoding="utf-8").read()
                assert not re.search(r'#include\s+[<"][^>"]*oracle', src), path


def test_workspace_queries_and_limits(lib):
    """Host-only size queries: monotone in users and edges, the per-edge
    FP64 weights add at least 8 bytes per edge, and the documented limits
    are refused with PSI_EINVAL and a message that a later success clears."""
    from paper_2206_09960_amd import _ffi

    def size(n, m, graphs=1, flags=0):
        a, b = ctypes.c_size_t(), ctypes.c_size_t()
        st = lib.psi_operator_workspace_size(n, m, graphs, flags, ctypes.byref(a), ctypes.byref(b))
        return st, a.value, b.value

    st0, p0, s0 = size(10_000, 100_000)
    assert st0 == _ffi.PSI_OK
    _, p1, s1 = size(20_000, 100_000)
    _, p2, s2 = size(10_000, 200_000)
    assert p1 > p0 and p2 > p0 and s2 >= s0 and s1 >= s0
    _, pw, _ = size(10_000, 100_000, flags=_ffi.PSI_WEIGHTED_FP64)
    assert pw >= p0 + 8 * 100_000
    _, pg, _ = size(10_000, 100_000, graphs=16)
    _, pg2, _ = size(10_000, 100_000, graphs=32)
    # per-graph state grows with the graphs; graph operators reserve no band
    # layout (single-graph only), whose entries alone take 4 bytes per edge
    assert pg2 > pg and pg <= p0 - 4 * 100_000 + 64 * 10_000
    for args, word in (((1 << 30, 0), b"n_users"), ((1 << 29, (1 << 31) - (1 << 29)), b"too large"),
                       ((10, -1), b"n_edges"), ((10, 10, 0), b"n_graphs")):
        st, _, _ = size(*args)
        assert st == _ffi.PSI_EINVAL, args
        assert word in lib.psi_last_error(), (args, lib.psi_last_error())
    assert size(10, 10)[0] == _ffi.PSI_OK and lib.psi_last_error() == b""


def test_build_compiles_every_source_for_gfx950_without_packed_fp32():
    """The build covers every HIP source, targets gfx950 and turns packed FP32
    instructions off in device code."""
    from paper_2206_09960_amd import build as b
    on_disk = sorted(f for f in os.listdir(b.CSRC) if f.endswith(".hip"))
    assert sorted(b.SOURCES) == on_disk
    flags = " ".join(b.FLAGS)
    assert "--offload-arch=gfx950" in flags or os.environ.get("PSI_OFFLOAD_ARCH")
    assert "-Xclang -target-feature -Xclang -packed-fp32-ops" in flags
