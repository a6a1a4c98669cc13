"""The C ABI library loads and exports every function include/ar.h declares (CPU only).

Also checks that the binding's ctypes structures have the sizes and field offsets the
C compiler gives the structures of include/ar.h (a tiny C program prints them).
"""
import ctypes
import os
import re
import subprocess
import sys

import pytest

from paper_2503_00308_amd import api

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ar.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ar_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_binding_symbols():
    assert set(declared_functions()) == set(api.SYMBOLS)


@pytest.mark.skipif(not os.path.exists(api.LIB_PATH), reason="library not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(api.LIB_PATH)
    for name in declared_functions():
        assert hasattr(lib, name), name
    out = subprocess.run(["nm", "-D", "--defined-only", api.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(re.findall(r"\bT (ar_[a-z_0-9]+)$", out, flags=re.M))
    assert set(declared_functions()) <= exported


@pytest.mark.skipif(not os.path.exists(api.LIB_PATH), reason="library not built")
def test_version_and_last_error_without_gpu():
    lib = api.load()
    assert lib.ar_version().startswith(b"abstract-render")
    assert isinstance(lib.ar_last_error(), bytes)
    assert lib.ar_scene_size(None) == 0


def test_struct_layout_matches_c(tmp_path):
    src = tmp_path / "layout.c"
    structs = {"ar_scene_desc": api.SceneDesc, "ar_intrinsics": api.Intrinsics, "ar_pose_box": api.PoseBox,
               "ar_options": api.Options, "ar_stats": api.Stats, "ar_server_config": api.ServerConfig,
               "ar_query_result": api.QueryResult, "ar_server_stats": api.ServerStats,
               "ar_scene_set": api.SceneSet}
    lines = ['#include <stdio.h>', '#include <stddef.h>', f'#include "{HEADER}"', "int main(void) {"]
    for cname, cls in structs.items():
        lines.append(f'  printf("{cname} %zu\\n", sizeof({cname}));')
        for fname, _ in cls._fields_:
            lines.append(f'  printf("{cname}.{fname} %zu\\n", offsetof({cname}, {fname}));')
    lines += ["  return 0;", "}"]
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c99", str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split("\n")
    got = dict(l.split() for l in out if l.strip())
    for cname, cls in structs.items():
        assert int(got[cname]) == ctypes.sizeof(cls), cname
        for fname, _ in cls._fields_:
            assert int(got[f"{cname}.{fname}"]) == getattr(cls, fname).offset, (cname, fname)


def test_server_argument_errors_without_gpu():
    """Null handles are rejected before any device call."""
    import ctypes
    lib = api.load()
    assert lib.ar_server_create(None, None) == api.AR_E_INVALID
    sid = ctypes.c_int32()
    assert lib.ar_server_add_scene(None, None, ctypes.byref(sid)) == api.AR_E_INVALID
    r = api.QueryResult()
    assert lib.ar_server_wait(None, 1, 0, ctypes.byref(r)) == api.AR_E_INVALID
    assert lib.ar_server_report(None, None) == api.AR_E_INVALID
    lib.ar_server_destroy(None)


def test_product_path_does_not_use_the_oracle():
    """The package and its HIP sources never import, include or name the oracle package,
    and importing the binding does not load it."""
    pkg = os.path.join(ROOT, "paper_2503_00308_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                text = open(os.path.join(dirpath, f)).read()
                assert not re.search(r"^\s*(from|import)\s+oracle\b", text, flags=re.M), f
                assert "oracle/" not in text, f
    code = ("import sys; sys.path.insert(0, %r); import paper_2503_00308_amd.api, paper_2503_00308_amd.synth; "
            "print(any(m == 'oracle' or m.startswith('oracle.') for m in sys.modules))" % ROOT)
    out = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=300).stdout.strip()
    assert out == "False"
