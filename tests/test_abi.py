"""CPU checks of the C ABI: the library loads and exports every declared symbol."""
import ctypes
import os
import re
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = [os.path.join(ROOT, "include", f) for f in sorted(os.listdir(os.path.join(ROOT, "include"))) if f.endswith(".h")]
LIB = os.path.join(ROOT, "paper_2504_07090_amd", "libbayesvis.so")


def declared_functions():
    text = "\n".join(open(h).read() for h in HEADERS)
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\*?\s*([a-z_][a-z0-9_]*)\s*\(",
                       text, flags=re.M)
    return sorted(set(names))


def test_header_declares_the_entry_points():
    names = declared_functions()
    for n in ("vis_forward", "vis_adjoint", "chi2_and_grad", "vis_field_create",
              "vis_basis_create", "vis_last_error", "vis_profile_read"):
        assert n in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_host_only_calls_without_gpu():
    lib = ctypes.CDLL(LIB)
    lib.vis_version.restype = ctypes.c_char_p
    assert b"gfx950" in lib.vis_version()
    lib.vis_last_error.restype = ctypes.c_char_p
    # a bad basis descriptor is rejected on the host before any device call
    class BasisDesc(ctypes.Structure):
        _fields_ = [("grid_nz", ctypes.c_int32), ("grid_nphi", ctypes.c_int32),
                    ("lmax", ctypes.c_int32), ("storage", ctypes.c_uint32)]
    n = ctypes.c_size_t()
    assert lib.vis_basis_workspace_bytes(ctypes.byref(BasisDesc(32, 96, -1, 1)), ctypes.byref(n)) == -1
    assert b"lmax" in lib.vis_last_error()
    assert lib.vis_basis_workspace_bytes(ctypes.byref(BasisDesc(32, 96, 20, 3)), ctypes.byref(n)) == 0
    # FP32 + bf16 hi/lo copies of a 3072 x 448 Y plus generator staging tables
    assert n.value >= 3072 * 448 * (4 + 2 + 2)


def test_binding_fails_loudly_without_library(tmp_path):
    """The product path has no CPU fallback: importing the binding without the
    built library raises."""
    code = ("import sys, os; sys.path.insert(0, %r); "
            "import paper_2504_07090_amd.vis as v" % str(tmp_path))
    pkg = tmp_path / "paper_2504_07090_amd"
    pkg.mkdir()
    for f in ("__init__.py", "vis.py", "workload.py"):
        (pkg / f).write_text(open(os.path.join(ROOT, "paper_2504_07090_amd", f)).read())
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True)
    assert r.returncode != 0 and "not built" in r.stderr


STRUCTS = {
    # C struct name -> (python module, ctypes class name)
    "vis_basis_desc": ("vis", "BasisDesc"),
    "vis_field_desc": ("vis", "FieldDesc"),
    "vis_field_info": ("vis", "FieldInfo"),
    "vis_kernel_time": ("vis", "KernelTime"),
    "hmc_server_config": ("serve", "ServerConfig"),
    "hmc_chain_init": ("serve", "ChainInit"),
    "hmc_result": ("serve", "Result"),
    "hmc_stats": ("serve", "Stats"),
}


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_binding_structs_match_the_header(tmp_path):
    """The ctypes mirrors of the ABI structs have the size and field offsets the
    C compiler gives the header's declarations."""
    import importlib
    mods = {m: importlib.import_module("paper_2504_07090_amd." + m) for m in ("vis", "serve")}
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "bayesvis.h"',
             '#include "bayesvis_serve.h"', "int main(void) {"]
    for cname, (mod, pyname) in STRUCTS.items():
        cls = getattr(mods[mod], pyname)
        lines.append(f'  printf("{cname} size %zu\\n", sizeof({cname}));')
        for fname, *_ in cls._fields_:
            lines.append(f'  printf("{cname} {fname} %zu\\n", offsetof({cname}, {fname}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)],
                   check=True, capture_output=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {}
    for line in out:
        if line:
            parts = line.split()
            got[(parts[0], parts[1])] = int(parts[2])
    for cname, (mod, pyname) in STRUCTS.items():
        cls = getattr(mods[mod], pyname)
        assert got[(cname, "size")] == ctypes.sizeof(cls), cname
        for fname, *_ in cls._fields_:
            assert got[(cname, fname)] == getattr(cls, fname).offset, (cname, fname)
