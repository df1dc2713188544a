"""CPU-side checks of the C ABI: the built library loads and exports every entry point the
public header declares (no device calls)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "bc.h")
LIB = os.path.join(ROOT, "paper_1409_7764_amd", "libbcmi.so")


def declared_symbols():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^BC_API\s+[\w\s\*]+?\b(bc_\w+)\s*\(", text, flags=re.M)))


@pytest.fixture(scope="module")
def libpath():
    if not os.path.exists(LIB):
        from paper_1409_7764_amd import build_lib
        build_lib.build()
    return LIB


def test_header_declares_the_boundary():
    names = declared_symbols()
    for required in ["bc_build_csr", "bc_exact", "bc_sampled", "bc_batch", "bc_serve_create", "bc_serve_submit",
                     "bc_serve_poll", "bc_serve_destroy", "bc_sssp", "bc_last_error", "bc_tune"]:
        assert required in names


def test_library_exports_every_declared_symbol(libpath):
    lib = ctypes.CDLL(libpath)
    missing = [s for s in declared_symbols() if not hasattr(lib, s)]
    assert not missing, missing
    lib.bc_version.restype = ctypes.c_char_p
    assert b"gfx950" in lib.bc_version()
    lib.bc_last_error.restype = ctypes.c_char_p
    assert lib.bc_last_error() == b""


def struct_fields(name):
    """Field names of a typedef struct in the public header, in order."""
    text = open(HEADER).read()
    end = re.search(r"\}\s*" + name + ";", text).start()
    body = text[text.rindex("typedef struct {", 0, end) + len("typedef struct {"):end]
    body = re.sub(r"/\*.*?\*/", "", body, flags=re.S)
    out = []
    for decl in body.split(";"):
        decl = decl.strip()
        if not decl:
            continue
        names = decl.split(",")   # "double a, b, c": the type goes with the first name
        for part in names:
            m = re.search(r"(\w+)\s*(\[\d+\])?\s*$", part.strip())
            out.append(m.group(1))
    return out


@pytest.mark.parametrize("name", ["bc_tuning", "bc_info"])
def test_binding_structs_match_the_header(name):
    """The Python binding's ctypes structures list the header's fields in the header's order."""
    from paper_1409_7764_amd import bcmi
    assert [f for f, _ in getattr(bcmi, name)._fields_] == struct_fields(name)


def test_library_holds_gfx950_code(libpath):
    data = open(libpath, "rb").read()
    assert b"gfx950" in data


def test_null_handle_errors_without_device(libpath):
    lib = ctypes.CDLL(libpath)
    lib.bc_graph_info.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
    assert lib.bc_graph_info(None, None, None) == -1          # BC_E_INVAL
    lib.bc_last_error.restype = ctypes.c_char_p
    assert b"null graph" in lib.bc_last_error()


def test_bench_refuses_more_than_one_gpu():
    """The benchmark measures one GPU: asking for more exits with a message, before any
    device work."""
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""
