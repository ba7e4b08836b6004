"""The C ABI library loads on a machine without a GPU and exports every
function include/tid.h declares; the binding declares the same set."""
import ctypes
import os
import re

from paper_1807_01409_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if not fn.endswith(".h"):
            continue
        text = open(os.path.join(ROOT, "include", fn)).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        for m in re.finditer(r"^\s*(?:const\s+)?[A-Za-z_][\w\s\*]*?\b(tid_\w+)\s*\(", text, re.M):
            names.add(m.group(1))
    return names


def test_header_parses():
    names = declared_functions()
    assert {"tid_load", "tid_scan", "tid_join", "tid_union", "tid_filter", "tid_query"} <= names


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(_lib.LIB_PATH)
    missing = [n for n in sorted(declared_functions()) if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_covers_header():
    assert declared_functions() == set(_lib.SIGNATURES)


def test_binding_loads_library():
    lib = _lib.load_library()
    assert lib.tid_last_error(None) == b""
