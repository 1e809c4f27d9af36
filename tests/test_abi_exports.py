"""The C-ABI library loads without a GPU and exports every function that
include/*.h declares (CPU; no compute call is made)."""
import ctypes as C
import glob
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = set()
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        text = open(h).read()
        text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
        text = re.sub(r"//[^\n]*", " ", text)
        for m in re.finditer(r"\b(?:int32_t|int64_t|void|const\s+char\s*\*)\s*\**\s*(bbc_\w+)\s*\(", text):
            names.add(m.group(1))
    return sorted(names)


def test_header_declares_the_path():
    names = declared_functions()
    for required in ("bbc_build_index", "bbc_search", "bbc_index_free", "bbc_last_error", "bbc_query_bytes",
                     "bbc_server_create", "bbc_server_submit", "bbc_server_poll", "bbc_server_destroy"):
        assert required in names


def test_library_exports_every_declared_function():
    import paper_2604_01960_amd as bbc
    lib = bbc.load()
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing
    # no device needed to read the error string
    lib.bbc_last_error.restype = C.c_char_p
    assert isinstance(lib.bbc_last_error(), bytes)
