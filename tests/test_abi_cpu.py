"""CPU checks of the C-ABI library: it loads and exports every function that
include/flinng.h declares (no compute call; there is no GPU here), and the
binding's structs match the header's field order and sizes."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "flinng.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[a-z_0-9]+\s*\*?\s*(flinng_[a-z_0-9]+)\s*\(", src, flags=re.M)
    return sorted(set(names))


def test_header_declares_the_boundary():
    names = declared_functions()
    for need in ("flinng_build", "flinng_query", "flinng_index_free", "flinng_last_error",
                 "flinng_serve_create", "flinng_serve_submit", "flinng_serve_wait",
                 "flinng_serve_destroy", "flinng_debug_hash", "flinng_debug_counts"):
        assert need in names


def test_library_exports_every_declared_symbol():
    import paper_2106_11565_amd._lib as L
    if not os.path.exists(L.LIB_PATH):
        pytest.fail("libflinng.so is not built (run __graft_entry__.build())")
    so = ctypes.CDLL(L.LIB_PATH)
    missing = [n for n in declared_functions() if not hasattr(so, n)]
    assert not missing, missing
    L.lib()  # binds every signature


def test_struct_layouts_match_header():
    import paper_2106_11565_amd._lib as L
    assert ctypes.sizeof(L.Params) == 8 * 4 + 8
    assert ctypes.sizeof(L.Input) == 8 + 8 + 8 + 4 + 4
    assert ctypes.sizeof(L.ServeConfig) == 8 + 4 * 4 + 8
    hdr = open(HEADER).read()
    for struct, cls in (("flinng_params", L.Params), ("flinng_input", L.Input),
                        ("flinng_index_info", L.IndexInfo), ("flinng_serve_config", L.ServeConfig),
                        ("flinng_serve_stats", L.ServeStats), ("flinng_theory", L.Theory)):
        body = re.search(r"typedef struct %s \{(.*?)\} %s;" % (struct, struct), hdr, re.S).group(1)
        body = re.sub(r"/\*.*?\*/", "", body, flags=re.S)
        fields = []
        for decl in body.split(";"):
            decl = decl.strip()
            if not decl:
                continue
            # "type a, b, c" -> a, b, c
            first, *rest = [x.strip() for x in decl.split(",")]
            fields.append(first.split()[-1].lstrip("*"))
            fields += [r.lstrip("*") for r in rest]
        assert fields == [f for f, _ in cls._fields_], (struct, fields)


def test_no_cpu_fallback_when_library_missing(tmp_path, monkeypatch):
    """The binding refuses to run without the HIP library (monkeypatch puts
    the module's state back afterwards)."""
    import paper_2106_11565_amd._lib as L
    monkeypatch.setattr(L, "LIB_PATH", str(tmp_path / "absent.so"))
    monkeypatch.setattr(L, "_lib", None)
    with pytest.raises(ImportError):
        L.lib()
