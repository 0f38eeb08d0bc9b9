"""The C-ABI library loads on a host without a GPU and exports every entry
point the public header declares (no compute call is made)."""
import ctypes
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "spt.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", " ", src, flags=re.S)
    src = re.sub(r"//[^\n]*", " ", src)
    src = re.sub(r"#[^\n]*", " ", src)
    names = set()
    for decl in src.split(";"):
        decl = " ".join(decl.split())
        m = re.match(r"^(?:extern \"C\" \{ )?(?:const )?[\w]+(?: \*+| )\s*\*?(spt_\w+)\s*\(", decl)
        if m:
            names.add(m.group(1))
    return names


def test_header_declares_the_path():
    names = declared_functions()
    for n in ("spt_encode", "spt_mttkrp", "spt_cp_als", "spt_mttkrp_batched", "spt_cp_als_batched", "spt_autotune",
              "spt_server_create", "spt_server_submit", "spt_server_wait", "spt_server_destroy", "spt_last_error"):
        assert n in names, n
    assert len(names) >= 20


def test_library_exports_every_declared_symbol():
    from paper_2509_00280_amd import spt
    if not os.path.exists(spt.LIB_PATH):
        from paper_2509_00280_amd import build
        build.build()
    lib = ctypes.CDLL(spt.LIB_PATH)
    missing = [n for n in sorted(declared_functions()) if not hasattr(lib, n)]
    assert not missing, missing
    lib.spt_version.restype = ctypes.c_char_p
    assert lib.spt_version().decode().startswith("spt-gfx950")


def test_binding_plan_struct_matches_header():
    # the ctypes mirror of spt_plan lists the header's fields in order with the same types
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", " ", src, flags=re.S)
    m = re.search(r"typedef struct \{([^}]*)\} spt_plan;", src)
    assert m, "spt_plan not found"
    fields = [" ".join(f.split()) for f in m.group(1).split(";") if f.strip()]
    want = []
    for f in fields:
        g = re.match(r"int (\w+)(\[SPT_MAX_MODES\])?$", f)
        assert g, f
        want.append((g.group(1), bool(g.group(2))))
    from paper_2509_00280_amd import spt
    got = [(name, hasattr(ty, "_length_")) for name, ty in spt.Plan._fields_]
    assert got == want
    assert ctypes.sizeof(spt.Plan) == 4 * sum(spt.MAX_MODES if arr else 1 for _, arr in want)
