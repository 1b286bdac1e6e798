"""The C-ABI library loads and exports every entry point declared in
include/trx.h (no GPU needed: nothing is called)."""

import ctypes
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "trx.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(trx_[a-z0-9_]+)\s*\(", src)))


def test_header_declares_the_entry_points():
    names = _declared()
    for n in ("trx_create", "trx_forward", "trx_chi2_grad", "trx_plan_create",
              "trx_plan_launch", "trx_autotune"):
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_1912_07759_amd import trx
    lib = ctypes.CDLL(trx.LIB_PATH)
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing
    assert sorted(trx.EXPORTS) == _declared()


def test_binding_struct_layouts_match_header():
    """Field order of the ctypes mirrors equals the header's structs."""
    from paper_1912_07759_amd import trx
    src = open(os.path.join(ROOT, "include", "trx.h")).read()
    for cname, py in (("trx_tables_desc", trx.TablesDesc), ("trx_batch", trx.BatchC)):
        body = re.search(r"typedef struct \{([^{}]*)\}\s*" + cname + ";", src).group(1)
        body = re.sub(r"/\*.*?\*/", "", body, flags=re.S)
        fields = []
        for decl in body.split(";"):
            decl = decl.strip()
            if decl:
                fields.append(re.findall(r"[A-Za-z_]\w*", decl)[-1])
        assert [f[0] for f in py._fields_] == fields, (cname, fields)
