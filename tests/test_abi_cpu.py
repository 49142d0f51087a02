"""Host-side checks of the C ABI library (no GPU needed, no compute calls)."""
import ctypes
import os
import re

import pytest

import paper_2510_01579_amd as M

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_symbols():
    names = set()
    inc = os.path.join(ROOT, "include")
    for fn in os.listdir(inc):
        if fn.endswith(".h"):
            text = open(os.path.join(inc, fn)).read()
            text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
            names.update(re.findall(r"\b(mmgap_[a-z0-9_]+)\s*\(", text))
    return sorted(names)


def test_library_is_built():
    assert os.path.exists(M.LIB_PATH), "run __graft_entry__.build() first"


def test_every_declared_symbol_is_exported():
    declared = _declared_symbols()
    assert len(declared) >= 7
    L = ctypes.CDLL(M.LIB_PATH)
    missing = [n for n in declared if not hasattr(L, n)]
    assert not missing, missing
    assert set(M.EXPORTS) <= set(declared)


def _struct_body(text, name):
    """Body of `typedef struct { ... } name;` (the struct right before the name)."""
    head = text[:text.index("} " + name + ";")]
    return head[head.rindex("typedef struct {") + len("typedef struct {"):]


def _field_order(body, names):
    order = []
    for f in re.findall(r"\b(" + "|".join(names) + r")\b", body):
        if f not in order:
            order.append(f)
    return order


def test_binding_structs_match_header():
    """Field order of mmgap_problem, mmgap_cim_params, mmgap_schedule and
    mmgap_job as declared in the header."""
    text = open(os.path.join(ROOT, "include", "mmgap.h")).read()
    for name, cls in (("mmgap_problem", M.Problem), ("mmgap_cim_params", M.CimParams),
                      ("mmgap_schedule", M.Schedule), ("mmgap_job", M.Job),
                      ("mmgap_server_stats_t", M.ServerStats)):
        names = [f[0] for f in cls._fields_]
        assert _field_order(_struct_body(text, name), names) == names, name


def test_product_does_not_import_the_oracle():
    """The GPU library and its binding never load the CPU oracle."""
    pkg = os.path.dirname(M.__file__)
    for dirpath, _, files in os.walk(pkg):
        for fn in files:
            if fn.endswith((".py", ".hip", ".h", ".cpp")):
                text = open(os.path.join(dirpath, fn)).read()
                assert "oracle" not in text.lower() or fn == "__init__.py" and "oracle" not in text
