"""CPU checks of the boundary: the HIP library loads and exports every symbol the header
declares; the binding's structures match the header's field order; no compute is launched."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pointemray.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(pe_[a-z_0-9]+)\s*\(", src)))


def test_header_declares_expected_api():
    names = _declared()
    for n in ["pe_ctx_create", "pe_scene_create", "pe_solve", "pe_submit", "pe_wait",
              "pe_cancel", "pe_render_gfb", "pe_trace_pixels", "pe_densifier_train_step",
              "pe_densifier_infer", "pe_last_error"]:
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_2408_15583_amd import _native
    if not os.path.exists(_native.LIB_PATH):
        pytest.fail("libpointemray.so is not built; run __graft_entry__.build()")
    L = ctypes.CDLL(_native.LIB_PATH)
    missing = [n for n in _declared() if not hasattr(L, n)]
    assert not missing, missing


def test_binding_covers_every_declared_symbol():
    from paper_2408_15583_amd import _native
    names = set(_native._SIGS) | {"pe_last_error"}
    assert set(_declared()) == names


def _struct_fields(name):
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    m = re.search(r"typedef struct \{([^{}]*)\}\s*" + name + ";", src)
    body = m.group(1)
    fields = []
    for decl in body.split(";"):
        decl = decl.strip()
        if not decl:
            continue
        parts = decl.replace("*", " ").split()
        ty_and_names = " ".join(parts[1:]) if parts[0] == "const" else " ".join(parts)
        toks = ty_and_names.split(",")
        first = toks[0].split()
        fields.append(first[-1].split("[")[0])
        fields += [t.strip().split("[")[0] for t in toks[1:]]
    return fields


@pytest.mark.parametrize("name", ["pe_scene_desc", "pe_solve_desc", "pe_stats", "pe_result",
                                  "pe_gfb_set", "pe_fuse_desc"])
def test_struct_layout_matches_header(name):
    from paper_2408_15583_amd import _native
    py = [f for f, _ in getattr(_native, name)._fields_]
    assert py == _struct_fields(name)


def test_last_error_is_callable_without_device():
    from paper_2408_15583_amd import _native
    if not os.path.exists(_native.LIB_PATH):
        pytest.skip("library not built")
    s = _native.lib().pe_last_error()
    assert s is not None


def test_product_does_not_touch_oracle():
    """The product package never imports or loads the oracle."""
    pkg = os.path.join(ROOT, "paper_2408_15583_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".cpp", ".hip", ".h")):
                txt = open(os.path.join(dirpath, f)).read()
                assert "oracle" not in txt.lower().replace("oracle-free", ""), f
