"""CPU checks of the built library: it loads and exports every entry point
that include/ccm.h declares (no device calls)."""
import ctypes
import os
import re

import paper_2501_15964_amd as ccm

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    text = open(os.path.join(ROOT, "include", "ccm.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ccm_[a-z0-9_]+)\s*\(", text)))


def test_header_symbols_exported():
    L = ccm.lib()
    names = declared_symbols()
    assert "ccm_solve_path" in names and "ccm_build_knn_graph" in names
    for name in names:
        assert hasattr(L, name), name
    assert sorted(ccm.EXPORTED_SYMBOLS) == names


def test_struct_sizes():
    assert ctypes.sizeof(ccm.CcmOptions) == 80
    assert ctypes.sizeof(ccm.CcmStats) == 144
    o = ccm.ccm_default_options()
    assert o.method == 0 and o.max_outer == 300 and o.cg_max_iter == 500
    assert o.locality == -1 and o.time_budget_s == 0.0 and o.window_chunk == 0
    assert o.dual_scale == -1
    assert ccm.ccm_version().startswith("libccm")


def test_binding_wraps_every_compute_entry_point():
    import paper_2501_15964_amd as pkg
    helpers = {"ccm_status_string", "ccm_last_error"}
    for name in pkg.EXPORTED_SYMBOLS:
        if name not in helpers:
            assert name in pkg.__all__ and callable(getattr(pkg, name)), name


def _header_struct_fields(name):
    text = open(os.path.join(ROOT, "include", "ccm.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    end = re.search(r"\}\s*" + name + r"\s*;", text).start()
    body = text[text.rindex("typedef struct {", 0, end) + len("typedef struct {"):end]
    fields = []
    for decl in body.split(";"):
        decl = decl.strip()
        if not decl:
            continue
        ctype, names = decl.split(None, 1)
        for nm in names.split(","):
            fields.append(re.sub(r"\[.*\]", "", nm).strip())
    return fields


def test_binding_structs_follow_the_header():
    # the ctypes layouts name the header's fields in the header's order, so a
    # field added to one side only fails here instead of shifting the others
    for cname, pyclass in (("ccm_options", ccm.CcmOptions), ("ccm_stats", ccm.CcmStats),
                           ("ccm_instance", ccm.CcmInstance)):
        assert [f[0] for f in pyclass._fields_] == _header_struct_fields(cname), cname
