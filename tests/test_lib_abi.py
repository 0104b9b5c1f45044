"""Host-side checks of the C-ABI library: it loads without a GPU and exports every symbol
include/tcw.h declares; the binding's struct layouts match the header's field lists."""

import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "tcw.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(tcw_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ("tcw_create", "tcw_step", "tcw_trails", "tcw_canon_hash", "tcw_claw_check", "tcw_walk_begin",
                 "tcw_walk_run", "tcw_search", "tcw_target_from_words", "tcw_target_from_channel"):
        assert must in names


def test_library_exports_every_declared_symbol():
    from paper_1606_07413_amd import tcw
    lib = tcw.load()
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing
    # the binding wraps exactly the declared entry points
    assert sorted(tcw.EXPORTED) == declared_functions()


def _c_struct_fields(name):
    text = open(HEADER).read()
    m = re.search(r"typedef struct " + name + r" \{(.*?)\} " + name + ";", text, re.S)
    body = re.sub(r"/\*.*?\*/", "", m.group(1), flags=re.S)
    fields = []
    for decl in body.split(";"):
        decl = decl.strip()
        if not decl:
            continue
        fields.append(re.findall(r"([a-z_0-9]+)\s*(?:\[[^\]]*\])?$", decl)[0])
    return fields


@pytest.mark.parametrize("cname,pyname", [("tcw_space", "Space"), ("tcw_walk_stats", "WalkStats"),
                                          ("tcw_walk_params", "WalkParams"), ("tcw_result", "Result")])
def test_struct_layouts_match_header(cname, pyname):
    from paper_1606_07413_amd import tcw
    py = [f[0] for f in getattr(tcw, pyname)._fields_]
    assert py == _c_struct_fields(cname)


def test_errors_without_gpu_are_loud():
    from paper_1606_07413_amd import tcw
    lib = tcw.load()
    h = ctypes.c_void_p()
    # device 99 does not exist (and on a CPU host there is no device at all)
    assert lib.tcw_create(ctypes.byref(h), 99, None) != 0
    assert lib.tcw_search(None, None, None, None) == -1


def test_default_params_per_n():
    from paper_1606_07413_amd import tcw
    lib = tcw.load()
    for n, walks, lg in [(2, 64, 12), (3, 1 << 16, 20), (4, 1 << 20, 26)]:
        p = tcw.WalkParams()
        lib.tcw_default_params(ctypes.byref(p), n)
        assert p.walks == walks and p.log2_table == lg and p.trail_cap_factor == 20 and p.budget_beta == 16
        assert p.chunk_parallel == 1


def test_binding_refuses_host_tensors():
    """Device-array arguments must be CUDA tensors: a host tensor is refused before any call."""
    import torch
    from paper_1606_07413_amd import tcw
    with pytest.raises(TypeError):
        tcw._dev(torch.zeros(4, dtype=torch.int64), 8, 4, "x", 0)
    assert tcw._dev(None, 8, 4, "x", 0) is None
