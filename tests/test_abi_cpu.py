"""CPU-side checks of the C-ABI library: it loads, exports every entry point
declared in include/subsurf4d.h, and answers the host-only queries."""
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "subsurf4d.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(subsurf4d_[a-z0-9_]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for need in ("subsurf4d_prepare_g", "subsurf4d_step", "subsurf4d_solve"):
        assert need in names


def test_library_exports_every_declared_symbol():
    from paper_2111_11866_amd import binding as B

    L = B.lib()
    for name in declared_functions():
        assert hasattr(L, name), name
    assert set(B.EXPORTED) == set(declared_functions())


def test_host_queries():
    from paper_2111_11866_amd import binding as B

    assert B.version().startswith("subsurf4d")
    assert B.workspace_bytes((24, 24, 24, 8), 8) > 0
    assert B.workspace_bytes((0, 24, 24, 8)) == 0
    assert B.workspace_bytes((24, 24, 24, 8), 8, B.MIXED) > B.workspace_bytes((24, 24, 24, 8), 8)
    assert B.lib().subsurf4d_status_string(-3) == b"workspace too small"
