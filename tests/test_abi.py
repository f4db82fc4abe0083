"""The C ABI library loads and exports every function include/pmwa.h
declares; parameter validation needs no GPU."""
import math
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "pmwa.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(pmwa_[a-z_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    from paper_1307_0328_amd import pmwa as P
    lib = P.lib()
    names = declared_functions()
    assert len(names) >= 10
    for n in names:
        assert hasattr(lib, n), n
    assert set(P.EXPORTS) == set(names)


def test_default_event_cap_and_validation():
    from paper_1307_0328_amd import pmwa as P
    ok = P.make_params(L=64, beta=16.0, V=1.0, mu=0.5, eta=0.05, dom_x=8, dom_y=8, dom_tau=2)
    cap = P.pmwa_default_event_cap(ok)
    assert 64 <= cap <= 512 and cap % 8 == 0
    for bad in [dict(L=2), dict(L=4, dom_x=3), dict(L=4, dom_x=4), dict(L=4, eta=0.0),
                dict(L=4, beta=-1.0), dict(L=4, chain_id=1 << 24), dict(L=4, ticks_log2=31),
                dict(L=4, eta=1.0, beta=9.0), dict(L=4, dom_tau=65)]:
        assert P.pmwa_default_event_cap(P.make_params(**bad)) == P.PMWA_EINVAL, bad
    assert P.lib().pmwa_strerror(P.PMWA_EOVERFLOW).startswith(b"capacity")


def test_create_rejects_bad_options_without_a_gpu():
    """Option ranges are checked before any device call."""
    import ctypes as C
    from paper_1307_0328_amd import pmwa as P
    arr = (P.pmwa_params * 1)(P.make_params(L=8, beta=4.0, dom_x=1, dom_y=1, dom_tau=1))
    for field, value in [("vertex_rows", 4), ("vertex_rows", 129), ("groups", 65), ("scatter_mode", 3),
                         ("event_cap", 40000), ("scatter_lds", 200 * 1024), ("vertex_mode", 4)]:
        o = P.pmwa_opts()
        setattr(o, field, value)
        h = C.c_void_p()
        assert P.lib().pmwa_create(arr, 1, C.byref(o), C.byref(h)) == P.PMWA_EINVAL, field
        assert not h.value
