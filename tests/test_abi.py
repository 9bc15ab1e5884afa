"""The C-ABI library loads on the CPU host and exports every function include/wenott.h declares
(no compute calls: there is no GPU here)."""
import ctypes
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "wenott.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(wenott_[a-z0-9_]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = _declared()
    for n in ("wenott_init", "wenott_rhs", "wenott_rk3_step", "wenott_round", "wenott_to_dense"):
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_2405_12301_amd import wenott
    lib = wenott.load()
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing
    assert set(wenott.EXPORTED) <= set(_declared())


def test_host_only_calls_without_a_gpu():
    from paper_2405_12301_amd import wenott
    o = wenott.default_opts()
    assert o.max_sweeps == 4 and o.rounds_per_stage == 1 and o.eps0 == 1e-10
    lib = wenott.load()
    assert lib.wenott_strerror(-5).decode().startswith("non-physical")
    # argument validation happens before any device call
    h = ctypes.c_void_p()
    assert lib.wenott_init(ctypes.byref(h), None, None, 1.4, None, None, None) == wenott.EINVAL
