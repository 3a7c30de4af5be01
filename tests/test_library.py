"""The C-ABI library loads and exports every entry point its header declares (no GPU needed)."""
import ctypes
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "ising.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(ising_[a-z0-9_]+)\s*\(", src)))


def test_header_declares_entry_points():
    names = _declared()
    for must in ("ising_create", "ising_destroy", "ising_solve", "ising_solve_dev", "ising_energy_dev",
                 "ising_prune_dev", "ising_unprune_dev", "ising_ds_dev", "ising_select_dev"):
        assert must in names


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(os.path.join(ROOT, "paper_2312_05837_amd", "libising.so"))
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_covers_every_declared_symbol():
    import paper_2312_05837_amd as P
    assert sorted(P.exported_symbols()) == _declared()
    for n in _declared():
        assert callable(getattr(P, n)), n
