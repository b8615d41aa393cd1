"""The C-ABI library loads and exports every function include/ba.h declares
(no compute calls: this runs without a GPU)."""
import ctypes
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "ba.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^[A-Za-z_][\w \*]*?\b(ba_\w+)\s*\(", src, flags=re.M)
    return sorted(set(n for n in names))


def test_header_declares_the_boundary():
    names = declared_functions()
    for n in ("ba_create", "ba_add_observations", "ba_lm_step", "ba_solve", "ba_destroy", "ba_last_error",
              "ba_gnn_create", "ba_gnn_train_step", "ba_set_gnn_weights"):
        assert n in names, n


def test_library_exports_every_declared_function():
    lib = ctypes.CDLL(os.path.join(ROOT, "paper_2609_04026_amd", "libba.so"))
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_signatures_cover_the_header():
    from paper_2609_04026_amd import binding
    src = open(binding.__file__).read()
    missing = [n for n in declared_functions() if f'"{n}"' not in src]
    assert not missing, missing
