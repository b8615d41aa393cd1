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


def test_binding_structures_match_the_header(tmp_path):
    """Every ctypes structure of the binding has the size and field offsets
    that a C compiler gives the header's struct of the same name."""
    import shutil
    import subprocess
    import pytest
    from paper_2609_04026_amd import binding
    if shutil.which("gcc") is None:
        pytest.skip("gcc is not available")
    structs = {"ba_loss": binding.Loss, "ba_problem_desc": binding.ProblemDesc,
               "ba_solve_options": binding.SolveOptions, "ba_step_report": binding.StepReport,
               "ba_summary": binding.Summary, "ba_gnn_batch": binding.GnnBatch}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "ba.h"', "int main(void) {"]
    expect = []
    for cname, cls in structs.items():
        lines.append(f'printf("%zu\\n", sizeof({cname}));')
        expect.append(ctypes.sizeof(cls))
        for f, _ in cls._fields_:
            lines.append(f'printf("%zu\\n", offsetof({cname}, {f.rstrip("_")}));')
            expect.append(getattr(cls, f).offset)
    lines += ["return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = [int(v) for v in subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split()]
    assert got == expect
