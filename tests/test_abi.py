"""C ABI checks that need no GPU: the library loads, exports every symbol the
public header declares, and the binding's struct layouts match the header."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mlsgd.h")


def _declared():
    src = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:int|const char\*)\s+(mlsgd_\w+)\s*\(", src, re.M)))


def test_header_declares_entry_points():
    names = _declared()
    for need in ["mlsgd_create", "mlsgd_sample_fields", "mlsgd_solve_state_adjoint",
                 "mlsgd_mlmc_gradient", "mlsgd_step"]:
        assert need in names


def test_library_exports_every_declared_symbol():
    import paper_2606_09291_amd as m
    if not os.path.exists(m.LIB_PATH):
        pytest.skip("libmlsgd.so not built")
    lib = m.lib()
    for name in _declared():
        assert hasattr(lib, name), name
    assert sorted(m.EXPORTS) == _declared()


def test_struct_sizes_match_header():
    """Compile a probe against the header with gcc and compare sizeof/offsetof
    with the ctypes mirrors."""
    import subprocess
    import tempfile
    import paper_2606_09291_amd as m
    probe = r'''
#include <stdio.h>
#include <stddef.h>
#include "mlsgd.h"
int main(void) {
  printf("%zu %zu %zu %zu %zu %zu %zu\n", sizeof(mlsgd_problem), sizeof(mlsgd_solve_stats),
         sizeof(mlsgd_grad_stats), sizeof(mlsgd_step_stats), offsetof(mlsgd_problem, y_d),
         offsetof(mlsgd_grad_stats, ms_total), offsetof(mlsgd_step_stats, eps));
  return 0;
}
'''
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "p.c")
        exe = os.path.join(d, "p")
        open(c, "w").write(probe)
        subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), c, "-o", exe], check=True)
        out = subprocess.run([exe], capture_output=True, text=True, check=True).stdout.split()
    got = [int(x) for x in out]
    want = [ctypes.sizeof(m._Problem), ctypes.sizeof(m._SolveStats), ctypes.sizeof(m._GradStats),
            ctypes.sizeof(m._StepStats), m._Problem.y_d.offset, m._GradStats.ms_total.offset,
            m._StepStats.eps.offset]
    assert got == want


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    import paper_2606_09291_amd as m
    monkeypatch.setattr(m, "_lib", None)
    monkeypatch.setattr(m, "LIB_PATH", str(tmp_path / "nope.so"))
    with pytest.raises(ImportError):
        m.lib()
