"""The C ABI: the library loads and exports every function include/lam.h declares,
and the binding's structs have the C layout.  No GPU calls."""
import ctypes
import os
import re
import subprocess

import pytest

from paper_1111_4363_amd import lam

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lam.h")


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(lam_[a-z_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = _declared_functions()
    for must in ["lam_create", "lam_residual_action", "lam_relax_sweep", "lam_vcycle", "lam_solve_step",
                 "lam_adjoint_step", "lam_destroy", "lam_strerror"]:
        assert must in names


def test_library_exports_every_declared_symbol():
    lib = lam.load_library()
    for name in _declared_functions():
        assert hasattr(lib, name), name


def test_binding_covers_every_declared_symbol():
    assert sorted(lam.SIGNATURES) == _declared_functions()


def test_strerror_names_every_code():
    for code in [0, -1, -2, -3, -4, -5, -6, -7]:
        assert lam.strerror(code) not in ("", "unknown error")


def test_struct_layout_matches_c(tmp_path):
    src = tmp_path / "layout.c"
    src.write_text(r'''
#include <stdio.h>
#include <stddef.h>
#include "lam.h"
#define P(T, f) printf(#T "." #f " %zu\n", offsetof(T, f));
int main(void) {
  printf("lam_grid %zu\nlam_time %zu\nlam_ham %zu\nlam_solver %zu\nlam_stats %zu\n",
         sizeof(lam_grid), sizeof(lam_time), sizeof(lam_ham), sizeof(lam_solver), sizeof(lam_stats));
  P(lam_grid, h) P(lam_grid, block) P(lam_grid, interp) P(lam_grid, coarse_op) P(lam_ham, v0) P(lam_ham, coef)
  P(lam_ham, t_total) P(lam_solver, n_inner) P(lam_solver, time_factor) P(lam_solver, coarse_reduction)
  P(lam_stats, t_solve_ms) P(lam_stats, resid_last) P(lam_stats, coarse_unmet) P(lam_solver, max_split) P(lam_solver, inner_tol)
  P(lam_stats, substeps) P(lam_stats, split_depth)
  return 0;
}
''')
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = dict(line.rsplit(" ", 1) for line in subprocess.run([str(exe)], capture_output=True, text=True,
                                                               check=True).stdout.splitlines())
    assert int(out["lam_grid"]) == ctypes.sizeof(lam.LamGrid)
    assert int(out["lam_time"]) == ctypes.sizeof(lam.LamTime)
    assert int(out["lam_ham"]) == ctypes.sizeof(lam.LamHam)
    assert int(out["lam_solver"]) == ctypes.sizeof(lam.LamSolver)
    assert int(out["lam_stats"]) == ctypes.sizeof(lam.LamStats)
    assert int(out["lam_grid.h"]) == lam.LamGrid.h.offset
    assert int(out["lam_grid.block"]) == lam.LamGrid.block.offset
    assert int(out["lam_grid.interp"]) == lam.LamGrid.interp.offset
    assert int(out["lam_grid.coarse_op"]) == lam.LamGrid.coarse_op.offset
    assert int(out["lam_ham.v0"]) == lam.LamHam.v0.offset
    assert int(out["lam_ham.coef"]) == lam.LamHam.coef.offset
    assert int(out["lam_ham.t_total"]) == lam.LamHam.t_total.offset
    assert int(out["lam_solver.n_inner"]) == lam.LamSolver.n_inner.offset
    assert int(out["lam_solver.time_factor"]) == lam.LamSolver.time_factor.offset
    assert int(out["lam_stats.t_solve_ms"]) == lam.LamStats.t_solve_ms.offset
    assert int(out["lam_stats.resid_last"]) == lam.LamStats.resid_last.offset
    assert int(out["lam_solver.coarse_reduction"]) == lam.LamSolver.coarse_reduction.offset
    assert int(out["lam_stats.coarse_unmet"]) == lam.LamStats.coarse_unmet.offset
    assert int(out["lam_solver.max_split"]) == lam.LamSolver.max_split.offset
    assert int(out["lam_solver.inner_tol"]) == lam.LamSolver.inner_tol.offset
    assert int(out["lam_stats.substeps"]) == lam.LamStats.substeps.offset
    assert int(out["lam_stats.split_depth"]) == lam.LamStats.split_depth.offset


def test_binding_rejects_host_tensors_before_any_call():
    import torch
    with pytest.raises(ValueError):
        lam._ptr(torch.zeros(4, dtype=torch.complex128), torch.complex128, 4, "x")
