"""lam_residual_action_noalloc (no context, no allocation, fixed device scratch)
against the context's lam_residual_action on the same inputs: two calls in a
row, the second on a smaller grid, so that the second reads only partial sums
it wrote itself.  Same kernels in the same order, so the outputs agree bit for
bit (rho, sigma and N)."""
import numpy as np
import pytest

from gpu_util import Case, note, t_c, t_r

pytestmark = pytest.mark.gpu

FIELD = dict(kind="sin2+fourier", e0=0.3, omega=2.0, t_total=0.4, coef=[0.2, -0.1, 0.05])


def _compare(case, t0):
    import torch
    from paper_1111_4363_amd import lam
    note(f"no-alloc residual {case} t0={t0}")
    c, l_ = case.random_state()
    c_t, l_t, psi_t = t_c(c), t_c(l_), t_c(case.psi0)
    prop = case.prop()
    rho_ref, sig_ref, N_ref = prop.residual_action(t0, psi_t, c_t, l_t)
    prop.close()
    P, nt = case.npts, case.n_t
    rho = torch.full((P * nt,), float("nan"), dtype=torch.complex128, device="cuda")
    sig = torch.full((P,), float("nan"), dtype=torch.complex128, device="cuda")
    norm = torch.full((1,), float("nan"), dtype=torch.float64, device="cuda")
    code = lam.residual_action_noalloc(case.shape, case.h, t_r(case.v0), nt, case.dt, t0, psi_t, c_t, l_t, rho,
                                       sig, norm, block=case.block, periodic=case.periodic, mass=case.mass,
                                       field_axis=case.field_axis, pulse=case.pulse)
    torch.cuda.synchronize()
    assert code == lam.LAM_OK
    assert torch.equal(rho, rho_ref)
    assert torch.equal(sig, sig_ref)
    assert float(norm.item()) == N_ref
    # the norm alone (no field outputs)
    norm2 = torch.zeros(1, dtype=torch.float64, device="cuda")
    code = lam.residual_action_noalloc(case.shape, case.h, t_r(case.v0), nt, case.dt, t0, psi_t, c_t, l_t, None,
                                       None, norm2, block=case.block, periodic=case.periodic, mass=case.mass,
                                       field_axis=case.field_axis, pulse=case.pulse)
    torch.cuda.synchronize()
    assert code == lam.LAM_OK and float(norm2.item()) == N_ref


def test_noalloc_residual_matches_context_twice_second_smaller():
    _compare(Case(shape=(24, 24, 24), h=0.3, n_t=8, block=(4, 4, 4), pulse=FIELD, seed=3), 0.1)
    _compare(Case(shape=(32, 32), h=0.2, n_t=6, block=(8, 8), periodic=True, pulse=FIELD, seed=4), 0.25)
