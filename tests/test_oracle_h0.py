"""Pins of the oracle's zero-velocity Hessian preconditioner (Section 2.2
names it; its construction is read from the Gauss-Newton Hessian at v = 0).
CPU only.

At v = 0 the full Hessian matvec (transport of the incremental state with
trapezoid sources, incremental adjoint, quadrature) must reduce to
H0 vt = L vt + (grad_h m0 . vt) grad_h m0, so an inner solve run to
convergence inverts the full Hessian there, up to the mean mode, which the
inner operator maps by beta_v like the spectral preconditioner
(H(0) z + beta_v mean(z) = r); a wrong sign, a dropped factor or a
transposed outer product of the data term fails."""
import numpy as np
import pytest

from paper_2209_08189_amd import synth

TWO_PI = 2 * np.pi


def _problem(orc, n=16, beta_w=0.0):
    shape = (n,) * 3
    m0 = synth.smooth_random_field(shape, 90, kmax=4.0)
    m1 = synth.smooth_random_field(shape, 91, kmax=4.0)
    o = orc.Oracle(shape, nt=4, beta=5e-3, beta_w=beta_w)
    o.set_images(m0, m1)
    o.set_velocity(np.zeros((3,) + shape))
    return o, shape


@pytest.mark.parametrize("beta_w", [0.0, 1e-3])
def test_converged_h0_inverts_the_hessian_at_zero(orc, beta_w):
    o, shape = _problem(orc, beta_w=beta_w)
    r = synth.random_field((3,) + shape, 92)
    o.set_precond(1, 400)
    z = o.precond(r)
    Hz = o.matvec_sym(z) + 5e-3 * z.mean(axis=(1, 2, 3), keepdims=True)
    err = np.linalg.norm(Hz - r) / np.linalg.norm(r)
    assert err < 1e-7, err


def test_h0_pcg_at_zero_converges_in_one_step(orc):
    """With a converged inner solve the preconditioner is H(0)^-1 up to the
    mean mode (beta_v there instead of the data term's coupling alone), so
    PCG at v = 0 reaches a 1e-6 residual in at most three outer iterations;
    the spectral preconditioner needs many."""
    o, shape = _problem(orc)
    rhs = -o.gradient_l2()
    o.set_precond(1, 400)
    _, its_h0, _ = o.pcg(rhs, 50, 1e-6)
    o.set_precond(0)
    _, its_sp, _ = o.pcg(rhs, 50, 1e-6)
    assert its_h0 <= 3 and its_sp > 5, (its_h0, its_sp)


def test_h0_one_inner_step_is_a_scaled_spectral_step(orc):
    """One inner CG step from z = 0 is the exact line minimisation along the
    spectral direction: z = (<r, P r> / <P r, H0 P r>) P r."""
    o, shape = _problem(orc)
    r = synth.random_field((3,) + shape, 93)
    o.set_precond(0)
    pr = o.precond(r)
    o.set_precond(1, 1)
    z = o.precond(r)
    H = o.matvec_sym(pr) + 5e-3 * pr.mean(axis=(1, 2, 3), keepdims=True)   # = (L_0 + D) pr at v = 0
    scale = np.sum(r * pr) / np.sum(pr * H)
    assert np.linalg.norm(z - scale * pr) < 1e-10 * np.linalg.norm(z)

