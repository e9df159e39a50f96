"""Pins of the oracle's Jacobian determinant J = det grad y (the map with
m(1) = m0 o y; Section 3.4 bounds it by [J_min, 1/J_min]) against closed
forms.  CPU only.

The compressible 1D flow v = (a sin x1, 0, 0) integrates exactly:
tan(x(t)/2) = tan(x0/2) exp(a t), so y(x) solves tan(y/2) = exp(-a) tan(x/2)
and dy/dx = exp(-a) / (cos^2(x/2) + exp(-2a) sin^2(x/2)).  A wrong sign of
the source gives 1/J, a dropped Heun term first order in time, a wrong foot
the wrong profile."""
import numpy as np

from paper_2209_08189_amd import synth

TWO_PI = 2 * np.pi


def exact_1d(x1, a):
    return np.exp(-a) / (np.cos(x1 / 2) ** 2 + np.exp(-2 * a) * np.sin(x1 / 2) ** 2)


def _J(orc, shape, v, nt):
    o = orc.Oracle(shape, nt=nt)
    z = np.zeros(shape)
    o.set_images(z, z)
    o.set_velocity(v)
    return o.jacobian_det()


def test_jacobian_compressible_1d_flow_second_order(orc):
    shape = (64, 16, 16)
    a = 0.5
    x1, _, _ = synth.grid(shape)
    v = np.zeros((3,) + shape)
    v[0] = np.broadcast_to(a * np.sin(x1), shape)
    ref = np.broadcast_to(exact_1d(x1, a), shape)
    errs = []
    for nt in (4, 8, 16):
        J = _J(orc, shape, v, nt)
        errs.append(np.abs(J - ref).max())
    assert errs[-1] < 2e-3, errs
    assert 3.0 < errs[0] / errs[1] < 5.0 and 3.0 < errs[1] / errs[2] < 5.0, errs
    # volume is preserved: the mean of det grad y over the torus is 1
    assert abs(_J(orc, shape, v, 16).mean() - 1.0) < 1e-3
    # the extremes: exp(-a) at x1 = 0 (compression of y) and exp(a) at pi
    J = _J(orc, shape, v, 16)
    assert abs(J.min() - np.exp(-a)) < 2e-3 and abs(J.max() - np.exp(a)) < 2e-3


def test_jacobian_divergence_free_is_one(orc):
    """v = (sin x2, sin x3, sin x1): each component is constant along its
    own axis, so the FD8 divergence vanishes exactly, the factor is 1 and
    the interpolation of the constant 1 reproduces it: J = 1 to rounding."""
    shape = (16, 16, 16)
    x1, x2, x3 = synth.grid(shape)
    v = np.stack([np.broadcast_to(f, shape) for f in (np.sin(x2), np.sin(x3), np.sin(x1))])
    J = _J(orc, shape, v, 4)
    assert np.abs(J - 1.0).max() < 1e-13


def test_jacobian_zero_and_constant_velocity(orc):
    shape = (16, 32, 16)
    assert np.array_equal(_J(orc, shape, np.zeros((3,) + shape), 4), np.ones(shape))
    v = np.zeros((3,) + shape)
    v[1] = 0.37
    assert np.abs(_J(orc, shape, v, 4) - 1.0).max() < 1e-13
