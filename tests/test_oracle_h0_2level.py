"""Pins of the oracle's two-level zero-velocity preconditioner (Section 2.2
names the two-level coarse-grid approximation as the default; the reading
is the zero-velocity Hessian H0 = L_0 + g g^T inverted on the half-resolution
grid for the Fourier band that grid represents, |k_d| < n_d / 4, and the
spectral L^-1 above the band).  CPU only.

Each pin fixes the result by something other than the routine itself:
  * no data term (constant template): H0 = L_0, so the preconditioner is the
    spectral L^-1 on both bands (one inner step is exact);
  * input above the band: the coarse solve sees nothing, z = L^-1 r whatever
    the template;
  * input inside the band with a converged inner solve: z is the prolonged
    solution of the coarse system, assembled here as a dense matrix from
    numpy FFTs and a numpy FD8 stencil and solved by numpy.linalg.solve."""
import numpy as np
import pytest

from paper_2209_08189_amd import synth

BETA = 5e-3
FD8 = (4 / 5, -1 / 5, 4 / 105, -1 / 280)


def kvec(n):
    return np.fft.fftfreq(n, 1.0 / n)


def band_limit(u, nc):
    """Keep the Fourier modes with |k_d| < nc/2 on every axis (numpy)."""
    U = np.fft.fftn(u)
    n = u.shape[0]
    k = kvec(n)
    m = np.abs(k) < nc / 2
    U = U * (m[:, None, None] & m[None, :, None] & m[None, None, :])
    return np.fft.ifftn(U).real


def restrict(u, nc):
    """Spectral restriction to an nc^3 grid (numpy): the kept band sampled on
    the coarse nodes, which are every second fine node."""
    n = u.shape[0]
    return band_limit(u, nc)[:: n // nc, :: n // nc, :: n // nc]


def fd8_grad(u):
    """8th-order central differences on the periodic grid [0, 2 pi)^3 (numpy)."""
    n = u.shape[0]
    h = 2 * np.pi / n
    g = np.zeros((3,) + u.shape)
    for ax in range(3):
        for j, c in enumerate(FD8, start=1):
            g[ax] += c * (np.roll(u, -j, axis=ax) - np.roll(u, j, axis=ax))
        g[ax] /= h
    return g


def problem(orc, n, template):
    shape = (n,) * 3
    o = orc.Oracle(shape, nt=2, beta=BETA)
    o.set_images(template, synth.smooth_random_field(shape, 71, kmax=3.0))
    o.set_velocity(np.zeros((3,) + shape))
    return o


def test_two_level_without_data_term_is_the_spectral_preconditioner(orc):
    n = 16
    o = problem(orc, n, np.full((n,) * 3, 0.3))
    r = synth.random_field((3, n, n, n), 72)
    o.set_precond(0)
    z_sp = o.precond(r)
    o.set_precond(2, 1)
    z = o.precond(r)
    assert np.linalg.norm(z - z_sp) <= 1e-12 * np.linalg.norm(z_sp)


def test_two_level_above_the_band_is_the_spectral_preconditioner(orc):
    n = 16
    o = problem(orc, n, synth.smooth_random_field((n,) * 3, 73, kmax=4.0))
    r = synth.random_field((3, n, n, n), 74)
    r = r - np.stack([band_limit(r[c], n // 2) for c in range(3)])   # modes above the band only
    o.set_precond(0)
    z_sp = o.precond(r)
    o.set_precond(2, 8)
    z = o.precond(r)
    assert np.linalg.norm(z - z_sp) <= 1e-12 * np.linalg.norm(z_sp)


def test_two_level_in_band_converged_equals_dense_coarse_solve(orc):
    n, nc = 16, 8
    m0 = synth.smooth_random_field((n,) * 3, 75, kmax=3.0)
    o = problem(orc, n, m0)
    r = synth.random_field((3, n, n, n), 76)
    r = np.stack([band_limit(r[c], nc) for c in range(3)])          # inside the band
    o.set_precond(2, 400)
    z = o.precond(r)
    # dense coarse operator H0_c = L_0 + g g^T on the 8^3 grid, column by column
    g = fd8_grad(restrict(m0, nc))
    k = kvec(nc)
    ksq = k[:, None, None] ** 2 + k[None, :, None] ** 2 + k[None, None, :] ** 2
    Nc = nc ** 3

    def H0c(x):
        x = x.reshape(3, nc, nc, nc)
        y = np.stack([np.fft.ifftn(BETA * ksq * np.fft.fftn(x[c])).real + BETA * x[c].mean() for c in range(3)])
        y += (g * x).sum(axis=0)[None] * g
        return y.ravel()

    H = np.stack([H0c(e) for e in np.eye(3 * Nc)], axis=1)
    rc = np.stack([restrict(r[c], nc) for c in range(3)]).ravel()
    zc = np.linalg.solve(H, rc).reshape(3, nc, nc, nc)
    # prolongation of a coarse field: its Fourier modes zero-padded to the fine grid
    zf = np.zeros((3, n, n, n))
    for c in range(3):
        Zc = np.fft.fftn(zc[c]) * (n / nc) ** 3
        kc = kvec(nc)
        keep = np.abs(kc) < nc / 2
        Zf = np.zeros((n, n, n), dtype=complex)
        idx = np.where(keep)[0]
        fi = np.mod(kc[idx].astype(int), n)
        Zf[np.ix_(fi, fi, fi)] = Zc[np.ix_(idx, idx, idx)]
        zf[c] = np.fft.ifftn(Zf).real
    err = np.linalg.norm(z - zf) / np.linalg.norm(zf)
    assert err < 1e-8, err


def test_two_level_pcg_between_spectral_and_full_resolution(orc):
    """On the Gauss-Newton system at v = 0 the two-level preconditioner needs
    no more PCG iterations than the spectral one and no fewer than the
    full-resolution H0 (both inner solves converged)."""
    n = 32
    shape = (n,) * 3
    m0 = synth.trig_template(shape)
    o = problem(orc, n, m0)
    rhs = -o.gradient_l2()
    counts = {}
    for kind, inner in ((0, 0), (2, 200), (1, 200)):
        o.set_precond(kind, inner)
        _, its, _ = o.pcg(rhs, 200, 1e-6)
        counts[kind] = its
    print("PCG iterations spectral / two-level / full H0:", counts)
    assert counts[1] <= counts[2] <= counts[0], counts
