"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle.

This module draws and samples inputs only; it holds none of the registration
method's arithmetic (no transport, no derivatives, no solver).  Where an input
is defined as "an image transported by a velocity" the caller performs that
transport with whichever implementation it is exercising.

Workloads (periodic grid on [0, 2 pi)^3, node-centred x_i = 2 pi i / N):

* ``trig_template`` / ``trig_velocity``: the closed-form 64^3 problem:
  m0 = (sin^2 x1 + sin^2 x2 + sin^2 x3) / 3 and
  v* = a (sin x3 cos x2 sin x2, sin x1 cos x3 sin x3, sin x2 cos x1 sin x1).
* ``phantom``: brain-like piecewise-constant phantom standing in for the
  paper's 256^3 T1 brain MRI (MUSE/NIREP): 4 classes (background, CSF-, GM-
  and WM-like) from thresholded sums of periodic Gaussian blobs, smoothed with
  a Gaussian of sigma = 1 voxel, intensities in [0, 1].
* ``smooth_velocity``: random band-limited velocity (|k| <= kmax) scaled to a
  given maximum displacement in voxels over unit time.
* ``noise``: independent N(0, sigma^2) noise fields.
"""
import numpy as np
import scipy.fft as sfft

# threads for the FFTs below (-1: all cores; worker pools set 1)
FFT_WORKERS = -1

TWO_PI = 2.0 * np.pi


def grid(shape):
    """Node coordinates x_d = 2 pi i_d / N_d as three broadcastable arrays."""
    n1, n2, n3 = shape
    x1 = (TWO_PI * np.arange(n1) / n1)[:, None, None]
    x2 = (TWO_PI * np.arange(n2) / n2)[None, :, None]
    x3 = (TWO_PI * np.arange(n3) / n3)[None, None, :]
    return x1, x2, x3


def trig_template(shape):
    x1, x2, x3 = grid(shape)
    m = (np.sin(x1) ** 2 + np.sin(x2) ** 2 + np.sin(x3) ** 2) / 3.0
    return np.broadcast_to(m, shape).copy()


def trig_velocity(shape, amplitude=0.5):
    x1, x2, x3 = grid(shape)
    v = np.empty((3,) + tuple(shape))
    v[0] = np.broadcast_to(np.sin(x3) * np.cos(x2) * np.sin(x2), shape)
    v[1] = np.broadcast_to(np.sin(x1) * np.cos(x3) * np.sin(x3), shape)
    v[2] = np.broadcast_to(np.sin(x2) * np.cos(x1) * np.sin(x1), shape)
    return amplitude * v


def _fft_k(n):
    return np.fft.fftfreq(n, d=1.0 / n)


def phantom(shape, seed, n_blobs=(20, 40), sigma=(8.0, 30.0), smooth_sigma=1.0,
            intensities=(0.0, 0.3, 0.6, 0.9), bg_frac=0.15):
    """Brain-like phantom.  Returns (image float64 in [0,1], labels uint8 in 0..3).

    Blob centres are uniform in [0.2 N, 0.8 N]^3 so the object sits in a zero
    background (the images are periodic); sigma in voxels; amplitudes in
    [0.5, 1].  Voxels with S < bg_frac * max S are background; the foreground
    is split into three classes at the 1/3 and 2/3 quantiles of S.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    shape = tuple(int(s) for s in shape)
    nb = int(rng.integers(n_blobs[0], n_blobs[1] + 1))
    axes = [np.arange(n, dtype=np.float64) for n in shape]
    # S = sum_b a_b g1_b (x) g2_b (x) g3_b: the blob profiles are separable,
    # so S is one (n1 x nb) (nb x n2 n3) product
    G = [np.empty((nb, n)) for n in shape]
    for b in range(nb):
        c = [rng.uniform(0.2 * n, 0.8 * n) for n in shape]
        s = rng.uniform(sigma[0], sigma[1])
        a = rng.uniform(0.5, 1.0)
        for ax, n, cc, Gd in zip(axes, shape, c, G):
            d = np.abs(ax - cc)
            d = np.minimum(d, n - d)                      # periodic distance
            Gd[b] = np.exp(-0.5 * (d / s) ** 2)
        G[0][b] *= a
    G23 = (G[1][:, :, None] * G[2][:, None, :]).reshape(nb, -1)
    S = (G[0].T @ G23).reshape(shape)
    fg = S >= bg_frac * S.max()
    q1, q2 = np.quantile(S[fg], [1.0 / 3.0, 2.0 / 3.0])
    labels = np.zeros(shape, dtype=np.uint8)
    labels[fg & (S < q1)] = 1
    labels[fg & (S >= q1) & (S < q2)] = 2
    labels[fg & (S >= q2)] = 3
    img = np.asarray(intensities, dtype=np.float64)[labels]
    if smooth_sigma > 0:
        k1, k2, k3 = (_fft_k(n) for n in shape)
        h = [TWO_PI / n for n in shape]
        # Gaussian of smooth_sigma voxels as a Fourier multiplier
        mult = (np.exp(-0.5 * (smooth_sigma * h[0] * k1) ** 2)[:, None, None]
                * np.exp(-0.5 * (smooth_sigma * h[1] * k2) ** 2)[None, :, None]
                * np.exp(-0.5 * (smooth_sigma * h[2] * k3[: shape[2] // 2 + 1]) ** 2)[None, None, :])
        img = sfft.irfftn(sfft.rfftn(img, workers=FFT_WORKERS) * mult, s=shape, workers=FFT_WORKERS)
    return np.clip(img, 0.0, 1.0), labels


def smooth_velocity(shape, seed, kmax=8.0, max_disp_voxels=6.0):
    """Random velocity: complex N(0,1) Fourier coefficients on 1 <= |k| <= kmax
    weighted by 1/(1+|k|^2), real part of the inverse FFT, scaled so that
    max_x |v(x)|_2 = max_disp_voxels * (2 pi / N) (displacement over t in [0,1])."""
    rng = np.random.Generator(np.random.PCG64(seed))
    shape = tuple(int(s) for s in shape)
    k1, k2, k3 = (_fft_k(n) for n in shape)
    ksq = k1[:, None, None] ** 2 + k2[None, :, None] ** 2 + k3[None, None, :] ** 2
    band = (ksq >= 1.0) & (ksq <= kmax * kmax)
    idx = np.nonzero(band)
    v = np.empty((3,) + shape)
    for c in range(3):
        coef = np.zeros(shape, dtype=np.complex128)
        z = rng.standard_normal(len(idx[0])) + 1j * rng.standard_normal(len(idx[0]))
        coef[idx] = z / (1.0 + ksq[idx])
        v[c] = sfft.ifftn(coef, workers=FFT_WORKERS).real
    vmax = np.sqrt((v ** 2).sum(axis=0)).max()
    h = TWO_PI / max(shape)
    return v * (max_disp_voxels * h / vmax)


def noise(shape, seed, sigma=0.02):
    rng = np.random.Generator(np.random.PCG64(seed))
    return sigma * rng.standard_normal(tuple(shape))


def random_field(shape, seed, lo=-1.0, hi=1.0):
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.uniform(lo, hi, size=tuple(shape))


def smooth_random_field(shape, seed, kmax=4.0):
    """Band-limited random scalar field (real part of random Fourier modes
    with |k| <= kmax), normalised to max |u| = 1."""
    rng = np.random.Generator(np.random.PCG64(seed))
    shape = tuple(int(s) for s in shape)
    k1, k2, k3 = (_fft_k(n) for n in shape)
    ksq = k1[:, None, None] ** 2 + k2[None, :, None] ** 2 + k3[None, None, :] ** 2
    idx = np.nonzero(ksq <= kmax * kmax)
    coef = np.zeros(shape, dtype=np.complex128)
    coef[idx] = rng.standard_normal(len(idx[0])) + 1j * rng.standard_normal(len(idx[0]))
    u = sfft.ifftn(coef, workers=FFT_WORKERS).real
    return u / np.abs(u).max()


# ----------------------------------------------------------- large grids
# The same recipes for grids where full 3D FP64 work is too slow on the
# host: FP32 arrays, the blob sum as one GEMM, the band-limited velocity
# evaluated separably from its few Fourier modes.

def phantom_large(shape, seed, n_blobs=(380, 420), sigma=(4.0, 60.0), smooth_sigma=1.0, texture=0.05,
                  kband=(64.0, 256.0), intensities=(0.0, 0.3, 0.6, 0.9), bg_frac=0.15, log=None):
    """Phantom of the large-grid configuration (FP32): blobs as in phantom()
    (more of them, wider range of widths), the same 4 classes, Gaussian
    smoothing, then band-limited texture (random complex coefficients of
    flat amplitude on kband[0] <= |k| <= kband[1], scaled to standard
    deviation `texture`) added inside the foreground; clipped to [0, 1].
    Returns (image float32, labels uint8); log(msg) reports the steps."""
    log = log or (lambda m: None)
    rng = np.random.Generator(np.random.PCG64(seed))
    shape = tuple(int(s) for s in shape)
    nb = int(rng.integers(n_blobs[0], n_blobs[1] + 1))
    axes = [np.arange(n, dtype=np.float64) for n in shape]
    G = [np.empty((nb, n), dtype=np.float32) for n in shape]
    for b in range(nb):
        c = [rng.uniform(0.2 * n, 0.8 * n) for n in shape]
        s = rng.uniform(sigma[0], sigma[1])
        a = rng.uniform(0.5, 1.0)
        for ax, n, cc, Gd in zip(axes, shape, c, G):
            d = np.abs(ax - cc)
            d = np.minimum(d, n - d)
            Gd[b] = np.exp(-0.5 * (d / s) ** 2)
        G[0][b] *= a
    G23 = (G[1][:, :, None] * G[2][:, None, :]).reshape(nb, -1)
    S = (G[0].T @ G23).reshape(shape)
    del G23
    log("blob sum of %d blobs" % nb)
    thr = bg_frac * S.max()
    fg = S >= thr
    q1, q2 = np.quantile(S[fg], [1.0 / 3.0, 2.0 / 3.0])
    labels = np.zeros(shape, dtype=np.uint8)
    labels[fg] = 1
    labels[S >= q1] = 2
    labels[S >= q2] = 3
    labels[~fg] = 0
    del S, fg
    log("labels")
    img = np.asarray(intensities, dtype=np.float32)[labels]
    k1, k2, k3 = (_fft_k(n) for n in shape)
    h = [TWO_PI / n for n in shape]
    if smooth_sigma > 0:
        mult = (np.exp(-0.5 * (smooth_sigma * h[0] * k1) ** 2)[:, None, None]
                * np.exp(-0.5 * (smooth_sigma * h[1] * k2) ** 2)[None, :, None]
                * np.exp(-0.5 * (smooth_sigma * h[2] * k3[: shape[2] // 2 + 1]) ** 2)[None, None, :]).astype(np.float32)
        img = sfft.irfftn(sfft.rfftn(img, workers=FFT_WORKERS) * mult, s=shape, workers=FFT_WORKERS).astype(np.float32)
        del mult
        log("smoothing")
    if texture > 0:
        kh = k3[: shape[2] // 2 + 1]
        ksq = (k1.astype(np.float32)[:, None, None] ** 2 + k2.astype(np.float32)[None, :, None] ** 2
               + kh.astype(np.float32)[None, None, :] ** 2)
        band = (ksq >= kband[0] ** 2) & (ksq <= kband[1] ** 2)
        del ksq
        nz = int(band.sum())
        coef = np.zeros(band.shape, dtype=np.complex64)
        coef[band] = (rng.standard_normal(nz, dtype=np.float32) + 1j * rng.standard_normal(nz, dtype=np.float32))
        del band
        tex = sfft.irfftn(coef, s=shape, workers=FFT_WORKERS).astype(np.float32)
        del coef
        tex *= texture / max(float(tex.std()), 1e-30)
        img += np.where(labels > 0, tex, np.float32(0.0))
        del tex
        log("texture")
    return np.clip(img, 0.0, 1.0), labels


def smooth_velocity_large(shape, seed, kmax=8.0, max_disp_voxels=20.0, log=None):
    """Band-limited velocity of smooth_velocity() (complex N(0,1) modes on
    1 <= |k| <= kmax weighted by 1 / (1 + |k|^2), real part), evaluated as
    a separable sum over the (2 kmax + 1)^3 modes in FP32; scaled to the
    given maximum displacement.  Returns float32 [3, n1, n2, n3]."""
    rng = np.random.Generator(np.random.PCG64(seed))
    shape = tuple(int(s) for s in shape)
    K = int(np.floor(kmax))
    kk = np.arange(-K, K + 1, dtype=np.float64)
    ksq = kk[:, None, None] ** 2 + kk[None, :, None] ** 2 + kk[None, None, :] ** 2
    band = (ksq >= 1.0) & (ksq <= kmax * kmax)
    E = [np.exp(1j * np.outer(kk, TWO_PI * np.arange(n) / n)) for n in shape]     # [2K+1, n]
    v = np.empty((3,) + shape, dtype=np.float32)
    for c in range(3):
        C = np.zeros(ksq.shape, dtype=np.complex128)
        nz = int(band.sum())
        C[band] = (rng.standard_normal(nz) + 1j * rng.standard_normal(nz)) / (1.0 + ksq[band])
        T1 = C.reshape(-1, 2 * K + 1) @ E[2]                                      # [a b, x3]
        T1 = T1.reshape(2 * K + 1, 2 * K + 1, shape[2])
        T2 = np.einsum("bj,abk->ajk", E[1], T1).reshape(2 * K + 1, -1)           # [a, x2 x3]
        E1 = E[0].T                                                               # [x1, a]
        v[c] = ((E1.real.astype(np.float32) @ T2.real.astype(np.float32))
                - (E1.imag.astype(np.float32) @ T2.imag.astype(np.float32))).reshape(shape)
        if log:
            log("velocity component %d" % c)
    vmax = 0.0
    for i in range(shape[0]):
        vmax = max(vmax, float(np.sqrt((v[:, i].astype(np.float64) ** 2).sum(axis=0)).max()))
    h = TWO_PI / max(shape)
    v *= np.float32(max_disp_voxels * h / vmax)
    return v


def noise32(shape, seed, sigma):
    """N(0, sigma^2) noise in FP32 (large grids)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return (rng.standard_normal(tuple(int(s) for s in shape), dtype=np.float32) * np.float32(sigma))


# ------------------------------------------------------------------ SYN
# The paper's synthetic resolution study (Section 4, SYN): a template made
# of ten star-shaped solids whose radius is a spherical harmonic, and a
# closed-form velocity of frequency K.  Readings: image coordinates are the
# node coordinates shifted to (-pi, pi]; |Y_l^m| does not depend on the
# azimuth, so the radius is |Re Y_l^m| = N_lm |cos(m (phi + phi_i))|
# |P_l^m(cos(theta + theta_i))| with the physics convention (theta polar,
# phi azimuth); labels are the integer intensities 0..10 (overlaps add).

def syn_coords(shape):
    """Image coordinates in (-pi, pi] per axis (node coordinate - pi)."""
    return [(TWO_PI * np.arange(n) / n - np.pi) for n in shape]


def syn_template(shape, seed, l=8, m=6, n_solids=10, return_params=False, rscale=1.0, log=None):
    """SYN template m0 = sum of n_solids indicator functions (uint8
    intensities 0..n_solids): solid i is {x : |x - c_i| <= |Re Y_l^m(theta +
    dtheta_i, phi + dphi_i)|} with c_i uniform in [-0.4 pi, 0.4 pi]^3 and
    dtheta_i, dphi_i random multiples of pi/2; (theta, phi) are the polar
    and azimuthal angles of x - c_i.  Each solid is evaluated on the
    bounding box of its largest radius only.  rscale multiplies the radius
    (1: the printed |Re Y_l^m|, at most 0.45).  return_params: also the
    list of (centre, dtheta, dphi) per solid.  log: optional callable
    given one progress line per solid."""
    from scipy.special import lpmv
    from math import factorial
    rng = np.random.Generator(np.random.PCG64(seed))
    shape = tuple(int(s) for s in shape)
    norm = np.sqrt((2 * l + 1) / (4 * np.pi) * factorial(l - m) / factorial(l + m))
    xs = np.linspace(-1.0, 1.0, 20001)
    rmax = float(norm * np.abs(lpmv(m, l, xs)).max()) * 1.01 * rscale
    ax = syn_coords(shape)
    h = [TWO_PI / n for n in shape]
    out = np.zeros(shape, dtype=np.uint8)
    params = []
    for _ in range(n_solids):
        c = rng.uniform(-0.4 * np.pi, 0.4 * np.pi, 3)
        dth, dph = (np.pi / 2) * rng.integers(0, 4, 2)
        params.append((c, float(dth), float(dph)))
        sl = []
        for d in range(3):
            lo = max(0, int(np.floor((c[d] - rmax + np.pi) / h[d])))
            hi = min(shape[d], int(np.ceil((c[d] + rmax + np.pi) / h[d])) + 1)
            sl.append(slice(lo, hi))
        y1 = ax[0][sl[0]][:, None, None] - c[0]
        y2 = ax[1][sl[1]][None, :, None] - c[1]
        y3 = ax[2][sl[2]][None, None, :] - c[2]
        rho = np.sqrt(y1 * y1 + y2 * y2 + y3 * y3)
        theta = np.arccos(np.clip(y3 / np.maximum(rho, 1e-300), -1.0, 1.0))
        phi = np.arctan2(y2, y1)
        radius = rscale * norm * np.abs(np.cos(m * (phi + dph))) * np.abs(lpmv(m, l, np.cos(theta + dth)))
        out[sl[0], sl[1], sl[2]] += (rho <= radius).astype(np.uint8)
        if log:
            log("SYN solid %d of %d" % (len(params), n_solids))
    return (out, params) if return_params else out


def syn_velocity(shape, K):
    """SYN velocity: v_x = sum_k k^-1/2 cos(k y) cos(k x), v_y = sum_k
    k^-1/2 sin(k z) sin(k y), v_z = sum_k k^-1/2 cos(k x) cos(k z), k = 1..K,
    with (x, y, z) = (x1, x2, x3) in (-pi, pi].  float32 [3, n1, n2, n3]."""
    shape = tuple(int(s) for s in shape)
    x, y, z = syn_coords(shape)
    v = np.zeros((3,) + shape, dtype=np.float32)
    for k in range(1, int(K) + 1):
        a = np.float32(k ** -0.5)
        cx, cy, cz = (np.cos(k * t).astype(np.float32) for t in (x, y, z))
        sy, sz = (np.sin(k * t).astype(np.float32) for t in (y, z))
        v[0] += a * cx[:, None, None] * cy[None, :, None]
        v[1] += a * sy[None, :, None] * sz[None, None, :]
        v[2] += a * cx[:, None, None] * cz[None, None, :]
    return v
