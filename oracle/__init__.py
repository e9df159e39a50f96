"""FP64 CPU oracle for the CLAIRE registration hot path (arXiv 2209.08189).

TEST INFRASTRUCTURE ONLY: the test suite, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` are the only callers.  It shares no code with
the HIP library; the numerical work is in ``claire_oracle.c`` (plain C, FP64),
this module only marshals numpy arrays.

Readings of the paper that the oracle fixes (grid nodes x_i = 2 pi i / N,
Heun RK2 feet, cubic Lagrange on floor(p)-1..floor(p)+2, central FD8, trapezoid
time quadrature, H1-seminorm regulariser with K = I, spectral preconditioner
(beta A)^-1 with the k = 0 mode mapped to 1/beta, PCG/Armijo constants, and
for beta_w > 0 the H1 norm of div v with spectral derivatives, K = beta A L^-1)
are listed in ``claire_oracle.c`` beside each function.
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "claire_oracle.c")
_SRCS = [_SRC, os.path.join(_HERE, "conv_oracle.c")]
_LIB = os.path.join(_HERE, "libclaire_oracle.so")
_lib = None

_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int)


def stale():
    """True if the compiled oracle is missing or older than its sources."""
    return not os.path.exists(_LIB) or os.path.getmtime(_LIB) < max(os.path.getmtime(f) for f in _SRCS)


def build(force=True):
    """Compile the oracle with gcc -O2 -fopenmp (no fast-math).  With
    force=False only when the library is missing or stale.  Called by the
    package build and at the start of a test session, never from a process
    that has already initialised the GPU."""
    if not force and not stale():
        return _LIB
    tmp = _LIB + ".tmp"
    cmd = ["gcc", "-O2", "-fopenmp", "-std=c11", "-fPIC", "-shared", "-Wall",
           "-o", tmp, *_SRCS, "-lm"]
    subprocess.check_call(cmd)
    os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        if stale():
            raise RuntimeError("the oracle library %s is missing or older than its sources; "
                               "build it first with oracle.build() (or __graft_entry__.build())" % _LIB)
        L = ctypes.CDLL(_LIB)
        i, d = ctypes.c_int, ctypes.c_double
        vp = ctypes.c_void_p
        sig = {
            "orc_interp": (None, [i, i, i, _dp, _dp, _dp]),
            "orc_interp_point": (d, [i, i, i, _dp, d, d, d]),
            "orc_grad": (None, [i, i, i, _dp, _dp]),
            "orc_div": (None, [i, i, i, _dp, _dp]),
            "orc_fft3": (None, [i, i, i, _dp, _dp, i]),
            "orc_spectral": (None, [i, i, i, _dp, _dp, i, i, d]),
            "orc_spectral_resample": (None, [i, i, i, _dp, i, i, i, _dp]),
            "orc_spec_div": (None, [i, i, i, _dp, _dp]),
            "orc_spec_grad": (None, [i, i, i, _dp, _dp]),
            "orc_reg_op": (None, [i, i, i, _dp, _dp, i, d, d]),
            "orc_set_beta_w": (None, [vp, d]),
            "orc_gradient_l2": (None, [vp, _dp]),
            "orc_matvec_sym": (None, [vp, _dp, _dp]),
            "orc_jacobian_det": (None, [vp, _dp]),
            "orc_set_beta": (None, [vp, d, d]),
            "orc_set_interp": (None, [vp, i]),
            "orc_interp_order": (None, [i, i, i, i, _dp, _dp, _dp]),
            "orc_interp_point_lin": (d, [i, i, i, _dp, d, d, d]),
            "orc_feet_order": (None, [i, i, i, i, i, _dp, _dp, _dp]),
            "orc_set_precond": (None, [vp, i, i]),
            "orc_param_search": (i, [vp, d, d, d, d, d, d, i, i, i, d, _dp, i, _ip, _dp, _dp]),
            "orc_param_continuation": (i, [vp, d, d, d, d, i, i, d, _dp, i, _ip]),
            "orc_feet": (None, [i, i, i, i, _dp, _dp, _dp]),
            "orc_adjoint_factor": (None, [i, i, i, i, _dp, _dp, _dp]),
            "orc_create": (vp, [i, i, i, i, d]),
            "orc_destroy": (None, [vp]),
            "orc_set_images": (None, [vp, _dp, _dp]),
            "orc_set_velocity": (None, [vp, _dp]),
            "orc_state": (None, [vp]),
            "orc_objective": (None, [vp, _dp, _dp, _dp]),
            "orc_gradient": (None, [vp, _dp, _dp, _dp, _dp]),
            "orc_matvec": (None, [vp, _dp, _dp]),
            "orc_precond": (None, [vp, _dp, _dp]),
            "orc_get_field": (None, [vp, i, i, _dp]),
            "orc_get_velocity": (None, [vp, _dp]),
            "orc_pcg": (i, [vp, _dp, _dp, i, d, i, _ip]),
            "orc_solve": (i, [vp, i, i, d, _ip, _dp, _dp, _ip, _dp]),
            "orc_num_threads": (i, []),
            "orc_set_num_threads": (None, [i]),
            "orc_set_matvec_perturbation": (None, [vp, d, ctypes.c_ulonglong]),
            "cnv_conv3": (None, [i, i, i, i, i, _dp, _dp, _dp, _dp]),
            "cnv_conv3_t": (None, [i, i, i, i, i, _dp, _dp, _dp]),
            "cnv_conv3_dw": (None, [i, i, i, i, i, _dp, _dp, _dp, _dp]),
            "cnv_lrelu": (None, [ctypes.c_long, _dp, d, _dp]),
            "cnv_pool2": (None, [i, i, i, i, _dp, _dp]),
            "cnv_up2cat": (None, [i, i, i, i, i, _dp, _dp, _dp]),
            "cnv_head": (None, [ctypes.c_long, i, i, _dp, _dp, _dp, _dp]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _p(a):
    return a.ctypes.data_as(_dp)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def num_threads():
    return lib().orc_num_threads()


def set_num_threads(n):
    """OpenMP threads of the following oracle calls (timing legs)."""
    lib().orc_set_num_threads(int(n))


# ------------------------------------------------------------- primitives

def interp(u, d):
    """I[u](x + d): tricubic Lagrange at node-relative displacements d (3,...)
    in index units."""
    u = _f64(u); d = _f64(d)
    out = np.empty_like(u)
    lib().orc_interp(*u.shape, _p(u), _p(d), _p(out))
    return out


def interp_linear(u, d):
    """I[u](x + d) with trilinear interpolation (d in index units)."""
    u = _f64(u); d = _f64(d)
    out = np.empty_like(u)
    lib().orc_interp_order(*u.shape, 1, _p(u), _p(d), _p(out))
    return out


def interp_point_linear(u, p):
    u = _f64(u)
    return lib().orc_interp_point_lin(*u.shape, _p(u), float(p[0]), float(p[1]), float(p[2]))


def interp_point(u, p):
    u = _f64(u)
    return lib().orc_interp_point(*u.shape, _p(u), float(p[0]), float(p[1]), float(p[2]))


def grad(u):
    u = _f64(u)
    g = np.empty((3,) + u.shape)
    lib().orc_grad(*u.shape, _p(u), _p(g))
    return g


def div(v):
    v = _f64(v)
    out = np.empty(v.shape[1:])
    lib().orc_div(*v.shape[1:], _p(v), _p(out))
    return out


def fft3(z, sign=-1):
    """Unscaled 3D DFT with exp(sign 2 pi i n k / N)."""
    z = np.asarray(z, dtype=np.complex128)
    re = np.ascontiguousarray(z.real); im = np.ascontiguousarray(z.imag)
    lib().orc_fft3(*z.shape, _p(re), _p(im), int(sign))
    return re + 1j * im


def spectral(u, kind, beta=1.0):
    """kind 0: beta*A (A = -Laplacian); 1: (beta*A)^-1 with k=0 -> 1/beta;
    2: identity through the FFT."""
    u = _f64(u)
    vec = u.ndim == 4
    uu = u if vec else u[None]
    out = np.empty_like(uu)
    lib().orc_spectral(*uu.shape[1:], _p(uu), _p(out), uu.shape[0], int(kind), float(beta))
    return out if vec else out[0]


def spec_div(v):
    """div v by spectral derivatives (Nyquist derivative wavenumber 0)."""
    v = _f64(v)
    out = np.empty(v.shape[1:])
    lib().orc_spec_div(*v.shape[1:], _p(v), _p(out))
    return out


def spec_grad(u):
    """grad u by spectral derivatives (Nyquist derivative wavenumber 0)."""
    u = _f64(u)
    g = np.empty((3,) + u.shape)
    lib().orc_spec_grad(*u.shape, _p(u), _p(g))
    return g


REG_L, REG_PRECOND, REG_K = 0, 1, 3


def reg_op(v, kind, beta_v, beta_w):
    """Per-mode operators on a vector field: kind 0 L (Hessian of the
    regularisation), 1 preconditioner L^-1 (k = 0 -> 1/beta_v), 3 the
    Leray-like K = beta_v A L^-1 (k = 0 -> I)."""
    v = _f64(v)
    out = np.empty_like(v)
    lib().orc_reg_op(*v.shape[1:], _p(v), _p(out), int(kind), float(beta_v), float(beta_w))
    return out


def spectral_resample(u, shape):
    u = _f64(u)
    out = np.empty(shape)
    lib().orc_spectral_resample(*u.shape, _p(u), *shape, _p(out))
    return out


def feet(v, nt):
    v = _f64(v)
    df = np.empty_like(v); db = np.empty_like(v)
    lib().orc_feet(*v.shape[1:], int(nt), _p(v), _p(df), _p(db))
    return df, db


def adjoint_factor(v, db, nt):
    v = _f64(v); db = _f64(db)
    c = np.empty(v.shape[1:])
    lib().orc_adjoint_factor(*v.shape[1:], int(nt), _p(v), _p(db), _p(c))
    return c


# ---------------------------------------------------------------- context

FIELD_STATE, FIELD_ADJOINT, FIELD_INC_STATE, FIELD_INC_ADJOINT = 0, 1, 2, 3
FIELD_FEET_F, FIELD_FEET_B, FIELD_ADJ_FACTOR = 4, 5, 6


class Oracle:
    """Registration problem on an n1 x n2 x n3 periodic grid over [0, 2pi)^3."""

    def __init__(self, shape, nt=4, beta=5e-4, beta_w=0.0, interp=3):
        """interp: 3 tricubic Lagrange (default), 1 trilinear."""
        self.shape = tuple(int(s) for s in shape)
        self.nt = int(nt)
        self.beta = float(beta)
        self.beta_w = float(beta_w)
        self._h = lib().orc_create(*self.shape, self.nt, self.beta)
        lib().orc_set_beta_w(self._h, self.beta_w)
        lib().orc_set_interp(self._h, int(interp))

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            lib().orc_destroy(h)
            self._h = None

    def set_images(self, m0, m1):
        m0 = _f64(m0); m1 = _f64(m1)
        lib().orc_set_images(self._h, _p(m0), _p(m1))

    def set_velocity(self, v):
        v = _f64(v)
        lib().orc_set_velocity(self._h, _p(v))

    def velocity(self):
        v = np.empty((3,) + self.shape)
        lib().orc_get_velocity(self._h, _p(v))
        return v

    def state(self):
        lib().orc_state(self._h)

    def objective(self):
        J, m, r = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
        lib().orc_objective(self._h, ctypes.byref(J), ctypes.byref(m), ctypes.byref(r))
        return J.value, m.value, r.value

    def gradient(self):
        g = np.empty((3,) + self.shape)
        J, m, r = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
        lib().orc_gradient(self._h, _p(g), ctypes.byref(J), ctypes.byref(m), ctypes.byref(r))
        return g, (J.value, m.value, r.value)

    def gradient_l2(self):
        """L2 gradient of J (L v + b); equals gradient() when beta_w = 0."""
        g = np.empty((3,) + self.shape)
        lib().orc_gradient_l2(self._h, _p(g))
        return g

    def matvec_sym(self, vt):
        """L2-symmetric Hessian L vt + b~ (= matvec when beta_w = 0)."""
        vt = _f64(vt)
        out = np.empty_like(vt)
        lib().orc_matvec_sym(self._h, _p(vt), _p(out))
        return out

    def matvec(self, vt):
        vt = _f64(vt)
        out = np.empty_like(vt)
        lib().orc_matvec(self._h, _p(vt), _p(out))
        return out

    def jacobian_det(self):
        """det grad y of the map y with m(1) = m0 o y at the current v."""
        J = np.empty(self.shape)
        lib().orc_jacobian_det(self._h, _p(J))
        return J

    def set_precond(self, kind, inner=5):
        """kind 0: spectral L^-1; 1: zero-velocity Hessian H0 by `inner` CG
        steps; 2: its two-level variant (H0 by `inner` CG steps on the
        half-resolution grid for the band it represents, L^-1 above); the
        outer PCG is flexible for kinds 1 and 2."""
        lib().orc_set_precond(self._h, int(kind), int(inner))

    def set_beta(self, beta_v, beta_w=0.0):
        self.beta, self.beta_w = float(beta_v), float(beta_w)
        lib().orc_set_beta(self._h, self.beta, self.beta_w)

    def param_search(self, jmin=0.25, beta_v_max=1.0, beta_v_min=1e-5, beta_w_max=1e-5, beta_w_min=1e-7,
                     rel_change=0.1, search_beta_w=True, max_outer=50, max_pcg=10, gtol=1e-2):
        """Returns (status, beta_v*, beta_w*, log rows [beta_v, beta_w, min J,
        max J, valid, GN, PCG, status, mismatch, 0])."""
        cap = 256
        log = np.zeros((cap, 10))
        nr = ctypes.c_int()
        bv, bw = ctypes.c_double(), ctypes.c_double()
        st = lib().orc_param_search(self._h, jmin, beta_v_max, beta_v_min, beta_w_max, beta_w_min, rel_change,
                                    int(search_beta_w), int(max_outer), int(max_pcg), float(gtol), _p(log), cap,
                                    ctypes.byref(nr), ctypes.byref(bv), ctypes.byref(bw))
        self.beta, self.beta_w = bv.value, bw.value
        return st, bv.value, bw.value, log[: min(nr.value, cap)]

    def param_continuation(self, beta_v, beta_w, beta_v_max=1.0, beta_w_max=1e-5, max_outer=50, max_pcg=10,
                           gtol=1e-2):
        cap = 256
        log = np.zeros((cap, 10))
        nr = ctypes.c_int()
        lib().orc_param_continuation(self._h, beta_v_max, beta_w_max, float(beta_v), float(beta_w), int(max_outer),
                                     int(max_pcg), float(gtol), _p(log), cap, ctypes.byref(nr))
        self.beta, self.beta_w = float(beta_v), float(beta_w)
        return log[: min(nr.value, cap)]

    def precond(self, r):
        r = _f64(r)
        out = np.empty_like(r)
        lib().orc_precond(self._h, _p(r), _p(out))
        return out

    def field(self, which, j=0):
        n = 3 if which in (FIELD_FEET_F, FIELD_FEET_B) else 1
        out = np.empty((n,) + self.shape) if n == 3 else np.empty(self.shape)
        lib().orc_get_field(self._h, int(which), int(j), _p(out))
        return out

    def pcg(self, rhs, max_pcg, eta, forced_iters=-1):
        rhs = _f64(rhs)
        x = np.empty_like(rhs)
        its = ctypes.c_int()
        neg = lib().orc_pcg(self._h, _p(rhs), _p(x), int(max_pcg), float(eta), int(forced_iters), ctypes.byref(its))
        return x, its.value, bool(neg)

    def set_matvec_perturbation(self, eps, seed=0):
        """Sensitivity probe (tests only): every PCG matvec output is
        multiplied elementwise by 1 + eps xi, xi uniform in [-1, 1) from a
        counter-based hash of (seed, call, index); eps = 0 switches it off."""
        lib().orc_set_matvec_perturbation(self._h, float(eps), int(seed))

    def solve(self, max_outer=5, max_pcg=10, gtol=1e-2, forced_pcg=None, forced_alpha=None):
        """Gauss-Newton-Krylov from the current velocity.  Returns
        (status, log rows [k, J, mismatch, reg, ||g||, pcg_its, alpha, ls_trials],
        gref).  status 0 converged, 1 iteration limit, 2 line search failed."""
        log = np.zeros((max_outer + 1, 8))
        nout = ctypes.c_int()
        gref = ctypes.c_double()
        fp = None
        fa = None
        if forced_pcg is not None:
            fpa = np.ascontiguousarray(forced_pcg, dtype=np.int32)
            fp = fpa.ctypes.data_as(_ip)
        if forced_alpha is not None:
            faa = _f64(forced_alpha)
            fa = _p(faa)
        st = lib().orc_solve(self._h, int(max_outer), int(max_pcg), float(gtol), fp, fa,
                             _p(log), ctypes.byref(nout), ctypes.byref(gref))
        return st, log[: nout.value + 1], gref.value


# ------------------------------------------------ network layers (FP64)
# Tensors are channels-last numpy arrays of shape (D, H, W, C); conv weights
# are (27, Ci, Co) with tap t = (tz * 3 + ty) * 3 + tx.

def conv3(x, w, b=None):
    x = _f64(x); w = _f64(w)
    D, H, W, Ci = x.shape
    Co = w.shape[2]
    out = np.empty((D, H, W, Co))
    bb = _f64(b) if b is not None else None
    lib().cnv_conv3(D, H, W, Ci, Co, _p(x), _p(w), _p(bb) if bb is not None else None, _p(out))
    return out


def conv3_t(gout, w):
    gout = _f64(gout); w = _f64(w)
    D, H, W, Co = gout.shape
    Ci = w.shape[1]
    gin = np.empty((D, H, W, Ci))
    lib().cnv_conv3_t(D, H, W, Ci, Co, _p(gout), _p(w), _p(gin))
    return gin


def conv3_dw(x, gout):
    x = _f64(x); gout = _f64(gout)
    D, H, W, Ci = x.shape
    Co = gout.shape[3]
    gw = np.empty((27, Ci, Co)); gb = np.empty(Co)
    lib().cnv_conv3_dw(D, H, W, Ci, Co, _p(x), _p(gout), _p(gw), _p(gb))
    return gw, gb


def lrelu(x, s=0.2):
    x = _f64(x)
    y = np.empty_like(x)
    lib().cnv_lrelu(x.size, _p(x), float(s), _p(y))
    return y


def pool2(x):
    x = _f64(x)
    D, H, W, C = x.shape
    out = np.empty((D // 2, H // 2, W // 2, C))
    lib().cnv_pool2(D, H, W, C, _p(x), _p(out))
    return out


def up2cat(a, b):
    a = _f64(a); b = _f64(b)
    D, H, W, Cb = b.shape
    Ca = a.shape[3]
    out = np.empty((D, H, W, Ca + Cb))
    lib().cnv_up2cat(D, H, W, Ca, Cb, _p(a), _p(b), _p(out))
    return out


def head(x, w, b=None):
    x = _f64(x); w = _f64(w)
    Ci, Co = w.shape
    n = x.size // Ci
    out = np.empty(x.shape[:-1] + (Co,))
    bb = _f64(b) if b is not None else None
    lib().cnv_head(n, Ci, Co, _p(x), _p(w), _p(bb) if bb is not None else None, _p(out))
    return out
