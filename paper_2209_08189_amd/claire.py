"""Thin ctypes binding of libclairehip.so (include/claire_hip.h).

Argument marshalling only: every step of the registration hot path runs in
the library's HIP kernels.  PyTorch provides device memory and the stream.
The library must have been built (``python -m paper_2209_08189_amd.build``);
there is no fallback.
"""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libclairehip.so")

CL_F32, CL_BF16, CL_F16 = 0, 1, 2
DTYPES = {"f32": CL_F32, "bf16": CL_BF16, "f16": CL_F16}
CL_OPTIONS_VERSION = 5
PRECOND = {"spectral": 0, "h0": 1, "h0_2level": 2}

FIELD_STATE, FIELD_ADJOINT, FIELD_INC_STATE, FIELD_INC_ADJOINT = 0, 1, 2, 3
FIELD_FEET_F, FIELD_FEET_B, FIELD_ADJ_FACTOR = 4, 5, 6

K_FEET, K_SL_STATE, K_SL_ADJOINT, K_SL_INC, K_FD, K_QUAD, K_FFT, K_VEC = range(8)
K_NAMES = ["feet", "sl_state", "sl_adjoint", "sl_inc", "fd", "quadrature", "fft", "vec"]

STATUS = {0: "ok", 1: "maxit", 2: "linesearch_fail", 3: "bounds"}


class cl_options(ctypes.Structure):
    _fields_ = [
        ("struct_version", ctypes.c_int),
        ("nt", ctypes.c_int),
        ("beta_v", ctypes.c_double),
        ("beta_w", ctypes.c_double),
        ("gtol", ctypes.c_double),
        ("max_outer", ctypes.c_int),
        ("max_pcg", ctypes.c_int),
        ("forcing", ctypes.c_int),
        ("eta_fixed", ctypes.c_double),
        ("storage_state", ctypes.c_int),
        ("storage_adjoint", ctypes.c_int),
        ("stream", ctypes.c_void_p),
        ("workspace_cap_bytes", ctypes.c_ulonglong),
        ("precond", ctypes.c_int),
        ("precond_inner", ctypes.c_int),
        ("interp_order", ctypes.c_int),
        ("overlap_spectral", ctypes.c_int),
        ("fault_flip_direction", ctypes.c_int),
    ]


class cl_solve_report(ctypes.Structure):
    _fields_ = [
        ("status", ctypes.c_int),
        ("outer_iters", ctypes.c_int),
        ("pcg_iters_total", ctypes.c_int),
        ("linesearch_trials", ctypes.c_int),
        ("J0", ctypes.c_double),
        ("J", ctypes.c_double),
        ("mismatch", ctypes.c_double),
        ("reg", ctypes.c_double),
        ("gnorm0", ctypes.c_double),
        ("gnorm", ctypes.c_double),
        ("gref", ctypes.c_double),
        ("ms", ctypes.c_double),
    ]

    def as_dict(self):
        d = {k: getattr(self, k) for k, _ in self._fields_}
        d["status_name"] = STATUS.get(self.status, str(self.status))
        return d


class cl_search_options(ctypes.Structure):
    _fields_ = [
        ("jmin", ctypes.c_double),
        ("beta_v_max", ctypes.c_double),
        ("beta_v_min", ctypes.c_double),
        ("beta_w_max", ctypes.c_double),
        ("beta_w_min", ctypes.c_double),
        ("rel_change", ctypes.c_double),
        ("search_beta_w", ctypes.c_int),
        ("verbose", ctypes.c_int),
    ]


class cl_search_report(ctypes.Structure):
    _fields_ = [
        ("beta_v", ctypes.c_double),
        ("beta_w", ctypes.c_double),
        ("jmin", ctypes.c_double),
        ("jmax", ctypes.c_double),
        ("status", ctypes.c_int),
        ("solves", ctypes.c_int),
        ("gn_total", ctypes.c_int),
        ("pcg_total", ctypes.c_int),
        ("ms", ctypes.c_double),
    ]

    def as_dict(self):
        d = {k: getattr(self, k) for k, _ in self._fields_}
        d["status_name"] = STATUS.get(self.status, str(self.status))
        return d


class cl_net_options(ctypes.Structure):
    _fields_ = [
        ("struct_version", ctypes.c_int),
        ("in_n", ctypes.c_int),
        ("base_channels", ctypes.c_int),
        ("slope", ctypes.c_float),
        ("lr", ctypes.c_float),
        ("beta1", ctypes.c_float),
        ("beta2", ctypes.c_float),
        ("eps", ctypes.c_float),
        ("seed", ctypes.c_ulonglong),
        ("stream", ctypes.c_void_p),
    ]


_lib = None
_vp = ctypes.c_void_p
_i = ctypes.c_int
_d = ctypes.c_double
_dp = ctypes.POINTER(ctypes.c_double)

SIGNATURES = {
    "cl_default_options": (None, [ctypes.POINTER(cl_options)]),
    "cl_query_workspace": (_i, [_i, _i, _i, ctypes.POINTER(cl_options), ctypes.POINTER(ctypes.c_ulonglong)]),
    "cl_layout": (_i, [ctypes.c_void_p]),
    "cl_create": (_i, [ctypes.POINTER(_vp), _i, _i, _i, ctypes.POINTER(cl_options)]),
    "cl_destroy": (None, [_vp]),
    "cl_set_images": (_i, [_vp, _vp, _vp, _i]),
    "cl_set_velocity": (_i, [_vp, _vp]),
    "cl_get_velocity": (_i, [_vp, _vp]),
    "cl_objective": (_i, [_vp, _dp, _dp, _dp]),
    "cl_gradient": (_i, [_vp, _vp, _dp, _dp]),
    "cl_hessian_matvec": (_i, [_vp, _vp, _vp]),
    "cl_precond_apply": (_i, [_vp, _vp, _vp]),
    "cl_solve": (_i, [_vp, ctypes.POINTER(cl_solve_report)]),
    "cl_solve_forced": (_i, [_vp, ctypes.POINTER(_i), _dp, _i, ctypes.POINTER(cl_solve_report)]),
    "cl_get_solve_log": (_i, [_vp, _dp, _i, ctypes.POINTER(_i)]),
    "cl_deformed_template": (_i, [_vp, _vp]),
    "cl_set_regularization": (_i, [_vp, _d, _d]),
    "cl_jacobian_det": (_i, [_vp, _vp, _dp, _dp]),
    "cl_default_search_options": (None, [ctypes.POINTER(cl_search_options)]),
    "cl_param_search": (_i, [_vp, ctypes.POINTER(cl_search_options), ctypes.POINTER(cl_search_report)]),
    "cl_param_continuation": (_i, [_vp, ctypes.POINTER(cl_search_options), _d, _d,
                                   ctypes.POINTER(cl_search_report)]),
    "cl_get_search_log": (_i, [_vp, _dp, _i, ctypes.POINTER(_i)]),
    "cl_get_field": (_i, [_vp, _i, _i, _vp]),
    "cl_interp": (_i, [_vp, _vp, _vp, _vp]),
    "cl_interp_noalloc": (_i, [_i, _i, _i, _i, _vp, _vp, _vp, _vp]),
    "cl_fd_grad": (_i, [_vp, _vp, _vp]),
    "cl_fd_div": (_i, [_vp, _vp, _vp]),
    "cl_spectral": (_i, [_vp, _i, _i, _vp, _vp]),
    "cl_dot": (_i, [_vp, _vp, _vp, ctypes.c_size_t, _dp]),
    "cl_copy_f32": (_i, [_vp, _vp, _vp, ctypes.c_size_t]),
    "cl_profile_enable": (_i, [_vp, ctypes.c_uint]),
    "cl_profile_query": (_i, [_vp, _i, _dp, ctypes.POINTER(ctypes.c_longlong)]),
    "cl_kernel_class_name": (ctypes.c_char_p, [_i]),
    "cl_net_default_options": (None, [ctypes.POINTER(cl_net_options)]),
    "cl_net_create": (_i, [ctypes.POINTER(_vp), ctypes.POINTER(cl_net_options)]),
    "cl_net_destroy": (None, [_vp]),
    "cl_net_num_params": (_i, [_vp, ctypes.POINTER(ctypes.c_size_t)]),
    "cl_net_get_params": (_i, [_vp, _vp]),
    "cl_net_set_params": (_i, [_vp, _vp]),
    "cl_net_forward": (_i, [_vp, _vp, _vp, _vp]),
    "cl_net_loss_grad": (_i, [_vp, _vp, _vp, _vp, _vp, _dp]),
    "cl_net_train_step": (_i, [_vp, _vp, _vp, _vp, _i, _dp]),
    "cl_net_last_error": (ctypes.c_char_p, [_vp]),
    "cl_nn_conv3": (_i, [_vp, _vp, _vp, _vp, _i, _i, _i, _i, _i, _i, _i, ctypes.c_float, _i, _vp, _vp]),
    "cl_nn_conv3_dw_workspace": (_i, [_i, _i, _i, _i, _i, ctypes.POINTER(ctypes.c_size_t)]),
    "cl_nn_conv3_dw": (_i, [_vp, _vp, _vp, _vp, _vp, _i, _i, _i, _i, _i, _vp]),
    "cl_resampler_create": (_i, [ctypes.POINTER(_vp), _i, _i, _i, _i, _i, _i, _vp]),
    "cl_resampler_destroy": (None, [_vp]),
    "cl_resample": (_i, [_vp, _vp, _vp, _i]),
    "cl_warm_start": (_i, [_vp, _vp, ctypes.POINTER(_i), _dp, _dp]),
    "cl_status_string": (ctypes.c_char_p, [_i]),
    "cl_last_error": (ctypes.c_char_p, [_vp]),
}


def lib():
    """Load libclairehip.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libclairehip.so is not built (python -m paper_2209_08189_amd.build)")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


class ClaireError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("%s (%d): %s" % (lib().cl_status_string(code).decode(), code, msg))
        self.code = code


def default_options():
    o = cl_options()
    lib().cl_default_options(ctypes.byref(o))
    return o


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


def query_workspace(shape, nt=4, storage_state="f32", storage_adjoint="f32", workspace_cap=0, precond="spectral",
                    precond_inner=5):
    """Device bytes a registration context of this shape and storage needs
    (host-only query, cl_query_workspace; the lean layout when the full one
    exceeds a nonzero workspace_cap)."""
    o = default_options()
    o.nt = int(nt)
    o.workspace_cap_bytes = int(workspace_cap)
    o.storage_state = DTYPES[storage_state]
    o.storage_adjoint = DTYPES[storage_adjoint]
    o.precond = PRECOND[precond]
    o.precond_inner = int(precond_inner)
    nb = ctypes.c_ulonglong()
    st = lib().cl_query_workspace(*[int(x) for x in shape], ctypes.byref(o), ctypes.byref(nb))
    if st != 0:
        raise ClaireError(st, "cl_query_workspace")
    return int(nb.value)


def interp_noalloc(u, d, out, interp_order=3, stream=None):
    """out = I[u](x + d) without a context (cl_interp_noalloc): u and out are
    FP32 device tensors of shape (n1, n2, n3), d is (3, n1, n2, n3) in index
    units; enqueued on `stream` (default: torch's current stream).  Nothing
    is allocated; concurrent calls on one GPU share the library's scratch."""
    import torch
    shape = tuple(int(x) for x in u.shape)
    if len(shape) != 3 or tuple(out.shape) != shape or tuple(d.shape) != (3,) + shape:
        raise ValueError("shapes: u and out (n1, n2, n3), d (3, n1, n2, n3)")
    for t in (u, d, out):
        if t.dtype != torch.float32 or not t.is_cuda or not t.is_contiguous():
            raise ValueError("u, d, out must be contiguous FP32 device tensors")
    if stream is None:
        stream = torch.cuda.current_stream().cuda_stream
    st = lib().cl_interp_noalloc(*shape, int(interp_order), _ptr(u), _ptr(d), _ptr(out), ctypes.c_void_p(stream))
    if st != 0:
        raise ClaireError(st, "cl_interp_noalloc")
    return out


class Registration:
    """One registration problem on an n1 x n2 x n3 periodic grid, on the
    current CUDA(HIP) device and torch's current stream."""

    def __init__(self, shape, nt=4, beta_v=5e-4, gtol=1e-2, max_outer=50, max_pcg=10,
                 forcing=1, eta_fixed=0.1, storage_state="f32", storage_adjoint="f32",
                 workspace_cap=0, stream=None, beta_w=0.0, precond="spectral", precond_inner=5,
                 interp="cubic", overlap_spectral=False, fault_flip_direction=False):
        import torch
        self.torch = torch
        self.shape = tuple(int(s) for s in shape)
        self.N = self.shape[0] * self.shape[1] * self.shape[2]
        o = default_options()
        o.nt = int(nt)
        o.beta_v = float(beta_v)
        o.beta_w = float(beta_w)
        o.precond = PRECOND[precond]
        o.precond_inner = int(precond_inner)
        o.interp_order = {"cubic": 3, "linear": 1}[interp]
        o.overlap_spectral = 1 if overlap_spectral else 0
        o.fault_flip_direction = 1 if fault_flip_direction else 0
        o.gtol = float(gtol)
        o.max_outer = int(max_outer)
        o.max_pcg = int(max_pcg)
        o.forcing = int(forcing)
        o.eta_fixed = float(eta_fixed)
        o.storage_state = DTYPES[storage_state]
        o.storage_adjoint = DTYPES[storage_adjoint]
        o.workspace_cap_bytes = int(workspace_cap)
        s = stream if stream is not None else torch.cuda.current_stream()
        self.stream = s
        o.stream = ctypes.c_void_p(s.cuda_stream)
        self.opt = o
        self.nt = o.nt
        h = ctypes.c_void_p()
        st = lib().cl_create(ctypes.byref(h), *self.shape, ctypes.byref(o))
        if st != 0:
            raise ClaireError(st, "cl_create")
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            lib().cl_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -------------------------------------------------------------- helpers
    def _chk(self, st):
        if st < 0:
            raise ClaireError(st, lib().cl_last_error(self._h).decode())
        return st

    def _dev(self, t, n, name):
        torch = self.torch
        if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float32 and t.is_contiguous()):
            raise TypeError("%s must be a contiguous float32 CUDA tensor" % name)
        if t.numel() != n:
            raise ValueError("%s has %d values, expected %d" % (name, t.numel(), n))
        return _ptr(t)

    def empty(self, ncomp=1):
        shp = ((ncomp,) if ncomp > 1 else ()) + self.shape
        return self.torch.empty(shp, dtype=self.torch.float32, device="cuda")

    # ------------------------------------------------------------------ API
    def set_images(self, m0, m1):
        self._chk(lib().cl_set_images(self._h, self._dev(m0, self.N, "m0"), self._dev(m1, self.N, "m1"), CL_F32))

    def set_velocity(self, v):
        self._chk(lib().cl_set_velocity(self._h, self._dev(v, 3 * self.N, "v")))

    def layout(self):
        """0: full memory layout, 1: lean (gradients by FD8 in the kernels)."""
        return int(lib().cl_layout(self._h))

    def velocity(self):
        out = self.empty(3)
        self._chk(lib().cl_get_velocity(self._h, _ptr(out)))
        return out

    def objective(self):
        J, m, r = _d(), _d(), _d()
        self._chk(lib().cl_objective(self._h, ctypes.byref(J), ctypes.byref(m), ctypes.byref(r)))
        return J.value, m.value, r.value

    def gradient(self, want_g=True):
        g = self.empty(3) if want_g else None
        gn, J = _d(), _d()
        self._chk(lib().cl_gradient(self._h, _ptr(g) if g is not None else None, ctypes.byref(gn), ctypes.byref(J)))
        return g, gn.value, J.value

    def hessian_matvec(self, vt, out=None):
        out = self.empty(3) if out is None else out
        self._chk(lib().cl_hessian_matvec(self._h, self._dev(vt, 3 * self.N, "vt"), self._dev(out, 3 * self.N, "Hvt")))
        return out

    def precond(self, r, out=None):
        out = self.empty(3) if out is None else out
        self._chk(lib().cl_precond_apply(self._h, self._dev(r, 3 * self.N, "r"), self._dev(out, 3 * self.N, "z")))
        return out

    def solve(self):
        rep = cl_solve_report()
        self._chk(lib().cl_solve(self._h, ctypes.byref(rep)))
        return rep.as_dict()

    def solve_forced(self, pcg_iters, alphas):
        n = len(pcg_iters)
        P = (ctypes.c_int * n)(*[int(x) for x in pcg_iters])
        A = (ctypes.c_double * n)(*[float(x) for x in alphas])
        rep = cl_solve_report()
        self._chk(lib().cl_solve_forced(self._h, P, A, n, ctypes.byref(rep)))
        return rep.as_dict()

    def solve_log(self):
        nrows = ctypes.c_int()
        lib().cl_get_solve_log(self._h, None, 0, ctypes.byref(nrows))
        buf = (ctypes.c_double * (8 * max(nrows.value, 1)))()
        lib().cl_get_solve_log(self._h, buf, nrows.value, ctypes.byref(nrows))
        return [list(buf[8 * r: 8 * r + 8]) for r in range(nrows.value)]

    def set_regularization(self, beta_v, beta_w=0.0):
        self._chk(lib().cl_set_regularization(self._h, float(beta_v), float(beta_w)))

    def jacobian_det(self, want_field=False):
        """(J field or None, min J, max J) of J = det grad y at the current v."""
        J = self.empty() if want_field else None
        lo, hi = _d(), _d()
        self._chk(lib().cl_jacobian_det(self._h, _ptr(J) if J is not None else None, ctypes.byref(lo),
                                        ctypes.byref(hi)))
        return J, lo.value, hi.value

    @staticmethod
    def search_options(**kw):
        so = cl_search_options()
        lib().cl_default_search_options(ctypes.byref(so))
        for k, v in kw.items():
            setattr(so, k, v)
        return so

    def param_search(self, **kw):
        """Two-stage beta_v / beta_w search under the J bounds; keyword
        arguments override cl_search_options fields."""
        so = self.search_options(**kw)
        rep = cl_search_report()
        self._chk(lib().cl_param_search(self._h, ctypes.byref(so), ctypes.byref(rep)))
        return rep.as_dict()

    def param_continuation(self, beta_v, beta_w, **kw):
        so = self.search_options(**kw)
        rep = cl_search_report()
        self._chk(lib().cl_param_continuation(self._h, ctypes.byref(so), float(beta_v), float(beta_w),
                                              ctypes.byref(rep)))
        return rep.as_dict()

    def search_log(self):
        """Rows [beta_v, beta_w, J min, J max, valid, GN, PCG, status, mismatch, ms]."""
        nrows = ctypes.c_int()
        lib().cl_get_search_log(self._h, None, 0, ctypes.byref(nrows))
        buf = (ctypes.c_double * (10 * max(nrows.value, 1)))()
        lib().cl_get_search_log(self._h, buf, nrows.value, ctypes.byref(nrows))
        return [list(buf[10 * r: 10 * r + 10]) for r in range(nrows.value)]

    def deformed_template(self):
        out = self.empty()
        self._chk(lib().cl_deformed_template(self._h, _ptr(out)))
        return out

    def field(self, which, j=0):
        out = self.empty(3 if which in (FIELD_FEET_F, FIELD_FEET_B) else 1)
        self._chk(lib().cl_get_field(self._h, int(which), int(j), _ptr(out)))
        return out

    def interp(self, u, d):
        out = self.empty()
        self._chk(lib().cl_interp(self._h, self._dev(u, self.N, "u"), self._dev(d, 3 * self.N, "d"), _ptr(out)))
        return out

    def fd_grad(self, u):
        out = self.empty(3)
        self._chk(lib().cl_fd_grad(self._h, self._dev(u, self.N, "u"), _ptr(out)))
        return out

    def fd_div(self, v):
        out = self.empty()
        self._chk(lib().cl_fd_div(self._h, self._dev(v, 3 * self.N, "v"), _ptr(out)))
        return out

    def spectral(self, kind, x):
        ncomp = x.numel() // self.N
        out = self.torch.empty_like(x)
        self._chk(lib().cl_spectral(self._h, int(kind), ncomp, self._dev(x, ncomp * self.N, "in"), _ptr(out)))
        return out

    def dot(self, a, b):
        out = _d()
        self._chk(lib().cl_dot(self._h, _ptr(a), _ptr(b), a.numel(), ctypes.byref(out)))
        return out.value

    def copy(self, src, dst):
        self._chk(lib().cl_copy_f32(self._h, _ptr(src), _ptr(dst), src.numel()))

    def profile_enable(self, mask):
        self._chk(lib().cl_profile_enable(self._h, int(mask)))

    def profile_query(self, kclass):
        ms, n = _d(), ctypes.c_longlong()
        self._chk(lib().cl_profile_query(self._h, int(kclass), ctypes.byref(ms), ctypes.byref(n)))
        return ms.value, n.value


def _stream_ptr(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return s, ctypes.c_void_p(s.cuda_stream)


def _raise(st, msg):
    if st < 0:
        raise ClaireError(st, msg)
    return st


class Net:
    """The learned warm-start network on an in_n^3 grid (device, torch stream)."""

    def __init__(self, in_n=128, seed=1, lr=1e-3, stream=None):
        import torch
        self.torch = torch
        o = cl_net_options()
        lib().cl_net_default_options(ctypes.byref(o))
        o.in_n = int(in_n)
        o.seed = int(seed)
        o.lr = float(lr)
        self.stream, o.stream = _stream_ptr(stream)
        h = ctypes.c_void_p()
        _raise(lib().cl_net_create(ctypes.byref(h), ctypes.byref(o)), "cl_net_create")
        self._h = h
        self.n = int(in_n)
        self.P = self.n ** 3
        nn = ctypes.c_size_t()
        lib().cl_net_num_params(h, ctypes.byref(nn))
        self.num_params = nn.value

    def close(self):
        if getattr(self, "_h", None):
            lib().cl_net_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _err(self, st):
        return _raise(st, lib().cl_net_last_error(self._h).decode())

    def params(self):
        out = self.torch.empty(self.num_params, dtype=self.torch.float32, device="cuda")
        self._err(lib().cl_net_get_params(self._h, _ptr(out)))
        return out

    def set_params(self, p):
        self._err(lib().cl_net_set_params(self._h, _ptr(p.contiguous())))

    def forward(self, m0, m1):
        out = self.torch.empty((3, self.n, self.n, self.n), dtype=self.torch.float32, device="cuda")
        self._err(lib().cl_net_forward(self._h, _ptr(m0), _ptr(m1), _ptr(out)))
        return out

    def loss_grad(self, m0, m1, label):
        g = self.torch.empty(self.num_params, dtype=self.torch.float32, device="cuda")
        L = _d()
        self._err(lib().cl_net_loss_grad(self._h, _ptr(m0), _ptr(m1), _ptr(label), _ptr(g), ctypes.byref(L)))
        return L.value, g

    def train_step(self, m0, m1, label, batch=1):
        L = _d()
        self._err(lib().cl_net_train_step(self._h, _ptr(m0), _ptr(m1), _ptr(label), int(batch), ctypes.byref(L)))
        return L.value


class Resampler:
    """Spectral resampling from grid a to grid b."""

    def __init__(self, a, b, stream=None):
        self.a, self.b = tuple(a), tuple(b)
        self.stream, sp = _stream_ptr(stream)
        h = ctypes.c_void_p()
        _raise(lib().cl_resampler_create(ctypes.byref(h), *self.a, *self.b, sp), "cl_resampler_create")
        self._h = h

    def __del__(self):
        if getattr(self, "_h", None):
            lib().cl_resampler_destroy(self._h)
            self._h = None

    def __call__(self, x):
        import torch
        ncomp = x.numel() // (self.a[0] * self.a[1] * self.a[2])
        out = torch.empty((ncomp,) + self.b if ncomp > 1 else self.b, dtype=torch.float32, device="cuda")
        _raise(lib().cl_resample(self._h, _ptr(x.contiguous()), _ptr(out), ncomp), "cl_resample")
        return out


def nn_conv3(x_bf16, w, b, Co=None, act=1, slope=0.2, transpose=False, out_f32=True):
    """Single 3x3x3 convolution layer on a channels-last BF16 tensor.  w is
    the FP32 weight [27][Ci][Co] of the forward layer; transpose=True
    applies its transpose (input Co channels, output Ci channels)."""
    import torch
    D, H, W, Cin = x_bf16.shape
    Ci, Cw = int(w.shape[1]), int(w.shape[2])
    if Cin != (Cw if transpose else Ci):
        raise ValueError("input channels do not match the weight")
    Cout = Ci if transpose else Cw
    out = torch.empty((D, H, W, Cout), dtype=torch.float32 if out_f32 else torch.bfloat16, device="cuda")
    wpack = torch.empty(28 * Ci * Cw * 2, dtype=torch.uint8, device="cuda")
    st = lib().cl_nn_conv3(_ptr(x_bf16), _ptr(w), _ptr(b) if b is not None else None, _ptr(out), int(out_f32),
                           D, H, W, Ci, Cw, int(act), float(slope), int(transpose), _ptr(wpack),
                           ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    _raise(st, "cl_nn_conv3")
    return out


def nn_conv3_dw(x_bf16, dz_bf16):
    import torch
    D, H, W, Ci = x_bf16.shape
    Co = dz_bf16.shape[3]
    nb = ctypes.c_size_t()
    lib().cl_nn_conv3_dw_workspace(D, H, W, Ci, Co, ctypes.byref(nb))
    ws = torch.empty(max(nb.value, 4), dtype=torch.uint8, device="cuda")
    gw = torch.empty((27, Ci, Co), dtype=torch.float32, device="cuda")
    gb = torch.empty(Co, dtype=torch.float32, device="cuda")
    st = lib().cl_nn_conv3_dw(_ptr(x_bf16), _ptr(dz_bf16), _ptr(gw), _ptr(gb), _ptr(ws), D, H, W, Ci, Co,
                              ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    _raise(st, "cl_nn_conv3_dw")
    return gw, gb


def warm_start(reg, net):
    """Predict the initial velocity of `reg` with `net`; keeps it only if it
    lowers the objective below J(0).  Returns (used, J_pred, J_zero)."""
    used = ctypes.c_int()
    Jp, J0 = _d(), _d()
    st = lib().cl_warm_start(reg._h, net._h, ctypes.byref(used), ctypes.byref(Jp), ctypes.byref(J0))
    reg._chk(st)
    return bool(used.value), Jp.value, J0.value
