"""The C-ABI library loads on the CPU and exports every function that
include/claire_hip.h declares; the Python binding covers all of them.  No
compute call is made (no GPU here)."""
import ctypes
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "claire_hip.h")


def declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(cl_[a-z0-9_]+)\s*\(", txt)))


def test_header_declares_the_boundary():
    names = declared()
    for required in ("cl_set_images", "cl_set_velocity", "cl_objective", "cl_gradient",
                     "cl_hessian_matvec", "cl_solve"):
        assert required in names


def test_library_exports_every_declared_symbol():
    from paper_2209_08189_amd import claire
    L = ctypes.CDLL(claire.LIB_PATH)
    missing = [n for n in declared() if not hasattr(L, n)]
    assert not missing, missing


def test_binding_covers_header():
    from paper_2209_08189_amd import claire
    assert set(declared()) == set(claire.SIGNATURES)


def test_status_strings_without_gpu():
    from paper_2209_08189_amd import claire
    L = claire.lib()
    assert L.cl_status_string(0) == b"ok"
    assert L.cl_status_string(-2) == b"unsupported grid shape"
    assert L.cl_kernel_class_name(3) == b"sl_inc"


def test_option_validation_without_gpu():
    """cl_query_workspace validates options and shape on the host only."""
    from paper_2209_08189_amd import claire
    L = claire.lib()
    o = claire.default_options()
    nb = ctypes.c_ulonglong()
    assert L.cl_query_workspace(256, 256, 256, ctypes.byref(o), ctypes.byref(nb)) == 0
    assert nb.value > 40 * 256 ** 3 * 4
    assert L.cl_query_workspace(100, 256, 256, ctypes.byref(o), ctypes.byref(nb)) == -2
    o.beta_w = 1e-5
    assert L.cl_query_workspace(64, 64, 64, ctypes.byref(o), ctypes.byref(nb)) == 0
    o.beta_w = -1e-5
    assert L.cl_query_workspace(64, 64, 64, ctypes.byref(o), ctypes.byref(nb)) == -1
    o.beta_w = float("nan")
    assert L.cl_query_workspace(64, 64, 64, ctypes.byref(o), ctypes.byref(nb)) == -1
    o = claire.default_options()
    o = claire.default_options(); o.struct_version = 99
    assert L.cl_query_workspace(64, 64, 64, ctypes.byref(o), ctypes.byref(nb)) == -1
    o = claire.default_options(); o.storage_state = 7
    assert L.cl_query_workspace(64, 64, 64, ctypes.byref(o), ctypes.byref(nb)) == -3


def test_workspace_counts_gradients_only_where_read():
    """Full minus lean workspace (host-only query): the n_t - 1 further
    source fields, plus the state gradients where a kernel reads them: none
    on grids the marching FD8 kernels cover (n3 >= 64, n2 >= 8, n_t <= 4)
    with the spectral or the two-level preconditioner, level 0 (3 fields)
    for the full-resolution zero-velocity preconditioner, all n_t + 1 levels
    on the other grids."""
    from paper_2209_08189_amd.claire import query_workspace as q
    cases = [((64, 64, 64), 4, "spectral", 0), ((64, 64, 64), 4, "h0_2level", 0), ((64, 64, 64), 4, "h0", 1),
             ((32, 64, 64), 2, "spectral", 0), ((64, 64, 32), 4, "spectral", 5), ((64, 64, 64), 6, "spectral", 7)]
    for shape, nt, pc, levels in cases:
        n = shape[0] * shape[1] * shape[2]
        full = q(shape, nt=nt, precond=pc)
        lean = q(shape, nt=nt, precond=pc, workspace_cap=1)
        assert full - lean == ((nt - 1) + 3 * levels) * 4 * n, (shape, nt, pc)
