"""Parity at the benchmark size: the 256^3 phantom pair, v = v_true and
vt = -P^-1 g, through the same C-ABI entry points and launch configuration
that bench.py times, against the FP64 oracle on every node.

Inputs follow the benchmark recipe (phantom seed 0, band-limited velocity
seed 1 with a 6-voxel maximum displacement, N(0, 0.02^2) noise seeds 2 and
3); m1 is the phantom transported by the oracle's FP64 semi-Lagrangian solve
plus noise, and both sides read the same FP32-rounded images.  Tolerances
are those of the small-size parity tests: 1e-5 relative L2 per transported
field, 1e-4 for the gradient and the Hessian matvec."""
import time

import numpy as np
import pytest

import oracle
from paper_2209_08189_amd import synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

N = 256


def rel(a, b):
    return float(np.linalg.norm(np.ravel(a - b)) / max(np.linalg.norm(np.ravel(b)), 1e-300))


def f32(a):
    return np.asarray(a, dtype=np.float32).astype(np.float64)


def test_gradient_and_matvec_at_256():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2209_08189_amd.claire import Registration
    torch.cuda.set_device(0)
    shape = (N, N, N)
    t0 = time.time()
    img, _ = synth.phantom(shape, 0)
    v = f32(synth.smooth_velocity(shape, 1, kmax=8.0, max_disp_voxels=6.0))
    n0, n1 = synth.noise(shape, 2, 0.02), synth.noise(shape, 3, 0.02)
    img = f32(img)
    o = oracle.Oracle(shape, nt=4, beta=5e-4)
    o.set_images(img, img)
    o.set_velocity(v)
    o.state()
    m1 = f32(o.field(oracle.FIELD_STATE, 4) + n1)
    m0 = f32(img + n0)
    o.set_images(m0, m1)
    o.set_velocity(v)
    g_ref, _ = o.gradient()
    m_ref, lam_ref = o.field(oracle.FIELD_STATE, 4), o.field(oracle.FIELD_ADJOINT, 0)
    vt = f32(-o.precond(g_ref))
    Hv_ref = o.matvec(vt)
    print("oracle at 256^3 (%d threads): %.1f s" % (oracle.num_threads(), time.time() - t0))

    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()
    host = lambda t: (torch.cuda.synchronize(), t.detach().cpu().numpy().astype(np.float64))[1]
    r = Registration(shape, nt=4, beta_v=5e-4)
    r.set_images(dev(m0), dev(m1))
    r.set_velocity(dev(v))
    g, _, _ = r.gradient()
    # the adjoint buffer is reused by the matvec's incremental adjoint: read
    # the state and adjoint before the matvec
    e_m, e_lam = rel(host(r.field(0, 4)), m_ref), rel(host(r.field(1, 0)), lam_ref)
    Hv = r.hessian_matvec(dev(vt))
    errs = {
        "m(1)": e_m,
        "lambda(0)": e_lam,
        "mt(1)": rel(host(r.field(2, 4)), o.field(oracle.FIELD_INC_STATE, 4)),
        "lambda~(0)": rel(host(r.field(3, 0)), o.field(oracle.FIELD_INC_ADJOINT, 0)),
        "g": rel(host(g), g_ref),
        "Hv": rel(host(Hv), Hv_ref),
    }
    print("256^3 relative L2 errors:", {k: "%.2e" % e for k, e in errs.items()})
    for k in ("m(1)", "lambda(0)", "mt(1)", "lambda~(0)"):
        assert errs[k] < 1e-5, k
    assert errs["g"] < 1e-4 and errs["Hv"] < 1e-4


@pytest.mark.parametrize("st,ad", [("f16", "f16"), ("f16", "bf16")])
def test_mixed_storage_phantom_128(st, ad):
    """Mixed-precision storage on a phantom problem: the 256^3 benchmark
    recipe generated at 128^3 with the same voxel-unit parameters (blob
    widths, 6-voxel displacement), so the crop-sized problem is periodic on
    its own.  Per-field relative L2 error against the FP64 oracle, bounded
    as in the 64^3 mixed-storage test: 6 (nt + 2)-step units of roundoff of
    the storage format, the adjoint amplified by |m1| / |lambda(1)|."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2209_08189_amd.claire import Registration
    torch.cuda.set_device(0)
    n = 128
    shape = (n, n, n)
    img, _ = synth.phantom(shape, 5)
    v = f32(synth.smooth_velocity(shape, 6, kmax=8.0, max_disp_voxels=6.0))
    img = f32(img)
    o = oracle.Oracle(shape, nt=4, beta=5e-4)
    o.set_images(img, img)
    o.set_velocity(v)
    o.state()
    m1 = f32(o.field(oracle.FIELD_STATE, 4) + synth.noise(shape, 8, 0.02))
    m0 = f32(img + synth.noise(shape, 7, 0.02))
    o.set_images(m0, m1)
    o.set_velocity(v)
    g_ref, _ = o.gradient()
    m_ref, lam_ref = o.field(oracle.FIELD_STATE, 4), o.field(oracle.FIELD_ADJOINT, 0)
    lam1 = o.field(oracle.FIELD_ADJOINT, 4)
    vt = f32(-o.precond(g_ref))
    Hv_ref = o.matvec(vt)
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()
    host = lambda t: (torch.cuda.synchronize(), t.detach().float().cpu().numpy().astype(np.float64))[1]
    r = Registration(shape, storage_state=st, storage_adjoint=ad)
    r.set_images(dev(m0), dev(m1))
    r.set_velocity(dev(v))
    g, _, _ = r.gradient()
    errs = {"m(1)": rel(host(r.field(0, 4)), m_ref), "lambda(0)": rel(host(r.field(1, 0)), lam_ref),
            "g": rel(host(g), g_ref)}
    Hv = host(r.hessian_matvec(dev(vt)))
    errs["Hvt"] = rel(Hv, Hv_ref)
    print("128^3 phantom, storage %s/%s:" % (st, ad), {k: "%.2e" % e for k, e in errs.items()})
    u = {"f16": 2.0 ** -11, "bf16": 2.0 ** -8}
    us, ua = u[st], u[ad]
    amp = np.linalg.norm(m1) / np.linalg.norm(lam1)
    assert errs["m(1)"] < 6 * us
    for k in ("lambda(0)", "g", "Hvt"):
        assert errs[k] < 6 * (ua + us * amp), k
