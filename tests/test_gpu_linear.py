"""Trilinear interpolation option (interp_order = 1, the paper's choice for
large grids) on the GPU against the FP64 oracle with the same option:
single gathers, each transport, gradient and Hessian matvec, the exact
integer-shift roll, and free-run GN decisions.  Tolerances as in the
tricubic parity tests (1e-5 per transport, 1e-4 for g and H vt)."""
import numpy as np
import pytest

import oracle
from paper_2209_08189_amd import synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2209_08189_amd import claire
    claire.lib()
    torch.cuda.set_device(0)


def reg(shape, **kw):
    from paper_2209_08189_amd.claire import Registration
    return Registration(shape, interp="linear", **kw)


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy().astype(np.float64)


def f32(a):
    return np.asarray(a, dtype=np.float32).astype(np.float64)


def rel(a, b):
    return float(np.linalg.norm(np.ravel(a - b)) / max(np.linalg.norm(np.ravel(b)), 1e-300))


@pytest.mark.parametrize("shape", [(32, 16, 64), (64, 64, 64), (16, 16, 16), (16, 16, 32)])
@pytest.mark.parametrize("feet", ["smooth", "rough", "mixed"])
def test_trilinear_gather(shape, feet):
    """Against the oracle's trilinear interpolation.  Grids with n3 >= 32
    gather tile by tile from LDS boxes; smooth displacements fit
    the boxes, rough ones (independent random shifts of up to +-6 voxels per
    node) send their tiles to the per-node global-memory path, and "mixed"
    holds both kinds of tile in one launch; 16^3 uses the per-node kernel."""
    u = f32(synth.random_field(shape, 11))
    smooth = np.stack([3.0 * synth.smooth_random_field(shape, 12 + a, kmax=3.0) for a in range(3)])
    rough = synth.random_field((3,) + shape, 15, lo=-6.0, hi=6.0)
    if feet == "smooth":
        d = smooth
    elif feet == "rough":
        d = rough
    else:
        d = smooth.copy()
        d[:, : shape[0] // 2] = rough[:, : shape[0] // 2]
    d = f32(d)
    r = reg(shape)
    out = host(r.interp(dev(u), dev(d)))
    e = rel(out, oracle.interp_linear(u, d))
    print("trilinear gather %s %s: %.2e" % (shape, feet, e))
    assert e < 1e-5
    r.close()


def _pair(n, interp):
    shape = (n,) * 3
    m0 = f32(synth.trig_template(shape))
    vs = f32(synth.trig_velocity(shape, 0.5))
    o = oracle.Oracle(shape, nt=4, beta=5e-4, interp=interp)
    o.set_images(m0, m0)
    o.set_velocity(vs)
    o.state()
    return shape, m0, f32(o.field(oracle.FIELD_STATE, 4)), vs


def test_transports_gradient_matvec():
    shape, m0, m1, vs = _pair(64, 1)
    v = f32(0.5 * vs)
    vt = f32(synth.trig_velocity(shape, 0.3)[[2, 0, 1]] + 0.1 * synth.random_field((3,) + shape, 9))
    o = oracle.Oracle(shape, nt=4, beta=5e-4, interp=1)
    o.set_images(m0, m1)
    o.set_velocity(v)
    g_ref, _ = o.gradient()
    Hv_ref = o.matvec(vt)
    r = reg(shape)
    r.set_images(dev(m0), dev(m1))
    r.set_velocity(dev(v))
    g, _, _ = r.gradient()
    # the context keeps lambda and lambda~ in one buffer: read lambda first
    errs = {"feet_f": rel(host(r.field(4)), o.field(oracle.FIELD_FEET_F)),
            "feet_b": rel(host(r.field(5)), o.field(oracle.FIELD_FEET_B)),
            "m(1)": rel(host(r.field(0, 4)), o.field(oracle.FIELD_STATE, 4)),
            "lambda(0)": rel(host(r.field(1, 0)), o.field(oracle.FIELD_ADJOINT, 0))}
    Hv = host(r.hessian_matvec(dev(vt)))
    errs.update({"mt(1)": rel(host(r.field(2, 4)), o.field(oracle.FIELD_INC_STATE, 4)),
                 "lamt(0)": rel(host(r.field(3, 0)), o.field(oracle.FIELD_INC_ADJOINT, 0))})
    print("linear transports:", {k: "%.1e" % v for k, v in errs.items()},
          "g %.1e Hv %.1e" % (rel(host(g), g_ref), rel(Hv, Hv_ref)))
    assert max(errs.values()) < 1e-5
    assert rel(host(g), g_ref) < 1e-4 and rel(Hv, Hv_ref) < 1e-4
    r.close()


UROUND = {"f16": 2.0 ** -11, "bf16": 2.0 ** -8}


@pytest.mark.parametrize("st,ad", [("f16", "f16"), ("f16", "bf16"), ("bf16", "bf16")])
def test_mixed_storage_transports(st, ad):
    """Trilinear steps on 16-bit boxes (the LDS copy holding each row pair
    as one aligned word, and the per-node path on the same storage): state
    stored as `st`, adjoint / incremental fields as `ad`, FP32 arithmetic.
    Errors against the FP64 oracle bounded as the tricubic mixed-storage
    test: (n_t + 2) roundings of the storage format, the adjoint with the
    extra factor |m1| / |lambda(1)| of its starting difference."""
    shape, m0, m1, vs = _pair(64, 1)
    v = f32(0.5 * vs)
    vt = f32(synth.trig_velocity(shape, 0.3)[[2, 0, 1]])
    o = oracle.Oracle(shape, nt=4, beta=5e-4, interp=1)
    o.set_images(m0, m1)
    o.set_velocity(v)
    g_ref, _ = o.gradient()
    Hv_ref = o.matvec(vt)
    r = reg(shape, storage_state=st, storage_adjoint=ad)
    r.set_images(dev(m0), dev(m1))
    r.set_velocity(dev(v))
    g, _, _ = r.gradient()
    errs = {"m(1)": rel(host(r.field(0, 4)), o.field(oracle.FIELD_STATE, 4)),
            "lambda(0)": rel(host(r.field(1, 0)), o.field(oracle.FIELD_ADJOINT, 0)),
            "g": rel(host(g), g_ref)}
    Hv = host(r.hessian_matvec(dev(vt)))
    errs["lambda~(0)"] = rel(host(r.field(3, 0)), o.field(oracle.FIELD_INC_ADJOINT, 0))
    errs["Hvt"] = rel(Hv, Hv_ref)
    print("linear storage %s/%s: %s" % (st, ad, {k: "%.2e" % e for k, e in errs.items()}))
    us, ua = UROUND[st], UROUND[ad]
    amp = np.linalg.norm(m1) / np.linalg.norm(o.field(oracle.FIELD_ADJOINT, 4))
    assert errs["m(1)"] < 6 * us
    for k in ("lambda(0)", "g", "lambda~(0)", "Hvt"):
        assert errs[k] < 6 * (ua + us * amp), k
    r.close()


def test_integer_shift_roll():
    n = 64
    shape = (n,) * 3
    m0 = f32(synth.trig_template(shape))
    r = reg(shape)
    r.set_images(dev(m0), dev(m0))
    v = np.zeros((3,) + shape)
    v[2] = (2 * np.pi / n) * 8       # two voxels per step along x3
    r.set_velocity(dev(v))
    assert np.array_equal(host(r.deformed_template()), np.roll(m0, 8, axis=2))
    r.close()


def test_free_solve_decisions():
    shape, m0, m1, _ = _pair(32, 1)
    o = oracle.Oracle(shape, nt=4, beta=0.1, interp=1)
    o.set_images(m0, m1)
    o.set_velocity(np.zeros((3,) + shape))
    st, log, gref = o.solve(max_outer=10, max_pcg=10, gtol=1e-2)
    r = reg(shape, beta_v=0.1, max_outer=10, max_pcg=10)
    r.set_images(dev(m0), dev(m1))
    rep = r.solve()
    glog = np.array(r.solve_log())
    print("oracle:", log[:, [1, 2, 4, 5, 6]].tolist())
    print("gpu:   ", glog[:, [1, 2, 4, 5, 6]].tolist())
    assert glog.shape == log.shape
    assert np.array_equal(glog[:, 5], log[:, 5]) and np.array_equal(glog[:, 6], log[:, 6])
    for c in (1, 2):
        assert np.all(np.abs(glog[:, c] - log[:, c]) <= 1e-5 * np.abs(log[:, c]))
    assert np.all(np.abs(glog[:, 4] - log[:, 4]) <= 1e-5 * gref)
    r.close()
