"""Two-level zero-velocity preconditioner on the GPU against the FP64 oracle
(Section 2.2 names the two-level coarse-grid approximation as the default):
its application (H0 inverted by inner CG on the half-resolution grid for
the band that grid represents, the spectral L^-1 above it), the free-run
decisions of the flexible outer PCG, and the PCG count against the
spectral and the full-resolution preconditioners.

Tolerances as for the full-resolution variant: the application (a few CG
steps, FFT pairs, spectral resampling, FP64 reductions) 1e-4 relative L2;
decisions equal; J, mismatch and ||g|| to 1e-5."""
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
    return Registration(shape, **kw)


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy().astype(np.float64)


def f32(a):
    return np.asarray(a, dtype=np.float32).astype(np.float64)


def rel(a, b):
    return float(np.linalg.norm(np.ravel(a - b)) / max(np.linalg.norm(np.ravel(b)), 1e-300))


def _pair(shape):
    m0 = f32(synth.trig_template(shape))
    vs = f32(synth.trig_velocity(shape, 0.5))
    o = oracle.Oracle(shape, nt=4, beta=5e-4)
    o.set_images(m0, m0)
    o.set_velocity(vs)
    o.state()
    return m0, f32(o.field(oracle.FIELD_STATE, 4)), vs


@pytest.mark.parametrize("shape,inner,bw", [((32, 32, 32), 1, 0.0), ((32, 32, 32), 6, 0.0),
                                            ((32, 64, 32), 6, 0.0), ((64, 32, 32), 4, 1e-3)])
def test_h0_2level_application_matches_oracle(shape, inner, bw):
    m0, m1, vs = _pair(shape)
    rr = f32(synth.random_field((3,) + shape, 96))
    o = oracle.Oracle(shape, nt=4, beta=5e-4, beta_w=bw)
    o.set_images(m0, m1)
    o.set_velocity(f32(0.5 * vs))
    o.set_precond(2, inner)
    z_ref = o.precond(rr)
    r = reg(shape, beta_w=bw, precond="h0_2level", precond_inner=inner)
    r.set_images(dev(m0), dev(m1))
    r.set_velocity(dev(0.5 * vs))
    z = host(r.precond(dev(rr)))
    e = rel(z, z_ref)
    print("two-level H0 %s inner %d beta_w %g: rel %.2e" % (shape, inner, bw, e))
    assert e < 1e-4
    # a second application after new images rebuilds the coarse template
    r.set_images(dev(m1), dev(m0))
    o.set_images(m1, m0)
    e2 = rel(host(r.precond(dev(rr))), o.precond(rr))
    assert e2 < 1e-4, e2
    r.close()


def test_h0_2level_free_solve_decisions_match_oracle():
    shape = (32, 32, 32)
    m0, m1, _ = _pair(shape)
    o = oracle.Oracle(shape, nt=4, beta=0.1)
    o.set_images(m0, m1)
    o.set_velocity(np.zeros((3,) + shape))
    o.set_precond(2, 5)
    st, log, gref = o.solve(max_outer=10, max_pcg=10, gtol=1e-2)
    r = reg(shape, beta_v=0.1, max_outer=10, max_pcg=10, precond="h0_2level", precond_inner=5)
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
    assert rep["status"] == st
    r.close()


def test_h0_2level_rejects_small_grids_and_lean_layout():
    from paper_2209_08189_amd.claire import ClaireError
    with pytest.raises(ClaireError):
        reg((16, 32, 32), precond="h0_2level")


def test_h0_2level_pcg_count_between_spectral_and_full():
    """64^3 closed-form pair, beta_v = 5e-4, <= 40 PCG per GN step: PCG
    totals of the three preconditioners and the final relative mismatch
    (the two-level variant ends within 1e-3 of the spectral one)."""
    shape = (64, 64, 64)
    m0, m1, _ = _pair(shape)
    mis0 = 0.5 * np.sum((m0 - m1) ** 2) * (2 * np.pi / 64) ** 3
    out = {}
    for name, kw in (("spectral", {}), ("h0_2level", {"precond": "h0_2level", "precond_inner": 8}),
                     ("h0", {"precond": "h0", "precond_inner": 8})):
        r = reg(shape, max_outer=30, max_pcg=40, **kw)
        r.set_images(dev(m0), dev(m1))
        rep = r.solve()
        out[name] = (rep["outer_iters"], rep["pcg_iters_total"], rep["mismatch"] / mis0, rep["status_name"])
        r.close()
    print(out)
    assert all(v[3] == "ok" for v in out.values())
    assert out["h0_2level"][1] <= out["spectral"][1]
    assert abs(out["h0_2level"][2] - out["spectral"][2]) <= 1e-3
