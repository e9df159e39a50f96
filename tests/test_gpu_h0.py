"""Zero-velocity Hessian preconditioner on the GPU against the FP64 oracle:
its application (inner CG on H0 = L + grad m0 grad m0^T with the spectral
preconditioner, L p by recurrence on the GPU, by FFT in the oracle), the
free-run decisions of the flexible outer PCG, and the PCG count against the
spectral preconditioner.

Tolerances: the application is a few CG steps, each an FFT pair and FP64
reductions: 1e-4 relative L2 (as the gradient and matvec).  Decisions
(PCG counts, step lengths) must be equal; J, mismatch and ||g|| to 1e-5."""
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


@pytest.mark.parametrize("shape,inner,bw", [((32, 32, 32), 1, 0.0), ((32, 32, 32), 5, 0.0),
                                            ((32, 16, 64), 5, 1e-3)])
def test_h0_application_matches_oracle(shape, inner, bw):
    m0, m1, vs = _pair(shape)
    v = f32(0.5 * vs)
    rr = f32(synth.random_field((3,) + shape, 95))
    o = oracle.Oracle(shape, nt=4, beta=5e-4, beta_w=bw)
    o.set_images(m0, m1)
    o.set_velocity(v)
    o.set_precond(1, inner)
    z_ref = o.precond(rr)
    r = reg(shape, beta_w=bw, precond="h0", precond_inner=inner)
    r.set_images(dev(m0), dev(m1))
    r.set_velocity(dev(v))
    z = host(r.precond(dev(rr)))
    e = rel(z, z_ref)
    print("H0 %s inner %d beta_w %g: rel %.2e" % (shape, inner, bw, e))
    assert e < 1e-4
    r.close()


@pytest.mark.parametrize("bw", [0.0, 1e-5])
def test_h0_free_solve_decisions_match_oracle(bw):
    shape = (32, 32, 32)
    m0, m1, _ = _pair(shape)
    o = oracle.Oracle(shape, nt=4, beta=0.1, beta_w=bw)
    o.set_images(m0, m1)
    o.set_velocity(np.zeros((3,) + shape))
    o.set_precond(1, 5)
    st, log, gref = o.solve(max_outer=10, max_pcg=10, gtol=1e-2)
    r = reg(shape, beta_v=0.1, beta_w=bw, max_outer=10, max_pcg=10, precond="h0", precond_inner=5)
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


def test_h0_needs_fewer_pcg_iterations():
    """64^3 closed-form pair, beta_v = 5e-4, <= 40 PCG: the H0 solve takes
    fewer PCG iterations in total than the spectral one and ends at the
    same relative mismatch within 1e-3."""
    shape = (64, 64, 64)
    m0, m1, _ = _pair(shape)
    mis0 = 0.5 * np.sum((m0 - m1) ** 2) * (2 * np.pi / 64) ** 3
    out = {}
    for name, kw in (("spectral", {}), ("h0", {"precond": "h0", "precond_inner": 5})):
        r = reg(shape, max_outer=30, max_pcg=40, **kw)
        r.set_images(dev(m0), dev(m1))
        rep = r.solve()
        out[name] = (rep["outer_iters"], rep["pcg_iters_total"], rep["mismatch"] / mis0, rep["status_name"])
        r.close()
    print("spectral: %d GN %d PCG r %.4e %s; h0: %d GN %d PCG r %.4e %s" % (out["spectral"] + out["h0"]))
    assert out["h0"][3] == "ok" and out["spectral"][3] == "ok"
    assert out["h0"][1] < out["spectral"][1]
    assert abs(out["h0"][2] - out["spectral"][2]) < 1e-3


def test_h0_rejected_in_lean_layout():
    from paper_2209_08189_amd.claire import ClaireError, query_workspace
    shape = (32, 32, 32)
    cap = query_workspace(shape, workspace_cap=1)
    with pytest.raises(ClaireError) as e:
        reg(shape, precond="h0", workspace_cap=cap)
    assert e.value.code == -7
