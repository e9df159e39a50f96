"""Allocation-free interpolation entry point (cl_interp_noalloc) against the
context entry point cl_interp: same kernels, so the outputs must agree
bitwise.  Two calls in a row, the second on a smaller grid, for tricubic and
trilinear interpolation; the library scratch keeps the first call's boxes,
which the second call must overwrite."""
import numpy as np
import pytest

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


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def case(shape, seed, smooth):
    rng = np.random.default_rng(seed)
    u = rng.standard_normal(shape)
    if smooth:
        # feet of an RK2 step of a smooth velocity: a few voxels at most
        v = synth.smooth_velocity(shape, seed + 1, kmax=4.0, max_disp_voxels=3.0)
        d = v * (np.array(shape, dtype=np.float64) / (2 * np.pi))[:, None, None, None]
    else:
        d = rng.uniform(-6.0, 6.0, (3,) + shape)
    return dev(u), dev(d)


@pytest.mark.parametrize("order", [3, 1])
@pytest.mark.parametrize("smooth", [True, False])
def test_noalloc_matches_context_interp_twice(order, smooth):
    from paper_2209_08189_amd.claire import Registration, interp_noalloc
    for shape, seed in (((64, 64, 128), 11), ((32, 16, 64), 12)):
        print("cl_interp_noalloc order %d smooth %s shape %s" % (order, smooth, shape), flush=True)
        u, d = case(shape, seed, smooth)
        r = Registration(shape, interp={3: "cubic", 1: "linear"}[order])
        ref = r.interp(u, d)
        out = torch.full(shape, float("nan"), dtype=torch.float32, device="cuda")
        interp_noalloc(u, d, out, interp_order=order)
        torch.cuda.synchronize()
        a, b = out.cpu().numpy(), ref.cpu().numpy()
        assert np.isfinite(a).all()
        assert np.array_equal(a.view(np.uint32), b.view(np.uint32)), shape
        del r


def test_noalloc_rejects_before_launch():
    from paper_2209_08189_amd.claire import ClaireError, interp_noalloc, lib
    import ctypes
    t = torch.zeros((16, 16, 16), dtype=torch.float32, device="cuda")
    d = torch.zeros((3, 16, 16, 16), dtype=torch.float32, device="cuda")
    o = torch.zeros((16, 16, 16), dtype=torch.float32, device="cuda")
    p = lambda x: ctypes.c_void_p(x.data_ptr())
    # a grid whose tile boxes exceed the library scratch (2^30 voxels): the
    # host check returns before any launch
    assert lib().cl_interp_noalloc(1024, 1024, 1024, 3, p(t), p(d), p(o), None) == -4
    assert lib().cl_interp_noalloc(16, 16, 24, 3, p(t), p(d), p(o), None) == -2
    assert lib().cl_interp_noalloc(16, 16, 16, 2, p(t), p(d), p(o), None) == -1
    assert lib().cl_interp_noalloc(16, 16, 16, 3, p(t), p(d), p(t), None) == -9
    with pytest.raises(ClaireError):
        interp_noalloc(t, d, t)
