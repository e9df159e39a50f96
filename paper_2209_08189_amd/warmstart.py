"""Learned warm start: data generation, training and evaluation.

Pairs come from the seeded brain-like phantom generator: m0 = phantom +
noise, m1 = phantom transported by a seeded smooth velocity (forward SL solve
through the library) + noise.  Labels are the plain FP32 Gauss-Newton
solver's converged velocities.  The network sees (m0, m1) and predicts v on
a coarser grid (spectral restriction / prolongation); it only proposes the
starting point of the solve, which stays the judge (a prediction that does
not lower the objective below J(0) is discarded).

Time-to-tolerance is wall time from images resident on the device to
||g|| <= gtol ||g(v = 0)|| for both runs; the learned run includes
restriction, inference, prolongation and the fallback test.
"""
import time

import numpy as np

from . import synth
from .claire import Net, Registration, Resampler, warm_start


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def make_pair(n, seed, max_disp=6.0):
    """Phantom pair on an n^3 grid.  Returns device tensors (m0, m1) and the
    labels of the clean phantom (host)."""
    shape = (n, n, n)
    img, labels = synth.phantom(shape, seed)
    v_true = synth.smooth_velocity(shape, seed + 1, kmax=8.0, max_disp_voxels=max_disp)
    reg = Registration(shape)
    ph = _dev(img)
    reg.set_images(ph, ph)
    reg.set_velocity(_dev(v_true))
    m1 = reg.deformed_template() + _dev(synth.noise(shape, seed + 3, 0.02))
    m0 = ph + _dev(synth.noise(shape, seed + 2, 0.02))
    reg.close()
    return m0, m1, labels


def solve(m0, m1, storage=("f32", "f32"), gtol=1e-2, net=None, max_outer=50, max_pcg=10):
    """Gauss-Newton solve from v = 0 (or from the network's warm start).
    Returns (report dict, final velocity tensor, seconds)."""
    import torch
    shape = tuple(m0.shape)
    reg = Registration(shape, gtol=gtol, max_outer=max_outer, max_pcg=max_pcg,
                       storage_state=storage[0], storage_adjoint=storage[1])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    reg.set_images(m0, m1)
    used = False
    if net is not None:
        used, _, _ = warm_start(reg, net)
    rep = reg.solve()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    rep["warm_start_used"] = used
    v = reg.velocity()
    reg.close()
    return rep, v, dt


def generate(seeds, n=256, n_net=128, log=None):
    """Training data on the network grid: list of (m0, m1, v_label) device
    tensors restricted from n^3 solves."""
    down = Resampler((n,) * 3, (n_net,) * 3)
    data = []
    for s in seeds:
        m0, m1, _ = make_pair(n, s)
        rep, v, dt = solve(m0, m1)
        data.append((down(m0), down(m1), down(v)))
        if log:
            log("label seed %d: %d GN, %d PCG, %.2f s" % (s, rep["outer_iters"], rep["pcg_iters_total"], dt))
    return data


def train(net, data, epochs, batch=1, log=None, seed=0):
    """Adam on the mean squared velocity error, shuffled each epoch."""
    import torch
    rng = np.random.default_rng(seed)
    hist = []
    for ep in range(epochs):
        order = rng.permutation(len(data))
        tot = 0.0
        for i in range(0, len(order), batch):
            idx = order[i:i + batch]
            m0 = torch.cat([data[k][0].reshape(-1) for k in idx])
            m1 = torch.cat([data[k][1].reshape(-1) for k in idx])
            lab = torch.cat([data[k][2].reshape(-1) for k in idx])
            tot += net.train_step(m0, m1, lab, batch=len(idx)) * len(idx)
        hist.append(tot / len(data))
        if log:
            log("epoch %d: loss %.4e" % (ep, hist[-1]))
    return hist


def evaluate(net, seeds, n=256, storage=("f16", "bf16"), log=None):
    """Per held-out seed: plain FP32 solve from v = 0 versus warm start +
    mixed-precision storage.  Returns a list of dicts."""
    rows = []
    for s in seeds:
        m0, m1, _ = make_pair(n, s)
        rp, vp, tp = solve(m0, m1)
        rl, vl, tl = solve(m0, m1, storage=storage, net=net)
        row = {"seed": s, "plain_s": tp, "plain_gn": rp["outer_iters"], "plain_pcg": rp["pcg_iters_total"],
               "plain_mismatch": rp["mismatch"], "learned_s": tl, "learned_gn": rl["outer_iters"],
               "learned_pcg": rl["pcg_iters_total"], "learned_mismatch": rl["mismatch"],
               "used_prediction": rl["warm_start_used"],
               "rel_mismatch_diff": abs(rl["mismatch"] - rp["mismatch"]) / rp["mismatch"],
               "status_plain": rp["status_name"], "status_learned": rl["status_name"]}
        rows.append(row)
        if log:
            log("eval seed %d: plain %.2f s (%d GN), learned+mixed %.2f s (%d GN, used=%s), mismatch diff %.2e"
                % (s, tp, rp["outer_iters"], tl, rl["outer_iters"], row["used_prediction"], row["rel_mismatch_diff"]))
    return rows
