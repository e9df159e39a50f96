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
import multiprocessing
import os
import time

import numpy as np

from . import synth
from .claire import Net, Registration, Resampler, warm_start


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def host_pair(n, seed, max_disp=6.0):
    """CPU side of a phantom pair: (phantom, labels, v_true, noise of m0,
    noise of m1), FP32 except the labels."""
    shape = (n, n, n)
    img, labels = synth.phantom(shape, seed)
    v_true = synth.smooth_velocity(shape, seed + 1, kmax=8.0, max_disp_voxels=max_disp)
    return (img.astype(np.float32), labels, v_true.astype(np.float32),
            synth.noise(shape, seed + 2, 0.02).astype(np.float32),
            synth.noise(shape, seed + 3, 0.02).astype(np.float32))


def _host_pair_job(args):
    return host_pair(*args)


def _pool_init():
    synth.FFT_WORKERS = 1


class HostPairs:
    """Process pool that generates the CPU side of phantom pairs.  Create it
    before the process touches the GPU (the workers are separate interpreters
    started by the spawn method); each worker is single-threaded."""

    def __init__(self, procs=None):
        procs = procs or max(1, min(16, (os.cpu_count() or 2) - 1))
        saved = {k: os.environ.get(k) for k in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS")}
        os.environ["OMP_NUM_THREADS"] = os.environ["OPENBLAS_NUM_THREADS"] = "1"
        try:
            self.pool = multiprocessing.get_context("spawn").Pool(procs, initializer=_pool_init)
        finally:
            for k, v in saved.items():
                if v is None:
                    os.environ.pop(k, None)
                else:
                    os.environ[k] = v

    def pairs(self, n, seeds, ahead=32):
        """Pairs in seed order, at most `ahead` generated ahead of the
        consumer (each pair holds about 0.5 GB of host memory at 256^3)."""
        from collections import deque
        seeds = list(seeds)
        q, k = deque(), 0
        while k < len(seeds) and len(q) < ahead:
            q.append(self.pool.apply_async(_host_pair_job, ((n, seeds[k]),)))
            k += 1
        while q:
            r = q.popleft().get()
            if k < len(seeds):
                q.append(self.pool.apply_async(_host_pair_job, ((n, seeds[k]),)))
                k += 1
            yield r

    def close(self):
        self.pool.close()
        self.pool.join()


def device_pair(host, with_velocity=False):
    """Device images (m0, m1) from host_pair(): m0 = phantom + noise, m1 =
    phantom transported by v_true (forward SL solve on the GPU) + noise; the
    clean phantom's labels (host); with_velocity: also v_true (device)."""
    img, labels, v_true, n0, n1 = host
    n = img.shape[0]
    reg = Registration((n, n, n))
    ph = _dev(img)
    vt = _dev(v_true)
    reg.set_images(ph, ph)
    reg.set_velocity(vt)
    m1 = reg.deformed_template() + _dev(n1)
    m0 = ph + _dev(n0)
    reg.close()
    return (m0, m1, labels, vt) if with_velocity else (m0, m1, labels)


def make_pair(n, seed, max_disp=6.0):
    """Phantom pair on an n^3 grid: device tensors (m0, m1) and the labels of
    the clean phantom (host)."""
    return device_pair(host_pair(n, seed, max_disp))


def solve(m0, m1, storage=("f32", "f32"), gtol=1e-2, net=None, max_outer=50, max_pcg=40, precond="spectral",
          precond_inner=12):
    """Gauss-Newton solve from v = 0 (or from the network's warm start).
    Returns (report dict, final velocity tensor, seconds)."""
    import torch
    shape = tuple(m0.shape)
    reg = Registration(shape, gtol=gtol, max_outer=max_outer, max_pcg=max_pcg,
                       storage_state=storage[0], storage_adjoint=storage[1], precond=precond,
                       precond_inner=precond_inner)
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


def generate(seeds, n=256, n_net=128, log=None, host=None, max_pcg=40, precond="spectral", log_every=1):
    """Training data on the network grid: list of (m0, m1, v_label) device
    tensors restricted from n^3 solves.  host: a HostPairs pool (optional);
    precond: preconditioner of the labelling solves."""
    down = Resampler((n,) * 3, (n_net,) * 3)
    data = []
    src = host.pairs(n, seeds) if host else (host_pair(n, s) for s in seeds)
    t0 = time.perf_counter()
    for i, (s, hp) in enumerate(zip(seeds, src)):
        m0, m1, _ = device_pair(hp)
        del hp
        rep, v, dt = solve(m0, m1, max_pcg=max_pcg, precond=precond)
        data.append((down(m0), down(m1), down(v)))
        if log and (i % log_every == 0 or i == len(seeds) - 1):
            log("label %d/%d seed %d: %d GN, %d PCG, %.2f s, %s (%.0f s elapsed)"
                % (i + 1, len(seeds), s, rep["outer_iters"], rep["pcg_iters_total"], dt, rep["status_name"],
                   time.perf_counter() - t0))
    return data


def predict(net, m0, m1):
    """The network's velocity on the grid of (m0, m1): restriction to the
    network grid, inference, spectral prolongation."""
    n = m0.shape[0]
    nn = net.n
    down = Resampler((n,) * 3, (nn,) * 3)
    up = Resampler((nn,) * 3, (n,) * 3)
    return up(net.forward(down(m0), down(m1)))


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


def evaluate(net, seeds, n=256, storage=("f16", "f16"), log=None, host=None, max_pcg=40):
    """Per held-out seed: plain FP32 solve from v = 0, mixed-precision storage
    from v = 0, warm start in FP32, and warm start + mixed storage.  Returns a
    list of dicts (times in seconds, GN iterations, mismatches, and the
    relative L2 error of the network's prediction against the plain
    solution)."""
    from .metrics import dice, warp_labels
    rows = []
    src = host.pairs(n, seeds) if host else (host_pair(n, s) for s in seeds)
    for s, hp in zip(seeds, src):
        m0, m1, lab0, v_true = device_pair(hp, with_velocity=True)
        del hp
        lab1 = warp_labels(lab0, v_true)           # labels of m1
        mis0 = 0.5 * float(((m0 - m1).double() ** 2).sum()) * (2.0 * np.pi / n) ** 3
        rp, vp, tp = solve(m0, m1, max_pcg=max_pcg)
        rm, _, tm = solve(m0, m1, storage=storage, max_pcg=max_pcg)
        rf, _, tf = solve(m0, m1, net=net, max_pcg=max_pcg)
        rl, vl, tl = solve(m0, m1, storage=storage, net=net, max_pcg=max_pcg)
        pred = predict(net, m0, m1)
        err = float((pred - vp).norm() / vp.norm())
        d_pre = dice(lab0, lab1)["D_vw"]
        d_plain = dice(warp_labels(lab0, vp), lab1)["D_vw"]
        d_learned = dice(warp_labels(lab0, vl), lab1)["D_vw"]
        row = {"seed": s, "plain_s": tp, "plain_gn": rp["outer_iters"], "plain_pcg": rp["pcg_iters_total"],
               "mixed_s": tm, "mixed_gn": rm["outer_iters"], "learned_f32_s": tf, "learned_f32_gn": rf["outer_iters"],
               "pred_rel_err": err, "dice_vw_pre": d_pre, "dice_vw_plain": d_plain, "dice_vw_learned": d_learned,
               "plain_mismatch": rp["mismatch"], "learned_s": tl, "learned_gn": rl["outer_iters"],
               "learned_pcg": rl["pcg_iters_total"], "learned_mismatch": rl["mismatch"],
               "used_prediction": rl["warm_start_used"],
               "rel_mismatch_diff": abs(rl["mismatch"] - rp["mismatch"]) / rp["mismatch"],
               # relative mismatch r = mismatch / mismatch at v = 0 (the
               # convention of the paper's tables); absolute difference in r
               "abs_diff_r": abs(rl["mismatch"] - rp["mismatch"]) / mis0,
               "status_plain": rp["status_name"], "status_learned": rl["status_name"]}
        rows.append(row)
        if log:
            log("eval seed %d: plain %.2f s (%d GN), mixed %.2f s (%d GN), learned %.2f s (%d GN), learned+mixed "
                "%.2f s (%d GN, used=%s), prediction error %.3f, mismatch diff %.2e (in r: %.2e)"
                % (s, tp, rp["outer_iters"], tm, rm["outer_iters"], tf, rf["outer_iters"], tl, rl["outer_iters"],
                   row["used_prediction"], err, row["rel_mismatch_diff"], row["abs_diff_r"]))
    return rows
