"""The large single-GPU configuration: a 1024^3 phantom pair (about 400
blobs, widths 4-60 voxels, band-limited texture on 64 <= |k| <= 256,
velocity of 20-voxel maximum displacement, n_t = 4), FP32 and 16-bit field
storage; each context takes the full memory layout when it fits the free
device memory and the lean one otherwise.  Reports the layout, the device
workspace and the device memory in use, the per-kernel launch times and
algorithmic GB/s from a capped solve, the exact integer-shift roll at this
size, and the solve's progress (time, GN / PCG iterations, relative mismatch
and gradient per GN iteration, Dice of the warped labels).

A storage entry with the suffix "+h2" (e.g. "f16+h2") solves with the
two-level zero-velocity preconditioner (12 inner CG steps on the
half-resolution grid) instead of the spectral one.

A storage entry with the suffix "+ws" (e.g. "f32+ws") starts its solve from
the multilevel learned warm start instead of v = 0: the images spectrally
restricted to 256^3, the network's prediction there (network grid 128^3,
kept only if it lowers J below J(0)), a Gauss-Newton solve at 256^3 to the
relative gradient tolerance 1e-2, and the velocity spectrally prolonged to
n^3; the prolonged velocity is again kept only if it lowers J below J(0) at
n^3.  It is computed once, before the first context that uses it.

    python -m paper_2209_08189_amd.large [--n 1024] [--max-outer 4] [--storage f32,f32+ws,bf16]
        [--net-params net_params.npy] > result.json
"""
import argparse
import json
import os
import sys
import time

import numpy as np

# algorithmic bytes per node of the SL launches: three FP32 displacement
# components, the FP32 factor or source of the adjoint and incremental
# steps, and the gathered field and the output at storage precision
# (4 / 2 bytes); with FP32 storage these are the benchmark's 5, 6 and 6 fields
SL_FP32 = {"sl_state": 3, "sl_adjoint": 4, "sl_inc": 4}
SL_STORED = 2
STORAGE_BYTES = {"f32": 4, "f16": 2, "bf16": 2}


def sl_bytes_per_node(name, st):
    return 4 * SL_FP32[name] + STORAGE_BYTES[st] * SL_STORED


def learned_warm_start(m0, m1, n, params, coarse=256, net_n=128, log=None):
    """The multilevel learned warm start on host images m0, m1 (n^3, FP32):
    spectral restriction to coarse^3, the network's prediction there and a
    Gauss-Newton solve (FP32 fields, relative gradient tolerance 1e-2) from
    it, spectral prolongation of the velocity to n^3.  Runs before any n^3
    context exists (the resamplers of the n^3 grid take about 14 GB each at
    1024^3).  Returns (velocity on the host, record)."""
    import torch
    from .claire import Net, Registration, Resampler, warm_start
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    down = Resampler((n,) * 3, (coarse,) * 3)
    c0 = down(m0.cuda())
    c1 = down(m1.cuda())
    del down
    torch.cuda.empty_cache()
    torch.cuda.synchronize()
    t_restrict = time.perf_counter() - t0
    net = Net(in_n=net_n, seed=1)
    net.set_params(torch.from_numpy(np.load(params)).cuda())
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    reg = Registration((coarse,) * 3)
    reg.set_images(c0, c1)
    used, Jp, J0 = warm_start(reg, net)
    t_net = time.perf_counter() - t1
    rep = reg.solve()
    torch.cuda.synchronize()
    t_solve = time.perf_counter() - t1 - t_net
    mis0 = 0.5 * float(((c0.double() - c1.double()) ** 2).sum()) * (2 * np.pi / coarse) ** 3
    _, jl, jh = reg.jacobian_det()
    vc = reg.velocity()
    reg.close()
    net.close()
    del reg, net, c0, c1
    torch.cuda.empty_cache()
    t2 = time.perf_counter()
    up = Resampler((coarse,) * 3, (n,) * 3)
    vf = up(vc).cpu()
    del up, vc
    torch.cuda.empty_cache()
    t_prolong = time.perf_counter() - t2
    rec = {"coarse": coarse, "net_grid": net_n, "params": os.path.basename(params),
           "prediction_used": used, "J_pred": Jp, "J_zero": J0,
           "coarse_solve": {"gn": rep["outer_iters"], "pcg": rep["pcg_iters_total"], "status": rep["status_name"],
                            "r": rep["mismatch"] / mis0, "rel_grad": rep["gnorm"] / rep["gref"], "J_range": [jl, jh]},
           "restrict_s": t_restrict, "net_s": t_net, "coarse_solve_s": t_solve, "prolong_s": t_prolong,
           "total_s": time.perf_counter() - t0}
    if log:
        log("warm start: %s" % json.dumps(rec))
    return vf, rec


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--n", type=int, default=1024)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--max-outer", type=int, default=4)
    ap.add_argument("--max-pcg", type=int, default=40)
    ap.add_argument("--storage", default="f32,f16",
                    help="comma-separated runs: f32, f16 or bf16 field storage; the suffix +ws starts the solve "
                         "from the multilevel learned warm start (needs --net-params), +h2 takes the two-level "
                         "zero-velocity preconditioner")
    ap.add_argument("--net-params", default=None, help="parameters of the 128^3 warm-start network (.npy)")
    ap.add_argument("--search", type=float, default=0.0,
                    help="J_min of a parameter search (beta_v, beta_w) run instead of the plain solve (0: off)")
    ap.add_argument("--continuation", type=float, default=0.0,
                    help="beta_v target of a parameter continuation (beta_w = 0) run before the capped solve "
                         "is reported instead (0: plain solve from v = 0)")
    a = ap.parse_args()
    log = lambda m: print("[large] " + m, file=sys.stderr, flush=True)
    from . import synth
    n = a.n
    shape = (n, n, n)
    t = time.perf_counter()
    img, lab0 = synth.phantom_large(shape, a.seed, log=log)
    log("phantom %.1f s" % (time.perf_counter() - t))
    v_true = synth.smooth_velocity_large(shape, a.seed + 1, kmax=8.0, max_disp_voxels=20.0, log=log)
    n0 = synth.noise32(shape, a.seed + 2, 0.02)
    n1 = synth.noise32(shape, a.seed + 3, 0.02)
    log("inputs %.1f s" % (time.perf_counter() - t))
    import torch
    from .claire import K_NAMES, Registration, query_workspace
    from .metrics import dice, warp_labels
    torch.cuda.set_device(0)
    dev = lambda x: torch.from_numpy(np.ascontiguousarray(x)).cuda()
    out = {"n": n, "seed": a.seed, "max_outer": a.max_outer, "max_pcg": a.max_pcg, "runs": {}}
    for key in a.storage.split(","):
        parts = key.split("+")
        st, ws, h2 = parts[0], "ws" in parts[1:], "h2" in parts[1:]
        if st not in STORAGE_BYTES or any(x not in ("ws", "h2") for x in parts[1:]):
            raise SystemExit("unknown storage entry %r" % key)
        if ws and a.net_params is None:
            raise SystemExit("%s needs --net-params" % key)
        if ws and "v_ws" not in out:
            if "m1" not in out:
                raise SystemExit("a run from v = 0 must come before the first +ws run (it makes m1)")
            out["v_ws"], out["warm_start"] = learned_warm_start(torch.from_numpy(img + n0), out["m1"], n,
                                                                a.net_params, log=log)
        pc = {"precond": "h0_2level", "precond_inner": 12} if h2 else {}
        reg = Registration(shape, max_outer=a.max_outer, max_pcg=a.max_pcg, storage_state=st, storage_adjoint=st, **pc)
        free, total = torch.cuda.mem_get_info()
        run = {"storage": st, "warm_start": ws, "precond": "h0_2level" if h2 else "spectral",
               "layout": "lean" if reg.layout() else "full",
               "workspace_GB": query_workspace(shape, storage_state=st, storage_adjoint=st,
                                               workspace_cap=free if reg.layout() else 0, **pc) / 1e9,
               "device_in_use_GB": (total - free) / 1e9, "device_GB": total / 1e9}
        log("%s: layout %s, %.1f of %.1f GB in use" % (key, run["layout"], run["device_in_use_GB"], run["device_GB"]))
        # m1 = phantom transported by v_true and the labels of m1, made once
        # by the first (FP32) context and kept on the host; device tensors
        # are freed as soon as the context holds a copy
        if "m1" not in out:
            x = dev(img)
            reg.set_images(x, x)
            del x
            vd = dev(v_true)
            reg.set_velocity(vd)
            del vd
            m1h = reg.deformed_template()
            out["m1"] = (m1h + dev(n1)).cpu()
            del m1h
            out["lab1"] = warp_labels(lab0, None, reg=reg).cpu()
        m1 = out["m1"]
        lab1 = out["lab1"]
        # exact roll: 4 voxels per unit time along x1 -> m(1) = roll(m0, 4)
        vs = torch.zeros((3,) + shape, dtype=torch.float32, device="cuda")
        vs[0] = (2 * np.pi / n) * 4
        reg.set_velocity(vs)
        del vs
        x = dev(img)
        reg.set_images(x, x)
        rolled = reg.deformed_template()
        xs = x if st == "f32" else x.to(torch.float16 if st == "f16" else torch.bfloat16).float()
        run["exact_roll"] = bool(torch.equal(rolled, torch.roll(xs, 4, dims=0)))
        del xs
        del rolled, x
        m0 = torch.from_numpy(img + n0)
        mis0 = 0.5 * float(((m0.double() - m1.double()) ** 2).sum()) * (2 * np.pi / n) ** 3
        x0, x1 = m0.cuda(), m1.cuda()
        reg.set_images(x0, x1)
        del x0, x1, m0
        if ws:
            # the prolonged velocity is kept only if it lowers J below J(0)
            reg.set_velocity(torch.zeros((3,) + shape, dtype=torch.float32, device="cuda"))
            J0 = reg.objective()[0]
            reg.set_velocity(out["v_ws"].cuda())
            Jw = reg.objective()[0]
            run["J_zero"], run["J_warm"], run["warm_used"] = J0, Jw, bool(Jw < J0)
            if not Jw < J0:
                reg.set_velocity(torch.zeros((3,) + shape, dtype=torch.float32, device="cuda"))
        else:
            reg.set_velocity(torch.zeros((3,) + shape, dtype=torch.float32, device="cuda"))
        torch.cuda.empty_cache()
        reg.profile_enable(0xFF)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        if a.search > 0:
            srep = reg.param_search(jmin=a.search, verbose=1)
            slog = reg.search_log()
            run["search"] = {"jmin_bound": a.search, "beta_v": srep["beta_v"], "beta_w": srep["beta_w"],
                             "status": srep["status_name"], "solves": srep["solves"], "gn_total": srep["gn_total"],
                             "pcg_total": srep["pcg_total"], "J_range": [srep["jmin"], srep["jmax"]],
                             "trials": [{"beta_v": row[0], "beta_w": row[1], "J": [row[2], row[3]],
                                         "valid": bool(row[4]), "gn": int(row[5]), "pcg": int(row[6]),
                                         "status": int(row[7]), "r": row[8] / mis0, "s": row[9] / 1e3}
                                        for row in slog]}
            rep = reg.solve()   # report at (beta_v*, beta_w*) from the kept solution
        elif a.continuation > 0:
            # the continuation schedule (beta_v = 1, 0.1, ... down to
            # 10^ceil(log10 target), then the target; beta_w = 0), one solve
            # per call so that every stage reports as it ends
            sched = [1.0]
            stop = 10.0 ** np.ceil(np.log10(a.continuation))
            while sched[-1] > stop * (1 + 1e-9):
                sched.append(sched[-1] / 10.0)
            if abs(sched[-1] - a.continuation) > 1e-9 * a.continuation:
                sched.append(a.continuation)
            trials = []
            for bv in sched:
                reg.set_regularization(bv, 0.0)
                ts = time.perf_counter()
                rep = reg.solve()
                _, jl, jh = reg.jacobian_det()
                trials.append({"beta_v": bv, "J": [jl, jh], "gn": rep["outer_iters"], "pcg": rep["pcg_iters_total"],
                               "status": rep["status_name"], "r": rep["mismatch"] / mis0,
                               "rel_grad": rep["gnorm"] / rep["gref"], "s": time.perf_counter() - ts})
                log("%s: continuation beta_v %.3g: J [%.3f, %.3f], %d GN, %d PCG, %s, r %.4f, %.1f s"
                    % (st, bv, jl, jh, rep["outer_iters"], rep["pcg_iters_total"], rep["status_name"],
                       trials[-1]["r"], trials[-1]["s"]))
            run["continuation"] = {"beta_v": a.continuation, "trials": trials}
        else:
            rep = reg.solve()
        torch.cuda.synchronize()
        run["solve_s"] = time.perf_counter() - t0
        kern = {}
        for k, name in enumerate(K_NAMES):
            ms, cnt = reg.profile_query(k)
            if cnt:
                kern[name] = {"launches": cnt, "avg_launch_ms": ms / cnt}
                if name in SL_FP32:
                    kern[name]["alg_GBs"] = sl_bytes_per_node(name, st) * n ** 3 / (ms / cnt * 1e-3) / 1e9
        reg.profile_enable(0)
        run.update({"gn": rep["outer_iters"], "pcg": rep["pcg_iters_total"], "status": rep["status_name"],
                    "rel_grad": rep["gnorm"] / rep["gref"], "r": rep["mismatch"] / mis0, "kernels": kern})
        # per GN iteration: relative mismatch, relative gradient, PCG iterations, step length
        run["history"] = [{"r": row[2] / mis0, "rel_grad": row[4] / rep["gref"], "pcg": int(row[5]),
                           "alpha": row[6]} for row in reg.solve_log()]
        run["dice_pre"] = dice(lab0, lab1)
        run["dice_post"] = dice(warp_labels(lab0, None, reg=reg), lab1)   # the solved velocity
        _, jl, jh = reg.jacobian_det()
        run["J_range"] = [jl, jh]
        log("%s: %s" % (key, json.dumps({k: x for k, x in run.items() if k not in ("kernels",)})))
        out["runs"][key] = run
        reg.close()
        del reg
        torch.cuda.empty_cache()
    for k in ("m1", "lab1", "v_ws"):
        out.pop(k, None)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
