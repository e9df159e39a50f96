"""FP32 against 16-bit field storage on one 512^3 phantom pair (the
benchmark's phantom recipe at 512^3, same voxel-unit parameters): time to
||g|| <= 1e-2 g_ref, GN / PCG iterations, relative mismatch r, Dice of the
warped labels and the device workspace of both configurations.

    python -m paper_2209_08189_amd.mixed512 [--n 512] [--seed 0] > result.json
"""
import argparse
import json
import sys
import time


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--n", type=int, default=512)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--max-pcg", type=int, default=40)
    a = ap.parse_args()
    from . import warmstart
    log = lambda m: print("[mixed512] " + m, file=sys.stderr, flush=True)
    t = time.perf_counter()
    hp = warmstart.host_pair(a.n, a.seed)
    log("inputs %.1f s" % (time.perf_counter() - t))
    import torch
    from .claire import Registration, query_workspace
    from .metrics import dice, relative_mismatch, warp_labels
    torch.cuda.set_device(0)
    m0, m1, lab0, v_true = warmstart.device_pair(hp, with_velocity=True)
    del hp
    lab1 = warp_labels(lab0, v_true)
    out = {"n": a.n, "seed": a.seed, "max_pcg": a.max_pcg, "dice_pre": dice(lab0, lab1)}
    for name, st in (("fp32", ("f32", "f32")), ("f16", ("f16", "f16"))):
        rep, v, dt = warmstart.solve(m0, m1, storage=st, max_pcg=a.max_pcg)
        reg = Registration(tuple(m0.shape))
        reg.set_images(m0, m1)
        reg.set_velocity(v)
        mt = reg.deformed_template()
        reg.close()
        out[name] = {"storage": st, "time_to_tol_s": dt, "gn": rep["outer_iters"], "pcg": rep["pcg_iters_total"],
                     "status": rep["status_name"], "r": relative_mismatch(m1, mt, m0),
                     "dice_post": dice(warp_labels(lab0, v), lab1),
                     "workspace_GB": query_workspace(tuple(m0.shape), storage_state=st[0],
                                                     storage_adjoint=st[1]) / 1e9}
        log("%s: %s" % (name, json.dumps({k: x for k, x in out[name].items() if k != "dice_post"})))
        del v
    out["abs_diff_r"] = abs(out["f16"]["r"] - out["fp32"]["r"])
    out["diff_dice_vw"] = out["f16"]["dice_post"]["D_vw"] - out["fp32"]["dice_post"]["D_vw"]
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
