"""Resolution study on the SYN pair (the paper's Experiment 2A on one GPU):
register the SYN template and reference at the base resolution and at
nearest-neighbour downsampled resolutions, each with the parameter search
under the Jacobian bounds, prolong every velocity spectrally to the base
grid and score the warped base labels by Dice against the reference labels.

Inputs: m0 = syn_template / 10 (ten solids, labels 0..10), m1 = m0
transported by the SYN velocity of frequency K (forward SL solve on the GPU
with n_t = 32 steps of the chosen interpolation), labels of m1 = the
template labels transported the same way.  As printed, the solids' radius
is at most 0.45 and the velocity moves points by up to sum_k k^-1/2 (2.8
for K = 4), so the solids rarely overlap (labels above 2 are empty) and a
solid is carried far outside itself (Dice 0 before and after registration):
--rscale and --vscale scale the radius and the velocity, and the record
states both.  n_t of the registrations grows
with the resolution (4 at 256^3) for trilinear interpolation, as the paper
does to keep the CFL number fixed, and is 4 for tricubic.

    python -m paper_2209_08189_amd.syn [--n 256] [--K 4] [--levels 256,128,64]
        [--interp linear] [--jmin 0.25] > result.json
"""
import argparse
import json
import sys
import time

import numpy as np


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--n", type=int, default=256)
    ap.add_argument("--K", type=int, default=4)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--levels", default="256,128,64")
    ap.add_argument("--interp", default="linear", choices=["linear", "cubic"])
    ap.add_argument("--jmin", type=float, default=0.25)
    ap.add_argument("--max-outer", type=int, default=20)
    ap.add_argument("--max-pcg", type=int, default=40)
    ap.add_argument("--rscale", type=float, default=2.5, help="radius scale of the SYN solids")
    ap.add_argument("--vscale", type=float, default=0.1, help="scale of the SYN velocity")
    a = ap.parse_args()
    log = lambda m: print("[syn] " + m, file=sys.stderr, flush=True)
    import torch
    from . import synth
    from .claire import Registration, Resampler
    from .metrics import dice, warp_labels
    torch.cuda.set_device(0)
    n = a.n
    shape = (n,) * 3
    labels0 = synth.syn_template(shape, a.seed, rscale=a.rscale)
    v_syn = torch.from_numpy(synth.syn_velocity(shape, a.K) * np.float32(a.vscale)).cuda()
    m0 = torch.from_numpy(labels0.astype(np.float32) / 10.0).cuda()
    gen = Registration(shape, nt=32, interp=a.interp)
    gen.set_images(m0, m0)
    gen.set_velocity(v_syn)
    m1 = gen.deformed_template()
    labels1 = warp_labels(labels0, None, nlabels=11, reg=gen)
    gen.close()
    del gen
    # labels present in the reference (an empty label would score Dice 1)
    cnt1 = np.bincount(labels1.cpu().numpy().ravel(), minlength=11)
    lab_ids = tuple(i for i in range(1, 11) if cnt1[i] > 0)
    pre = dice(labels0, labels1, labels=lab_ids)
    log("inputs: %d^3, K %d, label voxels %s, scored labels %s, Dice before D_a %.4f"
        % (n, a.K, np.bincount(labels0.ravel(), minlength=11)[1:].tolist(), lab_ids, pre["D_a"]))
    out = {"n": n, "K": a.K, "seed": a.seed, "interp": a.interp, "jmin": a.jmin, "rscale": a.rscale,
           "vscale": a.vscale, "label_voxels": np.bincount(labels0.ravel(), minlength=11)[1:].tolist(),
           "scored_labels": list(lab_ids), "dice_pre": pre, "levels": []}
    mis0 = 0.5 * float(((m0 - m1).double() ** 2).sum()) * (2 * np.pi / n) ** 3
    for L in [int(x) for x in a.levels.split(",")]:
        s = n // L
        nt = max(4, 4 * L // 256) if a.interp == "linear" else 4
        m0c = m0[::s, ::s, ::s].contiguous()
        m1c = m1[::s, ::s, ::s].contiguous()
        reg = Registration((L,) * 3, nt=nt, interp=a.interp, max_outer=a.max_outer, max_pcg=a.max_pcg)
        reg.set_images(m0c, m1c)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        srep = reg.param_search(jmin=a.jmin, verbose=1)
        torch.cuda.synchronize()
        ts = time.perf_counter() - t0
        vc = reg.velocity()
        reg.close()
        v = vc if L == n else Resampler((L,) * 3, shape)(vc)
        # the prolonged velocity on the base grid: labels, relative mismatch
        # and J bounds there
        base = Registration(shape, nt=max(4, 4 * n // 256) if a.interp == "linear" else 4, interp=a.interp)
        base.set_images(m0, m1)
        base.set_velocity(v)
        J, mis, _ = base.objective()
        _, jlo, jhi = base.jacobian_det()
        lw = warp_labels(labels0, None, nlabels=11, reg=base)
        base.close()
        d = dice(lw, labels1, labels=lab_ids)
        row = {"level": L, "nt": nt, "beta_v": srep["beta_v"], "beta_w": srep["beta_w"], "search_s": ts,
               "solves": srep["solves"], "gn_total": srep["gn_total"], "pcg_total": srep["pcg_total"],
               "J_range_level": [srep["jmin"], srep["jmax"]], "J_range_base": [jlo, jhi], "r_base": mis / mis0,
               "dice": d}
        out["levels"].append(row)
        log("level %d: beta_v %.3g beta_w %.3g, %d solves %.1f s, r %.4f, Dice D_a %.4f D_vw %.4f D_ivw %.4f"
            % (L, srep["beta_v"], srep["beta_w"], srep["solves"], ts, row["r_base"], d["D_a"], d["D_vw"], d["D_ivw"]))
        del v, vc
        torch.cuda.empty_cache()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
