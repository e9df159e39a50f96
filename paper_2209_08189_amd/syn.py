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
does to keep the CFL number fixed, and is 4 for tricubic; --nt-max caps it.
A 1024^3 context with n_t = 16 takes 244 GiB with 16-bit field storage (the
lean layout), so at that size the images and velocities stay in host memory
and enter the device only while a context copies them, and the base level
is scored with its own solving context.

At large base grids: --gen-nt / --gen-storage set the generator's steps and
field storage, --storage the registration contexts' field storage, and
--top-from-coarse registers the base level by one GN solve at the weights
the next coarser level's search found, warm-started from that level's
prolonged velocity, run in calls of --top-chunk GN iterations (the levels
are then processed coarse to fine).

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
    ap.add_argument("--nt-max", type=int, default=0, help="cap on n_t of the registrations (0: none)")
    ap.add_argument("--gen-nt", type=int, default=32, help="n_t of the forward solve that makes the reference")
    ap.add_argument("--gen-storage", default="f32", choices=["f32", "f16", "bf16"])
    ap.add_argument("--storage", default="f32", choices=["f32", "f16", "bf16"],
                    help="field storage of the registration and evaluation contexts")
    ap.add_argument("--top-from-coarse", action="store_true")
    ap.add_argument("--top-chunk", type=int, default=2)
    ap.add_argument("--gtol", type=float, default=1e-2,
                    help="relative gradient tolerance of every solve (the paper's SYN runs use 5e-2)")
    a = ap.parse_args()
    log = lambda m: print("[syn] " + m, file=sys.stderr, flush=True)
    import torch
    from . import synth
    from .claire import Registration, Resampler
    from .metrics import dice, warp_labels
    torch.cuda.set_device(0)
    n = a.n
    shape = (n,) * 3
    st = {"storage_state": a.storage, "storage_adjoint": a.storage}

    def nt_for(L):
        nt = max(4, 4 * L // 256) if a.interp == "linear" else 4
        return min(nt, a.nt_max) if a.nt_max else nt

    t_in = time.perf_counter()
    labels0 = synth.syn_template(shape, a.seed, rscale=a.rscale, log=log if n >= 512 else None)
    log("template %.1f s" % (time.perf_counter() - t_in))
    v_syn = torch.from_numpy(synth.syn_velocity(shape, a.K) * np.float32(a.vscale)).cuda()
    m0 = torch.from_numpy(labels0.astype(np.float32) / 10.0).cuda()
    log("inputs %.1f s" % (time.perf_counter() - t_in))
    gen = Registration(shape, nt=a.gen_nt, interp=a.interp, storage_state=a.gen_storage,
                       storage_adjoint=a.gen_storage)
    gen.set_images(m0, m0)
    gen.set_velocity(v_syn)
    m1 = gen.deformed_template()
    labels1 = warp_labels(labels0, None, nlabels=11, reg=gen)
    gen.close()
    del gen, v_syn
    torch.cuda.empty_cache()
    # labels present in the reference (an empty label would score Dice 1)
    labels1 = labels1.cpu().numpy()
    cnt1 = np.bincount(labels1.ravel(), minlength=11)
    lab_ids = tuple(i for i in range(1, 11) if cnt1[i] > 0)
    pre = dice(labels0, labels1, labels=lab_ids)
    log("inputs: %d^3, K %d, label voxels %s, scored labels %s, Dice before D_a %.4f"
        % (n, a.K, np.bincount(labels0.ravel(), minlength=11)[1:].tolist(), lab_ids, pre["D_a"]))
    out = {"n": n, "K": a.K, "seed": a.seed, "interp": a.interp, "jmin": a.jmin, "rscale": a.rscale,
           "vscale": a.vscale, "gen_nt": a.gen_nt, "gen_storage": a.gen_storage, "storage": a.storage,
           "top_from_coarse": a.top_from_coarse, "label_voxels": np.bincount(labels0.ravel(), minlength=11)[1:].tolist(),
           "scored_labels": list(lab_ids), "dice_pre": pre, "levels": []}
    mis0 = 0.5 * float(((m0 - m1).double() ** 2).sum()) * (2 * np.pi / n) ** 3
    # host copies of the images: at 1024^3 with n_t = 16 a context takes most
    # of the device, so the images (and velocities) are moved in only while a
    # context copies them
    m0_h, m1_h = m0.cpu(), m1.cpu()
    labels0_u8 = labels0.astype(np.uint8)
    big = n >= 1024

    def images_into(reg):
        a0, a1 = m0_h.cuda(), m1_h.cuda()
        reg.set_images(a0, a1)
        del a0, a1
        torch.cuda.empty_cache()

    def velocity_into(reg, v_h):
        vd = v_h.cuda()
        reg.set_velocity(vd)
        del vd
        torch.cuda.empty_cache()

    def free_mib():
        f, t = torch.cuda.mem_get_info()
        return "%.1f of %.1f GiB free" % (f / 2 ** 30, t / 2 ** 30)

    if big:
        del m0, m1
        torch.cuda.empty_cache()
    levels = [int(x) for x in a.levels.split(",")]
    if a.top_from_coarse:
        levels = sorted(levels)
    prev = None   # (beta_v, beta_w, velocity on the base grid) of the last level
    for L in levels:
        s = n // L
        nt = nt_for(L)
        if L == n and a.top_from_coarse and prev is not None:
            # one solve at the coarser level's weights from its velocity
            bv, bw, vp = prev
            vp_h = vp.cpu()
            del vp
            prev = None
            torch.cuda.empty_cache()
            reg = Registration(shape, nt=nt, interp=a.interp, beta_v=bv, beta_w=bw, max_outer=a.top_chunk,
                               max_pcg=a.max_pcg, gtol=a.gtol, **st)
            log("level %d: context n_t %d (layout %d), %s" % (L, nt, reg.layout(), free_mib()))
            images_into(reg)
            velocity_into(reg, vp_h)
            del vp_h
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            gn = pcg = 0
            while True:
                rep = reg.solve()
                gn += rep["outer_iters"]
                pcg += rep["pcg_iters_total"]
                log("level %d: %d GN, %d PCG, rel grad %.3g, %s, %.1f s"
                    % (L, gn, pcg, rep["gnorm"] / rep["gref"], rep["status_name"], time.perf_counter() - t0))
                if rep["status_name"] != "maxit" or gn >= a.max_outer:
                    break
            torch.cuda.synchronize()
            ts = time.perf_counter() - t0
            _, jl, jh = reg.jacobian_det()
            srep = {"beta_v": bv, "beta_w": bw, "solves": 1, "gn_total": gn, "pcg_total": pcg, "jmin": jl,
                    "jmax": jh, "status_name": rep["status_name"]}
        else:
            m0c = m0_h[::s, ::s, ::s].contiguous().cuda()
            m1c = m1_h[::s, ::s, ::s].contiguous().cuda()
            reg = Registration((L,) * 3, nt=nt, interp=a.interp, max_outer=a.max_outer, max_pcg=a.max_pcg,
                               gtol=a.gtol, **st)
            reg.set_images(m0c, m1c)
            del m0c, m1c
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            srep = reg.param_search(jmin=a.jmin, verbose=1)
            torch.cuda.synchronize()
            ts = time.perf_counter() - t0
        vc = reg.velocity()
        if L == n:
            # the base grid itself: score with the solving context
            v = vc
            base = reg
        else:
            reg.close()
            del reg
            v = Resampler((L,) * 3, shape)(vc)
            base = None
        del vc
        torch.cuda.empty_cache()
        # the prolonged velocity on the base grid: labels, relative mismatch
        # and J bounds there
        if base is None:
            v_h = v.cpu() if big else None
            if big:
                del v
                torch.cuda.empty_cache()
            base = Registration(shape, nt=nt_for(n), interp=a.interp, **st)
            images_into(base)
            if big:
                velocity_into(base, v_h)
                v = v_h
            else:
                base.set_velocity(v)
        elif big:
            v = v.cpu()
            torch.cuda.empty_cache()
            images_into(base)
        J, mis, _ = base.objective()
        _, jlo, jhi = base.jacobian_det()
        if big:
            log("level %d scoring: %s" % (L, free_mib()))
        lw = warp_labels(labels0_u8, None, nlabels=11, reg=base)
        base.close()
        del base
        torch.cuda.empty_cache()
        d = dice(lw, labels1, labels=lab_ids)
        del lw
        row = {"level": L, "nt": nt, "beta_v": srep["beta_v"], "beta_w": srep["beta_w"], "search_s": ts,
               "solves": srep["solves"], "gn_total": srep["gn_total"], "pcg_total": srep["pcg_total"],
               "J_range_level": [srep["jmin"], srep["jmax"]], "J_range_base": [jlo, jhi], "r_base": mis / mis0,
               "dice": d}
        if L == n and a.top_from_coarse and "status_name" in srep:
            row["protocol"] = "one solve at the coarser level's weights from its prolonged velocity"
            row["status"] = srep["status_name"]
        out["levels"].append(row)
        log("level %d: beta_v %.3g beta_w %.3g, %d solves %.1f s, r %.4f, Dice D_a %.4f D_vw %.4f D_ivw %.4f"
            % (L, srep["beta_v"], srep["beta_w"], srep["solves"], ts, row["r_base"], d["D_a"], d["D_vw"], d["D_ivw"]))
        if a.top_from_coarse and L < n:
            prev = (srep["beta_v"], srep["beta_w"], v)
        del v
        torch.cuda.empty_cache()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
