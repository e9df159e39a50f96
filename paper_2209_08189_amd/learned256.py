"""Learned warm start at its full scale: 2000 training pairs of the 256^3
brain-like phantom (seeds 1000-2999), each labelled with the converged
velocity of the plain Gauss-Newton solve (relative gradient 1e-2, images
and label restricted spectrally to the network's 128^3 grid), and 100
held-out pairs (seeds 10000-10099) on which the solve is timed from v = 0
and from the network's prediction.

Two steps, each one process:

  python -m paper_2209_08189_amd.learned256 train --out DIR [--init-params P]
      labels + Adam training; writes DIR/net_params.npy and DIR/train.json.
      The 2000 labelling solves take longer than one GPU session allows and
      labels do not outlive a session, so the training set is labelled and
      trained in shards (seeds 1000-1999, then 2000-2999 starting from the
      first shard's parameters)
  python -m paper_2209_08189_amd.learned256 eval --params DIR/net_params.npy --out FILE.json
      per held-out seed: plain FP32 and learned + mixed-precision solves, with
      the spectral preconditioner and with the zero-velocity preconditioner

  python -m paper_2209_08189_amd.learned256 step [--n 128] [--steps 3]
      times training steps and forward passes on random inputs (the
      convolution kernels' workload, for profiling)

Progress goes to stderr, one line per step.
"""
import argparse
import json
import os
import sys
import time

import numpy as np


def log(msg):
    print("[learned256] " + msg, file=sys.stderr, flush=True)


def seed_range(s):
    a, b = s.split(":")
    return list(range(int(a), int(b)))


def label_pairs(seeds, n, host, precond, max_pcg, log_every):
    """Training pairs restricted to the network grid: (m0, m1, v) with v the
    converged velocity of the Gauss-Newton solve from v = 0 (relative
    gradient 1e-2).  One context transports the phantom to make m1, one
    solves; both are reused from pair to pair (set_images / set_velocity
    reset every derived quantity).  Returns the pairs and per-pair solve
    records."""
    import torch
    from .claire import Registration, Resampler
    from .warmstart import _dev
    shape = (n,) * 3
    fwd = Registration(shape)
    sol = Registration(shape, gtol=1e-2, max_outer=50, max_pcg=max_pcg, precond=precond, precond_inner=12)
    down = Resampler(shape, (n // 2,) * 3)
    zero = torch.zeros((3,) + shape, dtype=torch.float32, device="cuda")
    data, recs = [], []
    t0 = time.perf_counter()
    for i, (s, hp) in enumerate(zip(seeds, host.pairs(n, seeds))):
        img, _, v_true, n0, n1 = hp
        ph = _dev(img)
        fwd.set_images(ph, ph)
        fwd.set_velocity(_dev(v_true))
        m1 = fwd.deformed_template() + _dev(n1)
        m0 = ph + _dev(n0)
        torch.cuda.synchronize()
        ts = time.perf_counter()
        sol.set_images(m0, m1)
        sol.set_velocity(zero)
        rep = sol.solve()
        torch.cuda.synchronize()
        dt = time.perf_counter() - ts
        data.append((down(m0), down(m1), down(sol.velocity())))
        recs.append({"seed": s, "s": dt, "gn": rep["outer_iters"], "pcg": rep["pcg_iters_total"],
                     "status": rep["status_name"], "rel_grad": rep["gnorm"] / rep["gref"]})
        if i % log_every == 0 or i == len(seeds) - 1:
            log("label %d/%d seed %d: %d GN, %d PCG, %.2f s, %s (%.0f s elapsed)"
                % (i + 1, len(seeds), s, rep["outer_iters"], rep["pcg_iters_total"], dt, rep["status_name"],
                   time.perf_counter() - t0))
    fwd.close()
    sol.close()
    return data, recs


def cmd_train(args):
    from . import warmstart
    host = warmstart.HostPairs()          # before the GPU is touched
    import torch
    from .claire import Net
    torch.cuda.set_device(0)
    seeds = seed_range(args.train_seeds)
    t0 = time.perf_counter()
    data, recs = label_pairs(seeds, args.n, host, args.label_precond, args.max_pcg, args.log_every)
    t_label = time.perf_counter() - t0
    host.close()
    log("labels: %d pairs in %.1f s" % (len(data), t_label))
    net = Net(in_n=args.n // 2, seed=1, lr=args.lr)
    if args.init_params:
        # continue from the parameters of an earlier shard (fresh Adam moments)
        net.set_params(torch.from_numpy(np.load(args.init_params)).cuda())
        log("initial parameters from %s" % args.init_params)
    t1 = time.perf_counter()
    hist = warmstart.train(net, data, args.epochs, batch=args.batch, log=log, seed=0)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t1
    # prediction error on the training labels (first 20 pairs)
    errs = []
    for m0, m1, lab in data[:20]:
        pred = net.forward(m0, m1)
        errs.append(float((pred - lab).norm() / lab.norm()))
    os.makedirs(args.out, exist_ok=True)
    np.save(os.path.join(args.out, "net_params.npy"), net.params().cpu().numpy())
    rec = {"train_seeds": args.train_seeds, "init_params": os.path.basename(args.init_params or ""),
           "label_solves": recs, "pairs": len(data), "grid": args.n, "net_grid": args.n // 2,
           "label_precond": args.label_precond, "max_pcg": args.max_pcg, "epochs": args.epochs,
           "batch": args.batch, "lr": args.lr, "label_s": t_label, "train_s": t_train,
           "train_sample_steps": args.epochs * len(data), "loss_per_epoch": hist,
           "train_pred_rel_err_first20": errs}
    json.dump(rec, open(os.path.join(args.out, "train.json"), "w"), indent=1)
    log("training: %d epochs in %.1f s, final loss %.4e, train prediction error %.3f"
        % (args.epochs, t_train, hist[-1], float(np.mean(errs))))


def summarise_training(tr):
    """A shard's training record with its per-pair labelling solves reduced
    to their statistics."""
    ls = tr.pop("label_solves", [])
    if ls:
        t = np.array([r["s"] for r in ls])
        tr["label_solve_s"] = {"mean": float(t.mean()), "max": float(t.max()), "total": float(t.sum())}
        tr["label_gn_mean"] = float(np.mean([r["gn"] for r in ls]))
        tr["label_pcg_mean"] = float(np.mean([r["pcg"] for r in ls]))
        tr["label_status"] = {k: int(sum(r["status"] == k for r in ls)) for k in sorted({r["status"] for r in ls})}
    return tr


def summarise(rows):
    """Means over the held-out seeds, the learned runs against the plain ones,
    and the spread between the two plain runs (spectral and zero-velocity
    preconditioner, both from v = 0 to the same tolerance): the latter is
    how far two correct stopping points of the same solve lie apart."""
    def mean(f):
        return float(np.mean([f(r) for r in rows]))

    summary = {}
    for name in ("plain", "learned_mixed", "plain_h0", "learned_mixed_h0"):
        summary[name] = {"time_to_tol_s": mean(lambda r: r[name]["s"]), "gn": mean(lambda r: r[name]["gn"]),
                         "pcg": mean(lambda r: r[name]["pcg"]), "r": mean(lambda r: r[name]["r"]),
                         "not_converged": int(sum(r[name]["status"] != "ok" for r in rows))}
    for a, b in (("learned_mixed", "plain"), ("learned_mixed_h0", "plain_h0"), ("plain_h0", "plain")):
        k = "%s_vs_%s" % (a, b)
        d_r = [abs(r[a]["r"] - r[b]["r"]) for r in rows]
        d_rel = [abs(r[a]["mismatch"] - r[b]["mismatch"]) / r[b]["mismatch"] for r in rows]
        ratio = [r[a]["s"] / r[b]["s"] for r in rows]
        summary[k] = {
            "mean_time_ratio": float(np.mean(ratio)),
            "ratio_of_mean_times": summary[a]["time_to_tol_s"] / summary[b]["time_to_tol_s"],
            "max_abs_diff_r": float(max(d_r)), "mean_abs_diff_r": float(np.mean(d_r)),
            "max_rel_mismatch_diff": float(max(d_rel)), "mean_rel_mismatch_diff": float(np.mean(d_rel)),
            "seeds_within_1e-3_rel_mismatch": int(sum(x <= 1e-3 for x in d_rel)),
            "seeds_within_1e-3_abs_r": int(sum(x <= 1e-3 for x in d_r))}
    summary["fallback_rate"] = mean(lambda r: 0.0 if r["learned_mixed"]["used_prediction"] else 1.0)
    summary["pred_rel_err"] = mean(lambda r: r["pred_rel_err"])
    summary["dice_vw"] = {"pre": mean(lambda r: r["dice_vw_pre"]), "plain": mean(lambda r: r["dice_vw_plain"]),
                          "learned_mixed": mean(lambda r: r["dice_vw_learned_mixed"])}
    return summary


def cmd_summarise(args):
    """Recompute the summary of an evaluation record from its rows."""
    rec = json.load(open(args.record))
    rec["summary"] = summarise(rec["rows"])
    json.dump(rec, open(args.out or args.record, "w"), indent=1)
    log("summary: %s" % json.dumps(rec["summary"]))


def cmd_eval(args):
    from . import warmstart
    host = warmstart.HostPairs()
    import torch
    from .claire import Net
    from .metrics import dice, warp_labels
    torch.cuda.set_device(0)
    n = args.n
    net = Net(in_n=n // 2, seed=1)
    net.set_params(torch.from_numpy(np.load(args.params)).cuda())
    seeds = seed_range(args.eval_seeds)
    storage = ("f16", "f16")
    rows = []
    t0 = time.perf_counter()
    for i, (s, hp) in enumerate(zip(seeds, host.pairs(n, seeds))):
        m0, m1, lab0, v_true = warmstart.device_pair(hp, with_velocity=True)
        del hp
        lab1 = warp_labels(lab0, v_true)
        mis0 = 0.5 * float(((m0 - m1).double() ** 2).sum()) * (2.0 * np.pi / n) ** 3
        row = {"seed": s, "mismatch_v0": mis0}
        legs = {
            "plain": dict(),
            "learned_mixed": dict(storage=storage, net=net),
            "plain_h0": dict(precond="h0"),
            "learned_mixed_h0": dict(storage=storage, net=net, precond="h0"),
        }
        vel = {}
        for name, kw in legs.items():
            rep, v, dt = warmstart.solve(m0, m1, max_pcg=args.max_pcg, **kw)
            row[name] = {"s": dt, "gn": rep["outer_iters"], "pcg": rep["pcg_iters_total"],
                         "mismatch": rep["mismatch"], "r": rep["mismatch"] / mis0, "rel_grad": rep["gnorm"] / rep["gref"],
                         "status": rep["status_name"], "used_prediction": bool(rep["warm_start_used"])}
            vel[name] = v
        pred = warmstart.predict(net, m0, m1)
        row["pred_rel_err"] = float((pred - vel["plain"]).norm() / vel["plain"].norm())
        row["dice_vw_pre"] = dice(lab0, lab1)["D_vw"]
        row["dice_vw_plain"] = dice(warp_labels(lab0, vel["plain"]), lab1)["D_vw"]
        row["dice_vw_learned_mixed"] = dice(warp_labels(lab0, vel["learned_mixed"]), lab1)["D_vw"]
        for a, b in (("learned_mixed", "plain"), ("learned_mixed_h0", "plain_h0")):
            row["%s_vs_%s" % (a, b)] = {
                "time_ratio": row[a]["s"] / row[b]["s"],
                "abs_diff_r": abs(row[a]["r"] - row[b]["r"]),
                "rel_mismatch_diff": abs(row[a]["mismatch"] - row[b]["mismatch"]) / row[b]["mismatch"]}
        rows.append(row)
        log("eval %d/%d seed %d: plain %.2f s (%d GN), learned+mixed %.2f s (%d GN, used %s), plain H0 %.2f s, "
            "learned+mixed H0 %.2f s; prediction error %.3f; |dr| %.1e (%.0f s elapsed)"
            % (i + 1, len(seeds), s, row["plain"]["s"], row["plain"]["gn"], row["learned_mixed"]["s"],
               row["learned_mixed"]["gn"], row["learned_mixed"]["used_prediction"], row["plain_h0"]["s"],
               row["learned_mixed_h0"]["s"], row["pred_rel_err"], row["learned_mixed_vs_plain"]["abs_diff_r"],
               time.perf_counter() - t0))
    host.close()

    summary = summarise(rows)
    rec = {"eval_seeds": args.eval_seeds, "grid": n, "net_grid": n // 2, "storage_mixed": list(storage),
           "max_pcg": args.max_pcg, "gtol": 1e-2, "params": os.path.basename(args.params),
           "summary": summary, "rows": rows}
    rec["training"] = [summarise_training(json.load(open(p))) for p in (args.train_record or []) if os.path.exists(p)]
    json.dump(rec, open(args.out, "w"), indent=1)
    log("summary: %s" % json.dumps(summary))


def cmd_step(args):
    """Time training steps (batch 2) and forward passes of the network on
    random inputs: the convolution kernels' workload, for profiling."""
    import torch
    from .claire import Net
    torch.cuda.set_device(0)
    n = args.n
    g = torch.Generator(device="cuda").manual_seed(0)
    m0 = torch.rand((2, n, n, n), device="cuda", generator=g)
    m1 = torch.rand((2, n, n, n), device="cuda", generator=g)
    lab = 0.01 * torch.randn((2, 3, n, n, n), device="cuda", generator=g)
    net = Net(in_n=n)
    net.train_step(m0, m1, lab, batch=2)
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(args.steps):
        loss = net.train_step(m0, m1, lab, batch=2)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t) / args.steps
    t = time.perf_counter()
    for _ in range(args.steps):
        net.forward(m0[0], m1[0])
    torch.cuda.synchronize()
    df = (time.perf_counter() - t) / args.steps
    print(json.dumps({"grid": n, "train_step_batch2_ms": dt * 1e3, "per_sample_ms": dt * 5e2,
                      "forward_ms": df * 1e3, "loss": loss}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    sm = sub.add_parser("summarise")
    sm.add_argument("--record", required=True)
    sm.add_argument("--out", default=None)
    st = sub.add_parser("step")
    st.add_argument("--n", type=int, default=128)
    st.add_argument("--steps", type=int, default=3)
    t = sub.add_parser("train")
    t.add_argument("--out", required=True)
    t.add_argument("--n", type=int, default=256)
    t.add_argument("--train-seeds", default="1000:3000")
    t.add_argument("--label-precond", default="h0", choices=["spectral", "h0"])
    t.add_argument("--max-pcg", type=int, default=40)
    t.add_argument("--epochs", type=int, default=10)
    t.add_argument("--batch", type=int, default=2)
    t.add_argument("--lr", type=float, default=1e-4)
    t.add_argument("--log-every", type=int, default=25)
    t.add_argument("--init-params", default=None, help="start from these parameters (an earlier shard's)")
    e = sub.add_parser("eval")
    e.add_argument("--params", required=True)
    e.add_argument("--out", required=True)
    e.add_argument("--train-record", action="append", help="train.json of each shard (repeatable)")
    e.add_argument("--n", type=int, default=256)
    e.add_argument("--eval-seeds", default="10000:10100")
    e.add_argument("--max-pcg", type=int, default=40)
    args = ap.parse_args()
    if args.cmd == "train":
        cmd_train(args)
    elif args.cmd == "step":
        cmd_step(args)
    elif args.cmd == "summarise":
        cmd_summarise(args)
    else:
        cmd_eval(args)


if __name__ == "__main__":
    main()
