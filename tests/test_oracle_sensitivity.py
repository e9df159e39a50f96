"""Sensitivity of the closed-form 64^3 problem's 5-step iterate (5 GN steps
x <= 10 PCG, decisions replayed) to relative perturbations of the matvec,
measured on the FP64 oracle itself (its sensitivity probe).

The stored envelope (tests/golden/cfg1_replay_spread.json, written by
make_cfg1_replay_spread.py from the oracle alone) sets the GPU replay's
bound: after the first PCG that stops unconverged at its iteration limit,
perturbations of 1e-8 relative -- below single-precision rounding -- move
the iterate by ~1e-3 in v and ~1e-2 in mismatch, and even 1e-12 moves the
mismatch by ~5e-3.  No single-precision implementation can be held to 1e-3
on this iterate; the 1e-3 bar applies to converged solves."""
import json
import os
import sys

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.join(HERE, "golden"))

GOLDEN = os.path.join(HERE, "golden", "cfg1_replay_spread.json")


@pytest.mark.slow
def test_replay_spread_reproduces_and_exceeds_bar(orc):
    import make_cfg1_replay_spread as mk
    rec = json.load(open(GOLDEN))
    o, shape = mk.problem()
    log, vref = mk.reference(o, shape)
    assert log[:-1, 5].astype(int).tolist() == rec["reference_pcg_iters"]
    assert abs(log[-1, 2] - rec["reference_final_mismatch"]) <= 1e-12 * rec["reference_final_mismatch"]
    # the oracle is deterministic (serial sums), so a stored run reproduces
    stored = [r for r in rec["runs"] if r["eps"] == 1e-8 and r["seed"] == 1][0]
    v, em = mk.replay(o, shape, log, 1e-8, 1)
    ev = np.linalg.norm(v - vref) / np.linalg.norm(vref)
    assert abs(ev - stored["rel_v"]) <= 1e-6 * stored["rel_v"]
    assert abs(em - stored["rel_mismatch"]) <= 1e-6 * stored["rel_mismatch"]
    # the replayed iterate moves by more than 1e-3 under sub-FP32 perturbations
    env = rec["envelope_eps_1e-6_to_1e-8"]
    assert env["rel_v"] > 1e-3 and env["rel_mismatch"] > 1e-3
    assert min(r["rel_mismatch"] for r in rec["runs"]) > 1e-3
    # an unperturbed replay is the reference bit for bit
    v0, em0 = mk.replay(o, shape, log, 0.0, 1)
    assert np.array_equal(v0, vref) and em0 == 0.0
