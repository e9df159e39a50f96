"""The oracle's parameter search and continuation (Section 3.4) checked
against the rules the paper states, on a 32^3 closed-form pair.  CPU only.

The rules: (i) beta_w = beta_w_max; beta_v starts at beta_v_max and drops
one decade per valid trial; after the first breach of [J_min, 1/J_min] each
trial bisects the last valid and the last breaching beta_v, until the next
midpoint would move beta_v by less than 10 % of the valid value; (ii) at
beta_v*, beta_w drops one decade per valid trial.  The context ends at the
last valid trial's solution.  The trial sequence on general images is
"parity unpinned" beyond these rules."""
import numpy as np
import pytest

from paper_2209_08189_amd import synth


def _pair(orc, n=32):
    shape = (n,) * 3
    m0 = synth.trig_template(shape).astype(np.float32).astype(np.float64)
    vs = synth.trig_velocity(shape, 0.5).astype(np.float32).astype(np.float64)
    o = orc.Oracle(shape, nt=4, beta=5e-4)
    o.set_images(m0, m0)
    o.set_velocity(vs)
    o.state()
    return shape, m0, o.field(orc.FIELD_STATE, 4).astype(np.float32).astype(np.float64)


@pytest.mark.parametrize("jmin", [0.69, 0.73])
def test_search_follows_the_stated_rules(orc, jmin):
    shape, m0, m1 = _pair(orc)
    o = orc.Oracle(shape, nt=4, beta=1.0)
    o.set_images(m0, m1)
    o.set_velocity(np.zeros((3,) + shape))
    st, bv_star, bw_star, log = o.param_search(jmin=jmin, max_outer=10, max_pcg=10)
    assert st == 0
    valid = log[:, 4] == 1
    # every valid flag is the bounds test of its row
    assert np.array_equal(valid, (log[:, 2] >= jmin) & (log[:, 3] <= 1 / jmin))
    stage1 = log[:, 1] == 1e-5
    rows1 = log[stage1]
    assert rows1[0, 0] == 1.0
    good, bad = None, None
    for k, r in enumerate(rows1):
        if k > 0:
            if bad is None:
                assert r[0] == rows1[k - 1, 0] / 10.0          # decade step
            else:
                assert r[0] == 0.5 * (good + bad)                # bisection midpoint
        if r[4]:
            good = r[0]
        else:
            bad = r[0]
    assert bad is not None and good == bv_star
    # the bisection stopped exactly when the next midpoint is within 10 %
    assert good - 0.5 * (good + bad) < 0.1 * good
    # stage (ii): decades at beta_v*, ending at a breach or at beta_w_min
    rows2 = log[~stage1]
    assert np.all(rows2[:, 0] == bv_star)
    assert np.allclose(rows2[:, 1], 1e-5 / 10.0 ** np.arange(1, len(rows2) + 1), rtol=1e-12)
    assert np.all(rows2[:-1, 4] == 1)
    last_valid = log[valid][-1]
    assert last_valid[0] == bv_star and last_valid[1] == bw_star
    # the context ends at the last valid solution (restored after a breach)
    J = o.jacobian_det()
    assert J.min() == last_valid[2] and J.max() == last_valid[3]
    assert (o.beta, o.beta_w) == (bv_star, bw_star)


def test_continuation_sequence(orc):
    """Continuation toward (0.015625, 1e-7): beta_v = 1, 0.1 (= 10^ceil(log10
    beta_v*)), then beta_v*; then beta_w = 1e-6, 1e-7 at beta_v*."""
    shape, m0, m1 = _pair(orc)
    o = orc.Oracle(shape, nt=4, beta=1.0)
    o.set_images(m0, m1)
    o.set_velocity(np.zeros((3,) + shape))
    log = o.param_continuation(0.015625, 1e-7, max_outer=10, max_pcg=10)
    seq = [(r[0], r[1]) for r in log]
    assert seq[0] == (1.0, 1e-5) and seq[1] == (0.1, 1e-5) and seq[2] == (0.015625, 1e-5)
    assert seq[3][0] == 0.015625 and abs(seq[3][1] - 1e-6) < 1e-18
    assert seq[4][0] == 0.015625 and abs(seq[4][1] - 1e-7) < 1e-18
    assert len(seq) == 5
    assert np.all(np.diff(log[:, 8]) <= 0)     # mismatch does not rise along the path


def test_search_reports_bounds_when_the_first_trial_breaches(orc):
    """J_min = 0.999 cannot hold even at beta_v = 1: one trial, status 3
    (bounds), beta_v* = beta_v_max, no beta_w stage."""
    shape, m0, m1 = _pair(orc)
    o = orc.Oracle(shape, nt=4, beta=1.0)
    o.set_images(m0, m1)
    o.set_velocity(np.zeros((3,) + shape))
    st, bv, bw, log = o.param_search(jmin=0.999, max_outer=10, max_pcg=10)
    assert st == 3 and bv == 1.0 and bw == 1e-5
    assert len(log) == 1 and log[0, 4] == 0
