"""Dice statistics of the paper's evaluation (Section 5.1, eqs. of D, D_a,
D_vw, D_ivw), pinned by hand-counted label maps."""
import numpy as np
import pytest

from paper_2209_08189_amd.metrics import dice


def test_dice_hand_counted():
    # label 1: |a| = 4, |b| = 2, overlap 2 -> D = 4/6; label 2: |a| = 2,
    # |b| = 4, overlap 1 -> D = 2/6; label 3 absent from both -> D = 1
    a = np.array([1, 1, 1, 1, 2, 2, 0, 0])
    b = np.array([1, 1, 0, 2, 2, 0, 2, 2])
    d = dice(a, b, labels=(1, 2))
    assert d["D"] == pytest.approx([4 / 6, 2 / 6])
    assert d["D_a"] == pytest.approx(0.5)
    # volumes |b^1| = 2, |b^2| = 4
    assert d["D_vw"] == pytest.approx((2 * 4 / 6 + 4 * 2 / 6) / 6)
    assert d["D_ivw"] == pytest.approx((4 / 6 / 2 + 2 / 6 / 4) / (1 / 2 + 1 / 4))


def test_dice_identity_and_disjoint():
    r = np.random.default_rng(0).integers(0, 4, size=(8, 8, 8))
    d = dice(r, r)
    assert d["D"] == [1.0, 1.0, 1.0] and d["D_a"] == d["D_vw"] == d["D_ivw"] == 1.0
    a = np.zeros(10, dtype=int)
    a[:5] = 1
    b = np.zeros(10, dtype=int)
    b[5:] = 1
    assert dice(a, b, labels=(1,))["D"] == [0.0]
