"""The learned access-path chooser judged on recorded timings (no GPU):
held-out workloads of the chooser's distribution, every available arm timed
on an MI355X (paper_2403_15807_amd/chooser_heldout.npz, written by
``python -m paper_2403_15807_amd.chooser --phase heldout``).  The learned
pick is the library's own host inference (vrs_chooser_pick) with the shipped
weights, so the regret figures are deterministic; they must beat the
selectivity-threshold heuristic's and equal the committed report."""

import json
import os

import numpy as np
import pytest

from paper_2403_15807_amd import chooser as CH
from paper_2403_15807_amd import vrs

pytestmark = pytest.mark.skipif(not os.path.exists(CH.HELDOUT), reason="no recorded held-out timings")


def test_learned_regret_beats_the_heuristic_on_recorded_timings():
    params, mean, std = CH.load_weights(CH.WEIGHTS)
    H = np.load(CH.HELDOUT)
    rows = CH.evaluate_recorded(H["F"], H["Y"], params, mean, std)
    reg = CH.summarize(rows)
    assert reg["learned"]["n"] >= 1900
    assert reg["learned"]["mean_regret"] < reg["heuristic"]["mean_regret"]
    assert reg["learned"]["median_regret"] <= reg["heuristic"]["median_regret"]
    assert reg["learned"]["frac_best"] > reg["heuristic"]["frac_best"]
    rep = json.load(open(CH.REPORT))
    for name in ("learned", "heuristic"):
        for key in ("mean_regret", "p95_regret", "frac_best", "n"):
            assert np.isclose(rep["regret"][name][key], reg[name][key], rtol=1e-9, atol=0), (name, key)


def test_allowed_arms_follow_the_planner_rules():
    H = np.load(CH.HELDOUT)
    nt = H["Y"].shape[1] // 2
    for f, y in zip(H["F"][:200], H["Y"][:200]):
        al = CH.allowed_arms(f, y, nt)
        assert not (al & ~np.isfinite(y)).any()           # only available arms
        if np.exp(f[3]) >= 0.9:
            assert not al[nt:].any()                      # no gather at the dense end
        a = CH.heuristic_arm(f, y, nt)
        assert np.isfinite(y[a])
