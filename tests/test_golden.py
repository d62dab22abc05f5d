"""The oracle still reproduces its stored regression summary (tests/golden)."""
import json
import os

from tests.golden.make_golden import summary

HERE = os.path.dirname(os.path.abspath(__file__))


def test_config0_oracle_summary_unchanged():
    with open(os.path.join(HERE, "golden", "config0_oracle.json")) as f:
        ref = json.load(f)
    got = summary()
    assert got["stats"] == ref["stats"]
    for key in ("image_sum", "image_l2", "image_max"):
        assert abs(got[key] - ref[key]) <= 1e-12 * max(1.0, abs(ref[key]))
    for (q, p, v), (q2, p2, v2) in zip(got["source_pixels"], ref["source_pixels"]):
        assert (q, p) == (q2, p2) and abs(v - v2) <= 1e-12
