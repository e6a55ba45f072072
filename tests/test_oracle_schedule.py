"""The gradual p-coarsening schedule against the values printed in the paper."""
import os

from oracle.problems import gradual_schedule

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "pmg_schedule.txt")


def test_schedule_matches_figure_caption():
    rows = [l.split() for l in open(GOLDEN) if l.strip() and not l.startswith("#")]
    assert len(rows) == 8
    for r in rows:
        k = int(r[0])
        assert gradual_schedule(k) == [int(t) for t in r[1:]]
