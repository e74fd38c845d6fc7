"""Host logic of the Algorithm 1 loop: the densification schedule of the 3DGS
pipeline the paper keeps (Sec. 5.1: every 100 steps from step 500) and the
accumulation window that feeds each densification."""
from paper_2505_05587_amd.train import Schedule


def test_default_schedule_matches_the_paper():
    s = Schedule()
    steps = [t for t in range(1, 2001) if s.is_densify(t)]
    assert steps[:4] == [500, 600, 700, 800]
    assert all(b - a == 100 for a, b in zip(steps, steps[1:]))
    assert not s.is_densify(15_100) and s.is_densify(15_000)
    # the first window holds the T_split gradient steps before step 500
    assert s.accumulate_from() == 401
    assert sum(1 for t in range(s.accumulate_from(), 500) if not s.is_densify(t)) == 99


def test_custom_schedule_window():
    s = Schedule(densify_from=8, densify_every=4, densify_until=8)
    assert [t for t in range(1, 30) if s.is_densify(t)] == [8]
    assert s.accumulate_from() == 5
