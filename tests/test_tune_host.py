"""CPU checks of the autotuner's launch choices: every candidate's label
parses back to the same choice (the benchmark's --c4-choice and the recorded
profiling choice rely on it), and malformed labels are refused."""
import pytest

from paper_2006_01573_amd import tune


def test_every_candidate_label_round_trips():
    cands = tune._candidates(True, 3) + tune._candidates(False, 7)
    assert {c.path for c in cands} == {"region", "solo", "tile"}
    for c in cands:
        for extra in ({}, {"adj_waves": 1}, {"adj_waves": 8, "box": 4}):
            ch = tune.Choice(c.path, c.shape, c.waves, c.persistent, extra.get("box", c.box),
                             extra.get("adj_waves", c.adj_waves))
            assert tune.Choice.parse(ch.label()) == ch


def test_candidate_region_shapes_are_plan_shapes():
    # every shape the tuner tries is one the plan accepts; the smaller regions
    # (groups of 8 and 4 lanes) only on the solo kernel
    from paper_2006_01573_amd import ctis
    cands = tune._candidates(True, 3)
    assert {c.shape for c in cands if c.path == "solo"} == set(ctis.REGION_SHAPES[1:])
    assert {c.shape for c in cands if c.path == "region"} == {(16, 16), (32, 8), (8, 32)}


def test_candidates_respect_the_box_side():
    # more than 8 waves per workgroup only for B <= 5
    assert max(c.waves for c in tune._candidates(False, 5)) == 16
    assert max(c.waves for c in tune._candidates(False, 6)) == 8
    assert not any(c.path != "tile" for c in tune._candidates(False, 3))


@pytest.mark.parametrize("label", ["", "tile", "mesh 64x16 W4 adjoint W1 Bauto", "tile 64x16 4 adjoint W1 Bauto",
                                   "region 16x16 W2 adjoint Wx B3", "solo 16x16 W4 persistent adjoint"])
def test_malformed_labels_are_refused(label):
    with pytest.raises(ValueError):
        tune.Choice.parse(label)


@pytest.mark.parametrize("n", [1, 2, 3, 4])
def test_balanced_split_covers_every_frame_once(n):
    from paper_2006_01573_amd import workloads as W
    cfgs = W.batched_configs(64)
    cases = [W.make_case(4, frame=k, cfg=c) for k, c in enumerate(cfgs)]
    groups = tune.balanced_split(cases, n)
    assert len(groups) == n
    assert sorted(k for g in groups for k in g) == list(range(64))
    assert all(g == sorted(g) for g in groups)
    work = [c.geometry.a * c.geometry.alpha * int(c.lambda_ptr[-1]) for c in cases]
    loads = [sum(work[k] for k in g) for g in groups]
    # greedy heaviest-first: no group exceeds another by more than the heaviest frame
    assert max(loads) - min(loads) <= max(work)


def test_concurrent_arrangements_are_bounded():
    assert tune.MAX_CONCURRENT == 4
    with pytest.raises(ValueError):
        tune.TunedBatch([], [(None, [])] * 5, concurrent=True)
