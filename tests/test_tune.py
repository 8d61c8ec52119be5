"""Host logic of the autotuner: bucketing, per-instance tuning arrays, repacking."""
import numpy as np

from paper_2509_16370_amd import tune
from paper_2509_16370_amd import workloads as wl


def _batch():
    shapes = [(8, 2), (16, 4), (8, 2), (32, 8), (16, 4), (8, 2)]
    return [wl.make_instance(n, m, 5 + 3 * i, 1e-4, (80, i, 0)) for i, (n, m) in enumerate(shapes)]


def test_buckets_group_by_shape_in_batch_order():
    packed = wl.pack(_batch())
    bk = tune.buckets(packed)
    assert list(bk) == [(8, 2), (16, 4), (32, 8)]
    assert bk[(8, 2)].tolist() == [0, 2, 5]
    assert bk[(16, 4)].tolist() == [1, 4]
    assert bk[(32, 8)].tolist() == [3]


def test_plan_arrays():
    packed = wl.pack(_batch())
    plan = {(8, 2): tune.Choice("fp64"), (16, 4): tune.Choice("scan", 16), (32, 8): tune.Choice("mixed")}
    chunk, fp64 = tune.plan_arrays(packed, plan)
    assert fp64.tolist() == [1, 0, 1, 0, 0, 1]
    assert chunk.tolist() == [0, 16, 0, 0, 16, 0]


def test_subset_equals_packing_the_subset():
    insts = _batch()
    packed = wl.pack(insts)
    ids = np.array([4, 0, 3])
    sub = tune.subset(packed, ids)
    ref = wl.pack([insts[i] for i in ids])
    for k in ref.arrays:
        assert np.array_equal(sub.arrays[k], ref.arrays[k]), k
        assert np.array_equal(sub.offsets[k], ref.offsets[k]), k
    assert np.array_equal(sub.N, ref.N) and np.array_equal(sub.delta, ref.delta)


def test_candidates_skip_segment_lengths_beyond_the_horizon():
    c = tune.candidates(12, 4, 100, lengths=(16, 64, 128))
    assert [x.key() for x in c] == ["fp64", "mixed", "scan:16", "scan:64"]


def test_plan_round_trip(tmp_path):
    plan = {(8, 2): tune.Choice("scan", 32, 1.5), (16, 4): tune.Choice("fp64", 0, 2.0)}
    p = tmp_path / "plan.json"
    tune.save_plan(plan, str(p))
    back = tune.load_plan(str(p))
    assert back == plan


def test_plan_round_trip_keeps_the_schedule(tmp_path):
    plan = tune.Plan({(16, 4): tune.Choice("fp64", 0, 2.0)}, mw_waves=8)
    p = tmp_path / "plan.json"
    tune.save_plan(plan, str(p))
    back = tune.load_plan(str(p))
    assert back == plan and back.mw_waves == 8
