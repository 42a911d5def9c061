"""Host-side logic of the autotuner (no GPU)."""
import sys
import types

from paper_2106_12802_amd import autotune


def test_choose_median_and_ties():
    t = [((1, 1), [5.0, 1.0, 9.0]), ((2, 2), [4.0, 4.0, 4.0]), ((3, 3), [4.0, 3.0, 100.0])]
    (cand, med) = autotune.choose(t)
    assert cand == (2, 2) and med == 4.0  # medians 5, 4, 4: first of the tie
    assert autotune.choose([((7, 7), [2.0])]) == ((7, 7), 2.0)


def test_grid_then_secondary_knobs(monkeypatch, tmp_path):
    """The primary grid picks the fastest launch shape, then each secondary knob is
    searched with the others held; the result is applied and cached."""
    state = {"chunk_paths": 1 << 23, "trace_blocks": 8192, "schedule": 0, "bvh_leaf_max": 3,
             "streams": 3, "tail_bounce": 3, "bvh_builder": 1, "conv_small_tiles": 128,
             "queue_sort": 1, "bvh_quantized": 0, "wave_extend": 0, "wave_shadow": 0,
             "net_fused_blocks": 1}
    monkeypatch.setattr(autotune.T, "get_tuning", lambda: dict(state))
    monkeypatch.setattr(autotune.T, "set_tuning", lambda **kw: state.update(kw))
    monkeypatch.setattr(autotune, "_device_key", lambda: "fake")
    fake_torch = types.SimpleNamespace(cuda=types.SimpleNamespace(synchronize=lambda: None))
    monkeypatch.setitem(sys.modules, "torch", fake_torch)
    clock = [0.0]
    monkeypatch.setattr(autotune.time, "perf_counter", lambda: clock[0])

    def workload():  # a cost model: best at 2^24 paths, 4096 blocks, 2 streams, tail 4
        s = state
        clock[0] += (abs(s["chunk_paths"] - (1 << 24)) / (1 << 20) + abs(s["trace_blocks"] - 4096)
                     / 1024 + abs(s["streams"] - 2) + abs(s["tail_bounce"] - 4) + s["schedule"]
                     + 1.0) * 1e-3
    path = str(tmp_path / "cache.json")
    res = autotune.tune(workload, "w", cache_path=path, reps=1)
    assert (res["chunk_paths"], res["trace_blocks"], res["schedule"]) == (1 << 24, 4096, 0)
    assert res["streams"] == 2 and res["tail_bounce"] == 4 and not res["cached"]
    assert state["streams"] == 2 and state["chunk_paths"] == 1 << 24
    state.update(streams=3, chunk_paths=1 << 23)
    again = autotune.tune(workload, "w", cache_path=path, reps=1)
    assert again["cached"] and state["streams"] == 2 and state["chunk_paths"] == 1 << 24
