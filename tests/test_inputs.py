"""Seeded workload generators (host only)."""
from mrs_inputs import scenes as S


def test_batch_specs_ranges_and_determinism():
    a = S.batch_specs(500, 32)
    assert a == S.batch_specs(500, 32) and len(a) == 32
    assert len({x[0] for x in a}) == 32
    for seed, tris, W, H, sh, sl in a:
        assert 10_000 <= tris <= 1_000_000
        assert 256 <= W <= 1920 and 256 <= H <= 1080 and W % 8 == 0 and H % 8 == 0
        assert 1 <= sh <= 8 and 16 <= sl <= 128
    # uneven: sizes and budgets spread over their ranges
    assert max(x[1] for x in a) > 10 * min(x[1] for x in a)
    assert max(x[2] * x[3] for x in a) > 4 * min(x[2] * x[3] for x in a)


def test_procedural_sized_tracks_budget():
    for n in (10_000, 60_000):
        sc = S.procedural_sized(9, n)
        assert 0.7 * n <= sc.num_tris <= 1.05 * n
