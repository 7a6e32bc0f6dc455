"""The committed autotuner cache (CPU only): it covers every transform of the
benchmark's batch in both modes, the fused-mode plans keep the default tiles,
and every entry is a valid pf_tune (radix orders 0..3, tiles >= 0)."""
import synth
from paper_1905_02803_amd import autotune


def test_cache_covers_the_benchmark_batch_in_both_modes():
    dims = synth.batch_sizes(4, 64)
    serial = autotune.tune_for(dims, mode="serial")
    fused = autotune.tune_for(dims, mode="fused")
    assert serial is not None and fused is not None
    assert len(serial) == len(fused) == len(dims)
    for (orders, tiles), (forders, ftiles) in zip(serial, fused):
        assert all(0 <= o <= 3 for o in orders + forders)
        assert all(t >= 0 for t in tiles)
        assert ftiles == (0, 0, 0)


def test_unknown_sizes_have_no_plans():
    assert autotune.tune_for([(7, 7, 7)]) is None
    assert autotune.tune_for([(7, 7, 7)], mode="fused") is None
