"""Host logic of the checkpointed adjoint's schedule (no GPU): how many of
the last steps the forward run records itself."""
import pytest

pytest.importorskip("torch")

from paper_2508_18202_amd.adjoint import stored_tail

GB = 1 << 30


def test_memory_sized_tail_is_whole_segments_within_the_fraction():
    # 0.388 GB per step (Smagorinsky records of 13 x 128x64x48), 270 GB free
    per_step = int(0.388 * GB)
    n = stored_tail(2000, 100, False, None, None, per_step, 270 * GB, 0.6)
    assert n % 100 == 0 and n * per_step <= 0.6 * 270 * GB < (n + 100) * per_step
    assert n == 400


def test_small_records_store_every_step():
    # 16-byte records of 13 x 128x64x48 cells: 2000 steps take 164 GB
    per_step = 16 * 13 * 128 * 64 * 48
    assert stored_tail(2000, 100, False, None, None, per_step, 280 * GB, 0.6) == 2000


def test_at_least_one_segment_even_without_memory():
    assert stored_tail(2000, 100, False, None, None, GB, 0, 0.6) == 100


def test_explicit_choices():
    assert stored_tail(2000, 100, False, True, None, GB, None) == 2000
    assert stored_tail(2000, 100, False, False, None, GB, None) == 100
    assert stored_tail(60, 100, False, False, None, GB, None) == 60
    assert stored_tail(2000, 100, False, None, 300, GB, None) == 300
    assert stored_tail(2000, 100, False, None, 2000, GB, None) == 2000
    assert stored_tail(2000, 100, True, None, None, GB, None) == 100


@pytest.mark.parametrize("bad", [50, 150, 0, 2100])
def test_stored_steps_must_be_whole_segments_or_the_run(bad):
    with pytest.raises(ValueError):
        stored_tail(2000, 100, False, None, bad, GB, None)


def test_store_all_refused_for_grouped_sweeps():
    with pytest.raises(ValueError):
        stored_tail(2000, 100, True, True, None, GB, None)
