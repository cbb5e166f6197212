"""Host-side checks of bench.py's measurement plumbing (no GPU needed)."""
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def test_traffic_counters_match_the_filter_sources():
    """The headline line's `traffic` comes from the committed FETCH_SIZE /
    WRITE_SIZE summary, which records a hash of the filter's sources; the
    counters must have been taken on the sources as they are now."""
    import bench
    t = bench.measured_traffic()
    assert t is not None, "the counter summary predates the current filter sources"
    # at least the records once per XCD L2, theta once and the outputs
    assert 27e6 < t < 100e6


def test_more_than_one_gpu_is_refused(monkeypatch, capsys):
    import bench
    import pytest
    monkeypatch.setattr(sys, "argv", ["bench.py", "--gpus", "2"])
    with pytest.raises(SystemExit) as e:
        bench.main()
    assert e.value.code == 2
    assert "one GPU" in capsys.readouterr().err
