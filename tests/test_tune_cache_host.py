"""The autotune cache file on the host (no GPU): opening parses the stored
results and skips lines that do not parse; a missing file is fine; NULL
closes; an empty path is rejected."""
import pytest

from paper_1703_06256_amd import hog


@pytest.fixture(autouse=True)
def _closed():
    yield
    hog.tune_cache_open(None)


def test_open_parses_results_and_skips_other_lines(tmp_path):
    p = tmp_path / "tiles.txt"
    p.write_text(
        "hogtune 00000000000000a1 2 24 1 0\n"
        "hogtune 00000000000000a2 3 0 4 1\n"
        "hogtune 00000000000000a1 6 12 1 0\n"       # the same key again: one entry
        "not a result\n"
        "hogtune zz 2 24 1 0\n"
        "hogtune 00000000000000a3 2 24\n"
        "hogtune 00000000000000a4 2 24 1 0 extra\n"
        "\n")
    hog.tune_cache_open(str(p))
    assert hog.tune_cache_stats() == (0, 0, 2)


def test_missing_file_is_an_empty_cache_and_none_closes(tmp_path):
    hog.tune_cache_open(str(tmp_path / "not_yet.txt"))
    assert hog.tune_cache_stats() == (0, 0, 0)
    assert not (tmp_path / "not_yet.txt").exists()  # written at the first result only
    hog.tune_cache_open(None)
    assert hog.tune_cache_stats() == (0, 0, 0)


def test_empty_path_is_rejected():
    with pytest.raises(hog.HogError) as e:
        hog.tune_cache_open("")
    assert e.value.status == hog.HOG_E_INVALID
