"""The autotuner's cache file (host side, no GPU): entries load, save back unchanged,
count, clear; malformed lines and invalid tunings are refused without adding anything."""
import pytest


@pytest.fixture()
def gp():
    from paper_1403_0802_amd import gp as gpmod
    gpmod.gp_tuning_cache_clear()
    yield gpmod
    gpmod.gp_tuning_cache_clear()


GOOD = ("p2p mixed gfx950 rec=1 seg=0 cls=0 n=23 tpp=12 ppi=9\t4 128 32 1 1 -1\n"
        "pip mixed gfx950 rec=1 seg=0 cls=0 n=25 tpp=9 ppi=6\t2 128 16 0 1 16\n")


def test_load_save_roundtrip(gp, tmp_path):
    src = tmp_path / "cache.txt"
    src.write_text(GOOD)
    gp.gp_tuning_cache_load(str(src))
    assert gp.gp_tuning_cache_size() == 2
    out = tmp_path / "out.txt"
    gp.gp_tuning_cache_save(str(out))
    assert sorted(out.read_text().splitlines()) == sorted(GOOD.splitlines())
    # loading again replaces equal keys
    gp.gp_tuning_cache_load(str(out))
    assert gp.gp_tuning_cache_size() == 2
    gp.gp_tuning_cache_clear()
    assert gp.gp_tuning_cache_size() == 0


@pytest.mark.parametrize("bad", [
    "pip mixed gfx950 n=1\t2 128 16 0\n",             # too few fields
    "pip mixed gfx950 n=1 2 128 16 0 1 16\n",         # no tab
    "pip mixed gfx950 n=1\t3 128 16 0 1 16\n",        # points per lane 3
    "pip mixed gfx950 n=1\t2 100 16 0 1 16\n",        # chunk not a multiple of 64
    "pip mixed gfx950 n=1\t2 128 16 0 2 16\n",        # PIP with two waves per item
    "xyz mixed gfx950 n=1\t2 128 16 0 1 16\n",        # unknown operation
    "pip mixed gfx950 n=1\t2 128 16 0 1 16 7\n",      # trailing field
])
def test_bad_lines_are_refused(gp, tmp_path, bad):
    src = tmp_path / "cache.txt"
    src.write_text(GOOD + bad)
    with pytest.raises(gp.GPError) as e:
        gp.gp_tuning_cache_load(str(src))
    assert e.value.status == gp.GP_E_INVALID_ARG
    assert gp.gp_tuning_cache_size() == 0


def test_missing_file(gp, tmp_path):
    with pytest.raises(gp.GPError):
        gp.gp_tuning_cache_load(str(tmp_path / "nope.txt"))
