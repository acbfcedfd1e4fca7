"""Host-side checkpoint logic of the full-map driver (no GPU needed)."""
import pytest

from paper_2008_05612_amd import fullmap


def test_checkpoint_is_tied_to_its_run(tmp_path):
    path = str(tmp_path / "ck.json")
    dims = (3, 3, 3)
    g = "sequences"
    fullmap._save_checkpoint(path, dims, 2, 30, False, None, g, 5, [1, 2, 3], 7)
    ck = fullmap._load_checkpoint(path, dims, 2, 30, 3, False, None, g)
    assert ck["next_block"] == 5 and ck["designability"] == [1, 2, 3] and ck["nondesign"] == 7
    # another energy table, form, block size, class count, symmetry or block
    # geometry is another run
    with pytest.raises(ValueError):
        fullmap._load_checkpoint(path, dims, 2, 30, 3, False, (0, -10, -10, -23), g)
    with pytest.raises(ValueError):
        fullmap._load_checkpoint(path, dims, 1, 30, 3, False, None, g)
    with pytest.raises(ValueError):
        fullmap._load_checkpoint(path, dims, 2, 28, 3, False, None, g)
    with pytest.raises(ValueError):
        fullmap._load_checkpoint(path, dims, 2, 30, 4, False, None, g)
    with pytest.raises(ValueError):
        fullmap._load_checkpoint(path, dims, 2, 30, 3, True, None, g)
    with pytest.raises(ValueError):
        fullmap._load_checkpoint(path, dims, 2, 30, 3, False, None, "wide")
    t = (0, -10, -10, -23)
    fullmap._save_checkpoint(path, dims, 2, 30, False, t, g, 1, [0, 0, 0], 0)
    assert fullmap._load_checkpoint(path, dims, 2, 30, 3, False, t, g)["next_block"] == 1
    with pytest.raises(ValueError):
        fullmap._load_checkpoint(path, dims, 2, 30, 3, False, None, g)
    assert fullmap._load_checkpoint(str(tmp_path / "none.json"), dims, 2, 30, 3, False, t,
                                    g) is None


def test_lattice_parsing():
    assert fullmap._parse_lattice("6x6") == (6, 6, 1)
    assert fullmap._parse_lattice("3x3x3") == (3, 3, 3)
