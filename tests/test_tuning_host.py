"""Host logic of the autotuner's table (no GPU): the text format that
shell_grid_create reads (csrc/tuning.cpp) round-trips through tune.py, short
lines of older tables take the defaults, the committed table holds only values
inside the kernels' ranges, and tune.py's model of the library's blocked
shapes keeps every candidate within the kernels' limits."""
import os

import pytest

from paper_1104_3408_amd import tune

HERE = os.path.dirname(os.path.abspath(__file__))
TABLE = os.path.join(os.path.dirname(HERE), "paper_1104_3408_amd", "tuning.txt")


def test_table_round_trip(tmp_path):
    entries = {(49, 48, 50, 0): dict(tune.DEFAULT, dr_rows=8, th_rows=3, dph_par=0, fuse=0),
               (17, 16, 50, 2): dict(tune.DEFAULT, filt_waves=4, th_plane=1, dph_mfma=1)}
    path = str(tmp_path / "t.txt")
    tune.write_table(path, entries)
    assert tune.read_table(path) == entries
    text = open(path).read().splitlines()
    assert text[0].startswith("# n_r n_theta n_fields precision " + " ".join(tune.FIELDS[:3]))


def test_short_lines_take_the_defaults(tmp_path):
    path = tmp_path / "old.txt"
    path.write_text("# an older table: ten columns\n33 32 50 0 9 4 8 8 8 8\n25 24 50 1 4 3 6 3 4 4 0\n")
    t = tune.read_table(str(path))
    assert t[(33, 32, 50, 0)] == dict(tune.DEFAULT, dr_rows=9, th_rows=4, dph_rows=8, ana_rows=8, syn_rows=8,
                                       filt_waves=8)
    assert t[(25, 24, 50, 1)]["dph_par"] == 0 and t[(25, 24, 50, 1)]["fuse"] == tune.DEFAULT["fuse"]


def test_committed_table_is_in_range():
    t = tune.read_table(TABLE)
    assert len(t) >= 15
    for (n_r, n_th, n_v, prec), v in t.items():
        assert n_v in (50, 58) and prec in (0, 1, 2)
        for f in ("dr_rows", "th_rows", "dph_rows", "ana_rows", "syn_rows"):
            assert 1 <= v[f] <= 20, (n_r, f)
        assert v["filt_waves"] in (4, 8, 16)
        assert v["dph_par"] in (-1, 0, 1)
        for f in ("th_plane", "fuse", "dph_mfma"):
            assert v[f] in (0, 1)
        if v["dph_mfma"]:
            assert (2 * n_th) % 16 == 0 and 2 * n_th <= 128


@pytest.mark.parametrize("n_out", [4, 9, 17, 24, 33, 49, 65, 80, 119, 128])
def test_blocked_shapes_stay_in_the_kernels_limits(n_out):
    for target in tune.ROW_TARGETS:
        sh = tune.blocked_shape(n_out, target)
        if sh is None:
            continue
        R, nw = sh
        assert 1 <= R <= 20 and nw in (8, 12, 16) and R * nw >= n_out
