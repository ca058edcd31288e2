"""Host-side grid-selection rule against the paper's Table 2 (Section 4.3)."""
import json
import math
import os

import pytest

from paper_2105_04006_amd import grid

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def test_table2_practical_nf():
    with open(os.path.join(GOLDEN, "table2_grid.json")) as fh:
        g = json.load(fh)
    for row in g["rows"]:
        assert grid.n_freq(row["f_min"], row["f_max"], row["df"]) == row["n_f"]
        # the window these spacings imply is about 120 days
        t_max = 0.2 * math.pi / row["df"]
        assert t_max == pytest.approx(120.0, rel=1e-3)
        assert grid.spacing_from_window(t_max, grid.ANGULAR) == pytest.approx(row["df"], rel=1e-12)


def test_cycles_spacing_is_tenfold_oversampling():
    assert grid.spacing_from_window(3650.0, grid.CYCLES) == pytest.approx(0.1 / 3650.0)
    assert grid.spacing_from_window(3650.0, grid.ANGULAR) == pytest.approx(
        2.0 * math.pi * grid.spacing_from_window(3650.0, grid.CYCLES))


def test_rejects_bad_arguments():
    with pytest.raises(ValueError):
        grid.spacing_from_window(0.0)
    with pytest.raises(ValueError):
        grid.n_freq(2.0, 1.0, 0.1)
