"""The oracle's fixed constants against the values the paper prints."""
import json
import os

import numpy as np

from oracle import epll64 as o

G = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_constants.json")))


def test_schedule_and_sizes():
    assert o.P == G["P"]["value"] == G["patch_side"]["value"] ** 2
    np.testing.assert_array_equal(o.DEFAULT_B, G["beta_times_sigma2"]["value"])
    assert len(o.DEFAULT_B) == G["T"]["value"]
    for s in (5.0, 20.0, 60.0):
        np.testing.assert_allclose(o.default_betas(s) * s * s, G["beta_times_sigma2"]["value"],
                                   rtol=1e-15)


def test_table1_macro_arithmetic():
    # Table 1 prints its per-step times through a macro; the selection row is
    # 43.614 - 0.08 s and the total 45.694 s (shown rounded to 45.69 s)
    assert round(43.614 - 0.08, 2) == G["epllc_selection_seconds"]["value"]
    assert round(45.694, 2) == G["epllc_481x321_seconds"]["value"]
