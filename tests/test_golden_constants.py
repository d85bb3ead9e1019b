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


def test_tree_levels_are_the_papers():
    # the offline tree builder collapses K = 200 level by level to the sizes
    # Sec. 3.2 prints
    from paper_1710_08124_amd import tree as btree
    assert [G["K_paper"]["value"]] + list(btree.LEVELS_K200) == G["tree_levels"]["value"]
