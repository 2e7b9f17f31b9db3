"""The oracle's defaults carry the constants the paper states."""
import json
import os

import oracle as O

HERE = os.path.dirname(os.path.abspath(__file__))


def test_defaults_match_paper_constants():
    c = json.load(open(os.path.join(HERE, "golden", "paper_constants.json")))
    p = O.Params()
    assert p.lam == c["smooth_min_lambda"]["value"]
    # raw-point cells 0.4 m with l = 0.2 m; voxel mode 0.1 m voxels, l = 0.2 m
    lo, hi = c["length_scale_in_voxels"]["value"]
    assert lo * 0.1 <= 0.2 <= hi * 0.1
    # leaf of 8 voxels per axis: a voxel-mode cluster spans 8 voxel edges
    m = O.Model(O.Params(voxel=0.1), [[0.05, 0.05, 0.05], [0.75, 0.75, 0.75],
                                      [0.85, 0.05, 0.05]])
    assert m.nclusters == 2 and c["leaf_voxels_per_axis"]["value"] == 8
    # one training point far from everything: o = k(0)/(1 + s^2) with k(0) = 1
    r = O.Model(O.Params(cell=10.0), [[1.0, 1.0, 1.0]]).query([[1.0, 1.0, 1.0]])
    assert abs(r["aux"][0, 0] - c["prior_variance_k_xx"]["value"] / (1 + 0.01 ** 2)) < 1e-15
