"""The paper's test cases as the benchmark runs them, against the values the
paper prints (Sec. 3, Table 1; fixture tests/golden/table1_simulations.json):
domain, cells, T, coarse and fine steps, Re, the number of cubes of the
second case, and the lid velocity of 1 that both grids start with."""
import json
import os

import numpy as np

from paper_1705_06149_amd import inputs

HERE = os.path.dirname(os.path.abspath(__file__))


def _golden():
    with open(os.path.join(HERE, "golden", "table1_simulations.json")) as fh:
        return json.load(fh)


def test_bench_sim_configs_match_table1():
    import bench
    gold = _golden()
    for sim in (1, 2):
        g = gold["sim%d" % sim]
        c = bench.paper_sim_config(sim)
        assert c["domain"] == g["domain"]
        assert c["cells"] == g["cells"]
        assert c["T"] == g["T"] and c["re"] == g["re"]
        assert c["coarse_dt"] == g["coarse_dt"] and c["fine_dt"] == g["fine_dt"]
        assert c["obstacles"] == g.get("obstacles", 0)
        # the slice lengths of the paper's time-slice counts are whole numbers of coarse steps
        for n in g["time_slices"]:
            ratio = g["T"] / n / g["coarse_dt"]
            assert abs(ratio - round(ratio)) < 1e-9


def test_sim2_cubes_and_lid(oracle):
    gold = _golden()
    n = gold["sim2"]["cells"][0]
    solid = inputs.median_plane_cubes(n, seed=49, count=gold["sim2"]["obstacles"])
    assert solid.shape == (n, n, n) and 0 < solid.mean() < 0.1
    # cubes sit around the median plane
    rows = np.nonzero(solid.any(axis=(0, 2)))[0]
    assert rows.min() >= n // 2 - 3 and rows.max() <= n // 2 + 3
    g = oracle.Grid(n, n, n, periodic_z=True, solid=solid)
    assert np.all(g.lid == gold["sim1"]["lid"])
