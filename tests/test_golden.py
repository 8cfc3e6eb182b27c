"""Values the paper prints, kept as text fixtures under tests/golden/."""
import json
import os

import numpy as np

from paper_2609_38139_amd import codes

GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def test_code_params_printed_in_paper(orc):
    spec = json.load(open(os.path.join(GOLD, "code_params.json")))
    for name, want in spec.items():
        if name.startswith("_"):
            continue
        c = codes.by_name(name)
        assert c.n == want["n"]
        assert c.n - orc.gf2_rank(c.H) - orc.gf2_rank(c.G) == want["k"]
        assert set(np.diff(c.H.rowptr).tolist()) == {want["check_weight"]}
        assert set(np.bincount(c.H.col, minlength=c.n).tolist()) == {want["qubit_degree"]}


def test_table_s1_evidence_is_inverse_check_degree(orc):
    """Table S1's Evidence column is 1/d_c for each family, and the Evidence
    thresholds used by the decoder are the matching LLR bounds."""
    t = json.load(open(os.path.join(GOLD, "table_s1.json")))
    fam = {"2D TC": "toric2d:4", "3D TC point": "toric3d_point:3",
           "3D TC membrane": "toric3d_membrane:3", "BB": "bb:6x6"}
    thr = orc.evidence_thresholds(8)
    for k, name in fam.items():
        dc = int(np.diff(codes.by_name(name).H.rowptr)[0])
        assert abs(t[k]["Evidence"] - 1 / dc) < 1e-12
        assert abs(1 / (1 + np.exp(-float(thr[dc]))) - t[k]["Evidence"]) < 1e-7
        assert t[k]["CLAMP"] == 1000


def test_default_priors_follow_table_s1():
    from oracle import oracle as O
    t = json.load(open(os.path.join(GOLD, "table_s1.json")))
    assert O.DecodeParams().q == t["2D TC"]["q"]
    assert O.DecodeParams().clamp == t["2D TC"]["CLAMP"]
