"""The operation-count model of Tables I-III against the paper's printed claims."""
import json
import os

from paper_2512_16543_amd import opcount as complexity


def test_complexity_model_against_printed_claims(golden_dir):
    g = json.load(open(os.path.join(golden_dir, "paper_complexity.json")))
    K = g["fig1_K"]
    # Fig. 1 regimes: slightly cheaper at r = K/2, several times dearer at r = K
    assert 0.8 < complexity.normalized_complexity(K, 50) < 1.0
    assert complexity.normalized_complexity(K, 100) > 2.5
    assert complexity.normalized_complexity(K, 5) < 0.1
    # Table V: each printed saving lies between the model's values at two
    # consecutive integer ranks below K/2 (mean ranks are fractional)
    Kv = g["table_v_K"]
    grid = [complexity.savings(Kv, r) for r in range(0, Kv // 2 + 1)]
    for row in g["table_v"]:
        s = row["savings"]
        assert any(grid[r + 1] <= s <= grid[r] for r in range(len(grid) - 1))
    # monotone: more retained energy -> lower savings
    sv = [row["savings"] for row in g["table_v"]]
    assert sv == sorted(sv)
