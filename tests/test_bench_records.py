"""The bench's JSONL run records (bench.run_records / write_records), on a
synthetic result line: one record per measured path, each a JSON object per
line with the configuration, dtype, timing and errors; the batch's records
carry per-cell errors beside the stored oracle's ranks and cond(S^m)."""

import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_run_records_one_line_per_path(tmp_path):
    gold = bench.load_json("config4.json")
    n = len(gold["cells"]) if gold else 0
    out = {"batched": {"mixed": {"seconds": 0.5, "builds_per_s": 48.0, "max_dEx_vs_oracle": 3e-6,
                                 "max_dK_vs_oracle": 1e-7, "cells_meeting_gate": n},
                       "f64": {"seconds": 0.6, "builds_per_s": 40.0}},
           "batched_per_cell": {"mixed": {"dEx": [1e-6] * n, "dK": [2e-8] * n}},
           "config": {"prec": "mixed"}, "phases_ms_batch_mixed": {"solve": 160.0},
           "phase_rates_batch_mixed": {}, "roofline": {"frac": 0.53},
           "paths": {"rings-k2": {"paths": {"f64": {"ms_per_build": 35.0, "Ex": -37.75,
                                                    "precision": "f64", "dEx_vs_oracle": 1e-14,
                                                    "maxdK_vs_oracle": 1e-13},
                                            "f64-gradient": {"ms_per_call": 160.0, "Ex": -37.75,
                                                             "precision": "f64"}}}}}
    recs = bench.run_records(out, "batch24", gold)
    path = tmp_path / "runs.jsonl"
    bench.write_records(str(path), recs)
    bench.write_records(str(path), recs)  # appends
    lines = path.read_text().splitlines()
    assert len(lines) == 2 * len(recs) == 8
    parsed = [json.loads(x) for x in lines]
    assert [r["path"] for r in parsed[:4]] == ["batched-mixed", "batched-f64", "f64", "f64-gradient"]
    mixed = parsed[0]
    assert mixed["dtype"] == "mixed" and mixed["roofline"]["frac"] == 0.53
    if gold:
        assert len(mixed["cells"]) == n
        assert mixed["cells"][0]["rank"] == gold["cells"][0]["rank"]
        assert mixed["cells"][0]["cond_S_max"] == max(gold["cells"][0]["cond_S"])
    assert parsed[3]["ms"] == 160.0 and parsed[2]["dEx"] == 1e-14
