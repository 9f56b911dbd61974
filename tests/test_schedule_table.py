"""The committed schedule table (paper_1208_6387_amd/schedules.json, written on the GPU by
python -m paper_1208_6387_amd.tune): every entry names a valid schedule, the one installed is the
fastest of its own measurements, and its key is the signature of the workload it was tuned on."""
import numpy as np
import pytest

import workloads as W
from paper_1208_6387_amd import tune

TABLE = tune.load_table()


def test_table_present_and_valid():
    assert TABLE, "no tuned schedules committed"
    for key, rec in TABLE.items():
        form, m, pats = key.split("|")
        assert form in tune.FORMS and m.startswith("m=") and int(m[2:]) >= 1
        assert rec["tile"] in (0, 64, 128, 256) and rec["work"] >= 1
        meas = rec["measured_ms"]
        assert len(meas) >= 11 and all(x["ms"] > 0 for x in meas)
        best = min(meas, key=lambda x: x["ms"])
        assert (best["tile"], best["work"]) == (rec["tile"], rec["work"]), key
        assert any(x["tile"] == 0 for x in meas), "the size rule is always a candidate"
        if rec["tile"] == 256:
            assert ";" not in pats, "the 256 tile is for single-pattern structures"


@pytest.mark.parametrize("cfg", [1, 2, 3, 4])
def test_keys_match_workload_signatures(cfg):
    p = W.config(cfg)
    n_occ = list(np.bincount(p.occ_pattern, minlength=len(p.patterns)))
    n_b = [pat.n_b for pat in p.patterns]
    keys = [tune.signature(n_b, n_occ, m, f) for f in ("fp64", "bf16x3")
            for m in sorted({p.n_rhs * p.n_perm, p.n_rhs})]
    found = [k for k in keys if k in TABLE]
    assert found, (p.name, keys)
