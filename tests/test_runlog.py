"""The Python layer's JSONL run log, on the CPU: one JSON object per line, numpy
values converted, nothing written while no path is set."""
import json

import numpy as np
import pytest


@pytest.fixture(scope="module")
def dfx():
    import paper_1707_03771_amd as m
    return m


def test_run_log_lines(dfx, tmp_path):
    path = tmp_path / "log.jsonl"
    dfx._log_run("dfx_scf", 3, 7, {"E": -1.5})  # no path set: nothing written
    dfx.set_run_log(path)
    try:
        dfx._log_run("dfx_scf", 3, 7, {"E": np.float64(-1.5), "niter": np.int32(4), "E_hist": [np.float64(-1.0), -1.5],
                                       "floor": np.array([1e-9, 0.0])})
        dfx._log_run("dfx_rhf_grad", 3, 7, {"max_abs_grad": 0.25})
    finally:
        dfx.set_run_log(None)
    dfx._log_run("dfx_scf", 3, 7, {"E": -2.0})
    rows = [json.loads(t) for t in path.read_text().splitlines()]
    assert len(rows) == 2
    assert rows[0]["entry"] == "dfx_scf" and rows[0]["E"] == -1.5 and rows[0]["niter"] == 4
    assert rows[0]["E_hist"] == [-1.0, -1.5] and rows[0]["floor"] == [1e-9, 0.0]
    assert rows[0]["natom"] == 3 and rows[0]["nbf"] == 7 and rows[0]["unix_time"] > 0
    assert rows[1]["entry"] == "dfx_rhf_grad"
