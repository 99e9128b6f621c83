"""The diagnostics trace (Solver.run): one JSON line per `every` steps with the
float64 diagnostics of pflbm_volume, on the 2-D static droplet."""
import json

import pytest

from paper_2511_11360_amd import workloads as wl

pytestmark = pytest.mark.gpu


def test_run_writes_one_json_line_per_interval(tmp_path):
    from paper_2511_11360_amd.solver import Solver
    d, phi, u = wl.static_droplet_2d(n=64, R=16.0)
    s = Solver(d, precision="fp64")
    s.init(phi, u)
    log = tmp_path / "diag.jsonl"
    s.run(23, 5, str(log), centre=(32.0, 32.0), R=16.0)
    recs = [json.loads(line) for line in log.read_text().splitlines()]
    assert [r["step"] for r in recs] == [0, 5, 10, 15, 20, 23]
    assert set(recs[0]) == {"step", "V_phi", "V_count", "sum_phi", "phi_min", "phi_max", "umax", "dp"}
    # the conservative AC model keeps sum phi to rounding
    for r in recs:
        assert abs(r["sum_phi"] - recs[0]["sum_phi"]) <= 1e-12 * recs[0]["sum_phi"]
    v = s.volume((32.0, 32.0), 16.0)
    assert recs[-1]["dp"] == v["p_in"] - v["p_out"] and recs[-1]["umax"] == v["umax"]
    # appending to an open file, no centre: no dp
    with open(log, "a") as f:
        s.run(4, 0, f)
    recs = [json.loads(line) for line in log.read_text().splitlines()]
    assert [r["step"] for r in recs[-2:]] == [23, 27] and "dp" not in recs[-1]
