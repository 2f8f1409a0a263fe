"""The experiment runners end to end on the GPU at tiny model times: the
reference channel and the planetary slice advance, report a finite imbalance
and conserve mass, the convergence study returns finite level differences
that shrink under refinement, and the benchmark hill advances."""
import io
import json

import numpy as np
import pytest

from paper_2605_29598_amd import experiments as X
from paper_2605_29598_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("kind", ["reference", "planetary"])
def test_runner_short_run(kind):
    buf = io.StringIO()
    hours = 0.01 if kind == "reference" else 0.05
    summary, series = X.run(kind, hours, hours / 2, W.R2, "fp64", out=buf)
    assert summary["steps"] == int(round(hours * 3600 / (0.5 if kind == "reference" else 10.0)))
    assert len(series) == 3 and all(np.isfinite(r["egeo"]) for r in series)
    assert series[0]["egeo"] < 1e-13 < series[-1]["egeo"]
    assert abs(series[-1]["mass_rel"]) < 1e-13
    lines = [json.loads(l) for l in buf.getvalue().splitlines()]
    assert "summary" in lines[-1]


def test_convergence_study_shrinks():
    buf = io.StringIO()
    rows = X.convergence(hours=1.0 / 120, levels=3, scheme=W.R2, nsx=300, nsz=20, out=buf)
    assert len(rows) == 2
    for k in ("l2_w", "l2_p"):
        assert 0 < rows[1][k] < rows[0][k], (k, rows)


@pytest.mark.parametrize("rotating", [False, True])
def test_hill_runner_short_run(rotating):
    """The Sec. 4.3 benchmark hill (lateral and top sponges, bell mountain)
    advances five steps: mass conserved, vertical motion over the hill, one
    summary line."""
    buf = io.StringIO()
    summary = X.run_hill(rotating, 5 * 8.0 / 3600.0, 2 * 8.0 / 3600.0, W.R2, out=buf)
    assert summary["steps"] == 5
    fin = summary["final"]
    assert abs(fin["mass_rel"]) < 1e-13
    assert 0 < fin["max_abs_w"] < 10 and all(np.isfinite(fin["u_minus_U_z800"]))
    lines = [json.loads(l) for l in buf.getvalue().splitlines()]
    assert len(lines) == 4 and "summary" in lines[-1]


def test_hill_nonconforming_runner_short_run():
    """The non-conforming benchmark mesh (terrain-following, two levels of
    hanging faces, lateral and top sponges) advances five steps with mass
    conserved."""
    buf = io.StringIO()
    summary = X.run_hill(False, 5 * 4.0 / 3600.0, 5 * 4.0 / 3600.0, W.R2, out=buf, nonconforming=True)
    assert summary["steps"] == 5
    assert abs(summary["final"]["mass_rel"]) < 1e-13 and 0 < summary["final"]["max_abs_w"] < 10


def test_hill_large_runner_short_run():
    """The larger-scale hill (isothermal background, 60 km lateral layers) on a
    reduced 10^3-element mesh advances five steps with mass conserved."""
    buf = io.StringIO()
    w = W.hill_large(nx=10, ny=10, nz=10)
    summary = X.run_hill(True, 5 * 4.0 / 3600.0, 5 * 4.0 / 3600.0, W.R2, out=buf, workload=w)
    assert summary["steps"] == 5
    assert abs(summary["final"]["mass_rel"]) < 1e-13 and 0 < summary["final"]["max_abs_w"] < 10


def test_column_runner_short_run():
    """The resting-column runner advances a few steps and reports the largest
    vertical velocity and its height (small: the initial imbalance only)."""
    buf = io.StringIO()
    rows = X.run_column(8.0, 5 * 8.0 / 3600.0, 2 * 8.0 / 3600.0, out=buf)
    assert [round(r["t_s"]) for r in rows] == [16, 32, 40]
    for r in rows:
        assert 0 < r["max_abs_w"] < 1e-3 and 0 < r["z_of_max"] < 16e3
    assert len(buf.getvalue().splitlines()) == 3
