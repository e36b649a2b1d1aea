"""Host-side pieces of the server (no GPU)."""
import numpy as np

from paper_2312_02999_amd.serve import latency_report, poisson_workload, Request


def test_poisson_workload_rate_and_sizes():
    off, names = poisson_workload(4000, 200.0, ["a", "b", "c", "d"], 10, seed=0)
    assert off[0] == 0 and np.all(np.diff(off) >= 0)
    rate = (len(off) - 1) / off[-1]
    assert abs(rate - 200.0) / 200.0 < 0.05
    counts = {k: names.count(k) for k in "abcd"}
    assert min(counts.values()) > 850


def test_latency_report_percentiles():
    reqs = []
    for k in range(100):
        r = Request("m", None, [None, None], arrival=float(k))
        r.finish = k + (k + 1) / 1000.0
        reqs.append(r)
    rep = latency_report(reqs)
    assert rep["frames"] == 200
    assert abs(rep["p50_ms"] - 50.5) < 1.0 and rep["p99_ms"] > 98.0
