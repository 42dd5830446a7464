"""GPU: the continuous-batching server returns, for every request, exactly
the result the same request gets alone on the single-run path (bitwise, in
both precisions), while requests arrive, overlap on the device, finish and
free their memory under a budget small enough to make later ones wait."""
import numpy as np
import pytest

from paper_2209_01983_amd import sale, workloads
from paper_2209_01983_amd.inputs import serve_trace

from parity import FIELDS, say  # noqa: E402

pytestmark = pytest.mark.gpu


def small_trace():
    tr = serve_trace(14, seed=7, rate=1e4, edge=(6, 28), steps=(5, 40))
    tr[3]["n"] = (31, 9, 17)    # a non-cubic one with ragged tiles
    return tr


@pytest.mark.parametrize("precision,order", [(sale.SALE_FP64, "fifo"), (sale.SALE_MIXED32, "fifo"),
                                             (sale.SALE_MIXED32, "sjf")])
def test_served_results_equal_alone_results(precision, order):
    say("serving equality, precision", precision, order)
    trace = small_trace()
    per = [sale.sale_workspace_bytes(workloads.request_problem(r, precision)[0]) for r in trace]
    budget = 3 * max(per) + (1 << 20)   # a few runs at a time: admission has to wait
    served, st = workloads.serve(trace, precision, budget, max_runs=8, slice_steps=7, order=order)
    assert [s.index for s in served] == list(range(len(trace)))
    assert st["requests"] == len(trace) and st["launches"] >= 2
    assert any(s.admitted > s.arrival + 1e-3 for s in served), "no request ever waited for memory"
    for s in served:
        req = trace[s.index]
        cfg, prob = workloads.request_problem(req, precision)
        r = sale.SaleRun(cfg, prob)
        r.step(req["steps"])
        ref = r.fields()
        for k in FIELDS:
            assert np.array_equal(s.fields[k], ref[k]), (s.index, k)
        assert s.finished >= s.admitted >= s.arrival
