"""Serving core on the host only (dry_run: no device work): FIFO admission by HBM
footprint within a capacity, slot limits, continuous admission as requests finish,
rejection of requests that can never fit, and failed plans reported per request."""
import numpy as np
import pytest

from paper_2604_03816_amd import circuits as C
from paper_2604_03816_amd import qsv
from paper_2604_03816_amd.serve import Server


def drain(sv, limit=100000):
    out = []
    for _ in range(limit):
        r, p = sv.step()
        out += sv.results()
        if r == 0 and p == 0:
            # planning threads may still hold requests; a step with nothing pending ends it
            out += sv.results()
            st = sv.stats()
            if st["finished"] + st["rejected"] >= st["submitted"]:
                return out
    raise AssertionError("server did not drain")


def test_all_requests_finish_within_capacity_and_slots():
    reqs = C.serving_stream(60, seed=11, n_lo=12, n_hi=20)
    cap = int(1.2 * (1 << 20) * 16)   # room for one of the largest states (plus small ones)
    sv = Server(max_slots=4, capacity_bytes=cap, dry_run=True)
    for r in reqs:
        sv.submit(r.n, r.dtype, qsv.ArrayGateList(C.brickwork_arrays(r.n, 3, r.seed)))
    res = drain(sv)
    st = sv.stats()
    assert st["finished"] == len(reqs) and all(x["status"] == 0 for x in res)
    assert st["peak_running"] <= 4
    assert st["peak_used_bytes"] <= cap
    assert st["admission_waits"] > 0            # the capacity really bound admission
    # FIFO: admission order follows submission order
    admits = sorted(res, key=lambda x: (x["t_admit"], x["id"]))
    assert [x["id"] for x in admits] == sorted(x["id"] for x in res)
    sv.close()


def test_requests_that_can_never_fit_are_rejected_not_blocking():
    sv = Server(max_slots=8, capacity_bytes=(1 << 14) * 16, dry_run=True)
    big = sv.submit(20, "c128", C.ghz(20))
    small = [sv.submit(10, "c64", C.ghz(10)) for _ in range(5)]
    res = {r["id"]: r for r in drain(sv)}
    assert res[big]["status"] == qsv.QSV_E_OOM
    assert all(res[i]["status"] == 0 for i in small)
    assert sv.stats()["rejected"] == 1
    sv.close()


def test_passes_match_the_plan():
    sv = Server(max_slots=16, dry_run=True)
    ids = {}
    for n in (12, 16, 20, 24):
        ops = C.brickwork(n, 10, n)
        ids[sv.submit(n, "c64", ops)] = qsv.Plan(n, "c64", ops).stats()["passes"]
    for r in drain(sv):
        assert r["passes"] == ids[r["id"]]
    sv.close()


def test_bad_circuit_is_an_argument_error():
    sv = Server(dry_run=True)
    with pytest.raises(qsv.QSVError):
        sv.submit(4, "c64", [C.Op("H", (7,))])
    sv.close()
