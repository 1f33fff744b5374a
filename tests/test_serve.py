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


# ------------------------------------------------------------------ adaptive precision (Eq. 11 / Eq. 12)

def _paper(key):
    import json
    import os
    with open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")) as f:
        return json.load(f)[key]["value"]


def test_precision_rule_reproduces_the_paper():
    ex = _paper("precision_bound_example")
    lhs = ex["g"] * 2 ** ex["n"] * 1.19e-7
    assert round(lhs) == ex["lhs"]                              # "approximately 2.5 x 10^1"
    assert qsv.precision_select(ex["n"], ex["g"]) == "c128"   # far above the threshold
    limit = _paper("precision_c64_gate_limit_20q")
    for g in (1, 10, limit - 1):
        assert qsv.precision_select(20, g) == "c64"
    for g in (limit, limit + 1, 200):
        assert qsv.precision_select(20, g) == "c128"
    # shallow moderate-width circuits (n <= 16, g < 50) stay in complex64
    assert qsv.precision_select(16, 49) == "c64"
    # an explicit tolerance moves the boundary: g * 2^n * 1.19e-7 <= tol
    assert qsv.precision_select(10, 100, eps_tol=100 * 1024 * 1.19e-7 * 1.0001) == "c64"
    assert qsv.precision_select(10, 100, eps_tol=100 * 1024 * 1.19e-7 * 0.9999) == "c128"
    with pytest.raises(qsv.QSVError):
        qsv.precision_select(0, 10)


def test_auto_requests_follow_the_rule():
    sv = Server(max_slots=8, dry_run=True, capacity_bytes=1 << 34)
    want = {}
    for n, depth in ((12, 2), (20, 2), (14, 10), (22, 1), (16, 3)):
        ops = C.brickwork(n, depth, 1)
        rid = sv.submit(n, "auto", ops)
        want[rid] = qsv.precision_select(n, len(ops))
    got = {r["id"]: r for r in drain(sv)}
    assert set(got) == set(want)
    for rid, dt in want.items():
        assert got[rid]["dtype"] == dt and got[rid]["requested"] == "auto" and not got[rid]["promoted"]
    st = sv.stats()
    assert st["auto_c64"] == sum(v == "c64" for v in want.values())
    assert st["auto_c128"] == sum(v == "c128" for v in want.values())
    sv.close()
