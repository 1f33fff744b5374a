"""Serving on the GPU: every served result matches the FP64 oracle, a request's final
state and results are identical alone and in a mix of concurrently running requests
(continuous batching changes nothing per request), graph replay equals direct launches,
and admission under a small HBM capacity still completes every request."""
import numpy as np
import pytest

import oracle
from paper_2604_03816_amd import circuits as C

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mods():
    import torch
    assert torch.cuda.is_available()
    from paper_2604_03816_amd import qsv, serve
    qsv.lib()
    return qsv, serve


def drain(sv):
    out = []
    for _ in range(100000):
        r, p = sv.step()
        out += sv.results()
        st = sv.stats()
        if r == 0 and p == 0 and st["finished"] + st["rejected"] >= st["submitted"]:
            return out + sv.results()
    raise AssertionError("server did not drain")


def zexp_oracle(n, ops):
    psi = oracle.simulate(n, ops)
    return np.array([oracle.pauli_expval(psi, ((q, "Z"),)).real for q in range(n)]), oracle.norm2(psi), psi


def mix(seed, count=24):
    rng = np.random.default_rng(seed)
    reqs = []
    for _ in range(count):
        n = int(rng.integers(6, 17))
        reqs.append((n, "c64" if rng.random() < 0.6 else "c128", C.brickwork(n, int(rng.integers(2, 9)), int(rng.integers(1 << 30)))))
    return reqs


def test_served_results_match_oracle(mods):
    qsv, serve = mods
    sv = serve.Server(max_slots=16)
    reqs = mix(1)
    ids = {sv.submit(n, dt, ops): (n, dt, ops) for n, dt, ops in reqs}
    res = drain(sv)
    assert len(res) == len(reqs)
    for r in res:
        n, dt, ops = ids[r["id"]]
        z, nrm, _ = zexp_oracle(n, ops)
        tol = 1e-12 if dt == "c128" else 5e-5
        assert r["status"] == 0
        assert abs(r["norm"] - nrm) <= tol
        assert np.max(np.abs(r["zexp"] - z)) <= tol, (n, dt)
    sv.close()


@pytest.mark.parametrize("dtype", ["c64", "c128"])
def test_alone_versus_in_the_mix(mods, dtype):
    qsv, serve = mods
    n = 15
    probe = C.brickwork(n, 12, 77)
    alone = serve.Server(max_slots=8, keep_states=True)
    pid = alone.submit(n, dtype, probe)
    ra = [r for r in drain(alone) if r["id"] == pid][0]
    sa = alone.get_state(pid, n, dtype)
    alone.close()
    # in a mix: other requests before, with and after the probe
    sv = serve.Server(max_slots=8, keep_states=True)
    others = mix(2, 20)
    for n2, dt2, ops2 in others[:10]:
        sv.submit(n2, dt2, ops2)
    sv.step()
    qid = sv.submit(n, dtype, probe)
    for n2, dt2, ops2 in others[10:]:
        sv.submit(n2, dt2, ops2)
    rm = [r for r in drain(sv) if r["id"] == qid][0]
    sm = sv.get_state(qid, n, dtype)
    assert sv.stats()["peak_running"] > 1
    assert np.array_equal(sa, sm), "final state differs between alone and in the mix"
    assert ra["norm"] == rm["norm"] and np.array_equal(ra["zexp"], rm["zexp"])
    # and equal to the plain path's state within tolerance (same circuit, one at a time)
    s = qsv.State(n, dtype)
    s.apply(probe)
    tol = 1e-12 if dtype == "c128" else 5e-6
    assert np.max(np.abs(s.get().astype(np.complex128) - sm.astype(np.complex128))) <= tol
    _, _, psi = zexp_oracle(n, probe)
    assert np.max(np.abs(psi - sm.astype(np.complex128))) <= tol
    sv.close()


def test_graph_replay_equals_direct_launches(mods):
    qsv, serve = mods
    reqs = mix(3, 16)
    outs = []
    for use_graph in (True, False):
        sv = serve.Server(max_slots=6, use_graph=use_graph, passes_per_step=2)
        ids = [sv.submit(n, dt, ops) for n, dt, ops in reqs]
        res = {r["id"]: r for r in drain(sv)}
        outs.append([(res[i]["norm"], tuple(res[i]["zexp"])) for i in ids])
        if use_graph:
            assert sv.stats()["graph_replays"] >= 2
        sv.close()
    assert outs[0] == outs[1]


def test_small_capacity_admission_on_device(mods):
    qsv, serve = mods
    reqs = mix(4, 12)
    cap = max((1 << n) * (8 if dt == "c64" else 16) for n, dt, _ in reqs) * 3 // 2 + (1 << 20)
    sv = serve.Server(max_slots=8, capacity_bytes=cap)
    ids = {sv.submit(n, dt, ops): (n, dt, ops) for n, dt, ops in reqs}
    res = drain(sv)
    st = sv.stats()
    assert st["finished"] == len(reqs)
    assert st["peak_used_bytes"] <= cap
    for r in res:
        n, dt, ops = ids[r["id"]]
        z, _, _ = zexp_oracle(n, ops)
        assert np.max(np.abs(r["zexp"] - z)) <= (1e-12 if dt == "c128" else 5e-5)
    sv.close()


def test_open_loop_stream_and_plain_path(mods):
    qsv, serve = mods
    reqs = C.serving_stream(40, seed=9, rate_hz=400.0, n_lo=12, n_hi=18, d_lo=5, d_hi=15)
    circuits = [qsv.ArrayGateList(C.brickwork_arrays(r.n, r.depth, r.seed)) for r in reqs]
    sv = serve.Server(max_slots=32)
    out = serve.run_batched(reqs, circuits, sv)
    assert out["completed"] == 40 and out["p99_ms"] >= out["p50_ms"] > 0
    sv.close()
    plain = serve.run_plain(reqs[:8], circuits[:8])
    assert plain["completed"] == 8


def test_auto_precision_and_norm_guard(mods):
    """dtype "auto": the precision of Eq. 12 (small circuits complex64, large complex128)
    and results against the oracle at that precision; with a norm guard that every
    complex64 run fails, each of them is repeated in complex128 under the same id."""
    qsv, serve = mods
    rng = np.random.default_rng(8)
    reqs = []
    for _ in range(10):
        n = int(rng.integers(6, 15))
        reqs.append((n, C.brickwork(n, int(rng.integers(1, 6)), int(rng.integers(1 << 30)))))
    reqs += [(16, C.brickwork(16, 40, 3)), (16, C.brickwork(16, 45, 4))]   # beyond Eq. 12's bound
    for guard in (0.0, 1e-300):
        sv = serve.Server(max_slots=8, norm_guard=guard)
        ids = {sv.submit(n, "auto", ops): (n, ops) for n, ops in reqs}
        res = drain(sv)
        assert len(res) == len(reqs)
        st = sv.stats()
        promoted = 0
        for r in res:
            n, ops = ids[r["id"]]
            chosen = qsv.precision_select(n, len(ops))
            assert r["requested"] == "auto"
            if guard > 0 and chosen == "c64":
                # complex64 rounding always moves the norm a little away from 1
                assert r["promoted"] and r["dtype"] == "c128"
                promoted += 1
            else:
                assert not r["promoted"] and r["dtype"] == chosen
            z, nrm, _ = zexp_oracle(n, ops)
            tol = 1e-12 if r["dtype"] == "c128" else 5e-5
            assert abs(r["norm"] - nrm) <= tol and np.max(np.abs(r["zexp"] - z)) <= tol
        assert st["promoted"] == promoted
        assert st["auto_c64"] + st["auto_c128"] == len(reqs)
        assert st["auto_c64"] > 0 and st["auto_c128"] > 0
        sv.close()


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_served_circuits_with_diagonal_and_permutation_ops(mods, dtype):
    """QFT (controlled phases: diagonal tables staged with the pass), circuits with
    SWAP / Toffoli (permutations) and GHZ circuits (CNOT chains fused into 5-qubit
    permutations: passes for the kernel variant with the wide op paths, in the same steps
    as passes for the lighter one) through the batched kernel."""
    qsv, serve = mods
    sv = serve.Server(max_slots=8)
    reqs = [(n, C.qft(n)) for n in (8, 12, 15)] + [(n, C.ghz(n)) for n in (14, 17)]
    rng = np.random.default_rng(5)
    for n in (9, 14):
        ops = C.brickwork(n, 4, int(rng.integers(1 << 30)))
        ops += [C.Op("SWAP", (0, n - 1)), C.Op("TOFFOLI", (1, n - 2, 3)), C.Op("CZ", (2, n - 3)), C.Op("T", (n - 1,))]
        reqs.append((n, ops))
    ids = {sv.submit(n, dtype, ops): (n, ops) for n, ops in reqs}
    res = drain(sv)
    assert len(res) == len(reqs)
    for r in res:
        n, ops = ids[r["id"]]
        z, nrm, _ = zexp_oracle(n, ops)
        tol = 1e-12 if dtype == "c128" else 5e-5
        assert r["status"] == 0 and abs(r["norm"] - nrm) <= tol and np.max(np.abs(r["zexp"] - z)) <= tol
    sv.close()


def _serve_golden(n, depth, seed):
    import json
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "serve_brickwork_n%d_d%d_s%d.json" % (n, depth, seed))
    with open(path) as f:
        return json.load(f)


SERVE_LARGE = [(20, 30, 21), (24, 20, 22), (26, 15, 23)]


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_large_served_requests_against_oracle_alone_and_in_mix(mods, dtype):
    """Requests at the large end of the served sizes (20, 24 and 26 qubits: 2^14 - 2^15
    tiles per pass in the batched kernel, 2^12 - 2^14 chunks per state in the batched
    reduction) against per-qubit <Z_i>, norm and seeded amplitudes the FP64 oracle stored
    (tests/golden/make_golden.py serve); the 24-qubit request's final state is the same
    bit for bit alone and in a mix with small requests of both precisions, and within
    tolerance of the single-state path's."""
    qsv, serve = mods
    tol_z = 1e-12 if dtype == "c128" else 5e-5
    tol_a = 1e-12 if dtype == "c128" else 5e-6
    gold = {case[0]: _serve_golden(*case) for case in SERVE_LARGE}
    circ = {n: C.brickwork(n, d, s) for n, d, s in SERVE_LARGE}
    # alone: the 24-qubit request by itself
    alone = serve.Server(max_slots=8, keep_states=True)
    aid = alone.submit(24, dtype, circ[24])
    ra = [r for r in drain(alone) if r["id"] == aid][0]
    sa = alone.get_state(aid, 24, dtype)
    alone.close()
    # in a mix: small requests of both precisions before, between and after the large ones
    sv = serve.Server(max_slots=16, keep_states=True)
    small = mix(11, 18)
    for n2, dt2, ops2 in small[:6]:
        sv.submit(n2, dt2, ops2)
    ids = {}
    for k, (n, _, _) in enumerate(SERVE_LARGE):
        ids[sv.submit(n, dtype, circ[n])] = n
        for n2, dt2, ops2 in small[6 + 4 * k: 10 + 4 * k]:
            sv.submit(n2, dt2, ops2)
    res = {r["id"]: r for r in drain(sv)}
    assert sv.stats()["peak_running"] > 1
    for rid, n in ids.items():
        r, g = res[rid], gold[n]
        assert r["status"] == 0 and r["n"] == n and r["dtype"] == dtype
        assert abs(r["norm"] - g["norm2"]) <= (1e-12 if dtype == "c128" else 1e-5), (n, r["norm"])
        err = np.max(np.abs(r["zexp"] - np.array(g["zexp"])))
        assert err <= tol_z, (n, dtype, err)
        st = sv.get_state(rid, n, dtype).astype(np.complex128)
        ref = np.array(g["re"]) + 1j * np.array(g["im"])
        aerr = np.max(np.abs(st[np.array(g["index"])] - ref))
        assert aerr <= tol_a, (n, dtype, aerr)
        if n == 24:
            assert np.array_equal(st.astype(sa.dtype), sa), "24-qubit state differs between alone and in the mix"
            assert ra["norm"] == r["norm"] and np.array_equal(ra["zexp"], r["zexp"])
            s = qsv.State(n, dtype)
            s.apply(circ[n])
            assert np.max(np.abs(s.get().astype(np.complex128) - st)) <= tol_a
            s.free()
    sv.close()
