"""Full-size parity at the benchmark's sizes, in the launch configuration bench.py times
(default plan options): seeded amplitudes, marginals and Pauli terms of the brickwork
circuits against values the FP64 oracle wrote to tests/golden/ (make_golden.py), plus
properties that hold at any size (norm, complex64 vs complex128 fidelity)."""
import json
import os

import numpy as np
import pytest

from paper_2604_03816_amd import circuits as C

pytestmark = pytest.mark.gpu
GOLD = os.path.join(os.path.dirname(__file__), "golden")
TOL = {"c128": 1e-12, "c64": 5e-6}


def load(n, depth, seed):
    path = os.path.join(GOLD, "brickwork_n%d_d%d_s%d.json" % (n, depth, seed))
    if not os.path.exists(path):
        pytest.skip("golden file %s not generated" % os.path.basename(path))
    with open(path) as f:
        return json.load(f)


@pytest.fixture(scope="module")
def qsv():
    import torch
    assert torch.cuda.is_available()
    from paper_2604_03816_amd import qsv as q
    q.lib()
    return q


def precision_gap(a, b, chunk=1 << 26):
    """Whole-state comparison of a complex64 state b with the complex128 state a of the
    same circuit, chunk by chunk on the device in FP64: max |a_k - b_k|, the raw overlap
    deficit 1 - |<a|b>|^2 and the normalised one 1 - |<a|b>|^2 / (<a|a> <b|b>).  The raw
    form follows b's norm drift; the normalised one is the state error proper."""
    import torch
    ov, na, nb, mx = 0j, 0.0, 0.0, 0.0
    for i in range(0, a.numel(), chunk):
        x = a[i:i + chunk]
        y = b[i:i + chunk].to(torch.complex128)
        ov += torch.vdot(x, y).item()
        na += torch.vdot(x, x).real.item()
        nb += torch.vdot(y, y).real.item()
        mx = max(mx, (x - y).abs().max().item())
    return {"max_abs_diff": mx, "raw_deficit": 1.0 - abs(ov) ** 2,
            "infidelity": 1.0 - abs(ov) ** 2 / (na * nb), "norm2_c64": nb, "norm2_c128": na}


def apply_as_bench(state, plan):
    """The benchmark step's launch sequence: the first pass builds |0...0> on chip, then
    every later pass is enqueued on its own (qsv_plan_apply_zero + qsv_plan_apply_range)."""
    npass = plan.stats()["passes"]
    state.apply_plan_zero(plan, 1)
    for i in range(1, npass):
        state.apply_plan(plan, i, 1)
    state.sync()


@pytest.mark.parametrize("n,depth,seed", [(22, 20, 7), (28, 20, 2), (30, 20, 3)])
def test_brickwork_full_size_against_oracle_samples(qsv, n, depth, seed):
    import torch
    g = load(n, depth, seed)
    ops = C.brickwork(n, depth, seed)
    idx = torch.tensor(g["index"], dtype=torch.int64, device="cuda")
    ref = np.array(g["re"]) + 1j * np.array(g["im"])
    got = {}
    for dtype in ("c128", "c64"):
        plan = qsv.Plan(n, dtype, ops)
        s = qsv.State(n, dtype)
        s.tensor.fill_(0.25 + 0.5j)   # whatever the buffer holds, the first pass starts from |0...0>
        torch.cuda.synchronize()
        apply_as_bench(s, plan)
        amps = s.tensor[idx].cpu().numpy().astype(np.complex128)
        err = np.max(np.abs(amps - ref))
        assert err <= TOL[dtype], (dtype, err)
        assert abs(s.norm() - g["norm2"]) <= (1e-12 if dtype == "c128" else 1e-5)
        marg = s.probs(g["marginal_qubits"])
        assert np.max(np.abs(marg - np.array(g["marginal"]))) <= (1e-12 if dtype == "c128" else 1e-6)
        terms = C.zz_chain_terms(n) + C.x_sum_terms(n)
        _, per = s.expval(terms, per_term=True)
        want = np.array(g["zz_terms"] + g["x_terms"])
        assert np.max(np.abs(per - want)) <= (1e-11 if dtype == "c128" else 1e-5)
        got[dtype] = s
        plan.free()
        del s
    # complex64 against complex128 over the whole state (properties at any size): every
    # amplitude within the complex64 bar, and the normalised infidelity within 1e-5
    gap = precision_gap(got["c128"].tensor, got["c64"].tensor)
    assert gap["max_abs_diff"] <= 5e-6, gap
    assert 0.0 <= gap["infidelity"] + 1e-12 and gap["infidelity"] <= 1e-5, gap
    assert gap["raw_deficit"] <= 1e-5, gap
    torch.cuda.synchronize()


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_bench_sequence_equals_whole_plan(qsv, dtype):
    """At 30 qubits with the default 2^12-amplitude tiles: the benchmark's sequence (first
    pass from |0...0> on chip, then one launch per pass) gives exactly the state of a
    reset followed by the whole plan in one call."""
    import torch
    n = 30
    ops = C.brickwork(n, 20, 3)
    plan = qsv.Plan(n, dtype, ops)
    a = qsv.State(n, dtype)
    apply_as_bench(a, plan)
    b = qsv.State(n, dtype)
    b.reset()
    b.apply_plan(plan)
    b.sync()
    assert torch.equal(a.tensor, b.tensor)
    plan.free()
    a.free()
    b.free()
    torch.cuda.synchronize()
