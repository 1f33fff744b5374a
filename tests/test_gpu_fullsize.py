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
        s.apply_plan(plan)
        s.sync()
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
    # complex64 against complex128 over the whole state (a property at any size):
    # fidelity deficit 1 - |<psi_128|psi_64>|^2 <= 1e-5
    a = got["c128"].tensor
    b = got["c64"].tensor.to(torch.complex128)
    ov = torch.vdot(a, b).abs().item() ** 2
    assert 1 - ov <= 1e-5, 1 - ov
    torch.cuda.synchronize()
