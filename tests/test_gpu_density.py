"""GPU parity of the density-matrix path (a 2n-qubit state holding vec(rho); gates as
U (x) conj(U), noise channels as Kraus superoperators) against the oracle's dense
density-matrix simulation, plus the Table 8 noise study."""
import numpy as np
import pytest

import oracle
from paper_2604_03816_amd import circuits as C

pytestmark = pytest.mark.gpu

TOL = {"c128": 1e-12, "c64": 5e-6}


@pytest.fixture(scope="module")
def qsv():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    from paper_2604_03816_amd import qsv as q
    q.lib()
    return q


def noisy_circuit(n, seed):
    rng = np.random.default_rng(seed)
    ops = []
    for layer in range(4):
        for q in range(n):
            ops.append(C.Op("U", (q,), matrix=C.haar_u2(rng)))
            if rng.random() < 0.5:
                ops.append(C.Op("DEPOLARIZE", (q,), (float(rng.uniform(0, 0.1)),)))
        for q in range(layer % 2, n - 1, 2):
            ops.append(C.Op("CNOT", (q, q + 1)))
            ops.append(C.Op("DEPOLARIZE", (q, q + 1), (float(rng.uniform(0, 0.1)),)))
        ops.append(C.Op("AMPDAMP", (int(rng.integers(n)),), (float(rng.uniform(0, 0.2)),)))
    return ops


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("n", [3, 5])
@pytest.mark.parametrize("fuse", [True, False])
def test_noisy_circuits_against_oracle(qsv, dtype, n, fuse):
    ops = noisy_circuit(n, 100 + n)
    ref = oracle.dm_simulate(n, ops)
    dm = qsv.DensityMatrix(n, dtype)
    dm.apply(ops, fuse=fuse)
    rho = dm.matrix()
    assert np.max(np.abs(rho - ref)) < TOL[dtype]
    for qubits in (None, [n - 1, 0], [1]):
        qs = list(range(n)) if qubits is None else qubits
        assert np.max(np.abs(dm.probs(qubits) - oracle.dm_probs(ref, qs))) < TOL[dtype]
    terms = [(0.5, ((0, "Z"), (1, "Z"))), (-1.0, ((n - 1, "X"),)), (0.25, ((0, "Y"), (2, "X"))), (2.0, ())]
    assert abs(dm.expval(terms) - oracle.dm_expval(ref, terms)) < 10 * TOL[dtype]
    dm.free()


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_noise_study_against_oracle(qsv, dtype):
    for n in (2, 3, 4, 5):
        ops = [C.Op("H", (0,)), C.Op("DEPOLARIZE", (0,), (0.01,))]
        for t in range(1, n):
            ops += [C.Op("CNOT", (0, t)), C.Op("DEPOLARIZE", (0,), (0.01,)), C.Op("DEPOLARIZE", (t,), (0.01,))]
        ref = oracle.dm_probs(oracle.dm_simulate(n, ops), list(range(n)))
        dm = qsv.DensityMatrix(n, dtype)
        dm.apply(ops)
        got = dm.probs()
        pi = np.zeros(1 << n)
        pi[0] = pi[-1] = 0.5
        assert abs(oracle.classical_fidelity(pi, got) - oracle.classical_fidelity(pi, ref)) < TOL[dtype]
        assert abs(oracle.tvd(pi, got) - oracle.tvd(pi, ref)) < TOL[dtype]
        dm.free()


def test_wide_noisy_ghz_invariants(qsv):
    # 12 system qubits: a 24-qubit vec(rho); unit trace, symmetric GHZ populations, and
    # complex64 against complex128
    n = 12
    ops = C.with_depolarizing(C.ghz(n), 0.002, 0.01)
    out = {}
    for dt in ("c128", "c64"):
        dm = qsv.DensityMatrix(n, dt)
        dm.apply(ops)
        p = dm.probs()
        assert abs(p.sum() - 1) < 10 * TOL[dt]
        assert abs(dm.expval([(1.0, ())]) - 1) < 10 * TOL[dt]
        out[dt] = p
        dm.free()
    p = out["c128"]
    assert p[0] > 0.4 and abs(p[0] - p[-1]) < 0.05
    assert np.max(np.abs(out["c64"] - p)) < 1e-5


def test_argument_errors(qsv):
    s = qsv.State(5, "c128")   # odd qubit count: not a density matrix
    with pytest.raises(qsv.QSVError):
        qsv.check(qsv.lib().qsv_dm_probs(s.h, None, 2, qsv._dptr(np.zeros(4))))
    s.free()
    dm = qsv.DensityMatrix(3, "c128")
    for bad in ([C.Op("DEPOLARIZE", (0, 1, 2), (0.1,))], [C.Op("DEPOLARIZE", (0,), (1.5,))],
                [C.Op("AMPDAMP", (0, 1), (0.1,))], [C.Op("H", (3,))]):
        with pytest.raises(qsv.QSVError):
            dm.apply(bad)
    dm.free()
