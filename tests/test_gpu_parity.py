"""GPU parity: libqsv's HIP path, called through the C ABI, against the FP64 oracle on the
same seeded inputs.  Tolerances: complex128 max|d alpha| <= 1e-12; complex64
max|d alpha| <= 5e-6 and fidelity deficit 1 - |<psi_oracle|psi_gpu>|^2 <= 1e-5 (the gpu
state is not renormalised, so norm drift counts as error)."""
import math

import numpy as np
import pytest

import oracle
from paper_2604_03816_amd import circuits as C

pytestmark = pytest.mark.gpu

TOL = {"c128": 1e-12, "c64": 5e-6}
DEFICIT = {"c128": 1e-12, "c64": 1e-5}


@pytest.fixture(scope="module")
def qsv():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    from paper_2604_03816_amd import qsv as q
    q.lib()
    return q


def rand_state(n, rng):
    v = rng.standard_normal(1 << n) + 1j * rng.standard_normal(1 << n)
    return np.ascontiguousarray(v / np.linalg.norm(v))


def rand_unitary(d, rng):
    z = rng.standard_normal((d, d)) + 1j * rng.standard_normal((d, d))
    q, r = np.linalg.qr(z)
    return q * (np.diag(r) / np.abs(np.diag(r)))


def check_state(got, ref, dtype, ctx=""):
    err = oracle.max_abs_diff(ref, got)
    assert err <= TOL[dtype], "max|d alpha| = %.3g %s" % (err, ctx)
    deficit = 1.0 - oracle.fidelity(ref, got)
    assert deficit <= DEFICIT[dtype], "fidelity deficit %.3g %s" % (deficit, ctx)
    return err


def run(qsv, n, dtype, ops, psi0=None, **opts):
    s = qsv.State(n, dtype)
    if psi0 is not None:
        s.set(psi0)
    s.apply(ops, **opts)
    return s


# ------------------------------------------------------------------ config 1 (10 qubits)

@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("fuse", [True, False])
def test_brickwork_10q_depth20(qsv, dtype, fuse):
    n = 10
    ops = C.brickwork(n, 20, seed=1)
    ref = oracle.simulate(n, ops)
    s = run(qsv, n, dtype, ops, fuse=fuse)
    check_state(s.get(), ref, dtype)
    p = s.probs()
    assert np.max(np.abs(p - oracle.probs(ref))) <= (1e-13 if dtype == "c128" else 1e-6)


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("n", [1, 2, 3, 5, 10, 12, 13, 14, 17, 20])
def test_ghz_closed_form(qsv, dtype, n):
    ops = C.ghz(n) if n > 1 else [C.Op("H", (0,))]
    s = run(qsv, n, dtype, ops)
    got = s.get().astype(np.complex128)
    amp = 1 / math.sqrt(2)
    tol = TOL[dtype]
    assert abs(got[0] - amp) <= tol and abs(got[-1] - amp) <= tol
    rest = got.copy()
    rest[0] = rest[-1] = 0
    assert np.max(np.abs(rest)) <= tol
    if n >= 2:
        e, per = s.expval([(1.0, ((0, "Z"), (n - 1, "Z"))), (1.0, ((n // 2, "X"),))], per_term=True)
        assert abs(per[0] - 1) <= 10 * tol and abs(per[1]) <= 10 * tol


def test_empty_circuit_leaves_zero_state(qsv):
    for dt in ("c64", "c128"):
        s = run(qsv, 15, dt, [])
        got = s.get()
        assert got[0] == 1 and np.count_nonzero(got) == 1


# ------------------------------------------------------------------ per-kernel parity

TARGET_SETS = {
    1: [(0,), (3,), (6,), (11,), (15,)],
    2: [(0, 1), (4, 0), (2, 9), (13, 15), (5, 14)],
    3: [(0, 1, 2), (7, 3, 12), (15, 14, 13), (0, 8, 15)],
    4: [(0, 1, 2, 3), (6, 11, 2, 15), (12, 13, 14, 15)],
    5: [(0, 1, 2, 3, 4), (9, 1, 15, 6, 12), (11, 12, 13, 14, 15)],
}


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("k", [1, 2, 3, 4, 5])
def test_single_dense_gate_every_target_class(qsv, dtype, k):
    """One dense k-qubit unitary on low (in-row), tile and high (strided) qubits, applied to
    a random state; n = 16 spans several tiles."""
    n = 16
    rng = np.random.default_rng(30 + k)
    for targets in TARGET_SETS[k]:
        psi0 = rand_state(n, rng)
        op = C.Op("U", targets, matrix=rand_unitary(1 << k, rng))
        ref = oracle.simulate(n, [op], psi=psi0.copy())
        for fuse in (True, False):
            s = run(qsv, n, dtype, [op], psi0=psi0, fuse=fuse)
            check_state(s.get(), ref, dtype)


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_diagonal_and_permutation_ops(qsv, dtype):
    n = 17
    rng = np.random.default_rng(77)
    psi0 = rand_state(n, rng)
    ops = []
    for targets in [(0,), (16,), (3, 14), (0, 8, 16), (1, 5, 9, 13, 16)]:
        d = np.exp(1j * rng.uniform(0, 2 * math.pi, size=1 << len(targets)))
        ops.append(C.Op("U", targets, matrix=np.diag(d)))
    ops += [C.Op("CNOT", (16, 0)), C.Op("SWAP", (2, 15)), C.Op("TOFFOLI", (4, 12, 16)), C.Op("X", (9,)),
            C.Op("Y", (13,)), C.Op("CZ", (0, 16)), C.Op("S", (15,))]
    perm = np.zeros((8, 8), dtype=complex)
    for r, c in enumerate([3, 0, 7, 1, 2, 6, 4, 5]):
        perm[r, c] = np.exp(1j * r)
    ops.append(C.Op("U", (14, 1, 7), matrix=perm))
    ref = oracle.simulate(n, ops, psi=psi0.copy())
    for opts in ({}, {"fuse": False}, {"kmax": 1}, {"tile_qubits": 8, "low_qubits": 3}):
        s = run(qsv, n, dtype, ops, psi0=psi0, **opts)
        check_state(s.get(), ref, dtype, opts)


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("seed", [0, 1, 2])
def test_random_multi_qubit_circuits(qsv, dtype, seed):
    rng = np.random.default_rng(500 + seed)
    n = 18
    ops = []
    for _ in range(120):
        k = int(rng.integers(1, 4))
        qs = tuple(int(q) for q in rng.permutation(n)[:k])
        ops.append(C.Op("U", qs, matrix=rand_unitary(1 << k, rng)))
    ref = oracle.simulate(n, ops)
    for opts in ({}, {"cost_aware": -1}, {"kmax": 2}, {"fuse": False}, {"pass_budget": -1},
                 {"tile_qubits": 10, "low_qubits": 2}, {"tile_qubits": 7, "low_qubits": 6}):
        s = run(qsv, n, dtype, ops, **opts)
        check_state(s.get(), ref, dtype, opts)


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("circuit", ["brickwork", "hea", "qft", "random1q"])
def test_workload_circuits_20q(qsv, dtype, circuit):
    n = 20
    ops = {"brickwork": lambda: C.brickwork(n, 20, 2),
           "hea": lambda: C.bind(C.hea(n, 6), C.hea_params(n, 6, seed=4)),
           "qft": lambda: C.qft(n),
           "random1q": lambda: C.random_1q(n, 9)}[circuit]()
    ref = oracle.simulate(n, ops)
    for opts in ({}, {"fuse": False}):
        s = run(qsv, n, dtype, ops, **opts)
        check_state(s.get(), ref, dtype, opts)


def test_plan_reuse_and_pass_ranges(qsv):
    n = 19
    ops = C.brickwork(n, 8, 11)
    ref = oracle.simulate(n, ops)
    plan = qsv.Plan(n, "c128", ops)
    npass = plan.stats()["passes"]
    assert npass >= 2
    s = qsv.State(n, "c128")
    s.apply_plan(plan, 0, 1)
    s.apply_plan(plan, 1, npass - 1)
    s.sync()
    check_state(s.get(), ref, "c128")
    s.reset()
    s.apply_plan(plan)
    s.sync()
    check_state(s.get(), ref, "c128")
    with pytest.raises(qsv.QSVError):
        s.apply_plan(qsv.Plan(n, "c64", ops))
    with pytest.raises(qsv.QSVError):
        s.apply_plan(plan, npass, 1)


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_refreshed_plan_on_device(qsv, dtype):
    """qsv_plan_refresh on a plan already applied on the device: the stale tables are
    replaced, and the refreshed plan applies the ansatz with the new angles (oracle)."""
    n, L = 20, 3
    tmpl = C.hea(n, L, ring=True)
    plan = qsv.Plan(n, dtype, C.bind(tmpl, C.hea_params(n, L, seed=31)))
    s = qsv.State(n, dtype)
    for seed in (32, 33):
        ops = C.bind(tmpl, C.hea_params(n, L, seed=seed))
        plan.refresh(ops)
        s.apply_plan_zero(plan)
        check_state(s.get(), oracle.simulate(n, ops), dtype, "seed %d" % seed)
    s.free()
    plan.free()


# ------------------------------------------------------------------ reductions

@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("n", [9, 14, 21])
def test_norm_probs_expval_random_state(qsv, dtype, n):
    rng = np.random.default_rng(900 + n)
    psi = rand_state(n, rng)
    s = qsv.State(n, dtype)
    s.set(psi)
    ref = psi if dtype == "c128" else psi.astype(np.complex64).astype(np.complex128)
    assert abs(s.norm() - oracle.norm2(np.ascontiguousarray(ref))) <= 1e-13
    p = s.probs()
    assert np.max(np.abs(p - oracle.probs(ref))) <= (1e-15 if dtype == "c128" else 1e-9)
    for qubits in [(0,), (n - 1,), (3, 1), (n - 1, 0, n // 2), tuple(range(0, n, 2)), (n - 2, n - 1)]:
        got = s.probs(qubits)
        want = oracle.probs(ref, qubits)
        assert np.max(np.abs(got - want)) <= 1e-14, qubits
    terms = C.zz_chain_terms(n, periodic=True) + C.x_sum_terms(n, coeff=0.7)
    terms += [(0.3, ((0, "Y"), (n - 1, "Y"))), (-1.2, ((1, "X"), (n - 2, "Y"), (n // 2, "Z"))),
              (0.5, ((2, "Y"),)), (2.0, ()), (0.9, tuple((q, "Z") for q in range(n)))]
    tot, per = s.expval(terms, per_term=True)
    want = oracle.expval_terms(ref, terms)
    assert np.max(np.abs(per - want)) <= 1e-13
    assert abs(tot - math.fsum(want)) <= 1e-12


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("n", [8, 12, 23])
def test_expval_many_z_terms(qsv, dtype, n):
    """More Z-only terms than one launch holds (random supports inside and outside the
    tile, the identity, a Y-free phase), mixed with X/Y terms, against the oracle."""
    rng = np.random.default_rng(700 + n)
    psi = rand_state(n, rng)
    s = qsv.State(n, dtype)
    s.set(psi)
    ref = psi if dtype == "c128" else psi.astype(np.complex64).astype(np.complex128)
    terms = []
    for _ in range(70):
        k = int(rng.integers(1, min(n, 6) + 1))
        terms.append((float(rng.normal()), tuple((int(q), "Z") for q in rng.permutation(n)[:k])))
    terms += [(1.5, ()), (0.4, ((n - 1, "X"), (0, "Z"))), (-0.8, ((1, "Y"), (n - 2, "Z"), (n // 2, "Z")))]
    tot, per = s.expval(terms, per_term=True)
    want = oracle.expval_terms(ref, terms)
    assert np.max(np.abs(per - want)) <= 1e-13
    assert abs(tot - math.fsum(want)) <= 1e-12


def test_reductions_are_deterministic(qsv):
    n = 22
    s = qsv.State(n, "c64")
    s.apply(C.brickwork(n, 4, 3))
    a = [s.norm() for _ in range(3)]
    terms = C.tfim_terms(n)
    b = [s.expval(terms) for _ in range(3)]
    assert a[0] == a[1] == a[2]
    assert b[0] == b[1] == b[2]


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_product_state_closed_form_22q(qsv, dtype):
    """HEA without entanglers: <Z_q> and <X_q> per qubit from 2x2 algebra; no oracle run."""
    n, layers = 22, 4
    params = C.hea_params(n, layers, seed=12)
    s = qsv.State(n, dtype)
    s.apply(C.bind(C.hea(n, layers, entangle=False), params))
    Z = np.array([[1, 0], [0, -1]])
    X = np.array([[0, 1], [1, 0]])
    terms, want = [], []
    for q in range(n):
        v = np.array([1, 0], dtype=complex)
        for l in range(layers):
            v = oracle.gate_matrix("RY", (params[2 * (l * n + q)],)) @ v
            v = oracle.gate_matrix("RZ", (params[2 * (l * n + q) + 1],)) @ v
        terms += [(1.0, ((q, "Z"),)), (1.0, ((q, "X"),))]
        want += [(v.conj() @ Z @ v).real, (v.conj() @ X @ v).real]
    _, per = s.expval(terms, per_term=True)
    tol = 1e-12 if dtype == "c128" else 2e-6
    assert np.max(np.abs(per - np.array(want))) <= tol


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_circuit_then_inverse_is_identity_24q(qsv, dtype):
    n = 24
    ops = C.brickwork(n, 10, 21)
    s = qsv.State(n, dtype)
    s.apply(ops)
    assert abs(s.norm() - 1) <= (1e-12 if dtype == "c128" else 1e-5)
    s.apply(C.inverse_ops(ops))
    got = s.get()
    tol = 1e-12 if dtype == "c128" else 2e-5
    assert abs(got[0] - 1) <= tol
    assert np.max(np.abs(got[1:])) <= tol


@pytest.mark.parametrize("n,dtype", [(33, "c64"), (34, "c64"), (32, "c128")])
def test_maximum_sizes_circuit_then_inverse(qsv, n, dtype):
    """The largest states the ABI accepts (34 qubits: 128 GiB in complex64) and the
    largest complex128 state the precision study uses (32 qubits, 64 GiB): a random
    brickwork and its inverse return |0...0> (checked on the device through the norm, a
    marginal and sampling, without copying the state to the host)."""
    import torch
    ops = C.brickwork(n, 3, 40 + n)
    s = qsv.State(n, dtype)
    s.apply(ops)
    tol = 1e-12 if dtype == "c128" else 1e-5
    assert abs(s.norm() - 1) <= tol
    s.apply(C.inverse_ops(ops))
    p = s.probs([0, n // 2, n - 1])
    assert abs(p[0] - 1) <= 10 * tol and np.max(np.abs(p[1:])) <= 10 * tol
    assert np.all(s.sample(np.linspace(0.0, 0.999, 64)) == 0)
    s.free()
    torch.cuda.empty_cache()


def test_empty_inputs(qsv):
    s = qsv.State(12, "c64")
    s.apply([])                                   # empty circuit: nothing to do
    assert abs(s.expval([]) - 0.0) == 0.0         # empty Pauli sum
    assert s.sample(np.zeros(0)).size == 0        # no shots
    assert abs(s.norm() - 1) < 1e-7
    s.free()


# ------------------------------------------------------------------ commutation-aware plans

@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("circuit", ["mix", "h_t_cz"])
def test_commutation_aware_plans(qsv, dtype, circuit):
    """Plans whose fusion and passes cross commuting ops (diagonal on every shared
    qubit) against the oracle, beside the per-qubit DAG and a narrow-tile geometry."""
    n = 20
    ops = C.commuting_mix(n, 500, 11) if circuit == "mix" else C.h_t_cz_bricks(n, 16, 3)
    ref = oracle.simulate(n, ops)
    for opts in ({}, {"commute": -1}, {"tile_qubits": 8, "low_qubits": 3}, {"kmax": 3}):
        s = run(qsv, n, dtype, ops, **opts)
        check_state(s.get(), ref, dtype, str(opts))
        s.free()


# ------------------------------------------------------------------ |0...0> built inside the first pass

@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("n", [10, 16, 22])
def test_apply_zero_matches_reset_then_apply(qsv, dtype, n):
    """qsv_plan_apply_zero ignores the buffer's contents: from a random state it gives
    the circuit applied to |0...0>, for the whole plan, a prefix of it and no pass."""
    rng = np.random.default_rng(60 + n)
    ops = C.brickwork(n, 6, 7) + C.ghz(n)
    ref = oracle.simulate(n, ops)
    plan = qsv.Plan(n, dtype, ops, tile_qubits=min(n, 8) if n > 12 else 0)
    s = qsv.State(n, dtype)
    s.set(rand_state(n, rng))
    s.apply_plan_zero(plan)
    check_state(s.get(), ref, dtype)
    npass = plan.stats()["passes"]
    if npass > 1:
        s.set(rand_state(n, rng))
        s.apply_plan_zero(plan, 1)
        s.apply_plan(plan, 1, npass - 1)
        check_state(s.get(), ref, dtype, "prefix then the rest")
    s.set(rand_state(n, rng))
    s.apply_plan_zero(plan, 0)
    z = np.zeros(1 << n, complex)
    z[0] = 1
    check_state(s.get(), z, dtype, "count 0")
    with pytest.raises(qsv.QSVError):
        s.apply_plan_zero(plan, npass + 1)
    s.free()
    plan.free()
