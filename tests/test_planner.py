"""Host-side tests of libqsv (no GPU): the C ABI loads and exports what include/qsv.h
declares; the library's gate set matches the oracle's; DAG fusion (Algorithm 2 with the
acyclicity fix) and pass scheduling preserve the circuit product (Eq. 10), which the
FP64 oracle checks by replaying the plan's fused gates in pass order."""
import ctypes
import os
import re

import numpy as np
import pytest

import oracle
from paper_2604_03816_amd import circuits as C
from paper_2604_03816_amd import qsv

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def rand_unitary(d, rng):
    z = rng.standard_normal((d, d)) + 1j * rng.standard_normal((d, d))
    q, r = np.linalg.qr(z)
    return q * (np.diag(r) / np.abs(np.diag(r)))


def plan_replay(n, plan):
    """Apply the plan's fused gates with the oracle, in the order the passes apply them."""
    fused = plan.fused_gates()
    psi = oracle.zero_state(n)
    order = []
    for idx, active in plan.passes():
        for i in idx:
            targets, m, diag = fused[i]
            if not diag:
                assert set(targets) <= set(active), "dense/perm op outside its tile"
            oracle.apply(psi, m, targets)
            order.append(i)
    assert sorted(order) == list(range(len(fused))), "every fused gate exactly once"
    return psi


# ------------------------------------------------------------------ the ABI

def test_library_exports_every_declared_symbol():
    hdr = open(os.path.join(ROOT, "include", "qsv.h")).read()
    declared = set(re.findall(r"\b(qsv_[a-z_]+)\s*\(", hdr))
    L = qsv.lib()
    missing = [name for name in sorted(declared) if not hasattr(L, name)]
    assert not missing, missing
    assert declared == set(qsv.EXPORTS)
    assert qsv.version().startswith("qsv")


@pytest.mark.parametrize("name,params", [("I", ()), ("X", ()), ("Y", ()), ("Z", ()), ("H", ()), ("S", ()),
                                         ("SDG", ()), ("T", ()), ("TDG", ()), ("RX", (0.7,)), ("RY", (-2.1,)),
                                         ("RZ", (4.0,)), ("U3", (0.3, 1.1, -0.4)), ("CNOT", ()), ("CZ", ()),
                                         ("SWAP", ()), ("TOFFOLI", ())])
def test_gate_set_matches_oracle(name, params):
    assert np.allclose(qsv.gate_matrix(name, params), oracle.gate_matrix(name, params), atol=1e-15)


def test_argument_errors():
    with pytest.raises(qsv.QSVError) as e:
        qsv.gate_matrix("NOPE")
    assert e.value.status == qsv.QSV_E_ARG
    bad = [C.Op("CNOT", (1, 1))]
    with pytest.raises(qsv.QSVError):
        qsv.Plan(4, "c64", bad)
    with pytest.raises(qsv.QSVError):
        qsv.Plan(4, "c64", [C.Op("H", (4,))])
    with pytest.raises(qsv.QSVError):
        qsv.Plan(40, "c64", [C.Op("H", (0,))])
    six = C.Op("U", tuple(range(6)), matrix=np.eye(64, dtype=complex))
    with pytest.raises(ValueError):
        qsv.Plan(8, "c64", [six])  # the binding's Gate struct holds 5 targets
    with pytest.raises(qsv.QSVError):
        qsv.Plan(16, "c64", C.ghz(16), tile_qubits=14)
    with pytest.raises(qsv.QSVError):
        qsv.Plan(16, "c64", C.ghz(16), kmax=6)
    with pytest.raises(qsv.QSVError):
        qsv.Plan(16, "c64", C.ghz(16), commute=2)
    with pytest.raises(qsv.QSVError):
        qsv.Plan(16, "c64", C.ghz(16), op_cost=-1.0)
    with pytest.raises(qsv.QSVError):   # matrix-core ops have 3 or 4 targets
        qsv.Plan(16, "c64", C.ghz(16), matrix_cores=5)


def test_op_cost_trades_fused_ops_for_arithmetic():
    """The per-op cost charged by the cost-aware fusion (Eq. 13 trade-off): a large one
    merges far more than a small one, and every resulting plan stays exact (oracle replay
    of the fused list equals the circuit)."""
    n = 10
    ops = C.brickwork(n, 12, seed=11)
    ref = oracle.simulate(n, ops)
    counts = {}
    for oc in (4.0, 8.0, 24.0, 64.0):
        p = qsv.Plan(n, "c128", ops, op_cost=oc, tile_qubits=8)
        counts[oc] = p.stats()["fused_out"]
        psi = oracle.zero_state(n)
        for t, m, d in p.fused_gates():
            oracle.apply(psi, m, t)
        assert oracle.max_abs_diff(ref, psi) <= 1e-12
        p.free()
    assert counts[64.0] < counts[8.0] < counts[4.0]


def test_null_arguments_return_errors():
    L = qsv.lib()
    assert L.qsv_alloc(10, 0, None, 0, None, None) == qsv.QSV_E_ARG
    assert L.qsv_plan_create(10, 0, None, 3, None, ctypes.byref(ctypes.c_void_p())) == qsv.QSV_E_ARG
    assert L.qsv_norm(None, None) == qsv.QSV_E_ARG
    assert L.qsv_free(None) == qsv.QSV_OK


def test_adopted_buffer_checks_come_before_any_device_call():
    # buffers are checked on the host: too small, or not 16-byte aligned (the kernels
    # move 16 bytes per lane); neither pointer is ever dereferenced
    L = qsv.lib()
    out = ctypes.c_void_p()
    assert L.qsv_alloc(10, 0, ctypes.c_void_p(0x10000), 4096, None, ctypes.byref(out)) == qsv.QSV_E_ARG
    assert L.qsv_alloc(10, 0, ctypes.c_void_p(0x10008), 8192, None, ctypes.byref(out)) == qsv.QSV_E_ARG
    assert "aligned" in L.qsv_last_error().decode()
    assert out.value is None


# ------------------------------------------------------------------ fusion soundness (Eq. 9 / Eq. 10)

def _random_gate_circuit(n, count, rng, kmax_gate=3):
    ops = []
    for _ in range(count):
        k = int(rng.integers(1, kmax_gate + 1))
        qs = tuple(int(q) for q in rng.permutation(n)[:k])
        ops.append(C.Op("U", qs, matrix=rand_unitary(1 << k, rng)))
    return ops


def test_paper_fusibility_counterexamples_stay_sound():
    """Gates u{0,1}, w1{1,3}, w2{3,2}, v{0,2}: Algorithm 2's rule (3) alone would merge u
    and v across w1 and w2; the shorter u{0,1}, w{1,2}, v{0,2} likewise.  The fused plan
    must still equal the circuit."""
    rng = np.random.default_rng(8)
    for qsets in ([(0, 1), (1, 3), (3, 2), (0, 2)], [(0, 1), (1, 2), (0, 2)]):
        ops = [C.Op("U", q, matrix=rand_unitary(4, rng)) for q in qsets]
        for kmax in (2, 3, 4, 5):
            for cost in (1, -1):
                plan = qsv.Plan(4, "c128", ops, kmax=kmax, cost_aware=cost)
                ref = oracle.simulate(4, ops)
                assert np.max(np.abs(plan_replay(4, plan) - ref)) < 1e-13


@pytest.mark.parametrize("seed", range(6))
@pytest.mark.parametrize("kmax", [1, 2, 3, 5])
@pytest.mark.parametrize("cost", [1, -1])
def test_fused_plan_equals_circuit_random(seed, kmax, cost):
    rng = np.random.default_rng(seed)
    n = 9
    ops = _random_gate_circuit(n, 60, rng)
    plan = qsv.Plan(n, "c128", ops, kmax=max(kmax, 3), cost_aware=cost, tile_qubits=6, low_qubits=2)
    ref = oracle.simulate(n, ops)
    assert np.max(np.abs(plan_replay(n, plan) - ref)) < 1e-12
    for targets, m, diag in plan.fused_gates():
        assert len(targets) <= max(kmax, 3)
        assert list(targets) == sorted(targets)
        off = m - np.diag(np.diag(m))
        assert diag == (np.max(np.abs(off)) == 0)


@pytest.mark.parametrize("circuit", ["brickwork", "hea", "qft", "ghz", "random1q"])
@pytest.mark.parametrize("dtype", ["c64", "c128"])
def test_plans_for_workload_circuits(circuit, dtype):
    n = 14
    ops = {"brickwork": lambda: C.brickwork(n, 12, 4),
           "hea": lambda: C.bind(C.hea(n, 3, ring=True), C.hea_params(n, 3, seed=2)),
           "qft": lambda: C.qft(n),
           "ghz": lambda: C.ghz(n),
           "random1q": lambda: C.random_1q(n, 5)}[circuit]()
    ref = oracle.simulate(n, ops)
    for opts in ({}, {"fuse": False}, {"kmax": 2}, {"cost_aware": -1}, {"tile_qubits": 8, "low_qubits": 3},
                 {"pass_budget": -1}):
        plan = qsv.Plan(n, dtype, ops, **opts)
        st = plan.stats()
        assert st["gates_in"] == len(ops)
        if opts.get("fuse", True) is False:
            assert st["passes"] == st["fused_out"] == len(ops)
        got = plan_replay(n, plan)
        assert np.max(np.abs(got - ref)) < 1e-12, opts


def test_fusion_reduces_gate_count_and_is_deterministic():
    n = 20
    ops = C.qft(n)
    a = qsv.Plan(n, "c128", ops, kmax=2, cost_aware=-1)
    b = qsv.Plan(n, "c128", ops, kmax=2, cost_aware=-1)
    sa, sb = a.stats(), b.stats()
    assert sa == sb
    assert sa["fused_out"] < len(ops)
    fa, fb = a.fused_gates(), b.fused_gates()
    assert all(x[0] == y[0] and np.array_equal(x[1], y[1]) for x, y in zip(fa, fb))
    # the brickwork at kmax=5 (pure Algorithm 2) fuses to fewer, wider gates than kmax=2
    bw = C.brickwork(16, 20, 3)
    s2 = qsv.Plan(16, "c64", bw, kmax=2, cost_aware=-1).stats()
    s5 = qsv.Plan(16, "c64", bw, kmax=5, cost_aware=-1).stats()
    assert s5["fused_out"] < s2["fused_out"] < len(bw)


def test_diagonal_gates_merge_and_need_no_tile_capacity():
    """A CZ ladder is diagonal: it fuses into diagonal ops that may touch qubits outside
    the pass's tile."""
    n = 16
    ops = [C.Op("H", (q,)) for q in range(n)] + [C.Op("CZ", (i, i + 1)) for i in range(n - 1)]
    ops += [C.Op("H", (q,)) for q in range(n)]
    # kmax = 1 keeps each CZ a separate diagonal op (no merge into the Hadamards)
    plan = qsv.Plan(n, "c128", ops, tile_qubits=8, low_qubits=4, kmax=1)
    st = plan.stats()
    assert st["diag_ops"] >= 1
    fused = plan.fused_gates()
    outside = 0
    for idx, active in plan.passes():
        for i in idx:
            t, m, diag = fused[i]
            if diag and not set(t) <= set(active):
                outside += 1
    assert outside >= 1
    ref = oracle.simulate(n, ops)
    assert np.max(np.abs(plan_replay(n, plan) - ref)) < 1e-12


def test_disjoint_diagonal_ops_merge_across_commuting_ops_only():
    """Diagonal ops on disjoint qubits have no DAG edge; with the commutation-aware DAG
    (the default) a diagonal op still joins the nearest earlier diagonal op within the
    width bound, moving back only past ops it commutes with.  The per-qubit DAG of
    Section 5.1 (commute = -1) keeps them apart."""
    n = 6
    layer = [C.Op("RZ", (q,), (0.3 + 0.1 * q,)) for q in range(n)]
    on = qsv.Plan(n, "c128", layer).stats()
    assert on["fused_out"] == on["diag_ops"] == 2          # 5 + 1 targets
    assert qsv.Plan(n, "c128", layer, commute=-1).stats()["fused_out"] == n
    assert qsv.Plan(n, "c128", layer, kmax=2).stats()["fused_out"] == 3
    # TOFFOLI(1, 2; 3) is diagonal on its controls: RZ on a control or on a free qubit
    # passes it and joins RZ(0); RZ on its target does not
    for q2, merged in ((3, False), (1, True), (4, True)):
        ops = [C.Op("RZ", (0,), (0.7,)), C.Op("TOFFOLI", (1, 2, 3)), C.Op("RZ", (q2,), (0.4,))]
        plan = qsv.Plan(n, "c128", ops, kmax=2)
        assert plan.stats()["fused_out"] == (2 if merged else 3), q2
        assert np.max(np.abs(plan_replay(n, plan) - oracle.simulate(n, ops))) < 1e-13


def test_identity_products_are_dropped():
    ops = [C.Op("X", (3,)), C.Op("X", (3,)), C.Op("CNOT", (0, 1)), C.Op("CNOT", (0, 1))]
    plan = qsv.Plan(5, "c64", ops)
    assert plan.stats()["fused_out"] == 0
    assert plan.stats()["passes"] == 0


def test_pass_tiles_hold_low_qubits_and_fit():
    n = 24
    plan = qsv.Plan(n, "c64", C.brickwork(n, 6, 1))
    for idx, active in plan.passes():
        assert len(active) == 12
        assert set(range(4)) <= set(active)   # complex64 tiles keep the 4 lowest qubits


def test_wide_gates_in_narrow_tiles():
    """A gate whose targets do not fit beside the reserved low qubits opens a pass with
    fewer low qubits instead of never being scheduled."""
    rng = np.random.default_rng(3)
    n = 14
    ops = [C.Op("U", (13, 12, 11), matrix=rand_unitary(8, rng)),
           C.Op("U", (9, 13, 7, 12, 10), matrix=rand_unitary(32, rng)),
           C.Op("U", (0, 13), matrix=rand_unitary(4, rng))]
    ref = oracle.simulate(n, ops)
    for tq, lq in ((7, 6), (6, 5), (8, 7), (6, 1)):
        for fuse in (True, False):
            plan = qsv.Plan(n, "c64", ops, tile_qubits=tq, low_qubits=lq, fuse=fuse)
            assert np.max(np.abs(plan_replay(n, plan) - ref)) < 1e-12
    with pytest.raises(qsv.QSVError):
        qsv.Plan(n, "c64", ops, tile_qubits=5, low_qubits=2)


def test_fusion_modes_and_matrix_core_option():
    n = 16
    ops = C.brickwork(n, 12, 9)
    plain = qsv.Plan(n, "c64", ops, fuse=False).stats()
    grouped = qsv.Plan(n, "c64", ops, fuse=2).stats()
    fused = qsv.Plan(n, "c64", ops).stats()
    # mode 2 keeps every gate (minus exact identities) but shares passes
    assert grouped["fused_out"] == plain["fused_out"] == plain["passes"]
    assert grouped["passes"] < plain["passes"]
    assert fused["fused_out"] < grouped["fused_out"]
    assert grouped["fma_per_amp"] == pytest.approx(plain["fma_per_amp"])
    assert fused["mfma_ops"] > 0 and fused["mfma_fma_per_amp"] > 0
    no_mc = qsv.Plan(n, "c64", ops, matrix_cores=-1).stats()
    assert no_mc["mfma_ops"] == 0 and no_mc["mfma_fma_per_amp"] == 0
    # complex128 runs them on FP64 matrix cores, at the FP64 VALU's rate except for 4-qubit
    # ops (three real products instead of four), which the planner then fuses more readily
    m128 = qsv.Plan(n, "c128", ops).stats()
    assert m128["mfma_ops"] > 0
    v128 = qsv.Plan(n, "c128", ops, matrix_cores=-1).stats()
    assert v128["mfma_ops"] == 0 and v128["fused_out"] >= m128["fused_out"]
    for bad in ({"fuse": 3}, {"fuse": -1}, {"matrix_cores": 2}, {"matrix_cores": 5}, {"matrix_cores": 6}, {"matrix_cores": -2}):
        with pytest.raises(qsv.QSVError):
            qsv.Plan(n, "c64", ops, **bad)


# ------------------------------------------------------------------ device tables (host re-enactment)

@pytest.mark.parametrize("seed", range(8))
@pytest.mark.parametrize("tq,lq", [(12, 5), (12, 4), (7, 6), (6, 5), (10, 2), (6, 1), (13, 8)])
def test_device_tables_reproduce_the_circuit(seed, tq, lq):
    """qsv_plan_emulate walks the exact tables the pass kernel reads (tile placement,
    strides, local bit positions, op pools); from a random state it must reproduce the
    oracle's result for every tile geometry."""
    rng = np.random.default_rng(1000 + seed)
    n = 14 + seed % 3
    ops = _random_gate_circuit(n, 40, rng)
    ops += [C.Op("U", (int(q),), matrix=np.diag(np.exp(1j * rng.uniform(0, 6, 2)))) for q in rng.permutation(n)[:4]]
    ops += [C.Op("CZ", (0, n - 1)), C.Op("TOFFOLI", (n - 1, 2, n - 3)), C.Op("SWAP", (1, n - 2))]
    v = rng.standard_normal(1 << n) + 1j * rng.standard_normal(1 << n)
    psi0 = np.ascontiguousarray(v / np.linalg.norm(v))
    ref = oracle.simulate(n, ops, psi=psi0.copy())
    for opts in ({}, {"fuse": False}, {"fuse": 2}, {"cost_aware": -1}, {"kmax": 1}, {"pass_budget": -1},
                 {"matrix_cores": -1}, {"matrix_cores": 4}):
        dt = "c64" if (seed % 2 or tq == 13) else "c128"   # 13-qubit tiles fit LDS only in complex64
        plan = qsv.Plan(n, dt, ops, tile_qubits=tq, low_qubits=lq, **opts)
        got = plan.emulate(psi0)
        assert np.max(np.abs(got - ref)) < 1e-12, opts


@pytest.mark.parametrize("circuit", ["brickwork", "hea", "qft"])
def test_device_tables_whole_state_and_workloads(circuit):
    for n in (9, 13, 15):
        ops = {"brickwork": lambda: C.brickwork(n, 10, 4),
               "hea": lambda: C.bind(C.hea(n, 3, ring=True), C.hea_params(n, 3, seed=2)),
               "qft": lambda: C.qft(n)}[circuit]()
        ref = oracle.simulate(n, ops)
        psi0 = np.zeros(1 << n, complex)
        psi0[0] = 1
        for dt in ("c64", "c128"):
            got = qsv.Plan(n, dt, ops).emulate(psi0)
            assert np.max(np.abs(got - ref)) < 1e-12


# ------------------------------------------------------------------ commutation-aware DAG

@pytest.mark.parametrize("seed", range(10))
@pytest.mark.parametrize("kmax", [2, 3, 5])
def test_commutation_aware_plan_equals_circuit(seed, kmax):
    """Fused ops applied in pass order (which may now run commuting ops ahead of earlier
    ones) reproduce the circuit; the per-qubit DAG gives the same state."""
    n = 9
    ops = C.commuting_mix(n, 80, 300 + seed)
    ref = oracle.simulate(n, ops)
    for commute in (1, -1):
        for cost in (1, -1):
            plan = qsv.Plan(n, "c128", ops, kmax=kmax, cost_aware=cost, commute=commute, tile_qubits=6,
                            low_qubits=2)
            assert np.max(np.abs(plan_replay(n, plan) - ref)) < 1e-12, (commute, cost)
            for targets, m, diag in plan.fused_gates():
                assert len(targets) <= max(kmax, 3)   # 3-qubit input gates stay as given


@pytest.mark.parametrize("seed", range(6))
@pytest.mark.parametrize("tq,lq", [(12, 5), (7, 3), (6, 1)])
def test_commutation_aware_device_tables(seed, tq, lq):
    rng = np.random.default_rng(400 + seed)
    n = 14
    ops = C.commuting_mix(n, 60, 400 + seed) + C.h_t_cz_bricks(n, 3, seed)
    v = rng.standard_normal(1 << n) + 1j * rng.standard_normal(1 << n)
    psi0 = np.ascontiguousarray(v / np.linalg.norm(v))
    ref = oracle.simulate(n, ops, psi=psi0.copy())
    for dt in ("c64", "c128"):
        for opts in ({}, {"commute": -1}, {"cost_aware": -1}, {"kmax": 2}):
            plan = qsv.Plan(n, dt, ops, tile_qubits=tq, low_qubits=lq, **opts)
            assert np.max(np.abs(plan.emulate(psi0) - ref)) < 1e-12, (dt, opts)


def test_commutation_never_adds_passes_and_cuts_them_on_commuting_circuits():
    n = 24
    cases = {"brickwork": C.brickwork(n, 10, 3), "qft": C.qft(n),
             "hea": C.bind(C.hea(n, 4, ring=True), C.hea_params(n, 4, seed=2)),
             "mix": C.commuting_mix(n, 400, 7), "h_t_cz": C.h_t_cz_bricks(n, 16, 2)}
    fewer = {}
    for name, ops in cases.items():
        for dt in ("c64", "c128"):
            on = qsv.Plan(n, dt, ops).stats()
            off = qsv.Plan(n, dt, ops, commute=-1).stats()
            assert on["passes"] <= off["passes"], (name, dt)
            fewer[(name, dt)] = off["passes"] - on["passes"]
    assert fewer[("h_t_cz", "c64")] >= 4 and fewer[("h_t_cz", "c128")] >= 1, fewer


def test_window_tiles_cut_passes_on_brickwork():
    """Passes are the best of a growing tile and fixed windows of consecutive qubits; on
    the 30-qubit depth-20 brickwork that needs 24 (complex64) / 25 (complex128) passes,
    where growing tiles alone needed 33 / 30 at the older budgets."""
    n = 30
    ops = C.brickwork(n, 20, 3)
    assert qsv.Plan(n, "c64", ops).stats()["passes"] <= 25
    assert qsv.Plan(n, "c128", ops).stats()["passes"] <= 26
    for _, active in qsv.Plan(n, "c64", ops).passes():
        assert len(active) == 12 and set(range(4)) <= set(active)


# ------------------------------------------------------------------ plan refresh

def _rotation_mix(n, count, rng, angles=None):
    """Rotations (RX, RY, RZ) with fixed gates (H, T, CNOT, CZ, a Haar 2-qubit unitary)
    between them; `angles` overrides the rotation angles in order."""
    ops, a = [], 0
    fixed = rand_unitary(4, np.random.default_rng(99))
    for _ in range(count):
        kind = rng.integers(0, 8)
        q = int(rng.integers(0, n))
        r = int((q + 1 + rng.integers(0, n - 1)) % n)
        if kind < 3:
            th = float(rng.uniform(-np.pi, np.pi))
            if angles is not None:
                th = float(angles[a])
            a += 1
            ops.append(C.Op(("RX", "RY", "RZ")[kind], (q,), (th,)))
        elif kind == 3:
            ops.append(C.Op("H", (q,)))
        elif kind == 4:
            ops.append(C.Op("T", (q,)))
        elif kind == 5:
            ops.append(C.Op("CNOT", (q, r)))
        elif kind == 6:
            ops.append(C.Op("CZ", (q, r)))
        else:
            ops.append(C.Op("U", (q, r), matrix=fixed))
    return ops, a


def _refreshed_equals_oracle(n, plan, ops, seed):
    rng = np.random.default_rng(seed)
    v = rng.standard_normal(1 << n) + 1j * rng.standard_normal(1 << n)
    psi0 = np.ascontiguousarray(v / np.linalg.norm(v))
    ref = oracle.simulate(n, ops, psi=psi0.copy())
    return np.max(np.abs(plan.emulate(psi0) - ref))


@pytest.mark.parametrize("seed", range(4))
@pytest.mark.parametrize("dtype", ["c64", "c128"])
def test_plan_refresh_reproduces_the_circuit_with_new_angles(seed, dtype):
    """A plan made from generic angles, refreshed with other angles, applies the circuit
    with those angles (FP64 oracle) and keeps its passes; the ansatz and a mix of
    rotations with fixed gates, under the default and several tile geometries."""
    n, L = 10, 4
    tmpl = C.hea(n, L, ring=True)
    for opts in ({}, {"tile_qubits": 7, "low_qubits": 3}, {"kmax": 3}, {"commute": -1}):
        plan = qsv.Plan(n, dtype, C.bind(tmpl, C.hea_params(n, L, seed=100 + seed)), **opts)
        passes = plan.stats()["passes"]
        for s2 in range(2):
            ops = C.bind(tmpl, C.hea_params(n, L, seed=200 + 10 * seed + s2))
            plan.refresh(ops)
            assert plan.stats()["passes"] == passes
            assert _refreshed_equals_oracle(n, plan, ops, seed) < 1e-12, opts
    rng = np.random.default_rng(300 + seed)
    ops, na = _rotation_mix(9, 120, rng)
    plan = qsv.Plan(9, dtype, ops, tile_qubits=7, low_qubits=2)
    for s2 in range(2):
        new_ops, _ = _rotation_mix(9, 120, np.random.default_rng(300 + seed),
                                   angles=np.random.default_rng(400 + s2).uniform(-np.pi, np.pi, na))
        plan.refresh(new_ops)
        assert _refreshed_equals_oracle(9, plan, new_ops, seed) < 1e-12


@pytest.mark.parametrize("special", [0.0, np.pi / 2, np.pi, -np.pi])
def test_plan_refresh_with_special_angles_is_exact_or_refused(special):
    """Angles of 0 or multiples of pi/2 give rotations extra structure (identity,
    diagonal, permutation).  Refreshing a generic plan with them must still be exact;
    a plan made from them may be refused for generic angles, but never be wrong."""
    n = 9
    rng = np.random.default_rng(5)
    ops, na = _rotation_mix(n, 100, rng)
    generic = np.random.default_rng(6).uniform(-np.pi, np.pi, na)
    sp = np.where(np.arange(na) % 3 == 0, special, generic)
    sp_ops, _ = _rotation_mix(n, 100, np.random.default_rng(5), angles=sp)
    gen_ops, _ = _rotation_mix(n, 100, np.random.default_rng(5), angles=generic)
    for dtype in ("c64", "c128"):
        plan = qsv.Plan(n, dtype, gen_ops)
        plan.refresh(sp_ops)
        assert _refreshed_equals_oracle(n, plan, sp_ops, 1) < 1e-12
        plan = qsv.Plan(n, dtype, sp_ops)
        try:
            plan.refresh(gen_ops)
        except qsv.QSVError as e:
            assert e.status == 4   # QSV_E_UNSUPPORTED: plan again
        else:
            assert _refreshed_equals_oracle(n, plan, gen_ops, 1) < 1e-12


def test_plan_refresh_refuses_what_it_cannot_refresh():
    n = 6
    base = [C.Op("H", (0,)), C.Op("RZ", (1,), (0.3,)), C.Op("RZ", (2,), (0.4,)), C.Op("CNOT", (0, 3))]
    plan = qsv.Plan(n, "c128", base)
    assert plan.stats()["diag_ops"] == 1            # RZ(1) and RZ(2) merged
    # a diagonal op would become dense: refused, and the plan is left as it was
    with pytest.raises(qsv.QSVError) as e:
        plan.refresh([base[0], C.Op("RX", (1,), (0.3,)), base[2], base[3]])
    assert e.value.status == 4
    assert _refreshed_equals_oracle(n, plan, base, 2) < 1e-12
    # another shape (targets or gate count): an argument error
    with pytest.raises(qsv.QSVError) as e:
        plan.refresh([base[0], C.Op("RZ", (4,), (0.3,)), base[2], base[3]])
    assert e.value.status == 1
    with pytest.raises(qsv.QSVError) as e:
        plan.refresh(base[:3])
    assert e.value.status == 1
    # a plan that dropped an identity product cannot be refreshed
    ident = qsv.Plan(n, "c64", [C.Op("X", (3,)), C.Op("X", (3,)), C.Op("H", (1,))])
    with pytest.raises(qsv.QSVError) as e:
        ident.refresh([C.Op("X", (3,)), C.Op("Y", (3,)), C.Op("H", (1,))])
    assert e.value.status == 4


def _is_permutation(m):
    nz = np.abs(m) > 0
    return bool(np.all(nz.sum(axis=0) == 1) and np.all(nz.sum(axis=1) == 1))


@pytest.mark.parametrize("dtype", ["c64", "c128"])
def test_matrix_core_ops_fit_each_pass_operand_block(dtype):
    # every 3- and 4-qubit dense op of a pass fits the pass's LDS operand block, so none
    # falls back to the VALU; priced at three quarters, 4-qubit ops are what the fusion
    # mostly makes on a brickwork
    n = 24
    ops = C.brickwork(n, 20, 3)
    plan = qsv.Plan(n, dtype, ops)
    st = plan.stats()
    fused = plan.fused_gates()
    dense = [len(q) for q, m, diag in fused if not diag and not _is_permutation(m)]
    assert st["mfma_ops"] == sum(1 for k in dense if k in (3, 4))
    assert sum(1 for k in dense if k == 4) > sum(1 for k in dense if k == 3)
    per = 2 if dtype == "c64" else 4
    block = 2048 if dtype == "c64" else 4096
    for idx, _ in plan.passes():
        used = 0
        for i in idx:
            q, m, diag = fused[i]
            if not diag and not _is_permutation(m) and len(q) in (3, 4):
                used = ((used + 3) & ~3) + per * 4 ** len(q)
        assert used <= block
