"""Pins for the FP64 oracle: each check compares it with something other than itself
(a library routine, a closed form, an invariant, or a value the paper prints), so that
a dropped term, a wrong sign, a wrong bit order or a transposed operand fails here."""
import json
import math
import os

import numpy as np
import pytest
import scipy.linalg

import oracle
from paper_2604_03816_amd import circuits as C

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")
PX = np.array([[0, 1], [1, 0]], dtype=complex)
PY = np.array([[0, -1j], [1j, 0]], dtype=complex)
PZ = np.array([[1, 0], [0, -1]], dtype=complex)
PAULI = {"X": PX, "Y": PY, "Z": PZ, "I": np.eye(2, dtype=complex)}


def golden(key):
    with open(GOLDEN) as f:
        return json.load(f)[key]["value"]


def rand_state(n, rng):
    v = rng.standard_normal(1 << n) + 1j * rng.standard_normal(1 << n)
    return np.ascontiguousarray(v / np.linalg.norm(v))


def rand_unitary(d, rng):
    z = rng.standard_normal((d, d)) + 1j * rng.standard_normal((d, d))
    q, r = np.linalg.qr(z)
    return q * (np.diag(r) / np.abs(np.diag(r)))


# ------------------------------------------------------------------ gate set (Eq. 4)

@pytest.mark.parametrize("name,P", [("RX", PX), ("RY", PY), ("RZ", PZ)])
def test_rotations_are_matrix_exponentials(name, P):
    for th in (0.0, 0.3, -1.7, 2.5, math.pi, 5.9):
        ref = scipy.linalg.expm(-0.5j * th * P)
        assert np.allclose(oracle.gate_matrix(name, (th,)), ref, atol=1e-14)


def test_single_qubit_identities():
    g = oracle.gate_matrix
    I2 = np.eye(2)
    assert np.allclose(g("H") @ g("H"), I2, atol=1e-15)
    assert np.allclose(g("S") @ g("S"), g("Z"), atol=1e-15)
    assert np.allclose(g("T") @ g("T"), g("S"), atol=1e-15)
    assert np.allclose(g("S") @ g("SDG"), I2, atol=1e-15)
    assert np.allclose(g("T") @ g("TDG"), I2, atol=1e-15)
    # Pauli algebra: XY = iZ, YZ = iX, ZX = iY; H X H = Z
    assert np.allclose(g("X") @ g("Y"), 1j * g("Z"))
    assert np.allclose(g("Y") @ g("Z"), 1j * g("X"))
    assert np.allclose(g("Z") @ g("X"), 1j * g("Y"))
    assert np.allclose(g("H") @ g("X") @ g("H"), g("Z"), atol=1e-15)
    # X, Y, Z equal i * R_P(pi) (rotation by pi is -i P)
    for name in "XYZ":
        assert np.allclose(1j * g("R" + name, (math.pi,)), g(name), atol=1e-15)


def test_u3_is_zyz_euler_rotation():
    g = oracle.gate_matrix
    rng = np.random.default_rng(11)
    for _ in range(20):
        th, ph, lam = rng.uniform(-7, 7, size=3)
        zyz = g("RZ", (ph,)) @ g("RY", (th,)) @ g("RZ", (lam,))
        assert np.allclose(g("U3", (th, ph, lam)), np.exp(0.5j * (ph + lam)) * zyz, atol=1e-14)


def _basis_action(name, nq, inp):
    """Run the oracle on basis state |inp> and return the unique output index and amplitude."""
    psi = oracle.zero_state(nq)
    for q in range(nq):
        if (inp >> q) & 1:
            oracle.apply(psi, PX, (q,))
    oracle.apply(psi, oracle.gate_matrix(name), tuple(range(nq)))
    nz = np.flatnonzero(np.abs(psi) > 1e-12)
    assert len(nz) == 1
    return int(nz[0]), psi[nz[0]]


def test_two_and_three_qubit_gates_by_truth_table():
    # CNOT(c=qubit0, t=qubit1): flips qubit 1 when qubit 0 is set
    assert [_basis_action("CNOT", 2, i)[0] for i in range(4)] == [0, 3, 2, 1]
    # SWAP exchanges the bits
    assert [_basis_action("SWAP", 2, i)[0] for i in range(4)] == [0, 2, 1, 3]
    # CZ: phase -1 on |11> only
    amps = [_basis_action("CZ", 2, i)[1] for i in range(4)]
    assert np.allclose(amps, [1, 1, 1, -1])
    # Toffoli(c1=0, c2=1, t=2)
    outs = [_basis_action("TOFFOLI", 3, i)[0] for i in range(8)]
    assert outs == [0, 1, 2, 7, 4, 5, 6, 3]


# ------------------------------------------------------------------ apply (Eq. 2, Eq. 3)

@pytest.mark.parametrize("n", [1, 2, 3, 5, 7])
def test_single_target_matches_kronecker_embedding(n):
    """Eq. 3: |psi'> = (I_{2^{n-t-1}} (x) U (x) I_{2^t}) |psi>, for every target t."""
    rng = np.random.default_rng(100 + n)
    for t in range(n):
        U = rand_unitary(2, rng)
        psi = rand_state(n, rng)
        ref = np.kron(np.kron(np.eye(1 << (n - t - 1)), U), np.eye(1 << t)) @ psi
        out = psi.copy()
        oracle.apply(out, U, (t,))
        assert np.max(np.abs(out - ref)) < 1e-13


def _tensordot_apply(psi, U, targets, n):
    """Independent route: reshape psi to a rank-n tensor (axis a <-> qubit n-1-a) and
    contract U's column indices with the target axes via numpy.tensordot."""
    k = len(targets)
    T = psi.reshape((2,) * n)
    Ut = U.reshape((2,) * (2 * k))          # row bits (k-1 .. 0), then column bits (k-1 .. 0)
    axes_psi = [n - 1 - targets[j] for j in reversed(range(k))]
    out = np.tensordot(Ut, T, axes=(list(range(k, 2 * k)), axes_psi))
    out = np.moveaxis(out, list(range(k)), axes_psi)
    return out.reshape(-1)


@pytest.mark.parametrize("k", [2, 3, 4, 5])
def test_multi_target_matches_tensordot(k):
    rng = np.random.default_rng(200 + k)
    for n in (k, k + 1, 8):
        for _ in range(4):
            targets = tuple(int(x) for x in rng.permutation(n)[:k])
            U = rand_unitary(1 << k, rng)
            psi = rand_state(n, rng)
            out = psi.copy()
            oracle.apply(out, U, targets)
            ref = _tensordot_apply(psi, U, targets, n)
            assert np.max(np.abs(out - ref)) < 1e-13, (n, targets)


def test_adjacent_two_qubit_gate_matches_kron():
    """CNOT(c=t, t=t+1) equals I (x) CNOT_{4x4 in (t+1, t) order} (x) I."""
    rng = np.random.default_rng(7)
    n = 6
    U = rand_unitary(4, rng)
    for t in range(n - 1):
        psi = rand_state(n, rng)
        ref = np.kron(np.kron(np.eye(1 << (n - t - 2)), U), np.eye(1 << t)) @ psi
        out = psi.copy()
        oracle.apply(out, U, (t, t + 1))
        assert np.max(np.abs(out - ref)) < 1e-13


def test_rejects_bad_targets():
    psi = oracle.zero_state(3)
    with pytest.raises(ValueError):
        oracle.apply(psi, np.eye(4), (1, 1))
    with pytest.raises(ValueError):
        oracle.apply(psi, np.eye(2), (3,))


# ------------------------------------------------------------------ closed forms

def test_ghz_amplitudes_and_probs():
    amp = golden("ghz_amplitude")
    for n in range(2, 13):
        psi = oracle.simulate(n, C.ghz(n))
        assert abs(psi[0] - amp) < 1e-15 and abs(psi[-1] - amp) < 1e-15
        rest = psi.copy()
        rest[0] = rest[-1] = 0
        assert np.max(np.abs(rest)) == 0.0
        ex = dict((k, v) for k, v in golden("bell_ideal_probs").items())
        if n == 2:
            p = oracle.probs(psi)
            assert np.allclose(p, [ex["00"], ex["10"], ex["01"], ex["11"]], atol=1e-15)
        # <Z_i Z_j> = 1, <X_i> = 0, <X^n> = 1
        assert abs(oracle.pauli_expval(psi, ((0, "Z"), (n - 1, "Z"))) - 1) < 1e-14
        assert abs(oracle.pauli_expval(psi, ((n // 2, "X"),))) < 1e-14
        assert abs(oracle.pauli_expval(psi, tuple((q, "X") for q in range(n))) - 1) < 1e-14


def test_qft_is_the_discrete_fourier_transform():
    """QFT|x> = N^{-1/2} sum_y exp(2 pi i x y / N)|y>; the generator omits the final
    qubit reversal, so output index y appears bit-reversed.  Reference: numpy.fft."""
    n = 6
    N = 1 << n
    ops = C.qft(n)
    assert len(ops) == n + n * (n - 1) // 2
    rev = np.array([int(format(y, "0%db" % n)[::-1], 2) for y in range(N)])
    for x in (0, 1, 5, 37, 63):
        psi = np.zeros(N, dtype=complex)
        psi[x] = 1
        out = oracle.simulate(n, ops, psi=psi)
        e = np.zeros(N)
        e[x] = 1
        dft = np.fft.ifft(e) * math.sqrt(N)          # (1/sqrt N) sum_y e^{+2 pi i x y/N}
        assert np.max(np.abs(out[rev] - dft)) < 1e-13, x


def test_product_state_closed_form():
    """HEA without entanglers: every qubit carries R = prod RZ(phi) RY(theta) |0>, computed
    here with scipy's expm; <Z_q>, <X_q> and <Z_q Z_q+1> = <Z_q><Z_q+1> follow."""
    n, layers = 6, 3
    tpl = C.hea(n, layers, entangle=False)
    params = C.hea_params(n, layers, seed=3)
    psi = oracle.simulate(n, C.bind(tpl, params))
    zs, xs = [], []
    for q in range(n):
        v = np.array([1, 0], dtype=complex)
        for l in range(layers):
            th, ph = params[2 * (l * n + q)], params[2 * (l * n + q) + 1]
            v = scipy.linalg.expm(-0.5j * ph * PZ) @ (scipy.linalg.expm(-0.5j * th * PY) @ v)
        zs.append((v.conj() @ PZ @ v).real)
        xs.append((v.conj() @ PX @ v).real)
    for q in range(n):
        assert abs(oracle.pauli_expval(psi, ((q, "Z"),)).real - zs[q]) < 1e-13
        assert abs(oracle.pauli_expval(psi, ((q, "X"),)).real - xs[q]) < 1e-13
    for q in range(n - 1):
        assert abs(oracle.pauli_expval(psi, ((q, "Z"), (q + 1, "Z"))).real - zs[q] * zs[q + 1]) < 1e-13


# ------------------------------------------------------------------ invariants

def test_norm_preserved_and_inverse_returns_to_zero():
    n = 10
    ops = C.brickwork(n, 20, seed=1)
    psi = oracle.simulate(n, ops)
    assert abs(oracle.norm2(psi) - 1) < 1e-13
    back = oracle.simulate(n, C.inverse_ops(ops), psi=psi.copy())
    e0 = np.zeros(1 << n, dtype=complex)
    e0[0] = 1
    assert np.max(np.abs(back - e0)) < 1e-12
    # named-gate inverses too (HEA with rotations and CZ)
    tpl = C.bind(C.hea(7, 3, ring=True), C.hea_params(7, 3, seed=9))
    psi = oracle.simulate(7, tpl)
    back = oracle.simulate(7, C.inverse_ops(tpl), psi=psi)
    assert abs(back[0] - 1) < 1e-13 and np.max(np.abs(back[1:])) < 1e-13


def test_norm_against_numpy():
    rng = np.random.default_rng(5)
    v = rng.standard_normal(1 << 12) + 1j * rng.standard_normal(1 << 12)
    assert abs(oracle.norm2(np.ascontiguousarray(v)) - np.vdot(v, v).real) < 1e-9


# ------------------------------------------------------------------ probs / expval

def test_marginal_probs_against_numpy_reshape():
    rng = np.random.default_rng(21)
    n = 7
    psi = rand_state(n, rng)
    P = (np.abs(psi) ** 2).reshape((2,) * n)      # axis a <-> qubit n-1-a
    for qubits in [(0,), (6,), (2, 5), (5, 2), (1, 4, 0), tuple(range(n)), (6, 0, 3, 1)]:
        keep = [n - 1 - q for q in qubits]
        drop = tuple(a for a in range(n) if a not in keep)
        M = P.sum(axis=drop)                            # remaining axes in ascending axis order
        order = sorted(keep)
        M = np.moveaxis(M, [order.index(a) for a in keep], range(len(keep)))
        # M[b_{q0}, b_{q1}, ...]; output index o = sum_j b_{qj} 2^j
        ref = M.transpose(list(reversed(range(len(keep))))).reshape(-1)
        assert np.allclose(oracle.probs(psi, qubits), ref, atol=1e-15), qubits


def _dense_pauli(n, string):
    ops = {q: p for q, p in string}
    M = np.array([[1.0 + 0j]])
    for q in reversed(range(n)):                  # kron(sigma_{n-1}, ..., sigma_0)
        M = np.kron(M, PAULI[ops.get(q, "I")])
    return M


def test_pauli_expval_against_dense_matrices():
    rng = np.random.default_rng(33)
    n = 6
    for _ in range(40):
        psi = rand_state(n, rng)
        nq = int(rng.integers(1, n + 1))
        qs = rng.permutation(n)[:nq]
        string = tuple((int(q), "XYZ"[int(rng.integers(0, 3))]) for q in qs)
        ref = np.vdot(psi, _dense_pauli(n, string) @ psi)
        got = oracle.pauli_expval(psi, string)
        assert abs(got - ref) < 1e-13, string


def test_fidelity_definition():
    rng = np.random.default_rng(4)
    a = rand_state(8, rng)
    assert abs(oracle.fidelity(a, a) - 1) < 1e-14
    assert abs(oracle.fidelity(a, np.exp(0.7j) * a) - 1) < 1e-14
    b = rand_state(8, rng)
    b -= np.vdot(a, b) * a
    assert oracle.fidelity(a, np.ascontiguousarray(b)) < 1e-28
    assert abs(oracle.fidelity(a, 0.5 * a) - 0.25) < 1e-14


# ------------------------------------------------------------------ gradients

def test_gradient_closed_form_single_rotation():
    """E(theta) = <0|RY(theta)^dag Z RY(theta)|0> = cos(theta); dE/dtheta = -sin(theta)."""
    tpl = [C.Op("RY", (0,), param=0)]
    terms = [(1.0, ((0, "Z"),))]
    for th in (0.1, 1.3, 2.9, 4.4):
        assert abs(oracle.energy(1, tpl, [th], terms) - math.cos(th)) < 1e-15
        g = oracle.param_shift_grad(1, tpl, [th], terms)
        assert abs(g[0] + math.sin(th)) < 1e-14


def test_param_shift_matches_finite_differences():
    n, layers = 4, 2
    tpl = C.hea(n, layers, ring=True)
    terms = C.tfim_terms(n)
    params = C.hea_params(n, layers, seed=6)
    ps = oracle.param_shift_grad(n, tpl, params, terms)
    fd = oracle.fd_grad(n, tpl, params, terms, h=1e-6)
    assert np.max(np.abs(ps - fd)) < 1e-8


# ------------------------------------------------------------------ generators

def test_generator_counts_and_unitarity():
    assert len(C.brickwork(10, 20, 1)) == 290
    assert len(C.brickwork(28, 20, 2)) == 830
    assert len(C.brickwork(30, 20, 3)) == 890
    assert len(C.qft(20)) == golden("qft20_gate_count")
    assert len(C.hea_params(24, 8, seed=6)) == 384
    ops = C.brickwork(6, 3, 42)
    for op in ops:
        if op.name == "U":
            assert np.allclose(op.matrix.conj().T @ op.matrix, np.eye(2), atol=1e-14)
    # deterministic in the seed
    a, b = C.brickwork(5, 4, 9), C.brickwork(5, 4, 9)
    assert all(np.array_equal(x.matrix, y.matrix) for x, y in zip(a, b) if x.name == "U")


def test_memory_arithmetic_from_the_paper():
    """Section 1 and Section 6: 2^n * 16 bytes; 24 GiB holds 30 (c128) / 31 (c64) qubits."""
    gib = 2 ** 30
    assert (2 ** 30) * 16 // gib == golden("state_bytes_30q_c128_gib")
    assert (2 ** 28) * 16 // gib == golden("state_bytes_28q_c128_gib")
    assert int(math.floor(math.log2(24 * gib / 16))) == golden("max_qubits_24gib_c128")
    assert int(math.floor(math.log2(24 * gib / 8))) == golden("max_qubits_24gib_c64")


# ------------------------------------------------------------------ sampling (Eq. 1 Born rule)

def test_sampling_ghz_closed_form():
    n = 5
    psi = oracle.simulate(n, C.ghz(n))
    u = np.array([0.0, 0.25, 0.49, 0.51, 0.75, 0.999999])
    assert list(oracle.sample(psi, range(n), u)) == [0, 0, 0, 31, 31, 31]
    # marginal over two qubits of GHZ: outcomes 00 or 11 only
    assert set(oracle.sample(psi, [3, 1], np.linspace(0, 0.99, 50)).tolist()) == {0, 3}


def test_sampling_brute_force_inverse_cdf():
    rng = np.random.default_rng(11)
    n = 4
    v = rng.standard_normal(1 << n) + 1j * rng.standard_normal(1 << n)
    v[5] = 0   # a zero-probability outcome is never drawn
    psi = np.ascontiguousarray(v)   # deliberately unnormalised
    for qubits in ([0, 1, 2, 3], [2, 0], [3]):
        p = np.zeros(1 << len(qubits))
        for k in range(1 << n):
            o = sum(((k >> q) & 1) << j for j, q in enumerate(qubits))
            p[o] += abs(psi[k]) ** 2
        u = rng.random(500)
        got = oracle.sample(psi, qubits, u)
        for ui, g in zip(u, got):
            t, acc, want = ui * p.sum(), 0.0, None
            for k in range(len(p)):
                acc += p[k]
                if t < acc:
                    want = k
                    break
            assert want is not None and g == want and p[g] > 0
    with pytest.raises(ValueError):
        oracle.sample(psi, [0], np.array([1.0]))


def test_sampling_frequencies_and_bit_order():
    rng = np.random.default_rng(12)
    n = 4
    th = rng.uniform(0.2, 1.3, n)
    # product state: qubit q is cos(th_q)|0> + sin(th_q)|1>
    psi = np.ones(1)
    for q in range(n):
        psi = np.kron(np.array([np.cos(th[q]), np.sin(th[q])]), psi)
    psi = np.ascontiguousarray(psi.astype(np.complex128))
    qubits = [2, 0]
    p1 = {q: np.sin(th[q]) ** 2 for q in qubits}
    expect = np.array([(p1[2] if o & 1 else 1 - p1[2]) * (p1[0] if o & 2 else 1 - p1[0]) for o in range(4)])
    shots = 200000
    got = oracle.sample(psi, qubits, rng.random(shots))
    freq = np.bincount(got, minlength=4) / shots
    sigma = np.sqrt(expect * (1 - expect) / shots)
    assert np.all(np.abs(freq - expect) < 5 * sigma)


# ------------------------------------------------------------------ density matrices (Table 8)

def _ghz_depolarized(n, p):
    ops = [C.Op("H", (0,)), C.Op("DEPOLARIZE", (0,), (p,))]
    for t in range(1, n):
        ops += [C.Op("CNOT", (0, t)), C.Op("DEPOLARIZE", (0,), (p,)), C.Op("DEPOLARIZE", (t,), (p,))]
    return ops


def test_noise_study_matches_table8():
    """The exact (infinite-shot) F_cl and TVD of the noise study agree with the paper's
    MSLE column within its 8192-shot noise; a depolarizing convention of p/4 per Pauli
    instead of p/3 would be off by about 0.009 on average."""
    table = golden("noise_study_msle")
    devs = []
    for n in (2, 3, 4, 5):
        rho = oracle.dm_simulate(n, _ghz_depolarized(n, 0.01))
        pn = oracle.dm_probs(rho, list(range(n)))
        pi = np.zeros(1 << n)
        pi[0] = pi[-1] = 0.5
        F, T = oracle.classical_fidelity(pi, pn), oracle.tvd(pi, pn)
        want_F, want_T = table[str(n)]
        assert abs(F - want_F) < 0.006 and abs(T - want_T) < 0.006
        devs.append(abs(F - want_F))
    assert np.mean(devs) < 0.004


def test_depolarized_bell_closed_form():
    # H(0) depol(0), CNOT depol(0) depol(1): a bit flip (X or Y) with probability 2p/3 per
    # qubit on the final Bell pair; Z errors before the CNOT do not change Z outcomes
    for p in (0.0, 0.01, 0.2, 0.75):
        rho = oracle.dm_simulate(2, _ghz_depolarized(2, p))
        q = 2 * p / 3
        anti = 2 * q * (1 - q)
        probs = oracle.dm_probs(rho, [0, 1])
        assert np.allclose(probs, [(1 - anti) / 2, anti / 2, anti / 2, (1 - anti) / 2], atol=1e-14)
        # each depolarizing channel scales Bloch components by 1 - 4p/3
        zz = oracle.dm_expval(rho, [(1.0, ((0, "Z"), (1, "Z")))])
        assert abs(zz - (1 - 4 * p / 3) ** 2) < 1e-14


def test_density_matrix_invariants_and_special_cases():
    rng = np.random.default_rng(21)
    n = 3
    ops = C.random_1q(n, 5, gates_per_qubit=2) + [C.Op("CNOT", (0, 2)), C.Op("CZ", (1, 2))]
    # no noise: the pure state's projector
    psi = oracle.simulate(n, ops)
    assert np.allclose(oracle.dm_simulate(n, ops), np.outer(psi, psi.conj()), atol=1e-14)
    # random noise: unit trace, Hermitian, positive semidefinite
    noisy = []
    for op in ops:
        noisy.append(op)
        noisy.append(C.Op("DEPOLARIZE", op.qubits, (float(rng.uniform(0, 0.3)),)))
        noisy.append(C.Op("AMPDAMP", (op.qubits[0],), (float(rng.uniform(0, 0.3)),)))
    rho = oracle.dm_simulate(n, noisy)
    assert abs(np.trace(rho) - 1) < 1e-13
    assert np.allclose(rho, rho.conj().T, atol=1e-14)
    assert np.min(np.linalg.eigvalsh(rho)) > -1e-13
    # fully depolarizing channels give the maximally mixed state
    one = oracle.dm_simulate(1, [C.Op("H", (0,)), C.Op("DEPOLARIZE", (0,), (0.75,))])
    assert np.allclose(one, np.eye(2) / 2, atol=1e-15)
    two = oracle.dm_simulate(2, [C.Op("H", (0,)), C.Op("CNOT", (0, 1)), C.Op("DEPOLARIZE", (0, 1), (15 / 16,))])
    assert np.allclose(two, np.eye(4) / 4, atol=1e-15)
    # amplitude damping of |1>: population gamma moves to |0>
    g = 0.3
    ad = oracle.dm_simulate(1, [C.Op("X", (0,)), C.Op("AMPDAMP", (0,), (g,))])
    assert np.allclose(ad, np.diag([g, 1 - g]), atol=1e-15)
