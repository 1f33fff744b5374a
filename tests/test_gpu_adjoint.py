"""Adjoint-method gradients (libqsv, through the C ABI) against the FP64 oracle's exact
parameter-shift gradient and central finite differences.  Relative error is
||g - g_ref||_2 / ||g_ref||_2 per parameter vector: <= 1e-6 (complex128), <= 1e-3 (complex64)."""
import numpy as np
import pytest

import oracle
from paper_2604_03816_amd import circuits as C

pytestmark = pytest.mark.gpu
REL = {"c128": 1e-6, "c64": 1e-3}


@pytest.fixture(scope="module")
def qsv():
    import torch
    assert torch.cuda.is_available()
    from paper_2604_03816_amd import qsv as q
    q.lib()
    return q


def rel(g, ref):
    return float(np.linalg.norm(g - ref) / np.linalg.norm(ref))


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_hea_tfim_12q_matches_parameter_shift(qsv, dtype):
    n, layers = 12, 8
    tpl = C.hea(n, layers, ring=True)
    terms = C.tfim_terms(n)
    params = C.hea_params(n, layers, seed=6, batch=2)
    E, G = qsv.adjoint_grad(n, tpl, params, terms, dtype)
    for b in range(2):
        e_ref = oracle.energy(n, tpl, params[b], terms)
        g_ref = oracle.param_shift_grad(n, tpl, params[b], terms)
        assert abs(E[b] - e_ref) <= (1e-12 if dtype == "c128" else 1e-4) * max(1.0, abs(e_ref))
        assert rel(G[b], g_ref) <= REL[dtype], rel(G[b], g_ref)


def test_special_angles_and_many_vectors(qsv):
    """Vectors with angles of 0 and multiples of pi/2 (rotations become the identity,
    diagonal or permutations) among generic ones, more vectors than the sweep keeps in
    flight: every gradient against the oracle's parameter shift."""
    n, layers = 8, 3
    tpl = C.hea(n, layers, ring=True)
    terms = C.tfim_terms(n)
    params = C.hea_params(n, layers, seed=21, batch=5)
    params[1][:] = 0.0
    params[2][::2] = np.pi / 2
    params[3][1::3] = np.pi
    E, G = qsv.adjoint_grad(n, tpl, params, terms, "c128")
    for b in range(5):
        e_ref = oracle.energy(n, tpl, params[b], terms)
        g_ref = oracle.param_shift_grad(n, tpl, params[b], terms)
        assert abs(E[b] - e_ref) <= 1e-12 * max(1.0, abs(e_ref)), b
        assert np.max(np.abs(G[b] - g_ref)) <= 1e-10, b


def test_24q_complex64_against_complex128_and_finite_differences(qsv):
    """At the gradient workload's size (24 qubits, 8 layers, 384 parameters, TFIM):
    complex64 gradients within 1e-3 relative error of complex128 ones, and complex128
    against central differences (h = 1e-6, FP64 energies) on a few parameters."""
    n, layers = 24, 8
    tpl = C.hea(n, layers, ring=True)
    terms = C.tfim_terms(n)
    params = C.hea_params(n, layers, seed=6, batch=2)
    E128, G128 = qsv.adjoint_grad(n, tpl, params, terms, "c128")
    E64, G64 = qsv.adjoint_grad(n, tpl, params, terms, "c64")
    for b in range(2):
        assert rel(G64[b], G128[b]) <= REL["c64"], rel(G64[b], G128[b])
        assert abs(E64[b] - E128[b]) <= 1e-4 * max(1.0, abs(E128[b]))
    h = 1e-6
    for j in (0, 191, 383):
        p = params[0].copy()
        p[j] += h
        ep, _ = qsv.adjoint_grad(n, tpl, p, terms, "c128")
        p[j] -= 2 * h
        em, _ = qsv.adjoint_grad(n, tpl, p, terms, "c128")
        assert abs(G128[0][j] - (ep - em) / (2 * h)) <= 1e-7


def test_finite_differences_small_circuit(qsv):
    """Central differences at h = 1e-6 in FP64 (truncation O(h^2), rounding ~1e-10)."""
    n, layers = 6, 3
    tpl = C.hea(n, layers, ring=True)
    terms = C.tfim_terms(n)
    params = C.hea_params(n, layers, seed=19)
    _, G = qsv.adjoint_grad(n, tpl, params, terms, "c128")
    fd = oracle.fd_grad(n, tpl, params, terms, h=1e-6)
    assert np.max(np.abs(G - fd)) <= 1e-7


def test_mixed_rotations_fixed_gates_and_shared_parameters(qsv):
    """RX/RY/RZ on repeated qubits (layers split), fixed gates between them, a parameter
    used by two gates (gradients accumulate), one parameter unused (zero), Y terms."""
    rng = np.random.default_rng(4)
    n = 7
    tpl = [C.Op("H", (0,)), C.Op("RX", (0,), param=0), C.Op("RY", (0,), param=1), C.Op("CNOT", (0, 3)),
           C.Op("RZ", (3,), param=2), C.Op("RX", (5,), param=3), C.Op("RY", (6,), param=0),
           C.Op("U", (2, 5), matrix=np.linalg.qr(rng.standard_normal((4, 4)) + 1j * rng.standard_normal((4, 4)))[0]),
           C.Op("RY", (2,), param=4), C.Op("RZ", (2,), param=5), C.Op("TOFFOLI", (1, 2, 4)), C.Op("RX", (4,), param=6)]
    P = 8
    terms = [(0.5, ((0, "Y"), (4, "Z"))), (-1.0, ((2, "X"), (5, "Y"))), (0.3, ((6, "Z"),)), (0.8, ((3, "X"),))]
    params = rng.uniform(0, 2 * np.pi, size=P)
    E, G = qsv.adjoint_grad(n, tpl, params, terms, "c128")
    assert abs(E - oracle.energy(n, tpl, params, terms)) <= 1e-12
    fd = oracle.fd_grad(n, tpl, params, terms, h=1e-6)
    assert np.max(np.abs(G - fd)) <= 1e-7
    assert G[7] == 0.0


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_generators_under_rz_and_layer_orders(qsv, dtype):
    """Layers evaluated before the previous layer's RZ rotations are undone (X and Y
    generators conjugated by them, and RZ generators that commute with them), next to
    layers that cannot be (an RY after the rotation on its qubit, fixed gates between
    layers): every order against the oracle's parameter shift, in both precisions."""
    n = 8
    tpl, p = [], 0
    for rep in range(3):
        for q in range(n):   # X and Y generators, then RZ on most qubits
            tpl.append(C.Op("RX" if q % 2 else "RY", (q,), param=p)); p += 1
        for q in range(n - 1):
            tpl.append(C.Op("RZ", (q,), param=p)); p += 1
        if rep == 1:         # an RY after an RZ on one qubit, RZ after RZ on another
            tpl.append(C.Op("RY", (2,), param=p)); p += 1
            tpl.append(C.Op("RZ", (3,), param=p)); p += 1
        for q in range(0, n - 1, 2):
            tpl.append(C.Op("CZ", (q, q + 1)))
        if rep == 0:         # a fixed gate with nothing after it but rotations
            tpl.append(C.Op("H", (n - 1,)))
    terms = C.tfim_terms(n)
    params = np.random.default_rng(17).uniform(-np.pi, np.pi, size=(2, p))
    E, G = qsv.adjoint_grad(n, tpl, params, terms, dtype)
    for b in range(2):
        e_ref = oracle.energy(n, tpl, params[b], terms)
        g_ref = oracle.param_shift_grad(n, tpl, params[b], terms)
        assert abs(E[b] - e_ref) <= (1e-12 if dtype == "c128" else 1e-4) * max(1.0, abs(e_ref))
        assert rel(G[b], g_ref) <= REL[dtype], rel(G[b], g_ref)


def test_autograd_function(qsv):
    import torch
    from paper_2604_03816_amd.autograd import AdjointExpval
    n, layers = 8, 2
    tpl = C.hea(n, layers, ring=True)
    terms = C.tfim_terms(n)
    p = torch.tensor(C.hea_params(n, layers, seed=2, batch=3), dtype=torch.float64, requires_grad=True)
    E = AdjointExpval.apply(p, n, tpl, terms, "c128")
    w = torch.tensor([1.0, -2.0, 0.5], dtype=torch.float64)
    (E * w).sum().backward()
    for b in range(3):
        g_ref = oracle.param_shift_grad(n, tpl, p.detach().numpy()[b], terms)
        assert np.max(np.abs(p.grad.numpy()[b] - w[b].item() * g_ref)) <= 1e-10


def test_argument_errors(qsv):
    tpl = [C.Op("RY", (0,), param=3)]
    with pytest.raises(qsv.QSVError):
        qsv.adjoint_grad(2, tpl, np.zeros(2), [(1.0, ((0, "Z"),))])   # param index out of range
    with pytest.raises(qsv.QSVError):
        qsv.adjoint_grad(2, [C.Op("RY", (5,), param=0)], np.zeros(1), [(1.0, ((0, "Z"),))])
    with pytest.raises(ValueError):
        qsv.OpList([C.Op("H", (0,), param=0)])
