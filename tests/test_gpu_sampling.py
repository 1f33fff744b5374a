"""GPU parity of measurement sampling (qsv_sample) against the oracle's inverse-transform
sampler on the same state and the same uniforms.  Outcomes are integers decided by FP64
sums taken in different orders (sequential in the oracle, per-chunk scans on the GPU),
so an outcome must be *valid* for every shot (probability > 0 and u * P inside its
cumulative interval, up to rounding) and must equal the oracle's wherever u * P is not
within rounding of an interval boundary."""
import numpy as np
import pytest

import oracle
from paper_2604_03816_amd import circuits as C

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def qsv():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    from paper_2604_03816_amd import qsv as q
    q.lib()
    return q


def check_against_oracle(psi, qubits, u, got):
    """psi: the device state copied to the host (complex128), so both sides sample the
    same distribution.  Returns the fraction of shots equal to the oracle's."""
    n = int(np.log2(psi.size))
    qs = list(range(n)) if qubits is None else list(qubits)
    p = oracle.probs(psi, qs)
    c = np.cumsum(p)
    t = u * c[-1]
    tol = 1e-12 * c[-1]
    assert np.all(p[got] > 0), "an outcome of probability zero was drawn"
    assert np.all(t >= c[got] - p[got] - tol) and np.all(t < c[got] + tol), "outcome outside its interval"
    want = oracle.sample(psi, qs, u)
    # distance from u * P to the nearest cumulative boundary
    b = np.concatenate(([0.0], c))
    i = np.clip(np.searchsorted(b, t), 1, len(b) - 1)
    near = np.minimum(np.abs(t - b[i - 1]), np.abs(t - b[i])) < tol
    assert np.all((got == want) | near)
    return float(np.mean(got == want))


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_ghz_closed_form(qsv, dtype):
    n = 20
    s = qsv.State(n, dtype)
    s.apply(C.ghz(n))
    u = np.array([0.0, 0.1, 0.3, 0.4999, 0.5001, 0.7, 0.9999])
    got = s.sample(u)
    assert got.tolist() == [0, 0, 0, 0, (1 << n) - 1, (1 << n) - 1, (1 << n) - 1]
    # marginal over three qubits: 000 or 111
    assert set(s.sample(np.linspace(0, 0.999, 200), [19, 3, 7]).tolist()) == {0, 7}
    s.free()


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("n", [9, 14, 17])
def test_random_states_full_and_marginal(qsv, dtype, n):
    rng = np.random.default_rng(40 + n)
    s = qsv.State(n, dtype)
    s.apply(C.brickwork(n, 8, 50 + n))
    psi = s.get().astype(np.complex128)
    u = rng.random(4000)
    match = check_against_oracle(psi, None, u, s.sample(u))
    assert match > 0.999
    for qubits in ([n - 1, 2, 5], list(range(n))[::-1], [0], [3, 1]):
        match = check_against_oracle(psi, qubits, u, s.sample(u, qubits))
        assert match > 0.999
    s.free()


def test_basis_state_many_chunks_and_sorted_order(qsv):
    # |k> with k deep inside the state: every chunk but one is empty; shots in any order
    n = 21
    k = 0b101100111000101011101
    s = qsv.State(n, "c128")
    ops = [C.Op("X", (q,)) for q in range(n) if (k >> q) & 1]
    s.apply(ops)
    u = np.random.default_rng(3).random(1000)
    assert np.all(s.sample(u) == k)
    assert np.all(s.sample(u, [4, 0, 20]) == ((k >> 4) & 1) | ((k & 1) << 1) | (((k >> 20) & 1) << 2))
    s.free()


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_repeated_uniforms_zero_and_top(qsv, dtype):
    """The shot order comes from a sort of the uniforms: repeated values, 0.0, -0.0 and
    the largest double below 1 in shuffled positions must give the oracle's outcomes."""
    n = 13
    s = qsv.State(n, dtype)
    s.apply(C.brickwork(n, 5, 21))
    psi = s.get().astype(np.complex128)
    base = np.random.default_rng(5).random(300)
    u = np.concatenate([base, base[::-1], base[:50], [0.0, -0.0, 0.0, -0.0], np.full(3, np.nextafter(1.0, 0.0))])
    np.random.default_rng(6).shuffle(u)
    got = s.sample(u)
    assert check_against_oracle(psi, None, u, got) > 0.999
    assert np.all(got[u == 0.0] == got[np.flatnonzero(u == 0.0)[0]])
    marg = [12, 0, 7]
    assert check_against_oracle(psi, marg, u, s.sample(u, marg)) > 0.999
    s.free()


@pytest.mark.parametrize("shots", [1, 2, 3, 257])
def test_few_shots_and_single_runs(qsv, shots):
    """The device groups sorted shots into runs of one chunk: one shot, a few shots in
    one or several chunks, and all shots in one chunk (a basis state) against the oracle."""
    n = 18
    s = qsv.State(n, "c128")
    s.apply(C.brickwork(n, 4, 30))
    psi = s.get()
    u = np.random.default_rng(40 + shots).random(shots)
    assert check_against_oracle(psi, None, u, s.sample(u)) == 1.0
    assert check_against_oracle(psi, [17, 2], u, s.sample(u, [17, 2])) == 1.0
    z = np.zeros(1 << n, complex)
    z[12345] = 1.0
    s.set(z)
    assert np.all(s.sample(u) == 12345)
    s.free()


def test_frequencies_match_probabilities(qsv):
    n = 12
    s = qsv.State(n, "c64")
    s.apply(C.brickwork(n, 6, 77))
    p = s.probs().astype(np.float64)
    p /= p.sum()
    shots = 400000
    got = s.sample(np.random.default_rng(9).random(shots))
    freq = np.bincount(got, minlength=1 << n) / shots
    top = np.argsort(p)[-20:]
    sigma = np.sqrt(p[top] * (1 - p[top]) / shots)
    assert np.all(np.abs(freq[top] - p[top]) < 5 * sigma)
    s.free()


def test_argument_errors(qsv):
    s = qsv.State(10, "c64")
    with pytest.raises(qsv.QSVError):
        s.sample(np.array([1.0]))
    with pytest.raises(qsv.QSVError):
        s.sample(np.array([-0.1]))
    with pytest.raises(qsv.QSVError):
        s.sample(np.array([0.5]), [1, 1])
    with pytest.raises(qsv.QSVError):
        s.sample(np.array([0.5]), [10])
    assert s.sample(np.zeros(0)).size == 0
    s.free()
