"""Seeded synthetic circuit generators: the inputs shared by the oracle and the GPU path.

This module produces circuit *descriptions* only: gate names from the canonical gate
set of the paper's Section 3 (Eq. 4), qubit tuples, rotation angles, and, for Haar
random single-qubit gates, the raw 2x2 unitary drawn from the seed (the paper's
Section 8.1 workload of random U(2) gates).  It holds none of the simulation
arithmetic: each consumer builds gate matrices from the names with its own code.

Conventions
-----------
* Qubit t is bit t of the amplitude index (qubit 0 is the least significant bit),
  as in the paper's Eq. 2 and Eq. 3.
* A multi-qubit gate ``Op(name, (q0, q1, ...))`` orders its local basis index with
  bit j <-> ``qubits[j]``.  CNOT(c, t) is ``Op("CNOT", (c, t))``, CZ is symmetric.
* Parametric rotations carry ``param`` = index into a parameter vector; their
  ``params`` tuple holds the bound angle.
* Noise channels (density-matrix runs) are ops too: ``Op("DEPOLARIZE", qubits, (p,))``
  (1 or 2 qubits: every non-identity Pauli string with probability p / (4^k - 1)) and
  ``Op("AMPDAMP", (q,), (gamma,))``.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence, Tuple

import numpy as np

__all__ = [
    "Op", "haar_u2", "haar_unitary", "brickwork", "brickwork_arrays", "ghz", "hea", "hea_params", "qft", "random_1q",
    "tfim_terms", "zz_chain_terms", "x_sum_terms", "bind", "inverse_ops",
    "serving_stream", "Request", "with_depolarizing", "CHANNELS", "h_t_cz_bricks", "commuting_mix",
]

CHANNELS = ("DEPOLARIZE", "AMPDAMP")


@dataclasses.dataclass(frozen=True)
class Op:
    name: str                      # canonical gate name (Eq. 4) or "U" for a raw unitary
    qubits: Tuple[int, ...]
    params: Tuple[float, ...] = ()
    matrix: Optional[np.ndarray] = None   # only for name == "U" (complex128, 2^k x 2^k)
    param: Optional[int] = None           # index into a parameter vector (rotations)


def haar_u2(rng: np.random.Generator, count: Optional[int] = None) -> np.ndarray:
    """Haar-random U(2): QR of a complex Gaussian 2x2 (entries (N(0,1) + i N(0,1))/sqrt 2)
    with the phases of R's diagonal moved into Q (Mezzadri's correction, without which
    plain QR is not Haar).  count=None gives one matrix; otherwise an array of `count`
    matrices whose Gaussians are drawn as one (count, 2, 2, 2) block ordered
    (matrix, real/imaginary part, row, column)."""
    c = 1 if count is None else count
    z = rng.standard_normal((c, 2, 2, 2))
    z = (z[:, 0] + 1j * z[:, 1]) / math.sqrt(2.0)
    q, r = np.linalg.qr(z)
    d = np.diagonal(r, axis1=1, axis2=2)
    q = q * (d / np.abs(d))[:, np.newaxis, :]
    q = np.ascontiguousarray(q, dtype=np.complex128)
    return q[0] if count is None else q


def brickwork(n: int, depth: int, seed: int) -> List[Op]:
    """Random brickwork: every layer puts a Haar U(2) on each qubit (ascending; one
    (n, 2, 2, 2) Gaussian block per layer), then CNOT(2i, 2i+1) on even layers and
    CNOT(2i+1, 2i+2) on odd layers (control = lower qubit).  Gate count =
    depth*n + sum of pairs per layer (290 at n=10, depth 20)."""
    rng = np.random.default_rng(seed)
    ops: List[Op] = []
    for layer in range(depth):
        us = haar_u2(rng, n)
        for q in range(n):
            ops.append(Op("U", (q,), matrix=us[q]))
        start = layer % 2
        for c in range(start, n - 1, 2):
            ops.append(Op("CNOT", (c, c + 1)))
    return ops


def brickwork_arrays(n: int, depth: int, seed: int):
    """The circuit of ``brickwork(n, depth, seed)`` as arrays (same draws, same order), for
    marshalling many circuits quickly: ``code`` per gate (0 = raw unitary, 1 = CNOT),
    ``targets`` (gates x 2, -1 padded), ``k`` (1 or 2), and the raw unitaries in order
    (u x 2 x 2 complex128)."""
    rng = np.random.default_rng(seed)
    codes, ks, tg, mats = [], [], [], []
    for layer in range(depth):
        mats.append(haar_u2(rng, n))
        codes += [0] * n
        ks += [1] * n
        tg += [(q, -1) for q in range(n)]
        start = layer % 2
        for c in range(start, n - 1, 2):
            codes.append(1)
            ks.append(2)
            tg.append((c, c + 1))
    return {"code": np.array(codes, dtype=np.int8), "k": np.array(ks, dtype=np.int32),
            "targets": np.array(tg, dtype=np.int32).reshape(-1, 2),
            "unitaries": np.concatenate(mats) if mats else np.zeros((0, 2, 2), complex)}


def ghz(n: int) -> List[Op]:
    """H on qubit 0 then a CNOT chain (i, i+1): the GHZ state (the paper's Section 9.1)."""
    ops = [Op("H", (0,))]
    for i in range(n - 1):
        ops.append(Op("CNOT", (i, i + 1)))
    return ops


def hea(n: int, layers: int, ring: bool = False, entangle: bool = True) -> List[Op]:
    """Hardware-efficient ansatz template: per layer RY(theta) then RZ(phi) on every
    qubit, then a CZ ladder (i, i+1) for i < n-1 (plus CZ(n-1, 0) when ``ring``).
    Parameter order: layer -> qubit -> (theta, phi); 2*n*layers parameters.
    Angles are unbound (params=()); use :func:`bind`."""
    ops: List[Op] = []
    p = 0
    for _ in range(layers):
        for q in range(n):
            ops.append(Op("RY", (q,), param=p))
            ops.append(Op("RZ", (q,), param=p + 1))
            p += 2
        if entangle:
            for i in range(n - 1):
                ops.append(Op("CZ", (i, i + 1)))
            if ring and n > 2:
                ops.append(Op("CZ", (n - 1, 0)))
    return ops


def hea_params(n: int, layers: int, seed: int, batch: Optional[int] = None) -> np.ndarray:
    """Angles uniform in [0, 2*pi) drawn in the order layer -> qubit -> (theta, phi)."""
    rng = np.random.default_rng(seed)
    shape = (2 * n * layers,) if batch is None else (batch, 2 * n * layers)
    return rng.uniform(0.0, 2.0 * math.pi, size=shape)


def bind(ops: Sequence[Op], params: Sequence[float]) -> List[Op]:
    """Fill each parametric op's angle from ``params[op.param]``."""
    out = []
    for op in ops:
        if op.param is not None:
            out.append(dataclasses.replace(op, params=(float(params[op.param]),)))
        else:
            out.append(op)
    return out


def qft(n: int) -> List[Op]:
    """Textbook QFT without the final qubit reversal: for j = n-1 .. 0, H(j) then
    controlled phases CP(pi/2^(j-k)) for k < j.  n + n(n-1)/2 gates (210 at n=20).
    CP has no entry in Eq. 4, so it is emitted as its raw diagonal unitary."""
    ops: List[Op] = []
    for j in range(n - 1, -1, -1):
        ops.append(Op("H", (j,)))
        for k in range(j - 1, -1, -1):
            lam = math.pi / (2 ** (j - k))
            m = np.diag([1.0, 1.0, 1.0, complex(math.cos(lam), math.sin(lam))]).astype(np.complex128)
            ops.append(Op("U", (k, j), matrix=m))
    return ops


def random_1q(n: int, seed: int, gates_per_qubit: int = 10) -> List[Op]:
    """The paper's Section 8.1 workload: 10n Haar U(2) gates, each on a uniformly chosen qubit."""
    rng = np.random.default_rng(seed)
    ops = []
    for _ in range(gates_per_qubit * n):
        q = int(rng.integers(0, n))
        ops.append(Op("U", (q,), matrix=haar_u2(rng)))
    return ops


def h_t_cz_bricks(n: int, depth: int, seed: int) -> List[Op]:
    """Layers of H or T on every qubit (a coin flip each) followed by CZ bricks (2i, 2i+1)
    on even layers and (2i+1, 2i+2) on odd ones.  T and CZ are diagonal, so long stretches
    of the circuit commute although they share qubits."""
    rng = np.random.default_rng(seed)
    ops: List[Op] = []
    for layer in range(depth):
        for q in range(n):
            ops.append(Op("T" if rng.random() < 0.5 else "H", (q,)))
        for q in range(layer % 2, n - 1, 2):
            ops.append(Op("CZ", (q, q + 1)))
    return ops


def haar_unitary(rng: np.random.Generator, d: int) -> np.ndarray:
    """A Haar-random d x d unitary: QR of a complex Gaussian with Mezzadri's phase fix."""
    z = rng.standard_normal((d, d)) + 1j * rng.standard_normal((d, d))
    q, r = np.linalg.qr(z)
    return q * (np.diag(r) / np.abs(np.diag(r)))


_haar = haar_unitary


def commuting_mix(n: int, count: int, seed: int) -> List[Op]:
    """Random gates many of which are diagonal on some of their qubits: random phases on
    1-3 qubits (20%), CZ / CNOT / TOFFOLI on random qubits (40%), controlled Haar
    unitaries on 2-3 qubits with the control on local bit 0 (15%), Haar U(2) / U(4)
    (25%).  Ops of the first three kinds commute whenever each shared qubit is a phase
    or control qubit of both."""
    rng = np.random.default_rng(seed)
    ops: List[Op] = []
    for _ in range(count):
        r = rng.random()
        if r < 0.2:
            k = int(rng.integers(1, 4))
            qs = tuple(int(q) for q in rng.permutation(n)[:k])
            ops.append(Op("U", qs, matrix=np.diag(np.exp(1j * rng.uniform(0, 2 * math.pi, 1 << k)))))
        elif r < 0.6:
            name, k = [("CZ", 2), ("CNOT", 2), ("TOFFOLI", 3)][int(rng.integers(0, 3))]
            ops.append(Op(name, tuple(int(q) for q in rng.permutation(n)[:k])))
        elif r < 0.75:
            k = int(rng.integers(2, 4))
            qs = tuple(int(q) for q in rng.permutation(n)[:k])
            u = _haar(rng, 1 << (k - 1))
            m = np.zeros((1 << k, 1 << k), complex)
            m[0::2, 0::2] = np.eye(1 << (k - 1))   # control (local bit 0) clear: identity
            m[1::2, 1::2] = u                       # control set: u on the other targets
            ops.append(Op("U", qs, matrix=m))
        else:
            k = int(rng.integers(1, 3))
            ops.append(Op("U", tuple(int(q) for q in rng.permutation(n)[:k]), matrix=_haar(rng, 1 << k)))
    return ops


def inverse_ops(ops: Sequence[Op]) -> List[Op]:
    """The inverse circuit as raw data: reversed order, each named gate replaced by its
    named inverse where one exists, raw unitaries by their conjugate transpose."""
    inv = {"H": "H", "X": "X", "Y": "Y", "Z": "Z", "CNOT": "CNOT", "CZ": "CZ",
           "SWAP": "SWAP", "TOFFOLI": "TOFFOLI", "I": "I", "S": "SDG", "SDG": "S",
           "T": "TDG", "TDG": "T"}
    out = []
    for op in reversed(list(ops)):
        if op.name == "U":
            out.append(Op("U", op.qubits, matrix=np.ascontiguousarray(op.matrix.conj().T)))
        elif op.name in ("RX", "RY", "RZ"):
            out.append(Op(op.name, op.qubits, params=(-op.params[0],)))
        elif op.name == "U3":
            th, ph, lam = op.params
            out.append(Op("U3", op.qubits, params=(-th, -lam, -ph)))
        else:
            out.append(Op(inv[op.name], op.qubits))
    return out


# ---------------------------------------------------------------- observables
# A Pauli term is (coeff, ((qubit, 'X'|'Y'|'Z'), ...)).

def with_depolarizing(ops: Sequence[Op], p1: float, p2: float) -> List[Op]:
    """The circuit with a depolarizing channel after every gate: probability p1 on the
    target of each 1-qubit gate, p2 on the pair of each 2-qubit gate (the noise model of
    the Bell / GHZ noise study)."""
    out: List[Op] = []
    for op in ops:
        out.append(op)
        if len(op.qubits) == 1 and p1 > 0:
            out.append(Op("DEPOLARIZE", op.qubits, (p1,)))
        elif len(op.qubits) == 2 and p2 > 0:
            out.append(Op("DEPOLARIZE", op.qubits, (p2,)))
    return out


def zz_chain_terms(n: int, periodic: bool = False, coeff: float = 1.0):
    terms = [(coeff, ((i, "Z"), (i + 1, "Z"))) for i in range(n - 1)]
    if periodic and n > 2:
        terms.append((coeff, ((n - 1, "Z"), (0, "Z"))))
    return terms


def x_sum_terms(n: int, coeff: float = 1.0):
    return [(coeff, ((i, "X"),)) for i in range(n)]


def tfim_terms(n: int, h: float = 0.7):
    """Transverse-field Ising H = -sum Z_i Z_{i+1 mod n} - h sum X_i (periodic)."""
    return zz_chain_terms(n, periodic=True, coeff=-1.0) + x_sum_terms(n, coeff=-h)


# ---------------------------------------------------------------- serving stream

@dataclasses.dataclass(frozen=True)
class Request:
    rid: int
    arrival_s: float
    n: int
    depth: int
    dtype: str          # "c64" or "c128"
    seed: int


def serving_stream(count: int = 4096, seed: int = 5, rate_hz: float = 200.0,
                   n_lo: int = 12, n_hi: int = 26, d_lo: int = 10, d_hi: int = 60,
                   p_c64: float = 0.7) -> List[Request]:
    """Open-loop request stream: qubits uniform in [n_lo, n_hi], brickwork depth uniform
    in [d_lo, d_hi], complex64 with probability p_c64, Poisson arrivals at rate_hz.
    Each request's circuit is ``brickwork(n, depth, seed)`` with its own seed."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate_hz, size=count)
    t = np.cumsum(gaps) - gaps[0]
    ns = rng.integers(n_lo, n_hi + 1, size=count)
    ds = rng.integers(d_lo, d_hi + 1, size=count)
    c64 = rng.random(size=count) < p_c64
    seeds = rng.integers(0, 2 ** 31 - 1, size=count)
    return [Request(i, float(t[i]), int(ns[i]), int(ds[i]), "c64" if c64[i] else "c128",
                    int(seeds[i])) for i in range(count)]
