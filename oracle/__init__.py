"""FP64 CPU oracle for the state-vector hot path -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  The GPU library never loads it, and it shares
no code with the GPU library: the two meet only through the seeded circuit
descriptions of ``paper_2604_03816_amd.circuits``.

The arithmetic lives in ``qsv_oracle.c`` (plain C99 double complex, gate by gate,
no fusion).  This module marshals numpy arrays to it and adds the plain
definitions that sit on top:

* ``simulate``            -- Eq. 10: U_m ... U_1 |0...0>, one gate at a time (Eq. 2/3)
* ``fidelity``            -- the Table 3 fidelity |<psi_ref|psi>|^2
* ``param_shift_grad``    -- exact gradient of exp(-i theta P/2) rotations
                              (the parameter-shift rule the paper's PennyLane path uses,
                              Section 7.4), evaluated with ``simulate`` + ``expval``
* ``fd_grad``             -- central finite differences
* ``dm_simulate``         -- density matrix of a circuit with noise channels (Kraus
                              operators; depolarizing and amplitude damping), dense
* ``sample``              -- computational-basis measurement sampling by inverse
                              transform of the Born probabilities (Eq. 1), the
                              backend's third operation (Section 4)
"""
from __future__ import annotations

import ctypes
import math
import os
from typing import Iterable, List, Sequence, Tuple

import numpy as np

from . import build as _build

_LIB = None


def lib():
    global _LIB
    if _LIB is None:
        path = _build.LIB
        if not os.path.exists(path):
            _build.build()
        L = ctypes.CDLL(path)
        c_p = ctypes.c_void_p
        L.or_init_zero.argtypes = [c_p, ctypes.c_int]
        L.or_apply.argtypes = [c_p, ctypes.c_int, ctypes.c_int, c_p, c_p]
        L.or_gate_matrix.argtypes = [ctypes.c_char_p, c_p, c_p, c_p]
        L.or_norm2.argtypes = [c_p, ctypes.c_int]
        L.or_norm2.restype = ctypes.c_double
        L.or_probs.argtypes = [c_p, ctypes.c_int, c_p, ctypes.c_int, c_p]
        L.or_pauli_expval.argtypes = [c_p, ctypes.c_int, ctypes.c_int, c_p, ctypes.c_char_p, c_p, c_p]
        L.or_inner.argtypes = [c_p, c_p, ctypes.c_int, c_p, c_p]
        L.or_num_threads.restype = ctypes.c_int
        _LIB = L
    return _LIB


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _nq(psi: np.ndarray) -> int:
    n = int(psi.size).bit_length() - 1
    if psi.dtype != np.complex128 or (1 << n) != psi.size or not psi.flags.c_contiguous:
        raise ValueError("oracle states are C-contiguous complex128 arrays of length 2^n")
    return n


def num_threads() -> int:
    return int(lib().or_num_threads())


# ------------------------------------------------------------------ gates (Eq. 4)

def gate_matrix(name: str, params: Sequence[float] = ()) -> np.ndarray:
    out = np.zeros(64, dtype=np.complex128)
    p = np.zeros(4, dtype=np.float64)
    p[: len(params)] = params
    k = ctypes.c_int(0)
    if lib().or_gate_matrix(name.encode(), _ptr(p), ctypes.byref(k), _ptr(out)) != 0:
        raise ValueError("unknown gate %r" % name)
    d = 1 << k.value
    return out[: d * d].reshape(d, d).copy()


def op_matrix(op) -> np.ndarray:
    if op.name == "U":
        return np.ascontiguousarray(op.matrix, dtype=np.complex128)
    return gate_matrix(op.name, op.params)


# ------------------------------------------------------------------ states

def zero_state(n: int) -> np.ndarray:
    psi = np.empty(1 << n, dtype=np.complex128)
    if lib().or_init_zero(_ptr(psi), n) != 0:
        raise ValueError("bad qubit count")
    return psi


def apply(psi: np.ndarray, U: np.ndarray, targets: Sequence[int]) -> None:
    n = _nq(psi)
    U = np.ascontiguousarray(U, dtype=np.complex128)
    t = np.ascontiguousarray(targets, dtype=np.int32)
    if U.shape != (1 << len(t), 1 << len(t)):
        raise ValueError("matrix shape does not match the target count")
    if lib().or_apply(_ptr(psi), n, len(t), _ptr(t), _ptr(U)) != 0:
        raise ValueError("bad targets %r" % (tuple(targets),))


def simulate(n: int, ops: Iterable, psi: np.ndarray = None) -> np.ndarray:
    """Eq. 10: apply the gates one at a time, in circuit order, to |0...0> (or psi)."""
    if psi is None:
        psi = zero_state(n)
    for op in ops:
        apply(psi, op_matrix(op), op.qubits)
    return psi


# ------------------------------------------------------------------ reductions

def norm2(psi: np.ndarray) -> float:
    return float(lib().or_norm2(_ptr(psi), _nq(psi)))


def probs(psi: np.ndarray, qubits: Sequence[int] = None) -> np.ndarray:
    n = _nq(psi)
    if qubits is None:
        qubits = list(range(n))
    q = np.ascontiguousarray(qubits, dtype=np.int32)
    out = np.empty(1 << len(q), dtype=np.float64)
    if lib().or_probs(_ptr(psi), n, _ptr(q), len(q), _ptr(out)) != 0:
        raise ValueError("bad qubits")
    return out


def sample(psi: np.ndarray, qubits: Sequence[int], uniforms: np.ndarray) -> np.ndarray:
    """Outcomes of measuring ``qubits`` (bit j of an outcome <-> qubits[j]), one per
    uniform u in [0, 1): the smallest k with u * P < p_0 + ... + p_k, where p is the
    marginal Born distribution over ``qubits`` and P its total (so an unnormalised
    state is sampled from its normalised distribution).  The running sum is plain
    sequential FP64; an outcome of probability zero is never returned."""
    p = probs(psi, qubits)
    c = np.cumsum(p)
    u = np.asarray(uniforms, dtype=np.float64)
    if np.any(u < 0) or np.any(u >= 1):
        raise ValueError("uniforms must lie in [0, 1)")
    k = np.searchsorted(c, u * c[-1], side="right")
    return np.minimum(k, np.flatnonzero(p)[-1]).astype(np.int64)


def pauli_expval(psi: np.ndarray, string: Sequence[Tuple[int, str]]) -> complex:
    """<psi|P|psi> for one Pauli string ((qubit, 'X'|'Y'|'Z'|'I'), ...)."""
    n = _nq(psi)
    q = np.ascontiguousarray([s[0] for s in string], dtype=np.int32)
    p = "".join(s[1] for s in string).encode()
    re, im = ctypes.c_double(), ctypes.c_double()
    if lib().or_pauli_expval(_ptr(psi), n, len(q), _ptr(q), p, ctypes.byref(re), ctypes.byref(im)) != 0:
        raise ValueError("bad Pauli string %r" % (string,))
    return complex(re.value, im.value)


def expval_terms(psi: np.ndarray, terms) -> np.ndarray:
    """Per-term coeff * Re<psi|P|psi> for terms (coeff, ((qubit, pauli), ...))."""
    return np.array([c * pauli_expval(psi, s).real for c, s in terms], dtype=np.float64)


def expval(psi: np.ndarray, terms) -> float:
    return float(math.fsum(expval_terms(psi, terms)))


def inner(a: np.ndarray, b: np.ndarray) -> complex:
    n = _nq(a)
    if _nq(b) != n:
        raise ValueError("size mismatch")
    re, im = ctypes.c_double(), ctypes.c_double()
    lib().or_inner(_ptr(a), _ptr(b), n, ctypes.byref(re), ctypes.byref(im))
    return complex(re.value, im.value)


def fidelity(ref: np.ndarray, psi: np.ndarray) -> float:
    """|<ref|psi>|^2 with psi taken as given (not renormalised), Table 3's definition."""
    psi = np.ascontiguousarray(psi, dtype=np.complex128)
    return abs(inner(ref, psi)) ** 2


def max_abs_diff(ref: np.ndarray, psi: np.ndarray) -> float:
    return float(np.max(np.abs(ref - np.asarray(psi, dtype=np.complex128))))


# ------------------------------------------------------------------ gradients

def energy(n: int, template, params: Sequence[float], terms) -> float:
    from paper_2604_03816_amd.circuits import bind
    return expval(simulate(n, bind(template, params)), terms)


def param_shift_grad(n: int, template, params: Sequence[float], terms) -> np.ndarray:
    """dE/dtheta_j = [E(theta + pi/2 e_j) - E(theta - pi/2 e_j)] / 2, exact for gates
    exp(-i theta P / 2) with P a Pauli operator when theta_j enters one gate only."""
    used = [op.param for op in template if op.param is not None]
    if len(used) != len(set(used)):
        raise ValueError("parameter-shift here assumes each parameter enters one gate")
    params = np.asarray(params, dtype=np.float64)
    g = np.zeros_like(params)
    for j in used:
        e = np.zeros_like(params)
        e[j] = math.pi / 2
        g[j] = 0.5 * (energy(n, template, params + e, terms) - energy(n, template, params - e, terms))
    return g


def fd_grad(n: int, template, params: Sequence[float], terms, h: float = 1e-6,
            which: Sequence[int] = None) -> np.ndarray:
    """Central differences [E(theta + h e_j) - E(theta - h e_j)] / (2h)."""
    params = np.asarray(params, dtype=np.float64)
    idx = range(len(params)) if which is None else which
    g = np.full_like(params, np.nan)
    for j in idx:
        e = np.zeros_like(params)
        e[j] = h
        g[j] = (energy(n, template, params + e, terms) - energy(n, template, params - e, terms)) / (2 * h)
    return g


# ------------------------------------------------------------------ density matrices

_PAULI = {"I": np.eye(2, dtype=complex), "X": np.array([[0, 1], [1, 0]], dtype=complex),
          "Y": np.array([[0, -1j], [1j, 0]]), "Z": np.array([[1, 0], [0, -1]], dtype=complex)}


def kraus_ops(op) -> List[np.ndarray]:
    """Kraus operators of an op on its own qubits (local bit j <-> op.qubits[j]): a gate
    is its single unitary; DEPOLARIZE(p) on k qubits is sqrt(1-p) I plus every
    non-identity Pauli string times sqrt(p / (4^k - 1)); AMPDAMP(gamma) is
    [[1, 0], [0, sqrt(1-gamma)]] and [[0, sqrt(gamma)], [0, 0]]."""
    if op.name == "DEPOLARIZE":
        k, p = len(op.qubits), float(op.params[0])
        strings = [""]
        for _ in range(k):
            strings = [s + c for s in strings for c in "IXYZ"]
        out = []
        for s in strings:
            m = np.ones((1, 1), dtype=complex)
            for c in s:                       # first letter = local bit 0 (rightmost factor)
                m = np.kron(_PAULI[c], m)
            w = 1.0 - p if set(s) == {"I"} else p / (4 ** k - 1)
            out.append(math.sqrt(w) * m)
        return out
    if op.name == "AMPDAMP":
        g = float(op.params[0])
        return [np.array([[1, 0], [0, math.sqrt(1 - g)]], dtype=complex),
                np.array([[0, math.sqrt(g)], [0, 0]], dtype=complex)]
    return [op_matrix(op)]


def _embed(n: int, M: np.ndarray, targets: Sequence[int]) -> np.ndarray:
    """The 2^n x 2^n operator of M on `targets` (identity elsewhere), column by column
    through the gate-by-gate ``apply`` (which does not assume unitarity)."""
    N = 1 << n
    full = np.zeros((N, N), dtype=complex)
    for j in range(N):
        e = np.zeros(N, dtype=complex)
        e[j] = 1.0
        apply(e, M, targets)
        full[:, j] = e
    return full


def dm_simulate(n: int, ops: Iterable, rho: np.ndarray = None) -> np.ndarray:
    """rho -> sum_a K_a rho K_a^dagger for every op in order, from |0...0><0...0|."""
    N = 1 << n
    if rho is None:
        rho = np.zeros((N, N), dtype=complex)
        rho[0, 0] = 1.0
    for op in ops:
        ks = [_embed(n, K, op.qubits) for K in kraus_ops(op)]
        rho = sum(K @ rho @ K.conj().T for K in ks)
    return rho


def dm_probs(rho: np.ndarray, qubits: Sequence[int]) -> np.ndarray:
    """Marginal of the diagonal over `qubits` (bit j of the outcome <-> qubits[j])."""
    n = int(rho.shape[0]).bit_length() - 1
    d = np.real(np.diag(rho))
    out = np.zeros(1 << len(qubits))
    for k in range(1 << n):
        o = sum(((k >> q) & 1) << j for j, q in enumerate(qubits))
        out[o] += d[k]
    return out


def dm_expval(rho: np.ndarray, terms) -> float:
    """sum_t coeff_t Tr(rho P_t), P_t as a dense Kronecker product."""
    n = int(rho.shape[0]).bit_length() - 1
    tot = 0.0
    for c, string in terms:
        letters = ["I"] * n
        for q, p in string:
            letters[q] = p
        P = np.ones((1, 1), dtype=complex)
        for q in range(n):
            P = np.kron(_PAULI[letters[q]], P)
        tot += c * float(np.real(np.trace(rho @ P)))
    return tot


def classical_fidelity(p: np.ndarray, q: np.ndarray) -> float:
    """(sum_x sqrt(p(x) q(x)))^2 (the noise study's F_cl)."""
    return float(np.sum(np.sqrt(np.clip(p, 0, None) * np.clip(q, 0, None))) ** 2)


def tvd(p: np.ndarray, q: np.ndarray) -> float:
    """Total variation distance (1/2) sum_x |p(x) - q(x)|."""
    return float(0.5 * np.sum(np.abs(p - q)))

