"""ctypes binding of libqsv.so (include/qsv.h).  Argument marshalling only: every
step of the simulation runs inside the library (host planner + HIP kernels).

PyTorch supplies device memory and streams: a :class:`State` owns a torch tensor
of dtype complex64 / complex128 on a ROCm device and hands its data pointer and the
current torch stream to ``qsv_alloc``.  If libqsv.so has not been built the import
fails -- there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os
from typing import Iterable, List, Optional, Sequence, Tuple

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
# QSV_LIB selects another build of the library (the host-sanitizer build of the CPU tests)
LIB_PATH = os.environ.get("QSV_LIB") or os.path.join(HERE, "_build", "libqsv.so")

QSV_OK, QSV_E_ARG, QSV_E_OOM, QSV_E_DEVICE, QSV_E_UNSUPPORTED = 0, 1, 2, 3, 4
C64, C128, AUTO = 0, 1, 2
_DT = {"c64": C64, "c128": C128, "complex64": C64, "complex128": C128}
_DT_SERVE = dict(_DT, auto=AUTO)   # the server also takes "auto" (precision by Eq. 12)
_STATUS = {1: "QSV_E_ARG", 2: "QSV_E_OOM", 3: "QSV_E_DEVICE", 4: "QSV_E_UNSUPPORTED"}


class QSVError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__("%s: %s" % (_STATUS.get(status, str(status)), msg))
        self.status = status


class Gate(ctypes.Structure):
    _fields_ = [("k", ctypes.c_int), ("targets", ctypes.c_int * 5), ("diag", ctypes.c_int),
                ("mat", ctypes.POINTER(ctypes.c_double))]


class PlanOpts(ctypes.Structure):
    _fields_ = [("fuse", ctypes.c_int), ("kmax", ctypes.c_int), ("cost_aware", ctypes.c_int),
                ("tile_qubits", ctypes.c_int), ("low_qubits", ctypes.c_int),
                ("pass_budget", ctypes.c_double), ("matrix_cores", ctypes.c_int), ("commute", ctypes.c_int),
                ("op_cost", ctypes.c_double)]


class PlanStats(ctypes.Structure):
    _fields_ = [("gates_in", ctypes.c_size_t), ("fused_out", ctypes.c_size_t), ("passes", ctypes.c_size_t),
                ("dense_ops", ctypes.c_size_t), ("diag_ops", ctypes.c_size_t), ("perm_ops", ctypes.c_size_t),
                ("mfma_ops", ctypes.c_size_t), ("fma_per_amp", ctypes.c_double), ("hbm_bytes", ctypes.c_double),
                ("mfma_fma_per_amp", ctypes.c_double)]

    def as_dict(self):
        return {f[0]: getattr(self, f[0]) for f in self._fields_}


class DMOp(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int), ("k", ctypes.c_int), ("targets", ctypes.c_int * 5),
                ("mat", ctypes.POINTER(ctypes.c_double)), ("p", ctypes.c_double)]


class PauliTerm(ctypes.Structure):
    _fields_ = [("coeff", ctypes.c_double), ("n", ctypes.c_int), ("qubits", ctypes.POINTER(ctypes.c_int)),
                ("paulis", ctypes.c_char_p)]


class COp(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int), ("k", ctypes.c_int), ("targets", ctypes.c_int * 5),
                ("mat", ctypes.POINTER(ctypes.c_double)), ("param", ctypes.c_int)]


EXPORTS = [
    "qsv_last_error", "qsv_version", "qsv_alloc", "qsv_free", "qsv_reset", "qsv_info", "qsv_get_state",
    "qsv_set_state", "qsv_gate_matrix", "qsv_plan_create", "qsv_plan_free", "qsv_plan_get_stats",
    "qsv_plan_refresh", "qsv_plan_fused_gate", "qsv_plan_pass_info", "qsv_plan_pass_ops", "qsv_plan_emulate", "qsv_plan_apply",
    "qsv_plan_apply_range", "qsv_plan_apply_zero",
    "qsv_apply_fused", "qsv_sync", "qsv_norm", "qsv_norm_noalloc", "qsv_expval_pauli", "qsv_probs", "qsv_sample", "qsv_adjoint_grad",
    "qsv_dm_apply", "qsv_dm_probs", "qsv_dm_expval_pauli", "qsv_precision_select",
    "qsv_server_create", "qsv_server_free", "qsv_server_submit", "qsv_server_step", "qsv_server_results",
    "qsv_server_get_stats", "qsv_server_get_state", "qsv_server_release",
]

_LIB = None


def lib():
    """Load libqsv.so (raises if it has not been built)."""
    global _LIB
    if _LIB is not None:
        return _LIB
    if not os.path.exists(LIB_PATH):
        raise ImportError("libqsv.so is not built (%s); run paper_2604_03816_amd/build.py" % LIB_PATH)
    L = ctypes.CDLL(LIB_PATH)
    vp, i, sz, dp = ctypes.c_void_p, ctypes.c_int, ctypes.c_size_t, ctypes.POINTER(ctypes.c_double)
    L.qsv_last_error.restype = ctypes.c_char_p
    L.qsv_version.restype = ctypes.c_char_p
    L.qsv_alloc.argtypes = [i, i, vp, sz, vp, ctypes.POINTER(vp)]
    L.qsv_free.argtypes = [vp]
    L.qsv_reset.argtypes = [vp]
    L.qsv_info.argtypes = [vp, ctypes.POINTER(i), ctypes.POINTER(i), ctypes.POINTER(vp)]
    L.qsv_get_state.argtypes = [vp, vp]
    L.qsv_set_state.argtypes = [vp, vp]
    L.qsv_gate_matrix.argtypes = [ctypes.c_char_p, dp, ctypes.POINTER(i), dp]
    L.qsv_plan_create.argtypes = [i, i, ctypes.POINTER(Gate), sz, ctypes.POINTER(PlanOpts), ctypes.POINTER(vp)]
    L.qsv_plan_free.argtypes = [vp]
    L.qsv_plan_get_stats.argtypes = [vp, ctypes.POINTER(PlanStats)]
    L.qsv_plan_refresh.argtypes = [vp, ctypes.POINTER(Gate), sz]
    L.qsv_plan_fused_gate.argtypes = [vp, sz, ctypes.POINTER(i), ctypes.POINTER(i), ctypes.POINTER(i), dp]
    L.qsv_plan_pass_info.argtypes = [vp, sz, ctypes.POINTER(i), ctypes.POINTER(i), ctypes.POINTER(i)]
    L.qsv_plan_pass_ops.argtypes = [vp, sz, ctypes.POINTER(i)]
    L.qsv_plan_emulate.argtypes = [vp, dp]
    L.qsv_plan_apply.argtypes = [vp, vp]
    L.qsv_plan_apply_range.argtypes = [vp, vp, sz, sz]
    L.qsv_plan_apply_zero.argtypes = [vp, vp, sz]
    L.qsv_apply_fused.argtypes = [vp, ctypes.POINTER(Gate), sz, ctypes.POINTER(PlanOpts), ctypes.POINTER(PlanStats)]
    L.qsv_sync.argtypes = [vp]
    L.qsv_norm.argtypes = [vp, dp]
    L.qsv_norm_noalloc.argtypes = [vp, i, i, vp, vp]
    L.qsv_expval_pauli.argtypes = [vp, ctypes.POINTER(PauliTerm), sz, dp, dp]
    L.qsv_probs.argtypes = [vp, ctypes.POINTER(i), i, vp, i]
    L.qsv_precision_select.argtypes = [i, sz, ctypes.c_double, ctypes.POINTER(i)]
    L.qsv_dm_apply.argtypes = [vp, ctypes.POINTER(DMOp), sz, ctypes.POINTER(PlanOpts)]
    L.qsv_dm_probs.argtypes = [vp, ctypes.POINTER(i), i, ctypes.POINTER(ctypes.c_double)]
    L.qsv_dm_expval_pauli.argtypes = [vp, ctypes.POINTER(PauliTerm), sz, ctypes.POINTER(ctypes.c_double),
                                      ctypes.POINTER(ctypes.c_double)]
    L.qsv_sample.argtypes = [vp, ctypes.POINTER(i), i, ctypes.POINTER(ctypes.c_double), ctypes.c_longlong,
                             ctypes.POINTER(ctypes.c_longlong)]
    L.qsv_adjoint_grad.argtypes = [i, i, ctypes.POINTER(COp), sz, dp, i, i, ctypes.POINTER(PauliTerm), sz,
                                   dp, dp, vp]
    _LIB = L
    return L


def check(status: int) -> None:
    if status != QSV_OK:
        raise QSVError(status, lib().qsv_last_error().decode())


def version() -> str:
    return lib().qsv_version().decode()


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


# ------------------------------------------------------------------ gates

def gate_matrix(name: str, params: Sequence[float] = ()) -> np.ndarray:
    """The library's Eq. 4 gate matrix (complex128, 2^k x 2^k)."""
    p = np.zeros(4, dtype=np.float64)
    p[: len(params)] = params
    out = np.zeros(2 * 64, dtype=np.float64)
    k = ctypes.c_int(0)
    check(lib().qsv_gate_matrix(name.encode(), _dptr(p), ctypes.byref(k), _dptr(out)))
    d = 1 << k.value
    return out[: 2 * d * d].view(np.complex128).reshape(d, d).copy()


_NAMED_CACHE = {}


def _named(name, params):
    key = (name, tuple(float(x) for x in params))
    m = _NAMED_CACHE.get(key)
    if m is None:
        m = gate_matrix(name, params)
        if len(_NAMED_CACHE) < 4096:
            _NAMED_CACHE[key] = m
    return m


class GateList:
    """A circuit marshalled into a ctypes qsv_gate array; one float64 buffer holds
    every matrix (re, im interleaved)."""

    def __init__(self, ops: Iterable):
        ops = list(ops)
        self.n = len(ops)
        self.arr = (Gate * max(1, len(ops)))()
        mats = []
        ks = []
        for i, op in enumerate(ops):
            m = op.matrix if op.name == "U" else _named(op.name, op.params)
            k = len(op.qubits)
            if not 1 <= k <= 5:
                raise ValueError("op %d: a gate acts on 1 to 5 qubits, got %d" % (i, k))
            if m.shape != (1 << k, 1 << k):
                raise ValueError("op %d: matrix shape %s does not match %d targets" % (i, m.shape, k))
            mats.append(m.reshape(-1))
            ks.append(k)
        self._buf = np.ascontiguousarray(np.concatenate(mats) if mats else np.zeros(1, complex),
                                         dtype=np.complex128)
        base = self._buf.ctypes.data
        off = 0
        dp = ctypes.POINTER(ctypes.c_double)
        for i, op in enumerate(ops):
            g = self.arr[i]
            k = ks[i]
            g.k = k
            g.targets[:k] = op.qubits
            g.diag = 0
            g.mat = ctypes.cast(base + 16 * off, dp)
            off += 1 << (2 * k)


_GATE_DTYPE = np.dtype({"names": ["k", "targets", "diag", "mat"],
                        "formats": ["<i4", ("<i4", (5,)), "<i4", "<u8"],
                        "offsets": [0, 4, 24, 32], "itemsize": 40})
assert _GATE_DTYPE.itemsize == ctypes.sizeof(Gate)


class ArrayGateList:
    """A circuit given as arrays (see circuits.brickwork_arrays) marshalled into qsv_gate
    structs with numpy, without a Python loop over gates.  code 0 = raw unitary (taken
    in order from ``unitaries``), code 1 = CNOT (the library's Eq. 4 matrix)."""

    def __init__(self, arr):
        code, k, tg, us = arr["code"], arr["k"], arr["targets"], arr["unitaries"]
        G = len(code)
        self.n = G
        cnot = gate_matrix("CNOT").reshape(-1)
        self._buf = np.ascontiguousarray(np.concatenate([us.reshape(-1), cnot]), dtype=np.complex128)
        base = self._buf.ctypes.data
        cnot_addr = base + 16 * 4 * len(us)
        a = np.zeros(max(1, G), dtype=_GATE_DTYPE)
        a["k"][:G] = k
        t = np.zeros((max(1, G), 5), dtype=np.int32)
        t[:G, :2] = tg
        t[:G, 1][k == 1] = 0
        a["targets"] = t
        uidx = np.cumsum(code == 0) - 1
        addr = np.where(code == 0, base + 64 * uidx, cnot_addr).astype(np.uint64)
        a["mat"][:G] = addr
        self._arr = a
        self.arr = a.ctypes.data_as(ctypes.POINTER(Gate))


def _opts(fuse=True, kmax=0, cost_aware=0, tile_qubits=0, low_qubits=0, pass_budget=0.0,
          matrix_cores=0, commute=0, op_cost=0.0) -> PlanOpts:
    """fuse: True/1 DAG fusion, False/0 plain (one gate per pass), 2 = no fusion but
    gates share passes; matrix_cores: dense ops on >= this many targets use MFMA
    (0 default, -1 never); commute: commutation-aware DAG (0/1 default on, -1 off or
    False)."""
    o = PlanOpts()
    o.fuse = int(fuse) if not isinstance(fuse, bool) else (1 if fuse else 0)
    o.matrix_cores = matrix_cores
    o.commute = int(commute) if not isinstance(commute, bool) else (1 if commute else -1)
    o.kmax = kmax
    o.cost_aware = cost_aware
    o.tile_qubits = tile_qubits
    o.low_qubits = low_qubits
    o.pass_budget = pass_budget
    o.op_cost = op_cost
    return o


class Plan:
    """qsv_plan: fused + scheduled circuit for one (n, dtype)."""

    def __init__(self, n: int, dtype: str, ops: Iterable, **opts):
        self.n = n
        self.dtype = dtype
        gl = ops if isinstance(ops, (GateList, ArrayGateList)) else GateList(ops)
        h = ctypes.c_void_p()
        o = _opts(**opts)
        check(lib().qsv_plan_create(n, _DT[dtype], gl.arr, gl.n, ctypes.byref(o), ctypes.byref(h)))
        self.h = h

    def stats(self) -> dict:
        st = PlanStats()
        check(lib().qsv_plan_get_stats(self.h, ctypes.byref(st)))
        return st.as_dict()

    def refresh(self, ops: Iterable) -> None:
        """qsv_plan_refresh: the same circuit shape with new matrices (raises QSVError
        when the plan's structure does not hold for them)."""
        gl = ops if isinstance(ops, (GateList, ArrayGateList)) else GateList(ops)
        check(lib().qsv_plan_refresh(self.h, gl.arr, gl.n))

    def fused_gates(self) -> List[Tuple[Tuple[int, ...], np.ndarray, bool]]:
        out = []
        for i in range(self.stats()["fused_out"]):
            k, diag = ctypes.c_int(), ctypes.c_int()
            t = (ctypes.c_int * 5)()
            m = np.zeros(2 * 1024, dtype=np.float64)
            check(lib().qsv_plan_fused_gate(self.h, i, ctypes.byref(k), t, ctypes.byref(diag), _dptr(m)))
            d = 1 << k.value
            out.append((tuple(t[:k.value]), m[: 2 * d * d].view(np.complex128).reshape(d, d).copy(), bool(diag.value)))
        return out

    def passes(self) -> List[Tuple[Tuple[int, ...], Tuple[int, ...]]]:
        """Per pass: (fused-gate indices in application order, tile qubits)."""
        out = []
        for i in range(self.stats()["passes"]):
            nops, nact = ctypes.c_int(), ctypes.c_int()
            act = (ctypes.c_int * 40)()
            check(lib().qsv_plan_pass_info(self.h, i, ctypes.byref(nops), ctypes.byref(nact), act))
            idx = (ctypes.c_int * max(1, nops.value))()
            check(lib().qsv_plan_pass_ops(self.h, i, idx))
            out.append((tuple(idx[: nops.value]), tuple(act[: nact.value])))
        return out

    def emulate(self, psi: np.ndarray) -> np.ndarray:
        """Host re-enactment of the passes (FP64) on a copy of psi (complex128)."""
        out = np.ascontiguousarray(psi, dtype=np.complex128).copy()
        check(lib().qsv_plan_emulate(self.h, out.view(np.float64).ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
        return out

    def free(self):
        if getattr(self, "h", None):
            lib().qsv_plan_free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


# ------------------------------------------------------------------ observables

class TermList:
    def __init__(self, terms):
        terms = list(terms)
        self._keep = []
        self.arr = (PauliTerm * max(1, len(terms)))()
        self.n = len(terms)
        for i, (c, string) in enumerate(terms):
            q = (ctypes.c_int * max(1, len(string)))(*[int(s[0]) for s in string])
            p = ctypes.c_char_p("".join(s[1] for s in string).encode())
            self._keep += [q, p]
            t = self.arr[i]
            t.coeff = float(c)
            t.n = len(string)
            t.qubits = ctypes.cast(q, ctypes.POINTER(ctypes.c_int))
            t.paulis = p


# ------------------------------------------------------------------ states

class State:
    """A 2^n amplitude state in a torch tensor on a ROCm device, registered with libqsv.

    The state starts as |0...0>.  All device work runs on the torch stream that is
    current when the State is created (or the one passed in)."""

    def __init__(self, n: int, dtype: str = "c64", device: str = "cuda:0", stream=None):
        import torch
        self.n = n
        self.dtype = dtype
        tdt = torch.complex64 if _DT[dtype] == C64 else torch.complex128
        self.tensor = torch.empty(1 << n, dtype=tdt, device=device)
        with torch.cuda.device(self.tensor.device):
            s = stream if stream is not None else torch.cuda.current_stream(self.tensor.device)
            self.stream = s
            h = ctypes.c_void_p()
            check(lib().qsv_alloc(n, _DT[dtype], ctypes.c_void_p(self.tensor.data_ptr()),
                                  self.tensor.numel() * self.tensor.element_size(),
                                  ctypes.c_void_p(s.cuda_stream), ctypes.byref(h)))
        self.h = h

    # -- application
    def apply(self, ops, **opts) -> dict:
        gl = ops if isinstance(ops, (GateList, ArrayGateList)) else GateList(ops)
        st = PlanStats()
        o = _opts(**opts)
        check(lib().qsv_apply_fused(self.h, gl.arr, gl.n, ctypes.byref(o), ctypes.byref(st)))
        return st.as_dict()

    def apply_plan_zero(self, plan: Plan, count: int = None) -> None:
        """The first ``count`` passes (default all) applied to |0...0>, the initial state
        built inside the first pass (no separate reset)."""
        check(lib().qsv_plan_apply_zero(self.h, plan.h, plan.stats()["passes"] if count is None else count))

    def apply_plan(self, plan: Plan, first: int = None, count: int = None) -> None:
        if first is None:
            check(lib().qsv_plan_apply(self.h, plan.h))
        else:
            check(lib().qsv_plan_apply_range(self.h, plan.h, first, count))

    def reset(self):
        check(lib().qsv_reset(self.h))

    def sync(self):
        check(lib().qsv_sync(self.h))

    # -- data movement
    def get(self) -> np.ndarray:
        out = np.empty(1 << self.n, dtype=np.complex64 if _DT[self.dtype] == C64 else np.complex128)
        check(lib().qsv_get_state(self.h, out.ctypes.data_as(ctypes.c_void_p)))
        return out

    def set(self, host: np.ndarray) -> None:
        want = np.complex64 if _DT[self.dtype] == C64 else np.complex128
        a = np.ascontiguousarray(host, dtype=want)
        if a.size != 1 << self.n:
            raise ValueError("size mismatch")
        check(lib().qsv_set_state(self.h, a.ctypes.data_as(ctypes.c_void_p)))

    # -- reductions
    def norm(self) -> float:
        out = ctypes.c_double()
        check(lib().qsv_norm(self.h, ctypes.byref(out)))
        return out.value

    def expval(self, terms, per_term: bool = False):
        tl = terms if isinstance(terms, TermList) else TermList(terms)
        per = np.zeros(max(1, tl.n), dtype=np.float64)
        tot = ctypes.c_double()
        check(lib().qsv_expval_pauli(self.h, tl.arr, tl.n, _dptr(per), ctypes.byref(tot)))
        return (tot.value, per[: tl.n].copy()) if per_term else tot.value

    def probs(self, qubits: Optional[Sequence[int]] = None, out=None):
        """Full distribution (qubits None) in the state's real precision, or the marginal
        over ``qubits`` in float64.  ``out`` may be a device torch tensor."""
        if qubits is None:
            m, qp = self.n, None
            full = True
        else:
            m = len(qubits)
            qa = (ctypes.c_int * m)(*[int(q) for q in qubits])
            qp = ctypes.cast(qa, ctypes.POINTER(ctypes.c_int))
            full = list(qubits) == list(range(self.n))
        rdt = (np.float32 if _DT[self.dtype] == C64 else np.float64) if full else np.float64
        if out is not None:
            check(lib().qsv_probs(self.h, qp, m, ctypes.c_void_p(out.data_ptr()), 1))
            return out
        host = np.empty(1 << m, dtype=rdt)
        check(lib().qsv_probs(self.h, qp, m, host.ctypes.data_as(ctypes.c_void_p), 0))
        return host

    def sample(self, uniforms, qubits: Optional[Sequence[int]] = None) -> np.ndarray:
        """One computational-basis outcome per uniform in [0, 1) (inverse transform of the
        Born distribution over ``qubits``, bit j <-> qubits[j]; None = all qubits)."""
        u = np.ascontiguousarray(uniforms, dtype=np.float64).ravel()
        out = np.empty(u.size, dtype=np.int64)
        if qubits is None:
            m, qp = self.n, None
        else:
            m = len(qubits)
            qa = (ctypes.c_int * m)(*[int(q) for q in qubits])
            qp = ctypes.cast(qa, ctypes.POINTER(ctypes.c_int))
        check(lib().qsv_sample(self.h, qp, m, u.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), u.size,
                               out.ctypes.data_as(ctypes.POINTER(ctypes.c_longlong))))
        return out

    def free(self):
        if getattr(self, "h", None):
            lib().qsv_free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def norm_noalloc(amps, out, stream=None) -> None:
    """qsv_norm_noalloc: sum |alpha_k|^2 of the device tensor `amps` (complex64 or
    complex128, 2^n elements) into the one-element float64 device tensor `out`, with no
    allocation; asynchronous on `stream` (default: the current torch stream)."""
    import torch
    dt = {torch.complex64: "c64", torch.complex128: "c128"}[amps.dtype]
    n = amps.numel().bit_length() - 1
    if amps.numel() != (1 << n) or not amps.is_contiguous():
        raise ValueError("amps must be a contiguous device tensor of 2^n elements")
    if out.dtype != torch.float64 or out.numel() < 1 or out.device != amps.device:
        raise ValueError("out must be a float64 device tensor on the state's device")
    s = stream if stream is not None else torch.cuda.current_stream(amps.device)
    check(lib().qsv_norm_noalloc(ctypes.c_void_p(amps.data_ptr()), n, _DT[dt], ctypes.c_void_p(out.data_ptr()),
                                 ctypes.c_void_p(s.cuda_stream)))


def simulate(n: int, ops, dtype: str = "c64", **opts) -> State:
    s = State(n, dtype)
    s.apply(ops, **opts)
    return s


# ------------------------------------------------------------------ adjoint gradients

_ROT = {"RX": 1, "RY": 2, "RZ": 3}


class OpList:
    """A parameterised circuit marshalled into a ctypes qsv_op array: RX/RY/RZ ops that
    carry a parameter index become kind 1/2/3; every other op is a fixed gate."""

    def __init__(self, template):
        template = list(template)
        self._mats = []
        self.arr = (COp * max(1, len(template)))()
        self.n = len(template)
        for i, op in enumerate(template):
            c = self.arr[i]
            for j, q in enumerate(op.qubits):
                c.targets[j] = int(q)
            if op.param is not None:
                if op.name not in _ROT:
                    raise ValueError("op %d: only RX/RY/RZ may carry a parameter" % i)
                c.kind = _ROT[op.name]
                c.k = 1
                c.param = int(op.param)
            else:
                m = np.ascontiguousarray(op.matrix, dtype=np.complex128) if op.name == "U" \
                    else gate_matrix(op.name, op.params)
                buf = np.ascontiguousarray(m.reshape(-1)).view(np.float64).copy()
                self._mats.append(buf)
                c.kind = 0
                c.k = len(op.qubits)
                c.mat = _dptr(buf)
                c.param = -1


def adjoint_grad(n: int, template, params, terms, dtype: str = "c128", stream=None):
    """Energies E_b = <psi(theta_b)|H|psi(theta_b)> and dE_b/dtheta by the adjoint method.

    params: (B, P) or (P,) array of angles; terms: Pauli sum [(coeff, ((q, 'X'), ...)), ...].
    Returns (E[B], G[B, P]) as float64 numpy arrays ((P,) inputs give E scalar, G[P])."""
    import torch
    p = np.ascontiguousarray(params, dtype=np.float64)
    single = p.ndim == 1
    if single:
        p = p[None, :]
    B, P = p.shape
    ol = template if isinstance(template, OpList) else OpList(template)
    tl = terms if isinstance(terms, TermList) else TermList(terms)
    E = np.zeros(B, dtype=np.float64)
    G = np.zeros((B, P), dtype=np.float64)
    s = stream if stream is not None else torch.cuda.current_stream()
    check(lib().qsv_adjoint_grad(n, _DT[dtype], ol.arr, ol.n, _dptr(p), B, P, tl.arr, tl.n, _dptr(E), _dptr(G),
                                 ctypes.c_void_p(s.cuda_stream)))
    return (E[0], G[0]) if single else (E, G)


# ------------------------------------------------------------------ density matrices

_CHANNEL_KIND = {"DEPOLARIZE": 1, "AMPDAMP": 2}


class DMOpList:
    """Gates and noise channels marshalled into qsv_dm_op structs."""

    def __init__(self, ops: Iterable):
        ops = list(ops)
        self.n = len(ops)
        self.arr = (DMOp * max(1, len(ops)))()
        self._keep = []
        for i, op in enumerate(ops):
            d = self.arr[i]
            k = len(op.qubits)
            d.k = k
            d.targets[:k] = op.qubits
            kind = _CHANNEL_KIND.get(op.name, 0)
            d.kind = kind
            if kind:
                d.p = float(op.params[0])
                continue
            m = op.matrix if op.name == "U" else _named(op.name, op.params)
            buf = np.ascontiguousarray(m, dtype=np.complex128).reshape(-1)
            self._keep.append(buf)
            d.mat = buf.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


class DensityMatrix:
    """An n-qubit density matrix held as vec(rho) in a 2n-qubit State (starts as
    |0...0><0...0|); gates act as U rho U^dagger, channels through their Kraus
    operators, all applied by libqsv's planner and kernels."""

    def __init__(self, n: int, dtype: str = "c128", device: str = "cuda:0", stream=None):
        self.n = n
        self.dtype = dtype
        self.state = State(2 * n, dtype, device=device, stream=stream)

    def apply(self, ops, **opts) -> None:
        ol = ops if isinstance(ops, DMOpList) else DMOpList(ops)
        po = _opts(**opts) if opts else None
        check(lib().qsv_dm_apply(self.state.h, ol.arr, ol.n, ctypes.byref(po) if po is not None else None))

    def reset(self) -> None:
        self.state.reset()

    def probs(self, qubits: Optional[Sequence[int]] = None) -> np.ndarray:
        m = self.n if qubits is None else len(qubits)
        qp = None
        if qubits is not None:
            qa = (ctypes.c_int * m)(*[int(q) for q in qubits])
            qp = ctypes.cast(qa, ctypes.POINTER(ctypes.c_int))
        out = np.empty(1 << m, dtype=np.float64)
        check(lib().qsv_dm_probs(self.state.h, qp, m, _dptr(out)))
        return out

    def expval(self, terms, per_term: bool = False):
        tl = terms if isinstance(terms, TermList) else TermList(terms)
        per = np.zeros(max(1, tl.n), dtype=np.float64)
        tot = ctypes.c_double()
        check(lib().qsv_dm_expval_pauli(self.state.h, tl.arr, tl.n, _dptr(per), ctypes.byref(tot)))
        return (tot.value, per[: tl.n].copy()) if per_term else tot.value

    def matrix(self) -> np.ndarray:
        """rho as a dense 2^n x 2^n host array (small n)."""
        v = self.state.get()
        N = 1 << self.n
        return v.reshape(N, N).T.copy()   # vec index row + N col

    def free(self) -> None:
        self.state.free()


def precision_select(n: int, n_gates: int, eps_tol: float = 0.0) -> str:
    """Eq. 12: "c64" when g * 2^n * 1.19e-7 <= eps_tol (default about 6.18), else "c128"."""
    out = ctypes.c_int()
    check(lib().qsv_precision_select(n, n_gates, eps_tol, ctypes.byref(out)))
    return "c64" if out.value == C64 else "c128"

