"""Writes the stored expected values for the full-size parity tests.

Calls only the FP64 oracle and the seeded input generators: the seeded brickwork
circuits at the benchmark sizes are simulated gate by gate on the host, and a seeded
sample of amplitudes plus a few reductions are written to JSON next to this script.

    python tests/golden/make_golden.py 28      # brickwork n=28 depth=20 seed=2 (4 GiB state)
    python tests/golden/make_golden.py 30      # brickwork n=30 depth=20 seed=3 (16 GiB state)
    python tests/golden/make_golden.py serve   # served request sizes: n=20, 24, 26 (per-qubit <Z_i>)
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
from paper_2604_03816_amd import circuits as C  # noqa: E402

CASES = {28: (20, 2), 30: (20, 3), 22: (20, 7)}
# served requests at the large end of the serving workload's 12-26 qubits
SERVE_CASES = [(20, 30, 21), (24, 20, 22), (26, 15, 23)]
SAMPLES = 1024


def serve_case(n, depth, seed):
    """Per-qubit <Z_i> and the norm (what a served request returns) plus seeded amplitudes
    (for states kept on the device) of one brickwork request."""
    ops = C.brickwork(n, depth, seed)
    t0 = time.time()
    psi = oracle.zero_state(n)
    for op in ops:
        oracle.apply(psi, oracle.op_matrix(op), op.qubits)
    rng = np.random.default_rng(777 + n)
    idx = np.unique(np.concatenate([[0, (1 << n) - 1], rng.integers(0, 1 << n, size=SAMPLES)]))
    zexp = [float(oracle.pauli_expval(psi, ((q, "Z"),)).real) for q in range(n)]
    rec = {
        "about": "FP64 oracle, gate by gate: served brickwork request n=%d depth=%d seed=%d (%d gates); "
                 "written by tests/golden/make_golden.py" % (n, depth, seed, len(ops)),
        "n": n, "depth": depth, "seed": seed, "gates": len(ops),
        "norm2": oracle.norm2(psi),
        "zexp": zexp,
        "index": [int(i) for i in idx],
        "re": [float(a.real) for a in psi[idx]],
        "im": [float(a.imag) for a in psi[idx]],
        "oracle_seconds": time.time() - t0,
    }
    path = os.path.join(HERE, "serve_brickwork_n%d_d%d_s%d.json" % (n, depth, seed))
    with open(path, "w") as f:
        json.dump(rec, f)
    print("wrote", path, "in %.0f s" % (time.time() - t0))


def main(n):
    depth, seed = CASES[n]
    ops = C.brickwork(n, depth, seed)
    t0 = time.time()
    psi = oracle.zero_state(n)
    for i, op in enumerate(ops):
        oracle.apply(psi, oracle.op_matrix(op), op.qubits)
        if i % 50 == 0:
            print("gate %d/%d  %.0f s" % (i, len(ops), time.time() - t0), flush=True)
    rng = np.random.default_rng(12345 + n)
    idx = np.unique(np.concatenate([[0, (1 << n) - 1], rng.integers(0, 1 << n, size=SAMPLES)]))
    amps = psi[idx]
    marg_q = [0, n // 2, n - 1]
    terms = C.zz_chain_terms(n) + C.x_sum_terms(n)
    per = oracle.expval_terms(psi, terms)
    rec = {
        "about": "FP64 oracle, gate by gate: brickwork n=%d depth=%d seed=%d (%d gates); written by "
                 "tests/golden/make_golden.py" % (n, depth, seed, len(ops)),
        "n": n, "depth": depth, "seed": seed, "gates": len(ops),
        "norm2": oracle.norm2(psi),
        "index": [int(i) for i in idx],
        "re": [float(a.real) for a in amps],
        "im": [float(a.imag) for a in amps],
        "marginal_qubits": marg_q,
        "marginal": [float(x) for x in oracle.probs(psi, marg_q)],
        "zz_terms": [float(x) for x in per[: n - 1]],
        "x_terms": [float(x) for x in per[n - 1:]],
        "oracle_threads": oracle.num_threads(),
        "oracle_seconds": time.time() - t0,
    }
    path = os.path.join(HERE, "brickwork_n%d_d%d_s%d.json" % (n, depth, seed))
    with open(path, "w") as f:
        json.dump(rec, f)
    print("wrote", path, "in %.0f s" % (time.time() - t0))


if __name__ == "__main__":
    if sys.argv[1] == "serve":
        for case in SERVE_CASES:
            serve_case(*case)
    else:
        main(int(sys.argv[1]))
