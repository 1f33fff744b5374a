"""Benchmark of the state-vector hot path on one MI355X.

One step = one pass of the hot path over one synthetic circuit already resident on the
device: reset the state to |0...0>, apply the fused circuit (every HBM pass of the
plan), then the reductions (norm and the <sum Z_i Z_i+1> expectation).  Planning is
host work done once before the timed region and reported separately.

Workload (headline): seeded random brickwork, 30 qubits, depth 20 (890 gates: a Haar
U(2) on every qubit per layer, CNOT pairs alternating even/odd), complex64 state with
FP32 arithmetic; the same circuit in complex128 is reported beside it.

value = fused gates x 2 x 2^n x bytes-per-amplitude / step time  ("fused-gate amplitude
GB/s": every fused gate must read and write each amplitude once; several fused gates
share one HBM round trip, so the figure can exceed the HBM peak).  Because it counts
the planner's fused gates, a plan that fuses into fewer, wider gates lowers it even when
the step gets faster; detail.gate_amplitude_GB_per_s counts the circuit's own gates
instead (the same for every plan), and ms_per_step compares plans directly.

roofline: the pass kernel, bound by HBM bandwidth.  Algorithmic bytes per launch = 2 x
2^n x bytes-per-amplitude (one read and one write of the state; the first pass, which
builds |0...0> on chip, only writes), averaged over the step's launches, divided by the
average launch duration (HIP events recorded around every pass launch inside the timed
steps, on the state's stream) and by the 8 TB/s peak.  Beside it, the ALU fraction of the
same launches: algorithmic flops per launch = 2 x (the plan's complex-arithmetic FMA per
amplitude / passes) x 2^n against a peak that combines the VALU rate for the VALU share
of the FMA (78.6 TFLOP/s: FP64 vector, and FP32 without packed math) with the
matrix-core rate for the matrix-core share (FP32 MFMA 157.3 TFLOP/s for complex64, FP64
MFMA 78.6 TFLOP/s for complex128).  traffic = HBM bytes per launch measured with rocprofv3 counters
(FETCH_SIZE + WRITE_SIZE, scaled by the same counters' reading for a device copy of
known size), taken from the summary under profiles/ when that summary was made from
the current kernel source, else null.

cpu_baseline: the FP64 CPU oracle (gate by gate, all host threads) on the first gates of
the same 30-qubit circuit, reported in the same unit with its own (unfused) gate count.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu] [--no-c128]
       [--no-serve] [--no-precision] [--no-adjoint] [--no-sampling] [--no-noise] [--copy-probe]
"""
import argparse
import dataclasses
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# VALU peak without packed FP32 (disabled in this build): 256 CUs x 64 FMA lanes per clock
# x 2 flops x 2.4 GHz = 78.6 TFLOP/s, which is also MI355X's FP64 vector peak.
VALU_PEAK_TFLOPS = 78.6
MFMA_FP32_PEAK_TFLOPS = 157.3
MFMA_FP64_PEAK_TFLOPS = 78.6
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_pass_brickwork30_hbm_traffic.md")
KERNEL_SOURCES = [os.path.join(ROOT, "paper_2604_03816_amd", "csrc", f) for f in ("kernels.hip", "planner.cpp")]


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--qubits", type=int, default=30)
    ap.add_argument("--depth", type=int, default=20)
    ap.add_argument("--seed", type=int, default=3)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-c128", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=20.0)
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--no-precision", action="store_true")
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--no-sampling", action="store_true")
    ap.add_argument("--no-noise", action="store_true")
    ap.add_argument("--no-commute", action="store_true")
    ap.add_argument("--no-fusion", action="store_true")
    ap.add_argument("--kernel-sweep", action="store_true",
                    help="also time one-op passes per op class (k, targets, VALU vs matrix cores)")
    ap.add_argument("--precision-qubits", type=int, nargs="*", default=[30, 32])
    ap.add_argument("--adjoint-qubits", type=int, default=24)
    ap.add_argument("--adjoint-batch", type=int, default=64)
    ap.add_argument("--serve-requests", type=int, default=4096)
    ap.add_argument("--plain-requests", type=int, default=256)
    ap.add_argument("--capacity-requests", type=int, default=1024)
    ap.add_argument("--copy-probe", action="store_true",
                    help="copy 4 GiB device to device once before the timed steps (counter calibration)")
    return ap.parse_args()


def time_steps(torch, qsv, state, plan, terms, steps, warmup):
    """Wall time per step, and the device time of every pass launch inside the timed
    steps (HIP events on the state's stream, around each single-pass launch)."""
    npass = plan.stats()["passes"]
    stream = state.stream

    def step(evs):
        # |0...0> is built inside the first pass (qsv_plan_apply_zero), not by a reset pass
        for i in range(npass):
            run = (lambda: state.apply_plan_zero(plan, 1)) if i == 0 else (lambda: state.apply_plan(plan, i, 1))
            if evs is not None:
                a = torch.cuda.Event(enable_timing=True)
                b = torch.cuda.Event(enable_timing=True)
                a.record(stream)
                run()
                b.record(stream)
                evs.append((a, b))
            else:
                run()
        state.norm()
        state.expval(terms)

    for _ in range(warmup):
        step(None)
    torch.cuda.synchronize()
    evs = []
    t0 = time.perf_counter()
    for _ in range(steps):
        step(evs)
    torch.cuda.synchronize()
    sec = (time.perf_counter() - t0) / steps
    times = [a.elapsed_time(b) for a, b in evs]
    return sec, sum(times) / len(times)


def source_digest() -> str:
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(dtype):
    """HBM bytes per pass launch from the committed counter summary, or None when the
    summary is missing or was taken from other kernel sources."""
    try:
        with open(TRAFFIC_FILE) as fh:
            kv = {}
            for line in fh:
                line = line.strip()
                if line.startswith("- ") and ":" in line:
                    k, v = line[2:].split(":", 1)
                    kv[k.strip()] = v.strip()
    except OSError:
        return None
    if kv.get("kernel_sources_sha256") != source_digest():
        return None
    v = kv.get("%s_hbm_bytes_per_launch" % dtype)
    return float(v) if v not in (None, "", "null") else None


def copy_probe(torch):
    """One 4 GiB device-to-device copy: the reference reading for HBM byte counters."""
    nbytes = 4 << 30
    src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    dst.copy_(src)
    torch.cuda.synchronize()
    del src, dst
    torch.cuda.empty_cache()
    return {"bytes_read": nbytes, "bytes_written": nbytes}


def run_dtype(torch, qsv, C, args, dtype, ops, terms):
    n = args.qubits
    t0 = time.perf_counter()
    plan = qsv.Plan(n, dtype, ops)
    plan_ms = (time.perf_counter() - t0) * 1e3
    st = plan.stats()
    state = qsv.State(n, dtype)
    sec, avg_pass_ms = time_steps(torch, qsv, state, plan, terms, args.steps, args.warmup)
    elem = 8 if dtype == "c64" else 16
    pass_bytes = 2.0 * (2 ** n) * elem
    value = st["fused_out"] * pass_bytes / sec / 1e9
    gate_value = st["gates_in"] * pass_bytes / sec / 1e9
    # algorithmic bytes per launch, averaged over the step's launches: every pass reads and
    # writes the state once, except the first, which builds |0...0> on chip and only writes
    npass = st["passes"]
    launch_bytes = (2.0 * npass - 1.0) / npass * (2 ** n) * elem
    achieved = launch_bytes / (avg_pass_ms * 1e-3) / 1e9
    # arithmetic of the average pass: the plan's FMA per amplitude (dense 4*2^k, diagonal
    # or phased permutation 4), 2 flops each, over every amplitude
    fma_v = (st["fma_per_amp"] - st["mfma_fma_per_amp"]) / st["passes"]
    fma_m = st["mfma_fma_per_amp"] / st["passes"]
    pass_flops = 2.0 * (fma_v + fma_m) * (2 ** n)
    mfma_peak = MFMA_FP32_PEAK_TFLOPS if dtype == "c64" else MFMA_FP64_PEAK_TFLOPS
    floor_s = 2.0 * (2 ** n) * (fma_v / (VALU_PEAK_TFLOPS * 1e12) + fma_m / (mfma_peak * 1e12))
    alu_peak = pass_flops / floor_s / 1e12
    alu_tflops = pass_flops / (avg_pass_ms * 1e-3) / 1e12
    hbm_frac = achieved / HBM_PEAK_GBS
    alu_frac = alu_tflops / alu_peak
    traffic = measured_traffic(dtype)
    # the pass kernel's roofline is HBM bandwidth (every pass reads and writes the state
    # once); the ALU fraction of the same launches is reported beside it
    roof = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": hbm_frac, "traffic": traffic,
            "alu": {"achieved": alu_tflops, "peak": alu_peak, "unit": "TFLOP/s", "frac": alu_frac}}
    # sanity of the result: the circuit preserves the norm
    norm = state.norm()
    out = {
        "value": value,
        "gate_amplitude_GB_per_s": gate_value,
        "ms_per_step": sec * 1e3,
        "plan_ms": plan_ms,
        "gates": st["gates_in"],
        "fused_gates": st["fused_out"],
        "passes": st["passes"],
        "avg_pass_ms": avg_pass_ms,
        "norm_minus_1": norm - 1.0,
        "roofline": roof,
        "hbm": {"achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": hbm_frac},
        "alu": {"achieved": alu_tflops, "peak": alu_peak, "unit": "TFLOP/s", "frac": alu_frac,
                "fma_per_amp_valu": fma_v, "fma_per_amp_mfma": fma_m},
        "traffic_bytes_per_launch": traffic,
        "algorithmic_bytes_per_launch": launch_bytes,
    }
    state.free()
    plan.free()
    torch.cuda.empty_cache()
    return out


def cpu_baseline(C, args, ops):
    import numpy as np
    import oracle
    n = args.qubits
    t0 = time.perf_counter()
    psi = oracle.zero_state(n)
    init_s = time.perf_counter() - t0
    done, t_apply = 0, 0.0
    while done < len(ops) and t_apply < args.cpu_seconds:
        op = ops[done]
        t1 = time.perf_counter()
        oracle.apply(psi, oracle.op_matrix(op), op.qubits)
        t_apply += time.perf_counter() - t1
        done += 1
    del psi
    value = done * 2.0 * (2 ** n) * 16 / t_apply / 1e9
    return {"value": value, "unit": "GB/s", "cores": oracle.num_threads(), "kind": "oracle",
            "sample": "first %d of %d gates of the %d-qubit depth-%d brickwork, complex128, gate by gate "
                      "(%.1f s of gate application; state init %.1f s not counted)"
                      % (done, len(ops), n, args.depth, t_apply, init_s),
            "host": host_info(),
            "one_thread": oracle_one_thread(24, args.depth, args.seed, min(5.0, args.cpu_seconds))}


def host_info():
    """CPU model, logical CPUs and RAM of the host the oracle ran on."""
    info = {"logical_cpus": os.cpu_count()}
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    info["cpu_model"] = line.split(":", 1)[1].strip()
                    break
        with open("/proc/meminfo") as f:
            for line in f:
                if line.startswith("MemTotal"):
                    info["ram_gib"] = round(int(line.split()[1]) / 2 ** 20, 1)
                    break
    except OSError:
        pass
    return info


_ONE_THREAD = r"""
import json, sys, time
sys.path.insert(0, sys.argv[1])
import oracle
from paper_2604_03816_amd import circuits as C
n, depth, seed, budget = int(sys.argv[2]), int(sys.argv[3]), int(sys.argv[4]), float(sys.argv[5])
ops = C.brickwork(n, depth, seed)
psi = oracle.zero_state(n)
done, t = 0, 0.0
while done < len(ops) and t < budget:
    t0 = time.perf_counter()
    oracle.apply(psi, oracle.op_matrix(ops[done]), ops[done].qubits)
    t += time.perf_counter() - t0
    done += 1
print(json.dumps({"n": n, "gates": done, "seconds": t, "threads": oracle.num_threads(),
                  "GB_per_s": done * 2.0 * 2 ** n * 16 / t / 1e9, "ms_per_gate": t / done * 1e3}))
"""


def oracle_one_thread(n, depth, seed, budget):
    """The oracle on one host thread (a child process with OMP_NUM_THREADS=1) on the first
    gates of the n-qubit brickwork: the shape of a single-threaded CPU simulator column."""
    import subprocess
    env = dict(os.environ, OMP_NUM_THREADS="1")
    r = subprocess.run([sys.executable, "-c", _ONE_THREAD, ROOT, str(n), str(depth), str(seed), str(budget)],
                       env=env, capture_output=True, text=True, timeout=300)
    if r.returncode != 0:
        return {"error": r.stderr[-500:]}
    return json.loads(r.stdout.strip().splitlines()[-1])


def serving(args):
    """Continuous batching on the request stream (4096 seeded requests, 12-26 qubits,
    brickwork depth 10-60, 70 % complex64, Poisson arrivals at 200/s), against the plain
    path (one circuit at a time, one gate per HBM pass) on a prefix of the same stream."""
    import torch
    from paper_2604_03816_amd import circuits as C
    from paper_2604_03816_amd import qsv, serve
    reqs = C.serving_stream(args.serve_requests, seed=5)
    t0 = time.perf_counter()
    circuits = [qsv.ArrayGateList(C.brickwork_arrays(r.n, r.depth, r.seed)) for r in reqs]
    gen_s = time.perf_counter() - t0
    sv = serve.Server(max_slots=64, use_graph=True)
    batched = serve.run_batched(reqs, circuits, sv)
    sv.close()
    torch.cuda.empty_cache()
    # the same stream with the precision left to the server (Eq. 12, default tolerance;
    # complex64 runs whose norm drifts by more than 1e-5 are repeated in complex128)
    auto_reqs = [dataclasses.replace(r, dtype="auto") for r in reqs]
    sv = serve.Server(max_slots=64, use_graph=True, norm_guard=1e-5)
    auto = serve.run_batched(auto_reqs, circuits, sv)
    sv.close()
    torch.cuda.empty_cache()
    # capacity: the same mixes with every request arriving at once (closed loop), on a
    # prefix of the stream; circuits/s is then the sustainable maximum for the mix
    kc = min(args.capacity_requests, len(reqs))
    sv = serve.Server(max_slots=64, use_graph=True)
    cap = serve.run_batched(reqs[:kc], circuits[:kc], sv, closed_loop=True)
    sv.close()
    torch.cuda.empty_cache()
    sv = serve.Server(max_slots=64, use_graph=True, norm_guard=1e-5)
    cap_auto = serve.run_batched(auto_reqs[:kc], circuits[:kc], sv, closed_loop=True)
    sv.close()
    torch.cuda.empty_cache()
    k = min(args.plain_requests, len(reqs))
    plain = serve.run_plain(reqs[:k], circuits[:k], fuse=False)
    plain_fused = serve.run_plain(reqs[:k], circuits[:k], fuse=True)
    # the same prefix fused one at a time with every request arriving at once: the plain
    # path's capacity, to set beside the batched capacity
    plain_fused_cap = serve.run_plain([dataclasses.replace(r, arrival_s=0.0) for r in reqs[:k]], circuits[:k],
                                      fuse=True)
    return {"workload": "%d requests, n~U{12..26}, brickwork depth~U{10..60}, 70%% complex64, Poisson 200/s, "
                        "seed 5" % len(reqs),
            "offered_per_s": 200.0, "input_generation_s": gen_s,
            "batched": batched,
            "batched_auto_precision": auto,
            "capacity": dict(cap, note="first %d requests of the same stream, all arriving at t = 0" % kc),
            "capacity_auto_precision": dict(cap_auto, note="as capacity, precision chosen by Eq. 12"),
            "plain": dict(plain, note="first %d requests of the same stream, one at a time, unfused" % k),
            "plain_fused": dict(plain_fused, note="first %d requests of the same stream, one at a time, "
                                                  "fused with the default plan options" % k),
            "plain_fused_capacity": dict(plain_fused_cap, note="as plain_fused, all arriving at t = 0")}


def precision_study(args):
    """Hardware-efficient ansatz (6 layers of RY, RZ on every qubit + CZ ladder, angles
    from seed 4) at 30 and 32 qubits: <sum Z_i Z_i+1> and <sum X_i> in complex64 and
    complex128, their difference, and the complex64 state against the complex128 one over
    the whole state (max |d alpha|, raw and normalised infidelity)."""
    import torch
    from paper_2604_03816_amd import circuits as C
    from paper_2604_03816_amd import qsv
    out = []
    for n in args.precision_qubits:
        layers = 6
        ops = C.bind(C.hea(n, layers), C.hea_params(n, layers, seed=4))
        zz, xs = C.zz_chain_terms(n), C.x_sum_terms(n)
        rec = {"n": n, "gates": len(ops)}
        states = {}
        for dt in ("c128", "c64"):
            plan = qsv.Plan(n, dt, ops)
            s = qsv.State(n, dt)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            s.apply_plan(plan)
            s.sync()
            t_apply = time.perf_counter() - t0
            t0 = time.perf_counter()
            ezz, exx = s.expval(zz), s.expval(xs)
            t_red = time.perf_counter() - t0
            rec[dt] = {"zz": ezz, "x": exx, "norm_minus_1": s.norm() - 1.0, "apply_ms": t_apply * 1e3,
                       "expval_ms": t_red * 1e3, "passes": plan.stats()["passes"]}
            states[dt] = s
            plan.free()
        gap = precision_gap(states["c128"].tensor, states["c64"].tensor)
        rec["c64_vs_c128"] = {"d_zz": abs(rec["c64"]["zz"] - rec["c128"]["zz"]),
                              "d_x": abs(rec["c64"]["x"] - rec["c128"]["x"]), **gap}
        for st in states.values():
            st.free()
        del states
        torch.cuda.empty_cache()
        out.append(rec)
    return out


def precision_gap(a, b, chunk=1 << 26):
    """complex64 state b against the complex128 state a of the same circuit over the whole
    state, chunk by chunk on the device in FP64: max |a_k - b_k|, the raw overlap deficit
    1 - |<a|b>|^2 (which follows b's norm drift) and the normalised infidelity
    1 - |<a|b>|^2 / (<a|a> <b|b>) (the state error proper)."""
    import torch
    ov, na, nb, mx = 0j, 0.0, 0.0, 0.0
    for i in range(0, a.numel(), chunk):
        x = a[i:i + chunk]
        y = b[i:i + chunk].to(torch.complex128)
        ov += torch.vdot(x, y).item()
        na += torch.vdot(x, x).real.item()
        nb += torch.vdot(y, y).real.item()
        mx = max(mx, (x - y).abs().max().item())
    return {"max_abs_diff": mx, "raw_deficit": 1.0 - abs(ov) ** 2,
            "infidelity": 1.0 - abs(ov) ** 2 / (na * nb), "norm2_c64_minus_1": nb - 1.0}


def commutation_bench(args):
    """Commutation-aware DAG (ops diagonal on every qubit they share left unordered, so
    fusion and pass scheduling may cross them) against the per-qubit DAG, on the
    30-qubit H/T + CZ bricks (depth 20, seed 2) and on the main step's brickwork:
    fused ops, passes and the time of one application (median of 3), per precision."""
    import torch
    from paper_2604_03816_amd import circuits as C
    from paper_2604_03816_amd import qsv
    n = args.qubits
    circuits = {"h_t_cz_bricks depth=20 seed=2": C.h_t_cz_bricks(n, 20, 2),
                "brickwork depth=%d seed=%d" % (args.depth, args.seed): C.brickwork(n, args.depth, args.seed)}
    out = {}
    for dt in ("c64", "c128"):
        s = qsv.State(n, dt)
        for name, ops in circuits.items():
            rec = {}
            for label, commute in (("per_qubit_dag", -1), ("commutation_dag", 1)):
                t0 = time.perf_counter()
                plan = qsv.Plan(n, dt, ops, commute=commute)
                plan_ms = (time.perf_counter() - t0) * 1e3
                ts = []
                for _ in range(3):
                    s.reset()
                    s.sync()
                    t0 = time.perf_counter()
                    s.apply_plan(plan)
                    s.sync()
                    ts.append((time.perf_counter() - t0) * 1e3)
                st = plan.stats()
                rec[label] = {"fused": st["fused_out"], "passes": st["passes"], "plan_ms": plan_ms,
                              "apply_ms": sorted(ts)[1]}
                plan.free()
            rec["speedup"] = rec["per_qubit_dag"]["apply_ms"] / rec["commutation_dag"]["apply_ms"]
            out["%s %s" % (name, dt)] = rec
        s.free()
        torch.cuda.empty_cache()
    return out


def adjoint_bench(args):
    """Adjoint gradients: 24-qubit ansatz, 8 layers of RY, RZ + CZ ring (384 parameters),
    transverse-field Ising H (periodic, h = 0.7), 64 parameter vectors; complex128 and
    complex64.  Reports wall time per batch, a central-difference spot check and the
    complex64 gradients' error against complex128."""
    import numpy as np
    from paper_2604_03816_amd import circuits as C
    from paper_2604_03816_amd import qsv
    n, layers, B = args.adjoint_qubits, 8, args.adjoint_batch
    tpl = C.hea(n, layers, ring=True)
    terms = C.tfim_terms(n)
    params = C.hea_params(n, layers, seed=6, batch=B)
    out = {"n": n, "params": params.shape[1], "batch": B}
    for dt in ("c128", "c64"):
        t0 = time.perf_counter()
        E, G = qsv.adjoint_grad(n, tpl, params, terms, dt)
        wall = time.perf_counter() - t0
        out[dt] = {"wall_s": wall, "gradients_per_s": B * params.shape[1] / wall, "energy0": float(E[0])}
        if dt == "c128":
            g128 = np.asarray(G)
        else:
            g64 = np.asarray(G)
    # central differences (h = 1e-6, complex128 energies) on 4 parameters of vector 0
    h = 1e-6
    idx = [0, 57, 200, 383 if params.shape[1] > 383 else params.shape[1] - 1]
    fd = []
    for j in idx:
        p = params[0].copy()
        p[j] += h
        ep, _ = qsv.adjoint_grad(n, tpl, p, terms, "c128")
        p[j] -= 2 * h
        em, _ = qsv.adjoint_grad(n, tpl, p, terms, "c128")
        fd.append((ep - em) / (2 * h))
    out["fd_check"] = {"params": idx, "max_abs_diff": float(max(abs(g128[0][j] - f) for j, f in zip(idx, fd)))}
    # complex64 gradients against complex128: relative error ||g64 - g128|| / ||g128|| per
    # parameter vector (the worst and the median over the batch) and the largest element error
    rel = np.linalg.norm(g64 - g128, axis=1) / np.linalg.norm(g128, axis=1)
    out["c64_vs_c128"] = {"rel_err_max": float(rel.max()), "rel_err_median": float(np.median(rel)),
                          "max_abs_diff": float(np.max(np.abs(g64 - g128)))}
    return out


def sampling_bench(args, ops):
    """Measurement sampling (inverse transform of the Born distribution) on the headline
    state: the 30-qubit brickwork in complex64, 2^20 shots over all qubits and over 8
    qubits; uniforms from seed 8.  Wall time of the synchronous call (one chunk-total pass
    over the state, prefix sums on the host; on the device the shots sorted, assigned to
    chunks and grouped, one pass over the chunks that hold shots)."""
    import numpy as np
    import torch
    from paper_2604_03816_amd import qsv
    n = args.qubits
    plan = qsv.Plan(n, "c64", ops)
    s = qsv.State(n, "c64")
    s.apply_plan(plan)
    s.sync()
    u = np.random.default_rng(8).random(1 << 20)
    out = {"n": n, "shots": int(u.size)}
    for name, qubits in (("all_qubits", None), ("8_qubits", [0, 5, 9, 13, 17, 21, 25, 29][: min(8, n)])):
        s.sample(u[:1024], qubits)
        t0 = time.perf_counter()
        got = s.sample(u, qubits)
        wall = time.perf_counter() - t0
        out[name] = {"wall_s": wall, "shots_per_s": u.size / wall, "distinct_outcomes": int(np.unique(got).size)}
    s.free()
    plan.free()
    torch.cuda.empty_cache()
    return out


def fusion_bench(args):
    """The fusion study at 28 qubits: the seeded brickwork (depth 20, seed 2, 830 gates)
    fused by the DAG planner (<= 5-qubit unitaries, several per HBM pass) against the
    same circuit unfused and gate by gate (one gate per pass, as the paper applies gates),
    in complex64 and complex128.  Per run: gates, fused gates, passes, the median of 3
    applications to |0...0> (HIP events), fused-gate amplitude GB/s and HBM GB/s, and
    max |d alpha| against the FP64 oracle's amplitudes at 1 026 seeded indices (stored by
    tests/golden/make_golden.py, which also records the oracle's own run time)."""
    import numpy as np
    import torch
    from paper_2604_03816_amd import circuits as C
    from paper_2604_03816_amd import qsv
    n, depth, seed = 28, 20, 2
    with open(os.path.join(ROOT, "tests", "golden", "brickwork_n%d_d%d_s%d.json" % (n, depth, seed))) as f:
        g = json.load(f)
    ref = np.array(g["re"]) + 1j * np.array(g["im"])
    ops = C.brickwork(n, depth, seed)
    out = {"n": n, "depth": depth, "seed": seed, "gates": len(ops),
           "oracle": {"seconds": g.get("oracle_seconds"), "threads": g.get("oracle_threads"),
                      "samples": len(g["index"])}}
    for dt in ("c64", "c128"):
        s = qsv.State(n, dt)
        elem = 8 if dt == "c64" else 16
        idx = torch.tensor(g["index"], dtype=torch.int64, device=s.tensor.device)
        rec = {}
        for label, fuse in (("fused", 1), ("unfused", 0)):
            plan = qsv.Plan(n, dt, ops, fuse=fuse)
            st = plan.stats()
            ts = []
            for _ in range(3):
                a = torch.cuda.Event(enable_timing=True)
                b = torch.cuda.Event(enable_timing=True)
                a.record(s.stream)
                s.apply_plan_zero(plan)
                b.record(s.stream)
                b.synchronize()
                ts.append(a.elapsed_time(b) * 1e-3)
            t = sorted(ts)[1]
            amps = s.tensor[idx].cpu().numpy().astype(np.complex128)
            rec[label] = {"fused_gates": st["fused_out"], "passes": st["passes"], "seconds": t,
                          "fused_gate_GB_per_s": st["fused_out"] * 2.0 * 2 ** n * elem / t / 1e9,
                          "hbm_GB_per_s": (2.0 * st["passes"] - 1.0) * 2 ** n * elem / t / 1e9,
                          "max_abs_diff_vs_oracle": float(np.max(np.abs(amps - ref)))}
            plan.free()
        rec["speedup"] = rec["unfused"]["seconds"] / rec["fused"]["seconds"]
        out[dt] = rec
        s.free()
        torch.cuda.empty_cache()
    return out


def kernel_sweep(args):
    """Pass kernel per op class at n qubits: one fused op per pass (a Haar k-qubit unitary,
    k = 1..5, or a diagonal 5-qubit phase table) on targets at the bottom of the index
    (qubits 0..k-1, inside the tile's contiguous runs), in the middle (qubits 4..3+k, tile
    qubits outside the runs) or at the top (n-k..n-1, strided tile rows); dense ops of
    3 and 4 qubits both on the VALU and on matrix cores.  Median of 5 launches (HIP events
    on the state's stream) after 2 warm-up launches; GB/s = 2 x 2^n x bytes-per-amplitude
    per launch."""
    import numpy as np
    import torch
    from paper_2604_03816_amd import circuits as C
    from paper_2604_03816_amd import qsv
    n = args.qubits
    rng = np.random.default_rng(9)
    where = {"low": lambda k: tuple(range(k)), "mid": lambda k: tuple(range(4, 4 + k)),
             "high": lambda k: tuple(range(n - k, n))}
    rows = []
    for dt in ("c64", "c128"):
        s = qsv.State(n, dt)
        elem = 8 if dt == "c64" else 16

        def timed(ops, mc):
            plan = qsv.Plan(n, dt, ops, matrix_cores=mc)
            st = plan.stats()
            ts = []
            for i in range(7):
                a = torch.cuda.Event(enable_timing=True)
                b = torch.cuda.Event(enable_timing=True)
                a.record(s.stream)
                s.apply_plan(plan)
                b.record(s.stream)
                b.synchronize()
                if i >= 2:
                    ts.append(a.elapsed_time(b))
            plan.free()
            ms = sorted(ts)[len(ts) // 2]
            gbs = 2.0 * (2 ** n) * elem / (ms * 1e-3) / 1e9
            return {"ms": ms, "GB_per_s": gbs, "hbm_frac": gbs / HBM_PEAK_GBS, "passes": st["passes"],
                    "mfma_ops": st["mfma_ops"]}

        for k in range(1, 6):
            U = C.haar_unitary(rng, 1 << k)
            for cls, tg in where.items():
                ops = [C.Op("U", tg(k), matrix=U)]
                engines = (("valu", -1), ("mfma", 3)) if k in (3, 4) else (("valu", -1),)
                for eng, mc in engines:
                    rows.append(dict(dtype=dt, op="dense", k=k, targets=cls, engine=eng, **timed(ops, mc)))
        D = np.diag(np.exp(1j * rng.uniform(0, 2 * math.pi, 32)))
        for cls, tg in where.items():
            rows.append(dict(dtype=dt, op="diag", k=5, targets=cls, engine="valu", **timed([C.Op("U", tg(5), matrix=D)], -1)))
        s.free()
        torch.cuda.empty_cache()
    return {"n": n, "rows": rows}


def noise_bench(args):
    """Density-matrix noise study (Table 8's circuits: H on qubit 0, CNOT from qubit 0 to
    every other qubit, single-qubit depolarizing p = 0.01 after every gate): exact F_cl
    and TVD against the ideal distribution for Bell and GHZ-3..5, and the same circuit at
    13 qubits (a 26-qubit vec(rho)) for timing; complex128."""
    import numpy as np
    import torch
    from paper_2604_03816_amd import circuits as C
    from paper_2604_03816_amd import qsv

    def circuit(n, p=0.01):
        ops = [C.Op("H", (0,)), C.Op("DEPOLARIZE", (0,), (p,))]
        for t in range(1, n):
            ops += [C.Op("CNOT", (0, t)), C.Op("DEPOLARIZE", (0,), (p,)), C.Op("DEPOLARIZE", (t,), (p,))]
        return ops

    out = []
    for n in (2, 3, 4, 5, 13):
        dm = qsv.DensityMatrix(n, "c128")
        ops = circuit(n)
        dm.apply(ops)
        torch.cuda.synchronize()
        dm.reset()
        t0 = time.perf_counter()
        dm.apply(ops)
        p = dm.probs()
        wall = time.perf_counter() - t0
        ideal = np.zeros(1 << n)
        ideal[0] = ideal[-1] = 0.5
        fcl = float(np.sum(np.sqrt(ideal * np.clip(p, 0, None))) ** 2)
        out.append({"n": n, "gates_and_channels": len(ops), "F_cl": fcl, "TVD": float(0.5 * np.abs(p - ideal).sum()),
                    "apply_and_probs_ms": wall * 1e3})
        dm.free()
        torch.cuda.empty_cache()
    return out


def progress(msg):
    """A progress line on stderr (the result line alone goes to stdout)."""
    print("[bench %.0fs] %s" % (time.perf_counter() - _T0, msg), file=sys.stderr, flush=True)


_T0 = time.perf_counter()


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py runs on one GPU only: the state-vector path here has no multi-GPU sharding "
              "(see DESIGN.md for how it would shard); use --gpus 1", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_2604_03816_amd import circuits as C
    from paper_2604_03816_amd import qsv
    if not os.path.exists(qsv.LIB_PATH):
        import __graft_entry__
        __graft_entry__.build()
    n = args.qubits
    probe = copy_probe(torch) if args.copy_probe else None
    ops = C.brickwork(n, args.depth, args.seed)
    terms = C.zz_chain_terms(n)
    progress("start")
    main_rec = run_dtype(torch, qsv, C, args, "c64", ops, terms)
    progress("complex64 step done")
    rec = {
        "metric": "fused-gate amplitude GB/s (% HBM peak) at 30q",
        "value": main_rec["value"],
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": main_rec["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "brickwork n=%d depth=%d seed=%d complex64" % (n, args.depth, args.seed),
                   "n_qubits": n, "depth": args.depth, "gates": main_rec["gates"],
                   "fused_gates": main_rec["fused_gates"], "passes": main_rec["passes"],
                   "state": "complex64"},
        "roofline": main_rec["roofline"],
        "hbm_frac": main_rec["hbm"]["frac"],
        "detail": {k: main_rec[k] for k in ("gate_amplitude_GB_per_s", "plan_ms", "avg_pass_ms", "norm_minus_1",
                                            "hbm", "alu")},
    }
    if probe is not None:
        rec["copy_probe"] = probe
    if not args.no_c128:
        r = run_dtype(torch, qsv, C, args, "c128", ops, terms)
        progress("complex128 step done")
        rec["c128"] = {"value": r["value"], "gate_amplitude_GB_per_s": r["gate_amplitude_GB_per_s"], "unit": "GB/s",
                       "dtype": "f64", "ms_per_step": r["ms_per_step"],
                       "fused_gates": r["fused_gates"], "passes": r["passes"], "avg_pass_ms": r["avg_pass_ms"],
                       "roofline": r["roofline"], "hbm": r["hbm"], "alu": r["alu"],
                       "norm_minus_1": r["norm_minus_1"]}
    if not args.no_serve:
        rec["serving"] = serving(args)
        progress("serving done")
    if not args.no_precision:
        rec["precision"] = precision_study(args)
        progress("precision done")
    if not args.no_adjoint:
        rec["adjoint"] = adjoint_bench(args)
        progress("adjoint done")
    if not args.no_sampling:
        rec["sampling"] = sampling_bench(args, ops)
        progress("sampling done")
    if not args.no_noise:
        rec["noise"] = noise_bench(args)
        progress("noise done")
    if not args.no_commute:
        rec["commutation"] = commutation_bench(args)
        progress("commutation done")
    if not args.no_fusion:
        rec["fusion"] = fusion_bench(args)
        progress("fusion done")
    if args.kernel_sweep:
        rec["kernel_sweep"] = kernel_sweep(args)
        progress("kernel_sweep done")
    if not args.no_cpu:
        rec["cpu_baseline"] = cpu_baseline(C, args, ops)
        progress("cpu_baseline done")
    print(json.dumps(rec))


if __name__ == "__main__":
    main()
