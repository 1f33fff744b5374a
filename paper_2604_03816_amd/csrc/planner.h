// planner.h -- host-side circuit planner of libqsv: DAG construction (Section 5.1),
// DAG gate fusion (Section 5.2, Algorithm 2, Eq. 9) and HBM pass scheduling.
#pragma once
#include <complex>
#include <string>
#include <vector>

#include "../../include/qsv.h"
#include "qsv_internal.h"

namespace qsv {

using cd = std::complex<double>;

// A gate as given by the caller, already validated: dense 2^k x 2^k row-major matrix,
// local bit j <-> t[j].
struct InGate {
    int k;
    int t[kMaxK];
    std::vector<cd> m;
};

// A fused gate: targets ascending, dense matrix with local bit j <-> q[j].
struct FGate {
    int k = 0;
    int q[kMaxK] = {0, 0, 0, 0, 0};
    std::vector<cd> m;
    int kind = OP_DENSE;  // OP_DENSE, OP_DIAG or OP_PERM (classified from the matrix)
    int first = 0;        // smallest circuit index among the fused members
    int members = 1;
    unsigned long long dq = 0;  // physical qubits on which the op is diagonal (it commutes
                                // with Z on each of them): exactly-zero couplings
    std::vector<int> mem;       // circuit indices of the members, in the order the fused
                                // matrix applies them
};

struct PlanOpts {
    int fuse = 1;
    int commute = 1;           // fuse == 1 only: commutation-aware DAG, fusion and scheduling
    int kmax = 5;
    int cost_aware = 1;
    int tile_qubits = 12;
    int low_qubits = 4;
    int whole_state_max = 12;  // n <= this: the whole state is one on-chip tile
    double pass_budget = 160;  // FMA per amplitude per pass (<0: unlimited)
    double sigma = 8;          // per-op on-chip cost in FMA-per-amplitude units
    int max_ops_per_pass = 0;  // 0: no limit
    int mfma_min_k = 0;        // dense ops with k >= this run on MFMA; 0: never
    bool fp32_mfma = false;    // complex64: MFMA at twice the VALU rate (cost halved in planning)
    int mfma_lds_floats = 2048;  // per-pass cap of operand floats staged in LDS (MFMA matrices,
                                 // diagonal tables)
    int amp_floats = 2;        // floats per staged complex entry (2: complex64, 4: complex128)
};

struct PassPlan {
    std::vector<int> active;  // physical qubits held by the tile, ascending
    std::vector<int> ops;     // indices into HostPlan::fused
    int low = 0;              // qubits 0..low-1 are the contiguous low part of the tile
    double cost = 0;
};

struct HostPlan {
    int n = 0;
    int dtype = 0;
    PlanOpts o;
    size_t gates_in = 0;
    std::vector<int> shape;        // the input circuit's shape: per gate k, then its k targets
    std::vector<FGate> fused;
    std::vector<PassPlan> passes;
    // device-format tables
    std::vector<DevOp> ops;
    std::vector<PassArgs> pargs;
    std::vector<long long> pgrid;  // tiles per pass
    std::vector<char> pwide;       // pass has a VALU dense op on >= 4 targets or a permutation on
                                   // >= 3 (the register-heavy paths of the pass kernels)
    std::vector<cd> pool;
    std::vector<int> ipool;
    std::vector<float> apool;      // MFMA operand blocks, one contiguous block per pass
    // stats
    size_t dense_ops = 0, diag_ops = 0, perm_ops = 0, mfma_ops = 0;
    double fma_per_amp = 0, mfma_fma_per_amp = 0;
};

// Planner defaults for a dtype (QSV_C64 / QSV_C128).
PlanOpts default_opts(int dtype);

// Defaults overridden by the caller's public options (NULL: defaults only); checks the
// public ranges.  Returns false with a message on a bad value.
bool plan_opts_from(int dtype, const qsv_plan_opts* pub, PlanOpts& o, std::string& err);

// Arithmetic of one op, in FMA per amplitude (dense 4*2^k, diagonal 4, permutation 0
// or 4 with phases).
double op_fma(const FGate& g);

// Scheduling cost of one op on chip (excluding sigma): op_fma, halved for complex64 dense
// ops that run on FP32 MFMA (twice the non-packed VALU rate; FP64 MFMA has the FP64 VALU
// rate), and times 3/4 for 4-qubit dense ops on matrix cores (three real products per
// block instead of four) when the pass's operand block holds four of them.
double op_cost(const FGate& g, const PlanOpts& o);

// The per-pass operand block holds at least four 4-qubit matrices (the planner's defaults
// for both dtypes; not served complex128 passes, whose block is capped lower).
bool wide_operand_block(const PlanOpts& o);

// A dense op of o.mfma_min_k .. kMaxMfmaK qubits: it runs on matrix cores when its
// operand fits the pass's LDS operand block.
bool mfma_eligible(const FGate& g, const PlanOpts& o);

// Physical qubits on which a fused gate is diagonal: target q[j] counts when every entry
// coupling rows and columns that differ in local bit j is exactly zero.
unsigned long long diag_qubit_mask(const FGate& g);

// Two ops commute when on every qubit they share both are diagonal (both are then block
// diagonal over the shared qubits' basis states, with blocks on disjoint qubits).
bool ops_commute(const FGate& a, const FGate& b);

// Classifies a dense matrix: OP_DIAG when every off-diagonal entry is exactly zero,
// OP_PERM when every row and column holds exactly one nonzero, else OP_DENSE.
int classify(const std::vector<cd>& m, int k);

// Runs fusion (when o.fuse) and pass scheduling; fills every field of `out`.
bool make_plan(int n, int dtype, const std::vector<InGate>& gates, const PlanOpts& o,
               HostPlan& out, std::string& err);

// Re-fills plan P, made by make_plan for a circuit of the same shape (same gate count,
// same targets gate by gate), with the matrices of `gates`: every fused matrix is
// rebuilt as the product of its members' new matrices in the plan's order, and the
// device tables are rebuilt; the fusion and the passes are kept.  This is exact when
// the plan's structure still holds for the new matrices, which is checked: a diagonal
// op must stay diagonal, a permutation keep its pattern, and every op stay diagonal on
// the qubits the planner took it to be diagonal on (the commutations it relied on).
// Returns false, leaving P unchanged, when a check fails or a fused product was dropped
// as the identity; the caller then plans from scratch.  Meant for circuits whose
// structure is fixed while their parameters change (gradient sweeps over parameter
// vectors), with a template plan made from parameters with no special values.
bool refresh_plan(HostPlan& P, const std::vector<InGate>& gates);

// True when `gates` has the shape of the circuit P was made for: the same gate count and,
// gate by gate, the same targets in the same order.
bool same_shape(const HostPlan& P, const std::vector<InGate>& gates);

}  // namespace qsv
