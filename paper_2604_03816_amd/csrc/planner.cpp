// planner.cpp -- DAG gate fusion (Section 5.2, Algorithm 2) and HBM pass scheduling.
//
// DAG (Section 5.1): one scan keeps, per qubit, the most recent gate; the edges are
// these immediate per-qubit predecessors, so |E| <= sum |q(v)| (Eq. 8).  Here the DAG
// is stored as a doubly linked list of nodes per qubit ("line"): prev/next of a node
// on each of its qubits.
//
// Fusion (Algorithm 2): repeated sweeps in topological order; for each gate v and each
// predecessor u, merge v into u when
//   (1) u is a predecessor of v,
//   (2) |q(u) U q(v)| <= kmax  (q_max^fuse),
//   (3) u is v's predecessor on every shared qubit,
//   (4) the merge keeps the graph acyclic.  The paper's conditions (1)-(3) alone allow
//       merges that skip an intervening gate (u{0,1}, w{1,2}, v{0,2}: u and v share
//       qubit 0 with nothing between them there, yet w must run between them).  A merge
//       is sound iff no other path u ~> v exists; we accept it when every other
//       predecessor of v precedes u in the sweep's topological order (then none is a
//       descendant of u), or every other successor of u follows v (then no path from u
//       through them reaches v).  Either rule also gives the fused node a valid slot in
//       the order, so one order serves the whole sweep.
//   (5) cost-aware mode only: the fused op costs no more arithmetic than its parts
//       plus the per-op overhead it removes -- the trade-off of Eq. 13, where fused
//       gates have a higher per-gate cost c_2 than unfused ones (c_1).
// The fused matrix is U_v . U_u on the union of the targets (Eq. 9), each factor
// embedded as identity on the qubits it does not act on; products in FP64.
//
// Pass scheduling: the fused gates, in topological order, are grouped greedily into
// HBM passes.  A pass holds a tile of 2^m amplitudes on chip: the L lowest qubits
// (contiguous in memory, so every tile row is a coalesced run) plus up to m - L other
// qubits.  A gate joins the current pass when its targets fit in the tile, none of
// its qubits is blocked by an earlier deferred gate, and the pass's arithmetic budget
// allows.  Diagonal gates need no tile capacity: qubits outside the tile are
// constant within a tile, so their phase is a per-tile constant.
#include "planner.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <queue>

namespace qsv {

PlanOpts default_opts(int dtype)
{
    PlanOpts o;
    // Budgets: measured on the 30-qubit depth-20 brickwork (the pass count / per-pass
    // arithmetic trade-off that minimises total time).
    if (dtype == 0) {   // complex64: 8-byte amplitudes
        o.tile_qubits = 12;
        o.low_qubits = 4;
        o.whole_state_max = 13;
        o.pass_budget = 224;
        o.sigma = 8;
        o.mfma_min_k = 3;
        o.fp32_mfma = true;
        o.amp_floats = 2;
        o.mfma_lds_floats = 2048;  // 8 KiB: room for every 3- and 4-qubit op of a pass on
                                   // matrix cores (complex entries: 2 KiB per 4-qubit op)
                                   // with four workgroups per CU (32 KiB tiles)
    } else {            // complex128: 16-byte amplitudes
        o.tile_qubits = 12;
        o.low_qubits = 3;   // 8 contiguous amplitudes: 128-byte runs, as complex64's 16
        o.whole_state_max = 12;
        o.pass_budget = 320;
        o.sigma = 8;
        o.amp_floats = 4;
        o.mfma_min_k = 3;          // FP64 matrix cores: no faster than FP64 VALU in peak,
        o.mfma_lds_floats = 4096;  // but free of the VALU path's per-row scalar loads
    }
    return o;
}

bool plan_opts_from(int dtype, const qsv_plan_opts* pub, PlanOpts& o, std::string& err)
{
    o = default_opts(dtype);
    if (!pub) return true;
    if (pub->fuse < 0 || pub->fuse > 2) { err = "fuse must be 0, 1 or 2"; return false; }
    o.fuse = pub->fuse;
    if (pub->kmax) o.kmax = pub->kmax;
    if (pub->cost_aware) o.cost_aware = pub->cost_aware;
    if (pub->tile_qubits) o.tile_qubits = pub->tile_qubits;
    if (pub->low_qubits) o.low_qubits = pub->low_qubits;
    if (pub->pass_budget != 0) o.pass_budget = pub->pass_budget;
    if (pub->matrix_cores) {
        if (pub->matrix_cores != -1 && (pub->matrix_cores < 3 || pub->matrix_cores > kMaxMfmaK)) {
            err = "matrix_cores must be 0, -1, 3 or 4 (matrix-core ops have 3 or 4 targets)";
            return false;
        }
        o.mfma_min_k = pub->matrix_cores < 0 ? 0 : pub->matrix_cores;
    }
    if (pub->op_cost < 0) { err = "op_cost must be >= 0"; return false; }
    if (pub->op_cost > 0) o.sigma = pub->op_cost;
    if (pub->commute < -1 || pub->commute > 1) { err = "commute must be 0, 1 or -1"; return false; }
    if (pub->commute) o.commute = pub->commute > 0;
    if (o.fuse != 1) o.commute = 0;
    if (o.fuse == 0) o.max_ops_per_pass = 1;
    return true;
}

int classify(const std::vector<cd>& m, int k)
{
    const int d = 1 << k;
    bool diag = true;
    for (int r = 0; r < d && diag; ++r)
        for (int c = 0; c < d; ++c)
            if (r != c && m[(size_t)r * d + c] != cd(0, 0)) { diag = false; break; }
    if (diag) return OP_DIAG;
    std::vector<int> colcount(d, 0);
    for (int r = 0; r < d; ++r) {
        int cnt = 0;
        for (int c = 0; c < d; ++c)
            if (m[(size_t)r * d + c] != cd(0, 0)) { ++cnt; ++colcount[c]; }
        if (cnt != 1) return OP_DENSE;
    }
    for (int c = 0; c < d; ++c)
        if (colcount[c] != 1) return OP_DENSE;
    return OP_PERM;
}

unsigned long long diag_qubit_mask(const FGate& g)
{
    const int d = 1 << g.k;
    unsigned long long dq = 0;
    for (int j = 0; j < g.k; ++j) {
        bool diag = true;
        for (int r = 0; r < d && diag; ++r)
            for (int c = 0; c < d; ++c)
                if (((r ^ c) >> j) & 1 && g.m[(size_t)r * d + c] != cd(0, 0)) { diag = false; break; }
        if (diag) dq |= 1ull << g.q[j];
    }
    return dq;
}

bool ops_commute(const FGate& a, const FGate& b)
{
    unsigned long long qa = 0, qb = 0;
    for (int j = 0; j < a.k; ++j) qa |= 1ull << a.q[j];
    for (int j = 0; j < b.k; ++j) qb |= 1ull << b.q[j];
    const unsigned long long shared = qa & qb;
    return (shared & ~(a.dq & b.dq)) == 0;
}

double op_fma(const FGate& g)
{
    const int d = 1 << g.k;
    if (g.kind == OP_DENSE) return 4.0 * d;     // 2^k complex MACs per amplitude
    if (g.kind == OP_DIAG) return 4.0;          // one complex multiply
    for (int r = 0; r < d; ++r) {               // permutation: free unless it has phases
        for (int c = 0; c < d; ++c) {
            const cd v = g.m[(size_t)r * d + c];
            if (v != cd(0, 0) && v != cd(1, 0)) return 4.0;
        }
    }
    return 0.0;
}

double op_cost(const FGate& g, const PlanOpts& o)
{
    const double f = op_fma(g);
    if (mfma_eligible(g, o)) {
        // matrix cores: complex64 at twice the FP32 VALU rate; a 4-qubit op takes three
        // real products where its real embedding would take four (priced so only where
        // a pass can stage four of them)
        return (o.fp32_mfma ? 0.5 : 1.0) * (g.k == 4 && wide_operand_block(o) ? 0.75 : 1.0) * f;
    }
    return f;
}

bool wide_operand_block(const PlanOpts& o)
{
    return o.mfma_lds_floats >= 4 * (o.amp_floats << 8);
}

bool mfma_eligible(const FGate& g, const PlanOpts& o)
{
    return g.kind == OP_DENSE && o.mfma_min_k > 0 && g.k >= o.mfma_min_k && g.k <= kMaxMfmaK;
}

namespace {

bool is_identity(const FGate& g)
{
    const int d = 1 << g.k;
    for (int r = 0; r < d; ++r)
        for (int c = 0; c < d; ++c)
            if (g.m[(size_t)r * d + c] != (r == c ? cd(1, 0) : cd(0, 0))) return false;
    return true;
}

// Embed matrix `a` (local bit j <-> qa[j], ascending, ka bits) into the ascending qubit
// list Q (kq bits): E[r', r] = a[sub(r'), sub(r)] when r' and r agree outside qa, else 0.
std::vector<cd> embed(const std::vector<cd>& a, const int* qa, int ka, const int* Q, int kq)
{
    const int dq = 1 << kq;
    int pos[kMaxK];
    int amask = 0;
    for (int j = 0; j < ka; ++j) {
        int p = 0;
        while (Q[p] != qa[j]) ++p;
        pos[j] = p;
        amask |= 1 << p;
    }
    auto sub = [&](int r) {
        int s = 0;
        for (int j = 0; j < ka; ++j) s |= ((r >> pos[j]) & 1) << j;
        return s;
    };
    const int da = 1 << ka;
    if (ka == kq) return a;   // a spans Q: its targets are Q itself, in the same order
    int sr[1 << kMaxK];
    for (int r = 0; r < dq; ++r) sr[r] = sub(r);
    std::vector<cd> e((size_t)dq * dq, cd(0, 0));
    for (int r = 0; r < dq; ++r)
        for (int c = 0; c < dq; ++c)
            if ((r & ~amask) == (c & ~amask)) e[(size_t)r * dq + c] = a[(size_t)sr[r] * da + sr[c]];
    return e;
}

// E(v) . B for a dq x dq matrix B over the ascending qubit list Q, without forming E(v):
// row r of the product mixes the rows of B that differ from r only in v's bits, in
// ascending order: the sums of the plain product E(v) B, term for term (zero entries
// of E(v) skipped).
std::vector<cd> apply_left(const std::vector<cd>& vm, const int* qv, int kv, const int* Q, int kq,
                           const std::vector<cd>& B)
{
    const int dq = 1 << kq, dv = 1 << kv;
    int pos[kMaxK], vmask = 0;
    for (int j = 0; j < kv; ++j) {
        int p = 0;
        while (Q[p] != qv[j]) ++p;
        pos[j] = p;
        vmask |= 1 << p;
    }
    int spread[1 << kMaxK];
    for (int a = 0; a < dv; ++a) {
        int x = 0;
        for (int j = 0; j < kv; ++j) x |= ((a >> j) & 1) << pos[j];
        spread[a] = x;
    }
    std::vector<cd> C((size_t)dq * dq, cd(0, 0));
    for (int r = 0; r < dq; ++r) {
        int ra = 0;
        for (int j = 0; j < kv; ++j) ra |= ((r >> pos[j]) & 1) << j;
        const int base = r & ~vmask;
        cd* out = &C[(size_t)r * dq];
        for (int a = 0; a < dv; ++a) {
            const cd w = vm[(size_t)ra * dv + a];
            if (w == cd(0, 0)) continue;
            const cd* in = &B[(size_t)(base | spread[a]) * dq];
            for (int c = 0; c < dq; ++c) out[c] += w * in[c];
        }
    }
    return C;
}

// Canonical form of an input gate: ascending targets, rows/columns permuted to match.
FGate canonical(const InGate& g, int index)
{
    FGate f;
    f.k = g.k;
    int order[kMaxK];
    for (int j = 0; j < g.k; ++j) order[j] = j;
    std::sort(order, order + g.k, [&](int a, int b) { return g.t[a] < g.t[b]; });
    for (int j = 0; j < g.k; ++j) f.q[j] = g.t[order[j]];
    const int d = 1 << g.k;
    auto remap = [&](int r) {  // new local index -> old local index
        int o = 0;
        for (int j = 0; j < g.k; ++j) o |= ((r >> j) & 1) << order[j];
        return o;
    };
    f.m.assign((size_t)d * d, cd(0, 0));
    for (int r = 0; r < d; ++r)
        for (int c = 0; c < d; ++c) f.m[(size_t)r * d + c] = g.m[(size_t)remap(r) * d + remap(c)];
    f.kind = classify(f.m, f.k);
    f.dq = diag_qubit_mask(f);
    f.first = index;
    f.mem.assign(1, index);
    return f;
}

struct Node {
    FGate g;
    bool alive = true;
    int prev[kMaxK];  // per target slot: node index of the predecessor on that qubit, -1 if none
    int next[kMaxK];
};

int slot_of(const Node& nd, int qubit)
{
    for (int j = 0; j < nd.g.k; ++j)
        if (nd.g.q[j] == qubit) return j;
    return -1;
}

// Kahn's algorithm; ties broken by the smallest member circuit index (deterministic).
std::vector<int> topo_order(const std::vector<Node>& nodes)
{
    const int N = (int)nodes.size();
    std::vector<int> indeg(N, 0);
    for (int i = 0; i < N; ++i) {
        if (!nodes[i].alive) continue;
        int seen[kMaxK], ns = 0;
        for (int j = 0; j < nodes[i].g.k; ++j) {
            const int p = nodes[i].prev[j];
            if (p < 0) continue;
            bool dup = false;
            for (int s = 0; s < ns; ++s) dup |= seen[s] == p;
            if (!dup) seen[ns++] = p;
        }
        indeg[i] = ns;
    }
    using Item = std::pair<int, int>;  // (first, node)
    std::priority_queue<Item, std::vector<Item>, std::greater<Item>> ready;
    for (int i = 0; i < N; ++i)
        if (nodes[i].alive && indeg[i] == 0) ready.push({nodes[i].g.first, i});
    std::vector<int> order;
    order.reserve(N);
    while (!ready.empty()) {
        const int u = ready.top().second;
        ready.pop();
        order.push_back(u);
        int seen[kMaxK], ns = 0;
        for (int j = 0; j < nodes[u].g.k; ++j) {
            const int s = nodes[u].next[j];
            if (s < 0) continue;
            bool dup = false;
            for (int t = 0; t < ns; ++t) dup |= seen[t] == s;
            if (dup) continue;
            seen[ns++] = s;
            if (--indeg[s] == 0) ready.push({nodes[s].g.first, s});
        }
    }
    return order;
}

FGate fuse_pair(const FGate& u, const FGate& v, int kmax, bool& ok)
{
    int Q[2 * kMaxK], kq = 0;
    for (int j = 0; j < u.k; ++j) Q[kq++] = u.q[j];
    for (int j = 0; j < v.k; ++j) {
        bool dup = false;
        for (int i = 0; i < u.k; ++i) dup |= u.q[i] == v.q[j];
        if (!dup) Q[kq++] = v.q[j];
    }
    ok = kq <= kmax;
    FGate f;
    if (!ok) return f;
    std::sort(Q, Q + kq);
    f.k = kq;
    for (int j = 0; j < kq; ++j) f.q[j] = Q[j];
    // Eq. 9: U_fused = U_v . U_u (u applied first)
    f.m = apply_left(v.m, v.q, v.k, Q, kq, embed(u.m, u.q, u.k, Q, kq));
    f.kind = classify(f.m, kq);
    f.dq = diag_qubit_mask(f);
    f.first = std::min(u.first, v.first);
    f.members = u.members + v.members;
    f.mem = u.mem;
    f.mem.insert(f.mem.end(), v.mem.begin(), v.mem.end());
    return f;
}

void run_fusion(std::vector<Node>& nodes, const PlanOpts& o)
{
    const int N = (int)nodes.size();
    std::vector<int> pos(N, 0);
    bool changed = true;
    while (changed) {
        changed = false;
        const std::vector<int> order = topo_order(nodes);
        for (int i = 0; i < (int)order.size(); ++i) pos[order[i]] = i;
        for (const int v : order) {
            if (!nodes[v].alive) continue;
            // distinct predecessors of v, nearest (latest in the order) first
            int preds[kMaxK], np = 0;
            for (int j = 0; j < nodes[v].g.k; ++j) {
                const int p = nodes[v].prev[j];
                if (p < 0) continue;
                bool dup = false;
                for (int s = 0; s < np; ++s) dup |= preds[s] == p;
                if (!dup) preds[np++] = p;
            }
            std::sort(preds, preds + np, [&](int a, int b) { return pos[a] > pos[b]; });
            for (int pi = 0; pi < np; ++pi) {
                const int u = preds[pi];
                Node& U = nodes[u];
                Node& V = nodes[v];
                // (3) u is v's predecessor on every shared qubit
                bool sole = true;
                for (int j = 0; j < V.g.k && sole; ++j)
                    if (slot_of(U, V.g.q[j]) >= 0 && V.prev[j] != u) sole = false;
                if (!sole) continue;
                // (4) acyclicity, by rule A (other preds of v precede u) or
                //     rule B (other succs of u follow v)
                bool ruleA = true, ruleB = true;
                for (int j = 0; j < V.g.k; ++j) {
                    const int p = V.prev[j];
                    if (p >= 0 && p != u && pos[p] > pos[u]) ruleA = false;
                }
                for (int j = 0; j < U.g.k; ++j) {
                    const int s = U.next[j];
                    if (s >= 0 && s != v && pos[s] < pos[v]) ruleB = false;
                }
                if (!ruleA && !ruleB) continue;
                // (2) width, checked before any product is formed
                {
                    unsigned long long qm = 0;
                    for (int j = 0; j < U.g.k; ++j) qm |= 1ull << U.g.q[j];
                    for (int j = 0; j < V.g.k; ++j) qm |= 1ull << V.g.q[j];
                    const int kq = __builtin_popcountll(qm);
                    if (kq > o.kmax) continue;
                    // (5), predicted: a product with a dense factor is dense (exact
                    // cancellation to a cheaper kind is rare and only costs a missed merge)
                    if (o.cost_aware > 0 && (U.g.kind == OP_DENSE || V.g.kind == OP_DENSE)) {
                        FGate probe;
                        probe.k = kq;
                        probe.kind = OP_DENSE;
                        if (op_cost(probe, o) > op_cost(U.g, o) + op_cost(V.g, o) + o.sigma) continue;
                    }
                }
                bool ok = false;
                FGate f = fuse_pair(U.g, V.g, o.kmax, ok);
                if (!ok) continue;
                // (5) arithmetic does not grow beyond what the merge saves
                if (o.cost_aware > 0 && op_cost(f, o) > op_cost(U.g, o) + op_cost(V.g, o) + o.sigma) continue;
                // merge v into u: relink the per-qubit lines
                int nprev[kMaxK], nnext[kMaxK];
                for (int j = 0; j < f.k; ++j) {
                    const int x = f.q[j];
                    const int su = slot_of(U, x), sv = slot_of(V, x);
                    if (su >= 0 && sv >= 0) {
                        nprev[j] = U.prev[su];
                        nnext[j] = V.next[sv];
                    } else if (su >= 0) {
                        nprev[j] = U.prev[su];
                        nnext[j] = U.next[su];
                    } else {
                        nprev[j] = V.prev[sv];
                        nnext[j] = V.next[sv];
                    }
                }
                for (int j = 0; j < f.k; ++j) {
                    const int x = f.q[j];
                    if (nprev[j] >= 0) {
                        Node& P = nodes[nprev[j]];
                        P.next[slot_of(P, x)] = u;
                    }
                    if (nnext[j] >= 0) {
                        Node& S = nodes[nnext[j]];
                        S.prev[slot_of(S, x)] = u;
                    }
                }
                U.g = std::move(f);
                for (int j = 0; j < U.g.k; ++j) {
                    U.prev[j] = nprev[j];
                    U.next[j] = nnext[j];
                }
                V.alive = false;
                if (!ruleA) pos[u] = pos[v];  // rule B: the fused node takes v's slot
                changed = true;
                break;
            }
        }
    }
}

// ---- commutation-aware DAG and fusion (option commute)
//
// Two ops commute when they are both diagonal on every qubit they share, so among the
// ops touching a qubit q only the order between a run of ops diagonal on q and the op
// not diagonal on q that ends the run matters.  The DAG below keeps exactly those
// per-qubit edges: an op diagonal on q depends on the last op not diagonal on q; an op
// not diagonal on q depends on every op of the diagonal run before it (or, without
// one, on the previous op not diagonal on q).  Every pair of ops that may not commute
// is then joined by a path, so any topological order applies the circuit's operator.
//
// Fusion follows the sweep of Algorithm 2 on this DAG.  Its candidates for v are v's
// DAG predecessors and, on each qubit of v, the nearest earlier ops that commute with v
// there (they have no edge to v: a diagonal run); a merge needs the width bound, rule
// A or rule B (either one rules out any path u ~> v besides a direct edge, which also
// makes u and v commute when they have no edge, so the product order U_v . U_u is
// right either way) and, in cost-aware mode, the arithmetic condition.
struct CNode {
    FGate g;
    bool alive = true;
    unsigned long long qm = 0;
    std::vector<int> pred, succ;
};

unsigned long long qubit_mask(const FGate& g)
{
    unsigned long long m = 0;
    for (int j = 0; j < g.k; ++j) m |= 1ull << g.q[j];
    return m;
}

void add_edge(std::vector<CNode>& N, int a, int b)
{
    if (a < 0 || a == b) return;
    std::vector<int>& s = N[a].succ;
    if (std::find(s.begin(), s.end(), b) != s.end()) return;
    s.push_back(b);
    N[b].pred.push_back(a);
}

// Kahn's algorithm over the edge lists; ties broken by the smallest member index.
std::vector<int> topo_order_dag(const std::vector<CNode>& N)
{
    const int G = (int)N.size();
    std::vector<int> indeg(G, 0);
    using Item = std::pair<int, int>;
    std::priority_queue<Item, std::vector<Item>, std::greater<Item>> ready;
    for (int i = 0; i < G; ++i) {
        if (!N[i].alive) continue;
        indeg[i] = (int)N[i].pred.size();
        if (indeg[i] == 0) ready.push({N[i].g.first, i});
    }
    std::vector<int> order;
    order.reserve(G);
    while (!ready.empty()) {
        const int u = ready.top().second;
        ready.pop();
        order.push_back(u);
        for (const int s : N[u].succ)
            if (--indeg[s] == 0) ready.push({N[s].g.first, s});
    }
    return order;
}

// In node x's list, replace `from` by `to` (dropping `from` when `to` is already there).
void relink(std::vector<int>& lst, int from, int to)
{
    const bool has_to = std::find(lst.begin(), lst.end(), to) != lst.end();
    for (size_t i = 0; i < lst.size(); ++i) {
        if (lst[i] != from) continue;
        if (has_to) lst.erase(lst.begin() + (long)i);
        else lst[i] = to;
        return;
    }
}

std::vector<FGate> fuse_commuting(const std::vector<FGate>& gates, int n, const PlanOpts& o, bool diag_only)
{
    const int G = (int)gates.size();
    std::vector<CNode> N(G);
    {
        std::vector<int> last_nd(n, -1);
        std::vector<std::vector<int>> run(n);
        for (int i = 0; i < G; ++i) {
            N[i].g = gates[i];
            N[i].qm = qubit_mask(gates[i]);
            for (int j = 0; j < gates[i].k; ++j) {
                const int q = gates[i].q[j];
                if ((gates[i].dq >> q) & 1) {
                    add_edge(N, last_nd[q], i);
                    run[q].push_back(i);
                } else {
                    if (run[q].empty()) add_edge(N, last_nd[q], i);
                    for (const int r : run[q]) add_edge(N, r, i);
                    run[q].clear();
                    last_nd[q] = i;
                }
            }
        }
    }
    constexpr int kWindow = 8;   // commuting candidates examined per qubit of v
    std::vector<int> pos(G, 0);
    std::vector<std::vector<int>> lines(n);
    std::vector<int> at((size_t)G * kMaxK, -1), atq((size_t)G * kMaxK, -1);
    bool changed = true;
    while (changed) {
        changed = false;
        const std::vector<int> order = topo_order_dag(N);
        for (int i = 0; i < (int)order.size(); ++i) pos[order[i]] = i;
        // per-qubit lists of the live ops in this sweep's order
        for (auto& l : lines) l.clear();
        for (const int v : order)
            for (int j = 0; j < N[v].g.k; ++j) {
                const int q = N[v].g.q[j];
                atq[(size_t)v * kMaxK + j] = q;
                at[(size_t)v * kMaxK + j] = (int)lines[q].size();
                lines[q].push_back(v);
            }
        const std::vector<int> snapshot_k = [&] {
            std::vector<int> k(G, 0);
            for (const int v : order) k[v] = N[v].g.k;
            return k;
        }();
        std::vector<int> cand;
        for (const int v : order) {
            if (!N[v].alive) continue;
            cand.assign(N[v].pred.begin(), N[v].pred.end());
            for (int j = 0; j < snapshot_k[v]; ++j) {
                const int q = atq[(size_t)v * kMaxK + j];
                const std::vector<int>& line = lines[q];
                int seen = 0;
                for (int t = at[(size_t)v * kMaxK + j] - 1; t >= 0 && seen < kWindow; --t) {
                    const int u = line[t];
                    if (!N[u].alive || u == v || !((N[u].qm >> q) & 1)) continue;
                    ++seen;
                    cand.push_back(u);
                    if (!ops_commute(N[u].g, N[v].g)) break;   // ops further back are ordered before u
                }
            }
            std::sort(cand.begin(), cand.end());
            cand.erase(std::unique(cand.begin(), cand.end()), cand.end());
            std::sort(cand.begin(), cand.end(), [&](int a, int b) { return pos[a] > pos[b]; });
            for (const int u : cand) {
                CNode& U = N[u];
                CNode& V = N[v];
                if (!U.alive || u == v || pos[u] >= pos[v] || !(U.qm & V.qm)) continue;
                if (diag_only && (U.g.kind != OP_DIAG || V.g.kind != OP_DIAG)) continue;
                const int kq = __builtin_popcountll(U.qm | V.qm);
                if (kq > o.kmax) continue;
                bool ruleA = true, ruleB = true;
                for (const int p : V.pred)
                    if (p != u && pos[p] > pos[u]) { ruleA = false; break; }
                for (const int sx : U.succ)
                    if (sx != v && pos[sx] < pos[v]) { ruleB = false; break; }
                if (!ruleA && !ruleB) continue;
                if (o.cost_aware > 0 && (U.g.kind == OP_DENSE || V.g.kind == OP_DENSE)) {
                    FGate probe;
                    probe.k = kq;
                    probe.kind = OP_DENSE;
                    if (op_cost(probe, o) > op_cost(U.g, o) + op_cost(V.g, o) + o.sigma) continue;
                }
                bool ok = false;
                FGate f = fuse_pair(U.g, V.g, o.kmax, ok);
                if (!ok) continue;
                if (o.cost_aware > 0 && op_cost(f, o) > op_cost(U.g, o) + op_cost(V.g, o) + o.sigma) continue;
                // merge v into u: u takes v's edges
                for (const int p : V.pred) {
                    if (p == u) continue;
                    relink(N[p].succ, v, u);
                    if (std::find(U.pred.begin(), U.pred.end(), p) == U.pred.end()) U.pred.push_back(p);
                }
                for (const int sx : V.succ) {
                    relink(N[sx].pred, v, u);
                    if (std::find(U.succ.begin(), U.succ.end(), sx) == U.succ.end()) U.succ.push_back(sx);
                }
                U.succ.erase(std::remove(U.succ.begin(), U.succ.end(), v), U.succ.end());
                U.g = std::move(f);
                U.qm = qubit_mask(U.g);
                V.alive = false;
                V.pred.clear();
                V.succ.clear();
                if (!ruleA) pos[u] = pos[v];   // rule B: the fused op takes v's slot
                changed = true;
                break;
            }
        }
    }
    std::vector<FGate> out;
    for (const int v : topo_order_dag(N)) out.push_back(N[v].g);
    return out;
}

// One pass built greedily from the ops not yet done (in their order).  grow: the tile
// starts as `A0` and takes the qubits of every op that joins, up to m; otherwise the
// tile is exactly `A0` and only ops inside it (or diagonal ops) join.  An op joins when
// none of its qubits is blocked by an earlier deferred op it may not commute with, the
// tile holds it and the pass's arithmetic budget allows.
PassPlan build_pass(int n, const std::vector<FGate>& fused, const std::vector<char>& done, const PlanOpts& o,
                    int m, int L, bool whole, unsigned long long A0, bool grow)
{
    const int F = (int)fused.size();
    const unsigned long long all = (n >= 64) ? ~0ull : ((1ull << n) - 1);
    PassPlan pp;
    int Lp = L;   // low qubits kept in this pass's tile
    unsigned long long A = whole ? all : A0;
    // qubits of deferred ops: where some deferred op is not diagonal (blocked), and
    // where all of them are (blocked_d).  A later op may run ahead of the deferred
    // ones when it touches no blocked qubit and is itself diagonal on every
    // blocked_d qubit it touches: it then commutes with each of them.
    unsigned long long blocked = 0, blocked_d = 0;
    auto defer = [&](unsigned long long gm, unsigned long long gd) {
        blocked |= gm & ~gd;
        blocked_d |= gm & gd;
        blocked_d &= ~blocked;
    };
    double budget = o.pass_budget;
    int afl = 0;   // operand floats staged so far, as the device tables stage them
    for (int i = 0; i < F; ++i) {
        if (done[i]) continue;
        const FGate& g = fused[i];
        unsigned long long gm = 0;
        for (int j = 0; j < g.k; ++j) gm |= 1ull << g.q[j];
        const unsigned long long gd = o.commute ? g.dq : 0;
        if ((gm & blocked) || (gm & ~gd & blocked_d)) { defer(gm, gd); continue; }
        const double c = op_cost(g, o) + o.sigma;
        const bool limit_ops = o.max_ops_per_pass > 0 && (int)pp.ops.size() >= o.max_ops_per_pass;
        // a matrix-core op whose operand no longer fits the pass's block would run on the
        // VALU at several times its planned cost: it waits for the next pass instead
        // (diagonal tables are staged too, where they fit).  With a block too small for
        // four 4-qubit matrices (served complex128 passes) that would cost more passes
        // than the VALU fallback: there the op stays in the pass.
        const bool mf = mfma_eligible(g, o);
        const int af = mf ? o.amp_floats << (2 * g.k) : g.kind == OP_DIAG ? o.amp_floats << g.k : 0;
        const bool fits_operands = whole || !mf || !wide_operand_block(o) ||
                                   ((afl + 3) & ~3) + af <= o.mfma_lds_floats || pp.ops.empty();
        const bool fits_budget = whole || o.pass_budget < 0 || c <= budget || pp.ops.empty();
        unsigned long long nA = (g.kind == OP_DIAG) ? A : (A | gm);
        if (grow && pp.ops.empty() && __builtin_popcountll(nA) > m) {
            // a gate wider than the tile's free slots opens a pass with fewer low qubits
            while (Lp > 0 && __builtin_popcountll(gm | ((1ull << Lp) - 1)) > m) --Lp;
            A = (1ull << Lp) - 1;
            nA = A | gm;
        }
        const bool fits_tile = grow ? __builtin_popcountll(nA) <= m : nA == A;
        if (!limit_ops && fits_budget && fits_operands && fits_tile) {
            A = nA;
            pp.ops.push_back(i);
            budget -= c;
            pp.cost += c;
            if (af > 0 && ((afl + 3) & ~3) + af <= o.mfma_lds_floats) afl = ((afl + 3) & ~3) + af;
        } else {
            defer(gm, gd);
            if ((blocked & all) == all) break;
        }
    }
    // fill the tile up to m qubits with the lowest unused qubits (longer runs)
    for (int b = 0; b < n && __builtin_popcountll(A) < m; ++b) A |= 1ull << b;
    for (int b = 0; b < n; ++b)
        if ((A >> b) & 1) pp.active.push_back(b);
    pp.low = Lp;
    return pp;
}

// Diagonal ops on disjoint qubits share no DAG edge, so fusion leaves them apart, yet
// they commute and their product is again diagonal, costing one complex multiply per
// amplitude like each of them (a layer of single-qubit phase rotations would otherwise
// cost one on-chip round trip per qubit).  Walking the fused list in order, a diagonal
// op moves back past every op it commutes with to the nearest earlier diagonal op whose
// union with it stays within the width bound, and the two become one.  Moving it back
// is exact: it commutes with every op it passes.
void merge_diagonals(std::vector<FGate>& ops, int kmax)
{
    constexpr int kWindow = 64;   // earlier ops examined per diagonal op
    std::vector<FGate> out;
    out.reserve(ops.size());
    for (FGate& v : ops) {
        if (v.kind == OP_DIAG) {
            const unsigned long long qv = qubit_mask(v);
            int hit = -1;
            for (int t = (int)out.size() - 1, seen = 0; t >= 0 && seen < kWindow; --t, ++seen) {
                const FGate& u = out[(size_t)t];
                if (u.kind == OP_DIAG && __builtin_popcountll(qubit_mask(u) | qv) <= kmax) {
                    hit = t;
                    break;
                }
                if (!ops_commute(u, v)) break;
            }
            if (hit >= 0) {
                bool ok = false;
                FGate f = fuse_pair(out[(size_t)hit], v, kmax, ok);
                if (ok && f.kind == OP_DIAG) {
                    out[(size_t)hit] = std::move(f);
                    continue;
                }
            }
        }
        out.push_back(std::move(v));
    }
    ops.clear();
    for (FGate& g : out)
        if (!is_identity(g)) ops.push_back(std::move(g));
}

// Pass scheduling.  Each pass is the best of several greedy candidates: the tile that
// grows with the ops in their order, and tiles fixed in advance to the low L qubits
// plus m - L consecutive others (every window position).  The fixed windows follow the
// locality of nearest-neighbour circuits: within a window an op can run several layers
// ahead of the ops outside it, where the growing tile stops at the first op that
// straddles its edge.  "Best" is the most arithmetic (plus per-op overhead) done, the
// growing tile winning ties; it always makes progress.
bool schedule_passes(int n, const std::vector<FGate>& fused, const PlanOpts& o, std::vector<PassPlan>& passes,
                     std::string& err)
{
    passes.clear();
    const int F = (int)fused.size();
    const bool whole = o.fuse && n <= o.whole_state_max;
    const int m = whole ? n : std::min(o.tile_qubits, n);
    const int L = std::min(o.low_qubits, m);
    const unsigned long long low = (L >= 64) ? ~0ull : ((1ull << L) - 1);
    const bool windows = !whole && o.fuse == 1 && n > m && m > L;
    std::vector<char> done(F, 0);
    int remaining = F;
    while (remaining > 0) {
        PassPlan best = build_pass(n, fused, done, o, m, L, whole, low, true);
        if (windows) {
            const int w = m - L;
            for (int a = L; a + w <= n; ++a) {
                const unsigned long long A0 = low | (((1ull << w) - 1) << a);
                PassPlan c = build_pass(n, fused, done, o, m, L, whole, A0, false);
                if (c.cost > best.cost) best = std::move(c);
            }
        }
        if (best.ops.empty()) { err = "internal: a gate does not fit any tile"; return false; }
        for (const int i : best.ops) done[i] = 1;
        remaining -= (int)best.ops.size();
        passes.push_back(std::move(best));
    }
    return true;
}

// Device tables of a planned circuit (op descriptors, matrix pools, staged operand
// blocks, pass arguments) and the arithmetic statistics, from P.fused and P.passes.
void build_device_tables(HostPlan& P)
{
    const int n = P.n, dtype = P.dtype;
    const PlanOpts& o = P.o;
    P.ops.clear();
    P.pargs.clear();
    P.pgrid.clear();
    P.pwide.clear();
    P.pool.clear();
    P.ipool.clear();
    P.apool.clear();
    P.dense_ops = P.diag_ops = P.perm_ops = P.mfma_ops = 0;
    P.fma_per_amp = P.mfma_fma_per_amp = 0;
    for (const PassPlan& pp : P.passes) {
        PassArgs a{};
        a.m = (int)pp.active.size();
        a.L = pp.low;
        for (int i = 0; i < a.m; ++i) a.phys[i] = (unsigned char)pp.active[i];
        a.nruns = 0;
        {
            unsigned long long A = 0;
            for (int b : pp.active) A |= 1ull << b;
            int b = 0;
            while (b < n) {
                if ((A >> b) & 1) { ++b; continue; }
                int s = b;
                while (b < n && !((A >> b) & 1)) ++b;
                a.run_pos[a.nruns] = (unsigned char)s;
                a.run_len[a.nruns] = (unsigned char)(b - s);
                ++a.nruns;
            }
        }
        a.op_begin = (int)P.ops.size();
        a.op_count = (int)pp.ops.size();
        a.a_off = (int)P.apool.size();
        a.a_len = 0;
        for (const int fi : pp.ops) {
            const FGate& g = P.fused[fi];
            DevOp d{};
            d.kind = g.kind;
            d.k = g.k;
            for (int j = 0; j < kMaxK; ++j) { d.lpos[j] = -1; d.gbit[j] = 0; }
            for (int j = 0; j < g.k; ++j) {
                d.gbit[j] = g.q[j];
                auto it = std::find(pp.active.begin(), pp.active.end(), g.q[j]);
                d.lpos[j] = (it == pp.active.end()) ? -1 : (int)(it - pp.active.begin());
            }
            const int dd = 1 << g.k;
            d.off = (int)P.pool.size();
            d.aoff = -1;
            if (g.kind == OP_DENSE) {
                P.pool.insert(P.pool.end(), g.m.begin(), g.m.end());
                ++P.dense_ops;
                // the matrix for the matrix cores: 2^k x 2^k complex entries, entry (r, c) at
                // r 2^k + (c ^ (r % 8)) (the kernel's reads then spread over the LDS
                // banks), in the state's precision as raw floats (the kernel forms its
                // real operands in registers), 16-byte aligned
                const int per = dtype == 0 ? 2 : 4;
                const int af = per * dd * dd;
                const int at = (a.a_len + 3) & ~3;
                if (o.mfma_min_k > 0 && g.k >= o.mfma_min_k && g.k <= kMaxMfmaK && (1 << (a.m - g.k)) >= 16 &&
                    at + af <= o.mfma_lds_floats) {
                    P.apool.resize((size_t)a.a_off + at, 0.0f);
                    d.aoff = at;
                    for (int e = 0; e < dd * dd; ++e) {
                        const int r = e / dd, c = (e % dd) ^ (r & 7);
                        const cd v = g.m[(size_t)r * dd + c];
                        if (dtype == 0) {
                            P.apool.push_back((float)v.real());
                            P.apool.push_back((float)v.imag());
                        } else {
                            const double re = v.real(), im = v.imag();
                            float w[4];
                            std::memcpy(w, &re, 8);
                            std::memcpy(w + 2, &im, 8);
                            P.apool.insert(P.apool.end(), w, w + 4);
                        }
                    }
                    a.a_len = at + af;
                    ++P.mfma_ops;
                    P.mfma_fma_per_amp += op_fma(g);
                }
            } else if (g.kind == OP_DIAG) {
                for (int r = 0; r < dd; ++r) P.pool.push_back(g.m[(size_t)r * dd + r]);
                ++P.diag_ops;
                // the table also goes to LDS (per-lane lookups stay on chip): the entries
                // in the state's precision as raw floats, 16-byte aligned
                const int per = dtype == 0 ? 2 : 4;
                const int at = (a.a_len + 3) & ~3;
                if (at + per * dd <= o.mfma_lds_floats) {
                    P.apool.resize((size_t)a.a_off + at, 0.0f);
                    for (int r = 0; r < dd; ++r) {
                        const cd v = g.m[(size_t)r * dd + r];
                        if (dtype == 0) {
                            P.apool.push_back((float)v.real());
                            P.apool.push_back((float)v.imag());
                        } else {
                            const double re = v.real(), im = v.imag();
                            float w[4];
                            std::memcpy(w, &re, 8);
                            std::memcpy(w + 2, &im, 8);
                            P.apool.insert(P.apool.end(), w, w + 4);
                        }
                    }
                    d.aoff = at;
                    a.a_len = at + per * dd;
                }
            } else {
                d.ioff = (int)P.ipool.size();
                d.flags = 0;
                for (int r = 0; r < dd; ++r) {
                    int src = 0;
                    for (int c = 0; c < dd; ++c)
                        if (g.m[(size_t)r * dd + c] != cd(0, 0)) src = c;
                    const cd ph = g.m[(size_t)r * dd + src];
                    P.ipool.push_back(src);
                    P.pool.push_back(ph);
                    if (ph != cd(1, 0)) d.flags = 1;
                }
                ++P.perm_ops;
            }
            P.fma_per_amp += op_fma(g);
            P.ops.push_back(d);
        }
        {
            bool wide = false;
            for (int i = a.op_begin; i < a.op_begin + a.op_count; ++i) {
                const DevOp& d = P.ops[(size_t)i];
                wide |= (d.kind == OP_DENSE && d.aoff < 0 && d.k >= 4) || (d.kind == OP_PERM && d.k >= 3);
            }
            P.pwide.push_back(wide ? 1 : 0);
        }
        P.pargs.push_back(a);
        P.pgrid.push_back(1ll << (n - a.m));
    }
}

}  // namespace

bool make_plan(int n, int dtype, const std::vector<InGate>& gates, const PlanOpts& o,
               HostPlan& P, std::string& err)
{
    P = HostPlan();
    P.n = n;
    P.dtype = dtype;
    P.o = o;
    P.gates_in = gates.size();
    for (const InGate& g : gates) {
        P.shape.push_back(g.k);
        P.shape.insert(P.shape.end(), g.t, g.t + g.k);
    }
    if (o.kmax < 1 || o.kmax > kMaxK) { err = "kmax must be in [1, 5]"; return false; }
    if (o.low_qubits < 1 || o.low_qubits > kLogThreads) { err = "low_qubits must be in [1, 8]"; return false; }
    if (o.tile_qubits < o.low_qubits + 1 || o.tile_qubits < kMaxK + 1 || o.tile_qubits > kMaxTileQubits) {
        err = "tile_qubits must be in [max(low_qubits+1, 6), 13]";
        return false;
    }

    // ---- DAG (Section 5.1): immediate predecessor per qubit
    std::vector<Node> nodes(gates.size());
    std::vector<int> last(n, -1);
    for (size_t i = 0; i < gates.size(); ++i) {
        Node& nd = nodes[i];
        nd.g = canonical(gates[i], (int)i);
        for (int j = 0; j < nd.g.k; ++j) {
            const int x = nd.g.q[j];
            nd.prev[j] = last[x];
            nd.next[j] = -1;
            if (last[x] >= 0) {
                Node& p = nodes[last[x]];
                p.next[slot_of(p, x)] = (int)i;
            }
            last[x] = (int)i;
        }
    }

    // ---- Algorithm 2 on the per-qubit DAG; with `commute`, diagonal ops are then also
    // merged across the commutation-aware DAG, and the whole fusion is run a second time
    // on that DAG: the plan with fewer passes (then less arithmetic) is kept
    {
        if (o.fuse == 1) run_fusion(nodes, o);
        std::vector<FGate> in;
        for (const int v : topo_order(nodes)) in.push_back(nodes[v].g);
        if (o.fuse == 1 && o.commute) in = fuse_commuting(in, n, o, true);
        for (FGate& g : in)
            if (!is_identity(g)) P.fused.push_back(std::move(g));
        if (o.fuse == 1 && o.commute) merge_diagonals(P.fused, o.kmax);
    }
    if (!schedule_passes(n, P.fused, o, P.passes, err)) return false;
    if (o.fuse == 1 && o.commute) {
        std::vector<FGate> in;
        in.reserve(gates.size());
        for (size_t i = 0; i < gates.size(); ++i) in.push_back(canonical(gates[i], (int)i));
        std::vector<FGate> alt;
        for (FGate& g : fuse_commuting(in, n, o, false))
            if (!is_identity(g)) alt.push_back(std::move(g));
        merge_diagonals(alt, o.kmax);
        std::vector<PassPlan> alt_passes;
        if (!schedule_passes(n, alt, o, alt_passes, err)) return false;
        auto arith = [&](const std::vector<FGate>& f) {
            double a = 0;
            for (const FGate& g : f) a += op_cost(g, o);
            return a;
        };
        if (alt_passes.size() < P.passes.size() ||
            (alt_passes.size() == P.passes.size() && arith(alt) < arith(P.fused))) {
            P.fused.swap(alt);
            P.passes.swap(alt_passes);
        }
    }

    build_device_tables(P);
    return true;
}


namespace {

// M <- E(g) M for a d x d matrix M over the fused op's targets: g's local bit j sits at
// M's local bit pos[j].  Each column of M is transformed like a state vector.
void apply_on_rows(std::vector<cd>& M, int d, const InGate& g, const int* pos)
{
    const int dg = 1 << g.k;
    int mask = 0;
    for (int j = 0; j < g.k; ++j) mask |= 1 << pos[j];
    int rows[1 << kMaxK];
    cd in[1 << kMaxK];
    for (int r0 = 0; r0 < d; ++r0) {
        if (r0 & mask) continue;
        for (int a = 0; a < dg; ++a) {
            int r = r0;
            for (int j = 0; j < g.k; ++j)
                if ((a >> j) & 1) r |= 1 << pos[j];
            rows[a] = r;
        }
        for (int c = 0; c < d; ++c) {
            for (int a = 0; a < dg; ++a) in[a] = M[(size_t)rows[a] * d + c];
            for (int a = 0; a < dg; ++a) {
                double re = 0, im = 0;   // plain products: every value here is finite
                for (int b = 0; b < dg; ++b) {
                    const cd u = g.m[(size_t)a * dg + b];
                    re += u.real() * in[b].real() - u.imag() * in[b].imag();
                    im += u.real() * in[b].imag() + u.imag() * in[b].real();
                }
                M[(size_t)rows[a] * d + c] = cd(re, im);
            }
        }
    }
}

}  // namespace

bool same_shape(const HostPlan& P, const std::vector<InGate>& gates)
{
    if (gates.size() != P.gates_in) return false;
    size_t at = 0;
    for (const InGate& g : gates) {
        if (at + 1 + (size_t)g.k > P.shape.size() || P.shape[at] != g.k) return false;
        for (int j = 0; j < g.k; ++j)
            if (P.shape[at + 1 + (size_t)j] != g.t[j]) return false;
        at += 1 + (size_t)g.k;
    }
    return at == P.shape.size();
}

bool refresh_plan(HostPlan& P, const std::vector<InGate>& gates)
{
    if (!same_shape(P, gates)) return false;
    size_t covered = 0;
    for (const FGate& f : P.fused) covered += f.mem.size();
    if (covered != gates.size()) return false;   // a product was dropped as the identity
    std::vector<std::vector<cd>> mats(P.fused.size());
    for (size_t fi = 0; fi < P.fused.size(); ++fi) {
        const FGate& f = P.fused[fi];
        const int d = 1 << f.k;
        std::vector<cd>& M = mats[fi];
        M.assign((size_t)d * d, cd(0, 0));
        for (int r = 0; r < d; ++r) M[(size_t)r * d + r] = cd(1, 0);
        for (const int i : f.mem) {
            if (i < 0 || (size_t)i >= gates.size()) return false;
            const InGate& g = gates[(size_t)i];
            int pos[kMaxK];
            for (int j = 0; j < g.k; ++j) {
                pos[j] = -1;
                for (int t = 0; t < f.k; ++t)
                    if (f.q[t] == g.t[j]) pos[j] = t;
                if (pos[j] < 0) return false;   // not the circuit the plan was made for
            }
            if ((int)g.m.size() != (1 << (2 * g.k))) return false;
            apply_on_rows(M, d, g, pos);
        }
        // the structure the planner used must still hold
        FGate probe;
        probe.k = f.k;
        for (int j = 0; j < f.k; ++j) probe.q[j] = f.q[j];
        probe.m = M;
        if ((diag_qubit_mask(probe) & f.dq) != f.dq) return false;
        if (f.kind == OP_DIAG || f.kind == OP_PERM) {
            for (int r = 0; r < d; ++r)
                for (int c = 0; c < d; ++c)
                    if (f.m[(size_t)r * d + c] == cd(0, 0) && M[(size_t)r * d + c] != cd(0, 0)) return false;
        }
    }
    for (size_t fi = 0; fi < P.fused.size(); ++fi) P.fused[fi].m.swap(mats[fi]);
    build_device_tables(P);
    return true;
}

}  // namespace qsv
