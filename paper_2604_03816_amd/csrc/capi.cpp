// capi.cpp -- the extern "C" boundary of libqsv.so (declared in include/qsv.h).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <complex>
#include <cstdint>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/qsv.h"
#include "planner.h"
#include "qsv_internal.h"

using namespace qsv;

namespace {

thread_local std::string g_err;

qsv_status fail(qsv_status st, const std::string& msg)
{
    g_err = msg;
    return st;
}

#define QSV_HIP(call)                                                                          \
    do {                                                                                       \
        hipError_t e_ = (call);                                                                \
        if (e_ != hipSuccess) return fail(QSV_E_DEVICE, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

size_t elem_bytes(int dtype) { return dtype == QSV_C64 ? 8 : 16; }

struct DeviceGuard {
    int prev = -1;
    explicit DeviceGuard(int dev)
    {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        if (prev != dev) (void)hipSetDevice(dev);
    }
    ~DeviceGuard()
    {
        int cur = -1;
        if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
    }
};

}  // namespace

namespace qsv {
qsv_status set_error(qsv_status st, const std::string& msg) { return fail(st, msg); }
}  // namespace qsv

struct qsv_state_s {
    int n = 0;
    int dtype = 0;
    void* buf = nullptr;
    bool owned = false;
    hipStream_t stream = nullptr;
    int device = 0;
    // reduction workspace (device) and its host mirror (pinned)
    double* d_work = nullptr;
    size_t work_bytes = 0;
    double* h_work = nullptr;
    size_t hwork_bytes = 0;
    // plan-table arenas for one-shot applications, used in turn: each a pinned staging
    // block and a device block, both grow-only, and an event recorded after the last
    // pass that reads the slot's tables.  With several slots the host can plan and
    // enqueue up to kTabSlots applications ahead of the device before it has to wait.
    struct TabSlot {
        unsigned char* h = nullptr;
        size_t hbytes = 0;
        unsigned char* d = nullptr;
        size_t dbytes = 0;
        hipEvent_t ev = nullptr;
        bool pending = false;
    };
    static constexpr int kTabSlots = 8;
    TabSlot tab[kTabSlots];
    int tab_next = 0;
};

struct qsv_plan_s {
    HostPlan hp;
    int device = -1;
    DevOp* d_ops = nullptr;
    void* d_pool = nullptr;
    int* d_ipool = nullptr;
    float* d_apool = nullptr;
};

namespace {

qsv_status ensure_work(qsv_state s, size_t bytes)
{
    if (bytes <= s->work_bytes) return QSV_OK;
    if (s->d_work) {
        QSV_HIP(hipStreamSynchronize(s->stream));
        QSV_HIP(hipFree(s->d_work));
        s->d_work = nullptr;
        s->work_bytes = 0;
    }
    const size_t want = std::max<size_t>(bytes, 1 << 16);
    if (hipMalloc((void**)&s->d_work, want) != hipSuccess) {
        (void)hipGetLastError();
        s->d_work = nullptr;
        return fail(QSV_E_OOM, "workspace allocation failed");
    }
    s->work_bytes = want;
    return QSV_OK;
}

qsv_status ensure_hwork(qsv_state s, size_t bytes)
{
    if (bytes <= s->hwork_bytes) return QSV_OK;
    if (s->h_work) {
        QSV_HIP(hipHostFree(s->h_work));
        s->h_work = nullptr;
        s->hwork_bytes = 0;
    }
    const size_t want = std::max<size_t>(bytes, 1 << 16);
    QSV_HIP(hipHostMalloc((void**)&s->h_work, want, hipHostMallocDefault));
    s->hwork_bytes = want;
    return QSV_OK;
}

struct NS {
    double s = 0, c = 0;
    void add(double x)
    {
        const double t = s + x;
        c += (std::fabs(s) >= std::fabs(x)) ? ((s - t) + x) : ((x - t) + s);
        s = t;
    }
    double value() const { return s + c; }
};

qsv_status check_state(qsv_state s)
{
    if (!s) return fail(QSV_E_ARG, "null state");
    return QSV_OK;
}

bool read_gate(const qsv_gate& g, int n, InGate& out, std::string& err)
{
    if (g.k < 1 || g.k > kMaxK) { err = "gate k must be in [1, 5]"; return false; }
    for (int j = 0; j < g.k; ++j) {
        if (g.targets[j] < 0 || g.targets[j] >= n) { err = "gate target out of range"; return false; }
        for (int i = 0; i < j; ++i)
            if (g.targets[i] == g.targets[j]) { err = "duplicate gate target"; return false; }
    }
    if (!g.mat) { err = "null gate matrix"; return false; }
    out.k = g.k;
    for (int j = 0; j < kMaxK; ++j) out.t[j] = j < g.k ? g.targets[j] : 0;
    const int d = 1 << g.k;
    out.m.assign((size_t)d * d, cd(0, 0));
    if (g.diag) {
        for (int r = 0; r < d; ++r) out.m[(size_t)r * d + r] = cd(g.mat[2 * r], g.mat[2 * r + 1]);
    } else {
        for (int i = 0; i < d * d; ++i) out.m[i] = cd(g.mat[2 * i], g.mat[2 * i + 1]);
    }
    for (const cd& v : out.m)
        if (!std::isfinite(v.real()) || !std::isfinite(v.imag())) { err = "non-finite gate matrix entry"; return false; }
    return true;
}

}  // namespace

namespace qsv {
bool read_gate_public(const qsv_gate& g, int n, InGate& out, std::string& err) { return read_gate(g, n, out, err); }
}  // namespace qsv

namespace {

// The plan's complex pool in the state's precision (matrices rounded once from FP64).
void pack_pool(const HostPlan& hp, unsigned char* dst)
{
    for (size_t i = 0; i < hp.pool.size(); ++i) {
        if (hp.dtype == QSV_C64) {
            float* f = reinterpret_cast<float*>(dst) + 2 * i;
            f[0] = (float)hp.pool[i].real();
            f[1] = (float)hp.pool[i].imag();
        } else {
            double* f = reinterpret_cast<double*>(dst) + 2 * i;
            f[0] = hp.pool[i].real();
            f[1] = hp.pool[i].imag();
        }
    }
}

qsv_status upload_plan(qsv_plan p, int device)
{
    if (p->device == device) return QSV_OK;
    if (p->device >= 0) {
        DeviceGuard g(p->device);
        (void)hipFree(p->d_ops);
        (void)hipFree(p->d_pool);
        (void)hipFree(p->d_ipool);
        (void)hipFree(p->d_apool);
        p->d_ops = nullptr;
        p->d_pool = nullptr;
        p->d_ipool = nullptr;
        p->d_apool = nullptr;
        p->device = -1;
    }
    const HostPlan& hp = p->hp;
    const size_t nops = std::max<size_t>(hp.ops.size(), 1);
    const size_t npool = std::max<size_t>(hp.pool.size(), 1);
    const size_t nipool = std::max<size_t>(hp.ipool.size(), 1);
    const size_t eb = elem_bytes(hp.dtype);
    const size_t napool = std::max<size_t>(hp.apool.size(), 1);
    if (hipMalloc((void**)&p->d_ops, nops * sizeof(DevOp)) != hipSuccess ||
        hipMalloc(&p->d_pool, npool * eb) != hipSuccess ||
        hipMalloc((void**)&p->d_ipool, nipool * sizeof(int)) != hipSuccess ||
        hipMalloc((void**)&p->d_apool, napool * sizeof(float)) != hipSuccess) {
        (void)hipGetLastError();
        (void)hipFree(p->d_ops);
        (void)hipFree(p->d_pool);
        (void)hipFree(p->d_ipool);
        (void)hipFree(p->d_apool);
        p->d_ops = nullptr;
        p->d_pool = nullptr;
        p->d_ipool = nullptr;
        p->d_apool = nullptr;
        return fail(QSV_E_OOM, "plan table allocation failed");
    }
    std::vector<unsigned char> pool(npool * eb, 0);
    pack_pool(hp, pool.data());
    if (!hp.ops.empty()) QSV_HIP(hipMemcpy(p->d_ops, hp.ops.data(), hp.ops.size() * sizeof(DevOp), hipMemcpyHostToDevice));
    QSV_HIP(hipMemcpy(p->d_pool, pool.data(), pool.size(), hipMemcpyHostToDevice));
    if (!hp.ipool.empty()) QSV_HIP(hipMemcpy(p->d_ipool, hp.ipool.data(), hp.ipool.size() * sizeof(int), hipMemcpyHostToDevice));
    if (!hp.apool.empty()) QSV_HIP(hipMemcpy(p->d_apool, hp.apool.data(), hp.apool.size() * sizeof(float), hipMemcpyHostToDevice));
    p->device = device;
    return QSV_OK;
}

// Parsed Pauli term: X/Y mask, Z/Y mask, number of Y factors.
struct PTerm {
    unsigned long long x = 0, z = 0;
    int ny = 0;
    double coeff = 0;
};

bool parse_terms(const qsv_pauli_term* terms, size_t nt, int n, std::vector<PTerm>& out, std::string& err)
{
    out.resize(nt);
    for (size_t i = 0; i < nt; ++i) {
        const qsv_pauli_term& t = terms[i];
        PTerm p;
        p.coeff = t.coeff;
        if (t.n < 0 || (t.n > 0 && (!t.qubits || !t.paulis))) { err = "bad Pauli term"; return false; }
        for (int j = 0; j < t.n; ++j) {
            const int q = t.qubits[j];
            if (q < 0 || q >= n) { err = "Pauli qubit out of range"; return false; }
            const unsigned long long b = 1ull << q;
            if ((p.x | p.z) & b) { err = "repeated qubit in a Pauli term"; return false; }
            switch (t.paulis[j]) {
            case 'I': break;
            case 'X': p.x |= b; break;
            case 'Y': p.x |= b; p.z |= b; ++p.ny; break;
            case 'Z': p.z |= b; break;
            default: err = "Pauli letters must be I, X, Y or Z"; return false;
            }
        }
        out[i] = p;
    }
    return true;
}

// Tile geometry for a set of must-have qubits: the low L qubits plus `need`, filled
// with the lowest other qubits up to m.
PassArgs tile_args(int n, int m, int L, unsigned long long need, std::vector<int>& active)
{
    unsigned long long A = need;
    for (int b = 0; b < L && b < n; ++b) A |= 1ull << b;
    for (int b = 0; b < n && __builtin_popcountll(A) < m; ++b) A |= 1ull << b;
    active.clear();
    for (int b = 0; b < n; ++b)
        if ((A >> b) & 1) active.push_back(b);
    PassArgs a{};
    a.m = (int)active.size();
    a.L = std::min(L, a.m);
    for (int i = 0; i < a.m; ++i) a.phys[i] = (unsigned char)active[i];
    int b = 0;
    while (b < n) {
        if ((A >> b) & 1) { ++b; continue; }
        const int s = b;
        while (b < n && !((A >> b) & 1)) ++b;
        a.run_pos[a.nruns] = (unsigned char)s;
        a.run_len[a.nruns] = (unsigned char)(b - s);
        ++a.nruns;
    }
    return a;
}

// Pauli matrix elements Re <a|P_i|b> (imag == false) or Im <a|P_i|b> (imag == true),
// unweighted, for states a and b of one shape (a == b for expectation values), in three
// steps: plan_elements groups the terms so that each group's X/Y supports fit one tile
// (one read pass per group) and lays out the per-workgroup partials; launch_elements
// enqueues the passes; combine_elements adds each term's partials (fixed order,
// compensated) once they are on the host.
struct ElemGroup {
    PassArgs a;
    TermArgs ta;
    bool zonly = false;     // every term Z-only: the Z kernel with zt
    ZTermArgs zt;
    long long ntiles;
    int grid;
    std::vector<int> idx;   // term indices
    size_t off;             // first double of this group's partials
};

// Two-state weights of a Pauli term with phase i^q: i^q for even parity, -i^q for odd.
void set_pauli_weights(TermArgs& t, int i, int q)
{
    static const double re[4] = {1, 0, -1, 0}, im[4] = {0, 1, 0, -1};
    q &= 3;
    t.kw[i][0] = re[q];
    t.kw[i][1] = im[q];
    t.kw[i][2] = -re[q];
    t.kw[i][3] = -im[q];
}

bool plan_elements(int n, const std::vector<PTerm>& terms, bool imag, std::vector<ElemGroup>& G, size_t& doubles,
                   std::string& err, int dtype, int xgrid = 4096)
{
    const PlanOpts o = default_opts(dtype);
    const int m = std::min(n, kExpvalMaxTileQubits);
    const int L = std::min(o.low_qubits, m);
    const unsigned long long lowmask = (L >= 64) ? ~0ull : ((1ull << L) - 1);
    std::vector<std::vector<int>> groups;
    std::vector<unsigned long long> gneed;
    // Z-only terms get groups of their own (the Z kernel costs one read pass however many
    // terms it holds); terms with X/Y factors are grouped by their X/Y supports
    const bool zkernel = m >= kLogThreads && n - m <= kMaxTileIndexBits;
    size_t nz = 0;
    if (zkernel) {
        for (size_t i = 0; i < terms.size(); ++i) {
            if (terms[i].x) continue;
            if (nz % kMaxTermsPerLaunch == 0) {
                groups.push_back({});
                gneed.push_back(0);
            }
            groups.back().push_back((int)i);
            ++nz;
        }
    }
    const size_t zgroups = groups.size();
    for (size_t i = 0; i < terms.size(); ++i) {
        const unsigned long long x = terms[i].x;
        if (zkernel && x == 0) continue;
        if (__builtin_popcountll(x | lowmask) > m) {
            err = "Pauli term flips more qubits than one tile holds";
            return false;
        }
        bool placed = false;
        for (size_t g = zgroups; g < groups.size() && !placed; ++g) {
            const unsigned long long need = gneed[g] | x;
            if (groups[g].size() < (size_t)kMaxTermsPerLaunch && __builtin_popcountll(need | lowmask) <= m) {
                groups[g].push_back((int)i);
                gneed[g] = need;
                placed = true;
            }
        }
        if (!placed) {
            groups.push_back({(int)i});
            gneed.push_back(x);
        }
    }
    G.clear();
    doubles = 0;
    for (size_t g = 0; g < groups.size(); ++g) {
        std::vector<int> active;
        ElemGroup E;
        E.a = tile_args(n, m, L, gneed[g], active);
        E.ta = TermArgs{};
        E.ta.nterms = (int)groups[g].size();
        for (int i = 0; i < E.ta.nterms; ++i) {
            const PTerm& p = terms[groups[g][i]];
            int xl = 0, zl = 0;
            unsigned long long zg = p.z;
            for (int j = 0; j < E.a.m; ++j) {
                const unsigned long long b = 1ull << active[j];
                if (p.x & b) xl |= 1 << j;
                if (p.z & b) { zl |= 1 << j; zg &= ~b; }
            }
            E.ta.xloc[i] = xl;
            E.ta.zloc[i] = zl;
            E.ta.zglob[i] = (long long)zg;
            E.ta.ny[i] = p.ny + (imag ? 3 : 0);   // Im z = Re(-i z), and -i = i^3
            set_pauli_weights(E.ta, i, E.ta.ny[i]);
        }
        if (g < zgroups) {
            // signs and lookups of the Z kernel (see ZTermArgs)
            E.zonly = true;
            E.zt = ZTermArgs{};
            E.zt.nterms = E.ta.nterms;
            const int NS = 1 << (E.a.m - kLogThreads);
            std::vector<int> outside;   // tile-number bit b <-> outside[b], ascending
            {
                unsigned long long A = 0;
                for (const int q : active) A |= 1ull << q;
                for (int q = 0; q < n; ++q)
                    if (!((A >> q) & 1)) outside.push_back(q);
            }
            for (int i = 0; i < E.ta.nterms; ++i) {
                const int q = E.ta.ny[i] & 3;
                E.zt.zoff[i] = ((q & 1) ? NS : 0) + (E.ta.zloc[i] >> kLogThreads);
                E.zt.zlo[i] = E.ta.zloc[i] & (kThreads - 1);
                if (q == 1 || q == 2) E.zt.neg |= 1u << i;
                if (q & 1) E.zt.zero |= 1u << i;
                for (size_t b = 0; b < outside.size(); ++b)
                    if ((E.ta.zglob[i] >> outside[b]) & 1) E.zt.gcol[b] |= 1u << i;
            }
        }
        E.ntiles = 1ll << (n - E.a.m);
        // Z-only groups end with a workgroup reduction per term, so fewer workgroups; the
        // X/Y kernel is bound by its per-term LDS work and gains from more of them
        // (measured at 30 qubits; callers that read back many groups ask for fewer)
        E.grid = (int)std::min<long long>(E.ntiles, E.zonly ? 1024 : xgrid);
        E.idx = groups[g];
        E.off = doubles;
        doubles += (size_t)E.grid * E.ta.nterms * 2;
        G.push_back(std::move(E));
    }
    return true;
}

hipError_t launch_elements(int dtype, const void* sa, const void* sb, const std::vector<ElemGroup>& G,
                           double* d_partial, hipStream_t stream)
{
    for (const ElemGroup& E : G) {
        const hipError_t e = E.zonly
            ? launch_expval_z(dtype, sa, sb, E.a, E.zt, E.ntiles, E.grid, d_partial + E.off, stream)
            : launch_expval(dtype, sa, sb, E.a, E.ta, E.ntiles, E.grid, d_partial + E.off, stream);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

void combine_elements(const std::vector<ElemGroup>& G, const double* h_partial, size_t nterms, std::vector<double>& out)
{
    out.assign(nterms, 0.0);
    for (const ElemGroup& E : G) {
        for (int i = 0; i < E.ta.nterms; ++i) {
            NS acc;
            for (int b = 0; b < E.grid; ++b) {
                acc.add(h_partial[E.off + ((size_t)b * E.ta.nterms + i) * 2]);
                acc.c += h_partial[E.off + ((size_t)b * E.ta.nterms + i) * 2 + 1];
            }
            out[E.idx[i]] = acc.value();
        }
    }
}

qsv_status pauli_elements(qsv_state s, const void* sa, const void* sb, const std::vector<PTerm>& terms, bool imag,
                          std::vector<double>& out)
{
    std::vector<ElemGroup> G;
    size_t doubles = 0;
    std::string err;
    if (!plan_elements(s->n, terms, imag, G, doubles, err, s->dtype)) return fail(QSV_E_UNSUPPORTED, err);
    const size_t bytes = std::max<size_t>(doubles, 1) * sizeof(double);
    qsv_status st = ensure_work(s, bytes);
    if (st != QSV_OK) return st;
    if ((st = ensure_hwork(s, bytes)) != QSV_OK) return st;
    QSV_HIP(launch_elements(s->dtype, sa, sb, G, s->d_work, s->stream));
    QSV_HIP(hipMemcpyAsync(s->h_work, s->d_work, bytes, hipMemcpyDeviceToHost, s->stream));
    QSV_HIP(hipStreamSynchronize(s->stream));
    combine_elements(G, s->h_work, terms.size(), out);
    return QSV_OK;
}

qsv_status expval_core(qsv_state s, const std::vector<PTerm>& terms, std::vector<double>& out)
{
    return pauli_elements(s, s->buf, s->buf, terms, false, out);
}

// dst = sum_t coeff_t P_t src, terms in batches of kMaxPauliApply launches.
qsv_status pauli_sum_apply(qsv_state s, const void* src, void* dst, const std::vector<PTerm>& terms)
{
    const long long N = 1ll << s->n;
    if (terms.empty()) {
        QSV_HIP(launch_zero(s->dtype, dst, N, s->stream));
        return QSV_OK;
    }
    for (size_t b = 0; b < terms.size(); b += kMaxPauliApply) {
        PauliSumArgs p{};
        p.nterms = (int)std::min<size_t>(kMaxPauliApply, terms.size() - b);
        for (int i = 0; i < p.nterms; ++i) {
            const PTerm& t = terms[b + i];
            p.x[i] = (long long)t.x;
            p.z[i] = (long long)t.z;
            p.ny[i] = t.ny;
            p.coeff[i] = t.coeff;
        }
        QSV_HIP(launch_pauli_apply(s->dtype, src, dst, N, p, b > 0 ? 1 : 0, s->stream));
    }
    return QSV_OK;
}

// Enqueues every pass of a host plan on the state's stream, its tables copied into the
// state's next arena slot: one asynchronous copy, no allocation once the slot is large
// enough, and no wait for the device unless the passes of the application kTabSlots
// back (which read this slot) are still queued.
// Uploads the plan's tables into s's arena and enqueues its passes on s's stream; with
// s2 (same shape and stream) every pass covers both states in one launch; from_zero: the
// input is |0...0> (the first pass builds it on chip; no passes: s is reset).
qsv_status enqueue_plan(qsv_state s, const HostPlan& hp, qsv_state s2 = nullptr, bool from_zero = false)
{
    if (from_zero && hp.passes.empty()) {
        QSV_HIP(launch_init_zero(s->dtype, s->buf, 1ll << s->n, s->stream));
        if (s2) QSV_HIP(launch_init_zero(s2->dtype, s2->buf, 1ll << s2->n, s2->stream));
        return QSV_OK;
    }
    auto al = [](size_t b) { return (b + 255) & ~(size_t)255; };
    const size_t eb = elem_bytes(hp.dtype);
    const size_t o_ops = 0;
    const size_t o_pool = o_ops + al(hp.ops.size() * sizeof(DevOp));
    const size_t o_ipool = o_pool + al(hp.pool.size() * eb);
    const size_t o_apool = o_ipool + al(hp.ipool.size() * sizeof(int));
    const size_t total = std::max<size_t>(o_apool + al(hp.apool.size() * sizeof(float)), 256);
    qsv_state_s::TabSlot& ts = s->tab[s->tab_next];
    s->tab_next = (s->tab_next + 1) % qsv_state_s::kTabSlots;
    if (ts.pending) {   // the passes that read this slot's tables (and so its copy) are done
        QSV_HIP(hipEventSynchronize(ts.ev));
        ts.pending = false;
    }
    if (!ts.ev) QSV_HIP(hipEventCreateWithFlags(&ts.ev, hipEventDisableTiming));
    if (total > ts.hbytes) {
        if (ts.h) QSV_HIP(hipHostFree(ts.h));
        ts.h = nullptr;
        ts.hbytes = 0;
        const size_t want = std::max<size_t>(total * 2, 1 << 16);
        QSV_HIP(hipHostMalloc((void**)&ts.h, want, hipHostMallocDefault));
        ts.hbytes = want;
    }
    if (total > ts.dbytes) {
        if (ts.d) QSV_HIP(hipFree(ts.d));   // no pass reads it any more (event above)
        ts.d = nullptr;
        ts.dbytes = 0;
        const size_t want = std::max<size_t>(total * 2, 1 << 16);
        if (hipMalloc((void**)&ts.d, want) != hipSuccess) {
            (void)hipGetLastError();
            return fail(QSV_E_OOM, "plan table allocation failed");
        }
        ts.dbytes = want;
    }
    unsigned char* h = ts.h;
    if (!hp.ops.empty()) std::memcpy(h + o_ops, hp.ops.data(), hp.ops.size() * sizeof(DevOp));
    pack_pool(hp, h + o_pool);
    if (!hp.ipool.empty()) std::memcpy(h + o_ipool, hp.ipool.data(), hp.ipool.size() * sizeof(int));
    if (!hp.apool.empty()) std::memcpy(h + o_apool, hp.apool.data(), hp.apool.size() * sizeof(float));
    QSV_HIP(hipMemcpyAsync(ts.d, h, total, hipMemcpyHostToDevice, s->stream));
    unsigned char* d = ts.d;
    for (size_t i = 0; i < hp.passes.size(); ++i)
        QSV_HIP(launch_pass(s->dtype, s->buf, hp.pargs[i], hp.pgrid[i], (const DevOp*)(d + o_ops), d + o_pool,
                            (const int*)(d + o_ipool), (const float*)(d + o_apool), s->stream,
                            s2 ? s2->buf : nullptr, from_zero && i == 0, hp.pwide[i] != 0));
    QSV_HIP(hipEventRecord(ts.ev, s->stream));
    ts.pending = true;
    return QSV_OK;
}

}  // namespace

extern "C" {

const char* qsv_last_error(void) { return g_err.c_str(); }

const char* qsv_version(void) { return "qsv 0.1 (gfx950)"; }

qsv_status qsv_alloc(int n, qsv_dtype dtype, void* buf, size_t buf_bytes, void* stream, qsv_state* out)
{
    if (!out) return fail(QSV_E_ARG, "out is null");
    *out = nullptr;
    if (n < 1 || n > kMaxQubits) return fail(QSV_E_ARG, "n_qubits must be in [1, 34]");
    if (dtype != QSV_C64 && dtype != QSV_C128) return fail(QSV_E_ARG, "bad dtype");
    const size_t bytes = elem_bytes(dtype) << n;
    if (buf && buf_bytes < bytes) return fail(QSV_E_ARG, "adopted buffer is smaller than 2^n amplitudes");
    if (buf && ((uintptr_t)buf & 15)) return fail(QSV_E_ARG, "adopted buffer must be 16-byte aligned");
    int dev = 0;
    QSV_HIP(hipGetDevice(&dev));
    qsv_state s = new qsv_state_s();
    s->n = n;
    s->dtype = dtype;
    s->stream = (hipStream_t)stream;
    s->device = dev;
    if (buf) {
        s->buf = buf;
    } else {
        if (hipMalloc(&s->buf, bytes) != hipSuccess) {
            (void)hipGetLastError();
            delete s;
            return fail(QSV_E_OOM, "state allocation of " + std::to_string(bytes) + " bytes failed");
        }
        s->owned = true;
    }
    hipError_t e = launch_init_zero(dtype, s->buf, 1ll << n, s->stream);
    if (e != hipSuccess) {
        if (s->owned) (void)hipFree(s->buf);
        delete s;
        return fail(QSV_E_DEVICE, std::string("init: ") + hipGetErrorString(e));
    }
    *out = s;
    return QSV_OK;
}

qsv_status qsv_free(qsv_state s)
{
    if (!s) return QSV_OK;
    DeviceGuard g(s->device);
    (void)hipStreamSynchronize(s->stream);
    if (s->owned) (void)hipFree(s->buf);
    if (s->d_work) (void)hipFree(s->d_work);
    if (s->h_work) (void)hipHostFree(s->h_work);
    for (qsv_state_s::TabSlot& ts : s->tab) {
        if (ts.d) (void)hipFree(ts.d);
        if (ts.h) (void)hipHostFree(ts.h);
        if (ts.ev) (void)hipEventDestroy(ts.ev);
    }
    delete s;
    return QSV_OK;
}

qsv_status qsv_reset(qsv_state s)
{
    qsv_status st = check_state(s);
    if (st != QSV_OK) return st;
    DeviceGuard g(s->device);
    QSV_HIP(launch_init_zero(s->dtype, s->buf, 1ll << s->n, s->stream));
    return QSV_OK;
}

qsv_status qsv_info(qsv_state s, int* n, qsv_dtype* dtype, void** ptr)
{
    qsv_status st = check_state(s);
    if (st != QSV_OK) return st;
    if (n) *n = s->n;
    if (dtype) *dtype = (qsv_dtype)s->dtype;
    if (ptr) *ptr = s->buf;
    return QSV_OK;
}

qsv_status qsv_get_state(qsv_state s, void* host_out)
{
    qsv_status st = check_state(s);
    if (st != QSV_OK) return st;
    if (!host_out) return fail(QSV_E_ARG, "host_out is null");
    DeviceGuard g(s->device);
    QSV_HIP(hipMemcpyAsync(host_out, s->buf, elem_bytes(s->dtype) << s->n, hipMemcpyDeviceToHost, s->stream));
    QSV_HIP(hipStreamSynchronize(s->stream));
    return QSV_OK;
}

qsv_status qsv_set_state(qsv_state s, const void* host_in)
{
    qsv_status st = check_state(s);
    if (st != QSV_OK) return st;
    if (!host_in) return fail(QSV_E_ARG, "host_in is null");
    DeviceGuard g(s->device);
    QSV_HIP(hipMemcpyAsync(s->buf, host_in, elem_bytes(s->dtype) << s->n, hipMemcpyHostToDevice, s->stream));
    QSV_HIP(hipStreamSynchronize(s->stream));
    return QSV_OK;
}

qsv_status qsv_sync(qsv_state s)
{
    qsv_status st = check_state(s);
    if (st != QSV_OK) return st;
    DeviceGuard g(s->device);
    QSV_HIP(hipStreamSynchronize(s->stream));
    return QSV_OK;
}

// Eq. 4 gate set, written from the definitions: rotations exp(-i theta P / 2),
// U3 in the OpenQASM 2 convention, multi-qubit gates by their basis action.
qsv_status qsv_gate_matrix(const char* name, const double* p, int* k, double* mat)
{
    if (!name || !k || !mat) return fail(QSV_E_ARG, "null argument");
    const std::string nm(name);
    const bool needs1 = nm == "RX" || nm == "RY" || nm == "RZ", needs3 = nm == "U3";
    if ((needs1 || needs3) && !p) return fail(QSV_E_ARG, "missing gate parameters");
    std::vector<cd> U;
    int kk = 1;
    const cd i1(0, 1);
    if (nm == "I") U = {1, 0, 0, 1};
    else if (nm == "X") U = {0, 1, 1, 0};
    else if (nm == "Y") U = {0, -i1, i1, 0};
    else if (nm == "Z") U = {1, 0, 0, -1};
    else if (nm == "H") { const double h = 1.0 / std::sqrt(2.0); U = {h, h, h, -h}; }
    else if (nm == "S") U = {1, 0, 0, i1};
    else if (nm == "SDG") U = {1, 0, 0, -i1};
    else if (nm == "T") U = {1, 0, 0, std::polar(1.0, M_PI / 4)};
    else if (nm == "TDG") U = {1, 0, 0, std::polar(1.0, -M_PI / 4)};
    else if (nm == "RX") { const double c = std::cos(p[0] / 2), s = std::sin(p[0] / 2); U = {c, -i1 * s, -i1 * s, c}; }
    else if (nm == "RY") { const double c = std::cos(p[0] / 2), s = std::sin(p[0] / 2); U = {c, -s, s, c}; }
    else if (nm == "RZ") U = {std::polar(1.0, -p[0] / 2), 0, 0, std::polar(1.0, p[0] / 2)};
    else if (nm == "U3") {
        const double c = std::cos(p[0] / 2), s = std::sin(p[0] / 2);
        U = {c, -std::polar(1.0, p[2]) * s, std::polar(1.0, p[1]) * s, std::polar(1.0, p[1] + p[2]) * c};
    } else if (nm == "CNOT" || nm == "CZ" || nm == "SWAP" || nm == "TOFFOLI") {
        kk = nm == "TOFFOLI" ? 3 : 2;
        const int d = 1 << kk;
        U.assign((size_t)d * d, 0);
        for (int in = 0; in < d; ++in) {
            int outi = in;
            cd amp = 1;
            if (nm == "CNOT" && (in & 1)) outi = in ^ 2;
            if (nm == "CZ" && in == 3) amp = -1;
            if (nm == "SWAP") outi = ((in & 1) << 1) | ((in >> 1) & 1);
            if (nm == "TOFFOLI" && (in & 3) == 3) outi = in ^ 4;
            U[(size_t)outi * d + in] = amp;
        }
    } else {
        return fail(QSV_E_ARG, "unknown gate name " + nm);
    }
    *k = kk;
    for (size_t i = 0; i < U.size(); ++i) {
        mat[2 * i] = U[i].real();
        mat[2 * i + 1] = U[i].imag();
    }
    return QSV_OK;
}

qsv_status qsv_plan_create(int n, qsv_dtype dtype, const qsv_gate* gates, size_t n_gates,
                           const qsv_plan_opts* opts, qsv_plan* out)
{
    if (!out) return fail(QSV_E_ARG, "out is null");
    *out = nullptr;
    if (n < 1 || n > kMaxQubits) return fail(QSV_E_ARG, "n_qubits must be in [1, 34]");
    if (dtype != QSV_C64 && dtype != QSV_C128) return fail(QSV_E_ARG, "bad dtype");
    if (n_gates && !gates) return fail(QSV_E_ARG, "gates is null");
    PlanOpts o;
    std::string oerr;
    if (!plan_opts_from(dtype, opts, o, oerr)) return fail(QSV_E_ARG, oerr);
    const int max_tile = dtype == QSV_C64 ? 13 : 12;   // 64 KiB of LDS
    if (o.tile_qubits > max_tile) return fail(QSV_E_ARG, "tile_qubits exceeds the LDS tile limit");
    std::vector<InGate> in(n_gates);
    std::string err;
    for (size_t i = 0; i < n_gates; ++i)
        if (!read_gate(gates[i], n, in[i], err)) return fail(QSV_E_ARG, "gate " + std::to_string(i) + ": " + err);
    qsv_plan p = new qsv_plan_s();
    if (!make_plan(n, dtype, in, o, p->hp, err)) {
        delete p;
        return fail(QSV_E_ARG, err);
    }
    *out = p;
    return QSV_OK;
}

qsv_status qsv_plan_free(qsv_plan p)
{
    if (!p) return QSV_OK;
    if (p->device >= 0) {
        DeviceGuard g(p->device);
        (void)hipFree(p->d_ops);
        (void)hipFree(p->d_pool);
        (void)hipFree(p->d_ipool);
        (void)hipFree(p->d_apool);
    }
    delete p;
    return QSV_OK;
}

qsv_status qsv_plan_refresh(qsv_plan p, const qsv_gate* gates, size_t n_gates)
{
    if (!p) return fail(QSV_E_ARG, "null plan");
    if (n_gates && !gates) return fail(QSV_E_ARG, "gates is null");
    std::vector<InGate> in(n_gates);
    std::string err;
    for (size_t i = 0; i < n_gates; ++i)
        if (!read_gate(gates[i], p->hp.n, in[i], err)) return fail(QSV_E_ARG, "gate " + std::to_string(i) + ": " + err);
    if (!same_shape(p->hp, in)) return fail(QSV_E_ARG, "the gates do not have the shape of the plan's circuit");
    HostPlan hp = p->hp;
    if (!refresh_plan(hp, in))
        return fail(QSV_E_UNSUPPORTED, "the plan's structure does not hold for these gates: make a new plan");
    if (p->device >= 0) {   // stale device tables: freed once no queued pass can read them
        DeviceGuard g(p->device);
        QSV_HIP(hipDeviceSynchronize());
        (void)hipFree(p->d_ops);
        (void)hipFree(p->d_pool);
        (void)hipFree(p->d_ipool);
        (void)hipFree(p->d_apool);
        p->d_ops = nullptr;
        p->d_pool = nullptr;
        p->d_ipool = nullptr;
        p->d_apool = nullptr;
        p->device = -1;
    }
    p->hp = std::move(hp);
    return QSV_OK;
}

qsv_status qsv_plan_get_stats(qsv_plan p, qsv_plan_stats* st)
{
    if (!p || !st) return fail(QSV_E_ARG, "null argument");
    const HostPlan& hp = p->hp;
    st->gates_in = hp.gates_in;
    st->fused_out = hp.fused.size();
    st->passes = hp.passes.size();
    st->dense_ops = hp.dense_ops;
    st->diag_ops = hp.diag_ops;
    st->perm_ops = hp.perm_ops;
    st->mfma_ops = hp.mfma_ops;
    st->fma_per_amp = hp.fma_per_amp;
    st->mfma_fma_per_amp = hp.mfma_fma_per_amp;
    st->hbm_bytes = (double)hp.passes.size() * 2.0 * (double)(elem_bytes(hp.dtype) << hp.n);
    return QSV_OK;
}

qsv_status qsv_plan_fused_gate(qsv_plan p, size_t i, int* k, int targets[5], int* diag, double* mat)
{
    if (!p || !k || !targets || !diag) return fail(QSV_E_ARG, "null argument");
    if (i >= p->hp.fused.size()) return fail(QSV_E_ARG, "fused gate index out of range");
    const FGate& g = p->hp.fused[i];
    *k = g.k;
    for (int j = 0; j < 5; ++j) targets[j] = j < g.k ? g.q[j] : -1;
    *diag = g.kind == OP_DIAG;
    if (mat)
        for (size_t e = 0; e < g.m.size(); ++e) {
            mat[2 * e] = g.m[e].real();
            mat[2 * e + 1] = g.m[e].imag();
        }
    return QSV_OK;
}

qsv_status qsv_plan_pass_info(qsv_plan p, size_t i, int* n_ops, int* n_active, int active[40])
{
    if (!p || !n_ops || !n_active || !active) return fail(QSV_E_ARG, "null argument");
    if (i >= p->hp.passes.size()) return fail(QSV_E_ARG, "pass index out of range");
    const PassPlan& pp = p->hp.passes[i];
    *n_ops = (int)pp.ops.size();
    *n_active = (int)pp.active.size();
    for (size_t j = 0; j < pp.active.size(); ++j) active[j] = pp.active[j];
    return QSV_OK;
}

qsv_status qsv_plan_pass_ops(qsv_plan p, size_t i, int* fused_idx)
{
    if (!p || !fused_idx) return fail(QSV_E_ARG, "null argument");
    if (i >= p->hp.passes.size()) return fail(QSV_E_ARG, "pass index out of range");
    const PassPlan& pp = p->hp.passes[i];
    for (size_t j = 0; j < pp.ops.size(); ++j) fused_idx[j] = pp.ops[j];
    return QSV_OK;
}

// Host re-enactment of the pass kernel over the device tables (tile placement from the
// free-bit runs, local offsets from the tile strides, ops by local bit positions), in
// FP64.  Lets host tests check the tables the GPU consumes without a GPU.
qsv_status qsv_plan_emulate(qsv_plan p, double* state)
{
    if (!p || !state) return fail(QSV_E_ARG, "null argument");
    const HostPlan& hp = p->hp;
    cd* st = reinterpret_cast<cd*>(state);
    for (size_t pi = 0; pi < hp.passes.size(); ++pi) {
        const PassArgs& a = hp.pargs[pi];
        const int T = 1 << a.m;
        std::vector<cd> lds(T);
        std::vector<long long> off(T);
        for (int e = 0; e < T; ++e) {
            long long o = 0;
            for (int i = 0; i < a.m; ++i)
                if ((e >> i) & 1) o += 1ll << a.phys[i];
            off[e] = o;
        }
        for (long long t = 0; t < hp.pgrid[pi]; ++t) {
            long long base = 0, rem = t;
            for (int r = 0; r < a.nruns; ++r) {
                base |= (rem & ((1ll << a.run_len[r]) - 1)) << a.run_pos[r];
                rem >>= a.run_len[r];
            }
            for (int e = 0; e < T; ++e) lds[e] = st[base + off[e]];
            for (int oi = 0; oi < a.op_count; ++oi) {
                const DevOp& op = hp.ops[a.op_begin + oi];
                const int K = op.k, D = 1 << K;
                auto roff = [&](int r) {
                    int o = 0;
                    for (int j = 0; j < K; ++j)
                        if ((r >> j) & 1) o += 1 << op.lpos[j];
                    return o;
                };
                if (op.kind == OP_DIAG) {
                    int gfix = 0;
                    for (int j = 0; j < K; ++j)
                        if (op.lpos[j] < 0) gfix |= (int)((base >> op.gbit[j]) & 1) << j;
                    for (int e = 0; e < T; ++e) {
                        int idx = gfix;
                        for (int j = 0; j < K; ++j)
                            if (op.lpos[j] >= 0) idx |= ((e >> op.lpos[j]) & 1) << j;
                        lds[e] *= hp.pool[op.off + idx];
                    }
                    continue;
                }
                for (int j = 0; j < K; ++j)
                    if (op.lpos[j] < 0 || op.lpos[j] >= a.m) return fail(QSV_E_ARG, "op target outside its tile");
                std::vector<cd> v(D), w(D);
                for (int g = 0; g < (T >> K); ++g) {
                    int b = g;
                    for (int j = 0; j < K; ++j) {
                        const int q = op.lpos[j];
                        b = ((b >> q) << (q + 1)) | (b & ((1 << q) - 1));
                    }
                    if (op.kind == OP_DENSE) {
                        for (int r = 0; r < D; ++r) v[r] = lds[b + roff(r)];
                        for (int r = 0; r < D; ++r) {
                            cd acc = 0;
                            for (int c = 0; c < D; ++c) acc += hp.pool[op.off + r * D + c] * v[c];
                            w[r] = acc;
                        }
                    } else {
                        for (int r = 0; r < D; ++r) v[r] = lds[b + roff(hp.ipool[op.ioff + r])];
                        for (int r = 0; r < D; ++r) w[r] = op.flags ? hp.pool[op.off + r] * v[r] : v[r];
                    }
                    for (int r = 0; r < D; ++r) lds[b + roff(r)] = w[r];
                }
            }
            for (int e = 0; e < T; ++e) st[base + off[e]] = lds[e];
        }
    }
    return QSV_OK;
}

qsv_status qsv_plan_apply_range(qsv_state s, qsv_plan p, size_t first, size_t count)
{
    qsv_status st = check_state(s);
    if (st != QSV_OK) return st;
    if (!p) return fail(QSV_E_ARG, "null plan");
    if (p->hp.n != s->n || p->hp.dtype != s->dtype) return fail(QSV_E_ARG, "plan does not match the state's n / dtype");
    const size_t np = p->hp.passes.size();
    if (first > np || count > np - first) return fail(QSV_E_ARG, "pass range out of bounds");
    DeviceGuard g(s->device);
    st = upload_plan(p, s->device);
    if (st != QSV_OK) return st;
    for (size_t i = first; i < first + count; ++i) {
        const PassArgs& a = p->hp.pargs[i];
        QSV_HIP(launch_pass(s->dtype, s->buf, a, p->hp.pgrid[i], p->d_ops, p->d_pool, p->d_ipool, p->d_apool,
                            s->stream, nullptr, false, p->hp.pwide[i] != 0));
    }
    return QSV_OK;
}

qsv_status qsv_plan_apply_zero(qsv_state s, qsv_plan p, size_t count)
{
    qsv_status st = check_state(s);
    if (st != QSV_OK) return st;
    if (!p) return fail(QSV_E_ARG, "null plan");
    if (p->hp.n != s->n || p->hp.dtype != s->dtype) return fail(QSV_E_ARG, "plan does not match the state's n / dtype");
    const size_t np = p->hp.passes.size();
    if (count > np) return fail(QSV_E_ARG, "pass count out of bounds");
    DeviceGuard g(s->device);
    if (count == 0) {
        QSV_HIP(launch_init_zero(s->dtype, s->buf, 1ll << s->n, s->stream));
        return QSV_OK;
    }
    st = upload_plan(p, s->device);
    if (st != QSV_OK) return st;
    for (size_t i = 0; i < count; ++i) {
        const PassArgs& a = p->hp.pargs[i];
        QSV_HIP(launch_pass(s->dtype, s->buf, a, p->hp.pgrid[i], p->d_ops, p->d_pool, p->d_ipool, p->d_apool,
                            s->stream, nullptr, i == 0, p->hp.pwide[i] != 0));
    }
    return QSV_OK;
}

qsv_status qsv_plan_apply(qsv_state s, qsv_plan p)
{
    if (!p) return fail(QSV_E_ARG, "null plan");
    return qsv_plan_apply_range(s, p, 0, p->hp.passes.size());
}

qsv_status qsv_apply_fused(qsv_state s, const qsv_gate* gates, size_t n_gates, const qsv_plan_opts* opts,
                           qsv_plan_stats* stats)
{
    qsv_status st = check_state(s);
    if (st != QSV_OK) return st;
    qsv_plan p = nullptr;
    st = qsv_plan_create(s->n, (qsv_dtype)s->dtype, gates, n_gates, opts, &p);
    if (st != QSV_OK) return st;
    if (stats) qsv_plan_get_stats(p, stats);
    {
        DeviceGuard g(s->device);
        st = enqueue_plan(s, p->hp);
        const hipError_t e = hipStreamSynchronize(s->stream);
        qsv_plan_free(p);
        if (st == QSV_OK && e != hipSuccess) return fail(QSV_E_DEVICE, std::string("apply: ") + hipGetErrorString(e));
    }
    return st;
}

qsv_status qsv_norm(qsv_state s, double* out)
{
    qsv_status st = check_state(s);
    if (st != QSV_OK) return st;
    if (!out) return fail(QSV_E_ARG, "out is null");
    DeviceGuard g(s->device);
    const long long N = 1ll << s->n;
    const int grid = norm_grid(N);
    const size_t bytes = (size_t)grid * 2 * sizeof(double);
    if ((st = ensure_work(s, bytes)) != QSV_OK) return st;
    if ((st = ensure_hwork(s, bytes)) != QSV_OK) return st;
    QSV_HIP(launch_norm(s->dtype, s->buf, N, s->d_work, grid, s->stream));
    QSV_HIP(hipMemcpyAsync(s->h_work, s->d_work, bytes, hipMemcpyDeviceToHost, s->stream));
    QSV_HIP(hipStreamSynchronize(s->stream));
    NS acc;
    for (int b = 0; b < grid; ++b) {
        acc.add(s->h_work[2 * b]);
        acc.c += s->h_work[2 * b + 1];
    }
    *out = acc.value();
    return QSV_OK;
}

qsv_status qsv_expval_pauli(qsv_state s, const qsv_pauli_term* terms, size_t n_terms, double* per_term,
                            double* sum)
{
    qsv_status st = check_state(s);
    if (st != QSV_OK) return st;
    if (n_terms && !terms) return fail(QSV_E_ARG, "terms is null");
    std::vector<PTerm> pt;
    std::string err;
    if (!parse_terms(terms, n_terms, s->n, pt, err)) return fail(QSV_E_ARG, err);
    DeviceGuard g(s->device);
    std::vector<double> vals;
    if ((st = expval_core(s, pt, vals)) != QSV_OK) return st;
    NS acc;
    for (size_t i = 0; i < n_terms; ++i) {
        const double v = pt[i].coeff * vals[i];
        if (per_term) per_term[i] = v;
        acc.add(v);
    }
    if (sum) *sum = acc.value();
    return QSV_OK;
}

qsv_status qsv_probs(qsv_state s, const int* qubits, int m, void* out, int out_on_device)
{
    qsv_status st = check_state(s);
    if (st != QSV_OK) return st;
    if (!out) return fail(QSV_E_ARG, "out is null");
    const int n = s->n;
    if (m < 1 || m > n) return fail(QSV_E_ARG, "m must be in [1, n]");
    bool full = (m == n);
    if (qubits) {
        for (int j = 0; j < m; ++j) {
            if (qubits[j] < 0 || qubits[j] >= n) return fail(QSV_E_ARG, "qubit out of range");
            for (int i = 0; i < j; ++i)
                if (qubits[i] == qubits[j]) return fail(QSV_E_ARG, "repeated qubit");
            if (qubits[j] != j) full = false;
        }
    }
    DeviceGuard g(s->device);
    const long long N = 1ll << n;
    if (full) {
        const size_t bytes = (size_t)N * (s->dtype == QSV_C64 ? 4 : 8);
        void* dst = out;
        void* tmp = nullptr;
        if (!out_on_device) {
            if (hipMalloc(&tmp, bytes) != hipSuccess) {
                (void)hipGetLastError();
                return fail(QSV_E_OOM, "probability buffer allocation failed");
            }
            dst = tmp;
        }
        hipError_t e = launch_probs_full(s->dtype, s->buf, N, dst, s->stream);
        if (e == hipSuccess && tmp) e = hipMemcpyAsync(out, tmp, bytes, hipMemcpyDeviceToHost, s->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
        if (tmp) (void)hipFree(tmp);
        if (e != hipSuccess) return fail(QSV_E_DEVICE, std::string("probs: ") + hipGetErrorString(e));
        return QSV_OK;
    }
    MargArgs a{};
    a.n = n;
    a.m = m;
    unsigned long long Q = 0;
    for (int j = 0; j < m; ++j) {
        a.q[j] = qubits ? qubits[j] : j;
        Q |= 1ull << a.q[j];
    }
    int r = 0;
    for (int b = 0; b < n; ++b)
        if (!((Q >> b) & 1)) a.rest[r++] = b;
    const long long M = 1ll << m, R = 1ll << (n - m);
    long long nchunks = std::max<long long>(1, (1ll << 20) / M);
    nchunks = std::min(nchunks, R);
    a.nchunks = nchunks;
    a.chunk = R / nchunks;
    const size_t pbytes = (size_t)(M * nchunks) * 2 * sizeof(double);
    const size_t obytes = (size_t)M * sizeof(double);
    if ((st = ensure_work(s, pbytes + (out_on_device ? 0 : obytes))) != QSV_OK) return st;
    double* partial = s->d_work;
    double* dout = out_on_device ? (double*)out : (double*)((char*)s->d_work + pbytes);
    QSV_HIP(launch_probs_marg(s->dtype, s->buf, a, partial, dout, s->stream));
    if (!out_on_device) QSV_HIP(hipMemcpyAsync(out, dout, obytes, hipMemcpyDeviceToHost, s->stream));
    QSV_HIP(hipStreamSynchronize(s->stream));
    return QSV_OK;
}

// Adjoint-method gradient (Jones and Gacon's reverse sweep), for rotations
// R_P(theta) = exp(-i theta P / 2) (Eq. 4):  dE/dtheta_l = Im <lambda_l| P_l |phi_l>, with
// phi_l the state just after op l and lambda_l = U_{l+1}^dag ... U_L^dag H |psi>.
// Consecutive rotations on distinct qubits commute, so every rotation of such a layer
// is evaluated at the layer's end in one read pass over (lambda, phi); between
// evaluation points phi and lambda are uncomputed with one fused plan of inverse gates.
namespace {

// Device scratch owned by one call; freed on every exit path.
struct DevBuf {
    void* p = nullptr;
    ~DevBuf() { if (p) (void)hipFree(p); }
    bool alloc(size_t bytes)
    {
        if (hipMalloc(&p, bytes ? bytes : 16) != hipSuccess) {
            (void)hipGetLastError();
            p = nullptr;
            return false;
        }
        return true;
    }
};

}  // namespace

qsv_status qsv_sample(qsv_state s, const int* qubits, int m, const double* uniforms, long long shots,
                      long long* out)
{
    qsv_status st = check_state(s);
    if (st != QSV_OK) return st;
    const int n = s->n;
    if (shots < 0) return fail(QSV_E_ARG, "shots must be >= 0");
    if (shots > 0 && (!uniforms || !out)) return fail(QSV_E_ARG, "uniforms or out is null");
    if (m < 1 || m > n) return fail(QSV_E_ARG, "m must be in [1, n]");
    bool identity = (m == n);
    if (qubits) {
        for (int j = 0; j < m; ++j) {
            if (qubits[j] < 0 || qubits[j] >= n) return fail(QSV_E_ARG, "qubit out of range");
            for (int i = 0; i < j; ++i)
                if (qubits[i] == qubits[j]) return fail(QSV_E_ARG, "repeated qubit");
            if (qubits[j] != j) identity = false;
        }
    } else if (m != n) {
        return fail(QSV_E_ARG, "qubits == NULL measures all n qubits (m must be n)");
    }
    for (long long i = 0; i < shots; ++i)
        if (!(uniforms[i] >= 0.0 && uniforms[i] < 1.0)) return fail(QSV_E_ARG, "uniforms must lie in [0, 1)");
    if (!identity && m > 26) return fail(QSV_E_UNSUPPORTED, "marginal sampling over more than 26 qubits");
    if (shots == 0) return QSV_OK;
    DeviceGuard g(s->device);

    // the distribution: the state itself (all qubits in order) or an FP64 marginal table
    DevBuf table;
    const void* src = s->buf;
    int sdt = s->dtype;
    if (!identity) {
        if (!table.alloc(sizeof(double) << m)) return fail(QSV_E_OOM, "sampling table allocation failed");
        if ((st = qsv_probs(s, qubits, m, table.p, 1)) != QSV_OK) return st;
        src = table.p;
        sdt = 2;
    }
    const int cb = std::min(m, kSampleChunkBits);
    const long long nchunks = 1ll << (m - cb);

    // chunk totals -> host prefix sums (sequential, FP64)
    DevBuf dtot;
    if (!dtot.alloc(sizeof(double) * nchunks)) return fail(QSV_E_OOM, "sampling buffer allocation failed");
    std::vector<double> S(nchunks), Cp(nchunks + 1, 0.0);
    QSV_HIP(launch_chunk_totals(sdt, src, cb, nchunks, (double*)dtot.p, s->stream));
    QSV_HIP(hipMemcpyAsync(S.data(), dtot.p, sizeof(double) * nchunks, hipMemcpyDeviceToHost, s->stream));
    QSV_HIP(hipStreamSynchronize(s->stream));
    long long lastnz = -1;
    for (long long c = 0; c < nchunks; ++c) {
        Cp[c + 1] = Cp[c] + S[c];
        if (S[c] > 0) lastnz = c;
    }
    const double P = Cp[nchunks];
    if (lastnz < 0 || !(P > 0)) return fail(QSV_E_ARG, "the state has no probability mass");

    // On the device: the shots in increasing order of u (equal values in index order);
    // each goes to the chunk whose prefix interval holds u * P, with its residual inside
    // that chunk; shots of one chunk form a run, resolved together by one workgroup
    long long c0 = 0;
    while (c0 < lastnz && S[c0] <= 0) ++c0;
    DevBuf du, dorder, dscratch, dcum, dres, dlist, dnruns, dgot, dout;
    const size_t sb = std::max(sort_uniforms_scratch(shots), sample_assign_scratch(shots));
    if (!du.alloc(sizeof(double) * shots) || !dorder.alloc(sizeof(long long) * shots) || !dscratch.alloc(sb) ||
        !dcum.alloc(sizeof(double) * (nchunks + 1)) || !dres.alloc(sizeof(double) * shots) ||
        !dlist.alloc(sizeof(SampleChunk) * std::min<long long>(shots, nchunks)) || !dnruns.alloc(sizeof(long long)) ||
        !dgot.alloc(sizeof(long long) * shots) || !dout.alloc(sizeof(long long) * shots))
        return fail(QSV_E_OOM, "sampling buffer allocation failed");
    QSV_HIP(hipMemcpyAsync(du.p, uniforms, sizeof(double) * shots, hipMemcpyHostToDevice, s->stream));
    QSV_HIP(hipMemcpyAsync(dcum.p, Cp.data(), sizeof(double) * (nchunks + 1), hipMemcpyHostToDevice, s->stream));
    QSV_HIP(sort_uniforms((const double*)du.p, shots, (long long*)dorder.p, dscratch.p, sb, s->stream));
    QSV_HIP(sample_assign((const double*)du.p, (const long long*)dorder.p, shots, (const double*)dcum.p, c0, lastnz, P,
                          (double*)dres.p, (SampleChunk*)dlist.p, (long long*)dnruns.p, dscratch.p, sb, s->stream));
    long long nruns = 0;
    QSV_HIP(hipMemcpyAsync(&nruns, dnruns.p, sizeof(long long), hipMemcpyDeviceToHost, s->stream));
    QSV_HIP(hipStreamSynchronize(s->stream));
    QSV_HIP(launch_sample_chunks(sdt, src, cb, (const SampleChunk*)dlist.p, nruns, (const double*)dres.p,
                                 (long long*)dgot.p, s->stream));
    QSV_HIP(scatter_outcomes((const long long*)dorder.p, (const long long*)dgot.p, shots, (long long*)dout.p,
                             s->stream));
    QSV_HIP(hipMemcpyAsync(out, dout.p, sizeof(long long) * shots, hipMemcpyDeviceToHost, s->stream));
    QSV_HIP(hipStreamSynchronize(s->stream));
    return QSV_OK;
}

}  // extern "C"

namespace {

// Superoperator of a channel with Kraus operators K (d x d each) on targets T, as a
// (d^2 x d^2) matrix on (T, T + n): local row index r_row + d r_col, column c_row + d c_col,
// entry sum_a K_a[r_row][c_row] conj(K_a[r_col][c_col]).
std::vector<cd> superop(const std::vector<std::vector<cd>>& kraus, int d)
{
    const int D = d * d;
    std::vector<cd> S((size_t)D * D, cd(0, 0));
    for (const auto& K : kraus)
        for (int rr = 0; rr < d; ++rr)
            for (int rc = 0; rc < d; ++rc)
                for (int cr = 0; cr < d; ++cr)
                    for (int cc = 0; cc < d; ++cc)
                        S[(size_t)(rr + d * rc) * D + (cr + d * cc)] +=
                            K[(size_t)rr * d + cr] * std::conj(K[(size_t)rc * d + cc]);
    return S;
}

bool dm_ops_to_gates(const qsv_dm_op* ops, size_t n_ops, int nsys, std::vector<InGate>& out, std::string& err)
{
    const cd I(0, 1);
    const std::vector<std::vector<cd>> pauli = {{1, 0, 0, 1}, {0, 1, 1, 0}, {0, -I, I, 0}, {1, 0, 0, -1}};
    for (size_t i = 0; i < n_ops; ++i) {
        const qsv_dm_op& o = ops[i];
        const std::string at = "op " + std::to_string(i) + ": ";
        if (o.kind == 0) {
            qsv_gate g{};
            g.k = o.k;
            for (int j = 0; j < 5; ++j) g.targets[j] = o.targets[j];
            g.mat = o.mat;
            InGate u;
            if (!read_gate(g, nsys, u, err)) { err = at + err; return false; }
            InGate v = u;
            for (int j = 0; j < u.k; ++j) v.t[j] = u.t[j] + nsys;
            for (cd& x : v.m) x = std::conj(x);
            out.push_back(std::move(u));
            out.push_back(std::move(v));
            continue;
        }
        if (o.kind != 1 && o.kind != 2) { err = at + "kind must be 0, 1 or 2"; return false; }
        if (!(o.p >= 0.0 && o.p <= 1.0)) { err = at + "channel probability must be in [0, 1]"; return false; }
        const int k = o.k;
        if (k < 1 || k > 2 || (o.kind == 2 && k != 1)) { err = at + "channel on 1 (or, depolarizing, 2) targets"; return false; }
        for (int j = 0; j < k; ++j) {
            if (o.targets[j] < 0 || o.targets[j] >= nsys) { err = at + "target out of range"; return false; }
            for (int l = 0; l < j; ++l)
                if (o.targets[l] == o.targets[j]) { err = at + "duplicate target"; return false; }
        }
        const int d = 1 << k;
        std::vector<std::vector<cd>> kraus;
        if (o.kind == 1) {
            const int np = d * d - 1;   // non-identity Pauli strings
            for (int a = 0; a <= np; ++a) {
                const double w = std::sqrt(a == 0 ? 1.0 - o.p : o.p / np);
                std::vector<cd> K((size_t)d * d);
                for (int r = 0; r < d; ++r)
                    for (int c = 0; c < d; ++c) {
                        cd v = w;
                        for (int j = 0; j < k; ++j) {   // Pauli (a >> 2j) & 3 on local bit j
                            const int pj = (a >> (2 * j)) & 3;
                            v *= pauli[pj][(size_t)((r >> j) & 1) * 2 + ((c >> j) & 1)];
                        }
                        K[(size_t)r * d + c] = v;
                    }
                kraus.push_back(std::move(K));
            }
        } else {
            kraus.push_back({1, 0, 0, std::sqrt(1.0 - o.p)});
            kraus.push_back({0, std::sqrt(o.p), 0, 0});
        }
        InGate g;
        g.k = 2 * k;
        for (int j = 0; j < kMaxK; ++j) g.t[j] = 0;
        for (int j = 0; j < k; ++j) {
            g.t[j] = o.targets[j];
            g.t[k + j] = o.targets[j] + nsys;
        }
        g.m = superop(kraus, d);
        out.push_back(std::move(g));
    }
    return true;
}

qsv_status dm_check(qsv_state s, int& nsys)
{
    qsv_status st = check_state(s);
    if (st != QSV_OK) return st;
    if (s->n < 2 || (s->n & 1)) return fail(QSV_E_ARG, "a density matrix needs a state of 2n qubits");
    nsys = s->n / 2;
    return QSV_OK;
}

}  // namespace

extern "C" {

qsv_status qsv_dm_apply(qsv_state s, const qsv_dm_op* ops, size_t n_ops, const qsv_plan_opts* opts)
{
    int nsys = 0;
    qsv_status st = dm_check(s, nsys);
    if (st != QSV_OK) return st;
    if (n_ops && !ops) return fail(QSV_E_ARG, "ops is null");
    std::vector<InGate> gates;
    std::string err;
    if (!dm_ops_to_gates(ops, n_ops, nsys, gates, err)) return fail(QSV_E_ARG, err);
    if (gates.empty()) return QSV_OK;
    PlanOpts o;
    if (!plan_opts_from(s->dtype, opts, o, err)) return fail(QSV_E_ARG, err);
    HostPlan hp;
    if (!make_plan(s->n, s->dtype, gates, o, hp, err)) return fail(QSV_E_ARG, err);
    DeviceGuard g(s->device);
    if ((st = enqueue_plan(s, hp)) != QSV_OK) return st;
    QSV_HIP(hipStreamSynchronize(s->stream));
    return QSV_OK;
}

qsv_status qsv_dm_probs(qsv_state s, const int* qubits, int m, double* out)
{
    int nsys = 0;
    qsv_status st = dm_check(s, nsys);
    if (st != QSV_OK) return st;
    if (!out) return fail(QSV_E_ARG, "out is null");
    if (!qubits) m = nsys;
    if (m < 1 || m > nsys) return fail(QSV_E_ARG, "m must be in [1, n]");
    MargArgs a{};
    a.n = nsys;
    a.m = m;
    unsigned long long Q = 0;
    for (int j = 0; j < m; ++j) {
        const int q = qubits ? qubits[j] : j;
        if (q < 0 || q >= nsys) return fail(QSV_E_ARG, "qubit out of range");
        if ((Q >> q) & 1) return fail(QSV_E_ARG, "repeated qubit");
        a.q[j] = q;
        Q |= 1ull << q;
    }
    int r = 0;
    for (int b = 0; b < nsys; ++b)
        if (!((Q >> b) & 1)) a.rest[r++] = b;
    const long long M = 1ll << m, Rn = 1ll << (nsys - m);
    long long nchunks = std::min(std::max<long long>(1, (1ll << 16) / M), Rn);
    a.nchunks = nchunks;
    a.chunk = Rn / nchunks;
    const size_t pbytes = (size_t)(M * nchunks) * 2 * sizeof(double);
    const size_t obytes = (size_t)M * sizeof(double);
    DeviceGuard g(s->device);
    if ((st = ensure_work(s, pbytes + obytes)) != QSV_OK) return st;
    double* partial = s->d_work;
    double* dout = (double*)((char*)s->d_work + pbytes);
    QSV_HIP(launch_probs_marg(s->dtype, s->buf, a, partial, dout, s->stream, true));
    QSV_HIP(hipMemcpyAsync(out, dout, obytes, hipMemcpyDeviceToHost, s->stream));
    QSV_HIP(hipStreamSynchronize(s->stream));
    return QSV_OK;
}

qsv_status qsv_dm_expval_pauli(qsv_state s, const qsv_pauli_term* terms, size_t n_terms, double* per_term,
                               double* sum)
{
    int nsys = 0;
    qsv_status st = dm_check(s, nsys);
    if (st != QSV_OK) return st;
    if (n_terms && !terms) return fail(QSV_E_ARG, "terms is null");
    std::vector<PTerm> pt;
    std::string err;
    if (!parse_terms(terms, n_terms, nsys, pt, err)) return fail(QSV_E_ARG, err);
    DeviceGuard g(s->device);
    const int grid = (int)std::min<long long>(1024, std::max<long long>(1, (1ll << nsys) / kThreads));
    NS total;
    for (size_t b0 = 0; b0 < pt.size(); b0 += kMaxPauliApply) {
        PauliSumArgs p{};
        p.nterms = (int)std::min<size_t>(kMaxPauliApply, pt.size() - b0);
        for (int i = 0; i < p.nterms; ++i) {
            p.x[i] = (long long)pt[b0 + i].x;
            p.z[i] = (long long)pt[b0 + i].z;
            p.ny[i] = pt[b0 + i].ny;
            p.coeff[i] = pt[b0 + i].coeff;
        }
        const size_t bytes = (size_t)grid * p.nterms * 2 * sizeof(double);
        if ((st = ensure_work(s, bytes)) != QSV_OK) return st;
        if ((st = ensure_hwork(s, bytes)) != QSV_OK) return st;
        QSV_HIP(launch_dm_pauli(s->dtype, s->buf, nsys, p, grid, s->d_work, s->stream));
        QSV_HIP(hipMemcpyAsync(s->h_work, s->d_work, bytes, hipMemcpyDeviceToHost, s->stream));
        QSV_HIP(hipStreamSynchronize(s->stream));
        for (int i = 0; i < p.nterms; ++i) {
            NS acc;
            for (int b = 0; b < grid; ++b) {
                acc.add(s->h_work[((size_t)b * p.nterms + i) * 2]);
                acc.c += s->h_work[((size_t)b * p.nterms + i) * 2 + 1];
            }
            const double v = pt[b0 + i].coeff * acc.value();
            if (per_term) per_term[b0 + i] = v;
            total.add(v);
        }
    }
    if (sum) *sum = total.value();
    return QSV_OK;
}

qsv_status qsv_adjoint_grad(int n, qsv_dtype dtype, const qsv_op* ops, size_t n_ops, const double* params, int B,
                            int P, const qsv_pauli_term* H, size_t n_terms, double* energy, double* grad,
                            void* stream)
{
    if (n < 1 || n > kMaxQubits) return fail(QSV_E_ARG, "n_qubits must be in [1, 34]");
    if (dtype != QSV_C64 && dtype != QSV_C128) return fail(QSV_E_ARG, "bad dtype");
    if (B < 0 || P < 0) return fail(QSV_E_ARG, "negative batch or parameter count");
    if ((n_ops && !ops) || (B && P && !params) || (n_terms && !H) || (B && !energy) || (B && P && !grad))
        return fail(QSV_E_ARG, "null argument");
    // validate ops; fixed gates are read once
    std::vector<InGate> fixed(n_ops);
    std::string err;
    for (size_t i = 0; i < n_ops; ++i) {
        const qsv_op& o = ops[i];
        if (o.kind == 0) {
            qsv_gate g{};
            g.k = o.k;
            for (int j = 0; j < 5; ++j) g.targets[j] = o.targets[j];
            g.diag = 0;
            g.mat = o.mat;
            if (!read_gate(g, n, fixed[i], err)) return fail(QSV_E_ARG, "op " + std::to_string(i) + ": " + err);
        } else if (o.kind >= 1 && o.kind <= 3) {
            if (o.targets[0] < 0 || o.targets[0] >= n) return fail(QSV_E_ARG, "rotation target out of range");
            if (o.param < 0 || o.param >= P) return fail(QSV_E_ARG, "rotation parameter index out of range");
        } else {
            return fail(QSV_E_ARG, "op kind must be 0 (gate), 1 (RX), 2 (RY) or 3 (RZ)");
        }
    }
    std::vector<PTerm> hterms;
    if (!parse_terms(H, n_terms, n, hterms, err)) return fail(QSV_E_ARG, err);
    if (B == 0) return QSV_OK;

    // gate of op i under parameter vector th (inverse = conjugate transpose)
    auto op_gate = [&](size_t i, const double* th, bool inverse) {
        InGate g;
        const qsv_op& o = ops[i];
        if (o.kind == 0) {
            g = fixed[i];
        } else {
            const double t = th[o.param];
            const double c = std::cos(t / 2), sn = std::sin(t / 2);
            const cd I(0, 1);
            g.k = 1;
            g.t[0] = o.targets[0];
            for (int j = 1; j < kMaxK; ++j) g.t[j] = 0;
            if (o.kind == 1) g.m = {c, -I * sn, -I * sn, c};
            else if (o.kind == 2) g.m = {c, -sn, sn, c};
            else g.m = {std::polar(1.0, -t / 2), 0, 0, std::polar(1.0, t / 2)};
        }
        if (inverse) {
            const int d = 1 << g.k;
            std::vector<cd> h((size_t)d * d);
            for (int r = 0; r < d; ++r)
                for (int c2 = 0; c2 < d; ++c2) h[(size_t)c2 * d + r] = std::conj(g.m[(size_t)r * d + c2]);
            g.m = h;
        }
        return g;
    };

    // The sweep's structure depends on the op kinds and targets only, not on the angles,
    // so it is planned once.  The circuit still to be undone is kept as a list of op
    // indices in time order.  Each step first undoes the fixed gates at its tail, then
    // takes a layer: walking back from the tail, a rotation joins the layer when no op
    // already passed over (a member or one left behind) touches its qubit.  An op left
    // behind blocks its qubits for everything earlier, so it shares no qubit with any
    // member that precedes it in time and commutes to before the whole layer; in that
    // equivalent order the layer is contiguous at the tail, and all its gradients come
    // from one evaluation at the current point.  The layer is then undone and leaves
    // the list.
    struct Layer {
        std::vector<long long> fixed;   // fixed gates undone first (descending time)
        std::vector<long long> ops;     // the layer's rotations (descending time)
        std::vector<ElemGroup> G;
        // Evaluated before the previous layer's rotations are undone (their undo joins
        // the next step's): each rotation's generator is then conjugated by the previous
        // layer's rotation on its qubit, conj[l] >= 0 naming that RZ (or -1: none, or
        // nothing to conjugate)
        bool deferred = false;
        std::vector<long long> conj;
    };
    std::vector<Layer> layers;
    size_t partial_doubles = 0;
    {
        std::vector<long long> rest(n_ops);
        for (size_t i = 0; i < n_ops; ++i) rest[i] = (long long)i;
        auto qubits_of = [&](long long i) {
            unsigned long long q = 0;
            if (ops[i].kind == 0) {
                for (int j = 0; j < fixed[i].k; ++j) q |= 1ull << fixed[i].t[j];
            } else {
                q = 1ull << ops[i].targets[0];
            }
            return q;
        };
        std::vector<long long> trailing;
        while (!rest.empty()) {
            while (!rest.empty() && ops[rest.back()].kind == 0) {
                trailing.push_back(rest.back());
                rest.pop_back();
            }
            if (rest.empty()) break;
            Layer Ly;
            Ly.fixed.swap(trailing);
            unsigned long long blocked = 0;
            std::vector<char> take(rest.size(), 0);
            const unsigned long long all = (n >= 64) ? ~0ull : ((1ull << n) - 1);
            for (long long r = (long long)rest.size() - 1; r >= 0 && (blocked & all) != all; --r) {
                const long long i = rest[(size_t)r];
                const unsigned long long q = qubits_of(i);
                if (ops[i].kind != 0 && !(blocked & q)) {
                    take[(size_t)r] = 1;
                    Ly.ops.push_back(i);
                }
                blocked |= q;
            }
            std::vector<long long> keep;
            keep.reserve(rest.size());
            for (size_t r = 0; r < rest.size(); ++r)
                if (!take[r]) keep.push_back(rest[r]);
            rest.swap(keep);
            layers.push_back(std::move(Ly));
        }
    }
    // A layer with no fixed gates of its own after it can be evaluated while the
    // previous layer's rotations are still applied, when each of its generators either
    // commutes with the previous layer's rotation on its qubit or is X or Y under an RZ
    // there: RZ(t) X RZ(t)^+ = cos t X + sin t Y and RZ(t) Y RZ(t)^+ = cos t Y - sin t X,
    // one partner product per amplitude with weights that depend on t.  The previous
    // layer's undo then joins the next step's plan (one round of passes fewer per pair of
    // layers).  No chains: the layer after a deferred one is evaluated as usual.
    for (size_t li = 1; li < layers.size(); ++li) {
        Layer& Ly = layers[li];
        const Layer& Pv = layers[li - 1];
        if (!Ly.fixed.empty() || Pv.deferred) continue;
        std::vector<long long> on(n, -1);   // the previous layer's rotation on each qubit
        for (const long long k : Pv.ops) on[ops[k].targets[0]] = k;
        bool ok = true;
        std::vector<long long> conj(Ly.ops.size(), -1);
        for (size_t l = 0; l < Ly.ops.size() && ok; ++l) {
            const qsv_op& o = ops[Ly.ops[l]];
            const long long pk = on[o.targets[0]];
            if (pk < 0) continue;
            if (ops[pk].kind != 3) ok = false;       // only RZ conjugations are taken
            else if (o.kind != 3) conj[l] = pk;      // X or Y generator under an RZ
        }
        if (!ok) continue;
        Ly.deferred = true;
        Ly.conj.swap(conj);
    }
    for (Layer& Ly : layers) {
        std::vector<PTerm> gterms(Ly.ops.size());
        for (size_t l = 0; l < Ly.ops.size(); ++l) {
            const qsv_op& o = ops[Ly.ops[l]];
            const unsigned long long bit = 1ull << o.targets[0];
            PTerm t;
            if (o.kind == 1) t.x = bit;                               // X
            else if (o.kind == 2) { t.x = bit; t.z = bit; t.ny = 1; }  // Y
            else t.z = bit;                                            // Z
            if (Ly.deferred && Ly.conj[l] >= 0) t.z = bit;             // parity-weighted X / Y pair
            t.coeff = 1.0;
            gterms[l] = t;
        }
        size_t d = 0;
        if (!plan_elements(n, gterms, true, Ly.G, d, err, dtype, 1024)) return fail(QSV_E_UNSUPPORTED, err);
        for (ElemGroup& E : Ly.G) E.off += partial_doubles;
        partial_doubles += d;
    }

    // the energy's matrix elements <phi|P_t|phi>: their partials follow the layers'
    std::vector<ElemGroup> Ge;
    {
        size_t d = 0;
        if (!plan_elements(n, hterms, false, Ge, d, err, dtype, 1024)) return fail(QSV_E_UNSUPPORTED, err);
        for (ElemGroup& E : Ge) E.off += partial_doubles;
        partial_doubles += d;
    }

    // Parameter vectors run on up to two (phi, lambda) pairs, each pair on a stream of its
    // own, vector b on pair b % pairs: the host enqueues vector b + 1 while the device
    // still runs vector b, so the start of one overlaps the end of the other and the
    // host's planning between vectors leaves no gap.  The second pair is optional (one
    // pair when it does not fit in memory or B = 1).
    struct Pair {
        qsv_state phi = nullptr, lam = nullptr;
        hipStream_t own = nullptr;   // created here (second pair only)
        int b = -1;                  // vector in flight on this pair
    };
    Pair pair[2];
    const hipStream_t caller = static_cast<hipStream_t>(stream);
    qsv_status st = qsv_alloc(n, dtype, nullptr, 0, stream, &pair[0].phi);
    if (st == QSV_OK) st = qsv_alloc(n, dtype, nullptr, 0, stream, &pair[0].lam);
    int pairs = st == QSV_OK ? 1 : 0;
    if (st == QSV_OK && B > 1) {
        hipEvent_t start = nullptr;
        bool ok = hipStreamCreateWithFlags(&pair[1].own, hipStreamNonBlocking) == hipSuccess;
        // work the caller queued before this call comes first on the second stream too
        ok = ok && hipEventCreateWithFlags(&start, hipEventDisableTiming) == hipSuccess &&
             hipEventRecord(start, caller) == hipSuccess && hipStreamWaitEvent(pair[1].own, start, 0) == hipSuccess;
        if (start) (void)hipEventDestroy(start);
        ok = ok && qsv_alloc(n, dtype, nullptr, 0, pair[1].own, &pair[1].phi) == QSV_OK &&
             qsv_alloc(n, dtype, nullptr, 0, pair[1].own, &pair[1].lam) == QSV_OK;
        if (ok) {
            pairs = 2;
        } else {   // run on one pair
            (void)hipGetLastError();
            qsv_free(pair[1].phi);
            qsv_free(pair[1].lam);
            pair[1].phi = pair[1].lam = nullptr;
            if (pair[1].own) (void)hipStreamDestroy(pair[1].own);
            pair[1].own = nullptr;
        }
    }
    // every layer's partials for one parameter vector, read back once per vector
    const size_t pbytes = std::max<size_t>(partial_doubles, 1) * sizeof(double);
    for (int p = 0; p < pairs && st == QSV_OK; ++p)
        if ((st = ensure_work(pair[p].lam, pbytes)) == QSV_OK) st = ensure_hwork(pair[p].lam, pbytes);
    std::vector<double> gv;
    // Inverse gates undone before each layer's evaluation (the previous layer's
    // rotations, then the layer's fixed gates), in application order.  Their structure,
    // and the forward circuit's, is the same for every parameter vector, so each is
    // planned once from generic angles (no multiples of pi/2, where rotations gain
    // structure) and refreshed with each vector's matrices (refresh_plan); a vector
    // whose matrices break a template's structure is planned from scratch.
    std::vector<std::vector<long long>> undo(layers.size());
    for (size_t li = 0; li < layers.size(); ++li) {
        if (layers[li].deferred) continue;   // evaluated before the previous layer's undo
        if (li > 1 && layers[li - 1].deferred)
            undo[li] = layers[li - 2].ops;   // the undo the deferred layer left behind
        if (li > 0) undo[li].insert(undo[li].end(), layers[li - 1].ops.begin(), layers[li - 1].ops.end());
        undo[li].insert(undo[li].end(), layers[li].fixed.begin(), layers[li].fixed.end());
    }
    auto gates_of = [&](const std::vector<long long>& idx, const double* th, bool inverse) {
        std::vector<InGate> g;
        g.reserve(idx.size());
        for (const long long k : idx) g.push_back(op_gate((size_t)k, th, inverse));
        return g;
    };
    std::vector<long long> all_ops(n_ops);
    for (size_t i = 0; i < n_ops; ++i) all_ops[i] = (long long)i;
    std::vector<double> th_generic((size_t)std::max(P, 1));
    for (size_t j = 0; j < th_generic.size(); ++j) th_generic[j] = 0.5 + 0.7548776662466927 * (double)(j + 1);
    HostPlan fwd_tmpl;
    std::vector<HostPlan> undo_tmpl(layers.size());
    if (st == QSV_OK && n_ops &&
        !make_plan(n, dtype, gates_of(all_ops, th_generic.data(), false), default_opts(dtype), fwd_tmpl, err))
        st = fail(QSV_E_ARG, err);
    for (size_t li = 0; li < layers.size() && st == QSV_OK; ++li)
        if (!undo[li].empty() &&
            !make_plan(n, dtype, gates_of(undo[li], th_generic.data(), true), default_opts(dtype), undo_tmpl[li], err))
            st = fail(QSV_E_ARG, err);
    // a template refreshed with a vector's gates, or a plan made for them
    auto plan_for = [&](const HostPlan& tmpl, const std::vector<InGate>& g, HostPlan& hp) -> qsv_status {
        hp = tmpl;
        if (refresh_plan(hp, g)) return QSV_OK;
        if (!make_plan(n, dtype, g, default_opts(dtype), hp, err)) return fail(QSV_E_ARG, err);
        return QSV_OK;
    };
    // the forward circuit's plan for vector b; the next vector's is built on the host
    // while the device runs the current one
    auto plan_forward = [&](int b, HostPlan& hp) -> qsv_status {
        if (!n_ops) return QSV_OK;
        return plan_for(fwd_tmpl, gates_of(all_ops, params + (size_t)b * P, false), hp);
    };
    // enqueue vector b on pair pr: forward, energy, co-state, reverse sweep, partials copy
    auto enqueue_vector = [&](int b, Pair& pr, const HostPlan& fwd) -> qsv_status {
        qsv_state phi = pr.phi, lam = pr.lam;
        const double* th = params + (size_t)b * P;
        qsv_status s2 = QSV_OK;
        // forward: phi = U(theta)|0>
        if (n_ops) {
            if ((s2 = enqueue_plan(phi, fwd, nullptr, true)) != QSV_OK) return s2;
        } else if ((s2 = qsv_reset(phi)) != QSV_OK) {
            return s2;
        }
        // energy (partials read back with the gradients) and co-state lambda = H phi
        hipError_t he = launch_elements(dtype, phi->buf, phi->buf, Ge, lam->d_work, lam->stream);
        if (he != hipSuccess) return fail(QSV_E_DEVICE, std::string("adjoint: ") + hipGetErrorString(he));
        if ((s2 = pauli_sum_apply(lam, phi->buf, lam->buf, hterms)) != QSV_OK) return s2;
        // reverse sweep, asynchronous: uncompute (fixed gates and the previous layer,
        // one plan applied to both states), then the layer's Im <lambda|P_j|phi>
        for (size_t li = 0; li < layers.size(); ++li) {
            if (!undo[li].empty()) {
                HostPlan hp;
                if ((s2 = plan_for(undo_tmpl[li], gates_of(undo[li], th, true), hp)) != QSV_OK) return s2;
                if ((s2 = enqueue_plan(phi, hp, lam)) != QSV_OK) return s2;   // one launch per pass, both states
            }
            const Layer& Ly = layers[li];
            if (Ly.deferred) {   // generators conjugated by this vector's RZ angles
                std::vector<ElemGroup> G = Ly.G;
                for (ElemGroup& E : G)
                    for (int i = 0; i < E.ta.nterms; ++i) {
                        const size_t l = (size_t)E.idx[i];
                        if (Ly.conj[l] < 0) continue;
                        const double t = th[ops[Ly.conj[l]].param], c = std::cos(t), sn = std::sin(t);
                        // Im <lambda|P'|phi> per element: Re(k conj(lambda[e ^ x]) phi[e]),
                        // k by the parity of e's bit on the qubit
                        const bool ygen = ops[Ly.ops[l]].kind == 2;
                        const double k0r = ygen ? c : sn, k0i = ygen ? sn : -c;
                        const double k1r = ygen ? -c : -sn, k1i = k0i;
                        E.ta.kw[i][0] = k0r;
                        E.ta.kw[i][1] = k0i;
                        E.ta.kw[i][2] = k1r;
                        E.ta.kw[i][3] = k1i;
                    }
                he = launch_elements(dtype, lam->buf, phi->buf, G, lam->d_work, lam->stream);
            } else {
                he = launch_elements(dtype, lam->buf, phi->buf, Ly.G, lam->d_work, lam->stream);
            }
            if (he != hipSuccess) return fail(QSV_E_DEVICE, std::string("adjoint: ") + hipGetErrorString(he));
        }
        if (hipMemcpyAsync(lam->h_work, lam->d_work, pbytes, hipMemcpyDeviceToHost, lam->stream) != hipSuccess)
            return fail(QSV_E_DEVICE, "adjoint: partials read-back failed");
        pr.b = b;
        return QSV_OK;
    };
    // wait for the vector in flight on pair pr and combine its partials
    auto finish_vector = [&](Pair& pr) -> qsv_status {
        if (pr.b < 0) return QSV_OK;
        const int b = pr.b;
        pr.b = -1;
        if (hipStreamSynchronize(pr.lam->stream) != hipSuccess) return fail(QSV_E_DEVICE, "adjoint: partials read-back failed");
        double* gb = grad + (size_t)b * P;
        for (int j = 0; j < P; ++j) gb[j] = 0.0;
        for (const Layer& Ly : layers) {
            combine_elements(Ly.G, pr.lam->h_work, Ly.ops.size(), gv);
            for (size_t l = 0; l < Ly.ops.size(); ++l) gb[ops[Ly.ops[l]].param] += gv[l];
        }
        combine_elements(Ge, pr.lam->h_work, hterms.size(), gv);
        NS e;
        for (size_t t = 0; t < hterms.size(); ++t) e.add(hterms[t].coeff * gv[t]);
        energy[b] = e.value();
        return QSV_OK;
    };
    HostPlan fwd_cur, fwd_next;
    if (st == QSV_OK) st = plan_forward(0, fwd_cur);
    for (int b = 0; b < B && st == QSV_OK; ++b) {
        Pair& pr = pair[b % pairs];
        if ((st = finish_vector(pr)) != QSV_OK) break;   // vector b - pairs
        if ((st = enqueue_vector(b, pr, fwd_cur)) != QSV_OK) break;
        if (b + 1 < B && (st = plan_forward(b + 1, fwd_next)) != QSV_OK) break;
        std::swap(fwd_cur, fwd_next);
    }
    for (int p = 0; p < pairs; ++p) {
        const qsv_status s2 = finish_vector(pair[p]);
        if (st == QSV_OK) st = s2;
    }
    for (int p = 0; p < 2; ++p) {
        qsv_free(pair[p].phi);   // waits for the pair's stream
        qsv_free(pair[p].lam);
        if (pair[p].own) (void)hipStreamDestroy(pair[p].own);
    }
    return st;
}

}  // extern "C"
