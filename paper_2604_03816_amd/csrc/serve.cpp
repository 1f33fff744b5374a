// serve.cpp -- continuous-batching serving core of libqsv.
//
// Requests (a circuit on n qubits, complex64 or complex128) are planned on a pool of
// host threads (DAG fusion + pass scheduling), queued FIFO, and admitted while a slot
// is free and their HBM footprint fits: footprint = state (2^n * s) + the plan's
// resident matrices and tables + reduction workspace, the terms of the paper's memory
// model (Eq. 14), against capacity = free device memory at start minus a reserve
// (Eq. 15).  Each step advances every running request by its next pass(es) in one
// batched launch per dtype and kernel variant (k_batch_pass: a persistent grid over all
// running states' tiles; passes without register-heavy ops take the lighter variant), then reduces the requests that finished (per-qubit <Z_i> and norm) in one
// batched launch, and retires them; requests that arrived meanwhile are admitted at
// the next step.  The step's launches are captured once in a hipGraph and replayed;
// only the small work tables change between steps (copied before each replay).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/qsv.h"
#include "planner.h"
#include "qsv_internal.h"

using namespace qsv;

namespace qsv {
qsv_status set_error(qsv_status st, const std::string& msg);   // capi.cpp
bool read_gate_public(const qsv_gate& g, int n, InGate& out, std::string& err);
}

namespace {

constexpr int kZQ = 12;   // chunk qubits of the batched <Z> reduction (k_zsum_batch)
constexpr int kServeTileQubits[2] = {12, 12};   // 2^12-amplitude tiles (32 / 64 KiB), as the plain path

struct Req {
    long long id = 0;
    int n = 0;
    int dtype = 0;
    int requested = 0;   // the dtype asked for (QSV_AUTO possible)
    int promoted = 0;
    bool keep_gates = false;   // an automatic complex64 run that the norm guard may repeat
    PlanOpts popts;
    std::vector<InGate> gates;
    HostPlan plan;
    std::atomic<int> planned{0};   // 0 queued, 1 planned, -1 failed
    std::string err;
    size_t state_bytes = 0, table_bytes = 0, work_bytes = 0, footprint = 0;
    void* state = nullptr;
    void* tables = nullptr;
    size_t table_cap = 0;
    DevOp* d_ops = nullptr;
    void* d_pool = nullptr;
    int* d_ipool = nullptr;
    float* d_apool = nullptr;
    size_t next_pass = 0;
    double t_submit = 0, t_admit = 0, t_finish = 0;
    long long z_off = 0;   // partial offset while finishing
};

size_t elem(int dtype) { return dtype == QSV_C64 ? 8 : 16; }

size_t round_pow2(size_t b)
{
    size_t r = 256;
    while (r < b) r <<= 1;
    return r;
}

}  // namespace

struct qsv_server_s {
    qsv_server_opts o{};
    hipStream_t stream = nullptr;
    int device = 0;
    std::chrono::steady_clock::time_point t0;
    // planning pool
    std::mutex mu;
    std::condition_variable cv;
    std::deque<std::shared_ptr<Req>> plan_q;
    std::vector<std::thread> workers;
    bool stop = false;
    // scheduling
    long long next_id = 1;
    std::deque<std::shared_ptr<Req>> pending;
    std::vector<std::shared_ptr<Req>> running;
    std::deque<qsv_result> done;
    std::unordered_map<long long, std::shared_ptr<Req>> kept;
    size_t capacity = 0, used = 0, pooled = 0;
    std::map<size_t, std::vector<void*>> pool;   // size class -> free device buffers
    // step work tables: [dtype][j] pass items, [dtype] z items
    std::vector<BatchItem*> h_items, d_items;
    std::vector<int*> h_count, d_count;
    ZItem* h_z[2] = {nullptr, nullptr};
    ZItem* d_z[2] = {nullptr, nullptr};
    int* h_zcount = nullptr;   // [2]
    int* d_zcount = nullptr;
    double* d_partial = nullptr;
    double* h_partial = nullptr;
    size_t partial_cap = 0;    // doubles
    hipGraphExec_t gexec = nullptr;
    hipGraph_t graph = nullptr;
    bool graph_dirty = true;
    hipEvent_t ev = nullptr;
    bool own_stream = false;
    qsv_server_stats st{};

    double now() const
    {
        return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
};

namespace {

void worker_loop(qsv_server s)
{
    for (;;) {
        std::shared_ptr<Req> r;
        {
            std::unique_lock<std::mutex> lk(s->mu);
            s->cv.wait(lk, [&] { return s->stop || !s->plan_q.empty(); });
            if (s->stop && s->plan_q.empty()) return;
            r = s->plan_q.front();
            s->plan_q.pop_front();
        }
        std::string err;
        if (make_plan(r->n, r->dtype, r->gates, r->popts, r->plan, err)) {
            const HostPlan& hp = r->plan;
            r->state_bytes = elem(r->dtype) << r->n;
            r->table_bytes = hp.ops.size() * sizeof(DevOp) + hp.pool.size() * elem(r->dtype) +
                             hp.ipool.size() * sizeof(int) + hp.apool.size() * sizeof(float) + 4 * 256;
            const long long chunks = 1ll << std::max(0, r->n - kZQ);
            r->work_bytes = (size_t)chunks * (kZQ + 1) * sizeof(double);
            r->footprint = r->state_bytes + r->table_bytes + r->work_bytes;   // Eq. 14
            if (!r->keep_gates) {
                r->gates.clear();
                r->gates.shrink_to_fit();
            }
            r->planned.store(1);
        } else {
            r->err = err;
            r->planned.store(-1);
        }
    }
}

void* pool_get(qsv_server s, size_t bytes)
{
    const size_t cls = round_pow2(bytes);
    auto it = s->pool.find(cls);
    if (it != s->pool.end() && !it->second.empty()) {
        void* p = it->second.back();
        it->second.pop_back();
        s->pooled -= cls;
        return p;
    }
    if (s->o.dry_run) return reinterpret_cast<void*>(cls);   // a non-null token
    void* p = nullptr;
    if (hipMalloc(&p, cls) != hipSuccess) {
        (void)hipGetLastError();
        // release cached buffers of other sizes and retry once
        for (auto& kv : s->pool)
            for (void* q : kv.second) (void)hipFree(q);
        s->pool.clear();
        s->pooled = 0;
        if (hipMalloc(&p, cls) != hipSuccess) {
            (void)hipGetLastError();
            return nullptr;
        }
    }
    return p;
}

void pool_put(qsv_server s, void* p, size_t bytes)
{
    if (!p) return;
    const size_t cls = round_pow2(bytes);
    s->pool[cls].push_back(p);
    s->pooled += cls;
}

void release_req(qsv_server s, Req& r)
{
    pool_put(s, r.state, r.state_bytes);
    pool_put(s, r.tables, r.table_cap);
    r.state = nullptr;
    r.tables = nullptr;
    s->used -= r.footprint;
}

qsv_status admit(qsv_server s, const std::shared_ptr<Req>& r)
{
    const HostPlan& hp = r->plan;
    const size_t eb = elem(r->dtype);
    r->state = pool_get(s, r->state_bytes);
    if (!r->state) return set_error(QSV_E_OOM, "state allocation failed");
    const size_t nops = hp.ops.size() * sizeof(DevOp), npool = hp.pool.size() * eb, nip = hp.ipool.size() * sizeof(int);
    const size_t nap = hp.apool.size() * sizeof(float);
    const size_t o_pool = (nops + 255) & ~size_t(255), o_ip = o_pool + ((npool + 255) & ~size_t(255));
    const size_t o_ap = o_ip + ((nip + 255) & ~size_t(255));
    r->table_cap = o_ap + ((nap + 255) & ~size_t(255)) + 256;
    r->tables = pool_get(s, r->table_cap);
    if (!r->tables) {
        pool_put(s, r->state, r->state_bytes);
        r->state = nullptr;
        return set_error(QSV_E_OOM, "plan table allocation failed");
    }
    r->d_ops = (DevOp*)r->tables;
    r->d_pool = (char*)r->tables + o_pool;
    r->d_ipool = (int*)((char*)r->tables + o_ip);
    r->d_apool = (float*)((char*)r->tables + o_ap);
    if (!s->o.dry_run) {
        std::vector<unsigned char> buf(r->table_cap, 0);
        if (nops) std::memcpy(buf.data(), hp.ops.data(), nops);
        for (size_t i = 0; i < hp.pool.size(); ++i) {
            if (r->dtype == QSV_C64) {
                float* f = reinterpret_cast<float*>(buf.data() + o_pool) + 2 * i;
                f[0] = (float)hp.pool[i].real();
                f[1] = (float)hp.pool[i].imag();
            } else {
                double* f = reinterpret_cast<double*>(buf.data() + o_pool) + 2 * i;
                f[0] = hp.pool[i].real();
                f[1] = hp.pool[i].imag();
            }
        }
        if (nip) std::memcpy(buf.data() + o_ip, hp.ipool.data(), nip);
        if (nap) std::memcpy(buf.data() + o_ap, hp.apool.data(), nap);
        hipError_t e = hipMemcpyAsync(r->tables, buf.data(), r->table_cap, hipMemcpyHostToDevice, s->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(s->stream);   // buf is pageable and goes out of scope
        if (e == hipSuccess) e = launch_init_zero(r->dtype, r->state, 1ll << r->n, s->stream);
        if (e != hipSuccess) return set_error(QSV_E_DEVICE, std::string("admit: ") + hipGetErrorString(e));
    }
    s->used += r->footprint;
    r->t_admit = s->now();
    r->next_pass = 0;
    return QSV_OK;
}

int passes_per_step(qsv_server s) { return std::max(1, s->o.passes_per_step); }

qsv_status ensure_partial(qsv_server s, size_t doubles)
{
    if (doubles <= s->partial_cap) return QSV_OK;
    size_t cap = std::max<size_t>(doubles, 1 << 16);
    cap = round_pow2(cap * sizeof(double)) / sizeof(double);
    if (s->d_partial) {
        (void)hipStreamSynchronize(s->stream);
        (void)hipFree(s->d_partial);
        (void)hipHostFree(s->h_partial);
        s->d_partial = nullptr;
        s->h_partial = nullptr;
    }
    if (hipMalloc((void**)&s->d_partial, cap * sizeof(double)) != hipSuccess ||
        hipHostMalloc((void**)&s->h_partial, cap * sizeof(double), hipHostMallocDefault) != hipSuccess) {
        (void)hipGetLastError();
        s->partial_cap = 0;
        return set_error(QSV_E_OOM, "server workspace allocation failed");
    }
    s->partial_cap = cap;
    s->graph_dirty = true;   // kernels captured with the old pointer
    return QSV_OK;
}

// The step's kernel sequence (captured into the graph, or launched directly).
hipError_t launch_step(qsv_server s)
{
    const int P = passes_per_step(s);
    const int grid = s->o.grid > 0 ? s->o.grid : 2048;
    // work list (wide, dtype, j) at slot (2 wide + dtype) P + j: passes with register-heavy
    // ops go to the wide kernel variant, the rest to the lighter one
    for (int j = 0; j < P; ++j)
        for (int w = 0; w < 2; ++w)
            for (int dt = 0; dt < 2; ++dt) {
                const int slot = (2 * w + dt) * P + j;
                hipError_t e = launch_batch_pass(dt, s->d_items[slot], s->d_count[slot], grid, kServeTileQubits[dt],
                                                 s->stream, w != 0);
                if (e != hipSuccess) return e;
            }
    for (int dt = 0; dt < 2; ++dt) {
        hipError_t e = launch_zsum_batch(dt, s->d_z[dt], s->d_zcount + dt, s->d_partial, 1024, s->stream);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

qsv_status run_step_device(qsv_server s, size_t zdoubles)
{
    const int P = passes_per_step(s);
    const int slots = std::max(1, s->o.max_slots);
    // work tables to the device (outside the graph)
    for (int i = 0; i < 4 * P; ++i) {
        const int cnt = *s->h_count[i];
        if (hipMemcpyAsync(s->d_count[i], s->h_count[i], sizeof(int), hipMemcpyHostToDevice, s->stream) != hipSuccess ||
            (cnt > 0 && hipMemcpyAsync(s->d_items[i], s->h_items[i], cnt * sizeof(BatchItem), hipMemcpyHostToDevice,
                                       s->stream) != hipSuccess))
            return set_error(QSV_E_DEVICE, "step table upload failed");
    }
    for (int dt = 0; dt < 2; ++dt) {
        const int cnt = s->h_zcount[dt];
        if (cnt > 0 && hipMemcpyAsync(s->d_z[dt], s->h_z[dt], cnt * sizeof(ZItem), hipMemcpyHostToDevice, s->stream) !=
                           hipSuccess)
            return set_error(QSV_E_DEVICE, "step table upload failed");
    }
    if (hipMemcpyAsync(s->d_zcount, s->h_zcount, 2 * sizeof(int), hipMemcpyHostToDevice, s->stream) != hipSuccess)
        return set_error(QSV_E_DEVICE, "step table upload failed");
    (void)slots;
    hipError_t e = hipSuccess;
    if (s->o.use_graph) {
        if (s->graph_dirty) {
            if (s->gexec) {
                (void)hipGraphExecDestroy(s->gexec);
                (void)hipGraphDestroy(s->graph);
                s->gexec = nullptr;
                s->graph = nullptr;
            }
            e = hipStreamBeginCapture(s->stream, hipStreamCaptureModeThreadLocal);
            if (e == hipSuccess) {
                hipError_t le = launch_step(s);
                e = hipStreamEndCapture(s->stream, &s->graph);
                if (le != hipSuccess) e = le;
            }
            if (e == hipSuccess) e = hipGraphInstantiate(&s->gexec, s->graph, nullptr, nullptr, 0);
            if (e != hipSuccess) return set_error(QSV_E_DEVICE, std::string("graph capture: ") + hipGetErrorString(e));
            s->graph_dirty = false;
        }
        e = hipGraphLaunch(s->gexec, s->stream);
        ++s->st.graph_replays;
    } else {
        e = launch_step(s);
    }
    if (e == hipSuccess && zdoubles > 0)
        e = hipMemcpyAsync(s->h_partial, s->d_partial, zdoubles * sizeof(double), hipMemcpyDeviceToHost, s->stream);
    if (e == hipSuccess) e = hipEventRecord(s->ev, s->stream);
    if (e == hipSuccess) e = hipEventSynchronize(s->ev);
    if (e != hipSuccess) return set_error(QSV_E_DEVICE, std::string("step: ") + hipGetErrorString(e));
    return QSV_OK;
}

}  // namespace

extern "C" {

qsv_status qsv_server_create(const qsv_server_opts* opts, void* stream, qsv_server* out)
{
    if (!out) return set_error(QSV_E_ARG, "out is null");
    *out = nullptr;
    qsv_server s = new qsv_server_s();
    if (opts) s->o = *opts;
    if (s->o.max_slots <= 0) s->o.max_slots = 64;
    s->o.max_slots = std::min(s->o.max_slots, kMaxBatchItems);
    if (s->o.passes_per_step <= 0) s->o.passes_per_step = 1;
    if (s->o.planner_threads <= 0) s->o.planner_threads = 4;
    if (s->o.reserve_bytes == 0) s->o.reserve_bytes = (size_t)1 << 30;
    s->stream = (hipStream_t)stream;
    s->t0 = std::chrono::steady_clock::now();
    if (!s->o.dry_run && !s->stream) {
        if (hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking) != hipSuccess) {
            delete s;
            return set_error(QSV_E_DEVICE, "stream creation failed");
        }
        s->own_stream = true;
    }
    if (!s->o.dry_run && prepare_batch_pass() != hipSuccess) {
        if (s->own_stream) (void)hipStreamDestroy(s->stream);
        delete s;
        return set_error(QSV_E_DEVICE, "batched pass kernel set-up failed");
    }
    const int P = s->o.passes_per_step;
    const int slots = s->o.max_slots;
    if (s->o.dry_run) {
        s->capacity = s->o.capacity_bytes ? s->o.capacity_bytes : ((size_t)1 << 34);
    } else {
        if (hipGetDevice(&s->device) != hipSuccess) {
            delete s;
            return set_error(QSV_E_DEVICE, "no HIP device");
        }
        size_t fr = 0, tot = 0;
        if (hipMemGetInfo(&fr, &tot) != hipSuccess) {
            delete s;
            return set_error(QSV_E_DEVICE, "hipMemGetInfo failed");
        }
        s->capacity = s->o.capacity_bytes ? s->o.capacity_bytes : (fr > s->o.reserve_bytes ? fr - s->o.reserve_bytes : 0);
        bool ok = hipEventCreateWithFlags(&s->ev, hipEventDisableTiming) == hipSuccess;
        s->h_items.assign(4 * P, nullptr);
        s->d_items.assign(4 * P, nullptr);
        s->h_count.assign(4 * P, nullptr);
        s->d_count.assign(4 * P, nullptr);
        for (int i = 0; ok && i < 4 * P; ++i) {
            ok = hipHostMalloc((void**)&s->h_items[i], slots * sizeof(BatchItem), hipHostMallocDefault) == hipSuccess &&
                 hipMalloc((void**)&s->d_items[i], slots * sizeof(BatchItem)) == hipSuccess &&
                 hipHostMalloc((void**)&s->h_count[i], sizeof(int), hipHostMallocDefault) == hipSuccess &&
                 hipMalloc((void**)&s->d_count[i], sizeof(int)) == hipSuccess;
        }
        for (int dt = 0; ok && dt < 2; ++dt)
            ok = hipHostMalloc((void**)&s->h_z[dt], slots * sizeof(ZItem), hipHostMallocDefault) == hipSuccess &&
                 hipMalloc((void**)&s->d_z[dt], slots * sizeof(ZItem)) == hipSuccess;
        ok = ok && hipHostMalloc((void**)&s->h_zcount, 2 * sizeof(int), hipHostMallocDefault) == hipSuccess &&
             hipMalloc((void**)&s->d_zcount, 2 * sizeof(int)) == hipSuccess;
        if (!ok || ensure_partial(s, 1 << 16) != QSV_OK) {
            (void)hipGetLastError();
            qsv_server_free(s);
            return set_error(QSV_E_OOM, "server table allocation failed");
        }
    }
    for (int i = 0; i < s->o.planner_threads; ++i) s->workers.emplace_back(worker_loop, s);
    *out = s;
    return QSV_OK;
}

qsv_status qsv_server_free(qsv_server s)
{
    if (!s) return QSV_OK;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
    }
    s->cv.notify_all();
    for (auto& t : s->workers) t.join();
    if (!s->o.dry_run) {
        (void)hipStreamSynchronize(s->stream);
        for (auto& r : s->running) release_req(s, *r);
        for (auto& kv : s->kept) release_req(s, *kv.second);
        for (auto& kv : s->pool)
            for (void* p : kv.second) (void)hipFree(p);
        if (s->gexec) (void)hipGraphExecDestroy(s->gexec);
        if (s->graph) (void)hipGraphDestroy(s->graph);
        for (size_t i = 0; i < s->h_items.size(); ++i) {
            (void)hipHostFree(s->h_items[i]);
            (void)hipFree(s->d_items[i]);
            (void)hipHostFree(s->h_count[i]);
            (void)hipFree(s->d_count[i]);
        }
        for (int dt = 0; dt < 2; ++dt) {
            (void)hipHostFree(s->h_z[dt]);
            (void)hipFree(s->d_z[dt]);
        }
        (void)hipHostFree(s->h_zcount);
        (void)hipFree(s->d_zcount);
        (void)hipFree(s->d_partial);
        (void)hipHostFree(s->h_partial);
        if (s->ev) (void)hipEventDestroy(s->ev);
        if (s->own_stream) (void)hipStreamDestroy(s->stream);
    }
    delete s;
    return QSV_OK;
}

qsv_status qsv_server_submit(qsv_server s, int n, qsv_dtype dtype, const qsv_gate* gates, size_t n_gates,
                             const qsv_plan_opts* popts, long long* id)
{
    if (!s || !id) return set_error(QSV_E_ARG, "null argument");
    if (n < 1 || n > kMaxQubits) return set_error(QSV_E_ARG, "n_qubits must be in [1, 34]");
    if (dtype != QSV_C64 && dtype != QSV_C128 && dtype != QSV_AUTO) return set_error(QSV_E_ARG, "bad dtype");
    if (n_gates && !gates) return set_error(QSV_E_ARG, "gates is null");
    auto r = std::make_shared<Req>();
    r->n = n;
    r->requested = dtype;
    if (dtype == QSV_AUTO) {
        qsv_dtype chosen = QSV_C128;
        (void)qsv_precision_select(n, n_gates, s->o.eps_tol, &chosen);
        dtype = chosen;
        r->keep_gates = (dtype == QSV_C64 && s->o.norm_guard > 0);
        ++(dtype == QSV_C64 ? s->st.auto_c64 : s->st.auto_c128);
    }
    r->dtype = dtype;
    std::string oerr;
    if (!plan_opts_from(dtype, popts, r->popts, oerr)) return set_error(QSV_E_ARG, oerr);
    // served tiles are capped at 2^12 amplitudes (the batched launch sizes its LDS for
    // that tile plus the capped operand block)
    const int cap = kServeTileQubits[dtype];
    r->popts.tile_qubits = std::min(r->popts.tile_qubits, cap);
    r->popts.whole_state_max = std::min(r->popts.whole_state_max, cap);
    r->popts.mfma_lds_floats = std::min(r->popts.mfma_lds_floats, kServeOperandFloats);
    if (r->popts.low_qubits >= r->popts.tile_qubits) r->popts.low_qubits = r->popts.tile_qubits - 1;
    r->gates.resize(n_gates);
    std::string err;
    for (size_t i = 0; i < n_gates; ++i)
        if (!read_gate_public(gates[i], n, r->gates[i], err))
            return set_error(QSV_E_ARG, "gate " + std::to_string(i) + ": " + err);
    {
        std::lock_guard<std::mutex> lk(s->mu);
        r->id = s->next_id++;
        r->t_submit = s->now();
        s->plan_q.push_back(r);
        s->pending.push_back(r);
    }
    s->cv.notify_one();
    ++s->st.submitted;
    *id = r->id;
    return QSV_OK;
}

qsv_status qsv_server_step(qsv_server s, int* n_running, int* n_pending)
{
    if (!s) return set_error(QSV_E_ARG, "null server");
    const int P = passes_per_step(s);
    // 1. admission, FIFO: the head waits for memory rather than being overtaken
    while (!s->pending.empty() && (int)s->running.size() < s->o.max_slots) {
        std::shared_ptr<Req> r = s->pending.front();
        const int pl = r->planned.load();
        if (pl == 0) break;
        if (pl < 0) {
            qsv_result res{};
            res.id = r->id;
            res.n = r->n;
            res.dtype = r->dtype;
            res.status = QSV_E_ARG;
            res.t_submit = r->t_submit;
            res.t_finish = s->now();
            s->done.push_back(res);
            s->pending.pop_front();
            continue;
        }
        if (r->footprint > s->capacity) {   // can never fit: reject rather than block forever
            qsv_result res{};
            res.id = r->id;
            res.n = r->n;
            res.dtype = r->dtype;
            res.status = QSV_E_OOM;
            res.t_submit = r->t_submit;
            res.t_finish = s->now();
            s->done.push_back(res);
            s->pending.pop_front();
            ++s->st.rejected;
            continue;
        }
        if (s->used + r->footprint + s->pooled > s->capacity) {
            // drop cached buffers first
            if (!s->o.dry_run)
                for (auto& kv : s->pool)
                    for (void* p : kv.second) (void)hipFree(p);
            s->pool.clear();
            s->pooled = 0;
            if (s->used + r->footprint > s->capacity) {
                ++s->st.admission_waits;
                break;
            }
        }
        const qsv_status st = admit(s, r);
        if (st != QSV_OK) return st;
        s->running.push_back(r);
        s->pending.pop_front();
        ++s->st.admitted;
        s->st.peak_running = std::max<long long>(s->st.peak_running, (long long)s->running.size());
        s->st.peak_used_bytes = std::max<long long>(s->st.peak_used_bytes, (long long)s->used);
    }
    // 2. work tables
    std::vector<std::shared_ptr<Req>> finishing;
    size_t zdoubles = 0;
    if (!s->o.dry_run) {
        for (int i = 0; i < 4 * P; ++i) *s->h_count[i] = 0;
        s->h_zcount[0] = s->h_zcount[1] = 0;
    }
    long long tiles_step = 0;
    for (auto& r : s->running) {
        const HostPlan& hp = r->plan;
        const size_t np = hp.passes.size();
        for (int j = 0; j < P && r->next_pass + j < np; ++j) {
            const size_t pi = r->next_pass + j;
            tiles_step += hp.pgrid[pi];
            if (s->o.dry_run) continue;
            const int slot = (2 * (hp.pwide[pi] ? 1 : 0) + r->dtype) * P + j;
            int& cnt = *s->h_count[slot];
            BatchItem& it = s->h_items[slot][cnt];
            it.state = r->state;
            it.ops = r->d_ops;
            it.pool = r->d_pool;
            it.ipool = r->d_ipool;
            it.apool = r->d_apool;
            it.a = hp.pargs[pi];
            it.ntiles = hp.pgrid[pi];
            it.tile_end = (cnt ? s->h_items[slot][cnt - 1].tile_end : 0) + it.ntiles;
            ++cnt;
        }
        if (r->next_pass + P >= np) {
            finishing.push_back(r);
            if (!s->o.dry_run) {
                const int dt = r->dtype;
                int& cnt = s->h_zcount[dt];
                ZItem& z = s->h_z[dt][cnt];
                z.state = r->state;
                z.n = r->n;
                z.nchunks = 1ll << std::max(0, r->n - kZQ);
                z.chunk_end = (cnt ? s->h_z[dt][cnt - 1].chunk_end : 0) + z.nchunks;
                z.partial_off = (long long)zdoubles;
                r->z_off = (long long)zdoubles;
                zdoubles += (size_t)z.nchunks * (kZQ + 1);
                ++cnt;
            }
        }
    }
    // 3. launch and wait
    if (!s->running.empty() && !s->o.dry_run) {
        qsv_status st = ensure_partial(s, zdoubles);
        if (st != QSV_OK) return st;
        st = run_step_device(s, zdoubles);
        if (st != QSV_OK) return st;
        ++s->st.steps;
        s->st.tiles += tiles_step;
    } else if (!s->running.empty()) {
        ++s->st.steps;
        s->st.tiles += tiles_step;
    }
    // 4. harvest
    const double tnow = s->now();
    for (auto& r : finishing) {
        qsv_result res{};
        res.id = r->id;
        res.n = r->n;
        res.dtype = r->dtype;
        res.status = QSV_OK;
        res.t_submit = r->t_submit;
        res.t_admit = r->t_admit;
        res.t_finish = tnow;
        res.passes = (long long)r->plan.passes.size();
        res.fused = (long long)r->plan.fused.size();
        if (!s->o.dry_run) {
            // norm = sum of chunk totals; <Z_i> = norm - 2 * sum over amplitudes with bit i set
            const long long nch = 1ll << std::max(0, r->n - kZQ);
            const double* p = s->h_partial + r->z_off;
            double tot = 0, tc = 0;
            std::vector<double> ones(r->n, 0.0), oc(r->n, 0.0);
            auto nadd2 = [](double& a, double& c, double x) {
                const double t = a + x;
                c += (std::fabs(a) >= std::fabs(x)) ? ((a - t) + x) : ((x - t) + a);
                a = t;
            };
            const int cq = std::min(r->n, kZQ);
            for (long long c = 0; c < nch; ++c) {
                const double* q = p + c * (kZQ + 1);
                nadd2(tot, tc, q[0]);
                for (int b = 0; b < cq; ++b) nadd2(ones[b], oc[b], q[1 + b]);
                for (int b = cq; b < r->n; ++b)
                    if (((c << cq) >> b) & 1) nadd2(ones[b], oc[b], q[0]);
            }
            res.norm = tot + tc;
            for (int b = 0; b < r->n; ++b) res.zexp[b] = res.norm - 2.0 * (ones[b] + oc[b]);
        }
        res.requested = r->requested;
        res.promoted = r->promoted;
        if (r->keep_gates && !s->o.dry_run && std::fabs(res.norm - 1.0) > s->o.norm_guard) {
            // the complex64 run drifted: run the request again in complex128, ahead of
            // the queue, under the same id and arrival time
            auto q = std::make_shared<Req>();
            q->id = r->id;
            q->n = r->n;
            q->dtype = QSV_C128;
            q->requested = r->requested;
            q->promoted = 1;
            q->t_submit = r->t_submit;
            std::string oerr;
            (void)plan_opts_from(QSV_C128, nullptr, q->popts, oerr);
            const int cap = kServeTileQubits[QSV_C128];
            q->popts.tile_qubits = std::min(q->popts.tile_qubits, cap);
            q->popts.whole_state_max = std::min(q->popts.whole_state_max, cap);
            q->popts.mfma_lds_floats = std::min(q->popts.mfma_lds_floats, kServeOperandFloats);
            if (q->popts.low_qubits >= q->popts.tile_qubits) q->popts.low_qubits = q->popts.tile_qubits - 1;
            q->popts.fuse = r->popts.fuse;
            q->popts.commute = r->popts.commute;
            if (q->popts.fuse == 0) q->popts.max_ops_per_pass = 1;
            q->gates.swap(r->gates);
            {
                std::lock_guard<std::mutex> lk(s->mu);
                s->plan_q.push_front(q);
                s->pending.push_front(q);
            }
            s->cv.notify_one();
            ++s->st.promoted;
            release_req(s, *r);
            continue;
        }
        s->done.push_back(res);
        ++s->st.finished;
        if (s->o.keep_states && !s->o.dry_run) {
            s->kept[r->id] = r;
        } else {
            release_req(s, *r);
        }
    }
    if (!finishing.empty()) {
        std::vector<std::shared_ptr<Req>> keep;
        for (auto& r : s->running)
            if (std::find(finishing.begin(), finishing.end(), r) == finishing.end()) keep.push_back(r);
        s->running.swap(keep);
    }
    for (auto& r : s->running) r->next_pass += P;
    if (n_running) *n_running = (int)s->running.size();
    if (n_pending) *n_pending = (int)s->pending.size();
    return QSV_OK;
}

// Default tolerance of Eq. 12: 49.5 gates x 2^20 x 1.19e-7, so that at 20 qubits circuits
// of fewer than 50 gates run in complex64 and those of 50 or more in complex128 (Section
// 8.4); the Section 5.4 example (20 qubits, 200 gates: about 25) stays in complex128.
constexpr double kDefaultEpsTol = 49.5 * 1048576.0 * 1.19e-7;

qsv_status qsv_precision_select(int n, size_t n_gates, double eps_tol, qsv_dtype* out)
{
    if (!out) return set_error(QSV_E_ARG, "out is null");
    if (n < 1 || n > kMaxQubits) return set_error(QSV_E_ARG, "n_qubits must be in [1, 34]");
    const double tol = eps_tol > 0 ? eps_tol : kDefaultEpsTol;
    const double bound = (double)n_gates * std::ldexp(1.0, n) * 1.19e-7;   // Eq. 11, complex64
    *out = bound <= tol ? QSV_C64 : QSV_C128;                               // Eq. 12
    return QSV_OK;
}

qsv_status qsv_server_results(qsv_server s, qsv_result* out, int max, int* count)
{
    if (!s || !count || (max > 0 && !out)) return set_error(QSV_E_ARG, "null argument");
    int c = 0;
    while (c < max && !s->done.empty()) {
        out[c++] = s->done.front();
        s->done.pop_front();
    }
    *count = c;
    return QSV_OK;
}

qsv_status qsv_server_get_stats(qsv_server s, qsv_server_stats* st)
{
    if (!s || !st) return set_error(QSV_E_ARG, "null argument");
    *st = s->st;
    st->capacity_bytes = (long long)s->capacity;
    st->used_bytes = (long long)s->used;
    st->running = (long long)s->running.size();
    st->pending = (long long)s->pending.size();
    return QSV_OK;
}

qsv_status qsv_server_get_state(qsv_server s, long long id, void* host_out)
{
    if (!s || !host_out) return set_error(QSV_E_ARG, "null argument");
    auto it = s->kept.find(id);
    if (it == s->kept.end()) return set_error(QSV_E_ARG, "no kept state with this id");
    Req& r = *it->second;
    hipError_t e = hipMemcpyAsync(host_out, r.state, r.state_bytes, hipMemcpyDeviceToHost, s->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
    if (e != hipSuccess) return set_error(QSV_E_DEVICE, std::string("get_state: ") + hipGetErrorString(e));
    return QSV_OK;
}

qsv_status qsv_server_release(qsv_server s, long long id)
{
    if (!s) return set_error(QSV_E_ARG, "null server");
    auto it = s->kept.find(id);
    if (it == s->kept.end()) return set_error(QSV_E_ARG, "no kept state with this id");
    release_req(s, *it->second);
    s->kept.erase(it);
    return QSV_OK;
}

}  // extern "C"
