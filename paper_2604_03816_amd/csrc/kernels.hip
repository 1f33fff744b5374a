// kernels.hip -- HIP kernels of libqsv for gfx950 (MI355X, CDNA4, wave64).
//
// State layout: 2^n interleaved complex numbers (float2 for complex64, double2 for
// complex128), qubit t = bit t of the index (Eq. 2 / Eq. 3).
//
// Apply pass (k_pass): one workgroup per tile.  A tile is 2^m amplitudes whose
// indices differ only in the pass's m tile qubits: the L lowest qubits (so each tile
// row is a contiguous run of 2^L amplitudes in HBM) plus m - L higher qubits (rows
// strided by 2^q).  The workgroup streams its tile from HBM into LDS, applies every
// op of the pass in order on the LDS copy (dense k-qubit unitaries, diagonal phase
// tables, generalised permutations), and streams it back: one HBM round trip per
// pass however many fused gates it carries.  When the whole state fits in LDS the
// single tile is the state and one launch runs the whole circuit.
//
// Reductions read the state once, accumulate in FP64 per thread (products of FP32
// operands are exact in FP64), reduce each workgroup in a fixed order, and leave
// one partial per workgroup; the host combines partials in a fixed order with
// Neumaier's compensated sum, so results are run-to-run deterministic.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <type_traits>

#include "qsv_internal.h"

namespace qsv {

// Address-space-qualified pointers: the state lives in global memory, plan tables are
// read-only (constant address space, so uniform reads become scalar loads).  Pointers
// that a kernel reads from memory (batched launches) carry no address space of their
// own; typing the helpers' parameters keeps every access global or scalar, never flat.
// (The host compilation pass of this file never runs these helpers and sees plain
// pointers.)
#if defined(__HIP_DEVICE_COMPILE__)
template <typename T> using gptr = __attribute__((address_space(1))) T*;
template <typename T> using cptr = const __attribute__((address_space(4))) T*;
#else
template <typename T> using gptr = T*;
template <typename T> using cptr = const T*;
#endif

template <typename R> struct CT;
template <> struct CT<float> { using T = float2; };
template <> struct CT<double> { using T = double2; };

template <typename C>
__device__ __forceinline__ C cmul(C a, C b)
{
    C r;
    r.x = a.x * b.x - a.y * b.y;
    r.y = a.x * b.y + a.y * b.x;
    return r;
}

template <typename C>
__device__ __forceinline__ void cmac(C& acc, C a, C b)
{
    acc.x = fma(a.x, b.x, acc.x);
    acc.x = fma(-a.y, b.y, acc.x);
    acc.y = fma(a.x, b.y, acc.y);
    acc.y = fma(a.y, b.x, acc.y);
}

__device__ __forceinline__ long long tile_base(const PassArgs& a, long long t)
{
    long long base = 0;
    for (int i = 0; i < a.nruns; ++i) {
        base |= (t & ((1ll << a.run_len[i]) - 1)) << a.run_pos[i];
        t >>= a.run_len[i];
    }
    return base;
}

// Offset (relative to the tile base) of the local bits [lo, hi) of local index e.
__device__ __forceinline__ long long local_off_bits(const PassArgs& a, int e, int lo, int hi)
{
    long long o = 0;
    for (int i = lo; i < hi; ++i) {
        if ((e >> i) & 1) o += (i < a.L) ? (1ll << i) : (1ll << a.hbit[i - a.L]);
    }
    return o;
}

// Move a tile between HBM and LDS.  Local index e = 256 * slice + tid: the bits below 8
// come from the thread id (offset computed once per thread), the bits above from the
// slice number; with the slice count NS a compile-time constant every slice's offset
// is a sum of uniform strides (scalar ALU) and all NS loads of a thread are issued
// back to back before the first is consumed.
__device__ __forceinline__ long long local_stride(const PassArgs& a, int i)
{
    return (i < a.L) ? (1ll << i) : (1ll << a.hbit[i - a.L]);
}

template <typename C, bool LOAD, int NS>
__device__ __forceinline__ void move_tile_n(gptr<C> __restrict__ st, C* __restrict__ lds, const PassArgs& a,
                                            long long toff)
{
    constexpr int LB = NS >= 32 ? 5 : NS >= 16 ? 4 : NS >= 8 ? 3 : NS >= 4 ? 2 : NS >= 2 ? 1 : 0;
    long long hs[LB > 0 ? LB : 1];
#pragma unroll
    for (int b = 0; b < LB; ++b) hs[b] = local_stride(a, kLogThreads + b);
    const int tid = threadIdx.x;
    C v[NS];
    if (LOAD) {
#pragma unroll
        for (int j = 0; j < NS; ++j) {
            long long so = 0;
#pragma unroll
            for (int b = 0; b < LB; ++b)
                if ((j >> b) & 1) so += hs[b];
            v[j] = st[toff + so];
        }
#pragma unroll
        for (int j = 0; j < NS; ++j) lds[(j << kLogThreads) + tid] = v[j];
    } else {
#pragma unroll
        for (int j = 0; j < NS; ++j) v[j] = lds[(j << kLogThreads) + tid];
#pragma unroll
        for (int j = 0; j < NS; ++j) {
            long long so = 0;
#pragma unroll
            for (int b = 0; b < LB; ++b)
                if ((j >> b) & 1) so += hs[b];
            st[toff + so] = v[j];
        }
    }
}

template <typename C, bool LOAD>
__device__ __forceinline__ void move_tile(gptr<C> __restrict__ st, C* __restrict__ lds, const PassArgs& a,
                                          long long base)
{
    const int tid = threadIdx.x;
    const int lowb = a.m < kLogThreads ? a.m : kLogThreads;
    const long long toff = base + local_off_bits(a, tid, 0, lowb);
    switch (a.m - kLogThreads) {
    case 0: move_tile_n<C, LOAD, 1>(st, lds, a, toff); break;
    case 1: move_tile_n<C, LOAD, 2>(st, lds, a, toff); break;
    case 2: move_tile_n<C, LOAD, 4>(st, lds, a, toff); break;
    case 3: move_tile_n<C, LOAD, 8>(st, lds, a, toff); break;
    case 4: move_tile_n<C, LOAD, 16>(st, lds, a, toff); break;
    case 5: move_tile_n<C, LOAD, 32>(st, lds, a, toff); break;
    default:   // tiles smaller than one slice (whole states below 256 amplitudes)
        if (tid < (1 << a.m)) {
            if (LOAD) lds[tid] = st[toff];
            else st[toff] = lds[tid];
        }
        break;
    }
}

// Offset of local basis row r of an op inside the tile: bit j of r sits at lpos[j].
template <int K>
__device__ __forceinline__ int row_off(int r, const DevOp& op)
{
    int o = 0;
#pragma unroll
    for (int j = 0; j < K; ++j)
        if ((r >> j) & 1) o += 1 << op.lpos[j];
    return o;
}

// Group g of an op: insert a zero bit at each target position (ascending).
template <int K>
__device__ __forceinline__ int group_base(int g, const DevOp& op)
{
    int b = g;
#pragma unroll
    for (int j = 0; j < K; ++j) {
        const int p = op.lpos[j];
        b = ((b >> p) << (p + 1)) | (b & ((1 << p) - 1));
    }
    return b;
}

template <typename C, int K>
__device__ void op_dense(C* __restrict__ lds, int T, const DevOp& op, cptr<C> __restrict__ M)
{
    constexpr int D = 1 << K;
    const int G = T >> K;
    for (int g = threadIdx.x; g < G; g += kThreads) {
        const int b = group_base<K>(g, op);
        C v[D];
#pragma unroll
        for (int r = 0; r < D; ++r) v[r] = lds[b + row_off<K>(r, op)];
        // rows are not unrolled for wide gates: the row's matrix entries are uniform
        // (scalar) loads, the inputs stay in registers
        constexpr int RU = K <= 2 ? D : 1;
#pragma unroll RU
        for (int r = 0; r < D; ++r) {
            C acc;
            acc.x = 0;
            acc.y = 0;
#pragma unroll
            for (int c = 0; c < D; ++c) cmac(acc, M[r * D + c], v[c]);
            lds[b + row_off<K>(r, op)] = acc;
        }
    }
}

// Dense complex64 op on FP32 matrix cores.  The op is the real-embedded 2D x 2D matrix
// (D = 2^K) times the tile viewed as D x (T / D) complex columns (one column per group of
// amplitudes that differ only in the op's targets).  A wave takes 16 groups at a time:
// lane (q, col) = (lane / 16, lane % 16) feeds group `col`, complex input rows 4 j + q
// (real part, then imaginary part, as two K = 4 steps), and receives output rows
// 8 rb + 2 q and 8 rb + 2 q + 1 of row block rb.  The A operands (host-arranged, see
// the planner; staged in LDS once per kernel) stay in registers for the whole op.  All reads of a block precede its
// writes, so the update is in place; waves own disjoint groups.
typedef float floatx4 __attribute__((ext_vector_type(4)));

template <int K>
__device__ void op_dense_mfma(float2* __restrict__ lds, int T, const DevOp& op, const float* __restrict__ A)
{
    constexpr int D = 1 << K, R2 = 2 * D, RB = R2 / 16, KS = R2 / 4;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int q = lane >> 4, col = lane & 15;
    float a[RB][KS];
#pragma unroll
    for (int rb = 0; rb < RB; ++rb)
#pragma unroll
        for (int ks = 0; ks < KS; ++ks) a[rb][ks] = A[(rb * KS + ks) * 64 + lane];
    const int nblk = (T >> K) >> 4;
    for (int blk = wave; blk < nblk; blk += kThreads / 64) {
        const int b = group_base<K>((blk << 4) + col, op);
        floatx4 acc[RB];
#pragma unroll
        for (int rb = 0; rb < RB; ++rb) acc[rb] = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int j = 0; j < KS / 2; ++j) {
            const float2 v = lds[b + row_off<K>(4 * j + q, op)];
#pragma unroll
            for (int rb = 0; rb < RB; ++rb) {
                acc[rb] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[rb][2 * j], v.x, acc[rb], 0, 0, 0);
                acc[rb] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[rb][2 * j + 1], v.y, acc[rb], 0, 0, 0);
            }
        }
#pragma unroll
        for (int rb = 0; rb < RB; ++rb) {
            lds[b + row_off<K>(8 * rb + 2 * q, op)] = make_float2(acc[rb][0], acc[rb][1]);
            lds[b + row_off<K>(8 * rb + 2 * q + 1, op)] = make_float2(acc[rb][2], acc[rb][3]);
        }
    }
}

template <typename C, int K>
__device__ void op_perm(C* __restrict__ lds, int T, const DevOp& op, cptr<C> __restrict__ ph,
                        cptr<int> __restrict__ src)
{
    constexpr int D = 1 << K;
    const int G = T >> K;
    const bool phased = op.flags != 0;
    for (int g = threadIdx.x; g < G; g += kThreads) {
        const int b = group_base<K>(g, op);
        C v[D];
#pragma unroll
        for (int r = 0; r < D; ++r) v[r] = lds[b + row_off<K>(src[r], op)];
#pragma unroll
        for (int r = 0; r < D; ++r) lds[b + row_off<K>(r, op)] = phased ? cmul(ph[r], v[r]) : v[r];
    }
}

template <typename C>
__device__ void op_diag(C* __restrict__ lds, int T, const DevOp& op, cptr<C> __restrict__ Dg,
                        long long base)
{
    // targets outside the tile contribute a per-tile constant part of the table index
    int gfix = 0, lp[kMaxDiagK];
#pragma unroll
    for (int j = 0; j < kMaxDiagK; ++j) {
        lp[j] = (j < op.k) ? op.lpos[j] : -1;
        if (j < op.k && lp[j] < 0) gfix |= (int)((base >> op.gbit[j]) & 1) << j;
    }
    for (int e = threadIdx.x; e < T; e += kThreads) {
        int idx = gfix;
#pragma unroll
        for (int j = 0; j < kMaxDiagK; ++j)
            if (lp[j] >= 0) idx |= ((e >> lp[j]) & 1) << j;
        lds[e] = cmul(lds[e], Dg[idx]);
    }
}

template <typename C>
__device__ __forceinline__ void apply_ops(C* __restrict__ lds, int T, cptr<DevOp> __restrict__ ops, int op_begin,
                          int op_count, cptr<C> __restrict__ pool, cptr<int> __restrict__ ipool,
                          const float* __restrict__ alds, long long base)
{
    for (int oi = 0; oi < op_count; ++oi) {
        const DevOp op = ops[op_begin + oi];
        cptr<C> M = pool + op.off;
        if constexpr (std::is_same<C, float2>::value) {
            if (op.kind == OP_DENSE && op.aoff >= 0) {
                const float* Am = alds + op.aoff;
                switch (op.k) {
                case 3: op_dense_mfma<3>(lds, T, op, Am); break;
                case 4: op_dense_mfma<4>(lds, T, op, Am); break;
                default: op_dense_mfma<5>(lds, T, op, Am); break;
                }
                __syncthreads();
                continue;
            }
        }
        if (op.kind == OP_DENSE) {
            switch (op.k) {
            case 1: op_dense<C, 1>(lds, T, op, M); break;
            case 2: op_dense<C, 2>(lds, T, op, M); break;
            case 3: op_dense<C, 3>(lds, T, op, M); break;
            case 4: op_dense<C, 4>(lds, T, op, M); break;
            default: op_dense<C, 5>(lds, T, op, M); break;
            }
        } else if (op.kind == OP_PERM) {
            cptr<int> S = ipool + op.ioff;
            switch (op.k) {
            case 1: op_perm<C, 1>(lds, T, op, M, S); break;
            case 2: op_perm<C, 2>(lds, T, op, M, S); break;
            case 3: op_perm<C, 3>(lds, T, op, M, S); break;
            case 4: op_perm<C, 4>(lds, T, op, M, S); break;
            default: op_perm<C, 5>(lds, T, op, M, S); break;
            }
        } else {
            op_diag<C>(lds, T, op, M, base);
        }
        __syncthreads();
    }
}

// The pass's MFMA operand block, global -> LDS (once per kernel, or per work item in
// batched launches).
__device__ __forceinline__ void stage_operands(float* __restrict__ alds, cptr<float> __restrict__ apool,
                                               const PassArgs& a)
{
    for (int i = threadIdx.x; i < a.a_len; i += kThreads) alds[i] = apool[a.a_off + i];
}

// One tile of one pass: HBM -> LDS, every op of the pass, LDS -> HBM.
template <typename C>
__device__ __forceinline__ void run_tile(gptr<C> __restrict__ st, C* __restrict__ lds, const PassArgs& a,
                                         long long tile, cptr<DevOp> __restrict__ ops, cptr<C> __restrict__ pool,
                                         cptr<int> __restrict__ ipool, const float* __restrict__ alds)
{
    const long long base = tile_base(a, tile);
    move_tile<C, true>(st, lds, a, base);
    __syncthreads();
    apply_ops<C>(lds, 1 << a.m, ops, a.op_begin, a.op_count, pool, ipool, alds, base);
    move_tile<C, false>(st, lds, a, base);
}

template <typename C>
__global__ __launch_bounds__(kThreads) void k_pass(C* __restrict__ st, const PassArgs a,
                                                   const DevOp* __restrict__ ops,
                                                   const C* __restrict__ pool,
                                                   const int* __restrict__ ipool,
                                                   const float* __restrict__ apool)
{
    extern __shared__ __align__(16) unsigned char smem[];
    C* lds = reinterpret_cast<C*>(smem);
    float* alds = reinterpret_cast<float*>(smem + (sizeof(C) << a.m));
    stage_operands(alds, (cptr<float>)apool, a);
    __syncthreads();
    run_tile<C>((gptr<C>)st, lds, a, blockIdx.x, (cptr<DevOp>)ops, (cptr<C>)pool, (cptr<int>)ipool, alds);
}

// Batched pass for continuous batching: one launch advances many independent states,
// each by its own current pass.  Work item w (a tile of one item's pass) is found by
// binary search over the items' tile prefix sums; the grid is persistent (fixed size,
// strided over the work list) so the launch can be captured once and replayed.
template <typename C>
__global__ __launch_bounds__(kThreads) void k_batch_pass(const BatchItem* __restrict__ items,
                                                         const int* __restrict__ count)
{
    extern __shared__ __align__(16) unsigned char smem[];
    C* lds = reinterpret_cast<C*>(smem);
    __shared__ long long ends[kMaxBatchItems];
    const int nitems = min(*count, kMaxBatchItems);
    if (nitems <= 0) return;
    for (int i = threadIdx.x; i < nitems; i += kThreads) ends[i] = items[i].tile_end;
    __syncthreads();
    const long long total = ends[nitems - 1];
    for (long long w = blockIdx.x; w < total; w += gridDim.x) {
        int lo = 0, hi = nitems - 1;
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (ends[mid] <= w) lo = mid + 1;
            else hi = mid;
        }
        // the search runs on LDS values, which live in vector registers; the result is
        // the same on every lane, and saying so keeps every later descriptor and op
        // table read a scalar (uniform) load
        lo = __builtin_amdgcn_readfirstlane(lo);
        const BatchItem& it = items[lo];
        const long long tile = w - (it.tile_end - it.ntiles);
        // pointers read from memory carry no address space: state in global memory
        // (global, not flat, loads and stores), plan tables read-only (scalar loads)
        float* alds = reinterpret_cast<float*>(smem + (sizeof(C) << it.a.m));
        if (it.a.a_len > 0) {
            stage_operands(alds, (cptr<float>)it.apool, it.a);
            __syncthreads();
        }
        run_tile<C>((gptr<C>)it.state, lds, it.a, tile, (cptr<DevOp>)it.ops, (cptr<C>)it.pool,
                    (cptr<int>)it.ipool, alds);
        __syncthreads();   // the next work item reuses the LDS tile
    }
}

template <typename C>
__global__ __launch_bounds__(kThreads) void k_zero(C* __restrict__ st, long long N)
{
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += stride) {
        C z;
        z.x = 0;
        z.y = 0;
        st[i] = z;
    }
}

template <typename C>
__global__ __launch_bounds__(kThreads) void k_init_zero(C* __restrict__ st, long long N)
{
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += stride) {
        C z;
        z.x = (i == 0) ? 1 : 0;
        z.y = 0;
        st[i] = z;
    }
}

// ------------------------------------------------------------------ reductions

struct NSum {
    double s, c;
};

__device__ __forceinline__ void nadd(NSum& a, double x)
{
    const double t = a.s + x;
    a.c += (fabs(a.s) >= fabs(x)) ? ((a.s - t) + x) : ((x - t) + a.s);
    a.s = t;
}

__device__ __forceinline__ NSum ncombine(NSum a, NSum b)
{
    NSum r = a;
    nadd(r, b.s);
    r.c += b.c;
    return r;
}

// Fixed-order workgroup reduction of Neumaier pairs: butterfly within each wave,
// then wave results combined in wave order by thread 0.  Returns the result in
// thread 0.
__device__ NSum block_reduce(NSum v, NSum* scratch)
{
    for (int d = 32; d >= 1; d >>= 1) {
        NSum o;
        o.s = __shfl_xor(v.s, d);
        o.c = __shfl_xor(v.c, d);
        v = ((threadIdx.x & d) == 0) ? ncombine(v, o) : ncombine(o, v);
    }
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) scratch[w] = v;
    __syncthreads();
    NSum r = {0.0, 0.0};
    if (threadIdx.x == 0) {
        r = scratch[0];
        for (int i = 1; i < (int)(blockDim.x >> 6); ++i) r = ncombine(r, scratch[i]);
    }
    __syncthreads();
    return r;
}

template <typename C>
__global__ __launch_bounds__(kThreads) void k_norm(const C* __restrict__ st, long long N,
                                                   double* __restrict__ partial)
{
    __shared__ NSum scratch[kThreads / 64];
    NSum a = {0.0, 0.0};
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += stride) {
        const C v = st[i];
        const double x = v.x, y = v.y;
        nadd(a, x * x + y * y);
    }
    const NSum r = block_reduce(a, scratch);
    if (threadIdx.x == 0) {
        partial[2 * blockIdx.x] = r.s;
        partial[2 * blockIdx.x + 1] = r.c;
    }
}

// Pauli matrix elements over tiles: value_t = sum_k Re( i^ny conj(a[k xor x]) b[k] ) *
// (-1)^popcount(k & zy), i.e. Re <a|P_t|b> (ny may carry an extra 3 to give Im instead).
// Each term's X/Y support lies inside the tile.  A thread owns local elements
// e = 256 j + tid (j < NS) of every tile.  The sign of element e splits into a part fixed
// by the tile and tid and a Walsh function of j, so for all terms without X/Y factors a
// single Walsh-Hadamard transform over j of the products conj(a_e) b_e (|a_e|^2 when
// a == b), done in registers once per tile, yields every term as one LDS lookup.  Terms
// with X/Y factors read their partner amplitude a[e xor x] from an LDS copy of the tile.
// FP64 per thread; the workgroup partials are combined in a fixed order.
struct TermRow {
    int x, z, q, pad;
    long long g;
};

template <typename C, int NS, bool TWO>
__device__ __forceinline__ void expval_tiles(gptr<C> __restrict__ sa, gptr<C> __restrict__ sb,
                                             unsigned char* __restrict__ smem, const TermRow* __restrict__ rows,
                                             const PassArgs& a, int nterms, bool anyx, long long ntiles,
                                             double (&acc)[kMaxTermsPerLaunch])
{
    constexpr int LB = NS >= 32 ? 5 : NS >= 16 ? 4 : NS >= 8 ? 3 : NS >= 4 ? 2 : NS >= 2 ? 1 : 0;
    constexpr int T = NS << kLogThreads;
    double* wre = reinterpret_cast<double*>(smem);               // T doubles: transform of Re
    double* wim = wre + T;                                       // T doubles: transform of Im (TWO)
    C* tla = reinterpret_cast<C*>(smem + (TWO ? 2 : 1) * T * sizeof(double));   // tile of a (anyx)
    C* tlb = tla + T;                                            // tile of b (anyx && TWO)
    long long hs[LB > 0 ? LB : 1];
#pragma unroll
    for (int b = 0; b < LB; ++b) hs[b] = local_stride(a, kLogThreads + b);
    const int tid = threadIdx.x;
    const long long tl = local_off_bits(a, tid, 0, kLogThreads);
    auto soff = [&](int j) {
        long long so = 0;
#pragma unroll
        for (int b = 0; b < LB; ++b)
            if ((j >> b) & 1) so += hs[b];
        return so;
    };
    for (long long tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        const long long base = tile_base(a, tile);
        C av[NS], bv[NS];
#pragma unroll
        for (int j = 0; j < NS; ++j) av[j] = sa[base + tl + soff(j)];
        if (TWO) {
#pragma unroll
            for (int j = 0; j < NS; ++j) bv[j] = sb[base + tl + soff(j)];
        }
        if (anyx) {
#pragma unroll
            for (int j = 0; j < NS; ++j) tla[(j << kLogThreads) + tid] = av[j];
            if (TWO) {
#pragma unroll
                for (int j = 0; j < NS; ++j) tlb[(j << kLogThreads) + tid] = bv[j];
            }
        }
        double re[NS], im[NS];
#pragma unroll
        for (int j = 0; j < NS; ++j) {
            const C be = TWO ? bv[j] : av[j];
            re[j] = (double)av[j].x * (double)be.x + (double)av[j].y * (double)be.y;
            im[j] = TWO ? (double)av[j].x * (double)be.y - (double)av[j].y * (double)be.x : 0.0;
        }
        // natural-order Walsh-Hadamard transform: w[z] = sum_j (-1)^popcount(j & z) r[j]
#pragma unroll
        for (int h = 1; h < NS; h <<= 1) {
#pragma unroll
            for (int j = 0; j < NS; ++j) {
                if (j & h) continue;
                const double u = re[j], v = re[j | h];
                re[j] = u + v;
                re[j | h] = u - v;
                if (TWO) {
                    const double ui = im[j], vi = im[j | h];
                    im[j] = ui + vi;
                    im[j | h] = ui - vi;
                }
            }
        }
#pragma unroll
        for (int j = 0; j < NS; ++j) {
            wre[(j << kLogThreads) + tid] = re[j];
            if (TWO) wim[(j << kLogThreads) + tid] = im[j];
        }
        __syncthreads();
        // the term index stays a compile-time constant so that acc lives in registers;
        // term rows come from LDS so that nothing per term is hoisted out of the tile loop
#pragma unroll
        for (int i = 0; i < kMaxTermsPerLaunch; ++i) {
            if (i < nterms) {
                const int x = __builtin_amdgcn_readfirstlane(rows[i].x);
                const int z = __builtin_amdgcn_readfirstlane(rows[i].z);
                const int q = __builtin_amdgcn_readfirstlane(rows[i].q);
                const long long g = rows[i].g;
                const int zhi = z >> kLogThreads;
                const bool neg = (__popc(tid & z & (kThreads - 1)) + __popcll(base & g)) & 1;
                double val;
                if (x == 0) {
                    const int w = (zhi << kLogThreads) + tid;
                    const double r = wre[w], m = TWO ? wim[w] : 0.0;
                    val = (q == 0) ? r : (q == 1) ? -m : (q == 2) ? -r : m;
                } else {
                    val = 0.0;
#pragma unroll 4
                    for (int j = 0; j < NS; ++j) {
                        const int e = (j << kLogThreads) | tid;
                        const C ap = tla[e ^ x];
                        const C be = TWO ? tlb[e] : tla[e];
                        const double pr = (double)ap.x * (double)be.x + (double)ap.y * (double)be.y;
                        const double pi = (double)ap.x * (double)be.y - (double)ap.y * (double)be.x;
                        const double v = (q == 0) ? pr : (q == 1) ? -pi : (q == 2) ? -pr : pi;
                        val += (__popc(j & zhi) & 1) ? -v : v;
                    }
                }
                acc[i] += neg ? -val : val;
            }
        }
        __syncthreads();   // the next tile overwrites LDS
    }
}

// LDS bytes of one k_expval workgroup for a tile of 2^m amplitudes.
__host__ __device__ constexpr size_t expval_lds_bytes(size_t elem, int m, bool two, bool anyx)
{
    return ((two ? 2 : 1) * sizeof(double) + (anyx ? (two ? 2 : 1) * elem : 0)) << m;
}

template <typename C, bool TWO>
__global__ __launch_bounds__(kThreads) void k_expval(const C* __restrict__ sa, const C* __restrict__ sb,
                                                     const PassArgs a, const TermArgs t, long long ntiles,
                                                     double* __restrict__ partial)
{
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ NSum scratch[kThreads / 64];
    __shared__ TermRow rows[kMaxTermsPerLaunch];
    bool anyx = false;
    for (int i = 0; i < t.nterms; ++i) anyx |= t.xloc[i] != 0;
    if (threadIdx.x < t.nterms) {
        const int i = threadIdx.x;
        rows[i] = TermRow{t.xloc[i], t.zloc[i], t.ny[i] & 3, 0, t.zglob[i]};
    }
    __syncthreads();
    double acc[kMaxTermsPerLaunch];
#pragma unroll
    for (int i = 0; i < kMaxTermsPerLaunch; ++i) acc[i] = 0.0;
    gptr<C> ga = (gptr<C>)const_cast<C*>(sa), gb = (gptr<C>)const_cast<C*>(sb);
    switch (a.m - kLogThreads) {   // tiles of 2^8 .. 2^11 amplitudes
    case 0: expval_tiles<C, 1, TWO>(ga, gb, smem, rows, a, t.nterms, anyx, ntiles, acc); break;
    case 1: expval_tiles<C, 2, TWO>(ga, gb, smem, rows, a, t.nterms, anyx, ntiles, acc); break;
    case 2: expval_tiles<C, 4, TWO>(ga, gb, smem, rows, a, t.nterms, anyx, ntiles, acc); break;
    default: expval_tiles<C, 8, TWO>(ga, gb, smem, rows, a, t.nterms, anyx, ntiles, acc); break;
    }
#pragma unroll
    for (int i = 0; i < kMaxTermsPerLaunch; ++i) {
        if (i < t.nterms) {
            NSum v = {acc[i], 0.0};
            const NSum r = block_reduce(v, scratch);
            if (threadIdx.x == 0) {
                partial[((long long)blockIdx.x * t.nterms + i) * 2] = r.s;
                partial[((long long)blockIdx.x * t.nterms + i) * 2 + 1] = r.c;
            }
        }
    }
}

// Whole states below 256 amplitudes: one workgroup, element per thread, straight from
// the definition (the tile is the state).
template <typename C, bool TWO>
__global__ __launch_bounds__(kThreads) void k_expval_small(const C* __restrict__ sa, const C* __restrict__ sb,
                                                           int n, const TermArgs t, double* __restrict__ partial)
{
    __shared__ NSum scratch[kThreads / 64];
    const int N = 1 << n;
    const int e = threadIdx.x;
    for (int i = 0; i < t.nterms; ++i) {
        double val = 0.0;
        if (e < N) {
            const C ap = sa[e ^ t.xloc[i]];
            const C be = TWO ? sb[e] : sa[e];
            const double re = (double)ap.x * (double)be.x + (double)ap.y * (double)be.y;
            const double im = (double)ap.x * (double)be.y - (double)ap.y * (double)be.x;
            const int q = t.ny[i] & 3;
            val = (q == 0) ? re : (q == 1) ? -im : (q == 2) ? -re : im;
            if (__popc(e & t.zloc[i]) & 1) val = -val;
        }
        const NSum r = block_reduce(NSum{val, 0.0}, scratch);
        if (threadIdx.x == 0) {
            partial[(long long)i * 2] = r.s;
            partial[(long long)i * 2 + 1] = r.c;
        }
    }
}

// out = sum_t coeff_t P_t in (accumulate != 0: out += ...), with
// (P in)[k] = i^ny (-1)^popcount((k xor x) & zy) in[k xor x].  Each thread gathers its
// amplitude's partners straight from HBM / L2.
template <typename C>
__global__ __launch_bounds__(kThreads) void k_pauli_apply(const C* __restrict__ in, C* __restrict__ out,
                                                          long long N, const PauliSumArgs p, int accumulate)
{
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x; k < N; k += stride) {
        double re = 0.0, im = 0.0;
        if (accumulate) {
            const C o = out[k];
            re = o.x;
            im = o.y;
        }
        for (int i = 0; i < p.nterms; ++i) {
            const long long j = k ^ p.x[i];
            const C v = in[j];
            double vr = v.x, vi = v.y;
            const int q = p.ny[i] & 3;   // multiply by i^q
            double tr = (q == 0) ? vr : (q == 1) ? -vi : (q == 2) ? -vr : vi;
            double ti = (q == 0) ? vi : (q == 1) ? vr : (q == 2) ? -vi : -vr;
            const double c = (__popcll(j & p.z[i]) & 1) ? -p.coeff[i] : p.coeff[i];
            re = fma(c, tr, re);
            im = fma(c, ti, im);
        }
        C o;
        o.x = re;
        o.y = im;
        out[k] = o;
    }
}

template <typename C, typename R>
__global__ __launch_bounds__(kThreads) void k_probs_full(const C* __restrict__ st, long long N,
                                                         R* __restrict__ out)
{
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += stride) {
        const C v = st[i];
        out[i] = v.x * v.x + v.y * v.y;
    }
}

template <typename C>
__global__ __launch_bounds__(kThreads) void k_probs_marg(const C* __restrict__ st, const MargArgs a,
                                                         double* __restrict__ partial)
{
    const long long M = 1ll << a.m;
    const long long total = M * a.nchunks;
    const long long gid = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (gid >= total) return;
    const long long o = gid % M;
    const long long ch = gid / M;
    long long ob = 0;
    for (int j = 0; j < a.m; ++j) ob |= ((o >> j) & 1) << a.q[j];
    const int nr = a.n - a.m;
    NSum s = {0.0, 0.0};
    for (long long r = ch * a.chunk; r < (ch + 1) * a.chunk; ++r) {
        long long idx = ob;
        for (int j = 0; j < nr; ++j) idx |= ((r >> j) & 1) << a.rest[j];
        const C v = st[idx];
        const double x = v.x, y = v.y;
        nadd(s, x * x + y * y);
    }
    partial[2 * (ch * M + o)] = s.s;
    partial[2 * (ch * M + o) + 1] = s.c;
}

// out[o] = Neumaier sum over chunks of partial[(chunk*M + o)] (pairs), fixed order.
__global__ __launch_bounds__(kThreads) void k_sum_chunks(const double* __restrict__ partial, long long M,
                                                         long long nchunks, double* __restrict__ out)
{
    const long long o = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (o >= M) return;
    NSum s = {0.0, 0.0};
    for (long long c = 0; c < nchunks; ++c) {
        nadd(s, partial[2 * (c * M + o)]);
        s.c += partial[2 * (c * M + o) + 1];
    }
    out[o] = s.s + s.c;
}

// Per-qubit <Z_i> and norm of finished served states, batched: work item = one chunk of
// 2^12 consecutive amplitudes of one state.  Each workgroup writes, for its chunk, the
// chunk's sum of |alpha|^2 and, for the qubits inside the chunk (bits < 12), the sum
// over amplitudes with that bit set; qubits >= 12 are constant over a chunk and are
// resolved on the host from the chunk sum.  Fixed partition and reduction order.
constexpr int kZChunkQubits = 12;

template <typename C>
__global__ __launch_bounds__(kThreads) void k_zsum_batch(const ZItem* __restrict__ items, const int* __restrict__ count,
                                                         double* __restrict__ partial)
{
    __shared__ NSum scratch[kThreads / 64];
    const int nitems = *count;
    if (nitems <= 0) return;
    const long long total = items[nitems - 1].chunk_end;
    for (long long w = blockIdx.x; w < total; w += gridDim.x) {
        int lo = 0, hi = nitems - 1;
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (items[mid].chunk_end <= w) lo = mid + 1;
            else hi = mid;
        }
        const ZItem& it = items[lo];
        const long long chunk = w - (it.chunk_end - it.nchunks);
        const int cq = it.n < kZChunkQubits ? it.n : kZChunkQubits;
        const int len = 1 << cq;
        const C* st = (const C*)it.state + (chunk << cq);
        double tot = 0.0, bits[kZChunkQubits];
#pragma unroll
        for (int b = 0; b < kZChunkQubits; ++b) bits[b] = 0.0;
        for (int e = threadIdx.x; e < len; e += kThreads) {
            const C v = st[e];
            const double p = (double)v.x * v.x + (double)v.y * v.y;
            tot += p;
#pragma unroll
            for (int b = 0; b < kZChunkQubits; ++b)
                if ((e >> b) & 1) bits[b] += p;
        }
        double* out = partial + (it.partial_off + chunk * (kZChunkQubits + 1));
        NSum r = block_reduce(NSum{tot, 0.0}, scratch);
        if (threadIdx.x == 0) out[0] = r.s + r.c;
#pragma unroll
        for (int b = 0; b < kZChunkQubits; ++b) {
            r = block_reduce(NSum{bits[b], 0.0}, scratch);
            if (threadIdx.x == 0) out[1 + b] = r.s + r.c;
        }
    }
}

// ------------------------------------------------------------------ launchers

hipError_t launch_zsum_batch(int dtype, const ZItem* items, const int* count, double* partial, int grid,
                             hipStream_t s)
{
    if (dtype == 0)
        hipLaunchKernelGGL(k_zsum_batch<float2>, dim3(grid), dim3(kThreads), 0, s, items, count, partial);
    else
        hipLaunchKernelGGL(k_zsum_batch<double2>, dim3(grid), dim3(kThreads), 0, s, items, count, partial);
    return hipGetLastError();
}

// One workgroup per tile.
template <typename R>
hipError_t launch_pass_t(void* st, const PassArgs& a, long long ntiles, const DevOp* ops, const void* pool,
                         const int* ipool, const float* apool, hipStream_t s)
{
    using C = typename CT<R>::T;
    static bool attr_set = false;
    if (!attr_set) {
        hipError_t e = hipFuncSetAttribute((const void*)k_pass<C>, hipFuncAttributeMaxDynamicSharedMemorySize, 65536);
        if (e != hipSuccess) return e;
        attr_set = true;
    }
    const size_t lds = (sizeof(C) << a.m) + sizeof(float) * (size_t)a.a_len;
    hipLaunchKernelGGL(k_pass<C>, dim3((unsigned)ntiles), dim3(kThreads), lds, s, (C*)st, a, ops, (const C*)pool,
                       ipool, apool);
    return hipGetLastError();
}

hipError_t launch_batch_pass(int dtype, const BatchItem* items, const int* count, int grid, int tile_qubits,
                             hipStream_t s)
{
    const size_t lds = ((dtype == 0 ? sizeof(float2) : sizeof(double2)) << tile_qubits) +
                       (dtype == 0 ? sizeof(float) * kServeOperandFloats : 0);
    if (dtype == 0) {
        static bool set = false;
        if (!set) {
            hipError_t e = hipFuncSetAttribute((const void*)k_batch_pass<float2>,
                                               hipFuncAttributeMaxDynamicSharedMemorySize, 65536);
            if (e != hipSuccess) return e;
            set = true;
        }
        hipLaunchKernelGGL(k_batch_pass<float2>, dim3(grid), dim3(kThreads), lds, s, items, count);
    } else {
        static bool set = false;
        if (!set) {
            hipError_t e = hipFuncSetAttribute((const void*)k_batch_pass<double2>,
                                               hipFuncAttributeMaxDynamicSharedMemorySize, 65536);
            if (e != hipSuccess) return e;
            set = true;
        }
        hipLaunchKernelGGL(k_batch_pass<double2>, dim3(grid), dim3(kThreads), lds, s, items, count);
    }
    return hipGetLastError();
}

hipError_t launch_pass(int dtype, void* st, const PassArgs& a, long long ntiles, const DevOp* ops,
                       const void* pool, const int* ipool, const float* apool, hipStream_t s)
{
    return dtype == 0 ? launch_pass_t<float>(st, a, ntiles, ops, pool, ipool, apool, s)
                      : launch_pass_t<double>(st, a, ntiles, ops, pool, ipool, apool, s);
}

hipError_t launch_init_zero(int dtype, void* st, long long N, hipStream_t s)
{
    const long long blocks = std::min<long long>((N + kThreads - 1) / kThreads, 8192);
    if (dtype == 0)
        hipLaunchKernelGGL(k_init_zero<float2>, dim3((unsigned)blocks), dim3(kThreads), 0, s, (float2*)st, N);
    else
        hipLaunchKernelGGL(k_init_zero<double2>, dim3((unsigned)blocks), dim3(kThreads), 0, s, (double2*)st, N);
    return hipGetLastError();
}

hipError_t launch_zero(int dtype, void* st, long long N, hipStream_t s)
{
    const long long blocks = std::min<long long>((N + kThreads - 1) / kThreads, 8192);
    if (dtype == 0)
        hipLaunchKernelGGL(k_zero<float2>, dim3((unsigned)blocks), dim3(kThreads), 0, s, (float2*)st, N);
    else
        hipLaunchKernelGGL(k_zero<double2>, dim3((unsigned)blocks), dim3(kThreads), 0, s, (double2*)st, N);
    return hipGetLastError();
}

int norm_grid(long long N)
{
    return (int)std::min<long long>(1024, std::max<long long>(1, N / kThreads));
}

hipError_t launch_norm(int dtype, const void* st, long long N, double* partial, int grid, hipStream_t s)
{
    if (dtype == 0)
        hipLaunchKernelGGL(k_norm<float2>, dim3(grid), dim3(kThreads), 0, s, (const float2*)st, N, partial);
    else
        hipLaunchKernelGGL(k_norm<double2>, dim3(grid), dim3(kThreads), 0, s, (const double2*)st, N, partial);
    return hipGetLastError();
}

hipError_t launch_expval(int dtype, const void* sa, const void* sb, const PassArgs& a, const TermArgs& t,
                         long long ntiles, int grid, double* partial, hipStream_t s)
{
    const bool two = sb != nullptr && sb != sa;
    if (a.m < kLogThreads) {   // the whole state is one small tile (grid must be 1)
        if (dtype == 0) {
            auto k = two ? k_expval_small<float2, true> : k_expval_small<float2, false>;
            hipLaunchKernelGGL(k, dim3(1), dim3(kThreads), 0, s, (const float2*)sa, (const float2*)sb, a.m, t, partial);
        } else {
            auto k = two ? k_expval_small<double2, true> : k_expval_small<double2, false>;
            hipLaunchKernelGGL(k, dim3(1), dim3(kThreads), 0, s, (const double2*)sa, (const double2*)sb, a.m, t,
                               partial);
        }
        return hipGetLastError();
    }
    if (a.m > kExpvalMaxTileQubits) return hipErrorInvalidValue;
    bool anyx = false;
    for (int i = 0; i < t.nterms; ++i) anyx |= t.xloc[i] != 0;
    if (dtype == 0) {
        auto k = two ? k_expval<float2, true> : k_expval<float2, false>;
        hipLaunchKernelGGL(k, dim3(grid), dim3(kThreads), expval_lds_bytes(sizeof(float2), a.m, two, anyx), s,
                           (const float2*)sa, (const float2*)sb, a, t, ntiles, partial);
    } else {
        auto k = two ? k_expval<double2, true> : k_expval<double2, false>;
        hipLaunchKernelGGL(k, dim3(grid), dim3(kThreads), expval_lds_bytes(sizeof(double2), a.m, two, anyx), s,
                           (const double2*)sa, (const double2*)sb, a, t, ntiles, partial);
    }
    return hipGetLastError();
}

hipError_t launch_pauli_apply(int dtype, const void* in, void* out, long long N, const PauliSumArgs& p,
                              int accumulate, hipStream_t s)
{
    const long long blocks = std::min<long long>((N + kThreads - 1) / kThreads, 16384);
    if (dtype == 0)
        hipLaunchKernelGGL(k_pauli_apply<float2>, dim3((unsigned)blocks), dim3(kThreads), 0, s, (const float2*)in,
                           (float2*)out, N, p, accumulate);
    else
        hipLaunchKernelGGL(k_pauli_apply<double2>, dim3((unsigned)blocks), dim3(kThreads), 0, s,
                           (const double2*)in, (double2*)out, N, p, accumulate);
    return hipGetLastError();
}

hipError_t launch_probs_full(int dtype, const void* st, long long N, void* out, hipStream_t s)
{
    const long long blocks = std::min<long long>((N + kThreads - 1) / kThreads, 8192);
    if (dtype == 0)
        hipLaunchKernelGGL((k_probs_full<float2, float>), dim3((unsigned)blocks), dim3(kThreads), 0, s,
                           (const float2*)st, N, (float*)out);
    else
        hipLaunchKernelGGL((k_probs_full<double2, double>), dim3((unsigned)blocks), dim3(kThreads), 0, s,
                           (const double2*)st, N, (double*)out);
    return hipGetLastError();
}

hipError_t launch_probs_marg(int dtype, const void* st, const MargArgs& a, double* partial, double* out,
                             hipStream_t s)
{
    const long long M = 1ll << a.m;
    const long long total = M * a.nchunks;
    const long long blocks = (total + kThreads - 1) / kThreads;
    if (dtype == 0)
        hipLaunchKernelGGL(k_probs_marg<float2>, dim3((unsigned)blocks), dim3(kThreads), 0, s,
                           (const float2*)st, a, partial);
    else
        hipLaunchKernelGGL(k_probs_marg<double2>, dim3((unsigned)blocks), dim3(kThreads), 0, s,
                           (const double2*)st, a, partial);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_sum_chunks, dim3((unsigned)((M + kThreads - 1) / kThreads)), dim3(kThreads), 0, s,
                       (const double*)partial, M, a.nchunks, out);
    return hipGetLastError();
}

}  // namespace qsv
