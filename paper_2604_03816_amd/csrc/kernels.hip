// kernels.hip -- HIP kernels of libqsv for gfx950 (MI355X, CDNA4, wave64).
//
// State layout: 2^n interleaved complex numbers (float2 for complex64, double2 for
// complex128), qubit t = bit t of the index (Eq. 2 / Eq. 3).
//
// Apply pass (k_pass): each workgroup takes tiles in turn.  A tile is 2^m amplitudes whose
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
#include <cstring>
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

// 16-byte register types for bulk moves (native vectors, so that arrays of them stay
// in registers): two complex64 or one complex128 amplitude.
typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef double doublex2 __attribute__((ext_vector_type(2)));
template <typename C> struct Lane16;
template <> struct Lane16<float2> { using T = floatx4; };
template <> struct Lane16<double2> { using T = doublex2; };

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

// PassArgs' arrays are indexed with compile-time indices only (fully unrolled loops
// with a uniform guard): a runtime index into a kernel argument becomes a vector load
// plus a wait on every outstanding memory operation, stores and prefetches included.
__device__ __forceinline__ long long tile_base(const PassArgs& a, long long t)
{
    long long base = 0;
#pragma unroll
    for (int i = 0; i < kMaxRuns; ++i) {
        if (i < a.nruns) {
            base |= (t & ((1ll << a.run_len[i]) - 1)) << a.run_pos[i];
            t >>= a.run_len[i];
        }
    }
    return base;
}

// Offset (relative to the tile base) of the local bits [lo, hi) of local index e.
__device__ __forceinline__ long long local_off_bits(const PassArgs& a, int e, int lo, int hi)
{
    long long o = 0;
#pragma unroll
    for (int i = 0; i < kMaxTileQubits; ++i) {
        if (i >= lo && i < hi && ((e >> i) & 1)) o += 1ll << a.phys[i];
    }
    return o;
}

// LDS position of tile element e.  The tile is stored XOR-swizzled so that the accesses
// of an op on high tile qubits, whose lanes differ in address bits above the bank
// period, spread over all banks: complex64 (8-byte elements) XORs element bits 1-4 with
// bits 4-7 (bit 0 untouched, so the two elements of a 16-byte lane move stay adjacent),
// complex128 (16 bytes) bits 0-3 with bits 3-6.  The map is a bijection on every range
// [0, 2^m) and linear over XOR: for disjoint bit sets a | b = a ^ b, so
// swz(a | b) = swz(a) ^ swz(b), which lets a uniform (scalar) part and a per-lane part be
// swizzled separately and combined with one XOR.
template <typename C>
__device__ __forceinline__ int swz(int e)
{
    if constexpr (sizeof(C) == 8) return e ^ (((e >> 4) & 15) << 1);
    else return e ^ ((e >> 3) & 15);
}

// Move a tile between HBM and LDS.  Every lane moves 16 bytes at a time: W = 1
// complex128 or W = 2 adjacent complex64 amplitudes (local bit 0 is qubit 0, so such a
// pair is contiguous in HBM).  Local index e = W (256 * slice + tid) + w: the bits from
// the thread id give an offset computed once per thread, the bits above from the slice
// number; with the slice count NS a compile-time constant every slice's offset is a sum
// of uniform strides (scalar ALU) and all NS accesses of a thread are issued back to
// back before the first is consumed.
__device__ __forceinline__ long long local_stride(const PassArgs& a, int i)
{
    return 1ll << a.phys[i];   // i is a compile-time constant at every call site
}

template <typename C, bool LOAD, int NS, int W, int NT = kThreads>
__device__ __forceinline__ void move_tile_n(gptr<C> __restrict__ st, C* __restrict__ lds, const PassArgs& a,
                                            long long toff)
{
    constexpr int LOGT = NT == 512 ? 9 : 8;
    static_assert(W == 1 || (W == 2 && sizeof(C) == 8), "16-byte lanes");
    using V = typename std::conditional<W == 2, floatx4, C>::type;
    // the state streams through once per pass: nontemporal loads and stores (measured
    // 2 % faster passes than plain ones); the builtins want native vector types
    using NV = typename std::conditional<sizeof(V) == 16, floatx4, float __attribute__((ext_vector_type(2)))>::type;
    constexpr int LW = W == 2 ? 1 : 0;
    constexpr int LB = NS >= 32 ? 5 : NS >= 16 ? 4 : NS >= 8 ? 3 : NS >= 4 ? 2 : NS >= 2 ? 1 : 0;
    long long hs[LB > 0 ? LB : 1];
#pragma unroll
    for (int b = 0; b < LB; ++b) hs[b] = local_stride(a, LOGT + LW + b);
    const int tid = threadIdx.x;
    // at most CH 16-byte units in registers at a time: wider tiles move in several
    // batches, so the largest tile does not set the kernel's register count
    constexpr int CH = NS < 8 ? NS : 8;
    V v[CH];
    V* l = reinterpret_cast<V*>(lds);
    // 16-byte unit u = NT j + tid holds tile elements W u .. W u + W - 1, stored at the
    // swizzled position of element W u (the swizzle keeps the pair together).  The
    // swizzle reads element bits below 8 only, which come from tid, and leaves the bits
    // from j alone, so the position is NT j + swz(W tid) / W: an immediate offset per j.
    const int ut = swz<C>(W * tid) / W;
    auto unit = [&](int j) { return (j << LOGT) + ut; };
    auto off = [&](int j) {
        long long so = 0;
#pragma unroll
        for (int b = 0; b < LB; ++b)
            if ((j >> b) & 1) so += hs[b];
        return so;
    };
#pragma unroll
    for (int j0 = 0; j0 < NS; j0 += CH) {
        if (LOAD) {
#pragma unroll
            for (int j = 0; j < CH; ++j)
                v[j] = __builtin_bit_cast(V, __builtin_nontemporal_load((const NV*)(st + toff + off(j0 + j))));
#pragma unroll
            for (int j = 0; j < CH; ++j) l[unit(j0 + j)] = v[j];
        } else {
#pragma unroll
            for (int j = 0; j < CH; ++j) v[j] = l[unit(j0 + j)];
#pragma unroll
            for (int j = 0; j < CH; ++j)
                __builtin_nontemporal_store(__builtin_bit_cast(NV, v[j]), (NV*)(st + toff + off(j0 + j)));
        }
    }
}

template <typename C, bool LOAD, int NT = kThreads>
__device__ __forceinline__ void move_tile(gptr<C> __restrict__ st, C* __restrict__ lds, const PassArgs& a,
                                          long long base)
{
    constexpr int LOGT = NT == 512 ? 9 : 8;
    const int tid = threadIdx.x;
    if constexpr (sizeof(C) == 8) {
        // complex64 pairs whenever qubit 0 is a tile qubit and a slice is full
        if (a.L >= 1 && a.m > LOGT) {
            const long long toff = base + local_off_bits(a, tid << 1, 1, LOGT + 1);
            switch (a.m - LOGT - 1) {
            case 0: move_tile_n<C, LOAD, 1, 2, NT>(st, lds, a, toff); break;
            case 1: move_tile_n<C, LOAD, 2, 2, NT>(st, lds, a, toff); break;
            case 2: move_tile_n<C, LOAD, 4, 2, NT>(st, lds, a, toff); break;
            case 3: move_tile_n<C, LOAD, 8, 2, NT>(st, lds, a, toff); break;
            default: move_tile_n<C, LOAD, 16, 2, NT>(st, lds, a, toff); break;
            }
            return;
        }
    }
    const int lowb = a.m < LOGT ? a.m : LOGT;
    const long long toff = base + local_off_bits(a, tid, 0, lowb);
    switch (a.m - LOGT) {
    case 0: move_tile_n<C, LOAD, 1, 1, NT>(st, lds, a, toff); break;
    case 1: move_tile_n<C, LOAD, 2, 1, NT>(st, lds, a, toff); break;
    case 2: move_tile_n<C, LOAD, 4, 1, NT>(st, lds, a, toff); break;
    case 3: move_tile_n<C, LOAD, 8, 1, NT>(st, lds, a, toff); break;
    case 4: move_tile_n<C, LOAD, 16, 1, NT>(st, lds, a, toff); break;
    case 5: move_tile_n<C, LOAD, 32, 1, NT>(st, lds, a, toff); break;
    default:   // tiles smaller than one slice (whole states below NT amplitudes)
        if (tid < (1 << a.m)) {
            if (LOAD) lds[swz<C>(tid)] = st[toff];
            else st[toff] = lds[swz<C>(tid)];
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

// Group g of an op: insert a zero bit at each target position (ascending).  The map is
// linear over XOR, so group_base(g0 + tid) = group_base(g0) ^ group_base(tid) when g0 is
// a multiple of the workgroup size: a per-thread part computed once per op and a
// uniform part per iteration.
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

template <typename C, int K, int NT = kThreads>
__device__ void op_dense(C* __restrict__ lds, int T, const DevOp& op, cptr<C> __restrict__ M)
{
    constexpr int D = 1 << K;
    const int G = T >> K;
    // LDS position of row r of group g0 + tid: swz(group_base(g0)) (uniform, scalar work)
    // ^ swz(group_base(tid)) ^ swz(row_off(r)) (per lane and per op)
    const int bt = swz<C>(group_base<K>(threadIdx.x, op));
    for (int g0 = 0; g0 < G; g0 += NT) {
        if (g0 + (int)threadIdx.x >= G) break;
        const int b = __builtin_amdgcn_readfirstlane(swz<C>(group_base<K>(g0, op))) ^ bt;
        C v[D];
#pragma unroll
        for (int r = 0; r < D; ++r) v[r] = lds[b ^ swz<C>(row_off<K>(r, op))];
        // rows are not unrolled for wide gates: the row's matrix entries are uniform
        // (scalar) loads, the inputs stay in registers
        constexpr int RU = K <= 2 ? D : 1;
#pragma unroll RU
        for (int r = 0; r < D; ++r) {
            C acc;
            acc.x = acc.y = 0;
#pragma unroll
            for (int c = 0; c < D; ++c) cmac(acc, M[r * D + c], v[c]);
            lds[b ^ swz<C>(row_off<K>(r, op))] = acc;
        }
    }
}

// Dense op on matrix cores: FP32 MFMA for complex64, FP64 MFMA for complex128 (the
// 3-qubit ops; 4-qubit ones take op_dense_mfma_3m below).  The op
// is the real-embedded 2D x 2D matrix (D = 2^K) times the tile viewed as D x (T / D)
// complex columns (one column per group of amplitudes that differ only in the op's
// targets).  A wave takes 16 groups at a time: lane (q, col) = (lane / 16, lane % 16)
// feeds group `col`, complex input rows 4 j + q (real part, then imaginary part, as two
// K = 4 steps), and receives output rows 8 rb + 2 q and 8 rb + 2 q + 1 of row block rb
// (A[i][k] sits in lane i + 16 k and B[k][j] in lane j + 16 k in both precisions; the
// output rows' order differs between the FP32 and FP64 instructions, which the planner's
// lanes' choice of A rows absorbs).  The op's complex matrix is staged in LDS once per
// pass, D x D in the state's precision (half the bytes of its real embedding
// [[Re, -Im], [Im, Re]]), each row's entries permuted for the LDS banks; each lane reads
// the complex entries of its A-operand slots
// once per op and keeps the real-embedded values in registers for the whole op.  All
// reads of a block precede its writes, so the update is in place; waves own disjoint
// groups.
typedef double doublex4 __attribute__((ext_vector_type(4)));

template <typename C, int K, int NT = kThreads>
__device__ void op_dense_mfma(C* __restrict__ lds, int T, const DevOp& op, const float* __restrict__ Araw)
{
    using R = typename std::conditional<sizeof(C) == 8, float, double>::type;
    using Acc = typename std::conditional<sizeof(C) == 8, floatx4, doublex4>::type;
    const C* __restrict__ Ac = reinterpret_cast<const C*>(Araw);
    constexpr int D = 1 << K, R2 = 2 * D, RB = R2 / 16, KS = R2 / 4;
    // the wave index is uniform: saying so keeps the block loop's bookkeeping and each
    // block's group base on the scalar unit
    const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6);
    const int q = lane >> 4, col = lane & 15;
    // A slot (rb, ks) of this lane is real-embedded entry (row 16 rb + i, column 4 ks + q),
    // i = lane % 16.  Input column 4 ks + q is the real (ks even) or imaginary (ks odd)
    // part of complex input 4 (ks / 2) + q, the order in which each lane feeds its complex
    // inputs.  Rows are arranged so that output element e of lane 16 q + col is (complex
    // row 8 rb + 2 q + e / 2, real / imaginary e % 2) in both precisions: the FP32
    // instruction returns row i = 4 q + e there, so row i <-> (i / 2, i % 2); the FP64 one
    // returns row i = 4 e + q (measured on gfx950), so row i <-> (2 (i % 4) + i / 8,
    // (i / 4) % 2).  The entry is Re where the row's and column's real / imaginary halves
    // agree (co == ks % 2), else -Im (co = 0) or +Im (co = 1); slots 2 j and 2 j + 1 share
    // one complex entry.
    const int i16 = lane & 15;
    const int ro = sizeof(C) == 8 ? (i16 >> 1) : 2 * (i16 & 3) + (i16 >> 3);
    const bool co = sizeof(C) == 8 ? (i16 & 1) : ((i16 >> 2) & 1);
    // entry (r, c) is staged at r D + (c ^ (r % 8)), so that the eight rows a group of
    // lanes reads in one access fall in different LDS banks
    const C* __restrict__ Al = Ac + ro * D;
    R a[RB][KS];
#pragma unroll
    for (int rb = 0; rb < RB; ++rb)
#pragma unroll
        for (int j = 0; j < KS / 2; ++j) {
            const C u = Al[8 * rb * D + ((4 * j + q) ^ ro)];
            a[rb][2 * j] = co ? u.y : u.x;
            a[rb][2 * j + 1] = co ? u.x : -u.y;
        }
    // this lane's row offsets (the same for every block)
    // (swizzled LDS positions: the lane's group and row parts are folded into rin / rout)
    const int bcol = swz<C>(group_base<K>(col, op));
    int rin[KS / 2], rout[2 * RB];
#pragma unroll
    for (int j = 0; j < KS / 2; ++j) rin[j] = swz<C>(row_off<K>(4 * j + q, op)) ^ bcol;
#pragma unroll
    for (int rb = 0; rb < RB; ++rb) {
        rout[2 * rb] = swz<C>(row_off<K>(8 * rb + 2 * q, op)) ^ bcol;
        rout[2 * rb + 1] = swz<C>(row_off<K>(8 * rb + 2 * q + 1, op)) ^ bcol;
    }
    const int nblk = (T >> K) >> 4;
    // complex64: two blocks per iteration (blocks blk and blk + waves), their LDS reads
    // issued together and their accumulation chains interleaved on the matrix pipe;
    // complex128: one (the FP64 pipe gains nothing from it, and the registers it would
    // take cost occupancy)
    constexpr int NW = NT / 64, U = sizeof(C) == 8 ? 2 : 1;
    for (int blk = wave; blk < nblk; blk += U * NW) {
        int sb[U];
        bool live[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int b = blk + u * NW;
            live[u] = b < nblk;   // uniform
            // the block's part of the group base is uniform (scalar unit); the lane's
            // part was computed once
            sb[u] = __builtin_amdgcn_readfirstlane(swz<C>(group_base<K>((live[u] ? b : blk) << 4, op)));
        }
        C v[U][KS / 2];
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
            for (int j = 0; j < KS / 2; ++j) v[u][j] = lds[sb[u] ^ rin[j]];
        Acc acc[U][RB];
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
            for (int rb = 0; rb < RB; ++rb) acc[u][rb] = Acc{0, 0, 0, 0};
#pragma unroll
        for (int j = 0; j < KS / 2; ++j) {
#pragma unroll
            for (int rb = 0; rb < RB; ++rb) {
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    if constexpr (sizeof(C) == 8) {
                        acc[u][rb] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[rb][2 * j], v[u][j].x, acc[u][rb], 0, 0, 0);
                        acc[u][rb] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[rb][2 * j + 1], v[u][j].y, acc[u][rb], 0, 0, 0);
                    } else {
                        acc[u][rb] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[rb][2 * j], v[u][j].x, acc[u][rb], 0, 0, 0);
                        acc[u][rb] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[rb][2 * j + 1], v[u][j].y, acc[u][rb], 0, 0, 0);
                    }
                }
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if (!live[u]) continue;
#pragma unroll
            for (int rb = 0; rb < RB; ++rb) {
                C o0, o1;
                o0.x = acc[u][rb][0];
                o0.y = acc[u][rb][1];
                o1.x = acc[u][rb][2];
                o1.y = acc[u][rb][3];
                lds[sb[u] ^ rout[2 * rb]] = o0;
                lds[sb[u] ^ rout[2 * rb + 1]] = o1;
            }
        }
    }
}

// 4-qubit dense op on matrix cores with three real products instead of the four of
// the real embedding (Gauss's form of a complex product).  With M = Ar + i Ai and an
// input column x = xr + i xi, t = Ar (xr + xi) gives Re(M x) = t - (Ar + Ai) xi and
// Im(M x) = t + (Ai - Ar) xr: per block of 16 groups three 16 x 16 x 16 real products,
// 12 matrix-core instructions where the real embedding takes 16.  Lane (q, col) =
// (lane / 16, lane % 16) feeds complex input row 4 j + q of group col at step j and
// holds row col of each A operand (A[i][k] sits in lane i + 16 k); output element e is
// complex row 4 q + e (FP32 instruction) or 4 e + q (FP64).  The staged operand is the
// one op_dense_mfma reads (entry (r, c) at 16 r + (c ^ (r % 8))); each lane forms its
// three A values per step from one complex entry.
template <typename C, int NT = kThreads>
__device__ void op_dense_mfma_3m(C* __restrict__ lds, int T, const DevOp& op, const float* __restrict__ Araw)
{
    using R = typename std::conditional<sizeof(C) == 8, float, double>::type;
    using Acc = typename std::conditional<sizeof(C) == 8, floatx4, doublex4>::type;
    constexpr int K = 4, D = 16;
    const C* __restrict__ Ac = reinterpret_cast<const C*>(Araw);
    const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6);
    const int q = lane >> 4, col = lane & 15;
    const C* __restrict__ Al = Ac + col * D;
    R ar[4], an[4], as[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const C u = Al[(4 * j + q) ^ (col & 7)];
        ar[j] = u.x;
        an[j] = -(u.x + u.y);
        as[j] = u.y - u.x;
    }
    const int bcol = swz<C>(group_base<K>(col, op));
    int rin[4], rout[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        rin[j] = swz<C>(row_off<K>(4 * j + q, op)) ^ bcol;
        rout[j] = swz<C>(row_off<K>(sizeof(C) == 8 ? 4 * q + j : 4 * j + q, op)) ^ bcol;
    }
    const int nblk = (T >> K) >> 4;
    // blocks per iteration: one for complex64, two for complex128 (the reverse of
    // op_dense_mfma's choice; each about 1 % faster per pass than the other count)
    constexpr int NW = NT / 64, U = sizeof(C) == 8 ? 1 : 2;
    auto mfma = [](R a, R b, Acc c) {
        if constexpr (sizeof(C) == 8) return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
        else return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    };
    for (int blk = wave; blk < nblk; blk += U * NW) {
        int sb[U];
        bool live[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int b = blk + u * NW;
            live[u] = b < nblk;   // uniform
            sb[u] = __builtin_amdgcn_readfirstlane(swz<C>(group_base<K>((live[u] ? b : blk) << 4, op)));
        }
        C v[U][4];
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
            for (int j = 0; j < 4; ++j) v[u][j] = lds[sb[u] ^ rin[j]];
        Acc t[U], yr[U], yi[U];
#pragma unroll
        for (int u = 0; u < U; ++u) t[u] = Acc{0, 0, 0, 0};
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
            for (int u = 0; u < U; ++u) t[u] = mfma(ar[j], v[u][j].x + v[u][j].y, t[u]);
#pragma unroll
        for (int u = 0; u < U; ++u) yr[u] = yi[u] = t[u];
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
            for (int u = 0; u < U; ++u) {
                yr[u] = mfma(an[j], v[u][j].y, yr[u]);
                yi[u] = mfma(as[j], v[u][j].x, yi[u]);
            }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if (!live[u]) continue;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                C o;
                o.x = yr[u][e];
                o.y = yi[u][e];
                lds[sb[u] ^ rout[e]] = o;
            }
        }
    }
}

template <typename C, int K, int NT = kThreads>
__device__ void op_perm(C* __restrict__ lds, int T, const DevOp& op, cptr<C> __restrict__ ph,
                        cptr<int> __restrict__ src)
{
    constexpr int D = 1 << K;
    const int G = T >> K;
    const bool phased = op.flags != 0;
    const int bt = swz<C>(group_base<K>(threadIdx.x, op));
    for (int g0 = 0; g0 < G; g0 += NT) {
        if (g0 + (int)threadIdx.x >= G) break;
        const int b = __builtin_amdgcn_readfirstlane(swz<C>(group_base<K>(g0, op))) ^ bt;
        C v[D];
#pragma unroll
        for (int r = 0; r < D; ++r) v[r] = lds[b ^ swz<C>(row_off<K>(src[r], op))];
#pragma unroll
        for (int r = 0; r < D; ++r) lds[b ^ swz<C>(row_off<K>(r, op))] = phased ? cmul(ph[r], v[r]) : v[r];
    }
}

// Diagonal op: the table (2^k phases) is read from LDS when the planner staged it there
// (per-lane indices; a global read here would also wait on every outstanding memory
// operation of the pass), else from the plan pool.
template <typename C, typename P, int NT = kThreads>
__device__ __forceinline__ void op_diag(C* __restrict__ lds, int T, const DevOp& op, P Dg, long long base)
{
    // targets outside the tile contribute a per-tile constant part of the table index
    int gfix = 0, lp[kMaxDiagK];
#pragma unroll
    for (int j = 0; j < kMaxDiagK; ++j) {
        lp[j] = (j < op.k) ? op.lpos[j] : -1;
        if (j < op.k && lp[j] < 0) gfix |= (int)((base >> op.gbit[j]) & 1) << j;
    }
    const int st = swz<C>(threadIdx.x);
    for (int e = threadIdx.x; e < T; e += NT) {
        int idx = gfix;
#pragma unroll
        for (int j = 0; j < kMaxDiagK; ++j)
            if (lp[j] >= 0) idx |= ((e >> lp[j]) & 1) << j;
        const int pe = swz<C>(e - (int)threadIdx.x) ^ st;   // e - tid: a multiple of NT
        lds[pe] = cmul(lds[pe], Dg[idx]);
    }
}

// Workgroup barrier for LDS data only: waits for this wave's LDS operations, then for
// every wave of the workgroup.  Unlike __syncthreads it does not wait for outstanding
// global memory operations (between two ops of a pass only LDS data changes hands).
// The memory clobber keeps the compiler from moving LDS accesses across it.
__device__ __forceinline__ void lds_sync()
{
    asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
}

// WIDE = false leaves out the register-heavy paths (VALU dense ops on 4 or 5 targets,
// permutations on 3 or more): the caller launches that variant only for passes without
// such ops, and its lower register count allows more resident workgroups.  NT is the
// workgroup size.  Ends with an LDS barrier after the last op.
template <typename C, bool WIDE = true, int NT = kThreads>
__device__ __forceinline__ void apply_ops(C* __restrict__ lds, int T, cptr<DevOp> __restrict__ ops, int op_begin,
                          int op_count, cptr<C> __restrict__ pool, cptr<int> __restrict__ ipool,
                          const float* __restrict__ alds, long long base)
{
    for (int oi = 0; oi < op_count; ++oi) {
        const DevOp op = ops[op_begin + oi];
        cptr<C> M = pool + op.off;
        if (op.kind == OP_DENSE && op.aoff >= 0) {
            // the planner gives matrix cores 3- and 4-qubit ops only (kMaxMfmaK)
            if (op.k == 3) op_dense_mfma<C, 3, NT>(lds, T, op, alds + op.aoff);
            else if (op.k == 4) op_dense_mfma_3m<C, NT>(lds, T, op, alds + op.aoff);
            lds_sync();
            continue;
        }
        if (op.kind == OP_DENSE) {
            switch (op.k) {
            case 1: op_dense<C, 1, NT>(lds, T, op, M); break;
            case 2: op_dense<C, 2, NT>(lds, T, op, M); break;
            case 3: op_dense<C, 3, NT>(lds, T, op, M); break;
            case 4: if constexpr (WIDE) op_dense<C, 4, NT>(lds, T, op, M); break;
            default: if constexpr (WIDE) op_dense<C, 5, NT>(lds, T, op, M); break;
            }
        } else if (op.kind == OP_PERM) {
            cptr<int> S = ipool + op.ioff;
            switch (op.k) {
            case 1: op_perm<C, 1, NT>(lds, T, op, M, S); break;
            case 2: op_perm<C, 2, NT>(lds, T, op, M, S); break;
            case 3: if constexpr (WIDE) op_perm<C, 3, NT>(lds, T, op, M, S); break;
            case 4: if constexpr (WIDE) op_perm<C, 4, NT>(lds, T, op, M, S); break;
            default: if constexpr (WIDE) op_perm<C, 5, NT>(lds, T, op, M, S); break;
            }
        } else if (op.aoff >= 0) {
            op_diag<C, const C*, NT>(lds, T, op, reinterpret_cast<const C*>(alds + op.aoff), base);
        } else {
            op_diag<C, cptr<C>, NT>(lds, T, op, M, base);
        }
        lds_sync();
    }
}

// The pass's MFMA operand block, global -> LDS (once per workgroup, or per work item in
// batched launches).
template <int NT = kThreads>
__device__ __forceinline__ void stage_operands(float* __restrict__ alds, cptr<float> __restrict__ apool,
                                               const PassArgs& a)
{
    for (int i = threadIdx.x; i < a.a_len; i += NT) alds[i] = apool[a.a_off + i];
}

// One tile of one pass: HBM -> LDS, every op of the pass, LDS -> HBM.
template <typename C, bool WIDE = true, int NT = kThreads>
__device__ __forceinline__ void run_tile(gptr<C> __restrict__ st, C* __restrict__ lds, const PassArgs& a,
                                         long long tile, cptr<DevOp> __restrict__ ops, cptr<C> __restrict__ pool,
                                         cptr<int> __restrict__ ipool, const float* __restrict__ alds,
                                         bool from_zero = false)
{
    const long long base = tile_base(a, tile);
    if (from_zero) {
        // the tile of |0...0> (Eq. 1): built on chip instead of read from HBM (element 0
        // keeps position 0 under the swizzle and every other element is zero)
        for (int e = threadIdx.x; e < (1 << a.m); e += NT) {
            C z;
            z.x = (base == 0 && e == 0) ? 1 : 0;
            z.y = 0;
            lds[e] = z;
        }
    } else {
        move_tile<C, true, NT>(st, lds, a, base);
    }
    __syncthreads();
    apply_ops<C, WIDE, NT>(lds, 1 << a.m, ops, a.op_begin, a.op_count, pool, ipool, alds, base);
    move_tile<C, false, NT>(st, lds, a, base);
}

// WIDE = false: the variant without the register-heavy op paths, for passes free of
// them (fewer registers, so more resident workgroups when LDS allows).
template <typename C, bool WIDE, int NT>
__global__ __launch_bounds__(NT) void k_pass(C* __restrict__ st, C* __restrict__ st2, const PassArgs a,
                                                   long long ntiles, int from_zero,
                                                   const DevOp* __restrict__ ops,
                                                   const C* __restrict__ pool,
                                                   const int* __restrict__ ipool,
                                                   const float* __restrict__ apool)
{
    // st2 != nullptr: the same pass on a second state of the same shape (tiles ntiles ..
    // 2 ntiles - 1 of the work list), e.g. the adjoint's two vectors.  from_zero: the
    // input is |0...0>, whatever the state buffers hold (a circuit's first pass, with the
    // initialisation folded in)
    extern __shared__ __align__(16) unsigned char smem[];
    C* lds = reinterpret_cast<C*>(smem);
    float* alds = reinterpret_cast<float*>(smem + (sizeof(C) << a.m));
    stage_operands<NT>(alds, (cptr<float>)apool, a);
    __syncthreads();
    const long long total = st2 ? 2 * ntiles : ntiles;
    for (long long t = blockIdx.x; t < total; t += gridDim.x) {
        const bool second = t >= ntiles;
        run_tile<C, WIDE, NT>((gptr<C>)(second ? st2 : st), lds, a, second ? t - ntiles : t, (cptr<DevOp>)ops,
                              (cptr<C>)pool, (cptr<int>)ipool, alds, from_zero != 0);
        __syncthreads();
    }
}

// Batched pass for continuous batching: one launch advances many independent states,
// each by its own current pass.  Work item w (a tile of one item's pass) is found by
// binary search over the items' tile prefix sums; the grid is persistent (fixed size,
// strided over the work list) so the launch can be captured once and replayed.
template <typename C, bool WIDE>
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
    int staged = -1;   // item whose operand block LDS holds (consecutive tiles often share one)
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
        if (it.a.a_len > 0 && lo != staged) {
            stage_operands(alds, (cptr<float>)it.apool, it.a);
            __syncthreads();
            staged = lo;
        }
        run_tile<C, WIDE>((gptr<C>)it.state, lds, it.a, tile, (cptr<DevOp>)it.ops, (cptr<C>)it.pool,
                          (cptr<int>)it.ipool, alds);
        __syncthreads();   // the next work item reuses the LDS tile
    }
}

// Fill with 16-byte stores: every chunk is `rest` except chunk 0, which is `first`
// (|0...0> has amplitude 1 at index 0).  The state's byte size is a multiple of 16.
__global__ __launch_bounds__(kThreads) void k_fill16(uint4* __restrict__ st, long long nchunks, uint4 first,
                                                     uint4 rest)
{
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < nchunks; i += stride)
        st[i] = (i == 0) ? first : rest;
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

// Squared norm: 16-byte loads (two complex64 or one complex128 amplitude per chunk),
// eight independent loads in flight per thread; each group of eight |a|^2 (FP64,
// exact for FP32 inputs) is summed pairwise and added to a Neumaier pair.
template <typename R>
__global__ __launch_bounds__(kThreads) void k_norm(const float4* __restrict__ st, long long nchunks,
                                                   double* __restrict__ partial)
{
    __shared__ NSum scratch[kThreads / 64];
    constexpr int U = 8;
    NSum a = {0.0, 0.0};
    const long long stride = (long long)gridDim.x * blockDim.x;
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    auto sq = [](float4 v) -> double {
        if constexpr (sizeof(R) == 4) {
            return ((double)v.x * v.x + (double)v.y * v.y) + ((double)v.z * v.z + (double)v.w * v.w);
        } else {
            const double2 d = *reinterpret_cast<const double2*>(&v);
            return d.x * d.x + d.y * d.y;
        }
    };
    for (; i + (U - 1) * stride < nchunks; i += U * stride) {
        float4 v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) v[u] = st[i + u * stride];
        double p[U];
#pragma unroll
        for (int u = 0; u < U; ++u) p[u] = sq(v[u]);
#pragma unroll
        for (int h = 1; h < U; h <<= 1)
#pragma unroll
            for (int u = 0; u < U; u += 2 * h) p[u] += p[u + h];
        nadd(a, p[0]);
    }
    for (; i < nchunks; i += stride) nadd(a, sq(st[i]));
    const NSum r = block_reduce(a, scratch);
    if (threadIdx.x == 0) {
        partial[2 * blockIdx.x] = r.s;
        partial[2 * blockIdx.x + 1] = r.c;
    }
}

// Pauli matrix elements over tiles: value_t = sum_k Re( i^ny conj(a[k xor x]) b[k] ) *
// (-1)^popcount(k & zy), i.e. Re <a|P_t|b> (ny may carry an extra 3 to give Im instead),
// for terms with X/Y factors (Z-only terms go to k_expval_z; here they take the generic
// per-element path).  Each term's X/Y support lies inside the tile.  A thread owns the
// local elements e = 256 j + tid (j < NS) of every tile and keeps them in registers; the
// partner amplitudes a[e xor x] come from an LDS copy of the tile of a.  FP64 per thread;
// the workgroup partials are combined in a fixed order.
struct TermRow {
    int x, z, q, pad;
    long long g;
    double k[4];   // two-state weights (see TermArgs::kw)
};

template <typename C, int NS, bool TWO>
__device__ __forceinline__ void expval_tiles(gptr<C> __restrict__ sa, gptr<C> __restrict__ sb,
                                             C* __restrict__ tla, const TermRow* __restrict__ rows,
                                             const PassArgs& a, int nterms, long long ntiles,
                                             double (&acc)[kMaxTermsPerLaunch])
{
    constexpr int LB = NS >= 32 ? 5 : NS >= 16 ? 4 : NS >= 8 ? 3 : NS >= 4 ? 2 : NS >= 2 ? 1 : 0;
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
    // real part of i^q w for w = conj(p) e
    auto phase_re = [](const C& p, const C& e, int q) {
        const double pr = (double)p.x * (double)e.x + (double)p.y * (double)e.y;
        const double pi = (double)p.x * (double)e.y - (double)p.y * (double)e.x;
        return (q == 0) ? pr : (q == 1) ? -pi : (q == 2) ? -pr : pi;
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
#pragma unroll
        for (int j = 0; j < NS; ++j) tla[(j << kLogThreads) + tid] = av[j];
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
                const bool gneg = __popcll(base & g) & 1;   // Z bits outside the tile
                double val = 0.0;
                if (!TWO && x != 0) {
                    // <a|P|a> over pairs (e, e ^ x), e with x's lowest bit clear: with
                    // w = conj(a[e ^ x]) a[e] the pair adds s(e) i^q (w + (-1)^{|x & z|}
                    // conj(w)), whose real part is 2 Re(i^q w) when |x & z| is even and
                    // 2 Re(i^(q+1) Im(w)) when it is odd: half the elements, one product
                    const int lb = __ffs(x) - 1;
                    const bool odd = __popc(x & z) & 1;
                    // T / 2 pairs, NP per thread (a 2^8 tile has fewer pairs than threads);
                    // the unrolled loop issues every partner read before the arithmetic
                    constexpr int NP = NS >= 2 ? NS / 2 : 1;
#pragma unroll
                    for (int p = 0; p < NP; ++p) {
                        const int pr = p * kThreads + tid;
                        if (NS == 1 && pr >= (kThreads >> 1)) break;
                        const int e = ((pr >> lb) << (lb + 1)) | (pr & ((1 << lb) - 1));
                        const C ap = tla[e ^ x];
                        const C ae = tla[e];
                        double v;
                        if (!odd) {
                            const double re = (double)ap.x * (double)ae.x + (double)ap.y * (double)ae.y;
                            v = (q == 0) ? re : (q == 2) ? -re : 0.0;
                        } else {
                            const double im = (double)ap.x * (double)ae.y - (double)ap.y * (double)ae.x;
                            v = (q == 1) ? -im : (q == 3) ? im : 0.0;
                        }
                        val += (__popc(e & z) & 1) ? -v : v;
                    }
                    val *= 2.0;
                } else if (!TWO) {
                    // x == 0 (Z-only terms normally go to k_expval_z): per element from LDS
#pragma unroll 1
                    for (int j = 0; j < NS; ++j) {
                        const int e = (j << kLogThreads) | tid;
                        const C ae = tla[e];
                        const double v = phase_re(ae, ae, q);
                        val += (__popc(e & z) & 1) ? -v : v;
                    }
                } else if (TWO) {
                    // per element: the partner from LDS, b[e] from this thread's registers,
                    // the weight by the parity of e's Z/Y bits (the bits outside the tile
                    // swap the two weights for the whole tile)
                    const double k0r = gneg ? rows[i].k[2] : rows[i].k[0], k0i = gneg ? rows[i].k[3] : rows[i].k[1];
                    const double k1r = gneg ? rows[i].k[0] : rows[i].k[2], k1i = gneg ? rows[i].k[1] : rows[i].k[3];
#pragma unroll
                    for (int j = 0; j < NS; ++j) {
                        const int e = (j << kLogThreads) | tid;
                        const C ap = tla[e ^ x];
                        const double wr = (double)ap.x * (double)bv[j].x + (double)ap.y * (double)bv[j].y;
                        const double wi = (double)ap.x * (double)bv[j].y - (double)ap.y * (double)bv[j].x;
                        const bool odd = __popc(e & z) & 1;
                        val += (odd ? k1r : k0r) * wr - (odd ? k1i : k0i) * wi;
                    }
                }
                acc[i] += (!TWO && gneg) ? -val : val;
            }
        }
        __syncthreads();   // the next tile overwrites LDS
    }
}

// LDS bytes of one k_expval workgroup for a tile of 2^m amplitudes: the tile of a.
__host__ __device__ constexpr size_t expval_lds_bytes(size_t elem, int m)
{
    return elem << m;
}

template <typename C, bool TWO>
__global__ __launch_bounds__(kThreads) void k_expval(const C* __restrict__ sa, const C* __restrict__ sb,
                                                     const PassArgs a, const TermArgs t, long long ntiles,
                                                     double* __restrict__ partial)
{
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ NSum scratch[kThreads / 64];
    __shared__ TermRow rows[kMaxTermsPerLaunch];
    if (threadIdx.x < t.nterms) {
        const int i = threadIdx.x;
        rows[i] = TermRow{t.xloc[i], t.zloc[i], t.ny[i] & 3, 0, t.zglob[i], {t.kw[i][0], t.kw[i][1], t.kw[i][2], t.kw[i][3]}};
    }
    __syncthreads();
    double acc[kMaxTermsPerLaunch];
#pragma unroll
    for (int i = 0; i < kMaxTermsPerLaunch; ++i) acc[i] = 0.0;
    gptr<C> ga = (gptr<C>)const_cast<C*>(sa), gb = (gptr<C>)const_cast<C*>(sb);
    C* tla = reinterpret_cast<C*>(smem);
    switch (a.m - kLogThreads) {   // tiles of 2^8 .. 2^11 amplitudes
    case 0: expval_tiles<C, 1, TWO>(ga, gb, tla, rows, a, t.nterms, ntiles, acc); break;
    case 1: expval_tiles<C, 2, TWO>(ga, gb, tla, rows, a, t.nterms, ntiles, acc); break;
    case 2: expval_tiles<C, 4, TWO>(ga, gb, tla, rows, a, t.nterms, ntiles, acc); break;
    default: expval_tiles<C, 8, TWO>(ga, gb, tla, rows, a, t.nterms, ntiles, acc); break;
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

// Z-only terms: <a|P|b> with P = i^q Z^z sums s(k) i^q conj(a_k) b_k.  As in
// expval_tiles, a thread's NS elements of a tile are Walsh-transformed over the slice
// bits, after which a term is one lookup W[zloc >> 8] times signs that are fixed per
// thread (thread-id bits of z, the phase) or per tile (Z bits outside the tile, a
// uniform mask built from the tile number's bits).  Each thread reads back only the
// transform values it wrote, so its LDS slots are private: no barrier, no tile copy.
template <typename C, int NS, bool TWO>
__device__ __forceinline__ void expval_z_tiles(gptr<C> __restrict__ sa, gptr<C> __restrict__ sb,
                                               double* __restrict__ w, const PassArgs& a, const ZTermArgs& t,
                                               long long ntiles, double (&acc)[kMaxTermsPerLaunch])
{
    constexpr int LB = NS >= 8 ? 3 : NS >= 4 ? 2 : NS >= 2 ? 1 : 0;
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
    unsigned tmask = t.neg;   // per-thread signs: the phase and the thread-id bits of z
#pragma unroll
    for (int i = 0; i < kMaxTermsPerLaunch; ++i)
        if (i < t.nterms) tmask ^= (unsigned)(__popc(tid & t.zlo[i]) & 1) << i;
    double* wt = w + tid;     // this thread's slots: wt[j << 8], j < NS (real), NS + j (imaginary)
    for (long long tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        const long long base = tile_base(a, tile);
        unsigned gm = 0;      // per-tile signs: Z bits outside the tile
#pragma unroll
        for (int b = 0; b < kMaxTileIndexBits; ++b)
            if ((tile >> b) & 1) gm ^= t.gcol[b];
        double re[NS], im[NS];
#pragma unroll
        for (int j = 0; j < NS; ++j) {
            const C av = sa[base + tl + soff(j)];
            const C bv = TWO ? sb[base + tl + soff(j)] : av;
            re[j] = (double)av.x * (double)bv.x + (double)av.y * (double)bv.y;
            im[j] = TWO ? (double)av.x * (double)bv.y - (double)av.y * (double)bv.x : 0.0;
        }
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
            wt[j << kLogThreads] = re[j];
            if (TWO) wt[(NS + j) << kLogThreads] = im[j];
        }
        const unsigned sg = gm ^ tmask;
#pragma unroll
        for (int i = 0; i < kMaxTermsPerLaunch; ++i) {
            if (i < t.nterms && (TWO || !((t.zero >> i) & 1))) {
                const double v = wt[t.zoff[i] << kLogThreads];
                acc[i] += ((sg >> i) & 1) ? -v : v;
            }
        }
    }
}

template <typename C, bool TWO>
__global__ __launch_bounds__(kThreads) void k_expval_z(const C* __restrict__ sa, const C* __restrict__ sb,
                                                       const PassArgs a, const ZTermArgs t, long long ntiles,
                                                       double* __restrict__ partial)
{
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ NSum scratch[kThreads / 64];
    double* w = reinterpret_cast<double*>(smem);
    double acc[kMaxTermsPerLaunch];
#pragma unroll
    for (int i = 0; i < kMaxTermsPerLaunch; ++i) acc[i] = 0.0;
    gptr<C> ga = (gptr<C>)const_cast<C*>(sa), gb = (gptr<C>)const_cast<C*>(sb);
    switch (a.m - kLogThreads) {   // tiles of 2^8 .. 2^11 amplitudes
    case 0: expval_z_tiles<C, 1, TWO>(ga, gb, w, a, t, ntiles, acc); break;
    case 1: expval_z_tiles<C, 2, TWO>(ga, gb, w, a, t, ntiles, acc); break;
    case 2: expval_z_tiles<C, 4, TWO>(ga, gb, w, a, t, ntiles, acc); break;
    default: expval_z_tiles<C, 8, TWO>(ga, gb, w, a, t, ntiles, acc); break;
    }
#pragma unroll
    for (int i = 0; i < kMaxTermsPerLaunch; ++i) {
        if (i < t.nterms) {
            const NSum r = block_reduce(NSum{acc[i], 0.0}, scratch);
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
            const bool odd = __popc(e & t.zloc[i]) & 1;
            if (TWO) {   // the two-state weights (TermArgs::kw)
                val = (odd ? t.kw[i][2] : t.kw[i][0]) * re - (odd ? t.kw[i][3] : t.kw[i][1]) * im;
            } else {
                const int q = t.ny[i] & 3;
                val = (q == 0) ? re : (q == 1) ? -im : (q == 2) ? -re : im;
                if (odd) val = -val;
            }
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

// ------------------------------------------------------------------ sampling

// Probability of entry i: |alpha_i|^2 in FP64 (state sources) or a table entry.
template <int SRC>
__device__ __forceinline__ double prob_at(const void* src, long long i)
{
    if constexpr (SRC == 0) {
        const float2 v = reinterpret_cast<const float2*>(src)[i];
        return (double)v.x * v.x + (double)v.y * v.y;
    } else if constexpr (SRC == 1) {
        const double2 v = reinterpret_cast<const double2*>(src)[i];
        return v.x * v.x + v.y * v.y;
    } else {
        return reinterpret_cast<const double*>(src)[i];
    }
}

// Inclusive prefix sums of one chunk (2^cb entries, cb <= 12) into scan[] in LDS, in a
// fixed order: each thread sums its run of E consecutive entries sequentially, the
// thread totals are scanned within each wave (shuffles) and across the four waves.
// Every chunk, in both sampling kernels, goes through this one function, so a chunk's
// total and its last prefix sum are the same number.
template <int SRC>
__device__ void chunk_scan(const void* src, long long chunk, int cb, double* scan, double* wsum)
{
    const int size = 1 << cb;
    const int E = size > kThreads ? size / kThreads : 1;
    const int tid = threadIdx.x;
    const long long base = chunk << cb;
    double run = 0.0;
    const bool mine = tid * E < size;
    if (mine) {
        for (int i = 0; i < E; ++i) {
            run += prob_at<SRC>(src, base + tid * E + i);
            scan[tid * E + i] = run;   // prefix within the thread's run
        }
    }
    // inclusive scan of the thread totals: within the wave, then across waves
    double x = mine ? run : 0.0;
    const int lane = tid & 63, w = tid >> 6;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const double y = __shfl_up(x, d);
        if (lane >= d) x += y;
    }
    if (lane == 63) wsum[w] = x;
    __syncthreads();
    double woff = 0.0;
    for (int i = 0; i < w; ++i) woff += wsum[i];
    const double off = woff + x - (mine ? run : 0.0);   // exclusive offset of this thread
    if (mine) {
        for (int i = 0; i < E; ++i) scan[tid * E + i] += off;
    }
    __syncthreads();
}

template <int SRC>
__global__ __launch_bounds__(kThreads) void k_chunk_totals(const void* __restrict__ src, int cb,
                                                           double* __restrict__ totals)
{
    extern __shared__ __align__(16) unsigned char smem[];
    double* scan = reinterpret_cast<double*>(smem);
    __shared__ double wsum[kThreads / 64];
    chunk_scan<SRC>(src, blockIdx.x, cb, scan, wsum);
    if (threadIdx.x == 0) totals[blockIdx.x] = scan[(1 << cb) - 1];
}

// One workgroup per listed chunk: rebuild the chunk's prefix sums, then every shot of
// the chunk finds the smallest k with residual < scan[k] (binary search).  Residuals
// are clamped into [0, total) first: below zero (rounding) picks the first entry of
// nonzero probability, at or above the total picks the last one.
template <int SRC>
__global__ __launch_bounds__(kThreads) void k_sample_chunks(const void* __restrict__ src, int cb,
                                                            const SampleChunk* __restrict__ list,
                                                            const double* __restrict__ residual,
                                                            long long* __restrict__ outcome)
{
    extern __shared__ __align__(16) unsigned char smem[];
    double* scan = reinterpret_cast<double*>(smem);
    __shared__ double wsum[kThreads / 64];
    const SampleChunk c = list[blockIdx.x];
    chunk_scan<SRC>(src, c.chunk, cb, scan, wsum);
    const int size = 1 << cb;
    const double total = scan[size - 1];
    const double below = nextafter(total, 0.0);
    for (long long i = c.lo + threadIdx.x; i < c.hi; i += kThreads) {
        double r = residual[i];
        r = r < 0.0 ? 0.0 : (r >= total ? below : r);
        int lo = 0, hi = size - 1;   // smallest k with r < scan[k]; scan[size - 1] > r
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (r < scan[mid]) hi = mid;
            else lo = mid + 1;
        }
        outcome[i] = (c.chunk << cb) + lo;
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

// DM: the buffer holds vec(rho) of an a.n-qubit density matrix (index row + 2^n col)
// and the probability of basis state k is the diagonal entry Re rho[k, k].
template <typename C, bool DM>
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
        if (DM) {
            nadd(s, (double)st[idx + (idx << a.n)].x);
        } else {
            const C v = st[idx];
            const double x = v.x, y = v.y;
            nadd(s, x * x + y * y);
        }
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

// Tr(rho P_t) for an n-qubit density matrix held as vec(rho) (index row + 2^n col):
// P|k> = i^ny (-1)^popcount(k & z) |k xor x>, so Tr(rho P) = sum_k rho[k, k xor x] *
// i^ny (-1)^popcount(k & z).  Only 2^n entries per term are read.  One FP64 Neumaier
// pair per workgroup and term, combined on the host in a fixed order.
template <typename C>
__global__ __launch_bounds__(kThreads) void k_dm_pauli(const C* __restrict__ st, int n, const PauliSumArgs p,
                                                       double* __restrict__ partial)
{
    __shared__ NSum scratch[kThreads / 64];
    const long long N = 1ll << n;
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (int t = 0; t < p.nterms; ++t) {
        const long long x = p.x[t], z = p.z[t];
        const int q = p.ny[t] & 3;
        NSum acc = {0.0, 0.0};
        for (long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x; k < N; k += stride) {
            const C v = st[k + ((k ^ x) << n)];
            double val = (q == 0) ? v.x : (q == 1) ? -v.y : (q == 2) ? -v.x : v.y;   // Re(i^q v)
            if (__popcll(k & z) & 1) val = -val;
            nadd(acc, val);
        }
        const NSum r = block_reduce(acc, scratch);
        if (threadIdx.x == 0) {
            partial[((long long)blockIdx.x * p.nterms + t) * 2] = r.s;
            partial[((long long)blockIdx.x * p.nterms + t) * 2 + 1] = r.c;
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

// Compute units of the current device (cached per device).
static int device_cus()
{
    static int cus[64] = {0};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
    if (cus[dev] == 0) {
        int c = 0;
        if (hipDeviceGetAttribute(&c, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || c <= 0) c = 256;
        cus[dev] = c;
    }
    return cus[dev];
}

// Workgroups stride over the tiles (the hardware keeps as many resident as registers and
// LDS allow; a finished workgroup's slot is refilled at once).
#ifndef QSV_PASS_THREADS_C64
#define QSV_PASS_THREADS_C64 256
#endif
#ifndef QSV_PASS_THREADS_C128
#define QSV_PASS_THREADS_C128 256
#endif

template <typename C, bool WIDE, int NT>
hipError_t launch_pass_nt(void* st, void* st2, const PassArgs& a, long long ntiles, const DevOp* ops,
                          const void* pool, const int* ipool, const float* apool, hipStream_t s, bool from_zero)
{
    const long long total = st2 ? 2 * ntiles : ntiles;
    static bool attr_set = false;
    if (!attr_set) {
        // a 64 KiB complex128 tile plus its operand block exceeds the 64 KiB default
        hipError_t e = hipFuncSetAttribute((const void*)k_pass<C, WIDE, NT>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, 163840);
        if (e != hipSuccess) return e;
        attr_set = true;
    }
    const size_t lds = (sizeof(C) << a.m) + sizeof(float) * (size_t)a.a_len;
    // at most 64 workgroups per CU, each striding over tiles: the operand block is staged
    // once per workgroup rather than once per tile (measured on 2^18-tile passes: 6 %
    // faster for complex64, 10 % for complex128 than one workgroup per tile)
    const long long grid = std::min<long long>(total, 64ll * device_cus());
    hipLaunchKernelGGL((k_pass<C, WIDE, NT>), dim3((unsigned)grid), dim3(NT), lds, s, (C*)st, (C*)st2, a, ntiles,
                       from_zero ? 1 : 0, ops, (const C*)pool, ipool, apool);
    return hipGetLastError();
}

template <typename R, bool WIDE>
hipError_t launch_pass_t(void* st, void* st2, const PassArgs& a, long long ntiles, const DevOp* ops,
                         const void* pool, const int* ipool, const float* apool, hipStream_t s, bool from_zero)
{
    using C = typename CT<R>::T;
    // workgroup size: NT threads for full tiles, 256 for tiles smaller than NT amplitudes
    constexpr int NTW = sizeof(C) == 8 ? QSV_PASS_THREADS_C64 : QSV_PASS_THREADS_C128;
    if (NTW != kThreads && a.m >= (NTW == 512 ? 9 : 8) + (sizeof(C) == 8 ? 1 : 0))
        return launch_pass_nt<C, WIDE, NTW>(st, st2, a, ntiles, ops, pool, ipool, apool, s, from_zero);
    return launch_pass_nt<C, WIDE, kThreads>(st, st2, a, ntiles, ops, pool, ipool, apool, s, from_zero);
}

template <typename C, bool WIDE>
static hipError_t launch_batch_pass_t(const BatchItem* items, const int* count, int grid, size_t lds, hipStream_t s)
{
    hipLaunchKernelGGL((k_batch_pass<C, WIDE>), dim3(grid), dim3(kThreads), lds, s, items, count);
    return hipGetLastError();
}

// The batched pass kernels may take more than the default 64 KiB of dynamic LDS; the
// limit is raised once, outside any stream capture (the server's step is captured).
hipError_t prepare_batch_pass()
{
    const void* fns[4] = {(const void*)k_batch_pass<float2, true>, (const void*)k_batch_pass<float2, false>,
                          (const void*)k_batch_pass<double2, true>, (const void*)k_batch_pass<double2, false>};
    for (const void* f : fns) {
        const hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, 98304);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_batch_pass(int dtype, const BatchItem* items, const int* count, int grid, int tile_qubits,
                             hipStream_t s, bool wide)
{
    // tile + the per-pass operand block (MFMA matrices, diagonal tables) of either dtype
    const size_t lds = ((dtype == 0 ? sizeof(float2) : sizeof(double2)) << tile_qubits) +
                       sizeof(float) * kServeOperandFloats;
    if (dtype == 0)
        return wide ? launch_batch_pass_t<float2, true>(items, count, grid, lds, s)
                    : launch_batch_pass_t<float2, false>(items, count, grid, lds, s);
    return wide ? launch_batch_pass_t<double2, true>(items, count, grid, lds, s)
                : launch_batch_pass_t<double2, false>(items, count, grid, lds, s);
}

hipError_t launch_pass(int dtype, void* st, const PassArgs& a, long long ntiles, const DevOp* ops,
                       const void* pool, const int* ipool, const float* apool, hipStream_t s, void* st2,
                       bool from_zero, bool wide)
{
    if (dtype == 0)
        return wide ? launch_pass_t<float, true>(st, st2, a, ntiles, ops, pool, ipool, apool, s, from_zero)
                    : launch_pass_t<float, false>(st, st2, a, ntiles, ops, pool, ipool, apool, s, from_zero);
    return wide ? launch_pass_t<double, true>(st, st2, a, ntiles, ops, pool, ipool, apool, s, from_zero)
                : launch_pass_t<double, false>(st, st2, a, ntiles, ops, pool, ipool, apool, s, from_zero);
}

static hipError_t launch_fill16(void* st, long long bytes, uint4 first, uint4 rest, hipStream_t s)
{
    const long long nchunks = bytes / 16;
    const long long blocks = std::min<long long>((nchunks + kThreads - 1) / kThreads, 8192);
    hipLaunchKernelGGL(k_fill16, dim3((unsigned)blocks), dim3(kThreads), 0, s, (uint4*)st, nchunks, first, rest);
    return hipGetLastError();
}

hipError_t launch_init_zero(int dtype, void* st, long long N, hipStream_t s)
{
    const uint4 zero = make_uint4(0, 0, 0, 0);
    uint4 one = zero;
    if (dtype == 0) {
        const float f = 1.0f;
        memcpy(&one.x, &f, 4);
    } else {
        const double d = 1.0;
        memcpy(&one.x, &d, 8);
    }
    return launch_fill16(st, N * (dtype == 0 ? 8 : 16), one, zero, s);
}

hipError_t launch_zero(int dtype, void* st, long long N, hipStream_t s)
{
    const uint4 zero = make_uint4(0, 0, 0, 0);
    return launch_fill16(st, N * (dtype == 0 ? 8 : 16), zero, zero, s);
}

int norm_grid(long long N)
{
    return (int)std::min<long long>(1024, std::max<long long>(1, N / kThreads));
}

hipError_t launch_norm(int dtype, const void* st, long long N, double* partial, int grid, hipStream_t s)
{
    const long long nchunks = N * (dtype == 0 ? 8 : 16) / 16;
    if (dtype == 0)
        hipLaunchKernelGGL(k_norm<float>, dim3(grid), dim3(kThreads), 0, s, (const float4*)st, nchunks, partial);
    else
        hipLaunchKernelGGL(k_norm<double>, dim3(grid), dim3(kThreads), 0, s, (const float4*)st, nchunks, partial);
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
    if (dtype == 0) {
        auto k = two ? k_expval<float2, true> : k_expval<float2, false>;
        hipLaunchKernelGGL(k, dim3(grid), dim3(kThreads), expval_lds_bytes(sizeof(float2), a.m), s,
                           (const float2*)sa, (const float2*)sb, a, t, ntiles, partial);
    } else {
        auto k = two ? k_expval<double2, true> : k_expval<double2, false>;
        hipLaunchKernelGGL(k, dim3(grid), dim3(kThreads), expval_lds_bytes(sizeof(double2), a.m), s,
                           (const double2*)sa, (const double2*)sb, a, t, ntiles, partial);
    }
    return hipGetLastError();
}

hipError_t launch_expval_z(int dtype, const void* sa, const void* sb, const PassArgs& a, const ZTermArgs& t,
                           long long ntiles, int grid, double* partial, hipStream_t s)
{
    const bool two = sb != nullptr && sb != sa;
    if (a.m < kLogThreads || a.m > kExpvalMaxTileQubits) return hipErrorInvalidValue;
    const size_t lds = ((two ? 2 : 1) * sizeof(double)) << a.m;
    if (dtype == 0) {
        auto k = two ? k_expval_z<float2, true> : k_expval_z<float2, false>;
        hipLaunchKernelGGL(k, dim3(grid), dim3(kThreads), lds, s, (const float2*)sa, (const float2*)sb, a, t, ntiles,
                           partial);
    } else {
        auto k = two ? k_expval_z<double2, true> : k_expval_z<double2, false>;
        hipLaunchKernelGGL(k, dim3(grid), dim3(kThreads), lds, s, (const double2*)sa, (const double2*)sb, a, t,
                           ntiles, partial);
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
                             hipStream_t s, bool density)
{
    const long long M = 1ll << a.m;
    const long long total = M * a.nchunks;
    const long long blocks = (total + kThreads - 1) / kThreads;
    if (dtype == 0) {
        auto k = density ? k_probs_marg<float2, true> : k_probs_marg<float2, false>;
        hipLaunchKernelGGL(k, dim3((unsigned)blocks), dim3(kThreads), 0, s, (const float2*)st, a, partial);
    } else {
        auto k = density ? k_probs_marg<double2, true> : k_probs_marg<double2, false>;
        hipLaunchKernelGGL(k, dim3((unsigned)blocks), dim3(kThreads), 0, s, (const double2*)st, a, partial);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_sum_chunks, dim3((unsigned)((M + kThreads - 1) / kThreads)), dim3(kThreads), 0, s,
                       (const double*)partial, M, a.nchunks, out);
    return hipGetLastError();
}

hipError_t launch_chunk_totals(int src_dtype, const void* src, int chunk_bits, long long nchunks, double* totals,
                               hipStream_t s)
{
    if (chunk_bits > kSampleChunkBits || nchunks <= 0) return hipErrorInvalidValue;
    const size_t lds = sizeof(double) << chunk_bits;
    auto k = src_dtype == 0 ? k_chunk_totals<0> : src_dtype == 1 ? k_chunk_totals<1> : k_chunk_totals<2>;
    hipLaunchKernelGGL(k, dim3((unsigned)nchunks), dim3(kThreads), lds, s, src, chunk_bits, totals);
    return hipGetLastError();
}

hipError_t launch_sample_chunks(int src_dtype, const void* src, int chunk_bits, const SampleChunk* list,
                                long long nlist, const double* residual, long long* outcome, hipStream_t s)
{
    if (chunk_bits > kSampleChunkBits) return hipErrorInvalidValue;
    if (nlist <= 0) return hipSuccess;
    const size_t lds = sizeof(double) << chunk_bits;
    auto k = src_dtype == 0 ? k_sample_chunks<0> : src_dtype == 1 ? k_sample_chunks<1> : k_sample_chunks<2>;
    hipLaunchKernelGGL(k, dim3((unsigned)nlist), dim3(kThreads), lds, s, src, chunk_bits, list, residual, outcome);
    return hipGetLastError();
}

hipError_t launch_dm_pauli(int dtype, const void* st, int n, const PauliSumArgs& p, int grid, double* partial,
                           hipStream_t s)
{
    if (dtype == 0)
        hipLaunchKernelGGL(k_dm_pauli<float2>, dim3(grid), dim3(kThreads), 0, s, (const float2*)st, n, p, partial);
    else
        hipLaunchKernelGGL(k_dm_pauli<double2>, dim3(grid), dim3(kThreads), 0, s, (const double2*)st, n, p, partial);
    return hipGetLastError();
}

}  // namespace qsv
