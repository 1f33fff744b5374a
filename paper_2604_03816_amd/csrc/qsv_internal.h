// qsv_internal.h -- structures shared by the host planner, the C-ABI layer and the
// HIP kernels of libqsv.so.  Not part of the public ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

namespace qsv {

constexpr int kMaxK = 5;            // widest fused gate (dense / permutation)
constexpr int kMaxMfmaK = 4;        // widest dense op the matrix-core path takes
constexpr int kMaxDiagK = 5;        // widest diagonal op
constexpr int kThreads = 256;       // threads per tile workgroup
constexpr int kLogThreads = 8;
constexpr int kMaxTileQubits = 13;  // 2^13 amplitudes: 64 KiB of complex64
constexpr int kMaxQubits = 34;

enum OpKind : int { OP_DENSE = 0, OP_DIAG = 1, OP_PERM = 2 };

// One op applied to a tile held on chip.  Targets are listed in the order of the
// op's local basis bits (ascending physical qubit).
struct DevOp {
    int kind;
    int k;
    int lpos[kMaxK];    // tile-local bit of each target, or -1 (diagonal op, qubit outside the tile)
    int gbit[kMaxK];    // physical qubit of each target
    int off;            // offset into the complex pool: dense 4^k, diagonal 2^k, permutation 2^k phases
    int ioff;           // permutation: offset into the int pool (2^k source rows)
    int flags;          // permutation: 1 when some phase differs from 1
    int aoff;           // float offset inside the pass's operand block in LDS, else -1: a dense
                        // op on matrix cores (its 2^k x 2^k complex matrix in the state's
                        // precision, entries of row r permuted by c ^ (r % 8)) or a diagonal op
                        // (its 2^k phases, bit copies of the pool entries)
};

// Everything a pass kernel needs to place its tile in the state vector.
// Local tile index bit i sits at physical bit phys[i]: bits 0..L-1 are physical bits
// 0..L-1, bits L..m-1 the other tile qubits in ascending order.  The tile number is
// deposited into the remaining (free) physical bits, which form nruns maximal runs
// (run_pos, run_len).  Kept small (bytes); kernels index the arrays only with
// compile-time indices, so every read is a scalar load.
constexpr int kMaxRuns = kMaxTileQubits + 2;
struct PassArgs {
    int m;
    int L;
    int op_begin;
    int op_count;
    int nruns;
    int a_off;          // the pass's MFMA operand block: float offset in the plan's operand array
    int a_len;          // and its length in floats (staged into LDS behind the tile)
    unsigned char phys[kMaxTileQubits];
    unsigned char run_pos[kMaxRuns];
    unsigned char run_len[kMaxRuns];
};

// Work list for the expectation kernel: up to kMaxTermsPerLaunch Pauli strings whose
// X/Y supports all lie inside the tile.
constexpr int kMaxTermsPerLaunch = 32;
// Tile qubits of the Pauli matrix-element kernels (2^11 amplitudes: the tile copy of a
// complex128 state, or the Z kernel's per-thread transform slots, fit 32 KiB of LDS).
constexpr int kExpvalMaxTileQubits = 11;

struct TermArgs {
    int nterms;
    int xloc[kMaxTermsPerLaunch];          // X/Y support as tile-local bit mask
    int zloc[kMaxTermsPerLaunch];          // Z/Y support inside the tile, local bit mask
    long long zglob[kMaxTermsPerLaunch];   // Z/Y support outside the tile, physical mask
    int ny[kMaxTermsPerLaunch];            // number of Y factors (phase i^ny)
    // Two-state kernel only: term i adds Re(k conj(a[e ^ x]) b[e]) per element e, with
    // k = (kw[i][0], kw[i][1]) where e's bits in the Z/Y support have even parity and
    // (kw[i][2], kw[i][3]) where odd.  A Pauli term has k = i^q and -i^q (q = ny, plus 3
    // for the imaginary part); other weights give sums of two Paulis that share x and z.
    double kw[kMaxTermsPerLaunch][4];
};

// Work list of the Z-only expectation kernel (every term's X/Y mask is zero).  The
// host folds each term's phase and global sign into lookups and masks:
//   zoff[i]   slot of the term in a thread's transform array: (q odd ? NS : 0) + (zloc >> 8)
//             (q = ny mod 4; odd q selects the imaginary transform)
//   zlo[i]    the term's Z bits among the thread-id bits (zloc & 255)
//   neg       bit i: the phase i^q is negative (q = 1 or 2)
//   zero      bit i: odd q, i.e. the imaginary transform, identically zero when a == b
//   gcol[b]   bit i: tile-number bit b is a qubit of term i's Z support outside the tile
constexpr int kMaxTileIndexBits = 24;
struct ZTermArgs {
    int nterms;
    unsigned neg;
    unsigned zero;
    int zoff[kMaxTermsPerLaunch];
    int zlo[kMaxTermsPerLaunch];
    unsigned gcol[kMaxTileIndexBits];
};

// A weighted Pauli sum applied to a state (co-state of the adjoint method).
constexpr int kMaxPauliApply = 64;
struct PauliSumArgs {
    int nterms;
    int ny[kMaxPauliApply];
    long long x[kMaxPauliApply];
    long long z[kMaxPauliApply];
    double coeff[kMaxPauliApply];
};

// Marginal probabilities: thread (o, chunk) sums |alpha|^2 over the indices whose
// bits at the measured qubits spell o, for the chunk-th range of the other bits.
struct MargArgs {
    int n, m;
    int q[kMaxQubits];      // measured qubits, output bit j <-> q[j]
    int rest[kMaxQubits];   // the other qubits, ascending
    long long chunk;        // rest-values per thread
    long long nchunks;
};

// One state's current pass inside a batched launch (continuous batching).
constexpr int kMaxBatchItems = 256;
struct BatchItem {
    void* state;
    const DevOp* ops;
    const void* pool;
    const int* ipool;
    const float* apool;
    long long ntiles;     // tiles of this pass
    long long tile_end;   // prefix sum of ntiles over the items up to and including this one
    PassArgs a;
};

// A finished served state whose <Z_i> and norm are reduced in a batched launch.
struct ZItem {
    const void* state;
    int n;
    int pad;
    long long nchunks;      // 2^max(0, n - 12) chunks of 2^min(n, 12) amplitudes
    long long chunk_end;    // prefix sum of nchunks
    long long partial_off;  // first double of this state's partials (13 per chunk)
};

// MFMA operand floats a served complex64 pass may stage in LDS (the batched launch
// reserves this much behind the tile).
constexpr int kServeOperandFloats = 2048;

// Largest tile (log2 amplitudes) a dtype's pass kernel holds in LDS (64 KiB).
__host__ __device__ constexpr int kMaxTileQubitsC(int dt) { return dt == 0 ? 13 : 12; }

// Launchers (kernels.hip).  dtype 0 = complex64, 1 = complex128.
// wide = false: the variant without the register-heavy op paths (every item's pass must
// be free of them: HostPlan::pwide).
// qsv_sample's shot order: order (device, n) = 0..n-1 sorted stably by the uniforms u
// (device, n values in [0, 1)); scratch: device memory of sort_uniforms_scratch(n) bytes.
size_t sort_uniforms_scratch(long long n);
hipError_t sort_uniforms(const double* u, long long n, long long* order, void* scratch, size_t scratch_bytes,
                         hipStream_t s);
hipError_t prepare_batch_pass();   // raises the batched kernels' LDS limit; call before capturing them
hipError_t launch_batch_pass(int dtype, const BatchItem* items, const int* count, int grid, int tile_qubits,
                             hipStream_t s, bool wide);
hipError_t launch_zsum_batch(int dtype, const ZItem* items, const int* count, double* partial, int grid,
                             hipStream_t s);
// st2 != nullptr applies the same pass to a second state of the same shape in the same
// launch; from_zero makes the pass read |0...0> instead of the state buffers; wide = false
// launches the variant without the register-heavy op paths (the pass must be free of
// them: HostPlan::pwide).
hipError_t launch_pass(int dtype, void* st, const PassArgs& a, long long ntiles, const DevOp* ops,
                       const void* pool, const int* ipool, const float* apool, hipStream_t s,
                       void* st2 = nullptr, bool from_zero = false, bool wide = true);
hipError_t launch_init_zero(int dtype, void* st, long long N, hipStream_t s);
hipError_t launch_zero(int dtype, void* st, long long N, hipStream_t s);
int norm_grid(long long N);
hipError_t launch_norm(int dtype, const void* st, long long N, double* partial, int grid, hipStream_t s);
// Z-only terms (a.m >= 8): no LDS tile copy and no barriers; grid as for launch_expval.
hipError_t launch_expval_z(int dtype, const void* sa, const void* sb, const PassArgs& a, const ZTermArgs& t,
                           long long ntiles, int grid, double* partial, hipStream_t s);
hipError_t launch_expval(int dtype, const void* sa, const void* sb, const PassArgs& a, const TermArgs& t,
                         long long ntiles, int grid, double* partial, hipStream_t s);
hipError_t launch_pauli_apply(int dtype, const void* in, void* out, long long N, const PauliSumArgs& p,
                              int accumulate, hipStream_t s);
hipError_t launch_probs_full(int dtype, const void* st, long long N, void* out, hipStream_t s);

// Sampling: the distribution is either |alpha|^2 of a state (src_dtype 0 / 1) or an FP64
// table (src_dtype 2), cut into chunks of 2^chunk_bits entries.  launch_chunk_totals
// writes each chunk's total; launch_sample_chunks resolves the shots of the listed chunks
// (chunk id, shot range [lo, hi) into the sorted residual / outcome arrays).
constexpr int kSampleChunkBits = 12;
struct SampleChunk {
    long long chunk;
    long long lo, hi;
};
hipError_t launch_chunk_totals(int src_dtype, const void* src, int chunk_bits, long long nchunks, double* totals,
                               hipStream_t s);
hipError_t launch_sample_chunks(int src_dtype, const void* src, int chunk_bits, const SampleChunk* list,
                                long long nlist, const double* residual, long long* outcome, hipStream_t s);
// qsv_sample's assignment of the sorted shots to chunks (residual per shot, the runs of
// equal chunks as a SampleChunk list, their number in *nruns, all device memory; scratch
// of sample_assign_scratch(n) bytes) and the final scatter out[order[k]] = got[k].
size_t sample_assign_scratch(long long n);
hipError_t sample_assign(const double* u, const long long* order, long long n, const double* cum, long long c0,
                         long long lastnz, double P, double* residual, SampleChunk* list, long long* nruns,
                         void* scratch, size_t scratch_bytes, hipStream_t s);
hipError_t scatter_outcomes(const long long* order, const long long* got, long long n, long long* out, hipStream_t s);
hipError_t launch_probs_marg(int dtype, const void* st, const MargArgs& a, double* partial, double* out,
                             hipStream_t s, bool density = false);
hipError_t launch_dm_pauli(int dtype, const void* st, int n, const PauliSumArgs& p, int grid, double* partial,
                           hipStream_t s);

}  // namespace qsv
