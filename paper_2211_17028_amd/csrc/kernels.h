// Launch wrappers of the HIP kernels (gfx950).  All sizes are powers of two;
// complex values are interleaved (re, im) pairs.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

#include "tn.h"

namespace tn {

// Operand selection for a gathered batch: instance i of the output reads
// operand instance (mode 0: i, mode 1: 0, mode 2: map[i]).
struct GemmArgs {
    const void* A;
    const void* B;
    void* C;
    const int32_t* ia;
    const int32_t* ib;
    int ia_mode, ib_mode;
    int64_t strideA, strideB;     // elements between operand instances
    int m_log, n_log, k_log;
    int transA, transB;           // A stored k x m / B stored n x k
    int64_t n_inst;
    // Gathered operands (MFMA kernels, ids >= K_GATHER_BASE): slice i of A
    // starts at element oa[i] of A and its element (row r, inner index p) sits
    // at oa[i] + sum_j bit_j(r) << a_row[j] + sum_j bit_j(p) << a_k[j]; slice i
    // of B element (p, column c) at ob[i] + sum_j bit_j(p) << b_k[j] +
    // sum_j bit_j(c) << b_col[j].  a_rowfast / b_colfast: the operand's lowest
    // stored bit is row / column bit 0 (else it is inner bit 0), which decides
    // the load order that keeps the loads coalesced.
    const int64_t* oa;
    const int64_t* ob;
    int8_t a_row[32], a_k[32], b_k[32], b_col[32];
    int a_rowfast, b_colfast;
};

// Bit permutation of each instance of a 2^r tensor: out bit j <- in bit p[j].
struct PermArgs {
    const void* src;
    void* dst;
    int64_t n_inst;
    int r;                         // rank
    int tb;                        // tile bits
    const int32_t* table;          // 3 * 2^tb: load in-offset, load lds pos, store out-offset
    int n_high;                    // r - tb
    int high_out[32];              // out bit positions of the high (block) bits
    int high_in[32];               // matching in bit positions
    int elems_log;                 // log2 elements moved per block (0 = default: 32 KB of data)
    int pair;                      // 1: the lowest input and output bits are tile bits 0 and
                                   //    the tile has >= 2 of each, so slots 2i, 2i+1 are adjacent
};

// One contraction of a grouped launch: C[i][r][c] = sum_p A_i[r][p] B_i[p][c]
// for every slice i < n_inst, operands addressed in their stored order as in
// GemmArgs' gathered form (slice offsets oa / ob, per-bit stored positions).
// C is written row-major per slice.  Jobs of one launch are independent (one
// level of the contraction trees) and sorted by block0.
struct GettJob {
    const void* A;
    const void* B;
    void* C;
    const int64_t* oa;
    const int64_t* ob;
    int64_t n_inst;
    int64_t block0;                // first block of this job in the launch
    int32_t m_log, n_log, k_log;
    int32_t split;                 // 1: one block per output element (long inner sums)
    int32_t rpt_log;               // split == 0: each thread computes 2^rpt_log rows of one column
    int32_t pad_;
    int8_t a_row[32], a_k[32], b_k[32], b_col[32];
};
// Events for the next grouped launch issued on this thread (gett, matrix-core
// and FP64 tile groups, split reductions): recorded at the kernel's start and
// end by the dispatch (timing of the kernel alone).
void set_launch_events(hipEvent_t start, hipEvent_t stop);
// blocks one job takes in a grouped launch
int64_t gett_job_blocks(const GettJob& j);
// One launch for all jobs of a level: block b runs job d_block_job[b] & 0x7fffffff
// (records in device memory), in FP64 when bit 31 is set, else in FP32.
void launch_gett_group(const GettJob* d_jobs, const int32_t* d_block_job, int64_t blocks, hipStream_t s);

// Grouped FP32 matrix-core contractions.  A job is one step: slices
// i < n_inst with C_i = A_i B_i, operands in stored order (per-bit positions as
// in GettJob), slice i reading A at oa[i], B at ob[i] and writing its row-major
// m x n block at oc[i] (elements).  merge = 1: a tile's columns hold `cnt`
// consecutive slices that share A (n < tile width); merge = 2: its rows hold
// `cnt` consecutive slices that share B (m < tile height); 0: one slice per
// tile.  Rows / columns past the shape or past cnt slices are padding.
struct MfmaJob {
    const void* A;
    const void* B;
    void* C;
    const int64_t* oa;
    const int64_t* ob;
    const int64_t* oc;
    int32_t m_log, n_log, k_log;
    int32_t merge;
    int32_t a_rowfast, b_colfast;  // lowest stored bit of A is a row bit / of B a column bit
    int8_t a_row[32], a_k[32], b_k[32], b_col[32];
    // Split inner sums (ksplit = S, a power of two, 1 = none): tile group p
    // runs S equal parts of the inner index in S blocks; each writes its
    // partial tile, row-major [BM][BN] complex, to partial[p][part]; the
    // split-reduce launch that follows adds the S partials in part order
    // 0, 1, ..., S-1 and writes C (no block waits on another).
    int32_t ksplit, pad_;
    void* partial;
};
struct MfmaTile {                  // one block of a grouped launch
    int32_t job, cnt;
    int64_t s0;                    // first slice
    int64_t tm0, tn0;              // tile origin inside the slice (unmerged dimensions)
    int32_t kpart, pair;           // ksplit > 1: inner part and tile-group index
};
// tile: an MFMA tile id (0..K_MFMA_TILES-1); one launch per tile shape.
void launch_mfma_group(int tile, const MfmaJob* d_jobs, const MfmaTile* d_tiles, int64_t n_tiles,
                       hipStream_t s);
// FP64 (complex128) on the same descriptors: 64 x 64 tiles (tile id 1's shape)
// or 32 x 32 (tile id 4's shape).
void launch_tile64_group(int tile, const MfmaJob* d_jobs, const MfmaTile* d_tiles, int64_t n_tiles,
                         hipStream_t s);
// After a grouped tile launch with split jobs (same job and tile lists, same
// stream): adds each group's partial tiles in part order and writes C.
void launch_split_reduce(int fp64, int tile, const MfmaJob* d_jobs, const MfmaTile* d_tiles, int64_t n_tiles,
                         hipStream_t s);
int mfma_tile_bm(int tile);
int mfma_tile_bn(int tile);

enum KernelClass { KC_MFMA = 0, KC_SMALL = 1, KC_SPLITK = 2, KC_TILED = 3, KC_GROUP = 4 };

// Kernel ids: 0..K_MFMA_TILES-1 = FP32 MFMA GEMM tile configurations,
// then the other variants.  The choice is a pure function of the shape (and
// of the tile hint for MFMA), so it is fixed when a schedule is prepared.
enum KernelId {
    K_MFMA_TILES = 8,
    K_SMALL32 = 10, K_SPLITK32 = 11,
    K_SMALL64 = 20, K_SPLITK64 = 21, K_TILED64 = 22,
    K_PERM32 = 30, K_PERM64 = 31,
    K_GROUP32 = 40, K_GROUP64 = 41, K_TILE64_GROUP = 42, K_SPLIT_REDUCE32 = 43, K_SPLIT_REDUCE64 = 44,
    K_GROUPMIX = 45,
    K_MFMA_GROUP_BASE = 200,   // + MFMA tile id: grouped matrix-core launch
    K_GATHER_BASE = 100,   // + MFMA tile id: the gathered-operand variant
};
int select_gemm(const GemmArgs& g, int fp64, int tile_hint);
bool mfma_tile_fits(int tile, const GemmArgs& g);
void launch_gemm_id(int id, const GemmArgs& g, hipStream_t s);
const char* kernel_name(int id);
int kernel_class(int id);

// FP32 / FP64 complex GEMM dispatch by shape; returns the kernel id.
int launch_gemm_c64(const GemmArgs& g, hipStream_t s, int tile_hint);
int launch_gemm_c128(const GemmArgs& g, hipStream_t s);

void launch_permute_c64(const PermArgs& p, hipStream_t s);
void launch_permute_c128(const PermArgs& p, hipStream_t s);

// per-term finalize: amp_t = scalar * prod_c root_c[idx[t][c]] (FP64),
// X_t = w_t |amp_t|^2; the term `zero_term` (if >= 0) takes its cluster
// values from the FP64 roots instead.
struct FinalizeArgs {
    int64_t n_terms;               // all terms of the plan (enumeration order)
    const int32_t* live_index;     // n_terms: live index or -1 (zero weight / pruned)
    const int32_t* root_idx;       // n_live * n_clusters
    int n_clusters;
    const int64_t* root_ptrs;      // n_clusters device addresses of complex64 roots
    const int64_t* root64_ptrs;    // n_clusters device addresses of complex128 roots (or 0)
    int64_t zero_term;             // term index using root64 (-1 = none)
    double scalar_re, scalar_im;
    const double* w;               // n_terms scaled weights
    double* x_out;                 // n_terms
    float* amp_out;                // 2 * n_terms
    double* x0_fp32_out;           // X of the zero term from the FP32 roots (diagnostic) or null
    int32_t re_value;              // 1: X = w Re(a) (doubled network), 0: X = w |a|^2
    int32_t pad_;
};

// The tail of all packed circuits (finalize of every term and the level sums)
// in two launches: per-block level partials of 256 terms each, then one
// block per (circuit, level) adding them in block order.
struct TailJob {
    FinalizeArgs f;
    const int64_t* starts;         // n_levels + 1 level starts
    double* sums;                  // n_levels (sum, comp) pairs
    int64_t block0;                // first block of this circuit in the term launch
    int32_t n_levels, pad_;
};
// d_part: blocks x (TN_MAX_LEVEL + 1) (sum, comp) pairs of scratch; the level
// sums and the FP32 diagnostic value go res_shift bytes past the addresses in
// the jobs (a results slot of a submitted estimate)
void launch_tail(const TailJob* d_jobs, int n_jobs, int64_t blocks, int max_levels, double* d_part,
                 int64_t res_shift, hipStream_t s);

// Neumaier level sums over contiguous ranges [start[u], start[u+1]).
void launch_level_sum(const double* x, const int64_t* starts, int n_levels, double* out_sum_comp,
                      hipStream_t s);

// PLAIN mode: fill the single-instance slot buffers of term t.
struct SlotFillArgs {
    int n;                         // number of slot leaves
    const int32_t* noise;          // noise index per slot leaf
    const int64_t* dst;            // device address of the 4-element buffer
    const float* bank;             // N * 4 * 8 floats: K_hat_i, complex64
    const int8_t* pattern;         // device patterns, n_terms * N
    int n_noise;
    int64_t term;
};
void launch_slot_fill(const SlotFillArgs& a, hipStream_t s);

void launch_copy_c64(const void* src, void* dst, int64_t n, hipStream_t s);

}  // namespace tn
