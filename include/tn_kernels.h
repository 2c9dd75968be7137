/*
 * tn_kernels.h -- direct entry points to the individual device kernels of
 * libtn_gfx950.so, for numerical tests of each kernel in isolation.
 *
 * tn_kernel_gemm: C[i] = op(A[ia[i]]) * op(B[ib[i]]) for i < n_inst, complex,
 *   m = 2^m_log rows, n = 2^n_log columns, k = 2^k_log inner dimension.
 *   A instances are strideA elements apart, stored m x k row-major (transA = 0)
 *   or k x m (transA = 1); B likewise k x n (transB = 0) or n x k (transB = 1).
 *   C instances are m*n elements apart, row-major.  ia/ib are device int32
 *   arrays of n_inst entries, or NULL for "instance i" (identity).
 *   fp64 = 0: complex64 data (FP32 MFMA / FMA kernels); 1: complex128.
 *   tile_hint: -1 = by shape, else an MFMA tile index (FP32 only).
 *   Returns the kernel class used (0 MFMA, 1 small, 2 split-k, 3 tiled) or a
 *   negative TN_E* code.  Asynchronous on `stream`.
 *
 * tn_kernel_permute: dst[i] = src[i] with its r legs reordered, for n_inst
 *   instances of 2^r elements: output bit j (counted from the least
 *   significant) takes input bit perm[j].  fp64 selects complex128 elements.
 *   Device pointers; `perm` is a host array of r ints.  block_elems_log: log2
 *   of the elements one block moves (0 = the library default; at most 12 for
 *   complex64, 11 for complex128).  Synchronizes `stream`.
 *
 * tn_kernel_mfma_group: one grouped matrix-core launch (complex64 data, FP32
 *   MFMA), the kernel batched execution runs for the contraction steps of one
 *   tree level.  Job j: slices s < n_slices with C_s = A_s B_s; the element
 *   (row r, inner p) of slice s of A sits at oa[s] + sum_i bit_i(r) << a_row[i]
 *   + sum_i bit_i(p) << a_k[i] (B likewise with ob, b_k, b_col); C_s is an
 *   m x n row-major block at oc[s].  merge = 1: a tile's columns hold `cnt`
 *   consecutive slices sharing A; 2: its rows hold `cnt` slices sharing B;
 *   0: one slice per tile (origin tm0, tn0).  Jobs and tiles are device
 *   arrays in the tn_mfma_job / tn_mfma_tile layouts; `tile` selects the tile
 *   shape (0..7: 128x64, 64x64, 128x32, 64x32, 32x32, 128x16, 64x16, 32x16).
 *   ksplit = S (a power of two dividing the job's count of 8-term inner chunks,
 *   at most BM x BNC; 1 = no split) splits each tile's inner sum
 *   over S tiles (kpart 0..S-1, same group index `pair`, listed S in a row):
 *   each writes its partial tile, row-major BM x BNC complex64, to
 *   partial + (pair * S + kpart) * BM * BNC (padding elements skipped), and
 *   C is written by tn_kernel_mfma_split_reduce on the same lists afterwards.
 *   Asynchronous on `stream`.  Returns 0 or a negative TN_E* code.
 *
 * tn_kernel_mfma_split_reduce: for every tile group of a split job in the
 *   lists of a preceding tn_kernel_mfma_group launch (same `tile`, jobs and
 *   tiles; enqueue it after that launch on the same stream), adds the S
 *   partial tiles in part order 0, 1, ..., S-1 (with more parts than tile
 *   rows: strided FP64 partial sums combined by a fixed tree; either way the
 *   results are the same run to run) and writes the job's C.  fp64 = 1 for complex128 partials and output
 *   (the library's FP64 tiles), 0 for complex64.  Tiles of unsplit jobs are
 *   skipped.  Asynchronous on `stream`.  Returns 0 or a negative TN_E* code.
 */
typedef struct {
    const void* A;
    const void* B;
    void* C;
    const int64_t* oa;
    const int64_t* ob;
    const int64_t* oc;
    int32_t m_log, n_log, k_log;
    int32_t merge;
    int32_t a_rowfast, b_colfast;  /* lowest stored bit of A is a row bit / of B a column bit */
    int8_t a_row[32], a_k[32], b_k[32], b_col[32];
    int32_t ksplit, pad_;          /* S >= 1: tiles come in groups of S over S parts of the inner index */
    void* partial;                 /* ksplit > 1: S partial tiles per group (device scratch) */
} tn_mfma_job;
typedef struct {
    int32_t job, cnt;
    int64_t s0, tm0, tn0;
    int32_t kpart, pair;           /* ksplit > 1: inner part (0..S-1) and group index */
} tn_mfma_tile;
#ifndef TN_KERNELS_H
#define TN_KERNELS_H
#include <stdint.h>
#ifdef __cplusplus
extern "C" {
#endif
int tn_kernel_gemm(int32_t fp64, const void* A, const void* B, void* C, const int32_t* ia,
                   const int32_t* ib, int64_t strideA, int64_t strideB, int32_t m_log, int32_t n_log,
                   int32_t k_log, int32_t transA, int32_t transB, int64_t n_inst, int32_t tile_hint,
                   void* stream);
int tn_kernel_permute(int32_t fp64, const void* src, void* dst, int64_t n_inst, int32_t r,
                      const int32_t* perm, int32_t block_elems_log, void* stream);
int tn_kernel_mfma_group(int32_t tile, const tn_mfma_job* d_jobs, const tn_mfma_tile* d_tiles,
                         int64_t n_tiles, void* stream);
int tn_kernel_mfma_split_reduce(int32_t tile, int32_t fp64, const tn_mfma_job* d_jobs,
                                const tn_mfma_tile* d_tiles, int64_t n_tiles, void* stream);

/* tn_kernel_group_sums: the level-sum kernel of the estimate (Algorithm 1's
 * sums, Neumaier-compensated in FP64, fixed order: deterministic) over
 * arbitrary ranges.  Group g sums d_x[d_starts[g] .. d_starts[g+1]) and writes
 * (sum, compensation) to d_out[2g], d_out[2g+1] (the sum already includes the
 * compensation).  All pointers are device addresses; d_starts has n_groups + 1
 * entries.  One block per group, asynchronous on `stream`.  Used with the
 * factored term sets of tn_terms_enumerate_factored (their group boundaries
 * from tn_terms_groups) on the X output of tn_exec_outputs.
 * Returns 0 or a negative TN_E* code. */
int tn_kernel_group_sums(const double* d_x, const int64_t* d_starts, int32_t n_groups, double* d_out,
                         void* stream);
#ifdef __cplusplus
}
#endif
#endif
