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
 */
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
#ifdef __cplusplus
}
#endif
#endif
