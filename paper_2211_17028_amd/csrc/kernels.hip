// HIP kernels for gfx950 (CDNA4, wave64).
//
// The contraction of one term network is a fixed sequence of pairwise
// contractions; each step here is a bit permutation of the operand legs
// (TTGT transpose) followed by a complex GEMM batched over the term
// instances that step serves.  Complex values are interleaved (re, im).

#include <hip/hip_runtime.h>
#include <hip/hip_ext.h>

#include <algorithm>
#include <type_traits>
#include <cstdint>

#include "kernels.h"

namespace tn {

// Events of the next grouped launch on this thread (set by the executor when
// it times launches): they are recorded by the dispatch itself at the
// kernel's start and end, so the interval is the kernel's execution only.
static thread_local hipEvent_t g_ev_start = nullptr, g_ev_stop = nullptr;

void set_launch_events(hipEvent_t start, hipEvent_t stop) {
    g_ev_start = start;
    g_ev_stop = stop;
}

template <typename... Args, typename F>
static void launch_k(F kernel, dim3 grid, dim3 block, hipStream_t s, Args... args) {
    if (g_ev_start || g_ev_stop) {
        hipEvent_t a = g_ev_start, b = g_ev_stop;
        g_ev_start = g_ev_stop = nullptr;
        hipExtLaunchKernelGGL(kernel, grid, block, 0, s, a, b, 0, args...);
    } else {
        hipLaunchKernelGGL(kernel, grid, block, 0, s, args...);
    }
}


typedef float v16f __attribute__((ext_vector_type(16)));
typedef double v4d __attribute__((ext_vector_type(4)));

__device__ __forceinline__ int64_t pick(int mode, const int32_t* map, int64_t i) {
    return mode == 0 ? i : (mode == 1 ? 0 : (int64_t)map[i]);
}

// ---------------------------------------------------------------------------
// K1: FP32 complex GEMM on MFMA.
//
// The complex product C = A B (m x k times k x n) is the real product
// C_r = A_r B_e of the interleaved real view A_r (m x 2k) with the embedding
// B_e (2k x 2n), B_e[2p+s][2j+t] = [[Re, Im], [-Im, Re]][s][t] of B[p][j]; the
// output comes out interleaved.  Each v_mfma_f32_32x32x2f32 covers one complex
// k index, 32 rows and 16 complex columns: 8 m n k real flops per complex MAC,
// as in the four-real-product form.  Block tile BM x BNC complex, k staged
// through LDS in chunks of 8 (planar re/im for A so that a half-wave reads
// consecutive words).
// ---------------------------------------------------------------------------
template <int BM, int BNC>
__global__ __launch_bounds__(64 * (BM >= 64 ? BM / 64 : 1) * (BNC >= 32 ? BNC / 32 : 1))
void k_gemm_mfma(GemmArgs g) {
    constexpr int WM = BM >= 64 ? BM / 64 : 1;
    constexpr int WN = BNC >= 32 ? BNC / 32 : 1;
    constexpr int NT = 64 * WM * WN;
    constexpr int TM = BM / WM / 32;
    constexpr int TN = BNC / WN / 16;
    constexpr int BKC = 8;
    constexpr int AE = (BM * BKC + NT - 1) / NT;     // A elements per thread per chunk
    constexpr int BE = (BKC * BNC + NT - 1) / NT;    // B elements per thread per chunk
    // double-buffered LDS: A planar (re, im) [k][row], B interleaved [k][col];
    // rows padded by one element so that threads staging consecutive k of the
    // same row (or column) land in different banks
    __shared__ float As_re[2][BKC][BM + 1];
    __shared__ float As_im[2][BKC][BM + 1];
    __shared__ float2 Bs[2][BKC][BNC + 1];

    const int m_log = g.m_log, n_log = g.n_log, k_log = g.k_log;
    const int64_t m = int64_t(1) << m_log, n = int64_t(1) << n_log, k = int64_t(1) << k_log;
    // n < BNC happens only for the 16-column tiles: the tile is padded with
    // zero columns that are never stored
    const int tn_log = n_log >= __builtin_ctz(BNC) ? n_log - __builtin_ctz(BNC) : 0;
    const int64_t tiles = (m / BM) << tn_log;
    const int64_t blk = blockIdx.x;
    const int64_t inst = blk / tiles;
    const int64_t tile = blk - inst * tiles;
    const int64_t tm0 = (tile >> tn_log) * BM;
    const int64_t tn0 = (tile & ((int64_t(1) << tn_log) - 1)) * BNC;
    const float2* __restrict__ A = (const float2*)g.A + pick(g.ia_mode, g.ia, inst) * g.strideA;
    const float2* __restrict__ B = (const float2*)g.B + pick(g.ib_mode, g.ib, inst) * g.strideB;
    float* __restrict__ C = (float*)g.C + inst * (2 * m * n);

    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int wm = wave % WM, wn = wave / WM;
    v16f acc[TM][TN];
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j)
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.0f;

    const int kc = k < BKC ? (int)k : BKC;
    const int kc_log = k_log < 3 ? k_log : 3;
    const int half = lane >> 5;             // 0: real slice, 1: imaginary slice
    const int sub = lane & 31;
    float2 ra[AE], rb[BE];
    // global -> registers for the chunk starting at k0
    auto load = [&](int64_t k0) {
#pragma unroll
        for (int q = 0; q < AE; ++q) {
            const int e = threadIdx.x + q * NT;
            float2 v = make_float2(0.0f, 0.0f);
            if (e < BM * kc) {
                if (!g.transA) {
                    const int r = e >> kc_log, p = e & (kc - 1);
                    v = A[(tm0 + r) * k + k0 + p];
                } else {
                    const int p = e / BM, r = e % BM;
                    v = A[(k0 + p) * m + tm0 + r];
                }
            }
            ra[q] = v;
        }
#pragma unroll
        for (int q = 0; q < BE; ++q) {
            const int e = threadIdx.x + q * NT;
            float2 v = make_float2(0.0f, 0.0f);
            if (e < kc * BNC) {
                int p, c;
                if (!g.transB) {
                    p = e / BNC;
                    c = e % BNC;
                } else {
                    c = e >> kc_log;
                    p = e & (kc - 1);
                }
                if (tn0 + c < n) v = g.transB ? B[(tn0 + c) * k + k0 + p] : B[(k0 + p) * n + tn0 + c];
            }
            rb[q] = v;
        }
    };
    // registers -> LDS buffer `buf`
    auto stash = [&](int buf) {
#pragma unroll
        for (int q = 0; q < AE; ++q) {
            const int e = threadIdx.x + q * NT;
            if (e < BM * kc) {
                int r, p;
                if (!g.transA) {
                    r = e >> kc_log;
                    p = e & (kc - 1);
                } else {
                    p = e / BM;
                    r = e % BM;
                }
                As_re[buf][p][r] = ra[q].x;
                As_im[buf][p][r] = ra[q].y;
            }
        }
#pragma unroll
        for (int q = 0; q < BE; ++q) {
            const int e = threadIdx.x + q * NT;
            if (e < kc * BNC) {
                int p, c;
                if (!g.transB) {
                    p = e / BNC;
                    c = e % BNC;
                } else {
                    c = e >> kc_log;
                    p = e & (kc - 1);
                }
                Bs[buf][p][c] = rb[q];
            }
        }
    };
    const int64_t nchunks = k / kc;
    load(0);
    stash(0);
    __syncthreads();
    for (int64_t ch = 0; ch < nchunks; ++ch) {
        const int buf = (int)(ch & 1);
        if (ch + 1 < nchunks) load((ch + 1) * kc);     // in flight during the MFMAs below
        for (int p = 0; p < kc; ++p) {
            float a[TM], b[TN];
#pragma unroll
            for (int i = 0; i < TM; ++i) {
                const int row = wm * (TM * 32) + i * 32 + sub;
                a[i] = half ? As_im[buf][p][row] : As_re[buf][p][row];
            }
#pragma unroll
            for (int j = 0; j < TN; ++j) {
                const int col = wn * (TN * 16) + j * 16 + (sub >> 1);
                const float2 bv = Bs[buf][p][col];
                const int t = sub & 1;
                b[j] = half == 0 ? (t == 0 ? bv.x : bv.y) : (t == 0 ? -bv.y : bv.x);
            }
#pragma unroll
            for (int i = 0; i < TM; ++i)
#pragma unroll
                for (int j = 0; j < TN; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[i], b[j], acc[i][j], 0, 0, 0);
        }
        if (ch + 1 < nchunks) stash(buf ^ 1);
        __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j) {
            const int64_t colf = 2 * (tn0 + wn * (TN * 16) + j * 16) + sub;
            if (colf >= 2 * n) continue;
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int64_t row = tm0 + wm * (TM * 32) + i * 32 + 8 * (r >> 2) + 4 * half + (r & 3);
                C[row * (2 * n) + colf] = acc[i][j][r];
            }
        }
}

// ---------------------------------------------------------------------------
// K1 with gathered operands: the same MFMA tiling, but A and B are read in
// their stored leg order (no transpose pass).  Offsets of the low row /
// column / inner bits come from small LDS tables; the high parts are added
// once per tile and per k chunk.
// ---------------------------------------------------------------------------
// Device-memory (global address space) views of pointers read from job
// descriptors: generic pointers would compile to flat loads, which count on
// the LDS wait counter as well, so every LDS wait would also wait for the
// global prefetch in flight.
#define TN_GLOBAL __attribute__((address_space(1)))
template <typename T>
__device__ __forceinline__ const TN_GLOBAL T* gload(const void* p) {
    return (const TN_GLOBAL T*)p;
}
template <typename T>
__device__ __forceinline__ TN_GLOBAL T* gstore(void* p) {
    return (TN_GLOBAL T*)p;
}
// element loads from global views (HIP's vector types do not copy across
// address spaces): one 8-byte load for complex64, two for complex128
__device__ __forceinline__ float2 gld(const TN_GLOBAL float2* p) {
    const uint64_t u = *(const TN_GLOBAL uint64_t*)p;
    float2 r;
    __builtin_memcpy(&r, &u, 8);
    return r;
}
__device__ __forceinline__ double2 gld(const TN_GLOBAL double2* p) {
    const TN_GLOBAL double* q = (const TN_GLOBAL double*)p;
    return make_double2(q[0], q[1]);
}
__device__ __forceinline__ void gst(TN_GLOBAL float2* p, float2 v) {
    uint64_t u;
    __builtin_memcpy(&u, &v, 8);
    *(TN_GLOBAL uint64_t*)p = u;
}
__device__ __forceinline__ void gst(TN_GLOBAL double2* p, double2 v) {
    TN_GLOBAL double* q = (TN_GLOBAL double*)p;
    q[0] = v.x;
    q[1] = v.y;
}

__device__ __forceinline__ int64_t deposit(int64_t x, const int8_t* pos, int lo, int hi) {
    // the positions are the same for every lane (a job record's legs): read
    // as eight words into scalar registers, then applied without per-lane
    // branches in a loop that stops at hi
    const uint32_t* pw = reinterpret_cast<const uint32_t*>(pos);
    uint32_t w[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) w[q] = __builtin_amdgcn_readfirstlane(pw[q]);
    int64_t o = 0;
#pragma unroll
    for (int j = 0; j < 32; ++j) {
        if (j >= hi) break;
        if (j >= lo) o |= (int64_t)((x >> j) & 1) << (int)((w[j >> 2] >> (8 * (j & 3))) & 63u);
    }
    return o;
}

// Offset steps of a chunk counter: with chunk index h (inner index h << lo),
// deposit(h + 1) = deposit(h) + step[ctz(~h)], where step[t] is the offset of
// inner bit lo + t minus the offsets of the bits below it, lo <= bit < lo + t.
// Filled by the first threads of a block; t < 32.
__device__ __forceinline__ void chunk_steps(const int8_t* pos, int lo, int hi, int64_t* step) {
    for (int t = threadIdx.x; t < hi - lo; t += blockDim.x) {
        int64_t below = 0;
        for (int j = 0; j < t; ++j) below += int64_t(1) << pos[lo + j];
        step[t] = (int64_t(1) << pos[lo + t]) - below;
    }
}

// Output offset (element index into C) of row i / column j of a grouped tile,
// -1 for padding: merge 2 stacks `cnt` slices along the rows, merge 1 along
// the columns, merge 0 holds one slice at origin (tm0, tn0).  Shared by the
// tile kernels and the split-sum reduction, so both address the same outputs.
__device__ __forceinline__ int64_t tile_out_row(const MfmaJob& J, const MfmaTile& T, int i) {
    const int m_log = J.m_log;
    const int64_t m = int64_t(1) << m_log, n = int64_t(1) << J.n_log;
    if (J.merge == 2) {
        const int seg = i >> m_log;
        return seg < T.cnt ? gload<int64_t>(J.oc)[T.s0 + seg] + (i & (m - 1)) * n : -1;
    }
    const int64_t r = T.tm0 + i;
    return r < m ? (J.merge == 1 ? 0 : gload<int64_t>(J.oc)[T.s0]) + r * n : -1;
}
__device__ __forceinline__ int64_t tile_out_col(const MfmaJob& J, const MfmaTile& T, int j) {
    const int n_log = J.n_log;
    const int64_t n = int64_t(1) << n_log;
    if (J.merge == 1) {
        const int seg = j >> n_log;
        return seg < T.cnt ? gload<int64_t>(J.oc)[T.s0 + seg] + (j & (n - 1)) : -1;
    }
    const int64_t c = T.tn0 + j;
    return c < n ? c : -1;
}

template <int BM, int BNC>
__global__ __launch_bounds__(64 * (BM >= 64 ? BM / 64 : 1) * (BNC >= 32 ? BNC / 32 : 1))
void k_gemm_mfma_g(GemmArgs g) {
    constexpr int WM = BM >= 64 ? BM / 64 : 1;
    constexpr int WN = BNC >= 32 ? BNC / 32 : 1;
    constexpr int NT = 64 * WM * WN;
    constexpr int TM = BM / WM / 32;
    constexpr int TN = BNC / WN / 16;
    constexpr int BKC = 8;
    constexpr int BM_LOG = __builtin_ctz(BM), BN_LOG = __builtin_ctz(BNC);
    constexpr int AE = (BM * BKC + NT - 1) / NT;
    constexpr int BE = (BKC * BNC + NT - 1) / NT;
    __shared__ float As_re[2][BKC][BM + 1];
    __shared__ float As_im[2][BKC][BM + 1];
    __shared__ float2 Bs[2][BKC][BNC + 1];
    __shared__ int64_t row_lo[BM], col_lo[BNC], ak_lo[BKC], bk_lo[BKC];

    const int m_log = g.m_log, n_log = g.n_log, k_log = g.k_log;
    const int64_t m = int64_t(1) << m_log, n = int64_t(1) << n_log, k = int64_t(1) << k_log;
    const int tn_log = n_log >= BN_LOG ? n_log - BN_LOG : 0;
    const int64_t tiles = (m / BM) << tn_log;
    const int64_t inst = (int64_t)blockIdx.x / tiles;
    const int64_t tile = (int64_t)blockIdx.x - inst * tiles;
    const int64_t tm0 = (tile >> tn_log) * BM;
    const int64_t tn0 = (tile & ((int64_t(1) << tn_log) - 1)) * BNC;
    const int kc = k < BKC ? (int)k : BKC;
    const int kc_log = k_log < 3 ? k_log : 3;
    const int nb_bits = n_log < BN_LOG ? n_log : BN_LOG;
    for (int i = threadIdx.x; i < BM; i += NT) row_lo[i] = deposit(i, g.a_row, 0, BM_LOG);
    for (int i = threadIdx.x; i < BNC; i += NT) col_lo[i] = deposit(i, g.b_col, 0, nb_bits);
    for (int i = threadIdx.x; i < BKC; i += NT) {
        ak_lo[i] = deposit(i, g.a_k, 0, kc_log);
        bk_lo[i] = deposit(i, g.b_k, 0, kc_log);
    }
    const float2* __restrict__ A = (const float2*)g.A + g.oa[inst] + deposit(tm0, g.a_row, BM_LOG, m_log);
    const float2* __restrict__ B = (const float2*)g.B + g.ob[inst] + deposit(tn0, g.b_col, nb_bits, n_log);
    float* __restrict__ C = (float*)g.C + inst * (2 * m * n);
    __syncthreads();

    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int wm = wave % WM, wn = wave / WM;
    v16f acc[TM][TN];
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j)
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.0f;
    const int half = lane >> 5;
    const int sub = lane & 31;
    float2 ra[AE], rb[BE];
    auto load = [&](int64_t k0) {
        const int64_t akh = deposit(k0, g.a_k, kc_log, k_log);
        const int64_t bkh = deposit(k0, g.b_k, kc_log, k_log);
#pragma unroll
        for (int q = 0; q < AE; ++q) {
            const int e = threadIdx.x + q * NT;
            float2 v = make_float2(0.0f, 0.0f);
            if (e < BM * kc) {
                int r, p;
                if (g.a_rowfast) {
                    r = e & (BM - 1);
                    p = e >> BM_LOG;
                } else {
                    p = e & (kc - 1);
                    r = e >> kc_log;
                }
                v = A[row_lo[r] + ak_lo[p] + akh];
            }
            ra[q] = v;
        }
#pragma unroll
        for (int q = 0; q < BE; ++q) {
            const int e = threadIdx.x + q * NT;
            float2 v = make_float2(0.0f, 0.0f);
            if (e < kc * BNC) {
                int p, c;
                if (g.b_colfast) {
                    c = e & (BNC - 1);
                    p = e >> BN_LOG;
                } else {
                    p = e & (kc - 1);
                    c = e >> kc_log;
                }
                if (tn0 + c < n) v = B[col_lo[c] + bk_lo[p] + bkh];
            }
            rb[q] = v;
        }
    };
    auto stash = [&](int buf) {
#pragma unroll
        for (int q = 0; q < AE; ++q) {
            const int e = threadIdx.x + q * NT;
            if (e < BM * kc) {
                int r, p;
                if (g.a_rowfast) {
                    r = e & (BM - 1);
                    p = e >> BM_LOG;
                } else {
                    p = e & (kc - 1);
                    r = e >> kc_log;
                }
                As_re[buf][p][r] = ra[q].x;
                As_im[buf][p][r] = ra[q].y;
            }
        }
#pragma unroll
        for (int q = 0; q < BE; ++q) {
            const int e = threadIdx.x + q * NT;
            if (e < kc * BNC) {
                int p, c;
                if (g.b_colfast) {
                    c = e & (BNC - 1);
                    p = e >> BN_LOG;
                } else {
                    p = e & (kc - 1);
                    c = e >> kc_log;
                }
                Bs[buf][p][c] = rb[q];
            }
        }
    };
    const int64_t nchunks = k / kc;
    load(0);
    stash(0);
    __syncthreads();
    for (int64_t ch = 0; ch < nchunks; ++ch) {
        const int buf = (int)(ch & 1);
        if (ch + 1 < nchunks) load((ch + 1) * kc);
        for (int p = 0; p < kc; ++p) {
            float a[TM], b[TN];
#pragma unroll
            for (int i = 0; i < TM; ++i) {
                const int row = wm * (TM * 32) + i * 32 + sub;
                a[i] = half ? As_im[buf][p][row] : As_re[buf][p][row];
            }
#pragma unroll
            for (int j = 0; j < TN; ++j) {
                const int col = wn * (TN * 16) + j * 16 + (sub >> 1);
                const float2 bv = Bs[buf][p][col];
                const int t = sub & 1;
                b[j] = half == 0 ? (t == 0 ? bv.x : bv.y) : (t == 0 ? -bv.y : bv.x);
            }
#pragma unroll
            for (int i = 0; i < TM; ++i)
#pragma unroll
                for (int j = 0; j < TN; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[i], b[j], acc[i][j], 0, 0, 0);
        }
        if (ch + 1 < nchunks) stash(buf ^ 1);
        __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j) {
            const int64_t colf = 2 * (tn0 + wn * (TN * 16) + j * 16) + sub;
            if (colf >= 2 * n) continue;
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int64_t row = tm0 + wm * (TM * 32) + i * 32 + 8 * (r >> 2) + 4 * half + (r & 3);
                C[row * (2 * n) + colf] = acc[i][j][r];
            }
        }
}

// ---------------------------------------------------------------------------
// Tuning of the grouped matrix-core kernel (measured on the 25-qubit workload's
// 128 x 32 level, 848 slices of 256 x 16 x 256 and 134 of 512 x 16 x 64):
//   MFMA_GROUP_WAVES   register budget of the 64-row waves: two waves per SIMD
//                      leave room for the second register set of the two-deep
//                      chunk pipeline (three spill it); 113 us against 117 us at
//                      three waves with one chunk of read-ahead;
//   MFMA_ROWS32        32-row waves (below) at four waves per SIMD: 100 us
//                      against 113 us on that level, and faster on every tile
//                      shape of 64 or 128 rows but 128 x 64;
//   MFMA_PREFETCH2     loads run two chunks ahead of the MFMAs (the operands of
//                      tiles that miss in L2 come from HBM in a few us);
//   MFMA_SKIP_PAD      column blocks past a tile's last slice skip their MFMAs
//                      (a fifth of that level's tiles hold one slice of two).
#ifndef MFMA_GROUP_WAVES
#define MFMA_GROUP_WAVES 2
#endif
#ifndef MFMA_GROUP_WAVES_128X64
#define MFMA_GROUP_WAVES_128X64 4
#endif
#ifndef MFMA_RA_128X64
#define MFMA_RA_128X64 2
#endif
#ifndef MFMA_GROUP_BKC
#define MFMA_GROUP_BKC 8
#endif
#ifndef MFMA_GROUP_SCHED
#define MFMA_GROUP_SCHED 1
#endif
#ifndef MFMA_PREFETCH2
#define MFMA_PREFETCH2 1
#endif
#ifndef MFMA_SKIP_PAD
#define MFMA_SKIP_PAD 1
#endif
#ifndef MFMA_ROWS32
#define MFMA_ROWS32 1
#endif
#ifndef MFMA_ROWS32_128X64
#define MFMA_ROWS32_128X64 0
#endif
#ifndef MFMA_GROUP_WAVES_ROWS32
#define MFMA_GROUP_WAVES_ROWS32 4
#endif
// Wave layout of the grouped kernel: WM x WN waves, each holding TM x TN
// 32 x 32 real MFMA blocks (32 rows x 16 complex columns each).  With
// MFMA_ROWS32 the tiles of 64 and 128 rows run 32-row waves (half the
// accumulators of a 64-row wave), so up to four waves share each SIMD: one
// wave alone issues FP32 MFMAs at about half the matrix core's rate, two at
// about 85 %, four at about 94 % (a loop of independent 32 x 32 x 2 MFMAs).
// The 128 x 64 tile keeps 64-row waves (its 32-row form measured slower: eight
// waves per block, each re-reading B).
template <int BM, int BNC>
struct MfmaGroupShape {
    static constexpr bool ROWS32 = MFMA_ROWS32 && BM >= 64 && (MFMA_ROWS32_128X64 || !(BM == 128 && BNC == 64));
    static constexpr int WM = ROWS32 ? BM / 32 : (BM >= 64 ? BM / 64 : 1);
    static constexpr int WN = BNC >= 32 ? BNC / 32 : 1;
    static constexpr int NT = 64 * WM * WN;
    static constexpr int WAVES = ROWS32 ? MFMA_GROUP_WAVES_ROWS32
                                 : (BM == 64 && BNC == 32) ? 2
                                 : (BM == 128 && BNC == 64) ? MFMA_GROUP_WAVES_128X64
                                                            : MFMA_GROUP_WAVES;
};
// Grouped matrix-core contractions (FP32 complex on mfma_f32_32x32x2f32, the
// real embedding of K1).  One block per tile descriptor; the tile's row and
// column offsets (A / B element offsets, C row / column offsets, -1 = padding)
// are built in LDS from the job's slice tables, so slices that share an
// operand can fill one tile (merge modes) and any stored layout is read
// without a transpose pass.
// ---------------------------------------------------------------------------
template <int BM, int BNC>
__global__ __launch_bounds__((MfmaGroupShape<BM, BNC>::NT), (MfmaGroupShape<BM, BNC>::WAVES))
void k_mfma_group(const MfmaJob* __restrict__ jobs, const MfmaTile* __restrict__ tiles) {
    constexpr int WM = MfmaGroupShape<BM, BNC>::WM;
    constexpr int WN = MfmaGroupShape<BM, BNC>::WN;
    constexpr int NT = MfmaGroupShape<BM, BNC>::NT;
    constexpr int TM = BM / WM / 32;
    constexpr int TN = BNC / WN / 16;
    constexpr int BKC = MFMA_GROUP_BKC, BKC_LOG = __builtin_ctz(MFMA_GROUP_BKC);
    constexpr int BM_LOG = __builtin_ctz(BM), BN_LOG = __builtin_ctz(BNC);
    constexpr int AE = BM * BKC / NT;
    constexpr int BE = (BKC * BNC + NT - 1) / NT;
    // LDS staging, flat: A as [half][p][row] (half 0 real, 1 imaginary parts),
    // B once as [p][2 col + t] (re, im).  The real embedding's second B row
    // (-im, re) is read by the upper half-wave as the swapped pair with the
    // real-part slot negated, so every lane reads its MFMA operand with one
    // 4-byte load and B is staged once.  Row pitch +8 words keeps k-fast
    // staging writes (8 rows x 8 inner indices per 64 lanes) in distinct banks;
    // the +32-word gap between A's halves keeps the two half-waves' reads apart.
    constexpr int AP = BM + 8, AH = BKC * AP + 32, ABUF = 2 * AH;
    constexpr int BP = 2 * BNC + 8, BBUF = BKC * BP;
    __shared__ __align__(16) float As[2 * ABUF];
    __shared__ __align__(16) float Bs[2 * BBUF];
    __shared__ int64_t row_a[BM], row_c[BM], col_b[BNC], col_c[BNC], ak_lo[BKC], bk_lo[BKC];
    __shared__ int64_t a_step[32], b_step[32];
    __shared__ MfmaJob J;
    const MfmaTile T = tiles[blockIdx.x];
    if (threadIdx.x == 0) J = jobs[T.job];
    __syncthreads();
    const int m_log = J.m_log, n_log = J.n_log, k_log = J.k_log;
    const int64_t m = int64_t(1) << m_log, n = int64_t(1) << n_log, k = int64_t(1) << k_log;
    const int kc = k < BKC ? (int)k : BKC;
    const int kc_log = k_log < BKC_LOG ? k_log : BKC_LOG;
    for (int i = threadIdx.x; i < BM; i += NT) {
        int64_t ra = -1;
        if (J.merge == 2) {
            const int seg = i >> m_log;
            if (seg < T.cnt) ra = gload<int64_t>(J.oa)[T.s0 + seg] + deposit(i & (m - 1), J.a_row, 0, m_log);
        } else {
            const int64_t r = T.tm0 + i;
            if (r < m) ra = gload<int64_t>(J.oa)[T.s0] + deposit(r, J.a_row, 0, m_log);
        }
        row_a[i] = ra;
        row_c[i] = tile_out_row(J, T, i);
    }
    for (int j = threadIdx.x; j < BNC; j += NT) {
        int64_t cb = -1;
        if (J.merge == 1) {
            const int seg = j >> n_log;
            if (seg < T.cnt) cb = gload<int64_t>(J.ob)[T.s0 + seg] + deposit(j & (n - 1), J.b_col, 0, n_log);
        } else {
            const int64_t c = T.tn0 + j;
            if (c < n) cb = gload<int64_t>(J.ob)[T.s0] + deposit(c, J.b_col, 0, n_log);
        }
        col_b[j] = cb;
        col_c[j] = tile_out_col(J, T, j);
    }
    for (int i = threadIdx.x; i < BKC; i += NT) {
        ak_lo[i] = i < kc ? deposit(i, J.a_k, 0, kc_log) : 0;
        bk_lo[i] = i < kc ? deposit(i, J.b_k, 0, kc_log) : 0;
    }
    chunk_steps(J.a_k, kc_log, k_log, a_step);
    chunk_steps(J.b_k, kc_log, k_log, b_step);
    __syncthreads();
    const TN_GLOBAL float2* __restrict__ A = gload<float2>(J.A);
    const TN_GLOBAL float2* __restrict__ B = gload<float2>(J.B);
    TN_GLOBAL float* __restrict__ C = gstore<float>(J.C);
    const bool a_rowfast = J.a_rowfast, b_colfast = J.b_colfast;

    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int wm = wave % WM, wn = wave / WM;
    v16f acc[TM][TN];
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j)
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.0f;
    const int half = lane >> 5;
    const int sub = lane & 31;
    // staging order: element e of a chunk is (row r, inner p) with r fast when
    // the operand's lowest stored bit is a row bit, else p fast; inner indices
    // p >= kc (k < 8) are zero
    auto a_rp = [&](int e, int& r, int& p) {
        if (a_rowfast) {
            r = e & (BM - 1);
            p = e >> BM_LOG;
        } else {
            p = e & (BKC - 1);
            r = e >> BKC_LOG;
        }
    };
    auto b_pc = [&](int e, int& p, int& c) {
        if (b_colfast) {
            c = e & (BNC - 1);
            p = e >> BN_LOG;
        } else {
            p = e & (BKC - 1);
            c = e >> BKC_LOG;
        }
    };
    // chunks of this block: all, or part kpart of ksplit equal parts (split
    // inner sum; the host keeps ksplit a power of two dividing the chunk count)
    const int64_t nch_all = k >= BKC ? k / BKC : 1;
    const int64_t c_begin = nch_all / J.ksplit * T.kpart;
    const int64_t c_end = c_begin + nch_all / J.ksplit;
    // offsets of the high inner bits of the chunk being loaded (chunks are
    // loaded in order: advanced by the step table after each load)
    int64_t kchunk = c_begin;
    int64_t akh = deposit(c_begin << kc_log, J.a_k, kc_log, k_log);
    int64_t bkh = deposit(c_begin << kc_log, J.b_k, kc_log, k_log);
    // offsets of this thread's staged elements inside a chunk (fixed over the
    // chunks; -1 = padding, loaded from element 0 and replaced by zero)
    int64_t aoff[AE], boff[BE];
#pragma unroll
    for (int q = 0; q < AE; ++q) {
        int r, p;
        a_rp(threadIdx.x + q * NT, r, p);
        const int64_t base = row_a[r];
        aoff[q] = (base >= 0 && p < kc) ? base + ak_lo[p] : -1;
    }
#pragma unroll
    for (int q = 0; q < BE; ++q) {
        const int e = threadIdx.x + q * NT;
        boff[q] = -1;
        if (e < BKC * BNC) {
            int p, c;
            b_pc(e, p, c);
            const int64_t base = col_b[c];
            if (base >= 0 && p < kc) boff[q] = base + bk_lo[p];
        }
    }
    // raw loads (padding lanes read element 0); padding is zeroed when staged,
    // so nothing waits on a load before the chunk's MFMAs
    auto load = [&](int64_t, float2* ra, float2* rb) {
#pragma unroll
        for (int q = 0; q < AE; ++q) ra[q] = gld(A + (aoff[q] >= 0 ? aoff[q] + akh : 0));
#pragma unroll
        for (int q = 0; q < BE; ++q) rb[q] = gld(B + (boff[q] >= 0 ? boff[q] + bkh : 0));
        const int t = __builtin_ctzll(~(uint64_t)kchunk);
        if (t < k_log - kc_log) {
            akh += a_step[t];
            bkh += b_step[t];
        }
        ++kchunk;
    };
    auto stash = [&](int buf, const float2* ra, const float2* rb) {
        float* as = As + buf * ABUF;
        float* bs = Bs + buf * BBUF;
#pragma unroll
        for (int q = 0; q < AE; ++q) {
            int r, p;
            a_rp(threadIdx.x + q * NT, r, p);
            const bool ok = aoff[q] >= 0;
            as[p * AP + r] = ok ? ra[q].x : 0.0f;
            as[AH + p * AP + r] = ok ? ra[q].y : 0.0f;
        }
#pragma unroll
        for (int q = 0; q < BE; ++q) {
            const int e = threadIdx.x + q * NT;
            if (e < BKC * BNC) {
                int p, c;
                b_pc(e, p, c);
                *(float2*)&bs[p * BP + 2 * c] = boff[q] >= 0 ? rb[q] : make_float2(0.0f, 0.0f);
            }
        }
    };
    // per-lane LDS offsets of the MFMA operands
    int a_off[TM], b_off[TN];
#pragma unroll
    for (int i = 0; i < TM; ++i) a_off[i] = half * AH + wm * (TM * 32) + i * 32 + sub;
#pragma unroll
    for (int j = 0; j < TN; ++j) b_off[j] = 2 * (wn * (TN * 16) + j * 16) + (half ? (sub ^ 1) : sub);
    const uint32_t b_sign = (half && !(sub & 1)) ? 0x80000000u : 0u;
    // operands read ahead per group of RA inner indices: the whole chunk, or two
    // on 128 x 64 tiles (held to four waves per SIMD, whose 128-register budget
    // the full read-ahead would exceed; a few spills remain outside the loop)
    constexpr bool WIDE = BM == 128 && BNC == 64 && !MfmaGroupShape<BM, BNC>::ROWS32;
    constexpr int RA = WIDE ? MFMA_RA_128X64 : BKC;
    // TNA: this wave's column blocks that hold outputs (the others are padding
    // past the tile's last slice or column, skipped)
    auto compute = [&](int buf, auto tna) {
        constexpr int TNA = decltype(tna)::value;
        const float* as = As + buf * ABUF;
        const float* bs = Bs + buf * BBUF;
#pragma unroll
        for (int g = 0; g < BKC; g += RA) {
            // all operands of the group read first, so the LDS reads of later
            // inner indices are in flight while the MFMAs of earlier ones run
            float a[RA][TM], b[RA][TNA];
#pragma unroll
            for (int p = 0; p < RA; ++p) {
#pragma unroll
                for (int i = 0; i < TM; ++i) a[p][i] = as[(g + p) * AP + a_off[i]];
#pragma unroll
                for (int j = 0; j < TNA; ++j)
                    b[p][j] = __uint_as_float(__float_as_uint(bs[(g + p) * BP + b_off[j]]) ^ b_sign);
            }
#pragma unroll
            for (int p = 0; p < RA; ++p)
#pragma unroll
                for (int i = 0; i < TM; ++i)
#pragma unroll
                    for (int j = 0; j < TNA; ++j)
                        acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[p][i], b[p][j], acc[i][j], 0, 0, 0);
            // keep the reads ahead of the MFMAs: DS reads of inner index p + 1
            // are scheduled before the MFMAs of inner index p
#if MFMA_GROUP_SCHED
            __builtin_amdgcn_sched_group_barrier(0x100, TM + TNA, 0);
#pragma unroll
            for (int p = 0; p < RA; ++p) {
                if (p + 1 < RA) __builtin_amdgcn_sched_group_barrier(0x100, TM + TNA, 0);
                __builtin_amdgcn_sched_group_barrier(0x008, TM * TNA, 0);
            }
#endif
        }
    };
    // column blocks of 16 holding outputs (padding is a suffix of the tile's
    // columns: slices past cnt, columns past n): all TN, the first only, or none
    int tn_act = 0;
#pragma unroll
    for (int j = 0; j < TN; ++j)
        if (col_c[wn * (TN * 16) + j * 16] >= 0) tn_act = j + 1;
    auto compute_active = [&](int buf) {
        if (!MFMA_SKIP_PAD || tn_act == TN) compute(buf, std::integral_constant<int, TN>{});
        else if (TN > 1 && tn_act == 1) compute(buf, std::integral_constant<int, 1>{});
    };
    const int64_t nchunks = c_end - c_begin;
    if (MFMA_PREFETCH2 && !WIDE) {
        // pipeline two chunks deep: LDS holds chunk ch, registers hold chunk
        // ch + 1, and the loads of chunk ch + 2 are in flight during chunk ch's
        // MFMAs (a chunk's loads have two chunks of matrix-core work to arrive
        // from HBM when they miss in L2).  Chunk c is staged in and read from
        // LDS buffer c & 1; the two register sets alternate with it.  (The
        // 128 x 64 tile's register budget holds one set.)
        float2 ra0[AE], rb0[BE], ra1[AE], rb1[BE];
        load(0, ra0, rb0);
        stash(0, ra0, rb0);
        if (nchunks > 1) load(BKC, ra1, rb1);
        __syncthreads();
        for (int64_t ch = 0; ch < nchunks; ch += 2) {
            if (ch + 2 < nchunks) load((ch + 2) * BKC, ra0, rb0);
            compute_active(0);
            if (ch + 1 < nchunks) stash(1, ra1, rb1);
            __syncthreads();
            if (ch + 1 >= nchunks) break;
            if (ch + 3 < nchunks) load((ch + 3) * BKC, ra1, rb1);
            compute_active(1);
            if (ch + 2 < nchunks) stash(0, ra0, rb0);
            __syncthreads();
        }
    } else {
        // pipeline: LDS holds chunk ch while the loads of chunk ch + 1 are in flight
        float2 ra[AE], rb[BE];
        load(0, ra, rb);
        stash(0, ra, rb);
        __syncthreads();
        for (int64_t ch = 0; ch < nchunks; ++ch) {
            const int buf = (int)(ch & 1);
            if (ch + 1 < nchunks) load((ch + 1) * BKC, ra, rb);
            compute_active(buf);
            if (ch + 1 < nchunks) stash(buf ^ 1, ra, rb);
            __syncthreads();
        }
    }

    // split inner sum: this block's part goes to its row-major [BM][BNC] partial
    // tile (padding skipped), added to the others' by k_split_reduce
    const bool to_partial = J.ksplit > 1;
    TN_GLOBAL float* __restrict__ O =
        to_partial ? gstore<float>(J.partial) + ((int64_t)T.pair * J.ksplit + T.kpart) * (2 * BM * BNC) : C;
    // output offsets of this lane's 16 rows and TN columns read ahead of the
    // stores (one LDS wait per row block instead of one per store)
    const int part = sub & 1;
    int64_t ccs[TN];
#pragma unroll
    for (int j = 0; j < TN; ++j) {
        const int col = wn * (TN * 16) + j * 16 + (sub >> 1);
        ccs[j] = to_partial ? (col_c[col] < 0 ? -1 : col) : col_c[col];
    }
#pragma unroll
    for (int i = 0; i < TM; ++i) {
        int64_t rcs[16];
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int row = wm * (TM * 32) + i * 32 + 8 * (r >> 2) + 4 * half + (r & 3);
            const int64_t rc = row_c[row];
            rcs[r] = to_partial ? (rc < 0 ? -1 : (int64_t)row * BNC) : rc;
        }
#pragma unroll
        for (int j = 0; j < TN; ++j) {
            if (ccs[j] < 0) continue;
#pragma unroll
            for (int r = 0; r < 16; ++r)
                if (rcs[r] >= 0) O[2 * (rcs[r] + ccs[j]) + part] = acc[i][j][r];
        }
    }
}

// ---------------------------------------------------------------------------
// Grouped gathered contractions: every small step of one tree level (all
// clusters, all plans) in one launch.  A block finds its job by binary search
// over the jobs' first blocks.  Operands are read in their stored order
// through the per-bit positions (no transpose pass); the low inner bits' offsets
// come from an LDS table, the high ones are added once per 256-wide chunk.
//   split == 0: one thread per output element, inner loop in registers;
//   split == 1: one block per output element (few outputs, long inner sums),
//               partial sums reduced in FP64 through LDS.
// ---------------------------------------------------------------------------
struct GettSmem {
    GettJob J;
    int64_t ak_lo[256], bk_lo[256];
    double red_r[256], red_i[256];
    int64_t a_step[32], b_step[32];
};

// One thread of a small step: column c of RPT consecutive rows (the column
// operand's element is loaded once for all of them; the row operand's
// elements are shared by the lanes of a wave, which hold consecutive
// columns).  The loads of P inner indices are issued before their products, so
// a thread waits once per P inner indices; products are added in inner-index
// order.
template <typename R, typename C2, int RPT>
__device__ __forceinline__ void gett_rows(const GettJob& J, const int64_t* __restrict__ ak_lo,
                                          const int64_t* __restrict__ bk_lo, const int64_t* __restrict__ a_step,
                                          const int64_t* __restrict__ b_step, int64_t local) {
    constexpr int RLOG = RPT == 1 ? 0 : RPT == 2 ? 1 : RPT == 4 ? 2 : 3;
    constexpr int P = sizeof(R) == 4 ? (RPT == 1 ? 8 : RPT <= 4 ? 4 : 2) : (RPT <= 2 ? 4 : RPT == 4 ? 2 : 1);
    const int m_log = J.m_log, n_log = J.n_log, k_log = J.k_log;
    const int mn_log = m_log + n_log;
    const int64_t k = int64_t(1) << k_log;
    const int kc_log = k_log < 8 ? k_log : 8;
    const int kc = 1 << kc_log;
    const int nstep = k_log - kc_log;
    const int64_t o = local * 256 + threadIdx.x;
    if (o >= (J.n_inst << (mn_log - RLOG))) return;
    const int64_t c = o & ((int64_t(1) << n_log) - 1);
    const int64_t rest = o >> n_log;
    const int64_t rg = rest & ((int64_t(1) << (m_log - RLOG)) - 1);
    const int64_t inst = rest >> (m_log - RLOG);
    const int64_t r0 = rg << RLOG;
    const TN_GLOBAL C2* __restrict__ Ap = gload<C2>(J.A) + gload<int64_t>(J.oa)[inst] + deposit(r0, J.a_row, 0, m_log);
    const TN_GLOBAL C2* __restrict__ Bp = gload<C2>(J.B) + gload<int64_t>(J.ob)[inst] + deposit(c, J.b_col, 0, n_log);
    int64_t rlo[RPT];
#pragma unroll
    for (int i = 0; i < RPT; ++i) rlo[i] = deposit(i, J.a_row, 0, RLOG);
    R sr[RPT], si[RPT];
#pragma unroll
    for (int i = 0; i < RPT; ++i) sr[i] = si[i] = 0;
    int64_t ahh = 0, bhh = 0;
    for (int64_t h = 0; h < k; h += kc) {
        const TN_GLOBAL C2* __restrict__ Ah = Ap + ahh;
        const TN_GLOBAL C2* __restrict__ Bh = Bp + bhh;
        {
            const int t = __builtin_ctzll(~(uint64_t)(h >> kc_log));
            if (t < nstep) {
                ahh += a_step[t];
                bhh += b_step[t];
            }
        }
        int p = 0;
        for (; p + P <= kc; p += P) {
            C2 b[P], a[P][RPT];
#pragma unroll
            for (int u = 0; u < P; ++u) {
                b[u] = gld(Bh + bk_lo[p + u]);
                const int64_t ap = ak_lo[p + u];
#pragma unroll
                for (int i = 0; i < RPT; ++i) a[u][i] = gld(Ah + (rlo[i] + ap));
            }
#pragma unroll
            for (int u = 0; u < P; ++u)
#pragma unroll
                for (int i = 0; i < RPT; ++i) {
                    sr[i] += a[u][i].x * b[u].x - a[u][i].y * b[u].y;
                    si[i] += a[u][i].x * b[u].y + a[u][i].y * b[u].x;
                }
        }
        for (; p < kc; ++p) {
            const C2 b = gld(Bh + bk_lo[p]);
            const int64_t ap = ak_lo[p];
            C2 a[RPT];
#pragma unroll
            for (int i = 0; i < RPT; ++i) a[i] = gld(Ah + (rlo[i] + ap));
#pragma unroll
            for (int i = 0; i < RPT; ++i) {
                sr[i] += a[i].x * b.x - a[i].y * b.y;
                si[i] += a[i].x * b.y + a[i].y * b.x;
            }
        }
    }
    TN_GLOBAL C2* __restrict__ Cp = gstore<C2>(J.C) + ((inst << mn_log) + (r0 << n_log) + c);
#pragma unroll
    for (int i = 0; i < RPT; ++i) {
        C2 out;
        out.x = sr[i];
        out.y = si[i];
        gst(Cp + ((int64_t)i << n_log), out);
    }
}

template <typename R, typename C2>
__device__ __forceinline__ void gett_block(const GettJob* __restrict__ jp, GettSmem& sm) {
    GettJob& J = sm.J;
    int64_t* ak_lo = sm.ak_lo;
    int64_t* bk_lo = sm.bk_lo;
    double* red_r = sm.red_r;
    double* red_i = sm.red_i;
    int64_t* a_step = sm.a_step;
    int64_t* b_step = sm.b_step;
    const int64_t bid = blockIdx.x;
    if (threadIdx.x == 0) J = *jp;
    __syncthreads();
    const int m_log = J.m_log, n_log = J.n_log, k_log = J.k_log;
    const int mn_log = m_log + n_log;
    const int64_t k = int64_t(1) << k_log;
    const int kc_log = k_log < 8 ? k_log : 8;
    const int kc = 1 << kc_log;
    for (int i = threadIdx.x; i < kc; i += 256) {
        ak_lo[i] = deposit(i, J.a_k, 0, kc_log);
        bk_lo[i] = deposit(i, J.b_k, 0, kc_log);
    }
    chunk_steps(J.a_k, kc_log, k_log, a_step);
    chunk_steps(J.b_k, kc_log, k_log, b_step);
    __syncthreads();
    const int nstep = k_log - kc_log;
    const int64_t local = bid - J.block0;
    if (J.split) {
        // one output element per block; thread t takes inner indices t + 256 h
        const int64_t o = local;
        const int64_t inst = o >> mn_log;
        const int64_t rc = o & ((int64_t(1) << mn_log) - 1);
        const int64_t r = rc >> n_log, c = rc & ((int64_t(1) << n_log) - 1);
        const TN_GLOBAL C2* __restrict__ Ap = gload<C2>(J.A) + gload<int64_t>(J.oa)[inst] + deposit(r, J.a_row, 0, m_log);
        const TN_GLOBAL C2* __restrict__ Bp = gload<C2>(J.B) + gload<int64_t>(J.ob)[inst] + deposit(c, J.b_col, 0, n_log);
        R sr = 0, si = 0;
        if ((int)threadIdx.x < kc) {
            const int64_t alo = ak_lo[threadIdx.x], blo = bk_lo[threadIdx.x];
            // U chunks per round (16 in FP32, 8 in FP64): their loads are all in
            // flight before the first product (the chunk count is a power of two)
            constexpr int U = sizeof(R) == 4 ? 16 : 8;
            const int64_t nh = k >> kc_log;
            const int64_t step = nh >= U ? U : nh;
            int64_t ah = alo, bh = blo;
            for (int64_t h0 = 0; h0 < nh; h0 += step) {
                C2 a[U], b[U];
#pragma unroll
                for (int u = 0; u < U; ++u)
                    if (u < step) {
                        a[u] = gld(Ap + ah);
                        b[u] = gld(Bp + bh);
                        const int t = __builtin_ctzll(~(uint64_t)(h0 + u));
                        if (t < nstep) {
                            ah += a_step[t];
                            bh += b_step[t];
                        }
                    }
#pragma unroll
                for (int u = 0; u < U; ++u)
                    if (u < step) {
                        sr += a[u].x * b[u].x - a[u].y * b[u].y;
                        si += a[u].x * b[u].y + a[u].y * b[u].x;
                    }
            }
        }
        // FP64 sum in a fixed order: a butterfly within each wave (both lanes
        // of a pair form the same sum), then the four waves in order
        double vr = (double)sr, vi = (double)si;
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
            vr += __shfl_xor(vr, off);
            vi += __shfl_xor(vi, off);
        }
        if ((threadIdx.x & 63) == 0) {
            red_r[threadIdx.x >> 6] = vr;
            red_i[threadIdx.x >> 6] = vi;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            C2 out;
            out.x = (R)(((red_r[0] + red_r[1]) + red_r[2]) + red_r[3]);
            out.y = (R)(((red_i[0] + red_i[1]) + red_i[2]) + red_i[3]);
            gst(gstore<C2>(J.C) + o, out);
        }
        return;
    }
    // one thread: column c of 2^rpt_log consecutive rows
    switch (J.rpt_log) {
        case 0: gett_rows<R, C2, 1>(J, ak_lo, bk_lo, a_step, b_step, local); break;
        case 1: gett_rows<R, C2, 2>(J, ak_lo, bk_lo, a_step, b_step, local); break;
        case 2: gett_rows<R, C2, 4>(J, ak_lo, bk_lo, a_step, b_step, local); break;
        default: gett_rows<R, C2, 8>(J, ak_lo, bk_lo, a_step, b_step, local); break;
    }
}

// One launch for the small steps of one tree level: block b runs job
// block_job[b] & 0x7fffffff, in FP64 when bit 31 is set (the dominant-term
// pass's jobs of the same level), else in FP32.  The table is built on the
// host, so a block finds its job with one load.
__global__ __launch_bounds__(256) void k_gett_group(const GettJob* __restrict__ jobs,
                                                    const int32_t* __restrict__ block_job) {
    __shared__ GettSmem sm;
    const uint32_t e = (uint32_t)block_job[blockIdx.x];
    const GettJob* jp = jobs + (e & 0x7fffffffu);
    if (e >> 31) gett_block<double, double2>(jp, sm);
    else gett_block<float, float2>(jp, sm);
}

// ---------------------------------------------------------------------------
// Small shapes: one thread per output element, k loop in registers.
// ---------------------------------------------------------------------------
template <typename R, typename C2>
__global__ __launch_bounds__(256) void k_gemm_small(GemmArgs g) {
    const int64_t total = g.n_inst << (g.m_log + g.n_log);
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= total) return;
    const int64_t n = int64_t(1) << g.n_log, m = int64_t(1) << g.m_log, k = int64_t(1) << g.k_log;
    const int64_t inst = idx >> (g.m_log + g.n_log);
    const int64_t rc = idx & ((int64_t(1) << (g.m_log + g.n_log)) - 1);
    const int64_t r = rc >> g.n_log, c = rc & (n - 1);
    const C2* A = (const C2*)g.A + pick(g.ia_mode, g.ia, inst) * g.strideA;
    const C2* B = (const C2*)g.B + pick(g.ib_mode, g.ib, inst) * g.strideB;
    R sr = 0, si = 0;
    for (int64_t p = 0; p < k; ++p) {
        const C2 a = g.transA ? A[p * m + r] : A[r * k + p];
        const C2 b = g.transB ? B[c * k + p] : B[p * n + c];
        sr += a.x * b.x - a.y * b.y;
        si += a.x * b.y + a.y * b.x;
    }
    C2 o;
    o.x = sr;
    o.y = si;
    ((C2*)g.C)[idx] = o;
}

// ---------------------------------------------------------------------------
// Tiny outputs with long k (inner products): one block per output element,
// strided partial sums, FP64 tree reduction in LDS.
// ---------------------------------------------------------------------------
template <typename R, typename C2>
__global__ __launch_bounds__(256) void k_gemm_splitk(GemmArgs g) {
    __shared__ double red_r[256];
    __shared__ double red_i[256];
    const int64_t n = int64_t(1) << g.n_log, m = int64_t(1) << g.m_log, k = int64_t(1) << g.k_log;
    const int64_t out = blockIdx.x;
    const int64_t inst = out >> (g.m_log + g.n_log);
    const int64_t rc = out & ((int64_t(1) << (g.m_log + g.n_log)) - 1);
    const int64_t r = rc >> g.n_log, c = rc & (n - 1);
    const C2* A = (const C2*)g.A + pick(g.ia_mode, g.ia, inst) * g.strideA;
    const C2* B = (const C2*)g.B + pick(g.ib_mode, g.ib, inst) * g.strideB;
    R sr = 0, si = 0;
    for (int64_t p = threadIdx.x; p < k; p += blockDim.x) {
        const C2 a = g.transA ? A[p * m + r] : A[r * k + p];
        const C2 b = g.transB ? B[c * k + p] : B[p * n + c];
        sr += a.x * b.x - a.y * b.y;
        si += a.x * b.y + a.y * b.x;
    }
    red_r[threadIdx.x] = (double)sr;
    red_i[threadIdx.x] = (double)si;
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
            red_r[threadIdx.x] += red_r[threadIdx.x + s];
            red_i[threadIdx.x] += red_i[threadIdx.x + s];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        C2 o;
        o.x = (R)red_r[0];
        o.y = (R)red_i[0];
        ((C2*)g.C)[out] = o;
    }
}

// ---------------------------------------------------------------------------
// FP64 tiled GEMM (complex128) for the dominant-term pass: 64x64 output tile,
// 256 threads each holding a 4x4 block, k staged through LDS in chunks of 8.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_gemm_tiled_c128(GemmArgs g) {
    constexpr int BM = 64, BN = 64, BK = 8;
    __shared__ double2 As[BK][BM];
    __shared__ double2 Bs[BK][BN];
    const int64_t m = int64_t(1) << g.m_log, n = int64_t(1) << g.n_log, k = int64_t(1) << g.k_log;
    const int tn_log = g.n_log - 6;
    const int64_t tiles = (m / BM) << tn_log;
    const int64_t inst = blockIdx.x / tiles;
    const int64_t tile = blockIdx.x - inst * tiles;
    const int64_t tm0 = (tile >> tn_log) * BM, tn0 = (tile & ((int64_t(1) << tn_log) - 1)) * BN;
    const double2* A = (const double2*)g.A + pick(g.ia_mode, g.ia, inst) * g.strideA;
    const double2* B = (const double2*)g.B + pick(g.ib_mode, g.ib, inst) * g.strideB;
    double2* C = (double2*)g.C + inst * m * n;
    const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
    double accr[4][4], acci[4][4];
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) accr[i][j] = acci[i][j] = 0.0;
    const int kc = k < BK ? (int)k : BK;
    for (int64_t k0 = 0; k0 < k; k0 += kc) {
        for (int e = threadIdx.x; e < BM * kc; e += 256) {
            int r, p;
            if (!g.transA) { r = e / kc; p = e % kc; As[p][r] = A[(tm0 + r) * k + k0 + p]; }
            else { p = e / BM; r = e % BM; As[p][r] = A[(k0 + p) * m + tm0 + r]; }
        }
        for (int e = threadIdx.x; e < kc * BN; e += 256) {
            int p, c;
            if (!g.transB) { p = e / BN; c = e % BN; Bs[p][c] = B[(k0 + p) * n + tn0 + c]; }
            else { c = e / kc; p = e % kc; Bs[p][c] = B[(tn0 + c) * k + k0 + p]; }
        }
        __syncthreads();
        for (int p = 0; p < kc; ++p) {
            double2 a[4], b[4];
            for (int i = 0; i < 4; ++i) a[i] = As[p][ty + 16 * i];
            for (int j = 0; j < 4; ++j) b[j] = Bs[p][tx + 16 * j];
            for (int i = 0; i < 4; ++i)
                for (int j = 0; j < 4; ++j) {
                    accr[i][j] += a[i].x * b[j].x - a[i].y * b[j].y;
                    acci[i][j] += a[i].x * b[j].y + a[i].y * b[j].x;
                }
        }
        __syncthreads();
    }
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) {
            double2 o;
            o.x = accr[i][j];
            o.y = acci[i][j];
            C[(tm0 + ty + 16 * i) * n + tn0 + tx + 16 * j] = o;
        }
}

// ---------------------------------------------------------------------------
// Grouped FP64 tiles (complex128 FMA): the descriptors of the grouped
// matrix-core launch (merge modes, slice tables, per-bit positions) on
// 16TT x 16TT output tiles (TT = 4: 64 x 64; TT = 2: 32 x 32, four times the tiles
// for jobs that would leave CUs idle); 256 threads, TT x TT outputs each, inner
// chunks of 8 staged in LDS through the tile's row / column offset tables.
// ---------------------------------------------------------------------------
#ifndef TILE64_MFMA
#define TILE64_MFMA 1
#endif
// MF = 1: the products run on the FP64 matrix cores (v_mfma_f64_16x16x4f64 on the
// real embedding, as the FP32 kernel: one instruction is 16 rows x 8 complex
// columns x 2 complex inner indices); the four waves take the tile's quadrants.
// Operands come from the same LDS rows; each lane reads one double per operand
// per instruction instead of a thread reading TT complex values of A and of B
// per inner index (the FMA form reads 1 byte of LDS per flop).
template <int TT, bool MF>
__global__ __launch_bounds__(256) void k_tile64_group(const MfmaJob* __restrict__ jobs,
                                                      const MfmaTile* __restrict__ tiles) {
    constexpr int BM = 16 * TT, BN = 16 * TT, BK = 8, BK_LOG = 3;
    constexpr int BM_LOG = __builtin_ctz(BM), BN_LOG = __builtin_ctz(BN);
    constexpr int SE = (BM * BK + 255) / 256;   // staged elements per thread and operand
    // +2 elements per row: k-fast staging writes of 16 lanes fall in distinct banks;
    // two buffers: chunk ch + 1 is stashed while chunk ch is multiplied
    __shared__ double2 As2[2][BK][BM + 2];
    __shared__ double2 Bs2[2][BK][BN + 2];
    __shared__ int64_t row_a[BM], row_c[BM], col_b[BN], col_c[BN], ak_lo[BK], bk_lo[BK];
    __shared__ int64_t a_step[32], b_step[32];
    __shared__ MfmaJob J;
    const MfmaTile T = tiles[blockIdx.x];
    if (threadIdx.x == 0) J = jobs[T.job];
    __syncthreads();
    const int m_log = J.m_log, n_log = J.n_log, k_log = J.k_log;
    const int64_t m = int64_t(1) << m_log, n = int64_t(1) << n_log, k = int64_t(1) << k_log;
    const int kc = k < BK ? (int)k : BK;
    const int kc_log = k_log < BK_LOG ? k_log : BK_LOG;
    for (int i = threadIdx.x; i < BM; i += 256) {
        int64_t ra = -1;
        if (J.merge == 2) {
            const int seg = i >> m_log;
            if (seg < T.cnt) ra = gload<int64_t>(J.oa)[T.s0 + seg] + deposit(i & (m - 1), J.a_row, 0, m_log);
        } else {
            const int64_t r = T.tm0 + i;
            if (r < m) ra = gload<int64_t>(J.oa)[T.s0] + deposit(r, J.a_row, 0, m_log);
        }
        row_a[i] = ra;
        row_c[i] = tile_out_row(J, T, i);
    }
    for (int j = threadIdx.x; j < BN; j += 256) {
        int64_t cb = -1;
        if (J.merge == 1) {
            const int seg = j >> n_log;
            if (seg < T.cnt) cb = gload<int64_t>(J.ob)[T.s0 + seg] + deposit(j & (n - 1), J.b_col, 0, n_log);
        } else {
            const int64_t c = T.tn0 + j;
            if (c < n) cb = gload<int64_t>(J.ob)[T.s0] + deposit(c, J.b_col, 0, n_log);
        }
        col_b[j] = cb;
        col_c[j] = tile_out_col(J, T, j);
    }
    for (int i = threadIdx.x; i < BK; i += 256) {
        ak_lo[i] = i < kc ? deposit(i, J.a_k, 0, kc_log) : 0;
        bk_lo[i] = i < kc ? deposit(i, J.b_k, 0, kc_log) : 0;
    }
    chunk_steps(J.a_k, kc_log, k_log, a_step);
    chunk_steps(J.b_k, kc_log, k_log, b_step);
    __syncthreads();
    const TN_GLOBAL double2* __restrict__ A = gload<double2>(J.A);
    const TN_GLOBAL double2* __restrict__ B = gload<double2>(J.B);
    TN_GLOBAL double2* __restrict__ C = gstore<double2>(J.C);
    const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
    double accr[MF ? 1 : TT][MF ? 1 : TT], acci[MF ? 1 : TT][MF ? 1 : TT];
    // matrix-core form: wave quadrant (rows wr0.., complex columns wc0..), WR x WC
    // instructions of 16 rows x 8 complex columns each
    constexpr int WR = MF ? BM / 32 : 1, WC = MF ? BN / 16 : 1;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int wr0 = (wave & 1) * (BM / 2), wc0 = (wave >> 1) * (BN / 2);
    const int kpart = (lane >> 4) & 1;           // real-embedding row: 0 = Re, 1 = Im of A's element
    const int tcol = lane & 1;                   // output component of this lane's column
    v4d acc[WR][WC];
    if constexpr (MF) {
#pragma unroll
        for (int i = 0; i < WR; ++i)
#pragma unroll
            for (int j = 0; j < WC; ++j) acc[i][j] = v4d{0.0, 0.0, 0.0, 0.0};
    } else {
#pragma unroll
        for (int i = 0; i < TT; ++i)
#pragma unroll
            for (int j = 0; j < TT; ++j) accr[i][j] = acci[i][j] = 0.0;
    }
    const int64_t nch_all = k >= BK ? k / BK : 1;
    const int64_t c_begin = nch_all / J.ksplit * T.kpart;
    const int64_t c_end = c_begin + nch_all / J.ksplit;
    int64_t akh = deposit(c_begin << kc_log, J.a_k, kc_log, k_log);
    int64_t bkh = deposit(c_begin << kc_log, J.b_k, kc_log, k_log);
    // this thread's staged elements: LDS slots and offsets inside a chunk
    // (fixed over the chunks; -1 = padding, staged as zero)
    int sa_r[SE], sa_p[SE], sb_c[SE], sb_p[SE];
    int64_t aoff[SE], boff[SE];
#pragma unroll
    for (int q = 0; q < SE; ++q) {
        const int e = threadIdx.x + q * 256;
        int r = 0, p = 0, pb = 0, c = 0;
        if (J.a_rowfast) {
            r = e & (BM - 1);
            p = e >> BM_LOG;
        } else {
            p = e & (BK - 1);
            r = e >> BK_LOG;
        }
        if (J.b_colfast) {
            c = e & (BN - 1);
            pb = e >> BN_LOG;
        } else {
            pb = e & (BK - 1);
            c = e >> BK_LOG;
        }
        const bool in = e < BM * BK;
        sa_r[q] = r;
        sa_p[q] = p;
        sb_c[q] = c;
        sb_p[q] = pb;
        aoff[q] = (in && row_a[r] >= 0 && p < kc) ? row_a[r] + ak_lo[p] : -1;
        boff[q] = (in && col_b[c] >= 0 && pb < kc) ? col_b[c] + bk_lo[pb] : -1;
    }
    // chunk ch + 1 is loaded into registers while chunk ch is multiplied
    double2 ra[SE], rb[SE];
    auto load = [&]() {
#pragma unroll
        for (int q = 0; q < SE; ++q) {
            ra[q] = aoff[q] >= 0 ? gld(A + (aoff[q] + akh)) : make_double2(0.0, 0.0);
            rb[q] = boff[q] >= 0 ? gld(B + (boff[q] + bkh)) : make_double2(0.0, 0.0);
        }
    };
    auto advance = [&](int64_t ch) {
        const int t = __builtin_ctzll(~(uint64_t)ch);
        if (t < k_log - kc_log) {
            akh += a_step[t];
            bkh += b_step[t];
        }
    };
    auto stash = [&](int buf) {
#pragma unroll
        for (int q = 0; q < SE; ++q) {
            if (threadIdx.x + q * 256 >= BM * BK) break;
            As2[buf][sa_p[q]][sa_r[q]] = ra[q];
            Bs2[buf][sb_p[q]][sb_c[q]] = rb[q];
        }
    };
    if (c_begin < c_end) {
        load();
        advance(c_begin);
        stash(0);
        __syncthreads();
    }
    for (int64_t ch = c_begin; ch < c_end; ++ch) {
        const int buf = (int)((ch - c_begin) & 1);
        const double2(*As)[BM + 2] = As2[buf];
        const double2(*Bs)[BN + 2] = Bs2[buf];
        if (ch + 1 < c_end) {
            load();
            advance(ch + 1);
        }
        if constexpr (MF) {
            // lane: A row (lane & 15), B real column (lane & 15) of its block,
            // real inner index lane >> 4 = 2 (complex inner) + kpart
#pragma unroll
            for (int ks = 0; ks < BK / 2; ++ks) {
                const int p = 2 * ks + (lane >> 5);
                double a[WR], b[WC];
#pragma unroll
                for (int i = 0; i < WR; ++i)
                    a[i] = reinterpret_cast<const double*>(&As[p][wr0 + 16 * i + (lane & 15)])[kpart];
#pragma unroll
                for (int j = 0; j < WC; ++j) {
                    const double v =
                        reinterpret_cast<const double*>(&Bs[p][wc0 + 8 * j + ((lane & 15) >> 1)])[tcol ^ kpart];
                    b[j] = (kpart && !tcol) ? -v : v;
                }
#pragma unroll
                for (int i = 0; i < WR; ++i)
#pragma unroll
                    for (int j = 0; j < WC; ++j)
                        acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], b[j], acc[i][j], 0, 0, 0);
            }
        } else {
#pragma unroll
            for (int p = 0; p < BK; ++p) {
                double2 a[TT], b[TT];
#pragma unroll
                for (int i = 0; i < TT; ++i) a[i] = As[p][ty + 16 * i];
#pragma unroll
                for (int j = 0; j < TT; ++j) b[j] = Bs[p][tx + 16 * j];
#pragma unroll
                for (int i = 0; i < TT; ++i)
#pragma unroll
                    for (int j = 0; j < TT; ++j) {
                        accr[i][j] += a[i].x * b[j].x - a[i].y * b[j].y;
                        acci[i][j] += a[i].x * b[j].y + a[i].y * b[j].x;
                    }
            }
        }
        // the other buffer was last read before the previous barrier
        if (ch + 1 < c_end) stash(buf ^ 1);
        __syncthreads();
    }
    // split inner sum: this block's part goes to its row-major [BM][BN] partial
    // tile (padding skipped), added to the others' by k_split_reduce
    const bool to_partial = J.ksplit > 1;
    TN_GLOBAL double2* __restrict__ O =
        to_partial ? gstore<double2>(J.partial) + ((int64_t)T.pair * J.ksplit + T.kpart) * (BM * BN) : C;
    if constexpr (MF) {
        // element e of a lane's result is row (lane >> 4) + 4 e of its
        // instruction's block (the FP64 instruction interleaves its rows, unlike
        // the FP32 one), real column lane & 15: complex column (lane & 15) / 2,
        // component tcol
        TN_GLOBAL double* __restrict__ Od = reinterpret_cast<TN_GLOBAL double*>(O);
#pragma unroll
        for (int j = 0; j < WC; ++j) {
            const int col = wc0 + 8 * j + ((lane & 15) >> 1);
            const int64_t cc = col_c[col];
            if (cc < 0) continue;
#pragma unroll
            for (int i = 0; i < WR; ++i)
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int row = wr0 + 16 * i + (lane >> 4) + 4 * e;
                    const int64_t rc = row_c[row];
                    if (rc >= 0)
                        Od[2 * (to_partial ? (int64_t)row * BN + col : rc + cc) + tcol] = acc[i][j][e];
                }
        }
        return;
    }
#pragma unroll
    for (int i = 0; i < TT; ++i) {
        const int row = ty + 16 * i;
        const int64_t rc = row_c[row];
        if (rc < 0) continue;
#pragma unroll
        for (int j = 0; j < TT; ++j) {
            const int col = tx + 16 * j;
            const int64_t cc = col_c[col];
            if (cc >= 0) gst(O + (to_partial ? (int64_t)row * BN + col : rc + cc), make_double2(accr[i][j], acci[i][j]));
        }
    }
}

void launch_tile64_group(int tile, const MfmaJob* d_jobs, const MfmaTile* d_tiles, int64_t n_tiles,
                         hipStream_t s) {
    if (n_tiles == 0) return;
    if (tile == 4)
        launch_k(k_tile64_group<2, TILE64_MFMA>, dim3((unsigned)n_tiles), dim3(256), s, d_jobs, d_tiles);
    else
        launch_k(k_tile64_group<4, TILE64_MFMA>, dim3((unsigned)n_tiles), dim3(256), s, d_jobs, d_tiles);
}

// ---------------------------------------------------------------------------
// Split inner sums: the S blocks of a tile group each wrote one partial tile;
// this launch (same job and tile lists, after the tile launch on the same
// stream, so the partials are complete and visible) adds them in part order
// 0, 1, ..., S-1 and writes C.  Block b takes rows [kpart BM / S, (kpart + 1)
// BM / S) of its group's tile; tiles of unsplit jobs return at once.
// ---------------------------------------------------------------------------
template <typename C2>
__global__ __launch_bounds__(256) void k_split_reduce(const MfmaJob* __restrict__ jobs,
                                                      const MfmaTile* __restrict__ tiles, int bm_log,
                                                      int bn_log) {
    __shared__ int64_t rc_s[128], cc_s[64];
    __shared__ double red_r[256], red_i[256];
    const MfmaTile T = tiles[blockIdx.x];
    const MfmaJob& J = jobs[T.job];
    const int S = J.ksplit;
    if (S <= 1) return;
    const int BM = 1 << bm_log, BN = 1 << bn_log;
    if (S > BM) {
        // more parts than tile rows (very long inner sums): block kpart takes
        // elements [kpart E, (kpart + 1) E) of the row-major tile, E = BM BN / S,
        // its threads add strided subsets of the S partials in FP64 and a fixed
        // tree combines them (deterministic)
        const int64_t E = ((int64_t)BM * BN) / S;
        const int64_t PT = (int64_t)BM * BN;
        const TN_GLOBAL C2* __restrict__ P = gload<C2>(J.partial) + (int64_t)T.pair * S * PT;
        TN_GLOBAL C2* __restrict__ C = gstore<C2>(J.C);
        for (int64_t e = 0; e < E; ++e) {
            const int64_t o = (int64_t)T.kpart * E + e;
            const int i = (int)(o >> bn_log), j = (int)(o & (BN - 1));
            double sr = 0.0, si = 0.0;
            for (int q = threadIdx.x; q < S; q += 256) {
                const C2 v = gld(P + ((int64_t)q * PT + o));
                sr += (double)v.x;
                si += (double)v.y;
            }
            red_r[threadIdx.x] = sr;
            red_i[threadIdx.x] = si;
            __syncthreads();
            for (int w = 128; w > 0; w >>= 1) {
                if ((int)threadIdx.x < w) {
                    red_r[threadIdx.x] += red_r[threadIdx.x + w];
                    red_i[threadIdx.x] += red_i[threadIdx.x + w];
                }
                __syncthreads();
            }
            if (threadIdx.x == 0) {
                const int64_t rc = tile_out_row(J, T, i), cc = tile_out_col(J, T, j);
                if (rc >= 0 && cc >= 0) {
                    C2 t;
                    t.x = red_r[0];
                    t.y = red_i[0];
                    gst(C + (rc + cc), t);
                }
            }
            __syncthreads();
        }
        return;
    }
    const int rows = BM / S, r0 = T.kpart * rows;
    for (int i = threadIdx.x; i < rows; i += 256) rc_s[i] = tile_out_row(J, T, r0 + i);
    for (int j = threadIdx.x; j < BN; j += 256) cc_s[j] = tile_out_col(J, T, j);
    __syncthreads();
    const TN_GLOBAL C2* __restrict__ P = gload<C2>(J.partial) + (int64_t)T.pair * S * (BM * BN);
    TN_GLOBAL C2* __restrict__ C = gstore<C2>(J.C);
    const int64_t PT = (int64_t)BM * BN;
    for (int e = threadIdx.x; e < rows * BN; e += 256) {
        const int i = e >> bn_log, j = e & (BN - 1);
        const int64_t rc = rc_s[i], cc = cc_s[j];
        if (rc < 0 || cc < 0) continue;
        const int64_t o = (int64_t)(r0 + i) * BN + j;
        C2 t = gld(P + o);
        for (int q = 1; q < S; ++q) {
            const C2 v = gld(P + (q * PT + o));
            t.x += v.x;
            t.y += v.y;
        }
        gst(C + (rc + cc), t);
    }
}

void launch_split_reduce(int fp64, int tile, const MfmaJob* d_jobs, const MfmaTile* d_tiles, int64_t n_tiles,
                         hipStream_t s) {
    if (n_tiles == 0) return;
    const int bm_log = __builtin_ctz(mfma_tile_bm(tile)), bn_log = __builtin_ctz(mfma_tile_bn(tile));
    if (fp64)
        launch_k(k_split_reduce<double2>, dim3((unsigned)n_tiles), dim3(256), s, d_jobs, d_tiles, bm_log, bn_log);
    else
        launch_k(k_split_reduce<float2>, dim3((unsigned)n_tiles), dim3(256), s, d_jobs, d_tiles, bm_log, bn_log);
}

// ---------------------------------------------------------------------------
// K2: batched bit permutation, staged through LDS.  A tile covers the lowest
// bits of both the input and the output index (up to 10 bits), so loads run
// along the input's fastest legs and stores along the output's.  The offsets
// inside a tile come from a precomputed table (staged in LDS once per block);
// the remaining (high) bits select the tile, whose base is computed once.
// A block moves kPermElems elements (several tiles when tiles are small).
// Consecutive load slots are consecutive input addresses and consecutive
// store slots consecutive output addresses, so when the tile has at least two
// low bits each thread moves element pairs (16 B for complex64).
// ---------------------------------------------------------------------------
// elements per block: 16 KB of tile data (2048 complex64; the best of a sweep
// over 2^9..2^12 on 2^22-element tensors); at most 256 tiles per block, so the
// whole LDS use (tiles, 12 KB table, bases) stays under 32 KB
template <typename T>
__host__ __device__ constexpr int perm_elems() { return 16384 / (int)sizeof(T); }
__host__ __device__ inline int perm_tiles_per_block(int tsize, int elems) {
    const int u = tsize >= elems ? 1 : elems / tsize;
    return u > 256 ? 256 : u;
}

template <typename T>
__host__ __device__ inline int perm_block_elems(const PermArgs& p) {
    return p.elems_log > 0 ? (1 << p.elems_log) : perm_elems<T>();
}

template <typename T>
__global__ __launch_bounds__(256) void k_permute(PermArgs p) {
    extern __shared__ unsigned char smem_raw[];
    const int tsize = 1 << p.tb;
    const int upb = perm_tiles_per_block(tsize, perm_block_elems<T>(p));  // tiles per block
    // tile elements, one padding element after every 32 (transposes write the
    // tile with a stride of 32 elements)
    T* tile = (T*)smem_raw;                                          // upb * tsize * 33 / 32 elements
    int32_t* tab = (int32_t*)(tile + (int64_t)upb * tsize + ((int64_t)upb * tsize >> 5));  // 3 * tsize
    int64_t* in_base = (int64_t*)(tab + ((3 * tsize + 1) & ~1));     // upb (8-byte aligned)
    int64_t* out_base = in_base + upb;                               // upb
    const int64_t highs = int64_t(1) << p.n_high;
    const int64_t units = p.n_inst * highs;
    const int64_t unit0 = (int64_t)blockIdx.x * upb;
    const int64_t size = int64_t(1) << p.r;
    for (int i = threadIdx.x; i < 3 * tsize; i += blockDim.x) tab[i] = p.table[i];
    for (int u = threadIdx.x; u < upb; u += blockDim.x) {
        const int64_t unit = unit0 + u;
        int64_t ib = 0, ob = 0;
        if (unit < units) {
            const int64_t inst = unit >> p.n_high;
            const int64_t h = unit & (highs - 1);
            for (int i = 0; i < p.n_high; ++i)
                if ((h >> i) & 1) {
                    ib |= int64_t(1) << p.high_in[i];
                    ob |= int64_t(1) << p.high_out[i];
                }
            ib += inst * size;
            ob += inst * size;
        }
        in_base[u] = unit < units ? ib : -1;
        out_base[u] = ob;
    }
    __syncthreads();
    const int32_t* ld_in = tab;
    const int32_t* ld_pos = tab + tsize;
    const int32_t* st_out = tab + 2 * tsize;
    const int total = upb * tsize;
    const T* __restrict__ src = (const T*)p.src;
    T* __restrict__ dst = (T*)p.dst;
    if (p.pair) {
        for (int e2 = threadIdx.x; e2 < total / 2; e2 += blockDim.x) {
            const int e = 2 * e2;
            const int u = e >> p.tb, l = e & (tsize - 1);
            if (in_base[u] < 0) continue;
            const T* s2 = src + in_base[u] + ld_in[l];
            const T a = s2[0], b = s2[1];
            const int t0 = u * tsize + ld_pos[l], t1 = u * tsize + ld_pos[l + 1];
            tile[t0 + (t0 >> 5)] = a;
            tile[t1 + (t1 >> 5)] = b;
        }
    } else {
        for (int e = threadIdx.x; e < total; e += blockDim.x) {
            const int u = e >> p.tb, l = e & (tsize - 1);
            if (in_base[u] < 0) continue;
            const int t0 = u * tsize + ld_pos[l];
            tile[t0 + (t0 >> 5)] = src[in_base[u] + ld_in[l]];
        }
    }
    __syncthreads();
    if (p.pair) {
        for (int e2 = threadIdx.x; e2 < total / 2; e2 += blockDim.x) {
            const int e = 2 * e2;
            const int u = e >> p.tb, l = e & (tsize - 1);
            if (in_base[u] < 0) continue;
            T* d2 = dst + out_base[u] + st_out[l];
            const int t0 = u * tsize + l;
            d2[0] = tile[t0 + (t0 >> 5)];
            d2[1] = tile[t0 + 1 + ((t0 + 1) >> 5)];
        }
    } else {
        for (int e = threadIdx.x; e < total; e += blockDim.x) {
            const int u = e >> p.tb, l = e & (tsize - 1);
            if (in_base[u] < 0) continue;
            const int t0 = u * tsize + l;
            dst[out_base[u] + st_out[l]] = tile[t0 + (t0 >> 5)];
        }
    }
}

// ---------------------------------------------------------------------------
// K3: per-term finalize (FP64): amplitude = scalar * prod of cluster values,
// X = w |amplitude|^2 (a doubled network's value is the amplitude itself:
// X = w Re(amplitude)).
// ---------------------------------------------------------------------------
// ---------------------------------------------------------------------------
// K4: Neumaier-compensated level sums in a fixed order (deterministic): each
// thread sums a fixed strided subset, then pairs (sum, comp) are combined in a
// fixed tree.  One block per level.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void neumaier_add(double& s, double& c, double x) {
    const double t = s + x;
    if (fabs(s) >= fabs(x)) c += (s - t) + x;
    else c += (x - t) + s;
    s = t;
}

// (sum, comp) pairs of a block's threads combined in a fixed tree (NT threads,
// NT a power of two); thread 0 gets the block's pair.
template <int NT>
__device__ __forceinline__ void neumaier_block(double& s, double& c, double* ss, double* cc) {
    ss[threadIdx.x] = s;
    cc[threadIdx.x] = c;
    __syncthreads();
    for (int w = NT / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            double s1 = ss[threadIdx.x], c1 = cc[threadIdx.x] + cc[threadIdx.x + w];
            neumaier_add(s1, c1, ss[threadIdx.x + w]);
            ss[threadIdx.x] = s1;
            cc[threadIdx.x] = c1;
        }
        __syncthreads();
    }
    s = ss[0];
    c = cc[0];
    __syncthreads();
}

// The same with wave shuffles (a fixed butterfly within each wave of 64 lanes),
// then the waves' pairs added by thread 0 in wave order: one barrier.  Only
// thread 0's pair is the block's.
template <int NT>
__device__ __forceinline__ void neumaier_block_shfl(double& s, double& c, double* ss, double* cc) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        const double s2 = __shfl_xor(s, off), c2 = __shfl_xor(c, off);
        c += c2;
        neumaier_add(s, c, s2);
    }
    const int w = (int)threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        ss[w] = s;
        cc[w] = c;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double S = ss[0], C = cc[0];
        for (int q = 1; q < NT / 64; ++q) {
            C += cc[q];
            neumaier_add(S, C, ss[q]);
        }
        s = S;
        c = C;
    }
    __syncthreads();
}

// Thread t adds elements b + t, b + t + 256, ... of [b, e) in that order; the
// loads of 8 elements are issued before their adds (the adds form a chain).
__device__ __forceinline__ void level_sum_block(const double* x, const int64_t* starts, double* out, int u) {
    __shared__ double ss[256];
    __shared__ double cc[256];
    const int64_t b = starts[u], e = starts[u + 1];
    double s = 0.0, c = 0.0;
    constexpr int U = 8;
    for (int64_t i0 = b + threadIdx.x; i0 < e; i0 += 256 * U) {
        double v[U];
#pragma unroll
        for (int q = 0; q < U; ++q) {
            const int64_t i = i0 + (int64_t)q * 256;
            v[q] = i < e ? x[i] : 0.0;
        }
#pragma unroll
        for (int q = 0; q < U; ++q)
            if (i0 + (int64_t)q * 256 < e) neumaier_add(s, c, v[q]);
    }
    neumaier_block<256>(s, c, ss, cc);
    if (threadIdx.x == 0) {
        out[2 * u] = s + c;
        out[2 * u + 1] = c;
    }
}

__global__ __launch_bounds__(256) void k_level_sum(const double* x, const int64_t* starts, double* out) {
    level_sum_block(x, starts, out, blockIdx.x);
}

// The tail of all packed circuits in two launches.  k_tail_terms: block b
// finalizes terms 256 (b - block0) ... of its circuit (X_t = w |a_t|^2 and a_t
// written to the per-term outputs) and writes, for every level u, the
// Neumaier pair of its terms of
// level u (a fixed tree over the block's lanes) to part[b][u].
// k_tail_sums: block (circuit, u) adds the circuit's block pairs of level u in
// block order (strided per lane, then a fixed tree): deterministic.
__device__ __forceinline__ int tail_job_of(const TailJob* __restrict__ jobs, int n_jobs, int64_t b) {
    int lo = 0, hi = n_jobs - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (jobs[mid].block0 <= b) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// Finalize of one block of 256 terms (FP64): amplitude = scalar * prod of the
// term's cluster values in cluster order, X = w |amplitude|^2 (a doubled
// network's value is the amplitude itself: X = w Re(amplitude)).  The term
// `zero_term` takes its cluster values from the FP64 roots, and its product
// over the FP32 roots goes to the results as a diagnostic.  The clusters' root
// addresses are staged in LDS (kFinPtrs per round), and each thread loads
// kFinBatch cluster indices, then their values, before multiplying, so a term
// costs two dependent loads per batch.
constexpr int kFinBatch = 8;
constexpr int kFinPtrs = 64;

__global__ __launch_bounds__(256) void k_tail_terms(const TailJob* __restrict__ jobs, int n_jobs,
                                                    double* __restrict__ part, int64_t res_shift) {
    __shared__ double ss[256];
    __shared__ double cc[256];
    __shared__ const TN_GLOBAL float2* rp32[kFinPtrs];
    __shared__ const TN_GLOBAL double2* rp64[kFinPtrs];
    const int64_t b = blockIdx.x;
    const TailJob& J = jobs[tail_job_of(jobs, n_jobs, b)];
    const FinalizeArgs& f = J.f;
    const int64_t t0 = (b - J.block0) * 256;
    const int64_t t = t0 + threadIdx.x;
    const bool in = t < f.n_terms;
    const int32_t li = in ? gload<int32_t>(f.live_index)[t] : -1;
    const bool hi = in && t == f.zero_term;
    const int ncl = f.n_clusters;
    const TN_GLOBAL int32_t* __restrict__ ri = gload<int32_t>(f.root_idx) + (int64_t)(li < 0 ? 0 : li) * ncl;
    double ar = f.scalar_re, ai = f.scalar_im;      // over the FP32 roots
    double hr = ar, hm = ai;                        // over the FP64 roots (zero_term)
    for (int c0 = 0; c0 < ncl; c0 += kFinPtrs) {
        const int nc = ncl - c0 < kFinPtrs ? ncl - c0 : kFinPtrs;
        __syncthreads();                            // the previous round's addresses are read
        if ((int)threadIdx.x < nc) {            // (FP64 addresses are 0 without the FP64 pass)
            const int64_t a32 = gload<int64_t>(f.root_ptrs)[c0 + threadIdx.x];
            const int64_t a64 = gload<int64_t>(f.root64_ptrs)[c0 + threadIdx.x];
            rp32[threadIdx.x] = gload<float2>((const void*)a32);
            rp64[threadIdx.x] = gload<double2>((const void*)a64);
        }
        __syncthreads();
        if (li < 0) continue;
        for (int q0 = 0; q0 < nc; q0 += kFinBatch) {
            int32_t j[kFinBatch];
            float2 v[kFinBatch];
            // loads past the round's last cluster repeat it (in bounds, not used):
            // unconditional loads are all issued before the first wait
#pragma unroll
            for (int q = 0; q < kFinBatch; ++q) j[q] = ri[c0 + (q0 + q < nc ? q0 + q : nc - 1)];
#pragma unroll
            for (int q = 0; q < kFinBatch; ++q) v[q] = gld(rp32[q0 + q < nc ? q0 + q : nc - 1] + j[q]);
#pragma unroll
            for (int q = 0; q < kFinBatch; ++q)
                if (q0 + q < nc) {
                    const double vr = (double)v[q].x, vi = (double)v[q].y;
                    const double nr = ar * vr - ai * vi;
                    const double ni = ar * vi + ai * vr;
                    ar = nr;
                    ai = ni;
                }
            if (hi) {
                double2 w[kFinBatch];
#pragma unroll
                for (int q = 0; q < kFinBatch; ++q) w[q] = gld(rp64[q0 + q < nc ? q0 + q : nc - 1] + j[q]);
#pragma unroll
                for (int q = 0; q < kFinBatch; ++q)
                    if (q0 + q < nc) {
                        const double nr = hr * w[q].x - hm * w[q].y;
                        const double ni = hr * w[q].y + hm * w[q].x;
                        hr = nr;
                        hm = ni;
                    }
            }
        }
    }
    double x = 0.0;
    if (in) {
        if (li < 0) {
            f.x_out[t] = 0.0;
            f.amp_out[2 * t] = 0.0f;
            f.amp_out[2 * t + 1] = 0.0f;
        } else {
            const double pr = hi ? hr : ar, pi = hi ? hm : ai;
            const double wt = f.w[t];
            x = wt * (f.re_value ? pr : pr * pr + pi * pi);
            f.x_out[t] = x;
            f.amp_out[2 * t] = (float)pr;
            f.amp_out[2 * t + 1] = (float)pi;
            if (hi && f.x0_fp32_out)
                *(double*)((char*)f.x0_fp32_out + res_shift) = wt * (f.re_value ? ar : ar * ar + ai * ai);
        }
    }
    const int64_t t_end = t0 + 256 < f.n_terms ? t0 + 256 : f.n_terms;
    double* out = part + b * (2 * (TN_MAX_LEVEL + 1));
    for (int u = 0; u < J.n_levels; ++u) {
        const int64_t lb = J.starts[u], le = J.starts[u + 1];
        if (le <= t0 || lb >= t_end) {           // no term of this block has level u
            if (threadIdx.x == 0) {
                out[2 * u] = 0.0;
                out[2 * u + 1] = 0.0;
            }
            continue;
        }
        double sv = (t >= lb && t < le) ? x : 0.0, cv = 0.0;
        neumaier_block_shfl<256>(sv, cv, ss, cc);
        if (threadIdx.x == 0) {
            out[2 * u] = sv;
            out[2 * u + 1] = cv;
        }
    }
}

__global__ __launch_bounds__(256) void k_tail_sums(const TailJob* __restrict__ jobs, const double* __restrict__ part,
                                                   int64_t res_shift) {
    __shared__ double ss[256];
    __shared__ double cc[256];
    const TailJob J = jobs[blockIdx.x];
    const int u = blockIdx.y;
    if (u >= J.n_levels) return;
    const int64_t nb = (J.f.n_terms + 255) / 256;
    double s = 0.0, c = 0.0;
    for (int64_t q = threadIdx.x; q < nb; q += 256) {
        const double* pr = part + (J.block0 + q) * (2 * (TN_MAX_LEVEL + 1)) + 2 * u;
        neumaier_add(s, c, pr[0]);
        c += pr[1];
    }
    neumaier_block_shfl<256>(s, c, ss, cc);
    if (threadIdx.x == 0) {
        double* sums = (double*)((char*)J.sums + res_shift);
        sums[2 * u] = s + c;
        sums[2 * u + 1] = c;
    }
}

__global__ void k_slot_fill(SlotFillArgs a) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= a.n * 8) return;
    const int leaf = i >> 3, w = i & 7;
    const int s = a.noise[leaf];
    const int choice = a.pattern[a.term * a.n_noise + s];
    ((float*)a.dst[leaf])[w] = a.bank[(s * 4 + choice) * 8 + w];
}

__global__ void k_copy_c64(const float2* src, float2* dst, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = src[i];
}

// ---------------------------------------------------------------------------
// launch wrappers
// ---------------------------------------------------------------------------
static inline unsigned grid1(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

struct TileCfg {
    int bm, bnc;
};
static const TileCfg kTiles[K_MFMA_TILES] = {{128, 64}, {64, 64}, {128, 32}, {64, 32},
                                               {32, 32}, {128, 16}, {64, 16}, {32, 16}};

bool mfma_tile_fits(int tile, const GemmArgs& g) {
    if (tile < 0 || tile >= K_MFMA_TILES) return false;
    if (g.m_log < 5 || (int64_t(1) << g.m_log) < kTiles[tile].bm) return false;
    // 16-column tiles also take n < 16 (zero-padded columns) when the GEMM is
    // long enough in m and k to be worth the matrix cores
    if (kTiles[tile].bnc == 16 && g.n_log < 4) return g.n_log >= 1 && g.m_log >= 7 && g.k_log >= 3;
    return (int64_t(1) << g.n_log) >= kTiles[tile].bnc;
}

int select_gemm(const GemmArgs& g, int fp64, int tile_hint) {
    const int mn_log = g.m_log + g.n_log;
    if (mn_log <= 4 && g.k_log >= 8) return fp64 ? K_SPLITK64 : K_SPLITK32;
    if (fp64) return (g.m_log >= 6 && g.n_log >= 6) ? K_TILED64 : K_SMALL64;
    if (mfma_tile_fits(tile_hint, g)) return tile_hint;
    for (int i = 0; i < K_MFMA_TILES; ++i)
        if (mfma_tile_fits(i, g)) return i;
    return K_SMALL32;
}

const char* kernel_name(int id) {
    static const char* mg[K_MFMA_TILES] = {"k_gemm_mfma_g<128,64>", "k_gemm_mfma_g<64,64>", "k_gemm_mfma_g<128,32>",
                                           "k_gemm_mfma_g<64,32>",  "k_gemm_mfma_g<32,32>", "k_gemm_mfma_g<128,16>",
                                           "k_gemm_mfma_g<64,16>",  "k_gemm_mfma_g<32,16>"};
    if (id >= K_GATHER_BASE && id < K_GATHER_BASE + K_MFMA_TILES) return mg[id - K_GATHER_BASE];
    static const char* mq[K_MFMA_TILES] = {"k_mfma_group<128,64>", "k_mfma_group<64,64>", "k_mfma_group<128,32>",
                                           "k_mfma_group<64,32>",  "k_mfma_group<32,32>", "k_mfma_group<128,16>",
                                           "k_mfma_group<64,16>",  "k_mfma_group<32,16>"};
    if (id >= K_MFMA_GROUP_BASE && id < K_MFMA_GROUP_BASE + K_MFMA_TILES) return mq[id - K_MFMA_GROUP_BASE];
    static const char* mf[K_MFMA_TILES] = {"k_gemm_mfma<128,64>", "k_gemm_mfma<64,64>", "k_gemm_mfma<128,32>",
                                           "k_gemm_mfma<64,32>",  "k_gemm_mfma<32,32>", "k_gemm_mfma<128,16>",
                                           "k_gemm_mfma<64,16>",  "k_gemm_mfma<32,16>"};
    if (id >= 0 && id < K_MFMA_TILES) return mf[id];
    switch (id) {
    case K_SMALL32: return "k_gemm_small<float>";
    case K_SPLITK32: return "k_gemm_splitk<float>";
    case K_SMALL64: return "k_gemm_small<double>";
    case K_SPLITK64: return "k_gemm_splitk<double>";
    case K_TILED64: return "k_gemm_tiled_c128";
    case K_PERM32: return "k_permute<float2>";
    case K_PERM64: return "k_permute<double2>";
    case K_GROUP32: return "k_gett_group<float>";
    case K_GROUP64: return "k_gett_group<double>";
    case K_GROUPMIX: return "k_gett_group<mixed>";
    case K_TILE64_GROUP: return "k_tile64_group";
    case K_SPLIT_REDUCE32: return "k_split_reduce<float>";
    case K_SPLIT_REDUCE64: return "k_split_reduce<double>";
    }
    return "unknown";
}

int kernel_class(int id) {
    if (id >= 0 && id < K_MFMA_TILES) return KC_MFMA;
    if (id >= K_GATHER_BASE && id < K_GATHER_BASE + K_MFMA_TILES) return KC_MFMA;
    if (id == K_SMALL32 || id == K_SMALL64) return KC_SMALL;
    if (id == K_SPLITK32 || id == K_SPLITK64) return KC_SPLITK;
    if (id == K_GROUP32 || id == K_GROUP64 || id == K_GROUPMIX || id == K_TILE64_GROUP ||
        id == K_SPLIT_REDUCE32 || id == K_SPLIT_REDUCE64)
        return KC_GROUP;
    if (id >= K_MFMA_GROUP_BASE && id < K_MFMA_GROUP_BASE + K_MFMA_TILES) return KC_GROUP;
    return KC_TILED;
}

int mfma_tile_bm(int tile) { return kTiles[tile].bm; }
int mfma_tile_bn(int tile) { return kTiles[tile].bnc; }

void launch_mfma_group(int tile, const MfmaJob* d_jobs, const MfmaTile* d_tiles, int64_t n_tiles,
                       hipStream_t s) {
    if (n_tiles == 0) return;
    const TileCfg& t = kTiles[tile];
#define TN_GLAUNCH(BM_, BN_)                                                                  \
    if (t.bm == BM_ && t.bnc == BN_) {                                                         \
        constexpr int nt = MfmaGroupShape<BM_, BN_>::NT;                                      \
        launch_k(k_mfma_group<BM_, BN_>, dim3((unsigned)n_tiles), dim3(nt), s, d_jobs, d_tiles);  \
        return;                                                                                \
    }
    TN_GLAUNCH(128, 64)
    TN_GLAUNCH(64, 64)
    TN_GLAUNCH(128, 32)
    TN_GLAUNCH(64, 32)
    TN_GLAUNCH(32, 32)
    TN_GLAUNCH(128, 16)
    TN_GLAUNCH(64, 16)
    TN_GLAUNCH(32, 16)
#undef TN_GLAUNCH
}

int64_t gett_job_blocks(const GettJob& j) {
    const int64_t outs = j.n_inst << (j.m_log + j.n_log);
    return j.split ? outs : ((outs >> j.rpt_log) + 255) / 256;
}

void launch_gett_group(const GettJob* d_jobs, const int32_t* d_block_job, int64_t blocks, hipStream_t s) {
    if (blocks == 0) return;
    launch_k(k_gett_group, dim3((unsigned)blocks), dim3(256), s, d_jobs, d_block_job);
}

static void launch_mfma_tile(const TileCfg& t, const GemmArgs& g, hipStream_t s, bool gather) {
    const int64_t ntiles = std::max<int64_t>(1, (int64_t(1) << g.n_log) / t.bnc);
    const int64_t tiles = ((int64_t(1) << g.m_log) / t.bm) * ntiles;
    const unsigned blocks = (unsigned)(tiles * g.n_inst);
#define TN_LAUNCH(BM_, BN_)                                                                   \
    if (t.bm == BM_ && t.bnc == BN_) {                                                         \
        constexpr int nt = 64 * (BM_ >= 64 ? BM_ / 64 : 1) * (BN_ >= 32 ? BN_ / 32 : 1);       \
        if (gather)                                                                            \
            hipLaunchKernelGGL((k_gemm_mfma_g<BM_, BN_>), dim3(blocks), dim3(nt), 0, s, g);    \
        else                                                                                   \
            hipLaunchKernelGGL((k_gemm_mfma<BM_, BN_>), dim3(blocks), dim3(nt), 0, s, g);      \
        return;                                                                                \
    }
    TN_LAUNCH(128, 64)
    TN_LAUNCH(64, 64)
    TN_LAUNCH(128, 32)
    TN_LAUNCH(64, 32)
    TN_LAUNCH(32, 32)
    TN_LAUNCH(128, 16)
    TN_LAUNCH(64, 16)
    TN_LAUNCH(32, 16)
#undef TN_LAUNCH
}

void launch_gemm_id(int id, const GemmArgs& g, hipStream_t s) {
    const int mn_log = g.m_log + g.n_log;
    const int64_t total = g.n_inst << mn_log;
    if (id >= 0 && id < K_MFMA_TILES) {
        launch_mfma_tile(kTiles[id], g, s, false);
        return;
    }
    if (id >= K_GATHER_BASE && id < K_GATHER_BASE + K_MFMA_TILES) {
        launch_mfma_tile(kTiles[id - K_GATHER_BASE], g, s, true);
        return;
    }
    switch (id) {
    case K_SMALL32:
        hipLaunchKernelGGL((k_gemm_small<float, float2>), dim3(grid1(total, 256)), dim3(256), 0, s, g);
        return;
    case K_SPLITK32:
        hipLaunchKernelGGL((k_gemm_splitk<float, float2>), dim3((unsigned)total), dim3(256), 0, s, g);
        return;
    case K_SMALL64:
        hipLaunchKernelGGL((k_gemm_small<double, double2>), dim3(grid1(total, 256)), dim3(256), 0, s, g);
        return;
    case K_SPLITK64:
        hipLaunchKernelGGL((k_gemm_splitk<double, double2>), dim3((unsigned)total), dim3(256), 0, s, g);
        return;
    case K_TILED64: {
        const int64_t tiles = (int64_t(1) << (g.m_log - 6)) << (g.n_log - 6);
        hipLaunchKernelGGL(k_gemm_tiled_c128, dim3((unsigned)(tiles * g.n_inst)), dim3(256), 0, s, g);
        return;
    }
    }
}

int launch_gemm_c64(const GemmArgs& g, hipStream_t s, int tile_hint) {
    const int id = select_gemm(g, 0, tile_hint);
    launch_gemm_id(id, g, s);
    return id;
}

int launch_gemm_c128(const GemmArgs& g, hipStream_t s) {
    const int id = select_gemm(g, 1, -1);
    launch_gemm_id(id, g, s);
    return id;
}

template <typename T>
static void launch_perm(const PermArgs& p, hipStream_t s) {
    const int tsize = 1 << p.tb;
    const int upb = perm_tiles_per_block(tsize, perm_block_elems<T>(p));
    const int64_t units = p.n_inst << p.n_high;
    const unsigned blocks = (unsigned)((units + upb - 1) / upb);
    const size_t elems = (size_t)upb * tsize;
    const size_t lds = (elems + (elems >> 5)) * sizeof(T) + ((3 * tsize + 1) & ~1) * sizeof(int32_t) +
                       2 * upb * sizeof(int64_t);
    hipLaunchKernelGGL((k_permute<T>), dim3(blocks), dim3(256), lds, s, p);
}

void launch_permute_c64(const PermArgs& p, hipStream_t s) { launch_perm<float2>(p, s); }
void launch_permute_c128(const PermArgs& p, hipStream_t s) { launch_perm<double2>(p, s); }

void launch_level_sum(const double* x, const int64_t* starts, int n_levels, double* out,
                      hipStream_t s) {
    hipLaunchKernelGGL(k_level_sum, dim3(n_levels), dim3(256), 0, s, x, starts, out);
}

void launch_tail(const TailJob* d_jobs, int n_jobs, int64_t blocks, int max_levels, double* d_part,
                 int64_t res_shift, hipStream_t s) {
    if (n_jobs == 0) return;
    if (blocks > 0)
        hipLaunchKernelGGL(k_tail_terms, dim3((unsigned)blocks), dim3(256), 0, s, d_jobs, n_jobs, d_part, res_shift);
    hipLaunchKernelGGL(k_tail_sums, dim3((unsigned)n_jobs, (unsigned)max_levels), dim3(256), 0, s, d_jobs,
                       (const double*)d_part, res_shift);
}

void launch_slot_fill(const SlotFillArgs& a, hipStream_t s) {
    if (a.n == 0) return;
    hipLaunchKernelGGL(k_slot_fill, dim3(grid1(a.n * 8, 256)), dim3(256), 0, s, a);
}

void launch_copy_c64(const void* src, void* dst, int64_t n, hipStream_t s) {
    if (n == 0) return;
    hipLaunchKernelGGL(k_copy_c64, dim3(grid1(n, 256)), dim3(256), 0, s, (const float2*)src,
                       (float2*)dst, n);
}

}  // namespace tn
