/*
 * tn.h -- C ABI of the MI355X term-network contractor for the SVD-based
 * approximate noisy-circuit simulation (arXiv 2211.17028).
 *
 * Problem (Section III, Problem 1): given a noisy circuit E = E_d o ... o E_1
 * of gates and single-qubit noise channels, an input product state |psi> and a
 * target state |v>, estimate <v| E(|psi><psi|) |v>.
 *
 * Method (Section IV, Algorithm 1): every noise superoperator
 * M = sum_k E_k (x) conj(E_k) is permuted (Fig. 3a) and split by SVD into
 * M = sum_{i=0..3} U_i (x) V_i (Fig. 3b-c).  The level-l approximation is
 * A(l) = sum_{u<=l} T_u, where T_u sums, over all choices of u noises and of
 * one correction i in {1,2,3} at each, the value X of the network in which
 * those noises carry U_i (x) V_i and all others U_0 (x) V_0.  Each X is a
 * product of a ket network and a bra network; for a channel the bra network is
 * the conjugate of the ket network, so X = w |a|^2 with a one ket-network
 * amplitude and w >= 0 a product of singular values.
 *
 * Conventions
 *   - Complex inputs are tn_c128 (two doubles).  Matrices are row-major.
 *   - A 2-qubit gate on (q0, q1) is 4x4 in the basis |b_q0 b_q1>, b_q0 the more
 *     significant bit.  A dense n-qubit state has qubit 0 as the most
 *     significant bit of its index.
 *   - A noise acts on one qubit, right after the op before it in the list.
 *   - Device pointers are HIP device addresses; `stream` is a hipStream_t
 *     passed as void* (NULL = the null stream).
 *
 * Errors: every int-returning call returns TN_OK (0) or a negative TN_E*
 * code; tn_last_error() then holds a message (thread-local, valid until the
 * next tn_* call on the same thread).  No C++ exception crosses this ABI.
 *
 * Ownership: the caller owns every input it passes (the library copies what
 * it keeps during the call), all device memory (inputs, outputs and the
 * workspace) and the result structs.  The library owns tn_plan, tn_terms and
 * tn_exec handles until the matching *_destroy call.
 */
#ifndef TN_H
#define TN_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    TN_OK = 0,
    TN_EINVAL = -1,        /* malformed argument, non-unitary gate, bad qubit index */
    TN_ENOTCPTP = -2,      /* Kraus set not trace preserving: ||sum E^+E - I|| > 1e-10 */
    TN_EUNSUPPORTED = -3,  /* noise on more than one qubit, gate on more than two */
    TN_EDEGENERATE = -4,   /* dominant singular value not strictly largest */
    TN_ENOMEM = -5,        /* workspace smaller than required */
    TN_EHIP = -6,          /* a HIP runtime call failed (message has the HIP string) */
    TN_ETOOBIG = -7,       /* plan exceeds a hard limit (slots per network, tensor rank) */
    TN_ESTATE = -8         /* call out of order (e.g. terms of another plan) */
};

typedef struct { double re, im; } tn_c128;

enum { TN_GATE = 0, TN_NOISE = 1 };

typedef struct {
    int32_t kind;          /* TN_GATE or TN_NOISE */
    int32_t nq;            /* gate: 1 or 2; noise: 1 */
    int32_t q[2];          /* qubit indices (q[1] unused when nq == 1) */
    int32_t n_kraus;       /* noise: number of 2x2 Kraus matrices (>= 1) */
    const tn_c128* mat;    /* gate: (2^nq)^2 entries; noise: n_kraus * 4 entries */
} tn_op;

typedef struct {
    int32_t n_qubits;
    int64_t n_ops;
    const tn_op* ops;      /* in time order */
} tn_circuit;

enum {
    TN_STATE_PRODUCT = 0,         /* data: n_qubits x 2 amplitudes */
    TN_STATE_CIRCUIT_OUTPUT = 1,  /* |v> = U_ideal |p>, data: n_qubits x 2 of |p>;
                                     U_ideal is the circuit with its noises removed */
    TN_STATE_DENSE = 2,           /* data: 2^n_qubits amplitudes (n_qubits <= 30) */
    /* bond-2 targets |v> = |p> + c |q> with p, q product states: the targets of
     * the polarization identity for off-diagonal elements (Section III, after
     * Problem 1).  data: n_qubits x 2 of |p>, then n_qubits x 2 of |q>, then c
     * (4 n_qubits + 1 entries).  In the network <v| is one 2-valued index shared
     * by a tensor per qubit and the branch weights (1, conj c). */
    TN_STATE_SUM2 = 3,
    TN_STATE_CIRCUIT_OUTPUT_SUM2 = 4  /* |v> = U_ideal (|p> + c |q>), data as TN_STATE_SUM2;
                                         reduced by the light cone like TN_STATE_CIRCUIT_OUTPUT */
};

typedef struct {
    int32_t kind;
    const tn_c128* data;
} tn_state;

typedef struct tn_plan_s* tn_plan;
typedef struct tn_terms_s* tn_terms;
typedef struct tn_exec_s* tn_exec;

#define TN_MAX_LEVEL 8

/* Planner options; zero-initialise for defaults. */
typedef struct {
    int32_t path_trials;    /* randomized greedy path trials per network (0 = 1024; 8192 for
                               the estimate of a bond-2 target) */
    uint64_t seed;          /* path search seed (0 = fixed default) */
    int32_t no_light_cone;  /* 1 = keep gates outside the slots' light cone */
    int32_t max_log_size;   /* cap on log2(elements) of one tensor (0 = 30) */
    int32_t no_diagonal_hyperedges;  /* 1 = give diagonal gates their own output legs
                                        instead of sharing their wires' index */
    double max_work_bytes;  /* cap on the complex64 live set of one cluster's path,
                               all instances of the full level-l expansion (0 = 64 GiB) */
    int32_t no_reconfigure; /* 1 = keep the best greedy path as found (no subtree
                               reconfiguration by dynamic programming) */
} tn_plan_opts;

/* Term pruning (level-2/3 candidates).  NULL = the full expansion. */
typedef struct {
    int32_t min_level;         /* only terms of level >= min_level are candidates */
    const uint8_t* keep;       /* n_candidates flags (1 = keep), in enumeration order
                                  of the candidates; NULL = keep all */
    int64_t n_keep;            /* length of keep */
} tn_prune_opts;

enum { TN_MODE_BATCHED = 0, TN_MODE_PLAIN = 1 };

typedef struct {
    int32_t mode;            /* TN_MODE_BATCHED or TN_MODE_PLAIN */
    int32_t use_graph;       /* batched: 1 = capture the step sequence in a hipGraph and
                                replay it; 0 = direct launches, the FP64 pass issued on
                                its side stream by a host thread the exec owns (started
                                at the first run, joined by tn_exec_destroy) */
    int32_t fp64_level0;     /* 1 = recompute the all-dominant term in FP64
                                (tn_estimate always does) */
    int32_t tune;            /* 1 = pick tiles by timing at prepare (autotuner): per-step
                                launches (no_group) time each step's GEMM tiles; grouped
                                launches of one plan: per FP32 tree level with tile
                                launches, whole estimates with the model's choice are
                                timed on the workspace against estimates with each tile
                                shape imposed on the whole level, and a shape is kept only
                                when it is over 3 % faster; choices are cached per level
                                signature for the process */
    int32_t time_kernels;    /* 1 = HIP events around every batched launch, recorded by
                                the dispatch itself (hipExtLaunchKernelGGL) so they bracket
                                the kernel and not the queue, accumulated per kernel
                                (tn_exec_kernel_stats); needs use_graph = 0 (TN_EINVAL
                                otherwise) */
    int32_t no_gather;       /* 1 = always transpose operands into GEMM order instead of
                                letting MFMA steps read them in stored order */
    int32_t no_group;        /* 1 = one launch per contraction step instead of one grouped
                                launch for the small steps of each tree level */
    int32_t max_ksplit;      /* largest number of blocks one tile's inner sum is split
                                over (0 = default 16, 1 = no split, at most 32) */
    int32_t mixed_shapes;    /* 1 = every matrix-core job keeps its own best tile shape;
                                0 = with one plan, jobs with at most a quarter of the flops
                                of their tree level's main tile shape take that shape and
                                join its launch */
    int32_t all_tiles;       /* 1 = matrix-core steps keep their tile launches at every tree
                                level; 0 = a FP32 level with under 32 MFLOP of work runs all
                                its steps in its one small-step launch */
} tn_exec_opts;

/* Accumulated per-kernel timing of the runs since the last reset (needs
 * time_kernels).  flops / bytes are the algorithmic work of those launches
 * (8 real flops per complex MAC; operand + result bytes; permute: read +
 * write). */
typedef struct {
    char name[48];
    int64_t launches;
    double ms;
    double flops;
    double bytes;
} tn_kernel_stat;

/* Per-circuit result of an estimate (host struct, filled by the library). */
typedef struct {
    int32_t level;                        /* effective level (clamped to N) */
    int32_t clamped;                      /* 1 if the requested level exceeded N */
    int64_t n_terms;                      /* terms in the term set */
    int64_t n_contracted;                 /* terms with non-zero weight */
    int64_t n_zero_weight;                /* terms skipped: some d_i is exactly 0 */
    double level_sum[TN_MAX_LEVEL + 1];   /* T_u, u = 0..level (compensated) */
    double level_comp[TN_MAX_LEVEL + 1];  /* Neumaier compensation of T_u (already added) */
    double A[TN_MAX_LEVEL + 1];           /* A(u) = sum_{u'<=u} T_u' */
    double bound;                         /* |F - A(level)| bound from the split norms */
    double x0_fp32;                       /* level-0 term from the FP32 batch (diagnostic);
                                             -1 in PLAIN mode and when the FP64 pass is the
                                             only one (a single live term, the level-0 one,
                                             with fp64_level0: no FP32 chain is scheduled) */
} tn_result;

/* ---------------------------------------------------------------------------
 * tn_plan_build -- validate the circuit, split every noise, build the ket
 * network of one term (all terms share its topology), reduce it by the slots'
 * light cone when the target is the circuit output, split it into independent
 * clusters, and choose a contraction path per cluster.  Host only.
 *
 *   circ   circuit (gates and 1-qubit noises, time order)
 *   psi    input state, TN_STATE_PRODUCT only
 *   v      target state (any TN_STATE_* kind)
 *   level  requested level l >= 0 (clamped to N; flagged in the result)
 *   opts   planner options or NULL
 *   out    receives the plan handle
 *
 * Errors: TN_EINVAL (bad indices, non-unitary gate: ||G^+G - I||_max > 1e-10),
 * TN_ENOTCPTP (Section II trace condition), TN_EUNSUPPORTED (multi-qubit
 * noise; the split of Section IV is defined on 4x4 superoperators),
 * TN_EDEGENERATE (d_1 >= (1 - 1e-12) d_0), TN_ETOOBIG (a cluster with more than
 * 64 slots, a path tensor above max_log_size, or a live set above max_work_bytes).
 * ------------------------------------------------------------------------- */
int tn_plan_build(const tn_circuit* circ, const tn_state* psi, const tn_state* v,
                  int32_t level, const tn_plan_opts* opts, tn_plan* out);

/* ---------------------------------------------------------------------------
 * tn_plan_build_doubled -- the exact value <v| E(|psi><psi|) |v> as one
 * network: the paper's exact baseline (the doubled network of Section IV,
 * Fig. 2), in which every noise is its full superoperator
 * M = sum_k E_k (x) conj(E_k) (Section III) joining the ket and bra halves.
 * Built from the same reduced ket network as tn_plan_build (the bra half is
 * its complex conjugate), with each noise slot pair replaced by the 4-leg
 * tensor T[ko][ki][bo][bi] = sum_k E_k[ko][ki] conj(E_k[bo][bi]).  No noise is
 * split, so a degenerate channel is accepted.  Host only.
 *
 * The plan has no slots: tn_terms_enumerate (any level) gives one term of
 * weight 1, and an estimate over it reports the exact value as level_sum[0] =
 * A[0] with bound 0 (computed in FP64 when fp64_level0 is set, which
 * tn_estimate always does; in FP32 otherwise).  The doubled network's tensors
 * are about the square of the ket network's, so max_log_size and
 * max_work_bytes decide which circuits fit.
 *
 * Arguments as tn_plan_build (no level).  Errors: TN_EINVAL, TN_ENOTCPTP,
 * TN_EUNSUPPORTED, TN_ETOOBIG as tn_plan_build.
 * ------------------------------------------------------------------------- */
int tn_plan_build_doubled(const tn_circuit* circ, const tn_state* psi, const tn_state* v,
                          const tn_plan_opts* opts, tn_plan* out);

/* ---------------------------------------------------------------------------
 * tn_terms_enumerate -- the term set of Algorithm 1 at level `level`:
 * u = 0..level; noise subsets p_1 < ... < p_u in lexicographic order; the
 * corrections (i_1..i_u) in {1,2,3}^u in lexicographic order.  Count:
 * sum_{u<=l} C(N,u) 3^u (Theorem 1).  Terms whose weight is exactly zero (some
 * chosen d_i == 0, e.g. the fourth singular value of a rank-3 channel) stay in
 * the set, flagged, and are never contracted.  `prune` may drop candidates of
 * level >= prune->min_level.  Host only.
 * ------------------------------------------------------------------------- */
int tn_terms_enumerate(tn_plan plan, int32_t level, const tn_prune_opts* prune,
                       tn_terms* out, int64_t* n_terms);

/* Copy the term set out: patterns (n_terms x N int8, entry = correction index
 * 0..3 per noise) and weights w_t = prod_s d_{c_s} (float64).  Either pointer may
 * be NULL.  Host only. */
int tn_terms_get(tn_terms terms, int8_t* patterns, double* weights);

/* ---------------------------------------------------------------------------
 * tn_exec_prepare -- build the device schedule for n plans (each with its term
 * set) packed together: per path step the instance maps of the batch, the
 * static placement of every intermediate in the workspace, and the upload of
 * fixed tensors, slot tensors and maps.
 *
 *   ws_bytes == 0 : only report the size needed in *need_bytes (no device call);
 *                   if `out` is not NULL it receives an unbound handle usable by
 *                   tn_exec_describe / tn_exec_const_bytes / tn_exec_destroy only.
 *   otherwise d_ws must hold >= *need_bytes bytes (else TN_ENOMEM); the upload
 *   is enqueued on `stream` and *out receives an executable handle bound to
 *   d_ws (the caller keeps d_ws alive and unmodified until tn_exec_destroy).
 *   With opts->tune = 1 the query reports the largest workspace of the
 *   schedules the autotuner times; a smaller d_ws that still holds the untuned
 *   schedule (the query with tune = 0) is accepted, and the autotuner then
 *   times only the candidates that fit in it.
 *   opts == NULL: batched, direct launches, FP64 dominant-term pass, every
 *   other field 0.
 * ------------------------------------------------------------------------- */
int tn_exec_prepare(int32_t n, const tn_plan* plans, const tn_terms* terms,
                    const tn_exec_opts* opts, void* d_ws, size_t ws_bytes, void* stream,
                    size_t* need_bytes, tn_exec* out);

/* Run a prepared schedule on `stream` and synchronize it; fill one tn_result
 * per plan (results[n]). */
int tn_exec_run(tn_exec ex, void* stream, tn_result* results);

/* Pipelined estimates: tn_exec_submit issues one estimate on `stream` (as
 * tn_exec_run, without waiting) and returns its ticket; tn_exec_collect waits
 * for that estimate and fills `results` (NULL: only wait).  Consecutive
 * estimates on one stream run back to back on the GPU (they share the
 * workspace in stream order), so the host's result handling and the next
 * issue overlap the GPU work.  Each submitted estimate's results go into one of
 * two host slots (written there by the tail kernels with direct launches,
 * copied there after a graph replay): at most two may be outstanding
 * (TN_ESTATE for a third), tickets are collected once each in submission
 * order (TN_ESTATE otherwise), and tn_exec_run needs none outstanding.
 * Submitting needs time_kernels = 0 (TN_EINVAL).  The stream must stay the
 * same between a submit and its collect. */
int tn_exec_submit(tn_exec ex, void* stream, int64_t* ticket);
int tn_exec_collect(tn_exec ex, int64_t ticket, tn_result* results);

/* `count` estimates of a prepared schedule on `stream` in one call: issued back
 * to back with at most two in flight (as tn_exec_submit / tn_exec_collect), the
 * results of estimate i and packed plan p written to results[i * n + p] (host
 * array of count * n tn_result, caller-owned); returns when the last one has
 * finished.  Every estimate recomputes Algorithm 1's level sums from the
 * resident inputs (Section IV), as tn_exec_run does.  Needs no estimate
 * outstanding (TN_ESTATE) and time_kernels = 0 (TN_EINVAL); count < 0 or a null
 * results array with count > 0 is TN_EINVAL.  On an error nothing is left
 * outstanding. */
int tn_exec_run_many(tn_exec ex, void* stream, int64_t count, tn_result* results);

/* Device pointers to the per-term values X_t (float64) and the per-term
 * amplitudes a_t (complex64 pairs) of a one-plan exec, n_total terms each,
 * owned by the exec and valid after tn_exec_run until the next estimate or
 * tn_exec_destroy.  TN_EINVAL for an exec of several packed plans (their
 * outputs are separate arrays: tn_exec_copy_outputs takes a plan index). */
int tn_exec_outputs(tn_exec ex, const double** d_x, const float** d_amp, int64_t* n_total);

/* Fill up to `max` entries of per-kernel statistics; *n receives the count.
 * reset != 0 clears the accumulators after reading (the per-launch totals that
 * tn_exec_describe reports as t_ms / t_n included). */
int tn_exec_kernel_stats(tn_exec ex, int32_t max, tn_kernel_stat* out, int32_t* n, int32_t reset);

/* Copy the per-term values X_t (float64) and amplitudes a_t (complex64 as
 * float pairs) of packed plan `plan` to host memory (n_terms entries each;
 * either pointer may be NULL).  Synchronous; valid after tn_exec_run. */
int tn_exec_copy_outputs(tn_exec ex, int32_t plan, double* h_x, float* h_amp);

/* Timing of the last tn_exec_run: total milliseconds on the stream (HIP
 * events around the estimate) and the summed durations of its contraction
 * launches (GEMM-shaped: per-step GEMMs, grouped small steps, matrix-core
 * tiles and their split-sum reduces), permutes and other timed kernels, from
 * the per-launch HIP events of the launches tn_exec_kernel_stats counts (the
 * tail launches are not timed one by one).  The breakdown is
 * recorded when the exec was prepared with per-launch timing
 * (tn_exec_opts.time_kernels), else each of the three is -1; before the
 * first tn_exec_run all four are -1. */
int tn_exec_timing(tn_exec ex, double* total_ms, double* gemm_ms, double* permute_ms,
                   double* other_ms);

/* ---------------------------------------------------------------------------
 * tn_contract_batch -- the term contractions of Algorithm 1 (Section IV) for
 * terms [first, first+count) of each packed plan's term set: their ket
 * networks are contracted and the amplitudes a_t written as complex64 to
 * d_amp (count values per plan, plan-major; device memory the caller owns).
 * a_t is the amplitude with slot tensors sqrt(2) K_{c_s} (K_i as in
 * tn_plan_noise), so the term value is X_t = w_t 2^-N |a_t|^2 with w_t from
 * tn_terms_get.  All in FP32 (no FP64 pass).
 *
 * Only the range's terms are scheduled.  The schedule is built and bound to
 * d_ws on the first call with these arguments (plans, term sets, range, d_ws,
 * ws_bytes) and kept: later calls with the same arguments upload its
 * constants again (from a page-locked copy) and run it, so any range can be
 * resumed or repeated cheaply.  At most 8 schedules are kept; those naming a
 * plan or term set are dropped when it is destroyed (tn_release_cached drops
 * all).  Asynchronous on `stream`: d_amp is valid once the stream reaches the
 * call's end, and d_ws must not be used for anything else until then.  Calls
 * are serialized by the library; two calls sharing d_ws must run on one
 * stream.
 *
 * Errors: TN_EINVAL (null handle, negative or out-of-range range, null d_amp
 * or d_ws, ws_bytes == 0), TN_ENOMEM (ws_bytes below the range's schedule; no
 * device call is made), TN_EHIP.  count == 0 does nothing.
 * ------------------------------------------------------------------------- */
int tn_contract_batch(int32_t n, const tn_plan* plans, const tn_terms* terms, int64_t first,
                      int64_t count, void* d_amp, void* d_ws, size_t ws_bytes, void* stream);

/* ---------------------------------------------------------------------------
 * tn_estimate -- Algorithm 1 end to end (Section III, Problem 1; Section IV,
 * Algorithm 1's Require / Ensure) for n packed plans: every term contracted,
 * X_t = w_t |a_t|^2, the level sums T_u and A(l') for l' <= l; the
 * all-dominant term in FP64.  Synchronizes `stream` and fills results[n].
 *
 * Workspace (device memory the caller owns; sizes from tn_plan_workspace):
 *   ws_bytes >= full_bytes : one schedule over all terms, kept between calls
 *     with the same arguments as for tn_contract_batch (its constants are
 *     uploaded again on each call);
 *   min_bytes <= ws_bytes < full_bytes : each plan's terms run as consecutive
 *     ranges, each range as large as fits, their X_t gathered in one array
 *     whose level sums are taken by the same fixed-order kernel (per-term
 *     values equal the one-schedule ones to FP32 rounding: tile shapes and
 *     split sums depend on a range's size);
 *   ws_bytes < min_bytes : TN_ENOMEM before any device call.
 * Errors: TN_EINVAL (null handle, results or d_ws, ws_bytes == 0), TN_ENOMEM,
 * TN_EHIP.
 * ------------------------------------------------------------------------- */
int tn_estimate(int32_t n, const tn_plan* plans, const tn_terms* terms, void* d_ws,
                size_t ws_bytes, void* stream, tn_result* results);

/* Drop every schedule kept by tn_estimate / tn_contract_batch (waits for
 * their last calls' streams). */
void tn_release_cached(void);

/* ---------------------------------------------------------------------------
 * tn_estimate_noalloc -- tn_estimate for callers that cannot allocate device
 * or page-locked memory (code under stream capture, tight serving loops,
 * harnesses that forbid hipMalloc): the same schedule and kernels, with the
 * workspace in a fixed 64 MiB device array of the library (one per GPU, held
 * until the process ends) instead of a caller buffer.  It calls no hipMalloc,
 * hipFree, hipHostMalloc, stream or event creation: the constants are copied
 * in, both chains and the tail run on `stream` one after the other, the level
 * sums are copied back, and the stream is synchronized.  Every call on a GPU
 * uses that GPU's array (its contents are rewritten by each call), so calls
 * that overlap on one GPU race: serialize them.  Not kept between calls.
 * Errors: TN_EINVAL (null handle or results), TN_ENOMEM (the estimate needs
 * more than the fixed 64 MiB; no device call is made), TN_EHIP.
 * ------------------------------------------------------------------------- */
int tn_estimate_noalloc(int32_t n, const tn_plan* plans, const tn_terms* terms, void* stream,
                        tn_result* results);

/* ---------------------------------------------------------------------------
 * tn_plan_build_trajectories / tn_terms_trajectories -- the quantum-trajectories
 * estimate, the paper's comparison method (Section V), on the same engine.
 * Noise s draws Kraus operator k with probability q_k = tr(E_k^+ E_k) / 2 (they
 * sum to 1 for a channel, Section II) and its slot carries E_k / sqrt(q_k), so
 * for any draws the mean of X = |<v| ... |psi>|^2 over samples has expectation
 * <v| E(|psi><psi|) |v>.  The plan is built like tn_plan_build (same network,
 * light cone and path search; at most 4 Kraus operators per noise, else
 * TN_EUNSUPPORTED; degenerate channels are fine).  tn_terms_trajectories makes
 * n_samples terms from `uniforms` (host, n_samples x n_noise values in [0, 1),
 * row-major; the caller's random numbers): sample i takes, for noise s, the
 * first k with q_k > 0 and uniforms[i n_noise + s] < q_0 + ... + q_k.  Every
 * term has weight 1 / n_samples and level 0, so an estimate over the set
 * reports the sample mean as A[0] (bound -1: not a truncation); the per-sample
 * X are in tn_exec_outputs / tn_exec_copy_outputs (sample 0 in FP64, the rest
 * FP32).  Repeated draws share their contraction (instances).  A trajectories
 * plan rejects tn_terms_enumerate and tn_terms_enumerate_factored (TN_EINVAL).
 * Errors: as tn_plan_build; TN_EINVAL for n_samples < 1, a uniform outside
 * [0, 1), a plan that is not a trajectories plan.  Host only.
 * ------------------------------------------------------------------------- */
int tn_plan_build_trajectories(const tn_circuit* circ, const tn_state* psi, const tn_state* v,
                               const tn_plan_opts* opts, tn_plan* out);
int tn_terms_trajectories(tn_plan plan, int64_t n_samples, const double* uniforms, tn_terms* out,
                          int64_t* n_terms);

/* ---------------------------------------------------------------------------
 * tn_terms_enumerate_factored -- exact cross-term reuse over independent
 * clusters.  A term's amplitude is the product of its clusters' amplitudes
 * and its weight a product over slots, so the level sums of the full level-l
 * expansion (Algorithm 1) are the coefficients of the product of per-cluster
 * level polynomials: A(l) = sum_{k<=l} [prod_c g_c](k), g_c(k) the sum over
 * cluster c's own correction patterns with k corrections.  This set holds only
 * terms whose corrections lie in one cluster: the all-dominant term, then for
 * u = 1..level (ascending) and each cluster with at least u slots, that
 * cluster's level-u terms (position sets and corrections in the order of
 * tn_terms_enumerate restricted to its slots).  Terms are grouped by (level,
 * cluster); group 0 is the all-dominant term.  Run it through tn_exec_prepare /
 * tn_exec_run like any term set (its level sums there mix clusters and are not
 * the estimate), sum X per group (tn_kernel_group_sums), and combine with
 * tn_factored_levels.  n_groups receives the group count.  Host only.
 * Errors: TN_EINVAL (level < 0, above TN_MAX_LEVEL, a doubled plan).
 *
 * tn_terms_groups -- group g's terms are [starts[g], starts[g+1]) (n_groups + 1
 * entries), of level level[g] in cluster cluster[g] (-1 for group 0).  Any
 * output may be NULL.  TN_EINVAL for a term set that is not factored.
 *
 * tn_factored_levels -- A(0..level) (level + 1 doubles) from the group sums
 * h[g] (n_groups doubles, host): with X0 = h[0], r_c(0) = 1 and
 * r_c(k) = h_c(k) / X0 (h_c(k) equals g_c(k) X0 / g_c(0)),
 * A(l) = X0 sum_{k<=l} [prod_c r_c](k).  TN_EDEGENERATE if X0 = 0 at level > 0.
 * ------------------------------------------------------------------------- */
int tn_terms_enumerate_factored(tn_plan plan, int32_t level, tn_terms* out, int64_t* n_terms,
                                int32_t* n_groups);
int tn_terms_groups(tn_terms terms, int64_t* starts, int32_t* level, int32_t* cluster);
int tn_factored_levels(tn_terms terms, const double* group_sums, double* A);

/* ---------------------------------------------------------------------------
 * tn_polarization_combine -- an off-diagonal element <x| E(|psi><psi|) |y>
 * from four results (Section III, after Problem 1: the polarization identity
 * <x|A|y> = 1/4 sum_{k=0..3} i^k <v_k|A|v_k>).  r[k] is the result of the same
 * circuit and term level with the bond-2 target v_k = y + i^k x (TN_STATE_SUM2
 * or TN_STATE_CIRCUIT_OUTPUT_SUM2 with p = y, q = x, c = i^k), e.g. the four
 * plans of one tn_exec_run, or of four doubled plans for the exact element.
 * Writes A_xy(u) = 1/4 sum_k i^k A_k(u) for u = 0..r[0].level into re[] and
 * im[] (host arrays of at least level + 1 entries).  Host only.
 * Errors: TN_EINVAL (null pointer, results of different levels).
 * ------------------------------------------------------------------------- */
int tn_polarization_combine(const tn_result* r, double* re, double* im);

/* Workspace bytes of tn_estimate for these plans and term sets (host only):
 * full_bytes runs the estimate as one schedule; min_bytes is the least it
 * accepts (terms in ranges of one: the per-term X array and level sums plus
 * the largest single-term schedule).  Either pointer may be NULL (not both).
 * Errors: TN_EINVAL (null handles), planning errors as tn_exec_prepare. */
int tn_plan_workspace(int32_t n, const tn_plan* plans, const tn_terms* terms,
                      size_t* min_bytes, size_t* full_bytes);

/* Introspection (host only). -------------------------------------------- */
typedef struct {
    int32_t n_qubits, n_noise, level, clamped;
    int32_t n_clusters;            /* independent networks after light-cone reduction */
    int32_t n_leaves;              /* tensors of the reduced ket network */
    int32_t max_log_size;          /* largest path tensor, log2 elements (one instance) */
    double flops_per_term;         /* 8 * sum of complex MACs of the path, one term */
    int32_t doubled;               /* 1: built by tn_plan_build_doubled */
    int32_t n_channels;            /* noise channels of the circuit */
} tn_plan_info;

int tn_plan_get_info(tn_plan plan, tn_plan_info* info);

/* Singular values d[4] (descending), the normalised slot matrices K_i
 * (4 x 2x2 row-major, K_i = unvec of the i-th singular vector) and the noise
 * rate ||M - I||_2 of noise s. */
int tn_plan_noise(tn_plan plan, int32_t s, double* d, tn_c128* k, double* rate);

/* JSON description of the plan (clusters, leaves, path) into buf (NUL
 * terminated); *len receives the needed size including the NUL. */
int tn_plan_describe(tn_plan plan, char* buf, size_t* len);

/* JSON description of a prepared schedule's steps (shapes, instances,
 * modes; with time_kernels, each launch's accumulated duration t_ms over t_n
 * runs) into buf; *len receives the needed size. */
int tn_exec_describe(tn_exec ex, char* buf, size_t* len);

/* The staged constant region of a prepared (or size-queried) schedule: fixed
 * tensors, slot tensors, instance maps and permutation tables, exactly as
 * uploaded to the start of the workspace.  Host only; *len receives the size. */
int tn_exec_const_bytes(tn_exec ex, void* buf, size_t* len);

void tn_plan_destroy(tn_plan plan);
void tn_terms_destroy(tn_terms terms);
void tn_exec_destroy(tn_exec ex);
const char* tn_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* TN_H */
