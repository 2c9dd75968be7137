// Internal host-side structures of the term-network contractor.
#pragma once

#include <complex>
#include <cstdint>
#include <string>
#include <vector>

#include "tn.h"

namespace tn {

using cd = std::complex<double>;
using u128 = unsigned __int128;

constexpr int kMaxSlotsPerCluster = 64;   // 2 bits per slot in a 128-bit key

// Error carrier used inside the library; converted to a TN_E* code at the ABI.
struct Error {
    int code;
    std::string msg;
};
[[noreturn]] void fail(int code, const std::string& msg);
void set_last_error(const std::string& msg);

// Split of one noise superoperator (Section IV, Fig. 3): M = sum_i U_i (x) V_i
// with U_i = d_i K_i and V_i = conj(K_i); K_i = unvec of the i-th singular
// vector of the permuted (Hermitian PSD) matrix.
struct NoiseSplit {
    int qubit = 0;
    int64_t op_index = 0;
    double d[4] = {0, 0, 0, 0};   // descending
    cd K[4][4];                   // K_i row-major 2x2
    bool zero[4] = {false, false, false, false};  // d_i treated as exactly 0
    double rate = 0;              // ||M - I||_2
    double norm_main = 0;         // ||U_0 (x) V_0||_2
    double norm_bar = 0;          // ||sum_{i>=1} U_i (x) V_i||_2
    // structure of the slot's past light cone (pruning features)
    std::vector<uint64_t> cone;   // bitset of qubits in the past light cone
    int cone_qubits = 0;
    int cone_2q_gates = 0;        // 2-qubit gates in the past light cone
    double khat_norm2[4] = {0, 0, 0, 0};  // ||sqrt(2) K_i||_2^2 (term bound factor)
    double q[4] = {0, 0, 0, 0};   // trajectories: draw probabilities tr(E_k^+ E_k) / 2
};

// One tensor of the reduced ket network.  All legs have dimension 2;
// legs[0] is the most significant bit of the element index.
struct Leaf {
    int slot = -1;                // -1: fixed tensor; else the noise index
    std::vector<int> legs;        // edge ids
    std::vector<cd> data;         // fixed tensors: 2^|legs| values (FP64)
};

struct PathStep {
    int a, b;                     // node ids: 0..L-1 leaves (cluster-local), L+j step j
};

struct Cluster {
    std::vector<int> leaves;      // global leaf ids
    std::vector<int> slots;       // noise indices, ascending (local slot j = slots[j])
    std::vector<PathStep> path;   // L-1 steps (contraction tree)
    double cmacs_per_term = 0;    // complex MACs of the path, one term
    int max_log = 0;              // largest node, log2 elements
};

struct Plan {
    uint64_t id = 0;
    int n_qubits = 0;
    int64_t n_ops = 0;
    int n_2q_gates = 0;
    int n_noise = 0;
    int level_req = 0;
    int level = 0;
    bool clamped = false;
    std::vector<NoiseSplit> noise;
    std::vector<Leaf> leaves;
    std::vector<Cluster> clusters;
    cd scalar = 1.0;              // product of factors outside every cluster
    // doubled network (exact value): ket and bra halves joined by every noise's
    // full superoperator tensor; no slots, one term, value Re(a) instead of |a|^2
    bool doubled = false;
    int n_channels = 0;           // noises of the circuit (all inside the network)
    // quantum-trajectories plan: slot k of a noise is its Kraus operator
    // E_k / sqrt(q_k) with weight 1 (terms are sampled, not enumerated)
    bool trajectories = false;
    int max_log = 0;
    double cmacs_per_term = 0;
    std::string target_kind;
};

struct Terms {
    const Plan* plan = nullptr;
    uint64_t plan_id = 0;
    int level = 0;
    int64_t n = 0;
    std::vector<int8_t> pat;      // n * N corrections
    std::vector<double> w;        // prod_s d_{c_s}
    std::vector<uint8_t> lvl;     // level of each term
    std::vector<uint8_t> zero;    // weight exactly zero (never contracted)
    std::vector<uint8_t> pruned;  // dropped by the pruning policy (never contracted)
    // factored term sets (corrections within one cluster): group g covers terms
    // [group_start[g], group_start[g + 1]) of level group_level[g] inside cluster
    // group_cluster[g]; group 0 is the all-dominant term (cluster -1)
    bool factored = false;
    std::vector<int64_t> group_start;
    std::vector<int32_t> group_level, group_cluster;
};

// plan.cpp
Plan* build_plan(const tn_circuit* circ, const tn_state* psi, const tn_state* v, int level,
                 const tn_plan_opts* opts);
Plan* build_plan_doubled(const tn_circuit* circ, const tn_state* psi, const tn_state* v,
                         const tn_plan_opts* opts);
Terms* enumerate_terms(const Plan* p, int level, const tn_prune_opts* prune);
Terms* enumerate_terms_factored(const Plan* p, int level);
Plan* build_plan_trajectories(const tn_circuit* circ, const tn_state* psi, const tn_state* v,
                              const tn_plan_opts* opts);
Terms* sample_terms(const Plan* p, int64_t n_samples, const double* uniforms);
void factored_levels(const Terms* t, const double* group_sums, double* A);
std::string describe_plan(const Plan* p);
int term_features(const Plan* p, const Terms* t, const double* level1_x, float* out);
constexpr int kNumFeatures = 36;
void jacobi_hermitian4(const cd a_in[4][4], double evals[4], cd evecs[4][4]);
double spectral_norm4(const cd a[4][4]);

}  // namespace tn
