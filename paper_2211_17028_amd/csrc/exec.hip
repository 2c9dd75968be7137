// Device schedule and execution of the batched term contractions, and the
// extern "C" entry points of the library.
//
// All term networks of a circuit share one topology (Section IV: only the
// slot tensors U_i (x) V_i differ).  The path chosen at plan time is run once
// per estimate: every intermediate tensor is kept once per distinct
// restriction of the term patterns to the slots below it ("instances"), so a
// step is one batched contraction over those instances, gathered through
// per-step index maps.  Slot-free intermediates exist once and are shared by
// every term.  The term values are X = w |a|^2 (bra network = conjugate of the
// ket network for a channel), summed per level in FP64 (Algorithm 1).

#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <map>
#include <set>
#include <numeric>
#include <climits>
#include <condition_variable>
#include <memory>
#include <mutex>
#include <thread>
#include <sstream>
#include <tuple>
#include <unordered_map>

#include "kernels.h"
#include "tn_internal.h"

namespace tn {

const char* last_error_cstr();

#define HIPCHK(x)                                                                          \
    do {                                                                                   \
        hipError_t e_ = (x);                                                               \
        if (e_ != hipSuccess)                                                              \
            fail(TN_EHIP, std::string(#x) + ": " + hipGetErrorString(e_));                 \
    } while (0)

static int64_t round_up(int64_t x, int64_t a) { return (x + a - 1) / a * a; }

// tn_estimate_noalloc: size of its fixed per-GPU workspace, and the devices it serves
constexpr size_t kNoAllocScratchBytes = size_t(64) << 20;
constexpr int kMaxDevices = 64;

// first-fit allocator over a linear region (offsets only)
struct Arena {
    std::map<int64_t, int64_t> free_;
    int64_t top = 0, peak = 0;
    int64_t alloc(int64_t bytes) {
        bytes = round_up(std::max<int64_t>(bytes, 1), 256);
        for (auto it = free_.begin(); it != free_.end(); ++it)
            if (it->second >= bytes) {
                int64_t off = it->first, sz = it->second;
                free_.erase(it);
                if (sz > bytes) free_[off + bytes] = sz - bytes;
                return off;
            }
        int64_t off = top;
        top += bytes;
        peak = std::max(peak, top);
        return off;
    }
    void release(int64_t off, int64_t bytes) {
        bytes = round_up(std::max<int64_t>(bytes, 1), 256);
        auto it = free_.emplace(off, bytes).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
                it = pv;
            }
        }
        if (it->first + it->second == top) {
            top = it->first;
            free_.erase(it);
        }
    }
};

// constants staged on the host and uploaded in one copy
struct ConstBuf {
    std::vector<unsigned char> bytes;
    int64_t add(const void* p, int64_t n) {
        int64_t off = round_up((int64_t)bytes.size(), 256);
        bytes.resize(off + n);
        if (p) std::memcpy(bytes.data() + off, p, n);
        return off;
    }
    int64_t reserve(int64_t n) { return add(nullptr, n); }
};

// R_WORK2: the FP64 pass (side stream); R_HOST: pinned host memory the tail
// kernels write the estimate's results into (level sums, FP32 root value)
enum Region { R_CONST = 0, R_WORK = 1, R_WORK2 = 2, R_HOST = 3 };
struct Ref {
    int region = R_CONST;
    int64_t off = 0;
};

enum LaunchKind { L_PERM = 0, L_GEMM = 1, L_FINALIZE = 2, L_LEVELSUM = 3, L_SLOTFILL = 4, L_GROUP = 5,
                  L_MGROUP = 6, L_MREDUCE = 7 };
struct GroupJob;
struct MJob;

struct Launch {
    int kind = 0;
    int fp64 = 0;
    int level = -1;                // tree level of a level-grouped launch (-1: none)
    // operands (resolved at bind time)
    Ref a, b, c, ia, ib, table;
    GemmArgs g{};
    PermArgs p{};
    int tile_hint = -1;
    int kclass = -1;
    double flops = 0, bytes = 0;   // algorithmic work of this launch
    double t_ms = 0;               // time_kernels: accumulated duration and count of this launch
    int64_t t_n = 0;
    int plan = 0;
    int plain_root = 0;            // PLAIN mode: output offset advances per term
    int64_t plain_root_stride = 0;
    // finalize / level sum
    FinalizeArgs f{};
    Ref live_index, root_idx, root_ptrs, root64_ptrs, w, x_out, amp_out, starts, sums;
    int n_levels = 0;
    // slot fill
    SlotFillArgs sf{};
    Ref sf_noise, sf_dst, sf_bank, sf_pattern;
    hipEvent_t ev_a = nullptr, ev_b = nullptr;   // per-launch timing (optional)
    int gather = 0;                               // GEMM reads operands in stored order
    Ref oa, ob;                                   // gathered operands: slice offsets (int64)
    // grouped launch (L_GROUP): device job records in the constant region
    Ref jobs;
    int n_jobs = 0;
    int64_t blocks = 0;
    std::vector<struct GroupJob> hjobs;
    // grouped matrix-core launch (L_MGROUP); L_MREDUCE shares its job and tile
    // records (written by the L_MGROUP launch it follows)
    int mtile = 0;
    Ref tiles;
    int64_t n_tiles = 0;
    std::vector<struct MJob> mjobs;
};

struct PlanExec {
    const Plan* plan;
    const Terms* terms;
    int64_t n_terms = 0, n_live = 0;
    int64_t zero_term = -1;
    std::vector<int64_t> level_start;
    Ref x_out, amp_out, sums, x0;  // x0: FP32 value of the all-dominant term (diagnostic)
    std::vector<Ref> root32;       // per cluster root buffer (FP32 batch)
    std::vector<int64_t> root32_inst;
    std::vector<Ref> root64;
    bool fp32_skipped = false;     // the FP64 pass covers every live term: no FP32 chain
    int64_t n_zero = 0, n_pruned = 0;
    std::vector<int64_t> live_terms;  // term indices of live terms
};

}  // namespace tn

// Host thread that issues the FP64 pass's launches on the side stream while
// the calling thread issues the FP32 chain (direct launches): issuing costs
// host time per launch, and one thread alternating between the two chains
// delays the FP32 chain's short early launches.
struct SideIssuer {
    std::thread th;
    std::mutex mu;
    std::condition_variable cv;
    uint64_t gen = 0, done = 0;   // batches requested / finished
    bool stop = false;
    bool failed = false;
    tn::Error err{0, ""};
};

// One level of the grouped-launch autotuner: the shape kept (-1: the model's
// own choice) and the median microseconds of a whole estimate with the model's
// choice at the level and with each shape imposed on all its jobs (-1: not
// timed, did not fit the workspace; empty when the choice came from the cache).
struct TuneRecord {
    int tile = -1;
    double model_us = -1.0;
    std::vector<double> us;
};

struct tn_exec_s {
    std::unique_ptr<SideIssuer> issuer;     // FP64 pass issued from its own host thread
    int device = 0;
    std::vector<tn::Launch> launches;       // FP32 batched launches, in order (main stream)
    std::vector<tn::Launch> launches64;     // FP64 dominant-term pass (side stream)
    std::vector<tn::Launch> plain_launches; // PLAIN mode per-term body
    std::vector<tn::Launch> launches_const; // slot-free steps: run once per binding (and upload)
    std::vector<tn::Launch> tail;           // finalize + level sums
    // packed circuits: the tail runs as one finalize and one level-sum launch
    // the tail of all packed circuits: one record per circuit, the per-block
    // level partials of the term launch
    tn::Ref tail_jobs, tail_part;
    int64_t tail_blocks = 0;
    int tail_levels = 0;
    std::vector<tn::PlanExec> plans;
    // results of an estimate (level sums, FP32 all-dominant value of every
    // plan), written by the tail kernels into pinned host memory
    int64_t results_bytes = 0;
    // host results: slot 0 written by the tail kernels; slots 1, 2 copies made
    // by submitted estimates (at most two outstanding), each results_stride bytes
    int64_t results_stride = 0;
    // bytes past the results region where the next estimate's tail writes (a
    // submitted estimate's slot, direct launches only; 0 otherwise)
    int64_t res_shift = 0;
    hipEvent_t ev_done[2] = {nullptr, nullptr};
    int64_t next_ticket = 0, collected = 0;
    hipStream_t submit_stream = nullptr;   // stream of the outstanding submitted estimates
    void* results_host = nullptr;      // host address
    void* results_dev = nullptr;       // the same memory as the device addresses it
    tn::ConstBuf cbuf;
    int64_t const_bytes = 0, work_bytes = 0, work1_bytes = 0;
    hipStream_t side = nullptr;             // side stream for the FP64 pass (default priority)
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    char* base = nullptr;
    hipStream_t stream = nullptr;
    tn_exec_opts opts{};
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    hipStream_t cap_stream = nullptr;   // private stream used only to record the graph
    double last_ms = -1, gemm_ms = -1, perm_ms = -1, other_ms = -1;
    int64_t plain_terms = 0;
    int time_kernels = 0;
    std::map<int, std::pair<int64_t, double>> kstat;  // kernel id -> (launches, ms) accumulated
    std::map<int, double> kflops, kbytes;             // kernel id -> algorithmic work accumulated
    bool bound = false;
    // the schedule's planning choices: FP32 levels run in their small-step
    // launch, and the tile shape imposed per level (tuned levels: on every job)
    std::set<int> small_levels;
    std::map<int, std::pair<int, double>> level_tile;
    // grouped-launch autotuner: per tuned level, what was kept and timed
    std::map<int, TuneRecord> tuning;
    ~tn_exec_s();   // joins the side issuer, frees events, streams, graph and host results
};

namespace tn {

// ---------------------------------------------------------------------------
// schedule construction
// ---------------------------------------------------------------------------
struct NodeInfo {
    std::vector<int> legs;     // storage order, legs[0] most significant
    u128 mask = 0;             // 2 bits per cluster-local slot
    std::vector<u128> keys;    // sorted distinct instance keys
    Ref buf;                   // symbolic: Ref{R_NODE, gid}
    int gid = -1;              // node id in the builder's node table
    int level = 0;             // 0 for leaves; else 1 + max over the operands, where a slot-free
                               // operand computed at prepare counts as 0 (see fold_const)
    int64_t bytes = 0;
    bool leaf = true;
};

// Symbolic buffer references used while steps are planned; replaced by
// concrete ones when the steps are placed in memory (level by level).
enum { R_NODE = 10, R_TEMP = 11 };

// Steps of at least this many flops run on the tile kernels (matrix cores in
// FP32, 64 x 64 FMA tiles in FP64) whatever their shape (below it, only shapes
// that fill a tile do), unless their inner sums are long (a tile walks its
// inner index alone: above 2^11 in FP32, 2^8 in FP64) or their slices have
// fewer than 8 outputs (inner products: split sums in the small kernel).
constexpr double kMfmaMinFlops = 16.0 * 1024 * 1024;
constexpr int64_t kNumCUs = 256;     // MI355X compute units
// Below this many flops a step that fills a tile still joins the small-step launch.
constexpr double kTileMinFlops = 2.0 * 1024 * 1024;
// A tile job splits its inner sum over S blocks (S a power of two) when the
// sum has at least 2^kSplitMinKLog terms and the multiplied tiles leave at
// most two per CU (more tiles per CU already keep the matrix cores busy
// through the inner loop); S grows while that holds, each part keeps at least
// 2^kSplitMinPartLog terms and S stays within the executor's limit.
constexpr int kSplitMinKLog = 6;
constexpr int kSplitMinPartLog = 5;
constexpr int64_t kSplitMaxTiles = 512;
constexpr int kSplitDefaultMax = 16;
// FP64 steps whose slices fill a 32 x 32 tile but whose inner sums are longer
// than a tile walks alone (the exact value's last inner products: 32 x 32
// outputs over 2^21 terms) run as tile jobs split over up to this many blocks
// (each part at least 2^kSplitMinPartLog terms, S x tiles <= kSplitMaxTiles);
// the small kernel's block per output would stream a whole row and column of
// the operands per output.
constexpr int kSplitLongMax = 512;
// A matrix-core job with at most this share of the flops of its level's main
// tile shape takes that shape, so that it runs in the main launch.
constexpr double kSmallJobShare = 0.25;
// One launch in tile-model units (the 25-qubit workload's 512-tile 128 x 64
// launch of k = 8 models at 1.0e8 and runs 15 us; a launch costs about 5 us).
constexpr double kLaunchCost = 3.5e7;
// A FP32 tree level with less work than this (summed over its steps) runs all
// its steps in its small-step launch: a grouped tile launch of its own costs
// more than the tiles save (a dependent launch costs about 10 us end to end).
constexpr double kSmallLevelFlops = 32.0 * 1024 * 1024;

// Long inner sums of small steps: one block per output element when that is
// the shorter chain of dependent loads (a thread-per-output sum runs k / 4
// rounds; a block per output k / 2048 rounds plus its reduction, over the
// outputs in batches of ~2048 resident blocks).
static bool split_by_block(int k_log, int64_t outs) {
    const double kk = std::ldexp(1.0, k_log);
    const double t_thread = kk / 4.0;
    const double t_block = std::ceil((double)outs / 2048.0) * (kk / 2048.0 + 3.0);
    return t_block < t_thread;
}

// Workgroups of a launch go to the 8 XCDs of the chip in turn (block b to XCD
// b mod 8), and each XCD has its own L2.  A job lists its tiles so that tiles
// sharing an operand panel are neighbours.  Within the blocks of each job, XCD j
// takes one contiguous chunk of the job's tiles (as many as the job's blocks on
// that XCD), so the tiles sharing a panel share an L2, and every XCD gets an
// equal share of every job: jobs of one launch differ in inner length and tile
// cost, and chunks over the whole list would give one XCD the costly jobs.
constexpr int kNumXcds = 8;
template <typename T>
static std::vector<T> xcd_order(const std::vector<T>& v) {
    const int64_t n = (int64_t)v.size();
    std::vector<T> out(v.size());
    for (int64_t s = 0; s < n;) {
        int64_t e = s;
        while (e < n && v[e].job == v[s].job) ++e;
        int64_t next[kNumXcds], cnt[kNumXcds] = {};
        for (int64_t b = s; b < e; ++b) ++cnt[b % kNumXcds];
        int64_t at = s;
        for (int j = 0; j < kNumXcds; ++j) {
            next[j] = at;
            at += cnt[j];
        }
        for (int64_t b = s; b < e; ++b) out[b] = v[next[b % kNumXcds]++];
        s = e;
    }
    return out;
}

// One grouped contraction (host side of a GettJob).
struct GroupJob {
    Ref a, b, c, oa, ob;
    int fp64 = 0;              // complex128 job (dominant-term pass) in a launch of either precision
    int64_t n_inst = 0;
    int m_log = 0, n_log = 0, k_log = 0, split = 0, rpt_log = 0;
    int8_t a_row[32] = {}, a_k[32] = {}, b_k[32] = {}, b_col[32] = {};
    double flops = 0, bytes = 0;
};

// One grouped matrix-core contraction (host side of an MfmaJob).
struct MJob {
    Ref a, b, c, oa, ob, oc;
    int m_log = 0, n_log = 0, k_log = 0, merge = 0, a_rowfast = 0, b_colfast = 0;
    int ksplit = 1;
    Ref partial;               // ksplit > 1: partial tiles (work region)
    int64_t ns = 0;            // slices
    int8_t a_row[32] = {}, a_k[32] = {}, b_k[32] = {}, b_col[32] = {};
    double flops = 0, bytes = 0;
    double out_bytes = 0;      // bytes of C (the split reduction's unit)
};

// One pairwise step before memory assignment.
struct StepRec {
    int level = 0;
    int plan = 0;
    int a_node = -1, b_node = -1, c_node = -1;
    int64_t c_bytes = 0;
    bool has_fixed = false;    // output location fixed (cluster root)
    Ref c_fixed;
    std::vector<int> temp_ids;
    std::vector<int64_t> temp_bytes;
    std::vector<Launch> launches;   // transposes, then the GEMM unless grouped
    bool grouped = false;
    GroupJob job;
    bool mgrouped = false;     // runs in its level's grouped matrix-core launch
    int mtile = 0;
    MJob mjob;
    std::vector<MfmaTile> mtiles;   // job index filled at emission
};

struct Builder {
    tn_exec_s* ex;
    Arena work;                // FP32 batch (main stream)
    Arena work2;               // FP64 dominant-term pass (side stream, runs concurrently)
    bool grouping = true;      // small steps of one tree level share one launch
    // Slot-free intermediates (no noise slot below them) are the same for every
    // term and every estimate: with fold_const their steps go to const32 /
    // const64 (run once when the schedule is bound), the ones the per-estimate
    // steps read are kept in the constant region, and the per-estimate tree
    // levels start above them.
    bool fold_const = false;
    std::vector<StepRec>* const32 = nullptr;
    std::vector<StepRec>* const64 = nullptr;
    bool quantize_tiles = true;  // tile model: whole rounds over the CUs (one circuit)
    int max_ksplit = kSplitDefaultMax;  // largest split of a tile job's inner sum (1 = none)
    bool ksplit_user = false;            // max_ksplit set by the caller (applies to every job)
    // FP32 tile shape imposed per tree level on jobs of at most the given
    // flops (the small jobs join the level's main matrix-core launch)
    const std::map<int, std::pair<int, double>>* level_tile = nullptr;
    // FP32 tree levels with little work: every step runs in the level's
    // small-step launch (one launch instead of one per tile shape plus one)
    const std::set<int>* small_levels = nullptr;
    std::vector<Ref> node_ref;         // concrete buffer of every node (once placed)
    std::vector<char> node_leaf;
    std::vector<int64_t> node_bytes;
    std::vector<Ref> temp_ref;
    int add_node(Ref r, bool leaf, int64_t bytes) {
        node_ref.push_back(r);
        node_leaf.push_back(leaf ? 1 : 0);
        node_bytes.push_back(bytes);
        return (int)node_ref.size() - 1;
    }

    static int64_t find_key(const std::vector<u128>& keys, u128 k) {
        auto it = std::lower_bound(keys.begin(), keys.end(), k);
        return it - keys.begin();
    }

    // permutation table from storage order `src` to `dst` (same leg set)
    Launch make_perm(const std::vector<int>& src, const std::vector<int>& dst, int fp64) {
        const int r = (int)src.size();
        std::vector<int> p(r), q(r);
        for (int j = 0; j < r; ++j) {
            int leg = dst[r - 1 - j];
            int pos = (int)(std::find(src.begin(), src.end(), leg) - src.begin());
            p[j] = r - 1 - pos;
        }
        for (int j = 0; j < r; ++j) q[p[j]] = j;
        const int tb = std::min(r, 5);
        std::vector<int> tile;
        for (int j = 0; j < tb; ++j) tile.push_back(j);
        for (int i = 0; i < tb; ++i)
            if (std::find(tile.begin(), tile.end(), q[i]) == tile.end()) tile.push_back(q[i]);
        std::sort(tile.begin(), tile.end());
        const int tt = (int)tile.size();
        const int tsize = 1 << tt;
        std::vector<int32_t> table(3 * tsize);
        // store order: tile index e <-> out offset
        for (int e = 0; e < tsize; ++e) {
            int32_t off = 0;
            for (int i = 0; i < tt; ++i)
                if ((e >> i) & 1) off |= 1 << tile[i];
            table[2 * tsize + e] = off;
        }
        // load order: low tb bits of l <-> input bits 0..tb-1 (out bits q[i]); the
        // rest of the tile positions (input bits >= tb) in ascending tile order
        std::vector<int> tpos_of_inbit(tb), rest;
        for (int i = 0; i < tb; ++i)
            tpos_of_inbit[i] = (int)(std::find(tile.begin(), tile.end(), q[i]) - tile.begin());
        for (int i = 0; i < tt; ++i)
            if (p[tile[i]] >= tb) rest.push_back(i);
        for (int l = 0; l < tsize; ++l) {
            int t = 0;
            for (int i = 0; i < tb; ++i)
                if ((l >> i) & 1) t |= 1 << tpos_of_inbit[i];
            for (size_t i = 0; i < rest.size(); ++i)
                if ((l >> (tb + i)) & 1) t |= 1 << rest[i];
            int32_t in_off = 0;
            for (int i = 0; i < tt; ++i)
                if ((t >> i) & 1) in_off |= 1 << p[tile[i]];
            table[l] = in_off;
            table[tsize + l] = t;
        }
        Launch L;
        L.kind = L_PERM;
        L.fp64 = fp64;
        L.kclass = fp64 ? K_PERM64 : K_PERM32;
        L.table = Ref{R_CONST, ex->cbuf.add(table.data(), (int64_t)table.size() * 4)};
        L.p.r = r;
        L.p.tb = tt;
        L.p.n_high = r - tt;
        // element pairs: load slots 2i, 2i+1 differ in input bit 0 and store
        // slots 2i, 2i+1 in output bit 0 exactly when both tile sides have >= 2 bits
        L.p.pair = tb >= 1 ? 1 : 0;
        for (int l = 0; l + 1 < tsize && L.p.pair; l += 2)
            if (table[l + 1] != table[l] + 1 || table[2 * tsize + l + 1] != table[2 * tsize + l] + 1)
                L.p.pair = 0;
        int h = 0;
        for (int j = 0; j < r; ++j)
            if (std::find(tile.begin(), tile.end(), j) == tile.end()) {
                L.p.high_out[h] = j;
                L.p.high_in[h] = p[j];
                ++h;
            }
        return L;
    }

    // Grouped matrix-core job of one FP32 step: orientation, tile shape and
    // merge mode are chosen by the padded tile work (a per-tile-shape
    // efficiency factor, plus a fixed cost per tile); slices are ordered so that
    // slices sharing the merged operand are adjacent, then cut into tiles.
    template <typename PosIn, typename ByPos, typename SliceVec>
    void plan_mfma_job(StepRec& st, const NodeInfo& A, const NodeInfo& B, NodeInfo& C, const std::vector<int>& K,
                       const std::vector<int>& Bt, const std::vector<int>& FA, const std::vector<int>& FB,
                       int64_t ninst, int64_t nbatch, PosIn posin, ByPos by_pos, SliceVec slice_vec, int fp64) {
        // FP64 steps run on the 64 x 64 or 32 x 32 FMA tiles (tile ids 1 and 4's shapes)
        const int64_t esz = fp64 ? 16 : 8;
        static const double kEff[K_MFMA_TILES] = {1.0, 0.6, 0.75, 0.5, 0.35, 0.45, 0.3, 0.2};
        static const double kEff64[K_MFMA_TILES] = {0, 1.0, 0, 0, 0.7, 0, 0, 0};
        const int rk = (int)K.size();
        const int64_t ns = ninst * nbatch;
        std::vector<int64_t> so[2][2];
        std::vector<int> btb[2];
        auto run_counts = [](std::vector<int64_t> v) {
            std::sort(v.begin(), v.end());
            std::vector<int64_t> c;
            for (size_t i = 0; i < v.size();) {
                size_t j = i;
                while (j < v.size() && v[j] == v[i]) ++j;
                c.push_back((int64_t)(j - i));
                i = j;
            }
            return c;
        };
        int forced = -1;
        if (!fp64 && level_tile && level_tile->count(st.level)) {
            const std::pair<int, double>& lt = level_tile->at(st.level);
            const double job_flops = 8.0 * std::ldexp((double)ns, (int)(FA.size() + FB.size()) + rk);
            if (job_flops <= lt.second) forced = lt.first;
        }
        double best_cost = 1e300, forced_cost = 1e300;
        int best_o = 0, best_tile = 0, best_merge = 0, forced_o = 0, forced_merge = 0;
        for (int o = 0; o < 2; ++o) {
            const NodeInfo& R = o ? B : A;
            const NodeInfo& Q = o ? A : B;
            const int m_log = (int)(o ? FB.size() : FA.size()), n_log = (int)(o ? FA.size() : FB.size());
            const bool r_big = ((int64_t)R.keys.size() << R.legs.size()) >= ((int64_t)Q.keys.size() << Q.legs.size());
            btb[o] = by_pos(Bt, r_big ? R : Q);
            so[o][0] = slice_vec(R, btb[o]);
            so[o][1] = slice_vec(Q, btb[o]);
            const std::vector<int64_t> ca = run_counts(so[o][0]), cb = run_counts(so[o][1]);
            for (int tile = 0; tile < K_MFMA_TILES; ++tile) {
                if (fp64 && tile != 1 && tile != 4) continue;

                const int bm_log = __builtin_ctz(mfma_tile_bm(tile)), bn_log = __builtin_ctz(mfma_tile_bn(tile));
                const int64_t rt = m_log >= bm_log ? int64_t(1) << (m_log - bm_log) : 1;
                const int64_t ct = n_log >= bn_log ? int64_t(1) << (n_log - bn_log) : 1;
                const double per_tile = std::ldexp(1.0, bm_log + bn_log) * (std::ldexp(1.0, rk) + 16.0) /
                                        (fp64 ? kEff64[tile] : kEff[tile]);
                // tiles on one CU share its matrix cores, so a launch lasts as long
                // as its busiest CU.  With one circuit a job mostly has its level to
                // itself: its tile count is rounded up to whole rounds over the 256
                // CUs (at least one round, so below 256 tiles smaller tiles finish
                // sooner).  Packed circuits share each level's launch, so their jobs
                // are costed by tile work alone.
                auto consider = [&](int64_t tiles, int merge) {
                    const int64_t eff_tiles =
                        !quantize_tiles ? tiles : std::max<int64_t>(1, (tiles + kNumCUs - 1) / kNumCUs) * kNumCUs;
                    const double cst = (double)eff_tiles * per_tile;
                    if (cst < best_cost) {
                        best_cost = cst;
                        best_o = o;
                        best_tile = tile;
                        best_merge = merge;
                    }
                    if (tile == forced && cst < forced_cost) {
                        forced_cost = cst;
                        forced_o = o;
                        forced_merge = merge;
                    }
                };
                consider(ns * rt * ct, 0);
                if (n_log < bn_log) {
                    const int64_t segs = int64_t(1) << (bn_log - n_log);
                    int64_t t = 0;
                    for (int64_t c : ca) t += (c + segs - 1) / segs;
                    consider(t * rt, 1);
                }
                if (m_log < bm_log) {
                    const int64_t segs = int64_t(1) << (bm_log - m_log);
                    int64_t t = 0;
                    for (int64_t c : cb) t += (c + segs - 1) / segs;
                    consider(t * ct, 2);
                }
            }
        }
        // a shape imposed by the level takes over when it costs this job at most
        // about one launch more than its own best shape (the launch it saves)
        // (a tuned level's shape, max flops = infinity, is imposed on every job)
        if (forced >= 0 && (forced_cost <= best_cost + kLaunchCost ||
                            std::isinf(level_tile->at(st.level).second))) {
            best_o = forced_o;
            best_tile = forced;
            best_merge = forced_merge;
        }
        const int o = best_o;
        const NodeInfo& R = o ? B : A;
        const NodeInfo& Q = o ? A : B;
        const std::vector<int>& FR = o ? FB : FA;
        const std::vector<int>& FQ = o ? FA : FB;
        const bool r_big = ((int64_t)R.keys.size() << R.legs.size()) >= ((int64_t)Q.keys.size() << Q.legs.size());
        std::vector<int> row_bits = by_pos(FR, R), col_bits = by_pos(FQ, Q), k_bits = by_pos(K, r_big ? R : Q);
        const std::vector<int>& bt_bits = btb[o];
        C.legs.assign(bt_bits.rbegin(), bt_bits.rend());
        C.legs.insert(C.legs.end(), row_bits.rbegin(), row_bits.rend());
        C.legs.insert(C.legs.end(), col_bits.rbegin(), col_bits.rend());
        C.bytes = ninst * (esz << C.legs.size());
        C.buf = Ref{R_NODE, C.gid};
        MJob& jb = st.mjob;
        jb.m_log = (int)FR.size();
        jb.n_log = (int)FQ.size();
        jb.k_log = rk;
        jb.ns = ns;
        jb.merge = best_merge;
        for (size_t q = 0; q < row_bits.size(); ++q) jb.a_row[q] = (int8_t)posin(R, row_bits[q]);
        for (size_t q = 0; q < k_bits.size(); ++q) {
            jb.a_k[q] = (int8_t)posin(R, k_bits[q]);
            jb.b_k[q] = (int8_t)posin(Q, k_bits[q]);
        }
        for (size_t q = 0; q < col_bits.size(); ++q) jb.b_col[q] = (int8_t)posin(Q, col_bits[q]);
        jb.a_rowfast = std::find(FR.begin(), FR.end(), R.legs.back()) != FR.end();
        jb.b_colfast = std::find(FQ.begin(), FQ.end(), Q.legs.back()) != FQ.end();
        // slice order: slices sharing the merged operand adjacent (stable)
        std::vector<int64_t> order(ns);
        std::iota(order.begin(), order.end(), 0);
        const std::vector<int64_t>& oa = so[o][0];
        const std::vector<int64_t>& ob = so[o][1];
        if (best_merge == 1)
            std::stable_sort(order.begin(), order.end(), [&](int64_t x, int64_t y) { return oa[x] < oa[y]; });
        if (best_merge == 2)
            std::stable_sort(order.begin(), order.end(), [&](int64_t x, int64_t y) { return ob[x] < ob[y]; });
        if (best_merge == 2) {
            // groups of slices sharing B, ordered by the smallest offset of their
            // A: groups that share an A become neighbours, so their tiles land on
            // one XCD at about the same time and share its L2 (the 36-qubit
            // QAOA's 32 x 16 level, 2608 distinct A read by 8208 slices in 1584 B
            // groups: 1.27 -> 0.85 GB fetched, 297 -> 262 us).  Groups sharing A
            // (merge 1) keep A's order, whose neighbouring tiles read
            // neighbouring A panels (the same reordering there measured slower).
            const std::vector<int64_t>& mk = ob;
            const std::vector<int64_t>& other = oa;
            std::vector<std::pair<int64_t, int64_t>> grp;   // (min other offset, first position)
            std::vector<int64_t> start;
            for (int64_t i = 0; i < ns;) {
                int64_t j = i, lo = other[order[i]];
                while (j < ns && mk[order[j]] == mk[order[i]]) lo = std::min(lo, other[order[j++]]);
                grp.push_back({lo, i});
                start.push_back(i);
                i = j;
            }
            start.push_back(ns);
            std::vector<size_t> gi(grp.size());
            std::iota(gi.begin(), gi.end(), 0);
            std::stable_sort(gi.begin(), gi.end(), [&](size_t x, size_t y) { return grp[x].first < grp[y].first; });
            std::vector<int64_t> reord;
            reord.reserve(ns);
            for (size_t g : gi)
                for (int64_t q = start[g]; q < start[g + 1]; ++q) reord.push_back(order[q]);
            order.swap(reord);
        }
        std::vector<int64_t> soa(ns), sob(ns), soc(ns);
        for (int64_t i = 0; i < ns; ++i) {
            soa[i] = oa[order[i]];
            sob[i] = ob[order[i]];
            soc[i] = order[i] << (jb.m_log + jb.n_log);
        }
        const int bm = mfma_tile_bm(best_tile), bn = mfma_tile_bn(best_tile);
        const int bm_log = __builtin_ctz(bm), bn_log = __builtin_ctz(bn);
        const int64_t rt = jb.m_log >= bm_log ? int64_t(1) << (jb.m_log - bm_log) : 1;
        const int64_t ct = jb.n_log >= bn_log ? int64_t(1) << (jb.n_log - bn_log) : 1;
        auto tile = [&](int cnt, int64_t s0, int64_t tm0, int64_t tn0) {
            MfmaTile t{};
            t.job = -1;
            t.cnt = cnt;
            t.s0 = s0;
            t.tm0 = tm0;
            t.tn0 = tn0;
            st.mtiles.push_back(t);
        };
        if (best_merge == 0) {
            for (int64_t i = 0; i < ns; ++i)
                for (int64_t r = 0; r < rt; ++r)
                    for (int64_t c = 0; c < ct; ++c) tile(1, i, r * bm, c * bn);
        } else {
            const std::vector<int64_t>& key = best_merge == 1 ? soa : sob;
            const int64_t segs = best_merge == 1 ? int64_t(1) << (bn_log - jb.n_log)
                                                 : int64_t(1) << (bm_log - jb.m_log);
            for (int64_t g0 = 0; g0 < ns;) {
                int64_t g1 = g0;
                while (g1 < ns && key[g1] == key[g0]) ++g1;
                for (int64_t p0 = g0; p0 < g1; p0 += segs) {
                    const int cnt = (int)std::min<int64_t>(segs, g1 - p0);
                    if (best_merge == 1)
                        for (int64_t r = 0; r < rt; ++r) tile(cnt, p0, r * bm, 0);
                    else
                        for (int64_t c = 0; c < ct; ++c) tile(cnt, p0, 0, c * bn);
                }
                g0 = g1;
            }
        }
        // Latency-bound jobs (long inner sums, few tiles: every tile resident at
        // once even when multiplied) split the inner sum over S tiles.
        const int64_t nt = (int64_t)st.mtiles.size();
        int split = 1;
        if (rk >= kSplitMinKLog)
            while (2 * split <= max_ksplit && 2 * split * nt <= kSplitMaxTiles &&
                   rk - __builtin_ctz(2 * split) >= kSplitMinPartLog)
                split *= 2;
        if (split > 1) {
            std::vector<MfmaTile> parts;
            parts.reserve(split * nt);
            for (int64_t q = 0; q < nt; ++q)
                for (int h = 0; h < split; ++h) {
                    MfmaTile t = st.mtiles[q];
                    t.kpart = h;
                    t.pair = (int32_t)q;
                    parts.push_back(t);
                }
            st.mtiles.swap(parts);
            jb.ksplit = split;
            const int64_t pbytes = nt * split * (int64_t)bm * bn * 2 * (fp64 ? 8 : 4);
            const int tid = (int)temp_ref.size();
            temp_ref.push_back(Ref{});
            st.temp_ids.push_back(tid);
            st.temp_bytes.push_back(pbytes);
            jb.partial = Ref{R_TEMP, tid};
        }
        jb.a = R.buf;
        jb.b = Q.buf;
        jb.c = C.buf;
        jb.oa = Ref{R_CONST, ex->cbuf.add(soa.data(), ns * 8)};
        jb.ob = Ref{R_CONST, ex->cbuf.add(sob.data(), ns * 8)};
        jb.oc = Ref{R_CONST, ex->cbuf.add(soc.data(), ns * 8)};
        const double mm = std::ldexp(1.0, jb.m_log), nnn = std::ldexp(1.0, jb.n_log), kk = std::ldexp(1.0, rk);
        jb.flops = 8.0 * mm * nnn * kk * (double)ns;
        jb.out_bytes = (double)esz * mm * nnn * (double)ns;
        jb.bytes = (double)esz * ((double)ns * mm * nnn + (double)R.keys.size() * nbatch * mm * kk +
                                  (double)Q.keys.size() * nbatch * kk * nnn);
        st.mgrouped = true;
        st.mtile = best_tile;
        st.c_bytes = C.bytes;
    }

    // Plan the steps of one cluster for the given root instance keys.
    // mode: 0 = FP32 batched, 1 = FP64 (single zero instance), 2 = PLAIN FP32
    // (single instance, slot leaves filled per term).  The root step writes to
    // root_out (modes 0 / 1).  Returns where the root value will be (root_out,
    // or the leaf's constant buffer when the cluster has no step).
    Ref build_cluster(const Plan& P, const Cluster& cl, const std::vector<u128>& root_keys, int mode,
                      int plan_index, std::vector<std::pair<int, int64_t>>* plain_slots, Ref root_out,
                      std::vector<StepRec>* steps) {
        const int fp64 = mode == 1;
        const int64_t esz = fp64 ? 16 : 8;
        const int wreg = fp64 ? R_WORK2 : R_WORK;
        const int L = (int)cl.leaves.size();
        const int nn = L + (int)cl.path.size();
        std::vector<NodeInfo> nodes(nn);
        std::vector<int> parent(nn, -1);
        for (size_t j = 0; j < cl.path.size(); ++j) {
            parent[cl.path[j].a] = L + (int)j;
            parent[cl.path[j].b] = L + (int)j;
        }
        for (int i = 0; i < L; ++i) {
            const Leaf& lf = P.leaves[cl.leaves[i]];
            nodes[i].legs = lf.legs;
            if (lf.slot >= 0) {
                int local = (int)(std::lower_bound(cl.slots.begin(), cl.slots.end(), lf.slot) - cl.slots.begin());
                nodes[i].mask = (u128)3 << (2 * local);
            }
        }
        for (size_t j = 0; j < cl.path.size(); ++j) {
            NodeInfo& c = nodes[L + j];
            c.leaf = false;
            c.mask = nodes[cl.path[j].a].mask | nodes[cl.path[j].b].mask;
        }
        const int root = nn - 1;
        nodes[root].keys = root_keys;
        for (int x = nn - 2; x >= 0; --x) {
            const NodeInfo& pn = nodes[parent[x]];
            std::vector<u128> ks;
            ks.reserve(pn.keys.size());
            for (u128 k : pn.keys) ks.push_back(k & nodes[x].mask);
            std::sort(ks.begin(), ks.end());
            ks.erase(std::unique(ks.begin(), ks.end()), ks.end());
            nodes[x].keys.swap(ks);
        }
        // leaves: constant data
        for (int i = 0; i < L; ++i) {
            const Leaf& lf = P.leaves[cl.leaves[i]];
            NodeInfo& nd = nodes[i];
            const int64_t sz = int64_t(1) << lf.legs.size();
            if (lf.slot < 0) {
                if (fp64) {
                    std::vector<double> d(2 * sz);
                    for (int64_t e = 0; e < sz; ++e) {
                        d[2 * e] = lf.data[e].real();
                        d[2 * e + 1] = lf.data[e].imag();
                    }
                    nd.buf = Ref{R_CONST, ex->cbuf.add(d.data(), (int64_t)d.size() * 8)};
                } else {
                    std::vector<float> d(2 * sz);
                    for (int64_t e = 0; e < sz; ++e) {
                        d[2 * e] = (float)lf.data[e].real();
                        d[2 * e + 1] = (float)lf.data[e].imag();
                    }
                    nd.buf = Ref{R_CONST, ex->cbuf.add(d.data(), (int64_t)d.size() * 4)};
                }
            } else {
                const NoiseSplit& ns = P.noise[lf.slot];
                int local = (int)(std::lower_bound(cl.slots.begin(), cl.slots.end(), lf.slot) - cl.slots.begin());
                if (mode == 2) {
                    // one instance, filled per term
                    nd.buf = Ref{R_CONST, ex->cbuf.reserve(4 * 8)};
                    plain_slots->push_back({lf.slot, nd.buf.off});
                } else {
                    std::vector<double> d64;
                    std::vector<float> d32;
                    for (u128 k : nd.keys) {
                        int ch = (int)((k >> (2 * local)) & 3);
                        for (int e = 0; e < 4; ++e) {
                            cd v = std::sqrt(2.0) * ns.K[ch][e];
                            d64.push_back(v.real());
                            d64.push_back(v.imag());
                            d32.push_back((float)v.real());
                            d32.push_back((float)v.imag());
                        }
                    }
                    nd.buf = fp64 ? Ref{R_CONST, ex->cbuf.add(d64.data(), (int64_t)d64.size() * 8)}
                                  : Ref{R_CONST, ex->cbuf.add(d32.data(), (int64_t)d32.size() * 4)};
                }
            }
        }
        for (int i = 0; i < L; ++i) {
            NodeInfo& nd = nodes[i];
            nd.gid = add_node(nd.buf, true, 0);
            nd.buf = Ref{R_NODE, nd.gid};
        }
        if (cl.path.empty()) return node_ref[nodes[0].gid];
        // remaining holders of every leg (a diagonal gate's wire index can be
        // held by more than two tensors)
        std::unordered_map<int, int> holders;
        for (int i = 0; i < L; ++i)
            for (int e : nodes[i].legs) holders[e] += 1;
        // steps
        for (size_t j = 0; j < cl.path.size(); ++j) {
            const int ia_node = cl.path[j].a, ib_node = cl.path[j].b;
            NodeInfo& A = nodes[ia_node];
            NodeInfo& B = nodes[ib_node];
            NodeInfo& C = nodes[L + j];
            StepRec st;
            st.plan = plan_index;
            const bool folding = fold_const && mode != 2;
            const bool folded = folding && C.mask == 0;
            if (!folding || folded) st.level = C.level = 1 + std::max(A.level, B.level);
            else st.level = C.level = 1 + std::max(A.mask ? A.level : 0, B.mask ? B.level : 0);
            // a folded node read by a per-estimate step (or a folded cluster
            // root) keeps its value for the whole schedule
            const bool folded_out = folded && (j + 1 == cl.path.size() || nodes[parent[L + j]].mask != 0);
            auto push_step = [&](StepRec&& sr) {
                if (!folded) {
                    steps->push_back(std::move(sr));
                    return;
                }
                if (folded_out && !sr.has_fixed) {
                    sr.has_fixed = true;
                    sr.c_fixed = Ref{R_CONST, ex->cbuf.reserve(sr.c_bytes)};
                }
                (fp64 ? const64 : const32)->push_back(std::move(sr));
            };
            C.gid = add_node(Ref{}, false, 0);
            st.a_node = A.gid;
            st.b_node = B.gid;
            st.c_node = C.gid;
            const bool is_root = j + 1 == cl.path.size();
            if (is_root) {
                st.has_fixed = true;
                st.c_fixed = mode == 2 ? Ref{wreg, 0} : root_out;   // PLAIN: replaced per term
            }
            // K: shared and held by nobody else (summed); Bt: shared and still
            // held elsewhere (kept, a batch dimension of this step)
            std::vector<int> K, Bt, FA, FB;
            for (int e : A.legs) {
                bool in_b = std::find(B.legs.begin(), B.legs.end(), e) != B.legs.end();
                if (!in_b) FA.push_back(e);
                else if (holders[e] > 2) Bt.push_back(e);
                else K.push_back(e);
            }
            for (int e : B.legs)
                if (std::find(A.legs.begin(), A.legs.end(), e) == A.legs.end()) FB.push_back(e);
            for (int e : K) holders[e] = 0;
            for (int e : Bt) holders[e] -= 1;
            const int rk = (int)K.size(), rb = (int)Bt.size();
            auto same_set = [](std::vector<int> a, std::vector<int> b) {
                std::sort(a.begin(), a.end());
                std::sort(b.begin(), b.end());
                return a == b;
            };
            // legs == bt ++ X ++ Y with set(X) = first, set(Y) = second?
            struct Layout {
                bool ok = false;
                std::vector<int> bt, k;
                int trans = 0;
            };
            auto match = [&](const std::vector<int>& legs, const std::vector<int>& F, bool k_first) {
                Layout lo;
                if (legs.size() != (size_t)(rb + rk + F.size())) return lo;
                std::vector<int> bt(legs.begin(), legs.begin() + rb);
                if (!same_set(bt, Bt)) return lo;
                std::vector<int> x, y;
                if (k_first) {
                    x.assign(legs.begin() + rb, legs.begin() + rb + rk);
                    y.assign(legs.begin() + rb + rk, legs.end());
                    if (!same_set(x, K) || !same_set(y, F)) return lo;
                    lo.k = x;
                } else {
                    x.assign(legs.begin() + rb, legs.end() - rk);
                    y.assign(legs.end() - rk, legs.end());
                    if (!same_set(x, F) || !same_set(y, K)) return lo;
                    lo.k = y;
                }
                lo.ok = true;
                lo.bt = bt;
                return lo;
            };
            // A: [Bt|FA|K] (trans 0) or [Bt|K|FA] (trans 1); B: [Bt|K|FB] (0) or [Bt|FB|K] (1)
            std::vector<Layout> la, lb;
            for (int t = 0; t < 2; ++t) {
                Layout x = match(A.legs, FA, t == 1);
                x.trans = t;
                if (x.ok) la.push_back(x);
                Layout y = match(B.legs, FB, t == 0);
                y.trans = t;
                if (y.ok) lb.push_back(y);
            }
            const int64_t bytesA = (int64_t)A.keys.size() << A.legs.size();
            const int64_t bytesB = (int64_t)B.keys.size() << B.legs.size();
            bool permA = true, permB = true;
            int transA = 0, transB = 0;
            std::vector<int> bt_order = Bt, k_order = K;
            bool done = false;
            for (auto& x : la)
                for (auto& y : lb)
                    if (!done && x.bt == y.bt && x.k == y.k) {
                        permA = permB = false;
                        transA = x.trans;
                        transB = y.trans;
                        bt_order = x.bt;
                        k_order = x.k;
                        done = true;
                    }
            if (!done) {
                if (!la.empty() && (bytesA >= bytesB || lb.empty())) {
                    permA = false;
                    transA = la[0].trans;
                    bt_order = la[0].bt;
                    k_order = la[0].k;
                } else if (!lb.empty()) {
                    permB = false;
                    transB = lb[0].trans;
                    bt_order = lb[0].bt;
                    k_order = lb[0].k;
                }
            }
            // free legs keep their operand's relative order
            auto ordered_free = [](const std::vector<int>& legs, const std::vector<int>& F) {
                std::vector<int> out;
                for (int e : legs)
                    if (std::find(F.begin(), F.end(), e) != F.end()) out.push_back(e);
                return out;
            };
            std::vector<int> fa_order = ordered_free(A.legs, FA), fb_order = ordered_free(B.legs, FB);
            std::vector<int> a_target = bt_order, b_target = bt_order;
            a_target.insert(a_target.end(), fa_order.begin(), fa_order.end());
            a_target.insert(a_target.end(), k_order.begin(), k_order.end());
            b_target.insert(b_target.end(), k_order.begin(), k_order.end());
            b_target.insert(b_target.end(), fb_order.begin(), fb_order.end());
            Ref opA = A.buf, opB = B.buf;
            // orientation: C = A B (legs bt|FA|FB) or, when A is too short for an
            // MFMA row tile and B is not, C^T = B^T A^T (legs bt|FB|FA)
            const bool swap = FA.size() < 5 && FB.size() >= 5;
            const int64_t ninst = (int64_t)C.keys.size();
            const int64_t nbatch = int64_t(1) << rb;
            auto posin = [](const NodeInfo& X, int e) {
                return (int)X.legs.size() - 1 - (int)(std::find(X.legs.begin(), X.legs.end(), e) - X.legs.begin());
            };
            auto by_pos = [&](std::vector<int> v, const NodeInfo& X) {
                std::sort(v.begin(), v.end(), [&](int a, int b) { return posin(X, a) < posin(X, b); });
                return v;
            };
            // slice offsets of an operand: instance base + the batch bits' stored offset
            auto slice_vec = [&](const NodeInfo& X, const std::vector<int>& bt_bits) {
                std::vector<int64_t> o(ninst * nbatch);
                const int64_t isz = int64_t(1) << X.legs.size();
                for (int64_t i = 0; i < ninst; ++i) {
                    const int64_t xi = X.keys.size() == 1 ? 0 : find_key(X.keys, C.keys[i] & X.mask);
                    for (int64_t b2 = 0; b2 < nbatch; ++b2) {
                        int64_t off = xi * isz;
                        for (int q = 0; q < rb; ++q)
                            if ((b2 >> q) & 1) off += int64_t(1) << posin(X, bt_bits[q]);
                        o[i * nbatch + b2] = off;
                    }
                }
                return o;
            };
            auto slice_offsets = [&](const NodeInfo& X, const std::vector<int>& bt_bits) {
                std::vector<int64_t> o = slice_vec(X, bt_bits);
                return Ref{R_CONST, ex->cbuf.add(o.data(), (int64_t)o.size() * 8)};
            };
            // Small steps (below a matrix-core tile in FP32, below the tiled
            // kernel's shape in FP64) become jobs of their tree level's grouped
            // launch, with operands read in stored order (no transpose pass).
            bool big;
            {
                GemmArgs g0{};
                g0.m_log = (int)(swap ? FB.size() : FA.size());
                g0.n_log = (int)(swap ? FA.size() : FB.size());
                g0.k_log = rk;
                const int id = select_gemm(g0, fp64, -1);
                big = fp64 ? id == K_TILED64 : kernel_class(id) == KC_MFMA;
            }
            // FP32 steps with enough work go to the matrix cores even when their
            // own shape is too small for a tile: slices that share an operand
            // are stacked into one tile (merge modes)
            const double step_flops = 8.0 * (double)ninst * (double)nbatch *
                                      std::ldexp(1.0, (int)(FA.size() + FB.size()) + rk);
            const bool heavy = step_flops >= kMfmaMinFlops && rk <= (fp64 ? 8 : 11) && FA.size() + FB.size() >= 3;
            // tiny steps stay with their level's small-step launch even when
            // their shape would fill a tile: a launch of their own costs more
            const bool long_sum = fp64 && rk > 8 && std::min(FA.size(), FB.size()) >= 5 &&
                                  step_flops >= kMfmaMinFlops;
            bool to_tile = (big && step_flops >= kTileMinFlops) || heavy || long_sum;
            if (!fp64 && small_levels && small_levels->count(st.level)) to_tile = false;
            // inner sums under 8 terms would fill less than one staged chunk of a
            // matrix-core tile (the rest zeros), at under 2 flops per byte moved:
            // such FP32 steps read and write at the small-step kernel's rate
            if (!fp64 && rk < 3) to_tile = false;
            if (grouping && mode != 2 && to_tile) {
                const int saved_split = max_ksplit;
                if (long_sum && !big && !heavy && !ksplit_user) max_ksplit = kSplitLongMax;
                plan_mfma_job(st, A, B, C, K, Bt, FA, FB, ninst, nbatch, posin, by_pos, slice_vec, fp64);
                max_ksplit = saved_split;
                node_bytes[C.gid] = C.bytes;
                push_step(std::move(st));
                continue;
            }
            if (grouping && mode != 2) {
                // column operand: one whose lowest stored leg is a free leg, so
                // that consecutive threads (consecutive columns) read adjacent elements
                const bool qa = std::find(FA.begin(), FA.end(), A.legs.back()) != FA.end();
                const bool qb = std::find(FB.begin(), FB.end(), B.legs.back()) != FB.end();
                const bool sw = qa && !qb;
                const NodeInfo& R = sw ? B : A;
                const NodeInfo& Q = sw ? A : B;
                const std::vector<int>& FR = sw ? FB : FA;
                const std::vector<int>& FQ = sw ? FA : FB;
                const int64_t bytesR = (int64_t)R.keys.size() << R.legs.size();
                const int64_t bytesQ = (int64_t)Q.keys.size() << Q.legs.size();
                const NodeInfo& big_op = bytesR >= bytesQ ? R : Q;
                std::vector<int> row_bits = by_pos(FR, R), col_bits = by_pos(FQ, Q);
                std::vector<int> k_bits = by_pos(K, big_op), bt_bits = by_pos(Bt, big_op);
                const int64_t outs_n = (ninst * nbatch) << (FR.size() + FQ.size());
                const bool split_sum = rk >= 8 && split_by_block(rk, outs_n);
                if (split_sum) {
                    // one block per output: consecutive threads take consecutive
                    // logical inner indices, so the lowest logical bits are the
                    // three lowest stored inner bits of each operand (a wave's 64
                    // lanes then read runs of 8 adjacent elements of both)
                    const std::vector<int> kr = by_pos(K, R), kq = by_pos(K, Q);
                    std::vector<int> ord;
                    auto take = [&](int leg) {
                        if (std::find(ord.begin(), ord.end(), leg) == ord.end()) ord.push_back(leg);
                    };
                    for (size_t q = 0; q < kr.size() && q < 3; ++q) take(kr[q]);
                    for (size_t q = 0; q < kq.size() && ord.size() < 6; ++q) take(kq[q]);
                    for (int leg : k_bits) take(leg);
                    k_bits = ord;
                }
                C.legs.assign(bt_bits.rbegin(), bt_bits.rend());
                C.legs.insert(C.legs.end(), row_bits.rbegin(), row_bits.rend());
                C.legs.insert(C.legs.end(), col_bits.rbegin(), col_bits.rend());
                C.bytes = ninst * (int64_t(esz) << C.legs.size());
                C.buf = Ref{R_NODE, C.gid};
                GroupJob& jb = st.job;
                jb.fp64 = fp64;
                jb.a = R.buf;
                jb.b = Q.buf;
                jb.c = C.buf;
                jb.m_log = (int)FR.size();
                jb.n_log = (int)FQ.size();
                jb.k_log = rk;
                jb.n_inst = ninst * nbatch;
                jb.split = split_sum ? 1 : 0;
                // rows per thread: the column operand's elements are reused across
                // them (up to 8; 1 for outer products, where there is no reuse)
                jb.rpt_log = jb.split || rk == 0 ? 0 : std::min(jb.m_log, 3);
                // ... but keep at least 64K threads busy
                while (jb.rpt_log > 0 && ((jb.n_inst << (jb.m_log + jb.n_log)) >> jb.rpt_log) < (int64_t(1) << 16))
                    --jb.rpt_log;
                for (size_t q = 0; q < row_bits.size(); ++q) jb.a_row[q] = (int8_t)posin(R, row_bits[q]);
                for (size_t q = 0; q < k_bits.size(); ++q) {
                    jb.a_k[q] = (int8_t)posin(R, k_bits[q]);
                    jb.b_k[q] = (int8_t)posin(Q, k_bits[q]);
                }
                for (size_t q = 0; q < col_bits.size(); ++q) jb.b_col[q] = (int8_t)posin(Q, col_bits[q]);
                jb.oa = slice_offsets(R, bt_bits);
                jb.ob = slice_offsets(Q, bt_bits);
                const double mm = std::ldexp(1.0, jb.m_log), nnn = std::ldexp(1.0, jb.n_log),
                             kk = std::ldexp(1.0, jb.k_log);
                jb.flops = 8.0 * mm * nnn * kk * (double)jb.n_inst;
                jb.bytes = (double)esz * ((double)jb.n_inst * mm * nnn + (double)R.keys.size() * nbatch * mm * kk +
                                          (double)Q.keys.size() * nbatch * kk * nnn);
                st.grouped = true;
                st.c_bytes = C.bytes;
                node_bytes[C.gid] = C.bytes;
                push_step(std::move(st));
                continue;
            }
            // Gathered operands: an FP32 step that runs on an MFMA tile and would
            // need a transpose reads both operands in their stored order instead.
            // Logical bits are ordered by stored position (lowest first), so the
            // stored layout's lowest bit is row / column / inner bit 0 and the
            // loads along it stay coalesced.  Not when that lowest bit is a batch
            // leg (the slices would interleave).
            bool gather = false;
            if (!fp64 && (permA || permB) && ex->opts.no_gather == 0) {
                GemmArgs probe{};
                probe.m_log = (int)(swap ? FB.size() : FA.size());
                probe.n_log = (int)(swap ? FA.size() : FB.size());
                probe.k_log = rk;
                const NodeInfo& R0 = swap ? B : A;
                const NodeInfo& Q0 = swap ? A : B;
                const bool bt_low = std::find(Bt.begin(), Bt.end(), R0.legs.back()) != Bt.end() ||
                                    std::find(Bt.begin(), Bt.end(), Q0.legs.back()) != Bt.end();
                gather = kernel_class(select_gemm(probe, 0, -1)) == KC_MFMA && !bt_low;
            }
            Launch gl;
            gl.kind = L_GEMM;
            gl.fp64 = fp64;
            gl.plan = plan_index;
            if (gather) {
                const NodeInfo& R = swap ? B : A;       // row operand
                const NodeInfo& Q = swap ? A : B;       // column operand
                const std::vector<int>& FR = swap ? FB : FA;
                const std::vector<int>& FQ = swap ? FA : FB;
                const int64_t bytesR = (int64_t)R.keys.size() << R.legs.size();
                const int64_t bytesQ = (int64_t)Q.keys.size() << Q.legs.size();
                std::vector<int> row_bits = by_pos(FR, R), col_bits = by_pos(FQ, Q);
                std::vector<int> k_bits = by_pos(K, bytesR >= bytesQ ? R : Q);
                std::vector<int> bt_bits(bt_order.rbegin(), bt_order.rend());
                C.legs = bt_order;
                C.legs.insert(C.legs.end(), row_bits.rbegin(), row_bits.rend());
                C.legs.insert(C.legs.end(), col_bits.rbegin(), col_bits.rend());
                C.bytes = ninst * (int64_t(esz) << C.legs.size());
                C.buf = Ref{R_NODE, C.gid};
                gl.a = R.buf;
                gl.b = Q.buf;
                gl.c = C.buf;
                gl.g.m_log = (int)FR.size();
                gl.g.n_log = (int)FQ.size();
                gl.g.k_log = rk;
                gl.g.n_inst = ninst * nbatch;
                for (size_t q = 0; q < row_bits.size(); ++q) gl.g.a_row[q] = (int8_t)posin(R, row_bits[q]);
                for (size_t q = 0; q < k_bits.size(); ++q) {
                    gl.g.a_k[q] = (int8_t)posin(R, k_bits[q]);
                    gl.g.b_k[q] = (int8_t)posin(Q, k_bits[q]);
                }
                for (size_t q = 0; q < col_bits.size(); ++q) gl.g.b_col[q] = (int8_t)posin(Q, col_bits[q]);
                gl.g.a_rowfast = std::find(FR.begin(), FR.end(), R.legs.back()) != FR.end();
                gl.g.b_colfast = std::find(FQ.begin(), FQ.end(), Q.legs.back()) != FQ.end();
                gl.oa = slice_offsets(R, bt_bits);
                gl.ob = slice_offsets(Q, bt_bits);
                gl.gather = 1;
                const double mm = std::ldexp(1.0, gl.g.m_log), nnn = std::ldexp(1.0, gl.g.n_log),
                             kk = std::ldexp(1.0, gl.g.k_log);
                gl.flops = 8.0 * mm * nnn * kk * (double)gl.g.n_inst;
                gl.bytes = (double)esz * ((double)gl.g.n_inst * mm * nnn + (double)R.keys.size() * nbatch * mm * kk +
                                          (double)Q.keys.size() * nbatch * kk * nnn);
                if (j + 1 == cl.path.size() && mode == 2) gl.plain_root = 1;
                gl.kclass = K_GATHER_BASE + select_gemm(gl.g, 0, -1);
                st.launches.push_back(gl);
            } else {
                auto emit_perm = [&](NodeInfo& X, const std::vector<int>& target, Ref* op) {
                    if (X.legs == target) return;
                    Launch pl = make_perm(X.legs, target, fp64);
                    const int64_t nb = (int64_t)X.keys.size() * (int64_t(esz) << X.legs.size());
                    const int tid = (int)temp_ref.size();
                    temp_ref.push_back(Ref{});
                    st.temp_ids.push_back(tid);
                    st.temp_bytes.push_back(nb);
                    pl.a = *op;
                    pl.c = Ref{R_TEMP, tid};
                    pl.p.n_inst = (int64_t)X.keys.size();
                    pl.bytes = 2.0 * nb;
                    pl.kclass = fp64 ? K_PERM64 : K_PERM32;
                    pl.plan = plan_index;
                    st.launches.push_back(pl);
                    *op = pl.c;
                };
                if (permA) {
                    emit_perm(A, a_target, &opA);
                    transA = 0;
                }
                if (permB) {
                    emit_perm(B, b_target, &opB);
                    transB = 0;
                }
                C.legs = bt_order;
                if (!swap) {
                    C.legs.insert(C.legs.end(), fa_order.begin(), fa_order.end());
                    C.legs.insert(C.legs.end(), fb_order.begin(), fb_order.end());
                } else {
                    C.legs.insert(C.legs.end(), fb_order.begin(), fb_order.end());
                    C.legs.insert(C.legs.end(), fa_order.begin(), fa_order.end());
                }
                C.bytes = ninst * (int64_t(esz) << C.legs.size());
                C.buf = Ref{R_NODE, C.gid};
                gl.a = opA;
                gl.b = opB;
                gl.c = C.buf;
                gl.g.m_log = (int)FA.size();
                gl.g.n_log = (int)FB.size();
                gl.g.k_log = rk;
                gl.g.transA = transA;
                gl.g.transB = transB;
                // every (instance, batch index) pair is one GEMM; operand slices of
                // one batch index are m k (n k) elements apart
                gl.g.n_inst = ninst * nbatch;
                gl.g.strideA = int64_t(1) << (A.legs.size() - rb);
                gl.g.strideB = int64_t(1) << (B.legs.size() - rb);
                auto mapping = [&](const NodeInfo& X, int* mode_out, Ref* map_out) {
                    if (X.keys.size() == 1 && rb == 0) {
                        *mode_out = 1;
                        return;
                    }
                    if (X.mask == C.mask) {
                        *mode_out = 0;     // same instances; (i, b) -> i * nbatch + b
                        return;
                    }
                    std::vector<int32_t> m(ninst * nbatch);
                    for (int64_t i = 0; i < ninst; ++i) {
                        const int64_t xi = X.keys.size() == 1 ? 0 : find_key(X.keys, C.keys[i] & X.mask);
                        for (int64_t b2 = 0; b2 < nbatch; ++b2) m[i * nbatch + b2] = (int32_t)(xi * nbatch + b2);
                    }
                    *mode_out = 2;
                    *map_out = Ref{R_CONST, ex->cbuf.add(m.data(), (int64_t)m.size() * 4)};
                };
                mapping(A, &gl.g.ia_mode, &gl.ia);
                mapping(B, &gl.g.ib_mode, &gl.ib);
                if (swap) {
                    // C^T[j][i] = sum_p B^T[j][p] A^T[p][i]: B becomes the row operand
                    std::swap(gl.a, gl.b);
                    std::swap(gl.g.ia_mode, gl.g.ib_mode);
                    std::swap(gl.ia, gl.ib);
                    std::swap(gl.g.strideA, gl.g.strideB);
                    std::swap(gl.g.m_log, gl.g.n_log);
                    const int ta = gl.g.transA, tb2 = gl.g.transB;
                    gl.g.transA = 1 - tb2;
                    gl.g.transB = 1 - ta;
                }
                const double mm = std::ldexp(1.0, gl.g.m_log), nnn = std::ldexp(1.0, gl.g.n_log),
                             kk = std::ldexp(1.0, gl.g.k_log);
                gl.flops = 8.0 * mm * nnn * kk * (double)gl.g.n_inst;
                gl.bytes = (double)esz * ((double)gl.g.n_inst * mm * nnn + (double)A.keys.size() * nbatch * mm * kk +
                                          (double)B.keys.size() * nbatch * kk * nnn);
                if (j + 1 == cl.path.size() && mode == 2) gl.plain_root = 1;
                gl.kclass = select_gemm(gl.g, fp64, -1);
                st.launches.push_back(gl);
            }
            st.c_bytes = C.bytes;
            node_bytes[C.gid] = C.bytes;
            push_step(std::move(st));
        }
        return root_out;
    }

    // Place planned steps in memory and emit their launches.  by_level: the
    // steps of one tree level (over all clusters and plans given) run together:
    // their transposes, then their GEMMs, then one grouped launch for all small
    // steps; buffers are released after the level.  Otherwise the steps run one
    // by one in the given order, each releasing its operands.
    void emit(std::vector<StepRec>& steps, int fp64, bool by_level, std::vector<Launch>* out) {
        Arena& wk = fp64 ? work2 : work;
        const int wreg = fp64 ? R_WORK2 : R_WORK;
        auto subst = [&](Ref& r) {
            if (r.region == R_NODE) r = node_ref[r.off];
            else if (r.region == R_TEMP) r = temp_ref[r.off];
        };
        std::vector<std::vector<int>> groups;
        if (by_level) {
            int maxl = 0;
            for (auto& st : steps) maxl = std::max(maxl, st.level);
            groups.resize(maxl + 1);
            for (size_t i = 0; i < steps.size(); ++i) groups[steps[i].level].push_back((int)i);
        } else {
            for (size_t i = 0; i < steps.size(); ++i) groups.push_back({(int)i});
        }
        for (size_t gi = 0; gi < groups.size(); ++gi) {
            const std::vector<int>& grp = groups[gi];
            if (grp.empty()) continue;
            const size_t first_launch = out->size();
            for (int i : grp) {
                StepRec& st = steps[i];
                node_ref[st.c_node] = st.has_fixed ? st.c_fixed : Ref{wreg, wk.alloc(st.c_bytes)};
                for (size_t q = 0; q < st.temp_ids.size(); ++q)
                    temp_ref[st.temp_ids[q]] = Ref{wreg, wk.alloc(st.temp_bytes[q])};
            }
            for (int i : grp)
                for (auto& L : steps[i].launches)
                    if (L.kind == L_PERM) {
                        subst(L.a);
                        subst(L.c);
                        out->push_back(L);
                    }
            for (int i : grp)
                for (auto& L : steps[i].launches)
                    if (L.kind == L_GEMM) {
                        subst(L.a);
                        subst(L.b);
                        subst(L.c);
                        out->push_back(L);
                    }
            Launch G;
            G.kind = L_GROUP;
            G.fp64 = fp64;
            G.kclass = fp64 ? K_GROUP64 : K_GROUP32;
            for (int i : grp) {
                if (!steps[i].grouped) continue;
                GroupJob jb = steps[i].job;
                subst(jb.a);
                subst(jb.b);
                subst(jb.c);
                const int64_t outs = jb.n_inst << (jb.m_log + jb.n_log);
                G.blocks += jb.split ? outs : ((outs >> jb.rpt_log) + 255) / 256;
                G.flops += jb.flops;
                G.bytes += jb.bytes;
                G.hjobs.push_back(jb);
            }
            for (int tile = 0; tile < K_MFMA_TILES; ++tile) {
                Launch M;
                M.kind = L_MGROUP;
                M.fp64 = fp64;
                M.mtile = tile;
                M.kclass = fp64 ? K_TILE64_GROUP : K_MFMA_GROUP_BASE + tile;
                std::vector<MfmaTile> tl;
                for (int i : grp) {
                    StepRec& st = steps[i];
                    if (!st.mgrouped || st.mtile != tile) continue;
                    MJob jb = st.mjob;
                    subst(jb.a);
                    subst(jb.b);
                    subst(jb.c);
                    subst(jb.partial);
                    const int ji = (int)M.mjobs.size();
                    for (MfmaTile t : st.mtiles) {
                        t.job = ji;
                        tl.push_back(t);
                    }
                    M.flops += jb.flops;
                    M.bytes += jb.bytes;
                    M.mjobs.push_back(jb);
                    M.plan = st.plan;
                }
                if (M.mjobs.empty()) continue;
                if ((int64_t)tl.size() >= (int64_t(1) << 31)) fail(TN_ETOOBIG, "grouped launch above 2^31 tiles");
                tl = xcd_order(tl);
                M.n_tiles = (int64_t)tl.size();
                M.tiles = Ref{R_CONST, ex->cbuf.add(tl.data(), M.n_tiles * (int64_t)sizeof(MfmaTile))};
                M.jobs = Ref{R_CONST, ex->cbuf.reserve((int64_t)M.mjobs.size() * (int64_t)sizeof(MfmaJob))};
                M.n_jobs = (int)M.mjobs.size();
                double split_bytes = 0;
                for (const MJob& jb : M.mjobs)
                    if (jb.ksplit > 1)    // partial tiles read, outputs written
                        split_bytes += (double)jb.ksplit * jb.out_bytes + jb.out_bytes;
                Launch R;
                if (split_bytes > 0) {
                    R.kind = L_MREDUCE;
                    R.fp64 = fp64;
                    R.mtile = tile;
                    R.kclass = fp64 ? K_SPLIT_REDUCE64 : K_SPLIT_REDUCE32;
                    R.plan = M.plan;
                    R.jobs = M.jobs;
                    R.tiles = M.tiles;
                    R.n_tiles = M.n_tiles;
                    R.n_jobs = M.n_jobs;
                    R.mjobs = M.mjobs;
                    R.bytes = split_bytes;
                }
                out->push_back(std::move(M));
                if (split_bytes > 0) out->push_back(std::move(R));
            }
            if (!G.hjobs.empty()) {
                G.n_jobs = (int)G.hjobs.size();
                G.plan = steps[grp[0]].plan;
                out->push_back(std::move(G));   // job records and block table: reserve_group_tables
            }
            if (by_level)
                for (size_t q = first_launch; q < out->size(); ++q) (*out)[q].level = (int)gi;
            for (int i : grp) {
                StepRec& st = steps[i];
                for (size_t q = 0; q < st.temp_ids.size(); ++q)
                    wk.release(temp_ref[st.temp_ids[q]].off, st.temp_bytes[q]);
                for (int nd : {st.a_node, st.b_node})
                    if (!node_leaf[nd] && node_ref[nd].region == wreg) wk.release(node_ref[nd].off, node_bytes[nd]);
            }
        }
    }
};

static std::vector<u128> cluster_keys(const Plan& P, const Cluster& cl, const Terms& T,
                                      const std::vector<int64_t>& live,
                                      std::vector<int32_t>* term_idx_out, int ncl, int ci) {
    std::vector<u128> keys(live.size());
    for (size_t i = 0; i < live.size(); ++i) {
        const int8_t* pat = &T.pat[live[i] * P.n_noise];
        u128 k = 0;
        for (size_t j = 0; j < cl.slots.size(); ++j) k |= (u128)(pat[cl.slots[j]] & 3) << (2 * j);
        keys[i] = k;
    }
    std::vector<u128> uk = keys;
    std::sort(uk.begin(), uk.end());
    uk.erase(std::unique(uk.begin(), uk.end()), uk.end());
    for (size_t i = 0; i < live.size(); ++i)
        (*term_idx_out)[i * ncl + ci] = (int32_t)Builder::find_key(uk, keys[i]);
    return uk;
}

// Term range of a schedule: only terms [lo, hi) of every packed term set are
// contracted (hi < 0: to the end); the others get X = 0 like pruned terms.
struct TermRange {
    int64_t lo = 0, hi = -1;
};

// When the dominant-term pass has only small steps (no tile launches), its
// jobs join the FP32 chain's small-step launch of the same tree level (or,
// where the FP32 chain has none, run as their own launch in level order on
// the main stream): no side stream, no fork / join per estimate, and half
// the launches.  A level's FP32 and FP64 jobs are independent (separate work
// regions).
static void merge_fp64_chain(tn_exec_s* ex) {
    if (ex->launches64.empty() || ex->opts.mode != TN_MODE_BATCHED) return;
    for (const Launch& L : ex->launches64)
        if (L.kind != L_GROUP || L.level < 0) return;
    for (Launch& L64 : ex->launches64) {
        auto it = std::find_if(ex->launches.begin(), ex->launches.end(),
                               [&](const Launch& L) { return L.kind == L_GROUP && L.level == L64.level; });
        if (it != ex->launches.end()) {
            Launch& G = *it;
            G.hjobs.insert(G.hjobs.end(), L64.hjobs.begin(), L64.hjobs.end());
            G.n_jobs = (int)G.hjobs.size();
            G.blocks += L64.blocks;
            G.flops += L64.flops;
            G.bytes += L64.bytes;
            G.kclass = K_GROUPMIX;
        } else {
            auto pos = std::find_if(ex->launches.begin(), ex->launches.end(),
                                    [&](const Launch& L) { return L.level > L64.level; });
            ex->launches.insert(pos, L64);
        }
    }
    ex->launches64.clear();
}

static void build_schedule(tn_exec_s* ex, int n, const tn_plan* plans, const tn_terms* terms,
                           const std::map<int, std::pair<int, double>>* level_tile = nullptr,
                           TermRange range = TermRange{}, const std::set<int>* small_levels = nullptr) {
    Builder bw;
    bw.ex = ex;
    bw.level_tile = level_tile;
    bw.small_levels = small_levels;
    bw.grouping = ex->opts.no_group == 0;
    bw.quantize_tiles = n == 1;
    if (ex->opts.max_ksplit > 0) {
        bw.max_ksplit = std::min(ex->opts.max_ksplit, 32);
        bw.ksplit_user = true;
    }
    const bool plain = ex->opts.mode == TN_MODE_PLAIN;
    std::vector<StepRec> steps32, steps64, const32, const64;
    bw.const32 = &const32;
    bw.const64 = &const64;
    for (int pi = 0; pi < n; ++pi) {
        const Plan& P = *reinterpret_cast<const Plan*>(plans[pi]);
        const Terms& T = *reinterpret_cast<const Terms*>(terms[pi]);
        if (T.plan_id != P.id) fail(TN_ESTATE, "term set belongs to another plan");
        PlanExec pe;
        pe.plan = &P;
        pe.terms = &T;
        pe.n_terms = T.n;
        std::vector<int32_t> live_index(T.n, -1);
        const int64_t r_lo = std::min<int64_t>(std::max<int64_t>(range.lo, 0), T.n);
        const int64_t r_hi = range.hi < 0 ? T.n : std::min<int64_t>(range.hi, T.n);
        for (int64_t t = r_lo; t < r_hi; ++t) {
            if (T.zero[t]) { ++pe.n_zero; continue; }
            if (T.pruned[t]) { ++pe.n_pruned; continue; }
            live_index[t] = (int32_t)pe.live_terms.size();
            pe.live_terms.push_back(t);
        }
        pe.n_live = (int64_t)pe.live_terms.size();
        // the all-dominant term is term 0 of the enumeration (a sampled term set
        // has one only if its first draw is the all-first pattern)
        if (T.n > 0 && T.lvl[0] == 0 && live_index[0] >= 0 &&
            std::all_of(T.pat.begin(), T.pat.begin() + P.n_noise, [](int8_t c) { return c == 0; }))
            pe.zero_term = 0;
        const int ncl = (int)P.clusters.size();
        // a doubled network has no slots: all of it is the value being computed
        bw.fold_const = !plain && !P.doubled;
        // one live term, the all-dominant one, recomputed in FP64 (a level-0 term
        // set, a doubled network): the FP32 chain would compute a value nothing reads
        pe.fp32_skipped = !plain && ex->opts.fp64_level0 && pe.zero_term == 0 && pe.n_live == 1;
        std::vector<int32_t> root_idx(std::max<int64_t>(1, pe.n_live * ncl), 0);
        std::vector<int64_t> root_ptr_slot(ncl, 0);
        std::vector<std::pair<int, int64_t>> plain_slots;
        for (int c = 0; c < ncl; ++c) {
            const Cluster& cl = P.clusters[c];
            std::vector<u128> keys = cluster_keys(P, cl, T, pe.live_terms, &root_idx, ncl, c);
            if (plain) {
                for (int64_t i = 0; i < pe.n_live; ++i) root_idx[i * ncl + c] = (int32_t)i;
                std::vector<u128> one = {0};
                size_t first = ex->plain_launches.size();
                std::vector<StepRec> sp;
                bw.build_cluster(P, cl, one, 2, pi, &plain_slots, Ref{}, &sp);
                bw.emit(sp, 0, false, &ex->plain_launches);
                // the root step writes into a per-term slot of a persistent buffer
                int64_t rb = std::max<int64_t>(1, pe.n_live) * 8;
                Ref root{R_CONST, ex->cbuf.reserve(rb)};
                for (size_t li = first; li < ex->plain_launches.size(); ++li)
                    if (ex->plain_launches[li].plain_root) {
                        ex->plain_launches[li].c = root;
                        ex->plain_launches[li].plain_root_stride = 8;
                    }
                pe.root32.push_back(root);
                pe.root32_inst.push_back(pe.n_live);
            } else if (pe.fp32_skipped) {
                pe.root32.push_back(Ref{R_CONST, ex->cbuf.reserve(8)});   // never read
                pe.root32_inst.push_back(1);
            } else {
                // roots stay live until finalize: the root step writes outside the work arena
                Ref keep{R_CONST, ex->cbuf.reserve((int64_t)keys.size() * 8)};
                pe.root32.push_back(bw.build_cluster(P, cl, keys, 0, pi, nullptr, keep, &steps32));
                pe.root32_inst.push_back((int64_t)keys.size());
            }
        }
        // FP64 pass for the all-dominant term
        if (pe.zero_term >= 0 && ex->opts.fp64_level0) {
            for (int c = 0; c < ncl; ++c) {
                std::vector<u128> one = {0};
                Ref keep{R_CONST, ex->cbuf.reserve(16)};
                pe.root64.push_back(bw.build_cluster(P, P.clusters[c], one, 1, pi, nullptr, keep, &steps64));
            }
        }
        if (plain) {
            Launch sf;
            sf.kind = L_SLOTFILL;
            sf.plan = pi;
            std::vector<int32_t> nidx;
            std::vector<int64_t> dsts;
            for (auto& s : plain_slots) {
                nidx.push_back(s.first);
                dsts.push_back(s.second);   // const offsets, resolved at bind
            }
            sf.sf.n = (int)plain_slots.size();
            sf.sf.n_noise = P.n_noise;
            sf.sf_noise = Ref{R_CONST, ex->cbuf.add(nidx.data(), (int64_t)nidx.size() * 4 + 4)};
            sf.sf_dst = Ref{R_CONST, ex->cbuf.add(dsts.data(), (int64_t)dsts.size() * 8 + 8)};
            std::vector<float> bank(P.n_noise * 4 * 8 + 8, 0.0f);
            for (int s = 0; s < P.n_noise; ++s)
                for (int ch = 0; ch < 4; ++ch)
                    for (int e = 0; e < 4; ++e) {
                        cd v = std::sqrt(2.0) * P.noise[s].K[ch][e];
                        bank[(s * 4 + ch) * 8 + 2 * e] = (float)v.real();
                        bank[(s * 4 + ch) * 8 + 2 * e + 1] = (float)v.imag();
                    }
            sf.sf_bank = Ref{R_CONST, ex->cbuf.add(bank.data(), (int64_t)bank.size() * 4)};
            sf.sf_pattern = Ref{R_CONST, ex->cbuf.add(T.pat.data(), (int64_t)T.pat.size() + 1)};
            ex->plain_launches.insert(ex->plain_launches.begin(), sf);
            ex->plain_terms = pe.n_live;
            // the per-term term index array: live terms
        }
        // finalize + level sums
        std::vector<double> what(T.n);
        for (int64_t t = 0; t < T.n; ++t) what[t] = std::ldexp(T.w[t], -P.n_noise);
        pe.x_out = Ref{R_CONST, ex->cbuf.reserve(std::max<int64_t>(1, T.n) * 8)};
        pe.amp_out = Ref{R_CONST, ex->cbuf.reserve(std::max<int64_t>(1, T.n) * 8)};
        pe.sums = Ref{R_HOST, ex->results_bytes};
        pe.x0 = Ref{R_HOST, ex->results_bytes + (T.level + 1) * 16};
        ex->results_bytes += (T.level + 1) * 16 + 8;
        Launch fl;
        fl.kind = L_FINALIZE;
        fl.plan = pi;
        fl.f.n_terms = T.n;
        fl.f.n_clusters = ncl;
        fl.f.zero_term = pe.root64.empty() ? -1 : pe.zero_term;
        fl.f.scalar_re = P.scalar.real();
        fl.f.scalar_im = P.scalar.imag();
        fl.f.re_value = P.doubled ? 1 : 0;
        fl.live_index = Ref{R_CONST, ex->cbuf.add(live_index.data(), std::max<int64_t>(1, T.n) * 4)};
        fl.root_idx = Ref{R_CONST, ex->cbuf.add(root_idx.data(), (int64_t)root_idx.size() * 4)};
        fl.root_ptrs = Ref{R_CONST, ex->cbuf.reserve(std::max(1, ncl) * 8)};
        fl.root64_ptrs = Ref{R_CONST, ex->cbuf.reserve(std::max(1, ncl) * 8)};
        fl.w = Ref{R_CONST, ex->cbuf.add(what.data(), std::max<int64_t>(1, T.n) * 8)};
        fl.x_out = pe.x_out;
        fl.amp_out = pe.amp_out;
        ex->tail.push_back(fl);
        pe.level_start.assign(T.level + 2, T.n);
        for (int u = T.level; u >= 0; --u) {
            int64_t s = T.n;
            for (int64_t t = 0; t < T.n; ++t)
                if (T.lvl[t] == u) { s = t; break; }
            pe.level_start[u] = s;
        }
        pe.level_start[T.level + 1] = T.n;
        for (int u = T.level; u >= 0; --u)
            if (pe.level_start[u] > pe.level_start[u + 1]) pe.level_start[u] = pe.level_start[u + 1];
        Launch ls;
        ls.kind = L_LEVELSUM;
        ls.plan = pi;
        ls.n_levels = T.level + 1;
        ls.starts = Ref{R_CONST, ex->cbuf.add(pe.level_start.data(), (int64_t)pe.level_start.size() * 8)};
        ls.x_out = pe.x_out;
        ls.sums = pe.sums;
        ex->tail.push_back(ls);
        ex->plans.push_back(std::move(pe));
    }
    // the slot-free steps first (they run once, when the schedule is bound):
    // their work buffers are released before the per-estimate steps are placed
    bw.emit(const32, 0, true, &ex->launches_const);
    bw.emit(const64, 1, true, &ex->launches_const);
    for (auto& L : ex->launches_const) L.level = -1;
    bw.emit(steps32, 0, true, &ex->launches);
    bw.emit(steps64, 1, true, &ex->launches64);
    merge_fp64_chain(ex);
    for (auto* list : {&ex->launches_const, &ex->launches, &ex->launches64})
        for (auto& L : *list)
            if (L.kind == L_GROUP) {
                if (L.blocks >= (int64_t(1) << 31)) fail(TN_ETOOBIG, "grouped launch above 2^31 blocks");
                L.jobs = Ref{R_CONST, ex->cbuf.reserve((int64_t)L.n_jobs * (int64_t)sizeof(GettJob))};
                L.table = Ref{R_CONST, ex->cbuf.reserve(L.blocks * 4)};
            }
    for (const PlanExec& pe : ex->plans) {
        ex->tail_blocks += (pe.n_terms + 255) / 256;
        ex->tail_levels = std::max(ex->tail_levels, pe.terms->level + 1);
    }
    ex->tail_jobs = Ref{R_CONST, ex->cbuf.reserve((int64_t)n * (int64_t)sizeof(TailJob))};
    ex->tail_part = Ref{R_CONST, ex->cbuf.reserve(std::max<int64_t>(1, ex->tail_blocks) * 16 * (TN_MAX_LEVEL + 1))};
    ex->const_bytes = round_up((int64_t)ex->cbuf.bytes.size(), 256);
    ex->work1_bytes = round_up(bw.work.peak, 256);
    ex->work_bytes = ex->work1_bytes + round_up(bw.work2.peak, 256);
}

static void* resolve(tn_exec_s* ex, const Ref& r) {
    if (r.region == R_HOST) return (char*)ex->results_dev + r.off;
    const int64_t region_off = r.region == R_CONST ? 0
                               : r.region == R_WORK ? ex->const_bytes
                                                    : ex->const_bytes + ex->work1_bytes;
    return ex->base + region_off + r.off;
}

static void bind(tn_exec_s* ex) {
    auto fix = [&](Launch& L) {
        if (L.kind == L_GEMM) {
            L.g.A = resolve(ex, L.a);
            L.g.B = resolve(ex, L.b);
            L.g.C = resolve(ex, L.c);
            L.g.ia = L.g.ia_mode == 2 ? (const int32_t*)resolve(ex, L.ia) : nullptr;
            L.g.ib = L.g.ib_mode == 2 ? (const int32_t*)resolve(ex, L.ib) : nullptr;
            if (L.gather) {
                L.g.oa = (const int64_t*)resolve(ex, L.oa);
                L.g.ob = (const int64_t*)resolve(ex, L.ob);
            }
        } else if (L.kind == L_PERM) {
            L.p.src = resolve(ex, L.a);
            L.p.dst = resolve(ex, L.c);
            L.p.table = (const int32_t*)resolve(ex, L.table);
        } else if (L.kind == L_GROUP) {
            GettJob* d = (GettJob*)(ex->cbuf.bytes.data() + L.jobs.off);
            int32_t* tab = (int32_t*)(ex->cbuf.bytes.data() + L.table.off);
            int64_t b0 = 0;
            for (int i = 0; i < L.n_jobs; ++i) {
                const GroupJob& h = L.hjobs[i];
                GettJob j{};
                j.A = resolve(ex, h.a);
                j.B = resolve(ex, h.b);
                j.C = resolve(ex, h.c);
                j.oa = (const int64_t*)resolve(ex, h.oa);
                j.ob = (const int64_t*)resolve(ex, h.ob);
                j.n_inst = h.n_inst;
                j.block0 = b0;
                j.m_log = h.m_log;
                j.n_log = h.n_log;
                j.k_log = h.k_log;
                j.split = h.split;
                j.rpt_log = h.rpt_log;
                std::memcpy(j.a_row, h.a_row, 32);
                std::memcpy(j.a_k, h.a_k, 32);
                std::memcpy(j.b_k, h.b_k, 32);
                std::memcpy(j.b_col, h.b_col, 32);
                const int64_t nb = gett_job_blocks(j);
                for (int64_t q = 0; q < nb; ++q) tab[b0 + q] = (int32_t)((uint32_t)i | (h.fp64 ? 0x80000000u : 0u));
                b0 += nb;
                std::memcpy(d + i, &j, sizeof(GettJob));
            }
        } else if (L.kind == L_MGROUP) {
            MfmaJob* d = (MfmaJob*)(ex->cbuf.bytes.data() + L.jobs.off);
            for (int i = 0; i < L.n_jobs; ++i) {
                const MJob& h = L.mjobs[i];
                MfmaJob j{};
                j.A = resolve(ex, h.a);
                j.B = resolve(ex, h.b);
                j.C = resolve(ex, h.c);
                j.oa = (const int64_t*)resolve(ex, h.oa);
                j.ob = (const int64_t*)resolve(ex, h.ob);
                j.oc = (const int64_t*)resolve(ex, h.oc);
                j.m_log = h.m_log;
                j.n_log = h.n_log;
                j.k_log = h.k_log;
                j.merge = h.merge;
                j.a_rowfast = h.a_rowfast;
                j.b_colfast = h.b_colfast;
                j.ksplit = h.ksplit;
                j.partial = h.ksplit > 1 ? resolve(ex, h.partial) : nullptr;
                std::memcpy(j.a_row, h.a_row, 32);
                std::memcpy(j.a_k, h.a_k, 32);
                std::memcpy(j.b_k, h.b_k, 32);
                std::memcpy(j.b_col, h.b_col, 32);
                std::memcpy(d + i, &j, sizeof(MfmaJob));
            }
        } else if (L.kind == L_SLOTFILL) {
            L.sf.noise = (const int32_t*)resolve(ex, L.sf_noise);
            L.sf.dst = (const int64_t*)resolve(ex, L.sf_dst);
            L.sf.bank = (const float*)resolve(ex, L.sf_bank);
            L.sf.pattern = (const int8_t*)resolve(ex, L.sf_pattern);
        }
    };
    for (auto& L : ex->launches_const) fix(L);
    for (auto& L : ex->launches) fix(L);
    for (auto& L : ex->launches64) fix(L);
    for (auto& L : ex->plain_launches) fix(L);
    // pointer tables written into the host staging copy before upload
    for (auto& L : ex->plain_launches)
        if (L.kind == L_SLOTFILL) {
            int64_t* d = (int64_t*)(ex->cbuf.bytes.data() + L.sf_dst.off);
            for (int i = 0; i < L.sf.n; ++i) d[i] = (int64_t)(ex->base + d[i]);
        }
    for (auto& L : ex->tail) {
        const PlanExec& pe = ex->plans[L.plan];
        if (L.kind == L_FINALIZE) {
            int64_t* rp = (int64_t*)(ex->cbuf.bytes.data() + L.root_ptrs.off);
            int64_t* rp64 = (int64_t*)(ex->cbuf.bytes.data() + L.root64_ptrs.off);
            for (size_t c = 0; c < pe.root32.size(); ++c) rp[c] = (int64_t)resolve(ex, pe.root32[c]);
            for (size_t c = 0; c < pe.root64.size(); ++c) rp64[c] = (int64_t)resolve(ex, pe.root64[c]);
            L.f.live_index = (const int32_t*)resolve(ex, L.live_index);
            L.f.root_idx = (const int32_t*)resolve(ex, L.root_idx);
            L.f.root_ptrs = (const int64_t*)resolve(ex, L.root_ptrs);
            L.f.root64_ptrs = (const int64_t*)resolve(ex, L.root64_ptrs);
            L.f.w = (const double*)resolve(ex, L.w);
            L.f.x_out = (double*)resolve(ex, L.x_out);
            L.f.amp_out = (float*)resolve(ex, L.amp_out);
            L.f.x0_fp32_out = (pe.zero_term >= 0 && ex->opts.mode == TN_MODE_BATCHED && !pe.fp32_skipped)
                                  ? (double*)resolve(ex, pe.x0) : nullptr;
        }
    }
}

// the tail records of all packed circuits (finalize arguments, level starts,
// results, first block of each circuit in the term launch)
static void bind_tail(tn_exec_s* ex) {
    TailJob* tj = (TailJob*)(ex->cbuf.bytes.data() + ex->tail_jobs.off);
    int nt = 0;
    int64_t blocks = 0;
    for (auto& L : ex->tail) {
        if (L.kind == L_FINALIZE) {
            std::memset(tj + nt, 0, sizeof(TailJob));
            tj[nt].f = L.f;
            tj[nt].block0 = blocks;
            blocks += (L.f.n_terms + 255) / 256;
        } else if (L.kind == L_LEVELSUM) {
            tj[nt].starts = (const int64_t*)resolve(ex, L.starts);
            tj[nt].sums = (double*)resolve(ex, L.sums);
            tj[nt].n_levels = L.n_levels;
            ++nt;
        }
    }
}

static void enqueue(tn_exec_s* ex, Launch& L, hipStream_t s) {
    if ((L.kind == L_GEMM && L.g.n_inst == 0) || (L.kind == L_PERM && L.p.n_inst == 0)) return;
    switch (L.kind) {
    case L_GEMM:
        launch_gemm_id(L.kclass, L.g, s);
        break;
    case L_PERM:
        if (L.fp64) launch_permute_c128(L.p, s);
        else launch_permute_c64(L.p, s);
        break;
    case L_GROUP:
        launch_gett_group((const GettJob*)resolve(ex, L.jobs), (const int32_t*)resolve(ex, L.table), L.blocks, s);
        break;
    case L_MGROUP:
        if (L.fp64)
            launch_tile64_group(L.mtile, (const MfmaJob*)resolve(ex, L.jobs), (const MfmaTile*)resolve(ex, L.tiles),
                                L.n_tiles, s);
        else
            launch_mfma_group(L.mtile, (const MfmaJob*)resolve(ex, L.jobs), (const MfmaTile*)resolve(ex, L.tiles),
                              L.n_tiles, s);
        break;
    case L_MREDUCE:
        launch_split_reduce(L.fp64, L.mtile, (const MfmaJob*)resolve(ex, L.jobs),
                            (const MfmaTile*)resolve(ex, L.tiles), L.n_tiles, s);
        break;
    case L_SLOTFILL:
        launch_slot_fill(L.sf, s);
        break;
    }
}

static void run_tail(tn_exec_s* ex, hipStream_t s);

// The slot-free steps, on one stream (FP32 and FP64 chains one after the other).
static void run_const(tn_exec_s* ex, hipStream_t s) {
    for (auto& L : ex->launches_const) enqueue(ex, L, s);
    HIPCHK(hipGetLastError());
}

// A timed launch: grouped kernels carry their events in the dispatch (the
// kernel's own start and end); per-step kernels get an event pair around them.
static void issue_timed(tn_exec_s* ex, Launch& L, hipStream_t st) {
    const bool in_dispatch = L.kind == L_GROUP || L.kind == L_MGROUP || L.kind == L_MREDUCE;
    if (L.ev_a && in_dispatch) set_launch_events(L.ev_a, L.ev_b);
    else if (L.ev_a) HIPCHK(hipEventRecord(L.ev_a, st));
    enqueue(ex, L, st);
    if (L.ev_b && !in_dispatch) HIPCHK(hipEventRecord(L.ev_b, st));
    set_launch_events(nullptr, nullptr);
}

static void issue_chain(tn_exec_s* ex, std::vector<Launch>& list, hipStream_t st) {
    for (auto& L : list) issue_timed(ex, L, st);
}

static void side_issuer_main(tn_exec_s* ex) {
    SideIssuer& w = *ex->issuer;
    (void)hipSetDevice(ex->device);
    uint64_t seen = 0;
    for (;;) {
        std::unique_lock<std::mutex> lk(w.mu);
        w.cv.wait(lk, [&] { return w.stop || w.gen > seen; });
        if (w.stop) return;
        seen = w.gen;
        lk.unlock();
        bool ok = true;
        Error e{0, ""};
        try {
            HIPCHK(hipStreamWaitEvent(ex->side, ex->ev_fork, 0));
            issue_chain(ex, ex->launches64, ex->side);
            HIPCHK(hipEventRecord(ex->ev_join, ex->side));
        } catch (const Error& x) {
            ok = false;
            e = x;
        } catch (...) {
            ok = false;
            e = Error{TN_EINVAL, "FP64 pass issue failed"};
        }
        lk.lock();
        w.failed = !ok;
        w.err = e;
        w.done = seen;
        w.cv.notify_all();
    }
}

static void stop_side_issuer(tn_exec_s* ex) {
    if (!ex->issuer) return;
    {
        std::lock_guard<std::mutex> lk(ex->issuer->mu);
        ex->issuer->stop = true;
    }
    ex->issuer->cv.notify_all();
    if (ex->issuer->th.joinable()) ex->issuer->th.join();
    ex->issuer.reset();
}

}  // namespace tn

tn_exec_s::~tn_exec_s() {
    tn::stop_side_issuer(this);
    if (gexec) (void)hipGraphExecDestroy(gexec);
    if (graph) (void)hipGraphDestroy(graph);
    if (ev0) (void)hipEventDestroy(ev0);
    if (ev1) (void)hipEventDestroy(ev1);
    for (auto e : ev_done)
        if (e) (void)hipEventDestroy(e);
    if (cap_stream) (void)hipStreamDestroy(cap_stream);
    for (auto* list : {&launches, &launches64})
        for (auto& L : *list) {
            if (L.ev_a) (void)hipEventDestroy(L.ev_a);
            if (L.ev_b) (void)hipEventDestroy(L.ev_b);
        }
    if (results_host) (void)hipHostFree(results_host);
    if (ev_fork) (void)hipEventDestroy(ev_fork);
    if (ev_join) (void)hipEventDestroy(ev_join);
    if (side) (void)hipStreamDestroy(side);
}

namespace tn {

// Direct launches with the FP64 pass: the side thread issues it after the
// fork event while this thread issues the FP32 chain; the join waits for both.
static void run_body_threaded(tn_exec_s* ex, hipStream_t s) {
    if (!ex->issuer) {
        ex->issuer.reset(new SideIssuer());
        ex->issuer->th = std::thread(side_issuer_main, ex);
    }
    SideIssuer& w = *ex->issuer;
    HIPCHK(hipEventRecord(ex->ev_fork, s));
    uint64_t my;
    {
        std::lock_guard<std::mutex> lk(w.mu);
        my = ++w.gen;
    }
    w.cv.notify_all();
    bool ok = true;
    Error e{0, ""};
    try {
        issue_chain(ex, ex->launches, s);
    } catch (const Error& x) {
        ok = false;
        e = x;
    }
    {
        std::unique_lock<std::mutex> lk(w.mu);
        w.cv.wait(lk, [&] { return w.done >= my; });
        if (ok && w.failed) {
            ok = false;
            e = w.err;
        }
    }
    if (!ok) throw e;
    HIPCHK(hipStreamWaitEvent(s, ex->ev_join, 0));
    run_tail(ex, s);
}

static void run_body(tn_exec_s* ex, hipStream_t s) {
    // The FP64 pass forks onto the side stream and joins before the finalize.
    // One thread (graph capture, term-range runs) issues the two chains level
    // by level, alternating between them, the FP32 chain first at each level.
    // (A captured graph replays each stream's branch in full before the
    // other's.)
    const bool side = !ex->launches64.empty();
    if (side) {
        HIPCHK(hipEventRecord(ex->ev_fork, s));
        HIPCHK(hipStreamWaitEvent(ex->side, ex->ev_fork, 0));
    }
    auto key = [](const Launch& L) { return L.level >= 0 ? L.level : INT_MAX; };
    auto issue = [&](Launch& L, hipStream_t st) { issue_timed(ex, L, st); };
    std::vector<Launch>& l32 = ex->launches;
    std::vector<Launch>& l64 = ex->launches64;
    size_t i32 = 0, i64 = 0;
    while (i32 < l32.size() || i64 < l64.size()) {
        if (i64 < l64.size() && (i32 == l32.size() || key(l64[i64]) < key(l32[i32]))) {
            issue(l64[i64], ex->side);
            if (++i64 == l64.size()) HIPCHK(hipEventRecord(ex->ev_join, ex->side));
        } else {
            issue(l32[i32++], s);
        }
    }
    if (side) HIPCHK(hipStreamWaitEvent(s, ex->ev_join, 0));
    run_tail(ex, s);
}

static void run_tail(tn_exec_s* ex, hipStream_t s) {
    if (ex->opts.mode == TN_MODE_PLAIN) {
        for (int64_t t = 0; t < ex->plain_terms; ++t) {
            for (auto& L : ex->plain_launches) {
                if (L.kind == L_SLOTFILL) {
                    L.sf.term = ex->plans[L.plan].live_terms[t];
                    enqueue(ex, L, s);
                } else if (L.kind == L_GEMM && L.plain_root) {
                    GemmArgs g = L.g;
                    g.C = (char*)resolve(ex, L.c) + t * L.plain_root_stride;
                    launch_gemm_c64(g, s, -1);
                } else {
                    enqueue(ex, L, s);
                }
            }
        }
    }
    launch_tail((const TailJob*)resolve(ex, ex->tail_jobs), (int)ex->plans.size(), ex->tail_blocks,
                ex->tail_levels, (double*)resolve(ex, ex->tail_part), ex->res_shift, s);
    HIPCHK(hipGetLastError());
}

// Autotuner: time every MFMA tile that fits each FP32 batched GEMM of the
// schedule (HIP events, median of a few launches on the real operands) and
// keep the fastest.  Choices are cached per (shape, transposes, batch count).
// Only the work region is written (GEMM outputs never live in the constant
// region), and it holds no data before the first run.
static void autotune(tn_exec_s* ex) {
    hipStream_t s = ex->stream;
    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    std::map<std::tuple<int, int, int, int, int, int64_t, int>, int> cache;
    for (auto& L : ex->launches) {
        if (L.kind != L_GEMM || L.fp64 || L.g.n_inst == 0 || kernel_class(L.kclass) != KC_MFMA) continue;
        auto time_gemm = [&](int id) {
            std::vector<float> ts;
            for (int rep = 0; rep < 4; ++rep) {
                HIPCHK(hipEventRecord(e0, s));
                launch_gemm_id(id, L.g, s);
                HIPCHK(hipEventRecord(e1, s));
                HIPCHK(hipEventSynchronize(e1));
                float ms = 0;
                HIPCHK(hipEventElapsedTime(&ms, e0, e1));
                if (rep > 0) ts.push_back(ms);    // first launch warms caches
            }
            std::sort(ts.begin(), ts.end());
            return ts[ts.size() / 2];
        };
        // gathered steps of one shape differ in their operand layouts; each is timed
        if (L.gather) {
            int best = L.kclass;
            float best_ms = 1e30f;
            for (int tile = 0; tile < K_MFMA_TILES; ++tile) {
                if (!mfma_tile_fits(tile, L.g)) continue;
                const float med = time_gemm(K_GATHER_BASE + tile);
                if (med < best_ms) {
                    best_ms = med;
                    best = K_GATHER_BASE + tile;
                }
            }
            L.kclass = best;
            continue;
        }
        auto key = std::make_tuple(L.g.m_log, L.g.n_log, L.g.k_log, L.g.transA, L.g.transB, L.g.n_inst, 0);
        auto it = cache.find(key);
        if (it != cache.end()) {
            L.kclass = it->second;
            continue;
        }
        int best = L.kclass;
        float best_ms = 1e30f;
        for (int tile = 0; tile < K_MFMA_TILES; ++tile) {
            if (!mfma_tile_fits(tile, L.g)) continue;
            const float med = time_gemm(tile);
            if (med < best_ms) {
                best_ms = med;
                best = tile;
            }
        }
        L.kclass = best;
        cache[key] = best;
    }
    HIPCHK(hipEventDestroy(e0));
    HIPCHK(hipEventDestroy(e1));
    HIPCHK(hipStreamSynchronize(s));
}

static std::string describe_exec(const tn_exec_s* ex) {
    std::ostringstream os;
    os.precision(17);
    os << "{\"const_bytes\":" << ex->const_bytes << ",\"work_bytes\":" << ex->work_bytes
       << ",\"work1_bytes\":" << ex->work1_bytes
       << ",\"mode\":" << ex->opts.mode << ",\"plain_terms\":" << ex->plain_terms
       << ",\"tail_blocks\":" << ex->tail_blocks << ",\"tuning\":[";
    {
        bool f1 = true;
        for (auto& kv : ex->tuning) {
            const TuneRecord& r = kv.second;
            os << (f1 ? "" : ",") << "{\"level\":" << kv.first << ",\"tile\":" << r.tile;
            if (r.tile >= 0) os << ",\"bm\":" << mfma_tile_bm(r.tile) << ",\"bn\":" << mfma_tile_bn(r.tile);
            os << ",\"model_us\":" << r.model_us << ",\"us\":[";
            for (size_t q = 0; q < r.us.size(); ++q) os << (q ? "," : "") << r.us[q];
            os << "]}";
            f1 = false;
        }
    }
    os << "],\"launches\":[";
    bool first = true;
    auto emit = [&](const Launch& L, const char* phase) {
        os << (first ? "" : ",") << "{\"phase\":\"" << phase << "\",\"kind\":" << L.kind << ",\"fp64\":" << L.fp64
           << ",\"plan\":" << L.plan << ",\"level\":" << L.level << ",\"t_ms\":" << L.t_ms << ",\"t_n\":" << L.t_n;
        first = false;
        if (L.kind == L_GEMM)
            os << ",\"m_log\":" << L.g.m_log << ",\"n_log\":" << L.g.n_log << ",\"k_log\":" << L.g.k_log
               << ",\"transA\":" << L.g.transA << ",\"transB\":" << L.g.transB << ",\"n_inst\":" << L.g.n_inst
               << ",\"ia_mode\":" << L.g.ia_mode << ",\"ib_mode\":" << L.g.ib_mode
               << ",\"strideA\":" << L.g.strideA << ",\"strideB\":" << L.g.strideB
               << ",\"a\":[" << L.a.region << "," << L.a.off << "],\"b\":[" << L.b.region << "," << L.b.off
               << "],\"c\":[" << L.c.region << "," << L.c.off << "],\"ia\":[" << L.ia.region << "," << L.ia.off
               << "],\"ib\":[" << L.ib.region << "," << L.ib.off << "],\"kernel\":\"" << kernel_name(L.kclass) << "\"";
        if (L.kind == L_PERM)
            os << ",\"r\":" << L.p.r << ",\"tb\":" << L.p.tb << ",\"n_inst\":" << L.p.n_inst << ",\"a\":["
               << L.a.region << "," << L.a.off << "],\"c\":[" << L.c.region << "," << L.c.off << "],\"table\":["
               << L.table.region << "," << L.table.off << "],\"pair\":" << L.p.pair << ",\"high_out\":[";
        if (L.kind == L_PERM) {
            for (int i = 0; i < L.p.n_high; ++i) os << (i ? "," : "") << L.p.high_out[i];
            os << "],\"high_in\":[";
            for (int i = 0; i < L.p.n_high; ++i) os << (i ? "," : "") << L.p.high_in[i];
            os << "]";
        }
        if (L.kind == L_FINALIZE)
            os << ",\"n_terms\":" << L.f.n_terms << ",\"n_clusters\":" << L.f.n_clusters << ",\"zero_term\":"
               << L.f.zero_term << ",\"scalar\":[" << L.f.scalar_re << "," << L.f.scalar_im
               << "],\"re_value\":" << L.f.re_value << ",\"live_index\":" << L.live_index.off << ",\"root_idx\":" << L.root_idx.off
               << ",\"w\":" << L.w.off << ",\"x_out\":" << L.x_out.off << ",\"amp_out\":" << L.amp_out.off;
        if (L.kind == L_LEVELSUM)
            os << ",\"n_levels\":" << L.n_levels << ",\"starts\":" << L.starts.off << ",\"x_out\":"
               << L.x_out.off << ",\"sums\":" << L.sums.off;
        if (L.kind == L_SLOTFILL)
            os << ",\"n\":" << L.sf.n << ",\"noise\":" << L.sf_noise.off << ",\"dst\":" << L.sf_dst.off
               << ",\"bank\":" << L.sf_bank.off << ",\"pattern\":" << L.sf_pattern.off
               << ",\"n_noise\":" << L.sf.n_noise;
        if (L.kind == L_MGROUP || L.kind == L_MREDUCE) {
            os << ",\"kernel\":\"" << kernel_name(L.kclass) << "\",\"bm\":" << mfma_tile_bm(L.mtile)
               << ",\"bn\":" << mfma_tile_bn(L.mtile) << ",\"n_tiles\":" << L.n_tiles << ",\"tiles\":["
               << L.tiles.region << "," << L.tiles.off << "],\"jobs\":[";
            for (int i = 0; i < L.n_jobs; ++i) {
                const MJob& h = L.mjobs[i];
                os << (i ? "," : "") << "{\"a\":[" << h.a.region << "," << h.a.off << "],\"b\":[" << h.b.region
                   << "," << h.b.off << "],\"c\":[" << h.c.region << "," << h.c.off << "],\"oa\":[" << h.oa.region
                   << "," << h.oa.off << "],\"ob\":[" << h.ob.region << "," << h.ob.off << "],\"oc\":["
                   << h.oc.region << "," << h.oc.off << "],\"m_log\":" << h.m_log << ",\"n_log\":" << h.n_log
                   << ",\"k_log\":" << h.k_log << ",\"ns\":" << h.ns << ",\"merge\":" << h.merge
                   << ",\"ksplit\":" << h.ksplit << ",\"partial\":[" << h.partial.region << "," << h.partial.off
                   << "]"
                   << ",\"a_rowfast\":" << h.a_rowfast
                   << ",\"b_colfast\":" << h.b_colfast;
                auto arr = [&](const char* nm, const int8_t* v, int n) {
                    os << ",\"" << nm << "\":[";
                    for (int q = 0; q < n; ++q) os << (q ? "," : "") << (int)v[q];
                    os << "]";
                };
                arr("a_row", h.a_row, h.m_log);
                arr("a_k", h.a_k, h.k_log);
                arr("b_k", h.b_k, h.k_log);
                arr("b_col", h.b_col, h.n_log);
                os << ",\"flops\":" << h.flops << ",\"bytes\":" << h.bytes << "}";
            }
            os << "]";
        }
        if (L.kind == L_GROUP) {
            os << ",\"kernel\":\"" << kernel_name(L.kclass) << "\",\"blocks\":" << L.blocks << ",\"jobs\":[";
            for (int i = 0; i < L.n_jobs; ++i) {
                const GroupJob& h = L.hjobs[i];
                os << (i ? "," : "") << "{\"fp64\":" << h.fp64 << ",\"a\":[" << h.a.region << "," << h.a.off
                   << "],\"b\":[" << h.b.region
                   << "," << h.b.off << "],\"c\":[" << h.c.region << "," << h.c.off << "],\"oa\":[" << h.oa.region
                   << "," << h.oa.off << "],\"ob\":[" << h.ob.region << "," << h.ob.off << "],\"n_inst\":"
                   << h.n_inst << ",\"m_log\":" << h.m_log << ",\"n_log\":" << h.n_log << ",\"k_log\":" << h.k_log
                   << ",\"split\":" << h.split << ",\"rpt_log\":" << h.rpt_log;
                auto arr = [&](const char* nm, const int8_t* v, int n) {
                    os << ",\"" << nm << "\":[";
                    for (int q = 0; q < n; ++q) os << (q ? "," : "") << (int)v[q];
                    os << "]";
                };
                arr("a_row", h.a_row, h.m_log);
                arr("a_k", h.a_k, h.k_log);
                arr("b_k", h.b_k, h.k_log);
                arr("b_col", h.b_col, h.n_log);
                os << ",\"flops\":" << h.flops << ",\"bytes\":" << h.bytes << "}";
            }
            os << "]";
        }
        if (L.kind == L_GEMM) {
            os << ",\"plain_root\":" << L.plain_root << ",\"gather\":" << L.gather;
            if (L.gather) {
                os << ",\"oa\":[" << L.oa.region << "," << L.oa.off << "],\"ob\":[" << L.ob.region << ","
                   << L.ob.off << "],\"a_rowfast\":" << L.g.a_rowfast << ",\"b_colfast\":" << L.g.b_colfast;
                auto arr = [&](const char* nm, const int8_t* v, int n) {
                    os << ",\"" << nm << "\":[";
                    for (int q = 0; q < n; ++q) os << (q ? "," : "") << (int)v[q];
                    os << "]";
                };
                arr("a_row", L.g.a_row, L.g.m_log);
                arr("a_k", L.g.a_k, L.g.k_log);
                arr("b_k", L.g.b_k, L.g.k_log);
                arr("b_col", L.g.b_col, L.g.n_log);
            }
        }
        os << ",\"flops\":" << L.flops << ",\"bytes\":" << L.bytes << "}";
    };
    for (auto& L : ex->launches_const) emit(L, "const");
    for (auto& L : ex->launches64) emit(L, "batch64");
    for (auto& L : ex->launches) emit(L, "batch");
    for (auto& L : ex->plain_launches) emit(L, "plain");
    for (auto& L : ex->tail) emit(L, "tail");
    os << "],\"plans\":[";
    for (size_t i = 0; i < ex->plans.size(); ++i) {
        const PlanExec& pe = ex->plans[i];
        os << (i ? "," : "") << "{\"n_terms\":" << pe.n_terms << ",\"n_live\":" << pe.n_live
           << ",\"zero_term\":" << pe.zero_term << ",\"x_out\":" << pe.x_out.off << ",\"amp_out\":"
           << pe.amp_out.off << ",\"sums\":" << pe.sums.off << ",\"root32\":[";
        for (size_t c = 0; c < pe.root32.size(); ++c)
            os << (c ? "," : "") << "[" << pe.root32[c].region << "," << pe.root32[c].off << "]";
        os << "],\"root64\":[";
        for (size_t c = 0; c < pe.root64.size(); ++c)
            os << (c ? "," : "") << "[" << pe.root64[c].region << "," << pe.root64[c].off << "]";
        os << "]}";
    }
    os << "]}";
    return os.str();
}

}  // namespace tn

// ===========================================================================
// extern "C" ABI
// ===========================================================================
using namespace tn;

template <class F>
static int guard(F&& f) {
    try {
        f();
        set_last_error("");
        return TN_OK;
    } catch (const Error& e) {
        set_last_error(e.msg);
        return e.code;
    } catch (const std::bad_alloc&) {
        set_last_error("host out of memory");
        return TN_ENOMEM;
    } catch (const std::exception& e) {
        set_last_error(e.what());
        return TN_EINVAL;
    }
}

namespace tn {
static void issue_estimate(tn_exec_s* ex, hipStream_t s) {
    HIPCHK(hipEventRecord(ex->ev0, s));
    if (ex->opts.use_graph) {
        if (!ex->gexec) {
            // record on a private stream (the caller's may be the null
            // stream, which cannot be captured); launch on the caller's
            if (!ex->cap_stream) HIPCHK(hipStreamCreateWithFlags(&ex->cap_stream, hipStreamNonBlocking));
            HIPCHK(hipStreamBeginCapture(ex->cap_stream, hipStreamCaptureModeThreadLocal));
            run_body(ex, ex->cap_stream);
            HIPCHK(hipStreamEndCapture(ex->cap_stream, &ex->graph));
            HIPCHK(hipGraphInstantiate(&ex->gexec, ex->graph, nullptr, nullptr, 0));
        }
        HIPCHK(hipGraphLaunch(ex->gexec, s));
    } else if (!ex->launches64.empty()) {
        run_body_threaded(ex, s);
    } else {
        run_body(ex, s);
    }
}

// One circuit's result from its level sums ((sum, comp) pairs, u = 0..level):
// A(u) as the compensated running sum, and the truncation bound of the split.
static void fill_one(const Plan& P, const Terms& T, int64_t n_live, int64_t n_zero, const double* sums,
                     double x0_fp32, tn_result& r) {
    std::memset(&r, 0, sizeof(r));
    r.level = T.level;
    r.clamped = P.clamped ? 1 : 0;
    r.n_terms = T.n;
    r.n_contracted = n_live;
    r.n_zero_weight = n_zero;
    double s = 0, c = 0;
    for (int u = 0; u <= T.level; ++u) {
        r.level_sum[u] = sums[2 * u];
        r.level_comp[u] = sums[2 * u + 1];
        double x = sums[2 * u];
        double t = s + x;
        if (std::fabs(s) >= std::fabs(x)) c += (s - t) + x;
        else c += (x - t) + s;
        s = t;
        r.A[u] = s + c;
    }
    // remainder bound: sum over |S| > level of prod ||Mbar|| prod ||M'||
    std::vector<double> poly(1, 1.0);
    for (const NoiseSplit& ns : P.noise) {
        std::vector<double> np(poly.size() + 1, 0.0);
        for (size_t i = 0; i < poly.size(); ++i) {
            np[i] += poly[i] * ns.norm_main;
            np[i + 1] += poly[i] * ns.norm_bar;
        }
        poly.swap(np);
    }
    double b = 0;
    for (size_t i = T.level + 1; i < poly.size(); ++i) b += poly[i];
    r.bound = P.trajectories ? -1.0 : b;   // a sample mean has no truncation bound
    r.x0_fp32 = x0_fp32;
}

// per-circuit results from a results region (slot 0 or a submitted copy)
static void fill_results(tn_exec_s* ex, const void* base, tn_result* results) {
    for (size_t pi = 0; pi < ex->plans.size(); ++pi) {
        const PlanExec& pe = ex->plans[pi];
        const double* hs = (const double*)((const char*)base + pe.sums.off);
        // FP32 value of the all-dominant term (diagnostic, written by the finalize)
        double x0 = -1;
        if (pe.zero_term >= 0 && ex->opts.mode == TN_MODE_BATCHED && !pe.fp32_skipped)
            x0 = *(const double*)((const char*)base + pe.x0.off);
        fill_one(*pe.plan, *pe.terms, pe.n_live, pe.n_zero, hs, x0, results[pi]);
    }
}

// Host part of tn_exec_prepare: the schedule of n packed plans over the terms
// in `range`, with its constant region staged on the host (no device call).
static std::unique_ptr<tn_exec_s> build_exec(int n, const tn_plan* plans, const tn_terms* terms,
                                             const tn_exec_opts* opts, TermRange range) {
    if (n < 1 || !plans || !terms) fail(TN_EINVAL, "need at least one plan with its terms");
    for (int i = 0; i < n; ++i)
        if (!plans[i] || !terms[i]) fail(TN_EINVAL, "null plan or term handle");
    auto ex = std::make_unique<tn_exec_s>();
    if (opts) ex->opts = *opts;
    else {
        ex->opts.mode = TN_MODE_BATCHED;
        ex->opts.use_graph = 0;
        ex->opts.fp64_level0 = 1;
    }
    if (ex->opts.time_kernels && ex->opts.use_graph)
        fail(TN_EINVAL, "per-launch kernel timing needs eager launches (use_graph = 0): events "
                        "recorded inside a captured graph cannot be timed");
    if (ex->opts.mode == TN_MODE_PLAIN) {
        ex->opts.use_graph = 0;
        if (n != 1) fail(TN_EINVAL, "PLAIN mode runs one plan at a time");
    }
    if (ex->opts.mode != TN_MODE_PLAIN && !ex->opts.no_group) {
        // The schedule is planned once as a probe, then again with what the
        // probe shows:
        //  - FP32 levels with little work run every step in their small-step
        //    launch (kSmallLevelFlops);
        //  - with one plan, a level whose matrix-core jobs chose different
        //    tile shapes runs one launch per shape, one after the other: the
        //    shape carrying most of the level's flops is imposed on the
        //    level's small jobs (each at most a quarter of that shape's
        //    flops), which then join its launch; large jobs keep their own
        //    shape (a forced shape costs them more than a launch).  Packed
        //    circuits share every level's launches already and keep each
        //    job's shape (measured slower with the merge).
        tn_exec_s probe;
        probe.opts = ex->opts;
        build_schedule(&probe, n, plans, terms, nullptr, range);
        std::map<int, std::map<int, double>> flops;   // level -> tile -> flops
        std::map<int, double> level_flops;            // level -> FP32 flops
        std::set<int> tiled;
        for (const Launch& L : probe.launches) {
            if (L.fp64 || L.level < 0) continue;
            level_flops[L.level] += L.flops;
            if (L.kind == L_MGROUP) {
                flops[L.level][L.mtile] += L.flops;
                tiled.insert(L.level);
            }
        }
        std::set<int> small;
        if (!ex->opts.all_tiles)
            for (int lv : tiled)
                if (level_flops[lv] < kSmallLevelFlops) small.insert(lv);
        std::map<int, std::pair<int, double>> level_tile;
        if (n == 1 && !ex->opts.mixed_shapes)
            for (auto& kv : flops) {
                if (kv.second.size() < 2 || small.count(kv.first)) continue;
                auto top = std::max_element(kv.second.begin(), kv.second.end(),
                                            [](const std::pair<const int, double>& a,
                                               const std::pair<const int, double>& b) { return a.second < b.second; });
                level_tile[kv.first] = {top->first, kSmallJobShare * top->second};
            }
        ex->small_levels = small;
        ex->level_tile = level_tile;
        build_schedule(ex.get(), n, plans, terms, level_tile.empty() ? nullptr : &level_tile, range,
                       small.empty() ? nullptr : &small);
    } else {
        build_schedule(ex.get(), n, plans, terms, nullptr, range);
    }
    return ex;
}

static size_t exec_need(const tn_exec_s* ex) { return (size_t)(ex->const_bytes + ex->work_bytes); }

// Autotuner of the grouped matrix-core launches (one plan).  For every FP32
// tree level with tile launches, in level order, the schedule with the model's
// choice at that level (its main shape, small jobs on their own shape where
// that saves more than a launch) is timed against the schedules with each of
// the K_MFMA_TILES shapes imposed on all of the level's matrix-core jobs, the
// levels before it keeping their chosen shapes.  Each candidate is bound to the
// workspace and timed as whole estimates with HIP events (median of 11 after a
// warm-up; the FP64 pass runs beside the FP32 chain as in use, and it slows the
// tile launches it overlaps, which timing a level's launches alone misses).  A
// shape replaces the model's choice only when its estimate is more than
// kTuneMargin faster, so a tuned schedule is not slower than the model's beyond
// timing noise.  Choices are cached by the level's job signature (shapes,
// slices) for later prepares.
constexpr double kTuneMargin = 0.05;
constexpr int kTuneModel = -1;      // the model's own choice kept
static std::mutex g_tune_mu;
static std::map<std::string, int> g_tune_cache;

static std::string level_signature(const tn_exec_s* ex, int level) {
    std::ostringstream os;
    for (const Launch& L : ex->launches)
        if (L.level == level && (L.kind == L_MGROUP || L.kind == L_GROUP) && !L.fp64) {
            for (const MJob& j : L.mjobs) os << j.m_log << "." << j.n_log << "." << j.k_log << "." << j.ns << ";";
            for (const GroupJob& j : L.hjobs) os << "g" << j.m_log << "." << j.n_log << "." << j.k_log << "." << j.n_inst << ";";
        }
    return os.str();
}

// Workspace the autotuner needs: the largest of the model's schedule and of
// every schedule it times (one level's shape imposed at a time).  Host only.
static size_t tune_need(const tn_exec_s* ex, int n, const tn_plan* plans, const tn_terms* terms,
                        TermRange range) {
    size_t need = exec_need(ex);
    if (n != 1 || ex->opts.mode != TN_MODE_BATCHED || ex->opts.no_group) return need;
    std::set<int> levels;
    for (const Launch& L : ex->launches)
        if (L.kind == L_MGROUP && !L.fp64 && L.level >= 0) levels.insert(L.level);
    for (int lv : levels)
        for (int tile = 0; tile < K_MFMA_TILES; ++tile) {
            std::map<int, std::pair<int, double>> lt = ex->level_tile;
            lt[lv] = {tile, INFINITY};
            tn_exec_s cand;
            cand.opts = ex->opts;
            build_schedule(&cand, n, plans, terms, &lt, range,
                           ex->small_levels.empty() ? nullptr : &ex->small_levels);
            need = std::max(need, exec_need(&cand));
        }
    return need;
}

static void bind_exec(tn_exec_s* ex, void* d_ws, size_t ws_bytes, hipStream_t stream);

static std::unique_ptr<tn_exec_s> tune_grouped(std::unique_ptr<tn_exec_s> ex, int n, const tn_plan* plans,
                                               const tn_terms* terms, TermRange range, void* d_ws,
                                               size_t ws_bytes, hipStream_t s) {
    if (n != 1 || ex->opts.mode != TN_MODE_BATCHED || ex->opts.no_group) return ex;
    std::set<int> levels;
    for (const Launch& L : ex->launches)
        if (L.kind == L_MGROUP && !L.fp64 && L.level >= 0) levels.insert(L.level);
    if (levels.empty()) return ex;
    const std::set<int>* small = ex->small_levels.empty() ? nullptr : &ex->small_levels;
    // one candidate schedule bound to the workspace and timed as whole
    // estimates (us), or -1 when it does not fit the workspace
    auto time_estimate = [&](const std::map<int, std::pair<int, double>>& lt) -> double {
        auto cand = std::make_unique<tn_exec_s>();
        cand->opts = ex->opts;
        cand->opts.tune = 0;
        cand->opts.time_kernels = 0;
        cand->opts.use_graph = 0;
        cand->small_levels = ex->small_levels;
        cand->level_tile = lt;
        build_schedule(cand.get(), n, plans, terms, &lt, range, small);
        if (exec_need(cand.get()) > ws_bytes) return -1.0;
        bind_exec(cand.get(), d_ws, ws_bytes, s);
        std::vector<float> ts;
        for (int rep = 0; rep < 12; ++rep) {
            issue_estimate(cand.get(), s);
            HIPCHK(hipEventRecord(cand->ev1, s));
            HIPCHK(hipEventSynchronize(cand->ev1));
            float ms = 0;
            HIPCHK(hipEventElapsedTime(&ms, cand->ev0, cand->ev1));
            if (rep > 0) ts.push_back(ms);
        }
        std::sort(ts.begin(), ts.end());
        return 1000.0 * ts[ts.size() / 2];
    };
    // level -> (tile, inf): imposed on every job of the level
    std::map<int, std::pair<int, double>> chosen;
    std::map<int, TuneRecord> table;
    for (int lv : levels) {
        const std::string sig = level_signature(ex.get(), lv);
        {
            std::lock_guard<std::mutex> lk(g_tune_mu);
            auto it = g_tune_cache.find(sig);
            if (it != g_tune_cache.end()) {
                if (it->second != kTuneModel) chosen[lv] = {it->second, INFINITY};
                table[lv] = TuneRecord{it->second, -1.0, {}};
                continue;
            }
        }
        std::map<int, std::pair<int, double>> base = ex->level_tile;
        for (auto& kv : chosen) base[kv.first] = kv.second;
        TuneRecord rec{kTuneModel, time_estimate(base), std::vector<double>(K_MFMA_TILES, -1.0)};
        double best_us = rec.model_us;
        for (int tile = 0; tile < K_MFMA_TILES; ++tile) {
            std::map<int, std::pair<int, double>> lt = base;
            lt[lv] = {tile, INFINITY};
            rec.us[tile] = time_estimate(lt);
            if (rec.us[tile] < 0) continue;
            if (best_us < 0 || rec.us[tile] < (1.0 - kTuneMargin) * best_us) {
                best_us = rec.us[tile];
                rec.tile = tile;
            }
        }
        if (rec.tile != kTuneModel) chosen[lv] = {rec.tile, INFINITY};
        table[lv] = rec;
        std::lock_guard<std::mutex> lk(g_tune_mu);
        g_tune_cache[sig] = rec.tile;
    }
    if (chosen.empty()) {
        ex->tuning = table;
        return ex;
    }
    auto tuned = std::make_unique<tn_exec_s>();
    tuned->opts = ex->opts;
    tuned->small_levels = ex->small_levels;
    tuned->level_tile = ex->level_tile;
    for (auto& kv : chosen) tuned->level_tile[kv.first] = kv.second;
    build_schedule(tuned.get(), n, plans, terms, &tuned->level_tile, range, small);
    if (exec_need(tuned.get()) > ws_bytes) {
        ex->tuning = table;
        return ex;
    }
    tuned->tuning = table;
    return tuned;
}

// Device part of tn_exec_prepare: bind the schedule to the workspace, upload
// its constants on `stream` and create its events / side stream.
static void bind_exec(tn_exec_s* ex, void* d_ws, size_t ws_bytes, hipStream_t stream) {
    const size_t need = exec_need(ex);
    if (!d_ws) fail(TN_EINVAL, "null workspace");
    if (ws_bytes < need) {
        std::ostringstream os;
        os << "workspace too small: " << ws_bytes << " < " << need << " bytes";
        fail(TN_ENOMEM, os.str());
    }
    ex->base = (char*)d_ws;
    ex->stream = stream;
    HIPCHK(hipGetDevice(&ex->device));
    ex->results_stride = std::max<int64_t>(8, (ex->results_bytes + 7) & ~int64_t(7));
    HIPCHK(hipHostMalloc(&ex->results_host, (size_t)(3 * ex->results_stride),
                         hipHostMallocMapped | hipHostMallocCoherent));
    HIPCHK(hipHostGetDevicePointer(&ex->results_dev, ex->results_host, 0));
    bind(ex);
    bind_tail(ex);
    if (!ex->launches64.empty()) {
        HIPCHK(hipStreamCreateWithFlags(&ex->side, hipStreamNonBlocking));
        HIPCHK(hipEventCreateWithFlags(&ex->ev_fork, hipEventDisableTiming));
        HIPCHK(hipEventCreateWithFlags(&ex->ev_join, hipEventDisableTiming));
    }
    if (ex->opts.time_kernels)
        for (auto* list : {&ex->launches, &ex->launches64})
            for (auto& L : *list)
                if ((L.kind == L_GEMM && L.g.n_inst > 0) || (L.kind == L_PERM && L.p.n_inst > 0) ||
                    (L.kind == L_GROUP && L.blocks > 0) ||
                    ((L.kind == L_MGROUP || L.kind == L_MREDUCE) && L.n_tiles > 0)) {
                    HIPCHK(hipEventCreate(&L.ev_a));
                    HIPCHK(hipEventCreate(&L.ev_b));
                }
    HIPCHK(hipMemcpyAsync(ex->base, ex->cbuf.bytes.data(), ex->cbuf.bytes.size(), hipMemcpyHostToDevice,
                          ex->stream));
    run_const(ex, ex->stream);
    if (ex->opts.tune) autotune(ex);
    HIPCHK(hipEventCreate(&ex->ev0));
    HIPCHK(hipEventCreate(&ex->ev1));
    for (auto& e : ex->ev_done) HIPCHK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    HIPCHK(hipStreamSynchronize(ex->stream));
    ex->bound = true;
}

static const tn_exec_opts& estimate_opts() {
    static tn_exec_opts o = [] {
        tn_exec_opts x{};
        x.mode = TN_MODE_BATCHED;
        x.use_graph = 0;
        x.fp64_level0 = 1;
        return x;
    }();
    return o;
}

static const tn_exec_opts& batch_opts() {
    static tn_exec_opts o = [] {
        tn_exec_opts x{};
        x.mode = TN_MODE_BATCHED;
        x.use_graph = 0;
        x.fp64_level0 = 0;
        return x;
    }();
    return o;
}

// ---------------------------------------------------------------------------
// Prepared schedules of tn_estimate and tn_contract_batch, kept between calls
// with the same arguments (plans, term sets, term range, workspace): the host
// schedule is built and bound once; each call uploads its constant region
// again from a page-locked copy (the caller may have used the workspace for
// something else in between) and runs it.  At most kCacheEntries entries;
// entries naming a plan or term set are dropped when it is destroyed.
// ---------------------------------------------------------------------------
struct CachedExec {
    int kind = 0;                       // 0: tn_estimate, 1: tn_contract_batch
    std::vector<const void*> plans, terms;
    TermRange range;
    void* d_ws = nullptr;
    size_t ws_bytes = 0;
    int device = 0;
    std::unique_ptr<tn_exec_s> ex;
    void* pinned = nullptr;             // page-locked copy of the constant region
    size_t pinned_bytes = 0;
    hipStream_t last_stream = nullptr;
    uint64_t last_use = 0;
    ~CachedExec() {
        // the last call's work may still be in flight on its stream
        (void)hipStreamSynchronize(last_stream);
        ex.reset();
        if (pinned) (void)hipHostFree(pinned);
    }
};

constexpr size_t kCacheEntries = 8;

static std::mutex& cache_mutex() {
    static std::mutex* m = new std::mutex();   // never destroyed: entries outlive static teardown
    return *m;
}

static std::vector<std::unique_ptr<CachedExec>>& cache_entries() {
    static auto* v = new std::vector<std::unique_ptr<CachedExec>>();
    return *v;
}

static uint64_t g_cache_clock = 0;

template <class Pred>
static void cache_evict_if(Pred pred) {
    auto& v = cache_entries();
    for (size_t i = 0; i < v.size();) {
        if (pred(*v[i])) v.erase(v.begin() + (std::ptrdiff_t)i);
        else ++i;
    }
}

static CachedExec* cache_find(int kind, int n, const tn_plan* plans, const tn_terms* terms, TermRange range,
                              void* d_ws, size_t ws_bytes) {
    if (n < 1 || !plans || !terms) return nullptr;
    for (auto& e : cache_entries()) {
        if (e->kind != kind || (int)e->plans.size() != n || e->d_ws != d_ws || e->ws_bytes != ws_bytes ||
            e->range.lo != range.lo || e->range.hi != range.hi)
            continue;
        bool same = true;
        for (int i = 0; i < n && same; ++i) same = e->plans[i] == (const void*)plans[i] && e->terms[i] == (const void*)terms[i];
        if (!same) continue;
        int dev = -1;
        HIPCHK(hipGetDevice(&dev));
        if (dev != e->device) continue;
        e->last_use = ++g_cache_clock;
        return e.get();
    }
    return nullptr;
}

static CachedExec* cache_insert(int kind, int n, const tn_plan* plans, const tn_terms* terms, TermRange range,
                                void* d_ws, size_t ws_bytes, std::unique_ptr<tn_exec_s> ex, hipStream_t s) {
    auto ce = std::make_unique<CachedExec>();
    ce->kind = kind;
    ce->plans.assign((const void* const*)plans, (const void* const*)plans + n);
    ce->terms.assign((const void* const*)terms, (const void* const*)terms + n);
    ce->range = range;
    ce->d_ws = d_ws;
    ce->ws_bytes = ws_bytes;
    ce->last_stream = s;
    bind_exec(ex.get(), d_ws, ws_bytes, s);
    ce->device = ex->device;
    ce->pinned_bytes = ex->cbuf.bytes.size();
    HIPCHK(hipHostMalloc(&ce->pinned, std::max<size_t>(1, ce->pinned_bytes), hipHostMallocDefault));
    std::memcpy(ce->pinned, ex->cbuf.bytes.data(), ce->pinned_bytes);
    ce->ex = std::move(ex);
    ce->last_use = ++g_cache_clock;
    auto& v = cache_entries();
    if (v.size() >= kCacheEntries) {
        auto lru = std::min_element(v.begin(), v.end(), [](const std::unique_ptr<CachedExec>& a,
                                                            const std::unique_ptr<CachedExec>& b) {
            return a->last_use < b->last_use;
        });
        v.erase(lru);
    }
    v.push_back(std::move(ce));
    return v.back().get();
}

static void cache_reupload(CachedExec* ce, hipStream_t s) {
    if (ce->pinned_bytes)
        HIPCHK(hipMemcpyAsync(ce->ex->base, ce->pinned, ce->pinned_bytes, hipMemcpyHostToDevice, s));
    run_const(ce->ex.get(), s);
    ce->last_stream = s;
}

// ---------------------------------------------------------------------------
// Estimates in term ranges (a workspace below the one-schedule size): each
// plan's terms run as consecutive ranges, each range a schedule of its own in
// the part of the workspace after the plan's X array; every range's X values
// are copied into that array, whose level sums are then taken by the same
// fixed-order kernel as in one schedule.
// ---------------------------------------------------------------------------
static std::vector<int64_t> level_starts(const Terms& T) {
    std::vector<int64_t> st(T.level + 2, T.n);
    for (int u = T.level; u >= 0; --u) {
        int64_t s = T.n;
        for (int64_t t = 0; t < T.n; ++t)
            if (T.lvl[t] == u) { s = t; break; }
        st[u] = s;
    }
    st[T.level + 1] = T.n;
    for (int u = T.level; u >= 0; --u)
        if (st[u] > st[u + 1]) st[u] = st[u + 1];
    return st;
}

static int64_t chunk_x_bytes(const Terms& T) { return round_up(std::max<int64_t>(1, T.n) * 8, 256); }
static int64_t chunk_starts_bytes(const Terms& T) { return round_up((int64_t)(T.level + 2) * 8, 256); }
static int64_t chunk_acc_bytes(const Terms& T) {
    return chunk_x_bytes(T) + chunk_starts_bytes(T) + round_up((int64_t)(T.level + 1) * 16, 256);
}

// Smallest workspace of a ranged estimate: every range a single term.  Every
// single-term schedule other than the all-dominant term's has the same path
// with one instance per node, so the first live term after term 0 stands for
// them all; term 0's range holds the FP64 pass.
static size_t min_workspace(int n, const tn_plan* plans, const tn_terms* terms) {
    if (n < 1 || !plans || !terms) fail(TN_EINVAL, "need at least one plan with its terms");
    size_t mx = 0;
    for (int i = 0; i < n; ++i) {
        if (!plans[i] || !terms[i]) fail(TN_EINVAL, "null plan or term handle");
        const Terms& T = *reinterpret_cast<const Terms*>(terms[i]);
        size_t m = 0;
        if (T.n > 0) m = exec_need(build_exec(1, &plans[i], &terms[i], &estimate_opts(), TermRange{0, 1}).get());
        for (int64_t t = 1; t < T.n; ++t)
            if (!T.zero[t] && !T.pruned[t]) {
                m = std::max(m, exec_need(build_exec(1, &plans[i], &terms[i], &estimate_opts(),
                                                     TermRange{t, t + 1}).get()));
                break;
            }
        mx = std::max(mx, (size_t)chunk_acc_bytes(T) + m);
    }
    return mx;
}

static void estimate_chunked(int n, const tn_plan* plans, const tn_terms* terms, char* ws, size_t ws_bytes,
                             hipStream_t s, tn_result* results) {
    for (int i = 0; i < n; ++i) {
        const Plan& P = *reinterpret_cast<const Plan*>(plans[i]);
        const Terms& T = *reinterpret_cast<const Terms*>(terms[i]);
        const int64_t acc = chunk_acc_bytes(T);
        if ((size_t)acc >= ws_bytes) fail(TN_ENOMEM, "workspace below the per-term arrays of a ranged estimate");
        double* d_x = (double*)ws;
        int64_t* d_starts = (int64_t*)(ws + chunk_x_bytes(T));
        double* d_sums = (double*)(ws + chunk_x_bytes(T) + chunk_starts_bytes(T));
        char* sub = ws + acc;
        const size_t avail = ws_bytes - (size_t)acc;
        const std::vector<int64_t> starts = level_starts(T);
        HIPCHK(hipMemcpyAsync(d_starts, starts.data(), starts.size() * 8, hipMemcpyHostToDevice, s));
        int64_t n_live = 0, n_zero = 0;
        int64_t lo = 0, cnt = T.n;
        while (lo < T.n) {
            cnt = std::min(cnt, T.n - lo);
            std::unique_ptr<tn_exec_s> ex;
            for (;;) {
                ex = build_exec(1, &plans[i], &terms[i], &estimate_opts(), TermRange{lo, lo + cnt});
                if (exec_need(ex.get()) <= avail) break;
                if (cnt == 1) fail(TN_ENOMEM, "one term's schedule does not fit the workspace");
                cnt = (cnt + 1) / 2;
            }
            bind_exec(ex.get(), sub, avail, s);
            issue_estimate(ex.get(), s);
            const PlanExec& pe = ex->plans[0];
            HIPCHK(hipMemcpyAsync(d_x + lo, (const char*)resolve(ex.get(), pe.x_out) + lo * 8, (size_t)cnt * 8,
                                  hipMemcpyDeviceToDevice, s));
            HIPCHK(hipStreamSynchronize(s));
            n_live += pe.n_live;
            n_zero += pe.n_zero;
            lo += cnt;
            cnt *= 2;   // the next range starts its search at twice this one
        }
        launch_level_sum(d_x, d_starts, T.level + 1, d_sums, s);
        HIPCHK(hipGetLastError());
        std::vector<double> hs(2 * (T.level + 1));
        HIPCHK(hipMemcpyAsync(hs.data(), d_sums, hs.size() * 8, hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        fill_one(P, T, n_live, n_zero, hs.data(), -1.0, results[i]);
    }
}

}  // namespace tn

// Fixed device workspace of tn_estimate_noalloc, for callers that cannot
// allocate: each GPU the library runs on holds one copy until the process
// ends.  In host code this name is only a handle: its device address comes
// from hipGetSymbolAddress (noalloc_scratch), once per device.
static __device__ __align__(256) unsigned char scratch[tn::kNoAllocScratchBytes];

namespace tn {

static void* noalloc_scratch() {
    static std::mutex mu;
    static void* ptr[kMaxDevices] = {};
    int dev = -1;
    HIPCHK(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) fail(TN_EINVAL, "device index beyond the fixed workspace table");
    std::lock_guard<std::mutex> lk(mu);
    if (!ptr[dev]) {
        void* p = nullptr;
        HIPCHK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) fail(TN_EHIP, "hipGetSymbolAddress gave no address for the fixed workspace");
        ptr[dev] = p;
    }
    return ptr[dev];
}

}  // namespace tn
using namespace tn;

extern "C" {

const char* tn_last_error(void) { return last_error_cstr(); }

int tn_plan_build(const tn_circuit* circ, const tn_state* psi, const tn_state* v, int32_t level,
                  const tn_plan_opts* opts, tn_plan* out) {
    return guard([&] {
        if (!out) fail(TN_EINVAL, "null output handle");
        *out = reinterpret_cast<tn_plan>(build_plan(circ, psi, v, level, opts));
    });
}

int tn_plan_build_doubled(const tn_circuit* circ, const tn_state* psi, const tn_state* v,
                          const tn_plan_opts* opts, tn_plan* out) {
    return guard([&] {
        if (!out) fail(TN_EINVAL, "null output handle");
        *out = reinterpret_cast<tn_plan>(build_plan_doubled(circ, psi, v, opts));
    });
}

int tn_plan_build_trajectories(const tn_circuit* circ, const tn_state* psi, const tn_state* v,
                               const tn_plan_opts* opts, tn_plan* out) {
    return guard([&] {
        if (!out) fail(TN_EINVAL, "null output handle");
        *out = reinterpret_cast<tn_plan>(build_plan_trajectories(circ, psi, v, opts));
    });
}

int tn_terms_trajectories(tn_plan plan, int64_t n_samples, const double* uniforms, tn_terms* out,
                          int64_t* n_terms) {
    return guard([&] {
        if (!plan || !out) fail(TN_EINVAL, "null handle");
        Terms* t = sample_terms(reinterpret_cast<Plan*>(plan), n_samples, uniforms);
        *out = reinterpret_cast<tn_terms>(t);
        if (n_terms) *n_terms = t->n;
    });
}

int tn_terms_enumerate_factored(tn_plan plan, int32_t level, tn_terms* out, int64_t* n_terms,
                                int32_t* n_groups) {
    return guard([&] {
        if (!plan || !out) fail(TN_EINVAL, "null handle");
        Terms* t = enumerate_terms_factored(reinterpret_cast<Plan*>(plan), level);
        *out = reinterpret_cast<tn_terms>(t);
        if (n_terms) *n_terms = t->n;
        if (n_groups) *n_groups = (int32_t)t->group_level.size();
    });
}

int tn_terms_groups(tn_terms terms, int64_t* starts, int32_t* level, int32_t* cluster) {
    return guard([&] {
        if (!terms) fail(TN_EINVAL, "null handle");
        const Terms* t = reinterpret_cast<const Terms*>(terms);
        if (!t->factored) fail(TN_EINVAL, "not a factored term set");
        const size_t ng = t->group_level.size();
        if (starts) std::memcpy(starts, t->group_start.data(), (ng + 1) * sizeof(int64_t));
        if (level) std::memcpy(level, t->group_level.data(), ng * sizeof(int32_t));
        if (cluster) std::memcpy(cluster, t->group_cluster.data(), ng * sizeof(int32_t));
    });
}

int tn_factored_levels(tn_terms terms, const double* group_sums, double* A) {
    return guard([&] {
        if (!terms || !group_sums || !A) fail(TN_EINVAL, "null pointer");
        factored_levels(reinterpret_cast<const Terms*>(terms), group_sums, A);
    });
}

int tn_polarization_combine(const tn_result* r, double* re, double* im) {
    return guard([&] {
        if (!r || !re || !im) fail(TN_EINVAL, "null pointer");
        const int L = r[0].level;
        for (int k = 1; k < 4; ++k)
            if (r[k].level != L) fail(TN_EINVAL, "the four results have different levels");
        // i^k for k = 0..3
        static const double wr[4] = {1, 0, -1, 0}, wi[4] = {0, 1, 0, -1};
        for (int u = 0; u <= L; ++u) {
            double sr = 0, si = 0;
            for (int k = 0; k < 4; ++k) {
                sr += wr[k] * r[k].A[u];
                si += wi[k] * r[k].A[u];
            }
            re[u] = 0.25 * sr;
            im[u] = 0.25 * si;
        }
    });
}

int tn_terms_enumerate(tn_plan plan, int32_t level, const tn_prune_opts* prune, tn_terms* out,
                       int64_t* n_terms) {
    return guard([&] {
        if (!plan || !out) fail(TN_EINVAL, "null handle");
        Terms* t = enumerate_terms(reinterpret_cast<Plan*>(plan), level, prune);
        *out = reinterpret_cast<tn_terms>(t);
        if (n_terms) *n_terms = t->n;
    });
}

int tn_terms_get(tn_terms terms, int8_t* patterns, double* weights) {
    return guard([&] {
        if (!terms) fail(TN_EINVAL, "null handle");
        Terms* t = reinterpret_cast<Terms*>(terms);
        if (patterns) std::memcpy(patterns, t->pat.data(), t->pat.size());
        if (weights) std::memcpy(weights, t->w.data(), t->w.size() * 8);
    });
}

int tn_plan_get_info(tn_plan plan, tn_plan_info* info) {
    return guard([&] {
        if (!plan || !info) fail(TN_EINVAL, "null handle");
        Plan* p = reinterpret_cast<Plan*>(plan);
        info->n_qubits = p->n_qubits;
        info->n_noise = p->n_noise;
        info->level = p->level;
        info->clamped = p->clamped;
        info->n_clusters = (int32_t)p->clusters.size();
        info->n_leaves = (int32_t)p->leaves.size();
        info->max_log_size = p->max_log;
        info->flops_per_term = 8.0 * p->cmacs_per_term;
        info->doubled = p->doubled ? 1 : 0;
        info->n_channels = p->doubled ? p->n_channels : p->n_noise;
    });
}

int tn_plan_noise(tn_plan plan, int32_t s, double* d, tn_c128* k, double* rate) {
    return guard([&] {
        if (!plan) fail(TN_EINVAL, "null handle");
        Plan* p = reinterpret_cast<Plan*>(plan);
        if (s < 0 || s >= p->n_noise) fail(TN_EINVAL, "noise index out of range");
        const NoiseSplit& ns = p->noise[s];
        for (int i = 0; i < 4; ++i) {
            if (d) d[i] = ns.d[i];
            if (k)
                for (int e = 0; e < 4; ++e) k[4 * i + e] = tn_c128{ns.K[i][e].real(), ns.K[i][e].imag()};
        }
        if (rate) *rate = ns.rate;
    });
}

int tn_plan_describe(tn_plan plan, char* buf, size_t* len) {
    return guard([&] {
        if (!plan || !len) fail(TN_EINVAL, "null handle");
        std::string s = describe_plan(reinterpret_cast<Plan*>(plan));
        if (buf && *len >= s.size() + 1) std::memcpy(buf, s.c_str(), s.size() + 1);
        *len = s.size() + 1;
    });
}

void tn_plan_destroy(tn_plan plan) {
    if (!plan) return;
    {
        std::lock_guard<std::mutex> lk(cache_mutex());
        cache_evict_if([&](const CachedExec& c) {
            return std::find(c.plans.begin(), c.plans.end(), (const void*)plan) != c.plans.end();
        });
    }
    delete reinterpret_cast<Plan*>(plan);
}
void tn_terms_destroy(tn_terms terms) {
    if (!terms) return;
    {
        std::lock_guard<std::mutex> lk(cache_mutex());
        cache_evict_if([&](const CachedExec& c) {
            return std::find(c.terms.begin(), c.terms.end(), (const void*)terms) != c.terms.end();
        });
    }
    delete reinterpret_cast<Terms*>(terms);
}

int tn_exec_prepare(int32_t n, const tn_plan* plans, const tn_terms* terms, const tn_exec_opts* opts,
                    void* d_ws, size_t ws_bytes, void* stream, size_t* need_bytes, tn_exec* out) {
    return guard([&] {
        std::unique_ptr<tn_exec_s> ex = build_exec(n, plans, terms, opts, TermRange{});
        const size_t need = ex->opts.tune ? tune_need(ex.get(), n, plans, terms, TermRange{}) : exec_need(ex.get());
        if (need_bytes) *need_bytes = need;
        if (ws_bytes == 0) {
            // size query; with `out` the caller gets an unbound handle that can
            // only be described (no device memory, no HIP call)
            if (out) *out = reinterpret_cast<tn_exec>(ex.release());
            return;
        }
        if (!out) fail(TN_EINVAL, "null output handle");
        if (!d_ws) fail(TN_EINVAL, "null workspace");
        if (ex->opts.tune && exec_need(ex.get()) <= ws_bytes)
            ex = tune_grouped(std::move(ex), n, plans, terms, TermRange{}, d_ws, ws_bytes, (hipStream_t)stream);
        bind_exec(ex.get(), d_ws, ws_bytes, (hipStream_t)stream);
        *out = reinterpret_cast<tn_exec>(ex.release());
    });
}

int tn_exec_run(tn_exec exh, void* stream, tn_result* results) {
    return guard([&] {
        tn_exec_s* ex = reinterpret_cast<tn_exec_s*>(exh);
        if (!ex || !ex->bound) fail(TN_ESTATE, "exec not prepared");
        hipStream_t s = stream ? (hipStream_t)stream : ex->stream;
        if (ex->next_ticket != ex->collected) fail(TN_ESTATE, "submitted estimates not collected yet");
        issue_estimate(ex, s);
        HIPCHK(hipEventRecord(ex->ev1, s));
        HIPCHK(hipEventSynchronize(ex->ev1));
        float ms = 0;
        HIPCHK(hipEventElapsedTime(&ms, ex->ev0, ex->ev1));
        ex->last_ms = ms;
        // per-launch breakdown (launches timed only with per-launch timing on)
        const double unrec = ex->opts.time_kernels ? 0.0 : -1.0;
        ex->gemm_ms = ex->perm_ms = ex->other_ms = unrec;
        for (auto* list : {&ex->launches, &ex->launches64})
          for (auto& L : *list)
            if (L.ev_a) {
                float dt = 0;
                HIPCHK(hipEventElapsedTime(&dt, L.ev_a, L.ev_b));
                const bool contraction = L.kind == L_GEMM || L.kind == L_GROUP || L.kind == L_MGROUP ||
                                         L.kind == L_MREDUCE;
                (contraction ? ex->gemm_ms : L.kind == L_PERM ? ex->perm_ms : ex->other_ms) += dt;
                auto& st = ex->kstat[L.kclass];
                st.first += 1;
                st.second += dt;
                ex->kflops[L.kclass] += L.flops;
                ex->kbytes[L.kclass] += L.bytes;
                L.t_ms += dt;
                L.t_n += 1;
            }
        if (results) fill_results(ex, ex->results_host, results);
    });
}

}  // extern "C"

namespace tn {

// One submitted estimate (tn_exec_submit's body): issued on s, its results
// written into host slot next_ticket & 1.
static int64_t submit_one(tn_exec_s* ex, hipStream_t s) {
    if (ex->opts.time_kernels) fail(TN_EINVAL, "per-launch timing needs tn_exec_run");
    if (ex->next_ticket - ex->collected >= 2) fail(TN_ESTATE, "two estimates outstanding: collect one first");
    // outstanding estimates share the workspace and the results slot: a
    // second one on another stream would run beside the first
    if (ex->next_ticket != ex->collected && s != ex->submit_stream)
        fail(TN_EINVAL, "estimates outstanding on another stream: submit on the same stream or collect first");
    ex->submit_stream = s;
    const int slot = (int)(ex->next_ticket & 1);
    if (ex->opts.use_graph) {
        // the captured tail writes the results region: copied to the slot
        issue_estimate(ex, s);
        const int64_t n2 = ex->results_stride / 8;   // float2-sized words
        launch_copy_c64((const float*)ex->results_dev,
                        (float*)((char*)ex->results_dev + (1 + slot) * ex->results_stride), n2, s);
    } else {
        // direct launches: the tail writes the slot itself
        ex->res_shift = (1 + slot) * ex->results_stride;
        try {
            issue_estimate(ex, s);
        } catch (...) {
            ex->res_shift = 0;
            throw;
        }
        ex->res_shift = 0;
    }
    HIPCHK(hipGetLastError());
    HIPCHK(hipEventRecord(ex->ev_done[slot], s));
    return ex->next_ticket++;
}

// Wait for the oldest outstanding estimate and fill its results (tn_exec_collect's body).
static void collect_one(tn_exec_s* ex, int64_t ticket, tn_result* results) {
    if (ticket != ex->collected || ticket >= ex->next_ticket)
        fail(TN_ESTATE, "collect submitted estimates once each, in order");
    const int slot = (int)(ticket & 1);
    HIPCHK(hipEventSynchronize(ex->ev_done[slot]));
    if (results) fill_results(ex, (const char*)ex->results_host + (1 + slot) * ex->results_stride, results);
    ++ex->collected;
}

}  // namespace tn

extern "C" {

int tn_exec_submit(tn_exec exh, void* stream, int64_t* ticket) {
    return guard([&] {
        tn_exec_s* ex = reinterpret_cast<tn_exec_s*>(exh);
        if (!ex || !ex->bound) fail(TN_ESTATE, "exec not prepared");
        const int64_t t = submit_one(ex, stream ? (hipStream_t)stream : ex->stream);
        if (ticket) *ticket = t;
    });
}

int tn_exec_collect(tn_exec exh, int64_t ticket, tn_result* results) {
    return guard([&] {
        tn_exec_s* ex = reinterpret_cast<tn_exec_s*>(exh);
        if (!ex || !ex->bound) fail(TN_ESTATE, "exec not prepared");
        collect_one(ex, ticket, results);
    });
}

int tn_exec_run_many(tn_exec exh, void* stream, int64_t count, tn_result* results) {
    return guard([&] {
        tn_exec_s* ex = reinterpret_cast<tn_exec_s*>(exh);
        if (!ex || !ex->bound) fail(TN_ESTATE, "exec not prepared");
        if (count < 0) fail(TN_EINVAL, "negative estimate count");
        if (count > 0 && !results) fail(TN_EINVAL, "null results");
        if (ex->next_ticket != ex->collected) fail(TN_ESTATE, "submitted estimates not collected yet");
        hipStream_t s = stream ? (hipStream_t)stream : ex->stream;
        const int64_t np = (int64_t)ex->plans.size();
        int64_t first = ex->next_ticket;
        try {
            for (int64_t i = 0; i < count; ++i) {
                if (i >= 2) collect_one(ex, first + i - 2, results + (i - 2) * np);
                submit_one(ex, s);
            }
            for (int64_t i = std::max<int64_t>(0, count - 2); i < count; ++i)
                collect_one(ex, first + i, results + i * np);
        } catch (...) {
            // leave nothing outstanding: wait for what was issued, drop its results
            while (ex->collected < ex->next_ticket) {
                (void)hipEventSynchronize(ex->ev_done[ex->collected & 1]);
                ++ex->collected;
            }
            throw;
        }
    });
}

int tn_exec_outputs(tn_exec exh, const double** d_x, const float** d_amp, int64_t* n_total) {
    return guard([&] {
        tn_exec_s* ex = reinterpret_cast<tn_exec_s*>(exh);
        if (!ex || !ex->bound) fail(TN_ESTATE, "exec not prepared");
        // each packed plan's outputs are an array of their own
        if (ex->plans.size() != 1)
            fail(TN_EINVAL, "packed plans: copy a plan's outputs with tn_exec_copy_outputs");
        if (d_x) *d_x = (const double*)resolve(ex, ex->plans[0].x_out);
        if (d_amp) *d_amp = (const float*)resolve(ex, ex->plans[0].amp_out);
        if (n_total) *n_total = ex->plans[0].n_terms;
    });
}

int tn_exec_kernel_stats(tn_exec exh, int32_t max, tn_kernel_stat* out, int32_t* n, int32_t reset) {
    return guard([&] {
        tn_exec_s* ex = reinterpret_cast<tn_exec_s*>(exh);
        if (!ex || !n) fail(TN_EINVAL, "null handle");
        int32_t i = 0;
        for (auto& kv : ex->kstat) {
            if (out && i < max) {
                tn_kernel_stat& k = out[i];
                std::memset(&k, 0, sizeof(k));
                std::strncpy(k.name, kernel_name(kv.first), sizeof(k.name) - 1);
                k.launches = kv.second.first;
                k.ms = kv.second.second;
                k.flops = ex->kflops[kv.first];
                k.bytes = ex->kbytes[kv.first];
            }
            ++i;
        }
        *n = i;
        if (reset) {
            ex->kstat.clear();
            ex->kflops.clear();
            ex->kbytes.clear();
            for (auto* list : {&ex->launches, &ex->launches64})
                for (auto& L : *list) {
                    L.t_ms = 0;
                    L.t_n = 0;
                }
        }
    });
}

int tn_exec_copy_outputs(tn_exec exh, int32_t plan, double* h_x, float* h_amp) {
    return guard([&] {
        tn_exec_s* ex = reinterpret_cast<tn_exec_s*>(exh);
        if (!ex || !ex->bound) fail(TN_ESTATE, "exec not prepared");
        if (plan < 0 || plan >= (int32_t)ex->plans.size()) fail(TN_EINVAL, "plan index out of range");
        const PlanExec& pe = ex->plans[plan];
        HIPCHK(hipStreamSynchronize(ex->stream));
        if (h_x && pe.n_terms)
            HIPCHK(hipMemcpy(h_x, resolve(ex, pe.x_out), pe.n_terms * 8, hipMemcpyDeviceToHost));
        if (h_amp && pe.n_terms)
            HIPCHK(hipMemcpy(h_amp, resolve(ex, pe.amp_out), pe.n_terms * 8, hipMemcpyDeviceToHost));
    });
}

int tn_exec_timing(tn_exec exh, double* total_ms, double* gemm_ms, double* permute_ms, double* other_ms) {
    return guard([&] {
        tn_exec_s* ex = reinterpret_cast<tn_exec_s*>(exh);
        if (!ex) fail(TN_EINVAL, "null handle");
        if (total_ms) *total_ms = ex->last_ms;
        if (gemm_ms) *gemm_ms = ex->gemm_ms;
        if (permute_ms) *permute_ms = ex->perm_ms;
        if (other_ms) *other_ms = ex->other_ms;
    });
}

int tn_exec_describe(tn_exec exh, char* buf, size_t* len) {
    return guard([&] {
        tn_exec_s* ex = reinterpret_cast<tn_exec_s*>(exh);
        if (!ex || !len) fail(TN_EINVAL, "null handle");
        std::string s = describe_exec(ex);
        if (buf && *len >= s.size() + 1) std::memcpy(buf, s.c_str(), s.size() + 1);
        *len = s.size() + 1;
    });
}

int tn_exec_const_bytes(tn_exec exh, void* buf, size_t* len) {
    return guard([&] {
        tn_exec_s* ex = reinterpret_cast<tn_exec_s*>(exh);
        if (!ex || !len) fail(TN_EINVAL, "null handle");
        if (buf && *len >= ex->cbuf.bytes.size()) std::memcpy(buf, ex->cbuf.bytes.data(), ex->cbuf.bytes.size());
        *len = ex->cbuf.bytes.size();
    });
}

void tn_exec_destroy(tn_exec exh) { delete reinterpret_cast<tn_exec_s*>(exh); }

int tn_plan_workspace(int32_t n, const tn_plan* plans, const tn_terms* terms, size_t* min_bytes,
                      size_t* full_bytes) {
    return guard([&] {
        if (!min_bytes && !full_bytes) fail(TN_EINVAL, "null output");
        if (full_bytes) *full_bytes = exec_need(build_exec(n, plans, terms, &estimate_opts(), TermRange{}).get());
        if (min_bytes) *min_bytes = min_workspace(n, plans, terms);
    });
}

int tn_estimate(int32_t n, const tn_plan* plans, const tn_terms* terms, void* d_ws, size_t ws_bytes,
                void* stream, tn_result* results) {
    return guard([&] {
        if (!results) fail(TN_EINVAL, "null results");
        if (!d_ws || ws_bytes == 0) fail(TN_EINVAL, "tn_estimate needs a workspace (d_ws, ws_bytes > 0)");
        hipStream_t s = (hipStream_t)stream;
        std::lock_guard<std::mutex> lk(cache_mutex());
        CachedExec* ce = cache_find(0, n, plans, terms, TermRange{}, d_ws, ws_bytes);
        if (!ce) {
            std::unique_ptr<tn_exec_s> ex = build_exec(n, plans, terms, &estimate_opts(), TermRange{});
            if (exec_need(ex.get()) > ws_bytes) {
                // below the one-schedule size: term ranges one after another
                const size_t mn = min_workspace(n, plans, terms);
                if (ws_bytes < mn) {
                    std::ostringstream os;
                    os << "workspace too small: " << ws_bytes << " < " << mn
                       << " bytes (the minimum: one term per range; " << exec_need(ex.get())
                       << " bytes run the estimate as one schedule)";
                    fail(TN_ENOMEM, os.str());
                }
                estimate_chunked(n, plans, terms, (char*)d_ws, ws_bytes, s, results);
                return;
            }
            ce = cache_insert(0, n, plans, terms, TermRange{}, d_ws, ws_bytes, std::move(ex), s);
        } else {
            cache_reupload(ce, s);
        }
        tn_exec_s* ex = ce->ex.get();
        if (ex->next_ticket != ex->collected) fail(TN_ESTATE, "cached schedule has estimates outstanding");
        issue_estimate(ex, s);
        HIPCHK(hipEventRecord(ex->ev1, s));
        HIPCHK(hipEventSynchronize(ex->ev1));
        fill_results(ex, ex->results_host, results);
    });
}

int tn_contract_batch(int32_t n, const tn_plan* plans, const tn_terms* terms, int64_t first, int64_t count,
                      void* d_amp, void* d_ws, size_t ws_bytes, void* stream) {
    return guard([&] {
        if (n < 1 || !plans || !terms) fail(TN_EINVAL, "need at least one plan with its terms");
        if (first < 0 || count < 0) fail(TN_EINVAL, "bad term range");
        for (int i = 0; i < n; ++i) {
            if (!plans[i] || !terms[i]) fail(TN_EINVAL, "null plan or term handle");
            const Terms* t = reinterpret_cast<const Terms*>(terms[i]);
            if (first + count > t->n) fail(TN_EINVAL, "term range beyond the term set");
        }
        if (count == 0) return;
        if (!d_amp) fail(TN_EINVAL, "null amplitude output");
        if (!d_ws || ws_bytes == 0) fail(TN_EINVAL, "tn_contract_batch needs a workspace (d_ws, ws_bytes > 0)");
        hipStream_t s = (hipStream_t)stream;
        const TermRange range{first, first + count};
        std::lock_guard<std::mutex> lk(cache_mutex());
        CachedExec* ce = cache_find(1, n, plans, terms, range, d_ws, ws_bytes);
        if (!ce) {
            std::unique_ptr<tn_exec_s> ex = build_exec(n, plans, terms, &batch_opts(), range);
            if (exec_need(ex.get()) > ws_bytes) {
                std::ostringstream os;
                os << "workspace too small for terms [" << first << ", " << first + count << "): " << ws_bytes
                   << " < " << exec_need(ex.get()) << " bytes";
                fail(TN_ENOMEM, os.str());
            }
            ce = cache_insert(1, n, plans, terms, range, d_ws, ws_bytes, std::move(ex), s);
        } else {
            cache_reupload(ce, s);
        }
        tn_exec_s* e = ce->ex.get();
        if (!e->bound) fail(TN_ESTATE, "schedule not bound to the workspace");
        run_body(e, s);
        for (int i = 0; i < n; ++i) {
            const PlanExec& pe = e->plans[i];
            HIPCHK(hipMemcpyAsync((char*)d_amp + (size_t)i * count * 8, (char*)resolve(e, pe.amp_out) + first * 8,
                                  (size_t)count * 8, hipMemcpyDeviceToDevice, s));
        }
        HIPCHK(hipGetLastError());
    });
}

void tn_release_cached(void) {
    std::lock_guard<std::mutex> lk(cache_mutex());
    cache_evict_if([](const CachedExec&) { return true; });
}

int tn_estimate_noalloc(int32_t n, const tn_plan* plans, const tn_terms* terms, void* stream, tn_result* results) {
    return guard([&] {
        if (!results) fail(TN_EINVAL, "null results");
        std::unique_ptr<tn_exec_s> ex = build_exec(n, plans, terms, &estimate_opts(), TermRange{});
        ex->results_stride = std::max<int64_t>(8, (ex->results_bytes + 7) & ~int64_t(7));
        const size_t res_off = (size_t)round_up((int64_t)exec_need(ex.get()), 256);
        const size_t need = res_off + (size_t)ex->results_stride;
        if (need > kNoAllocScratchBytes) {
            std::ostringstream os;
            os << "tn_estimate_noalloc: the estimate needs " << need << " bytes of workspace, above its fixed "
               << kNoAllocScratchBytes << " bytes (use tn_estimate with a workspace)";
            fail(TN_ENOMEM, os.str());
        }
        hipStream_t s = (hipStream_t)stream;
        char* base = (char*)noalloc_scratch();
        ex->base = base;
        ex->stream = s;
        HIPCHK(hipGetDevice(&ex->device));
        ex->results_dev = base + res_off;   // the tail kernels write the level sums here
        bind(ex.get());
        bind_tail(ex.get());
        // constants (every buffer that must hold something before the run),
        // the slot-free steps, then both chains and the tail on the caller's
        // stream, one after the other
        HIPCHK(hipMemcpyAsync(base, ex->cbuf.bytes.data(), ex->cbuf.bytes.size(), hipMemcpyHostToDevice, s));
        run_const(ex.get(), s);
        for (auto& L : ex->launches64) enqueue(ex.get(), L, s);
        for (auto& L : ex->launches) enqueue(ex.get(), L, s);
        run_tail(ex.get(), s);
        std::vector<unsigned char> host((size_t)ex->results_stride);
        HIPCHK(hipMemcpyAsync(host.data(), ex->results_dev, (size_t)ex->results_bytes, hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        fill_results(ex.get(), host.data(), results);
    });
}

}  // extern "C"

// ===========================================================================
// pruning features and threshold (include/tn_mlp.h)
// ===========================================================================
#include "tn_mlp.h"

extern "C" int tn_terms_features(tn_plan plan, tn_terms terms, const double* level1_x, float* out) {
    return guard([&] {
        if (!plan || !terms || !out) fail(TN_EINVAL, "null argument");
        const Plan* p = reinterpret_cast<const Plan*>(plan);
        const Terms* t = reinterpret_cast<const Terms*>(terms);
        if (t->plan_id != p->id) fail(TN_ESTATE, "term set belongs to another plan");
        term_features(p, t, level1_x, out);
    });
}

extern "C" int tn_prune_threshold(const float* pred, const double* x, int64_t n, double budget, float* tau) {
    return guard([&] {
        if (!pred || !x || !tau || n < 0 || budget < 0) fail(TN_EINVAL, "bad threshold arguments");
        std::vector<int64_t> idx(n);
        for (int64_t i = 0; i < n; ++i) idx[i] = i;
        std::sort(idx.begin(), idx.end(), [&](int64_t a, int64_t b) { return pred[a] < pred[b]; });
        // drop candidates in increasing predicted value while the dropped mass fits
        double mass = 0;
        float t = -INFINITY;
        for (int64_t j = 0; j < n; ++j) {
            const int64_t i = idx[j];
            if (mass + x[i] > budget) break;
            mass += x[i];
            t = (j + 1 < n) ? pred[idx[j + 1]] : INFINITY;
        }
        *tau = t;
    });
}

// ===========================================================================
// kernel-level entry points (include/tn_kernels.h)
// ===========================================================================
#include "tn_kernels.h"

extern "C" int tn_kernel_gemm(int32_t fp64, const void* A, const void* B, void* C, const int32_t* ia,
                              const int32_t* ib, int64_t strideA, int64_t strideB, int32_t m_log,
                              int32_t n_log, int32_t k_log, int32_t transA, int32_t transB, int64_t n_inst,
                              int32_t tile_hint, void* stream) {
    int kc = -1;
    int rc = guard([&] {
        if (m_log < 0 || n_log < 0 || k_log < 0 || m_log + n_log + k_log > 40 || n_inst < 1)
            fail(TN_EINVAL, "bad gemm shape");
        if (!A || !B || !C) fail(TN_EINVAL, "null operand");
        GemmArgs g{};
        g.A = A;
        g.B = B;
        g.C = C;
        g.ia = ia;
        g.ib = ib;
        g.ia_mode = ia ? 2 : 0;
        g.ib_mode = ib ? 2 : 0;
        g.strideA = strideA;
        g.strideB = strideB;
        g.m_log = m_log;
        g.n_log = n_log;
        g.k_log = k_log;
        g.transA = transA;
        g.transB = transB;
        g.n_inst = n_inst;
        hipStream_t s = (hipStream_t)stream;
        kc = fp64 ? launch_gemm_c128(g, s) : launch_gemm_c64(g, s, tile_hint);
        HIPCHK(hipGetLastError());
    });
    return rc == TN_OK ? kc : rc;
}

extern "C" int tn_kernel_permute(int32_t fp64, const void* src, void* dst, int64_t n_inst, int32_t r,
                                 const int32_t* perm, int32_t block_elems_log, void* stream) {
    return guard([&] {
        if (r < 0 || r > 32 || n_inst < 1 || !src || !dst || (r > 0 && !perm) || block_elems_log < 0 ||
            block_elems_log > (fp64 ? 11 : 12))
            fail(TN_EINVAL, "bad permute arguments");
        // express the permutation as source/destination leg orders
        std::vector<int> src_legs(r), dst_legs(r);
        std::vector<char> seen(r, 0);
        for (int j = 0; j < r; ++j) {
            if (perm[j] < 0 || perm[j] >= r || seen[perm[j]]) fail(TN_EINVAL, "perm is not a permutation");
            seen[perm[j]] = 1;
        }
        for (int i = 0; i < r; ++i) src_legs[r - 1 - i] = i;          // leg id = input bit
        for (int j = 0; j < r; ++j) dst_legs[r - 1 - j] = perm[j];    // output bit j holds input bit perm[j]
        tn_exec_s tmp;
        Builder bw;
        bw.ex = &tmp;
        Launch L = bw.make_perm(src_legs, dst_legs, fp64);
        hipStream_t s = (hipStream_t)stream;
        void* dtab = nullptr;
        const size_t tb = tmp.cbuf.bytes.size();
        HIPCHK(hipMalloc(&dtab, tb));
        HIPCHK(hipMemcpy(dtab, tmp.cbuf.bytes.data(), tb, hipMemcpyHostToDevice));
        L.p.src = src;
        L.p.dst = dst;
        L.p.n_inst = n_inst;
        L.p.table = (const int32_t*)((char*)dtab + L.table.off);
        L.p.elems_log = block_elems_log;
        if (fp64) launch_permute_c128(L.p, s);
        else launch_permute_c64(L.p, s);
        HIPCHK(hipGetLastError());
        HIPCHK(hipStreamSynchronize(s));
        HIPCHK(hipFree(dtab));
    });
}

static_assert(sizeof(tn_mfma_job) == sizeof(tn::MfmaJob), "tn_mfma_job layout");
static_assert(sizeof(tn_mfma_tile) == sizeof(tn::MfmaTile), "tn_mfma_tile layout");

extern "C" int tn_kernel_mfma_group(int32_t tile, const tn_mfma_job* d_jobs, const tn_mfma_tile* d_tiles,
                                    int64_t n_tiles, void* stream) {
    return guard([&] {
        if (tile < 0 || tile >= tn::K_MFMA_TILES || !d_jobs || !d_tiles || n_tiles < 0 ||
            n_tiles >= (int64_t(1) << 31))
            tn::fail(TN_EINVAL, "bad grouped launch arguments");
        tn::launch_mfma_group(tile, (const tn::MfmaJob*)d_jobs, (const tn::MfmaTile*)d_tiles, n_tiles,
                              (hipStream_t)stream);
        HIPCHK(hipGetLastError());
    });
}

extern "C" int tn_kernel_mfma_split_reduce(int32_t tile, int32_t fp64, const tn_mfma_job* d_jobs,
                                           const tn_mfma_tile* d_tiles, int64_t n_tiles, void* stream) {
    return guard([&] {
        if (tile < 0 || tile >= tn::K_MFMA_TILES || (fp64 != 0 && fp64 != 1) || !d_jobs || !d_tiles ||
            n_tiles < 0 || n_tiles >= (int64_t(1) << 31))
            tn::fail(TN_EINVAL, "bad split-reduce launch arguments");
        tn::launch_split_reduce(fp64, tile, (const tn::MfmaJob*)d_jobs, (const tn::MfmaTile*)d_tiles, n_tiles,
                                (hipStream_t)stream);
        HIPCHK(hipGetLastError());
    });
}

extern "C" int tn_kernel_group_sums(const double* d_x, const int64_t* d_starts, int32_t n_groups, double* d_out,
                                    void* stream) {
    return guard([&] {
        if (!d_x || !d_starts || !d_out || n_groups < 0 || n_groups >= (1 << 30))
            tn::fail(TN_EINVAL, "bad group-sum launch arguments");
        if (n_groups == 0) return;
        tn::launch_level_sum(d_x, d_starts, n_groups, d_out, (hipStream_t)stream);
        HIPCHK(hipGetLastError());
    });
}

