// Host-side planning: validation, noise split, reduced ket network, clusters,
// contraction path, term enumeration.  No device code.
//
// Method references: matrix representation of a channel (Section III),
// tensor permutation and SVD split (Section IV, Fig. 3), level-l terms and
// their enumeration order (Section IV, Algorithm 1).

#include <algorithm>
#include <atomic>
#include <functional>
#include <limits>
#include <memory>
#include <tuple>
#include <cmath>
#include <cstring>
#include <map>
#include <numeric>
#include <queue>
#include <random>
#include <sstream>
#include <thread>
#include <unordered_map>

#include "tn_internal.h"

namespace tn {

static thread_local std::string g_last_error;

void set_last_error(const std::string& msg) { g_last_error = msg; }
const char* last_error_cstr() { return g_last_error.c_str(); }

[[noreturn]] void fail(int code, const std::string& msg) { throw Error{code, msg}; }

// ---------------------------------------------------------------------------
// 4x4 complex Hermitian eigensolver (cyclic Jacobi).  Each rotation first
// turns a[p][q] real with a phase on column q, then applies the real
// symmetric Jacobi rotation that zeroes it.
// ---------------------------------------------------------------------------
static void mat4_mul(const cd a[4][4], const cd b[4][4], cd c[4][4]) {
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) {
            cd s = 0;
            for (int k = 0; k < 4; ++k) s += a[i][k] * b[k][j];
            c[i][j] = s;
        }
}

static void mat4_adjoint(const cd a[4][4], cd c[4][4]) {
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) c[i][j] = std::conj(a[j][i]);
}

void jacobi_hermitian4(const cd a_in[4][4], double evals[4], cd evecs[4][4]) {
    cd a[4][4], v[4][4];
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) {
            a[i][j] = 0.5 * (a_in[i][j] + std::conj(a_in[j][i]));
            v[i][j] = (i == j) ? 1.0 : 0.0;
        }
    double scale = 0;
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) scale = std::max(scale, std::abs(a[i][j]));
    if (scale == 0) scale = 1;
    for (int sweep = 0; sweep < 64; ++sweep) {
        double off = 0;
        for (int p = 0; p < 4; ++p)
            for (int q = p + 1; q < 4; ++q) off += std::norm(a[p][q]);
        if (off <= 1e-34 * scale * scale) break;
        for (int p = 0; p < 4; ++p)
            for (int q = p + 1; q < 4; ++q) {
                double apq = std::abs(a[p][q]);
                if (apq <= 1e-300) continue;
                cd ph = a[p][q] / apq;           // a[p][q] = apq * ph
                double app = a[p][p].real(), aqq = a[q][q].real();
                double tau = (aqq - app) / (2.0 * apq);
                double t = (tau >= 0 ? 1.0 : -1.0) / (std::fabs(tau) + std::sqrt(1.0 + tau * tau));
                double c = 1.0 / std::sqrt(1.0 + t * t), s = t * c;
                // G = D R with D = diag(.., conj(ph) at q, ..), R the real rotation
                cd g[4][4];
                for (int i = 0; i < 4; ++i)
                    for (int j = 0; j < 4; ++j) g[i][j] = (i == j) ? 1.0 : 0.0;
                g[p][p] = c;
                g[p][q] = s;
                g[q][p] = -s * std::conj(ph);
                g[q][q] = c * std::conj(ph);
                cd gh[4][4], tmp[4][4], na[4][4], nv[4][4];
                mat4_adjoint(g, gh);
                mat4_mul(gh, a, tmp);
                mat4_mul(tmp, g, na);
                mat4_mul(v, g, nv);
                for (int i = 0; i < 4; ++i)
                    for (int j = 0; j < 4; ++j) {
                        a[i][j] = na[i][j];
                        v[i][j] = nv[i][j];
                    }
                a[p][q] = a[q][p] = 0.0;
            }
    }
    int order[4] = {0, 1, 2, 3};
    std::sort(order, order + 4, [&](int x, int y) { return a[x][x].real() > a[y][y].real(); });
    for (int k = 0; k < 4; ++k) {
        evals[k] = a[order[k]][order[k]].real();
        for (int i = 0; i < 4; ++i) evecs[i][k] = v[i][order[k]];
    }
}

double spectral_norm4(const cd a[4][4]) {
    cd ah[4][4], h[4][4], ev[4][4];
    double w[4];
    mat4_adjoint(a, ah);
    mat4_mul(ah, a, h);
    jacobi_hermitian4(h, w, ev);
    return std::sqrt(std::max(0.0, w[0]));
}

// ---------------------------------------------------------------------------
// noise split
// ---------------------------------------------------------------------------
// trace preservation (Section II): sum_k E_k^+ E_k = I
static void check_cptp(const tn_op& op, int64_t index) {
    cd tp[2][2] = {{0, 0}, {0, 0}};
    for (int k = 0; k < op.n_kraus; ++k) {
        const tn_c128* e = op.mat + 4 * k;
        for (int i = 0; i < 2; ++i)
            for (int j = 0; j < 2; ++j)
                for (int r = 0; r < 2; ++r)
                    tp[i][j] += std::conj(cd(e[2 * r + i].re, e[2 * r + i].im)) *
                                cd(e[2 * r + j].re, e[2 * r + j].im);
    }
    double res = 0;
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j) res = std::max(res, std::abs(tp[i][j] - (i == j ? 1.0 : 0.0)));
    if (!(res <= 1e-10)) {
        std::ostringstream os;
        os << "noise at op " << index << " is not trace preserving: max|sum E^+E - I| = " << res;
        fail(TN_ENOTCPTP, os.str());
    }
}

static NoiseSplit split_noise(const tn_op& op, int64_t index) {
    NoiseSplit ns;
    ns.qubit = op.q[0];
    ns.op_index = index;
    check_cptp(op, index);
    // M = sum_k E_k (x) conj(E_k); rows (a,b) = 2a+b (ket a, bra b)
    cd m[4][4];
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) m[i][j] = 0;
    for (int k = 0; k < op.n_kraus; ++k) {
        const tn_c128* e = op.mat + 4 * k;
        for (int a = 0; a < 2; ++a)
            for (int b = 0; b < 2; ++b)
                for (int c = 0; c < 2; ++c)
                    for (int d = 0; d < 2; ++d)
                        m[2 * a + b][2 * c + d] += cd(e[2 * a + c].re, e[2 * a + c].im) *
                                                   std::conj(cd(e[2 * b + d].re, e[2 * b + d].im));
    }
    // noise rate ||M - I||_2 (Section IV)
    cd mi[4][4];
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) mi[i][j] = m[i][j] - (i == j ? 1.0 : 0.0);
    ns.rate = spectral_norm4(mi);
    // permutation (Fig. 3a): Mt[(a,c),(b,d)] = M[(a,b),(c,d)]; Hermitian PSD
    cd mt[4][4];
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b)
            for (int c = 0; c < 2; ++c)
                for (int d = 0; d < 2; ++d) mt[2 * a + c][2 * b + d] = m[2 * a + b][2 * c + d];
    double ev[4];
    cd vec[4][4];
    jacobi_hermitian4(mt, ev, vec);
    // singular values of a PSD matrix = its eigenvalues; tiny negative
    // rounding residue becomes |.|, and is flagged as an exact zero below
    // re-associate eigenvectors to the sorted |eigenvalues|
    int idx[4] = {0, 1, 2, 3};
    std::sort(idx, idx + 4, [&](int x, int y) { return std::fabs(ev[x]) > std::fabs(ev[y]); });
    for (int i = 0; i < 4; ++i) {
        int src = idx[i];
        for (int r = 0; r < 4; ++r) ns.K[i][r] = vec[r][src];   // K_i[a][c] = s_i[2a+c]
        ns.d[i] = std::fabs(ev[src]);
    }
    if (!(ns.d[1] < (1.0 - 1e-12) * ns.d[0])) {
        std::ostringstream os;
        os << "noise at op " << index << ": dominant singular value is not strictly largest (d0="
           << ns.d[0] << ", d1=" << ns.d[1] << ")";
        fail(TN_EDEGENERATE, os.str());
    }
    const double eps = std::numeric_limits<double>::epsilon();
    for (int i = 0; i < 4; ++i) ns.zero[i] = ns.d[i] <= 4.0 * eps * ns.d[0];
    // norms used by the remainder bound: ||U_0 (x) V_0|| and ||sum_{i>=1} U_i (x) V_i||
    cd mm[4][4], mb[4][4];
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b)
            for (int c = 0; c < 2; ++c)
                for (int d = 0; d < 2; ++d) {
                    // (U_i (x) V_i)[(a,b),(c,d)] = d_i K_i[a][c] conj(K_i[b][d])
                    cd s0 = ns.d[0] * ns.K[0][2 * a + c] * std::conj(ns.K[0][2 * b + d]);
                    cd sb = 0;
                    for (int i = 1; i < 4; ++i)
                        sb += ns.d[i] * ns.K[i][2 * a + c] * std::conj(ns.K[i][2 * b + d]);
                    mm[2 * a + b][2 * c + d] = s0;
                    mb[2 * a + b][2 * c + d] = sb;
                }
    ns.norm_main = spectral_norm4(mm);
    ns.norm_bar = spectral_norm4(mb);
    // ||sqrt(2) K_i||_2^2 = 2 sigma_max(K_i)^2, from the 2x2 Gram matrix
    for (int i = 0; i < 4; ++i) {
        const cd a = ns.K[i][0], b = ns.K[i][1], c = ns.K[i][2], d = ns.K[i][3];
        const double g11 = std::norm(a) + std::norm(c), g22 = std::norm(b) + std::norm(d);
        const double g12 = std::abs(std::conj(a) * b + std::conj(c) * d);
        const double tr = g11 + g22, det = g11 * g22 - g12 * g12;
        const double smax2 = 0.5 * (tr + std::sqrt(std::max(0.0, tr * tr - 4.0 * det)));
        ns.khat_norm2[i] = 2.0 * smax2;
    }
    return ns;
}

// ---------------------------------------------------------------------------
// small dense tensor algebra on the host (FP64), legs of dimension 2
// ---------------------------------------------------------------------------
// Contract two fixed tensors.  A leg they share is summed unless `keep`
// says another tensor still holds it (a diagonal gate's wire index), in which
// case it stays, once, in the result.  Result legs: x's kept legs in x order,
// then y's own legs in y order.
static Leaf contract_host(const Leaf& x, const Leaf& y, const std::function<bool(int)>& keep) {
    std::vector<int> out_legs, summed;
    for (int e : x.legs) {
        bool in_y = std::find(y.legs.begin(), y.legs.end(), e) != y.legs.end();
        if (in_y && !keep(e)) summed.push_back(e);
        else out_legs.push_back(e);
    }
    for (int e : y.legs)
        if (std::find(x.legs.begin(), x.legs.end(), e) == x.legs.end()) out_legs.push_back(e);
    Leaf out;
    out.legs = out_legs;
    const int rx = (int)x.legs.size(), ry = (int)y.legs.size(), ro = (int)out_legs.size();
    const int rs = (int)summed.size();
    auto pos = [](const std::vector<int>& legs, int e) {
        return (int)(std::find(legs.begin(), legs.end(), e) - legs.begin());
    };
    // for every output leg: its bit in x (or -1) and in y (or -1)
    std::vector<int> ox(ro, -1), oy(ro, -1), sx(rs), sy(rs);
    for (int i = 0; i < ro; ++i) {
        int px = pos(x.legs, out_legs[i]), py = pos(y.legs, out_legs[i]);
        if (px < rx) ox[i] = rx - 1 - px;
        if (py < ry) oy[i] = ry - 1 - py;
    }
    for (int i = 0; i < rs; ++i) {
        sx[i] = rx - 1 - pos(x.legs, summed[i]);
        sy[i] = ry - 1 - pos(y.legs, summed[i]);
    }
    const int64_t nout = int64_t(1) << ro;
    out.data.assign(nout, 0.0);
    for (int64_t o = 0; o < nout; ++o) {
        int64_t bx = 0, by = 0;
        for (int i = 0; i < ro; ++i)
            if ((o >> (ro - 1 - i)) & 1) {
                if (ox[i] >= 0) bx |= int64_t(1) << ox[i];
                if (oy[i] >= 0) by |= int64_t(1) << oy[i];
            }
        cd acc = 0;
        for (int64_t t = 0; t < (int64_t(1) << rs); ++t) {
            int64_t ix = bx, iy = by;
            for (int i = 0; i < rs; ++i)
                if ((t >> i) & 1) {
                    ix |= int64_t(1) << sx[i];
                    iy |= int64_t(1) << sy[i];
                }
            acc += x.data[ix] * y.data[iy];
        }
        out.data[o] = acc;
    }
    return out;
}

static bool is_diagonal(const tn_op& op) {
    const int d = 1 << op.nq;
    for (int r = 0; r < d; ++r)
        for (int c = 0; c < d; ++c)
            if (r != c && (op.mat[r * d + c].re != 0.0 || op.mat[r * d + c].im != 0.0)) return false;
    return true;
}

// ---------------------------------------------------------------------------
// reduced ket network
// ---------------------------------------------------------------------------
struct NetBuild {
    std::vector<Leaf> leaves;
    cd scalar = 1.0;
};

static void check_unitary(const tn_op& op, int64_t idx) {
    const int d = 1 << op.nq;
    double err = 0;
    for (int i = 0; i < d; ++i)
        for (int j = 0; j < d; ++j) {
            cd s = 0;
            for (int r = 0; r < d; ++r)
                s += std::conj(cd(op.mat[r * d + i].re, op.mat[r * d + i].im)) *
                     cd(op.mat[r * d + j].re, op.mat[r * d + j].im);
            err = std::max(err, std::abs(s - (i == j ? 1.0 : 0.0)));
        }
    if (!(err <= 1e-10)) {
        std::ostringstream os;
        os << "gate at op " << idx << " is not unitary: max|G^+G - I| = " << err;
        fail(TN_EINVAL, os.str());
    }
}

static NetBuild build_network(const tn_circuit* c, const tn_state* psi, const tn_state* v,
                              bool light_cone, bool diag_hyper) {
    const int n = c->n_qubits;
    NetBuild nb;
    std::vector<int> noise_of_op(c->n_ops, -1);
    int ns = 0;
    for (int64_t k = 0; k < c->n_ops; ++k)
        if (c->ops[k].kind == TN_NOISE) noise_of_op[k] = ns++;
    auto amp = [](const tn_c128* p, int q, int b) { return cd(p[2 * q + b].re, p[2 * q + b].im); };

    std::vector<std::pair<int64_t, bool>> seq;   // (op index, inverse)
    std::vector<char> touched(n, 0);
    // a bond-2 target <v| = <p| + conj(c) <q| is one 2-valued index b shared by
    // a tensor per qubit (conj of branch b's amplitudes) and the branch weights
    const bool sum2 = v->kind == TN_STATE_SUM2 || v->kind == TN_STATE_CIRCUIT_OUTPUT_SUM2;
    const bool cone_target = v->kind == TN_STATE_CIRCUIT_OUTPUT || v->kind == TN_STATE_CIRCUIT_OUTPUT_SUM2;
    auto vamp = [&](int b, int q, int s) { return amp(v->data + 2 * n * b, q, s); };
    cd branch[2] = {1.0, sum2 ? std::conj(cd(v->data[4 * n].re, v->data[4 * n].im)) : cd(0.0)};
    if (cone_target) {
        std::vector<char> keep(c->n_ops, 1);
        if (light_cone) {
            std::vector<char> live(n, 0);
            for (int64_t k = c->n_ops - 1; k >= 0; --k) {
                const tn_op& op = c->ops[k];
                if (op.kind == TN_NOISE) {
                    live[op.q[0]] = 1;
                } else {
                    bool hit = false;
                    for (int i = 0; i < op.nq; ++i) hit |= live[op.q[i]] != 0;
                    if (hit)
                        for (int i = 0; i < op.nq; ++i) live[op.q[i]] = 1;
                    else
                        keep[k] = 0;
                }
            }
        }
        for (int64_t k = 0; k < c->n_ops; ++k)
            if (keep[k]) {
                seq.push_back({k, false});
                for (int i = 0; i < c->ops[k].nq; ++i) touched[c->ops[k].q[i]] = 1;
            }
        for (int64_t k = c->n_ops - 1; k >= 0; --k)
            if (keep[k] && c->ops[k].kind == TN_GATE) seq.push_back({k, true});
        // <p_v,q | psi_q> for every qubit the reduced network does not touch
        // (per branch for a bond-2 target)
        for (int q = 0; q < n; ++q)
            if (!touched[q])
                for (int b = 0; b < (sum2 ? 2 : 1); ++b) {
                    const cd f = std::conj(vamp(b, q, 0)) * amp(psi->data, q, 0) +
                                 std::conj(vamp(b, q, 1)) * amp(psi->data, q, 1);
                    if (sum2) branch[b] *= f;
                    else nb.scalar *= f;
                }
    } else {
        for (int64_t k = 0; k < c->n_ops; ++k) seq.push_back({k, false});
        std::fill(touched.begin(), touched.end(), 1);
    }
    int edge = 0;
    std::vector<int> cur(n, -1);
    for (int q = 0; q < n; ++q)
        if (touched[q]) {
            Leaf l;
            l.legs = {edge};
            l.data = {amp(psi->data, q, 0), amp(psi->data, q, 1)};
            cur[q] = edge++;
            nb.leaves.push_back(std::move(l));
        }
    for (auto [k, inv] : seq) {
        const tn_op& op = c->ops[k];
        Leaf l;
        if (diag_hyper && op.kind == TN_GATE && is_diagonal(op)) {
            // a diagonal gate does not change the basis index of its wires: it is
            // a tensor on the current wire indices, shared with whatever else
            // touches them (hyperedge)
            const int d = 1 << op.nq;
            for (int i = 0; i < op.nq; ++i) l.legs.push_back(cur[op.q[i]]);
            l.data.resize(d);
            for (int r = 0; r < d; ++r) {
                cd g(op.mat[r * d + r].re, op.mat[r * d + r].im);
                l.data[r] = inv ? std::conj(g) : g;
            }
            nb.leaves.push_back(std::move(l));
            continue;
        }
        std::vector<int> ins, outs;
        for (int i = 0; i < op.nq; ++i) ins.push_back(cur[op.q[i]]);
        for (int i = 0; i < op.nq; ++i) {
            outs.push_back(edge);
            cur[op.q[i]] = edge++;
        }
        l.legs = outs;
        l.legs.insert(l.legs.end(), ins.begin(), ins.end());
        if (op.kind == TN_NOISE) {
            l.slot = noise_of_op[k];
        } else {
            const int d = 1 << op.nq;
            l.data.resize(d * d);
            for (int r = 0; r < d; ++r)
                for (int cc = 0; cc < d; ++cc) {
                    // element [outs..., ins...] = G[out][in] (or G^+ for the inverse)
                    cd g = inv ? std::conj(cd(op.mat[cc * d + r].re, op.mat[cc * d + r].im))
                               : cd(op.mat[r * d + cc].re, op.mat[r * d + cc].im);
                    l.data[r * d + cc] = g;
                }
        }
        nb.leaves.push_back(std::move(l));
    }
    if (sum2) {
        bool any = false;
        for (int q = 0; q < n; ++q) any |= touched[q] != 0;
        if (!any) {
            nb.scalar *= branch[0] + branch[1];
        } else {
            const int bond = edge++;
            for (int q = 0; q < n; ++q)
                if (touched[q]) {
                    Leaf l;
                    l.legs = {cur[q], bond};
                    l.data.resize(4);
                    for (int s = 0; s < 2; ++s)
                        for (int b = 0; b < 2; ++b) l.data[2 * s + b] = std::conj(vamp(b, q, s));
                    nb.leaves.push_back(std::move(l));
                }
            Leaf w;
            w.legs = {bond};
            w.data = {branch[0], branch[1]};
            nb.leaves.push_back(std::move(w));
        }
    } else if (v->kind == TN_STATE_DENSE) {
        Leaf l;
        for (int q = 0; q < n; ++q) l.legs.push_back(cur[q]);
        l.data.resize(size_t(1) << n);
        for (size_t i = 0; i < l.data.size(); ++i)
            l.data[i] = std::conj(cd(v->data[i].re, v->data[i].im));
        nb.leaves.push_back(std::move(l));
    } else {
        for (int q = 0; q < n; ++q)
            if (touched[q]) {
                Leaf l;
                l.legs = {cur[q]};
                l.data = {std::conj(amp(v->data, q, 0)), std::conj(amp(v->data, q, 1))};
                nb.leaves.push_back(std::move(l));
            }
    }
    return nb;
}

// Contract fixed tensors into fixed neighbours on the host (FP64) while the
// result is no larger than the larger operand (at most 4 legs): absorbs the
// boundary vectors, 1-qubit gates and cancelling neighbours.  Exact up to
// rounding; slot tensors are never touched.
static void fuse_fixed(NetBuild& nb) {
    std::vector<Leaf>& L = nb.leaves;
    std::vector<char> alive(L.size(), 1);
    std::unordered_map<int, std::vector<int>> owners;
    for (size_t i = 0; i < L.size(); ++i)
        for (int e : L[i].legs) owners[e].push_back((int)i);
    bool changed = true;
    while (changed) {
        changed = false;
        for (size_t i = 0; i < L.size(); ++i) {
            if (!alive[i] || L[i].slot >= 0) continue;
            // best neighbour: fixed, shares a leg, result rank <= max(rank, 4)
            int best = -1, best_rank = 1 << 30;
            for (int e : L[i].legs) {
                for (int j : owners[e]) {
                    if (j == (int)i || !alive[j] || L[j].slot >= 0) continue;
                    int shared = 0, kept = 0;
                    for (int f : L[i].legs)
                        if (std::find(L[j].legs.begin(), L[j].legs.end(), f) != L[j].legs.end()) {
                            ++shared;
                            if (owners[f].size() > 2) ++kept;
                        }
                    int r = (int)L[i].legs.size() + (int)L[j].legs.size() - 2 * shared + kept;
                    int lim = std::max<int>(4, std::max(L[i].legs.size(), L[j].legs.size()));
                    if (r <= lim && r < best_rank) {
                        best = j;
                        best_rank = r;
                    }
                }
            }
            if (best < 0) continue;
            const int ii = (int)i, jj = best;
            Leaf merged = contract_host(L[i], L[best], [&](int e) {
                for (int o : owners[e])
                    if (o != ii && o != jj) return true;
                return false;
            });
            for (int e : L[i].legs) {
                auto& v = owners[e];
                v.erase(std::remove(v.begin(), v.end(), (int)i), v.end());
            }
            for (int e : L[best].legs) {
                auto& v = owners[e];
                v.erase(std::remove(v.begin(), v.end(), best), v.end());
            }
            alive[i] = 0;
            L[best] = std::move(merged);
            for (int e : L[best].legs) owners[e].push_back(best);
            changed = true;
        }
    }
    std::vector<Leaf> out;
    for (size_t i = 0; i < L.size(); ++i) {
        if (!alive[i]) continue;
        if (L[i].slot < 0 && L[i].legs.empty()) {
            nb.scalar *= L[i].data[0];
            continue;
        }
        out.push_back(std::move(L[i]));
    }
    L.swap(out);
}

// ---------------------------------------------------------------------------
// contraction path: randomized greedy, scored by instance-weighted size
// ---------------------------------------------------------------------------
struct PathSearch {
    int level;
    std::vector<int> zcount;                 // non-zero corrections per local slot

    // number of distinct restricted patterns of a node with these slots
    double instances(uint64_t mask) const {
        double e[TN_MAX_LEVEL + 2] = {1.0};
        for (int i = 1; i <= level; ++i) e[i] = 0;
        for (int s = 0; s < 64; ++s)
            if ((mask >> s) & 1ULL)
                for (int u = level; u >= 1; --u) e[u] += e[u - 1] * zcount[s];
        double t = 0;
        for (int u = 0; u <= level; ++u) t += e[u];
        return t;
    }
};

static int union_size(const std::vector<int>& a, const std::vector<int>& b) {
    size_t i = 0, j = 0;
    int n = 0;
    while (i < a.size() || j < b.size()) {
        if (j == b.size() || (i < a.size() && a[i] < b[j])) ++i;
        else if (i == a.size() || b[j] < a[i]) ++j;
        else { ++i; ++j; }
        ++n;
    }
    return n;
}

// Cost of one pairwise step, in units of one complex multiply-add: the MACs of
// every instance plus kWriteCost per element written (an element written and
// read back costs about as much time as this many MACs on the matrix cores).
constexpr double kWriteCost = 16.0;

struct TrialResult {
    std::vector<PathStep> path;
    double cost = 0;          // instance-weighted step cost (MACs + write cost)
    double cost1 = 0;         // one-term complex MACs
    double peak = 0;          // instance-weighted elements live at once
    int max_log = 0;
    bool aborted = false;     // stopped once dearer than the best known path
};

// Leg bookkeeping of a contraction tree: a node's result keeps every leg that
// some leaf outside its subtree still holds; `total[e]` = leaves holding e.
struct LegCount {
    std::vector<std::pair<int, int>> v;   // (leg, holders inside), sorted by leg
};

static LegCount merge_counts(const LegCount& x, const LegCount& y, const std::unordered_map<int, int>& total,
                             std::vector<int>* union_legs, std::vector<int>* result_legs) {
    LegCount out;
    size_t i = 0, j = 0;
    while (i < x.v.size() || j < y.v.size()) {
        int e, c;
        if (j == y.v.size() || (i < x.v.size() && x.v[i].first < y.v[j].first)) {
            e = x.v[i].first;
            c = x.v[i].second;
            ++i;
        } else if (i == x.v.size() || y.v[j].first < x.v[i].first) {
            e = y.v[j].first;
            c = y.v[j].second;
            ++j;
        } else {
            e = x.v[i].first;
            c = x.v[i].second + y.v[j].second;
            ++i;
            ++j;
        }
        if (union_legs) union_legs->push_back(e);
        if (c < total.at(e)) {
            out.v.push_back({e, c});
            if (result_legs) result_legs->push_back(e);
        }
    }
    return out;
}

// Cost, per-term MACs, max tensor size and instance-weighted live-set peak of
// a path (steps in execution order).
static TrialResult evaluate_path(const std::vector<std::vector<int>>& leaf_legs,
                                 const std::vector<uint64_t>& leaf_mask, const PathSearch& ps,
                                 const std::vector<PathStep>& path, const std::unordered_map<int, int>& total) {
    const int L = (int)leaf_legs.size();
    std::vector<LegCount> cnt(L + path.size());
    std::vector<uint64_t> mask(L + path.size());
    std::vector<double> size(L + path.size());
    TrialResult tr;
    double live = 0;
    for (int i = 0; i < L; ++i) {
        for (int e : leaf_legs[i]) cnt[i].v.push_back({e, 1});
        mask[i] = leaf_mask[i];
        size[i] = ps.instances(mask[i]) * std::ldexp(1.0, (int)leaf_legs[i].size());
        live += size[i];
        tr.max_log = std::max(tr.max_log, (int)leaf_legs[i].size());
    }
    tr.peak = live;
    for (size_t j = 0; j < path.size(); ++j) {
        const int a = path[j].a, b = path[j].b, c = L + (int)j;
        std::vector<int> un, res;
        cnt[c] = merge_counts(cnt[a], cnt[b], total, &un, &res);
        mask[c] = mask[a] | mask[b];
        const double inst = ps.instances(mask[c]);
        size[c] = inst * std::ldexp(1.0, (int)res.size());
        tr.cost += inst * std::ldexp(1.0, (int)un.size()) + kWriteCost * size[c];
        tr.cost1 += std::ldexp(1.0, (int)un.size());
        tr.max_log = std::max(tr.max_log, (int)res.size());
        live += size[c];
        tr.peak = std::max(tr.peak, live);
        live -= size[a] + size[b];
    }
    tr.path = path;
    return tr;
}

static TrialResult greedy_trial(const std::vector<std::vector<int>>& leaf_legs,
                                const std::vector<uint64_t>& leaf_mask, const PathSearch& ps,
                                double alpha, double temp, uint64_t seed, const std::atomic<double>* abort_cost) {
    std::mt19937_64 rng(seed);
    std::uniform_real_distribution<double> uni(1e-12, 1.0);
    const int L = (int)leaf_legs.size();
    std::vector<std::vector<int>> legs(leaf_legs);
    std::vector<uint64_t> mask(leaf_mask);
    std::vector<char> alive(L, 1);
    std::unordered_map<int, std::vector<int>> owners;
    for (int i = 0; i < L; ++i)
        for (int e : legs[i]) owners[e].push_back(i);
    auto size_of = [&](int i) { return ps.instances(mask[i]) * std::ldexp(1.0, (int)legs[i].size()); };
    // legs of the result of merging a and b: every leg of either that some
    // other live tensor still holds (shared legs held only by a and b are summed)
    auto result_legs = [&](int a, int b) {
        std::vector<int> out;
        std::vector<int> un;
        std::set_union(legs[a].begin(), legs[a].end(), legs[b].begin(), legs[b].end(), std::back_inserter(un));
        for (int e : un) {
            const auto& ow = owners[e];
            for (int o : ow)
                if (o != a && o != b) {
                    out.push_back(e);
                    break;
                }
        }
        return out;
    };
    typedef std::tuple<double, int, int> Cand;
    std::priority_queue<Cand, std::vector<Cand>, std::greater<Cand>> pq;
    auto push = [&](int a, int b) {
        if (a == b) return;
        if (a > b) std::swap(a, b);
        std::vector<int> lc = result_legs(a, b);
        double sc = ps.instances(mask[a] | mask[b]) * std::ldexp(1.0, (int)lc.size()) -
                    alpha * (size_of(a) + size_of(b));
        double s = (sc >= 0 ? 1.0 : -1.0) * std::log2(1.0 + std::fabs(sc));
        if (temp > 0) s -= temp * (-std::log(-std::log(uni(rng))));
        pq.push(Cand(s, a, b));
    };
    for (auto& kv : owners)
        for (size_t x = 0; x < kv.second.size(); ++x)
            for (size_t y = x + 1; y < kv.second.size(); ++y) push(kv.second[x], kv.second[y]);
    TrialResult tr;
    int remaining = L;
    while (remaining > 1) {
        int a, b;
        if (!pq.empty()) {
            Cand cd_ = pq.top();
            pq.pop();
            a = std::get<1>(cd_);
            b = std::get<2>(cd_);
            if (!alive[a] || !alive[b]) continue;
        } else {
            // disconnected leftovers (cannot happen inside a cluster)
            a = -1;
            b = -1;
            for (int i = 0; i < (int)alive.size(); ++i)
                if (alive[i]) {
                    if (a < 0) a = i;
                    else if (b < 0) { b = i; break; }
                }
        }
        std::vector<int> lc = result_legs(a, b);
        uint64_t mc = mask[a] | mask[b];
        int u = union_size(legs[a], legs[b]);
        double inst = ps.instances(mc);
        tr.cost += inst * (std::ldexp(1.0, u) + kWriteCost * std::ldexp(1.0, (int)lc.size()));
        if (abort_cost && tr.cost > abort_cost->load(std::memory_order_relaxed)) {
            tr.aborted = true;
            return tr;
        }
        int c = (int)legs.size();
        legs.push_back(lc);
        mask.push_back(mc);
        alive.push_back(1);
        alive[a] = alive[b] = 0;
        for (int e : legs[a]) {
            auto& v = owners[e];
            v.erase(std::remove(v.begin(), v.end(), a), v.end());
        }
        for (int e : legs[b]) {
            auto& v = owners[e];
            v.erase(std::remove(v.begin(), v.end(), b), v.end());
        }
        for (int e : lc) owners[e].push_back(c);
        tr.path.push_back({a, b});
        --remaining;
        for (int e : lc)
            for (int o : owners[e])
                if (o != c) push(o, c);
    }
    return tr;
}

// Subtree reconfiguration: for every internal node of the tree, cut its
// subtree at up to kReconfLeaves pieces (expanding the dearest steps first),
// find the cheapest binary tree over those pieces by dynamic programming over
// subsets (same cost model, result sizes capped at 2^max_log) and keep it when
// it is cheaper.  Repeated until a pass changes nothing.
constexpr int kReconfLeaves = 8;
constexpr int kReconfCandidates = 8;      // distinct greedy paths reconfigured per cluster

static std::vector<PathStep> reconfigure(const std::vector<std::vector<int>>& leaf_legs,
                                         const std::vector<uint64_t>& leaf_mask, const PathSearch& ps,
                                         const std::vector<PathStep>& path,
                                         const std::unordered_map<int, int>& total, int max_log) {
    const int L = (int)leaf_legs.size();
    const int NN = L + (int)path.size();
    if (path.size() < 2) return path;
    std::vector<int> ca(NN, -1), cb(NN, -1), par(NN, -1);
    for (size_t j = 0; j < path.size(); ++j) {
        ca[L + j] = path[j].a;
        cb[L + j] = path[j].b;
        par[path[j].a] = par[path[j].b] = L + (int)j;
    }
    const int root = NN - 1;
    std::vector<LegCount> cnt(NN);
    std::vector<uint64_t> mask(NN);
    std::vector<double> step(NN, 0.0);
    std::vector<int> nres(NN, 0);
    for (int i = 0; i < L; ++i) {
        for (int e : leaf_legs[i]) cnt[i].v.push_back({e, 1});
        mask[i] = leaf_mask[i];
        nres[i] = (int)leaf_legs[i].size();
    }
    auto update = [&](int n) {
        std::vector<int> un, res;
        cnt[n] = merge_counts(cnt[ca[n]], cnt[cb[n]], total, &un, &res);
        mask[n] = mask[ca[n]] | mask[cb[n]];
        nres[n] = (int)res.size();
        const double inst = ps.instances(mask[n]);
        step[n] = inst * (std::ldexp(1.0, (int)un.size()) + kWriteCost * std::ldexp(1.0, nres[n]));
    };
    // bottom-up (path order is a valid topological order)
    for (int n = L; n < NN; ++n) update(n);
    std::function<void(int, std::vector<int>&)> postorder = [&](int n, std::vector<int>& out) {
        if (n < L) return;
        postorder(ca[n], out);
        postorder(cb[n], out);
        out.push_back(n);
    };
    for (int pass = 0; pass < 8; ++pass) {
        bool changed = false;
        std::vector<int> order;
        postorder(root, order);
        for (int node : order) {
            // region: node plus the internal nodes expanded below it
            std::vector<int> region{node}, items{ca[node], cb[node]};
            while ((int)items.size() < kReconfLeaves) {
                int pick = -1;
                for (size_t q = 0; q < items.size(); ++q)
                    if (items[q] >= L && (pick < 0 || step[items[q]] > step[items[pick]])) pick = (int)q;
                if (pick < 0) break;
                const int x = items[pick];
                region.push_back(x);
                items[pick] = ca[x];
                items.push_back(cb[x]);
            }
            const int k = (int)items.size();
            if (k < 3) continue;
            double old = 0;
            for (int r : region) old += step[r];
            // local leg ids of the legs the pieces hold
            std::vector<int> lid;
            for (int it : items)
                for (auto& pr : cnt[it].v) lid.push_back(pr.first);
            std::sort(lid.begin(), lid.end());
            lid.erase(std::unique(lid.begin(), lid.end()), lid.end());
            if (lid.size() > 256) continue;
            const int S = 1 << k;
            struct Bits {
                uint64_t w[4] = {0, 0, 0, 0};
                int pop() const {
                    return __builtin_popcountll(w[0]) + __builtin_popcountll(w[1]) + __builtin_popcountll(w[2]) +
                           __builtin_popcountll(w[3]);
                }
            };
            std::vector<Bits> res(S), held(S);
            std::vector<double> inst(S);
            std::vector<uint64_t> smask(S, 0);
            std::vector<std::vector<int>> cin(S, std::vector<int>(lid.size(), 0));
            for (int T = 1; T < S; ++T) {
                const int low = __builtin_ctz(T);
                const int rest = T & (T - 1);
                cin[T] = cin[rest];
                smask[T] = smask[rest] | mask[items[low]];
                for (auto& pr : cnt[items[low]].v) {
                    const int li = (int)(std::lower_bound(lid.begin(), lid.end(), pr.first) - lid.begin());
                    cin[T][li] += pr.second;
                }
                for (size_t li = 0; li < lid.size(); ++li)
                    if (cin[T][li] > 0 && cin[T][li] < total.at(lid[li])) res[T].w[li >> 6] |= 1ULL << (li & 63);
                inst[T] = ps.instances(smask[T]);
            }
            std::vector<double> best(S, std::numeric_limits<double>::infinity());
            std::vector<int> split(S, 0);
            for (int q = 0; q < k; ++q) best[1 << q] = 0;
            for (int T = 1; T < S; ++T) {
                if (__builtin_popcount(T) < 2) continue;
                const int nr = res[T].pop();
                if (T != S - 1 && nr > max_log) continue;
                const double wcost = kWriteCost * std::ldexp(1.0, nr);
                const int low = T & -T;
                for (int T1 = (T - 1) & T; T1 > 0; T1 = (T1 - 1) & T) {
                    if (!(T1 & low)) continue;
                    const int T2 = T ^ T1;
                    const double sub = best[T1] + best[T2];
                    if (!(sub < best[T])) continue;
                    Bits u;
                    for (int w = 0; w < 4; ++w) u.w[w] = res[T1].w[w] | res[T2].w[w];
                    const double c = sub + inst[T] * (std::ldexp(1.0, u.pop()) + wcost);
                    if (c < best[T]) {
                        best[T] = c;
                        split[T] = T1;
                    }
                }
            }
            if (!(best[S - 1] < old * (1.0 - 1e-9))) continue;
            // rebuild the region: reuse its node ids, node keeps the root id
            std::vector<int> free_ids(region.begin() + 1, region.end());
            std::function<int(int, bool)> build = [&](int T, bool is_root) -> int {
                if (__builtin_popcount(T) == 1) return items[__builtin_ctz(T)];
                const int n = is_root ? node : free_ids.back();
                if (!is_root) free_ids.pop_back();
                const int l = build(split[T], false), r = build(T ^ split[T], false);
                ca[n] = l;
                cb[n] = r;
                par[l] = par[r] = n;
                return n;
            };
            build(S - 1, true);
            // refresh the region bottom-up
            std::vector<int> sub_order;
            std::function<void(int)> walk = [&](int n) {
                if (n < L || std::find(items.begin(), items.end(), n) != items.end()) return;
                walk(ca[n]);
                walk(cb[n]);
                sub_order.push_back(n);
            };
            walk(node);
            for (int n : sub_order) update(n);
            changed = true;
        }
        if (!changed) break;
    }
    // emit: post-order, the larger subtree first
    std::vector<int> nleaves(NN, 1);
    std::vector<int> order;
    std::function<void(int)> count = [&](int n) {
        if (n < L) return;
        count(ca[n]);
        count(cb[n]);
        nleaves[n] = nleaves[ca[n]] + nleaves[cb[n]];
    };
    count(root);
    std::function<void(int)> emit = [&](int n) {
        if (n < L) return;
        int x = ca[n], y = cb[n];
        if (nleaves[y] > nleaves[x]) std::swap(x, y);
        emit(x);
        emit(y);
        order.push_back(n);
    };
    emit(root);
    std::vector<int> newid(NN, -1);
    for (int i = 0; i < L; ++i) newid[i] = i;
    std::vector<PathStep> out;
    for (size_t j = 0; j < order.size(); ++j) {
        const int n = order[j];
        out.push_back({newid[ca[n]], newid[cb[n]]});
        newid[n] = L + (int)j;
    }
    return out;
}

// Per-estimate depth.  Subtrees with no noise slot below them are computed
// once per prepared schedule, so an estimate runs only the steps with a slot
// below them, one tree level per dependent launch (about 10 us each on the
// target GPU, whatever the level's work).  The cheapest path absorbs constant
// tensors into a slot's arm one at a time, which costs a level each.  Two
// rewrites of the tree shorten those chains:
//   ((Y . C1) . C2) -> Y . (C1 . C2)     (C1, C2 constant: their product is
//                                         computed once)
//   ((X . Y) . C)   -> Y . (X . C)        (C constant, X's arm shallower than Y's)
// Each is kept when it lowers the rewritten node's per-estimate depth and the
// constant product stays within kDepthMaxConstLegs legs; the rewritten tree is
// kept when it is shallower, admissible, and dearer by at most kDepthCredit
// per level saved (about what the matrix cores do in one dependent launch).
constexpr int kDepthMaxConstLegs = 14;
constexpr double kDepthCredit = 2e7;   // cost units (complex MACs) of one dependent launch

static int per_estimate_depth(const std::vector<int>& ca, const std::vector<int>& cb,
                              const std::vector<uint64_t>& mask, int L, int n) {
    if (n < L || mask[n] == 0) return 0;
    const int a = per_estimate_depth(ca, cb, mask, L, ca[n]), b = per_estimate_depth(ca, cb, mask, L, cb[n]);
    return 1 + std::max(a, b);
}

static std::vector<PathStep> reduce_depth(const std::vector<std::vector<int>>& leaf_legs,
                                          const std::vector<uint64_t>& leaf_mask, const PathSearch& ps,
                                          const std::vector<PathStep>& path,
                                          const std::unordered_map<int, int>& total, int max_log) {
    const int L = (int)leaf_legs.size();
    const int NN = L + (int)path.size();
    if (path.size() < 2) return path;
    std::vector<int> ca(NN, -1), cb(NN, -1);
    for (size_t j = 0; j < path.size(); ++j) {
        ca[L + j] = path[j].a;
        cb[L + j] = path[j].b;
    }
    const int root = NN - 1;
    std::vector<LegCount> cnt(NN);
    std::vector<uint64_t> mask(NN, 0);
    std::vector<int> nres(NN, 0);
    for (int i = 0; i < L; ++i) {
        for (int e : leaf_legs[i]) cnt[i].v.push_back({e, 1});
        mask[i] = leaf_mask[i];
        nres[i] = (int)leaf_legs[i].size();
    }
    std::vector<double> step(NN, 0.0);
    auto update = [&](int n) {
        std::vector<int> un, res;
        cnt[n] = merge_counts(cnt[ca[n]], cnt[cb[n]], total, &un, &res);
        mask[n] = mask[ca[n]] | mask[cb[n]];
        nres[n] = (int)res.size();
        step[n] = ps.instances(mask[n]) * (std::ldexp(1.0, (int)un.size()) + kWriteCost * std::ldexp(1.0, nres[n]));
    };
    for (int n = L; n < NN; ++n) update(n);
    auto total_cost = [&]() {
        double c = 0;
        for (int n = L; n < NN; ++n) c += step[n];
        return c;
    };
    auto depth = [&](int n) { return per_estimate_depth(ca, cb, mask, L, n); };
    const double cost0 = total_cost();
    const int depth0 = depth(root);
    std::function<void(int, std::vector<int>&)> postorder = [&](int n, std::vector<int>& out) {
        if (n < L) return;
        postorder(ca[n], out);
        postorder(cb[n], out);
        out.push_back(n);
    };
    // the parent of every node (rebuilt after each rewrite)
    std::vector<int> par(NN, -1);
    auto reparent = [&]() {
        std::fill(par.begin(), par.end(), -1);
        for (int n = L; n < NN; ++n) par[ca[n]] = par[cb[n]] = n;
    };
    reparent();
    auto refresh_up = [&](int n) {
        for (int x = n; x >= 0; x = par[x]) update(x);
    };
    bool changed = true;
    for (int pass = 0; pass < 64 && changed; ++pass) {
        changed = false;
        std::vector<int> order;
        postorder(root, order);
        for (int N : order) {
            if (mask[N] == 0) continue;
            int C = ca[N], X = cb[N];
            if (mask[C] != 0) std::swap(C, X);
            if (mask[C] != 0 || X < L) continue;           // needs a constant child and an internal other
            const int d_old = depth(N);
            // candidate rewrites of N = (X . C)
            int A = ca[X], B = cb[X];
            int rule = 0, keep = -1, fold = -1;
            if (mask[A] == 0 || mask[B] == 0) {
                // X = (Y . C1): N = Y . (C1 . C2)
                keep = mask[A] == 0 ? B : A;
                fold = mask[A] == 0 ? A : B;
                rule = 1;
            } else {
                // X = (P . Q), both with slots: push C into the shallower one
                keep = depth(A) >= depth(B) ? A : B;
                fold = keep == A ? B : A;
                rule = 2;
            }
            // save, rewrite: X's id holds the new inner node (fold . C)
            const int sa = ca[N], sb = cb[N], xa = ca[X], xb = cb[X];
            ca[X] = fold;
            cb[X] = C;
            ca[N] = keep;
            cb[N] = X;
            reparent();
            update(X);
            refresh_up(N);
            const bool ok = depth(N) < d_old && nres[X] <= std::min(max_log, rule == 1 ? kDepthMaxConstLegs : max_log) &&
                            nres[N] <= max_log;
            if (ok) {
                changed = true;
                break;     // the traversal order changed: start a new pass
            }
            ca[N] = sa;
            cb[N] = sb;
            ca[X] = xa;
            cb[X] = xb;
            reparent();
            update(X);
            refresh_up(N);
        }
    }
    const double cost1 = total_cost();
    const int depth1 = depth(root);
    if (depth1 >= depth0 || cost1 > cost0 + kDepthCredit * (depth0 - depth1)) return path;
    // emit: post-order, the larger subtree first
    std::vector<int> nleaves(NN, 1);
    std::function<void(int)> count = [&](int n) {
        if (n < L) return;
        count(ca[n]);
        count(cb[n]);
        nleaves[n] = nleaves[ca[n]] + nleaves[cb[n]];
    };
    count(root);
    std::vector<int> order;
    std::function<void(int)> emit = [&](int n) {
        if (n < L) return;
        int x = ca[n], y = cb[n];
        if (nleaves[y] > nleaves[x]) std::swap(x, y);
        emit(x);
        emit(y);
        order.push_back(n);
    };
    emit(root);
    std::vector<int> newid(NN, -1);
    for (int i = 0; i < L; ++i) newid[i] = i;
    std::vector<PathStep> out;
    for (size_t j = 0; j < order.size(); ++j) {
        const int n = order[j];
        out.push_back({newid[ca[n]], newid[cb[n]]});
        newid[n] = L + (int)j;
    }
    return out;
}

static void plan_clusters(Plan& p, int trials, uint64_t seed, int max_log, double max_peak, bool reconf) {
    const int nl = (int)p.leaves.size();
    // union-find over shared legs
    std::vector<int> parent(nl);
    std::iota(parent.begin(), parent.end(), 0);
    std::function<int(int)> find = [&](int x) { return parent[x] == x ? x : parent[x] = find(parent[x]); };
    std::unordered_map<int, int> first_owner;
    for (int i = 0; i < nl; ++i)
        for (int e : p.leaves[i].legs) {
            auto it = first_owner.find(e);
            if (it == first_owner.end()) first_owner[e] = i;
            else parent[find(i)] = find(it->second);
        }
    std::map<int, std::vector<int>> groups;
    for (int i = 0; i < nl; ++i) groups[find(i)].push_back(i);
    p.clusters.clear();
    for (auto& kv : groups) {
        Cluster cl;
        cl.leaves = kv.second;
        for (int li : cl.leaves)
            if (p.leaves[li].slot >= 0) cl.slots.push_back(p.leaves[li].slot);
        std::sort(cl.slots.begin(), cl.slots.end());
        if ((int)cl.slots.size() > kMaxSlotsPerCluster)
            fail(TN_ETOOBIG, "a network cluster holds more than 64 noise slots");
        PathSearch ps;
        ps.level = p.level;
        for (int s : cl.slots) {
            int z = 0;
            for (int i = 1; i < 4; ++i) z += p.noise[s].zero[i] ? 0 : 1;
            ps.zcount.push_back(z);
        }
        std::vector<std::vector<int>> leaf_legs;
        std::vector<uint64_t> leaf_mask;
        for (int li : cl.leaves) {
            std::vector<int> lg = p.leaves[li].legs;
            std::sort(lg.begin(), lg.end());
            leaf_legs.push_back(lg);
            uint64_t m = 0;
            if (p.leaves[li].slot >= 0) {
                int local = (int)(std::lower_bound(cl.slots.begin(), cl.slots.end(), p.leaves[li].slot) -
                                  cl.slots.begin());
                m = 1ULL << local;
            }
            leaf_mask.push_back(m);
        }
        if (cl.leaves.size() == 1) {
            cl.max_log = (int)leaf_legs[0].size();
            p.clusters.push_back(cl);
            continue;
        }
        std::unordered_map<int, int> total;
        for (auto& lg : leaf_legs)
            for (int e : lg) ++total[e];
        const double alphas[4] = {1.0, 0.5, 0.0, 0.75};
        const double temps[3] = {0.5, 1.0, 2.0};
        // a path is admissible when one instance of every tensor fits in 2^max_log
        // elements and the instance-weighted live set fits in max_peak elements;
        // among admissible paths the cheapest wins (lowest trial index on ties),
        // else the smallest peak.  Trials run on all host threads; a trial stops
        // once it costs more than twice the best admissible path so far.  That
        // never stops a trial within twice the final best, so the candidates
        // below (the cheapest trials within that factor) do not depend on timing.
        auto admissible = [&](const TrialResult& r) { return r.max_log <= max_log && r.peak <= max_peak; };
        std::vector<TrialResult> results(trials);
        std::atomic<double> abort_cost{std::numeric_limits<double>::infinity()};
        std::atomic<int> next{0};
        const int nth = std::max(1, std::min<int>({(int)std::thread::hardware_concurrency(), 16, trials}));
        auto run_pool = [&](const std::function<void()>& fn) {
            std::vector<std::thread> pool;
            for (int q = 1; q < nth; ++q) pool.emplace_back(fn);
            fn();
            for (auto& th : pool) th.join();
        };
        run_pool([&]() {
            for (int t = next++; t < trials; t = next++) {
                const double alpha = alphas[t % 4];
                const double temp = t < 4 ? 0.0 : temps[t % 3];
                TrialResult tr = greedy_trial(leaf_legs, leaf_mask, ps, alpha, temp,
                                              seed * 1000003ULL + (uint64_t)t * 7919ULL + 17, &abort_cost);
                if (!tr.aborted) {
                    tr = evaluate_path(leaf_legs, leaf_mask, ps, tr.path, total);
                    if (admissible(tr)) {
                        double cur = abort_cost.load();
                        while (2.0 * tr.cost < cur && !abort_cost.compare_exchange_weak(cur, 2.0 * tr.cost)) {
                        }
                    }
                }
                results[t] = std::move(tr);
            }
        });
        TrialResult best;
        bool have = false;
        for (int t = 0; t < trials; ++t) {
            TrialResult& tr = results[t];
            if (tr.aborted) continue;
            bool ok = admissible(tr);
            bool best_ok = have && admissible(best);
            bool better = ok ? tr.cost < best.cost : (tr.max_log < best.max_log ||
                                                     (tr.max_log == best.max_log && tr.peak < best.peak));
            if (!have || (ok && !best_ok) || (ok == best_ok && better)) {
                best = tr;
                have = true;
            }
        }
        if (have && admissible(best) && reconf) {
            // reconfigure the cheapest few distinct trials within twice the best
            std::vector<int> cand;
            for (int t = 0; t < trials; ++t)
                if (!results[t].aborted && admissible(results[t]) && results[t].cost <= 2.0 * best.cost)
                    cand.push_back(t);
            std::stable_sort(cand.begin(), cand.end(),
                             [&](int x, int y) { return results[x].cost < results[y].cost; });
            std::vector<int> pick;
            for (int t : cand) {
                bool dup = false;
                for (int q : pick) dup |= results[q].cost == results[t].cost;
                if (!dup) pick.push_back(t);
                if ((int)pick.size() == kReconfCandidates) break;
            }
            std::vector<TrialResult> rc(pick.size());
            std::atomic<int> nx{0};
            run_pool([&]() {
                for (int q = nx++; q < (int)pick.size(); q = nx++) {
                    const TrialResult& src = results[pick[q]];
                    rc[q] = evaluate_path(leaf_legs, leaf_mask, ps,
                                          reconfigure(leaf_legs, leaf_mask, ps, src.path, total, max_log), total);
                }
            });
            for (auto& r : rc)
                if (admissible(r) && r.cost < best.cost) best = std::move(r);
        }
        if (!admissible(best)) {
            std::ostringstream os;
            os << "no contraction path keeps tensors within 2^" << max_log << " elements and the live set "
               << "within " << max_peak << " elements (best: 2^" << best.max_log << ", " << best.peak << ")";
            fail(TN_ETOOBIG, os.str());
        }
        {
            TrialResult shallow = evaluate_path(leaf_legs, leaf_mask, ps,
                                                reduce_depth(leaf_legs, leaf_mask, ps, best.path, total, max_log),
                                                total);
            if (admissible(shallow)) best = std::move(shallow);
        }
        cl.path = best.path;
        cl.cmacs_per_term = best.cost1;
        cl.max_log = best.max_log;
        p.clusters.push_back(cl);
    }
    p.max_log = 0;
    p.cmacs_per_term = 0;
    for (auto& cl : p.clusters) {
        p.max_log = std::max(p.max_log, cl.max_log);
        p.cmacs_per_term += cl.cmacs_per_term;
    }
}

static std::atomic<uint64_t> g_plan_id{1};

// Argument checks shared by both plan kinds: shapes, indices, unitary gates,
// Kraus counts (trace preservation is checked by the callers).
static std::unique_ptr<Plan> new_plan(const tn_circuit* c, const tn_state* psi, const tn_state* v) {
    if (!c || !psi || !v) fail(TN_EINVAL, "null circuit or state");
    if (c->n_qubits < 1 || c->n_qubits > 4096) fail(TN_EINVAL, "n_qubits out of range");
    if (c->n_ops < 0 || (c->n_ops > 0 && !c->ops)) fail(TN_EINVAL, "bad op list");
    if (psi->kind != TN_STATE_PRODUCT || !psi->data) fail(TN_EINVAL, "psi must be a product state");
    if (v->kind < 0 || v->kind > 4 || !v->data) fail(TN_EINVAL, "bad target state");
    if (v->kind == TN_STATE_DENSE && c->n_qubits > 30) fail(TN_EINVAL, "dense target needs n <= 30");
    auto p = std::make_unique<Plan>();
    p->id = g_plan_id++;
    p->n_qubits = c->n_qubits;
    static const char* kinds[5] = {"product", "circuit_output", "dense", "sum2", "circuit_output_sum2"};
    p->target_kind = kinds[v->kind];
    for (int64_t k = 0; k < c->n_ops; ++k) {
        const tn_op& op = c->ops[k];
        if (op.kind != TN_GATE && op.kind != TN_NOISE) fail(TN_EINVAL, "op kind must be gate or noise");
        if (op.kind == TN_NOISE && op.nq != 1)
            fail(TN_EUNSUPPORTED, "noise channels must act on exactly one qubit");
        if (op.nq < 1 || op.nq > 2) fail(TN_EUNSUPPORTED, "gates act on one or two qubits");
        if (!op.mat) fail(TN_EINVAL, "op without matrix");
        for (int i = 0; i < op.nq; ++i)
            if (op.q[i] < 0 || op.q[i] >= c->n_qubits) fail(TN_EINVAL, "qubit index out of range");
        if (op.nq == 2 && op.q[0] == op.q[1]) fail(TN_EINVAL, "2-qubit gate on one qubit");
        if (op.kind == TN_GATE) check_unitary(op, k);
        else if (op.n_kraus < 1 || op.n_kraus > 64) fail(TN_EINVAL, "noise needs 1..64 Kraus matrices");
    }
    p->n_ops = c->n_ops;
    for (int64_t k = 0; k < c->n_ops; ++k)
        if (c->ops[k].kind == TN_GATE && c->ops[k].nq == 2) ++p->n_2q_gates;
    return p;
}

struct PathOpts {
    int trials, max_log;
    uint64_t seed;
    double max_elems;
    bool reconf;
};

static PathOpts path_opts(const tn_plan_opts* opts) {
    PathOpts o;
    o.trials = (opts && opts->path_trials > 0) ? opts->path_trials : 1024;
    o.seed = (opts && opts->seed) ? opts->seed : 2211170280ULL;
    o.max_log = (opts && opts->max_log_size > 0) ? opts->max_log_size : 30;
    o.max_elems = ((opts && opts->max_work_bytes > 0) ? opts->max_work_bytes : 64.0 * (1ULL << 30)) / 8.0;
    o.reconf = !(opts && opts->no_reconfigure);
    return o;
}

static Plan* finish_plan(std::unique_ptr<Plan> p, const tn_circuit* c, const tn_state* psi, const tn_state* v,
                         int level, const tn_plan_opts* opts);

Plan* build_plan(const tn_circuit* c, const tn_state* psi, const tn_state* v, int level,
                 const tn_plan_opts* opts) {
    if (level < 0) fail(TN_EINVAL, "level must be >= 0");
    auto p = new_plan(c, psi, v);
    for (int64_t k = 0; k < c->n_ops; ++k)
        if (c->ops[k].kind == TN_NOISE) p->noise.push_back(split_noise(c->ops[k], k));
    return finish_plan(std::move(p), c, psi, v, level, opts);
}

// Slot matrices of the quantum-trajectories estimate (the paper's comparison
// method, Section V): Kraus operator k of a noise is drawn with probability
// q_k = tr(E_k^+ E_k) / 2 and its slot carries E_k / sqrt(q_k) with weight 1,
// so the mean of |a|^2 over draws is the exact value.  At most 4 Kraus
// operators (the slot choices of a term); operators with q_k = 0 are never
// drawn and flagged zero.
static NoiseSplit kraus_slots(const tn_op& op, int64_t index) {
    check_cptp(op, index);
    if (op.n_kraus > 4) fail(TN_EUNSUPPORTED, "trajectories take at most 4 Kraus operators per noise");
    NoiseSplit ns;
    ns.qubit = op.q[0];
    ns.op_index = index;
    for (int k = 0; k < 4; ++k) {
        ns.zero[k] = true;
        ns.d[k] = 0.0;
        for (int e = 0; e < 4; ++e) ns.K[k][e] = 0.0;
        if (k >= op.n_kraus) continue;
        const tn_c128* m = op.mat + 4 * k;
        double q = 0.0;
        for (int e = 0; e < 4; ++e) q += m[e].re * m[e].re + m[e].im * m[e].im;
        q *= 0.5;
        ns.q[k] = q;
        if (!(q > 0.0)) continue;
        ns.zero[k] = false;
        ns.d[k] = 1.0;
        const double r = 1.0 / std::sqrt(q);
        for (int e = 0; e < 4; ++e) ns.K[k][e] = cd(m[e].re * r, m[e].im * r);
    }
    return ns;
}

Plan* build_plan_trajectories(const tn_circuit* c, const tn_state* psi, const tn_state* v,
                              const tn_plan_opts* opts) {
    auto p = new_plan(c, psi, v);
    for (int64_t k = 0; k < c->n_ops; ++k)
        if (c->ops[k].kind == TN_NOISE) p->noise.push_back(kraus_slots(c->ops[k], k));
    p->trajectories = true;
    // the path's instance model: samples differ from the all-first pattern in
    // a few slots, like a level-3 term set
    const int level = std::min<int>(3, (int)p->noise.size());
    return finish_plan(std::move(p), c, psi, v, level, opts);
}

static Plan* finish_plan(std::unique_ptr<Plan> p, const tn_circuit* c, const tn_state* psi, const tn_state* v,
                         int level, const tn_plan_opts* opts) {
    // past light cone of every noise slot (features of the pruning policy)
    {
        const int words = (c->n_qubits + 63) / 64;
        for (NoiseSplit& ns : p->noise) {
            std::vector<uint64_t> cone(words, 0);
            cone[ns.qubit >> 6] |= 1ULL << (ns.qubit & 63);
            int g2 = 0;
            for (int64_t k = ns.op_index - 1; k >= 0; --k) {
                const tn_op& op = c->ops[k];
                if (op.kind != TN_GATE) continue;
                bool hit = false;
                for (int i = 0; i < op.nq; ++i) hit |= (cone[op.q[i] >> 6] >> (op.q[i] & 63)) & 1;
                if (!hit) continue;
                for (int i = 0; i < op.nq; ++i) cone[op.q[i] >> 6] |= 1ULL << (op.q[i] & 63);
                if (op.nq == 2) ++g2;
            }
            int cnt = 0;
            for (uint64_t w : cone) cnt += __builtin_popcountll(w);
            ns.cone = std::move(cone);
            ns.cone_qubits = cnt;
            ns.cone_2q_gates = g2;
        }
    }
    p->n_noise = (int)p->noise.size();
    p->level_req = level;
    p->level = std::min(level, p->n_noise);
    p->clamped = level > p->n_noise;
    if (p->level > TN_MAX_LEVEL) fail(TN_EINVAL, "level above TN_MAX_LEVEL");
    NetBuild nb = build_network(c, psi, v, !(opts && opts->no_light_cone),
                                !(opts && opts->no_diagonal_hyperedges));
    fuse_fixed(nb);
    p->leaves = std::move(nb.leaves);
    p->scalar = nb.scalar;
    PathOpts po = path_opts(opts);
    // a bond-2 target's shared index reaches every output wire; the greedy
    // trials find good orders for it less often (25-qubit grid: 3.9 GFLOP per
    // term at 1024 trials, 1.0 at 8192, 0.25 for a product target)
    if ((v->kind == TN_STATE_SUM2 || v->kind == TN_STATE_CIRCUIT_OUTPUT_SUM2) && !(opts && opts->path_trials > 0))
        po.trials = 8192;
    plan_clusters(*p, po.trials, po.seed, po.max_log, po.max_elems, po.reconf);
    return p.release();
}

// Exact value (the paper's exact baseline, the doubled network of Section IV /
// Fig. 2).  For every term the bra network is the complex conjugate of the ket
// network, so the doubled network is the reduced ket network of one term, its
// conjugate on fresh edge ids, and at every noise one fixed tensor joining the
// noise's ket legs (out, in) and bra legs (out, in):
//   T[a][c][b][d] = sum_k E_k[a][c] conj(E_k[b][d]),
// the channel's whole superoperator, which sums every correction of that noise
// at once.  No slots remain: one term of weight 1 whose network value a is the
// exact <v| E(|psi><psi|) |v> (real up to rounding; the exec reports Re(a)).
// The light-cone reduction of the ket network holds for every term and so for
// the doubled network.
Plan* build_plan_doubled(const tn_circuit* c, const tn_state* psi, const tn_state* v,
                         const tn_plan_opts* opts) {
    auto p = new_plan(c, psi, v);
    std::vector<const tn_op*> noise_ops;
    for (int64_t k = 0; k < c->n_ops; ++k)
        if (c->ops[k].kind == TN_NOISE) {
            check_cptp(c->ops[k], k);
            noise_ops.push_back(&c->ops[k]);
        }
    p->doubled = true;
    p->n_channels = (int)noise_ops.size();
    p->n_noise = 0;
    p->level_req = 0;
    p->level = 0;
    NetBuild ket = build_network(c, psi, v, !(opts && opts->no_light_cone),
                                 !(opts && opts->no_diagonal_hyperedges));
    fuse_fixed(ket);
    int top = 0;
    for (const Leaf& l : ket.leaves)
        for (int e : l.legs) top = std::max(top, e + 1);
    NetBuild nb;
    nb.scalar = ket.scalar * std::conj(ket.scalar);
    for (Leaf& l : ket.leaves) {
        if (l.slot >= 0) {
            const tn_op& op = *noise_ops[l.slot];
            Leaf t;
            t.legs = {l.legs[0], l.legs[1], l.legs[0] + top, l.legs[1] + top};
            t.data.assign(16, cd(0.0));
            for (int k = 0; k < op.n_kraus; ++k) {
                const tn_c128* e = op.mat + 4 * k;
                for (int a = 0; a < 2; ++a)
                    for (int cc = 0; cc < 2; ++cc)
                        for (int b = 0; b < 2; ++b)
                            for (int d = 0; d < 2; ++d)
                                t.data[8 * a + 4 * cc + 2 * b + d] +=
                                    cd(e[2 * a + cc].re, e[2 * a + cc].im) *
                                    std::conj(cd(e[2 * b + d].re, e[2 * b + d].im));
            }
            nb.leaves.push_back(std::move(t));
            continue;
        }
        Leaf bra;
        bra.legs = l.legs;
        for (int& e : bra.legs) e += top;
        bra.data = l.data;
        for (cd& x : bra.data) x = std::conj(x);
        nb.leaves.push_back(std::move(l));
        nb.leaves.push_back(std::move(bra));
    }
    fuse_fixed(nb);
    p->leaves = std::move(nb.leaves);
    p->scalar = nb.scalar;
    const PathOpts po = path_opts(opts);
    plan_clusters(*p, po.trials, po.seed, po.max_log, po.max_elems, po.reconf);
    return p.release();
}

// ---------------------------------------------------------------------------
// term enumeration (Algorithm 1 order)
// ---------------------------------------------------------------------------
Terms* enumerate_terms(const Plan* p, int level, const tn_prune_opts* prune) {
    if (level < 0) fail(TN_EINVAL, "level must be >= 0");
    if (p->trajectories) fail(TN_EINVAL, "a trajectories plan takes sampled terms (tn_terms_trajectories)");
    const int N = p->n_noise;
    const int L = std::min(level, N);
    if (L > TN_MAX_LEVEL) fail(TN_EINVAL, "level above TN_MAX_LEVEL");
    auto t = std::make_unique<Terms>();
    t->plan = p;
    t->plan_id = p->id;
    t->level = L;
    std::vector<int> pos, corr;
    int64_t cand = 0;
    for (int u = 0; u <= L; ++u) {
        pos.resize(u);
        for (int i = 0; i < u; ++i) pos[i] = i;
        while (true) {
            corr.assign(u, 1);
            while (true) {
                std::vector<int8_t> pat(N, 0);
                for (int i = 0; i < u; ++i) pat[pos[i]] = (int8_t)corr[i];
                double w = 1.0;
                bool zero = false;
                for (int s = 0; s < N; ++s) {
                    w *= p->noise[s].d[pat[s]];
                    zero |= p->noise[s].zero[pat[s]];
                }
                bool pruned = false;
                if (prune && u >= prune->min_level && prune->min_level >= 1) {
                    if (prune->keep) {
                        if (cand >= prune->n_keep) fail(TN_EINVAL, "prune keep array too short");
                        pruned = prune->keep[cand] == 0;
                    }
                    ++cand;
                }
                t->pat.insert(t->pat.end(), pat.begin(), pat.end());
                t->w.push_back(zero ? 0.0 : w);
                t->lvl.push_back((uint8_t)u);
                t->zero.push_back(zero ? 1 : 0);
                t->pruned.push_back(pruned ? 1 : 0);
                // next correction tuple (lexicographic over {1,2,3}^u)
                int j = u - 1;
                while (j >= 0 && corr[j] == 3) corr[j--] = 1;
                if (j < 0) break;
                ++corr[j];
            }
            // next position set (lexicographic combinations)
            int j = u - 1;
            while (j >= 0 && pos[j] == N - u + j) --j;
            if (j < 0) break;
            ++pos[j];
            for (int i = j + 1; i < u; ++i) pos[i] = pos[i - 1] + 1;
        }
    }
    if (prune && prune->keep && cand != prune->n_keep)
        fail(TN_EINVAL, "prune keep array length does not match the candidate count");
    t->n = (int64_t)t->w.size();
    return t.release();
}

// ---------------------------------------------------------------------------
// Factored term set (exact cross-term reuse over independent clusters).  A
// term's amplitude is the product of its clusters' amplitudes and its weight
// the product of per-slot values, so X = prod_c X_c and the level sums of the
// full expansion are the coefficients of the product of per-cluster level
// polynomials g_c(k) (sums of X_c over the cluster's own patterns with k
// corrections): A(l) = sum_{k<=l} [prod_c g_c](k).  The engine evaluates only
// terms whose corrections all lie in one cluster; with X0 the all-dominant
// term, h_c(k) = sum of X over those of cluster c and level k equals
// g_c(k) X0 / g_c(0), so with r_c(0) = 1 and r_c(k) = h_c(k) / X0,
// A(l) = X0 sum_{k<=l} [prod_c r_c](k).
// Order: the all-dominant term; then for u = 1..level, for each cluster with
// at least u slots, its position subsets and corrections in the order of
// tn_terms_enumerate restricted to the cluster's slots (levels ascending).
// ---------------------------------------------------------------------------
Terms* enumerate_terms_factored(const Plan* p, int level) {
    if (level < 0) fail(TN_EINVAL, "level must be >= 0");
    if (p->doubled) fail(TN_EINVAL, "a doubled network has no slots to factor");
    if (p->trajectories) fail(TN_EINVAL, "a trajectories plan takes sampled terms (tn_terms_trajectories)");
    const int N = p->n_noise;
    const int L = std::min(level, N);
    if (L > TN_MAX_LEVEL) fail(TN_EINVAL, "level above TN_MAX_LEVEL");
    auto t = std::make_unique<Terms>();
    t->plan = p;
    t->plan_id = p->id;
    t->level = L;
    t->factored = true;
    auto push = [&](const std::vector<int8_t>& pat, int u) {
        double w = 1.0;
        bool zero = false;
        for (int s = 0; s < N; ++s) {
            w *= p->noise[s].d[pat[s]];
            zero |= p->noise[s].zero[pat[s]];
        }
        t->pat.insert(t->pat.end(), pat.begin(), pat.end());
        t->w.push_back(zero ? 0.0 : w);
        t->lvl.push_back((uint8_t)u);
        t->zero.push_back(zero ? 1 : 0);
        t->pruned.push_back(0);
    };
    t->group_start.push_back(0);
    t->group_level.push_back(0);
    t->group_cluster.push_back(-1);
    push(std::vector<int8_t>(N, 0), 0);
    std::vector<int> pos, corr;
    for (int u = 1; u <= L; ++u)
        for (size_t c = 0; c < p->clusters.size(); ++c) {
            const std::vector<int>& sl = p->clusters[c].slots;
            const int ns = (int)sl.size();
            if (ns < u) continue;
            t->group_start.push_back((int64_t)t->w.size());
            t->group_level.push_back(u);
            t->group_cluster.push_back((int32_t)c);
            pos.resize(u);
            for (int i = 0; i < u; ++i) pos[i] = i;
            while (true) {
                corr.assign(u, 1);
                while (true) {
                    std::vector<int8_t> pat(N, 0);
                    for (int i = 0; i < u; ++i) pat[sl[pos[i]]] = (int8_t)corr[i];
                    push(pat, u);
                    int j = u - 1;
                    while (j >= 0 && corr[j] == 3) corr[j--] = 1;
                    if (j < 0) break;
                    ++corr[j];
                }
                int j = u - 1;
                while (j >= 0 && pos[j] == ns - u + j) --j;
                if (j < 0) break;
                ++pos[j];
                for (int i = j + 1; i < u; ++i) pos[i] = pos[i - 1] + 1;
            }
        }
    t->n = (int64_t)t->w.size();
    t->group_start.push_back(t->n);
    return t.release();
}

// Quantum-trajectories samples: sample i draws, for noise s, the first Kraus
// index k (among those with q_k > 0) with u[i][s] < q_0 + ... + q_k; every
// sample has weight 1 / n_samples, so the level-0 sum is the sample mean.
Terms* sample_terms(const Plan* p, int64_t n_samples, const double* u) {
    if (!p->trajectories) fail(TN_EINVAL, "samples need a trajectories plan");
    if (n_samples < 1 || !u) fail(TN_EINVAL, "need at least one sample and its uniforms");
    const int N = p->n_noise;
    auto t = std::make_unique<Terms>();
    t->plan = p;
    t->plan_id = p->id;
    t->level = 0;
    const double w = 1.0 / (double)n_samples;
    t->pat.resize((size_t)n_samples * N);
    for (int64_t i = 0; i < n_samples; ++i) {
        for (int s = 0; s < N; ++s) {
            const NoiseSplit& ns = p->noise[s];
            const double x = u[i * N + s];
            if (!(x >= 0.0 && x < 1.0)) fail(TN_EINVAL, "uniforms must lie in [0, 1)");
            double acc = 0.0;
            int pick = -1, last = 0;
            for (int k = 0; k < 4; ++k) {
                if (ns.zero[k]) continue;
                acc += ns.q[k];
                last = k;
                if (x < acc) { pick = k; break; }
            }
            t->pat[(size_t)i * N + s] = (int8_t)(pick < 0 ? last : pick);
        }
        t->w.push_back(w);
        t->lvl.push_back(0);
        t->zero.push_back(0);
        t->pruned.push_back(0);
    }
    t->n = n_samples;
    return t.release();
}

void factored_levels(const Terms* t, const double* hs, double* A) {
    if (!t->factored) fail(TN_EINVAL, "not a factored term set");
    const int L = t->level;
    const double x0 = hs[0];
    if (L > 0 && x0 == 0.0)
        fail(TN_EDEGENERATE, "the all-dominant term is zero: the factored levels need X0 != 0");
    // r_c(k) per cluster (groups are ordered by level, then cluster)
    std::vector<std::vector<double>> rc(t->plan->clusters.size(), std::vector<double>(L + 1, 0.0));
    for (auto& v : rc) v[0] = 1.0;
    for (size_t g = 1; g < t->group_level.size(); ++g) rc[t->group_cluster[g]][t->group_level[g]] += hs[g] / x0;
    // prod_c r_c truncated at degree L, clusters in index order
    std::vector<double> poly(L + 1, 0.0);
    poly[0] = 1.0;
    for (const std::vector<double>& r : rc) {
        std::vector<double> np(L + 1, 0.0);
        for (int a = 0; a <= L; ++a)
            for (int b = 0; a + b <= L; ++b) np[a + b] += poly[a] * r[b];
        poly.swap(np);
    }
    double acc = 0.0;
    for (int k = 0; k <= L; ++k) {
        acc += poly[k];
        A[k] = x0 * acc;
    }
}

// ---------------------------------------------------------------------------
// pruning features of every term (kNumFeatures floats per term)
//   per corrected slot j = 0..2 (in position order; zeros when absent), 9:
//     present, log(d_i / d_0), one-hot(i) x3, position op_index / n_ops,
//     cone qubits / n, cone 2-qubit gates / all 2-qubit gates,
//     log X of the level-1 term with the same (slot, correction) (0 if absent)
//   per pair (0,1), (0,2), (1,2), 2: cone overlap / smaller cone, |position
//     difference| / n_ops
//   global, 3: log of the term weight prod d / 2^N, level, and log of the
//     rigorous bound of the term, weight * prod_s ||K_hat_{c_s}||_2^2
//     (|a| <= prod of the slot norms for unit boundary states)
// ---------------------------------------------------------------------------
int term_features(const Plan* p, const Terms* t, const double* level1_x, float* out) {
    const int N = p->n_noise;
    const double tiny = 1e-300;
    for (int64_t k = 0; k < t->n; ++k) {
        float* f = out + k * kNumFeatures;
        for (int i = 0; i < kNumFeatures; ++i) f[i] = 0.0f;
        const int8_t* pat = &t->pat[k * N];
        int slots[3], corr[3], u = 0;
        for (int s = 0; s < N && u < 3; ++s)
            if (pat[s]) {
                slots[u] = s;
                corr[u] = pat[s];
                ++u;
            }
        for (int j = 0; j < u; ++j) {
            const NoiseSplit& ns = p->noise[slots[j]];
            float* g = f + 9 * j;
            g[0] = 1.0f;
            g[1] = (float)std::log(std::max(ns.d[corr[j]], tiny) / ns.d[0]);
            g[2 + (corr[j] - 1)] = 1.0f;
            g[5] = (float)((double)ns.op_index / std::max<int64_t>(1, p->n_ops));
            g[6] = (float)((double)ns.cone_qubits / p->n_qubits);
            g[7] = (float)((double)ns.cone_2q_gates / std::max(1, p->n_2q_gates));
            if (level1_x) {
                const double x1 = level1_x[1 + 3 * slots[j] + (corr[j] - 1)];
                g[8] = (float)std::log(std::max(x1, tiny));
            }
        }
        const int pairs[3][2] = {{0, 1}, {0, 2}, {1, 2}};
        for (int q = 0; q < 3; ++q) {
            const int a = pairs[q][0], b = pairs[q][1];
            if (b >= u) continue;
            const NoiseSplit& na = p->noise[slots[a]];
            const NoiseSplit& nb = p->noise[slots[b]];
            int inter = 0;
            for (size_t w = 0; w < na.cone.size(); ++w) inter += __builtin_popcountll(na.cone[w] & nb.cone[w]);
            f[27 + 2 * q] = (float)inter / (float)std::max(1, std::min(na.cone_qubits, nb.cone_qubits));
            f[28 + 2 * q] = (float)((double)std::llabs(na.op_index - nb.op_index) / std::max<int64_t>(1, p->n_ops));
        }
        const double what = std::ldexp(t->w[k], -N);
        f[33] = (float)std::log(std::max(what, tiny));
        f[34] = (float)t->lvl[k];
        double lb = std::log(std::max(what, tiny));
        for (int s = 0; s < N; ++s) lb += std::log(p->noise[s].khat_norm2[pat[s]]);
        f[35] = (float)lb;
    }
    return kNumFeatures;
}

std::string describe_plan(const Plan* p) {
    std::ostringstream os;
    os.precision(17);
    os << "{\"n_qubits\":" << p->n_qubits << ",\"n_noise\":" << p->n_noise << ",\"level\":" << p->level
       << ",\"target\":\"" << p->target_kind << "\",\"scalar\":[" << p->scalar.real() << ","
       << p->scalar.imag() << "],\"max_log\":" << p->max_log << ",\"cmacs_per_term\":" << p->cmacs_per_term
       << ",\"leaves\":[";
    for (size_t i = 0; i < p->leaves.size(); ++i) {
        const Leaf& l = p->leaves[i];
        os << (i ? "," : "") << "{\"slot\":" << l.slot << ",\"legs\":[";
        for (size_t j = 0; j < l.legs.size(); ++j) os << (j ? "," : "") << l.legs[j];
        os << "],\"data\":[";
        for (size_t j = 0; j < l.data.size(); ++j)
            os << (j ? "," : "") << l.data[j].real() << "," << l.data[j].imag();
        os << "]}";
    }
    os << "],\"clusters\":[";
    for (size_t c = 0; c < p->clusters.size(); ++c) {
        const Cluster& cl = p->clusters[c];
        os << (c ? "," : "") << "{\"leaves\":[";
        for (size_t j = 0; j < cl.leaves.size(); ++j) os << (j ? "," : "") << cl.leaves[j];
        os << "],\"slots\":[";
        for (size_t j = 0; j < cl.slots.size(); ++j) os << (j ? "," : "") << cl.slots[j];
        os << "],\"path\":[";
        for (size_t j = 0; j < cl.path.size(); ++j)
            os << (j ? "," : "") << "[" << cl.path[j].a << "," << cl.path[j].b << "]";
        os << "],\"cmacs_per_term\":" << cl.cmacs_per_term << ",\"max_log\":" << cl.max_log << "}";
    }
    os << "]}";
    return os.str();
}

}  // namespace tn
