// Term-pruning MLP: forward, backward and Adam kernels (FP32, gfx950).
//
// A small fully connected network reads per-term features (slot positions,
// singular values, light-cone sizes, gate neighbourhoods, level-1 magnitudes,
// weight) and predicts log X of a level-2/3 term.  It is trained on the term
// values the estimate itself produces.  Layout of the state buffer (floats):
//   [ mean[n_in] | inv_std[n_in] | params P | grads P | adam m P | adam v P ]
// params: per layer l, W_l (out_l x in_l, row-major) then b_l (out_l); layers
// n_in -> width (ReLU) -> ... -> width (ReLU) -> 1 (linear).
// All reductions run in a fixed order (no atomics), so results are
// deterministic.

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <random>
#include <string>
#include <vector>

#include "tn_internal.h"
#include "tn_mlp.h"

namespace tn {

#define HIPCHK_M(x)                                                                        \
    do {                                                                                   \
        hipError_t e_ = (x);                                                               \
        if (e_ != hipSuccess) fail(TN_EHIP, std::string(#x) + ": " + hipGetErrorString(e_)); \
    } while (0)

struct MlpLayout {
    int n_in, width, depth, n_layers;
    std::vector<int> din, dout;
    std::vector<int64_t> w_off, b_off;   // offsets inside params
    int64_t P;                           // parameter count
    int64_t norm_off, params_off, grads_off, m_off, v_off, total;
};

static MlpLayout layout_of(const tn_mlp_shape* s) {
    if (!s || s->n_in < 1 || s->n_in > 4096 || s->width < 1 || s->width > 4096 || s->depth < 1 || s->depth > 16)
        fail(TN_EINVAL, "bad MLP shape");
    MlpLayout L;
    L.n_in = s->n_in;
    L.width = s->width;
    L.depth = s->depth;
    L.n_layers = s->depth + 1;
    int64_t off = 0;
    for (int l = 0; l < L.n_layers; ++l) {
        const int din = l == 0 ? s->n_in : s->width;
        const int dout = l == L.n_layers - 1 ? 1 : s->width;
        L.din.push_back(din);
        L.dout.push_back(dout);
        L.w_off.push_back(off);
        off += (int64_t)din * dout;
        L.b_off.push_back(off);
        off += dout;
    }
    L.P = off;
    L.norm_off = 0;
    L.params_off = 2 * (int64_t)s->n_in;
    L.grads_off = L.params_off + L.P;
    L.m_off = L.grads_off + L.P;
    L.v_off = L.m_off + L.P;
    L.total = L.v_off + L.P;
    return L;
}

// workspace floats for a batch of n: normalized input, activations per hidden
// layer, output, two gradient buffers, loss partials
static int64_t ws_floats(const MlpLayout& L, int64_t n) {
    return n * L.n_in + (int64_t)L.depth * n * L.width + n + 2 * n * std::max(L.width, L.n_in) + 64 +
           std::max<int64_t>(4096, n / 64 + 64);
}

// ---------------------------------------------------------------------------
// kernels
// ---------------------------------------------------------------------------
__global__ void k_fill(float* p, int64_t n, float v) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// column mean and 1/std of x (n x d); one block per column, FP64 accumulation
__global__ __launch_bounds__(256) void k_col_stats(const float* x, int64_t n, int d, float* mean, float* istd) {
    __shared__ double s1[256], s2[256];
    const int c = blockIdx.x;
    double a = 0, b = 0;
    for (int64_t r = threadIdx.x; r < n; r += 256) {
        const double v = x[r * d + c];
        a += v;
        b += v * v;
    }
    s1[threadIdx.x] = a;
    s2[threadIdx.x] = b;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            s1[threadIdx.x] += s1[threadIdx.x + w];
            s2[threadIdx.x] += s2[threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double m = s1[0] / (double)n;
        const double var = s2[0] / (double)n - m * m;
        mean[c] = (float)m;
        istd[c] = var > 1e-12 ? (float)(1.0 / sqrt(var)) : 1.0f;
    }
}

__global__ void k_normalize(const float* x, const float* mean, const float* istd, float* y, int64_t n, int d) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n * d) return;
    const int c = (int)(i % d);
    y[i] = (x[i] - mean[c]) * istd[c];
}

// Y[n x out] = act(X[n x in] W^T + b); 64 x 64 output tile, 256 threads with
// 4 x 4 outputs each, inputs staged through LDS in chunks of 16
__global__ __launch_bounds__(256) void k_linear_fwd(const float* __restrict__ X, const float* __restrict__ W,
                                                    const float* __restrict__ b, float* __restrict__ Y, int64_t n,
                                                    int din, int dout, int relu) {
    __shared__ float Xs[16][64 + 1];
    __shared__ float Ws[16][64 + 1];
    const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
    const int64_t r0 = (int64_t)blockIdx.x * 64;
    const int o0 = blockIdx.y * 64;
    float acc[4][4] = {};
    for (int k0 = 0; k0 < din; k0 += 16) {
        for (int e = threadIdx.x; e < 16 * 64; e += 256) {
            const int kk = e & 15, rr = e >> 4;
            const int64_t r = r0 + rr;
            const int o = o0 + rr;
            Xs[kk][rr] = (r < n && k0 + kk < din) ? X[r * din + k0 + kk] : 0.0f;
            Ws[kk][rr] = (o < dout && k0 + kk < din) ? W[(int64_t)o * din + k0 + kk] : 0.0f;
        }
        __syncthreads();
        for (int kk = 0; kk < 16; ++kk) {
            float xv[4], wv[4];
            for (int i = 0; i < 4; ++i) xv[i] = Xs[kk][ty + 16 * i];
            for (int j = 0; j < 4; ++j) wv[j] = Ws[kk][tx + 16 * j];
            for (int i = 0; i < 4; ++i)
                for (int j = 0; j < 4; ++j) acc[i][j] = fmaf(xv[i], wv[j], acc[i][j]);
        }
        __syncthreads();
    }
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) {
            const int64_t r = r0 + ty + 16 * i;
            const int o = o0 + tx + 16 * j;
            if (r < n && o < dout) {
                float v = acc[i][j] + b[o];
                if (relu) v = v > 0.0f ? v : 0.0f;
                Y[r * dout + o] = v;
            }
        }
}

// squared-error gradient: dY = 2 w (y - t) / n; per-block partial losses (FP64)
__global__ __launch_bounds__(256) void k_loss_grad(const float* y, const float* t, const float* w, float* dy,
                                                   double* part, int64_t n) {
    __shared__ double red[256];
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    double l = 0;
    if (i < n) {
        const float wi = w ? w[i] : 1.0f;
        const float d = y[i] - t[i];
        dy[i] = 2.0f * wi * d / (float)n;
        l = (double)wi * (double)d * (double)d;
    }
    red[threadIdx.x] = l;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__global__ __launch_bounds__(256) void k_loss_reduce(const double* part, int nb, int64_t n, float* loss) {
    __shared__ double red[256];
    double s = 0;
    for (int i = threadIdx.x; i < nb; i += 256) s += part[i];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) *loss = (float)(red[0] / (double)n);
}

// dX[n x din] = (dZ[n x dout] W) * (A_prev > 0): gradient through a layer and
// the previous layer's ReLU (A_prev is that layer's output)
__global__ __launch_bounds__(256) void k_linear_bwd_data(const float* __restrict__ dZ, const float* __restrict__ W,
                                                         const float* __restrict__ Aprev, float* __restrict__ dX,
                                                         int64_t n, int din, int dout) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= n * din) return;
    const int64_t r = idx / din;
    const int i = (int)(idx - r * din);
    float s = 0.0f;
    for (int o = 0; o < dout; ++o) s = fmaf(dZ[r * dout + o], W[(int64_t)o * din + i], s);
    dX[idx] = Aprev[idx] > 0.0f ? s : 0.0f;
}

// dW[o][i] = sum_r dZ[r][o] A[r][i], db[o] = sum_r dZ[r][o]; one thread per
// weight (bias when i == din), rows summed in order
__global__ __launch_bounds__(256) void k_linear_bwd_weight(const float* __restrict__ dZ, const float* __restrict__ A,
                                                           float* __restrict__ dW, float* __restrict__ db, int64_t n,
                                                           int din, int dout) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (int64_t)dout * (din + 1)) return;
    const int o = (int)(idx / (din + 1));
    const int i = (int)(idx - (int64_t)o * (din + 1));
    double s = 0.0;
    if (i < din) {
        for (int64_t r = 0; r < n; ++r) s += (double)dZ[r * dout + o] * (double)A[r * din + i];
        dW[(int64_t)o * din + i] = (float)s;
    } else {
        for (int64_t r = 0; r < n; ++r) s += (double)dZ[r * dout + o];
        db[o] = (float)s;
    }
}

__global__ void k_adam(float* p, const float* g, float* m, float* v, int64_t P, float lr, float b1, float b2,
                       float eps, float c1, float c2) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= P) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

__global__ void k_log_targets(const double* x, float* t, int64_t n, double floor_v) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) t[i] = (float)log(x[i] > floor_v ? x[i] : floor_v);
}

static unsigned nblk(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

// forward through all layers; activations kept in the workspace
static void forward(const MlpLayout& L, const float* state, const float* x, int64_t n, float* ws, hipStream_t s,
                    float** out_y) {
    float* xn = ws;
    float* acts = xn + n * L.n_in;
    float* y = acts + (int64_t)L.depth * n * L.width;
    hipLaunchKernelGGL(k_normalize, dim3(nblk(n * L.n_in, 256)), dim3(256), 0, s, x, state + L.norm_off,
                       state + L.norm_off + L.n_in, xn, n, L.n_in);
    const float* in = xn;
    const float* params = state + L.params_off;
    for (int l = 0; l < L.n_layers; ++l) {
        const bool last = l == L.n_layers - 1;
        float* out = last ? y : acts + (int64_t)l * n * L.width;
        dim3 grid(nblk(n, 64), nblk(L.dout[l], 64));
        hipLaunchKernelGGL(k_linear_fwd, grid, dim3(256), 0, s, in, params + L.w_off[l], params + L.b_off[l], out, n,
                           L.din[l], L.dout[l], last ? 0 : 1);
        in = out;
    }
    *out_y = y;
}

static void gradients(const MlpLayout& L, float* state, const float* x, const float* t, const float* w, int64_t n,
                      float* ws, float* loss, hipStream_t s) {
    float* y = nullptr;
    forward(L, state, x, n, ws, s, &y);
    float* xn = ws;
    float* acts = xn + n * L.n_in;
    float* g0 = y + n;
    float* g1 = g0 + n * std::max(L.width, L.n_in);
    // FP64 partials start on a 256-byte boundary (the float regions before
    // them can have odd length)
    const int64_t part_off = ((g1 - ws) + n * std::max(L.width, L.n_in) + 63) / 64 * 64;
    double* part = (double*)(ws + part_off);
    const unsigned nb = nblk(n, 256);
    hipLaunchKernelGGL(k_loss_grad, dim3(nb), dim3(256), 0, s, y, t, w, g0, part, n);
    hipLaunchKernelGGL(k_loss_reduce, dim3(1), dim3(256), 0, s, part, (int)nb, n, loss);
    float* params = state + L.params_off;
    float* grads = state + L.grads_off;
    float* dz = g0;     // gradient w.r.t. the current layer's pre-activation
    float* other = g1;
    for (int l = L.n_layers - 1; l >= 0; --l) {
        const float* a_prev = l == 0 ? xn : acts + (int64_t)(l - 1) * n * L.width;
        const int64_t nw = (int64_t)L.dout[l] * (L.din[l] + 1);
        hipLaunchKernelGGL(k_linear_bwd_weight, dim3(nblk(nw, 256)), dim3(256), 0, s, dz, a_prev,
                           grads + L.w_off[l], grads + L.b_off[l], n, L.din[l], L.dout[l]);
        if (l > 0) {
            hipLaunchKernelGGL(k_linear_bwd_data, dim3(nblk(n * L.din[l], 256)), dim3(256), 0, s, dz,
                               params + L.w_off[l], a_prev, other, n, L.din[l], L.dout[l]);
            std::swap(dz, other);
        }
    }
}

}  // namespace tn

using namespace tn;

template <class F>
static int mguard(F&& f) {
    try {
        f();
        set_last_error("");
        return TN_OK;
    } catch (const Error& e) {
        set_last_error(e.msg);
        return e.code;
    } catch (const std::exception& e) {
        set_last_error(e.what());
        return TN_EINVAL;
    }
}

extern "C" {

int tn_mlp_sizes(const tn_mlp_shape* s, int64_t batch, int64_t* n_params, size_t* state_bytes, size_t* ws_bytes) {
    return mguard([&] {
        MlpLayout L = layout_of(s);
        if (n_params) *n_params = L.P;
        if (state_bytes) *state_bytes = (size_t)L.total * 4;
        if (ws_bytes) *ws_bytes = (size_t)ws_floats(L, std::max<int64_t>(1, batch)) * 4 + 4096 * 8;
    });
}

int tn_mlp_init(const tn_mlp_shape* s, uint64_t seed, void* d_state, void* stream) {
    return mguard([&] {
        MlpLayout L = layout_of(s);
        if (!d_state) fail(TN_EINVAL, "null state");
        std::vector<float> h(L.total, 0.0f);
        for (int i = 0; i < L.n_in; ++i) h[L.norm_off + L.n_in + i] = 1.0f;   // identity normalizer
        std::mt19937_64 rng(seed ? seed : 2211170280ULL);
        for (int l = 0; l < L.n_layers; ++l) {
            std::normal_distribution<double> nd(0.0, std::sqrt(2.0 / L.din[l]));   // He initialisation
            for (int64_t k = 0; k < (int64_t)L.din[l] * L.dout[l]; ++k) h[L.params_off + L.w_off[l] + k] = (float)nd(rng);
        }
        hipStream_t st = (hipStream_t)stream;
        HIPCHK_M(hipMemcpyAsync(d_state, h.data(), h.size() * 4, hipMemcpyHostToDevice, st));
        HIPCHK_M(hipStreamSynchronize(st));
    });
}

int tn_mlp_fit_normalizer(const tn_mlp_shape* s, void* d_state, const float* d_x, int64_t n, void* stream) {
    return mguard([&] {
        MlpLayout L = layout_of(s);
        if (!d_state || !d_x || n < 1) fail(TN_EINVAL, "bad normalizer arguments");
        float* st = (float*)d_state;
        hipLaunchKernelGGL(k_col_stats, dim3(L.n_in), dim3(256), 0, (hipStream_t)stream, d_x, n, L.n_in,
                           st + L.norm_off, st + L.norm_off + L.n_in);
        HIPCHK_M(hipGetLastError());
    });
}

int tn_mlp_forward(const tn_mlp_shape* s, const void* d_state, const float* d_x, int64_t n, float* d_y, void* d_ws,
                   void* stream) {
    return mguard([&] {
        MlpLayout L = layout_of(s);
        if (!d_state || !d_x || !d_y || !d_ws || n < 1) fail(TN_EINVAL, "bad forward arguments");
        float* y = nullptr;
        forward(L, (const float*)d_state, d_x, n, (float*)d_ws, (hipStream_t)stream, &y);
        HIPCHK_M(hipMemcpyAsync(d_y, y, n * 4, hipMemcpyDeviceToDevice, (hipStream_t)stream));
        HIPCHK_M(hipGetLastError());
    });
}

int tn_mlp_gradients(const tn_mlp_shape* s, void* d_state, const float* d_x, const float* d_t, const float* d_w,
                     int64_t n, void* d_ws, float* d_loss, void* stream) {
    return mguard([&] {
        MlpLayout L = layout_of(s);
        if (!d_state || !d_x || !d_t || !d_ws || !d_loss || n < 1) fail(TN_EINVAL, "bad gradient arguments");
        gradients(L, (float*)d_state, d_x, d_t, d_w, n, (float*)d_ws, d_loss, (hipStream_t)stream);
        HIPCHK_M(hipGetLastError());
    });
}

int tn_mlp_adam(const tn_mlp_shape* s, void* d_state, float lr, int32_t step, void* stream) {
    return mguard([&] {
        MlpLayout L = layout_of(s);
        if (!d_state || step < 1) fail(TN_EINVAL, "bad adam arguments");
        const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
        const float c1 = 1.0f - std::pow(b1, (float)step), c2 = 1.0f - std::pow(b2, (float)step);
        float* st = (float*)d_state;
        hipLaunchKernelGGL(k_adam, dim3(nblk(L.P, 256)), dim3(256), 0, (hipStream_t)stream, st + L.params_off,
                           st + L.grads_off, st + L.m_off, st + L.v_off, L.P, lr, b1, b2, eps, c1, c2);
        HIPCHK_M(hipGetLastError());
    });
}

int tn_mlp_log_targets(const double* d_x, float* d_t, int64_t n, double floor_v, void* stream) {
    return mguard([&] {
        if (!d_x || !d_t || n < 0 || !(floor_v > 0)) fail(TN_EINVAL, "bad target arguments");
        if (n == 0) return;
        hipLaunchKernelGGL(k_log_targets, dim3(nblk(n, 256)), dim3(256), 0, (hipStream_t)stream, d_x, d_t, n, floor_v);
        HIPCHK_M(hipGetLastError());
    });
}

int tn_mlp_train_step(const tn_mlp_shape* s, void* d_state, const float* d_x, const float* d_t, const float* d_w,
                      int64_t n, float lr, int32_t step, void* d_ws, float* d_loss, void* stream) {
    int rc = tn_mlp_gradients(s, d_state, d_x, d_t, d_w, n, d_ws, d_loss, stream);
    if (rc != TN_OK) return rc;
    return tn_mlp_adam(s, d_state, lr, step, stream);
}

int tn_pruner_train_step(const tn_mlp_shape* s, void* d_state, const float* d_x, const float* d_t,
                         const float* d_w, int64_t n, float lr, int32_t step, void* d_ws, float* d_loss,
                         void* stream) {
    return tn_mlp_train_step(s, d_state, d_x, d_t, d_w, n, lr, step, d_ws, d_loss, stream);
}

// saved model: header {magic, n_in, width, depth, P} then normalizer and parameters
static const char kPrunerMagic[8] = {'T', 'N', 'P', 'R', 'U', 'N', 'E', '1'};

int tn_pruner_save(const tn_mlp_shape* s, const void* d_state, void* h_buf, size_t buf_bytes, size_t* need_bytes,
                   void* stream) {
    return mguard([&] {
        MlpLayout L = layout_of(s);
        const size_t body = (size_t)(L.params_off + L.P) * 4;
        const size_t need = TN_PRUNER_HEADER_BYTES + body;
        if (need_bytes) *need_bytes = need;
        if (!h_buf) return;
        if (!d_state) fail(TN_EINVAL, "null state");
        if (buf_bytes < need) fail(TN_ENOMEM, "buffer smaller than the saved model");
        unsigned char* h = (unsigned char*)h_buf;
        std::memset(h, 0, TN_PRUNER_HEADER_BYTES);
        std::memcpy(h, kPrunerMagic, 8);
        const int32_t dims[3] = {s->n_in, s->width, s->depth};
        std::memcpy(h + 8, dims, sizeof(dims));
        const int64_t P = L.P;
        std::memcpy(h + 24, &P, 8);
        hipStream_t st = (hipStream_t)stream;
        HIPCHK_M(hipMemcpyAsync(h + TN_PRUNER_HEADER_BYTES, d_state, body, hipMemcpyDeviceToHost, st));
        HIPCHK_M(hipStreamSynchronize(st));
    });
}

int tn_pruner_load(const tn_mlp_shape* s, void* d_state, const void* h_buf, size_t buf_bytes, void* stream) {
    return mguard([&] {
        MlpLayout L = layout_of(s);
        const size_t body = (size_t)(L.params_off + L.P) * 4;
        if (!d_state || !h_buf) fail(TN_EINVAL, "null pointer");
        if (buf_bytes < TN_PRUNER_HEADER_BYTES + body) fail(TN_EINVAL, "buffer shorter than the saved model");
        const unsigned char* h = (const unsigned char*)h_buf;
        int32_t dims[3];
        int64_t P;
        std::memcpy(dims, h + 8, sizeof(dims));
        std::memcpy(&P, h + 24, 8);
        if (std::memcmp(h, kPrunerMagic, 8) != 0) fail(TN_EINVAL, "not a saved pruner model");
        if (dims[0] != s->n_in || dims[1] != s->width || dims[2] != s->depth || P != L.P)
            fail(TN_EINVAL, "saved model has another shape");
        hipStream_t st = (hipStream_t)stream;
        // normalizer and parameters; gradients and Adam moments start from zero
        std::vector<float> zeros((size_t)(L.total - L.grads_off), 0.0f);
        HIPCHK_M(hipMemcpyAsync(d_state, h + TN_PRUNER_HEADER_BYTES, body, hipMemcpyHostToDevice, st));
        HIPCHK_M(hipMemcpyAsync((float*)d_state + L.grads_off, zeros.data(), zeros.size() * 4,
                                hipMemcpyHostToDevice, st));
        HIPCHK_M(hipStreamSynchronize(st));
    });
}

}  // extern "C"
