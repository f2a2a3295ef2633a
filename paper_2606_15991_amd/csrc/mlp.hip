// mlp.hip -- training kernels of the tile-picker cost model: a multilayer
// perceptron with `depth` hidden ReLU layers of `hidden` units and one linear
// output, regressing log(time) of a (shape, configuration) pair.
//
// Forward:  H_0 = X,  H_l = relu(H_{l-1} W_l^T + b_l),  out = H_depth w^T + b
// Loss:     L = (1/B) sum_b (out_b - y_b)^2
// Backward: dZ_out = 2 (out - y) / B; for each layer, dW = dZ^T H_prev,
//           db = column sums of dZ, dH_prev = dZ W masked by H_prev > 0.
// Every reduction runs in a fixed order in one thread or one workgroup:
// no atomics, identical results on every run.  Parameters per layer are W
// (out x in, row-major) followed by b (out).
#include <math.h>

#include "host_internal.hpp"
#include "tg_device.hpp"

namespace tg {
namespace {

// Y[b][o] = act(sum_i X[b][i] W[o][i] + bias[o])
__global__ void dense_fwd(const float *__restrict__ X,
                          const float *__restrict__ W,
                          const float *__restrict__ bias, float *__restrict__ Y,
                          int batch, int in, int out, int relu) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (int64_t)batch * out) return;
    const int b = (int)(e / out), o = (int)(e % out);
    float s = bias[o];
    const float *x = X + (int64_t)b * in;
    const float *w = W + (int64_t)o * in;
    for (int i = 0; i < in; ++i) s = fmaf(x[i], w[i], s);
    Y[e] = (relu && s < 0.f) ? 0.f : s;
}

// dZ[b] = 2 (out[b] - y[b]) / B and loss = (1/B) sum (out - y)^2, one
// workgroup, fixed order.
__global__ __launch_bounds__(256) void loss_grad(const float *__restrict__ out,
                                                 const float *__restrict__ y,
                                                 float *__restrict__ dz,
                                                 float *__restrict__ loss,
                                                 int batch) {
    __shared__ float part[256];
    float s = 0.f;
    const float inv = 1.0f / (float)batch;
    for (int b = threadIdx.x; b < batch; b += 256) {
        const float d = out[b] - y[b];
        dz[b] = 2.0f * d * inv;
        s = fmaf(d, d, s);
    }
    part[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) part[threadIdx.x] += part[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) *loss = part[0] * inv;
}

// dW[o][i] = sum_b dZ[b][o] H[b][i]  (i < in);  db[o] = sum_b dZ[b][o]
// (thread i == in).  One thread per output entry, batch summed in order.
__global__ void dense_bwd_weight(const float *__restrict__ dZ,
                                 const float *__restrict__ H,
                                 float *__restrict__ dW,
                                 float *__restrict__ db, int batch, int in,
                                 int out) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= out * (in + 1)) return;
    const int o = e / (in + 1), i = e % (in + 1);
    float s = 0.f;
    if (i < in) {
        for (int b = 0; b < batch; ++b)
            s = fmaf(dZ[(int64_t)b * out + o], H[(int64_t)b * in + i], s);
        dW[(int64_t)o * in + i] = s;
    } else {
        for (int b = 0; b < batch; ++b) s += dZ[(int64_t)b * out + o];
        db[o] = s;
    }
}

// dH[b][i] = (H[b][i] > 0) * sum_o dZ[b][o] W[o][i]
__global__ void dense_bwd_input(const float *__restrict__ dZ,
                                const float *__restrict__ W,
                                const float *__restrict__ H,
                                float *__restrict__ dH, int batch, int in,
                                int out) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (int64_t)batch * in) return;
    const int b = (int)(e / in), i = (int)(e % in);
    if (!(H[e] > 0.f)) {
        dH[e] = 0.f;
        return;
    }
    float s = 0.f;
    for (int o = 0; o < out; ++o)
        s = fmaf(dZ[(int64_t)b * out + o], W[(int64_t)o * in + i], s);
    dH[e] = s;
}

// Adam (Kingma & Ba): m = b1 m + (1-b1) g; v = b2 v + (1-b2) g^2;
// p -= lr * (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps)
// The constants 1 - b1, 1 - b2 and the bias corrections are formed in
// binary64 on the host: 1 - 0.999 in binary32 loses 4 significant digits.
__global__ void adam_step(float *__restrict__ p, const float *__restrict__ g,
                          float *__restrict__ m, float *__restrict__ v,
                          int64_t n, float lr, float b1, float b2, float omb1,
                          float omb2, float eps, float c1, float c2) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n) return;
    const float gi = g[e];
    const float mi = b1 * m[e] + omb1 * gi;
    const float vi = b2 * v[e] + omb2 * (gi * gi);
    m[e] = mi;
    v[e] = vi;
    p[e] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

inline unsigned blocks_for(int64_t n, int t) {
    return (unsigned)((n + t - 1) / t);
}

struct Layout {
    int n_in, hidden, depth, batch;
    // parameter offsets of layer l's W and b (l = 0 .. depth; depth = output)
    size_t w_off(int l) const {
        size_t off = 0;
        int in = n_in;
        for (int k = 0; k < l; ++k) {
            const int out = k < depth ? hidden : 1;
            off += (size_t)out * in + out;
            in = out;
        }
        return off;
    }
    int in_of(int l) const { return l == 0 ? n_in : hidden; }
    int out_of(int l) const { return l < depth ? hidden : 1; }
    // workspace: H_1..H_depth (batch x hidden each), out (batch), two dZ
    // buffers (batch x hidden), the loss
    size_t ws_floats() const {
        return (size_t)depth * batch * hidden + batch +
               2 * (size_t)batch * hidden + 4;
    }
};

hipError_t forward(const Layout &L, const float *params, const float *X,
                   float *ws, float *out, hipStream_t st) {
    const float *prev = X;
    for (int l = 0; l <= L.depth; ++l) {
        const int in = L.in_of(l), o = L.out_of(l);
        const float *W = params + L.w_off(l);
        const float *b = W + (size_t)o * in;
        float *Y = l < L.depth ? ws + (size_t)l * L.batch * L.hidden : out;
        hipLaunchKernelGGL(dense_fwd, dim3(blocks_for((int64_t)L.batch * o,
                                                      256)),
                           dim3(256), 0, st, prev, W, b, Y, L.batch, in, o,
                           l < L.depth ? 1 : 0);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        prev = Y;
    }
    return hipSuccess;
}

}  // namespace
}  // namespace tg

using namespace tg;

extern "C" {

size_t tile_mlp_workspace_bytes(int32_t n_in, int32_t hidden, int32_t depth,
                                int32_t batch) {
    if (n_in <= 0 || hidden <= 0 || depth <= 0 || batch <= 0) return 0;
    Layout L{n_in, hidden, depth, batch};
    return L.ws_floats() * sizeof(float);
}

static tg_status check_mlp(const float *params, int32_t n_in, int32_t hidden,
                           int32_t depth, const float *X, int32_t batch,
                           void *ws, size_t ws_bytes) {
    if (!params || !X || n_in <= 0 || hidden <= 0 || depth <= 0 || batch <= 0)
        return TG_E_ARG;
    if (!ws || ws_bytes < tile_mlp_workspace_bytes(n_in, hidden, depth, batch))
        return TG_E_WORKSPACE;
    return TG_OK;
}

tg_status tile_mlp_forward(const float *params, int32_t n_in, int32_t hidden,
                           int32_t depth, const float *X, int32_t batch,
                           float *out, void *ws, size_t ws_bytes,
                           tg_stream stream) {
    tg_status st = check_mlp(params, n_in, hidden, depth, X, batch, ws,
                             ws_bytes);
    if (st != TG_OK) return st;
    if (!out) return TG_E_ARG;
    Layout L{n_in, hidden, depth, batch};
    hipError_t e = forward(L, params, X, static_cast<float *>(ws), out,
                           static_cast<hipStream_t>(stream));
    return e == hipSuccess ? TG_OK : TG_E_HIP;
}

tg_status tile_mlp_loss_grad(const float *params, int32_t n_in,
                             int32_t hidden, int32_t depth, const float *X,
                             const float *y, int32_t batch, float *grads,
                             float *loss, void *ws, size_t ws_bytes,
                             tg_stream stream) {
    tg_status st = check_mlp(params, n_in, hidden, depth, X, batch, ws,
                             ws_bytes);
    if (st != TG_OK) return st;
    if (!y || !grads || !loss) return TG_E_ARG;
    hipStream_t hs = static_cast<hipStream_t>(stream);
    Layout L{n_in, hidden, depth, batch};
    float *w = static_cast<float *>(ws);
    float *acts = w;                                        // H_1..H_depth
    float *out = w + (size_t)depth * batch * hidden;        // batch
    float *dz0 = out + batch;                               // batch x hidden
    float *dz1 = dz0 + (size_t)batch * hidden;              // batch x hidden
    hipError_t e = forward(L, params, X, w, out, hs);
    if (e != hipSuccess) return TG_E_HIP;
    hipLaunchKernelGGL(loss_grad, dim3(1), dim3(256), 0, hs, out, y, dz0, loss,
                       batch);
    if ((e = hipGetLastError()) != hipSuccess) return TG_E_HIP;
    float *dz = dz0, *dprev = dz1;
    for (int l = depth; l >= 0; --l) {
        const int in = L.in_of(l), o = L.out_of(l);
        const float *H = l == 0 ? X : acts + (size_t)(l - 1) * batch * hidden;
        const float *W = params + L.w_off(l);
        float *dW = grads + L.w_off(l);
        float *db = dW + (size_t)o * in;
        hipLaunchKernelGGL(dense_bwd_weight, dim3(blocks_for(o * (in + 1), 256)),
                           dim3(256), 0, hs, dz, H, dW, db, batch, in, o);
        if ((e = hipGetLastError()) != hipSuccess) return TG_E_HIP;
        if (l > 0) {
            hipLaunchKernelGGL(dense_bwd_input,
                               dim3(blocks_for((int64_t)batch * in, 256)),
                               dim3(256), 0, hs, dz, W, H, dprev, batch, in, o);
            if ((e = hipGetLastError()) != hipSuccess) return TG_E_HIP;
            float *t = dz;
            dz = dprev;
            dprev = t;
        }
    }
    return TG_OK;
}

tg_status tile_mlp_adam(float *params, const float *grads, float *m, float *v,
                        int64_t n, double lr, double beta1, double beta2,
                        double eps, int32_t t, tg_stream stream) {
    if (!params || !grads || !m || !v || n < 0 || t < 1) return TG_E_ARG;
    if (n == 0) return TG_OK;
    const float c1 = (float)(1.0 - pow(beta1, (double)t));
    const float c2 = (float)(1.0 - pow(beta2, (double)t));
    hipLaunchKernelGGL(adam_step, dim3(blocks_for(n, 256)), dim3(256), 0,
                       static_cast<hipStream_t>(stream), params, grads, m, v,
                       n, (float)lr, (float)beta1, (float)beta2,
                       (float)(1.0 - beta1), (float)(1.0 - beta2), (float)eps,
                       c1, c2);
    return hipGetLastError() == hipSuccess ? TG_OK : TG_E_HIP;
}

}  // extern "C"
