// k_mlp.hip -- the plan cost model: a 48-128-128-1 FP32 MLP trained on the
// GPU by the library's own forward, backward and Adam kernels.
//
// The paper's optimiser minimises the number of gate blocks (Sec. IV, Eq. 7);
// the learned planner replaces that count by a predicted run time per block
// and keeps the heuristic as fallback.  The network and its training step
// follow the FP64 reference in the test oracle:
//   h1 = relu(X W1^T + b1), h2 = relu(h1 W2^T + b2), y = h2 W3^T + b3,
//   L = mean (y - t)^2, gradients by the chain rule (relu'(0) = 0), Adam with
//   bias correction.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "qs_internal.h"

namespace qs {
namespace {

constexpr int NI = QS_COST_FEATURES, NH = 128, MAXB = 1024;
constexpr int OFF_W1 = 0, OFF_B1 = OFF_W1 + NH * NI, OFF_W2 = OFF_B1 + NH, OFF_B2 = OFF_W2 + NH * NH,
              OFF_W3 = OFF_B2 + NH, OFF_B3 = OFF_W3 + NH, NPARAM = OFF_B3 + 1;

// out[b][o] = act(sum_i in[b][i] W[o][i] + bias[o]); z keeps the
// pre-activation when non-null.  One thread per (b, o); fixed summation order.
__global__ void k_linear_fwd(const float *__restrict__ in, int B, int nin, const float *__restrict__ W,
                             const float *__restrict__ bias, int nout, float *__restrict__ z, float *__restrict__ out,
                             int relu)
{
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= B * nout) return;
    const int b = idx / nout, o = idx % nout;
    float s = bias[o];
    for (int i = 0; i < nin; ++i) s = fmaf(in[b * nin + i], W[o * nin + i], s);
    if (z) z[idx] = s;
    out[idx] = relu ? fmaxf(s, 0.f) : s;
}

// dy[b] = 2/B (y[b] - t[b]); loss[0] = mean (y - t)^2 (single block).
__global__ void k_mse(const float *__restrict__ y, const float *__restrict__ t, int B, float *__restrict__ dy,
                      float *__restrict__ loss)
{
    __shared__ float red[256];
    float s = 0.f;
    for (int b = threadIdx.x; b < B; b += blockDim.x) {
        const float d = y[b] - t[b];
        dy[b] = 2.f * d / (float)B;
        s = fmaf(d, d, s);
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = blockDim.x / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) loss[0] = red[0] / (float)B;
}

// din[b][i] = (sum_o dout[b][o] W[o][i]) * (zin[b][i] > 0 if zin)
__global__ void k_linear_bwd_in(const float *__restrict__ dout, int B, int nout, const float *__restrict__ W, int nin,
                                const float *__restrict__ zin, float *__restrict__ din)
{
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= B * nin) return;
    const int b = idx / nin, i = idx % nin;
    float s = 0.f;
    for (int o = 0; o < nout; ++o) s = fmaf(dout[b * nout + o], W[o * nin + i], s);
    if (zin && !(zin[idx] > 0.f)) s = 0.f;
    din[idx] = s;
}

// gW[o][i] = sum_b dout[b][o] in[b][i]; gb[o] = sum_b dout[b][o]
__global__ void k_linear_bwd_w(const float *__restrict__ dout, const float *__restrict__ in, int B, int nout, int nin,
                               float *__restrict__ gW, float *__restrict__ gb)
{
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx < nout * nin) {
        const int o = idx / nin, i = idx % nin;
        float s = 0.f;
        for (int b = 0; b < B; ++b) s = fmaf(dout[b * nout + o], in[b * nin + i], s);
        gW[idx] = s;
    } else if (idx < nout * nin + nout) {
        const int o = idx - nout * nin;
        float s = 0.f;
        for (int b = 0; b < B; ++b) s += dout[b * nout + o];
        gb[o] = s;
    }
}

// a[i] = b[i] = 0 (the Adam moments)
__global__ void k_zero2(float *__restrict__ a, float *__restrict__ b, int n)
{
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        a[i] = 0.f;
        b[i] = 0.f;
    }
}

// Adam with bias correction; omb1 = 1 - b1 and omb2 = 1 - b2 come from the
// host in double precision (1 - 0.999f in FP32 is off by 1.3e-5 relative).
__global__ void k_adam(float *__restrict__ p, const float *__restrict__ g, float *__restrict__ m, float *__restrict__ v,
                       int np, float lr, float b1, float b2, float omb1, float omb2, float eps, float c1, float c2)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= np) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + omb1 * gi;
    const float vi = b2 * v[i] + omb2 * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float mh = mi / c1, vh = vi / c2;
    p[i] -= lr * mh / (sqrtf(vh) + eps);
}

unsigned blocks_for(int n) { return (unsigned)((n + 255) / 256); }

}  // namespace
}  // namespace qs

struct qs_costmodel {
    hipStream_t stream = nullptr;
    int device = 0;
    float *params = nullptr, *grads = nullptr, *m = nullptr, *v = nullptr;
    float *ws = nullptr;        // activations: z1, h1, z2, h2, y, dy, dh2, dh1 (B x 128 each) + loss
    int t = 0;                  // Adam step count
};

namespace {

using namespace qs;

hipError_t forward(qs_costmodel *m, const float *X, int B, float **y_out)
{
    float *z1 = m->ws, *h1 = z1 + MAXB * NH, *z2 = h1 + MAXB * NH, *h2 = z2 + MAXB * NH, *y = h2 + MAXB * NH;
    const float *P = m->params;
    hipLaunchKernelGGL(k_linear_fwd, dim3(blocks_for(B * NH)), dim3(256), 0, m->stream, X, B, NI, P + OFF_W1, P + OFF_B1,
                       NH, z1, h1, 1);
    hipLaunchKernelGGL(k_linear_fwd, dim3(blocks_for(B * NH)), dim3(256), 0, m->stream, h1, B, NH, P + OFF_W2, P + OFF_B2,
                       NH, z2, h2, 1);
    hipLaunchKernelGGL(k_linear_fwd, dim3(blocks_for(B)), dim3(256), 0, m->stream, h2, B, NH, P + OFF_W3, P + OFF_B3, 1,
                       (float *)nullptr, y, 0);
    *y_out = y;
    return hipGetLastError();
}

// He-uniform initialisation from a seed (splitmix64 -> uniform), zero biases.
void init_params(uint64_t seed, std::vector<float> &p)
{
    p.assign(NPARAM, 0.f);
    uint64_t s = seed;
    auto next = [&]() {
        s += 0x9E3779B97F4A7C15ull;
        uint64_t z = s;
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        z ^= z >> 31;
        return (double)(z >> 11) * (1.0 / 9007199254740992.0);
    };
    auto fill = [&](int off, int fan_out, int fan_in) {
        const double bound = std::sqrt(6.0 / fan_in);
        for (int i = 0; i < fan_out * fan_in; ++i) p[off + i] = (float)((2.0 * next() - 1.0) * bound);
    };
    fill(OFF_W1, NH, NI);
    fill(OFF_W2, NH, NH);
    fill(OFF_W3, 1, NH);
}

}  // namespace

hipStream_t qs::costmodel_stream(const qs_costmodel *m) { return m->stream; }
int qs::costmodel_device(const qs_costmodel *m) { return m->device; }

extern "C" {

qs_status qs_costmodel_create(uint64_t seed, void *hip_stream, qs_costmodel **out)
{
    if (!out) { set_error("qs_costmodel_create: out is null"); return QS_EINVAL; }
    qs_costmodel *m = new qs_costmodel();
    m->stream = reinterpret_cast<hipStream_t>(hip_stream);
    (void)hipGetDevice(&m->device);
    hipError_t e = hipMalloc(&m->params, NPARAM * sizeof(float));
    if (e == hipSuccess) e = hipMalloc(&m->grads, NPARAM * sizeof(float));
    if (e == hipSuccess) e = hipMalloc(&m->m, NPARAM * sizeof(float));
    if (e == hipSuccess) e = hipMalloc(&m->v, NPARAM * sizeof(float));
    if (e == hipSuccess) e = hipMalloc(&m->ws, (size_t)(8 * MAXB * NH + 16) * sizeof(float));
    std::vector<float> p;
    init_params(seed, p);
    std::vector<float> zero(NPARAM, 0.f);
    if (e == hipSuccess) e = hipMemcpy(m->params, p.data(), NPARAM * sizeof(float), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(m->grads, zero.data(), NPARAM * sizeof(float), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(m->m, zero.data(), NPARAM * sizeof(float), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(m->v, zero.data(), NPARAM * sizeof(float), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        qs_costmodel_free(m);
        return hip_fail(e, "qs_costmodel_create");
    }
    *out = m;
    return QS_OK;
}

qs_status qs_costmodel_free(qs_costmodel *m)
{
    if (!m) return QS_OK;
    (void)hipSetDevice(m->device);
    (void)hipStreamSynchronize(m->stream);
    for (float *p : {m->params, m->grads, m->m, m->v, m->ws})
        if (p) (void)hipFree(p);
    delete m;
    return QS_OK;
}

qs_status qs_costmodel_get_params(const qs_costmodel *m, float *host_out)
{
    if (!m || !host_out) { set_error("qs_costmodel_get_params: null argument"); return QS_EINVAL; }
    hipError_t e = hipMemcpyAsync(host_out, m->params, NPARAM * sizeof(float), hipMemcpyDeviceToHost, m->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(m->stream);
    if (e != hipSuccess) return hip_fail(e, "qs_costmodel_get_params");
    return QS_OK;
}

qs_status qs_costmodel_set_params(qs_costmodel *m, const float *host_in)
{
    if (!m || !host_in) { set_error("qs_costmodel_set_params: null argument"); return QS_EINVAL; }
    hipError_t e = hipMemcpyAsync(m->params, host_in, NPARAM * sizeof(float), hipMemcpyHostToDevice, m->stream);
    if (e == hipSuccess) {
        // a new starting point: Adam starts over (step count and both moments)
        hipLaunchKernelGGL(k_zero2, dim3((NPARAM + 255) / 256), dim3(256), 0, m->stream, m->m, m->v, (int)NPARAM);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipStreamSynchronize(m->stream);
    if (e != hipSuccess) return hip_fail(e, "qs_costmodel_set_params");
    m->t = 0;
    return QS_OK;
}

qs_status qs_costmodel_get_grads(const qs_costmodel *m, float *host_out)
{
    if (!m || !host_out) { set_error("qs_costmodel_get_grads: null argument"); return QS_EINVAL; }
    hipError_t e = hipMemcpyAsync(host_out, m->grads, NPARAM * sizeof(float), hipMemcpyDeviceToHost, m->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(m->stream);
    if (e != hipSuccess) return hip_fail(e, "qs_costmodel_get_grads");
    return QS_OK;
}

qs_status qs_costmodel_predict(const qs_costmodel *m, const float *X_dev, float *y_dev, int B)
{
    if (!m || !X_dev || !y_dev || B < 1) { set_error("qs_costmodel_predict: bad arguments"); return QS_EINVAL; }
    qs_costmodel *mm = const_cast<qs_costmodel *>(m);
    for (int b0 = 0; b0 < B; b0 += MAXB) {
        const int nb = std::min(MAXB, B - b0);
        float *y = nullptr;
        hipError_t e = forward(mm, X_dev + (size_t)b0 * NI, nb, &y);
        if (e == hipSuccess) e = hipMemcpyAsync(y_dev + b0, y, nb * sizeof(float), hipMemcpyDeviceToDevice, m->stream);
        if (e != hipSuccess) return hip_fail(e, "qs_costmodel_predict");
    }
    return QS_OK;
}

qs_status qs_costmodel_train_step(qs_costmodel *m, const float *X_dev, const float *y_dev, int B, float lr,
                                  float *loss_host)
{
    if (!m || !X_dev || !y_dev || B < 1 || B > MAXB) { set_error("qs_costmodel_train_step: bad arguments (B 1..1024)"); return QS_EINVAL; }
    float *y = nullptr;
    hipError_t e = forward(m, X_dev, B, &y);
    float *z1 = m->ws, *h1 = z1 + MAXB * NH, *z2 = h1 + MAXB * NH, *h2 = z2 + MAXB * NH;
    float *dy = h2 + 2 * MAXB * NH, *dh2 = dy + MAXB * NH, *dh1 = dh2 + MAXB * NH, *loss = dh1 + MAXB * NH;
    const float *P = m->params;
    float *G = m->grads;
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_mse, dim3(1), dim3(256), 0, m->stream, y, y_dev, B, dy, loss);
        // layer 3
        hipLaunchKernelGGL(k_linear_bwd_w, dim3(blocks_for(NH + 1)), dim3(256), 0, m->stream, dy, h2, B, 1, NH,
                           G + OFF_W3, G + OFF_B3);
        hipLaunchKernelGGL(k_linear_bwd_in, dim3(blocks_for(B * NH)), dim3(256), 0, m->stream, dy, B, 1, P + OFF_W3, NH,
                           z2, dh2);
        // layer 2
        hipLaunchKernelGGL(k_linear_bwd_w, dim3(blocks_for(NH * NH + NH)), dim3(256), 0, m->stream, dh2, h1, B, NH, NH,
                           G + OFF_W2, G + OFF_B2);
        hipLaunchKernelGGL(k_linear_bwd_in, dim3(blocks_for(B * NH)), dim3(256), 0, m->stream, dh2, B, NH, P + OFF_W2, NH,
                           z1, dh1);
        // layer 1
        hipLaunchKernelGGL(k_linear_bwd_w, dim3(blocks_for(NH * NI + NH)), dim3(256), 0, m->stream, dh1, X_dev, B, NH, NI,
                           G + OFF_W1, G + OFF_B1);
        e = hipGetLastError();
    }
    if (e == hipSuccess) {
        m->t += 1;
        const double b1 = 0.9, b2 = 0.999;
        const float c1 = (float)(1.0 - std::pow(b1, m->t)), c2 = (float)(1.0 - std::pow(b2, m->t));
        hipLaunchKernelGGL(k_adam, dim3(blocks_for(NPARAM)), dim3(256), 0, m->stream, m->params, G, m->m, m->v, NPARAM, lr,
                           (float)b1, (float)b2, (float)(1.0 - b1), (float)(1.0 - b2), 1e-8f, c1, c2);
        e = hipGetLastError();
    }
    if (e == hipSuccess && loss_host) {
        e = hipMemcpyAsync(loss_host, loss, sizeof(float), hipMemcpyDeviceToHost, m->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(m->stream);
    }
    if (e != hipSuccess) return hip_fail(e, "qs_costmodel_train_step");
    return QS_OK;
}

}  // extern "C"
