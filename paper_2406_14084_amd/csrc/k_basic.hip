// k_basic.hip -- one-pass kernels: initial state, gate-by-gate application,
// probabilities and Pauli expectations.
//
// Paper: Eq. 1 (state, probabilities), Eq. 2 / Eq. 3 (gate application, the
// gate-by-gate scheme the blocked path is compared with, Sec. V-A / VI-F).
#include <algorithm>

#include "amp.h"
#include "qs_internal.h"

namespace qs {
namespace {

template <typename F>
__global__ __launch_bounds__(256) void k_init(typename AmpOf<F>::type *__restrict__ a, uint64_t N, uint64_t index)
{
    using V = typename AmpOf<F>::type;
    uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (; i < N; i += stride) {
        V z;
        z.x = (i == index) ? (F)1 : (F)0;
        z.y = (F)0;
        a[i] = z;
    }
}

// Gate matrix passed by value (k <= 3): 2 * 4^k scalars.
template <int K, typename F>
struct GateArgs {
    uint64_t off[1 << K];      // physical offset of local index c (circuit convention)
    int tsorted[K];            // target qubits ascending (for zero insertion)
    F m[2 << (2 * K)];
};

template <int K, typename F>
__device__ __forceinline__ uint64_t insert_zeros(uint64_t j, const int *ts)
{
    // ts ascending: open a zero at each target position
#pragma unroll
    for (int i = 0; i < K; ++i) {
        const uint64_t lo = j & ((1ull << ts[i]) - 1);
        j = ((j >> ts[i]) << (ts[i] + 1)) | lo;
    }
    return j;
}

// One thread per 2^K-tuple: gather, multiply by the gate matrix, scatter.
template <int K, typename F>
__global__ __launch_bounds__(256) void k_gate_val(typename AmpOf<F>::type *__restrict__ a, uint64_t ntuples,
                                                 GateArgs<K, F> g)
{
    using V = typename AmpOf<F>::type;
    constexpr int D = 1 << K;
    uint64_t j = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (; j < ntuples; j += stride) {
        const uint64_t base = insert_zeros<K, F>(j, g.tsorted);
        V in[D];
#pragma unroll
        for (int c = 0; c < D; ++c) in[c] = a[base | g.off[c]];
#pragma unroll
        for (int r = 0; r < D; ++r) {
            V acc = cmul<F, V>(g.m[2 * (r * D)], g.m[2 * (r * D) + 1], in[0]);
#pragma unroll
            for (int c = 1; c < D; ++c) cmac<F, V>(acc, g.m[2 * (r * D + c)], g.m[2 * (r * D + c) + 1], in[c]);
            a[base | g.off[r]] = acc;
        }
    }
}

// k = 4, 5: matrix in device memory (scratch), offsets by value.
template <int K>
struct GateOffs {
    uint64_t off[1 << K];
    int tsorted[K];
};

template <int K, typename F>
__global__ __launch_bounds__(256) void k_gate_ptr(typename AmpOf<F>::type *__restrict__ a, uint64_t ntuples,
                                                 GateOffs<K> g, const F *__restrict__ m)
{
    using V = typename AmpOf<F>::type;
    constexpr int D = 1 << K;
    uint64_t j = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (; j < ntuples; j += stride) {
        const uint64_t base = insert_zeros<K, F>(j, g.tsorted);
        V in[D];
#pragma unroll
        for (int c = 0; c < D; ++c) in[c] = a[base | g.off[c]];
        for (int r = 0; r < D; ++r) {
            V acc = cmul<F, V>(m[2 * (r * D)], m[2 * (r * D) + 1], in[0]);
#pragma unroll
            for (int c = 1; c < D; ++c) cmac<F, V>(acc, m[2 * (r * D + c)], m[2 * (r * D + c) + 1], in[c]);
            a[base | g.off[r]] = acc;
        }
    }
}

template <typename F>
__global__ __launch_bounds__(256) void k_probs(const typename AmpOf<F>::type *__restrict__ a, double *__restrict__ p,
                                              uint64_t N)
{
    uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (; i < N; i += stride) {
        const double x = (double)a[i].x, y = (double)a[i].y;
        p[i] = x * x + y * y;
    }
}

// Re sum_i conj(a_{i^x}) ph(i) a_i for one Pauli term per blockIdx.y;
// ph(i) = i^{#Y} (-1)^{popcount(i & z)}.  FP64 accumulation, one partial per
// workgroup (summed on the host in a fixed order).
template <typename F>
__global__ __launch_bounds__(256) void k_expect(const typename AmpOf<F>::type *__restrict__ a, uint64_t N,
                                               const qs_pauli *__restrict__ terms, double *__restrict__ partials)
{
    __shared__ double red[256 / 64];
    const qs_pauli t = terms[blockIdx.y];
    const uint64_t x = t.xmask, z = t.zmask;
    const int ny = __builtin_popcountll(x & z) & 3;
    // i^ny = (pr, pi)
    const double pr = (ny == 0) ? 1.0 : (ny == 2) ? -1.0 : 0.0;
    const double pi = (ny == 1) ? 1.0 : (ny == 3) ? -1.0 : 0.0;
    double s = 0.0;
    uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (; i < N; i += stride) {
        const uint64_t jx = i ^ x;
        const double ar = (double)a[i].x, ai = (double)a[i].y;
        const double br = (double)a[jx].x, bi = -(double)a[jx].y;
        const double sg = (__builtin_popcountll(i & z) & 1) ? -1.0 : 1.0;
        // Re( conj(a_jx) * ph * a_i ) with ph = sg * (pr + i pi)
        const double tr = sg * (pr * ar - pi * ai);
        const double ti = sg * (pr * ai + pi * ar);
        s += br * tr - bi * ti;
    }
    // wave reduction then across the 4 waves
    for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (lane == 0) red[wv] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        double tot = 0.0;
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) tot += red[w];
        partials[(uint64_t)blockIdx.y * gridDim.x + blockIdx.x] = tot;
    }
}

unsigned grid_for(uint64_t items, unsigned threads, unsigned cap)
{
    uint64_t g = (items + threads - 1) / threads;
    if (g > cap) g = cap;
    if (g == 0) g = 1;
    return (unsigned)g;
}

template <typename F>
hipError_t gate_F(qs_state *st, int k, const int *targets, const double *matrix, const void *d_matrix)
{
    using V = typename AmpOf<F>::type;
    const uint64_t ntuples = 1ull << (st->n - k);
    const unsigned grid = grid_for(ntuples, 256, 256u * 1024u);
    V *a = reinterpret_cast<V *>(st->amps);
    int ts[5];
    for (int j = 0; j < k; ++j) ts[j] = targets[j];
    std::sort(ts, ts + k);
    auto fill_off = [&](uint64_t *off) {
        for (int c = 0; c < (1 << k); ++c) {
            uint64_t o = 0;
            for (int j = 0; j < k; ++j)
                if ((c >> (k - 1 - j)) & 1) o |= 1ull << targets[j];
            off[c] = o;
        }
    };
    switch (k) {
#define QS_GATE_VAL(KK)                                                                                  \
    case KK: {                                                                                           \
        GateArgs<KK, F> g;                                                                               \
        fill_off(g.off);                                                                                 \
        for (int j = 0; j < KK; ++j) g.tsorted[j] = ts[j];                                               \
        for (int i = 0; i < (2 << (2 * KK)); ++i) g.m[i] = (F)matrix[i];                                 \
        hipLaunchKernelGGL((k_gate_val<KK, F>), dim3(grid), dim3(256), 0, st->stream, a, ntuples, g);   \
        return hipGetLastError();                                                                        \
    }
        QS_GATE_VAL(1)
        QS_GATE_VAL(2)
        QS_GATE_VAL(3)
#undef QS_GATE_VAL
#define QS_GATE_PTR(KK)                                                                                  \
    case KK: {                                                                                           \
        GateOffs<KK> g;                                                                                  \
        fill_off(g.off);                                                                                 \
        for (int j = 0; j < KK; ++j) g.tsorted[j] = ts[j];                                               \
        hipLaunchKernelGGL((k_gate_ptr<KK, F>), dim3(grid), dim3(256), 0, st->stream, a, ntuples, g,     \
                           reinterpret_cast<const F *>(d_matrix));                                       \
        return hipGetLastError();                                                                        \
    }
        QS_GATE_PTR(4)
        QS_GATE_PTR(5)
#undef QS_GATE_PTR
    default:
        return hipErrorInvalidValue;
    }
}

}  // namespace

hipError_t launch_init(qs_state *st, uint64_t index)
{
    const uint64_t N = 1ull << st->n;
    const unsigned grid = grid_for(N, 256, 256u * 1024u);
    if (st->dtype == QS_C64)
        hipLaunchKernelGGL(k_init<float>, dim3(grid), dim3(256), 0, st->stream, reinterpret_cast<c64 *>(st->amps), N, index);
    else
        hipLaunchKernelGGL(k_init<double>, dim3(grid), dim3(256), 0, st->stream, reinterpret_cast<c128 *>(st->amps), N, index);
    return hipGetLastError();
}

hipError_t launch_gate(qs_state *st, int k, const int *targets, const double *matrix, const void *d_matrix)
{
    if (st->dtype == QS_C64) return gate_F<float>(st, k, targets, matrix, d_matrix);
    return gate_F<double>(st, k, targets, matrix, d_matrix);
}

hipError_t launch_probs(qs_state *st, double *out)
{
    const uint64_t N = 1ull << st->n;
    const unsigned grid = grid_for(N, 256, 256u * 1024u);
    if (st->dtype == QS_C64)
        hipLaunchKernelGGL(k_probs<float>, dim3(grid), dim3(256), 0, st->stream, reinterpret_cast<const c64 *>(st->amps), out, N);
    else
        hipLaunchKernelGGL(k_probs<double>, dim3(grid), dim3(256), 0, st->stream, reinterpret_cast<const c128 *>(st->amps), out, N);
    return hipGetLastError();
}

int expect_partials(int n)
{
    const uint64_t N = 1ull << n;
    return (int)grid_for(N, 256, 2048);
}

hipError_t launch_expect(qs_state *st, int nterms, const qs_pauli *d_terms, double *partials, int nparts)
{
    const uint64_t N = 1ull << st->n;
    dim3 grid((unsigned)nparts, (unsigned)nterms);
    if (st->dtype == QS_C64)
        hipLaunchKernelGGL(k_expect<float>, grid, dim3(256), 0, st->stream, reinterpret_cast<const c64 *>(st->amps), N, d_terms, partials);
    else
        hipLaunchKernelGGL(k_expect<double>, grid, dim3(256), 0, st->stream, reinterpret_cast<const c128 *>(st->amps), N, d_terms, partials);
    return hipGetLastError();
}

}  // namespace qs
