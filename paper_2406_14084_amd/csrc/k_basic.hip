// k_basic.hip -- one-pass kernels: initial state, gate-by-gate application,
// probabilities and Pauli expectations.
//
// Paper: Eq. 1 (state, probabilities), Eq. 2 / Eq. 3 (gate application, the
// gate-by-gate scheme the blocked path is compared with, Sec. V-A / VI-F).
#include <algorithm>
#include <vector>

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

// Gate-by-gate kernels (one pass per gate, Eq. 2 / Eq. 3).  The host
// classifies each gate first (classify_gate): qubits on which the matrix is
// the identity unless the qubit is 1 are controls -- the pass then visits only
// the tuples with every control bit set; on the remaining K targets the
// matrix is diagonal (only the entries that differ from 1 are multiplied:
// CZ and CP touch a quarter of the state), a permutation with phases (only
// the rows that move or change are written; unit phases are pure data
// movement: CX moves half the state, SWAP half, X all of it) or dense.
// A tuple is the 2^K amplitudes base | off[c], base having zeros at every
// target and control position and ones at the controls.
constexpr int kMaxGateBits = 10;

struct TupleIndex {
    int nz;                        // targets + controls
    int zs[kMaxGateBits];          // their positions, ascending
    uint64_t cbits;                // control bits (all set in every visited tuple)
};

__device__ __forceinline__ uint64_t tuple_base(uint64_t j, const TupleIndex &t)
{
    for (int i = 0; i < t.nz; ++i) {
        const uint64_t lo = j & ((1ull << t.zs[i]) - 1);
        j = ((j >> t.zs[i]) << (t.zs[i] + 1)) | lo;
    }
    return j | t.cbits;
}

// Dense K-qubit matrix passed by value (K <= 3): 2 * 4^K scalars.
template <int K, typename F>
struct GateArgs {
    TupleIndex ti;
    uint64_t off[1 << K];      // physical offset of local index c (circuit convention)
    F m[2 << (2 * K)];
};

template <int K, typename F>
__global__ __launch_bounds__(256) void k_gate_val(typename AmpOf<F>::type *__restrict__ a, uint64_t ntuples,
                                                 GateArgs<K, F> g)
{
    using V = typename AmpOf<F>::type;
    constexpr int D = 1 << K;
    uint64_t j = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (; j < ntuples; j += stride) {
        const uint64_t base = tuple_base(j, g.ti);
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

// K = 4, 5 dense: matrix in device memory (the workspace), offsets by value.
template <int K>
struct GateOffs {
    TupleIndex ti;
    uint64_t off[1 << K];
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
        const uint64_t base = tuple_base(j, g.ti);
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

// Diagonal or permutation-with-phases on K <= 5 targets.  Only the nact
// active rows are touched: row r gets e[r] * a[base | off[src[r]]] (src[r] = r
// for a diagonal); unit = 1 when every e[r] is exactly 1 (a pure move).
struct GateSparse {
    TupleIndex ti;
    int nact;
    int unit;
    uint64_t off[32];          // off[i]: offset of active row i
    uint64_t soff[32];         // offset of its source column
    double e[64];              // its coefficient (re, im), FP64 (rounded to the state precision in the kernel)
};

template <int NMAX, typename F>
__global__ __launch_bounds__(256) void k_gate_sparse(typename AmpOf<F>::type *__restrict__ a, uint64_t ntuples,
                                                    GateSparse g)
{
    using V = typename AmpOf<F>::type;
    uint64_t j = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (; j < ntuples; j += stride) {
        const uint64_t base = tuple_base(j, g.ti);
        V in[NMAX];
        // every source is read before any row is written (a permutation may
        // write a row another row reads)
#pragma unroll
        for (int i = 0; i < NMAX; ++i)
            if (i < g.nact) in[i] = a[base | g.soff[i]];
#pragma unroll
        for (int i = 0; i < NMAX; ++i) {
            if (i < g.nact) {
                V v = in[i];
                if (!g.unit) v = cmul<F, V>((F)g.e[2 * i], (F)g.e[2 * i + 1], v);
                a[base | g.off[i]] = v;
            }
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

// Host classification of a k-qubit gate (targets t[0..k-1], t[0] = MSB of the
// local index) into controls and an active kind on the remaining targets.
struct GateClass {
    int kind = 0;                 // 0 dense, 1 diagonal, 2 permutation with phases
    int nt = 0;                   // active targets
    int tq[5];                    // their qubits, t[0] = MSB of the sub-matrix index
    uint64_t cbits = 0;           // control qubits (mask)
    std::vector<cplx> u;          // 2^nt x 2^nt sub-matrix (row-major)
};

GateClass classify_gate(int k, const int *targets, const double *matrix)
{
    const int D = 1 << k;
    auto M = [&](int r, int c) { return cplx(matrix[2 * (r * D + c)], matrix[2 * (r * D + c) + 1]); };
    // local bit of target j is k-1-j; a control bit b: rows/columns with b = 0
    // form an identity block and nothing mixes the b = 0 and b = 1 halves
    int cmask = 0;   // local bits found to be controls
    for (int b = k - 1; b >= 0; --b) {
        bool ctrl = true;
        for (int r = 0; r < D && ctrl; ++r) {
            if ((r & cmask) != cmask) continue;
            for (int c = 0; c < D && ctrl; ++c) {
                if ((c & cmask) != cmask) continue;
                const bool rb = (r >> b) & 1, cb = (c >> b) & 1;
                const cplx v = M(r, c);
                if (rb != cb) ctrl = (v == cplx(0, 0));
                else if (!rb) {
                    // b = 0 half: identity, and no mixing with other local indices
                    ctrl = (r == c) ? (v == cplx(1, 0)) : (v == cplx(0, 0));
                }
            }
        }
        // at least one active target must remain
        if (ctrl && __builtin_popcount(cmask | (1 << b)) < k) cmask |= 1 << b;
    }
    GateClass g;
    for (int j = 0; j < k; ++j) {
        const int b = k - 1 - j;
        if ((cmask >> b) & 1) g.cbits |= 1ull << targets[j];
        else g.tq[g.nt++] = targets[j];
    }
    const int d = 1 << g.nt;
    // sub-matrix on the active targets (controls fixed to 1)
    int lb[5], m = 0;      // local bit of active target i (i = 0 is the sub-matrix MSB)
    for (int j = 0; j < k; ++j)
        if (!((cmask >> (k - 1 - j)) & 1)) lb[m++] = k - 1 - j;
    auto lift = [&](int s) {
        int r = cmask;
        for (int i = 0; i < g.nt; ++i)
            if ((s >> (g.nt - 1 - i)) & 1) r |= 1 << lb[i];
        return r;
    };
    g.u.resize((size_t)d * d);
    for (int r = 0; r < d; ++r)
        for (int c = 0; c < d; ++c) g.u[(size_t)r * d + c] = M(lift(r), lift(c));
    bool diag = true, perm = true;
    for (int r = 0; r < d; ++r) {
        int nz = 0;
        for (int c = 0; c < d; ++c)
            if (g.u[(size_t)r * d + c] != cplx(0, 0)) {
                ++nz;
                if (c != r) diag = false;
            }
        if (nz != 1) perm = false;
    }
    if (perm) {
        for (int c = 0; c < d && perm; ++c) {
            int nz = 0;
            for (int r = 0; r < d; ++r) nz += g.u[(size_t)r * d + c] != cplx(0, 0);
            if (nz != 1) perm = false;
        }
    }
    g.kind = (diag && perm) ? 1 : perm ? 2 : 0;
    return g;
}

template <typename F>
hipError_t gate_F(qs_state *st, int k, const int *targets, const double *matrix)
{
    using V = typename AmpOf<F>::type;
    V *a = reinterpret_cast<V *>(st->amps);
    const GateClass g = classify_gate(k, targets, matrix);
    const int nc = __builtin_popcountll(g.cbits);
    const uint64_t ntuples = 1ull << (st->n - g.nt - nc);
    const unsigned grid = grid_for(ntuples, 256, 256u * 1024u);
    const int d = 1 << g.nt;
    TupleIndex ti;
    ti.nz = 0;
    for (int q = 0; q < st->n; ++q) {
        bool used = (g.cbits >> q) & 1;
        for (int i = 0; i < g.nt; ++i) used = used || g.tq[i] == q;
        if (used) ti.zs[ti.nz++] = q;
    }
    ti.cbits = g.cbits;
    auto offset = [&](int c) {
        uint64_t o = 0;
        for (int i = 0; i < g.nt; ++i)
            if ((c >> (g.nt - 1 - i)) & 1) o |= 1ull << g.tq[i];
        return o;
    };
    if (g.kind != 0) {
        GateSparse s;
        s.ti = ti;
        s.nact = 0;
        s.unit = 1;
        for (int r = 0; r < d; ++r) {
            int src = r;
            for (int c = 0; c < d; ++c)
                if (g.u[(size_t)r * d + c] != cplx(0, 0)) src = c;
            const cplx e = g.u[(size_t)r * d + src];
            if (src == r && e == cplx(1, 0)) continue;     // row unchanged
            s.off[s.nact] = offset(r);
            s.soff[s.nact] = offset(src);
            s.e[2 * s.nact] = e.real();
            s.e[2 * s.nact + 1] = e.imag();
            if (e != cplx(1, 0)) s.unit = 0;
            ++s.nact;
        }
        if (s.nact == 0) return hipSuccess;               // the identity
        if (s.nact <= 1) hipLaunchKernelGGL((k_gate_sparse<1, F>), dim3(grid), dim3(256), 0, st->stream, a, ntuples, s);
        else if (s.nact <= 2) hipLaunchKernelGGL((k_gate_sparse<2, F>), dim3(grid), dim3(256), 0, st->stream, a, ntuples, s);
        else if (s.nact <= 4) hipLaunchKernelGGL((k_gate_sparse<4, F>), dim3(grid), dim3(256), 0, st->stream, a, ntuples, s);
        else if (s.nact <= 8) hipLaunchKernelGGL((k_gate_sparse<8, F>), dim3(grid), dim3(256), 0, st->stream, a, ntuples, s);
        else if (s.nact <= 16) hipLaunchKernelGGL((k_gate_sparse<16, F>), dim3(grid), dim3(256), 0, st->stream, a, ntuples, s);
        else hipLaunchKernelGGL((k_gate_sparse<32, F>), dim3(grid), dim3(256), 0, st->stream, a, ntuples, s);
        return hipGetLastError();
    }
    switch (g.nt) {
#define QS_GATE_VAL(KK)                                                                                  \
    case KK: {                                                                                           \
        GateArgs<KK, F> ga;                                                                              \
        ga.ti = ti;                                                                                      \
        for (int c = 0; c < (1 << KK); ++c) ga.off[c] = offset(c);                                       \
        for (int i = 0; i < (1 << (2 * KK)); ++i) {                                                      \
            ga.m[2 * i] = (F)g.u[i].real();                                                              \
            ga.m[2 * i + 1] = (F)g.u[i].imag();                                                          \
        }                                                                                                \
        hipLaunchKernelGGL((k_gate_val<KK, F>), dim3(grid), dim3(256), 0, st->stream, a, ntuples, ga);  \
        return hipGetLastError();                                                                        \
    }
        QS_GATE_VAL(1)
        QS_GATE_VAL(2)
        QS_GATE_VAL(3)
#undef QS_GATE_VAL
    default:
        break;
    }
    // 4-5 active targets: the sub-matrix goes through the workspace, in stream order
    const size_t cnt = (size_t)2 * d * d;
    std::vector<F> mw(cnt);
    for (size_t i = 0; i < (size_t)d * d; ++i) {
        mw[2 * i] = (F)g.u[i].real();
        mw[2 * i + 1] = (F)g.u[i].imag();
    }
    if (cnt * sizeof(F) > st->scratch_bytes) return hipErrorInvalidValue;
    hipError_t e = hipMemcpyAsync(st->d_scratch, mw.data(), cnt * sizeof(F), hipMemcpyHostToDevice, st->stream);
    // the host buffer must outlive the copy
    if (e == hipSuccess) e = hipStreamSynchronize(st->stream);
    if (e != hipSuccess) return e;
    const F *dm = reinterpret_cast<const F *>(st->d_scratch);
    switch (g.nt) {
#define QS_GATE_PTR(KK)                                                                                  \
    case KK: {                                                                                           \
        GateOffs<KK> go;                                                                                 \
        go.ti = ti;                                                                                      \
        for (int c = 0; c < (1 << KK); ++c) go.off[c] = offset(c);                                       \
        hipLaunchKernelGGL((k_gate_ptr<KK, F>), dim3(grid), dim3(256), 0, st->stream, a, ntuples, go, dm); \
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

hipError_t launch_gate(qs_state *st, int k, const int *targets, const double *matrix)
{
    if (st->dtype == QS_C64) return gate_F<float>(st, k, targets, matrix);
    return gate_F<double>(st, k, targets, matrix);
}

int gate_kind(int k, const int *targets, const double *matrix, uint64_t *cbits, int *nt)
{
    const GateClass g = classify_gate(k, targets, matrix);
    if (cbits) *cbits = g.cbits;
    if (nt) *nt = g.nt;
    return g.kind;
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
