// k_qaoa.hip -- many small QAOA MaxCut circuits of uneven size in one
// persistent launch.
//
// Circuit per instance (QAOA, named among the paper's benchmark circuits,
// Sec. VI-A Table II): |+>^n, then for each of p layers the cost layer
// a_z <- exp(-i gamma C(z)) a_z with C(z) = number of cut edges, and RX(2 beta)
// on every qubit; output <C> = sum_z |a_z|^2 C(z) accumulated in FP64.
//
// gfx950 design:
//   - one persistent kernel pops tasks from an atomic queue; every workgroup
//     leaves when the queue is empty;
//   - an instance of at most CB qubits is one task: its whole state lives in
//     LDS (2^CB amplitudes), C(z) is tabulated once in LDS and reused by every
//     layer and by the final reduction (CB, the launch shape and the chunks
//     per task are chosen by timing them on the device: qs_batch_autotune);
//   - a larger instance keeps its state in a workspace in HBM and is split
//     into chunk tasks of 2^CB amplitudes per pass (two passes per layer: the
//     low CB qubits, then the remaining high ones with a few low ones); a pass
//     waits (bounded spin) for the instance's previous pass through a per-
//     instance completion counter, with agent-scope release/acquire fences;
//   - tasks are queued so that a task only ever waits for tasks queued before
//     it, which running workgroups have already taken: no deadlock.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <vector>

#include "amp.h"
#include "qs_internal.h"

namespace qs {
namespace {

struct QInst {
    int n, nedges, p, large;
    int edge_off;      // into the edge array (pairs)
    int tab_off;       // into the per-instance table (scalars): per layer (nedges+1) phases (cos, -sin) then (cos b, sin b)
    long long work_off;  // amplitude offset of the state in the workspace (large only)
    int res;           // output index
    int pad;
    long long cz_off;  // byte offset of the instance's C(z) values in the cut workspace (large only)
};

struct QTask {
    int inst, pass, chunk, count;   // large instances: chunks [chunk, chunk + count) of one pass
};

constexpr unsigned kSpinLimit = 1u << 24;   // ~1 s of polling before giving up (error flag)
// chunks of one pass per batched task (autotuned): each task ends with one
// agent-scope release, which writes back the XCD's L2, so fewer, larger tasks
// cost fewer write-backs but leave fewer tasks to spread over the device
constexpr int kGroups[] = {2, 8, 32, 128};
constexpr int kNumGroups = 4;
constexpr int kDefaultGroup = 1;
// LDS chunk sizes (qubits) the autotuner tries, per dtype: the larger keeps more
// instances whole in LDS, the smaller lets twice the workgroups share a CU (an
// instance above the smaller size keeps its state in the workspace under it)
constexpr int kNumCB = 2;
constexpr int kDefaultCB = 1;
constexpr int kCB64[kNumCB] = {12, 13}, kCB128[kNumCB] = {11, 12};

template <typename F, typename V>
__device__ __forceinline__ void rx_pair(V &a0, V &a1, F c, F s)
{
    // RX(2b) = [[c, -i s], [-i s, c]], c = cos b, s = sin b
    const V x = a0, y = a1;
    a0.x = qfma(c, x.x, s * y.y);
    a0.y = qfma(c, x.y, -s * y.x);
    a1.x = qfma(c, y.x, s * x.y);
    a1.y = qfma(c, y.y, -s * x.x);
}

// C(z) = number of edges (u, v) with bit u of z != bit v.  The edge list is
// uniform across the workgroup: read through the constant address space, so
// the endpoints come in by scalar loads.
using CInt2 = __attribute__((address_space(4))) int2;
__device__ __forceinline__ int cut_value(uint64_t z, const CInt2 *e, int ne)
{
    int c = 0;
    if ((z >> 32) == 0) {
        const uint32_t z32 = (uint32_t)z;
#pragma unroll 4
        for (int i = 0; i < ne; ++i) c += (int)(((z32 >> e[i].x) ^ (z32 >> e[i].y)) & 1u);
    } else {
#pragma unroll 4
        for (int i = 0; i < ne; ++i) c += (int)(((z >> e[i].x) ^ (z >> e[i].y)) & 1ull);
    }
    return c;
}

// LDS slot of local index l: one pad slot after every 32 amplitudes.
__device__ __forceinline__ int PAD(int l) { return l + (l >> 5); }

// RX(2b) on G qubits q0..q0+G-1 of the LDS state at once: each thread loads
// the 2^G amplitudes of one group into registers, applies the G rotations
// there and writes them back -- one LDS round trip and one barrier per G
// qubits instead of per qubit.
template <int G, typename F, typename V, int THREADS>
__device__ __forceinline__ void rx_group(V *st, int na, int q0, F c, F s, int tid)
{
    for (int bi = tid; bi < (na >> G); bi += THREADS) {
        const int base = ((bi >> q0) << (q0 + G)) | (bi & ((1 << q0) - 1));
        V a[1 << G];
#pragma unroll
        for (int m = 0; m < (1 << G); ++m) a[m] = st[PAD(base | (m << q0))];
#pragma unroll
        for (int j = 0; j < G; ++j)
#pragma unroll
            for (int m = 0; m < (1 << G); ++m)
                if (!((m >> j) & 1)) rx_pair<F, V>(a[m], a[m | (1 << j)], c, s);
#pragma unroll
        for (int m = 0; m < (1 << G); ++m) st[PAD(base | (m << q0))] = a[m];
    }
}

// RX(2b) on qubits qlo..qhi-1 of the LDS state (na amplitudes), up to five
// at a time (four for complex128 or 512-thread workgroups, to bound registers).
template <typename F, typename V, int THREADS>
__device__ __forceinline__ void rx_qubits(V *st, int na, int qlo, int qhi, F c, F s, int tid)
{
    constexpr int GMAX = (sizeof(F) == 8 || THREADS == 512) ? 4 : 5;
    for (int q0 = qlo; q0 < qhi;) {
        const int g = min(GMAX, qhi - q0);
        __syncthreads();
        switch (g) {
        case 5:
            if constexpr (GMAX >= 5) rx_group<5, F, V, THREADS>(st, na, q0, c, s, tid);
            break;
        case 4: rx_group<4, F, V, THREADS>(st, na, q0, c, s, tid); break;
        case 3: rx_group<3, F, V, THREADS>(st, na, q0, c, s, tid); break;
        case 2: rx_group<2, F, V, THREADS>(st, na, q0, c, s, tid); break;
        default: rx_group<1, F, V, THREADS>(st, na, q0, c, s, tid); break;
        }
        q0 += g;
    }
}

// Global amplitude index of local index l in chunk j of a pass.
__device__ __forceinline__ uint64_t pass_index(uint32_t l, uint64_t j, int n, int CB, bool second)
{
    if (!second) return (j << CB) | l;
    const int m = n - CB;               // high qubits CB..n-1 live in local bits CB-m..CB-1
    const uint32_t lowmask = (1u << (CB - m)) - 1u;
    return (uint64_t)(l & lowmask) | (j << (CB - m)) | ((uint64_t)(l >> (CB - m)) << CB);
}

template <int THREADS, int CB, typename F>
__global__ __launch_bounds__(THREADS) void k_qaoa(const QInst *__restrict__ inst, const QTask *__restrict__ tasks,
                                                  int task_begin, int ntasks, const int2 *__restrict__ edges,
                                                  const F *__restrict__ tab, typename AmpOf<F>::type *__restrict__ work,
                                                  unsigned *__restrict__ next, unsigned *__restrict__ done,
                                                  unsigned *__restrict__ err, double *__restrict__ res,
                                                  unsigned char *__restrict__ czw)
{
    using V = typename AmpOf<F>::type;
    constexpr int NA = 1 << CB;
    // the chunk in LDS, one pad slot per 32 amplitudes (PAD) so that groups of
    // register-resident qubits read with a lane stride of 33 slots
    __shared__ V st[NA + NA / 32];
    __shared__ unsigned char cz[NA];
    __shared__ double red[THREADS / 64];
    __shared__ int s_task;
    const int tid = threadIdx.x;

    for (;;) {
        if (tid == 0) s_task = (int)atomicAdd(next, 1u);
        __syncthreads();
        const int t = s_task;
        __syncthreads();
        if (t >= ntasks) break;
        const QTask tk = tasks[task_begin + t];
        const QInst I = inst[tk.inst];
        const int eoff = __builtin_amdgcn_readfirstlane(I.edge_off);
        const CInt2 *se = (const CInt2 *)(uintptr_t)(edges + eoff);
        const F *T = tab + I.tab_off;
        const int layer_scalars = 2 * (I.nedges + 1) + 2;

        if (!I.large) {
            // ---- whole instance in LDS
            const int na = 1 << I.n;
            __syncthreads();
            const F amp0 = (F)(1.0 / sqrt((double)na));
            for (int l = tid; l < na; l += THREADS) {
                st[PAD(l)].x = amp0;
                st[PAD(l)].y = (F)0;
                cz[l] = (unsigned char)cut_value((uint64_t)l, se, I.nedges);
            }
            __syncthreads();
            for (int layer = 0; layer < I.p; ++layer) {
                const F *L = T + layer * layer_scalars;
                for (int l = tid; l < na; l += THREADS) {
                    const int c = cz[l];
                    st[PAD(l)] = cmul<F, V>(L[2 * c], L[2 * c + 1], st[PAD(l)]);
                }
                const F cb = L[2 * (I.nedges + 1)], sb = L[2 * (I.nedges + 1) + 1];
                rx_qubits<F, V, THREADS>(st, na, 0, I.n, cb, sb, tid);
                __syncthreads();
            }
            double acc = 0.0;
            for (int l = tid; l < na; l += THREADS) {
                const double x = (double)st[PAD(l)].x, y = (double)st[PAD(l)].y;
                acc += (x * x + y * y) * (double)cz[l];
            }
            for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off, 64);
            if ((tid & 63) == 0) red[tid >> 6] = acc;
            __syncthreads();
            if (tid == 0) {
                double s = 0.0;
                for (int w = 0; w < THREADS / 64; ++w) s += red[w];
                res[I.res] = s;
            }
            __syncthreads();
            continue;
        }

        // ---- one chunk of a large instance, one pass
        const int nch = 1 << (I.n - CB);
        const bool second = (tk.pass & 1) != 0;
        const int layer = tk.pass >> 1;
        const bool first_pass = (tk.pass == 0);
        const bool last_pass = (tk.pass == 2 * I.p - 1);
        if (tk.pass > 0 && tid == 0) {
            const unsigned need = (unsigned)tk.pass * (unsigned)nch;
            unsigned spins = 0;
            while (__hip_atomic_load(&done[tk.inst], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < need) {
                __builtin_amdgcn_s_sleep(2);
                if (++spins > kSpinLimit) {
                    atomicOr(err, 1u);
                    break;
                }
            }
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        }
        __syncthreads();
        V *g = work + I.work_off;
        const F amp0 = (F)(1.0 / sqrt(ldexp(1.0, I.n)));
        const F *L = T + layer * layer_scalars;
        const F cb = L[2 * (I.nedges + 1)], sb = L[2 * (I.nedges + 1) + 1];
        const int qlo = second ? CB - (I.n - CB) : 0, qhi = CB;
        const int cnt = max(1, tk.count);
        double acc = 0.0;                  // last pass: this thread's part of <C> over the task's chunks
        for (int chunk = tk.chunk; chunk < tk.chunk + cnt; ++chunk) {
            for (int l = tid; l < NA; l += THREADS) {
                const uint64_t z = pass_index((uint32_t)l, (uint64_t)chunk, I.n, CB, second);
                if (first_pass) {
                    st[PAD(l)].x = amp0;
                    st[PAD(l)].y = (F)0;
                } else {
                    st[PAD(l)] = g[z];
                }
                if (first_pass) {
                    // C(z) once per instance; later passes read it back
                    const unsigned char cv = (unsigned char)cut_value(z, se, I.nedges);
                    cz[l] = cv;
                    czw[I.cz_off + (long long)z] = cv;
                } else if (!second || last_pass) {
                    cz[l] = czw[I.cz_off + (long long)z];
                }
            }
            __syncthreads();
            if (!second) {
                for (int l = tid; l < NA; l += THREADS) {
                    const int c = cz[l];
                    st[PAD(l)] = cmul<F, V>(L[2 * c], L[2 * c + 1], st[PAD(l)]);
                }
            }
            rx_qubits<F, V, THREADS>(st, NA, qlo, qhi, cb, sb, tid);
            __syncthreads();
            if (last_pass) {
                for (int l = tid; l < NA; l += THREADS) {
                    const double x = (double)st[PAD(l)].x, y = (double)st[PAD(l)].y;
                    acc += (x * x + y * y) * (double)cz[l];
                }
            } else {
                for (int l = tid; l < NA; l += THREADS) {
                    const uint64_t z = pass_index((uint32_t)l, (uint64_t)chunk, I.n, CB, second);
                    g[z] = st[PAD(l)];
                }
            }
            __syncthreads();               // st and cz are refilled by the next chunk
        }
        if (last_pass) {
            for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off, 64);
            if ((tid & 63) == 0) red[tid >> 6] = acc;
            __syncthreads();
            if (tid == 0) {
                double s = 0.0;
                for (int w = 0; w < THREADS / 64; ++w) s += red[w];
                atomicAdd(&res[I.res], s);
            }
        } else {
            // make the task's chunks visible to whichever workgroups run the next pass
            // (one release per task: on this device it writes back the XCD's L2)
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        }
        __syncthreads();
        if (tid == 0) atomicAdd(&done[tk.inst], (unsigned)cnt);
        __syncthreads();
    }
}

// Zero the queue counter(s), the completion counters, the error flag and the
// results (a kernel rather than a memset, so the launch can sit in a graph).
__global__ void k_qaoa_reset(unsigned *ctr, int nctr, double *res, int nres)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < nctr) ctr[i] = 0u;
    if (i < nres) res[i] = 0.0;
}

}  // namespace
}  // namespace qs

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
struct qs_batch {
    int count = 0;
    qs_dtype dtype = QS_C64;
    hipStream_t stream = nullptr;
    int device = 0;
    // per LDS chunk size (kNumCB of them): descriptors (which instances are "large" and
    // where their states sit depends on it), the batched queues and the sequential ones
    void *d_inst[qs::kNumCB] = {nullptr}, *d_tasks[qs::kNumCB] = {nullptr}, *d_seq_tasks[qs::kNumCB] = {nullptr};
    void *d_edges = nullptr, *d_tab = nullptr;
    void *d_work = nullptr, *d_ctr = nullptr;
    void *d_czw = nullptr;   // C(z) bytes of the large instances
    bool own_work = true;    // d_work / d_czw allocated by the batch (no caller workspace)
    int ntasks = 0;
    std::vector<int> seq_begin[qs::kNumCB], seq_count[qs::kNumCB];   // per instance: its tasks in d_seq_tasks
    int nctr = 0;                            // [0] next, [1] err, [2..2+count) done, then one "next" per sequential launch
    int threads = 256;                       // autotuned
    int grid_per_cu = 2;                     // autotuned
    int group = qs::kDefaultGroup;           // autotuned: index into the chunk groupings
    int cbi = qs::kDefaultCB;               // autotuned: index into the LDS chunk sizes
    int grp_begin[qs::kNumCB][qs::kNumGroups] = {{0}}, grp_count[qs::kNumCB][qs::kNumGroups] = {{0}};
    int cus = 256;
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
    double *graph_out = nullptr;
    // graphs are captured and replayed on a stream of the batch's own (the
    // caller's stream may be the legacy default stream, which cannot be
    // captured), ordered against the caller's stream with events
    hipStream_t gstream = nullptr;
    hipEvent_t ev_in = nullptr, ev_out = nullptr;
};

namespace {

int chunk_bits(qs_dtype dtype, int cbi) { return dtype == QS_C64 ? qs::kCB64[cbi] : qs::kCB128[cbi]; }

template <int CB, typename F>
hipError_t launch_qaoa_cb(qs_batch *b, int cbi, const void *tasks, int begin, int ntasks, unsigned *next, double *out,
                          int threads, int grid)
{
    using namespace qs;
    using V = typename AmpOf<F>::type;
    unsigned *ctr = reinterpret_cast<unsigned *>(b->d_ctr);
    const QInst *I = reinterpret_cast<const QInst *>(b->d_inst[cbi]);
    const QTask *T = reinterpret_cast<const QTask *>(tasks);
    const int2 *E = reinterpret_cast<const int2 *>(b->d_edges);
    const F *tab = reinterpret_cast<const F *>(b->d_tab);
    V *work = reinterpret_cast<V *>(b->d_work);
    unsigned char *czw = reinterpret_cast<unsigned char *>(b->d_czw);
    if (threads == 512)
        hipLaunchKernelGGL((k_qaoa<512, CB, F>), dim3(grid), dim3(512), 0, b->stream, I, T, begin, ntasks, E, tab, work,
                           next, ctr + 2, ctr + 1, out, czw);
    else
        hipLaunchKernelGGL((k_qaoa<256, CB, F>), dim3(grid), dim3(256), 0, b->stream, I, T, begin, ntasks, E, tab, work,
                           next, ctr + 2, ctr + 1, out, czw);
    return hipGetLastError();
}

template <typename F>
hipError_t launch_qaoa(qs_batch *b, int cbi, bool seq, int begin, int ntasks, unsigned *next, double *out, int threads,
                       int grid)
{
    using namespace qs;
    const void *tasks = seq ? b->d_seq_tasks[cbi] : b->d_tasks[cbi];
    constexpr bool c64 = sizeof(F) == 4;
    if (cbi == 0)
        return launch_qaoa_cb<c64 ? kCB64[0] : kCB128[0], F>(b, 0, tasks, begin, ntasks, next, out, threads, grid);
    return launch_qaoa_cb<c64 ? kCB64[1] : kCB128[1], F>(b, 1, tasks, begin, ntasks, next, out, threads, grid);
}

hipError_t run_batch(qs_batch *b, double *out, int threads, int grid_per_cu, int group, int cbi)
{
    using namespace qs;
    unsigned *ctr = reinterpret_cast<unsigned *>(b->d_ctr);
    const int nz = std::max(2 + b->count, b->count);
    hipLaunchKernelGGL(k_qaoa_reset, dim3((nz + 255) / 256), dim3(256), 0, b->stream, ctr, 2 + b->count, out, b->count);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int nt = b->grp_count[cbi][group], t0 = b->grp_begin[cbi][group];
    const int grid = std::max(1, std::min(nt, b->cus * grid_per_cu));
    if (b->dtype == QS_C64) return launch_qaoa<float>(b, cbi, false, t0, nt, ctr, out, threads, grid);
    return launch_qaoa<double>(b, cbi, false, t0, nt, ctr, out, threads, grid);
}

}  // namespace

extern "C" {

}  // extern "C"

namespace {

qs_status check_instances(int count, const qs_qaoa_instance *inst, qs_dtype dtype, const char *fn)
{
    using namespace qs;
    if (count < 1 || !inst) { set_error(std::string(fn) + ": bad arguments"); return QS_EINVAL; }
    if (dtype != QS_C64 && dtype != QS_C128) { set_error(std::string(fn) + ": bad dtype"); return QS_EINVAL; }
    const int CB = chunk_bits(dtype, 0);      // the smallest chunk size decides the two-pass limit
    for (int i = 0; i < count; ++i) {
        const qs_qaoa_instance &q = inst[i];
        if (q.n < 2 || q.n > 20 || q.nedges < 0 || q.nedges > 64 || q.p < 1 || q.p > 64 || (q.nedges && !q.edges) ||
            !q.gammas || !q.betas) {
            set_error(std::string(fn) + ": instance " + std::to_string(i) + " out of range (n 2..20, edges <= 64, p 1..64)");
            return QS_EINVAL;
        }
        for (int e = 0; e < 2 * q.nedges; ++e)
            if (q.edges[e] < 0 || q.edges[e] >= q.n) { set_error(std::string(fn) + ": bad edge"); return QS_EINVAL; }
        if (q.n > CB && q.n - CB > CB) { set_error(std::string(fn) + ": instance too large"); return QS_EINVAL; }
    }
    return QS_OK;
}

// amplitudes of the instances that keep their state outside LDS under the chunk
// size cbi (the smallest size, index 0, needs the most)
long long work_amplitudes(int count, const qs_qaoa_instance *inst, qs_dtype dtype, int cbi = 0)
{
    const int CB = chunk_bits(dtype, cbi);
    long long work = 0;
    for (int i = 0; i < count; ++i)
        if (inst[i].n > CB) work += 1ll << inst[i].n;
    return work;
}

// workspace layout: states (work amplitudes), then one cut-value byte per amplitude
size_t work_bytes(long long work, qs_dtype dtype, size_t *cz_off)
{
    const size_t ab = dtype == QS_C64 ? 8 : 16;
    const size_t states = ((size_t)work * ab + 255) & ~(size_t)255;
    *cz_off = states;
    return work ? states + (((size_t)work + 255) & ~(size_t)255) : 0;
}

}  // namespace

extern "C" {

qs_status qs_batch_qaoa_workspace_size(int count, const qs_qaoa_instance *inst, qs_dtype dtype, size_t *bytes)
{
    using namespace qs;
    if (!bytes) { set_error("qs_batch_qaoa_workspace_size: null output"); return QS_EINVAL; }
    qs_status rc = check_instances(count, inst, dtype, "qs_batch_qaoa_workspace_size");
    if (rc) return rc;
    size_t cz = 0;
    *bytes = work_bytes(work_amplitudes(count, inst, dtype), dtype, &cz);
    return QS_OK;
}

qs_status qs_batch_qaoa_create(int count, const qs_qaoa_instance *inst, qs_dtype dtype, void *hip_stream,
                               void *workspace, size_t ws_bytes, qs_batch **out)
{
    using namespace qs;
    if (!out) { set_error("qs_batch_qaoa_create: bad arguments"); return QS_EINVAL; }
    qs_status rc0 = check_instances(count, inst, dtype, "qs_batch_qaoa_create");
    if (rc0) return rc0;
    const size_t abytes = dtype == QS_C64 ? 8 : 16;
    size_t cz_off = 0;
    const size_t need = work_bytes(work_amplitudes(count, inst, dtype), dtype, &cz_off);
    if (workspace) {
        hipPointerAttribute_t attr;
        int cur = -1;
        (void)hipGetDevice(&cur);
        if (ws_bytes < need || ((uintptr_t)workspace & 255) != 0 || hipPointerGetAttributes(&attr, workspace) != hipSuccess ||
            attr.type != hipMemoryTypeDevice || attr.device != cur) {
            (void)hipGetLastError();
            set_error("qs_batch_qaoa_create: workspace must be 256-byte aligned device memory of the current device, at "
                      "least " + std::to_string(need) + " bytes");
            return QS_EINVAL;
        }
    }
    qs_batch *b = new qs_batch();
    b->count = count;
    b->dtype = dtype;
    b->stream = reinterpret_cast<hipStream_t>(hip_stream);
    (void)hipGetDevice(&b->device);
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, b->device) == hipSuccess && prop.multiProcessorCount > 0) b->cus = prop.multiProcessorCount;

    // edges and tables (phase table per layer computed in FP64, rounded once)
    std::vector<int> E;
    std::vector<double> tab;
    std::vector<int> edge_off(count), tab_off(count);
    for (int i = 0; i < count; ++i) {
        const qs_qaoa_instance &q = inst[i];
        edge_off[i] = (int)(E.size() / 2);
        for (int e = 0; e < 2 * q.nedges; ++e) E.push_back(q.edges[e]);
        tab_off[i] = (int)tab.size();
        for (int l = 0; l < q.p; ++l) {
            for (int c = 0; c <= q.nedges; ++c) {
                tab.push_back(std::cos(q.gammas[l] * c));
                tab.push_back(-std::sin(q.gammas[l] * c));
            }
            tab.push_back(std::cos(q.betas[l]));
            tab.push_back(std::sin(q.betas[l]));
        }
    }
    qs_status rc = QS_OK;
    auto alloc = [&](void **p, size_t bytes, const void *src, const char *what) {
        if (rc) return;
        hipError_t e = hipMalloc(p, std::max<size_t>(bytes, 16));
        if (e == hipSuccess && src && bytes) e = hipMemcpy(*p, src, bytes, hipMemcpyHostToDevice);
        if (e != hipSuccess) rc = hip_fail(e, what);
    };
    // per LDS chunk size: descriptors, the batched queues, the sequential queues
    for (int cbi = 0; cbi < kNumCB; ++cbi) {
        const int CB = chunk_bits(dtype, cbi);
        std::vector<QInst> I(count);
        long long work = 0;
        for (int i = 0; i < count; ++i) {
            const qs_qaoa_instance &q = inst[i];
            QInst &d = I[i];
            d.n = q.n;
            d.nedges = q.nedges;
            d.p = q.p;
            d.large = q.n > CB ? 1 : 0;
            d.edge_off = edge_off[i];
            d.tab_off = tab_off[i];
            d.work_off = d.large ? work : 0;
            d.cz_off = d.large ? work : 0;        // one byte per amplitude, same layout as the states
            if (d.large) work += 1ll << q.n;
            d.res = i;
            d.pad = 0;
        }
        // queue: passes of the large instances interleaved, independent small
        // instances (largest first) spread between the passes
        std::vector<int> large, small;
        for (int i = 0; i < count; ++i) (I[i].large ? large : small).push_back(i);
        auto by_n = [&](int a, int c) { return I[a].n > I[c].n || (I[a].n == I[c].n && a < c); };
        std::sort(large.begin(), large.end(), by_n);
        std::sort(small.begin(), small.end(), by_n);
        int maxpass = 0;
        for (int i : large) maxpass = std::max(maxpass, 2 * I[i].p);
        // one queue per chunk grouping, back to back
        std::vector<QTask> tasks;
        for (int gi = 0; gi < kNumGroups; ++gi) {
            b->grp_begin[cbi][gi] = (int)tasks.size();
            size_t si = 0;
            for (int st = 0; st < maxpass; ++st) {
                for (int i : large) {
                    if (st >= 2 * I[i].p) continue;
                    const int nch = 1 << (I[i].n - CB), grp = std::min(kGroups[gi], nch);
                    for (int j = 0; j < nch; j += grp) tasks.push_back({i, st, j, grp});
                }
                const size_t take = (small.size() * (size_t)(st + 1)) / (size_t)maxpass;
                for (; si < take; ++si) tasks.push_back({small[si], 0, 0, 0});
            }
            for (; si < small.size(); ++si) tasks.push_back({small[si], 0, 0, 0});
            b->grp_count[cbi][gi] = (int)tasks.size() - b->grp_begin[cbi][gi];
        }
        // per-instance task lists for the sequential reference
        std::vector<QTask> seq;
        b->seq_begin[cbi].resize(count);
        b->seq_count[cbi].resize(count);
        for (int i = 0; i < count; ++i) {
            b->seq_begin[cbi][i] = (int)seq.size();
            if (I[i].large) {
                for (int st = 0; st < 2 * I[i].p; ++st)
                    for (int j = 0; j < (1 << (I[i].n - CB)); ++j) seq.push_back({i, st, j, 1});
            } else {
                seq.push_back({i, 0, 0, 0});
            }
            b->seq_count[cbi][i] = (int)seq.size() - b->seq_begin[cbi][i];
        }
        alloc(&b->d_inst[cbi], I.size() * sizeof(QInst), I.data(), "qs_batch_qaoa_create: descriptors");
        alloc(&b->d_tasks[cbi], tasks.size() * sizeof(QTask), tasks.data(), "qs_batch_qaoa_create: tasks");
        alloc(&b->d_seq_tasks[cbi], seq.size() * sizeof(QTask), seq.data(), "qs_batch_qaoa_create: tasks");
    }
    b->ntasks = b->grp_count[b->cbi][kDefaultGroup];
    alloc(&b->d_edges, E.size() * sizeof(int), E.data(), "qs_batch_qaoa_create: edges");
    if (dtype == QS_C64) {
        std::vector<float> t32(tab.begin(), tab.end());
        alloc(&b->d_tab, t32.size() * sizeof(float), t32.data(), "qs_batch_qaoa_create: tables");
    } else {
        alloc(&b->d_tab, tab.size() * sizeof(double), tab.data(), "qs_batch_qaoa_create: tables");
    }
    // the workspace is laid out for the smallest chunk size (the most large
    // instances); a larger one uses a prefix of the same states and cut bytes
    const long long work = work_amplitudes(count, inst, dtype);
    if (workspace) {
        b->own_work = false;
        b->d_work = need ? workspace : nullptr;
        b->d_czw = need ? reinterpret_cast<char *>(workspace) + cz_off : nullptr;
    } else {
        alloc(&b->d_work, (size_t)work * abytes, nullptr, "qs_batch_qaoa_create: workspace");
        alloc(&b->d_czw, (size_t)std::max<long long>(work, 1), nullptr, "qs_batch_qaoa_create: cut workspace");
    }
    b->nctr = 2 + count + count;
    alloc(&b->d_ctr, (size_t)b->nctr * sizeof(unsigned), nullptr, "qs_batch_qaoa_create: counters");
    if (rc) {
        qs_batch_free(b);
        return rc;
    }
    *out = b;
    return QS_OK;
}

qs_status qs_batch_qaoa_run(qs_batch *b, double *out_dev, int use_graph)
{
    using namespace qs;
    if (!b || !out_dev) { set_error("qs_batch_qaoa_run: null argument"); return QS_EINVAL; }
    (void)hipSetDevice(b->device);
    if (!use_graph) {
        hipError_t e = run_batch(b, out_dev, b->threads, b->grid_per_cu, b->group, b->cbi);
        if (e != hipSuccess) return hip_fail(e, "qs_batch_qaoa_run");
        return QS_OK;
    }
    if (!b->gstream) {
        hipError_t e = hipStreamCreateWithFlags(&b->gstream, hipStreamNonBlocking);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&b->ev_in, hipEventDisableTiming);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&b->ev_out, hipEventDisableTiming);
        if (e != hipSuccess) return hip_fail(e, "qs_batch_qaoa_run: graph stream");
    }
    if (!b->gexec || b->graph_out != out_dev) {
        if (b->gexec) { (void)hipGraphExecDestroy(b->gexec); b->gexec = nullptr; }
        if (b->graph) { (void)hipGraphDestroy(b->graph); b->graph = nullptr; }
        hipStream_t user = b->stream;
        b->stream = b->gstream;
        hipError_t e = hipStreamBeginCapture(b->gstream, hipStreamCaptureModeThreadLocal);
        hipError_t e2 = (e == hipSuccess) ? run_batch(b, out_dev, b->threads, b->grid_per_cu, b->group, b->cbi) : hipSuccess;
        hipError_t e3 = (e == hipSuccess) ? hipStreamEndCapture(b->gstream, &b->graph) : hipSuccess;
        b->stream = user;
        if (e != hipSuccess) return hip_fail(e, "qs_batch_qaoa_run: begin capture");
        if (e2 != hipSuccess) return hip_fail(e2, "qs_batch_qaoa_run: capture");
        if (e3 != hipSuccess) return hip_fail(e3, "qs_batch_qaoa_run: end capture");
        e = hipGraphInstantiate(&b->gexec, b->graph, nullptr, nullptr, 0);
        if (e != hipSuccess) return hip_fail(e, "qs_batch_qaoa_run: instantiate");
        b->graph_out = out_dev;
    }
    hipError_t e = hipEventRecord(b->ev_in, b->stream);
    if (e == hipSuccess) e = hipStreamWaitEvent(b->gstream, b->ev_in, 0);
    if (e == hipSuccess) e = hipGraphLaunch(b->gexec, b->gstream);
    if (e == hipSuccess) e = hipEventRecord(b->ev_out, b->gstream);
    if (e == hipSuccess) e = hipStreamWaitEvent(b->stream, b->ev_out, 0);
    if (e != hipSuccess) return hip_fail(e, "qs_batch_qaoa_run: graph launch");
    return QS_OK;
}

qs_status qs_batch_qaoa_run_sequential(qs_batch *b, double *out_dev)
{
    using namespace qs;
    if (!b || !out_dev) { set_error("qs_batch_qaoa_run_sequential: null argument"); return QS_EINVAL; }
    (void)hipSetDevice(b->device);
    unsigned *ctr = reinterpret_cast<unsigned *>(b->d_ctr);
    hipLaunchKernelGGL(k_qaoa_reset, dim3((b->nctr + 255) / 256), dim3(256), 0, b->stream, ctr, b->nctr, out_dev, b->count);
    hipError_t e = hipGetLastError();
    const int cbi = b->cbi;
    for (int i = 0; i < b->count && e == hipSuccess; ++i) {
        unsigned *next = ctr + 2 + b->count + i;     // one queue counter per launch
        const int nt = b->seq_count[cbi][i], t0 = b->seq_begin[cbi][i];
        const int grid = std::max(1, std::min(nt, b->cus * b->grid_per_cu));
        if (b->dtype == QS_C64)
            e = launch_qaoa<float>(b, cbi, true, t0, nt, next, out_dev, b->threads, grid);
        else
            e = launch_qaoa<double>(b, cbi, true, t0, nt, next, out_dev, b->threads, grid);
    }
    if (e != hipSuccess) return hip_fail(e, "qs_batch_qaoa_run_sequential");
    return QS_OK;
}

qs_status qs_batch_autotune(qs_batch *b, int *chosen, double *best_ms)
{
    using namespace qs;
    if (!b) { set_error("qs_batch_autotune: null batch"); return QS_EINVAL; }
    (void)hipSetDevice(b->device);
    double *tmp = nullptr;
    hipError_t e = hipMalloc(&tmp, sizeof(double) * b->count);
    if (e != hipSuccess) return hip_fail(e, "qs_batch_autotune: hipMalloc");
    // launch shapes (threads, workgroups per CU) x chunk groupings x LDS chunk sizes (the
    // same table and numbering as qs_batch_set_choice)
    const int shapes[][2] = {{256, 1}, {256, 2}, {256, 4}, {512, 1}, {512, 2}};
    const int nshape = (int)(sizeof(shapes) / sizeof(shapes[0]));
    const int ncand = nshape * kNumGroups * kNumCB;
    hipEvent_t e0, e1;
    (void)hipEventCreate(&e0);
    (void)hipEventCreate(&e1);
    double best = 1e30;
    int bi = 0;
    for (int c = 0; c < ncand && e == hipSuccess; ++c) {
        float tbest = 1e30f;
        for (int rep = 0; rep < 3 && e == hipSuccess; ++rep) {
            e = hipEventRecord(e0, b->stream);
            if (e == hipSuccess)
                e = run_batch(b, tmp, shapes[c % nshape][0], shapes[c % nshape][1], (c / nshape) % kNumGroups,
                              c / (nshape * kNumGroups));
            if (e == hipSuccess) e = hipEventRecord(e1, b->stream);
            if (e == hipSuccess) e = hipEventSynchronize(e1);
            float ms = 0.f;
            if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
            if (rep > 0) tbest = std::min(tbest, ms);     // first run warms up
        }
        if (e == hipSuccess && tbest < best) { best = tbest; bi = c; }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    (void)hipFree(tmp);
    if (e != hipSuccess) return hip_fail(e, "qs_batch_autotune");
    b->threads = shapes[bi % nshape][0];
    b->grid_per_cu = shapes[bi % nshape][1];
    b->group = (bi / nshape) % kNumGroups;
    b->cbi = bi / (nshape * kNumGroups);
    b->ntasks = b->grp_count[b->cbi][b->group];
    if (b->gexec) { (void)hipGraphExecDestroy(b->gexec); b->gexec = nullptr; }
    if (b->graph) { (void)hipGraphDestroy(b->graph); b->graph = nullptr; }
    if (chosen) *chosen = bi;
    if (best_ms) *best_ms = best;
    return QS_OK;
}

qs_status qs_batch_set_choice(qs_batch *b, int choice)
{
    using namespace qs;
    constexpr int nshape = 5, ncand = nshape * kNumGroups * kNumCB;
    static const int shapes[nshape][2] = {{256, 1}, {256, 2}, {256, 4}, {512, 1}, {512, 2}};
    if (!b || choice < 0 || choice >= ncand) {
        set_error("qs_batch_set_choice: null batch or choice outside 0.." + std::to_string(ncand - 1));
        return QS_EINVAL;
    }
    b->threads = shapes[choice % nshape][0];
    b->grid_per_cu = shapes[choice % nshape][1];
    b->group = (choice / nshape) % kNumGroups;
    b->cbi = choice / (nshape * kNumGroups);
    b->ntasks = b->grp_count[b->cbi][b->group];
    if (b->gexec) { (void)hipGraphExecDestroy(b->gexec); b->gexec = nullptr; }
    if (b->graph) { (void)hipGraphDestroy(b->graph); b->graph = nullptr; }
    return QS_OK;
}

qs_status qs_batch_free(qs_batch *b)
{
    if (!b) return QS_OK;
    (void)hipSetDevice(b->device);
    (void)hipStreamSynchronize(b->stream);
    if (b->gstream) (void)hipStreamSynchronize(b->gstream);
    if (b->gexec) (void)hipGraphExecDestroy(b->gexec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    if (b->ev_in) (void)hipEventDestroy(b->ev_in);
    if (b->ev_out) (void)hipEventDestroy(b->ev_out);
    if (b->gstream) (void)hipStreamDestroy(b->gstream);
    for (int cbi = 0; cbi < qs::kNumCB; ++cbi)
        for (void *p : {b->d_inst[cbi], b->d_tasks[cbi], b->d_seq_tasks[cbi]})
            if (p) (void)hipFree(p);
    for (void *p : {b->d_edges, b->d_tab, b->d_ctr})
        if (p) (void)hipFree(p);
    if (b->own_work)
        for (void *p : {b->d_work, b->d_czw})
            if (p) (void)hipFree(p);
    delete b;
    return QS_OK;
}

qs_status qs_batch_error(qs_batch *b, int *err)
{
    using namespace qs;
    if (!b || !err) { set_error("qs_batch_error: null argument"); return QS_EINVAL; }
    unsigned v = 0;
    hipError_t e = hipMemcpyAsync(&v, reinterpret_cast<unsigned *>(b->d_ctr) + 1, sizeof(unsigned), hipMemcpyDeviceToHost,
                                  b->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
    if (e != hipSuccess) return hip_fail(e, "qs_batch_error");
    *err = (int)v;
    return QS_OK;
}

}  // extern "C"
