// api.cpp -- the extern "C" entry points of libqs (include/qs.h).
//
// Argument checking, handle bookkeeping, plan upload and the step loop of
// Alg. 3 (for each gate block: a swap pass or a blocked pass).  Every step
// of the state-vector path runs in the library's HIP kernels; nothing here
// touches amplitudes on the host.
#include <algorithm>
#include <cstring>
#include <new>
#include <string>

#include "qs_internal.h"

namespace {
thread_local std::string g_last_error;
constexpr size_t kScratchBytes = 8u << 20;   // per state: gate matrices, swap programs, reduction partials
}

namespace qs {
void set_error(const std::string &msg) { g_last_error = msg; }
qs_status hip_fail(hipError_t e, const char *what)
{
    g_last_error = std::string(what) + ": " + hipGetErrorString(e);
    return QS_EHIP;
}
}  // namespace qs

using qs::hip_fail;
using qs::set_error;

#define QS_CHECK_HIP(call, what)                                  \
    do {                                                          \
        hipError_t e_ = (call);                                   \
        if (e_ != hipSuccess) return hip_fail(e_, what);          \
    } while (0)

static qs_status check_attached(qs_state *st, const char *fn)
{
    if (!st) { set_error(std::string(fn) + ": null handle"); return QS_EINVAL; }
    if (!st->amps) { set_error(std::string(fn) + ": handle has no attached state memory"); return QS_ESTATE; }
    int dev = -1;
    if (hipGetDevice(&dev) == hipSuccess && dev != st->device) {
        hipError_t e = hipSetDevice(st->device);
        if (e != hipSuccess) return hip_fail(e, fn);
    }
    return QS_OK;
}

extern "C" {

const char *qs_last_error(void) { return g_last_error.c_str(); }

const char *qs_version(void) { return "libqs 0.1 (gfx950)"; }

qs_status qs_create(int n, qs_dtype dtype, qs_state **out)
{
    if (!out) { set_error("qs_create: out is null"); return QS_EINVAL; }
    if (n < 1 || n > 34) { set_error("qs_create: n must be 1..34"); return QS_EINVAL; }
    if (dtype != QS_C128 && dtype != QS_C64) { set_error("qs_create: bad dtype"); return QS_EINVAL; }
    qs_state *st = new (std::nothrow) qs_state();
    if (!st) { set_error("qs_create: out of host memory"); return QS_ENOMEM; }
    st->n = n;
    st->dtype = dtype;
    *out = st;
    return QS_OK;
}

static bool is_device_memory(const void *p, int *device)
{
    hipPointerAttribute_t attr;
    hipError_t e = hipPointerGetAttributes(&attr, p);
    if (e != hipSuccess || attr.type != hipMemoryTypeDevice) {
        (void)hipGetLastError();
        return false;
    }
    *device = attr.device;
    return true;
}

qs_status qs_workspace_size(int n, qs_dtype dtype, size_t *bytes)
{
    if (!bytes || n < 1 || n > 34 || (dtype != QS_C128 && dtype != QS_C64)) {
        set_error("qs_workspace_size: bad arguments");
        return QS_EINVAL;
    }
    *bytes = kScratchBytes;
    return QS_OK;
}

qs_status qs_attach(qs_state *st, void *amps_dev, size_t bytes, void *hip_stream, void *workspace, size_t ws_bytes)
{
    if (!st || !amps_dev) { set_error("qs_attach: null handle or memory"); return QS_EINVAL; }
    const size_t want = ((size_t)1 << st->n) * (st->dtype == QS_C64 ? 8 : 16);
    if (bytes != want) {
        set_error("qs_attach: expected " + std::to_string(want) + " bytes, got " + std::to_string(bytes));
        return QS_EINVAL;
    }
    if (((uintptr_t)amps_dev & 255) != 0) { set_error("qs_attach: state memory must be 256-byte aligned"); return QS_EINVAL; }
    int device = -1;
    if (!is_device_memory(amps_dev, &device)) { set_error("qs_attach: pointer is not device memory"); return QS_EINVAL; }
    if (workspace) {
        int wdev = -1;
        if (ws_bytes < kScratchBytes) {
            set_error("qs_attach: workspace needs " + std::to_string(kScratchBytes) + " bytes, got " + std::to_string(ws_bytes));
            return QS_EINVAL;
        }
        if (((uintptr_t)workspace & 255) != 0) { set_error("qs_attach: workspace must be 256-byte aligned"); return QS_EINVAL; }
        if (!is_device_memory(workspace, &wdev) || wdev != device) {
            set_error("qs_attach: workspace is not device memory on the state's device");
            return QS_EINVAL;
        }
    }
    QS_CHECK_HIP(hipSetDevice(device), "qs_attach: hipSetDevice");
    if (workspace) {
        if (st->own_scratch && st->d_scratch) {
            (void)hipSetDevice(st->device);
            (void)hipStreamSynchronize(st->stream);
            (void)hipFree(st->d_scratch);
            QS_CHECK_HIP(hipSetDevice(device), "qs_attach: hipSetDevice");
        }
        st->d_scratch = workspace;
        st->scratch_bytes = ws_bytes;
        st->own_scratch = false;
    } else if (!st->own_scratch || !st->d_scratch || st->device != device) {
        if (st->own_scratch && st->d_scratch) (void)hipFree(st->d_scratch);
        st->d_scratch = nullptr;
        st->own_scratch = false;
        QS_CHECK_HIP(hipMalloc(&st->d_scratch, kScratchBytes), "qs_attach: hipMalloc scratch");
        st->scratch_bytes = kScratchBytes;
        st->own_scratch = true;
    }
    st->device = device;
    st->amps = amps_dev;
    st->bytes = bytes;
    st->stream = reinterpret_cast<hipStream_t>(hip_stream);
    return QS_OK;
}

qs_status qs_destroy(qs_state *st)
{
    if (!st) return QS_OK;
    if (st->own_scratch && st->d_scratch) {
        (void)hipSetDevice(st->device);
        (void)hipStreamSynchronize(st->stream);
        (void)hipFree(st->d_scratch);
    }
    delete st;
    return QS_OK;
}

qs_status qs_get_amplitudes(qs_state *st, uint64_t first, uint64_t count, void *host_out)
{
    qs_status s = check_attached(st, "qs_get_amplitudes");
    if (s) return s;
    const uint64_t N = 1ull << st->n;
    if ((count && !host_out) || first > N || count > N - first) {
        set_error("qs_get_amplitudes: range outside the state or null output");
        return QS_EINVAL;
    }
    if (!count) return QS_OK;
    const size_t ab = st->dtype == QS_C64 ? 8 : 16;
    QS_CHECK_HIP(hipMemcpyAsync(host_out, reinterpret_cast<const char *>(st->amps) + first * ab, count * ab,
                                hipMemcpyDeviceToHost, st->stream), "qs_get_amplitudes: copy");
    QS_CHECK_HIP(hipStreamSynchronize(st->stream), "qs_get_amplitudes: sync");
    return QS_OK;
}

qs_status qs_init_zero(qs_state *st) { return qs_init_basis(st, 0); }

qs_status qs_init_basis(qs_state *st, uint64_t index)
{
    qs_status s = check_attached(st, "qs_init_basis");
    if (s) return s;
    if (index >> st->n) { set_error("qs_init_basis: index out of range"); return QS_EINVAL; }
    QS_CHECK_HIP(qs::launch_init(st, index), "qs_init_basis: launch");
    return QS_OK;
}

qs_status qs_apply_gate(qs_state *st, int k, const int *targets, const double *matrix)
{
    qs_status s = check_attached(st, "qs_apply_gate");
    if (s) return s;
    if (k < 1 || k > 5 || k > st->n || !targets || !matrix) { set_error("qs_apply_gate: k must be 1..5 (<= n), arrays non-null"); return QS_EINVAL; }
    uint64_t seen = 0;
    for (int j = 0; j < k; ++j) {
        if (targets[j] < 0 || targets[j] >= st->n || (seen >> targets[j] & 1)) {
            set_error("qs_apply_gate: bad or repeated target");
            return QS_EINVAL;
        }
        seen |= 1ull << targets[j];
    }
    QS_CHECK_HIP(qs::launch_gate(st, k, targets, matrix), "qs_apply_gate: launch");
    return QS_OK;
}

// Run the encoded program of a plan's blocks from a given device program
// buffer (plan tables or scratch).
static qs_status run_blocks(qs_state *st, const qs::Plan &p, const int *d_prog, const void *d_mats, const char *fn)
{
    for (size_t b = 0; b < p.blocks.size(); ++b) {
        const size_t tab = (size_t)p.h_prog[p.prog_off[b] + 5] * 4;
        hipError_t e = qs::launch_block_prog(st, p.r, p.C, d_prog + p.prog_off[b], d_mats, tab, p.block_kmax[b],
                                             p.block_mfma[b] != 0, (p.h_prog[p.prog_off[b] + 3] & 4) != 0);
        if (e != hipSuccess) return hip_fail(e, fn);
    }
    return QS_OK;
}

qs_status qs_gate_class(int k, const int *targets, const double *matrix, int *kind, uint64_t *ctrl_mask, int *active)
{
    if (k < 1 || k > 5 || !targets || !matrix || !kind) { set_error("qs_gate_class: k must be 1..5, arrays non-null"); return QS_EINVAL; }
    uint64_t seen = 0;
    for (int j = 0; j < k; ++j) {
        if (targets[j] < 0 || targets[j] > 63 || ((seen >> targets[j]) & 1)) { set_error("qs_gate_class: bad or repeated target"); return QS_EINVAL; }
        seen |= 1ull << targets[j];
    }
    *kind = qs::gate_kind(k, targets, matrix, ctrl_mask, active);
    return QS_OK;
}

qs_status qs_swap_qubits(qs_state *st, int s, const int *a, const int *b)
{
    qs_status rc = check_attached(st, "qs_swap_qubits");
    if (rc) return rc;
    if (s < 0 || s > 8 || (s > 0 && (!a || !b))) { set_error("qs_swap_qubits: s must be 0..8"); return QS_EINVAL; }
    if (s == 0) return QS_OK;
    qs::Plan p;
    std::string err;
    rc = qs::build_swap_plan(st->n, st->dtype, s, a, b, &p, &err);
    if (rc) { set_error(err); return rc; }
    const size_t bytes = p.h_prog.size() * sizeof(int32_t);
    if (bytes > st->scratch_bytes) { set_error("qs_swap_qubits: program too large"); return QS_EINVAL; }
    QS_CHECK_HIP(hipMemcpyAsync(st->d_scratch, p.h_prog.data(), bytes, hipMemcpyHostToDevice, st->stream), "qs_swap_qubits: upload");
    rc = run_blocks(st, p, reinterpret_cast<const int *>(st->d_scratch), st->d_scratch, "qs_swap_qubits: launch");
    if (rc) return rc;
    QS_CHECK_HIP(hipStreamSynchronize(st->stream), "qs_swap_qubits: sync");
    return QS_OK;
}

qs_status qs_fuse(const qs_circuit *circ, int kmax, const qs_plan_opts *opts, qs_plan **out)
{
    if (!out) { set_error("qs_fuse: out is null"); return QS_EINVAL; }
    qs_plan *pl = new (std::nothrow) qs_plan();
    if (!pl) { set_error("qs_fuse: out of host memory"); return QS_ENOMEM; }
    std::string err;
    qs_status rc;
    try {
        if (opts && (opts->planner == 1 || opts->planner == 3)) rc = qs::build_plan_search(circ, kmax, opts, &pl->p, &err);
        else rc = qs::build_plan(circ, kmax, opts, &pl->p, &err);
    } catch (const std::bad_alloc &) {
        rc = QS_ENOMEM;
        err = "qs_fuse: out of host memory";
    } catch (const std::exception &ex) {
        rc = QS_EINVAL;
        err = std::string("qs_fuse: ") + ex.what();
    }
    if (rc) {
        set_error(err);
        delete pl;
        return rc;
    }
    *out = pl;
    return QS_OK;
}

// Device tables of a plan on the state's device: allocated and uploaded with
// hipMemcpyAsync on the state's stream the first time, under the plan's lock;
// a later user on another stream waits for the upload through its event.
static qs_status plan_tables(qs_state *st, qs_plan *pl, const void **d_prog, const void **d_mats, const char *fn)
{
    const qs::Plan &p = pl->p;
    std::lock_guard<std::mutex> g(pl->mu);
    for (const qs_plan::DevTables &t : pl->dev) {
        if (t.device != st->device) continue;
        if (t.stream != st->stream) QS_CHECK_HIP(hipStreamWaitEvent(st->stream, t.ready, 0), fn);
        *d_prog = t.d_prog;
        *d_mats = t.d_mats;
        return QS_OK;
    }
    qs_plan::DevTables t;
    t.device = st->device;
    t.stream = st->stream;
    const size_t pb = std::max<size_t>(4, p.h_prog.size() * sizeof(int32_t));
    const size_t mb = (p.dtype == QS_C64) ? p.h_mats32.size() * sizeof(float) : p.h_mats.size() * sizeof(double);
    hipError_t e = hipMalloc(&t.d_prog, pb);
    if (e == hipSuccess) e = hipMalloc(&t.d_mats, std::max<size_t>(mb, 16));
    if (e == hipSuccess && !p.h_prog.empty())
        e = hipMemcpyAsync(t.d_prog, p.h_prog.data(), p.h_prog.size() * sizeof(int32_t), hipMemcpyHostToDevice, st->stream);
    const void *src = (p.dtype == QS_C64) ? (const void *)p.h_mats32.data() : (const void *)p.h_mats.data();
    if (e == hipSuccess && mb) e = hipMemcpyAsync(t.d_mats, src, mb, hipMemcpyHostToDevice, st->stream);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&t.ready, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventRecord(t.ready, st->stream);
    if (e != hipSuccess) {
        (void)hipStreamSynchronize(st->stream);
        if (t.d_prog) (void)hipFree(t.d_prog);
        if (t.d_mats) (void)hipFree(t.d_mats);
        if (t.ready) (void)hipEventDestroy(t.ready);
        return hip_fail(e, fn);
    }
    pl->dev.push_back(t);
    *d_prog = t.d_prog;
    *d_mats = t.d_mats;
    return QS_OK;
}

static qs_status check_plan(qs_state *st, const qs_plan *plan, const char *fn)
{
    if (!plan) { set_error(std::string(fn) + ": null plan"); return QS_EINVAL; }
    const qs::Plan &p = plan->p;
    if (p.n != st->n || p.dtype != st->dtype) {
        set_error(std::string(fn) + ": plan is for n=" + std::to_string(p.n) + " dtype " + std::to_string((int)p.dtype) +
                  ", state is n=" + std::to_string(st->n) + " dtype " + std::to_string((int)st->dtype));
        return QS_ESTATE;
    }
    if (!p.blocks.empty() && p.n - p.C > 31) {
        set_error(std::string(fn) + ": too many chunks for one launch");
        return QS_EUNSUPPORTED;
    }
    return QS_OK;
}

qs_status qs_apply_plan(qs_state *st, qs_plan *plan)
{
    qs_status rc = check_attached(st, "qs_apply_plan");
    if (rc) return rc;
    rc = check_plan(st, plan, "qs_apply_plan");
    if (rc) return rc;
    const void *d_prog = nullptr, *d_mats = nullptr;
    rc = plan_tables(st, plan, &d_prog, &d_mats, "qs_apply_plan: upload");
    if (rc) return rc;
    return run_blocks(st, plan->p, reinterpret_cast<const int *>(d_prog), d_mats, "qs_apply_plan: launch");
}

qs_status qs_apply_plan_timed(qs_state *st, qs_plan *plan, float *ms_out, int *kinds_out, int cap)
{
    qs_status rc = check_attached(st, "qs_apply_plan_timed");
    if (rc) return rc;
    if (!ms_out) { set_error("qs_apply_plan_timed: null argument"); return QS_EINVAL; }
    rc = check_plan(st, plan, "qs_apply_plan_timed");
    if (rc) return rc;
    const qs::Plan &p = plan->p;
    const int ns = (int)p.blocks.size();
    if (cap < ns) { set_error("qs_apply_plan_timed: output too small"); return QS_EINVAL; }
    const void *d_prog = nullptr, *d_mats = nullptr;
    rc = plan_tables(st, plan, &d_prog, &d_mats, "qs_apply_plan_timed: upload");
    if (rc) return rc;
    std::vector<hipEvent_t> ev(ns + 1, nullptr);
    qs_status out = QS_OK;
    hipError_t e = hipSuccess;
    for (auto &x : ev)
        if (e == hipSuccess) e = hipEventCreate(&x);
    if (e == hipSuccess) e = hipEventRecord(ev[0], st->stream);
    for (int b = 0; b < ns && e == hipSuccess; ++b) {
        e = qs::launch_block(st, p, d_prog, d_mats, b);
        if (e == hipSuccess) e = hipEventRecord(ev[b + 1], st->stream);
    }
    if (e == hipSuccess) e = hipEventSynchronize(ev[ns]);
    if (e != hipSuccess) out = hip_fail(e, "qs_apply_plan_timed");
    for (int b = 0; b < ns && out == QS_OK; ++b) {
        float ms = 0.f;
        hipError_t e2 = hipEventElapsedTime(&ms, ev[b], ev[b + 1]);
        if (e2 != hipSuccess) out = hip_fail(e2, "qs_apply_plan_timed: elapsed");
        ms_out[b] = ms;
        if (kinds_out) kinds_out[b] = p.blocks[b].permute_only ? 0 : 1;
    }
    for (auto &x : ev)
        if (x) (void)hipEventDestroy(x);
    return out;
}

qs_status qs_plan_free(qs_plan *plan)
{
    if (!plan) return QS_OK;
    int cur = -1;
    (void)hipGetDevice(&cur);
    for (qs_plan::DevTables &t : plan->dev) {
        (void)hipSetDevice(t.device);
        if (t.ready) {
            (void)hipEventSynchronize(t.ready);
            (void)hipEventDestroy(t.ready);
        }
        if (t.d_prog) (void)hipFree(t.d_prog);
        if (t.d_mats) (void)hipFree(t.d_mats);
    }
    if (cur >= 0 && !plan->dev.empty()) (void)hipSetDevice(cur);
    delete plan;
    return QS_OK;
}

qs_status qs_plan_dump(const qs_plan *plan, char *buf, size_t len, size_t *needed)
{
    if (!plan) { set_error("qs_plan_dump: null plan"); return QS_EINVAL; }
    std::string s = qs::dump_plan(plan->p);
    if (needed) *needed = s.size() + 1;
    if (buf && len > 0) {
        size_t c = std::min(len - 1, s.size());
        std::memcpy(buf, s.data(), c);
        buf[c] = 0;
    }
    return QS_OK;
}

qs_status qs_plan_get_stats(const qs_plan *plan, qs_plan_stats *out)
{
    if (!plan || !out) { set_error("qs_plan_get_stats: null argument"); return QS_EINVAL; }
    *out = plan->p.stats;
    return QS_OK;
}

qs_status qs_plan_block(const qs_plan *plan, int b, int *phys, int *gate_ids, int cap, int *ngids)
{
    if (!plan) { set_error("qs_plan_block: null plan"); return QS_EINVAL; }
    int idx = -1;
    for (size_t i = 0; i < plan->p.blocks.size(); ++i) {
        if (plan->p.blocks[i].permute_only) continue;
        if (++idx == b) {
            const qs::Block &blk = plan->p.blocks[i];
            if (phys)
                for (size_t j = 0; j < blk.P_in.size(); ++j) phys[j] = blk.P_in[j];
            if (gate_ids)
                for (int j = 0; j < (int)blk.gate_ids.size() && j < cap; ++j) gate_ids[j] = blk.gate_ids[j];
            if (ngids) *ngids = (int)blk.gate_ids.size();
            return QS_OK;
        }
    }
    set_error("qs_plan_block: block index out of range");
    return QS_EINVAL;
}

qs_status qs_plan_layout(const qs_plan *plan, int s, int *perm, int *nsteps)
{
    if (!plan) { set_error("qs_plan_layout: null plan"); return QS_EINVAL; }
    const int ns = (int)plan->p.blocks.size();
    if (nsteps) *nsteps = ns;
    if (s < 0 || s > ns || s >= (int)plan->p.layouts.size()) { set_error("qs_plan_layout: step out of range"); return QS_EINVAL; }
    if (perm)
        for (int q = 0; q < plan->p.n; ++q) perm[q] = plan->p.layouts[s][q];
    return QS_OK;
}

qs_status qs_plan_program(const qs_plan *plan, int32_t *words, size_t cap, size_t *nwords, int64_t *offsets,
                          int cap_steps, int *nsteps, int *r, int *C, double *mats, size_t cap_mats, size_t *nmats)
{
    if (!plan) { set_error("qs_plan_program: null plan"); return QS_EINVAL; }
    const qs::Plan &p = plan->p;
    if (nwords) *nwords = p.h_prog.size();
    if (words)
        for (size_t i = 0; i < p.h_prog.size() && i < cap; ++i) words[i] = p.h_prog[i];
    if (nsteps) *nsteps = (int)p.prog_off.size();
    if (offsets)
        for (int i = 0; i < (int)p.prog_off.size() && i < cap_steps; ++i) offsets[i] = p.prog_off[i];
    if (r) *r = p.r;
    if (C) *C = p.C;
    if (nmats) *nmats = p.h_mats.size();
    if (mats)
        for (size_t i = 0; i < p.h_mats.size() && i < cap_mats; ++i) mats[i] = p.h_mats[i];
    return QS_OK;
}

qs_status qs_probs(qs_state *st, double *out_dev)
{
    qs_status rc = check_attached(st, "qs_probs");
    if (rc) return rc;
    if (!out_dev) { set_error("qs_probs: null output"); return QS_EINVAL; }
    QS_CHECK_HIP(qs::launch_probs(st, out_dev), "qs_probs: launch");
    return QS_OK;
}

qs_status qs_expect(qs_state *st, int nterms, const qs_pauli *terms, double *out_host)
{
    qs_status rc = check_attached(st, "qs_expect");
    if (rc) return rc;
    if (nterms < 0 || (nterms > 0 && !terms) || !out_host) { set_error("qs_expect: bad arguments"); return QS_EINVAL; }
    for (int t = 0; t < nterms; ++t) {
        if (st->n < 64 && ((terms[t].xmask | terms[t].zmask) >> st->n)) {
            set_error("qs_expect: Pauli mask beyond n");
            return QS_EINVAL;
        }
    }
    double total = 0.0;
    const int parts = qs::expect_partials(st->n);
    // terms are processed in groups that fit the scratch buffer
    const size_t per_term = sizeof(qs_pauli) + (size_t)parts * sizeof(double);
    const int group = (int)std::max<size_t>(1, (st->scratch_bytes - 256) / per_term);
    std::vector<double> h_part;
    for (int t0 = 0; t0 < nterms; t0 += group) {
        const int nt = std::min(group, nterms - t0);
        char *base = reinterpret_cast<char *>(st->d_scratch);
        qs_pauli *d_terms = reinterpret_cast<qs_pauli *>(base);
        double *d_part = reinterpret_cast<double *>(base + ((nt * sizeof(qs_pauli) + 255) & ~(size_t)255));
        QS_CHECK_HIP(hipMemcpyAsync(d_terms, terms + t0, nt * sizeof(qs_pauli), hipMemcpyHostToDevice, st->stream), "qs_expect: upload");
        QS_CHECK_HIP(qs::launch_expect(st, nt, d_terms, d_part, parts), "qs_expect: launch");
        h_part.resize((size_t)nt * parts);
        QS_CHECK_HIP(hipMemcpyAsync(h_part.data(), d_part, h_part.size() * sizeof(double), hipMemcpyDeviceToHost, st->stream), "qs_expect: download");
        QS_CHECK_HIP(hipStreamSynchronize(st->stream), "qs_expect: sync");
        for (int t = 0; t < nt; ++t) {
            double s = 0.0;
            for (int i = 0; i < parts; ++i) s += h_part[(size_t)t * parts + i];
            total += terms[t0 + t].coeff * s;
        }
    }
    *out_host = total;
    return QS_OK;
}

}  // extern "C"
