// noalloc.hip -- qs_expect_noalloc: Pauli expectations with the reduction
// scratch in a fixed device array of the library instead of the handle's
// workspace, for callers that cannot allocate device memory.
//
// The array `scratch` below is one per GPU the library runs on, held until
// the process ends.  Host code never passes the array's name to a kernel or a
// copy (on the host that name is only a stand-in, not a device address): the
// first call on each device resolves the device address with
// hipGetSymbolAddress, with that device current, and keeps it per device.
// Every call on a GPU shares that GPU's array, so calls that overlap on one
// GPU race; each call rewrites every word it reads.
#include <mutex>

#include "amp.h"
#include "qs_internal.h"

namespace qs {
namespace {

constexpr int kNoAllocMaxTerms = 64;
constexpr int kNoAllocMaxParts = 2048;      // qs::expect_partials(n) <= 2048 for every n
constexpr size_t kTermBytes = 64 * 24;      // kNoAllocMaxTerms qs_pauli records (24 bytes each)
constexpr size_t kNoAllocBytes = kTermBytes + (size_t)kNoAllocMaxTerms * kNoAllocMaxParts * 8 + kNoAllocMaxTerms * 8;

__device__ __align__(256) unsigned char scratch[kNoAllocBytes];

// out[t] = sum over p of part[t * nparts + p], in ascending p (one thread per
// term: the same order as the host sum of qs_expect).
__global__ void k_sum_partials(const double *__restrict__ part, int nparts, int nterms, double *__restrict__ out)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nterms) return;
    double s = 0.0;
    for (int p = 0; p < nparts; ++p) s += part[(size_t)t * nparts + p];
    out[t] = s;
}

constexpr int kMaxDevices = 64;
std::mutex g_mu;
unsigned char *g_ptr[kMaxDevices] = {nullptr};

// Device address of this device's array (resolved once per device, with that
// device current).
hipError_t scratch_ptr(int device, unsigned char **out)
{
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> g(g_mu);
    if (!g_ptr[device]) {
        void *p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_ptr[device] = reinterpret_cast<unsigned char *>(p);
    }
    *out = g_ptr[device];
    return hipSuccess;
}

}  // namespace
}  // namespace qs

extern "C" qs_status qs_expect_noalloc(qs_state *st, int nterms, const qs_pauli *terms, double *out_host)
{
    using namespace qs;
    if (!st) { set_error("qs_expect_noalloc: null handle"); return QS_EINVAL; }
    if (!st->amps) { set_error("qs_expect_noalloc: handle has no attached state memory"); return QS_ESTATE; }
    if (nterms < 0 || nterms > kNoAllocMaxTerms || (nterms > 0 && !terms) || !out_host) {
        set_error("qs_expect_noalloc: nterms must be 0.." + std::to_string(kNoAllocMaxTerms) +
                  " (the fixed scratch holds that many terms), arrays non-null");
        return QS_EINVAL;
    }
    for (int t = 0; t < nterms; ++t) {
        if (st->n < 64 && ((terms[t].xmask | terms[t].zmask) >> st->n)) {
            set_error("qs_expect_noalloc: Pauli mask beyond n");
            return QS_EINVAL;
        }
    }
    const int parts = expect_partials(st->n);
    if (parts > kNoAllocMaxParts) { set_error("qs_expect_noalloc: too many partial sums"); return QS_EUNSUPPORTED; }
    if (nterms == 0) { *out_host = 0.0; return QS_OK; }
    int cur = -1;
    hipError_t e = hipGetDevice(&cur);
    if (e == hipSuccess && cur != st->device) e = hipSetDevice(st->device);
    unsigned char *base = nullptr;
    if (e == hipSuccess) e = scratch_ptr(st->device, &base);
    if (e != hipSuccess) return hip_fail(e, "qs_expect_noalloc: scratch address");
    qs_pauli *d_terms = reinterpret_cast<qs_pauli *>(base);
    double *d_part = reinterpret_cast<double *>(base + kTermBytes);
    double *d_sum = d_part + (size_t)kNoAllocMaxTerms * kNoAllocMaxParts;
    double h_sum[kNoAllocMaxTerms];
    e = hipMemcpyAsync(d_terms, terms, (size_t)nterms * sizeof(qs_pauli), hipMemcpyHostToDevice, st->stream);
    if (e == hipSuccess) e = launch_expect(st, nterms, d_terms, d_part, parts);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(kNoAllocMaxTerms), 0, st->stream, d_part, parts, nterms, d_sum);
        e = hipGetLastError();
    }
    if (e == hipSuccess)
        e = hipMemcpyAsync(h_sum, d_sum, (size_t)nterms * sizeof(double), hipMemcpyDeviceToHost, st->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(st->stream);
    if (e != hipSuccess) return hip_fail(e, "qs_expect_noalloc");
    double total = 0.0;
    for (int t = 0; t < nterms; ++t) total += terms[t].coeff * h_sum[t];
    *out_host = total;
    return QS_OK;
}
