// k_block.hip -- the blocked pass: one HBM read and one HBM write of the
// state per gate block, every op of the block applied on chip.
//
// Paper: Alg. 3 (for each chunk, for each gate of the block: apply), Sec. V-A
// (chunks staged on chip, one thread block per chunk, several amplitudes per
// thread), Sec. V-B / Eq. 4 (qubit swaps, here folded into the write-back).
//
// gfx950 design:
//   - a workgroup owns one chunk of 2^C amplitudes: local bit b is physical
//     qubit P_in[b]; the lowest L local bits are physical 0..L-1, so the
//     chunk is 2^(C-L) runs of 2^L contiguous amplitudes (>= 256 B for
//     complex128) and every global access of a wavefront is coalesced;
//   - each thread keeps 2^R amplitudes in VGPRs.  A phase fixes which R
//     chunk bits are register bits; every dense op of the phase acts on
//     register bits only and runs from registers with compile-time indexing
//     (one code path per register mask), diagonal ops run in any phase;
//   - between phases, one exchange through LDS (XOR-swizzled per exchange so
//     16 consecutive lanes touch 16 distinct 16-byte slots) re-maps which bits
//     are register bits;
//   - the write-back may permute the chunk's bits (P_out), which performs a
//     qubit swap at no extra HBM pass.
#include "amp.h"
#include "qs_internal.h"

namespace qs {
namespace {

template <int MASK>
struct MaskInfo {
    static constexpr int K = __builtin_popcount(MASK);
    static constexpr int D = 1 << K;
};

// deposit the low bits of v into the set bits of MASK (compile time)
template <int MASK>
__device__ __forceinline__ constexpr int pdep_c(int v)
{
    int r = 0, i = 0;
    for (int b = 0; b < 8; ++b)
        if ((MASK >> b) & 1) { r |= ((v >> i) & 1) << b; ++i; }
    return r;
}

// Dense op on the register bits in MASK: for every register index base with
// the MASK bits clear, the 2^K amplitudes base | pdep(c) are multiplied by the
// 2^K x 2^K matrix M (row-major, interleaved re/im, index bit i <-> i-th set
// bit of MASK).
template <int R, int MASK, typename F, typename V>
__device__ __forceinline__ void apply_dense(V (&v)[1 << R], const F *__restrict__ M)
{
    constexpr int D = MaskInfo<MASK>::D;
#pragma unroll
    for (int base = 0; base < (1 << R); ++base) {
        if (base & MASK) continue;
        V in[D];
#pragma unroll
        for (int c = 0; c < D; ++c) in[c] = v[base | pdep_c<MASK>(c)];
#pragma unroll
        for (int r = 0; r < D; ++r) {
            V acc;
            acc = cmul<F, V>(M[2 * (r * D)], M[2 * (r * D) + 1], in[0]);
#pragma unroll
            for (int c = 1; c < D; ++c) cmac<F, V>(acc, M[2 * (r * D + c)], M[2 * (r * D + c) + 1], in[c]);
            v[base | pdep_c<MASK>(r)] = acc;
        }
    }
}

template <int R, int MASK, typename F, typename V>
__device__ __forceinline__ void dense_dispatch(int mask, V (&v)[1 << R], const F *__restrict__ M)
{
    if constexpr (MASK < (1 << R)) {
        if (mask == MASK) {
            apply_dense<R, MASK, F, V>(v, M);
            return;
        }
        dense_dispatch<R, MASK + 1, F, V>(mask, v, M);
    }
}

// local index (within the chunk) of thread tid's register 0 in a layout:
// thread bit j <-> local bit T[j]
__device__ __forceinline__ uint32_t thread_local_bits(uint32_t tid, const int *__restrict__ T, int tb)
{
    uint32_t l = 0;
    for (int j = 0; j < tb; ++j) l |= ((tid >> j) & 1u) << T[j];
    return l;
}

// bits of v selected by mask, packed to the low end (ascending)
__device__ __forceinline__ uint32_t pext_u32(uint32_t v, uint32_t mask)
{
    uint32_t r = 0;
    int i = 0;
    for (int b = 0; b < 16; ++b)
        if ((mask >> b) & 1u) { r |= ((v >> b) & 1u) << i; ++i; }
    return r;
}

// physical offset of a local index
__device__ __forceinline__ uint64_t local_to_phys(uint32_t l, const int *__restrict__ P, int C)
{
    uint64_t o = 0;
    for (int b = 0; b < C; ++b)
        if ((l >> b) & 1u) o |= 1ull << P[b];
    return o;
}

// XOR swizzle of an LDS slot: bits >= 4 fold into the low nibble
__device__ __forceinline__ uint32_t swz(uint32_t l, uint32_t swlo, uint32_t swhi)
{
    uint32_t f = 0;
    uint32_t h = l >> 4;
#pragma unroll
    for (int b = 0; b < 8; ++b)
        if ((h >> b) & 1u) f ^= (swlo >> (4 * b)) & 15u;
#pragma unroll
    for (int b = 0; b < 2; ++b)
        if ((h >> (8 + b)) & 1u) f ^= (swhi >> (4 * b)) & 15u;
    return l ^ f;
}

template <int R, typename F>
__global__ __launch_bounds__(256) void k_block(typename AmpOf<F>::type *__restrict__ amps,
                                              const int *__restrict__ prog, const F *__restrict__ mats, int n)
{
    using V = typename AmpOf<F>::type;
    extern __shared__ unsigned char lds_raw[];
    V *lds = reinterpret_cast<V *>(lds_raw);
    constexpr int NR = 1 << R;

    const int nph = prog[0];
    const int C = prog[1];
    const int tb = C - R;
    const int *__restrict__ Pin = prog + PROG_HDR;
    const int *__restrict__ Pout = prog + PROG_HDR + C;
    const uint32_t tid = threadIdx.x;

    // chunk base: the workgroup index spread over the physical qubits outside the chunk
    uint64_t cmask = 0;
    for (int b = 0; b < C; ++b) cmask |= 1ull << Pin[b];
    uint64_t base = 0;
    {
        uint64_t w = blockIdx.x;
        int bi = 0;
        for (int q = 0; q < n; ++q) {
            if ((cmask >> q) & 1ull) continue;
            if ((w >> bi) & 1ull) base |= 1ull << q;
            ++bi;
        }
    }

    V v[NR];
    const int *ph = prog + PROG_HDR + 2 * C;
    // ---- load in phase 0's layout
    {
        const int *Rb = ph + PHASE_HDR;
        const int *T = Rb + R;
        uint64_t g = base | local_to_phys(thread_local_bits(tid, T, tb), Pin, C);
#pragma unroll
        for (int m = 0; m < NR; ++m) {
            uint64_t o = 0;
#pragma unroll
            for (int j = 0; j < R; ++j)
                if ((m >> j) & 1) o |= 1ull << Pin[Rb[j]];
            v[m] = amps[g | o];
        }
    }
    const int *prev = nullptr;
    for (int p = 0; p < nph; ++p) {
        const int nops = ph[0];
        const int *Rb = ph + PHASE_HDR;
        const int *T = Rb + R;
        if (p > 0) {
            // ---- exchange from the previous layout to this one through LDS
            const uint32_t swlo = (uint32_t)ph[1], swhi = (uint32_t)ph[2];
            const int *pR = prev + PHASE_HDR;
            const int *pT = pR + R;
            uint32_t wt = swz(thread_local_bits(tid, pT, tb), swlo, swhi);
            uint32_t rt = swz(thread_local_bits(tid, T, tb), swlo, swhi);
            __syncthreads();
#pragma unroll
            for (int m = 0; m < NR; ++m) {
                uint32_t lr = 0;
#pragma unroll
                for (int j = 0; j < R; ++j)
                    if ((m >> j) & 1) lr |= 1u << pR[j];
                lds[wt ^ swz(lr, swlo, swhi)] = v[m];
            }
            __syncthreads();
#pragma unroll
            for (int m = 0; m < NR; ++m) {
                uint32_t lr = 0;
#pragma unroll
                for (int j = 0; j < R; ++j)
                    if ((m >> j) & 1) lr |= 1u << Rb[j];
                v[m] = lds[rt ^ swz(lr, swlo, swhi)];
            }
        }
        // ---- ops of this phase
        const int *op = T + tb;
        for (int o = 0; o < nops; ++o, op += OP_WORDS) {
            const int w0 = op[0];
            const int kind = w0 & 0xff;
            const int variant = (w0 >> 8) & 0xff;
            const int k = (w0 >> 16) & 0xff;
            const int64_t moff = (int64_t)(uint32_t)op[1] | ((int64_t)op[2] << 32);
            const F *__restrict__ M = mats + moff;   // moff counts scalars
            if (kind == OP_DENSE) {
                dense_dispatch<R, 1, F, V>(variant, v, M);
            } else if (kind == OP_DIAG_REG) {
                // uniform entry per register
#pragma unroll
                for (int m = 0; m < NR; ++m) v[m] = cmul<F, V>(M[2 * m], M[2 * m + 1], v[m]);
            } else if (kind == OP_DIAG_ROW) {
                // this lane's row of 2^R entries; row = the op's thread-index bits of tid
                const uint32_t row = pext_u32(tid, (uint32_t)op[3]);
                const F *__restrict__ E = M + (size_t)row * (2 * NR);
#pragma unroll
                for (int m = 0; m < NR; ++m) v[m] = cmul<F, V>(E[2 * m], E[2 * m + 1], v[m]);
            } else if (kind == OP_SIGN_REG) {
                const uint32_t s = (uint32_t)op[3];
#pragma unroll
                for (int m = 0; m < NR; ++m)
                    if ((s >> m) & 1u) { v[m].x = -v[m].x; v[m].y = -v[m].y; }
            } else if (kind == OP_SIGN_ROW) {
                const uint32_t row = pext_u32(tid, (uint32_t)op[1]);
                const uint32_t s = (uint32_t)prog[op[3] + row];
#pragma unroll
                for (int m = 0; m < NR; ++m) {
                    const F sg = ((s >> m) & 1u) ? (F)-1 : (F)1;
                    v[m].x *= sg;
                    v[m].y *= sg;
                }
            } else {
                // general diagonal on local bits tl[0..k-1] (ascending); entry index bit i <-> tl[i]
                const int *tl = prog + op[3];
                uint32_t lt = thread_local_bits(tid, T, tb);
                uint32_t it = 0;
                for (int i = 0; i < k; ++i) it |= ((lt >> tl[i]) & 1u) << i;
#pragma unroll
                for (int m = 0; m < NR; ++m) {
                    uint32_t lr = 0;
#pragma unroll
                    for (int j = 0; j < R; ++j)
                        if ((m >> j) & 1) lr |= 1u << Rb[j];
                    uint32_t ir = 0;
                    for (int i = 0; i < k; ++i) ir |= ((lr >> tl[i]) & 1u) << i;
                    const uint32_t idx = it | ir;
                    v[m] = cmul<F, V>(M[2 * idx], M[2 * idx + 1], v[m]);
                }
            }
        }
        prev = ph;
        ph = op;
        // skip past nothing: op now points after the last op of this phase
    }
    // ---- store in the last layout, through P_out
    if ((prog[3] & 2) && nph == 1) {
        // No exchange (hence no barrier) separated the loads from the stores, and the
        // write-back permutes positions: a store may target an amplitude another wave
        // has not loaded yet.  Wait for this wave's loads, then for every wave.
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
    }
    {
        const int *Rb = prev + PHASE_HDR;
        const int *T = Rb + R;
        uint64_t g = base | local_to_phys(thread_local_bits(tid, T, tb), Pout, C);
#pragma unroll
        for (int m = 0; m < NR; ++m) {
            uint64_t o = 0;
#pragma unroll
            for (int j = 0; j < R; ++j)
                if ((m >> j) & 1) o |= 1ull << Pout[Rb[j]];
            amps[g | o] = v[m];
        }
    }
}

template <int R, typename F>
hipError_t launch_R(qs_state *st, const int *d_prog, const F *d_mats, int C)
{
    using V = typename AmpOf<F>::type;
    size_t lds = ((size_t)1 << C) * sizeof(V);
    auto kern = k_block<R, F>;
    static bool attr_set = false;
    if (!attr_set) {
        hipError_t e = hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
        if (e != hipSuccess) return e;
        attr_set = true;
    }
    unsigned threads = 1u << (C - R);
    uint64_t grid = 1ull << (st->n - C);
    hipLaunchKernelGGL(kern, dim3((unsigned)grid), dim3(threads), lds, st->stream,
                       reinterpret_cast<V *>(st->amps), d_prog, d_mats, st->n);
    return hipGetLastError();
}

template <typename F>
hipError_t launch_F(qs_state *st, int r, const int *d_prog, const F *d_mats, int C)
{
    switch (r) {
    case 1: return launch_R<1, F>(st, d_prog, d_mats, C);
    case 2: return launch_R<2, F>(st, d_prog, d_mats, C);
    case 3: return launch_R<3, F>(st, d_prog, d_mats, C);
    case 4: return launch_R<4, F>(st, d_prog, d_mats, C);
    case 5: return launch_R<5, F>(st, d_prog, d_mats, C);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace

hipError_t launch_block_prog(qs_state *st, int r, int C, const int *d_prog, const void *d_mats)
{
    if (C - r > 8 || C < r || st->n < C) return hipErrorInvalidValue;
    if (st->dtype == QS_C64) return launch_F<float>(st, r, d_prog, reinterpret_cast<const float *>(d_mats), C);
    return launch_F<double>(st, r, d_prog, reinterpret_cast<const double *>(d_mats), C);
}

hipError_t launch_block(qs_state *st, const Plan &p, int b)
{
    const int *prog = reinterpret_cast<const int *>(p.d_prog) + p.prog_off[b];
    return launch_block_prog(st, p.r, p.C, prog, p.d_mats);
}

}  // namespace qs
