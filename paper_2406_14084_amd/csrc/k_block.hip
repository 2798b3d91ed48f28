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
#include <algorithm>
#include <mutex>
#include <type_traits>

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
template <int R, int MASK, typename F, typename V, typename P>
__device__ __forceinline__ void apply_dense(V (&v)[1 << R], P M)
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

// Runs the dense op whose register mask equals `mask`; only masks of at most
// KMAX bits are compiled in (the planner picks the variant wide enough for
// its ops, which keeps register pressure low for plans of narrow ops).
#define QS_DENSE_CASE(MM)                                                                 \
    case MM:                                                                              \
        if constexpr ((MM) < (1 << R) && __builtin_popcount(MM) <= KMAX)                  \
            apply_dense<R, ((MM) < (1 << R) ? (MM) : 1), F, V, P>(v, M);                   \
        else                                                                              \
            __builtin_unreachable();                                                      \
        break;

template <int R, int KMAX, typename F, typename V, typename P>
__device__ __forceinline__ void dense_dispatch(int mask, V (&v)[1 << R], P M)
{
    switch (mask) {
        QS_DENSE_CASE(1) QS_DENSE_CASE(2) QS_DENSE_CASE(3) QS_DENSE_CASE(4) QS_DENSE_CASE(5)
        QS_DENSE_CASE(6) QS_DENSE_CASE(7) QS_DENSE_CASE(8) QS_DENSE_CASE(9) QS_DENSE_CASE(10)
        QS_DENSE_CASE(11) QS_DENSE_CASE(12) QS_DENSE_CASE(13) QS_DENSE_CASE(14) QS_DENSE_CASE(15)
        QS_DENSE_CASE(16) QS_DENSE_CASE(17) QS_DENSE_CASE(18) QS_DENSE_CASE(19) QS_DENSE_CASE(20)
        QS_DENSE_CASE(21) QS_DENSE_CASE(22) QS_DENSE_CASE(23) QS_DENSE_CASE(24) QS_DENSE_CASE(25)
        QS_DENSE_CASE(26) QS_DENSE_CASE(27) QS_DENSE_CASE(28) QS_DENSE_CASE(29) QS_DENSE_CASE(30)
        QS_DENSE_CASE(31)
    default:
        __builtin_unreachable();
    }
}
#undef QS_DENSE_CASE

// One 2x2 gate on each register bit of MASK, ascending, matrices back to back.
template <int R, int MASK, int J, typename F, typename V, typename P>
__device__ __forceinline__ void apply_multi1_from(V (&v)[1 << R], P M)
{
    if constexpr (J < R) {
        if constexpr ((MASK >> J) & 1) {
            apply_dense<R, (1 << J), F, V, P>(v, M);
            apply_multi1_from<R, MASK, J + 1, F, V, P>(v, M + 8);
        } else {
            apply_multi1_from<R, MASK, J + 1, F, V, P>(v, M);
        }
    }
}

template <int R, int MASK, typename F, typename V, typename P>
__device__ __forceinline__ void apply_multi1(V (&v)[1 << R], P M)
{
    apply_multi1_from<R, MASK, 0, F, V, P>(v, M);
}

#define QS_MULTI_CASE(MM)                                                                 \
    case MM:                                                                              \
        if constexpr ((MM) < (1 << R)) apply_multi1<R, ((MM) < (1 << R) ? (MM) : 1), F, V, P>(v, M); \
        else __builtin_unreachable();                                                     \
        break;

template <int R, typename F, typename V, typename P>
__device__ __forceinline__ void multi1_dispatch(int mask, V (&v)[1 << R], P M)
{
    switch (mask) {
        QS_MULTI_CASE(1) QS_MULTI_CASE(2) QS_MULTI_CASE(3) QS_MULTI_CASE(4) QS_MULTI_CASE(5)
        QS_MULTI_CASE(6) QS_MULTI_CASE(7) QS_MULTI_CASE(8) QS_MULTI_CASE(9) QS_MULTI_CASE(10)
        QS_MULTI_CASE(11) QS_MULTI_CASE(12) QS_MULTI_CASE(13) QS_MULTI_CASE(14) QS_MULTI_CASE(15)
        QS_MULTI_CASE(16) QS_MULTI_CASE(17) QS_MULTI_CASE(18) QS_MULTI_CASE(19) QS_MULTI_CASE(20)
        QS_MULTI_CASE(21) QS_MULTI_CASE(22) QS_MULTI_CASE(23) QS_MULTI_CASE(24) QS_MULTI_CASE(25)
        QS_MULTI_CASE(26) QS_MULTI_CASE(27) QS_MULTI_CASE(28) QS_MULTI_CASE(29) QS_MULTI_CASE(30)
        QS_MULTI_CASE(31)
    default:
        __builtin_unreachable();
    }
}
#undef QS_MULTI_CASE

// Real plane rotation on each register bit of MASK (ascending), as two shears per
// amplitude pair (x0, x1) = (bit clear, bit set): x0 += beta x1, then x1 += alpha x0,
// on the real and imaginary parts alike -- in place, one FMA each.  (The rotation's
// diagonal scaling, diag(cos, 1 / cos), is folded into the diagonal op before it.)
// Coefficients (beta, alpha) of the bits back to back.
__device__ __forceinline__ double fma_f(double a, double b, double c) { return __builtin_fma(a, b, c); }
__device__ __forceinline__ float fma_f(float a, float b, float c) { return __builtin_fmaf(a, b, c); }

template <int R, int MASK, int J, typename F, typename V, typename P>
__device__ __forceinline__ void apply_rot_from(V (&v)[1 << R], P M)
{
    if constexpr (J < R) {
        if constexpr ((MASK >> J) & 1) {
            const F beta = M[0], alpha = M[1];
#pragma unroll
            for (int base = 0; base < (1 << R); ++base) {
                if (base & (1 << J)) continue;
                V &x0 = v[base];
                V &x1 = v[base | (1 << J)];
                x0.x = fma_f(beta, x1.x, x0.x);
                x0.y = fma_f(beta, x1.y, x0.y);
                x1.x = fma_f(alpha, x0.x, x1.x);
                x1.y = fma_f(alpha, x0.y, x1.y);
            }
            apply_rot_from<R, MASK, J + 1, F, V, P>(v, M + 2);
        } else {
            apply_rot_from<R, MASK, J + 1, F, V, P>(v, M);
        }
    }
}

#define QS_ROT_CASE(MM)                                                                   \
    case MM:                                                                              \
        if constexpr ((MM) < (1 << R)) apply_rot_from<R, ((MM) < (1 << R) ? (MM) : 1), 0, F, V, P>(v, M); \
        else __builtin_unreachable();                                                     \
        break;

template <int R, typename F, typename V, typename P>
__device__ __forceinline__ void rot_dispatch(int mask, V (&v)[1 << R], P M)
{
    switch (mask) {
        QS_ROT_CASE(1) QS_ROT_CASE(2) QS_ROT_CASE(3) QS_ROT_CASE(4) QS_ROT_CASE(5)
        QS_ROT_CASE(6) QS_ROT_CASE(7) QS_ROT_CASE(8) QS_ROT_CASE(9) QS_ROT_CASE(10)
        QS_ROT_CASE(11) QS_ROT_CASE(12) QS_ROT_CASE(13) QS_ROT_CASE(14) QS_ROT_CASE(15)
        QS_ROT_CASE(16) QS_ROT_CASE(17) QS_ROT_CASE(18) QS_ROT_CASE(19) QS_ROT_CASE(20)
        QS_ROT_CASE(21) QS_ROT_CASE(22) QS_ROT_CASE(23) QS_ROT_CASE(24) QS_ROT_CASE(25)
        QS_ROT_CASE(26) QS_ROT_CASE(27) QS_ROT_CASE(28) QS_ROT_CASE(29) QS_ROT_CASE(30)
        QS_ROT_CASE(31)
    default:
        __builtin_unreachable();
    }
}
#undef QS_ROT_CASE

// Permutation op (multi-controlled X: X, CX, CCX): flip register bit T of every
// register whose bits in ctrl (uniform, bit T clear) equal cval (a control may
// require 1 or 0).  No
// arithmetic: each pair (m, m | 1 << T) swaps its bit patterns under a uniform
// mask.  (A switch over every (target, controls) pattern with compile-time
// moves, or selects between the pair, make the compiler index the register
// array dynamically, which puts the whole state in scratch memory.)  SWAP is
// encoded as three of these.
// exchange a and b where the uniform mask k is all ones: (a, b) ^= ((a ^ b) & k)
__device__ __forceinline__ void cswap(double &a, double &b, uint64_t k)
{
    const uint64_t x = __double_as_longlong(a), y = __double_as_longlong(b);
    const uint64_t d = (x ^ y) & k;
    a = __longlong_as_double(x ^ d);
    b = __longlong_as_double(y ^ d);
}
__device__ __forceinline__ void cswap(float &a, float &b, uint64_t k)
{
    const uint32_t x = __float_as_uint(a), y = __float_as_uint(b);
    const uint32_t d = (x ^ y) & (uint32_t)k;
    a = __uint_as_float(x ^ d);
    b = __uint_as_float(y ^ d);
}

template <int R, int T, typename V>
__device__ __forceinline__ void apply_mcx(V (&v)[1 << R], uint32_t ctrl, uint32_t cval)
{
#pragma unroll
    for (int m = 0; m < (1 << R); ++m) {
        if ((m >> T) & 1) continue;
        // all ones where register m's control bits hold cval (uniform, a scalar value)
        const uint64_t k = 0ull - (uint64_t)(((uint32_t)m & ctrl) == cval);
        cswap(v[m].x, v[m | (1 << T)].x, k);
        cswap(v[m].y, v[m | (1 << T)].y, k);
        // opaque to the optimiser: the cases of the dispatch switch must not be
        // merged into one that indexes the register array by a runtime value
        asm volatile("" : "+v"(v[m].x), "+v"(v[m].y), "+v"(v[m | (1 << T)].x), "+v"(v[m | (1 << T)].y));
    }
}

// A CX with one control (the common case: one register bit on a given value) as a
// compile-time exchange of the registers it pairs: after the case, the whole state is
// pinned to registers (the switch's cases must not merge into an indexed array), so
// the exchange costs one register move per dword instead of the masked exchange's
// two selects and two XORs.
template <int R, int T, int CB, int CV, typename V>
__device__ __forceinline__ void apply_cx_c(V (&v)[1 << R])
{
#pragma unroll
    for (int m = 0; m < (1 << R); ++m) {
        if ((m >> T) & 1) continue;
        if (((m >> CB) & 1) != CV) continue;
        const V t = v[m];
        v[m] = v[m | (1 << T)];
        v[m | (1 << T)] = t;
    }
#pragma unroll
    for (int m = 0; m < (1 << R); ++m) asm volatile("" : "+v"(v[m].x), "+v"(v[m].y));
}

template <int R, int T, typename V>
__device__ __forceinline__ void cx_t(uint32_t cb, uint32_t cv, V (&v)[1 << R])
{
    switch (cb * 2 + cv) {
#define QS_CXC(CBV, CVV)                                                                        \
    case CBV * 2 + CVV:                                                                         \
        if constexpr (CBV < R && CBV != T)                                                      \
            apply_cx_c<R, T, (CBV < R && CBV != T ? CBV : (T + 1) % R), CVV, V>(v);             \
        else                                                                                    \
            __builtin_unreachable();                                                            \
        break;
    QS_CXC(0, 0) QS_CXC(0, 1) QS_CXC(1, 0) QS_CXC(1, 1) QS_CXC(2, 0) QS_CXC(2, 1) QS_CXC(3, 0) QS_CXC(3, 1)
    QS_CXC(4, 0) QS_CXC(4, 1)
#undef QS_CXC
    default: __builtin_unreachable();
    }
}

// (ONE_CTRL: the one-control cases have their compile-time paths; off in the variants
// with dense ops, where the extra paths would push the register allocation into spills)
template <int R, bool ONE_CTRL, typename V>
__device__ __forceinline__ void mcx_dispatch(int var, uint32_t cval, V (&v)[1 << R])
{
    const uint32_t ctrl = (uint32_t)var >> 3;
    if (ONE_CTRL && __builtin_popcount(ctrl) == 1) {
        const uint32_t cb = __builtin_ctz(ctrl), cv = cval ? 1u : 0u;
        switch (var & 7) {
        case 0: cx_t<R, 0, V>(cb, cv, v); return;
        case 1: if constexpr (R > 1) { cx_t<R, (R > 1 ? 1 : 0), V>(cb, cv, v); return; } else __builtin_unreachable();
        case 2: if constexpr (R > 2) { cx_t<R, (R > 2 ? 2 : 0), V>(cb, cv, v); return; } else __builtin_unreachable();
        case 3: if constexpr (R > 3) { cx_t<R, (R > 3 ? 3 : 0), V>(cb, cv, v); return; } else __builtin_unreachable();
        case 4: if constexpr (R > 4) { cx_t<R, (R > 4 ? 4 : 0), V>(cb, cv, v); return; } else __builtin_unreachable();
        default: __builtin_unreachable();
        }
    }
    switch (var & 7) {
    case 0: apply_mcx<R, 0, V>(v, ctrl, cval); break;
    case 1: if constexpr (R > 1) apply_mcx<R, (R > 1 ? 1 : 0), V>(v, ctrl, cval); else __builtin_unreachable(); break;
    case 2: if constexpr (R > 2) apply_mcx<R, (R > 2 ? 2 : 0), V>(v, ctrl, cval); else __builtin_unreachable(); break;
    case 3: if constexpr (R > 3) apply_mcx<R, (R > 3 ? 3 : 0), V>(v, ctrl, cval); else __builtin_unreachable(); break;
    case 4: if constexpr (R > 4) apply_mcx<R, (R > 4 ? 4 : 0), V>(v, ctrl, cval); else __builtin_unreachable(); break;
    default: __builtin_unreachable();
    }
}

// bits of v selected by MASK, packed to the low end (compile time)
template <int MASK>
__device__ __forceinline__ constexpr int pext_c(int v)
{
    int r = 0, i = 0;
    for (int b = 0; b < 8; ++b)
        if ((MASK >> b) & 1) { r |= ((v >> b) & 1) << i; ++i; }
    return r;
}

typedef float floatx16 __attribute__((ext_vector_type(16)));

// Complex64 dense op of K = 4 or 5 of the five register bits on the matrix
// cores.  The wave's 64 * 2^(5-K) vectors of 2^K amplitudes form the columns
// of B; the op is the real product
//     [Re w; Im w] = [[Re U, -Im U], [Im U, Re U]] [Re v; Im v]
// computed by v_mfma_f32_32x32x2f32 (FP32 products, FP32 accumulation) on
// tiles of 32 vectors, with rows and columns interleaved (row 2i + 0/1 = real
// / imaginary part of element i).  The amplitudes travel registers -> the
// wave's own LDS region (S[element][vector]) -> B operands, and the results
// D -> S -> registers.  Operand layouts of the 32x32x2 product: A[i][k] and
// B[k][j] sit in lane i + 32 k (resp. j + 32 k); D[i][j] in lane j + 32 ((i / 4) % 2),
// accumulator 4 (i / 8) + i % 4.  A comes from the plan, already in lane
// order: A[(mb * 2^K + s) * 64 + lane] for row block mb and step s, where
// step s feeds part s % 2 of element 2 (s / 2) + lane / 32.
template <int MASK>
__device__ __forceinline__ void apply_mfma(c64 (&v)[32], const float *__restrict__ A, c64 *__restrict__ S, uint32_t lane)
{
    constexpr int K = __builtin_popcount(MASK);
    constexpr int D = 1 << K;            // elements per vector
    constexpr int NV = 64 << (5 - K);    // vectors of the wave
    constexpr int NMB = D / 16;          // blocks of 32 real rows
    constexpr int NT = NV / 32;          // tiles of 32 vectors
    constexpr int REST = 31 & ~MASK;
#pragma unroll
    for (int m = 0; m < 32; ++m) S[pext_c<MASK>(m) * NV + pext_c<REST>(m) * 64 + lane] = v[m];
    asm volatile("" ::: "memory");       // LDS ops of a wave run in order; keep the compiler from reordering
    float a[NMB][D];
#pragma unroll
    for (int mb = 0; mb < NMB; ++mb)
#pragma unroll
        for (int s = 0; s < D; ++s) a[mb][s] = A[(mb * D + s) * 64 + lane];
    const uint32_t n = lane & 31u, h = lane >> 5;
#pragma unroll
    for (int t = 0; t < NT; ++t) {
        c64 b[D / 2];
#pragma unroll
        for (int u = 0; u < D / 2; ++u) b[u] = S[(2 * u + h) * NV + 32 * t + n];
        floatx16 acc[NMB];
#pragma unroll
        for (int mb = 0; mb < NMB; ++mb)
#pragma unroll
            for (int g = 0; g < 16; ++g) acc[mb][g] = 0.f;
#pragma unroll
        for (int u = 0; u < D / 2; ++u)
#pragma unroll
            for (int mb = 0; mb < NMB; ++mb) {
                acc[mb] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[mb][2 * u], b[u].x, acc[mb], 0, 0, 0);
                acc[mb] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[mb][2 * u + 1], b[u].y, acc[mb], 0, 0, 0);
            }
        // accumulators g, g + 1 (g even) are rows 8 (g / 4) + 4 h + g % 4 and the
        // next one: the real and imaginary parts of one output element
#pragma unroll
        for (int mb = 0; mb < NMB; ++mb)
#pragma unroll
            for (int g = 0; g < 16; g += 2) {
                const uint32_t row = 16 * mb + 4 * (g / 4) + 2 * h + (g % 4) / 2;
                S[row * NV + 32 * t + n] = c64{acc[mb][g], acc[mb][g + 1]};
            }
    }
    asm volatile("" ::: "memory");
#pragma unroll
    for (int m = 0; m < 32; ++m) v[m] = S[pext_c<MASK>(m) * NV + pext_c<REST>(m) * 64 + lane];
}

#define QS_MFMA_CASE(MM)                                                                  \
    case MM:                                                                              \
        if constexpr (__builtin_popcount(MM) <= KMAX) apply_mfma<MM>(v, A, S, lane);      \
        else __builtin_unreachable();                                                     \
        break;

template <int KMAX>
__device__ __forceinline__ void mfma_dispatch(int mask, c64 (&v)[32], const float *__restrict__ A, c64 *__restrict__ S,
                                              uint32_t lane)
{
    switch (mask) {
        QS_MFMA_CASE(15) QS_MFMA_CASE(23) QS_MFMA_CASE(27) QS_MFMA_CASE(29) QS_MFMA_CASE(30) QS_MFMA_CASE(31)
    default:
        __builtin_unreachable();
    }
}
#undef QS_MFMA_CASE

// bits of v selected by mask, packed to the low end (ascending)
__device__ __forceinline__ uint32_t pext_u32(uint32_t v, uint32_t mask)
{
    uint32_t r = 0;
    int i = 0;
    for (int b = 0; b < 16; ++b)
        if ((mask >> b) & 1u) { r |= ((v >> b) & 1u) << i; ++i; }
    return r;
}


// XOR swizzle of an LDS slot (linear, bijective): local bits 4.. fold into
// the low nibble (nibble b-4 of swlo/swhi), bit 3 folds into bits 0-2
// (bits 28-30 of swhi).
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
    if ((l >> 3) & 1u) f ^= (swhi >> 28) & 7u;
    return l ^ f;
}

// Barrier for LDS traffic only: wait for this wave's LDS operations, then
// meet the other waves.  Outstanding global memory operations stay in flight.
__device__ __forceinline__ void lds_barrier()
{
    __builtin_amdgcn_s_waitcnt(0xC07F);   // lgkmcnt(0); vmcnt, expcnt left at their maxima
    __builtin_amdgcn_s_barrier();
}

// Negate an amplitude when bit 31 of sb is set (sign-bit XOR, no arithmetic).
__device__ __forceinline__ void flip(c128 &a, uint32_t sb)
{
    a.x = __longlong_as_double(__double_as_longlong(a.x) ^ ((unsigned long long)sb << 32));
    a.y = __longlong_as_double(__double_as_longlong(a.y) ^ ((unsigned long long)sb << 32));
}
__device__ __forceinline__ void flip(c64 &a, uint32_t sb)
{
    a.x = __uint_as_float(__float_as_uint(a.x) ^ sb);
    a.y = __uint_as_float(__float_as_uint(a.y) ^ sb);
}

// Register offsets from the R physical bit positions: the positions pass
// through an empty asm so the 2^R 64-bit sums are formed next to their use
// rather than hoisted out of the chunk loop (where they would pin registers).
template <int R>
__device__ __forceinline__ void reg_offsets(uint64_t (&o)[1 << R], const int (&pos)[R])
{
    uint64_t b[R];
#pragma unroll
    for (int j = 0; j < R; ++j) {
        int p = pos[j];
        asm volatile("" : "+s"(p));
        b[j] = 1ull << p;
    }
#pragma unroll
    for (int m = 0; m < (1 << R); ++m) {
        uint64_t x = 0;
#pragma unroll
        for (int j = 0; j < R; ++j)
            if ((m >> j) & 1) x |= b[j];
        o[m] = x;
    }
}

// Non-temporal (streaming) global accesses: the state passes through once per pass and
// is far larger than the caches.  Measured per access side: loads always (gate blocks
// 1.4-1.6 % faster), stores for complex128 only (complex128 blocks and swap passes a
// further 1-4 % faster; complex64 blocks 3-4 % slower with streaming stores).
typedef double qs_d2 __attribute__((ext_vector_type(2)));
typedef float qs_f2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ c128 ld_nt(const c128 *p)
{
    const qs_d2 t = __builtin_nontemporal_load(reinterpret_cast<const qs_d2 *>(p));
    c128 r;
    r.x = t.x;
    r.y = t.y;
    return r;
}
__device__ __forceinline__ c64 ld_nt(const c64 *p)
{
    const qs_f2 t = __builtin_nontemporal_load(reinterpret_cast<const qs_f2 *>(p));
    c64 r;
    r.x = t.x;
    r.y = t.y;
    return r;
}
__device__ __forceinline__ void st_nt(c128 *p, const c128 &v)
{
    qs_d2 t;
    t.x = v.x;
    t.y = v.y;
    __builtin_nontemporal_store(t, reinterpret_cast<qs_d2 *>(p));
}
__device__ __forceinline__ void st_nt(c64 *p, const c64 &v)
{
    qs_f2 t;
    t.x = v.x;
    t.y = v.y;
    __builtin_nontemporal_store(t, reinterpret_cast<qs_f2 *>(p));
}

template <int R, typename V>
__device__ __forceinline__ void load_regs(V (&v)[1 << R], const V *__restrict__ amps, uint64_t g, const int (&pos)[R])
{
    uint64_t o[1 << R];
    reg_offsets<R>(o, pos);
#pragma unroll
    for (int m = 0; m < (1 << R); ++m) v[m] = ld_nt(amps + (g | o[m]));
}

// g: the thread's part of the addresses, XOR the store's inversion mask (which may
// cover register positions too, hence XOR with the register offsets)
template <int R, bool NT, typename V>
__device__ __forceinline__ void store_regs(const V (&v)[1 << R], V *__restrict__ amps, uint64_t g, const int (&pos)[R])
{
    uint64_t o[1 << R];
    reg_offsets<R>(o, pos);
#pragma unroll
    for (int m = 0; m < (1 << R); ++m) {
        if constexpr (NT) st_nt(amps + (g ^ o[m]), v[m]);
        else amps[g ^ o[m]] = v[m];
    }
}

// Chunk base: the chunk index spread over the physical qubits outside the chunk
// (a deposit of c's bits into the clear bits of cmask, lowest first; one trip per
// outside qubit, all scalar).
__device__ __forceinline__ uint64_t chunk_base(uint64_t c, uint64_t cmask, int n)
{
    uint64_t base = 0;
    for (uint64_t m = ~cmask & ((n >= 64) ? ~0ull : ((1ull << n) - 1)); m; m &= m - 1, c >>= 1)
        base |= (c & 1ull) << __builtin_ctzll(m);
    return base;
}

// One workgroup per chunk: load the chunk into registers (phase 0 layout),
// run the phases (LDS exchanges between them), store through P_out.  Several
// workgroups share a CU, so one's HBM traffic overlaps another's arithmetic.
// (Persistent workgroups walking a static share of the chunks measured 8-14%
// slower, the plain copy pass included: the dispatcher's dynamic assignment
// balances the XCDs better than a fixed partition.)
// Workgroup size limit: 512 threads when each holds at most 8 amplitudes.
template <int R> struct MaxThreads { static constexpr int value = (R <= 3) ? 512 : 256; };
// Three waves per SIMD (at most 168 registers per lane) wherever 2^R amplitudes
// take at most 64 registers, so that three workgroups with half-buffer
// exchanges share a CU (two for the matrix-core variant, which would spill);
// 32 complex128 amplitudes (128 registers) get the whole register file.
template <int R, typename F, bool MF> struct MinWaves {
    static constexpr int value = (sizeof(F) * 2 << R) <= 256 ? (MF ? 2 : 3) : 1;
};

template <int R, int KMAX, typename F, bool MF>
__global__ __launch_bounds__(MaxThreads<R>::value) __attribute__((amdgpu_waves_per_eu(MinWaves<R, F, MF>::value, MinWaves<R, F, MF>::value)))
void k_block(typename AmpOf<F>::type *__restrict__ amps,
                                              const int *__restrict__ prog, const F *__restrict__ mats, int n)
{
    using V = typename AmpOf<F>::type;
    using CF = __attribute__((address_space(4))) F;
    extern __shared__ unsigned char lds_raw[];
    constexpr int NR = 1 << R;

    const int nph = prog[0];
    const int C = prog[1];
    const int flags = prog[3];
    const int tb = C - R;
    const uint32_t tid = threadIdx.x;
    const int *ph0 = prog + PROG_HDR + 2 * C;

    // the load/store map the planner puts right before the table: what would otherwise be
    // derived from the first and last layouts through chains of dependent scalar loads
    // before the first loads
    const int *__restrict__ mp = prog + prog[4] - kMapWords;
    const uint64_t cmask = (uint64_t)(uint32_t)mp[26] | ((uint64_t)(uint32_t)mp[27] << 32);

    // per-lane data of diagonal ops: staged once into LDS, after the exchange buffer
    // (half the chunk when every exchange of the block runs in two rounds); filled
    // below, after the chunk's loads are issued, so the two latencies overlap
    const bool half = (flags & 4) != 0;
    int *ltab = reinterpret_cast<int *>(lds_raw + ((size_t)sizeof(V) << (half ? C - 1 : C)));

    // global offsets: per thread (VGPR); per register bit j, its physical position when
    // loading and when storing (uniform) -- register offsets are rebuilt from these in every
    // chunk instead of being kept live in 2^R 64-bit registers.  (The two thread loops stay
    // separate, store side first: one joint loop spilled registers in some variants.)
    uint64_t gout_t = 0;
    for (int j = 0; j < tb; ++j) gout_t |= (uint64_t)((tid >> j) & 1u) << mp[28 + j];
    uint64_t gin_t = 0;
    for (int j = 0; j < tb; ++j) gin_t |= (uint64_t)((tid >> j) & 1u) << mp[j];
    int bin[R], bout[R];
#pragma unroll
    for (int j = 0; j < R; ++j) {
        bin[j] = mp[16 + j];
        bout[j] = mp[21 + j];
    }
    const bool hazard = (flags & 2) && nph == 1;

    // XCD-aware order: the dispatcher places workgroup b on XCD b % 8, so each XCD gets a
    // contiguous eighth of the chunk indices, walked in order (neighbouring chunks share
    // address-translation pages and L2 lines)
    const uint64_t nbk = gridDim.x;
    const uint64_t c = (nbk % 8 == 0) ? (uint64_t)(blockIdx.x % 8) * (nbk / 8) + blockIdx.x / 8 : (uint64_t)blockIdx.x;
    {
        V v[NR];
        const uint64_t cbase = chunk_base(c, cmask, n);
        load_regs<R>(v, amps, cbase | gin_t, bin);
        {
            // the table, in 16-byte words (the planner pads it to whole ones and aligns every
            // block's program): one per thread in flight per round trip, four for tables of
            // more than one per thread; the first round outside the loop (a loop header would
            // wait for every load in flight, the chunk's included).  Indices are clamped into
            // the table, so the loads need no per-lane branch; a group of words wholly past
            // the table's end is skipped by a uniform test.
            const int tab_off = prog[4], tab_words = prog[5];
            const int n4 = tab_words >> 2;
            const int nt = (int)blockDim.x;
            typedef int word4 __attribute__((ext_vector_type(4)));
            const word4 *__restrict__ P4 = reinterpret_cast<const word4 *>(prog + tab_off);
            word4 *L4 = reinterpret_cast<word4 *>(ltab);
            auto stage = [&](int b0, auto kgroups) __attribute__((always_inline)) {
                constexpr int K = decltype(kgroups)::value;
                word4 t[K];
#pragma unroll
                for (int k = 0; k < K; ++k)
                    if (K == 1 || b0 + k * nt < n4) t[k] = P4[min(b0 + k * nt + (int)tid, n4 - 1)];
#pragma unroll
                for (int k = 0; k < K; ++k) {
                    const int i = b0 + k * nt + (int)tid;
                    if (i < n4) L4[i] = t[k];
                }
            };
            if (n4) {
                if (n4 <= nt) {
                    stage(0, std::integral_constant<int, 1>());
                } else {
                    stage(0, std::integral_constant<int, 4>());
                    for (int b0 = 4 * nt; b0 < n4; b0 += 4 * nt) stage(b0, std::integral_constant<int, 4>());
                }
                __builtin_amdgcn_s_waitcnt(0xC07F);   // lgkmcnt(0): the table writes are done
                __builtin_amdgcn_s_barrier();
            }
        }
        if (hazard) {
            // the write-back permutes positions and no exchange orders loads before
            // stores: every wave must hold its part of the chunk before any store
            __builtin_amdgcn_s_waitcnt(0);
            __builtin_amdgcn_s_barrier();
        }
        const int *ph = ph0;
        const int *prev = nullptr;
        for (int p = 0; p < nph; ++p) {
            const int nops = ph[0];
            const int *Rb = ph + PHASE_HDR;
            const int *T = Rb + R;
            const int *X = T + tb;                 // exchange block of this phase
            if (p > 0) {
                // ---- exchange from the previous layout to this one through LDS
                // XOR of the contributions of the thread's set bits, branch-free: a
                // per-lane condition around the loads makes the compiler issue and wait
                // for them one at a time
                uint32_t wt = 0, rt = 0;
                const int xt = ph[3] & 0xffffff;
                // half-buffer rounds: thread positions of the split bit in the write and the
                // read layout (-1: one round through the whole buffer)
                const uint32_t hx = (uint32_t)ph[3] >> 24;
                const int hjw = (int)(hx & 15u) - 1, hjr = (int)(hx >> 4) - 1;
                if (xt > 0) {
                    // per-nibble XOR tables of the same words, staged in LDS
                    const int *Xl = ltab + (xt - 1);
                    const uint32_t n0 = tid & 15u, n1 = (tid >> 4) & 15u, n2 = (tid >> 8) & 1u;
                    wt = (uint32_t)Xl[n0] ^ (uint32_t)Xl[16 + n1] ^ (uint32_t)Xl[32 + n2];
                    rt = (uint32_t)Xl[kNibWords + n0] ^ (uint32_t)Xl[kNibWords + 16 + n1] ^
                         (uint32_t)Xl[kNibWords + 32 + n2];
                } else {
                    for (int j = 0; j < tb; ++j) {
                        const uint32_t sel = 0u - ((tid >> j) & 1u);
                        wt ^= (uint32_t)X[j] & sel;
                        rt ^= (uint32_t)X[tb + j] & sel;
                    }
                }
                const int *wo = X + 2 * tb;
                const int *ro = wo + NR;
                if (hjw < 0) {
                    lds_barrier();      // previous readers of the buffer are done
#pragma unroll
                    for (int m = 0; m < NR; ++m) *reinterpret_cast<V *>(lds_raw + (wt ^ (uint32_t)wo[m])) = v[m];
                    lds_barrier();      // every write is visible
#pragma unroll
                    for (int m = 0; m < NR; ++m) v[m] = *reinterpret_cast<const V *>(lds_raw + (rt ^ (uint32_t)ro[m]));
                } else if (hjw >= 6) {
                    // two rounds through half the buffer, the split bit a wave-index bit: a whole
                    // wave writes and reads in one round (uniform branch, four barriers for every
                    // wave); each side redefines all its registers from LDS, so no register
                    // copies merge the two sides
                    const uint32_t wave = __builtin_amdgcn_readfirstlane(tid >> 6);
                    const bool first = ((wave >> (hjw - 6)) & 1u) == 0;
                    lds_barrier();
                    if (first) {
#pragma unroll
                        for (int m = 0; m < NR; ++m) *reinterpret_cast<V *>(lds_raw + (wt ^ (uint32_t)wo[m])) = v[m];
                        lds_barrier();
#pragma unroll
                        for (int m = 0; m < NR; ++m) v[m] = *reinterpret_cast<const V *>(lds_raw + (rt ^ (uint32_t)ro[m]));
                        lds_barrier();
                        lds_barrier();
                    } else {
                        lds_barrier();
                        lds_barrier();
#pragma unroll
                        for (int m = 0; m < NR; ++m) *reinterpret_cast<V *>(lds_raw + (wt ^ (uint32_t)wo[m])) = v[m];
                        lds_barrier();
#pragma unroll
                        for (int m = 0; m < NR; ++m) v[m] = *reinterpret_cast<const V *>(lds_raw + (rt ^ (uint32_t)ro[m]));
                    }
                } else {
                    // two rounds through half the buffer: the threads whose bit hjw (= hjr, the
                    // planner keeps the split bit at one position) is h hold exactly the
                    // amplitudes of half h, before and after; each writes, then reads
                    const uint32_t mw = (tid >> hjw) & 1u, mr = (tid >> hjr) & 1u;
                    for (uint32_t h = 0; h < 2; ++h) {
                        lds_barrier();
                        if (mw == h) {
#pragma unroll
                            for (int m = 0; m < NR; ++m)
                                *reinterpret_cast<V *>(lds_raw + (wt ^ (uint32_t)wo[m])) = v[m];
                        }
                        lds_barrier();
                        if (mr == h) {
#pragma unroll
                            for (int m = 0; m < NR; ++m)
                                v[m] = *reinterpret_cast<const V *>(lds_raw + (rt ^ (uint32_t)ro[m]));
                        }
                    }
                }
            }
            // ---- ops of this phase
            const int *op = X + 2 * tb + 2 * NR;
            // one op: its kind and register mask select a compile-time code path
            auto run_op = [&](const int *__restrict__ op) __attribute__((always_inline)) {
                const int w0 = op[0];
                const int kind = w0 & 0xff;
                const int variant = (w0 >> 8) & 0xff;
                const int k = (w0 >> 16) & 0xff;
                // uniform across the workgroup: keep the coefficient address scalar
                const uint32_t mlo = __builtin_amdgcn_readfirstlane((uint32_t)op[1]);
                const uint32_t mhi = __builtin_amdgcn_readfirstlane((uint32_t)op[2]);
                // read through the constant address space: uniform loads of coefficients
                // become scalar (SMEM) loads instead of per-lane vector loads
                const CF *M = (const CF *)(uintptr_t)(mats + ((int64_t)mlo | ((int64_t)mhi << 32)));
                // KMAX == 0: a block of rotations and diagonals only (no dense paths
                // compiled in: less code and fewer registers)
                // (the order of these tests matters: a no-op test ahead of the others cost about
                // 5% of the pass, with the same instruction counts)
                if (kind == OP_MULTI1) {
                    if constexpr (KMAX > 0) multi1_dispatch<R, F, V, const CF *>(variant, v, M);
                    else __builtin_unreachable();
                } else if (kind == OP_MCX) {
                    mcx_dispatch<R, KMAX == 0, V>(variant, __builtin_amdgcn_readfirstlane((uint32_t)op[3]), v);
                } else if (kind == OP_ROT || kind == OP_ROTD) {
                    // one copy of the rotation paths for both kinds (code size)
                    rot_dispatch<R, F, V, const CF *>(variant, v, M);
                    if (kind == OP_ROTD) {
                        const CF *D = M + 2 * __builtin_popcount((uint32_t)variant);
#pragma unroll
                        for (int m = 0; m < NR; ++m) v[m] = cmul<F, V>(D[2 * m], D[2 * m + 1], v[m]);
                    }
                } else if (kind == OP_DENSE) {
                    if constexpr (KMAX > 0) dense_dispatch<R, KMAX, F, V, const CF *>(variant, v, M);
                    else __builtin_unreachable();
                } else if (kind == OP_SIGN_ROW) {
                    const uint32_t row = pext_u32(tid, (uint32_t)op[1]);
                    const uint32_t s = (uint32_t)ltab[op[3] + row];
#pragma unroll
                    for (int m = 0; m < NR; ++m) flip(v[m], (s << (31 - m)) & 0x80000000u);
                } else if (kind == OP_SIGN_REG) {
                    const uint32_t s = (uint32_t)op[3];
#pragma unroll
                    for (int m = 0; m < NR; ++m) flip(v[m], (s << (31 - m)) & 0x80000000u);
                } else if (kind == OP_DIAG_REG) {
#pragma unroll
                    for (int m = 0; m < NR; ++m) v[m] = cmul<F, V>(M[2 * m], M[2 * m + 1], v[m]);
                } else if (kind == OP_MFMA) {
                    if constexpr (MF && R == 5 && std::is_same<F, float>::value) {
                        // the wave works in its own 16 KiB of the exchange buffer; other
                        // waves may still be reading this phase's exchange slots there
                        lds_barrier();
                        const float *A = mats + ((int64_t)mlo | ((int64_t)mhi << 32));
                        mfma_dispatch<5>(variant, v, A, reinterpret_cast<c64 *>(lds_raw) + (tid >> 6) * (64 * 32),
                                            tid & 63u);
                    } else {
                        __builtin_unreachable();
                    }
                } else if (kind == OP_NOP) {
                    // padding: nothing
                } else {   // this lane's row of the op's table (LDS, or device memory)
                    const uint32_t row = pext_u32(tid, (uint32_t)op[1]);
                    // the row holds entries over the op's register bits only: register m
                    // takes entry pext(m, rmask); per register bit j the (uniform) byte
                    // stride of the entry index
                    const uint32_t rm = (uint32_t)variant >> 1;
                    const uint32_t kr = __builtin_popcount(rm);
                    uint32_t stride[R];
#pragma unroll
                    for (int j = 0; j < R; ++j)
                        stride[j] = ((rm >> j) & 1u) ? (uint32_t)sizeof(V) << __builtin_popcount(rm & ((1u << j) - 1u)) : 0u;
                    auto apply_row = [&](const unsigned char *__restrict__ E) __attribute__((always_inline)) {
#pragma unroll
                        for (int m = 0; m < NR; ++m) {
                            uint32_t off = 0;
#pragma unroll
                            for (int j = 0; j < R; ++j)
                                if ((m >> j) & 1) off += stride[j];
                            const V e = *reinterpret_cast<const V *>(E + off);
                            v[m] = cmul<F, V>(e.x, e.y, v[m]);
                            // keep at most four table reads in flight (register pressure)
                            if ((m & 3) == 3) __builtin_amdgcn_sched_barrier(0);
                        }
                    };
                    // two separate paths, so the LDS one is plain LDS reads (a pointer that
                    // may be either would become flat loads, waited on with the memory counter)
                    if (variant & 1)
                        apply_row(reinterpret_cast<const unsigned char *>(
                                      mats + ((int64_t)(uint32_t)op[2] | ((int64_t)op[3] << 32))) +
                                  ((size_t)row * sizeof(V) << kr));
                    else
                        apply_row(reinterpret_cast<const unsigned char *>(ltab + op[3]) + ((size_t)row * sizeof(V) << kr));
                }
            };
            if constexpr (KMAX == 0) {
                // blocks of rotations and diagonals (small code): two ops per trip, so
                // that results alternate between two register sets instead of being
                // copied back into one after every op (phases hold an even op count)
                for (int o = 0; o < nops; o += 2, op += 2 * OP_WORDS) {
                    run_op(op);
                    run_op(op + OP_WORDS);
                }
            } else {
                for (int o = 0; o < nops; ++o, op += OP_WORDS) run_op(op);
            }
            prev = ph;
            ph = op;
        }
        // ---- store in the last layout, through P_out
        const uint64_t inv = (uint64_t)(uint32_t)prog[6] | ((uint64_t)(uint32_t)prog[7] << 32);
        store_regs<R, std::is_same<F, double>::value>(v, amps, (cbase | gout_t) ^ inv, bout);
    }
}

template <int R, int KMAX, typename F, bool MF>
hipError_t launch_RK(qs_state *st, const int *d_prog, const F *d_mats, int C, size_t tab_bytes, bool half)
{
    using V = typename AmpOf<F>::type;
    const size_t lds = ((size_t)1 << (half ? C - 1 : C)) * sizeof(V) + ((tab_bytes + 15) & ~(size_t)15);
    if (lds > 160u * 1024u) return hipErrorInvalidValue;
    auto kern = k_block<R, KMAX, F, MF>;
    // the LDS limit is raised once per device (devices numbered below 64), under a lock
    static std::mutex mu;
    static uint64_t done = 0;
    {
        int dev = 0;
        hipError_t e = hipGetDevice(&dev);
        if (e != hipSuccess) return e;
        std::lock_guard<std::mutex> g(mu);
        if (dev >= 64 || !((done >> dev) & 1u)) {
            e = hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
            if (e != hipSuccess) return e;
            if (dev < 64) done |= 1ull << dev;
        }
    }
    const unsigned threads = 1u << (C - R);
    const uint64_t nchunks = 1ull << (st->n - C);
    hipLaunchKernelGGL(kern, dim3((unsigned)nchunks), dim3(threads), lds, st->stream,
                       reinterpret_cast<V *>(st->amps), d_prog, d_mats, st->n);
    return hipGetLastError();
}

// Kernel variant by the widest vector dense op of the block (none -- rotations
// and diagonals only --, 2, 3 or R register bits; fewer compiled-in cases keep
// register pressure and with it occupancy in check), plus the matrix-core
// variant for complex64 blocks with 4-5-qubit ops (vector ops up to 3 bits
// beside them).
template <int R, typename F>
hipError_t launch_R(qs_state *st, const int *d_prog, const F *d_mats, int C, size_t tab, int kmax, bool mfma, bool half)
{
    // half-buffer exchanges exist only outside the matrix-core variant
    if (half && mfma) return hipErrorInvalidValue;
    if constexpr (R == 5 && std::is_same<F, float>::value) {
        if (mfma) return launch_RK<5, 3, float, true>(st, d_prog, d_mats, C, tab, false);
    }
    if (mfma) return hipErrorInvalidValue;
    if (kmax == 0) return launch_RK<R, 0, F, false>(st, d_prog, d_mats, C, tab, half);
    if (kmax <= 2 || R <= 2) return launch_RK<R, (R < 2 ? R : 2), F, false>(st, d_prog, d_mats, C, tab, half);
    if (kmax == 3 || R == 3) return launch_RK<R, 3, F, false>(st, d_prog, d_mats, C, tab, half);
    return launch_RK<R, R, F, false>(st, d_prog, d_mats, C, tab, half);
}

template <typename F>
hipError_t launch_F(qs_state *st, int r, const int *d_prog, const F *d_mats, int C, size_t tab, int kmax, bool mfma,
                    bool half)
{
    switch (r) {
    case 1: return launch_R<1, F>(st, d_prog, d_mats, C, tab, kmax, mfma, half);
    case 2: return launch_R<2, F>(st, d_prog, d_mats, C, tab, kmax, mfma, half);
    case 3: return launch_R<3, F>(st, d_prog, d_mats, C, tab, kmax, mfma, half);
    case 4: return launch_R<4, F>(st, d_prog, d_mats, C, tab, kmax, mfma, half);
    case 5: return launch_R<5, F>(st, d_prog, d_mats, C, tab, kmax, mfma, half);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace

hipError_t launch_block_prog(qs_state *st, int r, int C, const int *d_prog, const void *d_mats, size_t tab_bytes,
                             int kmax_dense, bool mfma, bool half)
{
    if (C < r || st->n < C || (1 << (C - r)) > (r <= 3 ? 512 : 256)) return hipErrorInvalidValue;
    // matrix-core ops stage each wave's amplitudes in its own slice of the chunk buffer
    if (mfma && (st->dtype != QS_C64 || r != 5 || C - r < 6)) return hipErrorInvalidValue;
    if (st->dtype == QS_C64)
        return launch_F<float>(st, r, d_prog, reinterpret_cast<const float *>(d_mats), C, tab_bytes, kmax_dense, mfma,
                               half);
    return launch_F<double>(st, r, d_prog, reinterpret_cast<const double *>(d_mats), C, tab_bytes, kmax_dense, mfma,
                            half);
}

hipError_t launch_block(qs_state *st, const Plan &p, const void *d_prog, const void *d_mats, int b)
{
    const int *prog = reinterpret_cast<const int *>(d_prog) + p.prog_off[b];
    const size_t tab_bytes = (size_t)p.h_prog[p.prog_off[b] + 5] * 4;
    const bool half = (p.h_prog[p.prog_off[b] + 3] & 4) != 0;
    return launch_block_prog(st, p.r, p.C, prog, d_mats, tab_bytes, p.block_kmax[b], p.block_mfma[b] != 0, half);
}

}  // namespace qs
