// planner.cpp -- host planner of libqs: gate-block finding with qubit-reorder
// swaps, fusion inside blocks, and register-phase scheduling.
//
// Paper: Sec. IV (Eq. 5-7, Alg. 1 findGBs, Alg. 2 all-in-one optimisation).
//   Level "cache" (Alg. 2, second level): gate blocks whose qubits fit in a
//   chunk of C qubits (Eq. 5); blocks partition the gate list (Eq. 6); the
//   objective is few blocks, i.e. many gates per block (Eq. 7).  Here a
//   chunk is not the C lowest qubits but the L lowest physical qubits plus
//   any C-L others, gathered as 2^(C-L) runs of 2^L contiguous amplitudes,
//   so a block can cover high qubits without a swap pass.
//   Qubit reordering (Sec. II-B Eq. 4, Sec. V-B): a block may write its chunk
//   back with its bits permuted ("folded" swap, free), choosing which logical
//   qubits occupy the always-resident low positions for the next blocks;
//   standalone permutation passes restore canonical order at the end.
//   Level "fusion" (Alg. 2, third level): inside a block, gates are merged
//   into unitaries of at most kmax qubits (composed in FP64) when that does
//   not raise the arithmetic per amplitude; diagonal gates merge into one
//   diagonal (the paper's "D4" ops).
//   Register phases (Sec. V-A "multiple states per thread"): each block is
//   cut into phases; in a phase every thread keeps 2^r amplitudes whose
//   local indices differ in r chosen chunk bits, and every dense op of the
//   phase acts on those bits only, so it runs from registers.
#include <algorithm>
#include <array>
#include <chrono>
#include <cmath>
#include <cstring>
#include <numeric>
#include <sstream>
#include <stdexcept>
#include <string>

#include "qs_internal.h"

namespace qs {

namespace {

struct GateIn {
    int k;
    int t[5];
    std::vector<cplx> m;   // circuit convention: index bit (k-1-j) <-> t[j]
    bool diag;
};

bool matrix_is_diag(const std::vector<cplx> &m, int d)
{
    for (int r = 0; r < d; ++r)
        for (int c = 0; c < d; ++c)
            if (r != c && m[r * d + c] != cplx(0, 0)) return false;
    return true;
}

int popc(uint32_t x) { return __builtin_popcount(x); }

// X G X for X on the circuit index bits fl of the gate: every row and column index
// XOR fl (a diagonal stays diagonal, a permutation a permutation).
GateIn conjugate_x(const GateIn &G, uint32_t fl)
{
    GateIn r = G;
    const int d = 1 << G.k;
    for (int i = 0; i < d; ++i)
        for (int j = 0; j < d; ++j) r.m[(size_t)i * d + j] = G.m[(size_t)(i ^ fl) * d + (j ^ fl)];
    return r;
}

// ---------------------------------------------------------------------------
// Gate-block finding (Alg. 1 behaviour)
// ---------------------------------------------------------------------------
struct Blocker {
    const std::vector<GateIn> &g;
    int n;
    std::vector<int> stamp;   // per qubit: == cur -> blocked in this scan
    int cur = 0;

    Blocker(const std::vector<GateIn> &gates, int nq) : g(gates), n(nq), stamp(nq, 0) {}

    // Number of remaining gates executable in order with qubit set inS;
    // optionally collects them.  A gate that cannot run blocks its qubits.
    int count(const std::vector<int> &rem, const std::vector<char> &inS, int nS, std::vector<int> *take)
    {
        ++cur;
        int cnt = 0, nblockedS = 0;
        for (int idx : rem) {
            const GateIn &G = g[idx];
            bool ok = true;
            for (int j = 0; j < G.k; ++j) {
                int q = G.t[j];
                if (!inS[q] || stamp[q] == cur) { ok = false; break; }
            }
            if (ok) {
                ++cnt;
                if (take) take->push_back(idx);
            } else {
                for (int j = 0; j < G.k; ++j) {
                    int q = G.t[j];
                    if (stamp[q] != cur) {
                        stamp[q] = cur;
                        if (inS[q]) ++nblockedS;
                    }
                }
                if (nblockedS == nS) break;
            }
        }
        return cnt;
    }
};

// Greedy choice of the chunk's logical qubit set S (|S| = C) containing the
// forced set F, maximising the number of executable gates; then a
// one-exchange local search.
std::vector<char> choose_chunk(Blocker &B, const std::vector<int> &rem, const std::vector<int> &forced, int C,
                               int n)
{
    std::vector<char> inS(n, 0);
    int nS = 0;
    for (int q : forced) { inS[q] = 1; ++nS; }
    // first pending gate index per qubit (tie-break: earlier is better)
    std::vector<int> first(n, 1 << 30);
    for (size_t i = 0; i < rem.size(); ++i) {
        const GateIn &G = B.g[rem[i]];
        for (int j = 0; j < G.k; ++j) first[G.t[j]] = std::min(first[G.t[j]], (int)i);
    }
    while (nS < C) {
        int best = -1, bestc = -1, bestf = 1 << 30;
        for (int q = 0; q < n; ++q) {
            if (inS[q]) continue;
            inS[q] = 1;
            int c = B.count(rem, inS, nS + 1, nullptr);
            inS[q] = 0;
            if (c > bestc || (c == bestc && first[q] < bestf)) { best = q; bestc = c; bestf = first[q]; }
        }
        inS[best] = 1;
        ++nS;
    }
    // local search: exchange one free member with one outsider while it helps
    std::vector<char> isF(n, 0);
    for (int q : forced) isF[q] = 1;
    int curc = B.count(rem, inS, nS, nullptr);
    for (int round = 0; round < 2; ++round) {
        bool improved = false;
        for (int a = 0; a < n && !improved; ++a) {
            if (!inS[a] || isF[a]) continue;
            for (int b = 0; b < n; ++b) {
                if (inS[b]) continue;
                inS[a] = 0; inS[b] = 1;
                int c = B.count(rem, inS, nS, nullptr);
                if (c > curc) { curc = c; improved = true; break; }
                inS[a] = 1; inS[b] = 0;
            }
        }
        if (!improved) break;
    }
    return inS;
}

// ---------------------------------------------------------------------------
// Matrices on sets of local bits.  A "set op" holds a matrix whose index bit
// i corresponds to the i-th lowest bit of `mask` (a mask of chunk bits).
// ---------------------------------------------------------------------------
struct SetOp {
    bool diag = false;
    bool rot = false;            // real plane rotations (one per bit of mask); m = their dense matrix when one bit
    int perm = 0;                // permutation without arithmetic: 1 = multi-controlled X on bit ptarget (the
                                 // other bits of mask control), 2 = SWAP of the two bits of mask; m = its matrix
    int ptarget = -1;
    uint32_t pcval = 0;          // perm 1: the values its controls must hold (local bits)
    bool pin = false;            // diagonal split off a single-qubit gate: runs only while its bits are in registers
    uint32_t mask = 0;           // local chunk bits
    std::vector<cplx> m;         // dense: d*d; diag: d
    std::vector<std::array<double, 3>> rots;   // rot: (local bit, beta, alpha) of the shears of each bit
    std::vector<int> gate_ids;
};

int pext(uint32_t v, uint32_t mask)
{
    int r = 0, i = 0;
    for (int b = 0; b < 32; ++b)
        if (mask >> b & 1) { r |= (int)((v >> b) & 1) << i; ++i; }
    return r;
}
uint32_t pdep(int v, uint32_t mask)
{
    uint32_t r = 0;
    int i = 0;
    for (int b = 0; b < 32; ++b)
        if (mask >> b & 1) { r |= (uint32_t)((v >> i) & 1) << b; ++i; }
    return r;
}

// Dense matrix of op on mask U (U must contain op.mask).
std::vector<cplx> embed_dense(const SetOp &op, uint32_t U)
{
    int dU = 1 << popc(U);
    std::vector<cplx> out((size_t)dU * dU, cplx(0, 0));
    int d = 1 << popc(op.mask);
    uint32_t rest = U & ~op.mask;
    for (int u = 0; u < dU; ++u) {
        uint32_t gu = pdep(u, U);
        int ru = pext(gu, op.mask);
        for (int v = 0; v < dU; ++v) {
            uint32_t gv = pdep(v, U);
            if ((gu & rest) != (gv & rest)) continue;
            int rv = pext(gv, op.mask);
            if (op.diag) {
                if (ru == rv) out[(size_t)u * dU + v] = op.m[ru];
            } else {
                out[(size_t)u * dU + v] = op.m[(size_t)ru * d + rv];
            }
        }
    }
    (void)d;
    return out;
}

std::vector<cplx> matmul(const std::vector<cplx> &A, const std::vector<cplx> &B, int d)
{
    std::vector<cplx> C((size_t)d * d, cplx(0, 0));
    for (int i = 0; i < d; ++i)
        for (int k = 0; k < d; ++k) {
            cplx a = A[(size_t)i * d + k];
            if (a == cplx(0, 0)) continue;
            for (int j = 0; j < d; ++j) C[(size_t)i * d + j] += a * B[(size_t)k * d + j];
        }
    return C;
}

// later o applied after earlier e: result = o * e on the union.
SetOp compose(const SetOp &e, const SetOp &o)
{
    SetOp r;
    r.mask = e.mask | o.mask;
    r.gate_ids = e.gate_ids;
    r.gate_ids.insert(r.gate_ids.end(), o.gate_ids.begin(), o.gate_ids.end());
    if (e.diag && o.diag) {
        r.diag = true;
        r.pin = e.pin || o.pin;
        int d = 1 << popc(r.mask);
        r.m.resize(d);
        for (int u = 0; u < d; ++u) {
            uint32_t gu = pdep(u, r.mask);
            r.m[u] = o.m[pext(gu, o.mask)] * e.m[pext(gu, e.mask)];
        }
        return r;
    }
    r.diag = false;
    int d = 1 << popc(r.mask);
    r.m = matmul(embed_dense(o, r.mask), embed_dense(e, r.mask), d);
    return r;
}

// Relative cost of an op per amplitude (vector FMA units).  With matrix cores
// (complex64, k >= 4) a dense op runs at twice the vector rate plus an LDS
// round trip of the wave's amplitudes.
double op_cost(bool diag, int k, bool mfma = false)
{
    if (diag) return 5.0;
    if (mfma && k >= 4) return 2.0 * (double)(1 << k) + 8.0;
    return 4.0 * (double)(1 << k);
}
// a real rotation by two shears: two FMAs per amplitude (real and imaginary parts)
constexpr double kRotCost = 2.0;
// a permutation op: register moves only
constexpr double kPermCost = 0.25;

// Single-qubit gate U as diag(p) * Rot(theta) * diag(q), Rot = [[c, -s], [s, c]],
// c = cos theta, s = sin theta, theta in [0, pi/2] (the phases absorb every sign):
// c = |u00|, s = |u10|, q = (1, q1), p0 = u00 / c, p1 = u10 / s, q1 = -u01 / (p0 s).
// The rotation runs as two shears after a scaling that joins the phase before it:
//     Rot(theta) = [[1, 0], [t, 1]] [[1, -s c], [0, 1]] diag(c, 1 / c),   t = s / c,
// i.e. x0 += (-s c) x1, then x1 += t x0, each one FMA per real component, in place.
// 1 / c stays small only for theta <= pi/4; for a larger angle the gate is taken as
// X * U' with U' = X U (rows swapped, angle pi/2 - theta) and the X is left pending:
// the caller carries it forward (later gates on the bit are conjugated by X; the chunk
// is stored with the bit inverted), so every rotation has c >= 1/sqrt 2, t <= 1 and
// s c <= 1/2.  Outputs: pre = q scaled by (c, 1/c), post = p, (beta, alpha) = (-s c, t),
// *rot = the matrix of the two shears, *flip = whether the X is pending.  Accepted only
// when the factors reproduce U to 1e-14 (a non-unitary matrix stays a dense gate);
// diagonal gates (s = 0) never come here.
bool split_rotation(const std::vector<cplx> &u_in, cplx *pre, cplx *post, double *beta, double *alpha,
                    std::vector<cplx> *rot, bool *flip)
{
    std::vector<cplx> u = u_in;
    *flip = std::abs(u_in[2]) > std::abs(u_in[0]);
    if (*flip) u = {u_in[2], u_in[3], u_in[0], u_in[1]};
    const cplx u00 = u[0], u01 = u[1], u10 = u[2];
    const double theta = std::atan2(std::abs(u10), std::abs(u00));
    const double c = std::cos(theta), s = std::sin(theta);
    if (!(s > 1e-6)) return false;
    const cplx p0 = u00 / std::abs(u00);
    const cplx p1 = u10 / std::abs(u10);
    const cplx q1 = -u01 * std::conj(p0) / s;
    if (std::abs(std::abs(q1) - 1.0) > 1e-14) return false;
    const double t = s / c, b = -s * c;
    // shears times scaling: [[c, b / c], [t c, (t b + 1) / c]] = [[c, -s], [s, c]]
    const cplx shear[4] = {cplx(1, 0), cplx(b, 0), cplx(t, 0), cplx(t * b + 1.0, 0)};
    const cplx sc[2] = {cplx(c, 0), q1 / c};
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j) {
            const cplx rec = (i ? p1 : p0) * shear[2 * i + j] * sc[j];
            if (std::abs(rec - u[2 * i + j]) > 1e-14) return false;
        }
    pre[0] = sc[0];
    pre[1] = sc[1];
    post[0] = p0;
    post[1] = p1;
    *beta = b;
    *alpha = t;
    *rot = {shear[0], shear[1], shear[2], shear[3]};
    return true;
}

// A dense set op whose matrix is exactly a multi-controlled X (X, CX, CCX: flip one
// bit where every other bit of the op holds a given value, 1 or 0 per control) or a
// SWAP of its two bits becomes a permutation op: the kernel moves registers and does
// no arithmetic.
void classify_perm(SetOp *s)
{
    const int k = popc(s->mask), d = 1 << k;
    if (k > 3) return;
    auto matches = [&](auto f) {
        for (int r = 0; r < d; ++r)
            for (int c = 0; c < d; ++c)
                if (s->m[(size_t)r * d + c] != cplx(f(c) == r ? 1.0 : 0.0, 0.0)) return false;
        return true;
    };
    for (int t = 0; t < k; ++t) {
        const int ctrl = (d - 1) & ~(1 << t);
        for (int cv = ctrl;; cv = (cv - 1) & ctrl) {    // control values, all-ones first
            if (matches([&](int c) { return (c & ctrl) == cv ? c ^ (1 << t) : c; })) {
                s->perm = 1;
                s->ptarget = __builtin_ctz(pdep(1 << t, s->mask));
                s->pcval = pdep(cv, s->mask);
                return;
            }
            if (cv == 0) break;
        }
    }
    if (k == 2 && matches([](int c) { return ((c & 1) << 1) | ((c >> 1) & 1); })) s->perm = 2;
}

// Convert a circuit gate to a set op over local bits (loc[j] = local bit of t[j]).
SetOp gate_to_setop(const GateIn &G, const int *loc, int gid)
{
    SetOp s;
    s.diag = G.diag;
    s.gate_ids.push_back(gid);
    for (int j = 0; j < G.k; ++j) s.mask |= 1u << loc[j];
    int d = 1 << G.k;
    // circuit index bit (k-1-j) <-> t[j] <-> local bit loc[j]; set-op index bit i <-> i-th lowest local bit
    auto conv = [&](int ci) {
        uint32_t g = 0;
        for (int j = 0; j < G.k; ++j)
            if ((ci >> (G.k - 1 - j)) & 1) g |= 1u << loc[j];
        return pext(g, s.mask);
    };
    std::vector<int> map(d);
    for (int ci = 0; ci < d; ++ci) map[ci] = conv(ci);
    if (s.diag) {
        s.m.assign(d, cplx(0, 0));
        for (int ci = 0; ci < d; ++ci) s.m[map[ci]] = G.m[(size_t)ci * d + ci];
    } else {
        s.m.assign((size_t)d * d, cplx(0, 0));
        for (int r = 0; r < d; ++r)
            for (int c = 0; c < d; ++c) s.m[(size_t)map[r] * d + map[c]] = G.m[(size_t)r * d + c];
        classify_perm(&s);
    }
    return s;
}

// ---------------------------------------------------------------------------
// Register phases for one block
// ---------------------------------------------------------------------------
struct PhaseSched {
    int C, r, L, kmax;
    bool fuse;
    bool mfma;      // dense ops of k >= 4 run on matrix cores

    // count executable ops with register set Rmask; dense ops (and diagonals split
    // off single-qubit gates) need their bits in registers.  An op that cannot run
    // blocks its bits for later ops, except that diagonals commute with each other:
    // a diagonal left behind blocks only non-diagonal ops.
    int count(const std::vector<SetOp> &rem, uint32_t Rmask, std::vector<int> *take) const
    {
        uint32_t blocked = 0, blocked_diag = 0;
        int cnt = 0;
        for (size_t i = 0; i < rem.size(); ++i) {
            const SetOp &o = rem[i];
            const bool in_regs = (o.mask & ~Rmask) == 0;
            const bool ok = o.diag ? !(o.mask & blocked) && (!o.pin || in_regs)
                                   : !(o.mask & (blocked | blocked_diag)) && in_regs;
            if (ok) {
                ++cnt;
                if (take) take->push_back((int)i);
            } else if (o.diag) {
                blocked_diag |= o.mask;
            } else {
                blocked |= o.mask;
            }
        }
        return cnt;
    }

    uint32_t choose_R(const std::vector<SetOp> &rem, uint32_t allowed) const
    {
        uint32_t R = 0;
        int nR = 0;
        // earliest pending dense op's bits as tie-break order
        std::vector<int> first(C, 1 << 30);
        for (size_t i = 0; i < rem.size(); ++i)
            if (!rem[i].diag)
                for (int b = 0; b < C; ++b)
                    if (rem[i].mask >> b & 1) first[b] = std::min(first[b], (int)i);
        int avail = popc(allowed);
        int want = std::min(r, avail);
        while (nR < want) {
            int best = -1, bestc = -1, bestf = 1 << 30;
            for (int b = 0; b < C; ++b) {
                if (!(allowed >> b & 1) || (R >> b & 1)) continue;
                int c = count(rem, R | (1u << b), nullptr);
                if (c > bestc || (c == bestc && first[b] < bestf)) { best = b; bestc = c; bestf = first[b]; }
            }
            R |= 1u << best;
            ++nR;
        }
        return R;
    }

    // Register set for the next phase by a two-phase lookahead: every r-subset
    // of the allowed bits is scored by the ops it runs now plus the most the
    // best following phase could run (over the 12 best first choices); a set
    // that finishes the block scores highest, more so when it keeps clear of
    // the bits the write-back puts at the low physical positions (which would
    // need an extra store phase).  Falls back to the greedy choice when the
    // subsets are too many.  Fewer phases = fewer LDS exchanges.
    uint32_t choose_R_search(const std::vector<SetOp> &rem, uint32_t allowed, uint32_t all, uint32_t avoid_last) const
    {
        const int want = std::min(r, popc(allowed));
        auto subsets = [&](uint32_t from, int k) {
            std::vector<int> pos;
            for (int b = 0; b < C; ++b)
                if (from >> b & 1) pos.push_back(b);
            std::vector<uint32_t> out;
            const int m = (int)pos.size();
            if (k <= 0 || k > m) return out;
            for (uint32_t sel = (1u << k) - 1; sel < (1u << m);) {
                uint32_t R = 0;
                for (int i = 0; i < m; ++i)
                    if (sel >> i & 1) R |= 1u << pos[i];
                out.push_back(R);
                const uint32_t t = sel | (sel - 1);   // next subset with k bits (Gosper)
                sel = (t + 1) | (((~t & (t + 1)) - 1) >> (__builtin_ctz(sel) + 1));
            }
            return out;
        };
        std::vector<uint32_t> s1 = subsets(allowed, want);
        if (s1.empty() || s1.size() > 1000) return choose_R(rem, allowed);
        std::vector<std::pair<int, uint32_t>> c1;
        for (uint32_t R : s1) c1.push_back({count(rem, R, nullptr), R});
        std::stable_sort(c1.begin(), c1.end(), [](const std::pair<int, uint32_t> &a, const std::pair<int, uint32_t> &b) {
            return a.first > b.first;
        });
        const std::vector<uint32_t> s2 = subsets(all, std::min(r, popc(all)));
        const long long FINISH = 1ll << 40;
        long long best_score = -1;
        uint32_t best = c1.front().second;
        const size_t K = std::min<size_t>(12, c1.size());
        for (size_t i = 0; i < c1.size() && (i < K || c1[i].first == (int)rem.size()); ++i) {
            const uint32_t R = c1[i].second;
            long long score;
            if (c1[i].first == (int)rem.size()) {
                score = FINISH - ((R & avoid_last) ? 1 : 0);
            } else {
                std::vector<int> take;
                count(rem, R, &take);
                std::vector<char> used(rem.size(), 0);
                for (int t : take) used[t] = 1;
                std::vector<SetOp> rest;
                for (size_t j = 0; j < rem.size(); ++j)
                    if (!used[j]) rest.push_back(rem[j]);
                int c2 = 0;
                for (uint32_t R2 : s2) c2 = std::max(c2, count(rest, R2, nullptr));
                score = (long long)(c1[i].first + c2) * 1024 + c1[i].first;
            }
            if (score > best_score) { best_score = score; best = R; }
        }
        return best;
    }

    // fuse the ops of one phase (in order) under register set R.
    //  - a dense op merges into the single op that last touched its bits when
    //    the union stays in registers, within kmax, and costs no more;
    //  - a diagonal op merges into the dense op that last touched its bits if
    //    they are a subset, otherwise into the latest diagonal op F such that
    //    every op after F that shares its bits is itself diagonal (diagonals
    //    commute), as long as the merged diagonal has at most kMaxDiagBits bits.
    // Order of the fused ops of one phase, by list scheduling over their
    // dependences (ops sharing a bit depend on each other unless both are
    // diagonal; a diagonal moves ahead of permutations, conjugated): whenever
    // diagonals are ready they go out first, merged into as few ops as
    // kMaxDiagBits and the rules below allow (a +-1 diagonal stays a free sign
    // flip unless it joins a register-bit table); then all ready permutations;
    // then all ready rotations as one op; otherwise the earliest ready op.  A layer of split
    // single-qubit gates thus becomes one diagonal, one rotation op over all its
    // register bits, and one diagonal shared with the next layer.
    // A diagonal D after a permutation P equals P then D' before it, D'(x) = D(P x):
    // diagonals move ahead of permutation ops (their entries permuted, their bit set
    // growing by the permutation's bits), so a layer's phases merge across CX gates.
    static SetOp conjugate_through(const SetOp &d, const SetOp &pm)
    {
        if (!(d.mask & pm.mask)) return d;
        SetOp r = d;
        r.mask = d.mask | pm.mask;
        const int k = popc(r.mask);
        r.m.assign((size_t)1 << k, cplx(0, 0));
        const uint32_t ctrl = pm.perm == 1 ? (pm.mask & ~(1u << pm.ptarget)) : 0;
        for (int u = 0; u < (1 << k); ++u) {
            uint32_t x = pdep(u, r.mask), y = x;
            if (pm.perm == 1) {
                if ((x & ctrl) == pm.pcval) y ^= 1u << pm.ptarget;
            } else {
                const int a = __builtin_ctz(pm.mask), b = 31 - __builtin_clz(pm.mask);
                const uint32_t ba = (x >> a) & 1, bb = (x >> b) & 1;
                y = (x & ~((1u << a) | (1u << b))) | (ba << b) | (bb << a);
            }
            r.m[u] = d.m[pext(y, d.mask)];
        }
        return r;
    }

    std::vector<SetOp> reschedule(const std::vector<SetOp> &ops_in, uint32_t R) const
    {
        std::vector<SetOp> ops = ops_in;
        const size_t n = ops.size();
        std::vector<std::vector<int>> succ(n);
        std::vector<int> pending(n, 0);     // undone predecessors
        // a diagonal does not wait for permutation ops: it is conjugated through every one
        // still pending before it when it goes out (see diag_ahead)
        for (size_t j = 0; j < n; ++j)
            for (size_t i = 0; i < j; ++i)
                if ((ops[i].mask & ops[j].mask) && !(ops[i].diag && ops[j].diag) && !(ops[i].perm && ops[j].diag)) {
                    succ[i].push_back((int)j);
                    ++pending[j];
                }
        auto is_sign = [](const SetOp &x) {
            for (const cplx &z : x.m)
                if (!(z.imag() == 0.0 && (z.real() == 1.0 || z.real() == -1.0))) return false;
            return true;
        };
        std::vector<char> done(n, 0);
        std::vector<SetOp> out;
        size_t left = n;
        std::vector<int> finished;          // ops emitted in this round
        while (left) {
            for (int i : finished)
                for (int j : succ[i]) --pending[j];
            finished.clear();
            std::vector<int> ready;
            // a diagonal j whose permutation predecessors are pending moves ahead of every
            // pending op before it, crossing them from right to left: a permutation
            // conjugates it (its bit set grows), any other non-diagonal op must not share a
            // bit with it at that point; the result stays within kMaxDiagBits bits
            auto diag_ahead = [&](int j, SetOp *outp) {
                SetOp d = ops[j];
                for (int i = j - 1; i >= 0; --i) {
                    if (done[i] || ops[i].diag) continue;
                    if (ops[i].perm) d = conjugate_through(d, ops[i]);
                    else if (ops[i].mask & d.mask) return false;
                }
                if (popc(d.mask) > kMaxDiagBits) return false;
                if (outp) *outp = d;
                return true;
            };
            for (size_t j = 0; j < n; ++j)
                if (!done[j] && pending[j] == 0 && (!ops[j].diag || diag_ahead((int)j, nullptr))) ready.push_back((int)j);
            for (int j : ready)
                if (ops[j].diag) diag_ahead(j, &ops[j]);
            std::vector<int> rd, rr, rp;
            for (int j : ready) {
                if (ops[j].diag) rd.push_back(j);
                else if (ops[j].rot) rr.push_back(j);
                else if (ops[j].perm) rp.push_back(j);
            }
            if (rd.empty() && !rp.empty()) {
                // ready permutations (mutually independent) before rotations: they cost
                // nothing and let the rotations of a layer go out together
                for (int j : rp) {
                    out.push_back(ops[j]);
                    done[j] = 1;
                    finished.push_back(j);
                    --left;
                }
            } else if (!rd.empty()) {
                std::vector<SetOp> groups;
                for (int j : rd) {
                    const SetOp &o = ops[j];
                    bool placed = false;
                    for (SetOp &g : groups) {
                        const uint32_t U = g.mask | o.mask;
                        if (popc(U) > kMaxDiagBits) continue;
                        const bool same = is_sign(g) == is_sign(o) && diag_merge_ok(g, o, R);
                        if (same || (U & ~R) == 0) { g = compose(g, o); placed = true; break; }
                    }
                    if (!placed) groups.push_back(o);
                    done[j] = 1;
                    finished.push_back(j);
                    --left;
                }
                for (SetOp &g : groups) out.push_back(std::move(g));
            } else if (!rr.empty()) {
                SetOp g;
                g.rot = true;
                for (int j : rr) {
                    g.mask |= ops[j].mask;
                    g.rots.insert(g.rots.end(), ops[j].rots.begin(), ops[j].rots.end());
                    g.gate_ids.insert(g.gate_ids.end(), ops[j].gate_ids.begin(), ops[j].gate_ids.end());
                    done[j] = 1;
                    finished.push_back(j);
                    --left;
                }
                if (rr.size() == 1) g.m = ops[rr[0]].m;
                out.push_back(std::move(g));
            } else {
                out.push_back(ops[ready.front()]);
                done[ready.front()] = 1;
                finished.push_back(ready.front());
                --left;
            }
        }
        return out;
    }

    // Two diagonals merge freely, except that one split off a single-qubit gate
    // only merges into a diagonal on register bits (the merged op stays a
    // uniform per-register table instead of a per-lane one).
    static bool diag_merge_ok(const SetOp &f, const SetOp &o, uint32_t R)
    {
        return !(f.pin || o.pin) || ((f.mask | o.mask) & ~R) == 0;
    }

    std::vector<SetOp> fuse_phase(const std::vector<SetOp> &ops, uint32_t R) const
    {
        std::vector<SetOp> out;
        std::vector<int> owner(C, -1);
        auto set_owner = [&](uint32_t mask, int idx) {
            for (int b = 0; b < C; ++b)
                if ((mask >> b & 1) && owner[b] < idx) owner[b] = idx;
        };
        for (const SetOp &o : ops) {
            int F = -2;  // -2: none yet; -1: conflicting owners
            for (int b = 0; b < C; ++b) {
                if (!(o.mask >> b & 1) || owner[b] < 0) continue;
                if (F == -2) F = owner[b];
                else if (F != owner[b]) F = -1;
            }
            int merged_into = -1;
            if (fuse && F >= 0) {
                SetOp &f = out[F];
                uint32_t U = f.mask | o.mask;
                int kU = popc(U);
                auto cost = [&](const SetOp &x) {
                    return x.rot ? kRotCost : x.perm ? kPermCost : op_cost(x.diag, popc(x.mask), mfma);
                };
                double before = cost(f) + cost(o);
                bool ok;
                // split-off phases merge later, in reschedule, once a whole layer is ready
                if (f.diag && o.diag) ok = kU <= kMaxDiagBits && !f.pin && !o.pin;
                // a permutation stays free: it merges only into a dense op that covers its bits,
                // and a dense op only into it when the result is no wider than that dense op
                else if ((f.perm && (o.diag || o.rot || o.perm)) || (o.perm && (f.diag || f.rot || f.perm))) ok = false;
                else if (!f.diag && o.diag) ok = !f.rot && (o.mask & ~f.mask) == 0;
                else if (f.diag && o.rot) ok = false;        // keep the split: the phase stays a cheap diagonal
                else ok = (U & ~R) == 0 && kU <= kmax && op_cost(false, kU, mfma) <= before;
                if (ok) {
                    f = compose(f, o);
                    merged_into = F;
                }
            }
            if (fuse && merged_into < 0 && o.diag && !o.pin) {
                // the latest diagonal F with only diagonals after it on o's bits
                // (diagonals commute; split-off phases are passed over)
                for (int i = (int)out.size() - 1; i >= 0; --i) {
                    if (out[i].diag) {
                        if (out[i].pin) continue;
                        if (popc(out[i].mask | o.mask) <= kMaxDiagBits) {
                            out[i] = compose(out[i], o);
                            merged_into = i;
                        }
                        break;
                    }
                    if (out[i].mask & o.mask) break;   // a dense op on o's bits: cannot pass it
                }
            }
            if (merged_into >= 0) {
                set_owner(o.mask, merged_into);
            } else {
                out.push_back(o);
                set_owner(o.mask, (int)out.size() - 1);
            }
        }
        return out;
    }
};

Op to_kernel_op(const SetOp &s, const Layout &lay, int r)
{
    Op op;
    op.gate_ids = s.gate_ids;
    op.k = popc(s.mask);
    op.m = s.m;
    if (s.perm) {
        op.kind = s.perm == 1 ? OP_MCX : OP_SWAPR;
        int mask = 0;
        for (int j = 0; j < r; ++j) {
            if (s.mask >> lay.R[j] & 1) mask |= 1 << j;
            if (s.perm == 1 && lay.R[j] == s.ptarget) op.ptarget = j;
            if (s.perm == 1 && (s.pcval >> lay.R[j] & 1)) op.pcval |= 1 << j;
        }
        op.regmask = mask;
        if (popc((uint32_t)mask) != op.k || (s.perm == 1 && op.ptarget < 0))
            throw std::logic_error("permutation op on a bit outside the phase's registers");
        return op;
    }
    if (s.rot) {
        // coefficients (beta, alpha) per register bit, ascending register index
        op.kind = OP_ROT;
        op.m.clear();
        int mask = 0;
        for (int j = 0; j < r; ++j)
            for (const auto &t : s.rots)
                if ((int)t[0] == lay.R[j]) {
                    mask |= 1 << j;
                    op.m.push_back(cplx(t[1], t[2]));
                }
        op.regmask = mask;
        if (popc((uint32_t)mask) != (int)s.rots.size())
            throw std::logic_error("rotation op on a bit outside the phase's registers");
        return op;
    }
    if (s.diag) {
        op.kind = OP_DIAG;
        int i = 0;
        for (int b = 0; b < 32; ++b)
            if (s.mask >> b & 1) op.tl[i++] = b;
    } else {
        op.kind = OP_DENSE;
        int mask = 0;
        for (int j = 0; j < r; ++j)
            if (s.mask >> lay.R[j] & 1) mask |= 1 << j;
        op.regmask = mask;
    }
    return op;
}

// Local chunk bits an op touches (dense: its register bits; diagonal: its bits).
uint32_t op_local_mask(const Op &op, const Layout &lay, int r)
{
    uint32_t m = 0;
    if (op.kind == OP_DIAG) {
        for (int i = 0; i < op.k; ++i) m |= 1u << op.tl[i];
    } else {
        for (int j = 0; j < r; ++j)
            if (op.regmask >> j & 1) m |= 1u << lay.R[j];
    }
    return m;
}

// Group the phase's single-qubit dense ops that act on distinct register bits
// and are ready together (no earlier op of the phase touches their bits) into
// one OP_MULTI1; other ops keep their order.  One dispatch then applies up to r
// gates with compile-time data flow.
std::vector<Op> group_single_qubit(const std::vector<Op> &ops, const Layout &lay, int r)
{
    std::vector<Op> rem = ops, out;
    while (!rem.empty()) {
        uint32_t blocked = 0, grp = 0;
        std::vector<char> take(rem.size(), 0);
        for (size_t i = 0; i < rem.size(); ++i) {
            const Op &o = rem[i];
            const uint32_t lm = op_local_mask(o, lay, r);
            if (o.kind == OP_DENSE && o.k == 1 && !(lm & blocked) && !(o.regmask & grp)) {
                take[i] = 1;
                grp |= (uint32_t)o.regmask;
            }
            blocked |= lm;
        }
        if (__builtin_popcount(grp) >= 2) {
            Op g;
            g.kind = OP_MULTI1;
            g.regmask = (int)grp;
            g.k = __builtin_popcount(grp);
            for (int j = 0; j < r; ++j) {
                if (!(grp >> j & 1)) continue;
                for (size_t i = 0; i < rem.size(); ++i)
                    if (take[i] && rem[i].regmask == (1 << j)) {
                        g.m.insert(g.m.end(), rem[i].m.begin(), rem[i].m.end());
                        g.gate_ids.insert(g.gate_ids.end(), rem[i].gate_ids.begin(), rem[i].gate_ids.end());
                    }
            }
            out.push_back(std::move(g));
            std::vector<Op> rest;
            for (size_t i = 0; i < rem.size(); ++i)
                if (!take[i]) rest.push_back(rem[i]);
            rem.swap(rest);
        } else {
            out.push_back(rem.front());
            rem.erase(rem.begin());
        }
    }
    return out;
}

Layout make_layout(uint32_t Rmask, int C, int r, const std::vector<int> *store_order)
{
    Layout lay;
    int i = 0;
    for (int b = 0; b < C; ++b)
        if (Rmask >> b & 1) lay.R[i++] = b;
    int t = 0;
    if (store_order) {
        for (int b : *store_order)
            if (!(Rmask >> b & 1)) lay.T[t++] = b;
    } else {
        for (int b = 0; b < C; ++b)
            if (!(Rmask >> b & 1)) lay.T[t++] = b;
    }
    (void)r;
    return lay;
}


// Layout of a later phase of a block: register bits R; thread positions keep
// the previous layout's bit wherever it is still a thread bit (an exchange then
// moves as few thread positions as possible, which lets it run through half
// the LDS buffer, see encode_plan), except the first low.size() positions,
// which take the given bits (the store layout's output-low bits: coalesced
// stores); the rest ascending.
Layout make_layout_keep(uint32_t Rmask, int C, int r, const Layout &prev, const std::vector<int> &low)
{
    Layout lay;
    int i = 0;
    for (int b = 0; b < C; ++b)
        if (Rmask >> b & 1) lay.R[i++] = b;
    const int tb = C - r;
    std::vector<int> T(tb, -1);
    std::vector<char> placed(C, 0);
    int k0 = 0;
    for (int b : low) { T[k0++] = b; placed[b] = 1; }
    for (int j = k0; j < tb; ++j) {
        const int b = prev.T[j];
        if (!(Rmask >> b & 1) && !placed[b]) { T[j] = b; placed[b] = 1; }
    }
    int b = 0;
    for (int j = 0; j < tb; ++j) {
        if (T[j] >= 0) continue;
        while (b < C && ((Rmask >> b & 1) || placed[b])) ++b;
        T[j] = b;
        placed[b] = 1;
    }
    for (int j = 0; j < tb; ++j) lay.T[j] = T[j];
    return lay;
}

// A pass that only permutes: W = physical positions of the chunk (size C,
// containing 0..L-1), target_pos[i] = new position of the amplitude bit now at W[i].
Block make_perm_block(int C, int r, int L, const std::vector<int> &W, const std::vector<int> &target_pos)
{
    Block blk;
    blk.permute_only = true;
    std::vector<std::pair<int, int>> pr;
    for (size_t i = 0; i < W.size(); ++i) pr.push_back({W[i], target_pos[i]});
    std::sort(pr.begin(), pr.end());
    for (auto &x : pr) { blk.P_in.push_back(x.first); blk.P_out.push_back(x.second); }
    std::vector<int> store_order(C);
    std::iota(store_order.begin(), store_order.end(), 0);
    std::sort(store_order.begin(), store_order.end(), [&](int a, int b) { return blk.P_out[a] < blk.P_out[b]; });
    uint32_t lowmask_out = 0;
    for (int i = 0; i < L; ++i) lowmask_out |= 1u << store_order[i];
    uint32_t lowmask_in = (L > 0) ? ((1u << L) - 1) : 0;
    // one layout serves load and store when both use the same low local bits and the
    // registers avoid them; otherwise a load phase and a store phase with one exchange
    uint32_t R = 0;
    int cnt = 0;
    for (int b = C - 1; b >= 0 && cnt < r; --b)
        if (!(lowmask_in >> b & 1) && !(lowmask_out >> b & 1)) { R |= 1u << b; ++cnt; }
    if (cnt == r && lowmask_in == lowmask_out) {
        Phase ph;
        ph.lay = make_layout(R, C, r, &store_order);
        blk.phases.push_back(ph);
    } else {
        uint32_t R0 = 0, R1 = 0;
        int c0 = 0, c1 = 0;
        for (int b = C - 1; b >= 0 && c0 < r; --b)
            if (!(lowmask_in >> b & 1)) { R0 |= 1u << b; ++c0; }
        for (int b = C - 1; b >= 0 && c1 < r; --b)
            if (!(lowmask_out >> b & 1)) { R1 |= 1u << b; ++c1; }
        Phase ld, st;
        ld.lay = make_layout(R0, C, r, nullptr);
        st.lay = make_layout(R1, C, r, &store_order);
        blk.phases.push_back(ld);
        blk.phases.push_back(st);
    }
    return blk;
}

}  // namespace

// Plan for a standalone in-memory swap (Eq. 4): exchange physical bits a[j] <-> b[j].
qs_status build_swap_plan(int n, qs_dtype dtype, int s, const int *a, const int *b, Plan *p, std::string *err)
{
    if (n < 1 || n > 34 || s < 0 || s > 32) { *err = "qs_swap_qubits: bad n or s"; return QS_EINVAL; }
    uint64_t used = 0;
    for (int j = 0; j < s; ++j) {
        if (a[j] < 0 || a[j] >= n || b[j] < 0 || b[j] >= n || a[j] == b[j] || (used >> a[j] & 1) || (used >> b[j] & 1)) {
            *err = "qs_swap_qubits: qubits must be distinct and in range";
            return QS_EINVAL;
        }
        used |= (1ull << a[j]) | (1ull << b[j]);
    }
    p->n = n;
    p->dtype = dtype;
    int r = (dtype == QS_C64) ? 5 : 4;
    int C = std::min((dtype == QS_C64) ? 13 : 12, n);
    r = std::min(r, C);
    int L = std::min(4, C - r);
    p->C = C; p->r = r; p->L = L;
    p->blocks.clear();
    int j = 0;
    while (j < s) {
        std::vector<char> inW(n, 0);
        std::vector<int> W;
        for (int q = 0; q < L; ++q) { inW[q] = 1; W.push_back(q); }
        std::vector<int> tgt_of(n, -1);
        while (j < s) {
            int need = (!inW[a[j]]) + (!inW[b[j]]);
            if ((int)W.size() + need > C) break;
            if (!inW[a[j]]) { inW[a[j]] = 1; W.push_back(a[j]); }
            if (!inW[b[j]]) { inW[b[j]] = 1; W.push_back(b[j]); }
            tgt_of[a[j]] = b[j];
            tgt_of[b[j]] = a[j];
            ++j;
        }
        for (int q = n - 1; q >= 0 && (int)W.size() < C; --q)
            if (!inW[q]) { inW[q] = 1; W.push_back(q); }
        std::vector<int> tgt(W.size());
        for (size_t i = 0; i < W.size(); ++i) tgt[i] = (tgt_of[W[i]] >= 0) ? tgt_of[W[i]] : W[i];
        p->blocks.push_back(make_perm_block(C, r, L, W, tgt));
    }
    encode_plan(p);
    return QS_OK;
}

namespace {
}  // namespace

// ---------------------------------------------------------------------------
qs_status build_plan(const qs_circuit *c, int kmax, const qs_plan_opts *o, Plan *p, std::string *err)
{
    auto t0 = std::chrono::steady_clock::now();
    if (!c || c->n < 1 || c->n > 34 || c->ngates < 0 || (c->ngates > 0 && (!c->k || !c->targets || !c->matrices))) {
        *err = "qs_fuse: bad circuit (n must be 1..34, arrays non-null)";
        return QS_EINVAL;
    }
    if (kmax < 1 || kmax > 5) { *err = "qs_fuse: kmax must be 1..5"; return QS_EINVAL; }
    qs_plan_opts opts{};
    if (o) opts = *o;
    else { opts.enable_swaps = 1; opts.enable_fusion = 1; }
    if (opts.dtype != QS_C128 && opts.dtype != QS_C64) { *err = "qs_fuse: bad dtype"; return QS_EINVAL; }
    if (opts.planner < 0 || opts.planner > 3) { *err = "qs_fuse: planner must be 0..3"; return QS_EINVAL; }
    const int n = c->n;
    p->n = n;
    p->dtype = opts.dtype;
    p->ngates = c->ngates;
    p->kmax = kmax;

    // ---- gates
    std::vector<GateIn> gates(c->ngates);
    const double *mp = c->matrices;
    int maxk = 1;
    for (int g = 0; g < c->ngates; ++g) {
        GateIn &G = gates[g];
        G.k = c->k[g];
        if (G.k < 1 || G.k > 5 || G.k > n) { *err = "qs_fuse: gate " + std::to_string(g) + " has bad k"; return QS_EINVAL; }
        uint64_t seen = 0;
        for (int j = 0; j < G.k; ++j) {
            int q = c->targets[5 * g + j];
            if (q < 0 || q >= n || (seen >> q & 1)) {
                *err = "qs_fuse: gate " + std::to_string(g) + " has a bad or repeated target";
                return QS_EINVAL;
            }
            seen |= 1ull << q;
            G.t[j] = q;
        }
        int d = 1 << G.k;
        G.m.resize((size_t)d * d);
        for (int i = 0; i < d * d; ++i) G.m[i] = cplx(mp[2 * i], mp[2 * i + 1]);
        mp += 2 * (size_t)d * d;
        G.diag = matrix_is_diag(G.m, d);
        if (!G.diag) maxk = std::max(maxk, G.k);
    }

    // ---- geometry
    int r = opts.reg_qubits ? opts.reg_qubits : (opts.dtype == QS_C64 ? 5 : 4);
    if (r < 1 || r > kMaxReg) { *err = "qs_fuse: reg_qubits must be 1..5"; return QS_EINVAL; }
    r = std::max(r, maxk);                     // a dense gate must fit in registers
    int C = opts.chunk_qubits ? opts.chunk_qubits : (opts.dtype == QS_C64 ? 13 : 12);
    if (C < 1 || C > kMaxChunk) { *err = "qs_fuse: chunk_qubits must be 1..14"; return QS_EINVAL; }
    int L = opts.low_qubits ? opts.low_qubits : 4;
    C = std::min(C, n);
    // at most 512 threads per workgroup for r <= 3, 256 otherwise
    if (C - r > 9 || (r > 3 && C - r > 8)) r = std::max(r, C - 8);
    if (r > kMaxReg) { *err = "qs_fuse: chunk_qubits must be <= 13 (256 threads x 32 registers)"; return QS_EINVAL; }
    r = std::min(r, C);
    if (maxk > r) { *err = "qs_fuse: a gate is wider than the chunk"; return QS_EINVAL; }
    L = std::min(L, C - r);                    // low qubits live in thread bits of load/store layouts
    if (L < 0) L = 0;
    p->C = C; p->r = r; p->L = L;
    const int kf = std::min(kmax, r);
    const bool gbg = (opts.planner == 2);

    // ---- blocking with reorder swaps
    std::vector<int> l2p(n), p2l(n);
    std::iota(l2p.begin(), l2p.end(), 0);
    std::iota(p2l.begin(), p2l.end(), 0);
    std::vector<int> rem(c->ngates);
    std::iota(rem.begin(), rem.end(), 0);
    Blocker B(gates, n);
    // matrix-core ops: complex64, five register bits, whole wavefronts of threads
    p->mfma = opts.dtype == QS_C64 && !opts.no_mfma && r == 5 && C - r >= 6;
    PhaseSched PS{C, r, L, kf, opts.enable_fusion != 0, p->mfma};
    // single-qubit gates as phase * rotation * phase (needs the fusion pass to pay off)
    const bool split = opts.enable_fusion && !opts.no_split && !gbg;

    auto emit_block = [&](const std::vector<char> &inS, const std::vector<int> &take, bool last) {
        Block blk;
        // chunk positions = physical positions of S
        for (int q = 0; q < n; ++q)
            if (inS[q]) blk.P_in.push_back(l2p[q]);
        std::sort(blk.P_in.begin(), blk.P_in.end());
        std::vector<int> loc_of_phys(n, -1);
        for (int b = 0; b < C; ++b) loc_of_phys[blk.P_in[b]] = b;
        p->layouts.push_back(l2p);
        // ops in local bits
        std::vector<SetOp> ops;
        uint32_t flip = 0;
        for (int gi : take) {
            const GateIn &G = gates[gi];
            int loc[5];
            for (int j = 0; j < G.k; ++j) loc[j] = loc_of_phys[l2p[G.t[j]]];
            blk.gate_ids.push_back(gi);
            // a SWAP carries pending X gates (see below) over to the other bit and stays a SWAP
            if (split && G.k == 2 && ((flip >> loc[0]) ^ (flip >> loc[1])) & 1) {
                static const cplx sw[16] = {1, 0, 0, 0, 0, 0, 1, 0, 0, 1, 0, 0, 0, 0, 0, 1};
                if (std::equal(G.m.begin(), G.m.end(), sw)) {
                    flip ^= (1u << loc[0]) | (1u << loc[1]);
                    ops.push_back(gate_to_setop(G, loc, gi));
                    continue;
                }
            }
            // bits with an X pending: the gate acts on the state as X G X would on the
            // stored amplitudes, so its matrix indices flip on those bits
            uint32_t fl = 0;
            for (int j = 0; j < G.k; ++j)
                if (flip >> loc[j] & 1) fl |= 1u << (G.k - 1 - j);
            const GateIn Gc = fl ? conjugate_x(G, fl) : G;
            cplx pre[2], post[2];
            double rb, ra;
            bool fx = false;
            std::vector<cplx> rm;
            const bool is_x = Gc.k == 1 && Gc.m[0] == cplx(0, 0) && Gc.m[1] == cplx(1, 0) && Gc.m[2] == cplx(1, 0) &&
                              Gc.m[3] == cplx(0, 0);
            if (split && is_x) {
                // an X only toggles its bit's pending flip: no op at all
                flip ^= 1u << loc[0];
                continue;
            }
            if (split && Gc.k == 1 && !Gc.diag && split_rotation(Gc.m, pre, post, &rb, &ra, &rm, &fx)) {
                // phase (with the rotation's scaling), two shears, phase: the phases merge with
                // neighbouring diagonals; a pending X (fx) goes on to the end of the block
                SetOp d0, rt, d1;
                d0.diag = d1.diag = true;
                d0.pin = d1.pin = true;
                d0.mask = rt.mask = d1.mask = 1u << loc[0];
                d0.m = {pre[0], pre[1]};
                d1.m = {post[0], post[1]};
                rt.rot = true;
                rt.m = rm;
                rt.rots.push_back({(double)loc[0], rb, ra});
                rt.gate_ids.push_back(gi);
                ops.push_back(std::move(d0));
                ops.push_back(std::move(rt));
                ops.push_back(std::move(d1));
                if (fx) flip ^= 1u << loc[0];
                continue;
            }
            ops.push_back(gate_to_setop(Gc, loc, gi));
        }
        // X gates still pending on local bits: the store writes every amplitude with
        // these bits of its local index inverted
        blk.flip = flip;
        // ---- output placement (folded swap)
        std::vector<int> newpos(C);   // local bit b (logical p2l[P_in[b]]) -> physical
        for (int b = 0; b < C; ++b) newpos[b] = blk.P_in[b];
        if (opts.enable_swaps) {
            // members of S by next use after this block
            std::vector<int> done_mark(c->ngates, 0);
            for (int gi : take) done_mark[gi] = 1;
            std::vector<int> nextuse(n, 1 << 30);
            int pos = 0;
            for (int gi : rem) {
                if (done_mark[gi]) continue;
                for (int j = 0; j < gates[gi].k; ++j) {
                    int q = gates[gi].t[j];
                    nextuse[q] = std::min(nextuse[q], pos);
                }
                ++pos;
            }
            std::vector<int> locs(C);
            std::iota(locs.begin(), locs.end(), 0);
            if (last) {
                // put every logical qubit home when its home is in the chunk
                std::vector<int> free_pos;
                std::vector<char> placed(C, 0);
                std::vector<char> taken(n, 0);
                for (int b = 0; b < C; ++b) {
                    int q = p2l[blk.P_in[b]];
                    if (loc_of_phys[q] >= 0) { newpos[b] = q; placed[b] = 1; taken[q] = 1; }
                }
                for (int b = 0; b < C; ++b)
                    if (!taken[blk.P_in[b]]) free_pos.push_back(blk.P_in[b]);
                size_t fi = 0;
                for (int b = 0; b < C; ++b)
                    if (!placed[b]) newpos[b] = free_pos[fi++];
            } else {
                // by next use, soonest first, onto the chunk's physical positions in ascending
                // order: the L soonest-needed qubits go to 0..L-1 (always in the chunk), and the
                // next ones stay at low positions, so later chunks gather their runs from fewer,
                // closer address-translation pages (a pass over a chunk of low positions streams
                // up to 28 % faster than one over the highest positions)
                // A qubit with no gate left goes home (physical position = its index) when its
                // home is one of the chunk's positions above 0..L-1: the final passes that
                // restore the order then have less to move.
                std::vector<char> done_b(C, 0), used_pos(n, 0);
                for (int b = 0; b < C; ++b) {
                    const int q = p2l[blk.P_in[b]];
                    if (nextuse[q] == (1 << 30) && q >= L && loc_of_phys[q] >= 0) {
                        newpos[b] = q;
                        done_b[b] = 1;
                        used_pos[q] = 1;
                    }
                }
                std::stable_sort(locs.begin(), locs.end(), [&](int a, int b) {
                    return nextuse[p2l[blk.P_in[a]]] < nextuse[p2l[blk.P_in[b]]];
                });
                std::vector<int> posv;
                for (int b = 0; b < C; ++b)
                    if (!used_pos[blk.P_in[b]]) posv.push_back(blk.P_in[b]);
                std::sort(posv.begin(), posv.end());
                size_t pi = 0;
                for (int i = 0; i < C; ++i)
                    if (!done_b[locs[i]]) newpos[locs[i]] = posv[pi++];
            }
        }
        blk.P_out = newpos;
        // update maps
        std::vector<int> movedq(C);
        for (int b = 0; b < C; ++b) movedq[b] = p2l[blk.P_in[b]];
        for (int b = 0; b < C; ++b) { l2p[movedq[b]] = newpos[b]; p2l[newpos[b]] = movedq[b]; }

        // ---- phases
        std::vector<int> store_order;   // local bits ordered by output physical position
        {
            std::vector<int> lb(C);
            std::iota(lb.begin(), lb.end(), 0);
            std::sort(lb.begin(), lb.end(), [&](int a, int b) { return newpos[a] < newpos[b]; });
            store_order = lb;
        }
        uint32_t lowmask_in = (L > 0) ? ((1u << L) - 1) : 0;      // local bits at physical 0..L-1 on load
        uint32_t lowmask_out = 0;
        for (int i = 0; i < L; ++i) lowmask_out |= 1u << store_order[i];
        const std::vector<int> low_out(store_order.begin(), store_order.begin() + L);
        uint32_t all = (C >= 32) ? 0xffffffffu : ((1u << C) - 1);
        std::vector<SetOp> prem = ops;
        bool first = true;
        while (!prem.empty() || first) {
            uint32_t allowed = first ? (all & ~lowmask_in) : all;
            uint32_t R = PS.choose_R_search(prem, allowed, all, lowmask_out);
            std::vector<int> takeidx;
            PS.count(prem, R, &takeidx);
            std::vector<SetOp> phase_ops;
            std::vector<char> used(prem.size(), 0);
            for (int i : takeidx) { phase_ops.push_back(prem[i]); used[i] = 1; }
            std::vector<SetOp> rest;
            for (size_t i = 0; i < prem.size(); ++i)
                if (!used[i]) rest.push_back(prem[i]);
            prem.swap(rest);
            Phase ph;
            ph.lay = first ? make_layout(R, C, r, nullptr)
                           : make_layout_keep(R, C, r, blk.phases.back().lay, std::vector<int>());
            std::vector<Op> kops;
            std::vector<SetOp> fused = PS.fuse_phase(phase_ops, R);
            if (opts.enable_fusion) fused = PS.reschedule(fused, R);
            for (const SetOp &s : fused) {
                Op k = to_kernel_op(s, ph.lay, r);
                if (k.kind == OP_SWAPR) {
                    // SWAP(a, b) = CX(a -> b) CX(b -> a) CX(a -> b): three permutation ops
                    const int a = __builtin_ctz((unsigned)k.regmask), b = 31 - __builtin_clz((unsigned)k.regmask);
                    for (int t : {b, a, b}) {
                        Op x = k;
                        x.kind = OP_MCX;
                        x.ptarget = t;
                        x.pcval = k.regmask & ~(1 << t);
                        kops.push_back(x);
                    }
                    continue;
                }
                kops.push_back(k);
            }
            ph.ops = opts.enable_fusion ? group_single_qubit(kops, ph.lay, r) : kops;
            blk.phases.push_back(ph);
            first = false;
        }
        // store layout: registers away from the output-low bits, thread bits in output order
        {
            Phase &lastp = blk.phases.back();
            uint32_t Rl = 0;
            for (int j = 0; j < r; ++j) Rl |= 1u << lastp.lay.R[j];
            if ((Rl & lowmask_out) || (blk.phases.size() == 1 && lowmask_out != lowmask_in)) {
                // choose the r highest output positions that are not low, sparing one
                // chunk bit >= 4 that keeps its (non-low) thread position from the last
                // phase, so that this exchange too can run through half the LDS buffer
                int anchor = -1;
                for (int j = C - r - 1; j >= L && anchor < 0; --j) {
                    const int b = lastp.lay.T[j];
                    if (b >= 4 && !(lowmask_out >> b & 1)) anchor = b;
                }
                uint32_t R = 0;
                int cnt = 0;
                for (int i = C - 1; i >= 0 && cnt < r; --i) {
                    int b = store_order[i];
                    if (!(lowmask_out >> b & 1) && b != anchor) { R |= 1u << b; ++cnt; }
                }
                for (int i = C - 1; i >= 0 && cnt < r; --i) {      // too few bits: use the anchor too
                    int b = store_order[i];
                    if (!(lowmask_out >> b & 1) && !(R >> b & 1)) { R |= 1u << b; ++cnt; }
                }
                Phase sp;
                sp.lay = make_layout_keep(R, C, r, lastp.lay, low_out);
                blk.phases.push_back(sp);
            } else if (blk.phases.size() == 1) {
                lastp.lay = make_layout(Rl, C, r, &store_order);
            } else {
                // the last phase takes the store layout (its ops index registers by R, which
                // is unchanged) -- unless that leaves its exchange without a split bit while
                // every earlier exchange has one: then a separate store phase (one more
                // exchange) keeps the whole block on half-buffer exchanges
                auto has_split = [&](const Layout &x, const Layout &y) {
                    for (int j = 0; j < C - r; ++j)
                        if (x.T[j] == y.T[j] && x.T[j] >= 4) return true;
                    return false;
                };
                const size_t np = blk.phases.size();
                const Layout relaid = make_layout_keep(Rl, C, r, blk.phases[np - 2].lay, low_out);
                bool earlier = true;
                for (size_t q = 1; q + 1 < np; ++q) earlier &= has_split(blk.phases[q - 1].lay, blk.phases[q].lay);
                earlier &= has_split(blk.phases[np - 2].lay, lastp.lay);
                bool matrix_cores = false;
                for (const Phase &P : blk.phases)
                    for (const Op &op : P.ops) matrix_cores |= p->mfma && op.kind == OP_DENSE && op.k >= 4;
                if (has_split(blk.phases[np - 2].lay, relaid) || !earlier || matrix_cores) {
                    lastp.lay = relaid;
                } else {
                    int anchor = -1;
                    for (int j = C - r - 1; j >= L && anchor < 0; --j) {
                        const int b = lastp.lay.T[j];
                        if (b >= 4 && !(lowmask_out >> b & 1)) anchor = b;
                    }
                    uint32_t R = 0;
                    int cnt = 0;
                    for (int i = C - 1; i >= 0 && cnt < r; --i) {
                        int b = store_order[i];
                        if (!(lowmask_out >> b & 1) && b != anchor) { R |= 1u << b; ++cnt; }
                    }
                    for (int i = C - 1; i >= 0 && cnt < r; --i) {
                        int b = store_order[i];
                        if (!(lowmask_out >> b & 1) && !(R >> b & 1)) { R |= 1u << b; ++cnt; }
                    }
                    Phase sp;
                    sp.lay = make_layout_keep(R, C, r, lastp.lay, low_out);
                    blk.phases.push_back(sp);
                }
            }
        }
        p->blocks.push_back(std::move(blk));
    };

    auto emit_perm_pass = [&](const std::vector<int> &W, const std::vector<int> &target_pos) {
        p->layouts.push_back(l2p);
        Block blk = make_perm_block(C, r, L, W, target_pos);
        std::vector<int> movedq(C);
        for (int b = 0; b < C; ++b) movedq[b] = p2l[blk.P_in[b]];
        for (int b = 0; b < C; ++b) { l2p[movedq[b]] = blk.P_out[b]; p2l[blk.P_out[b]] = movedq[b]; }
        p->blocks.push_back(std::move(blk));
    };

    if (gbg) {
        // one block per gate: the gate's qubits plus the resident low qubits
        for (int gi = 0; gi < c->ngates; ++gi) {
            std::vector<char> inS(n, 0);
            int nS = 0;
            for (int j = 0; j < gates[gi].k; ++j) { inS[gates[gi].t[j]] = 1; ++nS; }
            for (int pp = 0; pp < L; ++pp)
                if (!inS[p2l[pp]]) { inS[p2l[pp]] = 1; ++nS; }
            for (int pp = 0; pp < n && nS < C; ++pp)
                if (!inS[p2l[pp]]) { inS[p2l[pp]] = 1; ++nS; }
            std::vector<int> take{gi};
            rem.erase(rem.begin());
            emit_block(inS, take, false);
        }
    } else {
        while (!rem.empty()) {
            std::vector<int> forced;
            for (int pp = 0; pp < L; ++pp) forced.push_back(p2l[pp]);
            std::vector<char> inS = choose_chunk(B, rem, forced, C, n);
            int nS = C;
            std::vector<int> take;
            B.count(rem, inS, nS, &take);
            if (take.empty()) { *err = "qs_fuse: internal error: empty gate block"; return QS_EINVAL; }
            // is this the last block?
            bool last = (take.size() == rem.size());
            std::vector<char> dm(c->ngates, 0);
            for (int gi : take) dm[gi] = 1;
            emit_block(inS, take, last);
            std::vector<int> nr;
            for (int gi : rem)
                if (!dm[gi]) nr.push_back(gi);
            rem.swap(nr);
        }
    }
    // ---- restore canonical order with permutation passes
    for (int guard = 0; guard < 4 * n + 8; ++guard) {
        std::vector<int> disp;
        for (int pp = 0; pp < n; ++pp)
            if (p2l[pp] != pp) disp.push_back(pp);
        if (disp.empty()) break;
        // follow cycles to collect up to C - L positions (plus the low ones)
        std::vector<char> inW(n, 0);
        std::vector<int> W;
        for (int pp = 0; pp < L; ++pp) { inW[pp] = 1; W.push_back(pp); }
        std::vector<char> seen(n, 0);
        for (int start : disp) {
            if ((int)W.size() >= C) break;
            int x = start;
            while (!seen[x] && (int)W.size() < C) {
                seen[x] = 1;
                if (!inW[x]) { inW[x] = 1; W.push_back(x); }
                x = p2l[x];      // the qubit at x wants to go home to position p2l[x]
                if (x == start) break;
            }
        }
        for (int pp = 0; pp < n && (int)W.size() < C; ++pp)
            if (!inW[pp]) { inW[pp] = 1; W.push_back(pp); }
        std::vector<int> tgt(W.size(), -1);
        std::vector<char> used(n, 0);
        for (size_t i = 0; i < W.size(); ++i) {
            int q = p2l[W[i]];
            if (inW[q]) { tgt[i] = q; used[q] = 1; }
        }
        std::vector<int> freep;
        for (int x : W)
            if (!used[x]) freep.push_back(x);
        size_t fi = 0;
        for (size_t i = 0; i < W.size(); ++i)
            if (tgt[i] < 0) tgt[i] = freep[fi++];
        emit_perm_pass(W, tgt);
    }
    p->layouts.push_back(l2p);
    for (int q = 0; q < n; ++q)
        if (l2p[q] != q) { *err = "qs_fuse: internal error: final layout not canonical"; return QS_EINVAL; }

    // ---- stats
    qs_plan_stats &s = p->stats;
    std::memset(&s, 0, sizeof(s));
    s.n = n;
    s.dtype = opts.dtype;
    s.gates = c->ngates;
    s.chunk_qubits = C;
    s.low_qubits = L;
    s.reg_qubits = r;
    s.planner = gbg ? 2 : 0;
    s.candidates = 1;
    s.predicted_ms = -1.0;
    s.predicted_heuristic_ms = -1.0;
    for (const Block &blk : p->blocks) {
        if (blk.permute_only) ++s.swap_passes;
        else ++s.blocks;
        for (const Phase &ph : blk.phases) {
            ++s.phases;
            for (const Op &op : ph.ops) {
                ++s.ops;
                if (op.kind == OP_DIAG) { ++s.ops_diag; s.flops_per_amp += 6.0; }
                else if (op.kind == OP_MULTI1) { s.ops_dense[1] += op.k; s.flops_per_amp += 16.0 * op.k; }
                else if (op.kind == OP_ROT) { s.ops_rot += op.k; s.flops_per_amp += 4.0 * op.k; }
                else if (op.kind == OP_MCX || op.kind == OP_SWAPR) ++s.ops_perm;
                else {
                    ++s.ops_dense[op.k];
                    s.flops_per_amp += 8.0 * (double)(1 << op.k);
                    if (p->mfma && op.k >= 4) ++s.ops_mfma;
                }
            }
        }
    }
    double amp_bytes = (opts.dtype == QS_C64) ? 8.0 : 16.0;
    s.hbm_bytes = (double)(s.blocks + s.swap_passes) * 2.0 * std::ldexp(1.0, n) * amp_bytes;
    encode_plan(p);
    p->plan_seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    s.plan_seconds = p->plan_seconds;
    return QS_OK;
}

// ---------------------------------------------------------------------------
// Encoding for the blocked kernel
// ---------------------------------------------------------------------------
namespace {
// Low-nibble images of local bits under the swizzle: bits 0-2 map to
// themselves, bit 3 to 8 ^ g3 (g3 in bits 0-2), bit b >= 4 to F[b-4].
uint32_t img(int b, const uint32_t *F, uint32_t g3) { return b < 3 ? (1u << b) : b == 3 ? (8u | g3) : F[b - 4]; }

bool independent4(uint32_t a, uint32_t b, uint32_t c, uint32_t d)
{
    uint32_t v[4] = {a, b, c, d};
    // span check over GF(2): all 16 XOR combinations distinct
    uint32_t seen = 0;
    for (int s = 0; s < 16; ++s) {
        uint32_t x = 0;
        for (int i = 0; i < 4; ++i)
            if (s >> i & 1) x ^= v[i];
        if (seen >> x & 1) return false;
        seen |= 1u << x;
    }
    return true;
}

bool independent3(uint32_t a, uint32_t b, uint32_t c)
{
    uint32_t v[3] = {a, b, c};
    uint32_t seen = 0;
    for (int s = 0; s < 8; ++s) {
        uint32_t x = 0;
        for (int i = 0; i < 3; ++i)
            if (s >> i & 1) x ^= v[i];
        if (seen >> x & 1) return false;
        seen |= 1u << x;
    }
    return true;
}

uint64_t choose_swizzle(const Layout &from, const Layout &to, int C, int r)
{
    int tb = C - r;
    if (tb < 4 || C <= 4) return 0;
    uint32_t F[16] = {0};
    uint32_t g3 = 0;
    uint64_t rng = 0x9E3779B97F4A7C15ull ^ (uint64_t)(from.T[0] * 131 + to.T[0] * 17 + C);
    auto next = [&]() { rng ^= rng << 13; rng ^= rng >> 7; rng ^= rng << 17; return rng; };
    bool inset[32] = {false};
    for (int i = 0; i < 4; ++i) { inset[from.T[i]] = true; inset[to.T[i]] = true; }
    // lanes 0-15 of a wavefront must hit 16 distinct 16-byte slots (mod 256 B), and
    // lanes 0-7 8 distinct slots (mod 128 B), on both sides of the exchange
    auto good = [&](const Layout &L) {
        return independent4(img(L.T[0], F, g3), img(L.T[1], F, g3), img(L.T[2], F, g3), img(L.T[3], F, g3)) &&
               independent3(img(L.T[0], F, g3) & 7, img(L.T[1], F, g3) & 7, img(L.T[2], F, g3) & 7);
    };
    for (int tries = 0; tries < 20000; ++tries) {
        if (good(from) && good(to)) break;
        for (int b = 4; b < C; ++b) F[b - 4] = inset[b] ? (uint32_t)(next() & 15) : 0;
        g3 = inset[3] ? (uint32_t)(next() & 7) : 0;
    }
    uint64_t w = 0;
    for (int b = 4; b < C; ++b) w |= (uint64_t)(F[b - 4] & 15) << (4 * (b - 4));
    w |= (uint64_t)(g3 & 7) << 60;      // nibble 15: fold of bit 3 into bits 0-2
    return w;
}

}  // namespace

// Every op word of the encoded program names a code path that the kernel
// variant chosen for its block has compiled in (the kernel treats any other
// value as unreachable): kinds 0 and 2..8, dense register masks within the
// variant's width, matrix-core masks only in matrix-core blocks.
static void check_program(const Plan &p)
{
    const int C = p.C, r = p.r, tb = C - r, NR = 1 << r;
    for (size_t b = 0; b < p.blocks.size(); ++b) {
        const int32_t *w = p.h_prog.data() + p.prog_off[b];
        const int bk = p.block_kmax[b];
        const bool bm = p.block_mfma[b] != 0;
        // the dense width compiled into the variant the launcher picks
        const int kw = bm ? 3 : bk == 0 ? 0 : (bk <= 2 || r <= 2) ? std::min(r, 2) : (bk == 3 || r == 3) ? 3 : r;
        const int32_t *ph = w + PROG_HDR + 2 * C;
        if ((w[3] & 4) && bm)
            throw std::logic_error("half-buffer exchanges in a matrix-core block");
        for (int q = 0; q < w[0]; ++q) {
            if (kw == 0 && !bm && (ph[0] & 1))
                throw std::logic_error("odd op count in a phase of a block without dense ops");
            const uint32_t hx = (uint32_t)ph[3] >> 24;
            const int hjw = (int)(hx & 15) - 1, hjr = (int)(hx >> 4) - 1;
            if ((hjw >= 0) != (q > 0 && (w[3] & 4) != 0) || hjw != hjr || hjw >= tb)
                throw std::logic_error("bad half-buffer exchange position");
            const int32_t *op = ph + PHASE_HDR + C + 2 * tb + 2 * NR;
            for (int o = 0; o < ph[0]; ++o, op += OP_WORDS) {
                const int kind = op[0] & 0xff, var = (op[0] >> 8) & 0xff;
                bool ok;
                switch (kind) {
                case OP_DENSE: ok = var > 0 && var < NR && __builtin_popcount(var) <= kw; break;
                case OP_MULTI1: ok = kw >= 1 && var > 0 && var < NR; break;
                case OP_ROT: case OP_ROTD: ok = var > 0 && var < NR; break;
                case OP_MCX:
                    ok = (var & 7) < r && (var >> 3) < NR && !(((var >> 3) >> (var & 7)) & 1) &&
                         (op[3] & ~(var >> 3)) == 0;
                    break;
                case OP_MFMA:
                    ok = bm && r == 5 && (var == 15 || var == 23 || var == 27 || var == 29 || var == 30 || var == 31);
                    break;
                case OP_DIAG_REG: case OP_DIAG_ROW: case OP_SIGN_REG: case OP_SIGN_ROW: case OP_NOP: ok = true; break;
                default: ok = false;
                }
                if (!ok)
                    throw std::logic_error("encoded op (kind " + std::to_string(kind) + ", mask " + std::to_string(var) +
                                           ") has no kernel path in its block");
            }
            ph = op;
        }
        // the load/store map (the kernel's only source of global addresses) sits between the
        // phases and the table and agrees with the first and last phases' layouts
        const int32_t *mp = w + w[4] - kMapWords;
        const int32_t *l0 = w + PROG_HDR + 2 * C + PHASE_HDR, *l1 = w + ((uint32_t)w[3] >> 8) + PHASE_HDR;
        const int32_t *Pin = w + PROG_HDR, *Pout = w + PROG_HDR + C;
        bool mok = w[4] % 4 == 0 && mp >= ph && tb <= 16 && r <= 5;
        uint64_t cm = 0;
        for (int b2 = 0; mok && b2 < C; ++b2) cm |= 1ull << Pin[b2];
        mok = mok && (uint32_t)mp[26] == (uint32_t)cm && (uint32_t)mp[27] == (uint32_t)(cm >> 32);
        for (int j = 0; mok && j < tb; ++j) mok = mp[j] == Pin[l0[r + j]] && mp[28 + j] == Pout[l1[r + j]];
        for (int j = 0; mok && j < r; ++j) mok = mp[16 + j] == Pin[l0[j]] && mp[21 + j] == Pout[l1[j]];
        if (!mok) throw std::logic_error("block " + std::to_string(b) + ": load/store map disagrees with its layouts");
    }
}

void encode_plan(Plan *p)
{
    p->h_prog.clear();
    p->h_mats.clear();
    p->prog_off.clear();
    p->block_kmax.clear();
    p->block_mfma.clear();
    const int C = p->C, r = p->r;
    for (const Block &blk : p->blocks) {
        int64_t start = (int64_t)p->h_prog.size();
        p->prog_off.push_back(start);
        int bk = 0;
        bool bm = false;
        for (const Phase &P : blk.phases)
            for (const Op &op : P.ops)
                if (op.kind == OP_DENSE && p->mfma && op.k >= 4) bm = true;
                else if (op.kind == OP_DENSE) bk = std::max(bk, op.k);
                else if (op.kind == OP_MULTI1) bk = std::max(bk, 1);
        p->block_kmax.push_back(bk);
        p->block_mfma.push_back(bm ? 1 : 0);
        std::vector<int32_t> w;
        w.push_back((int32_t)blk.phases.size());
        w.push_back(C);
        w.push_back(r);
        // flags: bit 0 = swap pass; bit 1 = the write-back moves amplitudes between
        // threads' load positions (P_out != P_in), so loads must all complete
        // before any store even when no exchange separates them
        // Half-buffer exchanges (every block but the complex64 matrix-core ones): when every
        // exchange of the block has a chunk bit b >= 4 at the same thread position j
        // in both layouts, each thread's amplitudes all share b's value before and
        // after, so the exchange runs in two rounds through a buffer of half the
        // chunk (b dropped from the LDS addresses): in round h the threads with bit
        // j = h write and, after a barrier, read.  (With b at different positions a
        // thread could read in round 0 and write in round 1, over registers already
        // replaced.)  Less LDS per workgroup, more workgroups per CU.  Wave-index
        // positions are preferred (whole waves take part in a round, no divergence).
        std::vector<int> split_w(blk.phases.size(), -1), split_r(blk.phases.size(), -1), split_b(blk.phases.size(), -1);
        bool half = !bm && !blk.permute_only && blk.phases.size() >= 2;
        for (size_t ph = 1; half && ph < blk.phases.size(); ++ph) {
            const Layout &a = blk.phases[ph - 1].lay, &b2 = blk.phases[ph].lay;
            int best = -1;
            for (int ja = 0; ja < C - r; ++ja)
                for (int jb = 0; jb < C - r; ++jb) {
                    if (ja != jb || a.T[ja] != b2.T[jb] || a.T[ja] < 4) continue;
                    const int score = (ja >= 6) + (jb >= 6) + (ja == jb);
                    if (score > best) { best = score; split_w[ph] = ja; split_r[ph] = jb; split_b[ph] = a.T[ja]; }
                }
            if (best < 0) half = false;
        }
        // the store inverts the pending-X bits: physical positions of those local bits
        uint64_t fphys = 0;
        for (int b = 0; b < C; ++b)
            if (blk.flip >> b & 1) fphys |= 1ull << blk.P_out[b];
        w.push_back((blk.permute_only ? 1 : 0) | (blk.P_out != blk.P_in || fphys ? 2 : 0) | (half ? 4 : 0));
        w.push_back(0);   // table offset, patched below
        w.push_back(0);   // table words
        w.push_back((int32_t)(uint32_t)(fphys & 0xffffffffu));
        w.push_back((int32_t)(uint32_t)(fphys >> 32));
        for (int b = 0; b < C; ++b) w.push_back(blk.P_in[b]);
        for (int b = 0; b < C; ++b) w.push_back(blk.P_out[b]);
        std::vector<int32_t> tab;   // per-lane data of diagonal ops, staged in LDS by the kernel
        const bool c64 = (p->dtype == QS_C64);
        // Per-lane tables staged in LDS are capped at 16 KiB so that the workgroups per CU
        // stay what the exchange buffer allows (half buffer: three, whole buffer: two);
        // larger tables are read from device memory (L2) instead.
        const size_t tab_cap = std::min<size_t>(4096, (160u * 1024u - ((size_t)(c64 ? 8 : 16) << C)) / 4);
        size_t last_hdr = 0;    // word offset of the last phase's header (the store layout)
        for (size_t ph = 0; ph < blk.phases.size(); ++ph) {
            const Phase &P = blk.phases[ph];
            uint64_t swz = (ph > 0) ? choose_swizzle(blk.phases[ph - 1].lay, P.lay, C, r) : 0;
            const size_t hdr = w.size();
            last_hdr = hdr;
            w.push_back((int32_t)P.ops.size());
            w.push_back((int32_t)(uint32_t)(swz & 0xffffffffu));
            w.push_back((int32_t)(uint32_t)(swz >> 32));
            w.push_back(0);
            for (int j = 0; j < r; ++j) w.push_back(P.lay.R[j]);
            for (int j = 0; j < C - r; ++j) w.push_back(P.lay.T[j]);
            const int NR = 1 << r;
            const int amp_bytes = (p->dtype == QS_C64) ? 8 : 16;
            {
                // exchange block: the swizzle is XOR-linear, so every slot splits into
                // per-thread-bit and per-register contributions, precomputed here
                const uint32_t swlo = (uint32_t)(swz & 0xffffffffu), swhi = (uint32_t)(swz >> 32);
                auto sw = [&](uint32_t l) {
                    uint32_t f = 0, hh = l >> 4;
                    for (int b = 0; b < 8; ++b)
                        if (hh >> b & 1) f ^= (swlo >> (4 * b)) & 15u;
                    for (int b = 0; b < 2; ++b)
                        if (hh >> (8 + b) & 1) f ^= (swhi >> (4 * b)) & 15u;
                    if (l >> 3 & 1) f ^= (swhi >> 28) & 7u;
                    return l ^ f;
                };
                const bool has = ph > 0;
                const Layout *pl = has ? &blk.phases[ph - 1].lay : nullptr;
                for (int j = 0; j < C - r; ++j) w.push_back(has ? (int32_t)(sw(1u << pl->T[j]) * amp_bytes) : 0);
                for (int j = 0; j < C - r; ++j) w.push_back(has ? (int32_t)(sw(1u << P.lay.T[j]) * amp_bytes) : 0);
                const size_t xw0 = w.size() - 2 * (size_t)(C - r);   // the thread-bit words
                for (int m = 0; m < NR; ++m) {
                    uint32_t lr = 0;
                    if (has)
                        for (int j = 0; j < r; ++j)
                            if (m >> j & 1) lr |= 1u << pl->R[j];
                    w.push_back(has ? (int32_t)(sw(lr) * amp_bytes) : 0);
                }
                for (int m = 0; m < NR; ++m) {
                    uint32_t lr = 0;
                    for (int j = 0; j < r; ++j)
                        if (m >> j & 1) lr |= 1u << P.lay.R[j];
                    w.push_back(has ? (int32_t)(sw(lr) * amp_bytes) : 0);
                }
                if (has && half) {
                    // drop the split bit from every byte address (linear, like the swizzle)
                    const int bb = split_b[ph] + (amp_bytes == 16 ? 4 : 3);
                    auto drop = [bb](uint32_t x) { return (x & ((1u << bb) - 1)) | ((x >> (bb + 1)) << bb); };
                    const size_t x0 = w.size() - 2 * (size_t)(C - r) - 2 * (size_t)NR;
                    for (size_t i = x0; i < w.size(); ++i) w[i] = (int32_t)drop((uint32_t)w[i]);
                    w[hdr + 3] |= (int32_t)((uint32_t)(split_w[ph] + 1) << 24 | (uint32_t)(split_r[ph] + 1) << 28);
                }
                // the thread's XOR of its bits' words, tabulated per nibble of the thread
                // index in the LDS table (header word 3, low 24 bits = its offset + 1):
                // write side W0[16] (thread bits 0-3), W1[16] (4-7), W2[2] (8), then the
                // read side the same way; the kernel forms each with three table reads
                if (has && tab.size() + 2 * kNibWords <= tab_cap) {
                    w[hdr + 3] |= (int32_t)tab.size() + 1;
                    const int tbits = C - r;
                    for (int side = 0; side < 2; ++side) {
                        const int32_t *xw = w.data() + xw0 + (size_t)side * tbits;
                        for (int part = 0; part < 3; ++part) {
                            const int lo = 4 * part, cnt = part < 2 ? 16 : 2;
                            for (int e = 0; e < cnt; ++e) {
                                uint32_t acc = 0;
                                for (int j = lo; j < lo + 4 && j < tbits; ++j)
                                    if (e >> (j - lo) & 1) acc ^= (uint32_t)xw[j];
                                tab.push_back((int32_t)acc);
                            }
                        }
                    }
                }
            }
            // blocks without dense ops run two ops per loop trip: an odd phase gets a
            // leading no-op (OP_NOP)
            // a rotation op followed by a diagonal on register bits only (not +-1) runs as one
            // op (OP_ROTD: the shears, then the diagonal): one dispatch instead of two
            auto reg_only_diag = [&](const Op &d) {
                if (d.kind != OP_DIAG) return false;
                for (int i = 0; i < d.k; ++i) {
                    bool in_r = false;
                    for (int j = 0; j < r; ++j) in_r |= P.lay.R[j] == d.tl[i];
                    if (!in_r) return false;
                }
                for (const cplx &z : d.m)
                    if (!(z.imag() == 0.0 && (z.real() == 1.0 || z.real() == -1.0))) return true;
                return false;
            };
            std::vector<char> fuse_next(P.ops.size(), 0);
            size_t nenc = P.ops.size();
            for (size_t i = 0; i + 1 < P.ops.size(); ++i)
                if (P.ops[i].kind == OP_ROT && reg_only_diag(P.ops[i + 1]) && !(i > 0 && fuse_next[i - 1])) {
                    fuse_next[i] = 1;
                    --nenc;
                }
            // an odd count in a block without dense ops: split a fused rotation + diagonal
            // back into its two ops rather than pad with a no-op (the no-op's path costs
            // register copies; the split costs one more dispatch and no arithmetic)
            if (bk == 0 && !bm && (nenc & 1))
                for (size_t i = P.ops.size(); i-- > 0;)
                    if (fuse_next[i]) {
                        fuse_next[i] = 0;
                        ++nenc;
                        break;
                    }
            w[hdr] = (int32_t)nenc;
            if (bk == 0 && !bm && (nenc & 1)) {
                w[hdr] = (int32_t)nenc + 1;
                w.push_back(OP_NOP);
                w.push_back(0);
                w.push_back(0);
                w.push_back(0);
            }
            for (size_t oi = 0; oi < P.ops.size(); ++oi) {
                const Op &op = P.ops[oi];
                int64_t moff = (int64_t)p->h_mats.size();
                if (fuse_next[oi]) {
                    // (a, b) per rotated register bit, then the 2^r diagonal entries in register order
                    const Op &d = P.ops[oi + 1];
                    for (const cplx &z : op.m) { p->h_mats.push_back(z.real()); p->h_mats.push_back(z.imag()); }
                    for (int m = 0; m < NR; ++m) {
                        uint32_t l = 0;
                        for (int j = 0; j < r; ++j)
                            if (m >> j & 1) l |= 1u << P.lay.R[j];
                        int idx = 0;
                        for (int t = 0; t < d.k; ++t) idx |= (int)((l >> d.tl[t]) & 1) << t;
                        p->h_mats.push_back(d.m[idx].real());
                        p->h_mats.push_back(d.m[idx].imag());
                    }
                    w.push_back(OP_ROTD | (op.regmask << 8) | (op.k << 16));
                    w.push_back((int32_t)(uint32_t)(moff & 0xffffffff));
                    w.push_back((int32_t)(uint32_t)(moff >> 32));
                    w.push_back(0);
                    ++oi;
                    continue;
                }
                if (op.kind == OP_DENSE && p->mfma && op.k >= 4) {
                    // Matrix-core form: the real embedding [[Re U, -Im U], [Im U, Re U]] of U,
                    // stored in the order the kernel feeds the 32x32x2 FP32 product: block mb
                    // of 32 output rows, step s, lane.  Output row mm = 2 i + (0 re | 1 im) of
                    // element i; at step s lane (m, h) = (lane % 32, lane / 32) holds the
                    // coefficient of part (s % 2) of input element 2 (s / 2) + h.
                    const int D = 1 << op.k, nmb = D / 16;
                    for (int mb = 0; mb < nmb; ++mb)
                        for (int s = 0; s < D; ++s)
                            for (int lane = 0; lane < 64; ++lane) {
                                const int mm = 32 * mb + lane % 32, row = mm / 2, po = mm % 2;
                                const int col = 2 * (s / 2) + lane / 32, pi = s % 2;
                                const cplx u = op.m[(size_t)row * D + col];
                                double a = (po == pi) ? u.real() : u.imag();
                                if (po == 0 && pi == 1) a = -a;
                                p->h_mats.push_back(a);
                            }
                    w.push_back(OP_MFMA | (op.regmask << 8) | (op.k << 16));
                    w.push_back((int32_t)(uint32_t)(moff & 0xffffffff));
                    w.push_back((int32_t)(uint32_t)(moff >> 32));
                    w.push_back(0);
                    continue;
                }
                if (op.kind == OP_MCX) {
                    const int var = op.ptarget | ((op.regmask & ~(1 << op.ptarget)) << 3);
                    w.push_back(OP_MCX | (var << 8) | (op.k << 16));
                    w.push_back(0);
                    w.push_back(0);
                    w.push_back(op.pcval);
                    continue;
                }
                if (op.kind == OP_DENSE || op.kind == OP_MULTI1 || op.kind == OP_ROT) {
                    // rotations: (a, b) per register bit in the real and imaginary slots
                    for (const cplx &z : op.m) { p->h_mats.push_back(z.real()); p->h_mats.push_back(z.imag()); }
                    w.push_back(op.kind | (op.regmask << 8) | (op.k << 16));
                    w.push_back((int32_t)(uint32_t)(moff & 0xffffffff));
                    w.push_back((int32_t)(uint32_t)(moff >> 32));
                    w.push_back(0);
                    continue;
                }
                // diagonal: split its bits into register bits and thread bits of this layout
                uint32_t opmask = 0;
                for (int i = 0; i < op.k; ++i) opmask |= 1u << op.tl[i];
                uint32_t tmask = 0;     // over thread-index bits
                int kt = 0;
                for (int j = 0; j < C - r; ++j)
                    if (opmask >> P.lay.T[j] & 1) { tmask |= 1u << j; ++kt; }
                bool sign = true;
                for (const cplx &z : op.m)
                    if (!(z.imag() == 0.0 && (z.real() == 1.0 || z.real() == -1.0))) { sign = false; break; }
                // entry for (row, m): local index from the row's thread bits and m's register bits
                auto entry = [&](int row, int m) {
                    uint32_t l = 0;
                    int i = 0;
                    for (int j = 0; j < C - r; ++j)
                        if (tmask >> j & 1) { l |= (uint32_t)((row >> i) & 1) << P.lay.T[j]; ++i; }
                    for (int j = 0; j < r; ++j)
                        if (m >> j & 1) l |= 1u << P.lay.R[j];
                    int idx = 0;
                    for (int t = 0; t < op.k; ++t) idx |= (int)((l >> op.tl[t]) & 1) << t;
                    return op.m[idx];
                };
                const int rows = 1 << kt;
                bool global_tab = false;      // the per-row table does not fit beside the chunk in LDS
                if (sign) {
                    std::vector<int32_t> masks(rows, 0);
                    for (int row = 0; row < rows; ++row)
                        for (int m = 0; m < NR; ++m)
                            if (entry(row, m).real() < 0) masks[row] |= (int32_t)(1u << m);
                    if (kt == 0) {
                        w.push_back(OP_SIGN_REG | (op.k << 16));
                        w.push_back(0);
                        w.push_back(0);
                        w.push_back(masks[0]);
                        continue;
                    }
                    if (tab.size() + (size_t)rows <= tab_cap) {
                        w.push_back(OP_SIGN_ROW | (op.k << 16));
                        w.push_back((int32_t)tmask);
                        w.push_back(0);
                        w.push_back((int32_t)tab.size());
                        tab.insert(tab.end(), masks.begin(), masks.end());
                        continue;
                    }
                    global_tab = true;        // as a +-1 diagonal read from device memory
                }
                if (kt == 0) {
                    for (int m = 0; m < NR; ++m) {
                        cplx z = entry(0, m);
                        p->h_mats.push_back(z.real());
                        p->h_mats.push_back(z.imag());
                    }
                    w.push_back(OP_DIAG_REG | (op.k << 16));
                    w.push_back((int32_t)(uint32_t)(moff & 0xffffffff));
                    w.push_back((int32_t)(uint32_t)(moff >> 32));
                    w.push_back(0);
                    continue;
                }
                // a row holds the entries over the op's register bits only (rmask, register
                // positions): 2^kr of them, entry e for every register m with pext(m, rmask) = e
                uint32_t rmask = 0;
                for (int j = 0; j < r; ++j)
                    if (opmask >> P.lay.R[j] & 1) rmask |= 1u << j;
                const int kr = popc(rmask), ne = 1 << kr;
                auto reg_of = [&](int e) {
                    int m = 0, i = 0;
                    for (int j = 0; j < r; ++j)
                        if (rmask >> j & 1) { m |= ((e >> i) & 1) << j; ++i; }
                    return m;
                };
                const size_t row_words = (size_t)ne * (c64 ? 2 : 4);
                if (global_tab || ((tab.size() + 3) & ~(size_t)3) + (size_t)rows * row_words > tab_cap) {
                    // table in device memory (variant bit 0): rows of 2^kr entries, interleaved re/im
                    for (int row = 0; row < rows; ++row)
                        for (int e = 0; e < ne; ++e) {
                            cplx z = entry(row, reg_of(e));
                            p->h_mats.push_back(z.real());
                            p->h_mats.push_back(z.imag());
                        }
                    w.push_back(OP_DIAG_ROW | ((1 | (int)(rmask << 1)) << 8) | (op.k << 16));
                    w.push_back((int32_t)tmask);
                    w.push_back((int32_t)(uint32_t)(moff & 0xffffffff));
                    w.push_back((int32_t)(uint32_t)(moff >> 32));
                    continue;
                }
                while (tab.size() % 4) tab.push_back(0);     // 16-byte aligned rows
                w.push_back(OP_DIAG_ROW | ((int)(rmask << 1) << 8) | (op.k << 16));
                w.push_back((int32_t)tmask);
                w.push_back(0);
                w.push_back((int32_t)tab.size());
                for (int row = 0; row < rows; ++row)
                    for (int e = 0; e < ne; ++e) {
                        cplx z = entry(row, reg_of(e));
                        if (c64) {
                            float f[2] = {(float)z.real(), (float)z.imag()};
                            int32_t u[2];
                            std::memcpy(u, f, 8);
                            tab.push_back(u[0]);
                            tab.push_back(u[1]);
                        } else {
                            double d[2] = {z.real(), z.imag()};
                            int32_t u[4];
                            std::memcpy(u, d, 16);
                            tab.insert(tab.end(), u, u + 4);
                        }
                    }
            }
        }
        if (last_hdr >= (1u << 23)) throw std::logic_error("block program too long");
        w[3] |= (int32_t)((uint32_t)last_hdr << 8);
        while (w.size() % 4) w.push_back(0);
        {
            // load/store map (kMapWords words, a multiple of 4, right before the table):
            // what the kernel would otherwise derive from the layouts before its first loads
            if (C - r > 16 || r > 5) throw std::logic_error("layout too large for the load/store map");
            const Layout &l0 = blk.phases.front().lay, &l1 = blk.phases.back().lay;
            std::vector<int32_t> mp(kMapWords, 0);
            uint64_t cm = 0;
            for (int b = 0; b < C; ++b) cm |= 1ull << blk.P_in[b];
            for (int j = 0; j < C - r; ++j) {
                mp[j] = blk.P_in[l0.T[j]];
                mp[28 + j] = blk.P_out[l1.T[j]];
            }
            for (int j = 0; j < r; ++j) {
                mp[16 + j] = blk.P_in[l0.R[j]];
                mp[21 + j] = blk.P_out[l1.R[j]];
            }
            mp[26] = (int32_t)(uint32_t)(cm & 0xffffffffu);
            mp[27] = (int32_t)(uint32_t)(cm >> 32);
            w.insert(w.end(), mp.begin(), mp.end());
        }
        while (tab.size() % 4) tab.push_back(0);    // whole 16-byte words: staged as such, and every
                                                    // block's program starts 16-byte aligned
        w[4] = (int32_t)w.size();
        w[5] = (int32_t)tab.size();
        w.insert(w.end(), tab.begin(), tab.end());
        p->h_prog.insert(p->h_prog.end(), w.begin(), w.end());
    }
    if (p->dtype == QS_C64) {
        p->h_mats32.resize(p->h_mats.size());
        for (size_t i = 0; i < p->h_mats.size(); ++i) p->h_mats32[i] = (float)p->h_mats[i];
    }
    if (p->h_mats.empty()) p->h_mats.push_back(0.0);
    if (p->h_prog.empty()) p->h_prog.push_back(0);
    if (p->dtype == QS_C64 && p->h_mats32.empty()) p->h_mats32.push_back(0.f);
    check_program(*p);
}

// ---------------------------------------------------------------------------
std::string dump_plan(const Plan &p)
{
    std::ostringstream os;
    os.precision(17);
    os << "# n=" << p.n << " C=" << p.C << " L=" << p.L << " r=" << p.r << " kmax=" << p.kmax
       << " dtype=" << (p.dtype == QS_C64 ? "c64" : "c128") << "\n";
    for (size_t bi = 0; bi < p.blocks.size(); ++bi) {
        const Block &b = p.blocks[bi];
        int lines = 1;
        for (const Phase &ph : b.phases) lines += 1 + (int)ph.ops.size();
        os << lines << "\n";
        os << (b.permute_only ? "SWAP" : "BLOCK") << " in";
        for (int x : b.P_in) os << " " << x;
        os << " out";
        for (int x : b.P_out) os << " " << x;
        os << "\n";
        for (const Phase &ph : b.phases) {
            os << "PHASE R";
            for (int j = 0; j < p.r; ++j) os << " " << ph.lay.R[j];
            os << " T";
            for (int j = 0; j < p.C - p.r; ++j) os << " " << ph.lay.T[j];
            os << "\n";
            for (const Op &op : ph.ops) {
                if (op.kind == OP_DIAG) {
                    os << "D" << op.k;
                    for (int j = 0; j < op.k; ++j) os << " " << op.tl[j];
                    os << " " << op.m[0].real() << " " << op.m[0].imag();
                } else {
                    os << (op.kind == OP_MULTI1 ? "M" : op.kind == OP_ROT ? "R" : op.kind == OP_MCX ? "X"
                           : op.kind == OP_SWAPR ? "S" : "U") << op.k;
                    for (int j = 0; j < p.r; ++j)
                        if (op.regmask >> j & 1) os << " " << ph.lay.R[j];
                }
                os << " ids";
                for (int g : op.gate_ids) os << " " << g;
                os << "\n";
            }
        }
    }
    return os.str();
}

}  // namespace qs
