// qs_internal.h -- structures shared by the host planner, the C ABI and the
// kernel launchers of libqs.  Not installed; the public interface is
// include/qs.h.
#pragma once

#include <complex>
#include <cstdint>
#include <mutex>
#include <string>
#include <vector>

#include <hip/hip_runtime.h>

#include "../../include/qs.h"

namespace qs {

using cplx = std::complex<double>;

// Largest chunk (in qubits) and register-bit count the blocked kernel is
// instantiated for.
constexpr int kMaxChunk = 14;
constexpr int kMaxReg = 5;
constexpr int kMaxDiagBits = 8;   // merged diagonals keep at most 2^8 entries

// ---------------------------------------------------------------------------
// Plan IR (host side)
// ---------------------------------------------------------------------------
enum OpKind {
    OP_DENSE = 0,      // dense 2^k x 2^k on register bits (regmask)
    OP_DIAG = 1,       // planner form of a diagonal on local bits tl[]; encoded as one of:
    OP_DIAG_REG = 2,   //   bits all in registers: 2^r entries in register order, uniform
    OP_DIAG_ROW = 3,   //   some bits are thread bits: 2^kt rows of 2^r entries, row = pext(tid, tmask)
    OP_SIGN_REG = 4,   //   entries all +-1, bits in registers: bit m of a mask negates register m
    OP_SIGN_ROW = 5,   //   entries all +-1 with thread bits: one such mask per row
    OP_MULTI1 = 6,     // one 2x2 gate on each register bit of regmask (they commute), ascending bit order
    OP_MFMA = 7,       // encoding of a complex64 dense op of k >= 4 register bits run on matrix cores
    OP_ROT = 8,        // a real plane rotation on each register bit of regmask, as three shears
                       // x0 += a x1, x1 += b x0, x0 += a x1 (coefficients (a, b) per bit, ascending)
    OP_MCX = 9,        // permutation, no arithmetic: flip register bit ptarget of every register whose
                       // bits in regmask & ~(1 << ptarget) (the controls) equal pcval (X, CX, CCX
                       // with controls on 1 or 0)
    OP_SWAPR = 10,     // planner only: SWAP of the two register bits of regmask, encoded as three OP_MCX
    OP_ROTD = 11,      // encoding only: an OP_ROT followed by a diagonal on register bits, in one op
    OP_NOP = 12        // encoding only: pads a phase of a block without dense ops to an even op count
};
// words of the per-nibble tables of an exchange's thread-bit words (write and read side each:
// 16 for thread bits 0-3, 16 for bits 4-7, 2 for bit 8)
constexpr int kNibWords = 34;
// words of the load/store map right before a block's table (see the encoding below)
constexpr int kMapWords = 44;

struct Op {
    int kind = OP_DENSE;
    // Dense: register-position mask (bit j set = register bit j is a target);
    //        matrix index bit i <-> the i-th lowest set bit of the mask.
    // Diag:  local chunk bits tl[0..k-1] ascending; table index bit i <-> tl[i].
    int regmask = 0;
    int ptarget = -1;             // OP_MCX: register position of the flipped bit
    int pcval = 0;                // OP_MCX: control values (register mask within the controls)
    int k = 0;
    int tl[kMaxDiagBits] = {0};
    std::vector<cplx> m;          // dense: (2^k)^2 row-major; diag: 2^k
    std::vector<int> gate_ids;    // original gates folded into this op (order of application)
};

struct Layout {
    int R[kMaxReg];               // local bits held in registers (ascending)
    int T[kMaxChunk];             // local bits of the thread index, thread bit b <-> T[b]
};

struct Phase {
    Layout lay;
    std::vector<Op> ops;
};

struct Block {
    std::vector<int> P_in;        // P_in[b]  = physical qubit of local bit b when loading (ascending)
    std::vector<int> P_out;       // P_out[b] = physical qubit local bit b is written to (a permutation of P_in)
    std::vector<Phase> phases;
    std::vector<int> gate_ids;    // original gates in execution order
    bool permute_only = false;    // a swap pass: no ops
    uint32_t flip = 0;            // local bits with an X pending at the end: stored inverted
};

struct Plan {
    int n = 0;
    qs_dtype dtype = QS_C128;
    int C = 12, L = 4, r = 4;
    int kmax = 5;
    bool mfma = false;                  // complex64 dense ops of k >= 4 are encoded as OP_MFMA
    std::vector<Block> blocks;          // steps, in order (swap passes are blocks with permute_only)
    std::vector<std::vector<int>> layouts;  // l2p before each step, plus the final one
    int ngates = 0;
    double plan_seconds = 0.0;
    qs_plan_stats stats{};
    std::string error;

    std::vector<int64_t> prog_off;      // per block: offset of its program in the program words (int32 words)
    std::vector<int> block_kmax;        // per block: widest vector dense op (selects the kernel variant)
    std::vector<char> block_mfma;       // per block: has matrix-core ops (complex64 variant with them)
    std::vector<int32_t> h_prog;
    std::vector<double> h_mats;
    std::vector<float> h_mats32;
};

// Build the plan (host).  Returns QS_OK or an error with *err filled.
qs_status build_plan(const qs_circuit *c, int kmax, const qs_plan_opts *o, Plan *p, std::string *err);
// Plan of permutation-only passes exchanging physical bits a[j] <-> b[j].
qs_status build_swap_plan(int n, qs_dtype dtype, int s, const int *a, const int *b, Plan *p, std::string *err);
// Serialise to the kernel program format (host arrays in p).
void encode_plan(Plan *p);
// Text dump.
std::string dump_plan(const Plan &p);
// Block features for the cost model (48 per step, swap passes included).
void block_features(const Plan &p, std::vector<float> *out);
// Candidate-plan search: planner 1 ranks by the cost model (opts->cost_model),
// planner 3 by the number of passes (the paper's objective, Eq. 7).
qs_status build_plan_search(const qs_circuit *c, int kmax, const qs_plan_opts *o, Plan *p, std::string *err);

// ---------------------------------------------------------------------------
// Program encoding read by the blocked kernel (int32 words per block):
//   [0] nphases, [1] C, [2] r, [3] flags (bit 0 swap pass, bit 1 P_out != P_in,
//       bit 2 every exchange runs in two rounds through half the LDS buffer; bits 8-31 the
//       word offset of the last phase's header from the block start: the store layout, for
//       validators -- the kernel takes its store addresses from the map below)
//   [4] table offset (words from block start, multiple of 4), [5] table words; the
//       kMapWords words before the table are the load/store map: [0..16) physical
//       position of thread bit j when loading (P_in of the first phase's T[j]), [16..21)
//       physical position of register bit j when loading (P_in of the first phase's
//       R[j]), [21..26) when storing (P_out of the last phase's R[j]), [26], [27] the
//       chunk's physical-qubit mask (low, high word), [28..44) physical position of thread
//       bit j when storing (P_out of the last phase's T[j]); unused entries 0
//   [6], [7] store inversion mask (physical bits, low / high word): the store writes the
//       amplitude of index x at x ^ mask (pending X gates of the block)
//   [8 .. 8+C)        P_in
//   [8+C .. 8+2C)     P_out
//   then per phase:
//     [0] nops, [1] swz_lo (F nibbles for high bits 0..7), [2] swz_hi (8..15),
//     [3] bits 0-23: 1 + word offset in the LDS table of the per-nibble XOR tables of the
//         thread-bit words below (write side, then read side, kNibWords each), or 0;
//         bits 24-27 / 28-31: 1 + thread position of the split bit in the write /
//         read layout (equal; 0 = one round through the whole buffer); the split bit is then
//         dropped from every offset of the exchange block
//     [4 .. 4+r)      R
//     [4+r .. 4+C)    T
//     exchange into this phase (zeros for phase 0), LDS byte offsets:
//       tb words: write-side contribution of thread bit j (previous layout)
//       tb words: read-side contribution of thread bit j (this layout)
//       2^r words: write-side offset of register m; 2^r words: read-side offset of register m
//       (slot of (thread, m) = XOR of the thread's bit contributions ^ offset of m)
//     then per op: 4 words: [kind | (variant << 8) | (k << 16)] [w1] [w2] [w3]
//       DENSE   : variant = register mask; w1,w2 = matrix offset (scalars, lo/hi)
//       MULTI1  : variant = register mask; w1,w2 = offset of one 2x2 matrix per set bit, ascending
//       DIAG_REG: w1,w2 = offset of 2^r entries (register order)
//       DIAG_ROW: w1 = tmask (thread-index bits of the row); variant bits 1-5 = rmask, the
//                 register positions the op touches: a row holds 2^kr entries (kr = popcount
//                 rmask), register m takes entry pext(m, rmask); variant bit 0 clear: w3 = word
//                 offset in the LDS table of 2^kt rows (complex128: 4 words per entry,
//                 complex64: 2); bit 0 set (table too large for LDS): w2,w3 = offset of the rows
//                 in the matrices
//       MFMA    : variant = register mask (k = 4, 5 of r = 5); w1,w2 = offset of the real-embedded
//                 matrix in matrix-core operand order (complex64 only)
//       SIGN_REG: w3 = mask over registers (bit m set: negate register m)
//       SIGN_ROW: w1 = tmask; w3 = word offset in the table of 2^kt row masks
//       ROT     : variant = register mask; w1,w2 = offset of (beta, alpha) per set bit,
//                 ascending: x0 += beta x1, then x1 += alpha x0 on each pair
//       MCX     : variant = target register position (bits 0-2) | control register mask << 3;
//                 w3 = the values the controls must hold (register mask, within the controls)
//       ROTD    : variant = register mask; w1,w2 = offset of (beta, alpha) per set bit, ascending, then
//                 the 2^r entries of a diagonal in register order (applied after the shears)
//       (blocks without dense ops hold an even op count per phase; an OP_NOP pads)
// The table (per-lane data of diagonal ops) is copied into LDS, after the
// exchange buffer, once per workgroup.
// The swizzle for the exchange INTO a phase: slot(l) = l ^ F(l >> 4) where
// F XORs nibble b of swz (bits 4b..4b+3) for every set bit b of (l >> 4).
// ---------------------------------------------------------------------------
enum { PROG_HDR = 8, PHASE_HDR = 4, OP_WORDS = 4 };

}  // namespace qs

// ---------------------------------------------------------------------------
// State handle
// ---------------------------------------------------------------------------
struct qs_state {
    int n = 0;
    qs_dtype dtype = QS_C128;
    void *amps = nullptr;
    size_t bytes = 0;
    hipStream_t stream = nullptr;
    int device = -1;
    void *d_scratch = nullptr;     // small device scratch: gate matrices for k >= 4, reduction partials
    size_t scratch_bytes = 0;
    bool own_scratch = false;      // allocated by qs_attach (no caller workspace): freed by qs_destroy
};

// A plan and its device tables, one set per device it has run on (uploaded
// on first use there, under the lock).
struct qs_plan {
    struct DevTables {
        int device = -1;
        void *d_prog = nullptr;        // int32 program words of all steps
        void *d_mats = nullptr;        // matrices (FP64 or FP32 by dtype)
        hipEvent_t ready = nullptr;    // recorded after the upload on the uploading stream
        hipStream_t stream = nullptr;  // that stream
    };
    qs::Plan p;
    std::mutex mu;
    std::vector<DevTables> dev;
};

// error helpers (api.cpp)
namespace qs {
void set_error(const std::string &msg);
qs_status hip_fail(hipError_t e, const char *what);
}

// kernel launchers (k_basic.hip / k_block.hip)
namespace qs {
hipError_t launch_init(qs_state *st, uint64_t index);
hipError_t launch_gate(qs_state *st, int k, const int *targets, const double *matrix);
// gate-by-gate kind of a gate: 0 dense, 1 diagonal, 2 permutation with phases, on *nt
// active targets once the controls in *cbits are peeled off (host only)
int gate_kind(int k, const int *targets, const double *matrix, uint64_t *cbits, int *nt);
hipError_t launch_swap(qs_state *st, int s, const int *a, const int *b);
hipError_t launch_probs(qs_state *st, double *out);
hipError_t launch_expect(qs_state *st, int nterms, const qs_pauli *terms, double *partials, int nparts);
int expect_partials(int n);
hipError_t launch_block(qs_state *st, const Plan &p, const void *d_prog, const void *d_mats, int b);
hipStream_t costmodel_stream(const qs_costmodel *m);
int costmodel_device(const qs_costmodel *m);
hipError_t launch_block_prog(qs_state *st, int r, int C, const int *d_prog, const void *d_mats, size_t tab_bytes,
                             int kmax_dense, bool mfma, bool half);
}
