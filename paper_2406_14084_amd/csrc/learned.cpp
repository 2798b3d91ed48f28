// learned.cpp -- block features for the plan cost model, and the learned
// planner that ranks candidate plans with it.
//
// The paper's optimiser scores a blocking by the number of gate blocks it
// needs (Sec. IV, Eq. 7): every block is one pass over the state.  On this
// GPU the passes are not equal -- a block's time depends on its fused ops,
// register phases, exchanges and write-back permutation -- so the learned
// planner scores a plan by the sum over its steps of a predicted time,
//   t(step) = 2^n * exp(model(features(step))) picoseconds,
// builds candidate plans over the geometry knobs the heuristic fixes (chunk
// size C, register bits r, contiguous low bits L, fusion width, and for
// complex64 whether 4-5-qubit ops use the matrix cores), and keeps
// the heuristic plan unless the model predicts a clear gain for another.
// The same search scored by the paper's own objective -- the fewest passes
// over the state -- is planner 3, the method without the learned model.
#include <algorithm>
#include <array>
#include <chrono>
#include <cmath>
#include <cstring>
#include <memory>
#include <thread>
#include <vector>

#include "qs_internal.h"

namespace qs {

namespace {
constexpr int NF = QS_COST_FEATURES;

int popc(uint32_t x) { return __builtin_popcount(x); }
}  // namespace

// 48 features per step (gate block or swap pass), all scaled to O(1).
void block_features(const Plan &p, std::vector<float> *out)
{
    out->clear();
    const int n = p.n, C = p.C, r = p.r, L = p.L;
    const int amp_bytes = p.dtype == QS_C64 ? 8 : 16;
    const int kf = std::min(p.kmax, r);
    for (size_t b = 0; b < p.blocks.size(); ++b) {
        const Block &blk = p.blocks[b];
        float f[NF] = {0};
        const int32_t *w = p.h_prog.data() + p.prog_off[b];
        const int nph = w[0], flags = w[3], tab_words = w[5];
        const bool perm_wb = (flags & 2) != 0;
        int dense[6] = {0}, ndiag_reg = 0, ndiag_row = 0, nsign_reg = 0, nsign_row = 0, nmulti = 0, nmulti_g = 0;
        int nops = 0, max_ops = 0, swz_phases = 0, diag_bits = 0, nmfma = 0, kdense_max = 0;
        double flops = 0, flops_k45 = 0, dense_width = 0, dense_k_sum = 0;
        const int32_t *q = w + PROG_HDR + 2 * C;
        for (int ph = 0; ph < nph; ++ph) {
            const int no = q[0];
            if (q[1] != 0 || q[2] != 0) ++swz_phases;
            nops += no;
            max_ops = std::max(max_ops, no);
            q += PHASE_HDR + C + 2 * (C - r) + 2 * (1 << r);
            for (int o = 0; o < no; ++o, q += OP_WORDS) {
                const int kind = q[0] & 0xff, mask = (q[0] >> 8) & 0xff, k = (q[0] >> 16) & 0xff;
                switch (kind) {
                case OP_DENSE:
                    ++dense[k];
                    flops += 8.0 * (1 << k);
                    if (k >= 4) flops_k45 += 8.0 * (1 << k);
                    dense_width += 1 << k;
                    dense_k_sum += k;
                    kdense_max = std::max(kdense_max, k);
                    break;
                case OP_MFMA:
                    ++dense[k];
                    ++nmfma;
                    flops += 8.0 * (1 << k);
                    flops_k45 += 8.0 * (1 << k);
                    dense_width += 1 << k;
                    dense_k_sum += k;
                    kdense_max = std::max(kdense_max, k);
                    break;
                case OP_MULTI1:
                    ++nmulti;
                    nmulti_g += popc((uint32_t)mask);
                    flops += 16.0 * popc((uint32_t)mask);
                    kdense_max = std::max(kdense_max, 1);
                    break;
                case OP_ROT:     // grouped like the single-qubit ops, at its own arithmetic
                    ++nmulti;
                    nmulti_g += popc((uint32_t)mask);
                    flops += 4.0 * popc((uint32_t)mask);
                    break;
                case OP_ROTD:    // a rotation op and a register diagonal in one dispatch
                    ++nmulti;
                    nmulti_g += popc((uint32_t)mask);
                    flops += 4.0 * popc((uint32_t)mask) + 6;
                    ++ndiag_reg;
                    break;
                case OP_DIAG_REG: ++ndiag_reg; flops += 6; diag_bits += k; break;
                case OP_DIAG_ROW: ++ndiag_row; flops += 6; diag_bits += k; break;
                case OP_SIGN_REG:
                    if (k == 0) break;      // padding no-op
                    ++nsign_reg;
                    diag_bits += k;
                    break;
                case OP_SIGN_ROW: ++nsign_row; diag_bits += k; break;
                default: break;
                }
            }
        }
        int run_in = 0;
        while (run_in < C && blk.P_in[run_in] == run_in) ++run_in;
        int run_out = 0;
        while (run_out < C && blk.P_out[run_out] == run_out) ++run_out;
        int hi20 = 0, moved = 0, mid = 0, pmax = 0;
        for (int j = 0; j < C; ++j) {
            hi20 += blk.P_in[j] >= 20;
            mid += blk.P_in[j] >= L && blk.P_in[j] < 12;
            moved += blk.P_out[j] != blk.P_in[j];
            pmax = std::max(pmax, blk.P_in[j]);
        }
        const double lds = (double)(1 << C) * amp_bytes + 4.0 * tab_words;
        const int threads = 1 << (C - r);
        const double occ = std::min({8.0, std::floor(160.0 * 1024 / lds), std::floor(2048.0 / threads)});
        f[0] = blk.permute_only ? 1.f : 0.f;
        f[1] = p.dtype == QS_C64 ? 1.f : 0.f;
        f[2] = n / 34.f;
        f[3] = C / 14.f;
        f[4] = r / 5.f;
        f[5] = L / 8.f;
        f[6] = nph / 8.f;
        f[7] = std::max(0, nph - 1) / 8.f;
        f[8] = perm_wb ? 1.f : 0.f;
        f[9] = (perm_wb && nph == 1) ? 1.f : 0.f;
        f[10] = kdense_max / 5.f;
        for (int k = 1; k <= 5; ++k) f[10 + k] = dense[k] / 8.f;
        f[16] = ndiag_reg / 8.f;
        f[17] = ndiag_row / 8.f;
        f[18] = nsign_reg / 8.f;
        f[19] = nsign_row / 8.f;
        f[20] = nmulti / 8.f;
        f[21] = nmulti_g / 16.f;
        f[22] = (float)(flops / 256.0);
        f[23] = (float)(std::log2(1.0 + flops) / 10.0);
        f[24] = tab_words / 1024.f;
        f[25] = run_in / 14.f;
        f[26] = run_out / 14.f;
        f[27] = hi20 / 14.f;
        f[28] = pmax / 34.f;
        f[29] = moved / 14.f;
        f[30] = blk.gate_ids.size() / 128.f;
        f[31] = nops / 32.f;
        f[32] = max_ops / 16.f;
        f[33] = amp_bytes / 16.f;
        f[34] = (float)(lds / (160.0 * 1024));
        f[35] = threads / 512.f;
        f[36] = (float)(occ / 8.0);
        f[37] = (n - C) / 24.f;
        f[38] = flops > 0 ? (float)(flops_k45 / flops) : 0.f;
        f[39] = (float)(dense_width / 128.0);
        f[40] = nmfma / 8.f;
        f[41] = swz_phases / 8.f;
        f[42] = kf / 5.f;
        f[43] = diag_bits / 32.f;
        const int ndense = dense[1] + dense[2] + dense[3] + dense[4] + dense[5];
        f[44] = ndense ? (float)(dense_k_sum / ndense / 5.0) : 0.f;
        f[45] = (float)(flops / amp_bytes / 32.0);
        f[46] = std::max(0, nph - 1) * amp_bytes / 128.f;
        f[47] = mid / 14.f;
        out->insert(out->end(), f, f + NF);
    }
}

namespace {

struct Candidate {
    qs_plan_opts o;
    int kmax;
    std::unique_ptr<Plan> plan;
    qs_status rc = QS_OK;
    double pred_ms = 0;
};

// Predicted milliseconds of each candidate: one batched forward over the
// steps of every plan (device buffers on the model's device).
qs_status predict_plans(const qs_costmodel *model, std::vector<Candidate *> &cands, std::string *err)
{
    std::vector<float> X;
    std::vector<size_t> rows;
    std::vector<float> f;
    for (Candidate *c : cands) {
        block_features(*c->plan, &f);
        rows.push_back(f.size() / NF);
        X.insert(X.end(), f.begin(), f.end());
    }
    const size_t B = X.size() / NF;
    std::vector<float> y(B, 0.f);
    if (B > 0) {
        float *dX = nullptr, *dy = nullptr;
        hipStream_t s = costmodel_stream(model);
        int prev_dev = 0;
        (void)hipGetDevice(&prev_dev);
        hipError_t e = hipSetDevice(costmodel_device(model));
        if (e == hipSuccess) e = hipMalloc(&dX, X.size() * sizeof(float));
        if (e == hipSuccess) e = hipMalloc(&dy, B * sizeof(float));
        if (e == hipSuccess) e = hipMemcpyAsync(dX, X.data(), X.size() * sizeof(float), hipMemcpyHostToDevice, s);
        qs_status rc = QS_OK;
        if (e == hipSuccess) rc = qs_costmodel_predict(model, dX, dy, (int)B);
        if (e == hipSuccess && rc == QS_OK) e = hipMemcpyAsync(y.data(), dy, B * sizeof(float), hipMemcpyDeviceToHost, s);
        if (e == hipSuccess && rc == QS_OK) e = hipStreamSynchronize(s);
        if (dX) (void)hipFree(dX);
        if (dy) (void)hipFree(dy);
        (void)hipSetDevice(prev_dev);
        if (e != hipSuccess) { *err = std::string("learned planner: ") + hipGetErrorString(e); return QS_EHIP; }
        if (rc) { *err = "learned planner: cost model prediction failed"; return rc; }
    }
    size_t at = 0;
    for (size_t i = 0; i < cands.size(); ++i) {
        const double amps_ps = std::ldexp(1.0, cands[i]->plan->n) * 1e-9;   // ps -> ms for 2^n amplitudes
        double s = 0;
        for (size_t j = 0; j < rows[i]; ++j) s += std::exp((double)y[at + j]) * amps_ps;
        at += rows[i];
        cands[i]->pred_ms = s;
    }
    return QS_OK;
}

}  // namespace

qs_status build_plan_search(const qs_circuit *c, int kmax, const qs_plan_opts *o, Plan *out, std::string *err)
{
    const bool learned = o && o->planner == 1;
    if (learned && !o->cost_model) { *err = "qs_fuse: planner 1 (learned) needs a cost model"; return QS_EINVAL; }
    auto t0 = std::chrono::steady_clock::now();
    qs_plan_opts base = *o;
    base.planner = 0;
    base.cost_model = nullptr;

    // the heuristic plan: the fallback and the reference the others must beat
    Candidate heur;
    heur.o = base;
    heur.kmax = kmax;
    heur.plan.reset(new Plan());
    qs_status rc = build_plan(c, kmax, &heur.o, heur.plan.get(), err);
    if (rc) return rc;

    std::vector<int> Cs, rs, Ls, ks;
    if (base.chunk_qubits) Cs = {base.chunk_qubits};
    else Cs = {11, 12, 13};
    if (base.reg_qubits) rs = {base.reg_qubits};
    else rs = {3, 4, 5};
    if (base.low_qubits) Ls = {base.low_qubits};
    else Ls = {3, 4, 5};
    for (int k = std::max(1, kmax - 3); k <= kmax; ++k) ks.push_back(k);
    std::vector<int> mfs{base.no_mfma};
    if (base.dtype == QS_C64 && !base.no_mfma) mfs.push_back(1);     // matrix cores on and off
    // block contents too: single-qubit gates split (phase, shear rotation, phase) or kept
    // whole (grouped 2x2 products, which also fuse into wider dense ops)
    std::vector<int> sps{base.no_split};
    if (!base.no_split && base.enable_fusion) sps.push_back(1);
    std::vector<Candidate> cands;
    for (int C : Cs)
        for (int r : rs)
            for (int L : Ls)
                for (int k : ks)
                    for (int nm : mfs)
                        for (int ns : sps) {
                            Candidate cd;
                            cd.o = base;
                            cd.o.chunk_qubits = C;
                            cd.o.reg_qubits = r;
                            cd.o.low_qubits = L;
                            cd.o.no_mfma = nm;
                            cd.o.no_split = ns;
                            cd.kmax = k;
                            cands.push_back(std::move(cd));
                        }
    // candidate plans are independent: build them on a few host threads
    const int nthr = (int)std::max(1u, std::min(8u, std::thread::hardware_concurrency()));
    std::vector<std::thread> pool;
    std::vector<std::string> errs(cands.size());
    for (int t = 0; t < nthr; ++t)
        pool.emplace_back([&, t]() {
            for (size_t i = t; i < cands.size(); i += nthr) {
                cands[i].plan.reset(new Plan());
                try {
                    cands[i].rc = build_plan(c, cands[i].kmax, &cands[i].o, cands[i].plan.get(), &errs[i]);
                } catch (...) {
                    cands[i].rc = QS_ENOMEM;
                }
            }
        });
    for (auto &th : pool) th.join();
    // keep valid, distinct geometries (the planner may widen r or clip C and L)
    std::vector<Candidate *> keep{&heur};
    std::vector<std::array<int, 6>> seen{{heur.plan->C, heur.plan->r, heur.plan->L, std::min(kmax, heur.plan->r),
                                          heur.plan->mfma ? 1 : 0, base.no_split}};
    for (Candidate &cd : cands) {
        if (cd.rc) continue;
        std::array<int, 6> sig{cd.plan->C, cd.plan->r, cd.plan->L, std::min(cd.kmax, cd.plan->r), cd.plan->mfma ? 1 : 0,
                               cd.o.no_split};
        if (std::find(seen.begin(), seen.end(), sig) != seen.end()) continue;
        seen.push_back(sig);
        keep.push_back(&cd);
    }
    Candidate *best = &heur;
    if (!learned) {
        // the paper's objective (Eq. 7): fewest passes over the state; ties keep the
        // earlier candidate (the heuristic first), then the fewer flops
        auto passes = [](const Candidate *cd) { return cd->plan->stats.blocks + cd->plan->stats.swap_passes; };
        for (Candidate *cd : keep)
            if (passes(cd) < passes(best) ||
                (passes(cd) == passes(best) && cd->plan->stats.flops_per_amp < best->plan->stats.flops_per_amp))
                best = cd;
        *out = std::move(*best->plan);
        qs_plan_stats &s = out->stats;
        s.planner = 3;
        s.candidates = (int)keep.size();
        out->plan_seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        s.plan_seconds = out->plan_seconds;
        return QS_OK;
    }
    std::string perr;
    rc = predict_plans(o->cost_model, keep, &perr);
    if (rc != QS_OK) {
        // no silent fallback: the caller asked for the learned planner
        *err = "qs_fuse: cost-model prediction failed: " + perr;
        return rc;
    }
    if (std::isfinite(heur.pred_ms)) {
        for (Candidate *cd : keep)
            if (std::isfinite(cd->pred_ms) && cd->pred_ms < best->pred_ms) best = cd;
        // fallback: a candidate replaces the heuristic only for a predicted gain of at least 2 %
        if (!(best->pred_ms < 0.98 * heur.pred_ms)) best = &heur;
    }
    *out = std::move(*best->plan);
    qs_plan_stats &s = out->stats;
    s.planner = (best == &heur) ? 0 : 1;
    s.candidates = (int)keep.size();
    s.predicted_ms = (rc == QS_OK) ? best->pred_ms : -1.0;
    s.predicted_heuristic_ms = (rc == QS_OK) ? heur.pred_ms : -1.0;
    out->plan_seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    s.plan_seconds = out->plan_seconds;
    return QS_OK;
}

}  // namespace qs

extern "C" qs_status qs_plan_block_features(const qs_plan *plan, float *host_out, int cap, int *nblocks)
{
    if (!plan || !nblocks) { qs::set_error("qs_plan_block_features: null argument"); return QS_EINVAL; }
    std::vector<float> f;
    qs::block_features(plan->p, &f);
    const int B = (int)(f.size() / QS_COST_FEATURES);
    *nblocks = B;
    if (host_out) std::memcpy(host_out, f.data(), (size_t)std::min(B, std::max(cap, 0)) * QS_COST_FEATURES * sizeof(float));
    return QS_OK;
}
