// sd_plan: grouping, per-group Clifford synthesis, device program compile.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>

#include "device_types.h"
#include "sd_internal.h"

using namespace sd;

extern "C" void sd_plan_options_default(sd_plan_options *o) {
    if (!o) return;
    o->skip_rule = 1;
    o->tile_log2_c64 = 13;
    o->tile_log2_c128 = 13;
    o->coalesce_log2_c64 = 4;
    o->coalesce_log2_c128 = 3;
    o->mode = SD_MODE_TILES;
    o->coalesce_min_log2_c64 = 2;
    o->tile_shrink_c64 = 1;
    o->small_state_tiles = 1;
}

namespace {

inline bool commute(const Term &a, const Term &b) {
    return ((popc(a.x & b.z) + popc(b.x & a.z)) & 1) == 0;
}

// Greedy partition (Sec. "Partitioning Hamiltonian Terms"): first fit in term
// order, i.e. greedy colouring of the anticommutation graph.
std::vector<std::vector<int64_t>> first_fit(const std::vector<Term> &T) {
    std::vector<std::vector<int64_t>> groups;
    for (int64_t k = 0; k < (int64_t)T.size(); ++k) {
        bool placed = false;
        for (auto &g : groups) {
            bool ok = true;
            for (int64_t j : g)
                if (!commute(T[k], T[j])) {
                    ok = false;
                    break;
                }
            if (ok) {
                g.push_back(k);
                placed = true;
                break;
            }
        }
        if (!placed) groups.push_back({k});
    }
    return groups;
}

}  // namespace

extern "C" sd_status sd_plan(const sd_hamiltonian *h, const sd_plan_options *opt_in,
                             sd_plan_t **out) {
    if (!h || !out) return fail(SD_ERR_ARG, "sd_plan: null argument");
    *out = nullptr;
    sd_plan_options opt;
    sd_plan_options_default(&opt);
    if (opt_in) opt = *opt_in;
    auto chk = [](int v, int lo, int hi) { return v >= lo && v <= hi; };
    if (!chk(opt.tile_log2_c64, kMinTileLog2, kMaxTileLog2) ||
        !chk(opt.tile_log2_c128, kMinTileLog2, kMaxTileLog2) ||
        !chk(opt.coalesce_log2_c64, 0, 6) || !chk(opt.coalesce_log2_c128, 0, 6) ||
        opt.coalesce_log2_c64 >= opt.tile_log2_c64 ||
        opt.coalesce_log2_c128 >= opt.tile_log2_c128 || opt.coalesce_min_log2_c64 < 0)
        return fail(SD_ERR_RANGE, "sd_plan: tile/coalescing options out of range");
    if (opt.mode != SD_MODE_TILES && opt.mode != SD_MODE_PAPER_LAYERS && opt.mode != SD_MODE_TERMWISE)
        return fail(SD_ERR_ARG, "sd_plan: unknown mode");
    auto t0 = std::chrono::steady_clock::now();
    sd_plan_t *p = new sd_plan_s();
    p->n = h->n;
    p->terms = h->terms;
    p->groups = first_fit(p->terms);

    // paper circuit per group (export, validation, cost model)
    SynthOptions so;
    so.skip_rule = opt.skip_rule != 0;
    so.step_i = true;
    int64_t model = 0;
    for (auto &g : p->groups) {
        std::vector<Row> rows;
        for (int64_t k : g) rows.push_back({p->terms[k].x, p->terms[k].z, 0});
        SynthResult r = synthesize(p->n, rows, so);
        if (!r.ok) {
            std::string e = r.error;
            delete p;
            return fail(SD_ERR_INTERNAL, "sd_plan: paper synthesis failed: " + e);
        }
        std::vector<int32_t> flat;
        for (auto &gt : r.gates) {
            flat.push_back(gt.kind);
            flat.push_back(gt.a);
            flat.push_back(gt.b);
        }
        model += 2 * (r.n_h_first + r.n_cnot_controls + r.n_diag + r.n_h_last) + 1;
        p->circuits.push_back(std::move(r));
        p->gate_flat.push_back(std::move(flat));
    }
    p->paper_model_passes = model;
    p->mode = opt.mode;
    build_layers(*p);

    auto compile = [&](int d, int D, Program *out) {
        return d == SD_C64 ? compile_program(p->n, p->terms, p->groups, D, opt.coalesce_log2_c64,
                                             std::min(opt.coalesce_min_log2_c64, opt.coalesce_log2_c64),
                                             out, opt.tile_shrink_c64 != 0)
                           : compile_program(p->n, p->terms, p->groups, D, opt.coalesce_log2_c128,
                                             opt.coalesce_log2_c128, out, false);
    };
    sd_status st = SD_OK;
    for (int d = 0; d < 2 && st == SD_OK; ++d) {
        const int D = d == SD_C64 ? opt.tile_log2_c64 : opt.tile_log2_c128;
        const int coal = d == SD_C64 ? opt.coalesce_log2_c64 : opt.coalesce_log2_c128;
        st = compile(d, D, &p->prog[d]);
        // A state of fewer than kLatencyTiles tiles leaves most CUs idle and
        // each pass waits on the latency of one tile: take the smallest tile
        // of at least 2^kTileMinLog2Fast that needs no more passes.
        if (st != SD_OK || !opt.small_state_tiles || p->n - std::min(D, p->n) >= kLatencyTilesLog2) continue;
        for (int Dt = kTileMinLog2Fast; Dt < std::min(D, p->n); ++Dt) {
            if (coal >= Dt) continue;
            Program alt;
            if (compile(d, Dt, &alt) != SD_OK) continue;
            if (alt.passes.size() <= p->prog[d].passes.size()) {
                p->prog[d] = std::move(alt);
                break;
            }
        }
    }
    if (st != SD_OK) {
        delete p;
        return st;
    }
    // workspace: packed pass tables for both dtypes, the layer-mode diagonal
    // tables, then the reduction scratch
    int64_t off = 0;
    for (int d = 0; d < 2; ++d) {
        p->ws_off_prog[d] = off;
        off += (pack_size(p->prog[d]) + 255) / 256 * 256;
    }
    p->ws_off_layers = off;
    off += (int64_t)(p->layer_data.size() * sizeof(uint64_t) + 255) / 256 * 256;
    p->ws_off_scratch = off;
    off += 64 * 1024;  // FP64 partial sums
    // per-term expectations: per-block partials, then one value per pass term
    p->ws_off_terms = off;
    {
        int64_t most = 0;
        for (int d = 0; d < 2; ++d) {
            int64_t t = 0;
            for (auto &ps : p->prog[d].passes) t += (int64_t)ps.terms.size();
            most = std::max(most, t);
        }
        off += ((int64_t)kTermGrid * kMaxPassTerms + most) * 8;
        off = (off + 255) / 256 * 256;
    }
    p->ws_needed = off;
    p->plan_seconds =
        std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    *out = p;
    return SD_OK;
}

extern "C" sd_status sd_plan_info_get(const sd_plan_t *p, sd_plan_info *info) {
    if (!p || !info) return fail(SD_ERR_ARG, "sd_plan_info_get: null argument");
    info->n_qubits = p->n;
    info->n_terms = (int64_t)p->terms.size();
    info->n_groups = (int32_t)p->groups.size();
    int64_t mx = 0;
    for (auto &g : p->groups) mx = std::max<int64_t>(mx, (int64_t)g.size());
    info->max_group_terms = mx;
    info->passes_c64 = (int32_t)p->prog[SD_C64].passes.size();
    info->passes_c128 = (int32_t)p->prog[SD_C128].passes.size();
    info->paper_model_passes = p->paper_model_passes;
    info->workspace_bytes = p->ws_needed;
    info->plan_seconds = p->plan_seconds;
    return SD_OK;
}

extern "C" sd_status sd_plan_export_group(const sd_plan_t *p, int32_t g, sd_group_view *v) {
    if (!p || !v) return fail(SD_ERR_ARG, "sd_plan_export_group: null argument");
    if (g < 0 || g >= (int32_t)p->groups.size())
        return fail(SD_ERR_RANGE, "sd_plan_export_group: group index out of range");
    const SynthResult &r = p->circuits[g];
    v->n_terms = (int32_t)p->groups[g].size();
    v->term_ids = p->groups[g].data();
    v->zmask = r.zmask.data();
    v->sign = r.sign.data();
    v->n_gates = (int32_t)r.gates.size();
    v->gates = p->gate_flat[g].data();
    v->n_independent = (int32_t)r.independent.size();
    // independent indices are positions within the group; export term ids
    static thread_local std::vector<int64_t> ind;
    ind.clear();
    for (int64_t i : r.independent) ind.push_back(p->groups[g][i]);
    v->independent = ind.data();
    return SD_OK;
}

extern "C" sd_status sd_plan_pass_count(const sd_plan_t *p, sd_dtype dt, int32_t *count) {
    if (!p || !count) return fail(SD_ERR_ARG, "sd_plan_pass_count: null argument");
    if (dt != SD_C64 && dt != SD_C128) return fail(SD_ERR_ARG, "bad dtype");
    *count = (int32_t)p->prog[dt].passes.size();
    return SD_OK;
}

extern "C" sd_status sd_plan_export_pass(const sd_plan_t *p, sd_dtype dt, int32_t i,
                                         sd_pass_view *v) {
    if (!p || !v) return fail(SD_ERR_ARG, "sd_plan_export_pass: null argument");
    if (dt != SD_C64 && dt != SD_C128) return fail(SD_ERR_ARG, "bad dtype");
    const auto &P = p->prog[dt].passes;
    if (i < 0 || i >= (int32_t)P.size()) return fail(SD_ERR_RANGE, "pass index out of range");
    v->group = P[i].group;
    v->n_terms = (int32_t)P[i].terms.size();
    v->term_ids = P[i].terms.data();
    v->rho = P[i].rho;
    v->tile_log2 = P[i].D;
    v->basis = P[i].basis.data();
    v->coalesce_log2 = P[i].c;
    v->free_mask = P[i].free_mask;
    v->pivot_vec = P[i].u.data();
    v->pivot_coord = P[i].mr.data();
    v->cz_s = P[i].B.data();
    v->zeta = P[i].zeta.data();
    v->ztile = P[i].ztile.data();
    v->coef = P[i].coef.data();
    v->z_sign = P[i].zq;
    return SD_OK;
}

extern "C" sd_status sd_plan_export_rounds(const sd_plan_t *p, sd_dtype dt, int32_t i,
                                           sd_round_view *v) {
    if (!p || !v) return fail(SD_ERR_ARG, "sd_plan_export_rounds: null argument");
    if (dt != SD_C64 && dt != SD_C128) return fail(SD_ERR_ARG, "bad dtype");
    const auto &P = p->prog[dt].passes;
    if (i < 0 || i >= (int32_t)P.size()) return fail(SD_ERR_RANGE, "pass index out of range");
    const PassHost &h = P[i];
    v->n_rounds = h.nr;
    v->lam_round = h.lam_round;
    for (int r = 0; r < 4; ++r) {
        for (int b = 0; b < 4; ++b) {
            v->reg[r][b] = h.reg[r][b];
            v->regpost[r][b] = h.regpost[r][b];
        }
        for (int x = 0; x < 2; ++x) v->xl[r][x] = h.xl[r][x];
        v->nx[r] = h.nx[r];
        v->bmask[r] = h.bmask[r];
        v->iflag[r] = h.iflag[r];
        v->dflag[r] = h.dflag[r];
        v->later[r] = h.later[r];
        v->lanes[r] = h.lanes[r].data();
        v->lanes_post[r] = h.lanes_post[r].data();
    }
    v->bucket = h.bucket.data();
    v->n_lanes = (int32_t)h.lanes[0].size();
    v->io_coalesced = h.io_k;
    for (int j = 0; j < 4; ++j) v->swz[j] = h.swz[j];
    v->staged = h.staged ? 1 : 0;
    v->shift0 = h.shift0 ? 1 : 0;
    for (int r = 0; r < 4; ++r) v->czmask[r] = h.czm[r];
    return SD_OK;
}

extern "C" void sd_plan_destroy(sd_plan_t *p) { delete p; }
