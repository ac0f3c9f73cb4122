// Layer-by-layer execution plan: the paper's circuit of each group turned into
// HBM passes as the paper's implementation does it (Sec. "Implementations"):
// one pass per H gate, one per run of CNOTs sharing a control (the fan-out is
// a single swap of amplitude pairs), one for all S and CZ gates, one for the
// diagonal exponential Lambda, then the same layers reversed for C^dagger
// (S becomes S^dagger; H, CNOT and CZ are their own inverses).
#include <cmath>
#include <cstring>

#include "sd_internal.h"

namespace sd {

namespace {
uint64_t dbits(double v) {
    uint64_t u;
    std::memcpy(&u, &v, 8);
    return u;
}
}  // namespace

void build_layers(sd_plan_s &p) {
    p.layers.assign(p.groups.size(), {});
    p.layer_data.clear();
    for (size_t g = 0; g < p.groups.size(); ++g) {
        const SynthResult &r = p.circuits[g];
        std::vector<LayerOp> fwd;
        int n_h = 0;
        // CZ pairs are collected per control into the current diagonal layer
        std::vector<std::pair<int, uint64_t>> cz;
        LayerOp diag;
        diag.kind = LayerOp::DIAG;
        bool diag_open = false;
        auto close_diag = [&]() {
            if (!diag_open) return;
            diag.cz_off = (int64_t)p.layer_data.size();
            diag.cz_n = (int64_t)cz.size();
            for (auto &pr : cz) {
                p.layer_data.push_back((uint64_t)pr.first);
                p.layer_data.push_back(pr.second);
            }
            fwd.push_back(diag);
            cz.clear();
            diag = LayerOp();
            diag.kind = LayerOp::DIAG;
            diag_open = false;
        };
        for (const Gate &gt : r.gates) {
            if (gt.kind == SD_GATE_H) {
                close_diag();
                LayerOp op;
                op.kind = LayerOp::H;
                op.a = gt.a;
                fwd.push_back(op);
                ++n_h;
            } else if (gt.kind == SD_GATE_CNOT) {
                close_diag();
                if (!fwd.empty() && fwd.back().kind == LayerOp::CNOT_FAN && fwd.back().a == gt.a) {
                    fwd.back().mask |= 1ull << gt.b;
                } else {
                    LayerOp op;
                    op.kind = LayerOp::CNOT_FAN;
                    op.a = gt.a;
                    op.mask = 1ull << gt.b;
                    fwd.push_back(op);
                }
            } else {
                diag_open = true;
                if (gt.kind == SD_GATE_S) {
                    diag.smask ^= 1ull << gt.a;   // S twice on a qubit is Z: kept exact below
                    diag.s_sign = 1;
                    if (!((diag.smask >> gt.a) & 1)) cz.push_back({gt.a, 1ull << gt.a});
                } else {
                    bool merged = false;
                    for (auto &pr : cz)
                        if (pr.first == gt.a) {
                            pr.second ^= 1ull << gt.b;
                            merged = true;
                            break;
                        }
                    if (!merged) cz.push_back({gt.a, 1ull << gt.b});
                }
            }
        }
        close_diag();
        // the diagonal exponential in the rotated frame, with the exact 2^-#H
        LayerOp lam;
        lam.kind = LayerOp::DIAG;
        lam.lam_off = (int64_t)p.layer_data.size();
        lam.lam_n = (int64_t)p.groups[g].size();
        for (size_t k = 0; k < p.groups[g].size(); ++k) {
            const double c = p.terms[p.groups[g][k]].c * (r.sign[k] ? -1.0 : 1.0);
            p.layer_data.push_back(r.zmask[k]);
            p.layer_data.push_back(dbits(c));
        }
        lam.scale = std::ldexp(1.0, -n_h);
        std::vector<LayerOp> &out = p.layers[g];
        out = fwd;
        out.push_back(lam);
        for (auto it = fwd.rbegin(); it != fwd.rend(); ++it) {
            LayerOp op = *it;
            if (op.kind == LayerOp::DIAG) op.s_sign = -op.s_sign;
            out.push_back(op);
        }
    }
}

}  // namespace sd
