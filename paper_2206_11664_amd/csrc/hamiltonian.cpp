// Hamiltonian construction, error reporting and version string.
#include <cmath>
#include <cstring>
#include <map>
#include <string>
#include <utility>

#include "sd_internal.h"

namespace sd {

static thread_local std::string g_last_error;

sd_status fail(sd_status s, const std::string &msg) {
    g_last_error = msg;
    return s;
}

}  // namespace sd

using namespace sd;

extern "C" const char *sd_last_error(void) { return g_last_error.c_str(); }

extern "C" const char *sd_status_string(sd_status s) {
    switch (s) {
        case SD_OK: return "SD_OK";
        case SD_ERR_ARG: return "SD_ERR_ARG: invalid argument";
        case SD_ERR_PARSE: return "SD_ERR_PARSE: malformed Pauli string";
        case SD_ERR_RANGE: return "SD_ERR_RANGE: value out of range";
        case SD_ERR_WORKSPACE: return "SD_ERR_WORKSPACE: workspace missing or too small";
        case SD_ERR_HIP: return "SD_ERR_HIP: HIP runtime error";
        case SD_ERR_INTERNAL: return "SD_ERR_INTERNAL: planner self-check failed";
        case SD_ERR_STATE: return "SD_ERR_STATE: object in wrong state";
    }
    return "unknown sd_status";
}

extern "C" const char *sd_version(void) { return "sdiag 0.1 (gfx950)"; }

namespace {

// Binary form of a Pauli string (Sec. "Tableau Representation": X->(1,0),
// Z->(0,1), Y->(1,1)).
sd_status parse_one(const char *s, int n, uint64_t *x, uint64_t *z) {
    *x = *z = 0;
    size_t len = std::strlen(s);
    bool dense = len > 0;
    for (size_t i = 0; i < len; ++i)
        if (!std::strchr("IXYZ", s[i])) {
            dense = false;
            break;
        }
    auto put = [&](char ch, int q) {
        if (ch == 'X' || ch == 'Y') *x |= 1ull << q;
        if (ch == 'Z' || ch == 'Y') *z |= 1ull << q;
    };
    if (dense) {
        if ((int)len != n)
            return fail(SD_ERR_PARSE, "dense Pauli string length " + std::to_string(len) +
                                          " != n_qubits " + std::to_string(n));
        for (int q = 0; q < n; ++q) put(s[q], q);
        return SD_OK;
    }
    uint64_t seen = 0;
    const char *p = s;
    while (*p) {
        while (*p == ' ' || *p == '\t') ++p;
        if (!*p) break;
        char ch = *p++;
        if (!std::strchr("IXYZ", ch))
            return fail(SD_ERR_PARSE, std::string("bad Pauli letter '") + ch + "' in \"" + s + "\"");
        if (*p < '0' || *p > '9')
            return fail(SD_ERR_PARSE, std::string("missing qubit index in \"") + s + "\"");
        long q = 0;
        while (*p >= '0' && *p <= '9') {
            q = q * 10 + (*p - '0');
            if (q > 1000000) break;
            ++p;
        }
        if (*p && *p != ' ' && *p != '\t')
            return fail(SD_ERR_PARSE, std::string("bad token in \"") + s + "\"");
        if (q >= n) return fail(SD_ERR_RANGE, "qubit index " + std::to_string(q) + " >= n_qubits");
        if ((seen >> q) & 1) return fail(SD_ERR_PARSE, std::string("repeated qubit in \"") + s + "\"");
        seen |= 1ull << q;
        put(ch, (int)q);
    }
    return SD_OK;  // an empty / all-whitespace string is the identity
}

sd_status finish(int32_t n, int64_t m, const uint64_t *x, const uint64_t *z,
                 const double *c, sd_hamiltonian **out) {
    sd_hamiltonian *h = new sd_hamiltonian();
    h->n = n;
    // merge exact duplicates at the first occurrence (coefficients summed)
    std::map<std::pair<uint64_t, uint64_t>, size_t> index;
    for (int64_t j = 0; j < m; ++j) {
        auto key = std::make_pair(x[j], z[j]);
        auto it = index.find(key);
        if (it != index.end()) {
            h->terms[it->second].c += c[j];
            continue;
        }
        index.emplace(key, h->terms.size());
        h->terms.push_back({x[j], z[j], c[j], j});
    }
    for (auto &t : h->terms) {
        h->xs.push_back(t.x);
        h->zs.push_back(t.z);
        h->cs.push_back(t.c);
        h->srcs.push_back(t.src);
    }
    *out = h;
    return SD_OK;
}

}  // namespace

extern "C" sd_status sd_hamiltonian_create(int32_t n, int64_t m, const char *const *paulis,
                                           const double *coeffs, sd_hamiltonian **out) {
    if (!out) return fail(SD_ERR_ARG, "sd_hamiltonian_create: out is null");
    *out = nullptr;
    if (n < 1 || n > 63) return fail(SD_ERR_RANGE, "n_qubits must be in 1..63");
    if (m < 0) return fail(SD_ERR_ARG, "n_terms < 0");
    if (m > 0 && (!paulis || !coeffs)) return fail(SD_ERR_ARG, "null term arrays");
    std::vector<uint64_t> x(m), z(m);
    for (int64_t j = 0; j < m; ++j) {
        if (!paulis[j]) return fail(SD_ERR_ARG, "null Pauli string");
        if (!std::isfinite(coeffs[j])) return fail(SD_ERR_ARG, "non-finite coefficient");
        sd_status s = parse_one(paulis[j], n, &x[j], &z[j]);
        if (s != SD_OK) return s;
    }
    return finish(n, m, x.data(), z.data(), coeffs, out);
}

extern "C" sd_status sd_hamiltonian_create_masks(int32_t n, int64_t m, const uint64_t *x,
                                                 const uint64_t *z, const double *c,
                                                 sd_hamiltonian **out) {
    if (!out) return fail(SD_ERR_ARG, "sd_hamiltonian_create_masks: out is null");
    *out = nullptr;
    if (n < 1 || n > 63) return fail(SD_ERR_RANGE, "n_qubits must be in 1..63");
    if (m < 0) return fail(SD_ERR_ARG, "n_terms < 0");
    if (m > 0 && (!x || !z || !c)) return fail(SD_ERR_ARG, "null term arrays");
    const uint64_t all = (1ull << n) - 1;
    for (int64_t j = 0; j < m; ++j) {
        if ((x[j] | z[j]) & ~all) return fail(SD_ERR_RANGE, "mask bit at a qubit >= n_qubits");
        if (!std::isfinite(c[j])) return fail(SD_ERR_ARG, "non-finite coefficient");
    }
    return finish(n, m, x, z, c, out);
}

extern "C" sd_status sd_hamiltonian_terms(const sd_hamiltonian *h, int32_t *n, int64_t *m,
                                          const uint64_t **x, const uint64_t **z,
                                          const double **c, const int64_t **src) {
    if (!h) return fail(SD_ERR_ARG, "sd_hamiltonian_terms: null handle");
    if (n) *n = h->n;
    if (m) *m = (int64_t)h->terms.size();
    if (x) *x = h->xs.data();
    if (z) *z = h->zs.data();
    if (c) *c = h->cs.data();
    if (src) *src = h->srcs.data();
    return SD_OK;
}

extern "C" void sd_hamiltonian_destroy(sd_hamiltonian *h) { delete h; }
