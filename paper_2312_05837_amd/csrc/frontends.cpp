// Problem front-ends (host code): QUBO, MaxCut and NAE-3SAT written as the Ising
// primal problem E(s) = s^T J s + h^T s of Sec. II, for the benchmark problem
// classes of Sec. IV-D (Table 3).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdlib>
#include <vector>

#include "ising.h"

namespace {

struct Triple {
    int32_t r, c;
    double v;
};

// Symmetric CSR from (row, col, value) triples (both directions already present):
// duplicates summed, explicit zeros dropped, columns ascending within a row.
void build_csr(int32_t n, std::vector<Triple> &t, std::vector<int32_t> &rp, std::vector<int32_t> &col,
               std::vector<double> &val) {
    std::sort(t.begin(), t.end(), [](const Triple &a, const Triple &b) { return a.r != b.r ? a.r < b.r : a.c < b.c; });
    rp.assign((size_t)n + 1, 0);
    col.clear();
    val.clear();
    for (size_t k = 0; k < t.size();) {
        size_t e = k;
        double s = 0.0;
        while (e < t.size() && t[e].r == t[k].r && t[e].c == t[k].c) s += t[e++].v;
        if (s != 0.0) {
            col.push_back(t[k].c);
            val.push_back(s);
            ++rp[(size_t)t[k].r + 1];
        }
        k = e;
    }
    for (int32_t i = 0; i < n; ++i) rp[(size_t)i + 1] += rp[i];
}

}  // namespace

extern "C" {

ising_status ising_from_qubo(int32_t n, const double *Q, const double *c, double *J_out, double *h_out,
                             double *offset_out) {
    if (n <= 0 || !Q || !J_out || !h_out || !offset_out) return ISING_EINVAL;
    const size_t N = (size_t)n;
    double total = 0.0, diag = 0.0, csum = 0.0;
    for (size_t i = 0; i < N; ++i) {
        double row = 0.0;
        for (size_t j = 0; j < N; ++j) {
            const double q = 0.5 * (Q[i * N + j] + Q[j * N + i]);  // symmetrised
            if (!std::isfinite(q)) return ISING_EINVAL;
            row += q;
            J_out[i * N + j] = i == j ? 0.0 : 0.25 * q;
        }
        const double ci = c ? c[i] : 0.0;
        if (!std::isfinite(ci)) return ISING_EINVAL;
        h_out[i] = 0.5 * (row + ci);
        total += row;
        diag += Q[i * N + i];
        csum += ci;
    }
    *offset_out = 0.25 * (total + diag) + 0.5 * csum;
    return ISING_OK;
}

ising_status ising_from_maxcut(int32_t n, int64_t m, const int32_t *edges, const double *w, int32_t *row_ptr,
                               int32_t *col, double *val, int64_t *nnz_out, double *total_weight) {
    if (n <= 0 || m < 0 || (m > 0 && !edges) || !nnz_out) return ISING_EINVAL;
    std::vector<Triple> t;
    t.reserve((size_t)(2 * m));
    double W = 0.0;
    for (int64_t k = 0; k < m; ++k) {
        const int32_t a = edges[2 * k], b = edges[2 * k + 1];
        const double x = w ? w[k] : 1.0;
        if (a < 0 || b < 0 || a >= n || b >= n || a == b || !std::isfinite(x)) return ISING_EINVAL;
        t.push_back({a, b, x});
        t.push_back({b, a, x});
        W += x;
    }
    std::vector<int32_t> rp, cl;
    std::vector<double> vl;
    build_csr(n, t, rp, cl, vl);
    *nnz_out = (int64_t)cl.size();
    if (total_weight) *total_weight = W;
    if (!row_ptr) return ISING_OK;  // sizing call
    if (!col || !val) return ISING_EINVAL;
    std::copy(rp.begin(), rp.end(), row_ptr);
    std::copy(cl.begin(), cl.end(), col);
    std::copy(vl.begin(), vl.end(), val);
    return ISING_OK;
}

ising_status ising_from_nae3sat(int32_t n, int64_t m, const int32_t *lits, int32_t *row_ptr, int32_t *col,
                                int32_t *val, int64_t *nnz_out, int64_t *base_out) {
    if (n <= 0 || m < 0 || (m > 0 && !lits) || !nnz_out) return ISING_EINVAL;
    std::vector<Triple> t;
    t.reserve((size_t)(6 * m));
    int64_t K = 0;
    static const int P[3][2] = {{0, 1}, {1, 2}, {0, 2}};
    for (int64_t k = 0; k < m; ++k) {
        int32_t v[3], sg[3];
        for (int u = 0; u < 3; ++u) {
            const int32_t l = lits[3 * k + u];
            if (l == 0 || std::abs((int64_t)l) > n) return ISING_EINVAL;
            v[u] = std::abs(l) - 1;
            sg[u] = l > 0 ? 1 : -1;
        }
        for (const auto &pq : P) {
            const int a = pq[0], b = pq[1];
            if (v[a] == v[b]) {
                K += 2 * sg[a] * sg[b];  // s_v^2 = 1: a constant term
            } else {
                t.push_back({v[a], v[b], (double)(sg[a] * sg[b])});
                t.push_back({v[b], v[a], (double)(sg[a] * sg[b])});
            }
        }
    }
    std::vector<int32_t> rp, cl;
    std::vector<double> vl;
    build_csr(n, t, rp, cl, vl);
    *nnz_out = (int64_t)cl.size();
    if (base_out) *base_out = K + 2 * m;
    if (!row_ptr) return ISING_OK;  // sizing call
    if (!col || !val) return ISING_EINVAL;
    std::copy(rp.begin(), rp.end(), row_ptr);
    std::copy(cl.begin(), cl.end(), col);
    for (size_t k = 0; k < vl.size(); ++k) val[k] = (int32_t)vl[k];
    return ISING_OK;
}

}  // extern "C"
