// Facet conditions on the sweep (Section 2.1 with fixed facets; Section 4.3).
//
// Requiring K_j = 1 on a facet set I and K_j = 0 on a set J cuts the span of
// the kernel basis down to an affine coset: writing K = B x, the conditions
// are the linear system B_I x = 1, B_J x = 0 over F2.  Its solutions are a
// particular solution x* plus the null space of B_{I u J}; the complexes are
// K* + span{B y : y in that null space} with K* = B x*.  The sweep then walks
// the null-space coordinates and adds K* to every state.

#include <cstring>

#include "internal.h"

namespace wpm {

int facet_conditions(int n, int m, const uint32_t *facets, int32_t M, const uint32_t *basis,
                     int32_t k, const uint32_t *forced_in, const uint32_t *forced_out,
                     uint32_t *basis_out, int32_t *k_out, uint32_t *offset_out, int32_t *feasible) {
    if (!k_out || !feasible || !offset_out || k < 0 || k > WPM_MAX_K ||
        (k > 0 && (!basis || !basis_out)))
        return WPM_EINVAL;
    int st = validate_facets(n, m, facets, M);
    if (st) return st;
    const int W = (M + 31) / 32;
    auto bit = [](const uint32_t *v, int j) { return v ? (v[j / 32] >> (j % 32)) & 1u : 0u; };
    // masks must not name facets >= M, nor put a facet on both sides
    for (int w = 0; w < W; ++w) {
        const uint32_t valid = (w == W - 1 && M % 32) ? ((1u << (M % 32)) - 1) : ~0u;
        const uint32_t a = forced_in ? forced_in[w] : 0u, b = forced_out ? forced_out[w] : 0u;
        if ((a | b) & ~valid) return WPM_EINVAL;
        if (a & b) return WPM_EINVAL;
    }
    // One equation per conditioned facet: row = coefficients over x (k bits),
    // rhs = required value of K_j.
    struct Eq {
        uint64_t row;
        uint32_t rhs;
    };
    std::vector<Eq> eqs;
    for (int j = 0; j < M; ++j) {
        const uint32_t in = bit(forced_in, j), out = bit(forced_out, j);
        if (!in && !out) continue;
        uint64_t row = 0;
        for (int t = 0; t < k; ++t)
            if ((basis[(size_t)t * W + j / 32] >> (j % 32)) & 1u) row |= 1ull << t;
        eqs.push_back({row, in});
    }
    // Gauss-Jordan elimination; pivots on the highest coordinate of each row.
    std::vector<Eq> piv;   // reduced rows, distinct pivot bits
    std::vector<int> pbit;
    for (Eq e : eqs) {
        for (size_t r = 0; r < piv.size(); ++r)
            if ((e.row >> pbit[r]) & 1ull) {
                e.row ^= piv[r].row;
                e.rhs ^= piv[r].rhs;
            }
        if (!e.row) {
            if (e.rhs) {  // 0 = 1: no complex satisfies the conditions
                *feasible = 0;
                *k_out = 0;
                std::memset(offset_out, 0, sizeof(uint32_t) * W);
                return WPM_OK;
            }
            continue;
        }
        const int b = 63 - __builtin_clzll(e.row);
        for (size_t r = 0; r < piv.size(); ++r)
            if ((piv[r].row >> b) & 1ull) {
                piv[r].row ^= e.row;
                piv[r].rhs ^= e.rhs;
            }
        piv.push_back(e);
        pbit.push_back(b);
    }
    *feasible = 1;
    // Particular solution: free coordinates 0, each pivot coordinate = its rhs.
    uint64_t is_piv = 0, xs = 0;
    for (size_t r = 0; r < piv.size(); ++r) {
        is_piv |= 1ull << pbit[r];
        if (piv[r].rhs) xs |= 1ull << pbit[r];
    }
    std::vector<uint32_t> off(W, 0u);
    for (int t = 0; t < k; ++t)
        if ((xs >> t) & 1ull)
            for (int w = 0; w < W; ++w) off[w] ^= basis[(size_t)t * W + w];
    std::memcpy(offset_out, off.data(), sizeof(uint32_t) * W);
    // Null space: one vector per free coordinate f, y = e_f + the pivot
    // coordinates whose reduced row contains f.
    int kk = 0;
    for (int f = 0; f < k; ++f) {
        if ((is_piv >> f) & 1ull) continue;
        uint64_t y = 1ull << f;
        for (size_t r = 0; r < piv.size(); ++r)
            if ((piv[r].row >> f) & 1ull) y |= 1ull << pbit[r];
        uint32_t *v = basis_out + (size_t)kk * W;
        std::memset(v, 0, sizeof(uint32_t) * W);
        for (int t = 0; t < k; ++t)
            if ((y >> t) & 1ull)
                for (int w = 0; w < W; ++w) v[w] ^= basis[(size_t)t * W + w];
        ++kk;
    }
    *k_out = kk;
    return WPM_OK;
}

}  // namespace wpm
