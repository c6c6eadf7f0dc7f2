// Convenient kernel basis and block pruning (Section 2.1).
//
// For a ridge r with parents P(r), only the facets in P(r) contribute to
// (AK)_r, so the rows of the basis matrix B at P(r) decide the degree of r.
// Column operations on B (a change of kernel basis) bring those rows to the
// form [Z | 0]: a few generators ("the block of r") carry everything that
// happens on P(r) and every other generator is zero there.  Then (AK)_r is
// the weight of the block's part of x pushed through Z, and most block
// combinations give a weight above 2, which no weak pseudo-manifold has.
// Repeating this on ridges with pairwise disjoint parent sets, pivoting only
// among the generators not yet in a block, keeps the earlier blocks intact
// and splits the coordinates into blocks I_1..I_l plus free coordinates; the
// sweep then visits the product X_1 x ... x X_l x F2^free instead of F2^k.
//
// The paper's blocks are Z_{m-n}: m-n generators whose restrictions to the
// m-n+1 parents are e_j + e_last, and at most two of them can be combined.
// This engine computes each block's allowed set directly as
//     X_b = { y in F2^{q_b} : |sum_j y_j z_j| <= 2 }
// (z_j = restriction of block generator j to P(r)), which equals the
// "at most two generators" set whenever the restrictions span all even
// vectors on P(r) (the Z_{m-n} case) and stays exact when a ridge has fewer
// parents or its restrictions span less.  Every weak pseudo-manifold has
// (AK)_r in {0, 2}, so it lies in the product: the result set is unchanged.
//
// Coordinate order of the returned basis: the free generators first
// (coordinates 0..f-1), then the blocks in the order they were formed.  The
// Gray-code sweep then walks the free coordinates inside each allowed block
// tuple: for a tuple with high part H (bits f..k-1 of x), the Gray indices
// [g^{-1}(H) 2^f, (g^{-1}(H) + 1) 2^f) cover exactly the x with that high
// part, because the binary-reflected Gray code g maps each aligned range of
// 2^f indices onto one value of the bits above f.

#include <algorithm>
#include <cmath>
#include <cstring>

#include "internal.h"

namespace wpm {

namespace {

constexpr int kMaxParentsForBlock = 9;  // q <= 8: local choice masks fit a byte

// Restriction of a facet-indexed bit vector to the parents of a ridge:
// bit i = entry at the i-th parent.
inline uint32_t restrict_to(const uint64_t *v, const int32_t *par, int p) {
    uint32_t pat = 0;
    for (int i = 0; i < p; ++i) pat |= (uint32_t)((v[par[i] >> 6] >> (par[i] & 63)) & 1ull) << i;
    return pat;
}

inline void xor_into(uint64_t *dst, const uint64_t *src, int MW) {
    for (int w = 0; w < MW; ++w) dst[w] ^= src[w];
}

}  // namespace

int convenient_basis(int n, int m, const uint32_t *facets, int32_t M, const uint32_t *basis,
                     int32_t k, int32_t min_free, uint32_t *basis_out, wpm_blocks *blocks) {
    if (!blocks || min_free < 0 || k < 0 || (k > 0 && (!basis || !basis_out))) return WPM_EINVAL;
    std::memset(blocks, 0, sizeof(*blocks));
    int st = validate_facets(n, m, facets, M);
    if (st) return st;
    if (k > WPM_MAX_K) return WPM_EKMAX;
    const int W = (M + 31) / 32, MW = (M + 63) / 64;
    Incidence inc;
    inc.build(n, facets, M);

    // vec[t]: generator t as MW 64-bit words
    std::vector<uint64_t> vec((size_t)std::max(k, 1) * MW, 0);
    for (int t = 0; t < k; ++t)
        for (int j = 0; j < M; ++j)
            if ((basis[(size_t)t * W + j / 32] >> (j % 32)) & 1u)
                vec[(size_t)t * MW + j / 64] |= 1ull << (j % 64);
    auto V = [&](int t) { return &vec[(size_t)t * MW]; };

    // Ridges that can prune: at least 4 parents (a ridge with p <= 3 can never
    // reach degree 4) and at most kMaxParentsForBlock.  More parents first
    // (larger blocks prune more), then lexicographic ridge order.
    std::vector<int32_t> cand;
    for (int r = 0; r < inc.N; ++r) {
        const int p = inc.parent_off[r + 1] - inc.parent_off[r];
        if (p >= 4 && p <= kMaxParentsForBlock) cand.push_back(r);
    }
    std::stable_sort(cand.begin(), cand.end(), [&](int32_t a, int32_t b) {
        return inc.parent_off[a + 1] - inc.parent_off[a] > inc.parent_off[b + 1] - inc.parent_off[b];
    });

    std::vector<int> free_ids(k);
    for (int t = 0; t < k; ++t) free_ids[t] = t;
    std::vector<std::vector<int>> block_ids;   // generator ids of each block
    std::vector<int32_t> block_ridge;
    std::vector<std::vector<uint8_t>> block_choice;
    std::vector<char> used_facet(M, 0);

    for (int32_t r : cand) {
        if ((int)block_ids.size() >= WPM_MAX_BLOCKS) break;
        if ((int)free_ids.size() - 2 < min_free) break;  // no room for a useful block
        const int32_t *par = &inc.parents[inc.parent_off[r]];
        const int p = inc.parent_off[r + 1] - inc.parent_off[r];
        bool disjoint = true;
        for (int i = 0; i < p; ++i) disjoint = disjoint && !used_facet[par[i]];
        if (!disjoint) continue;

        // Echelon form of the free generators' restrictions: piv[b] = the
        // pattern with leading bit b and the generator that carries it.
        int piv_gen[kMaxParentsForBlock];
        uint32_t piv_pat[kMaxParentsForBlock];
        for (int b = 0; b < p; ++b) piv_gen[b] = -1;
        auto reduce = [&](uint32_t pat, uint64_t *target) {
            for (int b = p - 1; b >= 0 && pat; --b) {
                if (!((pat >> b) & 1u) || piv_gen[b] < 0) continue;
                pat ^= piv_pat[b];
                if (target) xor_into(target, V(piv_gen[b]), MW);
            }
            return pat;
        };
        // Earlier block generators must be zero on P(r) after adding free
        // generators (which are zero on every earlier block's parents, so the
        // earlier blocks keep their shape).  Check before changing anything.
        std::vector<int> pivots;
        {
            // pattern-only elimination to test the span condition
            uint32_t tp[kMaxParentsForBlock];
            int tg[kMaxParentsForBlock];
            for (int b = 0; b < p; ++b) tg[b] = 0;
            auto treduce = [&](uint32_t pat) {
                for (int b = p - 1; b >= 0 && pat; --b)
                    if (((pat >> b) & 1u) && tg[b]) pat ^= tp[b];
                return pat;
            };
            int q = 0;
            for (int id : free_ids) {
                uint32_t pat = treduce(restrict_to(V(id), par, p));
                if (pat) {
                    const int b = 31 - __builtin_clz(pat);
                    tp[b] = pat;
                    tg[b] = 1;
                    ++q;
                }
            }
            if (q < 2) continue;
            if ((int)free_ids.size() - q < min_free) continue;
            bool spans = true;
            for (auto &blk : block_ids)
                for (int id : blk) spans = spans && treduce(restrict_to(V(id), par, p)) == 0u;
            if (!spans) continue;
            // The allowed count is a property of the span alone: the number
            // of its vectors of weight <= 2.  Skip ridges that prune nothing.
            uint32_t span_basis[kMaxParentsForBlock];
            int nb = 0;
            for (int b = 0; b < p; ++b)
                if (tg[b]) span_basis[nb++] = tp[b];
            int allowed = 0;
            for (uint32_t y = 0; y < (1u << q); ++y) {
                uint32_t pat = 0;
                for (int j = 0; j < q; ++j)
                    if ((y >> j) & 1u) pat ^= span_basis[j];
                allowed += __builtin_popcount(pat) <= 2;
            }
            if (allowed == (1 << q)) continue;
        }
        // Eliminate for real: pivots become the block, the other free
        // generators are reduced to zero on P(r).
        std::vector<int> rest;
        for (int id : free_ids) {
            const uint32_t pat = reduce(restrict_to(V(id), par, p), V(id));
            if (pat) {
                const int b = 31 - __builtin_clz(pat);
                piv_pat[b] = pat;
                piv_gen[b] = id;
                pivots.push_back(id);
            } else {
                rest.push_back(id);
            }
        }
        for (auto &blk : block_ids)
            for (int id : blk) reduce(restrict_to(V(id), par, p), V(id));
        // Allowed local combinations: weight of the pushed-through pattern <= 2.
        const int q = (int)pivots.size();
        std::vector<uint32_t> zp(q);
        for (int j = 0; j < q; ++j) zp[j] = restrict_to(V(pivots[j]), par, p);
        std::vector<uint8_t> choice;
        for (uint32_t y = 0; y < (1u << q); ++y) {
            uint32_t pat = 0;
            for (int j = 0; j < q; ++j)
                if ((y >> j) & 1u) pat ^= zp[j];
            if (__builtin_popcount(pat) <= 2) choice.push_back((uint8_t)y);
        }
        if ((int)choice.size() > WPM_MAX_CHOICES) return WPM_ELIMIT;  // cannot happen for p <= 9
        free_ids = rest;
        for (int i = 0; i < p; ++i) used_facet[par[i]] = 1;
        block_ids.push_back(pivots);
        block_ridge.push_back(r);
        block_choice.push_back(choice);
    }

    // Output: free generators, then the blocks.
    std::vector<int> order(free_ids);
    for (auto &blk : block_ids) order.insert(order.end(), blk.begin(), blk.end());
    for (int t = 0; t < k; ++t) {
        uint32_t *dst = basis_out + (size_t)t * W;
        const uint64_t *src = V(order[t]);
        for (int w = 0; w < W; ++w) dst[w] = (uint32_t)(src[w / 2] >> (32 * (w % 2)));
    }
    blocks->k = k;
    blocks->free_dims = (int32_t)free_ids.size();
    blocks->num_blocks = (int32_t)block_ids.size();
    double lv = (double)blocks->free_dims;
    for (size_t b = 0; b < block_ids.size(); ++b) {
        blocks->ridge[b] = block_ridge[b];
        blocks->size[b] = (uint8_t)block_ids[b].size();
        blocks->count[b] = (uint8_t)block_choice[b].size();
        for (size_t c = 0; c < block_choice[b].size(); ++c) blocks->choice[b][c] = block_choice[b][c];
        lv += std::log2((double)block_choice[b].size());
    }
    blocks->log2_vectors = k ? lv : 0.0;
    return WPM_OK;
}

int validate_blocks(const wpm_blocks &b, int32_t k) {
    if (b.k != k || b.num_blocks < 0 || b.num_blocks > WPM_MAX_BLOCKS || b.free_dims < 0)
        return WPM_EINVAL;
    int tot = b.free_dims;
    for (int i = 0; i < b.num_blocks; ++i) {
        const int q = b.size[i], c = b.count[i];
        if (q < 1 || q > 8 || c < 1 || c > WPM_MAX_CHOICES || c > (1 << q)) return WPM_EINVAL;
        for (int j = 0; j < c; ++j)
            if (b.choice[i][j] >= (1u << q) || (j && b.choice[i][j] <= b.choice[i][j - 1]))
                return WPM_EINVAL;
        tot += q;
    }
    return tot == k ? WPM_OK : WPM_EINVAL;
}

}  // namespace wpm
