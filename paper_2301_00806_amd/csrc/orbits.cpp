// IDCM orbits of Lambda(n, p) (Section 4.2).
//
// A matrix [M; I_p] of Lambda(n, p) has n distinct rows that are nonzero and
// not unit vectors (a dual characteristic map is nonzero at every vertex and
// injective), so it is an n-subset of the 2^p - 1 - p vectors of weight >= 2.
// The action of S_n permutes rows (the subset is unchanged) and S_p permutes
// coordinates, so an orbit is a subset up to coordinate permutations.  The
// representative kept is the orbit's least subset (rows sorted increasingly,
// subsets compared lexicographically); subsets are generated in that order and
// one is kept when no coordinate permutation maps it to a smaller one.  Each
// representative is returned as the characteristic matrix [I_n | M].

#include <algorithm>
#include <vector>

#include "internal.h"

namespace wpm {

int idcm_orbits(int n, int p, uint32_t *lam_out, int64_t cap, int64_t *count) {
    if (!count || p < 2 || p > 5 || n < 1 || n > 26) return WPM_EINVAL;
    std::vector<uint32_t> vecs;
    for (uint32_t v = 0; v < (1u << p); ++v)
        if (__builtin_popcount(v) >= 2) vecs.push_back(v);
    const int nv = (int)vecs.size();
    *count = 0;
    if (n > nv) return WPM_OK;
    // all coordinate permutations, as images of each vector
    std::vector<int> perm(p);
    for (int i = 0; i < p; ++i) perm[i] = i;
    std::vector<std::vector<uint32_t>> img;  // img[q][v]
    do {
        std::vector<uint32_t> m(1u << p);
        for (uint32_t v = 0; v < (1u << p); ++v) {
            uint32_t w = 0;
            for (int i = 0; i < p; ++i) w |= ((v >> i) & 1u) << perm[i];
            m[v] = w;
        }
        img.push_back(std::move(m));
    } while (std::next_permutation(perm.begin(), perm.end()));
    std::vector<int> idx(n);
    for (int i = 0; i < n; ++i) idx[i] = i;
    std::vector<uint32_t> S(n), T(n);
    int64_t found = 0;
    const int m = n + p;
    while (true) {
        for (int i = 0; i < n; ++i) S[i] = vecs[idx[i]];  // increasing
        bool least = true;
        for (size_t q = 1; q < img.size() && least; ++q) {
            for (int i = 0; i < n; ++i) T[i] = img[q][S[i]];
            std::sort(T.begin(), T.end());
            least = !std::lexicographical_compare(T.begin(), T.end(), S.begin(), S.end());
        }
        if (least) {
            if (lam_out && found < cap) {
                uint32_t *col = lam_out + (size_t)found * m;
                for (int i = 0; i < n; ++i) col[i] = 1u << i;
                for (int c = 0; c < p; ++c) {
                    uint32_t v = 0;
                    for (int i = 0; i < n; ++i) v |= ((S[i] >> c) & 1u) << i;
                    col[n + c] = v;
                }
            }
            ++found;
        }
        // next n-subset of [nv] in lexicographic order
        int i = n - 1;
        while (i >= 0 && idx[i] == nv - n + i) --i;
        if (i < 0) break;
        ++idx[i];
        for (int j = i + 1; j < n; ++j) idx[j] = idx[j - 1] + 1;
    }
    *count = found;
    return (lam_out && found > cap) ? WPM_ECAP : WPM_OK;
}

}  // namespace wpm
