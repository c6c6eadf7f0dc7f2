// Host-side instance preparation for the weak-pseudo-manifold sweep.
//
// Candidates (Section 4.2: facets of the binary matroid of lambda), ridges and
// the ridge-facet incidence matrix A (Section 2.1), an F2 basis of ker A
// (Section 2.1: every weak pseudo-manifold is one combination B x of a kernel
// basis), and the packed table the GPU sweep reads.
//
// The packed table re-expresses every basis vector in "ridge-slot"
// coordinates.  For a ridge r with p parents (facets containing r), the
// degree of r in a kernel vector K is even (K is in ker A), and the parent bit
// of the last parent is the XOR of the other p-1.  Writing S for the number of
// set bits among the first p-1 parents, deg_r = S + (S mod 2), so
//     deg_r in {0, 2}  <=>  S <= 2.
// Only ridges with p >= 4 can reach degree 4 (Proposition 2.1 needs {0,2});
// these are the critical ridges.  Their first p-1 parent bits are stored
// bit-sliced: slot word q of a 32-ridge group holds, at bit b, the q-th parent
// bit of ridge b of the group.  A basis vector becomes one row of such words,
// so Gray-code XOR of rows keeps every ridge's slots up to date and the check
// "at most 2 of the slots set" runs on 32 ridges per instruction.

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>

#include "../../include/wpm.h"
#include "internal.h"

namespace wpm {

namespace {

inline uint32_t rev32(uint32_t x) {
    x = ((x >> 1) & 0x55555555u) | ((x & 0x55555555u) << 1);
    x = ((x >> 2) & 0x33333333u) | ((x & 0x33333333u) << 2);
    x = ((x >> 4) & 0x0F0F0F0Fu) | ((x & 0x0F0F0F0Fu) << 4);
    x = ((x >> 8) & 0x00FF00FFu) | ((x & 0x00FF00FFu) << 8);
    return (x >> 16) | (x << 16);
}

// Lexicographic order of sorted vertex tuples, for sets of equal size: the
// set owning the smallest element of the symmetric difference comes first,
// which is descending order of the bit-reversed masks.
inline bool lex_before(uint32_t a, uint32_t b) { return rev32(a) > rev32(b); }

inline int popc(uint32_t x) { return __builtin_popcount(x); }

// Rank test of a set of F2^n columns by incremental echelon insertion.
bool spans_full(const uint32_t *cols, int cnt, int n) {
    uint32_t piv[32] = {0};
    int r = 0;
    for (int i = 0; i < cnt; ++i) {
        uint32_t v = cols[i];
        for (int b = n - 1; b >= 0 && v; --b) {
            if (!((v >> b) & 1u)) continue;
            if (piv[b]) {
                v ^= piv[b];
            } else {
                piv[b] = v;
                ++r;
                v = 0;
            }
        }
    }
    return r == n;
}

struct SplitMix {
    uint64_t s;
    uint64_t next() {
        uint64_t z = (s += 0x9E3779B97F4A7C15ull);
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        return z ^ (z >> 31);
    }
};

}  // namespace

int64_t ubt_bound(int n) {
    auto C = [](int a, int b) -> int64_t {
        if (b < 0 || a < b) return 0;
        int64_t r = 1;
        for (int i = 0; i < b; ++i) r = r * (a - i) / (i + 1);
        return r;
    };
    const int up = (n + 1) / 2, dn = n / 2;
    return C(n + 4 - up, 4) + C(n + 3 - dn, 4);
}

int build_candidates(int n, int m, const uint32_t *lambda, uint32_t *facets, int32_t cap,
                     int32_t *M_out) {
    if (!lambda || !M_out || n < 1 || m < n || m > 32 || n > 20) return WPM_EINVAL;
    for (int i = 0; i < m; ++i)
        if (n < 32 && (lambda[i] >> n)) return WPM_EINVAL;
    int idx[32];
    uint32_t cols[32];
    for (int i = 0; i < n; ++i) idx[i] = i;
    int32_t M = 0;
    while (true) {
        for (int i = 0; i < n; ++i) cols[i] = lambda[idx[i]];
        if (spans_full(cols, n, n)) {
            if (facets && M < cap) {
                uint32_t mask = 0;
                for (int i = 0; i < n; ++i) mask |= 1u << idx[i];
                facets[M] = mask;
            }
            ++M;
        }
        int i = n - 1;
        while (i >= 0 && idx[i] == m - n + i) --i;
        if (i < 0) break;
        ++idx[i];
        for (int q = i + 1; q < n; ++q) idx[q] = idx[q - 1] + 1;
    }
    *M_out = M;
    return (M > cap) ? WPM_ECAP : WPM_OK;
}

int validate_facets(int n, int m, const uint32_t *facets, int32_t M) {
    if (n < 2 || m < n || m > 32 || M < 0 || (M > 0 && !facets)) return WPM_EINVAL;
    std::vector<uint32_t> s(facets, facets + M);
    for (uint32_t f : s) {
        if (popc(f) != n) return WPM_EINVAL;
        if (m < 32 && (f >> m)) return WPM_EINVAL;
    }
    std::sort(s.begin(), s.end());
    for (size_t i = 1; i < s.size(); ++i)
        if (s[i] == s[i - 1]) return WPM_EINVAL;
    return WPM_OK;
}

void Incidence::build(int n_, const uint32_t *facets, int32_t M_) {
    n = n_;
    M = M_;
    ridges.clear();
    ridges.reserve((size_t)M * n);
    for (int j = 0; j < M; ++j) {
        uint32_t f = facets[j];
        for (uint32_t rest = f; rest; rest &= rest - 1) ridges.push_back(f & ~(rest & (~rest + 1u)));
    }
    std::sort(ridges.begin(), ridges.end(), lex_before);
    ridges.erase(std::unique(ridges.begin(), ridges.end()), ridges.end());
    N = (int32_t)ridges.size();
    facet_ridges.assign((size_t)M * n, 0);
    std::vector<int32_t> deg(N, 0);
    for (int j = 0; j < M; ++j) {
        uint32_t f = facets[j];
        int i = 0;
        for (uint32_t rest = f; rest; rest &= rest - 1) {
            uint32_t r = f & ~(rest & (~rest + 1u));
            int32_t id = (int32_t)(std::lower_bound(ridges.begin(), ridges.end(), r, lex_before) -
                                   ridges.begin());
            facet_ridges[(size_t)j * n + i++] = id;
            ++deg[id];
        }
    }
    parent_off.assign(N + 1, 0);
    for (int r = 0; r < N; ++r) parent_off[r + 1] = parent_off[r] + deg[r];
    parents.assign(parent_off[N], 0);
    std::vector<int32_t> fill(parent_off.begin(), parent_off.end() - 1);
    for (int j = 0; j < M; ++j)  // facets in increasing order: parent lists come out sorted
        for (int i = 0; i < n; ++i) {
            int32_t r = facet_ridges[(size_t)j * n + i];
            parents[fill[r]++] = j;
        }
}

// Null space of A over F2 by reduction to reduced row echelon form.
int kernel_basis(int n, int m, const uint32_t *facets, int32_t M, uint32_t *ridges_out,
                 int32_t cap_r, int32_t *N_out, uint32_t *basis, int32_t cap_k, int32_t *k_out) {
    if (!N_out || !k_out) return WPM_EINVAL;
    int st = validate_facets(n, m, facets, M);
    if (st) return st;
    Incidence inc;
    inc.build(n, facets, M);
    const int N = inc.N;
    *N_out = N;
    if (ridges_out)
        for (int r = 0; r < N && r < cap_r; ++r) ridges_out[r] = inc.ridges[r];
    const int MW = (M + 63) / 64;
    std::vector<uint64_t> A((size_t)N * MW, 0);
    for (int j = 0; j < M; ++j)
        for (int i = 0; i < n; ++i) {
            int r = inc.facet_ridges[(size_t)j * n + i];
            A[(size_t)r * MW + j / 64] |= 1ull << (j % 64);
        }
    std::vector<int32_t> pivot_col;
    int rank = 0;
    for (int col = 0; col < M && rank < N; ++col) {
        const int w = col / 64;
        const uint64_t bit = 1ull << (col % 64);
        int piv = -1;
        for (int r = rank; r < N; ++r)
            if (A[(size_t)r * MW + w] & bit) { piv = r; break; }
        if (piv < 0) continue;
        if (piv != rank)
            std::swap_ranges(A.begin() + (size_t)piv * MW, A.begin() + (size_t)(piv + 1) * MW,
                             A.begin() + (size_t)rank * MW);
        const uint64_t *pr = &A[(size_t)rank * MW];
        for (int r = 0; r < N; ++r) {
            if (r == rank || !(A[(size_t)r * MW + w] & bit)) continue;
            uint64_t *row = &A[(size_t)r * MW];
            for (int q = w; q < MW; ++q) row[q] ^= pr[q];
        }
        pivot_col.push_back(col);
        ++rank;
    }
    const int k = M - rank;
    *k_out = k;
    if (N > cap_r && ridges_out) return WPM_ECAP;
    if (k > cap_k) return WPM_ECAP;
    if (!basis) return WPM_OK;
    const int W = (M + 31) / 32;
    std::vector<char> is_piv(M, 0);
    for (int c : pivot_col) is_piv[c] = 1;
    int t = 0;
    for (int f = 0; f < M; ++f) {
        if (is_piv[f]) continue;
        uint32_t *v = basis + (size_t)t * W;
        std::memset(v, 0, sizeof(uint32_t) * W);
        v[f / 32] |= 1u << (f % 32);
        for (int i = 0; i < rank; ++i)
            if ((A[(size_t)i * MW + f / 64] >> (f % 64)) & 1ull) {
                const int p = pivot_col[i];
                v[p / 32] |= 1u << (p % 32);
            }
        ++t;
    }
    return WPM_OK;
}

// ---------------------------------------------------------------- packing

namespace {

int slot_stride_for(int q) { return q <= 4 ? 4 : 8; }

}  // namespace

int pack_instance(int n, int m, const uint32_t *facets, int32_t M, const uint32_t *basis,
                  int32_t k, const wpm_blocks *blocks, const wpm_conditions *conds,
                  int32_t max_facets, uint64_t seed, uint32_t *table, int64_t cap_words,
                  wpm_instance_info *info) {
    if (!info) return WPM_EINVAL;
    std::memset(info, 0, sizeof(*info));
    int st = validate_facets(n, m, facets, M);
    if (st) return st;
    if (k < 0 || (k > 0 && !basis) || max_facets < 0) return WPM_EINVAL;
    if (k > WPM_MAX_K) return WPM_EKMAX;
    if (blocks) {
        st = validate_blocks(*blocks, k);
        if (st) return st;
        if (blocks->num_blocks == 0) blocks = nullptr;
    }
    const uint32_t *offset = conds ? conds->offset : nullptr;
    const int nprops = conds ? conds->num_props : 0;
    int nclasses = 0;
    if (nprops < 0 || nprops > WPM_MAX_PROPS) return WPM_EINVAL;
    if (nprops > 0 && (!conds->prop_c0 || !conds->prop_classes || !conds->class_weight ||
                       !conds->class_mask))
        return WPM_EINVAL;
    for (int q = 0; q < nprops; ++q) {
        if (conds->prop_classes[q] < 0) return WPM_EINVAL;
        nclasses += conds->prop_classes[q];
    }
    if (nclasses > WPM_MAX_CLASSES) return WPM_EINVAL;
    const int max_groups = (conds && conds->max_groups) ? conds->max_groups : WPM_MAX_GROUPS;
    if (max_groups < 1 || max_groups > WPM_MAX_GROUPS) return WPM_EINVAL;
    if (offset && blocks) return WPM_EINVAL;  // block choices assume a linear span
    if (M > WPM_MAX_M) return WPM_ELIMIT;
    Incidence inc;
    inc.build(n, facets, M);
    const int W = (M + 31) / 32;

    // Basis membership of each facet: frow[j] bit t = K_t contains facet j;
    // offj[j] = the coset offset K* contains facet j.
    std::vector<uint64_t> frow(M, 0);
    for (int t = 0; t < k; ++t)
        for (int j = 0; j < M; ++j)
            if ((basis[(size_t)t * W + j / 32] >> (j % 32)) & 1u) frow[j] |= 1ull << t;
    std::vector<char> offj(M, 0);
    if (offset)
        for (int j = 0; j < M; ++j) offj[j] = (char)((offset[j / 32] >> (j % 32)) & 1u);

    std::vector<int32_t> crit;
    int maxp = 0;      // over the ridges that can be resident (p - 1 slot words)
    int maxp_all = 0;  // over all critical ridges (sampling buffers)
    for (int r = 0; r < inc.N; ++r) {
        const int p = inc.parent_off[r + 1] - inc.parent_off[r];
        if (p >= 4) {
            crit.push_back(r);
            maxp_all = std::max(maxp_all, p);
            if (p - 1 <= WPM_MAX_SLOTS) maxp = std::max(maxp, p);
        }
    }
    const int n_crit = (int)crit.size();
    const int Q = std::max(3, maxp - 1);
    const int QS = slot_stride_for(Q);

    // Sample the vectors the sweep visits (all of them when there are few),
    // bit-sliced: X[t][s] bit b = coefficient t of sample 64 s + b.  A pruned
    // instance visits only the product of its blocks' allowed sets times the
    // free coordinates, so its samples come from that set.  The filter's
    // pass rate is small (about 1e-3), so its last picks are ranked on the
    // few samples that pass the first ones: large instances, which hold
    // nearly all of a batch's work, get up to 2^18 samples; the sample count
    // scales with the instance (1 per 1024 vectors, at least 8192).
    constexpr double T_MIN = 8192.0, T_MAX = 262144.0;
    int T;
    bool exact = false;
    double visited = std::ldexp(1.0, k);
    if (blocks) {
        visited = std::ldexp(1.0, blocks->free_dims);
        for (int b = 0; b < blocks->num_blocks; ++b) visited *= (double)blocks->count[b];
    }
    const double want = std::min(T_MAX, std::max(T_MIN, visited / 1024.0));
    if (visited <= want) {
        T = (int)visited;
        exact = true;
    } else {
        T = (int)want & ~63;
    }
    const int TW = (T + 63) / 64;
    std::vector<uint64_t> X((size_t)std::max(k, 1) * TW, 0);
    auto put = [&](int s, uint64_t x) {
        for (uint64_t b = x; b; b &= b - 1)
            X[(size_t)__builtin_ctzll(b) * TW + s / 64] |= 1ull << (s % 64);
    };
    SplitMix rng{seed ^ 0x5EEDF00DCAFEull};
    if (!blocks) {
        if (exact) {
            for (int s = 0; s < T; ++s) put(s, (uint64_t)s);
        } else {
            for (int t = 0; t < k; ++t)
                for (int s = 0; s < TW; ++s) X[(size_t)t * TW + s] = rng.next();
        }
    } else {
        const int f = blocks->free_dims;
        const uint64_t fmask = f >= 64 ? ~0ull : (1ull << f) - 1;
        for (int s = 0; s < T; ++s) {
            uint64_t x, idx = (uint64_t)s;
            if (exact) {  // s in mixed radix: free part first, then block 0, 1, ...
                x = idx & fmask;
                idx >>= f;
            } else {
                x = rng.next() & fmask;
            }
            int sh = f;
            for (int b = 0; b < blocks->num_blocks; ++b) {
                const uint64_t cnt = blocks->count[b];
                uint64_t d;
                if (exact) {
                    d = idx % cnt;
                    idx /= cnt;
                } else {
                    d = rng.next() % cnt;
                }
                x |= (uint64_t)blocks->choice[b][d] << sh;
                sh += blocks->size[b];
            }
            put(s, x);
        }
    }
    const uint64_t tail_mask = (T % 64) ? ((1ull << (T % 64)) - 1) : ~0ull;
    // Membership of each facet that is a parent of a critical ridge, over the
    // samples (computed once per facet), then the fail set of every critical
    // ridge: at least 3 of its parents in K, i.e. degree 4 or more.
    std::vector<int32_t> fcol(M, -1);
    int nf = 0;
    for (int c = 0; c < n_crit; ++c) {
        const int r = crit[c];
        for (int q = inc.parent_off[r]; q < inc.parent_off[r + 1]; ++q)
            if (fcol[inc.parents[q]] < 0) fcol[inc.parents[q]] = nf++;
    }
    std::vector<uint64_t> cols((size_t)std::max(nf, 1) * TW);
    for (int j = 0; j < M; ++j) {
        if (fcol[j] < 0) continue;
        uint64_t *cj = cols.data() + (size_t)fcol[j] * TW;
        const uint64_t o = offj[j] ? ~0ull : 0ull;
        for (int s = 0; s < TW; ++s) cj[s] = o;
        for (uint64_t b = frow[j]; b; b &= b - 1) {
            const uint64_t *xt = X.data() + (size_t)__builtin_ctzll(b) * TW;
            for (int s = 0; s < TW; ++s) cj[s] ^= xt[s];
        }
    }
    std::vector<uint64_t> fail((size_t)n_crit * TW, 0);
    {
        std::vector<const uint64_t *> pc(maxp_all);
        for (int c = 0; c < n_crit; ++c) {
            const int r = crit[c];
            const int p0 = inc.parent_off[r], p = inc.parent_off[r + 1] - p0;
            for (int q = 0; q < p; ++q) pc[q] = cols.data() + (size_t)fcol[inc.parents[p0 + q]] * TW;
            uint64_t *fc = fail.data() + (size_t)c * TW;
            for (int s = 0; s < TW; ++s) {
                uint64_t c1 = 0, c2 = 0, c3 = 0;
                for (int q = 0; q < p; ++q) {
                    const uint64_t w = pc[q][s];
                    c3 |= c2 & w;
                    c2 |= c1 & w;
                    c1 |= w;
                }
                fc[s] = c3;
            }
            fc[TW - 1] &= tail_mask;
        }
    }
    std::vector<uint64_t>().swap(cols);
    std::vector<uint64_t>().swap(X);
    // Greedy ordering: repeatedly take the ridge that rejects the most samples
    // still alive; when none rejects any, order the rest by their own
    // rejection counts.  The filter group takes the first (at most) 32 ridges
    // with <= 5 parents (4 slot words); any order is exact.  Only the sample
    // words that still hold an alive sample are scanned.
    std::vector<uint64_t> alive(TW, ~0ull);
    alive[TW - 1] = tail_mask;
    std::vector<int32_t> aw(TW);
    for (int w = 0; w < TW; ++w) aw[w] = w;
    std::vector<int> solo(n_crit, 0);
    for (int c = 0; c < n_crit; ++c) {
        int s = 0;
        for (int w = 0; w < TW; ++w) s += __builtin_popcountll(fail[(size_t)c * TW + w]);
        solo[c] = s;
    }
    std::vector<char> used(n_crit, 0);
    auto greedy_pick = [&](bool need_small) -> int {
        int best = -1, best_gain = -1;
        for (int c = 0; c < n_crit; ++c) {
            if (used[c]) continue;
            const int r = crit[c];
            const int pr = inc.parent_off[r + 1] - inc.parent_off[r];
            if (need_small && pr > 5) continue;
            if (pr - 1 > WPM_MAX_SLOTS) continue;  // too many parents to be resident
            int g = 0;
            const uint64_t *fc = fail.data() + (size_t)c * TW;
            for (int w : aw) g += __builtin_popcountll(fc[w] & alive[w]);
            if (g > best_gain || (g == best_gain && g == 0 && solo[c] > solo[best])) {
                best = c;
                best_gain = g;
            }
        }
        if (best >= 0) {
            used[best] = 1;
            const uint64_t *fb = fail.data() + (size_t)best * TW;
            size_t keep = 0;
            for (int w : aw) {
                alive[w] &= ~fb[w];
                if (alive[w]) aw[keep++] = w;
            }
            aw.resize(keep);
        }
        return best;
    };
    auto count_alive = [&]() {
        int64_t s = 0;
        for (int w : aw) s += __builtin_popcountll(alive[w]);
        return s;
    };
    std::vector<int> filt, rest;
    while ((int)filt.size() < 32) {
        int c = greedy_pick(true);
        if (c < 0) break;
        filt.push_back(c);
    }
    const int64_t alive_filter = count_alive();
    while (true) {
        int c = greedy_pick(false);
        if (c < 0) break;
        rest.push_back(c);
    }
    const int64_t alive_full = count_alive();
    // Resident groups: the filter and the first ridges of the greedy order;
    // the rest of the critical ridges are deferred: the sweep checks them on
    // every vector that passes the resident groups.
    std::vector<int> deferred;
    const size_t resident_rest = (size_t)(max_groups - 1) * 32;
    if (rest.size() > resident_rest) {
        deferred.assign(rest.begin() + (long)resident_rest, rest.end());
        rest.resize(resident_rest);
    }
    for (int c = 0; c < n_crit; ++c)
        if (!used[c]) deferred.push_back(c);  // more than WPM_MAX_SLOTS + 1 parents
    const int G = 1 + (int)((rest.size() + 31) / 32);
    int64_t defer_words = 0;
    for (int c : deferred) defer_words += 1 + (inc.parent_off[crit[c] + 1] - inc.parent_off[crit[c]]);
    const int kp = std::max(k, 7);
    const int RS = ((4 + (G - 1) * QS + W) + 3) & ~3;
    const int nrows = kp + (offset ? 1 : 0);  // the offset row follows the basis rows
    const int64_t props_at = (int64_t)WPM_HDR_WORDS + (int64_t)nrows * RS;
    const int64_t defer_at = props_at + (nprops ? 2 * (int64_t)nprops + (int64_t)nclasses * (1 + W) : 0);
    const int64_t words = defer_at + defer_words;

    info->n = n;
    info->m = m;
    info->M = M;
    info->N = inc.N;
    info->k = k;
    info->W = W;
    info->n_crit = n_crit;
    info->groups = G;
    info->slots = QS;
    info->n_filter = (int)filt.size();
    info->row_words = RS;
    info->max_facets = max_facets;
    info->n_deferred = (int32_t)deferred.size();
    info->table_words = words;
    info->filter_pass = (double)alive_filter / T;
    info->full_pass = (double)alive_full / T;
    cost_features(*info, inc, crit, info->features);
    if (!table || cap_words < words) return WPM_ECAP;

    std::memset(table, 0, sizeof(uint32_t) * (size_t)words);
    uint32_t *h = table;
    h[HDR_MAGIC] = WPM_TABLE_MAGIC;
    h[HDR_K] = (uint32_t)k;
    h[HDR_KP] = (uint32_t)kp;
    h[HDR_M] = (uint32_t)M;
    h[HDR_W] = (uint32_t)W;
    h[HDR_G] = (uint32_t)G;
    h[HDR_QS] = (uint32_t)QS;
    h[HDR_RS] = (uint32_t)RS;
    h[HDR_MAXF] = (uint32_t)max_facets;
    h[HDR_NCRIT] = (uint32_t)n_crit;
    h[HDR_NFILT] = (uint32_t)filt.size();
    h[HDR_FLAGS] = offset ? HDR_FLAG_OFFSET : 0u;
    h[HDR_PROPS] = nprops ? (uint32_t)props_at : 0u;
    h[HDR_NPROPS] = (uint32_t)nprops;
    h[HDR_DEFER] = deferred.empty() ? 0u : (uint32_t)defer_at;
    h[HDR_NDEFER] = (uint32_t)deferred.size();
    uint32_t *rows = table + WPM_HDR_WORDS;
    // slot word (group g, slot q) bit b  <-  parent q of the b-th ridge of group g
    auto place = [&](int c, int word_base, int bit, int slots_used) {
        const int r = crit[c];
        const int p0 = inc.parent_off[r], p = inc.parent_off[r + 1] - p0;
        const int ns = std::min(p - 1, slots_used);
        for (int q = 0; q < ns; ++q) {
            const uint64_t fr = frow[inc.parents[p0 + q]];
            for (uint64_t b = fr; b; b &= b - 1) {
                const int t = __builtin_ctzll(b);
                rows[(size_t)t * RS + word_base + q] |= 1u << bit;
            }
            if (offj[inc.parents[p0 + q]]) rows[(size_t)kp * RS + word_base + q] |= 1u << bit;
        }
    };
    for (size_t b = 0; b < filt.size(); ++b) place(filt[b], 0, (int)b, 4);
    for (size_t i = 0; i < rest.size(); ++i) {
        const int g = 1 + (int)(i / 32), b = (int)(i % 32);
        place(rest[i], 4 + (g - 1) * QS, b, QS);
    }
    // A group of 4 slot words (a, b, c, d) is stored as (a, a^b, c, c^d): an
    // invertible linear change of coordinates, so Gray-code XOR updates still
    // apply, under which "at least 3 of a, b, c, d" takes two 3-input logic ops.
    auto transform4 = [&](int base) {
        auto one = [&](int t) {
            uint32_t *r = rows + (size_t)t * RS + base;
            r[1] ^= r[0];
            r[3] ^= r[2];
        };
        for (int t = 0; t < k; ++t) one(t);
        if (offset) one(kp);  // linear, so it applies to the offset as well
    };
    transform4(0);
    if (QS == 4)
        for (int g = 1; g < G; ++g) transform4(4 + (g - 1) * QS);
    const int koff = 4 + (G - 1) * QS;
    for (int t = 0; t < k; ++t)
        for (int w = 0; w < W; ++w) rows[(size_t)t * RS + koff + w] = basis[(size_t)t * W + w];
    if (offset)
        for (int w = 0; w < W; ++w) rows[(size_t)kp * RS + koff + w] = offset[w];
    // property section: c0, class count, then (weight, W mask words) per class
    uint32_t *pr = table + props_at;
    for (int q = 0, cls = 0; q < nprops; ++q) {
        *pr++ = (uint32_t)conds->prop_c0[q];
        *pr++ = (uint32_t)conds->prop_classes[q];
        for (int c = 0; c < conds->prop_classes[q]; ++c, ++cls) {
            *pr++ = (uint32_t)conds->class_weight[cls];
            for (int w = 0; w < W; ++w) *pr++ = conds->class_mask[(size_t)cls * W + w];
        }
    }
    // deferred ridges: parent count, then the parents' facet indices
    uint32_t *dr = table + defer_at;
    for (int c : deferred) {
        const int r = crit[c];
        const int p0 = inc.parent_off[r], p = inc.parent_off[r + 1] - p0;
        *dr++ = (uint32_t)p;
        for (int q = 0; q < p; ++q) *dr++ = (uint32_t)inc.parents[p0 + q];
    }
    return WPM_OK;
}

}  // namespace wpm
