// Filters on the enumerated complexes (Algorithm 4.4 after the sweep):
// Picard number, the seedness condition and isomorphism classes, all from
// minimal non-faces (Section 3: seedness from minimal non-faces; isomorphism
// by colour sequences of minimal non-faces).
//
// A complex is a list of facet vertex masks on [m] (m <= 16).  Its faces are
// the subsets of its facets; a minimal non-face (MNF) is a non-face whose
// proper subsets are all faces.  Faces have at most n vertices, so an MNF has
// at most n + 1, and the MNF set determines the complex.

#include <algorithm>
#include <atomic>
#include <cstring>
#include <thread>
#include <string>
#include <unordered_map>
#include <vector>

#include "internal.h"

namespace wpm {

namespace {

// What the filters and the isomorphism test need of one complex.
struct Cx {
    int m = 0;
    uint32_t used = 0;             // vertices that lie in some facet
    std::vector<uint32_t> mnf;     // minimal non-faces, increasing
    std::vector<std::string> col;  // colour sequence of each vertex (MNF sizes, increasing)
    std::string key;               // isomorphism invariant
};

void build(Cx &c, int m, const uint32_t *f, int64_t nf, std::vector<uint8_t> &face) {
    c.m = m;
    const uint32_t full = 1u << m;
    face.assign(full, 0);
    c.used = 0;
    for (int64_t i = 0; i < nf; ++i) {
        const uint32_t s = f[i];
        c.used |= s;
        for (uint32_t sub = s;; sub = (sub - 1) & s) {
            face[sub] = 1;
            if (!sub) break;
        }
    }
    c.mnf.clear();
    for (uint32_t s = 1; s < full; ++s) {
        if (face[s]) continue;
        bool minimal = true;
        for (uint32_t b = s; b && minimal; b &= b - 1) minimal = face[s & ~(b & (0u - b))];
        if (minimal) c.mnf.push_back(s);
    }
    c.col.assign(m, std::string());
    for (int v = 0; v < m; ++v) {
        std::vector<int> sz;
        for (uint32_t s : c.mnf)
            if ((s >> v) & 1u) sz.push_back(__builtin_popcount(s));
        std::sort(sz.begin(), sz.end());
        for (int z : sz) c.col[v].push_back((char)('0' + z));
    }
    std::vector<std::string> cs(c.col);
    std::sort(cs.begin(), cs.end());
    c.key = std::to_string(nf) + ":" + std::to_string(c.mnf.size()) + ":";
    for (auto &x : cs) c.key += x + "|";
}

// Run fn(i, scratch) for i in [0, num) on up to 16 host threads.
template <class Fn>
void parallel_for(int64_t num, Fn fn) {
    const int hw = (int)std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
    const int nt = (int)std::min<int64_t>(hw, std::max<int64_t>(1, num / 256));
    std::atomic<int64_t> next{0};
    auto work = [&]() {
        std::vector<uint8_t> scratch;
        for (;;) {
            const int64_t a = next.fetch_add(256);
            if (a >= num) break;
            const int64_t b = std::min(num, a + 256);
            for (int64_t i = a; i < b; ++i) fn(i, scratch);
        }
    };
    std::vector<std::thread> th;
    for (int t = 1; t < nt; ++t) th.emplace_back(work);
    work();
    for (auto &t : th) t.join();
}

// Is there a bijection phi of [m] with phi(MNF(a)) = MNF(b) that keeps
// colour sequences?  Vertices of a are assigned in order of increasing
// colour-class size; after each assignment, every MNF of a whose vertices
// are all assigned must map onto an MNF of b (b_mnf: membership over 2^m).
bool isomorphic(const Cx &a, const Cx &b, const std::vector<uint8_t> &b_mnf) {
    const int m = a.m;
    if (a.key != b.key) return false;
    std::vector<int> order(m), csz(m, 0);
    for (int v = 0; v < m; ++v) {
        order[v] = v;
        for (int w = 0; w < m; ++w) csz[v] += a.col[w] == a.col[v];
    }
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) {
        if (csz[x] != csz[y]) return csz[x] < csz[y];
        return a.col[x] < a.col[y];
    });
    std::vector<int> rank(m);
    for (int i = 0; i < m; ++i) rank[order[i]] = i;
    // MNFs of a grouped by the position of their last assigned vertex
    std::vector<std::vector<uint32_t>> due(m);
    for (uint32_t s : a.mnf) {
        int last = 0;
        for (uint32_t t = s; t; t &= t - 1) last = std::max(last, rank[__builtin_ctz(t)]);
        due[last].push_back(s);
    }
    std::vector<int> phi(m, -1), next(m, 0);
    uint32_t taken = 0;
    int d = 0;  // depth-first search with an explicit stack of candidates
    while (d >= 0) {
        if (d == m) return true;
        const int v = order[d];
        if (phi[v] >= 0) {  // back from a failed deeper choice: undo this one
            taken &= ~(1u << phi[v]);
            phi[v] = -1;
        }
        bool advanced = false;
        for (int w = next[d]; w < m; ++w) {
            if (((taken >> w) & 1u) || b.col[w] != a.col[v]) continue;
            phi[v] = w;
            bool ok = true;
            for (uint32_t s : due[d]) {
                uint32_t img = 0;
                for (uint32_t t = s; t; t &= t - 1) img |= 1u << phi[__builtin_ctz(t)];
                if (!b_mnf[img]) {
                    ok = false;
                    break;
                }
            }
            if (ok) {
                taken |= 1u << w;
                next[d] = w + 1;
                ++d;
                if (d < m) next[d] = 0;
                advanced = true;
                break;
            }
            phi[v] = -1;
        }
        if (!advanced) {
            next[d] = 0;
            --d;
        }
    }
    return false;
}

int check_list(int m, int64_t num, const int64_t *offsets, const uint32_t *facets) {
    if (m < 1 || m > 16 || num < 0 || (num > 0 && (!offsets || !facets))) return WPM_EINVAL;
    if (num > 0 && offsets[0] != 0) return WPM_EINVAL;
    for (int64_t i = 0; i < num; ++i) {
        if (offsets[i + 1] < offsets[i]) return WPM_EINVAL;
        for (int64_t j = offsets[i]; j < offsets[i + 1]; ++j)
            if (facets[j] >> m) return WPM_EINVAL;
    }
    return WPM_OK;
}

}  // namespace

int complex_filters(int n, int m, int64_t num, const int64_t *offsets, const uint32_t *facets,
                    uint8_t *flags) {
    if (n < 1 || !flags) return WPM_EINVAL;
    int st = check_list(m, num, offsets, facets);
    if (st) return st;
    parallel_for(num, [&](int64_t i, std::vector<uint8_t> &scratch) {
        Cx c;
        const uint32_t *f = facets + offsets[i];
        const int64_t nf = offsets[i + 1] - offsets[i];
        build(c, m, f, nf, scratch);
        uint8_t fl = 0;
        if (__builtin_popcount(c.used) == m) fl |= WPM_CX_FULL_PICARD;
        // seedness: no edge {v, w} of K such that every MNF holds both or neither
        bool seed = true;
        for (int v = 0; v < m && seed; ++v)
            for (int w = v + 1; w < m && seed; ++w) {
                const uint32_t e = (1u << v) | (1u << w);
                bool edge = false;
                for (int64_t j = 0; j < nf && !edge; ++j) edge = (f[j] & e) == e;
                if (!edge) continue;
                bool split = false;
                for (uint32_t s : c.mnf) {
                    const uint32_t h = s & e;
                    if (h != 0 && h != e) {
                        split = true;
                        break;
                    }
                }
                if (!split) seed = false;
            }
        if (seed) fl |= WPM_CX_SEED;
        flags[i] = fl;
    });
    return WPM_OK;
}

int iso_classes(int m, int64_t num, const int64_t *offsets, const uint32_t *facets,
                int64_t *class_of, int64_t *num_classes) {
    if (!class_of || !num_classes) return WPM_EINVAL;
    int st = check_list(m, num, offsets, facets);
    if (st) return st;
    // minimal non-faces, colours and invariant of every complex, in parallel
    std::vector<Cx> all(num);
    parallel_for(num, [&](int64_t i, std::vector<uint8_t> &scratch) {
        build(all[i], m, facets + offsets[i], offsets[i + 1] - offsets[i], scratch);
    });
    // classes in order of first appearance; candidates share the invariant
    std::vector<int64_t> rep_of_class;
    std::vector<std::vector<uint8_t>> rep_mnf;
    std::unordered_map<std::string, std::vector<int64_t>> bucket;
    for (int64_t i = 0; i < num; ++i) {
        auto &ids = bucket[all[i].key];
        int64_t found = -1;
        for (int64_t id : ids)
            if (isomorphic(all[i], all[rep_of_class[id]], rep_mnf[id])) {
                found = id;
                break;
            }
        if (found < 0) {
            found = (int64_t)rep_of_class.size();
            rep_of_class.push_back(i);
            std::vector<uint8_t> mem(1u << m, 0);
            for (uint32_t s : all[i].mnf) mem[s] = 1;
            rep_mnf.push_back(std::move(mem));
            ids.push_back(found);
        }
        class_of[i] = found;
    }
    *num_classes = (int64_t)rep_of_class.size();
    return WPM_OK;
}

}  // namespace wpm
