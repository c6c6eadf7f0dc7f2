// Work decomposition for the sweep and the cost-model features.
//
// The 2^kp Gray indices of an instance (or, for a pruned instance, each
// allowed block tuple's aligned range of 2^f indices) are cut into lane chunks
// of 2^c consecutive indices (c >= 7, so each lane walks whole 64-step blocks
// and every lane of a workgroup flips the same basis vector at the same step).
// An item hands `lanes` consecutive chunks to the lanes of one workgroup.
// Chunks are independent: any split or order of items gives the same counts.

#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>

#include "internal.h"

namespace wpm {

namespace {

// Index whose binary-reflected Gray code is g.
inline uint64_t gray_inverse(uint64_t g) {
    for (int sh = 1; sh < 64; sh <<= 1) g ^= g >> sh;
    return g;
}

// One instance's share of the queue: `subs` aligned sub-cubes of 2^f Gray
// indices (one per allowed block tuple; a single one covering [0, 2^kp) when
// the instance is not pruned), each cut into chunks of 2^c indices.
struct QInst {
    int32_t i, c, f, grp;
    uint64_t subs, chunks, per_sub, ni;  // chunks per sub-cube, items per sub-cube, items
    double item_cost;                    // cost of one full item
    const wpm_blocks *blk;               // NULL: not pruned
};

int queue_impl(const int32_t *k, const wpm_blocks *blocks, const float *cost,
               const int32_t *group, int32_t num, int32_t cbits, int32_t lanes,
               int32_t min_items_per_instance, int32_t max_items_per_instance, int32_t order,
               wpm_item *items, int64_t cap, int64_t *n_out, int64_t *items_per_instance) {
    if ((!k && !blocks) || !n_out || num < 0 || lanes < 1 || lanes > 1024 || cbits < 0 ||
        order < 0 || order > 1)
        return WPM_EINVAL;
    std::vector<QInst> v;
    v.reserve(num);
    int64_t total = 0;
    for (int i = 0; i < num; ++i) {
        if (items_per_instance) items_per_instance[i] = 0;
        const wpm_blocks *bl = blocks ? &blocks[i] : nullptr;
        const int ki = bl ? bl->k : k[i];
        if (ki < 0 || ki > WPM_MAX_K) return WPM_EINVAL;
        if (bl) {
            const int st = validate_blocks(*bl, ki);
            if (st) return st;
            if (bl->num_blocks == 0) bl = nullptr;
        }
        // k = 0: the only kernel vector is x = 0, the empty complex, which is
        // never a result; the instance needs no sweep.
        if (ki == 0) continue;
        int f;
        double subs_d = 1.0;
        if (bl) {
            f = bl->free_dims;
            if (f < 7) return WPM_EINVAL;
            for (int b = 0; b < bl->num_blocks; ++b) subs_d *= (double)bl->count[b];
            if (subs_d > 1e15) return WPM_ELIMIT;
        } else {
            f = std::max(ki, 7);
        }
        const uint64_t subs = (uint64_t)subs_d;
        int c = std::min(std::max(cbits, 7), f);
        // a pruned instance's tuples are separate ranges of 2^f indices: lower
        // the chunk so one tuple still fills whole workgroups
        if (bl) {
            int lanes_log2 = 0;
            while ((1 << lanes_log2) < lanes) ++lanes_log2;
            c = std::min(c, std::max(7, f - lanes_log2));
        }
        auto n_items = [&](int cc) -> double {
            const double per = std::ceil(std::ldexp(1.0, f - cc) / lanes);
            return per * (double)subs;
        };
        // shrink chunks until the instance fills min_items full workgroups ...
        const double want = (double)std::max(1, min_items_per_instance) * (double)lanes;
        while (c > 7 && (double)subs * std::ldexp(1.0, f - c) < want) --c;
        // ... but never split it into more than max_items items
        if (max_items_per_instance > 0)
            while (c < f && n_items(c) > (double)max_items_per_instance) ++c;
        if (n_items(c) > (double)(INT64_MAX / 4)) return WPM_ELIMIT;
        const uint64_t chunks = 1ull << (f - c);
        const uint64_t per_sub = (chunks + lanes - 1) / lanes;
        const uint64_t ni = per_sub * subs;
        total += (int64_t)ni;
        if (items_per_instance) items_per_instance[i] = (int64_t)ni;
        const double cv = cost ? (double)cost[i] : 1.0;
        v.push_back({i, c, f, group ? group[i] : 0, subs, chunks, per_sub, ni,
                     cv * (double)std::min<uint64_t>((uint64_t)lanes, chunks) * std::ldexp(1.0, c),
                     bl});
    }
    *n_out = total;
    if (total > cap || !items) return WPM_ECAP;
    // Groups in decreasing key order; inside a group, instance order or
    // decreasing item cost.  All full items of an instance cost the same, so
    // instance-major emission in cost order is longest-processing-time-first
    // up to the partial last items.
    std::stable_sort(v.begin(), v.end(), [&](const QInst &a, const QInst &b) {
        if (a.grp != b.grp) return a.grp > b.grp;
        return order == 1 && a.item_cost > b.item_cost;
    });
    int64_t w = 0;
    for (const QInst &in : v) {
        int digit[WPM_MAX_BLOCKS] = {0};
        int shift[WPM_MAX_BLOCKS] = {0};
        if (in.blk)
            for (int b = 1; b < in.blk->num_blocks; ++b) shift[b] = shift[b - 1] + in.blk->size[b - 1];
        for (uint64_t sidx = 0; sidx < in.subs; ++sidx) {
            uint64_t base = 0;  // first chunk of this sub-cube
            if (in.blk) {
                uint64_t h = 0;  // x bits f..k-1
                for (int b = 0; b < in.blk->num_blocks; ++b)
                    h |= (uint64_t)in.blk->choice[b][digit[b]] << shift[b];
                base = gray_inverse(h) << (in.f - in.c);
                for (int b = 0; b < in.blk->num_blocks; ++b) {  // mixed-radix increment
                    if (++digit[b] < in.blk->count[b]) break;
                    digit[b] = 0;
                }
            }
            for (uint64_t q = 0; q < in.per_sub; ++q) {
                wpm_item &it = items[w++];
                it.instance = (uint32_t)in.i;
                it.cbits = (uint16_t)in.c;
                const uint64_t off = q * (uint64_t)lanes;
                it.lanes = (uint16_t)std::min<uint64_t>((uint64_t)lanes, in.chunks - off);
                it.first = base + off;
            }
        }
    }
    return WPM_OK;
}

}  // namespace

int build_queue(const int32_t *k, const float *cost, const int32_t *group, int32_t num,
                int32_t cbits, int32_t lanes, int32_t min_items_per_instance,
                int32_t max_items_per_instance, int32_t order, wpm_item *items, int64_t cap,
                int64_t *n_out, int64_t *items_per_instance) {
    if (!k) return WPM_EINVAL;
    return queue_impl(k, nullptr, cost, group, num, cbits, lanes, min_items_per_instance,
                      max_items_per_instance, order, items, cap, n_out, items_per_instance);
}

int build_pruned_queue(const wpm_blocks *blocks, const float *cost, const int32_t *group,
                       int32_t num, int32_t cbits, int32_t lanes, int32_t min_items_per_instance,
                       int32_t max_items_per_instance, int32_t order, wpm_item *items,
                       int64_t cap, int64_t *n_out, int64_t *items_per_instance) {
    if (!blocks && num > 0) return WPM_EINVAL;
    return queue_impl(nullptr, blocks, cost, group, num, cbits, lanes, min_items_per_instance,
                      max_items_per_instance, order, items, cap, n_out, items_per_instance);
}

int pack_bins(const wpm_item *items, int64_t n, const float *cost, int32_t bins,
              wpm_item *out_items, int64_t *out_offsets, double *max_load) {
    if (n < 0 || bins < 1 || (n > 0 && (!items || !out_items)) || !out_offsets) return WPM_EINVAL;
    std::vector<double> c(n);
    for (int64_t i = 0; i < n; ++i)
        c[i] = (cost ? (double)cost[items[i].instance] : 1.0) * (double)items[i].lanes *
               std::ldexp(1.0, items[i].cbits);
    std::vector<int64_t> order(n);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int64_t a, int64_t b) { return c[a] > c[b]; });
    // min-heap of (load, bin)
    std::vector<std::pair<double, int32_t>> heap(bins);
    for (int32_t b = 0; b < bins; ++b) heap[b] = {0.0, b};
    auto cmp = [](const std::pair<double, int32_t> &a, const std::pair<double, int32_t> &b) {
        return a.first > b.first || (a.first == b.first && a.second > b.second);
    };
    std::make_heap(heap.begin(), heap.end(), cmp);
    std::vector<int32_t> bin_of(n);
    std::vector<int64_t> cnt(bins, 0);
    for (int64_t i : order) {
        std::pop_heap(heap.begin(), heap.end(), cmp);
        auto &top = heap.back();
        bin_of[i] = top.second;
        top.first += c[i];
        ++cnt[top.second];
        std::push_heap(heap.begin(), heap.end(), cmp);
    }
    out_offsets[0] = 0;
    for (int32_t b = 0; b < bins; ++b) out_offsets[b + 1] = out_offsets[b] + cnt[b];
    std::vector<int64_t> fill(out_offsets, out_offsets + bins);
    for (int64_t i : order) out_items[fill[bin_of[i]]++] = items[i];  // costly items first in each bin
    if (max_load) {
        double mx = 0;
        for (auto &h : heap) mx = std::max(mx, h.first);
        *max_load = mx;
    }
    return WPM_OK;
}

// Sixteen per-instance features for the cost model, all cheap to compute
// before any sweep:
//   0 n   1 m   2 k   3 log2 M   4 log2 N   5 critical ridges / 32   6 W
//   7 log2(max_facets + 1)   8..12 fraction of ridges with 1, 2, 3, 4, >=5
//   parents   13 groups   14 log10 estimated fast-filter pass rate
//   15 log10 estimated full-check pass rate (both from the packing samples)
void cost_features(const wpm_instance_info &info, const Incidence &inc,
                   const std::vector<int32_t> &crit, float *out) {
    std::memset(out, 0, sizeof(float) * 16);
    out[0] = (float)info.n;
    out[1] = (float)info.m;
    out[2] = (float)info.k;
    out[3] = (float)std::log2(std::max(1, info.M));
    out[4] = (float)std::log2(std::max(1, inc.N));
    out[5] = (float)crit.size() / 32.0f;
    out[6] = (float)info.W;
    out[7] = (float)std::log2((double)info.max_facets + 1.0);
    if (inc.N > 0) {
        int h[5] = {0, 0, 0, 0, 0};
        for (int r = 0; r < inc.N; ++r) {
            const int p = inc.parent_off[r + 1] - inc.parent_off[r];
            h[std::min(std::max(p, 1), 5) - 1]++;
        }
        for (int i = 0; i < 5; ++i) out[8 + i] = (float)h[i] / (float)inc.N;
    }
    out[13] = (float)info.groups;
    out[14] = (float)std::log10(std::max(info.filter_pass, 1e-9));
    out[15] = (float)std::log10(std::max(info.full_pass, 1e-9));
}

}  // namespace wpm
