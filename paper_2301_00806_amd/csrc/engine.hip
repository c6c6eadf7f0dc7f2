// Device side of the ABI: launches of the sweep and collection of results.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cstdio>
#include <cstring>
#include <memory>
#include <mutex>
#include <thread>
#include <vector>

#include "internal.h"
#include "launch.h"

namespace wpm {

namespace {
thread_local char g_hip_err[256] = "no HIP error";

__global__ void zero_u64(unsigned long long *p, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0ull;
}

int hip_fail(const char *what, hipError_t e) {
    set_hip_error(what, (int)e, hipGetErrorString(e));
    return WPM_EHIP;
}

#define HIP_TRY(expr)                                   \
    do {                                                \
        hipError_t _e = (expr);                         \
        if (_e != hipSuccess) return hip_fail(#expr, _e); \
    } while (0)

int zero(void *p, int64_t n, hipStream_t st) {
    if (!p || n <= 0) return WPM_OK;
    const int bs = 256;
    const int64_t nb = (n + bs - 1) / bs;
    hipLaunchKernelGGL(zero_u64, dim3((unsigned)nb), dim3(bs), 0, st, (unsigned long long *)p, n);
    HIP_TRY(hipGetLastError());
    return WPM_OK;
}

// Waves per SIMD of the kernel a schedule asks for (0: the default, 8).
int pick_waves(int w) { return w == 7 ? 7 : 8; }
}  // namespace

void set_hip_error(const char *what, int code, const char *text) {
    std::snprintf(g_hip_err, sizeof(g_hip_err), "%s: %d (%s)", what, code, text ? text : "?");
}

const char *last_hip_error() { return g_hip_err; }

int device_query(int32_t *num_cus, int64_t *wallclock_khz, int32_t *lds_per_block) {
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    int v = 0;
    if (num_cus) {
        HIP_TRY(hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev));
        *num_cus = v;
    }
    if (wallclock_khz) {
        HIP_TRY(hipDeviceGetAttribute(&v, hipDeviceAttributeWallClockRate, dev));
        *wallclock_khz = v;
    }
    if (lds_per_block) {
        HIP_TRY(hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
        *lds_per_block = v;
    }
    return WPM_OK;
}

int persistent_grid_waves(const wpm_batch *b, int wg_size, int waves, int32_t *grid);

int persistent_grid(const wpm_batch *b, int wg_size, int32_t *grid) {
    return persistent_grid_waves(b, wg_size, 0, grid);
}

int persistent_grid_waves(const wpm_batch *b, int wg_size, int waves, int32_t *grid) {
    if (!b || !grid || wg_size < 64 || wg_size > 512 || (wg_size % 64)) return WPM_EINVAL;
    if (b->max_row_words < 4 || b->max_row_words > WPM_MAX_ROW_WORDS || (b->max_row_words & 3)) return WPM_EINVAL;
    if (b->max_kp < 7 || b->max_kp > WPM_MAX_K) return WPM_EINVAL;
    const size_t lds = sweep_lds_bytes(b->max_kp, b->max_row_words, wg_size);
    int32_t cus = 0;
    int rc = device_query(&cus, nullptr, nullptr);
    if (rc) return rc;
    int nb = 0;
    HIP_TRY(occupancy_sweep(pick_waves(waves), &nb, wg_size, lds));
    *grid = std::max(1, nb) * cus;
    return WPM_OK;
}

namespace {
// The sweep with the dynamic queue's head at d_head (device, >= 2 words).
int enumerate_with(const wpm_batch *b, const wpm_sched *s, uint64_t *d_surv, uint64_t cap,
                   uint64_t *d_counts, uint64_t *d_total, uint64_t *d_stats, uint64_t *d_head,
                   void *stream) {
    if (!b || !s || !d_counts || !d_total || (cap > 0 && !d_surv)) return WPM_EINVAL;
    if (b->num_instances < 0 || !b->d_tables || !b->d_offsets) return WPM_EINVAL;
    if (b->max_row_words < 4 || b->max_row_words > WPM_MAX_ROW_WORDS || (b->max_row_words & 3))
        return WPM_EINVAL;
    if (b->max_kp < 7 || b->max_kp > WPM_MAX_K) return WPM_EINVAL;
    if (s->wg_size < 64 || s->wg_size > 512 || (s->wg_size % 64)) return WPM_EINVAL;
    if (s->num_items < 0 || (s->num_items > 0 && !s->d_items)) return WPM_EINVAL;
    if (s->mode < WPM_SCHED_PLAIN || s->mode > WPM_SCHED_PACKED) return WPM_EINVAL;
    if (s->mode == WPM_SCHED_PACKED && (!s->d_bin_offsets || s->grid < 1)) return WPM_EINVAL;
    if (s->mode == WPM_SCHED_PLAIN && s->num_items > 0 && !s->h_items) return WPM_EINVAL;
    if (s->mode == WPM_SCHED_DYNAMIC && !d_head) return WPM_EINVAL;
    if (s->waves_per_simd != 0 && s->waves_per_simd != 7 && s->waves_per_simd != 8) return WPM_EINVAL;
    hipStream_t st = (hipStream_t)stream;
    const int waves = pick_waves(s->waves_per_simd);
    const size_t lds = sweep_lds_bytes(b->max_kp, b->max_row_words, s->wg_size);
    int32_t lds_max = 0;
    if (cap >= (UINT64_MAX >> 2)) return WPM_EINVAL;
    int rc = device_query(nullptr, nullptr, &lds_max);
    if (rc) return rc;
    if (lds > (size_t)lds_max) return WPM_ELIMIT;

    int st_rc;
    if (!(s->flags & WPM_FLAG_ACCUMULATE)) {
        if ((st_rc = zero(d_counts, b->num_instances, st))) return st_rc;
        if ((st_rc = zero(d_total, WPM_TOTAL_WORDS, st))) return st_rc;
        if ((st_rc = zero(d_stats, 8, st))) return st_rc;
    }
    if (d_head && (st_rc = zero(d_head, 2, st))) return st_rc;
    if (s->num_items == 0) return WPM_OK;

    KArgs a;
    std::memset(&a, 0, sizeof(a));
    a.num_items = s->num_items;
    a.head = (unsigned long long *)d_head;
    a.surv = d_surv;
    a.cap = cap;
    a.counts = (unsigned long long *)d_counts;
    a.total = (unsigned long long *)d_total;
    a.stats = (unsigned long long *)d_stats;
    a.times = s->d_item_times;
    a.bins = s->d_bin_offsets;
    a.num_instances = b->num_instances;
    a.max_rs = b->max_row_words;
    a.max_kp = b->max_kp;
    // persistent workgroups reserve output slots in chunks (few global
    // atomics); one-shot workgroups of the plain mode reserve exactly
    a.chunk = (s->mode == WPM_SCHED_PLAIN) ? 0 : 128;
    const dim3 block((unsigned)s->wg_size);
    if (s->mode == WPM_SCHED_PLAIN) {
        // One launch per instance: a grid of exactly that instance's items
        // (items naming an unknown instance are rejected before any launch;
        // the kernel skips and counts any other malformed item).
        for (int64_t i = 0; i < s->num_items; ++i)
            if ((int64_t)s->h_items[i].instance >= (int64_t)b->num_instances) return WPM_EINVAL;
        a.mode = 0;
        int64_t i = 0;
        while (i < s->num_items) {
            int64_t e = i;
            while (e < s->num_items && s->h_items[e].instance == s->h_items[i].instance) ++e;
            a.item_base = i;
            a.num_items = e;
            const int64_t nb = e - i;
            HIP_TRY(launch_sweep(waves, dim3((unsigned)nb), block, lds, st, b->d_tables, b->d_offsets,
                                 s->d_items, a));
            i = e;
        }
        return WPM_OK;
    }
    int32_t grid = s->grid;
    if (grid <= 0 && (rc = persistent_grid_waves(b, s->wg_size, waves, &grid))) return rc;
    a.mode = (s->mode == WPM_SCHED_STATIC) ? 1 : (s->mode == WPM_SCHED_DYNAMIC) ? 2 : 3;
    HIP_TRY(launch_sweep(waves, dim3((unsigned)grid), block, lds, st, b->d_tables, b->d_offsets,
                         s->d_items, a));
    return WPM_OK;
}

// Scratch of the allocation-free entry point: the dynamic queue's head.
// Each device holds its own copy of this array (its host-side name is not a
// device address); its address on a device is looked up once, with that
// device current, and every call on the device shares it.
static __device__ __align__(256) unsigned long long scratch[WPM_STATIC_SCRATCH_WORDS];

constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[MAX_DEVICES] = {};

int scratch_on_current_device(uint64_t **out) {
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= MAX_DEVICES) return WPM_ELIMIT;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) return WPM_EHIP;
        g_scratch_ptr[dev] = p;
    }
    *out = (uint64_t *)g_scratch_ptr[dev];
    return WPM_OK;
}
}  // namespace

int enumerate(const wpm_batch *b, const wpm_sched *s, uint64_t *d_surv, uint64_t cap,
              uint64_t *d_counts, uint64_t *d_total, uint64_t *d_stats, void *stream) {
    if (!s) return WPM_EINVAL;
    return enumerate_with(b, s, d_surv, cap, d_counts, d_total, d_stats, (uint64_t *)s->d_scratch, stream);
}

int enumerate_noalloc(const wpm_batch *b, const wpm_sched *s, uint64_t *d_surv, uint64_t cap,
                      uint64_t *d_counts, uint64_t *d_total, uint64_t *d_stats, void *stream) {
    if (!s || s->d_scratch) return WPM_EINVAL;  // the scratch is the library's own
    // scratch words this schedule needs: the queue head of the dynamic mode
    const int64_t need = s->mode == WPM_SCHED_DYNAMIC ? 2 : 0;
    if (need > WPM_STATIC_SCRATCH_WORDS) return WPM_ELIMIT;
    uint64_t *head = nullptr;
    if (need) {
        const int rc = scratch_on_current_device(&head);
        if (rc) return rc;
    }
    return enumerate_with(b, s, d_surv, cap, d_counts, d_total, d_stats, head, stream);
}

namespace {

// Run fn(i) for i in [0, num) on up to 16 host threads (dynamic chunks of
// `grain`).
template <class Fn>
void host_parallel_for(int64_t num, Fn fn, int64_t grain = 16) {
    const int hw = (int)std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
    const int nt = (int)std::min<int64_t>(hw, std::max<int64_t>(1, (num + grain - 1) / grain));
    std::atomic<int64_t> next{0};
    auto work = [&]() {
        for (;;) {
            const int64_t a = next.fetch_add(grain);
            if (a >= num) break;
            for (int64_t i = a; i < std::min(num, a + grain); ++i) fn(i);
        }
    };
    std::vector<std::thread> th;
    for (int t = 1; t < nt; ++t) th.emplace_back(work);
    work();
    for (auto &t : th) t.join();
}

// One instance's facets in increasing vertex-mask order, and its basis (and
// coset offset) with the facet bits moved to those positions: the set bits of
// a complex's bit vector, read in increasing position, are then its facets in
// increasing mask order.
struct SortedFacets {
    int W = 0;
    std::vector<uint32_t> mask;   // [M] facet masks, increasing
    std::vector<uint32_t> basis;  // [k][W] permuted basis rows
    std::vector<uint32_t> off;    // [W] permuted offset (zero for a subspace)
};

SortedFacets sort_facets(const wpm_host_instance &in) {
    SortedFacets sf;
    const int M = in.M, W = (M + 31) / 32;
    sf.W = W;
    std::vector<int32_t> order(M);
    for (int j = 0; j < M; ++j) order[j] = j;
    std::sort(order.begin(), order.end(), [&](int32_t a, int32_t b) { return in.facets[a] < in.facets[b]; });
    std::vector<int32_t> pos(M);
    sf.mask.resize(M);
    for (int r = 0; r < M; ++r) {
        pos[order[r]] = r;
        sf.mask[r] = in.facets[order[r]];
    }
    auto permute = [&](const uint32_t *src, uint32_t *dst) {
        for (int w = 0; w < W; ++w)
            for (uint32_t v = src[w]; v; v &= v - 1) {
                const int r = pos[w * 32 + __builtin_ctz(v)];
                dst[r >> 5] |= 1u << (r & 31);
            }
    };
    sf.basis.assign((size_t)in.k * W, 0u);
    for (int t = 0; t < in.k; ++t) permute(in.basis + (size_t)t * W, sf.basis.data() + (size_t)t * W);
    sf.off.assign((size_t)W, 0u);
    if (in.offset) permute(in.offset, sf.off.data());
    return sf;
}

// Canonical order of two complexes given as permuted bit vectors (facets in
// increasing mask order): lexicographic order of their facet lists, a list
// that is a prefix of another coming first.  At the lowest differing position
// j the complex holding j continues with facet j; the other continues with a
// later facet (j comes first) or has ended (it comes first).
inline bool canon_less(const uint32_t *A, const uint32_t *B, int W) {
    for (int w = 0; w < W; ++w) {
        const uint32_t d = A[w] ^ B[w];
        if (!d) continue;
        const int b = __builtin_ctz(d);
        const bool a_has = (A[w] >> b) & 1u;
        const uint32_t *other = a_has ? B : A;
        const uint32_t above = b == 31 ? 0u : (other[w] >> (b + 1));
        bool more = above != 0u;
        for (int v = w + 1; v < W && !more; ++v) more = other[v] != 0u;
        return a_has == more;
    }
    return false;
}

}  // namespace

// Host expansion of the records into canonical facet lists.  The records are
// grouped by instance with a counting sort (host threads over slot ranges);
// each instance then expands its x values into permuted bit vectors, sorts
// them canonically, and writes [len, facets...] per complex.
int collect(const wpm_host_instance *insts, int32_t num, const uint64_t *d_surv, uint64_t cap,
            const uint64_t *d_counts, const uint64_t *d_total, uint64_t *h_counts, uint32_t *h_out,
            int64_t out_cap, int64_t *out_words, int64_t *h_offsets, void *stream) {
    if (num < 0 || !d_counts || !d_total || !h_counts || !out_words || !h_offsets ||
        (num > 0 && !insts))
        return WPM_EINVAL;
    for (int i = 0; i < num; ++i)
        if (insts[i].M < 0 || insts[i].M > WPM_MAX_M || insts[i].k < 0 || insts[i].k > WPM_MAX_K ||
            (insts[i].k > 0 && !insts[i].basis) || (insts[i].M > 0 && !insts[i].facets))
            return WPM_EINVAL;
    hipStream_t st = (hipStream_t)stream;
    uint64_t tot[WPM_TOTAL_WORDS] = {0, 0, 0, 0};
    HIP_TRY(hipMemcpyAsync(h_counts, d_counts, sizeof(uint64_t) * (size_t)num, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipMemcpyAsync(tot, d_total, sizeof(tot), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    const uint64_t total = tot[0], slots = tot[1];
    if (tot[2] != 0) return WPM_EINVAL;  // the sweep skipped malformed items
    if (slots > cap) {
        *out_words = -(int64_t)slots;  // record slots needed
        return WPM_ECAP;
    }
    uint64_t sum = 0;
    for (int i = 0; i < num; ++i) sum += h_counts[i];
    if (sum != total) return WPM_EINVAL;  // counts and total disagree: corrupted buffers
    // the records: read in place when they are in host memory, else copied
    const uint64_t *rec = d_surv;
    std::unique_ptr<uint64_t[]> rec_copy;  // uninitialised: the copy fills it
    {
        hipPointerAttribute_t attr;
        const bool host = hipPointerGetAttributes(&attr, d_surv) == hipSuccess &&
                          attr.type == hipMemoryTypeHost;
        (void)hipGetLastError();
        if (!host && slots) {
            rec_copy.reset(new uint64_t[2 * slots]);
            HIP_TRY(hipMemcpyAsync(rec_copy.get(), d_surv, sizeof(uint64_t) * 2 * slots, hipMemcpyDefault, st));
            HIP_TRY(hipStreamSynchronize(st));
            rec = rec_copy.get();
        }
    }
    // group the records by instance: per-range histograms, then scatter
    const int64_t ranges = std::max<int64_t>(1, std::min<int64_t>(64, (int64_t)(slots / 65536) + 1));
    const uint64_t per = (slots + ranges - 1) / (uint64_t)ranges;
    std::vector<int64_t> hist((size_t)ranges * (size_t)num, 0);
    std::atomic<int> bad{0};
    host_parallel_for(ranges, [&](int64_t r) {
        int64_t *h = hist.data() + (size_t)r * num;
        const uint64_t e = std::min<uint64_t>(slots, (uint64_t)(r + 1) * per);
        for (uint64_t q = (uint64_t)r * per; q < e; ++q) {
            const uint64_t inst = rec[2 * q + 1];
            if (inst == ~0ull) continue;
            if (inst >= (uint64_t)num) { bad = 1; return; }
            const uint64_t x = rec[2 * q];
            if (insts[inst].k < 64 && (x >> insts[inst].k)) { bad = 1; return; }
            ++h[inst];
        }
    }, 1);
    if (bad) return WPM_EINVAL;
    std::vector<int64_t> start((size_t)num + 1, 0);
    for (int i = 0; i < num; ++i) {
        int64_t c = 0;
        for (int64_t r = 0; r < ranges; ++r) {
            int64_t &h = hist[(size_t)r * num + i];
            const int64_t v = h;
            h = start[i] + c;  // this range's first position for instance i
            c += v;
        }
        if ((uint64_t)c != h_counts[i]) return WPM_EINVAL;
        start[i + 1] = start[i] + c;
    }
    std::unique_ptr<uint64_t[]> xs(new uint64_t[(size_t)std::max<int64_t>(1, start[num])]);
    host_parallel_for(ranges, [&](int64_t r) {
        int64_t *h = hist.data() + (size_t)r * num;
        const uint64_t e = std::min<uint64_t>(slots, (uint64_t)(r + 1) * per);
        for (uint64_t q = (uint64_t)r * per; q < e; ++q) {
            const uint64_t inst = rec[2 * q + 1];
            if (inst != ~0ull) xs[(size_t)h[inst]++] = rec[2 * q];
        }
    }, 1);
    // Per instance: the x values expanded into permuted bit vectors (kept
    // when the lists are to be written) and the words of its lists, one
    // length word plus |K| facets per complex.
    const bool write = h_out != nullptr;
    std::vector<SortedFacets> sfs(write ? (size_t)num : 0);
    std::vector<std::vector<uint32_t>> kvs(write ? (size_t)num : 0);
    std::vector<int64_t> iw((size_t)num, 0);
    host_parallel_for(num, [&](int64_t i) {
        const int64_t n_i = start[i + 1] - start[i];
        if (!n_i) return;
        SortedFacets sf = sort_facets(insts[i]);
        const int W = sf.W;
        std::vector<uint32_t> kv((size_t)n_i * (size_t)std::max(W, 1));
        int64_t w = n_i;
        for (int64_t r = 0; r < n_i; ++r) {
            uint32_t *K = kv.data() + (size_t)r * W;
            for (int q = 0; q < W; ++q) K[q] = sf.off[q];
            for (uint64_t b = xs[(size_t)(start[i] + r)]; b; b &= b - 1) {
                const uint32_t *row = sf.basis.data() + (size_t)__builtin_ctzll(b) * W;
                for (int q = 0; q < W; ++q) K[q] ^= row[q];
            }
            for (int q = 0; q < W; ++q) w += __builtin_popcount(K[q]);
        }
        iw[(size_t)i] = w;
        if (write) {
            sfs[(size_t)i] = std::move(sf);
            kvs[(size_t)i] = std::move(kv);
        }
    });
    xs.reset();
    int64_t words = 0;
    for (int i = 0; i < num; ++i) {
        h_offsets[i] = words;
        words += iw[(size_t)i];
    }
    h_offsets[num] = words;
    *out_words = words;
    if (!write || out_cap < words) return WPM_ECAP;
    // per instance: canonical sort of the bit vectors, then the facet lists
    host_parallel_for(num, [&](int64_t i) {
        const int64_t n_i = start[i + 1] - start[i];
        if (!n_i) return;
        const SortedFacets &sf = sfs[(size_t)i];
        const int W = sf.W;
        std::vector<uint32_t> &kv = kvs[(size_t)i];
        std::vector<int64_t> idx((size_t)n_i);
        for (int64_t r = 0; r < n_i; ++r) idx[(size_t)r] = r;
        std::sort(idx.begin(), idx.end(), [&](int64_t a, int64_t b) {
            return canon_less(kv.data() + (size_t)a * W, kv.data() + (size_t)b * W, W);
        });
        int64_t w = h_offsets[i];
        for (int64_t r : idx) {
            const uint32_t *K = kv.data() + (size_t)r * W;
            uint32_t *len = h_out + w++;
            uint32_t n = 0;
            for (int q = 0; q < W; ++q)
                for (uint32_t v = K[q]; v; v &= v - 1) {
                    h_out[w++] = sf.mask[q * 32 + __builtin_ctz(v)];
                    ++n;
                }
            *len = n;
        }
        std::vector<uint32_t>().swap(kv);
    }, 1);
    return WPM_OK;
}

}  // namespace wpm
