// extern "C" entry points declared in include/wpm.h.
#include "internal.h"

namespace wpm {
int enumerate(const wpm_batch *b, const wpm_sched *s, uint64_t *d_surv, uint64_t cap,
              uint64_t *d_counts, uint64_t *d_total, uint64_t *d_stats, void *stream);
int collect(const wpm_host_instance *insts, int32_t num, const uint64_t *d_surv, uint64_t cap,
            const uint64_t *d_counts, const uint64_t *d_total, uint64_t *h_counts, uint32_t *h_out,
            int64_t out_cap, int64_t *out_words, int64_t *h_offsets, void *stream);
int device_query(int32_t *num_cus, int64_t *wallclock_khz, int32_t *lds_per_block);
const char *last_hip_error();
}  // namespace wpm

extern "C" {

const char *wpm_strerror(int status) {
    switch (status) {
        case WPM_OK: return "ok";
        case WPM_EINVAL: return "invalid argument";
        case WPM_ECAP: return "buffer too small";
        case WPM_EKMAX: return "kernel dimension above 64";
        case WPM_EHIP: return "HIP runtime error";
        case WPM_ELIMIT: return "instance exceeds engine limits";
        default: return "unknown status";
    }
}

const char *wpm_last_hip_error(void) { return wpm::last_hip_error(); }

int wpm_build_candidates(int n, int m, const uint32_t *lambda, uint32_t *facets, int32_t cap,
                         int32_t *M_out) {
    return wpm::build_candidates(n, m, lambda, facets, cap, M_out);
}

int wpm_kernel_basis(int n, int m, const uint32_t *facets, int32_t M, uint32_t *ridges,
                     int32_t cap_r, int32_t *N_out, uint32_t *basis, int32_t cap_k,
                     int32_t *k_out) {
    return wpm::kernel_basis(n, m, facets, M, ridges, cap_r, N_out, basis, cap_k, k_out);
}

int64_t wpm_ubt_bound(int n) { return wpm::ubt_bound(n); }

int wpm_pack_instance(int n, int m, const uint32_t *facets, int32_t M, const uint32_t *basis,
                      int32_t k, int32_t max_facets, uint64_t seed, uint32_t *table,
                      int64_t cap_words, wpm_instance_info *info) {
    return wpm::pack_instance(n, m, facets, M, basis, k, max_facets, seed, table, cap_words, info);
}

int wpm_build_queue(const int32_t *k, const float *cost, int32_t num, int32_t cbits,
                    int32_t lanes, int32_t min_items_per_instance, int32_t max_items_per_instance,
                    int32_t order, wpm_item *items, int64_t cap, int64_t *n_out) {
    return wpm::build_queue(k, cost, num, cbits, lanes, min_items_per_instance,
                            max_items_per_instance, order, items, cap, n_out);
}

int wpm_enumerate(const wpm_batch *batch, const wpm_sched *sched, uint64_t *d_survivors,
                  uint64_t cap, uint64_t *d_counts, uint64_t *d_total, uint64_t *d_stats,
                  void *stream) {
    return wpm::enumerate(batch, sched, d_survivors, cap, d_counts, d_total, d_stats, stream);
}

int wpm_device_query(int32_t *num_cus, int64_t *wallclock_khz, int32_t *lds_per_block) {
    return wpm::device_query(num_cus, wallclock_khz, lds_per_block);
}

int wpm_collect(const wpm_host_instance *insts, int32_t num, const uint64_t *d_survivors,
                uint64_t cap, const uint64_t *d_counts, const uint64_t *d_total,
                uint64_t *h_counts, uint32_t *h_out, int64_t out_cap, int64_t *out_words,
                int64_t *h_offsets, void *stream) {
    return wpm::collect(insts, num, d_survivors, cap, d_counts, d_total, h_counts, h_out, out_cap,
                        out_words, h_offsets, stream);
}

}  // extern "C"
