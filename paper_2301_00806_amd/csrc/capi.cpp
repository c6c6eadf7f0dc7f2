// extern "C" entry points declared in include/wpm.h.
#include "internal.h"

namespace wpm {
int enumerate(const wpm_batch *b, const wpm_sched *s, uint64_t *d_surv, uint64_t cap,
              uint64_t *d_counts, uint64_t *d_total, uint64_t *d_stats, void *stream);
int enumerate_noalloc(const wpm_batch *b, const wpm_sched *s, uint64_t *d_surv, uint64_t cap,
                      uint64_t *d_counts, uint64_t *d_total, uint64_t *d_stats, void *stream);
int collect(const wpm_host_instance *insts, int32_t num, const uint64_t *d_surv, uint64_t cap,
            const uint64_t *d_counts, const uint64_t *d_total, uint64_t *h_counts, uint32_t *h_out,
            int64_t out_cap, int64_t *out_words, int64_t *h_offsets, void *stream);
int device_query(int32_t *num_cus, int64_t *wallclock_khz, int32_t *lds_per_block);
int persistent_grid(const wpm_batch *b, int wg_size, int32_t *grid);
const char *last_hip_error();
int64_t mlp_work_floats(int B);
int valu_probe_run(int op, int waves_per_simd, int iters, double *lane_ops_per_s);
int mlp_forward_launch(const float *params, const float *norm, const float *X, int B, float *Y,
                       void *stream);
int mlp_grad_launch(const float *params, const float *norm, const float *X, const float *T, int B,
                    float *grad, float *work, float *loss, void *stream);
int mlp_adam_launch(float *params, const float *grad, float *m, float *v, int step, float lr,
                    float beta1, float beta2, float eps, float weight_decay, void *stream);
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

int wpm_convenient_basis(int n, int m, const uint32_t *facets, int32_t M, const uint32_t *basis,
                         int32_t k, int32_t min_free, uint32_t *basis_out, wpm_blocks *blocks) {
    return wpm::convenient_basis(n, m, facets, M, basis, k, min_free, basis_out, blocks);
}

int wpm_idcm_orbits(int n, int p, uint32_t *lam_out, int64_t cap, int64_t *count) {
    return wpm::idcm_orbits(n, p, lam_out, cap, count);
}

int wpm_complex_filters(int n, int m, int64_t num, const int64_t *offsets,
                        const uint32_t *facets, uint8_t *flags) {
    return wpm::complex_filters(n, m, num, offsets, facets, flags);
}

int wpm_iso_classes(int m, int64_t num, const int64_t *offsets, const uint32_t *facets,
                    int64_t *class_of, int64_t *num_classes) {
    return wpm::iso_classes(m, num, offsets, facets, class_of, num_classes);
}

int wpm_facet_conditions(int n, int m, const uint32_t *facets, int32_t M, const uint32_t *basis,
                         int32_t k, const uint32_t *forced_in, const uint32_t *forced_out,
                         uint32_t *basis_out, int32_t *k_out, uint32_t *offset_out,
                         int32_t *feasible) {
    return wpm::facet_conditions(n, m, facets, M, basis, k, forced_in, forced_out, basis_out,
                                 k_out, offset_out, feasible);
}

int wpm_pack_instance(int n, int m, const uint32_t *facets, int32_t M, const uint32_t *basis,
                      int32_t k, const wpm_blocks *blocks, const wpm_conditions *conds,
                      int32_t max_facets, uint64_t seed, uint32_t *table, int64_t cap_words,
                      wpm_instance_info *info) {
    return wpm::pack_instance(n, m, facets, M, basis, k, blocks, conds, max_facets, seed, table,
                              cap_words, info);
}

int wpm_build_queue(const int32_t *k, const float *cost, const int32_t *group, int32_t num,
                    int32_t cbits, int32_t lanes, int32_t min_items_per_instance,
                    int32_t max_items_per_instance, int32_t order, wpm_item *items, int64_t cap,
                    int64_t *n_out, int64_t *items_per_instance) {
    return wpm::build_queue(k, cost, group, num, cbits, lanes, min_items_per_instance,
                            max_items_per_instance, order, items, cap, n_out, items_per_instance);
}

int wpm_build_pruned_queue(const wpm_blocks *blocks, const float *cost, const int32_t *group,
                           int32_t num, int32_t cbits, int32_t lanes,
                           int32_t min_items_per_instance, int32_t max_items_per_instance,
                           int32_t order, wpm_item *items, int64_t cap, int64_t *n_out,
                           int64_t *items_per_instance) {
    return wpm::build_pruned_queue(blocks, cost, group, num, cbits, lanes, min_items_per_instance,
                                   max_items_per_instance, order, items, cap, n_out,
                                   items_per_instance);
}

int wpm_pack_bins(const wpm_item *items, int64_t n, const float *cost, int32_t bins,
                  wpm_item *out_items, int64_t *out_offsets, double *max_load) {
    return wpm::pack_bins(items, n, cost, bins, out_items, out_offsets, max_load);
}

int wpm_enumerate(const wpm_batch *batch, const wpm_sched *sched, uint64_t *d_survivors,
                  uint64_t cap, uint64_t *d_counts, uint64_t *d_total, uint64_t *d_stats,
                  void *stream) {
    return wpm::enumerate(batch, sched, d_survivors, cap, d_counts, d_total, d_stats, stream);
}

int wpm_enumerate_noalloc(const wpm_batch *batch, const wpm_sched *sched, uint64_t *d_survivors,
                          uint64_t cap, uint64_t *d_counts, uint64_t *d_total, uint64_t *d_stats,
                          void *stream) {
    return wpm::enumerate_noalloc(batch, sched, d_survivors, cap, d_counts, d_total, d_stats, stream);
}

int wpm_persistent_grid(const wpm_batch *batch, int32_t wg_size, int32_t *grid) {
    return wpm::persistent_grid(batch, wg_size, grid);
}

int wpm_valu_probe(int op, int waves_per_simd, int iters, double *lane_ops_per_s) {
    return wpm::valu_probe_run(op, waves_per_simd, iters, lane_ops_per_s);
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

int64_t wpm_mlp_work_floats(int32_t batch) { return wpm::mlp_work_floats(batch); }

int wpm_mlp_forward(const float *d_params, const float *d_norm, const float *d_x, int32_t batch,
                    float *d_y, void *stream) {
    return wpm::mlp_forward_launch(d_params, d_norm, d_x, batch, d_y, stream);
}

int wpm_mlp_grad(const float *d_params, const float *d_norm, const float *d_x, const float *d_t,
                 int32_t batch, float *d_grad, float *d_work, float *d_loss, void *stream) {
    return wpm::mlp_grad_launch(d_params, d_norm, d_x, d_t, batch, d_grad, d_work, d_loss, stream);
}

int wpm_mlp_adam(float *d_params, const float *d_grad, float *d_m, float *d_v, int32_t step,
                 float lr, float beta1, float beta2, float eps, float weight_decay, void *stream) {
    return wpm::mlp_adam_launch(d_params, d_grad, d_m, d_v, step, lr, beta1, beta2, eps,
                                weight_decay, stream);
}

}  // extern "C"
