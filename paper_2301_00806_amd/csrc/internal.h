// Internal declarations shared by the engine's host sources (not part of the ABI).
#pragma once

#include <cstdint>
#include <vector>

#include "../../include/wpm.h"

namespace wpm {

// Packed instance table: a header of WPM_HDR_WORDS words, then kp rows of
// RS words, one per basis vector t (rows t >= k are zero):
//   [0, 4)                 slot words of the fast-filter group (<= 32 ridges)
//   [4, 4 + (G-1) QS)      slot words of groups 1..G-1, QS words per group
//                          (4-word groups stored as (a, a^b, c, c^d))
//   [4 + (G-1) QS, +W)     the basis vector itself as facet words
// then, for an affine coset, one more row in the same layout holding the
// offset K*, the property section (per property c0, class count, then per
// class its weight and W mask words) and the deferred-ridge section (per
// ridge its parent count, then the parents' facet indices).
constexpr uint32_t WPM_TABLE_MAGIC = 0x314D5057u;  // "WPM1"
constexpr int WPM_HDR_WORDS = 16;
enum {
    HDR_MAGIC = 0,
    HDR_K = 1,
    HDR_KP = 2,    // max(k, 7): the Gray range swept is 2^kp
    HDR_M = 3,
    HDR_W = 4,
    HDR_G = 5,
    HDR_QS = 6,
    HDR_RS = 7,
    HDR_MAXF = 8,
    HDR_NCRIT = 9,
    HDR_NFILT = 10,
    HDR_FLAGS = 11,   // bit 0: row kp holds the offset K* of an affine coset
    HDR_PROPS = 12,   // word offset of the property section (0: none)
    HDR_NPROPS = 13,  // affine properties besides the facet bound
    HDR_DEFER = 14,   // word offset of the deferred-ridge section (0: none)
    HDR_NDEFER = 15,  // deferred ridges: checked after the resident groups
};
constexpr uint32_t HDR_FLAG_OFFSET = 1;

struct Incidence {
    int n = 0, M = 0, N = 0;
    std::vector<uint32_t> ridges;        // lexicographic
    std::vector<int32_t> facet_ridges;   // [M][n]
    std::vector<int32_t> parent_off;     // [N+1]
    std::vector<int32_t> parents;        // increasing facet ids per ridge
    void build(int n, const uint32_t *facets, int32_t M);
};

int64_t ubt_bound(int n);
int validate_facets(int n, int m, const uint32_t *facets, int32_t M);
int build_candidates(int n, int m, const uint32_t *lambda, uint32_t *facets, int32_t cap,
                     int32_t *M_out);
int kernel_basis(int n, int m, const uint32_t *facets, int32_t M, uint32_t *ridges_out,
                 int32_t cap_r, int32_t *N_out, uint32_t *basis, int32_t cap_k, int32_t *k_out);
int pack_instance(int n, int m, const uint32_t *facets, int32_t M, const uint32_t *basis,
                  int32_t k, const wpm_blocks *blocks, const wpm_conditions *conds,
                  int32_t max_facets, uint64_t seed, uint32_t *table, int64_t cap_words,
                  wpm_instance_info *info);
int facet_conditions(int n, int m, const uint32_t *facets, int32_t M, const uint32_t *basis,
                     int32_t k, const uint32_t *forced_in, const uint32_t *forced_out,
                     uint32_t *basis_out, int32_t *k_out, uint32_t *offset_out, int32_t *feasible);
int convenient_basis(int n, int m, const uint32_t *facets, int32_t M, const uint32_t *basis,
                     int32_t k, int32_t min_free, uint32_t *basis_out, wpm_blocks *blocks);
int validate_blocks(const wpm_blocks &b, int32_t k);
int idcm_orbits(int n, int p, uint32_t *lam_out, int64_t cap, int64_t *count);
int complex_filters(int n, int m, int64_t num, const int64_t *offsets, const uint32_t *facets,
                    uint8_t *flags);
int iso_classes(int m, int64_t num, const int64_t *offsets, const uint32_t *facets,
                int64_t *class_of, int64_t *num_classes);
void cost_features(const wpm_instance_info &info, const Incidence &inc,
                   const std::vector<int32_t> &crit, float *out);
int build_queue(const int32_t *k, const float *cost, const int32_t *group, int32_t num,
                int32_t cbits, int32_t lanes, int32_t min_items_per_instance,
                int32_t max_items_per_instance, int32_t order, wpm_item *items, int64_t cap,
                int64_t *n_out, int64_t *items_per_instance);
int build_pruned_queue(const wpm_blocks *blocks, const float *cost, const int32_t *group,
                       int32_t num, int32_t cbits, int32_t lanes, int32_t min_items_per_instance,
                       int32_t max_items_per_instance, int32_t order, wpm_item *items,
                       int64_t cap, int64_t *n_out, int64_t *items_per_instance);

int pack_bins(const wpm_item *items, int64_t n, const float *cost, int32_t bins,
              wpm_item *out_items, int64_t *out_offsets, double *max_load);

void set_hip_error(const char *what, int code, const char *text);

}  // namespace wpm
