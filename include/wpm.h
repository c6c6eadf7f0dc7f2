/*
 * wpm.h - C ABI of the MI355X weak-pseudo-manifold sweep engine.
 *
 * The engine implements the enumeration of Choi, Jang and Vallee,
 * "The characterization of (n-1)-spheres with n+4 vertices having maximal
 * Buchstaber number" (arXiv 2301.00806):
 *   input  a set F of candidate facets (n-subsets of [m]) and the properties
 *          G (here: the upper-bound property of Section 4.2);
 *   output every weak pseudo-manifold K with facets in F satisfying G
 *          (problem statement of Section 2.1).
 * A complex K with facets in F is a 0/1 vector of length M = |F|; it is a weak
 * pseudo-manifold iff every entry of A K lies in {0, 2}, where A is the
 * ridge-facet incidence matrix (Proposition 2.1).  Such vectors lie in the F2
 * kernel of A, so the engine sweeps all 2^k combinations of a kernel basis
 * (Section 2.1) on the GPU and keeps the ones that pass the check.
 *
 * Conventions
 *   - Vertices are 0..m-1 (the paper uses 1..m); a vertex set is a uint32
 *     mask, bit v = vertex v.  m <= 32.
 *   - lambda[i] is column i of the n x m mod-2 characteristic matrix, bit t =
 *     row t (Section 3.1, characteristic maps).
 *   - Facets and ridges are listed in lexicographic order of their sorted
 *     vertex tuples.
 *   - A facet bit vector of length M is stored in W = ceil(M/32) uint32
 *     words, bit j of word j/32 = facet j.
 *   - A kernel coordinate vector x (bit t = coefficient of basis vector t) is
 *     a uint64; the complex is K = sum_t x_t K_t over F2.
 *   - The empty complex (x = 0) is not reported: it is not an
 *     (n-1)-dimensional pure complex.  Every count covers nonzero x only.
 *
 * Errors: every call returns WPM_OK (0) or a negative status; nothing aborts
 * or throws.  Capacity errors report the size needed in the *_out/needed
 * argument and leave every count exact.  Calls keep no global state except a
 * thread-local copy of the last HIP error (wpm_last_hip_error).  Host calls
 * are reentrant; device calls are ordered on the stream passed in.
 *
 * Ownership: the caller owns every buffer, host and device.  Device buffers
 * are plain device pointers (for example torch.empty(..., device="cuda")
 * .data_ptr()); `stream` is a hipStream_t passed as void*.  wpm_enumerate
 * makes no device allocation.
 */
#ifndef WPM_H
#define WPM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    WPM_OK = 0,
    WPM_EINVAL = -1, /* invalid argument or malformed input */
    WPM_ECAP = -2,   /* a caller buffer is too small; the size needed is reported */
    WPM_EKMAX = -3,  /* kernel dimension above WPM_MAX_K */
    WPM_EHIP = -4,   /* HIP runtime error; see wpm_last_hip_error() */
    WPM_ELIMIT = -5  /* instance outside the engine's table limits (WPM_MAX_*) */
};

#define WPM_MAX_K 64        /* kernel dimension (x is a uint64) */
#define WPM_MAX_M 1024      /* candidate facets per instance (W <= 32 words) */
#define WPM_MAX_GROUPS 16   /* 32-ridge groups of critical ridges (<= 512 ridges) */
#define WPM_MAX_SLOTS 8     /* parents-1 of a critical ridge */
#define WPM_LOW_BITS 6      /* Gray steps unrolled per block: 2^6 */
#define WPM_TABLE_ROWS 32   /* Gray-bit lookup rows staged per instance: 4 tables of 2^3 */
#define WPM_MAX_ROW_WORDS 160 /* words per row of a packed table (4 + 15 groups x 8 + 32) */
#define WPM_TOTAL_WORDS 4   /* uint64 words of the d_total argument of wpm_enumerate */
#define WPM_LANE_WINDOW 512 /* an item's lane chunks lie in one aligned window of this many */

/* Human-readable text of a status code (static storage). */
const char *wpm_strerror(int status);

/* Text of the last HIP error seen by this thread (static storage). */
const char *wpm_last_hip_error(void);

/*
 * Candidate facets F(lambda) (Section 4.2): the n-subsets S of [m] whose
 * columns {lambda(i) : i in S} form a basis of F2^n, i.e. the facets of the
 * binary matroid of lambda.  A mod-2 characteristic map over K exists with
 * matrix lambda iff K is a subcomplex of that matroid (Proposition 4.2 and
 * the paragraph before it), so these are the only facets a complex
 * supporting lambda can use.
 *   n, m       1 <= n <= m <= 32, n <= 20
 *   lambda     [m] host array, column i as an n-bit integer (< 2^n)
 *   facets     [cap] host array; receives vertex masks in lexicographic order
 *   M_out      receives |F(lambda)|; if it exceeds cap, WPM_ECAP
 */
int wpm_build_candidates(int n, int m, const uint32_t *lambda, uint32_t *facets, int32_t cap,
                         int32_t *M_out);

/*
 * Ridges and an F2 basis of the kernel of the ridge-facet incidence matrix
 * A(F) (Section 2.1: a_ij = 1 iff ridge r_i lies in facet F_j; weak
 * pseudo-manifolds lie in ker_F2 A; any basis reaches each of them as exactly
 * one combination).
 *   n, m       2 <= n <= m <= 32
 *   facets     [M] host array of distinct n-element vertex masks below 2^m
 *   ridges     [cap_r] host array; receives the (n-1)-subsets of the facets in
 *              lexicographic order; *N_out = their number
 *   basis      [cap_k * W] host array; receives basis vector t as W words at
 *              basis + t*W (bit j of word j/32 = facet j); *k_out = k
 *   The basis is the reduced-echelon null-space basis: vector t has a 1 at
 *   the t-th non-pivot facet and 0 at the other non-pivot facets.
 * Returns WPM_ECAP if N > cap_r or k > cap_k (sizes still reported),
 * WPM_EKMAX is not returned here (k may exceed 64; wpm_pack_instance rejects).
 */
int wpm_kernel_basis(int n, int m, const uint32_t *facets, int32_t M, uint32_t *ridges,
                     int32_t cap_r, int32_t *N_out, uint32_t *basis, int32_t cap_k,
                     int32_t *k_out);

/* Upper bound of Section 4.2: facet count of the cyclic polytope C^n(n+4),
 * C(n+4-ceil(n/2), 4) + C(n+3-floor(n/2), 4).  g(K) > 0 iff |K| <= it. */
int64_t wpm_ubt_bound(int n);

/* ------------------------------------------------- convenient basis (pruning) */

#define WPM_MAX_BLOCKS 16   /* blocks of a convenient basis */
#define WPM_MAX_CHOICES 40  /* allowed combinations per block (<= 1 + C(9,2)) */

/*
 * Block structure of a convenient kernel basis (Section 2.1, the partition
 * I_1..I_l and the sets X_1..X_l).  Coordinates 0..free_dims-1 of x are
 * free; block b owns the size[b] coordinates that follow the free ones and
 * the earlier blocks.  A kernel vector can be a weak pseudo-manifold only if
 * the part of x on each block is one of that block's allowed combinations
 * choice[b][0..count[b]-1] (bit j = the block's j-th coordinate), so the
 * sweep visits 2^free_dims * prod_b count[b] vectors instead of 2^k.
 */
typedef struct wpm_blocks {
    int32_t k;           /* kernel dimension */
    int32_t free_dims;   /* f: coordinates 0..f-1 are unconstrained */
    int32_t num_blocks;  /* l (0: no pruning, x ranges over F2^k) */
    int32_t reserved;
    int32_t ridge[WPM_MAX_BLOCKS];  /* ridge (index in lexicographic order) defining block b */
    uint8_t size[WPM_MAX_BLOCKS];   /* q_b, 1..8 */
    uint8_t count[WPM_MAX_BLOCKS];  /* |X_b| */
    uint8_t choice[WPM_MAX_BLOCKS][WPM_MAX_CHOICES]; /* allowed local masks, increasing */
    double log2_vectors; /* log2 of the vectors swept: f + sum_b log2 count[b] */
} wpm_blocks;

/*
 * Convenient basis of ker_F2 A(F) by column elimination on the rows of the
 * basis at the parents of chosen ridges (Section 2.1).  Ridges with 4..9
 * parents are taken greedily (more parents first, then lexicographic order)
 * when their parent sets are disjoint from the earlier blocks', when
 * eliminating on them among the still-free generators leaves every earlier
 * block generator zero on those parents (so earlier blocks keep their form),
 * and when they prune something.  For each block the allowed set is computed
 * exactly: the combinations of the block's generators whose restriction to
 * the ridge's parents has weight <= 2 (that is, (AK)_r in {0,2}, Proposition
 * 2.1).  With m - n + 1 parents spanning all even patterns this is the
 * paper's Z_{m-n} block with at most two generators combined,
 * 1 + (m-n) + C(m-n, 2) choices.  Every weak pseudo-manifold lies in the
 * product, so the result set of a sweep is unchanged.
 *   facets[M], basis[k*W]  as from wpm_kernel_basis (any basis of ker A)
 *   min_free               keep at least this many free coordinates (a sweep
 *                          needs >= 7: one lane walks 2^7-aligned Gray chunks);
 *                          0 gives the most pruning, for counting
 *   basis_out[k*W]         receives the convenient basis: the free generators,
 *                          then block 0, block 1, ... (same span as basis)
 *   blocks                 receives the structure above
 * x in the new coordinates describes K = sum_t x_t basis_out_t, as before.
 * Returns WPM_EKMAX if k > 64.
 */
int wpm_convenient_basis(int n, int m, const uint32_t *facets, int32_t M, const uint32_t *basis,
                         int32_t k, int32_t min_free, uint32_t *basis_out, wpm_blocks *blocks);

/* --------------------------------------------- facet conditions, properties */

#define WPM_MAX_PROPS 8     /* affine properties per instance besides the facet bound */
#define WPM_MAX_CLASSES 32  /* weight classes over all of an instance's properties */

/*
 * Forced-in and forced-out facets (Section 2.1's problem statement with facet
 * conditions; Section 4.3 fixes the facets around a vertex this way): the
 * complexes K in the span of `basis` with K_j = 1 for j in I and K_j = 0 for j
 * in J form an affine coset K* + span(basis_out), found here by F2
 * elimination on the rows I and J of the basis (the paper's column echelon
 * form of B restricted to those rows).
 *   facets[M], basis[k*W]    as from wpm_kernel_basis (any basis of ker A)
 *   forced_in, forced_out    [W] facet bit masks (bit j = facet j), or NULL
 *   basis_out[k*W]           receives k_out <= k vectors spanning the linear part
 *   offset_out[W]            receives K*: the all-zero x of the coset (zero
 *                            when I is empty: then the result is a subspace)
 *   feasible                 receives 0 when no K satisfies the conditions
 *                            (then k_out = 0), else 1
 * Returns WPM_EINVAL if I and J share a facet or name bits >= M.
 */
int wpm_facet_conditions(int n, int m, const uint32_t *facets, int32_t M, const uint32_t *basis,
                         int32_t k, const uint32_t *forced_in, const uint32_t *forced_out,
                         uint32_t *basis_out, int32_t *k_out, uint32_t *offset_out,
                         int32_t *feasible);

/*
 * Optional parts of a packed instance.
 *   offset        [W] offset K* of an affine coset (from wpm_facet_conditions),
 *                 or NULL: the sweep then visits K = K* + sum x_t K_t for every
 *                 x, including x = 0, whose complex is K* itself
 *   num_props     affine properties g(K) = c0 + sum_c weight_c |K & mask_c|,
 *                 kept when every g(K) > 0 (Section 2.1: the collection G;
 *                 the facet bound max_facets is the property of Section 4.2
 *                 and is passed on its own)
 *   prop_c0       [num_props] constant terms
 *   prop_classes  [num_props] weight classes of each property
 *   class_weight  [sum of prop_classes] integer weights
 *   class_mask    [sum of prop_classes][W] facet masks of the classes
 * Sums are evaluated in 64-bit integers.
 *   max_groups    0, or at most this many 32-ridge groups (1..WPM_MAX_GROUPS)
 *                 kept resident in the sweep; see "deferred ridges" below
 *
 * Deferred ridges.  The sweep holds at most WPM_MAX_GROUPS groups of 32
 * critical ridges (the most rejecting ones, in the packer's greedy order),
 * each with at most WPM_MAX_SLOTS + 1 parents.  Any further critical ridges
 * (and ridges with more parents) are deferred: the table lists their parents,
 * and the sweep checks them (degree <= 2 in K, Proposition 2.1) on every
 * vector that passes the resident groups, before it counts or records it.
 * Results and counts are exact in every case, also after a record-buffer
 * overflow.
 */
typedef struct wpm_conditions {
    const uint32_t *offset;
    int32_t num_props;
    const int32_t *prop_c0;
    const int32_t *prop_classes;
    const int32_t *class_weight;
    const uint32_t *class_mask;
    int32_t max_groups;
} wpm_conditions;

/* ------------------------------------------------------------ IDCM orbits */

/*
 * One characteristic matrix per IDCM orbit of Lambda(n, p) (Section 4.2: the
 * (n+p) x p matrices [M; I_p] over F2 with no repeated rows, under S_n x S_p;
 * the proposition on IDCM orbits there makes the binary matroids of one orbit
 * isomorphic, so the enumeration of Algorithm 4.4 needs one representative
 * each).  The rows of
 * M are distinct vectors of weight >= 2 (a dual characteristic map is nonzero
 * and injective), so an orbit is an n-subset of them up to coordinate
 * permutations; the representative is the orbit's least subset in
 * lexicographic order of the increasing row lists, and orbits come in that
 * order.
 *   n, p       1 <= n <= 26, 2 <= p <= 5 (the paper's case is p = 4)
 *   lam_out    [cap * (n+p)] host array: representative r is the matrix
 *              [I_n | M] as n+p columns (bit t = row t), the lambda argument
 *              of wpm_build_candidates with m = n + p
 *   count      receives the number of orbits; WPM_ECAP if it exceeds cap
 *              (lam_out may be NULL to count only)
 */
int wpm_idcm_orbits(int n, int p, uint32_t *lam_out, int64_t cap, int64_t *count);

/* ------------------------------------------------------ complexes (filters) */

#define WPM_CX_FULL_PICARD 1 /* K uses all m vertices: Pic(K) = m - n */
#define WPM_CX_SEED 2        /* K satisfies the seedness condition */

/*
 * Filters of Algorithm 4.4 on enumerated complexes.  A list of complexes is
 * offsets[num + 1] (offsets[0] = 0) into facets[]: complex i has the facet
 * vertex masks facets[offsets[i] .. offsets[i+1]), all below 2^m, m <= 16.
 *
 * wpm_complex_filters sets flags[i]:
 *   WPM_CX_FULL_PICARD  the complex uses every vertex of [m], so its Picard
 *                       number (vertices minus n) is m - n (Algorithm 4.4
 *                       discards complexes with Pic(K) < 4 at m = n + 4)
 *   WPM_CX_SEED         the seedness condition (Section 3, seedness from
 *                       minimal non-faces): no edge {v, w} of K such that every
 *                       minimal non-face contains both v and w or neither
 */
int wpm_complex_filters(int n, int m, int64_t num, const int64_t *offsets,
                        const uint32_t *facets, uint8_t *flags);

/*
 * Isomorphism classes of a list of complexes (Section 3, checking isomorphism
 * with minimal non-faces): vertices are coloured by the increasing sizes of
 * the minimal non-faces containing them, and two complexes are isomorphic iff
 * a colour-preserving relabelling maps one set of minimal non-faces onto the
 * other (the search assigns vertices class by class and backtracks on the
 * first non-face that does not map).  class_of[i] receives the class of
 * complex i, classes numbered 0, 1, ... in order of first appearance;
 * *num_classes receives their number.
 */
int wpm_iso_classes(int m, int64_t num, const int64_t *offsets, const uint32_t *facets,
                    int64_t *class_of, int64_t *num_classes);

/* Summary of a packed instance. */
typedef struct wpm_instance_info {
    int32_t n, m, M, N, k;
    int32_t W;            /* facet words */
    int32_t n_crit;       /* ridges with >= 4 parents (only these can fail) */
    int32_t groups;       /* 32-ridge groups, group 0 = the fast filter */
    int32_t slots;        /* slot words per ridge in groups >= 1 */
    int32_t n_filter;     /* ridges in the fast filter group */
    int32_t row_words;    /* words per basis row of the packed table */
    int32_t max_facets;   /* upper bound applied (0 = none) */
    int32_t n_deferred;   /* critical ridges checked after the resident groups */
    int64_t table_words;  /* size of the packed table in uint32 words */
    double filter_pass;   /* estimated fraction of x passing the filter */
    double full_pass;     /* estimated fraction of x passing every ridge */
    float features[16];   /* cost-model features (see wpm_cost_features) */
} wpm_instance_info;

/*
 * Pack one instance for the GPU sweep: selects the fast-filter ridges and lays
 * out the bit-sliced ridge-slot rows and facet rows of every basis vector.
 *   facets[M], basis[k*W]  as returned by the calls above
 *   blocks                 NULL, or the structure of a convenient basis passed
 *                          as `basis`: the ridges are then ranked on vectors
 *                          drawn from the pruned set the sweep will visit
 *   conds                  NULL, or an offset and affine properties (above);
 *                          blocks and an offset cannot be combined (WPM_EINVAL)
 *   max_facets             bound on |K| (0 = none; the paper applies
 *                          wpm_ubt_bound(n) when m = n + 4, Algorithm 4.4)
 *   seed                   seeds the sampling that ranks ridges (any value;
 *                          never changes results)
 *   table, cap_words       host output; with table == NULL or a too small
 *                          cap the call returns WPM_ECAP after filling info
 * Returns WPM_EKMAX if k > 64, WPM_ELIMIT if M exceeds WPM_MAX_M (critical
 * ridges beyond the resident groups are deferred, see above).
 */
int wpm_pack_instance(int n, int m, const uint32_t *facets, int32_t M, const uint32_t *basis,
                      int32_t k, const wpm_blocks *blocks, const wpm_conditions *conds,
                      int32_t max_facets, uint64_t seed, uint32_t *table, int64_t cap_words,
                      wpm_instance_info *info);

/* ------------------------------------------------------------ scheduling */

/* One unit of GPU work: lanes 0..lanes-1 of a workgroup sweep the Gray index
 * ranges [(first + l) * 2^cbits, (first + l + 1) * 2^cbits) of one instance. */
typedef struct wpm_item {
    uint32_t instance;
    uint16_t cbits;   /* per-lane chunk: 2^cbits consecutive Gray indices, >= 7 */
    uint16_t lanes;   /* lanes used, 1..workgroup size */
    uint64_t first;   /* first lane chunk */
} wpm_item;

enum {
    WPM_SCHED_PLAIN = 0,   /* one launch per instance over its own items */
    WPM_SCHED_STATIC = 1,  /* one persistent launch, workgroup g takes items g, g+G, ... */
    WPM_SCHED_DYNAMIC = 2, /* one persistent launch, items popped from a device queue */
    WPM_SCHED_PACKED = 3   /* one launch, workgroup g runs bin g of a host-packed assignment */
};

/*
 * Split instances into items.
 *   k[num]           kernel dimension of each instance
 *   cost[num]        relative cost per vector (NULL = 1.0 for all); an item's
 *                    cost is cost[i] * vectors in the item
 *   group[num]       optional launch group of each instance (NULL = all 0):
 *                    items come out group by group, in decreasing group key,
 *                    so each group can be launched under its own kernel template
 *   cbits            lane chunk bits (clamped to [7, max(k,7)] per instance)
 *   lanes            lanes per item (workgroup size)
 *   min_items_per_instance  lower cbits (down to 7) until an instance has at
 *                    least this many full items (values < 1 count as 1), so a
 *                    small instance still occupies whole workgroups
 *   max_items_per_instance  > 0: coarsen chunks so an instance yields at most
 *                    this many items (raises cbits; applied after the minimum)
 *   order            0 = instance order, 1 = decreasing item cost inside a
 *                    group (instance by instance: longest-processing-time
 *                    first up to each instance's partial last item)
 *   items, cap       output (host); *n_out = item count (WPM_ECAP if > cap)
 *   items_per_instance  optional [num] output: items of each instance
 *   Instances with k = 0 yield no items (their only vector is x = 0).
 */
int wpm_build_queue(const int32_t *k, const float *cost, const int32_t *group, int32_t num,
                    int32_t cbits, int32_t lanes, int32_t min_items_per_instance,
                    int32_t max_items_per_instance, int32_t order, wpm_item *items, int64_t cap,
                    int64_t *n_out, int64_t *items_per_instance);

/*
 * Items of a pruned sweep (Section 2.1: the product X_1 x ... x X_l of the
 * blocks' allowed sets times the free coordinates).  Arguments as for
 * wpm_build_queue, with blocks[num] in place of k (blocks[i].k is the kernel
 * dimension).  For each allowed block tuple with high part h (bits f..k-1 of
 * x), the items cover the Gray indices [g^-1(h) 2^f, (g^-1(h) + 1) 2^f),
 * g^-1 the inverse Gray code: exactly the 2^f vectors with that high part.
 * Tuples come in mixed-radix order, block 0 fastest; an item never spans two
 * tuples.  An instance with num_blocks = 0 gets the items wpm_build_queue
 * gives it.  Requires free_dims >= 7 when num_blocks > 0 (WPM_EINVAL).  For
 * a pruned instance cbits is clamped to [7, free_dims] and lowered to
 * free_dims - ceil(log2 lanes) (not below 7), so that one tuple fills whole
 * workgroups; the min/max item rules then apply to the instance's total.
 */
int wpm_build_pruned_queue(const wpm_blocks *blocks, const float *cost, const int32_t *group,
                           int32_t num, int32_t cbits, int32_t lanes,
                           int32_t min_items_per_instance, int32_t max_items_per_instance,
                           int32_t order, wpm_item *items, int64_t cap, int64_t *n_out,
                           int64_t *items_per_instance);

/*
 * Pack items into `bins` workgroup bins by longest-processing-time-first:
 * items in decreasing cost (cost[instance] * lanes * 2^cbits, cost NULL =
 * 1.0) each go to the bin with the least total so far (ties: lowest bin).
 *   items[n], out_items[n]   out_items lists the items bin by bin
 *   out_offsets[bins + 1]    bin b holds out_items[out_offsets[b] .. out_offsets[b+1])
 *   max_load                 optional: receives the largest bin total
 */
int wpm_pack_bins(const wpm_item *items, int64_t n, const float *cost, int32_t bins,
                  wpm_item *out_items, int64_t *out_offsets, double *max_load);

/* Device-resident batch.  One kernel serves every instance shape: it reads
 * the ridge groups, slot stride and facet words from each table's header.
 * max_row_words and max_kp size the workgroup's LDS; an item whose table is
 * larger is skipped and counted as malformed (d_total[2]). */
typedef struct wpm_batch {
    int32_t num_instances;
    int32_t max_row_words;     /* max info.row_words over the tables swept (multiple of 4, <= WPM_MAX_ROW_WORDS) */
    int32_t max_groups;        /* max info.groups (informational) */
    int32_t max_slots;         /* max info.slots (informational) */
    int32_t max_words;         /* max info.W (informational) */
    int32_t max_kp;            /* max over the tables swept of max(k, 7), <= WPM_MAX_K */
    const uint32_t *d_tables;  /* device: packed tables, concatenated (16-byte aligned each) */
    const int64_t *d_offsets;  /* device: word offset of each table in d_tables */
    int32_t flags;             /* reserved, 0 */
    int32_t reserved;
} wpm_batch;

#define WPM_FLAG_ACCUMULATE 1 /* do not clear d_counts, d_total, d_stats: add to them */

typedef struct wpm_sched {
    int32_t mode;              /* WPM_SCHED_* */
    int32_t wg_size;           /* threads per workgroup: 64, 128, 256 or 512 */
    int32_t grid;              /* persistent modes: workgroups (0 = occupancy x CUs) */
    int32_t flags;             /* WPM_FLAG_* */
    const wpm_item *d_items;   /* device: the items */
    const wpm_item *h_items;   /* host copy (PLAIN mode launches per instance from it) */
    int64_t num_items;
    uint32_t *d_scratch;       /* device: >= 4 words (queue head), cleared by the call */
    uint64_t *d_item_times;    /* optional device [num_items][2]: start, end (s_memrealtime) */
    const int64_t *d_bin_offsets; /* PACKED mode: device [grid + 1] from wpm_pack_bins */
    int32_t waves_per_simd;    /* register budget of the kernel: 7 or 8 waves per SIMD (0 = 8) */
    int32_t reserved;
} wpm_sched;

/* Workgroups a persistent launch of this batch uses by default: the
 * occupancy of the selected kernel instantiation times the compute units. */
int wpm_persistent_grid(const wpm_batch *batch, int32_t wg_size, int32_t *grid);

/*
 * The weak pseudo-manifolds of every item's instance (Section 2.1, problem
 * statement: every K with facets in F satisfying the properties G).  By
 * Proposition 2.1 a complex K is a weak pseudo-manifold iff every entry of
 * A K lies in {0, 2}; such K lie in ker_F2 A, so the sweep visits the kernel
 * vectors x in Gray order (the enumeration of Section 2.1, with the paper's
 * per-candidate ridge check of Section 2.3 in bit-sliced form) and keeps x
 * when every critical ridge has degree <= 2, |K| <= max_facets (the
 * upper-bound property of Section 4.2), every further property g(K) > 0, and
 * x != 0 (x = 0 is kept only for an affine coset, where it is K*).  Each kept
 * x is an output of Section 2.3's list, written as a record.
 *   batch       device tables (wpm_pack_instance), see wpm_batch
 *   sched       items (device, and a host copy in PLAIN mode), mode,
 *               workgroup size, grid, register budget
 *   d_survivors [cap][2] uint64 records {x, instance}, in device memory or
 *               in pinned host memory the device can address (the sweep
 *               then writes them there directly).  Waves reserve
 *               record slots in chunks, so the slots used may exceed the
 *               results; unused slots hold the sentinel {0, ~0}.  Records are
 *               in no particular order; slots at or beyond cap are not written.
 *   d_counts    [num_instances] uint64 device; set to each instance's exact
 *               number of results (cleared by the call unless
 *               WPM_FLAG_ACCUMULATE: then a batch can be swept by several calls
 *               into one set of counts)
 *   d_total     [WPM_TOTAL_WORDS] uint64 device: [0] total results, [1] record
 *               slots used ([1] > cap: the caller needs a larger buffer and
 *               wpm_collect returns WPM_ECAP; counts stay exact), [2] malformed
 *               items skipped (wpm_collect then returns WPM_EINVAL), [3] 0
 *   d_stats     optional [8] uint64 device counters: [0] candidates (vectors
 *               passing the fast filter), [1] vectors passing every resident
 *               ridge group, [2] of those, vectors rejected by the facet bound,
 *               the properties or a deferred ridge, [3] wave passes over the
 *               listed candidates, [4] wave steps whose candidates overflowed
 *               the list and were rechecked
 * Items must lie inside their instance's 2^max(k,7) Gray range with
 * 7 <= cbits <= max(k, 7), 1 <= lanes <= wg_size, and first mod
 * WPM_LANE_WINDOW + lanes <= WPM_LANE_WINDOW (wpm_build_queue and
 * wpm_build_pruned_queue emit such items); the kernel skips any other item
 * and counts it in d_total[2].  PLAIN mode rejects items naming an unknown
 * instance with WPM_EINVAL before launching.
 * Asynchronous: returns after enqueueing on `stream`.  No device memory is
 * allocated.
 */
int wpm_enumerate(const wpm_batch *batch, const wpm_sched *sched, uint64_t *d_survivors,
                  uint64_t cap, uint64_t *d_counts, uint64_t *d_total, uint64_t *d_stats,
                  void *stream);

/*
 * wpm_enumerate for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid allocation):
 * the same sweep and the same outputs, with the dynamic queue's head kept in
 * a device array of the library instead of sched->d_scratch, which must be
 * NULL.  The array holds WPM_STATIC_SCRATCH_WORDS uint64 words per device
 * (the queue needs 2); a schedule needing more is rejected with WPM_ELIMIT.
 * Each device the library runs on holds its own copy until the process
 * ends; its address is looked up on the first call on that device.  Every
 * call on one device shares the array and clears what it uses at its start,
 * so calls that overlap on one device (streams running concurrently) race:
 * order them on one stream.  No allocation of any kind is made.
 */
#define WPM_STATIC_SCRATCH_WORDS 32
int wpm_enumerate_noalloc(const wpm_batch *batch, const wpm_sched *sched, uint64_t *d_survivors,
                          uint64_t cap, uint64_t *d_counts, uint64_t *d_total, uint64_t *d_stats,
                          void *stream);

/* Device facts the scheduler needs: compute units, the s_memrealtime clock
 * rate (kHz, the unit of d_item_times) and the LDS limit per workgroup. */
int wpm_device_query(int32_t *num_cus, int64_t *wallclock_khz, int32_t *lds_per_block);

/* Integer VALU throughput probe (diagnostic; allocates and synchronises the
 * device, so never call it under graph capture).  op: 0 = 32-bit XOR with
 * register operands, 1 = 3-input bit logic (v_bitop3), 2 = AND-OR; one
 * 256-thread workgroup per CU per unit of waves_per_simd (1..8).
 * *lane_ops_per_s receives the measured 32-bit lane operations per second. */
int wpm_valu_probe(int op, int waves_per_simd, int iters, double *lane_ops_per_s);

/* Host view of an instance for wpm_collect. */
typedef struct wpm_host_instance {
    int32_t M, k;
    const uint32_t *facets; /* [M] */
    const uint32_t *basis;  /* [k * ceil(M/32)] */
    const uint32_t *offset; /* [ceil(M/32)] offset K* of an affine coset, or NULL */
} wpm_host_instance;

/*
 * The result set of Section 2.1's problem statement, per instance: every
 * kept x becomes its complex K = sum_t x_t K_t (+ K* for a coset), listed by
 * its facets.  Synchronises `stream`, copies counts and records to the host
 * and expands them.
 *   insts        [num] host views of the instances (facets, basis, offset)
 *   d_survivors, cap, d_counts, d_total   as passed to wpm_enumerate
 *   h_counts     [num] receives the exact per-instance counts
 *   h_out        [out_cap] uint32; per instance, in canonical order, each
 *                result as [len, facet masks ascending]; results of one
 *                instance are sorted lexicographically.  NULL asks only for
 *                out_words (and h_counts, h_offsets).  A result of instance
 *                i takes at most 1 + min(M_i, its facet bound) words, so
 *                out_cap = sum over i of count_i (1 + M_i) always suffices
 *                and saves the second call
 *   h_offsets    [num + 1] int64: word offset of each instance's results
 *   out_words    receives the words needed (when the record buffer
 *                overflowed: minus the record slots needed)
 * Returns WPM_ECAP if the record buffer overflowed (d_total[1] > cap) or
 * out_cap is too small, WPM_EINVAL if the sweep skipped malformed items or
 * the records disagree with the counts.
 */
int wpm_collect(const wpm_host_instance *insts, int32_t num, const uint64_t *d_survivors,
                uint64_t cap, const uint64_t *d_counts, const uint64_t *d_total,
                uint64_t *h_counts, uint32_t *h_out, int64_t out_cap, int64_t *out_words,
                int64_t *h_offsets, void *stream);

/* ------------------------------------------------------------ cost model */

/*
 * Learned cost model for the persistent scheduler: an MLP 16 -> 64 -> 64 -> 2
 * in fp32 with ReLU hidden layers, mapping the 16 features of
 * wpm_instance_info.features to [natural log of sweep time per kernel vector
 * in ns, log10 of the survivor density].  It orders and sizes work items
 * only; it never removes any vector from the sweep.
 * Parameters (device, WPM_MLP_PARAMS floats): W1[64][16] b1[64] W2[64][64]
 * b2[64] W3[2][64] b3[2] (row-major, W[out][in]).  Normalisation (device,
 * WPM_MLP_NORM floats): mean_x[16] std_x[16] mean_y[2] std_y[2]; inputs are
 * standardised and outputs de-standardised inside the kernels.
 */
#define WPM_MLP_IN 16
#define WPM_MLP_HIDDEN 64
#define WPM_MLP_OUT 2
#define WPM_MLP_PARAMS 5378
#define WPM_MLP_NORM 36

/* Floats of device work space wpm_mlp_grad needs for `batch` samples. */
int64_t wpm_mlp_work_floats(int32_t batch);

/* d_y[batch][2] = model(d_x[batch][16]) on `stream`. */
int wpm_mlp_forward(const float *d_params, const float *d_norm, const float *d_x, int32_t batch,
                    float *d_y, void *stream);

/* Gradient of the mean squared error on standardised targets d_t[batch][2]
 * into d_grad[WPM_MLP_PARAMS] (a fixed-order sum: bitwise reproducible);
 * d_loss[1] (optional) receives the loss.  d_work: wpm_mlp_work_floats(batch). */
int wpm_mlp_grad(const float *d_params, const float *d_norm, const float *d_x, const float *d_t,
                 int32_t batch, float *d_grad, float *d_work, float *d_loss, void *stream);

/* One Adam step (Kingma and Ba) with bias correction for step >= 1 and
 * an L2 term weight_decay * param added to the gradient. */
int wpm_mlp_adam(float *d_params, const float *d_grad, float *d_m, float *d_v, int32_t step,
                 float lr, float beta1, float beta2, float eps, float weight_decay, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* WPM_H */
