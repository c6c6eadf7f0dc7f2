/*
 * CPU oracle for the weak-pseudo-manifold enumeration.
 *
 * TEST INFRASTRUCTURE ONLY.  Only tests, the smoke check and the CPU-baseline
 * leg of the benchmark may load this library.  It shares no code, header or
 * table with the engine under paper_2301_00806_amd/.
 *
 * What it computes (Choi, Jang, Vallee, arXiv 2301.00806):
 *   Given a set F of candidate facets (n-subsets of [m]) and an optional
 *   upper bound on the number of facets, list every nonempty K subset of F in
 *   which every (n-1)-subset of a member of K lies in exactly 0 or 2 members
 *   of K.  That is the problem statement of Section 2.1 (weak
 *   pseudo-manifolds with facets in F satisfying the affine properties G),
 *   with the weak pseudo-manifold definition of the introduction and the
 *   property g(K) = f_{n-1}(C^n(n+4)) - |K| + 1 > 0 of Section 4.2.
 *
 * The oracle computes that definition directly.  It does not use the F2
 * kernel of the incidence matrix or any sweep over it: the enumerator is a
 * ridge-closing backtracking search, and a brute force over all subsets of F
 * checks the enumerator on tiny inputs.  The F2 rank routine below exists only
 * to pin the kernel dimensions printed in Table 1 and to select inputs.
 *
 * Candidates follow Section 4.2: F(lambda) are the n-subsets of columns of a
 * mod-2 characteristic matrix that form a basis of F2^n (the facets of the
 * binary matroid).  Independence is tested by definition: no nonempty subset
 * of the columns XORs to zero.
 *
 * Vertex sets are bit masks (bit v = vertex v, vertices 0..m-1, m <= 32).
 * Parity unpinned by the paper: the per-instance WPM counts and sets (the
 * paper prints only unions over unprinted orbit representatives, Table 2);
 * they are pinned here by brute force on tiny inputs and by the verifier.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_OK 0
#define OR_EINVAL (-1)
#define OR_ECAP (-2)
#define OR_ENOMEM (-3)

/* ---------------------------------------------------------------- basics */

int64_t or_binom(int a, int b) {
    if (b < 0 || a < 0 || b > a) return 0;
    int64_t r = 1;
    for (int i = 1; i <= b; ++i) r = r * (a - b + i) / i;
    return r;
}

/* Upper bound of Section 4.2: the number of facets of the cyclic polytope
 * C^n(n+4), C(n+4-ceil(n/2), 4) + C(n+3-floor(n/2), 4).  A complex with |K|
 * facets satisfies g(K) > 0 iff |K| <= this value. */
int64_t or_ubt_bound(int n) {
    int ceil_half = (n + 1) / 2, floor_half = n / 2;
    return or_binom(n + 4 - ceil_half, 4) + or_binom(n + 3 - floor_half, 4);
}

static int popc32(uint32_t x) {
    int c = 0;
    while (x) { x &= x - 1; ++c; }
    return c;
}

/* Lexicographic order of the sorted vertex tuples of two equal-size sets:
 * the set holding the smallest element of the symmetric difference is first. */
static int lex_cmp(const void *pa, const void *pb) {
    uint32_t a = *(const uint32_t *)pa, b = *(const uint32_t *)pb;
    if (a == b) return 0;
    uint32_t d = a ^ b;
    uint32_t low = d & (~d + 1u);
    return (a & low) ? -1 : 1;
}

/* Definition of linear independence over F2: no nonempty subset sums to 0. */
static int independent(const uint32_t *cols, int cnt) {
    for (uint32_t T = 1; T < (1u << cnt); ++T) {
        uint32_t x = 0;
        for (int i = 0; i < cnt; ++i)
            if ((T >> i) & 1u) x ^= cols[i];
        if (x == 0) return 0;
    }
    return 1;
}

/* F(lambda): n-subsets of [m] (lexicographic order) whose columns form a basis
 * of F2^n.  lam[i] holds column i as an n-bit integer.  Returns the count, or
 * a negative status; writes at most cap masks. */
int or_candidates(int n, int m, const uint32_t *lam, uint32_t *out, int cap) {
    if (n < 1 || m < n || m > 32 || n > 20) return OR_EINVAL;
    int idx[32];
    uint32_t cols[32];
    for (int i = 0; i < n; ++i) idx[i] = i;
    int count = 0;
    for (;;) {
        for (int i = 0; i < n; ++i) cols[i] = lam[idx[i]];
        if (independent(cols, n)) {
            uint32_t mask = 0;
            for (int i = 0; i < n; ++i) mask |= 1u << idx[i];
            if (count < cap) out[count] = mask;
            ++count;
        }
        int i = n - 1;
        while (i >= 0 && idx[i] == m - n + i) --i;
        if (i < 0) break;
        ++idx[i];
        for (int j = i + 1; j < n; ++j) idx[j] = idx[j - 1] + 1;
    }
    return count;
}

/* Ridges: every (n-1)-subset of some facet, deduplicated, lexicographic order.
 * Returns N, or a negative status. */
int or_ridges(int n, const uint32_t *facets, int M, uint32_t *out, int cap) {
    if (n < 2 || M < 0) return OR_EINVAL;
    int64_t tot = (int64_t)M * n;
    uint32_t *all = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)(tot > 0 ? tot : 1));
    if (!all) return OR_ENOMEM;
    int64_t c = 0;
    for (int j = 0; j < M; ++j) {
        uint32_t f = facets[j];
        for (int v = 0; v < 32; ++v)
            if ((f >> v) & 1u) all[c++] = f & ~(1u << v);
    }
    qsort(all, (size_t)c, sizeof(uint32_t), lex_cmp);
    int N = 0;
    for (int64_t i = 0; i < c; ++i) {
        if (i > 0 && all[i] == all[i - 1]) continue;
        if (N < cap) out[N] = all[i];
        ++N;
    }
    free(all);
    return N;
}

/* Position of a ridge mask in the sorted ridge list (binary search). */
static int find_ridge(const uint32_t *ridges, int N, uint32_t r) {
    int lo = 0, hi = N - 1;
    while (lo <= hi) {
        int mid = (lo + hi) / 2;
        int c = lex_cmp(&ridges[mid], &r);
        if (c == 0) return mid;
        if (c < 0) lo = mid + 1; else hi = mid - 1;
    }
    return -1;
}

/* Rank over F2 of the ridge-facet incidence matrix A(F) (Section 2.1), by
 * plain row reduction.  dim ker A = M - rank.  Returns the rank. */
int or_incidence_rank(int n, const uint32_t *facets, int M) {
    if (M == 0) return 0;
    int cap = M * n;
    uint32_t *ridges = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)cap);
    if (!ridges) return OR_ENOMEM;
    int N = or_ridges(n, facets, M, ridges, cap);
    if (N < 0) { free(ridges); return N; }
    int words = (M + 63) / 64;
    uint64_t *A = (uint64_t *)calloc((size_t)N * (size_t)words, sizeof(uint64_t));
    if (!A) { free(ridges); return OR_ENOMEM; }
    for (int j = 0; j < M; ++j) {
        uint32_t f = facets[j];
        for (int v = 0; v < 32; ++v) {
            if (!((f >> v) & 1u)) continue;
            int r = find_ridge(ridges, N, f & ~(1u << v));
            A[(size_t)r * words + j / 64] |= 1ull << (j % 64);
        }
    }
    int rank = 0;
    for (int col = 0; col < M && rank < N; ++col) {
        int w = col / 64;
        uint64_t bit = 1ull << (col % 64);
        int piv = -1;
        for (int r = rank; r < N; ++r)
            if (A[(size_t)r * words + w] & bit) { piv = r; break; }
        if (piv < 0) continue;
        if (piv != rank)
            for (int t = 0; t < words; ++t) {
                uint64_t tmp = A[(size_t)piv * words + t];
                A[(size_t)piv * words + t] = A[(size_t)rank * words + t];
                A[(size_t)rank * words + t] = tmp;
            }
        for (int r = rank + 1; r < N; ++r)
            if (A[(size_t)r * words + w] & bit)
                for (int t = 0; t < words; ++t) A[(size_t)r * words + t] ^= A[(size_t)rank * words + t];
        ++rank;
    }
    free(A);
    free(ridges);
    return rank;
}

int or_kernel_dim(int n, const uint32_t *facets, int M) {
    int r = or_incidence_rank(n, facets, M);
    return r < 0 ? r : M - r;
}

/* ------------------------------------------------ ridge-closing backtracking */

typedef struct {
    int n, M, N;
    const uint32_t *facets;
    int *fr;          /* M*n ridge ids of each facet */
    int *poff, *plist;/* parents of each ridge, CSR, increasing facet id */
    signed char *dec; /* -1 undecided, 0 out, 1 in */
    int *deg, *und;
    int size;
    int64_t maxf;     /* <= 0: no bound */
    int *trail;
    int tlen;
    /* output: per WPM [len, mask_1..mask_len] */
    uint32_t *out;
    int64_t out_cap, out_len, count;
    int64_t nodes, node_limit;
    int aborted;
} St;

static int assign(St *s, int j, int v) {
    s->dec[j] = (signed char)v;
    s->trail[s->tlen++] = j;
    if (v) ++s->size;
    const int *fr = s->fr + (size_t)j * s->n;
    for (int i = 0; i < s->n; ++i) {
        int r = fr[i];
        --s->und[r];
        if (v) ++s->deg[r];
    }
    if (v && s->maxf > 0 && s->size > s->maxf) return 0;
    for (int i = 0; i < s->n; ++i) {
        int r = fr[i];
        if (s->deg[r] > 2) return 0;
        if (s->deg[r] == 1 && s->und[r] == 0) return 0;
        if (s->deg[r] == 2 && s->und[r] > 0) {
            for (int q = s->poff[r]; q < s->poff[r + 1]; ++q) {
                int p = s->plist[q];
                if (s->dec[p] < 0 && !assign(s, p, 0)) return 0;
            }
        }
    }
    return 1;
}

static void undo(St *s, int mark) {
    while (s->tlen > mark) {
        int j = s->trail[--s->tlen];
        int v = s->dec[j];
        const int *fr = s->fr + (size_t)j * s->n;
        for (int i = 0; i < s->n; ++i) {
            ++s->und[fr[i]];
            if (v) --s->deg[fr[i]];
        }
        if (v) --s->size;
        s->dec[j] = -1;
    }
}

static void record(St *s) {
    int64_t need = s->out_len + 1 + s->size;
    if (s->out && need <= s->out_cap) {
        s->out[s->out_len] = (uint32_t)s->size;
        int64_t w = s->out_len + 1;
        for (int j = 0; j < s->M; ++j)
            if (s->dec[j] == 1) s->out[w++] = s->facets[j];
    }
    s->out_len = need;
    ++s->count;
}

static void search(St *s) {
    if (s->aborted) return;
    if (s->node_limit > 0 && ++s->nodes > s->node_limit) { s->aborted = 1; return; }
    /* An open ridge (exactly one chosen parent) must receive exactly one more
     * parent: branch over which one, taking the ridge with fewest choices. */
    int best = -1;
    for (int r = 0; r < s->N; ++r)
        if (s->deg[r] == 1 && (best < 0 || s->und[r] < s->und[best])) best = r;
    if (best >= 0) {
        int U[64], nu = 0;
        for (int q = s->poff[best]; q < s->poff[best + 1]; ++q)
            if (s->dec[s->plist[q]] < 0 && nu < 64) U[nu++] = s->plist[q];
        for (int a = 0; a < nu; ++a) {
            int mark = s->tlen;
            int ok = assign(s, U[a], 1);
            for (int b = 0; ok && b < nu; ++b)
                if (b != a && s->dec[U[b]] < 0) ok = assign(s, U[b], 0);
            if (ok) search(s);
            undo(s, mark);
        }
        return;
    }
    int f0 = -1;
    for (int j = 0; j < s->M; ++j)
        if (s->dec[j] < 0) { f0 = j; break; }
    if (f0 < 0) {
        if (s->size > 0) record(s);
        return;
    }
    int mark = s->tlen;
    if (assign(s, f0, 0)) search(s);
    undo(s, mark);
    mark = s->tlen;
    if (assign(s, f0, 1)) search(s);
    undo(s, mark);
}

/* Shared set-up: ridges, facet->ridge ids, ridge->parents. */
static int build_incidence(int n, const uint32_t *facets, int M, uint32_t **ridges_out,
                           int *N_out, int **fr_out, int **poff_out, int **plist_out) {
    int cap = M * n > 0 ? M * n : 1;
    uint32_t *ridges = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)cap);
    if (!ridges) return OR_ENOMEM;
    int N = or_ridges(n, facets, M, ridges, cap);
    int *fr = (int *)malloc(sizeof(int) * (size_t)cap);
    int *poff = (int *)calloc((size_t)N + 1, sizeof(int));
    int *plist = (int *)malloc(sizeof(int) * (size_t)cap);
    if (!fr || !poff || !plist) { free(ridges); free(fr); free(poff); free(plist); return OR_ENOMEM; }
    for (int j = 0; j < M; ++j) {
        int i = 0;
        for (int v = 0; v < 32; ++v) {
            if (!((facets[j] >> v) & 1u)) continue;
            int r = find_ridge(ridges, N, facets[j] & ~(1u << v));
            fr[(size_t)j * n + i++] = r;
            ++poff[r + 1];
        }
    }
    for (int r = 0; r < N; ++r) poff[r + 1] += poff[r];
    int *fill = (int *)calloc((size_t)N + 1, sizeof(int));
    if (!fill) { free(ridges); free(fr); free(poff); free(plist); return OR_ENOMEM; }
    for (int j = 0; j < M; ++j)
        for (int i = 0; i < n; ++i) {
            int r = fr[(size_t)j * n + i];
            plist[poff[r] + fill[r]++] = j;
        }
    free(fill);
    *ridges_out = ridges; *N_out = N; *fr_out = fr; *poff_out = poff; *plist_out = plist;
    return OR_OK;
}

static int check_facets(int n, const uint32_t *facets, int M) {
    if (n < 2 || n > 31 || M < 0) return OR_EINVAL;
    for (int j = 0; j < M; ++j) {
        if (popc32(facets[j]) != n) return OR_EINVAL;
        for (int i = 0; i < j; ++i)
            if (facets[i] == facets[j]) return OR_EINVAL;
    }
    return OR_OK;
}

/* Enumerate every weak pseudo-manifold with facets in `facets` and at most
 * max_facets facets (max_facets <= 0: no bound).  Each result is written to
 * out as [len, facet masks...] while it fits in out_cap words; *out_len gets
 * the number of words needed.  node_limit > 0 aborts a search that visits
 * more nodes (then the return value is OR_ECAP and *count is a lower bound).
 * Returns OR_OK or a negative status; *count gets the number of results. */
int or_enumerate(int n, const uint32_t *facets, int M, int64_t max_facets, uint32_t *out,
                 int64_t out_cap, int64_t *out_len, int64_t *count, int64_t node_limit,
                 int64_t *nodes) {
    int st = check_facets(n, facets, M);
    if (st) return st;
    St s;
    memset(&s, 0, sizeof(s));
    uint32_t *ridges = NULL;
    st = build_incidence(n, facets, M, &ridges, &s.N, &s.fr, &s.poff, &s.plist);
    if (st) return st;
    free(ridges);
    s.n = n; s.M = M; s.facets = facets; s.maxf = max_facets;
    s.dec = (signed char *)malloc((size_t)(M > 0 ? M : 1));
    s.deg = (int *)calloc((size_t)s.N + 1, sizeof(int));
    s.und = (int *)calloc((size_t)s.N + 1, sizeof(int));
    s.trail = (int *)malloc(sizeof(int) * (size_t)(M > 0 ? M : 1));
    if (!s.dec || !s.deg || !s.und || !s.trail) st = OR_ENOMEM;
    if (!st) {
        memset(s.dec, -1, (size_t)(M > 0 ? M : 1));
        for (int r = 0; r < s.N; ++r) s.und[r] = s.poff[r + 1] - s.poff[r];
        s.out = out; s.out_cap = out ? out_cap : 0; s.node_limit = node_limit;
        search(&s);
        *out_len = s.out_len;
        *count = s.count;
        if (nodes) *nodes = s.nodes;
        if (s.aborted) st = OR_ECAP;
    }
    free(s.fr); free(s.poff); free(s.plist); free(s.dec); free(s.deg); free(s.und); free(s.trail);
    return st;
}

/* Brute force over all 2^M subsets (M <= 40), in Gray order with incremental
 * ridge counters; same output format as or_enumerate. */
int or_bruteforce(int n, const uint32_t *facets, int M, int64_t max_facets, uint32_t *out,
                  int64_t out_cap, int64_t *out_len, int64_t *count) {
    int st = check_facets(n, facets, M);
    if (st) return st;
    if (M > 40) return OR_EINVAL;
    uint32_t *ridges = NULL;
    int N, *fr, *poff, *plist;
    st = build_incidence(n, facets, M, &ridges, &N, &fr, &poff, &plist);
    if (st) return st;
    int *deg = (int *)calloc((size_t)N + 1, sizeof(int));
    if (!deg) { free(ridges); free(fr); free(poff); free(plist); return OR_ENOMEM; }
    int64_t bad = 0, size = 0, len = 0, cnt = 0;
    uint64_t set = 0;
    uint64_t total = 1ull << M;
    for (uint64_t i = 1; i < total; ++i) {
        int j = __builtin_ctzll(i);
        int add = !((set >> j) & 1ull);
        set ^= 1ull << j;
        size += add ? 1 : -1;
        for (int t = 0; t < n; ++t) {
            int r = fr[(size_t)j * n + t];
            int d0 = deg[r];
            bad -= (d0 != 0 && d0 != 2);
            deg[r] = d0 + (add ? 1 : -1);
            bad += (deg[r] != 0 && deg[r] != 2);
        }
        if (bad == 0 && (max_facets <= 0 || size <= max_facets)) {
            if (out && len + 1 + size <= out_cap) {
                out[len] = (uint32_t)size;
                int64_t w = len + 1;
                for (int q = 0; q < M; ++q)
                    if ((set >> q) & 1ull) out[w++] = facets[q];
            }
            len += 1 + size;
            ++cnt;
        }
    }
    *out_len = len;
    *count = cnt;
    free(deg); free(ridges); free(fr); free(poff); free(plist);
    return OR_OK;
}

/* Verify one claimed result from its facet list alone: facets are distinct
 * n-sets drawn from the candidates, there is at least one, the bound holds,
 * and every ridge of a chosen facet lies in exactly two chosen facets.
 * Returns 1 if valid, 0 if not, negative on bad arguments. */
int or_verify(int n, const uint32_t *K, int len, const uint32_t *cands, int M, int64_t max_facets) {
    if (n < 2 || len < 0) return OR_EINVAL;
    if (len == 0) return 0;
    if (max_facets > 0 && len > max_facets) return 0;
    for (int a = 0; a < len; ++a) {
        if (popc32(K[a]) != n) return 0;
        int found = 0;
        for (int j = 0; j < M && !found; ++j) found = (cands[j] == K[a]);
        if (!found) return 0;
        for (int b = 0; b < a; ++b)
            if (K[a] == K[b]) return 0;
    }
    uint32_t *r = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)len * (size_t)n);
    if (!r) return OR_ENOMEM;
    int c = 0;
    for (int a = 0; a < len; ++a)
        for (int v = 0; v < 32; ++v)
            if ((K[a] >> v) & 1u) r[c++] = K[a] & ~(1u << v);
    qsort(r, (size_t)c, sizeof(uint32_t), lex_cmp);
    int ok = 1;
    for (int i = 0; i < c && ok;) {
        int j = i;
        while (j < c && r[j] == r[i]) ++j;
        if (j - i != 2) ok = 0;
        i = j;
    }
    free(r);
    return ok;
}
