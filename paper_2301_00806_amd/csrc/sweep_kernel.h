// The Gray-code sweep of the F2 kernel on gfx950 (device code).
//
// Every lane owns a chunk of 2^c consecutive Gray indices i of one instance
// and visits x = i ^ (i >> 1), so consecutive vectors differ in the single
// basis vector t = ctz(i + 1) and K changes by XOR with that basis row
// (Section 2.1: the weak pseudo-manifolds are among the 2^k combinations of a
// kernel basis).  Chunks are 2^c-aligned with c >= 7, so all lanes of a
// workgroup flip the same t at the same step: the XOR operands are
// wave-uniform.  They are held in VGPRs all the same: a VOP2 XOR with a
// scalar operand issues markedly slower than one with two VGPR operands.
//
// A step checks the ridges whose parents Proposition 2.1 constrains, in the
// bit-sliced slot form built by the packer (a ridge fails iff at least 3 of
// its first p-1 parent bits are set).  Work per block of 64 steps:
//   phase 1  the fast filter: 32 ridges in 4 slot words held in VGPRs,
//            updated by 4 XORs and tested by 2 bit-logic ops per step, the
//            block run as four interleaved chains of 16 steps whose fail
//            words one 3-input minimum and one compare test together.  When
//            a lane passes (a rarely taken branch), the passing lanes append
//            (step, lane) to the wave's candidate list in LDS; ballot and
//            mbcnt give the slots, the count is wave-uniform.
//   check    when the list is half full, at the end of a 4096-step segment
//            and at the end of the item, lane j of the wave takes entry j
//            (64 entries per pass) and rebuilds any word of the owner's
//            state from LDS tables alone (no per-lane state is kept beyond
//            the 4 phase-1 words).  Because the state is linear in x, the
//            state at step r of the current segment of lane l is the XOR of
//              Ref      the state at the item's reference index (an aligned
//                       index at or below the item's first chunk),
//              Lane(d)  the rows of the Gray bits that lane offset d sets,
//                       from four tables of its bits 0-2, 3-5, 6-8 and 9,
//              Seg      the rows of the Gray bits of the segment number
//                       (one row per wave, zero while c <= 12),
//              S(g12)   the rows of the Gray bits 0-11 of the step, from
//                       four tables of bits 0-2, 3-5, 6-8 and 9-11;
//            Ref is folded into the first lane table.  The remaining ridge
//            groups are checked with wave-uniform early exit, then the
//            facet count |K| (the upper-bound property of Section 4.2),
//            further affine properties g(K) > 0 (Section 2.1), the deferred
//            ridges (those beyond the resident groups, degree <= 2 read
//            directly off K) and x != 0 (x = 0 is allowed when the instance
//            is an affine coset K* + span, whose offset row is part of Ref).
//            Survivors are compacted with a wave ballot and prefix count into
//            per-wave chunks of record slots (one global atomic per chunk);
//            per-instance counts are flushed once per item.
// Dot products and parities reduce to AND, XOR and popcount on bit masks, as
// in Section 2.3.  The kernel is the same for every instance shape: ridge
// groups, slot strides and facet words are read from each table's header.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/wpm.h"

namespace wpm {

constexpr int DEV_HDR_WORDS = 16;  // must match the host packer's header size
enum {
    D_MAGIC = 0, D_K = 1, D_KP = 2, D_M = 3, D_W = 4, D_G = 5, D_QS = 6, D_RS = 7, D_MAXF = 8,
    D_FLAGS = 11, D_PROPS = 12, D_NPROPS = 13, D_DEFER = 14, D_NDEFER = 15
};
constexpr uint32_t D_TABLE_MAGIC = 0x314D5057u;  // "WPM1", written by the packer
constexpr uint32_t D_FLAG_OFFSET = 1;  // row kp holds the offset K* of an affine coset

// Lane offsets d inside an item's aligned window of 2^LANE_BITS chunks:
// the Gray code of d << c is (d ^ (d << 1)) << (c - 1), LANE_BITS + 1 bits.
constexpr int LANE_BITS = 9;
constexpr int LANE_ROWS = 8 + 8 + 8 + 2;  // tables of those bits 0-2, 3-5, 6-8, 9
constexpr int GRAY_ROWS = 32;             // tables of step Gray bits 0-2, 3-5, 6-8, 9-11
static_assert(GRAY_ROWS == WPM_TABLE_ROWS, "Gray-bit tables: 4 x 8 rows");
static_assert((1 << LANE_BITS) == WPM_LANE_WINDOW, "lane window of the ABI");

// Slots of d_total (uint64 words) the kernel updates.
enum { TOT_RESULTS = 0, TOT_SLOTS = 1, TOT_BAD_ITEMS = 2 };

struct KArgs {
    int64_t num_items;
    int64_t item_base;
    unsigned long long *head;
    uint64_t *surv;
    uint64_t cap;
    unsigned long long *counts;
    unsigned long long *total;  // [4]: results, record slots reserved, malformed items, reserved
    unsigned long long *stats;
    uint64_t *times;
    const int64_t *bins;  // mode 3: [grid + 1] item ranges per workgroup
    uint64_t chunk;       // record slots a wave reserves at a time (0: exactly what it needs)
    int mode;  // 0 direct (one item per workgroup), 1 static stride, 2 dynamic queue, 3 packed bins
    int num_instances;
    int max_rs, max_kp;  // the LDS of a workgroup holds tables up to these sizes
    int pad;
};

// Per ridge bit: at least 3 of the slot bits (a, b, c, d) set, given the
// stored words a, u = a^b, c, v = c^d.  Counting a + b = 2a when u = 0 and 1
// when u = 1 (likewise for c, d), the test is (u | a) & ~(u & v) & (v | c):
// two 3-input logic ops (v_bitop3; operand i is truth-table input 0xF0, 0xCC,
// 0xAA for i = 0, 1, 2).
__device__ __forceinline__ uint32_t fail4(uint32_t a, uint32_t u, uint32_t c, uint32_t v) {
    const uint32_t t = __builtin_amdgcn_bitop3_b32(u, a, v, 0x5C);  // (u | a) & ~(u & v)
    return __builtin_amdgcn_bitop3_b32(t, v, c, 0xE0);                // t & (v | c)
}

__device__ __forceinline__ uint32_t xor3(uint32_t a, uint32_t b, uint32_t c) {
    return __builtin_amdgcn_bitop3_b32(a, b, c, 0x96);
}

__device__ __forceinline__ uint64_t rfl64(uint64_t v) {
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
    return ((uint64_t)hi << 32) | lo;
}

// LDS of one workgroup (uint32 words), for row width RS and kp basis rows:
//   [nw][LIST_CAP]   a candidate list per wave
//   [4][bd]          the phase-1 words of every lane while its wave checks
//   [32][RS]         Gray-bit tables of the staged instance (steps' bits 0-11)
//   [26][RS]         lane tables of the current item (Ref in rows 0-7)
//   [nw][RS]         per-wave segment rows
//   [kp][4]          the phase-1 words of every basis row (block boundaries)
constexpr int PH1_CHAINS = 4;  // interleaved chains of the fast filter
constexpr int LIST_CAP = 256;   // candidates a wave's list holds
constexpr int LIST_FLUSH = 128; // a block ending with at least this many checks them
__host__ __device__ constexpr size_t sweep_lds_bytes(int max_kp, int max_row_words, int wg_size) {
    return sizeof(uint32_t) *
           ((size_t)(wg_size / 64) * LIST_CAP + (size_t)4 * wg_size +
            (size_t)(GRAY_ROWS + LANE_ROWS + wg_size / 64) * (size_t)max_row_words +
            (size_t)4 * (size_t)max_kp);
}

// This lane's index in its wave, computed where it is used (inline asm keeps
// it from being hoisted): a value kept from the kernel start would hold a
// VGPR through the whole sweep.
__device__ __forceinline__ int lane_now() {
    uint32_t l;
    asm volatile("v_mbcnt_lo_u32_b32 %0, -1, 0\n\tv_mbcnt_hi_u32_b32 %0, -1, %0" : "=v"(l));
    return (int)l;
}

// A uniform pointer through an opaque register copy: the loads it feeds are
// re-issued where they are used instead of holding scalar registers through
// phase 1.
template <class T>
__device__ __forceinline__ const T *opaque(const T *p) {
    asm volatile("" : "+s"(p));
    return p;
}

// Occupancy: the kernel is compiled for WAVES waves per SIMD.  Its state is
// the four phase-1 chains and loop control; everything a check needs comes
// from LDS.
template <int WAVES>
__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(WAVES)))
void sweep_kernel(const uint32_t *__restrict__ tables, const int64_t *__restrict__ offsets,
                  const wpm_item *__restrict__ items, KArgs a_in) {
    extern __shared__ __attribute__((aligned(16))) uint32_t lds_dyn[];
    __shared__ unsigned long long s_item;
    // The launch arguments live in LDS: the check reads them there, which
    // keeps them out of the scalar registers the fast loop needs.
    __shared__ KArgs s_a;
    if (threadIdx.x == 0) s_a = a_in;
    __syncthreads();
    const KArgs &a = s_a;
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int bd = blockDim.x;
    const int nw = bd >> 6;
    // the wave's index, as a wave-uniform (scalar) value
    const int wv = (int)__builtin_amdgcn_readfirstlane((uint32_t)(tid >> 6));
    auto tid_now = [&]() { return wv * 64 + lane_now(); };
    uint32_t *const lds_S = lds_dyn + nw * LIST_CAP;  // [4][bd] phase-1 words during checks
    uint32_t *const lds_T = lds_S + 4 * bd;           // tables start here
    int64_t staged = -1;
    // Per-wave bookkeeping, only touched by the checks: it lives in LDS, so
    // that none of it holds scalar registers through phase 1.
    // [out_pos, out_end) is the wave's current chunk of record slots.
    struct Book {
        uint64_t out_pos, out_end, wave_total;
        uint32_t item_cnt, n_cand, n_ridge, n_ubt, n_pass, n_redo;
    };
    __shared__ Book s_book[512 / 64];
    Book &bk = s_book[wv];
    bk.out_pos = bk.out_end = bk.wave_total = 0;
    bk.item_cnt = bk.n_cand = bk.n_ridge = bk.n_ubt = bk.n_pass = bk.n_redo = 0;
    // this wave's candidate list: entries (step r12 << 6) | lane
    uint32_t *lds_W = lds_dyn + wv * LIST_CAP;

    for (int64_t round = 0;; ++round) {
        int64_t it;
        if (a.mode == 0) {
            if (round > 0) break;
            it = a.item_base + (int64_t)blockIdx.x;
        } else if (a.mode == 1) {
            it = (int64_t)blockIdx.x + round * (int64_t)gridDim.x;
        } else if (a.mode == 3) {
            const int64_t b0 = a.bins[blockIdx.x], b1 = a.bins[blockIdx.x + 1];
            it = b0 + round;
            if (it >= b1) break;
        } else {
            if (tid_now() == 0) s_item = atomicAdd(a.head, 1ull);
            __syncthreads();
            it = (int64_t)s_item;
        }
        if (it >= a.num_items) break;
        uint64_t t_start = 0;
        if (tid_now() == 0 && a.times) t_start = __builtin_amdgcn_s_memrealtime();

        const wpm_item itm = items[it];
        const uint32_t inst = __builtin_amdgcn_readfirstlane(itm.instance);
        const int c = __builtin_amdgcn_readfirstlane((uint32_t)itm.cbits);
        const int lanes = __builtin_amdgcn_readfirstlane((uint32_t)itm.lanes);
        const uint64_t first = rfl64(itm.first);
        // A malformed item (unknown instance or table, a table larger than
        // the launch's LDS layout, chunk bits outside
        // [7, kp], lanes outside [1, workgroup], chunks beyond 2^kp, or a lane
        // window crossing an aligned group of 2^LANE_BITS chunks) is skipped
        // and counted; the caller sees it in d_total.
        bool bad = inst >= (uint32_t)a.num_instances;
        const uint32_t *__restrict__ tab = tables;
        int kp = 7, W = 0, G = 1, RS = 4, Qp = 4;
        bool has_off = false;
        if (!bad) {
            tab = tables + rfl64((uint64_t)offsets[inst]);
            kp = (int)tab[D_KP];
            W = (int)tab[D_W];
            G = (int)tab[D_G];
            Qp = (int)tab[D_QS];
            RS = (int)tab[D_RS];
            has_off = (tab[D_FLAGS] & D_FLAG_OFFSET) != 0u;
            bad = tab[D_MAGIC] != D_TABLE_MAGIC || kp < 7 || kp > a.max_kp || RS > a.max_rs || (RS & 3) ||
                  G < 1 || (Qp != 4 && Qp != 8) || 4 + (G - 1) * Qp + W > RS || c < 7 || c > kp ||
                  lanes < 1 || lanes > bd || (int)(first & ((1u << LANE_BITS) - 1)) + lanes > (1 << LANE_BITS) ||
                  first + (uint64_t)lanes > (1ull << (kp - c));
        }
        if (bad) {
            if (tid_now() == 0) {
                atomicAdd(a.total + TOT_BAD_ITEMS, 1ull);
                if (a.times) a.times[2 * it] = a.times[2 * it + 1] = 0;
            }
            __syncthreads();
            continue;
        }
        const uint32_t *__restrict__ rows = tab + DEV_HDR_WORDS;
        uint32_t *const lds_L = lds_T + GRAY_ROWS * RS;      // [26][RS]
        uint32_t *const lds_seg = lds_L + LANE_ROWS * RS;    // [nw][RS]
        uint32_t *const lds_R4 = lds_seg + nw * RS;          // [kp][4]

        // ---- set-up of the staged instance: Gray-bit tables (row v of
        // table b = XOR of the basis rows 3b + j over the set bits j of v;
        // rows >= kp count as zero) and the phase-1 words of every row.  A
        // thread takes one word of one table: its three row words are loaded
        // together, then the 8 rows are written.
        if ((int64_t)inst != staged) {
            for (int e = tid_now(); e < 4 * RS; e += bd) {
                const int b = e / RS, w = e - b * RS;
                const int t0 = 3 * b;
                const uint32_t r0 = t0 < kp ? rows[t0 * RS + w] : 0u;
                const uint32_t r1 = t0 + 1 < kp ? rows[(t0 + 1) * RS + w] : 0u;
                const uint32_t r2 = t0 + 2 < kp ? rows[(t0 + 2) * RS + w] : 0u;
                uint32_t *dst = lds_T + (8 * b) * RS + w;
#pragma unroll
                for (int v = 0; v < 8; ++v)
                    dst[v * RS] = ((v & 1) ? r0 : 0u) ^ ((v & 2) ? r1 : 0u) ^ ((v & 4) ? r2 : 0u);
            }
            for (int e = tid_now(); e < 4 * kp; e += bd) lds_R4[e] = rows[(e >> 2) * RS + (e & 3)];
            staged = inst;
        }
        // ---- set-up of the item: the reference index is the first chunk
        // rounded down to a multiple of 2^LANE_BITS; Ref = offset + the rows
        // of its Gray bits (all at or above c + LANE_BITS - 1).  Lane table
        // b, row v: the rows c - 1 + 3b + j over the set bits j of v (rows >=
        // kp count as zero), with Ref added to every row of table 0.  A
        // thread takes one word of one table, as above; the rows of Ref are
        // loaded unconditionally and masked, so their loads are independent.
        const uint64_t ref = first & ~(uint64_t)((1u << LANE_BITS) - 1);
        const uint64_t iref = ref << c;
        const uint64_t xref = iref ^ (iref >> 1);
        for (int e = tid_now(); e < 4 * RS; e += bd) {
            const int b = e / RS, w = e - b * RS;
            const int t0 = c - 1 + 3 * b;
            const int nv = b < 3 ? 8 : 2;
            const uint32_t r0 = t0 < kp ? rows[t0 * RS + w] : 0u;
            const uint32_t r1 = b < 3 && t0 + 1 < kp ? rows[(t0 + 1) * RS + w] : 0u;
            const uint32_t r2 = b < 3 && t0 + 2 < kp ? rows[(t0 + 2) * RS + w] : 0u;
            uint32_t base = 0;
            if (b == 0) {
                base = has_off ? rows[kp * RS + w] : 0u;
                for (int t = c + LANE_BITS - 1; t < kp; ++t)
                    base ^= rows[t * RS + w] & (0u - (uint32_t)((xref >> t) & 1ull));
            }
            uint32_t *dst = lds_L + (8 * b) * RS + w;
            for (int v = 0; v < nv; ++v)
                dst[v * RS] = base ^ ((v & 1) ? r0 : 0u) ^ ((v & 2) ? r1 : 0u) ^ ((v & 4) ? r2 : 0u);
        }
        for (int w = tid_now(); w < nw * RS; w += bd) lds_seg[w] = 0u;
        __syncthreads();

        bk.item_cnt = 0;  // results of this item found by this wave
        // wave-uniform test (readfirstlane tells the compiler so)
        if (wv * 64 < lanes) {
            const uint32_t dbase = (uint32_t)(first - ref);
            // LDS word offsets of the rows of a state: the lane part of lane
            // offset d and the step part of Gray bits g12
            auto lane_rows = [&](uint32_t d, uint32_t *o) {
                const uint32_t g = d ^ (d << 1);
                o[0] = (g & 7u) * (uint32_t)RS;
                o[1] = (8u + ((g >> 3) & 7u)) * (uint32_t)RS;
                o[2] = (16u + ((g >> 6) & 7u)) * (uint32_t)RS;
                o[3] = (24u + ((g >> 9) & 1u)) * (uint32_t)RS;
            };
            auto step_rows = [&](uint32_t g12, uint32_t *o) {
                o[0] = (g12 & 7u) * (uint32_t)RS;
                o[1] = (8u + ((g12 >> 3) & 7u)) * (uint32_t)RS;
                o[2] = (16u + ((g12 >> 6) & 7u)) * (uint32_t)RS;
                o[3] = (24u + ((g12 >> 9) & 7u)) * (uint32_t)RS;
            };
            const uint32_t *segw = lds_seg + wv * RS;
            // four consecutive state words at word offset off (a multiple of 4)
            // (read two tables at a time, so that few loads are in flight:
            // the check must not take registers from the phase-1 loop)
            auto word4 = [&](const uint32_t *lo, const uint32_t *so, int off) {
                auto acc2 = [](uint4 r, const uint32_t *p, const uint32_t *q) {
                    const uint4 x = *(const uint4 *)p, y = *(const uint4 *)q;
                    r.x = xor3(r.x, x.x, y.x);
                    r.y = xor3(r.y, x.y, y.y);
                    r.z = xor3(r.z, x.z, y.z);
                    r.w = xor3(r.w, x.w, y.w);
                    asm volatile("" : "+v"(r.x), "+v"(r.y), "+v"(r.z), "+v"(r.w)::"memory");
                    return r;
                };
                uint4 r = *(const uint4 *)(segw + off);
                r = acc2(r, lds_L + lo[0] + off, lds_L + lo[1] + off);
                r = acc2(r, lds_L + lo[2] + off, lds_L + lo[3] + off);
                r = acc2(r, lds_T + so[0] + off, lds_T + so[1] + off);
                r = acc2(r, lds_T + so[2] + off, lds_T + so[3] + off);
                return r;
            };
            // one state word at any word offset
            auto word1 = [&](const uint32_t *lo, const uint32_t *so, int off) {
                return xor3(xor3(lds_L[lo[0] + off], lds_L[lo[1] + off], lds_L[lo[2] + off]),
                            xor3(lds_L[lo[3] + off], lds_T[so[0] + off], lds_T[so[1] + off]),
                            xor3(lds_T[so[2] + off], lds_T[so[3] + off], segw[off]));
            };
            // this lane's state at the start of its chunk: the lane part of
            // its own offset (step part zero)
            uint32_t s0, s1, s2, s3;
            {
                uint32_t lo[4], so[4] = {0u, 8u * (uint32_t)RS, 16u * (uint32_t)RS, 24u * (uint32_t)RS};
                lane_rows(dbase + (uint32_t)tid_now(), lo);
                const uint4 st = word4(lo, so, 0);
                s0 = st.x;
                s1 = st.y;
                s2 = st.z;
                s3 = st.w;
            }
            // The XOR operands of the steps inside a block (rows 0-3, the
            // phase-1 words): wave-uniform, but held in VGPRs, which issue
            // faster than scalar operands; they are re-read from LDS after
            // every check, so that they hold no registers through it.
            uint32_t d[4][4];
            auto load_d = [&]() {
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    const uint4 r = *(const uint4 *)(lds_R4 + 4 * t);
                    d[t][0] = r.x;
                    d[t][1] = r.y;
                    d[t][2] = r.z;
                    d[t][3] = r.w;
                    asm volatile("" : "+v"(d[t][0]), "+v"(d[t][1]), "+v"(d[t][2]), "+v"(d[t][3]));
                }
            };
            load_d();

            const uint64_t nblk = 1ull << (c - 6);
            const int wbase = wv * 64;
            uint32_t cnt = 0;  // wave-uniform: entries in the list
            // Header and item fields for the checks, re-read through an
            // opaque pointer (scalar cache) rather than held in scalar
            // registers through phase 1.
            auto hv = [&](int i) -> uint32_t { return __builtin_amdgcn_readfirstlane(opaque(tab)[i]); };
            // a wave-uniform table word at a computed address
            auto uw = [](const uint32_t *q) -> uint32_t { return __builtin_amdgcn_readfirstlane(*opaque(q)); };
            auto iv = [&]() -> wpm_item { return *opaque(items + rfl64((uint64_t)it)); };
            for (uint64_t blk = 0; blk < nblk; ++blk) {
                // ---- phase 1: fast filter over 64 Gray steps, run as NC
                // interleaved chains of 64 / NC steps: chain j starts at step
                // j * L (L = 64 / NC), whose low Gray bits are those of
                // jL ^ (jL >> 1).  Steps s + jL flip the same basis vector for
                // every chain (s + 1 < L), so they share the XOR operand; the
                // chains' fail words are reduced by 3-input minima and one
                // compare, and one rarely taken branch appends the passing
                // lanes of all chains to the wave's list (ballot + mbcnt give
                // the slots).  Steps that would overflow the list are only
                // marked in a scalar mask and rechecked below.
                constexpr int NC = PH1_CHAINS, SL = 64 / NC;
                // the chain offsets' Gray bits lie in 3-5: one row of table 1
                static_assert(SL % 8 == 0 && NC * SL == 64, "chain starts with Gray bits 3-5 only");
                uint64_t redo = 0;
                uint32_t c[NC][4];
#pragma unroll
                for (int j = 0; j < NC; ++j) {
                    const uint32_t g = (uint32_t)(j * SL) ^ ((uint32_t)(j * SL) >> 1);
                    if (j == 0) {
                        c[0][0] = s0; c[0][1] = s1; c[0][2] = s2; c[0][3] = s3;
                    } else {
                        const uint4 o = *(const uint4 *)(lds_T + (8u + (g >> 3)) * RS);
                        c[j][0] = s0 ^ o.x;
                        c[j][1] = s1 ^ o.y;
                        c[j][2] = s2 ^ o.z;
                        c[j][3] = s3 ^ o.w;
                    }
                }
#pragma unroll
                for (int st = 0; st < SL; ++st) {
                    uint32_t f[NC];
#pragma unroll
                    for (int j = 0; j < NC; ++j) f[j] = fail4(c[j][0], c[j][1], c[j][2], c[j][3]);
                    uint32_t fm = f[0];
#pragma unroll
                    for (int j = 1; j < NC; ++j) fm = fm < f[j] ? fm : f[j];
                    if (__builtin_expect(__builtin_amdgcn_ballot_w64(fm == 0u) != 0, 0)) {
                        uint64_t bm[NC];
                        uint32_t nn[NC], tot = 0;
#pragma unroll
                        for (int j = 0; j < NC; ++j) {
                            bm[j] = __builtin_amdgcn_ballot_w64(f[j] == 0u);
                            nn[j] = (uint32_t)__builtin_popcountll(bm[j]);
                            tot += nn[j];
                        }
                        if (cnt + tot <= (uint32_t)LIST_CAP) {
                            const uint32_t ln = (uint32_t)lane_now();
                            const uint32_t e = ((((uint32_t)blk & 63u) << 6 | (uint32_t)st) << 6) | ln;
                            uint32_t base = cnt;
#pragma unroll
                            for (int j = 0; j < NC; ++j) {
                                if (f[j] == 0u)
                                    lds_W[base + __builtin_amdgcn_mbcnt_hi((uint32_t)(bm[j] >> 32),
                                                                           __builtin_amdgcn_mbcnt_lo((uint32_t)bm[j], 0u))] =
                                        e + ((uint32_t)(SL * j) << 6);
                                base += nn[j];
                            }
                            cnt = base;
                        } else {
#pragma unroll
                            for (int j = 0; j < NC; ++j) redo |= bm[j] ? 1ull << (st + SL * j) : 0ull;
                        }
                    }
                    if (st < SL - 1) {
                        const int t = __builtin_ctz((unsigned)(st + 1));
#pragma unroll
                        for (int j = 0; j < NC; ++j) {
#pragma unroll
                            for (int q = 0; q < 4; ++q) c[j][q] ^= d[t][q];
                            // opaque copies: keep each chain an in-place XOR
                            // update (re-associating it from the block start
                            // would hold extra base copies in VGPRs)
                            asm volatile("" : "+v"(c[j][0]), "+v"(c[j][1]), "+v"(c[j][2]), "+v"(c[j][3]));
                        }
                    }
                }
                // the last chain ends at step 63: the state the block
                // boundary continues from
                s0 = c[NC - 1][0];
                s1 = c[NC - 1][1];
                s2 = c[NC - 1][2];
                s3 = c[NC - 1][3];
                // ---- check the list when it is half full, before the
                // segment changes and at the end of the item; list the
                // overflow steps first.  Blocks with nothing to do skip all of
                // it on a scalar test.
                const bool seg_end = blk + 1 == nblk || ((blk + 1) & 63ull) == 0;
                if (redo != 0 || cnt >= (uint32_t)LIST_FLUSH || (seg_end && cnt != 0)) {
                    // the phase-1 words wait in LDS meanwhile (the barrier
                    // keeps them out of VGPRs)
                    {
                        uint32_t *sv = lds_S + tid_now();
                        sv[0] = s0;
                        sv[bd] = s1;
                        sv[2 * bd] = s2;
                        sv[3 * bd] = s3;
                    }
                    asm volatile("" ::: "memory");
                    // step Gray bits of r12 in this segment: bit 12 of the
                    // Gray index, the segment parity, toggles Gray bit 11
                    const uint64_t sbase = (blk >> 6) << 12;
                    const uint32_t par = (uint32_t)((blk >> 6) & 1ull) << 11;
                    uint64_t rd = redo;
                    bk.n_redo += (uint32_t)__builtin_popcountll(redo);
                    uint32_t lo_own[4];
                    lane_rows(dbase + (uint32_t)tid_now(), lo_own);
                    for (;;) {
                        // overflow steps: every lane rechecks the fast filter
                        // on its rebuilt group-0 words; passing lanes are listed
                        while (rd != 0 && cnt + 64u <= (uint32_t)LIST_CAP) {
                            const uint32_t st = (uint32_t)__builtin_ctzll(rd);
                            rd &= rd - 1;
                            const uint32_t r12 = ((uint32_t)(blk & 63ull) << 6) | st;
                            uint32_t so[4];
                            step_rows((r12 ^ (r12 >> 1)) ^ par, so);
                            const uint4 w4 = word4(lo_own, so, 0);
                            const bool p0 = fail4(w4.x, w4.y, w4.z, w4.w) == 0u;
                            const uint64_t bp = __builtin_amdgcn_ballot_w64(p0);
                            if (p0)
                                lds_W[cnt + __builtin_amdgcn_mbcnt_hi((uint32_t)(bp >> 32),
                                                                      __builtin_amdgcn_mbcnt_lo((uint32_t)bp, 0u))] =
                                    (r12 << 6) | (uint32_t)lane_now();
                            cnt += (uint32_t)__builtin_popcountll(bp);
                        }
                        if (cnt >= (uint32_t)LIST_FLUSH || rd != 0 || seg_end) {
                            bk.n_cand += cnt;
                            // ---- check: lane j takes entry base + j
#pragma unroll 1
                            for (uint32_t base = 0; base < cnt; base += 64) {
                                ++bk.n_pass;
                                const uint32_t ln = (uint32_t)lane_now();
                                const uint32_t ent = base + ln < cnt ? lds_W[base + ln] : 0u;
                                const uint32_t own = ent & 63u, r12 = ent >> 6;
                                uint32_t lo[4], so[4];
                                lane_rows(dbase + (uint32_t)(wbase + (int)own), lo);
                                step_rows((r12 ^ (r12 >> 1)) ^ par, so);
                                // group 0 passed in phase 1; the other groups in
                                // decreasing rejection order, stopping once no
                                // entry passes.  Entries of lanes beyond the
                                // item's last chunk are dropped.
                                const wpm_item ci = iv();
                                bool pass = base + ln < cnt &&
                                            wbase + (int)own < (int)__builtin_amdgcn_readfirstlane((uint32_t)ci.lanes);
                                const int Gp = (int)hv(D_G), Qs = (int)hv(D_QS);
#pragma unroll 1
                                for (int g = 1; g < Gp; ++g) {
                                    if (__builtin_amdgcn_ballot_w64(pass) == 0) break;
                                    const int off = 4 + (g - 1) * Qs;
                                    const uint4 v = word4(lo, so, off);
                                    uint32_t fl;
                                    if (Qs == 4) {
                                        fl = fail4(v.x, v.y, v.z, v.w);
                                    } else {
                                        // up to 8 plain slot words: at least 3 set
                                        const uint4 v2 = word4(lo, so, off + 4);
                                        const uint32_t sw[8] = {v.x, v.y, v.z, v.w, v2.x, v2.y, v2.z, v2.w};
                                        uint32_t c1 = sw[0], c2 = 0, c3 = 0;
#pragma unroll
                                        for (int q = 1; q < 8; ++q) {
                                            c3 |= c2 & sw[q];
                                            c2 |= c1 & sw[q];
                                            c1 |= sw[q];
                                        }
                                        fl = c3;
                                    }
                                    pass = pass && fl == 0u;
                                }
                                // Gray index of the owner's step (the chunk
                                // start is recomputed, not held through phase 1)
                                const uint64_t f0 = rfl64(ci.first);
                                const int cc = (int)__builtin_amdgcn_readfirstlane((uint32_t)ci.cbits);
                                const uint64_t i = ((f0 + (uint64_t)(wbase + (int)own)) << cc) + sbase + (uint64_t)r12;
                                const uint64_t x = i ^ (i >> 1);
                                // x = 0 is the empty complex, except in a coset (K = K*)
                                const int kk = (int)hv(D_K);
                                const bool offs = (hv(D_FLAGS) & D_FLAG_OFFSET) != 0u;
                                pass = pass && (x != 0 || offs) && (kk >= 64 || (x >> kk) == 0);
                                if (__builtin_amdgcn_ballot_w64(pass)) {
                                    const int Wp = (int)hv(D_W), ko = 4 + (Gp - 1) * Qs;
                                    uint32_t cntf = 0;
#pragma unroll 1
                                    for (int w = 0; w < Wp; w += 4) {
                                        const uint4 v = word4(lo, so, ko + w);
                                        cntf += __builtin_popcount(v.x) + __builtin_popcount(v.y) +
                                                __builtin_popcount(v.z) + __builtin_popcount(v.w);
                                    }
                                    const uint32_t mf = hv(D_MAXF);
                                    bool ok = pass && (mf == 0u || cntf <= mf);
                                    // further affine properties g(K) = c0 + sum_c w_c |K & mask_c| > 0
                                    const uint32_t np = hv(D_NPROPS);
                                    if (np != 0u && __builtin_amdgcn_ballot_w64(ok) != 0) {
                                        const uint32_t *pr = tab + hv(D_PROPS);
#pragma unroll 1
                                        for (uint32_t q = 0; q < np; ++q) {
                                            int64_t gv = (int32_t)uw(pr);
                                            const uint32_t ncls = uw(pr + 1);
                                            pr += 2;
#pragma unroll 1
                                            for (uint32_t cl = 0; cl < ncls; ++cl) {
                                                uint32_t sum = 0;
#pragma unroll 1
                                                for (int w = 0; w < Wp; ++w)
                                                    sum += __builtin_popcount(word1(lo, so, ko + w) & uw(pr + 1 + w));
                                                gv += (int64_t)(int32_t)uw(pr) * (int64_t)sum;
                                                pr += 1 + Wp;
                                            }
                                            ok = ok && gv > 0;
                                        }
                                    }
                                    // deferred ridges: degree <= 2 in K, read off
                                    // the facet words (parent count, then the
                                    // parents' facet indices, per ridge)
                                    const uint32_t nd = hv(D_NDEFER);
                                    if (nd != 0u && __builtin_amdgcn_ballot_w64(ok) != 0) {
                                        const uint32_t *dr = tab + hv(D_DEFER);
#pragma unroll 1
                                        for (uint32_t q = 0; q < nd; ++q) {
                                            const uint32_t p = uw(dr);
                                            uint32_t deg = 0;
#pragma unroll 1
                                            for (uint32_t j = 0; j < p; ++j) {
                                                const uint32_t f = uw(dr + 1 + j);
                                                deg += (word1(lo, so, ko + (int)(f >> 5)) >> (f & 31u)) & 1u;
                                            }
                                            ok = ok && deg <= 2u;
                                            dr += 1 + p;
                                        }
                                    }
                                    const uint64_t pball = __builtin_amdgcn_ballot_w64(pass);
                                    const uint64_t bal = __builtin_amdgcn_ballot_w64(ok);
                                    bk.n_ridge += (uint32_t)__builtin_popcountll(pball);
                                    bk.n_ubt += (uint32_t)__builtin_popcountll(pball & ~bal);
                                    if (bal) {
                                        const uint32_t nbal = (uint32_t)__builtin_popcountll(bal);
                                        bk.item_cnt += nbal;
                                        // the wave's current chunk of record slots
                                        // is [out_pos, out_end); results that do
                                        // not fit continue at the start of a newly
                                        // reserved chunk (one global atomic per
                                        // a.chunk slots), so slots stay unused only
                                        // at the end of each wave's last chunk
                                        const uint64_t out_pos = bk.out_pos;
                                        uint64_t out_end = bk.out_end;
                                        const uint32_t room = (uint32_t)(out_end - out_pos);
                                        uint64_t next = 0;
                                        if (nbal > room) {
                                            const uint64_t over = nbal - room;
                                            const uint64_t want = a.chunk > over ? a.chunk : over;
                                            unsigned long long rbase = 0;
                                            if (lane_now() == 0) rbase = atomicAdd(a.total + TOT_SLOTS, (unsigned long long)want);
                                            next = rfl64(rbase);
                                            out_end = next + want;
                                        }
                                        if (ok) {
                                            const uint32_t rk = __builtin_amdgcn_mbcnt_hi(
                                                (uint32_t)(bal >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)bal, 0u));
                                            const uint64_t pos = rk < room ? out_pos + rk : next + (rk - room);
                                            if (pos < a.cap) {
                                                a.surv[2 * pos] = x;
                                                a.surv[2 * pos + 1] = __builtin_amdgcn_readfirstlane(ci.instance);
                                            }
                                        }
                                        bk.out_pos = nbal > room ? next + (nbal - room) : out_pos + nbal;
                                        bk.out_end = out_end;
                                    }
                                }
                            }
                            cnt = 0;
                        }
                        if (rd == 0) break;
                    }
                    asm volatile("" ::: "memory");
                    {
                        const uint32_t *sv = lds_S + tid_now();
                        s0 = sv[0];
                        s1 = sv[bd];
                        s2 = sv[2 * bd];
                        s3 = sv[3 * bd];
                    }
                    load_d();
                }
                // ---- block boundary: one more Gray step, flipping t >= 6;
                // a flip of t >= 12 starts a new segment, whose rows join the
                // wave's segment row
                if (blk + 1 < nblk) {
                    const int t = 6 + __builtin_ctzll(blk + 1);
                    if (t >= 12) {
                        const int RSb = (int)hv(D_RS);
                        const uint32_t *row = opaque(tab) + DEV_HDR_WORDS + t * RSb;
                        uint32_t *sgw = lds_seg + wv * RSb;
                        for (int w = lane_now(); w < RSb; w += 64) sgw[w] ^= row[w];
                    }
                    const uint4 r4 = *(const uint4 *)(lds_R4 + 4 * t);
                    s0 ^= r4.x;
                    s1 ^= r4.y;
                    s2 ^= r4.z;
                    s3 ^= r4.w;
                }
            }
        }
        const uint32_t item_cnt = bk.item_cnt;
        if (item_cnt && lane_now() == 0) atomicAdd(a.counts + inst, (unsigned long long)item_cnt);
        bk.wave_total += item_cnt;
        __syncthreads();
        if (tid_now() == 0 && a.times) {
            a.times[2 * it] = t_start;
            a.times[2 * it + 1] = __builtin_amdgcn_s_memrealtime();
        }
    }
    // close this wave's output chunk and publish its totals
    const uint64_t out_pos = bk.out_pos, out_end = bk.out_end, wave_total = bk.wave_total;
    const uint32_t n_cand = bk.n_cand, n_ridge = bk.n_ridge, n_ubt = bk.n_ubt, n_pass = bk.n_pass;
    const uint32_t n_redo = bk.n_redo;
    for (uint64_t e0 = out_pos + (uint64_t)lane; e0 < out_end && e0 < a.cap; e0 += 64) {
        a.surv[2 * e0] = 0;
        a.surv[2 * e0 + 1] = ~0ull;
    }
    if (lane == 0 && wave_total) atomicAdd(a.total + TOT_RESULTS, (unsigned long long)wave_total);
    if (a.stats && lane == 0 && (n_cand | n_ridge | n_ubt | n_pass | n_redo)) {
        atomicAdd(a.stats + 0, (unsigned long long)n_cand);
        atomicAdd(a.stats + 1, (unsigned long long)n_ridge);
        atomicAdd(a.stats + 2, (unsigned long long)n_ubt);
        atomicAdd(a.stats + 3, (unsigned long long)n_pass);
        atomicAdd(a.stats + 4, (unsigned long long)n_redo);
    }
}

}  // namespace wpm
