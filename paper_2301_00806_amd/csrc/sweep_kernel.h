// The Gray-code sweep of the F2 kernel on gfx950 (device code).
//
// Every lane owns a chunk of 2^c consecutive Gray indices i of one instance
// and visits x = i ^ (i >> 1), so consecutive vectors differ in the single
// basis vector t = ctz(i + 1) and K changes by XOR with that basis row
// (Section 2.1: the weak pseudo-manifolds are among the 2^k combinations of a
// kernel basis).  Chunks are 2^c-aligned with c >= 7, so all lanes of a
// workgroup flip the same t at the same step: the XOR operands are
// wave-uniform and live in SGPRs.
//
// A step checks the ridges whose parents Proposition 2.1 constrains, in the
// bit-sliced slot form built by the packer (a ridge fails iff at least 3 of
// its first p-1 parent bits are set).  Work per block of 64 steps:
//   phase 1  the fast filter: 32 ridges in 4 slot words held in VGPRs,
//            updated by 4 XORs and tested by 2 bit-logic ops per step, the
//            two halves of the block as interleaved chains.  When a lane
//            passes (a rarely taken branch), the passing lanes append
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
// 0xAA for i = 0, 1, 2).  The test is symmetric in the pairs (a, u) and
// (c, v); which pair the second op reads decides whether its three operands
// sit in three VGPR banks under the compiler's allocation (a shared bank
// costs issue cycles), and this order gives distinct banks in the sweep loop.
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
//   [RS]             the item's reference state (set-up only)
//   [kp][4]          the phase-1 words of every basis row (block boundaries)
constexpr int LIST_CAP = 256;   // candidates a wave's list holds
constexpr int LIST_FLUSH = 128; // a block ending with at least this many checks them
__host__ __device__ constexpr size_t sweep_lds_bytes(int max_kp, int max_row_words, int wg_size) {
    return sizeof(uint32_t) *
           ((size_t)(wg_size / 64) * LIST_CAP + (size_t)4 * wg_size +
            (size_t)(GRAY_ROWS + LANE_ROWS + wg_size / 64 + 1) * (size_t)max_row_words +
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
// the two phase-1 chains and loop control; everything a check needs comes
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
        uint32_t *const lds_ref = lds_seg + nw * RS;         // [RS]
        uint32_t *const lds_R4 = lds_ref + RS;               // [kp][4]

        // ---- set-up of the staged instance: Gray-bit tables (row v of
        // table b = XOR of the basis rows 3b + j over the set bits j of v;
        // rows >= kp count as zero) and the phase-1 words of every row
        if ((int64_t)inst != staged) {
            for (int e = tid_now(); e < GRAY_ROWS * RS; e += bd) {
                const int v = e / RS, w = e - v * RS;
                const int t0 = 3 * (v >> 3);
                uint32_t acc = 0;
                for (int t = 0; t < 3; ++t)
                    if (((v >> t) & 1) && t0 + t < kp) acc ^= rows[(t0 + t) * RS + w];
                lds_T[e] = acc;
            }
            for (int e = tid_now(); e < 4 * kp; e += bd) lds_R4[e] = rows[(e >> 2) * RS + (e & 3)];
            staged = inst;
        }
        // ---- set-up of the item: the reference index is the first chunk
        // rounded down to a multiple of 2^LANE_BITS; Ref = offset + the rows
        // of its Gray bits (all at or above c + LANE_BITS - 1)
        const uint64_t ref = first & ~(uint64_t)((1u << LANE_BITS) - 1);
        const uint64_t iref = ref << c;
        const uint64_t xref = iref ^ (iref >> 1);
        for (int w = tid_now(); w < RS; w += bd) lds_ref[w] = has_off ? rows[kp * RS + w] : 0u;
        for (int w = tid_now(); w < nw * RS; w += bd) lds_seg[w] = 0u;
        __syncthreads();
        {
            const int nb = __builtin_popcountll(xref);
            for (int e = tid_now(); e < nb * RS; e += bd) {
                const int j = e / RS, w = e - j * RS;
                uint64_t m = xref;
                for (int q = 0; q < j; ++q) m &= m - 1;
                const int t = __builtin_ctzll(m);
                if (t < kp) atomicXor(lds_ref + w, rows[t * RS + w]);
            }
        }
        __syncthreads();
        // lane table b, row v: the rows c - 1 + 3b + j over the set bits j of
        // v (rows >= kp count as zero), plus Ref in table 0
        for (int e = tid_now(); e < LANE_ROWS * RS; e += bd) {
            const int v = e / RS, w = e - v * RS;
            const int b = v >> 3, vv = v & 7;
            const int nbits = b < 3 ? 3 : 1;
            const int t0 = c - 1 + 3 * b;
            uint32_t acc = b == 0 ? lds_ref[w] : 0u;
            for (int t = 0; t < nbits; ++t)
                if (((vv >> t) & 1) && t0 + t < kp) acc ^= rows[(t0 + t) * RS + w];
            lds_L[e] = acc;
        }
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
            uint32_t d[6][4];
#pragma unroll
            for (int t = 0; t < 6; ++t)
#pragma unroll
                for (int q = 0; q < 4; ++q) d[t][q] = __builtin_amdgcn_readfirstlane(lds_R4[t * 4 + q]);

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
                // ---- phase 1: fast filter over 64 Gray steps, run as two
                // interleaved chains: steps 0..31 from the block-start state
                // and steps 32..63 from the state at step 32 (the low Gray
                // bits of step 32 are bits 4 and 5).  Steps s and s + 32 flip
                // the same basis vector, so both chains share the XOR operand;
                // a step costs 7 VALU ops, and one rarely taken branch covers
                // two steps and appends the passing lanes to the wave's list
                // (ballot + mbcnt give the slots).  Steps that would overflow
                // the list are only marked in a scalar mask and rechecked below.
                uint64_t redo = 0;
                // rows 4 ^ 5: row 6 of the Gray-bit table of bits 3-5 (read
                // from LDS: scalar registers are the scarcer resource here)
                const uint4 r45 = *(const uint4 *)(lds_T + 14 * RS);
                uint32_t b0 = s0 ^ r45.x, b1 = s1 ^ r45.y, b2 = s2 ^ r45.z, b3 = s3 ^ r45.w;
#pragma unroll
                for (int s = 0; s < 32; ++s) {
                    const uint32_t fa = fail4(s0, s1, s2, s3);
                    const uint32_t fb = fail4(b0, b1, b2, b3);
                    const uint32_t fm = fa < fb ? fa : fb;
                    if (__builtin_expect(__builtin_amdgcn_ballot_w64(fm == 0u) != 0, 0)) {
                        const uint64_t ba = __builtin_amdgcn_ballot_w64(fa == 0u);
                        const uint64_t bb = __builtin_amdgcn_ballot_w64(fb == 0u);
                        const uint32_t na = (uint32_t)__builtin_popcountll(ba);
                        const uint32_t nb = (uint32_t)__builtin_popcountll(bb);
                        if (cnt + na + nb <= (uint32_t)LIST_CAP) {
                            // the lane id, recomputed here (a value kept
                            // from the kernel start would hold a VGPR)
                            const uint32_t ln = (uint32_t)lane_now();
                            const uint32_t e = ((((uint32_t)blk & 63u) << 6 | (uint32_t)s) << 6) | ln;
                            if (fa == 0u)
                                lds_W[cnt + __builtin_amdgcn_mbcnt_hi((uint32_t)(ba >> 32),
                                                                      __builtin_amdgcn_mbcnt_lo((uint32_t)ba, 0u))] = e;
                            if (fb == 0u)
                                lds_W[cnt + na + __builtin_amdgcn_mbcnt_hi((uint32_t)(bb >> 32),
                                                                           __builtin_amdgcn_mbcnt_lo((uint32_t)bb, 0u))] =
                                    e + (32u << 6);
                            cnt += na + nb;
                        } else {
                            redo |= (ba ? 1ull << s : 0ull) | (bb ? 1ull << (s + 32) : 0ull);
                        }
                    }
                    if (s < 31) {
                        const int t = __builtin_ctz((unsigned)(s + 1));
                        s0 ^= d[t][0];
                        s1 ^= d[t][1];
                        s2 ^= d[t][2];
                        s3 ^= d[t][3];
                        b0 ^= d[t][0];
                        b1 ^= d[t][1];
                        b2 ^= d[t][2];
                        b3 ^= d[t][3];
                        // opaque copies: keep each chain an in-place XOR
                        // update (re-associating it from the block start
                        // would hold extra base copies in VGPRs)
                        asm volatile("" : "+v"(s0), "+v"(s1), "+v"(s2), "+v"(s3));
                        asm volatile("" : "+v"(b0), "+v"(b1), "+v"(b2), "+v"(b3));
                    }
                }
                // the second chain ends at step 63: the state the block
                // boundary continues from
                s0 = b0;
                s1 = b1;
                s2 = b2;
                s3 = b3;
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
                                        uint64_t out_pos = bk.out_pos, out_end = bk.out_end;
                                        if (out_pos + nbal > out_end) {
                                            // close the current chunk with sentinel
                                            // records and reserve a new one (one
                                            // global atomic per a.chunk record slots)
                                            for (uint64_t e0 = out_pos + (uint64_t)lane_now(); e0 < out_end && e0 < a.cap;
                                                 e0 += 64) {
                                                a.surv[2 * e0] = 0;
                                                a.surv[2 * e0 + 1] = ~0ull;
                                            }
                                            const uint64_t want = a.chunk > nbal ? a.chunk : nbal;
                                            unsigned long long rbase = 0;
                                            if (lane_now() == 0) rbase = atomicAdd(a.total + TOT_SLOTS, (unsigned long long)want);
                                            out_pos = rfl64(rbase);
                                            out_end = out_pos + want;
                                        }
                                        if (ok) {
                                            const uint32_t rk = __builtin_amdgcn_mbcnt_hi(
                                                (uint32_t)(bal >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)bal, 0u));
                                            const uint64_t pos = out_pos + rk;
                                            if (pos < a.cap) {
                                                a.surv[2 * pos] = x;
                                                a.surv[2 * pos + 1] = __builtin_amdgcn_readfirstlane(ci.instance);
                                            }
                                        }
                                        bk.out_pos = out_pos + nbal;
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
