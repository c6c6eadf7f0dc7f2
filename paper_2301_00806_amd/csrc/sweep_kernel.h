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
//            (64 entries per pass).  The full state of the owner lane at
//            step r of its chunk is P ^ S(gray(r)): P (the owner's VGPRs,
//            fetched with ds_bpermute) is the state at the segment start and
//            S(gray(r)) the XOR of four 8-row LDS tables indexed by the Gray
//            bits 0-2, 3-5, 6-8 and 9-11.  The remaining ridge groups are
//            checked with wave-uniform early exit, then the facet count |K|
//            (the upper-bound property of Section 4.2), further affine
//            properties g(K) > 0 (Section 2.1) and x != 0 (x = 0 is allowed
//            when the instance is an affine coset K* + span, whose offset
//            row is added to every state).  Survivors are compacted with a
//            wave ballot and prefix count into per-wave chunks of record
//            slots (one global atomic per chunk); per-instance counts are
//            flushed once per item.
// P therefore changes only when a step flips a basis vector t >= 12, once
// per 4096 steps; phase 1 updates its 4 words at every block boundary.
// Dot products and parities reduce to AND, XOR and popcount on bit masks, as
// in Section 2.3.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/wpm.h"

namespace wpm {

constexpr int DEV_HDR_WORDS = 16;  // must match the host packer's header size
enum {
    D_K = 1, D_KP = 2, D_M = 3, D_W = 4, D_G = 5, D_QS = 6, D_RS = 7, D_MAXF = 8,
    D_FLAGS = 11, D_PROPS = 12, D_NPROPS = 13
};
constexpr uint32_t D_FLAG_OFFSET = 1;  // row kp holds the offset K* of an affine coset

struct KArgs {
    int64_t num_items;
    int64_t item_base;
    unsigned long long *head;
    uint64_t *surv;
    uint64_t cap;
    unsigned long long *counts;
    unsigned long long *total;
    unsigned long long *slots;  // record slots reserved so far (chunk allocator)
    unsigned long long *stats;
    uint64_t *times;
    const int64_t *bins;  // mode 3: [grid + 1] item ranges per workgroup
    uint64_t chunk;       // record slots a wave reserves at a time (0: exactly what it needs)
    int mode;  // 0 direct (one item per workgroup), 1 static stride, 2 dynamic queue, 3 packed bins
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

template <int QS>
__device__ __forceinline__ uint32_t fail_slots(const uint32_t *s) {
    if constexpr (QS == 4) {
        return fail4(s[0], s[1], s[2], s[3]);
    } else {
        uint32_t c1 = s[0], c2 = 0, c3 = 0;
#pragma unroll
        for (int q = 1; q < QS; ++q) {
            c3 |= c2 & s[q];
            c2 |= c1 & s[q];
            c1 |= s[q];
        }
        return c3;
    }
}

template <int GM, int QS, int WM>
struct Layout {
    static constexpr int KR = 4 + (GM - 1) * QS;  // register index of the facet words
    static constexpr int PW = KR + WM;
};

// P ^= row & msk over the words an instance uses.  Registers use the
// template stride QS; the row uses the instance's own stride mqs (<= QS).
// P = row over the words an instance uses (unused register words are 0).
template <int GM, int QS, int WM>
__device__ __forceinline__ void load_row(uint32_t *P, const uint32_t *row, int G, int W, int mqs) {
    constexpr int KR = Layout<GM, QS, WM>::KR;
#pragma unroll
    for (int q = 0; q < 4; ++q) P[q] = row[q];
#pragma unroll
    for (int g = 1; g < GM; ++g)
#pragma unroll
        for (int q = 0; q < QS; ++q)
            P[4 + (g - 1) * QS + q] = (g < G && (QS == 4 || q < mqs)) ? row[4 + (g - 1) * mqs + q] : 0u;
    const int koff = 4 + (G - 1) * mqs;
#pragma unroll
    for (int w = 0; w < WM; ++w) P[KR + w] = w < W ? row[koff + w] : 0u;
}

template <int GM, int QS, int WM>
__device__ __forceinline__ void xor_row(uint32_t *P, const uint32_t *row, uint32_t msk, int G,
                                        int W, int mqs) {
    constexpr int KR = Layout<GM, QS, WM>::KR;
#pragma unroll
    for (int q = 0; q < 4; ++q) P[q] ^= row[q] & msk;
#pragma unroll
    for (int g = 1; g < GM; ++g) {
        if (g < G) {
#pragma unroll
            for (int q = 0; q < QS; ++q)
                if (QS == 4 || q < mqs) P[4 + (g - 1) * QS + q] ^= row[4 + (g - 1) * mqs + q] & msk;
        }
    }
    const int koff = 4 + (G - 1) * mqs;
#pragma unroll
    for (int w = 0; w < WM; ++w)
        if (w < W) P[KR + w] ^= row[koff + w] & msk;
}

__device__ __forceinline__ uint64_t rfl64(uint64_t v) {
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
    return ((uint64_t)hi << 32) | lo;
}

// LDS of one workgroup: a candidate list per wave and the phase-1 save area,
// then the tables of the staged instance (RS words per row): 4 x 8 rows for
// the Gray bits 0-2, 3-5, 6-8 and 9-11, the kp basis rows plus the offset row,
// and the reference state of the current item.
constexpr int LIST_CAP = 256;   // candidates a wave's list holds
constexpr int LIST_FLUSH = 128; // a block ending with at least this many checks them
__host__ __device__ constexpr size_t sweep_lds_bytes(int max_kp, int max_row_words, int wg_size) {
    return (size_t)wg_size * (LIST_CAP / 64 + 4) * sizeof(uint32_t) +
           (size_t)(WPM_TABLE_ROWS + max_kp + 2) * (size_t)max_row_words * sizeof(uint32_t);
}

// Occupancy: every instantiation is compiled for WPM_SWEEP_WAVES waves per
// SIMD.  The hot state (the two phase-1 chains) needs few VGPRs; the words of
// P that do not fit are spilled, and P is only read by the list checks and
// written once per 4096 steps.
#ifndef WPM_SWEEP_WAVES
#define WPM_SWEEP_WAVES 7
#endif
template <int GM, int QS, int WM>
__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(WPM_SWEEP_WAVES)))
void sweep_kernel(const uint32_t *__restrict__ tables, const int64_t *__restrict__ offsets,
                  const wpm_item *__restrict__ items, KArgs a_in) {
    extern __shared__ uint32_t lds_dyn[];
    __shared__ unsigned long long s_item;
    // The launch arguments live in LDS: the check reads them there, which
    // keeps them out of the scalar registers the fast loop needs.
    __shared__ KArgs s_a;
    if (threadIdx.x == 0) s_a = a_in;
    __syncthreads();
    const KArgs &a = s_a;
    constexpr int KR = Layout<GM, QS, WM>::KR;
    constexpr int PW = Layout<GM, QS, WM>::PW;
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int bd = blockDim.x;
    uint32_t *lds_S = lds_dyn + (bd / 64) * LIST_CAP;  // [4][bd] phase-1 words
    uint32_t *lds_L = lds_S + 4 * bd;                  // [32][RS] Gray-bit tables
    int64_t staged = -1;
    // Per-wave bookkeeping, only touched by the checks: it lives in LDS, so
    // that none of it holds scalar registers through phase 1 (the memory
    // barriers of the check keep the compiler from caching it there).
    // [out_pos, out_end) is the wave's current chunk of record slots.
    struct Book {
        uint64_t out_pos, out_end, wave_total;
        uint32_t item_cnt, n_cand, n_ridge, n_ubt, n_pass, n_redo;
    };
    __shared__ Book s_book[512 / 64];
    Book &bk = s_book[tid >> 6];
    bk.out_pos = bk.out_end = bk.wave_total = 0;
    bk.item_cnt = bk.n_cand = bk.n_ridge = bk.n_ubt = bk.n_pass = bk.n_redo = 0;
    // this wave's candidate list: entries (step r12 << 6) | lane
    uint32_t *lds_W = lds_dyn + (tid >> 6) * LIST_CAP;

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
            if (tid == 0) s_item = atomicAdd(a.head, 1ull);
            __syncthreads();
            it = (int64_t)s_item;
        }
        if (it >= a.num_items) break;
        uint64_t t_start = 0;
        if (tid == 0 && a.times) t_start = __builtin_amdgcn_s_memrealtime();

        const wpm_item itm = items[it];
        const uint32_t inst = __builtin_amdgcn_readfirstlane(itm.instance);
        const int c = __builtin_amdgcn_readfirstlane((uint32_t)itm.cbits);
        const int lanes = __builtin_amdgcn_readfirstlane((uint32_t)itm.lanes);
        const uint64_t first = rfl64(itm.first);
        const uint32_t *__restrict__ tab = tables + rfl64((uint64_t)offsets[inst]);
        const int k = (int)tab[D_K], kp = (int)tab[D_KP], W = (int)tab[D_W], G = (int)tab[D_G];
        const int RS = (int)tab[D_RS];
        const int mqs = (QS == 4) ? 4 : (int)tab[D_QS];
        const uint32_t maxf = tab[D_MAXF];
        const bool has_off = (tab[D_FLAGS] & D_FLAG_OFFSET) != 0u;
        const uint32_t *__restrict__ rows = tab + DEV_HDR_WORDS;

        uint32_t *lds_R = lds_L + WPM_TABLE_ROWS * RS;  // [kp + 1][RS] basis rows, offset
        if ((int64_t)inst != staged) {
            for (int e = tid; e < (kp + (has_off ? 1 : 0)) * RS; e += bd) lds_R[e] = rows[e];
            __syncthreads();
            // table b, row v: XOR of the rows 3b + j over the set bits j of v
            // (rows >= kp count as zero)
            for (int e = tid; e < WPM_TABLE_ROWS * RS; e += bd) {
                const int v = e / RS, w = e - v * RS;
                const int t0 = 3 * (v >> 3);
                uint32_t acc = 0;
                for (int t = 0; t < 3; ++t)
                    if (((v >> t) & 1) && t0 + t < kp) acc ^= lds_R[(t0 + t) * RS + w];
                lds_L[e] = acc;
            }
            __syncthreads();
            staged = inst;
        }
        // State at the start of the item's first chunk (x of Gray index
        // first * 2^c, plus the coset offset), one word per lane; every lane
        // then adds only the rows where its own start differs from it.
        uint32_t *lds_P = lds_R + (kp + 1) * RS;
        const uint64_t iref = first << c;
        const uint64_t xref = iref ^ (iref >> 1);
        for (int w = tid; w < RS; w += bd) {
            uint32_t acc = has_off ? lds_R[kp * RS + w] : 0u;
            for (int t = 6; t < kp; ++t)
                if ((xref >> t) & 1ull) acc ^= lds_R[t * RS + w];
            lds_P[w] = acc;
        }
        __syncthreads();

        bk.item_cnt = 0;  // results of this item found by this wave
        // wave-uniform test (readfirstlane tells the compiler so)
        if ((int)__builtin_amdgcn_readfirstlane((uint32_t)(tid & ~63)) < lanes) {
            const bool active = tid < lanes;
            const uint64_t j = first + (uint64_t)tid;
            const uint64_t i0 = active ? (j << c) : 0;
            const uint64_t x0 = i0 ^ (i0 >> 1);
            uint32_t P[PW];
            load_row<GM, QS, WM>(P, lds_P, G, W, mqs);
            // rows where this lane's start differs from the reference start
            // (consecutive chunks: usually only the few rows above c - 1);
            // rows no lane of the wave needs are skipped as a whole
            const uint64_t dx = active ? (x0 ^ xref) : 0ull;
            for (int t = 6; t < kp; ++t) {
                const bool bit = ((dx >> t) & 1ull) != 0;
                if (__builtin_amdgcn_ballot_w64(bit) == 0) continue;
                xor_row<GM, QS, WM>(P, lds_R + t * RS, bit ? ~0u : 0u, G, W, mqs);
            }
            uint32_t s0 = P[0], s1 = P[1], s2 = P[2], s3 = P[3];
            uint32_t d[6][4];
#pragma unroll
            for (int t = 0; t < 6; ++t)
#pragma unroll
                for (int q = 0; q < 4; ++q) d[t][q] = __builtin_amdgcn_readfirstlane(lds_R[t * RS + q]);

            const uint64_t nblk = 1ull << (c - 6);
            const int koff = 4 + (G - 1) * mqs;
            const int wbase = tid & ~63;
            uint32_t cnt = 0;  // wave-uniform: entries in the list
            // Header and item fields for the checks, re-read through an
            // opaque pointer (scalar cache) rather than held in scalar
            // registers through phase 1.
            auto hv = [&](int i) -> uint32_t {
                const uint32_t *tv = tab;
                asm volatile("" : "+s"(tv));
                return tv[i];
            };
            auto iv = [&]() -> wpm_item {
                const wpm_item *ip = items + rfl64((uint64_t)it);
                asm volatile("" : "+s"(ip));
                return *ip;
            };
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
                uint32_t b0 = s0 ^ d[4][0] ^ d[5][0], b1 = s1 ^ d[4][1] ^ d[5][1];
                uint32_t b2 = s2 ^ d[4][2] ^ d[5][2], b3 = s3 ^ d[4][3] ^ d[5][3];
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
                            const uint32_t ln = __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u));
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
                // ---- check the list when it is half full, before P changes
                // and at the end of the item; list the overflow steps first.
                // Blocks with nothing to do skip all of it on a scalar test.
                const bool seg_end = blk + 1 == nblk || ((blk + 1) & 63ull) == 0;
                if (redo != 0 || cnt >= (uint32_t)LIST_FLUSH || (seg_end && cnt != 0)) {
                    // the phase-1 words wait in LDS meanwhile (the barrier
                    // keeps them out of VGPRs)
                    lds_S[tid] = s0;
                    lds_S[bd + tid] = s1;
                    lds_S[2 * bd + tid] = s2;
                    lds_S[3 * bd + tid] = s3;
                    asm volatile("" ::: "memory");
                    // state words at step r12 of the segment: P ^ the four
                    // table rows of its Gray bits (bit 12 of the Gray index,
                    // the segment parity, toggles Gray bit 11)
                    const uint64_t sbase = (blk >> 6) << 12;
                    const uint32_t par = (uint32_t)((blk >> 6) & 1ull) << 11;
                    uint64_t rd = redo;
                    bk.n_redo += (uint32_t)__builtin_popcountll(redo);
                    for (;;) {
                        // overflow steps: every lane rechecks the fast filter
                        // on the rebuilt group-0 words; passing lanes are listed
                        while (rd != 0 && cnt + 64u <= (uint32_t)LIST_CAP) {
                            const uint32_t st = (uint32_t)__builtin_ctzll(rd);
                            rd &= rd - 1;
                            const uint32_t r12 = ((uint32_t)(blk & 63ull) << 6) | st;
                            const uint32_t g12 = (r12 ^ (r12 >> 1)) ^ par;
                            const uint32_t *T0 = lds_L + (g12 & 7u) * RS;
                            const uint32_t *T1 = lds_L + (8u + ((g12 >> 3) & 7u)) * RS;
                            const uint32_t *T2 = lds_L + (16u + ((g12 >> 6) & 7u)) * RS;
                            const uint32_t *T3 = lds_L + (24u + (g12 >> 9)) * RS;
                            uint32_t w4[4];
#pragma unroll
                            for (int q = 0; q < 4; ++q)
                                w4[q] = __builtin_amdgcn_bitop3_b32(
                                    __builtin_amdgcn_bitop3_b32(P[q], T0[q], T1[q], 0x96), T2[q], T3[q], 0x96);
                            const bool p0 = fail4(w4[0], w4[1], w4[2], w4[3]) == 0u;
                            const uint64_t bp = __builtin_amdgcn_ballot_w64(p0);
                            if (p0)
                                lds_W[cnt + __builtin_amdgcn_mbcnt_hi((uint32_t)(bp >> 32),
                                                                      __builtin_amdgcn_mbcnt_lo((uint32_t)bp, 0u))] =
                                    (r12 << 6) | (uint32_t)lane;
                            cnt += (uint32_t)__builtin_popcountll(bp);
                        }
                        if (cnt >= (uint32_t)LIST_FLUSH || rd != 0 || seg_end) {
                            bk.n_cand += cnt;
                            // ---- check: lane j takes entry base + j; the
                            // owner's P words arrive by ds_bpermute
                            for (uint32_t base = 0; base < cnt; base += 64) {
                                ++bk.n_pass;
                                const uint32_t ent = base + (uint32_t)lane < cnt ? lds_W[base + lane] : 0u;
                                const uint32_t own = ent & 63u, r12 = ent >> 6;
                                const int src = (int)(own << 2);
                                const uint32_t g12 = (r12 ^ (r12 >> 1)) ^ par;
                                const uint32_t *T0 = lds_L + (g12 & 7u) * RS;
                                const uint32_t *T1 = lds_L + (8u + ((g12 >> 3) & 7u)) * RS;
                                const uint32_t *T2 = lds_L + (16u + ((g12 >> 6) & 7u)) * RS;
                                const uint32_t *T3 = lds_L + (24u + (g12 >> 9)) * RS;
                                // word of the listed state: owner's P ^ T0 ^ T1 ^ T2 ^ T3
                                auto word = [&](int pi, int off) {
                                    const uint32_t pw = (uint32_t)__builtin_amdgcn_ds_bpermute(src, (int)P[pi]);
                                    return __builtin_amdgcn_bitop3_b32(
                                        __builtin_amdgcn_bitop3_b32(pw, T0[off], T1[off], 0x96), T2[off], T3[off], 0x96);
                                };
                                // group 0 passed in phase 1; the other groups in
                                // decreasing rejection order, stopping once no
                                // entry passes.  Entries of lanes beyond the
                                // item's last chunk are dropped.
                                const wpm_item ci = iv();
                                bool pass = base + (uint32_t)lane < cnt &&
                                            wbase + (int)own < (int)__builtin_amdgcn_readfirstlane((uint32_t)ci.lanes);
                                const int Gp = (int)hv(D_G), Qp = (QS == 4) ? 4 : (int)hv(D_QS);
                                bool go = true;
#pragma unroll
                                for (int g = 1; g < GM; ++g) {
                                    go = go && g < Gp && __builtin_amdgcn_ballot_w64(pass) != 0;
                                    if (go) {
                                        uint32_t stw[QS];
#pragma unroll
                                        for (int q = 0; q < QS; ++q)
                                            stw[q] = (QS == 4 || q < Qp)
                                                         ? word(4 + (g - 1) * QS + q, 4 + (g - 1) * Qp + q)
                                                         : 0u;
                                        pass = pass && fail_slots<QS>(stw) == 0u;
                                    }
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
                                    const int Wp = (int)hv(D_W), ko = 4 + (Gp - 1) * Qp;
                                    // one word at a time: issuing every word's
                                    // reads at once would need 5 * WM VGPRs
                                    uint32_t cntf = 0;
#pragma unroll
                                    for (int w = 0; w < WM; ++w) {
                                        if (w < Wp) cntf += __builtin_popcount(word(KR + w, ko + w));
                                        asm volatile("" : "+v"(cntf)::"memory");
                                    }
                                    const uint32_t mf = hv(D_MAXF);
                                    bool ok = pass && (mf == 0u || cntf <= mf);
                                    // further affine properties g(K) = c0 + sum_c w_c |K & mask_c| > 0
                                    const uint32_t np = hv(D_NPROPS);
                                    if (np != 0u && __builtin_amdgcn_ballot_w64(ok) != 0) {
                                        const uint32_t *pr = tab + hv(D_PROPS);
                                        for (uint32_t q = 0; q < np; ++q) {
                                            int64_t gv = (int32_t)pr[0];
                                            const uint32_t ncls = pr[1];
                                            pr += 2;
                                            for (uint32_t cl = 0; cl < ncls; ++cl) {
                                                uint32_t sum = 0;
#pragma unroll
                                                for (int w = 0; w < WM; ++w) {
                                                    if (w < Wp) sum += __builtin_popcount(word(KR + w, ko + w) & pr[1 + w]);
                                                    asm volatile("" : "+v"(sum)::"memory");
                                                }
                                                gv += (int64_t)(int32_t)pr[0] * (int64_t)sum;
                                                pr += 1 + Wp;
                                            }
                                            ok = ok && gv > 0;
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
                                            for (uint64_t e0 = out_pos + (uint64_t)lane; e0 < out_end && e0 < a.cap;
                                                 e0 += 64) {
                                                a.surv[2 * e0] = 0;
                                                a.surv[2 * e0 + 1] = ~0ull;
                                            }
                                            const uint64_t want = a.chunk > nbal ? a.chunk : nbal;
                                            unsigned long long rbase = 0;
                                            if (lane == 0) rbase = atomicAdd(a.slots, (unsigned long long)want);
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
                    s0 = lds_S[tid];
                    s1 = lds_S[bd + tid];
                    s2 = lds_S[2 * bd + tid];
                    s3 = lds_S[3 * bd + tid];
                }
                // ---- block boundary: one more Gray step, flipping t >= 6;
                // P follows only the flips of t >= 12 (segment changes)
                if (blk + 1 < nblk) {
                    const int t = 6 + __builtin_ctzll(blk + 1);
                    const uint32_t *row = lds_R + t * RS;
                    if (t >= 12) {
                        // opaque copy: keeps the per-group tests from being
                        // hoisted out of the block loop as live lane masks
                        const int Gb = (int)hv(D_G), Wb = (int)hv(D_W), Qb = (QS == 4) ? 4 : (int)hv(D_QS);
                        xor_row<GM, QS, WM>(P, row, ~0u, Gb, Wb, Qb);
                    }
                    s0 ^= row[0];
                    s1 ^= row[1];
                    s2 ^= row[2];
                    s3 ^= row[3];
                }
            }
        }
        const uint32_t item_cnt = bk.item_cnt;
        if (item_cnt && lane == 0) atomicAdd(a.counts + inst, (unsigned long long)item_cnt);
        bk.wave_total += item_cnt;
        __syncthreads();
        if (tid == 0 && a.times) {
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
    if (lane == 0 && wave_total) atomicAdd(a.total, (unsigned long long)wave_total);
    if (a.stats && lane == 0 && (n_cand | n_ridge | n_ubt | n_pass | n_redo)) {
        atomicAdd(a.stats + 0, (unsigned long long)n_cand);
        atomicAdd(a.stats + 1, (unsigned long long)n_ridge);
        atomicAdd(a.stats + 2, (unsigned long long)n_ubt);
        atomicAdd(a.stats + 3, (unsigned long long)n_pass);
        atomicAdd(a.stats + 4, (unsigned long long)n_redo);
    }
}

}  // namespace wpm
