// Device helpers shared by the evaluation kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "ebic.h"

namespace ebic {

__device__ inline int tol(int k, int approx) {
    return (int)(((long long)(k - 1) * (1000 - approx)) / 1000);
}

// Buffer resource over `bytes` bytes at `p`: loads through it take the
// per-lane offset in a VGPR and a wave-uniform offset in an SGPR, and the
// hardware returns 0 for any offset past the end.
// A pointer into device (global) memory, typed as such: loads and stores
// through it compile to global_* instructions. Generic pointers compile to
// flat_* ones, which also count against the LDS/scalar wait counter, so an
// LDS read issued after them waits for the memory load too.
template <class T>
__device__ inline const __attribute__((address_space(1))) T *gmem(const T *p) {
    return (const __attribute__((address_space(1))) T *)p;
}
template <class T>
__device__ inline __attribute__((address_space(1))) T *gmem(T *p) {
    return (__attribute__((address_space(1))) T *)p;
}

__device__ inline __amdgpu_buffer_rsrc_t make_rsrc(const void *p, uint32_t bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(p), (short)0, (int)bytes,
                                             0x00020000);
}

__device__ inline int load_rank(__amdgpu_buffer_rsrc_t rs, int lane_off, int col_off) {
    return __builtin_amdgcn_raw_buffer_load_b16(rs, lane_off, col_off, 0);
}

// Support word of 64 rows (lane = row) for a series whose columns' byte
// offsets into the rank matrix sit in s_off[0..k). A step a -> b fits the
// increasing trend when rank[a] < rank[b] + fu and the decreasing one when
// rank[b] < rank[a] + fd, with, by tie rule: column index fu = [a < b],
// fd = [a > b] (then exactly one of the two holds); strict fu = fd = 0;
// loose fu = fd = 1. A column's byte offset c * rows_pad * 2 stays below 2^32
// (cols * rows_pad < 2^31), so compared as unsigned it keeps column order:
// a < b is off_a < off_b.
// A row fits when at most t steps break the increasing trend, or (neg) at
// most t break the decreasing one. The wave stops once every row is out.
template <int RULE>
__device__ inline uint64_t block_support_rule(__amdgpu_buffer_rsrc_t rs, const int32_t *s_off,
                                              int k, int t, int neg, int lane_off,
                                              bool valid_row) {
    int off_prev = __builtin_amdgcn_readfirstlane(s_off[0]);
    int prev = load_rank(rs, lane_off, off_prev);
    int inc_bad = 0, dec_bad = 0;  // steps against each trend
    auto step = [&](int off, int cur) {
        const uint32_t ua = (uint32_t)off_prev, ub = (uint32_t)off;
        const int fu = RULE == EBIC_TIE_INDEX ? (ua < ub) : (RULE == EBIC_TIE_LOOSE);
        const int fd = RULE == EBIC_TIE_INDEX ? (ua > ub) : (RULE == EBIC_TIE_LOOSE);
        inc_bad += !(prev < cur + fu);
        if (RULE != EBIC_TIE_INDEX) dec_bad += !(cur < prev + fd);
        prev = cur;
        off_prev = off;
    };
    int j = 1;
    for (; j + 3 < k; j += 4) {
        int off[4], r[4];
#pragma unroll
        for (int q = 0; q < 4; q++) {
            off[q] = __builtin_amdgcn_readfirstlane(s_off[j + q]);
            r[q] = load_rank(rs, lane_off, off[q]);
        }
#pragma unroll
        for (int q = 0; q < 4; q++) step(off[q], r[q]);
        const int done = j + 3;  // steps examined so far
        // with the column-index rule every step breaks exactly one trend
        const int dbad = RULE == EBIC_TIE_INDEX ? done - inc_bad : dec_bad;
        const bool dead = !valid_row || (inc_bad > t && (!neg || dbad > t));
        if (__ballot(!dead) == 0) return 0;
    }
    for (; j < k; j++) {
        const int off = __builtin_amdgcn_readfirstlane(s_off[j]);
        step(off, load_rank(rs, lane_off, off));
    }
    const int dbad = RULE == EBIC_TIE_INDEX ? (k - 1) - inc_bad : dec_bad;
    const bool fit = valid_row && (inc_bad <= t || (neg && dbad <= t));
    return __ballot(fit);
}

__device__ inline uint64_t block_support(__amdgpu_buffer_rsrc_t rs, const int32_t *s_off, int k,
                                         int t, int neg, int rule, int lane_off, bool valid_row) {
    switch (rule) {
        case EBIC_TIE_STRICT:
            return block_support_rule<EBIC_TIE_STRICT>(rs, s_off, k, t, neg, lane_off, valid_row);
        case EBIC_TIE_LOOSE:
            return block_support_rule<EBIC_TIE_LOOSE>(rs, s_off, k, t, neg, lane_off, valid_row);
        default:
            return block_support_rule<EBIC_TIE_INDEX>(rs, s_off, k, t, neg, lane_off, valid_row);
    }
}

// v_writelane_b32: returns `old` with lane `lane` set to the wave-uniform
// `val` (ignores the exec mask); same argument order as the compiler builtin
// of later releases. With an SGPR value the lane select must come from M0 on
// this architecture.
__device__ inline int writelane(int val, int lane, int old) {
    // readfirstlane makes both operands SGPRs (the values are wave-uniform)
    const int v = __builtin_amdgcn_readfirstlane(val);
    const int l = __builtin_amdgcn_readfirstlane(lane);
    asm volatile("s_mov_b32 m0, %2\n\tv_writelane_b32 %0, %1, m0" : "+v"(old) : "s"(v), "s"(l));
    return old;
}

// Sum over the 64 lanes (all lanes must be active): DPP butterflies within
// each 16-lane row (quad xor 1, quad xor 2, half-row mirror, row mirror),
// then the four row sums read out with readlane. Wave-uniform result.
__device__ inline int wave_sum(int v) {
    v += __builtin_amdgcn_update_dpp(0, v, 0xB1, 0xF, 0xF, false);   // quad_perm 1,0,3,2
    v += __builtin_amdgcn_update_dpp(0, v, 0x4E, 0xF, 0xF, false);   // quad_perm 2,3,0,1
    v += __builtin_amdgcn_update_dpp(0, v, 0x141, 0xF, 0xF, false);  // row_half_mirror
    v += __builtin_amdgcn_update_dpp(0, v, 0x140, 0xF, 0xF, false);  // row_mirror
    return __builtin_amdgcn_readlane(v, 0) + __builtin_amdgcn_readlane(v, 16) +
           __builtin_amdgcn_readlane(v, 32) + __builtin_amdgcn_readlane(v, 48);
}

// Index of the unordered column pair (lo < hi) among the C(C-1)/2 pairs in
// lexicographic order.
__host__ __device__ inline int64_t pair_index(int64_t lo, int64_t hi, int64_t C) {
    return lo * C - lo * (lo + 1) / 2 + (hi - lo - 1);
}

}  // namespace ebic
