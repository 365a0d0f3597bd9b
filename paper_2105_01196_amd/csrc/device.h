// Device helpers shared by the evaluation kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

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

// Gather form of the trend test for one 64-row block: lane = row, s_off
// holds each series column's byte offset in the column-major rank matrix,
// lane_off this lane's row offset. Returns the block's support word. Exits
// early once every row of the block has broken both trends beyond the
// tolerance t.
__device__ inline uint64_t block_support(__amdgpu_buffer_rsrc_t rs, const int32_t *s_off, int k,
                                         int t, int neg, int lane_off, bool valid_row) {
    int prev = load_rank(rs, lane_off, __builtin_amdgcn_readfirstlane(s_off[0]));
    int up = 0;
    int j = 1;
    for (; j + 3 < k; j += 4) {
        const int a = load_rank(rs, lane_off, __builtin_amdgcn_readfirstlane(s_off[j]));
        const int b = load_rank(rs, lane_off, __builtin_amdgcn_readfirstlane(s_off[j + 1]));
        const int c = load_rank(rs, lane_off, __builtin_amdgcn_readfirstlane(s_off[j + 2]));
        const int d = load_rank(rs, lane_off, __builtin_amdgcn_readfirstlane(s_off[j + 3]));
        up += (prev < a) + (a < b) + (b < c) + (c < d);
        prev = d;
        const int done = j + 3;  // steps examined so far
        const bool dead = !valid_row || ((done - up > t) && (!neg || up > t));
        if (__ballot(!dead) == 0) return 0;
    }
    for (; j < k; j++) {
        const int cur = load_rank(rs, lane_off, __builtin_amdgcn_readfirstlane(s_off[j]));
        up += prev < cur;
        prev = cur;
    }
    const bool fit = valid_row && (((k - 1 - up) <= t) || (neg && up <= t));
    return __ballot(fit);
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
