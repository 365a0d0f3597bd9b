// Pair-comparison table: for every unordered column pair lo < hi, the bitmap
// over rows of "lo precedes hi in this row" (smaller value first; a tie puts
// the smaller column index first). A step c_j -> c_{j+1} of a
// series keeps the increasing trend in exactly the rows of pair
// (min, max)'s bitmap, inverted when c_j > c_{j+1}, because the row order is
// strict and total. With the table resident, testing a step costs one bit
// per row instead of two 16-bit ranks and a compare.
//
// Layout: uint64 words, pair-major: word w of pair p covers rows 64w..64w+63
// at table[p * W64 + w] (p = pair_index(lo, hi, C)); padding rows read 0.
#include "device.h"
#include "internal.h"

namespace ebic {
namespace {

constexpr int kBuildWaves = 4;
constexpr int kAGroup = 4;   // columns a per wave
constexpr int kSpan = 16;    // 64-row blocks per wave (16 words = one 128-byte line per pair)

// One wave: columns a0..a0+3 against every b > a0, over 16 blocks of 64
// rows. lane = row within a block; a ballot of the 64 rank compares is the
// table word for (pair, block). The words are gathered into lanes
// (q * 16 + block) so that each pair's 16 words go out as one 128-byte store.
__global__ void __launch_bounds__(kBuildWaves * kWave)
    build_pairs_kernel(const uint16_t *__restrict__ ranks, int32_t rows, int32_t cols,
                       int32_t rows_pad, uint64_t *__restrict__ table, int32_t ngroups,
                       int32_t nspans) {
    const int wave_id = blockIdx.x * kBuildWaves + threadIdx.x / kWave;
    if (wave_id >= ngroups * nspans) return;
    const int lane = threadIdx.x % kWave;
    const int span = wave_id / ngroups, g = wave_id % ngroups;
    const int a0 = g * kAGroup;
    const int w64 = rows_pad / 64;
    const int blk0 = span * kSpan;
    const __amdgpu_buffer_rsrc_t rs = make_rsrc(ranks, (uint32_t)((size_t)cols * rows_pad * 2));
    const uint32_t col_bytes = (uint32_t)rows_pad * 2u;

    int ra[kAGroup][kSpan];
#pragma unroll
    for (int q = 0; q < kAGroup; q++)
#pragma unroll
        for (int b = 0; b < kSpan; b++)
            ra[q][b] = (a0 + q < cols && blk0 + b < w64)
                           ? load_rank(rs, ((blk0 + b) * 64 + lane) * 2,
                                       (int)((uint32_t)(a0 + q) * col_bytes))
                           : 0;

    const int my_q = lane / kSpan, my_b = lane % kSpan;
    for (int bcol = a0 + 1; bcol < cols; bcol++) {
        int rb[kSpan];
#pragma unroll
        for (int b = 0; b < kSpan; b++)
            rb[b] = (blk0 + b < w64) ? load_rank(rs, ((blk0 + b) * 64 + lane) * 2,
                                                 (int)((uint32_t)bcol * col_bytes))
                                     : 0;
        int lo = 0, hi = 0;
#pragma unroll
        for (int q = 0; q < kAGroup; q++) {
            if (a0 + q >= bcol) continue;
#pragma unroll
            for (int b = 0; b < kSpan; b++) {
                // a < b: a tie puts a first; padding rows (rank 0 everywhere) read 0
                const uint64_t m =
                    __ballot((blk0 + b) * 64 + lane < rows && ra[q][b] <= rb[b]);
                lo = writelane((int)(uint32_t)m, q * kSpan + b, lo);
                hi = writelane((int)(uint32_t)(m >> 32), q * kSpan + b, hi);
            }
        }
        if (a0 + my_q < bcol && blk0 + my_b < w64) {
            const int64_t p = pair_index(a0 + my_q, bcol, cols);
            table[p * w64 + blk0 + my_b] = ((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo;
        }
    }
}

}  // namespace

int launch_build_pairs(const uint16_t *ranks, int32_t rows, int32_t cols, int32_t rows_pad,
                       uint64_t *table, hipStream_t stream) {
    const int32_t ngroups = (cols + kAGroup - 1) / kAGroup;
    const int32_t nspans = (rows_pad / 64 + kSpan - 1) / kSpan;
    const int64_t waves = (int64_t)ngroups * nspans;
    const int64_t blocks = (waves + kBuildWaves - 1) / kBuildWaves;
    if (blocks > INT32_MAX) return fail(EBIC_ERR_INVALID_ARG, "pair table too large");
    build_pairs_kernel<<<(int)blocks, kBuildWaves * kWave, 0, stream>>>(
        ranks, rows, cols, rows_pad, table, ngroups, nspans);
    EBIC_HIP(hipGetLastError());
    return EBIC_OK;
}

}  // namespace ebic
