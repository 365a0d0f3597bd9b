// Pair-comparison table: for every unordered column pair lo < hi, the bitmap
// over rows of "lo precedes hi in this row" (smaller value first; a tie puts
// the smaller column index first). The strict table holds "lo's value is
// strictly smaller" instead, for the strict and loose tie rules. A step c_j -> c_{j+1} of a
// series keeps the increasing trend in exactly the rows of pair
// (min, max)'s bitmap, inverted when c_j > c_{j+1}, because the row order is
// strict and total. With the table resident, testing a step costs one bit
// per row instead of two 16-bit ranks and a compare.
//
// Layout: uint64 words, pair-major: word w of pair p covers rows 64w..64w+63
// at table[p * S + w] (p = pair_index(lo, hi, C)), with S the row words
// rounded up to 16 so that each pair starts on a 128-byte line and the
// 128-byte stores below fill whole lines; padding rows read 0.
#include "device.h"
#include "internal.h"

namespace ebic {
namespace {

constexpr int kBuildWaves = 4;
constexpr int kAGroup = 4;   // columns a per wave
constexpr int kSpan = 16;    // 64-row blocks per wave (16 words = one 128-byte line per pair)
constexpr int kBChunk = 32;  // columns b per wave

// One wave: columns a0..a0+3 against the b > a0 of one chunk of 32 columns,
// over 16 blocks of 64 rows (waves whose chunk lies wholly at or below a0
// have nothing to do). lane = row within a block; a ballot of the 64 rank
// compares is the table word for (pair, block). The words are gathered
// into lanes (q * 16 + block) so that each pair's 16 words go out as one
// 128-byte store.
template <bool STRICT>
__global__ void __launch_bounds__(kBuildWaves * kWave)
    build_pairs_kernel(const uint16_t *__restrict__ ranks, int32_t rows, int32_t cols,
                       int32_t rows_pad, uint64_t *__restrict__ table, int32_t stride,
                       int32_t ngroups, int32_t nspans, int32_t nchunks) {
    const int64_t wave_id = (int64_t)blockIdx.x * kBuildWaves + threadIdx.x / kWave;
    if (wave_id >= (int64_t)ngroups * nspans * nchunks) return;
    const int lane = threadIdx.x % kWave;
    // the row span varies fastest, so waves running together write
    // neighbouring lines of the same pairs rather than one line of many
    const int span = (int)(wave_id % nspans);
    const int64_t rest = wave_id / nspans;
    const int chunk = (int)(rest % nchunks), g = (int)(rest / nchunks);
    const int a0 = g * kAGroup;
    const int b_beg = max(a0 + 1, chunk * kBChunk), b_end = min(cols, (chunk + 1) * kBChunk);
    if (b_beg >= b_end) return;
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
    // column b's ranks, the next column's loads issued before this one's compares
    int rb[kSpan], rn[kSpan];
#pragma unroll
    for (int b = 0; b < kSpan; b++)
        rn[b] = (blk0 + b < w64)
                    ? load_rank(rs, ((blk0 + b) * 64 + lane) * 2, (int)((uint32_t)b_beg * col_bytes))
                    : 0;
    for (int bcol = b_beg; bcol < b_end; bcol++) {
#pragma unroll
        for (int b = 0; b < kSpan; b++) rb[b] = rn[b];
        if (bcol + 1 < b_end) {
#pragma unroll
            for (int b = 0; b < kSpan; b++)
                rn[b] = (blk0 + b < w64) ? load_rank(rs, ((blk0 + b) * 64 + lane) * 2,
                                                     (int)((uint32_t)(bcol + 1) * col_bytes))
                                         : 0;
        }
        int lo = 0, hi = 0;
#pragma unroll
        for (int q = 0; q < kAGroup; q++) {
            if (a0 + q >= bcol) continue;
#pragma unroll
            for (int b = 0; b < kSpan; b++) {
                // a < b: a tie puts a first (none in the strict table);
                // padding rows (rank 0 everywhere) read 0
                const bool before = STRICT ? ra[q][b] < rb[b] : ra[q][b] <= rb[b];
                const uint64_t m = __ballot((blk0 + b) * 64 + lane < rows && before);
                lo = writelane((int)(uint32_t)m, q * kSpan + b, lo);
                hi = writelane((int)(uint32_t)(m >> 32), q * kSpan + b, hi);
            }
        }
        if (a0 + my_q < bcol && blk0 + my_b < w64) {
            const int64_t p = pair_index(a0 + my_q, bcol, cols);
            table[p * stride + blk0 + my_b] = ((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo;
        }
    }
}

}  // namespace

int launch_build_pairs(const uint16_t *ranks, int32_t rows, int32_t cols, int32_t rows_pad,
                       uint64_t *table, bool strict, hipStream_t stream) {
    const int32_t ngroups = (cols + kAGroup - 1) / kAGroup;
    const int32_t nspans = (rows_pad / 64 + kSpan - 1) / kSpan;
    const int32_t nchunks = (cols + kBChunk - 1) / kBChunk;
    const int64_t waves = (int64_t)ngroups * nspans * nchunks;
    const int64_t blocks = (waves + kBuildWaves - 1) / kBuildWaves;
    if (blocks > INT32_MAX) return fail(EBIC_ERR_INVALID_ARG, "pair table too large");
    auto *kernel = strict ? build_pairs_kernel<true> : build_pairs_kernel<false>;
    kernel<<<(int)blocks, kBuildWaves * kWave, 0, stream>>>(
        ranks, rows, cols, rows_pad, table, pair_words(rows_pad), ngroups, nspans, nchunks);
    EBIC_HIP(hipGetLastError());
    return EBIC_OK;
}

}  // namespace ebic
