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
// 512-byte stores below fill whole lines; padding rows read 0.
#include "device.h"
#include "internal.h"

namespace ebic {
namespace {

constexpr int kPlaneWaves = 4;
constexpr int kBuildWaves = 4;
constexpr int kBChunk = 32;  // columns b per workgroup

// Three-input bitwise operation (v_bitop3_b32); IMM is the truth table, bit
// (a << 2 | b << 1 | c) of IMM the result for input bits a, b, c.
template <int IMM>
__device__ __forceinline__ uint32_t bitop3(uint32_t a, uint32_t b, uint32_t c) {
    return __builtin_amdgcn_bitop3_b32(a, b, c, IMM);
}
// Borrow of x - y after one more bit plane: the majority of ~x_i, y_i and
// the borrow so far; after the top plane it is x < y.
constexpr int kBorrow = 0x8E;
constexpr int kNotBorrow = 0x71;

// Bit planes of the ranks, in 64-row words: planes[(c * NB + i) * W + w]
// holds bit i of column c's ranks of rows 64w..64w+63 (W = rows_pad / 64).
// One wave per column and 64 words: lane = row within a word, one ballot
// per bit plane, gathered into lane (word - first word) so that each plane's
// 64 words go out as one 512-byte store.
template <int NB>
__global__ void __launch_bounds__(kPlaneWaves * kWave)
    rank_planes_kernel(const uint16_t *__restrict__ ranks, int32_t cols, int32_t rows_pad,
                       uint64_t *__restrict__ planes, int32_t nspans) {
    const int64_t wave_id = (int64_t)blockIdx.x * kPlaneWaves + threadIdx.x / kWave;
    if (wave_id >= (int64_t)cols * nspans) return;
    const int lane = threadIdx.x % kWave;
    const int c = (int)(wave_id / nspans), w0 = (int)(wave_id % nspans) * kWave;
    const int W = rows_pad / 64;
    const __amdgpu_buffer_rsrc_t rs = make_rsrc(ranks, (uint32_t)((size_t)cols * rows_pad * 2));
    const int col_off = (int)((uint32_t)c * (uint32_t)rows_pad * 2u);
    int lo[NB], hi[NB];
#pragma unroll
    for (int i = 0; i < NB; i++) lo[i] = hi[i] = 0;
    for (int b = 0; b < kWave && w0 + b < W; b++) {
        const int r = load_rank(rs, ((w0 + b) * 64 + lane) * 2, col_off);
#pragma unroll
        for (int i = 0; i < NB; i++) {
            const uint64_t m = __ballot((r >> i) & 1);
            lo[i] = writelane((int)(uint32_t)m, b, lo[i]);
            hi[i] = writelane((int)(uint32_t)(m >> 32), b, hi[i]);
        }
    }
    if (w0 + lane < W)
#pragma unroll
        for (int i = 0; i < NB; i++)
            planes[((int64_t)c * NB + i) * W + w0 + lane] =
                ((uint64_t)(uint32_t)hi[i] << 32) | (uint32_t)lo[i];
}

// Table words from the planes. A workgroup: kBuildWaves groups of QA
// columns a (one per wave) against one chunk of 32 columns b, over a span of
// row words: lane = (column b offset, word), G = 2^lg lanes per column b, so
// that a matrix of fewer than 64 row words still fills the wave (64 / G
// columns b at a time), and each pair's G words go out as one contiguous
// store. The columns b's planes are staged in LDS once for the four waves
// (double-buffered, one barrier per step). Each word is one borrow chain
// over the bit planes, 64 rows at once: lo before hi is r_lo <= r_hi, that
// is not (r_hi < r_lo) (a tie puts the smaller column index first); the
// strict table holds r_lo < r_hi. Rows past the matrix read 0. Groups of
// columns a vary fastest across workgroups, so workgroups running together
// read the same columns b's planes.
template <int NB, int QA, bool STRICT>
__global__ void __launch_bounds__(kBuildWaves * kWave)
    build_pairs_kernel(const uint64_t *__restrict__ planes, int32_t rows, int32_t cols, int32_t W,
                       uint64_t *__restrict__ table, int32_t stride, int32_t nblocks,
                       int32_t nspans, int32_t nchunks, int32_t lg) {
    __shared__ uint64_t s_b[2][NB][kWave];
    const int blk = (int)(blockIdx.x % nblocks);
    const int64_t rest = blockIdx.x / nblocks;
    const int span = (int)(rest % nspans), chunk = (int)(rest / nspans);
    const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    const int c_beg = chunk * kBChunk, c_end = min(cols, (chunk + 1) * kBChunk);
    // the workgroup's first column a must lie below the chunk's last column b
    if (blk * kBuildWaves * QA + 1 >= c_end) return;
    const int a0 = (blk * kBuildWaves + wave) * QA;
    const int sub = lane >> lg, per = kWave >> lg;
    const int w = (span << lg) + (lane & ((1 << lg) - 1));
    const bool live = w < W;
    const int r0 = w * 64;
    const uint64_t valid = r0 + 64 <= rows ? ~0ull : (r0 >= rows ? 0ull : (1ull << (rows - r0)) - 1ull);
    uint32_t A[QA][NB][2];
#pragma unroll
    for (int q = 0; q < QA; q++)
#pragma unroll
        for (int i = 0; i < NB; i++) {
            const uint64_t x =
                live && a0 + q < cols ? planes[((int64_t)(a0 + q) * NB + i) * W + w] : 0ull;
            A[q][i][0] = (uint32_t)x;
            A[q][i][1] = (uint32_t)(x >> 32);
        }
    // columns b from the first one any wave pairs with
    const int b_first = max(c_beg, blk * kBuildWaves * QA + 1);
    // stage step t's planes (columns b_first + t*per + sub) into buffer t % 2:
    // wave v loads planes v, v + kBuildWaves, ...
    auto stage = [&](int t) {
        const int b = b_first + t * per + sub;
        const bool ok = live && b < c_end;
        for (int i = wave; i < NB; i += kBuildWaves)
            s_b[t & 1][i][lane] = ok ? planes[((int64_t)b * NB + i) * W + w] : 0ull;
    };
    const int steps = (c_end - b_first + per - 1) / per;
    stage(0);
    for (int t = 0; t < steps; t++) {
        __syncthreads();  // step t staged; every wave is done with step t - 1
        if (t + 1 < steps) stage(t + 1);
        const int b = b_first + t * per + sub;
        const bool ok = live && b < c_end;
        uint32_t B[NB][2];
#pragma unroll
        for (int i = 0; i < NB; i++) {
            const uint64_t x = s_b[t & 1][i][lane];
            B[i][0] = (uint32_t)x;
            B[i][1] = (uint32_t)(x >> 32);
        }
        const int b_last = min(c_end, b_first + (t + 1) * per) - 1;
#pragma unroll
        for (int q = 0; q < QA; q++) {
            if (a0 + q >= b_last) continue;  // no lane of this wave has a pair (uniform)
            uint32_t out[2];
#pragma unroll
            for (int h = 0; h < 2; h++) {
                uint32_t c = 0;
                if (STRICT) {
#pragma unroll
                    for (int i = 0; i < NB; i++) c = bitop3<kBorrow>(A[q][i][h], B[i][h], c);
                } else {
#pragma unroll
                    for (int i = 0; i < NB - 1; i++) c = bitop3<kBorrow>(B[i][h], A[q][i][h], c);
                    c = bitop3<kNotBorrow>(B[NB - 1][h], A[q][NB - 1][h], c);
                }
                out[h] = c;
            }
            if (ok && a0 + q < b)
                table[pair_index(a0 + q, b, cols) * stride + w] =
                    (((uint64_t)out[1] << 32) | out[0]) & valid;
        }
    }
}

// Bit planes for ranks below 2^NB, then the table.
template <int NB, int QA>
int build_with(const uint16_t *ranks, int32_t rows, int32_t cols, int32_t rows_pad,
               uint64_t *table, bool strict, hipStream_t stream) {
    const int32_t W = rows_pad / 64;
    int lg = 0;  // lanes per column b: the words, up to a whole wave
    while ((1 << lg) < W && lg < 6) lg++;
    const int32_t nspans = (W + (1 << lg) - 1) >> lg;
    const int32_t pspans = (W + kWave - 1) / kWave;
    const int32_t nblocks = (cols + QA * kBuildWaves - 1) / (QA * kBuildWaves);
    const int32_t nchunks = (cols + kBChunk - 1) / kBChunk;
    const int64_t blocks = (int64_t)nblocks * nspans * nchunks;
    if (blocks > INT32_MAX) return fail(EBIC_ERR_INVALID_ARG, "pair table too large");
    const size_t bytes = (size_t)cols * NB * W * sizeof(uint64_t);
    void *planes = nullptr;
    if (hipMallocAsync(&planes, bytes, stream) != hipSuccess) {
        (void)hipGetLastError();
        return fail(EBIC_ERR_OOM, "rank bit planes (%zu bytes)", bytes);
    }
    const int64_t pwaves = (int64_t)cols * pspans;
    rank_planes_kernel<NB><<<(int)((pwaves + kPlaneWaves - 1) / kPlaneWaves), kPlaneWaves * kWave, 0,
                             stream>>>(ranks, cols, rows_pad, static_cast<uint64_t *>(planes), pspans);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) {
        const auto *pl = static_cast<const uint64_t *>(planes);
        if (strict)
            build_pairs_kernel<NB, QA, true><<<(int)blocks, kBuildWaves * kWave, 0, stream>>>(
                pl, rows, cols, W, table, pair_words(rows_pad), nblocks, nspans, nchunks, lg);
        else
            build_pairs_kernel<NB, QA, false><<<(int)blocks, kBuildWaves * kWave, 0, stream>>>(
                pl, rows, cols, W, table, pair_words(rows_pad), nblocks, nspans, nchunks, lg);
        e = hipGetLastError();
    }
    // stream-ordered: the planes are freed once the table is written, and no
    // other stream waits
    const hipError_t ef = hipFreeAsync(planes, stream);
    EBIC_HIP(e);
    EBIC_HIP(ef);
    return EBIC_OK;
}

}  // namespace

int launch_build_pairs(const uint16_t *ranks, int32_t rows, int32_t cols, int32_t rows_pad,
                       uint64_t *table, bool strict, hipStream_t stream) {
    // ranks lie in 0 .. cols - 1: planes for the bits that can be set
    int nb = 1;
    while (nb < 16 && (1 << nb) < cols) nb++;
    // two columns a per wave (one for the widest ranks) keep the kernel
    // within 128 VGPRs
    if (nb <= 6) return build_with<6, 2>(ranks, rows, cols, rows_pad, table, strict, stream);
    if (nb <= 8) return build_with<8, 2>(ranks, rows, cols, rows_pad, table, strict, stream);
    if (nb <= 10) return build_with<10, 2>(ranks, rows, cols, rows_pad, table, strict, stream);
    if (nb <= 12) return build_with<12, 2>(ranks, rows, cols, rows_pad, table, strict, stream);
    return build_with<14, 1>(ranks, rows, cols, rows_pad, table, strict, stream);
}

}  // namespace ebic
