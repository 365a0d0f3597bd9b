// Matrix ingest: finiteness check and per-row ranks.
//
// The trend test only ever compares two cells of a row: smaller, equal or
// larger. Replacing every cell by the number of cells of its row with a
// smaller value (equal values share it) keeps every such answer and turns
// the test into one 16-bit integer compare; how a tie counts (by column
// index, against both trends or for both) is the evaluator's choice. The ranks are stored
// column-major (cols x rows_pad), so a wavefront reading one column for 64
// consecutive rows touches 128 contiguous bytes. The paper keeps the matrix
// resident on the GPU and only ships populations per generation (Sec. 2.4,
// step 2); this is the one-time preparation of that resident copy.
#include "internal.h"

namespace ebic {
namespace {

constexpr int32_t kXcds = 8;  // accelerator complex dies, each with its own L2

// Sets *flag when any of the n values is NaN or infinite.
__global__ void __launch_bounds__(256) check_finite_kernel(const float *__restrict__ x, size_t n,
                                                           int *flag) {
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    int bad = 0;
    for (; i < n; i += stride) bad |= !isfinite(x[i]);
    if (__ballot(bad) != 0 && (threadIdx.x % kWave) == 0) atomicOr(flag, 1);
}

// Order-preserving integer key of a finite float: -0 becomes +0, then
// non-negative values get the sign bit set and negative ones have every
// bit flipped, so unsigned key order is the IEEE order of the values,
// denormals included, whatever the device's denormal mode (integer
// compares never flush).
__device__ inline uint32_t order_key(float v) {
    uint32_t b = __float_as_uint(v);
    if ((b << 1) == 0u) b = 0u;  // -0 == +0
    return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}

// One workgroup per row. The row's keys go to LDS, padded to a power of two
// with the largest key (above every finite value's), and are sorted there
// (bitonic network: every stage compares n/2 disjoint pairs, one per
// thread step, then a barrier); a cell's rank, the number of cells with a
// smaller value, is then the lower bound of its key in the sorted row
// (binary search). Equal values, and -0 and +0, get the same rank. Padding
// rows (r >= rows) get rank 0; the evaluators mask them out. Non-finite
// input is rejected by the caller after the flag check, so its ranks are
// never used.
__global__ void __launch_bounds__(256) rank_rows_kernel(const float *__restrict__ x, int32_t rows,
                                                        int32_t cols, int32_t rows_pad, int32_t n,
                                                        uint16_t *__restrict__ ranks) {
    extern __shared__ uint32_t s_sorted[];
    // Workgroups are dealt to the 8 XCDs in turn and each XCD has its own
    // L2: give XCD x the contiguous rows x * rows_pad/8 .. so that the 2-byte
    // ranks of neighbouring rows merge into whole lines in one L2 before
    // they are written back (rows_pad is a multiple of 64).
    const int32_t per_xcd = rows_pad / kXcds;
    const int32_t r = (int32_t)(blockIdx.x % kXcds) * per_xcd + (int32_t)(blockIdx.x / kXcds);
    if (r >= rows) {
        for (int32_t c = threadIdx.x; c < cols; c += blockDim.x)
            ranks[(size_t)c * rows_pad + r] = 0;
        return;
    }
    const float *xr = x + (size_t)r * cols;
    for (int32_t c = threadIdx.x; c < n; c += blockDim.x)
        s_sorted[c] = c < cols ? order_key(xr[c]) : 0xFFFFFFFFu;
    __syncthreads();
    for (int32_t k = 2; k <= n; k <<= 1) {
        for (int32_t lj = __builtin_ctz((uint32_t)k) - 1; lj >= 0; lj--) {
            const int32_t j = 1 << lj;
            for (int32_t q = threadIdx.x; q < n / 2; q += blockDim.x) {
                // lower index of the pair: q with a zero bit inserted at bit lj
                const int32_t i = ((q >> lj) << (lj + 1)) | (q & (j - 1));
                const uint32_t a = s_sorted[i], b = s_sorted[i + j];
                const bool up = (i & k) == 0;  // this run ascends
                if ((b < a) == up) {
                    s_sorted[i] = b;
                    s_sorted[i + j] = a;
                }
            }
            __syncthreads();
        }
    }
    for (int32_t c = threadIdx.x; c < cols; c += blockDim.x) {
        const uint32_t v = order_key(xr[c]);
        int32_t lo = 0, hi = n;  // first index whose key is not below v
        while (lo < hi) {
            const int32_t mid = (lo + hi) >> 1;
            if (s_sorted[mid] < v)
                lo = mid + 1;
            else
                hi = mid;
        }
        ranks[(size_t)c * rows_pad + r] = (uint16_t)lo;
    }
}

__global__ void zero_flag_kernel(int *flag) { *flag = 0; }

}  // namespace

int launch_prepare(const float *x, int32_t rows, int32_t cols, uint16_t *ranks, int *flag,
                   hipStream_t stream) {
    const size_t n = (size_t)rows * cols;
    zero_flag_kernel<<<1, 1, 0, stream>>>(flag);
    int blocks = (int)((n + 255) / 256);
    if (blocks > 4096) blocks = 4096;
    check_finite_kernel<<<blocks, 256, 0, stream>>>(x, n, flag);
    const int32_t rows_pad = rows_padded(rows);
    int32_t width = 2;  // the row padded to a power of two
    while (width < cols) width <<= 1;  // at most EBIC_MAX_COLS = 16,384: 64 KB of LDS
    rank_rows_kernel<<<rows_pad, 256, (size_t)width * sizeof(uint32_t), stream>>>(
        x, rows, cols, rows_pad, width, ranks);
    EBIC_HIP(hipGetLastError());
    return EBIC_OK;
}

}  // namespace ebic
