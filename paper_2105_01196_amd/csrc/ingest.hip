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

// Sets *flag when any of the n values is NaN or infinite.
__global__ void __launch_bounds__(256) check_finite_kernel(const float *__restrict__ x, size_t n,
                                                           int *flag) {
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    int bad = 0;
    for (; i < n; i += stride) bad |= !isfinite(x[i]);
    if (__ballot(bad) != 0 && (threadIdx.x % kWave) == 0) atomicOr(flag, 1);
}

// One workgroup per row: stage the row in LDS, then each thread ranks its
// columns by counting the cells with a smaller value. Padding rows
// (r >= rows) get rank 0; the evaluators mask them out.
__global__ void __launch_bounds__(256) rank_rows_kernel(const float *__restrict__ x, int32_t rows,
                                                        int32_t cols, int32_t rows_pad,
                                                        uint16_t *__restrict__ ranks) {
    extern __shared__ float s_row[];
    const int32_t r = blockIdx.x;
    if (r >= rows) {
        for (int32_t c = threadIdx.x; c < cols; c += blockDim.x)
            ranks[(size_t)c * rows_pad + r] = 0;
        return;
    }
    const float *xr = x + (size_t)r * cols;
    for (int32_t c = threadIdx.x; c < cols; c += blockDim.x) s_row[c] = xr[c];
    __syncthreads();
    for (int32_t c = threadIdx.x; c < cols; c += blockDim.x) {
        const float v = s_row[c];
        int32_t rank = 0;
        for (int32_t d = 0; d < cols; d++) rank += s_row[d] < v;
        ranks[(size_t)c * rows_pad + r] = (uint16_t)rank;
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
    rank_rows_kernel<<<rows_pad, 256, (size_t)cols * sizeof(float), stream>>>(x, rows, cols,
                                                                             rows_pad, ranks);
    EBIC_HIP(hipGetLastError());
    return EBIC_OK;
}

}  // namespace ebic
