// Block x column transposes of the frame matrix (Section 2.3's [frames, N]
// array): the row stage produces frames, the column stage (Section 3.1)
// wants each sub-filter path n contiguous. A 64 x 64 tile goes through LDS so
// that both the reads and the writes are 256-byte (float) runs; strided
// 4-byte accesses would cost the full HBM transaction each.
#include "fft_lds.hpp"
#include "launch.hpp"

namespace ipfb {

template <typename T>
__global__ __launch_bounds__(256) void k_transpose(const T* __restrict__ in, T* __restrict__ out, int64_t rows,
                                                   int64_t cols, int64_t tiles_c) {
  __shared__ T t[64][65];
  const int64_t tc = blockIdx.x % tiles_c, tr = blockIdx.x / tiles_c;
  const int lx = threadIdx.x & 63, ly = threadIdx.x >> 6;
  const int64_t c = tc * 64 + lx;
#pragma unroll 4
  for (int y = ly; y < 64; y += 4) {
    const int64_t r = tr * 64 + y;
    if (r < rows && c < cols) t[y][lx] = in[r * cols + c];
  }
  __syncthreads();
  const int64_t r2 = tr * 64 + lx;
#pragma unroll 4
  for (int y = ly; y < 64; y += 4) {
    const int64_t c2 = tc * 64 + y;
    if (c2 < cols && r2 < rows) out[c2 * rows + r2] = t[lx][y];
  }
}

hipError_t launch_transpose(int prec, const void* in, void* out, int64_t rows, int64_t cols, hipStream_t st) {
  if (rows == 0 || cols == 0) return hipSuccess;
  const int64_t tr = (rows + 63) / 64, tc = (cols + 63) / 64;
  const dim3 grid((unsigned)(tr * tc));
  if (prec == F32)
    k_transpose<float><<<grid, 256, 0, st>>>((const float*)in, (float*)out, rows, cols, tc);
  else
    k_transpose<double><<<grid, 256, 0, st>>>((const double*)in, (double*)out, rows, cols, tc);
  return hipGetLastError();
}

}  // namespace ipfb
