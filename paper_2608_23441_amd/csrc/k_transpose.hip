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

// 16-byte stores over the aligned body, single bytes over the ends
__global__ __launch_bounds__(256) void k_zero(unsigned char* __restrict__ p, size_t head, size_t nvec,
                                              size_t bytes) {
  const size_t stride = (size_t)gridDim.x * 256;
  const size_t i0 = (size_t)blockIdx.x * 256 + threadIdx.x;
  uint4* v = reinterpret_cast<uint4*>(p + head);
  for (size_t i = i0; i < nvec; i += stride) v[i] = make_uint4(0u, 0u, 0u, 0u);
  const size_t tail0 = head + nvec * 16;
  for (size_t i = i0; i < head; i += stride) p[i] = 0;
  for (size_t i = tail0 + i0; i < bytes; i += stride) p[i] = 0;
}

hipError_t launch_zero(void* p, size_t bytes, hipStream_t st) {
  if (bytes == 0) return hipSuccess;
  unsigned char* c = (unsigned char*)p;
  size_t head = (16 - ((uintptr_t)c & 15)) & 15;
  if (head > bytes) head = bytes;
  const size_t nvec = (bytes - head) / 16;
  size_t blocks = (nvec + 255) / 256;
  if (blocks < 1) blocks = 1;
  if (blocks > 4096) blocks = 4096;
  k_zero<<<dim3((unsigned)blocks), 256, 0, st>>>(c, head, nvec, bytes);
  return hipGetLastError();
}

}  // namespace ipfb
