// Device-side error diagnostics of Appendix B: the relative power-spectrum
// error delta(f) = <|X - Xhat|^2> / <|X|^2>, measured (Monte-Carlo, from two
// timestreams) or predicted for white input from the sub-filter responses.
#include "fft_lds.hpp"
#include "launch.hpp"
#include "reduce.hpp"

namespace ipfb {

template <typename T>
__global__ __launch_bounds__(256) void k_sub(const T* __restrict__ a, const T* __restrict__ b, T* __restrict__ d,
                                             int64_t n) {
  const int64_t stride = (int64_t)gridDim.x * 256;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += stride) d[i] = a[i] - b[i];
}

hipError_t launch_sub(int prec, const void* a, const void* b, void* d, int64_t n, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  int64_t blocks = (n + 255) / 256;
  if (blocks > 8192) blocks = 8192;
  if (prec == F32)
    k_sub<float><<<dim3((unsigned)blocks), 256, 0, st>>>((const float*)a, (const float*)b, (float*)d, n);
  else
    k_sub<double><<<dim3((unsigned)blocks), 256, 0, st>>>((const double*)a, (const double*)b, (double*)d, n);
  return hipGetLastError();
}

__global__ __launch_bounds__(256) void k_ratio(const double* __restrict__ num, const double* __restrict__ den,
                                               double* __restrict__ out, int n) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i < n) out[i] = num[i] / den[i];
}

hipError_t launch_ratio(const double* num, const double* den, double* out, int n, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  k_ratio<<<dim3((unsigned)((n + 255) / 256)), 256, 0, st>>>(num, den, out, n);
  return hipGetLastError();
}

// out[k] for f = k / nfreq (cycles per frame): with
// W_n(f) = sum_r h[rN + n] e^{-2 pi i r f}, mode 0 (Wiener):
// 1 - (1/N) sum_n |W_n|^2 / (|W_n|^2 + phi^2); mode 1 (naive):
// (inv_snr / N) sum_n 1 / |W_n|^2. One workgroup per frequency; each thread
// sums its columns in order, then a fixed-order sum over the workgroup.
__global__ __launch_bounds__(256) void k_delta_analytic(const double* __restrict__ win, int N, int ntap,
                                                        int64_t nfreq, double phi2, int mode, double inv_snr,
                                                        double* __restrict__ out) {
  __shared__ double red[256];
  const int64_t k = blockIdx.x;
  // e^{-2 pi i k / nfreq} with k reduced so the angle stays in [-pi, pi]
  const int64_t kr = (2 * k > nfreq) ? k - nfreq : k;
  double sn, cs;
  sincos(-2.0 * 3.14159265358979323846 * (double)kr / (double)nfreq, &sn, &cs);
  double acc = 0.0;
  for (int n = threadIdx.x; n < N; n += 256) {
    double wr = 0.0, wi = 0.0, zr = 1.0, zi = 0.0;
    for (int r = 0; r < ntap; ++r) {
      const double h = win[(int64_t)r * N + n];
      wr += h * zr;
      wi += h * zi;
      const double t = zr * cs - zi * sn;
      zi = zr * sn + zi * cs;
      zr = t;
    }
    const double a2 = wr * wr + wi * wi;
    acc += (mode == 0) ? a2 / (a2 + phi2) : 1.0 / a2;
  }
  const double tot = block_sum<256>(acc, red);
  if (threadIdx.x == 0) {
    const double mean = tot / (double)N;
    out[k] = (mode == 0) ? 1.0 - mean : inv_snr * mean;
  }
}

hipError_t launch_delta_analytic(const double* win64, int N, int ntap, int64_t nfreq, double phi, double snr,
                                 double* out, hipStream_t st) {
  if (nfreq <= 0) return hipSuccess;
  const int mode = phi > 0.0 ? 0 : 1;
  k_delta_analytic<<<dim3((unsigned)nfreq), 256, 0, st>>>(win64, N, ntap, nfreq, phi * phi, mode,
                                                          mode ? 1.0 / snr : 0.0, out);
  return hipGetLastError();
}

// Bitmasks are built a wavefront at a time: lane l of the wavefront that
// starts at sample e0 (a multiple of 64) decides sample e0 + l, the ballot
// gathers the 64 decisions, and lanes 0 and 32 store the two 32-bit words
// (bits past the last sample are 0).
__device__ __forceinline__ void store_ballot(bool bit, int64_t e0, int64_t nwords, uint32_t* __restrict__ bits) {
  const unsigned long long m = __ballot(bit);
  const int lane = threadIdx.x & 63;
  const int64_t w = (e0 >> 5) + (lane >> 5);
  if ((lane & 31) == 0 && w < nwords) bits[w] = (uint32_t)(lane ? (m >> 32) : m);
}

// bit e = j N + n set for j = 0 mod R and n0 <= n < n1
__global__ __launch_bounds__(256) void k_mask_structured(uint32_t* __restrict__ bits, int N, int64_t S, int R, int n0,
                                                         int n1) {
  const int64_t nwords = (S + 31) / 32;
  const int64_t span = (int64_t)gridDim.x * 256;
  for (int64_t base = (int64_t)blockIdx.x * 256; base < S; base += span) {  // uniform per workgroup
    const int64_t i = base + threadIdx.x;
    bool bit = false;
    if (i < S) {
      const int64_t j = i / N;
      const int n = (int)(i - j * N);
      bit = j % R == 0 && n >= n0 && n < n1;
    }
    store_ballot(bit, base + (threadIdx.x & ~63), nwords, bits);
  }
}

hipError_t launch_mask_structured(uint32_t* bits, int N, int64_t nblock, int R, int L, hipStream_t st) {
  const int64_t S = (int64_t)N * nblock;
  if (S <= 0) return hipSuccess;
  int64_t blocks = (S + 255) / 256;
  if (blocks > 8192) blocks = 8192;
  const int n0 = N / 2 - L / 2;
  k_mask_structured<<<dim3((unsigned)blocks), 256, 0, st>>>(bits, N, S, R, n0, n0 + L);
  return hipGetLastError();
}

__global__ __launch_bounds__(256) void k_mask_pack(const uint8_t* __restrict__ mask, int64_t S,
                                                   uint32_t* __restrict__ bits) {
  const int64_t nwords = (S + 31) / 32;
  const int64_t span = (int64_t)gridDim.x * 256;
  for (int64_t base = (int64_t)blockIdx.x * 256; base < S; base += span) {
    const int64_t i = base + threadIdx.x;
    store_ballot(i < S && mask[i] != 0, base + (threadIdx.x & ~63), nwords, bits);
  }
}

hipError_t launch_mask_pack(const uint8_t* mask, int64_t S, uint32_t* bits, hipStream_t st) {
  if (S <= 0) return hipSuccess;
  int64_t blocks = (S + 255) / 256;
  if (blocks > 8192) blocks = 8192;
  k_mask_pack<<<dim3((unsigned)blocks), 256, 0, st>>>(mask, S, bits);
  return hipGetLastError();
}

}  // namespace ipfb
