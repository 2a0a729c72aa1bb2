// Forward PFB (Section 2.2's polyphase equation, Section 2.3's y = F S W x with
// the window sliding down the [frames, N] array one frame per spectrum):
// used to channelise, and re-applied at a longer frame N' = u N to
// up-channelize the inverse (Section 4.3). Also the autospectrum
// A(f) = (1/b') sum_j |Y_j(f)|^2 (Section 4.1's error metric) and the 4-bit
// quantiser used to synthesise inputs (Section 4.3's mid-tread quantiser).
//
// Frames that fit in LDS (N/2 complex <= 128 KiB) use one workgroup per
// spectrum: the windowed p-frame sum is formed while loading, then an N/2-point
// complex FFT and the real-spectrum split. Longer frames (the x64 fine
// re-channelization, N' = 2^18) take the two-pass path of k_pfb_long.hip.
#include "fft_lds.hpp"
#include "launch.hpp"

namespace ipfb {

// WIDE: 8 elements per thread in FP32 as well (twice the threads), for
// launches of fewer workgroups than the device has CUs, where each
// workgroup's FFT latency, not occupancy, sets the time (16 frames of 2^14:
// 32 against 25 us).
template <typename T, int LOG2N, bool WIDE = false>
struct FwdCfg {
  static constexpr int H = 1 << (LOG2N - 1);
  static constexpr int C = H >= 1024 ? 1 : 1024 / H;
  static constexpr int EPT = (sizeof(T) == 4 && !WIDE) ? 16 : 8;
  static constexpr int NT0 = (H * C) / EPT;
  static constexpr int NT = NT0 < 64 ? 64 : (NT0 > 1024 ? 1024 : NT0);
};

// X[k] = (Z_k + conj Z_{H-k})/2 + e^{-2 pi i k/N} (Z_k - conj Z_{H-k}) / (2i)
template <typename T>
__device__ __forceinline__ cx<T> split_real(cx<T> zk, cx<T> zm, cx<T> ek) {
  const cx<T> A = zk + conj(zm);
  const cx<T> Bd = zk - conj(zm);
  const cx<T> eB = cmul(ek, Bd);
  return mk<T>(T(0.5) * (A.x + eB.y), T(0.5) * (A.y - eB.x));
}

template <typename T>
__device__ __forceinline__ cx<T> polyphase_pair(const T* __restrict__ x, const T* __restrict__ win,
                                                int64_t j, int64_t nblock, int ntap, int64_t N,
                                                int64_t m) {
  cx<T> acc = mk<T>(T(0), T(0));
  for (int r = 0; r < ntap; ++r) {
    int64_t src = j + r;
    if (src >= nblock) src %= nblock;
    const cx<T> xv = reinterpret_cast<const cx<T>*>(x + src * N)[m];
    const cx<T> wv = reinterpret_cast<const cx<T>*>(win + (int64_t)r * N)[m];
    acc.x += wv.x * xv.x;
    acc.y += wv.y * xv.y;
  }
  return acc;
}

template <typename T, int LOG2N, bool WIDE>
__global__ __launch_bounds__((FwdCfg<T, LOG2N, WIDE>::NT)) void k_pfb_fwd(const T* __restrict__ x,
                                                                        cx<T>* __restrict__ y, int64_t nblock,
                                                                        int ntap, const T* __restrict__ win,
                                                                        const cx<T>* __restrict__ twN) {
  using Cfg = FwdCfg<T, LOG2N, WIDE>;
  constexpr int N = 1 << LOG2N, H = Cfg::H, C = Cfg::C, NT = Cfg::NT;
  constexpr int LS = lds_len(H);
  __shared__ cx<T> s[C * LS];
  const int tid = threadIdx.x;
  const int64_t j0 = (int64_t)blockIdx.x * C;
  for (int e = tid; e < C * H; e += NT) {
    const int c = e / H, m = e % H;
    const int64_t j = j0 + c;
    cx<T> acc = mk<T>(T(0), T(0));
    if (j < nblock) acc = polyphase_pair<T>(x, win, j, nblock, ntap, N, m);
    s[c * LS + pidx(m)] = acc;
  }
  __syncthreads();
  lds_fft<T, H, NT, C, -1>(s, LS, twN, 2);
  for (int e = tid; e < C * (H + 1); e += NT) {
    const int c = e / (H + 1), k = e % (H + 1);
    const int64_t j = j0 + c;
    if (j < nblock) {
      const cx<T> zk = s[c * LS + pidx(k & (H - 1))];
      const cx<T> zm = s[c * LS + pidx((H - k) & (H - 1))];
      y[j * (H + 1) + k] = split_real(zk, zm, twN[k]);
    }
  }
}

template <typename T, int LOG2N>
static hipError_t launch_fwd_small_t(const void* x, void* y, int64_t nblock, int ntap, const void* winT,
                                     const void* twN, hipStream_t st) {
  using Cfg = FwdCfg<T, LOG2N>;
  using Wide = FwdCfg<T, LOG2N, true>;
  const int64_t grid = (nblock + Cfg::C - 1) / Cfg::C;
  if (grid == 0) return hipSuccess;
  if (Wide::NT != Cfg::NT && grid < 256)
    k_pfb_fwd<T, LOG2N, true><<<dim3((unsigned)grid), dim3(Wide::NT), 0, st>>>(
        (const T*)x, (cx<T>*)y, nblock, ntap, (const T*)winT, (const cx<T>*)twN);
  else
    k_pfb_fwd<T, LOG2N, false><<<dim3((unsigned)grid), dim3(Cfg::NT), 0, st>>>(
        (const T*)x, (cx<T>*)y, nblock, ntap, (const T*)winT, (const cx<T>*)twN);
  return hipGetLastError();
}

#define FWD_CASE(T, L) \
  case L: return launch_fwd_small_t<T, L>(x, y, nblock, ntap, winT, twN, st);

hipError_t launch_pfb_fwd_small(int prec, int log2n, const void* x, void* y, int64_t nblock, int ntap,
                                const void* winT, const void* twN, hipStream_t st) {
  if (prec == F32) {
    switch (log2n) {
      FWD_CASE(float, 2) FWD_CASE(float, 3) FWD_CASE(float, 4) FWD_CASE(float, 5) FWD_CASE(float, 6)
      FWD_CASE(float, 7) FWD_CASE(float, 8) FWD_CASE(float, 9) FWD_CASE(float, 10) FWD_CASE(float, 11)
      FWD_CASE(float, 12) FWD_CASE(float, 13) FWD_CASE(float, 14) FWD_CASE(float, 15)
      default: return hipErrorInvalidValue;
    }
  }
  switch (log2n) {
    FWD_CASE(double, 2) FWD_CASE(double, 3) FWD_CASE(double, 4) FWD_CASE(double, 5) FWD_CASE(double, 6)
    FWD_CASE(double, 7) FWD_CASE(double, 8) FWD_CASE(double, 9) FWD_CASE(double, 10) FWD_CASE(double, 11)
    FWD_CASE(double, 12) FWD_CASE(double, 13) FWD_CASE(double, 14)
    default: return hipErrorInvalidValue;
  }
}

// ---- autospectrum / channel power (deterministic two-stage sums) -------------
template <typename T>
__global__ __launch_bounds__(256) void k_power_partial(const cx<T>* __restrict__ y, int64_t nspec, int nchan,
                                                       int jchunk, double* __restrict__ part) {
  const int k = blockIdx.x * 256 + threadIdx.x;
  const int c = blockIdx.y;
  if (k >= nchan) return;
  const int64_t j0 = (int64_t)c * jchunk;
  int64_t j1 = j0 + jchunk;
  if (j1 > nspec) j1 = nspec;
  double acc = 0.0;
  for (int64_t j = j0; j < j1; ++j) {
    const cx<T> v = y[j * nchan + k];
    acc += (double)v.x * (double)v.x + (double)v.y * (double)v.y;
  }
  part[(int64_t)c * nchan + k] = acc;
}

// out may alias part's first row (the quantiser's scales reuse it): thread k
// reads only column k and writes out[k] after its last read, so no restrict.
__global__ __launch_bounds__(256) void k_power_final(const double* part, int nchunks, int nchan, double mult,
                                                     double* out) {
  const int k = blockIdx.x * 256 + threadIdx.x;
  if (k >= nchan) return;
  double acc = 0.0;
  for (int c = 0; c < nchunks; ++c) acc += part[(int64_t)c * nchan + k];
  out[k] = acc * mult;
}

hipError_t launch_power_partial(int prec, const void* y, int64_t nspec, int nchan, int jchunk, double* part,
                                hipStream_t st) {
  const int nchunks = (int)((nspec + jchunk - 1) / jchunk);
  if (nchunks == 0 || nchan == 0) return hipSuccess;
  dim3 grid((nchan + 255) / 256, nchunks);
  if (prec == F32)
    k_power_partial<float><<<grid, 256, 0, st>>>((const cx<float>*)y, nspec, nchan, jchunk, part);
  else
    k_power_partial<double><<<grid, 256, 0, st>>>((const cx<double>*)y, nspec, nchan, jchunk, part);
  return hipGetLastError();
}

hipError_t launch_power_final(const double* part, int nchunks, int nchan, double mult, double* out,
                              hipStream_t st) {
  if (nchan == 0) return hipSuccess;
  k_power_final<<<(nchan + 255) / 256, 256, 0, st>>>(part, nchunks, nchan, mult, out);
  return hipGetLastError();
}

__global__ __launch_bounds__(256) void k_scales(const double* __restrict__ halfpow, int nchan, double levels,
                                                float* __restrict__ sc) {
  const int k = blockIdx.x * 256 + threadIdx.x;
  if (k >= nchan) return;
  const double sig = sqrt(halfpow[k]);
  sc[k] = sig > 0.0 ? (float)(levels / sig) : 1.0f;
}

hipError_t launch_scales(const double* halfpow, int nchan, double levels, float* scales, hipStream_t st) {
  k_scales<<<(nchan + 255) / 256, 256, 0, st>>>(halfpow, nchan, levels, scales);
  return hipGetLastError();
}

template <typename T>
__global__ __launch_bounds__(256) void k_quantize(const cx<T>* __restrict__ y, int64_t total, int nchan,
                                                  const float* __restrict__ sc, uint8_t* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= total) return;
  const int k = (int)(i % nchan);
  const double s = (double)sc[k];
  const cx<T> v = y[i];
  const double qr = fmin(7.0, fmax(-7.0, rint(s * (double)v.x)));
  const double qi = fmin(7.0, fmax(-7.0, rint(s * (double)v.y)));
  const int r = (int)qr, m = (int)qi;
  out[i] = (uint8_t)(((r & 0xF) << 4) | (m & 0xF));
}

hipError_t launch_quantize(int prec, const void* y, int64_t nspec, int nchan, const float* scales,
                           uint8_t* packed, hipStream_t st) {
  const int64_t total = nspec * nchan;
  if (total == 0) return hipSuccess;
  const unsigned grid = (unsigned)((total + 255) / 256);
  if (prec == F32)
    k_quantize<float><<<grid, 256, 0, st>>>((const cx<float>*)y, total, nchan, scales, packed);
  else
    k_quantize<double><<<grid, 256, 0, st>>>((const cx<double>*)y, total, nchan, scales, packed);
  return hipGetLastError();
}

}  // namespace ipfb
