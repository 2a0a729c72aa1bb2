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
// re-channelization, N' = 2^18) use a four-step split N/2 = R1 * R2: pass A
// forms the polyphase sum and R1-point DFTs down strided columns and applies
// the inter-step twiddle; pass B runs the R2-point DFTs on contiguous rows and
// splits the real spectrum, pairing row k1 with row R1 - k1 in one workgroup.
#include "fft_lds.hpp"
#include "launch.hpp"

namespace ipfb {

template <typename T, int LOG2N>
struct FwdCfg {
  static constexpr int H = 1 << (LOG2N - 1);
  static constexpr int C = H >= 1024 ? 1 : 1024 / H;
  static constexpr int EPT = sizeof(T) == 4 ? 16 : 8;
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

template <typename T, int LOG2N>
__global__ __launch_bounds__((FwdCfg<T, LOG2N>::NT)) void k_pfb_fwd(const T* __restrict__ x,
                                                                  cx<T>* __restrict__ y, int64_t nblock,
                                                                  int ntap, const T* __restrict__ win,
                                                                  const cx<T>* __restrict__ twN) {
  using Cfg = FwdCfg<T, LOG2N>;
  constexpr int N = 1 << LOG2N, H = Cfg::H, C = Cfg::C, NT = Cfg::NT;
  __shared__ cx<T> s[C * H];
  const int tid = threadIdx.x;
  const int64_t j0 = (int64_t)blockIdx.x * C;
  for (int e = tid; e < C * H; e += NT) {
    const int c = e / H, m = e % H;
    const int64_t j = j0 + c;
    cx<T> acc = mk<T>(T(0), T(0));
    if (j < nblock) acc = polyphase_pair<T>(x, win, j, nblock, ntap, N, m);
    s[c * H + m] = acc;
  }
  __syncthreads();
  lds_fft<T, H, NT, C, -1>(s, H, twN, 2);
  for (int e = tid; e < C * (H + 1); e += NT) {
    const int c = e / (H + 1), k = e % (H + 1);
    const int64_t j = j0 + c;
    if (j < nblock) {
      const cx<T> zk = s[c * H + (k & (H - 1))];
      const cx<T> zm = s[c * H + ((H - k) & (H - 1))];
      y[j * (H + 1) + k] = split_real(zk, zm, twN[k]);
    }
  }
}

// ---- four-step pass A: polyphase sum + R1-point DFTs over m1 -----------------
template <typename T, int LOG2R1>
struct FwdACfg {
  static constexpr int R1 = 1 << LOG2R1;
  static constexpr int MB = sizeof(T) == 4 ? 16 : 8;  // consecutive m2 per workgroup
  static constexpr int LS = R1 + 1;
  static constexpr int EPT = sizeof(T) == 4 ? 16 : 8;
  static constexpr int NT0 = (R1 * MB) / EPT;
  static constexpr int NT = NT0 > 1024 ? 1024 : NT0;
};

template <typename T, int LOG2R1>
__global__ __launch_bounds__((FwdACfg<T, LOG2R1>::NT)) void k_pfb_fwd_A(
    const T* __restrict__ x, cx<T>* __restrict__ tmp, int64_t nblock, int ntap, const T* __restrict__ win,
    const cx<T>* __restrict__ twN, int N, int R2) {
  using Cfg = FwdACfg<T, LOG2R1>;
  constexpr int R1 = Cfg::R1, MB = Cfg::MB, LS = Cfg::LS, NT = Cfg::NT;
  __shared__ cx<T> s[MB * LS];
  const int tid = threadIdx.x;
  const int nmb = R2 / MB;
  const int64_t j = blockIdx.x / nmb;
  const int m2_0 = (blockIdx.x % nmb) * MB;
  for (int e = tid; e < R1 * MB; e += NT) {
    const int mb = e % MB, m1 = e / MB;
    const int64_t m = (int64_t)m1 * R2 + m2_0 + mb;
    s[mb * LS + m1] = polyphase_pair<T>(x, win, j, nblock, ntap, N, m);
  }
  __syncthreads();
  lds_fft<T, R1, NT, MB, -1>(s, LS, twN, N / R1);
  for (int e = tid; e < R1 * MB; e += NT) {
    const int mb = e % MB, k1 = e / MB;
    const int m2 = m2_0 + mb;
    const cx<T> w = twN[2 * m2 * k1];  // e^{-2 pi i m2 k1 / (N/2)}
    tmp[(j * R1 + k1) * (int64_t)R2 + m2] = cmul(s[mb * LS + k1], w);
  }
}

// ---- four-step pass B: R2-point DFTs over m2 + real split ---------------------
template <typename T, int LOG2R2>
struct FwdBCfg {
  static constexpr int R2 = 1 << LOG2R2;
  static constexpr int KB = sizeof(T) == 4 ? 16 : 8;  // row pairs per workgroup
  static constexpr int LS = R2 + 1;
  static constexpr int EPT = sizeof(T) == 4 ? 16 : 8;
  static constexpr int NT0 = (2 * KB * R2) / EPT;
  static constexpr int NT = NT0 > 1024 ? 1024 : NT0;
};

template <typename T, int LOG2R2>
__global__ __launch_bounds__((FwdBCfg<T, LOG2R2>::NT)) void k_pfb_fwd_B(
    const cx<T>* __restrict__ tmp, cx<T>* __restrict__ y, const cx<T>* __restrict__ twN, int N, int R1,
    int npb) {
  using Cfg = FwdBCfg<T, LOG2R2>;
  constexpr int R2 = Cfg::R2, KB = Cfg::KB, LS = Cfg::LS, NT = Cfg::NT;
  __shared__ cx<T> s[2 * KB * LS];
  const int tid = threadIdx.x;
  const int H = N / 2;
  const int64_t j = blockIdx.x / npb;
  const int w = blockIdx.x % npb;
  const bool special = (w == npb - 1);
  const int a = 1 + w * KB;
  const int count = special ? 1 : min(KB, R1 / 2 - a);
  // slot (half, i): half 0 holds rows a+i, half 1 their mirrors R1-a-i;
  // the special workgroup holds the self-paired rows 0 and R1/2.
  auto row_of = [&](int half, int i) -> int {
    if (special) return half == 0 ? 0 : R1 / 2;
    return half == 0 ? a + i : R1 - a - i;
  };
  for (int e = tid; e < 2 * KB * R2; e += NT) {
    const int sl = e / R2, m2 = e % R2;
    const int half = sl / KB, i = sl % KB;
    cx<T> v = mk<T>(T(0), T(0));
    if (i < count) v = tmp[(j * R1 + row_of(half, i)) * (int64_t)R2 + m2];
    s[sl * LS + m2] = v;
  }
  __syncthreads();
  lds_fft<T, R2, NT, 2 * KB, -1>(s, LS, twN, N / R2);
  cx<T>* yj = y + j * (int64_t)(H + 1);
  for (int e = tid; e < 2 * KB * R2; e += NT) {
    const int i = e % KB;
    const int t = e / KB;
    const int half = t & 1, k2 = t >> 1;
    if (i >= count) continue;
    const int sl = half * KB + i;
    const int row = row_of(half, i);
    int psl, pk2;
    if (!special) {
      psl = (1 - half) * KB + i;
      pk2 = R2 - 1 - k2;
    } else {
      psl = sl;
      pk2 = (half == 0) ? ((R2 - k2) & (R2 - 1)) : (R2 - 1 - k2);
    }
    const cx<T> zk = s[sl * LS + k2];
    const cx<T> zm = s[psl * LS + pk2];
    const int k = row + R1 * k2;
    yj[k] = split_real(zk, zm, twN[k]);
    if (special && half == 0 && k2 == 0) yj[H] = mk<T>(zk.x - zk.y, T(0));
  }
}

template <typename T, int LOG2N>
static hipError_t launch_fwd_small_t(const void* x, void* y, int64_t nblock, int ntap, const void* winT,
                                     const void* twN, hipStream_t st) {
  using Cfg = FwdCfg<T, LOG2N>;
  const int64_t grid = (nblock + Cfg::C - 1) / Cfg::C;
  if (grid == 0) return hipSuccess;
  k_pfb_fwd<T, LOG2N><<<dim3((unsigned)grid), dim3(Cfg::NT), 0, st>>>(
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

template <typename T, int L1>
static hipError_t launch_A_t(const void* x, void* tmp, int64_t nblock, int ntap, const void* winT,
                             const void* twN, int N, int R2, hipStream_t st) {
  using Cfg = FwdACfg<T, L1>;
  const int64_t grid = nblock * (R2 / Cfg::MB);
  k_pfb_fwd_A<T, L1><<<dim3((unsigned)grid), dim3(Cfg::NT), 0, st>>>(
      (const T*)x, (cx<T>*)tmp, nblock, ntap, (const T*)winT, (const cx<T>*)twN, N, R2);
  return hipGetLastError();
}

template <typename T, int L2>
static hipError_t launch_B_t(const void* tmp, void* y, int64_t nblock, const void* twN, int N, int R1,
                             hipStream_t st) {
  using Cfg = FwdBCfg<T, L2>;
  const int npb = (R1 / 2 - 1 + Cfg::KB - 1) / Cfg::KB + 1;
  const int64_t grid = nblock * npb;
  k_pfb_fwd_B<T, L2><<<dim3((unsigned)grid), dim3(Cfg::NT), 0, st>>>(
      (const cx<T>*)tmp, (cx<T>*)y, (const cx<T>*)twN, N, R1, npb);
  return hipGetLastError();
}

template <typename T>
static hipError_t launch_large_t(int log2n, const void* x, void* y, int64_t nblock, int ntap,
                                 const void* winT, const void* twN, void* tmp, hipStream_t st) {
  const int e = log2n - 1;  // log2 of N/2
  const int l1 = (e + 1) / 2, l2 = e / 2;
  const int N = 1 << log2n, R1 = 1 << l1, R2 = 1 << l2;
  if (nblock == 0) return hipSuccess;
  hipError_t err;
  switch (l1) {
    case 7: err = launch_A_t<T, 7>(x, tmp, nblock, ntap, winT, twN, N, R2, st); break;
    case 8: err = launch_A_t<T, 8>(x, tmp, nblock, ntap, winT, twN, N, R2, st); break;
    case 9: err = launch_A_t<T, 9>(x, tmp, nblock, ntap, winT, twN, N, R2, st); break;
    case 10: err = launch_A_t<T, 10>(x, tmp, nblock, ntap, winT, twN, N, R2, st); break;
    default: return hipErrorInvalidValue;
  }
  if (err != hipSuccess) return err;
  switch (l2) {
    case 7: return launch_B_t<T, 7>(tmp, y, nblock, twN, N, R1, st);
    case 8: return launch_B_t<T, 8>(tmp, y, nblock, twN, N, R1, st);
    case 9: return launch_B_t<T, 9>(tmp, y, nblock, twN, N, R1, st);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_pfb_fwd_large(int prec, int log2n, const void* x, void* y, int64_t nblock, int ntap,
                                const void* winT, const void* twN, void* tmp, hipStream_t st) {
  if (prec == F32) return launch_large_t<float>(log2n, x, y, nblock, ntap, winT, twN, tmp, st);
  return launch_large_t<double>(log2n, x, y, nblock, ntap, winT, twN, tmp, st);
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

__global__ __launch_bounds__(256) void k_power_final(const double* __restrict__ part, int nchunks, int nchan,
                                                     double mult, double* __restrict__ out) {
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
