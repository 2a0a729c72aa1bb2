// Row stage of the circulant inverse PFB (Section 3: an N-point inverse FFT
// per spectrum undoes F; Appendix C: the first of the three FFT stages).
//
// One workgroup inverts C spectra. The N-point inverse real FFT runs as an
// N/2-point complex inverse FFT on
//   Z[k] = (Y[k] + conj Y[N/2-k]) + i e^{+2 pi i k/N} (Y[k] - conj Y[N/2-k]),
// whose output z[m] holds the real samples 2m (real part) and 2m+1 (imaginary
// part). Dequantisation of the 4-bit input and the 1/N normalisation are
// folded into Y, so the spectra are read once, straight from HBM, and the
// frame is written once as contiguous float2/double2.
#include "fft_lds.hpp"
#include "launch.hpp"

namespace ipfb {

// fac[k] = 1/(s_k N) for the 4-bit format (computed once per call in FP64)
template <typename T, int FMT>
__device__ __forceinline__ cx<T> load_spec(const void* __restrict__ in, const T* __restrict__ fac,
                                           int64_t idx, int k, int N) {
  if constexpr (FMT == IN_C4) {
    const signed char b = reinterpret_cast<const signed char*>(in)[idx];
    const int re = b >> 4;                            // high nibble, sign-extended
    const int im = (signed char)(b << 4) >> 4;        // low nibble, sign-extended
    const T f = fac[k];
    return mk<T>(T(re) * f, T(im) * f);
  } else if constexpr (FMT == IN_CI8) {  // (re, im) as two signed bytes, any alignment
    const signed char* q = reinterpret_cast<const signed char*>(in) + 2 * idx;
    const T f = fac[k];
    return mk<T>(T((int)q[0]) * f, T((int)q[1]) * f);
  } else if constexpr (FMT == IN_CF32) {
    const cx<float> v = reinterpret_cast<const cx<float>*>(in)[idx];
    const T f = T(1.0 / (double)N);
    return mk<T>(T(v.x) * f, T(v.y) * f);
  } else if constexpr (FMT == IN_CF64) {
    const cx<double> v = reinterpret_cast<const cx<double>*>(in)[idx];
    const double f = 1.0 / (double)N;
    return mk<T>(T(v.x * f), T(v.y * f));
  } else {  // IN_ADJ: (N/2) irfft(c y) with c_0 = c_{N/2} = 2
    const cx<T> v = reinterpret_cast<const cx<T>*>(in)[idx];
    const T f = (k == 0 || k == N / 2) ? T(1) : T(0.5);
    return mk<T>(v.x * f, v.y * f);
  }
}

template <typename T, int LOG2N>
struct RowCfg {
  static constexpr int H = 1 << (LOG2N - 1);
  static constexpr int C = H >= 1024 ? 1 : 1024 / H;  // frames per workgroup
  static constexpr int EPT = sizeof(T) == 4 ? 16 : 8;
  static constexpr int NT0 = (H * C) / EPT;
  static constexpr int NT = NT0 < 64 ? 64 : (NT0 > 1024 ? 1024 : NT0);
};

template <typename T, int LOG2N, int FMT>
__global__ __launch_bounds__((RowCfg<T, LOG2N>::NT)) void k_row_irfft(
    const void* __restrict__ in, const T* __restrict__ sc, T* __restrict__ out, int64_t nrows,
    const cx<T>* __restrict__ twN) {
  using Cfg = RowCfg<T, LOG2N>;
  constexpr int N = 1 << LOG2N, H = Cfg::H, C = Cfg::C, NT = Cfg::NT;
  constexpr int LS = lds_len(H);
  __shared__ cx<T> s[C * LS];
  const int tid = threadIdx.x;
  const int64_t row0 = (int64_t)blockIdx.x * C;
  for (int e = tid; e < C * H; e += NT) {
    const int c = e / H, k = e % H;
    const int64_t row = row0 + c;
    cx<T> z = mk<T>(T(0), T(0));
    if (row < nrows) {
      const int64_t base = row * (H + 1);
      cx<T> yk = load_spec<T, FMT>(in, sc, base + k, k, N);
      cx<T> ym = load_spec<T, FMT>(in, sc, base + (H - k), H - k, N);
      if (k == 0) {  // DC and Nyquist imaginary parts carry nothing for a real frame
        yk.y = T(0);
        ym.y = T(0);
      }
      const cx<T> a = yk + conj(ym);
      const cx<T> bdiff = yk - conj(ym);
      const cx<T> w = conj(twN[k]);  // e^{+2 pi i k / N}
      const cx<T> t = cmul(w, bdiff);
      z = mk<T>(a.x - t.y, a.y + t.x);  // a + i t
    }
    s[c * LS + pidx(k)] = z;
  }
  __syncthreads();
  lds_fft<T, H, NT, C, +1>(s, LS, twN, 2);
  for (int e = tid; e < C * H; e += NT) {
    const int c = e / H, m = e % H;
    const int64_t row = row0 + c;
    if (row < nrows) reinterpret_cast<cx<T>*>(out + row * N)[m] = s[c * LS + pidx(m)];
  }
}

// Persistent form for 4-bit spectra: each workgroup inverts frames j, j + G,
// j + 2G, ... (G = grid size). The per-channel factors sit in LDS for the
// workgroup's life; a frame's packed bytes (an unaligned run of N/2+1 bytes) arrive as aligned
// 4-byte words staged through LDS, and the next frame's words are fetched
// into registers while the current frame's FFT runs.
template <typename T, int LOG2N>
struct RowPCfg {
  static constexpr int H = 1 << (LOG2N - 1);
  static constexpr int EPT = 8;
  static constexpr int NT0 = H / EPT;
  static constexpr int NT = NT0 < 64 ? 64 : (NT0 > 1024 ? 1024 : NT0);
  static constexpr int LS = lds_len(H);
  static constexpr int RAWW = (H + 1 + 3) / 4 + 2;  // words covering the run from its aligned start
  static constexpr int DPT = (RAWW + NT - 1) / NT;  // words fetched per thread
  // the pre-twiddles are read from the global table (it stays in L2): an
  // LDS copy would cost a workgroup per CU, and measured slower (101 against
  // 92 us at N = 4096, FP32)
  static constexpr int LDSB = LS * (int)sizeof(cx<T>) + (H + 1) * (int)sizeof(T) + RAWW * 4;
};

// The stream of global frame j: the last s with f0[s] <= j.
__device__ __forceinline__ int row_stream_of(int64_t j, const RowStream* __restrict__ tab, int nstreams) {
  int lo = 0, hi = nstreams - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (tab[mid].f0 <= j) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// MULTI: the frames of nstreams streams (tab: their spectra, scales,
// outputs and first global frames), numbered one stream after another; the
// per-channel factors are formed again whenever a workgroup moves to another
// stream. Otherwise one stream (in, chan_scale, out, nrows).
template <typename T, int LOG2N, bool MULTI>
__global__ __launch_bounds__((RowPCfg<T, LOG2N>::NT)) void k_row_c4p(
    const unsigned char* __restrict__ in1, const float* __restrict__ scale1, T* __restrict__ out1,
    int64_t nrows, const cx<T>* __restrict__ twN, const RowStream* __restrict__ tab, int nstreams) {
  using Cfg = RowPCfg<T, LOG2N>;
  constexpr int N = 1 << LOG2N, H = Cfg::H, NT = Cfg::NT, LS = Cfg::LS, EPT = Cfg::EPT;
  constexpr int RAWW = Cfg::RAWW, DPT = Cfg::DPT;
  static_assert(H % NT == 0 || NT == 64, "frame must split over the threads");
  __shared__ cx<T> s[LS];
  __shared__ T facs[H + 1];
  __shared__ unsigned int raw[RAWW];
  const int tid = threadIdx.x;
  // dequantisation factor 1/(s_k N), formed in FP64 from the stored FP32 scale
  auto set_facs = [&](const float* sc) {
    const __attribute__((address_space(1))) float* gsc = (const __attribute__((address_space(1))) float*)sc;
    for (int k = tid; k <= H; k += NT) facs[k] = T(1.0 / ((double)gsc[k] * (double)N));
  };
  if (!MULTI) set_facs(scale1);
  unsigned int pf[DPT];
  int snext = 0;  // MULTI: the stream of the frame fetched last
  auto fetch = [&](int64_t j) {
    const unsigned char* in = in1;
    int64_t jl = j, rows = nrows;
    if constexpr (MULTI) {
      snext = row_stream_of(j, tab, nstreams);
      in = tab[snext].spec;
      jl = j - tab[snext].f0;
      rows = tab[snext].b;
    }
    const int64_t total = rows * (int64_t)(H + 1);
    const int64_t b0 = jl * (int64_t)(H + 1);
    const int64_t a0 = b0 & ~int64_t(3);
    const int nd = (int)((b0 + H + 1 - a0 + 3) >> 2);
#pragma unroll
    for (int d = 0; d < DPT; ++d) {
      const int idx = tid + d * NT;
      const int64_t byte = a0 + 4 * (int64_t)idx;
      pf[d] = 0u;
      if (idx < nd) {
        if (byte + 4 <= total) {
          // read once: a non-temporal load, so that the input stream does not
          // push the frames this kernel writes out of the last-level cache
          // (the column pass that follows reads them back from there)
          pf[d] = ld_global_once(in + byte);
        } else {  // the array's last word may be partial: read its bytes one by one
          unsigned int w = 0u;
          for (int q = 0; q < 4 && byte + q < total; ++q) w |= ld_global_byte(in + byte + q) << (8 * q);
          pf[d] = w;
        }
      }
    }
  };
  int scur = -1;
  int64_t j = blockIdx.x;
  if (j < nrows) fetch(j);
  for (; j < nrows; j += gridDim.x) {
    const int sj = snext;
    if (MULTI && sj != scur) {  // uniform: the whole workgroup moves to another stream
      __syncthreads();          // the previous frame's factor reads are done
      set_facs(tab[sj].scale);
      scur = sj;
    }
#pragma unroll
    for (int d = 0; d < DPT; ++d) {
      const int idx = tid + d * NT;
      if (idx < RAWW) raw[idx] = pf[d];
    }
    __syncthreads();
    if (j + gridDim.x < nrows) fetch(j + gridDim.x);  // in flight during the FFT
    const int64_t jl = MULTI ? j - tab[sj].f0 : j;
    const unsigned char* rb = reinterpret_cast<const unsigned char*>(raw) + (int)((jl * (int64_t)(H + 1)) & 3);
    T* out = MULTI ? (T*)tab[sj].out : out1;
    cx<T>* orow = reinterpret_cast<cx<T>*>(out + jl * (int64_t)N);
    // Z_k = a + i t, a = Y_k + conj Y_{H-k}, t = e^{+2 pi i k/N} (Y_k - conj Y_{H-k});
    // k = 0 pairs DC with Nyquist (index H)
    auto zval = [&](int k) -> cx<T> {
      const signed char bk = (signed char)rb[k], bm = (signed char)rb[H - k];
      const T fk = facs[k], fm = facs[H - k];
      cx<T> yk = mk<T>(T(bk >> 4) * fk, T((signed char)(bk << 4) >> 4) * fk);
      cx<T> ym = mk<T>(T(bm >> 4) * fm, T((signed char)(bm << 4) >> 4) * fm);
      if (k == 0) {  // DC and Nyquist imaginary parts carry nothing for a real frame
        yk.y = T(0);
        ym.y = T(0);
      }
      const cx<T> a = yk + conj(ym);
      const cx<T> t = cmul(conj(twN[k]), yk - conj(ym));  // e^{+2 pi i k/N}
      return mk<T>(a.x - t.y, a.y + t.x);
    };
    // the FFT's own twiddles stay in global memory (L2): an LDS copy would
    // cost a workgroup per CU, which costs more than their latency
    using F = FftSplit<T, H, NT, 1>;
    static_assert(F::ok && F::R0 * NT == H, "one first-pass butterfly per thread");
    // one first-pass butterfly per thread, its inputs formed in registers from
    // the packed bytes; the last pass stores the frame (consecutive threads,
    // consecutive samples)
    constexpr int R0 = F::R0, LR0 = H / R0;
    cx<T> v[R0];
#pragma unroll
    for (int r = 0; r < R0; ++r) v[r] = zval(tid + r * LR0);
    fft_first_from_regs<T, R0, +1>(s, tid, v);
    __syncthreads();
    fft_middle<T, H, NT, 1, +1, true>(s, LS, twN, 2);
    fft_last_to<T, H, NT, 1, +1, true>(s, LS, twN, 2, [&](int, int m, cx<T> val) { st_global(orow + m, val); });
    __syncthreads();  // s and raw are rewritten for the next frame
  }
}

template <typename T, int LOG2N>
static hipError_t launch_row_t(int fmt, const void* in, const void* fac, void* out, int64_t nrows,
                               const void* twN, hipStream_t st) {
  using Cfg = RowCfg<T, LOG2N>;
  const int64_t grid = (nrows + Cfg::C - 1) / Cfg::C;
  if (grid == 0) return hipSuccess;
  const cx<T>* tw = reinterpret_cast<const cx<T>*>(twN);
  T* o = reinterpret_cast<T*>(out);
  const T* sc = reinterpret_cast<const T*>(fac);
  switch (fmt) {
    case IN_C4: k_row_irfft<T, LOG2N, IN_C4><<<dim3((unsigned)grid), dim3(Cfg::NT), 0, st>>>(in, sc, o, nrows, tw); break;
    case IN_CI8: k_row_irfft<T, LOG2N, IN_CI8><<<dim3((unsigned)grid), dim3(Cfg::NT), 0, st>>>(in, sc, o, nrows, tw); break;
    case IN_CF32: k_row_irfft<T, LOG2N, IN_CF32><<<dim3((unsigned)grid), dim3(Cfg::NT), 0, st>>>(in, sc, o, nrows, tw); break;
    case IN_CF64: k_row_irfft<T, LOG2N, IN_CF64><<<dim3((unsigned)grid), dim3(Cfg::NT), 0, st>>>(in, sc, o, nrows, tw); break;
    default: k_row_irfft<T, LOG2N, IN_ADJ><<<dim3((unsigned)grid), dim3(Cfg::NT), 0, st>>>(in, sc, o, nrows, tw); break;
  }
  return hipGetLastError();
}

#define ROW_CASE(T, L) \
  case L: return launch_row_t<T, L>(fmt, in, fac, out, nrows, twN, st);

hipError_t launch_row_irfft(int prec, int log2n, int fmt, const void* in, const void* fac,
                            void* out, int64_t nrows, const void* twN, hipStream_t st) {
  if (prec == F32) {
    switch (log2n) {
      ROW_CASE(float, 2) ROW_CASE(float, 3) ROW_CASE(float, 4) ROW_CASE(float, 5) ROW_CASE(float, 6)
      ROW_CASE(float, 7) ROW_CASE(float, 8) ROW_CASE(float, 9) ROW_CASE(float, 10) ROW_CASE(float, 11)
      ROW_CASE(float, 12) ROW_CASE(float, 13) ROW_CASE(float, 14) ROW_CASE(float, 15)
      default: return hipErrorInvalidValue;
    }
  }
  switch (log2n) {
    ROW_CASE(double, 2) ROW_CASE(double, 3) ROW_CASE(double, 4) ROW_CASE(double, 5) ROW_CASE(double, 6)
    ROW_CASE(double, 7) ROW_CASE(double, 8) ROW_CASE(double, 9) ROW_CASE(double, 10) ROW_CASE(double, 11)
    ROW_CASE(double, 12) ROW_CASE(double, 13) ROW_CASE(double, 14)
    default: return hipErrorInvalidValue;
  }
}

template <typename T, int LOG2N>
static hipError_t launch_row_c4_t(const void* in, const float* chan_scale, void* out, int64_t nrows,
                                  const void* twN, const RowStream* tab, int nstreams, hipStream_t st) {
  if constexpr (LOG2N >= 9 && RowPCfg<T, LOG2N>::LDSB <= 81920) {
    using Cp = RowPCfg<T, LOG2N>;
    const int64_t res = tab ? resident_workgroups(k_row_c4p<T, LOG2N, true>, Cp::NT)
                            : resident_workgroups(k_row_c4p<T, LOG2N, false>, Cp::NT);  // (cached after the first call)
    if (nrows == 0) return hipSuccess;
    const int64_t g = nrows < res ? nrows : res;
    if (tab)
      k_row_c4p<T, LOG2N, true><<<dim3((unsigned)g), dim3(Cp::NT), 0, st>>>(
          nullptr, nullptr, nullptr, nrows, (const cx<T>*)twN, tab, nstreams);
    else
      k_row_c4p<T, LOG2N, false><<<dim3((unsigned)g), dim3(Cp::NT), 0, st>>>(
          (const unsigned char*)in, chan_scale, (T*)out, nrows, (const cx<T>*)twN, nullptr, 0);
    return hipGetLastError();
  } else {
    return hipErrorNotSupported;
  }
}

#define ROWC4_CASE(T, L) \
  case L: return launch_row_c4_t<T, L>(in, chan_scale, out, nrows, twN, tab, nstreams, st);

hipError_t launch_row_c4(int prec, int log2n, const void* in, const float* chan_scale, void* out, int64_t nrows,
                         const void* twN, hipStream_t st, const RowStream* tab, int nstreams) {
  if (prec == F32) {
    switch (log2n) {
      ROWC4_CASE(float, 9) ROWC4_CASE(float, 10) ROWC4_CASE(float, 11) ROWC4_CASE(float, 12)
      ROWC4_CASE(float, 13)
      default: return hipErrorNotSupported;
    }
  }
  switch (log2n) {
    ROWC4_CASE(double, 9) ROWC4_CASE(double, 10) ROWC4_CASE(double, 11) ROWC4_CASE(double, 12)
    default: return hipErrorNotSupported;
  }
}

// fac[k] = 1 / (s_k N) in double, stored in the plan precision
template <typename T>
__global__ __launch_bounds__(256) void k_dequant_factors(const float* __restrict__ sc, int nchan, int N,
                                                         T* __restrict__ fac) {
  const int k = blockIdx.x * 256 + threadIdx.x;
  if (k < nchan) fac[k] = T(1.0 / ((double)sc[k] * (double)N));
}

hipError_t launch_dequant_factors(int prec, const float* chan_scale, int nchan, int N, void* fac,
                                  hipStream_t st) {
  const int grid = (nchan + 255) / 256;
  if (prec == F32)
    k_dequant_factors<float><<<grid, 256, 0, st>>>(chan_scale, nchan, N, (float*)fac);
  else
    k_dequant_factors<double><<<grid, 256, 0, st>>>(chan_scale, nchan, N, (double*)fac);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Transpose of the sliding multiply-and-sum (needed by the adjoint):
// x[i][n] = sum_{r<p} h[rN+n] z[(i-r) mod b][n]. Contiguous along n.
template <typename T>
__global__ __launch_bounds__(256) void k_adjoint_gather(const T* __restrict__ z, T* __restrict__ x,
                                                        int64_t nblock, int lblock, int ntap, int nchunk,
                                                        const T* __restrict__ win) {
  const int64_t i = blockIdx.x / nchunk;
  const int n = (blockIdx.x % nchunk) * 256 + threadIdx.x;
  if (n >= lblock) return;
  T acc = T(0);
  for (int r = 0; r < ntap; ++r) {
    int64_t src = (i - r) % nblock;
    if (src < 0) src += nblock;
    acc += win[(int64_t)r * lblock + n] * z[src * lblock + n];
  }
  x[i * lblock + n] = acc;
}

hipError_t launch_adjoint_gather(int prec, const void* z, void* x, int64_t nblock, int lblock, int ntap,
                                 const void* winT, hipStream_t st) {
  if (nblock == 0) return hipSuccess;
  const int nchunk = (lblock + 255) / 256;
  const dim3 grid((unsigned)(nblock * nchunk));
  if (prec == F32)
    k_adjoint_gather<float><<<grid, 256, 0, st>>>((const float*)z, (float*)x, nblock, lblock, ntap, nchunk,
                                                  (const float*)winT);
  else
    k_adjoint_gather<double><<<grid, 256, 0, st>>>((const double*)z, (double*)x, nblock, lblock, ntap,
                                                   nchunk, (const double*)winT);
  return hipGetLastError();
}

}  // namespace ipfb
