// The alternative solvers of Appendix C, against which the circulant inverse
// is compared: a Tikhonov-regularised solve of each sub-filter path's linear
// system (Section 2.3's d_n = W_n x_n, W_n the [b-p+1, b] Toeplitz matrix of
// the path's taps) by banded Cholesky, and FIR filtering of each path with
// its decorrelation kernel truncated to L lags.
#include "fft_lds.hpp"
#include "launch.hpp"

namespace ipfb {

// ---- Tikhonov by banded Cholesky ---------------------------------------------
// Per column n: x = c (W^T W + phi^2 I)^{-1} W^T d, W^T W + phi^2 I = H with
// H[i][j] = sum_k W[k][i] W[k][j] + phi^2 [i = j], banded (|i - j| < P), and
// (W^T d)_i = sum_r h_r d_{i-r} over the spectra 0 <= i - r < nspec.
// H = L L^T row by row (i = 0 .. b-1): L[i][j] = (H[i][j] - sum_{k<j} L[i][k]
// L[j][k]) / L[j][j] for i-P < j < i, L[i][i] = sqrt(H[i][i] - sum L[i][k]^2);
// forward y_i = ((W^T d)_i - sum_k L[i][k] y_k) / L[i][i]; backward
// x_i = (y_i - sum_{t=1}^{P-1} L[i+t][i] x_{i+t}) / L[i][i].
// One thread per column (the columns are the only independent work: each
// sweep is sequential in i), FP64 throughout. Every thread works on the same
// row at a time, so the rows whose Gram entries are the interior ones
// (j >= P-1 and j < nspec: all P - t products present) take them from a table
// made once, with no branch divergence. The diagonal is kept as its
// reciprocal, so the sweeps multiply instead of divide. The last P-1 rows of
// L, the last P data values and the last P-1 results stay in registers; the
// rows of L and y go to the workspace for the backward sweep (row i: the
// reciprocal diagonal, then L[i][i-t] for t = 1..P-1, then y_i; laid out
// [i][P+1][N] for coalesced access). Both sweeps fetch their inputs a few
// rows ahead (fewer for wide bands, whose P x P ring fills the registers), so
// a row's step does not wait on memory. d: the first nspec rows of x (the row
// stage's output), then x is overwritten with the result.
template <int P>
struct TikFetch {
  static constexpr int CH = P <= 5 ? 8 : (P <= 8 ? 4 : 1);  // rows of d ahead (forward sweep)
  static constexpr int CB = P <= 5 ? 4 : 1;                  // workspace rows ahead (backward sweep)
};
template <typename T, int P>
__global__ __launch_bounds__(64) void k_tik(T* __restrict__ x, int N, int64_t b, const double* __restrict__ win,
                                            double phi2, double cnorm, double* __restrict__ ws) {
  const int n = blockIdx.x * 64 + threadIdx.x;
  if (n >= N) return;
  const int64_t nspec = b - P + 1;
  double h[P], hint[P];
#pragma unroll
  for (int r = 0; r < P; ++r) h[r] = win[(int64_t)r * N + n];
#pragma unroll
  for (int t = 0; t < P; ++t) {  // interior Gram entries H[i][i-t]
    double s = t == 0 ? phi2 : 0.0;
#pragma unroll
    for (int r = 0; r + t < P; ++r) s += h[r + t] * h[r];
    hint[t] = s;
  }
  double lr[P][P];  // ring: lr[q] = row i - q (q = 1 .. P-1): [0] = 1/L[i-q][i-q], [t] = L[i-q][i-q-t]
  double yv[P], dv[P];
#pragma unroll
  for (int q = 0; q < P; ++q) {
    yv[q] = dv[q] = 0.0;
#pragma unroll
    for (int t = 0; t < P; ++t) lr[q][t] = 0.0;
  }
  const int64_t rs = (int64_t)(P + 1) * N;  // workspace stride of one row
  constexpr int kTikCh = TikFetch<P>::CH;
  double dch[kTikCh], dnx[kTikCh];
  auto load_d = [&](int64_t i0, double* v) {
#pragma unroll
    for (int u = 0; u < kTikCh; ++u) v[u] = (i0 + u < nspec) ? (double)x[(i0 + u) * N + n] : 0.0;
  };
  load_d(0, dch);
  for (int64_t i0 = 0; i0 < b; i0 += kTikCh) {
    if (i0 + kTikCh < b) load_d(i0 + kTikCh, dnx);
#pragma unroll
    for (int u = 0; u < kTikCh; ++u) {
      const int64_t i = i0 + u;
      if (i >= b) break;
      // shift the rings: slot q holds row / value i - q
#pragma unroll
      for (int q = P - 1; q > 0; --q) {
        yv[q] = yv[q - 1];
        dv[q] = dv[q - 1];
#pragma unroll
        for (int t = 0; t < P; ++t) lr[q][t] = lr[q - 1][t];
      }
      dv[0] = dch[u];
      // (W^T d)_i = sum_r h_r d_{i-r}, 0 <= i - r < nspec
      double rhs = 0.0;
#pragma unroll
      for (int r = 0; r < P; ++r)
        if (i - r >= 0 && i - r < nspec) rhs += h[r] * dv[r];
      // row i of L: entries for j = i - t, t = P-1 .. 1, then the diagonal
      double row[P];
#pragma unroll
      for (int t = 0; t < P; ++t) row[t] = 0.0;
#pragma unroll
      for (int t = P - 1; t >= 0; --t) {
        const int64_t j = i - t;
        if (j < 0) continue;
        double hij;
        if (j >= P - 1 && j < nspec) {
          hij = hint[t];
        } else {  // H[i][j] = sum over rows k = j - r, 0 <= r, r + t < P, 0 <= k < nspec of h_{r+t} h_r
          hij = t == 0 ? phi2 : 0.0;
#pragma unroll
          for (int r = 0; r + t < P; ++r) {
            const int64_t k = j - r;
            if (k >= 0 && k < nspec) hij += h[r + t] * h[r];
          }
        }
        // minus sum over k in [max(0, i-P+1), j-1] of L[i][k] L[j][k]:
        // L[i][k] = row[i-k], L[j][k] = lr[t][j-k] (row j is ring slot t)
#pragma unroll
        for (int v = t + 1; v < P; ++v) {  // k = i - v
          if (i - v < 0) continue;
          hij -= row[v] * (t == 0 ? row[v] : lr[t][v - t]);
        }
        if (t == 0) row[0] = 1.0 / sqrt(hij);  // the reciprocal diagonal
        else row[t] = hij * lr[t][0];
      }
      double yi = rhs;
#pragma unroll
      for (int v = 1; v < P; ++v)
        if (i - v >= 0) yi -= row[v] * yv[v];
      yi *= row[0];
      yv[0] = yi;
#pragma unroll
      for (int t = 0; t < P; ++t) {
        lr[0][t] = row[t];
        ws[i * rs + (int64_t)t * N + n] = row[t];
      }
      ws[i * rs + (int64_t)P * N + n] = yi;
    }
#pragma unroll
    for (int u = 0; u < kTikCh; ++u) dch[u] = dnx[u];
  }
  // backward: xs[q] = x_{i+q}; rows i+q of L in the ring again, kTikCh rows
  // of the workspace fetched ahead (fewer for wide bands: the register budget)
  constexpr int CB = TikFetch<P>::CB;
  double xs[P];
#pragma unroll
  for (int q = 0; q < P; ++q) {
    xs[q] = 0.0;
#pragma unroll
    for (int t = 0; t < P; ++t) lr[q][t] = 0.0;
  }
  double wch[CB][P + 1], wnx[CB][P + 1];
  auto load_w = [&](int64_t itop, double (*v)[P + 1]) {  // rows itop, itop - 1, ..., itop - CB + 1
#pragma unroll
    for (int u = 0; u < CB; ++u)
#pragma unroll
      for (int t = 0; t <= P; ++t) v[u][t] = (itop - u >= 0) ? ws[(itop - u) * rs + (int64_t)t * N + n] : 0.0;
  };
  load_w(b - 1, wch);
  for (int64_t itop = b - 1; itop >= 0; itop -= CB) {
    if (itop - CB >= 0) load_w(itop - CB, wnx);
#pragma unroll
    for (int u = 0; u < CB; ++u) {
      const int64_t i = itop - u;
      if (i < 0) break;
#pragma unroll
      for (int q = P - 1; q > 0; --q) {
        xs[q] = xs[q - 1];
#pragma unroll
        for (int t = 0; t < P; ++t) lr[q][t] = lr[q - 1][t];
      }
#pragma unroll
      for (int t = 0; t < P; ++t) lr[0][t] = wch[u][t];
      double xi = wch[u][P];
#pragma unroll
      for (int q = 1; q < P; ++q)
        if (i + q < b) xi -= lr[q][q] * xs[q];  // L[i+q][i] = row i+q at offset q
      xi *= lr[0][0];
      xs[0] = xi;
      x[i * N + n] = T(cnorm * xi);
    }
#pragma unroll
    for (int u = 0; u < CB; ++u)
#pragma unroll
      for (int t = 0; t <= P; ++t) wch[u][t] = wnx[u][t];
  }
}

template <int P>
static hipError_t launch_tik_p(int prec, void* x, int N, int64_t b, const double* win64, double phi, double cnorm,
                               double* ws, hipStream_t st) {
  const dim3 grid((unsigned)((N + 63) / 64));
  if (prec == F32) k_tik<float, P><<<grid, 64, 0, st>>>((float*)x, N, b, win64, phi * phi, cnorm, ws);
  else k_tik<double, P><<<grid, 64, 0, st>>>((double*)x, N, b, win64, phi * phi, cnorm, ws);
  return hipGetLastError();
}

hipError_t launch_tikhonov(int prec, void* x, int N, int ntap, int64_t b, const double* win64, double phi,
                           double cnorm, double* ws, hipStream_t st) {
  if (b < ntap || N < 1) return hipErrorInvalidValue;
  switch (ntap) {
    case 2: return launch_tik_p<2>(prec, x, N, b, win64, phi, cnorm, ws, st);
    case 3: return launch_tik_p<3>(prec, x, N, b, win64, phi, cnorm, ws, st);
    case 4: return launch_tik_p<4>(prec, x, N, b, win64, phi, cnorm, ws, st);
    case 5: return launch_tik_p<5>(prec, x, N, b, win64, phi, cnorm, ws, st);
    case 8: return launch_tik_p<8>(prec, x, N, b, win64, phi, cnorm, ws, st);
    case 16: return launch_tik_p<16>(prec, x, N, b, win64, phi, cnorm, ws, st);
    default: return hipErrorNotSupported;
  }
}

// ---- FIR decorrelation with truncated kernels --------------------------------
// A unit sample at frame 0 of every column (the circulant inverse turns it
// into the decorrelation kernels).
template <typename T>
__global__ __launch_bounds__(256) void k_delta_frames(T* __restrict__ x, int64_t total, int N) {
  const int64_t stride = (int64_t)gridDim.x * 256;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < total; e += stride) x[e] = e < N ? T(1) : T(0);
}

// g[l][n] = c[(c0 + l) mod b][n], l < L: the kernel lags c0 .. c0 + L - 1
template <typename T>
__global__ __launch_bounds__(256) void k_fir_extract(const T* __restrict__ c, T* __restrict__ g, int N, int64_t b,
                                                     int L, int64_t c0) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= (int64_t)L * N) return;
  const int l = (int)(e / N), n = (int)(e - (int64_t)l * N);
  int64_t j = (c0 + l) % b;
  if (j < 0) j += b;
  g[e] = c[j * N + n];
}

hipError_t launch_fir_setup(int prec, int stage, void* frames, void* g, int N, int64_t b, int L, int64_t c0,
                            hipStream_t st) {
  if (stage == 0) {
    const int64_t total = b * (int64_t)N;
    int64_t blocks = (total + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    if (prec == F32) k_delta_frames<float><<<dim3((unsigned)blocks), 256, 0, st>>>((float*)frames, total, N);
    else k_delta_frames<double><<<dim3((unsigned)blocks), 256, 0, st>>>((double*)frames, total, N);
  } else {
    const dim3 grid((unsigned)(((int64_t)L * N + 255) / 256));
    if (prec == F32) k_fir_extract<float><<<grid, 256, 0, st>>>((const float*)frames, (float*)g, N, b, L, c0);
    else k_fir_extract<double><<<grid, 256, 0, st>>>((const double*)frames, (double*)g, N, b, L, c0);
  }
  return hipGetLastError();
}

// x[j][n] = sum_{l<L} g[l][n] d[(j - c0 - l) mod b][n]. Workgroup: 64 columns
// x 4 groups of kFirTJ consecutive output frames; the 64 columns' kernels sit
// in LDS, zero-padded to a multiple of kFirCH lags. A thread keeps its
// kFirTJ outputs in registers and takes the taps kFirCH at a time: the chunk's
// taps and the kFirTJ + kFirCH - 1 inputs they reach, then kFirTJ x kFirCH
// multiply-adds from registers (FP64 sums).
constexpr int kFirTJ = 16, kFirCH = 8;
template <typename T>
__global__ __launch_bounds__(256) void k_fir(const T* __restrict__ d, const T* __restrict__ g, T* __restrict__ x,
                                             int N, int64_t b, int L, int64_t c0) {
  extern __shared__ unsigned char fir_smem[];
  T* gs = reinterpret_cast<T*>(fir_smem);  // [Lp][64]
  const int tid = threadIdx.x;
  const int col = tid & 63, rg = tid >> 6;
  const int ntile = (N + 63) / 64;
  const int tile = (int)(blockIdx.x % ntile);
  const int64_t fb = (int64_t)(blockIdx.x / ntile) * (4 * kFirTJ);
  const int n = tile * 64 + col;
  const int Lp = (L + kFirCH - 1) / kFirCH * kFirCH;
  for (int e = tid; e < Lp * 64; e += 256) {
    const int l = e >> 6, c = e & 63;
    const int nn = tile * 64 + c;
    gs[e] = (l < L && nn < N) ? g[(int64_t)l * N + nn] : T(0);
  }
  __syncthreads();
  if (n >= N) return;
  const int64_t j0 = fb + rg * kFirTJ;
  if (j0 >= b) return;
  double acc[kFirTJ];
#pragma unroll
  for (int o = 0; o < kFirTJ; ++o) acc[o] = 0.0;
  // din[t] = d[j0 - c0 - l0 - (kFirCH - 1) + t]: output o, tap l0 + c reads
  // t = o - c + kFirCH - 1. The next chunk's window is this one moved
  // kFirCH frames back: kFirCH new inputs, fetched during this chunk's
  // multiply-adds, and the rest shifted in registers.
  constexpr int NIN = kFirTJ + kFirCH - 1;
  auto wrap = [&](int64_t k) {
    k %= b;
    return k < 0 ? k + b : k;
  };
  double din[NIN], nx[kFirCH];
  {
    int64_t k = wrap(j0 - c0 - (kFirCH - 1));
#pragma unroll
    for (int t = 0; t < NIN; ++t) {
      din[t] = (double)d[k * N + n];
      k = (k + 1 == b) ? 0 : k + 1;
    }
  }
  for (int l0 = 0; l0 < Lp; l0 += kFirCH) {
    if (l0 + kFirCH < Lp) {
      int64_t k = wrap(j0 - c0 - (l0 + kFirCH) - (kFirCH - 1));
#pragma unroll
      for (int t = 0; t < kFirCH; ++t) {
        nx[t] = (double)d[k * N + n];
        k = (k + 1 == b) ? 0 : k + 1;
      }
    }
    double tg[kFirCH];
#pragma unroll
    for (int c = 0; c < kFirCH; ++c) tg[c] = (double)gs[(l0 + c) * 64 + col];
#pragma unroll
    for (int o = 0; o < kFirTJ; ++o)
#pragma unroll
      for (int c = 0; c < kFirCH; ++c) acc[o] += tg[c] * din[o - c + kFirCH - 1];
#pragma unroll
    for (int t = NIN - 1; t >= kFirCH; --t) din[t] = din[t - kFirCH];
#pragma unroll
    for (int t = 0; t < kFirCH; ++t) din[t] = nx[t];
  }
#pragma unroll
  for (int o = 0; o < kFirTJ; ++o)
    if (j0 + o < b) x[(j0 + o) * N + n] = T(acc[o]);
}

hipError_t launch_fir(int prec, const void* d, const void* g, void* x, int N, int64_t b, int L, int64_t c0,
                      hipStream_t st) {
  if (L < 1 || L > kFirMaxTaps) return hipErrorInvalidValue;
  const int64_t nfb = (b + 4 * kFirTJ - 1) / (4 * kFirTJ);
  const int64_t grid = nfb * ((N + 63) / 64);
  if (grid > 0x7fffffffLL) return hipErrorNotSupported;
  const int Lp = (L + kFirCH - 1) / kFirCH * kFirCH;
  const size_t lds = (size_t)Lp * 64 * (prec == F32 ? sizeof(float) : sizeof(double));
  if (prec == F32)
    k_fir<float><<<dim3((unsigned)grid), 256, lds, st>>>((const float*)d, (const float*)g, (float*)x, N, b, L, c0);
  else
    k_fir<double><<<dim3((unsigned)grid), 256, lds, st>>>((const double*)d, (const double*)g, (double*)x, N, b, L,
                                                           c0);
  return hipGetLastError();
}

}  // namespace ipfb
