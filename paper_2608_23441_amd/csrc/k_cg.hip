// Maximum-likelihood reconstruction with a time-domain prior (Section 4.2):
// minimise |d - A x|^2 + lam |D (x - prior)|^2, A = S W circular (acting on
// the frames after the N-point inverse FFT), D = diag(mask), by
// preconditioned conjugate gradient on (A^T A + lam D) x = A^T d + lam D prior.
//
// Vectors live in the transposed frame layout v_T[n][j] (sub-filter path n,
// frame j), so A^T A is a (2p-1)-tap circulant stencil along contiguous rows:
//   (A^T A x)_n[i] = sum_{t=-(p-1)}^{p-1} c_n[t] x_n[(i+t) mod b],
//   c_n[t] = sum_r h[rN+n] h[(r+t)N+n]  (autocorrelation of the column taps).
// The prior mask D is one bit per sample, kept in the transposed layout as
// rows of bw = ceil(b/32) 32-bit words (bit j of row n is frame j of path n),
// so the stencil reads 1/8 byte per element for it.
// Dot products and norms accumulate in FP64 per workgroup and are summed in a
// fixed order by one workgroup, which also updates the CG scalars in device
// memory: no host round trip inside the iteration loop.
#include "fft_lds.hpp"
#include "launch.hpp"
#include "reduce.hpp"

namespace ipfb {

constexpr int kCgNWG = 1024;  // workgroups of the element-wise kernels (fixed: deterministic sums)
constexpr int kCgNT = 256;

// bit j of row n of the transposed mask
__device__ __forceinline__ unsigned mask_bit(const uint32_t* __restrict__ mb, int64_t bw, int64_t n, int64_t j) {
  return (mb[n * bw + (j >> 5)] >> (j & 31)) & 1u;
}

// c_n[t] for t in [-(p-1), p-1], stored autoc[n * (2p-1) + t + p - 1], FP64
__global__ __launch_bounds__(256) void k_cg_autocorr(const double* __restrict__ win, int N, int ntap,
                                                     double* __restrict__ autoc) {
  const int n = blockIdx.x * 256 + threadIdx.x;
  if (n >= N) return;
  const int nt = 2 * ntap - 1;
  for (int t = -(ntap - 1); t <= ntap - 1; ++t) {
    double acc = 0.0;
    for (int r = 0; r < ntap; ++r) {
      const int s = r + t;
      if (s < 0 || s >= ntap) continue;
      acc += win[(int64_t)r * N + n] * win[(int64_t)s * N + n];
    }
    autoc[(int64_t)n * nt + t + ntap - 1] = acc;
  }
}

// q = (A^T A + lam D) p ; partial sums of p.q
template <typename T>
__global__ __launch_bounds__(kCgNT) void k_cg_normal(const T* __restrict__ p, T* __restrict__ q,
                                                     const double* __restrict__ autoc,
                                                     const uint32_t* __restrict__ mbits, int64_t bw, double lam,
                                                     int ntap, int64_t b, int64_t S, double* __restrict__ part) {
  __shared__ double sh[kCgNT];
  const int nt = 2 * ntap - 1;
  double acc = 0.0;
  for (int64_t e = (int64_t)blockIdx.x * kCgNT + threadIdx.x; e < S; e += (int64_t)gridDim.x * kCgNT) {
    const int64_t n = e / b, i = e - n * b;
    const T* row = p + n * b;
    const double* c = autoc + n * nt;
    double v = 0.0;
    for (int t = 0; t < nt; ++t) {
      int64_t k = i + t - (ntap - 1);
      if (k < 0) k += b;
      else if (k >= b) k -= b;
      v += c[t] * (double)row[k];
    }
    const double pe = (double)p[e];
    if (mask_bit(mbits, bw, n, i)) v += lam * pe;
    const T vt = T(v);
    q[e] = vt;
    acc += pe * (double)vt;
  }
  const double tot = block_sum<kCgNT>(acc, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = tot;
}

// Row-tiled forms of the two stencils: workgroup g takes rows g, g + G, ...
// (G = kCgNWG), each row in chunks of kCgCH elements staged in LDS with a
// halo of HMAX on both sides (wrapped circularly at the row ends), so no
// element index is ever divided or reduced modulo b except in the halo.
constexpr int kCgCH = kCgNT * 8;
constexpr int kCgHMAX = 64;  // ntap - 1 up to this; longer windows use the element-wise kernels

template <typename T>
__device__ __forceinline__ void cg_stage_row(const T* __restrict__ row, T* tile, int64_t c0, int len, int h,
                                             int64_t b) {
  for (int i = threadIdx.x; i < len + 2 * h; i += kCgNT) {
    int64_t k = c0 + i - h;
    if (k < 0 || k >= b) {
      k %= b;
      if (k < 0) k += b;
    }
    tile[i] = row[k];
  }
}

// q = (A^T A + lam D) p ; partial sums of p.q. Work items are (row, chunk)
// pairs; a workgroup fetches its next item's elements into registers while
// the current one is computed.
template <typename T>
__global__ __launch_bounds__(kCgNT) void k_cg_normal_rows(const T* __restrict__ p, T* __restrict__ q,
                                                          const double* __restrict__ autoc,
                                                          const uint32_t* __restrict__ mbits, int64_t bw, double lam,
                                                          int ntap, int64_t b, int64_t nrows,
                                                          double* __restrict__ part) {
  constexpr int EPT = kCgCH / kCgNT;
  __shared__ double sh[kCgNT];
  __shared__ double tile[kCgCH + 2 * kCgHMAX];  // widened once when staged
  __shared__ double cs[2 * kCgHMAX + 1];
  const int tid = threadIdx.x;
  const int h = ntap - 1, nt = 2 * ntap - 1;
  const int64_t nch = (b + kCgCH - 1) / kCgCH;
  const int64_t nw = nrows * nch;
  T pm[EPT], ph = T(0);
  unsigned mm[EPT];
  auto fetch = [&](int64_t w) {
    const int64_t n = w / nch, c0 = (w - n * nch) * kCgCH;
    const int len = (int)((b - c0) < kCgCH ? (b - c0) : kCgCH);
    const T* row = p + n * b;
#pragma unroll
    for (int k = 0; k < EPT; ++k) {
      const int i = tid + k * kCgNT;
      pm[k] = i < len ? row[c0 + i] : T(0);
      mm[k] = i < len ? mask_bit(mbits, bw, n, c0 + i) : 0u;
    }
    if (tid < 2 * h) {  // halo: h elements before the chunk, h after, wrapped at the row ends
      int64_t pos = tid < h ? c0 - h + tid : c0 + len + (tid - h);
      if (pos < 0 || pos >= b) {
        pos %= b;
        if (pos < 0) pos += b;
      }
      ph = row[pos];
    }
  };
  double acc = 0.0;
  int64_t w = blockIdx.x;
  if (w < nw) fetch(w);
  for (; w < nw; w += gridDim.x) {
    const int64_t n = w / nch, c0 = (w - n * nch) * kCgCH;
    const int len = (int)((b - c0) < kCgCH ? (b - c0) : kCgCH);
    double lm[EPT];
#pragma unroll
    for (int k = 0; k < EPT; ++k) {
      const int i = tid + k * kCgNT;
      if (i < len) tile[h + i] = (double)pm[k];
      lm[k] = mm[k] ? lam : 0.0;
    }
    if (tid < 2 * h) tile[tid < h ? tid : len + tid] = (double)ph;
    for (int t = tid; t < nt; t += kCgNT) cs[t] = autoc[n * nt + t];
    __syncthreads();
    if (w + gridDim.x < nw) fetch(w + gridDim.x);  // in flight during the stencil
#pragma unroll
    for (int k = 0; k < EPT; ++k) {
      const int i = tid + k * kCgNT;
      if (i >= len) continue;
      double v = 0.0;
      for (int t = 0; t < nt; ++t) v += cs[t] * tile[i + t];
      const double pe = tile[i + h];
      v += lm[k] * pe;
      const T vt = T(v);
      q[n * b + c0 + i] = vt;
      acc += pe * (double)vt;
    }
    __syncthreads();  // the next item overwrites the tile
  }
  const double tot = block_sum<kCgNT>(acc, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = tot;
}

// rhs = A^T d + lam D prior
template <typename T>
__global__ __launch_bounds__(kCgNT) void k_cg_rhs_rows(const T* __restrict__ d, T* __restrict__ rhs,
                                                       const double* __restrict__ win,
                                                       const uint32_t* __restrict__ mbits, int64_t bw,
                                                       const T* __restrict__ prior, double lam, int N, int ntap,
                                                       int64_t b, int64_t nrows) {
  __shared__ T tile[kCgCH + 2 * kCgHMAX];
  __shared__ double hs[kCgHMAX + 1];
  const int h = ntap - 1;
  for (int64_t n = blockIdx.x; n < nrows; n += gridDim.x) {
    const T* row = d + n * b;
    __syncthreads();
    for (int r = threadIdx.x; r < ntap; r += kCgNT) hs[r] = win[(int64_t)r * N + n];
    for (int64_t c0 = 0; c0 < b; c0 += kCgCH) {
      const int len = (int)((b - c0) < kCgCH ? (b - c0) : kCgCH);
      cg_stage_row(row, tile, c0, len, h, b);
      __syncthreads();
      for (int i = threadIdx.x; i < len; i += kCgNT) {
        double v = 0.0;
        for (int r = 0; r < ntap; ++r) v += hs[r] * (double)tile[i + h - r];  // d_n[(i - r) mod b]
        const int64_t e = n * b + c0 + i;
        if (mask_bit(mbits, bw, n, c0 + i)) v += lam * (double)prior[e];
        rhs[e] = T(v);
      }
      __syncthreads();
    }
  }
}

// rhs = A^T d + lam D prior : (A^T d)_n[i] = sum_r h[rN+n] d_n[(i-r) mod b]
template <typename T>
__global__ __launch_bounds__(kCgNT) void k_cg_rhs(const T* __restrict__ d, T* __restrict__ rhs,
                                                  const double* __restrict__ win,
                                                  const uint32_t* __restrict__ mbits, int64_t bw,
                                                  const T* __restrict__ prior, double lam, int N, int ntap,
                                                  int64_t b, int64_t S) {
  for (int64_t e = (int64_t)blockIdx.x * kCgNT + threadIdx.x; e < S; e += (int64_t)gridDim.x * kCgNT) {
    const int64_t n = e / b, i = e - n * b;
    const T* row = d + n * b;
    double v = 0.0;
    for (int r = 0; r < ntap; ++r) {
      int64_t k = (i - r) % b;
      if (k < 0) k += b;
      v += win[(int64_t)r * N + n] * (double)row[k];
    }
    if (mask_bit(mbits, bw, n, i)) v += lam * (double)prior[e];
    rhs[e] = T(v);
  }
}

// r = rhs - q ; partial sums of r.r
template <typename T>
__global__ __launch_bounds__(kCgNT) void k_cg_resid(const T* __restrict__ rhs, const T* __restrict__ q,
                                                    T* __restrict__ r, int64_t S, double* __restrict__ part) {
  __shared__ double sh[kCgNT];
  double acc = 0.0;
  for (int64_t e = (int64_t)blockIdx.x * kCgNT + threadIdx.x; e < S; e += (int64_t)gridDim.x * kCgNT) {
    const T v = rhs[e] - q[e];
    r[e] = v;
    acc += (double)v * (double)v;
  }
  const double tot = block_sum<kCgNT>(acc, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = tot;
}

// partial sums of a.b
template <typename T>
__global__ __launch_bounds__(kCgNT) void k_cg_dot(const T* __restrict__ a, const T* __restrict__ c, int64_t S,
                                                  double* __restrict__ part) {
  __shared__ double sh[kCgNT];
  double acc = 0.0;
  for (int64_t e = (int64_t)blockIdx.x * kCgNT + threadIdx.x; e < S; e += (int64_t)gridDim.x * kCgNT)
    acc += (double)a[e] * (double)c[e];
  const double tot = block_sum<kCgNT>(acc, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = tot;
}

// x += alpha p ; r -= alpha q ; partial sums of r.r
template <typename T>
__global__ __launch_bounds__(kCgNT) void k_cg_xr(T* __restrict__ x, T* __restrict__ r, const T* __restrict__ p,
                                                 const T* __restrict__ q, const double* __restrict__ sc, int64_t S,
                                                 double* __restrict__ part) {
  __shared__ double sh[kCgNT];
  const T alpha = T(sc[2]);
  double acc = 0.0;
  for (int64_t e = (int64_t)blockIdx.x * kCgNT + threadIdx.x; e < S; e += (int64_t)gridDim.x * kCgNT) {
    x[e] += alpha * p[e];
    const T v = r[e] - alpha * q[e];
    r[e] = v;
    acc += (double)v * (double)v;
  }
  const double tot = block_sum<kCgNT>(acc, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = tot;
}

// p = z + beta p   (beta from the scalars); first iteration p = z, without
// reading p (the workspace starts uninitialised, and 0 * NaN is NaN)
template <typename T>
__global__ __launch_bounds__(kCgNT) void k_cg_p(T* __restrict__ p, const T* __restrict__ z,
                                                const double* __restrict__ sc, int use_beta, int64_t S) {
  const int64_t e0 = (int64_t)blockIdx.x * kCgNT + threadIdx.x, stride = (int64_t)gridDim.x * kCgNT;
  if (!use_beta) {
    for (int64_t e = e0; e < S; e += stride) p[e] = z[e];
    return;
  }
  const T beta = T(sc[4]);
  for (int64_t e = e0; e < S; e += stride) p[e] = z[e] + beta * p[e];
}

// one workgroup: sum the partials in a fixed order and update the scalars
// sc = [rho, pq, alpha, rho_new, beta, rr]
__global__ __launch_bounds__(kCgNWG) void k_cg_scalar(const double* __restrict__ part, int mode,
                                                      double* __restrict__ sc, double* __restrict__ resid,
                                                      int k) {
  __shared__ double sh[kCgNWG];
  const double tot = block_sum<kCgNWG>(part[threadIdx.x], sh);
  if (threadIdx.x != 0) return;
  switch (mode) {
    case 0:  // rho0 = r.z
      sc[0] = tot;
      break;
    case 1:  // alpha = rho / p.q (an exactly converged system stops moving)
      sc[1] = tot;
      sc[2] = (tot != 0.0) ? sc[0] / tot : 0.0;
      break;
    case 2:  // residual norm
      sc[5] = tot;
      if (resid) resid[k] = sqrt(tot);
      break;
    default:  // beta = rho_new / rho
      sc[3] = tot;
      sc[4] = (sc[0] != 0.0) ? tot / sc[0] : 0.0;
      sc[0] = tot;
      break;
  }
}

// Set-up: the caller's time-order bitmask (bit e of word e/32 is sample
// e = j N + n) to the transposed rows of bw words (bit j of row n). One
// thread per output word; the 64 lanes of a wavefront take 64 neighbouring
// paths of one word column, so each of their 32 reads touches at most two
// input words.
__global__ __launch_bounds__(kCgNT) void k_maskbits_transpose(const uint32_t* __restrict__ in, int N, int64_t b,
                                                              int64_t bw, uint32_t* __restrict__ out) {
  const int64_t total = (int64_t)N * bw;
  for (int64_t t = (int64_t)blockIdx.x * kCgNT + threadIdx.x; t < total; t += (int64_t)gridDim.x * kCgNT) {
    const int64_t jw = t / N;
    const int n = (int)(t - jw * N);
    const int64_t j0 = jw * 32;
    const int nb = (b - j0) < 32 ? (int)(b - j0) : 32;
    uint32_t w = 0;
    for (int k = 0; k < nb; ++k) {
      const int64_t e = (j0 + k) * N + n;
      w |= ((in[e >> 5] >> (e & 31)) & 1u) << k;
    }
    out[(int64_t)n * bw + jw] = w;
  }
}

// ---- natural layout v[j][n] (frame j, sub-filter path n), 4 taps -----------
// The same two stencils run down the columns. A work item is a tile of kCgNT
// consecutive columns and a chunk of kCgFR frames; a thread walks its column
// through the chunk with the stencil's window in registers, so every access
// is a run of kCgNT consecutive samples of one frame and each sample is read
// once per item. Workgroup g takes items g, g + G, ... (G = kCgNWG): the
// partial sums are deterministic. The mask is the time-order bitmask itself
// (bit j N + n), read where the stencil needs it.
constexpr int kCgFR = 64;

__device__ __forceinline__ unsigned nat_bit(const uint32_t* __restrict__ mb, int64_t s) {
  return (mb[s >> 5] >> (s & 31)) & 1u;
}

__device__ __forceinline__ int64_t wrap_frame(int64_t k, int64_t b) {
  if (k < 0 || k >= b) {
    k %= b;
    if (k < 0) k += b;
  }
  return k;
}

// q = (A^T A + lam D) p ; partial sums of p.q
template <typename T, int NTAP>
__global__ __launch_bounds__(kCgNT) void k_cg_normal_nat(const T* __restrict__ p, T* __restrict__ q,
                                                         const double* __restrict__ autoc,
                                                         const uint32_t* __restrict__ mbits, double lam, int N,
                                                         int64_t b, double* __restrict__ part) {
  constexpr int H = NTAP - 1, NC = 2 * NTAP - 1;
  __shared__ double sh[kCgNT];
  const int ntile = (N + kCgNT - 1) / kCgNT;
  const int64_t nw = (int64_t)ntile * ((b + kCgFR - 1) / kCgFR);
  double acc = 0.0;
  for (int64_t w = blockIdx.x; w < nw; w += gridDim.x) {
    const int n = (int)(w % ntile) * kCgNT + threadIdx.x;
    const int64_t j0 = (w / ntile) * kCgFR;
    if (n >= N) continue;
    const int len = (int)(b - j0 < kCgFR ? b - j0 : kCgFR);
    double c[NC], win[NC];  // win[t] = p[j - H + t]
#pragma unroll
    for (int t = 0; t < NC; ++t) c[t] = autoc[(int64_t)n * NC + t];
#pragma unroll
    for (int t = 0; t < NC - 1; ++t) win[t] = (double)p[wrap_frame(j0 - H + t, b) * N + n];
    int64_t jn = wrap_frame(j0 + H, b);  // frame entering the window
#pragma unroll 4
    for (int k = 0; k < len; ++k) {
      win[NC - 1] = (double)p[jn * N + n];
      if (++jn == b) jn = 0;
      double v = 0.0;
#pragma unroll
      for (int t = 0; t < NC; ++t) v += c[t] * win[t];
      const double pe = win[H];
      const int64_t s = (j0 + k) * N + n;
      if (nat_bit(mbits, s)) v += lam * pe;
      const T vt = T(v);
      q[s] = vt;
      acc += pe * (double)vt;
#pragma unroll
      for (int t = 0; t < NC - 1; ++t) win[t] = win[t + 1];
    }
  }
  const double tot = block_sum<kCgNT>(acc, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = tot;
}

// rhs = A^T d + lam D prior : (A^T d)[j][n] = sum_r h[rN+n] d[(j-r) mod b][n]
template <typename T, int NTAP>
__global__ __launch_bounds__(kCgNT) void k_cg_rhs_nat(const T* __restrict__ d, T* __restrict__ rhs,
                                                      const double* __restrict__ win,
                                                      const uint32_t* __restrict__ mbits,
                                                      const T* __restrict__ prior, double lam, int N, int64_t b) {
  const int ntile = (N + kCgNT - 1) / kCgNT;
  const int64_t nw = (int64_t)ntile * ((b + kCgFR - 1) / kCgFR);
  for (int64_t w = blockIdx.x; w < nw; w += gridDim.x) {
    const int n = (int)(w % ntile) * kCgNT + threadIdx.x;
    const int64_t j0 = (w / ntile) * kCgFR;
    if (n >= N) continue;
    const int len = (int)(b - j0 < kCgFR ? b - j0 : kCgFR);
    double h[NTAP], dv[NTAP];  // dv[r] = d[j - r]
#pragma unroll
    for (int r = 0; r < NTAP; ++r) h[r] = win[(int64_t)r * N + n];
#pragma unroll
    for (int r = 1; r < NTAP; ++r) dv[r] = (double)d[wrap_frame(j0 - r, b) * N + n];
#pragma unroll 4
    for (int k = 0; k < len; ++k) {
      const int64_t s = (j0 + k) * N + n;
      dv[0] = (double)d[s];
      double v = 0.0;
#pragma unroll
      for (int r = 0; r < NTAP; ++r) v += h[r] * dv[r];
      if (nat_bit(mbits, s)) v += lam * (double)prior[s];
      rhs[s] = T(v);
#pragma unroll
      for (int r = NTAP - 1; r > 0; --r) dv[r] = dv[r - 1];
    }
  }
}

#define CG_DISPATCH(prec, call) \
  do {                          \
    if ((prec) == F32) {        \
      using T = float;          \
      call;                     \
    } else {                    \
      using T = double;         \
      call;                     \
    }                           \
  } while (0)

hipError_t launch_cg_autocorr(const double* win64, int N, int ntap, double* autoc, hipStream_t st) {
  k_cg_autocorr<<<(N + 255) / 256, 256, 0, st>>>(win64, N, ntap, autoc);
  return hipGetLastError();
}

hipError_t launch_cg_normal(int prec, const void* p, void* q, const double* autoc, const uint32_t* mbits,
                            double lam, int ntap, int64_t b, int64_t S, double* part, hipStream_t st) {
  const int64_t bw = (b + 31) / 32;
  if (ntap - 1 <= kCgHMAX && b > 0)
    CG_DISPATCH(prec, (k_cg_normal_rows<T><<<kCgNWG, kCgNT, 0, st>>>((const T*)p, (T*)q, autoc, mbits, bw, lam,
                                                                   ntap, b, S / b, part)));
  else
    CG_DISPATCH(prec, (k_cg_normal<T><<<kCgNWG, kCgNT, 0, st>>>((const T*)p, (T*)q, autoc, mbits, bw, lam, ntap,
                                                              b, S, part)));
  return hipGetLastError();
}

hipError_t launch_cg_rhs(int prec, const void* d, void* rhs, const double* win64, const uint32_t* mbits,
                         const void* prior, double lam, int N, int ntap, int64_t b, int64_t S, hipStream_t st) {
  const int64_t bw = (b + 31) / 32;
  if (ntap - 1 <= kCgHMAX && b > 0)
    CG_DISPATCH(prec, (k_cg_rhs_rows<T><<<kCgNWG, kCgNT, 0, st>>>((const T*)d, (T*)rhs, win64, mbits, bw,
                                                                (const T*)prior, lam, N, ntap, b, S / b)));
  else
    CG_DISPATCH(prec, (k_cg_rhs<T><<<kCgNWG, kCgNT, 0, st>>>((const T*)d, (T*)rhs, win64, mbits, bw,
                                                             (const T*)prior, lam, N, ntap, b, S)));
  return hipGetLastError();
}

hipError_t launch_cg_resid(int prec, const void* rhs, const void* q, void* r, int64_t S, double* part,
                           hipStream_t st) {
  CG_DISPATCH(prec, (k_cg_resid<T><<<kCgNWG, kCgNT, 0, st>>>((const T*)rhs, (const T*)q, (T*)r, S, part)));
  return hipGetLastError();
}

hipError_t launch_cg_dot(int prec, const void* a, const void* c, int64_t S, double* part, hipStream_t st) {
  CG_DISPATCH(prec, (k_cg_dot<T><<<kCgNWG, kCgNT, 0, st>>>((const T*)a, (const T*)c, S, part)));
  return hipGetLastError();
}

hipError_t launch_cg_xr(int prec, void* x, void* r, const void* p, const void* q, const double* sc, int64_t S,
                        double* part, hipStream_t st) {
  CG_DISPATCH(prec, (k_cg_xr<T><<<kCgNWG, kCgNT, 0, st>>>((T*)x, (T*)r, (const T*)p, (const T*)q, sc, S, part)));
  return hipGetLastError();
}

hipError_t launch_cg_p(int prec, void* p, const void* z, const double* sc, int use_beta, int64_t S,
                       hipStream_t st) {
  CG_DISPATCH(prec, (k_cg_p<T><<<kCgNWG, kCgNT, 0, st>>>((T*)p, (const T*)z, sc, use_beta, S)));
  return hipGetLastError();
}

hipError_t launch_cg_scalar(const double* part, int mode, double* sc, double* resid, int k, hipStream_t st) {
  k_cg_scalar<<<1, kCgNWG, 0, st>>>(part, mode, sc, resid, k);
  return hipGetLastError();
}

hipError_t launch_cg_normal_nat(int prec, const void* p, void* q, const double* autoc, const uint32_t* mbits,
                                double lam, int N, int ntap, int64_t b, double* part, hipStream_t st) {
  if (ntap != 4) return hipErrorNotSupported;
  CG_DISPATCH(prec, (k_cg_normal_nat<T, 4><<<kCgNWG, kCgNT, 0, st>>>((const T*)p, (T*)q, autoc, mbits, lam, N, b,
                                                                     part)));
  return hipGetLastError();
}

hipError_t launch_cg_rhs_nat(int prec, const void* d, void* rhs, const double* win64, const uint32_t* mbits,
                             const void* prior, double lam, int N, int ntap, int64_t b, hipStream_t st) {
  if (ntap != 4) return hipErrorNotSupported;
  CG_DISPATCH(prec, (k_cg_rhs_nat<T, 4><<<kCgNWG, kCgNT, 0, st>>>((const T*)d, (T*)rhs, win64, mbits,
                                                                  (const T*)prior, lam, N, b)));
  return hipGetLastError();
}

hipError_t launch_maskbits_transpose(const uint32_t* in, int N, int64_t b, uint32_t* out, hipStream_t st) {
  k_maskbits_transpose<<<kCgNWG, kCgNT, 0, st>>>(in, N, b, (b + 31) / 32, out);
  return hipGetLastError();
}

}  // namespace ipfb
