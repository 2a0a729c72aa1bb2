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
// re-channelization, N' = 2^18) pack two frames into one complex N'-point
// FFT done in two passes (see below).
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

// ---- long frames: two real frames per complex FFT, four-step L = P1 * P2 ----
// z_q[n] = d_{2q}[n] + i d_{2q+1}[n] (d_j the windowed p-frame sums), with the
// frame index n = a P2 + c (c contiguous in memory).
// Pass 1, per (q, block of MB consecutive c): the polyphase sums for all a of
// both frames (MB-wide loads), P1-point DFTs over a, the twiddle w_L^{c k1};
// writes T[q][k1][c] in MB-wide runs.
// Pass 2, per block of KB rows k1 and their mirrors P1 - k1, looping over a
// range of q: P2-point DFTs along the rows give X[k1 + P1 k2]; the two real
// spectra are split off,
//   Y_{2q}[k] = (X[k] + conj X[L-k]) / 2,  Y_{2q+1}[k] = (X[k] - conj X[L-k]) / 2i,
// written as KB-wide runs, with |Y|^2 summed over the workgroup's q range.
template <typename T, int LOG2P1>
struct Up1Cfg {
  static constexpr int P1 = 1 << LOG2P1;
  static constexpr int MB0 = 131072 / (P1 * (int)sizeof(cx<T>));
  static constexpr int MB = MB0 > 16 ? 16 : MB0;  // consecutive c per workgroup
  static constexpr int LS = lds_len(P1);
  static constexpr int EPT = sizeof(T) == 4 ? 16 : 8;
  static constexpr int NT0 = (P1 * MB) / EPT;
  static constexpr int NT = NT0 > 1024 ? 1024 : NT0;
};

// Small twiddle tables of a long-frame plan (all e^{-2 pi i m / len}):
// tP1 [P1], tP2 [P2], and w_L^m = tHi[m >> 9] * tLo[m & 511] (tLo: m < 512,
// tHi: multiples of 512). Kept small so that lookups stay in L1.
template <typename T>
struct LongTw {
  const cx<T>* tP1;
  const cx<T>* tP2;
  const cx<T>* tLo;
  const cx<T>* tHi;
};

template <typename T>
__device__ __forceinline__ cx<T> tw_long(const LongTw<T>& t, int64_t m) {
  return cmul(t.tHi[m >> 9], t.tLo[m & 511]);
}

template <typename T, int LOG2P1>
__global__ __launch_bounds__((Up1Cfg<T, LOG2P1>::NT)) void k_up1(
    const T* __restrict__ x, cx<T>* __restrict__ tmp, int64_t nblock, int ntap, const T* __restrict__ win,
    LongTw<T> tw, int L, int P2, int64_t nq) {
  using Cfg = Up1Cfg<T, LOG2P1>;
  constexpr int P1 = Cfg::P1, MB = Cfg::MB, LS = Cfg::LS, NT = Cfg::NT;
  __shared__ cx<T> s[MB * LS];
  const int tid = threadIdx.x;
  const int ncb = P2 / MB;
  const int64_t lg = xcd_remap(blockIdx.x, (int)(nq * ncb));
  const int64_t q = lg / ncb;
  const int c0 = (int)(lg % ncb) * MB;  // neighbouring column blocks share an XCD
  const int64_t j0 = 2 * q;
  const bool has1 = (j0 + 1) < nblock;
  for (int e = tid; e < P1 * MB; e += NT) {
    const int mb = e % MB, a = e / MB;
    const int64_t n = (int64_t)a * P2 + c0 + mb;
    T d0 = T(0), d1 = T(0), wprev = T(0);
    for (int r = 0; r <= ntap; ++r) {  // frames 2q .. 2q+p feed both sums
      int64_t f = j0 + r;
      if (f >= nblock) f %= nblock;
      const T xv = x[f * L + n];
      if (has1 && r >= 1) d1 += wprev * xv;
      if (r < ntap) {
        wprev = win[(int64_t)r * L + n];
        d0 += wprev * xv;
      }
    }
    s[mb * LS + pidx(a)] = mk<T>(d0, d1);
  }
  __syncthreads();
  lds_fft<T, P1, NT, MB, -1>(s, LS, tw.tP1, 1);
  cx<T>* tq = tmp + q * (int64_t)L;
  for (int e = tid; e < P1 * MB; e += NT) {
    const int mb = e % MB, k1 = e / MB;
    const int c = c0 + mb;
    tq[(int64_t)k1 * P2 + c] = cmul(s[mb * LS + pidx(k1)], tw_long(tw, (int64_t)c * k1));
  }
}

// Pass 1 for a fixed tap count: one workgroup per block of MB columns slides
// over a range of frame pairs, keeping the last frames of its columns in
// registers, so each pair loads only its two new frames (the windowed sums of
// Section 2.3's sliding window, each input sample read once per workgroup;
// the window slice is re-read from cache).
template <typename T, int LOG2P1>
struct Up1sCfg {
  static constexpr int P1 = 1 << LOG2P1;
  static constexpr int MB = 16;
  static constexpr int LS = lds_len(P1);
  static constexpr int NT = 1024;
  static constexpr int EPT = (P1 * MB) / NT;  // elements (a, c) per thread: a = tid/MB + i*(NT/MB)
};

template <typename T, int LOG2P1, int NTAP>
__global__ __launch_bounds__((Up1sCfg<T, LOG2P1>::NT)) void k_up1_slide(
    const T* __restrict__ x, cx<T>* __restrict__ tmp, int64_t nblock, const T* __restrict__ win,
    LongTw<T> tw, int L, int P2, int64_t nq, int qrange) {
  using Cfg = Up1sCfg<T, LOG2P1>;
  constexpr int P1 = Cfg::P1, MB = Cfg::MB, LS = Cfg::LS, NT = Cfg::NT, EPT = Cfg::EPT;
  __shared__ cx<T> s[MB * LS];
  const int tid = threadIdx.x;
  const int ncb = P2 / MB;
  // neighbouring column blocks (the two halves of each 128-byte line) share an XCD
  const int lg = xcd_remap(blockIdx.x, (int)gridDim.x);
  const int cb = lg % ncb;
  const int64_t qa = (int64_t)(lg / ncb) * qrange;
  const int64_t qb = (qa + qrange < nq) ? qa + qrange : nq;
  const int c0 = cb * MB;
  // sample offset of element i within a frame: off0 + i * (NT/MB) * P2
  const int off0 = (tid / MB) * P2 + c0 + (tid % MB);
  const int ostep = (NT / MB) * P2;
  T h[NTAP + 1][EPT];  // frames 2q .. 2q+NTAP of this thread's samples
  auto frame = [&](int64_t f) -> int64_t { return (f < nblock ? f : f % nblock) * (int64_t)L; };
  if (qa < qb) {
#pragma unroll
    for (int r = 0; r <= NTAP; ++r) {
      const int64_t fo = frame(2 * qa + r);
#pragma unroll
      for (int i = 0; i < EPT; ++i) h[r][i] = x[fo + off0 + i * ostep];
    }
  }
  for (int64_t q = qa; q < qb; ++q) {
    const bool has1 = (2 * q + 1) < nblock;
#pragma unroll
    for (int i = 0; i < EPT; ++i) {
      T d0 = T(0), d1 = T(0);
#pragma unroll
      for (int r = 0; r < NTAP; ++r) {
        const T wr = win[(int64_t)r * L + off0 + i * ostep];
        d0 += wr * h[r][i];
        d1 += wr * h[r + 1][i];
      }
      if (!has1) d1 = T(0);
      const int e = tid + i * NT;
      s[(e % MB) * LS + pidx(e / MB)] = mk<T>(d0, d1);
    }
    // slide: frames 2q+2 .. 2q+NTAP stay; the two new ones load after the FFT
#pragma unroll
    for (int r = 0; r + 2 <= NTAP; ++r)
#pragma unroll
      for (int i = 0; i < EPT; ++i) h[r][i] = h[r + 2][i];
    __syncthreads();
    lds_fft<T, P1, NT, MB, -1>(s, LS, tw.tP1, 1);
    cx<T>* tq = tmp + q * (int64_t)L;
    if (q + 1 < qb) {
      const int64_t fa = frame(2 * q + NTAP + 1), fb = frame(2 * q + NTAP + 2);
#pragma unroll
      for (int i = 0; i < EPT; ++i) {
        h[NTAP - 1][i] = x[fa + off0 + i * ostep];
        h[NTAP][i] = x[fb + off0 + i * ostep];
      }
    }
    for (int e = tid; e < P1 * MB; e += NT) {
      const int mb = e % MB, k1 = e / MB;
      const int c = c0 + mb;
      tq[(int64_t)k1 * P2 + c] = cmul(s[mb * LS + pidx(k1)], tw_long(tw, (int64_t)c * k1));
    }
    __syncthreads();
  }
}

template <typename T, int LOG2P2>
struct Up2Cfg {
  static constexpr int P2 = 1 << LOG2P2;
  static constexpr int KB0 = 65536 / (2 * P2 * (int)sizeof(cx<T>));
  static constexpr int KB = KB0 > 16 ? 16 : (KB0 < 1 ? 1 : KB0);  // rows per half (two workgroups per CU)
  static constexpr int LS = lds_len(P2);
  static constexpr int EPT = sizeof(T) == 4 ? 16 : 8;
  static constexpr int NT0 = (2 * KB * P2) / EPT;
  static constexpr int NT = NT0 > 1024 ? 1024 : NT0;
  static constexpr int NOUT = 2 * KB * (P2 / 2 + 1);  // outputs per q
  static constexpr int OPT = (NOUT + NT - 1) / NT;     // outputs per thread
};

template <typename T, int LOG2P2>
__global__ __launch_bounds__((Up2Cfg<T, LOG2P2>::NT), 4) void k_up2(
    const cx<T>* __restrict__ tmp, cx<T>* __restrict__ y, const cx<T>* __restrict__ tP2, int L, int P1,
    int64_t nblock, int64_t nq, int qchunk, int npb, double* __restrict__ part) {
  using Cfg = Up2Cfg<T, LOG2P2>;
  constexpr int P2 = Cfg::P2, KB = Cfg::KB, LS = Cfg::LS, NT = Cfg::NT;
  constexpr int NOUT = Cfg::NOUT, OPT = Cfg::OPT;
  __shared__ cx<T> s[2 * KB * LS];
  const int tid = threadIdx.x;
  const int K = L / 2 + 1;
  const int lg = xcd_remap(blockIdx.x, (int)gridDim.x);  // adjacent row blocks write the same lines
  const int w = lg % npb;
  const int qc = lg / npb;
  const bool special = (w == npb - 1);
  const int r0 = 1 + w * KB;
  const int count = special ? 1 : min(KB, P1 / 2 - r0);
  // slot (half, i): half 0 holds rows r0+i, half 1 their mirrors P1-r0-i; the
  // special workgroup holds the self-paired rows 0 and P1/2.
  auto row_of = [&](int half, int i) -> int {
    if (special) return half == 0 ? 0 : P1 / 2;
    return half == 0 ? r0 + i : P1 - r0 - i;
  };
  double acc[OPT];
#pragma unroll
  for (int o = 0; o < OPT; ++o) acc[o] = 0.0;
  const int64_t qa = (int64_t)qc * qchunk;
  const int64_t qb = (qa + qchunk < nq) ? qa + qchunk : nq;
  for (int64_t q = qa; q < qb; ++q) {
    const cx<T>* tq = tmp + q * (int64_t)L;
    for (int e = tid; e < 2 * KB * P2; e += NT) {
      const int sl = e / P2, c = e % P2;
      const int half = sl / KB, i = sl % KB;
      cx<T> v = mk<T>(T(0), T(0));
      if (i < count) v = tq[(int64_t)row_of(half, i) * P2 + c];
      s[sl * LS + pidx(c)] = v;
    }
    __syncthreads();
    lds_fft<T, P2, NT, 2 * KB, -1>(s, LS, tP2, 1);
    const bool has1 = (2 * q + 1) < nblock;
    cx<T>* y0 = y + (2 * q) * (int64_t)K;
    cx<T>* y1 = y0 + K;
#pragma unroll
    for (int o = 0; o < OPT; ++o) {
      const int e = tid + o * NT;
      if (e >= NOUT) continue;
      const int i = e % KB, t = e / KB;
      const int half = t & 1, k2 = t >> 1;  // k2 in [0, P2/2]
      if (i >= count) continue;
      const int k1 = row_of(half, i);
      if (k2 == P2 / 2 && k1 != 0) continue;  // only the Nyquist bin has k2 = P2/2
      const int sl = half * KB + i;
      int psl, pk2;
      if (k1 == 0) {
        psl = sl;
        pk2 = (P2 - k2) & (P2 - 1);
      } else if (special) {  // row P1/2 pairs with itself
        psl = sl;
        pk2 = P2 - 1 - k2;
      } else {
        psl = (1 - half) * KB + i;
        pk2 = P2 - 1 - k2;
      }
      const cx<T> zk = s[sl * LS + pidx(k2)];
      const cx<T> zm = conj(s[psl * LS + pidx(pk2)]);
      const cx<T> u = mk<T>(T(0.5) * (zk.x + zm.x), T(0.5) * (zk.y + zm.y));
      const cx<T> dv = mk<T>(T(0.5) * (zk.x - zm.x), T(0.5) * (zk.y - zm.y));
      const cx<T> v = mk<T>(dv.y, -dv.x);  // dv / i
      const int64_t k = (int64_t)k1 + (int64_t)P1 * k2;
      y0[k] = u;
      double pw = (double)u.x * (double)u.x + (double)u.y * (double)u.y;
      if (has1) {
        y1[k] = v;
        pw += (double)v.x * (double)v.x + (double)v.y * (double)v.y;
      }
      acc[o] += pw;
    }
    __syncthreads();
  }
  if (part) {
#pragma unroll
    for (int o = 0; o < OPT; ++o) {
      const int e = tid + o * NT;
      if (e >= NOUT) continue;
      const int i = e % KB, t = e / KB;
      const int half = t & 1, k2 = t >> 1;
      if (i >= count) continue;
      const int k1 = row_of(half, i);
      if (k2 == P2 / 2 && k1 != 0) continue;
      part[(int64_t)qc * K + (int64_t)k1 + (int64_t)P1 * k2] = acc[o];
    }
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

template <typename T>
static LongTw<T> long_tw(const void* twS, int P1, int P2, int L) {
  const cx<T>* b = (const cx<T>*)twS;
  LongTw<T> t;
  t.tP1 = b;
  t.tP2 = b + P1;
  t.tLo = b + P1 + P2;
  t.tHi = b + P1 + P2 + 512;
  (void)L;
  return t;
}

template <typename T, int L1>
static hipError_t launch_up1_t(const void* x, void* tmp, int64_t nblock, int ntap, const void* winT,
                               const LongTw<T>& tw, int L, int P2, int64_t nq, hipStream_t st) {
  using Cfg = Up1Cfg<T, L1>;
  const int64_t grid = nq * (P2 / Cfg::MB);
  k_up1<T, L1><<<dim3((unsigned)grid), dim3(Cfg::NT), 0, st>>>(
      (const T*)x, (cx<T>*)tmp, nblock, ntap, (const T*)winT, tw, L, P2, nq);
  return hipGetLastError();
}

template <typename T, int L2>
static hipError_t launch_up2_t(const void* tmp, void* y, const LongTw<T>& tw, int L, int P1, int64_t nblock,
                               int64_t nq, int qchunk, double* part, hipStream_t st) {
  using Cfg = Up2Cfg<T, L2>;
  const int npb = (P1 / 2 - 1 + Cfg::KB - 1) / Cfg::KB + 1;
  const int64_t nqc = (nq + qchunk - 1) / qchunk;
  k_up2<T, L2><<<dim3((unsigned)(npb * nqc)), dim3(Cfg::NT), 0, st>>>(
      (const cx<T>*)tmp, (cx<T>*)y, tw.tP2, L, P1, nblock, nq, qchunk, npb, part);
  return hipGetLastError();
}

template <typename T, int L1>
static hipError_t launch_up1s_t(const void* x, void* tmp, int64_t nblock, const void* winT, const LongTw<T>& tw,
                                int L, int P2, int64_t nq, hipStream_t st) {
  using Cfg = Up1sCfg<T, L1>;
  const int ncb = P2 / Cfg::MB;
  // enough workgroups to cover the CUs twice, each sliding over >= 4 pairs
  int64_t nr = (512 + ncb - 1) / ncb;
  if (nr > (nq + 3) / 4) nr = (nq + 3) / 4;
  if (nr < 1) nr = 1;
  const int qrange = (int)((nq + nr - 1) / nr);
  nr = (nq + qrange - 1) / qrange;
  k_up1_slide<T, L1, 4><<<dim3((unsigned)(ncb * nr)), dim3(Cfg::NT), 0, st>>>(
      (const T*)x, (cx<T>*)tmp, nblock, (const T*)winT, tw, L, P2, nq, qrange);
  return hipGetLastError();
}

template <typename T>
static hipError_t launch_large_t(int log2n, const void* x, void* y, int64_t nblock, int ntap, const void* winT,
                                 const void* twS, void* tmp, int qchunk, double* part, hipStream_t st) {
  if (nblock == 0) return hipSuccess;
  const int L = 1 << log2n;
  const int l1 = (log2n + 1) / 2, l2 = log2n / 2;
  const int P1 = 1 << l1, P2 = 1 << l2;
  const int64_t nq = (nblock + 1) / 2;
  const LongTw<T> tw = long_tw<T>(twS, P1, P2, L);
  hipError_t e;
  if (ntap == 4 && (l1 == 8 || l1 == 9) && nblock >= 4) {
    e = (l1 == 8) ? launch_up1s_t<T, 8>(x, tmp, nblock, winT, tw, L, P2, nq, st)
                  : launch_up1s_t<T, 9>(x, tmp, nblock, winT, tw, L, P2, nq, st);
  } else switch (l1) {
    case 8: e = launch_up1_t<T, 8>(x, tmp, nblock, ntap, winT, tw, L, P2, nq, st); break;
    case 9: e = launch_up1_t<T, 9>(x, tmp, nblock, ntap, winT, tw, L, P2, nq, st); break;
    case 10: e = launch_up1_t<T, 10>(x, tmp, nblock, ntap, winT, tw, L, P2, nq, st); break;
    default: return hipErrorInvalidValue;
  }
  if (e != hipSuccess) return e;
  switch (l2) {
    case 7: return launch_up2_t<T, 7>(tmp, y, tw, L, P1, nblock, nq, qchunk, part, st);
    case 8: return launch_up2_t<T, 8>(tmp, y, tw, L, P1, nblock, nq, qchunk, part, st);
    case 9: return launch_up2_t<T, 9>(tmp, y, tw, L, P1, nblock, nq, qchunk, part, st);
    case 10: return launch_up2_t<T, 10>(tmp, y, tw, L, P1, nblock, nq, qchunk, part, st);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_pfb_fwd_large(int prec, int log2n, const void* x, void* y, int64_t nblock, int ntap,
                                const void* winT, const void* twS, void* tmp, int qchunk, double* part,
                                hipStream_t st) {
  if (prec == F32) return launch_large_t<float>(log2n, x, y, nblock, ntap, winT, twS, tmp, qchunk, part, st);
  return launch_large_t<double>(log2n, x, y, nblock, ntap, winT, twS, tmp, qchunk, part, st);
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
