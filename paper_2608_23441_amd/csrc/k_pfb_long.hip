// Forward PFB for long frames (Section 2.2's polyphase sum and FFT, applied at
// the up-channelized frame length N' = u N of Section 4.3; the fused
// autospectrum is Section 4.1's error metric).
//
// A real frame v_j of length L (the windowed p-frame sum) is packed as the
// complex sequence z[m] = v_j[2m] + i v_j[2m+1] of length M = L/2, so each
// output spectrum costs one M-point complex FFT:
//   E[k] = (Z[k] + conj Z[M-k]) / 2,  O[k] = (Z[k] - conj Z[M-k]) / (2i),
//   Y[k] = E[k] + t,  Y[M-k] = conj(E[k] - t),  t = e^{-2 pi i k/L} O[k].
// The M-point FFT is four-step, M = P1 * P2 (FP32: P1 = P2 / 2 for odd log2 M),
// m = P2 a + c, k = k1 + P1 k2:
//   pass 1, per block of MB consecutive c and one frame: the windowed sums
//     for all a (each load a 128-byte run of one frame), the P1-point FFT
//     over a, the twiddle e^{-2 pi i c k1 / M}; T[j][k1][c] written as
//     128-byte runs. Neighbouring frames of one column block run on one XCD,
//     so the p reads of each input frame and of the window meet in its L2.
//   pass 2, per group of KB rows k1 with their mirrors P1 - k1 and a range of
//     frames: the P2-point FFT along each row gives Z[k1 + P1 k2]; every pair
//     (k, M - k) meets in one workgroup, which writes Y[k] and Y[M-k] as
//     KB-wide runs and sums |Y|^2 over its frames in FP64.
#include "fft_lds.hpp"
#include "launch.hpp"

namespace ipfb {

// Twiddle tables of a long-frame plan, all e^{-2 pi i m / len} (FP64-built,
// rounded once for FP32): tP1 [P1], tP2 [P2]; e^{-2 pi i m / M} =
// tMhi[m >> 9] * tMlo[m & 511]; e^{-2 pi i k / L} = tLhi[k >> 9] * tLlo[k & 511]
// for k in [0, M]. Small enough to stay in L1/L2.
template <typename T>
struct LfTw {
  const cx<T>* tP1;
  const cx<T>* tP2;
  const cx<T>* tMlo;
  const cx<T>* tMhi;
  const cx<T>* tLlo;
  const cx<T>* tLhi;
};

template <typename T>
__device__ __forceinline__ cx<T> tw2(const cx<T>* __restrict__ lo, const cx<T>* __restrict__ hi, int m) {
  return cmul(hi[m >> 9], lo[m & 511]);
}

template <typename T, int LOG2P1>
struct Lf1Cfg {
  static constexpr int P1 = 1 << LOG2P1;
  static constexpr int MB0 = 128 / (int)sizeof(cx<T>);    // 128-byte runs
  static constexpr int MBC = 8192 / P1;                    // keep P1 * MB <= 8192 elements
  static constexpr int MB = MB0 < MBC ? MB0 : (MBC < 1 ? 1 : MBC);
  static constexpr int EPT0 = sizeof(T) == 4 ? 16 : 8;
  static constexpr int NT0 = (P1 * MB) / EPT0;
  static constexpr int NT = NT0 < 64 ? 64 : (NT0 > 1024 ? 1024 : NT0);
  static constexpr int EPT = (P1 * MB) / NT;  // complex elements per thread
  static constexpr int LS = lds_len(P1);
};

// Pass 1, one output frame j and one column block per workgroup. Workgroups
// that share an XCD take the same column block and consecutive frames, so the
// window slice and each input frame (read by NTAP consecutive outputs) are
// served from that XCD's L2 after the first touch. NTAP > 0: tap count fixed
// at compile time (loads batched); NTAP == 0: any tap count.
template <typename T, int LOG2P1, int NTAP>
__global__ __launch_bounds__((Lf1Cfg<T, LOG2P1>::NT), 2) void k_lf1(
    const cx<T>* __restrict__ x, cx<T>* __restrict__ tmp, int64_t nblock, int ntap,
    const cx<T>* __restrict__ win, LfTw<T> tw, int M, int P2) {
  using Cfg = Lf1Cfg<T, LOG2P1>;
  constexpr int P1 = Cfg::P1, MB = Cfg::MB, NT = Cfg::NT, EPT = Cfg::EPT, LS = Cfg::LS;
  static_assert(EPT >= 1 && (P1 * MB) % NT == 0, "pass-1 tile must split evenly over the threads");
  __shared__ cx<T> s[MB * LS];
  const int tid = threadIdx.x;
  const int64_t lg = xcd_remap(blockIdx.x, (int)gridDim.x);
  const int cb = (int)(lg / nblock);
  const int64_t j = lg % nblock;
  const int c0 = cb * MB;
  // element i of this thread: column c0 + tid % MB, row a = tid / MB + i * (NT / MB)
  const int off0 = (tid / MB) * P2 + c0 + (tid % MB);
  constexpr int ASTEP = NT / MB;
  auto frame_off = [&](int64_t f) -> int64_t {
    while (f >= nblock) f -= nblock;
    return f * (int64_t)M;
  };
  const int nt = NTAP > 0 ? NTAP : ntap;
#pragma unroll
  for (int i = 0; i < EPT; ++i) {
    const int64_t o = off0 + (int64_t)i * ASTEP * P2;
    cx<T> acc = mk<T>(T(0), T(0));
#pragma unroll
    for (int r = 0; r < (NTAP > 0 ? NTAP : 1); ++r) {
      if (NTAP == 0) break;
      const cx<T> w = win[(int64_t)r * M + o];
      const cx<T> v = x[frame_off(j + r) + o];
      acc.x += w.x * v.x;
      acc.y += w.y * v.y;
    }
    if (NTAP == 0) {
      for (int r = 0; r < nt; ++r) {
        const cx<T> w = win[(int64_t)r * M + o];
        const cx<T> v = x[frame_off(j + r) + o];
        acc.x += w.x * v.x;
        acc.y += w.y * v.y;
      }
    }
    const int e = tid + i * NT;
    s[(e % MB) * LS + pidx(e / MB)] = acc;
  }
  __syncthreads();
  lds_fft<T, P1, NT, MB, -1>(s, LS, tw.tP1, 1);
  cx<T>* tj = tmp + j * (int64_t)M;
#pragma unroll
  for (int i = 0; i < EPT; ++i) {
    const int e = tid + i * NT;
    const int mb = e % MB, k1 = e / MB;
    const int c = c0 + mb;
    tj[(int64_t)k1 * P2 + c] = cmul(s[mb * LS + pidx(k1)], tw2(tw.tMlo, tw.tMhi, c * k1));
  }
}

// Pass 1, sliding form (4 taps, P1 <= 512): one workgroup per column block
// (128 or 64 bytes of columns, see below) and a range of frames. The
// window slice and the four frames of the sliding sum stay in registers (each
// input sample is loaded once per workgroup, the window once), and the next
// frame is fetched while the FFT of the current one runs.
template <typename T, int LOG2P1>
struct Lf1rCfg {
  static constexpr int P1 = 1 << LOG2P1;
  // 512 threads (two waves per SIMD, room for the ring and the window slice in
  // registers). Columns per block: 128-byte runs for P1 <= 256 (FP32: 8
  // elements per thread at P1 = 256), 64-byte runs at P1 = 512, where the
  // four frames and four window taps of 16 columns would not fit the
  // registers (FP32 then also holds 8 elements per thread)
  static constexpr int MB = (LOG2P1 <= 8 ? 128 : 64) / (int)sizeof(cx<T>);
  static constexpr int NT = 512;
  static constexpr int EPT = (P1 * MB) / NT;
  static constexpr int LS = lds_len(P1);
};

template <typename T, int LOG2P1>
__global__ __launch_bounds__((Lf1rCfg<T, LOG2P1>::NT)) void k_lf1r(const cx<T>* __restrict__ x,
                                                                  cx<T>* __restrict__ tmp, int64_t nblock,
                                                                  const cx<T>* __restrict__ win, LfTw<T> tw,
                                                                  int M, int P2, int nr, int frange) {
  using Cfg = Lf1rCfg<T, LOG2P1>;
  constexpr int P1 = Cfg::P1, MB = Cfg::MB, NT = Cfg::NT, EPT = Cfg::EPT, LS = Cfg::LS;
  constexpr int NTAP = 4;
  static_assert(EPT >= 1 && EPT <= 8, "register budget: 4 frames + 4 window taps of EPT elements");
  // two frame buffers, alternating by frame: the next frame's sums go to the
  // other buffer while slower threads still read this one for their stores
  __shared__ cx<T> sbuf[2 * MB * LS];
  // the twiddle tables live in LDS for the life of the workgroup: every FFT
  // pass and store then waits on LDS, not on global-memory latency
  // M = P1 * P2 <= 2 P1^2, so e^{-2 pi i 512 m / M} needs at most 2 P1^2 / 512 entries
  constexpr int NHI = (2 * P1 * P1) / 512 > 0 ? (2 * P1 * P1) / 512 : 1;
  __shared__ cx<T> tP1s[P1], tMlos[512], tMhis[NHI];
  const int tid = threadIdx.x;
  const int lg = xcd_remap(blockIdx.x, (int)gridDim.x);
  const int cb = lg / nr, rg = lg % nr;
  const int c0 = cb * MB;
  const int64_t ja = (int64_t)rg * frange;
  const int64_t jb = (ja + frange < nblock) ? ja + frange : nblock;
  if (ja >= jb) return;
  for (int i = tid; i < P1; i += NT) tP1s[i] = tw.tP1[i];
  for (int i = tid; i < 512; i += NT) tMlos[i] = tw.tMlo[i];
  for (int i = tid; i < (M >> 9); i += NT) tMhis[i] = tw.tMhi[i];
  const int off0 = (tid / MB) * P2 + c0 + (tid % MB);
  constexpr int ASTEP = NT / MB;
  // frames wrap once at most (nblock >= NTAP): f < nblock + NTAP
  auto frame_off = [&](int64_t f) -> int64_t { return (f < nblock ? f : f - nblock) * (int64_t)M; };
  cx<T> w[NTAP][EPT], ring[NTAP][EPT];
#pragma unroll
  for (int r = 0; r < NTAP; ++r) {
    const int64_t fo = frame_off(ja + r);
#pragma unroll
    for (int i = 0; i < EPT; ++i) {
      w[r][i] = win[(int64_t)r * M + off0 + i * ASTEP * P2];
      ring[r][i] = x[fo + off0 + i * ASTEP * P2];
    }
  }
  // element i of this thread is row a = tid / MB + i NT / MB of column
  // tid % MB: when a thread holds EPT = R0 elements these are exactly the
  // inputs of first-pass butterfly tid / MB, which then runs in registers
  using F = FftSplit<T, P1, NT, MB>;
  constexpr bool FIRST_IN_REGS = F::ok && F::R0 == EPT;
  for (int64_t j = ja; j < jb; ++j) {
    cx<T>* s = sbuf + ((j - ja) & 1) * (MB * LS);
    cx<T> v[EPT];
#pragma unroll
    for (int i = 0; i < EPT; ++i) {
      cx<T> acc = mk<T>(T(0), T(0));
#pragma unroll
      for (int r = 0; r < NTAP; ++r) {
        acc.x += w[r][i].x * ring[r][i].x;
        acc.y += w[r][i].y * ring[r][i].y;
      }
      v[i] = acc;
    }
    if constexpr (FIRST_IN_REGS) {
      fft_first_from_regs<T, EPT, -1>(s + (tid % MB) * LS, tid / MB, v);
    } else {
#pragma unroll
      for (int i = 0; i < EPT; ++i) {
        const int e = tid + i * NT;
        s[(e % MB) * LS + pidx(e / MB)] = v[i];
      }
    }
    // slide by one frame; frame j + NTAP loads while the FFT runs
#pragma unroll
    for (int r = 0; r + 1 < NTAP; ++r)
#pragma unroll
      for (int i = 0; i < EPT; ++i) ring[r][i] = ring[r + 1][i];
    if (j + 1 < jb) {
      const int64_t fo = frame_off(j + NTAP);
#pragma unroll
      for (int i = 0; i < EPT; ++i) ring[NTAP - 1][i] = x[fo + off0 + i * ASTEP * P2];
    }
    __syncthreads();
    if constexpr (FIRST_IN_REGS) fft_rest<T, P1, NT, MB, -1>(s, LS, tP1s, 1);
    else lds_fft<T, P1, NT, MB, -1>(s, LS, tP1s, 1);
    cx<T>* tj = tmp + j * (int64_t)M;
#pragma unroll
    for (int i = 0; i < EPT; ++i) {
      const int e = tid + i * NT;
      const int mb = e % MB, k1 = e / MB;
      const int c = c0 + mb;
      tj[(int64_t)k1 * P2 + c] = cmul(s[mb * LS + pidx(k1)], tw2(tMlos, tMhis, c * k1));
    }
    // no barrier: frame j + 1 writes the other buffer, and frame j + 2 writes
    // this one only after the barriers of frame j + 1, which every thread
    // reaches after its reads above
  }
}

template <typename T, int LOG2P2>
struct Lf2Cfg {
  static constexpr int P2 = 1 << LOG2P2;
  static constexpr int KB0 = 128 / (int)sizeof(cx<T>);           // 128-byte output runs
  static constexpr int KBC = 65536 / (2 * P2 * (int)sizeof(cx<T>));  // LDS tile <= 64 KiB
  static constexpr int KB = KB0 < KBC ? KB0 : (KBC < 1 ? 1 : KBC);
  static constexpr int EPT0 = 8;
  static constexpr int NT0 = (2 * KB * P2) / EPT0;
  static constexpr int NT = NT0 < 64 ? 64 : (NT0 > 1024 ? 1024 : NT0);
  static constexpr int EPT = (2 * KB * P2) / NT;      // tile elements per thread
  static constexpr int LS = lds_len(P2);
  static constexpr int NI = KB * P2 > P2 + 1 ? KB * P2 : P2 + 1;  // items (pairs) of the largest group
  static constexpr int IPT = (NI + NT - 1) / NT;                   // items per thread
};

// Pass 2. Workgroup kind: w < ngrp: rows r0 + i (half 0) and P1 - r0 - i
// (half 1), r0 = 1 + KB w, i < count; w == ngrp: the self-mirrored rows 0 and
// P1/2. Each workgroup loops over a chunk of frames, fetching the rows of the
// next frame into registers while the current one is transformed. part: NULL,
// or [nchunks][M+1] FP64 sums of |Y|^2 per frame chunk.
template <typename T, int LOG2P2>
__global__ __launch_bounds__((Lf2Cfg<T, LOG2P2>::NT)) void k_lf2(
    const cx<T>* __restrict__ tmp, cx<T>* __restrict__ y, LfTw<T> tw, int M, int P1, int64_t nblock,
    int fchunk, int ngrp, double* __restrict__ part) {
  using Cfg = Lf2Cfg<T, LOG2P2>;
  constexpr int P2 = Cfg::P2, KB = Cfg::KB, NT = Cfg::NT, LS = Cfg::LS, IPT = Cfg::IPT, EPT = Cfg::EPT;
  static_assert((2 * KB * P2) % NT == 0, "pass-2 tile must split evenly over the threads");
  __shared__ cx<T> s[2 * KB * LS];
  // twiddles, LDS-resident; M = P1 * P2 <= 2 P2^2, so k >> 9 <= 2 P2^2 / 512
  constexpr int NHI = (2 * P2 * P2) / 512 + 1;
  __shared__ cx<T> tP2s[P2], tLlos[512], tLhis[NHI];
  const int tid = threadIdx.x;
  const int K = M + 1;  // output bins per frame
  for (int i = tid; i < P2; i += NT) tP2s[i] = tw.tP2[i];
  for (int i = tid; i < 512; i += NT) tLlos[i] = tw.tLlo[i];
  for (int i = tid; i <= (M >> 9); i += NT) tLhis[i] = tw.tLhi[i];
  const int lg = xcd_remap(blockIdx.x, (int)gridDim.x);  // neighbouring groups write neighbouring runs
  const int w = lg % (ngrp + 1);
  const int ch = lg / (ngrp + 1);
  const bool special = (w == ngrp);
  const int r0 = 1 + w * KB;
  const int count = special ? 1 : min(KB, P1 / 2 - r0);
  auto row_of = [&](int half, int i) -> int {
    if (special) return half == 0 ? 0 : P1 / 2;
    return half == 0 ? r0 + i : P1 - r0 - i;
  };
  // items: regular group, e = i + KB k2 (i < count): row r0 + i at k2 with its
  // mirror (half 1, slot i) at P2-1-k2. Special group: e <= P2/2: row 0 at
  // k2 = e, mirror (P2 - e) mod P2; P2/2 < e <= P2: row P1/2 at k2 = e-P2/2-1,
  // mirror P2-1-k2.
  const int nitems = special ? P2 + 1 : KB * P2;
  double acc0[IPT], acc1[IPT];
#pragma unroll
  for (int o = 0; o < IPT; ++o) acc0[o] = acc1[o] = 0.0;
  const int64_t ja = (int64_t)ch * fchunk;
  const int64_t jb = (ja + fchunk < nblock) ? ja + fchunk : nblock;
  // tile element i of this thread: slot sl = e / P2, column c = e % P2
  cx<T> pf[EPT];
  auto fetch = [&](int64_t j) {
    const cx<T>* tj = tmp + j * (int64_t)M;
#pragma unroll
    for (int i = 0; i < EPT; ++i) {
      const int e = tid + i * NT;
      const int sl = e / P2, c = e % P2;
      const int half = sl / KB, q = sl % KB;
      pf[i] = mk<T>(T(0), T(0));
      if (q < count) pf[i] = ld_once(tj + (int64_t)row_of(half, q) * P2 + c);
    }
  };
  if (ja < jb) fetch(ja);
  for (int64_t j = ja; j < jb; ++j) {
#pragma unroll
    for (int i = 0; i < EPT; ++i) {
      const int e = tid + i * NT;
      s[(e / P2) * LS + pidx(e % P2)] = pf[i];
    }
    __syncthreads();
    if (j + 1 < jb) fetch(j + 1);  // in flight during the FFT and the stores
    lds_fft<T, P2, NT, 2 * KB, -1>(s, LS, tP2s, 1);
    cx<T>* yj = y + j * (int64_t)K;
#pragma unroll
    for (int o = 0; o < IPT; ++o) {
      const int e = tid + o * NT;
      if (e >= nitems) continue;
      int sl, k2, psl, pk2, k1;
      if (!special) {
        const int i = e % KB;
        if (i >= count) continue;
        k2 = e / KB;
        sl = i;
        psl = KB + i;
        pk2 = P2 - 1 - k2;
        k1 = r0 + i;
      } else if (e <= P2 / 2) {
        sl = 0; k2 = e; psl = 0; pk2 = (P2 - e) & (P2 - 1); k1 = 0;
      } else {
        sl = KB; k2 = e - P2 / 2 - 1; psl = KB; pk2 = P2 - 1 - k2; k1 = P1 / 2;
      }
      const int k = k1 + P1 * k2;
      const int km = M - k;  // mirror bin (M for k = 0)
      const cx<T> zk = s[sl * LS + pidx(k2)];
      const cx<T> zm = s[psl * LS + pidx(pk2)];
      // E = (Z_k + conj Z_m)/2, O = (Z_k - conj Z_m)/(2i), t = e^{-2 pi i k/L} O
      const cx<T> E = mk<T>(T(0.5) * (zk.x + zm.x), T(0.5) * (zk.y - zm.y));
      const cx<T> O = mk<T>(T(0.5) * (zk.y + zm.y), T(0.5) * (zm.x - zk.x));
      const cx<T> tO = cmul(tw2(tLlos, tLhis, k), O);
      const cx<T> yk = E + tO;
      const cx<T> ym = mk<T>(E.x - tO.x, tO.y - E.y);  // conj(E - t)
      yj[k] = yk;
      acc0[o] += (double)yk.x * (double)yk.x + (double)yk.y * (double)yk.y;
      if (km != k) {
        yj[km] = ym;
        acc1[o] += (double)ym.x * (double)ym.x + (double)ym.y * (double)ym.y;
      }
    }
    __syncthreads();  // the next frame overwrites s
  }
  if (part) {
    double* pc = part + (int64_t)ch * K;
#pragma unroll
    for (int o = 0; o < IPT; ++o) {
      const int e = tid + o * NT;
      if (e >= nitems) continue;
      int k2, k1;
      if (!special) {
        const int i = e % KB;
        if (i >= count) continue;
        k2 = e / KB;
        k1 = r0 + i;
      } else if (e <= P2 / 2) {
        k2 = e; k1 = 0;
      } else {
        k2 = e - P2 / 2 - 1; k1 = P1 / 2;
      }
      const int k = k1 + P1 * k2, km = M - k;
      pc[k] = acc0[o];
      if (km != k) pc[km] = acc1[o];
    }
  }
}

template <typename T>
static LfTw<T> lf_tables(const void* twS, int P1, int P2, int M) {
  const cx<T>* b = (const cx<T>*)twS;
  LfTw<T> t;
  t.tP1 = b;
  t.tP2 = t.tP1 + P1;
  t.tMlo = t.tP2 + P2;
  t.tMhi = t.tMlo + 512;
  t.tLlo = t.tMhi + (M >> 9 > 0 ? M >> 9 : 1);
  t.tLhi = t.tLlo + 512;
  return t;
}

template <typename T, int L1>
static hipError_t launch_lf1_t(const void* x, void* tmp, int64_t nblock, int ntap, const void* winT,
                               const LfTw<T>& tw, int M, int P2, hipStream_t st) {
  if constexpr (L1 <= 9) {
    if (ntap == 4 && nblock >= 4 && (M >> 9) <= (2 * (1 << L1) * (1 << L1)) / 512) {
      using Cr = Lf1rCfg<T, L1>;
      const int ncb = P2 / Cr::MB;
      // about one workgroup per CU, each sliding over a range of frames
      int64_t nr = (256 + ncb - 1) / ncb;
      if (nr > nblock) nr = nblock;
      const int frange = (int)((nblock + nr - 1) / nr);
      nr = (nblock + frange - 1) / frange;
      k_lf1r<T, L1><<<dim3((unsigned)(ncb * nr)), dim3(Cr::NT), 0, st>>>(
          (const cx<T>*)x, (cx<T>*)tmp, nblock, (const cx<T>*)winT, tw, M, P2, (int)nr, frange);
      return hipGetLastError();
    }
  }
  using Cfg = Lf1Cfg<T, L1>;
  const int64_t ncb = P2 / Cfg::MB;
  const dim3 grid((unsigned)(ncb * nblock));
  if (ntap == 4)
    k_lf1<T, L1, 4><<<grid, dim3(Cfg::NT), 0, st>>>((const cx<T>*)x, (cx<T>*)tmp, nblock, ntap,
                                                    (const cx<T>*)winT, tw, M, P2);
  else
    k_lf1<T, L1, 0><<<grid, dim3(Cfg::NT), 0, st>>>((const cx<T>*)x, (cx<T>*)tmp, nblock, ntap,
                                                    (const cx<T>*)winT, tw, M, P2);
  return hipGetLastError();
}

template <typename T, int L2>
static hipError_t launch_lf2_t(const void* tmp, void* y, const LfTw<T>& tw, int M, int P1, int64_t nblock,
                               int fchunk, double* part, hipStream_t st) {
  using Cfg = Lf2Cfg<T, L2>;
  if ((M >> 9) + 1 > (2 * Cfg::P2 * Cfg::P2) / 512 + 1) return hipErrorInvalidValue;  // LDS table size
  const int ngrp = (P1 / 2 - 1 + Cfg::KB - 1) / Cfg::KB;
  const int64_t nch = (nblock + fchunk - 1) / fchunk;
  k_lf2<T, L2><<<dim3((unsigned)((ngrp + 1) * nch)), dim3(Cfg::NT), 0, st>>>(
      (const cx<T>*)tmp, (cx<T>*)y, tw, M, P1, nblock, fchunk, ngrp, part);
  return hipGetLastError();
}

template <typename T>
static hipError_t launch_long_t(int pass, int log2n, const void* x, void* y, int64_t nblock, int ntap,
                                const void* winT, const void* twS, void* tmp, int fchunk, double* part,
                                hipStream_t st) {
  if (nblock == 0) return hipSuccess;
  const int log2m = log2n - 1;
  const int l2 = lf_log2p2(sizeof(T) == 8 ? F64 : F32, log2m), l1 = log2m - l2;
  const int M = 1 << log2m, P1 = 1 << l1, P2 = 1 << l2;
  const LfTw<T> tw = lf_tables<T>(twS, P1, P2, M);
  hipError_t e = hipSuccess;
  if (pass != 1) switch (l1) {
    case 7: e = launch_lf1_t<T, 7>(x, tmp, nblock, ntap, winT, tw, M, P2, st); break;
    case 8: e = launch_lf1_t<T, 8>(x, tmp, nblock, ntap, winT, tw, M, P2, st); break;
    case 9: e = launch_lf1_t<T, 9>(x, tmp, nblock, ntap, winT, tw, M, P2, st); break;
    case 10: e = launch_lf1_t<T, 10>(x, tmp, nblock, ntap, winT, tw, M, P2, st); break;
    default: return hipErrorInvalidValue;
  }
  if (e != hipSuccess || pass == 0) return e;
  switch (l2) {
    case 7: return launch_lf2_t<T, 7>(tmp, y, tw, M, P1, nblock, fchunk, part, st);
    case 8: return launch_lf2_t<T, 8>(tmp, y, tw, M, P1, nblock, fchunk, part, st);
    case 9: return launch_lf2_t<T, 9>(tmp, y, tw, M, P1, nblock, fchunk, part, st);
    default: return hipErrorInvalidValue;
  }
}

template <typename T, int L2>
static int lf_chunk_t(int P1, int64_t nblock) {
  using Cfg = Lf2Cfg<T, L2>;
  const int ngrp = (P1 / 2 - 1 + Cfg::KB - 1) / Cfg::KB;
  int64_t nch = resident_workgroups(k_lf2<T, L2>, Cfg::NT) / (ngrp + 1);
  if (nch < 1) nch = 1;
  if (nch > nblock) nch = nblock;
  return (int)((nblock + nch - 1) / nch);
}

int lf_frame_chunk(int prec, int log2n, int64_t nblock) {
  if (log2n < 15 || log2n > 20 || nblock < 1) return 1;
  const int log2m = log2n - 1;
  const int l2 = lf_log2p2(prec, log2m), l1 = log2m - l2;
  const int P1 = 1 << l1;
  if (prec == F32) {
    switch (l2) {
      case 7: return lf_chunk_t<float, 7>(P1, nblock);
      case 8: return lf_chunk_t<float, 8>(P1, nblock);
      default: return lf_chunk_t<float, 9>(P1, nblock);
    }
  }
  switch (l2) {
    case 7: return lf_chunk_t<double, 7>(P1, nblock);
    case 8: return lf_chunk_t<double, 8>(P1, nblock);
    default: return lf_chunk_t<double, 9>(P1, nblock);
  }
}

hipError_t launch_pfb_fwd_long(int prec, int log2n, int pass, const void* x, void* y, int64_t nblock, int ntap,
                               const void* winT, const void* twS, void* tmp, int fchunk, double* part,
                               hipStream_t st) {
  if (log2n < 15 || log2n > 20 || pass < -1 || pass > 1) return hipErrorInvalidValue;
  if (prec == F32) return launch_long_t<float>(pass, log2n, x, y, nblock, ntap, winT, twS, tmp, fchunk, part, st);
  return launch_long_t<double>(pass, log2n, x, y, nblock, ntap, winT, twS, tmp, fchunk, part, st);
}

}  // namespace ipfb
