// Column stage of the circulant inverse PFB (Section 3.1 with the Wiener
// weights of Section 4.1) computed in place on the frame matrix in its natural
// layout d[j][n] (frame j, sub-filter path n), with no transposes.
//
// Adjacent paths are paired into one complex sequence per pair p,
//   z_p[j] = d[j][2p] + i d[j][2p+1],
// which is the frame matrix itself read as complex numbers. A tile of TP
// adjacent pairs (128 bytes of every frame) is the unit of work, so every
// global access is a run of at least 128 bytes.
//
// For b <= 512 one pass does everything: the b-point FFT of each z_p, the
// separation of the two real spectra, the FP64 gains of both paths, and the
// inverse FFT. Larger b uses the four-step split b = b1 * b2, j = b2 j1 + j2,
// k = k1 + b1 k2:
//   pass A: FFT over j1 (stride b2 frames), times e^{-2 pi i j2 k1 / b};
//   pass B: FFT over j2 for the rows k1 and b1 - k1 together (so each
//           frequency k meets its mirror b - k), gain, inverse FFT over k2,
//           times e^{+2 pi i j2 k1 / b};
//   pass C: inverse FFT over k1, giving x[b2 j1 + j2] in time order.
// Every pass reads and writes exactly the same rows of its tile, so the three
// passes run in place on one buffer.
//
// The gain of path n at frequency f,
//   W_n(f) = sum_r h[rN + n] e^{-2 pi i r f / b},
//   G = W (1 + phi^2) / (|W|^2 + phi^2) / b,
// is evaluated on the fly in FP64 (as a polynomial in e^{-2 pi i f/b}); the
// two paths of a pair share one reciprocal. No N x b table ever touches HBM.
#include "fft_lds.hpp"
#include "launch.hpp"

namespace ipfb {

struct NatGain {
  const double* win;  // [ntap][lblock], FP64
  int lblock, ntap;
  double phi2;        // phi^2 (threshold filter: tau^2)
  double gnorm;       // (1 + phi^2) / b, or 1/b without the normalisation (other filters: 1/b)
  int naive;          // phi == 0: 1/conj(W), eigenvalues at rounding level dropped
  const double* nu;   // noise-to-signal filter: nu[f], f in [0, b/2]
  int norm;           // noise-to-signal filter: keep the (1 + nu) factor
};

// Filter kinds of the gain pass (a template parameter, so the Wiener pass is
// unchanged by the others): 0 Wiener / naive, 1 hard threshold |W| >= tau,
// 2 Wiener with a noise-to-signal ratio per frequency.
constexpr int kGainWiener = 0, kGainThreshold = 1, kGainNu = 2;

template <typename T>
struct NatCfg {
  static constexpr int TP = 128 / (int)sizeof(cx<T>);  // pairs per tile: 128 bytes per frame
  // pairs per workgroup of passes A and C: 512-byte runs per frame. When the
  // frames are not in the last-level cache (pass A after the row stage), HBM
  // serves the strided gather much faster in runs of 512 bytes than of 128
  static constexpr int TPO = 4 * TP;
  static constexpr int EPT = sizeof(T) == 4 ? 16 : 8;  // complex elements per thread in the FFTs
  static constexpr int clampnt(int v) { return v < 64 ? 64 : (v > 1024 ? 1024 : v); }
};

// W(z) = sum_{r < ntap} h_r z^r by Horner, taps read from global memory (any ntap).
__device__ __forceinline__ cx<double> horner_g(const double* __restrict__ win, int N, int n, int ntap,
                                               cx<double> z) {
  cx<double> w = mk<double>(0.0, 0.0);
  for (int r = ntap - 1; r >= 0; --r) {
    const double h = win[(int64_t)r * N + n];
    w = mk<double>(w.x * z.x - w.y * z.y + h, w.x * z.y + w.y * z.x);
  }
  return w;
}

// Gains of the two paths of a pair at one frequency. The truncation of the
// naive inverse compares |W| with the tap magnitude sum (wsa, wsc).
__device__ __forceinline__ void pair_gains(const NatGain& ga, cx<double> Wa, cx<double> Wc, double wsa,
                                           double wsc, cx<double>& Ga, cx<double>& Gc) {
  const double aa = Wa.x * Wa.x + Wa.y * Wa.y, ac = Wc.x * Wc.x + Wc.y * Wc.y;
  if (ga.naive) {
    const double sa = (sqrt(aa) <= 1e-12 * wsa) ? 0.0 : ga.gnorm / aa;
    const double sc = (sqrt(ac) <= 1e-12 * wsc) ? 0.0 : ga.gnorm / ac;
    Ga = mk<double>(Wa.x * sa, Wa.y * sa);
    Gc = mk<double>(Wc.x * sc, Wc.y * sc);
    return;
  }
  const double da = aa + ga.phi2, dc = ac + ga.phi2;
  // 1/(da dc): hardware reciprocal refined by one Newton step (error ~1 ulp)
  const double den = da * dc;
  double rc = __builtin_amdgcn_rcp(den);
  rc = rc * fma(-den, rc, 2.0);
  const double r = ga.gnorm * rc;
  const double sa = dc * r, sc = da * r;
  Ga = mk<double>(Wa.x * sa, Wa.y * sa);
  Gc = mk<double>(Wc.x * sc, Wc.y * sc);
}

// The other filters at frequency f in [0, b/2] (the same gain for both paths' formula):
// threshold: G = W / |W|^2 / b where |W|^2 >= tau^2, else 0;
// noise-to-signal: G = W c / (|W|^2 + nu_f) / b, c = 1 + nu_f or 1, set to 0
// where |W|^2 + nu_f is at rounding level against the squared tap magnitude
// sum (wsa, wsc), as the naive inverse truncates (nu_f = 0 at a zero of W).
template <int GK>
__device__ __forceinline__ void pair_gains_kind(const NatGain& ga, cx<double> Wa, cx<double> Wc, int f,
                                                double wsa, double wsc, cx<double>& Ga, cx<double>& Gc) {
  const double aa = Wa.x * Wa.x + Wa.y * Wa.y, ac = Wc.x * Wc.x + Wc.y * Wc.y;
  double sa, sc;
  if constexpr (GK == kGainThreshold) {
    sa = aa >= ga.phi2 ? ga.gnorm / aa : 0.0;
    sc = ac >= ga.phi2 ? ga.gnorm / ac : 0.0;
  } else {
    const double v = ga.nu[f];
    const double c = (ga.norm ? 1.0 + v : 1.0) * ga.gnorm;
    const double da = aa + v, dc = ac + v;
    sa = (da <= 1e-24 * wsa * wsa) ? 0.0 : c / da;
    sc = (dc <= 1e-24 * wsc * wsc) ? 0.0 : c / dc;
  }
  Ga = mk<double>(Wa.x * sa, Wa.y * sa);
  Gc = mk<double>(Wc.x * sc, Wc.y * sc);
}

// Passes A (DIR = -1) and C (DIR = +1): a b1-point FFT down the rows
// b2 j1 + j2 of TPO pairs [pa + TPO g, ...) clipped to pe, for one j2 per
// workgroup (ng groups g). All global loads of a thread are issued before the
// first LDS write; the four-step twiddles of pass A are gathered into LDS at
// the start.
template <typename T, int LOG2B1, int LOG2B2, int DIR>
__global__ __launch_bounds__((NatCfg<T>::clampnt(NatCfg<T>::TPO * (1 << LOG2B1) / NatCfg<T>::EPT)), 4) void k_nat_outer(
    cx<T>* __restrict__ z, int np, int pa, int pe, int ng, const cx<T>* __restrict__ tw, cx<T>* __restrict__ out,
    int r0, int nr) {
  constexpr int TP = NatCfg<T>::TPO;
  constexpr int B1 = 1 << LOG2B1, B2 = 1 << LOG2B2, B = B1 * B2;
  constexpr int NT = NatCfg<T>::clampnt(TP * B1 / NatCfg<T>::EPT);
  constexpr int LS = lds_len(B1);
  constexpr int NE = TP * B1, IT = (NE + NT - 1) / NT;
  __shared__ cx<T> s[TP * LS];
  __shared__ cx<T> tws[DIR < 0 ? B1 : 1];
  __shared__ cx<T> twf[B1];  // e^{-2 pi i m / b1}: the FFT's table, LDS-resident
  const int tid = threadIdx.x;
  const int g = blockIdx.x % ng, j2 = blockIdx.x / ng;
  const int p0 = pa + g * TP;
  for (int m = tid; m < B1; m += NT) {
    twf[m] = tw[m * B2];
    if (DIR < 0) tws[m] = tw[j2 * m];  // e^{-2 pi i j2 k1 / b}
  }
  cx<T> v[IT];
#pragma unroll
  for (int i = 0; i < IT; ++i) {
    const int e = tid + i * NT, q = e % TP, j1 = e / TP;
    v[i] = mk<T>(T(0), T(0));
    if ((NE % NT == 0 || e < NE) && p0 + q < pe) v[i] = z[(int64_t)(j1 * B2 + j2) * np + p0 + q];
  }
#pragma unroll
  for (int i = 0; i < IT; ++i) {
    const int e = tid + i * NT, q = e % TP, j1 = e / TP;
    if (NE % NT == 0 || e < NE) s[q * LS + pidx(j1)] = v[i];
  }
  __syncthreads();
  lds_fft<T, B1, NT, TP, DIR>(s, LS, twf, 1);
#pragma unroll
  for (int i = 0; i < IT; ++i) {
    const int e = tid + i * NT, q = e % TP, k1 = e / TP;
    if (NE % NT != 0 && e >= NE) continue;
    cx<T> u = s[q * LS + pidx(k1)];
    if (DIR < 0) u = cmul(u, tws[k1]);
    if (p0 + q >= pe) continue;
    const int row = k1 * B2 + j2;
    if (DIR > 0 && out) {  // only the frames [r0, r0 + nr), to out
      if (row >= r0 && row < r0 + nr) out[(int64_t)(row - r0) * np + p0 + q] = u;
    } else {
      z[(int64_t)row * np + p0 + q] = u;
    }
  }
}

// Work item `it` of the gain pass (one frequency k and its mirror b - k):
// row set and index of k (sk, k2) and of the mirror (sm, k2m). For kk > 0 the
// items are k2 in [0, b2) of row ka, mirrored in row kb at b2-1-k2; for
// kk = 0, k2 in [0, b2/2] of row 0 (mirror (b2-k2) mod b2) and then k2 in
// [0, b2/2) of row b1/2 (mirror b2-1-k2).
template <int NS, int B2>
__device__ __forceinline__ void gain_item(int kk, int it, int& sk, int& k2, int& sm, int& k2m) {
  if (NS == 2 && kk != 0) {
    sk = 0; k2 = it; sm = 1; k2m = B2 - 1 - it;
  } else if (it <= B2 / 2) {
    sk = 0; k2 = it; sm = 0; k2m = (B2 - it) & (B2 - 1);
  } else {
    sk = 1; k2 = it - (B2 / 2 + 1); sm = 1; k2m = B2 - 1 - k2;
  }
}

// Pass B (or the whole stage when b1 = 1): b2-point FFTs of the rows k1 and
// b1 - k1 of one tile, separation of the two real spectra of each pair, FP64
// gains, re-packing, inverse FFTs, and the inverse four-step twiddle.
template <typename T, int LOG2B1, int LOG2B2, int NTAP, int GK = kGainWiener>
__global__ __launch_bounds__((NatCfg<T>::clampnt(((1 << LOG2B1) > 1 ? 2 : 1) * NatCfg<T>::TP * (1 << LOG2B2) /
                                                 NatCfg<T>::EPT)),
                             4) void k_nat_mid(cx<T>* __restrict__ z, int np, int t0, int ntile, NatGain ga,
                                               const cx<T>* __restrict__ tw,
                                               const cx<double>* __restrict__ tw64) {
  constexpr int TP = NatCfg<T>::TP;
  constexpr int B1 = 1 << LOG2B1, B2 = 1 << LOG2B2, B = B1 * B2;
  constexpr int NS = B1 > 1 ? 2 : 1;  // row sets held by one workgroup
  constexpr int NT = NatCfg<T>::clampnt(NS * TP * B2 / NatCfg<T>::EPT);
  constexpr int LS = lds_len(B2);
  constexpr int NE = NS * TP * B2, IT = (NE + NT - 1) / NT;
  static_assert(NT % TP == 0, "a thread keeps one pair through the gain pass");
  __shared__ cx<T> s[NS * TP * LS];
  __shared__ cx<T> tws[B1 > 1 ? NS * B2 : 1];
  __shared__ cx<T> twf[B2];  // e^{-2 pi i m / b2}: the FFTs' table, LDS-resident
  __shared__ cx<double> twz[B2];  // the same in FP64, for the gains
  const int tid = threadIdx.x;
  const int tile = blockIdx.x % ntile, kk = blockIdx.x / ntile;
  const int p0 = (t0 + tile) * TP;
  // row sets: (k1, b1 - k1), or (0, b1/2) for kk = 0 (both their own mirrors)
  const int ka = kk, kb = (kk == 0) ? B1 / 2 : B1 - kk;

  if (B1 > 1)
    for (int t = tid; t < NS * B2; t += NT) tws[t] = tw[(t % B2) * ((t / B2) ? kb : ka)];  // e^{-2 pi i j2 k1/b}
  for (int m = tid; m < B2; m += NT) {
    twf[m] = tw[m * B1];
    twz[m] = tw64[m * B1];
  }
  constexpr int IPAR = NT / TP;  // gain items in flight across the workgroup
  constexpr int NIMAX = (NS == 1) ? (B2 / 2 + 1) : (B2 + 1);
  constexpr int IMAX = (NIMAX + IPAR - 1) / IPAR;
  const int NI = (NS == 1) ? (B2 / 2 + 1) : (kk == 0 ? B2 + 1 : B2);
  const int q = tid % TP;
  const bool valid = p0 + q < np;
  const int N = ga.lblock, na = 2 * (p0 + q), nc = na + 1;
  // e^{-2 pi i f / b} for f = k1 + b1 k2 is base * e^{-2 pi i k2 / b2}, with
  // base = e^{-2 pi i ka / b} for kk > 0; for kk = 0, 1 on row 0 and
  // -e^{+i pi / b2} on row b1/2 (the items of row b1/2 count k2 from b2/2+1).
  const cx<double> base_a = tw64[ka];
  const cx<double> h1 = tw64[B1 / 2];
  const cx<double> base_b = mk<double>(-h1.x, h1.y);
  constexpr int HT = NTAP > 0 ? NTAP : 1;
  double ha[HT], hc[HT];
#pragma unroll
  for (int r = 0; r < HT; ++r) {
    ha[r] = (NTAP > 0 && valid) ? ga.win[(int64_t)r * N + na] : 0.0;
    hc[r] = (NTAP > 0 && valid) ? ga.win[(int64_t)r * N + nc] : 0.0;
  }
  double wsa = 0.0, wsc = 0.0;
  if ((ga.naive || GK == kGainNu) && valid) {
    for (int r = 0; r < ga.ntap; ++r) {
      wsa += fabs(ga.win[(int64_t)r * N + na]);
      wsc += fabs(ga.win[(int64_t)r * N + nc]);
    }
  }
  // gains of item `it` (FP64): the two paths of pair q at the item's frequency
  auto gains = [&](int it, cx<double>& Ga, cx<double>& Gc) {
    int sk, k2, sm, k2m;
    gain_item<NS, B2>(kk, it, sk, k2, sm, k2m);
    const int kz = (NS == 2 && kk == 0 && sk == 1) ? k2 + B2 / 2 + 1 : k2;
    const cx<double> zf = cmul((NS == 2 && kk == 0 && sk == 1) ? base_b : base_a, twz[kz & (B2 - 1)]);
    cx<double> Wa, Wc;
    if constexpr (NTAP == 4) {
      const cx<double> z2 = cmul(zf, zf), z3 = cmul(z2, zf);
      Wa = mk<double>(ha[0] + ha[1] * zf.x + ha[2] * z2.x + ha[3] * z3.x, ha[1] * zf.y + ha[2] * z2.y + ha[3] * z3.y);
      Wc = mk<double>(hc[0] + hc[1] * zf.x + hc[2] * z2.x + hc[3] * z3.x, hc[1] * zf.y + hc[2] * z2.y + hc[3] * z3.y);
    } else {
      Wa = horner_g(ga.win, N, na, ga.ntap, zf);
      Wc = horner_g(ga.win, N, nc, ga.ntap, zf);
    }
    if constexpr (GK == kGainWiener) {
      pair_gains(ga, Wa, Wc, wsa, wsc, Ga, Gc);
    } else {
      // the item's frequency: row k1 of its set (b1/2 for the second set of
      // kk = 0) plus b1 k2, folded to [0, b/2] (the filter is even in f)
      const int f = ((NS == 2 && kk == 0 && sk == 1) ? B1 / 2 : ka) + B1 * k2;
      pair_gains_kind<GK>(ga, Wa, Wc, f <= B - f ? f : B - f, wsa, wsc, Ga, Gc);
    }
  };
  // FP32 form with 4 taps: the first NPRE gains of this thread are formed
  // (FP64, then rounded once) while the workgroup's loads are in flight, and
  // kept in registers until the spectra are ready; the rest follow the FFT
  // (only where the register budget holds them without spilling: b2 = 128)
  constexpr bool PRE = sizeof(T) == 4 && NTAP == 4 && B2 == 128 && GK == kGainWiener;
  constexpr int NPRE = PRE ? (IMAX < 2 ? IMAX : 2) : 1;  // gains held across the FFT
  cx<T> gpre[NPRE][2];
  {
    cx<T> v[IT];
#pragma unroll
    for (int i = 0; i < IT; ++i) {
      const int e = tid + i * NT, qq = e % TP, r = e / TP;
      const int j2 = r % B2, k1 = (r / B2) ? kb : ka;
      v[i] = mk<T>(T(0), T(0));
      if ((NE % NT == 0 || e < NE) && p0 + qq < np) v[i] = z[(int64_t)(k1 * B2 + j2) * np + p0 + qq];
    }
    if constexpr (PRE) {
      __syncthreads();  // twz ready (the loads above stay in flight)
#pragma unroll
      for (int i = 0; i < NPRE; ++i) {
        const int it = tid / TP + i * IPAR;
        cx<double> Ga = mk<double>(0.0, 0.0), Gc = Ga;
        if (valid && it < NI) gains(it, Ga, Gc);
        gpre[i][0] = mk<T>(T(Ga.x), T(Ga.y));
        gpre[i][1] = mk<T>(T(Gc.x), T(Gc.y));
      }
    }
#pragma unroll
    for (int i = 0; i < IT; ++i) {
      const int e = tid + i * NT, qq = e % TP, r = e / TP;
      if (NE % NT == 0 || e < NE) s[(r / B2 * TP + qq) * LS + pidx(r % B2)] = v[i];
    }
  }
  __syncthreads();
  lds_fft<T, B2, NT, NS * TP, -1>(s, LS, twf, 1);

  // apply: split the two real spectra of pair q at frequency k (and b - k),
  // weight them, re-pack; with g = G/2,
  //   A' = g_a (Z_k + conj Z_m),  C' = g_c (Z_k - conj Z_m) / i
  auto apply = [&](int it, cx<T> gat, cx<T> gct) {
    int sk, k2, sm, k2m;
    gain_item<NS, B2>(kk, it, sk, k2, sm, k2m);
    cx<T>* pk = s + (sk * TP + q) * LS + pidx(k2);
    cx<T>* pm = s + (sm * TP + q) * LS + pidx(k2m);
    const cx<T> zk = *pk, zm = *pm;
    if (sk == sm && k2 == k2m) {  // f = 0 or b/2: both spectra real there, gains real
      *pk = mk<T>(gat.x * zk.x, gct.x * zk.y);
      return;
    }
    const cx<T> ha2 = mk<T>(T(0.5) * gat.x, T(0.5) * gat.y), hc2 = mk<T>(T(0.5) * gct.x, T(0.5) * gct.y);
    const cx<T> A2 = mk<T>(zk.x + zm.x, zk.y - zm.y);
    const cx<T> C2 = mk<T>(zk.y + zm.y, zm.x - zk.x);
    const cx<T> Ap = cmul(ha2, A2), Cp = cmul(hc2, C2);
    // Z'_k = A' + i C',  Z'_{b-k} = conj(A') + i conj(C')
    *pk = mk<T>(Ap.x - Cp.y, Ap.y + Cp.x);
    *pm = mk<T>(Ap.x + Cp.y, Cp.x - Ap.y);
  };
  if constexpr (PRE) {
#pragma unroll
    for (int i = 0; i < NPRE; ++i) {
      const int it = tid / TP + i * IPAR;
      if (valid && it < NI) apply(it, gpre[i][0], gpre[i][1]);
    }
  }
  {
#pragma unroll 1
    for (int i = PRE ? NPRE : 0; i < IMAX; ++i) {
      const int it = tid / TP + i * IPAR;
      if (!valid || it >= NI) break;
      cx<double> Ga, Gc;
      gains(it, Ga, Gc);
      // the gains are formed in FP64 and rounded once to the data precision
      apply(it, mk<T>(T(Ga.x), T(Ga.y)), mk<T>(T(Gc.x), T(Gc.y)));
    }
  }
  __syncthreads();
  lds_fft<T, B2, NT, NS * TP, +1>(s, LS, twf, 1);

#pragma unroll
  for (int i = 0; i < IT; ++i) {
    const int e = tid + i * NT, q = e % TP, r = e / TP;
    if (NE % NT != 0 && e >= NE) continue;
    const int j2 = r % B2, set = r / B2;
    const int k1 = set ? kb : ka;
    cx<T> v = s[(set * TP + q) * LS + pidx(j2)];
    if (B1 > 1) v = cmulc(v, tws[r]);  // e^{+2 pi i j2 k1 / b}
    if (p0 + q < np) z[(int64_t)(k1 * B2 + j2) * np + p0 + q] = v;
  }
}

// The gain pass with the filter kind chosen at run time: the Wiener filter
// with the 4-tap fast path, the other kinds with the generic tap loop.
template <typename T, int L1, int L2>
static void launch_mid(int kind, dim3 grid, dim3 nt, cx<T>* z, int np, int tile0, int ntiles, const NatGain& ga,
                       const cx<T>* tw, const cx<double>* tw64, hipStream_t st) {
  if (kind == kGainThreshold)
    k_nat_mid<T, L1, L2, 0, kGainThreshold><<<grid, nt, 0, st>>>(z, np, tile0, ntiles, ga, tw, tw64);
  else if (kind == kGainNu)
    k_nat_mid<T, L1, L2, 0, kGainNu><<<grid, nt, 0, st>>>(z, np, tile0, ntiles, ga, tw, tw64);
  else if (ga.ntap == 4)
    k_nat_mid<T, L1, L2, 4><<<grid, nt, 0, st>>>(z, np, tile0, ntiles, ga, tw, tw64);
  else
    k_nat_mid<T, L1, L2, 0><<<grid, nt, 0, st>>>(z, np, tile0, ntiles, ga, tw, tw64);
}

template <typename T, int LOG2B>
static hipError_t launch_nat_t(int pass, void* zv, int lblock, int tile0, int ntiles, const NatGain& ga,
                               const void* twv, const double* tw64v, hipStream_t st, void* out, int r0, int nr,
                               int kind) {
  using Cfg = NatCfg<T>;
  cx<T>* z = (cx<T>*)zv;
  const cx<T>* tw = (const cx<T>*)twv;
  const cx<double>* tw64 = (const cx<double>*)tw64v;
  const int np = lblock / 2;
  const int nall = (np + Cfg::TP - 1) / Cfg::TP;
  if (ntiles < 0 || tile0 + ntiles > nall) ntiles = nall - tile0;
  if (tile0 < 0 || ntiles <= 0) return tile0 < 0 ? hipErrorInvalidValue : hipSuccess;
  if constexpr (LOG2B <= 9) {
    if (out) return hipErrorInvalidValue;  // the one-pass form works in place only
    if (pass != 1) return hipSuccess;
    constexpr int NT = Cfg::clampnt(Cfg::TP * (1 << LOG2B) / Cfg::EPT);
    launch_mid<T, 0, LOG2B>(kind, dim3(ntiles), dim3(NT), z, np, tile0, ntiles, ga, tw, tw64, st);
  } else {
    constexpr int L1 = LOG2B / 2, L2 = LOG2B - L1;
    constexpr int NTO = Cfg::clampnt(Cfg::TPO * (1 << L1) / Cfg::EPT);
    constexpr int NTM = Cfg::clampnt(2 * Cfg::TP * (1 << L2) / Cfg::EPT);
    // passes A and C: the pairs of tiles [tile0, tile0 + ntiles) in groups of TPO
    const int pa = tile0 * Cfg::TP;
    const int pe = (tile0 + ntiles) * Cfg::TP < np ? (tile0 + ntiles) * Cfg::TP : np;
    const int ng = (pe - pa + Cfg::TPO - 1) / Cfg::TPO;
    if (pass == 0)
      k_nat_outer<T, L1, L2, -1><<<dim3(ng * (1 << L2)), dim3(NTO), 0, st>>>(z, np, pa, pe, ng, tw, nullptr, 0, 0);
    if (pass == 1)
      launch_mid<T, L1, L2>(kind, dim3(ntiles * (1 << (L1 - 1))), dim3(NTM), z, np, tile0, ntiles, ga, tw, tw64, st);
    if (pass == 2)
      k_nat_outer<T, L1, L2, +1><<<dim3(ng * (1 << L2)), dim3(NTO), 0, st>>>(z, np, pa, pe, ng, tw, (cx<T>*)out,
                                                                              r0, nr);
  }
  return hipGetLastError();
}

#define NAT_CASE(T, L) \
  case L: return launch_nat_t<T, L>(pass, z, lblock, tile0, ntiles, ga, twB, twB64, st, out, r0, nr, kind);

int nat_tiles(int prec, int lblock) {
  const int tp = prec == F32 ? NatCfg<float>::TP : NatCfg<double>::TP;
  return (lblock / 2 + tp - 1) / tp;
}

hipError_t launch_col_wiener_nat(int prec, int log2b, int pass, void* z, int lblock, int ntap, const double* win64,
                                 double phi, int normalise, const void* twB, const double* twB64, hipStream_t st,
                                 int tile0, int ntiles, void* out, int r0, int nr, int kind, const double* nu) {
  if (lblock < 2 || (lblock & 1) || pass < 0 || pass > 2) return hipErrorInvalidValue;
  if (kind < kGainWiener || kind > kGainNu || (kind == kGainNu && !nu)) return hipErrorInvalidValue;
  if (out && (pass != 2 || r0 < 0 || nr < 0 || r0 + nr > (1 << log2b))) return hipErrorInvalidValue;
  NatGain ga;
  ga.win = win64;
  ga.lblock = lblock;
  ga.ntap = ntap;
  ga.phi2 = phi * phi;
  ga.naive = phi == 0.0;
  ga.gnorm = (normalise ? (1.0 + phi * phi) : 1.0) / (double)(1LL << log2b);
  ga.nu = nu;
  ga.norm = normalise;
  if (kind != kGainWiener) {  // phi carries tau for the threshold filter
    ga.naive = 0;
    ga.gnorm = 1.0 / (double)(1LL << log2b);
  }
  if (prec == F32) {
    switch (log2b) {
      NAT_CASE(float, 2) NAT_CASE(float, 3) NAT_CASE(float, 4) NAT_CASE(float, 5) NAT_CASE(float, 6)
      NAT_CASE(float, 7) NAT_CASE(float, 8) NAT_CASE(float, 9) NAT_CASE(float, 10) NAT_CASE(float, 11)
      NAT_CASE(float, 12) NAT_CASE(float, 13) NAT_CASE(float, 14) NAT_CASE(float, 15)
      default: return hipErrorInvalidValue;
    }
  }
  switch (log2b) {
    NAT_CASE(double, 2) NAT_CASE(double, 3) NAT_CASE(double, 4) NAT_CASE(double, 5) NAT_CASE(double, 6)
    NAT_CASE(double, 7) NAT_CASE(double, 8) NAT_CASE(double, 9) NAT_CASE(double, 10) NAT_CASE(double, 11)
    NAT_CASE(double, 12) NAT_CASE(double, 13) NAT_CASE(double, 14)
    default: return hipErrorInvalidValue;
  }
}

}  // namespace ipfb
