// Column stage of the circulant inverse PFB for an arbitrary number of frames
// b (the batched form: streams of uneven length). The b-point DFT down each
// sub-filter path (Section 3.1's decorrelation needs exactly length b: padding
// would change the circulant) is computed with Bluestein's chirp-z identity
//   jk = (j^2 + k^2 - (k-j)^2)/2  =>  X_k = conj(c_k) sum_j (x_j conj(c_j)) c_{k-j},
//   c_m = exp(i pi m^2 / b),
// a linear convolution evaluated as a cyclic one of power-of-two length
// M >= 2b-1 against the precomputed spectrum C = FFT_M(c). Two real columns
// (n, n+1) travel as one complex sequence. Each M-point FFT is a four-step
// M = M1 * M2 over global memory:
//   A  (per pair, block of MB consecutive j2): M1-point DFTs over j1 of
//      a[j1 M2 + j2], twiddle w_M^{j2 k1}            -> T[pair][k1][j2]
//   B  (per pair, block of KB rows k1): M2-point DFT along the row, times
//      C[k1 + M1 k2] (or its conjugate), inverse M2-point DFT, conj twiddle
//                                                     -> T in place
//   A' (per pair, block of MB j2): inverse M1-point DFTs over k1 -> the cyclic
//      convolution at j = j1 M2 + j2, times the post-chirp.
// Between the two convolutions one kernel splits the two real spectra, applies
// the FP64 Wiener gain of Section 4.1 and re-packs them (it needs X_k and
// X_{b-k}, which the four-step places far apart).
// Tunables (picked per convolution length by the batched plan's autotuner):
// the split M1 = 2^l1, the tile widths MB (columns per A/A' block) and KB (rows
// per B block), and the number of pairs per launch group (the four-step
// scratch of one group stays in the last-level cache when the group is small).
// The factor w_M^m = tHi[m >> 8] tLo[m & 255] comes from LDS copies of both
// tables (M <= 2^16, so tHi has at most 256 entries).
#include "fft_lds.hpp"
#include "launch.hpp"

namespace ipfb {

struct BluTw {  // all e^{-2 pi i m / len} in the data precision
  const void* tM1;   // [M1]
  const void* tM2;   // [M2]
  const void* tLo;   // [256]   w_M^{m & 255}
  const void* tHi;   // [M/256] w_M^{256 (m >> 8)}
};

constexpr int kBluMaxLog2M = 16;

template <typename T>
__device__ __forceinline__ cx<T> blu_twM(const cx<T>* lo, const cx<T>* hi, int m) {
  return cmul(hi[m >> 8], lo[m & 255]);
}

// LDS copies of tLo [256] and tHi [M/256]
template <typename T, int NT>
__device__ __forceinline__ void blu_tw_lds(cx<T>* lo, cx<T>* hi, const BluTw& tw, int M) {
  const cx<T>* glo = reinterpret_cast<const cx<T>*>(tw.tLo);
  const cx<T>* ghi = reinterpret_cast<const cx<T>*>(tw.tHi);
  const int nhi = M >> 8;
  for (int i = threadIdx.x; i < 256; i += NT) {
    lo[i] = glo[i];
    if (i < nhi) hi[i] = ghi[i];
  }
  if (nhi == 0 && threadIdx.x == 0) hi[0] = ghi[0];
}

template <int LOG2M1, int MB_>
struct BluACfg {
  static constexpr int M1 = 1 << LOG2M1;
  static constexpr int MB = MB_;
  static constexpr int LS = lds_len(M1);
  static constexpr int NT0 = (M1 * MB) / 8;
  static constexpr int NT = NT0 < 64 ? 64 : (NT0 > 512 ? 512 : NT0);
};

// MODE 0: input = real pair from x_T [N][b] times conj(chirp); MODE 1: input = complex a [pair][b].
// Pairs pair0 + blockIdx.x / (M2 / MB); Tm holds the launch group's pairs only.
template <typename T, int LOG2M1, int MB_, int MODE>
__global__ __launch_bounds__((BluACfg<LOG2M1, MB_>::NT)) void k_blu_A(
    const void* __restrict__ in, cx<T>* __restrict__ Tm, const cx<T>* __restrict__ chirp, int64_t b, int M2,
    int N, int64_t pair0, BluTw tw) {
  using Cfg = BluACfg<LOG2M1, MB_>;
  constexpr int M1 = Cfg::M1, LS = Cfg::LS, NT = Cfg::NT;
  constexpr int MB = Cfg::MB;
  __shared__ cx<T> s[MB * LS];
  __shared__ cx<T> tlo[256], thi[256];
  const int M = M1 * M2;
  blu_tw_lds<T, NT>(tlo, thi, tw, M);
  const int mb_eff = M2 < MB ? M2 : MB;
  const int nblk = M2 / mb_eff;
  const int64_t lpair = blockIdx.x / nblk, pair = pair0 + lpair;
  const int j20 = (blockIdx.x % nblk) * mb_eff;
  for (int e = threadIdx.x; e < M1 * MB; e += NT) {
    const int mb = e % MB, j1 = e / MB;
    cx<T> v = mk<T>(T(0), T(0));
    const int64_t j = (int64_t)j1 * M2 + j20 + mb;
    if (mb < mb_eff && j < b) {
      if constexpr (MODE == 0) {
        const T* xT = reinterpret_cast<const T*>(in);
        const int64_t n = 2 * pair;
        const T re = xT[n * b + j];
        const T im = (n + 1 < N) ? xT[(n + 1) * b + j] : T(0);
        v = cmulc(mk<T>(re, im), chirp[j]);
      } else {
        v = reinterpret_cast<const cx<T>*>(in)[pair * b + j];
      }
    }
    s[mb * LS + pidx(j1)] = v;
  }
  __syncthreads();
  lds_fft<T, M1, NT, MB, -1>(s, LS, reinterpret_cast<const cx<T>*>(tw.tM1), 1);
  cx<T>* tp = Tm + lpair * (int64_t)M;
  for (int e = threadIdx.x; e < M1 * MB; e += NT) {
    const int mb = e % MB, k1 = e / MB;
    if (mb >= mb_eff) continue;
    const int j2 = j20 + mb;
    tp[(int64_t)k1 * M2 + j2] = cmul(s[mb * LS + pidx(k1)], blu_twM(tlo, thi, j2 * k1));
  }
}

template <int LOG2M2, int KB_>
struct BluBCfg {
  static constexpr int M2 = 1 << LOG2M2;
  static constexpr int KB = KB_;
  static constexpr int LS = lds_len(M2);
  static constexpr int NT0 = (M2 * KB) / 8;
  static constexpr int NT = NT0 < 64 ? 64 : (NT0 > 512 ? 512 : NT0);
};

template <typename T, int LOG2M2, int KB_>
__global__ __launch_bounds__((BluBCfg<LOG2M2, KB_>::NT)) void k_blu_B(cx<T>* __restrict__ Tm,
                                                                      const cx<T>* __restrict__ Crow, int conjC,
                                                                      int M1, BluTw tw) {
  using Cfg = BluBCfg<LOG2M2, KB_>;
  constexpr int M2 = Cfg::M2, LS = Cfg::LS, NT = Cfg::NT, KB = Cfg::KB;
  __shared__ cx<T> s[KB * LS];
  __shared__ cx<T> tlo[256], thi[256];
  const int M = M1 * M2;
  blu_tw_lds<T, NT>(tlo, thi, tw, M);
  const int kb_eff = M1 < KB ? M1 : KB;
  const int nblk = M1 / kb_eff;
  const int64_t pair = blockIdx.x / nblk;
  const int k10 = (blockIdx.x % nblk) * kb_eff;
  cx<T>* tp = Tm + pair * (int64_t)M;
  for (int e = threadIdx.x; e < KB * M2; e += NT) {
    const int r = e / M2, c = e % M2;
    cx<T> v = mk<T>(T(0), T(0));
    if (r < kb_eff) v = tp[(int64_t)(k10 + r) * M2 + c];
    s[r * LS + pidx(c)] = v;
  }
  __syncthreads();
  const cx<T>* tM2 = reinterpret_cast<const cx<T>*>(tw.tM2);
  lds_fft<T, M2, NT, KB, -1>(s, LS, tM2, 1);
  for (int e = threadIdx.x; e < KB * M2; e += NT) {  // times C[k1 + M1 k2] (row layout Crow[k1][k2])
    const int r = e / M2, k2 = e % M2;
    if (r >= kb_eff) continue;
    cx<T> h = Crow[(int64_t)(k10 + r) * M2 + k2];
    if (conjC) h.y = -h.y;
    s[r * LS + pidx(k2)] = cmul(s[r * LS + pidx(k2)], h);
  }
  __syncthreads();
  lds_fft<T, M2, NT, KB, +1>(s, LS, tM2, 1);
  for (int e = threadIdx.x; e < KB * M2; e += NT) {
    const int r = e / M2, j2 = e % M2;
    if (r >= kb_eff) continue;
    const int k1 = k10 + r;
    tp[(int64_t)k1 * M2 + j2] = cmulc(s[r * LS + pidx(j2)], blu_twM(tlo, thi, j2 * k1));
  }
}

// MODE 0: Z[pair][j] = conj(c_j) conv_j / M (the b-point DFT); MODE 1: output
// the pair of real columns  x_T[n][j] + i x_T[n+1][j] = c_j conv_j / (M b)
template <typename T, int LOG2M1, int MB_, int MODE>
__global__ __launch_bounds__((BluACfg<LOG2M1, MB_>::NT)) void k_blu_Ainv(
    const cx<T>* __restrict__ Tm, void* __restrict__ out, const cx<T>* __restrict__ chirp, int64_t b, int M2,
    int N, int64_t pair0, BluTw tw) {
  using Cfg = BluACfg<LOG2M1, MB_>;
  constexpr int M1 = Cfg::M1, LS = Cfg::LS, NT = Cfg::NT;
  constexpr int MB = Cfg::MB;
  __shared__ cx<T> s[MB * LS];
  const int mb_eff = M2 < MB ? M2 : MB;
  const int nblk = M2 / mb_eff;
  const int64_t lpair = blockIdx.x / nblk, pair = pair0 + lpair;
  const int j20 = (blockIdx.x % nblk) * mb_eff;
  const int M = M1 * M2;
  const cx<T>* tp = Tm + lpair * (int64_t)M;
  for (int e = threadIdx.x; e < M1 * MB; e += NT) {
    const int mb = e % MB, k1 = e / MB;
    cx<T> v = mk<T>(T(0), T(0));
    if (mb < mb_eff) v = tp[(int64_t)k1 * M2 + j20 + mb];
    s[mb * LS + pidx(k1)] = v;
  }
  __syncthreads();
  lds_fft<T, M1, NT, MB, +1>(s, LS, reinterpret_cast<const cx<T>*>(tw.tM1), 1);
  const T sc = (MODE == 0) ? T(1.0 / (double)M) : T(1.0 / ((double)M * (double)b));
  for (int e = threadIdx.x; e < M1 * MB; e += NT) {
    const int mb = e % MB, j1 = e / MB;
    if (mb >= mb_eff) continue;
    const int64_t j = (int64_t)j1 * M2 + j20 + mb;
    if (j >= b) continue;
    const cx<T> v = scale(s[mb * LS + pidx(j1)], sc);
    if constexpr (MODE == 0) {
      reinterpret_cast<cx<T>*>(out)[pair * b + j] = cmulc(v, chirp[j]);
    } else {
      const cx<T> z = cmul(v, chirp[j]);
      T* xT = reinterpret_cast<T*>(out);
      const int64_t n = 2 * pair;
      xT[n * b + j] = z.x;
      if (n + 1 < N) xT[(n + 1) * b + j] = z.y;
    }
  }
}

// Split the two real spectra of each pair, apply the FP64 gain, re-pack, and
// pre-multiply by the chirp for the inverse transform:
//   X1 = (Z_k + conj Z_{b-k})/2,  X2 = (Z_k - conj Z_{b-k})/2i,
//   a_k = (G_n(k) X1 + i G_{n+1}(k) X2) c_k.
struct BluGain {
  const double* win;  // [ntap][N]
  int N, ntap;
  double phi2, gnorm;  // gnorm = 1 + phi^2 (or 1)
  int naive;
};

__device__ __forceinline__ cx<double> blu_gain(const BluGain& g, int n, const cx<double>* __restrict__ twb64,
                                               int64_t f) {
  const cx<double> t1 = twb64[f];
  cx<double> e = mk<double>(1.0, 0.0);
  double wr = 0.0, wi = 0.0, wabs = 0.0;
  for (int r = 0; r < g.ntap; ++r) {
    const double h = g.win[(int64_t)r * g.N + n];
    wr += h * e.x;
    wi += h * e.y;
    wabs += fabs(h);
    e = cmul(e, t1);
  }
  const double a2 = wr * wr + wi * wi;
  if (g.naive) {
    if (sqrt(a2) <= 1e-12 * wabs) return mk<double>(0.0, 0.0);
    return mk<double>(wr / a2, wi / a2);
  }
  const double s = g.gnorm / (a2 + g.phi2);
  return mk<double>(wr * s, wi * s);
}

// Gains of paths n and n+1 (4 taps each) at one frequency: W as a cubic in
// z = e^{-2 pi i k/b}, the two denominators sharing one reciprocal.
__device__ __forceinline__ void blu_gain_pair4(const BluGain& g, int n, bool has1, cx<double> z, cx<double>& Ga,
                                               cx<double>& Gc) {
  const int N = g.N;
  const double a0 = g.win[n], a1 = g.win[N + n], a2 = g.win[2 * N + n], a3 = g.win[3 * N + n];
  const int m = has1 ? n + 1 : n;
  const double c0 = g.win[m], c1 = g.win[N + m], c2 = g.win[2 * N + m], c3 = g.win[3 * N + m];
  const cx<double> z2 = cmul(z, z), z3 = cmul(z2, z);
  const cx<double> Wa = mk<double>(a0 + a1 * z.x + a2 * z2.x + a3 * z3.x, a1 * z.y + a2 * z2.y + a3 * z3.y);
  const cx<double> Wc = mk<double>(c0 + c1 * z.x + c2 * z2.x + c3 * z3.x, c1 * z.y + c2 * z2.y + c3 * z3.y);
  const double aa = Wa.x * Wa.x + Wa.y * Wa.y, ac = Wc.x * Wc.x + Wc.y * Wc.y;
  if (g.naive) {
    const double wa = fabs(a0) + fabs(a1) + fabs(a2) + fabs(a3), wc = fabs(c0) + fabs(c1) + fabs(c2) + fabs(c3);
    const double sa = (sqrt(aa) <= 1e-12 * wa) ? 0.0 : 1.0 / aa;
    const double sc = (sqrt(ac) <= 1e-12 * wc) ? 0.0 : 1.0 / ac;
    Ga = mk<double>(Wa.x * sa, Wa.y * sa);
    Gc = mk<double>(Wc.x * sc, Wc.y * sc);
    return;
  }
  const double da = aa + g.phi2, dc = ac + g.phi2;
  const double den = da * dc;
  double rc = __builtin_amdgcn_rcp(den);
  rc = rc * fma(-den, rc, 2.0);  // one Newton step: ~1 ulp
  const double sa = g.gnorm * dc * rc, sc = g.gnorm * da * rc;
  Ga = mk<double>(Wa.x * sa, Wa.y * sa);
  Gc = mk<double>(Wc.x * sc, Wc.y * sc);
}

// one pair (pair0 + blockIdx.y) per grid row, frequencies k = blockIdx.x * 256 + tid (grid-strided)
template <typename T>
__global__ __launch_bounds__(256) void k_blu_gain2(const cx<T>* __restrict__ Z, cx<T>* __restrict__ a,
                                                   const cx<T>* __restrict__ chirp,
                                                   const cx<double>* __restrict__ twb64, int64_t b, int64_t pair0,
                                                   BluGain g) {
  const int64_t pair = pair0 + blockIdx.y;
  const int n = (int)(2 * pair);
  const bool has1 = n + 1 < g.N;
  const cx<T>* zp = Z + pair * b;
  cx<T>* ap = a + pair * b;
  for (int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x; k < b; k += (int64_t)gridDim.x * 256) {
    const int64_t km = (k == 0) ? 0 : b - k;
    const cx<T> zk = zp[k], zm = zp[km];
    const cx<double> Zk = mk<double>(zk.x, zk.y), Zm = mk<double>(zm.x, -zm.y);  // conj Z_{b-k}
    const cx<double> X1 = mk<double>(0.5 * (Zk.x + Zm.x), 0.5 * (Zk.y + Zm.y));
    const cx<double> D = mk<double>(0.5 * (Zk.x - Zm.x), 0.5 * (Zk.y - Zm.y));
    const cx<double> X2 = mk<double>(D.y, -D.x);  // D / i
    cx<double> Ga, Gc;
    blu_gain_pair4(g, n, has1, twb64[k], Ga, Gc);
    const cx<double> Y1 = cmul(Ga, X1);
    const cx<double> Y2 = has1 ? cmul(Gc, X2) : mk<double>(0.0, 0.0);
    const cx<double> zo = mk<double>(Y1.x - Y2.y, Y1.y + Y2.x);  // Y1 + i Y2
    const cx<T> c = chirp[k];
    const cx<double> out = cmul(zo, mk<double>(c.x, c.y));
    ap[k] = mk<T>(T(out.x), T(out.y));
  }
}

template <typename T>
__global__ __launch_bounds__(256) void k_blu_gain(const cx<T>* __restrict__ Z, cx<T>* __restrict__ a,
                                                  const cx<T>* __restrict__ chirp,
                                                  const cx<double>* __restrict__ twb64, int64_t b, int64_t pair0,
                                                  int64_t npairs, BluGain g) {
  const int64_t total = npairs * b;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < total; e += (int64_t)gridDim.x * 256) {
    const int64_t lp = e / b, k = e - lp * b, pair = pair0 + lp;
    const int64_t km = (k == 0) ? 0 : b - k;
    const cx<T> zk = Z[pair * b + k], zm = Z[pair * b + km];
    const cx<double> Zk = mk<double>(zk.x, zk.y), Zm = mk<double>(zm.x, -zm.y);  // conj Z_{b-k}
    const cx<double> X1 = mk<double>(0.5 * (Zk.x + Zm.x), 0.5 * (Zk.y + Zm.y));
    const cx<double> D = mk<double>(0.5 * (Zk.x - Zm.x), 0.5 * (Zk.y - Zm.y));
    const cx<double> X2 = mk<double>(D.y, -D.x);  // D / i
    const int n = (int)(2 * pair);
    const cx<double> Y1 = cmul(blu_gain(g, n, twb64, k), X1);
    cx<double> Y2 = mk<double>(0.0, 0.0);
    if (n + 1 < g.N) Y2 = cmul(blu_gain(g, n + 1, twb64, k), X2);
    const cx<double> zp = mk<double>(Y1.x - Y2.y, Y1.y + Y2.x);  // Y1 + i Y2
    const cx<T> c = chirp[k];
    const cx<double> out = cmul(zp, mk<double>(c.x, c.y));
    a[pair * b + k] = mk<T>(T(out.x), T(out.y));
  }
}

// The inverse transform of the first convolution, the gain and the forward
// transform of the second convolution in one pass over the four-step scratch.
// With b = q M2 + r, the partner b - j of j = j1 M2 + j2 (1 <= j < b) lies in
// column (r - j2) mod M2, row q - j1 - [j2 > r]; the columns pair up as
// u = ceil(r/2) + t and r - u (mod M2), t < M2/2 (+1 when r is even: then
// u = r/2 and u = r/2 + M2/2 are their own partners). A workgroup takes H
// consecutive t, i.e. up to 2H columns closed under the pairing, so each
// X_k meets X_{b-k} in LDS (k = 0 is its own partner). Per column: inverse
// M1-point DFT over k1, Z_j = conv_j conj(c_j) / M, the gain of the two
// packed real spectra, a_j = (G_n X1 + i G_{n+1} X2) c_j (zero for j >= b),
// forward M1-point DFT, twiddle w_M^{j2 k1}, back to the same columns.
template <int LOG2M1, int H>
struct BluMidCfg {
  static constexpr int M1 = 1 << LOG2M1;
  static constexpr int C = 2 * H;
  static constexpr int LS = lds_len(M1);
  static constexpr int NT0 = (M1 * C) / 8;
  static constexpr int NT = NT0 < 64 ? 64 : (NT0 > 512 ? 512 : NT0);
};

template <typename T, int LOG2M1, int H, bool TAP4>
__global__ __launch_bounds__((BluMidCfg<LOG2M1, H>::NT)) void k_blu_mid(
    cx<T>* __restrict__ Tm, const cx<T>* __restrict__ chirp, const cx<double>* __restrict__ twb64, int64_t b,
    int M2, int64_t pair0, BluGain g, BluTw tw) {
  using Cfg = BluMidCfg<LOG2M1, H>;
  constexpr int M1 = Cfg::M1, LS = Cfg::LS, NT = Cfg::NT, C = Cfg::C;
  __shared__ cx<T> s[C * LS];
  __shared__ cx<T> tlo[256], thi[256];
  __shared__ int col[C], mate[C];
  const int M = M1 * M2;
  blu_tw_lds<T, NT>(tlo, thi, tw, M);
  const int q = (int)(b / M2), r = (int)(b - (int64_t)q * M2);
  const int npc = (r & 1) ? M2 / 2 : M2 / 2 + 1;  // number of column pairs
  const int nrun = (npc + H - 1) / H;
  const int64_t lpair = blockIdx.x / nrun, pair = pair0 + lpair;
  const int t0 = (blockIdx.x % nrun) * H;
  const int c0 = (r + 1) / 2;
  if (threadIdx.x < H) {  // slot i: column u; slot H + i: its partner (-1: none)
    const int i = threadIdx.x;
    int u = -1, l = -1;
    if (t0 + i < npc) {
      u = (c0 + t0 + i) & (M2 - 1);
      l = (r - u) & (M2 - 1);
      if (l == u) l = -1;
    }
    col[i] = u;
    col[H + i] = l;
    mate[i] = (l >= 0) ? H + i : i;
    mate[H + i] = i;
  }
  __syncthreads();
  cx<T>* tp = Tm + lpair * (int64_t)M;
  for (int e = threadIdx.x; e < M1 * C; e += NT) {
    const int sl = e % C, k1 = e / C;
    const int j2 = col[sl];
    s[sl * LS + pidx(k1)] = (j2 >= 0) ? tp[(int64_t)k1 * M2 + j2] : mk<T>(T(0), T(0));
  }
  __syncthreads();
  lds_fft<T, M1, NT, C, +1>(s, LS, reinterpret_cast<const cx<T>*>(tw.tM1), 1);
  // Each pair {j, b - j} is done by the thread holding its smaller member: the
  // gains at b - j are the conjugates of those at j (real taps), so
  // a_j = (Y1 + i Y2) c_j and a_{b-j} = (conj Y1 + i conj Y2) c_{b-j} with
  // Y1 = G_n(j) X1(j), Y2 = G_{n+1}(j) X2(j). Rows j >= b become zero.
  const int n = (int)(2 * pair);
  const bool has1 = n + 1 < g.N;
  const double invM = 1.0 / (double)M;
#pragma unroll 1
  for (int e = threadIdx.x; e < M1 * C; e += NT) {
    const int sl = e % C, j1 = e / C;
    const int j2 = col[sl];
    if (j2 < 0) continue;
    const int64_t j = (int64_t)j1 * M2 + j2;
    cx<T>* sj = s + sl * LS + pidx(j1);
    if (j >= b) {
      *sj = mk<T>(T(0), T(0));
      continue;
    }
    const int64_t jm = (j == 0) ? 0 : b - j;
    if (jm < j) continue;  // the partner's thread does this pair
    cx<T>* sm = sj;
    if (jm != j) sm = s + mate[sl] * LS + pidx(q - j1 - (j2 > r ? 1 : 0));
    const cx<T> cj = chirp[j], cm = chirp[jm];
    const cx<double> c = mk<double>(cj.x, cj.y), cmd = mk<double>(cm.x, cm.y);
    const cx<T> v = *sj, w = *sm;
    const cx<double> Zk = cmulc(mk<double>(v.x * invM, v.y * invM), c);
    const cx<double> Zm = cmulc(mk<double>(w.x * invM, w.y * invM), cmd);
    // X1 = (Z_j + conj Z_{b-j}) / 2, X2 = (Z_j - conj Z_{b-j}) / 2i
    const cx<double> X1 = mk<double>(0.5 * (Zk.x + Zm.x), 0.5 * (Zk.y - Zm.y));
    const cx<double> X2 = mk<double>(0.5 * (Zk.y + Zm.y), -0.5 * (Zk.x - Zm.x));
    cx<double> Ga, Gc;
    if constexpr (TAP4) {
      blu_gain_pair4(g, n, has1, twb64[j], Ga, Gc);
    } else {
      Ga = blu_gain(g, n, twb64, j);
      Gc = has1 ? blu_gain(g, n + 1, twb64, j) : mk<double>(0.0, 0.0);
    }
    const cx<double> Y1 = cmul(Ga, X1);
    const cx<double> Y2 = has1 ? cmul(Gc, X2) : mk<double>(0.0, 0.0);
    const cx<double> oj = cmul(mk<double>(Y1.x - Y2.y, Y1.y + Y2.x), c);  // (Y1 + i Y2) c_j
    *sj = mk<T>(T(oj.x), T(oj.y));
    if (jm != j) {
      const cx<double> om = cmul(mk<double>(Y1.x + Y2.y, -Y1.y + Y2.x), cmd);  // (conj Y1 + i conj Y2) c_{b-j}
      *sm = mk<T>(T(om.x), T(om.y));
    }
  }
  __syncthreads();
  lds_fft<T, M1, NT, C, -1>(s, LS, reinterpret_cast<const cx<T>*>(tw.tM1), 1);
  for (int e = threadIdx.x; e < M1 * C; e += NT) {
    const int sl = e % C, k1 = e / C;
    const int j2 = col[sl];
    if (j2 < 0) continue;
    tp[(int64_t)k1 * M2 + j2] = cmul(s[sl * LS + pidx(k1)], blu_twM(tlo, thi, j2 * k1));
  }
}

// ---- natural layout ----------------------------------------------------------
// The same convolutions computed in place on the frame matrix d[j][n] (as
// the rows left it): a tile of TP adjacent column pairs (128 bytes of every
// frame) is the unit of work, and the scratch of a launch group of tiles is
// laid out T[tile][k1][j2][q] (q the pair within the tile), so every access
// is a 128-byte run and no transpose is needed:
//   A  (tile, j2): d[j1 M2 + j2][tile] conj(c_j) -> M1-point FFT over j1 -> twiddle
//   B  (tile, k1): M2-point FFT over j2, times the filter spectrum (shared by
//                  the tile's pairs), inverse FFT, conjugate twiddle
//   M  (tile, column j2 and its partner): inverse over k1, gain, forward over j1
//   A' (tile, j2): inverse FFT over k1 -> c_j / (M b) -> d[j][tile] = x
template <typename T, int LOG2M>
struct BnCfg {
  static constexpr int TP = 128 / (int)sizeof(cx<T>);
  static constexpr int L = 1 << LOG2M;
  static constexpr int LS = lds_len(L);
  static constexpr int cl(int v) { return v < 64 ? 64 : (v > 1024 ? 1024 : v); }
  // 8 elements per thread in the FFT passes; 16 in the middle pass, whose
  // FP64 gain work favours fewer, fuller threads
  static constexpr int NT = cl(TP * L / 8);        // one sequence set of TP pairs
  static constexpr int NT2 = cl(2 * TP * L / 16);  // two columns' sets (the middle pass)
};

template <typename T, int LOG2M1>
__global__ __launch_bounds__((BnCfg<T, LOG2M1>::NT)) void k_bn_A(const cx<T>* __restrict__ x,
                                                                   cx<T>* __restrict__ Tm,
                                                                   const cx<T>* __restrict__ chirp, int64_t b,
                                                                   int M2, int np, int t0, int ntc, BluTw tw) {
  using Cfg = BnCfg<T, LOG2M1>;
  constexpr int TP = Cfg::TP, M1 = Cfg::L, LS = Cfg::LS, NT = Cfg::NT;
  __shared__ cx<T> s[TP * LS];
  __shared__ cx<T> tlo[256], thi[256];
  const int M = M1 * M2;
  blu_tw_lds<T, NT>(tlo, thi, tw, M);
  const int tl = blockIdx.x % ntc, j2 = blockIdx.x / ntc;
  const int p0 = (t0 + tl) * TP;
  for (int e = threadIdx.x; e < TP * M1; e += NT) {
    const int q = e % TP, j1 = e / TP;
    const int64_t j = (int64_t)j1 * M2 + j2;
    cx<T> v = mk<T>(T(0), T(0));
    if (j < b && p0 + q < np) v = cmulc(x[j * np + p0 + q], chirp[j]);
    s[q * LS + pidx(j1)] = v;
  }
  __syncthreads();
  lds_fft<T, M1, NT, TP, -1>(s, LS, reinterpret_cast<const cx<T>*>(tw.tM1), 1);
  cx<T>* tp = Tm + (int64_t)tl * M * TP;
  for (int e = threadIdx.x; e < TP * M1; e += NT) {
    const int q = e % TP, k1 = e / TP;
    tp[((int64_t)k1 * M2 + j2) * TP + q] = cmul(s[q * LS + pidx(k1)], blu_twM(tlo, thi, j2 * k1));
  }
}

template <typename T, int LOG2M2>
__global__ __launch_bounds__((BnCfg<T, LOG2M2>::NT)) void k_bn_B(cx<T>* __restrict__ Tm,
                                                                   const cx<T>* __restrict__ Crow, int conjC,
                                                                   int M1, int ntc, BluTw tw) {
  using Cfg = BnCfg<T, LOG2M2>;
  constexpr int TP = Cfg::TP, M2 = Cfg::L, LS = Cfg::LS, NT = Cfg::NT;
  __shared__ cx<T> s[TP * LS];
  __shared__ cx<T> tlo[256], thi[256];
  const int M = M1 * M2;
  blu_tw_lds<T, NT>(tlo, thi, tw, M);
  const int tl = blockIdx.x % ntc, k1 = blockIdx.x / ntc;
  cx<T>* tp = Tm + (int64_t)tl * M * TP + (int64_t)k1 * M2 * TP;  // row k1: [j2][q], contiguous
  for (int e = threadIdx.x; e < TP * M2; e += NT) s[(e % TP) * LS + pidx(e / TP)] = tp[e];
  __syncthreads();
  const cx<T>* tM2 = reinterpret_cast<const cx<T>*>(tw.tM2);
  lds_fft<T, M2, NT, TP, -1>(s, LS, tM2, 1);
  for (int e = threadIdx.x; e < TP * M2; e += NT) {  // times C[k1 + M1 k2], the same for every pair
    const int q = e % TP, k2 = e / TP;
    cx<T> h = Crow[(int64_t)k1 * M2 + k2];
    if (conjC) h.y = -h.y;
    s[q * LS + pidx(k2)] = cmul(s[q * LS + pidx(k2)], h);
  }
  __syncthreads();
  lds_fft<T, M2, NT, TP, +1>(s, LS, tM2, 1);
  for (int e = threadIdx.x; e < TP * M2; e += NT) {
    const int q = e % TP, j2 = e / TP;
    tp[e] = cmulc(s[q * LS + pidx(j2)], blu_twM(tlo, thi, j2 * k1));
  }
}

// Middle pass on one column u and its partner (r - u) mod M2 (see k_blu_mid),
// for the TP pairs of a tile; slot 0 holds column u, slot 1 its partner.
template <typename T, int LOG2M1, bool TAP4>
__global__ __launch_bounds__((BnCfg<T, LOG2M1>::NT2)) void k_bn_mid(
    cx<T>* __restrict__ Tm, const cx<T>* __restrict__ chirp, const cx<double>* __restrict__ twb64, int64_t b,
    int M2, int np, int t0, int ntc, BluGain g, BluTw tw) {
  using Cfg = BnCfg<T, LOG2M1>;
  constexpr int TP = Cfg::TP, M1 = Cfg::L, LS = Cfg::LS, NT = Cfg::NT2, C = 2 * TP;
  __shared__ cx<T> s[C * LS];
  __shared__ cx<T> tlo[256], thi[256];
  const int M = M1 * M2;
  blu_tw_lds<T, NT>(tlo, thi, tw, M);
  const int qb = (int)(b / M2), r = (int)(b - (int64_t)qb * M2);
  const int tl = blockIdx.x % ntc, t = blockIdx.x / ntc;
  const int p0 = (t0 + tl) * TP;
  const int u = (((r + 1) / 2) + t) & (M2 - 1);
  int l = (r - u) & (M2 - 1);
  const bool own = (l == u);  // u is its own partner
  if (own) l = -1;
  cx<T>* tp = Tm + (int64_t)tl * M * TP;
  for (int e = threadIdx.x; e < C * M1; e += NT) {
    const int q = e % TP, rest = e / TP, sl = rest & 1, k1 = rest >> 1;
    const int j2 = sl ? l : u;
    s[(sl * TP + q) * LS + pidx(k1)] = (j2 >= 0) ? tp[((int64_t)k1 * M2 + j2) * TP + q] : mk<T>(T(0), T(0));
  }
  __syncthreads();
  lds_fft<T, M1, NT, C, +1>(s, LS, reinterpret_cast<const cx<T>*>(tw.tM1), 1);
  const double invM = 1.0 / (double)M;
#pragma unroll 1
  for (int e = threadIdx.x; e < C * M1; e += NT) {
    const int q = e % TP, rest = e / TP, sl = rest & 1, j1 = rest >> 1;
    const int j2 = sl ? l : u;
    if (j2 < 0) continue;
    cx<T>* sj = s + (sl * TP + q) * LS + pidx(j1);
    const int64_t j = (int64_t)j1 * M2 + j2;
    if (j >= b || p0 + q >= np) {
      *sj = mk<T>(T(0), T(0));
      continue;
    }
    const int64_t jm = (j == 0) ? 0 : b - j;
    if (jm < j) continue;  // the partner's thread does this pair
    cx<T>* sm = sj;
    if (jm != j) sm = s + ((own ? sl : 1 - sl) * TP + q) * LS + pidx(qb - j1 - (j2 > r ? 1 : 0));
    const int n = 2 * (p0 + q);
    const bool has1 = n + 1 < g.N;
    const cx<T> cj = chirp[j], cm = chirp[jm];
    const cx<double> c = mk<double>(cj.x, cj.y), cmd = mk<double>(cm.x, cm.y);
    const cx<T> v = *sj, w = *sm;
    const cx<double> Zk = cmulc(mk<double>(v.x * invM, v.y * invM), c);
    const cx<double> Zm = cmulc(mk<double>(w.x * invM, w.y * invM), cmd);
    const cx<double> X1 = mk<double>(0.5 * (Zk.x + Zm.x), 0.5 * (Zk.y - Zm.y));
    const cx<double> X2 = mk<double>(0.5 * (Zk.y + Zm.y), -0.5 * (Zk.x - Zm.x));
    cx<double> Ga, Gc;
    if constexpr (TAP4) {
      blu_gain_pair4(g, n, has1, twb64[j], Ga, Gc);
    } else {
      Ga = blu_gain(g, n, twb64, j);
      Gc = has1 ? blu_gain(g, n + 1, twb64, j) : mk<double>(0.0, 0.0);
    }
    const cx<double> Y1 = cmul(Ga, X1);
    const cx<double> Y2 = has1 ? cmul(Gc, X2) : mk<double>(0.0, 0.0);
    const cx<double> oj = cmul(mk<double>(Y1.x - Y2.y, Y1.y + Y2.x), c);
    *sj = mk<T>(T(oj.x), T(oj.y));
    if (jm != j) {
      const cx<double> om = cmul(mk<double>(Y1.x + Y2.y, -Y1.y + Y2.x), cmd);
      *sm = mk<T>(T(om.x), T(om.y));
    }
  }
  __syncthreads();
  lds_fft<T, M1, NT, C, -1>(s, LS, reinterpret_cast<const cx<T>*>(tw.tM1), 1);
  for (int e = threadIdx.x; e < C * M1; e += NT) {
    const int q = e % TP, rest = e / TP, sl = rest & 1, k1 = rest >> 1;
    const int j2 = sl ? l : u;
    if (j2 < 0) continue;
    tp[((int64_t)k1 * M2 + j2) * TP + q] = cmul(s[(sl * TP + q) * LS + pidx(k1)], blu_twM(tlo, thi, j2 * k1));
  }
}

template <typename T, int LOG2M1>
__global__ __launch_bounds__((BnCfg<T, LOG2M1>::NT)) void k_bn_Ainv(const cx<T>* __restrict__ Tm,
                                                                      cx<T>* __restrict__ x,
                                                                      const cx<T>* __restrict__ chirp, int64_t b,
                                                                      int M2, int np, int t0, int ntc, BluTw tw) {
  using Cfg = BnCfg<T, LOG2M1>;
  constexpr int TP = Cfg::TP, M1 = Cfg::L, LS = Cfg::LS, NT = Cfg::NT;
  __shared__ cx<T> s[TP * LS];
  const int M = M1 * M2;
  const int tl = blockIdx.x % ntc, j2 = blockIdx.x / ntc;
  const int p0 = (t0 + tl) * TP;
  const cx<T>* tp = Tm + (int64_t)tl * M * TP;
  for (int e = threadIdx.x; e < TP * M1; e += NT) {
    const int q = e % TP, k1 = e / TP;
    s[q * LS + pidx(k1)] = tp[((int64_t)k1 * M2 + j2) * TP + q];
  }
  __syncthreads();
  lds_fft<T, M1, NT, TP, +1>(s, LS, reinterpret_cast<const cx<T>*>(tw.tM1), 1);
  const T sc = T(1.0 / ((double)M * (double)b));
  for (int e = threadIdx.x; e < TP * M1; e += NT) {
    const int q = e % TP, j1 = e / TP;
    const int64_t j = (int64_t)j1 * M2 + j2;
    if (j >= b || p0 + q >= np) continue;
    x[j * np + p0 + q] = cmul(scale(s[q * LS + pidx(j1)], sc), chirp[j]);
  }
}

// ---- launchers ---------------------------------------------------------------
// Tile widths other than 16 exist for M1, M2 >= 2^kBluTileMinLog2 only.
constexpr int kBluTileMinLog2 = 5;

template <typename T, int L1, int MB>
static hipError_t launch_blu_A_t(int mode, const void* in, void* Tm, const void* chirp, int64_t b, int M2, int N,
                                 int64_t pair0, int64_t npairs, const BluTw& tw, hipStream_t st) {
  using Cfg = BluACfg<L1, MB>;
  const int mb_eff = M2 < Cfg::MB ? M2 : Cfg::MB;
  const dim3 grid((unsigned)(npairs * (M2 / mb_eff)));
  if (mode == 0)
    k_blu_A<T, L1, MB, 0><<<grid, Cfg::NT, 0, st>>>(in, (cx<T>*)Tm, (const cx<T>*)chirp, b, M2, N, pair0, tw);
  else
    k_blu_A<T, L1, MB, 1><<<grid, Cfg::NT, 0, st>>>(in, (cx<T>*)Tm, (const cx<T>*)chirp, b, M2, N, pair0, tw);
  return hipGetLastError();
}

template <typename T, int L1, int MB>
static hipError_t launch_blu_Ainv_t(int mode, const void* Tm, void* out, const void* chirp, int64_t b, int M2,
                                    int N, int64_t pair0, int64_t npairs, const BluTw& tw, hipStream_t st) {
  using Cfg = BluACfg<L1, MB>;
  const int mb_eff = M2 < Cfg::MB ? M2 : Cfg::MB;
  const dim3 grid((unsigned)(npairs * (M2 / mb_eff)));
  if (mode == 0)
    k_blu_Ainv<T, L1, MB, 0><<<grid, Cfg::NT, 0, st>>>((const cx<T>*)Tm, out, (const cx<T>*)chirp, b, M2, N, pair0,
                                                       tw);
  else
    k_blu_Ainv<T, L1, MB, 1><<<grid, Cfg::NT, 0, st>>>((const cx<T>*)Tm, out, (const cx<T>*)chirp, b, M2, N, pair0,
                                                       tw);
  return hipGetLastError();
}

template <typename T, int L2, int KB>
static hipError_t launch_blu_B_t(void* Tm, const void* Crow, int conjC, int M1, int64_t npairs, const BluTw& tw,
                                 hipStream_t st) {
  using Cfg = BluBCfg<L2, KB>;
  const int kb_eff = M1 < Cfg::KB ? M1 : Cfg::KB;
  const dim3 grid((unsigned)(npairs * (M1 / kb_eff)));
  k_blu_B<T, L2, KB><<<grid, Cfg::NT, 0, st>>>((cx<T>*)Tm, (const cx<T>*)Crow, conjC, M1, tw);
  return hipGetLastError();
}

// One A (fwd = 1) or A' (fwd = 0) launch with tile width mb.
template <typename T, int L1>
static hipError_t blu_col_pass(int fwd, int mb, int mode, const void* in, void* out, const void* chirp, int64_t b,
                               int M2, int N, int64_t pair0, int64_t npairs, const BluTw& tw, hipStream_t st) {
  if (L1 < kBluTileMinLog2) mb = 16;
  switch (mb) {
#define BLU_CASE(MB)                                                                                          \
  case MB:                                                                                                   \
    return fwd ? launch_blu_A_t<T, L1, (L1 < kBluTileMinLog2 ? 16 : MB)>(mode, in, out, chirp, b, M2, N,     \
                                                                         pair0, npairs, tw, st)              \
               : launch_blu_Ainv_t<T, L1, (L1 < kBluTileMinLog2 ? 16 : MB)>(mode, in, out, chirp, b, M2, N,  \
                                                                            pair0, npairs, tw, st);
    BLU_CASE(8) BLU_CASE(16) BLU_CASE(32)
#undef BLU_CASE
    default: return hipErrorInvalidValue;
  }
}

template <typename T, int L2>
static hipError_t blu_row_pass(int kb, void* Tm, const void* Crow, int conjC, int M1, int64_t npairs,
                               const BluTw& tw, hipStream_t st) {
  if (L2 < kBluTileMinLog2) kb = 16;
  switch (kb) {
#define BLU_CASE(KB) \
  case KB: return launch_blu_B_t<T, L2, (L2 < kBluTileMinLog2 ? 16 : KB)>(Tm, Crow, conjC, M1, npairs, tw, st);
    BLU_CASE(8) BLU_CASE(16) BLU_CASE(32)
#undef BLU_CASE
    default: return hipErrorInvalidValue;
  }
}

#define BLU_L_SWITCH(L, CALL)                               \
  switch (L) {                                              \
    case 1: CALL(1) case 2: CALL(2) case 3: CALL(3)         \
    case 4: CALL(4) case 5: CALL(5) case 6: CALL(6)         \
    case 7: CALL(7) case 8: CALL(8)                         \
    default: return hipErrorInvalidValue;                   \
  }

// The steps of one cyclic convolution of length M = 2^l1 * 2^(log2m - l1)
// for pairs [pair0, pair0 + npairs): step 0 = A, 1 = B, 2 = A'.
template <typename T>
static hipError_t blu_step(int step, int mode, const void* in, void* out, void* Tm, const void* chirp,
                           const void* Crow, int conjC, int64_t b, int log2m, const BluCfg& cfg, int N,
                           int64_t pair0, int64_t npairs, const BluTw& tw, hipStream_t st) {
  const int l1 = cfg.l1, l2 = log2m - cfg.l1;
  const int M1 = 1 << l1, M2 = 1 << l2;
  hipError_t e = hipErrorInvalidValue;
  if (step == 0) {
#define CALL_A(L) \
  e = blu_col_pass<T, L>(1, cfg.mb, mode, in, Tm, chirp, b, M2, N, pair0, npairs, tw, st); break;
    BLU_L_SWITCH(l1, CALL_A)
#undef CALL_A
  } else if (step == 1) {
#define CALL_B(L) e = blu_row_pass<T, L>(cfg.kb, Tm, Crow, conjC, M1, npairs, tw, st); break;
    BLU_L_SWITCH(l2, CALL_B)
#undef CALL_B
  } else {
#define CALL_AI(L) \
  e = blu_col_pass<T, L>(0, cfg.mb, mode, Tm, out, chirp, b, M2, N, pair0, npairs, tw, st); break;
    BLU_L_SWITCH(l1, CALL_AI)
#undef CALL_AI
  }
  return e;
}

template <typename T, int L1, int H>
static hipError_t launch_blu_mid_t(void* Tm, const void* chirp, const double* twb64, int64_t b, int M2,
                                   int64_t pair0, int64_t npairs, const BluGain& g, const BluTw& tw,
                                   hipStream_t st) {
  using Cfg = BluMidCfg<L1, H>;
  const int r = (int)(b % M2);
  const int Tp = (r & 1) ? M2 / 2 : M2 / 2 + 1;
  const dim3 grid((unsigned)(npairs * ((Tp + H - 1) / H)));
  if (g.ntap == 4)
    k_blu_mid<T, L1, H, true><<<grid, Cfg::NT, 0, st>>>((cx<T>*)Tm, (const cx<T>*)chirp, (const cx<double>*)twb64,
                                                         b, M2, pair0, g, tw);
  else
    k_blu_mid<T, L1, H, false><<<grid, Cfg::NT, 0, st>>>((cx<T>*)Tm, (const cx<T>*)chirp,
                                                          (const cx<double>*)twb64, b, M2, pair0, g, tw);
  return hipGetLastError();
}

template <typename T, int L1>
static hipError_t blu_mid_pass(int mb, void* Tm, const void* chirp, const double* twb64, int64_t b, int M2,
                               int64_t pair0, int64_t npairs, const BluGain& g, const BluTw& tw, hipStream_t st) {
  if (L1 < kBluTileMinLog2) mb = 16;
  switch (mb) {
#define BLU_CASE(MB)                                                                                        \
  case MB:                                                                                                 \
    return launch_blu_mid_t<T, L1, (L1 < kBluTileMinLog2 ? 8 : MB / 2)>(Tm, chirp, twb64, b, M2, pair0,    \
                                                                        npairs, g, tw, st);
    BLU_CASE(8) BLU_CASE(16) BLU_CASE(32)
#undef BLU_CASE
    default: return hipErrorInvalidValue;
  }
}

// ---- natural-layout launchers
template <typename T, int L1>
static hipError_t launch_bn_A_t(const void* x, void* Tm, const void* chirp, int64_t b, int M2, int np, int t0, int ntc,
                                const BluTw& tw, hipStream_t st) {
  k_bn_A<T, L1><<<dim3((unsigned)(ntc * M2)), BnCfg<T, L1>::NT, 0, st>>>((const cx<T>*)x, (cx<T>*)Tm,
                                                                         (const cx<T>*)chirp, b, M2, np, t0, ntc, tw);
  return hipGetLastError();
}
template <typename T, int L2>
static hipError_t launch_bn_B_t(void* Tm, const void* Crow, int conjC, int M1, int ntc, const BluTw& tw,
                                hipStream_t st) {
  k_bn_B<T, L2><<<dim3((unsigned)(ntc * M1)), BnCfg<T, L2>::NT, 0, st>>>((cx<T>*)Tm, (const cx<T>*)Crow, conjC, M1,
                                                                         ntc, tw);
  return hipGetLastError();
}
template <typename T, int L1>
static hipError_t launch_bn_mid_t(void* Tm, const void* chirp, const double* twb64, int64_t b, int M2, int np, int t0,
                                  int ntc, const BluGain& g, const BluTw& tw, hipStream_t st) {
  const int r = (int)(b % M2);
  const int npc = (r & 1) ? M2 / 2 : M2 / 2 + 1;
  const dim3 grid((unsigned)(ntc * npc));
  if (g.ntap == 4)
    k_bn_mid<T, L1, true><<<grid, BnCfg<T, L1>::NT2, 0, st>>>((cx<T>*)Tm, (const cx<T>*)chirp,
                                                              (const cx<double>*)twb64, b, M2, np, t0, ntc, g, tw);
  else
    k_bn_mid<T, L1, false><<<grid, BnCfg<T, L1>::NT2, 0, st>>>((cx<T>*)Tm, (const cx<T>*)chirp,
                                                               (const cx<double>*)twb64, b, M2, np, t0, ntc, g, tw);
  return hipGetLastError();
}
template <typename T, int L1>
static hipError_t launch_bn_Ainv_t(const void* Tm, void* x, const void* chirp, int64_t b, int M2, int np, int t0,
                                   int ntc, const BluTw& tw, hipStream_t st) {
  k_bn_Ainv<T, L1><<<dim3((unsigned)(ntc * M2)), BnCfg<T, L1>::NT, 0, st>>>((const cx<T>*)Tm, (cx<T>*)x,
                                                                            (const cx<T>*)chirp, b, M2, np, t0, ntc,
                                                                            tw);
  return hipGetLastError();
}

template <typename T>
static hipError_t blu_nat_t(void* x, void* Tm, const void* chirp, const void* Crow, const double* twb64, int64_t b,
                            int log2m, const BluCfg& cfg, int N, const BluGain& g, const BluTw& tw, hipStream_t st) {
  constexpr int TP = BnCfg<T, 1>::TP;
  const int l1 = cfg.l1, l2 = log2m - cfg.l1;
  const int M1 = 1 << l1, M2 = 1 << l2;
  const int np = N / 2, nt = (np + TP - 1) / TP;
  const int ch = (cfg.pchunk > 0 && cfg.pchunk < nt) ? cfg.pchunk : nt;
  hipError_t e = hipSuccess;
  for (int t0 = 0; t0 < nt && e == hipSuccess; t0 += ch) {
    const int ntc = nt - t0 < ch ? nt - t0 : ch;
#define CALL(L) e = launch_bn_A_t<T, L>(x, Tm, chirp, b, M2, np, t0, ntc, tw, st); break;
    BLU_L_SWITCH(l1, CALL)
#undef CALL
    if (e != hipSuccess) break;
#define CALL(L) e = launch_bn_B_t<T, L>(Tm, Crow, 0, M1, ntc, tw, st); break;
    BLU_L_SWITCH(l2, CALL)
#undef CALL
    if (e != hipSuccess) break;
#define CALL(L) e = launch_bn_mid_t<T, L>(Tm, chirp, twb64, b, M2, np, t0, ntc, g, tw, st); break;
    BLU_L_SWITCH(l1, CALL)
#undef CALL
    if (e != hipSuccess) break;
#define CALL(L) e = launch_bn_B_t<T, L>(Tm, Crow, 1, M1, ntc, tw, st); break;
    BLU_L_SWITCH(l2, CALL)
#undef CALL
    if (e != hipSuccess) break;
#define CALL(L) e = launch_bn_Ainv_t<T, L>(Tm, x, chirp, b, M2, np, t0, ntc, tw, st); break;
    BLU_L_SWITCH(l1, CALL)
#undef CALL
  }
  return e;
}

bool blu_cfg_valid(int log2m, const BluCfg& c) {
  const int l2 = log2m - c.l1;
  if (log2m < 2 || log2m > kBluMaxLog2M) return false;
  if (c.l1 < 1 || c.l1 > 8 || l2 < 1 || l2 > 8) return false;
  if (c.mb != 8 && c.mb != 16 && c.mb != 32) return false;
  if (c.kb != 8 && c.kb != 16 && c.kb != 32) return false;
  if (c.fuse != 0 && c.fuse != 1) return false;
  if (c.nat != 0 && c.nat != 1) return false;
  return c.pchunk >= 0;
}

BluCfg blu_cfg_default(int log2m) {
  BluCfg c;
  c.l1 = (log2m + 1) / 2;
  c.mb = 16;
  c.kb = 16;
  c.pchunk = 0;
  c.fuse = 1;
  c.nat = 0;
  return c;
}

template <typename T>
static hipError_t blu_columns_t(const void* dT, void* xT, void* Tm, void* Z, void* A, const void* chirp,
                                const void* Crow, const double* twb64, int64_t b, int log2m, const BluCfg& cfg,
                                int N, int ntap, const BluGain& g, const BluTw& tw, hipStream_t st) {
  const int64_t npairs = (N + 1) / 2;
  const int64_t chunk = (cfg.pchunk > 0 && cfg.pchunk < npairs) ? cfg.pchunk : npairs;
  hipError_t e = hipSuccess;
  for (int64_t p0 = 0; p0 < npairs && e == hipSuccess; p0 += chunk) {
    const int64_t np = (npairs - p0) < chunk ? (npairs - p0) : chunk;
    e = blu_step<T>(0, 0, dT, nullptr, Tm, chirp, Crow, 0, b, log2m, cfg, N, p0, np, tw, st);
    if (e == hipSuccess) e = blu_step<T>(1, 0, nullptr, nullptr, Tm, chirp, Crow, 0, b, log2m, cfg, N, p0, np, tw, st);
    if (e != hipSuccess) break;
    if (cfg.fuse) {
      const int M2 = 1 << (log2m - cfg.l1);
#define CALL_M(L) e = blu_mid_pass<T, L>(cfg.mb, Tm, chirp, twb64, b, M2, p0, np, g, tw, st); break;
      BLU_L_SWITCH(cfg.l1, CALL_M)
#undef CALL_M
      if (e == hipSuccess) e = blu_step<T>(1, 0, nullptr, nullptr, Tm, chirp, Crow, 1, b, log2m, cfg, N, p0, np, tw, st);
      if (e == hipSuccess) e = blu_step<T>(2, 1, nullptr, xT, Tm, chirp, Crow, 1, b, log2m, cfg, N, p0, np, tw, st);
      continue;
    }
    e = blu_step<T>(2, 0, nullptr, Z, Tm, chirp, Crow, 0, b, log2m, cfg, N, p0, np, tw, st);
    if (e != hipSuccess) break;
    if (ntap == 4 && np <= 65535) {
      // 4 taps: one pair per grid row, no division per element
      const dim3 grid((unsigned)((b + 255) / 256 < 64 ? (b + 255) / 256 : 64), (unsigned)np);
      k_blu_gain2<T><<<grid, 256, 0, st>>>((const cx<T>*)Z, (cx<T>*)A, (const cx<T>*)chirp,
                                           (const cx<double>*)twb64, b, p0, g);
    } else {
      const unsigned grid = (unsigned)((np * b + 255) / 256 < 4096 ? (np * b + 255) / 256 : 4096);
      k_blu_gain<T><<<grid, 256, 0, st>>>((const cx<T>*)Z, (cx<T>*)A, (const cx<T>*)chirp,
                                          (const cx<double>*)twb64, b, p0, np, g);
    }
    e = hipGetLastError();
    for (int step = 0; step < 3 && e == hipSuccess; ++step)
      e = blu_step<T>(step, 1, A, xT, Tm, chirp, Crow, 1, b, log2m, cfg, N, p0, np, tw, st);
  }
  return e;
}

int blu_nat_tile_pairs(int prec) { return prec == F32 ? BnCfg<float, 1>::TP : BnCfg<double, 1>::TP; }

hipError_t launch_blu_nat(int prec, void* x, void* Tm, const void* chirp, const void* Crow, const double* twb64,
                          int64_t b, int log2m, const BluCfg& cfg, int N, int ntap, const double* win64, double phi,
                          int normalise, const void* const tw4[4], hipStream_t st) {
  if (!blu_cfg_valid(log2m, cfg) || (N & 1)) return hipErrorInvalidValue;
  BluTw tw{tw4[0], tw4[1], tw4[2], tw4[3]};
  BluGain g;
  g.win = win64;
  g.N = N;
  g.ntap = ntap;
  g.phi2 = phi * phi;
  g.gnorm = normalise ? 1.0 + phi * phi : 1.0;
  g.naive = (phi == 0.0);
  if (prec == F32) return blu_nat_t<float>(x, Tm, chirp, Crow, twb64, b, log2m, cfg, N, g, tw, st);
  return blu_nat_t<double>(x, Tm, chirp, Crow, twb64, b, log2m, cfg, N, g, tw, st);
}

hipError_t launch_blu_columns(int prec, const void* dT, void* xT, void* Tm, void* Z, void* A, const void* chirp,
                              const void* Crow, const double* twb64, int64_t b, int log2m, const BluCfg& cfg,
                              int N, int ntap, const double* win64, double phi, int normalise,
                              const void* const tw4[4], hipStream_t st) {
  if (!blu_cfg_valid(log2m, cfg)) return hipErrorInvalidValue;
  BluTw tw{tw4[0], tw4[1], tw4[2], tw4[3]};
  BluGain g;
  g.win = win64;
  g.N = N;
  g.ntap = ntap;
  g.phi2 = phi * phi;
  g.gnorm = normalise ? 1.0 + phi * phi : 1.0;
  g.naive = (phi == 0.0);
  if (prec == F32)
    return blu_columns_t<float>(dT, xT, Tm, Z, A, chirp, Crow, twb64, b, log2m, cfg, N, ntap, g, tw, st);
  return blu_columns_t<double>(dT, xT, Tm, Z, A, chirp, Crow, twb64, b, log2m, cfg, N, ntap, g, tw, st);
}

}  // namespace ipfb
