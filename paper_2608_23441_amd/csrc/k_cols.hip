// Column stage of the circulant inverse PFB (Section 3.1, the decorrelation
// x_n = F^dagger[ F d_n / (F w_n)^* ], with the Wiener weights of Section 4.1):
// for every sub-filter path n, a b-point FFT down column n of d, a pointwise
// FP64 gain, and the inverse FFT, written back in time order.
//
// The frame matrix arrives transposed (d_T[n][j], each column contiguous, from
// a tiled transpose of the row stage's output) and the result leaves the same
// way (x_T[n][j]); every global access is a contiguous run. One workgroup owns
// C columns. A real column of b samples becomes a b/2-point complex sequence
// z[m] = d_T[n][2m] + i d_T[n][2m+1]; after the forward
// FFT, the pass that separates the real spectrum X[k], applies the gain and
// re-packs for the inverse touches the pair (k, b/2-k) in one thread, in
// double precision. The gain is computed on the fly from the p taps of the
// column,  W_n(f) = sum_r h[rN+n] e^{-2 pi i r f / b},
//          G = W (1+phi^2) / (|W|^2 + phi^2) / b,
// so no N x b table ever touches HBM.
#include "fft_lds.hpp"
#include "launch.hpp"
#include "reduce.hpp"

namespace ipfb {

template <typename T, int LOG2B>
struct ColCfg {
  static constexpr int H = 1 << (LOG2B - 1);
  static constexpr int BYTES = H * (int)sizeof(cx<T>);
  static constexpr int C0 = 65536 / BYTES;  // 64 KiB of data: two workgroups per CU
  static constexpr int C = C0 < 1 ? 1 : (C0 > 16 ? 16 : C0);  // columns per workgroup
  static constexpr int LS = lds_len(H);                       // padded LDS stride
  static constexpr int EPT = sizeof(T) == 4 ? 16 : 8;
  static constexpr int NT0 = (H * C) / EPT;
  static constexpr int NT = NT0 < 64 ? 64 : (NT0 > 1024 ? 1024 : NT0);
  // waves per SIMD to keep: two workgroups per CU when their LDS allows it
  static constexpr int LDSB = C * LS * (int)sizeof(cx<T>);
  static constexpr int WPE0 = (LDSB <= 81920 ? 2 : 1) * (NT / 64) / 4;
  static constexpr int WPE = WPE0 < 1 ? 1 : WPE0;
};

struct GainArgs {
  const double* win;  // [ntap][lblock], FP64
  int lblock, ntap;
  double phi2;        // phi^2
  double gnorm;       // (1 + phi^2) / b  (or 1/b without the normalisation)
  int naive;          // phi == 0: 1/conj(W), truncated
  int precond;        // real gain 1/(|W|^2 + phi^2) / b: the inverse of A^T A + phi^2 I
};

// G_n(f) for f in [0, b); twB64[m] = e^{-2 pi i m / b}.
template <int B>
__device__ __forceinline__ cx<double> wiener_gain(const GainArgs& ga, int n, int f,
                                                  const cx<double>* __restrict__ twB64) {
  // e^{-2 pi i r f / b} as successive powers of the table entry for f
  const cx<double> t1 = twB64[f & (B - 1)];
  cx<double> e = mk<double>(1.0, 0.0);
  double wr = 0.0, wi = 0.0, wabs = 0.0;
  for (int r = 0; r < ga.ntap; ++r) {
    const double h = ga.win[(int64_t)r * ga.lblock + n];
    wr += h * e.x;
    wi += h * e.y;
    wabs += fabs(h);
    e = cmul(e, t1);
  }
  const double a2 = wr * wr + wi * wi;
  if (ga.precond) return mk<double>(1.0 / ((a2 + ga.phi2) * (double)B), 0.0);
  if (ga.naive) {
    // plain division by conj(W); eigenvalues at rounding level are dropped
    if (sqrt(a2) <= 1e-12 * wabs) return mk<double>(0.0, 0.0);
    const double s = 1.0 / (a2 * (double)B);
    return mk<double>(wr * s, wi * s);
  }
  const double s = ga.gnorm / (a2 + ga.phi2);
  return mk<double>(wr * s, wi * s);
}

// Both gains of a split pair, G_n(k) and G_n(b/2 - k), for 4 taps. With
// z = e^{-2 pi i k/b}, E = h0 + h2 z^2 and O = h1 z + h3 z^3:
//   W(k) = E + O,  W(b/2 - k) = conj(E - O)   (z at b/2 - k is -conj z),
// and the two denominators share one reciprocal.
template <int B>
__device__ __forceinline__ void gain_pair4(const GainArgs& ga, int n, int k, const cx<double>* __restrict__ twB64,
                                           cx<double>& Gk, cx<double>& Gm) {
  const int N = ga.lblock;
  const double h0 = ga.win[n], h1 = ga.win[N + n], h2 = ga.win[2 * N + n], h3 = ga.win[3 * N + n];
  const cx<double> z = twB64[k];
  const cx<double> z2 = cmul(z, z), z3 = cmul(z2, z);
  const cx<double> E = mk<double>(h0 + h2 * z2.x, h2 * z2.y);
  const cx<double> O = mk<double>(h1 * z.x + h3 * z3.x, h1 * z.y + h3 * z3.y);
  const cx<double> Wk = E + O, Wm = conj(E - O);
  const double ak = Wk.x * Wk.x + Wk.y * Wk.y, am = Wm.x * Wm.x + Wm.y * Wm.y;
  if (ga.naive) {  // plain division by conj(W); eigenvalues at rounding level are dropped
    const double wabs = fabs(h0) + fabs(h1) + fabs(h2) + fabs(h3);
    const double sk = (sqrt(ak) <= 1e-12 * wabs) ? 0.0 : 1.0 / (ak * (double)B);
    const double sm = (sqrt(am) <= 1e-12 * wabs) ? 0.0 : 1.0 / (am * (double)B);
    Gk = mk<double>(Wk.x * sk, Wk.y * sk);
    Gm = mk<double>(Wm.x * sm, Wm.y * sm);
    return;
  }
  const double dk = ak + ga.phi2, dm = am + ga.phi2;
  const double den = dk * dm;
  double rc = __builtin_amdgcn_rcp(den);
  rc = rc * fma(-den, rc, 2.0);  // one Newton step: ~1 ulp
  if (ga.precond) {
    Gk = mk<double>(dm * rc / (double)B, 0.0);
    Gm = mk<double>(dk * rc / (double)B, 0.0);
    return;
  }
  const double sk = ga.gnorm * dm * rc, sm = ga.gnorm * dk * rc;
  Gk = mk<double>(Wk.x * sk, Wk.y * sk);
  Gm = mk<double>(Wm.x * sm, Wm.y * sm);
}

template <typename T, int LOG2B>
__global__ __launch_bounds__((ColCfg<T, LOG2B>::NT), (ColCfg<T, LOG2B>::WPE)) void k_col_wiener(
    const T* __restrict__ dT, T* __restrict__ xT, GainArgs ga, const cx<T>* __restrict__ twB,
    const cx<double>* __restrict__ twB64, double* __restrict__ part, int nparts) {
  using Cfg = ColCfg<T, LOG2B>;
  constexpr int B = 1 << LOG2B, H = Cfg::H, C = Cfg::C, LS = Cfg::LS, NT = Cfg::NT;
  constexpr int HP = H / 2 + 1;
  // the FFT tile, also the dot product's reduction buffer (NT doubles) afterwards
  constexpr int SRED = (NT * (int)sizeof(double) + (int)sizeof(cx<T>) - 1) / (int)sizeof(cx<T>);
  __shared__ cx<T> s[C * LS > SRED ? C * LS : SRED];
  const int tid = threadIdx.x;
  const int N = ga.lblock;
  const int n0 = blockIdx.x * C;

  // C contiguous columns: z[m] = (d_T[n][2m], d_T[n][2m+1])
  for (int e = tid; e < H * C; e += NT) {
    const int c = e / H, m = e % H;
    const int n = n0 + c;
    cx<T> v = mk<T>(T(0), T(0));
    if (n < N) v = reinterpret_cast<const cx<T>*>(dT + (int64_t)n * B)[m];
    s[c * LS + pidx(m)] = v;
  }
  __syncthreads();
  lds_fft<T, H, NT, C, -1>(s, LS, twB, 2);

  // split the packed spectrum, apply the gain, re-pack for the inverse
  for (int e = tid; e < C * HP; e += NT) {
    const int c = e / HP, k = e % HP;
    const int n = n0 + c;
    if (n >= N) continue;
    cx<T>* col = s + c * LS;
    if (k == 0) {
      const cx<T> z0 = col[0];  // pidx(0) == 0
      const double x0 = (double)z0.x + (double)z0.y;  // X[0]
      const double xh = (double)z0.x - (double)z0.y;  // X[b/2]
      const double y0 = wiener_gain<B>(ga, n, 0, twB64).x * x0;
      const double yh = wiener_gain<B>(ga, n, H, twB64).x * xh;
      col[0] = mk<T>(T(y0 + yh), T(y0 - yh));
      continue;
    }
    const int km = H - k;
    const cx<T> zk = col[pidx(k)], zm = col[pidx(km)];
    const cx<double> Zk = mk<double>(zk.x, zk.y), Zm = mk<double>(zm.x, zm.y);
    const cx<double> ek = twB64[k];          // e^{-2 pi i k / b}
    const cx<double> A = Zk + conj(Zm);
    const cx<double> Bd = Zk - conj(Zm);
    const cx<double> eB = cmul(ek, Bd);
    // X[k] = A/2 - i e B/2 ;  X[H-k] = conj(A)/2 - i conj(e B)/2
    const cx<double> Xk = mk<double>(0.5 * (A.x + eB.y), 0.5 * (A.y - eB.x));
    const cx<double> Xm = mk<double>(0.5 * (A.x - eB.y), 0.5 * (-A.y - eB.x));
    cx<double> Gk, Gm;
    if (ga.ntap == 4) {
      gain_pair4<B>(ga, n, k, twB64, Gk, Gm);
    } else {
      Gk = wiener_gain<B>(ga, n, k, twB64);
      Gm = wiener_gain<B>(ga, n, km, twB64);
    }
    const cx<double> Yk = cmul(Gk, Xk);
    const cx<double> Ym = cmul(Gm, Xm);
    // Z'[k] = P + i conj(e) Q ;  Z'[H-k] = conj(P) + i e conj(Q)
    const cx<double> P = Yk + conj(Ym);
    const cx<double> Q = Yk - conj(Ym);
    const cx<double> t1 = cmulc(Q, ek);            // conj(e) Q
    const cx<double> t2 = cmul(ek, conj(Q));       // e conj(Q)
    col[pidx(k)] = mk<T>(T(P.x - t1.y), T(P.y + t1.x));
    if (km != k) col[pidx(km)] = mk<T>(T(P.x - t2.y), T(-P.y + t2.x));
  }
  __syncthreads();
  lds_fft<T, H, NT, C, +1>(s, LS, twB, 2);

  double acc = 0.0;
  for (int e = tid; e < H * C; e += NT) {
    const int c = e / H, m = e % H;
    const int n = n0 + c;
    if (n >= N) continue;
    const cx<T> v = s[c * LS + pidx(m)];
    reinterpret_cast<cx<T>*>(xT + (int64_t)n * B)[m] = v;
    if (part) {  // the dot product input . output of these columns (the CG's r . z)
      const cx<T> a = reinterpret_cast<const cx<T>*>(dT + (int64_t)n * B)[m];
      acc += (double)a.x * (double)v.x + (double)a.y * (double)v.y;
    }
  }
  if (part) {  // fixed-order sum over the workgroup, through the (now free) LDS
    double* red = reinterpret_cast<double*>(s);
    __syncthreads();
    const double tot = block_sum<NT>(acc, red);
    if (tid == 0) part[blockIdx.x] = tot;
    if (blockIdx.x == 0)  // the slots no workgroup of this launch fills
      for (int i = (int)gridDim.x + tid; i < nparts; i += NT) part[i] = 0.0;
  }
}

template <typename T, int LOG2B>
static hipError_t launch_col_t(const void* d, void* xo, const GainArgs& ga, const void* twB,
                               const double* twB64, hipStream_t st, double* part) {
  using Cfg = ColCfg<T, LOG2B>;
  static_assert((Cfg::NT & (Cfg::NT - 1)) == 0, "the dot product's tree needs a power-of-two workgroup");
  const int nwg = (ga.lblock + Cfg::C - 1) / Cfg::C;
  if (part && nwg > kCgParts) return hipErrorNotSupported;  // more workgroups than partial-sum slots
  k_col_wiener<T, LOG2B><<<dim3(nwg), dim3(Cfg::NT), 0, st>>>(
      (const T*)d, (T*)xo, ga, (const cx<T>*)twB, (const cx<double>*)twB64, part, kCgParts);
  return hipGetLastError();
}

#define COL_CASE(T, L) \
  case L: return launch_col_t<T, L>(d, xo, ga, twB, twB64, st, part);

hipError_t launch_col_wiener(int prec, int log2b, const void* d, void* xo, int lblock, int ntap,
                             const double* win64, double phi, int normalise, const void* twB,
                             const double* twB64, hipStream_t st, int precond, double* part) {
  GainArgs ga;
  ga.win = win64;
  ga.lblock = lblock;
  ga.ntap = ntap;
  ga.phi2 = phi * phi;
  ga.naive = (phi == 0.0) && !precond;
  ga.precond = precond;
  ga.gnorm = (normalise ? (1.0 + phi * phi) : 1.0) / (double)(1LL << log2b);
  if (prec == F32) {
    switch (log2b) {
      COL_CASE(float, 2) COL_CASE(float, 3) COL_CASE(float, 4) COL_CASE(float, 5) COL_CASE(float, 6)
      COL_CASE(float, 7) COL_CASE(float, 8) COL_CASE(float, 9) COL_CASE(float, 10) COL_CASE(float, 11)
      COL_CASE(float, 12) COL_CASE(float, 13) COL_CASE(float, 14) COL_CASE(float, 15)
      default: return hipErrorInvalidValue;
    }
  }
  switch (log2b) {
    COL_CASE(double, 2) COL_CASE(double, 3) COL_CASE(double, 4) COL_CASE(double, 5) COL_CASE(double, 6)
    COL_CASE(double, 7) COL_CASE(double, 8) COL_CASE(double, 9) COL_CASE(double, 10) COL_CASE(double, 11)
    COL_CASE(double, 12) COL_CASE(double, 13) COL_CASE(double, 14)
    default: return hipErrorInvalidValue;
  }
}

}  // namespace ipfb
