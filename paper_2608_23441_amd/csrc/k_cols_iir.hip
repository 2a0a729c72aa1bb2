// Column stage of the circulant Wiener inverse as two recursions along the
// frames (Section 3.1 decorrelation with the Section 4.1 Wiener weights; the
// Tikhonov form of Appendix C).
//
// For sub-filter path n, with zeta = e^{-2 pi i f / b}, the column spectrum is
// the polynomial W(zeta) = sum_{r<p} h_r zeta^r (h_r = h[rN+n]) and
//   |W|^2 + phi^2 = P(zeta) = c'_0 + sum_{t=1}^{p-1} c_t (zeta^t + zeta^-t),
// c_t = sum_r h_r h_{r+t}, c'_0 = c_0 + phi^2. P > 0 on the unit circle, so
// it factors as P = K Q(zeta) Q(1/zeta), Q(zeta) = prod_i (1 - r_i zeta) =
// 1 - sum_i a_i zeta^i, |r_i| < 1 (the roots of P inside the unit circle).
// The gain G = W (1+phi^2)/P, sampled at the b-th roots of unity, is the
// eigenvalue sequence of the circulant matrix that periodises the impulse
// response of kappa W(zeta)/(Q(zeta) Q(1/zeta)), kappa = (1+phi^2)/K. So,
// over the periodic sequence of b frames,
//   y = the causal ARMA filter W/Q applied to d      (forward in j),
//   v = the anti-causal all-pole filter 1/Q(1/zeta) on y (backward in j),
//   xhat = kappa v
// is the same linear map as F^dagger G F, with O(p) operations per sample.
//
// Frames split into segments of L. Pass 1 runs both recursions from zero
// state over each segment and keeps only their end states; a scan per column
// turns them into the exact periodic states entering every segment (the
// circular boundary solved through (I - A^b)^-1); pass 2 reruns the
// recursions from those states and writes xhat over d in place. The states
// are FP64 in both precisions.
//
// The factorisation runs on the device, one thread per column: the
// palindromic P reduces to a degree-(p-1) polynomial R in x = zeta + 1/zeta;
// its roots are found in u = 1/x (the reversed polynomial, whose leading
// coefficient P(zeta = i) >= phi^2 never vanishes) by Aberth-Ehrlich
// iteration, and r solves r + 1/r = 1/u inside the unit circle.
#include "fft_lds.hpp"
#include "launch.hpp"

namespace ipfb {

// Per-column coefficient block (FP64), M = p - 1 poles, shared by every
// stream of the column's window and phi:
//   h[M+1] numerator taps, a[M] with Q = 1 - sum a_i zeta^i, 1/K,
//   A^L, B^L (the causal and anti-causal states carried over a full segment
//   of L frames), N_L (the anti-causal left-end state produced by the causal
//   state entering a full segment).
// Per-(stream, column) block, for the stream's length b and its last
// segment of L' = b - (nseg - 1) L frames:
//   A^{L'}, B^{L'}, N_{L'}, (I - A^b)^-1, (I - B^b)^-1.
// segments per lane at most in the uniform-power carry (nseg <= 64 kIirQMax)
constexpr int kIirQMax = 8;

template <int M>
struct IirLayout {
  static constexpr int H = 0, A = M + 1, IK = 2 * M + 1, MAT = 2 * M + 2;
  static constexpr int AL = MAT, BL = MAT + M * M, NL = MAT + 2 * M * M;
  // A^{q L 2^k} and B^{q L 2^k} for q = 1..kIirQMax, k = 0..5 (the carry's
  // lane-to-lane steps): PA + ((q-1) 6 + k) M^2, PB likewise
  static constexpr int PA = MAT + 3 * M * M, PB = PA + kIirQMax * 6 * M * M;
  static constexpr int STRIDE = PB + kIirQMax * 6 * M * M;
  // the per-stream block
  static constexpr int ALL = 0, BLL = M * M, NLL = 2 * M * M, IA = 3 * M * M, IB = 4 * M * M;
  static constexpr int SSTRIDE = 5 * M * M;
};

int iir_coef_stride(int ntap) {
  switch (ntap) {
    case 4: return IirLayout<3>::STRIDE;
    default: return 0;
  }
}

int iir_stream_stride(int ntap) {
  switch (ntap) {
    case 4: return IirLayout<3>::SSTRIDE;
    default: return 0;
  }
}

__device__ __forceinline__ int64_t uniform64(int64_t v) {
  const uint64_t u = (uint64_t)v;
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)u);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(u >> 32));
  return (int64_t)(((uint64_t)hi << 32) | lo);
}

// The stream of global segment g (the same for the whole workgroup): the
// last s with seg0[s] <= g, or the single stream passed by value when there
// is no table. The fields come back as wavefront-uniform values.
__device__ __forceinline__ IirStream iir_stream_of(int64_t g, const IirStream& one, const IirStream* __restrict__ tab,
                                                   int nstreams) {
  IirStream r = one;
  if (tab && nstreams > 0) {  // a table (one entry or more) takes precedence
    int lo = 0, hi = nstreams - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (tab[mid].seg0 <= g) lo = mid;
      else hi = mid - 1;
    }
    r = tab[lo];
  }
  r.x = (void*)uniform64((int64_t)r.x);
  r.b = uniform64(r.b);
  r.seg0 = uniform64(r.seg0);
  return r;
}

// ---- small dense helpers (M x M, row major, FP64) ---------------------------
template <int M>
__device__ void mat_mul(const double* a, const double* b, double* c) {
  double t[M * M];
  for (int i = 0; i < M; ++i)
    for (int j = 0; j < M; ++j) {
      double s = 0.0;
      for (int k = 0; k < M; ++k) s += a[i * M + k] * b[k * M + j];
      t[i * M + j] = s;
    }
  for (int i = 0; i < M * M; ++i) c[i] = t[i];
}

template <int M>
__device__ void mat_pow(const double* a, int64_t e, double* out) {
  double base[M * M], r[M * M];
  for (int i = 0; i < M * M; ++i) {
    base[i] = a[i];
    r[i] = (i % (M + 1) == 0) ? 1.0 : 0.0;
  }
  while (e > 0) {
    if (e & 1) mat_mul<M>(r, base, r);
    e >>= 1;
    if (e) mat_mul<M>(base, base, base);
  }
  for (int i = 0; i < M * M; ++i) out[i] = r[i];
}

// out = (I - a)^-1 by Gauss-Jordan with partial pivoting
template <int M>
__device__ void inv_i_minus(const double* a, double* out) {
  double m[M * M], v[M * M];
  for (int i = 0; i < M * M; ++i) {
    const double id = (i % (M + 1) == 0) ? 1.0 : 0.0;
    m[i] = id - a[i];
    v[i] = id;
  }
  for (int c = 0; c < M; ++c) {
    int piv = c;
    for (int r = c + 1; r < M; ++r)
      if (fabs(m[r * M + c]) > fabs(m[piv * M + c])) piv = r;
    if (piv != c)
      for (int k = 0; k < M; ++k) {
        double t = m[c * M + k];
        m[c * M + k] = m[piv * M + k];
        m[piv * M + k] = t;
        t = v[c * M + k];
        v[c * M + k] = v[piv * M + k];
        v[piv * M + k] = t;
      }
    const double d = 1.0 / m[c * M + c];
    for (int k = 0; k < M; ++k) {
      m[c * M + k] *= d;
      v[c * M + k] *= d;
    }
    for (int r = 0; r < M; ++r) {
      if (r == c) continue;
      const double f = m[r * M + c];
      for (int k = 0; k < M; ++k) {
        m[r * M + k] -= f * m[c * M + k];
        v[r * M + k] -= f * v[c * M + k];
      }
    }
  }
  for (int i = 0; i < M * M; ++i) out[i] = v[i];
}

__device__ __forceinline__ cx<double> cdiv(cx<double> a, cx<double> b) {
  const double s = 1.0 / (b.x * b.x + b.y * b.y);
  return mk<double>((a.x * b.x + a.y * b.y) * s, (a.y * b.x - a.x * b.y) * s);
}

__device__ __forceinline__ cx<double> csqrt(cx<double> z) {
  const double r = sqrt(sqrt(z.x * z.x + z.y * z.y));
  const double t = 0.5 * atan2(z.y, z.x);
  return mk<double>(r * cos(t), r * sin(t));
}

// Roots of sum_{k=0}^{D} c[k] u^k (c[D] != 0) by Aberth-Ehrlich iteration.
template <int D>
__device__ void aberth(const double* c, cx<double>* z) {
  // starting points on a circle of the roots' geometric-mean radius
  const double rad = pow(fabs(c[0] / c[D]) + 1e-300, 1.0 / D) + 1e-3;
  for (int k = 0; k < D; ++k) {
    const double th = 6.283185307179586 * k / D + 0.4;
    z[k] = mk<double>(rad * cos(th), rad * sin(th));
  }
  for (int it = 0; it < 200; ++it) {
    double moved = 0.0, size = 0.0;
    for (int k = 0; k < D; ++k) {
      cx<double> pv = mk<double>(c[D], 0.0), dv = mk<double>(0.0, 0.0);
      for (int j = D - 1; j >= 0; --j) {
        dv = cmul(dv, z[k]) + pv;
        pv = cmul(pv, z[k]) + mk<double>(c[j], 0.0);
      }
      if (pv.x == 0.0 && pv.y == 0.0) continue;
      const cx<double> ratio = cdiv(pv, dv);
      cx<double> s = mk<double>(0.0, 0.0);
      for (int j = 0; j < D; ++j)
        if (j != k) s = s + cdiv(mk<double>(1.0, 0.0), z[k] - z[j]);
      const cx<double> w = cdiv(ratio, mk<double>(1.0, 0.0) - cmul(ratio, s));
      z[k] = z[k] - w;
      moved = fmax(moved, sqrt(w.x * w.x + w.y * w.y));
      size = fmax(size, sqrt(z[k].x * z[k].x + z[k].y * z[k].y));
    }
    if (moved <= 1e-17 * fmax(size, 1e-300)) break;
  }
}

// The causal and anti-causal zero-input state steps from the poles'
// polynomial: causal (transposed direct form II): y = s_0,
// s_i <- a_{i+1} y + s_{i+1}; anti-causal state (v_j, ..., v_{j+M-1}) one
// frame to the left: v_{j-1} = sum_i a_{i+1} v_{j+i}
template <int M>
__device__ void iir_steps(const double* a, double* A, double* B) {
  for (int i = 0; i < M * M; ++i) A[i] = B[i] = 0.0;
  for (int i = 0; i < M; ++i) {
    A[i * M + 0] = a[i];
    if (i + 1 < M) A[i * M + i + 1] = 1.0;
    B[0 * M + i] = a[i];
    if (i >= 1) B[i * M + i - 1] = 1.0;
  }
}

// N[t][i] = sum_{k=t}^{len-1} g[k-t] (e_0^T A^k)_i, g the all-pole impulse
// response (g_0 = 1, g_k = sum_i a_i g_{k-i}): the anti-causal left-end state
// that a causal state entering a segment of len frames produces
template <int M>
__device__ void iir_nmat(const double* a, const double* A, int len, double* Nm) {
  for (int i = 0; i < M * M; ++i) Nm[i] = 0.0;
  double row[M], gr[M];
  for (int i = 0; i < M; ++i) row[i] = gr[i] = 0.0;
  row[0] = 1.0;
  for (int k = 0; k < len; ++k) {
    double gk = (k == 0) ? 1.0 : 0.0;
    for (int i = 0; i < M; ++i) gk += a[i] * gr[i];
    for (int i = M - 1; i > 0; --i) gr[i] = gr[i - 1];
    gr[0] = gk;  // gr[t] = g_{k-t}
    for (int t = 0; t < M; ++t)
      for (int i = 0; i < M; ++i) Nm[t * M + i] += gr[t] * row[i];
    double nr[M];
    for (int j = 0; j < M; ++j) {
      double s = 0.0;
      for (int i = 0; i < M; ++i) s += row[i] * A[i * M + j];
      nr[j] = s;
    }
    for (int j = 0; j < M; ++j) row[j] = nr[j];
  }
}

// One thread per column: the factorisation and the full-segment matrices
// for segments of L frames.
template <int M>
__global__ __launch_bounds__(64) void k_iir_setup(const double* __restrict__ win, int N, double phi, int L,
                                                   double* __restrict__ coef, int precond) {
  using Ly = IirLayout<M>;
  const int n = blockIdx.x * 64 + threadIdx.x;
  if (n >= N) return;
  double* cf = coef + (int64_t)n * Ly::STRIDE;
  double h[M + 1];
  for (int r = 0; r <= M; ++r) h[r] = win[(int64_t)r * N + n];
  double c[M + 1];
  for (int t = 0; t <= M; ++t) {
    double s = 0.0;
    for (int r = 0; r + t <= M; ++r) s += h[r] * h[r + t];
    c[t] = s;
  }
  c[0] += phi * phi;
  // R(x) = c'_0 + sum_t c_t V_t(x), V_t(x) = zeta^t + zeta^-t: V_1 = x,
  // V_2 = x^2 - 2, V_t = x V_{t-1} - V_{t-2}
  double R[M + 1], vm2[M + 1], vm1[M + 1], vt[M + 1];
  for (int k = 0; k <= M; ++k) R[k] = vm2[k] = vm1[k] = 0.0;
  R[0] = c[0];
  vm2[0] = 2.0;  // V_0 (unused in the sum: c'_0 enters once)
  vm1[1] = 1.0;  // V_1
  for (int t = 1; t <= M; ++t) {
    if (t >= 2) {
      for (int k = 0; k <= M; ++k) vt[k] = (k > 0 ? vm1[k - 1] : 0.0) - vm2[k];
      for (int k = 0; k <= M; ++k) {
        vm2[k] = vm1[k];
        vm1[k] = vt[k];
      }
    }
    for (int k = 0; k <= M; ++k) R[k] += c[t] * vm1[k];
  }
  // roots in u = 1/x: the reversed polynomial, leading coefficient R[0] = P(i) > 0
  double rev[M + 1];
  for (int k = 0; k <= M; ++k) rev[k] = R[M - k];
  cx<double> u[M];
  aberth<M>(rev, u);
  // r with r + 1/r = 1/u and |r| < 1: r = 2u / (1 +- sqrt(1 - 4u^2))
  cx<double> q[M + 1];  // Q(zeta) coefficients, q[0] = 1
  q[0] = mk<double>(1.0, 0.0);
  for (int k = 1; k <= M; ++k) q[k] = mk<double>(0.0, 0.0);
  cx<double> q1 = mk<double>(1.0, 0.0);
  for (int i = 0; i < M; ++i) {
    const cx<double> u2 = cmul(u[i], u[i]);
    const cx<double> s = csqrt(mk<double>(1.0 - 4.0 * u2.x, -4.0 * u2.y));
    const cx<double> dp = mk<double>(1.0 + s.x, s.y), dm = mk<double>(1.0 - s.x, -s.y);
    const cx<double> den = (dp.x * dp.x + dp.y * dp.y >= dm.x * dm.x + dm.y * dm.y) ? dp : dm;
    const cx<double> r = cdiv(scale(u[i], 2.0), den);
    for (int k = i + 1; k >= 1; --k) q[k] = q[k] - cmul(r, q[k - 1]);  // times (1 - r zeta)
    q1 = cmul(q1, mk<double>(1.0 - r.x, -r.y));
  }
  double a[M];
  for (int i = 0; i < M; ++i) a[i] = -q[i + 1].x;
  double hs = 0.0;
  for (int r = 0; r <= M; ++r) hs += h[r];
  const double P1 = hs * hs + phi * phi;
  const double Q1 = q1.x;  // real: the roots come in conjugate pairs
  const double invK = Q1 * Q1 / P1;
  // numerator: the taps (Wiener), or 1 (the preconditioner 1/(|W|^2 + phi^2))
  for (int r = 0; r <= M; ++r) cf[Ly::H + r] = precond ? (r == 0 ? 1.0 : 0.0) : h[r];
  for (int i = 0; i < M; ++i) cf[Ly::A + i] = a[i];
  cf[Ly::IK] = invK;
  double A[M * M], B[M * M];
  iir_steps<M>(a, A, B);
  mat_pow<M>(A, L, cf + Ly::AL);
  mat_pow<M>(B, L, cf + Ly::BL);
  iir_nmat<M>(a, A, L, cf + Ly::NL);
  for (int q = 1; q <= kIirQMax; ++q) {
    double* pa = cf + Ly::PA + (q - 1) * 6 * M * M;
    double* pb = cf + Ly::PB + (q - 1) * 6 * M * M;
    mat_pow<M>(cf + Ly::AL, q, pa);
    mat_pow<M>(cf + Ly::BL, q, pb);
    for (int k = 1; k < 6; ++k) {
      mat_mul<M>(pa + (k - 1) * M * M, pa + (k - 1) * M * M, pa + k * M * M);
      mat_mul<M>(pb + (k - 1) * M * M, pb + (k - 1) * M * M, pb + k * M * M);
    }
  }
}

// One thread per (stream, column): the matrices that depend on the stream's
// length, for its last segment and its periodic boundary.
template <int M>
__global__ __launch_bounds__(64) void k_iir_setup_len(int N, int L, IirStream one, const IirStream* __restrict__ tab,
                                                       int nstreams, const double* __restrict__ coef,
                                                       double* __restrict__ scoef) {
  using Ly = IirLayout<M>;
  const int64_t t = (int64_t)blockIdx.x * 64 + threadIdx.x;
  if (t >= (int64_t)nstreams * N) return;
  const int si = (int)(t / N), n = (int)(t - (int64_t)si * N);
  const IirStream sd = tab ? tab[si] : one;
  const double* cf = coef + (int64_t)n * Ly::STRIDE;
  double* sc = scoef + t * Ly::SSTRIDE;
  double a[M], A[M * M], B[M * M], t1[M * M];
  for (int i = 0; i < M; ++i) a[i] = cf[Ly::A + i];
  iir_steps<M>(a, A, B);
  const int64_t b = sd.b;
  const int64_t nseg = (b + L - 1) / L;
  const int Ll = (int)(b - (nseg - 1) * L);
  mat_pow<M>(A, Ll, sc + Ly::ALL);
  mat_pow<M>(B, Ll, sc + Ly::BLL);
  iir_nmat<M>(a, A, Ll, sc + Ly::NLL);
  mat_pow<M>(A, b, t1);
  inv_i_minus<M>(t1, sc + Ly::IA);
  mat_pow<M>(B, b, t1);
  inv_i_minus<M>(t1, sc + Ly::IB);
}

// Frames of one column are streamed in chunks of kIirChunk, the next chunk
// fetched while the current one is used.
constexpr int kIirChunk = 16;

// (the frames come from a stream table, so the pointer is cast to global
// memory: flat loads would also hold up every LDS wait)
template <typename T>
__device__ __forceinline__ void load_chunk(const T* __restrict__ p, int64_t N, int k0, int Ls, T* v) {
  const __attribute__((address_space(1))) T* gp = (const __attribute__((address_space(1))) T*)p;
#pragma unroll
  for (int k = 0; k < kIirChunk; ++k) v[k] = (k0 + k < Ls) ? gp[(int64_t)(k0 + k) * N] : T(0);
}

// Pass 1: per (column, segment), both recursions from zero state: the causal
// state leaving the segment and the anti-causal left-end state
// (v_{j0}, ..., v_{j0+M-1}) = sum_{k>=t} g_{k-t} y_k. zs[(g N + n) 2M + .]
// for global segment g (the segments of all streams, one after another).
// Workgroup w takes segment g = nsegt - 1 - w / ntiles, last first: the
// reverse of the order the row stage wrote its frames in, so the most
// recently written ones (still in the last-level cache) are read first.
template <typename T, int M, int L>
__global__ __launch_bounds__(256) void k_iir_zs(int N, int ntiles, int64_t nsegt, IirStream one,
                                                 const IirStream* __restrict__ tab, int nstreams,
                                                 const double* __restrict__ coef, T* __restrict__ zs) {
  using Ly = IirLayout<M>;
  const int64_t g = nsegt - 1 - (int64_t)__builtin_amdgcn_readfirstlane(blockIdx.x / ntiles);
  const int n = (int)__builtin_amdgcn_readfirstlane(blockIdx.x % ntiles) * 256 + threadIdx.x;
  if (n >= N) return;
  const IirStream sd = iir_stream_of(g, one, tab, nstreams);
  const int64_t j0 = (g - sd.seg0) * L;
  const int Ls = (int)((sd.b - j0) < L ? (sd.b - j0) : L);
  const double* cf = coef + (int64_t)n * Ly::STRIDE;
  double h[M + 1], a[M];
  for (int r = 0; r <= M; ++r) h[r] = cf[Ly::H + r];
  for (int i = 0; i < M; ++i) a[i] = cf[Ly::A + i];
  const T* pd = (const T*)sd.x + j0 * (int64_t)N + n;
  double st[M], za[M], gr[M];
  for (int i = 0; i < M; ++i) st[i] = za[i] = gr[i] = 0.0;
  // one frame k of the segment: both recursions
  auto frame = [&](T xv, int k) {
    const double x = (double)xv;
    const double y = fma(h[0], x, st[0]);
#pragma unroll
    for (int i = 0; i + 1 < M; ++i) st[i] = fma(a[i], y, fma(h[i + 1], x, st[i + 1]));
    st[M - 1] = fma(a[M - 1], y, h[M] * x);
    double gk = a[0] * gr[0];
    if (k == 0) gk = 1.0;  // gr = 0 at the first frame
#pragma unroll
    for (int i = 1; i < M; ++i) gk = fma(a[i], gr[i], gk);
#pragma unroll
    for (int i = M - 1; i > 0; --i) gr[i] = gr[i - 1];
    gr[0] = gk;  // gr[t] = g_{k-t}
#pragma unroll
    for (int t = 0; t < M; ++t) za[t] += gr[t] * y;
  };
  if (Ls == L) {
    // a full segment: straight-line code with no per-frame checks, its
    // global loads issued a chunk ahead (FP32: the whole segment at once)
    constexpr int CH = sizeof(T) == 4 ? L : 16;
    typedef const __attribute__((address_space(1))) T GT;
    GT* gp = (GT*)pd;
    T v[2][CH];
#pragma unroll
    for (int kk = 0; kk < CH; ++kk) v[0][kk] = gp[(int64_t)kk * N];
#pragma unroll
    for (int c = 0; c < L / CH; ++c) {
      if (c + 1 < L / CH)
#pragma unroll
        for (int kk = 0; kk < CH; ++kk) v[(c + 1) & 1][kk] = gp[(int64_t)((c + 1) * CH + kk) * N];
#pragma unroll
      for (int kk = 0; kk < CH; ++kk) frame(v[c & 1][kk], c * CH + kk);
    }
  } else {
    T cur[kIirChunk], nxt[kIirChunk];
    load_chunk(pd, N, 0, Ls, cur);
    const int nch = (Ls + kIirChunk - 1) / kIirChunk;
#pragma unroll 1
    for (int c = 0; c < nch; ++c) {
      if (c + 1 < nch) load_chunk(pd, N, (c + 1) * kIirChunk, Ls, nxt);
#pragma unroll
      for (int kk = 0; kk < kIirChunk; ++kk) {
        const int k = c * kIirChunk + kk;
        if (k < Ls) frame(cur[kk], k);
      }
#pragma unroll
      for (int kk = 0; kk < kIirChunk; ++kk) cur[kk] = nxt[kk];
    }
  }
  T* o = zs + (g * N + n) * (2 * M);
#pragma unroll
  for (int i = 0; i < M; ++i) {
    o[i] = T(st[i]);
    o[M + i] = T(za[i]);
  }
}

template <int M>
__device__ __forceinline__ void matvec_add(const double* m, const double* x, const double* add, double* out) {
  double t[M];
#pragma unroll
  for (int i = 0; i < M; ++i) {
    double s = add[i];
#pragma unroll
    for (int j = 0; j < M; ++j) s += m[i * M + j] * x[j];
    t[i] = s;
  }
#pragma unroll
  for (int i = 0; i < M; ++i) out[i] = t[i];
}


// The carry scan moves 3x3 affine maps X -> P X + Y across the lanes of a
// wavefront with cross-lane exchanges.
template <int M>
__device__ __forceinline__ void shfl_map(const double* P, const double* Y, double* Po, double* Yo, int delta,
                                         bool up) {
#pragma unroll
  for (int i = 0; i < M * M; ++i) Po[i] = up ? __shfl_up(P[i], delta, 64) : __shfl_down(P[i], delta, 64);
#pragma unroll
  for (int i = 0; i < M; ++i) Yo[i] = up ? __shfl_up(Y[i], delta, 64) : __shfl_down(Y[i], delta, 64);
}

template <int M>
__device__ __forceinline__ void set_identity(double* P, double* Y) {
#pragma unroll
  for (int i = 0; i < M * M; ++i) P[i] = (i % (M + 1) == 0) ? 1.0 : 0.0;
#pragma unroll
  for (int i = 0; i < M; ++i) Y[i] = 0.0;
}

// Per column (one wavefront): the periodic states entering every segment,
// written over the pass-1 results: zs[s] = (causal state entering segment s,
// anti-causal state entering it from the right), for streams of any length
// (those of at most 64 kIirQMax segments take k_iir_carry_u below). Lane l
// takes the contiguous segments [l q, (l+1) q), q = ceil(nseg / 64): it
// composes its segments' affine maps, an inclusive scan of the maps across
// the lanes (Hillis-Steele) gives every lane its entering state, and the
// lanes then walk their segments. Causal: S_{s+1} = A^{len_s} S_s + zc_s,
// periodic S_0 = (I - A^b)^-1 (scan of all). Anti-causal, right to left:
// F_s = B^{len_s} F_{s+1} + c_s, c_s = za_s + N_{len_s} S_s, periodic
// F_0 = (I - B^b)^-1 (scan of all); segment s receives V_s = F_{s+1}. A
// lane reads its segments' states from global memory in each phase.
template <typename T, int M>
__global__ __launch_bounds__(256) void k_iir_carry(int N, int L, IirStream one, const IirStream* __restrict__ tab,
                                                   int nstreams, const double* __restrict__ coef,
                                                   const double* __restrict__ scoef, T* __restrict__ zs) {
  using Ly = IirLayout<M>;
  constexpr int NMAT = 8 * M * M;
  const int lane = threadIdx.x & 63;
  const int wv = threadIdx.x >> 6;
  const int groups = (N + 3) / 4;
  const int si = __builtin_amdgcn_readfirstlane(blockIdx.x / groups);  // the stream
  const int n = __builtin_amdgcn_readfirstlane((blockIdx.x % groups) * 4 + wv);
  // the column's eight segment matrices, staged in LDS once (read back as
  // wavefront-wide broadcasts in the dependent steps below), in the order
  // A^L, A^{L'}, B^L, B^{L'}, N_L, N_{L'}, (I - A^b)^-1, (I - B^b)^-1
  __shared__ double smat[4][NMAT];
  constexpr int MM = M * M;
  for (int i = lane; i < NMAT; i += 64) {
    double v = 0.0;
    if (n < N) {
      const int m = i / MM, e = i - m * MM;
      const double* cfm = coef + (int64_t)n * Ly::STRIDE;
      const double* scm = scoef + ((int64_t)si * N + n) * Ly::SSTRIDE;
      switch (m) {
        case 0: v = cfm[Ly::AL + e]; break;
        case 1: v = scm[Ly::ALL + e]; break;
        case 2: v = cfm[Ly::BL + e]; break;
        case 3: v = scm[Ly::BLL + e]; break;
        case 4: v = cfm[Ly::NL + e]; break;
        case 5: v = scm[Ly::NLL + e]; break;
        case 6: v = scm[Ly::IA + e]; break;
        default: v = scm[Ly::IB + e]; break;
      }
    }
    smat[wv][i] = v;
  }
  __syncthreads();
  if (n >= N) return;  // the whole wavefront
  constexpr int oAL = 0, oALL = MM, oBL = 2 * MM, oBLL = 3 * MM, oNL = 4 * MM, oNLL = 5 * MM, oIA = 6 * MM,
                oIB = 7 * MM;
  const double* cf = smat[wv];
  IirStream sd = tab ? tab[si] : one;
  sd.b = uniform64(sd.b);
  sd.seg0 = uniform64(sd.seg0);
  const int64_t nseg = (sd.b + L - 1) / L;
  if (nseg == 0) return;  // a stream without frames: nothing to carry
  const int64_t stride = (int64_t)N * 2 * M;
  T* z = zs + (sd.seg0 * N + n) * 2 * M;
  const int64_t q = (nseg + 63) / 64;
  const int64_t a0 = lane * q < nseg ? lane * q : nseg;
  const int64_t a1 = a0 + q < nseg ? a0 + q : nseg;
  const int cnt = (int)(a1 - a0);
  auto get = [&](int k, int i, bool za) -> double { return (double)z[(a0 + k) * stride + (za ? M : 0) + i]; };
  auto put = [&](int k, int i, bool za, double v) { z[(a0 + k) * stride + (za ? M : 0) + i] = T(v); };
  auto last_seg = [&](int k) { return a0 + k + 1 == nseg; };
  const double zero[M] = {};
  double P[M * M], Y[M], Po[M * M], Yo[M];
  // ---- causal: local composition, then the scan
  set_identity<M>(P, Y);
  for (int k = 0; k < cnt; ++k) {
    const double* As = cf + (last_seg(k) ? oALL : oAL);
    double zc[M];
    for (int i = 0; i < M; ++i) zc[i] = get(k, i, false);
    matvec_add<M>(As, Y, zc, Y);
    mat_mul<M>(As, P, P);
  }
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    shfl_map<M>(P, Y, Po, Yo, d, true);
    if (lane >= d) {  // (P, Y) after (Po, Yo): X -> P (Po X + Yo) + Y
      matvec_add<M>(P, Yo, Y, Y);
      mat_mul<M>(P, Po, P);
    }
  }
  double Tt[M], S0[M], S[M];
#pragma unroll
  for (int i = 0; i < M; ++i) Tt[i] = __shfl(Y[i], 63, 64);
  matvec_add<M>(cf + oIA, Tt, zero, S0);
  shfl_map<M>(P, Y, Po, Yo, 1, true);  // exclusive: the lanes to the left
  if (lane == 0) set_identity<M>(Po, Yo);
  matvec_add<M>(Po, S0, Yo, S);
  for (int k = 0; k < cnt; ++k) {
    const bool last = last_seg(k);
    double zc[M], c[M];
    for (int i = 0; i < M; ++i) {
      zc[i] = get(k, i, false);
      c[i] = get(k, i, true);
    }
    matvec_add<M>(cf + (last ? oNLL : oNL), S, c, c);
    for (int i = 0; i < M; ++i) {
      put(k, i, false, S[i]);
      put(k, i, true, c[i]);
    }
    matvec_add<M>(cf + (last ? oALL : oAL), S, zc, S);
  }
  // ---- anti-causal: local composition right to left, then the suffix scan
  set_identity<M>(P, Y);
  for (int k = cnt - 1; k >= 0; --k) {
    const double* Bs = cf + (last_seg(k) ? oBLL : oBL);
    double c[M];
    for (int i = 0; i < M; ++i) c[i] = get(k, i, true);
    matvec_add<M>(Bs, Y, c, Y);
    mat_mul<M>(Bs, P, P);
  }
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    shfl_map<M>(P, Y, Po, Yo, d, false);
    if (lane + d < 64) {  // (P, Y) before (Po, Yo) on the right: X -> P (Po X + Yo) + Y
      matvec_add<M>(P, Yo, Y, Y);
      mat_mul<M>(P, Po, P);
    }
  }
  double Ut[M], F0[M], F[M];
#pragma unroll
  for (int i = 0; i < M; ++i) Ut[i] = __shfl(Y[i], 0, 64);
  matvec_add<M>(cf + oIB, Ut, zero, F0);
  shfl_map<M>(P, Y, Po, Yo, 1, false);  // the lanes to the right
  if (lane == 63) set_identity<M>(Po, Yo);
  matvec_add<M>(Po, F0, Yo, F);
  for (int k = cnt - 1; k >= 0; --k) {
    double c[M];
    for (int i = 0; i < M; ++i) c[i] = get(k, i, true);
    for (int i = 0; i < M; ++i) put(k, i, true, F[i]);  // V_s = F_{s+1}
    matvec_add<M>(cf + (last_seg(k) ? oBLL : oBL), F, c, F);
  }
}

// The same periodic states for streams of at most 64 kIirQMax segments, with
// lane-to-lane steps that are powers of one matrix. Lane l takes q =
// ceil(nseg / 64) segments; every lane before the one holding the last
// segment (lane_last) has q full segments, so composing lanes m..l of the
// causal recursion is Y -> A^{qL (l-m+1)} Y + ..., the same matrix on every
// lane. The scans therefore exchange only 3-vectors and apply the tabulated
// A^{qL 2^k} (B^{qL 2^k}), instead of composing a matrix per lane:
//   causal: local zero-start composition Y_l, inclusive scan
//     E_l = sum_{m <= l} A^{qL(l-m)} Y_m (exact for l < lane_last), the
//     lanes' zero-start entering states Ex_l = E_{l-1}; lane_last walks its
//     segments from Ex to the zero-start total T; S_0 = (I - A^b)^-1 T; lane
//     l enters with A^{qL l} S_0 + Ex_l (binary powers of the table);
//   anti-causal (right to left, c_s = za_s + N_{len_s} S_s): local
//     zero-start U_l, inclusive suffix scan G_l = sum_{m >= l} B^{qL(m-l)} U_m
//     (lanes past lane_last hold 0, so windows that reach them add nothing),
//     F_0 = (I - B^b)^-1 G_0; lane l < lane_last is entered from the right
//     by B^{qL(lane_last-1-l)} W + G_{l+1}, W = B^{len(lane_last)} F_0, and
//     lane_last by F_0.
// One wavefront per (stream, column); the 20 matrices it uses staged in LDS.
// With STAGE, the workgroup's segment states also pass through LDS, loaded
// and stored by the whole workgroup as runs of its columns' states per
// segment: a lane reading its own column's segments straight from global
// memory touches a separate cache line for every 24 bytes. (At 4096 columns
// and 256 segments the loads and stores alone take 32 us with runs of four
// columns, 16.5 us with runs of sixteen; the kernel takes about 40 us, the
// rest being its dependent FP64 chains.)
// Columns per workgroup (one wavefront each): 16 when the states are staged,
// so that the workgroup's states of one segment are a 128-byte-aligned run of
// three lines (16 columns x 2M values x 4 bytes), else 4.
template <typename T, int QR>
constexpr int carry_u_cols() { return (sizeof(T) == 4 && QR == 4) ? 16 : 4; }

template <typename T, int M, int QR>
__global__ __launch_bounds__((64 * carry_u_cols<T, QR>())) void k_iir_carry_u(int N, int L, IirStream one, const IirStream* __restrict__ tab,
                                                     int nstreams, const double* __restrict__ coef,
                                                     const double* __restrict__ scoef, T* __restrict__ zs) {
  using Ly = IirLayout<M>;
  constexpr int MM = M * M;
  constexpr int NMAT = 20;  // A^L, A^L', B^L, B^L', N_L, N_L', (I-A^b)^-1, (I-B^b)^-1, then the two power tables
  constexpr int oAL = 0, oALL = MM, oBL = 2 * MM, oBLL = 3 * MM, oNL = 4 * MM, oNLL = 5 * MM, oIA = 6 * MM,
                oIB = 7 * MM, oPA = 8 * MM, oPB = 14 * MM;
  const int lane = threadIdx.x & 63;
  constexpr int COLS = carry_u_cols<T, QR>();
  const int wv = threadIdx.x >> 6;
  const int groups = (N + COLS - 1) / COLS;
  const int si = __builtin_amdgcn_readfirstlane(blockIdx.x / groups);  // the stream
  const int n = __builtin_amdgcn_readfirstlane((blockIdx.x % groups) * COLS + wv);
  IirStream sd = tab ? tab[si] : one;
  sd.b = uniform64(sd.b);
  sd.seg0 = uniform64(sd.seg0);
  const int64_t nseg = (sd.b + L - 1) / L;
  if (nseg == 0) return;  // a stream without frames (uniform over the workgroup: one stream)
  const int q = (int)((nseg + 63) / 64);  // 1 .. QR (the launch checked max_nseg)
  __shared__ double smat[COLS][NMAT * MM];
  // staged states: [column][segment][2M], the column blocks padded by one
  constexpr int SEGMAX = 64 * QR;
  constexpr int CS = SEGMAX * 2 * M + 1;
  // measured: staging pays in FP32 with up to 256 segments (QR = 4); with
  // eight segments per lane, or in FP64, its LDS costs more occupancy than
  // the gather it saves
  constexpr bool STAGE = sizeof(T) == 4 && QR == 4;
  __shared__ T zst[STAGE ? COLS * CS : 1];
  const int nb = (int)(blockIdx.x % groups) * COLS;  // the workgroup's first column
  const int ncol = N - nb < COLS ? N - nb : COLS;
  const int64_t stride_g = (int64_t)N * 2 * M;
  const int sgs = N * 2 * M;  // 32-bit: nseg * N * 2M < 2^31 (checked at launch)
  T* zb = zs + (sd.seg0 * N + nb) * 2 * M;
  // staging: thread t moves column t % COLS's 2M values of segment
  // pass * 64 + t / COLS (a wavefront: 64 / COLS segments, each a run of
  // COLS columns)
  const int sc = (int)(threadIdx.x % COLS), ss = (int)(threadIdx.x / COLS);
  if constexpr (STAGE) {
    T buf[QR][2 * M];
#pragma unroll
    for (int ps = 0; ps < QR; ++ps) {  // every load in flight at once
      const int sg = ps * 64 + ss;
      const bool ok = sg < nseg && sc < ncol;
#pragma unroll
      for (int i = 0; i < 2 * M; ++i) buf[ps][i] = ok ? zb[sg * sgs + sc * 2 * M + i] : T(0);
    }
#pragma unroll
    for (int ps = 0; ps < QR; ++ps)
#pragma unroll
      for (int i = 0; i < 2 * M; ++i) zst[sc * CS + (ps * 64 + ss) * 2 * M + i] = buf[ps][i];
  }
  // the matrices: each lane's (at most three) elements located first, then
  // all loads issued together
  constexpr int NLD = (NMAT * MM + 63) / 64;
  double mv[NLD];
#pragma unroll
  for (int it = 0; it < NLD; ++it) {
    const int i = lane + it * 64;
    mv[it] = 0.0;
    if (n < N && i < NMAT * MM) {
      const int m = i / MM, e = i - m * MM;
      const double* cfm = coef + (int64_t)n * Ly::STRIDE;
      const double* scm = scoef + ((int64_t)si * N + n) * Ly::SSTRIDE;
      int off = 0;
      switch (m) {  // offsets only: the loads stay out of the branches
        case 0: off = Ly::AL; break;
        case 1: off = Ly::ALL; break;
        case 2: off = Ly::BL; break;
        case 3: off = Ly::BLL; break;
        case 4: off = Ly::NL; break;
        case 5: off = Ly::NLL; break;
        case 6: off = Ly::IA; break;
        case 7: off = Ly::IB; break;
        default: off = m < 14 ? Ly::PA + ((q - 1) * 6 + (m - 8)) * MM : Ly::PB + ((q - 1) * 6 + (m - 14)) * MM;
      }
      const bool from_s = m < 8 && ((m & 1) || m >= 6);  // the length-dependent ones
      mv[it] = (from_s ? scm : cfm)[off + e];
    }
  }
#pragma unroll
  for (int it = 0; it < NLD; ++it)
    if (lane + it * 64 < NMAT * MM) smat[wv][lane + it * 64] = mv[it];
  __syncthreads();
  if (n < N) {  // the whole wavefront
  const double* cf = smat[wv];
  const int64_t stride = STAGE ? 2 * M : stride_g;
  T* z = STAGE ? zst + wv * CS : zs + (sd.seg0 * N + n) * 2 * M;
  const int64_t a0 = lane * (int64_t)q < nseg ? lane * (int64_t)q : nseg;
  const int64_t a1 = a0 + q < nseg ? a0 + q : nseg;
  const int cnt = (int)(a1 - a0);
  const int lane_last = (int)((nseg - 1) / q);
  // the lane's segment states: zc then za of each
  T r_zc[QR][M], r_za[QR][M];
#pragma unroll
  for (int k = 0; k < QR; ++k)
#pragma unroll
    for (int i = 0; i < M; ++i) {
      r_zc[k][i] = k < cnt ? z[(a0 + k) * stride + i] : T(0);
      r_za[k][i] = k < cnt ? z[(a0 + k) * stride + M + i] : T(0);
    }
  const double zero[M] = {};
  auto last_seg = [&](int k) { return a0 + k + 1 == nseg; };
  // ---- causal
  double Y[M] = {};
#pragma unroll
  for (int k = 0; k < QR; ++k) {
    if (k >= cnt) break;
    double zc[M];
#pragma unroll
    for (int i = 0; i < M; ++i) zc[i] = (double)r_zc[k][i];
    matvec_add<M>(cf + (last_seg(k) ? oALL : oAL), Y, zc, Y);
  }
#pragma unroll
  for (int k = 0; k < 6; ++k) {
    const int d = 1 << k;
    double Yo[M];
#pragma unroll
    for (int i = 0; i < M; ++i) Yo[i] = __shfl_up(Y[i], d, 64);
    if (lane >= d) matvec_add<M>(cf + oPA + k * MM, Yo, Y, Y);
  }
  double Ex[M], Tz[M], Tt[M], S0[M], S[M];
#pragma unroll
  for (int i = 0; i < M; ++i) {
    Ex[i] = __shfl_up(Y[i], 1, 64);
    if (lane == 0) Ex[i] = 0.0;
    Tz[i] = Ex[i];
  }
#pragma unroll
  for (int k = 0; k < QR; ++k) {  // lane_last: on to the zero-start total
    if (k >= cnt) break;
    double zc[M];
#pragma unroll
    for (int i = 0; i < M; ++i) zc[i] = (double)r_zc[k][i];
    matvec_add<M>(cf + (last_seg(k) ? oALL : oAL), Tz, zc, Tz);
  }
#pragma unroll
  for (int i = 0; i < M; ++i) Tt[i] = __shfl(Tz[i], lane_last, 64);
  matvec_add<M>(cf + oIA, Tt, zero, S0);
#pragma unroll
  for (int i = 0; i < M; ++i) S[i] = S0[i];
#pragma unroll
  for (int k = 0; k < 6; ++k) {  // A^{qL lane} S_0
    double t[M];
    matvec_add<M>(cf + oPA + k * MM, S, zero, t);
    if ((lane >> k) & 1)
#pragma unroll
      for (int i = 0; i < M; ++i) S[i] = t[i];
  }
#pragma unroll
  for (int i = 0; i < M; ++i) S[i] += Ex[i];
#pragma unroll
  for (int k = 0; k < QR; ++k) {  // the segments' entering states; c_s = za_s + N S_s
    if (k >= cnt) break;
    const bool last = last_seg(k);
    double zc[M], c[M];
#pragma unroll
    for (int i = 0; i < M; ++i) {
      zc[i] = (double)r_zc[k][i];
      c[i] = (double)r_za[k][i];
    }
    matvec_add<M>(cf + (last ? oNLL : oNL), S, c, c);
#pragma unroll
    for (int i = 0; i < M; ++i) {
      r_zc[k][i] = T(S[i]);
      r_za[k][i] = T(c[i]);
    }
    matvec_add<M>(cf + (last ? oALL : oAL), S, zc, S);
  }
  // ---- anti-causal
  double U[M] = {};
#pragma unroll
  for (int k = QR - 1; k >= 0; --k) {
    if (k >= cnt) continue;
    double c[M];
#pragma unroll
    for (int i = 0; i < M; ++i) c[i] = (double)r_za[k][i];
    matvec_add<M>(cf + (last_seg(k) ? oBLL : oBL), U, c, U);
  }
#pragma unroll
  for (int k = 0; k < 6; ++k) {
    const int d = 1 << k;
    double Uo[M];
#pragma unroll
    for (int i = 0; i < M; ++i) Uo[i] = __shfl_down(U[i], d, 64);
    if (lane + d < 64) matvec_add<M>(cf + oPB + k * MM, Uo, U, U);
  }
  double Ut[M], F0[M], Wz[M], Wt[M], Gn[M], V[M];
#pragma unroll
  for (int i = 0; i < M; ++i) {
    Ut[i] = __shfl(U[i], 0, 64);
    Gn[i] = __shfl_down(U[i], 1, 64);
  }
  matvec_add<M>(cf + oIB, Ut, zero, F0);
#pragma unroll
  for (int i = 0; i < M; ++i) Wz[i] = F0[i];
#pragma unroll
  for (int k = QR - 1; k >= 0; --k) {  // lane_last: W = B^{len} F_0
    if (k >= cnt) continue;
    matvec_add<M>(cf + (last_seg(k) ? oBLL : oBL), Wz, zero, Wz);
  }
#pragma unroll
  for (int i = 0; i < M; ++i) Wt[i] = __shfl(Wz[i], lane_last, 64);
  const int mpow = lane_last - 1 - lane;
#pragma unroll
  for (int i = 0; i < M; ++i) V[i] = Wt[i];
#pragma unroll
  for (int k = 0; k < 6; ++k) {  // B^{qL (lane_last - 1 - lane)} W
    double t[M];
    matvec_add<M>(cf + oPB + k * MM, V, zero, t);
    if (mpow >= 0 && ((mpow >> k) & 1))
#pragma unroll
      for (int i = 0; i < M; ++i) V[i] = t[i];
  }
#pragma unroll
  for (int i = 0; i < M; ++i) V[i] = lane < lane_last ? V[i] + Gn[i] : F0[i];
#pragma unroll
  for (int k = QR - 1; k >= 0; --k) {  // right to left: segment s receives F_{s+1}
    if (k >= cnt) continue;
    double c[M];
#pragma unroll
    for (int i = 0; i < M; ++i) {
      c[i] = (double)r_za[k][i];
      r_za[k][i] = T(V[i]);
    }
    matvec_add<M>(cf + (last_seg(k) ? oBLL : oBL), V, c, V);
  }
#pragma unroll
  for (int k = 0; k < QR; ++k)
    if (k < cnt)
#pragma unroll
      for (int i = 0; i < M; ++i) {
        z[(a0 + k) * stride + i] = r_zc[k][i];
        z[(a0 + k) * stride + M + i] = r_za[k][i];
      }
  }  // n < N
  if constexpr (STAGE) {
    __syncthreads();
#pragma unroll
    for (int ps = 0; ps < QR; ++ps) {
      const int sg = ps * 64 + ss;
      if (sg < nseg && sc < ncol)
#pragma unroll
        for (int i = 0; i < 2 * M; ++i) zb[sg * sgs + sc * 2 * M + i] = zst[sc * CS + sg * 2 * M + i];
    }
  }
}

// Pass 2: per (column, segment), the causal ARMA from its entering state,
// its outputs kept in registers (a full segment) or LDS (a partial one; each
// thread its own column: no barriers), then the anti-causal recursion
// backwards from the right-hand state; xhat = gain * v written over d, or
// (dst) its frames [doff, doff + dkeep) to dst. One wavefront of 64 columns
// per workgroup; workgroup w takes global segment w / ntiles.
template <typename T, int M, int L>
__global__ __launch_bounds__(64) void k_iir_apply(int N, int ntiles, IirStream one, const IirStream* __restrict__ tab,
                                                   int nstreams, const double* __restrict__ coef,
                                                   const T* __restrict__ zs, double gnorm, T* __restrict__ dst,
                                                   int64_t doff, int64_t dkeep) {
  using Ly = IirLayout<M>;
  extern __shared__ __align__(16) unsigned char iir_lds[];  // L * 64 T, for partial segments only
  T* ys = reinterpret_cast<T*>(iir_lds);
  const int tid = threadIdx.x;
  const int64_t g = __builtin_amdgcn_readfirstlane(blockIdx.x / ntiles);
  const int n = (int)__builtin_amdgcn_readfirstlane(blockIdx.x % ntiles) * 64 + tid;
  if (n >= N) return;
  const IirStream sd = iir_stream_of(g, one, tab, nstreams);
  const int64_t j0 = (g - sd.seg0) * L;
  const int Ls = (int)((sd.b - j0) < L ? (sd.b - j0) : L);
  const double* cf = coef + (int64_t)n * Ly::STRIDE;
  double h[M + 1], a[M], st[M], v[M];
  for (int r = 0; r <= M; ++r) h[r] = cf[Ly::H + r];
  for (int i = 0; i < M; ++i) a[i] = cf[Ly::A + i];
  const double gn = gnorm * cf[Ly::IK];
  const T* zz = zs + (g * N + n) * (2 * M);
  for (int i = 0; i < M; ++i) {
    st[i] = (double)zz[i];
    v[i] = (double)zz[M + i];
  }
  T* px = (T*)sd.x + j0 * (int64_t)N + n;
  // the causal ARMA: y_k from x_k, the state carried in st
  auto causal = [&](double xin) -> double {
    const double y = fma(h[0], xin, st[0]);
#pragma unroll
    for (int i = 0; i + 1 < M; ++i) st[i] = fma(a[i], y, fma(h[i + 1], xin, st[i + 1]));
    st[M - 1] = fma(a[M - 1], y, h[M] * xin);
    return y;
  };
  // the anti-causal all-pole step: w_k = y_k + sum_i a_i w_{k+1+i}
  auto anti = [&](double y) -> double {
    double w = y;
#pragma unroll
    for (int i = 0; i < M; ++i) w = fma(a[i], v[i], w);
#pragma unroll
    for (int i = M - 1; i > 0; --i) v[i] = v[i - 1];
    v[0] = w;
    return gn * w;
  };
  if (Ls == L && (int64_t)L * N * (int64_t)sizeof(T) < (int64_t(1) << 31)) {
    // a full segment: its frames in registers (the launch then gives no LDS,
    // so occupancy is set by registers alone), every load issued at once,
    // straight-line code; one address register for the whole column walk
    const __amdgpu_buffer_rsrc_t rs = buf_rsrc(px - n, (uint32_t)((int64_t)L * N * sizeof(T)));
    const int vo = n * (int)sizeof(T), rowb = N * (int)sizeof(T);
    T yv[L];
#pragma unroll
    for (int k = 0; k < L; ++k) yv[k] = buf_ld<T>(rs, vo, k * rowb);
#pragma unroll
    for (int k = 0; k < L; ++k) yv[k] = T(causal((double)yv[k]));
    if (!dst) {
#pragma unroll
      for (int k = L - 1; k >= 0; --k) buf_st<T>(T(anti((double)yv[k])), rs, vo, k * rowb);
    } else {
#pragma unroll
      for (int k = L - 1; k >= 0; --k) {
        const T val = T(anti((double)yv[k]));
        const int64_t o = j0 + k - doff;  // uniform: the output frame
        if (o >= 0 && o < dkeep) dst[o * N + n] = val;
      }
    }
    return;
  }
  T cur[kIirChunk], nxt[kIirChunk];
  load_chunk(px, N, 0, Ls, cur);
  const int nch = (Ls + kIirChunk - 1) / kIirChunk;
#pragma unroll 1
  for (int c = 0; c < nch; ++c) {
    if (c + 1 < nch) load_chunk(px, N, (c + 1) * kIirChunk, Ls, nxt);
#pragma unroll
    for (int kk = 0; kk < kIirChunk; ++kk) {
      const int k = c * kIirChunk + kk;
      if (k < Ls) ys[k * 64 + tid] = T(causal((double)cur[kk]));
    }
#pragma unroll
    for (int kk = 0; kk < kIirChunk; ++kk) cur[kk] = nxt[kk];
  }
#pragma unroll 4
  for (int k = Ls - 1; k >= 0; --k) {
    const T val = T(anti((double)ys[k * 64 + tid]));
    if (!dst) {
      ((__attribute__((address_space(1))) T*)px)[(int64_t)k * N] = val;
    } else {
      const int64_t o = j0 + k - doff;
      if (o >= 0 && o < dkeep) dst[o * N + n] = val;
    }
  }
}

template <int M>
static hipError_t launch_iir_m(int stage, int prec, const IirStream& one, const IirStream* tab, int nstreams,
                               int64_t nsegt, int64_t max_nseg, int N, const double* win64, double phi,
                               double gnorm, double* coef, double* scoef, void* zs, hipStream_t st, int precond,
                               void* dst, int64_t doff, int64_t dkeep) {
  const int L = prec == F32 ? kIirSegF32 : kIirSegF64;
  const int t256 = (N + 255) / 256, t64 = (N + 63) / 64;
  if (nsegt * t64 > 0x7fffffffLL) return hipErrorNotSupported;  // one-dimensional grids
  switch (stage) {
    case kIirSetup:
      k_iir_setup<M><<<dim3((unsigned)((N + 63) / 64)), 64, 0, st>>>(win64, N, phi, L, coef, precond);
      break;
    case kIirSetupLen:
      k_iir_setup_len<M><<<dim3((unsigned)(((int64_t)nstreams * N + 63) / 64)), 64, 0, st>>>(N, L, one, tab,
                                                                                              nstreams, coef, scoef);
      break;
    case kIirPass1:
      if (prec == F32)
        k_iir_zs<float, M, kIirSegF32><<<dim3((unsigned)(nsegt * t256)), 256, 0, st>>>(N, t256, nsegt, one, tab,
                                                                                       nstreams, coef, (float*)zs);
      else
        k_iir_zs<double, M, kIirSegF64><<<dim3((unsigned)(nsegt * t256)), 256, 0, st>>>(N, t256, nsegt, one, tab,
                                                                                        nstreams, coef, (double*)zs);
      break;
    case kIirCarry: {
      const dim3 g4((unsigned)((int64_t)nstreams * ((N + 3) / 4)));  // one wavefront per (stream, column)
#define CARRY(T) k_iir_carry<T, M><<<g4, 256, 0, st>>>(N, L, one, tab, nstreams, coef, scoef, (T*)zs)
      if (max_nseg * (int64_t)N * 2 * M >= (int64_t(1) << 31)) return hipErrorNotSupported;
#define CARRY_U(T, Q) \
  k_iir_carry_u<T, M, Q><<<dim3((unsigned)((int64_t)nstreams * ((N + carry_u_cols<T, Q>() - 1) / carry_u_cols<T, Q>()))), \
                           64 * carry_u_cols<T, Q>(), 0, st>>>(N, L, one, tab, nstreams, coef, scoef, (T*)zs)
      static_assert(kIirQMax == 8, "the uniform-power carry takes up to 8 segments per lane");
      if (prec == F32) {
        if (max_nseg <= 64 * 4) CARRY_U(float, 4);
        else if (max_nseg <= 64 * 8) CARRY_U(float, 8);
        else CARRY(float);
      } else {
        if (max_nseg <= 64 * 4) CARRY_U(double, 4);
        else if (max_nseg <= 64 * 8) CARRY_U(double, 8);
        else CARRY(double);
      }
#undef CARRY_U
#undef CARRY
      break;
    }
    default: {
      // LDS for the partial segments' outputs, unless every segment is full
      // (one stream of a multiple of L frames) and takes the register path
      const size_t es = prec == F32 ? sizeof(float) : sizeof(double);
      const bool all_full = !tab && one.b % L == 0 && (int64_t)L * N * (int64_t)es < (int64_t(1) << 31);
      const size_t lds = all_full ? 0 : (size_t)L * 64 * es;
      if (prec == F32)
        k_iir_apply<float, M, kIirSegF32><<<dim3((unsigned)(nsegt * t64)), 64, lds, st>>>(
            N, t64, one, tab, nstreams, coef, (const float*)zs, gnorm, (float*)dst, doff, dkeep);
      else
        k_iir_apply<double, M, kIirSegF64><<<dim3((unsigned)(nsegt * t64)), 64, lds, st>>>(
            N, t64, one, tab, nstreams, coef, (const double*)zs, gnorm, (double*)dst, doff, dkeep);
      break;
    }
  }
  return hipGetLastError();
}

hipError_t launch_col_iir(int stage, int prec, const IirStream& one, const IirStream* tab, int nstreams,
                          int64_t nsegt, int64_t max_nseg, int N, int ntap, const double* win64, double phi,
                          double gnorm, double* coef, double* scoef, void* zs, hipStream_t st, int precond,
                          void* dst, int64_t doff, int64_t dkeep) {
  if (N < 1 || nsegt < 1) return hipSuccess;
  if (dst && tab) return hipErrorInvalidValue;
  switch (ntap) {
    case 4:
      return launch_iir_m<3>(stage, prec, one, tab, nstreams, nsegt, max_nseg, N, win64, phi, gnorm, coef, scoef, zs,
                             st, precond, dst, doff, dkeep);
    default: return hipErrorNotSupported;
  }
}

}  // namespace ipfb
