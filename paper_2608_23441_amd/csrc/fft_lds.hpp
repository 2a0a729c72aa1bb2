// LDS-resident Stockham FFTs for gfx950 (wave64), used by every kernel of the
// circulant inverse PFB: the N-point row transforms that undo F, the b-point
// column transforms of the circulant decorrelation (Section 3.1), and the
// transforms of the forward PFB used for up-channelization (Section 2.2).
//
// A workgroup transforms C independent complex sequences of length L (a power
// of two) that sit in LDS at stride LS. Each pass loads all of a thread's
// butterfly inputs into registers, waits at a barrier, and writes the radix-R
// outputs in autosort (Stockham) order, so no bit reversal is ever needed.
// Twiddles come from a precomputed table of exp(-2 pi i m / LT) (computed in
// double precision on the host and rounded once for the float form).
#pragma once
#include <hip/hip_runtime.h>

namespace ipfb {

template <typename T>
struct alignas(2 * sizeof(T)) cx {
  T x, y;
};

template <typename T>
__device__ __forceinline__ cx<T> mk(T a, T b) { cx<T> r; r.x = a; r.y = b; return r; }
template <typename T>
__device__ __forceinline__ cx<T> operator+(cx<T> a, cx<T> b) { return mk<T>(a.x + b.x, a.y + b.y); }
template <typename T>
__device__ __forceinline__ cx<T> operator-(cx<T> a, cx<T> b) { return mk<T>(a.x - b.x, a.y - b.y); }
template <typename T>
__device__ __forceinline__ cx<T> cmul(cx<T> a, cx<T> b) {
  return mk<T>(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// a * conj(b)
template <typename T>
__device__ __forceinline__ cx<T> cmulc(cx<T> a, cx<T> b) {
  return mk<T>(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);
}
template <typename T>
__device__ __forceinline__ cx<T> conj(cx<T> a) { return mk<T>(a.x, -a.y); }
template <typename T>
__device__ __forceinline__ cx<T> scale(cx<T> a, T s) { return mk<T>(a.x * s, a.y * s); }
// Load of a value that this kernel reads once and does not write back: a
// non-temporal load. Read streams loaded this way leave the last-level cache
// to the lines the kernel writes, which the next kernel reads.
template <typename T>
__device__ __forceinline__ cx<T> ld_once(const cx<T>* p) {
  typedef T v2 __attribute__((ext_vector_type(2)));
  const v2 v = __builtin_nontemporal_load(reinterpret_cast<const v2*>(p));
  return mk<T>(v.x, v.y);
}
// Global-memory access through a pointer the compiler cannot place (one read
// from a table in memory): without the cast it emits flat instructions, which
// also count against the LDS wait counter, so every LDS wait would also wait
// for them.
template <typename T>
__device__ __forceinline__ void st_global(cx<T>* p, cx<T> v) {
  typedef T v2 __attribute__((ext_vector_type(2)));
  *(__attribute__((address_space(1))) v2*)p = v2{v.x, v.y};
}
__device__ __forceinline__ unsigned int ld_global_once(const unsigned char* p) {
  return __builtin_nontemporal_load((const __attribute__((address_space(1))) unsigned int*)p);
}
__device__ __forceinline__ unsigned int ld_global_byte(const unsigned char* p) {
  return *(const __attribute__((address_space(1))) unsigned char*)p;
}

// Buffer-resource access to a region of at most 2^31 bytes: a per-lane byte
// offset in one VGPR plus a uniform byte offset in an SGPR, so a strided walk
// over many rows keeps a single address register (flags word: gfx9 raw
// buffer, 32-bit data format; accesses past `bytes` read 0 and are dropped).
__device__ __forceinline__ __amdgpu_buffer_rsrc_t buf_rsrc(const void* base, uint32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)bytes, 0x00020000);
}
template <typename T>
__device__ __forceinline__ T buf_ld(__amdgpu_buffer_rsrc_t r, int voff, int soff) {
  if constexpr (sizeof(T) == 4) {
    return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0));
  } else {
    typedef unsigned int u2 __attribute__((ext_vector_type(2)));
    const u2 v = __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0);
    return __hiloint2double((int)v.y, (int)v.x);
  }
}
template <typename T>
__device__ __forceinline__ void buf_st(T val, __amdgpu_buffer_rsrc_t r, int voff, int soff) {
  if constexpr (sizeof(T) == 4) {
    __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(val), r, voff, soff, 0);
  } else {
    typedef unsigned int u2 __attribute__((ext_vector_type(2)));
    const u2 v = {(unsigned)__double2loint(val), (unsigned)__double2hiint(val)};
    __builtin_amdgcn_raw_buffer_store_b64(v, r, voff, soff, 0);
  }
}
// multiply by DIR*i  (DIR = -1: forward transform kernel e^{-i...}; +1 inverse)
template <int DIR, typename T>
__device__ __forceinline__ cx<T> mul_i(cx<T> a) {
  if constexpr (DIR < 0) return mk<T>(a.y, -a.x);
  else return mk<T>(-a.y, a.x);
}

// ---- small DFT codelets, in registers ------------------------------------
template <int DIR, typename T>
__device__ __forceinline__ void dft2(cx<T>* v) {
  cx<T> a = v[0];
  v[0] = a + v[1];
  v[1] = a - v[1];
}

template <int DIR, typename T>
__device__ __forceinline__ void dft4(cx<T>& a0, cx<T>& a1, cx<T>& a2, cx<T>& a3) {
  cx<T> y0 = a0 + a2, y1 = a0 - a2, y2 = a1 + a3, y3 = mul_i<DIR>(a1 - a3);
  a0 = y0 + y2;
  a2 = y0 - y2;
  a1 = y1 + y3;
  a3 = y1 - y3;
}

template <int DIR, typename T>
__device__ __forceinline__ void dft4v(cx<T>* v) { dft4<DIR>(v[0], v[1], v[2], v[3]); }

template <int DIR, typename T>
__device__ __forceinline__ void dft8(cx<T>* v) {
  const T h = T(0.70710678118654752440084436210485);
  cx<T> e0 = v[0], e1 = v[2], e2 = v[4], e3 = v[6];
  cx<T> o0 = v[1], o1 = v[3], o2 = v[5], o3 = v[7];
  dft4<DIR>(e0, e1, e2, e3);
  dft4<DIR>(o0, o1, o2, o3);
  // w8^1 = (h, DIR*h), w8^2 = DIR*i, w8^3 = (-h, DIR*h)
  o1 = mk<T>(h * (o1.x - T(DIR) * o1.y), h * (o1.y + T(DIR) * o1.x));
  o2 = mul_i<DIR>(o2);
  o3 = mk<T>(-h * (o3.x + T(DIR) * o3.y), h * (T(DIR) * o3.x - o3.y));
  v[0] = e0 + o0; v[4] = e0 - o0;
  v[1] = e1 + o1; v[5] = e1 - o1;
  v[2] = e2 + o2; v[6] = e2 - o2;
  v[3] = e3 + o3; v[7] = e3 - o3;
}

template <int DIR, typename T>
__device__ __forceinline__ cx<T> rot16(cx<T> a, int m) {
  // a * exp(DIR * 2 pi i m / 16), m in {1,2,3,4,6,9}
  const T c1 = T(0.92387953251128675612818318939679);
  const T s1 = T(0.38268343236508977172845998403040);
  const T h = T(0.70710678118654752440084436210485);
  T c, s;
  switch (m) {
    case 1: c = c1; s = s1; break;
    case 2: c = h; s = h; break;
    case 3: c = s1; s = c1; break;
    case 4: c = 0; s = 1; break;
    case 6: c = -h; s = h; break;
    default: c = -c1; s = -s1; break;  // m = 9: angle 202.5 deg
  }
  s *= T(DIR);
  return mk<T>(a.x * c - a.y * s, a.x * s + a.y * c);
}

template <int DIR, typename T>
__device__ __forceinline__ void dft16(cx<T>* v) {
  // X[k1 + 4 k2] = sum_{n2} w4^{n2 k2} w16^{n2 k1} sum_{n1} a[4 n1 + n2] w4^{n1 k1}
  cx<T> b[16];
#pragma unroll
  for (int n2 = 0; n2 < 4; ++n2) {
    cx<T> a0 = v[n2], a1 = v[n2 + 4], a2 = v[n2 + 8], a3 = v[n2 + 12];
    dft4<DIR>(a0, a1, a2, a3);
    b[n2 * 4 + 0] = a0;
    b[n2 * 4 + 1] = (n2 == 0) ? a1 : rot16<DIR>(a1, n2);
    b[n2 * 4 + 2] = (n2 == 0) ? a2 : rot16<DIR>(a2, 2 * n2);
    b[n2 * 4 + 3] = (n2 == 0) ? a3 : rot16<DIR>(a3, 3 * n2);
  }
#pragma unroll
  for (int k1 = 0; k1 < 4; ++k1) {
    cx<T> a0 = b[k1], a1 = b[4 + k1], a2 = b[8 + k1], a3 = b[12 + k1];
    dft4<DIR>(a0, a1, a2, a3);
    v[k1] = a0;
    v[k1 + 4] = a1;
    v[k1 + 8] = a2;
    v[k1 + 12] = a3;
  }
}

template <int R, int DIR, typename T>
__device__ __forceinline__ void dftR(cx<T>* v) {
  if constexpr (R == 2) dft2<DIR>(v);
  else if constexpr (R == 4) dft4v<DIR>(v);
  else if constexpr (R == 8) dft8<DIR>(v);
  else dft16<DIR>(v);
}

__host__ __device__ constexpr int ilog2c(int v) { return v <= 1 ? 0 : 1 + ilog2c(v >> 1); }

// LDS index of element i of a sequence: one padding slot after every 16
// elements, so the stride-R writes of the early Stockham passes (and the
// stride-16 writes of radix-16) spread over the banks instead of piling onto
// one. A sequence of length L therefore occupies lds_len(L) slots.
__device__ __forceinline__ int pidx(int i) { return i + (i >> 4); }
__host__ __device__ constexpr int lds_len(int L) { return L + (L >> 4) + 1; }

// ---- one Stockham pass ------------------------------------------------------
// s: C sequences of length L at stride LS (>= lds_len(L)), element i of a
// sequence at pidx(i). Ns: product of radices already done.
// tw: table of exp(-2 pi i m / LT) with LT = L * twmul. FULLTW: the table
// holds all LT entries and every w^{rk} is read from it (no products; for
// kernels whose time goes to vector arithmetic rather than memory).
//
// L, R and Ns are powers of two, so an element's padded index splits into a
// per-thread base plus a compile-time offset: the reads j + r L/R (j < L/R)
// and the writes m R Ns + k + r Ns (k < Ns) never carry into another
// 16-element block except through the r term, hence
//   pidx(a + r S) = pidx(a) + r S + (r S >> 4)  for S = L/R and S = Ns.
// Twiddles and the radix-R butterfly of one Stockham pass, in registers:
// v[r] = element j + r L/R of a sequence, k = j mod Ns.
template <typename T, int L, int R, int DIR, int Ns, bool FULLTW>
__device__ __forceinline__ void stockham_bfly(cx<T>* v, int k, const cx<T>* __restrict__ tw, int twmul) {
  if constexpr (Ns > 1) {
    // w^{rk} for r = 1..R-1 from the table entries for r = 1, 2, 4, 8
    // (power-of-two multiples of k): at most three products per twiddle
    const int step = (L / (Ns * R)) * twmul;
    cx<T> w[R];
    if constexpr (FULLTW) {
#pragma unroll
      for (int r = 1; r < R; ++r) w[r] = tw[r * k * step];  // r k step < (R-1)/R LT
    } else {
      w[1] = tw[k * step];
      if constexpr (R > 2) w[2] = tw[2 * k * step];
      if constexpr (R > 4) w[4] = tw[4 * k * step];
      if constexpr (R > 8) w[8] = tw[8 * k * step];
#pragma unroll
      for (int r = 3; r < R; ++r) {
        if ((r & (r - 1)) == 0) continue;
        const int hi = 1 << (31 - __builtin_clz(r));  // highest power of two in r
        w[r] = cmul(w[r - hi], w[hi]);
      }
    }
#pragma unroll
    for (int r = 1; r < R; ++r) v[r] = (DIR < 0) ? cmul(v[r], w[r]) : cmulc(v[r], w[r]);
  }
  dftR<R, DIR>(v);
}

template <typename T, int L, int R, int NT, int C, int DIR, int Ns, bool FULLTW = false>
__device__ __forceinline__ void stockham_pass(cx<T>* s, int LS, const cx<T>* __restrict__ tw, int twmul) {
  constexpr int LR = L / R;
  constexpr int NB = C * LR;
  constexpr int BPT = (NB + NT - 1) / NT;
  const int tid = threadIdx.x;
  cx<T> v[BPT][R];
#pragma unroll
  for (int i = 0; i < BPT; ++i) {
    const int g = tid + i * NT;
    if ((NB % NT == 0) || g < NB) {
      const int c = g / LR, j = g % LR;
      const cx<T>* src = s + c * LS + pidx(j);
#pragma unroll
      for (int r = 0; r < R; ++r) v[i][r] = src[r * LR + ((r * LR) >> 4)];
    }
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < BPT; ++i) {
    const int g = tid + i * NT;
    if ((NB % NT == 0) || g < NB) {
      const int c = g / LR, j = g % LR;
      const int k = j & (Ns - 1);
      stockham_bfly<T, L, R, DIR, Ns, FULLTW>(v[i], k, tw, twmul);
      cx<T>* dst = s + c * LS + pidx((j - k) * R + k);
#pragma unroll
      for (int r = 0; r < R; ++r) dst[r * Ns + ((r * Ns) >> 4)] = v[i][r];
    }
  }
  __syncthreads();
}

// Radix schedule: P passes of at most RMAXLOG bits each, bits spread evenly.
template <int L, int RMAXLOG>
struct FftSched {
  static constexpr int E = ilog2c(L);
  static constexpr int P = (E + RMAXLOG - 1) / RMAXLOG;
  static constexpr int bits(int pass) { return E / P + ((pass < E % P) ? 1 : 0); }
  static constexpr int nslog(int pass) { return pass == 0 ? 0 : nslog(pass - 1) + bits(pass - 1); }
};

// Largest radix (log2) lds_fft uses for EPT elements per thread.
__host__ __device__ constexpr int fft_rmaxlog(int ept) { return ept >= 16 ? 4 : (ept >= 8 ? 3 : (ept >= 4 ? 2 : 1)); }

// Passes PASS .. PEND-1 of the schedule (NSLOG: log2 of Ns at PASS).
template <typename T, int L, int NT, int C, int DIR, int RMAXLOG, int PASS, int PEND, int NSLOG, bool FULLTW>
__device__ __forceinline__ void stockham_range(cx<T>* s, int LS, const cx<T>* __restrict__ tw, int twmul) {
  if constexpr (PASS < PEND) {
    constexpr int bits = FftSched<L, RMAXLOG>::bits(PASS);
    stockham_pass<T, L, (1 << bits), NT, C, DIR, (1 << NSLOG), FULLTW>(s, LS, tw, twmul);
    stockham_range<T, L, NT, C, DIR, RMAXLOG, PASS + 1, PEND, NSLOG + bits, FULLTW>(s, LS, tw, twmul);
  }
}

template <typename T, int L, int NT, int C, int DIR, int RMAXLOG, int PASS, int NSLOG, bool FULLTW>
__device__ __forceinline__ void stockham_rec(cx<T>* s, int LS, const cx<T>* __restrict__ tw, int twmul) {
  stockham_range<T, L, NT, C, DIR, RMAXLOG, PASS, FftSched<L, RMAXLOG>::P, NSLOG, FULLTW>(s, LS, tw, twmul);
}

// Full unnormalised transform, exp(DIR * 2 pi i jk / L). Ends with a barrier.
template <typename T, int L, int NT, int C, int DIR, bool FULLTW = false>
__device__ __forceinline__ void lds_fft(cx<T>* s, int LS, const cx<T>* __restrict__ tw, int twmul) {
  if constexpr (L > 1) {
    constexpr int EPT = (L * C) / NT;  // elements per thread
    stockham_rec<T, L, NT, C, DIR, fft_rmaxlog(EPT), 0, 0, FULLTW>(s, LS, tw, twmul);
  }
}

// The same transform split for callers that hold the input in registers
// and/or consume the output straight from the last pass (no LDS round trip
// at either end). Schedule as lds_fft's for C sequences on NT threads:
//   First::R inputs per butterfly; butterfly j of a sequence takes the
//   elements j + r L/R (r < R), has no twiddles (Ns = 1), and its outputs go
//   to LDS at pidx(j R + r): fft_first_from_regs;
//   then, after a barrier, fft_middle (passes 1 .. P-2);
//   then fft_last_to, which hands output element j + r L/R_last of sequence
//   c to out(c, m, value) (consecutive j: consecutive m).
// Requires P >= 2.
template <typename T, int L, int NT, int C>
struct FftSplit {
  static constexpr int EPT = (L * C) / NT;
  static constexpr int RM = fft_rmaxlog(EPT);
  using S = FftSched<L, RM>;
  static constexpr int P = S::P;
  static constexpr int R0 = 1 << S::bits(0);
  static constexpr int RL = 1 << S::bits(P - 1);
  static constexpr bool ok = P >= 2;
};

template <typename T, int R, int DIR>
__device__ __forceinline__ void fft_first_from_regs(cx<T>* seq, int j, cx<T>* v) {
  dftR<R, DIR>(v);
  cx<T>* dst = seq + pidx(j * R);
#pragma unroll
  for (int r = 0; r < R; ++r) dst[r] = v[r];  // j R + r stays in one 16-element block (R <= 16)
}

template <typename T, int L, int NT, int C, int DIR, bool FULLTW = false>
__device__ __forceinline__ void fft_middle(cx<T>* s, int LS, const cx<T>* __restrict__ tw, int twmul) {
  using F = FftSplit<T, L, NT, C>;
  stockham_range<T, L, NT, C, DIR, F::RM, 1, F::P - 1, F::S::nslog(1), FULLTW>(s, LS, tw, twmul);
}

// Passes 1 .. P-1 after fft_first_from_regs (and its barrier), results in
// LDS. Ends with a barrier.
template <typename T, int L, int NT, int C, int DIR, bool FULLTW = false>
__device__ __forceinline__ void fft_rest(cx<T>* s, int LS, const cx<T>* __restrict__ tw, int twmul) {
  using F = FftSplit<T, L, NT, C>;
  stockham_range<T, L, NT, C, DIR, F::RM, 1, F::P, F::S::nslog(1), FULLTW>(s, LS, tw, twmul);
}

// No barrier at the end: LDS is only read. The caller waits before it
// overwrites s.
template <typename T, int L, int NT, int C, int DIR, bool FULLTW, class Out>
__device__ __forceinline__ void fft_last_to(const cx<T>* s, int LS, const cx<T>* __restrict__ tw, int twmul,
                                            Out out) {
  using F = FftSplit<T, L, NT, C>;
  constexpr int R = F::RL, LR = L / R, Ns = LR;
  constexpr int NB = C * LR;
  constexpr int BPT = (NB + NT - 1) / NT;
  const int tid = threadIdx.x;
#pragma unroll
  for (int i = 0; i < BPT; ++i) {
    const int g = tid + i * NT;
    if ((NB % NT == 0) || g < NB) {
      const int c = g / LR, j = g % LR;
      const cx<T>* src = s + c * LS + pidx(j);
      cx<T> v[R];
#pragma unroll
      for (int r = 0; r < R; ++r) v[r] = src[r * LR + ((r * LR) >> 4)];
      stockham_bfly<T, L, R, DIR, Ns, FULLTW>(v, j, tw, twmul);  // k = j mod Ns = j
#pragma unroll
      for (int r = 0; r < R; ++r) out(c, j + r * Ns, v[r]);
    }
  }
}

// Workgroup index remapping so that logically adjacent workgroups share an
// XCD (gfx950 dispatches workgroups round-robin over its 8 XCDs, each with
// its own L2): adjacent column groups then meet in the same L2.
__device__ __forceinline__ int xcd_remap(int bid, int nb) {
  const int q = nb >> 3, r = nb & 7;
  const int xcd = bid & 7, slot = bid >> 3;
  return (xcd < r) ? xcd * (q + 1) + slot : r * (q + 1) + (xcd - r) * q + slot;
}

}  // namespace ipfb
