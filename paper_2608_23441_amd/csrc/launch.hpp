// Internal launcher declarations shared by the kernel translation units and
// the C-ABI layer. Every launcher returns hipSuccess or the launch error.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ipfb {

enum Prec { F32 = 0, F64 = 1 };

// How many workgroups of `kernel` (nt threads, static LDS only) the current
// device holds at once: the grid for kernels that loop over their work.
// Cached per kernel and device.
template <typename K>
inline int resident_workgroups(K kernel, int nt) {
  static int cache[16] = {0};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0) dev = 0;
  const int slot = dev < 16 ? dev : 15;
  if (cache[slot] > 0) return cache[slot];
  int cus = 0, per = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) cus = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, kernel, nt, 0) != hipSuccess) per = 0;
  hipGetLastError();
  if (cus < 1) cus = 1;
  if (per < 1) per = 1;
  cache[slot] = cus * per;
  return cache[slot];
}
// Input spectrum formats of the inverse (match the public header).
enum InFmt { IN_C4 = 0, IN_CI8 = 1, IN_CF32 = 2, IN_CF64 = 3, IN_ADJ = 100 };

// Largest power-of-two lengths each LDS-resident kernel accepts.
constexpr int kMaxLog2RowF32 = 15;  // N real = 2^15 -> 16384 complex, 128 KiB
constexpr int kMaxLog2RowF64 = 14;
constexpr int kMaxLog2ColF32 = 15;
constexpr int kMaxLog2ColF64 = 14;

// Row stage: d_j = inverse real FFT of spectrum j, times per-channel factors.
// fmt IN_C4: packed 4-bit, factor fac[k] = 1/(s_k N) (plan precision, from
// launch_dequant_factors); IN_CF32/IN_CF64: factor 1/N; IN_ADJ: complex in the
// plan precision, factor c_k/2 (transpose of the half-spectrum DFT).
hipError_t launch_row_irfft(int prec, int log2n, int fmt, const void* in, const void* fac,
                            void* out, int64_t nrows, const void* twN, hipStream_t st);
hipError_t launch_dequant_factors(int prec, const float* chan_scale, int nchan, int N, void* fac,
                                  hipStream_t st);
// The row stage for 4-bit spectra in one persistent kernel that forms the
// factors 1/(s_k N) itself; hipErrorNotSupported where the frame length has
// no such kernel (then use launch_dequant_factors + launch_row_irfft).
// nrows = 0 launches nothing (it primes the occupancy query, for callers that
// later launch inside a graph capture).
// tab != NULL: the frames of nstreams streams at once (nrows = their total;
// in, chan_scale and out unused), numbered one stream after another.
struct RowStream {
  const unsigned char* spec;  // packed 4-bit spectra [b][N/2+1]
  const float* scale;         // channel scales [N/2+1]
  void* out;                  // frames [b][N]
  int64_t b;                  // frame count
  int64_t f0;                 // first global frame
};
hipError_t launch_row_c4(int prec, int log2n, const void* in, const float* chan_scale, void* out, int64_t nrows,
                         const void* twN, hipStream_t st, const RowStream* tab = nullptr, int nstreams = 0);

// Column stage as two recursions along the frames (the spectral
// factorisation of |W_n|^2 + phi^2 into causal and anti-causal parts), in
// place on the frame matrices x [b][N] of one or many streams: segments of
// kIirSeg{F32,F64} frames, numbered across the streams one after another
// (stream s owns global segments [seg0, seg0 + ceil(b / seg))). One launch
// per stage: kIirSetup computes the per-column coefficients for this phi
// into coef (N * iir_coef_stride(ntap) doubles), kIirSetupLen the
// per-(stream, column) matrices of each stream's length into scoef
// (nstreams * N * iir_stream_stride(ntap) doubles), kIirPass1 the segments'
// zero-state end states into zs (nsegt * N * 2 (ntap - 1) values of the plan
// precision), kIirCarry the periodic states entering each segment (over
// zs), kIirApply the two recursions from those states, writing xhat over x.
// tab NULL: `one` describes the single stream; else tab is a device array of
// nstreams (>= 1) entries and `one` is unused. max_nseg: the most segments
// of any stream.
// precond = 1 (kIirSetup): the coefficients of 1/(|W_n|^2 + phi^2) instead
// (numerator 1), the inverse of A^T A + phi^2 I; apply it with gnorm = 1.
// dst (kIirApply, tab NULL): NULL to write xhat over x; else frame j of
// xhat goes to dst frame j - doff if 0 <= j - doff < dkeep, and no other
// frame is written (x keeps d).
// hipErrorNotSupported (nothing launched) for tap counts without a kernel.
constexpr int kIirSegF32 = 64, kIirSegF64 = 64;
struct IirStream {
  void* x;       // the stream's frames [b][N], transformed in place
  int64_t b;     // its frame count
  int64_t seg0;  // its first global segment
};
enum { kIirSetup = 0, kIirSetupLen = 1, kIirPass1 = 2, kIirCarry = 3, kIirApply = 4 };
int iir_coef_stride(int ntap);
int iir_stream_stride(int ntap);
hipError_t launch_col_iir(int stage, int prec, const IirStream& one, const IirStream* tab, int nstreams,
                          int64_t nsegt, int64_t max_nseg, int N, int ntap, const double* win64, double phi,
                          double gnorm, double* coef, double* scoef, void* zs, hipStream_t st, int precond = 0,
                          void* dst = nullptr, int64_t doff = 0, int64_t dkeep = 0);

// Tikhonov-regularised solve of each path's linear sub-problem by banded
// Cholesky: x (first b - ntap + 1 rows: d) overwritten with
// cnorm (W^T W + phi^2 I)^{-1} W^T d; ws: (ntap + 1) * b * N doubles.
// ntap in {2, 3, 4, 5, 8, 16}, else hipErrorNotSupported.
hipError_t launch_tikhonov(int prec, void* x, int N, int ntap, int64_t b, const double* win64, double phi,
                           double cnorm, double* ws, hipStream_t st);
// FIR decorrelation: stage 0 fills frames [b][N] with a unit sample at frame
// 0; stage 1 copies lags c0 .. c0 + L - 1 (mod b) of the frames (the kernels,
// after the column stage) into g [L][N]. launch_fir: x[j][n] = sum_{l<L}
// g[l][n] d[(j - c0 - l) mod b][n], L <= kFirMaxTaps.
constexpr int kFirMaxTaps = 255;
hipError_t launch_fir_setup(int prec, int stage, void* frames, void* g, int N, int64_t b, int L, int64_t c0,
                            hipStream_t st);
hipError_t launch_fir(int prec, const void* d, const void* g, void* x, int N, int64_t b, int L, int64_t c0,
                      hipStream_t st);

// Column stage on the transposed frame matrix: per column n (contiguous in
// d_T[n][0..b)), x_T[n] = F^-1[ G_n F d_T[n] ] with the FP64 gain.
// precond = 1 applies the real gain 1/(|W_n|^2 + phi^2) instead (the inverse
// of A^T A + phi^2 I, used as the CG preconditioner). part != NULL: also the
// partial sums of d . xo, one per workgroup, in part[0, kCgParts) (unused
// slots zeroed; hipErrorNotSupported, launching nothing, where the stage
// needs more than kCgParts workgroups).
hipError_t launch_col_wiener(int prec, int log2b, const void* d, void* xo, int lblock, int ntap,
                             const double* win64, double phi, int normalise, const void* twB,
                             const double* twB64, hipStream_t st, int precond = 0, double* part = nullptr);

// The same column stage on the natural layout z = d[b][N] (read as N/2
// complex pairs per frame), in place: on return z holds x[b][N] in time
// order. pass 0, 1, 2 launch the four-step passes A, B, C in that order;
// for b <= 512 pass 1 does the whole stage and passes 0 and 2 launch nothing.
// The work splits into nat_tiles() column tiles (128 bytes of every frame);
// one call covers tiles [tile0, tile0 + ntiles) (ntiles < 0: to the end), and
// the three passes of a tile range may run before those of the next range.
// out != NULL (pass 2 with b > 512 only): frames [r0, r0 + nr) of the result
// go to out (nr frames, same row layout) instead of z, and the others nowhere.
// kind (the gain pass): 0 the Wiener filter (phi), 1 the hard threshold
// |W| >= phi, 2 the Wiener filter with noise-to-signal nu[f] per frequency
// (f in [0, b/2], device doubles).
int nat_tiles(int prec, int lblock);
hipError_t launch_col_wiener_nat(int prec, int log2b, int pass, void* z, int lblock, int ntap, const double* win64,
                                 double phi, int normalise, const void* twB, const double* twB64, hipStream_t st,
                                 int tile0 = 0, int ntiles = -1, void* out = nullptr, int r0 = 0, int nr = 0,
                                 int kind = 0, const double* nu = nullptr);

// Maximum-likelihood CG pieces (vectors in the transposed layout [N][b]).
hipError_t launch_cg_autocorr(const double* win64, int N, int ntap, double* autoc, hipStream_t st);
// mbits: the prior mask transposed to rows of ceil(b/32) words (bit j of row n)
hipError_t launch_cg_normal(int prec, const void* p, void* q, const double* autoc, const uint32_t* mbits,
                            double lam, int ntap, int64_t b, int64_t S, double* part, hipStream_t st);
hipError_t launch_cg_rhs(int prec, const void* d, void* rhs, const double* win64, const uint32_t* mbits,
                         const void* prior, double lam, int N, int ntap, int64_t b, int64_t S, hipStream_t st);
hipError_t launch_cg_resid(int prec, const void* rhs, const void* q, void* r, int64_t S, double* part,
                           hipStream_t st);
hipError_t launch_cg_dot(int prec, const void* a, const void* c, int64_t S, double* part, hipStream_t st);
hipError_t launch_cg_xr(int prec, void* x, void* r, const void* p, const void* q, const double* sc, int64_t S,
                        double* part, hipStream_t st);
hipError_t launch_cg_p(int prec, void* p, const void* z, const double* sc, int use_beta, int64_t S,
                       hipStream_t st);
hipError_t launch_cg_scalar(const double* part, int mode, double* sc, double* resid, int k, hipStream_t st);
// The same two stencils on the natural layout [b][N] (4 taps; else
// hipErrorNotSupported), the mask being the time-order bitmask itself.
hipError_t launch_cg_normal_nat(int prec, const void* p, void* q, const double* autoc, const uint32_t* mbits,
                                double lam, int N, int ntap, int64_t b, double* part, hipStream_t st);
hipError_t launch_cg_rhs_nat(int prec, const void* d, void* rhs, const double* win64, const uint32_t* mbits,
                             const void* prior, double lam, int N, int ntap, int64_t b, hipStream_t st);
// time-order bitmask (bit e = sample j N + n) -> transposed rows of ceil(b/32) words
hipError_t launch_maskbits_transpose(const uint32_t* in, int N, int64_t b, uint32_t* out, hipStream_t st);
constexpr int kCgParts = 1024;

// Tunable shape of the Bluestein column path for one convolution length
// M = 2^log2m: split M1 = 2^l1 (1 <= l1, log2m - l1 <= 8), tile widths
// mb, kb in {8, 16, 32}, pairs per launch group (0: all), fuse = 1: the
// inverse of the first convolution, the gain and the forward of the second in
// one pass over the scratch (0: three kernels through Z and A).
// nat = 1: the natural-layout path (in place on d[b][N], tiles of column
// pairs, always fused; mb, kb and fuse unused, pchunk counts tiles).
struct BluCfg {
  int l1 = 0, mb = 16, kb = 16, pchunk = 0, fuse = 1, nat = 0;
};
bool blu_cfg_valid(int log2m, const BluCfg& c);
BluCfg blu_cfg_default(int log2m);

// Arbitrary-length column stage (Bluestein): dT, xT [N][b] real; Tm scratch
// (min(pchunk, (N+1)/2) * 2^log2m complex), Z and A scratch ((N+1)/2 * b
// complex each; Z may alias xT and A may alias dT: pair p's rows are read
// before they are overwritten); chirp [b] complex e^{i pi m^2/b}; Crow
// [M1][M2] complex = FFT_M of the symmetric chirp filter in row layout for
// the split cfg.l1; twb64 [b] double complex e^{-2 pi i m/b};
// tw4 = {tM1 [M1], tM2 [M2], tLo [256], tHi [max(1, M/256)]}.
// The Bluestein column stage in place on the natural layout x[b][N] (the
// rows' output, overwritten with the result); Tm: scratch of
// min(pchunk, tiles) * tile_pairs * 2^log2m complex, tiles = ceil(N/2 / tile_pairs).
int blu_nat_tile_pairs(int prec);
hipError_t launch_blu_nat(int prec, void* x, void* Tm, const void* chirp, const void* Crow, const double* twb64,
                          int64_t b, int log2m, const BluCfg& cfg, int N, int ntap, const double* win64, double phi,
                          int normalise, const void* const tw4[4], hipStream_t st);
hipError_t launch_blu_columns(int prec, const void* dT, void* xT, void* Tm, void* Z, void* A, const void* chirp,
                              const void* Crow, const double* twb64, int64_t b, int log2m, const BluCfg& cfg,
                              int N, int ntap, const double* win64, double phi, int normalise,
                              const void* const tw4[4], hipStream_t st);

// Forward PFB with LDS-resident rows (N <= 2^kMaxLog2Row*).
hipError_t launch_pfb_fwd_small(int prec, int log2n, const void* x, void* y, int64_t nblock, int ntap,
                                const void* winT, const void* twN, hipStream_t st);

// Forward PFB for long frames (2^15 <= N <= 2^20): one frame per complex
// M = N/2-point FFT (even and odd samples packed), M = P1 * P2 with
// P2 = 2^lf_log2p2(prec, log2 M), in two passes through tmp (nblock * M complex).
// part: NULL, or [ceil(nblock / fchunk)][N/2+1] doubles receiving per-chunk
// sums of |Y_jk|^2. twS: tables [P1 | P2 | 512 | M/512 | 512 | M/512 + 1] of
// e^{-2 pi i m/P1}, e^{-2 pi i m/P2}, e^{-2 pi i m/M} (m < 512),
// e^{-2 pi i 512 m/M}, e^{-2 pi i k/N} (k < 512), e^{-2 pi i 512 m/N}.
// Frames per power-sum chunk of the second pass: one workgroup per row group
// and chunk, about as many workgroups as the device holds at once.
int lf_frame_chunk(int prec, int log2n, int64_t nblock);
// log2 P2 of the split M = P1 * P2. FP32: ceil(log2 M / 2), at most 9, so for
// odd log2 M the first pass takes the shorter FFT (P1 = P2 / 2), which leaves
// room in its registers for 128-byte column blocks (measured at M = 2^17: first
// pass 156 -> 121 us, second 120 -> 124 us). FP64: floor(log2 M / 2), the
// other way round (there the second pass would lose more than the first gains:
// 279 + 219 us against 262 + 253 us).
__host__ __device__ constexpr int lf_log2p2(int prec, int log2m) {
  return prec == F64 ? log2m / 2 : ((log2m + 1) / 2 < 9 ? (log2m + 1) / 2 : 9);
}
// pass 0 launches the first FFT pass only, 1 the second only, -1 both.
hipError_t launch_pfb_fwd_long(int prec, int log2n, int pass, const void* x, void* y, int64_t nblock, int ntap,
                               const void* winT, const void* twS, void* tmp, int fchunk, double* part,
                               hipStream_t st);

// Appendix B diagnostics: d = a - b (n reals); out = num / den (n doubles);
// the predicted delta(f) at f = k / nfreq for white input (phi > 0: Wiener,
// phi = 0: naive with the given SNR).
hipError_t launch_sub(int prec, const void* a, const void* b, void* d, int64_t n, hipStream_t st);
hipError_t launch_ratio(const double* num, const double* den, double* out, int n, hipStream_t st);
hipError_t launch_delta_analytic(const double* win64, int N, int ntap, int64_t nfreq, double phi, double snr,
                                 double* out, hipStream_t st);

// the structured prior mask as a time-order bitmask of ceil(S/32) words: bit
// e = j N + n set at frames j = 0 mod R of paths [N/2 - L/2, N/2 + L/2)
hipError_t launch_mask_structured(uint32_t* bits, int N, int64_t nblock, int R, int L, hipStream_t st);
// one byte per sample (nonzero = saved) -> time-order bitmask of ceil(S/32) words
hipError_t launch_mask_pack(const uint8_t* mask, int64_t S, uint32_t* bits, hipStream_t st);

// bytes zero bytes at p (a kernel, so that it may sit in a captured graph)
hipError_t launch_zero(void* p, size_t bytes, hipStream_t st);

// out[c][r] = in[r][c] for an in[rows][cols] matrix (64 x 64 LDS tiles)
hipError_t launch_transpose(int prec, const void* in, void* out, int64_t rows, int64_t cols, hipStream_t st);

// x[i][n] = sum_r h[rN+n] z[(i-r) mod b][n]
hipError_t launch_adjoint_gather(int prec, const void* z, void* x, int64_t nblock, int lblock, int ntap,
                                 const void* winT, hipStream_t st);

// part[c][k] = sum_{j in chunk c} |y_jk|^2 (FP64), nchunks = ceil(nspec / jchunk).
hipError_t launch_power_partial(int prec, const void* y, int64_t nspec, int nchan, int jchunk,
                                double* part, hipStream_t st);
// out[k] = mult * sum_c part[c][k]
hipError_t launch_power_final(const double* part, int nchunks, int nchan, double mult, double* out,
                              hipStream_t st);
// s_k = float(levels / sqrt(pw_k)), where pw_k = mean power / 2 is given.
hipError_t launch_scales(const double* halfpow, int nchan, double levels, float* scales, hipStream_t st);
hipError_t launch_quantize(int prec, const void* y, int64_t nspec, int nchan, const float* scales,
                           uint8_t* packed, hipStream_t st);

}  // namespace ipfb
