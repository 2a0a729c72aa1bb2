/*
 * ipfb.h - C ABI of libipfb, the MI355X (gfx950) implementation of the
 * circulant inverse polyphase filter bank and up-channelization of
 * Fay et al., "Inverting and Up-channelizing Critically-Sampled Polyphase
 * Filter Banks".
 *
 * Problem statement (Section 2.3 and Section 3): a real timestream x of
 * nblock frames of lblock samples, stored frame-major (x[j*lblock + n]), is
 * channelised by the PFB y = F S W x with an ntap-tap window h of length
 * ntap*lblock; spectrum j uses frames j..j+ntap-1, wrapping circularly (the
 * circulant model of Section 3.1), so there are nblock spectra of
 * lblock/2+1 channels, stored [nblock][lblock/2+1] as interleaved (re, im).
 *
 * Conventions common to every call:
 *  - Every data pointer is a device pointer owned by the caller unless the
 *    argument says "host". The library never frees caller memory.
 *  - stream is a hipStream_t (NULL = the default stream). Calls enqueue work
 *    and return without synchronising. A plan must not be used from two
 *    streams at once: it owns one workspace.
 *  - Arguments are validated before anything is enqueued; on failure the call
 *    returns a negative status, writes no output, and ipfb_last_error()
 *    returns a message (per thread).
 *  - Real arrays are float (IPFB_F32 plans) or double (IPFB_F64 plans);
 *    complex arrays are pairs of the same type.
 *  - Lengths: lblock is a power of two >= 4. Inverse: lblock <= 32768 (F32)
 *    / 16384 (F64). With ntap = 4 and phi >= 1e-3 the recursive column stage
 *    takes any nblock >= 1 (ipfb_plan_set_column_method); otherwise nblock
 *    is an integer in [2, 32768] (powers of two up to 2^15 (F32) / 2^14
 *    (F64) use the LDS column kernel, other lengths the Bluestein column
 *    path, set up on the first call). Forward PFB / up-channelization:
 *    lblock up to 2^20, any nblock >= 1. ML-CG: nblock a power of two within
 *    the LDS column limits.
 */
#ifndef IPFB_H
#define IPFB_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  IPFB_OK = 0,
  IPFB_EINVAL = -1,       /* bad argument (NULL pointer, size, mismatched plan) */
  IPFB_EUNSUPPORTED = -2, /* valid problem outside the supported shapes */
  IPFB_ENOMEM = -3,       /* device allocation failed */
  IPFB_EHIP = -4          /* HIP runtime or launch error */
} ipfb_status;

typedef enum { IPFB_F32 = 0, IPFB_F64 = 1 } ipfb_prec;

/* Spectrum formats accepted by the inverse.
 * IPFB_IN_C4: one byte per complex value, real part in the high nibble and
 *   imaginary part in the low nibble, each 4-bit two's complement in -7..7
 *   (Section 4.3's 15-level quantiser), with a per-channel float scale s_k:
 *   the spectrum is q / s_k.
 * IPFB_IN_CI8: two bytes per complex value, the real then the imaginary
 *   part, each an 8-bit two's complement code, with the same per-channel
 *   scale: the spectrum is q / s_k (a finer quantiser than Section 4.3's).
 * IPFB_IN_CF32 / IPFB_IN_CF64: interleaved float / double complex.
 * chan_scale arguments below are required for the two quantised formats
 * and ignored (may be NULL) for the float ones. */
typedef enum { IPFB_IN_C4 = 0, IPFB_IN_CI8 = 1, IPFB_IN_CF32 = 2, IPFB_IN_CF64 = 3 } ipfb_infmt;

typedef struct ipfb_plan_s* ipfb_plan;

/* Message for the last failed call on this thread ("" if none). */
const char* ipfb_last_error(void);

/* Version string of the library: name, target and "sources <16 hex digits>",
 * the first 16 hex digits of a SHA-256 over the sources it was built from
 * (every .hip and .hpp file under csrc and this header, by name and content, as
 * the package's build script computes it; "unknown" if built without it).
 * Static storage; never NULL. */
const char* ipfb_version(void);

/* Host helper: the sinc x Hamming window of Section 2.2 (Hamming taper with
 * numpy's cos(2 pi m/(M-1)) normalisation, Appendix A):
 *   out[m] = sinc((m - M/2)/lblock) * (0.54 - 0.46 cos(2 pi m/(M-1))),
 * M = ntap*lblock. out is a host array of M doubles. */
int ipfb_window_sinc_hamming(double* out, int ntap, int lblock);

/* Create a plan for frames of lblock samples, ntap taps, nblock frames.
 * window: host, ntap*lblock doubles, copied (the taps of Section 2.3's
 * reshaped [ntap, lblock] window). prec: IPFB_F32 or IPFB_F64.
 * The plan allocates its tables and workspace on the current device. */
int ipfb_plan_create(ipfb_plan* out, int lblock, int ntap, const double* window, int64_t nblock, int prec);
int ipfb_plan_destroy(ipfb_plan plan);
/* Bytes of the plan's workspace: the frame buffers every call uses as
 * scratch (the frame matrix d, its transposed copy where the column length
 * is a power of two, the long-frame intermediate). This is the size
 * ipfb_plan_set_workspace needs. */
int ipfb_plan_workspace_size(ipfb_plan plan, size_t* bytes);
/* Device bytes the plan holds itself: its tables, small buffers, scratch
 * allocated on first use, and its workspace unless the caller provides it. */
int ipfb_plan_device_bytes(ipfb_plan plan, size_t* bytes);
/* Gives the plan a caller-owned workspace (Section 3's inverse needs d and
 * the column-stage intermediate per call; this is where they live).
 * dev: device memory on the plan's device, 256-byte aligned, at least
 * ipfb_plan_workspace_size bytes (bytes: its size). The call waits for the
 * device to finish queued work, releases the plan's own workspace and uses
 * dev in every later call; its contents are scratch, not kept between calls.
 * The caller keeps dev allocated, does not touch it while calls on the plan
 * may run, and frees it only after ipfb_plan_destroy or after giving the plan
 * another workspace. dev = NULL gives the plan a workspace of its own again
 * (if that allocation fails the caller's stays in use). Scratch that some
 * calls allocate on first use (the ML-CG vectors, the diagnostics, the
 * Bluestein path of a non-power-of-two nblock) stays the plan's.
 * Errors: IPFB_EINVAL (too small, misaligned, NULL plan), IPFB_ENOMEM. */
int ipfb_plan_set_workspace(ipfb_plan plan, void* dev, size_t bytes);

/* How ipfb_wiener / ipfb_wiener_ex run the column stage (Section 3.1's
 * per-column circulant inverse with the Section 4.1 Wiener gain):
 * IPFB_COLS_FFT: b-point column FFTs, the FP64 gain, inverse FFTs (the
 *   paper's formulation);
 * IPFB_COLS_RECURSIVE: the same linear map as two recursions along the frames.
 *   The gain W_n (1+phi^2)/(|W_n|^2+phi^2) is a rational function of
 *   e^{-2 pi i f/b}; factoring |W_n|^2 + phi^2 = K Q(z) Q(1/z) with Q's roots
 *   inside the unit circle splits it into a causal filter W_n/Q (forward in
 *   the frame index) and an anti-causal all-pole filter 1/Q(1/z) (backward),
 *   run over the periodic sequence of nblock frames with exact periodic
 *   states (one read of the frames to find them, one to apply), any nblock;
 *   taken where ntap = 4 and phi >= 1e-3, the FFT form otherwise;
 * IPFB_COLS_AUTO (default): the recursive form where it applies, except for
 *   power-of-two nblock <= 512 (whose one-pass FFT stage is cheaper).
 * Both give the same result up to rounding. IPFB_EUNSUPPORTED for
 * IPFB_COLS_RECURSIVE on a plan whose tap count or frame length has no
 * recursive kernel. */
enum { IPFB_COLS_AUTO = 0, IPFB_COLS_FFT = 1, IPFB_COLS_RECURSIVE = 2 };
int ipfb_plan_set_column_method(ipfb_plan plan, int method);

/* Forward PFB (Section 2.2 polyphase equation, Section 2.3 y = F S W x),
 * circular: y_j[k] = sum_n e^{-2 pi i nk/N} sum_r h[rN+n] x[((j+r) mod b)N + n].
 * x: [nblock*lblock] real. y: [nblock][lblock/2+1] complex. */
int pfb_forward(ipfb_plan plan, const void* x, void* y, void* stream);

/* Adjoint of pfb_forward under the real inner product on x and Re<.,.> on
 * the half spectrum (the transpose of S W and of the half-spectrum DFT):
 *   z_j[n] = Re sum_{k=0}^{N/2} y_jk e^{2 pi i nk/N},
 *   x[iN+n] = sum_r h[rN+n] z_{(i-r) mod b}[n].
 * y: [nblock][lblock/2+1] complex, x: [nblock*lblock] real.
 * lblock <= 32768 (F32) / 16384 (F64). */
int pfb_adjoint(ipfb_plan plan, const void* y, void* x, void* stream);

/* Circulant Wiener inverse PFB (Section 3.1 decorrelation equation, Section
 * 4.1 Wiener weights): d_j = inverse real FFT of spectrum j (Section 3), then
 * per column n, x_n = F^dagger[ G_n F d_n ] with
 *   W_n(f) = sum_r h[rN+n] e^{-2 pi i r f / nblock},
 *   G_n = W_n (1+phi^2) / (|W_n|^2 + phi^2).
 * phi = 0 gives the plain division 1/conj(W_n), with eigenvalues at rounding
 * level (|W| <= 1e-12 sum_r |h[rN+n]|) truncated to zero.
 * spec: [nblock][lblock/2+1] in format infmt. chan_scale: device float
 * [lblock/2+1] for IPFB_IN_C4 and IPFB_IN_CI8, ignored (may be NULL) otherwise.
 * x_out: [nblock*lblock] real, time order. The imaginary parts of the DC and
 * Nyquist channels are ignored. The row stage writes the frame matrix into
 * x_out and the column stage transforms it there in place, so x_out must not
 * overlap spec or chan_scale. */
int ipfb_wiener(ipfb_plan plan, int infmt, const void* spec, const float* chan_scale, double phi,
                void* x_out, void* stream);

/* As ipfb_wiener, with normalise = 0 dropping the (1+phi^2) factor (Appendix B
 * calls it optional). */
int ipfb_wiener_ex(ipfb_plan plan, int infmt, const void* spec, const float* chan_scale, double phi,
                   int normalise, void* x_out, void* stream);

/* Other eigenvalue filters (Section 4.1: the circulant form gives the
 * eigenspectrum W_n(f) of every sub-filter, so any filter H_n(f) applies as
 * G = H / conj(W) at no extra cost). As ipfb_wiener_ex, with the gain
 *   IPFB_FILTER_WIENER:    the Wiener filter with phi = param;
 *   IPFB_FILTER_THRESHOLD: H = 1 where |W_n(f)| >= param, else 0 (the
 *                          truncated pseudo-inverse); param > 0;
 *   IPFB_FILTER_NU:        the general Wiener filter S/(S+N) with a
 *                          noise-to-signal ratio per frequency,
 *                          H = |W|^2 (1 + nu_f) / (|W|^2 + nu_f) (the
 *                          (1 + nu_f) factor dropped with normalise = 0);
 *                          nu: device double [nblock/2 + 1], nu_f >= 0 for
 *                          f = 0 .. nblock/2 (nu_{b-f} is taken as nu_f);
 *                          where |W|^2 + nu_f <= (1e-12 sum_r |h[rN+n]|)^2
 *                          (nu_f = 0 at an exact zero of W) the gain is 0,
 *                          the naive inverse's truncation.
 * Power-of-two nblock only (the LDS column path); param is ignored for
 * IPFB_FILTER_NU and nu for the others. */
enum { IPFB_FILTER_WIENER = 0, IPFB_FILTER_THRESHOLD = 1, IPFB_FILTER_NU = 2 };
int ipfb_wiener_filter(ipfb_plan plan, int infmt, const void* spec, const float* chan_scale, int kind, double param,
                       const double* nu, int normalise, void* x_out, void* stream);

/* The comparison solvers of Appendix C (time complexity), beside the
 * circulant inverse.
 * ipfb_tikhonov: per sub-filter path, the Tikhonov-regularised solution of
 * the LINEAR sub-problem d_n = W_n x_n of Section 2.3 (W_n the
 * [nblock - ntap + 1, nblock] Toeplitz matrix of the path's taps, no
 * circulant extension): x_n = c (W_n^T W_n + phi^2 I)^{-1} W_n^T d_n,
 * c = 1 + phi^2 (normalise = 1) or 1, solved by banded Cholesky (bandwidth
 * ntap - 1: O(nblock ntap^2) per path, sequential along the frames, the
 * paths in parallel). spec: [nblock - ntap + 1][lblock/2+1] spectra of a
 * linear (non-wrapping) PFB over nblock frames, in format infmt (chan_scale
 * as for ipfb_wiener); x_out: [nblock * lblock] real, also used to hold the
 * frames first. phi > 0; ntap in {2, 3, 4, 5, 8, 16}. The first call
 * allocates (ntap + 1) * nblock * lblock doubles of workspace.
 * ipfb_fir_kernels: the Wiener decorrelation kernels (the circulant inverse's
 * response to a unit sample at frame 0) truncated to ltaps lags
 * c - T .. c + T, c = ntap / 2 (the window's delay), T = (ltaps - 1)/2,
 * taken modulo nblock: kernels [ltaps][lblock] real (plan precision), on the
 * stream. ltaps odd, 1 <= ltaps <= 255, phi > 0. Needs a plan whose column
 * stage runs in place (power-of-two nblock, or ntap = 4).
 * ipfb_fir: the inverse with each path's decorrelation done by those
 * truncated kernels (FIR filtering, O(nblock ltaps) per path):
 * x_n[j] = sum_t g_n[t] d_n[(j - t) mod nblock]; spec, chan_scale, x_out as
 * for ipfb_wiener. The kernels are made on the first call and again when
 * phi, ltaps or normalise change (the first call allocates them:
 * 255 * lblock reals). */
int ipfb_tikhonov(ipfb_plan plan, int infmt, const void* spec, const float* chan_scale, double phi, int normalise,
                  void* x_out, void* stream);
int ipfb_fir_kernels(ipfb_plan plan, double phi, int ltaps, int normalise, void* kernels, void* stream);
int ipfb_fir(ipfb_plan plan, int infmt, const void* spec, const float* chan_scale, double phi, int ltaps,
             int normalise, void* x_out, void* stream);

/* Linear boundary, streaming (Section 3.1: real data are not circulant; the
 * data are extended to b frames, and the circulant inverse corrupts only the
 * samples within a decorrelation-kernel width of the ends). Input: nspec
 * spectra of a linear (non-wrapping) PFB, spectrum j from frames j..j+p-1,
 * covering nframes = nspec + ntap - 1 frames. The stream is inverted in
 * windows of `chunk` frames (overlap-save): a window holds
 * m = chunk - (ntap - 1) consecutive spectra, zero-extended to chunk frames,
 * and is inverted as ipfb_wiener_ex inverts a circular block; it keeps
 * L = m - 2 halo frames, those at least halo frames from its first frame and
 * from its last spectrum. Window c keeps output frames [c L, min((c+1) L,
 * nframes)) and starts at spectrum max(0, min(c L - halo, nspec - m)),
 * holding min(m, nspec - start) spectra (the stream's ends pull it inwards).
 * With nspec = m the result is the single-window zero-extension inverse.
 * chunk: a power of two in [4, 2^15] (F32) / [4, 2^14] (F64), with
 * chunk - (ntap - 1) - 2 halo >= 1; lblock as for ipfb_wiener's LDS path
 * (<= 2^15 F32 / 2^14 F64). The plan owns one window of chunk * lblock
 * samples and the tables. */
typedef struct ipfb_splan_s* ipfb_splan;
int ipfb_stream_plan_create(ipfb_splan* out, int lblock, int ntap, const double* window, int64_t chunk, int halo,
                            int prec);
int ipfb_stream_plan_destroy(ipfb_splan plan);
/* spec: [nspec][lblock/2+1] in format infmt (chan_scale as for ipfb_wiener);
 * x_out: [(nspec + ntap - 1) * lblock] real, time order, must not overlap spec.
 * normalise as in ipfb_wiener_ex. Asynchronous on stream; windows run one
 * after another on it, so calls on one plan must not overlap. */
int ipfb_wiener_stream(ipfb_splan plan, int infmt, const void* spec, const float* chan_scale, int64_t nspec,
                       double phi, int normalise, void* x_out, void* stream);

/* Up-channelization (Section 4.3): the forward PFB re-applied with the fine
 * plan's longer frame lblock_f (= u * lblock) and its window, circular over
 * nblock_f = S / lblock_f frames.
 * x: [nblock_f*lblock_f] real (the inverse's output). y_fine:
 * [nblock_f][lblock_f/2+1] complex. autospec: NULL, or device double
 * [lblock_f/2+1] receiving A(f) = (1/nblock_f) sum_j |Y_j(f)|^2
 * (Section 4.1's autospectrum), summed in a fixed order. */
int upchannelize(ipfb_plan fine, const void* x, void* y_fine, double* autospec, void* stream);

/* Maximum-likelihood reconstruction with a time-domain prior (Section 4.2,
 * the chi^2 with prior term): minimise |d - A x|^2 + lambda |D (x - prior)|^2
 * where d are the frames after the N-point inverse FFT of spec (Section 4.2:
 * A = S W once F is undone, circular), D = diag(mask), by preconditioned
 * conjugate gradient on (A^T A + lambda D) x = A^T d + lambda D prior
 * (the CG method the paper cites), with the preconditioner
 * F^dagger diag(1/(|W_n|^2 + phi_precond^2)) F per column.
 * spec/chan_scale/infmt as for ipfb_wiener. mask: device bitmask of
 * ceil(S/32) 32-bit words, S = nblock*lblock, in time order: sample
 * e = j*lblock + n is saved when bit (e mod 32) of word e/32 is 1 (least
 * significant bit first; bits past S are ignored). ipfb_mask_pack builds it
 * from one byte per sample.
 * prior: device [S] real (plan precision), read where the mask bit is 1.
 * x_init: NULL to start from the Wiener solution with phi_x0 (the paper's
 * initial guess), else a device [S] real starting point. Runs exactly iters
 * iterations (no early exit; an exactly converged system stops moving).
 * x_out: device [S] real, time order. resid_norms: NULL or device double
 * [iters+1] receiving |r_k|_2 (FP64 sums). Vectors are FP32 for F32 plans,
 * dot products and norms FP64. The first call on a plan allocates the
 * workspace (7 vectors of S reals and the mask bits transposed to the
 * column layout); later calls allocate nothing.
 * Two layouts: for power-of-two nblock <= 2^15 (2^14 in FP64) the vectors
 * are kept transposed and the preconditioner is an in-LDS column FFT; for
 * any other nblock, or when the plan's column method is
 * IPFB_COLS_RECURSIVE, they stay in the natural [nblock][lblock] layout, the
 * stencils run down the columns and the preconditioner is the recursive
 * column stage with numerator 1 (exact, periodic). That form needs ntap = 4,
 * phi_precond >= 1e-3, and phi_x0 >= 1e-3 unless x_init is given
 * (IPFB_EUNSUPPORTED otherwise); it iterates in x_out. */
int ipfb_ml_cg(ipfb_plan plan, int infmt, const void* spec, const float* chan_scale, const uint32_t* mask,
               const void* prior, double lambda, double phi_x0, double phi_precond, int iters,
               const void* x_init, void* x_out, double* resid_norms, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the solve
 * of ipfb_ml_cg, with the same arguments and the same results, whose CG
 * buffers live in a static device array of 64 MiB per device instead of a
 * workspace allocated by the plan. It calls no allocator (the plan, created
 * beforehand, keeps its own tables and frame buffers). The solve must fit the
 * array: 7 vectors of S reals, the mask bits and small tables, i.e. S up to
 * 2^21 samples for F32 plans and 2^20 for F64 plans at power-of-two shapes;
 * larger plans return IPFB_EUNSUPPORTED with the sizes in the message. Every
 * call on one device shares that device's array and leaves its contents
 * behind (nothing in it needs to start at zero: every buffer is written
 * before it is read), so calls that overlap on one device, from other
 * streams or threads, race and must be serialised by the caller. The first
 * call on a device looks up the array's address there (no allocation). */
int ipfb_ml_cg_noalloc(ipfb_plan plan, int infmt, const void* spec, const float* chan_scale, const uint32_t* mask,
                       const void* prior, double lambda, double phi_x0, double phi_precond, int iters,
                       const void* x_init, void* x_out, double* resid_norms, void* stream);

/* Autospectrum alone: autospec[k] = (1/nspec) sum_j |y_jk|^2 (double). */
int ipfb_autospectrum(ipfb_plan plan, const void* y, double* autospec, void* stream);

/* Prior mask of the sample-saving strategy (Section 4.2.2): every R-th
 * sample of the L sub-filter paths around the frame centre, i.e. sample
 * e = j*lblock + n is saved for j = 0 mod R and lblock/2 - L/2 <= n <
 * lblock/2 + L/2; the saved fraction is beta = L/(R lblock) when R divides
 * nblock. mask: device uint32 [ceil(nblock*lblock/32)], ipfb_ml_cg's bitmask
 * layout. L even, 0 <= L <= lblock; R >= 1. */
int ipfb_mask_structured(ipfb_plan plan, int R, int L, uint32_t* mask, void* stream);

/* Packs a byte-per-sample mask (device uint8 [nsamples], nonzero = saved)
 * into ipfb_ml_cg's bitmask (device uint32 [ceil(nsamples/32)]) on the
 * current device. nsamples = 0 enqueues nothing. */
int ipfb_mask_pack(const uint8_t* mask, int64_t nsamples, uint32_t* bits, void* stream);

/* Appendix B diagnostics. delta(f) = <|X(f) - Xhat(f)|^2> / <|X(f)|^2>, the
 * relative error of the power spectrum.
 * ipfb_delta_analytic: the prediction for white input from the plan's window,
 * at sub-stream frequencies f = k / nfreq, k < nfreq (out: device double
 * [nfreq]), with W_n(f) = sum_r h[rN+n] e^{-2 pi i r f}:
 *   phi > 0 (Wiener):  1 - (1/N) sum_n |W_n|^2 / (|W_n|^2 + phi^2)
 *   phi = 0 (naive):   (1/snr) (1/N) sum_n 1 / |W_n|^2   (snr > 0 required).
 * ipfb_autospectrum_error: the measured (Monte-Carlo) delta on the fine plan's
 * channels, delta[k] = sum_j |Y_jk - Yhat_jk|^2 / sum_j |Y_jk|^2 with Y, Yhat
 * the up-channelized spectra (as upchannelize) of x_true and x_hat (device
 * [nblock_f * lblock_f] real each, plan precision; delta: device double
 * [lblock_f/2+1]; a channel with no power in x_true gives 0/0). The plan
 * allocates a workspace of one timestream, one set of spectra and two
 * autospectra on the first call. */
int ipfb_delta_analytic(ipfb_plan plan, int64_t nfreq, double phi, double snr, double* out, void* stream);
int ipfb_autospectrum_error(ipfb_plan fine, const void* x_true, const void* x_hat, double* delta, void* stream);

/* Input synthesis (Section 4.3 quantiser): per-channel scale
 * s_k = float(levels_rms / sigma_k), sigma_k = sqrt(mean_j |y_jk|^2 / 2)
 * (1 for a channel with no power), then q = clip(rint(s_k y), -7, 7) on real
 * and imaginary parts, packed as IPFB_IN_C4. y: the plan's complex spectra
 * [nblock][lblock/2+1]; packed: uint8 [nblock][lblock/2+1]; scales: float
 * [lblock/2+1]. */
int ipfb_quantize_c4(ipfb_plan plan, const void* y, double levels_rms, uint8_t* packed, float* scales,
                     void* stream);

/* Batched form: nstreams independent timestreams sharing lblock, ntap, the
 * window and the precision, each with its own nblock (2 <= nblock <= 32768,
 * any integer). Each stream is inverted exactly as ipfb_wiener does (Section
 * 3.1 with the Section 4.1 gain), circularly over its own nblock frames: the
 * b-point column DFTs of a stream whose nblock is not a power of two use
 * Bluestein's chirp-z identity with FP64-built chirps and filter spectra.
 * window: host, ntap*lblock doubles; nblock: host array [nstreams]; both
 * copied. The plan owns per-length tables and one set of scratch buffers
 * sized for the longest stream (streams run one after another). */
typedef struct ipfb_bplan_s* ipfb_bplan;
int ipfb_batched_plan_create(ipfb_bplan* out, int lblock, int ntap, const double* window, int nstreams,
                             const int64_t* nblock, int prec);
int ipfb_batched_plan_destroy(ipfb_bplan plan);
int ipfb_batched_workspace_size(ipfb_bplan plan, size_t* bytes);
/* on = 1 (default): a call replays one HIP graph holding every stream's
 * launches, captured on the first call and again whenever the pointers, phi,
 * format or normalisation change; on = 0: launch directly on the stream. */
int ipfb_batched_use_graph(ipfb_bplan plan, int on);
/* The column stage of the batched form, as ipfb_plan_set_column_method for
 * one stream: IPFB_COLS_AUTO (default) and IPFB_COLS_RECURSIVE take the
 * recursive stage where it applies (ntap = 4, phi >= 1e-3), then for all
 * streams at once: one kernel for the rows of every stream (4-bit spectra),
 * and one launch per recursive pass over the segments of every stream;
 * IPFB_COLS_FFT keeps the per-stream FFT / Bluestein path. The first call
 * with a new phi sets the coefficients up (outside the graph); a call with
 * other pointers than the last waits for the stream and rewrites the plan's
 * stream tables. IPFB_EUNSUPPORTED for IPFB_COLS_RECURSIVE with ntap != 4. */
int ipfb_batched_set_column_method(ipfb_bplan plan, int method);
/* spec, chan_scale, x_out: host arrays [nstreams] of device pointers with the
 * per-stream layouts of ipfb_wiener (chan_scale ignored for the float formats).
 * normalise as in ipfb_wiener_ex. Asynchronous on stream (NULL = default). */
int ipfb_wiener_batched(ipfb_bplan plan, int infmt, const void* const* spec, const float* const* chan_scale,
                        double phi, int normalise, void* const* x_out, void* stream);

/* Shape of the Bluestein column path for the streams whose convolution length
 * is M = 2^log2m (M the least power of two >= 2 nblock - 1, for nblock not a
 * power of two): shape = {l1, mb, kb, pchunk, fuse, nat}: the four-step
 * split M = 2^l1 * 2^(log2m - l1) (1 <= l1 <= 8, 1 <= log2m - l1 <= 8), the
 * column-tile width mb and the row-tile height kb of the FFT passes (8, 16 or
 * 32), the column pairs per launch group (0: all lblock/2 at once), fuse = 1
 * to run the inverse of the first chirp convolution, the gain and the forward
 * transform of the second as one pass (0: three passes), and nat = 1 for the
 * path that works in place on the frame matrix in its natural layout, in
 * tiles of 128 bytes of column pairs (16 pairs FP32, 8 FP64; no transposes;
 * always fused; mb, kb and fuse unused; pchunk counts tiles per launch
 * group).
 * Every valid shape gives the same result up to rounding; they differ in
 * speed only. Where M1 or M2 is below 32 the tile width 16 is used whatever
 * mb or kb says. The default is {ceil(log2m/2), 16, 16, 0, 1, 0}. get: IPFB_EINVAL if
 * the plan has no stream of that length. set: IPFB_EINVAL for an invalid
 * shape; it waits for the device to go idle (it re-lays the chirp filter
 * spectra for a new split), so it must not overlap a batched call. */
int ipfb_batched_get_shape(ipfb_bplan plan, int log2m, int shape[6]);
int ipfb_batched_set_shape(ipfb_bplan plan, int log2m, const int shape[6]);
/* Autotuner of the batched form: for each convolution length of the plan, a
 * coordinate search (transposed path: (fuse, mb) jointly, then l1, kb,
 * pchunk; natural-layout path: l1, then pchunk) times the column
 * path of the longest stream of that length on the plan's own scratch buffers
 * (three timed runs after a warm-up, best kept) and installs the fastest
 * shape. cache_path (NULL: the IPFB_TUNE_CACHE environment variable; neither:
 * no cache) names a JSON file of shapes keyed by device, precision, lblock,
 * ntap and log2m: entries found there are installed without timing (force = 0)
 * and new results are merged into it. Plan creation installs the cache's
 * matching entries when IPFB_TUNE_CACHE is set. Synchronous; it overwrites
 * the plan's scratch buffers and must not overlap a batched call. */
int ipfb_batched_tune(ipfb_bplan plan, const char* cache_path, int force);

/* Instrumentation: per-kernel timing with HIP events recorded on the
 * launching stream around every kernel group the library enqueues (names:
 * "ipfb_rows", "ipfb_cols_fwd", "ipfb_cols_gain", "ipfb_cols_inv" (the three
 * column passes of ipfb_wiener; one pass, "ipfb_cols_gain", for nblock <= 512),
 * "pfb_fwd", "pfb_fwd_long_p1", "pfb_fwd_long_p2" (the two FFT passes of a
 * long-frame forward PFB), "adj_rows", "adj_gather", "autospec_partial",
 * "autospec_final", "cg_setup", "cg_iter", "cg_out").
 * ipfb_profile_enable(1) starts recording (process-wide); ipfb_profile_query
 * waits for the recorded events and returns the summed milliseconds and
 * launch count for one name; ipfb_profile_reset drops all records. */
int ipfb_profile_enable(int on);
int ipfb_profile_reset(void);
int ipfb_profile_query(const char* name, double* total_ms, int64_t* launches);

#ifdef __cplusplus
}
#endif

#endif /* IPFB_H */
