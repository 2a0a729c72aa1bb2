// C ABI of libipfb: plans, argument validation, and the enqueue of the HIP
// kernels that make up each call. No computation happens on the host besides
// the window helper and the twiddle tables built once per plan.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <complex>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/ipfb.h"
#include "launch.hpp"
#include "tune_cache.hpp"

using namespace ipfb;

namespace {

thread_local std::string g_err;

int fail(int status, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
  return status;
}

int ok() {
  g_err.clear();
  return IPFB_OK;
}

bool is_pow2(int64_t v) { return v > 0 && (v & (v - 1)) == 0; }
int ilog2(int64_t v) {
  int l = 0;
  while ((int64_t(1) << l) < v) ++l;
  return l;
}

// Fault injection for tests of the error paths: IPFB_FAULT_INJECT=alloc makes
// device allocations fail, =launch makes kernel enqueues report an error.
bool inject(const char* what) {
  const char* v = getenv("IPFB_FAULT_INJECT");
  return v && strcmp(v, what) == 0;
}

// e^{-2 pi i m / L}, m < L, in double, exact at multiples of L/4.
std::vector<double> twiddles(int64_t L) {
  std::vector<double> t(2 * L);
  for (int64_t m = 0; m < L; ++m) {
    double c, s;
    if ((4 * m) % L == 0) {
      const int q = (int)((4 * m) / L);
      const double cs[4] = {1.0, 0.0, -1.0, 0.0};
      const double sn[4] = {0.0, 1.0, 0.0, -1.0};
      c = cs[q];
      s = sn[q];
    } else {
      const long double a = 2.0L * 3.14159265358979323846264338327950288L * (long double)m / (long double)L;
      c = (double)cosl(a);
      s = (double)sinl(a);
    }
    t[2 * m] = c;
    t[2 * m + 1] = -s;
  }
  return t;
}

}  // namespace

struct ipfb_plan_s {
  int lblock = 0, ntap = 0, prec = 0, log2n = 0, log2b = -1;
  int64_t nblock = 0;
  int dev = 0;
  bool row_lds = false;  // frame fits the LDS-resident row kernels
  bool col_lds = false;  // nblock is a supported column length
  double* win64 = nullptr;
  void* winT = nullptr;
  void* twN = nullptr;
  void* twB = nullptr;
  void* twS = nullptr;   // long frames: small tables for the two passes
  double* twB64 = nullptr;
  void* work = nullptr;  // d (inverse) or z (adjoint): nblock*lblock reals
  void* work2 = nullptr; // transposed frame matrix for the column stage
  void* tmp = nullptr;   // four-step intermediate of long frames: nblock*lblock/2 complex
  double* part = nullptr;
  void* fac = nullptr;   // per-channel dequantisation factors 1/(s_k N)
  // maximum-likelihood CG workspace (allocated on first use): 7 vectors in the
  // transposed layout, the mask bits, the column autocorrelations, partial
  // sums, scalars
  void* cg = nullptr;
  // nblock not a power of two: a one-stream batched plan runs the Bluestein column path
  ipfb_bplan_s* blu1 = nullptr;
  int jchunk = 1, nchunks = 1;
  int fchunk = 1, nfchunks = 1;  // long frames: frames per power-sum chunk
  // Appendix B diagnostics (allocated on first use): x_true - x_hat, the
  // spectra of either, and the two autospectra
  void* diag = nullptr;
  // recursive column stage: per-column coefficients for the phi last set up
  // (NaN: none yet) and the per-segment states
  double* iir_coef = nullptr;
  double* iir_scoef = nullptr;
  void* iir_zs = nullptr;
  double iir_phi = NAN;
  // the same for the ML-CG preconditioner 1/(|W|^2 + phi^2) (natural layout)
  double* iir_coef_pc = nullptr;
  double* iir_scoef_pc = nullptr;
  double iir_phi_pc = NAN;
  int col_method = IPFB_COLS_AUTO;
  // Appendix C's comparison solvers (allocated on first use): the banded
  // Cholesky workspace, and the truncated decorrelation kernels with the
  // (phi, taps, normalisation) they were made for
  double* tik_ws = nullptr;
  void* fir_g = nullptr;
  double fir_phi = NAN;
  int fir_taps = 0, fir_norm = -1;
  size_t bytes = 0;
  bool ws_ext = false;  // work, work2, tmp point into a caller-owned workspace
};

namespace {

size_t esize(int prec) { return prec == IPFB_F32 ? sizeof(float) : sizeof(double); }

// Input spectrum formats; the quantised ones carry per-channel scales.
bool scaled_infmt(int f) { return f == IPFB_IN_C4 || f == IPFB_IN_CI8; }
size_t infmt_bytes(int f) { return f == IPFB_IN_C4 ? 1 : f == IPFB_IN_CI8 ? 2 : f == IPFB_IN_CF32 ? 8 : 16; }
int check_infmt(int infmt, const void* chan_scale) {
  if (infmt != IPFB_IN_C4 && infmt != IPFB_IN_CI8 && infmt != IPFB_IN_CF32 && infmt != IPFB_IN_CF64)
    return fail(IPFB_EINVAL, "unknown input format %d", infmt);
  if (scaled_infmt(infmt) && !chan_scale)
    return fail(IPFB_EINVAL, "chan_scale is required for the quantised formats (IPFB_IN_C4, IPFB_IN_CI8)");
  return IPFB_OK;
}

int dev_alloc(ipfb_plan p, void** ptr, size_t bytes) {
  if (bytes == 0) bytes = 16;
  if (inject("alloc")) return fail(IPFB_ENOMEM, "device allocation of %zu bytes failed (injected)", bytes);
  hipError_t e = hipMalloc(ptr, bytes);
  if (e != hipSuccess) {
    *ptr = nullptr;
    hipGetLastError();
    return fail(e == hipErrorOutOfMemory ? IPFB_ENOMEM : IPFB_EHIP, "hipMalloc(%zu): %s", bytes,
                hipGetErrorString(e));
  }
  p->bytes += bytes;
  return IPFB_OK;
}

int upload(void* dst, const void* src, size_t bytes) {
  hipError_t e = hipMemcpy(dst, src, bytes, hipMemcpyHostToDevice);
  if (e != hipSuccess) return fail(IPFB_EHIP, "hipMemcpy: %s", hipGetErrorString(e));
  return IPFB_OK;
}

int upload_table(ipfb_plan p, const std::vector<double>& t, int prec, void** dst) {
  const size_t n = t.size();
  int st = dev_alloc(p, dst, n * esize(prec));
  if (st) return st;
  if (prec == IPFB_F64) return upload(*dst, t.data(), n * sizeof(double));
  std::vector<float> f(n);
  for (size_t i = 0; i < n; ++i) f[i] = (float)t[i];
  return upload(*dst, f.data(), n * sizeof(float));
}

void free_bplan(ipfb_bplan p);

void free_plan(ipfb_plan p) {
  if (p->blu1) free_bplan(p->blu1);
  void* ptrs[] = {p->win64, p->winT, p->twN, p->twB, p->twB64, p->part, p->fac, p->twS,
                  p->cg, p->diag, p->iir_coef, p->iir_scoef, p->iir_zs, p->iir_coef_pc, p->iir_scoef_pc,
                  p->tik_ws, p->fir_g};
  for (void* q : ptrs)
    if (q) hipFree(q);
  if (!p->ws_ext) {
    void* ws[] = {p->work, p->work2, p->tmp};
    for (void* q : ws)
      if (q) hipFree(q);
  }
  delete p;
}

// The workspace a caller may provide: the plan's per-call frame buffers d
// (work), its transposed copy (work2) and the long-frame intermediate (tmp),
// each present or not with the plan's shape, at 256-byte-aligned offsets.
// Returns the total; o_* receive the offsets (SIZE_MAX where absent).
size_t ws_layout(ipfb_plan p, size_t* o_work, size_t* o_work2, size_t* o_tmp) {
  const size_t fb = ((size_t)p->nblock * p->lblock * esize(p->prec) + 255) & ~size_t(255);
  size_t off = 0;
  auto take = [&](bool need, size_t* o) {
    *o = need ? off : SIZE_MAX;
    if (need) off += fb;
  };
  take(p->row_lds, o_work);
  take(p->row_lds && p->col_lds, o_work2);
  take(!p->row_lds, o_tmp);
  return off;
}

struct DeviceGuard {
  int prev = -1;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) == hipSuccess && prev != dev) hipSetDevice(dev);
    else prev = -1;
  }
  ~DeviceGuard() {
    if (prev >= 0) hipSetDevice(prev);
  }
};

int launched(hipError_t e, const char* what) {
  if (inject("launch")) e = hipErrorLaunchFailure;
  if (e != hipSuccess) {
    hipGetLastError();
    return fail(IPFB_EHIP, "%s: %s", what, hipGetErrorString(e));
  }
  return ok();
}

// ---- per-kernel timing with HIP events on the launching stream ---------------
struct ProfRec {
  const char* name;
  hipEvent_t a, b;
};
std::mutex g_pm;
bool g_prof = false;
std::vector<ProfRec> g_recs;
std::vector<hipEvent_t> g_pool;

hipEvent_t ev_get() {
  std::lock_guard<std::mutex> lk(g_pm);
  if (!g_pool.empty()) {
    hipEvent_t e = g_pool.back();
    g_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  // timing-only events: no system-scope fence when recorded, so recording
  // them forces no cache write-back between the kernels they bracket
  if (hipEventCreateWithFlags(&e, hipEventDisableSystemFence) != hipSuccess) {
    hipGetLastError();
    return nullptr;
  }
  return e;
}

struct ProfScope {
  const char* name;
  hipStream_t st;
  hipEvent_t a = nullptr;
  ProfScope(const char* n, hipStream_t s) : name(n), st(s) {
    bool on;
    {
      std::lock_guard<std::mutex> lk(g_pm);
      on = g_prof;
    }
    if (n && on && (a = ev_get())) hipEventRecord(a, st);
  }
  ~ProfScope() {
    if (!a) return;
    hipEvent_t b = ev_get();
    if (!b) return;
    hipEventRecord(b, st);
    std::lock_guard<std::mutex> lk(g_pm);
    g_recs.push_back({name, a, b});
  }
};

int max_log2_row(int prec) { return prec == IPFB_F32 ? kMaxLog2RowF32 : kMaxLog2RowF64; }
int max_log2_col(int prec) { return prec == IPFB_F32 ? kMaxLog2ColF32 : kMaxLog2ColF64; }

int check_plan(ipfb_plan p) {
  if (!p) return fail(IPFB_EINVAL, "plan is NULL");
  return IPFB_OK;
}

}  // namespace

extern "C" {

const char* ipfb_last_error(void) { return g_err.c_str(); }

#ifndef IPFB_SOURCE_DIGEST
#define IPFB_SOURCE_DIGEST "unknown"
#endif
const char* ipfb_version(void) { return "ipfb-mi355x 0.1 (gfx950) sources " IPFB_SOURCE_DIGEST; }

int ipfb_window_sinc_hamming(double* out, int ntap, int lblock) {
  if (!out) return fail(IPFB_EINVAL, "window output is NULL");
  if (ntap < 1 || lblock < 1) return fail(IPFB_EINVAL, "ntap and lblock must be >= 1");
  const int64_t M = (int64_t)ntap * lblock;
  const long double pi = 3.14159265358979323846264338327950288L;
  for (int64_t m = 0; m < M; ++m) {
    const long double t = ((long double)m - (long double)M / 2.0L) / (long double)lblock;
    const long double sinc = (t == 0.0L) ? 1.0L : sinl(pi * t) / (pi * t);
    const long double taper = (M > 1) ? 0.54L - 0.46L * cosl(2.0L * pi * (long double)m / (long double)(M - 1)) : 1.0L;
    out[m] = (double)(sinc * taper);
  }
  return ok();
}

int ipfb_plan_create(ipfb_plan* out, int lblock, int ntap, const double* window, int64_t nblock, int prec) {
  if (!out) return fail(IPFB_EINVAL, "plan output pointer is NULL");
  *out = nullptr;
  if (!window) return fail(IPFB_EINVAL, "window is NULL");
  if (prec != IPFB_F32 && prec != IPFB_F64) return fail(IPFB_EINVAL, "prec must be IPFB_F32 or IPFB_F64");
  if (!is_pow2(lblock) || lblock < 4) return fail(IPFB_EINVAL, "lblock must be a power of two >= 4 (got %d)", lblock);
  if (lblock > (1 << 20)) return fail(IPFB_EUNSUPPORTED, "lblock > 2^20 is not supported");
  if (ntap < 1) return fail(IPFB_EINVAL, "ntap must be >= 1 (got %d)", ntap);
  if (nblock < 1) return fail(IPFB_EINVAL, "nblock must be >= 1");
  if (nblock > (int64_t(1) << 31) / 1) return fail(IPFB_EUNSUPPORTED, "nblock too large");
  if ((int64_t)lblock * nblock > (int64_t(1) << 40)) return fail(IPFB_EUNSUPPORTED, "timestream too long");

  ipfb_plan p = new ipfb_plan_s();
  p->lblock = lblock;
  p->ntap = ntap;
  p->prec = prec;
  p->nblock = nblock;
  p->log2n = ilog2(lblock);
  p->row_lds = p->log2n <= max_log2_row(prec);
  if (is_pow2(nblock) && nblock >= 4 && ilog2(nblock) <= max_log2_col(prec)) {
    p->col_lds = true;
    p->log2b = ilog2(nblock);
  }
  if (hipGetDevice(&p->dev) != hipSuccess) {
    hipGetLastError();
    delete p;
    return fail(IPFB_EHIP, "no HIP device available");
  }
  const int64_t M = (int64_t)ntap * lblock;
  int st = dev_alloc(p, (void**)&p->win64, M * sizeof(double));
  if (!st) st = upload(p->win64, window, M * sizeof(double));
  if (!st) st = dev_alloc(p, &p->winT, M * esize(prec));
  if (!st) {
    if (prec == IPFB_F64) st = upload(p->winT, window, M * sizeof(double));
    else {
      std::vector<float> w(M);
      for (int64_t i = 0; i < M; ++i) w[i] = (float)window[i];
      st = upload(p->winT, w.data(), M * sizeof(float));
    }
  }
  if (!st) st = upload_table(p, twiddles(lblock), prec, &p->twN);
  if (!st && p->col_lds) {
    std::vector<double> tb = twiddles(nblock);
    st = upload_table(p, tb, prec, &p->twB);
    if (!st) st = upload_table(p, tb, IPFB_F64, (void**)&p->twB64);
  }
  const size_t frames_bytes = (size_t)nblock * lblock * esize(prec);
  if (!st && p->row_lds) st = dev_alloc(p, &p->work, frames_bytes);
  if (!st && p->row_lds && p->col_lds) st = dev_alloc(p, &p->work2, frames_bytes);
  if (!st && p->row_lds) st = dev_alloc(p, &p->fac, (size_t)(lblock / 2 + 1) * esize(prec));
  const int iseg = prec == IPFB_F32 ? kIirSegF32 : kIirSegF64;
  const int64_t nseg = (nblock + iseg - 1) / iseg;
  if (!st && p->row_lds && iir_coef_stride(ntap) > 0) {  // the recursive column stage's buffers
    st = dev_alloc(p, (void**)&p->iir_coef, (size_t)lblock * iir_coef_stride(ntap) * sizeof(double));
    if (!st) st = dev_alloc(p, (void**)&p->iir_scoef, (size_t)lblock * iir_stream_stride(ntap) * sizeof(double));
    if (!st) st = dev_alloc(p, &p->iir_zs, (size_t)nseg * lblock * 2 * (ntap - 1) * esize(prec));
    if (!st) st = dev_alloc(p, (void**)&p->iir_coef_pc, (size_t)lblock * iir_coef_stride(ntap) * sizeof(double));
    if (!st) st = dev_alloc(p, (void**)&p->iir_scoef_pc, (size_t)lblock * iir_stream_stride(ntap) * sizeof(double));
  }
  if (!st && !p->row_lds) st = dev_alloc(p, &p->tmp, (size_t)nblock * lblock * esize(prec));
  if (!st && !p->row_lds) {
    // long frames: M = lblock/2-point complex FFTs, M = P1 * P2
    const int log2m = p->log2n - 1;
    const int64_t M = int64_t(1) << log2m;
    const int l2 = lf_log2p2(prec == IPFB_F32 ? F32 : F64, log2m);
    const int64_t P1 = int64_t(1) << (log2m - l2), P2 = int64_t(1) << l2;
    std::vector<double> t1 = twiddles(P1), t2 = twiddles(P2), tm = twiddles(M), tl = twiddles(lblock);
    std::vector<double> all;
    all.insert(all.end(), t1.begin(), t1.end());
    all.insert(all.end(), t2.begin(), t2.end());
    all.insert(all.end(), tm.begin(), tm.begin() + 2 * 512);  // e^{-2 pi i m/M}, m < 512
    for (int64_t m = 0; m < M / 512; ++m) {                    // e^{-2 pi i 512 m/M}
      all.push_back(tm[2 * (512 * m)]);
      all.push_back(tm[2 * (512 * m) + 1]);
    }
    all.insert(all.end(), tl.begin(), tl.begin() + 2 * 512);  // e^{-2 pi i k/L}, k < 512
    for (int64_t m = 0; m <= M / 512; ++m) {                   // e^{-2 pi i 512 m/L}, 512 m <= M
      all.push_back(tl[2 * (512 * m)]);
      all.push_back(tl[2 * (512 * m) + 1]);
    }
    st = upload_table(p, all, prec, &p->twS);
  }
  if (!st) {
    // deterministic two-stage power sums: at most 16 chunks of spectra
    p->nchunks = (int)(nblock < 16 ? nblock : 16);
    p->jchunk = (int)((nblock + p->nchunks - 1) / p->nchunks);
    p->nchunks = (int)((nblock + p->jchunk - 1) / p->jchunk);
    // long frames: the second FFT pass sums |Y|^2 over chunks of frames
    p->fchunk = p->row_lds ? 1 : lf_frame_chunk(prec, p->log2n, nblock);
    p->nfchunks = (int)((nblock + p->fchunk - 1) / p->fchunk);
    const int nrows = p->nchunks > p->nfchunks ? p->nchunks : p->nfchunks;
    st = dev_alloc(p, (void**)&p->part, (size_t)nrows * (lblock / 2 + 1) * sizeof(double));
  }
  if (st) {
    std::string keep = g_err;
    free_plan(p);
    g_err = keep;
    return st;
  }
  *out = p;
  return ok();
}

int ipfb_plan_destroy(ipfb_plan plan) {
  if (!plan) return fail(IPFB_EINVAL, "plan is NULL");
  DeviceGuard g(plan->dev);
  free_plan(plan);
  return ok();
}

int ipfb_plan_workspace_size(ipfb_plan plan, size_t* bytes) {
  if (check_plan(plan)) return IPFB_EINVAL;
  if (!bytes) return fail(IPFB_EINVAL, "bytes is NULL");
  size_t a, b, c;
  *bytes = ws_layout(plan, &a, &b, &c);
  return ok();
}

int ipfb_plan_device_bytes(ipfb_plan plan, size_t* bytes) {
  if (check_plan(plan)) return IPFB_EINVAL;
  if (!bytes) return fail(IPFB_EINVAL, "bytes is NULL");
  *bytes = plan->bytes;
  return ok();
}

int ipfb_plan_set_column_method(ipfb_plan p, int method) {
  if (check_plan(p)) return IPFB_EINVAL;
  if (method != IPFB_COLS_AUTO && method != IPFB_COLS_FFT && method != IPFB_COLS_RECURSIVE)
    return fail(IPFB_EINVAL, "unknown column method %d", method);
  if (method == IPFB_COLS_RECURSIVE && !p->iir_coef)
    return fail(IPFB_EUNSUPPORTED, "the recursive column stage needs ntap = 4 and lblock <= 2^%d (ntap %d)",
                max_log2_row(p->prec), p->ntap);
  p->col_method = method;
  return ok();
}

int ipfb_plan_set_workspace(ipfb_plan p, void* dev, size_t bytes) {
  if (check_plan(p)) return IPFB_EINVAL;
  size_t ow, ow2, ot;
  const size_t need = ws_layout(p, &ow, &ow2, &ot);
  if (dev && bytes < need)
    return fail(IPFB_EINVAL, "workspace of %zu bytes is smaller than the %zu bytes the plan needs", bytes, need);
  if (dev && ((uintptr_t)dev & 255)) return fail(IPFB_EINVAL, "workspace must be 256-byte aligned");
  if (!dev && !p->ws_ext) return ok();  // the plan already owns its workspace
  DeviceGuard g(p->dev);
  void** bufs[3] = {&p->work, &p->work2, &p->tmp};
  const size_t offs[3] = {ow, ow2, ot};
  const size_t fbytes = (size_t)p->nblock * p->lblock * esize(p->prec);
  void* next[3] = {nullptr, nullptr, nullptr};
  if (dev) {
    for (int i = 0; i < 3; ++i)
      if (offs[i] != SIZE_MAX) next[i] = (char*)dev + offs[i];
  } else {
    // back to a workspace of the plan's own: allocate it before letting the
    // caller's go, so that a failure leaves the plan as it was
    for (int i = 0; i < 3; ++i) {
      if (offs[i] == SIZE_MAX) continue;
      const int st = dev_alloc(p, &next[i], fbytes);
      if (st) {
        for (int k = 0; k < i; ++k)
          if (next[k]) {
            hipFree(next[k]);
            p->bytes -= fbytes;
          }
        return st;
      }
    }
  }
  // calls already queued may still use the current workspace
  hipError_t e = hipDeviceSynchronize();
  if (e != hipSuccess) return fail(IPFB_EHIP, "hipDeviceSynchronize: %s", hipGetErrorString(e));
  if (!p->ws_ext) {
    for (void** b : bufs)
      if (*b) {
        hipFree(*b);
        p->bytes -= fbytes;
      }
  }
  for (int i = 0; i < 3; ++i) *bufs[i] = next[i];
  p->ws_ext = dev != nullptr;
  return ok();
}

int pfb_forward(ipfb_plan p, const void* x, void* y, void* stream) {
  if (check_plan(p)) return IPFB_EINVAL;
  if (!x || !y) return fail(IPFB_EINVAL, "x and y must be non-NULL device pointers");
  DeviceGuard g(p->dev);
  hipStream_t st = (hipStream_t)stream;
  hipError_t e;
  if (p->row_lds) {
    ProfScope ps("pfb_fwd", st);
    e = launch_pfb_fwd_small(p->prec, p->log2n, x, y, p->nblock, p->ntap, p->winT, p->twN, st);
  } else {
    static const char* const names[2] = {"pfb_fwd_long_p1", "pfb_fwd_long_p2"};
    e = hipSuccess;
    for (int pass = 0; pass < 2 && e == hipSuccess; ++pass) {
      ProfScope ps(names[pass], st);
      e = launch_pfb_fwd_long(p->prec, p->log2n, pass, x, y, p->nblock, p->ntap, p->winT, p->twS, p->tmp,
                              p->fchunk, nullptr, st);
    }
  }
  return launched(e, "pfb_forward");
}

int pfb_adjoint(ipfb_plan p, const void* y, void* x, void* stream) {
  if (check_plan(p)) return IPFB_EINVAL;
  if (!x || !y) return fail(IPFB_EINVAL, "x and y must be non-NULL device pointers");
  if (!p->row_lds) return fail(IPFB_EUNSUPPORTED, "pfb_adjoint supports lblock <= 2^%d", max_log2_row(p->prec));
  DeviceGuard g(p->dev);
  hipStream_t st = (hipStream_t)stream;
  hipError_t e;
  {
    ProfScope ps("adj_rows", st);
    e = launch_row_irfft(p->prec, p->log2n, IN_ADJ, y, nullptr, p->work, p->nblock, p->twN, st);
  }
  if (e == hipSuccess) {
    ProfScope ps("adj_gather", st);
    e = launch_adjoint_gather(p->prec, p->work, x, p->nblock, p->lblock, p->ntap, p->winT, st);
  }
  return launched(e, "pfb_adjoint");
}

}  // extern "C"

namespace {

// Row stage into x_out: d [b][N].
hipError_t rows_into(ipfb_plan p, int infmt, const void* spec, const float* chan_scale, void* x_out,
                     hipStream_t st) {
  ProfScope ps("ipfb_rows", st);
  hipError_t e = hipErrorNotSupported;
  if (infmt == IPFB_IN_C4) e = launch_row_c4(p->prec, p->log2n, spec, chan_scale, x_out, p->nblock, p->twN, st);
  if (e == hipErrorNotSupported) {
    hipGetLastError();
    if (scaled_infmt(infmt)) e = launch_dequant_factors(p->prec, chan_scale, p->lblock / 2 + 1, p->lblock, p->fac, st);
    else e = hipSuccess;
    if (e == hipSuccess) e = launch_row_irfft(p->prec, p->log2n, infmt, spec, p->fac, x_out, p->nblock, p->twN, st);
  }
  return e;
}

// Row stage into x_out, then the column stage in place there (power-of-two
// nblock); kind/param/nu select the eigenvalue filter of the gain pass.
int wiener_lds(ipfb_plan p, int infmt, const void* spec, const float* chan_scale, int kind, double param,
               const double* nu, int normalise, void* x_out, void* stream) {
  DeviceGuard g(p->dev);
  hipStream_t st = (hipStream_t)stream;
  hipError_t e = rows_into(p, infmt, spec, chan_scale, x_out, st);
  // column stage in place on x_out: d [b][N] -> x [b][N]
  static const char* const pass_names[3] = {"ipfb_cols_fwd", "ipfb_cols_gain", "ipfb_cols_inv"};
  for (int pass = 0; pass < 3 && e == hipSuccess; ++pass) {
    if (p->log2b <= 9 && pass != 1) continue;  // one pass does the whole stage
    ProfScope ps(pass_names[pass], st);
    e = launch_col_wiener_nat(p->prec, p->log2b, pass, x_out, p->lblock, p->ntap, p->win64, param, normalise, p->twB,
                              p->twB64, st, 0, -1, nullptr, 0, 0, kind, nu);
  }
  return launched(e, "ipfb_wiener");
}

// Whether the Wiener inverse with this phi takes the recursive column stage.
// It needs a tap count with a kernel and phi >= kIirMinPhi (poles of the
// factorisation comfortably inside the unit circle); by default it is taken
// for every nblock except the powers of two up to 512, whose one-pass FFT
// stage reads and writes the frames once.
constexpr double kIirMinPhi = 1e-3;
bool use_recursive(ipfb_plan p, double phi) {
  if (!p->iir_coef || !(phi >= kIirMinPhi) || p->col_method == IPFB_COLS_FFT) return false;
  if (p->col_method == IPFB_COLS_RECURSIVE) return true;
  return !(p->col_lds && p->log2b <= 9);
}

// The recursive column stage in place on buf [b][N]: the Wiener filter
// (precond = 0: coefficient set iir_coef, output scaled by gnorm) or the CG
// preconditioner 1/(|W|^2 + phi^2) (precond = 1: set iir_coef_pc, gnorm 1).
// Each set is made again only when phi changes. names: NULL, or the profile
// names of the five stages. dst: NULL, or where frames [doff, doff + dkeep)
// of the result go (buf then keeps its input).
hipError_t rec_stage(ipfb_plan p, void* buf, double phi, int precond, double gnorm, hipStream_t st,
                     const char* const* names, void* dst = nullptr, int64_t doff = 0, int64_t dkeep = 0) {
  const int seg = p->prec == IPFB_F32 ? kIirSegF32 : kIirSegF64;
  const int64_t nseg = (p->nblock + seg - 1) / seg;
  const IirStream one = {buf, p->nblock, 0};
  double* coef = precond ? p->iir_coef_pc : p->iir_coef;
  double* scoef = precond ? p->iir_scoef_pc : p->iir_scoef;
  double& cached = precond ? p->iir_phi_pc : p->iir_phi;
  hipError_t e = hipSuccess;
  for (int stage = (phi == cached) ? kIirPass1 : kIirSetup; stage <= kIirApply && e == hipSuccess; ++stage) {
    ProfScope ps(names ? names[stage] : nullptr, st);
    e = launch_col_iir(stage, p->prec, one, nullptr, 1, nseg, nseg, p->lblock, p->ntap, p->win64, phi, gnorm, coef,
                       scoef, p->iir_zs, st, precond, dst, doff, dkeep);
    if (stage <= kIirSetupLen) cached = e == hipSuccess ? phi : NAN;
  }
  return e;
}

int wiener_recursive(ipfb_plan p, int infmt, const void* spec, const float* chan_scale, double phi, int normalise,
                     void* x_out, void* stream) {
  DeviceGuard g(p->dev);
  hipStream_t st = (hipStream_t)stream;
  hipError_t e = rows_into(p, infmt, spec, chan_scale, x_out, st);
  static const char* const names[5] = {"ipfb_cols_rec_setup", "ipfb_cols_rec_setup", "ipfb_cols_rec_pass1",
                                       "ipfb_cols_rec_carry", "ipfb_cols_rec_pass2"};
  if (e == hipSuccess) e = rec_stage(p, x_out, phi, 0, normalise ? 1.0 + phi * phi : 1.0, st, names);
  return launched(e, "ipfb_wiener");
}

}  // namespace

extern "C" {

int ipfb_wiener_ex(ipfb_plan p, int infmt, const void* spec, const float* chan_scale, double phi, int normalise,
                   void* x_out, void* stream) {
  if (check_plan(p)) return IPFB_EINVAL;
  if (!spec || !x_out) return fail(IPFB_EINVAL, "spec and x_out must be non-NULL device pointers");
  if (check_infmt(infmt, chan_scale)) return IPFB_EINVAL;
  if (!(phi >= 0.0) || !std::isfinite(phi)) return fail(IPFB_EINVAL, "phi must be finite and >= 0");
  if (!p->row_lds)
    return fail(IPFB_EUNSUPPORTED, "ipfb_wiener supports lblock <= 2^%d for this precision", max_log2_row(p->prec));
  if (use_recursive(p, phi)) return wiener_recursive(p, infmt, spec, chan_scale, phi, normalise, x_out, stream);
  if (!p->col_lds) {
    if (p->nblock < 2 || p->nblock > 32768)
      return fail(IPFB_EUNSUPPORTED, "ipfb_wiener supports nblock in [2, 32768] (got %lld)", (long long)p->nblock);
    DeviceGuard g(p->dev);
    if (!p->blu1) {  // built on the first call: Bluestein tables for this nblock
      std::vector<double> w((size_t)p->ntap * p->lblock);
      if (hipMemcpy(w.data(), p->win64, w.size() * sizeof(double), hipMemcpyDeviceToHost) != hipSuccess) {
        hipGetLastError();
        return fail(IPFB_EHIP, "reading back the window failed");
      }
      int s2 = ipfb_batched_plan_create(&p->blu1, p->lblock, p->ntap, w.data(), 1, &p->nblock, p->prec);
      if (s2) return s2;
      ipfb_batched_use_graph(p->blu1, 0);
      // the FFT form (this path is taken only when the recursive one is not)
      s2 = ipfb_batched_set_column_method(p->blu1, IPFB_COLS_FFT);
      if (s2) return s2;
    }
    const void* sp[1] = {spec};
    const float* scs[1] = {chan_scale};
    void* xo[1] = {x_out};
    return ipfb_wiener_batched(p->blu1, infmt, sp, chan_scale ? scs : nullptr, phi, normalise, xo, stream);
  }
  return wiener_lds(p, infmt, spec, chan_scale, 0, phi, nullptr, normalise, x_out, stream);
}

int ipfb_wiener_filter(ipfb_plan p, int infmt, const void* spec, const float* chan_scale, int kind, double param,
                       const double* nu, int normalise, void* x_out, void* stream) {
  if (check_plan(p)) return IPFB_EINVAL;
  if (!spec || !x_out) return fail(IPFB_EINVAL, "spec and x_out must be non-NULL device pointers");
  if (check_infmt(infmt, chan_scale)) return IPFB_EINVAL;
  if (kind != IPFB_FILTER_WIENER && kind != IPFB_FILTER_THRESHOLD && kind != IPFB_FILTER_NU)
    return fail(IPFB_EINVAL, "unknown filter kind %d", kind);
  if (kind == IPFB_FILTER_WIENER && (!(param >= 0.0) || !std::isfinite(param)))
    return fail(IPFB_EINVAL, "param (phi) must be finite and >= 0");
  if (kind == IPFB_FILTER_THRESHOLD && (!(param > 0.0) || !std::isfinite(param)))
    return fail(IPFB_EINVAL, "param (the threshold) must be finite and > 0: a zero threshold keeps the zero "
                             "eigenvalues");
  if (kind == IPFB_FILTER_NU && !nu) return fail(IPFB_EINVAL, "the noise-to-signal filter needs nu");
  if (!p->row_lds || !p->col_lds)
    return fail(IPFB_EUNSUPPORTED, "ipfb_wiener_filter needs a power-of-two nblock <= 2^%d and lblock <= 2^%d",
                max_log2_col(p->prec), max_log2_row(p->prec));
  return wiener_lds(p, infmt, spec, chan_scale, kind, param, nu, normalise, x_out, stream);
}

int ipfb_wiener(ipfb_plan p, int infmt, const void* spec, const float* chan_scale, double phi, void* x_out,
                void* stream) {
  return ipfb_wiener_ex(p, infmt, spec, chan_scale, phi, 1, x_out, stream);
}

// ---- Appendix C's comparison solvers ---------------------------------------
namespace {

// The column stage alone, in place on the frame matrix buf [b][N]:
// the recursive form where it applies, else the FFT form (power-of-two b).
hipError_t cols_into(ipfb_plan p, void* buf, double phi, int normalise, hipStream_t st) {
  hipError_t e = hipSuccess;
  if (use_recursive(p, phi)) return rec_stage(p, buf, phi, 0, normalise ? 1.0 + phi * phi : 1.0, st, nullptr);
  for (int pass = 0; pass < 3 && e == hipSuccess; ++pass) {
    if (p->log2b <= 9 && pass != 1) continue;
    e = launch_col_wiener_nat(p->prec, p->log2b, pass, buf, p->lblock, p->ntap, p->win64, phi, normalise, p->twB,
                              p->twB64, st, 0, -1, nullptr, 0, 0, 0, nullptr);
  }
  return e;
}

int fir_check(ipfb_plan p, double phi, int ltaps) {
  if (check_plan(p)) return IPFB_EINVAL;
  if (!(phi > 0.0) || !std::isfinite(phi)) return fail(IPFB_EINVAL, "phi must be finite and > 0");
  if (ltaps < 1 || !(ltaps & 1) || ltaps > kFirMaxTaps)
    return fail(IPFB_EINVAL, "ltaps must be odd and in [1, %d] (got %d)", kFirMaxTaps, ltaps);
  if (!p->row_lds || !(use_recursive(p, phi) || p->col_lds))
    return fail(IPFB_EUNSUPPORTED, "the decorrelation kernels need a plan whose column stage runs in place (a "
                                   "power-of-two nblock, or 4 taps)");
  return IPFB_OK;
}

// The truncated kernels into g [ltaps][N] (the column stage applied to a unit
// sample, through the plan's frame buffer).
hipError_t fir_kernels_into(ipfb_plan p, double phi, int ltaps, int normalise, void* g, hipStream_t st) {
  const int64_t c0 = p->ntap / 2 - (ltaps - 1) / 2;
  hipError_t e = launch_fir_setup(p->prec, 0, p->work, nullptr, p->lblock, p->nblock, ltaps, c0, st);
  if (e == hipSuccess) e = cols_into(p, p->work, phi, normalise, st);
  if (e == hipSuccess) e = launch_fir_setup(p->prec, 1, p->work, g, p->lblock, p->nblock, ltaps, c0, st);
  return e;
}

}  // namespace

extern "C" {

int ipfb_tikhonov(ipfb_plan p, int infmt, const void* spec, const float* chan_scale, double phi, int normalise,
                  void* x_out, void* stream) {
  if (check_plan(p)) return IPFB_EINVAL;
  if (!spec || !x_out) return fail(IPFB_EINVAL, "spec and x_out must be non-NULL device pointers");
  if (check_infmt(infmt, chan_scale)) return IPFB_EINVAL;
  if (!(phi > 0.0) || !std::isfinite(phi))
    return fail(IPFB_EINVAL, "phi must be finite and > 0 (W^T W alone is singular: b unknowns, b - p + 1 equations)");
  if (!p->row_lds) return fail(IPFB_EUNSUPPORTED, "lblock too large for the row stage");
  if (p->nblock < p->ntap) return fail(IPFB_EINVAL, "nblock must be >= ntap (at least one spectrum)");
  const int nt = p->ntap;
  if (nt != 2 && nt != 3 && nt != 4 && nt != 5 && nt != 8 && nt != 16)
    return fail(IPFB_EUNSUPPORTED, "the banded Cholesky solver takes ntap in {2, 3, 4, 5, 8, 16} (got %d)", nt);
  DeviceGuard g(p->dev);
  if (!p->tik_ws) {
    if (int s2 = dev_alloc(p, (void**)&p->tik_ws, (size_t)(nt + 1) * p->nblock * p->lblock * sizeof(double)))
      return s2;
  }
  hipStream_t st = (hipStream_t)stream;
  const int64_t nspec = p->nblock - nt + 1;
  hipError_t e;
  {
    ProfScope ps("tik_rows", st);
    e = hipErrorNotSupported;
    if (infmt == IPFB_IN_C4) e = launch_row_c4(p->prec, p->log2n, spec, chan_scale, x_out, nspec, p->twN, st);
    if (e == hipErrorNotSupported) {
      hipGetLastError();
      if (scaled_infmt(infmt)) e = launch_dequant_factors(p->prec, chan_scale, p->lblock / 2 + 1, p->lblock, p->fac, st);
      else e = hipSuccess;
      if (e == hipSuccess) e = launch_row_irfft(p->prec, p->log2n, infmt, spec, p->fac, x_out, nspec, p->twN, st);
    }
  }
  if (e == hipSuccess) {
    ProfScope ps("tik_solve", st);
    e = launch_tikhonov(p->prec, x_out, p->lblock, nt, p->nblock, p->win64, phi, normalise ? 1.0 + phi * phi : 1.0,
                        p->tik_ws, st);
  }
  return launched(e, "ipfb_tikhonov");
}

int ipfb_fir_kernels(ipfb_plan p, double phi, int ltaps, int normalise, void* kernels, void* stream) {
  if (int s = fir_check(p, phi, ltaps)) return s;
  if (!kernels) return fail(IPFB_EINVAL, "kernels must be a non-NULL device pointer");
  DeviceGuard g(p->dev);
  return launched(fir_kernels_into(p, phi, ltaps, normalise, kernels, (hipStream_t)stream), "ipfb_fir_kernels");
}

int ipfb_fir(ipfb_plan p, int infmt, const void* spec, const float* chan_scale, double phi, int ltaps,
             int normalise, void* x_out, void* stream) {
  if (int s = fir_check(p, phi, ltaps)) return s;
  if (!spec || !x_out) return fail(IPFB_EINVAL, "spec and x_out must be non-NULL device pointers");
  if (check_infmt(infmt, chan_scale)) return IPFB_EINVAL;
  DeviceGuard g(p->dev);
  if (!p->fir_g) {
    if (int s2 = dev_alloc(p, &p->fir_g, (size_t)kFirMaxTaps * p->lblock * esize(p->prec))) return s2;
  }
  hipStream_t st = (hipStream_t)stream;
  hipError_t e = hipSuccess;
  const int nn = normalise ? 1 : 0;
  if (!(phi == p->fir_phi) || ltaps != p->fir_taps || nn != p->fir_norm) {
    ProfScope ps("fir_kernels", st);
    e = fir_kernels_into(p, phi, ltaps, normalise, p->fir_g, st);
    p->fir_phi = e == hipSuccess ? phi : NAN;
    p->fir_taps = ltaps;
    p->fir_norm = nn;
  }
  if (e == hipSuccess) e = rows_into(p, infmt, spec, chan_scale, p->work, st);
  if (e == hipSuccess) {
    ProfScope ps("fir_apply", st);
    e = launch_fir(p->prec, p->work, p->fir_g, x_out, p->lblock, p->nblock, ltaps,
                   p->ntap / 2 - (ltaps - 1) / 2, st);
  }
  return launched(e, "ipfb_fir");
}

}  // extern "C"

// ---- linear boundary, streaming -------------------------------------------
struct ipfb_splan_s {
  ipfb_plan inner = nullptr;  // nblock = chunk: tables and the window buffer
  int64_t chunk = 0;
  int halo = 0;
};

int ipfb_stream_plan_create(ipfb_splan* out, int lblock, int ntap, const double* window, int64_t chunk, int halo,
                            int prec) {
  if (!out) return fail(IPFB_EINVAL, "plan output pointer is NULL");
  *out = nullptr;
  if (prec != IPFB_F32 && prec != IPFB_F64) return fail(IPFB_EINVAL, "prec must be IPFB_F32 or IPFB_F64");
  if (ntap < 1) return fail(IPFB_EINVAL, "ntap must be >= 1 (got %d)", ntap);
  if (!is_pow2(chunk) || chunk < 4 || ilog2(chunk) > max_log2_col(prec))
    return fail(IPFB_EINVAL, "chunk must be a power of two in [4, 2^%d] (got %lld)", max_log2_col(prec),
                (long long)chunk);
  if (halo < 0) return fail(IPFB_EINVAL, "halo must be >= 0");
  if (chunk - (ntap - 1) - 2 * (int64_t)halo < 1)
    return fail(IPFB_EINVAL, "chunk - (ntap - 1) - 2 halo must be >= 1 (chunk %lld, ntap %d, halo %d)",
                (long long)chunk, ntap, halo);
  ipfb_plan inner = nullptr;
  int st = ipfb_plan_create(&inner, lblock, ntap, window, chunk, prec);
  if (st) return st;
  if (!inner->row_lds) {
    ipfb_plan_destroy(inner);
    return fail(IPFB_EUNSUPPORTED, "the streaming inverse supports lblock <= 2^%d for this precision",
                max_log2_row(prec));
  }
  ipfb_splan sp = new ipfb_splan_s();
  sp->inner = inner;
  sp->chunk = chunk;
  sp->halo = halo;
  *out = sp;
  return ok();
}

int ipfb_stream_plan_destroy(ipfb_splan sp) {
  if (!sp) return fail(IPFB_EINVAL, "plan is NULL");
  int st = ipfb_plan_destroy(sp->inner);
  delete sp;
  return st ? st : ok();
}

int ipfb_wiener_stream(ipfb_splan sp, int infmt, const void* spec, const float* chan_scale, int64_t nspec,
                       double phi, int normalise, void* x_out, void* stream) {
  if (!sp) return fail(IPFB_EINVAL, "plan is NULL");
  ipfb_plan p = sp->inner;
  if (!spec || !x_out) return fail(IPFB_EINVAL, "spec and x_out must be non-NULL device pointers");
  if (check_infmt(infmt, chan_scale)) return IPFB_EINVAL;
  if (!(phi >= 0.0) || !std::isfinite(phi)) return fail(IPFB_EINVAL, "phi must be finite and >= 0");
  if (nspec < 1) return fail(IPFB_EINVAL, "nspec must be >= 1");
  DeviceGuard g(p->dev);
  hipStream_t st = (hipStream_t)stream;
  const int N = p->lblock, K = N / 2 + 1;
  const size_t es = esize(p->prec), fb = (size_t)N * es;
  const size_t inb = infmt_bytes(infmt);
  const int64_t B = sp->chunk, h = sp->halo, m = B - (p->ntap - 1), L = m - 2 * h;
  const int64_t nframes = nspec + p->ntap - 1;
  char* work = (char*)p->work;
  char* xo = (char*)x_out;
  hipError_t e = hipSuccess;
  bool row_c4 = infmt == IPFB_IN_C4;
  if (row_c4) {  // the persistent row kernel exists for this frame length?
    e = launch_row_c4(p->prec, p->log2n, nullptr, nullptr, nullptr, 0, nullptr, st);
    if (e == hipErrorNotSupported) {
      hipGetLastError();
      row_c4 = false;
      e = hipSuccess;
    }
  }
  if (e == hipSuccess && !row_c4 && scaled_infmt(infmt)) e = launch_dequant_factors(p->prec, chan_scale, K, N, p->fac, st);
  // windows of the overlap-save reading: window c keeps output frames
  // [c L, c L + nkeep); it starts at spectrum s0 and holds nvalid spectra,
  // zero-extended to B frames
  for (int64_t k0 = 0; k0 < nframes && e == hipSuccess; k0 += L) {
    int64_t s0 = k0 - h < nspec - m ? k0 - h : nspec - m;
    if (s0 < 0) s0 = 0;
    const int64_t nvalid = nspec - s0 < m ? nspec - s0 : m;
    const int64_t nkeep = nframes - k0 < L ? nframes - k0 : L;
    const int64_t off = k0 - s0;
    const char* sp_in = (const char*)spec + (size_t)s0 * K * inb;
    if (row_c4)
      e = launch_row_c4(p->prec, p->log2n, sp_in, chan_scale, work, nvalid, p->twN, st);
    else
      e = launch_row_irfft(p->prec, p->log2n, infmt, sp_in, p->fac, work, nvalid, p->twN, st);
    if (e == hipSuccess && nvalid < B) e = launch_zero(work + (size_t)nvalid * fb, (size_t)(B - nvalid) * fb, st);
    if (e != hipSuccess) break;
    if (use_recursive(p, phi)) {  // the recursive stage, its last pass writing the kept frames
      e = rec_stage(p, work, phi, 0, normalise ? 1.0 + phi * phi : 1.0, st, nullptr, xo + (size_t)k0 * fb, off,
                    nkeep);
    } else if (p->log2b > 9) {
      for (int pass = 0; pass < 2 && e == hipSuccess; ++pass)
        e = launch_col_wiener_nat(p->prec, p->log2b, pass, work, N, p->ntap, p->win64, phi, normalise, p->twB,
                                  p->twB64, st);
      if (e == hipSuccess)
        e = launch_col_wiener_nat(p->prec, p->log2b, 2, work, N, p->ntap, p->win64, phi, normalise, p->twB,
                                  p->twB64, st, 0, -1, xo + (size_t)k0 * fb, (int)off, (int)nkeep);
    } else {
      e = launch_col_wiener_nat(p->prec, p->log2b, 1, work, N, p->ntap, p->win64, phi, normalise, p->twB, p->twB64,
                                st);
      if (e == hipSuccess)
        e = hipMemcpyAsync(xo + (size_t)k0 * fb, work + (size_t)off * fb, (size_t)nkeep * fb,
                           hipMemcpyDeviceToDevice, st);
    }
  }
  return launched(e, "ipfb_wiener_stream");
}

}  // extern "C"

namespace {

// z = M^-1 r (the CG preconditioner) and the partial sums of r . z in
// part: formed by the column kernel itself where its workgroups fit the
// partial-sum slots, else by a separate dot-product pass.
hipError_t precond_dot(ipfb_plan p, const void* rT, void* zT, double phi_precond, int64_t S, double* part,
                       hipStream_t st) {
  hipError_t e = launch_col_wiener(p->prec, p->log2b, rT, zT, p->lblock, p->ntap, p->win64, phi_precond, 1, p->twB,
                                   p->twB64, st, 1, part);
  if (e != hipErrorNotSupported) return e;
  hipGetLastError();
  e = launch_col_wiener(p->prec, p->log2b, rT, zT, p->lblock, p->ntap, p->win64, phi_precond, 1, p->twB, p->twB64,
                        st, 1);
  if (e == hipSuccess) e = launch_cg_dot(p->prec, rT, zT, S, part, st);
  return e;
}

// The CG buffers of one solve: seven vectors in the transposed layout, the
// mask bits in the same layout, the column autocorrelations, the partial sums
// and the scalars.
struct CgBufs {
  void *xT, *rT, *zT, *pT, *qT, *rhsT, *priorT;
  uint32_t* maskT;
  double *autoc, *part, *sc;
};

size_t cg_mask_bytes(ipfb_plan p) {
  return (size_t)p->lblock * (size_t)((p->nblock + 31) / 32) * sizeof(uint32_t);
}

// Lays the CG buffers out from base: 7 vectors, the mask bits, then (256-byte
// aligned) the autocorrelations, partial sums and scalars. Returns the bytes.
size_t cg_layout(ipfb_plan p, char* base, CgBufs* o) {
  const size_t vb = (size_t)p->lblock * (size_t)p->nblock * esize(p->prec);
  auto up = [](size_t v) { return (v + 255) & ~(size_t)255; };
  size_t off = 7 * vb;
  const size_t om = off;
  off = up(off + cg_mask_bytes(p));
  const size_t oa = off;
  off = up(off + (size_t)p->lblock * (2 * p->ntap - 1) * sizeof(double));
  const size_t op = off;
  off = up(off + kCgParts * sizeof(double));
  const size_t os = off;
  off += 8 * sizeof(double);
  if (o) {
    void** v[7] = {&o->xT, &o->rT, &o->zT, &o->pT, &o->qT, &o->rhsT, &o->priorT};
    for (int i = 0; i < 7; ++i) *v[i] = base + i * vb;
    o->maskT = (uint32_t*)(base + om);
    o->autoc = (double*)(base + oa);
    o->part = (double*)(base + op);
    o->sc = (double*)(base + os);
  }
  return off;
}

// ML-CG runs on the natural layout [b][N] (stencils down the columns, the
// recursive preconditioner) where the transposed form's in-LDS column FFT
// does not apply (nblock not a power of two, or above 2^15), or when the
// plan asks for the recursive column method.
bool cg_natural(ipfb_plan p) { return !p->col_lds || p->col_method == IPFB_COLS_RECURSIVE; }

int ml_cg_check(ipfb_plan p, int infmt, const void* spec, const float* chan_scale, const uint32_t* mask,
                const void* prior, double lam, double phi_x0, double phi_precond, int iters, const void* x_init,
                void* x_out) {
  if (check_plan(p)) return IPFB_EINVAL;
  if (!spec || !mask || !prior || !x_out) return fail(IPFB_EINVAL, "spec, mask, prior and x_out must be non-NULL");
  if (check_infmt(infmt, chan_scale)) return IPFB_EINVAL;
  if (!(lam >= 0.0) || !std::isfinite(lam)) return fail(IPFB_EINVAL, "lambda must be finite and >= 0");
  if (!(phi_precond > 0.0) || !std::isfinite(phi_precond)) return fail(IPFB_EINVAL, "phi_precond must be > 0");
  if (!(phi_x0 >= 0.0) || !std::isfinite(phi_x0)) return fail(IPFB_EINVAL, "phi_x0 must be finite and >= 0");
  if (iters < 0) return fail(IPFB_EINVAL, "iters must be >= 0");
  if (!p->row_lds)
    return fail(IPFB_EUNSUPPORTED, "ipfb_ml_cg supports lblock <= 2^%d for this precision", max_log2_row(p->prec));
  if (cg_natural(p)) {
    if (!p->iir_coef_pc)
      return fail(IPFB_EUNSUPPORTED, "ipfb_ml_cg with nblock = %lld needs ntap = 4 (got %d); other tap counts take "
                                     "power-of-two nblock <= 2^%d",
                  (long long)p->nblock, p->ntap, max_log2_col(p->prec));
    if (!(phi_precond >= kIirMinPhi))
      return fail(IPFB_EUNSUPPORTED, "the recursive preconditioner needs phi_precond >= %g", kIirMinPhi);
    if (!x_init && !(phi_x0 >= kIirMinPhi))
      return fail(IPFB_EUNSUPPORTED, "the recursive Wiener start needs phi_x0 >= %g (or an x_init)", kIirMinPhi);
  }
  return IPFB_OK;
}

// Enqueues the whole solve on st with the buffers in c (the plan's frame
// buffers work and work2 hold d and its transpose).
hipError_t ml_cg_enqueue(ipfb_plan p, const CgBufs& c, int infmt, const void* spec, const float* chan_scale,
                         const uint32_t* mask, const void* prior, double lam, double phi_x0, double phi_precond,
                         int iters, const void* x_init, void* x_out, double* resid_norms, hipStream_t st) {
  const int64_t b = p->nblock, S = (int64_t)p->lblock * b;
  void* dT = p->work2;
  hipError_t e;
  {
    ProfScope ps("cg_setup", st);
    if (scaled_infmt(infmt)) e = launch_dequant_factors(p->prec, chan_scale, p->lblock / 2 + 1, p->lblock, p->fac, st);
    else e = hipSuccess;
    if (e == hipSuccess) e = launch_row_irfft(p->prec, p->log2n, infmt, spec, p->fac, p->work, b, p->twN, st);
    if (e == hipSuccess) e = launch_transpose(p->prec, p->work, dT, b, p->lblock, st);
    if (e == hipSuccess) e = launch_maskbits_transpose(mask, p->lblock, b, c.maskT, st);
    if (e == hipSuccess) e = launch_transpose(p->prec, prior, c.priorT, b, p->lblock, st);
    if (e == hipSuccess) e = launch_cg_autocorr(p->win64, p->lblock, p->ntap, c.autoc, st);
    if (e == hipSuccess)
      e = launch_cg_rhs(p->prec, dT, c.rhsT, p->win64, c.maskT, c.priorT, lam, p->lblock, p->ntap, b, S, st);
    if (e == hipSuccess) {
      if (x_init) e = launch_transpose(p->prec, x_init, c.xT, b, p->lblock, st);
      else e = launch_col_wiener(p->prec, p->log2b, dT, c.xT, p->lblock, p->ntap, p->win64, phi_x0, 1, p->twB,
                                 p->twB64, st);
    }
    // r0 = rhs - H x0, z0 = M^-1 r0, p0 = z0, rho0 = r0.z0
    if (e == hipSuccess) e = launch_cg_normal(p->prec, c.xT, c.qT, c.autoc, c.maskT, lam, p->ntap, b, S, c.part, st);
    if (e == hipSuccess) e = launch_cg_resid(p->prec, c.rhsT, c.qT, c.rT, S, c.part, st);
    if (e == hipSuccess) e = launch_cg_scalar(c.part, 2, c.sc, resid_norms, 0, st);
    // z0 = M^-1 r0 with the partial sums of r0 . z0 formed on the way out
    if (e == hipSuccess) e = precond_dot(p, c.rT, c.zT, phi_precond, S, c.part, st);
    if (e == hipSuccess) e = launch_cg_p(p->prec, c.pT, c.zT, c.sc, 0, S, st);
    if (e == hipSuccess) e = launch_cg_scalar(c.part, 0, c.sc, nullptr, 0, st);
  }
  for (int k = 1; k <= iters && e == hipSuccess; ++k) {
    ProfScope ps("cg_iter", st);
    e = launch_cg_normal(p->prec, c.pT, c.qT, c.autoc, c.maskT, lam, p->ntap, b, S, c.part, st);
    if (e == hipSuccess) e = launch_cg_scalar(c.part, 1, c.sc, nullptr, 0, st);
    if (e == hipSuccess) e = launch_cg_xr(p->prec, c.xT, c.rT, c.pT, c.qT, c.sc, S, c.part, st);
    if (e == hipSuccess) e = launch_cg_scalar(c.part, 2, c.sc, resid_norms, k, st);
    if (e == hipSuccess) e = precond_dot(p, c.rT, c.zT, phi_precond, S, c.part, st);
    if (e == hipSuccess) e = launch_cg_scalar(c.part, 3, c.sc, nullptr, 0, st);
    if (e == hipSuccess) e = launch_cg_p(p->prec, c.pT, c.zT, c.sc, 1, S, st);
  }
  if (e == hipSuccess) {
    ProfScope ps("cg_out", st);
    e = launch_transpose(p->prec, c.xT, x_out, p->lblock, b, st);
  }
  return e;
}

// The same solve on the natural layout: the iterate lives in x_out, d in the
// plan's frame buffer, the mask and prior are read as given; z = M^-1 r is r
// through the recursive stage with numerator 1.
hipError_t ml_cg_enqueue_nat(ipfb_plan p, const CgBufs& c, int infmt, const void* spec, const float* chan_scale,
                             const uint32_t* mask, const void* prior, double lam, double phi_x0, double phi_precond,
                             int iters, const void* x_init, void* x_out, double* resid_norms, hipStream_t st) {
  const int64_t b = p->nblock, S = (int64_t)p->lblock * b;
  const int N = p->lblock;
  const size_t vb = (size_t)S * esize(p->prec);
  void* x = x_out;
  // z = M^-1 r with the partial sums of r . z
  auto precond_dot_nat = [&]() -> hipError_t {
    hipError_t e2 = hipMemcpyAsync(c.zT, c.rT, vb, hipMemcpyDeviceToDevice, st);
    if (e2 == hipSuccess) e2 = rec_stage(p, c.zT, phi_precond, 1, 1.0, st, nullptr);
    if (e2 == hipSuccess) e2 = launch_cg_dot(p->prec, c.rT, c.zT, S, c.part, st);
    return e2;
  };
  hipError_t e;
  {
    ProfScope ps("cg_setup", st);
    e = rows_into(p, infmt, spec, chan_scale, p->work, st);
    if (e == hipSuccess) e = launch_cg_autocorr(p->win64, N, p->ntap, c.autoc, st);
    if (e == hipSuccess) e = launch_cg_rhs_nat(p->prec, p->work, c.rhsT, p->win64, mask, prior, lam, N, p->ntap, b, st);
    if (e == hipSuccess) {
      if (x_init) {
        if (x_init != x) e = hipMemcpyAsync(x, x_init, vb, hipMemcpyDeviceToDevice, st);
      } else {
        e = hipMemcpyAsync(x, p->work, vb, hipMemcpyDeviceToDevice, st);
        if (e == hipSuccess) e = rec_stage(p, x, phi_x0, 0, 1.0 + phi_x0 * phi_x0, st, nullptr);
      }
    }
    if (e == hipSuccess) e = launch_cg_normal_nat(p->prec, x, c.qT, c.autoc, mask, lam, N, p->ntap, b, c.part, st);
    if (e == hipSuccess) e = launch_cg_resid(p->prec, c.rhsT, c.qT, c.rT, S, c.part, st);
    if (e == hipSuccess) e = launch_cg_scalar(c.part, 2, c.sc, resid_norms, 0, st);
    if (e == hipSuccess) e = precond_dot_nat();
    if (e == hipSuccess) e = launch_cg_p(p->prec, c.pT, c.zT, c.sc, 0, S, st);
    if (e == hipSuccess) e = launch_cg_scalar(c.part, 0, c.sc, nullptr, 0, st);
  }
  for (int k = 1; k <= iters && e == hipSuccess; ++k) {
    ProfScope ps("cg_iter", st);
    e = launch_cg_normal_nat(p->prec, c.pT, c.qT, c.autoc, mask, lam, N, p->ntap, b, c.part, st);
    if (e == hipSuccess) e = launch_cg_scalar(c.part, 1, c.sc, nullptr, 0, st);
    if (e == hipSuccess) e = launch_cg_xr(p->prec, x, c.rT, c.pT, c.qT, c.sc, S, c.part, st);
    if (e == hipSuccess) e = launch_cg_scalar(c.part, 2, c.sc, resid_norms, k, st);
    if (e == hipSuccess) e = precond_dot_nat();
    if (e == hipSuccess) e = launch_cg_scalar(c.part, 3, c.sc, nullptr, 0, st);
    if (e == hipSuccess) e = launch_cg_p(p->prec, c.pT, c.zT, c.sc, 1, S, st);
  }
  return e;
}

hipError_t ml_cg_run(ipfb_plan p, const CgBufs& c, int infmt, const void* spec, const float* chan_scale,
                     const uint32_t* mask, const void* prior, double lam, double phi_x0, double phi_precond, int iters,
                     const void* x_init, void* x_out, double* resid_norms, hipStream_t st) {
  if (cg_natural(p))
    return ml_cg_enqueue_nat(p, c, infmt, spec, chan_scale, mask, prior, lam, phi_x0, phi_precond, iters, x_init,
                             x_out, resid_norms, st);
  return ml_cg_enqueue(p, c, infmt, spec, chan_scale, mask, prior, lam, phi_x0, phi_precond, iters, x_init, x_out,
                       resid_norms, st);
}

// ---- the entry point for callers that cannot allocate ------------------------
// One file-scope device array holds every buffer of ipfb_ml_cg_noalloc's
// solve. Each device the library runs on has its own copy at its own address,
// found once per device with hipGetSymbolAddress; host code uses only those
// addresses, never the array's name (which on the host is a stand-in, not a
// device address).
constexpr size_t kNoAllocScratchBytes = size_t(64) << 20;
__device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// The current device's copy of the scratch array (dev must be current).
int scratch_ptr(int dev, char** out) {
  if (dev < 0 || dev >= kMaxDevices) return fail(IPFB_EUNSUPPORTED, "device %d beyond the scratch table", dev);
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) {
      hipGetLastError();
      return fail(IPFB_EHIP, "hipGetSymbolAddress(scratch) on device %d: %s", dev, hipGetErrorString(e));
    }
    g_scratch_ptr[dev] = ptr;
  }
  *out = (char*)g_scratch_ptr[dev];
  return IPFB_OK;
}

}  // namespace

extern "C" {

int ipfb_ml_cg(ipfb_plan p, int infmt, const void* spec, const float* chan_scale, const uint32_t* mask,
               const void* prior, double lam, double phi_x0, double phi_precond, int iters, const void* x_init,
               void* x_out, double* resid_norms, void* stream) {
  if (int s = ml_cg_check(p, infmt, spec, chan_scale, mask, prior, lam, phi_x0, phi_precond, iters, x_init, x_out))
    return s;
  DeviceGuard g(p->dev);
  if (!p->cg) {
    if (int s2 = dev_alloc(p, &p->cg, cg_layout(p, nullptr, nullptr))) return s2;
  }
  CgBufs c;
  cg_layout(p, (char*)p->cg, &c);
  return launched(ml_cg_run(p, c, infmt, spec, chan_scale, mask, prior, lam, phi_x0, phi_precond, iters, x_init,
                            x_out, resid_norms, (hipStream_t)stream),
                  "ipfb_ml_cg");
}

int ipfb_ml_cg_noalloc(ipfb_plan p, int infmt, const void* spec, const float* chan_scale, const uint32_t* mask,
                       const void* prior, double lam, double phi_x0, double phi_precond, int iters,
                       const void* x_init, void* x_out, double* resid_norms, void* stream) {
  if (int s = ml_cg_check(p, infmt, spec, chan_scale, mask, prior, lam, phi_x0, phi_precond, iters, x_init, x_out))
    return s;
  const size_t need = cg_layout(p, nullptr, nullptr);
  if (need > kNoAllocScratchBytes)
    return fail(IPFB_EUNSUPPORTED,
                "ipfb_ml_cg_noalloc: this plan's solve needs %zu bytes of scratch, more than the %zu available "
                "(at most about %zu samples in this precision); use ipfb_ml_cg",
                need, kNoAllocScratchBytes,
                kNoAllocScratchBytes / (7 * esize(p->prec) + 1));
  DeviceGuard g(p->dev);
  char* base = nullptr;
  if (int s = scratch_ptr(p->dev, &base)) return s;
  CgBufs c;
  cg_layout(p, base, &c);
  return launched(ml_cg_run(p, c, infmt, spec, chan_scale, mask, prior, lam, phi_x0, phi_precond, iters, x_init,
                            x_out, resid_norms, (hipStream_t)stream),
                  "ipfb_ml_cg_noalloc");
}

int ipfb_autospectrum(ipfb_plan p, const void* y, double* autospec, void* stream) {
  if (check_plan(p)) return IPFB_EINVAL;
  if (!y || !autospec) return fail(IPFB_EINVAL, "y and autospec must be non-NULL device pointers");
  DeviceGuard g(p->dev);
  hipStream_t st = (hipStream_t)stream;
  const int K = p->lblock / 2 + 1;
  hipError_t e;
  {
    ProfScope ps("autospec_partial", st);
    e = launch_power_partial(p->prec, y, p->nblock, K, p->jchunk, p->part, st);
  }
  if (e == hipSuccess) {
    ProfScope ps("autospec_final", st);
    e = launch_power_final(p->part, p->nchunks, K, 1.0 / (double)p->nblock, autospec, st);
  }
  return launched(e, "ipfb_autospectrum");
}

int upchannelize(ipfb_plan fine, const void* x, void* y_fine, double* autospec, void* stream) {
  if (check_plan(fine)) return IPFB_EINVAL;
  if (!fine->row_lds && autospec && x && y_fine) {
    // long frames: the power sums ride along in the second FFT pass
    DeviceGuard g(fine->dev);
    hipStream_t st = (hipStream_t)stream;
    const int K = fine->lblock / 2 + 1;
    hipError_t e = hipSuccess;
    static const char* const names[2] = {"pfb_fwd_long_p1", "pfb_fwd_long_p2"};
    for (int pass = 0; pass < 2 && e == hipSuccess; ++pass) {
      ProfScope ps(names[pass], st);
      e = launch_pfb_fwd_long(fine->prec, fine->log2n, pass, x, y_fine, fine->nblock, fine->ntap, fine->winT,
                              fine->twS, fine->tmp, fine->fchunk, fine->part, st);
    }
    if (e == hipSuccess) {
      ProfScope ps("autospec_final", st);
      e = launch_power_final(fine->part, fine->nfchunks, K, 1.0 / (double)fine->nblock, autospec, st);
    }
    return launched(e, "upchannelize");
  }
  int s = pfb_forward(fine, x, y_fine, stream);
  if (s) return s;
  if (autospec) return ipfb_autospectrum(fine, y_fine, autospec, stream);
  return ok();
}

int ipfb_mask_structured(ipfb_plan p, int R, int L, uint32_t* mask, void* stream) {
  if (check_plan(p)) return IPFB_EINVAL;
  if (!mask) return fail(IPFB_EINVAL, "mask must be a non-NULL device pointer");
  if (R < 1) return fail(IPFB_EINVAL, "R must be >= 1");
  if (L < 0 || L > p->lblock || (L & 1)) return fail(IPFB_EINVAL, "L must be even and in [0, lblock]");
  DeviceGuard g(p->dev);
  return launched(launch_mask_structured(mask, p->lblock, p->nblock, R, L, (hipStream_t)stream),
                  "ipfb_mask_structured");
}

int ipfb_mask_pack(const uint8_t* mask, int64_t nsamples, uint32_t* bits, void* stream) {
  if (nsamples < 0) return fail(IPFB_EINVAL, "nsamples must be >= 0");
  if (nsamples > 0 && (!mask || !bits)) return fail(IPFB_EINVAL, "mask and bits must be non-NULL device pointers");
  return launched(launch_mask_pack(mask, nsamples, bits, (hipStream_t)stream), "ipfb_mask_pack");
}

int ipfb_delta_analytic(ipfb_plan p, int64_t nfreq, double phi, double snr, double* out, void* stream) {
  if (check_plan(p)) return IPFB_EINVAL;
  if (!out) return fail(IPFB_EINVAL, "out must be a non-NULL device pointer");
  if (nfreq < 1 || nfreq > (int64_t(1) << 31) - 1) return fail(IPFB_EINVAL, "nfreq must be in [1, 2^31)");
  if (!(phi >= 0.0) || !std::isfinite(phi)) return fail(IPFB_EINVAL, "phi must be finite and >= 0");
  if (phi == 0.0 && !(snr > 0.0 && std::isfinite(snr))) return fail(IPFB_EINVAL, "phi = 0 needs a finite snr > 0");
  DeviceGuard g(p->dev);
  return launched(launch_delta_analytic(p->win64, p->lblock, p->ntap, nfreq, phi, snr, out, (hipStream_t)stream),
                  "ipfb_delta_analytic");
}

int ipfb_autospectrum_error(ipfb_plan fine, const void* x_true, const void* x_hat, double* delta, void* stream) {
  if (check_plan(fine)) return IPFB_EINVAL;
  if (!x_true || !x_hat || !delta) return fail(IPFB_EINVAL, "x_true, x_hat and delta must be non-NULL");
  DeviceGuard g(fine->dev);
  const int64_t S = (int64_t)fine->nblock * fine->lblock;
  const int K = fine->lblock / 2 + 1;
  const size_t es = esize(fine->prec);
  const size_t diff_b = (size_t)S * es, y_b = (size_t)fine->nblock * K * 2 * es;
  if (!fine->diag) {
    int s2 = dev_alloc(fine, &fine->diag, diff_b + y_b + 2 * (size_t)K * sizeof(double));
    if (s2) return s2;
  }
  char* base = (char*)fine->diag;
  void* diff = base;
  void* Y = base + diff_b;
  double* A_true = (double*)(base + diff_b + y_b);
  double* A_diff = A_true + K;
  hipStream_t st = (hipStream_t)stream;
  hipError_t e = launch_sub(fine->prec, x_true, x_hat, diff, S, st);
  if (e != hipSuccess) return launched(e, "ipfb_autospectrum_error");
  // the forward PFB is linear: the spectra of x_true - x_hat are Y - Yhat
  int s2 = upchannelize(fine, x_true, Y, A_true, stream);
  if (!s2) s2 = upchannelize(fine, diff, Y, A_diff, stream);
  if (s2) return s2;
  return launched(launch_ratio(A_diff, A_true, delta, K, st), "ipfb_autospectrum_error");
}

int ipfb_quantize_c4(ipfb_plan p, const void* y, double levels_rms, uint8_t* packed, float* scales, void* stream) {
  if (check_plan(p)) return IPFB_EINVAL;
  if (!y || !packed || !scales) return fail(IPFB_EINVAL, "y, packed and scales must be non-NULL device pointers");
  if (!(levels_rms > 0.0)) return fail(IPFB_EINVAL, "levels_rms must be > 0");
  DeviceGuard g(p->dev);
  hipStream_t st = (hipStream_t)stream;
  const int K = p->lblock / 2 + 1;
  // halfpow_k = mean_j |y_jk|^2 / 2 lands in the last row of the partials
  double* halfpow = p->part;  // reuse: final sums overwrite chunk 0 after the partial pass
  hipError_t e = launch_power_partial(p->prec, y, p->nblock, K, p->jchunk, p->part, st);
  if (e == hipSuccess) e = launch_power_final(p->part, p->nchunks, K, 0.5 / (double)p->nblock, halfpow, st);
  if (e == hipSuccess) e = launch_scales(halfpow, K, levels_rms, scales, st);
  if (e == hipSuccess) e = launch_quantize(p->prec, y, p->nblock, K, scales, packed, st);
  return launched(e, "ipfb_quantize_c4");
}

int ipfb_profile_enable(int on) {
  std::lock_guard<std::mutex> lk(g_pm);
  g_prof = (on != 0);
  return IPFB_OK;
}

int ipfb_profile_reset(void) {
  std::lock_guard<std::mutex> lk(g_pm);
  for (auto& r : g_recs) {
    hipEventSynchronize(r.b);
    g_pool.push_back(r.a);
    g_pool.push_back(r.b);
  }
  g_recs.clear();
  return IPFB_OK;
}

int ipfb_profile_query(const char* name, double* total_ms, int64_t* launches) {
  if (!name || !total_ms || !launches) return fail(IPFB_EINVAL, "NULL argument");
  std::lock_guard<std::mutex> lk(g_pm);
  double tot = 0.0;
  int64_t n = 0;
  for (auto& r : g_recs) {
    if (strcmp(r.name, name) != 0) continue;
    if (hipEventSynchronize(r.b) != hipSuccess) return fail(IPFB_EHIP, "hipEventSynchronize failed");
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, r.a, r.b) != hipSuccess) return fail(IPFB_EHIP, "hipEventElapsedTime failed");
    tot += ms;
    ++n;
  }
  *total_ms = tot;
  *launches = n;
  return ok();
}

}  // extern "C"

// ============================================================================
// Batched form: many independent streams with their own nblock, one lblock,
// window and precision. Each stream runs the same steps as ipfb_wiener; a
// stream whose nblock is a power of two uses the LDS column kernel, any other
// length the Bluestein column path. The whole multi-stream sequence is
// captured once into a HIP graph and replayed by one graph launch per call.
// ============================================================================
namespace {

// In-place iterative radix-2 FFT (host, double): forward sign e^{-2 pi i jk/n}.
void host_fft(std::vector<std::complex<double>>& a) {
  const size_t n = a.size();
  for (size_t i = 1, j = 0; i < n; ++i) {
    size_t bit = n >> 1;
    for (; j & bit; bit >>= 1) j ^= bit;
    j ^= bit;
    if (i < j) std::swap(a[i], a[j]);
  }
  for (size_t len = 2; len <= n; len <<= 1) {
    std::vector<std::complex<double>> w(len / 2);
    for (size_t k = 0; k < len / 2; ++k) {
      const long double ang = -2.0L * 3.14159265358979323846264338327950288L * (long double)k / (long double)len;
      w[k] = std::complex<double>((double)cosl(ang), (double)sinl(ang));
    }
    for (size_t i = 0; i < n; i += len)
      for (size_t k = 0; k < len / 2; ++k) {
        const std::complex<double> u = a[i + k], v = a[i + k + len / 2] * w[k];
        a[i + k] = u + v;
        a[i + k + len / 2] = u - v;
      }
  }
}

struct BluTables {  // per distinct nblock b
  int log2m = 0;
  int crow_l1 = 0;        // split the Crow layout is built for
  void* chirp = nullptr;  // [b] complex, plan precision
  void* Crow = nullptr;   // [M1][M2] complex
  double* twb64 = nullptr;  // [b] complex double
  void* twB = nullptr;      // power-of-two b: Stockham table [b]
};

struct MTables {  // per distinct convolution length M
  void* buf = nullptr;  // tLo (256) | tHi (max(1, M/256))
};

}  // namespace

struct ipfb_bplan_s {
  int lblock = 0, ntap = 0, prec = 0, log2n = 0, dev = 0, nstreams = 0;
  std::vector<int64_t> nblock;
  double* win64 = nullptr;
  void* twN = nullptr;
  void* fac = nullptr;
  std::map<int64_t, BluTables> blu;
  std::map<int, MTables> mtab;
  std::map<int, BluCfg> bcfg;  // per log2m: shape of the Bluestein column path
  void* pow2tw = nullptr;      // e^{-2 pi i m/2^l} for l = 1..8, table l at offset 2^l - 2
  double tuned_us = 0.0;       // sum over lengths of the chosen shapes' time (last tune)
  int64_t blu_maxb = 0;
  void* f0 = nullptr;  // two frame buffers of max_b * lblock reals
  void* f1 = nullptr;
  void* Tm = nullptr;  // Bluestein four-step scratch
  std::vector<void*> allocs;
  size_t bytes = 0;
  hipStream_t cap = nullptr;
  hipGraphExec_t exec = nullptr;
  std::vector<uintptr_t> key;
  bool use_graph = true;
  // recursive column stage over all streams at once (4 taps): per-column and
  // per-(stream, column) coefficients, segment states of all streams, and the
  // device tables the multi-stream kernels read (rewritten when the caller's
  // pointers change)
  int col_method = IPFB_COLS_AUTO;
  double* rec_coef = nullptr;
  double* rec_scoef = nullptr;
  void* rec_zs = nullptr;
  IirStream* rec_tab = nullptr;
  RowStream* row_tab = nullptr;
  int64_t rec_nsegt = 0, rec_maxnseg = 0, rec_frames = 0;
  double rec_phi = NAN;
  std::vector<uintptr_t> rec_key;
};

namespace {

int balloc(ipfb_bplan p, void** ptr, size_t bytes) {
  if (bytes == 0) bytes = 16;
  if (inject("alloc")) return fail(IPFB_ENOMEM, "device allocation of %zu bytes failed (injected)", bytes);
  hipError_t e = hipMalloc(ptr, bytes);
  if (e != hipSuccess) {
    *ptr = nullptr;
    hipGetLastError();
    return fail(e == hipErrorOutOfMemory ? IPFB_ENOMEM : IPFB_EHIP, "hipMalloc(%zu): %s", bytes, hipGetErrorString(e));
  }
  p->allocs.push_back(*ptr);
  p->bytes += bytes;
  return IPFB_OK;
}

int bupload(ipfb_bplan p, const std::vector<double>& t, int prec, void** dst) {
  const size_t n = t.size();
  int st = balloc(p, dst, n * esize(prec));
  if (st) return st;
  if (prec == IPFB_F64) return upload(*dst, t.data(), n * sizeof(double));
  std::vector<float> f(n);
  for (size_t i = 0; i < n; ++i) f[i] = (float)t[i];
  return upload(*dst, f.data(), n * sizeof(float));
}

void free_bplan(ipfb_bplan p) {
  if (p->exec) hipGraphExecDestroy(p->exec);
  if (p->cap) hipStreamDestroy(p->cap);
  for (void* q : p->allocs) hipFree(q);
  delete p;
}

int blu_log2m(int64_t b) {
  int l = 0;
  while ((int64_t(1) << l) < 2 * b - 1) ++l;
  return l < 2 ? 2 : l;
}

// chirp c_m = e^{i pi m^2 / b}, with m^2 reduced mod 2b in integers
std::vector<double> chirp_table(int64_t b) {
  std::vector<double> t(2 * b);
  const long double pi = 3.14159265358979323846264338327950288L;
  for (int64_t m = 0; m < b; ++m) {
    const int64_t q = (m * m) % (2 * b);
    const long double a = pi * (long double)q / (long double)b;
    t[2 * m] = (double)cosl(a);
    t[2 * m + 1] = (double)sinl(a);
  }
  return t;
}

// Crow[k1][k2] = C[k1 + M1 k2], C = FFT_M of the symmetric chirp filter, for
// the split M1 = 2^l1 (host, double), re-uploaded into bt.Crow.
int blu_upload_crow(ipfb_bplan p, int64_t b, BluTables& bt, int l1) {
  const int64_t M = int64_t(1) << bt.log2m;
  const int64_t M1 = int64_t(1) << l1, M2 = M / M1;
  std::vector<double> ch = chirp_table(b);
  std::vector<std::complex<double>> c(M, {0.0, 0.0});
  for (int64_t m = 0; m < b; ++m) {
    c[m] = {ch[2 * m], ch[2 * m + 1]};
    if (m > 0) c[M - m] = c[m];
  }
  host_fft(c);
  std::vector<double> crow(2 * M);
  for (int64_t k1 = 0; k1 < M1; ++k1)
    for (int64_t k2 = 0; k2 < M2; ++k2) {
      const std::complex<double> v = c[k1 + M1 * k2];
      crow[2 * (k1 * M2 + k2)] = v.real();
      crow[2 * (k1 * M2 + k2) + 1] = v.imag();
    }
  int st;
  if (!bt.Crow) {
    st = bupload(p, crow, p->prec, &bt.Crow);
  } else if (p->prec == IPFB_F64) {
    st = upload(bt.Crow, crow.data(), crow.size() * sizeof(double));
  } else {
    std::vector<float> f(crow.begin(), crow.end());
    st = upload(bt.Crow, f.data(), f.size() * sizeof(float));
  }
  if (!st) bt.crow_l1 = l1;
  return st;
}

int build_blu(ipfb_bplan p, int64_t b) {
  BluTables bt;
  if (is_pow2(b) && b >= 4 && ilog2(b) <= max_log2_col(p->prec)) {
    std::vector<double> tb = twiddles(b);
    int st = bupload(p, tb, p->prec, &bt.twB);
    if (!st) st = bupload(p, tb, IPFB_F64, (void**)&bt.twb64);
    if (st) return st;
    p->blu[b] = bt;
    return IPFB_OK;
  }
  bt.log2m = blu_log2m(b);
  const int64_t M = int64_t(1) << bt.log2m;
  if (!p->bcfg.count(bt.log2m)) p->bcfg[bt.log2m] = blu_cfg_default(bt.log2m);
  int st = bupload(p, chirp_table(b), p->prec, &bt.chirp);
  if (!st) st = blu_upload_crow(p, b, bt, p->bcfg[bt.log2m].l1);
  if (!st) st = bupload(p, twiddles(b), IPFB_F64, (void**)&bt.twb64);
  if (st) return st;
  p->blu[b] = bt;
  if (!p->pow2tw) {
    std::vector<double> bank;
    for (int l = 1; l <= 8; ++l) {
      std::vector<double> t = twiddles(int64_t(1) << l);
      bank.insert(bank.end(), t.begin(), t.end());
    }
    st = bupload(p, bank, p->prec, &p->pow2tw);
    if (st) return st;
  }
  if (!p->mtab.count(bt.log2m)) {
    std::vector<double> tm = twiddles(M);
    std::vector<double> all;
    for (int m = 0; m < 256; ++m) {  // w_M^m, m < 256 (periodic in M)
      all.push_back(tm[2 * (m % M)]);
      all.push_back(tm[2 * (m % M) + 1]);
    }
    const int64_t nhi = M / 256 > 0 ? M / 256 : 1;
    for (int64_t m = 0; m < nhi; ++m) {
      all.push_back(tm[2 * ((256 * m) % M)]);
      all.push_back(tm[2 * ((256 * m) % M) + 1]);
    }
    MTables mt;
    st = bupload(p, all, p->prec, &mt.buf);
    if (st) return st;
    p->mtab[bt.log2m] = mt;
  }
  return IPFB_OK;
}

// The four twiddle tables of the Bluestein kernels for length 2^log2m split at l1.
void blu_tw4(ipfb_bplan p, int log2m, int l1, const void* tw4[4]) {
  const size_t es = 2 * esize(p->prec);
  const char* bank = (const char*)p->pow2tw;
  const int l2 = log2m - l1;
  tw4[0] = bank + ((size_t(1) << l1) - 2) * es;
  tw4[1] = bank + ((size_t(1) << l2) - 2) * es;
  tw4[2] = p->mtab[log2m].buf;
  tw4[3] = (const char*)p->mtab[log2m].buf + 256 * es;
}

// Makes cfg the shape used for length 2^log2m (re-laying Crow of every
// stream of that length for a new split); drops the captured graph.
int blu_apply_cfg(ipfb_bplan p, int log2m, const BluCfg& cfg) {
  if (!blu_cfg_valid(log2m, cfg)) return fail(IPFB_EINVAL, "invalid Bluestein shape for 2^%d", log2m);
  if (hipDeviceSynchronize() != hipSuccess) {  // no call in flight may read a Crow being re-laid
    hipGetLastError();
    return fail(IPFB_EHIP, "hipDeviceSynchronize failed");
  }
  for (auto& kv : p->blu) {
    if (kv.second.log2m != log2m || kv.second.crow_l1 == cfg.l1) continue;
    int st = blu_upload_crow(p, kv.first, kv.second, cfg.l1);
    if (st) return st;
  }
  p->bcfg[log2m] = cfg;
  if (p->exec) {
    hipGraphExecDestroy(p->exec);
    p->exec = nullptr;
  }
  p->key.clear();
  return IPFB_OK;
}

// ---- autotuner ---------------------------------------------------------------
std::string tune_key(ipfb_bplan p, int log2m) {
  hipDeviceProp_t prop;
  std::string arch = "gpu";
  int cus = 0;
  if (hipGetDeviceProperties(&prop, p->dev) == hipSuccess) {
    arch = prop.gcnArchName;
    arch = arch.substr(0, arch.find(':'));
    cus = prop.multiProcessorCount;
  } else {
    hipGetLastError();
  }
  char buf[256];
  snprintf(buf, sizeof(buf), "%s:%dcu|%s|N%d|T%d|m%d", arch.c_str(), cus, p->prec == IPFB_F64 ? "f64" : "f32",
           p->lblock, p->ntap, log2m);
  return buf;
}

// Loads the entries of the cache file that match this plan's lengths.
int tune_load(ipfb_bplan p, const std::string& path) {
  std::map<std::string, TuneEntry> ent;
  if (!tune_cache_read(path, ent)) return fail(IPFB_EINVAL, "tune cache %s does not parse", path.c_str());
  for (auto& kv : p->bcfg) {
    auto it = ent.find(tune_key(p, kv.first));
    if (it == ent.end()) continue;
    BluCfg c;
    c.l1 = it->second.l1;
    c.mb = it->second.mb;
    c.kb = it->second.kb;
    c.pchunk = it->second.pchunk;
    c.fuse = it->second.fuse;
    c.nat = it->second.nat;
    if (!blu_cfg_valid(kv.first, c)) continue;  // stale entry: keep the current shape
    int st = blu_apply_cfg(p, kv.first, c);
    if (st) return st;
  }
  return IPFB_OK;
}

// Best of three timed runs (after one warm-up) of the Bluestein column path
// for stream length b under shape cfg, on the plan's own buffers: from the
// rows' output to the result in time order (the transposed path's two
// transposes included).
int blu_time(ipfb_bplan p, int64_t b, const BluCfg& cfg, hipStream_t st, hipEvent_t e0, hipEvent_t e1,
             double* us) {
  BluTables& bt = p->blu[b];
  if (bt.crow_l1 != cfg.l1) {
    int s2 = blu_upload_crow(p, b, bt, cfg.l1);
    if (s2) return s2;
  }
  const void* tw4[4];
  blu_tw4(p, bt.log2m, cfg.l1, tw4);
  double best = 1e300;
  for (int r = 0; r < 4; ++r) {
    hipError_t e = hipEventRecord(e0, st);
    if (e == hipSuccess && cfg.nat) {
      e = launch_blu_nat(p->prec, p->f0, p->Tm, bt.chirp, bt.Crow, bt.twb64, b, bt.log2m, cfg, p->lblock, p->ntap,
                         p->win64, 0.1, 1, tw4, st);
    } else if (e == hipSuccess) {  // with the two transposes this path needs
      e = launch_transpose(p->prec, p->f0, p->f1, b, p->lblock, st);
      if (e == hipSuccess)
        e = launch_blu_columns(p->prec, p->f1, p->f0, p->Tm, p->f0, p->f1, bt.chirp, bt.Crow, bt.twb64, b, bt.log2m,
                               cfg, p->lblock, p->ntap, p->win64, 0.1, 1, tw4, st);
      if (e == hipSuccess) e = launch_transpose(p->prec, p->f0, p->f1, p->lblock, b, st);
    }
    if (e == hipSuccess) e = hipEventRecord(e1, st);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float ms = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    if (e != hipSuccess) {
      hipGetLastError();
      return fail(IPFB_EHIP, "autotuner run failed: %s", hipGetErrorString(e));
    }
    if (r > 0 && ms * 1e3 < best) best = ms * 1e3;
  }
  *us = best;
  return IPFB_OK;
}

// Coordinate search per convolution length: for the transposed path, fused or
// not jointly with the column tile, then the split, the row tile and the pairs
// per launch group; for the natural-layout path, the split and the tiles per
// launch group; each stage keeps the fastest, and the fastest overall wins.
int tune_length(ipfb_bplan p, int log2m, BluCfg* out, double* out_us) {
  int64_t b = 0;  // the longest stream of this length stands for all of them
  for (auto& kv : p->blu)
    if (kv.second.log2m == log2m && kv.first > b) b = kv.first;
  if (b == 0) return fail(IPFB_EINVAL, "no stream of convolution length 2^%d", log2m);
  hipStream_t st = p->cap;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    hipGetLastError();
    if (e0) hipEventDestroy(e0);
    return fail(IPFB_EHIP, "hipEventCreate failed");
  }
  BluCfg best = blu_cfg_default(log2m);
  double best_us = 0.0;
  int st2 = blu_time(p, b, best, st, e0, e1, &best_us);
  auto trial = [&](BluCfg c) {
    if (st2 || !blu_cfg_valid(log2m, c)) return;
    double us = 0.0;
    st2 = blu_time(p, b, c, st, e0, e1, &us);
    if (!st2 && us < best_us) {
      best = c;
      best_us = us;
    }
  };
  // fused or not together with the column tile (the fused pass is the most
  // sensitive to the tile width), then the split, then the row tile
  for (int fuse : {1, 0})
    for (int mb : {8, 16, 32}) {
      BluCfg c = best;
      c.fuse = fuse;
      c.mb = mb;
      if (c.fuse == best.fuse && c.mb == best.mb) continue;
      trial(c);
    }
  const BluCfg after_tile = best;
  const int d = (log2m + 1) / 2;
  for (int l1 : {d - 1, d + 1}) {
    BluCfg c = after_tile;
    c.l1 = l1;
    trial(c);
  }
  const BluCfg after_split = best;
  for (int kb : {8, 32}) {
    BluCfg c = after_split;
    c.kb = kb;
    trial(c);
  }
  const BluCfg after_mb = best;
  const int npairs = (p->lblock + 1) / 2;
  for (int pc : {512, 256, 128, 64}) {
    if (pc >= npairs) continue;
    BluCfg c = after_mb;
    c.pchunk = pc;
    trial(c);
  }
  // the natural-layout path, searched on its own (its best may lose to the
  // transposed path's): the split, then tiles per launch group
  const int ntiles = (p->lblock / 2 + blu_nat_tile_pairs(p->prec) - 1) / blu_nat_tile_pairs(p->prec);
  BluCfg nbest = blu_cfg_default(log2m);
  nbest.nat = 1;
  double nbest_us = 1e300;
  auto ntrial = [&](BluCfg c) {
    if (st2 || !blu_cfg_valid(log2m, c)) return;
    double us = 0.0;
    st2 = blu_time(p, b, c, st, e0, e1, &us);
    if (st2) return;
    if (us < nbest_us) {
      nbest = c;
      nbest_us = us;
    }
    if (us < best_us) {
      best = c;
      best_us = us;
    }
  };
  const BluCfg nstart = nbest;
  for (int l1 : {d, d - 1, d + 1}) {
    BluCfg c = nstart;
    c.l1 = l1;
    ntrial(c);
  }
  const BluCfg nsplit = nbest;
  for (int pc : {32, 16, 8}) {
    if (pc >= ntiles) continue;
    BluCfg c = nsplit;
    c.pchunk = pc;
    ntrial(c);
  }
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  if (st2) return st2;
  *out = best;
  *out_us = best_us;
  return IPFB_OK;
}

// All launches of one batched call on stream st.
hipError_t enqueue_batched(ipfb_bplan p, int infmt, const void* const* spec, const float* const* sc, double phi,
                           int normalise, void* const* xo, hipStream_t st) {
  const int N = p->lblock;
  const int K = N / 2 + 1;
  hipError_t e = hipSuccess;
  for (int s = 0; s < p->nstreams && e == hipSuccess; ++s) {
    const int64_t b = p->nblock[s];
    const BluTables& bt = p->blu[b];
    // power of two, or the natural-layout Bluestein path: rows straight into
    // the output, columns in place there; otherwise rows into f0 for the
    // transposed Bluestein path
    const bool in_place = bt.log2m == 0 || p->bcfg[bt.log2m].nat;
    void* rows_out = in_place ? xo[s] : p->f0;
    e = hipErrorNotSupported;
    if (infmt == IPFB_IN_C4) e = launch_row_c4(p->prec, p->log2n, spec[s], sc[s], rows_out, b, p->twN, st);
    if (e == hipErrorNotSupported) {
      hipGetLastError();
      e = hipSuccess;
      if (scaled_infmt(infmt)) e = launch_dequant_factors(p->prec, sc[s], K, N, p->fac, st);
      if (e == hipSuccess) e = launch_row_irfft(p->prec, p->log2n, infmt, spec[s], p->fac, rows_out, b, p->twN, st);
    }
    if (e != hipSuccess) break;
    if (bt.log2m == 0) {
      for (int pass = 0; pass < 3 && e == hipSuccess; ++pass)
        e = launch_col_wiener_nat(p->prec, ilog2(b), pass, xo[s], N, p->ntap, p->win64, phi, normalise, bt.twB,
                                  bt.twb64, st);
      continue;
    }
    const BluCfg& cfg = p->bcfg[bt.log2m];
    const void* tw4[4];
    blu_tw4(p, bt.log2m, cfg.l1, tw4);
    if (cfg.nat) {
      e = launch_blu_nat(p->prec, xo[s], p->Tm, bt.chirp, bt.Crow, bt.twb64, b, bt.log2m, cfg, N, p->ntap, p->win64,
                         phi, normalise, tw4, st);
      continue;
    }
    // Bluestein: d -> d_T in f1; Z in f0, A in f1 (d_T consumed by then), x_T in f0
    e = launch_transpose(p->prec, p->f0, p->f1, b, N, st);
    if (e != hipSuccess) break;
    e = launch_blu_columns(p->prec, p->f1, p->f0, p->Tm, p->f0, p->f1, bt.chirp, bt.Crow, bt.twb64, b, bt.log2m, cfg,
                           N, p->ntap, p->win64, phi, normalise, tw4, st);
    if (e == hipSuccess) e = launch_transpose(p->prec, p->f0, xo[s], N, b, st);  // x_T -> x (time order)
  }
  return e;
}

// The recursive column stage over every stream: rows of all streams (one
// multi-stream kernel for 4-bit spectra, else one launch per stream), then
// the segment passes of all streams together. The device tables must hold
// this call's pointers, and the coefficients this phi.
bool batched_recursive(ipfb_bplan p, double phi) {
  if (!p->rec_coef || !(phi >= kIirMinPhi) || p->col_method == IPFB_COLS_FFT) return false;
  return true;
}

hipError_t enqueue_batched_recursive(ipfb_bplan p, int infmt, const void* const* spec, const float* const* sc,
                                     double phi, int normalise, void* const* xo, hipStream_t st) {
  const int N = p->lblock;
  hipError_t e;
  {
    ProfScope ps("batched_rows", st);
    e = hipErrorNotSupported;
    if (infmt == IPFB_IN_C4)
      e = launch_row_c4(p->prec, p->log2n, nullptr, nullptr, nullptr, p->rec_frames, p->twN, st, p->row_tab,
                        p->nstreams);
    if (e == hipErrorNotSupported) {  // other formats and frame lengths: one launch per stream
      hipGetLastError();
      e = hipSuccess;
      for (int s = 0; s < p->nstreams && e == hipSuccess; ++s) {
        if (scaled_infmt(infmt)) e = launch_dequant_factors(p->prec, sc[s], N / 2 + 1, N, p->fac, st);
        if (e == hipSuccess)
          e = launch_row_irfft(p->prec, p->log2n, infmt, spec[s], p->fac, xo[s], p->nblock[s], p->twN, st);
      }
    }
  }
  static const char* const names[3] = {"batched_cols_rec_pass1", "batched_cols_rec_carry", "batched_cols_rec_pass2"};
  const IirStream none = {nullptr, 0, 0};
  for (int stage = kIirPass1; stage <= kIirApply && e == hipSuccess; ++stage) {
    ProfScope ps(names[stage - kIirPass1], st);
    e = launch_col_iir(stage, p->prec, none, p->rec_tab, p->nstreams, p->rec_nsegt, p->rec_maxnseg, N, p->ntap,
                       p->win64, phi, normalise ? 1.0 + phi * phi : 1.0, p->rec_coef, p->rec_scoef, p->rec_zs, st);
  }
  return e;
}

// Rewrites the multi-stream tables for these pointers (waits for the stream
// first: a graph launched earlier may still read them).
int batched_tables(ipfb_bplan p, const void* const* spec, const float* const* sc, void* const* xo, hipStream_t st) {
  std::vector<uintptr_t> key;
  for (int s = 0; s < p->nstreams; ++s) {
    key.push_back((uintptr_t)spec[s]);
    key.push_back((uintptr_t)(sc ? sc[s] : nullptr));
    key.push_back((uintptr_t)xo[s]);
  }
  if (key == p->rec_key) return IPFB_OK;
  const int seg = p->prec == IPFB_F32 ? kIirSegF32 : kIirSegF64;
  std::vector<IirStream> it(p->nstreams);
  std::vector<RowStream> rt(p->nstreams);
  int64_t g = 0, f = 0;
  for (int s = 0; s < p->nstreams; ++s) {
    it[s] = {xo[s], p->nblock[s], g};
    rt[s] = {(const unsigned char*)spec[s], sc ? sc[s] : nullptr, xo[s], p->nblock[s], f};
    g += (p->nblock[s] + seg - 1) / seg;
    f += p->nblock[s];
  }
  if (hipStreamSynchronize(st) != hipSuccess ||
      hipMemcpy(p->rec_tab, it.data(), it.size() * sizeof(IirStream), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(p->row_tab, rt.data(), rt.size() * sizeof(RowStream), hipMemcpyHostToDevice) != hipSuccess) {
    hipGetLastError();
    return fail(IPFB_EHIP, "writing the batched stream tables failed");
  }
  p->rec_key = key;
  return IPFB_OK;
}

}  // namespace

extern "C" {

int ipfb_batched_plan_create(ipfb_bplan* out, int lblock, int ntap, const double* window, int nstreams,
                             const int64_t* nblock, int prec) {
  if (!out) return fail(IPFB_EINVAL, "plan output pointer is NULL");
  *out = nullptr;
  if (!window || !nblock) return fail(IPFB_EINVAL, "window and nblock must be non-NULL host arrays");
  if (prec != IPFB_F32 && prec != IPFB_F64) return fail(IPFB_EINVAL, "prec must be IPFB_F32 or IPFB_F64");
  if (!is_pow2(lblock) || lblock < 4) return fail(IPFB_EINVAL, "lblock must be a power of two >= 4 (got %d)", lblock);
  if (ilog2(lblock) > max_log2_row(prec)) return fail(IPFB_EUNSUPPORTED, "lblock too large for the inverse");
  if (ntap < 1) return fail(IPFB_EINVAL, "ntap must be >= 1");
  if (nstreams < 1) return fail(IPFB_EINVAL, "nstreams must be >= 1");
  int64_t maxb = 0;
  for (int s = 0; s < nstreams; ++s) {
    if (nblock[s] < 2) return fail(IPFB_EINVAL, "stream %d: nblock must be >= 2", s);
    if (nblock[s] > 32768) return fail(IPFB_EUNSUPPORTED, "stream %d: nblock > 32768 is not supported", s);
    if (nblock[s] > maxb) maxb = nblock[s];
  }
  ipfb_bplan p = new ipfb_bplan_s();
  p->lblock = lblock;
  p->ntap = ntap;
  p->prec = prec;
  p->log2n = ilog2(lblock);
  p->nstreams = nstreams;
  p->nblock.assign(nblock, nblock + nstreams);
  if (hipGetDevice(&p->dev) != hipSuccess) {
    hipGetLastError();
    delete p;
    return fail(IPFB_EHIP, "no HIP device available");
  }
  const int64_t M = int64_t(1) << 20;
  int st = balloc(p, (void**)&p->win64, (size_t)ntap * lblock * sizeof(double));
  if (!st) st = upload(p->win64, window, (size_t)ntap * lblock * sizeof(double));
  if (!st) st = bupload(p, twiddles(lblock), prec, &p->twN);
  if (!st) st = balloc(p, &p->fac, (size_t)(lblock / 2 + 1) * esize(prec));
  int maxlog2m = 0;
  for (int s = 0; s < nstreams && !st; ++s)
    if (!p->blu.count(nblock[s])) {
      st = build_blu(p, nblock[s]);
      if (!st && p->blu[nblock[s]].log2m > maxlog2m) maxlog2m = p->blu[nblock[s]].log2m;
    }
  p->blu_maxb = maxb;
  const size_t fb = (size_t)maxb * lblock * esize(prec);
  if (!st) st = balloc(p, &p->f0, fb);
  if (!st) st = balloc(p, &p->f1, fb);
  if (!st && maxlog2m > 0) {  // whole tiles of column pairs cover at least (lblock + 1) / 2 pairs
    const int tp = blu_nat_tile_pairs(prec);
    const size_t pairs = (size_t)((lblock / 2 + tp - 1) / tp) * tp;
    const size_t np2 = pairs > (size_t)((lblock + 1) / 2) ? pairs : (size_t)((lblock + 1) / 2);
    st = balloc(p, &p->Tm, np2 * ((size_t)1 << maxlog2m) * 2 * esize(prec));
  }
  (void)M;
  if (!st && iir_coef_stride(ntap) > 0) {  // the recursive column stage over all streams
    const int seg = prec == IPFB_F32 ? kIirSegF32 : kIirSegF64;
    for (int s = 0; s < nstreams; ++s) {
      const int64_t ns = (nblock[s] + seg - 1) / seg;
      p->rec_nsegt += ns;
      p->rec_frames += nblock[s];
      if (ns > p->rec_maxnseg) p->rec_maxnseg = ns;
    }
    st = balloc(p, (void**)&p->rec_coef, (size_t)lblock * iir_coef_stride(ntap) * sizeof(double));
    if (!st) st = balloc(p, (void**)&p->rec_scoef, (size_t)nstreams * lblock * iir_stream_stride(ntap) * sizeof(double));
    if (!st) st = balloc(p, &p->rec_zs, (size_t)p->rec_nsegt * lblock * 2 * (ntap - 1) * esize(prec));
    if (!st) st = balloc(p, (void**)&p->rec_tab, (size_t)nstreams * sizeof(IirStream));
    if (!st) st = balloc(p, (void**)&p->row_tab, (size_t)nstreams * sizeof(RowStream));
    // prime the multi-stream row kernel's occupancy query outside any later graph capture
    if (!st && launch_row_c4(prec, p->log2n, nullptr, nullptr, nullptr, 0, nullptr, nullptr, p->row_tab, 0) !=
                   hipSuccess)
      hipGetLastError();
  }
  // shapes tuned earlier for this device and problem
  const char* cache = getenv("IPFB_TUNE_CACHE");
  if (!st && cache && *cache) st = tune_load(p, cache);
  // prime the row kernel's occupancy query outside any later graph capture
  if (!st && launch_row_c4(prec, p->log2n, nullptr, nullptr, nullptr, 0, nullptr, nullptr) != hipSuccess)
    hipGetLastError();
  if (!st && hipStreamCreateWithFlags(&p->cap, hipStreamNonBlocking) != hipSuccess) {
    hipGetLastError();
    st = fail(IPFB_EHIP, "hipStreamCreate failed");
  }
  if (st) {
    std::string keep = g_err;
    free_bplan(p);
    g_err = keep;
    return st;
  }
  *out = p;
  return ok();
}

int ipfb_batched_plan_destroy(ipfb_bplan p) {
  if (!p) return fail(IPFB_EINVAL, "plan is NULL");
  DeviceGuard g(p->dev);
  free_bplan(p);
  return ok();
}

int ipfb_batched_get_shape(ipfb_bplan p, int log2m, int shape[6]) {
  if (!p || !shape) return fail(IPFB_EINVAL, "NULL argument");
  auto it = p->bcfg.find(log2m);
  if (it == p->bcfg.end()) return fail(IPFB_EINVAL, "the plan has no stream of convolution length 2^%d", log2m);
  shape[0] = it->second.l1;
  shape[1] = it->second.mb;
  shape[2] = it->second.kb;
  shape[3] = it->second.pchunk;
  shape[4] = it->second.fuse;
  shape[5] = it->second.nat;
  return ok();
}

int ipfb_batched_set_shape(ipfb_bplan p, int log2m, const int shape[6]) {
  if (!p || !shape) return fail(IPFB_EINVAL, "NULL argument");
  if (!p->bcfg.count(log2m)) return fail(IPFB_EINVAL, "the plan has no stream of convolution length 2^%d", log2m);
  BluCfg c;
  c.l1 = shape[0];
  c.mb = shape[1];
  c.kb = shape[2];
  c.pchunk = shape[3];
  c.fuse = shape[4];
  c.nat = shape[5];
  DeviceGuard g(p->dev);
  int st = blu_apply_cfg(p, log2m, c);
  return st ? st : ok();
}

int ipfb_batched_tune(ipfb_bplan p, const char* cache_path, int force) {
  if (!p) return fail(IPFB_EINVAL, "plan is NULL");
  DeviceGuard g(p->dev);
  if (hipDeviceSynchronize() != hipSuccess) {
    hipGetLastError();
    return fail(IPFB_EHIP, "hipDeviceSynchronize failed");
  }
  std::string path = cache_path ? cache_path : "";
  if (path.empty()) {
    const char* env = getenv("IPFB_TUNE_CACHE");
    if (env) path = env;
  }
  std::map<std::string, TuneEntry> have;
  if (!path.empty() && !force && !tune_cache_read(path, have)) have.clear();  // unparsable: tune afresh
  std::map<std::string, TuneEntry> fresh;
  double total = 0.0;
  std::vector<int> lengths;
  for (auto& kv : p->bcfg) lengths.push_back(kv.first);
  if (!lengths.empty() && hipMemset(p->f0, 0, (size_t)p->blu_maxb * p->lblock * esize(p->prec)) != hipSuccess) {
    hipGetLastError();
    return fail(IPFB_EHIP, "hipMemset failed");
  }
  if (!lengths.empty() && hipMemset(p->f1, 0, (size_t)p->blu_maxb * p->lblock * esize(p->prec)) != hipSuccess) {
    hipGetLastError();
    return fail(IPFB_EHIP, "hipMemset failed");
  }
  for (int log2m : lengths) {
    const std::string key = tune_key(p, log2m);
    auto it = have.find(key);
    BluCfg c;
    double us = 0.0;
    if (it != have.end()) {
      c.l1 = it->second.l1;
      c.mb = it->second.mb;
      c.kb = it->second.kb;
      c.pchunk = it->second.pchunk;
      c.fuse = it->second.fuse;
      c.nat = it->second.nat;
      us = it->second.us;
    }
    if (it == have.end() || !blu_cfg_valid(log2m, c)) {
      int st = tune_length(p, log2m, &c, &us);
      if (st) return st;
      TuneEntry t;
      t.l1 = c.l1;
      t.mb = c.mb;
      t.kb = c.kb;
      t.pchunk = c.pchunk;
      t.fuse = c.fuse;
      t.nat = c.nat;
      t.us = us;
      fresh[key] = t;
    }
    int st = blu_apply_cfg(p, log2m, c);
    if (st) return st;
    total += us;
  }
  p->tuned_us = total;
  if (!path.empty() && !fresh.empty() && !tune_cache_write(path, fresh))
    return fail(IPFB_EINVAL, "cannot write the tune cache %s", path.c_str());
  return ok();
}

int ipfb_batched_workspace_size(ipfb_bplan p, size_t* bytes) {
  if (!p || !bytes) return fail(IPFB_EINVAL, "NULL argument");
  *bytes = p->bytes;
  return ok();
}

int ipfb_batched_set_column_method(ipfb_bplan p, int method) {
  if (!p) return fail(IPFB_EINVAL, "plan is NULL");
  if (method != IPFB_COLS_AUTO && method != IPFB_COLS_FFT && method != IPFB_COLS_RECURSIVE)
    return fail(IPFB_EINVAL, "unknown column method %d", method);
  if (method == IPFB_COLS_RECURSIVE && !p->rec_coef)
    return fail(IPFB_EUNSUPPORTED, "the recursive column stage needs ntap = 4 (ntap %d)", p->ntap);
  p->col_method = method;
  return ok();
}

int ipfb_batched_use_graph(ipfb_bplan p, int on) {
  if (!p) return fail(IPFB_EINVAL, "plan is NULL");
  p->use_graph = (on != 0);
  return ok();
}

int ipfb_wiener_batched(ipfb_bplan p, int infmt, const void* const* spec, const float* const* chan_scale,
                        double phi, int normalise, void* const* x_out, void* stream) {
  if (!p) return fail(IPFB_EINVAL, "plan is NULL");
  if (!spec || !x_out) return fail(IPFB_EINVAL, "spec and x_out must be non-NULL host arrays of device pointers");
  if (check_infmt(infmt, chan_scale)) return IPFB_EINVAL;
  if (!(phi >= 0.0) || !std::isfinite(phi)) return fail(IPFB_EINVAL, "phi must be finite and >= 0");
  for (int s = 0; s < p->nstreams; ++s) {
    if (!spec[s] || !x_out[s] || (scaled_infmt(infmt) && !chan_scale[s]))
      return fail(IPFB_EINVAL, "stream %d: NULL pointer", s);
  }
  DeviceGuard g(p->dev);
  hipStream_t st = (hipStream_t)stream;
  const bool rec = batched_recursive(p, phi);
  if (rec) {
    if (int s2 = batched_tables(p, spec, chan_scale, x_out, st)) return s2;
    if (!(phi == p->rec_phi)) {  // the coefficients for this phi, outside the graph
      const IirStream none = {nullptr, 0, 0};
      hipError_t e = hipSuccess;
      for (int stage = kIirSetup; stage <= kIirSetupLen && e == hipSuccess; ++stage) {
        ProfScope ps("batched_cols_rec_setup", st);
        e = launch_col_iir(stage, p->prec, none, p->rec_tab, p->nstreams, p->rec_nsegt, p->rec_maxnseg, p->lblock,
                           p->ntap, p->win64, phi, 1.0, p->rec_coef, p->rec_scoef, p->rec_zs, st);
      }
      p->rec_phi = e == hipSuccess ? phi : NAN;
      if (e != hipSuccess) return launched(e, "ipfb_wiener_batched");
    }
  }
  auto enqueue = [&](hipStream_t s) {
    return rec ? enqueue_batched_recursive(p, infmt, spec, chan_scale, phi, normalise, x_out, s)
               : enqueue_batched(p, infmt, spec, chan_scale, phi, normalise, x_out, s);
  };
  if (!p->use_graph) return launched(enqueue(st), "ipfb_wiener_batched");
  std::vector<uintptr_t> key;
  key.push_back((uintptr_t)rec);
  key.push_back((uintptr_t)infmt);
  key.push_back((uintptr_t)normalise);
  uint64_t phibits;
  memcpy(&phibits, &phi, sizeof(phibits));
  key.push_back((uintptr_t)phibits);
  for (int s = 0; s < p->nstreams; ++s) {
    key.push_back((uintptr_t)spec[s]);
    key.push_back((uintptr_t)(chan_scale ? chan_scale[s] : nullptr));
    key.push_back((uintptr_t)x_out[s]);
  }
  if (!p->exec || key != p->key) {
    if (p->exec) {
      hipGraphExecDestroy(p->exec);
      p->exec = nullptr;
    }
    hipError_t e = hipStreamBeginCapture(p->cap, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return launched(e, "hipStreamBeginCapture");
    hipError_t ee = enqueue(p->cap);
    hipGraph_t graph = nullptr;
    e = hipStreamEndCapture(p->cap, &graph);
    if (ee != hipSuccess) e = ee;
    if (e == hipSuccess) e = hipGraphInstantiate(&p->exec, graph, nullptr, nullptr, 0);
    if (graph) hipGraphDestroy(graph);
    if (e != hipSuccess) {
      p->exec = nullptr;
      return launched(e, "graph capture of the batched inverse");
    }
    p->key = key;
  }
  return launched(hipGraphLaunch(p->exec, st), "ipfb_wiener_batched");
}

}  // extern "C"
