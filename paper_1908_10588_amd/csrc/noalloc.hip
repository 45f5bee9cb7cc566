// H_eff,2 * theta (paper Section 2.1.2, eq. two-site Hamiltonian) for callers
// that cannot allocate device memory (code under HIP graph capture, tight
// serving loops): the four stages of tdmrg_heff2_apply -- L * theta GEMM,
// the W_i and W_{i+1} channel stages, the R GEMM -- on the same kernels, with
// the two contraction intermediates in a file-scope device array instead of
// the context's growable workspace.
//
// The array is a fixed part of the library's code object: every GPU the
// library is loaded on holds its own copy (kNoAllocScratchBytes) until the
// process ends.  Host code never passes the array's name to a kernel (on the
// host it is only a stand-in symbol); its device address is looked up once per
// device with hipGetSymbolAddress when a context is created on that device
// (noalloc_init) and that address is used everywhere.  Every call on a GPU
// shares the array, so calls that overlap on one GPU (several streams or host
// threads) race; the stages overwrite every element they read, so nothing has
// to be cleared between calls.
#include <algorithm>
#include <mutex>
#include <string>

#include "internal.h"

namespace tdmrg {

constexpr size_t kNoAllocScratchBytes = size_t(64) << 20;  // 64 MiB per GPU
constexpr int kNoAllocMaxDevices = 64;

static __device__ __align__(256) double scratch[kNoAllocScratchBytes / sizeof(double)];

static std::mutex g_scratch_mu;
static void* g_scratch_ptr[kNoAllocMaxDevices] = {};

// Device address of the scratch array on `device` (which must be current).
hipError_t noalloc_init(int device) {
  if (device < 0 || device >= kNoAllocMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_ptr[device]) return hipSuccess;
  void* ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return e;
  if (!ptr) return hipErrorInvalidSymbol;
  g_scratch_ptr[device] = ptr;
  return hipSuccess;
}

size_t noalloc_scratch_bytes() { return kNoAllocScratchBytes; }

static void* scratch_of(int device) {
  if (device < 0 || device >= kNoAllocMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  return g_scratch_ptr[device];
}

namespace {

GemmOperand opnd(const double* p, long im, long sr, long ld, int trans) {
  GemmOperand o;
  o.p = p;
  o.im = im;
  o.sb = 0;
  o.sr = sr;
  o.ld = ld;
  o.trans = trans;
  o.conj = 0;
  return o;
}

GemmArgs plain_gemm(int M, int N, int K, int nred, GemmOperand A, GemmOperand B, double* C, long c_im, long ldc) {
  GemmArgs g;
  g.M = M;
  g.N = N;
  g.K = K;
  g.nbatch = 1;
  g.nred = nred;
  g.role = 0;
  g.A = A;
  g.B = B;
  g.C = C;
  g.c_im = c_im;
  g.c_sb = 0;
  g.ldc = ldc;
  g.alpha_re = 1.0;
  g.alpha_im = 0.0;
  g.beta_re = 0.0;
  g.beta_im = 0.0;
  return g;
}

MixArgs channel_stage(const tdmrg_wop* W, const double* in, long in_im, double* out, long out_im, int P, int Q) {
  MixArgs a;
  a.in = in;
  a.in_im = in_im;
  a.out = out;
  a.out_im = out_im;
  a.P = P;
  a.Q = Q;
  a.din = W->d;
  a.dout = W->d;
  a.nout = W->wr;
  a.rowptr = W->f_rowptr;
  a.col = W->f_col;
  a.vre = W->f_v;
  a.vim = W->f_v + W->f_nnz;
  return a;
}

}  // namespace

// Doubles of scratch the product needs: X_a [2][max(wl, wr)][|theta|] and
// X_b [2][wc][|theta|].
double noalloc_heff2_doubles(const tdmrg_heff_shape& s) {
  const double th = (double)s.Dl * s.d1 * s.d2 * s.Dr;
  return 2.0 * ((double)std::max(s.wl, s.wr) + s.wc) * th;
}

tdmrg_status heff2_noalloc(tdmrg_ctx* ctx, const tdmrg_heff_shape& s, const double* L, const tdmrg_wop* W1,
                           const tdmrg_wop* W2, const double* R, const double* theta, double* y, Arith ar) {
  double* base = (double*)scratch_of(ctx->device);
  if (!base) return fail(ctx, TDMRG_EDEVICE, "the no-allocation scratch array has no device address on this GPU");
  const double need = noalloc_heff2_doubles(s);
  if (need * sizeof(double) > (double)kNoAllocScratchBytes)
    return fail(ctx, TDMRG_ESHAPE,
                "heff2_apply_noalloc: the intermediates need " + std::to_string((long long)(need * sizeof(double))) +
                    " bytes, more than the " + std::to_string(kNoAllocScratchBytes) + "-byte scratch array");
  const long th = (long)s.Dl * s.d1 * s.d2 * s.Dr;
  const int wmax = std::max(s.wl, s.wr);
  double* XA = base;
  double* XB = base + 2 * (long)wmax * th;
  hipStream_t st = ctx->stream;
  const int N1 = s.d1 * s.d2 * s.Dr;
  // X1[wl][a][s'][t'][b'] = sum_a' L[wl][a][a'] theta[a'][s'][t'][b']
  hipError_t e = launch_cgemm(plain_gemm(s.wl * s.Dl, N1, s.Dl, 1, opnd(L, (long)s.wl * s.Dl * s.Dl, 0, s.Dl, 0),
                                         opnd(theta, th, 0, N1, 0), XA, (long)s.wl * th, N1),
                              ar, st);
  // X2[wc][a][s][t'][b'] = sum_{wl,s'} W1[wl][wc][s][s'] X1[wl][a][s'][t'][b']
  if (e == hipSuccess)
    e = launch_mix(channel_stage(W1, XA, (long)s.wl * th, XB, (long)s.wc * th, s.Dl, s.d2 * s.Dr), st);
  // X3[wr][a][s][t][b'] = sum_{wc,t'} W2[wc][wr][t][t'] X2[wc][a][s][t'][b']
  if (e == hipSuccess)
    e = launch_mix(channel_stage(W2, XB, (long)s.wc * th, XA, (long)s.wr * th, s.Dl * s.d1, s.Dr), st);
  // y[a][s][t][b] = sum_{wr,b'} X3[wr][a][s][t][b'] R[wr][b][b']
  if (e == hipSuccess)
    e = launch_cgemm(plain_gemm(s.Dl * s.d1 * s.d2, s.Dr, s.Dr, s.wr, opnd(XA, (long)s.wr * th, th, s.Dr, 0),
                                opnd(R, (long)s.wr * s.Dr * s.Dr, (long)s.Dr * s.Dr, s.Dr, 1), y, th, s.Dr),
                     ar, st);
  if (e != hipSuccess) return fail(ctx, TDMRG_EDEVICE, std::string("heff2_apply_noalloc: ") + hipGetErrorString(e));
  return TDMRG_OK;
}

}  // namespace tdmrg
