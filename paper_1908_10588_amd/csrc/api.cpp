// The C ABI (include/tdmrg.h): argument validation, handle management, the
// 2TDVP sweep engine and the observables.
#include <rocsolver/rocsolver.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <string>
#include <vector>

#include "internal.h"

using namespace tdmrg;


static thread_local std::string g_create_err;

#define TRY_HIP(expr)                                                                            \
  do {                                                                                           \
    hipError_t e_ = (expr);                                                                      \
    if (e_ != hipSuccess)                                                                        \
      return fail(ctx, TDMRG_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_));        \
  } while (0)
#define TRY(expr)                  \
  do {                             \
    tdmrg_status s_ = (expr);      \
    if (s_ != TDMRG_OK) return s_; \
  } while (0)

static Arith arith_of(int prec) {
  switch (prec) {
    case TDMRG_FP32: return Arith::F32;
    case TDMRG_BF16X3: return Arith::BF16X3;
    case TDMRG_BF16X6: return Arith::BF16X6;
    default: return Arith::F64;
  }
}
static bool prec_ok(int prec) {
  return prec == TDMRG_FP64 || prec == TDMRG_FP32 || prec == TDMRG_BF16X3 || prec == TDMRG_BF16X6;
}

static tdmrg_status use_device(tdmrg_ctx* ctx) {
  TRY_HIP(hipSetDevice(ctx->device));
  return TDMRG_OK;
}

// ------------------------------------------------------------------ context
extern "C" tdmrg_status tdmrg_ctx_create(int device, void* hip_stream, void* arena, size_t arena_bytes,
                                         tdmrg_ctx** out) {
  if (!out) {
    g_create_err = "out is NULL";
    return TDMRG_EINVAL;
  }
  *out = nullptr;
  if ((arena == nullptr) != (arena_bytes == 0)) {
    g_create_err = "arena and arena_bytes must both be given or both be empty";
    return TDMRG_EINVAL;
  }
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || count <= 0) {
    g_create_err = "no HIP device available";
    return TDMRG_EDEVICE;
  }
  if (device < 0 || device >= count) {
    g_create_err = "device index out of range";
    return TDMRG_EINVAL;
  }
  if (hipSetDevice(device) != hipSuccess) {
    g_create_err = "hipSetDevice failed";
    return TDMRG_EDEVICE;
  }
  if (arena) {  // must be device memory of this GPU
    hipPointerAttribute_t at;
    if (hipPointerGetAttributes(&at, arena) != hipSuccess || at.type != hipMemoryTypeDevice || at.device != device) {
      (void)hipGetLastError();
      g_create_err = "the arena is not device memory of this GPU";
      return TDMRG_EINVAL;
    }
  }
  tdmrg_ctx* ctx = new tdmrg_ctx();
  ctx->device = device;
  ctx->stream = (hipStream_t)hip_stream;
  if (arena) {  // 256-byte aligned blocks from the first aligned address on
    const uintptr_t a = (uintptr_t)arena, al = (a + 255) & ~(uintptr_t)255;
    const size_t skip = (size_t)(al - a);
    if (arena_bytes > skip + 256) {
      ctx->arena.base = (char*)al;
      ctx->arena.bytes = (arena_bytes - skip) & ~(size_t)255;
      ctx->arena.free_blocks[0] = ctx->arena.bytes;
    } else {
      g_create_err = "arena smaller than one block";
      delete ctx;
      return TDMRG_EINVAL;
    }
  }
  // rocSOLVER runs inside the SVD; no atomics keeps its results (and the
  // whole step) bitwise reproducible
  if (rocblas_create_handle(&ctx->blas) != rocblas_status_success ||
      rocblas_set_stream(ctx->blas, ctx->stream) != rocblas_status_success ||
      rocblas_set_atomics_mode(ctx->blas, rocblas_atomics_not_allowed) != rocblas_status_success) {
    g_create_err = "rocblas handle creation failed";
    delete ctx;
    return TDMRG_EDEVICE;
  }
  {
    const hipError_t e = noalloc_init(device);
    if (e != hipSuccess) {
      g_create_err = std::string("scratch array lookup failed: ") + hipGetErrorString(e);
      rocblas_destroy_handle(ctx->blas);
      delete ctx;
      return TDMRG_EDEVICE;
    }
  }
  if (hipHostMalloc((void**)&ctx->host, 65536, hipHostMallocDefault) != hipSuccess) {
    g_create_err = "pinned host allocation failed";
    rocblas_destroy_handle(ctx->blas);
    delete ctx;
    return TDMRG_ENOMEM;
  }
  *out = ctx;
  return TDMRG_OK;
}

static void free_buf(tdmrg_ctx* ctx, DevBuf& b) {
  if (b.p) dev_free(ctx, b.p);
  b.p = nullptr;
  b.bytes = 0;
}

extern "C" void tdmrg_ctx_destroy(tdmrg_ctx* ctx) {
  if (!ctx) return;
  (void)hipSetDevice(ctx->device);
  (void)hipStreamSynchronize(ctx->stream);
  for (DevBuf* b : {&ctx->xa, &ctx->xb, &ctx->kry, &ctx->wvec, &ctx->theta, &ctx->svd_z, &ctx->svd_u,
                    &ctx->svd_vt, &ctx->svd_s, &ctx->svd_e, &ctx->envA, &ctx->envB, &ctx->small,
                    &ctx->meta, &ctx->batch, &ctx->bscal, &ctx->bpart, &ctx->vjpA, &ctx->vjpB,
                    &ctx->vjpC, &ctx->vjpD, &ctx->vjpL, &ctx->vjpR, &ctx->vjpU, &ctx->vjpV, &ctx->sub,
                    &ctx->adjw, &ctx->adjt, &ctx->kryU, &ctx->wvecU, &ctx->smallU, &ctx->splitk, &ctx->cqr, &ctx->qr, &ctx->gbuf, &ctx->gsmall, &ctx->hqr, &ctx->heev, &ctx->rocws})
    free_buf(ctx, *b);
  graphs_clear(ctx);
  if (ctx->cap_stream) (void)hipStreamDestroy(ctx->cap_stream);
  for (auto& kv : ctx->ident_ops) tdmrg_wop_destroy(kv.second);
  for (hipEvent_t e : ctx->tune_ev)
    if (e) (void)hipEventDestroy(e);
  if (ctx->host) (void)hipHostFree(ctx->host);
  if (ctx->blas) rocblas_destroy_handle(ctx->blas);
  prof_release(ctx);
  pair_release(ctx);
  delete ctx;
}

extern "C" tdmrg_status tdmrg_ctx_set_fusion(tdmrg_ctx* ctx, int mode) {
  if (!ctx) return TDMRG_EINVAL;
  if (mode < 0 || mode > 2) return fail(ctx, TDMRG_EINVAL, "fusion mode must be 0, 1 or 2");
  ctx->fuse_mode = mode;
  return TDMRG_OK;
}

extern "C" tdmrg_status tdmrg_ctx_set_channel_gemm(tdmrg_ctx* ctx, int mode) {
  if (!ctx) return TDMRG_EINVAL;
  if (mode < 0 || mode > 2) return fail(ctx, TDMRG_EINVAL, "channel GEMM mode must be 0, 1 or 2");
  ctx->chan_gemm = mode;
  return TDMRG_OK;
}

extern "C" tdmrg_status tdmrg_ctx_set_mix_in_gemm(tdmrg_ctx* ctx, int on) {
  if (!ctx) return TDMRG_EINVAL;
  ctx->mix_in_gemm = on ? 1 : 0;
  graph_epoch_bump();  // captured Lanczos steps hold the other launch sequence
  return TDMRG_OK;
}

extern "C" tdmrg_status tdmrg_ctx_set_autotune(tdmrg_ctx* ctx, int on) {
  if (!ctx) return TDMRG_EINVAL;
  ctx->autotune = on ? 1 : 0;
  return TDMRG_OK;
}

extern "C" tdmrg_status tdmrg_ctx_set_graphs(tdmrg_ctx* ctx, int on) {
  if (!ctx) return TDMRG_EINVAL;
  ctx->graphs = on ? 1 : 0;
  return TDMRG_OK;
}

extern "C" tdmrg_status tdmrg_ctx_graph_counters(const tdmrg_ctx* ctx, long* out) {
  if (!ctx || !out) return TDMRG_EINVAL;
  for (int i = 0; i < 3; ++i) out[i] = ctx->graph_counts[i];
  return TDMRG_OK;
}

extern "C" tdmrg_status tdmrg_ctx_set_verbose(tdmrg_ctx* ctx, int level) {
  if (!ctx || level < 0) return TDMRG_EINVAL;
  ctx->verbose = level;
  return TDMRG_OK;
}

extern "C" tdmrg_status tdmrg_ctx_tile_table(tdmrg_ctx* ctx, int cap, int* n, int* entries) {
  if (!ctx || !n) return TDMRG_EINVAL;
  *n = (int)ctx->tiles.size();
  if (!entries) return TDMRG_OK;
  int r = 0;
  for (const auto& kv : ctx->tiles) {
    if (r >= cap) break;
    for (int c = 0; c < 8; ++c) entries[9 * r + c] = kv.first[c];
    entries[9 * r + 8] = kv.second;
    ++r;
  }
  return TDMRG_OK;
}

extern "C" tdmrg_status tdmrg_ctx_set_svd_method(tdmrg_ctx* ctx, int method) {
  if (!ctx) return TDMRG_EINVAL;
  if (method < 0 || method > 3) return fail(ctx, TDMRG_EINVAL, "SVD method must be 0, 1, 2 or 3");
  ctx->svd_method = method;
  return TDMRG_OK;
}

extern "C" tdmrg_status tdmrg_ctx_set_eigensolver(tdmrg_ctx* ctx, int method) {
  if (!ctx) return TDMRG_EINVAL;
  if (method < 0 || method > 1) return fail(ctx, TDMRG_EINVAL, "eigensolver must be 0 or 1");
  ctx->eig_method = method;
  return TDMRG_OK;
}

extern "C" tdmrg_status tdmrg_ctx_set_svd_schedule(tdmrg_ctx* ctx, int schedule) {
  if (!ctx) return TDMRG_EINVAL;
  if (schedule < 0 || schedule > 1) return fail(ctx, TDMRG_EINVAL, "SVD schedule must be 0 or 1");
  ctx->svd_schedule = schedule;
  return TDMRG_OK;
}

extern "C" tdmrg_status tdmrg_ctx_svd_counters(tdmrg_ctx* ctx, long long out[8]) {
  if (!ctx || !out) return TDMRG_EINVAL;
  for (int k = 0; k < 8; ++k) out[k] = ctx->svd_count[k];
  return TDMRG_OK;
}

extern "C" tdmrg_status tdmrg_ctx_set_profiling(tdmrg_ctx* ctx, int on) {
  if (!ctx) return TDMRG_EINVAL;
  TRY(use_device(ctx));
  TRY_HIP(hipStreamSynchronize(ctx->stream));
  TRY(prof_flush(ctx));
  Profiler& P = ctx->prof;
  for (int k = 0; k < 4; ++k) {
    P.ms[k] = P.flops[k] = P.bytes[k] = 0.0;
    P.launches[k] = 0;
  }
  P.on = on != 0;
  return TDMRG_OK;
}

extern "C" tdmrg_status tdmrg_ctx_get_profile(tdmrg_ctx* ctx, tdmrg_profile* out) {
  if (!ctx || !out) return TDMRG_EINVAL;
  TRY(use_device(ctx));
  TRY_HIP(hipStreamSynchronize(ctx->stream));
  TRY(prof_flush(ctx));
  const Profiler& P = ctx->prof;
  for (int k = 0; k < 4; ++k) {
    out->ms[k] = P.ms[k];
    out->flops[k] = P.flops[k];
    out->bytes[k] = P.bytes[k];
    out->launches[k] = P.launches[k];
  }
  return TDMRG_OK;
}

extern "C" const char* tdmrg_last_error(const tdmrg_ctx* ctx) {
  return ctx ? ctx->err.c_str() : g_create_err.c_str();
}

extern "C" tdmrg_status tdmrg_ctx_synchronize(tdmrg_ctx* ctx) {
  if (!ctx) return TDMRG_EINVAL;
  TRY(use_device(ctx));
  TRY_HIP(hipStreamSynchronize(ctx->stream));
  return TDMRG_OK;
}

extern "C" tdmrg_status tdmrg_ctx_workspace_bytes(const tdmrg_ctx* ctx, size_t* bytes) {
  if (!ctx || !bytes) return TDMRG_EINVAL;
  size_t t = 0;
  for (const DevBuf* b : {&ctx->xa, &ctx->xb, &ctx->kry, &ctx->wvec, &ctx->theta, &ctx->svd_z,
                          &ctx->svd_u, &ctx->svd_vt, &ctx->svd_s, &ctx->svd_e, &ctx->envA,
                          &ctx->envB, &ctx->small, &ctx->meta, &ctx->batch, &ctx->bscal, &ctx->bpart,
                          &ctx->vjpA, &ctx->vjpB, &ctx->vjpC, &ctx->vjpD, &ctx->vjpL, &ctx->vjpR, &ctx->vjpU,
                          &ctx->vjpV, &ctx->sub, &ctx->adjw, &ctx->adjt, &ctx->kryU, &ctx->wvecU,
                          &ctx->smallU, &ctx->splitk, &ctx->cqr, &ctx->qr, &ctx->gbuf, &ctx->gsmall, &ctx->hqr,
                          &ctx->heev})
    t += b->bytes;
  *bytes = t;
  return TDMRG_OK;
}

extern "C" tdmrg_status tdmrg_ctx_set_batch_budget(tdmrg_ctx* ctx, size_t bytes) {
  if (!ctx) return TDMRG_EINVAL;
  ctx->batch_budget = bytes;
  return TDMRG_OK;
}

static tdmrg_status check_shape(tdmrg_ctx* ctx, const tdmrg_heff_shape* s, bool two);
static tdmrg_status check_wops(tdmrg_ctx* ctx, const tdmrg_heff_shape* s, const tdmrg_wop* W1,
                               const tdmrg_wop* W2, bool two);

static tdmrg_status check_batch(tdmrg_ctx* ctx, int n, const tdmrg_heff_shape* shapes, const double* const* L,
                                const tdmrg_wop* const* W1, const tdmrg_wop* const* W2,
                                const double* const* R, const void* const* x, const void* const* y) {
  if (n < 0 || (n > 0 && (!shapes || !L || !W1 || !W2 || !R || !x)))
    return fail(ctx, TDMRG_EINVAL, "invalid batch arrays");
  for (int p = 0; p < n; ++p) {
    TRY(check_shape(ctx, &shapes[p], true));
    TRY(check_wops(ctx, &shapes[p], W1[p], W2[p], true));
    if (!L[p] || !R[p] || !x[p] || (y && !y[p])) return fail(ctx, TDMRG_EINVAL, "tensor pointer is NULL");
  }
  return TDMRG_OK;
}

extern "C" tdmrg_status tdmrg_heff2_apply_batched(tdmrg_ctx* ctx, int n, const tdmrg_heff_shape* shapes,
                                                  const double* const* L, const tdmrg_wop* const* W1,
                                                  const tdmrg_wop* const* W2, const double* const* R,
                                                  const double* const* theta, double* const* y,
                                                  tdmrg_precision prec) {
  if (!ctx) return TDMRG_EINVAL;
  TRY(check_batch(ctx, n, shapes, L, W1, W2, R, (const void* const*)theta, (const void* const*)y));
  if (!prec_ok(prec)) return fail(ctx, TDMRG_EUNSUPPORTED, "unknown precision");
  if (n == 0) return TDMRG_OK;
  TRY(use_device(ctx));
  return heff2_batched(ctx, n, shapes, L, W1, W2, R, theta, y, arith_of(prec));
}

extern "C" tdmrg_status tdmrg_local_expm_batched(tdmrg_ctx* ctx, int n, const tdmrg_heff_shape* shapes,
                                                 const double* const* L, const tdmrg_wop* const* W1,
                                                 const tdmrg_wop* const* W2, const double* const* R,
                                                 double* const* theta_inout, double tau, double tol,
                                                 int m_max, tdmrg_precision prec, int* iters) {
  if (!ctx) return TDMRG_EINVAL;
  TRY(check_batch(ctx, n, shapes, L, W1, W2, R, (const void* const*)theta_inout, nullptr));
  if (!std::isfinite(tau) || !(tol >= 0.0) || m_max < 1 || m_max > 64)
    return fail(ctx, TDMRG_EINVAL, "invalid tau, tol or m_max");
  if (!prec_ok(prec)) return fail(ctx, TDMRG_EUNSUPPORTED, "unknown precision");
  if (n == 0) return TDMRG_OK;
  TRY(use_device(ctx));
  int nonconv = 0;
  TRY(local_expm_batched(ctx, n, shapes, L, W1, W2, R, theta_inout, tau, tol, m_max, arith_of(prec), iters,
                         &nonconv));
  return nonconv ? fail(ctx, TDMRG_ENOCONV, "some Lanczos exponentials missed the tolerance") : TDMRG_OK;
}

// --------------------------------------------------------------- operators
static tdmrg_status upload(tdmrg_ctx* ctx, void** dst, const void* src, size_t bytes) {
  *dst = nullptr;
  if (hipMalloc(dst, bytes ? bytes : 8) != hipSuccess) return fail(ctx, TDMRG_ENOMEM, "device allocation failed");
  if (src && bytes) TRY_HIP(hipMemcpy(*dst, src, bytes, hipMemcpyHostToDevice));
  return TDMRG_OK;
}

tdmrg_status tdmrg::wop_make(tdmrg_ctx* ctx, int wl, int wr, int d, const double* planar,
                             tdmrg_wop** out) {
  static long next_id = 0;
  tdmrg_wop* w = new tdmrg_wop();
  w->ctx = ctx;
  w->id = ++next_id;
  w->wl = wl;
  w->wr = wr;
  w->d = d;
  const size_t blk = (size_t)d * d;
  const size_t tot = (size_t)wl * wr * blk;
  w->host.assign(planar, planar + 2 * tot);
  auto at = [&](int a, int b, int s, int sp, int part) {
    return planar[part * tot + ((size_t)a * wr + b) * blk + (size_t)s * d + sp];
  };
  // forward CSR over rows (c < wr, s)
  std::vector<int> rp, col;
  std::vector<double> vr, vi;
  rp.push_back(0);
  for (int c = 0; c < wr; ++c)
    for (int s = 0; s < d; ++s) {
      for (int a = 0; a < wl; ++a)
        for (int sp = 0; sp < d; ++sp) {
          const double x = at(a, c, s, sp, 0), y = at(a, c, s, sp, 1);
          if (x != 0.0 || y != 0.0) {
            col.push_back(a * d + sp);
            vr.push_back(x);
            vi.push_back(y);
          }
        }
      rp.push_back((int)col.size());
    }
  w->f_nnz = (int)col.size();
  std::vector<double> v(vr);
  v.insert(v.end(), vi.begin(), vi.end());
  tdmrg_status st;
  if ((st = upload(ctx, (void**)&w->f_rowptr, rp.data(), rp.size() * sizeof(int))) ||
      (st = upload(ctx, (void**)&w->f_col, col.data(), col.size() * sizeof(int))) ||
      (st = upload(ctx, (void**)&w->f_v, v.data(), v.size() * sizeof(double)))) {
    tdmrg_wop_destroy(w);
    return st;
  }
  // row blocks of the forward CSR for the multi-row channel kernel
  {
    HostBlocks hb;
    build_mix_blocks(wr * d, rp.data(), col.data(), vr.data(), vi.data(), &hb);
    w->f_blk.ncols = (long)hb.bcol.size();
    if ((st = upload(ctx, (void**)&w->f_blk.bptr, hb.bptr.data(), hb.bptr.size() * sizeof(int))) ||
        (st = upload(ctx, (void**)&w->f_blk.bcol, hb.bcol.data(), hb.bcol.size() * sizeof(int))) ||
        (st = upload(ctx, (void**)&w->f_blk.bval, hb.bval.data(), hb.bval.size() * sizeof(double))) ||
        (st = upload(ctx, (void**)&w->f_blk.bmask, hb.bmask.data(), hb.bmask.size() * sizeof(unsigned)))) {
      tdmrg_wop_destroy(w);
      return st;
    }
  }
  // backward CSR over rows (c < wl, s)
  rp.clear(); col.clear(); vr.clear(); vi.clear();
  rp.push_back(0);
  for (int c = 0; c < wl; ++c)
    for (int s = 0; s < d; ++s) {
      for (int b = 0; b < wr; ++b)
        for (int sp = 0; sp < d; ++sp) {
          const double x = at(c, b, s, sp, 0), y = at(c, b, s, sp, 1);
          if (x != 0.0 || y != 0.0) {
            col.push_back(b * d + sp);
            vr.push_back(x);
            vi.push_back(y);
          }
        }
      rp.push_back((int)col.size());
    }
  w->b_nnz = (int)col.size();
  v = vr;
  v.insert(v.end(), vi.begin(), vi.end());
  if ((st = upload(ctx, (void**)&w->b_rowptr, rp.data(), rp.size() * sizeof(int))) ||
      (st = upload(ctx, (void**)&w->b_col, col.data(), col.size() * sizeof(int))) ||
      (st = upload(ctx, (void**)&w->b_v, v.data(), v.size() * sizeof(double)))) {
    tdmrg_wop_destroy(w);
    return st;
  }
  *out = w;
  return TDMRG_OK;
}

extern "C" tdmrg_status tdmrg_wop_create(tdmrg_ctx* ctx, int wl, int wr, int d,
                                         const double* planar_host, tdmrg_wop** out) {
  if (!ctx || !out) return TDMRG_EINVAL;
  *out = nullptr;
  if (wl < 1 || wr < 1 || d < 1 || !planar_host) return fail(ctx, TDMRG_EINVAL, "invalid operator shape or data");
  const size_t tot = 2 * (size_t)wl * wr * d * d;
  for (size_t k = 0; k < tot; ++k)
    if (!std::isfinite(planar_host[k])) return fail(ctx, TDMRG_EINVAL, "operator is not finite");
  TRY(use_device(ctx));
  return wop_make(ctx, wl, wr, d, planar_host, out);
}

tdmrg_status tdmrg::wop_adjoint(tdmrg_ctx* ctx, const tdmrg_wop* W, const tdmrg_wop** out) {
  if (!W->adj) {
    const int wl = W->wl, wr = W->wr, d = W->d;
    const size_t blk = (size_t)d * d, tot = (size_t)wl * wr * blk;
    std::vector<double> h(2 * tot);
    for (size_t b = 0; b < (size_t)wl * wr; ++b)
      for (int s = 0; s < d; ++s)
        for (int sp = 0; sp < d; ++sp) {
          const size_t src = b * blk + (size_t)sp * d + s, dst = b * blk + (size_t)s * d + sp;
          h[dst] = W->host[src];
          h[tot + dst] = -W->host[tot + src];
        }
    tdmrg_wop* a = nullptr;
    TRY(wop_make(ctx, wl, wr, d, h.data(), &a));
    const_cast<tdmrg_wop*>(W)->adj = a;
  }
  *out = W->adj;
  return TDMRG_OK;
}

tdmrg_status tdmrg::wop_dense(tdmrg_ctx* ctx, const tdmrg_wop* W, int right, const double** out) {
  double* const* have = right ? &W->dense_r : &W->dense_l;
  if (!*have) {
    const int wl = W->wl, wr = W->wr, d = W->d;
    const size_t rows = (size_t)wr * d, cols = (size_t)wl * d, n = rows * cols;
    std::vector<double> h(2 * n);
    const size_t tot = (size_t)wl * wr * d * d;
    for (int w = 0; w < wl; ++w)
      for (int c = 0; c < wr; ++c)
        for (int s = 0; s < d; ++s)
          for (int sp = 0; sp < d; ++sp) {
            const size_t src = (((size_t)w * wr + c) * d + s) * d + sp;
            const size_t row = right ? (size_t)c * d + s : (size_t)s * wr + c;
            const size_t dst = row * cols + (size_t)w * d + sp;
            h[dst] = W->host[src];
            h[n + dst] = W->host[tot + src];
          }
    double* dev = nullptr;
    if (hipMalloc((void**)&dev, sizeof(double) * 2 * n) != hipSuccess)
      return fail(ctx, TDMRG_ENOMEM, "device allocation of a dense operator form failed");
    if (hipMemcpy(dev, h.data(), sizeof(double) * 2 * n, hipMemcpyHostToDevice) != hipSuccess) {
      (void)hipFree(dev);
      return fail(ctx, TDMRG_EDEVICE, "upload of a dense operator form failed");
    }
    *const_cast<double**>(have) = dev;
  }
  *out = *have;
  return TDMRG_OK;
}

extern "C" void tdmrg_wop_destroy(tdmrg_wop* w) {
  if (!w) return;
  tdmrg::graph_epoch_bump();
  if (w->adj) tdmrg_wop_destroy(w->adj);
  for (void* p : {(void*)w->f_rowptr, (void*)w->f_col, (void*)w->f_v, (void*)w->b_rowptr,
                  (void*)w->b_col, (void*)w->b_v, (void*)w->dense_l, (void*)w->dense_r, (void*)w->f_blk.bptr,
                  (void*)w->f_blk.bcol, (void*)w->f_blk.bval, (void*)w->f_blk.bmask})
    if (p) (void)hipFree(p);
  delete w;
}

extern "C" tdmrg_status tdmrg_wop_nnz(const tdmrg_wop* w, long* nnz) {
  if (!w || !nnz) return TDMRG_EINVAL;
  *nnz = w->f_nnz;
  return TDMRG_OK;
}

// --------------------------------------------------------------------- MPO
extern "C" void tdmrg_mpo_destroy(tdmrg_mpo* mpo) {
  if (!mpo) return;
  for (auto v : {&mpo->W, &mpo->ident, &mpo->proj})
    for (tdmrg_wop* w : *v) tdmrg_wop_destroy(w);
  for (double* p : mpo->dense)
    if (p) (void)hipFree(p);
  delete mpo;
}

extern "C" tdmrg_status tdmrg_mpo_build(tdmrg_ctx* ctx, const tdmrg_model* model, tdmrg_mpo** out) {
  return tdmrg::mpo_build(ctx, model, false, out);
}

tdmrg_status tdmrg::mpo_build(tdmrg_ctx* ctx, const tdmrg_model* model, bool keep_zero, tdmrg_mpo** out) {
  if (!ctx || !out) return TDMRG_EINVAL;
  *out = nullptr;
  TRY(validate_model(ctx, model));
  TRY(use_device(ctx));
  std::vector<int> dims, wd;
  std::vector<std::vector<double>> W;
  std::vector<int> el;
  TRY(build_mpo_host(ctx, model, &dims, &wd, &W, &el, keep_zero));
  tdmrg_mpo* mpo = new tdmrg_mpo();
  mpo->ctx = ctx;
  mpo->n = (int)dims.size();
  mpo->n_el = model->n_el;
  mpo->pop_site = el;
  mpo->dims = dims;
  mpo->wdims = wd;
  for (int s = 0; s < mpo->n; ++s) {
    tdmrg_wop* w = nullptr;
    tdmrg_status st = wop_make(ctx, wd[s], wd[s + 1], dims[s], W[s].data(), &w);
    if (st != TDMRG_OK) {
      tdmrg_mpo_destroy(mpo);
      return st;
    }
    mpo->W.push_back(w);
    double* dev = nullptr;
    if (hipMalloc((void**)&dev, sizeof(double) * W[s].size()) != hipSuccess ||
        hipMemcpy(dev, W[s].data(), sizeof(double) * W[s].size(), hipMemcpyHostToDevice) != hipSuccess) {
      if (dev) (void)hipFree(dev);
      tdmrg_mpo_destroy(mpo);
      return fail(ctx, TDMRG_ENOMEM, "upload of the dense MPO failed");
    }
    mpo->dense.push_back(dev);
    // w = 1 identity for norms and overlaps
    std::vector<double> id(2 * (size_t)dims[s] * dims[s], 0.0);
    for (int k = 0; k < dims[s]; ++k) id[(size_t)k * dims[s] + k] = 1.0;
    st = wop_make(ctx, 1, 1, dims[s], id.data(), &w);
    if (st != TDMRG_OK) {
      tdmrg_mpo_destroy(mpo);
      return st;
    }
    mpo->ident.push_back(w);
  }
  for (int i = 0; i < model->n_el; ++i) {
    // |i><i| on the electronic site, or n_i = |1><1| on the site of state i
    const int d = dims[el[i]], k = model->el_per_state ? 1 : i;
    std::vector<double> pr(2 * (size_t)d * d, 0.0);
    pr[(size_t)k * d + k] = 1.0;
    tdmrg_wop* w = nullptr;
    tdmrg_status st = wop_make(ctx, 1, 1, d, pr.data(), &w);
    if (st != TDMRG_OK) {
      tdmrg_mpo_destroy(mpo);
      return st;
    }
    mpo->proj.push_back(w);
  }
  *out = mpo;
  return TDMRG_OK;
}

extern "C" tdmrg_status tdmrg_mpo_host_query(const tdmrg_model* model, int* n_sites, int* dims,
                                             int* wdims) {
  TRY(validate_model(nullptr, model));
  std::vector<int> d, wd;
  std::vector<std::vector<double>> W;
  std::vector<int> el;
  TRY(build_mpo_host(nullptr, model, &d, &wd, &W, &el));
  if (n_sites) *n_sites = (int)d.size();
  if (dims) std::copy(d.begin(), d.end(), dims);
  if (wdims) std::copy(wd.begin(), wd.end(), wdims);
  return TDMRG_OK;
}

static int sat_mul(long a, long b, int cap);

extern "C" tdmrg_status tdmrg_workspace_query(const tdmrg_model* model, int D_max, int krylov_max,
                                              tdmrg_precision precision, size_t* bytes) {
  if (!bytes) return TDMRG_EINVAL;
  if (D_max < 1 || krylov_max < 1 || krylov_max > 64 || !prec_ok(precision)) return TDMRG_EINVAL;
  TRY(validate_model(nullptr, model));
  std::vector<int> d, wd;
  std::vector<std::vector<double>> W;
  std::vector<int> el;
  TRY(build_mpo_host(nullptr, model, &d, &wd, &W, &el));
  // bond capacities of an MPS created with D_cap = D_max (tdmrg_mps_init)
  const int n = (int)d.size();
  std::vector<int> left(n + 1, 1), right(n + 1, 1), caps(n + 1);
  for (int b = 1; b <= n; ++b) left[b] = sat_mul(left[b - 1], d[b - 1], D_max);
  for (int b = n - 1; b >= 0; --b) right[b] = sat_mul(right[b + 1], d[b], D_max);
  for (int b = 0; b <= n; ++b) caps[b] = std::max(1, std::min({left[b], right[b], D_max}));
  // the default channel-stage choice of a context (fusion by the cost model)
  *bytes = plan_sweep(d, wd, caps, krylov_max, W, 1).total();
  return TDMRG_OK;
}

extern "C" tdmrg_status tdmrg_mpo_host_site(const tdmrg_model* model, int site, double* planar_host) {
  TRY(validate_model(nullptr, model));
  std::vector<int> d, wd;
  std::vector<std::vector<double>> W;
  std::vector<int> el;
  TRY(build_mpo_host(nullptr, model, &d, &wd, &W, &el));
  if (site < 0 || site >= (int)d.size() || !planar_host) return TDMRG_EINVAL;
  std::copy(W[site].begin(), W[site].end(), planar_host);
  return TDMRG_OK;
}

extern "C" tdmrg_status tdmrg_mpo_info(const tdmrg_mpo* mpo, int* n_sites, int* dims, int* wdims) {
  if (!mpo) return TDMRG_EINVAL;
  if (n_sites) *n_sites = mpo->n;
  if (dims) std::copy(mpo->dims.begin(), mpo->dims.end(), dims);
  if (wdims) std::copy(mpo->wdims.begin(), mpo->wdims.end(), wdims);
  return TDMRG_OK;
}

extern "C" tdmrg_status tdmrg_mpo_get_site(const tdmrg_mpo* mpo, int site, double* planar_host) {
  if (!mpo || !planar_host || site < 0 || site >= mpo->n) return TDMRG_EINVAL;
  const std::vector<double>& h = mpo->W[site]->host;
  std::copy(h.begin(), h.end(), planar_host);
  return TDMRG_OK;
}

extern "C" const tdmrg_wop* tdmrg_mpo_site(const tdmrg_mpo* mpo, int site) {
  if (!mpo || site < 0 || site >= mpo->n) return nullptr;
  return mpo->W[site];
}

// --------------------------------------------------------------------- MPS
static int sat_mul(long a, long b, int cap) {
  const long r = a * b;
  return (int)std::min<long>(r, cap);
}

extern "C" void tdmrg_mps_destroy(tdmrg_mps* mps) {
  if (!mps) return;
  tdmrg::graph_epoch_bump();
  for (auto v : {&mps->site, &mps->L, &mps->R})
    for (double* p : *v)
      if (p) (void)hipFree(p);
  delete mps;
}

static tdmrg_status mps_alloc(tdmrg_ctx* ctx, const std::vector<int>& dims, int D_cap,
                              tdmrg_mps** out) {
  tdmrg_mps* m = new tdmrg_mps();
  m->ctx = ctx;
  m->n = (int)dims.size();
  m->dims = dims;
  const int n = m->n;
  // full-rank bound min(prod left dims, prod right dims), capped at D_cap
  std::vector<int> left(n + 1, 1), right(n + 1, 1);
  for (int b = 1; b <= n; ++b) left[b] = sat_mul(left[b - 1], dims[b - 1], D_cap);
  for (int b = n - 1; b >= 0; --b) right[b] = sat_mul(right[b + 1], dims[b], D_cap);
  m->cap.resize(n + 1);
  for (int b = 0; b <= n; ++b) m->cap[b] = std::max(1, std::min({left[b], right[b], D_cap}));
  m->bond.assign(n + 1, 1);
  m->site.assign(n, nullptr);
  for (int s = 0; s < n; ++s) {
    const size_t bytes = sizeof(double) * 2 * (size_t)m->cap[s] * dims[s] * m->cap[s + 1];
    if (hipMalloc((void**)&m->site[s], bytes) != hipSuccess) {
      tdmrg_mps_destroy(m);
      return fail(ctx, TDMRG_ENOMEM, "MPS allocation failed");
    }
  }
  *out = m;
  return TDMRG_OK;
}

extern "C" tdmrg_status tdmrg_mps_init(tdmrg_ctx* ctx, const tdmrg_mpo* mpo, const int* occ, int D_cap,
                                       tdmrg_mps** out) {
  if (!ctx || !out) return TDMRG_EINVAL;
  *out = nullptr;
  if (!mpo || !occ) return fail(ctx, TDMRG_EINVAL, "mpo or occ is NULL");
  if (D_cap < 1) return fail(ctx, TDMRG_EINVAL, "D_cap must be >= 1");
  for (int s = 0; s < mpo->n; ++s)
    if (occ[s] < 0 || occ[s] >= mpo->dims[s]) return fail(ctx, TDMRG_EINVAL, "occupation out of range");
  TRY(use_device(ctx));
  tdmrg_mps* m = nullptr;
  TRY(mps_alloc(ctx, mpo->dims, D_cap, &m));
  for (int s = 0; s < m->n; ++s) {
    std::vector<double> h(2 * (size_t)m->dims[s], 0.0);
    h[occ[s]] = 1.0;
    if (hipMemcpy(m->site[s], h.data(), h.size() * sizeof(double), hipMemcpyHostToDevice) != hipSuccess) {
      tdmrg_mps_destroy(m);
      return fail(ctx, TDMRG_EDEVICE, "upload of the product state failed");
    }
  }
  *out = m;
  return TDMRG_OK;
}

extern "C" tdmrg_status tdmrg_mps_copy(const tdmrg_mps* src, tdmrg_mps** out) {
  if (!src || !out) return TDMRG_EINVAL;
  tdmrg_ctx* ctx = src->ctx;
  TRY(use_device(ctx));
  tdmrg_mps* m = nullptr;
  TRY(mps_alloc(ctx, src->dims, src->cap.empty() ? 1 : *std::max_element(src->cap.begin(), src->cap.end()), &m));
  m->cap = src->cap;
  m->bond = src->bond;
  for (int s = 0; s < m->n; ++s) {
    const size_t bytes = sizeof(double) * 2 * (size_t)src->bond[s] * src->dims[s] * src->bond[s + 1];
    if (hipMemcpyAsync(m->site[s], src->site[s], bytes, hipMemcpyDeviceToDevice, ctx->stream) != hipSuccess) {
      tdmrg_mps_destroy(m);
      return fail(ctx, TDMRG_EDEVICE, "MPS copy failed");
    }
  }
  if (hipStreamSynchronize(ctx->stream) != hipSuccess) {
    tdmrg_mps_destroy(m);
    return fail(ctx, TDMRG_EDEVICE, "MPS copy failed");
  }
  *out = m;
  return TDMRG_OK;
}

extern "C" tdmrg_status tdmrg_mps_bond_dims(const tdmrg_mps* mps, int* bonds) {
  if (!mps || !bonds) return TDMRG_EINVAL;
  std::copy(mps->bond.begin(), mps->bond.end(), bonds);
  return TDMRG_OK;
}

extern "C" tdmrg_status tdmrg_mps_set_site(tdmrg_mps* mps, int site, int Dl, int Dr, const double* planar_host) {
  if (!mps) return TDMRG_EINVAL;
  tdmrg_ctx* ctx = mps->ctx;
  if (site < 0 || site >= mps->n || !planar_host) return fail(ctx, TDMRG_EINVAL, "bad site or data");
  if (Dl < 1 || Dr < 1 || Dl > mps->cap[site] || Dr > mps->cap[site + 1])
    return fail(ctx, TDMRG_ESHAPE, "bond dimension exceeds the MPS capacity");
  if ((site == 0 && Dl != 1) || (site == mps->n - 1 && Dr != 1))
    return fail(ctx, TDMRG_ESHAPE, "boundary bonds must be 1");
  const size_t cnt = 2 * (size_t)Dl * mps->dims[site] * Dr;
  for (size_t k = 0; k < cnt; ++k)
    if (!std::isfinite(planar_host[k])) return fail(ctx, TDMRG_EINVAL, "site tensor is not finite");
  TRY(use_device(ctx));
  TRY_HIP(hipStreamSynchronize(ctx->stream));
  TRY_HIP(hipMemcpy(mps->site[site], planar_host, cnt * sizeof(double), hipMemcpyHostToDevice));
  mps->bond[site] = Dl;
  mps->bond[site + 1] = Dr;
  mps->env_valid = false;
  return TDMRG_OK;
}

extern "C" tdmrg_status tdmrg_mps_get_site(const tdmrg_mps* mps, int site, int* Dl, int* d, int* Dr,
                                           double* planar_host) {
  if (!mps || site < 0 || site >= mps->n) return TDMRG_EINVAL;
  tdmrg_ctx* ctx = mps->ctx;
  if (Dl) *Dl = mps->bond[site];
  if (d) *d = mps->dims[site];
  if (Dr) *Dr = mps->bond[site + 1];
  if (planar_host) {
    TRY(use_device(ctx));
    TRY_HIP(hipStreamSynchronize(ctx->stream));
    const size_t cnt = 2 * (size_t)mps->bond[site] * mps->dims[site] * mps->bond[site + 1];
    TRY_HIP(hipMemcpy(planar_host, mps->site[site], cnt * sizeof(double), hipMemcpyDeviceToHost));
  }
  return TDMRG_OK;
}

// ---------------------------------------------------------- single steps
static tdmrg_status check_shape(tdmrg_ctx* ctx, const tdmrg_heff_shape* s, bool two) {
  if (!s) return fail(ctx, TDMRG_EINVAL, "shape is NULL");
  if (s->Dl < 1 || s->d1 < 1 || s->Dr < 1 || s->wl < 1 || s->wr < 1 ||
      (two && (s->d2 < 1 || s->wc < 1)))
    return fail(ctx, TDMRG_EINVAL, "shape entries must be >= 1");
  const double el = (double)s->Dl * s->d1 * (two ? s->d2 : 1) * s->Dr;
  if (el * std::max({s->wl, s->wc, s->wr}) > 4.0e9)
    return fail(ctx, TDMRG_EUNSUPPORTED, "problem exceeds 32-bit intermediate indexing");
  return TDMRG_OK;
}

static tdmrg_status check_wops(tdmrg_ctx* ctx, const tdmrg_heff_shape* s, const tdmrg_wop* W1,
                               const tdmrg_wop* W2, bool two) {
  if (!W1 || (two && !W2)) return fail(ctx, TDMRG_EINVAL, "operator is NULL");
  if (two) {
    if (W1->wl != s->wl || W1->wr != s->wc || W1->d != s->d1 || W2->wl != s->wc || W2->wr != s->wr ||
        W2->d != s->d2)
      return fail(ctx, TDMRG_ESHAPE, "operators do not match the shape");
  } else if (W1->wl != s->wl || W1->wr != s->wr || W1->d != s->d1) {
    return fail(ctx, TDMRG_ESHAPE, "operator does not match the shape");
  }
  return TDMRG_OK;
}

extern "C" tdmrg_status tdmrg_heff2_apply(tdmrg_ctx* ctx, const tdmrg_heff_shape* shape, const double* L,
                                          const tdmrg_wop* W1, const tdmrg_wop* W2, const double* R,
                                          const double* theta, double* y, tdmrg_precision prec) {
  if (!ctx) return TDMRG_EINVAL;
  TRY(check_shape(ctx, shape, true));
  TRY(check_wops(ctx, shape, W1, W2, true));
  if (!L || !R || !theta || !y) return fail(ctx, TDMRG_EINVAL, "tensor pointer is NULL");
  if (!prec_ok(prec)) return fail(ctx, TDMRG_EUNSUPPORTED, "unknown precision");
  TRY(use_device(ctx));
  return heff2(ctx, *shape, L, W1, W2, R, theta, y, arith_of(prec));
}

extern "C" tdmrg_status tdmrg_heff2_apply_noalloc(tdmrg_ctx* ctx, const tdmrg_heff_shape* shape, const double* L,
                                                  const tdmrg_wop* W1, const tdmrg_wop* W2, const double* R,
                                                  const double* theta, double* y, tdmrg_precision prec) {
  if (!ctx) return TDMRG_EINVAL;
  TRY(check_shape(ctx, shape, true));
  TRY(check_wops(ctx, shape, W1, W2, true));
  if (!L || !R || !theta || !y) return fail(ctx, TDMRG_EINVAL, "tensor pointer is NULL");
  if (!prec_ok(prec)) return fail(ctx, TDMRG_EUNSUPPORTED, "unknown precision");
  TRY(use_device(ctx));
  return heff2_noalloc(ctx, *shape, L, W1, W2, R, theta, y, arith_of(prec));
}

extern "C" tdmrg_status tdmrg_heff1_apply(tdmrg_ctx* ctx, const tdmrg_heff_shape* shape, const double* L,
                                          const tdmrg_wop* W, const double* R, const double* M,
                                          double* y, tdmrg_precision prec) {
  if (!ctx) return TDMRG_EINVAL;
  TRY(check_shape(ctx, shape, false));
  TRY(check_wops(ctx, shape, W, nullptr, false));
  if (!L || !R || !M || !y) return fail(ctx, TDMRG_EINVAL, "tensor pointer is NULL");
  if (!prec_ok(prec)) return fail(ctx, TDMRG_EUNSUPPORTED, "unknown precision");
  TRY(use_device(ctx));
  return heff1(ctx, shape->Dl, shape->d1, shape->Dr, L, W, R, M, y, arith_of(prec));
}

extern "C" tdmrg_status tdmrg_local_expm(tdmrg_ctx* ctx, const tdmrg_heff_shape* shape, int two_site,
                                         const double* L, const tdmrg_wop* W1, const tdmrg_wop* W2,
                                         const double* R, double* theta_inout, double tau, double tol,
                                         int m_max, tdmrg_precision prec, int* iters) {
  if (!ctx) return TDMRG_EINVAL;
  TRY(check_shape(ctx, shape, two_site != 0));
  TRY(check_wops(ctx, shape, W1, W2, two_site != 0));
  if (!L || !R || !theta_inout) return fail(ctx, TDMRG_EINVAL, "tensor pointer is NULL");
  if (!std::isfinite(tau) || !(tol >= 0.0) || m_max < 1 || m_max > 64)
    return fail(ctx, TDMRG_EINVAL, "invalid tau, tol or m_max");
  if (!prec_ok(prec)) return fail(ctx, TDMRG_EUNSUPPORTED, "unknown precision");
  TRY(use_device(ctx));
  ExpmResult r;
  TRY(local_expm(ctx, *shape, two_site != 0, L, W1, W2, R, theta_inout, tau, tol, m_max, arith_of(prec), &r));
  if (iters) *iters = r.iters;
  return r.converged ? TDMRG_OK : fail(ctx, TDMRG_ENOCONV, "Lanczos tolerance not reached");
}

extern "C" tdmrg_status tdmrg_heff2_apply_vjp(tdmrg_ctx* ctx, const tdmrg_heff_shape* shape, const double* L,
                                              const tdmrg_wop* W1, const tdmrg_wop* W2, const double* R,
                                              const double* theta, const double* ybar, double* Lbar,
                                              double* W1bar, double* W2bar, double* Rbar, double* thetabar) {
  if (!ctx) return TDMRG_EINVAL;
  TRY(check_shape(ctx, shape, true));
  TRY(check_wops(ctx, shape, W1, W2, true));
  if (!L || !R || !theta || !ybar) return fail(ctx, TDMRG_EINVAL, "tensor pointer is NULL");
  TRY(use_device(ctx));
  return heff2_vjp(ctx, *shape, L, W1, W2, R, theta, ybar, Lbar, W1bar, W2bar, Rbar, thetabar, false);
}

extern "C" tdmrg_status tdmrg_local_expm_vjp(tdmrg_ctx* ctx, const tdmrg_heff_shape* shape, const double* L,
                                             const tdmrg_wop* W1, const tdmrg_wop* W2, const double* R,
                                             const double* theta_in, double tau, const double* ybar,
                                             double* Lbar, double* W1bar, double* W2bar, double* Rbar,
                                             double* thetabar, int nquad, double tol, int m_max) {
  if (!ctx) return TDMRG_EINVAL;
  TRY(check_shape(ctx, shape, true));
  TRY(check_wops(ctx, shape, W1, W2, true));
  if (!L || !R || !theta_in || !ybar) return fail(ctx, TDMRG_EINVAL, "tensor pointer is NULL");
  if (!std::isfinite(tau) || nquad < 1 || nquad > 64 || !(tol >= 0.0) || m_max < 1 || m_max > 64)
    return fail(ctx, TDMRG_EINVAL, "invalid tau, nquad, tol or m_max");
  TRY(use_device(ctx));
  return local_expm2_vjp(ctx, *shape, L, W1, W2, R, theta_in, tau, ybar, Lbar, W1bar, W2bar, Rbar, thetabar,
                         nquad, tol, m_max, false);
}

extern "C" tdmrg_status tdmrg_heff0_apply(tdmrg_ctx* ctx, int Dl, int Dr, int w, const double* L, const double* R,
                                          const double* C, double* y, tdmrg_precision prec) {
  if (!ctx) return TDMRG_EINVAL;
  if (Dl < 1 || Dr < 1 || w < 1) return fail(ctx, TDMRG_EINVAL, "shape entries must be >= 1");
  if ((double)Dl * Dr * w > 4.0e9) return fail(ctx, TDMRG_EUNSUPPORTED, "problem exceeds 32-bit intermediate indexing");
  if (!L || !R || !C || !y) return fail(ctx, TDMRG_EINVAL, "tensor pointer is NULL");
  if (!prec_ok(prec)) return fail(ctx, TDMRG_EUNSUPPORTED, "unknown precision");
  TRY(use_device(ctx));
  return heff0(ctx, Dl, Dr, w, L, R, C, y, arith_of(prec));
}

extern "C" tdmrg_status tdmrg_local_expm0(tdmrg_ctx* ctx, int Dl, int Dr, int w, const double* L, const double* R,
                                          double* C_inout, double tau, double tol, int m_max, tdmrg_precision prec,
                                          int* iters) {
  if (!ctx) return TDMRG_EINVAL;
  if (Dl < 1 || Dr < 1 || w < 1) return fail(ctx, TDMRG_EINVAL, "shape entries must be >= 1");
  if ((double)Dl * Dr * w > 4.0e9) return fail(ctx, TDMRG_EUNSUPPORTED, "problem exceeds 32-bit intermediate indexing");
  if (!L || !R || !C_inout) return fail(ctx, TDMRG_EINVAL, "tensor pointer is NULL");
  if (!std::isfinite(tau) || !(tol >= 0.0) || m_max < 1 || m_max > 64)
    return fail(ctx, TDMRG_EINVAL, "invalid tau, tol or m_max");
  if (!prec_ok(prec)) return fail(ctx, TDMRG_EUNSUPPORTED, "unknown precision");
  TRY(use_device(ctx));
  ExpmResult r;
  TRY(local_expm0(ctx, Dl, Dr, w, L, R, C_inout, tau, tol, m_max, arith_of(prec), &r));
  if (iters) *iters = r.iters;
  return r.converged ? TDMRG_OK : fail(ctx, TDMRG_ENOCONV, "Lanczos tolerance not reached");
}

extern "C" tdmrg_status tdmrg_qr_split(tdmrg_ctx* ctx, int rows, int cols, const double* M, int right, double* Q,
                                       double* C, int* cholesky_ok) {
  if (!ctx) return TDMRG_EINVAL;
  if (rows < 1 || cols < 1 || !M || !Q || !C) return fail(ctx, TDMRG_EINVAL, "invalid qr_split arguments");
  if (right ? rows > cols : cols > rows)
    return fail(ctx, TDMRG_ESHAPE, "qr_split: the bond side must not exceed the other side");
  if (M == Q || M == C || Q == C) return fail(ctx, TDMRG_EINVAL, "qr_split: buffers must not alias");
  TRY(use_device(ctx));
  bool ok = false;
  TRY(qr_split(ctx, rows, cols, M, right != 0, Q, C, &ok));
  if (cholesky_ok) *cholesky_ok = ok ? 1 : 0;
  return TDMRG_OK;
}

extern "C" tdmrg_status tdmrg_theta_form(tdmrg_ctx* ctx, int Dl, int d1, int Dm, int d2, int Dr,
                                         const double* M, const double* B, double* theta) {
  if (!ctx) return TDMRG_EINVAL;
  if (Dl < 1 || d1 < 1 || Dm < 1 || d2 < 1 || Dr < 1 || !M || !B || !theta)
    return fail(ctx, TDMRG_EINVAL, "invalid theta_form arguments");
  TRY(use_device(ctx));
  return theta_form(ctx, Dl, d1, Dm, d2, Dr, M, B, theta);
}

extern "C" tdmrg_status tdmrg_svd_truncate(tdmrg_ctx* ctx, int Dl, int d1, int d2, int Dr,
                                           const double* theta, double eps, int D_max, int sv_mode,
                                           double tie_rel, int k_cap, double* U, double* S, double* Vh,
                                           int* k, double* disc) {
  if (!ctx) return TDMRG_EINVAL;
  if (Dl < 1 || d1 < 1 || d2 < 1 || Dr < 1 || !theta || !k || !disc || D_max < 1 || k_cap < 1 ||
      !(eps >= 0.0) || sv_mode < 0 || sv_mode > 2 || !(tie_rel >= 0.0) || tie_rel >= 1.0)
    return fail(ctx, TDMRG_EINVAL, "invalid svd_truncate arguments");
  TRY(use_device(ctx));
  if (!U || !S || !Vh) return fail(ctx, TDMRG_EINVAL, "U, S and Vh are required");
  return svd_truncate(ctx, Dl * d1, d2 * Dr, theta, eps, D_max, sv_mode, tie_rel, k_cap, 0, U, Vh, S, k, disc);
}

static tdmrg_status wop_env_check(tdmrg_ctx* ctx, int Dl, int d, int Dr, const tdmrg_wop* W, const double* a,
                                  const double* b, const double* c) {
  if (Dl < 1 || d < 1 || Dr < 1 || !W || !a || !b || !c) return fail(ctx, TDMRG_EINVAL, "invalid env arguments");
  if (W->d != d) return fail(ctx, TDMRG_ESHAPE, "operator dimension does not match");
  return TDMRG_OK;
}

extern "C" tdmrg_status tdmrg_env_update_left(tdmrg_ctx* ctx, int Dl, int d, int Dr, const double* Lin,
                                              const tdmrg_wop* W, const double* A, double* Lout,
                                              tdmrg_precision prec) {
  if (!ctx) return TDMRG_EINVAL;
  TRY(wop_env_check(ctx, Dl, d, Dr, W, Lin, A, Lout));
  if (!prec_ok(prec)) return fail(ctx, TDMRG_EUNSUPPORTED, "unknown precision");
  TRY(use_device(ctx));
  return env_left(ctx, Lin, W, A, Dl, Dr, A, Dl, Dr, Lout, arith_of(prec));
}

extern "C" tdmrg_status tdmrg_env_update_right(tdmrg_ctx* ctx, int Dl, int d, int Dr, const double* Rin,
                                               const tdmrg_wop* W, const double* B, double* Rout,
                                               tdmrg_precision prec) {
  if (!ctx) return TDMRG_EINVAL;
  TRY(wop_env_check(ctx, Dl, d, Dr, W, Rin, B, Rout));
  if (!prec_ok(prec)) return fail(ctx, TDMRG_EUNSUPPORTED, "unknown precision");
  TRY(use_device(ctx));
  return env_right(ctx, Rin, W, B, Dl, Dr, B, Dl, Dr, Rout, arith_of(prec));
}

// ------------------------------------------------------------------ sweep
static const double kOne[2] = {1.0, 0.0};

tdmrg_status tdmrg::ensure_envs(tdmrg_ctx* ctx, tdmrg_mps* mps, const tdmrg_mpo* mpo) {
  const int n = mps->n;
  if (mps->env_mpo != mpo || mps->L.size() != (size_t)(n + 1)) {
    for (auto v : {&mps->L, &mps->R})
      for (double* p : *v)
        if (p) (void)hipFree(p);
    mps->L.assign(n + 1, nullptr);
    mps->R.assign(n + 1, nullptr);
    for (int b = 0; b <= n; ++b) {
      const size_t bytes = sizeof(double) * 2 * (size_t)mpo->wdims[b] * mps->cap[b] * mps->cap[b];
      if (hipMalloc((void**)&mps->L[b], bytes) != hipSuccess || hipMalloc((void**)&mps->R[b], bytes) != hipSuccess)
        return fail(ctx, TDMRG_ENOMEM, "environment allocation failed");
    }
    mps->env_mpo = mpo;
    mps->env_valid = false;
  }
  if (!mps->env_valid) {
    TRY_HIP(hipMemcpyAsync(mps->L[0], kOne, 2 * sizeof(double), hipMemcpyHostToDevice, ctx->stream));
    TRY_HIP(hipMemcpyAsync(mps->R[n], kOne, 2 * sizeof(double), hipMemcpyHostToDevice, ctx->stream));
    for (int i = n - 1; i >= 1; --i) {
      const int Dl = mps->bond[i], Dr = mps->bond[i + 1];
      TRY(env_right(ctx, mps->R[i + 1], mpo->W[i], mps->site[i], Dl, Dr, mps->site[i], Dl, Dr, mps->R[i],
                    Arith::F64));
    }
    TRY_HIP(hipStreamSynchronize(ctx->stream));
    mps->env_valid = true;
  }
  return TDMRG_OK;
}

extern "C" tdmrg_status tdmrg_tdvp2_sweep(tdmrg_ctx* ctx, tdmrg_mps* mps, const tdmrg_mpo* mpo, double dt_fs,
                                          int D_max, double eps, const tdmrg_opts* opts,
                                          tdmrg_step_stats* stats) {
  if (!ctx) return TDMRG_EINVAL;
  if (!mps || !mpo) return fail(ctx, TDMRG_EINVAL, "mps or mpo is NULL");
  if (mps->n != mpo->n || mps->dims != mpo->dims) return fail(ctx, TDMRG_ESHAPE, "mps and mpo do not match");
  if (mps->n < 2) return fail(ctx, TDMRG_ESHAPE, "need at least two sites");
  if (!std::isfinite(dt_fs) || !(eps >= 0.0) || D_max < 1) return fail(ctx, TDMRG_EINVAL, "invalid dt, eps or D_max");
  tdmrg_opts o{TDMRG_FP64, 1e-12, 40, 0, 1e-12};
  if (opts) o = *opts;
  if (!prec_ok(o.precision) || o.krylov_max < 1 || o.krylov_max > 64 || !(o.krylov_tol >= 0.0) ||
      o.sv_mode < 0 || o.sv_mode > 2 || !(o.tie_rel >= 0.0) || o.tie_rel >= 1.0)
    return fail(ctx, TDMRG_EINVAL, "invalid options");
  TRY(use_device(ctx));
  TRY(reserve_sweep(ctx, mps, mpo, o.krylov_max));
  TRY(ensure_envs(ctx, mps, mpo));
  const Arith ar = arith_of(o.precision);
  const int n = mps->n;
  const double tau = dt_fs / (2.0 * TDMRG_HBAR_EV_FS);
  // two-site tensor buffer at the largest pair this MPS can hold
  size_t thmax = 0;
  for (int i = 0; i + 1 < n; ++i)
    thmax = std::max(thmax, (size_t)mps->cap[i] * mps->dims[i] * mps->dims[i + 1] * mps->cap[i + 2]);
  TRY(ensure(ctx, ctx->theta, sizeof(double) * 2 * thmax));
  double* theta = (double*)ctx->theta.p;
  tdmrg_step_stats st{};
  using clk = std::chrono::steady_clock;
  auto secs = [](clk::time_point a, clk::time_point b) { return std::chrono::duration<double>(b - a).count(); };
  int nonconv = 0;
  auto expm = [&](const tdmrg_heff_shape& s, bool two, const double* L, const tdmrg_wop* W1,
                  const tdmrg_wop* W2, const double* R, double* x, double t, int slot) -> tdmrg_status {
    auto t0 = clk::now();
    ExpmResult r;
    TRY(local_expm(ctx, s, two, L, W1, W2, R, x, t, o.krylov_tol, o.krylov_max, ar, &r));
    st.total_krylov += r.iters;
    st.max_krylov = std::max(st.max_krylov, r.iters);
    if (!r.converged) ++nonconv;
    st.seconds[slot] += secs(t0, clk::now());
    return TDMRG_OK;
  };
  auto add_disc = [&](double d) {
    st.sum_disc += d;
    st.max_disc = std::max(st.max_disc, d);
  };
  // ---- left -> right
  for (int i = 0; i + 1 < n; ++i) {
    const int Dl = mps->bond[i], Dm = mps->bond[i + 1], Dr = mps->bond[i + 2];
    const int d1 = mps->dims[i], d2 = mps->dims[i + 1];
    TRY(theta_form(ctx, Dl, d1, Dm, d2, Dr, mps->site[i], mps->site[i + 1], theta));
    tdmrg_heff_shape s{Dl, d1, d2, Dr, mpo->wdims[i], mpo->wdims[i + 1], mpo->wdims[i + 2]};
    TRY(expm(s, true, mps->L[i], mpo->W[i], mpo->W[i + 1], mps->R[i + 2], theta, tau, 0));
    auto t0 = clk::now();
    int k = 0;
    double disc = 0.0;
    TRY(svd_truncate(ctx, Dl * d1, d2 * Dr, theta, eps, std::min(D_max, mps->cap[i + 1]), o.sv_mode, o.tie_rel,
                     mps->cap[i + 1], 1, mps->site[i], mps->site[i + 1], nullptr, &k, &disc));
    st.seconds[1] += secs(t0, clk::now());
    add_disc(disc);
    mps->bond[i + 1] = k;
    t0 = clk::now();
    TRY(env_left(ctx, mps->L[i], mpo->W[i], mps->site[i], Dl, k, mps->site[i], Dl, k, mps->L[i + 1], ar));
    st.seconds[2] += secs(t0, clk::now());
    if (i + 2 < n) {
      tdmrg_heff_shape s1{k, d2, 1, Dr, mpo->wdims[i + 1], 1, mpo->wdims[i + 2]};
      TRY(expm(s1, false, mps->L[i + 1], mpo->W[i + 1], nullptr, mps->R[i + 2], mps->site[i + 1], -tau, 3));
    }
  }
  // ---- right -> left
  for (int i = n - 2; i >= 0; --i) {
    const int Dl = mps->bond[i], Dm = mps->bond[i + 1], Dr = mps->bond[i + 2];
    const int d1 = mps->dims[i], d2 = mps->dims[i + 1];
    TRY(theta_form(ctx, Dl, d1, Dm, d2, Dr, mps->site[i], mps->site[i + 1], theta));
    tdmrg_heff_shape s{Dl, d1, d2, Dr, mpo->wdims[i], mpo->wdims[i + 1], mpo->wdims[i + 2]};
    TRY(expm(s, true, mps->L[i], mpo->W[i], mpo->W[i + 1], mps->R[i + 2], theta, tau, 0));
    auto t0 = clk::now();
    int k = 0;
    double disc = 0.0;
    TRY(svd_truncate(ctx, Dl * d1, d2 * Dr, theta, eps, std::min(D_max, mps->cap[i + 1]), o.sv_mode, o.tie_rel,
                     mps->cap[i + 1], 2, mps->site[i], mps->site[i + 1], nullptr, &k, &disc));
    st.seconds[1] += secs(t0, clk::now());
    add_disc(disc);
    mps->bond[i + 1] = k;
    t0 = clk::now();
    TRY(env_right(ctx, mps->R[i + 2], mpo->W[i + 1], mps->site[i + 1], k, Dr, mps->site[i + 1], k, Dr,
                  mps->R[i + 1], ar));
    st.seconds[2] += secs(t0, clk::now());
    if (i > 0) {
      tdmrg_heff_shape s1{Dl, d1, 1, k, mpo->wdims[i], 1, mpo->wdims[i + 1]};
      TRY(expm(s1, false, mps->L[i], mpo->W[i], nullptr, mps->R[i + 1], mps->site[i], -tau, 3));
    }
  }
  TRY_HIP(hipStreamSynchronize(ctx->stream));
  st.not_converged = nonconv;
  if (stats) *stats = st;
  return nonconv ? fail(ctx, TDMRG_ENOCONV, "some local exponentials missed the Lanczos tolerance") : TDMRG_OK;
}

extern "C" tdmrg_status tdmrg_tdvp1_sweep(tdmrg_ctx* ctx, tdmrg_mps* mps, const tdmrg_mpo* mpo, double dt_fs,
                                          const tdmrg_opts* opts, tdmrg_step_stats* stats) {
  if (!ctx) return TDMRG_EINVAL;
  if (!mps || !mpo) return fail(ctx, TDMRG_EINVAL, "mps or mpo is NULL");
  if (mps->n != mpo->n || mps->dims != mpo->dims) return fail(ctx, TDMRG_ESHAPE, "mps and mpo do not match");
  if (mps->n < 2) return fail(ctx, TDMRG_ESHAPE, "need at least two sites");
  if (!std::isfinite(dt_fs)) return fail(ctx, TDMRG_EINVAL, "invalid dt");
  tdmrg_opts o{TDMRG_FP64, 1e-12, 40, 0, 1e-12};
  if (opts) o = *opts;
  if (!prec_ok(o.precision) || o.krylov_max < 1 || o.krylov_max > 64 || !(o.krylov_tol >= 0.0))
    return fail(ctx, TDMRG_EINVAL, "invalid options");
  const int n = mps->n;
  // the bonds stay as they are: each must fit the block it is split from
  for (int b = 1; b < n; ++b)
    if ((long)mps->bond[b] > (long)mps->bond[b - 1] * mps->dims[b - 1] ||
        (long)mps->bond[b] > (long)mps->dims[b] * mps->bond[b + 1])
      return fail(ctx, TDMRG_ESHAPE, "bond " + std::to_string(b) + " exceeds the block on one of its sides");
  TRY(use_device(ctx));
  TRY(ensure_envs(ctx, mps, mpo));
  const Arith ar = arith_of(o.precision);
  const double tau = dt_fs / (2.0 * TDMRG_HBAR_EV_FS);
  size_t smax = 0, bmax = 0;
  for (int i = 0; i < n; ++i) {
    smax = std::max(smax, (size_t)mps->bond[i] * mps->dims[i] * mps->bond[i + 1]);
    bmax = std::max(bmax, (size_t)mps->bond[i + 1] * mps->bond[i + 1]);
  }
  // product of the bond matrix with the next site | orthonormal factor | bond matrix
  TRY(ensure(ctx, ctx->theta, sizeof(double) * 2 * (2 * smax + bmax)));
  double* P = (double*)ctx->theta.p;
  double* Q = P + 2 * smax;
  double* C = Q + 2 * smax;
  hipStream_t st = ctx->stream;
  tdmrg_step_stats sts{};
  using clk = std::chrono::steady_clock;
  auto secs = [](clk::time_point a, clk::time_point b) { return std::chrono::duration<double>(b - a).count(); };
  int nonconv = 0;
  auto note = [&](const ExpmResult& r) {
    sts.total_krylov += r.iters;
    sts.max_krylov = std::max(sts.max_krylov, r.iters);
    if (!r.converged) ++nonconv;
  };
  auto forward = [&](int i) -> tdmrg_status {  // M_i = exp(-i tau H_eff,1) M_i
    auto t0 = clk::now();
    const tdmrg_heff_shape s1{mps->bond[i], mps->dims[i], 1, mps->bond[i + 1], mpo->wdims[i], 1, mpo->wdims[i + 1]};
    ExpmResult r;
    TRY(local_expm(ctx, s1, false, mps->L[i], mpo->W[i], nullptr, mps->R[i + 1], mps->site[i], tau, o.krylov_tol,
                   o.krylov_max, ar, &r));
    note(r);
    sts.seconds[0] += secs(t0, clk::now());
    return TDMRG_OK;
  };
  auto backward = [&](int b) -> tdmrg_status {  // C = exp(+i tau H_eff,0) C on bond b
    auto t0 = clk::now();
    ExpmResult r;
    TRY(local_expm0(ctx, mps->bond[b], mps->bond[b], mpo->wdims[b], mps->L[b], mps->R[b], C, -tau, o.krylov_tol,
                    o.krylov_max, ar, &r));
    note(r);
    sts.seconds[3] += secs(t0, clk::now());
    return TDMRG_OK;
  };
  auto split = [&](int i, bool right) -> tdmrg_status {  // site i = Q, bond matrix into C
    auto t0 = clk::now();
    const int Dl = mps->bond[i], d = mps->dims[i], Dr = mps->bond[i + 1];
    bool ok = true;
    TRY(right ? qr_split(ctx, Dl, d * Dr, mps->site[i], true, Q, C, &ok)
              : qr_split(ctx, Dl * d, Dr, mps->site[i], false, Q, C, &ok));
    if (!ok) ctx->svd_count[7]++;
    TRY_HIP(hipMemcpyAsync(mps->site[i], Q, sizeof(double) * 2 * (size_t)Dl * d * Dr, hipMemcpyDeviceToDevice, st));
    sts.seconds[1] += secs(t0, clk::now());
    return TDMRG_OK;
  };
  // ---- left -> right
  for (int i = 0; i < n; ++i) {
    TRY(forward(i));
    if (i + 1 == n) break;
    const int Dl = mps->bond[i], Dr = mps->bond[i + 1];
    TRY(split(i, false));
    auto t0 = clk::now();
    TRY(env_left(ctx, mps->L[i], mpo->W[i], mps->site[i], Dl, Dr, mps->site[i], Dl, Dr, mps->L[i + 1], ar));
    sts.seconds[2] += secs(t0, clk::now());
    TRY(backward(i + 1));
    // M_{i+1} = C M_{i+1}
    const int d2 = mps->dims[i + 1], Dr2 = mps->bond[i + 2];
    TRY(theta_form(ctx, Dr, 1, Dr, d2, Dr2, C, mps->site[i + 1], P));
    TRY_HIP(hipMemcpyAsync(mps->site[i + 1], P, sizeof(double) * 2 * (size_t)Dr * d2 * Dr2, hipMemcpyDeviceToDevice,
                           st));
  }
  // ---- right -> left
  for (int i = n - 1; i >= 0; --i) {
    TRY(forward(i));
    if (i == 0) break;
    const int Dl = mps->bond[i], Dr = mps->bond[i + 1];
    TRY(split(i, true));
    auto t0 = clk::now();
    TRY(env_right(ctx, mps->R[i + 1], mpo->W[i], mps->site[i], Dl, Dr, mps->site[i], Dl, Dr, mps->R[i], ar));
    sts.seconds[2] += secs(t0, clk::now());
    TRY(backward(i));
    // M_{i-1} = M_{i-1} C
    const int Dl0 = mps->bond[i - 1], d0 = mps->dims[i - 1];
    TRY(theta_form(ctx, Dl0, d0, Dl, 1, Dl, mps->site[i - 1], C, P));
    TRY_HIP(hipMemcpyAsync(mps->site[i - 1], P, sizeof(double) * 2 * (size_t)Dl0 * d0 * Dl, hipMemcpyDeviceToDevice,
                           st));
  }
  TRY_HIP(hipStreamSynchronize(st));
  sts.not_converged = nonconv;
  if (stats) *stats = sts;
  return nonconv ? fail(ctx, TDMRG_ENOCONV, "some local exponentials missed the Lanczos tolerance") : TDMRG_OK;
}

extern "C" tdmrg_status tdmrg_spectrum(tdmrg_ctx* ctx, int n_t, double dt_fs, const double* C, double tau_fs,
                                       int n_E, const double* E, double* sigma) {
  if (!ctx) return TDMRG_EINVAL;
  if (n_t < 2 || n_E < 1 || !C || !E || !sigma) return fail(ctx, TDMRG_EINVAL, "invalid spectrum arguments");
  if (!(dt_fs > 0.0) || !std::isfinite(dt_fs) || !(tau_fs > 0.0))
    return fail(ctx, TDMRG_EINVAL, "dt and tau must be positive");
  TRY(use_device(ctx));
  TRY_HIP(launch_spectrum(C, n_t, dt_fs, tau_fs, TDMRG_HBAR_EV_FS, E, n_E, sigma, ctx->stream));
  return TDMRG_OK;
}

// ------------------------------------------------------------ observables
// <bra| O |ket> for an MPO O given per site (w = 1 operators or the full MPO)
static tdmrg_status contract_chain(tdmrg_ctx* ctx, const tdmrg_mps* bra, const tdmrg_mps* ket,
                                   const std::vector<const tdmrg_wop*>& ops, double* re, double* im) {
  const int n = ket->n;
  size_t need = 2;
  for (int b = 0; b <= n; ++b)
    need = std::max(need, 2 * (size_t)(b == 0 ? 1 : ops[b - 1]->wr) * bra->bond[b] * ket->bond[b]);
  TRY(ensure(ctx, ctx->envA, need * sizeof(double)));
  TRY(ensure(ctx, ctx->envB, need * sizeof(double)));
  double* cur = (double*)ctx->envA.p;
  double* nxt = (double*)ctx->envB.p;
  TRY_HIP(hipMemcpyAsync(cur, kOne, 2 * sizeof(double), hipMemcpyHostToDevice, ctx->stream));
  for (int s = 0; s < n; ++s) {
    TRY(env_left(ctx, cur, ops[s], bra->site[s], bra->bond[s], bra->bond[s + 1], ket->site[s], ket->bond[s],
                 ket->bond[s + 1], nxt, Arith::F64));
    std::swap(cur, nxt);
  }
  TRY_HIP(hipMemcpyAsync(ctx->host, cur, 2 * sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
  TRY_HIP(hipStreamSynchronize(ctx->stream));
  *re = ctx->host[0];
  *im = ctx->host[1];
  return TDMRG_OK;
}

extern "C" tdmrg_status tdmrg_observables(tdmrg_ctx* ctx, const tdmrg_mps* mps, const tdmrg_mpo* mpo,
                                          const tdmrg_mps* psi0, tdmrg_obs* obs) {
  if (!ctx) return TDMRG_EINVAL;
  if (!mps || !mpo || !obs || !obs->pops) return fail(ctx, TDMRG_EINVAL, "NULL argument");
  if (mps->n != mpo->n || mps->dims != mpo->dims) return fail(ctx, TDMRG_ESHAPE, "mps and mpo do not match");
  if (psi0 && (psi0->n != mps->n || psi0->dims != mps->dims)) return fail(ctx, TDMRG_ESHAPE, "psi0 does not match");
  TRY(use_device(ctx));
  std::vector<const tdmrg_wop*> ops(mpo->ident.begin(), mpo->ident.end());
  double re, im;
  TRY(contract_chain(ctx, mps, mps, ops, &re, &im));
  obs->norm2 = re;
  for (int i = 0; i < mpo->n_el; ++i) {
    ops[mpo->pop_site[i]] = mpo->proj[i];
    TRY(contract_chain(ctx, mps, mps, ops, &re, &im));
    obs->pops[i] = re;
    ops[mpo->pop_site[i]] = mpo->ident[mpo->pop_site[i]];
  }
  std::vector<const tdmrg_wop*> H(mpo->W.begin(), mpo->W.end());
  TRY(contract_chain(ctx, mps, mps, H, &re, &im));
  obs->energy = re;
  obs->c_re = obs->c_im = 0.0;
  if (psi0) {
    std::vector<const tdmrg_wop*> id(mpo->ident.begin(), mpo->ident.end());
    TRY(contract_chain(ctx, psi0, mps, id, &re, &im));
    obs->c_re = re;
    obs->c_im = im;
  }
  double size = 0.0;
  for (int s = 0; s < mps->n; ++s) size += (double)mps->bond[s] * mps->dims[s] * mps->bond[s + 1];
  obs->mps_size = size;
  return TDMRG_OK;
}
