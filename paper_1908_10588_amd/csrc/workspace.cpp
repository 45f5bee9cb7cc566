// Workspace of a context: the library's own allocations or a caller-owned
// arena (a device buffer the caller allocates, for example with torch.empty,
// and passes to tdmrg_ctx_create), and the plan of what a 2TDVP sweep needs,
// which tdmrg_workspace_query reports and an arena context reserves before a
// sweep launches anything.
#include <rocblas/rocblas.h>

#include <algorithm>
#include <cstring>

#include "internal.h"

#define TRY_STATUS(expr)           \
  do {                             \
    tdmrg_status s_ = (expr);      \
    if (s_ != TDMRG_OK) return s_; \
  } while (0)

namespace tdmrg {

namespace {
constexpr size_t kAlign = 256;
size_t align_up(size_t b) { return (b + kAlign - 1) & ~(kAlign - 1); }
}  // namespace

tdmrg_status dev_alloc(tdmrg_ctx* ctx, size_t bytes, void** out) {
  *out = nullptr;
  bytes = align_up(std::max<size_t>(bytes, 1));
  Arena& A = ctx->arena;
  if (!A.base) {
    if (hipMalloc(out, bytes) != hipSuccess) {
      *out = nullptr;
      return fail(ctx, TDMRG_ENOMEM, "device allocation of " + std::to_string(bytes) + " bytes failed");
    }
    return TDMRG_OK;
  }
  for (auto it = A.free_blocks.begin(); it != A.free_blocks.end(); ++it) {
    if (it->second < bytes) continue;
    const size_t off = it->first, rest = it->second - bytes;
    A.free_blocks.erase(it);
    if (rest) A.free_blocks[off + bytes] = rest;
    A.used_blocks[off] = bytes;
    *out = A.base + off;
    return TDMRG_OK;
  }
  size_t largest = 0;
  for (const auto& kv : A.free_blocks) largest = std::max(largest, kv.second);
  return fail(ctx, TDMRG_ENOMEM,
              "workspace arena exhausted: " + std::to_string(bytes) + " bytes asked, largest free block " +
                  std::to_string(largest) + " of an arena of " + std::to_string(A.bytes) + " bytes");
}

void dev_free(tdmrg_ctx* ctx, void* p) {
  if (!p) return;
  Arena& A = ctx->arena;
  if (!A.base) {
    (void)hipFree(p);
    return;
  }
  const size_t off = (size_t)((char*)p - A.base);
  auto u = A.used_blocks.find(off);
  if (u == A.used_blocks.end()) return;
  size_t start = off, size = u->second;
  A.used_blocks.erase(u);
  auto next = A.free_blocks.lower_bound(start);
  if (next != A.free_blocks.end() && next->first == start + size) {  // merge with the block after
    size += next->second;
    next = A.free_blocks.erase(next);
  }
  if (next != A.free_blocks.begin()) {  // and with the block before
    auto prev = std::prev(next);
    if (prev->first + prev->second == start) {
      start = prev->first;
      size += prev->second;
      A.free_blocks.erase(prev);
    }
  }
  A.free_blocks[start] = size;
}

size_t rocsolver_ws_bound(long n) {
  // rocSOLVER on gfx950 asks for at most 2.7 n^2 complex of workspace for
  // zheevd (measured for n = 16 .. 4096): 48 n^2 bytes + 1 MiB
  return (size_t)48 * (size_t)n * (size_t)n + ((size_t)1 << 20);
}

size_t heev_bytes(int n) {
  // A and V [2][n][n], Z [n][n], tau [2][n], d and e [n]
  return sizeof(double) * (5 * (size_t)n * n + 4 * (size_t)n + 64);
}

size_t rocsolver_qr_ws_bound(long n) {
  // about 2100 n bytes for zgelqf/zgeqrf and the generation of Q (measured
  // for n = 16 .. 4096)
  return (size_t)4096 * (size_t)n + ((size_t)1 << 20);
}

tdmrg_status rocws_reserve(tdmrg_ctx* ctx, size_t bytes) {
  if (!ctx->arena.base || bytes <= ctx->rocws.bytes) return TDMRG_OK;
  TRY_STATUS(ensure(ctx, ctx->rocws, bytes));
  if (rocblas_set_workspace(ctx->blas, ctx->rocws.p, ctx->rocws.bytes) != rocblas_status_success)
    return fail(ctx, TDMRG_EDEVICE, "rocblas_set_workspace failed");
  return TDMRG_OK;
}

bool pair_fusion_plan(const double* W1, int wl, int wc, int d1, const double* W2, int wr, int d2, int fuse_mode,
                      long* products) {
  *products = 0;
  if (fuse_mode == 0) return false;
  const size_t n1 = (size_t)wl * wc * d1 * d1, n2 = (size_t)wc * wr * d2 * d2;
  // nonzero entries per channel block
  std::vector<long> c1((size_t)wl * wc, 0), c2((size_t)wc * wr, 0);
  long nnz1 = 0, nnz2 = 0;
  for (size_t o = 0; o < n1; ++o)
    if (W1[o] != 0.0 || W1[n1 + o] != 0.0) {
      c1[o / ((size_t)d1 * d1)]++;
      nnz1++;
    }
  for (size_t o = 0; o < n2; ++o)
    if (W2[o] != 0.0 || W2[n2 + o] != 0.0) {
      c2[o / ((size_t)d2 * d2)]++;
      nnz2++;
    }
  long prod = 0;
  for (int y = 0; y < wr; ++y)
    for (int c = 0; c < wc; ++c)
      for (int x = 0; x < wl; ++x) prod += c1[(size_t)x * wc + c] * c2[(size_t)c * wr + y];
  *products = prod;
  if (fuse_mode == 2) return true;
  // cost model: fusing saves the write and read of the middle intermediate
  // (32 * wc * d1 * d2 bytes per (D_l, D_r) pair, at ~5 TB/s) and costs the
  // extra multiply-adds of the denser fused operator (8 flops each, at ~40
  // TFLOP/s of FP64 vector arithmetic)
  const long separate = nnz1 * d2 + nnz2 * d1;
  const double budget = 32.0 * wc * d1 * d2 / 5.0 * 40.0 / 8.0;
  return (double)(prod - separate) <= budget;
}

size_t WsPlan::total() const {
  size_t t = 0;
  for (size_t b : {theta, small, kry, wvec, xa, xb, splitk, svd_u, svd_z, svd_s, svd_e, svd_vt, sub, cqr, heev, envA,
                   envB, rocws})
    t += align_up(b);
  return t + pairs;
}

WsPlan plan_sweep(const std::vector<int>& dims, const std::vector<int>& wdims, const std::vector<int>& caps,
                  int krylov_max, const std::vector<std::vector<double>>& W, int fuse_mode) {
  const int n = (int)dims.size();
  const size_t m_max = (size_t)std::min(std::max(krylov_max, 1), 64);
  const size_t D8 = sizeof(double);
  WsPlan P;
  // Lanczos scalars and partial sums (fixed layout)
  P.small = D8 * (16 * 64 + 2 * 64 * 1024 + 64);
  // split-K partial products: fewer than 128 output tiles, at most about
  // 1024 / tiles + 2 chunks of them, 64 x 64 complex each
  P.splitk = D8 * 2 * (size_t)(1024 + 2 * 127) * 4096;
  long nmax = 1;
  for (int i = 0; i + 1 < n; ++i) {
    const size_t Dl = caps[i], Dr = caps[i + 2], d1 = dims[i], d2 = dims[i + 1];
    const size_t rows = Dl * d1, cols = d2 * Dr, th = rows * cols;
    const size_t mn = std::min(rows, cols), mx = std::max(rows, cols);
    const size_t w = std::max({wdims[i], wdims[i + 1], wdims[i + 2]});
    const size_t kmax = std::min<size_t>(caps[i + 1], mn);
    P.theta = std::max(P.theta, D8 * 2 * th);
    P.kry = std::max(P.kry, D8 * 2 * th * m_max);
    P.wvec = std::max(P.wvec, D8 * 4 * th);
    // contraction intermediates of H_eff,2 (separate, fused or dense channel
    // stages), H_eff,1 and the environment updates (each at most w |theta|)
    P.xa = std::max(P.xa, D8 * 2 * w * th);
    P.xb = std::max(P.xb, D8 * 2 * w * th);
    // SVD: Jacobi (theta copy, rotations), Gram + eigensolver (on either
    // side), subspace iteration (block b) and its Cholesky QR
    P.svd_u = std::max(P.svd_u, D8 * 2 * std::max(th, mx * mx));
    P.svd_z = std::max(P.svd_z, D8 * 2 * mx * mx);
    P.svd_s = std::max(P.svd_s, D8 * 2 * mx + 64);
    P.svd_e = std::max(P.svd_e, D8 * mx + 64);
    P.svd_vt = std::max(P.svd_vt, D8 * 4 * mx * kmax);
    const size_t over = std::max<size_t>(32, kmax / 2);
    const size_t b = std::min<size_t>(std::min<size_t>((kmax + over + 15) / 16 * 16, 512), mn);
    P.sub = std::max(P.sub, D8 * (2 * 5 * mx * b + 14 * b * b + 5 * b + 32 * b + 64));
    const size_t bc = std::max<size_t>(512, kmax);
    P.cqr = std::max(P.cqr, D8 * (8 * bc * bc + bc + 64));
    nmax = std::max<long>(nmax, (long)mx);
    // hand-written eigensolver (Rayleigh-Ritz block or Gram matrix up to kHeevRoute)
    const size_t h = std::min<size_t>(mx, kHeevRoute);
    P.heev = std::max(P.heev, heev_bytes((int)h));
    // the fused channel operator of the pair, when it pays
    long products = 0;
    if (pair_fusion_plan(W[i].data(), wdims[i], wdims[i + 1], dims[i], W[i + 1].data(), wdims[i + 2], dims[i + 1],
                         fuse_mode, &products))
      P.pairs += align_up(sizeof(int) * ((size_t)wdims[i + 2] * dims[i] * dims[i + 1] + 1)) +
                 align_up(sizeof(int) * (size_t)products) + align_up(D8 * 2 * (size_t)products) +
                 align_up(mix_blocks_bytes((long)wdims[i + 2] * dims[i] * dims[i + 1], products));
  }
  // observables: transfer matrices of the whole MPO on every bond
  for (int b = 0; b <= n; ++b) {
    const size_t e = D8 * 2 * (size_t)std::max(wdims[b], 1) * caps[b] * caps[b];
    P.envA = std::max(P.envA, e);
    P.envB = std::max(P.envB, e);
  }
  P.rocws = rocsolver_ws_bound(nmax);
  return P;
}

tdmrg_status reserve_sweep(tdmrg_ctx* ctx, const tdmrg_mps* mps, const tdmrg_mpo* mpo, int krylov_max) {
  if (!ctx->arena.base) return TDMRG_OK;
  std::vector<std::vector<double>> W(mpo->n);
  for (int s = 0; s < mpo->n; ++s) W[s] = mpo->W[s]->host;
  const WsPlan P = plan_sweep(mps->dims, mpo->wdims, mps->cap, krylov_max, W, ctx->fuse_mode);
  const std::pair<DevBuf*, size_t> bufs[] = {
      {&ctx->theta, P.theta}, {&ctx->small, P.small}, {&ctx->kry, P.kry},       {&ctx->wvec, P.wvec},
      {&ctx->xa, P.xa},       {&ctx->xb, P.xb},       {&ctx->splitk, P.splitk}, {&ctx->svd_u, P.svd_u},
      {&ctx->svd_z, P.svd_z}, {&ctx->svd_s, P.svd_s}, {&ctx->svd_e, P.svd_e},   {&ctx->svd_vt, P.svd_vt},
      {&ctx->sub, P.sub},     {&ctx->cqr, P.cqr},     {&ctx->heev, P.heev},     {&ctx->envA, P.envA},
      {&ctx->envB, P.envB}};
  // the shortfall first, so that nothing is freed or moved when it cannot fit
  size_t need = 0, free_total = 0;
  for (const auto& kv : bufs)
    if (kv.first->bytes < kv.second) need += align_up(kv.second);
  if (ctx->rocws.bytes < P.rocws) need += align_up(P.rocws);
  for (const auto& kv : ctx->arena.free_blocks) free_total += kv.second;
  size_t growing = 0;  // blocks that are replaced come back to the free list
  for (const auto& kv : bufs)
    if (kv.first->bytes < kv.second) growing += kv.first->bytes;
  if (ctx->rocws.bytes < P.rocws) growing += ctx->rocws.bytes;
  if (need > free_total + growing)
    return fail(ctx, TDMRG_ENOMEM,
                "workspace arena too small for this sweep: " + std::to_string(need) + " more bytes needed, " +
                    std::to_string(free_total) + " free (tdmrg_workspace_query gives the size)");
  for (const auto& kv : bufs) TRY_STATUS(ensure(ctx, *kv.first, kv.second));
  TRY_STATUS(rocws_reserve(ctx, P.rocws));
  return TDMRG_OK;
}

}  // namespace tdmrg
