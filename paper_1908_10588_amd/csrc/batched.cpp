// Batched form: many independent two-site problems of uneven shapes.
//
// Each of the four stages of H_eff,2 * theta (eq. two-site Hamiltonian) runs
// as one persistent grouped launch over the tiles (GEMM stages) or output
// elements (channel stages) of every problem in the batch.  The Lanczos
// exponentials of all problems advance in lockstep: one grouped H_eff
// product per Krylov step for the problems that are still iterating, the
// HBM-bound vector kernels per problem.  Problems are processed in waves
// whose intermediates and Krylov vectors fit a device-memory budget.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "internal.h"

namespace tdmrg {

#define TRY_HIP(expr)                                                                             \
  do {                                                                                            \
    hipError_t e_ = (expr);                                                                       \
    if (e_ != hipSuccess)                                                                         \
      return fail(ctx, TDMRG_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_));         \
  } while (0)
#define TRY(expr)                  \
  do {                             \
    tdmrg_status s_ = (expr);      \
    if (s_ != TDMRG_OK) return s_; \
  } while (0)

static GemmOperand bop(const double* p, long im, long sb, long sr, long ld, int trans, int conj) {
  GemmOperand o;
  o.p = p; o.im = im; o.sb = sb; o.sr = sr; o.ld = ld; o.trans = trans; o.conj = conj;
  return o;
}

static GemmArgs bgemm(int M, int N, int K, int nred, GemmOperand A, GemmOperand B, double* C, long c_im,
                      long ldc) {
  GemmArgs g;
  g.M = M; g.N = N; g.K = K; g.nbatch = 1; g.nred = nred; g.role = 0;
  g.A = A; g.B = B; g.C = C; g.c_im = c_im; g.c_sb = 0; g.ldc = ldc;
  g.alpha_re = 1.0; g.alpha_im = 0.0; g.beta_re = 0.0; g.beta_im = 0.0;
  return g;
}

static MixArgs bmix(const tdmrg_wop* W, const double* in, long in_im, double* out, long out_im, int P,
                    int Q) {
  MixArgs a;
  a.in = in; a.in_im = in_im; a.out = out; a.out_im = out_im;
  a.P = P; a.Q = Q; a.din = W->d; a.dout = W->d; a.nout = W->wr;
  a.rowptr = W->f_rowptr; a.col = W->f_col; a.vre = W->f_v; a.vim = W->f_v + W->f_nnz;
  return a;
}

// Uploads the per-problem descriptors of one grouped launch into the
// context's metadata buffer at byte offset *off (kept 256-byte aligned).
template <typename T>
static tdmrg_status upload_meta(tdmrg_ctx* ctx, const std::vector<T>& v, size_t* off, const T** dev) {
  const size_t bytes = v.size() * sizeof(T);
  char* base = (char*)ctx->meta.p;
  if (*off + bytes > ctx->meta.bytes) return fail(ctx, TDMRG_ENOMEM, "batch metadata overflow");
  TRY_HIP(hipMemcpyAsync(base + *off, v.data(), bytes, hipMemcpyHostToDevice, ctx->stream));
  *dev = (const T*)(base + *off);
  *off += (bytes + 255) & ~size_t(255);
  return TDMRG_OK;
}

struct BatchItem {
  tdmrg_heff_shape s;
  const double *L, *R;
  const tdmrg_wop *W1, *W2;
  const double* x;  // input vector (planar)
  double* y;        // output vector (planar)
  double* xa;       // intermediates of this problem
  double* xb;
};

// y_p = H_eff,2 x_p for every item: four grouped launches.
tdmrg_status heff2_grouped(tdmrg_ctx* ctx, const std::vector<BatchItem>& items, Arith ar) {
  const int np = (int)items.size();
  if (np == 0) return TDMRG_OK;
  // metadata: up to 4 x GemmArgs + 2 x MixArgs + prefix arrays per problem
  const size_t need = (size_t)np * (4 * sizeof(GemmArgs) + 2 * sizeof(MixArgs) + 4 * sizeof(int) +
                                    2 * sizeof(long)) + 32 * 256;
  // the host copies of the metadata must stay valid until the copies land
  TRY_HIP(hipStreamSynchronize(ctx->stream));
  TRY(ensure(ctx, ctx->meta, need));
  // per problem: dense channel GEMMs (g2d, g3d) or the sparse channel pass (m2, m3)
  std::vector<GemmArgs> g1(np), g4(np), g2d, g3d;
  std::vector<MixArgs> m2, m3;
  std::vector<int> t1(np + 1, 0), t4(np + 1, 0), t2d(1, 0), t3d(1, 0);
  std::vector<long> e2(1, 0), e3(1, 0);
  for (int p = 0; p < np; ++p) {
    const BatchItem& it = items[p];
    const tdmrg_heff_shape& s = it.s;
    const long th = (long)s.Dl * s.d1 * s.d2 * s.Dr;
    const int N1 = s.d1 * s.d2 * s.Dr;
    const long n2 = (long)s.d2 * s.Dr;
    if (channel_gemm_pays(ctx, s, it.W1, it.W2)) {
      // layouts as in the single-problem dense path: X1[a][wl][.], X2[a][s][wc][.], X3[wr][a][s][t][b']
      const double *W1m, *W2m;
      TRY(wop_dense(ctx, it.W1, 0, &W1m));
      TRY(wop_dense(ctx, it.W2, 1, &W2m));
      g1[p] = bgemm(s.Dl, N1, s.Dl, 1, bop(it.L, (long)s.wl * s.Dl * s.Dl, (long)s.Dl * s.Dl, 0, s.Dl, 0, 0),
                    bop(it.x, th, 0, 0, N1, 0, 0), it.xa, (long)s.wl * th, (long)s.wl * N1);
      g1[p].nbatch = s.wl;
      g1[p].c_sb = N1;
      GemmArgs g2 = bgemm(s.d1 * s.wc, (int)n2, s.wl * s.d1, 1,
                          bop(W1m, (long)s.d1 * s.wc * s.wl * s.d1, 0, 0, (long)s.wl * s.d1, 0, 0),
                          bop(it.xa, (long)s.wl * th, (long)s.wl * N1, 0, n2, 0, 0), it.xb, (long)s.wc * th, n2);
      g2.nbatch = s.Dl;
      g2.c_sb = (long)s.wc * N1;
      GemmArgs g3 = bgemm(s.wr * s.d2, s.Dr, s.wc * s.d2, 1,
                          bop(W2m, (long)s.wr * s.d2 * s.wc * s.d2, 0, 0, (long)s.wc * s.d2, 0, 0),
                          bop(it.xb, (long)s.wc * th, (long)s.wc * n2, 0, s.Dr, 0, 0), it.xa, (long)s.wr * th,
                          s.Dr);
      g3.nbatch = s.Dl * s.d1;
      g3.c_sb = n2;
      g3.c_mi = s.d2;
      g3.c_so = th;
      g2d.push_back(g2);
      g3d.push_back(g3);
      t2d.push_back(t2d.back() + cgemm_tiles(g2));
      t3d.push_back(t3d.back() + cgemm_tiles(g3));
    } else {
      g1[p] = bgemm(s.wl * s.Dl, N1, s.Dl, 1, bop(it.L, (long)s.wl * s.Dl * s.Dl, 0, 0, s.Dl, 0, 0),
                    bop(it.x, th, 0, 0, N1, 0, 0), it.xa, (long)s.wl * th, N1);
      m2.push_back(bmix(it.W1, it.xa, (long)s.wl * th, it.xb, (long)s.wc * th, s.Dl, s.d2 * s.Dr));
      m3.push_back(bmix(it.W2, it.xb, (long)s.wc * th, it.xa, (long)s.wr * th, s.Dl * s.d1, s.Dr));
      e2.push_back(e2.back() + (long)s.wc * th);
      e3.push_back(e3.back() + (long)s.wr * th);
    }
    g4[p] = bgemm(s.Dl * s.d1 * s.d2, s.Dr, s.Dr, s.wr, bop(it.xa, (long)s.wr * th, 0, th, s.Dr, 0, 0),
                  bop(it.R, (long)s.wr * s.Dr * s.Dr, 0, (long)s.Dr * s.Dr, s.Dr, 1, 0), it.y, th, s.Dr);
    t1[p + 1] = t1[p] + cgemm_tiles(g1[p]);
    t4[p + 1] = t4[p] + cgemm_tiles(g4[p]);
  }
  const int nd = (int)g2d.size(), ns = (int)m2.size();
  size_t off = 0;
  const GemmArgs *dg1 = nullptr, *dg4 = nullptr, *dg2 = nullptr, *dg3 = nullptr;
  const MixArgs *dm2 = nullptr, *dm3 = nullptr;
  const int *dt1 = nullptr, *dt4 = nullptr, *dt2 = nullptr, *dt3 = nullptr;
  const long *de2 = nullptr, *de3 = nullptr;
  TRY(upload_meta(ctx, g1, &off, &dg1));
  TRY(upload_meta(ctx, g4, &off, &dg4));
  TRY(upload_meta(ctx, t1, &off, &dt1));
  TRY(upload_meta(ctx, t4, &off, &dt4));
  if (nd) {
    TRY(upload_meta(ctx, g2d, &off, &dg2));
    TRY(upload_meta(ctx, g3d, &off, &dg3));
    TRY(upload_meta(ctx, t2d, &off, &dt2));
    TRY(upload_meta(ctx, t3d, &off, &dt3));
  }
  if (ns) {
    TRY(upload_meta(ctx, m2, &off, &dm2));
    TRY(upload_meta(ctx, m3, &off, &dm3));
    TRY(upload_meta(ctx, e2, &off, &de2));
    TRY(upload_meta(ctx, e3, &off, &de3));
  }
  hipStream_t st = ctx->stream;
  // algorithmic flops / bytes of the four stages summed over the problems
  double fl[4] = {0, 0, 0, 0}, by[4] = {0, 0, 0, 0};
  if (ctx->prof.on) {
    for (const BatchItem& it : items) {
      const tdmrg_heff_shape& s = it.s;
      const double th = (double)s.Dl * s.d1 * s.d2 * s.Dr;
      fl[0] += 8.0 * s.wl * (double)s.Dl * s.Dl * s.d1 * s.d2 * s.Dr;
      by[0] += 16.0 * ((double)s.wl * s.Dl * s.Dl + th + (double)s.wl * th);
      fl[1] += 8.0 * (double)it.W1->f_nnz * s.Dl * s.d2 * s.Dr;
      by[1] += 16.0 * ((double)s.wl + s.wc) * th;
      fl[2] += 8.0 * (double)it.W2->f_nnz * s.Dl * s.d1 * s.Dr;
      by[2] += 16.0 * ((double)s.wc + s.wr) * th;
      fl[3] += 8.0 * s.wr * (double)s.Dr * s.Dr * s.Dl * s.d1 * s.d2;
      by[3] += 16.0 * ((double)s.wr * s.Dr * s.Dr + (double)s.wr * th + th);
    }
  }
  Profiler::Pending pe;
  auto begin = [&](int stage) -> tdmrg_status { return ctx->prof.on ? prof_begin(ctx, &pe, stage) : TDMRG_OK; };
  auto end = [&](int stage) -> tdmrg_status { return ctx->prof.on ? prof_end(ctx, pe, fl[stage], by[stage]) : TDMRG_OK; };
  TRY(begin(0));
  TRY_HIP(launch_cgemm_grouped(dg1, dt1, np, 0, 0, t1[np], ar, st));
  TRY(end(0));
  TRY(begin(1));
  if (nd) TRY_HIP(launch_cgemm_grouped(dg2, dt2, nd, 0, 0, t2d[nd], ar, st));
  if (ns) TRY_HIP(launch_mix_grouped(dm2, de2, ns, e2[ns], st));
  TRY(end(1));
  TRY(begin(2));
  if (nd) TRY_HIP(launch_cgemm_grouped(dg3, dt3, nd, 0, 0, t3d[nd], ar, st));
  if (ns) TRY_HIP(launch_mix_grouped(dm3, de3, ns, e3[ns], st));
  TRY(end(2));
  TRY(begin(3));
  TRY_HIP(launch_cgemm_grouped(dg4, dt4, np, 0, 1, t4[np], ar, st));
  TRY(end(3));
  // keep the host vectors alive until the asynchronous uploads completed
  TRY_HIP(hipStreamSynchronize(st));
  if (ctx->prof.on) TRY(prof_flush(ctx));
  return TDMRG_OK;
}

static size_t item_ws_doubles(const tdmrg_heff_shape& s, int m_max) {
  const size_t th = (size_t)s.Dl * s.d1 * s.d2 * s.Dr;
  const size_t wa = (size_t)std::max(s.wl, s.wr), wb = (size_t)s.wc;
  return 2 * th * (wa + wb) + (m_max > 0 ? 2 * th * (size_t)(m_max + 1) : 0) + 64;
}

// Split [0, n) into consecutive waves whose workspace fits `budget` doubles.
static std::vector<std::pair<int, int>> plan_waves(const tdmrg_heff_shape* shapes, int n, int m_max,
                                                   size_t budget) {
  std::vector<std::pair<int, int>> waves;
  int a = 0;
  size_t used = 0;
  for (int p = 0; p < n; ++p) {
    const size_t w = item_ws_doubles(shapes[p], m_max);
    if (p > a && used + w > budget) {
      waves.push_back({a, p});
      a = p;
      used = 0;
    }
    used += w;
  }
  if (a < n) waves.push_back({a, n});
  return waves;
}

static size_t batch_budget_doubles(tdmrg_ctx* ctx) {
  if (ctx->batch_budget) return ctx->batch_budget / sizeof(double);
  size_t free_b = 0, total_b = 0;
  if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) return (size_t)1 << 31;
  return (size_t)(0.6 * (double)(free_b + ctx->batch.bytes)) / sizeof(double);
}

tdmrg_status heff2_batched(tdmrg_ctx* ctx, int n, const tdmrg_heff_shape* shapes, const double* const* L,
                           const tdmrg_wop* const* W1, const tdmrg_wop* const* W2, const double* const* R,
                           const double* const* theta, double* const* y, Arith ar) {
  const size_t budget = batch_budget_doubles(ctx);
  for (auto [a, b] : plan_waves(shapes, n, 0, budget)) {
    size_t need = 0;
    for (int p = a; p < b; ++p) need += item_ws_doubles(shapes[p], 0);
    TRY(ensure(ctx, ctx->batch, need * sizeof(double)));
    double* cur = (double*)ctx->batch.p;
    std::vector<BatchItem> items;
    for (int p = a; p < b; ++p) {
      const tdmrg_heff_shape& s = shapes[p];
      const size_t th = (size_t)s.Dl * s.d1 * s.d2 * s.Dr;
      BatchItem it{s, L[p], R[p], W1[p], W2[p], theta[p], y[p], cur, cur + 2 * th * std::max(s.wl, s.wr)};
      cur += item_ws_doubles(s, 0);
      items.push_back(it);
    }
    TRY(heff2_grouped(ctx, items, ar));
  }
  return TDMRG_OK;
}

// Lanczos exponentials of all problems in lockstep (same steps as the
// single-problem local_expm); iters[p] receives each problem's count.
tdmrg_status local_expm_batched(tdmrg_ctx* ctx, int n, const tdmrg_heff_shape* shapes,
                                const double* const* L, const tdmrg_wop* const* W1,
                                const tdmrg_wop* const* W2, const double* const* R, double* const* theta,
                                double tau, double tol, int m_max, Arith ar, int* iters, int* nonconv) {
  const size_t budget = batch_budget_doubles(ctx);
  *nonconv = 0;
  for (auto [a, b] : plan_waves(shapes, n, m_max, budget)) {
    const int np = b - a;
    size_t need = 0;
    for (int p = a; p < b; ++p) need += item_ws_doubles(shapes[p], m_max);
    TRY(ensure(ctx, ctx->batch, need * sizeof(double)));
    // per-problem scalars: alpha, beta, cr, ci, dre, dim, c_re, c_im (64 each), err, beta0
    const size_t scal = 8 * 64 + 16;
    TRY(ensure(ctx, ctx->bscal, sizeof(double) * scal * np));
    TRY(ensure(ctx, ctx->bpart, sizeof(double) * 2 * 64 * 1024));
    double* sc = (double*)ctx->bscal.p;
    double* part_re = (double*)ctx->bpart.p;
    double* part_im = part_re + 64 * 1024;
    hipStream_t st = ctx->stream;
    struct Prob {
      BatchItem it;
      long n;
      double *V, *w, *alpha, *beta, *cr, *ci, *dre, *dim, *c_re, *c_im, *err, *beta0;
      bool active;
      int iters;
    };
    std::vector<Prob> P(np);
    double* cur = (double*)ctx->batch.p;
    for (int q = 0; q < np; ++q) {
      const int p = a + q;
      const tdmrg_heff_shape& s = shapes[p];
      const size_t th = (size_t)s.Dl * s.d1 * s.d2 * s.Dr;
      Prob& pr = P[q];
      pr.n = (long)th;
      double* xa = cur;
      double* xb = xa + 2 * th * std::max(s.wl, s.wr);
      pr.V = xb + 2 * th * s.wc;
      pr.w = pr.V + 2 * th * m_max;
      cur += item_ws_doubles(s, m_max);
      pr.it = BatchItem{s, L[p], R[p], W1[p], W2[p], nullptr, pr.w, xa, xb};
      double* b0 = sc + scal * q;
      pr.alpha = b0; pr.beta = b0 + 64; pr.cr = b0 + 128; pr.ci = b0 + 192; pr.dre = b0 + 256;
      pr.dim = b0 + 320; pr.c_re = b0 + 384; pr.c_im = b0 + 448; pr.err = b0 + 512; pr.beta0 = b0 + 520;
      pr.active = true;
      pr.iters = 0;
    }
    auto dots = [&](const double* V, long vs, int nv, long nn, const double* w, double* ore, double* oim,
                    int mode) -> tdmrg_status {
      TRY_HIP(launch_multidot(V, vs, nv, nn, w, part_re, part_im, st));
      TRY_HIP(launch_reduce_partials(part_re, part_im, nv, dot_chunks(nn), ore, oim, mode, st));
      return TDMRG_OK;
    };
    for (int q = 0; q < np; ++q) {
      Prob& pr = P[q];
      double* th = theta[a + q];
      TRY(dots(th, 2 * pr.n, 1, pr.n, th, pr.beta0, nullptr, 1));
      TRY_HIP(launch_scale_by_inv(th, pr.n, pr.beta0, pr.V, st));
    }
    std::vector<double> errs(np);
    for (int j = 0; j < m_max; ++j) {
      std::vector<BatchItem> items;
      std::vector<int> act;
      for (int q = 0; q < np; ++q)
        if (P[q].active) {
          BatchItem it = P[q].it;
          it.x = P[q].V + (long)j * 2 * P[q].n;
          items.push_back(it);
          act.push_back(q);
        }
      if (act.empty()) break;
      TRY(heff2_grouped(ctx, items, ar));
      for (int q : act) {
        Prob& pr = P[q];
        const long vs = 2 * pr.n;
        // two Gram-Schmidt passes; the first one's v_j coefficient gives alpha_j
        // and the second one's update gives beta_j = ||w|| (single-problem form)
        TRY(dots(pr.V, vs, j + 1, pr.n, pr.w, pr.cr, pr.ci, 0));
        TRY_HIP(launch_copy_scalar(pr.cr + j, pr.alpha + j, st));
        TRY_HIP(launch_multiaxpy(pr.V, vs, j + 1, pr.n, pr.cr, pr.ci, pr.w, st));
        TRY(dots(pr.V, vs, j + 1, pr.n, pr.w, pr.cr, pr.ci, 0));
        TRY_HIP(launch_multiaxpy_norm(pr.V, vs, j + 1, pr.n, pr.cr, pr.ci, pr.w, part_re, pr.beta + j, st));
        TRY_HIP(launch_tridiag_expm(pr.alpha, pr.beta, j + 1, tau, pr.c_re, pr.c_im, pr.err, st));
        TRY_HIP(hipMemcpyAsync(&errs[q], pr.err, sizeof(double), hipMemcpyDeviceToHost, st));
      }
      TRY_HIP(hipStreamSynchronize(st));
      for (int q : act) {
        Prob& pr = P[q];
        const long vs = 2 * pr.n;
        pr.iters = j + 1;
        if (!(errs[q] == errs[q])) return fail(ctx, TDMRG_EINVAL, "Lanczos produced NaN");
        if (errs[q] <= tol || j == m_max - 1) {
          if (errs[q] > tol) ++*nonconv;
          TRY_HIP(launch_combine(pr.V, vs, j + 1, pr.n, pr.c_re, pr.c_im, pr.beta0, theta[a + q], st));
          pr.active = false;
        } else {
          TRY_HIP(launch_scale_by_inv(pr.w, pr.n, pr.beta + j, pr.V + (long)(j + 1) * vs, st));
        }
      }
    }
    TRY_HIP(hipStreamSynchronize(st));
    if (iters)
      for (int q = 0; q < np; ++q) iters[a + q] = P[q].iters;
  }
  return TDMRG_OK;
}

}  // namespace tdmrg
