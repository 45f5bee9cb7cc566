// Host drivers of the hot-path steps: effective-Hamiltonian products,
// environment updates, two-site tensor formation, the Lanczos exponential
// and the SVD truncation.  Every arithmetic step runs in a kernel of
// kernels.hip (or rocSOLVER for the SVD); this file only sizes and orders the
// launches on the context stream.
#include <rocsolver/rocsolver.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstring>

#include "internal.h"

namespace tdmrg {

#define TRY_HIP(expr)                                                                       \
  do {                                                                                      \
    hipError_t e_ = (expr);                                                                 \
    if (e_ != hipSuccess) return fail(ctx, TDMRG_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)
#define TRY(expr)                       \
  do {                                  \
    tdmrg_status s_ = (expr);           \
    if (s_ != TDMRG_OK) return s_;      \
  } while (0)

tdmrg_status fail(const tdmrg_ctx* ctx, tdmrg_status st, const std::string& msg) {
  if (ctx) const_cast<tdmrg_ctx*>(ctx)->err = msg;
  return st;
}

static std::atomic<unsigned long> g_graph_epoch{1};

void graph_epoch_bump() { g_graph_epoch.fetch_add(1); }
unsigned long graph_epoch() { return g_graph_epoch.load(); }

void graphs_clear(tdmrg_ctx* ctx) {
  for (auto& kv : ctx->lgraphs)
    if (kv.second.exec) (void)hipGraphExecDestroy(kv.second.exec);
  ctx->lgraphs.clear();
}

// Drops the cached step graphs captured before the last epoch advance.
static void graphs_sweep(tdmrg_ctx* ctx) {
  const unsigned long now = graph_epoch();
  if (ctx->lgraph_epoch == now) return;
  for (auto it = ctx->lgraphs.begin(); it != ctx->lgraphs.end();) {
    if (it->second.epoch != now) {
      if (it->second.exec) (void)hipGraphExecDestroy(it->second.exec);
      it = ctx->lgraphs.erase(it);
    } else {
      ++it;
    }
  }
  ctx->lgraph_epoch = now;
}

tdmrg_status ensure(tdmrg_ctx* ctx, DevBuf& b, size_t bytes) {
  if (bytes <= b.bytes) return TDMRG_OK;
  if (b.p) {
    TRY_HIP(hipStreamSynchronize(ctx->stream));
    dev_free(ctx, b.p);
    b.p = nullptr;
    b.bytes = 0;
    graph_epoch_bump();
  }
  // growth headroom for the library's own allocations; an arena is planned
  // (reserve_sweep), so its blocks are taken at the size asked for
  size_t want = ctx->arena.base ? bytes : bytes + bytes / 4 + 4096;
  want = (want + 255) & ~size_t(255);
  TRY(dev_alloc(ctx, want, &b.p));
  b.bytes = want;
  return TDMRG_OK;
}

void build_mix_blocks(int nrows, const int* rowptr, const int* col, const double* vre, const double* vim,
                      HostBlocks* out) {
  const int R = kMixRows;
  const int nblk = (nrows + R - 1) / R;
  out->bptr.assign(1, 0);
  out->bcol.clear();
  out->bmask.clear();
  std::vector<double> re, im;
  for (int B = 0; B < nblk; ++B) {
    std::map<int, size_t> where;  // column -> its slot in this block (ascending)
    const int r0 = B * R, r1 = std::min(nrows, r0 + R);
    for (int r = r0; r < r1; ++r)
      for (int e = rowptr[r]; e < rowptr[r + 1]; ++e) where.emplace(col[e], 0);
    const size_t first = out->bcol.size();
    for (auto& kv : where) {
      kv.second = out->bcol.size();
      out->bcol.push_back(kv.first);
      out->bmask.push_back(0u);
      re.insert(re.end(), R, 0.0);
      im.insert(im.end(), R, 0.0);
    }
    for (int r = r0; r < r1; ++r)
      for (int e = rowptr[r]; e < rowptr[r + 1]; ++e) {
        const size_t u = where[col[e]];
        re[u * R + (r - r0)] = vre[e];
        im[u * R + (r - r0)] = vim[e];
        out->bmask[u] |= 1u << (r - r0);
      }
    (void)first;
    out->bptr.push_back((int)out->bcol.size());
  }
  out->bval = re;
  out->bval.insert(out->bval.end(), im.begin(), im.end());
}

size_t mix_blocks_bytes(long nrows, long nnz) {
  const long nblk = (nrows + kMixRows - 1) / kMixRows;
  return sizeof(int) * (nblk + 1) + (sizeof(int) + sizeof(unsigned) + 2 * sizeof(double) * kMixRows) * nnz + 4 * 256;
}

static MixArgs mix_fwd(const tdmrg_wop* W, const double* in, long in_im, double* out, long out_im,
                       int P, int Q) {
  MixArgs a;
  a.in = in; a.in_im = in_im; a.out = out; a.out_im = out_im;
  a.P = P; a.Q = Q; a.din = W->d; a.dout = W->d; a.nout = W->wr;
  a.rowptr = W->f_rowptr; a.col = W->f_col; a.vre = W->f_v; a.vim = W->f_v + W->f_nnz;
  a.blk = W->f_blk.view();
  return a;
}
static MixArgs mix_bwd(const tdmrg_wop* W, const double* in, long in_im, double* out, long out_im,
                       int P, int Q) {
  MixArgs a;
  a.in = in; a.in_im = in_im; a.out = out; a.out_im = out_im;
  a.P = P; a.Q = Q; a.din = W->d; a.dout = W->d; a.nout = W->wl;
  a.rowptr = W->b_rowptr; a.col = W->b_col; a.vre = W->b_v; a.vim = W->b_v + W->b_nnz;
  return a;
}

static GemmOperand op(const double* p, long im, long sb, long sr, long ld, int trans, int conj) {
  GemmOperand o;
  o.p = p; o.im = im; o.sb = sb; o.sr = sr; o.ld = ld; o.trans = trans; o.conj = conj;
  return o;
}

static GemmArgs gemm(int M, int N, int K, int nbatch, int nred, GemmOperand A, GemmOperand B,
                     double* C, long c_im, long c_sb, long ldc) {
  GemmArgs g;
  g.M = M; g.N = N; g.K = K; g.nbatch = nbatch; g.nred = nred; g.role = 0;
  g.A = A; g.B = B; g.C = C; g.c_im = c_im; g.c_sb = c_sb; g.ldc = ldc;
  g.alpha_re = 1.0; g.alpha_im = 0.0; g.beta_re = 0.0; g.beta_im = 0.0;
  return g;
}

// ---- GEMM tile autotuning: the first call of a shape class (transposes,
// precision and power-of-two buckets of M, N, K * nred and the batch count)
// that overwrites its output and is large enough runs every tile variant,
// timed with events, and the fastest is kept for the class.  The variants
// agree bitwise, so tuning changes no result.
static std::array<int, 8> tile_key(const GemmArgs& g, Arith ar) {
  auto lg = [](double x) {
    int b = 0;
    while (b < 48 && std::ldexp(1.0, b) < x) ++b;
    return b;
  };
  return {g.A.trans, g.B.trans, (int)ar, lg(g.M), lg(g.N), lg((double)g.K * g.nred), lg(g.nbatch), g.role == 3};
}

// ---- split K: a product with few output tiles and a long reduction (the
// b x b Gram and Rayleigh quotient matrices of the subspace SVD have 9 tiles
// and K in the thousands; the channel reductions of the adjoints are alike)
// would occupy a few CUs for its whole loop, each K slice of 16 waiting on
// its loads.  The reduction is cut into S chunks computed as a third grid
// dimension into workspace and summed in a fixed order: with one reduction
// block, K ranges of at least 128; with several, runs of whole blocks (the
// last run may be shorter and has a launch of its own).  The split depends on
// the shape only, so results stay deterministic.
struct SplitPlan {
  int S = 0;      // chunks in all
  int kc = 0;     // K per chunk (one block), else 0
  int r = 0;      // blocks per full chunk (several blocks), else 0
  int full = 0;   // chunks of r blocks; a remainder chunk follows if S > full
};

static bool splitk_plan(const GemmArgs& g, SplitPlan* sp) {
  if (g.c_mi != 0 || g.ktot != 0 || g.role == 3) return false;
  const long tiles = (long)((g.M + 63) / 64) * ((g.N + 63) / 64) * g.nbatch;
  if (tiles >= 128) return false;
  const long wide = (1024 + tiles - 1) / tiles;  // chunks that still fit about 1024 workgroups
  if (g.nred > 1) {
    if (g.role != 0) return false;
    const long kb = (g.K + 15) / 16;  // K slices per block
    if (g.nred * kb < 24) return false;
    const long rmin = (8 + kb - 1) / kb;  // at least 8 slices per chunk
    const long smax = std::min<long>(wide, g.nred / rmin);
    if (smax < 2) return false;
    const int r = (int)((g.nred + smax - 1) / smax);
    sp->r = r;
    sp->full = g.nred / r;
    sp->S = sp->full + (g.nred % r != 0);
    sp->kc = 0;
    return sp->S >= 2;
  }
  if (g.K < 384) return false;
  const long s = std::min<long>(g.K / 128, wide);
  if (s < 2) return false;
  const int c = (int)(((g.K + s - 1) / s + 15) / 16 * 16);
  sp->kc = c;
  sp->S = (g.K + c - 1) / c;
  sp->full = sp->S;
  sp->r = 0;
  return sp->S >= 2;
}

hipError_t tuned_cgemm(tdmrg_ctx* ctx, const GemmArgs& g, Arith ar, hipStream_t s) {
  SplitPlan sp;
  if (splitk_plan(g, &sp)) {
    const int S = sp.S;
    const long mnb = (long)g.M * g.N * g.nbatch;
    if (ensure(ctx, ctx->splitk, sizeof(double) * 2 * (size_t)S * mnb) != TDMRG_OK) return hipErrorOutOfMemory;
    GemmArgs p = g;
    p.C = (double*)ctx->splitk.p;  // FP64 partial products, also for an FP32-stored C
    p.c_f32 = 0;
    p.c_im = (long)S * mnb;
    p.c_sk = mnb;
    p.c_sb = (long)g.M * g.N;
    p.ldc = g.N;
    p.alpha_re = 1.0;
    p.alpha_im = 0.0;
    p.beta_re = 0.0;
    p.beta_im = 0.0;
    if (sp.r > 0) {  // chunk c < full covers reduction blocks [c r, (c+1) r), each with the whole K
      p.nred = sp.r;
      p.ktot = sp.full * g.K;
      p.A.sk = (long)sp.r * g.A.sr;
      p.B.sk = (long)sp.r * g.B.sr;
    } else {
      p.K = sp.kc;
      p.ktot = g.K;
      p.A.sk = g.A.trans ? (long)sp.kc * g.A.ld : sp.kc;  // chunk c starts at K index c * kc
      p.B.sk = g.B.trans ? sp.kc : (long)sp.kc * g.B.ld;
    }
    hipError_t e = launch_cgemm(p, ar, s);
    if (e != hipSuccess) return e;
    if (S > sp.full) {  // the remaining blocks [full r, nred) into the last chunk
      const long b0 = (long)sp.full * sp.r;
      GemmArgs q = p;
      q.nred = g.nred - (int)b0;
      q.ktot = 0;
      // operand pointers advance in elements of their storage (FP32 or FP64)
      q.A.p = g.A.f32 ? (const double*)((const float*)g.A.p + b0 * g.A.sr) : g.A.p + b0 * g.A.sr;
      q.B.p = g.B.f32 ? (const double*)((const float*)g.B.p + b0 * g.B.sr) : g.B.p + b0 * g.B.sr;
      q.C = p.C + (long)sp.full * mnb;
      e = launch_cgemm(q, ar, s);
      if (e != hipSuccess) return e;
    }
    return launch_splitk_reduce(p.C, S, g.nbatch, g.M, g.N, g.C, g.c_im, g.c_sb, g.ldc, g.alpha_re, g.alpha_im,
                                g.beta_re, g.beta_im, g.c_f32, s);
  }
  if (!ctx->autotune) return launch_cgemm(g, ar, s);
  const std::array<int, 8> key = tile_key(g, ar);
  auto it = ctx->tiles.find(key);
  if (it != ctx->tiles.end()) return launch_cgemm_tile(g, ar, it->second, s);
  const double work = (double)g.M * g.N * (double)g.K * g.nred * g.nbatch;
  if (work < 2e8 || g.beta_re != 0.0 || g.beta_im != 0.0 || ctx->prof.on) return launch_cgemm(g, ar, s);
  for (hipEvent_t* e : {&ctx->tune_ev[0], &ctx->tune_ev[1]})
    if (!*e) {
      hipError_t err = hipEventCreate(e);
      if (err != hipSuccess) return err;
    }
  float best = INFINITY;
  int bv = 0;
  for (int v = 0; v < kGemmTileVariants; ++v) {
    // one untimed run, then the best of three timed ones (a single timing
    // lets run-to-run noise pick a slower variant for the whole class)
    hipError_t err = launch_cgemm_tile(g, ar, v, s);
    float ms = INFINITY;
    for (int rep = 0; rep < 3 && err == hipSuccess; ++rep) {
      err = hipEventRecord(ctx->tune_ev[0], s);
      if (err == hipSuccess) err = launch_cgemm_tile(g, ar, v, s);
      if (err == hipSuccess) err = hipEventRecord(ctx->tune_ev[1], s);
      if (err == hipSuccess) err = hipEventSynchronize(ctx->tune_ev[1]);
      float t = 0.f;
      if (err == hipSuccess) err = hipEventElapsedTime(&t, ctx->tune_ev[0], ctx->tune_ev[1]);
      if (err == hipSuccess) ms = std::min(ms, t);
    }
    if (err != hipSuccess) return err;
    if (ms < best) {
      best = ms;
      bv = v;
    }
  }
  ctx->tiles[key] = bv;
  return hipSuccess;  // the output holds the (identical) result of the last variant
}

// Event pair around one profiled launch.
tdmrg_status prof_begin(tdmrg_ctx* ctx, Profiler::Pending* p, int stage) {
  Profiler& P = ctx->prof;
  for (hipEvent_t* e : {&p->a, &p->b}) {
    if (P.pool.empty()) {
      hipEvent_t ev;
      TRY_HIP(hipEventCreate(&ev));
      P.pool.push_back(ev);
    }
    *e = P.pool.back();
    P.pool.pop_back();
  }
  p->stage = stage;
  TRY_HIP(hipEventRecord(p->a, ctx->stream));
  return TDMRG_OK;
}

tdmrg_status prof_end(tdmrg_ctx* ctx, Profiler::Pending& p, double flops, double bytes) {
  Profiler& P = ctx->prof;
  TRY_HIP(hipEventRecord(p.b, ctx->stream));
  P.pending.push_back(p);
  P.flops[p.stage] += flops;
  P.bytes[p.stage] += bytes;
  P.launches[p.stage] += 1;
  return TDMRG_OK;
}

tdmrg_status prof_flush(tdmrg_ctx* ctx) {
  Profiler& P = ctx->prof;
  for (auto& p : P.pending) {
    float ms = 0.f;
    TRY_HIP(hipEventElapsedTime(&ms, p.a, p.b));
    P.ms[p.stage] += ms;
    P.pool.push_back(p.a);
    P.pool.push_back(p.b);
  }
  P.pending.clear();
  return TDMRG_OK;
}

void prof_release(tdmrg_ctx* ctx) {
  Profiler& P = ctx->prof;
  for (auto& p : P.pending) {
    P.pool.push_back(p.a);
    P.pool.push_back(p.b);
  }
  P.pending.clear();
  for (hipEvent_t e : P.pool) (void)hipEventDestroy(e);
  P.pool.clear();
}

// ---------------------------------------------------------------------------
// fused two-site channel operator
// ---------------------------------------------------------------------------
void pair_release(tdmrg_ctx* ctx) {
  graph_epoch_bump();
  for (auto& kv : ctx->pairs) {
    for (void* p : {(void*)kv.second.rowptr, (void*)kv.second.col, (void*)kv.second.v, (void*)kv.second.blk.bptr,
                    (void*)kv.second.blk.bcol, (void*)kv.second.blk.bval, (void*)kv.second.blk.bmask})
      if (p) dev_free(ctx, p);
  }
  ctx->pairs.clear();
}

tdmrg_status pair_op(tdmrg_ctx* ctx, const tdmrg_wop* W1, const tdmrg_wop* W2, const PairOp** out) {
  *out = nullptr;
  if (ctx->fuse_mode == 0) return TDMRG_OK;
  const std::pair<long, long> key{W1->id, W2->id};
  auto found = ctx->pairs.find(key);
  if (found != ctx->pairs.end()) {
    if (found->second.nnz > 0) *out = &found->second;
    return TDMRG_OK;
  }
  const int wl = W1->wl, wc = W1->wr, wr = W2->wr, d1 = W1->d, d2 = W2->d;
  const size_t n1 = (size_t)wl * wc * d1 * d1, n2 = (size_t)wc * wr * d2 * d2;
  PairOp& P = ctx->pairs[key];
  long products = 0;
  if (!pair_fusion_plan(W1->host.data(), wl, wc, d1, W2->host.data(), wr, d2, ctx->fuse_mode, &products)) {
    P.nnz = -1;
    return TDMRG_OK;
  }
  struct E {
    int a, b;
    double re, im;
  };
  // nonzero entries of every channel block
  std::vector<std::vector<E>> b1((size_t)wl * wc), b2((size_t)wc * wr);
  for (int x = 0; x < wl; ++x)
    for (int c = 0; c < wc; ++c)
      for (int s = 0; s < d1; ++s)
        for (int sp = 0; sp < d1; ++sp) {
          const size_t o = (((size_t)x * wc + c) * d1 + s) * d1 + sp;
          const double re = W1->host[o], im = W1->host[n1 + o];
          if (re != 0.0 || im != 0.0) b1[(size_t)x * wc + c].push_back({s, sp, re, im});
        }
  for (int c = 0; c < wc; ++c)
    for (int y = 0; y < wr; ++y)
      for (int t = 0; t < d2; ++t)
        for (int tp = 0; tp < d2; ++tp) {
          const size_t o = (((size_t)c * wr + y) * d2 + t) * d2 + tp;
          const double re = W2->host[o], im = W2->host[n2 + o];
          if (re != 0.0 || im != 0.0) b2[(size_t)c * wr + y].push_back({t, tp, re, im});
        }
  const int dd = d1 * d2;
  // accumulate the products per output row (y, s, t)
  std::vector<std::map<long, std::pair<double, double>>> rows((size_t)wr * dd);
  for (int y = 0; y < wr; ++y)
    for (int c = 0; c < wc; ++c) {
      const auto& B2 = b2[(size_t)c * wr + y];
      if (B2.empty()) continue;
      for (int x = 0; x < wl; ++x)
        for (const E& e1 : b1[(size_t)x * wc + c])
          for (const E& e2 : B2) {
            const long col = ((long)x * d1 + e1.b) * d2 + e2.b;
            auto& acc = rows[(size_t)y * dd + e1.a * d2 + e2.a][col];
            acc.first += e1.re * e2.re - e1.im * e2.im;
            acc.second += e1.re * e2.im + e1.im * e2.re;
          }
    }
  std::vector<int> rp(1, 0), col;
  std::vector<double> vr, vi;
  for (auto& r : rows) {
    for (auto& kv : r)
      if (kv.second.first != 0.0 || kv.second.second != 0.0) {
        col.push_back((int)kv.first);
        vr.push_back(kv.second.first);
        vi.push_back(kv.second.second);
      }
    rp.push_back((int)col.size());
  }
  if (col.empty()) {
    P.nnz = -1;
    return TDMRG_OK;
  }
  std::vector<double> v(vr);
  v.insert(v.end(), vi.begin(), vi.end());
  TRY(dev_alloc(ctx, rp.size() * sizeof(int), (void**)&P.rowptr));
  TRY(dev_alloc(ctx, col.size() * sizeof(int), (void**)&P.col));
  TRY(dev_alloc(ctx, v.size() * sizeof(double), (void**)&P.v));
  HostBlocks hb;
  build_mix_blocks((int)rp.size() - 1, rp.data(), col.data(), vr.data(), vi.data(), &hb);
  TRY(dev_alloc(ctx, hb.bptr.size() * sizeof(int), (void**)&P.blk.bptr));
  TRY(dev_alloc(ctx, hb.bcol.size() * sizeof(int), (void**)&P.blk.bcol));
  TRY(dev_alloc(ctx, hb.bval.size() * sizeof(double), (void**)&P.blk.bval));
  TRY(dev_alloc(ctx, hb.bmask.size() * sizeof(unsigned), (void**)&P.blk.bmask));
  P.blk.ncols = (long)hb.bcol.size();
  TRY_HIP(hipMemcpy(P.blk.bptr, hb.bptr.data(), hb.bptr.size() * sizeof(int), hipMemcpyHostToDevice));
  TRY_HIP(hipMemcpy(P.blk.bcol, hb.bcol.data(), hb.bcol.size() * sizeof(int), hipMemcpyHostToDevice));
  TRY_HIP(hipMemcpy(P.blk.bval, hb.bval.data(), hb.bval.size() * sizeof(double), hipMemcpyHostToDevice));
  TRY_HIP(hipMemcpy(P.blk.bmask, hb.bmask.data(), hb.bmask.size() * sizeof(unsigned), hipMemcpyHostToDevice));
  TRY_HIP(hipMemcpy(P.rowptr, rp.data(), rp.size() * sizeof(int), hipMemcpyHostToDevice));
  TRY_HIP(hipMemcpy(P.col, col.data(), col.size() * sizeof(int), hipMemcpyHostToDevice));
  TRY_HIP(hipMemcpy(P.v, v.data(), v.size() * sizeof(double), hipMemcpyHostToDevice));
  P.nnz = (long)col.size();
  *out = &P;
  return TDMRG_OK;
}

// H_eff,2 theta with both channel stages in one pass through W12.
bool channel_gemm_pays(const tdmrg_ctx* ctx, const tdmrg_heff_shape& s, const tdmrg_wop* W1,
                       const tdmrg_wop* W2) {
  if (ctx->chan_gemm != 1) return ctx->chan_gemm == 2;
  // time estimates: the sparse channel pass streams about 2.5e12 B/s and
  // 2.5e12 flop/s of its stored nonzeros; the dense GEMMs run about 35e12
  // flop/s on every operator entry and stream their operands at 5e12 B/s
  const double th = (double)s.Dl * s.d1 * s.d2 * s.Dr;
  const double fs = 8.0 * ((double)W1->f_nnz * s.d2 + (double)W2->f_nnz * s.d1) * s.Dl * s.Dr;
  const double fd = 8.0 * th * ((double)s.wl * s.wc * s.d1 + (double)s.wc * s.wr * s.d2);
  const double by = 16.0 * th * ((double)s.wl + 2.0 * s.wc + s.wr);
  const double t_sparse = std::max(fs, by) / 2.5e12;
  const double t_dense = fd / 35e12 + by / 5e12;
  return t_dense < t_sparse;
}

// H_eff,2 * theta with the channel stages as dense GEMMs (four GEMMs):
//   X1[a][wl][s'][t'][b'] = sum_a' L[wl][a][a'] theta[a'][s'][t'][b']            (batch wl)
//   X2[a][s][wc][t'][b']  = sum_{wl,s'} W1[wl][wc][s][s'] X1[a][wl][s'][t'][b']   (batch a)
//   X3[wr][a][s][t][b']   = sum_{wc,t'} W2[wc][wr][t][t'] X2[a][s][wc][t'][b']   (batch (a, s))
//   y[a][s][t][b]         = sum_{wr,b'} X3[wr][a][s][t][b'] R[wr][b][b']
// The operator matrices are the dense forms of the wop handles; the
// layouts make every contraction index of the channel stages contiguous.
static tdmrg_status heff2_dense(tdmrg_ctx* ctx, const tdmrg_heff_shape& s, const double* L, const tdmrg_wop* W1,
                                const tdmrg_wop* W2, const double* R, const double* theta, double* y, Arith ar) {
  const long th = (long)s.Dl * s.d1 * s.d2 * s.Dr;
  const double *W1m, *W2m;
  TRY(wop_dense(ctx, W1, 0, &W1m));
  TRY(wop_dense(ctx, W2, 1, &W2m));
  const int wmax = std::max(s.wl, s.wr);
  TRY(ensure(ctx, ctx->xa, sizeof(double) * 2 * (size_t)wmax * th));
  TRY(ensure(ctx, ctx->xb, sizeof(double) * 2 * (size_t)s.wc * th));
  double* XA = (double*)ctx->xa.p;
  double* XB = (double*)ctx->xb.p;
  const bool prof = ctx->prof.on;
  Profiler::Pending pe;
  const double cb = 16.0;
  const int f32 = ar != Arith::F64;  // mixed forms keep the intermediates in FP32
  const long n1 = (long)s.d1 * s.d2 * s.Dr, n2 = (long)s.d2 * s.Dr;
  GemmArgs g1 = gemm(s.Dl, (int)n1, s.Dl, s.wl, 1,
                     op(L, (long)s.wl * s.Dl * s.Dl, (long)s.Dl * s.Dl, 0, s.Dl, 0, 0),
                     op(theta, th, 0, 0, n1, 0, 0), XA, (long)s.wl * th, n1, (long)s.wl * n1);
  g1.role = prof ? 1 : 0;
  g1.c_f32 = f32;
  if (prof) TRY(prof_begin(ctx, &pe, 0));
  TRY_HIP(tuned_cgemm(ctx, g1, ar, ctx->stream));
  if (prof)
    TRY(prof_end(ctx, pe, 8.0 * s.wl * s.Dl * (double)s.Dl * n1,
                 cb * ((double)s.wl * s.Dl * s.Dl + th + (double)s.wl * th)));
  GemmArgs g2 = gemm(s.d1 * s.wc, (int)n2, s.wl * s.d1, s.Dl, 1,
                     op(W1m, (long)s.d1 * s.wc * s.wl * s.d1, 0, 0, (long)s.wl * s.d1, 0, 0),
                     op(XA, (long)s.wl * th, (long)s.wl * n1, 0, n2, 0, 0), XB, (long)s.wc * th,
                     (long)s.wc * n1, n2);
  g2.B.f32 = f32;
  g2.c_f32 = f32;
  if (prof) TRY(prof_begin(ctx, &pe, 1));
  TRY_HIP(tuned_cgemm(ctx, g2, ar, ctx->stream));
  if (prof)  // algorithmic work counts the stored nonzeros, as for the sparse pass
    TRY(prof_end(ctx, pe, 8.0 * (double)W1->f_nnz * s.d2 * s.Dl * s.Dr, cb * ((double)s.wl + s.wc) * th));
  GemmArgs g3 = gemm(s.wr * s.d2, s.Dr, s.wc * s.d2, s.Dl * s.d1, 1,
                     op(W2m, (long)s.wr * s.d2 * s.wc * s.d2, 0, 0, (long)s.wc * s.d2, 0, 0),
                     op(XB, (long)s.wc * th, (long)s.wc * n2, 0, s.Dr, 0, 0), XA, (long)s.wr * th, n2, s.Dr);
  g3.c_mi = s.d2;
  g3.c_so = th;
  g3.B.f32 = f32;
  g3.c_f32 = f32;
  if (prof) TRY(prof_begin(ctx, &pe, 2));
  TRY_HIP(tuned_cgemm(ctx, g3, ar, ctx->stream));
  if (prof)
    TRY(prof_end(ctx, pe, 8.0 * (double)W2->f_nnz * s.d1 * s.Dl * s.Dr, cb * ((double)s.wc + s.wr) * th));
  const int M4 = s.Dl * s.d1 * s.d2;
  GemmArgs g4 = gemm(M4, s.Dr, s.Dr, 1, s.wr, op(XA, (long)s.wr * th, 0, th, s.Dr, 0, 0),
                     op(R, (long)s.wr * s.Dr * s.Dr, 0, (long)s.Dr * s.Dr, s.Dr, 1, 0), y, th, 0, s.Dr);
  g4.role = prof ? 2 : 0;
  g4.A.f32 = f32;
  if (prof) TRY(prof_begin(ctx, &pe, 3));
  TRY_HIP(tuned_cgemm(ctx, g4, ar, ctx->stream));
  if (prof)
    TRY(prof_end(ctx, pe, 8.0 * s.wr * s.Dr * (double)s.Dr * M4,
                 cb * ((double)s.wr * s.Dr * s.Dr + (double)s.wr * th + th)));
  return TDMRG_OK;
}

static tdmrg_status heff2_fused(tdmrg_ctx* ctx, const tdmrg_heff_shape& s, const double* L,
                                const tdmrg_wop* W1, const tdmrg_wop* W2, const PairOp* W12, const double* R,
                                const double* theta, double* y, Arith ar) {
  const long th = (long)s.Dl * s.d1 * s.d2 * s.Dr;
  TRY(ensure(ctx, ctx->xa, sizeof(double) * 2 * (size_t)s.wl * th));
  TRY(ensure(ctx, ctx->xb, sizeof(double) * 2 * (size_t)s.wr * th));
  double* XA = (double*)ctx->xa.p;
  double* XB = (double*)ctx->xb.p;
  const bool prof = ctx->prof.on;
  Profiler::Pending pe;
  const double cb = 16.0;
  const int N1 = s.d1 * s.d2 * s.Dr;
  const bool in_gemm = ctx->mix_in_gemm && (ar == Arith::F64 || ar == Arith::F32);  // no BF16 form
  // mixed forms keep the intermediates in FP32 (the mix in the loader reads FP64)
  const int f32 = ar != Arith::F64 && !in_gemm;
  // X1[wl][a][s'][t'][b'] = sum_a' L[wl][a][a'] theta[a'][s'][t'][b']
  GemmArgs g1 = gemm(s.wl * s.Dl, N1, s.Dl, 1, 1, op(L, (long)s.wl * s.Dl * s.Dl, 0, 0, s.Dl, 0, 0),
                     op(theta, th, 0, 0, N1, 0, 0), XA, (long)s.wl * th, 0, N1);
  g1.role = prof ? 1 : 0;  // own kernel name only inside a profiled region
  g1.c_f32 = f32;
  if (prof) TRY(prof_begin(ctx, &pe, 0));
  TRY_HIP(tuned_cgemm(ctx, g1, ar, ctx->stream));
  if (prof)
    TRY(prof_end(ctx, pe, 8.0 * s.wl * s.Dl * (double)s.Dl * N1,
                 cb * ((double)s.wl * s.Dl * s.Dl + th + (double)s.wl * th)));
  const int M4 = s.Dl * s.d1 * s.d2;
  if (in_gemm) {
    // y[a][s][t][b] = sum_{wr,b'} (sum_{wl,s',t'} W12[wl][wr][(s,t)][(s',t')] X1[wl][a][s'][t'][b']) R[wr][b][b']:
    // the channel mix is formed tile by tile in the A loader of the last GEMM
    GemmArgs g4 = gemm(M4, s.Dr, s.Dr, 1, s.wr, op(XA, (long)s.wl * th, 0, 0, s.Dr, 0, 0),
                       op(R, (long)s.wr * s.Dr * s.Dr, 0, (long)s.Dr * s.Dr, s.Dr, 1, 0), y, th, 0, s.Dr);
    g4.role = 3;
    g4.mx_rowptr = W12->rowptr;
    g4.mx_col = W12->col;
    g4.mx_v = W12->v;
    g4.mx_nnz = W12->nnz;
    g4.mx_din = s.d1 * s.d2;
    g4.mx_dout = s.d1 * s.d2;
    g4.mx_ws = th;
    if (prof) TRY(prof_begin(ctx, &pe, 3));
    TRY_HIP(tuned_cgemm(ctx, g4, ar, ctx->stream));
    if (prof)
      TRY(prof_end(ctx, pe,
                   8.0 * s.wr * s.Dr * (double)s.Dr * M4 +
                       8.0 * ((double)W1->f_nnz * s.d2 + (double)W2->f_nnz * s.d1) * s.Dl * s.Dr,
                   cb * ((double)s.wr * s.Dr * s.Dr + (double)s.wl * th + th)));
    return TDMRG_OK;
  }
  // X3[wr][a][s][t][b'] = sum_{wl,s',t'} W12[wl][wr][(s,t)][(s',t')] X1[wl][a][s'][t'][b']
  MixArgs m;
  m.in = XA; m.in_im = (long)s.wl * th; m.out = XB; m.out_im = (long)s.wr * th;
  m.P = s.Dl; m.Q = s.Dr; m.din = s.d1 * s.d2; m.dout = s.d1 * s.d2; m.nout = s.wr;
  m.rowptr = W12->rowptr; m.col = W12->col; m.vre = W12->v; m.vim = W12->v + W12->nnz;
  m.blk = W12->blk.view();
  m.f32 = f32;
  if (prof) TRY(prof_begin(ctx, &pe, 1));
  TRY_HIP(launch_mix(m, ctx->stream));
  if (prof)  // algorithmic work of the two channel stages (stored nonzeros of W_i, W_{i+1})
    TRY(prof_end(ctx, pe, 8.0 * ((double)W1->f_nnz * s.d2 + (double)W2->f_nnz * s.d1) * s.Dl * s.Dr,
                 cb * ((double)s.wl + s.wr) * th));
  // y[a][s][t][b] = sum_{wr,b'} X3[wr][a][s][t][b'] R[wr][b][b']
  GemmArgs g4 = gemm(M4, s.Dr, s.Dr, 1, s.wr, op(XB, (long)s.wr * th, 0, th, s.Dr, 0, 0),
                     op(R, (long)s.wr * s.Dr * s.Dr, 0, (long)s.Dr * s.Dr, s.Dr, 1, 0), y, th, 0, s.Dr);
  g4.role = prof ? 2 : 0;
  g4.A.f32 = f32;
  if (prof) TRY(prof_begin(ctx, &pe, 3));
  TRY_HIP(tuned_cgemm(ctx, g4, ar, ctx->stream));
  if (prof)
    TRY(prof_end(ctx, pe, 8.0 * s.wr * s.Dr * (double)s.Dr * M4,
                 cb * ((double)s.wr * s.Dr * s.Dr + (double)s.wr * th + th)));
  return TDMRG_OK;
}

tdmrg_status heff2(tdmrg_ctx* ctx, const tdmrg_heff_shape& s, const double* L, const tdmrg_wop* W1,
                   const tdmrg_wop* W2, const double* R, const double* theta, double* y, Arith ar) {
  const long th = (long)s.Dl * s.d1 * s.d2 * s.Dr;
  if (channel_gemm_pays(ctx, s, W1, W2)) return heff2_dense(ctx, s, L, W1, W2, R, theta, y, ar);
  const PairOp* W12 = nullptr;
  TRY(pair_op(ctx, W1, W2, &W12));
  if (W12) return heff2_fused(ctx, s, L, W1, W2, W12, R, theta, y, ar);
  const int wmax = std::max(s.wl, s.wr);
  TRY(ensure(ctx, ctx->xa, sizeof(double) * 2 * (size_t)wmax * th));
  TRY(ensure(ctx, ctx->xb, sizeof(double) * 2 * (size_t)s.wc * th));
  double* XA = (double*)ctx->xa.p;
  double* XB = (double*)ctx->xb.p;
  const bool prof = ctx->prof.on;
  Profiler::Pending pe;
  const double cb = 16.0;  // bytes per FP64 complex
  const int N1 = s.d1 * s.d2 * s.Dr;
  const int f32 = ar != Arith::F64;  // mixed forms keep the intermediates in FP32
  // X1[wl][a][s'][t'][b'] = sum_a' L[wl][a][a'] theta[a'][s'][t'][b']   (L channels stacked as rows)
  GemmArgs g1 = gemm(s.wl * s.Dl, N1, s.Dl, 1, 1, op(L, (long)s.wl * s.Dl * s.Dl, 0, 0, s.Dl, 0, 0),
                     op(theta, th, 0, 0, N1, 0, 0), XA, (long)s.wl * th, 0, N1);
  g1.role = prof ? 1 : 0;  // own kernel name only inside a profiled region
  g1.c_f32 = f32;
  if (prof) TRY(prof_begin(ctx, &pe, 0));
  TRY_HIP(tuned_cgemm(ctx, g1, ar, ctx->stream));
  if (prof)
    TRY(prof_end(ctx, pe, 8.0 * s.wl * s.Dl * (double)s.Dl * N1,
                 cb * ((double)s.wl * s.Dl * s.Dl + th + (double)s.wl * th)));
  // X2[wc][a][s][t'][b'] = sum_{wl,s'} W1[wl][wc][s][s'] X1[wl][a][s'][t'][b']
  if (prof) TRY(prof_begin(ctx, &pe, 1));
  MixArgs m1 = mix_fwd(W1, XA, (long)s.wl * th, XB, (long)s.wc * th, s.Dl, s.d2 * s.Dr);
  m1.f32 = f32;
  TRY_HIP(launch_mix(m1, ctx->stream));
  if (prof)
    TRY(prof_end(ctx, pe, 8.0 * W1->f_nnz * (double)s.Dl * s.d2 * s.Dr,
                 cb * ((double)s.wl + s.wc) * th));
  // X3[wr][a][s][t][b'] = sum_{wc,t'} W2[wc][wr][t][t'] X2[wc][a][s][t'][b']
  if (prof) TRY(prof_begin(ctx, &pe, 2));
  MixArgs m2 = mix_fwd(W2, XB, (long)s.wc * th, XA, (long)s.wr * th, s.Dl * s.d1, s.Dr);
  m2.f32 = f32;
  TRY_HIP(launch_mix(m2, ctx->stream));
  if (prof)
    TRY(prof_end(ctx, pe, 8.0 * W2->f_nnz * (double)s.Dl * s.d1 * s.Dr,
                 cb * ((double)s.wc + s.wr) * th));
  // y[a][s][t][b] = sum_{wr,b'} X3[wr][a][s][t][b'] R[wr][b][b']
  const int M4 = s.Dl * s.d1 * s.d2;
  GemmArgs g4 = gemm(M4, s.Dr, s.Dr, 1, s.wr, op(XA, (long)s.wr * th, 0, th, s.Dr, 0, 0),
                     op(R, (long)s.wr * s.Dr * s.Dr, 0, (long)s.Dr * s.Dr, s.Dr, 1, 0), y, th, 0, s.Dr);
  g4.role = prof ? 2 : 0;
  g4.A.f32 = f32;
  if (prof) TRY(prof_begin(ctx, &pe, 3));
  TRY_HIP(tuned_cgemm(ctx, g4, ar, ctx->stream));
  if (prof)
    TRY(prof_end(ctx, pe, 8.0 * s.wr * s.Dr * (double)s.Dr * M4,
                 cb * ((double)s.wr * s.Dr * s.Dr + (double)s.wr * th + th)));
  return TDMRG_OK;
}

tdmrg_status heff2_rect(tdmrg_ctx* ctx, int Dlo, int Dli, int d1, int d2, int Dro, int Dri, const double* L,
                        const tdmrg_wop* W1, const tdmrg_wop* W2, const double* R, const double* theta, double* out,
                        double alpha_re, double alpha_im, double beta) {
  const int wl = W1->wl, wc = W1->wr, wr = W2->wr;
  const long tho = (long)Dlo * d1 * d2 * Dri;  // one channel of the intermediates
  const int wmax = std::max(wl, wr);
  TRY(ensure(ctx, ctx->xa, sizeof(double) * 2 * (size_t)wmax * tho));
  TRY(ensure(ctx, ctx->xb, sizeof(double) * 2 * (size_t)wc * tho));
  double* XA = (double*)ctx->xa.p;
  double* XB = (double*)ctx->xb.p;
  const int N1 = d1 * d2 * Dri;
  // X1[wl][a][s'][t'][b'] = sum_a' L[wl][a][a'] theta[a'][s'][t'][b']
  GemmArgs g1 = gemm(wl * Dlo, N1, Dli, 1, 1, op(L, (long)wl * Dlo * Dli, 0, 0, Dli, 0, 0),
                     op(theta, (long)Dli * N1, 0, 0, N1, 0, 0), XA, (long)wl * tho, 0, N1);
  TRY_HIP(tuned_cgemm(ctx, g1, Arith::F64, ctx->stream));
  // X2[wc][a][s][t'][b'], X3[wr][a][s][t][b']: the two channel stages
  TRY_HIP(launch_mix(mix_fwd(W1, XA, (long)wl * tho, XB, (long)wc * tho, Dlo, d2 * Dri), ctx->stream));
  TRY_HIP(launch_mix(mix_fwd(W2, XB, (long)wc * tho, XA, (long)wr * tho, Dlo * d1, Dri), ctx->stream));
  // out[a][s][t][b] = alpha sum_{wr,b'} X3[wr][a][s][t][b'] R[wr][b][b'] + beta out
  const int M4 = Dlo * d1 * d2;
  GemmArgs g4 = gemm(M4, Dro, Dri, 1, wr, op(XA, (long)wr * tho, 0, tho, Dri, 0, 0),
                     op(R, (long)wr * Dro * Dri, 0, (long)Dro * Dri, Dri, 1, 0), out, (long)M4 * Dro, 0, Dro);
  g4.alpha_re = alpha_re;
  g4.alpha_im = alpha_im;
  g4.beta_re = beta;
  TRY_HIP(tuned_cgemm(ctx, g4, Arith::F64, ctx->stream));
  return TDMRG_OK;
}

tdmrg_status heff1(tdmrg_ctx* ctx, int Dl, int d, int Dr, const double* L, const tdmrg_wop* W,
                   const double* R, const double* M, double* y, Arith ar) {
  const int wl = W->wl, wr = W->wr;
  const long th = (long)Dl * d * Dr;
  TRY(ensure(ctx, ctx->xa, sizeof(double) * 2 * (size_t)wl * th));
  TRY(ensure(ctx, ctx->xb, sizeof(double) * 2 * (size_t)wr * th));
  double* XA = (double*)ctx->xa.p;
  double* XB = (double*)ctx->xb.p;
  const int N1 = d * Dr;
  GemmArgs g1 = gemm(wl * Dl, N1, Dl, 1, 1, op(L, (long)wl * Dl * Dl, 0, 0, Dl, 0, 0),
                     op(M, th, 0, 0, N1, 0, 0), XA, (long)wl * th, 0, N1);
  TRY_HIP(tuned_cgemm(ctx, g1, ar, ctx->stream));
  TRY_HIP(launch_mix(mix_fwd(W, XA, (long)wl * th, XB, (long)wr * th, Dl, Dr), ctx->stream));
  GemmArgs g2 = gemm(Dl * d, Dr, Dr, 1, wr, op(XB, (long)wr * th, 0, th, Dr, 0, 0),
                     op(R, (long)wr * Dr * Dr, 0, (long)Dr * Dr, Dr, 1, 0), y, th, 0, Dr);
  TRY_HIP(tuned_cgemm(ctx, g2, ar, ctx->stream));
  return TDMRG_OK;
}

// y[a][b] = sum_{w,a',b'} L[w][a][a'] C[a'][b'] R[w][b][b'] (eq. zero-site
// Hamiltonian): the two environments meet on the MPO bond between them; the
// one-site product without its site, so two GEMM stages and no channel mix.
tdmrg_status heff0(tdmrg_ctx* ctx, int Dl, int Dr, int w, const double* L, const double* R, const double* C,
                   double* y, Arith ar) {
  const long th = (long)Dl * Dr;
  TRY(ensure(ctx, ctx->xa, sizeof(double) * 2 * (size_t)w * th));
  double* XA = (double*)ctx->xa.p;
  GemmArgs g1 = gemm(w * Dl, Dr, Dl, 1, 1, op(L, (long)w * Dl * Dl, 0, 0, Dl, 0, 0), op(C, th, 0, 0, Dr, 0, 0), XA,
                     (long)w * th, 0, Dr);
  TRY_HIP(tuned_cgemm(ctx, g1, ar, ctx->stream));
  GemmArgs g2 = gemm(Dl, Dr, Dr, 1, w, op(XA, (long)w * th, 0, th, Dr, 0, 0),
                     op(R, (long)w * Dr * Dr, 0, (long)Dr * Dr, Dr, 1, 0), y, th, 0, Dr);
  TRY_HIP(tuned_cgemm(ctx, g2, ar, ctx->stream));
  return TDMRG_OK;
}

tdmrg_status env_left(tdmrg_ctx* ctx, const double* Lin, const tdmrg_wop* W, const double* bra,
                      int Db, int Db2, const double* ket, int Dk, int Dk2, double* Lout, Arith ar) {
  const int wl = W->wl, wr = W->wr, d = W->d;
  const long tk = (long)Db * d * Dk2;  // one channel of T1/T2
  TRY(ensure(ctx, ctx->xa, sizeof(double) * 2 * (size_t)wl * tk));
  TRY(ensure(ctx, ctx->xb, sizeof(double) * 2 * (size_t)wr * tk));
  double* XA = (double*)ctx->xa.p;
  double* XB = (double*)ctx->xb.p;
  const int N1 = d * Dk2;
  // T1[w][b][s'][a'] = sum_b' Lin[w][b][b'] ket[b'][s'][a']
  GemmArgs g1 = gemm(wl * Db, N1, Dk, 1, 1, op(Lin, (long)wl * Db * Dk, 0, 0, Dk, 0, 0),
                     op(ket, (long)Dk * N1, 0, 0, N1, 0, 0), XA, (long)wl * tk, 0, N1);
  TRY_HIP(tuned_cgemm(ctx, g1, ar, ctx->stream));
  // T2[w'][b][s][a'] = sum_{w,s'} W[w][w'][s][s'] T1[w][b][s'][a']
  TRY_HIP(launch_mix(mix_fwd(W, XA, (long)wl * tk, XB, (long)wr * tk, Db, Dk2), ctx->stream));
  // Lout[w'][a][a'] = sum_{b,s} conj(bra[b][s][a]) T2[w'][b][s][a']
  GemmArgs g3 = gemm(Db2, Dk2, Db * d, wr, 1, op(bra, (long)Db * d * Db2, 0, 0, Db2, 1, 1),
                     op(XB, (long)wr * tk, tk, 0, Dk2, 0, 0), Lout, (long)wr * Db2 * Dk2,
                     (long)Db2 * Dk2, Dk2);
  TRY_HIP(tuned_cgemm(ctx, g3, ar, ctx->stream));
  return TDMRG_OK;
}

tdmrg_status env_right(tdmrg_ctx* ctx, const double* Rin, const tdmrg_wop* W, const double* bra,
                       int Db, int Db2, const double* ket, int Dk, int Dk2, double* Rout, Arith ar) {
  const int wl = W->wl, wr = W->wr, d = W->d;
  const long tk = (long)Dk * d * Db2;  // one channel of T1/T2: [a'][s][b]
  TRY(ensure(ctx, ctx->xa, sizeof(double) * 2 * (size_t)wr * tk));
  TRY(ensure(ctx, ctx->xb, sizeof(double) * 2 * (size_t)wl * tk));
  double* XA = (double*)ctx->xa.p;
  double* XB = (double*)ctx->xb.p;
  // T1[x][a'][s'][b] = sum_b' ket[a'][s'][b'] Rin[x][b][b']
  GemmArgs g1 = gemm(Dk * d, Db2, Dk2, wr, 1, op(ket, (long)Dk * d * Dk2, 0, 0, Dk2, 0, 0),
                     op(Rin, (long)wr * Db2 * Dk2, (long)Db2 * Dk2, 0, Dk2, 1, 0), XA, (long)wr * tk,
                     tk, Db2);
  TRY_HIP(tuned_cgemm(ctx, g1, ar, ctx->stream));
  // T2[w][a'][s][b] = sum_{x,s'} W[w][x][s][s'] T1[x][a'][s'][b]
  TRY_HIP(launch_mix(mix_bwd(W, XA, (long)wr * tk, XB, (long)wl * tk, Dk, Db2), ctx->stream));
  // Rout[w][a][a'] = sum_{s,b} conj(bra[a][s][b]) T2[w][a'][s][b]
  const int K = d * Db2;
  GemmArgs g3 = gemm(Db, Dk, K, wl, 1, op(bra, (long)Db * K, 0, 0, K, 0, 1),
                     op(XB, (long)wl * tk, tk, 0, K, 1, 0), Rout, (long)wl * Db * Dk, (long)Db * Dk, Dk);
  TRY_HIP(tuned_cgemm(ctx, g3, ar, ctx->stream));
  return TDMRG_OK;
}

tdmrg_status theta_form(tdmrg_ctx* ctx, int Dl, int d1, int Dm, int d2, int Dr, const double* M,
                        const double* B, double* theta) {
  const int Mr = Dl * d1, N = d2 * Dr;
  GemmArgs g = gemm(Mr, N, Dm, 1, 1, op(M, (long)Mr * Dm, 0, 0, Dm, 0, 0),
                    op(B, (long)Dm * N, 0, 0, N, 0, 0), theta, (long)Mr * N, 0, N);
  TRY_HIP(tuned_cgemm(ctx, g, Arith::F64, ctx->stream));
  return TDMRG_OK;
}

// Layout of the small scalar workspace (doubles).
struct Small {
  double *alpha, *beta, *cr, *ci, *dre, *dim, *c_re, *c_im, *err, *beta0, *part_re, *part_im;
  int* ik;
  int* jd;  // device Lanczos step counter
  double* disc;
};
static constexpr int kMaxKrylov = 64;
static constexpr int kPartStride = 1024;

static tdmrg_status small_ws_in(tdmrg_ctx* ctx, DevBuf& buf, Small* sm) {
  const size_t nd = 16 * kMaxKrylov + 2 * (size_t)kMaxKrylov * kPartStride + 64;
  TRY(ensure(ctx, buf, nd * sizeof(double)));
  double* p = (double*)buf.p;
  sm->alpha = p; p += kMaxKrylov;
  sm->beta = p; p += kMaxKrylov;
  sm->cr = p; p += kMaxKrylov;
  sm->ci = p; p += kMaxKrylov;
  sm->dre = p; p += kMaxKrylov;
  sm->dim = p; p += kMaxKrylov;
  sm->c_re = p; p += kMaxKrylov;
  sm->c_im = p; p += kMaxKrylov;
  sm->err = p; p += 8;
  sm->beta0 = p; p += 8;
  sm->disc = p; p += 8;
  sm->ik = (int*)p;
  sm->jd = sm->ik + 8;
  p += 8;
  p += 8 * kMaxKrylov - 48;  // keep the partial-sum area aligned
  sm->part_re = p; p += (size_t)kMaxKrylov * kPartStride;
  sm->part_im = p;
  return TDMRG_OK;
}

static tdmrg_status small_ws(tdmrg_ctx* ctx, Small* sm) { return small_ws_in(ctx, ctx->small, sm); }

// out_re[j], out_im[j] = <V_j, w> for j < nv (fixed-order reduction)
static tdmrg_status dots(tdmrg_ctx* ctx, const Small& sm, const double* V, long vstride, int nv,
                         long n, const double* w, double* out_re, double* out_im, int mode) {
  TRY_HIP(launch_multidot(V, vstride, nv, n, w, sm.part_re, sm.part_im, ctx->stream));
  TRY_HIP(launch_reduce_partials(sm.part_re, sm.part_im, nv, dot_chunks(n), out_re, out_im, mode,
                                 ctx->stream));
  return TDMRG_OK;
}

// Lanczos basis of (H, x) for exp(-i tau H) x: V (m_max planar vectors of
// the problem size, stride 2n) and the scalars in sm (alpha, beta, beta0 =
// |x|, and c = exp(-i tau T_m) e1 of the last step); *m = basis size.  w
// holds two vectors: the work vector and X, the operand of the H products
// (a copy of the current basis vector, so that every step reads the same
// addresses).  The kernels of a step take the step index j from a device
// counter, so one step's launches are identical for every j: with graphs
// enabled they are captured once per operand set and replayed.
// sites = 2: H_eff,2 on a two-site tensor; 1: H_eff,1 (shape d2 unused);
// 0: H_eff,0 on a Dl x Dr bond matrix (d1 = d2 = 1, wl = wr = the MPO bond).
static tdmrg_status lanczos_core(tdmrg_ctx* ctx, const tdmrg_heff_shape& s, int sites, const double* L,
                                 const tdmrg_wop* W1, const tdmrg_wop* W2, const double* R, const double* x,
                                 double tau, double tol, int m_max, Arith ar, double* V, double* w, const Small& sm,
                                 ExpmResult* res, int* m) {
  const long n = sites == 2 ? (long)s.Dl * s.d1 * s.d2 * s.Dr : (long)s.Dl * s.d1 * s.Dr;
  const long vs = 2 * n;
  double* X = w + vs;
  hipStream_t st = ctx->stream;  // the capture below points it (and ctx->stream) elsewhere for a moment
  // beta0 = ||x||, v_0 = x / beta0 (also the first operand X)
  TRY(dots(ctx, sm, x, vs, 1, n, x, sm.beta0, nullptr, 1));
  TRY_HIP(launch_scale_by_inv(x, n, sm.beta0, V, st));
  TRY_HIP(launch_scale_by_inv(x, n, sm.beta0, X, st));
  TRY_HIP(launch_counter_set(sm.jd, 0, st));
  const int nchunk = dot_chunks(n);
  // one step at j = *jd: w = H X; two classical Gram-Schmidt passes against
  // v_0 .. v_j (the first pass's coefficient of v_j is <v_j, H v_j>, so
  // alpha_j is its real part and the three-term step is contained in it; the
  // second pass also yields beta_j = ||w||); exp(-i tau T_{j+1}) e1 and the
  // error estimate (read back); the next basis vector; j += 1.
  auto step = [&]() -> tdmrg_status {
    if (sites == 2) TRY(heff2(ctx, s, L, W1, W2, R, X, w, ar));
    else if (sites == 1) TRY(heff1(ctx, s.Dl, s.d1, s.Dr, L, W1, R, X, w, ar));
    else TRY(heff0(ctx, s.Dl, s.Dr, s.wl, L, R, X, w, ar));
    TRY_HIP(launch_multidot_dev(V, vs, sm.jd, m_max, n, w, sm.part_re, sm.part_im, 0, st));
    TRY_HIP(launch_reduce_partials_dev(sm.part_re, sm.part_im, sm.jd, m_max, nchunk, sm.cr, sm.ci, 0, st));
    TRY_HIP(launch_copy_scalar_dev(sm.cr, sm.alpha, sm.jd, st));
    // first pass's update and second pass's dots: fused (one read of the
    // basis) up to kGsFusedMax vectors, separate kernels beyond; each kernel
    // checks the count on the device, so the step's launches stay fixed
    TRY_HIP(launch_gs_fused_dev(V, vs, sm.jd, n, sm.cr, sm.ci, w, sm.part_re, sm.part_im, st));
    TRY_HIP(launch_multiaxpy_dev(V, vs, sm.jd, n, sm.cr, sm.ci, w, kGsFusedMax + 1, st));
    TRY_HIP(launch_multidot_dev(V, vs, sm.jd, m_max, n, w, sm.part_re, sm.part_im, kGsFusedMax + 1, st));
    TRY_HIP(launch_reduce_partials_dev(sm.part_re, sm.part_im, sm.jd, m_max, nchunk, sm.cr, sm.ci, 0, st));
    TRY_HIP(launch_multiaxpy_norm_dev(V, vs, sm.jd, n, sm.cr, sm.ci, w, sm.part_re, sm.beta, st));
    TRY_HIP(launch_tridiag_expm_dev(sm.alpha, sm.beta, sm.jd, tau, sm.c_re, sm.c_im, sm.err, st));
    TRY_HIP(hipMemcpyAsync(ctx->host, sm.err, sizeof(double), hipMemcpyDeviceToHost, st));
    TRY_HIP(launch_lanczos_next(w, n, sm.beta, V, vs, X, sm.jd, m_max, st));
    TRY_HIP(launch_counter_add(sm.jd, 1, st));
    return TDMRG_OK;
  };
  // graph of one step, by operand set (shapes, operators, environments,
  // buffers, tau); profiling runs every step eagerly
  const bool use_graph = ctx->graphs && !ctx->prof.on;
  hipGraphExec_t exec = nullptr;
  std::vector<long> key;
  if (use_graph) {
    graphs_sweep(ctx);
    long tb;
    std::memcpy(&tb, &tau, sizeof(tb));
    key = {(long)sites, s.Dl, s.d1, s.d2, s.Dr, s.wl, s.wc, s.wr, (long)L, (long)W1, (long)W2, (long)R,
           (long)V, (long)w, (long)sm.alpha, tb, (long)ar, m_max, ctx->fuse_mode, ctx->chan_gemm};
    auto it = ctx->lgraphs.find(key);
    if (it != ctx->lgraphs.end()) exec = it->second.exec;
  }
  res->iters = 0;
  res->converged = false;
  for (int j = 0; j < m_max; ++j) {
    if (exec) {
      TRY_HIP(hipGraphLaunch(exec, st));
      ctx->graph_counts[1]++;
    } else {
      TRY(step());
      ctx->graph_counts[2]++;
    }
    TRY_HIP(hipStreamSynchronize(st));
    if (ctx->prof.on) TRY(prof_flush(ctx));
    const double err = ctx->host[0];
    res->iters = j + 1;
    if (!(err == err)) return fail(ctx, TDMRG_EINVAL, "Lanczos produced NaN (non-finite input?)");
    if (err <= tol || j == m_max - 1) {
      res->converged = err <= tol;
      *m = j + 1;
      return TDMRG_OK;
    }
    if (use_graph && !exec && ctx->lgraphs.find(key) == ctx->lgraphs.end()) {
      // the eager step has sized every buffer and tuned every GEMM class of
      // this operand set: capture the step (nothing runs) and replay it.  An
      // epoch advance during the eager step dropped no graph of this key.
      // The step's launches are recorded on the context's own capture
      // stream (the caller's stream may be the null stream, which cannot be
      // captured); the graph is then launched on the caller's stream.
      graphs_sweep(ctx);
      hipGraph_t g = nullptr;
      hipGraphExec_t e = nullptr;
      bool ok = ctx->cap_stream || hipStreamCreate(&ctx->cap_stream) == hipSuccess;
      const hipStream_t real = st;
      if (ok) ok = hipStreamBeginCapture(ctx->cap_stream, hipStreamCaptureModeRelaxed) == hipSuccess;
      if (ok) {
        st = ctx->stream = ctx->cap_stream;
        const tdmrg_status cs = step();
        st = ctx->stream = real;
        ok = (hipStreamEndCapture(ctx->cap_stream, &g) == hipSuccess) && cs == TDMRG_OK && g;
        if (ok) ok = hipGraphInstantiate(&e, g, nullptr, nullptr, 0) == hipSuccess;
        if (g) (void)hipGraphDestroy(g);
      }
      (void)hipGetLastError();
      if (ok) {
        ctx->lgraphs[key] = {e, graph_epoch()};
        ctx->graph_counts[0]++;
        exec = e;
      } else {
        if (e) (void)hipGraphExecDestroy(e);
        ctx->lgraphs[key] = {nullptr, graph_epoch()};  // not capturable: eager
      }
    }
  }
  *m = m_max;
  return TDMRG_OK;
}

tdmrg_status local_expm(tdmrg_ctx* ctx, const tdmrg_heff_shape& s, bool two_site, const double* L,
                        const tdmrg_wop* W1, const tdmrg_wop* W2, const double* R, double* theta,
                        double tau, double tol, int m_max, Arith ar, ExpmResult* res) {
  return local_expm_sites(ctx, s, two_site ? 2 : 1, L, W1, W2, R, theta, tau, tol, m_max, ar, res);
}

tdmrg_status local_expm0(tdmrg_ctx* ctx, int Dl, int Dr, int w, const double* L, const double* R, double* C,
                         double tau, double tol, int m_max, Arith ar, ExpmResult* res) {
  const tdmrg_heff_shape s{Dl, 1, 1, Dr, w, 1, w};
  return local_expm_sites(ctx, s, 0, L, nullptr, nullptr, R, C, tau, tol, m_max, ar, res);
}

tdmrg_status local_expm_sites(tdmrg_ctx* ctx, const tdmrg_heff_shape& s, int sites, const double* L,
                              const tdmrg_wop* W1, const tdmrg_wop* W2, const double* R, double* theta,
                              double tau, double tol, int m_max, Arith ar, ExpmResult* res) {
  const long n = sites == 2 ? (long)s.Dl * s.d1 * s.d2 * s.Dr : (long)s.Dl * s.d1 * s.Dr;
  const long vs = 2 * n;
  m_max = std::min(std::max(m_max, 1), kMaxKrylov);
  Small sm;
  TRY(small_ws(ctx, &sm));
  TRY(ensure(ctx, ctx->kry, sizeof(double) * (size_t)vs * m_max));
  TRY(ensure(ctx, ctx->wvec, sizeof(double) * 2 * (size_t)vs));  // work vector and operand
  double* V = (double*)ctx->kry.p;
  int m = 0;
  TRY(lanczos_core(ctx, s, sites, L, W1, W2, R, theta, tau, tol, m_max, ar, V, (double*)ctx->wvec.p, sm, res, &m));
  // theta = beta0 * sum_k c_k v_k
  TRY_HIP(launch_combine(V, vs, m, n, sm.c_re, sm.c_im, sm.beta0, theta, ctx->stream));
  return TDMRG_OK;
}

tdmrg_status expm_basis(tdmrg_ctx* ctx, const tdmrg_heff_shape& s, const double* L, const tdmrg_wop* W1,
                        const tdmrg_wop* W2, const double* R, const double* x, double tau, double tol, int m_max,
                        DevBuf& Vbuf, DevBuf& wbuf, DevBuf& sbuf, KrylovBasis* kb) {
  const long n = (long)s.Dl * s.d1 * s.d2 * s.Dr;
  const long vs = 2 * n;
  m_max = std::min(std::max(m_max, 1), kMaxKrylov);
  Small sm;
  TRY(small_ws_in(ctx, sbuf, &sm));
  TRY(ensure(ctx, Vbuf, sizeof(double) * (size_t)vs * m_max));
  TRY(ensure(ctx, wbuf, sizeof(double) * 2 * (size_t)vs));  // work vector and operand
  ExpmResult r;
  kb->V = (double*)Vbuf.p;
  kb->n = n;
  TRY(lanczos_core(ctx, s, 2, L, W1, W2, R, x, tau, tol, m_max, Arith::F64, kb->V, (double*)wbuf.p, sm, &r,
                   &kb->m));
  kb->alpha = sm.alpha;
  kb->beta = sm.beta;
  kb->beta0 = sm.beta0;
  kb->c_re = sm.c_re;
  kb->c_im = sm.c_im;
  kb->err = sm.err;
  return TDMRG_OK;
}

tdmrg_status expm_from_basis(tdmrg_ctx* ctx, const KrylovBasis& kb, double tau, double* out) {
  hipStream_t st = ctx->stream;
  TRY_HIP(launch_tridiag_expm(kb.alpha, kb.beta, kb.m, tau, kb.c_re, kb.c_im, kb.err, st));
  TRY_HIP(launch_combine(kb.V, 2 * kb.n, kb.m, kb.n, kb.c_re, kb.c_im, kb.beta0, out, st));
  return TDMRG_OK;
}

// Hermitian eigenproblem of a planar b x b matrix C (read only; Cw holds the
// interleaved copy rocSOLVER works on): W[i][j] = component i of the eigenvector of the j-th
// largest eigenvalue; lam ascending (rocSOLVER order).
tdmrg_status heev_values(tdmrg_ctx* ctx, const double* C, int n, double* lam, int* info) {
  hipStream_t st = ctx->stream;
  if (n < 1 || n > kHeevMax) return fail(ctx, TDMRG_ESHAPE, "heev: order out of range");
  TRY(ensure(ctx, ctx->heev, heev_bytes(n)));
  const long nn = (long)n * n;
  double* A = (double*)ctx->heev.p;
  double* V = A + 2 * nn;
  double* Z = V + 2 * nn;
  double* tau = Z + nn;
  double* e = tau + 2 * n;
  TRY_HIP(launch_hetrd(C, n, A, V, lam, e, tau, st));
  if (n == 1) {
    TRY_HIP(launch_fill(Z, 1, 1.0, st));
    TRY_HIP(hipMemsetAsync(info, 0, sizeof(int), st));
    return TDMRG_OK;
  }
  TRY(rocws_reserve(ctx, rocsolver_ws_bound(n)));
  rocblas_status rs = rocsolver_dstedc(ctx->blas, rocblas_evect_tridiagonal, n, lam, e, Z, n, info);
  if (rs != rocblas_status_success)
    return fail(ctx, TDMRG_EDEVICE, "rocsolver_dstedc failed with status " + std::to_string((int)rs));
  return TDMRG_OK;
}

tdmrg_status heev_vectors(tdmrg_ctx* ctx, int n, int k, int transpose, int conj, double* out) {
  if (k < 1) return TDMRG_OK;
  const long nn = (long)n * n;
  const double* V = (const double*)ctx->heev.p + 2 * nn;
  const double* Z = V + 2 * nn;
  const double* tau = Z + nn;
  TRY_HIP(launch_unmtr(V, tau, Z, n, k, transpose, conj, out, ctx->stream));
  return TDMRG_OK;
}

// Eigenpairs of the b x b Rayleigh quotient C (planar row-major): lam
// ascending, W[i][j] = component i of the eigenvector of the j-th largest.
static tdmrg_status heevd_small(tdmrg_ctx* ctx, const double* C, int b, double* Cw, double* W, double* lam,
                                double* work, int* info) {
  hipStream_t st = ctx->stream;
  if (b <= kHeevRoute && ctx->eig_method == 0) {
    TRY(heev_values(ctx, C, b, lam, info));
    return heev_vectors(ctx, b, b, 0, 0, W);
  }
  const long bb = (long)b * b;
  // the row-major buffer read column-major is C^T = conj(C): eigenvectors
  // come out conjugated, eigenvalues are the same
  TRY_HIP(launch_interleave(C, bb, Cw, st));
  TRY(rocws_reserve(ctx, rocsolver_ws_bound(b)));
  rocblas_status rs = rocsolver_zheevd(ctx->blas, rocblas_evect_original, rocblas_fill_upper, b,
                                       (rocblas_double_complex*)Cw, b, lam, work, info);
  if (rs != rocblas_status_success)
    return fail(ctx, TDMRG_EDEVICE, "rocsolver_zheevd failed with status " + std::to_string((int)rs));
  TRY_HIP(launch_eigvec_extract(Cw, b, b, 1, 0, W, st));
  return TDMRG_OK;
}

// Rinv (planar b x b, row stride b, zero below the diagonal blocks) receives
// R^(-1) for the n x n diagonal block of G at offset o, where that block is
// R^H R (upper triangle of G read; G is overwritten by Schur complements).
// Recursive halving: R11 and its inverse from the leading block, R12 =
// R11^(-H) A12, the Schur complement A22 - R12^H R12 factored in turn, and
// (R^(-1))12 = -R11^(-1) R12 R22^(-1); leaves of at most kCholLeaf rows are
// factored and inverted in LDS.  S1, S2 are b x b scratch blocks.
static tdmrg_status chol_inv_rec(tdmrg_ctx* ctx, double* G, double* Rinv, double* S1, double* S2, int b, int o,
                                 int n, int* status) {
  hipStream_t st = ctx->stream;
  const long bb = (long)b * b;
  auto at = [&](double* M, int r, int c) { return M + (long)r * b + c; };
  if (n <= kCholLeaf) {
    TRY_HIP(launch_chol_leaf(at(G, o, o), bb, b, n, at(Rinv, o, o), bb, b, status, st));
    return TDMRG_OK;
  }
  const int n1 = ((n / 2 + 15) / 16) * 16, n2 = n - n1;
  const int o2 = o + n1;
  TRY(chol_inv_rec(ctx, G, Rinv, S1, S2, b, o, n1, status));
  // R12 = R11^(-H) A12
  TRY_HIP(tuned_cgemm(ctx, gemm(n1, n2, n1, 1, 1, op(at(Rinv, o, o), bb, 0, 0, b, 1, 1), op(at(G, o, o2), bb, 0, 0, b, 0, 0),
                            at(S1, o, o2), bb, 0, b), Arith::F64, st));
  // A22 <- A22 - R12^H R12
  GemmArgs gs = gemm(n2, n2, n1, 1, 1, op(at(S1, o, o2), bb, 0, 0, b, 1, 1), op(at(S1, o, o2), bb, 0, 0, b, 0, 0),
                     at(G, o2, o2), bb, 0, b);
  gs.alpha_re = -1.0;
  gs.beta_re = 1.0;
  TRY_HIP(tuned_cgemm(ctx, gs, Arith::F64, st));
  TRY(chol_inv_rec(ctx, G, Rinv, S1, S2, b, o2, n2, status));
  // (R^(-1))12 = -R11^(-1) (R12 R22^(-1))
  TRY_HIP(tuned_cgemm(ctx, gemm(n1, n2, n2, 1, 1, op(at(S1, o, o2), bb, 0, 0, b, 0, 0),
                            op(at(Rinv, o2, o2), bb, 0, 0, b, 0, 0), at(S2, o, o2), bb, 0, b), Arith::F64, st));
  GemmArgs gi = gemm(n1, n2, n1, 1, 1, op(at(Rinv, o, o), bb, 0, 0, b, 0, 0), op(at(S2, o, o2), bb, 0, 0, b, 0, 0),
                     at(Rinv, o, o2), bb, 0, b);
  gi.alpha_re = -1.0;
  TRY_HIP(tuned_cgemm(ctx, gi, Arith::F64, st));
  return TDMRG_OK;
}

// Q = X D R^(-1) with D = diag(X^H X)^(-1/2) and D X^H X D = R^H R: one
// column-scaled Cholesky QR pass over the p x b planar row-major block X
// (ld b; Q may not alias X).  right = true: X is b x p (ld p) and the rows
// are made orthonormal, Q = R^(-H) D X with D X X^H D = R^H R.  *status
// (device) becomes nonzero when the Gram matrix is not numerically positive
// definite.
static tdmrg_status cholqr_once(tdmrg_ctx* ctx, const double* X, long p, int b, double* Q, int* status,
                                bool right = false) {
  hipStream_t st = ctx->stream;
  const long bb = (long)b * b, pb = p * b;
  TRY(ensure(ctx, ctx->cqr, sizeof(double) * (8 * (size_t)bb + (size_t)b + 64)));
  double* G = (double*)ctx->cqr.p;
  double* T = G + 2 * bb;
  double* S1 = T + 2 * bb;
  double* S2 = S1 + 2 * bb;
  double* dcol = S2 + 2 * bb;
  auto mat = [&](const double* M, long plane, int trans, int conj) { return op(M, plane, 0, 0, b, trans, conj); };
  auto wide = [&](const double* M, int trans, int conj) { return op(M, pb, 0, 0, p, trans, conj); };
  if (right)
    TRY_HIP(tuned_cgemm(ctx, gemm(b, b, (int)p, 1, 1, wide(X, 0, 0), wide(X, 1, 1), G, bb, 0, b), Arith::F64, st));
  else
    TRY_HIP(tuned_cgemm(ctx, gemm(b, b, (int)p, 1, 1, mat(X, pb, 1, 1), mat(X, pb, 0, 0), G, bb, 0, b), Arith::F64,
                        st));
  TRY_HIP(launch_gram_colscale(G, b, dcol, status, st));
  TRY_HIP(launch_fill(T, 2 * bb, 0.0, st));
  TRY(chol_inv_rec(ctx, G, T, S1, S2, b, 0, b, status));
  TRY_HIP(launch_rowscale(T, b, dcol, st));
  if (right)
    TRY_HIP(tuned_cgemm(ctx, gemm(b, (int)p, b, 1, 1, mat(T, bb, 1, 1), wide(X, 0, 0), Q, pb, 0, (int)p), Arith::F64,
                        st));
  else
    TRY_HIP(tuned_cgemm(ctx, gemm((int)p, b, b, 1, 1, mat(X, pb, 0, 0), mat(T, bb, 0, 0), Q, pb, 0, b), Arith::F64,
                        st));
  return TDMRG_OK;
}

// Householder split with rocSOLVER, for any rank: the row-major M read
// column-major is M^T (cols x rows).  left: LQ of M^T = L Q' gives M = Q'^T
// L^T, so Q = Q'^T (rows x k, orthonormal columns) and C = L^T (k x cols,
// upper trapezoidal); right: QR of M^T = Q'' R gives M = R^T Q''^T, so
// Q = Q''^T (k x cols, orthonormal rows) and C = R^T (rows x k).  k =
// min(rows, cols).  Read back from the factored buffer, Q'^T and Q''^T are
// the buffer itself in row-major order, L^T and R^T its triangles.
tdmrg_status qr_householder(tdmrg_ctx* ctx, int rows, int cols, const double* M, bool right, double* Q, double* C) {
  hipStream_t st = ctx->stream;
  const int k = std::min(rows, cols);
  const long n = (long)rows * cols;
  TRY(ensure(ctx, ctx->hqr, sizeof(double) * (2 * (size_t)n + 2 * (size_t)k + 8)));
  double* A = (double*)ctx->hqr.p;
  rocblas_double_complex* A_ = (rocblas_double_complex*)A;
  rocblas_double_complex* tau = (rocblas_double_complex*)(A + 2 * n);
  TRY_HIP(launch_interleave(M, n, A, st));
  TRY(rocws_reserve(ctx, rocsolver_qr_ws_bound(std::max(rows, cols))));
  rocblas_status rs;
  if (!right) {
    rs = rocsolver_zgelqf(ctx->blas, cols, rows, A_, cols, tau);
    if (rs == rocblas_status_success) TRY_HIP(launch_extract_ld(A, cols, k, cols, 1, C, st));
    if (rs == rocblas_status_success) rs = rocsolver_zunglq(ctx->blas, k, rows, k, A_, cols, tau);
    if (rs == rocblas_status_success) TRY_HIP(launch_extract_ld(A, cols, rows, k, 0, Q, st));
  } else {
    rs = rocsolver_zgeqrf(ctx->blas, cols, rows, A_, cols, tau);
    if (rs == rocblas_status_success) TRY_HIP(launch_extract_ld(A, cols, rows, k, 2, C, st));
    if (rs == rocblas_status_success) rs = rocsolver_zungqr(ctx->blas, cols, k, k, A_, cols, tau);
    if (rs == rocblas_status_success) TRY_HIP(launch_extract_ld(A, cols, k, cols, 0, Q, st));
  }
  if (rs != rocblas_status_success)
    return fail(ctx, TDMRG_EDEVICE, "rocSOLVER Householder factorisation failed with status " + std::to_string((int)rs));
  return TDMRG_OK;
}

// Orthonormal split of a site tensor for the one-site scheme (the
// left-orthonormalisation M = L Q of Section 2.1.2 and its mirror image):
// two column-scaled Cholesky QR passes, then the bond matrix as the exact
// projection C = Q^H M (or M Q^H), so that Q C reproduces M to rounding.
// Where a pass breaks down (M numerically rank deficient) the split comes
// from Householder QR (qr_householder), which holds for any rank.
tdmrg_status qr_split(tdmrg_ctx* ctx, int rows, int cols, const double* M, bool right, double* Q, double* C,
                      bool* cholesky_ok) {
  hipStream_t st = ctx->stream;
  const int b = right ? rows : cols;
  const long p = right ? cols : rows;
  if (b < 1 || p < b) return fail(ctx, TDMRG_ESHAPE, "qr_split: the bond exceeds the block it is split from");
  if (b > kMaxSubspace) {  // beyond the one-workgroup Cholesky leaves: Householder for any size
    *cholesky_ok = false;
    return qr_householder(ctx, rows, cols, M, right, Q, C);
  }
  const long pb = p * b, bb = (long)b * b;
  TRY(ensure(ctx, ctx->qr, sizeof(double) * (2 * (size_t)pb + 1)));
  double* Q1 = (double*)ctx->qr.p;
  int* status = (int*)(Q1 + 2 * pb);
  TRY_HIP(launch_fill((double*)status, 1, 0.0, st));
  TRY(cholqr_once(ctx, M, p, b, Q1, status, right));
  TRY(cholqr_once(ctx, Q1, p, b, Q, status + 1, right));
  if (right)
    TRY_HIP(tuned_cgemm(ctx, gemm(b, b, (int)p, 1, 1, op(M, pb, 0, 0, p, 0, 0), op(Q, pb, 0, 0, p, 1, 1), C, bb, 0, b),
                        Arith::F64, st));
  else
    TRY_HIP(tuned_cgemm(ctx, gemm(b, b, (int)p, 1, 1, op(Q, pb, 0, 0, b, 1, 1), op(M, pb, 0, 0, b, 0, 0), C, bb, 0, b),
                        Arith::F64, st));
  TRY_HIP(hipMemcpyAsync(ctx->host, status, 2 * sizeof(int), hipMemcpyDeviceToHost, st));
  TRY_HIP(hipStreamSynchronize(st));
  int hs[2];
  std::memcpy(hs, ctx->host, sizeof(hs));
  *cholesky_ok = !hs[0] && !hs[1];
  if (!*cholesky_ok) TRY(qr_householder(ctx, rows, cols, M, right, Q, C));
  return TDMRG_OK;
}

// Block size of the subspace iteration for a rank cap D_max.
static int subspace_block(int D_max) {
  const int over = std::max(32, D_max / 2);
  return ((D_max + over + 15) / 16) * 16;
}

// Truncated SVD by subspace iteration with Rayleigh-Ritz (only the leading
// singular triplets are ever needed: at most D_max are kept).
//   A = theta (orthonormal factor on the left) or theta^H (on the right), p x q.
//   Q (p x b) starts as an orthonormalised random block; each iteration
//   forms Z = A^H Q, the Rayleigh quotient C = Z^H Z = Q^H A A^H Q and its
//   eigenpairs (W, lambda), Y = A Z = A A^H Q and the Ritz residuals
//   r_j = |(Y - Q C) w_j| = |A A^H u_j - lambda_j u_j| of u_j = Q w_j.  When
//   the kept pairs have converged, U = Q W (orthonormal) and the other factor
//   is Z W = A^H U, the exact projection, so no singular value is divided by.
//   Otherwise Q = orth(Y W) by column-scaled Cholesky QR; columns
//   whose Ritz value is below the rounding level of Y are replaced by random
//   ones first, so that a numerically rank-deficient theta keeps a full-rank
//   block.  The
//   Rayleigh-Ritz step (an eigensolver call) runs only at checks: the first
//   iteration and then the iteration at which the Ritz values predict
//   convergence; plain iterations orthonormalise Y itself.
// The DBSS rank uses the leading b values and |theta|_F^2 for the tail.
// *done stays false when the iteration does not settle (the caller then
// takes the full eigensolver route).
static tdmrg_status svd_subspace(tdmrg_ctx* ctx, int rows, int cols, const double* theta, double eps, int D_max,
                                 int sv_mode, double tie_rel, int k_cap, int mode, double* out1, double* out2,
                                 double* S_out, int* k_out, double* disc_out, bool* done) {
  *done = false;
  hipStream_t st = ctx->stream;
  const bool left = (mode != 2);
  const int p = left ? rows : cols;
  const int q = left ? cols : rows;
  const int b = std::min(std::min(subspace_block(D_max), kMaxSubspace), std::min(rows, cols));
  const long th = (long)rows * cols;
  const long pb = (long)p * b, qb = (long)q * b, bb = (long)b * b;
  const size_t nd = 2 * (4 * (size_t)pb + qb) + 14 * (size_t)bb + 5 * (size_t)b +
                    (size_t)colnorm_part_doubles(b) + 64;
  TRY(ensure(ctx, ctx->sub, nd * sizeof(double)));
  double* w = (double*)ctx->sub.p;
  double* Q = w; w += 2 * pb;
  double* Q2 = w; w += 2 * pb;
  double* Y = w; w += 2 * pb;
  double* E = w; w += 2 * pb;
  double* Zb = w; w += 2 * qb;
  double* C = w; w += 2 * bb;
  double* Cw = w; w += 2 * bb;
  double* W = w; w += 2 * bb;
  double* G = w; w += 2 * bb;
  double* T = w; w += 2 * bb;
  double* S1 = w; w += 2 * bb;
  double* S2 = w; w += 2 * bb;
  double* lam = w; w += b;   // read-back block: lam | Sv | res | disc | ints
  double* Sv = w; w += b;
  double* res = w; w += b;
  double* disc_d = w; w += 1;
  int* ints = (int*)w; w += 8;  // [0..1] Cholesky status per pass, [3] rank, [4] zheevd info
  double* work = w; w += b;
  double* dcol = w; w += b;
  double* part = w;
  Small sm;
  TRY(small_ws(ctx, &sm));

  // operands: A X (p x b) and A^H X (q x b) for planar row-major X with ld b
  auto opA = [&]() { return left ? op(theta, th, 0, 0, cols, 0, 0) : op(theta, th, 0, 0, cols, 1, 1); };
  auto opAH = [&]() { return left ? op(theta, th, 0, 0, cols, 1, 1) : op(theta, th, 0, 0, cols, 0, 0); };
  auto mat = [&](const double* X, long plane, int trans, int conj) { return op(X, plane, 0, 0, b, trans, conj); };
  // Q = orth(X) by column-scaled Cholesky QR (two passes through Q2): with
  // D = diag(G)^(-1/2) and D G D = R^H R (blocked Cholesky with inverse),
  // X D R^(-1) has orthonormal columns.  Like Gram-Schmidt it keeps column j
  // in the span of columns 0..j, so a block in Ritz order stays well
  // conditioned under the power steps.
  // One pass leaves Q orthonormal to about eps * cond(X D)^2, enough for a
  // plain power step; the basis that a Rayleigh-Ritz check (and the output
  // U = Q W) uses gets the second pass.
  // A shifted first pass (shift 11 (p b + b (b + 1)) u |X D|_2^2 on the
  // scaled Gram matrix, after Fukaya et al., shifted Cholesky QR, SIAM J.
  // Sci. Comput. 2020) makes the factorisation succeed for any condition
  // number up to 1/u; its output then has a condition number of about
  // u^(-1/2) and two plain passes finish it.
  auto orth = [&](const double* X, int passes, bool shifted = false) -> tdmrg_status {
    const double u = std::ldexp(1.0, -53);
    const double shift = 11.0 * ((double)p * b + (double)b * (b + 1)) * u * b;  // |X D|_2^2 <= |X D|_F^2 = b
    const double* src = X;
    for (int k = 0; k < passes; ++k) {
      double* dst = ((passes - 1 - k) % 2 == 0) ? Q : Q2;  // the last pass lands in Q
      TRY_HIP(tuned_cgemm(ctx, gemm(b, b, p, 1, 1, mat(src, pb, 1, 1), mat(src, pb, 0, 0), G, bb, 0, b), Arith::F64, st));
      TRY_HIP(launch_gram_colscale(G, b, dcol, ints + std::min(k, 1), st, shifted && k == 0 ? shift : 0.0));
      TRY_HIP(launch_fill(T, 2 * bb, 0.0, st));
      TRY(chol_inv_rec(ctx, G, T, S1, S2, b, 0, b, ints + std::min(k, 1)));
      TRY_HIP(launch_rowscale(T, b, dcol, st));
      TRY_HIP(tuned_cgemm(ctx, gemm(p, b, b, 1, 1, mat(src, pb, 0, 0), mat(T, bb, 0, 0), dst, pb, 0, b), Arith::F64, st));
      src = dst;
    }
    return TDMRG_OK;
  };

  // |theta|_F
  TRY(dots(ctx, sm, theta, 2 * th, 1, th, theta, sm.beta0, nullptr, 1));
  TRY_HIP(launch_fill((double*)ints, 4, 0.0, st));
  const unsigned long long seed = 0x243F6A8885A308D3ull;
  TRY_HIP(launch_randfill(E, 2 * pb, seed, st));
  TRY(orth(E, 2));

  // Rayleigh-Ritz checks run where the Ritz values predict convergence; in
  // between, Q keeps the column order of the last check (Cholesky QR
  // preserves it), so Y's columns stay nearly orthogonal.  Before the first
  // check the block is not in Ritz order: the first power step from the
  // random block leaves every column leaning towards the leading singular
  // vector, so that step is orthonormalised by the shifted pass plus two
  // plain ones, and the steps up to the first check by two passes.  The
  // first check comes at the iteration at which the previous subspace SVD
  // of this context converged (schedule 0), or at iteration 1 (schedule 1).
  const int max_it = 40;
  double prev = INFINITY;
  int next_check = ctx->svd_schedule == 1 ? 1 : std::min(std::max(ctx->svd_first_check, 2), 8), j0 = b;
  bool ordered = false;
  for (int it = 1; it <= max_it; ++it) {
    const bool check = (it == next_check) || it == max_it;
    TRY_HIP(tuned_cgemm(ctx, gemm(q, b, p, 1, 1, opAH(), mat(Q, pb, 0, 0), Zb, qb, 0, b), Arith::F64, st));
    if (check) {
      TRY_HIP(tuned_cgemm(ctx, gemm(b, b, q, 1, 1, mat(Zb, qb, 1, 1), mat(Zb, qb, 0, 0), C, bb, 0, b), Arith::F64, st));
      TRY(heevd_small(ctx, C, b, Cw, W, lam, work, ints + 4));
      TRY_HIP(launch_eig_to_sv(lam, b, Sv, st));
      TRY_HIP(launch_choose_rank_partial(Sv, b, sm.beta0, eps, D_max, sv_mode, tie_rel, ints + 3, disc_d, st));
    }
    // Y = A Z = A A^H Q
    TRY_HIP(tuned_cgemm(ctx, gemm(p, b, q, 1, 1, opA(), mat(Zb, qb, 0, 0), Y, pb, 0, b), Arith::F64, st));
    double* X = Y;
    if (check) {
      // E = Y - Q C;  residual columns (E W)_j
      TRY_HIP(hipMemcpyAsync(E, Y, sizeof(double) * 2 * pb, hipMemcpyDeviceToDevice, st));
      GemmArgs ge = gemm(p, b, b, 1, 1, mat(Q, pb, 0, 0), mat(C, bb, 0, 0), E, pb, 0, b);
      ge.alpha_re = -1.0;
      ge.beta_re = 1.0;
      TRY_HIP(tuned_cgemm(ctx, ge, Arith::F64, st));
      TRY_HIP(tuned_cgemm(ctx, gemm(p, b, b, 1, 1, mat(E, pb, 0, 0), mat(W, bb, 0, 0), Q2, pb, 0, b), Arith::F64, st));
      TRY_HIP(launch_colnorms(Q2, pb, p, b, b, part, res, st));
      TRY_HIP(hipMemcpyAsync(ctx->host, lam, sizeof(double) * (3 * (size_t)b + 1 + 8), hipMemcpyDeviceToHost, st));
      TRY_HIP(hipStreamSynchronize(st));
      if (ctx->prof.on) TRY(prof_flush(ctx));
      const double* hl = ctx->host;
      const double* hr = ctx->host + 2 * b;
      int hi[8];
      std::memcpy(hi, ctx->host + 3 * b + 1, sizeof(hi));
      const double hdisc = ctx->host[3 * b];
      if (hi[0] || hi[1] || hi[4]) {  // a Cholesky pass or the eigensolver failed
        ctx->svd_count[5]++;
        return TDMRG_OK;
      }
      const int k = hi[3];
      const double lam0 = std::max(hl[b - 1], 0.0);
      const double lamb = std::max(hl[0], 0.0);  // smallest Ritz value: the rate of the block
      double worst = 0.0, maxres = 0.0;
      int more = 1;
      for (int j = 0; j < k; ++j) {
        const double lj = std::max(hl[b - 1 - j], 0.0);
        const double tol = std::max(1e-15 * lam0, 1e-12 * std::sqrt(lj * lam0));
        worst = std::max(worst, hr[j] / tol);
        maxres = std::max(maxres, hr[j]);
        if (hr[j] > tol) {  // residual of pair j shrinks by about lamb / lj per iteration
          const double rho = lj > 0.0 ? lamb / lj : 1.0;
          const int n = rho < 0.9 ? (int)std::ceil(std::log(hr[j] / tol) / -std::log(rho)) : 4;
          more = std::max(more, n);
        }
      }
      if (!(worst == worst)) return TDMRG_OK;  // NaN: leave it to the eigensolver route
      const bool stalled = it >= 3 && maxres > 0.5 * prev && maxres <= 1e-11 * lam0;
      prev = maxres;
      if (worst <= 1.0 || stalled || lam0 == 0.0) {
        if (k > k_cap)
          return fail(ctx, TDMRG_ESHAPE, "kept rank " + std::to_string(k) + " exceeds capacity " + std::to_string(k_cap));
        if (left) {
          // out1 = U = Q W_k [rows][k];  out2 = (Z W_k)^H = U^H theta = S Vh [k][cols]
          TRY_HIP(tuned_cgemm(ctx, gemm(rows, k, b, 1, 1, mat(Q, pb, 0, 0), mat(W, bb, 0, 0), out1, (long)rows * k, 0, k),
                               Arith::F64, st));
          TRY_HIP(tuned_cgemm(ctx, gemm(k, cols, b, 1, 1, mat(W, bb, 1, 1), mat(Zb, qb, 1, 1), out2, (long)k * cols, 0, cols),
                               Arith::F64, st));
          if (mode == 0) TRY_HIP(launch_scale_sv(out2, k, cols, Sv, 1, 1, st));
        } else {
          // out2 = Vh = (Q W_k)^H [k][cols];  out1 = Z W_k = theta V = U S [rows][k]
          TRY_HIP(tuned_cgemm(ctx, gemm(k, cols, b, 1, 1, mat(W, bb, 1, 1), mat(Q, pb, 1, 1), out2, (long)k * cols, 0, cols),
                               Arith::F64, st));
          TRY_HIP(tuned_cgemm(ctx, gemm(rows, k, b, 1, 1, mat(Zb, qb, 0, 0), mat(W, bb, 0, 0), out1, (long)rows * k, 0, k),
                               Arith::F64, st));
        }
        if (S_out) TRY_HIP(hipMemcpyAsync(S_out, Sv, sizeof(double) * k, hipMemcpyDeviceToDevice, st));
        *k_out = k;
        *disc_out = hdisc;
        *done = true;
        ctx->svd_first_check = it;
        ctx->svd_count[2]++;
        ctx->svd_count[3] += it;
        ctx->svd_count[6]++;
        return TDMRG_OK;
      }
      ctx->svd_count[6]++;
      next_check = it + std::min(std::max(more, 1), 6);
      j0 = 0;
      while (j0 < b && hl[b - 1 - j0] > 1e-13 * lam0) ++j0;
      // next basis from Y W (Ritz order)
      TRY_HIP(tuned_cgemm(ctx, gemm(p, b, b, 1, 1, mat(Y, pb, 0, 0), mat(W, bb, 0, 0), E, pb, 0, b), Arith::F64, st));
      X = E;
      ordered = true;
    }
    // columns below the rounding level of Y are renewed, then Q = orth(X)
    TRY_HIP(launch_randfill_cols(X, p, b, std::max(j0, 1), seed + 0x9E3779B97F4A7C15ull * it, st));
    if (!ordered) {
      TRY(orth(X, it == 1 ? 3 : 2, it == 1));
      if (it == 1 && next_check > 1) {
        // a first power step beyond the reach of the shifted pass (theta
        // numerically rank deficient within the block): start again from
        // the random block with the check at iteration 1
        TRY_HIP(hipMemcpyAsync(ctx->host, ints, 2 * sizeof(int), hipMemcpyDeviceToHost, st));
        TRY_HIP(hipStreamSynchronize(st));
        int hs[2];
        std::memcpy(hs, ctx->host, sizeof(hs));
        if (hs[0] || hs[1]) {
          TRY_HIP(launch_fill((double*)ints, 1, 0.0, st));
          TRY(orth(E, 2));
          next_check = 1;
          it = 0;
        }
      }
    } else {
      TRY(orth(X, (it + 1 == next_check || it + 1 == max_it) ? 2 : 1));
    }
  }
  ctx->svd_count[4]++;
  return TDMRG_OK;
}

// SVD truncation through the Hermitian eigenproblem of a Gram matrix.
//   G = theta theta^H (left factor wanted) or theta^H theta (right factor),
//   built by the FP64 MFMA GEMM; rocSOLVER zheevd gives its eigenpairs
//   (eigenvalues s_j^2, eigenvectors the singular vectors on that side);
//   the DBSS rank is chosen on the device from s_j = sqrt(max(lambda, 0));
//   the orthonormal factor is read from the eigenvectors and the other one
//   is the exact projection of theta onto it (one more GEMM), so that
//   U_k S_k V_k^H = U_k U_k^H theta without dividing by singular values.
// mode 0: out1 = U [rows][k], out2 = Vh [k][cols] (rows of Vh with s_j = 0 are
//         zero), S_out = s;  mode 1: out1 = U, out2 = S Vh;  mode 2: out1 =
//         U S, out2 = Vh.
tdmrg_status svd_truncate(tdmrg_ctx* ctx, int rows, int cols, const double* theta, double eps,
                          int D_max, int sv_mode, double tie_rel, int k_cap, int mode, double* out1,
                          double* out2, double* S_out, int* k_out, double* disc_out) {
  const bool left = (mode != 2);  // which factor comes out orthonormal from the eigenvectors
  const int n = left ? rows : cols;
  const long nn = (long)n * n;
  Small sm;
  TRY(small_ws(ctx, &sm));
  const int len = left ? cols : rows;
  // The Jacobi route rotates the side with fewer vectors when the kept
  // singular values are bounded away from zero (eps > 0, not keep-all); the
  // factor this mode needs then comes from a division (see below).
  const bool jleft = (sv_mode != 2 && eps > 0.0) ? rows <= cols : left;
  const int nj = jleft ? rows : cols;
  // Rotation work per sweep ~ nj^2 (nj + len).  Small problems take the
  // one-workgroup Jacobi SVD; larger ones only when tiny singular values are
  // kept (keep-all mode or eps < 1e-10), where the Gram route would lose them.
  // The one-workgroup kernel takes about 8 ns per unit of nj^2 (rows + cols)
  // (64 x 300: 11.6 ms, 128 x 600: 118 ms) against a floor of about 2 ms for
  // the Gram route at these sizes (measured), hence the small limit.
  const double jwork = (double)nj * nj * (rows + cols);
  const bool need_tiny = (sv_mode == 2) || (sv_mode == 0 && eps < 1e-10);
  int method = ctx->svd_method;
  if (method == 0) {
    const int b = subspace_block(D_max);
    if (nj <= kJacobiMaxVectors && (jwork <= 2.5e5 || (need_tiny && jwork <= 1.5e8))) method = 1;
    else if (!need_tiny && b <= kMaxSubspace && 2 * b <= std::min(rows, cols)) method = 3;
    else method = 2;
  }
  if (method == 1 && nj > kJacobiMaxVectors)
    return fail(ctx, TDMRG_EUNSUPPORTED, "Jacobi SVD takes at most " + std::to_string(kJacobiMaxVectors) + " vectors");
  if (method == 3) {
    if (sv_mode == 2) return fail(ctx, TDMRG_EUNSUPPORTED, "subspace SVD cannot keep every singular value");
    bool done = false;
    TRY(svd_subspace(ctx, rows, cols, theta, eps, D_max, sv_mode, tie_rel, k_cap, mode, out1, out2, S_out, k_out,
                     disc_out, &done));
    if (done) return TDMRG_OK;
    method = 2;  // did not settle: full eigensolver
  }
  if (method == 1) {
    ctx->svd_count[0]++;
    // Small problem: one-sided Jacobi on theta itself keeps the accuracy of a
    // direct SVD for every kept singular value, however small.
    TRY(ensure(ctx, ctx->svd_u, sizeof(double) * 2 * (size_t)rows * cols));
    TRY(ensure(ctx, ctx->svd_z, sizeof(double) * 2 * (size_t)nj * nj));
    TRY(ensure(ctx, ctx->svd_s, sizeof(double) * 2 * (size_t)std::max(rows, cols) + 64));
    TRY(ensure(ctx, ctx->svd_e, sizeof(int) * (size_t)std::max(rows, cols) + 64));
    double* Wk = (double*)ctx->svd_u.p;
    double* Vacc = (double*)ctx->svd_z.p;
    double* sig = (double*)ctx->svd_s.p;
    int* perm = (int*)ctx->svd_e.p;
    hipStream_t st = ctx->stream;
    const int nsv = std::min(rows, cols);
    const long th = (long)rows * cols;
    // the smaller side first; should the division's Cholesky QR break down
    // (a kept singular value at rounding level), the needed side again
    for (int attempt = 0; attempt < 2; ++attempt) {
      const bool jl = attempt == 0 ? jleft : left;
      if (attempt == 1) {
        if (jleft == left) break;
        TRY(ensure(ctx, ctx->svd_z, sizeof(double) * 2 * (size_t)n * n));
        Vacc = (double*)ctx->svd_z.p;
      }
      TRY_HIP(launch_jacobi_svd(theta, rows, cols, jl ? 1 : 0, Wk, Vacc, sig, perm, 60, st));
      TRY_HIP(launch_choose_rank(sig, nsv, eps, D_max, sv_mode, tie_rel, sm.ik, sm.disc, st));
      TRY_HIP(hipMemcpyAsync(ctx->host, sm.ik, sizeof(int), hipMemcpyDeviceToHost, st));
      TRY_HIP(hipMemcpyAsync(ctx->host + 1, sm.disc, sizeof(double), hipMemcpyDeviceToHost, st));
      TRY_HIP(hipStreamSynchronize(st));
      int k = 0;
      std::memcpy(&k, ctx->host, sizeof(int));
      const double disc = ctx->host[1];
      if (k > k_cap)
        return fail(ctx, TDMRG_ESHAPE, "kept rank " + std::to_string(k) + " exceeds capacity " + std::to_string(k_cap));
      if (jl == left) {
        TRY_HIP(launch_jacobi_assemble(Wk, Vacc, sig, perm, rows, cols, left ? 1 : 0, k, mode, out1, out2, st));
      } else {
        // Rotations ran on the other side: the orthonormal factor this mode
        // needs is the rotated block divided by the singular values (exact
        // up to about eps s_0 / s_j in direction, weighted by s_j in theta),
        // made orthonormal again by one Cholesky QR pass; the other factor is
        // the projection of theta onto it, as in the other routes.
        int* qr_fail = sm.ik + 2;
        TRY_HIP(launch_fill((double*)(sm.ik + 2), 1, 0.0, st));
        if (left) {  // Jacobi on the columns: U = W S^-1, then U <- orth(U)
          TRY(ensure(ctx, ctx->svd_vt, sizeof(double) * 2 * (size_t)rows * k));
          double* Ud = (double*)ctx->svd_vt.p;
          TRY_HIP(launch_jacobi_assemble(Wk, Vacc, sig, perm, rows, cols, 0, k, mode, Ud, out2, st));
          TRY(cholqr_once(ctx, Ud, rows, k, out1, qr_fail));
          if (mode == 1)  // S Vh = U^H theta (mode 0 keeps Vh from the rotations)
            TRY_HIP(tuned_cgemm(ctx, gemm(k, cols, rows, 1, 1, op(out1, (long)rows * k, 0, 0, k, 1, 1),
                                          op(theta, th, 0, 0, cols, 0, 0), out2, (long)k * cols, 0, cols),
                                 Arith::F64, st));
        } else {  // Jacobi on the rows: Vh = W^H S^-1, rows orthonormalised; U S = theta Vh^H
          TRY(ensure(ctx, ctx->svd_vt, sizeof(double) * 4 * (size_t)cols * k));
          double* Vd = (double*)ctx->svd_vt.p;     // Vh^H, cols x k
          double* Vq = Vd + 2 * (size_t)cols * k;  // orthonormalised
          TRY_HIP(launch_jacobi_assemble(Wk, Vacc, sig, perm, rows, cols, 1, k, 0, out1, out2, st));
          TRY_HIP(launch_conj_transpose_rect(out2, k, cols, Vd, st));
          TRY(cholqr_once(ctx, Vd, cols, k, Vq, qr_fail));
          TRY_HIP(launch_conj_transpose_rect(Vq, cols, k, out2, st));
          TRY_HIP(tuned_cgemm(ctx, gemm(rows, k, cols, 1, 1, op(theta, th, 0, 0, cols, 0, 0),
                                        op(Vq, (long)cols * k, 0, 0, k, 0, 0), out1, (long)rows * k, 0, k),
                               Arith::F64, st));
        }
        TRY_HIP(hipMemcpyAsync(ctx->host, qr_fail, sizeof(int), hipMemcpyDeviceToHost, st));
        TRY_HIP(hipStreamSynchronize(st));
        int f = 0;
        std::memcpy(&f, ctx->host, sizeof(int));
        if (f) continue;
      }
      if (S_out) TRY_HIP(hipMemcpyAsync(S_out, sig, sizeof(double) * k, hipMemcpyDeviceToDevice, st));
      *k_out = k;
      *disc_out = disc;
      return TDMRG_OK;
    }
    return fail(ctx, TDMRG_EDEVICE, "Jacobi SVD: no usable side");
  }
  ctx->svd_count[1]++;
  TRY(ensure(ctx, ctx->svd_u, sizeof(double) * 2 * (size_t)nn));  // Gram, planar
  TRY(ensure(ctx, ctx->svd_z, sizeof(double) * 2 * (size_t)nn));  // Gram, interleaved
  TRY(ensure(ctx, ctx->svd_s, sizeof(double) * 2 * (size_t)n + 64));
  TRY(ensure(ctx, ctx->svd_e, sizeof(double) * (size_t)n + 64));
  hipStream_t st = ctx->stream;
  double* G = (double*)ctx->svd_u.p;
  double* Z = (double*)ctx->svd_z.p;
  double* lam = (double*)ctx->svd_s.p;
  double* Sv = lam + n;
  double* E = (double*)ctx->svd_e.p;
  int* info = sm.ik + 1;
  // Gram matrix, row-major planar
  GemmArgs gg;
  if (left)  // G[i][j] = sum_c theta[i][c] conj(theta[j][c])
    gg = gemm(n, n, cols, 1, 1, op(theta, (long)rows * cols, 0, 0, cols, 0, 0),
              op(theta, (long)rows * cols, 0, 0, cols, 1, 1), G, nn, 0, n);
  else  // G[i][j] = sum_r conj(theta[r][i]) theta[r][j]
    gg = gemm(n, n, rows, 1, 1, op(theta, (long)rows * cols, 0, 0, cols, 1, 1),
              op(theta, (long)rows * cols, 0, 0, cols, 0, 0), G, nn, 0, n);
  TRY_HIP(tuned_cgemm(ctx, gg, Arith::F64, st));
  const bool hand = n <= kHeevRoute && ctx->eig_method == 0;
  if (hand) {
    TRY(heev_values(ctx, G, n, lam, info));
  } else {
    // read column-major, the row-major buffer is G^T = conj(G): eigenvectors z
    // of conj(G) are conj() of those of G, eigenvalues are the same
    TRY_HIP(launch_interleave(G, nn, Z, st));
    TRY(rocws_reserve(ctx, rocsolver_ws_bound(n)));
    rocblas_status rs = rocsolver_zheevd(ctx->blas, rocblas_evect_original, rocblas_fill_upper, n,
                                         (rocblas_double_complex*)Z, n, lam, E, info);
    if (rs != rocblas_status_success)
      return fail(ctx, TDMRG_EDEVICE, "rocsolver_zheevd failed with status " + std::to_string((int)rs));
  }
  TRY_HIP(launch_eig_to_sv(lam, n, Sv, st));
  const int nsv = std::min(rows, cols);  // at most min(rows, cols) nonzero singular values
  TRY_HIP(launch_choose_rank(Sv, nsv, eps, D_max, sv_mode, tie_rel, sm.ik, sm.disc, st));
  TRY_HIP(hipMemcpyAsync(ctx->host, sm.ik, 2 * sizeof(int), hipMemcpyDeviceToHost, st));
  TRY_HIP(hipMemcpyAsync(ctx->host + 1, sm.disc, sizeof(double), hipMemcpyDeviceToHost, st));
  TRY_HIP(hipStreamSynchronize(st));
  int kk[2];
  std::memcpy(kk, ctx->host, sizeof(kk));
  const double disc = ctx->host[1];
  if (kk[1] != 0)
    return fail(ctx, TDMRG_EDEVICE, std::string(hand ? "dstedc" : "zheevd") + " did not converge (info " +
                                        std::to_string(kk[1]) + ")");
  const int k = kk[0];
  if (k > k_cap)
    return fail(ctx, TDMRG_ESHAPE, "kept rank " + std::to_string(k) + " exceeds capacity " + std::to_string(k_cap));
  const long th = (long)rows * cols;
  if (left) {
    // U[i][j] = conj(z_{n-1-j}[i])  (eigenvectors of G are conj(z); the
    // library's eigensolver gives those of G directly)
    if (hand) TRY(heev_vectors(ctx, n, k, 0, 0, out1));
    else TRY_HIP(launch_eigvec_extract(Z, n, k, 1, 0, out1, st));
    // out2[j][c] = sum_i conj(U[i][j]) theta[i][c] = s_j Vh[j][c]
    GemmArgs gm = gemm(k, cols, rows, 1, 1, op(out1, (long)rows * k, 0, 0, k, 1, 1),
                       op(theta, th, 0, 0, cols, 0, 0), out2, (long)k * cols, 0, cols);
    TRY_HIP(tuned_cgemm(ctx, gm, Arith::F64, st));
    if (mode == 0) TRY_HIP(launch_scale_sv(out2, k, cols, Sv, 1, 1, st));
  } else {
    // V[c][j] = conj(z_{n-1-j}[c]);  Vh[j][c] = conj(V[c][j]) = z_{n-1-j}[c]
    // (library eigensolver: V[c][j] = x_j[c], so Vh[j][c] = conj(x_j[c]))
    if (hand) TRY(heev_vectors(ctx, n, k, 1, 1, out2));
    else TRY_HIP(launch_eigvec_extract(Z, n, k, 0, 1, out2, st));
    // out1[r][j] = sum_c theta[r][c] conj(Vh[j][c]) = U[r][j] s_j
    GemmArgs gm = gemm(rows, k, cols, 1, 1, op(theta, th, 0, 0, cols, 0, 0),
                       op(out2, (long)k * cols, 0, 0, cols, 1, 1), out1, (long)rows * k, 0, k);
    TRY_HIP(tuned_cgemm(ctx, gm, Arith::F64, st));
  }
  if (S_out) TRY_HIP(hipMemcpyAsync(S_out, Sv, sizeof(double) * k, hipMemcpyDeviceToDevice, st));
  *k_out = k;
  *disc_out = disc;
  return TDMRG_OK;
}

}  // namespace tdmrg
