// Global time integrators on whole MPS (paper Section 2.1.1): the
// 4th-order Runge-Kutta update (eqs. runge kutta 1-4, runge kutta) and the
// global Krylov method (eqs. Krylov subspace, global Krylov).  H is applied
// to a compressed MPS as an exact MPO x MPS product (bonds multiplied by the
// MPO bonds), sums of MPS are block-diagonal bond concatenations, and every
// intermediate is compressed: left-to-right orthonormalisation (Cholesky QR
// where the bond fits its block, Householder QR where it does not or where
// the block is rank deficient), then right-to-left SVD truncation with the DBSS rank rule
// of the sweep, capped at D_max.  The global Krylov basis comes from the
// Lanczos three-term recurrence on compressed MPS; the new state is
// beta_0 sum_k c_k v_k with c = exp(-i dt/hbar T_m) e_1 from the device
// tridiagonal exponential, compressed once more.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <complex>
#include <cstring>
#include <vector>

#include "internal.h"

using namespace tdmrg;

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

namespace {

typedef std::complex<double> cplx;

// An MPS vector owned by the step: exact bonds, site buffers at capacity
// (bonds only shrink while it is compressed in place).  Kernels that read a
// vector may still be queued when it goes out of scope (a sum enqueues its
// block copies and returns), so the destructor waits for the context's
// stream before the buffers are freed.
struct Vec {
  tdmrg_mps* m = nullptr;
  Vec() = default;
  Vec(const Vec&) = delete;
  Vec& operator=(const Vec&) = delete;
  Vec(Vec&& o) noexcept : m(o.m) { o.m = nullptr; }
  Vec& operator=(Vec&& o) noexcept {
    std::swap(m, o.m);
    return *this;
  }
  ~Vec() {
    if (!m) return;
    (void)hipStreamSynchronize(m->ctx->stream);
    tdmrg_mps_destroy(m);
  }
};

tdmrg_status vec_alloc(tdmrg_ctx* ctx, const std::vector<int>& dims, const std::vector<int>& bonds, Vec* out) {
  tdmrg_mps* m = new tdmrg_mps();
  m->ctx = ctx;
  m->n = (int)dims.size();
  m->dims = dims;
  m->bond = bonds;
  m->cap = bonds;
  m->site.assign(m->n, nullptr);
  out->m = m;
  for (int s = 0; s < m->n; ++s) {
    const size_t bytes = sizeof(double) * 2 * std::max<size_t>(1, (size_t)bonds[s] * dims[s] * bonds[s + 1]);
    if (hipMalloc((void**)&m->site[s], bytes) != hipSuccess)
      return fail(ctx, TDMRG_ENOMEM, "allocation of an intermediate MPS failed");
  }
  return TDMRG_OK;
}

long site_len(const tdmrg_mps* m, int s) { return (long)m->bond[s] * m->dims[s] * m->bond[s + 1]; }

// Largest bond of an uncompressed intermediate (an MPO x MPS product or a
// sum) that this implementation accepts.  Products and sums up to this bond
// have been checked against the oracle on the device; a step at full size on
// a 4-mode model with boson bases 25/19/11/19 (intermediate bonds of about
// 1500) once ended in an illegal memory access whose cause is not known, so
// larger intermediates are refused (TDMRG_EUNSUPPORTED) rather than run.
constexpr int kMaxIntermediateBond = 192;

tdmrg_status check_intermediate(tdmrg_ctx* ctx, const std::vector<int>& bonds) {
  const int mx = *std::max_element(bonds.begin(), bonds.end());
  if (mx > kMaxIntermediateBond)
    return fail(ctx, TDMRG_EUNSUPPORTED,
                "global step: an intermediate MPS would have bond " + std::to_string(mx) + " > " +
                    std::to_string(kMaxIntermediateBond) + " (the largest validated intermediate bond)");
  return TDMRG_OK;
}

// out (M x N) = A (M x K) B (K x N), planar row-major, dense
GemmArgs gemm_plain(int M, int N, int K, const double* A, const double* B, double* out) {
  GemmArgs g{};
  g.M = M;
  g.N = N;
  g.K = K;
  g.nbatch = 1;
  g.nred = 1;
  g.role = 0;
  g.A = GemmOperand{A, (long)M * K, 0, 0, K, 0, 0};
  g.B = GemmOperand{B, (long)K * N, 0, 0, N, 0, 0};
  g.C = out;
  g.c_im = (long)M * N;
  g.c_sb = 0;
  g.ldc = N;
  g.alpha_re = 1.0;
  return g;
}

// y = H x (exact MPO x MPS product)
tdmrg_status apply_mpo(tdmrg_ctx* ctx, const tdmrg_mpo* mpo, const tdmrg_mps* x, Vec* y) {
  std::vector<int> bonds(x->n + 1);
  for (int b = 0; b <= x->n; ++b) bonds[b] = x->bond[b] * mpo->wdims[b];
  TRY(check_intermediate(ctx, bonds));
  TRY(vec_alloc(ctx, x->dims, bonds, y));
  for (int s = 0; s < x->n; ++s)
    TRY_HIP(launch_mpo_apply(mpo->dense[s], mpo->wdims[s], mpo->wdims[s + 1], x->dims[s], x->site[s], x->bond[s],
                             x->bond[s + 1], y->m->site[s], ctx->stream));
  return TDMRG_OK;
}

// y = sum_k c_k x_k (c_k scales the first site of x_k)
tdmrg_status lincomb(tdmrg_ctx* ctx, const std::vector<cplx>& c, const std::vector<const tdmrg_mps*>& xs, Vec* y) {
  const int n = xs[0]->n;
  std::vector<int> bonds(n + 1, 0);
  bonds[0] = bonds[n] = 1;
  for (int b = 1; b < n; ++b)
    for (const tdmrg_mps* x : xs) bonds[b] += x->bond[b];
  TRY(check_intermediate(ctx, bonds));
  TRY(vec_alloc(ctx, xs[0]->dims, bonds, y));
  hipStream_t st = ctx->stream;
  for (int s = 0; s < n; ++s) {
    const int d = xs[0]->dims[s];
    TRY_HIP(launch_fill(y->m->site[s], 2 * site_len(y->m, s), 0.0, st));
    int a0 = 0, b0 = 0;
    for (size_t k = 0; k < xs.size(); ++k) {
      const tdmrg_mps* x = xs[k];
      const cplx f = (s == 0) ? c[k] : cplx(1.0, 0.0);
      TRY_HIP(launch_block_copy(y->m->site[s], bonds[s], bonds[s + 1], x->site[s], x->bond[s], x->bond[s + 1], d,
                                s == 0 ? 0 : a0, s == n - 1 ? 0 : b0, f.real(), f.imag(), st));
      a0 += x->bond[s];
      b0 += x->bond[s + 1];
    }
  }
  return TDMRG_OK;
}

// <x|y> by the transfer-matrix chain with identity operators
tdmrg_status overlap(tdmrg_ctx* ctx, const tdmrg_mpo* mpo, const tdmrg_mps* x, const tdmrg_mps* y, cplx* out) {
  const int n = y->n;
  size_t need = 2;
  for (int b = 0; b <= n; ++b) need = std::max(need, 2 * (size_t)x->bond[b] * y->bond[b]);
  TRY(ensure(ctx, ctx->envA, need * sizeof(double)));
  TRY(ensure(ctx, ctx->envB, need * sizeof(double)));
  double* cur = (double*)ctx->envA.p;
  double* nxt = (double*)ctx->envB.p;
  const double one[2] = {1.0, 0.0};
  TRY_HIP(hipMemcpyAsync(cur, one, 2 * sizeof(double), hipMemcpyHostToDevice, ctx->stream));
  for (int s = 0; s < n; ++s) {
    TRY(env_left(ctx, cur, mpo->ident[s], x->site[s], x->bond[s], x->bond[s + 1], y->site[s], y->bond[s],
                 y->bond[s + 1], nxt, Arith::F64));
    std::swap(cur, nxt);
  }
  TRY_HIP(hipMemcpyAsync(ctx->host, cur, 2 * sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
  TRY_HIP(hipStreamSynchronize(ctx->stream));
  *out = cplx(ctx->host[0], ctx->host[1]);
  return TDMRG_OK;
}

// In-place compression (see the file header); adds the discarded weight.
tdmrg_status compress(tdmrg_ctx* ctx, tdmrg_mps* y, int D_max, double eps, double tie_rel, double* disc) {
  const int n = y->n;
  hipStream_t st = ctx->stream;
  // three scratch blocks, each as large as the largest site or bond matrix
  size_t big = 1;
  for (int s = 0; s < n; ++s) big = std::max(big, (size_t)site_len(y, s));
  for (int b = 0; b <= n; ++b) big = std::max(big, 2 * (size_t)y->bond[b] * y->bond[b]);
  TRY(ensure(ctx, ctx->gbuf, sizeof(double) * 2 * 3 * big));
  double* Q = (double*)ctx->gbuf.p;
  double* P = Q + 2 * big;
  double* C = P + 2 * big;
  // left to right: orthonormal site, the rest absorbed into the next site
  for (int s = 0; s + 1 < n; ++s) {
    const int Dl = y->bond[s], d = y->dims[s], Dr = y->bond[s + 1];
    const int rows = Dl * d;
    int k = Dr;
    if (Dr <= rows) {
      bool ok = true;
      TRY(qr_split(ctx, rows, Dr, y->site[s], false, Q, C, &ok));
    } else {  // wide: the bond shrinks to the block's size
      k = rows;
      TRY(qr_householder(ctx, rows, Dr, y->site[s], false, Q, C));
    }
    TRY_HIP(hipMemcpyAsync(y->site[s], Q, sizeof(double) * 2 * (size_t)rows * k, hipMemcpyDeviceToDevice, st));
    const int d2 = y->dims[s + 1], Dr2 = y->bond[s + 2];
    TRY(theta_form(ctx, k, 1, Dr, d2, Dr2, C, y->site[s + 1], P));
    TRY_HIP(hipMemcpyAsync(y->site[s + 1], P, sizeof(double) * 2 * (size_t)k * d2 * Dr2, hipMemcpyDeviceToDevice,
                           st));
    y->bond[s + 1] = k;
  }
  // right to left: DBSS truncation, U S absorbed into the previous site.
  // The site is Dl x (d Dr) with Dl much smaller than d Dr after an MPO
  // application, so it is first split M = L Q (Householder, Q with
  // orthonormal rows) and the truncated SVD runs on the small Dl x k0 factor
  // L = U S V^H; the new site is V_k^H Q and U_k S_k goes to the left.
  for (int s = n - 1; s >= 1; --s) {
    const int Dl = y->bond[s], d = y->dims[s], Dr = y->bond[s + 1];
    const int cols = d * Dr;
    const int k0 = std::min(Dl, cols);
    const int kcap = std::min(k0, D_max);
    int k = 0;
    double dd = 0.0;
    TRY(qr_householder(ctx, Dl, cols, y->site[s], true, Q, C));  // C: Dl x k0, Q: k0 x cols
    // L = C = U S V^H (Dl x k0): out1 = U S (Dl x k) into P, out2 = V^H (k x k0) after it
    double* US = P;
    double* Vh = P + 2 * (size_t)Dl * kcap;
    TRY(svd_truncate(ctx, Dl, k0, C, eps, kcap, 0, tie_rel, kcap, 2, US, Vh, nullptr, &k, &dd));
    *disc += dd;
    // new site = V_k^H Q (k x cols)
    TRY_HIP(tuned_cgemm(ctx, gemm_plain(k, cols, k0, Vh, Q, y->site[s]), Arith::F64, st));
    TRY_HIP(hipMemcpyAsync(C, US, sizeof(double) * 2 * (size_t)Dl * k, hipMemcpyDeviceToDevice, st));
    const int Dl0 = y->bond[s - 1], d0 = y->dims[s - 1];
    TRY(theta_form(ctx, Dl0, d0, Dl, 1, k, y->site[s - 1], C, P));  // C now holds U_k S_k
    TRY_HIP(hipMemcpyAsync(y->site[s - 1], P, sizeof(double) * 2 * (size_t)Dl0 * d0 * k, hipMemcpyDeviceToDevice,
                           st));
    y->bond[s] = k;
  }
  return TDMRG_OK;
}

int max_bond(const tdmrg_mps* m) { return *std::max_element(m->bond.begin(), m->bond.end()); }

}  // namespace

extern "C" tdmrg_status tdmrg_global_step(tdmrg_ctx* ctx, tdmrg_mps* mps, const tdmrg_mpo* mpo, double dt_fs,
                                          int method, int m_max, double tol, int D_max, double eps,
                                          tdmrg_global_stats* stats) {
  if (!ctx) return TDMRG_EINVAL;
  if (!mps || !mpo) return fail(ctx, TDMRG_EINVAL, "mps or mpo is NULL");
  if (mps->n != mpo->n || mps->dims != mpo->dims) return fail(ctx, TDMRG_ESHAPE, "mps and mpo do not match");
  if (mps->n < 2) return fail(ctx, TDMRG_ESHAPE, "need at least two sites");
  if (!std::isfinite(dt_fs) || !(eps >= 0.0) || D_max < 1 || (method < 0 || method > 2) || m_max < 1 ||
      m_max > 64 || !(tol >= 0.0))
    return fail(ctx, TDMRG_EINVAL, "invalid dt, method, m_max, tol, D_max or eps");
  // the caller's capacity bounds every bond of the result (it is at most the
  // full-rank bound of each bond, which no compression exceeds either)
  D_max = std::min(D_max, *std::max_element(mps->cap.begin(), mps->cap.end()));
  if (hipSetDevice(ctx->device) != hipSuccess) return fail(ctx, TDMRG_EDEVICE, "hipSetDevice failed");
  using clk = std::chrono::steady_clock;
  const auto t0 = clk::now();
  const double tie = 1e-12;
  double disc = 0.0;
  int peak = 1, used = 0;
  // the input as a vector of its own
  Vec psi;
  TRY(vec_alloc(ctx, mps->dims, mps->bond, &psi));
  for (int s = 0; s < mps->n; ++s)
    TRY_HIP(hipMemcpyAsync(psi.m->site[s], mps->site[s], sizeof(double) * 2 * (size_t)site_len(mps, s),
                           hipMemcpyDeviceToDevice, ctx->stream));
  // compressed c (H x)
  auto Hc = [&](const tdmrg_mps* x, cplx c, Vec* out) -> tdmrg_status {
    Vec hx;
    TRY(apply_mpo(ctx, mpo, x, &hx));
    peak = std::max(peak, max_bond(hx.m));
    TRY(compress(ctx, hx.m, D_max, eps, tie, &disc));
    TRY(lincomb(ctx, {c}, {hx.m}, out));
    return TDMRG_OK;
  };
  auto comb = [&](const std::vector<cplx>& c, const std::vector<const tdmrg_mps*>& xs, Vec* out) -> tdmrg_status {
    TRY(lincomb(ctx, c, xs, out));
    peak = std::max(peak, max_bond(out->m));
    TRY(compress(ctx, out->m, D_max, eps, tie, &disc));
    return TDMRG_OK;
  };
  Vec result;
  if (method == 1) {  // RK4
    const cplx f(0.0, -dt_fs / TDMRG_HBAR_EV_FS);
    Vec K1, K2, K3, K4, a2, a3, a4;
    TRY(Hc(psi.m, f, &K1));
    TRY(comb({1.0, 0.5}, {psi.m, K1.m}, &a2));
    TRY(Hc(a2.m, f, &K2));
    TRY(comb({1.0, 0.5}, {psi.m, K2.m}, &a3));
    TRY(Hc(a3.m, f, &K3));
    TRY(comb({1.0, 1.0}, {psi.m, K3.m}, &a4));
    TRY(Hc(a4.m, f, &K4));
    TRY(comb({1.0, 1.0 / 6, 1.0 / 3, 1.0 / 3, 1.0 / 6}, {psi.m, K1.m, K2.m, K3.m, K4.m}, &result));
    used = 4;
  } else if (method == 2) {  // Taylor expansion of order m_max
    const double tau = dt_fs / TDMRG_HBAR_EV_FS;
    // T_0 = psi, T_k = compressed (-i tau / k) H T_{k-1}; the sum compressed once
    std::vector<Vec> T(m_max + 1);
    std::vector<cplx> ones(m_max + 1, 1.0);
    std::vector<const tdmrg_mps*> xs = {psi.m};
    for (int k = 1; k <= m_max; ++k) {
      TRY(Hc(xs.back(), cplx(0.0, -tau / k), &T[k]));
      xs.push_back(T[k].m);
    }
    TRY(comb(ones, xs, &result));
    used = m_max;
  } else {  // global Krylov
    const double tau = dt_fs / TDMRG_HBAR_EV_FS;
    cplx nn;
    TRY(overlap(ctx, mpo, psi.m, psi.m, &nn));
    const double beta0 = std::sqrt(std::max(nn.real(), 0.0));
    if (!(beta0 > 0.0)) return fail(ctx, TDMRG_EINVAL, "the state has zero norm");
    std::vector<Vec> V;
    V.emplace_back();
    TRY(lincomb(ctx, {1.0 / beta0}, {psi.m}, &V.back()));
    std::vector<double> alpha, beta;
    // device block: alpha | beta | c_re | c_im | err
    TRY(ensure(ctx, ctx->gsmall, sizeof(double) * (4 * 64 + 8)));
    double* d_alpha = (double*)ctx->gsmall.p;
    double* d_beta = d_alpha + 64;
    double* d_cre = d_beta + 64;
    double* d_cim = d_cre + 64;
    double* d_err = d_cim + 64;
    std::vector<double> cre(m_max), cim(m_max);
    for (int j = 0; j < m_max; ++j) {
      Vec w;
      TRY(Hc(V[j].m, 1.0, &w));
      cplx a;
      TRY(overlap(ctx, mpo, V[j].m, w.m, &a));
      alpha.push_back(a.real());
      std::vector<cplx> c = {1.0, -a.real()};
      std::vector<const tdmrg_mps*> xs = {w.m, V[j].m};
      if (j > 0) {
        c.push_back(-beta[j - 1]);
        xs.push_back(V[j - 1].m);
      }
      Vec r;
      TRY(comb(c, xs, &r));
      cplx rr;
      TRY(overlap(ctx, mpo, r.m, r.m, &rr));
      const double b = std::sqrt(std::max(rr.real(), 0.0));
      // c = exp(-i tau T_{j+1}) e_1 on the device
      beta.push_back(b);
      TRY_HIP(hipMemcpyAsync(d_alpha, alpha.data(), sizeof(double) * alpha.size(), hipMemcpyHostToDevice,
                             ctx->stream));
      TRY_HIP(hipMemcpyAsync(d_beta, beta.data(), sizeof(double) * beta.size(), hipMemcpyHostToDevice,
                             ctx->stream));
      TRY_HIP(launch_tridiag_expm(d_alpha, d_beta, j + 1, tau, d_cre, d_cim, d_err, ctx->stream));
      TRY_HIP(hipMemcpyAsync(cre.data(), d_cre, sizeof(double) * (j + 1), hipMemcpyDeviceToHost, ctx->stream));
      TRY_HIP(hipMemcpyAsync(cim.data(), d_cim, sizeof(double) * (j + 1), hipMemcpyDeviceToHost, ctx->stream));
      TRY_HIP(hipStreamSynchronize(ctx->stream));
      const double err = b * std::abs(cplx(cre[j], cim[j]));
      used = j + 1;
      if (!(err == err)) return fail(ctx, TDMRG_EINVAL, "global Krylov produced NaN");
      if (err <= tol || j == m_max - 1 || b == 0.0) {
        std::vector<cplx> cc(j + 1);
        std::vector<const tdmrg_mps*> vs(j + 1);
        for (int k = 0; k <= j; ++k) {
          cc[k] = beta0 * cplx(cre[k], cim[k]);
          vs[k] = V[k].m;
        }
        TRY(comb(cc, vs, &result));
        break;
      }
      V.emplace_back();
      TRY(lincomb(ctx, {1.0 / b}, {r.m}, &V.back()));
    }
  }
  // write the result into the caller's MPS (bonds <= D_max <= its capacity)
  for (int b = 0; b <= mps->n; ++b)
    if (result.m->bond[b] > mps->cap[b]) return fail(ctx, TDMRG_ESHAPE, "result bond exceeds the MPS capacity");
  for (int s = 0; s < mps->n; ++s)
    TRY_HIP(hipMemcpyAsync(mps->site[s], result.m->site[s], sizeof(double) * 2 * (size_t)site_len(result.m, s),
                           hipMemcpyDeviceToDevice, ctx->stream));
  mps->bond = result.m->bond;
  mps->env_valid = false;
  TRY_HIP(hipStreamSynchronize(ctx->stream));
  if (stats) {
    stats->vectors = used;
    stats->max_intermediate_bond = peak;
    stats->sum_disc = disc;
    stats->seconds = std::chrono::duration<double>(clk::now() - t0).count();
  }
  return TDMRG_OK;
}
