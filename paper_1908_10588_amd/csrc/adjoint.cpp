// Hand-written adjoints of the two-site effective-Hamiltonian product and of
// the local Lanczos exponential.
//
// Convention: for a real loss f and a complex array z the cotangent is
// zbar = df/dRe(z) + i df/dIm(z); for f = Re<ybar, y> and y = H theta this
// gives thetabar = H^H ybar and, for every operand X of H, Xbar equal to the
// contraction of ybar with the conjugate of y's partial derivative.
//
// For y = H_eff,2 theta (eq. two-site Hamiltonian),
//   y[a,s,t,b] = sum L[w][a][a'] W1[w][x][s][s'] W2[x][v][t][t'] R[v][b][b'] theta[a',s',t',b'],
// every cotangent is the contraction of ybar with the product of all other
// operands, evaluated stage by stage with the same GEMM and channel kernels
// as the forward product (environment-like contractions).
//
// For y = exp(-i tau H) theta:  thetabar = exp(+i tau H^H) ybar, and the
// operand cotangents follow from the Frechet derivative
//   dy = int_0^1 exp(-i tau (1-s) H) (-i tau dH) exp(-i tau s H) theta ds,
// i.e. Xbar = int_0^1 [VJP of H at v_s with cotangent i tau u_s] ds with
// v_s = exp(-i tau s H) theta and u_s = exp(+i tau (1-s) H^H) ybar, evaluated by
// Gauss-Legendre quadrature on [0, 1] (the integrand is analytic in s).
#include <algorithm>
#include <cmath>
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

static GemmOperand aop(const double* p, long im, long sb, long sr, long ld, int trans, int conj) {
  GemmOperand o;
  o.p = p; o.im = im; o.sb = sb; o.sr = sr; o.ld = ld; o.trans = trans; o.conj = conj;
  return o;
}

static GemmArgs agemm(int M, int N, int K, int nbatch, int nred, GemmOperand A, GemmOperand B, double* C,
                      long c_im, long c_sb, long ldc, bool acc) {
  GemmArgs g;
  g.M = M; g.N = N; g.K = K; g.nbatch = nbatch; g.nred = nred; g.role = 0;
  g.A = A; g.B = B; g.C = C; g.c_im = c_im; g.c_sb = c_sb; g.ldc = ldc;
  g.alpha_re = 1.0; g.alpha_im = 0.0; g.beta_re = acc ? 1.0 : 0.0; g.beta_im = 0.0;
  return g;
}

static MixArgs amix(const tdmrg_wop* W, bool backward, const double* in, long in_im, double* out,
                    long out_im, int P, int Q) {
  MixArgs a;
  a.in = in; a.in_im = in_im; a.out = out; a.out_im = out_im;
  a.P = P; a.Q = Q; a.din = W->d; a.dout = W->d;
  if (backward) {
    a.nout = W->wl; a.rowptr = W->b_rowptr; a.col = W->b_col; a.vre = W->b_v; a.vim = W->b_v + W->b_nnz;
  } else {
    a.nout = W->wr; a.rowptr = W->f_rowptr; a.col = W->f_col; a.vre = W->f_v; a.vim = W->f_v + W->f_nnz;
  }
  return a;
}

tdmrg_status heff2_vjp(tdmrg_ctx* ctx, const tdmrg_heff_shape& s, const double* L, const tdmrg_wop* W1,
                       const tdmrg_wop* W2, const double* R, const double* theta, const double* ybar,
                       double* Lbar, double* W1bar, double* W2bar, double* Rbar, double* thetabar,
                       bool acc) {
  hipStream_t st = ctx->stream;
  const long th = (long)s.Dl * s.d1 * s.d2 * s.Dr;
  const int wmax = std::max({s.wl, s.wc, s.wr});
  const int Dl = s.Dl, Dr = s.Dr, d1 = s.d1, d2 = s.d2;
  const int N1 = d1 * d2 * Dr, M4 = Dl * d1 * d2;
  // thetabar = H^H ybar: the same product with every factor daggered
  if (thetabar) {
    TRY(ensure(ctx, ctx->vjpL, sizeof(double) * 2 * (size_t)s.wl * Dl * Dl));
    TRY(ensure(ctx, ctx->vjpR, sizeof(double) * 2 * (size_t)s.wr * Dr * Dr));
    double* LH = (double*)ctx->vjpL.p;
    double* RH = (double*)ctx->vjpR.p;
    TRY_HIP(launch_conj_transpose(L, s.wl, Dl, LH, st));
    TRY_HIP(launch_conj_transpose(R, s.wr, Dr, RH, st));
    const tdmrg_wop *A1, *A2;
    TRY(wop_adjoint(ctx, W1, &A1));
    TRY(wop_adjoint(ctx, W2, &A2));
    TRY(heff2(ctx, s, LH, A1, A2, RH, ybar, thetabar, Arith::F64));
  }
  if (!Lbar && !W1bar && !W2bar && !Rbar) return TDMRG_OK;
  for (DevBuf* b : {&ctx->vjpA, &ctx->vjpB, &ctx->vjpC})
    TRY(ensure(ctx, *b, sizeof(double) * 2 * (size_t)wmax * th));
  // D also holds the [wc][wl][d1][d1] products of the W1 cotangent
  TRY(ensure(ctx, ctx->vjpD, sizeof(double) * 2 * std::max((size_t)wmax * th, (size_t)s.wc * s.wl * d1 * d1)));
  double* A = (double*)ctx->vjpA.p;
  double* B = (double*)ctx->vjpB.p;
  double* C = (double*)ctx->vjpC.p;
  double* D = (double*)ctx->vjpD.p;
  if (Rbar || W2bar) {
    // forward partials: X1 = L theta (A), X2 = W1 X1 (B), X3 = W2 X2 (C)
    TRY_HIP(tuned_cgemm(ctx, agemm(s.wl * Dl, N1, Dl, 1, 1, aop(L, (long)s.wl * Dl * Dl, 0, 0, Dl, 0, 0),
                               aop(theta, th, 0, 0, N1, 0, 0), A, (long)s.wl * th, 0, N1, false),
                         Arith::F64, st));
    TRY_HIP(launch_mix(amix(W1, false, A, (long)s.wl * th, B, (long)s.wc * th, Dl, d2 * Dr), st));
    if (Rbar) {
      TRY_HIP(launch_mix(amix(W2, false, B, (long)s.wc * th, C, (long)s.wr * th, Dl * d1, Dr), st));
      // Rbar[v][b][b'] = sum_{ast} ybar[ast][b] conj(X3[v][ast][b'])
      TRY_HIP(tuned_cgemm(ctx, agemm(Dr, Dr, M4, s.wr, 1, aop(ybar, th, 0, 0, Dr, 1, 0),
                                 aop(C, (long)s.wr * th, th, 0, Dr, 0, 1), Rbar, (long)s.wr * Dr * Dr,
                                 (long)Dr * Dr, Dr, acc),
                           Arith::F64, st));
    }
    if (W2bar) {
      // W2bar[x][v][t][t'] = sum_{(a s), b, b'} ybar[(as)][t][b] conj(X2[x][(as)][t'][b'] R[v][b][b']):
      // the right environment goes onto ybar once, Y[v][(as)][t][b'] = sum_b ybar[(as)][t][b] conj(R[v][b][b']),
      // then W2bar[x][v][t][t'] = sum_{(as), b'} Y[v][(as)][t][b'] conj(X2[x][(as)][t'][b'])
      TRY_HIP(tuned_cgemm(ctx, agemm(M4, Dr, Dr, s.wr, 1, aop(ybar, th, 0, 0, Dr, 0, 0),
                                 aop(R, (long)s.wr * Dr * Dr, (long)Dr * Dr, 0, Dr, 0, 1), D, (long)s.wr * th,
                                 th, Dr, false),
                           Arith::F64, st));
      // every x in one product: Y reordered to [(as)][v][t][b'] (in A, free
      // once X2 is formed) makes (v, t) the rows, x the batch
      TRY_HIP(launch_swap_outer(D, (long)s.wr * th, s.wr, Dl * d1, (long)d2 * Dr, A, (long)s.wr * th, false, st));
      const long w2im = (long)s.wc * s.wr * d2 * d2;
      TRY_HIP(tuned_cgemm(ctx, agemm(s.wr * d2, d2, Dr, s.wc, Dl * d1,
                                 aop(A, (long)s.wr * th, 0, (long)s.wr * d2 * Dr, Dr, 0, 0),
                                 aop(B, (long)s.wc * th, th, (long)d2 * Dr, Dr, 1, 1), W2bar, w2im,
                                 (long)s.wr * d2 * d2, d2, acc),
                           Arith::F64, st));
    }
  }
  if (Lbar || W1bar) {
    // backward partials: T1 = theta R^T per channel v (A), G = W2-stage back to x (B)
    TRY_HIP(tuned_cgemm(ctx, agemm(M4, Dr, Dr, s.wr, 1, aop(theta, th, 0, 0, Dr, 0, 0),
                               aop(R, (long)s.wr * Dr * Dr, (long)Dr * Dr, 0, Dr, 1, 0), A, (long)s.wr * th,
                               th, Dr, false),
                         Arith::F64, st));
    TRY_HIP(launch_mix(amix(W2, true, A, (long)s.wr * th, B, (long)s.wc * th, Dl * d1, Dr), st));
    if (Lbar) {
      // Z[w][a'][s][t][b] = sum W1[w][x][s][s'] G[x][a'][s'][t][b]
      TRY_HIP(launch_mix(amix(W1, true, B, (long)s.wc * th, C, (long)s.wl * th, Dl, d2 * Dr), st));
      // Lbar[w][a][a'] = sum_{stb} ybar[a][stb] conj(Z[w][a'][stb])
      TRY_HIP(tuned_cgemm(ctx, agemm(Dl, Dl, N1, s.wl, 1, aop(ybar, th, 0, 0, N1, 0, 0),
                                 aop(C, (long)s.wl * th, th, 0, N1, 1, 1), Lbar, (long)s.wl * Dl * Dl,
                                 (long)Dl * Dl, Dl, acc),
                           Arith::F64, st));
    }
    if (W1bar) {
      // W1bar[w][x][s][s'] = sum_{a, a', tb} ybar[a][s][tb] conj(L[w][a][a'] G[x][a'][s'][tb]):
      // the left environment goes onto ybar once, Yl[w][a'][s][tb] = sum_a conj(L[w][a][a']) ybar[a][s][tb],
      // then W1bar[w][x][s][s'] = sum_{a', tb} Yl[w][a'][s][tb] conj(G[x][a'][s'][tb])
      const long w1im = (long)s.wl * s.wc * d1 * d1;
      const int Q = d2 * Dr;
      TRY_HIP(tuned_cgemm(ctx, agemm(Dl, N1, Dl, s.wl, 1, aop(L, (long)s.wl * Dl * Dl, (long)Dl * Dl, 0, Dl, 1, 1),
                                 aop(ybar, th, 0, 0, N1, 0, 0), D, (long)s.wl * th, th, N1, false),
                           Arith::F64, st));
      // every w in one product: Yl reordered to [a'][w][s][tb] (in A, free
      // once G is formed) makes (w, s) the rows and x the batch; the result
      // [x][w][s][s'] (in D) is added to W1bar with its outer axes exchanged
      TRY_HIP(launch_swap_outer(D, (long)s.wl * th, s.wl, Dl, (long)d1 * Q, A, (long)s.wl * th, false, st));
      const long tim = (long)s.wc * s.wl * d1 * d1;
      TRY_HIP(tuned_cgemm(ctx, agemm(s.wl * d1, d1, Q, s.wc, Dl, aop(A, (long)s.wl * th, 0, (long)s.wl * d1 * Q, Q, 0, 0),
                                 aop(B, (long)s.wc * th, th, (long)d1 * Q, Q, 1, 1), D, tim,
                                 (long)s.wl * d1 * d1, d1, false),
                           Arith::F64, st));
      TRY_HIP(launch_swap_outer(D, tim, s.wc, s.wl, (long)d1 * d1, W1bar, w1im, acc, st));
    }
  }
  return TDMRG_OK;
}

// Gauss-Legendre nodes and weights on [0, 1]: Newton's method on the
// Legendre polynomial P_n (three-term recurrence), w = 2 / ((1 - z^2) P_n'(z)^2)
// on [-1, 1], mapped to [0, 1].
static void gauss_legendre01(int n, std::vector<double>* x, std::vector<double>* w) {
  // Newton iteration on P_n from Chebyshev initial guesses
  x->assign(n, 0.0);
  w->assign(n, 0.0);
  for (int i = 0; i < n; ++i) {
    double z = std::cos(M_PI * (i + 0.75) / (n + 0.5));
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = z;
      for (int k = 2; k <= n; ++k) {
        const double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      const double pn = (n == 1) ? z : p1, pn1 = (n == 1) ? 1.0 : p0;
      const double dp = n * (z * pn - pn1) / (z * z - 1.0);
      const double dz = pn / dp;
      z -= dz;
      if (std::fabs(dz) < 1e-16) break;
    }
    double p0 = 1.0, p1 = z;
    for (int k = 2; k <= n; ++k) {
      const double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
      p0 = p1;
      p1 = p2;
    }
    const double pn1 = (n == 1) ? 1.0 : p0, pn = (n == 1) ? z : p1;
    const double dp = n * (z * pn - pn1) / (z * z - 1.0);
    (*x)[i] = 0.5 * (1.0 - z);
    (*w)[i] = 1.0 / ((1.0 - z * z) * dp * dp);  // 2/((1-z^2)P'^2) on [-1,1], halved on [0,1]
  }
}

// Spectral interval [lo, hi] of a Krylov basis's T_m (Gershgorin bounds of
// the tridiagonal, read back).
static tdmrg_status krylov_interval(tdmrg_ctx* ctx, const KrylovBasis& kb, double* lo, double* hi) {
  hipStream_t st = ctx->stream;
  double* h = ctx->host;
  TRY_HIP(hipMemcpyAsync(h, kb.alpha, sizeof(double) * kb.m, hipMemcpyDeviceToHost, st));
  TRY_HIP(hipMemcpyAsync(h + 64, kb.beta, sizeof(double) * kb.m, hipMemcpyDeviceToHost, st));
  TRY_HIP(hipStreamSynchronize(st));
  *lo = INFINITY;
  *hi = -INFINITY;
  for (int i = 0; i < kb.m; ++i) {
    const double r = (i > 0 ? std::fabs(h[64 + i - 1]) : 0.0) + (i + 1 < kb.m ? std::fabs(h[64 + i]) : 0.0);
    *lo = std::min(*lo, h[i] - r);
    *hi = std::max(*hi, h[i] + r);
  }
  return TDMRG_OK;
}

// Gauss-Legendre nodes the Frechet integral needs: the integrand is a sum of
// terms exp(i w s) with |w| <= wmax (w = tau times a difference of two
// eigenvalues of H), and the n-point rule's error on [0, 1] for such a term is
// at most (n!)^4 wmax^(2n) / ((2n+1) ((2n)!)^3).  Smallest n in [2, nmax]
// with that below 1e-15.
static int quad_nodes(double wmax, int nmax) {
  if (!(wmax >= 0.0) || !std::isfinite(wmax)) return nmax;
  for (int n = 2; n < nmax; ++n) {
    const double lg = 4.0 * std::lgamma(n + 1.0) + 2.0 * n * std::log(std::max(wmax, 1e-300)) -
                      std::log(2.0 * n + 1.0) - 3.0 * std::lgamma(2.0 * n + 1.0);
    if (lg <= std::log(1e-15)) return n;
  }
  return nmax;
}

tdmrg_status local_expm2_vjp(tdmrg_ctx* ctx, const tdmrg_heff_shape& s, const double* L, const tdmrg_wop* W1,
                             const tdmrg_wop* W2, const double* R, const double* theta_in, double tau,
                             const double* ybar, double* Lbar, double* W1bar, double* W2bar, double* Rbar,
                             double* thetabar, int nquad, double tol, int m_max, bool acc) {
  hipStream_t st = ctx->stream;
  const long th = (long)s.Dl * s.d1 * s.d2 * s.Dr;
  const size_t vb = sizeof(double) * 2 * (size_t)th;
  // adjoint operands for the backward propagations
  TRY(ensure(ctx, ctx->vjpL, sizeof(double) * 2 * (size_t)s.wl * s.Dl * s.Dl));
  TRY(ensure(ctx, ctx->vjpR, sizeof(double) * 2 * (size_t)s.wr * s.Dr * s.Dr));
  double* LH = (double*)ctx->vjpL.p;
  double* RH = (double*)ctx->vjpR.p;
  TRY_HIP(launch_conj_transpose(L, s.wl, s.Dl, LH, st));
  TRY_HIP(launch_conj_transpose(R, s.wr, s.Dr, RH, st));
  const tdmrg_wop *A1, *A2;
  TRY(wop_adjoint(ctx, W1, &A1));
  TRY(wop_adjoint(ctx, W2, &A2));
  // One Krylov basis of (H^H, ybar) serves thetabar = exp(+i tau H^H) ybar and
  // every u_s; one of (H, theta) serves every v_s (a basis built to the
  // tolerance at time tau resolves every shorter time of the same sign).
  const bool ops = Lbar || W1bar || W2bar || Rbar;
  KrylovBasis ku, kv;
  TRY(expm_basis(ctx, s, LH, A1, A2, RH, ybar, -tau, tol, m_max, ctx->kryU, ctx->wvecU, ctx->smallU, &ku));
  if (thetabar) TRY(expm_from_basis(ctx, ku, -tau, thetabar));
  if (!ops) return TDMRG_OK;
  TRY(expm_basis(ctx, s, L, W1, W2, R, theta_in, tau, tol, m_max, ctx->kry, ctx->wvec, ctx->small, &kv));
  TRY(ensure(ctx, ctx->vjpU, vb));
  TRY(ensure(ctx, ctx->vjpV, vb));
  double* u = (double*)ctx->vjpU.p;
  double* v = (double*)ctx->vjpV.p;
  double lo_u, hi_u, lo_v, hi_v;
  TRY(krylov_interval(ctx, ku, &lo_u, &hi_u));
  TRY(krylov_interval(ctx, kv, &lo_v, &hi_v));
  const int nq = quad_nodes(std::fabs(tau) * (std::max(hi_u, hi_v) - std::min(lo_u, lo_v)), nquad);
  ctx->quad_nodes_used += nq;
  ctx->quad_calls++;
  std::vector<double> xs, ws;
  gauss_legendre01(nq, &xs, &ws);
  for (int q = 0; q < nq; ++q) {
    // v = exp(-i tau s H) theta;  u = i tau w_q exp(+i tau (1-s) H^H) ybar
    TRY(expm_from_basis(ctx, kv, tau * xs[q], v));
    TRY(expm_from_basis(ctx, ku, -tau * (1.0 - xs[q]), u));
    TRY_HIP(launch_cscale(u, th, 0.0, tau * ws[q], st));
    TRY(heff2_vjp(ctx, s, L, W1, W2, R, v, u, Lbar, W1bar, W2bar, Rbar, nullptr, acc || q > 0));
  }
  return TDMRG_OK;
}

// ------------------------------------------------------------------------
// Adjoints of the remaining steps of a 2TDVP time step (used by the
// gradient of a whole evolution).  Every cotangent output accumulates (+=).

// w x w identity channel map on a one-dimensional site: a one-site problem
// (L, W, R, M) is the two-site problem (L, W, I, R, M) with d2 = 1.
tdmrg_status ident_wop(tdmrg_ctx* ctx, int w, const tdmrg_wop** out) {
  auto it = ctx->ident_ops.find(w);
  if (it == ctx->ident_ops.end()) {
    std::vector<double> h(2 * (size_t)w * w, 0.0);
    for (int i = 0; i < w; ++i) h[(size_t)i * w + i] = 1.0;
    tdmrg_wop* a = nullptr;
    TRY(wop_make(ctx, w, w, 1, h.data(), &a));
    it = ctx->ident_ops.emplace(w, a).first;
  }
  *out = it->second;
  return TDMRG_OK;
}

tdmrg_status local_expm1_vjp(tdmrg_ctx* ctx, int Dl, int Dr, const double* L, const tdmrg_wop* W,
                             const double* R, const double* M_in, double tau, const double* ybar, double* Lbar,
                             double* Wbar, double* Rbar, double* Mbar, int nquad, double tol, int m_max) {
  const tdmrg_wop* I;
  TRY(ident_wop(ctx, W->wr, &I));
  const tdmrg_heff_shape s{Dl, W->d, 1, Dr, W->wl, W->wr, W->wr};
  return local_expm2_vjp(ctx, s, L, W, I, R, M_in, tau, ybar, Lbar, Wbar, nullptr, Rbar, Mbar, nquad, tol, m_max,
                         true);
}

// Lout[c][a][a'] = sum conj(bra[b][s][a]) Lin[w][b][b'] W[w][c][s][s'] ket[b'][s'][a']
// (the left environment update); cotangents from Obar = dL/dLout.
tdmrg_status env_left_vjp(tdmrg_ctx* ctx, const double* Lin, const tdmrg_wop* W, const double* bra, int Db,
                          int Db2, const double* ket, int Dk, int Dk2, const double* Obar, double* Lin_bar,
                          double* Wbar, double* bra_bar, double* ket_bar) {
  hipStream_t st = ctx->stream;
  const int wl = W->wl, wr = W->wr, d = W->d;
  const long tk = (long)Db * d * Dk2;
  const int wmax = std::max(wl, wr);
  for (DevBuf* b : {&ctx->vjpA, &ctx->vjpB, &ctx->vjpC, &ctx->vjpD})
    TRY(ensure(ctx, *b, sizeof(double) * 2 * (size_t)wmax * tk));
  double* T1 = (double*)ctx->vjpA.p;
  double* T2 = (double*)ctx->vjpB.p;
  double* T2b = (double*)ctx->vjpC.p;
  double* T1b = (double*)ctx->vjpD.p;
  const int N1 = d * Dk2;
  const long oim = (long)wr * Db2 * Dk2;
  // forward partials T1 = Lin ket, T2 = W T1
  TRY_HIP(tuned_cgemm(ctx, agemm(wl * Db, N1, Dk, 1, 1, aop(Lin, (long)wl * Db * Dk, 0, 0, Dk, 0, 0),
                             aop(ket, (long)Dk * N1, 0, 0, N1, 0, 0), T1, (long)wl * tk, 0, N1, false),
                       Arith::F64, st));
  TRY_HIP(launch_mix(amix(W, false, T1, (long)wl * tk, T2, (long)wr * tk, Db, Dk2), st));
  // bra_bar[b s][a] += sum_{c,a'} T2[c][b s][a'] conj(Obar[c][a][a'])
  if (bra_bar)
    TRY_HIP(tuned_cgemm(ctx, agemm(Db * d, Db2, Dk2, 1, wr, aop(T2, (long)wr * tk, 0, tk, Dk2, 0, 0),
                               aop(Obar, oim, 0, (long)Db2 * Dk2, Dk2, 1, 1), (double*)bra_bar, (long)Db * d * Db2,
                               0, Db2, true),
                         Arith::F64, st));
  // T2b[c][b s][a'] = sum_a bra[b s][a] Obar[c][a][a']
  TRY_HIP(tuned_cgemm(ctx, agemm(Db * d, Dk2, Db2, wr, 1, aop(bra, (long)Db * d * Db2, 0, 0, Db2, 0, 0),
                             aop(Obar, oim, (long)Db2 * Dk2, 0, Dk2, 0, 0), T2b, (long)wr * tk, tk, Dk2, false),
                       Arith::F64, st));
  if (Wbar) {
    // Wbar[w][c][s][s'] += sum_{b,a'} T2b[c][b][s][a'] conj(T1[w][b][s'][a'])
    const long wim = (long)wl * wr * d * d;
    for (int w = 0; w < wl; ++w)
      TRY_HIP(tuned_cgemm(ctx, agemm(d, d, Dk2, wr, Db, aop(T2b, (long)wr * tk, tk, (long)d * Dk2, Dk2, 0, 0),
                                 aop(T1 + (long)w * tk, (long)wl * tk, 0, (long)d * Dk2, Dk2, 1, 1),
                                 Wbar + (long)w * wr * d * d, wim, (long)d * d, d, true),
                           Arith::F64, st));
  }
  if (!Lin_bar && !ket_bar) return TDMRG_OK;
  // T1b[w][b][s'][a'] = sum_{c,s} conj(W[w][c][s][s']) T2b[c][b][s][a']  (adjoint operator, backward)
  const tdmrg_wop* Wa;
  TRY(wop_adjoint(ctx, W, &Wa));
  TRY_HIP(launch_mix(amix(Wa, true, T2b, (long)wr * tk, T1b, (long)wl * tk, Db, Dk2), st));
  // Lin_bar[w][b][b'] += sum_{s' a'} T1b[w][b][s' a'] conj(ket[b'][s' a'])
  if (Lin_bar)
    TRY_HIP(tuned_cgemm(ctx, agemm(Db, Dk, N1, wl, 1, aop(T1b, (long)wl * tk, tk, 0, N1, 0, 0),
                               aop(ket, (long)Dk * N1, 0, 0, N1, 1, 1), Lin_bar, (long)wl * Db * Dk,
                               (long)Db * Dk, Dk, true),
                         Arith::F64, st));
  // ket_bar[b'][s' a'] += sum_{w,b} conj(Lin[w][b][b']) T1b[w][b][s' a']
  if (ket_bar)
    TRY_HIP(tuned_cgemm(ctx, agemm(Dk, N1, Db, 1, wl, aop(Lin, (long)wl * Db * Dk, 0, (long)Db * Dk, Dk, 1, 1),
                               aop(T1b, (long)wl * tk, 0, tk, N1, 0, 0), ket_bar, (long)Dk * N1, 0, N1, true),
                         Arith::F64, st));
  return TDMRG_OK;
}

// Rout[w][a][a'] = sum conj(bra[a][s][b]) W[w][x][s][s'] ket[a'][s'][b'] Rin[x][b][b']
// (the right environment update); cotangents from Obar = dL/dRout.
tdmrg_status env_right_vjp(tdmrg_ctx* ctx, const double* Rin, const tdmrg_wop* W, const double* bra, int Db,
                           int Db2, const double* ket, int Dk, int Dk2, const double* Obar, double* Rin_bar,
                           double* Wbar, double* bra_bar, double* ket_bar) {
  hipStream_t st = ctx->stream;
  const int wl = W->wl, wr = W->wr, d = W->d;
  const long tk = (long)Dk * d * Db2;  // one channel: [a'][s][b]
  const int wmax = std::max(wl, wr);
  for (DevBuf* b : {&ctx->vjpA, &ctx->vjpB, &ctx->vjpC, &ctx->vjpD})
    TRY(ensure(ctx, *b, sizeof(double) * 2 * (size_t)wmax * tk));
  double* T1 = (double*)ctx->vjpA.p;
  double* T2 = (double*)ctx->vjpB.p;
  double* T2b = (double*)ctx->vjpC.p;
  double* T1b = (double*)ctx->vjpD.p;
  const int K = d * Db2;
  const long oim = (long)wl * Db * Dk;
  // forward partials: T1[x][a' s'][b] = sum_b' ket[a' s'][b'] Rin[x][b][b'];  T2 = W T1 (to the left channels)
  TRY_HIP(tuned_cgemm(ctx, agemm(Dk * d, Db2, Dk2, wr, 1, aop(ket, (long)Dk * d * Dk2, 0, 0, Dk2, 0, 0),
                             aop(Rin, (long)wr * Db2 * Dk2, (long)Db2 * Dk2, 0, Dk2, 1, 0), T1, (long)wr * tk, tk,
                             Db2, false),
                       Arith::F64, st));
  TRY_HIP(launch_mix(amix(W, true, T1, (long)wr * tk, T2, (long)wl * tk, Dk, Db2), st));
  // bra_bar[a][s b] += sum_{w,a'} conj(Obar[w][a][a']) T2[w][a'][s b]
  if (bra_bar)
    TRY_HIP(tuned_cgemm(ctx, agemm(Db, K, Dk, 1, wl, aop(Obar, oim, 0, (long)Db * Dk, Dk, 0, 1),
                               aop(T2, (long)wl * tk, 0, tk, K, 0, 0), bra_bar, (long)Db * K, 0, K, true),
                         Arith::F64, st));
  // T2b[w][a'][s b] = sum_a Obar[w][a][a'] bra[a][s b]
  TRY_HIP(tuned_cgemm(ctx, agemm(Dk, K, Db, wl, 1, aop(Obar, oim, (long)Db * Dk, 0, Dk, 1, 0),
                             aop(bra, (long)Db * K, 0, 0, K, 0, 0), T2b, (long)wl * tk, tk, K, false),
                       Arith::F64, st));
  if (Wbar) {
    // Wbar[w][x][s][s'] += sum_{a',b} T2b[w][a'][s][b] conj(T1[x][a'][s'][b])
    const long wim = (long)wl * wr * d * d;
    for (int x = 0; x < wr; ++x)
      TRY_HIP(tuned_cgemm(ctx, agemm(d, d, Db2, wl, Dk, aop(T2b, (long)wl * tk, tk, (long)d * Db2, Db2, 0, 0),
                                 aop(T1 + (long)x * tk, (long)wr * tk, 0, (long)d * Db2, Db2, 1, 1),
                                 Wbar + (long)x * d * d, wim, (long)wr * d * d, d, true),
                           Arith::F64, st));
  }
  if (!Rin_bar && !ket_bar) return TDMRG_OK;
  // T1b[x][a'][s'][b] = sum_{w,s} conj(W[w][x][s][s']) T2b[w][a'][s][b]  (adjoint operator, forward)
  const tdmrg_wop* Wa;
  TRY(wop_adjoint(ctx, W, &Wa));
  TRY_HIP(launch_mix(amix(Wa, false, T2b, (long)wl * tk, T1b, (long)wr * tk, Dk, Db2), st));
  // Rin_bar[x][b][b'] += sum_{a' s'} T1b[x][a' s'][b] conj(ket[a' s'][b'])
  if (Rin_bar)
    TRY_HIP(tuned_cgemm(ctx, agemm(Db2, Dk2, Dk * d, wr, 1, aop(T1b, (long)wr * tk, tk, 0, Db2, 1, 0),
                               aop(ket, (long)Dk * d * Dk2, 0, 0, Dk2, 0, 1), Rin_bar, (long)wr * Db2 * Dk2,
                               (long)Db2 * Dk2, Dk2, true),
                         Arith::F64, st));
  // ket_bar[a' s'][b'] += sum_{x,b} T1b[x][a' s'][b] conj(Rin[x][b][b'])
  if (ket_bar)
    TRY_HIP(tuned_cgemm(ctx, agemm(Dk * d, Dk2, Db2, 1, wr, aop(T1b, (long)wr * tk, 0, tk, Db2, 0, 0),
                               aop(Rin, (long)wr * Db2 * Dk2, 0, (long)Db2 * Dk2, Dk2, 0, 1), ket_bar,
                               (long)Dk * d * Dk2, 0, Dk2, true),
                         Arith::F64, st));
  return TDMRG_OK;
}

// theta = M B (contraction over the middle bond): Mbar += thetabar B^H, Bbar += M^H thetabar.
tdmrg_status theta_form_vjp(tdmrg_ctx* ctx, int Dl, int d1, int Dm, int d2, int Dr, const double* M,
                            const double* B, const double* thetabar, double* Mbar, double* Bbar) {
  hipStream_t st = ctx->stream;
  const int Mr = Dl * d1, N = d2 * Dr;
  const long th = (long)Mr * N;
  if (Mbar)
    TRY_HIP(tuned_cgemm(ctx, agemm(Mr, Dm, N, 1, 1, aop(thetabar, th, 0, 0, N, 0, 0),
                               aop(B, (long)Dm * N, 0, 0, N, 1, 1), Mbar, (long)Mr * Dm, 0, Dm, true),
                         Arith::F64, st));
  if (Bbar)
    TRY_HIP(tuned_cgemm(ctx, agemm(Dm, N, Mr, 1, 1, aop(M, (long)Mr * Dm, 0, 0, Dm, 1, 1),
                               aop(thetabar, th, 0, 0, N, 0, 0), Bbar, (long)Dm * N, 0, N, true),
                         Arith::F64, st));
  return TDMRG_OK;
}

// Adjoint of the rank-k truncation theta -> (A, C) with A = U_k orthonormal
// (m x k) and C = S_k V_k^H = A^H theta (k x n), for a loss that is
// invariant under A -> A Q, C -> Q^H C for unitary Q (the gauge of the kept
// bond).  With the full SVD of theta, U_perp the left singular vectors not
// kept (s_j) and Ubar_t = Abar + theta Cbar^H,
//   thetabar = A Cbar + U_perp (Z C) + A Z^H (U_perp^H theta)
//              + (I - U_all U_all^H) Ubar_t S_k^-2 C,
//   Z[j][i] = (U_perp^H Ubar_t)[j][i] / (s_i^2 - s_j^2),
// the first-order change of the kept singular subspace (projector
// derivative) chained with dC = dA^H theta + A^H dtheta.  Pairs with
// |s_i^2 - s_j^2| <= 1e-14 s_0^2 (a multiplet split by the cut) are dropped.
static tdmrg_status svd_left_vjp(tdmrg_ctx* ctx, int m, int n, const double* theta, const double* A,
                                 const double* S, const double* C, const double* Abar, const double* Cbar, int k,
                                 double* thetabar) {
  hipStream_t st = ctx->stream;
  const int r = std::min(m, n);
  const int kp = r - k;  // discarded within the rank
  const long mn = (long)m * n;
  // workspace: U_all [m][r], Vh_all [r][n], s_all [r], Ubar_t [m][k], Y/Z [kp][k], T_zc [kp][n],
  // T_ut [kp][n], T_zt [k][n], Us [m][k], T_us [r][k], T_usc [r][n]
  const size_t need = 2 * ((size_t)m * r + (size_t)r * n + (size_t)m * k + (size_t)kp * k + 2 * (size_t)kp * n +
                           (size_t)k * n + (size_t)m * k + (size_t)r * k + (size_t)r * n) + (size_t)r + 64;
  TRY(ensure(ctx, ctx->adjw, need * sizeof(double)));
  double* w = (double*)ctx->adjw.p;
  double* Ua = w; w += 2 * (long)m * r;
  double* Vha = w; w += 2 * (long)r * n;
  double* sa = w; w += r;
  double* Ut = w; w += 2 * (long)m * k;
  double* Z = w; w += 2 * (long)kp * k;
  double* Tzc = w; w += 2 * (long)kp * n;
  double* Tut = w; w += 2 * (long)kp * n;
  double* Tzt = w; w += 2 * (long)k * n;
  double* Us = w; w += 2 * (long)m * k;
  double* Tus = w; w += 2 * (long)r * k;
  double* Tusc = w;
  int kk = 0;
  double disc = 0.0;
  // Every singular triplet is needed.  Past the crossover of the two routes
  // (the one-workgroup Jacobi SVD takes about 8 ns per unit of m^2 (m + n),
  // the Gram route has a floor of about 2 ms) the Gram route serves: its
  // s_j^2 carry an absolute error of about eps s_0^2, which enters only
  // through 1/(s_i^2 - s_j^2) between a kept and a discarded value, and any
  // orthonormal basis of a near-null space gives the same cotangent there
  // (the U_perp term with s_j -> 0 equals the null-space projection term).
  const int method = ctx->svd_method;
  if (method == 0 && (double)m * m * (m + n) > 2.5e5) ctx->svd_method = 2;
  const tdmrg_status sst = svd_truncate(ctx, m, n, theta, 0.0, r, 2, 0.0, r, 0, Ua, Vha, sa, &kk, &disc);
  ctx->svd_method = method;
  TRY(sst);
  if (kk != r) return fail(ctx, TDMRG_EDEVICE, "full SVD of the truncation adjoint returned a short rank");
  const double* Up = Ua + k;  // columns k .. r-1 of U_all (row stride r)
  // Ubar_t = Abar + theta Cbar^H
  TRY_HIP(hipMemcpyAsync(Ut, Abar, sizeof(double) * 2 * (size_t)m * k, hipMemcpyDeviceToDevice, st));
  TRY_HIP(tuned_cgemm(ctx, agemm(m, k, n, 1, 1, aop(theta, mn, 0, 0, n, 0, 0), aop(Cbar, (long)k * n, 0, 0, n, 1, 1),
                             Ut, (long)m * k, 0, k, true),
                       Arith::F64, st));
  // thetabar = A Cbar
  TRY_HIP(tuned_cgemm(ctx, agemm(m, n, k, 1, 1, aop(A, (long)m * k, 0, 0, k, 0, 0), aop(Cbar, (long)k * n, 0, 0, n, 0, 0),
                             thetabar, mn, 0, n, false),
                       Arith::F64, st));
  if (kp > 0) {
    // Z = (U_perp^H Ubar_t) o F
    TRY_HIP(tuned_cgemm(ctx, agemm(kp, k, m, 1, 1, aop(Up, (long)m * r, 0, 0, r, 1, 1), aop(Ut, (long)m * k, 0, 0, k, 0, 0),
                               Z, (long)kp * k, 0, k, false),
                         Arith::F64, st));
    TRY_HIP(launch_gap_scale(Z, kp, k, sa + k, S, sa, st));
    // thetabar += U_perp (Z C)
    TRY_HIP(tuned_cgemm(ctx, agemm(kp, n, k, 1, 1, aop(Z, (long)kp * k, 0, 0, k, 0, 0), aop(C, (long)k * n, 0, 0, n, 0, 0),
                               Tzc, (long)kp * n, 0, n, false),
                         Arith::F64, st));
    TRY_HIP(tuned_cgemm(ctx, agemm(m, n, kp, 1, 1, aop(Up, (long)m * r, 0, 0, r, 0, 0), aop(Tzc, (long)kp * n, 0, 0, n, 0, 0),
                               thetabar, mn, 0, n, true),
                         Arith::F64, st));
    // thetabar += A (Z^H (U_perp^H theta))
    TRY_HIP(tuned_cgemm(ctx, agemm(kp, n, m, 1, 1, aop(Up, (long)m * r, 0, 0, r, 1, 1), aop(theta, mn, 0, 0, n, 0, 0),
                               Tut, (long)kp * n, 0, n, false),
                         Arith::F64, st));
    TRY_HIP(tuned_cgemm(ctx, agemm(k, n, kp, 1, 1, aop(Z, (long)kp * k, 0, 0, k, 1, 1), aop(Tut, (long)kp * n, 0, 0, n, 0, 0),
                               Tzt, (long)k * n, 0, n, false),
                         Arith::F64, st));
    TRY_HIP(tuned_cgemm(ctx, agemm(m, n, k, 1, 1, aop(A, (long)m * k, 0, 0, k, 0, 0), aop(Tzt, (long)k * n, 0, 0, n, 0, 0),
                               thetabar, mn, 0, n, true),
                         Arith::F64, st));
  }
  {
    // thetabar += (I - U_all U_all^H) Ubar_t S^-2 C  (the part outside the
    // computed singular vectors: the null space, and directions of zero
    // singular values a one-sided Jacobi SVD leaves as zero columns)
    TRY_HIP(hipMemcpyAsync(Us, Ut, sizeof(double) * 2 * (size_t)m * k, hipMemcpyDeviceToDevice, st));
    TRY_HIP(launch_scale_cols_inv2(Us, m, k, S, st));
    TRY_HIP(tuned_cgemm(ctx, agemm(m, n, k, 1, 1, aop(Us, (long)m * k, 0, 0, k, 0, 0), aop(C, (long)k * n, 0, 0, n, 0, 0),
                               thetabar, mn, 0, n, true),
                         Arith::F64, st));
    TRY_HIP(tuned_cgemm(ctx, agemm(r, k, m, 1, 1, aop(Ua, (long)m * r, 0, 0, r, 1, 1), aop(Us, (long)m * k, 0, 0, k, 0, 0),
                               Tus, (long)r * k, 0, k, false),
                         Arith::F64, st));
    TRY_HIP(tuned_cgemm(ctx, agemm(r, n, k, 1, 1, aop(Tus, (long)r * k, 0, 0, k, 0, 0), aop(C, (long)k * n, 0, 0, n, 0, 0),
                               Tusc, (long)r * n, 0, n, false),
                         Arith::F64, st));
    GemmArgs gn = agemm(m, n, r, 1, 1, aop(Ua, (long)m * r, 0, 0, r, 0, 0), aop(Tusc, (long)r * n, 0, 0, n, 0, 0),
                        thetabar, mn, 0, n, true);
    gn.alpha_re = -1.0;
    TRY_HIP(tuned_cgemm(ctx, gn, Arith::F64, st));
  }
  return TDMRG_OK;
}

tdmrg_status svd_trunc_vjp(tdmrg_ctx* ctx, int m, int n, const double* theta, int mode, const double* out1,
                           const double* out2, const double* S, int k, const double* out1_bar, const double* out2_bar,
                           double* thetabar) {
  if (mode == 1) return svd_left_vjp(ctx, m, n, theta, out1, S, out2, out1_bar, out2_bar, k, thetabar);
  // mode 2: out1 = U S [m][k], out2 = Vh [k][n]; theta^H = V (S U^H) is the mode-1 form
  // of the transpose with A = out2^H, C = out1^H
  const long mn = (long)m * n;
  TRY(ensure(ctx, ctx->adjt, sizeof(double) * 2 * (size_t)(2 * mn + 4 * (size_t)k * std::max(m, n))));
  double* w = (double*)ctx->adjt.p;
  double* thH = w; w += 2 * mn;
  double* tbH = w; w += 2 * mn;
  double* A = w; w += 2 * (long)n * k;
  double* C = w; w += 2 * (long)k * m;
  double* Ab = w; w += 2 * (long)n * k;
  double* Cb = w;
  hipStream_t st = ctx->stream;
  TRY_HIP(launch_conj_transpose_rect(theta, m, n, thH, st));
  TRY_HIP(launch_conj_transpose_rect(out2, k, n, A, st));
  TRY_HIP(launch_conj_transpose_rect(out1, m, k, C, st));
  TRY_HIP(launch_conj_transpose_rect(out2_bar, k, n, Ab, st));
  TRY_HIP(launch_conj_transpose_rect(out1_bar, m, k, Cb, st));
  TRY(svd_left_vjp(ctx, n, m, thH, A, S, C, Ab, Cb, k, tbH));
  TRY_HIP(launch_conj_transpose_rect(tbH, n, m, thetabar, st));
  return TDMRG_OK;
}

}  // namespace tdmrg
