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
  for (DevBuf* b : {&ctx->vjpA, &ctx->vjpB, &ctx->vjpC, &ctx->vjpD})
    TRY(ensure(ctx, *b, sizeof(double) * 2 * (size_t)wmax * th));
  double* A = (double*)ctx->vjpA.p;
  double* B = (double*)ctx->vjpB.p;
  double* C = (double*)ctx->vjpC.p;
  double* D = (double*)ctx->vjpD.p;
  if (Rbar || W2bar) {
    // forward partials: X1 = L theta (A), X2 = W1 X1 (B), X3 = W2 X2 (C)
    TRY_HIP(launch_cgemm(agemm(s.wl * Dl, N1, Dl, 1, 1, aop(L, (long)s.wl * Dl * Dl, 0, 0, Dl, 0, 0),
                               aop(theta, th, 0, 0, N1, 0, 0), A, (long)s.wl * th, 0, N1, false),
                         Arith::F64, st));
    TRY_HIP(launch_mix(amix(W1, false, A, (long)s.wl * th, B, (long)s.wc * th, Dl, d2 * Dr), st));
    if (Rbar) {
      TRY_HIP(launch_mix(amix(W2, false, B, (long)s.wc * th, C, (long)s.wr * th, Dl * d1, Dr), st));
      // Rbar[v][b][b'] = sum_{ast} ybar[ast][b] conj(X3[v][ast][b'])
      TRY_HIP(launch_cgemm(agemm(Dr, Dr, M4, s.wr, 1, aop(ybar, th, 0, 0, Dr, 1, 0),
                                 aop(C, (long)s.wr * th, th, 0, Dr, 0, 1), Rbar, (long)s.wr * Dr * Dr,
                                 (long)Dr * Dr, Dr, acc),
                           Arith::F64, st));
    }
    if (W2bar) {
      const long w2im = (long)s.wc * s.wr * d2 * d2;
      for (int x = 0; x < s.wc; ++x) {
        // E[v][a s t'][b] = sum_b' X2[x][a s t'][b'] R[v][b][b']
        TRY_HIP(launch_cgemm(agemm(M4, Dr, Dr, s.wr, 1, aop(B + (long)x * th, (long)s.wc * th, 0, 0, Dr, 0, 0),
                                   aop(R, (long)s.wr * Dr * Dr, (long)Dr * Dr, 0, Dr, 1, 0), D,
                                   (long)s.wr * th, th, Dr, false),
                             Arith::F64, st));
        // W2bar[x][v][t][t'] = sum_{(a s), b} ybar[(as)][t][b] conj(E[v][(as)][t'][b])
        TRY_HIP(launch_cgemm(agemm(d2, d2, Dr, s.wr, Dl * d1, aop(ybar, th, 0, (long)d2 * Dr, Dr, 0, 0),
                                   aop(D, (long)s.wr * th, th, (long)d2 * Dr, Dr, 1, 1),
                                   W2bar + (long)x * s.wr * d2 * d2, w2im, (long)d2 * d2, d2, acc),
                             Arith::F64, st));
      }
    }
  }
  if (Lbar || W1bar) {
    // backward partials: T1 = theta R^T per channel v (A), G = W2-stage back to x (B)
    TRY_HIP(launch_cgemm(agemm(M4, Dr, Dr, s.wr, 1, aop(theta, th, 0, 0, Dr, 0, 0),
                               aop(R, (long)s.wr * Dr * Dr, (long)Dr * Dr, 0, Dr, 1, 0), A, (long)s.wr * th,
                               th, Dr, false),
                         Arith::F64, st));
    TRY_HIP(launch_mix(amix(W2, true, A, (long)s.wr * th, B, (long)s.wc * th, Dl * d1, Dr), st));
    if (Lbar) {
      // Z[w][a'][s][t][b] = sum W1[w][x][s][s'] G[x][a'][s'][t][b]
      TRY_HIP(launch_mix(amix(W1, true, B, (long)s.wc * th, C, (long)s.wl * th, Dl, d2 * Dr), st));
      // Lbar[w][a][a'] = sum_{stb} ybar[a][stb] conj(Z[w][a'][stb])
      TRY_HIP(launch_cgemm(agemm(Dl, Dl, N1, s.wl, 1, aop(ybar, th, 0, 0, N1, 0, 0),
                                 aop(C, (long)s.wl * th, th, 0, N1, 1, 1), Lbar, (long)s.wl * Dl * Dl,
                                 (long)Dl * Dl, Dl, acc),
                           Arith::F64, st));
    }
    if (W1bar) {
      const long w1im = (long)s.wl * s.wc * d1 * d1;
      const int Q = d2 * Dr;
      for (int w = 0; w < s.wl; ++w) {
        // F[x][a][s'][tb] = sum_a' L[w][a][a'] G[x][a'][s'][tb]
        TRY_HIP(launch_cgemm(agemm(Dl, N1, Dl, s.wc, 1,
                                   aop(L + (long)w * Dl * Dl, (long)s.wl * Dl * Dl, 0, 0, Dl, 0, 0),
                                   aop(B, (long)s.wc * th, th, 0, N1, 0, 0), D, (long)s.wc * th, th, N1, false),
                             Arith::F64, st));
        // W1bar[w][x][s][s'] = sum_{a, tb} ybar[a][s][tb] conj(F[x][a][s'][tb])
        TRY_HIP(launch_cgemm(agemm(d1, d1, Q, s.wc, Dl, aop(ybar, th, 0, (long)d1 * Q, Q, 0, 0),
                                   aop(D, (long)s.wc * th, th, (long)d1 * Q, Q, 1, 1),
                                   W1bar + (long)w * s.wc * d1 * d1, w1im, (long)d1 * d1, d1, acc),
                             Arith::F64, st));
      }
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

tdmrg_status local_expm2_vjp(tdmrg_ctx* ctx, const tdmrg_heff_shape& s, const double* L, const tdmrg_wop* W1,
                             const tdmrg_wop* W2, const double* R, const double* theta_in, double tau,
                             const double* ybar, double* Lbar, double* W1bar, double* W2bar, double* Rbar,
                             double* thetabar, int nquad, double tol, int m_max) {
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
  ExpmResult r;
  if (thetabar) {  // thetabar = exp(+i tau H^H) ybar
    TRY_HIP(hipMemcpyAsync(thetabar, ybar, vb, hipMemcpyDeviceToDevice, st));
    TRY(local_expm(ctx, s, true, LH, A1, A2, RH, thetabar, -tau, tol, m_max, Arith::F64, &r));
  }
  if (!Lbar && !W1bar && !W2bar && !Rbar) return TDMRG_OK;
  TRY(ensure(ctx, ctx->vjpU, vb));
  TRY(ensure(ctx, ctx->vjpV, vb));
  double* u = (double*)ctx->vjpU.p;
  double* v = (double*)ctx->vjpV.p;
  std::vector<double> xs, ws;
  gauss_legendre01(nquad, &xs, &ws);
  for (int q = 0; q < nquad; ++q) {
    // v = exp(-i tau s H) theta
    TRY_HIP(hipMemcpyAsync(v, theta_in, vb, hipMemcpyDeviceToDevice, st));
    TRY(local_expm(ctx, s, true, L, W1, W2, R, v, tau * xs[q], tol, m_max, Arith::F64, &r));
    // u = i tau w_q exp(+i tau (1-s) H^H) ybar
    TRY_HIP(hipMemcpyAsync(u, ybar, vb, hipMemcpyDeviceToDevice, st));
    TRY(local_expm(ctx, s, true, LH, A1, A2, RH, u, -tau * (1.0 - xs[q]), tol, m_max, Arith::F64, &r));
    TRY_HIP(launch_cscale(u, th, 0.0, tau * ws[q], st));
    TRY(heff2_vjp(ctx, s, L, W1, W2, R, v, u, Lbar, W1bar, W2bar, Rbar, nullptr, q > 0));
  }
  return TDMRG_OK;
}

}  // namespace tdmrg
