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
  if (xs.size() > 1) TRY(check_intermediate(ctx, bonds));  // one vector: a rescaled copy
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

// ---- the variational procedure (eq. variational app) ----------------------
// |phi> minimising || |phi> - sum_k c_k O_k |x_k> ||^2 by sweeping two-site
// updates: with |phi> mixed-canonical around the pair (i, i+1), the
// minimum is Phi = sum_k c_k L_k (O_k,i O_k,i+1) R_k theta_k, theta_k =
// x_k,i x_k,i+1, L_k / R_k the left / right blocks of <phi| O_k |x_k>
// (bra bonds of phi, ket bonds of x_k); Phi is truncated by the DBSS rule
// (eps, D_max), left to right into U (left-orthonormal) and S V^H, right to
// left into U S and V^H.  A sweep is both directions; sweeping stops when
// |phi|^2 (the last pair's singular values) changes by at most tol relative
// (the global steps use 1e-15, about the rounding level of the norm), or
// after max_sweeps (16).  The start is a right-canonical copy of x_0.  No
// intermediate with bonds D * w or sum_k D_k is ever formed.
struct FitTerm {
  cplx c;
  const std::vector<tdmrg_wop*>* ops;  // one operator per site (the MPO, or identities)
  const tdmrg_mps* x;
};

// device arrays owned by one fit, released through the context's allocator
struct Scratch {
  tdmrg_ctx* ctx;
  std::vector<void*> ptrs;
  explicit Scratch(tdmrg_ctx* c) : ctx(c) {}
  ~Scratch() {
    (void)hipStreamSynchronize(ctx->stream);
    for (void* p : ptrs) dev_free(ctx, p);
  }
  tdmrg_status get(size_t doubles, double** out) {
    void* p = nullptr;
    TRY(dev_alloc(ctx, sizeof(double) * std::max<size_t>(doubles, 2), &p));
    ptrs.push_back(p);
    *out = (double*)p;
    return TDMRG_OK;
  }
};

tdmrg_status fit(tdmrg_ctx* ctx, const std::vector<FitTerm>& terms, int D_max, double eps, double tie, int max_sweeps,
                 double tol, double* disc_out, int* sweeps_out, Vec* out) {
  const tdmrg_mps* x0 = terms[0].x;
  const int n = x0->n;
  const std::vector<int>& dims = x0->dims;
  hipStream_t st = ctx->stream;
  // bond capacities of phi: min(D_max, full-rank cut); it starts with x_0's bonds
  std::vector<int> caps(n + 1, 1);
  {
    std::vector<long> left(n + 1, 1), right(n + 1, 1);
    for (int b = 1; b <= n; ++b) left[b] = std::min<long>(left[b - 1] * dims[b - 1], D_max);
    for (int b = n - 1; b >= 0; --b) right[b] = std::min<long>(right[b + 1] * dims[b], D_max);
    for (int b = 0; b <= n; ++b) caps[b] = (int)std::max<long>(1, std::min({left[b], right[b], (long)D_max}));
    for (int b = 0; b <= n; ++b) caps[b] = std::max(caps[b], x0->bond[b]);
  }
  TRY(vec_alloc(ctx, dims, caps, out));
  tdmrg_mps* phi = out->m;
  phi->bond = x0->bond;
  for (int s = 0; s < n; ++s)
    TRY_HIP(hipMemcpyAsync(phi->site[s], x0->site[s], sizeof(double) * 2 * (size_t)site_len(x0, s),
                           hipMemcpyDeviceToDevice, st));
  Scratch sc(ctx);
  // work blocks: Phi, theta of a term, and the QR pieces of the start
  size_t phimax = 1, thmax = 1, qmax = 1, cmax = 1;
  for (int i = 0; i + 1 < n; ++i) {
    phimax = std::max(phimax, (size_t)caps[i] * dims[i] * dims[i + 1] * caps[i + 2]);
    for (const FitTerm& t : terms)
      thmax = std::max(thmax, (size_t)t.x->bond[i] * dims[i] * dims[i + 1] * t.x->bond[i + 2]);
  }
  for (int s = 0; s < n; ++s) {
    qmax = std::max(qmax, (size_t)caps[s] * dims[s] * caps[s + 1]);
    cmax = std::max(cmax, (size_t)caps[s] * caps[s]);
  }
  double *Phi, *Th, *Q, *C, *Sv;
  TRY(sc.get(2 * phimax, &Phi));
  TRY(sc.get(2 * std::max(thmax, qmax), &Th));
  TRY(sc.get(2 * qmax, &Q));
  TRY(sc.get(2 * cmax, &C));
  TRY(sc.get((size_t)D_max + 8, &Sv));
  // right-canonical start: M_s = C Q from the right, C absorbed into site s-1
  for (int s = n - 1; s >= 1; --s) {
    const int Dl = phi->bond[s], d = dims[s], Dr = phi->bond[s + 1];
    bool ok = true;
    TRY(qr_split(ctx, Dl, d * Dr, phi->site[s], true, Q, C, &ok));
    TRY_HIP(hipMemcpyAsync(phi->site[s], Q, sizeof(double) * 2 * (size_t)Dl * d * Dr, hipMemcpyDeviceToDevice, st));
    const int Dl0 = phi->bond[s - 1], d0 = dims[s - 1];
    TRY(theta_form(ctx, Dl0, d0, Dl, 1, Dl, phi->site[s - 1], C, Th));
    TRY_HIP(hipMemcpyAsync(phi->site[s - 1], Th, sizeof(double) * 2 * (size_t)Dl0 * d0 * Dl, hipMemcpyDeviceToDevice,
                           st));
  }
  // environments of every term: L[k][b] [w_b][phi bond][x_k bond], R likewise
  const size_t nt = terms.size();
  std::vector<std::vector<double*>> Lk(nt, std::vector<double*>(n + 1)), Rk(nt, std::vector<double*>(n + 1));
  const double one[2] = {1.0, 0.0};
  for (size_t k = 0; k < nt; ++k) {
    const FitTerm& t = terms[k];
    for (int b = 0; b <= n; ++b) {
      const int w = b == 0 ? (*t.ops)[0]->wl : (*t.ops)[b - 1]->wr;
      TRY(sc.get(2 * (size_t)w * caps[b] * t.x->bond[b], &Lk[k][b]));
      TRY(sc.get(2 * (size_t)w * caps[b] * t.x->bond[b], &Rk[k][b]));
    }
    TRY_HIP(hipMemcpyAsync(Lk[k][0], one, 2 * sizeof(double), hipMemcpyHostToDevice, st));
    TRY_HIP(hipMemcpyAsync(Rk[k][n], one, 2 * sizeof(double), hipMemcpyHostToDevice, st));
    for (int s = n - 1; s >= 2; --s)
      TRY(env_right(ctx, Rk[k][s + 1], (*t.ops)[s], phi->site[s], phi->bond[s], phi->bond[s + 1], t.x->site[s],
                    t.x->bond[s], t.x->bond[s + 1], Rk[k][s], Arith::F64));
  }
  // Phi of pair i from every term into the Phi block
  auto pair = [&](int i) -> tdmrg_status {
    for (size_t k = 0; k < nt; ++k) {
      const FitTerm& t = terms[k];
      const tdmrg_mps* x = t.x;
      TRY(theta_form(ctx, x->bond[i], dims[i], x->bond[i + 1], dims[i + 1], x->bond[i + 2], x->site[i],
                     x->site[i + 1], Th));
      TRY(heff2_rect(ctx, phi->bond[i], x->bond[i], dims[i], dims[i + 1], phi->bond[i + 2], x->bond[i + 2],
                     Lk[k][i], (*t.ops)[i], (*t.ops)[i + 1], Rk[k][i + 2], Th, Phi, t.c.real(), t.c.imag(),
                     k == 0 ? 0.0 : 1.0));
    }
    return TDMRG_OK;
  };
  double last = -1.0;
  int sweep = 0;
  std::vector<double> hs(D_max + 8);
  for (sweep = 1; sweep <= max_sweeps; ++sweep) {
    double disc = 0.0, dd = 0.0;
    int k = 0;
    for (int i = 0; i + 1 < n; ++i) {  // left to right
      TRY(pair(i));
      const int rows = phi->bond[i] * dims[i], cols = dims[i + 1] * phi->bond[i + 2];
      TRY(svd_truncate(ctx, rows, cols, Phi, eps, std::min(D_max, caps[i + 1]), 0, tie, caps[i + 1], 1,
                       phi->site[i], phi->site[i + 1], nullptr, &k, &dd));
      phi->bond[i + 1] = k;
      for (size_t t = 0; t < nt; ++t) {
        const tdmrg_mps* x = terms[t].x;
        TRY(env_left(ctx, Lk[t][i], (*terms[t].ops)[i], phi->site[i], phi->bond[i], k, x->site[i], x->bond[i],
                     x->bond[i + 1], Lk[t][i + 1], Arith::F64));
      }
    }
    for (int i = n - 2; i >= 0; --i) {  // right to left
      TRY(pair(i));
      const int rows = phi->bond[i] * dims[i], cols = dims[i + 1] * phi->bond[i + 2];
      TRY(svd_truncate(ctx, rows, cols, Phi, eps, std::min(D_max, caps[i + 1]), 0, tie, caps[i + 1], 2,
                       phi->site[i], phi->site[i + 1], i == 0 ? Sv : nullptr, &k, &dd));
      disc += dd;
      phi->bond[i + 1] = k;
      for (size_t t = 0; t < nt; ++t) {
        const tdmrg_mps* x = terms[t].x;
        TRY(env_right(ctx, Rk[t][i + 2], (*terms[t].ops)[i + 1], phi->site[i + 1], k, phi->bond[i + 2],
                      x->site[i + 1], x->bond[i + 1], x->bond[i + 2], Rk[t][i + 1], Arith::F64));
      }
    }
    // |phi|^2 from the singular values of the last pair
    TRY_HIP(hipMemcpyAsync(hs.data(), Sv, sizeof(double) * k, hipMemcpyDeviceToHost, st));
    TRY_HIP(hipStreamSynchronize(st));
    double nrm = 0.0;
    for (int j = 0; j < k; ++j) nrm += hs[j] * hs[j];
    *disc_out = disc;
    if (last >= 0.0 && std::abs(nrm - last) <= tol * std::max(nrm, 1e-300)) break;
    last = nrm;
  }
  *sweeps_out = std::min(sweep, max_sweeps);
  return TDMRG_OK;
}

}  // namespace

extern "C" tdmrg_status tdmrg_ctx_set_mpo_apply(tdmrg_ctx* ctx, int mode) {
  if (!ctx) return TDMRG_EINVAL;
  if (mode != 0 && mode != 1) return fail(ctx, TDMRG_EINVAL, "MPO application mode must be 0 or 1");
  ctx->mpo_apply = mode;
  return TDMRG_OK;
}

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
  // compressed c (H x): the direct product then compressed, or the
  // variational fit (tdmrg_ctx_set_mpo_apply)
  const bool variational = ctx->mpo_apply == 1;
  const int fit_sweeps = 16;
  const double fit_tol = 1e-15;
  auto Hc = [&](const tdmrg_mps* x, cplx c, Vec* out) -> tdmrg_status {
    Vec hx;
    if (variational) {
      double dd = 0.0;
      int sw = 0;
      TRY(fit(ctx, {FitTerm{cplx(1.0, 0.0), &mpo->W, x}}, D_max, eps, tie, fit_sweeps, fit_tol, &dd, &sw, &hx));
      disc += dd;
    } else {
      TRY(apply_mpo(ctx, mpo, x, &hx));
      peak = std::max(peak, max_bond(hx.m));
      TRY(compress(ctx, hx.m, D_max, eps, tie, &disc));
    }
    peak = std::max(peak, max_bond(hx.m));
    TRY(lincomb(ctx, {c}, {hx.m}, out));
    return TDMRG_OK;
  };
  auto comb = [&](const std::vector<cplx>& c, const std::vector<const tdmrg_mps*>& xs, Vec* out) -> tdmrg_status {
    if (variational) {
      std::vector<FitTerm> terms;
      for (size_t k = 0; k < xs.size(); ++k) terms.push_back(FitTerm{c[k], &mpo->ident, xs[k]});
      double dd = 0.0;
      int sw = 0;
      TRY(fit(ctx, terms, D_max, eps, tie, fit_sweeps, fit_tol, &dd, &sw, out));
      disc += dd;
      peak = std::max(peak, max_bond(out->m));
      return TDMRG_OK;
    }
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
