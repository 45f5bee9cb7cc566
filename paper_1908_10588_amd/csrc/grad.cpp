// Gradient of an electronic population after a 2TDVP evolution with respect
// to the coupling constants of the vibronic model: the adjoint of the whole
// time evolution, for the ranks the forward run chose (the truncation ranks
// are piecewise constant in the parameters).
//
// Forward: the symmetric 2TDVP step (procedure after eq. two-site
// Hamiltonian, sweep reading of tdmrg_tdvp2_sweep), with the sites and the
// right environments checkpointed at the start of every time step.
// Reverse: from the last step to the first, the step is recomputed from its
// checkpoint with the inputs of every local operation recorded (bitwise the
// same operations), and the cotangents are carried back through the
// operations in reverse order -- the right-to-left half-sweep first, each
// pair as backward one-site exponential -> environment update -> truncation
// -> two-site exponential -> two-site tensor formation.  MPO cotangents
// accumulate over the whole run; the coupling constants enter the MPO
// linearly (eq. MPO), so dP/dp = sum_i Re <Wbar_i, W_i(p + e_p) - W_i(p)>.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
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

// Inputs of one pair update, recorded during the recomputation of a step.
struct Rec {
  int Dl = 0, Dm = 0, Dr = 0, d1 = 0, d2 = 0, k = 0;
  double *Min = nullptr, *Bin = nullptr, *th = nullptr, *thp = nullptr, *S = nullptr, *o1 = nullptr,
         *o2 = nullptr, *cin = nullptr;
};

// Device allocations owned by one gradient call.
struct Owned {
  std::vector<void*> ptrs;
  tdmrg_mpo* mpo = nullptr;
  tdmrg_mps* mps = nullptr;
  ~Owned() {
    for (void* p : ptrs) (void)hipFree(p);
    if (mps) tdmrg_mps_destroy(mps);
    if (mpo) tdmrg_mpo_destroy(mpo);
  }
};

const double kUnit[2] = {1.0, 0.0};

}  // namespace

static tdmrg_status dalloc(tdmrg_ctx* ctx, Owned& own, size_t doubles, double** out) {
  void* p = nullptr;
  if (hipMalloc(&p, sizeof(double) * std::max<size_t>(doubles, 2)) != hipSuccess)
    return fail(ctx, TDMRG_ENOMEM, "device allocation for the gradient failed");
  own.ptrs.push_back(p);
  *out = (double*)p;
  return TDMRG_OK;
}

static tdmrg_status dcopy(tdmrg_ctx* ctx, double* dst, const double* src, size_t doubles) {
  TRY_HIP(hipMemcpyAsync(dst, src, sizeof(double) * doubles, hipMemcpyDeviceToDevice, ctx->stream));
  return TDMRG_OK;
}

static tdmrg_status dzero(tdmrg_ctx* ctx, double* p, size_t doubles) {
  TRY_HIP(launch_fill(p, (long)doubles, 0.0, ctx->stream));
  return TDMRG_OK;
}

// Parameters of the model in a fixed order: E_i, V_ij (i < j), omega_I,
// g1[I][i][j] (i <= j), g2[k].  bump(m, idx, delta) changes one parameter of
// a model copy (both entries of a symmetric pair).
namespace {
struct ModelCopy {
  tdmrg_model m;
  std::vector<double> E, V, omega, g1, g2;
  explicit ModelCopy(const tdmrg_model* src) : m(*src) {
    const int ne = src->n_el, nm = src->n_modes;
    E.assign(src->E, src->E + ne);
    if (src->V) V.assign(src->V, src->V + (size_t)ne * ne);
    omega.assign(src->omega, src->omega + nm);
    g1.assign(src->g1, src->g1 + (size_t)nm * ne * ne);
    if (src->n_g2) g2.assign(src->g2, src->g2 + src->n_g2);
    m.E = E.data();
    m.V = src->V ? V.data() : nullptr;
    m.omega = omega.data();
    m.g1 = g1.data();
    m.g2 = src->n_g2 ? g2.data() : nullptr;
  }
};
}  // namespace

extern "C" tdmrg_status tdmrg_tdvp2_population_grad(tdmrg_ctx* ctx, const tdmrg_model* model, const int* occ,
                                                    int D_cap, int steps, double dt_fs, int D_max, double eps,
                                                    const tdmrg_opts* opts, int state, int nquad,
                                                    tdmrg_model_grad* grad, int* ranks, tdmrg_grad_info* info) {
  if (!ctx) return TDMRG_EINVAL;
  if (!model || !occ) return fail(ctx, TDMRG_EINVAL, "model or occ is NULL");
  TRY(validate_model(ctx, model));
  if (steps < 1 || D_cap < 1 || D_max < 1 || !(eps >= 0.0) || !std::isfinite(dt_fs))
    return fail(ctx, TDMRG_EINVAL, "invalid steps, D_cap, D_max, eps or dt");
  if (state < 0 || state >= model->n_el) return fail(ctx, TDMRG_EINVAL, "state out of range");
  if (model->el_per_state) return fail(ctx, TDMRG_EUNSUPPORTED, "the gradient takes the single electronic site");
  if (nquad < 2 || nquad > 64) return fail(ctx, TDMRG_EINVAL, "nquad must be in [2, 64]");
  tdmrg_opts o{TDMRG_FP64, 1e-12, 40, 0, 1e-12};
  if (opts) o = *opts;
  if (o.precision != TDMRG_FP64) return fail(ctx, TDMRG_EUNSUPPORTED, "the gradient runs in FP64 only");
  if (hipSetDevice(ctx->device) != hipSuccess) return fail(ctx, TDMRG_EDEVICE, "hipSetDevice failed");
  using clk = std::chrono::steady_clock;
  const auto t_start = clk::now();
  const long nodes0 = ctx->quad_nodes_used, calls0 = ctx->quad_calls;
  hipStream_t st = ctx->stream;
  Owned own;
  TRY(mpo_build(ctx, model, true, &own.mpo));  // zero couplings keep their channels
  TRY(tdmrg_mps_init(ctx, own.mpo, occ, D_cap, &own.mps));
  tdmrg_mpo* mpo = own.mpo;
  tdmrg_mps* mps = own.mps;
  const int n = mps->n;
  const std::vector<int>& dims = mps->dims;
  const std::vector<int>& cap = mps->cap;
  const std::vector<int>& wd = mpo->wdims;
  TRY(ensure_envs(ctx, mps, mpo));
  const double tau = dt_fs / (2.0 * TDMRG_HBAR_EV_FS);
  auto site_cap = [&](int j) { return 2 * (size_t)cap[j] * dims[j] * cap[j + 1]; };
  auto env_cap = [&](int b) { return 2 * (size_t)wd[b] * cap[b] * cap[b]; };
  auto pair_cap = [&](int i) { return 2 * (size_t)cap[i] * dims[i] * dims[i + 1] * cap[i + 2]; };

  // ---- forward with checkpoints (sites and right environments, compact)
  std::vector<std::vector<int>> ck_bond(steps + 1);
  std::vector<double*> ck(steps + 1, nullptr);
  std::vector<std::vector<size_t>> ck_site_off(steps + 1), ck_env_off(steps + 1);
  auto save = [&](int t) -> tdmrg_status {
    ck_bond[t] = mps->bond;
    size_t tot = 0;
    ck_site_off[t].assign(n, 0);
    ck_env_off[t].assign(n + 1, 0);
    for (int j = 0; j < n; ++j) {
      ck_site_off[t][j] = tot;
      tot += 2 * (size_t)mps->bond[j] * dims[j] * mps->bond[j + 1];
    }
    for (int b = 1; b <= n; ++b) {
      ck_env_off[t][b] = tot;
      tot += 2 * (size_t)wd[b] * mps->bond[b] * mps->bond[b];
    }
    TRY(dalloc(ctx, own, tot, &ck[t]));
    for (int j = 0; j < n; ++j)
      TRY(dcopy(ctx, ck[t] + ck_site_off[t][j], mps->site[j], 2 * (size_t)mps->bond[j] * dims[j] * mps->bond[j + 1]));
    for (int b = 1; b <= n; ++b)
      TRY(dcopy(ctx, ck[t] + ck_env_off[t][b], mps->R[b], 2 * (size_t)wd[b] * mps->bond[b] * mps->bond[b]));
    return TDMRG_OK;
  };
  auto restore = [&](int t) -> tdmrg_status {
    mps->bond = ck_bond[t];
    for (int j = 0; j < n; ++j)
      TRY(dcopy(ctx, mps->site[j], ck[t] + ck_site_off[t][j], 2 * (size_t)mps->bond[j] * dims[j] * mps->bond[j + 1]));
    for (int b = 1; b <= n; ++b)
      TRY(dcopy(ctx, mps->R[b], ck[t] + ck_env_off[t][b], 2 * (size_t)wd[b] * mps->bond[b] * mps->bond[b]));
    TRY_HIP(hipMemcpyAsync(mps->L[0], kUnit, 2 * sizeof(double), hipMemcpyHostToDevice, st));
    mps->env_valid = true;
    return TDMRG_OK;
  };
  for (int t = 0; t < steps; ++t) {
    TRY(save(t));
    TRY(tdmrg_tdvp2_sweep(ctx, mps, mpo, dt_fs, D_max, eps, &o, nullptr));
    if (ctx->verbose) {
      std::fprintf(stderr, "population gradient: forward step %d/%d, max bond %d\n", t + 1, steps,
                   *std::max_element(mps->bond.begin(), mps->bond.end()));
      std::fflush(stderr);
    }
  }
  ck_bond[steps] = mps->bond;

  // ---- observable P = <psi| P_state |psi> and its cotangents Mbar_j = 2 E_j M_j
  std::vector<const tdmrg_wop*> ops(mpo->ident.begin(), mpo->ident.end());
  ops[mpo->pop_site[state]] = mpo->proj[state];
  std::vector<double*> Mbar(n), Lbar(n + 1), Rbar(n + 1), Wbar(n), Lam(n + 1), Rho(n + 1);
  for (int j = 0; j < n; ++j) TRY(dalloc(ctx, own, site_cap(j), &Mbar[j]));
  for (int b = 0; b <= n; ++b) {
    TRY(dalloc(ctx, own, env_cap(b), &Lbar[b]));
    TRY(dalloc(ctx, own, env_cap(b), &Rbar[b]));
    TRY(dalloc(ctx, own, 2 * (size_t)cap[b] * cap[b], &Lam[b]));
    TRY(dalloc(ctx, own, 2 * (size_t)cap[b] * cap[b], &Rho[b]));
    TRY(dzero(ctx, Lbar[b], env_cap(b)));
    TRY(dzero(ctx, Rbar[b], env_cap(b)));
  }
  for (int i = 0; i < n; ++i) {
    const size_t wsz = 2 * (size_t)wd[i] * wd[i + 1] * dims[i] * dims[i];
    TRY(dalloc(ctx, own, wsz, &Wbar[i]));
    TRY(dzero(ctx, Wbar[i], wsz));
  }
  {
    const std::vector<int>& bd = mps->bond;
    TRY_HIP(hipMemcpyAsync(Lam[0], kUnit, 2 * sizeof(double), hipMemcpyHostToDevice, st));
    TRY_HIP(hipMemcpyAsync(Rho[n], kUnit, 2 * sizeof(double), hipMemcpyHostToDevice, st));
    for (int j = 0; j < n; ++j)
      TRY(env_left(ctx, Lam[j], ops[j], mps->site[j], bd[j], bd[j + 1], mps->site[j], bd[j], bd[j + 1], Lam[j + 1],
                   Arith::F64));
    for (int j = n - 1; j >= 0; --j)
      TRY(env_right(ctx, Rho[j + 1], ops[j], mps->site[j], bd[j], bd[j + 1], mps->site[j], bd[j], bd[j + 1], Rho[j],
                    Arith::F64));
    for (int j = 0; j < n; ++j) {
      TRY(heff1(ctx, bd[j], dims[j], bd[j + 1], Lam[j], ops[j], Rho[j + 1], mps->site[j], Mbar[j], Arith::F64));
      TRY_HIP(launch_cscale(Mbar[j], (long)bd[j] * dims[j] * bd[j + 1], 2.0, 0.0, st));
    }
    TRY_HIP(hipMemcpyAsync(ctx->host, Lam[n], 2 * sizeof(double), hipMemcpyDeviceToHost, st));
    TRY_HIP(hipStreamSynchronize(st));
  }
  const double pop = ctx->host[0];
  const double t_forward = std::chrono::duration<double>(clk::now() - t_start).count();

  // ---- records of one step (at capacity) and cotangent temporaries
  std::vector<Rec> lr(n - 1), rl(n - 1);
  size_t thmax = 0, smax = 0;
  for (int i = 0; i + 1 < n; ++i) {
    thmax = std::max(thmax, pair_cap(i));
    smax = std::max({smax, site_cap(i), site_cap(i + 1)});
    for (Rec* r : {&lr[i], &rl[i]}) {
      TRY(dalloc(ctx, own, site_cap(i), &r->Min));
      TRY(dalloc(ctx, own, site_cap(i + 1), &r->Bin));
      TRY(dalloc(ctx, own, pair_cap(i), &r->th));
      TRY(dalloc(ctx, own, pair_cap(i), &r->thp));
      TRY(dalloc(ctx, own, (size_t)cap[i + 1], &r->S));
      TRY(dalloc(ctx, own, site_cap(i), &r->o1));
      TRY(dalloc(ctx, own, site_cap(i + 1), &r->o2));
      TRY(dalloc(ctx, own, std::max(site_cap(i), site_cap(i + 1)), &r->cin));
    }
  }
  double *thb, *thpb, *X, *Y;
  TRY(dalloc(ctx, own, thmax, &thb));
  TRY(dalloc(ctx, own, thmax, &thpb));
  TRY(dalloc(ctx, own, smax, &X));
  TRY(dalloc(ctx, own, smax, &Y));
  TRY(ensure(ctx, ctx->theta, sizeof(double) * thmax));
  double* theta = (double*)ctx->theta.p;
  const int ntol = o.krylov_max;
  const double ktol = o.krylov_tol;

  // recompute one step with records (the operations of tdmrg_tdvp2_sweep)
  auto record_step = [&]() -> tdmrg_status {
    ExpmResult er;
    for (int i = 0; i + 1 < n; ++i) {
      Rec& r = lr[i];
      r.Dl = mps->bond[i]; r.Dm = mps->bond[i + 1]; r.Dr = mps->bond[i + 2];
      r.d1 = dims[i]; r.d2 = dims[i + 1];
      const int Dl = r.Dl, Dm = r.Dm, Dr = r.Dr, d1 = r.d1, d2 = r.d2;
      TRY(dcopy(ctx, r.Min, mps->site[i], 2 * (size_t)Dl * d1 * Dm));
      TRY(dcopy(ctx, r.Bin, mps->site[i + 1], 2 * (size_t)Dm * d2 * Dr));
      TRY(theta_form(ctx, Dl, d1, Dm, d2, Dr, mps->site[i], mps->site[i + 1], theta));
      const size_t th = 2 * (size_t)Dl * d1 * d2 * Dr;
      TRY(dcopy(ctx, r.th, theta, th));
      tdmrg_heff_shape s{Dl, d1, d2, Dr, wd[i], wd[i + 1], wd[i + 2]};
      TRY(local_expm(ctx, s, true, mps->L[i], mpo->W[i], mpo->W[i + 1], mps->R[i + 2], theta, tau, ktol, ntol,
                     Arith::F64, &er));
      TRY(dcopy(ctx, r.thp, theta, th));
      int k = 0;
      double disc = 0.0;
      TRY(svd_truncate(ctx, Dl * d1, d2 * Dr, theta, eps, std::min(D_max, cap[i + 1]), o.sv_mode, o.tie_rel,
                       cap[i + 1], 1, mps->site[i], mps->site[i + 1], r.S, &k, &disc));
      r.k = k;
      mps->bond[i + 1] = k;
      TRY(dcopy(ctx, r.o1, mps->site[i], 2 * (size_t)Dl * d1 * k));
      TRY(dcopy(ctx, r.o2, mps->site[i + 1], 2 * (size_t)k * d2 * Dr));
      TRY(env_left(ctx, mps->L[i], mpo->W[i], mps->site[i], Dl, k, mps->site[i], Dl, k, mps->L[i + 1], Arith::F64));
      if (i + 2 < n) {
        TRY(dcopy(ctx, r.cin, mps->site[i + 1], 2 * (size_t)k * d2 * Dr));
        tdmrg_heff_shape s1{k, d2, 1, Dr, wd[i + 1], 1, wd[i + 2]};
        TRY(local_expm(ctx, s1, false, mps->L[i + 1], mpo->W[i + 1], nullptr, mps->R[i + 2], mps->site[i + 1], -tau,
                       ktol, ntol, Arith::F64, &er));
      }
    }
    for (int i = n - 2; i >= 0; --i) {
      Rec& r = rl[i];
      r.Dl = mps->bond[i]; r.Dm = mps->bond[i + 1]; r.Dr = mps->bond[i + 2];
      r.d1 = dims[i]; r.d2 = dims[i + 1];
      const int Dl = r.Dl, Dm = r.Dm, Dr = r.Dr, d1 = r.d1, d2 = r.d2;
      TRY(dcopy(ctx, r.Min, mps->site[i], 2 * (size_t)Dl * d1 * Dm));
      TRY(dcopy(ctx, r.Bin, mps->site[i + 1], 2 * (size_t)Dm * d2 * Dr));
      TRY(theta_form(ctx, Dl, d1, Dm, d2, Dr, mps->site[i], mps->site[i + 1], theta));
      const size_t th = 2 * (size_t)Dl * d1 * d2 * Dr;
      TRY(dcopy(ctx, r.th, theta, th));
      tdmrg_heff_shape s{Dl, d1, d2, Dr, wd[i], wd[i + 1], wd[i + 2]};
      TRY(local_expm(ctx, s, true, mps->L[i], mpo->W[i], mpo->W[i + 1], mps->R[i + 2], theta, tau, ktol, ntol,
                     Arith::F64, &er));
      TRY(dcopy(ctx, r.thp, theta, th));
      int k = 0;
      double disc = 0.0;
      TRY(svd_truncate(ctx, Dl * d1, d2 * Dr, theta, eps, std::min(D_max, cap[i + 1]), o.sv_mode, o.tie_rel,
                       cap[i + 1], 2, mps->site[i], mps->site[i + 1], r.S, &k, &disc));
      r.k = k;
      mps->bond[i + 1] = k;
      TRY(dcopy(ctx, r.o1, mps->site[i], 2 * (size_t)Dl * d1 * k));
      TRY(dcopy(ctx, r.o2, mps->site[i + 1], 2 * (size_t)k * d2 * Dr));
      TRY(env_right(ctx, mps->R[i + 2], mpo->W[i + 1], mps->site[i + 1], k, Dr, mps->site[i + 1], k, Dr,
                    mps->R[i + 1], Arith::F64));
      if (i > 0) {
        TRY(dcopy(ctx, r.cin, mps->site[i], 2 * (size_t)Dl * d1 * k));
        tdmrg_heff_shape s1{Dl, d1, 1, k, wd[i], 1, wd[i + 1]};
        TRY(local_expm(ctx, s1, false, mps->L[i], mpo->W[i], nullptr, mps->R[i + 1], mps->site[i], -tau, ktol, ntol,
                       Arith::F64, &er));
      }
    }
    return TDMRG_OK;
  };

  // ---- reverse
  for (int t = steps - 1; t >= 0; --t) {
    if (ctx->verbose) {
      std::fprintf(stderr, "population gradient: reverse step %d/%d\n", steps - t, steps);
      std::fflush(stderr);
    }
    TRY(restore(t));
    TRY(record_step());
    if (mps->bond != ck_bond[t + 1])
      return fail(ctx, TDMRG_EDEVICE, "recomputed step " + std::to_string(t) + " chose other ranks than the forward run");
    if (ranks)
      for (int i = 0; i + 1 < n; ++i) {
        ranks[((size_t)t * 2 + 0) * (n - 1) + i] = lr[i].k;
        ranks[((size_t)t * 2 + 1) * (n - 1) + i] = rl[i].k;
      }
    auto rst = [&](int b) { return ck[t] + ck_env_off[t][b]; };  // right environments at the start of step t
    // right-to-left half-sweep, reversed (pairs 0 .. n-2)
    for (int i = 0; i + 1 < n; ++i) {
      const Rec& r = rl[i];
      const int Dl = r.Dl, Dm = r.Dm, Dr = r.Dr, d1 = r.d1, d2 = r.d2, k = r.k;
      const size_t sa = 2 * (size_t)Dl * d1 * k, sb = 2 * (size_t)k * d2 * Dr;
      if (i > 0) {
        TRY(local_expm1_vjp(ctx, Dl, k, mps->L[i], mpo->W[i], mps->R[i + 1], r.cin, -tau, Mbar[i], Lbar[i], Wbar[i],
                            Rbar[i + 1], X, nquad, ktol, ntol));
      } else {
        TRY(dcopy(ctx, X, Mbar[i], sa));
      }
      TRY(dcopy(ctx, Y, Mbar[i + 1], sb));
      TRY(env_right_vjp(ctx, mps->R[i + 2], mpo->W[i + 1], r.o2, k, Dr, r.o2, k, Dr, Rbar[i + 1], Rbar[i + 2],
                        Wbar[i + 1], Y, Y));
      TRY(dzero(ctx, Rbar[i + 1], env_cap(i + 1)));
      TRY(svd_trunc_vjp(ctx, Dl * d1, d2 * Dr, r.thp, 2, r.o1, r.o2, r.S, k, X, Y, thpb));
      tdmrg_heff_shape s{Dl, d1, d2, Dr, wd[i], wd[i + 1], wd[i + 2]};
      TRY(local_expm2_vjp(ctx, s, mps->L[i], mpo->W[i], mpo->W[i + 1], mps->R[i + 2], r.th, tau, thpb, Lbar[i],
                          Wbar[i], Wbar[i + 1], Rbar[i + 2], thb, nquad, ktol, ntol, true));
      TRY(dzero(ctx, Mbar[i], 2 * (size_t)Dl * d1 * Dm));
      TRY(dzero(ctx, Mbar[i + 1], 2 * (size_t)Dm * d2 * Dr));
      TRY(theta_form_vjp(ctx, Dl, d1, Dm, d2, Dr, r.Min, r.Bin, thb, Mbar[i], Mbar[i + 1]));
    }
    // left-to-right half-sweep, reversed (pairs n-2 .. 0)
    for (int i = n - 2; i >= 0; --i) {
      const Rec& r = lr[i];
      const int Dl = r.Dl, Dm = r.Dm, Dr = r.Dr, d1 = r.d1, d2 = r.d2, k = r.k;
      const size_t sa = 2 * (size_t)Dl * d1 * k, sb = 2 * (size_t)k * d2 * Dr;
      if (i + 2 < n) {
        TRY(local_expm1_vjp(ctx, k, Dr, mps->L[i + 1], mpo->W[i + 1], rst(i + 2), r.cin, -tau, Mbar[i + 1],
                            Lbar[i + 1], Wbar[i + 1], Rbar[i + 2], Y, nquad, ktol, ntol));
      } else {
        TRY(dcopy(ctx, Y, Mbar[i + 1], sb));
      }
      TRY(dcopy(ctx, X, Mbar[i], sa));
      TRY(env_left_vjp(ctx, mps->L[i], mpo->W[i], r.o1, Dl, k, r.o1, Dl, k, Lbar[i + 1], Lbar[i], Wbar[i], X, X));
      TRY(dzero(ctx, Lbar[i + 1], env_cap(i + 1)));
      TRY(svd_trunc_vjp(ctx, Dl * d1, d2 * Dr, r.thp, 1, r.o1, r.o2, r.S, k, X, Y, thpb));
      tdmrg_heff_shape s{Dl, d1, d2, Dr, wd[i], wd[i + 1], wd[i + 2]};
      TRY(local_expm2_vjp(ctx, s, mps->L[i], mpo->W[i], mpo->W[i + 1], rst(i + 2), r.th, tau, thpb, Lbar[i],
                          Wbar[i], Wbar[i + 1], Rbar[i + 2], thb, nquad, ktol, ntol, true));
      TRY(dzero(ctx, Mbar[i], 2 * (size_t)Dl * d1 * Dm));
      TRY(dzero(ctx, Mbar[i + 1], 2 * (size_t)Dm * d2 * Dr));
      TRY(theta_form_vjp(ctx, Dl, d1, Dm, d2, Dr, r.Min, r.Bin, thb, Mbar[i], Mbar[i + 1]));
    }
    TRY(dzero(ctx, Lbar[0], env_cap(0)));
  }
  // the right environments of the initial state (built site by site from the right)
  {
    const std::vector<int>& bd = ck_bond[0];
    for (int i = 1; i < n; ++i) {
      const double* site0 = ck[0] + ck_site_off[0][i];
      TRY(env_right_vjp(ctx, ck[0] + ck_env_off[0][i + 1], mpo->W[i], site0, bd[i], bd[i + 1], site0, bd[i],
                        bd[i + 1], Rbar[i], Rbar[i + 1], Wbar[i], nullptr, nullptr));
    }
  }
  // ---- MPO cotangents -> coupling constants
  std::vector<std::vector<double>> Wb(n);
  for (int i = 0; i < n; ++i) {
    Wb[i].resize(2 * (size_t)wd[i] * wd[i + 1] * dims[i] * dims[i]);
    TRY_HIP(hipMemcpyAsync(Wb[i].data(), Wbar[i], sizeof(double) * Wb[i].size(), hipMemcpyDeviceToHost, st));
  }
  TRY_HIP(hipStreamSynchronize(st));
  std::vector<int> d0, w0;
  std::vector<std::vector<double>> W0;
  std::vector<int> el0;
  TRY(build_mpo_host(ctx, model, &d0, &w0, &W0, &el0, true));
  // dP/dp for a model copy with one parameter changed by delta (the MPO is affine in it)
  auto dP = [&](ModelCopy& mc, double delta, double* out) -> tdmrg_status {
    std::vector<int> d1v, w1v;
    std::vector<std::vector<double>> W1;
    std::vector<int> el1;
    TRY(build_mpo_host(ctx, &mc.m, &d1v, &w1v, &W1, &el1, true));
    if (w1v != w0 || d1v != d0) return fail(ctx, TDMRG_EDEVICE, "MPO channel structure changed under a parameter step");
    double acc = 0.0;
    for (int i = 0; i < n; ++i)
      for (size_t e = 0; e < Wb[i].size(); ++e) acc += Wb[i][e] * (W1[i][e] - W0[i][e]);
    *out = acc / delta;
    return TDMRG_OK;
  };
  auto step_of = [](double v) { return v == -1.0 ? 2.0 : 1.0; };  // keep every term nonzero
  const int ne = model->n_el, nm = model->n_modes;
  if (grad && grad->E)
    for (int i = 0; i < ne; ++i) {
      ModelCopy mc(model);
      const double dl = step_of(mc.E[i]);
      mc.E[i] += dl;
      TRY(dP(mc, dl, &grad->E[i]));
    }
  if (grad && grad->V) {
    std::fill(grad->V, grad->V + (size_t)ne * ne, 0.0);
    for (int i = 0; i < ne; ++i)
      for (int j = i + 1; j < ne; ++j) {
        ModelCopy mc(model);
        const double dl = step_of(mc.V[(size_t)i * ne + j]);
        mc.V[(size_t)i * ne + j] += dl;
        mc.V[(size_t)j * ne + i] += dl;
        double g = 0.0;
        TRY(dP(mc, dl, &g));
        grad->V[(size_t)i * ne + j] = grad->V[(size_t)j * ne + i] = g;
      }
  }
  if (grad && grad->omega)
    for (int I = 0; I < nm; ++I) {
      ModelCopy mc(model);
      const double dl = step_of(mc.omega[I]);
      mc.omega[I] += dl;
      TRY(dP(mc, dl, &grad->omega[I]));
    }
  if (grad && grad->g1)
    for (int I = 0; I < nm; ++I)
      for (int i = 0; i < ne; ++i)
        for (int j = i; j < ne; ++j) {
          ModelCopy mc(model);
          const size_t a = ((size_t)I * ne + i) * ne + j, b = ((size_t)I * ne + j) * ne + i;
          const double dl = step_of(mc.g1[a]);
          mc.g1[a] += dl;
          if (b != a) mc.g1[b] += dl;
          double g = 0.0;
          TRY(dP(mc, dl, &g));
          grad->g1[a] = grad->g1[b] = g;
        }
  if (grad && grad->g2)
    for (int k = 0; k < model->n_g2; ++k) {
      ModelCopy mc(model);
      const double dl = step_of(mc.g2[k]);
      mc.g2[k] += dl;
      TRY(dP(mc, dl, &grad->g2[k]));
    }
  if (info) {
    info->pop = pop;
    info->seconds_forward = t_forward;
    info->seconds_total = std::chrono::duration<double>(clk::now() - t_start).count();
    const long nexp = ctx->quad_calls - calls0;
    info->mean_nodes = nexp > 0 ? (double)(ctx->quad_nodes_used - nodes0) / nexp : 0.0;
  }
  return TDMRG_OK;
}
