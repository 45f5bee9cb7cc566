// MPO of the vibronic Hamiltonian (paper eq. MPO and Section 2.2) by a
// finite-state construction, built on the host.
//
// The Hamiltonian is a sum of terms c * prod_s op_s, each a product of local
// operators on distinct chain sites.  On the bond b between sites b-1 and b a
// multi-site term whose sites straddle b occupies a channel:
//   * "suffix" terms (first operator left of the electronic site) are keyed
//     by the operators they still have to apply (sites >= b); the coefficient
//     is applied with the first operator, so channels sum the partial
//     products of all terms that share the same remainder
//     (e.g. sum_I g_ij^I q_I waiting for |i><j|);
//   * "prefix" terms (first operator on or right of the electronic site) are
//     keyed by the operators already applied (sites < b); the coefficient is
//     applied with the last operator (e.g. |i><j| waiting for sum_J g_ij^J q_J).
// Two extra channels carry "nothing applied yet" (identity) and "a complete
// term" (identity).  Transitions between shared channels are added once.
#include <algorithm>
#include <cmath>
#include <map>
#include <set>
#include <utility>
#include <vector>

#include "internal.h"

namespace tdmrg {

enum OpCode { OP_I = 0, OP_NHALF, OP_Q, OP_Q2, OP_HEL, OP_OCC, OP_CR, OP_AN, OP_EL_BASE = 100 };

static int el_code(int i, int j, int n_el) {
  if (i > j) std::swap(i, j);
  return OP_EL_BASE + i * n_el + j;
}

// Real local operator matrix d x d (row-major).
static std::vector<double> local_op(int code, int d, const tdmrg_model* m) {
  std::vector<double> o((size_t)d * d, 0.0);
  switch (code) {
    case OP_I:
      for (int k = 0; k < d; ++k) o[k * d + k] = 1.0;
      break;
    case OP_NHALF:
      for (int k = 0; k < d; ++k) o[k * d + k] = k + 0.5;
      break;
    case OP_Q:  // (b^+ + b)/sqrt(2)
      for (int k = 0; k + 1 < d; ++k) o[k * d + k + 1] = o[(k + 1) * d + k] = std::sqrt((k + 1) / 2.0);
      break;
    case OP_Q2:  // exact truncated matrix elements of q^2
      for (int k = 0; k < d; ++k) {
        o[k * d + k] = (2.0 * k + 1.0) / 2.0;
        if (k + 2 < d) o[k * d + k + 2] = o[(k + 2) * d + k] = std::sqrt((k + 1.0) * (k + 2.0)) / 2.0;
      }
      break;
    case OP_OCC:  // per-state site: n = |1><1|
      o[3] = 1.0;
      break;
    case OP_CR:  // a^+ = |1><0|
      o[2] = 1.0;
      break;
    case OP_AN:  // a = |0><1|
      o[1] = 1.0;
      break;
    case OP_HEL:
      for (int i = 0; i < d; ++i)
        for (int j = 0; j < d; ++j) o[i * d + j] = (i == j) ? m->E[i] : (m->V ? m->V[i * d + j] : 0.0);
      break;
    default: {
      const int ij = code - OP_EL_BASE;
      const int i = ij / d, j = ij % d;
      o[i * d + j] = 1.0;
      o[j * d + i] = 1.0;
    }
  }
  return o;
}

struct Term {
  double c;
  std::vector<std::pair<int, int>> ops;  // (site, code), ascending site
};

typedef std::pair<int, std::vector<std::pair<int, int>>> ChanKey;  // (kind, ops)

tdmrg_status validate_model(const tdmrg_ctx* ctx, const tdmrg_model* m) {
  if (!m) return fail(ctx, TDMRG_EINVAL, "model is NULL");
  if (m->n_el < 1 || m->n_modes < 1) return fail(ctx, TDMRG_EINVAL, "need n_el >= 1 and n_modes >= 1");
  if (!m->E || !m->omega || !m->nbasis || !m->g1 || !m->order)
    return fail(ctx, TDMRG_EINVAL, "model array pointer is NULL");
  if (m->n_el > 1 && !m->V) return fail(ctx, TDMRG_EINVAL, "V is NULL");
  if (m->n_g2 < 0 || (m->n_g2 > 0 && (!m->g2 || !m->g2_I || !m->g2_J || !m->g2_i || !m->g2_j)))
    return fail(ctx, TDMRG_EINVAL, "second-order term arrays invalid");
  auto finite = [](double x) { return std::isfinite(x); };
  for (int i = 0; i < m->n_el; ++i)
    if (!finite(m->E[i])) return fail(ctx, TDMRG_EINVAL, "E is not finite");
  if (m->V)
    for (int i = 0; i < m->n_el * m->n_el; ++i)
      if (!finite(m->V[i])) return fail(ctx, TDMRG_EINVAL, "V is not finite");
  for (int i = 0; i < m->n_el; ++i)
    for (int j = 0; j < m->n_el; ++j)
      if (m->V && i != j && m->V[i * m->n_el + j] != m->V[j * m->n_el + i])
        return fail(ctx, TDMRG_EINVAL, "V is not symmetric");
  for (int I = 0; I < m->n_modes; ++I) {
    if (!finite(m->omega[I])) return fail(ctx, TDMRG_EINVAL, "omega is not finite");
    if (m->nbasis[I] < 2) return fail(ctx, TDMRG_EINVAL, "nbasis must be >= 2");
  }
  const long ng1 = (long)m->n_modes * m->n_el * m->n_el;
  for (long k = 0; k < ng1; ++k)
    if (!finite(m->g1[k])) return fail(ctx, TDMRG_EINVAL, "g1 is not finite");
  for (int I = 0; I < m->n_modes; ++I)
    for (int i = 0; i < m->n_el; ++i)
      for (int j = 0; j < m->n_el; ++j) {
        const long a = ((long)I * m->n_el + i) * m->n_el + j, b = ((long)I * m->n_el + j) * m->n_el + i;
        if (m->g1[a] != m->g1[b]) return fail(ctx, TDMRG_EINVAL, "g1 is not symmetric in (i, j)");
      }
  for (int k = 0; k < m->n_g2; ++k) {
    if (!finite(m->g2[k])) return fail(ctx, TDMRG_EINVAL, "g2 is not finite");
    if (m->g2_I[k] < 0 || m->g2_I[k] >= m->n_modes || m->g2_J[k] < 0 || m->g2_J[k] >= m->n_modes ||
        m->g2_i[k] < 0 || m->g2_i[k] >= m->n_el || m->g2_j[k] < 0 || m->g2_j[k] >= m->n_el)
      return fail(ctx, TDMRG_EINVAL, "g2 index out of range");
  }
  if (m->el_per_state != 0 && m->el_per_state != 1) return fail(ctx, TDMRG_EINVAL, "el_per_state must be 0 or 1");
  const int n_sites = m->n_modes + (m->el_per_state ? m->n_el : 1);
  std::vector<int> seen(m->n_modes, 0), seen_el(m->n_el, 0);
  int n_el_sites = 0;
  for (int s = 0; s < n_sites; ++s) {
    const int o = m->order[s];
    if (o < 0) {
      const int i = -1 - o;
      if (m->el_per_state ? (i >= m->n_el || seen_el[i]) : (o != -1))
        return fail(ctx, TDMRG_EINVAL, "order has an invalid electronic entry");
      if (m->el_per_state) seen_el[i] = 1;
      ++n_el_sites;
      continue;
    }
    if (o >= m->n_modes || seen[o]) return fail(ctx, TDMRG_EINVAL, "order is not a permutation");
    seen[o] = 1;
  }
  if (n_el_sites != (m->el_per_state ? m->n_el : 1))
    return fail(ctx, TDMRG_EINVAL, m->el_per_state ? "order must contain -1 .. -n_el once each"
                                                   : "order must contain exactly one -1");
  return TDMRG_OK;
}

// Builds W[s] as dense host arrays [2][wl][wr][d][d] (imaginary part zero).
tdmrg_status build_mpo_host(const tdmrg_ctx* ctx, const tdmrg_model* m, std::vector<int>* dims_out,
                            std::vector<int>* wdims_out, std::vector<std::vector<double>>* W_out,
                            std::vector<int>* pop_sites, bool keep_zero) {
  const bool ps = m->el_per_state != 0;
  const int n = m->n_modes + (ps ? m->n_el : 1);
  std::vector<int> pos(m->n_modes), dims(n), es(m->n_el);
  int el = n;  // first electronic site
  for (int s = 0; s < n; ++s) {
    if (m->order[s] < 0) {
      el = std::min(el, s);
      if (ps) {
        es[-1 - m->order[s]] = s;
        dims[s] = 2;
      } else {
        for (int i = 0; i < m->n_el; ++i) es[i] = s;
        dims[s] = m->n_el;
      }
    } else {
      pos[m->order[s]] = s;
      dims[s] = m->nbasis[m->order[s]];
    }
  }
  // ---- terms
  std::vector<Term> terms;
  auto add = [&](double c, std::vector<std::pair<int, int>> ops) {
    if (c == 0.0 && !keep_zero) return;
    std::sort(ops.begin(), ops.end());
    terms.push_back(Term{c, ops});
  };
  // electronic factor |i><j| (+ h.c. for i != j) times the mode operators in
  // `rest`: one term on the electronic site, or with per-state sites n_i
  // (i == j) or the two terms a_i^+ a_j and a_j^+ a_i
  auto add_el = [&](double c, int i, int j, std::vector<std::pair<int, int>> rest) {
    if (!ps) {
      rest.push_back({el, el_code(i, j, m->n_el)});
      add(c, rest);
      return;
    }
    if (i == j) {
      rest.push_back({es[i], OP_OCC});
      add(c, rest);
      return;
    }
    auto r2 = rest;
    rest.push_back({es[i], OP_CR});
    rest.push_back({es[j], OP_AN});
    add(c, rest);
    r2.push_back({es[i], OP_AN});
    r2.push_back({es[j], OP_CR});
    add(c, r2);
  };
  if (ps) {
    for (int i = 0; i < m->n_el; ++i) add_el(m->E[i], i, i, {});
    for (int i = 0; i < m->n_el; ++i)
      for (int j = i + 1; j < m->n_el; ++j) add_el(m->V[i * m->n_el + j], i, j, {});
  } else {
    add(1.0, {{el, OP_HEL}});
  }
  for (int I = 0; I < m->n_modes; ++I) add(m->omega[I], {{pos[I], OP_NHALF}});
  for (int I = 0; I < m->n_modes; ++I)
    for (int i = 0; i < m->n_el; ++i)
      for (int j = i; j < m->n_el; ++j) add_el(m->g1[((long)I * m->n_el + i) * m->n_el + j], i, j, {{pos[I], OP_Q}});
  for (int k = 0; k < m->n_g2; ++k) {
    const int I = m->g2_I[k], J = m->g2_J[k];
    const int i = std::min(m->g2_i[k], m->g2_j[k]), j = std::max(m->g2_i[k], m->g2_j[k]);
    if (I == J) add_el(m->g2[k], i, j, {{pos[I], OP_Q2}});
    else add_el(m->g2[k], i, j, {{pos[I], OP_Q}, {pos[J], OP_Q}});
  }
  // ---- channels
  const ChanKey START{0, {}}, DONE{1, {}};
  std::vector<std::map<ChanKey, int>> chan(n + 1);
  for (int b = 0; b <= n; ++b) {
    if (b < n) {
      const int idx = (int)chan[b].size();
      chan[b][START] = idx;
    }
    if (b > 0) {
      const int idx = (int)chan[b].size();
      chan[b][DONE] = idx;
    }
  }
  auto key = [&](const Term& t, int b) {
    const bool suffix = t.ops.front().first < el;
    ChanKey k{suffix ? 3 : 2, {}};
    for (auto& o : t.ops)
      if (suffix ? (o.first >= b) : (o.first < b)) k.second.push_back(o);
    return k;
  };
  for (auto& t : terms) {
    if (t.ops.size() < 2) continue;
    for (int b = t.ops.front().first + 1; b <= t.ops.back().first; ++b) {
      ChanKey k = key(t, b);
      if (!chan[b].count(k)) {
        const int idx = (int)chan[b].size();
        chan[b][k] = idx;
      }
    }
  }
  std::vector<int> wd(n + 1);
  for (int b = 0; b <= n; ++b) wd[b] = (int)chan[b].size();
  // ---- tensors
  W_out->assign(n, {});
  for (int s = 0; s < n; ++s) {
    const int d = dims[s], wl = wd[s], wr = wd[s + 1];
    std::vector<double>& W = (*W_out)[s];
    W.assign(2 * (size_t)wl * wr * d * d, 0.0);
    auto acc = [&](int a, int b, double c, const std::vector<double>& o) {
      double* blk = W.data() + ((size_t)a * wr + b) * d * d;
      for (int x = 0; x < d * d; ++x) blk[x] += c * o[x];
    };
    const std::vector<double> eye = local_op(OP_I, d, m);
    if (chan[s].count(START) && chan[s + 1].count(START)) acc(chan[s][START], chan[s + 1][START], 1.0, eye);
    if (chan[s].count(DONE) && chan[s + 1].count(DONE)) acc(chan[s][DONE], chan[s + 1][DONE], 1.0, eye);
    std::set<std::pair<int, int>> once;
    for (auto& t : terms) {
      const int first = t.ops.front().first, last = t.ops.back().first;
      if (s < first || s > last) continue;
      int code = OP_I;
      for (auto& o : t.ops)
        if (o.first == s) code = o.second;
      const std::vector<double> o = local_op(code, d, m);
      if (first == last) {
        acc(chan[s][START], chan[s + 1][DONE], t.c, o);
        continue;
      }
      const bool suffix = first < el;
      const int cin = (s == first) ? chan[s][START] : chan[s][key(t, s)];
      const int cout = (s == last) ? chan[s + 1][DONE] : chan[s + 1][key(t, s + 1)];
      const bool carries_coef = suffix ? (s == first) : (s == last);
      if (carries_coef) {
        acc(cin, cout, t.c, o);
      } else if (!once.count({cin, cout})) {
        once.insert({cin, cout});
        acc(cin, cout, 1.0, o);
      }
    }
  }
  *dims_out = dims;
  *wdims_out = wd;
  *pop_sites = es;
  (void)ctx;
  return TDMRG_OK;
}

}  // namespace tdmrg
