"""Local operators and the el-vib Hamiltonian (paper Section 2.2).

H = H_el + H_vib + H_el-vib with (eqs. Hel_2, Hvib_2, Helvib_2)
  H_el     = sum_i E_i |i><i| + sum_{i != j} V_ij |i><j|
  H_vib    = sum_I w_I (b_I^+ b_I + 1/2)          (zero-point energy kept)
  H_el-vib = sum_{I,i,j} g_ij^I q_I |i><j| + second-order terms
with q = (b^+ + b)/sqrt(2) in the truncated occupation basis |0>..|d-1>.

Readings of the paper fixed here:
* one electronic site of dimension n_el, or (model["el_sites"] ==
  "per_state") one site of dimension 2 per electronic state, as the paper's
  ordering study has it: |i><j| becomes a_i^+ a_j with hard-core occupation
  operators (the dynamics stays in the one-excitation sector, where the
  exchange sign of fermions never arises), |i><i| becomes n_i;
* the quadratic operator q_I^2 uses the exact matrix elements of q^2 in the
  truncated basis (not the square of the truncated q);
* second-order terms are given once per distinct monomial; an off-diagonal
  electronic part |i><j| (i != j) comes with its Hermitian conjugate.
"""
import numpy as np
import scipy.sparse as sp


def op_number(d):
    return np.diag(np.arange(d, dtype=float)).astype(complex)


def op_q(d):
    """q = (b^+ + b)/sqrt(2): <k|q|k+1> = <k+1|q|k> = sqrt((k+1)/2)."""
    q = np.zeros((d, d))
    for k in range(d - 1):
        q[k, k + 1] = q[k + 1, k] = np.sqrt((k + 1) / 2.0)
    return q.astype(complex)


def op_q2(d):
    """Exact truncated-basis matrix of q^2 = (b^+ b^+ + b b + 2 b^+ b + 1)/2:
    <k|q^2|k> = (2k+1)/2 and <k|q^2|k+2> = <k+2|q^2|k> = sqrt((k+1)(k+2))/2."""
    q2 = np.zeros((d, d))
    for k in range(d):
        q2[k, k] = (2 * k + 1) / 2.0
        if k + 2 < d:
            q2[k, k + 2] = q2[k + 2, k] = np.sqrt((k + 1) * (k + 2)) / 2.0
    return q2.astype(complex)


def op_el(n_el, i, j):
    """|i><j| + |j><i| for i != j, |i><i| for i == j."""
    m = np.zeros((n_el, n_el), dtype=complex)
    m[i, j] = 1.0
    m[j, i] = 1.0
    return m


def per_state(model):
    return model.get("el_sites", "single") == "per_state"


def el_site_of(model, i):
    """Chain site of electronic state i (per-state sites are coded -1 - i in
    the order; a single electronic site is coded -1)."""
    order = list(model["order"])
    return order.index(-1 - i) if per_state(model) else order.index(-1)


def site_dims(model):
    if per_state(model):
        return [2 if s < 0 else int(model["nbasis"][s]) for s in model["order"]]
    return [model["n_el"] if s < 0 else int(model["nbasis"][s]) for s in model["order"]]


def local_matrix(model, site, key):
    """Matrix of a local operator named by `key` on chain site `site`."""
    d = site_dims(model)[site]
    if key == "I":
        return np.eye(d, dtype=complex)
    if key == "n+":  # n + 1/2
        return op_number(d) + 0.5 * np.eye(d)
    if key == "n":
        return op_number(d)
    if key == "q":
        return op_q(d)
    if key == "q2":
        return op_q2(d)
    if isinstance(key, tuple) and key[0] == "el":
        return op_el(d, key[1], key[2])
    if isinstance(key, tuple) and key[0] == "hel":  # whole electronic Hamiltonian
        E, V = model["E"], model["V"]
        h = np.diag(np.asarray(E, dtype=complex))
        for i in range(d):
            for j in range(d):
                if i != j:
                    h[i, j] += V[i, j]
        return h
    if key == "cr":  # a^+ on a per-state site: |1><0|
        return np.array([[0, 0], [1, 0]], dtype=complex)
    if key == "an":  # a: |0><1|
        return np.array([[0, 1], [0, 0]], dtype=complex)
    if key == "occ":  # n = a^+ a
        return np.array([[0, 0], [0, 1]], dtype=complex)
    if isinstance(key, tuple) and key[0] == "proj":
        m = np.zeros((d, d), dtype=complex)
        m[key[1], key[1]] = 1.0
        return m
    raise KeyError(key)


def _terms_per_state(model):
    """H with one site per electronic state: |i><i| -> n_i and, for i != j,
    |i><j| + |j><i| -> a_i^+ a_j + a_j^+ a_i (two terms)."""
    order = list(model["order"])
    n_el = model["n_el"]
    es = [el_site_of(model, i) for i in range(n_el)]
    pos = {m: s for s, m in enumerate(order) if m >= 0}
    out = []

    def el_terms(i, j):
        """The electronic factor of |i><j| (+ h.c. for i != j) as a list of {site: op}."""
        if i == j:
            return [{es[i]: "occ"}]
        return [{es[i]: "cr", es[j]: "an"}, {es[i]: "an", es[j]: "cr"}]

    def add(c, el, rest):
        for e in el_terms(*el):
            ops = dict(e)
            ops.update(rest)
            out.append((c, ops))

    for i in range(n_el):
        add(float(model["E"][i]), (i, i), {})
    for i in range(n_el):
        for j in range(i + 1, n_el):
            if model["V"][i, j] != 0.0:
                add(float(model["V"][i, j]), (i, j), {})
    omega = model["omega"]
    for I in range(len(omega)):
        out.append((float(omega[I]), {pos[I]: "n+"}))
    for I in range(len(omega)):
        for i in range(n_el):
            for j in range(i, n_el):
                g = float(model["g1"][I, i, j])
                if g != 0.0:
                    add(g, (i, j), {pos[I]: "q"})
    for I, J, i, j, v in zip(model["g2_I"], model["g2_J"], model["g2_i"], model["g2_j"],
                             model["g2_val"]):
        if v == 0.0:
            continue
        i, j = min(int(i), int(j)), max(int(i), int(j))
        if I == J:
            add(float(v), (i, j), {pos[int(I)]: "q2"})
        else:
            add(float(v), (i, j), {pos[int(I)]: "q", pos[int(J)]: "q"})
    return out


def terms(model):
    """The Hamiltonian as a list of (coefficient, {chain site: op key}).

    Every term is a product of local operators on distinct sites."""
    if per_state(model):
        return _terms_per_state(model)
    order = list(model["order"])
    el = order.index(-1)
    pos = {m: s for s, m in enumerate(order) if m >= 0}
    out = [(1.0, {el: ("hel",)})]
    omega = model["omega"]
    for I in range(len(omega)):
        out.append((float(omega[I]), {pos[I]: "n+"}))
    g1 = model["g1"]
    n_el = model["n_el"]
    for I in range(len(omega)):
        for i in range(n_el):
            for j in range(i, n_el):
                g = float(g1[I, i, j])
                if g != 0.0:
                    out.append((g, {el: ("el", i, j), pos[I]: "q"}))
    for I, J, i, j, v in zip(model["g2_I"], model["g2_J"], model["g2_i"], model["g2_j"],
                             model["g2_val"]):
        if v == 0.0:
            continue
        i, j = min(i, j), max(i, j)
        if I == J:
            out.append((float(v), {el: ("el", int(i), int(j)), pos[int(I)]: "q2"}))
        else:
            out.append((float(v), {el: ("el", int(i), int(j)), pos[int(I)]: "q", pos[int(J)]: "q"}))
    return out


def dense_hamiltonian(model):
    """Sparse matrix of H in the full product basis, chain site 0 most
    significant (the index order of an MPS contracted left to right)."""
    dims = site_dims(model)
    n = len(dims)
    total = None
    for coef, ops in terms(model):
        factors = []
        for s in range(n):
            if s in ops:
                factors.append(sp.csr_matrix(local_matrix(model, s, ops[s])))
            else:
                factors.append(sp.identity(dims[s], dtype=complex, format="csr"))
        m = factors[0]
        for f in factors[1:]:
            m = sp.kron(m, f, format="csr")
        m = coef * m
        total = m if total is None else total + m
    return total.tocsr()
