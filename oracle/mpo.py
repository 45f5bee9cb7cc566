"""The Hamiltonian as an MPO (paper eq. MPO), W[s][w, w', sigma, sigma'].

Construction: a finite-state machine whose channels on bond b (between chain
sites b-1 and b) are
  0: nothing applied yet,  1: a complete term already applied,
  2..: one channel per distinct *prefix* (the ordered local operators a
       multi-site term has applied on sites < b) of terms still unfinished.
Terms sharing a prefix share its channel; a term's coefficient is applied
with its last operator.  Bond 0 keeps only channel 0 and bond n only channel
1, so W[0] has shape (1, w1, d, d) and W[n-1] has shape (w_{n-1}, 1, d, d).
"""
import numpy as np

from .hamiltonian import local_matrix, site_dims, terms


def build_mpo(model):
    dims = site_dims(model)
    n = len(dims)
    term_list = [(c, dict(sorted(ops.items()))) for c, ops in terms(model)]

    # channel key -> index, per bond
    chan = [dict() for _ in range(n + 1)]
    START, DONE = ("start",), ("done",)

    def prefix(ops, b):
        return tuple((s, ops[s]) for s in ops if s < b)

    for b in range(n + 1):
        if b < n:
            chan[b][START] = len(chan[b])
        if b > 0:
            chan[b][DONE] = len(chan[b])
    for _, ops in term_list:
        sites = list(ops)
        if len(sites) < 2:
            continue
        for b in range(sites[0] + 1, sites[-1] + 1):
            key = prefix(ops, b)
            if key not in chan[b]:
                chan[b][key] = len(chan[b])

    W = []
    for s in range(n):
        d = dims[s]
        w = np.zeros((len(chan[s]), len(chan[s + 1]), d, d), dtype=complex)
        eye = np.eye(d, dtype=complex)
        if START in chan[s] and START in chan[s + 1]:
            w[chan[s][START], chan[s + 1][START]] = eye
        if DONE in chan[s] and DONE in chan[s + 1]:
            w[chan[s][DONE], chan[s + 1][DONE]] = eye
        set_once = set()
        for c, ops in term_list:
            sites = list(ops)
            first, last = sites[0], sites[-1]
            if s < first or s > last:
                continue
            op = local_matrix(model, s, ops[s]) if s in ops else eye
            if first == last:  # single-site term
                w[chan[s][START], chan[s + 1][DONE]] += c * op
                continue
            cin = chan[s][START] if s == first else chan[s][prefix(ops, s)]
            if s == last:
                w[cin, chan[s + 1][DONE]] += c * op
                continue
            cout = chan[s + 1][prefix(ops, s + 1)]
            if (cin, cout) not in set_once:  # shared channels: apply once
                set_once.add((cin, cout))
                w[cin, cout] += op
        W.append(w)
    return W


def mpo_bond_dims(W):
    return [W[0].shape[0]] + [w.shape[1] for w in W]


def mpo_to_dense(W):
    """Contract the MPO into a dense matrix (tiny systems only)."""
    acc = W[0][0]  # (w1, d, d)
    acc = np.transpose(acc, (1, 2, 0))  # (row, col, w)
    for w in W[1:]:
        # acc[R, C, a] * w[a, b, s, t] -> [R, s, C, t, b]
        acc = np.einsum("RCa,abst->RsCtb", acc, w)
        r, s, c, t, b = acc.shape
        acc = acc.reshape(r * s, c * t, b)
    assert acc.shape[2] == 1
    return acc[:, :, 0]
