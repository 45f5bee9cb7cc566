"""Pins of the oracle's Hamiltonian and MPO (paper Section 2.2, eq. MPO).

Everything here is checked against something other than the oracle's own
formulae: textbook operator identities built in a larger basis, matrix
elements written out state by state, and the dense Kronecker Hamiltonian.
"""
import itertools
import json
import os

import numpy as np
import pytest

from oracle import hamiltonian as ham
from oracle import mpo as mpom
from oracle.mps import full_rank_caps, mps_size, product_state
import synth

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")))


def _ladder(d):
    b = np.zeros((d, d))
    for k in range(1, d):
        b[k - 1, k] = np.sqrt(k)
    return b


@pytest.mark.parametrize("d", [2, 3, 6, 10])
def test_boson_operators_from_ladder(d):
    """q and q^2 equal (b + b^+)/sqrt2 and its square built in a basis two
    states larger and then truncated (exact truncated matrix elements)."""
    big = _ladder(d + 2)
    qbig = (big + big.T) / np.sqrt(2.0)
    assert np.allclose(ham.op_q(d), qbig[:d, :d], atol=1e-15)
    assert np.allclose(ham.op_q2(d), (qbig @ qbig)[:d, :d], atol=1e-14)
    assert np.allclose(ham.op_number(d), (big.T @ big)[:d, :d], atol=1e-15)


def test_q2_is_not_square_of_truncated_q():
    """The reading kept: q2 differs from (q_trunc)^2 in the last diagonal entry."""
    d = 6
    q = ham.op_q(d)
    assert abs((q @ q)[-1, -1] - 2.5) < 1e-14
    assert abs(ham.op_q2(d)[-1, -1] - 5.5) < 1e-14


def _elementwise_hamiltonian(model):
    """<n|H|n'> from the definitions, state by state (no Kronecker products)."""
    dims = ham.site_dims(model)
    order = list(model["order"])
    el = order.index(-1)
    basis = list(itertools.product(*[range(d) for d in dims]))
    index = {s: k for k, s in enumerate(basis)}
    H = np.zeros((len(basis), len(basis)), dtype=complex)

    def qel(n, m):  # <n|q|m>
        return np.sqrt(max(n, m) / 2.0) if abs(n - m) == 1 else 0.0

    def q2el(n, m):  # <n|q^2|m> = sum_k <n|q|k><k|q|m> over the untruncated basis
        return sum(qel(n, k) * qel(k, m) for k in range(max(n, m) + 2))

    pos = {mo: s for s, mo in enumerate(order) if mo >= 0}
    for a in basis:
        for b in basis:
            ia, ib = a[el], b[el]
            same_modes = all(a[s] == b[s] for s in range(len(dims)) if s != el)
            h = 0.0
            if same_modes:
                h += model["E"][ia] if ia == ib else model["V"][ia, ib]
                if ia == ib:
                    h += sum(model["omega"][I] * (a[pos[I]] + 0.5) for I in pos)
            for I in pos:
                s = pos[I]
                others = all(a[t] == b[t] for t in range(len(dims)) if t not in (el, s))
                if others:
                    h += model["g1"][I, ia, ib] * qel(a[s], b[s])
            for I, J, i, j, v in zip(model["g2_I"], model["g2_J"], model["g2_i"], model["g2_j"],
                                     model["g2_val"]):
                elfac = 1.0 if (ia, ib) in ((i, j), (j, i)) else 0.0
                if elfac == 0.0:
                    continue
                sI, sJ = pos[int(I)], pos[int(J)]
                rest = all(a[t] == b[t] for t in range(len(dims)) if t not in (el, sI, sJ))
                if not rest:
                    continue
                if I == J:
                    h += v * q2el(a[sI], b[sI])
                else:
                    h += v * qel(a[sI], b[sI]) * qel(a[sJ], b[sJ])
            H[index[a], index[b]] = h
    return H


def _tiny_models():
    m1 = synth.config1_model(3)
    m1["nbasis"] = np.array([3, 2, 3, 2])
    m2 = synth.config5_model(1)
    keep = [0, 1, 2, 3]
    sel = [k for k in range(len(m2["g2_I"])) if m2["g2_I"][k] in keep and m2["g2_J"][k] in keep]
    m2 = dict(m2, omega=m2["omega"][:4], nbasis=np.array([3, 2, 4, 2]), g1=m2["g1"][:4],
              g2_I=m2["g2_I"][sel], g2_J=m2["g2_J"][sel], g2_i=m2["g2_i"][sel],
              g2_j=m2["g2_j"][sel], g2_val=m2["g2_val"][sel], order=np.array([2, 0, -1, 3, 1]))
    # add one bilinear term straddling the electronic site and one on one side
    m2["g2_I"] = np.append(m2["g2_I"], [2, 0]); m2["g2_J"] = np.append(m2["g2_J"], [3, 2])
    m2["g2_i"] = np.append(m2["g2_i"], [0, 1]); m2["g2_j"] = np.append(m2["g2_j"], [1, 1])
    m2["g2_val"] = np.append(m2["g2_val"], [0.013, -0.02])
    m3 = synth.config3_model(2, ordering="B", modes_per_bath=1, nbasis=3)
    m3["g1"][0, 0, 2] = m3["g1"][0, 2, 0] = 0.04  # a non-local linear term
    return [m1, m2, m3]


@pytest.mark.parametrize("k", range(3))
def test_dense_hamiltonian_elementwise(k):
    model = _tiny_models()[k]
    H = ham.dense_hamiltonian(model).toarray()
    assert np.abs(H - H.conj().T).max() < 1e-15
    assert np.abs(H - _elementwise_hamiltonian(model)).max() < 1e-13


@pytest.mark.parametrize("k", range(3))
def test_mpo_contracts_to_dense_hamiltonian(k):
    model = _tiny_models()[k]
    W = mpom.build_mpo(model)
    dims = ham.site_dims(model)
    assert W[0].shape[0] == 1 and W[-1].shape[1] == 1
    for s, w in enumerate(W):
        assert w.shape[2] == w.shape[3] == dims[s]
    Hmpo = mpom.mpo_to_dense(W)
    assert np.abs(Hmpo - ham.dense_hamiltonian(model).toarray()).max() < 1e-13


def test_mpo_bond_dimension_linear_two_state():
    """Electronic site first, linear couplings only: channels {start, done,
    |1><1|, |2><2|, |1><2|+|2><1|} on every inner bond."""
    W = mpom.build_mpo(synth.config1_model(0))
    assert mpom.mpo_bond_dims(W) == [1, 5, 5, 5, 5, 1]


def test_paper_m_limit_and_mps_size():
    g = GOLD["pyrazine4_default_order"]
    assert max(full_rank_caps(g["local_dims"])) == g["m_limit"]
    psi = product_state(g["local_dims"], [0] * len(g["local_dims"]))
    assert mps_size(psi) == sum(g["local_dims"])


def test_time_units():
    g = GOLD["time_step"]
    assert abs(g["dt_au"] * synth.AU_TIME_FS - g["dt_fs_approx"]) < 0.005
