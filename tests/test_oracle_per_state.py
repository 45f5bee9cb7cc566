"""Pins of the per-state electronic sites (one chain site of dimension 2 per
electronic state, the representation of the paper's ordering study,
Section 3.1): the dense Hamiltonian written in occupation operators against
the single-site one it must equal on the one-excitation sector, the MPO
against that dense Hamiltonian, and 2TDVP at full rank against exact
propagation."""
import numpy as np
import pytest

from oracle import exact, tdvp
from oracle import hamiltonian as ham
from oracle import mpo as mpom
from oracle import mps as mpsm
from oracle import observables as obs
import synth


def _small(seed, nbasis=(3, 3, 3, 3)):
    m = synth.config1_model(seed)
    m["nbasis"] = np.array(nbasis)
    return m


def _sf(nbasis=3):
    """Three electronic states with inter-state couplings, linear and
    second-order couplings to two modes (all operator kinds present)."""
    m = synth.sf_table1_model(nbasis=nbasis)
    rng = np.random.default_rng(5)
    m["omega"] = np.array([0.1, 0.17])
    m["nbasis"] = np.array([nbasis, nbasis])
    g1 = np.zeros((2, 3, 3))
    for I in range(2):
        x = 0.05 * rng.standard_normal((3, 3))
        g1[I] = x + x.T
    m["g1"] = g1
    m.update(g2_I=np.array([0, 0]), g2_J=np.array([0, 1]), g2_i=np.array([0, 1]),
             g2_j=np.array([0, 2]), g2_val=np.array([0.004, -0.003]))
    m["order"] = np.array([0, -1, 1])
    m["occ"] = np.array([0, 0, 0])
    return m


@pytest.mark.parametrize("which", ["config1", "sf"])
def test_one_excitation_sector_equals_single_site_hamiltonian(which):
    """H restricted to states with exactly one occupied electronic site is the
    single-site H with |i> <-> the state whose site i is occupied."""
    single = _small(0) if which == "config1" else _sf()
    per = synth.per_state_model(single)
    Hs = ham.dense_hamiltonian(single).toarray()
    Hp = ham.dense_hamiltonian(per).toarray()
    n_el = single["n_el"]
    dims_p = ham.site_dims(per)
    mode_dims = [int(single["nbasis"][x]) for x in single["order"] if x >= 0]
    # index maps: single-site basis (el state i, mode occupations) -> per-state basis
    idx = []
    for i in range(n_el):
        for flat in range(int(np.prod(mode_dims))):
            occ_modes = np.unravel_index(flat, mode_dims)
            occ = []
            k = 0
            for x in per["order"]:
                if x < 0:
                    occ.append(1 if -1 - x == i else 0)
                else:
                    occ.append(occ_modes[[y for y in single["order"] if y >= 0].index(x)])
            idx.append(np.ravel_multi_index(occ, dims_p))
    # the single-site basis order: el site position in the chain decides the flattening
    order_s = list(single["order"])
    el = order_s.index(-1)
    dims_s = ham.site_dims(single)
    perm = []
    for i in range(n_el):
        for flat in range(int(np.prod(mode_dims))):
            occ_modes = list(np.unravel_index(flat, mode_dims))
            occ = occ_modes[:el] + [i] + occ_modes[el:]
            perm.append(np.ravel_multi_index(occ, dims_s))
    Hs_p = Hs[np.ix_(perm, perm)]
    sub = Hp[np.ix_(idx, idx)]
    assert np.abs(sub - Hs_p).max() < 1e-14
    # and the sector is invariant: no matrix element leaves it
    rest = np.setdiff1d(np.arange(Hp.shape[0]), idx)
    assert np.abs(Hp[np.ix_(rest, idx)]).max() == 0.0


@pytest.mark.parametrize("order", [None, [0, -1, 1, -2, 2, 3], [-2, 0, 1, 2, 3, -1]])
def test_mpo_equals_dense_hamiltonian(order):
    per = synth.per_state_model(_small(1), order=order)
    W = mpom.build_mpo(per)
    dense = ham.dense_hamiltonian(per).toarray()
    M = W[0]
    for w in W[1:]:
        M = np.einsum("awst,wbuv->absutv", M, w).reshape(M.shape[0], w.shape[1], M.shape[2] * w.shape[2],
                                                        M.shape[3] * w.shape[3])
    assert np.abs(M[0, 0] - dense).max() < 1e-13


def test_dynamics_match_the_single_site_representation():
    """Full-rank 2TDVP in the per-state chain reproduces exact propagation and
    the populations of the single-site chain."""
    single = _small(2)
    per = synth.per_state_model(single, order=[0, -1, 1, -2, 2, 3])
    psi0 = exact.product_vector(per)
    full = mpsm.from_dense_full_rank(psi0, ham.site_dims(per))
    st = tdvp.TDVP2(full, mpom.build_mpo(per), sv_mode=2)
    for _ in range(6):
        st.step(per["dt_fs"], 10 ** 6, 0.0)
    ref = exact.evolve(per, psi0, [6 * per["dt_fs"]])[0]
    assert np.linalg.norm(mpsm.to_dense(st.mps) - ref) < 1e-10
    p_single = exact.el_populations(single, exact.evolve(single, exact.product_vector(single),
                                                         [6 * per["dt_fs"]])[0])
    assert np.abs(obs.populations(per, st.mps) - p_single).max() < 1e-10
    assert abs(obs.populations(per, st.mps).sum() - 1.0) < 1e-12


@pytest.mark.parametrize("order", ["default", "optimized", "worst"])
def test_superposed_excitation_state(order):
    """The initial state of the ordering study: right-canonical and equal to
    sum_i c_i |e_i> (x) |vacuum> in the dense basis."""
    model = synth.lvc4_per_state_model(0, order)
    model["nbasis"] = np.array([3, 2, 2, 3])  # small enough to compare densely
    c = np.array([0.6, 0.8j])
    psi = synth.superposed_excitation_state(model, c)
    for a in psi[1:]:
        assert mpsm.right_orth_error(a) < 1e-15
    dims = ham.site_dims(model)
    ref = np.zeros(int(np.prod(dims)), dtype=complex)
    for i in range(2):
        occ = [0] * len(dims)
        occ[ham.el_site_of(model, i)] = 1
        ref[np.ravel_multi_index(occ, dims)] = c[i]
    assert np.abs(mpsm.to_dense(psi) - ref).max() < 1e-15
    assert max(mpsm.bond_dims(psi)) <= 2
