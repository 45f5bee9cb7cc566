"""CPU-only checks of the C ABI: the library loads, exports every function
declared in include/tdmrg.h, validates arguments without a GPU, and its host
MPO construction contracts to the oracle's Hamiltonian."""
import ctypes
import os
import re

import numpy as np
import pytest

import paper_1908_10588_amd as T
import synth
from oracle import hamiltonian as ham
from oracle import mpo as ompo

HEADER = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include",
                      "tdmrg.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(tdmrg_[a-z0-9_]+)\s*\(", src)))


def test_header_and_binding_agree():
    assert _declared() == T.exported_symbols()


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(T.LIB_PATH)
    for name in _declared():
        assert hasattr(lib, name), name


def test_ctx_create_without_gpu_or_bad_args():
    L = T.lib()
    h = ctypes.c_void_p()
    assert L.tdmrg_ctx_create(0, None, None, 0, None) == 1  # EINVAL: out is NULL
    assert L.tdmrg_ctx_create(0, None, None, 4096, ctypes.byref(h)) == 1  # arena size without an arena
    st = L.tdmrg_ctx_create(0, None, None, 0, ctypes.byref(h))
    assert st in (0, 1, 3)  # OK on a GPU machine, EDEVICE without one
    if st == 0:
        L.tdmrg_ctx_destroy(h)
    else:
        assert L.tdmrg_last_error(None)


def test_null_handles_rejected():
    L = T.lib()
    assert L.tdmrg_heff2_apply(None, None, None, None, None, None, None, None, 0) == 1
    assert L.tdmrg_tdvp2_sweep(None, None, None, 0.5, 4, 0.0, None, None) == 1
    assert L.tdmrg_observables(None, None, None, None, None) == 1
    assert L.tdmrg_mps_bond_dims(None, None) == 1
    n = ctypes.c_long()
    assert L.tdmrg_wop_nnz(None, ctypes.byref(n)) == 1


def _host_mpo_status(model):
    m, keep = T._model_struct(model)
    n = ctypes.c_int()
    return T.lib().tdmrg_mpo_host_query(ctypes.byref(m), ctypes.byref(n), None, None)


def test_model_validation():
    good = synth.config1_model(0)
    assert _host_mpo_status(good) == 0
    bad = dict(good, E=np.array([np.nan, 0.3]))
    assert _host_mpo_status(bad) == 1
    bad = dict(good, nbasis=np.array([8, 1, 8, 8]))
    assert _host_mpo_status(bad) == 1
    bad = dict(good, order=np.array([-1, 0, 0, 2, 3]))
    assert _host_mpo_status(bad) == 1
    bad = dict(good, order=np.array([0, 1, 2, 3, 1]))
    assert _host_mpo_status(bad) == 1
    g1 = good["g1"].copy()
    g1[0, 0, 1] += 0.1
    assert _host_mpo_status(dict(good, g1=g1)) == 1
    bad = dict(good, g2_I=np.array([7]), g2_J=np.array([0]), g2_i=np.array([0]),
               g2_j=np.array([0]), g2_val=np.array([0.1]))
    assert _host_mpo_status(bad) == 1


def _tiny_models():
    out = []
    m1 = synth.config1_model(3)
    m1["nbasis"] = np.array([3, 2, 3, 2])
    out.append(m1)
    m2 = synth.config5_model(1)
    keep = [0, 1, 2, 3]
    sel = [k for k in range(len(m2["g2_I"])) if m2["g2_I"][k] in keep and m2["g2_J"][k] in keep]
    m2 = dict(m2, omega=m2["omega"][:4], nbasis=np.array([3, 2, 4, 2]), g1=m2["g1"][:4],
              g2_I=np.append(m2["g2_I"][sel], [2, 0]), g2_J=np.append(m2["g2_J"][sel], [3, 2]),
              g2_i=np.append(m2["g2_i"][sel], [0, 1]), g2_j=np.append(m2["g2_j"][sel], [1, 1]),
              g2_val=np.append(m2["g2_val"][sel], [0.013, -0.02]),
              order=np.array([2, 0, -1, 3, 1]))
    out.append(m2)
    m3 = synth.config3_model(2, ordering="B", modes_per_bath=1, nbasis=3)
    m3["g1"][0, 0, 2] = m3["g1"][0, 2, 0] = 0.04
    out.append(m3)
    m4 = synth.config3_model(4, ordering="A", modes_per_bath=2, nbasis=2)
    out.append(m4)
    return out


@pytest.mark.parametrize("k", range(4))
def test_library_mpo_equals_oracle_hamiltonian(k):
    """The library's finite-state MPO (a different construction from the
    oracle's) contracts to the same dense Hamiltonian."""
    model = _tiny_models()[k]
    W = T.mpo_host(model)
    assert W[0].shape[0] == 1 and W[-1].shape[1] == 1
    H = ompo.mpo_to_dense(W)
    ref = ham.dense_hamiltonian(model).toarray()
    assert np.abs(H - ref).max() < 1e-13


def test_library_mpo_channel_counts():
    """Electronic site first, linear couplings: 5 channels on inner bonds;
    the paper-style ordering of the 24-mode model keeps channels small."""
    W = T.mpo_host(synth.config1_model(0))
    assert [w.shape[1] for w in W[:-1]] == [5, 5, 5, 5]
    W2 = T.mpo_host(synth.config2_model(0))
    assert max(w.shape[1] for w in W2) <= 20
    W3 = T.mpo_host(synth.config3_model(0, ordering="B"))
    assert max(w.shape[1] for w in W3) <= 5


def _lvc4(order):
    """Two states, four modes: kappa on every mode for both states, lambda
    on one (the structure of the paper's 4-mode pyrazine model), one site per
    state in the given chain order (-1 / -2 = states 0 / 1)."""
    g1 = np.zeros((4, 2, 2))
    g1[:, 0, 0] = [0.04, -0.05, 0.09, 0.0]
    g1[:, 1, 1] = [-0.03, 0.06, -0.1, 0.0]
    g1[3, 0, 1] = g1[3, 1, 0] = 0.18
    m = dict(n_el=2, E=np.array([-0.4, 0.4]), V=np.zeros((2, 2)), omega=np.array([0.07, 0.12, 0.16, 0.11]),
             nbasis=np.array([3, 3, 3, 3]), g1=g1, g2_I=np.zeros(0, int), g2_J=np.zeros(0, int),
             g2_i=np.zeros(0, int), g2_j=np.zeros(0, int), g2_val=np.zeros(0),
             order=np.array([-1, 0, 1, 2, 3]), occ=np.array([1, 0, 0, 0, 0]))
    return synth.per_state_model(m, order=order)


@pytest.mark.parametrize("k,order", [(0, None), (1, [0, -1, 1, -2, 2, 3]), (1, [3, 2, -2, 1, 0, -1]),
                                     (2, None), (3, [-3, 0, -1, -2, 1, 2, 3, 4, 5])])
def test_library_per_state_mpo_equals_oracle_hamiltonian(k, order):
    """Per-state electronic sites: the library's MPO contracts to the oracle's
    dense Hamiltonian in occupation operators (all term kinds: energies,
    couplings between states, linear and second-order el-vib terms)."""
    model = synth.per_state_model(_tiny_models()[k], order=order)
    W = T.mpo_host(model)
    assert len(W) == len(model["order"])
    H = ompo.mpo_to_dense(W)
    ref = ham.dense_hamiltonian(model).toarray()
    assert np.abs(H - ref).max() < 1e-13


def test_per_state_order_validation():
    m = _lvc4(None)
    assert _host_mpo_status(m) == 0
    assert _host_mpo_status(dict(m, order=np.array([-1, -1, 0, 1, 2, 3]))) == 1   # state 1 missing
    assert _host_mpo_status(dict(m, order=np.array([-1, -3, 0, 1, 2, 3]))) == 1   # no state 2
    assert _host_mpo_status(dict(m, order=np.array([-1, 0, 1, 2, 3]))) == 1      # too short


def test_per_state_mpo_bond_dimensions():
    """MPO bond dimensions (m_MPO) of the 4-mode two-state model for three
    orderings, counted by hand from the construction (channels: start, done,
    and one per distinct prefix of an unfinished term).  States first (the
    default ordering of the paper's study): after state 0 the prefixes n_0,
    a_0^+, a_0 (5); after state 1 n_0, n_1, a_0^+ a_1, a_0 a_1^+ (6); before
    the last mode only the two hopping prefixes of its lambda term (4).  Modes
    around the states (the strongly coupled sites in the middle): 4 4 6 6 4.
    States at the two ends: the prefixes of state 0 stay open across the whole
    chain (up to 7).  The paper reports 4 for the default ordering with its
    construction, which also merges channels through n_0 + n_1 = 1 and the
    Hermitian pair."""
    bonds = {}
    for name, order in (("default", None), ("middle", [2, 0, -1, 3, -2, 1]), ("ends", [-1, 0, 1, 2, 3, -2])):
        W = T.mpo_host(_lvc4(order))
        bonds[name] = [w.shape[1] for w in W[:-1]]
    assert bonds == {"default": [5, 6, 6, 6, 4], "middle": [4, 4, 6, 6, 4], "ends": [5, 6, 7, 7, 7]}


def test_workspace_query_bounds():
    """tdmrg_workspace_query (host only): grows with D_max and the Krylov
    limit, covers at least the Krylov basis and the two-site tensor of the
    largest pair, and rejects invalid arguments."""
    import synth
    model = synth.config2_model(0)
    q = {(D, m): T.tdmrg_workspace_query(model, D, m) for D in (32, 64, 128) for m in (20, 40)}
    assert q[(32, 40)] < q[(64, 40)] < q[(128, 40)]
    assert q[(128, 20)] < q[(128, 40)]
    th = 128 * 30 * 30 * 128  # largest two-site tensor at D_max 128 (d = 30 x 30)
    assert q[(128, 40)] > 16 * th * (40 + 1)
    assert q[(128, 40)] < 16 * th * 100  # no runaway terms
    m, keep = T._model_struct(model)
    b = ctypes.c_size_t()
    L = T.lib()
    assert L.tdmrg_workspace_query(ctypes.byref(m), 0, 40, 0, ctypes.byref(b)) == 1
    assert L.tdmrg_workspace_query(ctypes.byref(m), 64, 65, 0, ctypes.byref(b)) == 1
    assert L.tdmrg_workspace_query(ctypes.byref(m), 64, 40, 7, ctypes.byref(b)) == 1
    assert L.tdmrg_workspace_query(None, 64, 40, 0, ctypes.byref(b)) == 1
