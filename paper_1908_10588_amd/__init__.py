"""Python binding of libtdmrg (include/tdmrg.h), the MI355X 2TDVP library.

The functions below carry the names of the C entry points and only marshal
arguments: every step of the computation runs in the library's HIP kernels.
Device tensors are torch tensors (float64, planar complex layout [2][...]) on
the context's GPU; host arrays are numpy.  Importing this module loads the
shared library and raises if it has not been built (there is no fallback).

Small wrappers (Ctx, Wop, MPO, MPS) own the opaque handles and free them.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libtdmrg.so")

HBAR_EV_FS = 0.6582119569
FP64, FP32, BF16X3, BF16X6 = 0, 1, 2, 3
STATUS = {0: "OK", 1: "EINVAL", 2: "ENOMEM", 3: "EDEVICE", 4: "ENOCONV", 5: "ESHAPE",
          6: "EUNSUPPORTED"}

c_int, c_double, c_void_p, c_long = ctypes.c_int, ctypes.c_double, ctypes.c_void_p, ctypes.c_long
P = ctypes.POINTER


class HeffShape(ctypes.Structure):
    _fields_ = [(n, c_int) for n in ("Dl", "d1", "d2", "Dr", "wl", "wc", "wr")]


class Model(ctypes.Structure):
    _fields_ = [("n_el", c_int), ("n_modes", c_int), ("E", P(c_double)), ("V", P(c_double)),
                ("omega", P(c_double)), ("nbasis", P(c_int)), ("g1", P(c_double)),
                ("n_g2", c_int), ("g2_I", P(c_int)), ("g2_J", P(c_int)), ("g2_i", P(c_int)),
                ("g2_j", P(c_int)), ("g2", P(c_double)), ("order", P(c_int)), ("el_per_state", c_int)]


class Opts(ctypes.Structure):
    _fields_ = [("precision", c_int), ("krylov_tol", c_double), ("krylov_max", c_int),
                ("sv_mode", c_int), ("tie_rel", c_double)]


class StepStats(ctypes.Structure):
    _fields_ = [("max_disc", c_double), ("sum_disc", c_double), ("max_krylov", c_int),
                ("total_krylov", c_int), ("not_converged", c_int), ("seconds", c_double * 4)]


class Profile(ctypes.Structure):
    _fields_ = [("ms", c_double * 4), ("flops", c_double * 4), ("bytes", c_double * 4),
                ("launches", c_long * 4)]


class GlobalStats(ctypes.Structure):
    _fields_ = [("vectors", c_int), ("max_intermediate_bond", c_int), ("sum_disc", c_double), ("seconds", c_double)]


class ModelGrad(ctypes.Structure):
    _fields_ = [("E", P(c_double)), ("V", P(c_double)), ("omega", P(c_double)), ("g1", P(c_double)),
                ("g2", P(c_double))]


class GradInfo(ctypes.Structure):
    _fields_ = [("pop", c_double), ("seconds_forward", c_double), ("seconds_total", c_double),
                ("mean_nodes", c_double)]


class Obs(ctypes.Structure):
    _fields_ = [("pops", P(c_double)), ("norm2", c_double), ("energy", c_double),
                ("c_re", c_double), ("c_im", c_double), ("mps_size", c_double)]


_SIGS = {
    "tdmrg_ctx_create": (c_int, [c_int, c_void_p, c_void_p, ctypes.c_size_t, P(c_void_p)]),
    "tdmrg_workspace_query": (c_int, [P(Model), c_int, c_int, c_int, P(ctypes.c_size_t)]),
    "tdmrg_ctx_destroy": (None, [c_void_p]),
    "tdmrg_last_error": (ctypes.c_char_p, [c_void_p]),
    "tdmrg_ctx_synchronize": (c_int, [c_void_p]),
    "tdmrg_ctx_workspace_bytes": (c_int, [c_void_p, P(ctypes.c_size_t)]),
    "tdmrg_ctx_set_profiling": (c_int, [c_void_p, c_int]),
    "tdmrg_ctx_get_profile": (c_int, [c_void_p, P(Profile)]),
    "tdmrg_mpo_build": (c_int, [c_void_p, P(Model), P(c_void_p)]),
    "tdmrg_mpo_destroy": (None, [c_void_p]),
    "tdmrg_mpo_host_query": (c_int, [P(Model), P(c_int), P(c_int), P(c_int)]),
    "tdmrg_mpo_host_site": (c_int, [P(Model), c_int, P(c_double)]),
    "tdmrg_mpo_info": (c_int, [c_void_p, P(c_int), P(c_int), P(c_int)]),
    "tdmrg_mpo_get_site": (c_int, [c_void_p, c_int, P(c_double)]),
    "tdmrg_mpo_site": (c_void_p, [c_void_p, c_int]),
    "tdmrg_wop_create": (c_int, [c_void_p, c_int, c_int, c_int, P(c_double), P(c_void_p)]),
    "tdmrg_wop_destroy": (None, [c_void_p]),
    "tdmrg_wop_nnz": (c_int, [c_void_p, P(c_long)]),
    "tdmrg_mps_init": (c_int, [c_void_p, c_void_p, P(c_int), c_int, P(c_void_p)]),
    "tdmrg_mps_copy": (c_int, [c_void_p, P(c_void_p)]),
    "tdmrg_mps_destroy": (None, [c_void_p]),
    "tdmrg_mps_bond_dims": (c_int, [c_void_p, P(c_int)]),
    "tdmrg_mps_set_site": (c_int, [c_void_p, c_int, c_int, c_int, P(c_double)]),
    "tdmrg_mps_get_site": (c_int, [c_void_p, c_int, P(c_int), P(c_int), P(c_int), P(c_double)]),
    "tdmrg_heff2_apply": (c_int, [c_void_p, P(HeffShape), c_void_p, c_void_p, c_void_p, c_void_p,
                                  c_void_p, c_void_p, c_int]),
    "tdmrg_heff2_apply_noalloc": (c_int, [c_void_p, P(HeffShape), c_void_p, c_void_p, c_void_p, c_void_p,
                                          c_void_p, c_void_p, c_int]),
    "tdmrg_heff1_apply": (c_int, [c_void_p, P(HeffShape), c_void_p, c_void_p, c_void_p, c_void_p,
                                  c_void_p, c_int]),
    "tdmrg_local_expm": (c_int, [c_void_p, P(HeffShape), c_int, c_void_p, c_void_p, c_void_p,
                                 c_void_p, c_void_p, c_double, c_double, c_int, c_int, P(c_int)]),
    "tdmrg_heff2_apply_batched": (c_int, [c_void_p, c_int, P(HeffShape), P(c_void_p), P(c_void_p),
                                          P(c_void_p), P(c_void_p), P(c_void_p), P(c_void_p),
                                          c_int]),
    "tdmrg_local_expm_batched": (c_int, [c_void_p, c_int, P(HeffShape), P(c_void_p), P(c_void_p),
                                         P(c_void_p), P(c_void_p), P(c_void_p), c_double, c_double,
                                         c_int, c_int, P(c_int)]),
    "tdmrg_ctx_set_batch_budget": (c_int, [c_void_p, ctypes.c_size_t]),
    "tdmrg_ctx_set_fusion": (c_int, [c_void_p, c_int]),
    "tdmrg_ctx_set_mpo_apply": (c_int, [c_void_p, c_int]),
    "tdmrg_ctx_set_mix_in_gemm": (c_int, [c_void_p, c_int]),
    "tdmrg_ctx_set_svd_method": (c_int, [c_void_p, c_int]),
    "tdmrg_ctx_set_svd_schedule": (c_int, [c_void_p, c_int]),
    "tdmrg_ctx_set_eigensolver": (c_int, [c_void_p, c_int]),
    "tdmrg_tdvp2_population_grad": (c_int, [c_void_p, P(Model), P(c_int), c_int, c_int, c_double, c_int, c_double,
                                            P(Opts), c_int, c_int, P(ModelGrad), P(c_int), P(GradInfo)]),
    "tdmrg_ctx_set_channel_gemm": (c_int, [c_void_p, c_int]),
    "tdmrg_ctx_set_autotune": (c_int, [c_void_p, c_int]),
    "tdmrg_ctx_set_verbose": (c_int, [c_void_p, c_int]),
    "tdmrg_ctx_set_graphs": (c_int, [c_void_p, c_int]),
    "tdmrg_ctx_graph_counters": (c_int, [c_void_p, P(ctypes.c_long)]),
    "tdmrg_ctx_tile_table": (c_int, [c_void_p, c_int, P(c_int), P(c_int)]),
    "tdmrg_ctx_svd_counters": (c_int, [c_void_p, c_void_p]),
    "tdmrg_heff2_apply_vjp": (c_int, [c_void_p, P(HeffShape)] + [c_void_p] * 11),
    "tdmrg_local_expm_vjp": (c_int, [c_void_p, P(HeffShape), c_void_p, c_void_p, c_void_p, c_void_p,
                                     c_void_p, c_double, c_void_p, c_void_p, c_void_p, c_void_p,
                                     c_void_p, c_void_p, c_int, c_double, c_int]),
    "tdmrg_theta_form": (c_int, [c_void_p, c_int, c_int, c_int, c_int, c_int, c_void_p, c_void_p,
                                 c_void_p]),
    "tdmrg_svd_truncate": (c_int, [c_void_p, c_int, c_int, c_int, c_int, c_void_p, c_double, c_int,
                                   c_int, c_double, c_int, c_void_p, c_void_p, c_void_p, P(c_int),
                                   P(c_double)]),
    "tdmrg_env_update_left": (c_int, [c_void_p, c_int, c_int, c_int, c_void_p, c_void_p, c_void_p,
                                      c_void_p, c_int]),
    "tdmrg_env_update_right": (c_int, [c_void_p, c_int, c_int, c_int, c_void_p, c_void_p, c_void_p,
                                       c_void_p, c_int]),
    "tdmrg_tdvp2_sweep": (c_int, [c_void_p, c_void_p, c_void_p, c_double, c_int, c_double, P(Opts),
                                  P(StepStats)]),
    "tdmrg_observables": (c_int, [c_void_p, c_void_p, c_void_p, c_void_p, P(Obs)]),
    "tdmrg_heff0_apply": (c_int, [c_void_p, c_int, c_int, c_int, c_void_p, c_void_p, c_void_p, c_void_p,
                                  c_int]),
    "tdmrg_local_expm0": (c_int, [c_void_p, c_int, c_int, c_int, c_void_p, c_void_p, c_void_p, c_double,
                                  c_double, c_int, c_int, P(c_int)]),
    "tdmrg_qr_split": (c_int, [c_void_p, c_int, c_int, c_void_p, c_int, c_void_p, c_void_p, P(c_int)]),
    "tdmrg_tdvp1_sweep": (c_int, [c_void_p, c_void_p, c_void_p, c_double, P(Opts), P(StepStats)]),
    "tdmrg_global_step": (c_int, [c_void_p, c_void_p, c_void_p, c_double, c_int, c_int, c_double, c_int, c_double,
                                  P(GlobalStats)]),
    "tdmrg_spectrum": (c_int, [c_void_p, c_int, c_double, c_void_p, c_double, c_int, c_void_p, c_void_p]),
}

_lib = None


def lib():
    """The loaded libtdmrg.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_1908_10588_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def exported_symbols():
    return sorted(_SIGS)


class TdmrgError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


def _check(st, ctx=None, allow=()):
    if st != 0 and st not in allow:
        msg = lib().tdmrg_last_error(ctx)
        raise TdmrgError(st, msg.decode() if msg else "")
    return st


def _dptr(t):
    """Device pointer of a torch tensor (float64, contiguous, on the GPU)."""
    import torch
    if not isinstance(t, torch.Tensor) or t.dtype != torch.float64 or not t.is_cuda or \
            not t.is_contiguous():
        raise TypeError("expected a contiguous float64 CUDA tensor")
    return ctypes.c_void_p(t.data_ptr())


def to_planar(x):
    x = np.asarray(x)
    return np.ascontiguousarray(np.stack([x.real, x.imag]).astype(np.float64))


def from_planar(p):
    p = np.asarray(p)
    return p[0] + 1j * p[1]


def to_device(x, device="cuda"):
    import torch
    return torch.from_numpy(to_planar(x)).to(device)


def from_device(t):
    return from_planar(t.detach().cpu().numpy())


# ------------------------------------------------------------------ wrappers
class Ctx:
    """A library context on one GPU.  arena: optional caller-owned device
    buffer (a torch tensor on that GPU, e.g. torch.empty(n, dtype=torch.uint8))
    that every workspace buffer is carved from; it is kept alive with the
    context (see tdmrg_ctx_create and tdmrg_workspace_query)."""

    def __init__(self, device=0, stream=None, arena=None):
        import torch
        if stream is None:
            stream = torch.cuda.current_stream(device).cuda_stream
        h = c_void_p()
        ptr, nbytes = None, 0
        if arena is not None:
            if not isinstance(arena, torch.Tensor) or not arena.is_cuda or not arena.is_contiguous():
                raise TypeError("arena must be a contiguous CUDA tensor")
            ptr, nbytes = c_void_p(arena.data_ptr()), arena.numel() * arena.element_size()
        _check(lib().tdmrg_ctx_create(device, c_void_p(stream), ptr, ctypes.c_size_t(nbytes), ctypes.byref(h)))
        self.h = h
        self.device = device
        self.arena = arena

    def close(self):
        if self.h:
            lib().tdmrg_ctx_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def check(self, st, allow=()):
        return _check(st, self.h, allow)

    def synchronize(self):
        self.check(lib().tdmrg_ctx_synchronize(self.h))

    def workspace_bytes(self):
        b = ctypes.c_size_t()
        self.check(lib().tdmrg_ctx_workspace_bytes(self.h, ctypes.byref(b)))
        return b.value

    def set_profiling(self, on):
        self.check(lib().tdmrg_ctx_set_profiling(self.h, int(bool(on))))

    def profile(self):
        p = Profile()
        self.check(lib().tdmrg_ctx_get_profile(self.h, ctypes.byref(p)))
        return dict(ms=list(p.ms), flops=list(p.flops), bytes=list(p.bytes),
                    launches=list(p.launches))

    def set_channel_gemm(self, mode):
        """0 never, 1 cost model (default), 2 always (see tdmrg_ctx_set_channel_gemm)."""
        self.check(lib().tdmrg_ctx_set_channel_gemm(self.h, int(mode)))

    def set_autotune(self, on):
        self.check(lib().tdmrg_ctx_set_autotune(self.h, int(bool(on))))

    def set_mix_in_gemm(self, on):
        """Fused channel stage inside the last GEMM's A loader (default off)."""
        self.check(lib().tdmrg_ctx_set_mix_in_gemm(self.h, int(bool(on))))

    def set_mpo_apply(self, mode):
        """Global steps: 0 direct MPO x MPS product + compression, 1 variational fit."""
        self.check(lib().tdmrg_ctx_set_mpo_apply(self.h, int(mode)))

    def set_graphs(self, on):
        """Lanczos step graphs on/off (see tdmrg_ctx_set_graphs)."""
        self.check(lib().tdmrg_ctx_set_graphs(self.h, int(bool(on))))

    def graph_counters(self):
        """{'captured', 'replayed', 'eager'} Lanczos step counts (tdmrg_ctx_graph_counters)."""
        out = (ctypes.c_long * 3)()
        self.check(lib().tdmrg_ctx_graph_counters(self.h, out))
        return dict(zip(("captured", "replayed", "eager"), list(out)))

    def set_verbose(self, level):
        """Progress lines on stderr from long calls (see tdmrg_ctx_set_verbose)."""
        self.check(lib().tdmrg_ctx_set_verbose(self.h, int(level)))

    def tile_table(self):
        """Tuned GEMM tile variant per shape class (see tdmrg_ctx_tile_table)."""
        n = c_int()
        self.check(lib().tdmrg_ctx_tile_table(self.h, 0, ctypes.byref(n), None))
        rows = (c_int * (9 * max(n.value, 1)))()
        self.check(lib().tdmrg_ctx_tile_table(self.h, n.value, ctypes.byref(n), rows))
        keys = ("trans_a", "trans_b", "precision", "log2_M", "log2_N", "log2_K", "log2_batch", "mix_a", "variant")
        return [dict(zip(keys, list(rows)[9 * r:9 * r + 9])) for r in range(n.value)]

    SVD_METHODS = {"auto": 0, "jacobi": 1, "gram": 2, "subspace": 3}

    def set_svd_method(self, method):
        """'auto', 'jacobi', 'gram' or 'subspace' (see tdmrg_ctx_set_svd_method)."""
        self.check(lib().tdmrg_ctx_set_svd_method(self.h, self.SVD_METHODS[method]))

    def set_svd_schedule(self, schedule):
        """First Rayleigh-Ritz check of the subspace SVD: 0 adaptive, 1 at the
        first iteration (see tdmrg_ctx_set_svd_schedule)."""
        self.check(lib().tdmrg_ctx_set_svd_schedule(self.h, int(schedule)))

    EIGENSOLVERS = {"reduction": 0, "zheevd": 1}

    def set_eigensolver(self, method):
        """'reduction' (Householder reduction in one workgroup + tridiagonal
        divide and conquer, n <= 240) or 'zheevd' (see tdmrg_ctx_set_eigensolver)."""
        self.check(lib().tdmrg_ctx_set_eigensolver(self.h, self.EIGENSOLVERS[method]))

    def svd_counters(self):
        out = (ctypes.c_longlong * 8)()
        self.check(lib().tdmrg_ctx_svd_counters(self.h, out))
        keys = ("jacobi", "gram", "subspace", "subspace_iters", "subspace_unsettled", "subspace_factor_fail",
                "subspace_rr_checks", "one_site_split_svd")
        return dict(zip(keys, list(out)))


class Wop:
    """An MPO site tensor W[wl][wr][d][d] (complex numpy) on the device."""

    def __init__(self, ctx, W, _handle=None, _owner=None):
        self.ctx = ctx
        if _handle is not None:
            self.h, self._owner = _handle, _owner
            return
        wl, wr, d, d2 = W.shape
        assert d == d2
        pl = to_planar(W)
        h = c_void_p()
        ctx.check(lib().tdmrg_wop_create(ctx.h, wl, wr, d,
                                         pl.ctypes.data_as(P(c_double)), ctypes.byref(h)))
        self.h, self._owner = h, None

    def nnz(self):
        n = c_long()
        self.ctx.check(lib().tdmrg_wop_nnz(self.h, ctypes.byref(n)))
        return n.value

    def __del__(self):
        if getattr(self, "_owner", 1) is None and getattr(self, "h", None):
            lib().tdmrg_wop_destroy(self.h)
            self.h = None


def _model_struct(model):
    keep = {}

    def arr(name, x, dt):
        a = np.ascontiguousarray(np.asarray(x, dtype=dt))
        keep[name] = a
        return a.ctypes.data_as(P(c_double if dt == np.float64 else c_int))

    n_el = int(model["n_el"])
    n_modes = len(model["omega"])
    m = Model()
    m.n_el, m.n_modes = n_el, n_modes
    m.E = arr("E", model["E"], np.float64)
    m.V = arr("V", np.asarray(model["V"]).reshape(-1), np.float64)
    m.omega = arr("omega", model["omega"], np.float64)
    m.nbasis = arr("nbasis", model["nbasis"], np.int32)
    m.g1 = arr("g1", np.asarray(model["g1"]).reshape(-1), np.float64)
    m.n_g2 = len(model["g2_val"])
    m.g2_I = arr("g2_I", model["g2_I"], np.int32)
    m.g2_J = arr("g2_J", model["g2_J"], np.int32)
    m.g2_i = arr("g2_i", model["g2_i"], np.int32)
    m.g2_j = arr("g2_j", model["g2_j"], np.int32)
    m.g2 = arr("g2", model["g2_val"], np.float64)
    m.order = arr("order", model["order"], np.int32)
    m.el_per_state = 1 if model.get("el_sites", "single") == "per_state" else 0
    return m, keep


def tdmrg_workspace_query(model, D_max, krylov_max=40, precision=FP64):
    """Bytes of workspace arena a 2TDVP sweep of this model needs at D_max
    (host only)."""
    m, keep = _model_struct(model)
    b = ctypes.c_size_t()
    _check(lib().tdmrg_workspace_query(ctypes.byref(m), int(D_max), int(krylov_max), int(precision),
                                       ctypes.byref(b)))
    return b.value


def mpo_host(model):
    """The library's MPO built on the host only: list of complex W[s]."""
    m, keep = _model_struct(model)
    n = c_int()
    _check(lib().tdmrg_mpo_host_query(ctypes.byref(m), ctypes.byref(n), None, None))
    dims = (c_int * n.value)()
    wd = (c_int * (n.value + 1))()
    _check(lib().tdmrg_mpo_host_query(ctypes.byref(m), None, dims, wd))
    out = []
    for s in range(n.value):
        buf = np.zeros((2, wd[s], wd[s + 1], dims[s], dims[s]))
        _check(lib().tdmrg_mpo_host_site(ctypes.byref(m), s, buf.ctypes.data_as(P(c_double))))
        out.append(from_planar(buf))
    return out


class MPO:
    def __init__(self, ctx, model):
        self.ctx = ctx
        m, keep = _model_struct(model)
        h = c_void_p()
        ctx.check(lib().tdmrg_mpo_build(ctx.h, ctypes.byref(m), ctypes.byref(h)))
        self.h = h
        n = c_int()
        lib().tdmrg_mpo_info(self.h, ctypes.byref(n), None, None)
        self.n = n.value
        dims = (c_int * self.n)()
        wd = (c_int * (self.n + 1))()
        lib().tdmrg_mpo_info(self.h, None, dims, wd)
        self.dims, self.wdims = list(dims), list(wd)
        self.n_el = int(model["n_el"])

    def site_tensor(self, s):
        out = np.zeros((2, self.wdims[s], self.wdims[s + 1], self.dims[s], self.dims[s]))
        self.ctx.check(lib().tdmrg_mpo_get_site(self.h, s, out.ctypes.data_as(P(c_double))))
        return from_planar(out)

    def wop(self, s):
        return Wop(self.ctx, None, _handle=c_void_p(lib().tdmrg_mpo_site(self.h, s)), _owner=self)

    def __del__(self):
        if getattr(self, "h", None):
            lib().tdmrg_mpo_destroy(self.h)
            self.h = None


class MPS:
    def __init__(self, ctx, mpo=None, occ=None, D_cap=None, _handle=None, _n=None):
        self.ctx = ctx
        if _handle is not None:
            self.h, self.n = _handle, _n
            return
        o = np.ascontiguousarray(np.asarray(occ, dtype=np.int32))
        h = c_void_p()
        ctx.check(lib().tdmrg_mps_init(ctx.h, mpo.h, o.ctypes.data_as(P(c_int)), int(D_cap),
                                       ctypes.byref(h)))
        self.h, self.n = h, mpo.n

    def copy(self):
        h = c_void_p()
        self.ctx.check(lib().tdmrg_mps_copy(self.h, ctypes.byref(h)))
        return MPS(self.ctx, _handle=h, _n=self.n)

    def bond_dims(self):
        b = (c_int * (self.n + 1))()
        self.ctx.check(lib().tdmrg_mps_bond_dims(self.h, b))
        return list(b)

    def get_site(self, s):
        Dl, d, Dr = c_int(), c_int(), c_int()
        self.ctx.check(lib().tdmrg_mps_get_site(self.h, s, ctypes.byref(Dl), ctypes.byref(d),
                                                ctypes.byref(Dr), None))
        out = np.zeros((2, Dl.value, d.value, Dr.value))
        self.ctx.check(lib().tdmrg_mps_get_site(self.h, s, None, None, None,
                                                out.ctypes.data_as(P(c_double))))
        return from_planar(out)

    def set_site(self, s, A):
        pl = to_planar(A)
        self.ctx.check(lib().tdmrg_mps_set_site(self.h, s, A.shape[0], A.shape[2],
                                                pl.ctypes.data_as(P(c_double))))

    def tensors(self):
        return [self.get_site(s) for s in range(self.n)]

    def __del__(self):
        if getattr(self, "h", None):
            lib().tdmrg_mps_destroy(self.h)
            self.h = None


def tdmrg_tdvp2_sweep(ctx, mps, mpo, dt_fs, D_max, eps, precision=FP64, krylov_tol=1e-12,
                      krylov_max=40, sv_mode=0, tie_rel=1e-12):
    o = Opts(precision, krylov_tol, krylov_max, sv_mode, tie_rel)
    st = StepStats()
    ctx.check(lib().tdmrg_tdvp2_sweep(ctx.h, mps.h, mpo.h, float(dt_fs), int(D_max), float(eps),
                                      ctypes.byref(o), ctypes.byref(st)), allow=(4,))
    return st


def tdmrg_tdvp1_sweep(ctx, mps, mpo, dt_fs, precision=FP64, krylov_tol=1e-12, krylov_max=40):
    o = Opts(precision, krylov_tol, krylov_max, 0, 1e-12)
    st = StepStats()
    ctx.check(lib().tdmrg_tdvp1_sweep(ctx.h, mps.h, mpo.h, float(dt_fs), ctypes.byref(o), ctypes.byref(st)),
              allow=(4,))
    return st


def tdmrg_global_step(ctx, mps, mpo, dt_fs, D_max, eps, method="krylov", m_max=16, tol=1e-10):
    """One global time step (method "krylov", "rk4" or "taylor", whose order
    is m_max); returns the stats."""
    st = GlobalStats()
    ctx.check(lib().tdmrg_global_step(ctx.h, mps.h, mpo.h, float(dt_fs), {"krylov": 0, "rk4": 1, "taylor": 2}[method],
                                      int(m_max), float(tol), int(D_max), float(eps), ctypes.byref(st)))
    return st


def tdmrg_spectrum(ctx, C, dt_fs, E, tau_fs, sigma):
    """C: planar [2][n_t] device tensor; E, sigma: [n_E] device tensors."""
    ctx.check(lib().tdmrg_spectrum(ctx.h, int(C.shape[-1]), float(dt_fs), _dptr(C), float(tau_fs), int(E.numel()),
                                   _dptr(E), _dptr(sigma)))


def tdmrg_heff0_apply(ctx, Dl, Dr, w, L, R, C, y, precision=FP64):
    ctx.check(lib().tdmrg_heff0_apply(ctx.h, int(Dl), int(Dr), int(w), _dptr(L), _dptr(R), _dptr(C), _dptr(y),
                                      precision))


def tdmrg_local_expm0(ctx, Dl, Dr, w, L, R, C, tau, tol=1e-13, m_max=40, precision=FP64):
    it = c_int()
    st = ctx.check(lib().tdmrg_local_expm0(ctx.h, int(Dl), int(Dr), int(w), _dptr(L), _dptr(R), _dptr(C),
                                           float(tau), float(tol), int(m_max), precision, ctypes.byref(it)),
                   allow=(4,))
    return it.value, st == 0


def tdmrg_qr_split(ctx, rows, cols, M, right, Q, C):
    """Returns 1 when the Cholesky QR passes held, 0 when the SVD route was taken."""
    ok = c_int()
    ctx.check(lib().tdmrg_qr_split(ctx.h, int(rows), int(cols), _dptr(M), int(bool(right)), _dptr(Q), _dptr(C),
                                   ctypes.byref(ok)))
    return ok.value


def tdmrg_tdvp2_population_grad(ctx, model, occ, D_cap, steps, dt_fs, D_max, eps, state, nquad=12,
                                krylov_tol=1e-12, krylov_max=40, sv_mode=0, tie_rel=1e-12):
    """Gradient of P_state after `steps` 2TDVP steps with respect to the model's
    constants (see tdmrg_tdvp2_population_grad).  Returns a dict with pop,
    E, V, omega, g1, g2 (gradients shaped like the model's arrays), ranks
    [steps][2][n_sites-1] and the timings."""
    m, keep = _model_struct(model)
    n_el, n_modes, n_g2 = int(model["n_el"]), len(model["omega"]), len(model["g2_val"])
    out = {"E": np.zeros(n_el), "V": np.zeros((n_el, n_el)), "omega": np.zeros(n_modes),
           "g1": np.zeros((n_modes, n_el, n_el)), "g2": np.zeros(max(n_g2, 1))}
    g = ModelGrad(*[out[k].ctypes.data_as(P(c_double)) for k in ("E", "V", "omega", "g1", "g2")])
    occ_a = np.ascontiguousarray(np.asarray(occ, dtype=np.int32))
    ranks = np.zeros((steps, 2, n_modes), dtype=np.int32)  # n_sites - 1 = n_modes
    o = Opts(FP64, krylov_tol, krylov_max, sv_mode, tie_rel)
    info = GradInfo()
    ctx.check(lib().tdmrg_tdvp2_population_grad(
        ctx.h, ctypes.byref(m), occ_a.ctypes.data_as(P(c_int)), int(D_cap), int(steps), float(dt_fs), int(D_max),
        float(eps), ctypes.byref(o), int(state), int(nquad), ctypes.byref(g), ranks.ctypes.data_as(P(c_int)),
        ctypes.byref(info)))
    out["g2"] = out["g2"][:n_g2]
    out.update(pop=info.pop, ranks=ranks, seconds_forward=info.seconds_forward, seconds_total=info.seconds_total,
               mean_nodes=info.mean_nodes)
    return out


def tdmrg_observables(ctx, mps, mpo, psi0=None):
    pops = np.zeros(mpo.n_el)
    ob = Obs()
    ob.pops = pops.ctypes.data_as(P(c_double))
    ctx.check(lib().tdmrg_observables(ctx.h, mps.h, mpo.h, psi0.h if psi0 is not None else None,
                                      ctypes.byref(ob)))
    return dict(pops=pops, norm2=ob.norm2, energy=ob.energy, C=complex(ob.c_re, ob.c_im),
                mps_size=ob.mps_size)


def tdmrg_heff2_apply(ctx, shape, L, W1, W2, R, theta, y, precision=FP64):
    s = HeffShape(*shape)
    ctx.check(lib().tdmrg_heff2_apply(ctx.h, ctypes.byref(s), _dptr(L), W1.h, W2.h, _dptr(R),
                                      _dptr(theta), _dptr(y), precision))


def tdmrg_heff2_apply_noalloc(ctx, shape, L, W1, W2, R, theta, y, precision=FP64):
    """tdmrg_heff2_apply with its intermediates in the library's fixed device
    scratch array (nothing allocated)."""
    s = HeffShape(*shape)
    ctx.check(lib().tdmrg_heff2_apply_noalloc(ctx.h, ctypes.byref(s), _dptr(L), W1.h, W2.h, _dptr(R),
                                              _dptr(theta), _dptr(y), precision))


def tdmrg_heff1_apply(ctx, shape, L, W, R, M, y, precision=FP64):
    s = HeffShape(*shape)
    ctx.check(lib().tdmrg_heff1_apply(ctx.h, ctypes.byref(s), _dptr(L), W.h, _dptr(R), _dptr(M),
                                      _dptr(y), precision))


def tdmrg_local_expm(ctx, shape, two_site, L, W1, W2, R, theta, tau, tol=1e-13, m_max=40,
                     precision=FP64):
    s = HeffShape(*shape)
    it = c_int()
    st = ctx.check(lib().tdmrg_local_expm(ctx.h, ctypes.byref(s), int(two_site), _dptr(L), W1.h,
                                          W2.h if W2 is not None else None, _dptr(R),
                                          _dptr(theta), float(tau), float(tol), int(m_max),
                                          precision, ctypes.byref(it)), allow=(4,))
    return it.value, st == 0


def _ptrs(items, f):
    arr = (c_void_p * max(len(items), 1))()
    for k, x in enumerate(items):
        arr[k] = f(x)
    return arr


def tdmrg_heff2_apply_batched(ctx, shapes, Ls, W1s, W2s, Rs, thetas, ys, precision=FP64):
    n = len(shapes)
    sh = (HeffShape * max(n, 1))(*[HeffShape(*s) for s in shapes])
    dp = lambda t: _dptr(t).value
    ctx.check(lib().tdmrg_heff2_apply_batched(
        ctx.h, n, sh, _ptrs(Ls, dp), _ptrs(W1s, lambda w: w.h.value), _ptrs(W2s, lambda w: w.h.value),
        _ptrs(Rs, dp), _ptrs(thetas, dp), _ptrs(ys, dp), precision))


def tdmrg_local_expm_batched(ctx, shapes, Ls, W1s, W2s, Rs, thetas, tau, tol=1e-13, m_max=40,
                             precision=FP64):
    n = len(shapes)
    sh = (HeffShape * max(n, 1))(*[HeffShape(*s) for s in shapes])
    dp = lambda t: _dptr(t).value
    its = (c_int * max(n, 1))()
    st = ctx.check(lib().tdmrg_local_expm_batched(
        ctx.h, n, sh, _ptrs(Ls, dp), _ptrs(W1s, lambda w: w.h.value), _ptrs(W2s, lambda w: w.h.value),
        _ptrs(Rs, dp), _ptrs(thetas, dp), float(tau), float(tol), int(m_max), precision, its),
        allow=(4,))
    return list(its)[:n], st == 0


def _optr(t):
    return None if t is None else _dptr(t)


def tdmrg_heff2_apply_vjp(ctx, shape, L, W1, W2, R, theta, ybar, Lbar=None, W1bar=None,
                          W2bar=None, Rbar=None, thetabar=None):
    s = HeffShape(*shape)
    ctx.check(lib().tdmrg_heff2_apply_vjp(ctx.h, ctypes.byref(s), _dptr(L), W1.h, W2.h, _dptr(R),
                                          _dptr(theta), _dptr(ybar), _optr(Lbar), _optr(W1bar),
                                          _optr(W2bar), _optr(Rbar), _optr(thetabar)))


def tdmrg_local_expm_vjp(ctx, shape, L, W1, W2, R, theta_in, tau, ybar, Lbar=None, W1bar=None,
                         W2bar=None, Rbar=None, thetabar=None, nquad=8, tol=1e-13, m_max=40):
    s = HeffShape(*shape)
    ctx.check(lib().tdmrg_local_expm_vjp(ctx.h, ctypes.byref(s), _dptr(L), W1.h, W2.h, _dptr(R),
                                         _dptr(theta_in), float(tau), _dptr(ybar), _optr(Lbar),
                                         _optr(W1bar), _optr(W2bar), _optr(Rbar), _optr(thetabar),
                                         int(nquad), float(tol), int(m_max)))


def tdmrg_theta_form(ctx, Dl, d1, Dm, d2, Dr, M, B, theta):
    ctx.check(lib().tdmrg_theta_form(ctx.h, Dl, d1, Dm, d2, Dr, _dptr(M), _dptr(B), _dptr(theta)))


def tdmrg_svd_truncate(ctx, Dl, d1, d2, Dr, theta, eps, D_max, sv_mode, tie_rel, k_cap, U, S, Vh):
    k, disc = c_int(), c_double()
    ctx.check(lib().tdmrg_svd_truncate(ctx.h, Dl, d1, d2, Dr, _dptr(theta), float(eps), int(D_max),
                                       int(sv_mode), float(tie_rel), int(k_cap), _dptr(U),
                                       _dptr(S), _dptr(Vh), ctypes.byref(k), ctypes.byref(disc)))
    return k.value, disc.value


def tdmrg_env_update_left(ctx, Dl, d, Dr, Lin, W, A, Lout, precision=FP64):
    ctx.check(lib().tdmrg_env_update_left(ctx.h, Dl, d, Dr, _dptr(Lin), W.h, _dptr(A), _dptr(Lout),
                                          precision))


def tdmrg_env_update_right(ctx, Dl, d, Dr, Rin, W, B, Rout, precision=FP64):
    ctx.check(lib().tdmrg_env_update_right(ctx.h, Dl, d, Dr, _dptr(Rin), W.h, _dptr(B),
                                           _dptr(Rout), precision))
