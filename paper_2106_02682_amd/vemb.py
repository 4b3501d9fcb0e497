"""ctypes binding of libvemb (C ABI in include/vemb.h).

Argument marshalling only: every step of the iteration runs in the HIP
kernels of libvemb.so.  If the library is missing, loading fails loudly;
there is no CPU fallback.  torch supplies device buffers and the HIP stream
for the batched entry points.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libvemb.so")

VEMB_OK = 0
STATUS = {0: "VEMB_OK", -1: "VEMB_E_INVALID", -2: "VEMB_E_UNSUPPORTED", -3: "VEMB_E_NOMEM", -4: "VEMB_E_HIP",
          -5: "VEMB_E_NUMERIC", -6: "VEMB_E_DIVERGED", -7: "VEMB_E_NOCONV"}
PAULI = {"I": 0, "X": 1, "Y": 2, "Z": 3, "F": 4}  # "F": an end of a fermionic hopping
OPSET = {"complete": 0, "pauli1": 1}
PRECISION = {"fp64": 0, "mixed": 1, "fp32": 2}
RHO, RHO_TILDE = 0, 1

EXPORTS = [
    "vemb_default_options", "vemb_create_problem", "vemb_problem_info", "vemb_step", "vemb_dual_bound",
    "vemb_primal_energy", "vemb_marginals", "vemb_get_state", "vemb_set_state", "vemb_destroy",
    "vemb_last_error", "vemb_psd_project_batched", "vemb_eigvalsh_batched", "vemb_last_sweeps",
    "vemb_psd_project_batched_ex", "vemb_set_profiling", "vemb_get_profile", "vemb_refine",
    "vemb_tuned_threads", "vemb_problem_threads", "vemb_batch_create", "vemb_batch_step", "vemb_batch_dual_bounds",
    "vemb_batch_primal_energies", "vemb_batch_info", "vemb_batch_sync", "vemb_batch_destroy",
    "vemb_warm_size", "vemb_warm_encode", "vemb_warm_start", "vemb_mlp_create", "vemb_mlp_num_params",
    "vemb_mlp_set_params", "vemb_mlp_get_params", "vemb_mlp_fit_normalization", "vemb_mlp_get_normalization",
    "vemb_mlp_set_normalization", "vemb_mlp_forward", "vemb_mlp_gradients", "vemb_mlp_adam_step",
    "vemb_mlp_train_step", "vemb_mlp_destroy", "vemb_diagnostics", "vemb_diagnostics_enqueue",
    "vemb_diagnostics_collect", "vemb_set_profiling_mask", "vemb_dense_create", "vemb_dense_get_info",
    "vemb_dense_step", "vemb_dense_dual_bound", "vemb_dense_primal_energy", "vemb_dense_get_state",
    "vemb_dense_set_state", "vemb_dense_last_sweeps", "vemb_dense_destroy", "vemb_psd_project_sign",
    "vemb_set_profiling_every", "vemb_psd_project_sign_noalloc", "vemb_batch_set_profiling",
    "vemb_batch_get_profile", "vemb_tile_map", "vemb_set_allocator", "vemb_divergence_check",
    "vemb_penalties", "vemb_set_penalty_scale", "vemb_batch_set_active", "vemb_batch_get_active",
    "vemb_warm_start_ex",
]
BATCH_KERNELS = ["pair_update", "pair_xstep", "cluster_update", "dft_forward", "dft_inverse", "pair_jacobi",
                 "momentum_jacobi", "sign_gemm_real", "sign_gemm_complex"]
KERNELS = ["pair_update", "pair_xstep", "pair_projection", "cluster_update", "dft_forward", "momentum_projection",
           "dft_inverse", "bound_build", "lambda_min", "projections"]


class VembError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code


class vemb_term(ctypes.Structure):
    _fields_ = [("coeff", ctypes.c_double), ("nsites", ctypes.c_int32), ("pauli", ctypes.c_int32 * 2),
                ("offset", (ctypes.c_int32 * 2) * 2)]


class vemb_hamiltonian(ctypes.Structure):
    _fields_ = [("nterms", ctypes.c_int32), ("terms", ctypes.POINTER(vemb_term))]


class vemb_lattice(ctypes.Structure):
    _fields_ = [("ndim", ctypes.c_int32), ("extent", ctypes.c_int32 * 2), ("periodic", ctypes.c_int32 * 2)]


class vemb_clusters(ctypes.Structure):
    _fields_ = [("shape", ctypes.c_int32 * 2)]


class vemb_options(ctypes.Structure):
    _fields_ = [("mu", ctypes.c_double), ("nu", ctypes.c_double), ("eps", ctypes.c_double),
                ("opset", ctypes.c_int32), ("precision", ctypes.c_int32), ("max_sweeps", ctypes.c_int32),
                ("sign", ctypes.c_int32), ("warm_refresh", ctypes.c_int32), ("tpb", ctypes.c_int32),
                ("fermionic", ctypes.c_int32), ("lb_every", ctypes.c_int32), ("adapt_every", ctypes.c_int32)]


class vemb_info(ctypes.Structure):
    _fields_ = [("M", ctypes.c_int32), ("P", ctypes.c_int32), ("L", ctypes.c_int32), ("m", ctypes.c_int32),
                ("n", ctypes.c_int32), ("n_op", ctypes.c_int32), ("Mx", ctypes.c_int32), ("My", ctypes.c_int32),
                ("K_unique", ctypes.c_int32), ("t", ctypes.c_int64)]


_DP = ctypes.POINTER(ctypes.c_double)


class vemb_profile(ctypes.Structure):
    _fields_ = [("ms", ctypes.c_double * 10), ("launches", ctypes.c_int64 * 10)]


class vemb_batch_profile(ctypes.Structure):
    _fields_ = [("ms", ctypes.c_double * 9), ("launches", ctypes.c_int64 * 9)]


class vemb_state(ctypes.Structure):
    _fields_ = [("t", ctypes.c_int64), ("X", _DP), ("rho0", _DP), ("rho", _DP), ("rho_t", _DP), ("Lam", _DP),
                ("Lam1", _DP), ("Lam2", _DP), ("Vpair", _DP), ("Vmom", _DP)]


class vemb_site_field(ctypes.Structure):
    _fields_ = [("x", ctypes.c_int32), ("y", ctypes.c_int32), ("pauli", ctypes.c_int32), ("coeff", ctypes.c_double)]


class vemb_dense_info(ctypes.Structure):
    _fields_ = [("M", ctypes.c_int32), ("Q", ctypes.c_int32), ("L", ctypes.c_int32), ("m", ctypes.c_int32),
                ("n", ctypes.c_int32), ("n_op", ctypes.c_int32), ("K", ctypes.c_int32), ("t", ctypes.c_int64)]


class vemb_dense_state(ctypes.Structure):
    _fields_ = [("t", ctypes.c_int64), ("X", _DP), ("rho0", _DP), ("rho", _DP), ("rho_t", _DP), ("Lam", _DP),
                ("Lam1", _DP), ("Lam2", _DP)]


_lib = None


def lib():
    """Loads libvemb.so; raises if it has not been built (no fallback exists)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2106_02682_amd.build`")
    L = ctypes.CDLL(LIB_PATH)
    vp = ctypes.c_void_p
    L.vemb_default_options.argtypes = [ctypes.POINTER(vemb_options)]
    L.vemb_default_options.restype = None
    L.vemb_create_problem.argtypes = [ctypes.POINTER(vemb_hamiltonian), ctypes.POINTER(vemb_lattice),
                                      ctypes.POINTER(vemb_clusters), ctypes.POINTER(vemb_options), vp,
                                      ctypes.POINTER(vp)]
    L.vemb_problem_info.argtypes = [vp, ctypes.POINTER(vemb_info)]
    L.vemb_step.argtypes = [vp, ctypes.c_int]
    L.vemb_refine.argtypes = [vp, ctypes.c_int]
    L.vemb_tuned_threads.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, vp]
    L.vemb_problem_threads.argtypes = [vp, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int)]
    L.vemb_dual_bound.argtypes = [vp, _DP]
    L.vemb_primal_energy.argtypes = [vp, _DP, _DP]
    L.vemb_diagnostics.argtypes = [vp, _DP, _DP, _DP]
    L.vemb_diagnostics_enqueue.argtypes = [vp]
    L.vemb_diagnostics_collect.argtypes = [vp, _DP, _DP, _DP]
    L.vemb_set_profiling_mask.argtypes = [vp, ctypes.c_uint32]
    L.vemb_set_profiling_every.argtypes = [vp, ctypes.c_int]
    L.vemb_marginals.argtypes = [vp, ctypes.c_int, _DP, _DP]
    L.vemb_get_state.argtypes = [vp, ctypes.POINTER(vemb_state)]
    L.vemb_set_state.argtypes = [vp, ctypes.POINTER(vemb_state)]
    L.vemb_destroy.argtypes = [vp]
    L.vemb_destroy.restype = None
    L.vemb_last_error.argtypes = []
    L.vemb_last_error.restype = ctypes.c_char_p
    L.vemb_psd_project_batched.argtypes = [vp, vp, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, vp]
    L.vemb_eigvalsh_batched.argtypes = [vp, vp, ctypes.c_int, ctypes.c_int, ctypes.c_int, vp]
    L.vemb_set_profiling.argtypes = [vp, ctypes.c_int]
    L.vemb_get_profile.argtypes = [vp, ctypes.POINTER(vemb_profile)]
    L.vemb_last_sweeps.argtypes = [vp, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int)]
    L.vemb_psd_project_batched_ex.argtypes = [vp, vp, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                              ctypes.c_int, vp, ctypes.c_int, vp]
    L.vemb_batch_create.argtypes = [ctypes.POINTER(vp), ctypes.c_int, ctypes.c_int, ctypes.POINTER(vp)]
    L.vemb_batch_step.argtypes = [vp, ctypes.c_int]
    L.vemb_batch_dual_bounds.argtypes = [vp, _DP, ctypes.POINTER(ctypes.c_int)]
    L.vemb_batch_primal_energies.argtypes = [vp, _DP, _DP]
    L.vemb_batch_info.argtypes = [vp, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int)]
    L.vemb_batch_sync.argtypes = [vp]
    L.vemb_set_allocator.argtypes = [ALLOC_FN, FREE_FN, vp]
    L.vemb_divergence_check.argtypes = [_DP, ctypes.c_int, ctypes.c_double, ctypes.c_double]
    L.vemb_tile_map.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_int),
                                ctypes.POINTER(ctypes.c_int)]
    L.vemb_batch_set_profiling.argtypes = [vp, ctypes.c_int]
    L.vemb_batch_get_profile.argtypes = [vp, ctypes.POINTER(vemb_batch_profile)]
    L.vemb_batch_destroy.argtypes = [vp]
    L.vemb_batch_destroy.restype = None
    _FP = ctypes.POINTER(ctypes.c_float)
    _I64 = ctypes.POINTER(ctypes.c_int64)
    L.vemb_warm_size.argtypes = [vp, ctypes.c_int, _I64]
    L.vemb_warm_encode.argtypes = [vp, ctypes.c_int, vp]
    L.vemb_warm_start.argtypes = [vp, ctypes.c_int, vp]
    L.vemb_mlp_create.argtypes = [ctypes.POINTER(ctypes.c_int32), ctypes.c_int, _FP, ctypes.c_int, vp,
                                  ctypes.POINTER(vp)]
    L.vemb_mlp_num_params.argtypes = [vp, _I64]
    L.vemb_mlp_set_params.argtypes = [vp, _FP]
    L.vemb_mlp_get_params.argtypes = [vp, _FP]
    L.vemb_mlp_fit_normalization.argtypes = [vp, vp, ctypes.c_int, ctypes.c_float]
    L.vemb_mlp_get_normalization.argtypes = [vp, _FP, _FP]
    L.vemb_mlp_set_normalization.argtypes = [vp, _FP, _FP]
    L.vemb_mlp_forward.argtypes = [vp, vp, vp, ctypes.c_int]
    L.vemb_mlp_gradients.argtypes = [vp, vp, vp, ctypes.c_int, _DP, vp]
    L.vemb_mlp_adam_step.argtypes = [vp, ctypes.c_float]
    L.vemb_mlp_train_step.argtypes = [vp, vp, vp, ctypes.c_int, vp, ctypes.c_int, ctypes.c_float, _DP]
    L.vemb_mlp_destroy.argtypes = [vp]
    L.vemb_mlp_destroy.restype = None
    L.vemb_dense_create.argtypes = [ctypes.POINTER(vemb_hamiltonian), ctypes.POINTER(vemb_lattice),
                                    ctypes.POINTER(vemb_clusters), ctypes.POINTER(vemb_site_field), ctypes.c_int,
                                    ctypes.POINTER(vemb_options), vp, ctypes.POINTER(vp)]
    L.vemb_dense_get_info.argtypes = [vp, ctypes.POINTER(vemb_dense_info)]
    L.vemb_dense_step.argtypes = [vp, ctypes.c_int]
    L.vemb_dense_dual_bound.argtypes = [vp, _DP]
    L.vemb_dense_primal_energy.argtypes = [vp, _DP, _DP]
    L.vemb_dense_get_state.argtypes = [vp, ctypes.POINTER(vemb_dense_state)]
    L.vemb_dense_set_state.argtypes = [vp, ctypes.POINTER(vemb_dense_state)]
    L.vemb_dense_last_sweeps.argtypes = [vp, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int)]
    L.vemb_dense_destroy.argtypes = [vp]
    L.vemb_psd_project_sign.argtypes = [vp, vp, ctypes.c_int, vp]
    L.vemb_psd_project_sign_noalloc.argtypes = [vp, vp, ctypes.c_int, vp]
    L.vemb_dense_destroy.restype = None
    for name in EXPORTS:
        if name not in ("vemb_default_options", "vemb_destroy", "vemb_last_error", "vemb_batch_destroy",
                        "vemb_mlp_destroy", "vemb_dense_destroy"):
            getattr(L, name).restype = ctypes.c_int
    _lib = L
    return L


def _check(rc):
    if rc != VEMB_OK:
        raise VembError(rc, lib().vemb_last_error().decode())
    return rc


def _ptr(a):
    return a.ctypes.data_as(_DP) if a is not None else None


ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)


class TorchAllocator:
    """Device memory of the library from torch's caching allocator (vemb_set_allocator).

    Each request becomes a uint8 tensor on the current device, kept alive here until the library
    returns its pointer; the library frees only after synchronising the streams that used the memory.
    ``count`` / ``bytes`` tally every request, ``live`` maps the outstanding pointers to their tensors."""

    def __init__(self):
        self.live = {}
        self.count = 0
        self.bytes = 0
        self.frees = 0

        def _alloc(nbytes, ctx):
            try:
                import torch

                t = torch.empty(int(nbytes) + 256, dtype=torch.uint8, device="cuda")
                ptr = (t.data_ptr() + 255) & ~255
                self.live[ptr] = t
                self.count += 1
                self.bytes += int(nbytes)
                return ptr
            except Exception:  # noqa: BLE001 -- no exception may cross into the library
                return None

        def _free(ptr, ctx):
            try:
                if self.live.pop(int(ptr), None) is not None:
                    self.frees += 1
            except Exception:  # noqa: BLE001
                pass

        self._alloc = ALLOC_FN(_alloc)
        self._free = FREE_FN(_free)

    def install(self):
        _check(lib().vemb_set_allocator(self._alloc, self._free, None))

    @staticmethod
    def uninstall():
        """Back to hipMalloc / hipFree (no library object may be alive)."""
        _check(lib().vemb_set_allocator(ALLOC_FN(), FREE_FN(), None))


_allocator = None
_allocator_decided = False


def torch_allocator():
    """The TorchAllocator the binding installed, or None (no GPU, or VEMB_ALLOCATOR=hip)."""
    _ensure_allocator()
    return _allocator


def _ensure_allocator():
    """Before the first device allocation: route the library's device memory through torch's caching
    allocator when torch has a GPU (set VEMB_ALLOCATOR=hip to keep hipMalloc)."""
    global _allocator, _allocator_decided
    if _allocator_decided:
        return
    _allocator_decided = True
    if os.environ.get("VEMB_ALLOCATOR", "torch") == "hip":
        return
    try:
        import torch
    except ImportError:
        return
    if torch.cuda.is_available():
        a = TorchAllocator()
        a.install()
        _allocator = a


def current_stream():
    """torch's current HIP stream as a void pointer (NULL when torch has no GPU)."""
    try:
        import torch

        if torch.cuda.is_available():
            _ensure_allocator()
            return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    except ImportError:
        pass
    return ctypes.c_void_p(None)


def default_options():
    o = vemb_options()
    lib().vemb_default_options(ctypes.byref(o))
    return o


def _marshal(terms, extent, cluster, opset, precision, mu, nu, eps, max_sweeps, sign, warm_refresh, tpb,
             fermionic=False, lb_every=0, adapt_every=0):
    """ctypes structs of a term list (``synth`` format: (coeff, ((pauli, (ox, oy)), ...))), lattice,
    clusters and options; the term array is returned too, to stay alive with the Hamiltonian."""
    arr = (vemb_term * max(1, len(terms)))()
    for t, (coeff, factors) in enumerate(terms):
        arr[t].coeff = float(coeff)
        arr[t].nsites = len(factors)
        for s, (pl, off) in enumerate(factors[:2]):
            arr[t].pauli[s] = PAULI[pl]
            arr[t].offset[s][0] = int(off[0])
            arr[t].offset[s][1] = int(off[1])
    H = vemb_hamiltonian(len(terms), arr)
    ndim = 1 if extent[1] == 1 else 2
    lat = vemb_lattice(ndim, (ctypes.c_int32 * 2)(extent[0], extent[1]), (ctypes.c_int32 * 2)(1, 1))
    cl = vemb_clusters((ctypes.c_int32 * 2)(cluster[0], cluster[1]))
    o = default_options()
    o.mu, o.nu, o.eps = mu, nu, eps
    o.opset = OPSET[opset]
    o.precision = PRECISION[precision]
    o.max_sweeps = max_sweeps
    o.sign = sign
    o.warm_refresh = warm_refresh
    o.tpb = tpb
    o.fermionic = 1 if fermionic else 0
    o.lb_every = int(lb_every)
    o.adapt_every = int(adapt_every)
    return H, lat, cl, o, arr


def create_problem(terms, extent, cluster, opset="complete", precision="fp64", mu=10.0, nu=10.0, eps=2.0,
                   max_sweeps=40, sign=-1, warm_refresh=64, tpb=0, stream=None, fermionic=False, lb_every=0,
                   adapt_every=0):
    """Terms in the ``synth`` format: (coeff, ((pauli, (ox, oy)), ...)); "F" letters are the ends of a
    fermionic hopping (fermionic problems)."""
    H, lat, cl, o, _keep = _marshal(terms, extent, cluster, opset, precision, mu, nu, eps, max_sweeps, sign,
                                    warm_refresh, tpb, fermionic, lb_every, adapt_every)
    h = ctypes.c_void_p()
    _ensure_allocator()
    st = stream if stream is not None else current_stream()
    _check(lib().vemb_create_problem(ctypes.byref(H), ctypes.byref(lat), ctypes.byref(cl), ctypes.byref(o), st,
                                     ctypes.byref(h)))
    return h


def problem_info(h):
    info = vemb_info()
    _check(lib().vemb_problem_info(h, ctypes.byref(info)))
    return {f: getattr(info, f) for f, _ in vemb_info._fields_}


def step(h, iters):
    _check(lib().vemb_step(h, int(iters)))


def penalties(h):
    """Parameters in force: dict mu, nu, eps, scale (joint scale of the adaptive mode), last_feas, last_gap."""
    v = [ctypes.c_double() for _ in range(6)]
    _check(lib().vemb_penalties(h, *[ctypes.byref(x) for x in v]))
    return dict(zip(("mu", "nu", "eps", "scale", "last_feas", "last_gap"), (x.value for x in v)))


def set_penalty_scale(h, scale, last_feas=-1.0, last_gap=-1.0):
    _check(lib().vemb_set_penalty_scale(h, ctypes.c_double(scale), ctypes.c_double(last_feas),
                                        ctypes.c_double(last_gap)))


def refine(h, iters=1):
    _check(lib().vemb_refine(h, int(iters)))


def dual_bound(h):
    v = ctypes.c_double()
    _check(lib().vemb_dual_bound(h, ctypes.byref(v)))
    return v.value


def primal_energy(h):
    e, f = ctypes.c_double(), ctypes.c_double()
    _check(lib().vemb_primal_energy(h, ctypes.byref(e), ctypes.byref(f)))
    return e.value, f.value


def diagnostics(h):
    """(bound per site, energy per site, feasibility error) with one synchronisation."""
    lb, e, f = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
    _check(lib().vemb_diagnostics(h, ctypes.byref(lb), ctypes.byref(e), ctypes.byref(f)))
    return lb.value, e.value, f.value


def diagnostics_enqueue(h):
    _check(lib().vemb_diagnostics_enqueue(h))


def diagnostics_collect(h):
    lb, e, f = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
    _check(lib().vemb_diagnostics_collect(h, ctypes.byref(lb), ctypes.byref(e), ctypes.byref(f)))
    return lb.value, e.value, f.value


def marginals(h, which=RHO):
    info = problem_info(h)
    rho0 = np.zeros((info["m"], info["m"]))
    pairs = np.zeros((info["P"], info["n"], info["n"]))
    _check(lib().vemb_marginals(h, which, _ptr(rho0), _ptr(pairs)))
    return rho0, pairs


def _state_arrays(info):
    M, P, m, n, k = info["M"], info["P"], info["m"], info["n"], info["n_op"]
    return {"X": np.zeros((M, k, k)), "rho0": np.zeros((m, m)), "rho": np.zeros((P, n, n)),
            "rho_t": np.zeros((P, n, n)), "Lam": np.zeros((P, n, n)), "Lam1": np.zeros((P, m, m)),
            "Lam2": np.zeros((P, m, m))}


_STATE_KEYS = ("X", "rho0", "rho", "rho_t", "Lam", "Lam1", "Lam2")


def get_state(h, with_eigvecs=False):
    """State arrays; with_eigvecs adds the kept eigenvectors (Vpair, Vmom) for bit-exact resume."""
    info = problem_info(h)
    arrs = _state_arrays(info)
    if with_eigvecs:
        arrs["Vpair"] = np.zeros((info["P"], info["n"], info["n"]))
        arrs["Vmom"] = np.zeros((info["K_unique"], info["n_op"], info["n_op"], 2))
    ptrs = [_ptr(arrs[k]) for k in _STATE_KEYS] + [_ptr(arrs.get("Vpair")), _ptr(arrs.get("Vmom"))]
    st = vemb_state(0, *ptrs)
    _check(lib().vemb_get_state(h, ctypes.byref(st)))
    arrs["t"] = st.t
    return arrs


def set_state(h, state):
    arrs = {k: np.ascontiguousarray(state[k], dtype=np.float64) for k in _STATE_KEYS}
    for k in ("Vpair", "Vmom"):
        if state.get(k) is not None:
            arrs[k] = np.ascontiguousarray(state[k], dtype=np.float64)
    ptrs = [_ptr(arrs[k]) for k in _STATE_KEYS] + [_ptr(arrs.get("Vpair")), _ptr(arrs.get("Vmom"))]
    st = vemb_state(int(state.get("t", 0)), *ptrs)
    _check(lib().vemb_set_state(h, ctypes.byref(st)))


def destroy(h):
    if h:
        lib().vemb_destroy(h)


def psd_project_batched(inp, out, is_complex=False, precision="fp64", stream=None):
    """Device tensors (torch, float64; complex as interleaved float64 pairs)."""
    n = inp.shape[-2]
    batch = inp.numel() // (n * n * (2 if is_complex else 1))
    st = stream if stream is not None else current_stream()
    _check(lib().vemb_psd_project_batched(ctypes.c_void_p(inp.data_ptr()), ctypes.c_void_p(out.data_ptr()), n,
                                          batch, int(is_complex), PRECISION[precision], st))


def psd_project_sign(inp, out, stream=None):
    """Pi of one n x n symmetric FP64 matrix (torch device tensors, n a multiple of 16) by the matrix-sign
    iteration on matrix cores."""
    n = inp.shape[-1]
    st = stream if stream is not None else current_stream()
    _check(lib().vemb_psd_project_sign(ctypes.c_void_p(inp.data_ptr()), ctypes.c_void_p(out.data_ptr()), n, st))


def psd_project_sign_noalloc(inp, out, stream=None):
    """As psd_project_sign, with the scratch in the library's static device array (n <= 512): no
    allocation; asynchronous on the stream."""
    n = inp.shape[-1]
    st = stream if stream is not None else current_stream()
    _check(lib().vemb_psd_project_sign_noalloc(ctypes.c_void_p(inp.data_ptr()), ctypes.c_void_p(out.data_ptr()), n,
                                               st))


def tile_map(kind, n, count=1):
    """(grid, map) of the symmetric-product kernels (see vemb_tile_map): map is an int array (grid, 4) of
    {live, block, tile row, tile column} per workgroup.  Host only: needs no GPU."""
    g = ctypes.c_int()
    _check(lib().vemb_tile_map(int(kind), int(n), int(count), ctypes.byref(g), None))
    m = np.zeros((g.value, 4), dtype=np.int32)
    _check(lib().vemb_tile_map(int(kind), int(n), int(count), ctypes.byref(g),
                               m.ctypes.data_as(ctypes.POINTER(ctypes.c_int))))
    return g.value, m


def psd_project_batched_ex(inp, out, is_complex=False, precision="fp64", max_sweeps=0, sweeps=None, tpb=0,
                           stream=None):
    """As psd_project_batched; ``sweeps`` is an optional int32 device tensor of length batch, ``tpb`` the
    LDS solver variant (0 = autotuned; 64 / 128 = register-resident for n = 64)."""
    n = inp.shape[-2]
    batch = inp.numel() // (n * n * (2 if is_complex else 1))
    st = stream if stream is not None else current_stream()
    sp = ctypes.c_void_p(sweeps.data_ptr()) if sweeps is not None else ctypes.c_void_p(None)
    _check(lib().vemb_psd_project_batched_ex(ctypes.c_void_p(inp.data_ptr()), ctypes.c_void_p(out.data_ptr()), n,
                                             batch, int(is_complex), PRECISION[precision], int(max_sweeps), sp,
                                             int(tpb), st))


def set_profiling(h, enable=True, kernels=None):
    """Kernel timing on / off; ``kernels`` (names from KERNELS) restricts it to those."""
    if kernels is None:
        _check(lib().vemb_set_profiling(h, int(bool(enable))))
    else:
        mask = 0
        for k in kernels:
            mask |= 1 << KERNELS.index(k)
        _check(lib().vemb_set_profiling_mask(h, mask if enable else 0))


def get_profile(h):
    """{kernel: (total device ms, launches)} since profiling was enabled."""
    pr = vemb_profile()
    _check(lib().vemb_get_profile(h, ctypes.byref(pr)))
    return {k: (pr.ms[i], pr.launches[i]) for i, k in enumerate(KERNELS)}


def tuned_threads(n, is_complex=False, precision="fp64", batch=1, stream=None):
    st = stream if stream is not None else current_stream()
    rc = lib().vemb_tuned_threads(int(n), int(is_complex), PRECISION[precision], int(batch), st)
    if rc < 0:
        _check(rc)
    return rc


def problem_threads(h):
    a, b = ctypes.c_int(), ctypes.c_int()
    _check(lib().vemb_problem_threads(h, ctypes.byref(a), ctypes.byref(b)))
    return a.value, b.value


def last_sweeps(h, check=True):
    """(pair max, momentum max) sweeps of the last iteration; raises VembError (VEMB_E_NOCONV) when an
    eigensolve stopped unconverged, unless check=False, which returns (pair, momentum, status)."""
    a, b = ctypes.c_int(), ctypes.c_int()
    rc = lib().vemb_last_sweeps(h, ctypes.byref(a), ctypes.byref(b))
    if not check:
        return a.value, b.value, rc
    _check(rc)
    return a.value, b.value


def divergence_check(feas, lb, energy):
    """The watchdog's decision (vemb_divergence_check) on a feasibility history: 0, or the status code."""
    f = np.ascontiguousarray(feas, dtype=np.float64)
    return lib().vemb_divergence_check(_ptr(f), len(f), float(lb), float(energy))


def eigvalsh_batched(inp, w, is_complex=False, stream=None):
    n = inp.shape[-2]
    batch = inp.numel() // (n * n * (2 if is_complex else 1))
    st = stream if stream is not None else current_stream()
    _check(lib().vemb_eigvalsh_batched(ctypes.c_void_p(inp.data_ptr()), ctypes.c_void_p(w.data_ptr()), n, batch,
                                       int(is_complex), st))


class Problem:
    """Owning wrapper of one problem handle."""

    def __init__(self, terms, extent, cluster, **kw):
        self.h = create_problem(terms, extent, cluster, **kw)
        self.info = problem_info(self.h)

    @classmethod
    def from_workload(cls, w, **kw):
        kw.setdefault("fermionic", getattr(w, "fermionic", False))
        kw.setdefault("opset", w.opset)
        kw.setdefault("mu", w.mu)
        kw.setdefault("nu", w.nu)
        kw.setdefault("eps", w.eps)
        return cls(w.terms, w.extent, w.cluster, **kw)

    def step(self, iters=1):
        step(self.h, iters)

    def penalties(self):
        return penalties(self.h)

    def set_penalty_scale(self, scale, last_feas=-1.0, last_gap=-1.0):
        set_penalty_scale(self.h, scale, last_feas, last_gap)

    def refine(self, iters=1):
        refine(self.h, iters)

    def dual_bound(self):
        return dual_bound(self.h)

    def last_sweeps(self, check=True):
        return last_sweeps(self.h, check)

    def set_profiling(self, enable=True, kernels=None):
        set_profiling(self.h, enable, kernels)

    def get_profile(self):
        return get_profile(self.h)

    def set_profiling_every(self, every):
        """Time only every `every`-th iteration (see set_profiling)."""
        _check(lib().vemb_set_profiling_every(self.h, int(every)))

    def primal_energy(self):
        return primal_energy(self.h)

    def diagnostics(self):
        return diagnostics(self.h)

    def diagnostics_enqueue(self):
        diagnostics_enqueue(self.h)

    def diagnostics_collect(self):
        return diagnostics_collect(self.h)

    def marginals(self, which=RHO):
        return marginals(self.h, which)

    def get_state(self, with_eigvecs=False):
        return get_state(self.h, with_eigvecs)

    def set_state(self, s):
        set_state(self.h, s)

    def close(self):
        if self.h:
            destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


class Batch:
    """Several problems stepped together (one launch per step kernel and per
    eigensolver size class, replayed from HIP graphs).  Holds references to the
    Problem objects so they outlive the batch."""

    def __init__(self, problems, use_graph=True):
        self.problems = list(problems)
        if not self.problems or any(p.h is None for p in self.problems):
            raise ValueError("a batch needs open problems")
        arr = (ctypes.c_void_p * len(self.problems))(*[p.h for p in self.problems])
        out = ctypes.c_void_p()
        _check(lib().vemb_batch_create(arr, len(self.problems), int(bool(use_graph)), ctypes.byref(out)))
        self.h = out

    def step(self, iters=1):
        _check(lib().vemb_batch_step(self.h, int(iters)))

    def sync(self):
        _check(lib().vemb_batch_sync(self.h))

    def dual_bounds(self, check=True):
        """Per-problem bounds; check=False returns (bounds, status codes) instead of raising."""
        lb = np.zeros(len(self.problems))
        st = (ctypes.c_int * len(self.problems))()
        lib().vemb_batch_dual_bounds(self.h, _ptr(lb), st)
        if not check:
            return lb, list(st)
        for rc in st:
            _check(rc)
        return lb

    def primal_energies(self, check=True):
        e = np.zeros(len(self.problems))
        f = np.zeros(len(self.problems))
        rc = lib().vemb_batch_primal_energies(self.h, _ptr(e), _ptr(f))
        if check:
            _check(rc)
        return e, f

    def set_active(self, index, active=True):
        """Mask (False) or unmask (True) one instance: a masked instance is skipped by later steps."""
        _check(lib().vemb_batch_set_active(self.h, int(index), int(bool(active))))

    def active(self):
        a = (ctypes.c_int * len(self.problems))()
        _check(lib().vemb_batch_get_active(self.h, a))
        return [bool(x) for x in a]

    def set_profiling(self, every):
        """Time the kernels of every ``every``-th iteration (0 = off); resets the accumulated times."""
        _check(lib().vemb_batch_set_profiling(self.h, int(every)))

    def get_profile(self):
        """{kernel: (total device ms, timed launches)} since the last set_profiling."""
        out = vemb_batch_profile()
        _check(lib().vemb_batch_get_profile(self.h, ctypes.byref(out)))
        return {k: (out.ms[i], out.launches[i]) for i, k in enumerate(BATCH_KERNELS)}

    def info(self):
        a, b = ctypes.c_int(), ctypes.c_int()
        _check(lib().vemb_batch_info(self.h, ctypes.byref(a), ctypes.byref(b)))
        return {"classes": a.value, "launches_per_iteration": b.value}

    def close(self):
        if self.h:
            lib().vemb_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


# ---------------------------------------------------------------------------
# Learned warm start
# ---------------------------------------------------------------------------

def _dev(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _fp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_float))


WARM_NEAR = 3


def warm_size(h, near=WARM_NEAR):
    c = ctypes.c_int64()
    _check(lib().vemb_warm_size(h, int(near), ctypes.byref(c)))
    return c.value


def warm_encode(h, out, near=WARM_NEAR):
    """out: device float32 tensor of warm_size(h, near) elements."""
    _check(lib().vemb_warm_encode(h, int(near), _dev(out)))


def warm_start(h, vec, near=WARM_NEAR, far_cold=False):
    """vec: device float32 tensor of warm_size(h, near) elements; far_cold starts the offsets beyond
    `near` cold instead of from the far slot."""
    if far_cold:
        _check(lib().vemb_warm_start_ex(h, int(near), _dev(vec), 1))
        return
    _check(lib().vemb_warm_start(h, int(near), _dev(vec)))


class MLP:
    """The warm-start network (parameters and work buffers on the device)."""

    def __init__(self, dims, params=None, max_batch=512, stream=None):
        self.dims = [int(d) for d in dims]
        arr = (ctypes.c_int32 * len(self.dims))(*self.dims)
        out = ctypes.c_void_p()
        p = None
        if params is not None:
            params = np.ascontiguousarray(params, dtype=np.float32)
            p = _fp(params)
        _ensure_allocator()
        st = current_stream() if stream is None else stream
        _check(lib().vemb_mlp_create(arr, len(self.dims), p, int(max_batch), st, ctypes.byref(out)))
        self.h = out
        c = ctypes.c_int64()
        _check(lib().vemb_mlp_num_params(self.h, ctypes.byref(c)))
        self.num_params = c.value

    def set_params(self, params):
        params = np.ascontiguousarray(params, dtype=np.float32)
        assert params.size == self.num_params
        _check(lib().vemb_mlp_set_params(self.h, _fp(params)))

    def get_params(self):
        out = np.empty(self.num_params, np.float32)
        _check(lib().vemb_mlp_get_params(self.h, _fp(out)))
        return out

    def fit_normalization(self, targets, rel_floor=0.0):
        _check(lib().vemb_mlp_fit_normalization(self.h, _dev(targets), int(targets.shape[0]), float(rel_floor)))

    def get_normalization(self):
        O = self.dims[-1]
        mean, std = np.empty(O, np.float32), np.empty(O, np.float32)
        _check(lib().vemb_mlp_get_normalization(self.h, _fp(mean), _fp(std)))
        return mean, std

    def set_normalization(self, mean, std):
        mean = np.ascontiguousarray(mean, np.float32)
        std = np.ascontiguousarray(std, np.float32)
        _check(lib().vemb_mlp_set_normalization(self.h, _fp(mean), _fp(std)))

    def forward(self, x, y):
        _check(lib().vemb_mlp_forward(self.h, _dev(x), _dev(y), int(x.shape[0])))

    def gradients(self, x, t, grad=None):
        loss = ctypes.c_double()
        _check(lib().vemb_mlp_gradients(self.h, _dev(x), _dev(t), int(x.shape[0]), ctypes.byref(loss), _dev(grad)))
        return loss.value

    def adam_step(self, lr):
        _check(lib().vemb_mlp_adam_step(self.h, float(lr)))

    def train_step(self, X, T, rows=None, batch=None, lr=1e-3, want_loss=False):
        batch = int(batch if batch is not None else (rows.shape[0] if rows is not None else X.shape[0]))
        loss = ctypes.c_double()
        _check(lib().vemb_mlp_train_step(self.h, _dev(X), _dev(T), int(X.shape[0]), _dev(rows), batch, float(lr),
                                         ctypes.byref(loss) if want_loss else None))
        return loss.value if want_loss else None

    def close(self):
        if self.h:
            lib().vemb_mlp_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


# ---------------------------------------------------------------------------
# Dense Algorithm 5 (no translation invariance): one marginal per cluster and per
# cluster pair, one dense X; site fields make the clusters differ.
# ---------------------------------------------------------------------------
_DENSE_KEYS = ("X", "rho0", "rho", "rho_t", "Lam", "Lam1", "Lam2")


class Dense:
    """Owning wrapper of one dense problem.  fields: iterable of (letter, (x, y), coeff), letter X or Z.
    Pairs (i, j), i < j, in lexicographic order; state arrays are stacked in that order."""

    def __init__(self, terms, extent, cluster, fields=(), opset="complete", precision="fp64", mu=10.0, nu=10.0,
                 eps=2.0, max_sweeps=40, sign=-1, warm_refresh=64, tpb=0, stream=None, fermionic=False,
                 adapt_every=0):
        H, lat, cl, o, keep = _marshal(terms, extent, cluster, opset, precision, mu, nu, eps, max_sweeps, sign,
                                       warm_refresh, tpb, fermionic, 0, adapt_every)
        fields = list(fields)
        farr = (vemb_site_field * max(1, len(fields)))()
        for f, (letter, (x, y), coeff) in enumerate(fields):
            farr[f].x, farr[f].y = int(x), int(y)
            farr[f].pauli = PAULI[letter]
            farr[f].coeff = float(coeff)
        self.h = ctypes.c_void_p()
        _ensure_allocator()
        st = stream if stream is not None else current_stream()
        _check(lib().vemb_dense_create(ctypes.byref(H), ctypes.byref(lat), ctypes.byref(cl), farr, len(fields),
                                       ctypes.byref(o), st, ctypes.byref(self.h)))
        info = vemb_dense_info()
        _check(lib().vemb_dense_get_info(self.h, ctypes.byref(info)))
        self.info = {f: getattr(info, f) for f, _ in vemb_dense_info._fields_}

    @classmethod
    def from_workload(cls, w, fields=(), **kw):
        kw.setdefault("fermionic", getattr(w, "fermionic", False))
        kw.setdefault("opset", w.opset)
        kw.setdefault("mu", w.mu)
        kw.setdefault("nu", w.nu)
        kw.setdefault("eps", w.eps)
        return cls(w.terms, w.extent, w.cluster, fields=fields, **kw)

    def t(self):
        info = vemb_dense_info()
        _check(lib().vemb_dense_get_info(self.h, ctypes.byref(info)))
        return info.t

    def step(self, iters=1):
        _check(lib().vemb_dense_step(self.h, int(iters)))

    def dual_bound(self):
        v = ctypes.c_double()
        _check(lib().vemb_dense_dual_bound(self.h, ctypes.byref(v)))
        return v.value

    def primal_energy(self):
        e, f = ctypes.c_double(), ctypes.c_double()
        _check(lib().vemb_dense_primal_energy(self.h, ctypes.byref(e), ctypes.byref(f)))
        return e.value, f.value

    def last_sweeps(self):
        a, b = ctypes.c_int(), ctypes.c_int()
        _check(lib().vemb_dense_last_sweeps(self.h, ctypes.byref(a), ctypes.byref(b)))
        return a.value, b.value

    def _arrays(self):
        i = self.info
        M, Q, m, n, K = i["M"], i["Q"], i["m"], i["n"], i["K"]
        return {"X": np.zeros((K, K)), "rho0": np.zeros((M, m, m)), "rho": np.zeros((Q, n, n)),
                "rho_t": np.zeros((Q, n, n)), "Lam": np.zeros((Q, n, n)), "Lam1": np.zeros((Q, m, m)),
                "Lam2": np.zeros((Q, m, m))}

    def get_state(self):
        arrs = self._arrays()
        st = vemb_dense_state(0, *[_ptr(arrs[k]) for k in _DENSE_KEYS])
        _check(lib().vemb_dense_get_state(self.h, ctypes.byref(st)))
        arrs["t"] = st.t
        return arrs

    def set_state(self, state):
        shapes = self._arrays()
        arrs = {}
        for k in _DENSE_KEYS:
            if state.get(k) is not None:
                arrs[k] = np.ascontiguousarray(state[k], dtype=np.float64)
                if arrs[k].shape != shapes[k].shape:
                    raise ValueError(f"{k}: shape {arrs[k].shape}, expected {shapes[k].shape}")
        st = vemb_dense_state(int(state.get("t", 0)), *[_ptr(arrs.get(k)) for k in _DENSE_KEYS])
        _check(lib().vemb_dense_set_state(self.h, ctypes.byref(st)))

    def close(self):
        if self.h:
            lib().vemb_dense_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
