"""Thin ctypes binding of libfsa.so (the C ABI declared in include/fsa.h).

Argument marshalling only: every step of the solver runs in the library's HIP kernels.
Torch tensors provide device memory (their data pointers) and the HIP stream.  The library
must have been built (``python -m paper_1905_00182_amd.build`` or ``__graft_entry__.build``);
``lib()`` raises if it is missing rather than falling back to anything else.
"""
import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfsa.so")

OK, EINVAL, ENOMEM, EDEVICE, ENONFINITE, ESTATE, EUNSUPPORTED = 0, -1, -2, -3, -4, -5, -6
BC = {"periodic": 0, "extrap": 1, "inflow": 2, "nonreflect": 3}
SCHEME = {"weno5js": 0, "teno5": 1}
PRECISION = {"fp64": 0, "mixed32": 1, "learned32": 2}
VARIABLES = {"component": 0, "characteristic": 1}
ABI_VERSION = 4          # the fsa_desc / fsa_stats layout mirrored below (include/fsa.h)
MLP_NPARAM = 1667
MOTION = {"static": 0, "rotating": 1, "external": 2}
TERM = {"conv_x": 1, "conv_y": 2, "conv_z": 4, "visc": 8, "ib": 16, "sponge": 32, "all": 63}


class FsaError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{msg} (status {code})")
        self.code = code


class FsaDesc(C.Structure):
    _fields_ = [
        ("dim", C.c_int32),
        ("n", C.c_int32 * 3),
        ("lo", C.c_double * 3),
        ("h", C.c_double),
        ("bc", (C.c_int32 * 2) * 3),
        ("gamma", C.c_double),
        ("mu", C.c_double),
        ("scheme", C.c_int32),
        ("precision", C.c_int32),
        ("terms", C.c_int32),
        ("nan_check", C.c_int32),
        ("weno_eps", C.c_double),
        ("teno_ct", C.c_double),
        ("teno_eps", C.c_double),
        ("prim_inf", C.c_double * 5),
        ("inflow_amp", C.c_double),
        ("seed", C.c_uint64),
        ("sponge_width", (C.c_double * 2) * 3),
        ("sponge_sigma", C.c_double),
        ("ib_alpha", C.c_double),
        ("ib_beta", C.c_double),
        ("selector_stride", C.c_int32),
        ("src_amp", C.c_double),
        ("src_b", C.c_double),
        ("src_omega", C.c_double),
        ("src_x", C.c_double * 3),
        ("max_markers", C.c_int32),
        ("max_probes", C.c_int32),
        ("max_window_cells", C.c_int64),
        ("variables", C.c_int32),
        ("origin", C.c_int32 * 3),
        ("global_n", C.c_int32 * 3),
    ]


class FsaStats(C.Structure):
    _fields_ = [
        ("alpha", C.c_double * 3),
        ("t", C.c_double),
        ("step", C.c_int64),
        ("nonfinite", C.c_int32),
        ("n_markers", C.c_int32),
        ("n_probes", C.c_int32),
        ("window_cells", C.c_int32),
        ("rows_per_wave", C.c_int32),
        ("learned_sides", C.c_int64),
        ("fallback_sides", C.c_int64),
        ("significant_sides", C.c_int64),
    ]


_lib = None

class FsaPlateDesc(C.Structure):
    _fields_ = [
        ("length", C.c_double),
        ("n_elements", C.c_int32),
        ("rho_s", C.c_double),
        ("k_s", C.c_double),
        ("k_b", C.c_double),
        ("n_markers", C.c_int32),
        ("s_mark", C.c_void_p),
        ("dv_mark", C.c_void_p),
        ("edge", C.c_double * 2),
        ("a0", C.c_double),
        ("beta", C.c_double),
        ("alpha_m", C.c_double),
        ("freq", C.c_double),
        ("phi", C.c_double),
        ("t0", C.c_double),
    ]


_SIGS = {
    "fsa_abi_version": (C.c_int32, []),
    "fsa_status_str": (C.c_char_p, [C.c_int32]),
    "fsa_last_error": (C.c_char_p, [C.c_void_p]),
    "fsa_workspace_bytes": (C.c_int32, [C.POINTER(FsaDesc), C.POINTER(C.c_size_t)]),
    "fsa_init": (C.c_int32, [C.POINTER(FsaDesc), C.c_void_p, C.c_size_t, C.c_void_p, C.POINTER(C.c_void_p)]),
    "fsa_destroy": (C.c_int32, [C.c_void_p]),
    "fsa_set_markers": (C.c_int32, [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32,
                                    C.c_double]),
    "fsa_set_marker_kinematics": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_void_p]),
    "fsa_set_probes": (C.c_int32, [C.c_void_p, C.c_int32, C.c_void_p]),
    "fsa_alpha": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_void_p]),
    "fsa_alpha_noalloc": (C.c_int32, [C.POINTER(FsaDesc), C.c_void_p, C.c_void_p, C.c_void_p]),
    "fsa_rhs": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_void_p]),
    "fsa_rk3_step": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_double]),
    "fsa_rk3_steps": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_double, C.c_int32]),
    "fsa_rk3_steps_resume": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_double, C.c_int32]),
    "fsa_ib_interp": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p]),
    "fsa_ib_spread": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p, C.c_double]),
    "fsa_probe_dp": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_void_p]),
    "fsa_diagnostics": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "fsa_marker_force": (C.c_int32, [C.c_void_p, C.c_void_p]),
    "fsa_get_state": (C.c_int32, [C.c_void_p, C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_int64)]),
    "fsa_set_state": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_double, C.c_int64]),
    "fsa_mlp_set": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_int32, C.c_double]),
    "fsa_set_mlp": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_int32, C.c_double]),
    "fsa_mlp_get": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_int32]),
    "fsa_mlp_forward": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p]),
    "fsa_mlp_grad": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p]),
    "fsa_mlp_train_step": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64, C.c_float, C.c_void_p]),
    "fsa_harvest": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_double, C.c_uint64, C.c_int64, C.c_void_p, C.c_void_p,
                                C.POINTER(C.c_int64)]),
    "fsa_face_flags": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "fsa_debug_teno_bits": (C.c_int32, [C.c_void_p, C.c_void_p]),
    "fsa_timing_enable": (C.c_int32, [C.c_void_p, C.c_int32]),
    "fsa_timing_read": (C.c_int32, [C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_int64)]),
    "fsa_sync": (C.c_int32, [C.c_void_p]),
    "fsa_stats_get": (C.c_int32, [C.c_void_p, C.POINTER(FsaStats)]),
    # include/fsa_plate.h
    "fsa_marker_info": (C.c_int32, [C.c_void_p, C.POINTER(C.c_int32), C.POINTER(C.c_int32), C.POINTER(C.c_int32)]),
    "fsa_plate_create": (C.c_int32, [C.POINTER(FsaPlateDesc), C.POINTER(C.c_void_p)]),
    "fsa_plate_destroy": (C.c_int32, [C.c_void_p]),
    "fsa_plate_markers": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_void_p]),
    "fsa_plate_step": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_double]),
    "fsa_plate_get_state": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.POINTER(C.c_double)]),
    "fsa_plate_set_state": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_double]),
    "fsa_plate_last_error": (C.c_char_p, [C.c_void_p]),
    "fsa_plate_coupled_steps": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_double, C.c_int32, C.c_int32]),
    # several blocks of one domain on one GPU
    "fsa_mb_workspace_bytes": (C.c_int32, [C.POINTER(FsaDesc), C.c_int32, C.POINTER(C.c_size_t)]),
    "fsa_mb_init": (C.c_int32, [C.POINTER(FsaDesc), C.c_int32, C.c_void_p, C.c_size_t, C.c_void_p,
                                C.POINTER(C.c_void_p)]),
    "fsa_mb_destroy": (C.c_int32, [C.c_void_p]),
    "fsa_mb_last_error": (C.c_char_p, [C.c_void_p]),
    "fsa_mb_block_info": (C.c_int32, [C.c_void_p, C.c_int32, C.POINTER(C.c_int32), C.POINTER(C.c_int32),
                                      C.POINTER(C.c_int32), C.POINTER(C.c_int32)]),
    "fsa_mb_set_markers": (C.c_int32, [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32,
                                       C.c_double]),
    "fsa_mb_set_marker_kinematics": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_void_p]),
    "fsa_mb_scatter": (C.c_int32, [C.c_void_p, C.c_void_p]),
    "fsa_mb_gather": (C.c_int32, [C.c_void_p, C.c_void_p]),
    "fsa_mb_rk3_steps": (C.c_int32, [C.c_void_p, C.c_double, C.c_int32]),
    "fsa_mb_marker_force": (C.c_int32, [C.c_void_p, C.c_void_p]),
}


class Plate:
    """The flexible plate of include/fsa_plate.h (host code) for a case whose extra holds the
    clamp kinematics ("plate") and the structure ("flex"); the markers are the case's."""

    def __init__(self, case, t0=0.0):
        p, fl = case.extra["plate"], case.extra["flex"]
        self._s = np.ascontiguousarray(p["s"], dtype=np.float64)
        self._dv = np.ascontiguousarray(case.markers["dV"], dtype=np.float64)
        self.nm, self.ndof = len(self._s), 4 * (int(fl["nel"]) + 1)
        d = FsaPlateDesc()
        d.length, d.n_elements, d.rho_s, d.k_s, d.k_b = fl["length"], fl["nel"], fl["rho_s"], fl["k_s"], fl["k_b"]
        d.n_markers, d.s_mark, d.dv_mark = self.nm, self._s.ctypes.data, self._dv.ctypes.data
        d.edge[0], d.edge[1] = p["edge"]
        d.a0, d.beta, d.alpha_m, d.freq, d.phi, d.t0 = p["A0"], p["beta"], p["alpha_m"], p["f"], p["phi"], t0
        h = C.c_void_p()
        rc = lib().fsa_plate_create(C.byref(d), C.byref(h))
        if rc != OK:
            raise FsaError(rc, "fsa_plate_create")
        self.h = h

    def _check(self, rc):
        if rc != OK:
            raise FsaError(rc, lib().fsa_plate_last_error(self.h).decode())

    def markers(self):
        X = np.empty((2, self.nm))
        U = np.empty((2, self.nm))
        self._check(lib().fsa_plate_markers(self.h, X.ctypes.data, U.ctypes.data))
        return X, U

    def step(self, F, dt):
        F = np.ascontiguousarray(F, dtype=np.float64)
        if F.shape != (2, self.nm):
            raise ValueError(f"F must have shape (2, {self.nm}), not {F.shape}")
        self._check(lib().fsa_plate_step(self.h, F.ctypes.data, dt))

    def coupled_steps(self, solver, Q, dt, nsteps, resume=True):
        """nsteps coupled fluid-plate steps in the library (fsa_plate_coupled_steps)."""
        rc = lib().fsa_plate_coupled_steps(solver.ctx, self.h, _ptr(solver._state(Q)), dt, nsteps, 1 if resume else 0)
        if rc != OK:
            raise FsaError(rc, f"coupled steps: plate: {lib().fsa_plate_last_error(self.h).decode()}; "
                               f"solver: {lib().fsa_last_error(solver.ctx).decode()}")
        return Q

    def get_state(self):
        e, v, a, t = np.empty(self.ndof), np.empty(self.ndof), np.empty(self.ndof), C.c_double()
        self._check(lib().fsa_plate_get_state(self.h, e.ctypes.data, v.ctypes.data, a.ctypes.data, C.byref(t)))
        return e, v, a, t.value

    def set_state(self, e, v, a, t):
        e, v = np.ascontiguousarray(e, dtype=np.float64), np.ascontiguousarray(v, dtype=np.float64)
        a = None if a is None else np.ascontiguousarray(a, dtype=np.float64)
        for x in (e, v) + (() if a is None else (a,)):
            if x.shape != (self.ndof,):
                raise ValueError(f"plate state arrays must have {self.ndof} entries, not {x.shape}")
        self._check(lib().fsa_plate_set_state(self.h, e.ctypes.data, v.ctypes.data,
                                              None if a is None else a.ctypes.data, t))

    def close(self):
        if getattr(self, "h", None):
            lib().fsa_plate_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def lib():
    """Load libfsa.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        if L.fsa_abi_version() != ABI_VERSION:
            raise RuntimeError(f"{LIB_PATH} has ABI version {L.fsa_abi_version()}, the binding mirrors "
                               f"{ABI_VERSION}: rebuild it with __graft_entry__.build()")
        _lib = L
    return _lib


def make_desc(case, nan_check=False) -> FsaDesc:
    d = FsaDesc()
    d.dim = case.dim
    for k in range(3):
        d.n[k] = case.n[k]
        d.lo[k] = case.lo[k]
        for s in range(2):
            d.bc[k][s] = BC[case.bc[k][s]]
            d.sponge_width[k][s] = case.sponge_width[k][s]
    d.h = case.h
    d.gamma = case.gamma
    d.mu = case.mu
    d.scheme = SCHEME[case.scheme]
    d.precision = PRECISION[case.precision]
    d.terms = case.terms
    d.nan_check = 1 if nan_check else 0
    d.selector_stride = int(case.extra.get("selector_stride", 1))
    d.src_amp = case.src_amp
    d.src_b = case.src_b
    d.src_omega = case.src_omega
    for k in range(3):
        d.src_x[k] = case.src_x[k]
    d.weno_eps = case.weno_eps
    d.teno_ct = case.teno_ct
    d.teno_eps = case.teno_eps
    for k in range(5):
        d.prim_inf[k] = case.prim_inf[k]
    d.inflow_amp = case.inflow_amp
    d.seed = case.seed
    d.sponge_sigma = case.sponge_sigma
    d.ib_alpha = case.ib_alpha
    d.ib_beta = case.ib_beta
    d.max_markers, d.max_probes, d.max_window_cells = capacities(case)
    d.variables = VARIABLES[case.variables]
    return d


class MultiBlock:
    """One domain cut into `nblocks` slabs along its last direction on the current HIP device
    and torch's current stream (include/fsa.h, fsa_mb_*): each block an ordinary context over
    its layers and FSA_HALO halo layers, halo copies and the cross-block wave-speed maximum
    after every stage; the whole state goes in with scatter and comes out with gather."""

    def __init__(self, case, nblocks, stream=None):
        import torch

        self.torch = torch
        self.case = case
        self.nq = case.dim + 2
        self.shape = (self.nq,) + case.shape
        self.nblocks = nblocks
        self.device = torch.device("cuda", torch.cuda.current_device())
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        self.desc = make_desc(case)
        nbytes = C.c_size_t()
        self._check(lib().fsa_mb_workspace_bytes(C.byref(self.desc), nblocks, C.byref(nbytes)), None)
        self.workspace = torch.empty(nbytes.value, dtype=torch.uint8, device=self.device)
        mb = C.c_void_p()
        self._check(lib().fsa_mb_init(C.byref(self.desc), nblocks, C.c_void_p(self.workspace.data_ptr()),
                                      nbytes.value, C.c_void_p(self.stream.cuda_stream), C.byref(mb)), None)
        self.mb = mb
        self.nm = 0
        if case.markers is not None:
            m = case.markers
            self.set_markers(m["X"], m["dV"], m.get("U"), m.get("motion", "static"), m.get("omega", 0.0))

    def close(self):
        if getattr(self, "mb", None):
            lib().fsa_mb_destroy(self.mb)
            self.mb = None
        self.workspace = None

    def __del__(self):
        try:
            self.close()
        except Exception:      # interpreter shutdown: the module's globals may be gone
            pass

    def _check(self, rc, mb="self"):
        if rc != OK:
            m = self.mb if mb == "self" else None
            msg = lib().fsa_mb_last_error(m).decode() if m else lib().fsa_status_str(rc).decode()
            raise FsaError(rc, msg)

    def _state(self, Q):
        t = self.torch
        if not isinstance(Q, t.Tensor) or Q.dtype != t.float64 or Q.device != self.device or not Q.is_contiguous() \
                or tuple(Q.shape) != tuple(self.shape):
            raise ValueError(f"Q must be a contiguous float64 tensor of shape {self.shape} on {self.device}")
        return Q

    def block_info(self, b):
        v = [C.c_int32() for _ in range(4)]
        self._check(lib().fsa_mb_block_info(self.mb, b, *[C.byref(x) for x in v]))
        return tuple(x.value for x in v)       # first layer, layers, halo below, halo above

    def set_markers(self, X, dV, U=None, motion="static", omega=0.0):
        dV = _host(dV)
        n = dV.shape[0]
        X = _host(X)
        if X.shape != (self.nq - 2, n):
            raise ValueError(f"X must have shape {(self.nq - 2, n)}, not {X.shape}")
        Ua = _host(U) if U is not None else None
        if Ua is not None and Ua.shape != X.shape:
            raise ValueError(f"U must have shape {X.shape}, not {Ua.shape}")
        self._check(lib().fsa_mb_set_markers(self.mb, n, X.ctypes.data, dV.ctypes.data,
                                             Ua.ctypes.data if Ua is not None else None, MOTION[motion], omega))
        self.nm = n

    def set_marker_kinematics(self, X, U=None):
        X = _host(X)
        if X.shape != (self.nq - 2, self.nm):
            raise ValueError(f"X must have shape {(self.nq - 2, self.nm)}, not {X.shape}")
        Ua = _host(U) if U is not None else None
        if Ua is not None and Ua.shape != X.shape:
            raise ValueError(f"U must have shape {X.shape}, not {Ua.shape}")
        self._check(lib().fsa_mb_set_marker_kinematics(self.mb, X.ctypes.data,
                                                       Ua.ctypes.data if Ua is not None else None))

    def scatter(self, Q):
        self._check(lib().fsa_mb_scatter(self.mb, _ptr(self._state(Q))))

    def gather(self, Q=None):
        Q = self.torch.empty(self.shape, dtype=self.torch.float64, device=self.device) if Q is None else self._state(Q)
        self._check(lib().fsa_mb_gather(self.mb, _ptr(Q)))
        return Q

    def rk3_steps(self, dt, nsteps):
        self._check(lib().fsa_mb_rk3_steps(self.mb, dt, nsteps))

    def marker_force(self):
        F = np.zeros((self.nq - 2, self.nm))
        if self.nm:
            self._check(lib().fsa_mb_marker_force(self.mb, F.ctypes.data))
        return F


def capacities(case):
    """Workspace capacities (markers, probes, window cells) for a case: case.extra's
    max_markers / max_probes / max_window_cells when given, else the case's own markers and
    probes (at least 64 each) and, for markers that do not move, the box of their supports
    with a margin (moving markers: 0, the whole grid)."""
    ex = case.extra
    m = case.markers
    nm = int(np.asarray(m["dV"]).shape[0]) if m is not None else 0
    npr = int(np.asarray(case.probes).shape[1]) if case.probes is not None else 0
    mm = int(ex.get("max_markers", max(nm, 64)))
    mp = int(ex.get("max_probes", max(npr, 64)))
    if "max_window_cells" in ex:
        mw = int(ex["max_window_cells"])
    elif nm and m.get("motion", "static") != "external":
        X = np.asarray(m["X"], dtype=np.float64).reshape(case.dim, nm)
        ext = X.max(axis=1) - X.min(axis=1)
        mw = int(np.prod(np.floor(ext / case.h) + 8))     # a support reaches 2 cells either side
    else:
        mw = 0
    return mm, mp, mw


def _host(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _ptr(t):
    return C.c_void_p(t.data_ptr())


def alpha_noalloc(case, Q, out, stream=None):
    """fsa_alpha_noalloc: the wave speeds of Q (case's grid and gas) into the device tensor
    out[3], on torch's current stream (or `stream`), with no context and no allocation."""
    import torch

    nq = case.dim + 2
    for x, shape, what in ((Q, (nq,) + case.shape, "Q"), (out, (3,), "out")):
        if not (isinstance(x, torch.Tensor) and x.dtype == torch.float64 and x.is_cuda and x.is_contiguous()
                and tuple(x.shape) == shape):
            raise ValueError(f"{what} must be a contiguous float64 CUDA tensor of shape {shape}")
    if Q.device != out.device:
        raise ValueError("Q and out must be on one device")
    st = stream if stream is not None else torch.cuda.current_stream(Q.device)
    d = make_desc(case)
    rc = lib().fsa_alpha_noalloc(C.byref(d), _ptr(Q), _ptr(out), C.c_void_p(st.cuda_stream))
    if rc != OK:
        raise FsaError(rc, "fsa_alpha_noalloc: " + lib().fsa_status_str(rc).decode())
    return out


class Solver:
    """One library context on the current HIP device and torch's current stream."""

    def __init__(self, case, nan_check=False, stream=None):
        import torch

        self.torch = torch
        self.case = case
        self.dim = case.dim
        self.nq = case.dim + 2
        self.shape = (self.nq,) + case.shape
        self.device = torch.device("cuda", torch.cuda.current_device())
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        self.desc = make_desc(case, nan_check)
        nbytes = C.c_size_t()
        self._check(lib().fsa_workspace_bytes(C.byref(self.desc), C.byref(nbytes)), None)
        # the context's device memory: a torch allocation the library carves up
        self.workspace = torch.empty(nbytes.value, dtype=torch.uint8, device=self.device)
        ctx = C.c_void_p()
        self._check(lib().fsa_init(C.byref(self.desc), C.c_void_p(self.workspace.data_ptr()), nbytes.value,
                                   C.c_void_p(self.stream.cuda_stream), C.byref(ctx)), None)
        self.ctx = ctx
        self.nm = 0
        self.np = 0
        if case.markers is not None:
            m = case.markers
            self.set_markers(m["X"], m["dV"], m.get("U"), m.get("motion", "static"), m.get("omega", 0.0))
        if case.probes is not None:
            self.set_probes(case.probes)

    def close(self):
        if getattr(self, "ctx", None):
            lib().fsa_destroy(self.ctx)     # (waits for the stream: the workspace is then free)
            self.ctx = None
        self.workspace = None

    def __del__(self):
        try:
            self.close()
        except Exception:      # interpreter shutdown: the module's globals may be gone
            pass

    def _check(self, rc, ctx="self"):
        if rc != OK:
            c = self.ctx if ctx == "self" else None
            msg = lib().fsa_last_error(c).decode() if c else lib().fsa_status_str(rc).decode()
            raise FsaError(rc, msg)

    def _dev(self, x, shape, dtype, what):
        """A device argument: a contiguous tensor of this dtype and shape on the context's
        device (anything else would let a kernel read or write outside it)."""
        t = self.torch
        if not isinstance(x, t.Tensor):
            raise ValueError(f"{what} must be a torch tensor")
        if x.dtype != dtype:
            raise ValueError(f"{what} must be {dtype}, not {x.dtype}")
        if x.device != self.device:
            raise ValueError(f"{what} must be on {self.device}, not {x.device}")
        if not x.is_contiguous():
            raise ValueError(f"{what} must be contiguous")
        if tuple(x.shape) != tuple(shape):
            raise ValueError(f"{what} must have shape {tuple(shape)}, not {tuple(x.shape)}")
        return x

    def _state(self, Q, what="Q"):
        return self._dev(Q, self.shape, self.torch.float64, what)

    # -- set-up
    def _host_shape(self, A, shape, what):
        A = _host(A)
        if tuple(A.shape) != tuple(shape):
            raise ValueError(f"{what} must have shape {tuple(shape)}, not {tuple(A.shape)}")
        return A

    def set_markers(self, X, dV, U=None, motion="static", omega=0.0):
        dV = _host(dV)
        n = dV.shape[0]
        X = self._host_shape(X, (self.nq - 2, n), "X")
        Ua = self._host_shape(U, (self.nq - 2, n), "U") if U is not None else None
        self._check(lib().fsa_set_markers(self.ctx, n, X.ctypes.data, dV.ctypes.data,
                                          Ua.ctypes.data if Ua is not None else None, MOTION[motion], omega))
        self.nm = n

    def set_marker_kinematics(self, X, U=None):
        X = self._host_shape(X, (self.nq - 2, self.nm), "X")
        Ua = self._host_shape(U, (self.nq - 2, self.nm), "U") if U is not None else None
        self._check(lib().fsa_set_marker_kinematics(self.ctx, X.ctypes.data,
                                                    Ua.ctypes.data if Ua is not None else None))

    def set_probes(self, Xp):
        Xp = _host(Xp)
        n = Xp.shape[1] if Xp.ndim == 2 else 0
        if n and Xp.shape[0] != self.nq - 2:
            raise ValueError(f"probe points must have shape ({self.nq - 2}, n), not {tuple(Xp.shape)}")
        self._check(lib().fsa_set_probes(self.ctx, n, Xp.ctypes.data))
        self.np = n

    # -- field operations (asynchronous on the stream)
    def alpha(self, Q):
        out = np.zeros(3)
        self._check(lib().fsa_alpha(self.ctx, _ptr(self._state(Q)), out.ctypes.data))
        return out

    def rhs(self, Q, out=None):
        Q = self._state(Q)
        L = self._state(out, "out") if out is not None else self.torch.empty_like(Q)
        self._check(lib().fsa_rhs(self.ctx, _ptr(Q), _ptr(L)))
        return L

    def rk3_step(self, Q, dt):
        self._check(lib().fsa_rk3_step(self.ctx, _ptr(self._state(Q)), dt))
        return Q

    def rk3_steps(self, Q, dt, nsteps):
        self._check(lib().fsa_rk3_steps(self.ctx, _ptr(self._state(Q)), dt, nsteps))
        return Q

    def rk3_steps_resume(self, Q, dt, nsteps=1):
        """Continue from the previous step call on this Q (unchanged since): see fsa.h."""
        self._check(lib().fsa_rk3_steps_resume(self.ctx, _ptr(self._state(Q)), dt, nsteps))
        return Q

    def ib_interp(self, field):
        t = self.torch
        ncomp = field.shape[0] if isinstance(field, t.Tensor) and field.dim() > 0 else 0
        if ncomp < 1:
            raise ValueError("field must be [ncomp] + grid shape with ncomp >= 1")
        field = self._dev(field, (ncomp,) + self.case.shape, t.float64, "field")
        out = t.empty((ncomp, self.nm), dtype=t.float64, device=self.device)
        self._check(lib().fsa_ib_interp(self.ctx, _ptr(field), ncomp, _ptr(out)))
        return out

    def ib_spread(self, F, field, scale=1.0):
        t = self.torch
        ncomp = F.shape[0] if isinstance(F, t.Tensor) and F.dim() > 0 else 0
        if ncomp < 1:
            raise ValueError("F must be [ncomp][markers] with ncomp >= 1")
        F = self._dev(F, (ncomp, self.nm), t.float64, "F")
        field = self._dev(field, (ncomp,) + self.case.shape, t.float64, "field")
        self._check(lib().fsa_ib_spread(self.ctx, _ptr(F), ncomp, _ptr(field), scale))
        return field

    def probe_dp(self, Q, out=None):
        t = self.torch
        Q = self._state(Q)
        dp = self._dev(out, (self.np,), t.float64, "out") if out is not None else \
            t.empty(self.np, dtype=t.float64, device=self.device)
        self._check(lib().fsa_probe_dp(self.ctx, _ptr(Q), _ptr(dp)))
        return dp

    # -- synchronising calls
    def marker_force(self):
        out = np.zeros((self.dim, self.nm))
        self._check(lib().fsa_marker_force(self.ctx, out.ctypes.data))
        return out

    def get_state(self):
        xi = np.zeros((self.dim, max(self.nm, 1)))
        t = C.c_double()
        step = C.c_int64()
        self._check(lib().fsa_get_state(self.ctx, xi.ctypes.data, C.byref(t), C.byref(step)))
        return xi[:, : self.nm], t.value, step.value

    def set_state(self, xi, t, step):
        xa = self._host_shape(xi, (self.nq - 2, self.nm), "xi") if xi is not None else None
        self._check(lib().fsa_set_state(self.ctx, xa.ctypes.data if xa is not None else None, t, step))

    def diagnostics(self, Q, dilatation=True):
        """(totals [nq] on the host, dilatation [shape] on the device or None)."""
        t = self.torch
        Q = self._state(Q)
        tot = np.zeros(self.nq)
        dil = t.empty(self.case.shape, dtype=t.float64, device=Q.device) if dilatation else None
        self._check(lib().fsa_diagnostics(self.ctx, _ptr(Q), tot.ctypes.data, _ptr(dil) if dil is not None else None))
        return tot, dil

    # -- learned selector
    def mlp_set(self, params, conf_threshold=0.8):
        p = np.ascontiguousarray(params, dtype=np.float32)
        assert p.shape == (MLP_NPARAM,)
        self._check(lib().fsa_mlp_set(self.ctx, p.ctypes.data, MLP_NPARAM, conf_threshold))

    def set_mlp_bf16(self, params, conf_threshold=0.8):
        """Parameters as BF16: a torch.bfloat16 tensor or their uint16 bit patterns."""
        t = self.torch
        if isinstance(params, t.Tensor):
            if params.dtype != t.bfloat16:
                raise ValueError("a tensor of BF16 parameters must have dtype torch.bfloat16")
            params = params.detach().cpu().contiguous().view(t.int16).numpy().view(np.uint16)
        p = np.asarray(params)
        if p.dtype != np.uint16:      # (a cast would read values as bit patterns)
            raise ValueError(f"BF16 parameters: a torch.bfloat16 tensor or uint16 bit patterns, not {p.dtype}")
        p = np.ascontiguousarray(p)
        if p.shape != (MLP_NPARAM,):
            raise ValueError(f"the network has {MLP_NPARAM} parameters, not {p.shape}")
        self._check(lib().fsa_set_mlp(self.ctx, p.ctypes.data, MLP_NPARAM, conf_threshold))

    def mlp_get(self):
        p = np.zeros(MLP_NPARAM, dtype=np.float32)
        self._check(lib().fsa_mlp_get(self.ctx, p.ctypes.data, MLP_NPARAM))
        return p

    def _feats(self, feats, labels=None):
        t = self.torch
        n = feats.shape[0] if isinstance(feats, t.Tensor) and feats.dim() == 2 else -1
        feats = self._dev(feats, (n, 16), t.float32, "feats")
        if labels is not None:
            labels = self._dev(labels, (n,), t.uint8, "labels")
        return feats, labels, n

    def mlp_forward(self, feats):
        t = self.torch
        feats, _, n = self._feats(feats)
        z = t.empty((n, 3), dtype=t.float32, device=self.device)
        self._check(lib().fsa_mlp_forward(self.ctx, _ptr(feats), feats.shape[0], _ptr(z)))
        return z

    def mlp_grad(self, feats, labels):
        t = self.torch
        feats, labels, _ = self._feats(feats, labels)
        g = t.empty(MLP_NPARAM, dtype=t.float32, device=self.device)
        loss = t.empty(1, dtype=t.float32, device=self.device)
        self._check(lib().fsa_mlp_grad(self.ctx, _ptr(feats), _ptr(labels), feats.shape[0], _ptr(g), _ptr(loss)))
        return g, loss

    def mlp_train_step(self, feats, labels, lr, loss=None):
        feats, labels, _ = self._feats(feats, labels)
        if loss is not None:
            loss = self._dev(loss, (1,), self.torch.float32, "loss")
        self._check(lib().fsa_mlp_train_step(self.ctx, _ptr(feats), _ptr(labels), feats.shape[0], lr,
                                             _ptr(loss) if loss is not None else None))

    def harvest(self, Q, keep_rate, seed, max_out):
        t = self.torch
        feats = t.empty((max(max_out, 1), 16), dtype=t.float32, device=Q.device)
        labels = t.empty(max(max_out, 1), dtype=t.uint8, device=Q.device)
        n = C.c_int64()
        self._check(lib().fsa_harvest(self.ctx, _ptr(self._state(Q)), keep_rate, seed, max_out, _ptr(feats),
                                      _ptr(labels), C.byref(n)))
        k = min(n.value, max_out)
        return feats[:k], labels[:k], n.value

    def face_flags(self, Q):
        t = self.torch
        nx, ny = self.case.n[0], self.case.n[1]
        fx = t.empty((ny, nx + 1), dtype=t.int32, device=Q.device)
        fy = t.empty((ny + 1, nx), dtype=t.int32, device=Q.device)
        self._check(lib().fsa_face_flags(self.ctx, _ptr(self._state(Q)), _ptr(fx), _ptr(fy)))
        return fx, fy

    def face_counts(self):
        """Faces per direction: x, y (and z)."""
        nx, ny, nz = self.case.n[0], self.case.n[1], self.case.n[2] if self.dim == 3 else 1
        fc = [(nx + 1) * ny * nz, nx * (ny + 1) * nz]
        return fc + ([nx * ny * (nz + 1)] if self.dim == 3 else [])

    def debug_teno_bits(self, on=True):
        """Turn the TENO5 keep-pattern read-out on (returns its device buffer [3][faces],
        int32 words) or off (fsa_debug_teno_bits)."""
        t = self.torch
        if not on:
            self._check(lib().fsa_debug_teno_bits(self.ctx, None))
            self._dbg = None
            return None
        self._dbg = t.zeros((3, sum(self.face_counts())), dtype=t.int32, device=self.device)
        self._check(lib().fsa_debug_teno_bits(self.ctx, _ptr(self._dbg)))
        return self._dbg

    def timing(self, on=True):
        self._check(lib().fsa_timing_enable(self.ctx, 1 if on else 0))

    def timing_read(self):
        ms = C.c_double()
        n = C.c_int64()
        self._check(lib().fsa_timing_read(self.ctx, C.byref(ms), C.byref(n)))
        return ms.value, n.value

    def sync(self):
        self._check(lib().fsa_sync(self.ctx))

    def stats(self):
        s = FsaStats()
        self._check(lib().fsa_stats_get(self.ctx, C.byref(s)))
        return s
