"""ctypes wrapper of the FP64 CPU oracle (oracle/ora.c).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's CPU-baseline
leg are the only users.  It imports nothing from the GPU package; a case is passed in as any
object carrying the fields of ``ora_desc`` plus optional markers and probes (see ``Oracle``).
"""
import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libora.so")

BC = {"periodic": 0, "extrap": 1, "inflow": 2, "nonreflect": 3}
SCHEME = {"weno5js": 0, "teno5": 1}
VARIABLES = {"component": 0, "characteristic": 1}
MOTION = {"static": 0, "rotating": 1, "external": 2}
TERMS = {"conv_x": 1, "conv_y": 2, "conv_z": 4, "visc": 8, "ib": 16, "sponge": 32, "all": 63}


class OraDesc(C.Structure):
    _fields_ = [
        ("dim", C.c_int32),
        ("n", C.c_int32 * 3),
        ("lo", C.c_double * 3),
        ("h", C.c_double),
        ("bc", (C.c_int32 * 2) * 3),
        ("gamma", C.c_double),
        ("mu", C.c_double),
        ("scheme", C.c_int32),
        ("terms", C.c_int32),
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
        ("src_amp", C.c_double),
        ("src_b", C.c_double),
        ("src_omega", C.c_double),
        ("src_x", C.c_double * 3),
        ("charwise", C.c_int32),
    ]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            from .build import build

            build()
        _lib = C.CDLL(LIB_PATH)
        P = C.POINTER
        d, i64, vp = C.c_double, C.c_int64, C.c_void_p
        dp = P(C.c_double)
        _lib.ora_create.restype = vp
        _lib.ora_create.argtypes = [P(OraDesc)]
        _lib.ora_destroy.argtypes = [vp]
        _lib.ora_set_markers.argtypes = [vp, C.c_int, dp, dp, dp, C.c_int, d]
        _lib.ora_set_marker_kinematics.argtypes = [vp, dp, dp]
        _lib.ora_set_probes.argtypes = [vp, C.c_int, dp]
        _lib.ora_alpha.argtypes = [vp, dp, dp]
        _lib.ora_rhs.argtypes = [vp, dp, dp]
        _lib.ora_rhs_cells.argtypes = [vp, dp, i64, P(C.c_int64), dp]
        _lib.ora_rk3_step.argtypes = [vp, dp, d]
        _lib.ora_ib_interp.argtypes = [vp, dp, C.c_int, dp]
        _lib.ora_ib_spread.argtypes = [vp, dp, C.c_int, dp, d]
        _lib.ora_probe_dp.argtypes = [vp, dp, dp]
        _lib.ora_marker_force.argtypes = [vp, dp]
        _lib.ora_get_state.argtypes = [vp, dp, dp, P(C.c_int64)]
        _lib.ora_set_state.argtypes = [vp, dp, d, i64]
        _lib.ora_teno_flags_n.argtypes = [dp, C.c_long, d, d, vp]
        _lib.ora_threads.argtypes = [C.c_int]
        _lib.ora_record_stages.argtypes = [vp, vp]
        _lib.ora_char_vectors.argtypes = [vp, dp, dp, C.c_int, dp, dp]
        _lib.ora_teno_bits.argtypes = [vp, dp, vp]
        _lib.ora_teno_values_n.argtypes = [vp, dp, dp, C.c_long, vp, vp, vp, dp, dp]
        _lib.ora_delta4.restype = d
        _lib.ora_delta4.argtypes = [d]
        _lib.ora_recon5.restype = d
        _lib.ora_recon5.argtypes = [d, d, d, d, d, C.c_int, d, d, d]
        _lib.ora_teno_flags.restype = C.c_int
        _lib.ora_teno_flags.argtypes = [d, d, d, d, d, d, d]
        _lib.ora_face_features.argtypes = [vp, dp, C.c_int, C.c_long, C.c_long, C.c_long, C.c_int, dp]
        _lib.ora_face_features.restype = C.c_int
        _lib.ora_face_label.argtypes = [vp, dp, C.c_int, C.c_long, C.c_long, C.c_long, C.c_int, d]
        _lib.ora_face_label.restype = C.c_int
        _lib.ora_totals.argtypes = [vp, dp, dp]
        _lib.ora_totals.restype = C.c_int
        _lib.ora_dilatation.argtypes = [vp, dp, dp]
        _lib.ora_dilatation.restype = C.c_int
        _lib.ora_face_significant.argtypes = [vp, dp, C.c_int, C.c_long, C.c_long, C.c_long, C.c_int]
        _lib.ora_face_significant.restype = C.c_int
        _lib.ora_splitmix64.restype = C.c_uint64
        _lib.ora_splitmix64.argtypes = [C.c_uint64, C.c_uint64]
        for name in ("ora_set_markers", "ora_set_probes", "ora_alpha", "ora_rhs", "ora_rhs_cells",
                     "ora_rk3_step", "ora_ib_interp", "ora_ib_spread", "ora_probe_dp",
                     "ora_marker_force", "ora_get_state", "ora_set_state"):
            getattr(_lib, name).restype = C.c_int
    return _lib


def _ptr(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def delta4(r):
    return lib().ora_delta4(float(r))


def recon5(v, scheme="weno5js", weno_eps=1e-6, teno_ct=1e-6, teno_eps=1e-40):
    a, b, c, d, e = (float(x) for x in v)
    return lib().ora_recon5(a, b, c, d, e, SCHEME[scheme], weno_eps, teno_ct, teno_eps)


def teno_flags(v, teno_ct=1e-6, teno_eps=1e-40):
    a, b, c, d, e = (float(x) for x in v)
    return lib().ora_teno_flags(a, b, c, d, e, teno_ct, teno_eps)


def threads(n=0):
    """Set the oracle's OpenMP thread count (n >= 1) and return the count in effect."""
    return lib().ora_threads(int(n))


def teno_flags_n(V, teno_ct=1e-6, teno_eps=1e-40):
    """teno_flags of every row of V [n][5]."""
    V = np.ascontiguousarray(V, dtype=np.float64).reshape(-1, 5)
    out = np.zeros(V.shape[0], dtype=np.int32)
    lib().ora_teno_flags_n(_ptr(V), V.shape[0], teno_ct, teno_eps, out.ctypes.data)
    return out


def splitmix64(seed, ctr):
    return lib().ora_splitmix64(seed, ctr)


def make_desc(case) -> OraDesc:
    d = OraDesc()
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
    d.terms = case.terms
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
    d.src_amp = case.src_amp
    d.src_b = case.src_b
    d.src_omega = case.src_omega
    for a in range(3):
        d.src_x[a] = case.src_x[a]
    d.charwise = VARIABLES[case.variables]
    return d


class Oracle:
    """One oracle context: grid, scheme, markers, probes, penalty integral, time and step."""

    def __init__(self, case):
        self.case = case
        self.desc = make_desc(case)
        self.ctx = lib().ora_create(C.byref(self.desc))
        if not self.ctx:
            raise ValueError("oracle rejected the descriptor")
        self.dim = case.dim
        self.nq = case.dim + 2
        self.shape = tuple(reversed(case.n[: case.dim]))  # (ny, nx) or (nz, ny, nx)
        self.nm = 0
        self.np = 0
        if getattr(case, "markers", None) is not None:
            m = case.markers
            self.set_markers(m["X"], m["dV"], m.get("U"), m.get("motion", "static"), m.get("omega", 0.0))
        if getattr(case, "probes", None) is not None:
            self.set_probes(case.probes)

    def __del__(self):
        if getattr(self, "ctx", None):
            lib().ora_destroy(self.ctx)
            self.ctx = None

    def _check(self, rc, what):
        if rc != 0:
            raise ValueError(f"oracle {what} failed ({rc})")

    def set_markers(self, X, dV, U=None, motion="static", omega=0.0):
        X = _f64(X)
        dV = _f64(dV)
        n = dV.shape[0]
        Ua = _f64(U) if U is not None else None
        Up = _ptr(Ua) if Ua is not None else None
        self._check(lib().ora_set_markers(self.ctx, n, _ptr(X), _ptr(dV), Up, MOTION[motion], omega),
                    "set_markers")
        self.nm = n

    def set_marker_kinematics(self, X, U=None):
        X = _f64(X)
        Ua = _f64(U) if U is not None else None
        self._check(lib().ora_set_marker_kinematics(self.ctx, _ptr(X), _ptr(Ua) if Ua is not None else None),
                    "set_marker_kinematics")

    def set_probes(self, Xp):
        Xp = _f64(Xp)
        n = Xp.shape[1] if Xp.ndim == 2 else 0
        self._check(lib().ora_set_probes(self.ctx, n, _ptr(Xp)), "set_probes")
        self.np = n

    def _state(self, Q):
        Q = _f64(Q)
        assert Q.shape == (self.nq,) + self.shape, Q.shape
        return Q

    def alpha(self, Q):
        Q = self._state(Q)
        out = np.zeros(3)
        self._check(lib().ora_alpha(self.ctx, _ptr(Q), _ptr(out)), "alpha")
        return out

    def rhs(self, Q):
        Q = self._state(Q)
        L = np.empty_like(Q)
        self._check(lib().ora_rhs(self.ctx, _ptr(Q), _ptr(L)), "rhs")
        return L

    def rhs_cells(self, Q, cells):
        Q = self._state(Q)
        cells = np.ascontiguousarray(cells, dtype=np.int64)
        out = np.empty((self.nq, cells.shape[0]))
        self._check(lib().ora_rhs_cells(self.ctx, _ptr(Q), cells.shape[0],
                                        cells.ctypes.data_as(C.POINTER(C.c_int64)), _ptr(out)),
                    "rhs_cells")
        return out

    def rk3_step(self, Q, dt):
        """Advance Q (a float64 array, modified in place and returned) by one step."""
        assert Q.dtype == np.float64 and Q.flags.c_contiguous
        self._check(lib().ora_rk3_step(self.ctx, _ptr(Q), dt), "rk3_step")
        return Q

    def ib_interp(self, field):
        field = _f64(field)
        ncomp = field.shape[0]
        out = np.empty((ncomp, self.nm))
        self._check(lib().ora_ib_interp(self.ctx, _ptr(field), ncomp, _ptr(out)), "ib_interp")
        return out

    def ib_spread(self, F, field, scale=1.0):
        F = _f64(F)
        assert field.dtype == np.float64 and field.flags.c_contiguous
        self._check(lib().ora_ib_spread(self.ctx, _ptr(F), F.shape[0], _ptr(field), scale), "ib_spread")
        return field

    def probe_dp(self, Q):
        Q = self._state(Q)
        out = np.empty(self.np)
        self._check(lib().ora_probe_dp(self.ctx, _ptr(Q), _ptr(out)), "probe_dp")
        return out

    def face_features(self, Q, d, idx, side):
        """15 features of one face side; idx = (i, j[, k]) of the cell left of the face."""
        Q = self._state(Q)
        out = np.empty(15)
        i, j = idx[0], idx[1]
        k = idx[2] if len(idx) > 2 else 0
        self._check(lib().ora_face_features(self.ctx, _ptr(Q), d, i, j, k, side, _ptr(out)), "face_features")
        return out

    def face_label(self, Q, d, idx, side, alpha):
        Q = self._state(Q)
        i, j = idx[0], idx[1]
        k = idx[2] if len(idx) > 2 else 0
        r = lib().ora_face_label(self.ctx, _ptr(Q), d, i, j, k, side, alpha)
        if r < 0:
            raise ValueError("face_label failed")
        return r

    def totals(self, Q):
        """sum over cells of q_m h^dim, per component."""
        Q = self._state(Q)
        out = np.empty(self.nq)
        self._check(lib().ora_totals(self.ctx, _ptr(Q), _ptr(out)), "totals")
        return out

    def dilatation(self, Q):
        """div u at every cell (fourth-order central differences)."""
        Q = self._state(Q)
        out = np.empty(Q.shape[1:])
        self._check(lib().ora_dilatation(self.ctx, _ptr(Q), _ptr(out)), "dilatation")
        return out

    def face_significant(self, Q, d, idx, side):
        """True when some primitive variable of the side's five cells varies by more than
        1e-8 of its natural scale."""
        Q = self._state(Q)
        i, j = idx[0], idx[1]
        k = idx[2] if len(idx) > 2 else 0
        r = lib().ora_face_significant(self.ctx, _ptr(Q), d, i, j, k, side)
        if r < 0:
            raise ValueError("face_significant failed")
        return bool(r)

    def marker_force(self):
        out = np.empty((self.dim, self.nm))
        self._check(lib().ora_marker_force(self.ctx, _ptr(out)), "marker_force")
        return out

    def char_vectors(self, qa, qb, direction):
        """Left rows L[nq][nq] and right columns R[nq][nq] of the characteristic-wise
        reconstruction at the Roe average of the conserved states qa, qb along `direction`."""
        qa = np.ascontiguousarray(qa, dtype=np.float64)
        qb = np.ascontiguousarray(qb, dtype=np.float64)
        L = np.zeros((self.nq, self.nq))
        R = np.zeros((self.nq, self.nq))
        rc = lib().ora_char_vectors(self.ctx, _ptr(qa), _ptr(qb), direction, _ptr(L), _ptr(R))
        if rc != 0:
            raise ValueError("ora_char_vectors failed")
        return L, R

    # -- test hooks on the TENO5 decisions
    def record_stages(self, on=True):
        """While on, rk3_step copies each stage's input state into self.stage_states
        [3][nq][...] (a fresh array per call of this method)."""
        if on:
            self.stage_states = np.zeros((3, self.nq) + self.shape)
            lib().ora_record_stages(self.ctx, self.stage_states.ctypes.data)
        else:
            lib().ora_record_stages(self.ctx, None)

    def face_counts(self):
        n = list(self.case.n[: self.dim]) + [1] * (3 - self.dim)
        return [int(np.prod([n[a] + (a == d) for a in range(3)])) for d in range(self.dim)]

    def teno_bits(self, Q):
        """Keep patterns of every face of Q (uint32, directions concatenated)."""
        Q = self._state(Q)
        out = np.zeros(sum(self.face_counts()), dtype=np.uint32)
        self._check(lib().ora_teno_bits(self.ctx, _ptr(Q), out.ctypes.data), "teno_bits")
        return out

    def teno_values(self, Q, faces, comps, sides, alpha=None):
        """For entries (face index in teno_bits' layout, component, side): the five split-flux
        values [n][5] and chi [n][3], at Q's wave speeds (or the given alpha[3])."""
        Q = self._state(Q)
        a = _f64(self.alpha(Q) if alpha is None else alpha)
        g = np.ascontiguousarray(faces, dtype=np.int64)
        m = np.ascontiguousarray(comps, dtype=np.int32)
        sd = np.ascontiguousarray(sides, dtype=np.int32)
        v, chi = np.zeros((g.size, 5)), np.zeros((g.size, 3))
        self._check(lib().ora_teno_values_n(self.ctx, _ptr(Q), _ptr(a), g.size, g.ctypes.data, m.ctypes.data,
                                            sd.ctypes.data, _ptr(v), _ptr(chi)), "teno_values")
        return v, chi

    def get_state(self):
        xi = np.empty((self.dim, max(self.nm, 1)))
        t = C.c_double()
        step = C.c_int64()
        self._check(lib().ora_get_state(self.ctx, _ptr(xi), C.byref(t), C.byref(step)), "get_state")
        return xi[:, : self.nm], t.value, step.value

    def set_state(self, xi, t, step):
        xi = _f64(xi) if xi is not None else np.zeros((self.dim, max(self.nm, 1)))
        self._check(lib().ora_set_state(self.ctx, _ptr(xi), t, step), "set_state")
