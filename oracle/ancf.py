"""Oracle (test infrastructure only: tests, the smoke check and the bench's CPU baseline use
it; the library never does): the flexible plate of Sec. 2's beam equation by absolute nodal
coordinates (Shabana's planar element as the paper adopts it: per node the position X and
the slope dX/ds, cubic Hermite interpolation along the arc length s), plain numpy in FP64.

The equation, with the sign reading under which both rigidities restore (the printed
bracket and signs are garbled):
    rho_s X_tt = d/ds[K_S (|X_s| - 1) X_s] - K_B X_ssss + F_f,
and its weak form over the nodal coordinates e (the clamped leading edge's four prescribed):
    M e_tt + K e + f_s(e) = Q,
    M   = int rho_s S^T S ds,      K = int K_B S''^T S'' ds,
    f_s = int K_S (|S' e| - 1) S'^T S' e ds     (five-point Gauss-Legendre per element),
    Q   = sum_k S(s_k)^T F_k dV_k              (the IB markers' forces: midpoint rule).
Time step (a reading: the paper names no scheme): Newmark's average-acceleration rule
(beta = 1/4, gamma = 1/2) with M and K implicit and the stretching force explicit at the
Newmark predictor; the fluid force is the one of the step just taken (explicit staggered
coupling, Sec. 2).  The leading edge follows the flapping kinematics of Sec. 4.1.
"""
import math

import numpy as np


def hermite(xi, l):
    """Cubic Hermite shape functions (position, slope at the left node; position, slope at
    the right node) at local coordinate xi in [0, 1] of an element of length l, and their
    first and second derivatives with respect to the arc length."""
    N = np.array([1 - 3 * xi**2 + 2 * xi**3, l * (xi - 2 * xi**2 + xi**3), 3 * xi**2 - 2 * xi**3,
                  l * (-xi**2 + xi**3)])
    dN = np.array([-6 * xi + 6 * xi**2, l * (1 - 4 * xi + 3 * xi**2), 6 * xi - 6 * xi**2,
                   l * (-2 * xi + 3 * xi**2)]) / l
    d2N = np.array([-6 + 12 * xi, l * (-4 + 6 * xi), 6 - 12 * xi, l * (-2 + 6 * xi)]) / l**2
    return N, dN, d2N


def shape_matrix(n):
    """The 2 x 8 matrix mapping an element's coordinates (node j: x, y, x_s, y_s; node j+1:
    the same) to the two components of the interpolated quantity."""
    S = np.zeros((2, 8))
    for a in range(4):
        S[0, 2 * a] = n[a]
        S[1, 2 * a + 1] = n[a]
    return S


def flapping_clamp(p):
    """Leading-edge kinematics of Sec. 4.1 for the plate dict p: X0(t) = edge + (A0/2)
    cos(2 pi f t) [cos beta, sin beta] and the slope (cos alpha, -sin alpha) with
    alpha = (alpha_m/2) sin(2 pi f t + phi) (nose up for alpha > 0), with first and second
    time derivatives."""
    w = 2.0 * math.pi * p["f"]
    b = np.array([math.cos(p["beta"]), math.sin(p["beta"])])
    edge = np.asarray(p["edge"], dtype=np.float64)

    def clamp(t):
        r = edge + 0.5 * p["A0"] * math.cos(w * t) * b
        rt = -0.5 * p["A0"] * w * math.sin(w * t) * b
        rtt = -0.5 * p["A0"] * w * w * math.cos(w * t) * b
        al = 0.5 * p["alpha_m"] * math.sin(w * t + p["phi"])
        alt = 0.5 * p["alpha_m"] * w * math.cos(w * t + p["phi"])
        altt = -0.5 * p["alpha_m"] * w * w * math.sin(w * t + p["phi"])
        d = np.array([math.cos(al), -math.sin(al)])
        dp = np.array([-math.sin(al), -math.cos(al)])      # d(d)/d(alpha)
        dt_ = dp * alt
        dtt = -d * alt * alt + dp * altt
        return r, d, rt, dt_, rtt, dtt

    return clamp


class Plate:
    """A plate of length `length` in `nel` elements, linear density rho_s, rigidities k_s and
    k_b, loaded through markers at arc positions s_mark with weights dv_mark, its leading edge
    (s = 0) clamped to `clamp(t)` -> (position, slope, their velocities, their accelerations);
    straight along the clamp's slope and moving with it at t = t0."""

    def __init__(self, length, nel, rho_s, k_s, k_b, s_mark, dv_mark, clamp, t0=0.0):
        self.L, self.nel, self.l = float(length), int(nel), float(length) / nel
        self.rho_s, self.k_s, self.k_b = float(rho_s), float(k_s), float(k_b)
        self.s_mark = np.asarray(s_mark, dtype=np.float64)
        self.dv_mark = np.asarray(dv_mark, dtype=np.float64)
        self.clamp = clamp
        self.ndof = 4 * (self.nel + 1)
        x, w = np.polynomial.legendre.leggauss(5)
        self.gx, self.gw = 0.5 * (x + 1.0), 0.5 * w            # on [0, 1]
        self.M = np.zeros((self.ndof, self.ndof))
        self.K = np.zeros((self.ndof, self.ndof))
        for j in range(self.nel):
            sl = slice(4 * j, 4 * j + 8)
            for xi, wq in zip(self.gx, self.gw):
                N, _, d2N = hermite(xi, self.l)
                S, S2 = shape_matrix(N), shape_matrix(d2N)
                self.M[sl, sl] += self.rho_s * self.l * wq * (S.T @ S)
                self.K[sl, sl] += self.k_b * self.l * wq * (S2.T @ S2)
        self.t = float(t0)
        r, d, rt, dt_, rtt, dtt = clamp(self.t)
        self.e = np.zeros(self.ndof)
        self.v = np.zeros(self.ndof)
        for i in range(self.nel + 1):
            s = i * self.l
            self.e[4 * i:4 * i + 2] = r + s * d
            self.e[4 * i + 2:4 * i + 4] = d
            self.v[4 * i:4 * i + 2] = rt + s * dt_
            self.v[4 * i + 2:4 * i + 4] = dt_
        # largest stretching frequency of the unstretched plate, bounded by an element's:
        # K_S int dN dN^T ds against the element mass, per coordinate
        ke = np.zeros((4, 4))
        me = np.zeros((4, 4))
        for xi, wq in zip(self.gx, self.gw):
            N, dN, _ = hermite(xi, self.l)
            ke += self.k_s * self.l * wq * np.outer(dN, dN)
            me += self.rho_s * self.l * wq * np.outer(N, N)
        self.omega_s = math.sqrt(max(np.linalg.eigvals(np.linalg.solve(me, ke)).real)) if self.k_s > 0 else 0.0
        # initial acceleration of the free coordinates: no load
        f = self.stretch_force(self.e)
        ap = np.concatenate([rtt, dtt])
        self.a = np.zeros(self.ndof)
        self.a[:4] = ap
        rhs = -(f + self.K @ self.e)[4:] - self.M[4:, :4] @ ap
        self.a[4:] = np.linalg.solve(self.M[4:, 4:], rhs)
        self._dt = None

    def set_state(self, e, v, t, a=None):
        """Checkpoint restore: coordinates, their velocities and the time; the accelerations
        as given, else from the equation without load."""
        self.e, self.v, self.t = np.array(e, dtype=np.float64), np.array(v, dtype=np.float64), float(t)
        if a is not None:
            self.a = np.array(a, dtype=np.float64)
            return self
        r, d, rt, dt_, rtt, dtt = self.clamp(self.t)
        ap = np.concatenate([rtt, dtt])
        self.a = np.zeros(self.ndof)
        self.a[:4] = ap
        rhs = -(self.stretch_force(self.e) + self.K @ self.e)[4:] - self.M[4:, :4] @ ap
        self.a[4:] = np.linalg.solve(self.M[4:, 4:], rhs)
        return self

    def stretch_force(self, e):
        """f_s(e) = int K_S (|X_s| - 1) S'^T X_s ds, five Gauss points per element."""
        f = np.zeros(self.ndof)
        for j in range(self.nel):
            sl = slice(4 * j, 4 * j + 8)
            for xi, wq in zip(self.gx, self.gw):
                _, dN, _ = hermite(xi, self.l)
                S1 = shape_matrix(dN)
                xs = S1 @ e[sl]
                f[sl] += self.k_s * self.l * wq * (math.hypot(xs[0], xs[1]) - 1.0) * (S1.T @ xs)
        return f

    def _locate(self, s):
        j = min(int(s / self.l), self.nel - 1)
        return j, s / self.l - j

    def load(self, F):
        """Q = sum_k S(s_k)^T F_k dV_k for marker forces F[2][n]."""
        Q = np.zeros(self.ndof)
        for k, s in enumerate(self.s_mark):
            j, xi = self._locate(s)
            N, _, _ = hermite(xi, self.l)
            Q[4 * j:4 * j + 8] += shape_matrix(N).T @ (np.asarray(F)[:, k] * self.dv_mark[k])
        return Q

    def markers(self):
        """Marker positions and velocities [2][n]: S(s_k) e and S(s_k) e_t."""
        X = np.zeros((2, len(self.s_mark)))
        U = np.zeros_like(X)
        for k, s in enumerate(self.s_mark):
            j, xi = self._locate(s)
            N, _, _ = hermite(xi, self.l)
            S = shape_matrix(N)
            X[:, k] = S @ self.e[4 * j:4 * j + 8]
            U[:, k] = S @ self.v[4 * j:4 * j + 8]
        return X, U

    SUBSTEP_LIMIT = 1.9

    def step(self, F, dt):
        """Advance by dt under the marker forces F[2][n] (force per unit length on the plate):
        n equal sub-steps under the same forces, n the least with (dt / n) omega_s < 1.9, so
        that each keeps the explicit stretching force within its stability limit 2."""
        n = max(1, math.ceil(float(dt) * self.omega_s / self.SUBSTEP_LIMIT))
        for _ in range(n):
            self._newmark(F, float(dt) / n)
        return self

    def _newmark(self, F, dt):
        """One Newmark step of size dt (average acceleration, stretching force explicit)."""
        beta, gamma = 0.25, 0.5
        et = self.e + dt * self.v + dt * dt * (0.5 - beta) * self.a     # predictors
        vt = self.v + dt * (1.0 - gamma) * self.a
        t1 = self.t + dt
        r, d, rt, dt_, rtt, dtt = self.clamp(t1)
        ep, vp, ap = np.concatenate([r, d]), np.concatenate([rt, dt_]), np.concatenate([rtt, dtt])
        Q = self.load(F) - self.stretch_force(et)
        A = self.M[4:, 4:] + beta * dt * dt * self.K[4:, 4:]
        rhs = Q[4:] - self.M[4:, :4] @ ap - self.K[4:, 4:] @ et[4:] - self.K[4:, :4] @ ep
        af = np.linalg.solve(A, rhs)
        self.e[4:] = et[4:] + beta * dt * dt * af
        self.v[4:] = vt[4:] + gamma * dt * af
        self.a[4:] = af
        self.e[:4], self.v[:4], self.a[:4] = ep, vp, ap
        self.t = t1
        return self
