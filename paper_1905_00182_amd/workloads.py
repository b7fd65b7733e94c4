"""Seeded synthetic workloads: case descriptions, initial states, marker and probe sets.

This module only generates inputs.  It holds none of the solver's arithmetic (no fluxes,
reconstructions, delta weights or updates); the GPU library and the CPU oracle both take
what it builds.  The recipes follow the problem statements of the paper's validation cases
(Sec. 3.1 cylinder scattering, Sec. 3.2-3.3 cylinder in uniform flow, Sec. 3.6 sphere
scattering, Sec. 4.1 flapping plate) at the sizes of the benchmark configurations; every
random number comes from a fixed seed.

Readings taken where the paper is silent (each also listed in the design notes):
  * time step dt = CFL h / sum_d (|u_inf,d| + c_inf), CFL = 0.5, fixed at t = 0;
  * penalty constants beta = kb rho h / (3/8 dt), alpha = ka rho h / (3/8 dt^2),
    kb = 1, ka = 0.1 (the paper only calls them large positive constants, Sec. 2 Eq. (7));
  * viscosity mu = rho_inf U D / Re, with U = c_inf for the quiescent cases;
  * Gaussian pulse p' = A exp(-ln 2 r^2 / b^2), A = 1e-3 p_inf, b = 3 h, isentropic density
    rho' = p' / c_inf^2 (Sec. 3.1 gives the pressure form);
  * cubic sponge sigma_max = 20 c_inf / L_s toward the far-field state.
"""
from dataclasses import dataclass, field, replace
import math
from typing import Optional

import numpy as np

GAMMA = 1.4
TERMS_ALL = 63
TERM = {"conv_x": 1, "conv_y": 2, "conv_z": 4, "visc": 8, "ib": 16, "sponge": 32}


@dataclass
class Case:
    name: str
    dim: int
    n: tuple
    lo: tuple
    h: float
    bc: tuple
    mu: float
    scheme: str = "weno5js"
    gamma: float = GAMMA
    terms: int = TERMS_ALL
    weno_eps: float = 1e-6
    teno_ct: float = 1e-6
    teno_eps: float = 1e-40
    prim_inf: tuple = (1.0, 0.0, 0.0, 0.0, 1.0 / GAMMA)
    inflow_amp: float = 0.0
    seed: int = 190500182
    sponge_width: tuple = ((0.0, 0.0), (0.0, 0.0), (0.0, 0.0))
    sponge_sigma: float = 0.0
    ib_alpha: float = 0.0
    ib_beta: float = 0.0
    # periodic Gaussian pressure source (3D): A_p = -src_amp exp(-src_b log2 |x - src_x|^2)
    # cos(src_omega t) into the energy equation as A_p / (gamma - 1); src_amp = 0: none
    src_amp: float = 0.0
    src_b: float = 16.0
    src_omega: float = 2.0 * np.pi
    src_x: tuple = (2.0, 0.0, 0.0)
    precision: str = "fp64"
    # the variables the reconstruction acts on: "component" (the conserved components one by
    # one) or "characteristic" (the flux Jacobian's characteristic fields at each face)
    variables: str = "component"
    markers: Optional[dict] = None
    probes: Optional[np.ndarray] = None
    dt: float = 0.0
    steps: int = 0
    extra: dict = field(default_factory=dict)

    @property
    def nq(self):
        return self.dim + 2

    @property
    def shape(self):
        return tuple(reversed(self.n[: self.dim]))

    @property
    def ncell(self):
        return int(np.prod(self.n[: self.dim]))

    def with_(self, **kw):
        return replace(self, **kw)


# ---------------------------------------------------------------------------------------
# grids and states
# ---------------------------------------------------------------------------------------

def centres(case):
    """Cell-centre coordinates as arrays broadcast to the state shape (z, y, x order)."""
    axes = [case.lo[d] + (np.arange(case.n[d]) + 0.5) * case.h for d in range(case.dim)]
    grids = np.meshgrid(*reversed(axes), indexing="ij")  # (z,) y, x
    return list(reversed(grids))  # x, y (, z)


def conserved(case, rho, vel, p):
    """Primitive fields -> conserved state [rho, m_1..m_dim, E] (ideal gas)."""
    Q = np.empty((case.nq,) + case.shape)
    Q[0] = rho
    ke = np.zeros(case.shape)
    for a in range(case.dim):
        Q[1 + a] = rho * vel[a]
        ke = ke + vel[a] * vel[a]
    Q[case.dim + 1] = p / (case.gamma - 1.0) + 0.5 * rho * ke
    return Q


def uniform_state(case):
    rho = np.full(case.shape, case.prim_inf[0])
    vel = [np.full(case.shape, case.prim_inf[1 + a]) for a in range(case.dim)]
    p = np.full(case.shape, case.prim_inf[4])
    return conserved(case, rho, vel, p)


def _splitmix64(seed, ctr):
    """SplitMix64 output number ctr for a seed (uint64 numpy arrays, wrapping arithmetic)."""
    with np.errstate(over="ignore"):
        z = np.uint64(seed) + (ctr.astype(np.uint64) + np.uint64(1)) * np.uint64(0x9E3779B97F4A7C15)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        return z ^ (z >> np.uint64(31))


def seeded_uniform(seed, count):
    """count uniform numbers in [0, 1) from the counter-based SplitMix64 stream of seed."""
    r = _splitmix64(seed, np.arange(count, dtype=np.uint64))
    return (r >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)


def pulse_state(case, centre, amp_rel=1e-3, halfwidth=None):
    """Quiescent gas plus an isentropic Gaussian pressure pulse (Sec. 3.1 form)."""
    b = 3.0 * case.h if halfwidth is None else halfwidth
    xs = centres(case)
    r2 = sum((xs[d] - centre[d]) ** 2 for d in range(case.dim))
    p_inf = case.prim_inf[4]
    c2 = case.gamma * p_inf / case.prim_inf[0]
    dp = amp_rel * p_inf * np.exp(-math.log(2.0) * r2 / (b * b))
    rho = case.prim_inf[0] + dp / c2
    vel = [np.full(case.shape, case.prim_inf[1 + a]) for a in range(case.dim)]
    return conserved(case, rho, vel, p_inf + dp)


def perturbed_state(case, seed, amp=1e-3, nmodes=6, step_amp=0.0):
    """Far-field state plus seeded smooth periodic modes of relative size amp on rho, u, p,
    and optionally a jump of relative size step_amp across a seeded ellipse (to exercise the
    non-linear weights and the TENO cut-off)."""
    rng = np.random.default_rng(seed)
    xs = centres(case)
    L = [case.n[d] * case.h for d in range(case.dim)]

    def modes():
        s = np.zeros(case.shape)
        for _ in range(nmodes):
            k = rng.integers(-3, 4, size=case.dim)
            ph = rng.uniform(0, 2 * np.pi)
            a = rng.uniform(-1, 1)
            arg = sum(2 * np.pi * k[d] * (xs[d] - case.lo[d]) / L[d] for d in range(case.dim))
            s = s + a * np.sin(arg + ph)
        return s / nmodes

    rho_inf, p_inf = case.prim_inf[0], case.prim_inf[4]
    c_inf = math.sqrt(case.gamma * p_inf / rho_inf)
    rho = rho_inf * (1.0 + amp * modes())
    p = p_inf * (1.0 + amp * modes())
    vel = [case.prim_inf[1 + a] + amp * c_inf * modes() for a in range(case.dim)]
    if step_amp:
        c0 = [case.lo[d] + L[d] * rng.uniform(0.3, 0.7) for d in range(case.dim)]
        ax = [L[d] * rng.uniform(0.1, 0.25) for d in range(case.dim)]
        inside = sum(((xs[d] - c0[d]) / ax[d]) ** 2 for d in range(case.dim)) < 1.0
        rho = np.where(inside, rho * (1.0 + step_amp), rho)
        p = np.where(inside, p * (1.0 + 0.5 * step_amp), p)
    return conserved(case, rho, vel, p)


def free_stream_with_noise(case, amp, seed):
    """Uniform far-field flow with a seeded uniform +-amp perturbation on every velocity
    component of every cell (counter = 3 * cell + component on the stream seed + 1)."""
    nc = case.ncell
    r = seeded_uniform(seed + 1, 3 * nc).reshape(nc, 3)
    rho = np.full(case.shape, case.prim_inf[0])
    vel = [case.prim_inf[1 + a] + amp * (2.0 * r[:, a] - 1.0).reshape(case.shape) for a in range(case.dim)]
    p = np.full(case.shape, case.prim_inf[4])
    return conserved(case, rho, vel, p)


# ---------------------------------------------------------------------------------------
# markers and probes
# ---------------------------------------------------------------------------------------

def circle_markers(n, radius, centre=(0.0, 0.0)):
    th = 2.0 * np.pi * np.arange(n) / n
    X = np.stack([centre[0] + radius * np.cos(th), centre[1] + radius * np.sin(th)])
    dV = np.full(n, 2.0 * np.pi * radius / n)
    return X, dV


def fibonacci_sphere(n, radius, centre=(0.0, 0.0, 0.0)):
    k = np.arange(n)
    z = 1.0 - (2.0 * k + 1.0) / n
    r = np.sqrt(np.maximum(0.0, 1.0 - z * z))
    ph = k * np.pi * (3.0 - math.sqrt(5.0))
    X = np.stack([centre[0] + radius * r * np.cos(ph), centre[1] + radius * r * np.sin(ph),
                  centre[2] + radius * z])
    dV = np.full(n, 4.0 * np.pi * radius * radius / n)
    return X, dV


def ring_probes(n, radius):
    th = 2.0 * np.pi * np.arange(n) / n
    return np.stack([radius * np.cos(th), radius * np.sin(th)])


# ---------------------------------------------------------------------------------------
# case recipes
# ---------------------------------------------------------------------------------------

def _dt(case, cfl=0.5):
    c_inf = math.sqrt(case.gamma * case.prim_inf[4] / case.prim_inf[0])
    rate = sum(abs(case.prim_inf[1 + d]) + c_inf for d in range(case.dim))
    return cfl * case.h / rate


def _penalty(case, kb=1.0, ka=0.1):
    rho = case.prim_inf[0]
    beta = kb * rho * case.h / (0.375 * case.dt)
    alpha = ka * rho * case.h / (0.375 * case.dt * case.dt)
    return alpha, beta


def _finish(case):
    case = case.with_(dt=_dt(case))
    a, b = _penalty(case)
    return case.with_(ib_alpha=a, ib_beta=b)


def config1(n=128, scheme="weno5js", steps=100):
    """2D cylinder scattering: [-5,5]^2, quiescent gas, pulse at (2,0), cylinder D = 1 with
    64 markers, Re = 150, sponge layer 1 wide on every side."""
    L = 10.0
    h = L / n
    c = Case(name="c1_cylinder_scattering", dim=2, n=(n, n, 1), lo=(-5.0, -5.0, 0.0), h=h,
             bc=(("extrap", "extrap"), ("extrap", "extrap"), ("periodic", "periodic")),
             mu=1.0 / 150.0, scheme=scheme,
             sponge_width=((1.0, 1.0), (1.0, 1.0), (0.0, 0.0)), sponge_sigma=20.0, steps=steps)
    X, dV = circle_markers(64, 0.5)
    c = c.with_(markers={"X": X, "dV": dV, "U": None, "motion": "static", "omega": 0.0},
                probes=ring_probes(32, 3.0))
    return _finish(c)


def config1_state(case):
    return pulse_state(case, (2.0, 0.0))


def config2(n=2048, h=1.0 / 16.0, sponge=10.0, steps=2000, nprobe=360, rprobe=50.0):
    """2D rotating cylinder in a uniform Mach 0.2 stream: n^2 cells of size 1/16 centred on
    the cylinder (D = 1, 512 markers, surface speed 0.5 U), TENO5 with C_T = 1e-6, Re = 150,
    inflow on x- with a seeded 1e-4 U velocity perturbation, zero-gradient elsewhere, cubic
    sponge 10 wide, probes on a radius-50 ring."""
    U0 = 0.2
    L = n * h
    c = Case(name="c2_rotating_cylinder", dim=2, n=(n, n, 1), lo=(-L / 2, -L / 2, 0.0), h=h,
             bc=(("inflow", "extrap"), ("extrap", "extrap"), ("periodic", "periodic")),
             mu=U0 / 150.0, scheme="teno5", prim_inf=(1.0, U0, 0.0, 0.0, 1.0 / GAMMA),
             inflow_amp=1e-4 * U0,
             sponge_width=((sponge, sponge), (sponge, sponge), (0.0, 0.0)),
             sponge_sigma=20.0 / sponge, steps=steps)
    X, dV = circle_markers(512, 0.5)
    probes = ring_probes(nprobe, min(rprobe, 0.45 * L)) if nprobe else None
    c = c.with_(markers={"X": X, "dV": dV, "U": None, "motion": "rotating", "omega": 0.2},
                probes=probes)
    return _finish(c)


def config2_state(case):
    """Initial condition of the rotating-cylinder case: the uniform far-field stream (the
    seeded perturbation enters with the inflow)."""
    return uniform_state(case)


def config2_noisy_state(case):
    """The rotating-cylinder case with the inflow perturbation already in every cell: a
    stress input for parity tests (every face sees non-trivial TENO5 decisions)."""
    return free_stream_with_noise(case, case.inflow_amp, case.seed)


def config3(n=256, scheme="teno5", steps=500, nmark=10000, L=12.0):
    """3D sphere scattering: [-6,6]^3, quiescent gas, pulse at (2,0,0), sphere R = 0.5 with
    Fibonacci markers, Re = 100, probes on a radius-4 sphere."""
    h = L / n
    c = Case(name="c3_sphere_scattering", dim=3, n=(n, n, n), lo=(-L / 2,) * 3, h=h,
             bc=(("extrap", "extrap"),) * 3, mu=1.0 / 100.0, scheme=scheme,
             sponge_width=((1.0, 1.0),) * 3, sponge_sigma=20.0, steps=steps)
    X, dV = fibonacci_sphere(nmark, 0.5)
    P, _ = fibonacci_sphere(64, min(4.0, 0.4 * L))
    c = c.with_(markers={"X": X, "dV": dV, "U": None, "motion": "static", "omega": 0.0}, probes=P)
    return _finish(c)


def config3_state(case):
    return pulse_state(case, (2.0, 0.0, 0.0))


def config3_source(n=256, scheme="teno5", steps=500, nmark=10000, L=12.0):
    """The sphere case driven by the paper's periodic Gaussian pressure source instead of a
    pulse (Sec. 3, scattering by a stationary sphere: A = 0.01, B = 16, omega = 2 pi, source at
    x = 2, all in units of the sphere radius, the ambient density and sound speed).  With the
    sphere of radius R = 0.5 here: B / R^2, omega / R and the source at (2R, 0, 0) in grid
    units; the gas starts quiescent."""
    R = 0.5
    c = config3(n=n, scheme=scheme, steps=steps, nmark=nmark, L=L)
    return c.with_(name="c3_sphere_periodic_source", src_amp=0.01, src_b=16.0 / R**2, src_omega=2.0 * np.pi / R,
                   src_x=(2.0 * R, 0.0, 0.0))


def plate_kinematics(case, t):
    """Marker positions X [2][n] and velocities U [2][n] of the rigid plate of `config5` at
    time t (Sec. 4.1, the clamped leading edge's motion): X0(t) = (A0/2) cos(2 pi f t)
    [cos beta, sin beta] added to the edge's rest point, pitch alpha(t) = (alpha_m/2)
    sin(2 pi f t + phi) about the edge, nose up for alpha > 0, so that a marker at chord
    position s sits at X0 + s (cos alpha, -sin alpha)."""
    p = case.extra["plate"]
    w = 2.0 * math.pi * p["f"]
    s = p["s"]
    b = p["beta"]
    x0 = p["edge"][0] + 0.5 * p["A0"] * math.cos(w * t) * math.cos(b)
    y0 = p["edge"][1] + 0.5 * p["A0"] * math.cos(w * t) * math.sin(b)
    vx0 = -0.5 * p["A0"] * w * math.sin(w * t) * math.cos(b)
    vy0 = -0.5 * p["A0"] * w * math.sin(w * t) * math.sin(b)
    al = 0.5 * p["alpha_m"] * math.sin(w * t + p["phi"])
    dal = 0.5 * p["alpha_m"] * w * math.cos(w * t + p["phi"])
    X = np.stack([x0 + s * math.cos(al), y0 - s * math.sin(al)])
    U = np.stack([vx0 - s * math.sin(al) * dal, vy0 - s * math.cos(al) * dal])
    return X, U


def config5(n=1024, L=16.0, nmark=256, steps=2000, scheme="teno5"):
    """2D rigid flapping plate in a uniform stream (the prescribed-kinematics stand-in for the
    flexible foil of Sec. 4.1): [-8,8]^2, U0 = 0.1, Re = 200 on the chord, plate of chord 1
    with 256 markers clamped at its leading edge, heave amplitude A0/2 = 0.5 across the stream
    (beta = 90 degrees), pitch amplitude alpha_m/2 = 30 degrees, reduced frequency
    k = 2 pi f c / U0 = 0.8, phi = 0; inflow on x-, zero-gradient elsewhere, sponge 2 wide.
    Markers move every step (`plate_kinematics`)."""
    U0, chord = 0.1, 1.0
    h = L / n
    c = Case(name="c5_flapping_plate", dim=2, n=(n, n, 1), lo=(-L / 2, -L / 2, 0.0), h=h,
             bc=(("inflow", "extrap"), ("extrap", "extrap"), ("periodic", "periodic")),
             mu=U0 * chord / 200.0, scheme=scheme, prim_inf=(1.0, U0, 0.0, 0.0, 1.0 / GAMMA),
             sponge_width=((2.0, 2.0), (2.0, 2.0), (0.0, 0.0)), sponge_sigma=20.0 / 2.0, steps=steps)
    s = (np.arange(nmark) + 0.5) * chord / nmark
    plate = {"s": s, "edge": (-0.5 * chord, 0.0), "A0": 1.0, "beta": 0.5 * math.pi,
             "alpha_m": math.radians(60.0), "phi": 0.0, "f": 0.8 * U0 / (2.0 * math.pi * chord)}
    c = c.with_(extra={"plate": plate})
    X, _ = plate_kinematics(c, 0.0)
    c = c.with_(markers={"X": X, "dV": np.full(nmark, chord / nmark), "U": plate_kinematics(c, 0.0)[1],
                         "motion": "external", "omega": 0.0})
    return _finish(c)


def config5_flexible(n=1024, L=16.0, nmark=256, steps=2000, scheme="teno5", nel=40, mass_ratio=5.0):
    """Config 5 with the flexible plate of Sec. 4.1: the rigid case's stream, markers and
    clamped leading-edge kinematics, the plate now a structure of its own (absolute nodal
    coordinates, `nel` elements) with mass ratio m* = rho_s / (rho_f c) (5 as the paper's text
    gives it for the flexible plate; the configuration's statement is 1) and bending rigidity
    E* = K_B / (rho_f U0^2 c^3) = 1, and stretching rigidity K_S = 400 rho_f U0^2 c (not
    given: stiff enough to keep the plate within 0.5% of its length; the plate sub-steps to
    stay within the explicit stretching limit).  The markers follow the structure, which the
    fluid's marker forces load every step."""
    c = config5(n=n, L=L, nmark=nmark, steps=steps, scheme=scheme)
    U0, chord, rho = 0.1, 1.0, 1.0
    flex = {"length": chord, "nel": nel, "rho_s": mass_ratio * rho * chord, "k_s": 400.0 * rho * U0**2 * chord,
            "k_b": 1.0 * rho * U0**2 * chord**3}
    name = "c5_flexible_plate" if mass_ratio == 5.0 else f"c5_flexible_plate_m{mass_ratio:g}"
    return c.with_(name=name, extra={**c.extra, "flex": flex})


def insect_kinematics(case, t):
    """Markers of the hovering insect at time t (Sec. 3, insect in hovering flight): the body
    (static) and the two wings, rigid ellipses hinged at the body's sides and flapping
    symmetrically by alpha(t) = alpha0 [1 + sin(2 pi f t)] (upward from the horizontal).
    Returns X[2][n], U[2][n] in the order body, right wing, left wing (the left wing is the
    mirror image of the right one in x = 0)."""
    p = case.extra["insect"]
    w = 2.0 * math.pi * p["f"]
    al = p["alpha0"] * (1.0 + math.sin(w * t))
    alt = p["alpha0"] * w * math.cos(w * t)
    th = p["theta"]
    ca, sa = math.cos(al), math.sin(al)
    hx = p["hinge"]
    # right wing: centre at the hinge plus a along the wing's axis (cos al, sin al)
    cx, cy = hx + p["a"] * ca, p["a"] * sa
    ex, ey = p["a"] * np.cos(th), p["b"] * np.sin(th)
    xr = cx + ca * ex - sa * ey
    yr = cy + sa * ex + ca * ey
    ur = -alt * yr                        # rotation about the hinge (hx, 0) at rate alt
    vr = alt * (xr - hx)
    nb = len(p["body_x"])
    X = np.concatenate([np.stack([p["body_x"], p["body_y"]]), np.stack([xr, yr]), np.stack([-xr, yr])], axis=1)
    U = np.concatenate([np.zeros((2, nb)), np.stack([ur, vr]), np.stack([-ur, vr])], axis=1)
    return X, U


def insect(n=800, L=16.0, sponge=2.0, steps=2000, scheme="teno5", nprobe=64, rprobe=5.0):
    """2D hovering insect (Sec. 3): a circular body of diameter 0.5 and two elliptic wings of
    length 1 and width 0.4 (the wing length is the unit), hinged at the body's sides, in a
    quiescent fluid; Re = rho U_max / mu = 200 and M = U_max / c = 0.1 with U_max the
    reference velocity, the flapping frequency from St = f / U_max = 0.25 (the paper's wing-tip
    reading of U_max does not fit its alpha0 and St together; U_max is taken as the reference
    speed and f from St), alpha0 = 25.3 degrees; 50 cells per wing length on [-L/2, L/2]^2,
    zero-gradient sides, sponge `sponge` wide; markers about one cell apart, the wings'
    at equal parameter steps with their arc-length weights.  The markers move every step
    (`insect_kinematics`)."""
    umax = 0.1
    h = L / n
    c = Case(name="insect_hovering", dim=2, n=(n, n, 1), lo=(-L / 2, -L / 2, 0.0), h=h,
             bc=(("extrap", "extrap"), ("extrap", "extrap"), ("periodic", "periodic")),
             mu=umax / 200.0, scheme=scheme, prim_inf=(1.0, 0.0, 0.0, 0.0, 1.0 / GAMMA),
             sponge_width=((sponge, sponge), (sponge, sponge), (0.0, 0.0)), sponge_sigma=20.0 / max(sponge, 1e-9),
             steps=steps)
    rb, a, b = 0.25, 0.5, 0.2
    nb = max(8, int(round(2 * math.pi * rb / h)))
    tb = 2 * math.pi * (np.arange(nb) + 0.5) / nb
    perim = math.pi * (3 * (a + b) - math.sqrt((3 * a + b) * (a + 3 * b)))
    nw = max(8, int(round(perim / h)))
    th = 2 * math.pi * (np.arange(nw) + 0.5) / nw
    dvw = np.hypot(a * np.sin(th), b * np.cos(th)) * (2 * math.pi / nw)   # |dX/dtheta| dtheta
    ins = {"hinge": rb, "a": a, "b": b, "theta": th, "alpha0": math.radians(25.3), "f": 0.25 * umax,
           "body_x": rb * np.cos(tb), "body_y": rb * np.sin(tb)}
    c = c.with_(extra={"insect": ins})
    X, U = insect_kinematics(c, 0.0)
    dV = np.concatenate([np.full(nb, 2 * math.pi * rb / nb), dvw, dvw])
    c = c.with_(markers={"X": X, "dV": dV, "U": U, "motion": "external", "omega": 0.0},
                probes=ring_probes(nprobe, rprobe) if nprobe else None)
    return _finish(c)


def config4(n=384, steps=500):
    """Precision variant of the sphere case at 384^3 (FP32 faces, FP64 state)."""
    c = config3(n=n, scheme="teno5", steps=steps)
    return c.with_(name="c4_sphere_precision", precision="mixed32")


def periodic_box(dim=2, n=32, scheme="weno5js", mu=0.0, terms=TERMS_ALL, L=1.0, prim_inf=None):
    """Periodic box without sponge or markers, used by the invariant tests."""
    h = L / n
    nn = (n, n, n if dim == 3 else 1)
    pi = prim_inf if prim_inf is not None else (1.0, 0.0, 0.0, 0.0, 1.0 / GAMMA)
    c = Case(name=f"periodic{dim}d", dim=dim, n=nn, lo=(0.0, 0.0, 0.0), h=h,
             bc=(("periodic", "periodic"),) * 3, mu=mu, scheme=scheme, terms=terms, prim_inf=pi)
    return c.with_(dt=_dt(c))
