"""Seeded synthetic inputs shaped like the paper's drop and thread workloads.

This module is shared by the tests, the benchmark, the CPU oracle's callers
and the GPU binding's callers.  It holds only input recipes (initial density
profiles, their derivative with respect to the shape coefficients, seeded
noise and parameter draws, coexistence densities of the equation of state used
to pick initial densities); none of the lattice Boltzmann step's arithmetic
lives here.

Geometry: node (k, j) sits at z = k, r = j + 1/2; fields are float64[nr, nz].
"""
from dataclasses import dataclass, field
from functools import lru_cache

import numpy as np

# ---------------------------------------------------------------- geometry --


def node_coords(nz, nr):
    z = np.arange(nz, dtype=np.float64)[None, :]
    r = np.arange(nr, dtype=np.float64)[:, None] + 0.5
    return np.broadcast_to(z, (nr, nz)), np.broadcast_to(r, (nr, nz))


def legendre(l, x):
    """Legendre polynomial P_l(x) by the three-term recurrence."""
    p0 = np.ones_like(x)
    if l == 0:
        return p0
    p1 = np.array(x, dtype=np.float64)
    for k in range(1, l):
        p0, p1 = p1, ((2 * k + 1) * x * p1 - k * p0) / (k + 1)
    return p1


def tanh_profile(d, radius, rho_l, rho_g, width):
    """Liquid (rho_l) inside d < radius, gas (rho_g) outside, tanh of the given
    width in between."""
    return 0.5 * (rho_l + rho_g) - 0.5 * (rho_l - rho_g) * np.tanh((d - radius) / width)


def drop_shape(nz, nr, zc, radius, coeffs):
    """Distance d from (zc, 0), polar angle theta and the surface radius
    R_s(theta) = radius + sum_l a_l P_l(cos theta) at every node.
    ``coeffs`` maps l -> a_l (lattice units)."""
    z, r = node_coords(nz, nr)
    dz = z - zc
    d = np.sqrt(dz * dz + r * r)
    cth = np.where(d > 0, dz / np.where(d > 0, d, 1.0), 1.0)
    rs = np.full_like(d, float(radius))
    for l, a in coeffs.items():
        rs = rs + float(a) * legendre(int(l), cth)
    return d, cth, rs


def drop_density(nz, nr, zc, radius, rho_l, rho_g, width=2.0, coeffs=None):
    """Axisymmetric drop centred on the axis at z = zc (Legendre-perturbed
    sphere)."""
    d, _, rs = drop_shape(nz, nr, zc, radius, coeffs or {})
    return tanh_profile(d, rs, rho_l, rho_g, width)


def drop_density_jacobian(nz, nr, zc, radius, rho_l, rho_g, width, coeffs, ls):
    """d rho0 / d a_l for each l in ls: float64[len(ls), nr, nz]."""
    d, cth, rs = drop_shape(nz, nr, zc, radius, coeffs)
    sech2 = 1.0 / np.cosh((d - rs) / width) ** 2
    base = 0.5 * (rho_l - rho_g) / width * sech2
    return np.stack([base * legendre(int(l), cth) for l in ls])


def thread_density(nz, nr, radius, rho_l, rho_g, width=2.0, eps=0.0, mode=1):
    """Liquid thread along the axis with radius R(z) = radius*(1 + eps*cos(2 pi
    mode z / nz))."""
    z, r = node_coords(nz, nr)
    rz = radius * (1.0 + eps * np.cos(2.0 * np.pi * mode * z / nz))
    return tanh_profile(r, rz, rho_l, rho_g, width)


def uniform_noise(seed, shape, amplitude):
    """i.i.d. U(-amplitude, amplitude) from numpy's PCG64."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.uniform(-amplitude, amplitude, size=shape)


# ------------------------------------------- coexistence (input recipe) --


@lru_cache(maxsize=64)
def coexistence_densities(G, rho0=1.0):
    """(rho_gas, rho_liquid) of a flat interface from the mechanical-stability
    rule of the Shan–Chen equation of state, p = rho/3 + G/6 psi^2 with
    psi = rho0 (1 - exp(-rho/rho0)):  p(rho_g) = p(rho_l) and
    integral_{rho_g}^{rho_l} (p_0 - p) psi' / psi^2 drho = 0.
    Used only to choose initial densities near equilibrium."""
    from scipy import integrate, optimize

    def psi(x):
        return rho0 * (1.0 - np.exp(-x / rho0))

    def dpsi(x):
        return np.exp(-x / rho0)

    def p(x):
        return x / 3.0 + G / 6.0 * psi(x) ** 2

    def eqs(v):
        lg, ll = v
        a, b = np.exp(lg), np.exp(ll)
        p0 = p(a)
        area = integrate.quad(lambda x: (p0 - p(x)) * dpsi(x) / psi(x) ** 2, a, b, limit=200)[0]
        return [p(b) - p0, area]

    sol = optimize.fsolve(eqs, [np.log(0.1), np.log(2.3)], xtol=1e-13)
    return float(np.exp(sol[0])), float(np.exp(sol[1]))


@lru_cache(maxsize=1)
def _tau_table():
    import json
    import os
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "coexistence_tau.json")
    with open(path) as fh:
        return json.load(fh)


def scheme_coexistence(G, tau):
    """(rho_gas, rho_liquid) at which a flat interface settles under the
    velocity-shift scheme at coupling G and relaxation time tau: bilinear
    interpolation of the table coexistence_tau.json (flat-interface runs,
    G in [-6, -5] by 0.1, tau in [0.6, 1] by 0.05; see the script that
    writes it, tests/golden/make_coexistence_table.py).  The velocity shift
    makes these depend on tau; at tau = 1 they are close to the
    mechanical-stability values of coexistence_densities.  Raises
    ValueError outside the table or next to a (G, tau) whose interface does
    not stay finite."""
    t = _tau_table()
    gs, ts = np.array(t["G"]), np.array(t["tau"])
    if not (gs[0] - 1e-12 <= G <= gs[-1] + 1e-12 and ts[0] - 1e-12 <= tau <= ts[-1] + 1e-12):
        raise ValueError(f"(G, tau) = ({G}, {tau}) outside the coexistence table")
    i = int(min(max(np.searchsorted(gs, G) - 1, 0), len(gs) - 2))
    j = int(min(max(np.searchsorted(ts, tau) - 1, 0), len(ts) - 2))
    a = (G - gs[i]) / (gs[i + 1] - gs[i])
    b = (tau - ts[j]) / (ts[j + 1] - ts[j])
    out = []
    for key in ("rho_g", "rho_l"):
        v = t[key]
        c = [v[i][j], v[i][j + 1], v[i + 1][j], v[i + 1][j + 1]]
        if any(x is None for x in c):
            raise ValueError(f"(G, tau) = ({G}, {tau}) next to an unstable table entry")
        out.append((1 - a) * ((1 - b) * c[0] + b * c[1]) + a * ((1 - b) * c[2] + b * c[3]))
    return float(out[0]), float(out[1])


# ------------------------------------------------------------ workloads --


@dataclass
class Case:
    """One synthetic instance: grid, parameters and initial fields."""
    name: str
    nz: int
    nr: int
    G: float
    tau: float
    wall: int  # 0 no-slip, 1 free-slip
    rho: np.ndarray
    uz: np.ndarray
    ur: np.ndarray
    steps: int
    rho_l: float = 0.0
    rho_g: float = 0.0
    extra: dict = field(default_factory=dict)


def static_drop(nz=64, nr=32, radius=10.0, rho_l=2.0, rho_g=0.15, G=-5.5, tau=1.0, wall=0, steps=2000):
    """Static drop on the axis, tanh width 2 (configuration 'static drop
    64 x 32')."""
    rho = drop_density(nz, nr, nz / 2.0, radius, rho_l, rho_g, 2.0)
    z = np.zeros_like(rho)
    return Case("static_drop", nz, nr, G, tau, wall, rho, z, z.copy(), steps, rho_l, rho_g,
                {"zc": nz / 2.0, "radius": radius})


def oscillating_drop(nz=256, nr=128, radius=40.0, G=-5.5, tau=0.8, wall=0, seed=2024, steps=20000,
                     amp=0.05, noise=1e-4):
    """Drop with a P2 shape perturbation of amplitude amp*R plus seeded
    uniform noise on rho (configuration 'drop oscillation 256 x 128'),
    started at the scheme's coexistence densities for (G, tau)."""
    rho_g, rho_l = scheme_coexistence(G, tau)
    rho = drop_density(nz, nr, nz / 2.0, radius, rho_l, rho_g, 2.0, {2: amp * radius})
    rho = rho + uniform_noise(seed, rho.shape, noise)
    z = np.zeros_like(rho)
    return Case("oscillating_drop", nz, nr, G, tau, wall, rho, z, z.copy(), steps, rho_l, rho_g,
                {"zc": nz / 2.0, "radius": radius, "a2": amp * radius})


def rp_thread(nz=4096, nr=512, radius=64.0, eps=0.1, mode=1, G=-5.5, tau=0.8, wall=1, steps=50000):
    """Liquid thread with a cos(2 pi z / nz) radius perturbation of amplitude
    eps*R (configuration 'Rayleigh–Plateau 4096 x 512'), started at the
    scheme's coexistence densities for (G, tau).  tau = 0.8: at the nominal
    0.7 the thread diverges within a few hundred steps (the tau does not
    change the work per node)."""
    rho_g, rho_l = scheme_coexistence(G, tau)
    rho = thread_density(nz, nr, radius, rho_l, rho_g, 2.0, eps, mode)
    z = np.zeros_like(rho)
    return Case("rp_thread", nz, nr, G, tau, wall, rho, z, z.copy(), steps, rho_l, rho_g,
                {"radius": radius, "eps": eps, "mode": mode})


def rp_wavelength(lam, nr=450, radius=60.0, G=-6.0, tau=1.0, eps=4e-3, wall=1, steps=80000):
    """Unperturbed liquid cylinder of radius R on a lam x nr lattice (one
    wavelength, periodic in z) with the axial velocity eps sin(2 pi z / lam)
    inside the liquid, weighted by the liquid fraction (the Rayleigh–Plateau
    wavelength sweep, lam x 450, G = -6).  R = 60 and tau = 1 (nu = 1/6,
    Oh = 0.094) follow from the sweep's kappa* = 0.65 panel and Oh = 0.09."""
    rho_g, rho_l = coexistence_densities(G)
    rho = thread_density(lam, nr, radius, rho_l, rho_g, 2.0)
    z, _ = node_coords(lam, nr)
    uz = eps * np.sin(2.0 * np.pi * z / lam) * (rho - rho_g) / (rho_l - rho_g)
    return Case("rp_wavelength", lam, nr, G, tau, wall, rho, np.ascontiguousarray(uz), np.zeros_like(rho), steps,
                rho_l, rho_g, {"radius": radius, "eps": eps, "kappa": 2.0 * np.pi * radius / lam})


def adjoint_coeffs(seed, radius=40.0, ls=(2, 3, 4, 5, 6), frac=0.05):
    """Seeded Legendre coefficients a_l ~ U[-frac*R, frac*R]."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return {l: float(v) for l, v in zip(ls, rng.uniform(-frac * radius, frac * radius, size=len(ls)))}


def stable_tau_min(G):
    """Lower end of the tau range drawn for coupling G: 0.65 at G = -5.0 and
    1.0 at G = -6.0, linear in between (0.825 at -5.5).  With the oracle the
    velocity-shift Shan–Chen scheme keeps drops and threads bounded at these
    values and diverges below about 0.65 (G = -5), 0.8 (G = -5.5) and 1.0
    (G = -6)."""
    return 0.65 + 0.35 * min(1.0, max(0.0, -5.0 - G))


def ensemble(n=256, seed=7, sizes=((64, 32), (128, 64), (256, 128), (512, 256))):
    """Seeded batch of independent drops and threads of uneven sizes
    (configuration 'batched ensemble').  G ~ U[-6, -5]; tau ~ U[tau_min(G),
    1.0], where tau_min(G) is the scheme's stability limit (the workload's
    nominal range U[0.55, 1.0] diverges for most G in [-6, -5]); free-slip
    wall; each instance starts at the scheme's coexistence densities for its
    (G, tau)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    cases = []
    for k in range(n):
        nz, nr = sizes[int(rng.integers(len(sizes)))]
        G = float(rng.uniform(-6.0, -5.0))
        u = float(rng.uniform(0.0, 1.0))
        tau = stable_tau_min(G) + u * (1.0 - stable_tau_min(G))
        kind = int(rng.integers(2))
        rho_g, rho_l = scheme_coexistence(G, tau)
        if kind == 0:
            rho = drop_density(nz, nr, nz / 2.0, 0.3 * nr, rho_l, rho_g, 2.0)
        else:
            rho = thread_density(nz, nr, 0.25 * nr, rho_l, rho_g, 2.0, 0.1, 1)
        z = np.zeros_like(rho)
        cases.append(Case(f"inst{k}", nz, nr, G, tau, 1, rho, z, z.copy(), 10000, rho_l, rho_g,
                          {"kind": "drop" if kind == 0 else "thread"}))
    return cases


def random_state_fields(seed, nz, nr, rho_lo=0.3, rho_hi=2.0, u_amp=0.02):
    """Smooth-ish random density and velocity fields for parity tests: a
    low-order random Fourier mix in z and r, plus small noise, with u_r odd
    about the axis built in (u_r ~ r near r = 0)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    z, r = node_coords(nz, nr)
    rho = np.full((nr, nz), 0.5 * (rho_lo + rho_hi))
    uz = np.zeros((nr, nz))
    ur = np.zeros((nr, nz))
    for _ in range(4):
        kz = int(rng.integers(0, 4))
        kr = float(rng.uniform(0.5, 3.0))
        ph = float(rng.uniform(0, 2 * np.pi))
        amp = float(rng.uniform(-1, 1))
        mode = np.cos(2 * np.pi * kz * z / nz + ph) * np.cos(np.pi * kr * r / nr)
        rho += 0.25 * (rho_hi - rho_lo) * amp * mode
        uz += u_amp * float(rng.uniform(-1, 1)) * mode
        ur += u_amp * float(rng.uniform(-1, 1)) * np.sin(np.pi * kr * r / nr) * np.cos(2 * np.pi * kz * z / nz + ph)
    rho += rng.uniform(-0.01, 0.01, size=rho.shape)
    return np.clip(rho, rho_lo, rho_hi), uz, ur
