"""Pins of the oracle's finite-difference stencils and Shan–Chen force
against exact calculus: polynomial exactness (the stencils of Sec. II.D are
fourth-order accurate), the Taylor identity of the lattice force
(Eq. sc3dc), and fourth-order convergence of the axisymmetric extra force to
its continuum form (Eq. scaxis22)."""
import numpy as np
import pytest

import oracle as O

NG = 6


def _ext(fun, nz, nr):
    """Extended field with rows -NG..nr+NG-1 filled from fun(z, r), r the
    physical radius (row j at r = j + 1/2)."""
    rows = np.arange(-NG, nr + NG) + 0.5
    z = np.arange(nz, dtype=float)
    return fun(z[None, :], rows[:, None])


# monomials z^a r^b with a + b <= 4 and their exact derivatives
MONOMIALS = [(a, b) for a in range(5) for b in range(5) if a + b <= 4]


def _mono(a, b, z0=9.3, r0=3.1):
    f = lambda z, r: (z - z0) ** a * (r - r0) ** b
    def d(z, r, da, db):
        from math import factorial
        if da > a or db > b:
            return 0.0 * z * r
        ca = factorial(a) / factorial(a - da)
        cb = factorial(b) / factorial(b - db)
        return ca * cb * (z - z0) ** (a - da) * (r - r0) ** (b - db)
    return f, d


@pytest.mark.parametrize("a,b", MONOMIALS)
def test_stencils_exact_on_quartics(a, b):
    """Every first-derivative stencil of Sec. II.D is exact on polynomials of
    total degree <= 4; the compositions used for d_rr and d_zr are then exact
    too (interior points, away from the periodic seam)."""
    nz, nr = 24, 14
    f, d = _mono(a, b)
    E = _ext(f, nz, nr)
    for (z, r) in [(8, 5), (12, 7), (10, 4)]:
        zz, rr = float(z), r + 0.5
        assert O.stencil_point("d_r", E, z, r) == pytest.approx(d(zz, rr, 0, 1), abs=1e-9)
        assert O.stencil_point("d_z", E, z, r) == pytest.approx(d(zz, rr, 1, 0), abs=1e-9)
        assert O.stencil_point("d1_r", E, z, r) == pytest.approx(d(zz, rr, 0, 1), abs=1e-9)
        assert O.stencil_point("d_rr", E, z, r) == pytest.approx(d(zz, rr, 0, 2), abs=1e-9)
        assert O.stencil_point("d_zr", E, z, r) == pytest.approx(d(zz, rr, 1, 1), abs=1e-9)


def test_stencil_error_is_fifth_order_term():
    """On r^5 the isotropic d_r is no longer exact: the stencils stop at
    fourth order (guards a stencil that is secretly of higher order, e.g. a
    wrong weight that happens to cancel the quartic error)."""
    nz, nr = 24, 14
    E = _ext(lambda z, r: (r - 3.1) ** 5 + 0 * z, nz, nr)
    val = O.stencil_point("d_r", E, 8, 6)
    exact = 5 * (6.5 - 3.1) ** 4
    assert abs(val - exact) > 1e-3


@pytest.mark.parametrize("a,b", MONOMIALS)
def test_sc_force_taylor_identity(a, b):
    """Eq. sc3dc: sum_i W_i c_i psi(x + c_i) = c_s^2 grad psi + (c_s^4/2)
    grad(lap psi), exact for polynomials of degree <= 4 (the next term of
    the lattice sum is fifth order)."""
    nz, nr = 24, 14
    f, d = _mono(a, b)
    E = _ext(f, nz, nr)
    cs2 = 1.0 / 3.0
    for (z, r) in [(8, 5), (13, 8)]:
        zz, rr = float(z), r + 0.5
        lap_z = d(zz, rr, 3, 0) + d(zz, rr, 1, 2)
        lap_r = d(zz, rr, 2, 1) + d(zz, rr, 0, 3)
        ez = cs2 * d(zz, rr, 1, 0) + 0.5 * cs2 * cs2 * lap_z
        er = cs2 * d(zz, rr, 0, 1) + 0.5 * cs2 * cs2 * lap_r
        assert O.stencil_point("sc_z", E, z, r) == pytest.approx(ez, abs=1e-10)
        assert O.stencil_point("sc_r", E, z, r) == pytest.approx(er, abs=1e-10)


def _gaussian_drop_state(s, G):
    """State whose pseudopotential is an axisymmetric Gaussian of width s
    centred on the axis: psi = A exp(-((z - zc)^2 + r^2) / s^2)."""
    nz, nr = int(8 * s), int(4 * s)
    zc = nz / 2.0
    z = np.arange(nz, dtype=float)[None, :]
    r = (np.arange(nr) + 0.5)[:, None]
    A = 0.6
    psi = A * np.exp(-((z - zc) ** 2 + r ** 2) / s ** 2)
    rho = -np.log(1.0 - psi)  # psi = 1 - exp(-rho)
    p = O.make_params(nz, nr, G=G, tau=1.0, wall=1, axisym=1)
    f = O.equilibrium(p, rho, 0 * rho, 0 * rho)
    return p, f, z, r, zc, A


def _fsym_exact(z, r, zc, A, s, G):
    """Eq. scaxis22 in gradient form: F = -(G/2) c_s^4 psi grad(r^-1 d_r psi),
    differentiated analytically (not the expanded form of Eq. scAxisExtra)."""
    psi = A * np.exp(-((z - zc) ** 2 + r ** 2) / s ** 2)
    # q = r^-1 d_r psi = -(2/s^2) psi, hence grad q = -(2/s^2) grad psi
    dpsi_dz = -2.0 * (z - zc) / s ** 2 * psi
    dpsi_dr = -2.0 * r / s ** 2 * psi
    pre = -(G / 2.0) / 9.0 * psi
    return pre * (-2.0 / s ** 2) * dpsi_dz, pre * (-2.0 / s ** 2) * dpsi_dr


def test_axisymmetric_force_fourth_order_convergence():
    """The lattice F^{gamma,sym} converges to the continuum extra force at
    fourth order away from the axis: doubling the resolution (s) cuts the
    error of the dimensionless force s^3 F by ~16 (Sec. II.D asks for at
    least fourth order).  On the rows next to the axis the 1/r and 1/r^2
    factors amplify the truncation error, so the order there drops to about
    three; it must still converge."""
    G = -5.0
    far, near = [], []
    for s in (12.0, 24.0):
        p, f, z, r, zc, A = _gaussian_drop_state(s, G)
        fl = O.fields(p, f)
        ez, er = _fsym_exact(z, r, zc, A, s, G)
        assert np.abs(ez).max() > 0
        e = np.maximum(np.abs(fl["fsym_z"] - ez), np.abs(fl["fsym_r"] - er)) * s ** 3
        rr = np.broadcast_to(r, e.shape)
        far.append(e[rr >= s / 2].max())
        near.append(e[rr < s / 2].max())
    assert 12.0 < far[0] / far[1] < 20.0, far
    assert near[0] / near[1] > 5.5, near


def test_total_force_matches_3d_continuum():
    """Sec. II.D: 2D lattice force + F^{gamma,sym} approximates the 3D
    continuum Shan–Chen force -G c_s^2 psi grad psi - (G/2) c_s^4 psi
    grad(lap_3D psi) with lap_3D = d_zz + d_rr + r^-1 d_r.  For the Gaussian,
    lap_3D psi = psi (4 rho^2/s^4 - 6/s^2) with rho^2 = (z-zc)^2 + r^2."""
    G = -5.0
    errs = []
    for s in (6.0, 12.0):
        p, f, z, r, zc, A = _gaussian_drop_state(s, G)
        fl = O.fields(p, f)
        psi = fl["psi"]
        d2 = (z - zc) ** 2 + r ** 2
        gz = -2 * (z - zc) / s ** 2 * psi
        gr = -2 * r / s ** 2 * psi
        # grad(lap psi) with lap psi = psi * (4 d2 / s^4 - 6 / s^2)
        L = 4 * d2 / s ** 4 - 6 / s ** 2
        glz = gz * L + psi * 8 * (z - zc) / s ** 4
        glr = gr * L + psi * 8 * r / s ** 4
        cs2 = 1.0 / 3.0
        ez = -G * cs2 * psi * gz - (G / 2) * cs2 * cs2 * psi * glz
        er = -G * cs2 * psi * gr - (G / 2) * cs2 * cs2 * psi * glr
        fz = fl["fsc_z"] + fl["fsym_z"]
        fr = fl["fsc_r"] + fl["fsym_r"]
        scale = np.abs(ez).max()
        errs.append(max(np.abs(fz - ez).max(), np.abs(fr - er).max()) / scale)
    # the lattice sum's leading error is O(h^4) relative to the O(h^0) term
    assert errs[1] < 2e-3
    assert errs[0] / errs[1] > 8.0, errs


def test_ghost_mirror_parities():
    """Sec. II.E, symmetry at the axis: the oracle's fields of an
    axisymmetric state obey d_r psi -> 0 as r -> 0 (odd extension), and the
    scheme is reflection-symmetric in z, so a drop centred on a node keeps
    rho(zc + k) = rho(zc - k) and u_z(zc + k) = -u_z(zc - k)."""
    from lbm_inputs import coexistence_densities, drop_density
    G = -5.0
    p, f, z, r, zc, A = _gaussian_drop_state(6.0, G)
    fl = O.fields(p, f)
    assert np.abs(fl["dr_psi"][0]).max() < 0.6 * np.abs(fl["dr_psi"][2]).max()
    nz, nr = 48, 24
    rg, rl = coexistence_densities(G)
    rho0 = drop_density(nz, nr, 24.0, 9.0, rl, rg, 2.0, {2: 1.0})
    p = O.make_params(nz, nr, G=G, tau=1.0, wall=1, axisym=1)
    f2 = O.run(p, O.equilibrium(p, rho0, 0 * rho0, 0 * rho0), 200)
    rho, uz, ur = O.moments(p, f2)
    assert np.abs(uz).max() > 1e-4  # the drop is moving
    k = np.arange(1, nz // 2)
    assert np.allclose(rho[:, 24 + k], rho[:, 24 - k], rtol=0, atol=1e-12)
    assert np.allclose(uz[:, 24 + k], -uz[:, 24 - k], rtol=0, atol=1e-12)
    assert np.allclose(ur[:, 24 + k], ur[:, 24 - k], rtol=0, atol=1e-12)
