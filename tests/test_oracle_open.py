"""Pins of the oracle's closed z ends (no-slip discs) and open rows
(imposed-equilibrium inlet and outlet, Sec. II.E) against closed-form flows
and exact invariants.

The radial flow between two parallel discs (Sec. III) has the steady
solution u_r = U2 (4 R_i / H^2) z (H - z) / r with U2 = 3 Q / (4 pi R_i H);
the paper runs it on 32 x 120 with R_i = 9.5, R = N_r - 1/2, H = N_z,
rho = 1, nu = 0.167 (tau = 1) and Q = 0.5 (U2 = 3.93e-4).  Nodes sit at
z = k + 1/2 from the first disc (walls half-way to the ghost nodes)."""
import numpy as np
import pytest

import oracle as O
from lbm_inputs import coexistence_densities, drop_density

NZ, NR, H, RI, Q = 32, 120, 32.0, 9.5, 0.5
U2 = 3.0 * Q / (4.0 * np.pi * RI * H)


def _disc_flow(steps, axisym=1):
    zp = np.arange(NZ) + 0.5
    ur_in = U2 * (4.0 * RI / H ** 2) * zp * (H - zp) / RI
    p = O.make_params(NZ, NR, G=0.0, tau=1.0, wall=0, axisym=axisym, flags=O.FLAG_ZWALLS, in_row=9, out_row=NR - 1,
                      rho_in=1.0, rho_out=1.0, uz_in=np.zeros(NZ), ur_in=ur_in)
    one = np.ones((NR, NZ))
    f = O.run(p, O.equilibrium(p, one, 0 * one, 0 * one), steps)
    return p, f, zp, ur_in


def test_paper_u2_value():
    """U2 = 3Q/(4 pi R_i H) reproduces the printed 3.93e-4."""
    assert U2 == pytest.approx(3.93e-4, abs=5e-7)


def test_radial_flow_between_discs_matches_closed_form():
    """Steady state (10 000 steps; the last 1000 change u_r by < 1e-6 U2):
    - u_r is within 3 % of U2 of the closed form on every row of the domain
      (the equilibrium inlet passes 2.5 % less than the nominal flux: the
      populations the first interior row sends back are overwritten);
    - scaled to the measured flux, it is within 0.5 % of U2 on the developed
      rows 20..100 (the z-parabola and the 1/r decay);
    - the radial mass flux sum_z 2 pi r rho u_r is the same on every row to
      1 % (continuity) and within 3 % of the imposed Q;
    - u_z stays below 2 % of U2, and the flow is mirror-symmetric about the
      mid-plane between the discs."""
    p, f, zp, _ = _disc_flow(9000)
    _, _, ur_prev = O.moments(p, f)
    f = O.run(p, f, 1000)
    rho, uz, ur = O.moments(p, f)
    assert np.abs(ur - ur_prev).max() < 1e-6 * U2
    r = np.arange(NR) + 0.5
    exact = U2 * (4.0 * RI / H ** 2) * zp[None, :] * (H - zp[None, :]) / r[:, None]
    dom = slice(10, NR - 1)
    assert np.abs(ur[dom] - exact[dom]).max() < 0.03 * U2
    flux = 2.0 * np.pi * r * (rho * ur).sum(axis=1)
    assert flux[dom].max() / flux[dom].min() - 1.0 < 0.01
    assert abs(flux[dom].mean() / Q - 1.0) < 0.03
    dev = slice(20, 100)
    scaled = exact * flux[dom].mean() / Q
    assert np.abs(ur[dev] - scaled[dev]).max() < 0.005 * U2
    assert np.abs(uz[dom]).max() < 0.02 * U2
    assert np.abs(ur - ur[:, ::-1]).max() < 1e-14 and np.abs(uz + uz[:, ::-1]).max() < 1e-14


def test_planar_channel_between_discs_is_poiseuille():
    """Planar mode (no axisymmetric terms) with the same walls and open rows
    is plane Poiseuille flow between plates: once developed (rows 40..100)
    the profile is the inlet parabola scaled to the measured flux, within
    0.5 % of its peak, and the pressure p = rho c_s^2 falls along r at
    dp/dr = -12 mu U / H^2 (U the mean velocity), within 2 %."""
    p, f, zp, ur_in = _disc_flow(12000, axisym=0)
    rho, uz, ur = O.moments(p, f)
    flux = (rho * ur).sum(axis=1)
    dev = slice(40, 100)
    shape = ur_in[None, :] * flux[dev, None] / ur_in.sum()
    assert np.abs(ur[dev] - shape).max() < 0.005 * ur_in.max()
    mean_u = flux[dev].mean() / NZ
    mu = 1.0 / 3.0 * (p.tau - 0.5)
    dp = np.polyfit(np.arange(40, 100), rho[dev].mean(axis=1) / 3.0, 1)[0]
    assert dp == pytest.approx(-12.0 * mu * mean_u / H ** 2, rel=0.02)


@pytest.mark.parametrize("wall", [0, 1])
def test_closed_box_conserves_mass_and_mirror_symmetry(wall):
    """A planar Shan–Chen drop in a box closed by the z walls and the outer
    wall: every link is a permutation of the populations, so sum rho is
    conserved to rounding; a drop centred between the z walls stays
    mirror-symmetric about the centre plane (axisymmetric run) to rounding."""
    G = -5.5
    rg, rl = coexistence_densities(G)
    nz, nr = 40, 24
    rho = drop_density(nz, nr, (nz - 1) / 2.0, 9.0, rl, rg)
    z0 = np.zeros_like(rho)
    p = O.make_params(nz, nr, G=G, tau=1.0, wall=wall, axisym=0, flags=O.FLAG_ZWALLS)
    f0 = O.equilibrium(p, rho, z0, z0)
    f = O.run(p, f0, 400)
    m0, m1 = O.moments(p, f0)[0].sum(), O.moments(p, f)[0].sum()
    assert abs(m1 / m0 - 1.0) < 1e-13
    pa = O.make_params(nz, nr, G=G, tau=1.0, wall=wall, axisym=1, flags=O.FLAG_ZWALLS)
    ra, uza, ura = O.moments(pa, O.run(pa, O.equilibrium(pa, rho, z0, z0), 400))
    assert np.abs(ra - ra[:, ::-1]).max() < 1e-12
    assert np.abs(uza + uza[:, ::-1]).max() < 1e-13 and np.abs(ura - ura[:, ::-1]).max() < 1e-13


def test_open_row_validation():
    """Rows out of range, an outlet at or below the inlet, and an inlet
    without a velocity profile are rejected."""
    one = np.ones((NR, NZ))
    for kw in (dict(in_row=NR), dict(out_row=0), dict(in_row=50, out_row=40, ur_in=np.zeros(NZ))):
        p = O.make_params(NZ, NR, G=0.0, **kw)
        with pytest.raises(ValueError):
            O.run(p, O.equilibrium(p, one, 0 * one, 0 * one), 1)
    p = O.make_params(NZ, NR, G=0.0, in_row=5)
    p.uz_in = None
    with pytest.raises(ValueError):
        O.run(p, O.equilibrium(p, one, 0 * one, 0 * one), 1)
