"""Pins of the oracle's Guo forcing option (the force incorporation of Guo,
Zheng and Shi, Phys. Rev. E 65, 046308 (2002), which the paper compares
with the Shan–Chen velocity shift in Sec. IV.A and Table I)."""
import numpy as np
import pytest

import oracle as O
import oracle.diagnostics as D
from lbm_inputs import coexistence_densities, drop_density, node_coords, random_state_fields, tanh_profile

pytestmark = pytest.mark.filterwarnings("ignore")


def test_guo_collision_moments():
    """Guo's forcing term carries no mass, adds (1 - 1/(2 tau)) F of
    momentum and (1 - 1/(2 tau)) (u F + F u) of momentum flux, with the
    equilibrium at the hydrodynamic velocity u = (j + F/2)/rho.  So the
    collision keeps sum f* = rho - rho u_r/r and sum c f* = j + F + H,
    and its second moment is
    Pi - (Pi - rho (c_s^2 I + u u))/tau + (1 - 1/(2 tau)) (u F + F u)
      - c_s^2 (rho u_r / r) I,
    where Pi = sum c c f of the incoming populations."""
    nz, nr, tau = 24, 16, 0.8
    rho, uz, ur = random_state_fields(21, nz, nr, rho_lo=0.4, rho_hi=1.6, u_amp=0.02)
    p = O.make_params(nz, nr, G=-5.0, tau=tau, wall=1, axisym=1, flags=O.FLAG_GUO)
    rng = np.random.Generator(np.random.PCG64(3))
    f = O.equilibrium(p, rho, uz, ur) * (1.0 + 0.01 * rng.uniform(-1, 1, size=(9, nr, nz)))
    fl = O.fields(p, f)
    cz, cr, _ = O.lattice()
    cz = cz[:, None, None].astype(float)
    cr = cr[:, None, None].astype(float)
    r = (np.arange(nr) + 0.5)[:, None]
    fs = fl["fstar"]
    u_z, u_r, Fz, Fr, rh = fl["u_z"], fl["u_r"], fl["f_z"], fl["f_r"], fl["rho"]
    assert np.abs(fl["ueq_z"] - u_z).max() == 0 and np.abs(fl["ueq_r"] - u_r).max() == 0
    tol = 1e-13
    mass = rh * u_r / r
    assert np.allclose(fs.sum(0), rh - mass, rtol=0, atol=tol)
    assert np.allclose((cz * fs).sum(0), fl["jz"] + Fz + fl["h_z"], rtol=0, atol=tol)
    assert np.allclose((cr * fs).sum(0), fl["jr"] + Fr + fl["h_r"], rtol=0, atol=tol)
    k = 1.0 - 0.5 / tau
    for (a, b, ua, ub, Fa, Fb, d) in ((cz, cz, u_z, u_z, Fz, Fz, 1.0), (cr, cr, u_r, u_r, Fr, Fr, 1.0),
                                      (cz, cr, u_z, u_r, Fz, Fr, 0.0)):
        Pi = (a * b * f).sum(0)
        want = Pi - (Pi - rh * (d / 3.0 + ua * ub)) / tau + k * (ua * Fb + Fa * ub) - d * mass / 3.0
        assert np.allclose((a * b * fs).sum(0), want, rtol=0, atol=1e-13)


def _flat(G, axisym, steps=20000):
    rg, rl = coexistence_densities(G)
    p = O.make_params(1, 64, G=G, tau=1.0, wall=1, axisym=axisym, flags=O.FLAG_GUO)
    _, r = node_coords(1, 64)
    rho = tanh_profile(r, 32.0, rl, rg, 2.0)
    return O.fields(p, O.run(p, O.equilibrium(p, rho, 0 * rho, 0 * rho), steps))


@pytest.mark.parametrize("k", [0, 1, 2])
def test_guo_table1_surface_tension(golden, k):
    """Table I (Guo columns): the surface tension of Eq. st (no
    tau-correction) of a flat interface with Guo forcing, planar and
    axisymmetric.  This reading reproduces the printed values within 0.6 /
    2.8 / 5.1 % (planar) and 1.1 / 3.1 / 5.5 % (axisymmetric) for G = -4.5 /
    -5.0 / -5.5 -- below the printed values, by more at stronger coupling;
    tolerance 6 %.  The two schemes agree to 0.5 % (the printed pairs differ
    by 0.3-0.7 %), and the Guo values are about 35 % below the Shan–Chen
    ones, as printed."""
    t = golden["table1_surface_tension_guo"]
    G = t["G"][k]
    g2 = D.surface_tension_sc(*[_flat(G, 0)[n] for n in ("rho", "f_r")], G, 1.0)[1]
    ga = D.surface_tension_sc(*[_flat(G, 1)[n] for n in ("rho", "f_r")], G, 1.0)[1]
    assert g2 == pytest.approx(t["gamma_2d"][k], rel=0.06)
    assert ga == pytest.approx(t["gamma_axis"][k], rel=0.06)
    assert abs(ga - g2) / g2 < 0.005
    sc = golden["table1_surface_tension_sc"]["gamma_2d"][k]
    assert 0.55 < g2 / sc < 0.7


def test_guo_hagen_poiseuille(golden):
    """Sec. III.A pipe flow with the body force entered through Guo's term:
    the same parabolic profile with the printed U1 = 3.84e-3 (1 %)."""
    hp = golden["hagen_poiseuille"]
    nz, nr = hp["nz"], hp["nr"]
    p = O.make_params(nz, nr, G=0.0, tau=hp["tau"], gz=hp["g"], wall=0, axisym=1, flags=O.FLAG_GUO)
    rho = np.ones((nr, nz))
    f = O.run(p, O.equilibrium(p, rho, 0 * rho, 0 * rho), 15000)
    _, uz, ur = O.moments(p, f)
    _, r = node_coords(nz, nr)
    a = np.polyfit(r[:4, 0] ** 2, uz[:4, 0], 1)
    assert a[1] == pytest.approx(hp["U1"], rel=0.01)
    assert np.abs(ur).max() < 1e-12
