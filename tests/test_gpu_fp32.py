"""Errors of the FP32 shifted-storage path against FP64.

Populations are stored and collided in FP32 as g_i = f_i - W_i rho_ref
(the paper fixes no precision; its scheme is Sec. II).  There is no exact
pin for this mode, so each result is compared with the FP64 oracle, or with
the GPU FP64 path where the oracle would take minutes (that path matches the
oracle to round-off, see test_gpu_parity.py):

- density and velocity fields of the oscillating drop (256 x 128) after
  2000 steps, for four choices of rho_ref;
- the l = 2 oscillation frequency of the same drop over 20000 steps
  (Sec. IV.B), against the oracle's: relative error <= 0.5 %;
- the break-up step of a Rayleigh-Plateau thread (Sec. IV.C) on the
  4096 x 512 lattice with the 7th harmonic perturbation (kappa* ~ 0.69).
"""
import numpy as np
import pytest
import torch
from scipy.optimize import curve_fit

import oracle as O
import oracle.diagnostics as D
from lbm_inputs import oscillating_drop, thread_density

pytestmark = pytest.mark.gpu


def _lib():
    from paper_1310_1871_amd import lbm_axi as L
    return L


def _say(msg):
    print(msg, flush=True)


def _sim(case, precision, rho_ref=0.0):
    L = _lib()
    p = L.make_params(case.nz, case.nr, G=case.G, tau=case.tau, wall=case.wall, axisym=1, precision=precision,
                      rho_ref=rho_ref)
    return L.AxiLBM(p, torch.from_numpy(case.rho).cuda())


def _fit_frequency(ts, A, t_min=3000.0):
    """Fit g(t) = R_D + a exp(-b t) sin(w t + d) (Sec. IV.B) to A(t) for
    t > t_min (after the start-up transient; the drop settles near R_D ~ 40)
    from a few starting phases and periods; returns |w| of the best fit."""
    g = lambda t, R0, a, b, w, d: R0 + a * np.exp(-b * t) * np.sin(w * t + d)
    m = ts > t_min
    R_guess = float(A[-200:].mean())
    best = None
    for d0 in (0.0, 1.5, 3.0, 4.5):
        for period in (3000.0, 3700.0, 4500.0):
            try:
                popt, _ = curve_fit(g, ts[m], A[m], p0=[R_guess, A[m][0] - R_guess, 2e-4, 2 * np.pi / period, d0],
                                    maxfev=20000)
            except RuntimeError:
                continue
            res = float(np.sum((g(ts[m], *popt) - A[m]) ** 2))
            if best is None or res < best[0]:
                best = (res, popt)
    assert best is not None
    return abs(best[1][3]), best[1]


def _gpu_intercepts(case, precision, rho_ref, steps, every):
    sim = _sim(case, precision, rho_ref)
    mid = 0.5 * (case.rho_l + case.rho_g)
    ts, A = [], []
    for k in range(steps // every):
        sim.step(every)
        rho, _, _ = sim.moments()
        col = rho[:, case.nz // 2].cpu().numpy()
        ts.append((k + 1) * every)
        A.append(D.axis_intercept(col[:, None], 0, mid))
    sim.close()
    return np.array(ts, dtype=np.float64), np.array(A)


def test_fp32_field_error_oscillating_drop():
    """max |d rho| and max |d u| of FP32 storage vs the FP64 oracle after
    2000 steps of the oscillating drop (256 x 128, G = -5.5, tau = 0.8) for
    rho_ref = 0, rho_g, (rho_l + rho_g)/2 and rho_l.  The printed table is
    the stated error; the bounds are loose envelopes of it.  The gas density
    is the default shift: the gas fills most of the (2 pi r weighted)
    volume, and a shift far from a phase's density costs that phase its
    low-order bits (rho = sum g + rho_ref cancels)."""
    case = oscillating_drop()
    steps = 2000
    p = O.make_params(case.nz, case.nr, G=case.G, tau=case.tau, wall=case.wall, axisym=1)
    f = O.run(p, O.equilibrium(p, case.rho, case.uz, case.ur), steps)
    ro, uzo, uro = O.moments(p, f)
    errs = {}
    for kind, rr in (("zero", 0.0), ("gas", case.rho_g), ("mid", 0.5 * (case.rho_l + case.rho_g)),
                     ("liquid", case.rho_l)):
        _say(f"fp32 field error rho_ref={kind} ({rr:.4f}) 256x128 {steps} steps")
        sim = _sim(case, 1, rr)
        sim.step(steps)
        rho32, uz32, ur32 = (t.cpu().numpy() for t in sim.moments())
        sim.close()
        drho = float(np.abs(rho32 - ro).max())
        du = float(max(np.abs(uz32 - uzo).max(), np.abs(ur32 - uro).max()))
        errs[kind] = (drho, du)
        _say(f"  max|d rho| = {drho:.3e}  max|d u| = {du:.3e}  (max|u| = {np.abs(uzo).max():.3e})")
    for drho, du in errs.values():
        assert drho < 1e-2 and du < 1e-3
    assert errs["gas"][0] < 1e-3 and errs["gas"][1] < 1e-4


def test_fp32_mass_drift_planar():
    """Plain 2D mode (no axisymmetric terms) with the specular axis and a
    free-slip wall conserves sum rho exactly in exact arithmetic (Sec. II:
    collision and streaming move mass without creating it), so any drift is
    FP32 rounding.  Stored values are rounded at every step, and over smooth
    regions those roundings are correlated, so the drift grows about
    linearly: the printed relative drift over 2000 steps is the stated
    figure (about 1e-5 for the unshifted and gas-shifted stores).  Bound:
    3e-5 for those two shifts, 3e-4 for the liquid shift."""
    L = _lib()
    case = oscillating_drop()
    for rr, bound in ((0.0, 3e-5), (case.rho_g, 3e-5), (case.rho_l, 3e-4)):
        _say(f"fp32 planar mass drift rho_ref={rr:.4f}")
        p = L.make_params(case.nz, case.nr, G=case.G, tau=case.tau, wall=L.WALL_FREESLIP, axisym=0,
                          precision=L.FP32_SHIFTED, rho_ref=rr)
        sim = L.AxiLBM(p, torch.from_numpy(case.rho).cuda())
        m0 = float(sim.populations().sum())
        sim.step(2000)
        m1 = float(sim.populations().sum())
        sim.close()
        _say(f"  relative drift {abs(m1 - m0) / m0:.3e}")
        assert abs(m1 - m0) / m0 < bound


def test_fp32_drop_frequency_vs_oracle():
    """l = 2 frequency of the oscillating drop (256 x 128, tau = 0.8, 20000
    steps, A(t) every 10 steps, period about 3100 steps) from FP32 storage
    (rho_ref = rho_g) vs the FP64 oracle's: relative difference <= 0.5 %.
    The GPU FP64 trace is also fitted and must reproduce the oracle's
    frequency to 1e-6.  Both are compared with Miller and Scriven's
    frequency (Sec. IV.B) at the fitted R_D: +2.1 % (bound 3 %).  The paper
    fixes no damping; the fitted decay rate b (4.7e-4 per step) is set
    beside Lamb's (l - 1)(2 l + 1) nu / R_D^2 for a free drop (3.1e-4): 1.5
    times it, the excess that the gas, the interface boundary layers (a
    tenth of Lamb's rate by Miller and Scriven's correction) and the
    diffuse interface of a few nodes add; bound 1-2."""
    case = oscillating_drop()
    steps, every = 20000, 10
    mid = 0.5 * (case.rho_l + case.rho_g)
    _say("fp32 drop frequency: oracle 256x128 20000 steps")
    p = O.make_params(case.nz, case.nr, G=case.G, tau=case.tau, wall=case.wall, axisym=1)
    f = O.equilibrium(p, case.rho, case.uz, case.ur)
    ts, Ao = [], []
    for k in range(steps // every):
        f = O.run(p, f, every)
        rr, _, _ = O.moments(p, f)
        ts.append((k + 1) * every)
        Ao.append(D.axis_intercept(rr, case.nz // 2, mid))
    ts, Ao = np.array(ts, dtype=np.float64), np.array(Ao)
    w_o, _ = _fit_frequency(ts, Ao)
    _say("fp32 drop frequency: GPU FP64 and FP32 traces")
    t64, A64 = _gpu_intercepts(case, 0, 0.0, steps, every)
    t32, A32 = _gpu_intercepts(case, 1, case.rho_g, steps, every)
    assert np.max(np.abs(A64 - Ao)) < 1e-6
    w64, _ = _fit_frequency(t64, A64)
    w32, _ = _fit_frequency(t32, A32)
    err = abs(w32 - w_o) / w_o
    _say(f"  omega oracle {w_o:.6e}  GPU FP64 {w64:.6e}  GPU FP32 {w32:.6e}  rel err FP32 {err:.3e}  "
         f"max|dA| FP32 {np.max(np.abs(A32 - Ao)):.3e}")
    assert abs(w64 - w_o) / w_o < 1e-6
    assert err <= 5e-3
    # the frequency against Miller and Scriven's w_2 (Eq. freq-drop-miller)
    # at the fitted R_D, with the surface tension of Eq. stc from a flat
    # interface at the same (G, tau) and the measured bulk densities
    gam = _flat_surface_tension(case.G, case.tau)
    rin, rout = float(rr[0, case.nz // 2]), float(rr[-1, 0])
    nu = (case.tau - 0.5) / 3.0
    for name, (t_, A_) in (("FP64", (t64, A64)), ("FP32", (t32, A32))):
        w, popt = _fit_frequency(t_, A_)
        R0 = popt[0]
        w0 = np.sqrt(24 * gam / (R0 ** 3 * (2 * rout + 3 * rin)))
        al = 25 * nu * rin * rout / (np.sqrt(2) * R0 * (2 * rout + 3 * rin) * (np.sqrt(nu) * (rin + rout)))
        ms = w0 - 0.5 * al * np.sqrt(w0) + 0.25 * al * al
        lamb = 5.0 * nu / R0 ** 2  # (l - 1)(2 l + 1) nu / R^2, l = 2
        _say(f"  {name}: R_D {R0:.3f}  omega {w:.6e}  Miller-Scriven {ms:.6e}  rel err {w / ms - 1:+.4f}  "
             f"decay {popt[2]:.3e}  Lamb {lamb:.3e}  ratio {popt[2] / lamb:.3f}")
        # the paper reports about 1 % at G = -6, tau = 1 on 320 x 128 (the
        # oracle pin reproduces that); this drop (G = -5.5, tau = 0.8,
        # R = 40) is 2.1 % fast
        assert abs(w / ms - 1.0) < 0.03
        assert 1.0 < popt[2] / lamb < 2.0


def _flat_surface_tension(G, tau):
    """gamma-tilde (Eq. stc) of a flat interface on 1 x 64 at (G, tau),
    from the oracle (Table I's set-up)."""
    from lbm_inputs import node_coords, scheme_coexistence, tanh_profile
    rg, rl = scheme_coexistence(G, tau)
    p = O.make_params(1, 64, G=G, tau=tau, wall=1, axisym=0)
    _, r = node_coords(1, 64)
    rho = tanh_profile(r, 32.0, rl, rg, 2.0)
    fl = O.fields(p, O.run(p, O.equilibrium(p, rho, 0 * rho, 0 * rho), 20000))
    return D.surface_tension_sc(fl["rho"], fl["f_r"], G, tau)[0]


# bulk densities the scheme settles to at G = -5.5, tau = 0.8 (measured on a
# long thread run; the flat-interface mechanical-stability values 2.3075 /
# 0.1048 hold at tau = 1, and at tau = 0.8 the gas condenses onto the thread)
RP_RHO_L, RP_RHO_G = 2.277, 0.0744


def _breakup(precision, rho_ref, nz, nr, steps_max, every):
    L = _lib()
    G, tau, R = -5.5, 0.8, 64.0
    rl, rg = RP_RHO_L, RP_RHO_G
    rho = thread_density(nz, nr, R, rl, rg, 2.0, 0.1, 7)
    p = L.make_params(nz, nr, G=G, tau=tau, wall=L.WALL_FREESLIP, axisym=1, precision=precision, rho_ref=rho_ref)
    sim = L.AxiLBM(p, torch.from_numpy(rho).cuda())
    mid = 0.5 * (rl + rg)
    t = 0
    while t < steps_max:
        sim.step(every)
        t += every
        rho_d, _, _ = sim.moments()
        if float(rho_d[0].min()) < mid:
            sim.close()
            return t
    sim.close()
    return None


def test_fp32_breakup_step_rayleigh_plateau():
    """Break-up step (first step, on a 50-step grid, at which an axis node
    falls below rho_mid) of the 4096 x 512 thread of radius 64 with a
    0.1 R cos(2 pi 7 z / 4096) perturbation (kappa* = 0.69 < 1, so it breaks;
    Sec. IV.C), G = -5.5, tau = 0.8, free-slip wall: FP32 (rho_ref = rho_g)
    vs FP64 within 1 %.  The FP64 run is the GPU path (the oracle would take
    about ten minutes here); it breaks near step 27000."""
    nz, nr = 4096, 512
    _say("fp32 breakup: 4096x512 7th harmonic, FP64 then FP32")
    b64 = _breakup(0, 0.0, nz, nr, 40000, 50)
    b32 = _breakup(1, RP_RHO_G, nz, nr, 40000, 50)
    _say(f"  breakup step FP64 {b64}  FP32 {b32}")
    assert b64 is not None and b32 is not None
    assert 20000 < b64 < 35000
    assert abs(b32 - b64) <= max(100, 0.01 * b64)


@pytest.mark.parametrize("flags", [16, 4])
def test_fp32_options_field_error(flags):
    """The run-time option path in FP32 shifted storage (rho_ref = rho_g):
    the mid-link source (flag 16) and Guo forcing (flag 4) on the
    oscillating drop at tau = 1 (with Guo forcing the scheme diverges at
    tau = 0.8 on this drop, in the oracle as on the GPU), 2000 steps,
    against the FP64 oracle with the same option, within the envelope of
    the default path (max |d rho| < 1e-3, max |d u| < 1e-4)."""
    L = _lib()
    case = oscillating_drop(tau=1.0)
    steps = 2000
    p = O.make_params(case.nz, case.nr, G=case.G, tau=case.tau, wall=case.wall, axisym=1, flags=flags)
    ro, uzo, uro = O.moments(p, O.run(p, O.equilibrium(p, case.rho, case.uz, case.ur), steps))
    _say(f"fp32 option {flags} field error 256x128 {steps} steps")
    pg = L.make_params(case.nz, case.nr, G=case.G, tau=case.tau, wall=case.wall, axisym=1,
                       precision=L.FP32_SHIFTED, rho_ref=case.rho_g, flags=flags)
    sim = L.AxiLBM(pg, torch.from_numpy(case.rho).cuda())
    sim.step(steps)
    rho32, uz32, ur32 = (t.cpu().numpy() for t in sim.moments())
    sim.close()
    drho = float(np.abs(rho32 - ro).max())
    du = float(max(np.abs(uz32 - uzo).max(), np.abs(ur32 - uro).max()))
    _say(f"  max|d rho| = {drho:.3e}  max|d u| = {du:.3e}")
    assert drho < 1e-3 and du < 1e-4
