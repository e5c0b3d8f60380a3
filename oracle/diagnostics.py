"""FP64 diagnostics of the oracle's fields (test infrastructure only).

Each function works on numpy fields ``[nr, nz]`` with node (k, j) at z = k,
r = j + 1/2, and cites the passage of the paper that defines the quantity.
Where the paper leaves an observable open, the reading used is stated.
"""
import numpy as np

CS2 = 1.0 / 3.0


def radii(nr):
    return np.arange(nr, dtype=np.float64) + 0.5


def psi(rho, rho0=1.0):
    """Pseudopotential (Sec. II.A)."""
    return rho0 * (1.0 - np.exp(-rho / rho0))


def pressure(rho, G, rho0=1.0):
    """Bulk non-ideal pressure p_NI (Sec. II.A, Eq. pressure)."""
    return CS2 * rho + 0.5 * CS2 * G * psi(rho, rho0) ** 2


def mass_3d(rho):
    """3D mass: density weighted with 2*pi*r (Sec. II.B; validation note of
    Sec. II.C)."""
    r = radii(rho.shape[0])[:, None]
    return float(np.sum(2.0 * np.pi * r * rho))


def mass_2d(rho):
    return float(np.sum(rho))


def momentum_z_3d(rho, uz):
    r = radii(rho.shape[0])[:, None]
    return float(np.sum(2.0 * np.pi * r * rho * uz))


def kinetic_energy(rho, uz, ur):
    """E_ke = pi * sum_z sum_r r rho |u|^2 (Sec. III, steady-state criterion)."""
    r = radii(rho.shape[0])[:, None]
    return float(np.pi * np.sum(r * rho * (uz * uz + ur * ur)))


def axis_intercept(rho, z_col, rho_mid):
    """A(t): radial intercept of the drop at column z_col (Sec. IV.B).
    Reading: the outermost crossing of rho = rho_mid along r, linearly
    interpolated between nodes."""
    col = rho[:, int(z_col)]
    r = radii(rho.shape[0])
    inside = col >= rho_mid
    idx = np.nonzero(inside)[0]
    if idx.size == 0:
        return 0.0
    j = idx[-1]
    if j + 1 >= col.size:
        return float(r[-1])
    a, b = col[j], col[j + 1]
    return float(r[j] + (a - rho_mid) / (a - b))


def equivalent_radius(rho, rho_l, rho_g):
    """Radius of the sphere with the drop's 3D volume, from the liquid
    fraction phi = (rho - rho_g)/(rho_l - rho_g) weighted with 2*pi*r."""
    phi = (rho - rho_g) / (rho_l - rho_g)
    v = mass_3d(phi)
    return float((3.0 * v / (4.0 * np.pi)) ** (1.0 / 3.0))


def surface_tension_sc(rho, f_r, G, tau, rho0=1.0):
    """Surface tension of a z-independent interface along r with the
    tau-correction of the Shan–Chen forcing (Sec. II.A, Eq. stc).
    Reading: the profile is taken along r on column 0, d/dr is the
    one-dimensional fourth-order stencil with the mirror at the axis and at the
    wall, and the integrals are plain sums over the rows (unit spacing)."""
    p = psi(rho[:, 0], rho0)
    nr = p.size
    ng = 6
    e = np.concatenate([p[ng - 1::-1], p, p[: nr - ng - 1: -1]])
    j = np.arange(nr) + ng
    d = (-e[j + 2] + 8.0 * e[j + 1] - 8.0 * e[j - 1] + e[j - 2]) / 12.0
    term1 = -(G * CS2 * CS2 / 2.0) * np.sum(d * d)
    term2 = (tau - 0.5) ** 2 * np.sum(f_r[:, 0] ** 2 / rho[:, 0])
    return float(term1 + term2), float(term1), float(term2)


def interface_radius_weights(nz, nr, zc, thetas, ds=0.5, s_max=None):
    """Sparse linear map rho -> r(theta) of the ray-integral interface radius.

    Reading (the paper fixes no interface-shape observable): along the ray from
    (zc, 0) at angle theta, r(theta) = sum_k ds * phi(zc + s_k cos(theta),
    s_k sin(theta)) with s_k = (k + 1/2) ds, where phi is the bilinear
    interpolant of the node values (z periodic, even mirror below row 0, rows
    clamped above the last row).  Returns, per angle, (node indices, weights)
    such that r = sum_w w * value[node]."""
    if s_max is None:
        s_max = min(nz / 2.0, float(nr)) - 1.0
    nk = int(np.floor(s_max / ds))
    out = []
    for th in thetas:
        acc = {}
        for k in range(nk):
            s = (k + 0.5) * ds
            z = zc + s * np.cos(th)
            r = s * np.sin(th)
            y = r - 0.5  # row coordinate
            j0 = int(np.floor(y))
            ty = y - j0
            k0 = int(np.floor(z))
            tz = z - k0
            for dj, wy in ((0, 1.0 - ty), (1, ty)):
                jj = j0 + dj
                if jj < 0:
                    jj = -1 - jj
                if jj > nr - 1:
                    jj = nr - 1
                for dk, wz in ((0, 1.0 - tz), (1, tz)):
                    kk = (k0 + dk) % nz
                    w = ds * wy * wz
                    if w != 0.0:
                        idx = jj * nz + kk
                        acc[idx] = acc.get(idx, 0.0) + w
        keys = np.array(sorted(acc), dtype=np.int64)
        out.append((keys, np.array([acc[k] for k in keys], dtype=np.float64)))
    return out


def interface_radius(rho, weights, rho_l, rho_g):
    """r(theta) for each angle from the weights of interface_radius_weights."""
    flat = ((rho - rho_g) / (rho_l - rho_g)).ravel()
    return np.array([np.dot(w, flat[idx]) for idx, w in weights])


def drops(rho, rho_mid):
    """Drops on the axis once a thread has broken up (Sec. IV.C).

    Reading: a drop is a maximal run of consecutive columns, periodic in z,
    whose axis node (row 0) has rho >= rho_mid.  Its 3D volume is the solid
    of revolution of the interface radius R(z) of axis_intercept,
    sum_z pi R(z)^2, and its centre the volume-weighted mean column, counted
    without wrapping from the first gas column onward and then taken modulo
    nz.  Returns (n, volumes, centres): n = -1 with no drops if every axis
    node is liquid (an unbroken thread), n = 0 if none is.  Drops are listed
    from the first gas column onward."""
    nz = rho.shape[1]
    liquid = rho[0] >= rho_mid
    if liquid.all():
        return -1, [], []
    if not liquid.any():
        return 0, [], []
    start = int(np.argmin(liquid))  # first gas column
    vols, cents = [], []
    k = 0
    while k < nz:
        if not liquid[(start + k) % nz]:
            k += 1
            continue
        v = m = 0.0
        while k < nz and liquid[(start + k) % nz]:
            R = axis_intercept(rho, (start + k) % nz, rho_mid)
            w = np.pi * (R * R)
            v += w
            m += w * float(start + k)
            k += 1
        vols.append(v)
        cents.append((m / v) % nz)
    return len(vols), vols, cents


def breakup_step(rho_axis_history, rho_mid):
    """First index at which any axis node (row 0) falls below rho_mid
    (reading of the break-up time), or None."""
    for t, row in enumerate(rho_axis_history):
        if np.min(row) < rho_mid:
            return t
    return None
