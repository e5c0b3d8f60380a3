"""Plain FP64 CPU oracle of the axisymmetric Shan–Chen lattice Boltzmann step.

TEST INFRASTRUCTURE ONLY.  The test suite, the smoke check and the CPU-baseline
leg of the benchmark are the only users; the HIP library never imports, links
or loads anything here.  The arithmetic lives in ``lbm_axi_oracle.c`` (plain
loops, no fast-math, no contraction); this module marshals numpy arrays into
it through ctypes.

Arrays: populations are ``float64[9, nr, nz]`` (direction, row, column), fields
``float64[nr, nz]``; node (k, j) sits at z = k, r = j + 1/2 (paper Sec. II.E).
The complex-step variants (``complex128`` arrays, complex G and tau) evaluate
the same step in complex arithmetic.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))

# order of the intermediate fields returned by fields()
FIELD_NAMES = (
    "rho", "jz", "jr", "psi",
    "fsc_z", "fsc_r",
    "dr_psi", "drr_psi", "d1r_psi", "dzr_psi",
    "fsym_z", "fsym_r",
    "f_z", "f_r",
    "ueq_z", "ueq_r", "u_z", "u_r",
    "dr_uz", "dz_ur", "dr_ur",
    "h_z", "h_r",
)

WALL_NOSLIP = 0
WALL_FREESLIP = 1


class Params(ctypes.Structure):
    _fields_ = [
        ("nz", ctypes.c_int32), ("nr", ctypes.c_int32),
        ("G", ctypes.c_double), ("G_im", ctypes.c_double),
        ("tau", ctypes.c_double), ("tau_im", ctypes.c_double),
        ("psi_rho0", ctypes.c_double), ("gz", ctypes.c_double),
        ("wall", ctypes.c_int32), ("axisym", ctypes.c_int32),
        ("flags", ctypes.c_int32), ("in_row", ctypes.c_int32),
        ("out_row", ctypes.c_int32), ("pad", ctypes.c_int32),
        ("rho_in", ctypes.c_double), ("rho_out", ctypes.c_double),
        ("uz_in", ctypes.c_void_p), ("ur_in", ctypes.c_void_p),
    ]


FLAG_GUO = 4  # Guo forcing instead of the velocity shift (see the C source)
FLAG_NO_WALL_DERIV = 2  # derivative terms zero on rows whose stencils cross the wall
FLAG_ZWALLS = 8  # no-slip walls at both ends of z instead of periodic z
FLAG_MIDLINK = 16  # source h_i averaged over the two ends of each link (see the C source)


def make_params(nz, nr, G=-5.5, tau=1.0, psi_rho0=1.0, gz=0.0, wall=WALL_NOSLIP, axisym=1,
                G_im=0.0, tau_im=0.0, flags=0, in_row=-1, out_row=-1, rho_in=1.0, rho_out=1.0,
                uz_in=None, ur_in=None):
    """Oracle parameters.  Open boundaries (see the C source): in_row /
    out_row >= 0 impose f^eq(rho_in, uz_in[z], ur_in[z]) on the inlet row and
    f^eq(rho_out, u one row inside) on the outlet row after each collision."""
    p = Params(int(nz), int(nr), float(G), float(G_im), float(tau), float(tau_im),
               float(psi_rho0), float(gz), int(wall), int(axisym), int(flags), int(in_row), int(out_row), 0,
               float(rho_in), float(rho_out), None, None)
    if in_row >= 0:
        uz = np.ascontiguousarray(np.zeros(nz) if uz_in is None else uz_in, dtype=np.float64)
        ur = np.ascontiguousarray(np.zeros(nz) if ur_in is None else ur_in, dtype=np.float64)
        assert uz.shape == (nz,) and ur.shape == (nz,)
        p.uz_in, p.ur_in = uz.ctypes.data, ur.ctypes.data
        p._keep = (uz, ur)  # the C side reads these arrays during run()
    return p


_lib = None
_libc = None


def _load():
    global _lib, _libc
    if _lib is None:
        # ORACLE_LIB_SUFFIX=_san selects the sanitizer build (CPU sanitizer test)
        suffix = os.environ.get("ORACLE_LIB_SUFFIX", "")
        path = os.path.join(_HERE, f"liboracle{suffix}.so")
        cpath = os.path.join(_HERE, f"liboracle_complex{suffix}.so")
        if not (os.path.exists(path) and os.path.exists(cpath)):
            from . import build as _b
            _b.build(sanitize=suffix == "_san")
        _lib = ctypes.CDLL(path)
        _libc = ctypes.CDLL(cpath)
        P = ctypes.POINTER(Params)
        vp = ctypes.c_void_p
        for lib, pre in ((_lib, "or_"), (_libc, "orc_")):
            getattr(lib, pre + "run").argtypes = [P, vp, vp, ctypes.c_int64]
            getattr(lib, pre + "run").restype = ctypes.c_int
            getattr(lib, pre + "fields").argtypes = [P, vp, vp]
            getattr(lib, pre + "fields").restype = ctypes.c_int
            getattr(lib, pre + "moments").argtypes = [P, vp, vp, vp, vp]
            getattr(lib, pre + "moments").restype = ctypes.c_int
            getattr(lib, pre + "equilibrium").argtypes = [P, vp, vp, vp, vp]
            getattr(lib, pre + "equilibrium").restype = None
            getattr(lib, pre + "stream").argtypes = [P, vp, vp]
            getattr(lib, pre + "stream").restype = None
            getattr(lib, pre + "num_fields").restype = ctypes.c_int
        _lib.or_stencil_point.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, vp, ctypes.c_int, ctypes.c_int]
        _lib.or_stencil_point.restype = ctypes.c_double
        _lib.or_lattice.argtypes = [vp, vp, vp]
        _lib.or_ghost_rows.restype = ctypes.c_int
        assert _lib.or_num_fields() == len(FIELD_NAMES)
    return _lib, _libc


def _arr(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


def _ptr(a):
    return ctypes.c_void_p(a.ctypes.data)


def _pick(complex_step):
    lib, libc = _load()
    return (libc, "orc_", np.complex128) if complex_step else (lib, "or_", np.float64)


def set_threads(n):
    """Number of OpenMP threads the oracle's loops use from now on (in this
    process); the default is every host thread."""
    ctypes.CDLL("libgomp.so.1").omp_set_num_threads(int(n))


def lattice():
    """(cz, cr, w) as the oracle holds them."""
    lib, _ = _load()
    cz = np.zeros(9, np.int32)
    cr = np.zeros(9, np.int32)
    w = np.zeros(9, np.float64)
    lib.or_lattice(_ptr(cz), _ptr(cr), _ptr(w))
    return cz, cr, w


def ghost_rows():
    lib, _ = _load()
    return lib.or_ghost_rows()


def equilibrium(p, rho, uz, ur, complex_step=False):
    lib, pre, dt = _pick(complex_step)
    rho, uz, ur = _arr(rho, dt), _arr(uz, dt), _arr(ur, dt)
    f = np.zeros((9, p.nr, p.nz), dt)
    getattr(lib, pre + "equilibrium")(ctypes.byref(p), _ptr(rho), _ptr(uz), _ptr(ur), _ptr(f))
    return f


def run(p, f, n_steps, complex_step=False):
    """State after n_steps full steps from post-streaming state f."""
    lib, pre, dt = _pick(complex_step)
    fin = _arr(f, dt)
    assert fin.shape == (9, p.nr, p.nz)
    out = np.empty_like(fin)
    rc = getattr(lib, pre + "run")(ctypes.byref(p), _ptr(fin), _ptr(out), int(n_steps))
    if rc != 0:
        raise ValueError(f"oracle run failed ({rc})")
    return out


def fields(p, f, complex_step=False):
    """Dict of every intermediate of one step from state f, plus h[9] and the
    post-collision (pre-streaming) populations fstar[9]."""
    lib, pre, dt = _pick(complex_step)
    fin = _arr(f, dt)
    n = p.nz * p.nr
    k = len(FIELD_NAMES)
    out = np.zeros((k + 18) * n, dt)
    rc = getattr(lib, pre + "fields")(ctypes.byref(p), _ptr(fin), _ptr(out))
    if rc != 0:
        raise ValueError(f"oracle fields failed ({rc})")
    d = {name: out[i * n:(i + 1) * n].reshape(p.nr, p.nz) for i, name in enumerate(FIELD_NAMES)}
    d["h"] = out[k * n:(k + 9) * n].reshape(9, p.nr, p.nz)
    d["fstar"] = out[(k + 9) * n:(k + 18) * n].reshape(9, p.nr, p.nz)
    return d


def moments(p, f, complex_step=False):
    """(rho, u_z, u_r) with the hydrodynamic velocity of Eq. uhydro."""
    lib, pre, dt = _pick(complex_step)
    fin = _arr(f, dt)
    rho = np.zeros((p.nr, p.nz), dt)
    uz = np.zeros_like(rho)
    ur = np.zeros_like(rho)
    rc = getattr(lib, pre + "moments")(ctypes.byref(p), _ptr(fin), _ptr(rho), _ptr(uz), _ptr(ur))
    if rc != 0:
        raise ValueError(f"oracle moments failed ({rc})")
    return rho, uz, ur


def stream(p, fstar, complex_step=False):
    lib, pre, dt = _pick(complex_step)
    fin = _arr(fstar, dt)
    out = np.zeros_like(fin)
    getattr(lib, pre + "stream")(ctypes.byref(p), _ptr(fin), _ptr(out))
    return out


STENCILS = {"d_r": 0, "d_z": 1, "d1_r": 2, "d_zr": 3, "d_rr": 4, "sc_z": 5, "sc_r": 6}


def stencil_point(kind, ext, z, r):
    """Evaluate one stencil at (z, r) on a caller-filled extended field
    ext[nr + 2*NG, nz] (row index r + NG)."""
    lib, _ = _load()
    ext = _arr(ext, np.float64)
    ng = lib.or_ghost_rows()
    nr = ext.shape[0] - 2 * ng
    return lib.or_stencil_point(STENCILS[kind], ext.shape[1], nr, _ptr(ext), int(z), int(r))
