"""Thin ctypes binding of the lbm_axi C ABI (include/lbm_axi.h).

Argument marshalling only: PyTorch provides device memory and the stream,
every step of the method runs in the HIP library.  Importing this module on
a machine where the built library is missing raises ImportError; there is no
CPU fallback.
"""
import contextlib
import ctypes
import os
import warnings

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
# LBM_AXI_LIB names another build of the library (the host-sanitized one of
# the CPU sanitizer test); the default is the in-tree HIP build
LIB_PATH = os.environ.get("LBM_AXI_LIB", os.path.join(_HERE, "liblbm_axi.so"))

OK = 0
EINVAL = -1
ENOMEM = -2
EHIP = -3
ENONFINITE = -4
EUNSUP = -5
WARN_STABILITY = 1  # success with a warning: G < -6 (Sec. II.D stability rule of thumb)

WALL_NOSLIP = 0
WALL_FREESLIP = 1
FP64 = 0
FP32_SHIFTED = 1
FLAG_GUO = 4  # Guo forcing instead of the velocity shift (include/lbm_axi.h)
FLAG_NO_WALL_DERIV = 2  # derivative terms zero on rows whose stencils cross the wall
FLAG_ZWALLS = 8  # no-slip walls at both ends of z (mid-grid bounce-back) instead of periodic z
FLAG_MIDLINK = 16  # source h_i averaged over each link instead of the node value
NREDUCE = 4
NINTERFACE = 7
MAX_DROPS = 64
KERNEL_TILE = 0
KERNEL_STRIP = 1
KERNEL_TILE_ALTERNATE = 2
KERNEL_TILE_COLUMNS = 3
KERNEL_TILE_PAIRS = 4


class Params(ctypes.Structure):
    _fields_ = [
        ("nz", ctypes.c_int32), ("nr", ctypes.c_int32),
        ("G", ctypes.c_double), ("tau", ctypes.c_double),
        ("psi_rho0", ctypes.c_double), ("gz", ctypes.c_double),
        ("wall", ctypes.c_int32), ("axisym", ctypes.c_int32),
        ("precision", ctypes.c_int32), ("flags", ctypes.c_int32),
        ("rho_ref", ctypes.c_double),
    ]


def make_params(nz, nr, G=-5.5, tau=1.0, psi_rho0=1.0, gz=0.0, wall=WALL_NOSLIP, axisym=1,
                precision=FP64, rho_ref=0.0, flags=0):
    return Params(int(nz), int(nr), float(G), float(tau), float(psi_rho0), float(gz), int(wall),
                  int(axisym), int(precision), int(flags), float(rho_ref))


class LbmAxiError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"lbm_axi error {code}: {msg}")
        self.code = code


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(
            f"HIP library {LIB_PATH} is not built; run __graft_entry__.build() (hipcc, gfx950)")
    lib = ctypes.CDLL(LIB_PATH)
    vp, P = ctypes.c_void_p, ctypes.POINTER(Params)
    sigs = {
        "lbm_axi_check_params": (ctypes.c_int, [P]),
        "lbm_axi_workspace_bytes": (ctypes.c_size_t, [P]),
        "lbm_axi_create": (ctypes.c_int, [P, vp, vp, vp, vp, ctypes.c_size_t, vp, ctypes.POINTER(vp)]),
        "lbm_axi_step": (ctypes.c_int, [vp, ctypes.c_int64]),
        "lbm_axi_moments": (ctypes.c_int, [vp, vp, vp, vp]),
        "lbm_axi_reduce": (ctypes.c_int, [vp, ctypes.POINTER(ctypes.c_double)]),
        "lbm_axi_interface": (ctypes.c_int, [vp, ctypes.c_double, ctypes.c_int32, vp, ctypes.POINTER(ctypes.c_double)]),
        "lbm_axi_set_open": (ctypes.c_int, [vp, ctypes.c_int32, ctypes.c_double, vp, vp, ctypes.c_int32,
                                            ctypes.c_double]),
        "lbm_axi_drops": (ctypes.c_int, [vp, ctypes.c_double, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32),
                                         ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)]),
        "lbm_axi_populations": (ctypes.c_int, [vp, vp]),
        "lbm_axi_state_bytes": (ctypes.c_size_t, [vp]),
        "lbm_axi_get_state": (ctypes.c_int, [vp, vp]),
        "lbm_axi_set_state": (ctypes.c_int, [vp, vp]),
        "lbm_axi_record": (ctypes.c_int, [vp, ctypes.c_int64, vp]),
        "lbm_axi_set_kernel": (ctypes.c_int, [vp, ctypes.c_int32, ctypes.c_int32]),
        "lbm_axi_set_stream": (ctypes.c_int, [vp, vp]),
        "lbm_axi_set_coupling": (ctypes.c_int, [vp, ctypes.c_double, ctypes.c_double]),
        "lbm_axi_destroy": (None, [vp]),
        "lbm_axi_last_error": (ctypes.c_char_p, []),
    }
    for name, (res, args) in sigs.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


lib = _load()


def last_error():
    return lib.lbm_axi_last_error().decode()


class StabilityWarning(UserWarning):
    """Parameters outside the stability rule of thumb of Sec. II.D."""


def check(rc):
    if rc > 0:
        warnings.warn(last_error(), StabilityWarning, stacklevel=3)
        return rc
    if rc != OK:
        raise LbmAxiError(rc, last_error())
    return rc


def check_params(params):
    """Validate parameters without a device (lbm_axi_check_params): OK or
    WARN_STABILITY (with a warning), LbmAxiError otherwise."""
    return check(lib.lbm_axi_check_params(ctypes.byref(params)))


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _stream_handle(stream):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def workspace_bytes(params):
    return int(lib.lbm_axi_workspace_bytes(ctypes.byref(params)))


class AxiLBM:
    """One axisymmetric Shan–Chen lattice on one GPU.

    ``rho0``, ``uz0``, ``ur0`` are float64 tensors [nr, nz] (velocities may be
    None) on the device; the populations start at f^eq(rho0, u0).

    The library works on ``stream`` if one is given, else on the caller's
    current stream at each call.  With a stream of its own, every call that
    reads or writes caller tensors is ordered on both sides: the handle's
    stream first waits for the caller's (which may still use that memory),
    and the caller's stream then waits for the handle's work on it.
    """

    def __init__(self, params, rho0, uz0=None, ur0=None, device="cuda", stream=None):
        self.params = params
        self.device = torch.device(device)
        nbytes = workspace_bytes(params)
        if nbytes == 0:
            raise LbmAxiError(EINVAL, last_error())
        # uint8 storage; torch's caching allocator aligns blocks to >= 512 B
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self.stream = stream
        rho0 = self._field(rho0)
        uz0 = self._field(uz0) if uz0 is not None else None
        ur0 = self._field(ur0) if ur0 is not None else None
        h = ctypes.c_void_p()
        with self._handoff(sync=False):
            if self._own_stream():
                # the allocator reuses the workspace only after the
                # handle's stream has finished with it
                self.workspace.record_stream(self.stream)
            check(lib.lbm_axi_create(ctypes.byref(params), _ptr(rho0), _ptr(uz0), _ptr(ur0),
                                     _ptr(self.workspace), nbytes, _stream_handle(stream), ctypes.byref(h)))
        self._h = h
        self._keep = (rho0, uz0, ur0)  # inputs stay alive until the init kernel has run

    def _own_stream(self):
        return self.stream is not None and self.stream != torch.cuda.current_stream(self.device)

    @contextlib.contextmanager
    def _handoff(self, sync=True):
        """Stream order around a call that reads or writes caller tensors
        (see the class docstring); also points the handle at its stream."""
        cur = torch.cuda.current_stream(self.device)
        other = self._own_stream()
        if other:
            self.stream.wait_stream(cur)
        if sync:
            self._sync_stream()
        yield
        if other:
            cur.wait_stream(self.stream)

    def _field(self, a):
        t = torch.as_tensor(a, dtype=torch.float64, device=self.device).contiguous()
        if tuple(t.shape) != (self.params.nr, self.params.nz):
            raise ValueError(f"field shape {tuple(t.shape)} != (nr, nz) = ({self.params.nr}, {self.params.nz})")
        return t

    @property
    def nz(self):
        return self.params.nz

    @property
    def nr(self):
        return self.params.nr

    def _sync_stream(self):
        check(lib.lbm_axi_set_stream(self._h, _stream_handle(self.stream)))

    def step(self, n=1):
        self._sync_stream()
        check(lib.lbm_axi_step(self._h, int(n)))

    def moments(self):
        """(rho, u_z, u_r) float64 tensors [nr, nz] of the current state."""
        shape = (self.nr, self.nz)
        rho = torch.empty(shape, dtype=torch.float64, device=self.device)
        uz = torch.empty_like(rho)
        ur = torch.empty_like(rho)
        with self._handoff():
            check(lib.lbm_axi_moments(self._h, _ptr(rho), _ptr(uz), _ptr(ur)))
        return rho, uz, ur

    def reduce(self):
        """[3D mass, 3D z-momentum, kinetic energy, 2D mass] as Python floats
        (synchronises the stream)."""
        self._sync_stream()
        out = (ctypes.c_double * NREDUCE)()
        rc = lib.lbm_axi_reduce(self._h, out)
        vals = [float(v) for v in out]
        if rc == ENONFINITE:
            raise LbmAxiError(rc, last_error() + f" {vals}")
        check(rc)
        return vals

    def interface(self, rho_mid, z_col=None, radius_out=None):
        """Interface diagnostics (include/lbm_axi.h, lbm_axi_interface):
        dict with A, neck, r_max, rho_axis_min, rho_in, rho_out, dp; the
        radius profile R(z) goes into ``radius_out`` (float64 device tensor
        [nz]) if given.  Synchronises the stream."""
        z_col = self.nz // 2 if z_col is None else int(z_col)
        out = (ctypes.c_double * NINTERFACE)()
        with self._handoff():
            check(lib.lbm_axi_interface(self._h, float(rho_mid), z_col,
                                        _ptr(radius_out) if radius_out is not None else None, out))
        keys = ("A", "neck", "r_max", "rho_axis_min", "rho_in", "rho_out", "dp")
        return {k: float(v) for k, v in zip(keys, out)}

    def set_open(self, in_row=-1, rho_in=1.0, uz_in=None, ur_in=None, out_row=-1, rho_out=1.0):
        """Open boundaries (include/lbm_axi.h, lbm_axi_set_open): imposed
        f^eq(rho_in, u_in(z)) on row in_row, f^eq(rho_out, u one row inside)
        on row out_row; -1 turns a row off.  uz_in, ur_in: float64 arrays or
        tensors of nz values."""
        if in_row >= 0:
            uz = self._column(uz_in)
            ur = self._column(ur_in)
            self._open_keep = (uz, ur)  # alive until the stream has copied them
        else:
            uz = ur = None
        with self._handoff():
            check(lib.lbm_axi_set_open(self._h, int(in_row), float(rho_in), _ptr(uz), _ptr(ur), int(out_row),
                                       float(rho_out)))

    def _column(self, a):
        t = torch.as_tensor(a, dtype=torch.float64, device=self.device).contiguous()
        if tuple(t.shape) != (self.nz,):
            raise ValueError(f"profile shape {tuple(t.shape)} != (nz,) = ({self.nz},)")
        return t

    def drops(self, rho_mid, max_drops=MAX_DROPS):
        """Drops on the axis (include/lbm_axi.h, lbm_axi_drops): (n, volumes,
        centres) with n = -1 for an unbroken thread.  Synchronises the
        stream."""
        self._sync_stream()
        n = ctypes.c_int32()
        vol = (ctypes.c_double * max(1, max_drops))()
        cen = (ctypes.c_double * max(1, max_drops))()
        check(lib.lbm_axi_drops(self._h, float(rho_mid), int(max_drops), ctypes.byref(n), vol, cen))
        k = min(max(n.value, 0), max_drops)
        return n.value, [float(v) for v in vol[:k]], [float(c) for c in cen[:k]]

    def state_bytes(self):
        return int(lib.lbm_axi_state_bytes(self._h))

    def get_state(self, out=None):
        """Copy of the populations (the library's storage type, [9][nr][nz]);
        into ``out`` (a contiguous device tensor of state_bytes bytes) if
        given."""
        if out is None:
            out = torch.empty(self.state_bytes(), dtype=torch.uint8, device=self.device)
        elif out.numel() * out.element_size() != self.state_bytes() or not out.is_contiguous():
            raise ValueError("state buffer of the wrong size or not contiguous")
        with self._handoff():
            check(lib.lbm_axi_get_state(self._h, _ptr(out)))
        return out

    def set_state(self, src):
        if src.numel() * src.element_size() != self.state_bytes() or not src.is_contiguous():
            raise ValueError("state buffer of the wrong size or not contiguous")
        with self._handoff():
            check(lib.lbm_axi_set_state(self._h, _ptr(src)))

    def record(self, n, out):
        """Write the states f^t .. f^{t+n-1} into ``out`` (a contiguous
        device tensor of n * state_bytes bytes) and leave the lattice at
        f^{t+n-1}."""
        if n < 1 or out.numel() * out.element_size() != n * self.state_bytes() or not out.is_contiguous():
            raise ValueError("record buffer of the wrong size or not contiguous")
        with self._handoff():
            check(lib.lbm_axi_record(self._h, int(n), _ptr(out)))

    def populations(self):
        """Current populations f_i as a float64 tensor [9, nr, nz], decoded
        by the library (lbm_axi_populations: the shift is added back in FP32
        storage)."""
        out = torch.empty((9, self.nr, self.nz), dtype=torch.float64, device=self.device)
        with self._handoff():
            check(lib.lbm_axi_populations(self._h, _ptr(out)))
        return out

    def set_kernel(self, kind, chunk_rows=48):
        """Step kernel: KERNEL_TILE, KERNEL_STRIP with chunks of chunk_rows
        rows, KERNEL_TILE_ALTERNATE, KERNEL_TILE_COLUMNS or
        KERNEL_TILE_PAIRS (include/lbm_axi.h, lbm_axi_set_kernel)."""
        check(lib.lbm_axi_set_kernel(self._h, int(kind), int(chunk_rows)))

    def set_coupling(self, G, tau):
        check(lib.lbm_axi_set_coupling(self._h, float(G), float(tau)))
        self.params.G = float(G)
        self.params.tau = float(tau)

    def close(self):
        if getattr(self, "_h", None):
            lib.lbm_axi_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
