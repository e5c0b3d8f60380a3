"""ctypes binding of the batched-ensemble C ABI (include/lbm_axi_batch.h).

Argument marshalling only: the ensemble runs in the HIP library (one
persistent launch per step, replayed from a captured HIP graph on a
non-default stream).  Device memory comes from torch.
"""
import contextlib
import ctypes

import torch

from . import lbm_axi as L

_lib = L.lib
_vp = ctypes.c_void_p
_i32 = ctypes.c_int32
_sigs = {
    "lbm_axi_batch_workspace_bytes": (ctypes.c_size_t, [ctypes.POINTER(L.Params), _i32]),
    "lbm_axi_batch_create": (ctypes.c_int, [ctypes.POINTER(L.Params), _i32, ctypes.POINTER(_vp), _vp,
                                            ctypes.c_size_t, _vp, ctypes.POINTER(_vp)]),
    "lbm_axi_batch_step": (ctypes.c_int, [_vp, ctypes.c_int64]),
    "lbm_axi_batch_step_per_instance": (ctypes.c_int, [_vp, ctypes.c_int64]),
    "lbm_axi_batch_moments": (ctypes.c_int, [_vp, _i32, _vp, _vp, _vp]),
    "lbm_axi_batch_get_state": (ctypes.c_int, [_vp, _i32, _vp]),
    "lbm_axi_batch_populations": (ctypes.c_int, [_vp, _i32, _vp]),
    "lbm_axi_batch_num_configs": (_i32, [_vp]),
    "lbm_axi_batch_config_info": (ctypes.c_int, [_vp, _i32, ctypes.POINTER(_i32), ctypes.POINTER(_i32),
                                                 ctypes.POINTER(_i32)]),
    "lbm_axi_batch_set_schedule": (ctypes.c_int, [_vp, _i32, _i32, _i32]),
    "lbm_axi_batch_autotune": (ctypes.c_int, [_vp, _i32, ctypes.POINTER(_i32), ctypes.POINTER(ctypes.c_double)]),
    "lbm_axi_batch_nodes": (ctypes.c_int64, [_vp]),
    "lbm_axi_batch_destroy": (None, [_vp]),
}
for _name, (_res, _args) in _sigs.items():
    _fn = getattr(_lib, _name)
    _fn.restype = _res
    _fn.argtypes = _args


class AxiBatch:
    """Independent lattices advanced together.

    ``params``: list of lbm_axi Params (same precision); ``rho0``: list of
    float64 device tensors [nr, nz].  The batch issues its work on ``stream``
    (default: a new non-default torch stream, so steps are graph-replayed).
    Calls that read or write caller tensors are ordered on both sides: the
    batch's stream first waits for the caller's current stream (which may
    still use that memory), and the caller's stream then waits for the
    batch's work on it."""

    def __init__(self, params, rho0, device="cuda", stream=None):
        n = len(params)
        if len(rho0) != n:
            raise ValueError(f"{len(rho0)} initial densities for {n} instances")
        self.params = list(params)
        arr = (L.Params * n)(*params)
        self._arr = arr
        nbytes = int(_lib.lbm_axi_batch_workspace_bytes(arr, n))
        if nbytes == 0:
            raise L.LbmAxiError(L.EINVAL, L.last_error())
        self.device = torch.device(device)
        self.stream = stream if stream is not None else torch.cuda.Stream(device=self.device)
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self._rho0 = [torch.as_tensor(r, dtype=torch.float64, device=self.device).contiguous() for r in rho0]
        for p, r in zip(params, self._rho0):
            if tuple(r.shape) != (p.nr, p.nz):
                raise ValueError("rho0 shape does not match its parameters")
        ptrs = (_vp * n)(*[r.data_ptr() for r in self._rho0])
        h = _vp()
        with self._handoff():
            # the allocator reuses the workspace only after the batch's
            # stream has finished with it
            self.workspace.record_stream(self.stream)
            L.check(_lib.lbm_axi_batch_create(arr, n, ptrs, _vp(self.workspace.data_ptr()), nbytes,
                                              _vp(self.stream.cuda_stream), ctypes.byref(h)))
        self._h = h
        self.n = n

    @contextlib.contextmanager
    def _handoff(self):
        """Stream order around a call that reads or writes caller tensors
        (see the class docstring)."""
        cur = torch.cuda.current_stream(self.device)
        other = self.stream != cur
        if other:
            self.stream.wait_stream(cur)
        yield
        if other:
            cur.wait_stream(self.stream)

    def nodes(self):
        return int(_lib.lbm_axi_batch_nodes(self._h))

    def step(self, n=1):
        L.check(_lib.lbm_axi_batch_step(self._h, int(n)))

    def step_per_instance(self, n=1):
        L.check(_lib.lbm_axi_batch_step_per_instance(self._h, int(n)))

    def set_schedule(self, config, grid_per_cu, order):
        L.check(_lib.lbm_axi_batch_set_schedule(self._h, int(config), int(grid_per_cu), int(order)))

    def configs(self):
        out = []
        for c in range(_lib.lbm_axi_batch_num_configs(self._h)):
            tz, tr, nt = _i32(), _i32(), _i32()
            L.check(_lib.lbm_axi_batch_config_info(self._h, c, ctypes.byref(tz), ctypes.byref(tr), ctypes.byref(nt)))
            out.append((tz.value, tr.value, nt.value))
        return out

    def autotune(self, steps_per_trial=4):
        """Time every schedule on the batch, keep the fastest; returns
        ((config, grid_per_cu, order), microseconds per step)."""
        ch = (_i32 * 3)()
        us = ctypes.c_double()
        L.check(_lib.lbm_axi_batch_autotune(self._h, int(steps_per_trial), ch, ctypes.byref(us)))
        return (ch[0], ch[1], ch[2]), us.value

    def moments(self, k):
        p = self.params[k]
        rho = torch.empty((p.nr, p.nz), dtype=torch.float64, device=self.device)
        uz = torch.empty_like(rho)
        ur = torch.empty_like(rho)
        with self._handoff():
            L.check(_lib.lbm_axi_batch_moments(self._h, int(k), _vp(rho.data_ptr()), _vp(uz.data_ptr()),
                                               _vp(ur.data_ptr())))
        return rho, uz, ur

    def populations(self, k):
        """Instance k's populations f_i as float64 [9, nr, nz], decoded by
        the library (lbm_axi_batch_populations: the shift is added back in
        FP32 storage)."""
        p = self.params[k]
        out = torch.empty((9, p.nr, p.nz), dtype=torch.float64, device=self.device)
        with self._handoff():
            L.check(_lib.lbm_axi_batch_populations(self._h, int(k), _vp(out.data_ptr())))
        return out

    def synchronize(self):
        self.stream.synchronize()

    def close(self):
        if getattr(self, "_h", None):
            self.stream.synchronize()
            _lib.lbm_axi_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
