"""Reverse-mode gradients of an interface-shape loss through the axisymmetric
Shan–Chen lattice Boltzmann run (FP64), on top of the C ABI in
include/lbm_axi_adjoint.h.

Loss: L = sum over sample steps t = every, 2 every, ..., T of
sum_m (r(theta_m, t) - r_target(theta_m, t))^2, with r(theta) the
ray-integral interface radius of the density.  Gradients with respect to the
initial density field, G and tau come from the hand-written adjoint kernels
with checkpoint-every-K recomputation; this module only sequences the calls
and holds device buffers (torch) -- every arithmetic step runs in the HIP
library.
"""
import ctypes
import math

import torch

from . import lbm_axi as L

_lib = L.lib
_vp = ctypes.c_void_p
_i32 = ctypes.c_int32
_d = ctypes.c_double
_sigs = {
    "lbm_axi_adjoint_workspace_bytes": (ctypes.c_size_t, [_i32, _i32]),
    "lbm_axi_adjoint_step": (ctypes.c_int, [ctypes.POINTER(L.Params), _vp, _vp, _vp, _vp, _vp, ctypes.c_size_t, _vp]),
    "lbm_axi_adjoint_run": (ctypes.c_int, [ctypes.POINTER(L.Params), _vp, _i32, _vp, _vp, _vp, _vp, ctypes.c_size_t,
                                           _vp]),
    "lbm_axi_init_vjp": (ctypes.c_int, [_vp, _vp, _vp, _i32, _i32, _vp, _vp]),
    "lbm_axi_density": (ctypes.c_int, [_vp, _i32, _i32, _vp, _vp]),
    "lbm_axi_ray_weights": (ctypes.c_int, [_i32, _i32, _d, _vp, _i32, _d, _d, _i32, _vp, _vp, _vp, _vp, _vp, _vp,
                                           _vp, ctypes.POINTER(_i32), ctypes.POINTER(_i32)]),
    "lbm_axi_ray_forward": (ctypes.c_int, [_vp, _i32, _vp, _vp, _vp, _d, _d, _vp, _vp]),
    "lbm_axi_ray_vjp": (ctypes.c_int, [_vp, _i32, _vp, _vp, _vp, _vp, _d, _d, _i32, _i32, _vp, _vp]),
    "lbm_axi_misfit": (ctypes.c_int, [_vp, _vp, _i32, _vp, _vp, _vp]),
}
for _name, (_res, _args) in _sigs.items():
    _fn = getattr(_lib, _name)
    _fn.restype = _res
    _fn.argtypes = _args


def _p(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _s():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _check(rc):
    if rc != L.OK:
        raise L.LbmAxiError(rc, L.last_error())


class RayProbe:
    """Ray-integral interface radius r(theta_m) of a density field: a sparse
    linear map built by the library on the host and kept on the device."""

    def __init__(self, nz, nr, zc, thetas, rho_l, rho_g, ds=0.5, s_max=None, device="cuda"):
        if s_max is None:
            s_max = min(nz / 2.0, float(nr)) - 1.0
        self.nz, self.nr = int(nz), int(nr)
        self.rho_l, self.rho_g = float(rho_l), float(rho_g)
        th = (ctypes.c_double * len(thetas))(*[float(t) for t in thetas])
        self.m = len(thetas)
        nnz, nn = _i32(), _i32()
        _check(_lib.lbm_axi_ray_weights(self.nz, self.nr, float(zc), th, self.m, float(ds), float(s_max), 0,
                                        None, None, None, None, None, None, None, ctypes.byref(nnz), ctypes.byref(nn)))
        cap = nnz.value
        rp = (_i32 * (self.m + 1))()
        col = (_i32 * cap)()
        val = (ctypes.c_double * cap)()
        npt = (_i32 * (nn.value + 1))()
        nodes = (_i32 * nn.value)()
        nrow = (_i32 * cap)()
        nval = (ctypes.c_double * cap)()
        _check(_lib.lbm_axi_ray_weights(self.nz, self.nr, float(zc), th, self.m, float(ds), float(s_max), cap,
                                        rp, col, val, npt, nodes, nrow, nval, ctypes.byref(nnz), ctypes.byref(nn)))
        dev = torch.device(device)
        i32 = lambda a: torch.tensor(list(a), dtype=torch.int32, device=dev)
        f64 = lambda a: torch.tensor(list(a), dtype=torch.float64, device=dev)
        self.row_ptr, self.col, self.val = i32(rp), i32(col), f64(val)
        self.node_ptr, self.nodes, self.node_row, self.node_val = i32(npt), i32(nodes), i32(nrow), f64(nval)
        self.n_nodes = nn.value
        self._rho = torch.empty((self.nr, self.nz), dtype=torch.float64, device=dev)

    def radius_of_state(self, f, out):
        """out[m] = r(theta_m) of the density of state f ([9, nr, nz] FP64)."""
        _check(_lib.lbm_axi_density(_p(f), self.nz, self.nr, _p(self._rho), _s()))
        _check(_lib.lbm_axi_ray_forward(_p(self._rho), self.m, _p(self.row_ptr), _p(self.col), _p(self.val),
                                        self.rho_l, self.rho_g, _p(out), _s()))

    def add_vjp(self, rbar, lam):
        """lam += d(sum_m rbar_m r_m)/d f (same value in every direction)."""
        _check(_lib.lbm_axi_ray_vjp(_p(rbar), self.n_nodes, _p(self.node_ptr), _p(self.node_row),
                                    _p(self.node_val), _p(self.nodes), self.rho_l, self.rho_g, self.nz, self.nr,
                                    _p(lam), _s()))


def _params(nz, nr, G, tau, wall, axisym, gz=0.0):
    return L.make_params(nz, nr, G=G, tau=tau, wall=wall, axisym=axisym, gz=gz, precision=L.FP64)


def _state_view(sim):
    return sim.get_state().view(torch.float64).reshape(9, sim.nr, sim.nz)


def radius_history(rho0, G, tau, probe, steps, every, wall=0, axisym=1):
    """r(theta_m, t) at t = every, 2 every, ..., steps (FP64, [n_samples, m])."""
    nz, nr = probe.nz, probe.nr
    sim = L.AxiLBM(_params(nz, nr, G, tau, wall, axisym), rho0)
    out = torch.zeros((steps // every, probe.m), dtype=torch.float64, device=rho0.device)
    for k in range(steps // every):
        sim.step(every)
        probe.radius_of_state(_state_view(sim), out[k])
    sim.close()
    return out


def adjoint_step(params, f, lam_next, lam, grad_acc, ws):
    _check(_lib.lbm_axi_adjoint_step(ctypes.byref(params), _p(f), _p(lam_next), _p(lam), _p(grad_acc), _p(ws),
                                     ws.numel() * ws.element_size(), _s()))


def adjoint_run(params, states, k, lam, tmp, grad_acc, ws):
    """k reverse steps over states[0..k) (lam: lam^{t0+k} in, lam^{t0} out)."""
    _check(_lib.lbm_axi_adjoint_run(ctypes.byref(params), _p(states), int(k), _p(lam), _p(tmp), _p(grad_acc), _p(ws),
                                    ws.numel() * ws.element_size(), _s()))


# The backward pass recomputes each checkpoint segment on a second stream
# while the previous segment is reversed, on lattices of at most this many
# nodes: there neither the forward steps nor the reverse steps fill the GPU
# (256 x 128: (forward + backward) / forward 3.57 -> 2.81, 384 x 192 4.40 ->
# 3.80, 512 x 256 4.65 -> 4.07); on 1024 x 512 and 2048 x 1024 it changed
# nothing beyond the run-to-run spread.  Set to 0 to keep one stream.
OVERLAP_MAX_NODES = 1 << 18
_side_streams = {}


def _side_stream(dev):
    """One recompute stream per device (default priority), made once."""
    idx = torch.device(dev).index
    idx = torch.cuda.current_device() if idx is None else idx
    if idx not in _side_streams:
        _side_streams[idx] = torch.cuda.Stream(device=idx)
    return _side_streams[idx]


class ShapeLoss(torch.autograd.Function):
    """loss = sum_t sum_m (r(theta_m, t) - target[t, m])^2 of a run started
    from f^eq(rho0, 0); differentiable in rho0, G and tau.

    Checkpoints the state every ``checkpoint`` steps in the forward pass and
    recomputes each segment's states in the backward pass."""

    @staticmethod
    def forward(ctx, rho0, G, tau, probe, target, steps, every, checkpoint, wall, axisym):
        G_, tau_ = float(G), float(tau)
        nz, nr = probe.nz, probe.nr
        assert steps % every == 0 and steps % checkpoint == 0
        params = _params(nz, nr, G_, tau_, wall, axisym)
        sim = L.AxiLBM(params, rho0.detach())
        dev = rho0.device
        loss = torch.zeros(1, dtype=torch.float64, device=dev)
        nsamp = steps // every
        rbar = torch.zeros((nsamp, probe.m), dtype=torch.float64, device=dev)
        r = torch.empty(probe.m, dtype=torch.float64, device=dev)
        ckpts = []
        t = 0
        while t < steps:
            if t % checkpoint == 0:
                ckpts.append(_state_view(sim).clone())
            # advance to the next checkpoint or sample step in one call
            nxt = min((t // every + 1) * every, (t // checkpoint + 1) * checkpoint, steps)
            sim.step(nxt - t)
            t = nxt
            if t % every == 0:
                k = t // every - 1
                probe.radius_of_state(_state_view(sim), r)
                _check(_lib.lbm_axi_misfit(_p(r), _p(target[k]), probe.m, _p(loss), _p(rbar[k]), _s()))
        sim.close()
        ctx.save_for_backward(rho0)
        ctx.meta = (params, probe, rbar, ckpts, steps, every, checkpoint)
        return loss[0].clone()

    @staticmethod
    def backward(ctx, gout):
        (rho0,) = ctx.saved_tensors
        params, probe, rbar, ckpts, steps, every, checkpoint = ctx.meta
        nz, nr = probe.nz, probe.nr
        dev = rho0.device
        ws = torch.empty(_lib.lbm_axi_adjoint_workspace_bytes(nz, nr) // 8, dtype=torch.float64, device=dev)
        grad_acc = torch.zeros(2, dtype=torch.float64, device=dev)
        lam_a = torch.zeros((9, nr, nz), dtype=torch.float64, device=dev)
        lam_b = torch.zeros_like(lam_a)
        scaled_rbar = rbar * gout.to(torch.float64)
        # lam currently holds dL/df^T (T = steps)
        if steps % every == 0:
            probe.add_vjp(scaled_rbar[steps // every - 1], lam_a)
        # The states of segment s - 1 are recomputed (on a second stream on
        # small lattices, see OVERLAP_MAX_NODES) while the reverse sweep of
        # segment s runs on this one: two state buffers, ordered by events.
        # The reverse sweep, and so every accumulation, keeps its order on
        # this stream, so the gradients do not depend on the overlap.
        main = torch.cuda.current_stream(dev)
        side = _side_stream(dev) if nz * nr <= OVERLAP_MAX_NODES else main
        side.wait_stream(main)
        bufs = [torch.empty((checkpoint, 9, nr, nz), dtype=torch.float64, device=dev) for _ in range(2)]
        swept = [None, None]  # event after the last reverse sweep that read each buffer
        recorded = {}
        with torch.cuda.stream(side):
            sim = L.AxiLBM(params, rho0.detach())

        def recompute(s):
            # the states f^t, t0 <= t < t0 + checkpoint, in one call
            b = s % 2
            with torch.cuda.stream(side):
                if swept[b] is not None:
                    side.wait_event(swept[b])
                sim.set_state(ckpts[s].reshape(-1).view(torch.uint8))
                sim.record(checkpoint, bufs[b])
                recorded[s] = torch.cuda.Event()
                recorded[s].record(side)

        nseg = len(ckpts)
        if nseg:
            recompute(nseg - 1)
        for s in reversed(range(nseg)):
            if s > 0:
                recompute(s - 1)
            main.wait_event(recorded.pop(s))
            seg_states = bufs[s % 2]
            t0 = s * checkpoint
            # reverse sweep in runs between sample steps; after lam^t is
            # formed at a sample step t > 0, its misfit VJP is added
            hi = checkpoint
            for j in range(checkpoint - 1, 0, -1):
                if (t0 + j) % every == 0:
                    adjoint_run(params, seg_states[j], hi - j, lam_a, lam_b, grad_acc, ws)
                    probe.add_vjp(scaled_rbar[(t0 + j) // every - 1], lam_a)
                    hi = j
            adjoint_run(params, seg_states[0], hi, lam_a, lam_b, grad_acc, ws)
            if t0 > 0 and t0 % every == 0:
                probe.add_vjp(scaled_rbar[t0 // every - 1], lam_a)
            swept[s % 2] = torch.cuda.Event()
            swept[s % 2].record(main)
        # the side stream's work is complete once main has waited for the
        # last recompute; the buffers and the handle were used on both
        main.wait_stream(side)
        for b in bufs:
            b.record_stream(side)
        sim.close()
        rho_bar = torch.empty((nr, nz), dtype=torch.float64, device=dev)
        _check(_lib.lbm_axi_init_vjp(_p(lam_a), None, None, nz, nr, _p(rho_bar), _s()))
        g = grad_acc.to(torch.float64)
        return rho_bar, g[0].reshape(()), g[1].reshape(()), None, None, None, None, None, None, None


def shape_loss(rho0, G, tau, probe, target, steps, every=50, checkpoint=100, wall=0, axisym=1):
    """Differentiable interface-shape loss (see ShapeLoss)."""
    if not torch.is_tensor(G):
        G = torch.tensor(float(G), dtype=torch.float64, device=rho0.device)
    if not torch.is_tensor(tau):
        tau = torch.tensor(float(tau), dtype=torch.float64, device=rho0.device)
    return ShapeLoss.apply(rho0, G, tau, probe, target, steps, every, checkpoint, wall, axisym)


def default_thetas(m=16):
    """theta_m = (m + 1/2) pi / M, m < M: rays over the half plane r > 0."""
    return [(k + 0.5) * math.pi / m for k in range(m)]
