"""Batched ensemble on the GPU: every instance of a batch matches the oracle
(FP64) and is bitwise equal to the same instance advanced by ordinary
per-instance launches, by a batch of one, by direct (non-graph) launches and
under every schedule the autotuner may pick."""
import numpy as np
import pytest
import torch

import oracle as O
from lbm_inputs import coexistence_densities, drop_density, ensemble, random_state_fields, thread_density

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)


def _libs():
    from paper_1310_1871_amd import batch as B
    from paper_1310_1871_amd import lbm_axi as L
    return L, B


def _small_ensemble(precision, n=6, seed=3):
    L, _ = _libs()
    rng = np.random.Generator(np.random.PCG64(seed))
    sizes = [(64, 32), (100, 37), (128, 64), (70, 6), (33, 20), (256, 16)]
    params, rhos, meta = [], [], []
    for k in range(n):
        nz, nr = sizes[k % len(sizes)]
        G = float(rng.uniform(-5.5, -5.0))
        tau = float(rng.uniform(0.85, 1.0))
        rg, rl = coexistence_densities(round(G, 6))
        if k % 2 == 0:
            rho = drop_density(nz, nr, nz / 2.0, 0.3 * nr + 2, rl, rg, 2.0, {2: 1.0})
        else:
            rho = thread_density(nz, nr, 0.3 * nr + 1, rl, rg, 2.0, 0.1, 1)
        wall = k % 2
        params.append(L.make_params(nz, nr, G=G, tau=tau, wall=wall, precision=precision,
                                    rho_ref=rl if precision == L.FP32_SHIFTED else 0.0))
        rhos.append(torch.from_numpy(rho).cuda())
        meta.append((nz, nr, G, tau, wall, rho))
    return params, rhos, meta


def test_fp64_batch_matches_oracle():
    L, B = _libs()
    params, rhos, meta = _small_ensemble(L.FP64)
    _say("fp64 batch of 6, 200 steps, vs oracle")
    b = B.AxiBatch(params, rhos)
    b.step(200)
    for k, (nz, nr, G, tau, wall, rho) in enumerate(meta):
        rg_, uzg, urg = (t.cpu().numpy() for t in b.moments(k))
        p = O.make_params(nz, nr, G=G, tau=tau, wall=wall)
        ro, uzo, uro = O.moments(p, O.run(p, O.equilibrium(p, rho, 0 * rho, 0 * rho), 200))
        err = max(np.abs(rg_ - ro).max(), np.abs(uzg - uzo).max(), np.abs(urg - uro).max())
        _say(f"  instance {k} ({nz}x{nr}) max err {err:.2e}")
        assert err < 1e-10
    b.close()


def test_guo_forcing_batch_matches_oracle():
    """Instances with the Guo forcing option mixed with default ones in one
    batch (FP64): each against the oracle with its own forcing."""
    L, B = _libs()
    cases = [(64, 32, -5.5, 1.0, 0, L.FLAG_GUO), (96, 40, -5.0, 0.9, 1, 0), (70, 24, -5.5, 1.0, 1, L.FLAG_GUO)]
    params, rhos, raw = [], [], []
    for nz, nr, G, tau, wall, flags in cases:
        rg, rl = coexistence_densities(G)
        rho = drop_density(nz, nr, nz / 2.0, 0.3 * nr, rl, rg, 2.0)
        params.append(L.make_params(nz, nr, G=G, tau=tau, wall=wall, flags=flags))
        rhos.append(torch.from_numpy(rho).cuda())
        raw.append(rho)
    _say("guo batch of 3, 200 steps, vs oracle")
    b = B.AxiBatch(params, rhos)
    b.step(200)
    for k, ((nz, nr, G, tau, wall, flags), rho) in enumerate(zip(cases, raw)):
        rg_, uzg, urg = (t.cpu().numpy() for t in b.moments(k))
        p = O.make_params(nz, nr, G=G, tau=tau, wall=wall, flags=flags)
        ro, uzo, uro = O.moments(p, O.run(p, O.equilibrium(p, rho, 0 * rho, 0 * rho), 200))
        err = max(np.abs(rg_ - ro).max(), np.abs(uzg - uzo).max(), np.abs(urg - uro).max())
        _say(f"  instance {k} flags {flags} max err {err:.2e}")
        assert err < 1e-10
    b.close()


def test_zwalls_batch_matches_oracle():
    """Instances closed by z walls (alone and with the Guo forcing) mixed
    with a periodic one in one batch (FP64): each against the oracle."""
    L, B = _libs()
    cases = [(64, 32, -5.5, 1.0, 0, L.FLAG_ZWALLS), (96, 40, -5.0, 0.9, 1, 0),
             (70, 24, -5.5, 1.0, 1, L.FLAG_ZWALLS | L.FLAG_GUO)]
    params, rhos, raw = [], [], []
    for nz, nr, G, tau, wall, flags in cases:
        rg, rl = coexistence_densities(G)
        rho = drop_density(nz, nr, nz / 3.0, 0.3 * nr, rl, rg, 2.0)
        params.append(L.make_params(nz, nr, G=G, tau=tau, wall=wall, flags=flags))
        rhos.append(torch.from_numpy(rho).cuda())
        raw.append(rho)
    _say("z-wall batch of 3, 200 steps, vs oracle")
    b = B.AxiBatch(params, rhos)
    b.step(200)
    for k, ((nz, nr, G, tau, wall, flags), rho) in enumerate(zip(cases, raw)):
        rg_, uzg, urg = (t.cpu().numpy() for t in b.moments(k))
        p = O.make_params(nz, nr, G=G, tau=tau, wall=wall, flags=flags)
        ro, uzo, uro = O.moments(p, O.run(p, O.equilibrium(p, rho, 0 * rho, 0 * rho), 200))
        err = max(np.abs(rg_ - ro).max(), np.abs(uzg - uzo).max(), np.abs(urg - uro).max())
        _say(f"  instance {k} flags {flags} max err {err:.2e}")
        assert err < 1e-10
    b.close()


@pytest.mark.parametrize("precision", [0, 1])
def test_batch_bitwise_equals_per_instance_and_solo(precision):
    L, B = _libs()
    params, rhos, meta = _small_ensemble(precision)
    _say(f"bitwise batch test precision={precision}")
    ref = B.AxiBatch(params, rhos)
    ref.step(50)
    per = B.AxiBatch(params, rhos)
    per.step_per_instance(50)
    for k in range(len(params)):
        a, c = ref.populations(k), per.populations(k)
        assert torch.equal(a, c), k
        solo = B.AxiBatch([params[k]], [rhos[k]])
        solo.step(50)
        assert torch.equal(a, solo.populations(0)), k
        solo.close()
    ref.close()
    per.close()


def test_instances_beyond_4gib_of_the_workspace():
    """Three FP64 instances of 16383 x 1500 (1.77 GB per population buffer):
    the first buffer of the third instance straddles 4 GiB from the start
    of the batch workspace and every second buffer lies beyond it (14.8 GiB
    in all), while each buffer stays below the 4 GiB reach of the kernels'
    32-bit offsets.  After 6 steps every instance equals a one-instance
    batch of it, bit for bit, so nothing on the host or in the work list
    truncates an instance's place in the workspace."""
    L, B = _libs()
    nz, nr = 16383, 1500
    params, rhos = [], []
    for k in range(3):
        # a random field of 127 columns, repeated 129 times along z
        rho, _, _ = random_state_fields(70 + k, 127, nr, rho_lo=0.4, rho_hi=1.8, u_amp=0.0)
        params.append(L.make_params(nz, nr, G=-4.5, tau=0.9, wall=k % 2))
        rhos.append(torch.from_numpy(rho).cuda().repeat(1, nz // 127).contiguous())
    _say("batch instances beyond 4 GiB: 3 x 16383x1500 FP64")
    big = B.AxiBatch(params, rhos)
    big.step(6)
    for k in range(3):
        solo = B.AxiBatch([params[k]], [rhos[k]])
        solo.step(6)
        a, c = big.populations(k), solo.populations(0)
        _say(f"  instance {k}: max |df| = {(a - c).abs().max().item():.3e}")
        assert torch.equal(a, c), k
        del a, c
        solo.close()
    big.close()


def test_graph_replay_equals_direct_launches():
    """Graph replays (non-default stream) against direct launches (null
    stream), checked after every replay with eager work in between."""
    L, B = _libs()
    params, rhos, _ = _small_ensemble(L.FP32_SHIFTED)
    g = B.AxiBatch(params, rhos)
    d = B.AxiBatch(params, rhos, stream=torch.cuda.default_stream())
    _say("graph replay vs direct")
    for rep in range(4):
        g.step(6)
        d.step(6)
        for k in range(len(params)):
            assert torch.equal(g.populations(k), d.populations(k)), (rep, k)
        _ = torch.ones(1000, device="cuda").sum().item()  # eager work between replays
    g.close()
    d.close()


def test_outputs_are_ordered_on_the_callers_stream():
    """moments and populations of a batch on its own stream, reduced on the
    caller's stream as soon as they return and freed at once (the allocator
    hands their memory to the next call), with steps in between: equal to
    the same batch run on the caller's stream, bit for bit."""
    L, B = _libs()
    params, rhos, _ = _small_ensemble(L.FP64)
    g = B.AxiBatch(params, rhos)
    d = B.AxiBatch(params, rhos, stream=torch.cuda.current_stream())
    _say("batch outputs on the caller's stream")
    got, want = [], []
    for rep in range(5):
        g.step(3)
        d.step(3)
        for b, acc in ((g, got), (d, want)):
            for k in range(len(params)):
                rho, uz, ur = b.moments(k)
                acc.append(torch.stack([rho.sum(), uz.abs().sum(), ur.abs().sum()]))
                del rho, uz, ur
                acc.append(b.populations(k).sum(dim=(1, 2)))
    assert torch.equal(torch.cat(got).cpu(), torch.cat(want).cpu())
    g.close()
    d.close()


def test_batch_step_captured_into_a_caller_graph():
    """lbm_axi_batch_step on the batch's stream while the caller captures
    it (torch.cuda.graph on that stream): the persistent launches go into
    the caller's graph, an odd step count is refused there, and each of
    several replays, with eager work between them, equals eager steps of a
    second batch bit for bit."""
    L, B = _libs()
    params, rhos, _ = _small_ensemble(L.FP64)
    s = torch.cuda.Stream()
    cap = B.AxiBatch(params, rhos, stream=s)
    ref = B.AxiBatch(params, rhos)
    cap.step(2)  # the batch's own graphs exist before the capture
    ref.step(2)
    torch.cuda.synchronize()
    _say("caller graph capture of lbm_axi_batch_step")
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        with pytest.raises(L.LbmAxiError) as e:
            cap.step(5)
        cap.step(4)
    assert e.value.code == L.EINVAL
    for rep in range(3):
        g.replay()
        ref.step(4)
        _ = torch.ones(1000, device="cuda").sum().item()  # eager work between the replays
        for k in range(len(params)):
            assert torch.equal(cap.populations(k), ref.populations(k)), (rep, k)
    cap.close()
    ref.close()


def test_schedules_agree_and_autotune_restores_state():
    L, B = _libs()
    params, rhos, _ = _small_ensemble(L.FP32_SHIFTED)
    b = B.AxiBatch(params, rhos)
    b.step(10)
    before = [b.populations(k) for k in range(len(params))]
    choice, us = b.autotune(steps_per_trial=2)
    _say(f"autotune choice {choice} {us:.1f} us/step, configs {b.configs()}")
    after = [b.populations(k) for k in range(len(params))]
    for x, y in zip(before, after):
        assert torch.equal(x, y)
    # with one kernel configuration, the grid size and the work-list order
    # only change which workgroup computes a tile: bitwise equal results
    outs = {}
    for sched in [(1, 1, 0), (1, 3, 1), (1, 4, 2), (2, 2, 1), (3, 4, 0)]:
        c = B.AxiBatch(params, rhos)
        c.set_schedule(*sched)
        c.step(20)
        outs[sched] = [c.populations(k) for k in range(len(params))]
        c.close()
    for sched in [(1, 3, 1), (1, 4, 2)]:
        for x, y in zip(outs[(1, 1, 0)], outs[sched]):
            assert torch.equal(x, y)
    # other tile shapes are other compiled kernels whose FP32 rounding
    # differs (contraction into FMAs, order of sums): after 20 steps the
    # populations agree to a few ulp of the stored magnitudes (~1e-7 each
    # step), far below any indexing or boundary mistake (>= 1e-3)
    for sched in [(2, 2, 1), (3, 4, 0)]:
        diff = max(float((x - y).abs().max()) for x, y in zip(outs[(1, 1, 0)], outs[sched]))
        _say(f"schedule {sched} vs (1, 1, 0): max |d f| = {diff:.3e}")
        assert diff < 1e-5
    b.close()


def test_full_ensemble_runs_finite():
    """The 256-instance ensemble (FP32 shifted storage) stays finite."""
    L, B = _libs()
    cases = ensemble()
    params = [L.make_params(c.nz, c.nr, G=c.G, tau=c.tau, wall=c.wall, precision=L.FP32_SHIFTED, rho_ref=c.rho_l)
              for c in cases]
    _say(f"full ensemble: {len(cases)} instances")
    b = B.AxiBatch(params, [torch.from_numpy(c.rho).cuda() for c in cases])
    b.step(500)
    for k in range(0, len(cases), 17):
        rho, uz, ur = b.moments(k)
        assert torch.isfinite(rho).all() and torch.isfinite(uz).all(), k
        assert float(uz.abs().max()) < 0.2
    b.close()


@pytest.mark.parametrize("prec_name,nz,nr", [("fp32", 4096, 512), ("fp32", 4100, 515), ("fp64", 4100, 515)])
def test_large_lattice_path_matches_batch_kernel(prec_name, nz, nr):
    """The single-lattice step on a large lattice uses 64 x 16 tiles of 512
    threads: in FP32 each XCD takes a slab of tile columns (4096 x 512), or
    runs of whole tile rows when 8 does not divide the tile columns (65 of
    them at 4100 x 515); in FP64 runs of tile rows.  The batch kernel with
    its 64 x 16 / 512 configuration runs the same tile body with another
    mapping of workgroups to tiles and another store policy, so after 4
    steps the two must agree bit for bit: a tile done twice, or left out,
    would show."""
    L, B = _libs()
    fp32 = prec_name == "fp32"
    G = -5.5
    rg, rl = coexistence_densities(G)
    rho = thread_density(nz, nr, 64.0, rl, rg, 2.0, 0.1, 1)
    p = L.make_params(nz, nr, G=G, tau=0.8, wall=L.WALL_FREESLIP,
                      precision=L.FP32_SHIFTED if fp32 else L.FP64, rho_ref=rg if fp32 else 0.0)
    _say(f"large-lattice path vs batch kernel: {prec_name} {nz}x{nr}")
    sim = L.AxiLBM(p, torch.from_numpy(rho).cuda())
    sim.step(4)
    single = sim.populations()
    sim.close()
    b = B.AxiBatch([p], [torch.from_numpy(rho).cuda()])
    b.set_schedule(b.configs().index((64, 16, 512)), 2, 0)
    b.step(4)
    batched = b.populations(0)
    b.close()
    assert torch.equal(single, batched)
