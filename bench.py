"""Benchmark of the fused axisymmetric Shan–Chen step on one MI355X.

Workload: Rayleigh–Plateau liquid thread on a 4096 x 512 (z, r) lattice,
thread radius 64 with a 0.1 R cos(2 pi z / nz) perturbation, G = -5.5,
free-slip outer wall, tau = 0.8 (the scheme diverges at tau = 0.7 for this
G; tau does not change the work per node), started at the scheme's own
coexistence densities for (G, tau).  Synthetic inputs resident in HBM before
the timed region.

One step = one launch of the fused kernel over all 2,097,152 nodes.  Prints
one JSON line: FP64 MLUPS as ``value``, the FP32-shifted-storage MLUPS (shift
rho_ref = gas density), the HBM roofline of the dominant (FP64 step) kernel,
the adjoint's (forward + backward) / forward time on the 256 x 128 drop, the
batched ensemble's aggregate MLUPS (256 instances, persistent graph-replayed
launch vs one launch per instance) and the CPU oracle timed on the host cores
over a bounded sample of the 4096 x 512 workload.
"""
import argparse
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

NZ, NR = 4096, 512
G, TAU, RADIUS, EPS = -5.5, 0.8, 64.0, 0.1
HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, vendor figure
BYTES_PER_LU = {"f64": 9 * 2 * 8, "f32": 9 * 2 * 4}  # read + write every population once
# the kernel, the launch code that picks its tile shape, order and store
# policy, and the buffer layout: a change to any of them invalidates the
# committed counter figures
KERNEL_SOURCES = ("paper_1310_1871_amd/csrc/step_kernel.hpp", "paper_1310_1871_amd/csrc/lattice.hpp",
                  "paper_1310_1871_amd/csrc/lbm_axi.hip", "paper_1310_1871_amd/csrc/common.hpp")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "hbm_traffic_axi_step_4096x512.md")
# --kernel: the step kernels of lbm_axi_set_kernel
KERNELS = {"tile": "KERNEL_TILE", "strip": "KERNEL_STRIP", "tile-alternate": "KERNEL_TILE_ALTERNATE",
           "tile-columns": "KERNEL_TILE_COLUMNS", "tile-pairs": "KERNEL_TILE_PAIRS"}


def kernel_source_hash():
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(tag):
    """HBM bytes per launch from the committed rocprofv3 counter summary, or
    None if absent or taken on a different kernel source."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    txt = open(TRAFFIC_FILE).read()
    m = re.search(r"kernel_source_sha256_16:\s*([0-9a-f]+)", txt)
    if not m or m.group(1) != kernel_source_hash():
        return None
    m = re.search(rf"traffic_bytes_per_launch_{tag}:\s*([0-9.eE+]+)", txt)
    return float(m.group(1)) if m else None


def workload_density():
    from lbm_inputs import scheme_coexistence, thread_density
    rg, rl = scheme_coexistence(G, TAU)
    return thread_density(NZ, NR, RADIUS, rl, rg, 2.0, EPS, 1), rl, rg


def time_gpu(precision, rho, rho_ref, steps, warmup, kernel="tile", strip_rows=43):
    import torch
    from paper_1310_1871_amd import lbm_axi as L
    p = L.make_params(NZ, NR, G=G, tau=TAU, wall=L.WALL_FREESLIP, axisym=1, precision=precision, rho_ref=rho_ref)
    sim = L.AxiLBM(p, torch.from_numpy(rho).cuda())
    sim.set_kernel(getattr(L, KERNELS[kernel]), strip_rows)
    sim.step(warmup)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    t0.record(stream)
    sim.step(steps)
    t1.record(stream)
    torch.cuda.synchronize()
    ms = t0.elapsed_time(t1)
    diag = sim.reduce()
    sim.close()
    return ms / steps, diag


def copy_calibration():
    """A plain device copy of known size (256 MiB read + 256 MiB written),
    whose FETCH_SIZE / WRITE_SIZE counters calibrate the step kernel's."""
    import torch
    a = torch.ones(32 * 1024 * 1024, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    for _ in range(5):
        b.copy_(a)
    torch.cuda.synchronize()


def adjoint_ratio(nz=256, nr=128, steps=2000):
    """(forward + backward) / forward time of the checkpointed adjoint on the
    adjoint workload: 256 x 128 drop (R = 40), 2000 steps, interface radius
    sampled every 50 steps on 16 rays, checkpoints every 100 steps,
    gradients for a_2..a_6 (through rho0), G and tau.  Other lattices keep
    the drop radius at 0.3125 nr."""
    import numpy as np
    import torch
    from lbm_inputs import adjoint_coeffs, coexistence_densities, drop_density
    from paper_1310_1871_amd import adjoint as A
    R, Gc, tauc, every, ck = 0.3125 * nr, -5.5, 0.8, 50, 100
    rg, rl = coexistence_densities(Gc)
    probe = A.RayProbe(nz, nr, nz / 2.0, A.default_thetas(16), rl, rg)
    rho_t = torch.from_numpy(drop_density(nz, nr, nz / 2.0, R, rl, rg, 2.0, adjoint_coeffs(11, R))).cuda()
    target = A.radius_history(rho_t, Gc, tauc, probe, steps, every)
    rho0 = torch.from_numpy(drop_density(nz, nr, nz / 2.0, R, rl, rg, 2.0, adjoint_coeffs(12, R))).cuda()
    times = {}
    for rep in range(2):  # the first repetition warms up
        r0 = rho0.clone().requires_grad_(True)
        G = torch.tensor(Gc, dtype=torch.float64, device="cuda", requires_grad=True)
        tau = torch.tensor(tauc, dtype=torch.float64, device="cuda", requires_grad=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        loss = A.shape_loss(r0, G, tau, probe, target, steps, every, ck)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        loss.backward()
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        times = {"fwd_s": t1 - t0, "bwd_s": t2 - t1, "loss": float(loss.item()),
                 "dL_dG": float(G.grad.item()), "dL_dtau": float(tau.grad.item())}
    times["fwd_bwd_over_fwd"] = round((times["fwd_s"] + times["bwd_s"]) / times["fwd_s"], 3)
    times["workload"] = (f"drop {nz}x{nr} R={R:g}, {steps} steps, 16 rays every {every} steps, "
                         f"checkpoint every {ck}, FP64")
    return times


def batch_throughput(steps=200):
    """Batched ensemble: 256 seeded drops/threads of sizes 64x32 .. 512x256,
    FP32 shifted storage; aggregate MLUPS of the autotuned persistent launch
    (graph replay) and of one launch per instance per step."""
    import torch
    from lbm_inputs import ensemble
    from paper_1310_1871_amd import batch as B
    from paper_1310_1871_amd import lbm_axi as L
    cases = ensemble()
    params = [L.make_params(c.nz, c.nr, G=c.G, tau=c.tau, wall=c.wall, precision=L.FP32_SHIFTED, rho_ref=c.rho_g)
              for c in cases]
    b = B.AxiBatch(params, [torch.from_numpy(c.rho).cuda() for c in cases])
    choice, _ = b.autotune(steps_per_trial=4)
    nodes = b.nodes()
    out = {"instances": len(cases), "nodes": nodes, "schedule": {"config": b.configs()[choice[0]],
                                                                  "grid_per_cu": choice[1], "order": choice[2]}}
    for name, fn in (("persistent_graph", b.step), ("per_instance_launches", b.step_per_instance)):
        fn(20)
        b.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(b.stream)
        fn(steps)
        e1.record(b.stream)
        b.synchronize()
        ms = e0.elapsed_time(e1) / steps
        out[name] = {"ms_per_step": round(ms, 5), "MLUPS": round(nodes / (ms * 1e-3) / 1e6, 1)}
        if name == "persistent_graph":
            # algorithmic bytes of one step of every instance (FP32 storage:
            # 72 B per node), over the launch time; the ensemble's two buffers
            # (2 x 462 MB) exceed the 256 MB memory-side cache
            gbs = BYTES_PER_LU["f32"] * nodes / (ms * 1e-3) / 1e9
            out[name]["roofline"] = {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS,
                                     "unit": "GB/s", "frac": round(gbs / HBM_PEAK_GBS, 4)}
    out["speedup_persistent_vs_per_instance"] = round(out["per_instance_launches"]["ms_per_step"] /
                                                      out["persistent_graph"]["ms_per_step"], 3)
    b.close()
    return out


def _omp_threads():
    import ctypes
    try:
        return int(ctypes.CDLL("libgomp.so.1").omp_get_max_threads())
    except OSError:
        return os.cpu_count()


def _oracle_rate(p, f, budget_s):
    """MLUPS of the oracle as it stands on whole steps of (p, f), over about
    budget_s seconds: chunks of whole steps (each about a tenth of the
    budget) until the budget is spent, after one start-up step."""
    import oracle as O
    f = O.run(p, f, 1)  # start-up (thread pool, first touch) outside the sample
    t0 = time.perf_counter()
    f = O.run(p, f, 1)
    chunk = max(1, int(0.1 * budget_s / max(time.perf_counter() - t0, 1e-4)))
    steps, el = 0, 0.0
    while el < budget_s:
        t0 = time.perf_counter()
        f = O.run(p, f, chunk)
        el += time.perf_counter() - t0
        steps += chunk
    return p.nz * p.nr * steps / el / 1e6, steps, el


def cpu_baseline(rho, budget_s=12.0):
    """The oracle as it stands, timed on the host: the 4096 x 512 thread
    workload (the benchmarked one) on every host thread (about budget_s
    seconds of whole steps) and on one (about budget_s / 2), and the 64 x 32
    static drop and the 256 x 128 oscillating drop on every thread (2000
    steps each, about a second)."""
    import numpy as np
    import oracle as O
    from lbm_inputs import oscillating_drop, static_drop
    threads = _omp_threads()
    p = O.make_params(NZ, NR, G=G, tau=TAU, wall=O.WALL_FREESLIP, axisym=1)
    f = O.equilibrium(p, rho, np.zeros_like(rho), np.zeros_like(rho))
    v_all, n_all, t_all = _oracle_rate(p, f, budget_s)
    O.set_threads(1)
    try:
        v_one, n_one, t_one = _oracle_rate(p, f, budget_s / 2)
    finally:
        O.set_threads(threads)
    others = {}
    for case in (static_drop(), oscillating_drop(tau=0.8)):
        q = O.make_params(case.nz, case.nr, G=case.G, tau=case.tau, wall=case.wall, axisym=1)
        fc = O.equilibrium(q, case.rho, case.uz, case.ur)
        t0 = time.perf_counter()
        n = 2000
        O.run(q, fc, n)
        el = time.perf_counter() - t0
        others[f"{case.nz}x{case.nr}"] = {"MLUPS": round(case.nz * case.nr * n / el / 1e6, 2), "steps": n,
                                          "seconds": round(el, 2), "cores": threads}
    return {"value": v_all, "unit": "MLUPS", "cores": int(threads), "kind": "oracle",
            "sample": (f"{n_all} full steps of the 4096x512 thread workload (FP64 C oracle, OpenMP), "
                       f"{t_all:.1f} s"),
            "one_core": {"value": v_one, "unit": "MLUPS", "cores": 1, "steps": n_one, "seconds": round(t_one, 2)},
            "other_workloads": others}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--skip-cpu", action="store_true", help="omit the CPU oracle baseline")
    ap.add_argument("--skip-fp32", action="store_true")
    ap.add_argument("--skip-adjoint", action="store_true")
    ap.add_argument("--adjoint-lattice", type=int, nargs=3, metavar=("NZ", "NR", "STEPS"), default=(256, 128, 2000),
                    help="lattice and step count of the adjoint leg (default: the 256 x 128 drop, 2000 steps)")
    ap.add_argument("--skip-batch", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain copy kernel of known size (for counter calibration)")
    ap.add_argument("--kernel", choices=tuple(KERNELS), default="tile",
                    help="step kernel of the FP64 and FP32 legs (lbm_axi_set_kernel); tile is the library default")
    ap.add_argument("--strip-rows", type=int, default=43, help="chunk height of the strip kernel")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path (a lattice would be "
              "split into z slabs with a halo exchange per step); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    rho, rl, rg = workload_density()
    print(f"bench: thread {NZ}x{NR} FP64 {args.steps} steps (+{args.warmup} warm-up)", file=sys.stderr, flush=True)
    ms64, diag64 = time_gpu(0, rho, 0.0, args.steps, args.warmup, args.kernel, args.strip_rows)
    lups = NZ * NR
    mlups64 = lups / (ms64 * 1e-3) / 1e6
    achieved = BYTES_PER_LU["f64"] * lups / (ms64 * 1e-3) / 1e9
    out = {
        "metric": "MLUPS & % HBM roofline, FP64 vs FP32-storage; adjoint fwd+bwd / fwd ratio",
        "value": round(mlups64, 2),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms64, 6),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "rayleigh_plateau_thread_4096x512", "nz": NZ, "nr": NR, "G": G, "tau": TAU,
                   "wall": "free-slip", "thread_radius": RADIUS, "perturbation": "0.1 R cos(2 pi z / nz)",
                   "rho_l": round(rl, 5), "rho_g": round(rg, 5), "bytes_per_lu": BYTES_PER_LU["f64"]},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": measured_traffic("f64") if args.kernel == "tile" else None,
                     "kernel": f"axi_{args.kernel}_kernel<FP64>"},
        "diagnostics_f64": {"mass_3d": diag64[0], "kinetic_energy": diag64[2]},
    }
    if not args.skip_fp32:
        print(f"bench: thread {NZ}x{NR} FP32-shifted storage", file=sys.stderr, flush=True)
        ms32, diag32 = time_gpu(1, rho, rg, args.steps, args.warmup, args.kernel, args.strip_rows)
        mlups32 = lups / (ms32 * 1e-3) / 1e6
        ach32 = BYTES_PER_LU["f32"] * lups / (ms32 * 1e-3) / 1e9
        out["fp32_storage"] = {"value": round(mlups32, 2), "unit": "MLUPS", "ms_per_step": round(ms32, 6),
                               "speedup_vs_f64": round(ms64 / ms32, 3), "rho_ref": round(rg, 5),
                               "roofline": {"bound": "hbm", "achieved": round(ach32, 1), "peak": HBM_PEAK_GBS,
                                            "unit": "GB/s", "frac": round(ach32 / HBM_PEAK_GBS, 4),
                                            "traffic": measured_traffic("f32") if args.kernel == "tile" else None},
                               "mass_3d_rel_diff_vs_f64": abs(diag32[0] - diag64[0]) / diag64[0]}
    out["adjoint"] = None
    if not args.skip_adjoint:
        anz, anr, asteps = args.adjoint_lattice
        print(f"bench: adjoint (fwd+bwd)/fwd on the {anz}x{anr} drop", file=sys.stderr, flush=True)
        out["adjoint"] = adjoint_ratio(anz, anr, asteps)
    if not args.skip_batch:
        print("bench: batched ensemble of 256 instances", file=sys.stderr, flush=True)
        out["batch"] = batch_throughput()
    if args.copy_calibration:
        copy_calibration()
    if not args.skip_cpu:
        print("bench: CPU oracle baseline", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(rho)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
