"""Benchmark of the DSMC step on one MI355X.

A step is one pass of the whole per-step path (move with boundary
interactions, freestream injection, counting sort by cell, NTC/VHS
collisions, cell moment sampling) over the particle set.  Default workload:
the lid-driven cavity on 40^3 hexes x 6 jittered tets (384,000 tets),
Kn = 0.1, 30 particles per cell (11.52M particles), FP32 velocity storage,
FP64 positions, arithmetic and moments.  The timed steps are replayed from
captured HIP graphs (two steps per graph; --eager for ordinary launches);
per-kernel times come from ten ordinary steps after the timed region, since
HIP events are not recorded inside a replayed graph.  Prints one JSON line.
"""
import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Algorithmic HBM bytes of each stage of the step: what the method has to
# move, for the FP32-velocity layout of 44 bytes per particle (x,y,z f64 24,
# v f32 12, cell i32 4, pid u32 4), independent of how the kernels do it:
#  move:     read x, v, cell, pid (44); write x, cell (28); write v of a
#            particle that met a wall (12 per wall interaction)
#  scan:     the cell histogram and offsets (8 per cell)
#  sort:     read and write every particle once (44 + 44)
#  collide:  read v, pid (16); write v of collided particles (12 each); per
#            cell the offset and (sigma c)_max (16) and the 13 FP64 moment
#            sums read and written (208)
# Stage -> kernels whose launch times it sums.
BYTES = {
    "move": lambda np_, nt, f: np_ * (72.0 + (12.0 + 8.0 * f["rot"]) * f["walls"]),
    "scan": lambda np_, nt, f: nt * 8.0,
    "sort": lambda np_, nt, f: np_ * (88.0 + 16.0 * f["rot"]),
    "collide_sample": lambda np_, nt, f: (np_ * (16.0 + 12.0 * f["touched"] + f["rot"] * (8.0 + 8.0 * f["touched"]))
                                          + nt * (224.0 + 64.0 * f["rot"])),
}
STAGES = {"move": ["move", "move_walls"], "scan": ["scan"], "sort": ["sort_perm", "sort_gather"],
          "collide_sample": ["collide_sample"]}

# rocprofv3 --pmc measurements of the dominant stage's kernels (FETCH_SIZE +
# WRITE_SIZE per step, summed over the stage's kernels and scaled by the
# copy-kernel calibration) and the source digest they were taken on; the
# traffic figure is reported only while the digest matches.
TRAFFIC = {"stage": "move", "digest": "f678485dc442d1cf", "bytes_per_launch": 1255226834,
           "workload": "cavity_40^3x6_Kn0.1", "source": "profiles/step_kernels_cavity40.md"}


# rocprofv3 --pmc TCP_TOTAL_CACHE_ACCESSES_sum of the move kernel (vector
# L1 line accesses per dispatch, the unit of the line-read calibration) on
# the same source digest: the move kernel's bound is the L1's line-access
# rate, set by its divergent 16-byte loads of the cells' planes and
# neighbour codes.
L1 = {"kernel": "move", "digest": "f678485dc442d1cf", "accesses_per_launch": 302200000,
      "workload": "cavity_40^3x6_Kn0.1", "source": "profiles/step_kernels_cavity40.md"}


def _kernel_digest():
    h = hashlib.sha256()
    for f in ["kernels.hip", "device_common.h", "kernels.h"]:
        h.update(open(os.path.join(ROOT, "paper_2607_08195_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:16]


def _host_cpu():
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"nproc": os.cpu_count(), "model": model}


def _oracle_cavity_small(seed):
    """One full run of the CPU-finishable cavity in a fresh process: returns
    (particle-steps, seconds)."""
    from paper_2607_08195_amd import workloads as W
    from oracle import Oracle
    wl = W.cavity_small()
    wl.run.seed = seed
    o = Oracle(wl)
    n0 = o.np
    t0 = time.perf_counter()
    o.step(500)
    return 0.5 * (n0 + o.np) * 500, time.perf_counter() - t0


def cpu_baseline(wl, steps, procs):
    """The oracle as it stands, on the host cores: (1) single-threaded on a
    bounded sample of the benchmark workload, `steps` steps from its initial
    fill (the reported value); (2) the full 500-step run of the
    CPU-finishable cavity (6^3 x 6 tets, 25,920 particles) single-threaded;
    (3) `procs` such runs at once in independent processes with disjoint
    seeds (aggregate particle-steps/s over the group's wall time)."""
    import multiprocessing as mp
    from concurrent.futures import ProcessPoolExecutor
    from oracle import Oracle
    o = Oracle(wl)
    n = o.np
    t0 = time.perf_counter()
    o.step(steps)
    dt = time.perf_counter() - t0
    del o
    ps, ts = _oracle_cavity_small(0)
    with ProcessPoolExecutor(max_workers=procs, mp_context=mp.get_context("spawn")) as ex:
        ex.submit(time.sleep, 0).result()          # workers started before the clock
        t1 = time.perf_counter()
        runs = list(ex.map(_oracle_cavity_small, range(1, procs + 1)))
        tw = time.perf_counter() - t1
    agg = sum(r[0] for r in runs) / tw
    return dict(value=n * steps / dt, unit="particle-steps/s", cores=1, kind="oracle",
                sample=f"{wl.name}: {steps} steps from the initial fill ({n * steps:.3g} particle-steps, "
                       f"{dt:.1f} s, 1 thread)",
                cavity_small_full={"value": ps / ts, "steps": 500, "particle_steps": ps, "seconds": round(ts, 2),
                                   "cores": 1},
                aggregate={"value": agg, "processes": procs, "workload": "cavity_6^3x6_Kn1 x 500 steps each",
                           "seconds": round(tw, 2), "per_process_mean": sum(r[0] / r[1] for r in runs) / procs},
                host=_host_cpu())


def copy_rate(sim, nbytes=1 << 30, reps=5):
    """Read + write GB/s of the library's plain copy kernel on nbytes each
    way: the bandwidth a streaming kernel achieves on this GPU."""
    import torch
    src = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    dst = torch.empty_like(src)
    sim.device_copy(dst.data_ptr(), src.data_ptr(), nbytes)
    sim.sync()
    t0 = time.perf_counter()
    for _ in range(reps):
        sim.device_copy(dst.data_ptr(), src.data_ptr(), nbytes)
    sim.sync()
    dt = (time.perf_counter() - t0) / reps
    del src, dst
    return 2 * nbytes / dt / 1e9


def calibrate_copy(dsmc, W, nbytes=2 << 30, reps=10):
    """A plain copy kernel of known size: its FETCH_SIZE / WRITE_SIZE counters
    per dispatch divided by nbytes give the counter scale factors."""
    import torch
    sim = dsmc.Simulation(W.cavity(n_hex=2, ppc=2))
    src = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    dst = torch.empty_like(src)
    sim.device_copy(dst.data_ptr(), src.data_ptr(), nbytes)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        sim.device_copy(dst.data_ptr(), src.data_ptr(), nbytes)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / reps
    print(json.dumps({"copy_bytes_each_way": nbytes, "ms": dt * 1e3, "GBps_read_plus_write": 2 * nbytes / dt / 1e9}))
    sim.close()


def line_read_rate(sim, shares=(1, 4, 64), iters=256, blocks=8192, reps=3):
    """Vector-L1 accesses per CU and ns of scattered 16-byte reads from a
    2 MiB (L2-resident) table, one line per `share` lanes per load: per
    share the accesses in the unit of rocprofv3's TCP_TOTAL_CACHE_ACCESSES
    (a 16-byte load counts two per distinct line of a wave instruction, at
    least eight per instruction; measured with the counter for shares 1, 4
    and 64), the time and the rate."""
    import torch
    nbytes = 2 << 20
    tab = torch.zeros(nbytes, dtype=torch.uint8, device="cuda")
    sink = torch.zeros(1, dtype=torch.int32, device="cuda")
    torch.cuda.synchronize()
    out = {}
    for share in shares:
        sim.device_line_reads(tab.data_ptr(), nbytes, sink.data_ptr(), share, iters, blocks)
        sim.sync()
        t0 = time.perf_counter()
        for _ in range(reps):
            sim.device_line_reads(tab.data_ptr(), nbytes, sink.data_ptr(), share, iters, blocks)
        sim.sync()
        dt = (time.perf_counter() - t0) / reps
        acc = blocks * 4.0 * iters * 2 * max(64 // share, 4)
        out[share] = {"ms": round(dt * 1e3, 4), "line_accesses": acc, "per_cu_ns": round(acc / 256 / (dt * 1e9), 4)}
    del tab, sink
    return out


def calibrate_l1(dsmc, W):
    sim = dsmc.Simulation(W.cavity(n_hex=2, ppc=2))
    r = line_read_rate(sim)
    print(json.dumps({"line_reads": r, "peak_per_cu_ns": max(v["per_cu_ns"] for v in r.values())}))
    sim.close()


def bench_ensemble(args, dsmc, W, window=50):
    """64 independent cavities (Kn log-uniform in [0.01, 1], lid 20-200 m/s,
    6^3-24^3 hexes x 6 tets, 20 particles per cell) advanced together in one
    context with the schedule the autotuner picks, the DSMC steps replayed
    from captured HIP graphs, and the DIG coupling step with the learned
    closure on the odd-numbered half of the cases every `window` steps.
    value = particle-steps/s summed over the cases, couplings included; the
    plain steps alone, with ordinary launches and from graphs, are timed
    beside it.  The closure is trained first on the ensemble's own cells."""
    import numpy as np
    import torch
    cases = W.cavity_ensemble(64)
    for wl in cases:
        wl.run.ewma_on = 1
    stream = torch.cuda.Stream()
    sim = dsmc.Simulation(cases, stream=stream)
    np0 = sim.stats()["n_particles"]
    tune = sim.autotune(trial_steps=3)
    timings = {}
    for mode in ["eager", "graph"]:
        run = sim.step if mode == "eager" else sim.graph_step
        run(args.warmup)
        sim.sync()
        t0 = time.perf_counter()
        run(args.steps)
        sim.sync()
        timings[mode] = time.perf_counter() - t0
    n1 = sim.stats()["n_particles"]
    plain = 0.5 * (np0 + n1) * args.steps
    # the persistent move (tiles pulled from an XCD-sliced device work queue)
    # in the same graph-replayed batched step
    sim.set_tuning(17, tune["collide"], tune["sort"])
    sim.graph_step(args.warmup)
    sim.sync()
    t0 = time.perf_counter()
    sim.graph_step(args.steps)
    sim.sync()
    timings["graph_persistent"] = time.perf_counter() - t0
    sim.set_tuning(tune["move"], tune["collide"], tune["sort"])
    # the same cases one after another, each in a context of its own, with
    # the same kernels and schedule (graph-replayed): the batched launch
    # against sequential per-case launches
    seq_t, seq_ps = 0.0, 0.0
    for wl in cases:
        one = dsmc.Simulation(wl, stream=stream)
        one.set_tuning(tune["move"], tune["collide"], tune["sort"])
        na = one.stats()["n_particles"]
        one.graph_step(args.warmup)
        one.sync()
        a = time.perf_counter()
        one.graph_step(args.steps)
        one.sync()
        seq_t += time.perf_counter() - a
        seq_ps += 0.5 * (na + one.stats()["n_particles"]) * args.steps
        one.close()
    print(f"# ensemble: batched graph {1e3 * timings['graph'] / args.steps:.2f} ms/step, sequential per-case "
          f"{1e3 * seq_t / args.steps:.2f} ms/step", file=sys.stderr, flush=True)
    # coupling on the odd cases with a closure trained on their cells
    on = np.arange(len(cases)) % 2 == 1
    sim.dig_enable(on.astype(np.int32))
    prm = dict(kn_max=1.0, passes=3, n_m=100, eps_m=1e-4, cfl=0.5, feedback=1, warm_start=1, unconverged=1)
    sim.dig_couple(**dict(prm, n_m=0, feedback=0))
    x, t, v = sim.closure_data()
    begin = sim.case_cells()
    v &= np.repeat(on, np.diff(begin))
    net = dsmc.Mlp()
    net.init_weights(seed=1)
    t0 = time.perf_counter()
    train = net.train(x[v], t[v], steps=200, batch=4096, lr=1e-3, seed=1)
    torch.cuda.synchronize()
    train_s = time.perf_counter() - t0
    sim.set_closure(net, gate_tol=0.5)
    sim.graph_step(window)
    sim.dig_couple(**prm)
    sim.sync()
    cycles = max(1, args.steps // window)
    np2 = sim.stats()["n_particles"]
    t_step = t_couple = 0.0
    rep = None
    for _ in range(cycles):
        a = time.perf_counter()
        sim.graph_step(window)
        sim.sync()
        b = time.perf_counter()
        rep = sim.dig_couple(**prm)
        c = time.perf_counter()
        t_step += b - a
        t_couple += c - b
    n3 = sim.stats()["n_particles"]
    elapsed = t_step + t_couple
    out = {
        "metric": "particle-steps/s",
        "value": 0.5 * (np2 + n3) * cycles * window / elapsed,
        "unit": "particle-steps/s",
        "n_gpus": 1,
        "steps": cycles * window,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * elapsed / (cycles * window),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "cavity_ensemble_64", "cases": len(cases), "tets": sim.nt, "particles": int(np0),
                   "coupled_cases": int(on.sum()), "window": window, "coupling": prm},
        "ms_per_coupling": 1e3 * t_couple / cycles,
        "graph_ms_per_dsmc_step": 1e3 * t_step / (cycles * window),
        "plain_eager_ms_per_step": 1e3 * timings["eager"] / args.steps,
        "plain_graph_ms_per_step": 1e3 * timings["graph"] / args.steps,
        "plain_value_graph": plain / timings["graph"],
        "plain_graph_persistent_ms_per_step": 1e3 * timings["graph_persistent"] / args.steps,
        "sequential_per_case": {"ms_per_step": 1e3 * seq_t / args.steps, "value": seq_ps / seq_t,
                                "launches": "each case in a context of its own, graph-replayed, same schedule"},
        "batched_over_sequential": (plain / timings["graph"]) / (seq_ps / seq_t),
        "closure_training": {"steps": 200, "batch": 4096, "seconds": round(train_s, 3),
                             "loss_first": train["loss_first"], "loss_last": train["loss_last"]},
        "last_report": rep,
        "autotuned": tune,
    }
    net.close()
    sim.close()
    print(json.dumps(out))


def bench_sphere(args, dsmc, W, develop=600):
    """Hypersonic argon flow over a 1 m sphere (Mach 10 at 200 K, Kn 0.05 on
    the diameter, diffuse wall at 500 K) in a 6 x 4 x 4 m box: 1.96M tets
    (cubed-sphere O-grid graded 5:1 towards the wall inside a Cartesian box),
    freestream inflow on five faces, vacuum outflow, 50M particles at the
    initial freestream fill.  `develop` untimed steps form the shock (about
    two flow-through times), the autotuner picks the schedules on the
    developed flow, then surface sampling is switched on and
    --warmup and --steps ordinary steps follow; value = particle-steps/s over
    the timed steps.  The sphere's drag coefficient from the surface sums is
    reported beside it."""
    import numpy as np
    import torch
    wl = W.sphere_flow(N=22, K=16, grade=5.0, n_particles=50_000_000, vel_fp32=1)
    sim = dsmc.Simulation(wl, capacity=80_000_000)
    sim.step(develop)
    tune = sim.autotune(trial_steps=3)  # on the developed flow (uneven cell occupancy)
    sim.surface_sampling(True)
    sim.step(args.warmup)
    sim.sync()
    s0 = sim.stats()
    sim.profile(True)
    t0 = time.perf_counter()
    sim.step(args.steps)
    sim.sync()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    prof = sim.profile_read()
    sim.profile(False)
    s1 = sim.stats()
    sums, _, ns = sim.surface()
    sel = wl.mesh.bgroup == 6
    m, info = wl.species.mass, wl.info
    drag = m * wl.run.F_N * sums[sel, 0].sum() / (ns * wl.run.dt)
    cd = drag / (0.5 * m * info["n_inf"] * info["u"] ** 2 * math.pi * info["R"] ** 2)
    nc, _ = sim.pair_counts()
    counts = np.bincount(sim.state()["cell"], minlength=sim.nt)
    npart = 0.5 * (s0["n_particles"] + s1["n_particles"])
    out = {
        "metric": "particle-steps/s",
        "value": npart * args.steps / elapsed,
        "unit": "particle-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": develop + args.warmup,
        "ms_per_step": 1e3 * elapsed / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "sphere_mach10_kn0.05", "tets": sim.nt, "particles": int(s1["n_particles"]),
                   "initial_particles": 50_000_000, "velocity_storage": "f32"},
        "hops_per_particle_step": round((s1["hops"] - s0["hops"]) / (npart * args.steps), 3),
        "particles_per_cell": {"min": int(counts.min()), "median": float(np.median(counts)),
                               "max": int(counts.max())},
        "kernel_ms": {k: round(ms / cnt, 4) for k, (ms, cnt) in prof.items() if cnt},
        "drag_coefficient": round(float(cd), 4),
        "surface_steps": ns,
        "autotuned": tune,
    }
    sim.close()
    print(json.dumps(out))


def bench_dig(args, dsmc, W, window=50):
    """DIG-coupled cavity at Kn = 0.01 on the 384,000-tet mesh (30 particles
    per cell): cycles of `window` DSMC steps followed by one coupling step
    (sampled state, HoT, gate, learned closure, FV solve, feedback).  The
    closure network is first trained on the run's own cell data.  --steps
    counts DSMC steps (rounded to whole windows).  --dig-solver nk takes the
    Newton-Krylov solve (20 Newton steps, GMRES(40), initial CFL 10) instead
    of 100 pseudo-time iterations."""
    import torch
    wl = W.cavity(n_hex=40, Kn=0.01, ppc=30, jitter=0.1, vel_fp32=1, ewma_on=1, n_a=1000)
    sim = dsmc.Simulation(wl)
    net = dsmc.Mlp()
    net.init_weights(seed=1)
    prm = dict(kn_max=1.0, passes=3, n_m=100, eps_m=1e-4, cfl=0.5, feedback=1, warm_start=1, unconverged=1)
    if args.dig_solver == "nk":
        prm.update(n_m=20, eps_m=1e-3, cfl=10.0, solver=1, krylov=40)
    sim.step(window)
    sim.dig_couple(**dict(prm, n_m=0, feedback=0))
    x, t, v = sim.closure_data()
    t0 = time.perf_counter()
    train = net.train(x[v], t[v], steps=200, batch=4096, lr=1e-3, seed=1)
    torch.cuda.synchronize()
    train_s = time.perf_counter() - t0
    sim.set_closure(net, gate_tol=0.5)
    cycles = max(1, args.steps // window)
    for _ in range(max(1, args.warmup // window)):
        sim.step(window)
        sim.dig_couple(**prm)
    sim.sync()
    np0 = sim.stats()["n_particles"]
    t_step = t_couple = 0.0
    reps = []
    for _ in range(cycles):
        a = time.perf_counter()
        sim.step(window)
        sim.sync()
        b = time.perf_counter()
        reps.append(sim.dig_couple(**prm))
        c = time.perf_counter()
        t_step += b - a
        t_couple += c - b
    n1 = sim.stats()["n_particles"]
    elapsed = t_step + t_couple
    out = {
        "metric": "particle-steps/s",
        "value": 0.5 * (np0 + n1) * cycles * window / elapsed,
        "unit": "particle-steps/s",
        "n_gpus": 1,
        "steps": cycles * window,
        "warmup": max(1, args.warmup // window) * window,
        "ms_per_step": 1e3 * elapsed / (cycles * window),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "dig_cavity_40^3x6_Kn0.01", "tets": sim.nt, "particles": int(np0),
                   "window": window, "coupling": prm},
        "ms_per_coupling": 1e3 * t_couple / cycles,
        "ms_per_dsmc_step": 1e3 * t_step / (cycles * window),
        "closure_training": {"steps": 200, "batch": 4096, "seconds": round(train_s, 3),
                             "loss_first": train["loss_first"], "loss_last": train["loss_last"]},
        "last_report": reps[-1],
    }
    net.close()
    sim.close()
    print(json.dumps(out))


def _ttf_geometry(wl, nb=10, nline=40):
    """Bins of the time-to-fields comparison: cell -> one of nb^3 boxes over
    the unit cube, cell volumes, and the cells of the two centreline slabs
    (2h wide, h the hex spacing) with their index along the line: the
    vertical line x = z = 1/2 (binned in y) and the horizontal line
    y = z = 1/2 (binned in x)."""
    import numpy as np
    xyz, tets = wl.mesh.xyz, wl.mesh.tets
    cen = xyz[tets].mean(axis=1)
    a, b, c, d = (xyz[tets[:, k]] for k in range(4))
    vol = np.abs(np.einsum("ij,ij->i", b - a, np.cross(c - a, d - a))) / 6.0
    ijk = np.minimum((cen * nb).astype(int), nb - 1)
    h = 1.0 / wl.info["n_hex"]
    near = lambda i, j: (np.abs(cen[:, i] - 0.5) < h) & (np.abs(cen[:, j] - 0.5) < h)
    line = lambda ax: np.minimum((cen[:, ax] * nline).astype(int), nline - 1)
    return dict(bin=ijk[:, 0] * nb * nb + ijk[:, 1] * nb + ijk[:, 2], nbins=nb ** 3, vol=vol, nline=nline,
                vsel=near(0, 2), vidx=line(1), hsel=near(1, 2), hidx=line(0))


def _ttf_reduce(S, G):
    """Cell moment sums [nt, 13] -> sums over the boxes and the line bins."""
    import numpy as np
    box = np.stack([np.bincount(G["bin"], weights=S[:, k], minlength=G["nbins"]) for k in range(7)], axis=1)
    lv = np.stack([np.bincount(G["vidx"][G["vsel"]], weights=S[G["vsel"], k], minlength=G["nline"])
                   for k in range(4)], axis=1)
    lh = np.stack([np.bincount(G["hidx"][G["hsel"]], weights=S[G["hsel"], k], minlength=G["nline"])
                   for k in range(4)], axis=1)
    return box, lv, lh


def _ttf_fields(red, n, G, wl):
    """Fields of binned sums over n steps (eq. dsmc_temperatures pooled over
    each bin): density, velocity, temperature per box; u_x / U_lid along the
    vertical line and u_y / U_lid along the horizontal line."""
    import numpy as np
    box, lv, lh = red
    m, FN = wl.species.mass, wl.run.F_N
    V = np.bincount(G["bin"], weights=G["vol"], minlength=G["nbins"])
    S0 = np.maximum(box[:, 0], 1e-300)
    u = box[:, 1:4] / S0[:, None]
    T = m / (3 * KB_) * ((box[:, 4] + box[:, 5] + box[:, 6]) / S0 - (u * u).sum(axis=1))
    rho = m * FN * box[:, 0] / n / np.maximum(V, 1e-300)
    U = wl.info["lid_speed"]
    return dict(u=u, rho=rho, T=T, vline=lv[:, 1] / np.maximum(lv[:, 0], 1e-300) / U,
                hline=lh[:, 2] / np.maximum(lh[:, 0], 1e-300) / U)


def _ttf_err(F, R):
    import numpy as np
    rel = lambda a, b: float(np.linalg.norm(a - b) / np.linalg.norm(b))
    out = dict(u=rel(F["u"], R["u"]), rho=rel(F["rho"], R["rho"]), T=rel(F["T"], R["T"]),
               vline=rel(F["vline"], R["vline"]), hline=rel(F["hline"], R["hline"]))
    out["e"] = max(out["u"], out["rho"], out["T"])
    return out


KB_ = 1.380649e-23


TTF_LEVELS = (0.10, 0.05, 0.04, 0.03, 0.02, 0.01)


def bench_time_to_fields(args, dsmc, W, block=500):
    """Time to fields on the coupled-cavity configuration (384,000 jittered
    tets, Kn = 0.01, 30 particles per cell, lid 50 m/s): wall seconds of GPU
    work until a method's fields are within 1% (and, for the record, within
    each of TTF_LEVELS) of a long plain reference.

    Reference: plain DSMC, `ttf_transient` steps, then `ttf_sampled` steps
    averaged; its noise is the difference between its two sampled halves
    (stored with --ttf-ref-out and read back with --ttf-ref-in, so that
    several races share one reference).
    Fields: 10^3 boxes (density, velocity, temperature pooled per box) and
    the two centreline velocity profiles (reported beside the error).
    Error e = max of the relative L2 differences of velocity, density and
    temperature over the boxes.  Each method adds its moment sums every
    `block` steps; at step t its fields are those of the steps since the
    block boundary nearest below t/2 (the last-half window), and its time to
    a level is the first GPU time with e at or below it.  Methods
    (--ttf-methods): plain DSMC; the coupled method with the sampled HoT (one
    coupling cycle every --ttf-window steps on the moving average over 1000
    steps, warm-started from M^k, the particles adjusted to M^{k+1} after
    the solve as in Algorithm 1) with the Newton-Krylov solve (--ttf-nm
    Newton steps, the first coupling --ttf-first-nm) or the pseudo-time
    marching (--ttf-solver march); and the same with the learned closure,
    trained first on five runs at Kn log-spaced in (0.01, 0.1] (Kn 0.01
    held out), 384,000 cells each."""
    import numpy as np
    import torch
    nh, kn, lid = args.ttf_hex, args.ttf_kn, args.ttf_lid
    window = args.ttf_window
    methods = args.ttf_methods.split(",")
    mk = lambda seed, kn_=kn, **kw: W.cavity(n_hex=nh, Kn=kn_, ppc=30, jitter=0.1, vel_fp32=1, seed=seed, n_ss=0,
                                             lid_speed=lid, grade=args.ttf_grade, **kw)
    wl = mk(0)
    G = _ttf_geometry(wl)
    res = {"metric": "GPU seconds to fields within 1% L2 of a long plain reference",
           "config": {"workload": f"cavity_{nh}^3x6_Kn{kn:g}_lid{lid:g}" + (f"_grade{args.ttf_grade:g}"
                                                                              if args.ttf_grade else ""),
                      "ppc": 30, "bins": "10^3 boxes",
                      "block_steps": block, "coupling_window": window, "levels": list(TTF_LEVELS)}}
    log = lambda msg: print("# " + msg, file=sys.stderr, flush=True)

    def stepper(sim, n):
        sim.graph_step(n)

    keys = ("u", "rho", "T", "vline", "hline")
    if args.ttf_ref_in:
        z = np.load(args.ttf_ref_in)
        R = {k: z["R_" + k] for k in keys}
        res["reference"] = json.loads(str(z["meta"]))
        log("reference read from " + args.ttf_ref_in)
    else:
        ref = dsmc.Simulation(mk(101), stream=torch.cuda.Stream())
        t0 = time.perf_counter()
        for done in range(0, args.ttf_transient, 10000):
            stepper(ref, min(10000, args.ttf_transient - done))
            ref.sync()
            log(f"reference transient step {done + min(10000, args.ttf_transient - done)}")
        s_a, n_a = ref.sums(dsmc.SAMPLE_STEADY)
        half = args.ttf_sampled // 2
        marks = []
        for target in (half, args.ttf_sampled):
            done = 0
            while done < target - (0 if not marks else half):
                k = min(10000, target - (0 if not marks else half) - done)
                stepper(ref, k)
                ref.sync()
                done += k
                log(f"reference sampled step {done + (half if marks else 0)}")
            marks.append(ref.sums(dsmc.SAMPLE_STEADY))
        ref_s = time.perf_counter() - t0
        ref.close()
        (s_b, n_b), (s_c, n_c) = marks
        R = _ttf_fields(_ttf_reduce(s_c - s_a, G), n_c - n_a, G, wl)
        R1 = _ttf_fields(_ttf_reduce(s_b - s_a, G), n_b - n_a, G, wl)
        R2 = _ttf_fields(_ttf_reduce(s_c - s_b, G), n_c - n_b, G, wl)
        res["reference"] = {"transient_steps": args.ttf_transient, "sampled_steps": args.ttf_sampled,
                            "seconds": round(ref_s, 1), "halves_difference": _ttf_err(R1, R2)}
        if args.ttf_ref_out:
            np.savez(args.ttf_ref_out, meta=json.dumps(res["reference"]), **{"R_" + k: R[k] for k in keys})
    log(f"reference halves differ by {res['reference']['halves_difference']}")
    log("reference result " + json.dumps(res["reference"]))

    def race(name, sim, cap, couple=None):
        snaps = {0: tuple(np.zeros_like(a) for a in _ttf_reduce(np.zeros((sim.nt, 13)), G))}
        t_gpu, step, hist, reached = 0.0, 0, [], {}
        reps, t_couple = [], 0.0
        while step < cap:
            a = time.perf_counter()
            end = step + block
            while step < end:
                nxt = end if couple is None else min(end, (step // window + 1) * window)
                stepper(sim, nxt - step)
                step = nxt
                if couple is not None and step % window == 0:
                    c0 = time.perf_counter()
                    reps.append(couple(sim, len(reps)))
                    t_couple += time.perf_counter() - c0
            sim.sync()
            t_gpu += time.perf_counter() - a
            S, n = sim.sums(dsmc.SAMPLE_STEADY)
            snaps[step] = _ttf_reduce(S, G)
            h = (step // 2) // block * block
            F = _ttf_fields(tuple(x - y for x, y in zip(snaps[step], snaps[h])), step - h, G, wl)
            err = _ttf_err(F, R)
            hist.append((step, round(t_gpu, 3), {k: round(v, 5) for k, v in err.items()}))
            for lv in TTF_LEVELS:
                if err["e"] <= lv and str(lv) not in reached:
                    reached[str(lv)] = {"step": step, "seconds": round(t_gpu, 2)}
            if step % 5000 == 0 or err["e"] <= 0.01:
                extra = "" if not reps else (f" couple iters {reps[-1]['iters']} krylov {reps[-1]['krylov_steps']} "
                                             f"resid {reps[-1]['residual']:.3g} closure {reps[-1]['n_closure']} "
                                             f"np {reps[-1]['np_after']}")
                log(f"{name} step {step} t {t_gpu:.2f} s e {err['e']:.4f} (u {err['u']:.4f}){extra}")
            if err["e"] <= 0.01:
                break
        out = {"reached": reached.get("0.01"), "levels": reached, "steps_run": step, "seconds_run": round(t_gpu, 2),
               "final_error": hist[-1][2], "history": hist[::max(1, len(hist) // 40)]}
        if reps:
            out["couplings"] = len(reps)
            out["coupling_seconds"] = round(t_couple, 2)
            out["first_coupling"] = {k: reps[0][k] for k in ("iters", "krylov_steps", "residual", "converged",
                                                              "fed_back", "n_rejected")}
            out["last_coupling"] = {k: reps[-1][k] for k in ("iters", "krylov_steps", "residual", "converged",
                                                             "fed_back", "n_rejected", "n_closure", "n_fallback")}
            out["closure_cells_mean"] = float(np.mean([r["n_closure"] for r in reps]))
        log(f"{name} result " + json.dumps(out))
        return out

    if "plain" in methods:
        sim = dsmc.Simulation(mk(102), stream=torch.cuda.Stream())
        res["plain"] = race("plain", sim, args.ttf_cap)
        sim.close()
    nk = args.ttf_solver == "nk"
    prm = dict(kn_max=1.0, passes=3, n_m=args.ttf_nm, eps_m=args.ttf_eps, cfl=args.ttf_cfl, feedback=1,
               warm_start=1, unconverged=1, solver=1 if nk else 0, krylov=args.ttf_krylov if nk else 0)
    first = dict(prm, n_m=args.ttf_first_nm if args.ttf_first_nm > 0 else args.ttf_nm)
    res["coupling"] = dict(prm, first_n_m=first["n_m"])

    def couple(sim, k):
        return sim.dig_couple(**(first if k == 0 else prm))

    if "dig" in methods:
        sim = dsmc.Simulation(mk(103, ewma_on=1, n_a=1000), stream=torch.cuda.Stream())
        res["dig"] = race("dig", sim, args.ttf_dig_cap, couple=couple)
        sim.close()
    if "mlp" in methods:
        # learned closure: training pairs from five other Knudsen numbers,
        # log-spaced in (0.01, 0.1] (Kn 0.01 is held out: it is the race's)
        train_kn = [round(0.01 * 10 ** (i / 5), 4) for i in range(1, 6)]
        xs, ts = [], []
        t0 = time.perf_counter()
        for k, kn_t in enumerate(train_kn):
            tr = dsmc.Simulation(mk(200 + k, kn_=kn_t, ewma_on=1, n_a=1000), stream=torch.cuda.Stream())
            stepper(tr, args.ttf_train_steps)
            tr.dig_couple(**dict(prm, n_m=0, feedback=0))
            x, t, v = tr.closure_data()
            xs.append(x[v]); ts.append(t[v])
            tr.close()
            log(f"closure training data from Kn {kn_t}: {int(v.sum())} cells")
        net = dsmc.Mlp()
        net.init_weights(seed=1)
        X, T = np.concatenate(xs), np.concatenate(ts)
        tr_rep = net.train(X, T, steps=args.ttf_train_iters, batch=4096, lr=1e-3, seed=2)
        torch.cuda.synchronize()
        res["closure_training"] = {"samples": int(len(X)), "knudsen": train_kn,
                                   "steps_per_run": args.ttf_train_steps, "adam_steps": args.ttf_train_iters,
                                   "loss_first": tr_rep["loss_first"], "loss_last": tr_rep["loss_last"],
                                   "seconds": round(time.perf_counter() - t0, 1), "gate_tol": args.ttf_gate}
        sim = dsmc.Simulation(mk(104, ewma_on=1, n_a=1000), stream=torch.cuda.Stream())
        sim.set_closure(net, gate_tol=args.ttf_gate)
        res["dig_mlp"] = race("dig+mlp", sim, args.ttf_dig_cap, couple=couple)
        sim.close()
        net.close()
    print(json.dumps(res))


def mixed_cavity(dsmc, W, n=32):
    """The lid-driven cavity of cavity_large on a mixed-element mesh: n^3
    hexahedral blocks (10 % vertex jitter) split into tetrahedra, pyramids,
    prisms and hexahedra, decomposed by the library into tetrahedra (about
    377,000 for n = 32); Kn 0.1, 30 particles per tetrahedron, FP32
    velocities."""
    import numpy as np
    m = W.mixed_box(n, n, n, jitter=0.1, seed=1)
    d = dsmc.decompose(m.xyz, m.cells, m.bfaces, m.bgroup)
    mesh = W.Mesh(xyz=d["xyz"], tets=d["tets"], bfaces=d["bfaces"], bgroup=d["bgroup"], bpartner=None, h=m.h)
    wl = W.cavity_on_mesh(mesh, Kn=0.1, ppc=30, vel_fp32=1, n_ss=10000, steps=20000,
                          name=f"mixed_cavity_{n}^3_Kn0.1")
    kinds, counts = np.unique(m.kind, return_counts=True)
    names = {4: "tetrahedra", 5: "pyramids", 6: "prisms", 8: "hexahedra"}
    wl.info["cells"] = {names[int(k)]: int(c) for k, c in zip(kinds, counts)}
    return wl


def bench_coarse_fields(args, dsmc, W):
    """Fields on coarse meshes against a resolved reference, the comparison
    behind the paper's cavity cost table (its coupled method runs on a mesh
    far coarser than the one plain DSMC needs): the lid-driven cavity (lid
    50 m/s) at Kn --cf-kn; reference = plain DSMC on --cf-ref-hex^3 x 6
    tets, --cf-transient steps then --cf-sampled sampled; then, on each
    mesh of --cf-hex, plain DSMC and the coupled method (sampled HoT, one
    Newton-Krylov coupling cycle every --cf-window steps throughout, warm
    started, feedback after each solve) for the same steps with --cf-ppc
    particles per tet.  Fields pooled over 10^3 boxes as in the time-to-
    fields record; reported: each run's error against the reference, the
    reference's half-to-half difference and the GPU seconds."""
    import numpy as np
    import torch
    kn, T, S = args.cf_kn, args.cf_transient, args.cf_sampled
    log = lambda msg: print("# " + msg, file=sys.stderr, flush=True)

    def mk(nh, ppc, seed, **kw):
        return W.cavity(n_hex=nh, Kn=kn, ppc=ppc, jitter=0.1, vel_fp32=1, seed=seed, n_ss=T, lid_speed=50.0, **kw)

    def run(wl, couple=None, halves=False):
        sim = dsmc.Simulation(wl, stream=torch.cuda.Stream())
        G = _ttf_geometry(wl)
        t0 = time.perf_counter()
        reps = []
        marks = []
        step, total = 0, T + S
        targets = [T + S // 2, T + S] if halves else [T + S]
        while step < total:
            nxt = min(total, step + (args.cf_window if couple else 10000))
            for t in targets:
                if step < t < nxt:
                    nxt = t
            sim.graph_step(nxt - step)
            step = nxt
            if couple and step % args.cf_window == 0 and step < total:
                reps.append(sim.dig_couple(**couple))
            if step in targets:
                sim.sync()
                marks.append(sim.sums(dsmc.SAMPLE_STEADY))
        sim.sync()
        secs = time.perf_counter() - t0
        sim.close()
        fields = [_ttf_fields(_ttf_reduce(sm, G), n, G, wl) for sm, n in marks]
        if halves:
            (s1, n1), (s2, n2) = marks
            fields = [_ttf_fields(_ttf_reduce(s1, G), n1, G, wl),
                      _ttf_fields(_ttf_reduce(s2 - s1, G), n2 - n1, G, wl),
                      _ttf_fields(_ttf_reduce(s2, G), n2, G, wl)]
        return fields, secs, reps

    out = {"metric": "relative L2 field error against a resolved plain-DSMC reference",
           "config": {"workload": f"cavity_Kn{kn:g}_lid50", "reference_mesh": f"{args.cf_ref_hex}^3x6",
                      "transient_steps": T, "sampled_steps": S, "coupling_window": args.cf_window,
                      "coarse_ppc": args.cf_ppc}, "runs": []}
    (R1, R2, R), secs, _ = run(mk(args.cf_ref_hex, 30, 301), halves=True)
    out["reference"] = {"seconds": round(secs, 1), "halves_difference": _ttf_err(R1, R2)}
    log("reference " + json.dumps(out["reference"]))
    prm = dict(kn_max=1.0, passes=3, n_m=20, eps_m=1e-3, cfl=10.0, feedback=1, warm_start=1, unconverged=1,
               solver=1, krylov=40)
    for nh in [int(x) for x in args.cf_hex.split(",")]:
        for name, cpl in (("plain", None), ("coupled", prm)):
            wl = mk(nh, args.cf_ppc, 302 + nh, **({"ewma_on": 1, "n_a": 1000} if cpl else {}))
            (F,), secs, reps = run(wl, couple=cpl)
            e = _ttf_err(F, R)
            r = {"n_hex": nh, "method": name, "tets": int(wl.mesh.n_tets), "seconds": round(secs, 2),
                 "error": {k: round(v, 5) for k, v in e.items()}}
            if reps:
                r["couplings"] = len(reps)
                r["last_coupling"] = {k: reps[-1][k] for k in ("iters", "krylov_steps", "residual", "failed",
                                                               "fed_back")}
            log(json.dumps(r))
            out["runs"].append(r)
    print(json.dumps(out))


def bench_dig_bias(args, dsmc, W):
    """Fixed point of the coupling step against the DSMC steady state: the
    lid-driven cavity at Kn 0.01 (lid 50 m/s, 30 particles per cell) on
    n^3 x 6 tets for each n of --bias-hex, plain DSMC for --bias-transient
    steps, then the moving average restarted and run for --bias-avg steps;
    one coupling cycle without feedback solves the synthetic equations to a
    1e-7 density residual ratio (Newton-Krylov) from that state with its
    HoT.  Reported: the relative L2 difference of the solved and the sampled
    velocity pooled over 10^3 boxes (the time-to-fields metric) and the
    ratio of their norms.  A consistent fixed point would give the sampled
    state's noise only (which shrinks with the averaging length)."""
    import numpy as np
    import torch
    out = {"metric": "relative L2 difference of solved and sampled box velocities",
           "config": {"workload": f"cavity_Kn{args.bias_kn:g}_lid50", "ppc": 30, "jitter": args.bias_jitter,
                      "grade": args.bias_grade,
                      "transient_steps": args.bias_transient, "averaged_steps": args.bias_avg},
           "meshes": []}
    rel = lambda a, b: float(np.linalg.norm(a - b) / np.linalg.norm(b))
    for nh in [int(x) for x in args.bias_hex.split(",")]:
        wl = W.cavity(n_hex=nh, Kn=args.bias_kn, ppc=30, jitter=args.bias_jitter, vel_fp32=1, seed=7, n_ss=0,
                      lid_speed=50.0, ewma_on=1, n_a=args.bias_avg, grade=args.bias_grade)
        G = _ttf_geometry(wl)
        vol = G["vol"]

        def boxed(P):
            w = P[:, 0] * vol
            num = np.stack([np.bincount(G["bin"], weights=w * P[:, 1 + k], minlength=G["nbins"]) for k in range(3)],
                           axis=1)
            return num / np.bincount(G["bin"], weights=w, minlength=G["nbins"])[:, None]

        sim = dsmc.Simulation(wl, stream=torch.cuda.Stream())
        t0 = time.perf_counter()
        for done in range(0, args.bias_transient, 10000):
            sim.graph_step(min(10000, args.bias_transient - done))
            sim.sync()
        sim.set_sums(dsmc.SAMPLE_EWMA, np.zeros((sim.nt, 13)), np.zeros(sim.nt, np.int32))
        for done in range(0, args.bias_avg, 10000):
            sim.graph_step(min(10000, args.bias_avg - done))
            sim.sync()
            print(f"# n_hex {nh}: averaged {done + min(10000, args.bias_avg - done)} steps", file=sys.stderr, flush=True)
        t1 = time.perf_counter()
        rep = sim.dig_couple(kn_max=1.0, passes=3, feedback=0, warm_start=0, n_m=200, eps_m=1e-7, cfl=10.0,
                             solver=1, krylov=40)
        t2 = time.perf_counter()
        ph, pn = sim.dig_get("half"), sim.dig_get("new")
        half, new = boxed(ph), boxed(pn)
        # where the difference lies: cells near the lid's four edges (within
        # 0.1 of the cavity length), and the boxes of largest difference
        cen = wl.mesh.xyz[wl.mesh.tets].mean(axis=1)
        edge = np.minimum.reduce([np.hypot(1 - cen[:, 1], cen[:, 0]), np.hypot(1 - cen[:, 1], 1 - cen[:, 0]),
                                  np.hypot(1 - cen[:, 1], cen[:, 2]), np.hypot(1 - cen[:, 1], 1 - cen[:, 2])])
        du2 = vol * ((pn[:, 1:4] - ph[:, 1:4]) ** 2).sum(axis=1)
        near = edge < 0.1
        d2 = ((new - half) ** 2).sum(axis=1)
        top = np.argsort(-d2)[:5]
        nb = round(G["nbins"] ** (1 / 3))
        centres = (np.stack(np.unravel_index(top, (nb, nb, nb)), axis=1) + 0.5) / nb
        m = {"n_hex": nh, "tets": sim.nt, "solved_vs_sampled": round(rel(new, half), 5),
             "norm_ratio": round(float(np.linalg.norm(new) / np.linalg.norm(half)), 5),
             "lid_edge_cells": round(float(near.mean()), 4),
             "lid_edge_share_of_difference": round(float(du2[near].sum() / du2.sum()), 4),
             "largest_boxes": [[round(float(x), 2) for x in c] + [round(float(np.sqrt(d2[k])), 3),
                                                                   round(float(np.linalg.norm(half[k])), 2)]
                               for c, k in zip(centres, top)],
             "newton_steps": rep["iters"], "krylov_steps": rep["krylov_steps"], "converged": rep["converged"],
             "dsmc_seconds": round(t1 - t0, 1), "solve_seconds": round(t2 - t1, 2)}
        print("# " + json.dumps(m), file=sys.stderr, flush=True)
        out["meshes"].append(m)
        sim.close()
    print(json.dumps(out))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--workload", default="cavity_large",
                    choices=["cavity_large", "cavity_small", "cavity_vss", "cavity_n2", "cavity_mixed",
                             "ensemble64", "dig_cavity40", "time_to_fields", "dig_bias", "coarse_fields", "sphere"])
    ap.add_argument("--dig-solver", default="march", choices=["march", "nk"], help="solve of dig_cavity40")
    ap.add_argument("--cf-kn", type=float, default=0.05)
    ap.add_argument("--cf-ref-hex", type=int, default=40)
    ap.add_argument("--cf-hex", default="10,20")
    ap.add_argument("--cf-ppc", type=int, default=120)
    ap.add_argument("--cf-transient", type=int, default=5000)
    ap.add_argument("--cf-sampled", type=int, default=40000)
    ap.add_argument("--cf-window", type=int, default=200)
    ap.add_argument("--bias-hex", default="20,30,40", help="mesh sizes of the dig_bias workload")
    ap.add_argument("--bias-jitter", type=float, default=0.1)
    ap.add_argument("--bias-grade", type=float, default=0.0, help="wall refinement of the dig_bias meshes")
    ap.add_argument("--bias-kn", type=float, default=0.01)
    ap.add_argument("--bias-transient", type=int, default=10000)
    ap.add_argument("--bias-avg", type=int, default=80000)
    ap.add_argument("--ttf-hex", type=int, default=40)
    ap.add_argument("--ttf-kn", type=float, default=0.01)
    ap.add_argument("--ttf-lid", type=float, default=50.0)
    ap.add_argument("--ttf-grade", type=float, default=0.0, help="wall refinement of the time-to-fields mesh")
    ap.add_argument("--ttf-transient", type=int, default=50000)
    ap.add_argument("--ttf-sampled", type=int, default=100000)
    ap.add_argument("--ttf-cap", type=int, default=120000, help="plain DSMC steps at most")
    ap.add_argument("--ttf-dig-cap", type=int, default=40000, help="coupled-method steps at most")
    ap.add_argument("--ttf-methods", default="plain,dig,mlp", help="races to run: plain, dig, mlp")
    ap.add_argument("--ttf-solver", default="nk", choices=["nk", "march"])
    ap.add_argument("--ttf-window", type=int, default=500, help="DSMC steps between coupling cycles")
    ap.add_argument("--ttf-nm", type=int, default=20, help="Newton steps (marching: iterations) per coupling")
    ap.add_argument("--ttf-first-nm", type=int, default=80, help="the same for the first coupling (0: --ttf-nm)")
    ap.add_argument("--ttf-eps", type=float, default=1e-3)
    ap.add_argument("--ttf-cfl", type=float, default=10.0)
    ap.add_argument("--ttf-krylov", type=int, default=40)
    ap.add_argument("--ttf-ref-out", default="", help="store the reference fields (.npz)")
    ap.add_argument("--ttf-ref-in", default="", help="read the reference fields (.npz) instead of running it")
    ap.add_argument("--ttf-gate", type=float, default=0.5)
    ap.add_argument("--ttf-train-steps", type=int, default=3000)
    ap.add_argument("--ttf-train-iters", type=int, default=2000)
    ap.add_argument("--graph", action="store_true",
                    help="step through captured HIP graphs (the default for the cavity workloads)")
    ap.add_argument("--eager", action="store_true", help="step with ordinary launches instead of graphs")
    ap.add_argument("--cpu-steps", type=int, default=4,
                    help="oracle steps of the benchmark workload timed single-threaded")
    ap.add_argument("--cpu-procs", type=int, default=0,
                    help="concurrent oracle processes of the aggregate (0: the host's cores, at most 16)")
    ap.add_argument("--cpu-only", action="store_true", help="time the oracle alone (no GPU)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="time a plain device copy of 2 GiB (HBM calibration of the traffic counters)")
    ap.add_argument("--calibrate-l1", action="store_true",
                    help="time scattered line reads (vector-L1 access-rate calibration)")
    args = ap.parse_args()
    args.graph = not args.eager
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the multi-GPU decomposition is "
              "described, not implemented", file=sys.stderr)
        sys.exit(2)

    procs = args.cpu_procs or max(1, min(16, os.cpu_count() or 1))
    if args.cpu_only:
        from paper_2607_08195_amd import workloads as W
        wl = W.cavity_large()
        print(json.dumps({"workload": wl.name, "cpu_baseline": cpu_baseline(wl, args.cpu_steps, procs)}))
        return

    import numpy as np
    import torch
    from paper_2607_08195_amd import dsmc, workloads as W

    if args.calibrate_copy:
        return calibrate_copy(dsmc, W)
    if args.calibrate_l1:
        return calibrate_l1(dsmc, W)
    if args.workload == "ensemble64":
        return bench_ensemble(args, dsmc, W)
    if args.workload == "sphere":
        return bench_sphere(args, dsmc, W)
    if args.workload == "dig_cavity40":
        return bench_dig(args, dsmc, W)
    if args.workload == "time_to_fields":
        return bench_time_to_fields(args, dsmc, W)
    if args.workload == "dig_bias":
        return bench_dig_bias(args, dsmc, W)
    if args.workload == "coarse_fields":
        return bench_coarse_fields(args, dsmc, W)
    wl = {"cavity_large": W.cavity_large, "cavity_vss": W.cavity_large_vss, "cavity_small": W.cavity_small,
          "cavity_n2": W.cavity_large_n2, "cavity_mixed": lambda: mixed_cavity(dsmc, W)}[args.workload]()
    sim = dsmc.Simulation(wl)
    np0 = sim.stats()["n_particles"]
    sim.step(args.warmup)
    sim.sync()
    s0 = sim.stats()
    torch.cuda.synchronize()
    if args.graph:
        sim.close()
        stream = torch.cuda.Stream()
        sim = dsmc.Simulation(wl, stream=stream)
        sim.graph_step(args.warmup)
        sim.sync()
        s0 = sim.stats()
    sim.profile(not args.graph)
    t0 = time.perf_counter()
    if args.graph:
        sim.graph_step(args.steps)
    else:
        sim.step(args.steps)
    sim.sync()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = sim.profile_read()
    sim.profile(False)
    s1 = sim.stats()
    if args.graph:
        # kernel times come from HIP events, which a replayed graph does not
        # record: time a few ordinary steps of the same state for them
        sim.profile(True)
        sim.step(10)
        sim.sync()
        prof = sim.profile_read()
        sim.profile(False)
    elapsed = t1 - t0
    npart = 0.5 * (s0["n_particles"] + s1["n_particles"])
    psteps = npart * args.steps
    value = psteps / elapsed
    walls_pp = (s1["wall_hits"] - s0["wall_hits"]) / psteps
    hops_pp = (s1["hops"] - s0["hops"]) / psteps
    nt = sim.nt
    _, nacc = sim.pair_counts()
    touched_pp = 2.0 * nacc.sum() / max(npart, 1)

    per_launch = {}
    for name, (ms, cnt) in prof.items():
        if cnt:
            per_launch[name] = ms / cnt
    stage_ms = {k: sum(per_launch.get(n, 0.0) for n in ks) for k, ks in STAGES.items()}
    frac = {"walls": walls_pp, "touched": touched_pp, "rot": 1.0 if wl.species.dof_rot else 0.0}
    bytes_launch = {k: fn(npart, nt, frac) for k, fn in BYTES.items()}
    gbs = {k: bytes_launch[k] / (stage_ms[k] * 1e-3) / 1e9 for k in bytes_launch if stage_ms[k] > 0}
    dominant = max(gbs, key=lambda k: stage_ms[k])
    step_bytes = sum(bytes_launch.values())
    peak = 8000.0
    digest = _kernel_digest()
    traffic = None
    if (TRAFFIC and TRAFFIC.get("digest") == digest and TRAFFIC.get("stage") == dominant
            and TRAFFIC.get("workload") == wl.name):
        traffic = TRAFFIC["bytes_per_launch"] / 1e9 / (stage_ms[dominant] * 1e-3)
    roofline = dict(bound="hbm", kernel=dominant, kernels=STAGES[dominant], achieved=round(gbs[dominant], 1),
                    peak=peak, unit="GB/s", frac=round(gbs[dominant] / peak, 4),
                    traffic=None if traffic is None else round(traffic, 1),
                    bytes_per_particle_step=round(bytes_launch[dominant] / npart, 2))
    copy_gbs = copy_rate(sim)
    # the move kernel against the vector L1's line-access rate, measured here
    l1 = None
    if L1 and L1.get("digest") == digest and L1.get("workload") == wl.name and per_launch.get("move", 0) > 0:
        lr = line_read_rate(sim)
        peak_l1 = max(v["per_cu_ns"] for v in lr.values())
        floor_ms = L1["accesses_per_launch"] / 256 / peak_l1 / 1e6
        l1 = {"kernel": "move", "accesses_per_launch": L1["accesses_per_launch"],
              "peak_per_cu_ns": peak_l1, "floor_ms": round(floor_ms, 4), "kernel_ms": round(per_launch["move"], 4),
              "frac": round(floor_ms / per_launch["move"], 4)}

    out = {
        "metric": "particle-steps/s",
        "value": value,
        "unit": "particle-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * elapsed / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": wl.name, "tets": nt, "particles": int(np0),
                   "Kn": wl.info.get("Kn"), "velocity_storage": "f32" if wl.run.vel_fp32 else "f64",
                   **({"gas": "nitrogen, 2 rotational degrees of freedom"} if wl.species.dof_rot else {}),
                   **({"cells": wl.info["cells"]} if "cells" in wl.info else {})},
        "launch": "hip_graph" if args.graph else "eager",
        "step_algorithmic_GBps": round(step_bytes / (elapsed / args.steps) / 1e9, 1),
        "hops_per_particle_step": round(hops_pp, 3),
        "kernel_ms": {k: round(v, 4) for k, v in per_launch.items()},
        "stage_ms": {k: round(v, 4) for k, v in stage_ms.items()},
        "stage_algorithmic_GBps": {k: round(v, 1) for k, v in gbs.items()},
        "step_algorithmic_bytes_per_particle": round(step_bytes / npart, 1),
        "roofline": roofline,
        "l1_roofline": l1,
        "copy_kernel_GBps": round(copy_gbs, 1),
        "kernel_digest": digest,
    }
    sim.close()
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(wl, args.cpu_steps, procs)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
