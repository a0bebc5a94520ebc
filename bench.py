"""Benchmark: IPC Newton steps of the contact-rich soft-gripper scene on one MI355X.

Workload: two 10k-tet pads squeezing a ~180k-tet soft cylinder (log-normal
Young's modulus) that rests on a finely meshed static ground patch, 200k tets
in all, dhat = 5e-4 m, dt = 5 ms.  Synthetic seeded geometry; FP64 throughout.

Timed: K full steps (every Newton iteration with assembly, PCG, CCD, line
search), after W untimed warm-up steps, between device synchronisations; by
default steps 2-100 of the scene (K = 99, W = 1): the squeeze and the lift.  The
JSON line reports Newton iterations per second as ``value`` plus steps per
second, the roofline object of the dominant kernel (durations from HIP events
the library records on its own stream during the timed steps) and the oracle's
CPU throughput on a bounded sample of the same workload.
"""
import argparse
import ctypes
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Newton iters/s & sim steps/s at 200k tets; batched scenes/s; adjoint/forward time"
HBM_PEAK_GBS = 8000.0
K_SPMV = 0   # the library's timed-kernel id of the Hessian product
# calibrated hardware traffic of the product, valid while its source is unchanged
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_spmv_contact_rich_200k_traffic.json")
PRODUCT_SRC = os.path.join(ROOT, "paper_2609_25653_amd", "csrc", "ipc_solver.hip")


def product_traffic():
    """Per-launch HBM bytes of the product from the committed counter runs, or
    None when the product's source file changed since they were taken."""
    import hashlib
    try:
        rec = json.load(open(TRAFFIC_FILE))
        sha = hashlib.sha256(open(PRODUCT_SRC, "rb").read()).hexdigest()
    except (OSError, ValueError):
        return None
    return rec.get("bytes_per_launch") if rec.get("source_sha256") == sha else None


def cpu_baseline(scene):
    """The oracle on the host cores: one complete Newton iteration of step 0
    of the same scene (step set-up with its broad phase and friction lag,
    assembly, PCG to the scene's tolerance, CCD and line search), timed as a
    whole.  The oracle runs its FEM element loop on OpenMP threads and
    everything else on one thread."""
    import numpy as np
    import oracle as O
    sc = dict(scene)
    sc["max_newton"] = np.asarray(1.0)   # stop after the first Newton iteration
    o = O.Oracle(sc)
    t0 = time.perf_counter()
    rc, st = o.step()
    t = time.perf_counter() - t0
    threads = int(os.environ.get("OMP_NUM_THREADS", len(os.sched_getaffinity(0))))
    try:
        model = [l.split(":", 1)[1].strip() for l in open("/proc/cpuinfo") if l.startswith("model name")][0]
    except Exception:
        model = "unknown"
    return {"value": 1.0 / t, "unit": "Newton iters/s", "cores": threads, "kind": "oracle",
            "sample": (f"one complete Newton iteration of step 0 of the 200k-tet scene ({t:.1f} s: set-up, assembly, "
                       f"{st['pcg_iters_total']} PCG iterations, CCD, line search); OpenMP on {threads} threads over the "
                       f"FEM element loop only, the rest single-threaded; CPU {model}")}


def bench_oracle(args):
    """The oracle alone on the host cores (no GPU): the first --steps steps of
    the 200k-tet squeeze, each complete, with the number of OpenMP threads
    that OMP_NUM_THREADS gives (the FEM element loop; the rest runs on one
    thread).  The CPU baseline of the contact workload over whole steps."""
    import numpy as np
    import ipcscenes
    import oracle as O
    scene = ipcscenes.contact_rich(n_steps=args.steps, s_g=args.s_g)
    o = O.Oracle(scene)
    threads = int(os.environ.get("OMP_NUM_THREADS", len(os.sched_getaffinity(0))))
    try:
        model = [l.split(":", 1)[1].strip() for l in open("/proc/cpuinfo") if l.startswith("model name")][0]
    except Exception:
        model = "unknown"
    steps = []
    t0 = time.perf_counter()
    for k in range(args.steps):
        ts = time.perf_counter()
        rc, st = o.step()
        dt = time.perf_counter() - ts
        steps.append({"step": k, "status": int(rc), "newton": int(st["newton_iters"]), "pcg": int(st["pcg_iters_total"]),
                      "s": dt})
        print(f"# oracle step {k}: rc={rc} newton={st['newton_iters']} pcg={st['pcg_iters_total']} {dt:.1f} s",
              file=sys.stderr, flush=True)
    t = time.perf_counter() - t0
    newton = sum(x["newton"] for x in steps)
    print(json.dumps({
        "metric": "oracle Newton iters/s at 200k tets", "value": newton / t, "unit": "Newton iters/s", "steps": args.steps,
        "steps_per_s": args.steps / t, "newton_per_step": newton / args.steps, "kind": "oracle", "cores": threads,
        "cpu": model, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "contact-rich squeeze: 2 pads + soft cylinder on a ground patch",
                   "tets": int(len(scene["tets"])), "ground_spacing": args.s_g},
        "per_step": steps}))


def write_traffic(fetch_csv, write_csv):
    """Calibrate FETCH_SIZE / WRITE_SIZE (KiB per dispatch) by the 256 MiB
    device copy of a --traffic-run and store the product's bytes per launch
    (mean over the dispatches of the product variant the solver used)."""
    import csv
    import hashlib

    def per_kernel(path):
        out = {}
        for r in csv.DictReader(open(path)):
            out.setdefault(r["Kernel_Name"], []).append(float(r["Counter_Value"]))
        return out

    f, w = per_kernel(fetch_csv), per_kernel(write_csv)
    copy = [k for k in f if "copyBuffer" in k]
    # the product variant the solver runs (one lane count per run)
    spmv = [max((k for k in f if "k_spmv" in k), key=lambda k: len(f[k]))]
    kib = 256 * 1024   # the probe copies 256 MiB
    fac_f = kib / max(max(f[k]) for k in copy)
    fac_w = kib / max(max(w[k]) for k in copy)
    sf = [v for k in spmv for v in f[k]]
    sw = [v for k in spmv for v in w[k]]
    traffic = 1024.0 * (fac_f * sum(sf) / len(sf) + fac_w * sum(sw) / len(sw))
    rec = {"kernel": "k_spmv", "bytes_per_launch": traffic, "fetch_kib": sum(sf) / len(sf), "write_kib": sum(sw) / len(sw),
           "fetch_scale": fac_f, "write_scale": fac_w, "launches": len(sf),
           "source_sha256": hashlib.sha256(open(PRODUCT_SRC, "rb").read()).hexdigest()}
    rec["source"] = "python bench.py --traffic-run (1 warm-up + 1 timed step of the contact workload) under rocprofv3 --pmc"
    json.dump(rec, open(TRAFFIC_FILE, "w"), indent=1)
    print(json.dumps(rec))


def probe_spmv(sim):
    """One assembly, one plain copy of known size, then 20 timed products."""
    import torch
    from paper_2609_25653_amd import lib
    y, _ = sim.state()
    sim.begin_step(0)
    sim.energy_grad_hess(y, torch.ones_like(y), energy=False, grad=False)
    src = torch.ones(32 << 20, dtype=torch.float64, device="cuda")   # 256 MiB
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    lanes, times = sim.autotune(20)
    us, by = ctypes.c_double(), ctypes.c_double()
    sim._check(lib().ipc_time_kernel(sim._h, 0, 20, ctypes.byref(us), ctypes.byref(by)))
    print(json.dumps({"probe": "spmv", "lanes_per_row": lanes, "autotune_us": times, "copy_bytes_read": src.numel() * 8, "copy_bytes_written": dst.numel() * 8,
                      "spmv_launches": 20, "spmv_avg_us": us.value, "spmv_algorithmic_bytes": by.value}))


def copy_bandwidth():
    """The measured achievable bandwidth: a plain 1 GiB device-to-device copy
    (torch's copy kernel; read + write bytes), best of 6, between CUDA events
    on torch's stream."""
    import torch
    n = 1 << 27
    src = torch.ones(n, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    best = float("inf")
    for _ in range(6):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        dst.copy_(src)
        e1.record()
        e1.synchronize()
        best = min(best, e0.elapsed_time(e1))
    del src, dst
    torch.cuda.empty_cache()
    return 2.0 * n * 8 / (best * 1e-3) / 1e9


def product_roofline(sim, lib, traffic=None):
    """The Hessian product's roofline: algorithmic bytes per launch over its
    average duration inside PCG during the last timed step (HIP events that
    each dispatch records; the step ran with ipc_profile on), and, as a
    secondary figure, over 200 back-to-back launches on the last matrix."""
    tot, nl, by = ctypes.c_double(), ctypes.c_int64(), ctypes.c_double()
    sim._check(lib().ipc_kernel_time(sim._h, K_SPMV, ctypes.byref(tot), ctypes.byref(nl), ctypes.byref(by)))
    sim._check(lib().ipc_profile(sim._h, 0))
    us_pcg = 1e3 * tot.value / max(nl.value, 1)
    bytes_launch = by.value / max(nl.value, 1)
    us, by2 = ctypes.c_double(), ctypes.c_double()
    sim._check(lib().ipc_time_kernel(sim._h, K_SPMV, 200, ctypes.byref(us), ctypes.byref(by2)))
    achieved = bytes_launch / (us_pcg * 1e-6) / 1e9
    copy = copy_bandwidth()
    b2b = by2.value / (us.value * 1e-6) / 1e9
    return {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
            "achievable": {"copy_gbs": copy, "frac_of_copy": achieved / copy, "back_to_back_frac_of_copy": b2b / copy,
                           "note": "a plain 1 GiB device copy (read + write), best of 6: the measured bandwidth ceiling"},
            "traffic": traffic, "kernel": "k_spmv (Hessian product: block CSR + row-sorted pair-local blocks)",
            "bytes_per_launch": bytes_launch, "avg_us": us_pcg, "launches_timed": int(nl.value),
            "timing": "HIP events stamped by each product launch inside PCG during the last timed step",
            "back_to_back": {"avg_us": us.value, "achieved": by2.value / (us.value * 1e-6) / 1e9,
                             "frac": by2.value / (us.value * 1e-6) / 1e9 / HBM_PEAK_GBS, "launches_timed": 200,
                             "timing": "200 back-to-back launches on the last matrix between two HIP events"},
            "traffic_note": "FETCH_SIZE + WRITE_SIZE: bytes between L2 and the memory fabric (Infinity Cache or HBM)"}


def bench_batched(args):
    """256 squeeze scenes of 1k-40k tets stepped together, against a sample of
    the same scenes spread over the size range, each stepped alone."""
    import numpy as np
    import torch
    import ipcscenes
    from paper_2609_25653_amd import Sim, lib
    n_total = args.warmup + args.steps
    scenes = ipcscenes.batched_squeeze(n_scenes=args.scenes, n_steps=n_total)
    tets = np.array([len(s["tets"]) for s in scenes])
    t0 = time.perf_counter()
    sim = Sim(scenes)
    t_create = time.perf_counter() - t0
    print(f"# batched: {len(scenes)} scenes, {tets.sum()} tets, created in {t_create:.1f} s", file=sys.stderr, flush=True)
    # A scene whose Newton loop ends without convergence (3) or without a
    # decreasing line-search step (4) stays at its last iterate and goes on;
    # such scene-steps are counted and named, and left out of the throughput.
    ok_codes = (3, 4)
    status = {}
    failed = []
    for _ in range(args.warmup):
        sim.step(allow_status=ok_codes)
    lanes, _ = sim.autotune(10)
    torch.cuda.synchronize()
    newton = []
    t0 = time.perf_counter()
    for k in range(args.steps):
        if k == args.steps - 1:
            # the product's launches inside PCG stamp HIP events in the last
            # timed step, as in the contact workload
            sim._check(lib().ipc_profile(sim._h, 1))
        rc, st = sim.step(allow_status=ok_codes)
        for i, s in enumerate(st):
            status[s["status"]] = status.get(s["status"], 0) + 1
            if s["status"] != 0:
                failed.append({"step": sim.step_index - 1, "scene": i, "status": s["status"], "tets": int(tets[i]),
                               "E": float(scenes[i]["tet_E"][0]), "mu": float(scenes[i]["mu"]),
                               "newton": s["newton_iters"], "alpha_min": s["alpha_min"]})
                print(f"# step {sim.step_index - 1} scene {i}: status {s['status']} tets={tets[i]} newton={s['newton_iters']} "
                      f"alpha_min={s['alpha_min']:.3g} pairs={s['n_pt_max'] + s['n_ee_max']}", file=sys.stderr, flush=True)
        newton.append(max(s["newton_iters"] for s in st))
        print(f"# step {sim.step_index}: rc={rc} max newton={newton[-1]} "
              f"pairs={sum(s['n_pt_max'] + s['n_ee_max'] for s in st)}", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t = time.perf_counter() - t0
    converged = status.get(0, 0)
    roof = product_roofline(sim, lib)
    # one at a time: a sample spread over the size range, same steps
    order = np.argsort(tets)
    pick = order[np.linspace(0, len(scenes) - 1, min(args.single_sample, len(scenes))).round().astype(int)]
    t_single = 0.0
    single_ok = single_all = 0
    for i in pick:
        s1 = Sim(scenes[i])
        for _ in range(args.warmup):
            s1.step(allow_status=ok_codes)
        s1.autotune(5)
        torch.cuda.synchronize()
        a = time.perf_counter()
        for _ in range(args.steps):
            _, st1 = s1.step(allow_status=ok_codes)
            single_ok += st1[0]["status"] == 0
            single_all += 1
        torch.cuda.synchronize()
        t_single += time.perf_counter() - a
        del s1
    # converged scene-steps per second of the sample, as for the batch
    single_rate = single_ok / t_single
    line = {
        "metric": "batched scene-steps/s", "value": converged / t, "unit": "scene-steps/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": 1e3 * t / args.steps, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"{len(scenes)} uneven squeeze scenes stepped together", "tets": int(tets.sum()),
                   "tets_min": int(tets.min()), "tets_max": int(tets.max()), "parallelism": "single GPU"},
        "value_counts": "converged scene-steps only",
        "one_at_a_time": {"value": single_rate, "unit": "scene-steps/s",
                          "sample": f"{len(pick)} scenes spread over the size range, each stepped alone over the same steps "
                                    f"({single_ok} of {single_all} scene-steps converged)"},
        "speedup_vs_one_at_a_time": (converged / t) / single_rate,
        "max_newton_per_step": newton, "spmv_lanes_per_row": lanes, "fem_blocks": list(sim.fem_blocks), "pcg_coarse": sim.pcg_coarse,
        "roofline": roof,
        "scene_steps_by_status": {str(k): v for k, v in sorted(status.items())},
        "failed_scene_steps": failed,
    }
    print(json.dumps(line))


def bench_adjoint(args):
    """Squeeze steps 40-89 with theta = (E per pad tet, mu): forward rollout
    with checkpoints every 10 steps, then the backward pass (recompute + one
    adjoint solve per step); loss = squared distance of the 64 tracked pad
    vertices to targets from a run with perturbed theta, summed over steps."""
    import numpy as np
    import torch
    import ipcscenes
    from paper_2609_25653_amd import Sim
    from paper_2609_25653_amd.rollout import rollout
    sc, info = ipcscenes.adjoint_squeeze(0)
    first, K, every = info["first_step"], info["n_steps"], info["checkpoint_every"]
    sim = Sim(sc)
    for k in range(first):
        sim.step(k, allow_status=(3,))
    lanes, _ = sim.autotune(10)
    y0, v0 = sim.state()
    y0, v0 = y0.clone(), v0.clone()
    tr = torch.as_tensor(info["tracked"], device="cuda").long()
    idx = (3 * tr[:, None] + torch.arange(3, device="cuda")[None, :]).reshape(-1)
    E0 = torch.as_tensor(sc["tet_E"], device="cuda")
    mu0 = float(sc["mu"])
    # targets: the tracked vertices over the same window with perturbed parameters
    with torch.no_grad():
        Et = E0 * torch.as_tensor(info["target_E_scale"], device="cuda")
        _, _, targets = rollout(sim, Et, mu0 * info["target_mu_scale"], y0, v0, first, K, every, observe=idx)
    def run(every):
        E = E0.clone().requires_grad_(True)
        mu = torch.tensor([mu0], dtype=torch.float64, device="cuda", requires_grad=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, _, Y = rollout(sim, E, mu, y0, v0, first, K, every, observe=idx)
        loss = ((Y - targets) ** 2).sum()
        torch.cuda.synchronize()
        t_fwd = time.perf_counter() - t0
        t0 = time.perf_counter()
        loss.backward()
        torch.cuda.synchronize()
        return t_fwd, time.perf_counter() - t0, loss, E, mu

    # with checkpoints every `every` steps (the backward pass recomputes each
    # segment), then with every state kept (no recompute): the backward pass
    # is then the adjoint solves and VJPs alone
    t_fwd, t_bwd, loss, E, mu = run(every)
    t_fwd_keep, t_bwd_keep, loss_keep, E_keep, mu_keep = run(0)
    same = bool(torch.equal(E.grad, E_keep.grad)) and bool(torch.equal(mu.grad, mu_keep.grad))
    line = {
        "metric": "adjoint/forward time", "value": t_bwd / t_fwd, "unit": "ratio", "n_gpus": 1, "steps": K, "warmup": first,
        "ms_per_step": 1e3 * t_fwd / K, "higher_is_better": False, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "squeeze steps 40-89, theta = per-tet E (20k) and mu, 64 tracked vertices",
                   "tets": int(len(sc["tets"])), "parallelism": "single GPU"},
        "forward_s": t_fwd, "backward_s": t_bwd, "backward_ms_per_step": 1e3 * t_bwd / K,
        "note": f"value: backward (recompute of each {every}-step segment from its checkpoint + one adjoint solve per "
                f"step) over forward",
        "without_recompute": {"forward_s": t_fwd_keep, "backward_s": t_bwd_keep, "ratio": t_bwd_keep / t_fwd_keep,
                              "backward_ms_per_step": 1e3 * t_bwd_keep / K, "forward_ms_per_step": 1e3 * t_fwd_keep / K,
                              "note": "every state kept by the forward pass; the backward pass is the adjoint solves alone"},
        "gradients_equal_with_and_without_recompute": same,
        "loss": float(loss.detach()), "dL_dE_norm": float(E.grad.norm()), "dL_dmu": float(mu.grad[0]),
        "spmv_lanes_per_row": lanes, "pcg_coarse": sim.pcg_coarse,
    }
    print(json.dumps(line))


def bench_arm(args):
    """The squeeze on the joint-space arm (joint springs, only the top link
    anchored) against the same squeeze on link-space target drives: steps
    [warmup, warmup + steps) of each, timed alike."""
    import numpy as np
    import torch
    import ipcscenes
    from paper_2609_25653_amd import Sim
    n_total = args.warmup + args.steps
    out = {}
    for name, sc in (("arm", ipcscenes.arm_squeeze(n_steps=n_total)),
                     ("fk_targets", ipcscenes.gripper_squeeze(n_steps=n_total))):
        sim = Sim(sc)
        for _ in range(args.warmup):
            sim.step(allow_status=(3,))
        lanes, _ = sim.autotune(10)
        torch.cuda.synchronize()
        newton, pcg, not_ok = [], [], 0
        t0 = time.perf_counter()
        for _ in range(args.steps):
            rc, st = sim.step(allow_status=(3,))
            not_ok += st[0]["status"] != 0
            newton.append(st[0]["newton_iters"])
            pcg.append(st[0]["pcg_iters_total"])
            print(f"# {name} step {sim.step_index}: rc={rc} newton={newton[-1]} pcg={pcg[-1]} "
                  f"pairs={st[0]['n_pt_max'] + st[0]['n_ee_max']}", file=sys.stderr, flush=True)
        torch.cuda.synchronize()
        t = time.perf_counter() - t0
        out[name] = dict(t=t, newton=newton, pcg=pcg, not_ok=not_ok, lanes=lanes, coarse=sim.pcg_coarse, tets=len(sc["tets"]),
                         bodies=len(sc["body_q"]), joint_springs=len(sc["joint_spring"]), drive_slots=len(sc["driven_body"]))
        del sim
    a, f = out["arm"], out["fk_targets"]
    line = {
        "metric": "Newton iterations/s", "value": sum(a["newton"]) / a["t"], "unit": "Newton it/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": 1e3 * a["t"] / args.steps, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"squeeze on the joint-space arm, steps {args.warmup}-{n_total - 1}", "tets": a["tets"],
                   "bodies": a["bodies"], "joint_springs": a["joint_springs"], "drive_slots": a["drive_slots"],
                   "parallelism": "single GPU"},
        "steps_per_s": args.steps / a["t"], "newton_per_step": a["newton"], "pcg_per_step": a["pcg"],
        "steps_not_converged": a["not_ok"], "spmv_lanes_per_row": a["lanes"], "pcg_coarse": a["coarse"],
        "fk_targets": {"workload": "the same squeeze on link-space target drives", "tets": f["tets"],
                       "newton_it_per_s": sum(f["newton"]) / f["t"], "steps_per_s": args.steps / f["t"],
                       "ms_per_step": 1e3 * f["t"] / args.steps, "newton_per_step": f["newton"],
                       "pcg_per_step": f["pcg"], "steps_not_converged": f["not_ok"], "pcg_coarse": f["coarse"]},
    }
    print(json.dumps(line))


DM_TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_dm_apply_cylinder_L3_traffic.json")
DM_SRC = os.path.join(ROOT, "paper_2609_25653_amd", "csrc", "ipc_dualmesh.hip")


def bench_dualmesh(args):
    """Dual-mesh mapping (Eq. (7)): the soft cylinder's surface (6602 coarse
    vertices) subdivided 3 levels (422402 fine vertices), 100 frames of a
    deformation trajectory per launch; a step is one launch."""
    import hashlib
    import numpy as np
    import torch
    import ipcscenes
    from paper_2609_25653_amd.dualmesh import DualMesh
    tri, frames = ipcscenes.dualmesh_frames(n_frames=args.frames)
    dm = DualMesh(tri, frames.shape[1], 3)
    xc = torch.as_tensor(frames, device="cuda")
    xf = torch.empty((frames.shape[0], dm.n_fine, 3), dtype=torch.float64, device="cuda")
    if args.traffic_run:
        src = torch.ones(32 << 20, dtype=torch.float64, device="cuda")   # 256 MiB
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
        for k in range(args.warmup + args.steps):
            dm.apply(xc, xf)
            print(f"# traffic run launch {k}", file=sys.stderr, flush=True)
        torch.cuda.synchronize()
        return
    for _ in range(args.warmup):
        dm.apply(xc, xf)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        dm.apply(xc, xf)
    torch.cuda.synchronize()
    t = time.perf_counter() - t0
    us, by = dm.time(xc, xf, 50)
    achieved = by / (us * 1e-6) / 1e9
    traffic = None
    try:
        rec = json.load(open(DM_TRAFFIC_FILE))
        if rec.get("source_sha256") == hashlib.sha256(open(DM_SRC, "rb").read()).hexdigest():
            traffic = rec.get("bytes_per_launch")
    except (OSError, ValueError):
        pass
    roof = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
            "traffic": traffic, "kernel": "k_dm_apply (W X^c for every frame)", "bytes_per_launch": by, "avg_us": us,
            "launches_timed": 50}
    per_launch = frames.shape[0] * dm.n_fine
    line = {
        "metric": "fine vertex-frames/s", "value": args.steps * per_launch / t, "unit": "fine vertex-frames/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": 1e3 * t / args.steps, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"dual-mesh mapping: cylinder surface {dm.n_coarse} -> {dm.n_fine} vertices (3 Loop levels), "
                               f"{frames.shape[0]} frames per launch", "nnz_W": dm.nnz, "max_row": dm.max_row,
                   "parallelism": "single GPU"},
        "roofline": roof,
    }
    if not args.no_cpu_baseline:
        from oracle.loop_subdiv import loop_subdivide
        t0 = time.perf_counter()
        for f in (0, frames.shape[0] - 1):
            loop_subdivide(frames[f], tri, 3)
        tc = time.perf_counter() - t0
        line["cpu_baseline"] = {"value": 2 * dm.n_fine / tc, "unit": "fine vertex-frames/s", "cores": 1, "kind": "oracle",
                                "sample": f"2 of the {frames.shape[0]} frames, level-by-level subdivision in Python ({tc:.1f} s)"}
    print(json.dumps(line))


def write_dm_traffic(fetch_csv, write_csv):
    """As write_traffic, for the dual-mesh kernel of a --workload dualmesh
    --traffic-run."""
    import csv
    import hashlib

    def per_kernel(path):
        out = {}
        for r in csv.DictReader(open(path)):
            out.setdefault(r["Kernel_Name"], []).append(float(r["Counter_Value"]))
        return out

    f, w = per_kernel(fetch_csv), per_kernel(write_csv)
    copy = [k for k in f if "copyBuffer" in k]
    dmk = [k for k in f if "k_dm_apply" in k]
    kib = 256 * 1024
    fac_f = kib / max(max(f[k]) for k in copy)
    fac_w = kib / max(max(w[k]) for k in copy)
    sf = [v for k in dmk for v in f[k]]
    sw = [v for k in dmk for v in w[k]]
    traffic = 1024.0 * (fac_f * sum(sf) / len(sf) + fac_w * sum(sw) / len(sw))
    rec = {"kernel": "k_dm_apply", "bytes_per_launch": traffic, "fetch_kib": sum(sf) / len(sf), "write_kib": sum(sw) / len(sw),
           "fetch_scale": fac_f, "write_scale": fac_w, "launches": len(sf),
           "source_sha256": hashlib.sha256(open(DM_SRC, "rb").read()).hexdigest(),
           "source": "python bench.py --workload dualmesh --traffic-run under rocprofv3 --pmc"}
    json.dump(rec, open(DM_TRAFFIC_FILE, "w"), indent=1)
    print(json.dumps(rec))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None,
                    help="timed steps (default: contact and batched 99, arm 160, dualmesh 200 launches, oracle 5)")
    ap.add_argument("--warmup", type=int, default=None,
                    help="untimed warm-up steps (default: contact and batched 1, arm 40, dualmesh 10)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--s-g", type=float, default=8e-4, help="ground patch spacing (m): 0.8 mm keeps the median active pairs inside 50k-300k")
    ap.add_argument("--workload", choices=["contact", "batched", "adjoint", "arm", "dualmesh", "oracle"], default="contact",
                    help="contact: the 200k-tet squeeze (default line); batched: 256 uneven squeeze scenes stepped "
                         "together vs one at a time; adjoint: 50-step squeeze rollout, forward vs backward time; "
                         "arm: the squeeze on the joint-space arm vs on link-space target drives; "
                         "dualmesh: the render mesh of the soft cylinder, 3 Loop levels, 100 frames per launch; "
                         "oracle: the first --steps steps of the 200k-tet squeeze on the CPU oracle alone (no GPU)")
    ap.add_argument("--frames", type=int, default=100, help="dualmesh: frames per launch")
    ap.add_argument("--scenes", type=int, default=256, help="batched: number of scenes")
    ap.add_argument("--single-sample", type=int, default=16, help="batched: scenes stepped one at a time for the baseline")
    ap.add_argument("--traffic-from", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"), default=None,
                    help="write the product's calibrated per-launch HBM traffic from the counter files of two "
                         "'rocprofv3 --pmc FETCH_SIZE' / '--pmc WRITE_SIZE' runs of --traffic-run, then exit")
    ap.add_argument("--traffic-run", action="store_true",
                    help="for hardware-counter runs: a plain 256 MiB device copy (the counters' calibration), then "
                         "the contact workload with --warmup and --steps and no line")
    ap.add_argument("--probe", choices=["spmv"], default=None,
                    help="spmv: assemble the Hessian of the 200k-tet scene once, then run a plain 256 MiB device copy "
                         "and 20 back-to-back block-CSR products (for hardware-counter runs)")
    args = ap.parse_args()
    # the contact default times steps 2-100 of the 100-step scene: the squeeze
    # and the lift; the first step (the most pairs) warms up
    steps_default = {"contact": 99, "batched": 99, "arm": 160, "dualmesh": 200, "oracle": 5, "adjoint": 50}
    warmup_default = {"contact": 1, "batched": 1, "arm": 40, "dualmesh": 10, "oracle": 0, "adjoint": 40}
    if args.steps is None:
        args.steps = 4 if (args.traffic_run or args.probe) else steps_default[args.workload]
    if args.warmup is None:
        args.warmup = 1 if (args.traffic_run or args.probe) else warmup_default[args.workload]
    if args.traffic_from:
        if args.workload == "dualmesh":
            return write_dm_traffic(*args.traffic_from)
        return write_traffic(*args.traffic_from)
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported", file=sys.stderr)
        sys.exit(2)
    if args.workload == "oracle":
        return bench_oracle(args)
    import numpy as np
    import torch

    import ipcscenes
    from paper_2609_25653_amd import Sim, lib

    if args.workload == "batched":
        return bench_batched(args)
    if args.workload == "adjoint":
        return bench_adjoint(args)
    if args.workload == "arm":
        return bench_arm(args)
    if args.workload == "dualmesh":
        return bench_dualmesh(args)
    n_total = args.warmup + args.steps
    scene = ipcscenes.contact_rich(n_steps=n_total, s_g=args.s_g)
    sim = Sim(scene)
    if args.probe == "spmv":
        return probe_spmv(sim)
    if args.traffic_run:
        src = torch.ones(32 << 20, dtype=torch.float64, device="cuda")   # 256 MiB
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
        for k in range(args.warmup + args.steps):
            rc, st = sim.step(allow_status=(3,))
            print(f"# traffic run step {k}: rc={rc} newton={st[0]['newton_iters']}", file=sys.stderr, flush=True)
        torch.cuda.synchronize()
        return
    for _ in range(args.warmup):
        sim.step(allow_status=(3,))
    # autotune the product's lanes per row on the last warm-up matrix
    lanes, tune_us = sim.autotune(20)
    print(f"# autotune: {lanes} lanes per row; us per product {tune_us}", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    newton = pcg = 0
    pairs = []
    status = {}
    t0 = time.perf_counter()
    for k in range(args.steps):
        if k == args.steps - 1:
            # the last timed step runs with the library's kernel timing on:
            # every product launch inside PCG stamps HIP events at its own
            # start and end (eager launches for this step only)
            sim._check(lib().ipc_profile(sim._h, 1))
        rc, st = sim.step(allow_status=(3, 4))
        status[st[0]["status"]] = status.get(st[0]["status"], 0) + 1
        newton += st[0]["newton_iters"]
        pcg += st[0]["pcg_iters_total"]
        pairs.append(st[0]["n_pt_max"] + st[0]["n_ee_max"])
        nloc = sim._query(7)
        print(f"# step {sim.step_index}: rc={rc} newton={st[0]['newton_iters']} pcg={st[0]['pcg_iters_total']} "
              f"pairs={pairs[-1]} pair_local={nloc} cand_max={st[0]['n_cand_max']} alpha_min={st[0]['alpha_min']:.3g}", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t = time.perf_counter() - t0
    # Dominant kernel: the Hessian product inside PCG (see product_roofline).
    roof = product_roofline(sim, lib, product_traffic())
    line = {
        "metric": METRIC, "value": newton / t, "unit": "Newton iters/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": 1e3 * t / args.steps, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "contact-rich squeeze: 2 pads + soft cylinder on a ground patch",
                   "tets": int(len(scene["tets"])), "vertices": int(len(scene["X"])), "dhat": float(scene["dhat"]),
                   "dt": float(scene["h"]), "ground_spacing": args.s_g, "parallelism": "single GPU"},
        "steps_per_s": args.steps / t,
        "newton_per_step": newton / args.steps,
        "pcg_per_newton": pcg / max(newton, 1),
        "active_pairs": {"min": int(min(pairs)), "median": float(np.median(pairs)), "max": int(max(pairs))},
        "steps_by_status": {str(k): v for k, v in sorted(status.items())},
        "roofline": roof,
        "spmv_lanes_per_row": lanes, "fem_blocks": list(sim.fem_blocks), "pcg_coarse": sim.pcg_coarse,
    }
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(scene)
    print(json.dumps(line))


if __name__ == "__main__":
    main()
