"""Oracle references for the GPU parity tests at the benchmark configurations
(tests/test_gpu_configs.py).  Calls only oracle/ and the seeded scene
generators: every stored value is the oracle's.  Run from the repository root:

    OMP_NUM_THREADS=8 python tests/golden/make_config_refs.py [squeeze|contact|batched|adjoint ...]

Windows (the oracle takes minutes per step at 200k tets and seconds at 20k):
  squeeze  the 20k-tet gripper squeeze (200 steps): states after steps 1-6
           from the initial state, and the state after step 96 with those
           after steps 97-102 (closing turns into lifting at step 100);
  contact  the 200k-tet contact-rich scene: the state after step 0, the first
           Newton direction of step 0 solved to a relative residual of 1e-10,
           and the CCD bound of that direction;
  contact_ccd  CCD bounds at the initial state of that direction scaled by
           30, 300 and 3000 (steps that collide);
  batched  4 scenes of the 256-scene batch (the smallest, the scenes at the
           size tertiles and scene 255): the state after step 36 and those
           after steps 37-40;
  adjoint  the differentiation workload over steps 40-49: the state after
           step 40, targets (tracked vertices after step 49 under E exp(0.2 Z),
           mu x 1.1), and the loss and its gradient (E per tet, mu) at the
           nominal parameters.
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)
import ipcscenes  # noqa: E402
import oracle as O  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "config_refs")
BATCHED_PICK_RULE = "smallest, size tertiles, scene 255"


def log(*a):
    print(*a, flush=True)


def run(o, n0, n1, keep):
    """Steps n0 .. n1 - 1; keeps (y, v) after every step in keep."""
    out = {}
    t0 = time.time()
    for k in range(n0, n1):
        o.step_index = k
        rc, st = o.step()
        if rc != 0:
            raise RuntimeError(f"oracle step {k} returned {rc}")
        if k + 1 in keep:
            out[k + 1] = o.state()
        log(f"  step {k}: newton {st['newton_iters']} pcg {st['pcg_iters_total']} "
            f"pairs {st['n_pt_max'] + st['n_ee_max']} ({time.time() - t0:.0f} s)")
    return out


def squeeze():
    sc = ipcscenes.gripper_squeeze(n_steps=200)
    o = O.Oracle(sc)
    st = run(o, 0, 102, set(range(1, 7)) | set(range(96, 103)))
    for k, (y, v) in st.items():
        np.save(os.path.join(OUT, f"squeeze_y{k}.npy"), y)
        if k == 96:                    # the velocity only where a window starts
            np.save(os.path.join(OUT, f"squeeze_v{k}.npy"), v)


def contact():
    sc = ipcscenes.contact_rich(n_steps=100)
    o = O.Oracle(sc)
    o.begin_step(0)
    y, _ = o.state()
    g, _ = o.gradient(y)
    p, it = o.pcg(y, -g, 1e-10)
    a = o.ccd(y, p)
    np.save(os.path.join(OUT, "contact_p0.npy"), p)
    np.save(os.path.join(OUT, "contact_alpha0.npy"), np.array([a, float(it)]))
    log(f"  first direction: {it} PCG iterations, CCD bound {a!r}")
    o.set_state(*o.state())
    st = run(o, 0, 1, {1})
    np.save(os.path.join(OUT, "contact_y1.npy"), st[1][0])


def contact_ccd():
    sc = ipcscenes.contact_rich(n_steps=100)
    o = O.Oracle(sc)
    y, _ = o.state()
    p = np.load(os.path.join(OUT, "contact_p0.npy"))
    a = [o.ccd(y, f * p) for f in CCD_SCALES]
    log(f"  CCD bounds {a}")
    np.save(os.path.join(OUT, "contact_ccd_scaled.npy"), np.array(a))


CCD_SCALES = (30.0, 300.0, 3000.0)


def batched_pick():
    scenes = ipcscenes.batched_squeeze(n_scenes=256, n_steps=100)
    tets = np.array([len(s["tets"]) for s in scenes])
    order = np.argsort(tets, kind="stable")
    pick = [int(order[0]), int(order[len(order) // 3]), int(order[2 * len(order) // 3]), 255]
    return scenes, pick


def batched():
    scenes, pick = batched_pick()
    for i in pick:
        log(f" scene {i}: {len(scenes[i]['tets'])} tets")
        o = O.Oracle(scenes[i])
        st = run(o, 0, 40, set(range(36, 41)))
        for k, (y, v) in st.items():
            np.save(os.path.join(OUT, f"batched{i}_y{k}.npy"), y)
            if k == 36:
                np.save(os.path.join(OUT, f"batched{i}_v{k}.npy"), v)


def adjoint():
    sc, info = ipcscenes.adjoint_squeeze(0)
    first, K = info["first_step"], 10
    o = O.Oracle(sc)
    st = run(o, 0, first, {first})
    y0, v0 = st[first]
    np.save(os.path.join(OUT, f"adjoint_y{first}.npy"), y0)
    np.save(os.path.join(OUT, f"adjoint_v{first}.npy"), v0)
    tracked = info["tracked"]
    E0 = np.asarray(sc["tet_E"], np.float64)
    mu0 = float(sc["mu"])
    # targets: the tracked vertices after the window under perturbed parameters
    ot = O.Oracle(sc)
    ot.set_params(E0 * info["target_E_scale"], mu0 * info["target_mu_scale"])
    ot.set_state(y0, v0)
    run(ot, first, first + K, set())
    yt, _ = ot.state()
    target = yt[(3 * tracked[:, None] + np.arange(3)[None, :]).ravel()].reshape(-1, 3)
    np.save(os.path.join(OUT, "adjoint_target.npy"), target)
    t0 = time.time()
    loss, Eb, mb = O.rollout_loss(sc, y0, v0, first, K, tracked, target, E0, mu0, grad=True, checkpoint_every=5, eta=1e-10)
    log(f"  loss {loss!r}, |dL/dE| {np.linalg.norm(Eb):.3g}, dL/dmu {mb!r} ({time.time() - t0:.0f} s)")
    np.save(os.path.join(OUT, "adjoint_grad.npy"), np.concatenate([[loss, mb], Eb]))


if __name__ == "__main__":
    os.makedirs(OUT, exist_ok=True)
    for what in (sys.argv[1:] or ["squeeze", "contact", "batched", "adjoint"]):
        log(f"== {what}")
        globals()[what]()
