"""Joint-space drives (the E_joint term of Eq. (3) as joint springs): pins of
the oracle.  CPU only.

Every body-to-body spring of the arm scene maps a point of one body's frame
to a point of the other's.  With this step's joint points the pairs of each
link must be related by one rigid motion (a wrong rotation axis, sense or
pivot would not be), and composing those motions outward from the anchored
link gives the forward kinematics of the joint references: there every
spring has zero length, so the oracle's spring energy vanishes.  A joint
point moved off its reference leaves a stretched spring."""
import numpy as np
import pytest

import ipcscenes as S
import oracle as O


def rigid_fit(P, Q):
    """R, t minimising |R P_i + t - Q_i| (least squares, proper rotation)."""
    cp, cq = P.mean(0), Q.mean(0)
    U, _, Vt = np.linalg.svd((P - cp).T @ (Q - cq))
    D = np.diag([1.0, 1.0, np.sign(np.linalg.det(Vt.T @ U.T))])
    R = Vt.T @ D @ U.T
    return R, cq - R @ cp


def fk_state(sc, n):
    """Body states (p, A) and FEM positions at the joint references of step n."""
    xb = sc["sp_xb"].copy()
    xb[sc["joint_spring"]] = sc["joint_xbar"][n]
    ka, kb, ia, ib, xa = sc["sp_ka"], sc["sp_kb"], sc["sp_ia"], sc["sp_ib"], sc["sp_xa"]
    nb = len(sc["body_q"])
    p = sc["body_q"][:, :3].copy()
    A = np.tile(np.eye(3), (nb, 1, 1))
    known = np.zeros(nb, bool)
    for s in np.nonzero(kb == 2)[0]:            # the anchored link keeps its rest pose
        known[ia[s]] = True
    edges = {}
    for s in np.nonzero((ka == 1) & (kb == 1))[0]:
        edges.setdefault((ia[s], ib[s]), []).append((xa[s], xb[s]))
    residual = 0.0
    grew = True
    while grew:
        grew = False
        for (a, b), pairs in edges.items():
            Pa = np.array([u for u, _ in pairs]); Pb = np.array([v for _, v in pairs])
            if known[b] and not known[a]:      # a-frame point -> b-frame point
                R, t = rigid_fit(Pa, Pb)
                residual = max(residual, np.abs(Pa @ R.T + t - Pb).max())
                A[a] = A[b] @ R; p[a] = p[b] + A[b] @ t; known[a] = True; grew = True
            elif known[a] and not known[b]:
                R, t = rigid_fit(Pb, Pa)
                residual = max(residual, np.abs(Pb @ R.T + t - Pa).max())
                A[b] = A[a] @ R; p[b] = p[a] + A[a] @ t; known[b] = True; grew = True
    X = sc["X"].copy()
    for s in np.nonzero((ka == 0) & (kb == 1))[0]:   # stitched FEM vertices ride on their body
        X[ia[s]] = p[ib[s]] + A[ib[s]] @ xb[s]
    y = np.concatenate([X.ravel()] + [np.concatenate([p[b], A[b].T.ravel()]) for b in range(nb)])
    return y, residual, known


@pytest.mark.parametrize("n", [0, 7, 63, 119])
def test_joint_springs_vanish_at_the_joint_reference(n):
    sc = S.tiny_scene("arm_box", h=0.005, n_steps=120)
    y, residual, known = fk_state(sc, n)
    assert residual < 1e-15                          # each link's pairs: one rigid motion
    assert known.sum() == len(known) - 1             # all bodies but the free box are linked
    o = O.Oracle(sc)
    o.set_state(y, np.zeros_like(y))
    o.begin_step(n)
    _, terms = o.energy(y)
    assert terms[3] < 1e-22, terms[3]                # spring term of the incremental potential
    # the same state against a joint point moved off its reference by 10 um
    sc2 = dict(sc)
    sc2["joint_xbar"] = sc["joint_xbar"].copy()
    sc2["joint_xbar"][n, 0, 2] += 1e-5
    o2 = O.Oracle(sc2)
    o2.set_state(y, np.zeros_like(y))
    o2.begin_step(n)
    _, terms2 = o2.energy(y)
    k = sc["sp_k"][sc["joint_spring"][0]]
    assert terms2[3] == pytest.approx(0.5 * k * 1e-10 * float(sc["h"]) ** 2, rel=1e-6)


def _arm_without_perturbation(n_steps, h):
    from ipcscenes import scenes as SS
    b = SS._Builder()
    b.add_body((0.3, 0.3, 0.01 + 5e-4), (0.02, 0.02, 0.02), 0.05, contact=True)
    drive, _, _ = SS._add_arm_gripper(b, np.random.default_rng(0), center_xy=(0.3, 0.3), z_mid=0.01 + 5e-4,
                                      inner_half_gap=0.0115, pad_cells=(4, 2, 2), pad_E=1e5, pad_nu=0.45,
                                      n_steps=n_steps, h=h, t_close=0.5, v_close=0.01, v_lift=0.02, pert=False)
    b.add_static(*SS.ground_quad())
    return b.finish(SS._params(h=h, n_steps=n_steps), drive)


def test_lift_raises_the_hand_without_turning_it():
    """The lift bends joints 2, 4, 6 by phi, -2 phi, phi: at the joint
    references (no yaw perturbation) the hand is higher by the prescribed
    lift and keeps its orientation."""
    sc = _arm_without_perturbation(240, 0.005)
    y0, _, _ = fk_state(sc, 0)
    y1, _, _ = fk_state(sc, 239)
    nv = len(sc["X"])
    hand = 5                                          # box, 2 x (base, finger), hand, then the chain
    q0 = y0[3 * nv + 12 * hand: 3 * nv + 12 * hand + 12]
    q1 = y1[3 * nv + 12 * hand: 3 * nv + 12 * hand + 12]
    lift = 0.02 * (240 * 0.005 - 0.5)
    assert q1[2] - q0[2] == pytest.approx(lift, abs=1e-12)
    A1 = q1[3:].reshape(3, 3).T
    assert np.abs(A1 - np.eye(3)).max() < 1e-12


def _hanging_arm(n_steps):
    """The arm with its pads hanging in the air: static joint references
    (no closing, no lift, no perturbation), gravity only."""
    from ipcscenes import scenes as SS
    b = SS._Builder()
    drive, _, _ = SS._add_arm_gripper(b, np.random.default_rng(0), center_xy=(0.3, 0.3), z_mid=0.0105,
                                      inner_half_gap=0.0115, pad_cells=(4, 2, 2), pad_E=1e5, pad_nu=0.45,
                                      n_steps=n_steps, h=0.01, t_close=0.5, v_close=0.0, v_lift=0.0, pert=False)
    return b.finish(SS._params(h=0.01, n_steps=n_steps), drive)


def test_hanging_arm_carries_its_weight_joint_by_joint():
    """Implicit Euler from rest under constant loads settles at the static
    equilibrium of Eq. (1), where inertia vanishes and every subtree of the
    arm is in force balance: the springs joining it to its parent (joint
    springs, axis springs, finger mounts, pad stitches) pull it up by exactly
    its weight, and the anchor springs carry the whole arm.  The anchor's
    spring points have zero first moment, so the anchored link drops by
    W / (4 k) and does not move sideways.  A wrong sign or side in a spring
    gradient, a misplaced joint point or a wrong mass breaks a balance."""
    n_steps = 30
    sc = _hanging_arm(n_steps)
    X, T, nv, nb = sc["X"], sc["tets"], len(sc["X"]), len(sc["body_q"])
    g = np.asarray(sc["g"], float)
    o = O.Oracle(sc)
    for _ in range(n_steps):
        rc, _ = o.step()
        assert rc == 0
    y, v = o.state()
    assert np.abs(v).max() < 1e-9                    # settled
    Q = y[3 * nv:].reshape(nb, 12)
    xb = sc["sp_xb"].copy()
    xb[sc["joint_spring"]] = sc["joint_xbar"][n_steps - 1]
    tgt = sc["drive_q"][n_steps - 1]

    def node(kind, i):
        return ("b", int(i)) if kind == 1 else ("o", int(sc["vobj"][i])) if kind == 0 else ("w", 0)

    def point(kind, i, xbar):
        if kind == 0:
            return y[3 * i: 3 * i + 3]
        q = Q[i] if kind == 1 else tgt[i]
        return q[:3] + q[3:].reshape(3, 3).T @ xbar

    vol = np.abs(np.einsum("ij,ij->i", np.cross(X[T[:, 1]] - X[T[:, 0]], X[T[:, 2]] - X[T[:, 0]]),
                           X[T[:, 3]] - X[T[:, 0]])) / 6.0
    mass = {("b", b): sc["body_mass"][b] for b in range(nb)}
    for t in range(len(T)):
        key = ("o", int(sc["vobj"][T[t, 0]]))
        mass[key] = mass.get(key, 0.0) + vol[t] * sc["tet_rho"][t]
    # spring groups: unordered pairs of objects, with the force each spring puts on its a side
    groups = {}
    for s in range(len(sc["sp_k"])):
        a, b = node(sc["sp_ka"][s], sc["sp_ia"][s]), node(sc["sp_kb"][s], sc["sp_ib"][s])
        d = point(sc["sp_ka"][s], sc["sp_ia"][s], sc["sp_xa"][s]) - point(sc["sp_kb"][s], sc["sp_ib"][s], xb[s])
        groups.setdefault(frozenset((a, b)), []).append((a, -sc["sp_k"][s] * d))
    adj = {}
    for e in groups:
        u, w = tuple(e)
        adj.setdefault(u, set()).add(w); adj.setdefault(w, set()).add(u)
    assert set(adj) == set(mass) | {("w", 0)}
    assert sum(len(n) for n in adj.values()) == 2 * len(mass)      # a tree rooted at the world

    def subtree(child, parent):
        seen, todo = {child}, [child]
        while todo:
            for w in adj[todo.pop()] - {parent}:
                if w not in seen:
                    seen.add(w); todo.append(w)
        return seen

    order, parent_of, todo = [], {("w", 0): None}, [("w", 0)]
    while todo:
        u = todo.pop(); order.append(u)
        for w in adj[u]:
            if w not in parent_of:
                parent_of[w] = u; todo.append(w)
    W_all = -sum(mass.values()) * g
    for child in order[1:]:
        par = parent_of[child]
        f = sum(fa if a == child else -fa for a, fa in groups[frozenset((child, par))])
        W_sub = -sum(mass[k] for k in subtree(child, par)) * g
        assert np.abs(f - W_sub).max() < 1e-5 * np.abs(W_all).max(), (child, f, W_sub)
    top = sc["driven_body"][0]
    k = sc["sp_k"][sc["sp_kb"] == 2]
    assert np.all(k == k[0]) and len(k) == 4
    drop = W_all / (4 * k[0])
    assert np.abs((Q[top, :3] - sc["body_q"][top, :3]) + drop).max() < 1e-5 * np.abs(drop).max()
