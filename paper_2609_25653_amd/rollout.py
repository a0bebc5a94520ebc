"""Differentiable rollouts: ``IPCRollout``, a torch.autograd.Function over K steps.

Forward runs the library's steps from (y0, ydot0) with parameters (E per tet,
mu per scene) and keeps (y, ydot) every ``checkpoint_every`` steps, plus the
observed DOFs of every step when ``observe`` is given (e.g. the tracked
vertices of a loss summed over the trajectory).  Backward walks the
checkpoint segments in reverse: it recomputes a segment's states from its
checkpoint, then calls the library's one-step adjoint for each step of the
segment, newest first, adding the observed DOFs' upstream gradients as it
passes their step, accumulating dL/dE and dL/dmu and carrying the state
adjoints (ybar, vbar) back to the start.  Memory: one (y, ydot) pair per
checkpoint, the states of one segment and the observed trajectory.  With
``checkpoint_every=0`` the forward pass keeps every state instead and the
backward pass recomputes nothing (memory: one (y, ydot) pair per step).
"""
import torch


class IPCRollout(torch.autograd.Function):
    """(E, mu, y0, ydot0) -> (y_K, ydot_K, Y_obs) over steps first_step .. first_step+K-1.

    ``sim`` is a ``Sim`` over the scene(s); E has one entry per tet of all
    scenes, mu one per scene.  ``observe`` (a long tensor of DOF indices, or
    None) selects the DOFs recorded after every step: Y_obs[k] = y_{k+1}[observe]
    (an empty tensor when None).  The Newton and adjoint solves use the scenes'
    own tolerances; ``eta`` is the adjoint PCG's relative residual."""

    @staticmethod
    def forward(ctx, E, mu, y0, ydot0, sim, first_step, n_steps, checkpoint_every, eta, observe):
        E = E.detach().contiguous()
        mu = mu.detach().contiguous()
        sim.set_params(E, mu.cpu().numpy())
        y, v = y0.detach().contiguous().clone(), ydot0.detach().contiguous().clone()
        sim.set_state(y, v)
        ckpts, obs = [], []
        keep_all = checkpoint_every == 0
        if keep_all:
            ckpts.append((0, [(y, v)]))
        for k in range(n_steps):
            if not keep_all and k % checkpoint_every == 0:
                ckpts.append((k, y, v))
            sim.step(first_step + k)
            y, v = sim.state()
            if keep_all:
                ckpts[0][1].append((y, v))
            if observe is not None:
                obs.append(y[observe])
        ctx.sim, ctx.first, ctx.n, ctx.every, ctx.eta, ctx.observe = sim, first_step, n_steps, checkpoint_every, eta, observe
        ctx.ckpts = ckpts
        ctx.save_for_backward(E, mu)
        Y = torch.stack(obs) if obs else torch.zeros(0, dtype=torch.float64, device=y.device)
        return y, v, Y

    @staticmethod
    def backward(ctx, ybar, vbar, gobs):
        sim = ctx.sim
        E, mu = ctx.saved_tensors
        sim.set_params(E, mu.cpu().numpy())
        zeros = lambda: torch.zeros(sim.ndof, dtype=torch.float64, device=sim.device)
        ybar = zeros() if ybar is None else ybar.contiguous().clone()
        vbar = zeros() if vbar is None else vbar.contiguous().clone()
        Ebar = torch.zeros(sim.n_tets, dtype=torch.float64, device=sim.device)
        mubar = torch.zeros(sim.n_scenes, dtype=torch.float64, device=sim.device)
        segments = ctx.ckpts if ctx.every == 0 else [(c0, (y, v)) for c0, y, v in ctx.ckpts]
        for c0, first_state in reversed(segments):
            if ctx.every == 0:   # every state kept by the forward pass
                states, c1 = first_state, ctx.n
            else:
                c1 = min(c0 + ctx.every, ctx.n)
                states = [first_state]
                sim.set_state(*first_state)
                for k in range(c0, c1):
                    sim.step(ctx.first + k)
                    states.append(sim.state())
            for k in range(c1 - 1, c0 - 1, -1):
                if ctx.observe is not None and gobs is not None and gobs.numel():
                    ybar = ybar.index_add(0, ctx.observe, gobs[k])
                yp, vp = states[k - c0]
                yn = states[k - c0 + 1][0]
                ybar, vbar, _ = sim.step_vjp(yp, vp, ctx.first + k, yn, ybar, vbar, Ebar, mubar, ctx.eta)
        # the context's state is left at the start of the rollout
        return Ebar, mubar.to(mu.dtype).reshape(mu.shape), ybar, vbar, None, None, None, None, None, None


def rollout(sim, E, mu, y0, ydot0, first_step, n_steps, checkpoint_every=10, eta=1e-12, observe=None):
    """Differentiable rollout; returns (y_K, ydot_K), or (y_K, ydot_K, Y_obs)
    with Y_obs[k] = y_{k+1}[observe] when ``observe`` is given.  checkpoint_every
    = 0 keeps every state (no recompute in the backward pass).  See ``IPCRollout``."""
    mu = torch.as_tensor(mu, dtype=torch.float64, device=sim.device).reshape(-1)
    if mu.numel() == 1 and sim.n_scenes > 1:
        mu = mu.expand(sim.n_scenes).contiguous()
    if observe is not None:
        observe = torch.as_tensor(observe, device=sim.device).long()
    y, v, Y = IPCRollout.apply(E, mu, y0, ydot0, sim, first_step, n_steps, checkpoint_every, eta, observe)
    return (y, v) if observe is None else (y, v, Y)
