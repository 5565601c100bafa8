"""Differentiable rollout: theta^N = S_{N-1} o ... o S_0 (theta^0; P(U, V, W)).

``ScalarRollout`` is a torch.autograd.Function whose forward refines the
coarse velocity once (it is frozen over the rollout), runs N scalar steps on a
ring of three buffers as one step sequence, and keeps the pair
(theta^{n-1}, theta^n) every K steps and every state of the last segment; each
kept state is written straight into a buffer of its own, so nothing is
copied.  Its backward walks the checkpoint segments in reverse: it recomputes
the states of each segment but the last from its checkpoint (one step
sequence each), runs the fused reverse step of each
step (transposed implicit solve fused with the transposed stencils), adds the
segment's dense face-velocity gradient from the stored (theta^n, mu^n)
pairs (one library call per group of at most 16 steps), and finally maps the dense face gradient to the coarse faces with the
transposed refinement.  Every step of the computation is a library call.
"""
import torch

MAX_GRAD_STEPS = 16


class ScalarRollout(torch.autograd.Function):

    @staticmethod
    def forward(fctx, mr, nsteps, ckpt_every, theta0, U, V, W):
        if nsteps < 1:
            raise ValueError("nsteps must be >= 1")
        if int(ckpt_every) != ckpt_every or ckpt_every < 1:
            raise ValueError("ckpt_every must be a positive integer, got %r" % (ckpt_every,))
        K = int(ckpt_every)
        u, v, w = mr.interpolate_velocity(U.detach(), V.detach(), W.detach())
        last = ((nsteps - 1) // K) * K          # first step of the last segment
        th0 = theta0.detach().clone()
        # theta^m that the backward reads (the checkpoint pairs (theta^{s-1},
        # theta^s) and every state of the last segment) is written straight
        # into a buffer of its own; the others rotate through three buffers
        pool = [mr.empty(mr.shape_cell) for _ in range(3)]
        prev = cur = th0
        ckpts = {0: (None, th0)}
        tail = {0: th0} if last == 0 else {}
        outs = []
        for n in range(nsteps):
            m = n + 1
            if m % K == 0 or (m + 1) % K == 0 or last <= m < nsteps:
                out = mr.empty(mr.shape_cell)
            else:
                out = next(b for b in pool if b is not prev and b is not cur)
            outs.append(out)
            prev, cur = cur, out
            if m < nsteps and m % K == 0:
                ckpts[m] = (prev, cur)
            if last <= m < nsteps:
                tail[m] = cur
        # the whole rollout is one step sequence (column sweeps where the
        # library prefers them); every output differs from the two levels
        # before it
        mr.scalar_steps(0, None, th0, outs, u, v, w)
        fctx.mr = mr
        fctx.nsteps = nsteps
        fctx.K = K
        fctx.ckpts = ckpts
        fctx.tail = tail
        fctx.uvw = (u, v, w)
        return cur.clone()

    @staticmethod
    def backward(fctx, g_out):
        mr, N, K = fctx.mr, fctx.nsteps, fctx.K
        u, v, w = fctx.uvw
        g_out = g_out.contiguous()
        gu = torch.zeros_like(u)
        gv = torch.zeros_like(v)
        gw = torch.zeros_like(w)
        mu_next = None
        mu_cur = mr.empty(mr.shape_cell)
        mr.adjoint_seed(N - 1, g_out, mu_cur)
        g_theta0 = None
        for s in reversed(range(0, N, K)):
            e = min(s + K, N)
            if s == (N - 1) // K * K:
                # the last segment's states were kept by the forward pass
                states = fctx.tail
                fctx.tail = None
            else:
                # recompute theta^s .. theta^{e-1} from the checkpoint
                pprev, pcur = fctx.ckpts[s]
                states = {s: pcur}
                outs = [mr.empty(mr.shape_cell) for _ in range(s, e - 1)]
                if outs:
                    mr.scalar_steps(s, pprev, pcur, outs, u, v, w)
                for n, out in zip(range(s, e - 1), outs):
                    states[n + 1] = out
            # reverse steps e-1 .. max(s, 1) as one sequence (mu^n kept for the
            # velocity gradient), then the start-up step's reverse on its own
            mus = {e - 1: mu_cur}
            lo = max(s, 1)
            if e - 1 >= lo:
                outs = [mr.empty(mr.shape_cell) for _ in range(e - lo)]
                mr.scalar_steps_backward(e - 1, mu_next, mu_cur, outs, u, v, w)
                for q, out in enumerate(outs):
                    mus[e - 2 - q] = out
                mu_next = outs[-2] if len(outs) > 1 else mu_cur
                mu_cur = outs[-1]
            if s == 0:
                out = mr.empty(mr.shape_cell)
                mr.scalar_step_backward(0, mu_next, mu_cur, None, out, u, v, w)
                g_theta0 = out
                mu_next, mu_cur = mu_cur, out
            mus = {n: m for n, m in mus.items() if s <= n < e}
            # one velocity-gradient call per group of at most MAX_GRAD_STEPS steps
            for g0 in range(s, e, MAX_GRAD_STEPS):
                idx = list(range(g0, min(g0 + MAX_GRAD_STEPS, e)))
                mr.velocity_grad(idx, [states[n] for n in idx], [mus[n] for n in idx], gu, gv, gw)
            del states, mus
        gU, gV, gW = mr.interpolate_velocity_backward(gu, gv, gw)
        return None, None, None, g_theta0, gU, gV, gW


def rollout(mr, theta0, U, V, W, nsteps, ckpt_every=10):
    """theta^nsteps as a differentiable function of (theta0, U, V, W)."""
    return ScalarRollout.apply(mr, nsteps, ckpt_every, theta0, U, V, W)
