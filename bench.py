"""Benchmark of the multiple-resolution dense-grid scalar step on one MI355X.

One benchmark step is one whole run of the FP64 workload
rb1024x1024x512-m2-fp64 (coarse 512x512x256 -> dense 1024x1024x512, tanh z
grid with clustering 2.5, Ra 1e9, Pr 7): refine the coarse velocity, check its
divergence, then 50 scalar steps with the Nusselt profile every 10 steps (the
steps run as one sequence; theta^10 .. theta^40 go to buffers of their own and
the five profiles are taken after it: the velocity is frozen, so nothing in
the steps depends on them).
This is the largest workload that fits one GPU, in the paper's precision.
Inputs are resident in HBM before the timed region.  value = dense-cell
updates per second over the whole job.

Also reported, outside the timed region: the same run with FP32 storage (the
precision tier on the same grid), the 256^3 FP64 and FP32 runs, the adjoint
workloads (256^3 and 1024x1024x512, FP32: forward and backward times), the
inter-grid kernels (integration, Nu_T, refinement in time, one coarse step of
M_t = 4), the step and refinement with side walls in x and y, the step with an
explicit z-diffusion share of 1/2 and with fourth-order face values, the step
kernel on the 576^3 workload in both precisions, the copy-kernel bandwidth,
the roofline of the dominant kernel (the fused scalar step) and the oracle's
CPU time on a bounded sample.

usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]
"""
import argparse
import glob
import hashlib
import json
import os
import re
import sys
import time

import numpy as np
import torch

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

from paper_1805_03426_amd import inputs  # noqa: E402
from paper_1805_03426_amd.configs import WORKLOADS  # noqa: E402

HBM_PEAK_GBS = 8000.0
METRIC = "dense-cell updates/s per scalar step, % HBM peak; FP32 vs FP64; adjoint/fwd"
WORKLOAD = "rb1024x1024x512-m2-fp64"
SMALL_WORKLOAD = "rb256-m2-fp64"
ADJOINT_WORKLOAD = "rb256-m2-adjoint-fp32"
CPU_WORKLOAD = "rb256-m2-fp64"
STEP_KERNELS = {"line": "line_kernel", "sweep": "sweep_kernel (with each range's backsub_kernel)"}
# committed counter summaries of the step kernels, by workload
PROFILE_TRAFFIC = {"rb1024x1024x512-m2-fp64": os.path.join(ROOT, "profiles", "scalar_step_rb1024x1024x512_fp64_traffic.md"),
                   "rb256-m2-fp64": os.path.join(ROOT, "profiles", "scalar_step_rb256_fp64_traffic.md")}

_INPUTS = {}


def workload_inputs(w):
    """Seeded host inputs of a workload, generated once per grid (the FP32 and
    FP64 runs of one grid share them)."""
    key = (w.nc, w.m, w.gamma, w.kmax, w.cfl, w.urms, w.noise)
    if key not in _INPUTS:
        _INPUTS[key] = inputs.workload_inputs(w)
    return _INPUTS[key]


def kernel_source_hash(method="sweep"):
    """Hash of the sources that define the step kernel of a method and its
    launch shape (the kernel code, its launch code and the shared header), to
    tell whether the committed counters of that kernel are stale."""
    names = {"sweep": ("k_sweep.hip", "mr_internal.h"),
             "line": ("line_kernel.h", "k_line_fwd.hip", "k_step.hip", "mr_internal.h", "mr_api.hip")}[method]
    h = hashlib.sha256()
    for name in names:
        h.update(open(os.path.join(ROOT, "paper_1805_03426_amd", "csrc", name), "rb").read())
    return h.hexdigest()[:16]


def committed_traffic(wname, method):
    """Measured HBM bytes per step of the step kernels of a workload from the
    committed rocprofv3 counter summary, or None if absent or taken on other
    sources."""
    path = PROFILE_TRAFFIC.get(wname)
    if path is None or not os.path.exists(path):
        return None
    text = open(path).read()
    m_hash = re.search(r"source hash:\s*([0-9a-f]+)", text)
    m_bytes = re.search(r"bytes per step \(scaled\):\s*([0-9.eE+]+)", text)
    if not m_hash or not m_bytes or m_hash.group(1) != kernel_source_hash(method):
        return None
    return float(m_bytes.group(1))


class Run:
    """Device-resident inputs and buffers of one workload run."""

    def __init__(self, w, precision):
        from paper_1805_03426_amd.context import Context
        d = workload_inputs(w)
        self.w = w
        self.dt = d["dt"]
        self.ctx = Context(d["xf"], d["yf"], d["zf"], w.m, w.ra, w.pr, d["dt"], n_avg=w.n_avg,
                           precision=precision)
        dt_ = self.ctx.dtype
        self.U, self.V, self.W = (torch.from_numpy(d[k]).to("cuda", dt_) for k in ("U", "V", "W"))
        self.th0 = torch.from_numpy(d["theta0"]).to("cuda", dt_)
        c = self.ctx
        self.u, self.v, self.w_ = c.empty(c.shape_cell), c.empty(c.shape_cell), c.empty(c.shape_w)
        # ring[0] holds theta^0; ring[1..3] rotate; ring[4..] keep the levels
        # whose Nusselt profile is taken before the last one
        self.nu_levels = [n for n in range(w.nu_every, w.steps + 1, w.nu_every)] if w.nu_every else []
        kept = [n for n in self.nu_levels if n < w.steps]
        self.kept = {n: 4 + q for q, n in enumerate(kept)}
        self.ring = [self.th0] + [c.empty(c.shape_cell) for _ in range(3 + len(kept))]
        self.runner = c.step_runner(self.ring, self.u, self.v, self.w_)
        self.div = torch.empty(2, dtype=torch.float64, device="cuda")
        self.nprof = max(1, len(self.nu_levels))
        self.prof = torch.empty((max(1, self.nprof), c.nz + 6), dtype=torch.float64, device="cuda")
        self.host_inputs = d

    def step_groups(self):
        """Ranges [n0, n1) of steps launched back to back: the whole run."""
        return [(0, self.w.steps)]

    def run(self, events=None):
        """One whole run: refinement, divergence check, the steps as one
        mr_scalar_steps call (the library picks the fused line solver or the
        column sweeps; the levels whose Nusselt profile is taken go to buffers
        of their own), then the Nusselt profile of each of those levels.  With
        ``events`` (one (start, end) event pair per range of ``step_groups``)
        it records a pair on the current stream around the step launches."""
        c, w = self.ctx, self.w
        c.interpolate_velocity(self.U, self.V, self.W, out=(self.u, self.v, self.w_))
        c.divergence(self.u, self.v, self.w_, out=self.div)
        # outs[q] receives theta^{q+1}: a kept buffer, else one of three that
        # rotate (each output differs from the two levels before it)
        outs = [self.kept.get(n + 1, 1 + n % 3) for n in range(w.steps)]
        if events is not None:
            events[0][0].record()
        self.runner.steps(0, 0, 0, outs)
        if events is not None:
            events[0][1].record()
        for q, n in enumerate(self.nu_levels):
            c.nusselt(self.ring[outs[n - 1]], self.w_, profile=self.prof[q], sync=False)
        return self.ring[outs[-1]]


def time_runs(run, k, warmup, kernel_times=None):
    """Wall time of k whole runs after warm-up.  With kernel_times, the step
    kernel's time (ms per launch) of every range of back-to-back step launches,
    from an event pair around the range, is appended once per launch."""
    for _ in range(warmup):
        run.run()
    torch.cuda.synchronize()
    groups = run.step_groups()
    pools = [[(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
              for _ in groups] for _ in range(k)]
    t0 = time.perf_counter()
    for r in range(k):
        run.run(pools[r] if kernel_times is not None else None)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    if kernel_times is not None:
        for pool in pools:
            for (a, b), (n0, n1) in zip(pool, groups):
                kernel_times.extend([a.elapsed_time(b) / (n1 - n0)] * (n1 - n0))
    return el


def kernel_ms(times):
    return float(np.mean(times))


def copy_bandwidth():
    from paper_1805_03426_amd.context import copy_probe
    n = 1 << 30
    a = torch.empty(n, dtype=torch.uint8, device="cuda")
    b = torch.empty_like(a)
    a.fill_(1)
    for _ in range(3):
        copy_probe(a, b)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    reps = 10
    for _ in range(reps):
        copy_probe(a, b)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del a, b
    return 2.0 * n / (ms * 1e-3) / 1e9


def adjoint_alg_values(w, N, K):
    """Algorithmic values moved per dense cell by the forward and the backward
    pass of a checkpointed rollout (N steps, checkpoint every K):
    forward  = refinement 3(1 + 1/M^3) + 6 per step + 2 for the copy of theta^0
               + 2 for the returned copy (the kept states are written in place);
    backward = loss gradient 3 + seed 2 + per segment: recompute (len-1) x 6
               (not for the last segment, whose states the forward kept),
               reverse steps len x 6, velocity gradient 2 len + 6; + transposed
               refinement 3(1 + 1/M^3) + 3 zeroed gradients."""
    mcube = w.m[0] * w.m[1] * w.m[2]
    ref = 3.0 * (1.0 + 1.0 / mcube)
    segs = [min(s + K, N) - s for s in range(0, N, K)]
    fwd = ref + 6.0 * N + 2.0 + 2.0
    recompute = sum(6.0 * (L - 1) for L in segs[:-1])
    bwd = 3.0 + 2.0 + recompute + sum(6.0 * L + 2.0 * L + 6.0 for L in segs) + ref + 3.0
    return fwd, bwd


def adjoint_times(wname=ADJOINT_WORKLOAD, reps=3):
    """Forward (refine + N steps) and backward (recompute + reverse steps +
    velocity gradient + transposed refinement) of an adjoint workload (FP32):
    median times, cell-step throughput and % of HBM peak of each pass."""
    from paper_1805_03426_amd.autograd import rollout
    w = WORKLOADS[wname]
    r = Run(w, "fp32")
    N, K = w.steps, w.ckpt_every
    th0 = r.th0.clone().requires_grad_(True)
    U, V, W = (t.clone().requires_grad_(True) for t in (r.U, r.V, r.W))
    target = torch.from_numpy(inputs.theta_initial(r.host_inputs["zf"], r.ctx.nx, r.ctx.ny,
                                                   seed=inputs.SEED_TARGET)).to("cuda", torch.float32)
    del r.ring, r.runner, r.u, r.v, r.w_   # the rollout refines and steps on its own buffers
    tf, tb = [], []
    for rep in range(reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        out = rollout(r.ctx, th0, U, V, W, N, K)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        g = out - target
        torch.autograd.backward(out, g)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        if rep > 0:
            tf.append(t1 - t0)
            tb.append(t2 - t1)
        th0.grad = U.grad = V.grad = W.grad = None
        del out, g
    r.ctx.close()
    tf, tb = float(np.median(tf)), float(np.median(tb))
    vf, vb = adjoint_alg_values(w, N, K)
    frac = lambda values, t: values * 4 * w.cells / t / 1e9 / HBM_PEAK_GBS
    return dict(workload=wname, steps=N, ckpt_every=K, forward_s=tf, backward_s=tb,
                backward_over_forward=tb / tf,
                forward_cell_steps_per_s=w.cells * N / tf, backward_cell_steps_per_s=w.cells * N / tb,
                forward_hbm_frac_alg=frac(vf, tf), backward_hbm_frac_alg=frac(vb, tb),
                alg_values_per_cell=dict(forward=vf, backward=vb))


def _event_ms(fn, reps=20, warmup=3):
    """Mean time (ms) of fn() enqueued reps times on the current stream."""
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def intergrid_times(w, mt=4):
    """Inter-grid kernels of the workload (FP64): dense-to-coarse integration,
    Nu_T, refinement with and without the time interpolation, and one coarse
    step of mt scalar steps; algorithmic bytes per launch and % of HBM peak."""
    r = Run(w, "fp64")
    c = r.ctx
    cells, coarse = w.cells, w.cells // (w.m[0] * w.m[1] * w.m[2])
    ncw = coarse + c.ncx * c.ncy            # coarse W has one more level
    dense_w = cells + c.nx * c.ny
    U1, V1, W1 = (t.flip(0).contiguous() for t in (r.U, r.V, r.W))   # a second coarse level
    W1[0].zero_()
    W1[-1].zero_()
    tc = c.empty(c.shape_coarse)
    diss = torch.empty(4, dtype=torch.float64, device="cuda")
    uvw = (r.u, r.v, r.w_)
    out = {}

    def rec(name, ms, nbytes):
        out[name] = dict(ms=ms, alg_bytes=nbytes, hbm_frac=nbytes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS)

    rec("integrate_scalar", _event_ms(lambda: c.integrate_scalar(r.th0, out=tc)), 8 * (cells + coarse))
    rec("thermal_dissipation", _event_ms(lambda: c.thermal_dissipation(r.th0, out=diss, sync=False)), 8 * cells)
    rec("interpolate_velocity", _event_ms(lambda: c.interpolate_velocity(r.U, r.V, r.W, out=uvw)),
        8 * (2 * coarse + ncw + 2 * cells + dense_w))
    rec("interpolate_velocity_time",
        _event_ms(lambda: c.interpolate_velocity_time(r.U, r.V, r.W, U1, V1, W1, 1, mt, out=uvw)),
        8 * (2 * (2 * coarse + ncw) + 2 * cells + dense_w))
    ring = [r.th0.clone(), c.empty(c.shape_cell), c.empty(c.shape_cell)]
    state = {"n0": 0, "p": 0, "c": 0}

    def one_coarse_step():
        state["p"], state["c"] = c.coarse_step(state["n0"], mt, r.U, r.V, r.W, U1, V1, W1, uvw, ring,
                                               state["p"], state["c"], tc)
        state["n0"] += mt

    ms = _event_ms(one_coarse_step, reps=5, warmup=1)
    out["coarse_step"] = dict(mt=mt, ms=ms, dense_cell_updates_per_s=cells * mt / (ms * 1e-3))
    c.close()
    return out


def sequence_ms(r, count=10, reps=3):
    """Mean time per step (ms) of step sequences of the given length on a
    Run's buffers (one mr_scalar_steps call each), after one warm-up call."""
    state = {"n": 0, "prev": 0, "cur": 0}

    def seq():
        n0 = state["n"]
        outs = [1 + n % 3 for n in range(n0, n0 + count)]   # ring[0] holds theta^0
        r.runner.steps(n0, state["prev"], state["cur"], outs)
        state.update(n=n0 + count, prev=outs[-2], cur=outs[-1])

    return _event_ms(seq, reps=reps, warmup=1) / count


def large_step_times():
    """The step on the 576^3 (M = 3) workload in FP32 and in FP64 (the
    precision tier's reference run), in sequences of 10 steps: mean time per
    step and % of HBM peak (6 values per dense cell)."""
    out = {}
    for name, prec in (("rb576-m3-fp32", "fp32"), ("rb576-m3-fp32", "fp64")):
        w = WORKLOADS[name]
        r = Run(w, prec)
        c = r.ctx
        c.interpolate_velocity(r.U, r.V, r.W, out=(r.u, r.v, r.w_))
        ms = sequence_ms(r)
        nbytes = 6 * (8 if prec == "fp64" else 4) * w.cells
        key = name if prec == "fp32" else name.replace("fp32", "fp64")
        out[key] = dict(step_method=c.step_method, step_ms=ms, dense_cell_updates_per_s=w.cells / (ms * 1e-3),
                        step_hbm_frac_alg=nbytes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS)
        c.close()
        del r
        torch.cuda.empty_cache()
    return out


def whole_runs(w, precision, k, warmup):
    """k timed whole runs of a workload in a precision: job throughput and the
    step kernel's mean time and % of HBM peak (6 values per cell)."""
    r = Run(w, precision)
    ev = []
    el = time_runs(r, k, warmup, ev)
    ms = kernel_ms(ev)
    vb = 8 if precision == "fp64" else 4
    out = dict(workload=w.name, precision=precision, step_method=r.ctx.step_method,
               value=w.cells * w.steps * k / el,
               unit="dense-cell updates/s", ms_per_run=el / k * 1e3, step_kernel_ms=ms,
               step_hbm_frac_alg=6 * vb * w.cells / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS)
    r.ctx.close()
    del r
    torch.cuda.empty_cache()
    return out


def walls_times(w):
    """The workload's FP64 step and refinement with adiabatic no-slip side
    walls in x and y (the generator's coarse velocity with its low wall faces
    zeroed): mean kernel times and % of HBM peak."""
    from paper_1805_03426_amd.context import Context
    d = workload_inputs(w)
    ctx = Context(d["xf"], d["yf"], d["zf"], w.m, w.ra, w.pr, d["dt"], n_avg=w.n_avg, side_x="walls",
                  side_y="walls")
    U, V, W = (torch.from_numpy(d[k]).to("cuda", torch.float64) for k in ("U", "V", "W"))
    U[:, :, 0] = 0.0
    V[:, 0, :] = 0.0
    u, v, w_ = ctx.empty(ctx.shape_cell), ctx.empty(ctx.shape_cell), ctx.empty(ctx.shape_w)
    ref_ms = _event_ms(lambda: ctx.interpolate_velocity(U, V, W, out=(u, v, w_)), reps=10)
    ring = [torch.from_numpy(d["theta0"]).to("cuda", torch.float64)] + [ctx.empty(ctx.shape_cell) for _ in range(3)]
    runner = ctx.step_runner(ring, u, v, w_)
    state = {"n": 0, "prev": 0, "cur": 0}

    def step():
        n, out = state["n"], 1 + state["n"] % 3
        runner.step(n, state["prev"], state["cur"], out)
        state.update(n=n + 1, prev=state["cur"], cur=out)

    ms = _event_ms(step, reps=20, warmup=3)
    ctx.close()
    return dict(step_kernel_ms=ms, step_hbm_frac_alg=48 * w.cells / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                refine_ms=ref_ms)


def variant_step_times(w, **variant):
    """The workload's FP64 step in a variant of the method (``variant`` goes to
    the Context: z_explicit = 1/2 for the Crank-Nicolson z share, face_order = 4
    for fourth-order face values): mean kernel time and % of HBM peak (the same
    algorithmic 48 B per cell)."""
    from paper_1805_03426_amd.context import Context
    d = workload_inputs(w)
    ctx = Context(d["xf"], d["yf"], d["zf"], w.m, w.ra, w.pr, d["dt"], n_avg=w.n_avg, **variant)
    U, V, W = (torch.from_numpy(d[k]).to("cuda", torch.float64) for k in ("U", "V", "W"))
    u, v, w_ = ctx.interpolate_velocity(U, V, W)
    ring = [torch.from_numpy(d["theta0"]).to("cuda", torch.float64)] + [ctx.empty(ctx.shape_cell) for _ in range(3)]
    runner = ctx.step_runner(ring, u, v, w_)
    state = {"n": 0, "prev": 0, "cur": 0}

    def step():
        n, out = state["n"], 1 + state["n"] % 3
        runner.step(n, state["prev"], state["cur"], out)
        state.update(n=n + 1, prev=state["cur"], cur=out)

    ms = _event_ms(step, reps=20, warmup=3)
    ctx.close()
    return dict(variant, step_kernel_ms=ms, step_hbm_frac_alg=48 * w.cells / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS)


def host_cpu():
    """The host's logical CPU count, the threads this process may use, and its
    CPU model (for the CPU baseline's context)."""
    model = None
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    avail = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    return dict(nproc=os.cpu_count(), affinity=avail, model=model)


def cpu_baseline(w, budget_s=15.0):
    """The oracle's FP64 scalar step on a bounded sample: as many whole-field
    steps of workload w as fit in the budget (at least one).  The oracle is
    plain NumPy; its elementwise kernels run on one core."""
    import oracle as O
    d = workload_inputs(w)
    g = O.Grid(d["xf"], d["yf"], d["zf"], w.m)
    p = O.ScalarParams.from_ra_pr(w.ra, w.pr, d["dt"], n_avg=w.n_avg)
    uvw = O.refine_velocity(g, d["U"], d["V"], d["W"])
    prev = cur = d["theta0"]
    t0 = time.perf_counter()
    n = 0
    while True:
        nxt = O.scalar_step(g, p, n, prev, cur, *uvw)
        prev, cur = cur, nxt
        n += 1
        if time.perf_counter() - t0 > budget_s or n >= 40:
            break
    el = time.perf_counter() - t0
    return dict(value=w.cells * n / el, unit="dense-cell updates/s", cores=1, kind="oracle",
                sample="%d whole-field FP64 scalar steps of %s (%d cells; the 1024x1024x512 grid's "
                       "4.3 GB fields are not run by the oracle), NumPy single-threaded, %.1f s"
                       % (n, w.name, w.cells, el),
                host=host_cpu())


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true", help="skip FP32 / adjoint / copy measurements")
    ap.add_argument("--workload", default=WORKLOAD, choices=sorted(k for k in WORKLOADS if k.endswith("fp64")),
                    help="FP64 workload timed as the headline (default: the largest one-GPU grid)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="launch the copy kernel on 1 GiB once (counter calibration for profiles)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU: the scalar step is a single-GPU kernel here "
              "(a multi-GPU y-slab decomposition is designed but not built); run with --gpus 1",
              file=sys.stderr)
        sys.exit(2)
    torch.cuda.set_device(0)
    w = WORKLOADS[args.workload]
    print("bench: %s, %d runs + %d warmup" % (w.name, args.steps, args.warmup), file=sys.stderr, flush=True)
    run = Run(w, "fp64")
    step_kernel = STEP_KERNELS[run.ctx.step_method]
    events = []
    el = time_runs(run, args.steps, args.warmup, events)
    cells_per_run = w.cells * w.steps
    value = cells_per_run * args.steps / el
    ms_step = kernel_ms(events)
    alg_bytes = 6 * 8 * w.cells
    achieved = alg_bytes / (ms_step * 1e-3) / 1e9
    traffic = committed_traffic(w.name, run.ctx.step_method)
    run.ctx.close()
    del run
    torch.cuda.empty_cache()

    extras = {}
    if not args.no_extras:
        print("bench: FP32 tier on the same grid", file=sys.stderr, flush=True)
        extras["fp32"] = whole_runs(w, "fp32", max(1, args.steps), 1)
        ws = WORKLOADS[SMALL_WORKLOAD]
        print("bench: %s FP64 and FP32" % ws.name, file=sys.stderr, flush=True)
        extras["rb256"] = {prec: whole_runs(ws, prec, max(1, args.steps), 1) for prec in ("fp64", "fp32")}
        print("bench: adjoint", file=sys.stderr, flush=True)
        extras["adjoint"] = adjoint_times()
        torch.cuda.empty_cache()
        print("bench: inter-grid kernels", file=sys.stderr, flush=True)
        extras["intergrid"] = intergrid_times(ws)
        torch.cuda.empty_cache()
        print("bench: side walls", file=sys.stderr, flush=True)
        extras["walls_xy"] = walls_times(ws)
        torch.cuda.empty_cache()
        print("bench: step with an explicit z share", file=sys.stderr, flush=True)
        extras["z_explicit"] = variant_step_times(ws, z_explicit=0.5)
        torch.cuda.empty_cache()
        print("bench: step with fourth-order faces", file=sys.stderr, flush=True)
        extras["face_order4"] = variant_step_times(ws, face_order=4)
        torch.cuda.empty_cache()
        print("bench: step at 576^3 (FP32, FP64)", file=sys.stderr, flush=True)
        extras["large_steps"] = large_step_times()
        torch.cuda.empty_cache()
        print("bench: adjoint at 1024x1024x512", file=sys.stderr, flush=True)
        extras["adjoint_large"] = adjoint_times("rb1024x1024x512-m2-fp32", reps=2)
        torch.cuda.empty_cache()
        extras["copy_bandwidth_GBs"] = copy_bandwidth()

    if args.copy_probe:
        from paper_1805_03426_amd.context import copy_probe
        a = torch.ones(1 << 30, dtype=torch.uint8, device="cuda")
        b = torch.empty_like(a)
        copy_probe(a, b)
        torch.cuda.synchronize()
        del a, b

    cpu = None
    if not args.no_cpu_baseline:
        print("bench: CPU baseline (oracle)", file=sys.stderr, flush=True)
        cpu = cpu_baseline(WORKLOADS[CPU_WORKLOAD])

    line = {
        "metric": METRIC,
        "value": value,
        "unit": "dense-cell updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": el / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic (seeded divergence-free velocity, conduction profile + noise)",
        "config": {"workload": w.name, "coarse": list(w.nc), "dense": list(w.n), "refinement": list(w.m),
                   "z_tanh": w.gamma, "ra": w.ra, "pr": w.pr, "scalar_steps_per_run": w.steps,
                   "nusselt_every": w.nu_every, "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "kernel": step_kernel, "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": traffic, "avg_kernel_ms": ms_step,
                     "alg_bytes_per_launch": alg_bytes,
                     # measured HBM bytes (committed counters) over the live kernel time
                     "traffic_frac": (traffic / (ms_step * 1e-3) / 1e9 / HBM_PEAK_GBS) if traffic else None},
        "cpu_baseline": cpu,
    }
    line.update(extras)
    print(json.dumps(line))


if __name__ == "__main__":
    main()
