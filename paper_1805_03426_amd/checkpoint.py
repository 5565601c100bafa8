"""On-disk state of a scalar run, for stopping and resuming it.

The Euler-leapfrog integration (Eqs. 6-7) advances from two levels, so the
state is the pair (theta^{n-1}, theta^n) and the step index n (which fixes the
kind of the next step: start-up, leapfrog or averaging).  The file is a
safetensors file (tensors and string metadata only, nothing executable): the
two levels in the context's storage precision, n, and the grid size,
precision and time-stepping parameters, which ``load`` checks against the
context the run resumes in.  A resumed run computes the same bits as one that
never stopped, since the library's steps depend only on these inputs.
"""
import json

from safetensors.torch import load_file, save_file

_KEYS = ("nx", "ny", "nz", "precision", "dt", "ra", "pr", "n_avg")


def _meta(ctx):
    d = ctx.desc
    return {"nx": str(ctx.nx), "ny": str(ctx.ny), "nz": str(ctx.nz), "precision": ctx.precision,
            "dt": repr(float(d.dt)), "ra": repr(float(d.ra)), "pr": repr(float(d.pr)), "n_avg": str(int(d.n_avg))}


def save(path, ctx, n, th_prev, th_cur):
    """Write theta^{n-1} (``th_prev``; may be None at n = 0), theta^n and n for
    the run of context ``ctx`` to ``path``."""
    if n < 0:
        raise ValueError("n must be >= 0")
    if th_prev is None:
        if n > 0:
            raise ValueError("n > 0 needs theta^{n-1}")
        th_prev = th_cur
    for name, t in (("th_prev", th_prev), ("th_cur", th_cur)):
        if tuple(t.shape) != ctx.shape_cell or t.dtype != ctx.dtype:
            raise ValueError("%s: expected %s %s, got %s %s" % (name, ctx.shape_cell, ctx.dtype, tuple(t.shape),
                                                                t.dtype))
    meta = _meta(ctx)
    meta["n"] = str(int(n))
    tensors = {"th_prev": th_prev.detach().to("cpu", copy=True).contiguous(),
               "th_cur": th_cur.detach().to("cpu", copy=True).contiguous()}
    save_file(tensors, path, metadata=meta)


def load(path, ctx):
    """Read a state written by ``save`` for a run in context ``ctx``: returns
    (n, theta^{n-1}, theta^n) as device tensors.  Raises ValueError when the
    file was written for another grid, precision or time-stepping setup."""
    with open(path, "rb") as f:
        header_len = int.from_bytes(f.read(8), "little")
        meta = json.loads(f.read(header_len)).get("__metadata__", {})
    want = _meta(ctx)
    for k in _KEYS:
        if meta.get(k) != want[k]:
            raise ValueError("checkpoint %s: %s is %r, the context has %r" % (path, k, meta.get(k), want[k]))
    t = load_file(path, device="cpu")
    dev = ctx.device
    return int(meta["n"]), t["th_prev"].to(dev), t["th_cur"].to(dev)
