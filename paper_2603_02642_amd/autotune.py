"""Launch-schedule autotuner for batched solves.

The schedule knob of the persistent solver is the size of the workgroup that
owns one instance (block_threads: 64..512 work-items, i.e. 1..8 wavefronts
sharing the instance's cone tasks).  More wavefronts per instance shorten each
instance's passes; fewer let more instances share a compute unit (the LDS an
instance needs -- gains, adjoint accumulator, factors -- bounds how many fit).
The tuner times, on the batch itself, one solve with identical work for every
candidate (fixed iteration counts, no early exit) and leaves the context set to
the fastest.  Timing is HIP events on the context's stream.  The solves start
from the cold point, so tune before warm-starting a batch.
"""
from __future__ import annotations

from typing import Dict, Sequence, Tuple

from . import nrto

CANDIDATES = (64, 128, 256, 512)


def _copy(o: nrto.Options) -> nrto.Options:
    c = nrto.Options()
    for name, _ in nrto.Options._fields_:
        setattr(c, name, getattr(o, name))
    return c


def tune_block_threads(ctx: "nrto.Context", stream, candidates: Sequence[int] = CANDIDATES, admm: int = 2,
                       inner: int = 10) -> Tuple[int, Dict[int, float]]:
    """Returns (best block_threads, {candidate: ms}); ctx keeps its options with
    block_threads = best.  stream: the torch stream ctx was created on."""
    import torch
    base = _copy(ctx.options)
    times: Dict[int, float] = {}
    for th in candidates:
        o = _copy(base)
        o.block_threads = th
        o.max_admm, o.max_inner = admm, inner
        o.eps_kkt = 0.0
        o.eps_dr_abs = o.eps_dr_rel = 0.0
        try:
            ctx.set_options(o)
        except nrto.NrtoError:
            continue                      # e.g. the LDS need exceeds the compute unit's
        with torch.cuda.stream(stream):
            ctx.linearize()
            ctx.solve_async()
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(stream)
            ctx.solve_async()
            b.record(stream)
        b.synchronize()
        times[th] = a.elapsed_time(b)
    if not times:
        ctx.set_options(base)
        raise nrto.NrtoError("no block size could be set up for this batch")
    best = min(times, key=times.get)
    base.block_threads = best
    ctx.set_options(base)
    return best, times
