"""Autotuner for the batched solve: Krylov method (GMRES or COCG), restart
lengths, inner step limits and tolerance, and the rows per LDS tile of the
fused operator pass.

Each candidate runs the batched solve (vdc_solve) on an evenly spaced sample
of the job list (the list is cost-ordered by energy, so the sample spans the
range); the candidate with the smallest solver-kernel time per converged
right-hand side (HIP events, vdc_last_kernel_times) wins.  Candidates that
leave a sampled job unconverged are discarded.  Results are cached in a JSON
file keyed by basis shape, job count bucket and precision.
"""
import json
import os
from dataclasses import asdict, replace

from . import vdc

# GMRES restart lengths and COCG (Sec. III.A) in FP64; FGMRES with FP32 GMRES
# inner cycles, and FP64 refinement with FP32 COCG correction solves (inner
# step limit, inner tolerance)
FP64_CANDIDATES = ([dict(method=vdc.GMRES, restart=m) for m in (4, 5, 6, 8, 10, 15)] +
                   [dict(method=vdc.COCG)])
FP32_CANDIDATES = ([dict(method=vdc.GMRES, inner_restart=mi, inner_tol=ti, outer_restart=mo)
                    for mi, ti, mo in ((4, 1e-3, 32), (6, 1e-3, 24), (6, 1e-2, 32), (8, 1e-3, 16),
                                       (8, 1e-2, 24), (8, 1e-3, 24), (10, 1e-3, 16), (12, 1e-4, 12),
                                       (15, 1e-4, 8))] +
                   [dict(method=vdc.COCG, inner_restart=mi, inner_tol=ti)
                    for mi, ti in ((60, 1e-3), (100, 1e-3), (100, 1e-4), (200, 1e-5))])
TILE_CANDIDATES = (0, 4, 8)


def _key(models, n_jobs, precision, precond):
    shapes = sorted({(m.Ng, m.Nu) for m in models})
    bucket = 1 << max(0, (n_jobs - 1).bit_length())
    return f"{precision}:p{precond}:{shapes}:{bucket}:methods"


def autotune(models, jobs, finals, base=None, sample=384, cache=None, reps=2):
    """Returns (best Opts, report list).  models: list of vdc.Model2D."""
    base = base or vdc.Opts()
    models = list(models) if isinstance(models, (list, tuple)) else [models]
    precision = "fp64" if base.precision == vdc.FP64 else "fp32"
    key = _key(models, len(jobs), precision, base.precond)
    if cache and os.path.exists(cache):
        with open(cache) as fh:
            saved = json.load(fh)
        if key in saved:
            return replace(base, **saved[key]["opts"]), saved[key]["report"]
    step = max(1, len(jobs) // sample)
    sub = jobs[::step][:sample]
    cands = FP64_CANDIDATES if base.precision == vdc.FP64 else FP32_CANDIDATES
    report, best = [], None
    for c in cands:
        for t in TILE_CANDIDATES:
            o = replace(base, tile_rows=t, **c)
            s = vdc.Solver(models, sub, finals, o)
            ms = []
            for _ in range(reps):
                s.run()
                ms.append(vdc.last_kernel_times()[1])
            infos = s.infos()
            ok = all(i["status"] == vdc.CONVERGED for i in infos)
            per = min(ms) / max(1, len(sub))
            report.append(dict(opts={**c, "tile_rows": t}, ms_per_solve=per, converged=ok))
            if ok and (best is None or per < best[0]):
                best = (per, {**c, "tile_rows": t})
    if best is None:
        return base, report
    chosen = replace(base, **best[1])
    if cache:
        saved = {}
        if os.path.exists(cache):
            with open(cache) as fh:
                saved = json.load(fh)
        saved[key] = dict(opts=best[1], report=report)
        with open(cache, "w") as fh:
            json.dump(saved, fh, indent=1)
    return chosen, report


def opts_dict(o):
    return {k: v for k, v in asdict(o).items()}
