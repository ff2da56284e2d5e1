"""Oracle checks of GPU results at full size, run in worker processes (the
oracle's level-shift tables and sparse LU take seconds per right-hand side
at these sizes and hold the GIL).  Every function here calls the oracle only
and returns small summaries; the GPU results come in as arrays."""
import os

import numpy as np


def pool_map(fn, args, workers=None):
    """fn(*a) for a in args in spawned worker processes (at most 16, one
    thread each), results in order."""
    import multiprocessing as mp
    from concurrent.futures import ProcessPoolExecutor
    args = list(args)
    n = max(1, min(workers or 16, os.cpu_count() or 1, len(args)))
    with ProcessPoolExecutor(max_workers=n, mp_context=mp.get_context("spawn")) as ex:
        futs = [ex.submit(fn, *a) for a in args]
        return [f.result() for f in futs]


def _single_thread():
    from threadpoolctl import threadpool_limits
    return threadpool_limits(limits=1)


def check_2d_job(p, Ng, Nu, job, finals, psi_gpu):
    """Two-state model: the oracle's ||b - A psi_gpu|| / ||b||, its LU solution's
    distance to psi_gpu (relative) and its amplitudes T [n_final][2]."""
    from oracle import model2d as m2
    from oracle import solvers
    with _single_thread():
        eps_i, vi, mu = job[0], tuple(job[1]), job[2]
        mdl = m2.Model2D(p, Ng, Nu, m2.total_energy(p, eps_i, vi))
        A = mdl.matrix()
        b = mdl.phi(vi, m2.MU[mu])
        res = float(np.linalg.norm(b - A @ psi_gpu) / np.linalg.norm(b))
        psi = solvers.lu_solve(A, b)
        err = float(np.linalg.norm(psi_gpu - psi) / np.linalg.norm(psi))
        T = np.array([[mdl.phi(vf, mf) @ psi for mf in m2.MU] for vf in finals])
        return dict(res=res, psi_err=err, T=T)


def unique_pair_tables(p, eps):
    """The CO2-like model's six level-shift functions (oracle pair_tables) at
    each distinct value of eps, spread back to every point."""
    from oracle import poly
    u, inv = np.unique(np.asarray(eps, dtype=np.float64), return_inverse=True)
    t = poly.pair_tables(p, u)
    return {k: v[inv] for k, v in t.items()}


def check_co2_job(p, sizes, job, finals, psi_full):
    """CO2-like model: the oracle's ||b - A psi_gpu|| / ||b|| with its own
    assembled A, and the amplitudes Phi_f^T psi_gpu [n_final][3]."""
    from oracle import poly
    with _single_thread():
        eps_i, v, mu = job
        E = poly.total_energy(p, eps_i, v)
        M = poly.PolyModel(p, sizes, E, tables=unique_pair_tables)
        A = M.matrix()
        b = M.phi(v, poly.WAVES[mu])
        res = float(np.linalg.norm(b - A @ psi_full) / np.linalg.norm(b))
        T = np.array([[M.phi(vf, w) @ psi_full for w in poly.WAVES] for vf in finals])
        nA = float(abs(A).sum(axis=1).max())
        return dict(res=res, T=T, normA_inf=nA, norm_psi=float(np.linalg.norm(psi_full)),
                    norm_b=float(np.linalg.norm(b)))


def grad_one_energy(p, target, Ng, Nu, eps_i, v_i, finals):
    """Loss and gradient (oracle adjoint.loss_and_grad) at one incident
    energy, with the target cross sections of the parameters ``target``."""
    from oracle import adjoint as adj
    with _single_thread():
        sig_t, _ = adj.forward(target, Ng, Nu, [eps_i], v_i, finals)
        L, g, sig = adj.loss_and_grad(p, Ng, Nu, [eps_i], v_i, finals, sig_t)
        return dict(L=L, g=g, sig=sig, sig_t=sig_t)
