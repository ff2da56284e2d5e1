"""Linear solvers for (E - H_ef) Psi = Phi (oracle; test infrastructure).

* lu_solve: the plain definition of the solution, by a library LU
  factorisation (SuperLU on the sparse matrix, or LAPACK getrf on a dense one).
* gmres: textbook restarted GMRES(m) of Saad and Schultz as described in
  Sec. III.A: Arnoldi with modified Gram-Schmidt builds A V_n = V_{n+1} H_n,
  the (n+1) x n least-squares problem for y_n is solved by Givens rotations,
  x_n = x_0 + M^{-1} V_n y_n (right preconditioning by M, Sec. III.B: the
  diagonal of A, or any block-diagonal section of it given as a solve).  Stopping rule of Sec. III: ||b - A x|| < tol ||b||,
  checked on the true residual at the end of each cycle.
"""
import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla


def lu_solve(A, b):
    if sp.issparse(A):
        return spla.splu(sp.csc_matrix(A)).solve(np.asarray(b, dtype=np.complex128))
    lu, piv = sla.lu_factor(np.asarray(A, dtype=np.complex128))
    return sla.lu_solve((lu, piv), np.asarray(b, dtype=np.complex128))


def gmres(A, b, m=50, tol=1e-10, max_iter=20000, dinv=None, history=False, psolve=None):
    """Restarted GMRES(m), x0 = 0, right preconditioner z = M^{-1} v: psolve(v)
    when given, else dinv * v (dinv = 1 without either).

    Returns (x, info) with info = dict(iters, restarts, rel_res, converged[, hist]).
    """
    b = np.asarray(b, dtype=np.complex128)
    n = b.size
    if dinv is None:
        dinv = np.ones(n, dtype=np.complex128)
    if psolve is None:
        psolve = (lambda v: dinv * v)
    bnorm = np.linalg.norm(b)
    x = np.zeros(n, dtype=np.complex128)
    if bnorm == 0.0:
        return x, dict(iters=0, restarts=0, rel_res=0.0, converged=True)
    matvec = (lambda v: A @ v)
    r = b - matvec(x)
    beta = np.linalg.norm(r)
    iters, restarts, hist = 0, 0, []
    while True:
        V = np.zeros((m + 1, n), dtype=np.complex128)
        H = np.zeros((m + 1, m), dtype=np.complex128)
        cs = np.zeros(m, dtype=np.float64)
        sn = np.zeros(m, dtype=np.complex128)
        g = np.zeros(m + 1, dtype=np.complex128)
        g[0] = beta
        V[0] = r / beta
        k = 0
        for j in range(m):
            w = matvec(psolve(V[j]))
            for i in range(j + 1):                       # modified Gram-Schmidt
                H[i, j] = np.vdot(V[i], w)
                w = w - H[i, j] * V[i]
            hnext = np.linalg.norm(w)
            H[j + 1, j] = hnext
            for i in range(j):                           # previous rotations
                t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
                H[i + 1, j] = -np.conj(sn[i]) * H[i, j] + cs[i] * H[i + 1, j]
                H[i, j] = t
            a, bb = H[j, j], H[j + 1, j]                 # new rotation
            den = np.hypot(abs(a), abs(bb))
            if den == 0.0:
                cs[j], sn[j] = 1.0, 0.0
            elif abs(a) == 0.0:
                cs[j], sn[j] = 0.0, 1.0
            else:
                cs[j] = abs(a) / den
                sn[j] = (a / abs(a)) * np.conj(bb) / den
            H[j, j] = cs[j] * a + sn[j] * bb
            H[j + 1, j] = 0.0
            g[j + 1] = -np.conj(sn[j]) * g[j]
            g[j] = cs[j] * g[j]
            iters += 1
            k = j + 1
            hist.append(abs(g[j + 1]) / bnorm)
            if abs(g[j + 1]) <= tol * bnorm or iters >= max_iter:
                break
            if hnext == 0.0:                             # exact (lucky) breakdown
                break
            V[j + 1] = w / hnext
        y = sla.solve_triangular(H[:k, :k], g[:k], lower=False)
        x = x + psolve(V[:k].T @ y)
        r = b - matvec(x)
        beta = np.linalg.norm(r)
        restarts += 1
        if beta <= tol * bnorm or iters >= max_iter:
            break
    info = dict(iters=iters, restarts=restarts, rel_res=beta / bnorm,
                converged=bool(beta <= tol * bnorm))
    if history:
        info["hist"] = np.array(hist)
    return x, info
