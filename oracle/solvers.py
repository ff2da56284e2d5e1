"""Linear solvers for (E - H_ef) Psi = Phi (oracle; test infrastructure).

* lu_solve: the plain definition of the solution, by a library LU
  factorisation (SuperLU on the sparse matrix, or LAPACK getrf on a dense one).
* gmres: textbook restarted GMRES(m) of Saad and Schultz as described in
  Sec. III.A: Arnoldi with modified Gram-Schmidt builds A V_n = V_{n+1} H_n,
  the (n+1) x n least-squares problem for y_n is solved by Givens rotations,
  x_n = x_0 + M^{-1} V_n y_n (right preconditioning by M, Sec. III.B: the
  diagonal of A, or any block-diagonal section of it given as a solve).  Stopping rule of Sec. III: ||b - A x|| < tol ||b||,
  checked on the true residual at the end of each cycle.
* cocg: the conjugate orthogonal conjugate gradient method of Sec. III.A
  (conjugate gradients with the symmetrized bilinear form <a|b>_S = sum a_i
  b_i in place of the scalar product, for complex symmetric A), preconditioned
  as M^{-1} A M^{-T} y = M^{-1} b, x = M^{-T} y (Sec. III.B), written in the
  coupled two-term form with K = M M^T applied as a solve.
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


def bilinear(a, b):
    """<a|b>_S = <a*|b> = sum_i a_i b_i: the symmetrized bilinear form of
    Sec. III.A (no complex conjugation)."""
    return np.sum(np.asarray(a) * np.asarray(b))


def cocg(A, b, tol=1e-10, max_iter=20000, psolve=None, history=False):
    """Preconditioned COCG, x0 = 0 (Sec. III.A, III.B).

    The basis vectors of the paper's recurrence are, up to scaling, the
    residuals r_k, conjugate orthogonal in the preconditioned form:
    <r_i | K^{-1} r_j>_S = 0 for i != j.  With K = M M^T (psolve = K^{-1},
    identity when None) the iteration is conjugate gradients on
    M^{-1} A M^{-T} with <.|.>_S, mapped back to x = M^{-T} y:
        r = b, z = K^{-1} r, p = z, rho = <r|z>_S
        repeat: q = A p, alpha = rho / <p|q>_S, x += alpha p, r -= alpha q,
                z = K^{-1} r, rho' = <r|z>_S, p = z + (rho'/rho) p.
    Stops when the updated residual satisfies ||r|| <= tol ||b|| and the true
    residual b - A x does as well; if only the updated one does, the
    iteration restarts from the true residual.  A vanishing <p|q>_S or
    <r|z>_S is a breakdown (the bilinear form is not definite).

    Returns (x, info) with info = dict(iters, restarts, rel_res, converged,
    breakdown[, residuals]) (residuals: the r_k, when history is set).
    """
    b = np.asarray(b, dtype=np.complex128)
    if psolve is None:
        psolve = (lambda v: v)
    bnorm = np.linalg.norm(b)
    x = np.zeros_like(b)
    if bnorm == 0.0:
        return x, dict(iters=0, restarts=0, rel_res=0.0, converged=True, breakdown=False)
    r = b.copy()
    z = psolve(r)
    p = z.copy()
    rho = bilinear(r, z)
    iters, restarts, breakdown, rs = 0, 0, False, [r.copy()]
    rel = 1.0
    while iters < max_iter:
        q = A @ p
        mu = bilinear(p, q)
        if mu == 0.0 or rho == 0.0:
            breakdown = True
            break
        alpha = rho / mu
        x = x + alpha * p
        r = r - alpha * q
        iters += 1
        if np.linalg.norm(r) <= tol * bnorm:
            rt = b - A @ x
            rel = np.linalg.norm(rt) / bnorm
            if rel <= tol:
                break
            r = rt                                   # restart from the true residual
            z = psolve(r)
            p = z.copy()
            rho = bilinear(r, z)
            restarts += 1
            continue
        if history:
            rs.append(r.copy())
        z = psolve(r)
        rho_new = bilinear(r, z)
        p = z + (rho_new / rho) * p
        rho = rho_new
    rel = np.linalg.norm(b - A @ x) / bnorm
    info = dict(iters=iters, restarts=restarts, rel_res=rel, converged=bool(rel <= tol),
                breakdown=breakdown)
    if history:
        info["residuals"] = rs
    return x, info
