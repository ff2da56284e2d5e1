"""Loss and gradient of cross sections with respect to the model parameters
(oracle; test infrastructure).

Loss: L = sum over incident energies eps_i and final states v_f of
(sigma_{v_f <- v_i}(eps_i) - sigma*_{v_f}(eps_i))^2, sigma from Eq. (16)
(summed over mu_i, mu_f), parameters in PARAM_NAMES order.

Gradient by the adjoint method written out plainly: for each (eps_i, mu_i)
  Psi = A^-1 Phi_i,  T_f = Phi_f^T Psi,
  W_f = dL/dT_f (complex weight so that dL = Re sum_f W_f dT_f)
      = 2 c g_f conj(T_f),  c = 2 pi^3/eps_i, g_f = dL/dsigma_f,
  zeta = A^-T (sum_f W_f Phi_f) = A^-1 (...)   (A^T = A, Sec. III.A),
  dL/dp += Re[ sum_f W_f (dPhi_f/dp)^T Psi + zeta^T (dPhi_i/dp) - zeta^T (dA/dp) Psi ].
dA/dp is assembled as an explicit sparse matrix from the derivatives of its
ingredients (H_0, U, and the sandwich O diag(F) O of Eq. (23)); the level
shift's derivatives come from differentiating the segment-wise principal
value (in eps) and from transforming dg/dB (the transform is linear in g).
Solves use LU (dense for small bases when requested).
"""
import math

import numpy as np
import scipy.sparse as sp

from . import levelshift as ls
from . import model2d as m2
from .observables import sigma_prefactor
from .solvers import lu_solve

PARAM_NAMES = m2.PARAM_NAMES
PAIRS = ((1, 1), (1, 2), (2, 2))


def _g_func(p, mu, d1, d2):
    A1, B1 = p["A%d%s" % (d1, mu)], p["B%d%s" % (d1, mu)]
    A2, B2 = p["A%d%s" % (d2, mu)], p["B%d%s" % (d2, mu)]
    l = p["l_" + mu]
    return (lambda x: ls.pair_g(np.atleast_1d(x), A1, B1, A2, B2, l)), (A1, B1, A2, B2, l)


def deps_tables(p, eps):
    """d F[f_d^mu f_d'^mu] / d eps at the points eps, for the six functions."""
    x = ls.grid_nodes(p["K"], p["X"])
    out = {}
    for mu in m2.MU:
        for d1, d2 in PAIRS:
            gfun, (A1, B1, A2, B2, l) = _g_func(p, mu, d1, d2)
            re = ls.dpv_linear_segments_deps(eps, x, gfun(x)) / (2 * math.pi)
            e = np.atleast_1d(eps)
            ge = gfun(e)
            rate = np.where(e > 0, (l + 0.5) / np.where(e > 0, e, 1.0), 0.0) - 0.5 * (1 / B1 + 1 / B2)
            out[(mu, d1, d2)] = re - 0.5j * ge * rate
    return out


def dparam_tables(p, eps, name):
    """d F[f_d^mu f_d'^mu](eps) / d(name) for name among the A's and B's."""
    kind, d, mu = name[0], int(name[1]), name[2]
    out = {}
    zero = np.zeros(np.shape(np.atleast_1d(eps)), dtype=complex)
    for mu2 in m2.MU:
        for d1, d2 in PAIRS:
            key = (mu2, d1, d2)
            if mu2 != mu or d not in (d1, d2):
                out[key] = zero
                continue
            mult = 2.0 if d1 == d2 else 1.0        # g is linear (d=d') or sqrt in A_d
            gfun, (A1, B1, A2, B2, l) = _g_func(p, mu2, d1, d2)
            if kind == "A":
                A = p["A%d%s" % (d, mu)]
                F = ls.level_shift_table(eps, A1, B1, A2, B2, l, K=p["K"], X=p["X"])
                out[key] = F * (mult / (2.0 * A))
            else:
                B = p["B%d%s" % (d, mu)]
                dg = (lambda xx, gfun=gfun, B=B, mult=mult: gfun(xx) * np.atleast_1d(xx) * mult / (2 * B * B))
                out[key] = ls.level_shift_table(eps, A1, B1, A2, B2, l, g_override=dg, K=p["K"], X=p["X"])
    return out


def _F_from(mdl, tables, dO=None):
    """sum_mu O_d^mu diag(t^mu_dd') O_d'^mu as a 2x2 block sparse matrix; with
    dO given, the derivative sum_mu (dO diag(t) O + O diag(t) dO)."""
    n = mdl.n

    def Fd(mu, d, dp):
        return sp.diags(tables[(mu, min(d, dp), max(d, dp))], 0, format="csr")

    blocks = [[None, None], [None, None]]
    for d in (1, 2):
        for dp in (1, 2):
            acc = sp.csr_matrix((n, n), dtype=complex)
            for mu in m2.MU:
                Od, Odp = mdl.O[(d, mu)], mdl.O[(dp, mu)]
                if dO is None:
                    acc = acc + Od @ Fd(mu, d, dp) @ Odp
                else:
                    a = dO.get((d, mu))
                    b = dO.get((dp, mu))
                    if a is not None:
                        acc = acc + a @ Fd(mu, d, dp) @ Odp
                    if b is not None:
                        acc = acc + Od @ Fd(mu, d, dp) @ b
            blocks[d - 1][dp - 1] = acc
    return sp.bmat(blocks, format="csr")


def dA_dp(mdl, name, v_i):
    """Explicit sparse dA/d(name) at the model's energy E = eps_i + E_{v_i}."""
    p, n = mdl.p, mdl.n
    Ng, Nu = mdl.Ng, mdl.Nu
    Z = sp.csr_matrix((n, n))
    I = mdl.I
    ng = np.repeat(np.arange(Ng), Nu).astype(float)
    nu = np.tile(np.arange(Nu), Ng).astype(float)
    if name in ("omega_g", "omega_u"):
        w = (v_i[0] - ng) if name == "omega_g" else (v_i[1] - nu)   # d eps_nu / d omega
        D = sp.diags(w, 0, format="csr")
        dt = deps_tables(p, mdl.eps_nu)
        tab = {k: v * w for k, v in dt.items()}
        return sp.bmat([[D, Z], [Z, D]], format="csr") - _F_from(mdl, tab)
    if name == "kappa1":
        return -sp.bmat([[mdl.Qg, Z], [Z, Z]], format="csr")
    if name == "kappa2":
        return -sp.bmat([[Z, Z], [Z, mdl.Qg]], format="csr")
    if name == "lam":
        return -sp.bmat([[Z, mdl.Qu], [mdl.Qu, Z]], format="csr")
    if name == "gap":
        return -sp.bmat([[Z, Z], [Z, I]], format="csr")
    if name in ("lam1", "lam2"):
        key = (1, "e") if name == "lam1" else (2, "o")
        return -_F_from(mdl, mdl.tables, dO={key: mdl.Qg})
    return -_F_from(mdl, dparam_tables(p, mdl.eps_nu, name))


def dphi_dp(mdl, v, mu, name, v_i):
    """d Phi^{v mu} / d(name); eps_v = E - E_v = eps_i + E_{v_i} - E_v."""
    p = mdl.p
    eps = mdl.E - m2.vib_energy(p, v)
    ev = mdl.unit(v)
    parts = []
    for d in (1, 2):
        A, B, l = m2.widths_of(p)[(d, mu)]
        f = float(ls.coupling_f(np.array([eps]), A, B, l)[0])
        O = mdl.O[(d, mu)]
        Oe = O @ ev
        if name == "A%d%s" % (d, mu):
            df = f / (2 * A)
            parts.append(df * Oe)
        elif name == "B%d%s" % (d, mu):
            parts.append(f * eps / (2 * B * B) * Oe)
        elif name in ("omega_g", "omega_u") and eps > 0:
            de = (v_i[0] - v[0]) if name == "omega_g" else (v_i[1] - v[1])
            fp = f * ((l + 0.5) / (2 * eps) - 1 / (2 * B))
            parts.append(fp * de * Oe)
        elif (name == "lam1" and (d, mu) == (1, "e")) or (name == "lam2" and (d, mu) == (2, "o")):
            parts.append(f * (mdl.Qg @ ev))
        else:
            parts.append(np.zeros(mdl.n))
    return np.concatenate(parts)


def forward(p, Ng, Nu, eps_list, v_i, finals, solver=lu_solve):
    """sigma[e, f] summed over mu_i, mu_f, plus the per-(e, mu_i) pieces."""
    sig = np.zeros((len(eps_list), len(finals)))
    pieces = []
    for e_idx, eps_i in enumerate(eps_list):
        E = m2.total_energy(p, eps_i, v_i)
        mdl = m2.Model2D(p, Ng, Nu, E)
        A = mdl.matrix()
        c = sigma_prefactor(eps_i)
        for mu_i in m2.MU:
            psi = solver(A, mdl.phi(v_i, mu_i))
            T = np.array([[mdl.phi(vf, mf) @ psi for mf in m2.MU] for vf in finals])
            sig[e_idx] += c * np.sum(np.abs(T) ** 2, axis=1)
            pieces.append((e_idx, mu_i, mdl, A, psi, T, c))
    return sig, pieces


def loss(p, Ng, Nu, eps_list, v_i, finals, sigma_target, solver=lu_solve):
    sig, _ = forward(p, Ng, Nu, eps_list, v_i, finals, solver)
    return float(np.sum((sig - sigma_target) ** 2)), sig


def loss_and_grad(p, Ng, Nu, eps_list, v_i, finals, sigma_target, dense=False):
    """(L, dL/dp in PARAM_NAMES order, sigma)."""
    solver = (lambda A, b: lu_solve(A.toarray(), b)) if dense else lu_solve
    sig, pieces = forward(p, Ng, Nu, eps_list, v_i, finals, solver)
    gsig = 2.0 * (sig - sigma_target)
    L = float(np.sum((sig - sigma_target) ** 2))
    grad = np.zeros(len(PARAM_NAMES))
    for (e_idx, mu_i, mdl, A, psi, T, c) in pieces:
        W = 2.0 * c * gsig[e_idx][:, None] * np.conj(T)           # [n_final, 2]
        rhs = np.zeros(2 * mdl.n, dtype=complex)
        for fi, vf in enumerate(finals):
            for mi, mf in enumerate(m2.MU):
                rhs += W[fi, mi] * mdl.phi(vf, mf)
        zeta = solver(A, rhs)
        for k, name in enumerate(PARAM_NAMES):
            tot = -(zeta @ (dA_dp(mdl, name, v_i) @ psi))
            tot += zeta @ dphi_dp(mdl, v_i, mu_i, name, v_i)
            for fi, vf in enumerate(finals):
                for mi, mf in enumerate(m2.MU):
                    if W[fi, mi] != 0:
                        tot += W[fi, mi] * (dphi_dp(mdl, vf, mf, name, v_i) @ psi)
            grad[k] += tot.real
    return L, grad, sig


def finite_difference_grad(p, Ng, Nu, eps_list, v_i, finals, sigma_target, h=1e-6, names=None):
    """Central differences with relative step h: p_k (1 +- h)."""
    from .model2d import PARAM_NAMES as names_all
    names = names or names_all
    out = {}
    for name in names:
        step = h * p[name]
        pp, pm = dict(p), dict(p)
        pp[name] = p[name] + step
        pm[name] = p[name] - step
        lp, _ = loss(pp, Ng, Nu, eps_list, v_i, finals, sigma_target)
        lm, _ = loss(pm, Ng, Nu, eps_list, v_i, finals, sigma_target)
        out[name] = (lp - lm) / (2 * step)
    return out
