"""Widths and the level-shift integral transform (oracle; test infrastructure).

Paper: Sec. II.B, Eq. (19) defines the transform
    F[f](eps) = int f(x) / (eps - x + i eta) dx
              = PV int f(x)/(eps - x) dx  -  i pi f(eps),
Eq. (20)/(22) the width shape  2 pi |f_d^mu|^2 = Gamma = a eps^(l+1/2) exp(-b eps),
written here with b = 1/B.  For the generalized model (Sec. II.C) the
transform is applied to products f_d^mu f_d'^mu = sqrt(Gamma_d Gamma_d') / 2pi
(f >= 0 by convention), Eq. (23).

Reading of "discrete Hilbert transform on a 4096-point grid": the real part
Delta(eps) = PV int L(x)/(eps - x) dx / (2 pi), where L is the piecewise-linear
interpolant of g = sqrt(Gamma_d Gamma_d') on the square-root-spaced nodes
x_k = (k sqrt(X)/(K-1))^2, k = 0..K-1.  The integral of a linear function
against 1/(eps - x) over one segment is elementary; the oracle sums those
segment integrals one by one.  The imaginary part is the analytic
-pi f_d f_d' theta(eps) = -g(eps)/2 (Gamma = 0 for eps <= 0, Sec. II.A: the
continuum starts at eps = 0).
"""
import numpy as np

HARTREE_EV = 27.211386245988


def width(eps, A, B, l):
    """Gamma(eps) = A eps^(l+1/2) exp(-eps/B) for eps > 0, else 0 (Eq. (22))."""
    eps = np.asarray(eps, dtype=np.float64)
    out = np.zeros_like(eps)
    m = eps > 0
    out[m] = A * eps[m] ** (l + 0.5) * np.exp(-eps[m] / B)
    return out


def coupling_f(eps, A, B, l):
    """f(eps) = +sqrt(Gamma(eps) / 2 pi), the sign convention f >= 0."""
    return np.sqrt(width(eps, A, B, l) / (2.0 * np.pi))


def grid_nodes(K=4096, X=40.0):
    """Square-root-spaced product-integration nodes on [0, X]."""
    k = np.arange(K, dtype=np.float64)
    return (k * np.sqrt(X) / (K - 1)) ** 2


def pair_g(x, A1, B1, A2, B2, l):
    """g(x) = sqrt(Gamma_1(x) Gamma_2(x)) for two widths with the same l."""
    return np.sqrt(width(x, A1, B1, l) * width(x, A2, B2, l))


def pv_linear_segments(eps, x, g):
    """PV int_{x_0}^{x_{K-1}} L(t)/(eps - t) dt for the piecewise-linear L.

    On segment [x_k, x_{k+1}] with slope s_k, L(t) = L_k(eps) - s_k (eps - t),
    where L_k(eps) = g_k + s_k (eps - x_k) is the segment's line at eps, so
        int L/(eps - t) dt = L_k(eps) ln|(eps - x_k)/(eps - x_{k+1})| - s_k h_k.
    At an exact node the two logarithms of the neighbouring segments carry
    equal and opposite coefficients (principal value), so ln|0| is taken as 0.
    """
    eps = np.atleast_1d(np.asarray(eps, dtype=np.float64))
    xk, xk1 = x[:-1], x[1:]
    h = xk1 - xk
    s = (g[1:] - g[:-1]) / h
    out = np.empty(eps.shape, dtype=np.float64)
    for i, e in enumerate(eps.ravel()):
        ta = e - xk
        tb = e - xk1
        la = np.where(ta == 0.0, 0.0, np.log(np.abs(np.where(ta == 0.0, 1.0, ta))))
        lb = np.where(tb == 0.0, 0.0, np.log(np.abs(np.where(tb == 0.0, 1.0, tb))))
        line = g[:-1] + s * ta
        out.flat[i] = np.sum(line * (la - lb) - s * h)
    return out


def level_shift(eps, A1, B1, A2, B2, l, K=4096, X=40.0):
    """Complex F[f_1 f_2](eps) = Delta(eps) - i g(eps)/2 for one pair of widths.

    Delta = PV int L(x)/(eps-x) dx / 2pi on the K-node grid (reading above).
    """
    x = grid_nodes(K, X)
    g = pair_g(x, A1, B1, A2, B2, l)
    re = pv_linear_segments(eps, x, g) / (2.0 * np.pi)
    im = -0.5 * pair_g(np.atleast_1d(np.asarray(eps, dtype=np.float64)), A1, B1, A2, B2, l)
    return re + 1j * im


def level_shift_table(eps, A1, B1, A2, B2, l, g_override=None, K=4096, X=40.0):
    """Same as level_shift but lets the caller replace g by another sampled
    function of x (used for parameter derivatives: the transform is linear in g)."""
    x = grid_nodes(K, X)
    if g_override is None:
        gx = pair_g(x, A1, B1, A2, B2, l)
        ge = pair_g(np.atleast_1d(np.asarray(eps, dtype=np.float64)), A1, B1, A2, B2, l)
    else:
        gx = g_override(x)
        ge = g_override(np.atleast_1d(np.asarray(eps, dtype=np.float64)))
    re = pv_linear_segments(eps, x, gx) / (2.0 * np.pi)
    return re - 0.5j * ge


def dpv_linear_segments_deps(eps, x, g):
    """d/d eps of pv_linear_segments, segment by segment.

    d/d eps [L_k(eps) (ln|eps-x_k| - ln|eps-x_{k+1}|)]
        = s_k (ln|eps-x_k| - ln|eps-x_{k+1}|) + L_k(eps) (1/(eps-x_k) - 1/(eps-x_{k+1})).
    The second term at a node again pairs with the neighbouring segment:
    L_k(x_k) = g_k = L_{k-1}(x_k), so the 1/0 terms cancel and are dropped.
    """
    eps = np.atleast_1d(np.asarray(eps, dtype=np.float64))
    xk, xk1 = x[:-1], x[1:]
    h = xk1 - xk
    s = (g[1:] - g[:-1]) / h
    out = np.empty(eps.shape, dtype=np.float64)
    for i, e in enumerate(eps.ravel()):
        ta = e - xk
        tb = e - xk1
        za, zb = ta == 0.0, tb == 0.0
        la = np.where(za, 0.0, np.log(np.abs(np.where(za, 1.0, ta))))
        lb = np.where(zb, 0.0, np.log(np.abs(np.where(zb, 1.0, tb))))
        ia = np.where(za, 0.0, 1.0 / np.where(za, 1.0, ta))
        ib = np.where(zb, 0.0, 1.0 / np.where(zb, 1.0, tb))
        line = g[:-1] + s * ta
        out.flat[i] = np.sum(s * (la - lb) + line * (ia - ib))
    return out
