"""T-matrix and cross sections (oracle; test infrastructure).

Eq. (15)/(24): T_{mu_f v_f <- mu_i v_i} = <Phi^{v_f mu_f} | Psi^{mu_i}_{v_i}>,
with Phi real, so the scalar product is the plain sum Phi_f^T Psi.
Eq. (16)/(24): sigma_{v_f <- v_i} = 2 pi^3 / eps_i  sum_{mu_i mu_f} |T|^2,
in atomic units: eps_i in hartree, sigma in a_0^2 (T is dimensionless since
V ~ energy^(1/2)).
Final channels are open when eps_f = E - E_{v_f} > 0 (Eq. (2)); for a closed
channel f(eps_f) = 0, so Phi_f = 0 and T = 0 without special-casing.
"""
import numpy as np

from .levelshift import HARTREE_EV
from .model2d import Model2D, MU, total_energy
from .solvers import lu_solve


def amplitude(model, psi, v_f, mu_f):
    return complex(model.phi(v_f, mu_f) @ psi)


def sigma_prefactor(eps_i):
    return 2.0 * np.pi ** 3 / (float(eps_i) / HARTREE_EV)


def solve_job(p, Ng, Nu, eps_i, v_i, mu_i, finals, solver=None):
    """One right-hand side (E, v_i, mu_i): Psi, and T for every (v_f, mu_f).

    Returns (psi, T) with T an array [len(finals), 2] over mu_f in (e, o).
    """
    E = total_energy(p, eps_i, v_i)
    mdl = Model2D(p, Ng, Nu, E)
    A = mdl.matrix()
    b = mdl.phi(v_i, mu_i)
    psi = (solver or lu_solve)(A, b)
    T = np.array([[amplitude(mdl, psi, vf, mf) for mf in MU] for vf in finals])
    return psi, T


def cross_sections(p, Ng, Nu, eps_i, v_i, finals, solver=None):
    """sigma_{v_f <- v_i}(eps_i) for each v_f in finals, summed over mu_i, mu_f."""
    tot = np.zeros(len(finals))
    for mu_i in MU:
        _, T = solve_job(p, Ng, Nu, eps_i, v_i, mu_i, finals, solver)
        tot += np.sum(np.abs(T) ** 2, axis=1)
    return sigma_prefactor(eps_i) * tot
