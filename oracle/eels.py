"""Two-dimensional electron energy-loss spectra (oracle; test infrastructure).

Eq. (17): S(eps_i, d) = sum_{v_f} sigma_{v_f <- v_i}(eps_i) rho(d - d_{v_f}), with
the energy loss d_{v_f} = E_{v_f} - E_{v_i} fixed by energy conservation and rho
the spectrometer's resolution, a Gaussian of full width at half maximum w
(10 meV in Sec. II.B), normalised to unit area:
    rho(x) = (2 sqrt(ln 2 / pi) / w) exp(-4 ln 2 x^2 / w^2).
The sum runs over every final state of the basis (closed channels have
sigma = 0).  The contributions of the two right-hand sides mu_i = e, o (the
gerade and ungerade symmetry blocks, Sec. IV) are kept apart: the spectrum
of one right-hand side uses its share of sigma (Eq. (16) without the sum
over mu_i).
"""
import numpy as np

from .model2d import MU, Model2D, total_energy, vib_energy
from .observables import sigma_prefactor
from .solvers import lu_solve


def resolution(x, fwhm=0.010):
    x = np.asarray(x, dtype=np.float64)
    return (2.0 * np.sqrt(np.log(2.0) / np.pi) / fwhm) * np.exp(-4.0 * np.log(2.0) * x * x / fwhm ** 2)


def final_shares(p, Ng, Nu, eps_i, v_i, mu_i, psi=None):
    """This right-hand side's share of sigma_{v_f <- v_i} for every final state
    (n_g, n_u) of the basis, and the energy losses: arrays [Ng, Nu].  psi is
    the full-layout solution (solved by LU when not given)."""
    E = total_energy(p, eps_i, v_i)
    mdl = Model2D(p, Ng, Nu, E)
    if psi is None:
        psi = lu_solve(mdl.matrix(), mdl.phi(v_i, MU[mu_i]))
    sig = np.zeros((Ng, Nu))
    loss = np.zeros((Ng, Nu))
    pref = sigma_prefactor(eps_i)
    for g in range(Ng):
        for u in range(Nu):
            T = [complex(mdl.phi((g, u), mf) @ psi) for mf in MU]
            sig[g, u] = pref * sum(abs(t) ** 2 for t in T)
            loss[g, u] = vib_energy(p, (g, u)) - vib_energy(p, v_i)
    return sig, loss


def spectrum(shares, losses, grid, fwhm=0.010):
    """S on the energy-loss grid: sum over final states of share x rho."""
    shares = np.ravel(shares)
    losses = np.ravel(losses)
    grid = np.asarray(grid, dtype=np.float64)
    return np.array([np.sum(shares * resolution(d - losses, fwhm)) for d in grid])
