"""Seeded synthetic workloads: model parameters and job lists.

This module only draws and lists inputs; it holds none of the method's
arithmetic and imports nothing from the solver or from the oracle, so both
sides (and the tests) can take their inputs from here.

Base model: the generalized two-state model of Sec. II.C with
w_g = 0.15, w_u = 0.10 eV, k_1 = -0.1, k_2 = +0.1, lam = lam_1 = lam_2 = 0.05,
E_1 = 1.0 eV, gap E_2 - E_1 = 0.5 eV, all four widths A = 0.2, B = 1.0 with
l = 0 for the even and l = 1 for the odd partial wave (the l pattern of
Table II), level shift on a 4096-node square-root grid up to 40 eV.
"""
import numpy as np

PARAM_NAMES = ("omega_g", "omega_u", "kappa1", "kappa2", "lam", "lam1", "lam2", "gap",
               "A1e", "A2e", "A1o", "A2o", "B1e", "B2e", "B1o", "B2o")

SEED = 20230725


def base_params():
    return dict(omega_g=0.15, omega_u=0.10, kappa1=-0.1, kappa2=0.1, lam=0.05,
                lam1=0.05, lam2=0.05, gap=0.5,
                A1e=0.2, A2e=0.2, A1o=0.2, A2o=0.2,
                B1e=1.0, B2e=1.0, B1o=1.0, B2o=1.0,
                E1=1.0, l_e=0, l_o=1, K=4096, X=40.0)


def draw_params(seed, base=None):
    """Each of the 16 continuous parameters times U(0.8, 1.2), in PARAM_NAMES
    order, from numpy's default_rng(seed); E1, l and the grid stay fixed."""
    p = dict(base or base_params())
    rng = np.random.default_rng(seed)
    fac = rng.uniform(0.8, 1.2, size=len(PARAM_NAMES))
    for name, f in zip(PARAM_NAMES, fac):
        p[name] = p[name] * float(f)
    return p


def params_vector(p):
    return np.array([p[k] for k in PARAM_NAMES], dtype=np.float64)


def params_from_vector(vec, like):
    p = dict(like)
    for k, v in zip(PARAM_NAMES, vec):
        p[k] = float(v)
    return p


# ---- job lists ----------------------------------------------------------
# A job is (eps_i, (n_g, n_u) of v_i, mu_i) with mu_i in {0: even, 1: odd}.
# Vibrational labels v = 0, 1, 2, ... denote the tuning-mode progression
# (n_g = v, n_u = 0).

def single_jobs():
    """One energy eps_i = 1.0 eV, v_i = 0, both partial waves; 40 x 40 basis."""
    return dict(params=base_params(), Ng=40, Nu=40,
                jobs=[(1.0, (0, 0), 0), (1.0, (0, 0), 1)],
                finals=[(k, 0) for k in range(6)])


def batched_jobs(n_energies=512, n_basis=120, seed=SEED):
    """512 energies on [0.1, 3.0] eV x v_i in {0,1,2} x mu in {e, o}, one
    parameter draw; 120 x 120 basis per state (28800 unknowns)."""
    p = draw_params(seed)
    eps = np.linspace(0.1, 3.0, n_energies)
    jobs = [(float(e), (v, 0), mu) for e in eps for v in range(3) for mu in range(2)]
    return dict(params=p, Ng=n_basis, Nu=n_basis, jobs=jobs,
                finals=[(k, 0) for k in range(6)])


def uneven_instances(n_inst=64, seed=SEED + 3, nmin=40, nmax=160):
    """64 instances, each with its own parameter draw, an n x n basis with
    n ~ U{40..160} and one energy eps_i ~ U[0.1, 3.0]; v_i = 0, both mu."""
    rng = np.random.default_rng(seed)
    out = []
    for k in range(n_inst):
        n = int(rng.integers(nmin, nmax + 1))
        e = float(rng.uniform(0.1, 3.0))
        out.append(dict(params=draw_params(seed * 1000 + k), Ng=n, Nu=n, eps=e))
    return out


def adjoint_workload(n_energies=256, n_basis=120, seed=SEED):
    """Model at the base parameters, 256 energies on [0.1, 3.0] eV, v_i = 0,
    finals v_f = 0..5; the target spectrum comes from a second draw (seed+1)."""
    return dict(params=base_params(), target_params=draw_params(seed + 1),
                Ng=n_basis, Nu=n_basis, eps=np.linspace(0.1, 3.0, n_energies),
                v_i=(0, 0), finals=[(k, 0) for k in range(6)])



# ---------------------------------------------------------------- ECD86 model

def ecd86_params():
    """The pseudo Jahn-Teller model of Estrada, Cederbaum and Domcke with the
    values of Table I, in this descriptor: couplings to the continuum
    independent of the coordinates (lam1 = lam2 = 0), state 1 coupled only to
    the even wave and state 2 only to the odd one (no width for (2, e) and
    (1, o)), l = 2 for the even and l = 1 for the odd wave; the width
    a eps^(l+1/2) exp(-b eps) is A = a, B = 1/b.  B2e and B1o only stand in
    for the absent widths."""
    return dict(omega_g=0.258, omega_u=0.091, kappa1=-0.212, kappa2=0.254, lam=0.318,
                lam1=0.0, lam2=0.0, gap=2.85 - 2.45,
                A1e=0.086, A2e=0.0, A1o=0.0, A2o=0.186,
                B1e=1.0 / 0.833, B2e=1.0, B1o=1.0, B2o=1.0 / 0.375,
                E1=2.45, l_e=2, l_o=1, K=4096, X=40.0)


def ecd86_jobs(n_energies=256, n_basis=60):
    """256 energies on [0.1, 5.0] eV x mu in {e, o} from v_i = 0, finals
    v_f = 0..5; 60 x 60 basis per state (the cross sections change by less
    than 1e-6 relative from 60 to 100 per mode up to 4 eV)."""
    eps = np.linspace(0.1, 5.0, n_energies)
    jobs = [(float(e), (0, 0), mu) for e in eps for mu in range(2)]
    return dict(params=ecd86_params(), Ng=n_basis, Nu=n_basis, jobs=jobs,
                finals=[(k, 0) for k in range(6)])

# ---------------------------------------------------------------- CO2-like model
#
# Three states (sigma, Pi_x, Pi_y), four modes (symmetric stretch s, bend x and
# y, asymmetric stretch a), partial waves s, p_x, p_y; CO2-like frequencies and
# state energies, couplings drawn per seed.

CO2_SIZES = dict(s=24, x=24, y=24, a=8)


def co2like_params(seed=SEED + 2):
    """Frequencies w_s = 0.172, w_b = 0.083, w_a = 0.291 eV, E_sigma = 0.5,
    E_pi = 3.5 eV; linear couplings k_sigma, k_pi, c_sp with magnitude
    10^U(-3, -1) eV and a random sign; quadratic ones (g*_*, c_rt) with
    magnitude 10^U(-3, -2) eV and a random sign; the dimensionless factors
    c_sp2, l_sigma, l_pi with magnitude 10^U(-2, log10 0.2) and a random sign;
    h_sigma, h_pi ~ U(0.5, 1.5); widths A = 0.2 U(0.8, 1.2), B = 1.0 U(0.8, 1.2)
    for each (state class, wave class); numpy default_rng(seed), in that order."""
    p = dict(omega_s=0.172, omega_b=0.083, omega_a=0.291, E_sigma=0.5, E_pi=3.5, K=4096, X=40.0)
    rng = np.random.default_rng(seed)
    for k in ("k_sigma", "k_pi", "c_sp"):
        p[k] = float(rng.choice((-1.0, 1.0)) * 10.0 ** rng.uniform(-3.0, -1.0))
    for k in ("gs_sigma", "gb_sigma", "ga_sigma", "gs_pi", "gb_pi", "ga_pi", "c_rt"):
        p[k] = float(rng.choice((-1.0, 1.0)) * 10.0 ** rng.uniform(-3.0, -2.0))
    for k in ("c_sp2", "l_sigma", "l_pi"):
        p[k] = float(rng.choice((-1.0, 1.0)) * 10.0 ** rng.uniform(-2.0, np.log10(0.2)))
    for k in ("h_sigma", "h_pi"):
        p[k] = float(rng.uniform(0.5, 1.5))
    for c in ("sigma", "pi"):
        for w in ("s", "p"):
            p["A_%s_%s" % (c, w)] = float(0.2 * rng.uniform(0.8, 1.2))
            p["B_%s_%s" % (c, w)] = float(1.0 * rng.uniform(0.8, 1.2))
    return p


def co2like_jobs(n_energies=128, sizes=None, seed=SEED + 2):
    """128 incident energies on [0.05, 4.0] eV, v_i = 0, partial waves s, p_x,
    p_y: 384 right-hand sides."""
    eps = np.linspace(0.05, 4.0, n_energies)
    jobs = [(float(e), (0, 0, 0, 0), mu) for e in eps for mu in (0, 1, 2)]
    return dict(params=co2like_params(seed), sizes=dict(sizes or CO2_SIZES), jobs=jobs,
                finals=[(v, 0, 0, 0) for v in range(4)] + [(0, 2, 0, 0), (0, 0, 0, 2)])


# ---------------------------------------------------------------- term lists
#
# Models written as polynomial term lists (the general descriptor): a dict
# with omega [M], nbasis [M], e_state [D], uterms / vterms as lists of
# (d, d' or mu, coeff, powers [M]), width {(d, mu): (A, B)}, l [P], K, X.

def terms_from_2d(p, Ng, Nu):
    """The generalized two-state model (modes g, u; waves e, o) as terms."""
    return dict(omega=[p["omega_g"], p["omega_u"]], nbasis=[Ng, Nu],
                e_state=[p["E1"], p["E1"] + p["gap"]],
                uterms=[(0, 0, p["kappa1"], [1, 0]), (1, 1, p["kappa2"], [1, 0]),
                        (0, 1, p["lam"], [0, 1])],
                vterms=[(0, 0, 1.0, [0, 0]), (0, 0, p["lam1"], [1, 0]), (1, 0, 1.0, [0, 1]),
                        (0, 1, 1.0, [0, 1]), (1, 1, 1.0, [0, 0]), (1, 1, p["lam2"], [1, 0])],
                width={(0, 0): (p["A1e"], p["B1e"]), (1, 0): (p["A2e"], p["B2e"]),
                       (0, 1): (p["A1o"], p["B1o"]), (1, 1): (p["A2o"], p["B2o"])},
                l=[p["l_e"], p["l_o"]], K=p["K"], X=p["X"])


def terms_from_co2(p, sizes):
    """The CO2-like model (states sigma, Pi_x, Pi_y; modes s, x, y, a;
    waves s, p_x, p_y) as terms."""
    def m(s=0, x=0, y=0, a=0):
        return [s, x, y, a]
    u = [(0, 0, p["k_sigma"], m(s=1)), (0, 0, p["gs_sigma"], m(s=2)), (0, 0, p["gb_sigma"], m(x=2)),
         (0, 0, p["gb_sigma"], m(y=2)), (0, 0, p["ga_sigma"], m(a=2))]
    for d, sgn in ((1, 1.0), (2, -1.0)):
        u += [(d, d, p["k_pi"], m(s=1)), (d, d, p["gs_pi"], m(s=2)), (d, d, p["gb_pi"], m(x=2)),
              (d, d, p["gb_pi"], m(y=2)), (d, d, p["ga_pi"], m(a=2)),
              (d, d, sgn * p["c_rt"], m(x=2)), (d, d, -sgn * p["c_rt"], m(y=2))]
    u += [(1, 2, 2.0 * p["c_rt"], m(x=1, y=1)),
          (0, 1, p["c_sp"], m(x=1)), (0, 1, p["c_sp"] * p["c_sp2"], m(s=1, x=1)),
          (0, 2, p["c_sp"], m(y=1)), (0, 2, p["c_sp"] * p["c_sp2"], m(s=1, y=1))]
    v = [(0, 0, 1.0, m()), (0, 0, p["l_sigma"], m(s=1)), (1, 0, p["h_pi"], m(x=1)),
         (2, 0, p["h_pi"], m(y=1)), (0, 1, p["h_sigma"], m(x=1)), (1, 1, 1.0, m()),
         (1, 1, p["l_pi"], m(s=1)), (0, 2, p["h_sigma"], m(y=1)), (2, 2, 1.0, m()),
         (2, 2, p["l_pi"], m(s=1))]
    width = {}
    for d, c in ((0, "sigma"), (1, "pi"), (2, "pi")):
        for mu, w in ((0, "s"), (1, "p"), (2, "p")):
            width[(d, mu)] = (p["A_%s_%s" % (c, w)], p["B_%s_%s" % (c, w)])
    return dict(omega=[p["omega_s"], p["omega_b"], p["omega_b"], p["omega_a"]],
                nbasis=[sizes["s"], sizes["x"], sizes["y"], sizes["a"]],
                e_state=[p["E_sigma"], p["E_pi"], p["E_pi"]], uterms=u, vterms=v, width=width,
                l=[0, 1, 1], K=p["K"], X=p["X"])


def quartic_model(seed=SEED + 4, nbasis=(14, 11, 6)):
    """A third model of the class, with the higher-order terms the paper's CO2
    model has (Sec. III.C): three states, three modes (w = 0.12, 0.09, 0.2
    eV), two partial waves (l = 0, 1).  U: state energies 0.9, 1.6, 2.4 eV,
    linear, quadratic and quartic terms on the diagonal, the states coupled
    by q_1, q_0 q_1 and q_2^2; O: 1 + a q_0 + b q_0^2 for state 0 in the
    first wave, q_1 and q_0 q_2 for the others.  Coefficient magnitudes
    10^U(-3, -1) eV (linear), 10^U(-3, -2) (quadratic, cross), 10^U(-4, -3)
    (quartic), random signs; widths A = 0.2 U(0.5, 1.5), B = U(0.8, 1.2)."""
    rng = np.random.default_rng(seed)

    def c(lo, hi):
        return float(rng.choice((-1.0, 1.0)) * 10.0 ** rng.uniform(lo, hi))
    u = [(0, 0, c(-3, -1), [1, 0, 0]), (0, 0, c(-3, -2), [2, 0, 0]), (0, 0, c(-4, -3), [4, 0, 0]),
         (1, 1, c(-3, -1), [1, 0, 0]), (1, 1, c(-3, -2), [0, 2, 0]), (1, 1, c(-4, -3), [0, 4, 0]),
         (2, 2, c(-3, -1), [0, 0, 1]), (2, 2, c(-4, -3), [2, 2, 0]),
         (0, 1, c(-3, -1), [0, 1, 0]), (0, 1, c(-3, -2), [1, 1, 0]), (1, 2, c(-3, -2), [0, 0, 2]),
         (0, 2, c(-3, -2), [1, 0, 1])]
    v = [(0, 0, 1.0, [0, 0, 0]), (0, 0, c(-2, -1), [1, 0, 0]), (0, 0, c(-3, -2), [2, 0, 0]),
         (1, 0, 1.0, [0, 1, 0]), (2, 0, 0.7, [1, 0, 1]),
         (1, 1, 1.0, [0, 0, 0]), (1, 1, c(-2, -1), [0, 0, 1]), (0, 1, 0.8, [0, 1, 0])]
    width = {}
    for d in range(3):
        for mu in range(2):
            width[(d, mu)] = (float(0.2 * rng.uniform(0.5, 1.5)), float(rng.uniform(0.8, 1.2)))
    return dict(omega=[0.12, 0.09, 0.2], nbasis=list(nbasis), e_state=[0.9, 1.6, 2.4],
                uterms=u, vterms=v, width=width, l=[0, 1], K=4096, X=40.0)
