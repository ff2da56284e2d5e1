"""GPU parity of the term-list model (vdc_model_create / vdc_model_apply /
vdc_model_solve / vdc_sum_partial_waves):

  * the two-state and CO2-like models written as terms reproduce the
    specialised operators (vdc_matvec, vdc_co2_apply) - both FP64, in a
    different order, and with level-shift tables from the same transform
    evaluated on other points of a wave (so far/near node clusters may
    differ): within 1e-14 |A| |x| plus the tables' rounding bound (64 ulp of
    the transform's sum of magnitudes) pushed through |O|^T diag |O|;
  * a third model with quartic and cross terms against the oracle assembled
    from the same term list (operator with the same bound; solves: oracle
    residual <= 1e-10 + 1e-13, amplitudes within 1e-8 of LU);
  * dispatch of two-state term lists to the two-state kernels;
  * the mu_i sum of Eq. (16) in the library."""
import math

import numpy as np
import pytest
import scipy.sparse as sp

from oracle import levelshift as ls
from oracle import model2d as m2
from oracle import poly
from oracle import solvers
from oracle import terms
from paper_2307_13483_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def vdc():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2307_13483_amd import vdc as v
    v.lib()
    return v


def _table_bound(desc, eps, mu, d, e):
    A1, B1 = desc["width"][(d, mu)]
    A2, B2 = desc["width"][(e, mu)]
    l = desc["l"][mu]
    x = ls.grid_nodes(desc["K"], desc["X"])
    g = ls.pair_g(x, A1, B1, A2, B2, l)
    s = np.diff(g) / np.diff(x)
    c = np.concatenate([[s[0]], np.diff(s), [-s[-1]]])
    out = np.empty(len(eps))
    for k, ev in enumerate(eps):
        t = ev - x
        psi = np.abs(t * np.log(np.abs(np.where(t == 0, 1.0, t))))
        out[k] = 64 * 2.2e-16 * np.sum(np.abs(c) * psi) / (2 * np.pi) + 1e-15
    return out


def _bound(desc, E, x):
    """1e-14 |A| |x| + sum_mu |O_d|^T diag(table bound) |O_e| |x_e| per block."""
    tm = terms.TermModel(desc, E)
    A = tm.matrix()
    ax = np.abs(x)
    n = tm.n
    b = 1e-14 * (abs(A) @ ax) + 1e-15
    for d in range(tm.D):
        for e in range(tm.D):
            for mu in range(tm.P):
                Od, Oe = tm.O.get((d, mu)), tm.O.get((e, mu))
                if Od is None or Oe is None or (mu, min(d, e), max(d, e)) not in tm.tables:
                    continue
                tb = _table_bound(desc, tm.eps_nu, mu, d, e)
                b[d * n:(d + 1) * n] += abs(Od).T @ (tb * (abs(Oe) @ ax[e * n:(e + 1) * n]))
    return A, b


@pytest.mark.parametrize("Ng,Nu,seed", [(1, 1, 0), (7, 5, 2), (33, 20, 4)])
def test_two_state_terms_reproduce_the_two_state_operator(vdc, Ng, Nu, seed):
    import torch
    p = inputs.draw_params(seed)
    desc = inputs.terms_from_2d(p, Ng, Nu)
    gm = vdc.TermModel(desc)
    assert gm.kind() == 1
    sm = vdc.Model2D(p, Ng, Nu)
    rng = np.random.default_rng(seed)
    lab = m2.parity_of(Ng, Nu)
    E = 2.3
    xs = []
    for parity in (0, 1):
        x = rng.standard_normal(2 * Ng * Nu) + 1j * rng.standard_normal(2 * Ng * Nu)
        x[lab != (1.0 if parity == 0 else -1.0)] = 0.0
        xs.append(x)
    X = torch.tensor(np.array(xs))
    yg = vdc.model_apply(gm, E, X).cpu().numpy()
    ys = vdc.matvec(sm, E, X, [0, 1]).cpu().numpy()
    for k in range(2):
        A, b = _bound(desc, E, xs[k])
        assert np.all(np.abs(yg[k] - ys[k]) <= b), np.max(np.abs(yg[k] - ys[k]) / b)
        assert np.all(np.abs(yg[k] - A @ xs[k]) <= b)


def _co2_full_index(sizes, px, py):
    Ns, Nx, Ny, Na = (sizes[k] for k in ("s", "x", "y", "a"))
    n = Ns * Nx * Ny * Na
    s, a, x, y = np.meshgrid(np.arange(Ns), np.arange(Na), np.arange(Nx), np.arange(Ny),
                             indexing="ij")
    t = ((x + px) & 1) | (((y + py) & 1) << 1)
    return np.where(t != 3, t * n + ((s * Nx + x) * Ny + y) * Na + a, -1).ravel()


@pytest.mark.parametrize("sizes,eps", [(dict(s=4, x=5, y=6, a=3), 1.7), (dict(s=2, x=9, y=4, a=2), 3.1)])
def test_co2_terms_reproduce_the_co2_operator(vdc, sizes, eps):
    import torch
    p = inputs.co2like_params()
    desc = inputs.terms_from_co2(p, sizes)
    gm = vdc.TermModel(desc)
    cm = vdc.Co2Model(p, sizes)
    E = poly.total_energy(p, eps, (0, 0, 0, 0))
    rng = np.random.default_rng(5)
    n = gm.npts
    for (px, py) in ((0, 0), (1, 0), (0, 1), (1, 1)):
        idx = _co2_full_index(sizes, px, py)
        z = rng.standard_normal(idx.size) + 1j * rng.standard_normal(idx.size)
        z[idx < 0] = 0
        full = np.zeros(3 * n, dtype=complex)
        full[idx[idx >= 0]] = z[idx >= 0]
        yc = vdc.co2_apply(cm, E, z[None], [(px, py)]).cpu().numpy()[0]
        yc_full = np.zeros(3 * n, dtype=complex)
        yc_full[idx[idx >= 0]] = yc[idx >= 0]
        yg = vdc.model_apply(gm, E, torch.tensor(full[None])).cpu().numpy()[0]
        A, b = _bound(desc, E, full)
        assert np.all(np.abs(yg - yc_full) <= b), (px, py)
        assert np.all(np.abs(yg - A @ full) <= b), (px, py)


@pytest.mark.parametrize("nbasis", [(1, 1, 1), (5, 3, 2), (14, 11, 6)])
def test_quartic_model_operator_matches_oracle(vdc, nbasis):
    import torch
    desc = inputs.quartic_model(nbasis=nbasis)
    gm = vdc.TermModel(desc)
    rng = np.random.default_rng(7)
    N = 3 * int(np.prod(nbasis))
    X = rng.standard_normal((3, N)) + 1j * rng.standard_normal((3, N))
    for E in (0.4, 1.9, 3.3):
        Y = vdc.model_apply(gm, E, torch.tensor(X)).cpu().numpy()
        for k in range(3):
            A, b = _bound(desc, E, X[k])
            assert np.all(np.abs(Y[k] - A @ X[k]) <= b), (E, k)


def _check_solves(desc, jobs, finals, T, sig, psi, infos, P):
    for k, (eps_i, vi, mu) in enumerate(jobs):
        assert infos[k]["status"] == 0, infos[k]
        E = terms.total_energy(desc, eps_i, vi)
        tm = terms.TermModel(desc, E)
        A = tm.matrix()
        b = tm.phi(vi, mu)
        N = A.shape[0]
        res = np.linalg.norm(b - A @ psi[k][:N]) / np.linalg.norm(b)
        assert res <= 1e-10 + 1e-13, (k, res)
        ref = solvers.lu_solve(A, b)
        assert np.linalg.norm(psi[k][:N] - ref) <= 1e-8 * np.linalg.norm(ref)
        Tref = np.array([[tm.phi(vf, mf) @ ref for mf in range(P)] for vf in finals])
        assert np.max(np.abs(T[k][:, :P] - Tref)) <= 1e-8 * np.max(np.abs(Tref))
        pref = 2 * math.pi ** 3 / (eps_i / ls.HARTREE_EV)
        assert np.allclose(sig[k], pref * np.sum(np.abs(T[k]) ** 2, axis=1), rtol=1e-12, atol=0)


@pytest.mark.parametrize("method,precond", [("gmres", 1), ("cocg", 1), ("gmres", 0)])
def test_quartic_model_solves_match_oracle(vdc, method, precond):
    desc = inputs.quartic_model()
    gm = vdc.TermModel(desc)
    jobs = [(0.35, (0, 0, 0), 0), (1.2, (1, 0, 0), 1), (2.6, (0, 1, 0), 0), (1.9, (0, 0, 1), 1)]
    finals = [(0, 0, 0), (1, 0, 0), (0, 1, 0), (2, 0, 1)]
    opts = vdc.Opts(restart=30, precond=precond, max_iter=20000, tol=1e-10,
                    method=vdc.COCG if method == "cocg" else vdc.GMRES)
    T, sig, psi, infos = vdc.model_solve(gm, jobs, finals, opts, want_psi=True)
    _check_solves(desc, jobs, finals, T.cpu().numpy(), sig.cpu().numpy(), psi.cpu().numpy(),
                  infos, 2)


def test_two_term_models_in_one_launch(vdc):
    """Jobs of two term-list models of different sizes (and a CO2-like one
    with three partial waves) in one persistent launch."""
    d1 = inputs.quartic_model(nbasis=(9, 7, 4))
    d2 = inputs.quartic_model(seed=inputs.SEED + 5, nbasis=(6, 5, 3))
    d3 = inputs.terms_from_co2(inputs.co2like_params(), dict(s=3, x=4, y=4, a=2))
    models = [vdc.TermModel(d) for d in (d1, d2, d3)]
    jobs = [(1.1, (0, 0, 0), 0, 0), (0.8, (1, 0, 0), 1, 1), (2.2, (0, 0, 0, 0), 2, 2),
            (1.5, (0, 0, 0), 1, 0), (1.3, (0, 0, 0, 0), 0, 2)]
    finals = [(0, 0, 0), (1, 0, 0)]
    T, sig, psi, infos = vdc.model_solve(models, jobs, finals,
                                         vdc.Opts(restart=25, precond=vdc.PREC_JACOBI),
                                         want_psi=True)
    T, sig, psi = T.cpu().numpy(), sig.cpu().numpy(), psi.cpu().numpy()
    assert T.shape[2] == 3
    for k, jb in enumerate(jobs):
        desc = (d1, d2, d3)[jb[3]]
        P = len(desc["l"])
        fin = [tuple(list(f) + [0] * (len(desc["nbasis"]) - 3)) for f in finals]
        _check_solves(desc, [jb[:3]], fin, T[k:k + 1], sig[k:k + 1], psi[k:k + 1],
                      infos[k:k + 1], P)
        assert np.all(T[k][:, P:] == 0)


def test_co2_terms_solve_matches_co2_solver(vdc):
    p = inputs.co2like_params()
    sizes = dict(s=3, x=5, y=5, a=2)
    desc = inputs.terms_from_co2(p, sizes)
    gm = vdc.TermModel(desc)
    cm = vdc.Co2Model(p, sizes)
    jobs = [(0.9, (0, 0, 0, 0), 0), (2.4, (0, 0, 0, 0), 1), (3.1, (1, 0, 0, 0), 2)]
    finals = [(0, 0, 0, 0), (1, 0, 0, 0), (0, 2, 0, 0)]
    Tg, sg, _, ig = vdc.model_solve(gm, jobs, finals, vdc.Opts(restart=30, precond=vdc.PREC_JACOBI))
    Tc, sc, _, ic = vdc.co2_solve(cm, jobs, finals, vdc.Opts(restart=20, precision=vdc.FP64,
                                                             precond=vdc.PREC_BLOCK))
    assert all(i["status"] == 0 for i in ig + ic)
    Tg, Tc = Tg.cpu().numpy(), Tc.cpu().numpy()
    assert np.max(np.abs(Tg - Tc)) <= 1e-8 * np.max(np.abs(Tc))


def test_dispatch_to_two_state_kernels(vdc):
    """Two-state term lists with dispatch run on the two-state kernels (kind
    0, every vdc_solve option), and without it on the term-list kernels; the
    amplitudes agree with the two-state model's to the solves' accuracy."""
    p = inputs.draw_params(12)
    Ng, Nu = 24, 20
    desc = inputs.terms_from_2d(p, Ng, Nu)
    fast, gen = vdc.TermModel(desc, dispatch=True), vdc.TermModel(desc, dispatch=False)
    assert fast.kind() == 0 and gen.kind() == 1
    jobs = [(0.7, (0, 0), 0), (1.8, (1, 0), 1), (2.9, (2, 0), 0)]
    finals = [(0, 0), (1, 0), (2, 0)]
    o = vdc.Opts(precond=vdc.PREC_BLOCK, method=vdc.COCG, precision=vdc.FP32_INNER,
                 inner_restart=200, inner_tol=1e-5, max_iter=20000)
    Tf, sf, _, inf_f = vdc.model_solve(fast, jobs, finals, o)
    Tr, sr, _, _ = vdc.solve(vdc.Model2D(p, Ng, Nu), jobs, finals, o)
    Tg, sgn, _, _ = vdc.model_solve(gen, jobs, finals, vdc.Opts(restart=30, precond=vdc.PREC_JACOBI))
    Tf, Tr, Tg = Tf.cpu().numpy(), Tr.cpu().numpy(), Tg.cpu().numpy()
    scale = np.max(np.abs(Tr))
    assert np.max(np.abs(Tf - Tr)) <= 1e-9 * scale
    assert np.max(np.abs(Tg - Tr)) <= 1e-8 * scale
    # a term list that is not the two-state model is not dispatched
    q = dict(desc, uterms=desc["uterms"] + [(0, 0, 0.01, [2, 0])])
    assert vdc.TermModel(q, dispatch=True).kind() == 1


def test_partial_wave_sum_in_the_library(vdc):
    import torch
    p = inputs.draw_params(13)
    model = vdc.Model2D(p, 16, 12)
    eps = [0.6, 1.3, 2.2]
    jobs = [(e, (0, 0), mu) for e in eps for mu in (0, 1)]
    finals = [(0, 0), (1, 0), (2, 0)]
    _, share, _, _ = vdc.solve(model, jobs, finals, vdc.Opts(restart=20))
    sig = vdc.sum_partial_waves([k // 2 for k in range(len(jobs))], len(eps), share)
    ref = share.view(len(eps), 2, len(finals)).sum(dim=1)
    assert torch.equal(sig, ref)
    # against the oracle's cross sections (summed over mu_i and mu_f)
    from oracle import observables as ob
    for k, e in enumerate(eps):
        s_ref = ob.cross_sections(p, 16, 12, e, (0, 0), finals)
        assert np.allclose(sig[k].cpu().numpy(), s_ref, rtol=1e-8, atol=0)
