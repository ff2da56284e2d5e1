"""The HIP kernels checked on the CPU: the library's own sources built as
host code against the stand-in for HIP in tests/emu (tests/_emulated.py),
every GPU thread a fiber, device memory under AddressSanitizer.  A run
fails on any access outside an allocation (AddressSanitizer aborts), on
threads of a workgroup waiting at different barriers (the runtime aborts),
and on results that miss the oracle: the same acceptance as the GPU parity
tests (true residual <= 1e-10 + rounding, solution and amplitudes within
1e-8 of LU).  What it cannot see: anything of the GPU's own execution
(timing, register allocation, the compiler's GPU code)."""
import math
import os

import numpy as np
import scipy.sparse as sp
import pytest

import _emulated as emu
import _oracle_pool as op
from oracle import levelshift as ls
from oracle import poly
from oracle import solvers
from oracle import terms
from paper_2307_13483_amd import inputs

pytestmark = pytest.mark.skipif(not emu.available(), reason="clang++ of the ROCm toolchain absent")


@pytest.fixture(scope="module")
def exe(tmp_path_factory):
    return emu.build(str(tmp_path_factory.mktemp("emu")), jobs=min(8, os.cpu_count() or 1))


# a ragged multi-model batch: shapes that leave partial tiles, column blocks
# and row sweeps, a 1 x 1 basis, both partial waves
MODELS = [(inputs.draw_params(31), 13, 29), (inputs.draw_params(32), 7, 5),
          (inputs.draw_params(33), 1, 1)]
JOBS = [(0.9, (0, 0), 0, 0), (2.3, (1, 0), 1, 0), (1.3, (0, 0), 1, 1), (2.0, (0, 1), 0, 1),
        (1.7, (0, 0), 0, 2), (2.6, (0, 0), 1, 2)]
FINALS = [(0, 0)]


def _paths():
    from paper_2307_13483_amd import vdc
    return {
        "gmres_block": vdc.Opts(restart=12, precond=vdc.PREC_BLOCK),
        "fgmres_block": vdc.Opts(precision=vdc.FP32_INNER, precond=vdc.PREC_BLOCK, inner_restart=8,
                                 inner_tol=1e-3, outer_restart=8),
        "cocg_rows": vdc.Opts(method=vdc.COCG, precond=vdc.PREC_ROWS),
        "cocg_fp32_block": vdc.Opts(method=vdc.COCG, precision=vdc.FP32_INNER,
                                    precond=vdc.PREC_BLOCK, inner_restart=200, inner_tol=1e-5),
        "cocg_fp32_rows": vdc.Opts(method=vdc.COCG, precision=vdc.FP32_INNER, precond=vdc.PREC_ROWS,
                                   inner_restart=200, inner_tol=1e-5),
        "cocg_fp32_block_checked": vdc.Opts(method=vdc.COCG, precision=vdc.FP32_INNER,
                                            precond=vdc.PREC_BLOCK, inner_restart=200,
                                            inner_tol=1e-5, check_optical=1),
    }


def _solve(exe, tmp_path, opts, **env):
    case, out = str(tmp_path / "case.bin"), str(tmp_path / "out.bin")
    emu.write_solve_case(case, MODELS, JOBS, FINALS, opts)
    rc, text = emu.run(exe, ["solve", case, out], **env)
    assert rc == 0, text[-3000:]
    rows = emu.job_lines(text)
    assert len(rows) == len(JOBS) and all(r[0] == 0 for r in rows), text[-2000:]
    nj, nf = len(JOBS), len(FINALS)
    max_nc = max(Ng * Nu for _, Ng, Nu in MODELS)
    raw = np.fromfile(out, dtype=np.float64)
    T = raw[:4 * nj * nf].view(np.complex128).reshape(nj, nf, 2)
    sig = raw[4 * nj * nf:5 * nj * nf].reshape(nj, nf)
    psi = raw[5 * nj * nf:].view(np.complex128).reshape(nj, 2 * max_nc)
    return T, sig, psi


def _check_against_oracle(T, sig, psi):
    for k, (eps_i, vi, mu, m) in enumerate(JOBS):
        p, Ng, Nu = MODELS[m]
        c = op.check_2d_job(p, Ng, Nu, (eps_i, vi, mu), FINALS, psi[k, :2 * Ng * Nu])
        assert c["res"] <= 1e-10 + 1e-13, (k, c["res"])
        assert c["psi_err"] <= 1e-8, (k, c["psi_err"])
        scale = max(1e-300, np.max(np.abs(c["T"])))
        assert np.max(np.abs(T[k] - c["T"])) <= 1e-8 * scale, k
        pref = 2 * math.pi ** 3 / (eps_i / ls.HARTREE_EV)
        assert np.allclose(sig[k], pref * np.sum(np.abs(T[k]) ** 2, axis=1), rtol=1e-12, atol=0)


@pytest.mark.parametrize("path", ["gmres_block", "fgmres_block", "cocg_rows", "cocg_fp32_block",
                                  "cocg_fp32_rows", "cocg_fp32_block_checked"])
def test_two_state_batch_under_emulation(exe, tmp_path, path):
    """Three models of ragged sizes in one persistent launch on every solver
    kernel: no access outside an allocation, no barrier mismatch, and every
    solve matches the oracle."""
    T, sig, psi = _solve(exe, tmp_path, _paths()[path])
    _check_against_oracle(T, sig, psi)


def test_last_workgroup_slots_under_emulation(exe, tmp_path):
    """The persistent queue taken by the grid's last workgroups (their
    slots end the workspace): the same results, still in bounds."""
    T, sig, psi = _solve(exe, tmp_path, _paths()["cocg_fp32_block"], EMU_CUS=64, EMU_REVERSE=1)
    _check_against_oracle(T, sig, psi)


def _co2_sector_index(sizes, px, py):
    Ns, Nx, Ny, Na = (sizes[k] for k in ("s", "x", "y", "a"))
    n = Ns * Nx * Ny * Na
    s, a, x, y = np.meshgrid(np.arange(Ns), np.arange(Na), np.arange(Nx), np.arange(Ny),
                             indexing="ij")
    t = ((x + px) & 1) | (((y + py) & 1) << 1)
    full = t * n + ((s * Nx + x) * Ny + y) * Na + a
    return np.where(t != 3, full, -1).ravel()


# (s, x, y, a): the march along n_s with no n_a +- 2 neighbour; with both,
# the rings wrapping and more level-shift rows than threads; a plane of
# several wavefronts with a partial last one; a plane past the march's limit
# (the two grid-wide passes)
CO2_SIZES = [dict(s=3, x=5, y=4, a=2), dict(s=7, x=6, y=7, a=6), dict(s=5, x=9, y=11, a=5),
             dict(s=2, x=30, y=30, a=1), dict(s=2, x=35, y=30, a=1)]


@pytest.mark.parametrize("sizes", CO2_SIZES, ids=lambda d: "x".join(str(d[k]) for k in "sxya"))
def test_co2_operator_under_emulation(exe, tmp_path, sizes):
    """The CO2-like operator entry point (the march along n_s, or the two
    grid-wide passes for wide planes) on the four reflection sectors against
    the oracle's assembled matrix, and the bend-plane block factor and apply
    on the same vectors against the oracle's block slices."""
    P = inputs.co2like_params()
    eps = 1.4
    E = poly.total_energy(P, eps, (0, 0, 0, 0))
    M = poly.PolyModel(P, sizes, E)
    A = M.matrix().tocsr()
    n = M.n
    rng = np.random.default_rng(5)
    sectors = [(0, 0), (1, 0), (0, 1), (1, 1)]     # vector v: (v & 1, (v >> 1) & 1)
    xs = []
    for (px, py) in sectors:
        idx = _co2_sector_index(sizes, px, py)
        z = rng.standard_normal(n) + 1j * rng.standard_normal(n)
        z[idx < 0] = 0
        xs.append(z)
    desc, xf = str(tmp_path / "co2.bin"), str(tmp_path / "x.bin")
    emu.write_co2_desc(desc, P, sizes)
    np.array(xs).astype(np.complex128).tofile(xf)
    for which in ((0, 1) if sizes["y"] <= 24 else (0,)):
        out = str(tmp_path / ("y%d.bin" % which))
        rc, text = emu.run(exe, ["co2", desc, xf, "4", str(which), repr(E), out])
        assert rc == 0, text[-3000:]
        y = np.fromfile(out, dtype=np.complex128).reshape(4, n)
        assert np.all(np.isfinite(y))
        if which == 1:
            _check_block_apply(M, A, sizes, sectors, xs, y)
            continue
        for k, (px, py) in enumerate(sectors):
            idx = _co2_sector_index(sizes, px, py)
            full = np.zeros(3 * n, dtype=complex)
            full[idx[idx >= 0]] = xs[k][idx >= 0]
            ref = A @ full
            got = np.zeros_like(ref)
            got[idx[idx >= 0]] = y[k][idx >= 0]
            assert np.all(y[k][idx < 0] == 0)
            bound = 1e-12 * (abs(A) @ np.abs(full)) + 1e-13
            assert np.all(np.abs(got - ref) <= bound), k


def _check_block_apply(M, A, sizes, sectors, xs, y):
    """y = M^{-1} x for the bend-plane blocks: backward error against the
    oracle's block-diagonal part of A, within the bound of the FP16/FP32
    factor (as in the GPU test of the block preconditioner)."""
    key = np.zeros(3 * M.n, dtype=np.int64)
    for b, ii in enumerate(poly.bend_blocks(sizes)):
        key[ii] = b
    Ac = A.tocoo()
    keep = key[Ac.row] == key[Ac.col]
    B = sp.csr_matrix((Ac.data[keep], (Ac.row[keep], Ac.col[keep])), shape=A.shape)
    normB = np.max(np.abs(B).sum(axis=1))
    tol = 8 * (2 * 2.0 ** -11 + (2 * sizes["y"] + 2) * 2.0 ** -24)
    for k, (px, py) in enumerate(sectors):
        idx = _co2_sector_index(sizes, px, py)
        full = np.zeros(3 * M.n, dtype=complex)
        full[idx[idx >= 0]] = xs[k][idx >= 0]
        yf = np.zeros(3 * M.n, dtype=complex)
        yf[idx[idx >= 0]] = y[k][idx >= 0]
        assert np.all(y[k][idx < 0] == 0), k
        assert np.max(np.abs(B @ yf - full)) <= tol * normB * np.max(np.abs(yf)), k


def test_term_list_solve_under_emulation(exe, tmp_path):
    """The term-list kernels (stencil compilation, level-shift planes, the
    batched COCG) on a small quartic three-state model against the oracle's
    LU of the same term lists."""
    from paper_2307_13483_amd import vdc
    desc = inputs.quartic_model(nbasis=(6, 5, 3))
    jobs = [(0.5, (0, 0, 0), 0), (1.6, (1, 0, 0), 1), (2.4, (0, 1, 0), 0)]
    finals = [(0, 0, 0), (1, 0, 0)]
    opts = vdc.Opts(restart=30, precond=vdc.PREC_JACOBI, method=vdc.COCG, max_iter=20000)
    case, out = str(tmp_path / "terms.bin"), str(tmp_path / "tout.bin")
    emu.write_terms_case(case, desc, jobs, finals, opts)
    rc, text = emu.run(exe, ["terms", case, "0", out])
    assert rc == 0, text[-3000:]
    rows = emu.job_lines(text)
    assert len(rows) == len(jobs) and all(r[0] == 0 for r in rows), text[-2000:]
    nj, nf, P = len(jobs), len(finals), 2
    N = 3 * 6 * 5 * 3
    raw = np.fromfile(out, dtype=np.float64)
    T = raw[:2 * nj * nf * P].view(np.complex128).reshape(nj, nf, P)
    psi = raw[2 * nj * nf * P + nj * nf:].view(np.complex128).reshape(nj, N)
    for k, (eps_i, vi, mu) in enumerate(jobs):
        tm = terms.TermModel(desc, terms.total_energy(desc, eps_i, vi))
        A = tm.matrix()
        b = tm.phi(vi, mu)
        assert np.linalg.norm(b - A @ psi[k]) / np.linalg.norm(b) <= 1e-10 + 1e-13
        ref = solvers.lu_solve(A, b)
        assert np.linalg.norm(psi[k] - ref) <= 1e-8 * np.linalg.norm(ref)
        Tref = np.array([[tm.phi(vf, mf) @ ref for mf in range(P)] for vf in finals])
        assert np.max(np.abs(T[k] - Tref)) <= 1e-8 * np.max(np.abs(Tref))


@pytest.mark.parametrize("method", ["gmres", "cocg"])
def test_co2_solve_under_emulation(exe, tmp_path, method):
    """The CO2-like solver kernels (the bend-plane factor, then GMRES or COCG
    with the block preconditioner's apply and the operator inside one
    persistent launch) on a small model, three partial waves and an excited
    initial state, against the oracle's LU: true residual <= 1e-10 +
    rounding, solution within 1e-8, amplitudes and cross sections."""
    from paper_2307_13483_amd import vdc
    P = inputs.co2like_params()
    sizes = dict(s=3, x=4, y=5, a=2)
    jobs = [(0.8, (0, 0, 0, 0), 0), (2.0, (0, 0, 0, 0), 1), (1.4, (1, 0, 0, 0), 2)]
    finals = [(0, 0, 0, 0), (1, 0, 0, 0), (0, 1, 0, 0)]
    opts = vdc.Opts(restart=20, precision=vdc.FP64, precond=vdc.PREC_BLOCK, max_iter=5000,
                    method=vdc.COCG if method == "cocg" else vdc.GMRES)
    desc, case, out = (str(tmp_path / n) for n in ("co2.bin", "case.bin", "out.bin"))
    emu.write_co2_desc(desc, P, sizes)
    emu.write_co2_solve_case(case, jobs, finals, opts)
    rc, text = emu.run(exe, ["co2solve", desc, case, out])
    assert rc == 0, text[-3000:]
    rows = emu.job_lines(text)
    assert len(rows) == len(jobs) and all(r[0] == 0 for r in rows), text[-2000:]
    nj, nf = len(jobs), len(finals)
    n = sizes["s"] * sizes["x"] * sizes["y"] * sizes["a"]
    raw = np.fromfile(out, dtype=np.float64)
    T = raw[:2 * nj * nf * 3].view(np.complex128).reshape(nj, nf, 3)
    sig = raw[2 * nj * nf * 3:2 * nj * nf * 3 + nj * nf].reshape(nj, nf)
    psi = raw[2 * nj * nf * 3 + nj * nf:].view(np.complex128).reshape(nj, n)
    for k, (eps, v, mu) in enumerate(jobs):
        E = poly.total_energy(P, eps, v)
        M = poly.PolyModel(P, sizes, E)
        A = M.matrix().tocsr()
        b = M.phi(v, poly.WAVES[mu])
        x_lu = solvers.lu_solve(A, b)
        px, py = vdc.co2_sector(v, mu)
        idx = _co2_sector_index(sizes, px, py)
        assert np.all(psi[k][idx < 0] == 0)
        full = np.zeros(3 * n, dtype=complex)
        full[idx[idx >= 0]] = psi[k][idx >= 0]
        assert np.linalg.norm(b - A @ full) / np.linalg.norm(b) <= 1e-10 + 1e-13, k
        assert np.linalg.norm(full - x_lu) <= 1e-8 * np.linalg.norm(x_lu), k
        for f, vf in enumerate(finals):
            for m_, muf in enumerate(poly.WAVES):
                Tref = M.phi(vf, muf) @ x_lu
                assert abs(T[k, f, m_] - Tref) <= 1e-7 * max(1e-300, np.max(np.abs(x_lu))), (k, f, m_)
        pref = 2 * math.pi ** 3 / (eps / ls.HARTREE_EV)
        assert np.allclose(sig[k], pref * np.sum(np.abs(T[k]) ** 2, axis=1), rtol=1e-12, atol=0)
