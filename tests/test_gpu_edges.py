"""Edge cases of the two-state solve on the GPU against the oracle: the
widest rows the descriptor allows (N_u = 1024, where the FP64 operator's
LDS tile no longer fits a row and the solvers take the two-pass global
form, and the FP32 tile holds one row) and the tallest columns (N_g = 1024
over N_u = 2), through FP64 GMRES, FGMRES, FP64 COCG, FP32-inner COCG and
the row blocks; and an empty job list.  Acceptance as in the parity tests:
true residual <= 1e-10 + rounding, solution and amplitudes within 1e-8 of
LU."""
import numpy as np
import pytest

import _oracle_pool as op
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


CASES = [(3, 1024, "gmres"), (3, 1024, "fgmres_fp32"), (3, 1024, "cocg"), (3, 1024, "cocg_fp32"),
         (3, 1024, "cocg_rows"), (1024, 2, "gmres"), (1024, 2, "cocg_fp32")]


@pytest.mark.parametrize("Ng,Nu,path", CASES)
def test_widest_and_tallest_bases(vdc, Ng, Nu, path):
    p = inputs.draw_params(41)
    jobs = [(0.9, (0, 0), 0), (2.2, (min(1, Ng - 1), 0), 1), (1.5, (0, 1), 0)]
    finals = [(0, 0), (0, 1)]
    fp32 = "fp32" in path
    cocg = path.startswith("cocg")
    opts = vdc.Opts(restart=20, precond=vdc.PREC_ROWS if "rows" in path else vdc.PREC_BLOCK,
                    precision=vdc.FP32_INNER if fp32 else vdc.FP64,
                    method=vdc.COCG if cocg else vdc.GMRES,
                    inner_restart=200 if cocg else 8, inner_tol=1e-5 if cocg else 1e-3,
                    outer_restart=16, max_iter=20000)
    T, sigma, psi, infos = vdc.solve(vdc.Model2D(p, Ng, Nu), jobs, finals, opts, want_psi=True)
    assert all(i["status"] == vdc.CONVERGED for i in infos)
    T, psi = T.cpu().numpy(), psi.cpu().numpy()
    checks = op.pool_map(op.check_2d_job, [(p, Ng, Nu, j, finals, psi[k])
                                           for k, j in enumerate(jobs)])
    for k, c in enumerate(checks):
        assert c["res"] <= 1e-10 + 1e-13, (k, c["res"])
        assert c["psi_err"] <= 1e-8, (k, c["psi_err"])
        assert np.max(np.abs(T[k] - c["T"])) <= 1e-8 * max(1e-300, np.max(np.abs(c["T"])))


def test_empty_job_list(vdc):
    """No jobs: the call succeeds, launches nothing and returns empty results."""
    model = vdc.Model2D(inputs.draw_params(42), 6, 5)
    s = vdc.Solver(model, [], [(0, 0)], vdc.Opts()).run()
    assert s.infos() == [] and s.T.shape[0] == 0 and s.sigma.shape[0] == 0
