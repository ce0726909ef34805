"""Pin for Theorem sgt-fp with S = x, T = I (norm preservation): on
orthonormal rows the ratios rho_i are chi^2_r / r, so their mean is 1 within
4 sqrt(2/(r m)) and a KS test against chi^2_r / r does not reject."""
import numpy as np
from scipy import stats as sps

import synth
from oracle import omega, project, stats

ALPHA16 = 0.99999995572


def test_jl_orthonormal_rows():
    n, m, r = 2048, 512, 64
    q = synth.np_haar(n, m, np.random.default_rng(4)).T      # m orthonormal rows
    om = omega.omega_f16(31, 0, n, r)
    y = project.project_f64(q, om)
    rho = stats.row_ratios(q, y, ALPHA16, r)
    assert abs(rho.mean() - 1.0) < 4 * np.sqrt(2.0 / (r * m))
    assert sps.kstest(rho * r, sps.chi2(r).cdf).pvalue > 1e-3
