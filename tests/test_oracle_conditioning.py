"""The fixed step counts of the full-run parity cases are well conditioned:
the oracle started from initial data perturbed by one ulp stays within 2e-11
(relative L-infinity, per variable) of the unperturbed run."""
import numpy as np
import pytest

from parity_cases import cases_1d


@pytest.mark.parametrize("case", cases_1d(), ids=lambda c: c[0])
def test_self_drift_below_fifth_of_bar(ref, case):
    name, eq, k, n, lo, hi, bc, filt, u0, t_end, steps, dirichlet = case
    P = ref.problem1d(eq, k, n, lo, hi, bc=bc, filter=filt, cfl=0.1, dirichlet=dirichlet)
    rng = np.random.default_rng(0)
    u0b = u0 * (1 + 1.1e-16 * rng.choice([-1, 1], size=u0.shape))
    a, ra, rc = ref.run1d(P, u0, t_end, steps)
    b, _, _ = ref.run1d(P, u0b, t_end, steps)
    assert rc == 0
    drift = max(float(np.max(np.abs(a[v] - b[v])) / np.max(np.abs(a[v]))) for v in range(a.shape[0]))
    assert drift <= 2e-11, (name, ra.steps, drift)
