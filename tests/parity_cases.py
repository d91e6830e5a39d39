"""Full-run parity cases of the 1D path and the step counts they run for.

A run that passes shocks amplifies rounding: the oracle run twice from
initial data that differ by one ulp drifts apart by up to ~1e-9 within a few
hundred steps for P^3 shock problems.  Each case's fixed step count is
chosen so that this self-drift of the oracle stays at or below 2e-11, a
fifth of the 1e-10 parity bar (pinned in test_oracle_conditioning.py); the
GPU-vs-oracle bar then measures the implementation, not the problem's
conditioning."""
import dg_inputs as I

LAX_L = I.conserved(0.445, 0.698, 3.528)
LAX_R = I.conserved(0.5, 0.0, 0.571)


def cases_1d():
    """(name, eq, k, n, lo, hi, bc, filter, u0, t_end, max_steps, dirichlet)."""
    out = []
    w = I.shu_osher(20000, 2)
    for filt in (1, 2):
        out.append((f"shu_osher_20000_f{filt}", 2, 2, 20000, -5.0, 5.0, (1, 1), filt, w.u0, 100.0,
                    500, None))
    for k in range(4):
        lax = I.lax(300, k)
        steps = 100 if k == 3 else 200
        out.append((f"lax_outflow_p{k}", 2, k, 300, -1.0, 1.0, (1, 1), 1, lax.u0, 0.13, steps, None))
        out.append((f"lax_reflect_hybrid_p{k}", 2, k, 300, -1.0, 1.0, (2, 2), 2, lax.u0, 0.05, steps,
                    None))
        out.append((f"lax_dirichlet_p{k}", 2, k, 300, -1.0, 1.0, (3, 3), 1, lax.u0, 0.05, steps,
                    [list(LAX_L), list(LAX_R)]))
    return out
