"""Bitwise reproducibility of dg_run on the GPU.

* Two runs from the same state give bitwise identical states and reports.
  The kernels' reductions are order independent (maxima through atomic max
  of the bit patterns, the ledger a fixed two-pass partition) and every list
  the kernels build with atomic appends (troubled cells, cells for the
  positivity limiter) is processed cell by cell, so its order does not
  matter.
* Resume: N steps then N more steps equal 2N steps in one call, bit for bit
  (the time step is chosen on the device from the state, and dg_run's
  launch batching does not change what a step computes)."""
import math

import numpy as np
import pytest

import dg_inputs as I

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dg():
    import torch

    assert torch.cuda.is_available()
    import paper_2407_19169_amd as dg

    return dg


def _dmr(dg, prec, filt, k=2):
    w = I.double_mach(64, 16, k)
    post, pre = I.conserved2d(*w.extra["post"]), I.conserved2d(1.4, 0.0, 0.0, 1.0)
    speed = w.extra["shock_speed"] / math.sin(math.pi / 3)
    mesh = dg.make_mesh(2, (64, 16), (0.0, 0.0), (4.0, 1.0), (3, 1, 4, 5),
                        dirichlet=[list(post)] * 4, shock_x0=1 / 6, shock_speed=speed,
                        post=list(post), pre=list(pre))
    s = dg.Solver(mesh, k, 2, dg.make_options(precision=prec, filter=filt, cfl=0.1, positivity=1))
    return s, w.u0


def _shu_osher(dg, prec, filt, n=20000):
    w = I.shu_osher(n, 2)
    mesh = dg.make_mesh(1, (n,), (w.lo,), (w.hi,), (1, 1))
    s = dg.Solver(mesh, 2, 2, dg.make_options(precision=prec, filter=filt, cfl=0.1))
    return s, w.u0


WORKLOADS = [("dmr_hybrid_pp", _dmr, 2), ("dmr_jump_pp", _dmr, 1),
             ("shu_osher_hybrid", _shu_osher, 2), ("shu_osher_jump", _shu_osher, 1)]


def _report_tuple(r):
    return (r.steps, r.t, r.dt_min, r.dt_max, tuple(r.ledger), tuple(r.boundary_flux),
            r.troubled_cells, r.status, r.restarts)


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("name,make,filt", WORKLOADS)
def test_two_runs_bitwise_identical(dg, name, make, filt, prec):
    states, reps = [], []
    for _ in range(2):
        s, u0 = make(dg, prec, filt)
        s.set_state(u0)
        reps.append(_report_tuple(dg.dg_run(s.h, 1e30, 37)))
        states.append(s.get_state().cpu().numpy())
        s.close()
    assert reps[0] == reps[1]
    assert np.array_equal(states[0], states[1])


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("name,make,filt", WORKLOADS)
def test_resume_equals_continuous(dg, name, make, filt, prec):
    """19 + 19 steps (an odd count, so the second call starts from the other
    buffer role) equal 38 steps."""
    s, u0 = make(dg, prec, filt)
    s.set_state(u0)
    dg.dg_run(s.h, 1e30, 19)
    r2 = dg.dg_run(s.h, 1e30, 19)
    a = s.get_state().cpu().numpy()
    s.close()
    s, u0 = make(dg, prec, filt)
    s.set_state(u0)
    r = dg.dg_run(s.h, 1e30, 38)
    b = s.get_state().cpu().numpy()
    s.close()
    assert r2.steps == r.steps == 38 and r2.t == r.t
    assert r2.troubled_cells == r.troubled_cells
    assert tuple(r2.ledger) == tuple(r.ledger)
    assert np.array_equal(a, b)
