"""The allocation-free entry point dg_max_wavespeed_noalloc (for callers that
cannot allocate device memory) against dg_max_wavespeed, through the C ABI:
the same maximum bit for bit, on two calls in a row, the second with a
smaller input, and with no workspace bound for it."""
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


def _dmr_solver(dg, nx, ny, k, prec):
    w = I.double_mach(nx, ny, k)
    post, pre = I.conserved2d(*w.extra["post"]), I.conserved2d(1.4, 0.0, 0.0, 1.0)
    speed = w.extra["shock_speed"] / math.sin(math.pi / 3)
    mesh = dg.make_mesh(2, (nx, ny), (0.0, 0.0), (4.0, 1.0), (3, 1, 4, 5),
                        dirichlet=[list(post)] * 4, shock_x0=1 / 6, shock_speed=speed,
                        post=list(post), pre=list(pre))
    s = dg.Solver(mesh, k, 2, dg.make_options(precision=prec, filter=1, cfl=0.1, positivity=1))
    s.set_state(w.u0)
    return s


def test_noalloc_matches_workspace_version_twice(dg):
    import torch

    # first call: a 2D FP64 state of 128 x 40 cells (20 workgroups)
    s1 = _dmr_solver(dg, 128, 40, 2, 0)
    want1 = dg.dg_max_wavespeed(s1.h)
    got1, bad1, rc1 = dg.dg_max_wavespeed_noalloc(s1.h, s1._ptrs[0])
    assert rc1 == 0 and got1 == want1 and bad1 == -1
    # second call, smaller: a 1D mixed-precision Euler state of 700 cells
    w = I.shu_osher(700, 2)
    mesh = dg.make_mesh(1, (700,), (w.lo,), (w.hi,), (1, 1))
    s2 = dg.Solver(mesh, 2, 2, dg.make_options(precision=1, filter=2, cfl=0.1))
    s2.set_state(w.u0)
    want2 = dg.dg_max_wavespeed(s2.h)
    got2, bad2, rc2 = dg.dg_max_wavespeed_noalloc(s2.h, s2._ptrs[0])
    assert rc2 == 0 and got2 == want2 and bad2 == -1
    assert got2 != got1
    # the first solver again, after a time step changed its state
    dg.dg_run(s1.h, 1e30, 2)
    torch.cuda.synchronize()
    want3 = dg.dg_max_wavespeed(s1.h)
    got3, _, _ = dg.dg_max_wavespeed_noalloc(s1.h, s1._ptrs[0])
    assert got3 == want3
    s1.close()
    s2.close()


def test_noalloc_reports_first_bad_cell(dg):
    """A state with negative pressure in two cells: the lowest index is
    reported, and the maximum is not finite (the sound speed of a negative
    pressure), as dg_max_wavespeed reports it."""
    import torch

    n = 1000
    rng = np.random.default_rng(3)
    u = np.zeros((3, 2, n))
    u[:, 0] = I.conserved(1 + rng.random(n), rng.uniform(-1, 1, n), 1 + rng.random(n))
    for j in (611, 402):
        u[2, 0, j] = 0.5 * u[1, 0, j] ** 2 / u[0, 0, j] - 0.01   # p < 0
    mesh = dg.make_mesh(1, (n,), (0.0,), (1.0,), (1, 1))
    s = dg.Solver(mesh, 1, 2, dg.make_options(filter=1, cfl=0.1))
    s.set_state(u)
    alpha, bad, rc = dg.dg_max_wavespeed_noalloc(s.h, s._ptrs[0])
    assert bad == 402 and rc == dg.DG_ERR_NONFINITE and math.isnan(alpha)
    with pytest.raises(dg.DGError) as e:
        dg.dg_max_wavespeed(s.h)
    assert e.value.code == dg.DG_ERR_NONFINITE
    # repaired, the same state's maximum matches again (the scratch keeps no
    # state between calls)
    u[2, 0, [402, 611]] += 1.0
    s.set_state(u)
    alpha, bad, rc = dg.dg_max_wavespeed_noalloc(s.h, s._ptrs[0])
    assert rc == 0 and bad == -1 and alpha == dg.dg_max_wavespeed(s.h)
    s.close()


def test_noalloc_rejects_meshes_beyond_its_scratch(dg):
    """More than 16,777,216 cells: DG_ERR_ARG, checked before any device
    access (the solver is created but nothing is bound)."""
    mesh = dg.make_mesh(2, (8192, 2049), (0.0, 0.0), (1.0, 1.0), (0, 0, 0, 0))
    h = dg.dg_create(mesh, 1, 2, dg.make_options(filter=1, cfl=0.1))
    try:
        with pytest.raises(dg.DGError) as e:
            dg.dg_max_wavespeed_noalloc(h, 256)
        assert e.value.code == dg.DG_ERR_ARG
    finally:
        dg.dg_destroy(h)
