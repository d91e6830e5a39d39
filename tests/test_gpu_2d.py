"""GPU parity of the 2D Q^k path (C ABI, gfx950 kernels) against the FP64
oracle.

Bars: FP64 per call (one residual stage, one filter / hybrid application,
the CFL max) relative L-infinity <= 1e-13; FP64 full runs <= 1e-10 after the
stated step counts; sampled cells of one step at the full workload sizes
<= 1e-12 (FP64) and <= 2e-5 (mixed: FP32 bulk)."""
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


def rel_linf(got, want):
    return float(np.max(np.abs(np.asarray(got) - np.asarray(want))) / max(np.max(np.abs(want)), 1e-300))


def random_euler2d(seed, k, ny, nx, amp=0.05):
    rng = np.random.default_rng(seed)
    u = np.zeros((4, (k + 1) ** 2, ny, nx))
    u[:, 0] = I.conserved2d(1 + 0.5 * rng.random((ny, nx)), rng.uniform(-0.5, 0.5, (ny, nx)),
                            rng.uniform(-0.5, 0.5, (ny, nx)), 1 + 0.5 * rng.random((ny, nx)))
    if k > 0:
        u[:, 1:] = amp * rng.standard_normal((4, (k + 1) ** 2 - 1, ny, nx)) * np.abs(u[:, :1])
    return u


DMR_POST = I.conserved2d(8.0, 8.25 * math.cos(math.pi / 6), -8.25 * math.sin(math.pi / 6), 116.5)
DMR_PRE = I.conserved2d(1.4, 0.0, 0.0, 1.0)


def _mesh_kwargs(bcs):
    st = I.conserved2d(1.1, 0.2, -0.1, 0.9)
    return dict(dirichlet=[list(st)] * 4, shock_x0=0.3, shock_speed=5.0,
                post=list(DMR_POST / 8.0 + np.array([0.5, 0, 0, 2.0])), pre=list(DMR_PRE))


def _pair(dg, ref, eq, k, nx, ny, bcs, filt, prec=0, cfl=0.1, box=(0.0, 1.0, 0.0, 0.8),
          reading=0, pp=0):
    kw = _mesh_kwargs(bcs)
    mesh = dg.make_mesh(2, (nx, ny), (box[0], box[2]), (box[1], box[3]), bcs, **kw)
    opt = dg.make_options(precision=prec, filter=filt, cfl=cfl, adv_speed=(0.8, -0.5),
                          cf_reading=reading, positivity=pp)
    s = dg.Solver(mesh, k, eq, opt)
    P = ref.problem2d(eq, k, nx, ny, box[0], box[1], box[2], box[3], bc=bcs, filter=filt, cfl=cfl,
                      adv_speed=(0.8, -0.5), dirichlet=kw["dirichlet"], shock_x0=kw["shock_x0"],
                      shock_speed=kw["shock_speed"], post=kw["post"], pre=kw["pre"],
                      cf_reading=reading, pp=pp)
    return s, P


def _dmr(dg, ref, nx, ny, k, filt, prec=0, pp=1, basis=0):
    w = I.double_mach(nx, ny, k)
    post, pre = I.conserved2d(*w.extra["post"]), I.conserved2d(1.4, 0.0, 0.0, 1.0)
    speed = w.extra["shock_speed"] / math.sin(math.pi / 3)
    mesh = dg.make_mesh(2, (nx, ny), (0.0, 0.0), (4.0, 1.0), (3, 1, 4, 5),
                        dirichlet=[list(post)] * 4, shock_x0=1 / 6, shock_speed=speed,
                        post=list(post), pre=list(pre))
    s = dg.Solver(mesh, k, 2, dg.make_options(precision=prec, filter=filt, cfl=0.1, positivity=pp,
                                              basis=basis))
    P = ref.problem2d(2, k, nx, ny, 0.0, 4.0, 0.0, 1.0, bc=(3, 1, 4, 5), filter=filt, cfl=0.1,
                      dirichlet=[list(post)] * 4, shock_x0=1 / 6, shock_speed=speed, post=post,
                      pre=pre, pp=pp, basis=basis)
    return w, s, P


CASES = [
    # eq, k, nx, ny, bcs
    (2, 0, 17, 9, (0, 0, 0, 0)),
    (2, 1, 16, 16, (0, 0, 0, 0)),
    (2, 1, 33, 20, (1, 1, 2, 2)),
    (2, 2, 20, 13, (0, 0, 0, 0)),
    (2, 2, 31, 17, (3, 1, 4, 5)),
    (2, 2, 1, 1, (0, 0, 0, 0)),
    (2, 3, 18, 35, (2, 2, 1, 1)),
    (2, 3, 40, 24, (3, 1, 4, 5)),
    (0, 2, 19, 21, (0, 0, 0, 0)),
    (0, 3, 17, 16, (1, 1, 3, 3)),
    # periodic in one direction only: the jump filter's interior launch
    # then spans a full tile row (x) or column (y) range, and its boundary
    # launch only the rows (columns) at the non-periodic edges
    (2, 2, 50, 26, (0, 0, 2, 2)),
    (2, 1, 45, 12, (1, 1, 0, 0)),
    # one tile column (x not periodic) or one tile row (y not periodic)
    (2, 2, 5, 40, (1, 1, 0, 0)),
    (2, 1, 40, 3, (0, 0, 2, 2)),
]


@pytest.mark.parametrize("eq,k,nx,ny,bcs", CASES)
def test_stage_and_filter_per_call_2d(dg, ref, eq, k, nx, ny, bcs):
    import torch

    nm = (k + 1) ** 2
    if eq == 2:
        un, ua, ub = (random_euler2d(s, k, ny, nx) for s in (1, 2, 3))
    else:
        rng = np.random.default_rng(4)
        un, ua, ub = (rng.standard_normal((1, nm, ny, nx)) for _ in range(3))
    dt = 0.05 / nx
    for filt in (0, 1, 2):
        s, P = _pair(dg, ref, eq, k, nx, ny, bcs, filt)
        for stage, us in ((0, un), (1, ua), (2, ub)):
            s.set_state(un)
            if stage:
                dg.buffer_view(s, stage).copy_(torch.as_tensor(us))
            dg.dg_stage(s.h, stage, dt)
            dg.dg_jump_filter(s.h, stage, dt)
            torch.cuda.synchronize()
            got = dg.buffer_view(s, {0: 1, 1: 2, 2: 0}[stage]).cpu().numpy()
            w = ref.stage2d(P, stage, dt, un, us, t=0.0)
            tf = (1.0, 0.5, 1.0)[stage] * dt
            want, _ = ref.post2d(P, stage, dt, w, t=tf)
            for v in range(got.shape[0]):
                err = rel_linf(got[v], want[v])
                assert err <= 1e-13, (eq, k, nx, ny, bcs, filt, stage, v, err)
            if filt == 1:
                Eg = s.exponents().cpu().numpy().reshape(ny, nx, 2 * k + 1)
                Ew, _ = ref.exponents2d(P, dt, w, t=tf)
                assert rel_linf(Eg, Ew) <= 1e-13
        s.close()


@pytest.mark.parametrize("k", [2, 3])
def test_stage_zero_dt_2d(dg, ref, k):
    """A per-call stage with dt = 0 is the bare Shu-Osher combination
    (3/4 u_n + 1/4 u_a, 1/3 u_n + 2/3 u_b), FP64, against the oracle."""
    import torch

    nx, ny = 20, 13
    un, ua, ub = (random_euler2d(s, k, ny, nx) for s in (1, 2, 3))
    s, P = _pair(dg, ref, 2, k, nx, ny, (0, 0, 0, 0), 0)
    for stage, us in ((1, ua), (2, ub)):
        s.set_state(un)
        dg.buffer_view(s, stage).copy_(torch.as_tensor(us))
        dg.dg_stage(s.h, stage, 0.0)
        dg.dg_jump_filter(s.h, stage, 0.0)
        torch.cuda.synchronize()
        got = dg.buffer_view(s, {1: 2, 2: 0}[stage]).cpu().numpy()
        want = ref.stage2d(P, stage, 0.0, un, us, t=0.0)
        for v in range(4):
            assert rel_linf(got[v], want[v]) <= 1e-15, (stage, v)
    s.close()


def test_hybrid_per_call_many_troubled_cells(dg, ref):
    """Hybrid post-stage operator (Algorithm 1) on a 480 x 360 random Euler
    state (Q2, periodic) in which every cell is troubled: more
    troubled cells than the exponent and blend launches have wavefronts, so
    each wavefront takes several cells in turn.  Every troubled cell's
    exponents must come from the unfiltered stage output, neighbours
    included, whatever order the cells are processed in: FP64 result vs the
    oracle at 1e-13."""
    import torch

    k, nx, ny = 2, 480, 360
    un = random_euler2d(11, k, ny, nx, amp=0.05)
    dt = 0.05 / nx
    s, P = _pair(dg, ref, 2, k, nx, ny, (0, 0, 0, 0), 2)
    s.set_state(un)
    dg.dg_stage(s.h, 0, dt)
    dg.dg_jump_filter(s.h, 0, dt)
    torch.cuda.synchronize()
    got = dg.buffer_view(s, 1).cpu().numpy()
    s.close()
    w = ref.stage2d(P, 0, dt, un, un, t=0.0)
    want, troubled = ref.post2d(P, 0, dt, w, t=dt)
    assert troubled > 4 * 16384 and np.all(np.isfinite(want)), troubled
    for v in range(4):
        err = rel_linf(got[v], want[v])
        assert err <= 1e-13, (v, err)


@pytest.mark.parametrize("reading", [1, 2])
@pytest.mark.parametrize("k,nx,ny,bcs", [(1, 33, 20, (1, 1, 2, 2)), (2, 31, 17, (3, 1, 4, 5)),
                                         (3, 18, 35, (2, 2, 1, 1))])
def test_filter_readings_per_call(dg, ref, reading, k, nx, ny, bcs):
    """The two other readings of the mesh factors of (c_fx, c_fy): (h_y, h_x)
    as printed in Sec. 3.2 and none; non-square cells (h_x != h_y), so every
    reading gives different exponents.  One stage plus filter, FP64,
    relative L-infinity <= 1e-13 (the default reading is covered above)."""
    import torch

    un = random_euler2d(1, k, ny, nx)
    dt = 0.05 / nx
    s, P = _pair(dg, ref, 2, k, nx, ny, bcs, 1, reading=reading)
    s.set_state(un)
    dg.dg_stage(s.h, 0, dt)
    dg.dg_jump_filter(s.h, 0, dt)
    torch.cuda.synchronize()
    got = dg.buffer_view(s, 1).cpu().numpy()
    w = ref.stage2d(P, 0, dt, un, un, t=0.0)
    want, _ = ref.post2d(P, 0, dt, w, t=dt)
    for v in range(4):
        assert rel_linf(got[v], want[v]) <= 1e-13, (reading, v)
    Eg = s.exponents().cpu().numpy().reshape(ny, nx, 2 * k + 1)
    Ew, _ = ref.exponents2d(P, dt, w, t=dt)
    assert rel_linf(Eg, Ew) <= 1e-13
    s.close()


def _strong_state(seed, k, ny, nx):
    """Euler cells with large higher modes (many need the positivity limiter),
    some near vacuum."""
    rng = np.random.default_rng(seed)
    u = np.zeros((4, (k + 1) ** 2, ny, nx))
    u[:, 0] = I.conserved2d(10.0 ** rng.uniform(-2, 0.5, (ny, nx)), rng.uniform(-2, 2, (ny, nx)),
                            rng.uniform(-2, 2, (ny, nx)), 10.0 ** rng.uniform(-3, 1, (ny, nx)))
    u[:, 1:] = 0.5 * rng.standard_normal((4, (k + 1) ** 2 - 1, ny, nx)) * u[:, :1]
    return u


@pytest.mark.parametrize("k", [1, 2, 3])
def test_positivity_limiter_per_call_2d(dg, ref, k):
    """The 2D positivity limiter after no operator / the jump filter / the
    hybrid, one call each, FP64, relative L-infinity <= 1e-13 against the
    oracle's post-stage operator with the limiter.  Input: the first stage of
    the double Mach problem (64 x 16), whose shock cells have negative
    pressure at test points."""
    import torch

    for filt in (0, 1, 2):
        w, s, P = _dmr(dg, ref, 64, 16, k, filt)
        dt = 0.1 / ref.max_wavespeed2d(P, w.u0)
        s.set_state(w.u0)
        dg.dg_stage(s.h, 0, dt)
        dg.dg_jump_filter(s.h, 0, dt)
        torch.cuda.synchronize()
        got = dg.buffer_view(s, 1).cpu().numpy()
        st = ref.stage2d(P, 0, dt, w.u0, w.u0, t=0.0)
        want, _ = ref.post2d(P, 0, dt, st, t=dt)
        Pn = ref.problem2d(2, k, 64, 16, 0.0, 4.0, 0.0, 1.0, bc=P.bc, filter=filt, cfl=0.1,
                           dirichlet=[list(P.dirichlet[0])] * 4, shock_x0=P.shock_x0,
                           shock_speed=P.shock_speed, post=list(P.post), pre=list(P.pre), pp=0)
        plain, _ = ref.post2d(Pn, 0, dt, st, t=dt)
        assert np.any(want != plain)           # the limiter acted
        for v in range(4):
            assert rel_linf(got[v], want[v]) <= 1e-13, (k, filt, v, rel_linf(got[v], want[v]))
        s.close()


@pytest.mark.parametrize("eq,k,nx,ny,bcs", CASES[:5])
def test_max_wavespeed_2d(dg, ref, eq, k, nx, ny, bcs):
    u = random_euler2d(5, k, ny, nx) if eq == 2 else np.ones((1, (k + 1) ** 2, ny, nx))
    s, P = _pair(dg, ref, eq, k, nx, ny, bcs, 1)
    s.set_state(u)
    assert dg.dg_max_wavespeed(s.h) == pytest.approx(ref.max_wavespeed2d(P, u), rel=1e-14)
    s.close()


def _run_pair(dg, ref, w, eq, filt, steps, t_end=1e30, prec=0, pp=0, reading=0):
    mesh = dg.make_mesh(2, (w.nx, w.ny), (w.xlo, w.ylo), (w.xhi, w.yhi), w.bc)
    s = dg.Solver(mesh, w.k, eq, dg.make_options(precision=prec, filter=filt, cfl=w.cfl,
                                                 positivity=pp, cf_reading=reading))
    s.set_state(w.u0)
    rep = dg.dg_run(s.h, t_end, steps)
    got = s.get_state().cpu().numpy()
    P = ref.problem2d(eq, w.k, w.nx, w.ny, w.xlo, w.xhi, w.ylo, w.yhi, bc=w.bc, filter=filt,
                      cfl=w.cfl, pp=pp, cf_reading=reading)
    want, orep, rc = ref.run2d(P, w.u0, t_end, steps)
    s.close()
    return got, want, rep, orep, rc


@pytest.mark.parametrize("k", [1, 2, 3])
def test_vortex_run_parity(dg, ref, k):
    """Smooth isentropic vortex (seeded centre), 40x40, jump filter, 60 steps."""
    w = I.vortex2d(40, k, seed=3001)
    got, want, rep, orep, rc = _run_pair(dg, ref, w, 2, 1, 60)
    assert rc == 0 and rep.steps == orep.steps == 60
    for v in range(4):
        assert rel_linf(got[v], want[v]) <= 1e-10
    h2 = (10.0 / 40) ** 2
    for v in range(4):
        q0 = h2 * w.u0[v, 0].sum()
        assert abs(rep.ledger[v] - q0) < 1e-12 * max(1.0, abs(q0))


@pytest.mark.parametrize("n", [32, 34])
def test_quadrant_hybrid_run_parity(dg, ref, n):
    """Seeded four-quadrant Riemann problem, 32x32 and 34x34 (ragged tiles
    on a periodic mesh, whose slots past the edge hold the wrapped cells),
    Q2, hybrid with the positivity limiter, 30 steps."""
    w = I.quadrant2d(n, 2, seed=3002)
    got, want, rep, orep, rc = _run_pair(dg, ref, w, 2, 2, 30, pp=1)
    assert rc == 0 and rep.steps == 30
    for v in range(4):
        assert rel_linf(got[v], want[v]) <= 1e-10
    assert rep.troubled_cells > 0


@pytest.mark.parametrize("k,filt", [(3, 1), (2, 2), (3, 2), (1, 2)])
def test_double_mach_small_run_parity(dg, ref, k, filt):
    """Double Mach reflection on 64x16 with the moving top boundary, the
    printed filter coefficient and the positivity limiter, 20 steps: the jump
    filter and the hybrid limiter (Algorithm 1), FP64 within 1e-10."""
    w, s, P = _dmr(dg, ref, 64, 16, k, filt)
    s.set_state(w.u0)
    rep = dg.dg_run(s.h, 1e30, 20)
    got = s.get_state().cpu().numpy()
    want, orep, rc = ref.run2d(P, w.u0, 1e30, 20)
    assert rc == 0 and rep.status == 0, (rc, rep.status)
    assert rep.steps == orep.steps == 20 and rep.restarts == orep.restarts
    assert rep.troubled_cells == orep.troubled_cells
    for v in range(4):
        assert rel_linf(got[v], want[v]) <= 1e-10, (v, rel_linf(got[v], want[v]))
    s.close()


@pytest.mark.parametrize("k,filt,nx,ny", [(2, 2, 40, 12), (1, 1, 21, 5)])
def test_double_mach_ragged_run_parity(dg, ref, k, filt, nx, ny):
    """The double Mach run on meshes that fill no tile evenly: 40x12 with the
    hybrid limiter (the indicator's 16x8 tiles: the second tile row holds 4
    of its 8 rows), 21x5 with the jump filter (one tile row, so every tile is
    a boundary tile); FP64 within 1e-10 after 12 steps."""
    w, s, P = _dmr(dg, ref, nx, ny, k, filt)
    s.set_state(w.u0)
    rep = dg.dg_run(s.h, 1e30, 12)
    got = s.get_state().cpu().numpy()
    want, orep, rc = ref.run2d(P, w.u0, 1e30, 12)
    assert rc == 0 and rep.status == 0, (rc, rep.status)
    assert rep.steps == orep.steps == 12 and rep.restarts == orep.restarts
    assert rep.troubled_cells == orep.troubled_cells
    for v in range(4):
        assert rel_linf(got[v], want[v]) <= 1e-10, (v, rel_linf(got[v], want[v]))
    s.close()


@pytest.mark.parametrize("filt", [1, 2])
def test_double_mach_mixed_l1(dg, ref, filt):
    """Mixed precision (FP32 bulk, FP64 mode 0 and positivity checks) on the
    double Mach problem, Q3, 64x16, 40 steps: cell averages within the strong-
    shock bound 1e-3 (relative L1 per variable) of the FP64 oracle."""
    w, s, P = _dmr(dg, ref, 64, 16, 3, filt, prec=1)
    s.set_state(w.u0)
    rep = dg.dg_run(s.h, 1e30, 40)
    got = s.get_state().cpu().numpy()
    s.close()
    want, orep, rc = ref.run2d(P, w.u0, 1e30, 40)
    assert rc == 0 and rep.status == 0 and rep.steps == 40
    for v in range(4):
        l1 = np.sum(np.abs(got[v, 0] - want[v, 0])) / np.sum(np.abs(want[v, 0]))
        print(f"double Mach Q3 mixed filter {filt}: var {v} relative L1 {l1:.3e}")
        assert l1 < 1e-3, (v, l1)


def test_mixed_precision_vortex_2d(dg, ref):
    """FP32 bulk / FP64 mode 0: cell averages within 1e-6 (relative L1) of
    the FP64 oracle after 60 steps; conservation to FP64 roundoff."""
    w = I.vortex2d(40, 2, seed=3001)
    got, want, rep, orep, rc = _run_pair(dg, ref, w, 2, 1, 60, prec=1)
    h2 = (10.0 / 40) ** 2
    for v in range(4):
        l1 = np.sum(np.abs(got[v, 0] - want[v, 0])) / np.sum(np.abs(want[v, 0]))
        assert l1 < 1e-6, (v, l1)
        q0 = h2 * w.u0[v, 0].sum()
        assert abs(rep.ledger[v] - q0) < 1e-12 * max(1.0, h2 * np.abs(got[v, 0]).sum())


def _patch_step(ref, P_full, u0, jy, ix, dt, r=7):
    """Oracle step of a (2r+1)^2 patch around (jy, ix); the centre cell's
    value after one step depends on cells within radius 6 only."""
    ny, nx = u0.shape[-2:]
    rows = np.arange(jy - r, jy + r + 1) % ny
    cols = np.arange(ix - r, ix + r + 1) % nx
    patch = np.ascontiguousarray(u0[:, :, rows][:, :, :, cols])
    hx = (P_full.xhi - P_full.xlo) / nx
    hy = (P_full.yhi - P_full.ylo) / ny
    P = ref.problem2d(P_full.eq, P_full.k, 2 * r + 1, 2 * r + 1, P_full.xlo + (ix - r) * hx,
                      P_full.xlo + (ix + r + 1) * hx, P_full.ylo + (jy - r) * hy,
                      P_full.ylo + (jy + r + 1) * hy, bc=(1, 1, 1, 1), filter=P_full.filter,
                      cfl=P_full.cfl, cf_reading=P_full.cf_reading, pp=P_full.pp)
    out = ref.step2d(P, dt, patch, t=0.0)
    return out[:, :, r, r]


@pytest.mark.parametrize("prec", [0, 1])
def test_full_size_vortex_sampled_step(dg, ref, prec):
    """1024x1024, Q2, periodic, jump filter (vortex workload): one dg_run step
    on the GPU vs oracle steps of patches around 24 sampled cells."""
    n, k = 1024, 2
    w = I.vortex2d(n, k, seed=3001)
    mesh = dg.make_mesh(2, (n, n), (0.0, -5.0), (10.0, 5.0), (0, 0, 0, 0))
    s = dg.Solver(mesh, k, 2, dg.make_options(precision=prec, filter=1, cfl=0.1))
    s.set_state(w.u0)
    rep = dg.dg_run(s.h, 1e30, 1)
    got = s.get_state().cpu().numpy()
    P = ref.problem2d(2, k, n, n, 0.0, 10.0, -5.0, 5.0, bc=(0, 0, 0, 0), filter=1, cfl=0.1)
    dt = 0.1 / ref.max_wavespeed2d(P, w.u0)
    assert rep.dt_max == pytest.approx(dt, rel=1e-14)
    rng = np.random.default_rng(7)
    samples = [(int(jy), int(ix)) for jy, ix in rng.integers(0, n, (20, 2))]
    samples += [(512, 512), (0, 0), (n - 1, 3), (400, 600)]
    tol = 1e-12 if prec == 0 else 2e-5
    for jy, ix in samples:
        want = _patch_step(ref, P, w.u0, jy, ix, dt)
        err = np.max(np.abs(got[:, :, jy, ix] - want)) / np.max(np.abs(want[:, 0]))
        assert err <= tol, (jy, ix, err)
    s.close()


@pytest.mark.parametrize("prec", [0, 1])
def test_full_size_quadrant_sampled_step(dg, ref, prec):
    """1024x1024, Q2, periodic, jump filter (four-quadrant Riemann workload,
    seed 3002): one dg_run step on the GPU vs oracle steps of patches around
    cells on the two discontinuity lines (x = 5, y = 0, including their
    crossing and the periodic seams) and random ones."""
    n, k = 1024, 2
    w = I.quadrant2d(n, k, seed=3002)
    mesh = dg.make_mesh(2, (n, n), (0.0, -5.0), (10.0, 5.0), (0, 0, 0, 0))
    s = dg.Solver(mesh, k, 2, dg.make_options(precision=prec, filter=1, cfl=0.1))
    s.set_state(w.u0)
    rep = dg.dg_run(s.h, 1e30, 1)
    assert rep.status == 0
    got = s.get_state().cpu().numpy()
    s.close()
    P = ref.problem2d(2, k, n, n, 0.0, 10.0, -5.0, 5.0, bc=(0, 0, 0, 0), filter=1, cfl=0.1)
    dt = 0.1 / ref.max_wavespeed2d(P, w.u0)
    assert rep.dt_max == pytest.approx(dt, rel=1e-14)
    rng = np.random.default_rng(8)
    samples = [(512, 512), (511, 511), (512, 511), (511, 512), (0, 0), (1023, 1023), (0, 512),
               (512, 0), (300, 511), (300, 512), (511, 700), (512, 700)]
    samples += [(int(jy), int(ix)) for jy, ix in rng.integers(0, n, (8, 2))]
    tol = 1e-12 if prec == 0 else 2e-5
    for jy, ix in samples:
        want = _patch_step(ref, P, w.u0, jy, ix, dt)
        err = np.max(np.abs(got[:, :, jy, ix] - want)) / np.max(np.abs(want[:, 0]))
        assert err <= tol, (jy, ix, err)


@pytest.mark.parametrize("filt", [1, 2])
def test_full_size_double_mach_sampled_step(dg, ref, filt):
    """4096x1024, Q3, FP64 and mixed precision, positivity limiter (double-
    Mach workload), one GPU step.  Jump filter: oracle steps of patches
    around sampled cells along the shock.  Hybrid: its blend weight uses the
    domain maximum of eta, which no patch sees, so the step is checked by
    properties that hold at any size: admissible averages, troubled cells
    found, constant states away from the shock kept to roundoff."""
    w = I.double_mach(4096, 1024, 3)
    post, pre = I.conserved2d(*w.extra["post"]), I.conserved2d(1.4, 0.0, 0.0, 1.0)
    speed = w.extra["shock_speed"] / math.sin(math.pi / 3)
    mesh = dg.make_mesh(2, (4096, 1024), (0.0, 0.0), (4.0, 1.0), (3, 1, 4, 5),
                        dirichlet=[list(post)] * 4, shock_x0=1 / 6, shock_speed=speed,
                        post=list(post), pre=list(pre))
    for prec, tol in ((0, 1e-12), (1, 2e-5)):
        s = dg.Solver(mesh, 3, 2, dg.make_options(precision=prec, filter=filt, cfl=0.1,
                                                  positivity=1))
        s.set_state(w.u0)
        rep = dg.dg_run(s.h, 1e30, 1)
        assert rep.status == 0 and rep.restarts == 0
        got = s.get_state().cpu().numpy()
        s.close()
        P = ref.problem2d(2, 3, 4096, 1024, 0.0, 4.0, 0.0, 1.0, bc=(3, 1, 4, 5), filter=1,
                          cfl=0.1, dirichlet=[list(post)] * 4, shock_x0=1 / 6, shock_speed=speed,
                          post=post, pre=pre, pp=1)
        dt = 0.1 / ref.max_wavespeed2d(P, w.u0)
        assert rep.dt_max == pytest.approx(dt, rel=1e-14)
        if filt == 2:
            rho, p = got[0, 0], (0.4 * (got[3, 0] - 0.5 * (got[1, 0] ** 2 + got[2, 0] ** 2) / got[0, 0]))
            assert rho.min() > 0 and p.min() > 0
            assert rep.troubled_cells > 0
            for jy in (100, 500, 900):
                ix = int((1 / 6 + (jy + 0.5) / 1024 / math.sqrt(3)) * 1024)
                for dx in (-40, 40):
                    # constant states: the residual vanishes up to rounding
                    d = got[:, :, jy, ix + dx] - w.u0[:, :, jy, ix + dx]
                    assert np.max(np.abs(d)) <= tol * np.max(np.abs(w.u0[:, 0, jy, ix + dx]))
            continue
        rng = np.random.default_rng(11)
        for jy in list(rng.integers(20, 1000, 10)) + [500]:
            y = (jy + 0.5) / 1024
            ix = int((1 / 6 + y / math.sqrt(3)) * 1024)  # on the shock
            for dx in (-8, 0, 3, 40):
                want = _patch_step(ref, P, w.u0, int(jy), ix + dx, dt)
                err = np.max(np.abs(got[:, :, jy, ix + dx] - want)) / np.max(np.abs(want[:, 0]))
                assert err <= tol, (prec, jy, ix + dx, err)


# ---- P^k (total degree, the paper's 2D space): basis = 1 on both sides ----
def _pk_mask(k):
    return np.array([1.0 if p + q <= k else 0.0 for p in range(k + 1) for q in range(k + 1)])


@pytest.mark.parametrize("k,nx,ny,bcs", [(1, 16, 16, (0, 0, 0, 0)), (2, 31, 17, (3, 1, 4, 5)),
                                         (3, 18, 35, (2, 2, 1, 1))])
def test_pk_stage_and_filter_per_call(dg, ref, k, nx, ny, bcs):
    """P^k (compact planes on the device): one residual stage plus one filter
    / hybrid application per call, FP64, relative L-infinity <= 1e-13."""
    import torch

    mask = _pk_mask(k)[None, :, None, None]
    un, ua, ub = (random_euler2d(s, k, ny, nx) * mask for s in (1, 2, 3))
    dt = 0.05 / nx
    kw = _mesh_kwargs(bcs)
    box = (0.0, 1.0, 0.0, 0.8)
    mesh = dg.make_mesh(2, (nx, ny), (box[0], box[2]), (box[1], box[3]), bcs, **kw)
    for filt in (0, 1, 2):
        s = dg.Solver(mesh, k, 2, dg.make_options(filter=filt, cfl=0.1, basis=1))
        P = ref.problem2d(2, k, nx, ny, *box, bc=bcs, filter=filt, cfl=0.1,
                          dirichlet=kw["dirichlet"], shock_x0=kw["shock_x0"],
                          shock_speed=kw["shock_speed"], post=kw["post"], pre=kw["pre"], basis=1)
        for stage, us in ((0, un), (1, ua), (2, ub)):
            sel = dg.pk_modes(k)
            s.set_state(un)
            if stage:
                dg.buffer_view(s, stage).copy_(torch.as_tensor(np.ascontiguousarray(us[:, sel])))
            dg.dg_stage(s.h, stage, dt)
            dg.dg_jump_filter(s.h, stage, dt)
            torch.cuda.synchronize()
            got = np.zeros_like(un)
            got[:, sel] = dg.buffer_view(s, {0: 1, 1: 2, 2: 0}[stage]).cpu().numpy()
            w = ref.stage2d(P, stage, dt, un, us, t=0.0)
            tf = (1.0, 0.5, 1.0)[stage] * dt
            want, _ = ref.post2d(P, stage, dt, w, t=tf)
            assert np.all(want[:, _pk_mask(k) == 0.0] == 0.0)
            for v in range(4):
                err = rel_linf(got[v], want[v])
                assert err <= 1e-13, (k, filt, stage, v, err)
        s.close()


@pytest.mark.parametrize("k", [1, 2, 3])
def test_pk_vortex_run_parity(dg, ref, k):
    """P^k vortex (seeded centre), 40x40, jump filter, 60 steps: FP64 within
    1e-10 of the oracle's P^k run.  dg_set_state receives the Q^k
    projection and keeps its P^k part."""
    w = I.vortex2d(40, k, seed=3001)
    mesh = dg.make_mesh(2, (w.nx, w.ny), (w.xlo, w.ylo), (w.xhi, w.yhi), w.bc)
    s = dg.Solver(mesh, k, 2, dg.make_options(filter=1, cfl=w.cfl, basis=1))
    s.set_state(w.u0)
    rep = dg.dg_run(s.h, 1e30, 60)
    got = s.get_state().cpu().numpy()
    s.close()
    P = ref.problem2d(2, k, w.nx, w.ny, w.xlo, w.xhi, w.ylo, w.yhi, bc=w.bc, filter=1, cfl=w.cfl,
                      basis=1)
    u0 = w.u0 * _pk_mask(k)[None, :, None, None]
    want, orep, rc = ref.run2d(P, u0, 1e30, 60)
    assert rc == 0 and rep.steps == orep.steps == 60
    assert np.all(got[:, _pk_mask(k) == 0.0] == 0.0)
    for v in range(4):
        assert rel_linf(got[v], want[v]) <= 1e-10, v


def test_pk_mixed_quadrant_hybrid(dg, ref):
    """P^2 four-quadrant Riemann problem, 32x32, hybrid, mixed precision, 30
    steps: cell averages within 1e-6 (relative L1) of the FP64 oracle."""
    w = I.quadrant2d(32, 2, seed=3002)
    mesh = dg.make_mesh(2, (w.nx, w.ny), (w.xlo, w.ylo), (w.xhi, w.yhi), w.bc)
    s = dg.Solver(mesh, 2, 2, dg.make_options(precision=1, filter=2, cfl=w.cfl, basis=1))
    s.set_state(w.u0)
    rep = dg.dg_run(s.h, 1e30, 30)
    got = s.get_state().cpu().numpy()
    s.close()
    P = ref.problem2d(2, 2, w.nx, w.ny, w.xlo, w.xhi, w.ylo, w.yhi, bc=w.bc, filter=2, cfl=w.cfl,
                      basis=1)
    want, orep, rc = ref.run2d(P, w.u0 * _pk_mask(2)[None, :, None, None], 1e30, 30)
    assert rc == 0 and rep.status == 0 and rep.steps == 30
    assert np.all(got[:, _pk_mask(2) == 0.0] == 0.0)
    for v in range(4):
        l1 = np.sum(np.abs(got[v, 0] - want[v, 0])) / np.sum(np.abs(want[v, 0]))
        print(f"P2 mixed hybrid quadrant: var {v} relative L1 {l1:.3e}")
        assert l1 < 1e-6, (v, l1)


def test_basis_option_checked(dg):
    mesh = dg.make_mesh(2, (8, 8), (0.0, 0.0), (1.0, 1.0), (0, 0, 0, 0))
    with pytest.raises(dg.DGError) as e:
        dg.Solver(mesh, 2, 2, dg.make_options(basis=2))
    assert e.value.code == dg.DG_ERR_ARG
