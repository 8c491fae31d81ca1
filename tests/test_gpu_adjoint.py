"""GPU parity of the ADI step adjoint and the autograd wrappers against the oracle.

Gradient tolerances: FP64 GPU vs FP64 oracle <= 1e-10 normwise; FP32 GPU (on
FP32-rounded inputs) vs the FP64 oracle <= 1e-4 normwise.
"""

import numpy as np
import pytest

from workloads import gen

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def trid():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2201_03950_amd as trid

    trid.load_library()
    return trid


def _t(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def _nerr(x, ref):
    return float(np.linalg.norm((x - ref).ravel()) / np.linalg.norm(ref.ravel()))


@pytest.mark.parametrize("dt", [np.float64, np.float32])
@pytest.mark.parametrize("dims,batch", [((20, 17, 13), 2), ((33, 9, 40), 1), ((41, 30), 3)])
def test_adi_step_adjoint_matches_oracle(trid, orc, dt, dims, batch):
    rng = np.random.default_rng(sum(dims))
    shape = gen.mesh_shape(dims, batch)
    u = rng.uniform(0, 1, shape).astype(dt)
    s = (0.2 * rng.lognormal(0.0, 0.5, shape)).astype(dt)
    ubar = rng.standard_normal(shape).astype(dt)
    sbar0 = rng.standard_normal(shape).astype(dt)
    ub_ref, sb_ref = orc.adi_step_adjoint(u, s, ubar, sbar0)
    tub, tsb = _t(ubar), _t(sbar0)
    trid.adi_step_adjoint(_t(u), _t(s), tub, tsb)
    tol = 1e-11 if dt == np.float64 else 1e-5
    assert _nerr(tub.cpu().numpy().astype(np.float64), ub_ref) <= tol
    assert _nerr(tsb.cpu().numpy().astype(np.float64), sb_ref) <= tol


@pytest.mark.parametrize("dt,tol", [(np.float64, 1e-10), (np.float32, 1e-4)])
def test_differentiable_adi_128cubed_20_steps(trid, orc, dt, tol):
    """The differentiable workload at full size: 128^3, 20 steps, s = 0.2 kappa."""
    from paper_2201_03950_amd import autograd

    kappa, u0, kstar = gen.diffusion3d((128, 128, 128), dtype=np.float64)
    s0, steps = 0.2, 20
    k_in, u_in = kappa.astype(dt).astype(np.float64), u0.astype(dt).astype(np.float64)
    target = orc.adi_step(u_in, s=s0 * kstar.astype(dt).astype(np.float64), nsteps=steps)
    loss_ref, du_ref, ds_ref = orc.adi_forward_backward(u_in, s0 * k_in, target, steps)
    dk_ref = s0 * ds_ref
    tk = _t(k_in.astype(dt)).requires_grad_(True)
    tu = _t(u_in.astype(dt)).requires_grad_(True)
    tt = _t(target.astype(dt))
    uT = autograd.adi(tu, s0 * tk, steps)
    loss = torch.sum((uT.double() - tt.double()) ** 2)
    loss.backward()
    assert abs(float(loss.detach()) - loss_ref) <= tol * loss_ref
    assert _nerr(tu.grad.cpu().numpy().astype(np.float64), du_ref) <= tol
    assert _nerr(tk.grad.cpu().numpy().astype(np.float64), dk_ref) <= tol


def test_tridsolve_fn_gradcheck(trid):
    from paper_2201_03950_amd import autograd

    g = torch.Generator().manual_seed(0)
    shape = (2, 5, 7)
    a = (torch.rand(shape, generator=g, dtype=torch.float64) * 2 - 1).cuda()
    c = (torch.rand(shape, generator=g, dtype=torch.float64) * 2 - 1).cuda()
    b = (a.abs() + c.abs() + 1 + torch.rand(shape, generator=g, dtype=torch.float64).cuda())
    d = torch.randn(shape, generator=g, dtype=torch.float64).cuda()
    for axis in (0, 1):
        args = [v.clone().requires_grad_(True) for v in (a, b, c, d)]
        assert torch.autograd.gradcheck(lambda *xs: autograd.gtsv(*xs, axis), args, eps=1e-6, atol=1e-8)


def test_tridsolve_s_fn_gradcheck(trid):
    from paper_2201_03950_amd import autograd

    g = torch.Generator().manual_seed(1)
    shape = (2, 6, 5)
    s = (0.3 * torch.rand(shape, generator=g, dtype=torch.float64) + 0.05).cuda().requires_grad_(True)
    d = torch.randn(shape, generator=g, dtype=torch.float64).cuda().requires_grad_(True)
    for axis in (0, 1):
        assert torch.autograd.gradcheck(lambda ss, dd: autograd.gtsv_s(ss, dd, axis), [s, d], eps=1e-6, atol=1e-8)


def test_adi_fn_gradcheck_small(trid):
    from paper_2201_03950_amd import autograd

    g = torch.Generator().manual_seed(2)
    shape = (1, 4, 5, 6)
    u = torch.rand(shape, generator=g, dtype=torch.float64).cuda().requires_grad_(True)
    s = (0.2 * torch.rand(shape, generator=g, dtype=torch.float64) + 0.05).cuda().requires_grad_(True)
    assert torch.autograd.gradcheck(lambda uu, ss: autograd.adi(uu, ss, 3), [u, s], eps=1e-6, atol=1e-8)


@pytest.mark.parametrize("dt", [np.float64, np.float32])
@pytest.mark.parametrize("dims,batch", [((20, 17, 13), 2), ((41, 30), 3), ((64, 32, 16), 1)])
def test_kept_step_matches_plain_step_and_recompute(trid, dt, dims, batch):
    """A step that keeps its intermediates gives the same field as the plain
    step, its last intermediate is the increment, and its reverse pass equals
    the recomputing one (same kernels, same arithmetic: bitwise)."""
    rng = np.random.default_rng(7 + sum(dims))
    shape = gen.mesh_shape(dims, batch)
    u = _t(rng.uniform(0, 1, shape).astype(dt))
    s = _t((0.2 * rng.lognormal(0.0, 0.5, shape)).astype(dt))
    u_plain = u.clone()
    trid.adi_step(u_plain, s=s, nsteps=1, stream=True)  # the per-step kernels the kept step uses
    u_keep = u.clone()
    ws = [torch.empty_like(u) for _ in range(len(dims))]
    trid.adi_step_keep(u_keep, s, *ws)
    assert torch.equal(u_keep, u_plain)
    assert torch.equal(u_keep, u + ws[-1])
    ubar = _t(rng.standard_normal(shape).astype(dt))
    sbar = _t(rng.standard_normal(shape).astype(dt))
    ub1, sb1 = ubar.clone(), sbar.clone()
    trid.adi_step_adjoint(u, s, ub1, sb1)
    ub2, sb2 = ubar.clone(), sbar.clone()
    trid.adi_step_adjoint_kept(u, s, ws[0], ws[1], ws[2] if len(ws) == 3 else None, ub2, sb2)
    assert torch.equal(ub1, ub2) and torch.equal(sb1, sb2)


@pytest.mark.parametrize("keep", [True, False])
def test_adi_fn_gradcheck_keep_modes(trid, keep):
    from paper_2201_03950_amd import autograd

    g = torch.Generator().manual_seed(3)
    shape = (1, 4, 5, 6)
    u = torch.rand(shape, generator=g, dtype=torch.float64).cuda().requires_grad_(True)
    s = (0.2 * torch.rand(shape, generator=g, dtype=torch.float64) + 0.05).cuda().requires_grad_(True)
    assert torch.autograd.gradcheck(lambda uu, ss: autograd.adi(uu, ss, 3, keep), [u, s], eps=1e-6, atol=1e-8)


def test_kept_step_argument_checks(trid):
    u = torch.zeros((1, 4, 5, 6), dtype=torch.float64, device="cuda")
    s = torch.full_like(u, 0.2)
    w = torch.empty_like(u)
    with pytest.raises(trid.TridError):
        trid.adi_step_keep(u, s, w, w, torch.empty_like(u))  # aliasing intermediates
    with pytest.raises(trid.TridError):
        trid.adi_step_keep(u, s, u, torch.empty_like(u), torch.empty_like(u))  # w1 aliases u


@pytest.mark.parametrize("dt", [np.float64, np.float32])
@pytest.mark.parametrize("dims,batch", [((20, 17, 13), 2), ((41, 30), 3), ((33, 9, 40), 1)])
def test_adi_step_adjoint_constant_s_matches_oracle(trid, orc, dt, dims, batch):
    """s NULL: the step with the constant s0; s_bar receives dL/ds_i at s = s0
    (the oracle's per-point gradient with every s_i = s0), s_bar NULL skips it."""
    rng = np.random.default_rng(5 + sum(dims))
    shape = gen.mesh_shape(dims, batch)
    s0 = float(dt(0.2))  # the value the FP32 path computes with
    u = rng.uniform(0, 1, shape).astype(dt)
    ubar = rng.standard_normal(shape).astype(dt)
    sbar0 = rng.standard_normal(shape).astype(dt)
    ub_ref, sb_ref = orc.adi_step_adjoint(u, np.full(shape, s0), ubar, sbar0)
    tub, tsb = _t(ubar), _t(sbar0)
    trid.adi_step_adjoint(_t(u), None, tub, tsb, s0=s0)
    tol = 1e-11 if dt == np.float64 else 1e-5
    assert _nerr(tub.cpu().numpy().astype(np.float64), ub_ref) <= tol
    assert _nerr(tsb.cpu().numpy().astype(np.float64), sb_ref) <= tol
    tub2 = _t(ubar)
    trid.adi_step_adjoint(_t(u), None, tub2, None, s0=s0)
    assert torch.equal(tub, tub2)
    # the constant step's own reverse equals the per-point one with s = s0 everywhere
    tub3, tsb3 = _t(ubar), _t(sbar0)
    trid.adi_step_adjoint(_t(u), _t(np.full(shape, s0, dtype=dt)), tub3, tsb3)
    assert torch.equal(tub, tub3) and torch.equal(tsb, tsb3)
