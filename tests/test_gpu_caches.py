"""Bounded caches of captured launches, and the ordering of one handle's calls
across streams (GPU)."""

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


def _field_err(x, ref):
    return float(np.max(np.abs(x - ref)) / np.max(np.abs(ref)))


def test_adi_graph_cache_stays_bounded_under_moving_pointers(trid, orc):
    """Every call on a new tensor captures a new graph; the cache keeps at most
    its capacity, evicted graphs are recaptured when their tensor comes back,
    and every replay gives the oracle's step."""
    u0 = gen.adi3d_field((20, 18, 16), seed=3)
    ref = orc.adi_step(u0, s0=0.2, nsteps=2)
    cap = trid.cache_report()["adi_graph_cap"]
    us = [_t(u0) for _ in range(cap + 8)]
    for u in us:
        trid.adi_step(u, s0=0.2, nsteps=2, graph=True)
        assert trid.cache_report()["adi_graphs"] <= cap
    for u in us:
        assert _field_err(u.cpu().numpy(), ref) <= 1e-12
    # the first tensors' graphs were evicted: a new call recaptures and is still right
    us[0].copy_(_t(u0))
    trid.adi_step(us[0], s0=0.2, nsteps=2, graph=True)
    assert _field_err(us[0].cpu().numpy(), ref) <= 1e-12
    assert trid.cache_report()["adi_graphs"] <= cap


def test_adi_graph_key_includes_the_forced_tile_plan(trid, orc):
    u0 = gen.adi3d_field((64, 16, 8), seed=4)
    ref = orc.adi_step(u0, s0=0.2, nsteps=1)
    u = _t(u0)
    # size the handle's workspace for this mesh first (growing it drops every
    # captured graph), so that the count below sees only the two new captures
    trid.adi_step(_t(u0), s0=0.2, nsteps=1)
    n0 = trid.cache_report()["adi_graphs"]
    trid.set_tile(16, 0)
    try:
        trid.adi_step(u, s0=0.2, nsteps=1, graph=True)
        u.copy_(_t(u0))
        trid.set_tile(8, 0)
        trid.adi_step(u, s0=0.2, nsteps=1, graph=True)  # a different plan: a new capture
    finally:
        trid.set_tile(0, 0)
    assert trid.cache_report()["adi_graphs"] >= min(n0 + 2, trid.cache_report()["adi_graph_cap"])
    assert _field_err(u.cpu().numpy(), ref) <= 1e-12


def test_varlen_graph_cache_stays_bounded(trid, orc):
    a32, b32, c32, d64, off = gen.varlen_batch(300, 32, 2048, seed=140)
    ref = orc.gtsv_varlen(a32, b32, c32, d64, off)
    a, b, c, d = (_t(v.astype(np.float64)) for v in (a32, b32, c32, d64))
    cap = trid.cache_report()["varlen_graph_cap"]
    xs = [torch.zeros_like(d) for _ in range(cap + 5)]
    for x in xs:
        trid.gtsv_varlen(trid.PREC_F64, a, b, c, d, x, off)
    rep = trid.cache_report()
    assert 1 <= rep["varlen_schedules"] <= rep["varlen_schedule_cap"]
    assert rep["varlen_graphs"] <= cap * rep["varlen_schedules"]
    for x in xs:
        got = x.cpu().numpy()
        assert float(np.max(np.abs(got - ref)) / np.max(np.abs(ref))) <= 1e-12


def test_adi_steps_on_two_streams_share_the_workspace(trid, orc):
    """Two meshes stepped by one handle on alternating streams: both steps use
    the handle's d workspace, and the stream switch orders them."""
    dims = (96, 80, 64)
    u1, u2 = gen.adi3d_field(dims, seed=5), gen.adi3d_field(dims, seed=6)
    r1, r2 = orc.adi_step(u1, s0=0.2, nsteps=3), orc.adi_step(u2, s0=0.2, nsteps=3)
    t1, t2 = _t(u1), _t(u2)
    sa, sb = torch.cuda.Stream(), torch.cuda.Stream()
    torch.cuda.synchronize()
    for _ in range(3):
        with torch.cuda.stream(sa):
            trid.adi_step(t1, s0=0.2, nsteps=1)
        with torch.cuda.stream(sb):
            trid.adi_step(t2, s0=0.2, nsteps=1)
    torch.cuda.synchronize()
    assert _field_err(t1.cpu().numpy(), r1) <= 1e-12
    assert _field_err(t2.cpu().numpy(), r2) <= 1e-12
