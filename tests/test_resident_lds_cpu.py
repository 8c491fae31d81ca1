"""Host-side check of the LDS-resident 2D loops' shared-memory accesses (CPU).

The resident kernels (the 2D ADI loop and the Hundsdorfer-Verwer steps of the
SLV stand-in) keep each mesh in one workgroup's LDS and separate their phases
by workgroup barriers only.  This test replays, on the host, every thread's
LDS addresses of every phase -- the same thread-to-(line, tile) mapping,
layout formula and guarded reads as the kernels, with the layout the library
itself chooses (trid_resident_layout) -- and checks, for each phase:
  - every address lies inside its array (also the fallback addresses of
    guarded reads);
  - every mesh point of an array the phase writes is written exactly once;
  - no thread reads (with its guard true) a point another thread writes in the
    same phase, and no two threads write the same point (no barrier orders
    them).
It covers the automatic layouts and forced tile sizes, with the thread count
the library launches and with 1024 threads for 8-row tiles.
"""

import ctypes

import numpy as np
import pytest

from paper_2201_03950_amd import _binding as B


@pytest.fixture(scope="module")
def lib():
    import os

    if not os.path.exists(B.LIB_PATH):
        from paper_2201_03950_amd import build

        build.build()
    return B.load_library()


@pytest.fixture()
def h(lib):
    hp = ctypes.c_void_p()
    assert lib.trid_create(ctypes.byref(hp)) == 0
    yield hp
    lib.trid_destroy(hp)


def layout(lib, h, f64, nx, ny, hv, per_point, force_m=0):
    out = (ctypes.c_int64 * 10)()
    rc = lib.trid_resident_layout(h, 1 if f64 else 0, nx, ny, 1 if hv else 0, 1 if per_point else 0, force_m, out, 10)
    if rc != 0:
        return None
    keys = ("m", "px", "py", "ldx", "skw", "tp", "region", "cl", "threads", "bytes")
    return dict(zip(keys, (int(v) for v in out)))


def res_at(g, y, x):
    return y * g["ldx"] + (y // g["m"]) * g["skw"] + x + (x // g["m"] if g["tp"] else 0)


class Phase:
    """LDS accesses of one phase: (array, index, thread) for reads whose guard
    holds, for every read's address, and for writes."""

    def __init__(self):
        self.reads, self.addrs, self.writes = [], [], []

    def read(self, arr, idx, ok, fallback, t):
        idx = np.where(ok, idx, fallback)
        self.addrs.append((arr, idx))
        self.reads.append((arr, idx[ok], t[ok]))

    def write(self, arr, idx, ok, t):
        self.writes.append((arr, idx[ok], t[ok]))
        self.addrs.append((arr, idx[ok]))


def x_phase(g, nx, ny, nt, ph, src, reads_own, writes_own, coef_arrays):
    """Thread t owns tile t % px of row yb + t / px; reads the 3 x (M + 2)
    neighbourhood of src, its own points of reads_own and coef_arrays, writes
    its own points of writes_own."""
    m, px = g["m"], g["px"]
    t = np.arange(nt)
    la = nt // px
    for yb in range(0, ny, la):
        y, p = yb + t // px, t % px
        x0 = p * m
        live = y < ny
        ya = np.where(live, y, 0)
        xc = np.where(x0 < nx, x0, 0)  # tiles past the line's end address column 0
        base = res_at(g, ya, xc)
        dn = res_at(g, ya + 1, xc) - base
        ds = base - res_at(g, np.where(ya > 0, ya - 1, 0), xc)
        hn, hs = live & (y + 1 < ny), live & (y > 0)
        hw, he = live & (x0 > 0) & (x0 < nx), live & (x0 + m < nx)
        for off, ok in ((-ds, hs), (0, live), (dn, hn)):
            ph.read(src, base + off - 1 - g["tp"], ok & hw, base, t)
            for k in range(m):
                ph.read(src, base + off + k, ok & (x0 + k < nx), base, t)
            ph.read(src, base + off + m + g["tp"], ok & he, base, t)
        for k in range(m):
            v = live & (x0 + k < nx)
            for arr in list(reads_own) + list(coef_arrays):
                ph.read(arr, base + k, v, base, t)
            for arr in writes_own:
                ph.write(arr, base + k, v, t)


def y_phase(g, nx, ny, nt, ph, src, src_halo, reads_own, writes_own, coef_arrays):
    """Thread t owns tile t % py of column xb + t / py; reads its column of src
    (with one point above and below when src_halo), its own points of reads_own
    and coef_arrays, writes its own points of writes_own."""
    m, py = g["m"], g["py"]
    t = np.arange(nt)
    lb = nt // py
    for xb in range(0, nx, lb):
        x, q = xb + t // py, t % py
        y0 = q * m
        live = x < nx
        xa = np.where(live, x, 0)
        if src_halo:
            v = live & (y0 > 0) & (y0 < ny)
            o = res_at(g, np.where(v, y0 - 1, 0), xa)
            ph.read(src, o, v, o, t)
        for k in range(m):
            v = live & (y0 + k < ny)
            off = res_at(g, np.where(v, y0 + k, 0), xa)
            ph.read(src, off, v, off, t)
            for arr in list(reads_own) + list(coef_arrays):
                ph.read(arr, off, v, off, t)
            for arr in writes_own:
                ph.write(arr, off, v, t)
        if src_halo:
            v = live & (y0 + m < ny)
            o = res_at(g, np.where(v, y0 + m, 0), xa)
            ph.read(src, o, v, o, t)


def check_phase(g, nx, ny, ph, name):
    region = g["region"]
    for arr, idx in ph.addrs:
        assert idx.size == 0 or (idx.min() >= 0 and idx.max() < region), (name, arr, idx.min(), idx.max(), region)
    yy, xx = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
    points = np.sort(res_at(g, yy, xx).ravel())
    assert np.unique(points).size == points.size, "two mesh points share an LDS slot"
    is_point = np.zeros(region, dtype=bool)
    is_point[points] = True
    for arr, idx, thr in ph.reads:  # a read whose guard holds reads a point of the mesh
        assert is_point[idx].all(), (name, arr, "guarded read of a slot outside the mesh", int(idx[~is_point[idx]][0]))
    writer = {}
    for arr in sorted({a for a, _, _ in ph.writes}):
        idx = np.concatenate([i for a, i, _ in ph.writes if a == arr])
        thr = np.concatenate([tt for a, _, tt in ph.writes if a == arr])
        order = np.argsort(idx, kind="stable")
        assert np.array_equal(idx[order], points), (name, arr, "points not written exactly once")
        w = np.full(region, -1)
        w[idx] = thr
        writer[arr] = w
    for arr, idx, thr in ph.reads:
        if arr in writer and idx.size:
            other = writer[arr][idx]
            bad = (other >= 0) & (other != thr)
            assert not bad.any(), (name, arr, "read of a point another thread writes in the same phase",
                                   int(idx[bad][0]), int(thr[bad][0]), int(other[bad][0]))


def check_hv(g, nx, ny, nt):
    U, R, Z, CB, CA, CC = range(6)
    coef_x = [CA, CB, CC] if g["cl"] == 2 else ([CB] if g["cl"] == 1 else [])
    coef_y = [CB] if g["cl"] >= 1 else []
    # A: from U, Z = U + dt/2 F(U) and R = X^-1(...)
    ph = Phase()
    x_phase(g, nx, ny, nt, ph, U, [], [Z, R], coef_x)
    check_phase(g, nx, ny, ph, "hv A")
    # B: R = Y^-1 (R - th dt F2(U)), in place
    ph = Phase()
    y_phase(g, nx, ny, nt, ph, U, True, [R], [R], coef_y)
    check_phase(g, nx, ny, ph, "hv B")
    # C: from R, Z = X^-1 (Z + ...), in place
    ph = Phase()
    x_phase(g, nx, ny, nt, ph, R, [Z], [Z], coef_x)
    check_phase(g, nx, ny, ph, "hv C")
    # D: U = Y^-1 (Z - th dt F2(R))
    ph = Phase()
    y_phase(g, nx, ny, nt, ph, R, True, [Z], [U], coef_y)
    check_phase(g, nx, ny, ph, "hv D")


def check_adi(g, nx, ny, nt, per_point):
    U, D, S = range(3)
    ph = Phase()
    x_phase(g, nx, ny, nt, ph, U, [], [D], [S] if per_point else [])
    check_phase(g, nx, ny, ph, "adi A")
    ph = Phase()
    y_phase(g, nx, ny, nt, ph, D, False, [U], [U], [S] if per_point else [])
    check_phase(g, nx, ny, ph, "adi B")


MESHES = [(33, 70), (100, 50), (40, 20), (128, 128), (70, 33), (8, 128), (127, 9), (64, 64), (96, 96), (1, 5)]


@pytest.mark.parametrize("f64", [True, False])
@pytest.mark.parametrize("nx,ny", MESHES, ids=["%dx%d" % m for m in MESHES])
def test_hv_resident_lds_accesses(lib, h, f64, nx, ny):
    for force in (0, 8, 10, 12, 14):
        g = layout(lib, h, f64, nx, ny, True, False, force)
        if g is None:
            continue
        for nt in sorted({g["threads"], 512, 1024 if g["m"] == 8 else 512}):
            if nt // g["px"] < 1 or nt // g["py"] < 1:
                continue
            check_hv(g, nx, ny, nt)


@pytest.mark.parametrize("per_point", [False, True])
@pytest.mark.parametrize("f64", [True, False])
@pytest.mark.parametrize("nx,ny", MESHES, ids=["%dx%d" % m for m in MESHES])
def test_adi_resident_lds_accesses(lib, h, f64, per_point, nx, ny):
    for force in (0, 8, 14):
        g = layout(lib, h, f64, nx, ny, False, per_point, force)
        if g is None:
            continue
        for nt in sorted({g["threads"], 512, 1024 if g["m"] == 8 else 512}):
            check_adi(g, nx, ny, nt, per_point)


def test_layout_query_argument_checks(lib, h):
    out = (ctypes.c_int64 * 10)()
    assert lib.trid_resident_layout(h, 1, 33, 70, 1, 0, 0, out, 10) == 0
    assert out[0] in (8, 10, 12, 14) and out[8] in (64, 128, 256, 512, 1024)
    assert lib.trid_resident_layout(h, 1, 33, 70, 1, 0, 9, out, 10) == 1  # no such tile size
    assert lib.trid_resident_layout(h, 1, 200, 70, 1, 0, 0, out, 10) == 4  # line longer than 128
    assert lib.trid_resident_layout(h, 1, 33, 70, 1, 0, 0, None, 10) == 1
    assert lib.trid_resident_layout(h, 1, 33, 70, 1, 0, 0, out, 9) == 1
    assert lib.trid_resident_layout(None, 1, 33, 70, 1, 0, 0, out, 10) == 1
