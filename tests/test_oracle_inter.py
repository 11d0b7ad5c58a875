"""Pins for the oracle's intermolecular grid term (trilinear interpolation).

Checked against: node values (exact), fields in span{1, x, y, z, xy, yz, zx,
xyz} that trilinear interpolation reproduces exactly together with their
analytic gradients, a separable (lerp-along-x, then y, then z) evaluation
written independently, central finite differences, and the outside-the-box
penalty's value and slope at the box face.
"""
import numpy as np
import pytest

from oracle import dock_ref as R
from paper_2410_10447_amd import synth

H = 0.375


def _box(n):
    half = (n - 1) * H / 2
    return np.array([-half, -half, -half])


def test_exact_at_nodes():
    grd = synth.grids(20, 3, 5)
    rng = np.random.default_rng(0)
    idx = rng.integers(0, 20, (200, 3))
    x = grd.origin + H * idx.astype(float)
    for m in range(3):
        v, _ = R.trilinear(grd.maps[m], grd.origin, H, x)
        want = grd.maps[m][idx[:, 2], idx[:, 1], idx[:, 0]].astype(float)
        assert np.array_equal(v, want)


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_trilinear_fields_reproduced(seed):
    n = 16
    o = _box(n)
    rng = np.random.default_rng(seed)
    c = rng.normal(size=8)
    ax = o[0] + H * np.arange(n)
    Z, Y, X = np.meshgrid(ax, ax, ax, indexing="ij")

    def f(x, y, z):
        return (c[0] + c[1] * x + c[2] * y + c[3] * z + c[4] * x * y + c[5] * y * z
                + c[6] * z * x + c[7] * x * y * z)

    def grad(x, y, z):
        return np.stack([c[1] + c[4] * y + c[6] * z + c[7] * y * z,
                         c[2] + c[4] * x + c[5] * z + c[7] * x * z,
                         c[3] + c[5] * y + c[6] * x + c[7] * x * y], axis=-1)

    mp = f(X, Y, Z)
    pts = rng.uniform(o[0] + 1e-3, -o[0] - 1e-3, (500, 3))
    v, g = R.trilinear(mp, o, H, pts)
    assert np.abs(v - f(*pts.T)).max() < 1e-11
    assert np.abs(g - grad(*pts.T)).max() < 1e-10


def _separable(mp, o, h, p):
    """Independent evaluation: lerp along x, then y, then z (one point)."""
    nz, ny, nx = mp.shape
    u = (p - o) / h
    i = [min(max(int(np.floor(u[a])), 0), (nx, ny, nz)[a] - 2) for a in range(3)]
    f = [u[a] - i[a] for a in range(3)]
    c = mp[i[2]:i[2] + 2, i[1]:i[1] + 2, i[0]:i[0] + 2].astype(float)
    cx = c[:, :, 0] + f[0] * (c[:, :, 1] - c[:, :, 0])
    cy = cx[:, 0] + f[1] * (cx[:, 1] - cx[:, 0])
    return cy[0] + f[2] * (cy[1] - cy[0])


def test_eight_corner_sum_matches_separable_lerps():
    grd = synth.grids(24, 2, 7)
    rng = np.random.default_rng(4)
    pts = rng.uniform(grd.origin[0], -grd.origin[0], (300, 3))
    v, _ = R.trilinear(grd.maps[0], grd.origin, H, pts)
    ref = np.array([_separable(grd.maps[0], grd.origin, H, p) for p in pts])
    assert np.abs(v - ref).max() <= 1e-12 * max(1.0, np.abs(ref).max())


def test_gradient_finite_difference_inside_cells():
    grd = synth.grids(24, 2, 8)
    rng = np.random.default_rng(5)
    # points away from cell faces so the FD stencil stays in one cell
    cells = rng.integers(1, 22, (200, 3)).astype(float)
    frac = rng.uniform(0.1, 0.9, (200, 3))
    pts = grd.origin + H * (cells + frac)
    _, g = R.trilinear(grd.maps[1], grd.origin, H, pts)
    h = 1e-6
    for a in range(3):
        e = np.zeros(3); e[a] = h
        vp, _ = R.trilinear(grd.maps[1], grd.origin, H, pts + e)
        vm, _ = R.trilinear(grd.maps[1], grd.origin, H, pts - e)
        fd = (vp - vm) / (2 * h)
        assert np.abs(fd - g[:, a]).max() <= 1e-6 * max(1.0, np.abs(g[:, a]).max())


def test_outside_box_clamps_and_penalty():
    n = 10
    o = _box(n)
    hi = -o
    mp = np.arange(n ** 3, dtype=float).reshape(n, n, n)
    p_in = np.array([[hi[0], 0.1, 0.2]])
    p_out = np.array([[hi[0] + 0.7, 0.1, 0.2]])
    v_in, g_in = R.trilinear(mp, o, H, p_in)
    v_out, g_out = R.trilinear(mp, o, H, p_out)
    assert v_in[0] == v_out[0]           # value taken at the clamped point
    assert g_out[0, 0] == 0.0 and g_in[0, 0] != 0.0
    assert np.array_equal(g_out[0, 1:], g_in[0, 1:])
    pen, gp = R.outside_penalty(p_out, (n, n, n), o, H)
    assert np.isclose(pen[0], 100.0 * 0.7 ** 2, rtol=1e-14)
    assert np.isclose(gp[0, 0], 2 * 100.0 * 0.7, rtol=1e-14)
    # C^1 at the face: value and slope -> 0 as the point approaches the box
    for d in (1e-3, 1e-6):
        pen, gp = R.outside_penalty(np.array([[hi[0] + d, 0, 0]]), (n, n, n), o, H)
        assert pen[0] <= 100 * d * d * (1 + 1e-9) and abs(gp[0, 0]) <= 200 * d * (1 + 1e-9)
    pen, gp = R.outside_penalty(np.array([[0.0, 0.0, 0.0]]), (n, n, n), o, H)
    assert pen[0] == 0.0 and not gp.any()


def test_atom_energy_combines_three_maps():
    """e_i = map[cls] + q map_e + |q| map_d, checked at grid nodes."""
    lig = synth.ligand(6, 0, 3)
    grd = synth.grids(16, 10, 9)
    p = R.prepare(lig, synth.force_field())
    idx = np.array([[3, 4, 5], [7, 7, 7], [1, 2, 3], [10, 11, 12], [5, 5, 9], [8, 2, 6]])
    x = (grd.origin + H * idx)[None]
    e, _ = R.inter_terms(p, grd, x)
    m = grd.maps.astype(float)
    for i in range(6):
        ix, iy, iz = idx[i]
        want = (m[lig.cls[i], iz, iy, ix] + lig.charge[i] * m[8, iz, iy, ix]
                + abs(lig.charge[i]) * m[9, iz, iy, ix])
        assert np.isclose(e[0, i], want, rtol=1e-15, atol=1e-12)
