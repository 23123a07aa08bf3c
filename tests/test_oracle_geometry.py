"""Pins of the CPU reference's voxelisation and fluid-node numbering.

The paper images each electrode voxel as one grid block (Sec. 2, MAC grid).
The synthetic primitives are exact integers in 1/256 lattice units, so these
pins are exact: lattice-point counts of circles and spheres, a brute-force
recount, and the ordering of the compacted fluid list.
"""
import math

import numpy as np
import pytest

import oracle


def _gauss_count_2d(R):
    # lattice points (p, q) in Z^2 with p^2 + q^2 <= R^2, enumerated directly
    return sum(1 for p in range(-R, R + 1) for q in range(-R, R + 1) if p * p + q * q <= R * R)


def _gauss_count_3d(R):
    return sum(1 for p in range(-R, R + 1) for q in range(-R, R + 1) for s in range(-R, R + 1)
               if p * p + q * q + s * s <= R * R)


def test_gauss_circle_hand_values():
    # hand-checkable: R=1 -> centre + 4 axis points; R=2 -> 13
    assert _gauss_count_2d(1) == 5
    assert _gauss_count_2d(2) == 13
    assert _gauss_count_3d(1) == 7


@pytest.mark.parametrize("R", [1, 2, 3, 4, 5, 6, 7, 8])
def test_disk_voxel_count_is_lattice_point_count(R):
    # A disk centred on a voxel centre (cx = 256*a + 128) covers exactly the
    # integer lattice points of radius R around that voxel.
    nx, ny = 40, 40
    prim = np.array([[256 * R, 256 * 20 + 128, 256 * 20 + 128, 0]], dtype=np.int64)
    lab = oracle.voxelize(2, nx, ny, 1, 0, 0, prim)
    assert int((lab == 1).sum()) == _gauss_count_2d(R)


@pytest.mark.parametrize("R", [1, 2, 3, 4])
def test_sphere_voxel_count_is_lattice_point_count(R):
    n = 16
    c = 256 * 8 + 128
    prim = np.array([[256 * R, c, c, c]], dtype=np.int64)
    lab = oracle.voxelize(3, n, n, n, 0, 0, prim)
    assert int((lab == 1).sum()) == _gauss_count_3d(R)


def _brute_labels(dim, nx, ny, nz, walls_y, bx, prims):
    """Direct definition: a voxel is solid iff some periodic image of a
    primitive contains its centre; walls first; clip x to the interior."""
    nz = 1 if dim == 2 else nz
    lab = np.zeros((nz, ny, nx), dtype=np.uint8)
    if dim == 2 and walls_y:
        lab[:, 0, :] = 2
        lab[:, ny - 1, :] = 2
    for (r, cx, cy, cz) in prims:
        for k in range(nz):
            for j in range(ny):
                for i in range(bx, nx - bx):
                    if lab[k, j, i] == 2:
                        continue
                    hit = False
                    sy = [0] if (dim == 2 and walls_y) else [-1, 0, 1]
                    sz = [-1, 0, 1] if dim == 3 else [0]
                    for oy in sy:
                        for oz in sz:
                            X = 128 * (2 * i + 1) - cx
                            Y = 128 * (2 * (j + oy * ny) + 1) - cy
                            Z = (128 * (2 * (k + oz * nz) + 1) - cz) if dim == 3 else 0
                            if X * X + Y * Y + Z * Z <= r * r:
                                hit = True
                    if hit:
                        lab[k, j, i] = 1
    return lab.reshape(-1)


def test_brute_force_recount_2d_walls():
    prims, nf = oracle.disks(24, 16, 2, 1, 7, 0.7, 2.0, 3.5, 1.0)
    lab = oracle.voxelize(2, 24, 16, 1, 1, 2, prims)
    ref = _brute_labels(2, 24, 16, 1, 1, 2, prims)
    assert np.array_equal(lab, ref)
    # the generator's own fluid count agrees with the voxelisation
    assert int((lab == 0).sum()) == nf


def test_brute_force_recount_2d_periodic():
    prims, nf = oracle.disks(24, 16, 2, 0, 11, 0.75, 2.0, 3.0, 1.0)
    lab = oracle.voxelize(2, 24, 16, 1, 0, 2, prims)
    assert np.array_equal(lab, _brute_labels(2, 24, 16, 1, 0, 2, prims))
    assert int((lab == 0).sum()) == nf


def test_brute_force_recount_3d():
    prims = oracle.spheres(14, 12, 12, 2, 5, 0.6, 1.5, 2.5)
    assert prims.shape[0] > 3
    lab = oracle.voxelize(3, 14, 12, 12, 0, 2, prims)
    assert np.array_equal(lab, _brute_labels(3, 14, 12, 12, 0, 2, prims))


def test_compaction_order_and_map():
    rng = np.random.default_rng(3)
    lab = rng.choice(np.array([0, 1, 2], dtype=np.uint8), size=1000, p=[0.5, 0.3, 0.2])
    m, f = oracle.compact(lab)
    fluid = np.flatnonzero(lab == 0)
    assert np.array_equal(f, fluid)                       # lexicographic, x fastest
    assert np.array_equal(m[fluid], np.arange(fluid.size))
    assert np.all(m[lab == 1] == -1) and np.all(m[lab == 2] == -2)


def test_rsa_disks_respect_gap_and_porosity():
    nx, ny = 128, 64
    prims, nf = oracle.disks(nx, ny, 2, 1, 2110, 0.7, 4.0, 8.0, 2.0)
    lab = oracle.voxelize(2, nx, ny, 1, 1, 2, prims)
    phi = (lab == 0).sum() / lab.size
    assert phi <= 0.7 and phi > 0.6
    # buffers (2 planes at each x end) are fluid except the wall rows
    g = lab.reshape(ny, nx)
    assert np.all(g[1:-1, :2] == 0) and np.all(g[1:-1, -2:] == 0)
    for a in range(len(prims)):
        for b in range(a + 1, len(prims)):
            d2 = (prims[a, 1] - prims[b, 1]) ** 2 + (prims[a, 2] - prims[b, 2]) ** 2
            assert d2 >= (prims[a, 0] + prims[b, 0] + 512) ** 2
    assert prims[:, 0].min() >= 4 * 256 and prims[:, 0].max() <= 8 * 256


def test_sphere_count_formula():
    # E[V] = (4 pi / 3) (b^4 - a^4) / (4 (b - a)) = 424.1 voxels for r in [3, 6]
    ev = 4 * math.pi / 3 * (6 ** 4 - 3 ** 4) / (4 * 3)
    assert abs(ev - 424.115) < 1e-3
    nx = ny = nz = 128
    nbuf = 2 * 2 * ny * nz
    nint = nx * ny * nz - nbuf
    phi_int = (0.5 * nx * ny * nz - nbuf) / nint
    n_expected = round(-math.log(phi_int) * nint / ev)
    assert oracle.sphere_count(nx, ny, nz, 2, 0.5, 3.0, 6.0) == n_expected


def test_boolean_model_porosity_close_to_target():
    n = 48
    prims = oracle.spheres(n, n, n, 2, 2110, 0.5, 3.0, 6.0)
    lab = oracle.voxelize(3, n, n, n, 0, 2, prims)
    phi = (lab == 0).mean()
    assert abs(phi - 0.5) < 0.05


def test_generator_is_deterministic_and_seed_sensitive():
    a = oracle.spheres(32, 32, 32, 2, 1, 0.5, 3.0, 6.0)
    b = oracle.spheres(32, 32, 32, 2, 1, 0.5, 3.0, 6.0)
    c = oracle.spheres(32, 32, 32, 2, 2, 0.5, 3.0, 6.0)
    assert np.array_equal(a, b)
    assert not np.array_equal(a, c)


def test_splitmix64_reference_vector(oracle_lib):
    # SplitMix64 first outputs from seed 0, as printed with the published
    # reference implementation (Vigna's splitmix64.c): 0xE220A8397B1DCDAF, ...
    import ctypes
    st = ctypes.c_uint64(0)
    oracle_lib.geomgen_splitmix64.restype = ctypes.c_uint64
    oracle_lib.geomgen_splitmix64.argtypes = [ctypes.c_void_p]
    x0 = oracle_lib.geomgen_splitmix64(ctypes.byref(st))
    x1 = oracle_lib.geomgen_splitmix64(ctypes.byref(st))
    assert x0 == 0xE220A8397B1DCDAF
    assert x1 == 0x6E789E6AA1B965F4


# ---------------------------------------------------------------- fibres (Sec. 5)

def _brute_fibres(nx, ny, nz, bx, fib):
    """Direct definition in floating point on small lattices: a voxel centre
    within r of the fibre's infinite core line (distance by projection)."""
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    c = np.stack([x + 0.5, y + 0.5, z + 0.5], axis=-1) * 256.0
    lab = np.zeros((nz, ny, nx), dtype=np.uint8)
    for r, ox, oy, oz, dx, dy, dz, _ in fib:
        d = np.array([dx, dy, dz], dtype=np.float64)
        v = c - np.array([ox, oy, oz], dtype=np.float64)
        t = v @ d / (d @ d)
        dist2 = ((v - t[..., None] * d) ** 2).sum(-1)
        lab[dist2 <= float(r) ** 2 * (1 + 1e-12)] = 1
    lab[:, :, :bx] = 0
    lab[:, :, nx - bx:] = 0
    return lab.reshape(-1)


@pytest.mark.parametrize("R", [1, 2, 3, 4])
def test_axis_fibre_covers_the_lattice_disk(R):
    # a fibre along x through voxel centres covers, in every interior plane,
    # exactly the lattice points of radius R
    n, bx = 20, 2
    c = 256 * 10 + 128
    fib = np.array([[256 * R, 256 * 3, c, c, 1024, 0, 0, 0]], dtype=np.int64)
    lab = oracle.voxelize_fibres(n, n, n, bx, fib)
    assert int((lab == 1).sum()) == (n - 2 * bx) * _gauss_count_2d(R)


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_fibre_voxels_brute_force(seed):
    nx, ny, nz, bx = 26, 21, 17, 2
    fib = oracle.fibres(nx, ny, nz, bx, seed, 0.7, 1.5, 3.0)
    assert 3 <= fib.shape[0] <= 200
    lab = oracle.voxelize_fibres(nx, ny, nz, bx, fib)
    assert np.array_equal(lab, _brute_fibres(nx, ny, nz, bx, fib))


def test_fibre_draws_ranges_and_isotropy():
    nx, ny, nz, bx = 150, 150, 150, 2
    fib = oracle.fibres(nx, ny, nz, bx, 2110, 0.5, 1.0, 4.0)
    r, o, d = fib[:, 0], fib[:, 1:4], fib[:, 4:7].astype(np.float64)
    assert r.min() >= 256 and r.max() <= 1024
    assert o[:, 0].min() >= 256 * bx and o[:, 0].max() < 256 * (nx - bx)
    assert o[:, 1:].min() >= 0 and o[:, 1].max() < 256 * ny and o[:, 2].max() < 256 * nz
    q = (d ** 2).sum(1)
    assert q.min() > 0 and q.max() <= 1024 ** 2
    u = d / np.sqrt(q)[:, None]
    n = u.shape[0]
    # isotropic directions: mean ~ 0, second moment ~ I/3 (a few standard errors)
    assert np.abs(u.mean(0)).max() < 4 / np.sqrt(3 * n)
    assert np.abs(u.T @ u / n - np.eye(3) / 3).max() < 4 * np.sqrt(4 / 45 / n)


@pytest.mark.parametrize("phi,r", [(0.5, 2.0), (0.6, 3.0), (0.7, 4.0), (0.8, 2.0)])
def test_fibre_porosity_close_to_target(phi, r):
    n, bx = 96, 2
    fib = oracle.fibres(n, n, n, bx, 2110, phi, r, r)
    lab = oracle.voxelize_fibres(n, n, n, bx, fib)
    assert abs((lab == 0).mean() - phi) < 0.03


def test_fibre_generator_is_deterministic_and_rejects_bad_input():
    a = oracle.fibres(40, 30, 30, 2, 9, 0.6, 2.0, 2.0)
    b = oracle.fibres(40, 30, 30, 2, 9, 0.6, 2.0, 2.0)
    c = oracle.fibres(40, 30, 30, 2, 10, 0.6, 2.0, 2.0)
    assert np.array_equal(a, b) and not np.array_equal(a, c)
    for bad in ((2000, 30, 30, 2, 9, 0.6, 2.0, 2.0), (40, 30, 30, 2, 9, 1.0, 2.0, 2.0),
                (40, 30, 30, 2, 9, 0.6, 2.0, 80.0)):
        with pytest.raises(RuntimeError):
            oracle.fibres(*bad)
