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
