"""Simple-connectivity check of Omega (Sec. 2 restricts the method to
contourwise simply connected domains).  The library's Betti numbers of the
voxel union are pinned by textbook solids with known numbers (ball, shell,
solid torus, figure eight, corner-touching voxels) and by an independent
count on random masks: scipy's component labelling for b0 and b2 and an
explicit cell-by-cell Euler characteristic."""
import numpy as np
import pytest
from scipy import ndimage

from oracle import geometry, grid
from paper_1803_01346_amd import scfft, workloads


def _betti(mask):
    return scfft.scfft_mask_betti_host(mask)


def _ring(n=12, lo=3, hi=9, z=(5, 7)):
    m = np.zeros((n, n, n), np.uint8)
    m[z[0]:z[1], lo:hi, lo:hi] = 1
    m[z[0]:z[1], lo + 2:hi - 2, lo + 2:hi - 2] = 0
    return m


def test_textbook_solids():
    n = 12
    assert _betti(np.zeros((n, n, n), np.uint8)) == (0, 0, 0)
    assert _betti(np.ones((n, n, n), np.uint8)) == (1, 0, 0)
    one = np.zeros((n, n, n), np.uint8)
    one[4, 5, 6] = 1
    assert _betti(one) == (1, 0, 0)
    ball = np.zeros((n, n, n), np.uint8)
    ball[2:10, 2:10, 2:10] = 1
    assert _betti(ball) == (1, 0, 0)
    shell = ball.copy()
    shell[4:8, 4:8, 4:8] = 0                     # a closed cavity
    assert _betti(shell) == (1, 0, 1)
    assert _betti(_ring()) == (1, 1, 0)           # solid torus
    eight = _ring(n=16, lo=3, hi=13)
    eight[5:7, 5:11, 7:9] = 1                     # a bar splitting the hole in two
    assert _betti(eight) == (1, 2, 0)
    two = np.zeros((n, n, n), np.uint8)
    two[1:4, 1:4, 1:4] = 1
    two[6:9, 6:9, 6:9] = 1
    assert _betti(two) == (2, 0, 0)
    two[4, 4, 4] = two[5, 5, 5] = 1                # a chain joined at corners
    assert _betti(two) == (1, 0, 0)


def test_corner_and_edge_contact():
    # four voxels of one layer meeting pairwise at vertical edges around an
    # empty voxel: a ring (the closed voxels touch), whose hole opens upwards
    m = np.zeros((5, 5, 5), np.uint8)
    for y, x in ((1, 2), (2, 1), (3, 2), (2, 3)):
        m[2, y, x] = 1
    assert _betti(m) == (1, 1, 0)
    # two voxels touching at one corner: one component, no hole
    m = np.zeros((4, 4, 4), np.uint8)
    m[1, 1, 1] = m[2, 2, 2] = 1
    assert _betti(m) == (1, 0, 0)
    # Omega reaching the grid border still has the unbounded complement outside
    m = np.zeros((6, 6, 6), np.uint8)
    m[:, :, :] = 1
    m[2:4, 2:4, :] = 0                             # a tunnel through the whole box
    assert _betti(m) == (1, 1, 0)


def _euler(mask):
    """chi = V - E + F - C counted cell by cell on the lattice of voxel corners."""
    p = np.pad(mask != 0, 1)
    nz, ny, nx = p.shape
    V = E = F = 0
    # cells indexed by lattice points; a cell is in the union when any voxel
    # containing it is filled (voxel (i, j, k) of p spans corners i..i+1)
    def occ(sx, sy, sz):
        # OR over the voxels around each cell of the given extent: s = 1 means
        # the cell spans that axis (one voxel index), 0 that it sits on a
        # lattice plane (two voxel indices: below and above)
        out = np.zeros((nz - 1, ny - 1, nx - 1), bool)
        for dz in ((0,) if sz else (0, 1)):
            for dy in ((0,) if sy else (0, 1)):
                for dx in ((0,) if sx else (0, 1)):
                    out |= p[dz:dz + nz - 1, dy:dy + ny - 1, dx:dx + nx - 1]
        return int(out.sum())
    V = occ(0, 0, 0)
    E = occ(1, 0, 0) + occ(0, 1, 0) + occ(0, 0, 1)
    F = occ(1, 1, 0) + occ(1, 0, 1) + occ(0, 1, 1)
    C = int(mask.astype(bool).sum())
    return V - E + F - C


@pytest.mark.parametrize("seed", range(6))
def test_random_masks_against_independent_count(seed):
    rng = np.random.default_rng(seed)
    shape = (7 + seed, 9, 11 - seed)
    mask = (rng.random(shape) < 0.35 + 0.05 * seed).astype(np.uint8)
    b0, b1, b2 = _betti(mask)
    _, n26 = ndimage.label(mask, structure=np.ones((3, 3, 3)))
    comp, n6 = ndimage.label(np.pad(mask == 0, 1, constant_values=True), structure=ndimage.generate_binary_structure(3, 1))
    outer = comp[0, 0, 0]
    assert b0 == n26
    assert b2 == n6 - (1 if outer else 0)
    assert b1 == b0 + b2 - _euler(mask)
    assert b1 >= 0


def _lib_mask(shapes, n=(64, 64, 64), L=(1.2, 1.2, 1.2)):
    orc = geometry.voxelize(grid.Grid(n, L), shapes)
    l = 1e-3
    g = scfft.make_grid(n, [v * l for v in L])
    m = scfft.make_material(25, 1e8, 1e-4, 20, l)
    sh, ns = scfft.make_shapes(shapes, l)
    lib = scfft.scfft_voxelize_host(g, m, sh, ns)
    assert np.array_equal(lib, orc)
    return lib


def test_workload_shapes():
    assert _betti(_lib_mask(workloads.shape_cube(0.8))) == (1, 0, 0)
    assert _betti(_lib_mask(workloads.shape_cup(1.0, 0.8, 1.6, 0.2))) == (1, 0, 0)
    assert _betti(_lib_mask(workloads.shape_sphere(1.0))) == (1, 0, 0)
    # the lens: the radial slit makes the bored cylinder simply connected,
    # without it the bore leaves a closed contour around it
    lens = workloads.shape_lens(1.0, 4.0 / 3.0, 0.2, 0.1)
    assert _betti(_lib_mask(lens)) == (1, 0, 0)
    assert _betti(_lib_mask(lens[:2])) == (1, 1, 0)
    # a tube open at both ends
    tube = [workloads.prim("cylinder", "add", (0, 0, 0), (1.0, 0.0, 0.8), 2),
            workloads.prim("cylinder", "sub", (0, 0, 0), (0.7, 0.0, 1.0), 2)]
    assert _betti(_lib_mask(tube)) == (1, 1, 0)


def test_host_entry_point_status_and_errors():
    lib = scfft.load()
    import ctypes as C
    m = _ring()
    n = (C.c_int32 * 3)(m.shape[2], m.shape[1], m.shape[0])
    b = (C.c_int64 * 3)()
    st = lib.scfft_mask_betti_host(n, m.ctypes.data_as(C.POINTER(C.c_uint8)), b)
    assert st == scfft.WARN_TOPOLOGY and tuple(b) == (1, 1, 0)
    assert lib.scfft_mask_betti_host(n, None, b) == scfft.ERR_ARG
    bad = (C.c_int32 * 3)(0, 4, 4)
    assert lib.scfft_mask_betti_host(bad, m.ctypes.data_as(C.POINTER(C.c_uint8)), b) == scfft.ERR_SHAPE
    assert scfft.scfft_status_string(scfft.WARN_TOPOLOGY) != "unknown status"


@pytest.mark.parametrize("name", list(workloads.CONFIGS))
def test_named_workloads_are_simply_connected(name):
    c = workloads.config(name)
    g = scfft.make_grid(c["n"], [v * c["l_m"] for v in c["half_width"]])
    m = scfft.make_material(c["n_power"], c["jc"], 1e-4, c["rho_out"], c["l_m"])
    sh, ns = scfft.make_shapes(c["shapes"], c["l_m"])
    assert _betti(scfft.scfft_voxelize_host(g, m, sh, ns)) == (1, 0, 0)
