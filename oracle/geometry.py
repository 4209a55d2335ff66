"""Voxelizer: node masks of shapes built from primitives (test infrastructure).

Sec. 2 poses the problem on a superconducting domain Omega inside the box D;
the discrete method needs chi(node) = 1 for nodes in Omega, 0 in Omega_out.

Rules (readings; the paper gives no voxelization rule):
  * a node belongs to an added primitive iff it is strictly inside it;
  * a node is removed by a subtracted primitive iff it is inside or on it;
  * "strictly" uses the tie margin eps = 1e-9 * min cell size, so a node on a
    surface (up to that margin) is outside Omega;
  * shapes are applied in order: chi = ((P1 add) add P2) sub P3 ...
Primitives (dimensionless coordinates):
  box       center c, half-extents (ax, ay, az)
  cylinder  center c, axis index, radius R, half-height a
  sphere    center c, radius R
The signed margin g (positive inside) is
  box:      min_a (half_a - |x_a - c_a|)
  cylinder: min(R - rho, a - |x_axis - c_axis|)
  sphere:   R - |x - c|
"""
import numpy as np


def shape(kind, op="add", center=(0.0, 0.0, 0.0), size=(0.0, 0.0, 0.0), axis=2):
    return dict(kind=kind, op=op, center=tuple(float(v) for v in center),
                size=tuple(float(v) for v in size), axis=int(axis))


def box(center, half, op="add"):
    return shape("box", op, center, half)


def cylinder(center, radius, half_height, axis=2, op="add"):
    return shape("cylinder", op, center, (radius, 0.0, half_height), axis)


def sphere(center, radius, op="add"):
    return shape("sphere", op, center, (radius, 0.0, 0.0))


def margin(s, x, y, z):
    c = s["center"]
    p = (x - c[0], y - c[1], z - c[2])
    if s["kind"] == "box":
        a = s["size"]
        return np.minimum(np.minimum(a[0] - np.abs(p[0]), a[1] - np.abs(p[1])), a[2] - np.abs(p[2]))
    if s["kind"] == "cylinder":
        ax = s["axis"]
        others = [p[i] for i in range(3) if i != ax]
        rho = np.sqrt(others[0] ** 2 + others[1] ** 2)
        return np.minimum(s["size"][0] - rho, s["size"][2] - np.abs(p[ax]))
    if s["kind"] == "sphere":
        return s["size"][0] - np.sqrt(p[0] ** 2 + p[1] ** 2 + p[2] ** 2)
    raise ValueError("unknown primitive %r" % s["kind"])


def voxelize(grid, shapes):
    """uint8 mask of shape (Nz, Ny, Nx): 1 in Omega, 0 in Omega_out."""
    x, y, z = grid.mesh_nodes()
    eps = 1e-9 * min(grid.h)
    chi = np.zeros(grid.shape, dtype=bool)
    for s in shapes:
        g = margin(s, x, y, z)
        if s["op"] == "add":
            chi |= g > eps
        elif s["op"] == "sub":
            chi &= ~(g > -eps)
        else:
            raise ValueError("unknown op %r" % s["op"])
    return chi.astype(np.uint8)
